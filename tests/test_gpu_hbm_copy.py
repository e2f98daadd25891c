"""GPU tests of the copy-bandwidth utility behind the bench's ceilings: the
copy between two buffers moves every byte, the in-place form (dst == src)
reads and writes every word back unchanged, on sizes that end in a partial
workgroup and that take several passes of the grid-stride loop."""
import sys

import pytest
import torch

from paper_1507_02518_amd import kbc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 16 * 1000 + 16 * 7, 16 * 256 * (1 << 21) + 16 * 300])
def test_copy_and_in_place_rewrite(nbytes):
    print(f"hbm_copy {nbytes} bytes", flush=True)
    sys.stdout.flush()
    g = torch.Generator(device="cuda").manual_seed(nbytes % 1000003)
    a = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    keep = a.clone()
    b = torch.zeros(nbytes + 16, dtype=torch.uint8, device="cuda")
    kbc.kbc_hbm_copy(b.data_ptr(), a.data_ptr(), nbytes)
    kbc.kbc_hbm_copy(a.data_ptr(), a.data_ptr(), nbytes)
    torch.cuda.synchronize()
    assert torch.equal(b[:nbytes], keep)
    assert int(b[nbytes:].count_nonzero()) == 0
    assert torch.equal(a, keep)

