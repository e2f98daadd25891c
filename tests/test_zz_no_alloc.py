"""The no-allocation entry point kbc_energy_series_noalloc against
kbc_energy_series, through the C-ABI: two calls in a row on one GPU, the
second on a smaller box with fewer steps, every storage form and both
streaming patterns; and its argument checks."""
import sys

import numpy as np
import pytest

from paper_1507_02518_amd import inputs, kbc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _series(shape, nu, dtype, streaming, u, n, noalloc, pre=0):
    with kbc.Box(shape, nu, dtype, streaming=streaming) as b:
        b.init_velocity(u)
        if pre:
            b.step(pre)
        if noalloc:
            k = kbc.kbc_energy_series_noalloc(b.h, n)
        else:
            k = b.energy_series(n)
        return k, b.populations(), b.t


# The energy sums of both entry points run in the same order on the same
# velocity bits, so they agree bit for bit; the assertion allows rounding
# order (1e-12 relative, the FP64 energy bar) and the test reports which.
# Solenoidal starts only: FP16 storage overflows on the acoustic transients of
# a start with divergence.
@pytest.mark.parametrize("dtype", [kbc.F64, kbc.F32_DEV, kbc.F32_DEV_X, kbc.F16_DEV])
@pytest.mark.parametrize("streaming", [kbc.PULL, kbc.AA])
def test_noalloc_series_equals_the_allocating_series(dtype, streaming):
    calls = [((32, 32, 32), inputs.hit(32, 3.0, 0.04, seed=21), 40, 3),
             ((13, 7, 5), inputs.hit((13, 7, 5), 2.0, 0.04, seed=22), 7, 0)]
    for shape, u, n, pre in calls:
        say(f"noalloc dtype={dtype} streaming={streaming} shape={shape} n={n}")
        ka, fa, ta = _series(shape, 2e-3, dtype, streaming, u, n, noalloc=True, pre=pre)
        kb, fb, tb = _series(shape, 2e-3, dtype, streaming, u, n, noalloc=False, pre=pre)
        assert ta == tb == n + pre
        assert np.array_equal(fa, fb)
        rel = np.abs(ka / kb - 1).max()
        say(f"  max rel dk {rel:.3e}, bitwise {np.array_equal(ka, kb)}")
        assert rel <= 1e-12


def test_noalloc_series_limits_and_errors():
    u = inputs.taylor_green(8, 0.04)
    with kbc.Box(8, 1e-3) as b:
        with pytest.raises(kbc.KbcError) as e:
            kbc.kbc_energy_series_noalloc(b.h, 1)
        assert e.value.code == kbc.KBC_ESTATE
        b.init_velocity(u)
        for bad in (-1, kbc.NOALLOC_MAX_STEPS + 1):
            with pytest.raises(kbc.KbcError) as e:
                kbc.kbc_energy_series_noalloc(b.h, bad)
            assert e.value.code == kbc.KBC_EINVAL
        assert b.t == 0
        assert kbc.kbc_energy_series_noalloc(b.h, 0).size == 0
        k = kbc.kbc_energy_series_noalloc(b.h, 3)
        assert b.t == 3 and np.all(np.isfinite(k))
        f = b.populations()
        f[5, 1, 2, 3] = np.nan
        b.set_populations(f, 3)
        with pytest.raises(kbc.KbcError) as e:
            kbc.kbc_energy_series_noalloc(b.h, 2)
        assert e.value.code == kbc.KBC_EUNSTABLE
