"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, its ctypes mirror matches the C layout, argument errors come back
as codes without touching a GPU, and the host-side index math is exact."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1507_02518_amd import kbc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kbc.h")
CSRC = os.path.join(ROOT, "paper_1507_02518_amd", "csrc")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kbc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = kbc.load()
    names = _declared()
    assert "kbc_create" in names and "kbc_step" in names and "kbc_energy" in names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", kbc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, flags=re.M), n


def test_options_struct_layout_matches_header():
    src = r"""
    #include <stddef.h>
    #include <stdio.h>
    #include "kbc.h"
    int main(void) {
      printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(kbc_options),
             offsetof(kbc_options, variant), offsetof(kbc_options, streaming),
             offsetof(kbc_options, gamma_mode), offsetof(kbc_options, device),
             offsetof(kbc_options, gamma_value), offsetof(kbc_options, gamma_eps),
             offsetof(kbc_options, stream));
      return 0;
    }
    """
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                               check=True).stdout.split()]
    O = kbc.kbc_options
    want = [ctypes.sizeof(O)] + [getattr(O, f).offset for f in
                                 ("variant", "streaming", "gamma_mode", "device",
                                  "gamma_value", "gamma_eps", "stream")]
    assert vals == want


def test_options_defaults():
    o = kbc.kbc_options_default()
    assert o.variant == kbc.S_DTQ and o.streaming == kbc.PULL
    assert o.gamma_mode == kbc.GAMMA_ENTROPIC and o.device == -1 and not o.stream


@pytest.mark.parametrize("shape,nu,dtype", [
    ((0, 4, 4), 1e-3, kbc.F64),
    ((4, -1, 4), 1e-3, kbc.F64),
    ((4, 4, 4), 0.0, kbc.F64),
    ((4, 4, 4), -1e-3, kbc.F64),
    ((4, 4, 4), float("nan"), kbc.F64),
    ((4, 4, 4), 1e-3, 7),
    ((2048, 1024, 1024), 1e-3, kbc.F64),
    # a direction plane above 4 GiB (32-bit in-plane byte offsets)
    ((1024, 1024, 1024), 1e-3, kbc.F64),
    ((1024, 1024, 1025), 1e-3, kbc.F32_DEV),
])
def test_create_rejects_bad_arguments(shape, nu, dtype):
    with pytest.raises(kbc.KbcError) as e:
        kbc.kbc_create(shape, nu, dtype)
    assert e.value.code == kbc.KBC_EINVAL
    assert kbc.kbc_last_error()


def test_create_rejects_bad_options():
    o = kbc.kbc_options_default()
    o.variant = 9
    with pytest.raises(kbc.KbcError) as e:
        kbc.kbc_create((4, 4, 4), 1e-3, kbc.F64, o)
    assert e.value.code == kbc.KBC_EINVAL
    o = kbc.kbc_options_default()
    o.streaming = 5
    with pytest.raises(kbc.KbcError):
        kbc.kbc_create((4, 4, 4), 1e-3, kbc.F64, o)
    o = kbc.kbc_options_default()
    o.gamma_mode = 3
    with pytest.raises(kbc.KbcError) as e:
        kbc.kbc_create((4, 4, 4), 1e-3, kbc.F64, o)
    assert e.value.code == kbc.KBC_EINVAL


def test_null_handles_are_rejected():
    lib = kbc.load()
    assert lib.kbc_destroy(None) == kbc.KBC_OK
    assert lib.kbc_step(None, 1) == kbc.KBC_EINVAL
    k = ctypes.c_double()
    assert lib.kbc_energy(None, ctypes.byref(k)) == kbc.KBC_EINVAL
    assert lib.kbc_energy_series(None, 1, ctypes.byref(k)) == kbc.KBC_EINVAL
    assert lib.kbc_sync(None) == kbc.KBC_EINVAL
    assert lib.kbc_moments(None, None, None) == kbc.KBC_EINVAL
    assert b"null handle" in lib.kbc_last_error()


def test_hbm_copy_rejects_bad_arguments():
    """Argument errors of the copy utility come back before any launch (the
    addresses below are never dereferenced)."""
    lib = kbc.load()
    p, q = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000)
    assert lib.kbc_hbm_copy(None, q, 64, None) == kbc.KBC_EINVAL
    assert lib.kbc_hbm_copy(p, q, 24, None) == kbc.KBC_EINVAL
    assert b"multiple of 16" in lib.kbc_last_error()
    # overlapping but distinct ranges, in both orders
    assert lib.kbc_hbm_copy(ctypes.c_void_p(0x100010), p, 64, None) == kbc.KBC_EINVAL
    assert lib.kbc_hbm_copy(p, ctypes.c_void_p(0x100030), 64, None) == kbc.KBC_EINVAL
    assert b"overlap" in lib.kbc_last_error()


def test_fast_division_host_check():
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang++ not present")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "fd")
        subprocess.run([clang, "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I", CSRC,
                        os.path.join(ROOT, "tests", "host", "fastdiv_check.cpp"), "-o", exe],
                       check=True)
        r = subprocess.run([exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr


def test_log1p_series_host_check():
    """The exact stabilizer's ln(1 + x) for |x| < 1/16 (a degree-9 Chebyshev
    economization, compiled here for the CPU) against the C library's
    extended-precision log1pl: within 5e-16 relative everywhere on the
    interval (about two ulp; the analysis gives below 4e-16)."""
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang++ not present")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "lg")
        subprocess.run([clang, "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I", CSRC,
                        os.path.join(ROOT, "tests", "host", "log1p_check.cpp"), "-o", exe],
                       check=True)
        r = subprocess.run([exe, "5e-16"], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr


def test_population_layouts_host_check():
    """pop_index over the x-blocked layout and planes (with and without a
    gap): a bijection onto the allocated extent (injective with a gap),
    contiguous chunks, slot spans and the chunk sizes chosen."""
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang++ not present")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "lay")
        subprocess.run([clang, "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I", CSRC,
                        os.path.join(ROOT, "tests", "host", "layout_check.cpp"), "-o", exe],
                       check=True)
        r = subprocess.run([exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr


def test_pool_create_rejects_bad_arguments():
    for budget, dtype, slots in [(1 << 30, 9, 8), (1 << 30, kbc.F32_DEV, 0),
                                 (1024, kbc.F32_DEV, 8), (1 << 30, kbc.F32_DEV, 70000)]:
        with pytest.raises(kbc.KbcError) as e:
            kbc.kbc_pool_create(budget, dtype, None, slots, None)
        assert e.value.code == kbc.KBC_EINVAL
    o = kbc.kbc_options_default()
    o.gamma_mode = kbc.GAMMA_EXACT
    with pytest.raises(kbc.KbcError) as e:
        kbc.kbc_pool_create(1 << 30, kbc.F32_DEV, o, 8, None)
    assert e.value.code == kbc.KBC_EINVAL and "single boxes" in kbc.kbc_last_error()
    lib = kbc.load()
    assert lib.kbc_pool_destroy(None) == kbc.KBC_OK
    assert lib.kbc_pool_advance(None, 1) == kbc.KBC_EINVAL


def test_device_collision_built_for_the_host_matches_the_oracle(orc):
    """kbc::collide (the kernels' per-node update, compiled here for the CPU)
    against the oracle's collision for all eight variants, natural and
    central: FP64 within 5e-15, FP32 deviation storage with FP64-formed
    non-equilibrium within 3e-8 (measured 1.7e-15 and 7e-9), and the exact
    stabilizer (root of Eq. result1) against the oracle's bisection within
    5e-15 (measured 1.7e-15; the exact and estimated gamma differ by ~3e-3),
    and far from equilibrium (10-30% perturbations, starts outside the
    interval of positive populations) within 2e-13 (measured 5e-14)."""
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang++ not present")
    odir = os.path.join(ROOT, "oracle")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "cc")
        subprocess.run([clang, "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", "-I", CSRC, "-I", odir,
                        os.path.join(ROOT, "tests", "host", "collide_check.cpp"),
                        "-L", odir, "-lkbc_oracle", f"-Wl,-rpath,{odir}", "-o", exe],
                       check=True, capture_output=True)
        r = subprocess.run([exe, "5e-15", "3e-8", "5e-15"], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr


def test_stats_struct_layout_matches_header():
    src = r"""
    #include <stddef.h>
    #include <stdio.h>
    #include "kbc.h"
    int main(void) {
      printf("%zu %zu %zu %zu\n", sizeof(kbc_stats), offsetof(kbc_stats, div2),
             offsetof(kbc_stats, dudx_moment), offsetof(kbc_stats, skewness));
      return 0;
    }
    """
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                               check=True).stdout.split()]
    S = kbc.kbc_stats
    assert vals == [ctypes.sizeof(S), S.div2.offset, S.dudx_moment.offset, S.skewness.offset]
