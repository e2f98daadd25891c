"""Static check of the built AA kernels: a node's 27 loads all precede its
27 stores.  The in-place AA sweeps read and write the same locations through
two pointers into one buffer, so the order in the generated gfx950 code is
what makes them race free; this test reads it from the compiler's own
assembly of our sources."""
import glob
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1507_02518_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def asm():
    """gfx950 assembly of every instance of the step kernels (one per storage
    form and stabilizer mode, compiled in parallel), concatenated."""
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not present")
    from concurrent.futures import ThreadPoolExecutor

    def one(sx):
        s, x = sx
        with tempfile.TemporaryDirectory() as d:
            subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17",
                            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                            f"-DKBC_INST_STORAGE={s}", f"-DKBC_INST_EXACT={x}",
                            "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
                            os.path.join(CSRC, "kbc_step_inst.hip"), "--offload-device-only",
                            "-save-temps", "-o", os.path.join(d, "k.o")],
                           check=True, cwd=d, capture_output=True)
            path = glob.glob(os.path.join(d, "*gfx950*.s"))[0]
            return open(path).read()

    units = [(s, x) for x in (1, 0) for s in range(4)]
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return "\n".join(ex.map(one, units))


def _kernels(asm, pattern):
    names = re.findall(r"^(_ZN3kbc\S*" + pattern + r"\S*):", asm, flags=re.M)
    out = {}
    for nm in names:
        i = asm.index(nm + ":")
        j = asm.index(".Lfunc_end", i)
        ops = [ln.split()[0] for ln in asm[i:j].split("\n")
               if ln.startswith("\t") and ln.strip() and not ln.strip().startswith((".", ";"))]
        out[nm] = [op for op in ops if op.startswith(("global_load", "global_store",
                                                     "buffer_load", "buffer_store"))]
    return out


def test_aa_step_kernels_load_everything_before_storing(asm):
    """27 population loads, then only stores: 27 in the even sweep, in the
    exact-stabilizer odd sweep and in the plain FP32 and FP16 odd sweeps; 45
    in the FP64 and FP32-X odd sweeps, whose stores are line-aligned (9
    directions with v_x = 0, 18 aligned, 18 for rows split between
    workgroups, of which a thread executes at most 27)."""
    ks = _kernels(asm, r"k_stepILi\dELi\dELi[12]E")
    # 4 storage forms x 8 variants x 2 sweeps x (estimate, exact gamma)
    assert len(ks) == 4 * 8 * 2 * 2
    for nm, ops in ks.items():
        loads = [op for op in ops if "load" in op]
        stores = [op for op in ops if "store" in op]
        odd_aligned = re.search(r"k_stepILi[03]ELi\dELi2ELb0E", nm) is not None
        assert len(loads) == 27, (nm, len(loads))
        assert len(stores) == (45 if odd_aligned else 27), (nm, len(stores))
        first_store = next(i for i, op in enumerate(ops) if "store" in op)
        assert first_store == 27 and all("store" in op for op in ops[27:]), nm


def _is_pop(op, storage):
    """Whether a global/buffer access has the width of a stored population:
    FP64 (storage 0) dwordx2, FP32 (1, 3) dword, FP16 (2) 16-bit."""
    suffix = op.split("_", 2)[2]
    if storage == "0":
        return suffix == "dwordx2"
    if storage in ("1", "3"):
        return suffix == "dword"
    return suffix.startswith(("ushort", "short", "b16"))


def _blocks(asm, nm, storage):
    """Population loads (L) and stores (S) of each basic block of a kernel,
    in listing order.  Accesses of another width (the FP16 pool kernel reads
    its boxes' scale exponents as bytes) are not populations."""
    i = asm.index(nm + ":")
    j = asm.index(".Lfunc_end", i)
    blocks = [[]]
    for ln in asm[i:j].split("\n")[1:]:
        t = ln.strip()
        if re.match(r"^\.LBB\d+_\d+:", t):
            blocks.append([])
            continue
        op = t.split()[0] if t else ""
        if op.startswith(("global_load", "buffer_load")) and _is_pop(op, storage):
            blocks[-1].append("L")
        elif op.startswith(("global_store", "buffer_store")) and _is_pop(op, storage):
            blocks[-1].append("S")
    return blocks


def test_pool_kernels_load_everything_before_storing(asm):
    """The pool kernel loops over tiles, so its loads and stores may sit in
    different basic blocks (the instruction scheduler never moves code
    between blocks); inside any block no population load may follow a
    population store."""
    names = re.findall(r"^(_ZN3kbc\S*k_pool_stepILi\dELi\dELi[12]E\S*):", asm, flags=re.M)
    # 4 storage forms x 8 variants x 2 sweeps x (tile loop, single tile)
    assert len(names) == 4 * 8 * 2 * 2
    for nm in names:
        storage = re.search(r"k_pool_stepILi(\d)E", nm).group(1)
        blocks = _blocks(asm, nm, storage)
        seq = [op for b in blocks for op in b]
        assert seq.count("L") == 27 and seq.count("S") == 27, nm
        for b in blocks:
            text = "".join(b)
            assert "SL" not in text, (nm, text)


_FP_OP = re.compile(r"^v_(fma|fmac|fmamk|fmaak|mul|add|sub|subrev|mac|ldexp|rcp|sqrt|div\w*|cvt\w*)_f(16|32|64)")


def _fp_ops(asm, nm):
    from collections import Counter

    i = asm.index(nm + ":")
    j = asm.index(".Lfunc_end", i)
    ops = [ln.split()[0] for ln in asm[i:j].split("\n")
           if ln.startswith("\t") and ln.strip() and _FP_OP.match(ln.split()[0])]
    # fma, fmac (accumulating) and fmamk / fmaak (one literal operand) are the
    # same fused operation
    return Counter(re.sub(r"^v_(fmac|fmamk|fmaak)_", "v_fma_", op.replace("_e32", "").replace("_e64", ""))
                   for op in ops)


def test_every_sweep_and_the_pool_collide_with_the_same_arithmetic(asm):
    """A box gives the same bits alone and in the pool, in pull and AA
    streaming, only if every kernel evaluates the collision with the same
    floating-point instructions (same contractions into FMAs): per storage
    form and variant, the multiset of floating-point opcodes of the pull, AA
    even and AA odd step kernels (FP16 also the pull sweep on 64-node chunks)
    and of the pool's two sweeps (with and without the tile loop) is the
    same."""
    names = re.findall(r"^(_ZN3kbc\S*(?:k_stepILi\dELi\dELi\dELb0|k_pool_stepILi\dELi\dELi\d)E\S*):",
                       asm, flags=re.M)
    groups = {}
    for nm in names:
        m = re.search(r"(k_step|k_pool_step)ILi(\d)ELi(\d)ELi(\d)", nm)
        groups.setdefault((m.group(2), m.group(3)), []).append((nm, _fp_ops(asm, nm)))
    assert len(groups) == 4 * 8
    for key, lst in groups.items():
        # pull, AA even, AA odd, the pool's two sweeps with and without the
        # tile loop; FP16 (storage 2) adds the pull sweep on 64-node chunks
        assert len(lst) == (8 if key[0] == "2" else 7), (key, len(lst))
        ref = lst[0][1]
        assert sum(ref.values()) > 300, key
        for nm, ops in lst[1:]:
            assert ops == ref, (key, nm, ops - ref, ref - ops)
