"""Build libkbc.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1507_02518_amd.build [extra hipcc flags]

Each translation unit compiles to an object in parallel (the step kernels
once per storage form and stabilizer mode), then hipcc links the library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libkbc.so")
ARCH = os.environ.get("KBC_OFFLOAD_ARCH", "gfx950")

# (object name, source, defines); storage forms 0 FP64, 1 FP32 dev, 2 FP16
# dev, 3 FP32 dev X; exact stabilizer 0/1
UNITS = [("kbc_kernels", "kbc_kernels.hip", []),
         ("kbc_api", "kbc_api.hip", []),
         ("kbc_pool", "kbc_pool.hip", [])]
UNITS += [(f"kbc_step_s{s}_x{x}", "kbc_step_inst.hip",
           [f"-DKBC_INST_STORAGE={s}", f"-DKBC_INST_EXACT={x}"])
          for x in (1, 0) for s in (0, 1, 2, 3)]

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def _jobs() -> int:
    env = os.environ.get("MAX_JOBS")
    n = int(env) if env and env.isdigit() else (os.cpu_count() or 4)
    return max(1, min(n, 16))


def compile_flags(extra=None):
    return [*HIPCC_FLAGS, *(extra or []), "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, extra=None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    flags = compile_flags(extra)

    def one(unit):
        name, src, defs = unit
        out = os.path.join(OBJ, name + ".o")
        cmd = [hipcc, *flags, *defs, "-c", os.path.join(CSRC, src), "-o", out + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(ln for ln in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in ln)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {name}:\n{msg}")
        if msg.strip() and verbose:
            print(msg, flush=True)
        os.replace(out + ".tmp", out)
        return out

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        objs = list(ex.map(one, UNITS))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
