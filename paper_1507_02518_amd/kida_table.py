"""The statistics of the Kida vortex flow at Re = 6000 (section V.A).

The paper's table of statistics follows the Kida vortex (Eq. kida, U_0 =
0.05, Re = U_0 N / nu = 6000) with KBC s = d+t+q at N = 100, 200, 400 (runs
A, B, C) and LBGK at N = 600 (run D, the resolved reference), and reports at
t = 0.25, 0.5, 0.75 (in units of N / U_0): the kinetic energy, enstrophy and
dissipation rate, the longitudinal skewness factors S^3 .. S^6, and the
turbulence, Taylor and Kolmogorov scales, every gradient by the eighth-order
stencil.  ``kida_table`` computes the same rows on the GPU, plus the mean
and standard deviation of the stabilizer (section V.C).

Populations start at the product-form equilibrium of rho = 1 and the Kida
velocity; the paper's pre-solved consistent initial density is not
reproduced, so the rows are comparable with the paper's, not equal to them.

    python -m paper_1507_02518_amd.kida_table --n 100 [--lbgk] [--dtype f64]
"""
from __future__ import annotations

import json
import sys
import time

from . import analysis, inputs, kbc

ROWS = ["k*1e4", "Omega*N^2", "eps*N*1e5", "S3*1e2", "S4", "S5", "S6", "l0/N*1e1", "u0*1e2",
        "tau0/N", "Re0", "lambda/N*1e2", "u_lambda*1e2", "tau_lambda/N", "Re_lambda",
        "eta/N*1e3", "u_eta*1e3", "tau_eta/N*1e1"]


def table_rows(st: dict, n: int, nu: float) -> dict:
    """The table's rows (in its scaling) from kbc_statistics output."""
    sc = analysis.turbulence_scales(st["k"], st["epsilon"], nu)
    s = st["skewness"]
    vals = [st["k"] * 1e4, st["omega"] * n * n, st["epsilon"] * n * 1e5, s[3] * 1e2, s[4], s[5],
            s[6], sc["l0"] / n * 10, sc["u0"] * 100, sc["tau0"] / n, sc["Re0"],
            sc["lambda"] / n * 100, sc["u_lambda"] * 100, sc["tau_lambda"] / n, sc["Re_lambda"],
            sc["eta"] / n * 1e3, sc["u_eta"] * 1e3, sc["tau_eta"] / n * 10]
    return dict(zip(ROWS, vals))


def kida_table(n: int, re: float = 6000.0, u0: float = 0.05, times=(0.25, 0.5, 0.75),
               lbgk: bool = False, dtype=kbc.F64, streaming=kbc.AA, log=None) -> dict:
    nu = u0 * n / re
    t0 = time.perf_counter()
    out = {"n": n, "re": re, "nu": nu, "model": "LBGK" if lbgk else "KBC s=d+t+q",
           "dtype": dtype, "times": {}}
    with kbc.Box(n, nu, dtype, variant=kbc.S_DTQ, streaming=streaming,
                 gamma=2.0 if lbgk else None) as b:
        b.init_velocity(inputs.kida(n, u0))
        done = 0
        for t in times:
            steps = int(round(t * n / u0))
            b.step(steps - done)
            done = steps
            st = b.statistics(8)
            row = table_rows(st, n, nu)
            if not lbgk:
                g = b.gamma_statistics()
                row["gamma_mean"] = g["mean"]
                row["gamma_std"] = g["std"]
            row["Omega_FD2*N^2"] = b.enstrophy() * n * n
            out["times"][f"{t:g}"] = row
            if log:
                log(f"[kida] N={n} t={t:g} ({steps} steps, {time.perf_counter() - t0:.1f} s): "
                    + ", ".join(f"{k}={v:.4g}" for k, v in list(row.items())[:7]))
    out["wall_s"] = time.perf_counter() - t0
    return out


def main(argv=None):
    import argparse

    ap = argparse.ArgumentParser(description="Kida vortex statistics at Re = 6000")
    ap.add_argument("--n", type=int, nargs="+", default=[100])
    ap.add_argument("--re", type=float, default=6000.0)
    ap.add_argument("--lbgk", action="store_true", help="LBGK (gamma = 2) instead of KBC")
    ap.add_argument("--dtype", default="f64", choices=sorted(kbc.DTYPES))
    args = ap.parse_args(argv)
    for n in args.n:
        res = kida_table(n, args.re, lbgk=args.lbgk, dtype=kbc.DTYPES[args.dtype],
                         log=lambda m: print(m, file=sys.stderr, flush=True))
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
