"""Stability of KBC, LBGK and RLB on the Kida vortex flow (section V).

The Kida vortex (Eq. kida) on an N^3 periodic box with U_0 = 0.05 and
Re = U_0 N / nu.  The paper fixes N = 100 and U_0, raises Re in steps of 500,
and calls a run stable once the mean enstrophy Omega has decayed below 5% of
its initial value.  Three families are compared, all with the same storage,
streaming and kernels (only gamma differs):

* KBC: the entropic stabilizer gamma* of section IV, for each of the eight
  shear parts s (natural d, d+t, d+q, d+t+q and their central-moment
  counterparts);
* LBGK: gamma = 2 (then s does not matter);
* RLB: gamma = 1/beta, again for each of the eight s.

A run is *unstable* when the state stops being finite or the kinetic energy
rises above `growth` times its initial value (an unforced decaying flow
cannot gain energy; the margin absorbs acoustic exchange in the weakly
compressible scheme), *stable* when Omega < 0.05 Omega_0, and *undecided*
when `max_steps` pass first.  Populations start at the product-form
equilibrium of rho = 1 and the Kida velocity; the paper's pre-solved
consistent initial density is not reproduced.
"""
from __future__ import annotations

import math
import time

from . import inputs, kbc

NATURAL = {"d": kbc.S_D, "d+t": kbc.S_DT, "d+q": kbc.S_DQ, "d+t+q": kbc.S_DTQ}
CENTRAL = {"d~": kbc.S_CD, "d~+t~": kbc.S_CDT, "d~+q~": kbc.S_CDQ, "d~+t~+q~": kbc.S_CDTQ}


def models():
    """name -> (variant, gamma kind) for the 17 models of the comparison."""
    out = {}
    for s, v in {**NATURAL, **CENTRAL}.items():
        out[f"KBC s={s}"] = (v, "entropic")
    out["LBGK"] = (kbc.S_DTQ, "lbgk")
    for s, v in {**NATURAL, **CENTRAL}.items():
        out[f"RLB s={s}"] = (v, "rlb")
    return out


def kida_run(variant, gamma_kind, re, n=100, u0=0.05, dtype=kbc.F32_DEV_X,
             streaming=kbc.AA, max_steps=40000, check=250, growth=1.5, u=None):
    """One Kida run; returns a dict with the verdict and its step count."""
    nu = u0 * n / re
    beta = 1.0 / (6.0 * nu + 1.0)      # nu = (1/3)(1/(2 beta) - 1/2)
    gamma = {"entropic": None, "lbgk": 2.0, "rlb": 1.0 / beta}[gamma_kind]
    if u is None:
        u = inputs.kida(n, u0)
    t0 = time.perf_counter()
    with kbc.Box(n, nu, dtype, variant=variant, streaming=streaming, gamma=gamma) as b:
        b.init_velocity(u)
        k0, w0 = b.energy(), b.enstrophy()
        peak, t = 1.0, 0
        verdict = "undecided"
        while t < max_steps:
            step = min(check, max_steps - t)
            b.step(step)
            t += step
            try:
                k, w = b.energy(), b.enstrophy()
            except kbc.KbcError as e:
                if e.code != kbc.KBC_EUNSTABLE:
                    raise
                verdict = "unstable"
                break
            if not (math.isfinite(k) and math.isfinite(w)) or k > growth * k0:
                verdict = "unstable"
                break
            peak = max(peak, w / w0)
            if w < 0.05 * w0:
                verdict = "stable"
                break
        b.sync()
    return {"re": re, "nu": nu, "verdict": verdict, "steps": t, "omega_peak_ratio": peak,
            "wall_s": time.perf_counter() - t0}


def sweep(names=None, re_step=500, re_max=20000, extra_re=(1e5, 1e6, 1e7), n=100, u0=0.05,
          dtype=kbc.F64, max_steps=40000, log=None):
    """Raise Re in steps of `re_step` for each model until its first run that
    is not stable, up to `re_max`; models stable throughout are also run at
    each Re in `extra_re`.  Returns name -> {"max_stable_re", "first_failure_re",
    "extra", "runs"}."""
    table = models()
    names = list(table) if names is None else names
    u = inputs.kida(n, u0)
    out = {}

    def one(name, re):
        variant, kind = table[name]
        r = kida_run(variant, kind, re, n, u0, dtype, max_steps=max_steps, u=u)
        if log:
            log(f"[stability] {name} Re={re:g}: {r['verdict']} after {r['steps']} steps "
                f"(peak Omega/Omega0 {r['omega_peak_ratio']:.2f}, {r['wall_s']:.2f} s)")
        return r

    for name in names:
        runs, best, fail = [], 0, None
        re = re_step
        while re <= re_max:
            r = one(name, re)
            runs.append(r)
            if r["verdict"] != "stable":
                fail = re
                break
            best = re
            re += re_step
        extra = {}
        if fail is None:
            for re in extra_re:
                r = one(name, re)
                runs.append(r)
                extra[f"{re:g}"] = r["verdict"]
        out[name] = {"max_stable_re": best, "first_failure_re": fail, "extra": extra,
                     "runs": runs}
    return out


def main(argv=None):
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="Kida-vortex stability sweep (section V)")
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--re-step", type=int, default=500)
    ap.add_argument("--re-max", type=int, default=20000)
    ap.add_argument("--dtype", default="f64", choices=sorted(kbc.DTYPES))
    ap.add_argument("--max-steps", type=int, default=40000)
    ap.add_argument("--models", default=None, help="comma-separated model names")
    args = ap.parse_args(argv)
    names = args.models.split(",") if args.models else None
    res = sweep(names, args.re_step, args.re_max, n=args.n, dtype=kbc.DTYPES[args.dtype],
                max_steps=args.max_steps, log=lambda m: print(m, file=sys.stderr, flush=True))
    summary = {k: {"max_stable_re": v["max_stable_re"], "first_failure_re": v["first_failure_re"],
                   "extra": v["extra"]} for k, v in res.items()}
    print(json.dumps({"workload": f"Kida vortex N={args.n}, U0=0.05, Re in steps of "
                                  f"{args.re_step} to {args.re_max}, {args.dtype} AA",
                      "criterion": "stable: Omega < 0.05 Omega0; unstable: non-finite or "
                                   "k > 1.5 k0", "models": summary}))
    return res


if __name__ == "__main__":
    main()
