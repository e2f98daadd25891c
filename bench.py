"""Throughput of the fused D3Q27 KBC stream+collide step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload (synthetic, seeded): a 256^3 periodic box of decaying homogeneous
isotropic turbulence, initial spectrum E(k) ~ k^4 exp(-2 (k/k0)^2), k0 = 4,
u_rms = 0.04, rho = 1, nu = 5e-4, populations at the product-form
equilibrium; KBC model s = d+t+q with the entropic stabilizer.  One step is
one launch of the fused kernel over all 16.8 M nodes.  The headline line is
FP64 storage with pull streaming (the form matched element-wise to the CPU
oracle); the other storage forms, the s = d variant, the central-moment
default s = d~+t~+q~ and the exact stabilizer (root of the entropy condition
at every node) are measured on the same field and listed under "forms".

The 512^3 in-place (AA) run of decaying HIT (k0 = 8, u_rms = 0.04,
nu = 2.5e-4, seed 2) in FP32 / FP16 deviation storage and FP64 is timed under
"big_forms"; the batched ensemble (64 boxes) and a served request trace
(Poisson arrivals, 512 requests) are each compared with a plain loop of
single boxes on the same inputs.

Prints one JSON line with MLUPS, the roofline of the step kernel (HBM bound,
algorithmic bytes 2 * 27 * bytes-per-population per node and step, timed with
HIP events on the stream the kernel runs on), and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
N = 256
NU = 5e-4
K0 = 4.0
URMS = 0.04
SEED = 0
METRIC = "MLUPS + HBM-roofline %, D3Q27 KBC 256^3; ensemble p50/p99 vs plain loop"
COUNTERS = os.path.join(ROOT, "profiles", "step_f64_pull_256_counters.txt")
BIG_N, BIG_NU, BIG_K0, BIG_SEED = 512, 2.5e-4, 8.0, 2
CSRC = os.path.join(ROOT, "paper_1507_02518_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the files that define the step kernel's code and launch shape (the host API
# files do not)
KERNEL_SOURCES = ("kbc_device.h", "kbc_internal.h", "kbc_step.h", "kbc_step_inst.hip",
                  "kbc_kernels.hip")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters():
    """HBM bytes per step launch from the committed rocprofv3 --pmc summary,
    or None if it is absent or was taken on different kernel sources."""
    if not os.path.exists(COUNTERS):
        return None
    vals = {}
    for line in open(COUNTERS):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_digest") != kernel_source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


VALU_COUNTS = os.path.join(ROOT, "profiles", "step_kernels_valu_256.txt")
# VALU wave instructions the chip can issue per second: one per SIMD every
# four cycles (a wave64 instruction occupies a 16-lane SIMD for four), 1024
# SIMDs at 2.4 GHz
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4
STORAGE_INDEX = {"F64": 0, "F32_DEV": 1, "F16_DEV": 2, "F32_DEV_X": 3}
VARIANT_INDEX = {None: 3, "S_D": 0, "S_CDTQ": 7, "exact": 3}


def read_valu_counts():
    """VALU wave instructions per wave of each step kernel at 256^3 from the
    committed rocprofv3 summary, or {} if it was taken on other sources."""
    if not os.path.exists(VALU_COUNTS):
        return {}
    vals = {}
    for line in open(VALU_COUNTS):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.rsplit("=", 1)
            vals[k.strip()] = v.strip()
    if vals.pop("kernel_source_digest", None) != kernel_source_digest():
        return {}
    return {k: float(v) for k, v in vals.items()}


def valu_issue_ms(counts, storage, streaming, var, n):
    """Time to issue the VALU instructions of one step (one wave per 64
    nodes), from the measured counts: the kernel's VALU issue bound."""
    gx = "true" if var == "exact" else "false"
    sweeps = (0,) if streaming == "PULL" else (1, 2)
    # FP16 and exact-stabilizer pull boxes in 64-node chunks run the kernel
    # with that geometry compiled in
    c64 = ("true" if streaming == "PULL" and n % 64 == 0 and n > 64
           and (storage == "F16_DEV" or var == "exact") else "false")
    names = [f"k_step<{STORAGE_INDEX[storage]}, {VARIANT_INDEX[var]}, {sw}, {gx}, "
             f"{c64 if sw == 0 else 'false'}>" for sw in sweeps]
    if not all(nm in counts for nm in names):
        return None
    per_wave = sum(counts[nm] for nm in names) / len(names)
    return per_wave * (n ** 3 / 64) / VALU_ISSUE_PER_S * 1e3


def time_form(kbc, torch, u_dev, dtype, streaming, steps, warmup, stream, variant=None,
              gamma=None, n=N, nu=NU):
    # the box enqueues on `stream` (a torch stream of default priority); the
    # events are recorded on the same stream, so they bracket the launches
    variant = kbc.S_DTQ if variant is None else variant
    with kbc.Box(n, nu, dtype, variant=variant, streaming=streaming, gamma=gamma,
                 stream=stream.cuda_stream) as box:
        kbc.kbc_init_velocity_device(box.h, u_dev.data_ptr(), None)
        box.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        box.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ms = e0.elapsed_time(e1) / steps
        bpn = box.bytes_per_node_step()
        k = box.energy()
    mlups = n ** 3 / (ms * 1e-3) / 1e6
    gbs = bpn * n ** 3 / (ms * 1e-3) / 1e9
    return {"ms_per_step": ms, "mlups": mlups, "algorithmic_GBs": gbs,
            "frac_hbm_peak": gbs / PEAK_HBM_GBS, "bytes_per_node_step": bpn,
            "wall_s": wall, "energy_after": k}


def copy_ceiling(kbc, torch, stream):
    """Achievable HBM bandwidth of a plain streaming copy between two 2 GiB
    buffers, and of the same stream in place (each 16-byte word read and
    written back to its own address, as an in-place AA sweep does), in GB/s
    counting the bytes read plus the bytes written."""
    nbytes = 2 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = []
    for dst in (b, a):
        for _ in range(3):
            kbc.kbc_hbm_copy(dst.data_ptr(), a.data_ptr(), nbytes, stream.cuda_stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            kbc.kbc_hbm_copy(dst.data_ptr(), a.data_ptr(), nbytes, stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out.append(2 * nbytes / (ms * 1e-3) / 1e9)
    del a, b
    return out[0], out[1]


def add_ceiling_fracs(forms, copy_gbs, inplace_gbs):
    """Each form's algorithmic GB/s against the measured ceiling of its
    streaming: the copy between two buffers for pull, the in-place stream
    for AA."""
    for name, r in forms.items():
        if not isinstance(r, dict) or "algorithmic_GBs" not in r:
            continue
        if "_aa" in name:
            r["frac_of_inplace_ceiling"] = round(r["algorithmic_GBs"] / inplace_gbs, 4)
        else:
            r["frac_of_copy_ceiling"] = round(r["algorithmic_GBs"] / copy_gbs, 4)


def ensemble_and_serving(kbc, args):
    """Batched ensemble (64 boxes, 500 steps) and a served request trace,
    each against a plain one-box-at-a-time loop on the same inputs."""
    import tempfile

    from paper_1507_02518_amd import serve

    out = {}
    cache = os.path.join(tempfile.gettempdir(), "kbc_pool_tune.txt")
    if args.ensemble:
        es = args.ensemble_steps
        log(f"[bench] ensemble: 64 boxes, edges {{24..96}}, {es} steps, FP32 storage")
        boxes = serve.ensemble_boxes(64, seed=0, steps=es)
        # warm-up, in which the launch-shape tuner measures its candidates
        serve.run_ensemble(boxes, kbc.F32_DEV_X, batched=True, g=10, tune_cache=cache)
        pool = serve.run_ensemble(boxes, kbc.F32_DEV_X, batched=True, tune_cache=cache)
        loop = serve.run_ensemble(boxes, kbc.F32_DEV_X, batched=False)
        same = all(pool["results"][i] == loop["results"][i] for i in pool["results"])
        out["ensemble"] = {
            "boxes": len(boxes), "steps": es, "storage": "f32dev_x",
            "lattice_updates": pool["lattice_updates"],
            "pool": {"wall_s": round(pool["wall_s"], 4), "mlups": round(pool["mlups"], 1),
                     "launch": {"block": pool["launch"]["block"], "grid": pool["launch"]["grid"]}},
            "loop": {"wall_s": round(loop["wall_s"], 4), "mlups": round(loop["mlups"], 1)},
            "speedup": round(loop["wall_s"] / pool["wall_s"], 3),
            "results_equal": same}
        log(f"[bench]   pool {pool['mlups']:.0f} MLUPS vs loop {loop['mlups']:.0f} MLUPS, equal={same}")
    if args.serve_requests > 0:
        log(f"[bench] serving: {args.serve_requests} requests, Poisson 20/s")
        trace = serve.serving_trace(args.serve_requests, rate=20.0, seed=0)

        def lat(runs):
            # one entry per repetition, then the spread over them
            d = {"p50_s": round(runs[0]["p50_s"], 3), "p99_s": round(runs[0]["p99_s"], 3),
                 "mlups": round(runs[0]["mlups"], 1), "wall_s": round(runs[0]["wall_s"], 3)}
            if len(runs) > 1:
                for key in ("p50_s", "p99_s", "mlups"):
                    v = [r[key] for r in runs]
                    d[key + "_runs"] = [round(x, 3) for x in v]
                    d[key + "_spread"] = round((max(v) - min(v)) / min(v), 4)
            return d

        def say(name, r):
            log(f"[bench]   {name}: p50 {r['p50_s']:.2f}s p99 {r['p99_s']:.2f}s {r['mlups']:.0f} MLUPS")

        # policies: "aged" shortest remaining work first with aging (weight
        # 0.3, batches of >= 4M nodes and 50 steps), the default; "srpt" the
        # same without aging in batches of >= 8M nodes and 25 steps (best
        # median); "loop" first come first served, one box at a time
        runs = {}
        for rep in range(args.serve_reps):
            for pol in args.serve_policies.split(","):
                if pol == "aged":
                    r = serve.run_serving(trace, kbc.F32_DEV_X, budget=200 << 30, g=50,
                                          tune_cache=cache, min_nodes=4 << 20, age_weight=0.3)
                elif pol == "srpt":
                    r = serve.run_serving(trace, kbc.F32_DEV_X, budget=200 << 30, g=25,
                                          tune_cache=cache, min_nodes=8 << 20)
                elif pol == "loop":
                    r = serve.run_sequential(trace, kbc.F32_DEV_X)
                else:
                    raise SystemExit(f"unknown serving policy {pol!r}")
                say(f"{pol} (run {rep + 1})", r)
                runs.setdefault(pol, []).append(r)
        first = next(iter(runs.values()))[0]
        same = all(rr["results"][i] == first["results"][i]
                   for rs in runs.values() for rr in rs for i in first["results"])
        names = {"aged": ("pool_aged", "shortest remaining work first with aging (weight 0.3), "
                                       "batches >= 4M nodes of 50 steps"),
                 "srpt": ("pool", "shortest remaining work first, batches >= 8M nodes"),
                 "loop": ("loop", "first come first served, one box at a time")}
        out["serving"] = {"requests": len(trace), "rate_per_s": 20.0, "storage": "f32dev_x",
                          "hbm_budget_GB": 200, "repetitions": args.serve_reps,
                          "lattice_updates": first["lattice_updates"], "results_equal": same}
        for pol, rs in runs.items():
            key, desc = names[pol]
            out["serving"][key] = dict(lat(rs), policy=desc)
    return out


def precision_128(kbc, inputs, log):
    """128^3 decaying HIT (k0 = 4, u_rms = 0.04, nu = 5e-4, seed 1), 2000
    steps in each storage form: k(t) and Omega(t) every 10 steps against the
    FP64 path and, where stored, the oracle's series."""
    golden = os.path.join(ROOT, "tests", "golden", "oracle_hit128_series.txt")
    ref = None
    if os.path.exists(golden):
        import numpy as np
        ref = np.loadtxt(golden)
    u = inputs.hit(128, 4.0, 0.04, seed=1)
    out, series = {}, {}
    for name, dt, st in [("f64_pull", kbc.F64, kbc.PULL), ("f64_aa", kbc.F64, kbc.AA),
                         ("f32dev_pull", kbc.F32_DEV, kbc.PULL),
                         ("f32devx_pull", kbc.F32_DEV_X, kbc.PULL),
                         ("f32devx_aa", kbc.F32_DEV_X, kbc.AA), ("f16dev_aa", kbc.F16_DEV, kbc.AA)]:
        log(f"[precision] 128^3 {name}")
        with kbc.Box(128, 5e-4, dt, streaming=st) as b:
            b.init_velocity(u)
            ts, ks, ws = [0], [b.energy()], [b.enstrophy()]
            for t in range(10, 2001, 10):
                b.step(10)
                ts.append(t)
                ks.append(b.energy())
                ws.append(b.enstrophy())
        series[name] = (ts, ks, ws)
    t64, k64, w64 = series["f64_pull"]
    for name, (ts, ks, ws) in series.items():
        r = {"k_final": ks[-1], "omega_final": ws[-1],
             "max_rel_err_k_vs_f64": max(abs(a / b - 1) for a, b in zip(ks, k64)),
             "max_rel_err_omega_vs_f64": max(abs(a / b - 1) for a, b in zip(ws, w64))}
        if ref is not None:
            idx = {int(row[0]): row for row in ref}
            pts = [(k, w, idx[t]) for t, k, w in zip(ts, ks, ws) if t in idx]
            r["oracle_points"] = len(pts)
            r["max_rel_err_k_vs_oracle"] = max(abs(k / row[1] - 1) for k, w, row in pts)
            r["max_rel_err_omega_vs_oracle"] = max(abs(w / row[2] - 1) for k, w, row in pts)
        out[name] = r
    return out


def precision_512(kbc, inputs, log, steps=2000):
    """512^3 decaying HIT (k0 = 8, u_rms = 0.04, nu = 2.5e-4, seed 2),
    in-place AA, `steps` steps per storage form: MLUPS, HBM rate, energy,
    enstrophy and the shell spectrum against the FP64 run on the same field."""
    import torch

    from paper_1507_02518_amd import analysis

    n = 512
    log("[precision] building the 512^3 field")
    u = inputs.hit(n, 8.0, 0.04, seed=2)
    stream = torch.cuda.Stream()
    out, spec = {}, {}
    for name, dt in [("f64_aa", kbc.F64), ("f32dev_aa", kbc.F32_DEV),
                     ("f32devx_aa", kbc.F32_DEV_X), ("f16dev_aa", kbc.F16_DEV)]:
        log(f"[precision] 512^3 {name}")
        with kbc.Box(n, 2.5e-4, dt, streaming=kbc.AA, stream=stream.cuda_stream) as b:
            b.init_velocity(u)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.step(steps)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            k, w = b.energy(), b.enstrophy()
            _, uu = b.moments()
            spec[name] = analysis.spectrum(uu)
            del uu
            bpn = b.bytes_per_node_step()
        out[name] = {"ms_per_step": ms, "mlups": n ** 3 / (ms * 1e-3) / 1e6,
                     "algorithmic_GBs": bpn * n ** 3 / (ms * 1e-3) / 1e9, "k_final": k,
                     "omega_final": w}
    # resolution comparison (not parity): the oracle's 128^3 run of the same
    # flow (nu / 4, steps / 4), shells kappa <= 32
    golden = os.path.join(ROOT, "tests", "golden", "oracle_resolution128_spectrum.txt")
    e128 = None
    if os.path.exists(golden) and steps == 2000:
        import numpy as np
        e128 = np.loadtxt(golden)[:, 2]
    for name in out:
        out[name]["rel_err_k_vs_f64"] = abs(out[name]["k_final"] / out["f64_aa"]["k_final"] - 1)
        out[name]["rel_err_omega_vs_f64"] = abs(out[name]["omega_final"] /
                                                out["f64_aa"]["omega_final"] - 1)
        out[name]["spectrum_err_vs_f64"] = analysis.spectrum_error(spec[name], spec["f64_aa"])
        if e128 is not None:
            out[name]["resolution_vs_oracle128_kappa_le_32"] = dict(
                analysis.spectrum_error(spec[name], e128, kmax=32),
                k_ratio=out[name]["k_final"] / float(e128.sum()))
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


ONE_CORE_SNIPPET = """
import sys, time
sys.path.insert(0, {root!r})
import oracle
from paper_1507_02518_amd import inputs
u = inputs.hit({n}, {k0}, {urms}, seed={seed})
F = oracle.init_feq(u)
t0 = time.perf_counter()
oracle.run(F, oracle.beta_from_nu({nu}), {steps})
print(time.perf_counter() - t0, oracle.num_threads())
"""


def cpu_baseline(u, steps, one_core_n=128, one_core_steps=1):
    """The oracle on the host cores: all threads on `steps` steps of the 256^3
    box, and one thread (a child process with OMP_NUM_THREADS=1) on
    `one_core_steps` steps of a 128^3 box of the same flow."""
    import subprocess

    import oracle

    F = oracle.init_feq(u)
    beta = oracle.beta_from_nu(NU)
    t0 = time.perf_counter()
    oracle.run(F, beta, steps)
    dt = time.perf_counter() - t0
    del F
    code = ONE_CORE_SNIPPET.format(root=ROOT, n=one_core_n, k0=K0, urms=URMS, seed=SEED, nu=NU,
                                   steps=one_core_steps)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         check=True).stdout.split()
    dt1, thr1 = float(one[0]), int(one[1])
    return {"value": N ** 3 * steps / dt / 1e6, "unit": "MLUPS",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} step(s) of the same 256^3 HIT box, FP64, s=d+t+q, "
                      f"{dt:.1f} s of CPU time on {oracle.num_threads()} OpenMP threads",
            "one_core": {"value": one_core_n ** 3 * one_core_steps / dt1 / 1e6, "unit": "MLUPS",
                         "cores": thr1,
                         "sample": f"{one_core_steps} step(s) of a {one_core_n}^3 box of the "
                                   f"same flow, {dt1:.1f} s on one thread"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "host_cpus_usable": len(os.sched_getaffinity(0))}


FORMS_256 = [  # name, storage, streaming, variant ("exact": the exact stabilizer)
    ("f64_aa", "F64", "AA", None), ("f32dev_pull", "F32_DEV", "PULL", None),
    ("f32dev_aa", "F32_DEV", "AA", None), ("f32devx_pull", "F32_DEV_X", "PULL", None),
    ("f32devx_aa", "F32_DEV_X", "AA", None), ("f16dev_aa", "F16_DEV", "AA", None),
    ("f16dev_pull", "F16_DEV", "PULL", None), ("f64_pull_s_d", "F64", "PULL", "S_D"),
    ("f64_pull_central", "F64", "PULL", "S_CDTQ"),
    ("f32devx_pull_central", "F32_DEV_X", "PULL", "S_CDTQ"),
    ("f16dev_aa_central", "F16_DEV", "AA", "S_CDTQ"),
    ("f64_pull_exact_gamma", "F64", "PULL", "exact"),
    ("f32devx_pull_exact_gamma", "F32_DEV_X", "PULL", "exact")]
BIG_FORMS = [("f32devx_aa", "F32_DEV_X"), ("f16dev_aa", "F16_DEV"), ("f32dev_aa", "F32_DEV"),
             ("f64_aa", "F64")]


def _select(spec, names):
    if spec == "all":
        return list(names)
    if spec == "none":
        return []
    want = spec.split(",")
    bad = [w for w in want if w not in names]
    if bad:
        raise SystemExit(f"unknown form(s) {bad}; choose from {list(names)}")
    return want


def run_forms(kbc, torch, u_dev, table, names, steps, warmup, stream, n, nu):
    out = {}
    counts = read_valu_counts() if n == N else {}
    for name, dt, st, var in table:
        if name not in names:
            continue
        log(f"[bench] {n}^3 {name}")
        gamma = None
        var_name = var
        if var == "exact":
            var, gamma = None, "exact"
        variant = getattr(kbc, var) if var else None
        r = time_form(kbc, torch, u_dev, getattr(kbc, dt), getattr(kbc, st), steps, warmup,
                      stream, variant, gamma, n=n, nu=nu)
        t_valu = valu_issue_ms(counts, dt, st, var_name, n) if counts else None
        if t_valu is not None:
            r["valu_issue_ms"] = t_valu
            r["frac_valu_roofline"] = t_valu / r["ms_per_step"]
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
        log(f"[bench]   {r['mlups']:.0f} MLUPS, {r['algorithmic_GBs']:.0f} GB/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="all",
                    help="256^3 forms to time besides the headline: all, none or a list")
    ap.add_argument("--no-forms", dest="forms", action="store_const", const="none")
    ap.add_argument("--big-forms", default="f32devx_aa,f16dev_aa,f64_aa",
                    help="512^3 AA forms (all, none or a list of "
                         + ",".join(n for n, _ in BIG_FORMS) + ")")
    ap.add_argument("--big-steps", type=int, default=20)
    ap.add_argument("--big-warmup", type=int, default=4)
    ap.add_argument("--no-ensemble", dest="ensemble", action="store_false")
    ap.add_argument("--ensemble-steps", type=int, default=500)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-policies", default="aged,loop",
                    help="comma list of aged, srpt, loop")
    ap.add_argument("--serve-reps", type=int, default=2,
                    help="repetitions per policy, interleaved (the line gives their spread)")
    ap.add_argument("--precision", action="store_true",
                    help="run the storage-precision study (128^3 and 512^3) instead")
    ap.add_argument("--precision-steps-512", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the KBC box runs on a single MI355X "
              f"(--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)
    forms_256 = _select(args.forms, [f[0] for f in FORMS_256])
    forms_512 = _select(args.big_forms, [f[0] for f in BIG_FORMS])

    import torch

    from paper_1507_02518_amd import inputs, kbc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    kbc.load()

    if args.precision:
        res = {"metric": "storage precision: error vs FP64, D3Q27 KBC decaying HIT",
               "hit128_2000_steps": precision_128(kbc, inputs, log),
               "hit512": precision_512(kbc, inputs, log, args.precision_steps_512),
               "steps_512": args.precision_steps_512}
        print(json.dumps(res), flush=True)
        return

    log(f"[bench] building the 256^3 HIT field (seed {SEED})")
    u = inputs.hit(N, K0, URMS, seed=SEED)
    u_dev = torch.from_numpy(u).cuda()
    stream = torch.cuda.Stream()
    assert stream.cuda_stream, "need a non-null stream"
    torch.cuda.synchronize()

    log("[bench] FP64 pull (headline)")
    head = time_form(kbc, torch, u_dev, kbc.F64, kbc.PULL, args.steps, args.warmup, stream)
    log(f"[bench]   {head['mlups']:.0f} MLUPS, {head['algorithmic_GBs']:.0f} GB/s")

    forms = run_forms(kbc, torch, u_dev, FORMS_256, forms_256, args.steps, args.warmup, stream,
                      N, NU)
    log("[bench] copy ceiling (between two buffers and in place)")
    copy_gbs, inplace_gbs = copy_ceiling(kbc, torch, stream)
    log(f"[bench]   {copy_gbs:.0f} GB/s copy, {inplace_gbs:.0f} GB/s in place")
    add_ceiling_fracs(forms, copy_gbs, inplace_gbs)
    del u_dev
    torch.cuda.empty_cache()

    big = {}
    if forms_512:
        log(f"[bench] building the {BIG_N}^3 HIT field (k0 = {BIG_K0}, seed {BIG_SEED})")
        ub = torch.from_numpy(inputs.hit(BIG_N, BIG_K0, URMS, seed=BIG_SEED)).cuda()
        torch.cuda.synchronize()
        table = [(nm, dt, "AA", None) for nm, dt in BIG_FORMS]
        big = run_forms(kbc, torch, ub, table, forms_512, args.big_steps, args.big_warmup, stream,
                        BIG_N, BIG_NU)
        add_ceiling_fracs(big, copy_gbs, inplace_gbs)
        del ub
        torch.cuda.empty_cache()

    batched = ensemble_and_serving(kbc, args)

    traffic_bytes = read_counters()
    roofline = {
        "bound": "hbm",
        "achieved": round(head["algorithmic_GBs"], 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(head["algorithmic_GBs"] / PEAK_HBM_GBS, 4),
        "traffic": traffic_bytes,
        "kernel": "k_step<F64, d+t+q, pull>",
        "bytes_per_node_step": head["bytes_per_node_step"],
        "nodes_per_launch": N ** 3,
        "copy_ceiling_GBs": round(copy_gbs, 1),
        "frac_of_copy_ceiling": round(head["algorithmic_GBs"] / copy_gbs, 4),
        "inplace_ceiling_GBs": round(inplace_gbs, 1),
    }
    cpu = None
    if not args.no_cpu:
        log(f"[bench] CPU oracle sample ({args.cpu_steps} step(s) at 256^3, then one thread)")
        cpu = cpu_baseline(u, args.cpu_steps)
        log(f"[bench]   {cpu['value']:.3f} MLUPS on {cpu['cores']} threads, "
            f"{cpu['one_core']['value']:.3f} MLUPS on one")

    out = {
        "metric": METRIC,
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "D3Q27 KBC (s=d+t+q, entropic gamma) step, 256^3 periodic "
                               "decaying HIT, k0=4, u_rms=0.04, nu=5e-4, seed 0, FP64 pull",
                   "nodes": N ** 3, "streaming": "pull", "storage": "f64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "big_forms": {"workload": f"{BIG_N}^3 decaying HIT, k0={BIG_K0:g}, u_rms={URMS}, "
                                  f"nu={BIG_NU}, seed {BIG_SEED}, in place (AA), s=d+t+q",
                      "steps": args.big_steps, "warmup": args.big_warmup, **big} if big else None,
    }
    out.update(batched)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
