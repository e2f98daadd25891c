"""Ensembles and a serving loop on top of the pool C-ABI.

``run_ensemble`` advances a fixed set of boxes together (one pool, batched
launches) or one at a time (a plain loop over ``Box``).  ``run_serving``
replays a trace of requests arriving over wall-clock time: requests are
admitted as soon as they have arrived and the HBM budget and a slot allow,
every resident box advances in each batch, finished boxes return their
kinetic energy and enstrophy and leave.  ``run_sequential`` serves the same
trace first-in first-out, one box at a time.  All three produce per-box
results with the same kernels and arithmetic, so their outputs are equal and
the comparison is one of throughput and latency only.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs, kbc


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the trace start
    shape: tuple            # (nx, ny, nz)
    nu: float
    steps: int
    u: np.ndarray = field(repr=False)

    @property
    def nodes(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]


def ensemble_boxes(count=64, seed=0, edges=(24, 32, 48, 64, 96), steps=500,
                   nu_range=(2e-4, 5e-3)):
    """Boxes of the batched-ensemble workload: seeded edges, half
    Taylor-Green (U = u_rms draw), half decaying HIT (u_rms in [0.02, 0.05],
    k0 in {2, 4}), viscosity log-uniform."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(edges))
        urms = float(rng.uniform(0.02, 0.05))
        nu = float(np.exp(rng.uniform(np.log(nu_range[0]), np.log(nu_range[1]))))
        if i % 2 == 0:
            u = inputs.taylor_green(n, urms)
        else:
            u = inputs.hit(n, float(rng.choice([2.0, 4.0])), urms, seed=seed * 1000 + i)
        out.append(Request(i, 0.0, (n, n, n), nu, steps, u))
    return out


def serving_trace(count=96, rate=20.0, seed=0, edges=(32, 48, 64, 96, 128, 192),
                  steps_range=(200, 5000), nu_range=(2.5e-4, 2e-3), u_rms=0.03, k0=4.0):
    """Poisson arrivals at `rate` per second; edge uniform over `edges`, steps
    and viscosity log-uniform.  One seeded HIT start per edge is shared by
    the requests of that size (they differ in viscosity and step count)."""
    rng = np.random.default_rng(seed)
    fields = {}
    out = []
    t = 0.0
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice(edges))
        steps = int(round(np.exp(rng.uniform(np.log(steps_range[0]), np.log(steps_range[1])))))
        nu = float(np.exp(rng.uniform(np.log(nu_range[0]), np.log(nu_range[1]))))
        if n not in fields:
            fields[n] = inputs.hit(n, k0, u_rms, seed=seed * 7919 + n)
        out.append(Request(i, t, (n, n, n), nu, steps, fields[n]))
    return out


def run_ensemble(reqs, dtype=kbc.F32_DEV_X, batched=True, g=50, budget=None,
                 tune_cache=None, launch=None):
    """Advance all boxes to their step counts; returns timing and results."""
    lu = sum(r.nodes * r.steps for r in reqs)
    results = {}
    if batched:
        need = sum(27 * r.nodes * (8 if dtype == kbc.F64 else (2 if dtype == kbc.F16_DEV else 4))
                   for r in reqs)
        budget = budget or int(need * 1.1 + (64 << 20))
        with kbc.Pool(budget, dtype, max_slots=max(1, len(reqs)), tune_cache=tune_cache) as pool:
            if launch:
                pool.set_launch(*launch)
            t0 = time.perf_counter()
            slots = {r.rid: pool.admit(r.u, r.nu, r.steps) for r in reqs}
            left = max(r.steps for r in reqs)
            while left > 0:
                pool.advance(min(g, left))
                left -= min(g, left)
            pool.sync()
            for r in reqs:
                results[r.rid] = pool.result(slots[r.rid])
            wall = time.perf_counter() - t0
            info = pool.info()
    else:
        t0 = time.perf_counter()
        for r in reqs:
            with kbc.Box(r.shape, r.nu, dtype, streaming=kbc.AA) as b:
                b.init_velocity(r.u)
                b.step(r.steps)
                results[r.rid] = (b.energy(), b.enstrophy())
        wall = time.perf_counter() - t0
        info = None
    return {"wall_s": wall, "lattice_updates": lu, "mlups": lu / wall / 1e6,
            "results": results, "launch": info}


def _percentiles(lat):
    a = np.array(sorted(lat))
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def run_serving(trace, dtype=kbc.F32_DEV_X, budget=200 << 30, g=25, max_slots=1024,
                tune_cache=None, log=None, policy="srpt", min_nodes=8 << 20, age_weight=0.0):
    """Continuous batching over wall-clock arrivals.

    policy "all": every resident box advances in every batch (processor
    sharing).  policy "srpt": each batch advances the resident boxes with the
    least remaining work (nodes x steps left) first, adding boxes until the
    batch holds at least `min_nodes` nodes, enough to fill the GPU; the
    others wait, which lets short requests overtake long ones.  With
    age_weight w > 0 a box's remaining work is reduced by w x (its waiting
    time) x (the pool's measured rate), so a long request that has waited
    long enough goes ahead of newly arrived short ones (w -> infinity tends
    to first-come first-served).
    """
    elem = 8 if dtype == kbc.F64 else (2 if dtype == kbc.F16_DEV else 4)
    for r in trace:
        if 27 * r.nodes * elem > budget:
            raise ValueError(f"request {r.rid} ({r.shape}) needs {27 * r.nodes * elem} bytes of "
                             f"populations, more than the HBM budget of {budget} bytes")
    pending = list(trace)
    active = {}
    left = {}
    done = {}
    results = {}
    work_done = 0
    with kbc.Pool(budget, dtype, max_slots=max_slots, tune_cache=tune_cache) as pool:
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            # admit every arrived request that fits (in arrival order)
            while pending and pending[0].arrival <= now:
                r = pending[0]
                try:
                    slot = pool.admit(r.u, r.nu, r.steps)
                except kbc.KbcError as e:
                    if e.code != kbc.KBC_ECAPACITY:
                        raise
                    if not active:
                        # nothing resident will ever free room for it
                        raise RuntimeError(f"request {r.rid} ({r.shape}) does not fit the empty "
                                           f"pool: {e}") from e
                    break
                active[slot] = r
                left[slot] = r.steps
                pending.pop(0)
            if not active:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                continue
            runnable = [sl for sl in active if left[sl] > 0]
            if policy == "srpt":
                # node-steps per second so far (a typical rate before any work)
                rate = max(work_done / now, 1e9) if work_done > 0 and now > 0 else 2e10
                runnable.sort(key=lambda sl: active[sl].nodes * left[sl]
                              - age_weight * (now - active[sl].arrival) * rate)
                chosen, nodes = [], 0
                for sl in runnable:
                    chosen.append(sl)
                    nodes += active[sl].nodes
                    if nodes >= min_nodes:
                        break
            else:
                chosen = runnable
            if chosen:
                pool.advance(g, chosen)
                for sl in chosen:
                    work_done += active[sl].nodes * min(g, left[sl])
                    left[sl] -= min(g, left[sl])
            # collect finished boxes
            finished = 0
            for slot in list(active):
                if left[slot] == 0 and pool.poll(slot) == 0:
                    r = active.pop(slot)
                    del left[slot]
                    results[r.rid] = pool.result(slot)
                    pool.release(slot)
                    done[r.rid] = time.perf_counter() - t0
                    finished += 1
                    if log:
                        log(f"[serve] request {r.rid} done at {done[r.rid]:.3f}s")
            if not finished:
                time.sleep(2e-4)
        pool.sync()
        wall = time.perf_counter() - t0
        info = pool.info()
    lat = [done[r.rid] - r.arrival for r in trace]
    lu = sum(r.nodes * r.steps for r in trace)
    p50, p99 = _percentiles(lat)
    return {"wall_s": wall, "lattice_updates": lu, "mlups": lu / wall / 1e6, "p50_s": p50,
            "p99_s": p99, "results": results, "latencies": lat, "launch": info}


def run_sequential(trace, dtype=kbc.F32_DEV_X):
    """First-in first-out, one box at a time, each on its own lattice."""
    t0 = time.perf_counter()
    done = {}
    results = {}
    for r in trace:
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        with kbc.Box(r.shape, r.nu, dtype, streaming=kbc.AA) as b:
            b.init_velocity(r.u)
            b.step(r.steps)
            results[r.rid] = (b.energy(), b.enstrophy())
        done[r.rid] = time.perf_counter() - t0
    wall = time.perf_counter() - t0
    lat = [done[r.rid] - r.arrival for r in trace]
    lu = sum(r.nodes * r.steps for r in trace)
    p50, p99 = _percentiles(lat)
    return {"wall_s": wall, "lattice_updates": lu, "mlups": lu / wall / 1e6, "p50_s": p50,
            "p99_s": p99, "results": results, "latencies": lat}
