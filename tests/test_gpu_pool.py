"""GPU tests of the batched ensemble (pool): parity with the oracle, each box
identical alone and in a mix, HBM-budget admission, failure isolation and
launch-shape independence."""
import os
import sys
import tempfile

import numpy as np
import pytest

from paper_1507_02518_amd import inputs, kbc, serve

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pop_bytes(shape, dtype):
    return 27 * shape[0] * shape[1] * shape[2] * {kbc.F64: 8, kbc.F16_DEV: 2}.get(dtype, 4)


def _alone(shape, nu, u, steps, dtype, gamma=None):
    with kbc.Box(shape, nu, dtype, streaming=kbc.AA, gamma=gamma) as b:
        b.init_velocity(u)
        b.step(steps)
        rho, uu = b.moments()
        return b.energy(), b.enstrophy(), rho, uu


BOXES = [((13, 9, 7), 3e-4, 7), ((16, 16, 16), 1e-3, 12), ((20, 6, 11), 5e-3, 9),
         ((8, 8, 8), 2e-4, 1)]


# Bounds on rho, u (absolute) and k (relative) after at most 12 steps of
# solenoidal starts with u_rms = 0.03 (|u_a| up to about 0.1), where the
# largest stored deviation |f - W| is about 0.025.  FP64 differs by rounding
# order only.  The deviation forms round every stored population once per
# step, independently: FP32 at up to 0.025 * 2^-24 = 1.5e-9, FP16 (11
# significant bits of the scaled deviation) at up to 0.025 / 2048 = 1.2e-5.
# rho and u sum 27 of them per node and step, a random walk over 12 x 27
# roundings: sqrt(324) x 1.5e-9 = 3e-8 (FP32), sqrt(324) x 1.2e-5 / 4 = 5e-5
# (FP16, where most deviations are far below the largest); measured 1.1e-8
# and 5.2e-5.  k, about u^2 with u ~ 0.03, averages the node errors: measured
# 9.9e-8 and 4.6e-5, bounds 3e-7 and 2e-4.
@pytest.mark.parametrize("dtype,tol_ru,tol_k", [(kbc.F64, 1e-14, 1e-12),
                                                (kbc.F32_DEV_X, 3e-8, 3e-7),
                                                (kbc.F16_DEV, 2e-4, 2e-4)])
@pytest.mark.parametrize("variant", [kbc.S_DTQ, kbc.S_CDTQ])
def test_pool_boxes_match_oracle(orc, variant, dtype, tol_ru, tol_k):
    """Four boxes of different shapes, viscosities and step counts advanced
    together by the pool kernel, in FP64 and in FP32 / FP16 deviation
    storage: density, velocity and energy of each against the oracle."""
    with kbc.Pool(64 << 20, dtype, variant=variant, max_slots=8) as pool:
        slots = []
        for i, (shape, nu, steps) in enumerate(BOXES):
            # solenoidal: FP16 storage overflows on the acoustic transients
            # of a start with divergence
            u = inputs.hit(shape, 2.0, 0.03, seed=i)
            slots.append((pool.admit(u, nu, steps), shape, nu, steps, u))
        for _ in range(4):
            pool.advance(3)
        worst = [0.0, 0.0]
        for slot, shape, nu, steps, u in slots:
            k, w, rho, ug = pool.result(slot, shape)
            F = orc.run(orc.init_feq(u), orc.beta_from_nu(nu), steps, variant=variant)
            rho_o, u_o = orc.macros(F)
            e_ru = max(np.abs(rho - rho_o).max(), np.abs(ug - u_o).max())
            e_k = abs(k / orc.energy(u_o) - 1)
            worst = [max(worst[0], e_ru), max(worst[1], e_k)]
            assert e_ru <= tol_ru and e_k <= tol_k, (shape, e_ru, e_k)
    say(f"pool vs oracle (variant {variant}, dtype {dtype}): max |d rho|, |d u| {worst[0]:.3e}, "
        f"max rel dk {worst[1]:.3e}")


@pytest.mark.parametrize("dtype", [kbc.F64, kbc.F32_DEV_X, kbc.F16_DEV])
def test_each_box_is_identical_alone_and_in_the_mix(dtype):
    """Staggered admissions (boxes join at different times and parities),
    batches of different lengths: every box equals its own solo run bit for
    bit."""
    specs = [((24, 24, 24), 4e-4, 31, 0), ((13, 17, 9), 1e-3, 18, 1), ((32, 32, 32), 2e-4, 25, 2),
             ((10, 10, 10), 3e-3, 40, 3), ((7, 19, 5), 6e-4, 11, 4), ((64, 5, 3), 8e-4, 14, 5)]
    fields = [inputs.hit(s, 3.0, 0.04, seed=seed) for s, _, _, seed in specs]
    budget = sum(_pop_bytes(s, dtype) for s, _, _, _ in specs) + (16 << 20)
    got = {}
    with kbc.Pool(budget, dtype, max_slots=8) as pool:
        slot = {}
        slot[0] = pool.admit(fields[0], specs[0][1], specs[0][2])
        pool.advance(3)
        slot[1] = pool.admit(fields[1], specs[1][1], specs[1][2])
        pool.advance(4)
        slot[2] = pool.admit(fields[2], specs[2][1], specs[2][2])
        slot[3] = pool.admit(fields[3], specs[3][1], specs[3][2])
        pool.advance(5)
        slot[4] = pool.admit(fields[4], specs[4][1], specs[4][2])
        pool.advance(1)
        slot[5] = pool.admit(fields[5], specs[5][1], specs[5][2])
        for g in (2, 7, 1, 9, 9, 9, 9):
            pool.advance(g)
        pool.sync()
        for i, (s, nu, steps, _) in enumerate(specs):
            assert pool.poll(slot[i]) == 0
            got[i] = pool.result(slot[i], s)
    for i, (s, nu, steps, _) in enumerate(specs):
        k, w, rho, u = _alone(s, nu, fields[i], steps, dtype)
        assert got[i][0] == k and got[i][1] == w, (i, got[i][:2], (k, w))
        assert np.array_equal(got[i][2], rho) and np.array_equal(got[i][3], u), i
    say(f"alone vs mix dtype={dtype}: bitwise equal")


def test_launch_groups_keep_each_box_identical():
    """Boxes whose populations together exceed the last-level-cache target of
    a launch group (216 MiB) run in several groups, each taking all its steps
    of a batch before the next; with two parities and boxes of different
    sizes every box still equals its own solo run bit for bit."""
    dtype = kbc.F64
    specs = [((64, 64, 64), 4e-4, 23), ((64, 64, 64), 1e-3, 17), ((60, 64, 64), 2e-4, 20),
             ((56, 56, 64), 3e-3, 13), ((40, 40, 40), 6e-4, 29), ((48, 48, 48), 5e-4, 21),
             ((64, 64, 48), 7e-4, 15), ((32, 32, 32), 2e-3, 19)]
    fields = [inputs.hit(sh, 3.0, 0.04, seed=10 + i) for i, (sh, _, _) in enumerate(specs)]
    first = sum(_pop_bytes(sh, dtype) for sh, _, _ in specs[:6])
    assert first > 216 << 20
    budget = sum(_pop_bytes(sh, dtype) for sh, _, _ in specs) + (16 << 20)
    got = {}
    with kbc.Pool(budget, dtype, max_slots=8) as pool:
        slot = {i: pool.admit(fields[i], nu, st) for i, (_, nu, st) in enumerate(specs[:6])}
        pool.advance(3)
        for i in (6, 7):
            slot[i] = pool.admit(fields[i], specs[i][1], specs[i][2])
        for g in (4, 5, 8, 8, 8):
            pool.advance(g)
        pool.sync()
        for i, (sh, _, _) in enumerate(specs):
            assert pool.poll(slot[i]) == 0
            got[i] = pool.result(slot[i], sh)
    for i, (sh, nu, steps) in enumerate(specs):
        k, w, rho, u = _alone(sh, nu, fields[i], steps, dtype)
        assert got[i][0] == k and got[i][1] == w, (i, got[i][:2], (k, w))
        assert np.array_equal(got[i][2], rho) and np.array_equal(got[i][3], u), i
    say("launch groups: every box bitwise equal to its solo run")


@pytest.mark.parametrize("policy,min_nodes,age_weight", [("srpt", 1 << 16, 0.0),
                                                         ("srpt", 1 << 16, 0.3),
                                                         ("all", 0, 0.0)])
def test_serving_policies_return_the_loops_results(policy, min_nodes, age_weight):
    """A short served trace (requests arriving while others run, uneven
    sizes and step counts) under each scheduling policy: every request
    finishes and its energy and enstrophy equal, bit for bit, those of the
    first-come first-served loop of single boxes."""
    trace = serve.serving_trace(12, rate=4000.0, seed=3, edges=(16, 24, 32),
                                steps_range=(100, 400), u_rms=0.03, k0=2.0)
    srv = serve.run_serving(trace, kbc.F32_DEV_X, budget=1 << 30, g=10, max_slots=16,
                            policy=policy, min_nodes=min_nodes, age_weight=age_weight)
    seq = serve.run_sequential(trace, kbc.F32_DEV_X)
    assert sorted(srv["results"]) == [r.rid for r in trace]
    for r in trace:
        assert srv["results"][r.rid] == seq["results"][r.rid], r.rid
    assert all(lat > 0 for lat in srv["latencies"])
    say(f"serving {policy} (min {min_nodes}, aging {age_weight}): p50 {srv['p50_s']:.3f}s "
        f"p99 {srv['p99_s']:.3f}s, results equal to the loop")


def test_budget_and_slots_bound_admission():
    s = (16, 16, 16)
    u = inputs.taylor_green(s, 0.04)
    one = _pop_bytes(s, kbc.F32_DEV_X)
    grain = 65536
    per = (one + grain - 1) // grain * grain
    with kbc.Pool(2 * per, kbc.F32_DEV_X, max_slots=4) as pool:
        a = pool.admit(u, 1e-3, 5)
        b = pool.admit(u, 1e-3, 5)
        with pytest.raises(kbc.KbcError) as e:
            pool.admit(u, 1e-3, 5)
        assert e.value.code == kbc.KBC_ECAPACITY
        assert pool.info()["bytes_used"] == 2 * per
        pool.advance(5)
        pool.result(a)
        pool.release(a)
        c = pool.admit(u, 1e-3, 5)
        assert c == a
        pool.release(b)
        pool.release(c)
        assert pool.info()["bytes_used"] == 0
    with kbc.Pool(64 << 20, kbc.F32_DEV_X, max_slots=2) as pool:
        pool.admit(u, 1e-3, 1)
        pool.admit(u, 1e-3, 1)
        with pytest.raises(kbc.KbcError) as e:
            pool.admit(u, 1e-3, 1)
        assert e.value.code == kbc.KBC_ECAPACITY


def test_result_before_the_end_is_a_state_error_and_bad_input_is_rejected():
    s = (8, 8, 8)
    u = inputs.taylor_green(s, 0.04)
    with kbc.Pool(16 << 20, kbc.F32_DEV_X, max_slots=4) as pool:
        a = pool.admit(u, 1e-3, 10)
        pool.advance(3)
        with pytest.raises(kbc.KbcError) as e:
            pool.result(a)
        assert e.value.code == kbc.KBC_ESTATE
        bad = u.copy()
        bad[0, 1, 1, 1] = 1.5
        with pytest.raises(kbc.KbcError) as e:
            pool.admit(bad, 1e-3, 10)
        assert e.value.code == kbc.KBC_EUNSTABLE
        assert pool.info()["boxes"] == 1


def test_a_diverging_box_does_not_perturb_the_others():
    """Forced LBGK (gamma = 2): an under-resolved box at tiny viscosity
    blows up (energy grows by orders of magnitude or turns non-finite; the
    oracle sees the same blow-up near step 175); the resolved box next to it
    equals its solo run."""
    s = (16, 16, 16)
    wild = inputs.hit(s, 2.0, 0.05, seed=0)
    calm = inputs.taylor_green(s, 0.02)
    with kbc.Pool(64 << 20, kbc.F64, max_slots=4, gamma=2.0) as pool:
        a = pool.admit(wild, 1e-5, 300)
        b = pool.admit(calm, 1e-2, 300)
        for _ in range(10):
            pool.advance(30)
        c = pool.admit(calm, 1e-2, 10)
        pool.advance(7, [c])
        pool.advance(7, [c])
        k0 = 1.5 * 0.05 ** 2
        try:
            ka_, _ = pool.result(a)
            diverged = not np.isfinite(ka_) or ka_ > 100 * k0
        except kbc.KbcError as e:
            diverged = e.code == kbc.KBC_EUNSTABLE
        assert diverged
        k, w, rho, u = pool.result(b, s)
        kc, wc, rhoc, uc = pool.result(c, s)
    ka, wa, rhoa, ua = _alone(s, 1e-2, calm, 300, kbc.F64, gamma=2.0)
    assert k == ka and w == wa and np.array_equal(rho, rhoa) and np.array_equal(u, ua)
    kc2, wc2, rhoc2, uc2 = _alone(s, 1e-2, calm, 10, kbc.F64, gamma=2.0)
    assert kc == kc2 and np.array_equal(uc, uc2)


def test_launch_shape_does_not_change_results_and_tuner_settles():
    specs = [((24, 24, 24), 4e-4), ((40, 12, 9), 1e-3), ((33, 33, 33), 2e-4)]
    fields = [inputs.hit(s, 3.0, 0.04, seed=i) for i, (s, _) in enumerate(specs)]
    outs = []
    for launch in [(128, 512, 1), (512, 4096, 8), (64, 7, 3), (256, 0, 1), (512, 0, 2)]:
        with kbc.Pool(256 << 20, kbc.F32_DEV_X, max_slots=4) as pool:
            pool.set_launch(*launch)
            slots = [pool.admit(f, nu, 20) for f, (_, nu) in zip(fields, specs)]
            pool.advance(20)
            outs.append([pool.result(sl, s) for sl, (s, _) in zip(slots, specs)])
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert a[0] == b[0] and np.array_equal(a[3], b[3])
    # the tuner: a round of 2 x 12 timed batches for the class of these boxes,
    # then the chosen shape; a second pool reads it back from the cache file
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tune.txt")
        with kbc.Pool(256 << 20, kbc.F32_DEV_X, max_slots=4, tune_cache=cache) as pool:
            slots = [pool.admit(f, nu, 600) for f, (_, nu) in zip(fields, specs)]
            for _ in range(26):
                pool.advance(20)
            pool.sync()
            info = pool.info()
            assert not info["tuning"]
            for _ in range(4):
                pool.advance(20)
            res = [pool.result(sl, s) for sl, (s, _) in zip(slots, specs)]
        assert os.path.exists(cache)
        with kbc.Pool(256 << 20, kbc.F32_DEV_X, max_slots=4, tune_cache=cache) as pool:
            slots2 = [pool.admit(f, nu, 20) for f, (_, nu) in zip(fields, specs)]
            pool.advance(20)
            info2 = pool.info()
            assert not info2["tuning"]
            assert (info2["block"], info2["grid"], info2["sub"]) == (info["block"], info["grid"],
                                                                      info["sub"])
    for sl_res, (s, nu), f in zip(res, specs, fields):
        k, w, rho, u = _alone(s, nu, f, 600, kbc.F32_DEV_X)
        assert sl_res[0] == k and np.array_equal(sl_res[3], u)
    say(f"tuned launch: block={info['block']} grid={info['grid']} sub={info['sub']}")
