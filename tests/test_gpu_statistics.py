"""GPU flow statistics (section V) against the oracle's numpy statistics on
the same state: gradient statistics (2nd and 8th order), the stabilizer's
mean / std / min / max, and the x-correlations."""
import sys

import numpy as np
import pytest

from oracle import statistics as ost
from paper_1507_02518_amd import inputs, kbc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(shape=(24, 20, 18), steps=8, **kw):
    u0 = inputs.hit(shape, 3.0, 0.05, seed=21) if shape[0] == shape[1] == shape[2] else \
        inputs.smooth_random(shape, 0.05, seed=21)
    b = kbc.Box(shape, 2e-3, **kw)
    b.init_velocity(u0)
    b.step(steps)
    return b


@pytest.mark.parametrize("order", [2, 8])
def test_gradient_statistics_match_oracle(order):
    with _state() as b:
        got = b.statistics(order)
        _, u = b.moments()
        w2 = b.enstrophy()
    ref = ost.statistics(u, 2e-3, order)
    for key in ("k", "omega", "epsilon", "div2"):
        assert got[key] == pytest.approx(ref[key], rel=1e-12), key
    for n in range(2, 7):
        assert got["dudx_moments"][n] == pytest.approx(ref["dudx_moments"][n], rel=1e-11,
                                                       abs=1e-30), n
    for n in range(3, 7):
        assert got["skewness"][n] == pytest.approx(ref["skewness"][n], rel=1e-10, abs=1e-12), n
    if order == 2:
        assert got["omega"] == pytest.approx(w2, rel=1e-13)
    say(f"order {order}: Omega {got['omega']:.6e} eps {got['epsilon']:.6e} "
        f"S3 {got['skewness'][3]:.4f} S4 {got['skewness'][4]:.4f}")


@pytest.mark.parametrize("variant,gamma", [(kbc.S_DTQ, None), (kbc.S_CDTQ, None),
                                           (kbc.S_DTQ, "exact"), (kbc.S_D, 1.7)])
def test_gamma_statistics_match_oracle(orc, variant, gamma):
    nu = 2e-3
    with _state(variant=variant, gamma=gamma) as b:
        got = b.gamma_statistics()
        F = b.populations()
    kw = {"exact": True} if gamma == "exact" else ({"gamma": gamma} if gamma else {})
    _, gf = orc.collide_field(F, orc.beta_from_nu(nu), variant=variant, want_gamma=True, **kw)
    ref = ost.gamma_statistics(gf)
    say(f"variant {variant} gamma {gamma}: mean {got['mean']:.6f} std {got['std']:.3e} "
        f"[{got['min']:.4f}, {got['max']:.4f}]")
    assert got["mean"] == pytest.approx(ref["mean"], rel=1e-13)
    assert got["min"] == pytest.approx(ref["min"], rel=1e-12)
    assert got["max"] == pytest.approx(ref["max"], rel=1e-12)
    if gamma is not None and gamma != "exact":
        assert got["std"] == 0.0 and got["mean"] == gamma
    else:
        assert got["std"] == pytest.approx(ref["std"], rel=1e-8)
        assert got["std"] > 1e-4


def test_correlation_matches_oracle():
    with _state(shape=(40, 12, 10)) as b:
        r11, r22 = b.correlation(20)
        _, u = b.moments()
    o11, o22 = ost.correlation_x(u, 20)
    assert np.abs(r11 - o11).max() < 1e-13 and np.abs(r22 - o22).max() < 1e-13
    assert r11[0] == 1.0 and r22[0] == 1.0


def test_statistics_argument_errors():
    with _state(shape=(8, 8, 8), steps=1) as b:
        with pytest.raises(kbc.KbcError) as e:
            b.statistics(4)
        assert e.value.code == kbc.KBC_EINVAL
        with pytest.raises(kbc.KbcError) as e:
            b.correlation(8)
        assert e.value.code == kbc.KBC_EINVAL


def test_kida_statistics_follow_the_papers_run_a():
    """Kida vortex, N = 100, Re = 6000, KBC s = d+t+q (the paper's run A):
    k, Omega and epsilon (eighth-order gradients) within 2% and the even
    skewness factors within 6% of the printed table at t = 0.25, 0.5, 0.75.
    The start here is the equilibrium of rho = 1, not the paper's pre-solved
    density, so the match is close but not exact (context, not parity)."""
    import os

    from paper_1507_02518_amd import kida_table

    ref = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden",
                                  "paper_table_statistics_A.txt"))
    res = kida_table.kida_table(100)
    for row in ref:
        got = res["times"][f"{row[0]:g}"]
        say(f"t={row[0]:g}: k {got['k*1e4']:.4g}/{row[1]} Omega {got['Omega*N^2']:.4g}/{row[2]} "
            f"eps {got['eps*N*1e5']:.4g}/{row[3]} S4 {got['S4']:.4g}/{row[5]} "
            f"S6 {got['S6']:.4g}/{row[7]}")
        assert got["k*1e4"] == pytest.approx(row[1], rel=0.02)
        assert got["Omega*N^2"] == pytest.approx(row[2], rel=0.02)
        assert got["eps*N*1e5"] == pytest.approx(row[3], rel=0.02)
        assert got["S4"] == pytest.approx(row[5], rel=0.06)
        assert got["S6"] == pytest.approx(row[7], rel=0.06)
        assert 1.5 < got["gamma_mean"] < 2.2 and got["gamma_std"] > 0.0
