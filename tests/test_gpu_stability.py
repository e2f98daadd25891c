"""GPU checks of the Kida-vortex workload and the stability comparison
(section V): short KBC / LBGK / RLB runs on the Kida start against the
oracle, and the stability classification on a small box."""
import sys

import numpy as np
import pytest

from paper_1507_02518_amd import inputs, kbc, stability

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", ["KBC s=d+t+q", "KBC s=d~", "LBGK", "RLB s=d+t", "RLB s=d~"])
def test_kida_short_runs_match_oracle(orc, name):
    """24^3 Kida start, Re = 2000 (nu = U0 N / Re), 20 steps, every model
    family: populations element-wise against the oracle."""
    n, u0, re, steps = 24, 0.05, 2000.0, 20
    nu = u0 * n / re
    beta = orc.beta_from_nu(nu)
    variant, kind = stability.models()[name]
    gamma = {"entropic": None, "lbgk": 2.0, "rlb": 1.0 / beta}[kind]
    u = inputs.kida(n, u0)
    with kbc.Box(n, nu, kbc.F64, variant=variant, streaming=kbc.AA, gamma=gamma) as b:
        b.init_velocity(u)
        b.step(steps)
        f = b.populations()
    F = orc.run(orc.init_feq(u), beta, steps, variant=variant, gamma=gamma)
    err = np.abs(f - F).max()
    say(f"Kida {name}: max|df| {err:.3e}")
    assert err <= 1e-13


def test_stability_classification_on_a_small_box():
    """32^3 Kida at a very high Reynolds number: KBC decays to 5% of its
    initial enstrophy (stable); regularised LB with s = d+t loses
    finiteness or gains energy (unstable), the contrast section V reports."""
    r_kbc = stability.kida_run(kbc.S_DTQ, "entropic", 1e6, n=32, dtype=kbc.F64, max_steps=20000)
    r_rlb = stability.kida_run(kbc.S_DT, "rlb", 1e6, n=32, dtype=kbc.F64, max_steps=20000)
    say(f"KBC: {r_kbc['verdict']} after {r_kbc['steps']}; RLB d+t: {r_rlb['verdict']} "
        f"after {r_rlb['steps']}")
    assert r_kbc["verdict"] == "stable"
    assert r_rlb["verdict"] == "unstable"
