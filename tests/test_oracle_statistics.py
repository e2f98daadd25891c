"""Pins of the oracle's flow statistics (section V): stencil order, exact
single-mode values, a discrete identity that ties Omega, epsilon and the
divergence together, the Taylor-Green closed form, and the paper's own table
of statistics for the derived scales."""
import os

import numpy as np
import pytest

import oracle as o
from oracle import statistics as st
from paper_1507_02518_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("order,rate", [(2, 2), (8, 8)])
def test_stencil_converges_at_its_order(order, rate):
    """Relative error of d/dx sin(theta x) falls as theta^order."""
    errs = []
    for n in (32, 64):
        th = 2 * np.pi / n
        x = np.arange(n)
        f = np.sin(th * x)[None, None, :] * np.ones((2, 2, 1))
        d = st.derivative(f, 0, order)[0, 0]
        errs.append(np.abs(d - th * np.cos(th * x)).max() / th)
    assert np.log2(errs[0] / errs[1]) == pytest.approx(rate, abs=0.05)


def test_skewness_of_a_single_mode():
    """u_x = sin(2 pi x / N): du/dx is a scaled cosine, so S^3 = S^5 = 0,
    S^4 = <c^4>/<c^2>^2 = 3/2 and S^6 = <c^6>/<c^2>^3 = 5/2 exactly."""
    n = 24
    u = np.zeros((3, 4, 4, n))
    u[0] = np.sin(2 * np.pi * np.arange(n) / n)[None, None, :]
    for order in (2, 8):
        s = st.statistics(u, 0.01, order)["skewness"]
        assert abs(s[3]) < 1e-13 and abs(s[5]) < 1e-13
        assert s[4] == pytest.approx(1.5, rel=1e-13)
        assert s[6] == pytest.approx(2.5, rel=1e-13)


@pytest.mark.parametrize("order", [2, 8])
def test_dissipation_enstrophy_divergence_identity(order):
    """For any periodic field and any central stencil D (antisymmetric,
    commuting): <|curl u|^2> = <|Du|^2> - <(div u)^2> and
    (1/2)<|Du + Du^T|^2> = <|Du|^2> + <(div u)^2>, so
    epsilon - 2 nu Omega = 2 nu <(div u)^2> exactly (up to rounding)."""
    rng = np.random.default_rng(5)
    u = rng.standard_normal((3, 10, 12, 14))
    nu = 0.003
    s = st.statistics(u, nu, order)
    assert s["epsilon"] - 2 * nu * s["omega"] == pytest.approx(2 * nu * s["div2"], rel=1e-12)
    assert s["div2"] > 0.1


@pytest.mark.parametrize("order", [2, 8])
def test_taylor_green_closed_form(order):
    """u = U (sin x cos y cos z, -cos x sin y cos z, 0) on x_j = 2 pi j/N:
    every derivative multiplies a mode by the stencil symbol
    sigma = 2 sum_m c_m sin(m 2pi/N), the field stays divergence-free on the
    grid, Omega = (3/8) U^2 sigma^2 and epsilon = 2 nu Omega."""
    n, U, nu = 20, 0.05, 0.002
    u = inputs.taylor_green(n, U)
    s = st.statistics(u, nu, order)
    sigma = 2 * sum(c * np.sin(m * 2 * np.pi / n) for m, c in enumerate(st.FD_WEIGHTS[order], 1))
    assert s["omega"] == pytest.approx(3.0 / 8.0 * U * U * sigma * sigma, rel=1e-12)
    assert s["div2"] < 1e-30
    assert s["epsilon"] == pytest.approx(2 * nu * s["omega"], rel=1e-12)
    assert s["k"] == pytest.approx(U * U / 8, rel=1e-13)


def test_second_order_enstrophy_matches_the_lattice_diagnostic():
    """The oracle's lattice enstrophy (C, FD2) equals the numpy statistics
    with the second-order stencil."""
    u = inputs.hit(16, 2.0, 0.04, seed=9)
    assert st.statistics(u, 1e-3, 2)["omega"] == pytest.approx(o.enstrophy(u), rel=1e-13)


def test_scales_reproduce_the_papers_table():
    """From the printed k and epsilon of the resolved run (N = 600, nu =
    0.005) the derived turbulence, Taylor and Kolmogorov scales reproduce the
    other printed rows to their printed precision."""
    rows = np.loadtxt(os.path.join(GOLDEN, "paper_table_statistics_D.txt"))
    N, nu = 600, 0.005
    for r in rows:
        k = r[1] * 1e-4
        eps = r[2] * 1e-5 / N
        sc = st.scales(k, eps, nu)
        got = [sc["l0"] / N * 10, sc["u0"] * 100, sc["tau0"] / N, sc["Re0"],
               sc["lambda"] / N * 100, sc["u_lambda"] * 100, sc["tau_lambda"] / N,
               sc["Re_lambda"], sc["eta"] / N * 1e3, sc["u_eta"] * 1e3, sc["tau_eta"] / N * 10]
        for g, want in zip(got, r[3:]):
            assert g == pytest.approx(want, rel=2.5e-3), (r[0], got, r[3:])


def test_scale_identities():
    """Re_lambda^2 = (20/3) Re_0 and eta / l_0 = Re_0^(-3/4)."""
    sc = st.scales(7.1e-4, 3.3e-8, 2e-3)
    assert sc["Re_lambda"] ** 2 == pytest.approx(20.0 / 3.0 * sc["Re0"], rel=1e-13)
    assert sc["eta"] / sc["l0"] == pytest.approx(sc["Re0"] ** -0.75, rel=1e-13)


def test_correlation_of_a_single_mode():
    n = 32
    u = np.zeros((3, 3, 5, n))
    x = np.arange(n)
    u[0] = np.sin(2 * np.pi * x / n)[None, None, :]
    u[1] = np.sin(2 * np.pi * np.arange(3) / 3)[:, None, None] * np.ones((1, 5, n))
    r11, r22 = st.correlation_x(u, n // 2)
    assert np.abs(r11 - np.cos(2 * np.pi * np.arange(n // 2 + 1) / n)).max() < 1e-14
    assert np.abs(r22 - 1.0).max() < 1e-14


def test_gamma_statistics_of_an_equilibrium_field():
    """At equilibrium <dh|dh> = 0, so every node takes the fallback gamma = 2."""
    F = o.init_feq(inputs.taylor_green(8, 0.05))
    _, g = o.collide_field(F, o.beta_from_nu(1e-3), want_gamma=True)
    s = st.gamma_statistics(g)
    assert s["mean"] == 2.0 and s["std"] == 0.0
