"""Pins of the oracle's single-node arithmetic against what the paper fixes.

Each test checks the oracle against an independent fact: a closed form, an
invariant the construction guarantees, a special case that reduces to a
textbook scheme, or the defining extremum principle computed here by brute
force.  None of them retypes the oracle's own formula.
"""
import math
import os

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
VARIANTS = [0, 1, 2, 3]


def _vel(orc):
    return orc.velocities().astype(np.float64)


def _mom(v, g, p, q, r):
    """Brute-force natural moment sum_i g_i vx^p vy^q vz^r."""
    return float((g * v[:, 0] ** p * v[:, 1] ** q * v[:, 2] ** r).sum())


def _random_state(orc, rng, eps=0.05, umax=0.1):
    rho = 1.0 + 0.05 * rng.uniform(-1, 1)
    u = rng.uniform(-umax, umax, size=3)
    f = orc.feq(rho, u) * (1.0 + eps * rng.uniform(-1, 1, size=27))
    return f


# ---------------------------------------------------------------- lattice --

def test_velocity_set_is_tensor_product(orc):
    v = orc.velocities()
    assert len({tuple(x) for x in v}) == 27
    assert set(v.ravel()) == {-1, 0, 1}
    # index convention i = (vx+1) + 3(vy+1) + 9(vz+1); opposite is 26 - i
    for i in range(27):
        assert i == (v[i, 0] + 1) + 3 * (v[i, 1] + 1) + 9 * (v[i, 2] + 1)
        assert (v[26 - i] == -v[i]).all()


def test_weights_match_paper_table(orc):
    # golden: the paper's 1-D weights W_0 = 2/3, W_{+-1} = 1/6 multiplied out
    rows = np.loadtxt(os.path.join(GOLDEN, "weights_d3q27.txt"))
    v = orc.velocities()
    W = orc.weights()
    for nonzero, num, den in rows:
        sel = (v != 0).sum(axis=1) == int(nonzero)
        assert np.all(W[sel] == num / den)
    assert abs(W.sum() - 1.0) < 1e-15


def test_weights_isotropy_and_sound_speed(orc):
    v = _vel(orc)
    W = orc.weights()
    cs2 = 1.0 / 3.0  # c_s = 1/sqrt(3)
    for a in range(3):
        assert abs((W * v[:, a]).sum()) < 1e-16
        for b in range(3):
            want = cs2 if a == b else 0.0
            assert abs((W * v[:, a] * v[:, b]).sum() - want) < 1e-15
    # fourth-order isotropy of the product lattice
    assert abs((W * v[:, 0] ** 4).sum() - 3 * cs2 ** 2) < 1e-15
    assert abs((W * v[:, 0] ** 2 * v[:, 1] ** 2).sum() - cs2 ** 2) < 1e-15


def test_beta_viscosity_relation(orc):
    for nu in [1e-5, 2.5e-4, 1e-3, 0.02, 0.1, 1.0]:
        beta = orc.beta_from_nu(nu)
        assert 0.0 < beta < 1.0
        assert abs((1.0 / 3.0) * (1.0 / (2 * beta) - 0.5) - nu) < 1e-15 * max(1.0, nu) * 10
    assert orc.beta_from_nu(0.001) == pytest.approx(1.0 / 1.006, rel=1e-15)


# ------------------------------------------------------------ equilibrium --

def test_feq_conserves_density_and_momentum(orc):
    rng = np.random.default_rng(1)
    v = _vel(orc)
    for _ in range(200):
        rho = rng.uniform(0.5, 2.0)
        u = rng.uniform(-0.5, 0.5, size=3)
        f = orc.feq(rho, u)
        assert abs(f.sum() - rho) < 4e-16 * rho * 4
        assert np.allclose((v * f[:, None]).sum(0), rho * u, atol=2e-15, rtol=0)


def test_feq_at_rest_is_weights(orc):
    for rho in [1.0, 0.7, 1.3]:
        assert np.array_equal(orc.feq(rho, [0.0, 0.0, 0.0]), rho * orc.weights())


def _entropy_maximizer(W, v, rho, u):
    """Maximize S = -sum f ln(f/W) under sum f = rho, sum v f = rho u.

    Stationarity gives f_i = W_i exp(l0 + l . v_i); the four multipliers are
    found by Newton's method on the constraints.
    """
    lam = np.array([math.log(rho), 0.0, 0.0, 0.0])
    basis = np.concatenate([np.ones((27, 1)), v], axis=1)
    target = np.concatenate([[rho], rho * np.asarray(u)])
    for _ in range(60):
        f = W * np.exp(basis @ lam)
        r = basis.T @ f - target
        J = basis.T @ (f[:, None] * basis)
        lam = lam - np.linalg.solve(J, r)
        if np.abs(r).max() < 1e-17:
            break
    return W * np.exp(basis @ lam)


def test_feq_is_the_entropy_maximizer(orc):
    rng = np.random.default_rng(2)
    W = orc.weights()
    v = _vel(orc)
    for _ in range(50):
        rho = rng.uniform(0.6, 1.5)
        u = rng.uniform(-0.4, 0.4, size=3)
        ref = _entropy_maximizer(W, v, rho, u)
        assert np.allclose(orc.feq(rho, u), ref, rtol=2e-14, atol=0)


def test_feq_matches_polynomial_to_second_order(orc):
    W = orc.weights()
    v = _vel(orc)
    d = np.array([0.6, -0.3, 0.74])
    errs = []
    for a in [0.04, 0.02, 0.01]:
        u = a * d
        uv = v @ u
        uu = u @ u
        poly = W * (1 + 3 * uv + 4.5 * uv ** 2 - 1.5 * uu)
        errs.append(np.abs(orc.feq(1.0, u) - poly).max())
    # third-order remainder: halving u divides the error by ~8
    assert 7.0 < errs[0] / errs[1] < 9.0
    assert 7.0 < errs[1] / errs[2] < 9.0


def test_feq_positive_iff_velocity_below_one(orc):
    assert (orc.feq(1.0, [0.99, -0.99, 0.5]) > 0).all()
    with np.errstate(all="ignore"):
        f = orc.feq(1.0, [1.2, 0.0, 0.0])
    assert not (f > 0).all()


def test_equilibrium_moments_factorize(orc):
    """M^eq_pqr = m_p(u_x) m_q(u_y) m_r(u_z), m_0=1, m_1=u, m_2=(2 sqrt(1+3u^2)-1)/3."""
    rng = np.random.default_rng(3)
    v = _vel(orc)

    def m(p, x):
        return [1.0, x, (2.0 * math.sqrt(1 + 3 * x * x) - 1.0) / 3.0][p]

    for _ in range(20):
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.3, 0.3, size=3)
        f = orc.feq(rho, u)
        for r in range(3):
            for q in range(3):
                for p in range(3):
                    want = rho * m(p, u[0]) * m(q, u[1]) * m(r, u[2])
                    assert abs(_mom(v, f, p, q, r) - want) < 2e-15


# ---------------------------------------------------------------- moments --

def test_natural_moments_definition_on_unit_vectors(orc):
    v = orc.velocities()
    for i in range(27):
        e = np.zeros(27)
        e[i] = 1.0
        rho, M = orc.natural_moments(e)
        assert rho == 1.0
        for r in range(3):
            for q in range(3):
                for p in range(3):
                    assert M[p + 3 * q + 9 * r] == float(v[i, 0] ** p * v[i, 1] ** q * v[i, 2] ** r)


def test_moment_representation_round_trip(orc):
    """Eq. moment_rep inverts Eq. natmoments (pins the third-order names)."""
    rng = np.random.default_rng(4)
    for _ in range(100):
        f = rng.uniform(0.001, 0.5, size=27)
        rho, M = orc.natural_moments(f)
        assert np.allclose(orc.f_from_moments(rho, M), f, rtol=0, atol=5e-15)


# ------------------------------------------------------------------ parts --

def test_parts_carry_the_moments_they_name(orc):
    rng = np.random.default_rng(5)
    v = _vel(orc)
    for _ in range(30):
        f = rng.uniform(0.001, 0.5, size=27)
        rho, M = orc.natural_moments(f)
        k, d, t, q = orc.parts(rho, M)
        mf = lambda p, qq, r: _mom(v, f, p, qq, r)  # noqa: E731
        # k: density and momentum, nothing of order 2 or 3
        assert abs(k.sum() - rho) < 1e-14
        for a in range(3):
            e = [0, 0, 0]
            e[a] = 1
            assert abs(_mom(v, k, *e) - mf(*e)) < 1e-14
        # d: traceless second-order part: normal stress differences and
        # off-diagonal stresses of f
        dm = lambda p, qq, r: _mom(v, d, p, qq, r)  # noqa: E731
        assert abs(d.sum()) < 1e-14
        assert abs(dm(2, 0, 0) + dm(0, 2, 0) + dm(0, 0, 2)) < 1e-14
        assert abs((dm(2, 0, 0) - dm(0, 0, 2)) - (mf(2, 0, 0) - mf(0, 0, 2))) < 1e-14
        assert abs((dm(0, 2, 0) - dm(0, 0, 2)) - (mf(0, 2, 0) - mf(0, 0, 2))) < 1e-14
        for pqr in [(1, 1, 0), (1, 0, 1), (0, 1, 1)]:
            assert abs(dm(*pqr) - mf(*pqr)) < 1e-14
        # t: the trace, with zero mass
        tm = lambda p, qq, r: _mom(v, t, p, qq, r)  # noqa: E731
        assert abs(t.sum()) < 1e-14
        assert abs(tm(2, 0, 0) + tm(0, 2, 0) + tm(0, 0, 2)
                   - (mf(2, 0, 0) + mf(0, 2, 0) + mf(0, 0, 2))) < 1e-14
        # q: the third-order moments
        qm = lambda p, qq, r: _mom(v, q, p, qq, r)  # noqa: E731
        for pqr in [(1, 2, 0), (1, 0, 2), (2, 1, 0), (0, 1, 2), (2, 0, 1), (0, 2, 1), (1, 1, 1)]:
            assert abs(qm(*pqr) - mf(*pqr)) < 1e-14


def _low_moments(v, g):
    out = []
    for r in range(3):
        for q in range(3):
            for p in range(3):
                if p + q + r <= 3:
                    out.append(_mom(v, g, p, q, r))
    return np.array(out)


def test_h_part_of_dtq_has_no_moment_below_fourth_order(orc):
    rng = np.random.default_rng(6)
    v = _vel(orc)
    for _ in range(30):
        f = rng.uniform(0.001, 0.5, size=27)
        rho, M = orc.natural_moments(f)
        k, _, _, _ = orc.parts(rho, M)
        s = orc.s_part(rho, M, 3)
        h = f - k - s
        assert np.abs(_low_moments(v, h)).max() < 2e-14


# -------------------------------------------------------------- collision --

@pytest.mark.parametrize("variant", VARIANTS)
def test_deviations_carry_no_conserved_moments(orc, variant):
    rng = np.random.default_rng(7 + variant)
    v = _vel(orc)
    for _ in range(50):
        F = _random_state(orc, rng)
        c = orc.collide(F, 0.99, variant)
        for g in (c["ds"], c["dh"]):
            assert abs(g.sum()) < 2e-16 * 27
            assert np.abs((v * g[:, None]).sum(0)).max() < 2e-16 * 27
        # mass and momentum conserved by the collision
        assert abs(c["P"].sum() - F.sum()) < 4e-15
        assert np.abs((v * (c["P"] - F)[:, None]).sum(0)).max() < 4e-15


@pytest.mark.parametrize("variant", VARIANTS)
def test_gamma_two_is_lbgk(orc, variant):
    rng = np.random.default_rng(11 + variant)
    for _ in range(50):
        F = _random_state(orc, rng)
        beta = rng.uniform(0.5, 0.9999)
        c = orc.collide(F, beta, variant, gamma=2.0)
        rho = F.sum()
        u = (_vel(orc) * F[:, None]).sum(0) / rho
        lbgk = F + 2.0 * beta * (orc.feq(rho, u) - F)
        assert np.allclose(c["P"], lbgk, rtol=0, atol=1e-15)


def test_gamma_inverse_beta_is_regularized_lb(orc):
    """s = d+t, gamma = 1/beta: only second-order non-equilibrium survives."""
    rng = np.random.default_rng(13)
    v = _vel(orc)
    for _ in range(50):
        F = _random_state(orc, rng)
        beta = rng.uniform(0.5, 0.9999)
        c = orc.collide(F, beta, 1, gamma=1.0 / beta)
        neq = c["P"] - c["feq"]
        for r in range(3):
            for q in range(3):
                for p in range(3):
                    if p + q + r >= 3:
                        assert abs(_mom(v, neq, p, q, r)) < 2e-16 * 64


def test_equilibrium_is_a_fixed_point(orc):
    rng = np.random.default_rng(17)
    for variant in VARIANTS:
        for _ in range(20):
            f = orc.feq(rng.uniform(0.8, 1.2), rng.uniform(-0.2, 0.2, size=3))
            c = orc.collide(f, 0.999, variant)
            assert c["gamma"] == 2.0          # <dh|dh> at roundoff level
            assert np.allclose(c["P"], f, rtol=0, atol=6e-16)


def _esp(feq, X, Y):
    return float((X * Y / feq).sum())


@pytest.mark.parametrize("variant", VARIANTS)
def test_entropic_scalar_product_and_gamma_optimality(orc, variant):
    """gamma* maximises the quadratic entropy: <f' - f^eq | dh> = 0."""
    rng = np.random.default_rng(19 + variant)
    for _ in range(50):
        F = _random_state(orc, rng)
        beta = rng.uniform(0.9, 0.9999)
        c = orc.collide(F, beta, variant)
        fe, ds, dh, P = c["feq"], c["ds"], c["dh"], c["P"]
        assert _esp(fe, ds, dh) == pytest.approx(_esp(fe, dh, ds), rel=1e-13)
        assert _esp(fe, dh, dh) > 0
        n1 = math.sqrt(_esp(fe, P - fe, P - fe))
        n2 = math.sqrt(_esp(fe, dh, dh))
        assert abs(_esp(fe, P - fe, dh)) <= 1e-11 * n1 * n2
        # the printed estimate itself
        g = 1 / beta - (2 - 1 / beta) * _esp(fe, ds, dh) / _esp(fe, dh, dh)
        assert c["gamma"] == pytest.approx(g, rel=1e-11, abs=1e-11)


def _entropy_gain(W, fe, fp):
    """S[f'] - S[f^eq] with S[f] = -sum f ln(f/W), written for accuracy."""
    x = (fp - fe) / fe
    return -float(((fp - fe) * np.log(fe / W) + fp * np.log1p(x)).sum())


def test_gamma_estimate_converges_to_entropy_maximum(orc):
    """gamma* is the first-order estimate of the entropy-maximising gamma."""
    W = orc.weights()
    rng = np.random.default_rng(23)
    beta = 0.995
    base = orc.feq(1.0, [0.05, -0.03, 0.02])
    shape = rng.uniform(-1, 1, size=27)
    errs = []
    for eps in [1e-1, 1e-2, 1e-3]:
        F = base * (1 + eps * shape)
        c = orc.collide(F, beta, 3)
        fe, ds, dh = c["feq"], c["ds"], c["dh"]

        def neg_gain(g):
            fp = F - beta * (2 * ds + g * dh)
            if (fp <= 0).any():
                return 1e300
            return -_entropy_gain(W, fe, fp)

        gstar = c["gamma"]
        res = minimize_scalar(neg_gain, bracket=(gstar - 0.5, gstar, gstar + 0.5),
                              tol=1e-14)
        gmax = res.x
        gex = orc.gamma_exact(fe, ds, dh, beta)
        assert abs(gex - gmax) < 1e-5 * max(1.0, abs(gmax))
        errs.append(abs(gstar - gex))
    # |gamma* - gamma_exact| shrinks linearly with the non-equilibrium amplitude
    assert errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5
