"""Pins of the oracle's central-moment KBC variants (section IV, the four
models s = d~, d~+t~, d~+q~, d~+t~+q~; appendix, Eqs. cm1-cm23 and
cmf000-cmfxyz).

The oracle computes central moments from their definition (section III) and
the parts from the exact inverse of the central-moment map.  These tests hold
it against the paper's printed formulas, written out here independently:
the natural-to-central mapping (Eqs. cm1-cm23) and the population
representation in the central basis for the rest, face, edge and corner
classes (Eqs. cmf000, cmfx00, cmfxy0, cmfxyz), term group by term group.
Other pins: closed-form equilibrium central moments, the natural parts at
u = 0, conservation, the LBGK and regularised special cases, and lattice
behaviour.
"""
import itertools

import numpy as np
import pytest

import oracle as o
from paper_1507_02518_amd import inputs

CENTRAL = [o.S_CD, o.S_CDT, o.S_CDQ, o.S_CDTQ]


def _idx(p, q, r):
    return p + 3 * q + 9 * r


def _node(seed, amp=0.02, u=(0.07, -0.04, 0.05), rho=1.03):
    rng = np.random.default_rng(seed)
    return o.feq(rho, np.array(u)) * (1.0 + amp * rng.standard_normal(27))


# ---------------------------------------------------------------- mapping ----

def _paper_central_from_natural(M):
    """Eqs. cm1-cm23: central named moments from natural ones (section III
    names, third order read as Q_xyy = M_120, Q_yzz = M_012)."""
    m = lambda p, q, r: M[_idx(p, q, r)]  # noqa: E731
    ux, uy, uz = m(1, 0, 0), m(0, 1, 0), m(0, 0, 1)
    T = m(2, 0, 0) + m(0, 2, 0) + m(0, 0, 2)
    Nxz, Nyz = m(2, 0, 0) - m(0, 0, 2), m(0, 2, 0) - m(0, 0, 2)
    Pxy, Pxz, Pyz = m(1, 1, 0), m(1, 0, 1), m(0, 1, 1)
    Qxyy, Qxzz, Qxxy, Qyzz = m(1, 2, 0), m(1, 0, 2), m(2, 1, 0), m(0, 1, 2)
    Qxxz, Qyyz, Qxyz = m(2, 0, 1), m(0, 2, 1), m(1, 1, 1)
    c = {}
    c["Pxy"] = Pxy - ux * uy
    c["Pxz"] = Pxz - ux * uz
    c["Pyz"] = Pyz - uy * uz
    c["Nxz"] = Nxz - ux ** 2 + uz ** 2
    c["Nyz"] = Nyz - uy ** 2 + uz ** 2
    c["T"] = T - (ux ** 2 + uy ** 2 + uz ** 2)
    P_xy, P_xz, P_yz, N_xz, N_yz, Tt = (c[k] for k in ("Pxy", "Pxz", "Pyz", "Nxz", "Nyz", "T"))
    c["Qxyz"] = Qxyz - ux * P_yz - uy * P_xz - uz * P_xy - ux * uy * uz
    c["Qxyy"] = Qxyy - (6 * uy * P_xy + ux * (3 * uy ** 2 + 2 * N_yz - N_xz + Tt)) / 3
    c["Qxzz"] = Qxzz - (6 * uz * P_xz + ux * (3 * uz ** 2 - N_xz - N_yz + Tt)) / 3
    c["Qxxy"] = Qxxy - (6 * ux * P_xy + uy * (3 * ux ** 2 + 2 * N_xz - N_yz + Tt)) / 3
    c["Qyzz"] = Qyzz - (6 * uz * P_yz + uy * (3 * uz ** 2 - N_xz - N_yz + Tt)) / 3
    c["Qxxz"] = Qxxz - (6 * ux * P_xz + uz * (3 * ux ** 2 + 2 * N_xz - N_yz + Tt)) / 3
    c["Qyyz"] = Qyyz - (6 * uy * P_yz + uz * (3 * uy ** 2 + 2 * N_yz - N_xz + Tt)) / 3
    Q = c
    x2, y2, z2 = ux ** 2, uy ** 2, uz ** 2
    c["M022"] = m(0, 2, 2) - (y2 * z2 + 4 * uy * uz * P_yz + (y2 + z2) * Tt / 3
                              - (y2 + z2) * N_xz / 3 + (-y2 + 2 * z2) * N_yz / 3
                              + 2 * uy * Q["Qyzz"] + 2 * uz * Q["Qyyz"])
    c["M202"] = m(2, 0, 2) - (x2 * z2 + 4 * ux * uz * P_xz + (x2 + z2) * Tt / 3
                              + (-x2 + 2 * z2) * N_xz / 3 - (x2 + z2) * N_yz / 3
                              + 2 * ux * Q["Qxzz"] + 2 * uz * Q["Qxxz"])
    c["M220"] = m(2, 2, 0) - (x2 * y2 + 4 * ux * uy * P_xy + (x2 + y2) * Tt / 3
                              + (-x2 + 2 * y2) * N_xz / 3 + (2 * x2 - y2) * N_yz / 3
                              + 2 * ux * Q["Qxyy"] + 2 * uy * Q["Qxxy"])
    c["M211"] = m(2, 1, 1) - (x2 * uy * uz + 2 * ux * uz * P_xy + 2 * ux * uy * P_xz
                              + x2 * P_yz + uy * uz * Tt / 3 + 2 * uy * uz * N_xz / 3
                              - uy * uz * N_yz / 3 + 2 * ux * Q["Qxyz"] + uz * Q["Qxxy"]
                              + uy * Q["Qxxz"])
    c["M121"] = m(1, 2, 1) - (ux * y2 * uz + 2 * uy * uz * P_xy + y2 * P_xz
                              + 2 * ux * uy * P_yz + ux * uz * Tt / 3 - ux * uz * N_xz / 3
                              + 2 * ux * uz * N_yz / 3 + 2 * uy * Q["Qxyz"] + uz * Q["Qxyy"]
                              + ux * Q["Qyyz"])
    c["M112"] = m(1, 1, 2) - (ux * uy * z2 + z2 * P_xy + 2 * uy * uz * P_xz
                              + 2 * ux * uz * P_yz + ux * uy * Tt / 3 - ux * uy * N_xz / 3
                              - ux * uy * N_yz / 3 + 2 * uz * Q["Qxyz"] + uy * Q["Qxzz"]
                              + ux * Q["Qyzz"])
    c["M122"] = m(1, 2, 2) - (ux * y2 * z2 + 2 * uy * z2 * P_xy + 2 * y2 * uz * P_xz
                              + 4 * ux * uy * uz * P_yz + (ux * y2 + ux * z2) * Tt / 3
                              + (-ux * y2 - ux * z2) * N_xz / 3 + (-ux * y2 + 2 * ux * z2) * N_yz / 3
                              + 4 * uy * uz * Q["Qxyz"] + z2 * Q["Qxyy"] + y2 * Q["Qxzz"]
                              + 2 * ux * uy * Q["Qyzz"] + 2 * ux * uz * Q["Qyyz"]
                              + 2 * uy * c["M112"] + 2 * uz * c["M121"] + ux * c["M022"])
    c["M212"] = m(2, 1, 2) - (x2 * uy * z2 + 2 * ux * z2 * P_xy + 4 * ux * uy * uz * P_xz
                              + 2 * x2 * uz * P_yz + (x2 * uy + uy * z2) * Tt / 3
                              + (-x2 * uy + 2 * uy * z2) * N_xz / 3 + (-x2 * uy - uy * z2) * N_yz / 3
                              + 4 * ux * uz * Q["Qxyz"] + 2 * ux * uy * Q["Qxzz"] + z2 * Q["Qxxy"]
                              + x2 * Q["Qyzz"] + 2 * uy * uz * Q["Qxxz"]
                              + 2 * uz * c["M211"] + 2 * ux * c["M112"] + uy * c["M202"])
    c["M221"] = m(2, 2, 1) - (x2 * y2 * uz + 4 * ux * uy * uz * P_xy + 2 * ux * y2 * P_xz
                              + 2 * x2 * uy * P_yz + (x2 * uz + y2 * uz) * Tt / 3
                              + (-x2 * uz + 2 * y2 * uz) * N_xz / 3 + (2 * x2 * uz - y2 * uz) * N_yz / 3
                              + 4 * ux * uy * Q["Qxyz"] + 2 * ux * uz * Q["Qxyy"]
                              + 2 * uy * uz * Q["Qxxy"] + y2 * Q["Qxxz"] + x2 * Q["Qyyz"]
                              + 2 * uy * c["M211"] + 2 * ux * c["M121"] + uz * c["M220"])
    c["M222"] = m(2, 2, 2) - (x2 * y2 * z2 + 4 * ux * uy * z2 * P_xy + 4 * ux * y2 * uz * P_xz
                              + 4 * x2 * uy * uz * P_yz + (x2 * y2 + x2 * z2 + y2 * z2) * Tt / 3
                              + (-x2 * y2 - x2 * z2 + 2 * y2 * z2) * N_xz / 3
                              + (-x2 * y2 + 2 * x2 * z2 - y2 * z2) * N_yz / 3
                              + 8 * ux * uy * uz * Q["Qxyz"] + 2 * ux * z2 * Q["Qxyy"]
                              + 2 * ux * y2 * Q["Qxzz"] + 2 * uy * z2 * Q["Qxxy"]
                              + 2 * x2 * uy * Q["Qyzz"] + 2 * y2 * uz * Q["Qxxz"]
                              + 2 * x2 * uz * Q["Qyyz"] + x2 * c["M022"] + y2 * c["M202"]
                              + z2 * c["M220"] + 4 * uy * uz * c["M211"] + 4 * ux * uz * c["M121"]
                              + 4 * ux * uy * c["M112"] + 2 * ux * c["M122"] + 2 * uy * c["M212"]
                              + 2 * uz * c["M221"])
    return c


def _named_central(Mt):
    """The appendix's names for the oracle's central moments Mt[p + 3q + 9r]."""
    m = lambda p, q, r: Mt[_idx(p, q, r)]  # noqa: E731
    return {
        "Pxy": m(1, 1, 0), "Pxz": m(1, 0, 1), "Pyz": m(0, 1, 1),
        "Nxz": m(2, 0, 0) - m(0, 0, 2), "Nyz": m(0, 2, 0) - m(0, 0, 2),
        "T": m(2, 0, 0) + m(0, 2, 0) + m(0, 0, 2),
        "Qxyz": m(1, 1, 1), "Qxyy": m(1, 2, 0), "Qxzz": m(1, 0, 2), "Qxxy": m(2, 1, 0),
        "Qyzz": m(0, 1, 2), "Qxxz": m(2, 0, 1), "Qyyz": m(0, 2, 1),
        "M022": m(0, 2, 2), "M202": m(2, 0, 2), "M220": m(2, 2, 0), "M211": m(2, 1, 1),
        "M121": m(1, 2, 1), "M112": m(1, 1, 2), "M122": m(1, 2, 2), "M212": m(2, 1, 2),
        "M221": m(2, 2, 1), "M222": m(2, 2, 2),
    }


@pytest.mark.parametrize("seed", range(6))
def test_central_moments_follow_the_papers_mapping(seed):
    """Oracle central moments (direct sums) equal Eqs. cm1-cm23 applied to
    the natural moments, and the first-order central moments vanish."""
    F = _node(seed, u=np.random.default_rng(100 + seed).uniform(-0.2, 0.2, 3))
    _, M = o.natural_moments(F)
    rho, u, Mt = o.central_moments(F)
    assert np.allclose(u, [M[1], M[3], M[9]], atol=0, rtol=1e-14)
    assert Mt[_idx(0, 0, 0)] == pytest.approx(1.0, abs=1e-15)
    for p, q, r in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        assert abs(Mt[_idx(p, q, r)]) < 1e-16
    paper = _paper_central_from_natural(M)
    ours = _named_central(Mt)
    for k, v in paper.items():
        assert ours[k] == pytest.approx(v, abs=2e-15), k


def test_equilibrium_central_moments_factorise():
    """Central moments of the product-form equilibrium: Mt_pqr = m_p m_q m_r
    with m_0 = 1, m_1 = 0, m_2 = (2 sqrt(1 + 3u^2) - 1)/3 - u^2 per axis."""
    for u in ([0.0, 0.0, 0.0], [0.1, -0.05, 0.03], [0.3, 0.2, -0.25]):
        u = np.array(u)
        _, uu, Mt = o.central_moments(o.feq(0.9, u))
        m = [np.array([1.0, 0.0, (2 * np.sqrt(1 + 3 * a * a) - 1) / 3 - a * a]) for a in u]
        for p, q, r in itertools.product(range(3), repeat=3):
            assert Mt[_idx(p, q, r)] == pytest.approx(m[0][p] * m[1][q] * m[2][r], abs=3e-16)


# --------------------------------------------------- representation ----

def _group(name):
    if name == "1":
        return "k"
    if name[0] in "PN":
        return "d"
    if name == "T":
        return "t"
    if name[0] == "Q":
        return "q"
    return "h"


def _cmf000(ux, uy, uz, s, l, d):
    """Eq. cmf000 (rest population), coefficient of each term / rho."""
    return 1.0, {
        "1": -(ux ** 2 - 1) * (uy ** 2 - 1) * (uz ** 2 - 1),
        "Pxy": -4 * ux * uy * (uz ** 2 - 1), "Pxz": -4 * ux * uz * (uy ** 2 - 1),
        "Pyz": -4 * uy * uz * (ux ** 2 - 1),
        "Nxz": (ux ** 2 * (uy ** 2 + uz ** 2 - 2) + uz ** 2 * (1 - 2 * uy ** 2) + uy ** 2) / 3,
        "Nyz": (uy ** 2 * (ux ** 2 + uz ** 2 - 2) + uz ** 2 * (1 - 2 * ux ** 2) + ux ** 2) / 3,
        "T": -(ux ** 2 * uy ** 2 + ux ** 2 * uz ** 2 + uy ** 2 * uz ** 2
               - 2 * (ux ** 2 + uy ** 2 + uz ** 2) + 3) / 3,
        "Qxyz": -8 * ux * uy * uz,
        "Qxyy": -2 * ux * (uz ** 2 - 1), "Qxzz": -2 * ux * (uy ** 2 - 1),
        "Qxxy": -2 * uy * (uz ** 2 - 1), "Qyzz": -2 * uy * (ux ** 2 - 1),
        "Qxxz": -2 * uz * (uy ** 2 - 1), "Qyyz": -2 * uz * (ux ** 2 - 1),
        "M022": 1 - ux ** 2, "M202": 1 - uy ** 2, "M220": 1 - uz ** 2,
        "M211": -4 * uy * uz, "M121": -4 * ux * uz, "M112": -4 * ux * uy,
        "M122": -2 * ux, "M212": -2 * uy, "M221": -2 * uz, "M222": -1.0,
    }


def _cmfx00(ux, uy, uz, s, l, d):
    """Eq. cmfx00 (population (sigma, 0, 0))."""
    a = s + ux          # sigma + u_x
    b = s + 2 * ux      # sigma + 2 u_x
    return 1.0 / 6.0, {
        "1": 3 * ux * (uy ** 2 - 1) * (uz ** 2 - 1) * a,
        "Pxy": 6 * uy * (uz ** 2 - 1) * b, "Pxz": 6 * uz * (uy ** 2 - 1) * b,
        "Pyz": 12 * ux * uy * uz * a,
        "Nxz": -(s * ux * (uy ** 2 + uz ** 2 - 2) + ux ** 2 * (uy ** 2 + uz ** 2 - 2)
                 - 2 * (uy ** 2 - 1) * (uz ** 2 - 1)),
        "Nyz": (uz ** 2 * (2 * ux * a - uy ** 2) - ux * (uy ** 2 + 1) * a + uy ** 2 + uz ** 2 - 1),
        "T": (uz ** 2 * (ux * a + uy ** 2) + ux * (uy ** 2 - 2) * a - uy ** 2 - uz ** 2 + 1),
        "Qxyz": 12 * uy * uz * b,
        "Qxyy": 3 * (uz ** 2 - 1) * b, "Qxzz": 3 * (uy ** 2 - 1) * b,
        "Qxxy": 6 * uy * (uz ** 2 - 1), "Qyzz": 6 * ux * uy * a,
        "Qxxz": 6 * uz * (uy ** 2 - 1), "Qyyz": 6 * ux * uz * a,
        "M022": 3 * ux * a, "M202": 3 * (uy ** 2 - 1), "M220": 3 * (uz ** 2 - 1),
        "M211": 12 * uy * uz, "M121": 6 * uz * b, "M112": 6 * uy * b,
        "M122": 3 * b, "M212": 6 * uy, "M221": 6 * uz, "M222": 3.0,
    }


def _cmfxy0(ux, uy, uz, s, l, d, printed=False):
    """Eq. cmfxy0 (population (sigma, lambda, 0)).

    The Pi~_yz term is printed as -u_x u_z (lambda + 2u_y)(sigma + u_x); the
    representation is the inverse of the central map only with a factor 2,
    -2 u_x u_z (lambda + 2u_y)(sigma + u_x), which is also the x<->y mirror of
    the equation's own Pi~_xz term and the y<->z mirror of the Pi~_yz term of
    Eq. cmfx0z.  printed=True keeps the printed coefficient."""
    a, b = s + ux, s + 2 * ux
    c, e = l + uy, l + 2 * uy
    z1 = uz ** 2 - 1
    return 1.0 / 4.0, {
        "1": -ux * uy * z1 * c * a,
        "Pxy": -z1 * e * b, "Pxz": -2 * uy * uz * c * b,
        "Pyz": (-1 if printed else -2) * ux * uz * e * a,
        "Nxz": (s * ux * (uy * c + uz ** 2 - 1) + ux ** 2 * (uy * c + uz ** 2 - 1)
                - 2 * uy * z1 * c) / 3,
        "Nyz": (s * ux * (uy * c - 2 * uz ** 2 + 2) + ux ** 2 * (uy * c - 2 * uz ** 2 + 2)
                + uy * z1 * c) / 3,
        "T": (-s * ux * (uy * c + uz ** 2 - 1) - ux ** 2 * (uy * c + uz ** 2 - 1)
              - uy * z1 * c) / 3,
        "Qxyz": -2 * uz * e * b,
        "Qxyy": -z1 * b, "Qxzz": -uy * c * b,
        "Qxxy": -z1 * e, "Qyzz": -ux * e * a,
        "Qxxz": -2 * uy * uz * c, "Qyyz": -2 * ux * uz * a,
        "M022": -ux * a, "M202": -uy * c, "M220": 1 - uz ** 2,
        "M211": -2 * uz * e, "M121": -2 * uz * b, "M112": -e * b,
        "M122": -b, "M212": -e, "M221": -2 * uz, "M222": -1.0,
    }


def _cmfxyz(ux, uy, uz, s, l, d):
    """Eq. cmfxyz (population (sigma, lambda, delta))."""
    a, b = s + ux, s + 2 * ux
    c, e = l + uy, l + 2 * uy
    g, h = d + uz, d + 2 * uz
    X, Y = ux * a, uy * c
    return 1.0 / 8.0, {
        "1": ux * uy * uz * g * c * a,
        "Pxy": uz * g * e * b, "Pxz": uy * h * c * b, "Pyz": ux * h * e * a,
        "Nxz": (-d * uz * (X - 2 * Y) - uz ** 2 * (X - 2 * Y) - ux * uy * c * a) / 3,
        "Nyz": (d * uz * (2 * X - Y) + uz ** 2 * (2 * X - Y) - ux * uy * c * a) / 3,
        "T": (d * uz * (Y + X) + uz ** 2 * (Y + X) + ux * uy * c * a) / 3,
        "Qxyz": h * e * b,
        "Qxyy": uz * g * b, "Qxzz": uy * c * b,
        "Qxxy": uz * g * e, "Qyzz": ux * e * a,
        "Qxxz": uy * h * c, "Qyyz": ux * h * a,
        "M022": ux * a, "M202": uy * c, "M220": uz * g,
        "M211": h * e, "M121": h * b, "M112": e * b,
        "M122": b, "M212": e, "M221": h, "M222": 1.0,
    }


def _classes():
    out = [(_cmf000, (0, 0, 0))]
    out += [(_cmfx00, (s, 0, 0)) for s in (-1, 1)]
    out += [(_cmfxy0, (s, l, 0)) for s in (-1, 1) for l in (-1, 1)]
    out += [(_cmfxyz, sgn) for sgn in itertools.product((-1, 1), repeat=3)]
    return out


@pytest.mark.parametrize("seed", range(4))
def test_central_parts_match_the_printed_representation(seed):
    """The oracle's k~, d~, t~, q~ and h~ = f - k~ - d~ - t~ - q~ equal, for
    the rest, face, edge and corner populations of every sign, the matching
    term groups of Eqs. cmf000, cmfx00, cmfxy0 and cmfxyz."""
    rng = np.random.default_rng(seed)
    F = _node(seed, amp=0.03, u=rng.uniform(-0.25, 0.25, 3))
    rho, u, Mt = o.central_moments(F)
    k, d, t, q = o.central_parts(rho, u, Mt)
    ours = {"k": k, "d": d, "t": t, "q": q, "h": F - k - d - t - q}
    named = _named_central(Mt)
    named["1"] = 1.0
    for fn, (s, l, dd) in _classes():
        i = (s + 1) + 3 * (l + 1) + 9 * (dd + 1)
        pref, coef = fn(u[0], u[1], u[2], s, l, dd)
        groups = {"k": 0.0, "d": 0.0, "t": 0.0, "q": 0.0, "h": 0.0}
        for name, cval in coef.items():
            groups[_group(name)] += rho * pref * cval * named[name]
        for gname, val in groups.items():
            assert ours[gname][i] == pytest.approx(val, abs=3e-15), (fn.__name__, s, l, dd, gname)
        assert sum(groups.values()) == pytest.approx(F[i], abs=3e-15)


def test_printed_cmfxy0_pi_yz_term_breaks_the_round_trip():
    """The coefficient of Pi~_yz as printed in Eq. cmfxy0 does not rebuild
    f_(sigma, lambda, 0) from its own central moments; with the factor 2 the
    printed equation does (the reading the oracle follows)."""
    F = _node(2, amp=0.03, u=(0.13, -0.21, 0.17))
    rho, u, Mt = o.central_moments(F)
    named = _named_central(Mt)
    named["1"] = 1.0
    for s, l in ((-1, 1), (1, 1)):
        i = (s + 1) + 3 * (l + 1) + 9
        for printed, ok in ((True, False), (False, True)):
            pref, coef = _cmfxy0(u[0], u[1], u[2], s, l, 0, printed=printed)
            val = sum(rho * pref * cv * named[n] for n, cv in coef.items())
            assert (abs(val - F[i]) < 1e-14) == ok


def test_central_columns_invert_the_moment_map():
    """Brute force: the central moments of column m of the representation
    (computed here by direct sums about the same u) are the unit vector e_m."""
    V = o.velocities()
    u = np.array([0.11, -0.07, 0.19])
    for m in range(27):
        col = o.central_column(u, m)
        mom = np.zeros(27)
        for p, q, r in itertools.product(range(3), repeat=3):
            mom[_idx(p, q, r)] = np.sum(col * (V[:, 0] - u[0]) ** p * (V[:, 1] - u[1]) ** q
                                        * (V[:, 2] - u[2]) ** r)
        e = np.zeros(27)
        e[m] = 1.0
        assert np.abs(mom - e).max() < 1e-14, m


def test_central_parts_reduce_to_natural_parts_at_rest():
    """At u = 0 central and natural moments coincide, so d~, t~, q~ equal the
    table-s_parts d, t, q (an independent implementation in the oracle)."""
    G = _node(7, amp=0.05, u=(0.0, 0.0, 0.0))
    F = 0.5 * (G + G[::-1])          # opposite pairs averaged: zero momentum
    rho, u, Mt = o.central_moments(F)
    assert np.abs(u).max() < 1e-16
    kc, dc, tc, qc = o.central_parts(rho, u, Mt)
    rho_n, M = o.natural_moments(F)
    kn, dn, tn, qn = o.parts(rho_n, M)
    for a, b in ((kc, kn), (dc, dn), (tc, tn), (qc, qn)):
        assert np.abs(a - b).max() < 1e-16


def test_central_parts_carry_only_their_moments():
    """Each part's central moments about the node's u are the ones it names:
    k~ only order 0, d~ the deviatoric second order, t~ the trace, q~ the
    third order (brute-force sums)."""
    V = o.velocities()
    F = _node(11, amp=0.04, u=(0.12, 0.09, -0.15))
    rho, u, Mt = o.central_moments(F)
    k, d, t, q = o.central_parts(rho, u, Mt)

    def cm(g):
        out = np.zeros(27)
        for p, q_, r in itertools.product(range(3), repeat=3):
            out[_idx(p, q_, r)] = np.sum(g * (V[:, 0] - u[0]) ** p * (V[:, 1] - u[1]) ** q_
                                         * (V[:, 2] - u[2]) ** r) / rho
        return out

    want = {
        "k": {_idx(0, 0, 0): 1.0},
        "d": {_idx(1, 1, 0): Mt[_idx(1, 1, 0)], _idx(1, 0, 1): Mt[_idx(1, 0, 1)],
              _idx(0, 1, 1): Mt[_idx(0, 1, 1)]},
        "t": {},
        "q": {m: Mt[m] for m in (_idx(1, 2, 0), _idx(1, 0, 2), _idx(2, 1, 0), _idx(0, 1, 2),
                                 _idx(2, 0, 1), _idx(0, 2, 1), _idx(1, 1, 1))},
    }
    tr = (Mt[_idx(2, 0, 0)] + Mt[_idx(0, 2, 0)] + Mt[_idx(0, 0, 2)]) / 3
    for a in range(3):
        m = _idx(2, 0, 0) if a == 0 else (_idx(0, 2, 0) if a == 1 else _idx(0, 0, 2))
        want["d"][m] = Mt[m] - tr
        want["t"][m] = tr
    for name, g in (("k", k), ("d", d), ("t", t), ("q", q)):
        got = cm(g)
        exp = np.zeros(27)
        for m, v in want[name].items():
            exp[m] = v
        assert np.abs(got - exp).max() < 2e-15, name


# ---------------------------------------------------------- collision ----

@pytest.mark.parametrize("variant", CENTRAL)
def test_central_ds_dh_carry_no_mass_or_momentum(variant):
    V = o.velocities()
    F = _node(3, amp=0.03, u=(0.1, -0.08, 0.06))
    r = o.collide(F, o.beta_from_nu(1e-3), variant)
    for part in ("ds", "dh"):
        assert abs(r[part].sum()) < 1e-15
        assert np.abs(V.T @ r[part]).max() < 1e-15
    assert abs(r["P"].sum() - F.sum()) < 4e-16


@pytest.mark.parametrize("variant", CENTRAL)
def test_central_gamma2_is_lbgk(variant):
    F = _node(4, amp=0.03)
    beta = o.beta_from_nu(2e-3)
    r = o.collide(F, beta, variant, gamma=2.0)
    assert np.abs(r["P"] - (F + 2 * beta * (r["feq"] - F))).max() < 1e-16


def test_central_regularised_special_case():
    """s = d~+t~ with gamma = 1/beta: f' - f^eq = (1 - 2 beta) ds~, so its
    central moments above second order vanish and the second-order ones are
    (1 - 2 beta) times those of f - f^eq."""
    V = o.velocities()
    F = _node(5, amp=0.03, u=(0.09, 0.05, -0.07))
    beta = o.beta_from_nu(5e-3)
    r = o.collide(F, beta, o.S_CDT, gamma=1.0 / beta)
    rho, u, _ = o.central_moments(F)
    neq_post = r["P"] - r["feq"]
    neq_pre = F - r["feq"]
    for p, q, rr in itertools.product(range(3), repeat=3):
        w = (V[:, 0] - u[0]) ** p * (V[:, 1] - u[1]) ** q * (V[:, 2] - u[2]) ** rr
        post, pre = np.sum(neq_post * w), np.sum(neq_pre * w)
        if p + q + rr == 2:
            assert post == pytest.approx((1 - 2 * beta) * pre, abs=1e-15)
        else:
            assert abs(post) < 1e-15


@pytest.mark.parametrize("variant", CENTRAL)
def test_central_entropic_gamma_is_quadratic_optimum(variant):
    """<f' - f^eq | dh> = 0 at gamma* (the maximum of the quadratic entropy),
    in the central basis as in the natural one."""
    F = _node(6, amp=0.03)
    r = o.collide(F, o.beta_from_nu(1e-4), variant)
    ip = np.sum((r["P"] - r["feq"]) * r["dh"] / r["feq"])
    scale = np.sum(r["dh"] ** 2 / r["feq"])
    assert abs(ip) < 1e-12 * scale


def test_central_equilibrium_is_a_fixed_point():
    for variant in CENTRAL:
        fe = o.feq(1.01, np.array([0.1, -0.2, 0.05]))
        r = o.collide(fe, 0.99, variant)
        assert np.abs(r["P"] - fe).max() < 3e-16


# ----------------------------------------------------------- lattice ----

def test_central_lattice_conserves_mass_and_momentum():
    u = inputs.hit(12, 2.0, 0.05, seed=4)
    F = o.init_feq(u)
    V = o.velocities()
    m0, j0 = F.sum(), np.tensordot(V.T, F, axes=(1, 0)).sum(axis=(1, 2, 3))
    F = o.run(F, o.beta_from_nu(1e-3), 20, variant=o.S_CDTQ)
    m1, j1 = F.sum(), np.tensordot(V.T, F, axes=(1, 0)).sum(axis=(1, 2, 3))
    assert abs(m1 / m0 - 1) < 1e-13
    assert np.abs(j1 - j0).max() / m0 < 1e-14
