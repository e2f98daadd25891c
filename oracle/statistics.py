"""Flow statistics of section V, written plainly in numpy (TEST
INFRASTRUCTURE ONLY, like the rest of this package: only the tests, the
smoke check and the CPU leg of the benchmark may use it).

* velocity gradients by central differences, second order or the nine-point
  eighth-order stencil the paper uses for its table of statistics;
* enstrophy Omega = (1/2) <|curl u'|^2>, dissipation
  epsilon = (nu/2) <(d_a u'_b + d_b u'_a)(d_a u'_b + d_b u'_a)>, the moments
  <(du'_x/dx)^n> and the longitudinal skewness factors
  S^n = (-1)^n <(du'_x/dx)^n> / <(du'_x/dx)^2>^(n/2) (section V.A);
* the turbulence, Taylor and Kolmogorov scales built from k, epsilon and nu
  (the caption of the table of statistics);
* longitudinal and transversal velocity correlations along x (section V.B);
* mean and standard deviation of the stabilizer gamma over the nodes
  (section V.C), from the oracle's collision.

Fields are numpy arrays u[3][nz][ny][nx]; the grid spacing is one lattice
unit and every field is periodic.
"""
from __future__ import annotations

import numpy as np

# first-derivative central-difference weights c_m of f(x+m) - f(x-m)
FD_WEIGHTS = {
    2: (0.5,),
    8: (4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0),
}
_AXIS = {0: 2, 1: 1, 2: 0}   # coordinate a -> array axis of [z][y][x]


def derivative(f, a: int, order: int = 8):
    """d f / d x_a by the central stencil of the given order (periodic)."""
    ax = _AXIS[a]
    out = np.zeros_like(f)
    for m, c in enumerate(FD_WEIGHTS[order], start=1):
        out += c * (np.roll(f, -m, axis=ax) - np.roll(f, m, axis=ax))
    return out


def gradient(u, order: int = 8):
    """G[a][b] = d u_a / d x_b."""
    return np.array([[derivative(u[a], b, order) for b in range(3)] for a in range(3)])


def statistics(u, nu: float, order: int = 8) -> dict:
    """k, Omega, epsilon, <(div u)^2>, <(du_x/dx)^n> (n = 2..6) and S^n
    (n = 3..6) of the velocity field u."""
    u = np.asarray(u, dtype=np.float64)
    up = u - u.mean(axis=(1, 2, 3), keepdims=True)
    k = 0.5 * np.mean(np.sum(up * up, axis=0))
    G = gradient(up, order)
    wx = G[2][1] - G[1][2]
    wy = G[0][2] - G[2][0]
    wz = G[1][0] - G[0][1]
    omega = 0.5 * np.mean(wx * wx + wy * wy + wz * wz)
    strain = 0.0
    for a in range(3):
        for b in range(3):
            s = G[a][b] + G[b][a]
            strain = strain + s * s
    eps = 0.5 * nu * np.mean(strain)
    div = G[0][0] + G[1][1] + G[2][2]
    dux = G[0][0]
    mom = {n: float(np.mean(dux ** n)) for n in range(2, 7)}
    skew = {n: (-1) ** n * mom[n] / mom[2] ** (n / 2) for n in range(3, 7)}
    return {"k": float(k), "omega": float(omega), "epsilon": float(eps),
            "div2": float(np.mean(div * div)), "dudx_moments": mom, "skewness": skew}


def scales(k: float, eps: float, nu: float) -> dict:
    """Turbulence, Taylor and Kolmogorov scales from k, epsilon and nu."""
    l0 = k ** 1.5 / eps
    u0 = k ** 0.5
    up = (2.0 * k / 3.0) ** 0.5
    lam = (15.0 * nu * up * up / eps) ** 0.5
    eta = (nu ** 3 / eps) ** 0.25
    u_eta = (nu * eps) ** 0.25
    return {"l0": l0, "u0": u0, "tau0": l0 / u0, "Re0": l0 * u0 / nu,
            "lambda": lam, "u_lambda": up, "tau_lambda": lam / up, "Re_lambda": lam * up / nu,
            "eta": eta, "u_eta": u_eta, "tau_eta": (nu / eps) ** 0.5}


def correlation_x(u, rmax: int):
    """rho11(r) = <u'_x(x) u'_x(x+r)>/<u'_x^2>, rho22(r) likewise for u'_y,
    for r = 0..rmax along x (periodic)."""
    up = u - u.mean(axis=(1, 2, 3), keepdims=True)
    out = np.zeros((2, rmax + 1))
    for c in range(2):
        f = up[c]
        den = np.mean(f * f)
        for r in range(rmax + 1):
            out[c, r] = np.mean(f * np.roll(f, -r, axis=2)) / den
    return out[0], out[1]


def gamma_statistics(gamma_field) -> dict:
    g = np.asarray(gamma_field, dtype=np.float64)
    return {"mean": float(g.mean()), "std": float(g.std()), "min": float(g.min()),
            "max": float(g.max())}
