"""Host-side post-processing of read-back fields (section V.A diagnostics).

``spectrum``: shell energy spectrum E(kappa) of a velocity field read back
with kbc_moments; kappa = round(|k|) over the integer wave vectors of the
periodic box, E normalised so that sum_kappa E(kappa) = k, the kinetic
energy (1/2)<|u - <u>|^2>.  ``spectrum_error`` compares two spectra shell
by shell.
"""
from __future__ import annotations

import numpy as np


def spectrum(u) -> np.ndarray:
    import scipy.fft as sfft

    u = np.asarray(u, dtype=np.float64)
    _, nz, ny, nx = u.shape
    e = None
    for a in range(3):
        c = u[a] - u[a].mean()
        ch = sfft.rfftn(c, workers=-1) / (nx * ny * nz)
        p = np.abs(ch) ** 2
        e = p if e is None else e + p
    # half spectrum: modes 0 < kx < nx/2 stand for themselves and their conjugates
    kx = np.fft.rfftfreq(nx, 1.0 / nx)
    w = np.where((kx == 0) | ((nx % 2 == 0) & (kx == nx // 2)), 1.0, 2.0)
    e = 0.5 * e * w[None, None, :]
    kz = np.fft.fftfreq(nz, 1.0 / nz)[:, None, None]
    ky = np.fft.fftfreq(ny, 1.0 / ny)[None, :, None]
    kk = np.rint(np.sqrt(kx[None, None, :] ** 2 + ky ** 2 + kz ** 2)).astype(np.int64)
    return np.bincount(kk.ravel(), weights=e.ravel())


def spectrum_error(E, E_ref, kmax=None):
    """Max and L2 relative error over shells 1..kmax (default len/3)."""
    n = min(len(E), len(E_ref))
    kmax = kmax or n // 3
    a, b = np.asarray(E[1:kmax + 1]), np.asarray(E_ref[1:kmax + 1])
    rel = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
    l2 = float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))
    return {"max_rel": float(rel.max()), "l2_rel": l2, "shells": int(kmax)}


def turbulence_scales(k: float, eps: float, nu: float) -> dict:
    """Turbulence, Taylor and Kolmogorov scales of section V.A from the
    kinetic energy k, the dissipation rate eps and the viscosity nu:
    l0 = k^(3/2)/eps, u0 = k^(1/2), tau0 = l0/u0, Re0 = l0 u0/nu;
    lambda = (15 nu u'^2/eps)^(1/2) with u' = (2k/3)^(1/2), tau_lambda =
    lambda/u', Re_lambda = lambda u'/nu; eta = (nu^3/eps)^(1/4),
    u_eta = (nu eps)^(1/4), tau_eta = (nu/eps)^(1/2)."""
    l0 = k ** 1.5 / eps
    u0 = k ** 0.5
    up = (2.0 * k / 3.0) ** 0.5
    lam = (15.0 * nu * up * up / eps) ** 0.5
    return {"l0": l0, "u0": u0, "tau0": l0 / u0, "Re0": l0 * u0 / nu,
            "lambda": lam, "u_lambda": up, "tau_lambda": lam / up, "Re_lambda": lam * up / nu,
            "eta": (nu ** 3 / eps) ** 0.25, "u_eta": (nu * eps) ** 0.25,
            "tau_eta": (nu / eps) ** 0.5}
