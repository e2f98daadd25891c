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
