"""Seeded synthetic inputs: initial velocity fields for periodic boxes.

This module holds no arithmetic of the lattice Boltzmann method itself; it
only builds velocity fields u[3][nz][ny][nx] (float64, x fastest) that both
the GPU path and its CPU oracle start from.

* ``taylor_green``: u = (U sin x cos y cos z, -U cos x sin y cos z, 0) with
  node coordinates x_j = 2 pi j / N (no half-cell offset).
* ``hit``: decaying homogeneous isotropic turbulence, a random solenoidal
  field whose shell spectrum follows E(k) ~ k^4 exp(-2 (k/k0)^2), the shape
  of the paper's narrow-band initial spectrum (section V.D), scaled to a
  given r.m.s. velocity u' = sqrt(<|u|^2>/3).
* ``kida``: the Kida vortex of section V.
* ``shear_wave``: u_x = U sin(2 pi y / N_y), the viscosity probe.
* ``smooth_random``: a few random Fourier modes on any (ragged) box.
* ``smooth_random_device``: the same kind of field built in device memory
  (torch), for boxes too large to build on the host.
"""
from __future__ import annotations

import numpy as np


def _coords(n: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(n) / n


def _shape3(shape):
    if np.isscalar(shape):
        return int(shape), int(shape), int(shape)
    nx, ny, nz = (int(s) for s in shape)
    return nx, ny, nz


def taylor_green(shape, U: float = 0.05) -> np.ndarray:
    nx, ny, nz = _shape3(shape)
    x = _coords(nx)[None, None, :]
    y = _coords(ny)[None, :, None]
    z = _coords(nz)[:, None, None]
    u = np.zeros((3, nz, ny, nx))
    u[0] = U * np.sin(x) * np.cos(y) * np.cos(z)
    u[1] = -U * np.cos(x) * np.sin(y) * np.cos(z)
    return u


def kida(shape, U0: float = 0.05) -> np.ndarray:
    nx, ny, nz = _shape3(shape)
    x = _coords(nx)[None, None, :]
    y = _coords(ny)[None, :, None]
    z = _coords(nz)[:, None, None]
    u = np.zeros((3, nz, ny, nx))
    u[0] = U0 * np.sin(x) * (np.cos(3 * y) * np.cos(z) - np.cos(y) * np.cos(3 * z))
    u[1] = U0 * np.sin(y) * (np.cos(3 * z) * np.cos(x) - np.cos(z) * np.cos(3 * x))
    u[2] = U0 * np.sin(z) * (np.cos(3 * x) * np.cos(y) - np.cos(x) * np.cos(3 * y))
    return u


def shear_wave(shape, U: float = 1e-3) -> np.ndarray:
    nx, ny, nz = _shape3(shape)
    y = _coords(ny)[None, :, None]
    u = np.zeros((3, nz, ny, nx))
    u[0] = U * np.sin(y) * np.ones((nz, 1, nx))
    return u


def hit(n, k0: float = 4.0, u_rms: float = 0.04, seed: int = 0) -> np.ndarray:
    """Random solenoidal field with shell spectrum ~ k^4 exp(-2 (k/k0)^2).

    White Gaussian noise is transformed (real-to-complex, so Hermitian
    symmetry holds by construction), projected onto the plane normal to each
    wave vector, and every integer shell round(|k|) is rescaled so its
    energy follows the target spectrum.  Nyquist planes of even-sized axes
    (their own conjugate partners) are dropped.  The mean is removed and the
    field is scaled to the requested per-component r.m.s. value.
    """
    import scipy.fft as sfft

    nx, ny, nz = _shape3(n)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((3, nz, ny, nx))
    wh = sfft.rfftn(w, axes=(1, 2, 3), workers=-1)
    del w
    kz = np.fft.fftfreq(nz, 1.0 / nz)[:, None, None]
    ky = np.fft.fftfreq(ny, 1.0 / ny)[None, :, None]
    kx = np.fft.rfftfreq(nx, 1.0 / nx)[None, None, :]
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2s = np.where(k2 == 0, 1.0, k2)
    kdotw = (kx * wh[0] + ky * wh[1] + kz * wh[2]) / k2s
    wh[0] -= kx * kdotw
    wh[1] -= ky * kdotw
    wh[2] -= kz * kdotw
    del kdotw
    drop = k2 == 0
    if nx % 2 == 0:
        drop = drop | (kx == nx // 2)
    if ny % 2 == 0:
        drop = drop | (np.abs(ky) == ny // 2)
    if nz % 2 == 0:
        drop = drop | (np.abs(kz) == nz // 2)
    wh[:, drop] = 0.0
    # modes with 0 < kx < nx/2 stand for themselves and their conjugates
    mult = np.where((kx == 0) | ((nx % 2 == 0) & (kx == nx // 2)), 1.0, 2.0)
    mult = np.broadcast_to(mult, k2.shape)
    shell = np.rint(np.sqrt(k2)).astype(np.int64)
    e_now = np.bincount(shell.ravel(),
                        weights=(mult * (np.abs(wh) ** 2).sum(axis=0)).ravel())
    kk = np.arange(e_now.size, dtype=np.float64)
    e_target = kk ** 4 * np.exp(-2.0 * (kk / k0) ** 2)
    scale = np.zeros_like(e_now)
    ok = e_now > 0
    scale[ok] = np.sqrt(e_target[ok] / e_now[ok])
    wh *= scale[shell][None]
    u = sfft.irfftn(wh, s=(nz, ny, nx), axes=(1, 2, 3), workers=-1)
    del wh
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    rms = np.sqrt((u ** 2).sum(axis=0).mean() / 3.0)
    u *= u_rms / rms
    return np.ascontiguousarray(u)


def smooth_random(shape, amplitude: float = 0.03, modes: int = 4, seed: int = 0) -> np.ndarray:
    """Sum of a few random low-wavenumber sinusoids per component."""
    nx, ny, nz = _shape3(shape)
    rng = np.random.default_rng(seed)
    x = _coords(nx)[None, None, :]
    y = _coords(ny)[None, :, None]
    z = _coords(nz)[:, None, None]
    u = np.zeros((3, nz, ny, nx))
    for a in range(3):
        for _ in range(modes):
            kx, ky, kz = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            amp = rng.uniform(-1, 1) * amplitude / modes
            u[a] += amp * np.sin(kx * x + ky * y + kz * z + ph)
    return u


def smooth_random_device(shape, amplitude: float = 0.1, modes: int = 4, seed: int = 0,
                         device: str = "cuda"):
    """Sum of `modes` plane waves per component, built as a float64 torch
    tensor [3][nz][ny][nx] on `device`: every wave has wave numbers 1-3 with
    a random sign along each axis (so no axis is uniform) and a random phase,
    amplitude / modes each, so |u_a| <= amplitude."""
    import torch

    nx, ny, nz = _shape3(shape)
    rng = np.random.default_rng(seed)

    def coord(n):
        return torch.arange(n, dtype=torch.float64, device=device) * (2.0 * np.pi / n)

    x, y, z = coord(nx), coord(ny), coord(nz)
    u = torch.zeros((3, nz, ny, nx), dtype=torch.float64, device=device)
    for a in range(3):
        for _ in range(modes):
            k = rng.integers(1, 4, size=3) * rng.choice([-1, 1], size=3)
            ph = float(rng.uniform(0, 2 * np.pi))
            arg = ((float(k[2]) * z)[:, None, None] + (float(k[1]) * y)[None, :, None]
                   + (float(k[0]) * x + ph)[None, None, :])
            u[a].add_(arg.sin_(), alpha=amplitude / modes)
            del arg
    return u


def random_density(shape, amplitude: float = 0.01, seed: int = 0) -> np.ndarray:
    nx, ny, nz = _shape3(shape)
    rng = np.random.default_rng(seed + 7919)
    return 1.0 + amplitude * rng.uniform(-1, 1, size=(nz, ny, nx))
