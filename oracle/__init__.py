"""Plain FP64 CPU oracle for the D3Q27 KBC lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  This package checks the GPU library; only the
test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU path.

The arithmetic lives in ``kbc_oracle.c`` (plain C, IEEE double, one function
per passage of Boesch, Chikatamarla & Karlin, arXiv:1507.02518).  This module
only marshals numpy arrays into it through ctypes.  ``spectrum`` is the one
diagnostic written here, with numpy's FFT as a library primitive.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkbc_oracle.so")

S_D, S_DT, S_DQ, S_DTQ = 0, 1, 2, 3
# the same four variants in the central-moment basis (d~, d~+t~, d~+q~, d~+t~+q~)
S_CD, S_CDT, S_CDQ, S_CDTQ = 4, 5, 6, 7
GAMMA_ESTIMATE, GAMMA_FIXED, GAMMA_EXACT = 0, 1, 2
DEFAULT_GAMMA_EPS = 1e-28

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.kbco_velocity.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.kbco_weight.argtypes = [ctypes.c_int]
    lib.kbco_weight.restype = ctypes.c_double
    lib.kbco_beta_from_nu.argtypes = [ctypes.c_double]
    lib.kbco_beta_from_nu.restype = ctypes.c_double
    lib.kbco_feq.argtypes = [ctypes.c_double, _D, _D]
    lib.kbco_natural_moments.argtypes = [_D, _D]
    lib.kbco_natural_moments.restype = ctypes.c_double
    lib.kbco_f_from_moments.argtypes = [ctypes.c_double, _D, _D]
    lib.kbco_parts.argtypes = [ctypes.c_double, _D, _D, _D, _D, _D]
    lib.kbco_s_part.argtypes = [ctypes.c_double, _D, ctypes.c_int, _D]
    lib.kbco_central_moments.argtypes = [_D, _D, _D]
    lib.kbco_central_moments.restype = ctypes.c_double
    lib.kbco_central_parts.argtypes = [ctypes.c_double, _D, _D, _D, _D, _D, _D]
    lib.kbco_central_column.argtypes = [_D, ctypes.c_int, _D]
    lib.kbco_s_of.argtypes = [_D, ctypes.c_int, _D]
    lib.kbco_collide.argtypes = [_D, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
    lib.kbco_collide.restype = ctypes.c_double
    lib.kbco_gamma_exact.argtypes = [_D, _D, _D, ctypes.c_double]
    lib.kbco_gamma_exact.restype = ctypes.c_double
    lib.kbco_init_feq.argtypes = [_I64, _I64, _I64, _D, _D, _D]
    lib.kbco_collide_field.argtypes = [_I64, _I64, _I64, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       _D, _D, _D]
    lib.kbco_stream.argtypes = [_I64, _I64, _I64, _D, _D]
    lib.kbco_step.argtypes = [_I64, _I64, _I64, ctypes.c_double, ctypes.c_int,
                              ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, _D, _D]
    lib.kbco_macros.argtypes = [_I64, _I64, _I64, _D, _D, _D]
    lib.kbco_energy.argtypes = [_I64, _I64, _I64, _D]
    lib.kbco_energy.restype = ctypes.c_double
    lib.kbco_enstrophy.argtypes = [_I64, _I64, _I64, _D]
    lib.kbco_enstrophy.restype = ctypes.c_double
    lib.kbco_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _vec(a, n=27):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == (n,), a.shape
    return a


def _field_shape(F):
    assert F.ndim == 4 and F.shape[0] == 27, F.shape
    _, nz, ny, nx = F.shape
    return nx, ny, nz


# ---- lattice ---------------------------------------------------------------

def velocities() -> np.ndarray:
    lib = _load()
    out = np.zeros((27, 3), dtype=np.int64)
    v = (ctypes.c_int * 3)()
    for i in range(27):
        lib.kbco_velocity(i, v)
        out[i] = list(v)
    return out


def weights() -> np.ndarray:
    lib = _load()
    return np.array([lib.kbco_weight(i) for i in range(27)])


def beta_from_nu(nu: float) -> float:
    return _load().kbco_beta_from_nu(float(nu))


# ---- one node --------------------------------------------------------------

def feq(rho: float, u) -> np.ndarray:
    u = _vec(u, 3)
    out = np.zeros(27)
    _load().kbco_feq(float(rho), _ptr(u), _ptr(out))
    return out


def natural_moments(f):
    """Return (rho, M[27]) with M[p + 3q + 9r] = M_pqr."""
    f = _vec(f)
    M = np.zeros(27)
    rho = _load().kbco_natural_moments(_ptr(f), _ptr(M))
    return rho, M


def f_from_moments(rho: float, M) -> np.ndarray:
    M = _vec(M)
    out = np.zeros(27)
    _load().kbco_f_from_moments(float(rho), _ptr(M), _ptr(out))
    return out


def parts(rho: float, M):
    """Return (k, d, t, q) of the table of parts."""
    M = _vec(M)
    k, d, t, q = (np.zeros(27) for _ in range(4))
    _load().kbco_parts(float(rho), _ptr(M), _ptr(k), _ptr(d), _ptr(t), _ptr(q))
    return k, d, t, q


def s_part(rho: float, M, variant: int = S_DTQ) -> np.ndarray:
    M = _vec(M)
    out = np.zeros(27)
    _load().kbco_s_part(float(rho), _ptr(M), int(variant), _ptr(out))
    return out


def central_moments(f):
    """Return (rho, u[3], Mt[27]) with Mt[p + 3q + 9r] = Mt_pqr."""
    f = _vec(f)
    Mt, u = np.zeros(27), np.zeros(3)
    rho = _load().kbco_central_moments(_ptr(f), _ptr(Mt), _ptr(u))
    return rho, u, Mt


def central_parts(rho: float, u, Mt):
    """Return (k~, d~, t~, q~) of the central-basis representation."""
    u, Mt = _vec(u, 3), _vec(Mt)
    k, d, t, q = (np.zeros(27) for _ in range(4))
    _load().kbco_central_parts(float(rho), _ptr(u), _ptr(Mt), _ptr(k), _ptr(d), _ptr(t),
                               _ptr(q))
    return k, d, t, q


def central_column(u, m: int) -> np.ndarray:
    """Weight of Mt_m (m = p + 3q + 9r) in f_i / rho at velocity u."""
    u = _vec(u, 3)
    out = np.zeros(27)
    _load().kbco_central_column(_ptr(u), int(m), _ptr(out))
    return out


def s_of(f, variant: int = S_DTQ) -> np.ndarray:
    """Shear part of f for any variant (natural 0-3, central 4-7)."""
    f = _vec(f)
    out = np.zeros(27)
    _load().kbco_s_of(_ptr(f), int(variant), _ptr(out))
    return out


def collide(F, beta: float, variant: int = S_DTQ, gamma: float | None = None,
            gamma_eps: float = DEFAULT_GAMMA_EPS, exact: bool = False):
    """One node collision.  Returns dict with P, feq, ds, dh, gamma."""
    F = _vec(F)
    P, fe, ds, dh = (np.zeros(27) for _ in range(4))
    if gamma is not None:
        mode, gval = GAMMA_FIXED, float(gamma)
    else:
        mode, gval = (GAMMA_EXACT if exact else GAMMA_ESTIMATE), 0.0
    g = _load().kbco_collide(_ptr(F), float(beta), int(variant), mode, gval,
                             float(gamma_eps), _ptr(P), _ptr(fe), _ptr(ds), _ptr(dh))
    return {"P": P, "feq": fe, "ds": ds, "dh": dh, "gamma": g}


def gamma_exact(feq_, ds, dh, beta: float) -> float:
    return _load().kbco_gamma_exact(_ptr(_vec(feq_)), _ptr(_vec(ds)), _ptr(_vec(dh)),
                                    float(beta))


# ---- lattice fields --------------------------------------------------------

def init_feq(u, rho=None) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.ndim == 4 and u.shape[0] == 3
    _, nz, ny, nx = u.shape
    if rho is not None:
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        assert rho.shape == (nz, ny, nx)
    F = np.empty((27, nz, ny, nx))
    _load().kbco_init_feq(nx, ny, nz, _ptr(u), _ptr(rho), _ptr(F))
    return F


def _gamma_args(gamma, exact):
    if gamma is not None:
        return GAMMA_FIXED, float(gamma)
    return (GAMMA_EXACT if exact else GAMMA_ESTIMATE), 0.0


def collide_field(F, beta, variant=S_DTQ, gamma=None, gamma_eps=DEFAULT_GAMMA_EPS,
                  exact=False, want_gamma=False):
    F = np.ascontiguousarray(F, dtype=np.float64)
    nx, ny, nz = _field_shape(F)
    P = np.empty_like(F)
    gf = np.empty((nz, ny, nx)) if want_gamma else None
    mode, gval = _gamma_args(gamma, exact)
    _load().kbco_collide_field(nx, ny, nz, float(beta), int(variant), mode, gval,
                               float(gamma_eps), _ptr(F), _ptr(P), _ptr(gf))
    return (P, gf) if want_gamma else P


def stream(P) -> np.ndarray:
    P = np.ascontiguousarray(P, dtype=np.float64)
    nx, ny, nz = _field_shape(P)
    out = np.empty_like(P)
    _load().kbco_stream(nx, ny, nz, _ptr(P), _ptr(out))
    return out


def run(F, beta, steps, variant=S_DTQ, gamma=None, gamma_eps=DEFAULT_GAMMA_EPS,
        exact=False, callback=None):
    """Advance F by `steps` collide+stream steps; returns the new field.

    callback(t, F) is called for t = 0..steps (before the first step and after
    every step) when given.
    """
    F = np.array(F, dtype=np.float64, order="C", copy=True)
    nx, ny, nz = _field_shape(F)
    P = np.empty_like(F)
    G = np.empty_like(F)
    mode, gval = _gamma_args(gamma, exact)
    lib = _load()
    if callback is not None:
        callback(0, F)
    for t in range(steps):
        lib.kbco_step(nx, ny, nz, float(beta), int(variant), mode, gval,
                      float(gamma_eps), _ptr(F), _ptr(P), _ptr(G))
        F, G = G, F
        if callback is not None:
            callback(t + 1, F)
    return F


def macros(F):
    F = np.ascontiguousarray(F, dtype=np.float64)
    nx, ny, nz = _field_shape(F)
    rho = np.empty((nz, ny, nx))
    u = np.empty((3, nz, ny, nx))
    _load().kbco_macros(nx, ny, nz, _ptr(F), _ptr(rho), _ptr(u))
    return rho, u


def energy(u) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    _, nz, ny, nx = u.shape
    return _load().kbco_energy(nx, ny, nz, _ptr(u))


def enstrophy(u) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    _, nz, ny, nx = u.shape
    return _load().kbco_enstrophy(nx, ny, nz, _ptr(u))


def spectrum(u) -> np.ndarray:
    """Shell energy spectrum E(kappa), kappa = 0..kmax (section V.A).

    E(kappa) = sum over integer wave vectors with round(|k|) = kappa of
    (1/2)|u_hat(k)|^2, u_hat the DFT of u' = u - <u> normalised by the number
    of nodes, so that sum_kappa E(kappa) = k (the kinetic energy).
    """
    u = np.asarray(u, dtype=np.float64)
    _, nz, ny, nx = u.shape
    up = u - u.mean(axis=(1, 2, 3), keepdims=True)
    uh = np.fft.fftn(up, axes=(1, 2, 3)) / (nx * ny * nz)
    e = 0.5 * (np.abs(uh) ** 2).sum(axis=0)
    kz = np.fft.fftfreq(nz, 1.0 / nz)[:, None, None]
    ky = np.fft.fftfreq(ny, 1.0 / ny)[None, :, None]
    kx = np.fft.fftfreq(nx, 1.0 / nx)[None, None, :]
    kk = np.rint(np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)).astype(np.int64)
    return np.bincount(kk.ravel(), weights=e.ravel())


def num_threads() -> int:
    return _load().kbco_num_threads()
