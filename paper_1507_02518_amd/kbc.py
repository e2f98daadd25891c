"""ctypes binding of libkbc.so (C-ABI declared in include/kbc.h).

Argument marshalling only: every function below forwards to the C entry
point of the same name, and all computation on the populations runs in the
library's HIP kernels.  Loading fails loudly if libkbc.so is missing; there
is no fallback path.

``Box`` is a small convenience wrapper around a handle.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkbc.so")

KBC_OK = 0
KBC_EINVAL = -1
KBC_ENOMEM = -2
KBC_EDEVICE = -3
KBC_EUNSTABLE = -4
KBC_ECAPACITY = -5
KBC_ESTATE = -6

F64, F32_DEV, F16_DEV, F32_DEV_X = 0, 1, 2, 3
S_D, S_DT, S_DQ, S_DTQ = 0, 1, 2, 3
S_CD, S_CDT, S_CDQ, S_CDTQ = 4, 5, 6, 7   # central-moment variants
PULL, AA = 0, 1
GAMMA_ENTROPIC, GAMMA_FIXED, GAMMA_EXACT = 0, 1, 2


def _set_gamma(o, gamma):
    """gamma: None -> entropic estimate; "exact" -> root of the entropy
    condition; a number -> that fixed value."""
    if gamma is None:
        o.gamma_mode, o.gamma_value = GAMMA_ENTROPIC, 2.0
    elif isinstance(gamma, str):
        if gamma != "exact":
            raise ValueError(f"gamma must be None, 'exact' or a number, not {gamma!r}")
        o.gamma_mode, o.gamma_value = GAMMA_EXACT, 2.0
    else:
        o.gamma_mode, o.gamma_value = GAMMA_FIXED, float(gamma)

DTYPES = {"f64": F64, "f32": F32_DEV, "f16": F16_DEV, "f32x": F32_DEV_X}


class KbcError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} failed ({code}): {msg}")
        self.code = code


class kbc_stats(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("epsilon", ctypes.c_double),
        ("div2", ctypes.c_double),
        ("dudx_moment", ctypes.c_double * 5),
        ("skewness", ctypes.c_double * 4),
    ]


class kbc_options(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("streaming", ctypes.c_int32),
        ("gamma_mode", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("gamma_value", ctypes.c_double),
        ("gamma_eps", ctypes.c_double),
        ("stream", ctypes.c_void_p),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_H = ctypes.c_void_p


def load():
    """Load libkbc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1507_02518_amd.build` "
            "(there is no non-GPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    I64P = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "kbc_options_default": (None, [ctypes.POINTER(kbc_options)]),
        "kbc_create": (ctypes.c_int, [I64P, ctypes.c_double, ctypes.c_int32,
                                      ctypes.POINTER(kbc_options), ctypes.POINTER(_H)]),
        "kbc_destroy": (ctypes.c_int, [_H]),
        "kbc_init_velocity": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p]),
        "kbc_init_velocity_device": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p]),
        "kbc_step": (ctypes.c_int, [_H, ctypes.c_int64]),
        "kbc_moments": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_void_p]),
        "kbc_energy": (ctypes.c_int, [_H, _D]),
        "kbc_energy_series": (ctypes.c_int, [_H, ctypes.c_int64, _D]),
        "kbc_energy_series_noalloc": (ctypes.c_int, [_H, ctypes.c_int64, _D]),
        "kbc_enstrophy": (ctypes.c_int, [_H, _D]),
        "kbc_statistics": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.POINTER(kbc_stats)]),
        "kbc_gamma_statistics": (ctypes.c_int, [_H, ctypes.c_void_p]),
        "kbc_correlation": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
        "kbc_get_populations": (ctypes.c_int, [_H, ctypes.c_void_p]),
        "kbc_set_populations": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_int64]),
        "kbc_sample_populations": (ctypes.c_int, [_H, ctypes.c_void_p, ctypes.c_int64,
                                                  ctypes.c_void_p]),
        "kbc_time": (ctypes.c_int, [_H, I64P]),
        "kbc_sync": (ctypes.c_int, [_H]),
        "kbc_bytes_per_node_step": (ctypes.c_int, [_H, _D]),
        "kbc_stream": (ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_void_p)]),
        "kbc_hbm_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]),
        "kbc_pool_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32,
                                           ctypes.POINTER(kbc_options), ctypes.c_int32,
                                           ctypes.c_char_p, ctypes.POINTER(_H)]),
        "kbc_pool_destroy": (ctypes.c_int, [_H]),
        "kbc_pool_admit": (ctypes.c_int, [_H, I64P, ctypes.c_double, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]),
        "kbc_pool_advance": (ctypes.c_int, [_H, ctypes.c_int64]),
        "kbc_pool_advance_slots": (ctypes.c_int, [_H, ctypes.c_int64, ctypes.c_void_p,
                                                  ctypes.c_int32]),
        "kbc_pool_poll": (ctypes.c_int, [_H, ctypes.c_int32, I64P]),
        "kbc_pool_result": (ctypes.c_int, [_H, ctypes.c_int32, _D, _D, ctypes.c_void_p,
                                           ctypes.c_void_p]),
        "kbc_pool_release": (ctypes.c_int, [_H, ctypes.c_int32]),
        "kbc_pool_sync": (ctypes.c_int, [_H]),
        "kbc_pool_info": (ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_size_t),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32)]),
        "kbc_pool_set_launch": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int32]),
        "kbc_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, func: str):
    if rc != KBC_OK:
        raise KbcError(rc, func, load().kbc_last_error().decode())
    return rc


def _arr(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == tuple(shape), (a.shape, shape)
    return a


def _p(a):
    return None if a is None else a.ctypes.data


# ---- C-ABI mirrors -----------------------------------------------------------

def kbc_options_default() -> kbc_options:
    o = kbc_options()
    load().kbc_options_default(ctypes.byref(o))
    return o


def kbc_create(shape, nu: float, dtype: int = F64, opt: kbc_options | None = None) -> int:
    s = (ctypes.c_int64 * 3)(*[int(v) for v in shape])
    h = _H()
    _check(load().kbc_create(s, float(nu), int(dtype),
                             ctypes.byref(opt) if opt is not None else None, ctypes.byref(h)),
           "kbc_create")
    return h.value


def kbc_destroy(h: int):
    _check(load().kbc_destroy(h), "kbc_destroy")


def kbc_init_velocity(h: int, u, rho=None):
    """u: [3][nz][ny][nx] float64 host array; rho: [nz][ny][nx] or None."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    _check(load().kbc_init_velocity(h, _p(u), _p(rho)), "kbc_init_velocity")


def kbc_init_velocity_device(h: int, u_ptr: int, rho_ptr: int | None = None):
    _check(load().kbc_init_velocity_device(h, u_ptr, rho_ptr), "kbc_init_velocity_device")


def kbc_step(h: int, n: int = 1):
    _check(load().kbc_step(h, int(n)), "kbc_step")


def kbc_moments(h: int, rho_out=None, u_out=None):
    _check(load().kbc_moments(h, _p(rho_out), _p(u_out)), "kbc_moments")


def kbc_energy(h: int) -> float:
    k = ctypes.c_double()
    _check(load().kbc_energy(h, ctypes.byref(k)), "kbc_energy")
    return k.value


def kbc_energy_series(h: int, n: int) -> np.ndarray:
    k = np.zeros(max(int(n), 0), dtype=np.float64)
    _check(load().kbc_energy_series(h, int(n), k.ctypes.data_as(_D) if n > 0 else None),
           "kbc_energy_series")
    return k


NOALLOC_MAX_STEPS = 65536


def kbc_energy_series_noalloc(h: int, n: int) -> np.ndarray:
    k = np.zeros(max(int(n), 0), dtype=np.float64)
    _check(load().kbc_energy_series_noalloc(h, int(n), k.ctypes.data_as(_D) if n > 0 else None),
           "kbc_energy_series_noalloc")
    return k


def kbc_enstrophy(h: int) -> float:
    w = ctypes.c_double()
    _check(load().kbc_enstrophy(h, ctypes.byref(w)), "kbc_enstrophy")
    return w.value


def kbc_statistics(h: int, order: int = 8) -> dict:
    st = kbc_stats()
    _check(load().kbc_statistics(h, int(order), ctypes.byref(st)), "kbc_statistics")
    return {"k": st.k, "omega": st.omega, "epsilon": st.epsilon, "div2": st.div2,
            "dudx_moments": {n: st.dudx_moment[n - 2] for n in range(2, 7)},
            "skewness": {n: st.skewness[n - 3] for n in range(3, 7)}}


def kbc_gamma_statistics(h: int) -> dict:
    out = np.zeros(4)
    _check(load().kbc_gamma_statistics(h, _p(out)), "kbc_gamma_statistics")
    return {"mean": out[0], "std": out[1], "min": out[2], "max": out[3]}


def kbc_correlation(h: int, rmax: int):
    r11, r22 = np.zeros(rmax + 1), np.zeros(rmax + 1)
    _check(load().kbc_correlation(h, int(rmax), _p(r11), _p(r22)), "kbc_correlation")
    return r11, r22


def kbc_get_populations(h: int, f_out):
    _check(load().kbc_get_populations(h, _p(f_out)), "kbc_get_populations")


def kbc_sample_populations(h: int, nodes) -> np.ndarray:
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.empty((nodes.size, 27))
    _check(load().kbc_sample_populations(h, _p(nodes), nodes.size, _p(out)),
           "kbc_sample_populations")
    return out


def kbc_set_populations(h: int, f, t: int = 0):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(load().kbc_set_populations(h, _p(f), int(t)), "kbc_set_populations")


def kbc_time(h: int) -> int:
    t = ctypes.c_int64()
    _check(load().kbc_time(h, ctypes.byref(t)), "kbc_time")
    return t.value


def kbc_sync(h: int):
    _check(load().kbc_sync(h), "kbc_sync")


def kbc_bytes_per_node_step(h: int) -> float:
    b = ctypes.c_double()
    _check(load().kbc_bytes_per_node_step(h, ctypes.byref(b)), "kbc_bytes_per_node_step")
    return b.value


def kbc_stream(h: int) -> int:
    s = ctypes.c_void_p()
    _check(load().kbc_stream(h, ctypes.byref(s)), "kbc_stream")
    return s.value or 0


def kbc_hbm_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream: int = 0):
    _check(load().kbc_hbm_copy(dst_ptr, src_ptr, int(nbytes), stream or None), "kbc_hbm_copy")


def kbc_pool_create(budget_bytes: int, dtype: int = F32_DEV_X, opt: kbc_options | None = None,
                    max_slots: int = 256, tune_cache: str | None = None) -> int:
    h = _H()
    _check(load().kbc_pool_create(int(budget_bytes), int(dtype),
                                  ctypes.byref(opt) if opt is not None else None, int(max_slots),
                                  tune_cache.encode() if tune_cache else None, ctypes.byref(h)),
           "kbc_pool_create")
    return h.value


def kbc_pool_destroy(p: int):
    _check(load().kbc_pool_destroy(p), "kbc_pool_destroy")


def kbc_pool_admit(p: int, shape, nu: float, u, steps: int) -> int:
    s = (ctypes.c_int64 * 3)(*[int(v) for v in shape])
    u = np.ascontiguousarray(u, dtype=np.float64)
    slot = ctypes.c_int32()
    _check(load().kbc_pool_admit(p, s, float(nu), _p(u), int(steps), ctypes.byref(slot)),
           "kbc_pool_admit")
    return slot.value


def kbc_pool_advance(p: int, g: int):
    _check(load().kbc_pool_advance(p, int(g)), "kbc_pool_advance")


def kbc_pool_advance_slots(p: int, g: int, slots):
    arr = np.ascontiguousarray(slots, dtype=np.int32)
    _check(load().kbc_pool_advance_slots(p, int(g), _p(arr) if arr.size else None, arr.size),
           "kbc_pool_advance_slots")


def kbc_pool_poll(p: int, slot: int) -> int:
    r = ctypes.c_int64()
    _check(load().kbc_pool_poll(p, int(slot), ctypes.byref(r)), "kbc_pool_poll")
    return r.value


def kbc_pool_result(p: int, slot: int, rho_out=None, u_out=None):
    k = ctypes.c_double()
    w = ctypes.c_double()
    _check(load().kbc_pool_result(p, int(slot), ctypes.byref(k), ctypes.byref(w), _p(rho_out),
                                  _p(u_out)), "kbc_pool_result")
    return k.value, w.value


def kbc_pool_release(p: int, slot: int):
    _check(load().kbc_pool_release(p, int(slot)), "kbc_pool_release")


def kbc_pool_sync(p: int):
    _check(load().kbc_pool_sync(p), "kbc_pool_sync")


def kbc_pool_info(p: int) -> dict:
    used = ctypes.c_size_t()
    boxes, block, grid, sub, tuning = (ctypes.c_int32() for _ in range(5))
    _check(load().kbc_pool_info(p, ctypes.byref(used), ctypes.byref(boxes), ctypes.byref(block),
                                ctypes.byref(grid), ctypes.byref(sub), ctypes.byref(tuning)),
           "kbc_pool_info")
    return {"bytes_used": used.value, "boxes": boxes.value, "block": block.value,
            "grid": grid.value, "sub": sub.value, "tuning": bool(tuning.value)}


def kbc_pool_set_launch(p: int, block: int, grid: int, sub: int = 4):
    _check(load().kbc_pool_set_launch(p, int(block), int(grid), int(sub)), "kbc_pool_set_launch")


def kbc_last_error() -> str:
    return load().kbc_last_error().decode()


# ---- convenience wrapper -----------------------------------------------------

class Box:
    """One periodic box: owns a handle; numpy in, numpy out."""

    def __init__(self, shape, nu, dtype=F64, variant=S_DTQ, streaming=PULL,
                 gamma=None, gamma_eps=0.0, stream=None, device=-1):
        if isinstance(dtype, str):
            dtype = DTYPES[dtype]
        if isinstance(shape, int):
            shape = (shape, shape, shape)
        self.shape = tuple(int(s) for s in shape)
        self.dtype = dtype
        o = kbc_options_default()
        o.variant = variant
        o.streaming = streaming
        _set_gamma(o, gamma)
        o.gamma_eps = float(gamma_eps)
        o.device = device
        o.stream = stream
        self.h = kbc_create(self.shape, nu, dtype, o)

    @property
    def nodes(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]

    def _field_shape(self):
        nx, ny, nz = self.shape
        return (nz, ny, nx)

    def init_velocity(self, u, rho=None):
        kbc_init_velocity(self.h, _arr(u, (3,) + self._field_shape()),
                          _arr(rho, self._field_shape()))
        return self

    def step(self, n=1):
        kbc_step(self.h, n)
        return self

    def moments(self):
        rho = np.empty(self._field_shape())
        u = np.empty((3,) + self._field_shape())
        kbc_moments(self.h, rho, u)
        return rho, u

    def energy(self) -> float:
        return kbc_energy(self.h)

    def energy_series(self, n: int) -> np.ndarray:
        """Advance n steps; k after each of them."""
        return kbc_energy_series(self.h, n)

    def enstrophy(self) -> float:
        return kbc_enstrophy(self.h)

    def statistics(self, order: int = 8) -> dict:
        return kbc_statistics(self.h, order)

    def gamma_statistics(self) -> dict:
        return kbc_gamma_statistics(self.h)

    def correlation(self, rmax: int):
        return kbc_correlation(self.h, rmax)

    def populations(self):
        f = np.empty((27,) + self._field_shape())
        kbc_get_populations(self.h, f)
        return f

    def sample(self, nodes):
        return kbc_sample_populations(self.h, nodes)

    def set_populations(self, f, t=0):
        kbc_set_populations(self.h, _arr(f, (27,) + self._field_shape()), t)
        return self

    @property
    def t(self) -> int:
        return kbc_time(self.h)

    def sync(self):
        kbc_sync(self.h)

    @property
    def stream(self) -> int:
        return kbc_stream(self.h)

    def bytes_per_node_step(self) -> float:
        return kbc_bytes_per_node_step(self.h)

    def close(self):
        if getattr(self, "h", None):
            kbc_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """A batched ensemble of boxes on one GPU (continuous batching)."""

    def __init__(self, budget_bytes, dtype=F32_DEV_X, variant=S_DTQ, max_slots=256,
                 tune_cache=None, gamma=None, device=-1, stream=None):
        if isinstance(dtype, str):
            dtype = DTYPES[dtype]
        o = kbc_options_default()
        o.variant = variant
        _set_gamma(o, gamma)
        o.device = device
        o.stream = stream
        self.dtype = dtype
        self.h = kbc_pool_create(budget_bytes, dtype, o, max_slots, tune_cache)

    def admit(self, u, nu, steps) -> int:
        """u: [3][nz][ny][nx]; returns the slot."""
        nz, ny, nx = u.shape[1:]
        return kbc_pool_admit(self.h, (nx, ny, nz), nu, u, steps)

    def advance(self, g, slots=None):
        if slots is None:
            kbc_pool_advance(self.h, g)
        else:
            kbc_pool_advance_slots(self.h, g, list(slots))

    def poll(self, slot) -> int:
        return kbc_pool_poll(self.h, slot)

    def result(self, slot, shape=None):
        """(k, Omega) or, with shape=(nx, ny, nz), (k, Omega, rho, u)."""
        if shape is None:
            return kbc_pool_result(self.h, slot)
        nx, ny, nz = shape
        rho = np.empty((nz, ny, nx))
        u = np.empty((3, nz, ny, nx))
        k, w = kbc_pool_result(self.h, slot, rho, u)
        return k, w, rho, u

    def release(self, slot):
        kbc_pool_release(self.h, slot)

    def sync(self):
        kbc_pool_sync(self.h)

    def info(self) -> dict:
        return kbc_pool_info(self.h)

    def set_launch(self, block, grid, sub=4):
        kbc_pool_set_launch(self.h, block, grid, sub)

    def close(self):
        if getattr(self, "h", None):
            kbc_pool_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def beta_from_nu(nu: float) -> float:
    """beta = 1/(6 nu + 1): the viscosity relation the library applies."""
    return 1.0 / (6.0 * nu + 1.0)


__all__ = [n for n in dir() if n.startswith("kbc_")] + ["Box", "Pool", "KbcError", "load"]
