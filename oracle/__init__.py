"""FP64 CPU oracle for the stencil sweeps (ctypes binding to ``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  It shares no code
with the GPU path.  Inputs are converted to float64 exactly (float32 and
binary16 values are exactly representable), results are float64.

Pins (tests/test_oracle_pins.py) tie it to the mathematics rather than to
itself: brute-force operator matrices, Fourier symbols, conservation,
polynomial moments, the leapfrog energy invariant and closed form, the
dot-product identity and finite differences.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    from .build_oracle import build_liboracle
    return build_liboracle(force=force)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(LIB_PATH)
    lib.oracle_sweep.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, _dp,
                                 ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.oracle_sweep_adjoint.argtypes = lib.oracle_sweep.argtypes
    lib.oracle_fd2_weights.argtypes = [ctypes.c_int, _dp]
    lib.oracle_laplacian3d.argtypes = [ctypes.c_int, _dp]
    lib.oracle_wave_forward.argtypes = [_i64p, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                        _dp, _dp, _dp, _i64p, _dp, ctypes.c_int64, _dp]
    lib.oracle_wave_adjoint.argtypes = [_i64p, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                        _dp, _dp, _dp]
    lib.oracle_wave_gradient.argtypes = [_i64p, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                         _dp, _dp, _dp, _i64p, _dp, ctypes.c_int64, _dp,
                                         ctypes.c_int, _dp, _dp]
    lib.oracle_varcoef_taps.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_varcoef_sweep.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, _dp,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.oracle_round_storage.argtypes = [_dp, ctypes.c_int64, ctypes.c_int]
    lib.oracle_sweep_stored.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, ctypes.c_int, _dp,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.oracle_wave_forward_stored.argtypes = lib.oracle_wave_forward.argtypes + [ctypes.c_int]
    lib.oracle_wave_gradient_stored.argtypes = lib.oracle_wave_gradient.argtypes + [ctypes.c_int]
    lib.oracle_sponge_profile.argtypes = [_i64p, ctypes.c_int, ctypes.c_double, _dp]
    lib.oracle_wave_forward_damped.argtypes = [_i64p, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                               _dp, _dp, _dp, _dp, _i64p, _dp, ctypes.c_int64, _dp]
    lib.oracle_wave_adjoint_damped.argtypes = [_i64p, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                               _dp, _dp, _dp, _dp]
    lib.oracle_wave_gradient_damped.argtypes = [_i64p, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                                _dp, _dp, _dp, _dp, _i64p, _dp, ctypes.c_int64, _dp,
                                                ctypes.c_int, _dp, _dp]
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _n3(shape: Tuple[int, ...]):
    if len(shape) == 2:
        n = (shape[1], shape[0], 1)
    elif len(shape) == 3:
        n = (shape[2], shape[1], shape[0])
    else:
        raise ValueError("grid must be 2D or 3D")
    return (ctypes.c_int64 * 3)(*n)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")


# Storage formats of the floor diagnostic: every stored state is rounded to
# the format (nearest, ties to even); None means exact FP64.
STORAGE = {None: 0, "binary32": 1, "binary16": 2}


def _storage(name) -> int:
    if name not in STORAGE:
        raise ValueError(f"storage must be one of {sorted(k for k in STORAGE if k)} or None")
    return STORAGE[name]


def round_storage(u, storage) -> np.ndarray:
    """u rounded to the storage format (a float64 copy)."""
    a = _f64(u).copy()
    _check(_load().oracle_round_storage(_ptr(a), a.size, _storage(storage)), "round_storage")
    return a


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def sweep(u: np.ndarray, coeffs: Sequence[float], shape: int, r: int, boundary: int,
          steps: int, adjoint: bool = False, storage=None) -> np.ndarray:
    """`steps` applications of the linear stencil (or its transpose) to u.
    storage="binary16"/"binary32" rounds every step's result to that format
    (the floor diagnostic; forward sweep only)."""
    lib = _load()
    u64 = _f64(u)
    c64 = _f64(coeffs)
    ndim = u64.ndim
    if c64.size != (2 * r + 1) ** ndim:
        raise ValueError("coefficient array must be dense (2r+1)^ndim")
    out = np.empty_like(u64)
    if storage is not None:
        if adjoint:
            raise ValueError("the storage diagnostic covers the forward sweep")
        _check(lib.oracle_sweep_stored(ndim, _n3(u64.shape), shape, r, _ptr(c64), boundary, steps,
                                       _storage(storage), _ptr(u64), _ptr(out)), "sweep_stored")
        return out
    fn = lib.oracle_sweep_adjoint if adjoint else lib.oracle_sweep
    _check(fn(ndim, _n3(u64.shape), shape, r, _ptr(c64), boundary, steps, _ptr(u64), _ptr(out)),
           "sweep")
    return out


def varcoef_taps(ndim: int, shape: int, r: int) -> int:
    """Number of offsets of the shape (one coefficient field each)."""
    k = int(_load().oracle_varcoef_taps(ndim, shape, r))
    if k < 0:
        raise ValueError("bad stencil")
    return k


def varcoef_sweep(u: np.ndarray, fields: np.ndarray, shape: int, r: int, boundary: int,
                  steps: int, adjoint: bool = False) -> np.ndarray:
    """`steps` applications of the variable-coefficient stencil (or its
    transpose); fields[k] is the coefficient field of the k-th in-shape
    offset in (dz,dy,dx) order, shaped like u."""
    lib = _load()
    u64 = _f64(u)
    f64 = _f64(fields)
    ndim = u64.ndim
    nt = varcoef_taps(ndim, shape, r)
    if f64.shape != (nt,) + u64.shape:
        raise ValueError(f"fields must have shape {(nt,) + u64.shape}")
    out = np.empty_like(u64)
    _check(lib.oracle_varcoef_sweep(ndim, _n3(u64.shape), shape, r, _ptr(f64), boundary, steps,
                                    1 if adjoint else 0, _ptr(u64), _ptr(out)), "varcoef_sweep")
    return out


def fd2_weights(r: int) -> np.ndarray:
    w = np.empty(r + 1, dtype=np.float64)
    _check(_load().oracle_fd2_weights(r, _ptr(w)), "fd2_weights")
    return w


def laplacian3d(r: int = 4) -> np.ndarray:
    d = np.empty((2 * r + 1) ** 3, dtype=np.float64)
    _check(_load().oracle_laplacian3d(r, _ptr(d)), "laplacian3d")
    return d


def wave_forward(u_prev, u0, kappa, steps: int, r: int = 4, boundary: int = 1,
                 lap: Optional[np.ndarray] = None, src=None, wavelet=None,
                 rec_z: int = -1, storage=None):
    """Leapfrog forward.  Returns (u_{T-1}, u_T, traces or None).
    storage="binary32"/"binary16" rounds every new state (floor diagnostic)."""
    lib = _load()
    a = _f64(u_prev).copy()
    b = _f64(u0).copy()
    k = _f64(kappa)
    lp = _f64(laplacian3d(r) if lap is None else lap)
    nz, ny, nx = b.shape
    srcp = (ctypes.c_int64 * 3)(*src) if src is not None else None
    wv = _f64(wavelet) if wavelet is not None else None
    traces = np.zeros((steps, ny, nx), dtype=np.float64) if rec_z >= 0 else None
    args = (_n3(b.shape), r, _ptr(lp), boundary, steps, _ptr(k), _ptr(a), _ptr(b), srcp,
            _ptr(wv) if wv is not None else None, rec_z, _ptr(traces) if traces is not None else None)
    if storage is None:
        _check(lib.oracle_wave_forward(*args), "wave_forward")
    else:
        _check(lib.oracle_wave_forward_stored(*args, _storage(storage)), "wave_forward_stored")
    return a, b, traces


def wave_adjoint(a_in, b_in, kappa, steps: int, r: int = 4, boundary: int = 1,
                 lap: Optional[np.ndarray] = None):
    """Transpose of (u_{-1}, u_0) -> (u_{T-1}, u_T).  (a, b) are the co-states
    of (u_{T-1}, u_T); returns the co-states of (u_{-1}, u_0)."""
    lib = _load()
    a = _f64(a_in).copy()
    b = _f64(b_in).copy()
    k = _f64(kappa)
    lp = _f64(laplacian3d(r) if lap is None else lap)
    _check(lib.oracle_wave_adjoint(_n3(b.shape), r, _ptr(lp), boundary, steps, _ptr(k),
                                   _ptr(a), _ptr(b)), "wave_adjoint")
    return a, b


def wave_gradient(u_prev0, u0, kappa, steps: int, src, wavelet, rec_z: int, target,
                  ckpt_every: int = 0, r: int = 4, boundary: int = 1,
                  lap: Optional[np.ndarray] = None, storage=None):
    """(dJ/dkappa, J) for J = 1/2 sum_t ||u_t[rec_z] - target[t-1]||^2.
    storage="binary32" rounds every stored state, co-state and the running
    gradient (floor diagnostic)."""
    lib = _load()
    k = _f64(kappa)
    up = _f64(u_prev0)
    u = _f64(u0)
    lp = _f64(laplacian3d(r) if lap is None else lap)
    tg = _f64(target)
    wv = _f64(wavelet)
    grad = np.empty_like(k)
    loss = ctypes.c_double(0.0)
    srcp = (ctypes.c_int64 * 3)(*src) if src is not None else None
    args = (_n3(k.shape), r, _ptr(lp), boundary, steps, _ptr(k), _ptr(up), _ptr(u), srcp, _ptr(wv),
            rec_z, _ptr(tg), ckpt_every, _ptr(grad), ctypes.byref(loss))
    if storage is None:
        _check(lib.oracle_wave_gradient(*args), "wave_gradient")
    else:
        _check(lib.oracle_wave_gradient_stored(*args, _storage(storage)), "wave_gradient_stored")
    return grad, float(loss.value)


def sponge_profile(shape, width: int, strength: float) -> np.ndarray:
    """Damping field gamma of the absorbing layer on a grid of array shape
    (nz, ny, nx): a quadratic ramp of `width` cells along every face."""
    g = np.empty(tuple(shape), dtype=np.float64)
    _check(_load().oracle_sponge_profile(_n3(g.shape), int(width), float(strength), _ptr(g)), "sponge_profile")
    return g


def wave_forward_damped(u_prev, u0, kappa, gamma, steps: int, r: int = 4, boundary: int = 1,
                        lap: Optional[np.ndarray] = None, src=None, wavelet=None, rec_z: int = -1):
    """Damped leapfrog (absorbing layer with damping field gamma).  Returns
    (u_{T-1}, u_T, traces or None)."""
    lib = _load()
    a = _f64(u_prev).copy()
    b = _f64(u0).copy()
    k = _f64(kappa)
    gm = _f64(gamma)
    lp = _f64(laplacian3d(r) if lap is None else lap)
    nz, ny, nx = b.shape
    srcp = (ctypes.c_int64 * 3)(*src) if src is not None else None
    wv = _f64(wavelet) if wavelet is not None else None
    traces = np.zeros((steps, ny, nx), dtype=np.float64) if rec_z >= 0 else None
    _check(lib.oracle_wave_forward_damped(_n3(b.shape), r, _ptr(lp), boundary, steps, _ptr(k), _ptr(gm),
                                          _ptr(a), _ptr(b), srcp, _ptr(wv) if wv is not None else None, rec_z,
                                          _ptr(traces) if traces is not None else None), "wave_forward_damped")
    return a, b, traces


def wave_adjoint_damped(a_in, b_in, kappa, gamma, steps: int, r: int = 4, boundary: int = 1,
                        lap: Optional[np.ndarray] = None):
    """Transpose of the damped state map (u_{-1}, u_0) -> (u_{T-1}, u_T)."""
    lib = _load()
    a = _f64(a_in).copy()
    b = _f64(b_in).copy()
    k = _f64(kappa)
    gm = _f64(gamma)
    lp = _f64(laplacian3d(r) if lap is None else lap)
    _check(lib.oracle_wave_adjoint_damped(_n3(b.shape), r, _ptr(lp), boundary, steps, _ptr(k), _ptr(gm),
                                          _ptr(a), _ptr(b)), "wave_adjoint_damped")
    return a, b


def wave_gradient_damped(u_prev0, u0, kappa, gamma, steps: int, src, wavelet, rec_z: int, target,
                         ckpt_every: int = 0, r: int = 4, boundary: int = 1, lap: Optional[np.ndarray] = None):
    """(dJ/dkappa, J) for the damped leapfrog."""
    lib = _load()
    k = _f64(kappa)
    gm = _f64(gamma)
    up = _f64(u_prev0)
    u = _f64(u0)
    lp = _f64(laplacian3d(r) if lap is None else lap)
    tg = _f64(target)
    wv = _f64(wavelet)
    grad = np.empty_like(k)
    loss = ctypes.c_double(0.0)
    srcp = (ctypes.c_int64 * 3)(*src) if src is not None else None
    _check(lib.oracle_wave_gradient_damped(_n3(k.shape), r, _ptr(lp), boundary, steps, _ptr(k), _ptr(gm), _ptr(up),
                                           _ptr(u), srcp, _ptr(wv), rec_z, _ptr(tg), ckpt_every, _ptr(grad),
                                           ctypes.byref(loss)), "wave_gradient_damped")
    return grad, float(loss.value)
