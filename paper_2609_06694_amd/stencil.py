"""Python API over libstencil: plans as objects, torch tensors as buffers.

PyTorch supplies device memory and the current stream only.  Every sweep,
adjoint and gradient runs in the library's HIP kernels; there is no CPU or
PyTorch fallback, and a missing library raises on first use.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _abi
from ._abi import check, lib

_DTYPES = {"f32": (_abi.ST_F32, torch.float32), "f16": (_abi.ST_F16, torch.float16),
           "f64": (_abi.ST_F64, torch.float64)}
_BC = {"periodic": _abi.ST_PERIODIC, "zero": _abi.ST_ZERO}
_SHAPES = {"star": _abi.ST_STAR, "box": _abi.ST_BOX}


def _enum(table, v):
    if isinstance(v, str):
        return table[v]
    return int(v)


def _stream_ptr(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _opts(variant=0, tile_x=0, tile_y=0, tsteps=0, zchunk=0, ckpt_every=0):
    return _abi.StPlanOpts(int(variant), int(tile_x), int(tile_y), int(tsteps), int(zchunk),
                           int(ckpt_every))


def _problem(ndim, n, shape, radius, coeffs, dtype, boundary, update, keep):
    c_arr = None
    if coeffs is not None:
        c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float32).ravel())
        keep.append(c)
        c_arr = c.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    n3 = list(n) + [1] * (3 - len(n))
    return _abi.StProblem(int(ndim), (ctypes.c_int64 * 3)(*[int(v) for v in n3]), int(shape),
                          int(radius), c_arr, int(dtype), int(boundary), int(update))


class _Workspace:
    """Grow-only device byte buffer reused across calls of one object."""

    def __init__(self, device):
        self.device = device
        self.buf: Optional[torch.Tensor] = None

    def get(self, nbytes: int) -> Tuple[Optional[ctypes.c_void_p], int]:
        if nbytes == 0:
            return None, 0
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        return ctypes.c_void_p(self.buf.data_ptr()), int(self.buf.numel())


class _Plan:
    def __init__(self):
        self._h = ctypes.c_void_p()

    @property
    def handle(self):
        return self._h

    def describe(self) -> dict:
        return self._describe(lib().stencil_plan_describe)

    def _describe(self, fn) -> dict:
        v, tx, ty, k, zc = (ctypes.c_int32() for _ in range(5))
        check(fn(self._h, ctypes.byref(v), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(k),
                 ctypes.byref(zc)))
        return {"variant": _abi.VARIANT_NAMES.get(v.value, v.value), "tile_x": tx.value,
                "tile_y": ty.value, "tsteps": k.value, "zchunk": zc.value}

    def coefficients(self) -> Tuple[np.ndarray, float]:
        """(dense coefficients the plan applies, weight sum its difference-form
        kernels use); host only."""
        dense = np.zeros(9 ** 3, dtype=np.float32)
        wsum = ctypes.c_double()
        check(lib().stencil_plan_coefficients(self._h, dense.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                               dense.size, ctypes.byref(wsum)))
        return dense, float(wsum.value)

    def workspace_bytes(self, steps: int, mode: int = 0) -> int:
        return int(lib().stencil_workspace_bytes(self._h, int(steps), int(mode)))

    def autotune(self, device="cuda", stream=None) -> dict:
        nbytes = self.workspace_bytes(0, 2)
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=device)
        check(lib().stencil_autotune(self._h, ctypes.c_void_p(scratch.data_ptr()), nbytes,
                                     _stream_ptr(stream)))
        tried, rejected = ctypes.c_int32(), ctypes.c_int32()
        check(lib().stencil_autotune_stats(self._h, ctypes.byref(tried), ctypes.byref(rejected)))
        return {"tried": tried.value, "rejected": rejected.value}

    def close(self):
        if self._h:
            lib().stencil_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stencil(_Plan):
    """A linear constant-coefficient sweep u <- sum_d c_d u(B(x+d)) on one grid."""

    def __init__(self, n: Sequence[int], shape, radius: int, coeffs, dtype: str = "f32",
                 boundary="periodic", **opts):
        super().__init__()
        self.n = tuple(int(v) for v in n)
        self.ndim = len(self.n)
        self.dtype_code, self.torch_dtype = _DTYPES[dtype]
        keep: list = []
        prob = _problem(self.ndim, self.n, _enum(_SHAPES, shape), radius, coeffs, self.dtype_code,
                        _enum(_BC, boundary), _abi.ST_LINEAR, keep)
        o = _opts(**opts) if opts else None
        check(lib().stencil_plan(ctypes.byref(prob), ctypes.byref(o) if o is not None else None,
                                 ctypes.byref(self._h)))
        self.grid_shape = tuple(reversed(self.n))
        self._ws: Optional[_Workspace] = None

    def _check(self, t: torch.Tensor, name: str):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if t.dtype != self.torch_dtype or tuple(t.shape) != self.grid_shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.torch_dtype} tensor of shape {self.grid_shape}")

    def _run(self, fn, u, steps, out, stream):
        self._check(u, "u")
        if out is None:
            out = torch.empty_like(u)
        self._check(out, "out")
        if self._ws is None:
            self._ws = _Workspace(u.device)
        ws, nb = self._ws.get(self.workspace_bytes(steps))
        check(fn(self._h, _ptr(u), _ptr(out), int(steps), None, ws, nb, _stream_ptr(stream)))
        return out

    def apply(self, u: torch.Tensor, steps: int, out: Optional[torch.Tensor] = None, stream=None):
        return self._run(lib().stencil_apply, u, steps, out, stream)

    def apply_adjoint(self, v: torch.Tensor, steps: int, out: Optional[torch.Tensor] = None, stream=None):
        return self._run(lib().stencil_apply_adjoint, v, steps, out, stream)


def varcoef_taps(ndim: int, shape, radius: int) -> int:
    """Number of coefficient fields of a variable-coefficient stencil: one
    per offset of the shape."""
    s = _enum(_SHAPES, shape)
    return (2 * radius + 1) ** ndim if s == _abi.ST_BOX else 1 + 2 * ndim * radius


class VarCoefStencil(_Plan):
    """The sweep u <- sum_k f_k(x) u(B(x + d_k)) with one coefficient field
    per offset d_k of the shape ((dz,dy,dx) order of the in-shape offsets).
    `fields` is a device tensor of shape (taps, nz, ny, nx) in the storage
    type."""

    def __init__(self, n: Sequence[int], shape, radius: int, dtype: str = "f32", boundary="periodic", **opts):
        super().__init__()
        self.n = tuple(int(v) for v in n)
        self.ndim = len(self.n)
        self.dtype_code, self.torch_dtype = _DTYPES[dtype]
        keep: list = []
        prob = _problem(self.ndim, self.n, _enum(_SHAPES, shape), radius, None, self.dtype_code,
                        _enum(_BC, boundary), _abi.ST_VARCOEF, keep)
        o = _opts(**opts) if opts else None
        check(lib().stencil_plan(ctypes.byref(prob), ctypes.byref(o) if o is not None else None,
                                 ctypes.byref(self._h)))
        self.grid_shape = tuple(reversed(self.n))
        self.taps = varcoef_taps(self.ndim, shape, radius)
        self._ws: Optional[_Workspace] = None

    def _check(self, t: torch.Tensor, name: str, shape):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if t.dtype != self.torch_dtype or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.torch_dtype} tensor of shape {shape}")

    def _run(self, fn, u, fields, steps, out, stream):
        self._check(u, "u", self.grid_shape)
        self._check(fields, "fields", (self.taps,) + self.grid_shape)
        if out is None:
            out = torch.empty_like(u)
        self._check(out, "out", self.grid_shape)
        if self._ws is None:
            self._ws = _Workspace(u.device)
        ws, nb = self._ws.get(self.workspace_bytes(steps))
        check(fn(self._h, _ptr(u), _ptr(out), _ptr(fields), int(steps), ws, nb, _stream_ptr(stream)))
        return out

    def apply(self, u: torch.Tensor, fields: torch.Tensor, steps: int, out: Optional[torch.Tensor] = None,
              stream=None):
        return self._run(lib().stencil_apply_varcoef, u, fields, steps, out, stream)

    def apply_adjoint(self, v: torch.Tensor, fields: torch.Tensor, steps: int,
                      out: Optional[torch.Tensor] = None, stream=None):
        return self._run(lib().stencil_apply_varcoef_adjoint, v, fields, steps, out, stream)


class _VarCoefSweepFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, fields, stencil: "VarCoefStencil", steps: int):
        ctx.stencil = stencil
        ctx.steps = steps
        ctx.save_for_backward(fields)
        return stencil.apply(u.contiguous(), fields, steps)

    @staticmethod
    def backward(ctx, g):
        (fields,) = ctx.saved_tensors
        return ctx.stencil.apply_adjoint(g.contiguous(), fields, ctx.steps), None, None, None


def varcoef_sweep(u: torch.Tensor, fields: torch.Tensor, stencil: "VarCoefStencil", steps: int) -> torch.Tensor:
    """Differentiable A^steps u for a variable-coefficient stencil (the
    gradient with respect to u is the transposed sweep; the fields are
    treated as constants)."""
    return _VarCoefSweepFn.apply(u, fields, stencil, steps)


class _SweepFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, stencil: Stencil, steps: int):
        ctx.stencil = stencil
        ctx.steps = steps
        return stencil.apply(u.contiguous(), steps)

    @staticmethod
    def backward(ctx, g):
        return ctx.stencil.apply_adjoint(g.contiguous(), ctx.steps), None, None


def sweep(u: torch.Tensor, stencil: Stencil, steps: int) -> torch.Tensor:
    """Differentiable A^steps u; the backward pass runs the transposed sweep."""
    return _SweepFn.apply(u, stencil, steps)


class WaveModel(_Plan):
    """3D leapfrog u_{t+1} = 2u_t - u_{t-1} + kappa * L(u_t), L a radius-r star
    (default: the order-2r central second-difference Laplacian).

    sponge=(width, strength) adds the absorbing layer: a damping field
    gamma = sum over axes of strength ((width - e) / width)^2 within `width`
    cells of each face, and the step u_{t+1} = A (2u_t + kappa L u_t) -
    B u_{t-1} with A = 1/(1 + gamma/2), B = (1 - gamma/2) A; it applies to
    the forward, adjoint and gradient calls alike.

    dtype="f64" stores every field (state, kappa, wavelet, traces) in
    binary64 and runs the forward leapfrog in binary64; the adjoint and the
    gradient take f32 models only."""

    def __init__(self, n: Sequence[int], radius: int = 4, boundary="zero", coeffs=None, sponge=None,
                 dtype: str = "f32", **opts):
        super().__init__()
        if dtype not in ("f32", "f64"):
            raise ValueError("the wave model stores f32 or f64")
        self.dtype_code, self.torch_dtype = _DTYPES[dtype]
        self.sponge = (0, 0.0) if sponge is None else (int(sponge[0]), float(sponge[1]))
        self.n = tuple(int(v) for v in n)
        keep: list = []
        prob = _problem(3, self.n, _abi.ST_STAR, radius, coeffs, self.dtype_code, _enum(_BC, boundary),
                        _abi.ST_WAVE, keep)
        o = _opts(**opts) if opts else None
        check(lib().stencil_plan(ctypes.byref(prob), ctypes.byref(o) if o is not None else None,
                                 ctypes.byref(self._h)))
        self.grid_shape = tuple(reversed(self.n))
        self._ws: Optional[_Workspace] = None

    def describe_reverse(self) -> dict:
        """Configuration of the adjoint and gradient steps (a map cell of its own)."""
        return self._describe(lib().stencil_plan_describe_reverse)

    def _chk(self, ops):
        """Each (name, tensor, shape, min_len) must be a contiguous device
        tensor of the model's storage type (target: float32) and of that
        shape (or, with min_len, at least that many elements); None passes.
        Shapes and lengths are checked for every operand before any
        placement check."""
        for name, t, shape, min_len in ops:
            if t is None:
                continue
            want = torch.float32 if name == "target" else self.torch_dtype
            if not isinstance(t, torch.Tensor) or t.dtype != want:
                raise ValueError(f"{name} must be a {want} tensor")
            if shape is not None and tuple(t.shape) != tuple(shape):
                raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
            if min_len is not None and t.numel() < min_len:
                raise ValueError(f"{name} must hold at least {min_len} values, got {t.numel()}")
        for name, t, _, _ in ops:
            if t is not None and (not t.is_cuda or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous device tensor")

    def _ops(self, steps, u_prev=None, kappa=None, wavelet=None, traces=None, target=None, **grids):
        g = self.grid_shape
        tr = (int(steps), self.n[1], self.n[0])
        ops = [(k, v, g, None) for k, v in grids.items()]
        ops += [("u_prev", u_prev, g, None), ("kappa", kappa, g, None), ("wavelet", wavelet, None, int(steps)),
                ("traces", traces, tr, None), ("target", target, tr, None)]
        return ops

    def _args(self, u_prev, kappa, src=None, wavelet=None, rec_z=-1, traces=None, target=None):
        if kappa is None:
            raise ValueError("kappa is required")
        s = (-1, -1, -1) if src is None else tuple(int(v) for v in src)
        return _abi.StWaveArgs(_ptr(u_prev), _ptr(kappa), (ctypes.c_int64 * 3)(*s), _ptr(wavelet),
                               int(rec_z), _ptr(traces), _ptr(target), self.sponge[0], self.sponge[1])

    def _workspace(self, device, nbytes):
        if self._ws is None:
            self._ws = _Workspace(device)
        return self._ws.get(nbytes)

    def forward(self, u0, u_prev, kappa, steps: int, src=None, wavelet=None, rec_z: int = -1,
                record: bool = False, out=None, stream=None, prev_inout: bool = False):
        """Returns (u_T, u_{T-1}, traces or None).  u0 is not modified; u_prev
        is copied first unless prev_inout, in which case it is overwritten
        with u_{T-1} and returned."""
        if src is not None and wavelet is None:
            raise ValueError("a source needs a wavelet")
        self._chk(self._ops(steps, u_prev, kappa, wavelet if src is not None else None, u0=u0, out=out))
        prev = u_prev if prev_inout else u_prev.clone()
        out = torch.empty_like(u0) if out is None else out
        traces = None
        if record and rec_z >= 0:
            traces = torch.empty((steps, self.n[1], self.n[0]), dtype=self.torch_dtype, device=u0.device)
        wa = self._args(prev, kappa, src, wavelet, rec_z, traces)
        ws, nb = self._workspace(u0.device, self.workspace_bytes(steps))
        check(lib().stencil_apply(self._h, _ptr(u0), _ptr(out), int(steps), ctypes.byref(wa), ws, nb,
                                  _stream_ptr(stream)))
        return out, prev, traces

    def adjoint(self, a, b, kappa, steps: int, stream=None):
        """Transpose of (u_{-1}, u_0) -> (u_{T-1}, u_T): (a, b) are co-states of
        (u_{T-1}, u_T); returns the co-states of (u_{-1}, u_0)."""
        self._chk(self._ops(steps, kappa=kappa, a=a, b=b))
        a_io = a.clone()
        out = torch.empty_like(b)
        wa = self._args(a_io, kappa)
        ws, nb = self._workspace(b.device, self.workspace_bytes(steps))
        check(lib().stencil_apply_adjoint(self._h, _ptr(b), _ptr(out), int(steps), ctypes.byref(wa), ws,
                                          nb, _stream_ptr(stream)))
        return a_io, out

    def gradient(self, u0, u_prev, kappa, steps: int, src, wavelet, rec_z: int, target,
                 traces: Optional[torch.Tensor] = None, stream=None):
        """(dJ/dkappa, J) with J = 1/2 sum_t ||u_t[rec_z] - target[t-1]||^2."""
        if target is None:
            raise ValueError("the gradient needs a target")
        if src is not None and wavelet is None:
            raise ValueError("a source needs a wavelet")
        if not 0 <= int(rec_z) < self.n[2]:
            raise ValueError(f"rec_z must lie in [0, {self.n[2]})")
        self._chk(self._ops(steps, u_prev, kappa, wavelet if src is not None else None, traces, target, u0=u0))
        dk = torch.empty_like(kappa)
        loss = torch.empty(1, dtype=torch.float64, device=u0.device)
        wa = self._args(u_prev, kappa, src, wavelet, rec_z, traces, target)
        ws, nb = self._workspace(u0.device, self.workspace_bytes(steps, 1))
        check(lib().stencil_wave_gradient(self._h, _ptr(u0), ctypes.byref(wa), int(steps), _ptr(dk),
                                          _ptr(loss), ws, nb, _stream_ptr(stream)))
        return dk, loss


class _WaveMisfitFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, model: WaveModel, u0, u_prev, steps, src, wavelet, rec_z, target):
        dk, loss = model.gradient(u0, u_prev, kappa.contiguous(), steps, src, wavelet, rec_z, target)
        ctx.save_for_backward(dk)
        return loss[0].to(torch.float32)

    @staticmethod
    def backward(ctx, g):
        (dk,) = ctx.saved_tensors
        return dk * g.to(dk.dtype), None, None, None, None, None, None, None, None


def wave_misfit(kappa, model: WaveModel, u0, u_prev, steps, src, wavelet, rec_z, target):
    """Differentiable trace misfit J(kappa); backward returns the adjoint-state
    gradient computed with checkpointing."""
    return _WaveMisfitFn.apply(kappa, model, u0, u_prev, steps, src, wavelet, rec_z, target)


class BatchedStencil(_Plan):
    """Many independent 2D linear sweeps advanced together: one launch per
    time block for the whole batch.  tsteps: the batch depth (default 3),
    or -1 for each member's own map depth."""

    def __init__(self, cases: List[dict], **opts):
        super().__init__()
        keep: list = []
        arr = (_abi.StProblem * len(cases))()
        self.shapes = []
        dts = set()
        for i, c in enumerate(cases):
            code, tdt = _DTYPES[c.get("dtype", "f32")]
            dts.add(tdt)
            arr[i] = _problem(2, c["n"], _enum(_SHAPES, c["shape"]), c["radius"], c["coeffs"], code,
                              _enum(_BC, c.get("boundary", "periodic")), _abi.ST_LINEAR, keep)
            self.shapes.append((int(c["n"][1]), int(c["n"][0])))
        self.torch_dtype = dts.pop() if len(dts) == 1 else None
        o = _opts(**opts) if opts else None
        check(lib().stencil_plan_batched(arr, len(cases), ctypes.byref(o) if o is not None else None,
                                         ctypes.byref(self._h)))
        self._ws: Optional[_Workspace] = None

    def schedule(self, steps: int, cus: int = 0) -> dict:
        """Grouped launches, member tables and workgroups of an apply of
        `steps` steps on a device of `cus` compute units (0: the current
        device's); host only for cus > 0."""
        n, t = ctypes.c_int32(), ctypes.c_int32()
        wg = ctypes.c_int64()
        check(lib().stencil_plan_describe_batched(self._h, int(steps), int(cus), ctypes.byref(n), ctypes.byref(t),
                                                  ctypes.byref(wg)))
        return {"launches": n.value, "tables": t.value, "workgroups": wg.value}

    def apply(self, us: List[torch.Tensor], steps: int, outs: Optional[List[torch.Tensor]] = None,
              stream=None) -> List[torch.Tensor]:
        if len(us) != len(self.shapes):
            raise ValueError("one tensor per batch member is required")
        if outs is not None and len(outs) != len(self.shapes):
            raise ValueError("one output tensor per batch member is required")
        lists = [("member tensors", us)] + ([("member outputs", outs)] if outs is not None else [])
        for what, ts in lists:   # dtypes and shapes first, then placement
            for t, shp in zip(ts, self.shapes):
                if not isinstance(t, torch.Tensor) or t.dtype != self.torch_dtype or tuple(t.shape) != shp:
                    raise ValueError(f"{what} must be {self.torch_dtype} of shape {shp}")
        for what, ts in lists:
            for t in ts:
                if not t.is_cuda or not t.is_contiguous():
                    raise ValueError(f"{what} must be contiguous device tensors")
        if outs is None:
            outs = [torch.empty_like(u) for u in us]
        ins = (ctypes.c_void_p * len(us))(*[u.data_ptr() for u in us])
        ots = (ctypes.c_void_p * len(us))(*[o.data_ptr() for o in outs])
        if self._ws is None:
            self._ws = _Workspace(us[0].device)
        ws, nb = self._ws.get(self.workspace_bytes(steps))
        check(lib().stencil_apply_batched(self._h, ins, ots, int(steps), ws, nb, _stream_ptr(stream)))
        return outs

