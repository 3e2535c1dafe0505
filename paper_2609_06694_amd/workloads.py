"""Seeded synthetic inputs for the stencil workloads.

This module only draws inputs: grids, coefficient sets, material fields,
source wavelets.  It holds none of the stencil arithmetic, so both the GPU
library and the FP64 CPU oracle can consume exactly the same stored values.

Every generator uses numpy's PCG64 (``numpy.random.default_rng(seed)``) and
rounds draws made in float64 to the storage type with round-to-nearest-even.
Coefficients are always float32; grid values are float32 or binary16.

Layout convention shared by every consumer: row-major with x unit-stride,
2D arrays are ``[ny, nx]``, 3D arrays are ``[nz, ny, nx]``; the dense
coefficient array has ``(2r+1)**ndim`` entries ordered ``(dz, dy, dx)``
lexicographically with dx fastest (Section 2.1 defines a stencil as the pair
of offset set and coefficients).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

STAR, BOX = 0, 1
PERIODIC, ZERO = 0, 1
LINEAR, WAVE = 0, 1
F32, F16, F64 = 0, 1, 2

SHAPE_NAMES = {STAR: "star", BOX: "box"}
DTYPE_NP = {F32: np.float32, F16: np.float16, F64: np.float64}
DTYPE_TAGS = {F32: "f32", F16: "f16", F64: "f64"}

# Seeds fixed per workload so every run and every consumer sees the same draw.
SEED_JACOBI2D = 1
SEED_WAVE3D = 2
SEED_BOX = 3
SEED_BATCH = 4
SEED_WAVEGRAD = 5


@dataclass
class LinearCase:
    """One linear constant-coefficient sweep: u^{t+1}(x) = sum_d c_d u^t(x+d)."""
    name: str
    ndim: int
    n: Tuple[int, int, int]          # (nx, ny, nz); nz = 1 in 2D
    shape: int
    radius: int
    coeffs: np.ndarray               # float32, (2r+1)**ndim dense
    boundary: int
    steps: int
    u0: np.ndarray                   # float32 or float16, [nz,]ny,nx
    dtype: int = F32

    @property
    def cells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclass
class WaveCase:
    """Acoustic leapfrog: u_{t+1} = 2 u_t - u_{t-1} + kappa * L(u_t)."""
    name: str
    n: Tuple[int, int, int]
    radius: int
    boundary: int
    steps: int
    kappa: np.ndarray                # float32 [nz, ny, nx]
    u0: np.ndarray                   # float32, state at t = 0
    u_prev: np.ndarray               # float32, state at t = -1
    src: Optional[Tuple[int, int, int]] = None   # (x, y, z) of the point source
    wavelet: Optional[np.ndarray] = None         # float32 [steps]; added to u_{t+1}
    rec_z: int = -1                              # receiver plane index, -1 = none
    target: Optional[np.ndarray] = None          # float32 [steps, ny, nx]
    kappa_true: Optional[np.ndarray] = None      # perturbed model the target is made from
    ckpt_every: int = 20

    @property
    def cells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


def offsets_in_shape(ndim: int, shape: int, r: int):
    """Offsets (dz, dy, dx) of the star or box of radius r, lexicographic."""
    rz = r if ndim == 3 else 0
    out = []
    for dz in range(-rz, rz + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                nonzero = (dz != 0) + (dy != 0) + (dx != 0)
                if shape == BOX or nonzero <= 1:
                    out.append((dz, dy, dx))
    return out


def dense_index(ndim: int, r: int, dz: int, dy: int, dx: int) -> int:
    w = 2 * r + 1
    rz = r if ndim == 3 else 0
    return ((dz + rz) * w + (dy + r)) * w + (dx + r)


def random_unit_sum_coeffs(rng: np.random.Generator, ndim: int, shape: int, r: int) -> np.ndarray:
    """Draw U[0,1) for each offset of the shape in lexicographic order,
    normalise by the float64 sum, round to float32; off-shape entries are 0."""
    offs = offsets_in_shape(ndim, shape, r)
    draw = rng.random(len(offs))
    draw = draw / draw.sum()
    c = np.zeros((2 * r + 1) ** ndim, dtype=np.float32)
    for (dz, dy, dx), v in zip(offs, draw):
        c[dense_index(ndim, r, dz, dy, dx)] = np.float32(v)
    return c


def _uniform(rng, lo, hi, shape, dtype):
    """U[lo,hi) drawn in float64 slab by slab (bounded temporaries), rounded
    to dtype with round-to-nearest-even."""
    out = np.empty(shape, dtype=dtype)
    if len(shape) == 3 and shape[0] > 1:
        for z in range(shape[0]):
            out[z] = (lo + (hi - lo) * rng.random(shape[1:])).astype(dtype)
    else:
        out[...] = (lo + (hi - lo) * rng.random(shape)).astype(dtype)
    return out


def _grid_shape(ndim, n):
    return (n[1], n[0]) if ndim == 2 else (n[2], n[1], n[0])


# --------------------------------------------------------------------------
# Workload 1: 2D 5-point Jacobi, periodic.
# --------------------------------------------------------------------------
def jacobi2d(n: int = 512, steps: int = 10, seed: int = SEED_JACOBI2D) -> LinearCase:
    rng = np.random.default_rng(seed)
    c = np.zeros(9, dtype=np.float32)
    c[dense_index(2, 1, 0, 0, 0)] = 0.5
    for dy, dx in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        c[dense_index(2, 1, 0, dy, dx)] = 0.125
    u0 = _uniform(rng, -1.0, 1.0, (n, n), np.float32)
    return LinearCase("jacobi2d_star1", 2, (n, n, 1), STAR, 1, c, PERIODIC, steps, u0, F32)


# --------------------------------------------------------------------------
# Workload 2: 3D acoustic leapfrog, radius-4 Laplacian, zero frame.
# --------------------------------------------------------------------------
def gaussian_pulse(n: Tuple[int, int, int], center, sigma: float) -> np.ndarray:
    """exp(-|x-c|^2 / (2 sigma^2)) as a product of 1D factors, float32."""
    nx, ny, nz = n
    gx = np.exp(-((np.arange(nx) - center[0]) ** 2) / (2.0 * sigma * sigma))
    gy = np.exp(-((np.arange(ny) - center[1]) ** 2) / (2.0 * sigma * sigma))
    gz = np.exp(-((np.arange(nz) - center[2]) ** 2) / (2.0 * sigma * sigma))
    out = np.empty((nz, ny, nx), dtype=np.float32)
    gyx = gy[:, None] * gx[None, :]
    for z in range(nz):
        out[z] = (gz[z] * gyx).astype(np.float32)
    return out


def wave3d(n: int = 512, steps: int = 20, seed: int = SEED_WAVE3D,
           kappa_lo: float = 0.05, kappa_hi: float = 0.2, sigma: float = 8.0) -> WaveCase:
    rng = np.random.default_rng(seed)
    shp = (n, n, n)
    kappa = _uniform(rng, kappa_lo, kappa_hi, shp, np.float32)
    u0 = gaussian_pulse(shp, (n // 2, n // 2, n // 2), sigma)
    return WaveCase("wave3d_star4", shp, 4, ZERO, steps, kappa, u0, u0.copy())


# --------------------------------------------------------------------------
# Workload 3: box stencils, fp16 storage with an f32 twin.
# --------------------------------------------------------------------------
def box3d(n: int = 512, steps: int = 50, dtype: int = F16, seed: int = SEED_BOX) -> LinearCase:
    rng = np.random.default_rng(seed)
    c = random_unit_sum_coeffs(rng, 3, BOX, 1)
    u0 = _uniform(rng, 0.0, 1.0, (n, n, n), DTYPE_NP[dtype])
    return LinearCase(f"box3d_r1_{DTYPE_TAGS[dtype]}", 3, (n, n, n), BOX, 1, c, PERIODIC, steps, u0, dtype)


def box2d(n: int = 4096, steps: int = 100, dtype: int = F16, seed: int = SEED_BOX + 10) -> LinearCase:
    rng = np.random.default_rng(seed)
    c = random_unit_sum_coeffs(rng, 2, BOX, 2)
    u0 = _uniform(rng, 0.0, 1.0, (n, n), DTYPE_NP[dtype])
    return LinearCase(f"box2d_r2_{DTYPE_TAGS[dtype]}", 2, (n, n, 1), BOX, 2, c, PERIODIC, steps, u0, dtype)


def star3d(n=(512, 512, 512), r: int = 1, steps: int = 10, dtype: int = F32, seed: int = SEED_BOX + 30) -> LinearCase:
    """A 3D star of radius r (r = 1: the 7-point star of the paper's kernel
    matrix) on an nx x ny x nz grid; unit-sum coefficients, U[0,1) data,
    periodic boundaries."""
    rng = np.random.default_rng(seed)
    c = random_unit_sum_coeffs(rng, 3, STAR, r)
    nx, ny, nz = n
    u0 = _uniform(rng, 0.0, 1.0, (nz, ny, nx), DTYPE_NP[dtype])
    return LinearCase(f"star3d_r{r}_{DTYPE_TAGS[dtype]}", 3, (nx, ny, nz), STAR, r, c, PERIODIC, steps, u0, dtype)


def box3d_r2(n: int = 512, steps: int = 10, dtype: int = F32, seed: int = SEED_BOX + 20) -> LinearCase:
    """The 125-point 3D box (radius 2), the compute-bound corner of the
    paper's kernel matrix (Sections 4.3 and 7.2.3): same coefficient and data law as the
    27-point box."""
    rng = np.random.default_rng(seed)
    c = random_unit_sum_coeffs(rng, 3, BOX, 2)
    u0 = _uniform(rng, 0.0, 1.0, (n, n, n), DTYPE_NP[dtype])
    return LinearCase(f"box3d_r2_{DTYPE_TAGS[dtype]}", 3, (n, n, n), BOX, 2, c, PERIODIC, steps, u0, dtype)


# --------------------------------------------------------------------------
# Workload 4: 64 uneven 2D grids with mixed stencils.
# --------------------------------------------------------------------------
BATCH_KINDS = [(STAR, 1), (STAR, 2), (STAR, 3), (STAR, 4), (BOX, 1), (BOX, 2)]


def batch2d(count: int = 64, lo: int = 256, hi: int = 2048, steps: int = 32,
            seed: int = SEED_BATCH) -> List[LinearCase]:
    """Per grid, in order: nx, ny log-uniform in [lo, hi]; stencil kind
    uniform over star r=1..4, box r=1..2; unit-sum coefficients; u0 ~ U[0,1)."""
    rng = np.random.default_rng(seed)
    cases = []
    for g in range(count):
        nx = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        ny = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        shape, r = BATCH_KINDS[int(rng.integers(len(BATCH_KINDS)))]
        c = random_unit_sum_coeffs(rng, 2, shape, r)
        u0 = _uniform(rng, 0.0, 1.0, (ny, nx), np.float32)
        cases.append(LinearCase(f"batch{g:02d}_{SHAPE_NAMES[shape]}{r}_{nx}x{ny}", 2,
                                (nx, ny, 1), shape, r, c, PERIODIC, steps, u0, F32))
    return cases


# --------------------------------------------------------------------------
# Workload 5: gradient of the 3D wave model with respect to kappa.
# --------------------------------------------------------------------------
def ricker(steps: int, period: float) -> np.ndarray:
    """Ricker wavelet w(t) = (1 - 2 pi^2 f^2 (t-t0)^2) exp(-pi^2 f^2 (t-t0)^2),
    f = 1/period, t0 = period, sampled at t = 1..steps (entry t-1 is the
    amplitude added to u_t)."""
    f = 1.0 / period
    t = np.arange(1, steps + 1, dtype=np.float64)
    a = (math.pi * f * (t - period)) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def wavegrad3d(n: int = 256, steps: int = 200, seed: int = SEED_WAVEGRAD,
               kappa_lo: float = 0.05, kappa_hi: float = 0.19, ckpt_every: int = 20,
               src_z: int = 16, rec_z: int = 8, blob_z: int = 40, blob_sigma: float = 8.0,
               wavelength_cells: float = 15.0) -> WaveCase:
    """Inputs of the gradient workload.  The target traces are NOT drawn here:
    they are the forward model's output at ``kappa_true`` and are produced by
    whichever consumer needs them (the oracle in the tests)."""
    rng = np.random.default_rng(seed)
    shp = (n, n, n)
    kappa = _uniform(rng, kappa_lo, kappa_hi, shp, np.float32)
    blob = gaussian_pulse(shp, (n // 2, n // 2, blob_z), blob_sigma)
    kappa_true = (kappa.astype(np.float64) * (1.0 + 0.05 * blob.astype(np.float64))).astype(np.float32)
    mean_speed = math.sqrt(0.5 * (kappa_lo + kappa_hi))
    period = wavelength_cells / mean_speed
    wav = ricker(steps, period)
    zeros = np.zeros((n, n, n), dtype=np.float32)
    return WaveCase("wavegrad3d_star4", shp, 4, ZERO, steps, kappa, zeros, zeros.copy(),
                    src=(n // 2, n // 2, src_z), wavelet=wav, rec_z=rec_z,
                    target=None, kappa_true=kappa_true, ckpt_every=ckpt_every)


def varcoef_fields(rng: np.random.Generator, taps: int, grid_shape, dtype=np.float32) -> np.ndarray:
    """Coefficient fields of a variable-coefficient stencil: per cell, taps
    draws U[0,1) normalised by their FP64 sum (a cell-wise unit-sum average,
    so repeated sweeps stay bounded), rounded to the storage type.  Shape
    (taps,) + grid_shape."""
    f = rng.random((taps,) + tuple(grid_shape))
    f /= f.sum(axis=0, keepdims=True)
    return f.astype(dtype)


def small_random_grid(rng: np.random.Generator, ndim: int, n, dtype=np.float32, lo=-1.0, hi=1.0):
    """Small grid for parity tests: U[lo,hi) rounded to dtype."""
    return _uniform(rng, lo, hi, _grid_shape(ndim, n), dtype)
