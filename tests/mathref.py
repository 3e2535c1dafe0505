"""Independent mathematical references used to pin the oracle.

Nothing here is called by the oracle or by the GPU library.  The operators
are assembled a different way from the oracle's loops: as sums of Kronecker
products of 1D shift matrices, c_d * (S_z^dz (x) S_y^dy (x) S_x^dx), which
is the matrix of u -> sum_d c_d u(x+d) on a row-major [nz][ny][nx] grid.
"""
from __future__ import annotations

import numpy as np

STAR, BOX = 0, 1
PERIODIC, ZERO = 0, 1

# Central second-difference weights of order 8 (exact rationals of the
# standard eighth-order finite-difference table).
FD8 = np.array([-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0])


def shift_matrix(n: int, d: int, boundary: int) -> np.ndarray:
    """(S^d u)[i] = u[i+d]: periodic wraps, zero drops indices outside."""
    if boundary == PERIODIC:
        return np.roll(np.eye(n), d, axis=1)
    return np.eye(n, k=d)


def offsets(ndim: int, shape: int, r: int):
    rz = r if ndim == 3 else 0
    out = []
    for dz in range(-rz, rz + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                if shape == BOX or ((dz != 0) + (dy != 0) + (dx != 0)) <= 1:
                    out.append((dz, dy, dx))
    return out


def coeff_at(c: np.ndarray, ndim: int, r: int, dz: int, dy: int, dx: int) -> float:
    w = 2 * r + 1
    rz = r if ndim == 3 else 0
    return float(c[((dz + rz) * w + (dy + r)) * w + (dx + r)])


def operator_matrix(grid_shape, c, shape: int, r: int, boundary: int) -> np.ndarray:
    """Dense matrix of one sweep on a grid of shape [nz,]ny,nx."""
    ndim = len(grid_shape)
    if ndim == 2:
        ny, nx = grid_shape
        nz = 1
    else:
        nz, ny, nx = grid_shape
    size = nz * ny * nx
    M = np.zeros((size, size))
    for dz, dy, dx in offsets(ndim, shape, r):
        cd = coeff_at(c, ndim, r, dz, dy, dx)
        if cd == 0.0:
            continue
        Sz = shift_matrix(nz, dz, boundary) if ndim == 3 else np.eye(1)
        Sy = shift_matrix(ny, dy, boundary)
        Sx = shift_matrix(nx, dx, boundary)
        M += cd * np.kron(Sz, np.kron(Sy, Sx))
    return M


def varcoef_matrix(grid_shape, fields, shape: int, r: int, boundary: int) -> np.ndarray:
    """Dense matrix of one variable-coefficient sweep: sum over the in-shape
    offsets d_k of diag(f_k) times the Kronecker shift matrix of d_k."""
    ndim = len(grid_shape)
    nz, ny, nx = (1,) + tuple(grid_shape) if ndim == 2 else tuple(grid_shape)
    size = nz * ny * nx
    M = np.zeros((size, size))
    for k, (dz, dy, dx) in enumerate(offsets(ndim, shape, r)):
        Sz = shift_matrix(nz, dz, boundary) if ndim == 3 else np.eye(1)
        S = np.kron(Sz, np.kron(shift_matrix(ny, dy, boundary), shift_matrix(nx, dx, boundary)))
        M += np.asarray(fields[k], dtype=np.float64).reshape(size)[:, None] * S
    return M


def laplacian_dense_fd8() -> np.ndarray:
    """Dense 9^3 star array of the 3D eighth-order Laplacian from FD8."""
    r = 4
    W = 9
    d = np.zeros(W ** 3)
    d[(r * W + r) * W + r] = 3 * FD8[0]
    for j in range(1, 5):
        for s in (-1, 1):
            d[((r + s * j) * W + r) * W + r] = FD8[j]
            d[(r * W + r + s * j) * W + r] = FD8[j]
            d[(r * W + r) * W + r + s * j] = FD8[j]
    return d


def lap_zero_numpy(u: np.ndarray) -> np.ndarray:
    """3D eighth-order Laplacian with zero outside, by padding and slicing."""
    p = np.pad(u, 4)
    nz, ny, nx = u.shape
    out = 3 * FD8[0] * u
    for j in range(1, 5):
        w = FD8[j]
        out = out + w * (p[4 + j:4 + j + nz, 4:4 + ny, 4:4 + nx] + p[4 - j:4 - j + nz, 4:4 + ny, 4:4 + nx])
        out = out + w * (p[4:4 + nz, 4 + j:4 + j + ny, 4:4 + nx] + p[4:4 + nz, 4 - j:4 - j + ny, 4:4 + nx])
        out = out + w * (p[4:4 + nz, 4:4 + ny, 4 + j:4 + j + nx] + p[4:4 + nz, 4:4 + ny, 4 - j:4 - j + nx])
    return out


def rel_l2(y, ref) -> float:
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((y - ref).ravel())
    return float(num / den) if den > 0 else float(num)
