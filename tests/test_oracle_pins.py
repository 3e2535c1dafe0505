"""Pins of the FP64 oracle against mathematics (CPU only).

Each test checks the oracle against something other than itself: an
operator matrix assembled from Kronecker products of shift matrices,
Fourier symbols, conservation of the sum, polynomial moments, the
leapfrog's discrete energy and closed-form mode solution, the dot-product
identity of a transpose, and finite differences of the loss.  A dropped
term, a wrong sign, a flipped offset or a transposed operand in the oracle
fails at least one of them.
"""
import math

import numpy as np
import pytest

import mathref as mr
from paper_2609_06694_amd import workloads as wl

STAR, BOX, PERIODIC, ZERO = mr.STAR, mr.BOX, mr.PERIODIC, mr.ZERO


def _rand_coeffs(rng, ndim, shape, r):
    c = np.zeros((2 * r + 1) ** ndim)
    for dz, dy, dx in mr.offsets(ndim, shape, r):
        w = 2 * r + 1
        rz = r if ndim == 3 else 0
        c[((dz + rz) * w + dy + r) * w + dx + r] = rng.uniform(-1, 1)
    return c


# Tiny grids, including sizes below 2r+1 where periodic wraps overlap.
BRUTE_CASES = [
    (2, (5, 7), STAR, 1), (2, (6, 5), STAR, 2), (2, (4, 9), STAR, 4), (2, (7, 6), BOX, 1),
    (2, (5, 8), BOX, 2), (2, (3, 3), BOX, 2), (3, (4, 5, 6), STAR, 1), (3, (5, 4, 3), BOX, 1),
    (3, (3, 4, 9), STAR, 4), (3, (6, 6, 6), STAR, 2), (3, (4, 6, 5), BOX, 2),
]


@pytest.mark.parametrize("boundary", [PERIODIC, ZERO])
@pytest.mark.parametrize("ndim,shape_,kind,r", BRUTE_CASES)
def test_sweep_matches_brute_force_matrix(oracle_lib, ndim, shape_, kind, r, boundary):
    rng = np.random.default_rng(hash((ndim, shape_, kind, r, boundary)) % 2**32)
    c = _rand_coeffs(rng, ndim, kind, r)
    u = rng.standard_normal(shape_)
    M = mr.operator_matrix(shape_, c, kind, r, boundary)
    steps = 3
    ref = np.linalg.matrix_power(M, steps) @ u.ravel()
    got = oracle_lib.sweep(u, c, kind, r, boundary, steps)
    assert np.max(np.abs(got.ravel() - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    # the transpose: flipped offsets, same boundary
    refT = np.linalg.matrix_power(M.T, steps) @ u.ravel()
    gotT = oracle_lib.sweep(u, c, kind, r, boundary, steps, adjoint=True)
    assert np.max(np.abs(gotT.ravel() - refT)) <= 1e-12 * max(1.0, np.max(np.abs(refT)))


def test_zero_steps_is_identity(oracle_lib):
    u = np.random.default_rng(1).standard_normal((4, 5))
    c = np.ones(9)
    assert np.array_equal(oracle_lib.sweep(u, c, BOX, 1, PERIODIC, 0), u)


def test_jacobi_sine_mode_decays_by_symbol(oracle_lib):
    """The 2D Jacobi workload's stencil (centre 1/2, neighbours 1/8) has the
    symbol 1/2 + (cos kx + cos ky)/4; a mode with kx = pi/2, ky = 0 on a
    512-periodic grid is scaled by exactly 0.75 per step."""
    case = wl.jacobi2d(n=512, steps=10)
    x = np.arange(512)
    u = np.tile(np.sin(2 * math.pi * 128 * x / 512 + 0.3), (512, 1))
    got = oracle_lib.sweep(u, case.coeffs, STAR, 1, PERIODIC, case.steps)
    assert np.max(np.abs(got - 0.75 ** 10 * u)) < 1e-13


@pytest.mark.parametrize("ndim,kind,r,n", [(2, BOX, 2, (12, 10)), (3, BOX, 1, (8, 6, 10)),
                                           (3, STAR, 3, (7, 9, 8)), (2, STAR, 4, (11, 13)),
                                           (3, BOX, 2, (9, 7, 10))])
def test_fourier_symbol_general(oracle_lib, ndim, kind, r, n):
    """e^{i k.x} is an eigenvector of a periodic sweep with eigenvalue
    sum_d c_d e^{i k.d}; the real part of lambda^T e^{i k.x} is the result."""
    rng = np.random.default_rng(7)
    c = _rand_coeffs(rng, ndim, kind, r)
    grids = np.meshgrid(*[np.arange(m) for m in n], indexing="ij")
    ks = [2 * math.pi * rng.integers(0, m) / m for m in n]
    phase = sum(k * g for k, g in zip(ks, grids))
    lam = 0j
    for dz, dy, dx in mr.offsets(ndim, kind, r):
        d = (dy, dx) if ndim == 2 else (dz, dy, dx)
        lam += mr.coeff_at(c, ndim, r, dz, dy, dx) * np.exp(1j * sum(k * dd for k, dd in zip(ks, d)))
    T = 4
    u0 = np.cos(phase)
    want = np.real(lam ** T * np.exp(1j * phase))
    got = oracle_lib.sweep(u0, c, kind, r, PERIODIC, T)
    assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, abs(lam) ** T)


@pytest.mark.parametrize("ndim,kind,r", [(2, STAR, 1), (2, BOX, 2), (3, BOX, 1), (3, STAR, 4), (3, BOX, 2)])
def test_sum_conservation_periodic(oracle_lib, ndim, kind, r):
    """Under periodic boundaries sum(u^T) = s^T sum(u^0), s = sum of coefficients."""
    rng = np.random.default_rng(3)
    c = wl.random_unit_sum_coeffs(rng, ndim, kind, r).astype(np.float64)
    s = float(c.sum())
    shape_ = (33, 40) if ndim == 2 else (12, 11, 13)
    u = rng.random(shape_)
    T = 7
    got = oracle_lib.sweep(u, c, kind, r, PERIODIC, T)
    assert abs(got.sum() - s ** T * u.sum()) < 1e-11 * u.size


@pytest.mark.parametrize("ndim,kind,r", [(2, BOX, 2), (3, STAR, 2), (3, BOX, 1), (3, BOX, 2)])
def test_polynomial_moments_zero_boundary(oracle_lib, ndim, kind, r):
    """Away from the edges, sum_d c_d p(x+d) = sum_alpha m_alpha D^alpha p(x)/alpha!
    with m_alpha = sum_d c_d d^alpha; checked for a quadratic p."""
    rng = np.random.default_rng(11)
    c = _rand_coeffs(rng, ndim, kind, r)
    shape_ = (20, 22) if ndim == 2 else (14, 15, 16)
    grids = np.meshgrid(*[np.arange(m, dtype=np.float64) for m in shape_], indexing="ij")
    A = rng.standard_normal((ndim, ndim))
    A = A + A.T
    b = rng.standard_normal(ndim)
    c0 = rng.standard_normal()
    X = np.stack(grids, axis=-1)
    p = 0.5 * np.einsum("...i,ij,...j->...", X, A, X) + X @ b + c0
    offs = mr.offsets(ndim, kind, r)
    m0 = 0.0
    m1 = np.zeros(ndim)
    m2 = np.zeros((ndim, ndim))
    for dz, dy, dx in offs:
        d = np.array((dy, dx) if ndim == 2 else (dz, dy, dx), dtype=np.float64)
        cd = mr.coeff_at(c, ndim, r, dz, dy, dx)
        m0 += cd
        m1 += cd * d
        m2 += cd * np.outer(d, d)
    grad = X @ A + b
    want = m0 * p + grad @ m1 + 0.5 * np.sum(A * m2)
    got = oracle_lib.sweep(p, c, kind, r, ZERO, 1)
    sl = tuple(slice(r, m - r) for m in shape_)
    assert np.max(np.abs(got[sl] - want[sl])) < 1e-9 * np.max(np.abs(want[sl]))


def test_fd8_weights_closed_form_and_exactness(oracle_lib):
    w = oracle_lib.fd2_weights(4)
    assert np.max(np.abs(w - mr.FD8)) < 1e-13
    full = np.concatenate([w[:0:-1], w])
    j = np.arange(-4, 5, dtype=np.float64)
    for x in (0.0, 0.37, -1.5):
        for k in range(0, 10):
            exact = k * (k - 1) * x ** (k - 2) if k >= 2 else 0.0
            assert abs(np.sum(full * (x + j) ** k) - exact) < 1e-7 * max(1.0, abs(x) ** k * 10 ** k)
    # degree 10 is where the eighth-order formula first fails: -1152 at x = 0
    assert abs(np.sum(full * j ** 10) - (-1152.0)) < 1e-8
    # lower orders reduce to the textbook three- and five-point formulas
    assert np.allclose(oracle_lib.fd2_weights(1), [-2.0, 1.0], atol=1e-15)
    assert np.allclose(oracle_lib.fd2_weights(2), [-2.5, 4.0 / 3.0, -1.0 / 12.0], atol=1e-14)


def test_laplacian3d_layout(oracle_lib):
    assert np.max(np.abs(oracle_lib.laplacian3d(4) - mr.laplacian_dense_fd8())) < 1e-13


def _wave_case_small(rng, n=(6, 6, 6)):
    nz, ny, nx = n
    kappa = rng.uniform(0.05, 0.2, n)
    u0 = rng.standard_normal(n)
    up = rng.standard_normal(n)
    return kappa, up, u0


def test_wave_forward_brute_force(oracle_lib):
    """Leapfrog with dense matrices: u_{t+1} = 2u - u_prev + K M u, source and
    receiver plane, against the oracle on a 6^3 grid (5 steps)."""
    rng = np.random.default_rng(5)
    n = (6, 7, 5)
    kappa, up, u0 = _wave_case_small(rng, n)
    M = mr.operator_matrix(n, mr.laplacian_dense_fd8(), STAR, 4, ZERO)
    K = np.diag(kappa.ravel())
    src = (2, 3, 1)   # (x, y, z)
    wav = rng.standard_normal(5)
    a, b = up.ravel().copy(), u0.ravel().copy()
    traces = []
    for t in range(5):
        c = 2 * b - a + K @ (M @ b)
        c[(src[2] * n[1] + src[1]) * n[2] + src[0]] += wav[t]
        traces.append(c.reshape(n)[3].copy())
        a, b = b, c
    ga, gb, tr = oracle_lib.wave_forward(up, u0, kappa, 5, src=src, wavelet=wav, rec_z=3)
    assert np.max(np.abs(gb.ravel() - b)) < 1e-11 * np.max(np.abs(b))
    assert np.max(np.abs(ga.ravel() - a)) < 1e-11 * np.max(np.abs(a))
    assert np.max(np.abs(tr - np.array(traces))) < 1e-11 * np.max(np.abs(traces))


def test_wave_energy_invariant(oracle_lib):
    """E = ||u_{t+1}-u_t||^2_{1/kappa} - <u_{t+1}, L u_t> is conserved exactly
    by the leapfrog with a symmetric L (no source)."""
    rng = np.random.default_rng(9)
    n = (16, 14, 15)
    kappa = rng.uniform(0.05, 0.2, n)
    u0 = wl.gaussian_pulse((15, 14, 16), (7, 7, 8), 2.0).astype(np.float64)
    up = u0 * 0.99

    def energy(prev, cur):
        return np.sum((cur - prev) ** 2 / kappa) - np.sum(cur * mr.lap_zero_numpy(prev))

    e0 = energy(up, u0)
    a, b = up, u0
    for _ in range(6):
        a, b, _tr = oracle_lib.wave_forward(a, b, kappa, 5)
        e = energy(a, b)
        assert abs(e - e0) <= 1e-12 * abs(e0) + 1e-13


def test_wave_closed_form_constant_kappa(oracle_lib):
    """Constant kappa, periodic, mode cos(k x) with u_{-1} = u_0: the amplitude
    is cos(theta (t+1/2)) / cos(theta/2), cos theta = 1 + kappa lambda / 2,
    lambda = w0 + 2 sum_j w_j cos(j k)."""
    n = (6, 5, 32)  # nz, ny, nx
    kx = 2 * math.pi * 3 / 32
    lam = mr.FD8[0] + 2 * sum(mr.FD8[j] * math.cos(j * kx) for j in range(1, 5))
    kap = 0.15
    theta = math.acos(1 + kap * lam / 2)
    x = np.arange(32)
    u0 = np.broadcast_to(np.cos(kx * x), n).copy()
    kappa = np.full(n, kap)
    T = 37
    _a, b, _tr = oracle_lib.wave_forward(u0, u0, kappa, T, boundary=PERIODIC)
    amp = math.cos(theta * (T + 0.5)) / math.cos(theta / 2)
    assert np.max(np.abs(b - amp * u0)) < 1e-12


def test_wave_adjoint_dot_product(oracle_lib):
    """<F(p,q), (a,b)> = <(p,q), F^T(a,b)> for the leapfrog state map."""
    rng = np.random.default_rng(13)
    n = (9, 8, 10)
    kappa, p, q = _wave_case_small(rng, n)
    a, b = rng.standard_normal(n), rng.standard_normal(n)
    fp, fq, _ = oracle_lib.wave_forward(p, q, kappa, 7)
    ta, tb = oracle_lib.wave_adjoint(a, b, kappa, 7)
    lhs = np.sum(fp * a) + np.sum(fq * b)
    rhs = np.sum(p * ta) + np.sum(q * tb)
    scale = np.sqrt(np.sum(fp ** 2) + np.sum(fq ** 2)) * np.sqrt(np.sum(a ** 2) + np.sum(b ** 2))
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_wave_adjoint_brute_force_transpose(oracle_lib):
    """The adjoint map equals the transpose of the dense forward map."""
    rng = np.random.default_rng(17)
    n = (4, 5, 4)
    size = 80
    kappa = rng.uniform(0.05, 0.2, n)
    M = mr.operator_matrix(n, mr.laplacian_dense_fd8(), STAR, 4, ZERO)
    K = np.diag(kappa.ravel())
    step = np.block([[np.zeros((size, size)), np.eye(size)], [-np.eye(size), 2 * np.eye(size) + K @ M]])
    F = np.linalg.matrix_power(step, 4)
    a, b = rng.standard_normal(n), rng.standard_normal(n)
    ref = F.T @ np.concatenate([a.ravel(), b.ravel()])
    ta, tb = oracle_lib.wave_adjoint(a, b, kappa, 4)
    got = np.concatenate([ta.ravel(), tb.ravel()])
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


def _grad_problem(rng, n, T):
    kappa = rng.uniform(0.05, 0.19, n)
    zeros = np.zeros(n)
    src = (n[2] // 2, n[1] // 2, n[0] - 3)
    wav = wl.ricker(T, 6.0).astype(np.float64)
    rec = 1
    kt = kappa * (1 + 0.05 * rng.random(n))
    _, _, target = oracle_lib_forward(kt, zeros, src, wav, rec, T)
    return kappa, zeros, src, wav, rec, target


def oracle_lib_forward(kappa, zeros, src, wav, rec, T):
    import oracle
    return oracle.wave_forward(zeros, zeros, kappa, T, src=src, wavelet=wav, rec_z=rec)


def _loss(oracle_lib, kappa, zeros, src, wav, rec, T, target):
    _, _, tr = oracle_lib.wave_forward(zeros, zeros, kappa, T, src=src, wavelet=wav, rec_z=rec)
    return 0.5 * np.sum((tr - target) ** 2)


def test_wave_gradient_full_jacobian_fd(oracle_lib):
    """Every component of dJ/dkappa against a central difference (6^3, 5 steps)."""
    rng = np.random.default_rng(19)
    n = (6, 6, 6)
    T = 5
    kappa, zeros, src, wav, rec, target = _grad_problem(rng, n, T)
    g, J = oracle_lib.wave_gradient(zeros, zeros, kappa, T, src, wav, rec, target)
    assert abs(J - _loss(oracle_lib, kappa, zeros, src, wav, rec, T, target)) < 1e-14 * max(J, 1e-30) + 1e-30
    eps = 1e-6
    fd = np.zeros(n)
    for idx in np.ndindex(*n):
        kp = kappa.copy(); kp[idx] += eps
        km = kappa.copy(); km[idx] -= eps
        fd[idx] = (_loss(oracle_lib, kp, zeros, src, wav, rec, T, target)
                   - _loss(oracle_lib, km, zeros, src, wav, rec, T, target)) / (2 * eps)
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd)) + 1e-14


def test_wave_gradient_directional_fd_and_checkpoints(oracle_lib):
    """Directional central difference on a 14^3 x 24-step case, and the
    checkpointed gradient equals the keep-every-state gradient bitwise."""
    rng = np.random.default_rng(23)
    n = (14, 12, 13)
    T = 24
    kappa, zeros, src, wav, rec, target = _grad_problem(rng, n, T)
    g_all, J = oracle_lib.wave_gradient(zeros, zeros, kappa, T, src, wav, rec, target, ckpt_every=0)
    for K in (1, 5, 7, 24):
        g_ck, J_ck = oracle_lib.wave_gradient(zeros, zeros, kappa, T, src, wav, rec, target, ckpt_every=K)
        assert np.array_equal(g_ck, g_all) and J_ck == J
    d = wl.gaussian_pulse((13, 12, 14), (6, 6, 7), 3.0).astype(np.float64)
    eps = 1e-5
    jp = _loss(oracle_lib, kappa + eps * d, zeros, src, wav, rec, T, target)
    jm = _loss(oracle_lib, kappa - eps * d, zeros, src, wav, rec, T, target)
    fd = (jp - jm) / (2 * eps)
    ad = float(np.sum(g_all * d))
    assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_oracle_rejects_bad_arguments(oracle_lib):
    u = np.zeros((4, 4))
    with pytest.raises(ValueError):
        oracle_lib.sweep(u, np.zeros(9), 2, 1, PERIODIC, 1)      # bad shape tag
    with pytest.raises(ValueError):
        oracle_lib.sweep(u, np.zeros(9), BOX, 1, 5, 1)           # bad boundary
    with pytest.raises(ValueError):
        oracle_lib.sweep(u, np.zeros(25), BOX, 1, PERIODIC, 1)   # wrong coefficient count


# ---- variable coefficients -------------------------------------------------
VC_CASES = [(2, (5, 7), STAR, 1), (2, (6, 5), BOX, 2), (3, (4, 5, 6), STAR, 1), (3, (5, 4, 3), BOX, 1),
            (3, (3, 4, 9), STAR, 4), (3, (6, 5, 7), STAR, 2)]


@pytest.mark.parametrize("boundary", [PERIODIC, ZERO])
@pytest.mark.parametrize("ndim,shape_,kind,r", VC_CASES)
def test_varcoef_matches_brute_force_matrix(oracle_lib, ndim, shape_, kind, r, boundary):
    """Forward and transpose against sum_k diag(f_k) S_k built from Kronecker
    shift matrices (grids smaller than 2r+1 included)."""
    rng = np.random.default_rng(hash(("vc", ndim, shape_, kind, r, boundary)) % 2**32)
    nt = len(mr.offsets(ndim, kind, r))
    f = rng.uniform(-1, 1, (nt,) + shape_)
    u = rng.standard_normal(shape_)
    M = mr.varcoef_matrix(shape_, f, kind, r, boundary)
    steps = 3
    ref = np.linalg.matrix_power(M, steps) @ u.ravel()
    got = oracle_lib.varcoef_sweep(u, f, kind, r, boundary, steps)
    assert np.max(np.abs(got.ravel() - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    refT = np.linalg.matrix_power(M.T, steps) @ u.ravel()
    gotT = oracle_lib.varcoef_sweep(u, f, kind, r, boundary, steps, adjoint=True)
    assert np.max(np.abs(gotT.ravel() - refT)) <= 1e-12 * max(1.0, np.max(np.abs(refT)))


@pytest.mark.parametrize("ndim,kind,r,n", [(3, STAR, 1, (9, 8, 10)), (3, BOX, 1, (6, 7, 5)),
                                           (2, STAR, 3, (11, 12)), (3, STAR, 4, (10, 9, 11))])
@pytest.mark.parametrize("boundary", [PERIODIC, ZERO])
def test_varcoef_constant_fields_reduce_to_constant_sweep(oracle_lib, ndim, kind, r, n, boundary):
    """Fields that are constant in space give the constant-coefficient sweep."""
    rng = np.random.default_rng(23)
    c = _rand_coeffs(rng, ndim, kind, r)
    offs = mr.offsets(ndim, kind, r)
    f = np.stack([np.full(n, mr.coeff_at(c, ndim, r, *d)) for d in offs])
    u = rng.standard_normal(n)
    got = oracle_lib.varcoef_sweep(u, f, kind, r, boundary, 4)
    want = oracle_lib.sweep(u, c, kind, r, boundary, 4)
    assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("ndim,kind,r", [(3, STAR, 2), (3, BOX, 1), (2, BOX, 2)])
def test_varcoef_transpose_column_sums(oracle_lib, ndim, kind, r):
    """Periodic transpose: every scattered term lands in the grid, so
    sum(A^T v) = sum_x (sum_k f_k(x)) v(x); and <Au, v> = <u, A^T v>."""
    rng = np.random.default_rng(31)
    n = (13, 11, 12) if ndim == 3 else (17, 15)
    nt = len(mr.offsets(ndim, kind, r))
    f = rng.uniform(-1, 1, (nt,) + n)
    u = rng.standard_normal(n)
    v = rng.standard_normal(n)
    ATv = oracle_lib.varcoef_sweep(v, f, kind, r, PERIODIC, 1, adjoint=True)
    assert abs(ATv.sum() - (f.sum(axis=0) * v).sum()) <= 1e-11 * np.abs(f).sum()
    Au = oracle_lib.varcoef_sweep(u, f, kind, r, PERIODIC, 1)
    assert abs(np.vdot(Au, v) - np.vdot(u, ATv)) <= 1e-12 * np.linalg.norm(Au) * np.linalg.norm(v)


# ---- Storage-rounding diagnostic (the numerical floor of a storage format) ----

def _format_probe_values(rng, fmt):
    """Values spanning normals, subnormals, exact ties and overflow of the
    format: random magnitudes, plus midpoints between neighbouring values
    (where ties-to-even decides) and values around the overflow threshold."""
    if fmt == "binary16":
        p, emin, top = 11, -14, 65504.0
    else:
        p, emin, top = 24, -126, float(np.finfo(np.float32).max)
    mags = np.exp(rng.uniform(np.log(2.0 ** (emin - p)), np.log(top), 4000))
    vals = list(mags * rng.choice([-1.0, 1.0], mags.size))
    for e in (emin - 3, emin, 0, 5):   # midpoints: (k + 1/2) ulp above 2^e (subnormal below emin)
        lead = max(e, emin)
        ulp = 2.0 ** (lead - p + 1)
        for k in (0, 1, 2, 3, 1000):
            vals += [2.0 ** e + (k + 0.5) * ulp if e >= emin else (k + 0.5) * ulp]
    vals += [top, -top, top * (1 + 2.0 ** -(p + 1)) * 0.999999, 1e300, -1e300, 0.0, -0.0]
    if fmt == "binary16":
        vals += [65519.0, 65520.0, -65520.0, 65536.0]
    return np.array(vals, dtype=np.float64)


@pytest.mark.parametrize("fmt,npdt", [("binary16", np.float16), ("binary32", np.float32)])
def test_round_storage_matches_numpy_casts(oracle_lib, fmt, npdt):
    """The oracle's rounding to a storage format, written from the format's
    definition, agrees with numpy's float64 -> float16/float32 conversion on
    normals, subnormals, exact ties and overflow."""
    x = _format_probe_values(np.random.default_rng(5), fmt)
    with np.errstate(over="ignore"):
        ref = x.astype(npdt).astype(np.float64)
    got = oracle_lib.round_storage(x, fmt)
    assert np.array_equal(got, ref, equal_nan=True)
    assert np.array_equal(np.signbit(got), np.signbit(ref))


@pytest.mark.parametrize("ndim,kind,r,n", [(2, BOX, 2, (23, 19)), (3, BOX, 1, (9, 8, 7)), (3, STAR, 4, (10, 9, 11))])
def test_stored_sweep_rounds_every_step(oracle_lib, ndim, kind, r, n):
    """The binary16 floor sweep equals single exact steps each followed by
    numpy's binary16 rounding, and the exact mode equals the plain sweep."""
    rng = np.random.default_rng(61)
    c = _rand_coeffs(rng, ndim, kind, r)
    u = rng.random(n).astype(np.float16).astype(np.float64)
    T = 4
    v = u
    for _ in range(T):
        v = oracle_lib.sweep(v, c, kind, r, PERIODIC, 1).astype(np.float16).astype(np.float64)
    got = oracle_lib.sweep(u, c, kind, r, PERIODIC, T, storage="binary16")
    assert np.array_equal(got, v)
    import ctypes
    lib = oracle_lib._load()
    c64, u64 = np.ascontiguousarray(c, dtype=np.float64), np.ascontiguousarray(u)
    out0 = np.empty_like(u64)
    dp = ctypes.POINTER(ctypes.c_double)
    nn = (n[1], n[0], 1) if ndim == 2 else (n[2], n[1], n[0])
    assert lib.oracle_sweep_stored(ndim, (ctypes.c_int64 * 3)(*nn), kind, r, c64.ctypes.data_as(dp), ZERO, T, 0,
                                   u64.ctypes.data_as(dp), out0.ctypes.data_as(dp)) == 0
    assert np.array_equal(out0, oracle_lib.sweep(u, c, kind, r, ZERO, T))
    exact = oracle_lib.sweep(u, c, kind, r, PERIODIC, T)
    assert not np.array_equal(got, exact)


def test_stored_wave_forward_rounds_every_state(oracle_lib):
    """The binary32 floor leapfrog equals exact single steps (source
    included) each followed by numpy's binary32 rounding."""
    rng = np.random.default_rng(67)
    n = (9, 8, 10)
    kappa = rng.uniform(0.05, 0.2, n[::-1]).astype(np.float32).astype(np.float64)
    u0 = rng.standard_normal(n[::-1]).astype(np.float32).astype(np.float64)
    up = rng.standard_normal(n[::-1]).astype(np.float32).astype(np.float64)
    T, src, rec = 5, (4, 3, 6), 2
    wav = wl.ricker(T, 3.0).astype(np.float64)
    a, b = up, u0
    tr = []
    for t in range(T):
        _, nb, trt = oracle_lib.wave_forward(a, b, kappa, 1, src=src, wavelet=wav[t:t + 1], rec_z=rec)
        a, b = b, nb.astype(np.float32).astype(np.float64)
        tr.append(b[rec])
    ga, gb, gtr = oracle_lib.wave_forward(up, u0, kappa, T, src=src, wavelet=wav, rec_z=rec, storage="binary32")
    assert np.array_equal(ga, a) and np.array_equal(gb, b) and np.array_equal(gtr, np.stack(tr))


def test_stored_gradient_exact_mode_and_floor_size(oracle_lib):
    """The gradient's floor diagnostic: mode 0 of the stored entry point is
    the exact gradient bit for bit; binary32 storage moves it by a small
    nonzero amount (order of the format's precision times the conditioning)."""
    import ctypes
    import oracle
    rng = np.random.default_rng(71)
    n = (12, 11, 13)
    T = 16
    kappa, zeros, src, wav, rec, target = _grad_problem(rng, n, T)
    kappa = kappa.astype(np.float32).astype(np.float64)
    target = target.astype(np.float32).astype(np.float64)
    g, J = oracle_lib.wave_gradient(zeros, zeros, kappa, T, src, wav, rec, target, ckpt_every=5)
    lib = oracle._load()
    lp = oracle.laplacian3d(4)
    g0 = np.empty_like(kappa)
    J0 = ctypes.c_double()
    i64 = ctypes.c_int64 * 3
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.oracle_wave_gradient_stored(i64(n[2], n[1], n[0]), 4, lp.ctypes.data_as(dp), 1, T,
                                           kappa.ctypes.data_as(dp), zeros.ctypes.data_as(dp),
                                           zeros.ctypes.data_as(dp), i64(*src), wav.ctypes.data_as(dp), rec,
                                           target.ctypes.data_as(dp), 5, g0.ctypes.data_as(dp),
                                           ctypes.byref(J0), 0) == 0
    assert np.array_equal(g0, g) and J0.value == J
    g32, J32 = oracle_lib.wave_gradient(zeros, zeros, kappa, T, src, wav, rec, target, ckpt_every=5,
                                        storage="binary32")
    e = mr.rel_l2(g32, g)
    assert 0 < e < 1e-3
    with pytest.raises(ValueError):
        oracle_lib.wave_gradient(zeros, zeros, kappa, T, src, wav, rec, target, storage="binary8")


# ---- Absorbing layer: damped leapfrog, its transpose and its gradient ----

def test_sponge_profile_shape(oracle_lib):
    """Zero away from the faces, the full strength on a face cell, the sum of
    the axes' ramps on edges and corners, symmetric about each mid-plane."""
    W, s = 3, 0.7
    g = oracle_lib.sponge_profile((9, 10, 12), W, s)   # (nz, ny, nx)
    assert np.all(g[W:-W, W:-W, W:-W] == 0)
    assert g[5, 5, 0] == s and g[5, 5, 11] == s
    assert abs(g[5, 5, 1] - s * (2 / 3) ** 2) < 1e-15 and abs(g[5, 5, 2] - s * (1 / 3) ** 2) < 1e-15
    assert abs(g[0, 0, 0] - 3 * s) < 1e-15
    assert np.array_equal(g, g[::-1, ::-1, ::-1])
    assert np.all(oracle_lib.sponge_profile((9, 10, 12), 0, s) == 0)


def _damped_case(rng, n, W=2, s=0.9):
    kappa = rng.uniform(0.05, 0.2, n)
    gamma = oracle_lib_profile(n, W, s)
    return kappa, gamma


def oracle_lib_profile(n, W, s):
    import oracle
    return oracle.sponge_profile(n, W, s)


def test_damped_forward_brute_force_and_zero_damping(oracle_lib):
    """The damped step against dense matrices, u_{t+1} = A(2u + K M u) - B u_prev
    (A = 1/(1+gamma/2), B = (1-gamma/2)/(1+gamma/2)), with source and receiver;
    a zero damping field gives the plain leapfrog bit for bit."""
    rng = np.random.default_rng(81)
    n = (6, 7, 5)
    kappa, gamma = _damped_case(rng, n)
    up, u0 = rng.standard_normal(n), rng.standard_normal(n)
    M = mr.operator_matrix(n, mr.laplacian_dense_fd8(), STAR, 4, ZERO)
    g = gamma.ravel()
    A, B = 1 / (1 + g / 2), (1 - g / 2) / (1 + g / 2)
    src, wav = (2, 3, 1), rng.standard_normal(5)
    a, b = up.ravel().copy(), u0.ravel().copy()
    traces = []
    for t in range(5):
        c = A * (2 * b + kappa.ravel() * (M @ b)) - B * a
        c[(src[2] * n[1] + src[1]) * n[2] + src[0]] += wav[t]
        traces.append(c.reshape(n)[3].copy())
        a, b = b, c
    ga, gb, tr = oracle_lib.wave_forward_damped(up, u0, kappa, gamma, 5, src=src, wavelet=wav, rec_z=3)
    assert np.max(np.abs(gb.ravel() - b)) < 1e-11 * np.max(np.abs(b))
    assert np.max(np.abs(ga.ravel() - a)) < 1e-11 * np.max(np.abs(a))
    assert np.max(np.abs(tr - np.array(traces))) < 1e-11 * np.max(np.abs(traces))
    za, zb, ztr = oracle_lib.wave_forward_damped(up, u0, kappa, np.zeros(n), 5, src=src, wavelet=wav, rec_z=3)
    pa, pb, ptr = oracle_lib.wave_forward(up, u0, kappa, 5, src=src, wavelet=wav, rec_z=3)
    assert np.array_equal(za, pa) and np.array_equal(zb, pb) and np.array_equal(ztr, ptr)


def test_damped_energy_decreases_by_the_damping_work(oracle_lib):
    """With a symmetric L the damped step loses exactly
    E_{t-1/2} - E_{t+1/2} = 1/2 sum gamma/kappa (u_{t+1} - u_{t-1})^2 >= 0 of
    the leapfrog energy E = ||u_{t+1} - u_t||^2_{1/kappa} - <u_{t+1}, L u_t>."""
    rng = np.random.default_rng(83)
    n = (16, 14, 15)
    kappa = rng.uniform(0.05, 0.2, n)
    gamma = oracle_lib.sponge_profile(n, 5, 0.6)
    u0 = wl.gaussian_pulse((15, 14, 16), (3, 7, 8), 2.0).astype(np.float64)   # pulse inside the layer
    up = u0 * 0.97

    def energy(prev, cur):
        return np.sum((cur - prev) ** 2 / kappa) - np.sum(cur * mr.lap_zero_numpy(prev))

    a, b = up, u0
    e_prev = energy(a, b)
    e0 = e_prev
    for _ in range(12):
        na, nb, _ = oracle_lib.wave_forward_damped(a, b, kappa, gamma, 1)
        e = energy(na, nb)
        work = 0.5 * np.sum(gamma / kappa * (nb - a) ** 2)
        assert work > 0
        assert abs((e_prev - e) - work) <= 1e-12 * abs(e0)
        a, b, e_prev = na, nb, e
    assert e_prev < 0.999 * e0


def test_damped_adjoint_brute_force_transpose_and_dot(oracle_lib):
    """The damped adjoint equals the transpose of the dense damped state map,
    satisfies the dot-product identity on a larger grid, and with a zero
    damping field agrees with the plain adjoint."""
    rng = np.random.default_rng(87)
    n = (4, 5, 4)
    size = 80
    kappa, gamma = _damped_case(rng, n, W=2, s=1.3)
    M = mr.operator_matrix(n, mr.laplacian_dense_fd8(), STAR, 4, ZERO)
    g = gamma.ravel()
    A, B = np.diag(1 / (1 + g / 2)), np.diag((1 - g / 2) / (1 + g / 2))
    step = np.block([[np.zeros((size, size)), np.eye(size)], [-B, A @ (2 * np.eye(size) + np.diag(kappa.ravel()) @ M)]])
    F = np.linalg.matrix_power(step, 4)
    a, b = rng.standard_normal(n), rng.standard_normal(n)
    ref = F.T @ np.concatenate([a.ravel(), b.ravel()])
    ta, tb = oracle_lib.wave_adjoint_damped(a, b, kappa, gamma, 4)
    got = np.concatenate([ta.ravel(), tb.ravel()])
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))

    n = (11, 9, 10)
    kappa, gamma = _damped_case(rng, n, W=3, s=0.8)
    p, q, a, b = (rng.standard_normal(n) for _ in range(4))
    fp, fq, _ = oracle_lib.wave_forward_damped(p, q, kappa, gamma, 7)
    ta, tb = oracle_lib.wave_adjoint_damped(a, b, kappa, gamma, 7)
    lhs = np.sum(fp * a) + np.sum(fq * b)
    rhs = np.sum(p * ta) + np.sum(q * tb)
    scale = np.sqrt(np.sum(fp ** 2) + np.sum(fq ** 2)) * np.sqrt(np.sum(a ** 2) + np.sum(b ** 2))
    assert abs(lhs - rhs) <= 1e-12 * scale
    za, zb = oracle_lib.wave_adjoint_damped(a, b, kappa, np.zeros(n), 7)
    pa, pb = oracle_lib.wave_adjoint(a, b, kappa, 7)
    assert np.max(np.abs(za - pa)) <= 1e-12 * np.max(np.abs(pa))
    assert np.max(np.abs(zb - pb)) <= 1e-12 * np.max(np.abs(pb))


def test_damped_gradient_full_jacobian_fd(oracle_lib):
    """Every component of dJ/dkappa of the damped model against a central
    difference of its loss (6^3, 5 steps); the loss is the trace misfit;
    checkpointing leaves the gradient bitwise unchanged; a zero damping field
    gives the plain gradient."""
    rng = np.random.default_rng(89)
    n = (6, 6, 6)
    T = 5
    kappa, zeros, src, wav, rec, target = _grad_problem(rng, n, T)
    gamma = oracle_lib.sponge_profile(n, 2, 1.1)
    g, J = oracle_lib.wave_gradient_damped(zeros, zeros, kappa, gamma, T, src, wav, rec, target)

    def loss(k):
        _, _, tr = oracle_lib.wave_forward_damped(zeros, zeros, k, gamma, T, src=src, wavelet=wav, rec_z=rec)
        return 0.5 * np.sum((tr - target) ** 2)

    assert abs(J - loss(kappa)) < 1e-14 * J
    eps = 1e-6
    fd = np.zeros(n)
    for idx in np.ndindex(*n):
        kp = kappa.copy(); kp[idx] += eps
        km = kappa.copy(); km[idx] -= eps
        fd[idx] = (loss(kp) - loss(km)) / (2 * eps)
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd)) + 1e-14
    gk, Jk = oracle_lib.wave_gradient_damped(zeros, zeros, kappa, gamma, T, src, wav, rec, target, ckpt_every=2)
    assert np.array_equal(gk, g) and Jk == J
    gz, Jz = oracle_lib.wave_gradient_damped(zeros, zeros, kappa, np.zeros(n), T, src, wav, rec, target)
    gp, Jp = oracle_lib.wave_gradient(zeros, zeros, kappa, T, src, wav, rec, target)
    assert np.array_equal(gz, gp) and Jz == Jp
