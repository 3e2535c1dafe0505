"""GPU parity: the HIP kernels against the FP64 oracle, element by element.

Tolerances (rel-L2 over all cells, accumulated in float64): 1e-5 for f32
storage, 2e-3 for fp16 storage.  Sizes span several tiles with ragged tails,
grids smaller than the stencil, every fused depth and every tile family.
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
from mathref import rel_l2
from paper_2609_06694_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f16": 2e-3, "f64": 1e-12}


def legal_depth(tx, ty, k, r, lds_bytes=64 * 1024):
    """Largest fused depth <= k whose two LDS buffers (plus 4 spare rows) fit."""
    while k > 1 and 2 * (tx + 2 * k * r) * (ty + 2 * k * r + 4) * 4 > lds_bytes:
        k //= 2
    return k


@pytest.fixture(scope="module")
def st():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_06694_amd import stencil
    return stencil


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


CASES_2D = [(wl.STAR, r) for r in (1, 2, 3, 4)] + [(wl.BOX, 1), (wl.BOX, 2)]


@pytest.mark.parametrize("shape,r", CASES_2D)
@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_2d_sweep_vs_oracle(st, shape, r, dtype, bc):
    rng = np.random.default_rng(100 * r + shape)
    npdt = np.float32 if dtype == "f32" else np.float16
    c = wl.random_unit_sum_coeffs(rng, 2, shape, r)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny), (tx, ty, k), steps in [((197, 131), (64, 32, 1), 3), ((197, 131), (128, 16, 4), 9),
                                         ((70, 300), (64, 64, 8), 8), ((5, 7), (64, 16, 2), 5)]:
        u = wl.small_random_grid(rng, 2, (nx, ny), npdt, 0.0, 1.0)
        k = legal_depth(tx, ty, k, r)
        s = st.Stencil((nx, ny), shape, r, c, dtype=dtype, boundary=bc, variant=1, tile_x=tx, tile_y=ty,
                       tsteps=k)
        got = _host(s.apply(_dev(u), steps)).astype(np.float64)
        ref = oracle.sweep(u, c, shape, r, bcode, steps)
        e = rel_l2(got, ref)
        assert e <= TOL[dtype], (nx, ny, tx, ty, k, steps, e)


@pytest.mark.parametrize("shape,r", CASES_2D)
@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_2d_tile_waves_vs_oracle(st, shape, r, dtype, bc):
    """LDS tiles run by 8 or 16 waves: 64-column windows whose outputs are
    64 - 2kR wide (one pass per fused step), and wider or odd-width tiles
    that still take several passes; grids of several tiles with ragged
    edges, and one smaller than a tile."""
    rng = np.random.default_rng(900 + 100 * r + shape)
    npdt = np.float32 if dtype == "f32" else np.float16
    c = wl.random_unit_sum_coeffs(rng, 2, shape, r)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    cfgs = []
    for k in (1, 4, 10):
        for h, nw in ((64, 16), (32, 8)):
            bx, by = 64 - 2 * k * r, h - 2 * k * r
            if bx >= 16 and by >= 8:
                cfgs.append((bx, by, k, nw))
    cfgs += [(100, 40, legal_depth(100, 40, 2, r), 8), (128, 32, legal_depth(128, 32, 2, r), 16),
             (64, 16, legal_depth(64, 16, 3, r), 16)]
    for (nx, ny), steps in [((197, 131), 11), ((9, 12), 5)]:
        u = wl.small_random_grid(rng, 2, (nx, ny), npdt, 0.0, 1.0)
        ref = oracle.sweep(u, c, shape, r, bcode, steps)
        for tx, ty, k, nw in cfgs:
            s = st.Stencil((nx, ny), shape, r, c, dtype=dtype, boundary=bc, variant=1, tile_x=tx, tile_y=ty,
                           tsteps=k, zchunk=nw)
            assert s.describe()["zchunk"] == nw
            got = _host(s.apply(_dev(u), steps)).astype(np.float64)
            e = rel_l2(got, ref)
            assert e <= TOL[dtype], (nx, ny, tx, ty, k, nw, steps, e)


@pytest.mark.parametrize("shape,r", CASES_2D)
@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_2d_rowmarch_vs_oracle(st, shape, r, dtype, bc):
    """Row-march kernel: window widths 256/512, fused depths 1..8, automatic
    and explicit chunks (several chunks and strips, ragged tails, grids
    smaller than one window and than the radius)."""
    rng = np.random.default_rng(700 + 100 * r + shape)
    npdt = np.float32 if dtype == "f32" else np.float16
    c = wl.random_unit_sum_coeffs(rng, 2, shape, r)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny), (nt, k, ych), steps in [((197, 131), (256, 1, 0), 3), ((197, 131), (256, 4, 0), 9),
                                          ((600, 45), (512, 2, 20), 5), ((70, 300), (256, 8, 37), 8),
                                          ((5, 7), (256, 2, 0), 5), ((3, 300), (512, 3, 64), 7)]:
        u = wl.small_random_grid(rng, 2, (nx, ny), npdt, 0.0, 1.0)
        s = st.Stencil((nx, ny), shape, r, c, dtype=dtype, boundary=bc, variant=5, tile_x=nt, tile_y=ych,
                       tsteps=k)
        got = _host(s.apply(_dev(u), steps)).astype(np.float64)
        ref = oracle.sweep(u, c, shape, r, bcode, steps)
        e = rel_l2(got, ref)
        assert e <= TOL[dtype], (nx, ny, nt, k, ych, steps, e)


CASES_3D = [(wl.STAR, r) for r in (1, 2, 3, 4)] + [(wl.BOX, 1), (wl.BOX, 2)]


@pytest.mark.parametrize("shape,r", CASES_3D)
@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_3d_sweep_vs_oracle(st, shape, r, dtype, bc):
    rng = np.random.default_rng(1000 + 10 * r + shape)
    npdt = np.float32 if dtype == "f32" else np.float16
    c = wl.random_unit_sum_coeffs(rng, 3, shape, r)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny, nz), (ty, zc), steps in [((70, 37, 29), (16, 0), 2), ((130, 20, 41), (8, 16), 3),
                                          ((65, 70, 13), (32, 5), 1), ((6, 5, 7), (16, 0), 2)]:
        u = wl.small_random_grid(rng, 3, (nx, ny, nz), npdt, 0.0, 1.0)
        s = st.Stencil((nx, ny, nz), shape, r, c, dtype=dtype, boundary=bc, variant=2, tile_y=ty, zchunk=zc)
        got = _host(s.apply(_dev(u), steps)).astype(np.float64)
        ref = oracle.sweep(u, c, shape, r, bcode, steps)
        e = rel_l2(got, ref)
        assert e <= TOL[dtype], (nx, ny, nz, ty, zc, steps, e)


@pytest.mark.parametrize("r", [1, 2])
@pytest.mark.parametrize("dtype", ["f32", "f16", "f64"])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_3d_box_y_march_vs_oracle(st, r, dtype, bc):
    """The march along y (variant ym3d, the few-plane slab structure of the
    boxes): ragged x, few z planes (fewer than a tile's rows, fewer than
    2r+1), y chunks with a ragged tail, grids smaller than 2r+1 in every
    axis; forward, in place and transpose against the oracle, and equal to
    the z-march up to rounding order."""
    rng = np.random.default_rng(7100 + 10 * r + {"f32": 0, "f16": 1, "f64": 2}[dtype])
    npdt = {"f32": np.float32, "f16": np.float16, "f64": np.float64}[dtype]
    c = wl.random_unit_sum_coeffs(rng, 3, wl.BOX, r)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    tys = (8, 16) if dtype == "f64" else (8, 16, 32)
    for (nx, ny, nz), zc, steps in [((300, 90, 8), 32, 2), ((70, 130, 3), 0, 3), ((129, 64, 17), 16, 1),
                                    ((6, 5, 4), 0, 2), ((64, 41, 1), 16, 2)]:
        ty = tys[(nx + nz) % len(tys)]
        u = wl.small_random_grid(rng, 3, (nx, ny, nz), npdt, 0.0, 1.0)
        s = st.Stencil((nx, ny, nz), "box", r, c, dtype=dtype, boundary=bc, variant=10, tile_y=ty, zchunk=zc)
        assert s.describe()["variant"] == "ym3d"
        ref = oracle.sweep(u, c, wl.BOX, r, bcode, steps)
        got = _host(s.apply(_dev(u), steps)).astype(np.float64)
        e = rel_l2(got, ref)
        assert e <= TOL[dtype], (nx, ny, nz, ty, zc, steps, e)
        du = _dev(u)
        s.apply(du, steps, out=du)   # in place
        assert rel_l2(_host(du).astype(np.float64), ref) <= TOL[dtype]
        zm = st.Stencil((nx, ny, nz), "box", r, c, dtype=dtype, boundary=bc, variant=2, tile_y=8)
        assert rel_l2(got, _host(zm.apply(_dev(u), steps)).astype(np.float64)) <= TOL[dtype]
        v = wl.small_random_grid(rng, 3, (nx, ny, nz), npdt, 0.0, 1.0)
        gotT = _host(s.apply_adjoint(_dev(v), steps)).astype(np.float64)
        assert rel_l2(gotT, oracle.sweep(v, c, wl.BOX, r, bcode, steps, adjoint=True)) <= TOL[dtype]


@pytest.mark.parametrize("shape,r", CASES_3D)
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_3d_f64_vs_oracle(st, shape, r, bc):
    """f64 storage and arithmetic (the f32 coefficient values widened): all
    3D stencils, 8- and 16-row tiles, plane chunks, ragged tails, grids
    smaller than 2r+1, in place, and the transpose."""
    rng = np.random.default_rng(6400 + 10 * r + shape)
    c = wl.random_unit_sum_coeffs(rng, 3, shape, r)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny, nz), (ty, zc), steps in [((70, 37, 29), (16, 0), 2), ((130, 20, 41), (8, 16), 3),
                                          ((6, 5, 7), (16, 0), 2)]:
        u = wl.small_random_grid(rng, 3, (nx, ny, nz), np.float64, 0.0, 1.0)
        s = st.Stencil((nx, ny, nz), shape, r, c, dtype="f64", boundary=bc, variant=2, tile_y=ty, zchunk=zc)
        ref = oracle.sweep(u, c, shape, r, bcode, steps)
        got = _host(s.apply(_dev(u), steps))
        assert got.dtype == np.float64
        assert rel_l2(got, ref) <= TOL["f64"], (nx, ny, nz, ty, zc, steps, rel_l2(got, ref))
        d = _dev(u)
        s.apply(d, steps, out=d)
        assert rel_l2(_host(d), ref) <= TOL["f64"], ("in place", nx, ny, nz)
        refT = oracle.sweep(u, c, shape, r, bcode, steps, adjoint=True)
        assert rel_l2(_host(s.apply_adjoint(_dev(u), steps)), refT) <= TOL["f64"], ("adjoint", nx, ny, nz)


@pytest.mark.parametrize("shape,r", CASES_2D)
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_2d_f64_vs_oracle(st, shape, r, bc):
    """2D f64 storage through the row march: fused depths 1-3, both window
    widths, row chunks, ragged tails, a grid smaller than 2r+1, in place,
    and the transpose."""
    rng = np.random.default_rng(6600 + 10 * r + shape)
    c = wl.random_unit_sum_coeffs(rng, 2, shape, r)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny), nt, k, ych, steps in [((300, 141), 512, 1, 0, 3), ((700, 90), 256, 2, 32, 5),
                                        ((5, 4), 256, 2, 0, 4)]:
        u = wl.small_random_grid(rng, 2, (nx, ny), np.float64, 0.0, 1.0)
        s = st.Stencil((nx, ny), shape, r, c, dtype="f64", boundary=bc, variant=5, tile_x=nt, tile_y=ych,
                       tsteps=k)
        ref = oracle.sweep(u, c, shape, r, bcode, steps)
        got = _host(s.apply(_dev(u), steps))
        assert got.dtype == np.float64
        assert rel_l2(got, ref) <= TOL["f64"], ((nx, ny), nt, k, rel_l2(got, ref))
        d = _dev(u)
        s.apply(d, steps, out=d)
        assert rel_l2(_host(d), ref) <= TOL["f64"], ("in place", (nx, ny))
        refT = oracle.sweep(u, c, shape, r, bcode, steps, adjoint=True)
        assert rel_l2(_host(s.apply_adjoint(_dev(u), steps)), refT) <= TOL["f64"], ("adjoint", (nx, ny))


VC_CASES = [(wl.STAR, r) for r in (1, 2, 3, 4)] + [(wl.BOX, 1)]


@pytest.mark.parametrize("shape,r", VC_CASES)
@pytest.mark.parametrize("dtype", ["f32", "f16", "f64"])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_3d_varcoef_vs_oracle(st, shape, r, dtype, bc):
    """Variable coefficients: forward and transpose against the oracle over
    several tiles with ragged tails, plane chunks, grids smaller than 2r+1,
    8- and 16-row tiles, in place; and the dot-product identity."""
    rng = np.random.default_rng(7100 + 10 * r + shape)
    npdt = {"f32": np.float32, "f16": np.float16, "f64": np.float64}[dtype]
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    cases = [((70, 21, 17), (8, 0), 2), ((130, 37, 23), (8, 7), 3), ((5, 4, 6), (8, 0), 2)]
    if shape == wl.STAR and r == 1:
        cases.append(((66, 35, 19), (16, 5), 2))
    for (nx, ny, nz), (ty, zc), steps in cases:
        ntap = st.varcoef_taps(3, wl.SHAPE_NAMES[shape], r)
        f = wl.varcoef_fields(rng, ntap, (nz, ny, nx), npdt)
        u = wl.small_random_grid(rng, 3, (nx, ny, nz), npdt, 0.0, 1.0)
        s = st.VarCoefStencil((nx, ny, nz), shape, r, dtype=dtype, boundary=bc, variant=7, tile_y=ty, zchunk=zc)
        fd = _dev(f)
        ref = oracle.varcoef_sweep(u, f, shape, r, bcode, steps)
        got = _host(s.apply(_dev(u), fd, steps)).astype(np.float64)
        assert rel_l2(got, ref) <= TOL[dtype], ((nx, ny, nz), ty, zc, rel_l2(got, ref))
        d = _dev(u)
        s.apply(d, fd, steps, out=d)
        assert rel_l2(_host(d).astype(np.float64), ref) <= TOL[dtype], ("in place", (nx, ny, nz))
        refT = oracle.varcoef_sweep(u, f, shape, r, bcode, steps, adjoint=True)
        gotT = _host(s.apply_adjoint(_dev(u), fd, steps)).astype(np.float64)
        assert rel_l2(gotT, refT) <= TOL[dtype], ("adjoint", (nx, ny, nz), ty, zc, rel_l2(gotT, refT))
    if dtype != "f16":
        # <A x, y> = <x, A^T y> with one step, FP64 dot products.
        x = wl.small_random_grid(rng, 3, (41, 19, 13), npdt)
        y = wl.small_random_grid(rng, 3, (41, 19, 13), npdt)
        f = wl.varcoef_fields(rng, ntap, (13, 19, 41), npdt)
        s = st.VarCoefStencil((41, 19, 13), shape, r, dtype=dtype, boundary=bc)
        Ax = _host(s.apply(_dev(x), _dev(f), 1)).astype(np.float64)
        ATy = _host(s.apply_adjoint(_dev(y), _dev(f), 1)).astype(np.float64)
        lhs, rhs = float(np.sum(Ax * y)), float(np.sum(x.astype(np.float64) * ATy))
        assert abs(lhs - rhs) <= TOL[dtype] * np.linalg.norm(Ax) * np.linalg.norm(y.astype(np.float64))


@pytest.mark.parametrize("shape,r", VC_CASES)
@pytest.mark.parametrize("dtype", ["f32", "f16", "f64"])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_2d_varcoef_vs_oracle(st, shape, r, dtype, bc):
    """2D variable coefficients (one plane, no z reach): forward, transpose,
    several tiles with ragged tails, a grid smaller than 2r+1, in place."""
    rng = np.random.default_rng(7300 + 10 * r + shape)
    npdt = {"f32": np.float32, "f16": np.float16, "f64": np.float64}[dtype]
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    ntap = st.varcoef_taps(2, wl.SHAPE_NAMES[shape], r)
    for (nx, ny), ty, steps in [((130, 70), 8, 3), ((300, 41), 16 if (shape == wl.STAR and r == 1) else 8, 2),
                                ((5, 4), 8, 2)]:
        f = wl.varcoef_fields(rng, ntap, (ny, nx), npdt)
        u = wl.small_random_grid(rng, 2, (nx, ny), npdt, 0.0, 1.0)
        s = st.VarCoefStencil((nx, ny), shape, r, dtype=dtype, boundary=bc, variant=7, tile_y=ty)
        fd = _dev(f)
        ref = oracle.varcoef_sweep(u, f, shape, r, bcode, steps)
        got = _host(s.apply(_dev(u), fd, steps)).astype(np.float64)
        assert rel_l2(got, ref) <= TOL[dtype], ((nx, ny), ty, rel_l2(got, ref))
        d = _dev(u)
        s.apply(d, fd, steps, out=d)
        assert rel_l2(_host(d).astype(np.float64), ref) <= TOL[dtype], ("in place", (nx, ny))
        refT = oracle.varcoef_sweep(u, f, shape, r, bcode, steps, adjoint=True)
        gotT = _host(s.apply_adjoint(_dev(u), fd, steps)).astype(np.float64)
        assert rel_l2(gotT, refT) <= TOL[dtype], ("adjoint", (nx, ny), rel_l2(gotT, refT))


def test_varcoef_autograd_backward_is_transpose(st):
    """The differentiable variable-coefficient sweep back-propagates through
    the transposed sweep: grad_u <g, A^T u> equals A^T g."""
    rng = np.random.default_rng(91)
    n = (70, 33, 21)
    s = st.VarCoefStencil(n, "star", 2, boundary="zero")
    f = _dev(wl.varcoef_fields(rng, 13, n[::-1], np.float32))
    u = _dev(wl.small_random_grid(rng, 3, n, np.float32)).requires_grad_(True)
    g = _dev(wl.small_random_grid(rng, 3, n, np.float32))
    out = st.varcoef_sweep(u, f, s, 3)
    (out * g).sum().backward()
    want = s.apply_adjoint(g, f, 3)
    assert torch.allclose(u.grad, want, rtol=0, atol=0)
    ref = oracle.varcoef_sweep(_host(g), _host(f), wl.STAR, 2, wl.ZERO, 3, adjoint=True)
    assert rel_l2(_host(u.grad).astype(np.float64), ref) <= 1e-5


def test_varcoef_steps_and_argument_checks(st):
    """Zero steps copy; a constant-coefficient entry point rejects a
    variable-coefficient plan; wrongly shaped fields are refused."""
    rng = np.random.default_rng(77)
    s = st.VarCoefStencil((40, 30, 20), "star", 2)
    u = wl.small_random_grid(rng, 3, (40, 30, 20), np.float32)
    f = _dev(wl.varcoef_fields(rng, 13, (20, 30, 40), np.float32))
    d = _dev(u)
    assert torch.equal(s.apply(d, f, 0), d)
    with pytest.raises(ValueError):
        s.apply(d, f[:12].contiguous(), 1)
    from paper_2609_06694_amd import _abi
    lib = _abi.lib()
    rc = lib.stencil_apply(s._h, d.data_ptr(), d.data_ptr(), 1, None, None, 0, None)
    assert rc == _abi.ST_EINVAL


@pytest.mark.parametrize("shape", [wl.STAR, wl.BOX])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_3d_two_step_vs_oracle(st, shape, dtype, bc):
    """Radius-1 3D sweeps with two steps per launch: several 62 x 30 tiles
    with ragged tails, plane chunks, odd step counts (a final one-step
    launch), grids smaller than a tile, in place."""
    rng = np.random.default_rng(3030 + shape)
    npdt = np.float32 if dtype == "f32" else np.float16
    c = wl.random_unit_sum_coeffs(rng, 3, shape, 1)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny, nz), ty, zc, steps in [((130, 70, 23), 32, 0, 4), ((63, 31, 40), 16, 7, 5),
                                        ((200, 95, 17), 32, 16, 2), ((5, 4, 6), 16, 0, 3)]:
        u = wl.small_random_grid(rng, 3, (nx, ny, nz), npdt, 0.0, 1.0)
        s = st.Stencil((nx, ny, nz), shape, 1, c, dtype=dtype, boundary=bc, variant=2, tile_y=ty, tsteps=2,
                       zchunk=zc)
        ref = oracle.sweep(u, c, shape, 1, bcode, steps)
        got = _host(s.apply(_dev(u), steps)).astype(np.float64)
        assert rel_l2(got, ref) <= TOL[dtype], (nx, ny, nz, zc, steps, rel_l2(got, ref))
        d = _dev(u)
        s.apply(d, steps, out=d)
        assert rel_l2(_host(d).astype(np.float64), ref) <= TOL[dtype], ("in place", nx, ny, nz)


def test_inplace_and_zero_steps(st):
    rng = np.random.default_rng(5)
    c = wl.random_unit_sum_coeffs(rng, 2, wl.BOX, 1)
    u = wl.small_random_grid(rng, 2, (150, 90), np.float32)
    s = st.Stencil((150, 90), "box", 1, c, tsteps=2)
    for steps in (0, 1, 3, 4, 5):
        d = _dev(u)
        s.apply(d, steps, out=d)   # u_in == u_out
        ref = oracle.sweep(u, c, wl.BOX, 1, wl.PERIODIC, steps)
        assert rel_l2(_host(d), ref) <= 1e-6, steps


@pytest.mark.parametrize("ndim,shape,r", [(2, wl.STAR, 3), (2, wl.BOX, 2), (3, wl.STAR, 2), (3, wl.BOX, 1),
                                         (3, wl.BOX, 2)])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_linear_adjoint_vs_oracle_and_dot(st, ndim, shape, r, bc):
    rng = np.random.default_rng(7 + r)
    n = (91, 67) if ndim == 2 else (70, 19, 23)
    c = (rng.uniform(-1, 1, (2 * r + 1) ** ndim) * (wl.random_unit_sum_coeffs(rng, ndim, shape, r) != 0)).astype(np.float32)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    x = wl.small_random_grid(rng, ndim, n, np.float32)
    y = wl.small_random_grid(rng, ndim, n, np.float32)
    s = st.Stencil(n, shape, r, c, boundary=bc)
    steps = 3
    ATy = _host(s.apply_adjoint(_dev(y), steps))
    Ax = _host(s.apply(_dev(x), steps))
    assert rel_l2(ATy, oracle.sweep(y, c, shape, r, bcode, steps, adjoint=True)) <= 1e-5
    lhs = float(np.sum(Ax.astype(np.float64) * y))
    rhs = float(np.sum(x.astype(np.float64) * ATy))
    scale = np.linalg.norm(Ax.astype(np.float64)) * np.linalg.norm(y.astype(np.float64))
    assert abs(lhs - rhs) <= 1e-5 * scale


@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_3d_box_fp16_mfma_vs_oracle(st, bc):
    """Matrix-core 27-point box (fp16 storage): several tiles, ragged y and
    z, x a multiple of 8 but not of the tile, grids smaller than a tile, and
    explicit plane chunks; forward against the oracle and the vector-ALU
    kernel, and the transposed sweep against the oracle."""
    rng = np.random.default_rng(4242)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny, nz), zc, steps in [((64, 64, 20), 0, 3), ((136, 70, 33), 5, 4), ((8, 5, 7), 0, 3),
                                    ((200, 130, 18), 16, 2)]:
        c = wl.random_unit_sum_coeffs(rng, 3, wl.BOX, 1)
        u = wl.small_random_grid(rng, 3, (nx, ny, nz), np.float16, 0.0, 1.0)
        s = st.Stencil((nx, ny, nz), "box", 1, c, dtype="f16", boundary=bc, variant=6, tile_y=64, zchunk=zc)
        assert s.describe()["variant"] == "zm3d_mfma"
        got = _host(s.apply(_dev(u), steps)).astype(np.float64)
        ref = oracle.sweep(u, c, wl.BOX, 1, bcode, steps)
        assert rel_l2(got, ref) <= TOL["f16"], (nx, ny, nz, zc, rel_l2(got, ref))
        valu = st.Stencil((nx, ny, nz), "box", 1, c, dtype="f16", boundary=bc, variant=2, tile_y=16)
        alt = _host(valu.apply(_dev(u), steps)).astype(np.float64)
        assert rel_l2(got, alt) <= TOL["f16"], (nx, ny, nz, zc)
        v = wl.small_random_grid(rng, 3, (nx, ny, nz), np.float16, 0.0, 1.0)
        gotT = _host(s.apply_adjoint(_dev(v), steps)).astype(np.float64)
        assert rel_l2(gotT, oracle.sweep(v, c, wl.BOX, 1, bcode, steps, adjoint=True)) <= TOL["f16"]


@pytest.mark.parametrize("bc", ["periodic", "zero"])
@pytest.mark.parametrize("r,ty", [(1, 8), (1, 16), (1, 32), (2, 8), (2, 16), (2, 32)])
def test_3d_box_fp16_packed_half_vs_oracle(st, bc, r, ty):
    """Packed-half 27- and 125-point boxes (fp16 storage, two cells per
    lane, binary16 weights with the residual sum on the centre): several
    tiles with ragged x (even), y and z tails, grids smaller than a tile and
    than 2r+1, plane chunks, nx not a multiple of 4, nx = 2; forward and
    transpose against the oracle at the fp16 gate and within 5x of the
    binary16 storage floor."""
    rng = np.random.default_rng(5150 + ty + 100 * r)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny, nz), zc, steps in [((256, 40, 20), 0, 3), ((202, 70, 33), 5, 4), ((10, 5, 7), 0, 3),
                                    ((130, 33, 18), 8, 5), ((2, 3, 4), 0, 2), ((386, 17, 9), 0, 6)]:
        c = wl.random_unit_sum_coeffs(rng, 3, wl.BOX, r)
        u = wl.small_random_grid(rng, 3, (nx, ny, nz), np.float16, 0.0, 1.0)
        s = st.Stencil((nx, ny, nz), "box", r, c, dtype="f16", boundary=bc, variant=8, tile_y=ty, zchunk=zc)
        assert s.describe()["variant"] == "zm3d_h2"
        got = _host(s.apply(_dev(u), steps)).astype(np.float64)
        ref = oracle.sweep(u, c, wl.BOX, r, bcode, steps)
        floor = rel_l2(oracle.sweep(u, c, wl.BOX, r, bcode, steps, storage="binary16"), ref)
        e = rel_l2(got, ref)
        assert e <= TOL["f16"] and e <= 5 * floor, (nx, ny, nz, zc, e, floor)
        v = wl.small_random_grid(rng, 3, (nx, ny, nz), np.float16, 0.0, 1.0)
        gotT = _host(s.apply_adjoint(_dev(v), steps)).astype(np.float64)
        assert rel_l2(gotT, oracle.sweep(v, c, wl.BOX, r, bcode, steps, adjoint=True)) <= TOL["f16"]


@pytest.mark.parametrize("bc", ["periodic", "zero"])
@pytest.mark.parametrize("ty", [8, 16, 32])
def test_3d_star_fp16_packed_half_vs_oracle(st, bc, ty):
    """Packed-half 7-point star (fp16 storage; the radius-1 box kernel with
    the off-axis rows left out): ragged even sizes, grids smaller than a
    tile and than 3, plane chunks; forward and transpose against the oracle
    at the fp16 gate and within 5x of the binary16 storage floor, and the
    forward equal to the packed-half box given the star's weights with
    zeros off the axes."""
    rng = np.random.default_rng(7170 + ty)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny, nz), zc, steps in [((256, 40, 20), 0, 3), ((202, 70, 33), 5, 4), ((10, 5, 7), 0, 3),
                                    ((2, 3, 4), 0, 2), ((386, 17, 9), 0, 6)]:
        c = wl.random_unit_sum_coeffs(rng, 3, wl.STAR, 1)
        u = wl.small_random_grid(rng, 3, (nx, ny, nz), np.float16, 0.0, 1.0)
        s = st.Stencil((nx, ny, nz), "star", 1, c, dtype="f16", boundary=bc, variant=8, tile_y=ty, zchunk=zc)
        assert s.describe()["variant"] == "zm3d_h2"
        got_dev = s.apply(_dev(u), steps)
        got = _host(got_dev).astype(np.float64)
        ref = oracle.sweep(u, c, wl.STAR, 1, bcode, steps)
        floor = rel_l2(oracle.sweep(u, c, wl.STAR, 1, bcode, steps, storage="binary16"), ref)
        e = rel_l2(got, ref)
        assert e <= TOL["f16"] and e <= 5 * floor, (nx, ny, nz, zc, e, floor)
        sb = st.Stencil((nx, ny, nz), "box", 1, c, dtype="f16", boundary=bc, variant=8, tile_y=ty, zchunk=zc)
        assert np.array_equal(_host(sb.apply(_dev(u), steps)), _host(got_dev)), (nx, ny, nz, zc)
        v = wl.small_random_grid(rng, 3, (nx, ny, nz), np.float16, 0.0, 1.0)
        gotT = _host(s.apply_adjoint(_dev(v), steps)).astype(np.float64)
        assert rel_l2(gotT, oracle.sweep(v, c, wl.STAR, 1, bcode, steps, adjoint=True)) <= TOL["f16"]


@pytest.mark.parametrize("r", [1, 2])
@pytest.mark.parametrize("bc", ["periodic", "zero"])
@pytest.mark.parametrize("nt,k,ych", [(256, 1, 0), (256, 2, 0), (512, 3, 32), (256, 4, 16), (512, 8, 0)])
def test_2d_box_fp16_packed_half_vs_oracle(st, r, bc, nt, k, ych):
    """Packed-half row march (fp16 boxes, two cells per lane, k fused steps
    with every level rounded to binary16): ragged even nx, grids narrower
    than a window, few rows, step counts that leave a shorter last block;
    forward and transpose against the oracle at the fp16 gate and within 5x
    of the binary16 storage floor."""
    rng = np.random.default_rng(6160 + 10 * r + k)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    for (nx, ny), steps in [((1030, 517), 7), ((2, 9), 5), ((600, 3), 4), ((1536, 300), 9)]:
        c = wl.random_unit_sum_coeffs(rng, 2, wl.BOX, r)
        u = wl.small_random_grid(rng, 2, (nx, ny), np.float16, 0.0, 1.0)
        s = st.Stencil((nx, ny), "box", r, c, dtype="f16", boundary=bc, variant=9, tile_x=nt, tile_y=ych, tsteps=k)
        assert s.describe()["variant"] == "ym2d_h2"
        got = _host(s.apply(_dev(u), steps)).astype(np.float64)
        ref = oracle.sweep(u, c, wl.BOX, r, bcode, steps)
        floor = rel_l2(oracle.sweep(u, c, wl.BOX, r, bcode, steps, storage="binary16"), ref)
        e = rel_l2(got, ref)
        assert e <= TOL["f16"] and e <= 5 * floor, (nx, ny, steps, e, floor)
        v = wl.small_random_grid(rng, 2, (nx, ny), np.float16, 0.0, 1.0)
        gotT = _host(s.apply_adjoint(_dev(v), steps)).astype(np.float64)
        assert rel_l2(gotT, oracle.sweep(v, c, wl.BOX, r, bcode, steps, adjoint=True)) <= TOL["f16"]


def test_graph_capture_replays_match_eager(st):
    """A sweep captured in a HIP graph (torch.cuda.graph) replays bitwise
    equal to the eager call, every replay, with eager work and
    synchronisation between replays (tile kernel, row march, z-march)."""
    rng = np.random.default_rng(31)
    for n, shape, r, kw, steps in [((512, 512), wl.STAR, 1, {}, 10),
                                   ((700, 300), wl.BOX, 2, dict(variant=5, tile_x=256, tsteps=2), 5),
                                   ((96, 70, 40), wl.STAR, 4, {}, 3)]:
        c = wl.random_unit_sum_coeffs(rng, len(n), shape, r)
        u = _dev(wl.small_random_grid(rng, len(n), n, np.float32, 0.0, 1.0))
        s = st.Stencil(n, shape, r, c, **kw)
        eager = _host(s.apply(u, steps))
        out = torch.empty_like(u)
        s.apply(u, steps, out=out)   # allocates the workspace before capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            s.apply(u, steps, out=out)
        for rep in range(4):
            out.fill_(float(rep + 1))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(_host(out), eager), (n, rep)


def test_autograd_sweep_backward_is_transpose(st):
    rng = np.random.default_rng(8)
    c = wl.random_unit_sum_coeffs(rng, 2, wl.BOX, 2)
    s = st.Stencil((96, 80), "box", 2, c)
    u = _dev(wl.small_random_grid(rng, 2, (96, 80), np.float32)).requires_grad_(True)
    w = _dev(wl.small_random_grid(rng, 2, (96, 80), np.float32))
    (st.sweep(u, s, 4) * w).sum().backward()
    ref = oracle.sweep(_host(w), c, wl.BOX, 2, wl.PERIODIC, 4, adjoint=True)
    assert rel_l2(_host(u.grad), ref) <= 1e-5


def _wave_inputs(rng, n):
    nx, ny, nz = n
    kappa = rng.uniform(0.05, 0.2, (nz, ny, nx)).astype(np.float32)
    u0 = wl.gaussian_pulse(n, (nx // 2, ny // 3, nz // 2), 3.0)
    up = (u0 * np.float32(0.97)).astype(np.float32)
    return kappa, u0, up


@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("variant,ty,zc", [(3, 16, 0), (3, 8, 9), (3, 32, 64), (4, 8, 0), (4, 16, 9), (4, 8, 5)])
@pytest.mark.parametrize("aniso", [False, True])
def test_wave_forward_vs_oracle(st, bc, variant, ty, zc, aniso):
    """Both forward kernel families (partial-sum queue, LDS ring), with the
    isotropic Laplacian and with an anisotropic radius-4 star."""
    rng = np.random.default_rng(21)
    n = (75, 41, 33)
    kappa, u0, up = _wave_inputs(rng, n)
    steps = 7
    src = (30, 20, 17)
    wav = wl.ricker(steps, 4.0)
    bcode = wl.ZERO if bc == "zero" else wl.PERIODIC
    lap = None
    if aniso:   # a valid but anisotropic star: different weights per axis and sign
        lap = oracle.laplacian3d(4)
        for j, f in ((1, 1.1), (2, 0.9), (3, 1.2), (4, 0.8)):
            lap[(4 * 9 + 4) * 9 + 4 + j] *= f
            lap[(4 * 9 + 4 - j) * 9 + 4] *= 1.0 / f
        lap = lap.astype(np.float32)
    m = st.WaveModel(n, boundary=bc, tile_y=ty, zchunk=zc, variant=variant, coeffs=lap)
    uT, uT1, tr = m.forward(_dev(u0), _dev(up), _dev(kappa), steps, src=src, wavelet=_dev(wav), rec_z=5,
                            record=True)
    ra, rb, rtr = oracle.wave_forward(up, u0, kappa, steps, boundary=bcode, src=src, wavelet=wav, rec_z=5,
                                      lap=None if lap is None else lap.astype(np.float64))
    assert rel_l2(_host(uT), rb) <= 1e-5
    assert rel_l2(_host(uT1), ra) <= 1e-5
    assert rel_l2(_host(tr), rtr) <= 1e-5


@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("ty,zc", [(32, 0), (16, 9), (8, 5), (32, 16)])
def test_wave_two_planes_per_barrier_bitwise(st, bc, ty, zc):
    """Staging the two planes of a march step per barrier (tile_x=2) gives
    the one-plane-per-barrier result bit for bit (the same per-cell
    arithmetic): forward with source and receiver against the oracle too,
    and under the zero frame the absorbing layer and the gradient (whose
    recompute writes L(u_t))."""
    rng = np.random.default_rng(23)
    n = (75, 41, 33)
    kappa, u0, up = _wave_inputs(rng, n)
    steps, src = 6, (30, 20, 17)
    wav = wl.ricker(steps, 4.0)
    bcode = wl.ZERO if bc == "zero" else wl.PERIODIC
    outs = []
    for tx in (0, 2):
        m = st.WaveModel(n, boundary=bc, tile_y=ty, zchunk=zc, variant=4, tile_x=tx)
        assert m.describe()["tile_x"] == tx
        outs.append([_host(a) for a in m.forward(_dev(u0), _dev(up), _dev(kappa), steps, src=src,
                                                 wavelet=_dev(wav), rec_z=5, record=True)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    ra, rb, rtr = oracle.wave_forward(up, u0, kappa, steps, boundary=bcode, src=src, wavelet=wav, rec_z=5)
    assert rel_l2(outs[1][0], rb) <= 1e-5 and rel_l2(outs[1][1], ra) <= 1e-5 and rel_l2(outs[1][2], rtr) <= 1e-5
    if bc != "zero":
        return
    sp = []
    for tx in (0, 2):
        m = st.WaveModel(n, tile_y=ty, zchunk=zc, variant=4, tile_x=tx, sponge=(6, 0.8))
        sp.append([_host(a) for a in m.forward(_dev(u0), _dev(up), _dev(kappa), steps)[:2]])
    for a, b in zip(*sp):
        assert np.array_equal(a, b)
    kg, zeros, gsrc, gwav, rec, target = _grad_case(steps=20, blob=False)
    gr = []
    for tx in (0, 2):
        m = st.WaveModel(kg.shape[::-1], tile_y=ty, zchunk=zc, variant=4, tile_x=tx, ckpt_every=6)
        dk, loss = m.gradient(_dev(zeros), _dev(zeros), _dev(kg), 20, gsrc, _dev(gwav), rec, _dev(target))
        gr.append((_host(dk), _host(loss)))
    assert np.array_equal(gr[0][0], gr[1][0]) and np.array_equal(gr[0][1], gr[1][1])


@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("r,ty,zc", [(4, 8, 0), (4, 16, 9), (2, 8, 5), (1, 16, 0), (3, 8, 16)])
@pytest.mark.parametrize("aniso", [False, True])
def test_wave_f64_forward_vs_oracle(st, bc, r, ty, zc, aniso):
    """FP64 leapfrog (binary64 fields, weights and arithmetic) with source and
    receiver against the FP64 oracle at the f64 gate, on ragged tiles and z
    chunks; both the built-in Laplacian (its rationals rounded once to
    binary64 on both sides) and an anisotropic star given in f32."""
    rng = np.random.default_rng(41 + r)
    n = (75, 41, 33)
    nx, ny, nz = n
    kappa = rng.uniform(0.05, 0.2, (nz, ny, nx))
    u0 = wl.gaussian_pulse(n, (nx // 2, ny // 3, nz // 2), 3.0).astype(np.float64)
    up = u0 * 0.97
    steps, src, rec = 7, (30, 20, 17), 5
    wav = wl.ricker(steps, 4.0).astype(np.float64)
    bcode = wl.ZERO if bc == "zero" else wl.PERIODIC
    lap = None
    if aniso:
        w = 2 * r + 1
        lap = oracle.laplacian3d(r)
        for j in range(1, r + 1):
            lap[(r * w + r) * w + r + j] *= 1.0 + 0.1 * j
            lap[(r * w + r - j) * w + r] *= 1.0 - 0.05 * j
        lap = lap.astype(np.float32)
    m = st.WaveModel(n, radius=r, boundary=bc, coeffs=lap, dtype="f64", tile_y=ty, zchunk=zc)
    d = m.describe()
    assert (d["variant"], d["tile_y"], d["tsteps"]) == ("wave3d", ty, 1)
    uT, uT1, tr = m.forward(_dev(u0), _dev(up), _dev(kappa), steps, src=src, wavelet=_dev(wav), rec_z=rec,
                            record=True)
    assert uT.dtype == torch.float64 and tr.dtype == torch.float64
    ra, rb, rtr = oracle.wave_forward(up, u0, kappa, steps, r=r, boundary=bcode, src=src, wavelet=wav, rec_z=rec,
                                      lap=None if lap is None else lap.astype(np.float64))
    e = max(rel_l2(_host(uT), rb), rel_l2(_host(uT1), ra), rel_l2(_host(tr), rtr))
    print(f"f64 wave r={r} {bc} ty={ty} zc={zc} aniso={aniso}: rel-L2 {e:.2e}")
    assert e <= TOL["f64"]


@pytest.mark.parametrize("steps", [1, 4, 5])
def test_wave_f64_sponge_inplace_and_f32_contrast(st, steps):
    """FP64 leapfrog with the absorbing layer against the oracle's damped
    recursion, in place (u_in == u_out, odd and even step counts); and the
    same case through the f32 model, whose binary32 storage sits orders of
    magnitude above the f64 gate (so the f64 path is not f32 in disguise)."""
    rng = np.random.default_rng(51)
    n = (67, 35, 30)
    nx, ny, nz = n
    W, s = 6, 1.2
    kappa = rng.uniform(0.05, 0.2, (nz, ny, nx))
    u0 = wl.gaussian_pulse(n, (nx // 3, ny // 3, nz // 2), 3.0).astype(np.float64)
    up = u0 * 0.98
    src = (nx // 2, ny // 2, nz // 2)
    wav = wl.ricker(steps, 4.0).astype(np.float64)
    # The strength crosses the C ABI as a binary32 value; the layer then
    # evaluates in binary64 from exactly that value.
    gamma = oracle.sponge_profile((nz, ny, nx), W, float(np.float32(s)))
    ra, rb, _ = oracle.wave_forward_damped(up, u0, kappa, gamma, steps, src=src, wavelet=wav)
    m = st.WaveModel(n, dtype="f64", sponge=(W, s))
    u = _dev(u0)
    prev = _dev(up)
    m.forward(u, prev, _dev(kappa), steps, src=src, wavelet=_dev(wav), out=u, prev_inout=True)
    e = max(rel_l2(_host(u), rb), rel_l2(_host(prev), ra))
    m32 = st.WaveModel(n, sponge=(W, s))
    u32, p32, _ = m32.forward(_dev(u0.astype(np.float32)), _dev(up.astype(np.float32)),
                              _dev(kappa.astype(np.float32)), steps, src=src,
                              wavelet=_dev(wav.astype(np.float32)))
    e32 = max(rel_l2(_host(u32), rb), rel_l2(_host(p32), ra))
    print(f"f64 sponge steps={steps}: rel-L2 {e:.2e} (f32 model: {e32:.2e})")
    assert e <= TOL["f64"]
    assert e32 > 1e3 * TOL["f64"]


@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("n,ty,zc", [((75, 41, 33), 8, 0), ((130, 37, 29), 16, 9), ((20, 9, 11), 8, 4)])
@pytest.mark.parametrize("steps", [2, 3, 4, 7])
def test_wave_two_step_fused_vs_oracle(st, bc, n, ty, zc, steps):
    """Two leapfrog steps per launch (temporal blocking) against the oracle,
    with source and receiver, on grids narrower and wider than one tile."""
    rng = np.random.default_rng(23 + steps)
    kappa, u0, up = _wave_inputs(rng, n)
    src = (n[0] // 2 + 1, n[1] // 2, n[2] // 2 - 1)
    wav = wl.ricker(steps, 3.0)
    rec = n[2] // 3
    bcode = wl.ZERO if bc == "zero" else wl.PERIODIC
    m = st.WaveModel(n, boundary=bc, tile_y=ty, zchunk=zc, tsteps=2, variant=3)
    assert m.describe()["tsteps"] == 2
    uT, uT1, tr = m.forward(_dev(u0), _dev(up), _dev(kappa), steps, src=src, wavelet=_dev(wav), rec_z=rec,
                            record=True)
    ra, rb, rtr = oracle.wave_forward(up, u0, kappa, steps, boundary=bcode, src=src, wavelet=wav, rec_z=rec)
    e = (rel_l2(_host(uT), rb), rel_l2(_host(uT1), ra), rel_l2(_host(tr), rtr))
    assert max(e) <= 1e-5, e


def test_wave_two_step_inplace_output(st):
    rng = np.random.default_rng(29)
    n = (70, 30, 26)
    kappa, u0, up = _wave_inputs(rng, n)
    m = st.WaveModel(n, tsteps=2, variant=3)
    for steps in (4, 5, 6):
        d = _dev(u0)
        p = _dev(up)
        m.forward(d, p, _dev(kappa), steps, out=d, prev_inout=True)
        ra, rb, _ = oracle.wave_forward(up, u0, kappa, steps)
        assert rel_l2(_host(d), rb) <= 1e-5 and rel_l2(_host(p), ra) <= 1e-5, steps


@pytest.mark.parametrize("steps", [1, 2, 5])
def test_wave_adjoint_vs_oracle_and_dot(st, steps):
    rng = np.random.default_rng(31)
    n = (67, 35, 30)
    kappa, p, q = _wave_inputs(rng, n)
    a = rng.standard_normal(q.shape).astype(np.float32)
    b = rng.standard_normal(q.shape).astype(np.float32)
    m = st.WaveModel(n)
    ta, tb = m.adjoint(_dev(a), _dev(b), _dev(kappa), steps)
    ra, rb = oracle.wave_adjoint(a, b, kappa, steps)
    assert rel_l2(_host(ta), ra) <= 1e-5 and rel_l2(_host(tb), rb) <= 1e-5
    fq, fp, _ = m.forward(_dev(q), _dev(p), _dev(kappa), steps)
    lhs = float(np.sum(_host(fp).astype(np.float64) * a) + np.sum(_host(fq).astype(np.float64) * b))
    rhs = float(np.sum(p.astype(np.float64) * _host(ta)) + np.sum(q.astype(np.float64) * _host(tb)))
    scale = np.sqrt(np.sum(_host(fp).astype(np.float64) ** 2) + np.sum(_host(fq).astype(np.float64) ** 2)) * \
        np.sqrt(np.sum(a.astype(np.float64) ** 2) + np.sum(b.astype(np.float64) ** 2))
    assert abs(lhs - rhs) <= 1e-5 * scale


def _grad_case(n=(40, 36, 44), steps=30, seed=41, blob=True):
    """Gradient inputs.  blob=True: the target comes from kappa with a +5%
    Gaussian blob (small residual, as in the full-size workload); blob=False:
    the target is zero, so the residual is the recorded trace itself."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    kappa = rng.uniform(0.05, 0.19, (nz, ny, nx)).astype(np.float32)
    zeros = np.zeros_like(kappa)
    src = (nx // 2, ny // 2, 12)
    wav = wl.ricker(steps, 8.0)
    rec = 6
    if blob:
        b = wl.gaussian_pulse(n, (nx // 2, ny // 2, 24), 4.0).astype(np.float64)
        kt = (kappa * (1 + 0.05 * b)).astype(np.float32)
        _, _, target = oracle.wave_forward(zeros, zeros, kt, steps, src=src, wavelet=wav, rec_z=rec)
    else:
        target = np.zeros((steps, ny, nx))
    return kappa, zeros, src, wav, rec, target.astype(np.float32)


@pytest.mark.parametrize("family", ["ring", "queue"])
def test_wave_gradient_vs_oracle(st, family):
    """Large residual (zero target): the f32 gradient must meet the 1e-5 gate,
    through the ring kernels (L(u_t) written by the recompute, pointwise
    reverse step) and through the queue kernels (u_t staged in the reverse
    step)."""
    kappa, zeros, src, wav, rec, target = _grad_case(blob=False)
    steps = 30
    kw = {} if family == "ring" else dict(variant=3)
    m = st.WaveModel(kappa.shape[::-1], ckpt_every=7, **kw)
    dk, loss = m.gradient(_dev(zeros), _dev(zeros), _dev(kappa), steps, src, _dev(wav), rec, _dev(target))
    g_ref, J_ref = oracle.wave_gradient(zeros, zeros, kappa, steps, src, wav, rec, target, ckpt_every=0)
    eJ = abs(float(_host(loss)[0]) - J_ref) / abs(J_ref)
    eg = rel_l2(_host(dk), g_ref)
    print(f"gradient (zero target): loss rel err {eJ:.3e}, dkappa rel-L2 {eg:.3e}")
    assert eJ <= 1e-5 and eg <= 1e-5


def test_wave_gradient_small_residual_conditioning(st):
    """+5% blob target: the residual r = P u - d is a small difference of two
    wavefields and dkappa is linear in it, so an f32 wavefield error e moves
    dkappa by about e |d| / |r| relative (J, quadratic in r, by twice that).
    The gate is the f32 field gate 1e-5 scaled by that conditioning, both
    norms from the oracle; the binary32 storage floor of the same recursion
    is printed beside the measured error."""
    kappa, zeros, src, wav, rec, target = _grad_case(blob=True)
    steps = 30
    m = st.WaveModel(kappa.shape[::-1], ckpt_every=7)
    dk, loss = m.gradient(_dev(zeros), _dev(zeros), _dev(kappa), steps, src, _dev(wav), rec, _dev(target))
    g_ref, J_ref = oracle.wave_gradient(zeros, zeros, kappa, steps, src, wav, rec, target, ckpt_every=0)
    g_fl, _ = oracle.wave_gradient(zeros, zeros, kappa, steps, src, wav, rec, target, storage="binary32")
    cond = float(np.linalg.norm(target.astype(np.float64)) / np.sqrt(2 * J_ref))
    eJ = abs(float(_host(loss)[0]) - J_ref) / abs(J_ref)
    eg = rel_l2(_host(dk), g_ref)
    print(f"gradient (blob target): loss rel err {eJ:.3e} (gate {2e-5 * cond:.2e}), dkappa rel-L2 {eg:.3e} "
          f"(gate {1e-5 * cond:.2e}, binary32 floor {rel_l2(g_fl, g_ref):.2e}); |d|/|r| = {cond:.1f}")
    assert eJ <= 2e-5 * cond and eg <= 1e-5 * cond


def test_wave_gradient_checkpoints_bitwise_equal(st):
    kappa, zeros, src, wav, rec, target = _grad_case(n=(33, 30, 36), steps=25, seed=43)
    outs = []
    for K in (25, 7, 1, 4):
        m = st.WaveModel(kappa.shape[::-1], ckpt_every=K)
        dk, loss = m.gradient(_dev(zeros), _dev(zeros), _dev(kappa), 25, src, _dev(wav), rec, _dev(target))
        outs.append((_host(dk), float(_host(loss)[0])))
    for dk, J in outs[1:]:
        assert np.array_equal(dk, outs[0][0]) and J == outs[0][1]


def test_wave_misfit_autograd_and_fd(st):
    """torch.autograd through the adjoint sweep; directional central FD of
    the FP64 oracle's loss along a smooth direction."""
    kappa, zeros, src, wav, rec, target = _grad_case(n=(36, 34, 40), steps=28, seed=47, blob=False)
    m = st.WaveModel(kappa.shape[::-1], ckpt_every=9)
    k = _dev(kappa).requires_grad_(True)
    J = st.wave_misfit(k, m, _dev(zeros), _dev(zeros), 28, src, _dev(wav), rec, _dev(target))
    J.backward()
    g = _host(k.grad).astype(np.float64)
    d = wl.gaussian_pulse((36, 34, 40), (18, 17, 22), 5.0).astype(np.float64)
    eps = 1e-3
    kp = (kappa + eps * d).astype(np.float32)
    km = (kappa - eps * d).astype(np.float32)
    _, Jp = oracle.wave_gradient(zeros, zeros, kp, 28, src, wav, rec, target)
    _, Jm = oracle.wave_gradient(zeros, zeros, km, 28, src, wav, rec, target)
    dd = (kp.astype(np.float64) - km.astype(np.float64)) / 2   # realised f32 direction
    fd = (Jp - Jm) / 2
    ad = float(np.sum(g * dd))
    print(f"directional derivative: adjoint {ad:.9e}, central FD {fd:.9e}, rel {abs(fd - ad) / abs(ad):.3e}")
    assert abs(fd - ad) <= 1e-4 * abs(ad)


def _batched_cases(count, lo, hi, steps, seed, dtype=np.float32):
    cases = wl.batch2d(count=count, lo=lo, hi=hi, steps=steps, seed=seed)
    for c in cases:
        c.u0 = c.u0.astype(dtype)
    return cases


@pytest.mark.parametrize("dtype,bc", [("f32", "periodic"), ("f16", "zero"), ("f64", "periodic"), ("f64", "zero")])
def test_batched_matches_plain_and_oracle(st, dtype, bc):
    """Every member of a grouped batch equals the oracle and its own
    single-grid plan; in place with odd and even block counts; members
    with different fused depths (so some finish before the last launch and
    the later launches run on re-divided member tables): depth 8 (clamped
    per member for f64) and each member's own map depth (tsteps=-1)."""
    npdt = {"f32": np.float32, "f16": np.float16, "f64": np.float64}[dtype]
    cases = _batched_cases(10, 64, 400, 7, 9, npdt)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    spec = [dict(n=c.n[:2], shape=c.shape, radius=c.radius, coeffs=c.coeffs, dtype=dtype, boundary=bc)
            for c in cases]
    for opts in ({}, {"tsteps": 1}, {"tsteps": 3}, {"tsteps": 8}, {"tsteps": -1}):
        bs = st.BatchedStencil(spec, **opts)
        ins = [_dev(c.u0) for c in cases]
        outs = bs.apply(ins, 7)
        for c, o, i in zip(cases, outs, ins):
            ref = oracle.sweep(c.u0, c.coeffs, c.shape, c.radius, bcode, 7)
            assert rel_l2(_host(o).astype(np.float64), ref) <= TOL[dtype], (c.name, opts)
            plain = st.Stencil(c.n[:2], c.shape, c.radius, c.coeffs, dtype=dtype, boundary=bc,
                               tsteps=1).apply(i, 7)
            assert rel_l2(_host(o).astype(np.float64), _host(plain).astype(np.float64)) <= TOL[dtype], c.name
        for steps in (5, 6):   # in place
            ins = [_dev(c.u0) for c in cases]
            outs2 = bs.apply(ins, steps, outs=ins)
            for c, o in zip(cases, outs2):
                ref = oracle.sweep(c.u0, c.coeffs, c.shape, c.radius, bcode, steps)
                assert rel_l2(_host(o).astype(np.float64), ref) <= TOL[dtype], (c.name, steps, opts)


def test_batched_zero_steps_and_single_member(st):
    cases = _batched_cases(1, 300, 300, 4, 21)
    c = cases[0]
    bs = st.BatchedStencil([dict(n=c.n[:2], shape=c.shape, radius=c.radius, coeffs=c.coeffs)])
    u = _dev(c.u0)
    assert torch.equal(bs.apply([u], 0)[0], u)
    got = _host(bs.apply([u], 4)[0])
    assert rel_l2(got, oracle.sweep(c.u0, c.coeffs, c.shape, c.radius, wl.PERIODIC, 4)) <= 1e-5



@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_degenerate_extents(st, bc):
    """Grids with extent 1 (or a few cells) along one or two axes through
    every kernel family: the halos wrap many times (periodic) or read only
    the zero frame, and tiles are almost all overhang."""
    rng = np.random.default_rng(808)
    bcode = wl.PERIODIC if bc == "periodic" else wl.ZERO
    cases2 = [((1, 300), wl.STAR, 3, dict(variant=1, tile_x=64, tile_y=16, tsteps=2)),
              ((300, 1), wl.BOX, 2, dict(variant=1, tile_x=64, tile_y=32, tsteps=2)),
              ((1, 300), wl.BOX, 1, dict(variant=5, tile_x=256, tsteps=3)),
              ((700, 1), wl.STAR, 4, dict(variant=5, tile_x=512, tsteps=2)),
              ((2, 2), wl.STAR, 4, dict(variant=5, tile_x=256, tsteps=4))]
    for n, shape, r, kw in cases2:
        c = wl.random_unit_sum_coeffs(rng, 2, shape, r)
        u = wl.small_random_grid(rng, 2, n, np.float32, 0.0, 1.0)
        s = st.Stencil(n, shape, r, c, boundary=bc, **kw)
        got = _host(s.apply(_dev(u), 5)).astype(np.float64)
        assert rel_l2(got, oracle.sweep(u, c, shape, r, bcode, 5)) <= 1e-5, (n, kw)
    cases3 = [((1, 1, 70), wl.STAR, 4, {}), ((90, 1, 1), wl.STAR, 2, dict(variant=2, tile_y=8)),
              ((1, 40, 3), wl.BOX, 1, {}), ((8, 1, 30), wl.BOX, 1, dict(dtype="f16", variant=6, tile_y=64)),
              ((3, 2, 50), wl.BOX, 2, dict(variant=2, tile_y=16)), ((70, 1, 4), wl.BOX, 2, {})]
    for n, shape, r, kw in cases3:
        dt = kw.get("dtype", "f32")
        c = wl.random_unit_sum_coeffs(rng, 3, shape, r)
        u = wl.small_random_grid(rng, 3, n, np.float16 if dt == "f16" else np.float32, 0.0, 1.0)
        s = st.Stencil(n, shape, r, c, boundary=bc, **kw)
        got = _host(s.apply(_dev(u), 3)).astype(np.float64)
        assert rel_l2(got, oracle.sweep(u, c, shape, r, bcode, 3)) <= TOL[dt], (n, kw)
    for n, kw in [((1, 1, 40), dict(variant=4, tile_y=32)), ((50, 1, 2), dict(variant=4, tile_y=8)),
                  ((3, 60, 1), dict(variant=3, tile_y=16))]:
        kappa = (0.05 + 0.1 * rng.random(n[::-1])).astype(np.float32)
        u0 = wl.small_random_grid(rng, 3, n, np.float32, -1.0, 1.0)
        up = (u0 * np.float32(0.9)).astype(np.float32)
        m = st.WaveModel(n, boundary=bc, **kw)
        uT, uT1, _ = m.forward(_dev(u0), _dev(up), _dev(kappa), 4)
        ra, rb, _ = oracle.wave_forward(up, u0, kappa, 4, boundary=bcode)
        assert rel_l2(_host(uT), rb) <= 1e-5 and rel_l2(_host(uT1), ra) <= 1e-5, (n, kw)
    # The f64 leapfrog on the same kinds of extents (both tile heights).
    for n, ty in [((1, 1, 40), 16), ((50, 1, 2), 8), ((3, 60, 1), 16), ((2, 2, 2), 8)]:
        kappa = 0.05 + 0.1 * rng.random(n[::-1])
        u0 = wl.small_random_grid(rng, 3, n, np.float64, -1.0, 1.0)
        up = u0 * 0.9
        m = st.WaveModel(n, boundary=bc, dtype="f64", tile_y=ty)
        uT, uT1, _ = m.forward(_dev(u0), _dev(up), _dev(kappa), 4)
        ra, rb, _ = oracle.wave_forward(up, u0, kappa, 4, boundary=bcode)
        assert rel_l2(_host(uT), rb) <= TOL["f64"] and rel_l2(_host(uT1), ra) <= TOL["f64"], (n, ty)
