"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times: the wave workloads on every cell, the others on sampled
output blocks.

The oracle computes a sampled block of the final state from a sub-box that
extends R*T cells beyond it (T steps of a radius-R stencil move information
at most R cells per step), taken with wrap-around for periodic boundaries and
clipped to the grid for the zero boundary (where clipping reproduces the
zero frame exactly).  Inside the block the sub-box result equals the
full-grid result.  Tolerances as in the small parity tests.
"""
import numpy as np
import pytest
import torch

import oracle
from mathref import rel_l2
from paper_2609_06694_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def st():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_06694_amd import stencil
    return stencil


def _extract(a, lo, hi, periodic):
    """a[lo:hi] per axis (array axis order), wrapping if periodic."""
    idx = [np.arange(l, h) for l, h in zip(lo, hi)]
    if periodic:
        idx = [i % n for i, n in zip(idx, a.shape)]
    return a[np.ix_(*idx)]


def _sample_linear(case, got, starts, block, storage=None):
    """Check sampled blocks of a linear sweep's output against the oracle.
    With `storage`, also returns the storage floor on the same blocks (the
    oracle with every step rounded to that format; rounding is per cell, so
    the dependency sub-box argument holds for it too)."""
    per = case.boundary == wl.PERIODIC
    m = case.radius * case.steps
    errs, floors = [], []
    for s0 in starts:
        if per:
            lo = [s - m for s in s0]
            hi = [s + b + m for s, b in zip(s0, block)]
            sub = _extract(case.u0, lo, hi, True)
            inner = tuple(slice(m, m + b) for b in block)
        else:
            lo = [max(0, s - m) for s in s0]
            hi = [min(n, s + b + m) for s, b, n in zip(s0, block, case.u0.shape)]
            sub = case.u0[tuple(slice(l, h) for l, h in zip(lo, hi))]
            inner = tuple(slice(s - l, s - l + b) for s, l, b in zip(s0, lo, block))
        ref = oracle.sweep(sub, case.coeffs, case.shape, case.radius, wl.ZERO, case.steps)[inner]
        g = got[tuple(slice(s, s + b) for s, b in zip(s0, block))]
        errs.append(rel_l2(g.astype(np.float64), ref))
        if storage:
            fl = oracle.sweep(sub, case.coeffs, case.shape, case.radius, wl.ZERO, case.steps,
                              storage=storage)[inner]
            floors.append(rel_l2(fl, ref))
    if storage:
        return max(errs), max(floors)
    return max(errs)


def _check_fp16(tag, e, floor):
    """fp16 gate: 2e-3 rel-L2, and within 5x of the binary16 storage floor."""
    print(f"{tag} sampled rel-L2 {e:.3e}, binary16 floor {floor:.3e}, ratio {e / floor:.2f}")
    assert e <= 2e-3 and e <= 5 * floor


def test_fullsize_jacobi2d(st):
    case = wl.jacobi2d()
    s = st.Stencil(case.n[:2], "star", 1, case.coeffs)
    got = s.apply(torch.from_numpy(case.u0).cuda(), case.steps).cpu().numpy()
    ref = oracle.sweep(case.u0, case.coeffs, wl.STAR, 1, wl.PERIODIC, case.steps)
    assert rel_l2(got, ref) <= 1e-5


@pytest.mark.parametrize("dtype", [wl.F16, wl.F32])
def test_fullsize_box3d(st, dtype):
    case = wl.box3d(dtype=dtype)
    dt = "f16" if dtype == wl.F16 else "f32"
    s = st.Stencil(case.n, "box", 1, case.coeffs, dtype=dt)
    got = s.apply(torch.from_numpy(case.u0).cuda(), case.steps).cpu().numpy()
    starts = [(0, 0, 0), (507, 250, 480)]   # [z, y, x]: a corner (wraps) and a far face
    if dtype == wl.F16:
        _check_fp16("box3d f16 512^3 x50", *_sample_linear(case, got, starts, (5, 8, 8), "binary16"))
        return
    e = _sample_linear(case, got, starts, (5, 8, 8))
    print(f"box3d {dt} 512^3 x50 sampled rel-L2 {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("dtype", [wl.F16, wl.F32, wl.F64])
def test_fullsize_star3d(st, dtype):
    """The 7-point star on 512^3 x 10 steps in each storage type."""
    case = wl.star3d(dtype=dtype)
    dt = wl.DTYPE_TAGS[dtype]
    s = st.Stencil(case.n, "star", 1, case.coeffs, dtype=dt)
    got = s.apply(torch.from_numpy(case.u0).cuda(), case.steps).cpu().numpy()
    starts = [(0, 0, 0), (505, 250, 478)]
    if dtype == wl.F16:
        _check_fp16("star3d f16 512^3 x10", *_sample_linear(case, got, starts, (4, 6, 8), "binary16"))
        return
    e = _sample_linear(case, got, starts, (4, 6, 8))
    print(f"star3d {dt} 512^3 x10 sampled rel-L2 {e:.2e}")
    assert e <= {wl.F32: 1e-5, wl.F64: 1e-12}[dtype]


@pytest.mark.parametrize("shape,r", [("star", 1), ("box", 1)])
def test_fullsize_varcoef(st, shape, r):
    """Variable coefficients on 512^3 x 6 steps (f32, periodic); fields and
    data are seeded device-side draws (cell-wise unit-sum fields), sampled
    blocks are checked against the oracle on their dependency sub-box."""
    n, steps = 512, 6
    ntap = st.varcoef_taps(3, shape, r)
    g = torch.Generator(device="cuda")
    g.manual_seed(4242 + ntap)
    f = torch.rand((ntap, n, n, n), generator=g, device="cuda")
    f /= f.sum(dim=0, keepdim=True)
    u = torch.rand((n, n, n), generator=g, device="cuda")
    s = st.VarCoefStencil((n, n, n), shape, r)
    got = s.apply(u, f, steps).cpu().numpy()
    kind = wl.STAR if shape == "star" else wl.BOX
    m = r * steps
    errs = []
    for s0, blk in [((0, 0, 0), (4, 6, 8)), ((509, 250, 478), (3, 6, 8))]:
        idx = [torch.arange(a - m, a + b + m, device="cuda") % n for a, b in zip(s0, blk)]
        zz, yy, xx = torch.meshgrid(*idx, indexing="ij")
        usub = u[zz, yy, xx].cpu().numpy()
        fsub = f[:, zz, yy, xx].cpu().numpy()
        ref = oracle.varcoef_sweep(usub, fsub, kind, r, wl.ZERO, steps)
        ref = ref[m:m + blk[0], m:m + blk[1], m:m + blk[2]]
        gb = got[np.ix_(*[np.arange(a, a + b) % n for a, b in zip(s0, blk)])]
        errs.append(rel_l2(gb.astype(np.float64), ref))
    print(f"varcoef {shape}{r} 512^3 x{steps} sampled rel-L2 {max(errs):.2e}")
    assert max(errs) <= 1e-5


@pytest.mark.parametrize("dtype", [wl.F16, wl.F32])
def test_fullsize_box3d_r2(st, dtype):
    """The 125-point box on 512^3 x 10 steps (the compute-bound case)."""
    case = wl.box3d_r2(dtype=dtype)
    dt = "f16" if dtype == wl.F16 else "f32"
    s = st.Stencil(case.n, "box", 2, case.coeffs, dtype=dt)
    got = s.apply(torch.from_numpy(case.u0).cuda(), case.steps).cpu().numpy()
    starts = [(0, 0, 0), (505, 250, 478)]
    if dtype == wl.F16:
        _check_fp16("box3d r2 f16 512^3 x10", *_sample_linear(case, got, starts, (4, 6, 8), "binary16"))
        return
    e = _sample_linear(case, got, starts, (4, 6, 8))
    print(f"box3d r2 {dt} 512^3 x10 sampled rel-L2 {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("dtype", [wl.F16, wl.F32, wl.F64])
def test_fullsize_box2d(st, dtype):
    case = wl.box2d(dtype=dtype)
    dt = wl.DTYPE_TAGS[dtype]
    s = st.Stencil(case.n[:2], "box", 2, case.coeffs, dtype=dt)
    got = s.apply(torch.from_numpy(case.u0).cuda(), case.steps).cpu().numpy()
    starts = [(0, 0), (2000, 3001), (4080, 4080), (1234, 0)]
    if dtype == wl.F16:
        _check_fp16("box2d f16 4096^2 x100", *_sample_linear(case, got, starts, (16, 16), "binary16"))
        return
    e = _sample_linear(case, got, starts, (16, 16))
    print(f"box2d {dt} 4096^2 x100 sampled rel-L2 {e:.2e}")
    assert e <= {"f32": 1e-5, "f64": 1e-12}[dt]


def test_fullsize_varcoef2d(st):
    """Variable-coefficient 5-point star on 4096^2 x 20 steps (f32,
    periodic), as the benchmark runs it; sampled blocks against the oracle
    on their dependency sub-boxes."""
    n, steps, r = 4096, 20, 1
    ntap = st.varcoef_taps(2, "star", r)
    g = torch.Generator(device="cuda")
    g.manual_seed(5151)
    f = torch.rand((ntap, n, n), generator=g, device="cuda")
    f /= f.sum(dim=0, keepdim=True)
    u = torch.rand((n, n), generator=g, device="cuda")
    s = st.VarCoefStencil((n, n), "star", r)
    got = s.apply(u, f, steps).cpu().numpy()
    m = r * steps
    errs = []
    for s0, blk in [((0, 0), (16, 16)), ((4090, 2047), (6, 16)), ((1000, 4080), (16, 16))]:
        idx = [torch.arange(a - m, a + b + m, device="cuda") % n for a, b in zip(s0, blk)]
        yy, xx = torch.meshgrid(*idx, indexing="ij")
        ref = oracle.varcoef_sweep(u[yy, xx].cpu().numpy(), f[:, yy, xx].cpu().numpy(), wl.STAR, r, wl.ZERO,
                                   steps)[m:m + blk[0], m:m + blk[1]]
        gb = got[np.ix_(*[np.arange(a, a + b) % n for a, b in zip(s0, blk)])]
        errs.append(rel_l2(gb.astype(np.float64), ref))
    print(f"varcoef2d star1 4096^2 x{steps} sampled rel-L2 {max(errs):.2e}")
    assert max(errs) <= 1e-5


def test_fullsize_wave3d(st):
    """The headline workload (512^3, 20 steps, zero frame) compared with the
    oracle on every cell of u_T and u_{T-1}, with the margin printed beside
    the binary32 storage floor of the same run; and the same inputs through
    the f64 leapfrog against the same oracle result at the f64 gate."""
    case = wl.wave3d(n=512, steps=20)
    m = st.WaveModel(case.n, radius=4, boundary="zero")
    out, prev, _ = m.forward(torch.from_numpy(case.u0).cuda(), torch.from_numpy(case.u_prev).cuda(),
                             torch.from_numpy(case.kappa).cuda(), case.steps)
    got, gotp = out.cpu().numpy(), prev.cpu().numpy()
    del out, prev
    T = case.steps
    ra, rb, _ = oracle.wave_forward(case.u_prev, case.u0, case.kappa, T)
    e = max(rel_l2(got, rb), rel_l2(gotp, ra))
    del got, gotp
    torch.cuda.empty_cache()
    m64 = st.WaveModel(case.n, radius=4, boundary="zero", dtype="f64")
    o64, p64, _ = m64.forward(torch.from_numpy(case.u0).cuda().double(),
                              torch.from_numpy(case.u_prev).cuda().double(),
                              torch.from_numpy(case.kappa).cuda().double(), case.steps)
    e64 = max(rel_l2(o64.cpu().numpy(), rb), rel_l2(p64.cpu().numpy(), ra))
    del o64, p64
    torch.cuda.empty_cache()
    print(f"wave 512^3 x{T} f64 all cells: rel-L2 {e64:.3e} (gate 1e-12)")
    assert e64 <= 1e-12
    fa, fb, _ = oracle.wave_forward(case.u_prev, case.u0, case.kappa, T, storage="binary32")
    floor = max(rel_l2(fb, rb), rel_l2(fa, ra))
    print(f"wave 512^3 x{T} all cells: rel-L2 {e:.3e} (gate 1e-5, margin {1e-5 / e:.1f}x; "
          f"binary32 storage floor {floor:.3e}, ratio {e / floor:.2f})")
    assert e <= 1e-5


def test_fullsize_wave_gradient_vs_oracle(st):
    """The gradient workload at its full size and law (256^3, 200 steps,
    checkpoints every 20, Ricker source at z = 16, receivers on z = 8,
    target from the +5% blob model): dkappa and J against the FP64 oracle.

    The residual r = P u - d is a small difference of two wavefields, and
    dkappa is linear in it, so an f32 wavefield error e moves dkappa by
    about e * |d| / |r| relative (J, quadratic in r, by twice that).  The
    gate is the f32 field gate 1e-5 scaled by that conditioning, both
    norms taken from the oracle."""
    case = wl.wavegrad3d()
    T, n = case.steps, case.n
    _, _, target = oracle.wave_forward(case.u_prev, case.u0, case.kappa_true, T, src=case.src,
                                       wavelet=case.wavelet, rec_z=case.rec_z)
    target = target.astype(np.float32)
    dev = torch.device("cuda")
    z = torch.from_numpy(case.u0).to(dev)
    m = st.WaveModel(n, ckpt_every=case.ckpt_every)
    dk, loss = m.gradient(z, z, torch.from_numpy(case.kappa).to(dev), T, case.src,
                          torch.from_numpy(case.wavelet).to(dev), case.rec_z, torch.from_numpy(target).to(dev))
    got, J = dk.cpu().numpy(), float(loss.item())
    del dk, m, z
    torch.cuda.empty_cache()
    g_ref, J_ref = oracle.wave_gradient(case.u_prev, case.u0, case.kappa, T, case.src, case.wavelet,
                                        case.rec_z, target, ckpt_every=case.ckpt_every)
    cond = float(np.linalg.norm(target.astype(np.float64)) / np.sqrt(2 * J_ref))
    eg = rel_l2(got, g_ref)
    eJ = abs(J - J_ref) / J_ref
    print(f"gradient 256^3 x{T}: dkappa rel-L2 {eg:.3e} (gate {1e-5 * cond:.3e}), loss rel {eJ:.3e} "
          f"(gate {2e-5 * cond:.3e}); |d|/|r| = {cond:.1f}")
    assert eg <= 1e-5 * cond and eJ <= 2e-5 * cond


def test_fullsize_batch64_separate_launches(st):
    cases = wl.batch2d()
    errs = []
    for c in cases:
        s = st.Stencil(c.n[:2], wl.SHAPE_NAMES[c.shape], c.radius, c.coeffs)
        got = s.apply(torch.from_numpy(c.u0).cuda(), c.steps).cpu().numpy()
        ny, nx = c.u0.shape
        errs.append(_sample_linear(c, got, [(0, 0), (ny - 8, nx // 3)], (8, 8)))
    print(f"64 grids x32 sampled rel-L2 max {max(errs):.2e}")
    assert max(errs) <= 1e-5


def test_fullsize_batch64_grouped_launch(st):
    """The 64-grid workload through the grouped batched launch, as the
    benchmark runs it, on sampled blocks of every member."""
    cases = wl.batch2d()
    bs = st.BatchedStencil([dict(n=c.n[:2], shape=wl.SHAPE_NAMES[c.shape], radius=c.radius, coeffs=c.coeffs)
                            for c in cases])
    outs = bs.apply([torch.from_numpy(c.u0).cuda() for c in cases], 32)
    errs = []
    for c, o in zip(cases, outs):
        ny, nx = c.u0.shape
        errs.append(_sample_linear(c, o.cpu().numpy(), [(0, 0), (ny // 2, nx - 8)], (8, 8)))
    print(f"64 grids x32 grouped, sampled rel-L2 max {max(errs):.2e}")
    assert max(errs) <= 1e-5


def test_fullsize_wave_gradient_checkpointing(st):
    """At the full gradient size (256^3, 200 steps), checkpointing every 20
    steps gives exactly the gradient of keeping every state; the loss is the
    misfit of the traces the gradient recorded; and it agrees with the misfit
    of a plain forward run (which rounds its states in f32 arithmetic rather
    than once per step) to within the residual's conditioning."""
    case = wl.wavegrad3d()
    n = case.n
    dev = torch.device("cuda")
    kap = torch.from_numpy(case.kappa).to(dev)
    zeros = torch.zeros(n[::-1], dtype=torch.float32, device=dev)
    wav = torch.from_numpy(case.wavelet).to(dev)
    fwd = st.WaveModel(n)
    _, _, target = fwd.forward(zeros, zeros, torch.from_numpy(case.kappa_true).to(dev), case.steps,
                               src=case.src, wavelet=wav, rec_z=case.rec_z, record=True)
    target = target.contiguous()
    res = []
    for K in (20, 200):
        m = st.WaveModel(n, ckpt_every=K)
        tr = torch.empty_like(target)
        dk, loss = m.gradient(zeros, zeros, kap, case.steps, case.src, wav, case.rec_z, target, traces=tr)
        res.append((dk.cpu().numpy(), float(loss.item()), tr))
        del m
        torch.cuda.empty_cache()
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1] == res[1][1]
    assert torch.equal(res[0][2], res[1][2])
    J_own = 0.5 * float(((res[0][2].double() - target.double()) ** 2).sum().item())
    assert abs(J_own - res[0][1]) <= 1e-12 * abs(J_own)
    _, _, tr = fwd.forward(zeros, zeros, kap, case.steps, src=case.src, wavelet=wav, rec_z=case.rec_z,
                           record=True)
    J = 0.5 * float(((tr.double() - target.double()) ** 2).sum().item())
    cond = float(target.double().norm().item()) / np.sqrt(2 * J)
    print(f"gradient-path loss vs plain-forward loss: rel {abs(J - res[0][1]) / J:.2e} (gate {2e-5 * cond:.2e})")
    assert abs(J - res[0][1]) <= 2e-5 * cond * abs(J)
    g = res[0][0]
    assert np.isfinite(g).all() and np.abs(g).max() > 0
