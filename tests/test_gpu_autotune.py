"""GPU tests of the autotuner: it only adopts candidates that pass the
parity check against the plain single-step configuration, a planted
wrong-but-faster candidate family is rejected, and the tuned plan still
matches the FP64 oracle."""
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


def test_autotune_2d_adopts_a_passing_candidate(st):
    rng = np.random.default_rng(61)
    c = wl.random_unit_sum_coeffs(rng, 2, wl.BOX, 2)
    u = wl.small_random_grid(rng, 2, (600, 500), np.float32, 0.0, 1.0)
    s = st.Stencil((600, 500), "box", 2, c)
    stats = s.autotune()
    d = s.describe()
    print("2D tuned:", d, stats)
    assert stats["tried"] >= 8 and stats["rejected"] == 0 and d["variant"] in ("tb2d", "ym2d")
    got = s.apply(torch.from_numpy(u).cuda(), 9).cpu().numpy()
    assert rel_l2(got, oracle.sweep(u, c, wl.BOX, 2, wl.PERIODIC, 9)) <= 1e-5


def test_autotune_rejects_planted_wrong_candidates(st, monkeypatch):
    """With the fault switch, every fused-step 2D candidate (and every
    16-row 3D candidate) computes with a perturbed centre weight; all of them
    must be rejected before timing."""
    monkeypatch.setenv("STENCIL_TUNE_FAULT", "1")
    rng = np.random.default_rng(62)
    c = wl.random_unit_sum_coeffs(rng, 2, wl.STAR, 3)
    u = wl.small_random_grid(rng, 2, (700, 300), np.float32, 0.0, 1.0)
    s = st.Stencil((700, 300), "star", 3, c, boundary="zero")
    stats = s.autotune()
    d = s.describe()
    print("faulted 2D tuned:", d, stats)
    assert stats["rejected"] > 0 and d["tsteps"] == 1
    got = s.apply(torch.from_numpy(u).cuda(), 6).cpu().numpy()
    assert rel_l2(got, oracle.sweep(u, c, wl.STAR, 3, wl.ZERO, 6)) <= 1e-5


def test_autotune_3d_and_wave(st, monkeypatch):
    monkeypatch.setenv("STENCIL_TUNE_FAULT", "1")
    rng = np.random.default_rng(63)
    c = wl.random_unit_sum_coeffs(rng, 3, wl.BOX, 1)
    u = wl.small_random_grid(rng, 3, (130, 70, 90), np.float16, 0.0, 1.0)
    s = st.Stencil((130, 70, 90), "box", 1, c, dtype="f16")
    stats = s.autotune()
    print("3D tuned:", s.describe(), stats)
    assert stats["rejected"] > 0 and s.describe()["tile_y"] != 16
    got = s.apply(torch.from_numpy(u).cuda(), 3).cpu().numpy()
    assert rel_l2(got.astype(np.float64), oracle.sweep(u, c, wl.BOX, 1, wl.PERIODIC, 3)) <= 2e-3
    m = st.WaveModel((96, 64, 80))
    stats = m.autotune()
    print("wave tuned:", m.describe(), stats)
    assert stats["rejected"] > 0 and m.describe()["tile_y"] != 16


def test_autotune_batched_picks_a_batch_depth(st):
    """Tuning a batched plan tunes every member case and then the depth of
    the grouped launch itself; the tuned batch still matches the oracle."""
    cases = wl.batch2d(count=6, lo=96, hi=300, steps=9, seed=5)
    bs = st.BatchedStencil([dict(n=c.n[:2], shape=c.shape, radius=c.radius, coeffs=c.coeffs) for c in cases])
    stats = bs.autotune()
    d = bs.describe()
    print("batch tuned:", d, stats)
    assert d["variant"] == "ym2d" and d["tsteps"] in (1, 2, 3, 4, 6, 8)
    assert stats["tried"] >= 6 and stats["rejected"] == 0
    outs = bs.apply([torch.from_numpy(c.u0).cuda() for c in cases], 9)
    for c, o in zip(cases, outs):
        assert rel_l2(o.cpu().numpy(), oracle.sweep(c.u0, c.coeffs, c.shape, c.radius, wl.PERIODIC, 9)) <= 1e-5


def test_autotune_varcoef(st, monkeypatch):
    """The variable-coefficient kernel is tuned like the others: with the
    fault switch, every 16-row candidate reads the wrong fields and must be
    rejected; the tuned plan still matches the oracle (3D and 2D)."""
    monkeypatch.setenv("STENCIL_TUNE_FAULT", "1")
    rng = np.random.default_rng(64)
    n = (130, 70, 90)
    f = wl.varcoef_fields(rng, 7, n[::-1], np.float32)
    u = wl.small_random_grid(rng, 3, n, np.float32, 0.0, 1.0)
    s = st.VarCoefStencil(n, "star", 1)
    stats = s.autotune()
    d = s.describe()
    print("varcoef tuned:", d, stats)
    assert stats["tried"] >= 6 and stats["rejected"] >= 1 and d["variant"] == "vc3d" and d["tile_y"] == 8
    got = s.apply(torch.from_numpy(u).cuda(), torch.from_numpy(f).cuda(), 3).cpu().numpy()
    assert rel_l2(got, oracle.varcoef_sweep(u, f, wl.STAR, 1, wl.PERIODIC, 3)) <= 1e-5
    monkeypatch.delenv("STENCIL_TUNE_FAULT")
    f2 = wl.varcoef_fields(rng, 9, (300, 500), np.float32)
    u2 = wl.small_random_grid(rng, 2, (500, 300), np.float32, 0.0, 1.0)
    s2 = st.VarCoefStencil((500, 300), "box", 1, boundary="zero")
    stats2 = s2.autotune()
    assert stats2["tried"] >= 1 and stats2["rejected"] == 0   # one legal tile for the box
    got2 = s2.apply(torch.from_numpy(u2).cuda(), torch.from_numpy(f2).cuda(), 4).cpu().numpy()
    assert rel_l2(got2, oracle.varcoef_sweep(u2, f2, wl.BOX, 1, wl.ZERO, 4)) <= 1e-5


def test_autotune_f64(st):
    """f64 plans tune over their legal families only (2D: the row march; 3D:
    the one-step z-march) and stay at the f64 gate."""
    rng = np.random.default_rng(65)
    c = wl.random_unit_sum_coeffs(rng, 2, wl.BOX, 2)
    u = wl.small_random_grid(rng, 2, (600, 300), np.float64, 0.0, 1.0)
    s = st.Stencil((600, 300), "box", 2, c, dtype="f64")
    stats = s.autotune()
    d = s.describe()
    print("f64 2D tuned:", d, stats)
    assert stats["tried"] >= 4 and stats["rejected"] == 0 and d["variant"] == "ym2d"
    got = s.apply(torch.from_numpy(u).cuda(), 7).cpu().numpy()
    assert rel_l2(got, oracle.sweep(u, c, wl.BOX, 2, wl.PERIODIC, 7)) <= 1e-12
    c3 = wl.random_unit_sum_coeffs(rng, 3, wl.STAR, 2)
    u3 = wl.small_random_grid(rng, 3, (100, 60, 70), np.float64, 0.0, 1.0)
    s3 = st.Stencil((100, 60, 70), "star", 2, c3, dtype="f64", boundary="zero")
    stats3 = s3.autotune()
    d3 = s3.describe()
    print("f64 3D tuned:", d3, stats3)
    assert stats3["rejected"] == 0 and d3["variant"] == "zm3d" and d3["tsteps"] <= 1 and d3["tile_y"] in (8, 16)
    got3 = s3.apply(torch.from_numpy(u3).cuda(), 3).cpu().numpy()
    assert rel_l2(got3, oracle.sweep(u3, c3, wl.STAR, 2, wl.ZERO, 3)) <= 1e-12
    # A batch of f64 grids: member cases and the grouped depth are tuned at
    # the f64 gate, and the tuned batch keeps it.
    cases = wl.batch2d(count=4, lo=96, hi=260, steps=6, seed=66)
    for cb in cases:
        cb.u0 = cb.u0.astype(np.float64)
    bs = st.BatchedStencil([dict(n=cb.n[:2], shape=cb.shape, radius=cb.radius, coeffs=cb.coeffs, dtype="f64")
                            for cb in cases])
    statsb = bs.autotune()
    print("f64 batch tuned:", bs.describe(), statsb)
    assert statsb["rejected"] == 0 and bs.describe()["variant"] == "ym2d"
    outs = bs.apply([torch.from_numpy(cb.u0).cuda() for cb in cases], 6)
    for cb, o in zip(cases, outs):
        assert rel_l2(o.cpu().numpy(), oracle.sweep(cb.u0, cb.coeffs, cb.shape, cb.radius, wl.PERIODIC, 6)) <= 1e-12


def test_autotune_f64_wave(st, monkeypatch):
    """The FP64 leapfrog tunes tile height and plane chunk within its own
    family; the planted wrong candidates (16-row tiles) are rejected at the
    f64 gate, and the tuned plan stays at the oracle's values."""
    monkeypatch.setenv("STENCIL_TUNE_FAULT", "1")
    n = (96, 64, 80)
    m = st.WaveModel(n, dtype="f64", boundary="zero")
    stats = m.autotune()
    d = m.describe()
    print("f64 wave tuned:", d, stats)
    assert stats["rejected"] > 0 and d["variant"] == "wave3d" and d["tile_y"] == 8 and d["tsteps"] <= 1
    monkeypatch.delenv("STENCIL_TUNE_FAULT")
    m2 = st.WaveModel(n, dtype="f64", boundary="zero")
    stats2 = m2.autotune()
    d2 = m2.describe()
    print("f64 wave tuned (no fault):", d2, stats2)
    assert stats2["rejected"] == 0 and d2["variant"] == "wave3d" and d2["tile_y"] in (8, 16)
    rng = np.random.default_rng(67)
    kappa = rng.uniform(0.05, 0.2, n[::-1])
    u0 = wl.gaussian_pulse(n, (40, 30, 35), 3.0).astype(np.float64)
    up = u0 * 0.97
    uT, uT1, _ = m2.forward(torch.from_numpy(u0).cuda(), torch.from_numpy(up).cuda(),
                            torch.from_numpy(kappa).cuda(), 5)
    ra, rb, _ = oracle.wave_forward(up, u0, kappa, 5)
    assert rel_l2(uT.cpu().numpy(), rb) <= 1e-12 and rel_l2(uT1.cpu().numpy(), ra) <= 1e-12


def test_autotune_reverse_step(st, monkeypatch):
    """The reverse (adjoint/gradient) step has its own tuned map cell: the
    planted fault (16-row candidates, shifted centre weight of L^T) is
    rejected before timing, and the tuned plan's gradient matches the
    untuned plan's and the FP64 oracle."""
    monkeypatch.setenv("STENCIL_TUNE_FAULT", "1")
    rng = np.random.default_rng(64)
    nx, ny, nz = 72, 60, 88
    steps = 24
    kappa = rng.uniform(0.05, 0.19, (nz, ny, nx)).astype(np.float32)
    zeros = np.zeros_like(kappa)
    src, rec = (nx // 2, ny // 2, 20), 9
    wav = wl.ricker(steps, 8.0)
    target = np.zeros((steps, ny, nx), np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def grad(m):
        dk, loss = m.gradient(dev(zeros), dev(zeros), dev(kappa), steps, src, dev(wav), rec, dev(target))
        return dk.cpu().numpy(), float(loss.cpu().numpy()[0])

    base = st.WaveModel((nx, ny, nz), ckpt_every=6)
    g0, J0 = grad(base)
    m = st.WaveModel((nx, ny, nz), ckpt_every=6)
    before = m.describe_reverse()
    stats = m.autotune()
    after = m.describe_reverse()
    print("reverse step:", before, "->", after, stats)
    assert stats["rejected"] > 0 and after["tile_y"] != 16 and after["variant"] == "wave3d_lds"
    g1, J1 = grad(m)
    g_ref, J_ref = oracle.wave_gradient(zeros, zeros, kappa, steps, src, wav, rec, target, ckpt_every=0)
    print(f"tuned vs untuned dkappa rel-L2 {rel_l2(g1, g0):.2e}; vs oracle {rel_l2(g1, g_ref):.2e}")
    assert rel_l2(g1, g0) <= 1e-6 and abs(J1 - J0) <= 1e-6 * abs(J0)
    assert rel_l2(g1, g_ref) <= 1e-5 and abs(J1 - J_ref) <= 1e-5 * abs(J_ref)
