"""The absorbing layer fused into the leapfrog kernels (forward, transposed
state map, checkpointed gradient) against the FP64 oracle's damped model.

Layer: damping gamma = sum over axes of s ((W - e) / W)^2 within W cells of
each face; step u_{t+1} = A (2u + kappa L u) - B u_prev, A = 1/(1 + gamma/2),
B = (1 - gamma/2) A.  Gates as for the plain wave: 1e-5 rel-L2 (f32)."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n,ty,zc,W,s", [((75, 41, 33), 8, 0, 6, 0.8), ((130, 37, 29), 16, 9, 5, 1.5),
                                         ((70, 66, 40), 32, 16, 10, 0.3), ((20, 12, 11), 8, 4, 3, 2.0)])
def test_sponge_forward_vs_oracle(st, n, ty, zc, W, s):
    """Damped forward with source and receiver, on tiles narrower and wider
    than the grid and with z chunks, a pulse reaching into the layer."""
    rng = np.random.default_rng(301 + W)
    nx, ny, nz = n
    kappa = rng.uniform(0.05, 0.2, (nz, ny, nx)).astype(np.float32)
    u0 = wl.gaussian_pulse(n, (nx // 3, ny // 3, nz // 2), 3.0)
    up = (u0 * np.float32(0.97)).astype(np.float32)
    steps, src, rec = 12, (nx // 2, ny // 2, nz // 2), 2
    wav = wl.ricker(steps, 4.0)
    gamma = oracle.sponge_profile((nz, ny, nx), W, s)
    m = st.WaveModel(n, tile_y=ty, zchunk=zc, sponge=(W, s))
    uT, uT1, tr = m.forward(_dev(u0), _dev(up), _dev(kappa), steps, src=src, wavelet=_dev(wav), rec_z=rec,
                            record=True)
    ra, rb, rtr = oracle.wave_forward_damped(up, u0, kappa, gamma, steps, src=src, wavelet=wav, rec_z=rec)
    e = max(rel_l2(_host(uT), rb), rel_l2(_host(uT1), ra), rel_l2(_host(tr), rtr))
    pa, pb, _ = oracle.wave_forward(up, u0, kappa, steps, src=src, wavelet=wav, rec_z=rec)
    print(f"sponge fwd {n} W={W} s={s}: rel-L2 {e:.2e} (damping changes u_T by {rel_l2(pb, rb):.2e})")
    assert e <= 1e-5
    assert rel_l2(pb, rb) > 1e-3   # the layer acts


@pytest.mark.parametrize("steps", [1, 2, 5])
def test_sponge_adjoint_vs_oracle_and_dot(st, steps):
    """Transposed damped state map against the oracle's block transpose, and
    the dot-product identity with the GPU forward."""
    rng = np.random.default_rng(311)
    n = (67, 35, 30)
    nx, ny, nz = n
    W, s = 6, 1.2
    kappa = rng.uniform(0.05, 0.2, (nz, ny, nx)).astype(np.float32)
    gamma = oracle.sponge_profile((nz, ny, nx), W, s)
    a, b, p, q = (rng.standard_normal((nz, ny, nx)).astype(np.float32) for _ in range(4))
    m = st.WaveModel(n, sponge=(W, s))
    ta, tb = m.adjoint(_dev(a), _dev(b), _dev(kappa), steps)
    ra, rb = oracle.wave_adjoint_damped(a, b, kappa, gamma, steps)
    assert rel_l2(_host(ta), ra) <= 1e-5 and rel_l2(_host(tb), rb) <= 1e-5
    fq, fp, _ = m.forward(_dev(q), _dev(p), _dev(kappa), steps)
    f64 = lambda t: _host(t).astype(np.float64)
    lhs = float(np.sum(f64(fp) * a) + np.sum(f64(fq) * b))
    rhs = float(np.sum(p.astype(np.float64) * f64(ta)) + np.sum(q.astype(np.float64) * f64(tb)))
    scale = np.sqrt(np.sum(f64(fp) ** 2) + np.sum(f64(fq) ** 2)) * np.sqrt(np.sum(a.astype(np.float64) ** 2) +
                                                                           np.sum(b.astype(np.float64) ** 2))
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_sponge_gradient_vs_oracle_and_checkpoints(st):
    """Gradient of the trace misfit of the damped model (zero target, so the
    residual is the trace itself) against the oracle at 1e-5; checkpointed
    and keep-all gradients are bitwise equal."""
    rng = np.random.default_rng(321)
    n = (40, 36, 44)
    nx, ny, nz = n
    W, s, steps = 6, 0.9, 30
    kappa = rng.uniform(0.05, 0.19, (nz, ny, nx)).astype(np.float32)
    zeros = np.zeros_like(kappa)
    gamma = oracle.sponge_profile((nz, ny, nx), W, s)
    src, rec = (nx // 2, ny // 2, 12), 6
    wav = wl.ricker(steps, 8.0)
    target = np.zeros((steps, ny, nx), dtype=np.float32)
    g_ref, J_ref = oracle.wave_gradient_damped(zeros, zeros, kappa, gamma, steps, src, wav, rec, target)
    outs = []
    for K in (7, 30):
        m = st.WaveModel(n, ckpt_every=K, sponge=(W, s))
        dk, loss = m.gradient(_dev(zeros), _dev(zeros), _dev(kappa), steps, src, _dev(wav), rec, _dev(target))
        outs.append((_host(dk), float(_host(loss)[0])))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]
    eJ = abs(outs[0][1] - J_ref) / J_ref
    eg = rel_l2(outs[0][0], g_ref)
    g_plain, _ = oracle.wave_gradient(zeros, zeros, kappa, steps, src, wav, rec, target)
    print(f"sponge gradient: loss rel {eJ:.2e}, dkappa rel-L2 {eg:.2e} (layer changes dkappa by "
          f"{rel_l2(g_plain, g_ref):.2e})")
    assert eJ <= 1e-5 and eg <= 1e-5
