"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, and rejects bad arguments with the
documented status codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2609_06694_amd import _abi
from paper_2609_06694_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libstencil.so not built")
    return _abi.lib()


def header_functions():
    text = open(os.path.join(ROOT, "include", "stencil.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stencil_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    declared = header_functions()
    assert set(declared) == set(_abi.EXPORTED)
    for name in declared:
        assert hasattr(L, name), name
    assert b"gfx950" in L.stencil_version()


def _prob(ndim=2, n=(64, 48, 1), shape=0, r=1, coeffs="ok", dtype=0, bc=0, update=0):
    keep = []
    if isinstance(coeffs, str):
        c = wl.random_unit_sum_coeffs(np.random.default_rng(0), ndim, shape, r)
    else:
        c = coeffs
    ptr = None
    if c is not None:
        c = np.ascontiguousarray(c, dtype=np.float32)
        keep.append(c)
        ptr = c.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    p = _abi.StProblem(ndim, (ctypes.c_int64 * 3)(*n), shape, r, ptr, dtype, bc, update)
    return p, keep


def _plan(L, p, opts=None):
    h = ctypes.c_void_p()
    st = L.stencil_plan(ctypes.byref(p), ctypes.byref(opts) if opts is not None else None, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw,code", [
    (dict(ndim=4), _abi.ST_EINVAL),
    (dict(shape=7), _abi.ST_EINVAL),
    (dict(dtype=3), _abi.ST_EINVAL),
    (dict(bc=9), _abi.ST_EINVAL),
    (dict(r=0), _abi.ST_EINVAL),
    (dict(r=5), _abi.ST_EINVAL),
    (dict(coeffs=None), _abi.ST_EINVAL),
    (dict(n=(64, 48, 2)), _abi.ST_ESHAPE),
    (dict(n=(0, 48, 1)), _abi.ST_ESHAPE),
    (dict(n=(1 << 25, 4, 1)), _abi.ST_ESHAPE),
    # a 4 GiB plane overflows the 32-bit in-plane byte offsets of the plane marches
    (dict(ndim=3, n=(32768, 32768, 2)), _abi.ST_ESHAPE),
    (dict(ndim=3, n=(23200, 23200, 2), dtype=2), _abi.ST_ESHAPE),
    (dict(n=(40000, 40000, 1), update=2, coeffs=None), _abi.ST_ESHAPE),
    (dict(shape=1, r=3), _abi.ST_EUNSUPPORTED),
    (dict(ndim=3, n=(8, 8, 8), shape=1, r=3), _abi.ST_EUNSUPPORTED),
    (dict(ndim=3, n=(8, 8, 8), update=1, coeffs=None, dtype=1), _abi.ST_EUNSUPPORTED),
    (dict(ndim=2, n=(8, 8, 1), update=1, coeffs=None), _abi.ST_EUNSUPPORTED),
])
def test_plan_validation_codes(L, kw, code):
    p, keep = _prob(**kw)
    st, h = _plan(L, p)
    assert st == code, L.stencil_last_error()
    assert not h.value
    assert L.stencil_last_error() != b""


@pytest.mark.parametrize("kw", [dict(ndim=3, n=(32768, 32768, 2), dtype=1),   # 2 GiB planes
                                dict(n=(40000, 40000, 1)),                      # 2D linear: cells < 2^31
                                dict(n=(32000, 32000, 1), update=2, coeffs=None, dtype=1)])
def test_plan_accepts_large_planes(L, kw):
    p, keep = _prob(**kw)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK, L.stencil_last_error()
    L.stencil_plan_destroy(h)


def test_star_rejects_off_axis_coefficients(L):
    c = np.zeros(9, dtype=np.float32)
    c[0] = 0.5   # corner (dy=-1, dx=-1) is outside the star
    p, keep = _prob(coeffs=c)
    st, _ = _plan(L, p)
    assert st == _abi.ST_EINVAL
    c[0] = np.nan
    p, keep = _prob(shape=1, coeffs=c)
    assert _plan(L, p)[0] == _abi.ST_EINVAL


def test_plan_describe_and_workspace(L):
    p, keep = _prob(n=(512, 512, 1))
    st, h = _plan(L, p)
    assert st == _abi.ST_OK
    v, tx, ty, k, zc = (ctypes.c_int32() for _ in range(5))
    assert L.stencil_plan_describe(h, ctypes.byref(v), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(k),
                                   ctypes.byref(zc)) == _abi.ST_OK
    assert v.value == _abi.ST_VARIANT_TB2D and 8 <= tx.value <= 512 and k.value >= 1
    assert zc.value in (0, 4, 8, 16)   # waves per tile
    assert L.stencil_workspace_bytes(h, 10, 0) == 512 * 512 * 4
    assert L.stencil_workspace_bytes(None, 10, 0) == 0
    L.stencil_plan_destroy(h)
    L.stencil_plan_destroy(None)   # NULL-safe


def test_wave_plan_gradient_workspace(L):
    p, keep = _prob(ndim=3, n=(32, 24, 40), update=1, coeffs=None, bc=1, r=4)
    opts = _abi.StPlanOpts(0, 0, 0, 0, 0, 7)
    st, h = _plan(L, p, opts)
    assert st == _abi.ST_OK, L.stencil_last_error()
    cells = 32 * 24 * 40
    need = L.stencil_workspace_bytes(h, 30, 1)
    # 2*(S-1) checkpoints + K states + 3 scratch + 2 adjoint grids + traces
    S, K = 5, 7
    assert need >= (2 * (S - 1) + K + 5) * cells * 4 + 30 * 32 * 24 * 4
    L.stencil_plan_destroy(h)


def test_plan_options_validated(L):
    p, keep = _prob(n=(256, 256, 1))
    assert _plan(L, p, _abi.StPlanOpts(1, 4, 16, 1, 0, 0))[0] == _abi.ST_EINVAL   # tile_x < 8
    assert _plan(L, p, _abi.StPlanOpts(1, 64, 16, 1, 12, 0))[0] == _abi.ST_EINVAL  # waves per tile
    assert _plan(L, p, _abi.StPlanOpts(0, 0, 0, 17, 0, 0))[0] == _abi.ST_EINVAL   # depth
    assert _plan(L, p, _abi.StPlanOpts(2, 0, 0, 0, 0, 0))[0] == _abi.ST_EINVAL    # 3D family on 2D
    assert _plan(L, p, _abi.StPlanOpts(0, 512, 512, 16, 0, 0))[0] == _abi.ST_EINVAL  # LDS budget
    st, h = _plan(L, p, _abi.StPlanOpts(1, 128, 16, 2, 0, 0))
    assert st == _abi.ST_OK
    L.stencil_plan_destroy(h)
    st, h = _plan(L, p, _abi.StPlanOpts(1, 44, 44, 10, 16, 0))   # 64 x 64 window, 16 waves
    assert st == _abi.ST_OK
    L.stencil_plan_destroy(h)


def test_apply_argument_errors_before_device(L):
    p, keep = _prob(n=(64, 48, 1))
    st, h = _plan(L, p)
    assert st == _abi.ST_OK
    fake = ctypes.c_void_p(0x1000)
    assert L.stencil_apply(None, fake, fake, 1, None, None, 0, None) == _abi.ST_EINVAL
    assert L.stencil_apply(h, None, fake, 1, None, None, 0, None) == _abi.ST_EINVAL
    assert L.stencil_apply(h, fake, fake, -1, None, None, 0, None) == _abi.ST_EINVAL
    assert L.stencil_apply(h, fake, ctypes.c_void_p(0x2000), 3, None, None, 0, None) == _abi.ST_EWORKSPACE
    wa = _abi.StWaveArgs()
    assert L.stencil_apply(h, fake, fake, 1, ctypes.byref(wa), None, 0, None) == _abi.ST_EINVAL
    assert L.stencil_wave_gradient(h, fake, None, 3, fake, fake, None, 0, None) == _abi.ST_EINVAL
    L.stencil_plan_destroy(h)


def test_wave_argument_errors_before_device(L):
    p, keep = _prob(ndim=3, n=(16, 16, 16), update=1, coeffs=None, bc=1, r=4)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK
    fake = ctypes.c_void_p(0x1000)
    assert L.stencil_apply(h, fake, fake, 1, None, None, 0, None) == _abi.ST_EINVAL
    wa = _abi.StWaveArgs(ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), (ctypes.c_int64 * 3)(99, 0, 0),
                         None, -1, None, None)
    assert L.stencil_apply(h, fake, fake, 1, ctypes.byref(wa), None, 0, None) == _abi.ST_EINVAL  # source
    wa = _abi.StWaveArgs(fake, ctypes.c_void_p(0x4000), (ctypes.c_int64 * 3)(-1, 0, 0), None, -1, None, None)
    assert L.stencil_apply(h, fake, ctypes.c_void_p(0x5000), 1, ctypes.byref(wa), None, 0, None) == _abi.ST_EINVAL
    wa = _abi.StWaveArgs(ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), (ctypes.c_int64 * 3)(-1, 0, 0),
                         None, 99, None, None)
    assert L.stencil_apply(h, fake, fake, 1, ctypes.byref(wa), None, 0, None) == _abi.ST_EINVAL  # receiver
    L.stencil_plan_destroy(h)


def test_f64_wave_plan_forward_only(L):
    """An f64 wave plan is accepted for the forward leapfrog (the FP64 z-march
    family, 16-row tiles by default; 32-row tiles and fused steps illegal);
    the adjoint and the gradient refuse it before any device work, and the
    absorbing layer still needs the zero frame."""
    p, keep = _prob(ndim=3, n=(40, 24, 16), update=1, coeffs=None, dtype=2, r=4)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK, L.stencil_last_error()
    v, tx, ty, k, zc = (ctypes.c_int32() for _ in range(5))
    assert L.stencil_plan_describe(h, ctypes.byref(v), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(k),
                                   ctypes.byref(zc)) == _abi.ST_OK
    assert (v.value, tx.value, ty.value, k.value) == (_abi.ST_VARIANT_WAVE3D, 0, 16, 1)
    assert L.stencil_workspace_bytes(h, 3, 0) == 40 * 24 * 16 * 8
    fake = ctypes.c_void_p(0x1000)
    wa = _abi.StWaveArgs(ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), (ctypes.c_int64 * 3)(-1, 0, 0),
                         None, -1, None, None)
    assert L.stencil_apply_adjoint(h, fake, ctypes.c_void_p(0x2000), 1, ctypes.byref(wa), None, 0,
                                   None) == _abi.ST_EUNSUPPORTED
    assert L.stencil_wave_gradient(h, fake, ctypes.byref(wa), 3, fake, fake, None, 0, None) == _abi.ST_EUNSUPPORTED
    assert L.stencil_workspace_bytes(h, 0, 2) >= 5 * 40 * 24 * 16 * 8   # autotune scratch in binary64
    L.stencil_plan_destroy(h)
    for opts in (_abi.StPlanOpts(4, 0, 32, 1, 0, 0), _abi.StPlanOpts(3, 0, 32, 1, 0, 0),
                 _abi.StPlanOpts(3, 0, 8, 2, 0, 0), _abi.StPlanOpts(3, 2, 8, 1, 0, 0)):
        assert _plan(L, p, opts)[0] == _abi.ST_EINVAL
    st, h = _plan(L, p, _abi.StPlanOpts(3, 0, 8, 1, 8, 0))
    assert st == _abi.ST_OK
    L.stencil_plan_destroy(h)
    p, keep = _prob(ndim=3, n=(40, 24, 16), update=1, coeffs=None, dtype=2, r=4, bc=_abi.ST_PERIODIC)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK
    wa = _abi.StWaveArgs(ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), (ctypes.c_int64 * 3)(-1, 0, 0),
                         None, -1, None, None, 3, ctypes.c_float(0.5))
    assert L.stencil_apply(h, fake, ctypes.c_void_p(0x2000), 1, ctypes.byref(wa), None, 0,
                           None) == _abi.ST_EUNSUPPORTED
    L.stencil_plan_destroy(h)


def test_batched_plan_host_checks(L):
    cases = wl.batch2d(count=6, lo=64, hi=200, steps=4)
    keep = []
    arr = (_abi.StProblem * len(cases))()
    for i, c in enumerate(cases):
        cc = np.ascontiguousarray(c.coeffs)
        keep.append(cc)
        arr[i] = _abi.StProblem(2, (ctypes.c_int64 * 3)(*c.n), c.shape, c.radius,
                                cc.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 0, 0, 0)
    h = ctypes.c_void_p()
    assert L.stencil_plan_batched(arr, len(cases), None, ctypes.byref(h)) == _abi.ST_OK
    assert L.stencil_workspace_bytes(h, 4, 0) >= sum(c.cells * 4 for c in cases)
    fake = (ctypes.c_void_p * len(cases))(*([0x1000] * len(cases)))
    assert L.stencil_apply_batched(h, fake, fake, -2, None, 0, None) == _abi.ST_EINVAL
    assert L.stencil_apply_batched(h, fake, fake, 4, None, 0, None) == _abi.ST_EWORKSPACE
    assert L.stencil_apply(h, fake[0], fake[0], 1, None, None, 0, None) == _abi.ST_EINVAL
    L.stencil_plan_destroy(h)
    # Each member's own map depth (tsteps = -1): the plan reports -1, and
    # members that finish early add member tables to the workspace; below
    # -1 is rejected.
    grids = sum((c.cells * 4 + 255) // 256 * 256 for c in cases)
    for k, code in ((-1, _abi.ST_OK), (-2, _abi.ST_EINVAL), (8, _abi.ST_OK)):
        o = _abi.StPlanOpts(0, 0, 0, k, 0, 0)
        hk = ctypes.c_void_p()
        assert L.stencil_plan_batched(arr, len(cases), ctypes.byref(o), ctypes.byref(hk)) == code, k
        if code != _abi.ST_OK:
            continue
        ts = ctypes.c_int32()
        L.stencil_plan_describe(hk, None, None, None, ctypes.byref(ts), None)
        assert ts.value == k
        assert L.stencil_workspace_bytes(hk, 32, 0) > grids
        L.stencil_plan_destroy(hk)
    arr[2].dtype = 1   # mixed storage types are rejected
    assert L.stencil_plan_batched(arr, len(cases), None, ctypes.byref(h)) == _abi.ST_EINVAL
    assert L.stencil_plan_batched(arr, 0, None, ctypes.byref(h)) == _abi.ST_EINVAL


def test_dispatch_cache_file_overrides_default(tmp_path):
    """A tuning-cache line for a case key replaces the compiled-in entry
    (checked in a fresh process, since the map loads the file once)."""
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    # ndim shape r dtype bc update size_class slab variant tile_x tile_y tsteps zchunk
    cache.write_text("2 0 1 0 0 0 0 0 1 128 16 3 0\n")
    code = (
        "import ctypes, numpy as np\n"
        "from paper_2609_06694_amd import _abi\n"
        "L=_abi.lib()\n"
        "c=np.zeros(9,np.float32); c[4]=1\n"
        "p=_abi.StProblem(2,(ctypes.c_int64*3)(300,200,1),0,1,c.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),0,0,0)\n"
        "h=ctypes.c_void_p(); assert L.stencil_plan(ctypes.byref(p),None,ctypes.byref(h))==0\n"
        "v,tx,ty,k,z=(ctypes.c_int32() for _ in range(5))\n"
        "L.stencil_plan_describe(h,ctypes.byref(v),ctypes.byref(tx),ctypes.byref(ty),ctypes.byref(k),ctypes.byref(z))\n"
        "print(v.value,tx.value,ty.value,k.value)\n")
    env = dict(os.environ, STENCIL_TUNE_CACHE=str(cache), PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, cwd=ROOT)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "128", "16", "3"]


def test_f64_plan_uses_zmarch_with_short_tiles(L):
    """A 3D f64 linear plan is accepted and dispatched to the z-march with
    8- or 16-row tiles (the f64 kernels hold twice the registers)."""
    p, keep = _prob(ndim=3, n=(64, 40, 30), shape=1, r=1, dtype=2)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK, L.stencil_last_error()
    v, tx, ty, k, z = (ctypes.c_int32() for _ in range(5))
    L.stencil_plan_describe(h, ctypes.byref(v), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(k), ctypes.byref(z))
    assert v.value == _abi.ST_VARIANT_ZM3D and ty.value in (8, 16) and k.value <= 1
    L.stencil_plan_destroy(h)


def test_f64_2d_plan_uses_row_march_and_batches(L):
    """2D f64 sweeps go to the row march (the only 2D family with an f64
    path); a batched plan accepts f64 members, and needs them all f64."""
    p, keep = _prob(ndim=2, n=(300, 200, 1), shape=0, r=2, dtype=2)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK, L.stencil_last_error()
    v = ctypes.c_int32()
    L.stencil_plan_describe(h, ctypes.byref(v), None, None, None, None)
    assert v.value == 5
    L.stencil_plan_destroy(h)
    arr = (_abi.StProblem * 2)(p, p)
    hb = ctypes.c_void_p()
    assert L.stencil_plan_batched(arr, 2, None, ctypes.byref(hb)) == _abi.ST_OK, L.stencil_last_error()
    L.stencil_plan_destroy(hb)
    p32, keep32 = _prob(ndim=2, n=(300, 200, 1), shape=0, r=2, dtype=0)
    arr = (_abi.StProblem * 2)(p, p32)
    hb = ctypes.c_void_p()
    assert L.stencil_plan_batched(arr, 2, None, ctypes.byref(hb)) == _abi.ST_EINVAL
    assert not hb.value


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_builtin_laplacian_weight_sum_is_exactly_zero(L, r):
    """The built-in order-2r Laplacian annihilates constants, so the weight
    sum its difference-form kernels add back is exactly 0, although the sum
    of its f32-rounded weights is not (for r >= 2); its weights are the
    oracle's FP64 table rounded to f32."""
    import oracle
    p, keep = _prob(ndim=3, n=(16, 16, 16), update=1, coeffs=None, bc=1, r=r)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK
    w = (2 * r + 1) ** 3
    dense = np.zeros(w, dtype=np.float32)
    s = ctypes.c_double(1.0)
    assert L.stencil_plan_coefficients(h, dense.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w,
                                       ctypes.byref(s)) == _abi.ST_OK
    assert s.value == 0.0
    assert np.array_equal(dense, oracle.laplacian3d(r).astype(np.float32))
    if r >= 2:
        assert float(np.sum(dense.astype(np.float64))) != 0.0
    L.stencil_plan_destroy(h)


def test_plan_coefficients_of_given_weights(L):
    """A plan with given weights reports them unchanged, and their FP64 sum
    rounded to f32; NULL and batched plans are rejected."""
    p, keep = _prob(ndim=2, n=(64, 48, 1), shape=1, r=2)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK
    dense = np.zeros(25, dtype=np.float32)
    s = ctypes.c_double()
    assert L.stencil_plan_coefficients(h, dense.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 25,
                                       ctypes.byref(s)) == _abi.ST_OK
    assert np.array_equal(dense, keep[0])
    assert s.value == float(np.float32(np.sum(keep[0].astype(np.float64))))
    assert L.stencil_plan_coefficients(h, None, -1, None) == _abi.ST_EINVAL
    assert L.stencil_plan_coefficients(None, None, 0, None) == _abi.ST_EINVAL
    L.stencil_plan_destroy(h)


def test_binding_rejects_misshaped_wave_and_batch_operands(L):
    """The Python binding checks every operand's shape and length before any
    call reaches the device (an undersized buffer would be read or written
    out of bounds by the kernels)."""
    import torch
    from paper_2609_06694_amd import stencil
    n = (12, 10, 9)
    m = stencil.WaveModel(n)
    good = torch.zeros(n[::-1])
    bad = torch.zeros((9, 10, 11))
    with pytest.raises(ValueError, match="shape"):
        m.forward(bad, good, good, 3)
    with pytest.raises(ValueError, match="shape"):
        m.forward(good, bad, good, 3)
    with pytest.raises(ValueError, match="kappa"):
        m.forward(good, good, bad, 3)
    with pytest.raises(ValueError, match="at least 3"):
        m.forward(good, good, good, 3, src=(1, 1, 1), wavelet=torch.zeros(2))
    with pytest.raises(ValueError, match="wavelet"):
        m.forward(good, good, good, 3, src=(1, 1, 1))
    with pytest.raises(ValueError, match="shape"):
        m.adjoint(bad, good, good, 3)
    with pytest.raises(ValueError, match="target"):
        m.gradient(good, good, good, 3, (1, 1, 1), torch.zeros(3), 2, torch.zeros((3, 10, 11)))
    with pytest.raises(ValueError, match="rec_z"):
        m.gradient(good, good, good, 3, (1, 1, 1), torch.zeros(3), 9, torch.zeros((3, 10, 12)))
    with pytest.raises(ValueError, match="device"):   # right shapes, host memory
        m.forward(good, good, good, 3)
    bs = stencil.BatchedStencil([dict(n=(20, 16), shape="star", radius=1, coeffs=np.full(9, 0.1, np.float32) *
                                      np.array([0, 1, 0, 1, 1, 1, 0, 1, 0], np.float32))])
    with pytest.raises(ValueError):
        bs.apply([torch.zeros((16, 20))], 2)   # host tensor
    with pytest.raises(ValueError, match="one output"):
        bs.apply([torch.zeros((16, 20))], 2, outs=[])


def test_binding_f64_wave_operand_types(L):
    """An f64 wave model takes float64 state, kappa, wavelet and traces
    (float32 target), checked on the host; other storage types are refused."""
    import torch
    from paper_2609_06694_amd import stencil
    n = (12, 10, 9)
    with pytest.raises(ValueError, match="f32 or f64"):
        stencil.WaveModel(n, dtype="f16")
    m = stencil.WaveModel(n, dtype="f64")
    assert m.describe()["variant"] == "wave3d"
    g64 = torch.zeros(n[::-1], dtype=torch.float64)
    g32 = torch.zeros(n[::-1], dtype=torch.float32)
    with pytest.raises(ValueError, match="float64"):
        m.forward(g32, g64, g64, 3)
    with pytest.raises(ValueError, match="float64"):
        m.forward(g64, g64, g32, 3)
    with pytest.raises(ValueError, match="float64"):
        m.forward(g64, g64, g64, 3, src=(1, 1, 1), wavelet=torch.zeros(3))
    with pytest.raises(ValueError, match="device"):   # right types and shapes, host memory
        m.forward(g64, g64, g64, 3, src=(1, 1, 1), wavelet=torch.zeros(3, dtype=torch.float64))


def test_sponge_argument_checks_before_device(L):
    """The absorbing layer needs the zero frame and the LDS-ring kernels;
    width and strength are range-checked on the host."""
    fake = ctypes.c_void_p(0x1000)

    def wa(width, strength):
        return _abi.StWaveArgs(ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), (ctypes.c_int64 * 3)(-1, 0, 0),
                               None, -1, None, None, width, strength)

    p, keep = _prob(ndim=3, n=(32, 24, 20), update=1, coeffs=None, bc=1, r=4)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK
    for width, strength in ((11, 0.5), (-1, 0.5), (4, -0.1), (4, float("nan")), (4, 5.0)):
        assert L.stencil_apply(h, fake, ctypes.c_void_p(0x2000), 2, ctypes.byref(wa(width, strength)), None, 0,
                               None) == _abi.ST_EINVAL, (width, strength)
        assert L.stencil_apply_adjoint(h, fake, ctypes.c_void_p(0x2000), 2, ctypes.byref(wa(width, strength)),
                                       None, 0, None) == _abi.ST_EINVAL
    L.stencil_plan_destroy(h)
    p, keep = _prob(ndim=3, n=(32, 24, 20), update=1, coeffs=None, bc=0, r=4)   # periodic
    st, h = _plan(L, p)
    assert L.stencil_apply(h, fake, ctypes.c_void_p(0x2000), 2, ctypes.byref(wa(4, 0.5)), None, 0,
                           None) == _abi.ST_EUNSUPPORTED
    L.stencil_plan_destroy(h)
    p, keep = _prob(ndim=3, n=(32, 24, 20), update=1, coeffs=None, bc=1, r=4)
    st, h = _plan(L, p, _abi.StPlanOpts(_abi.ST_VARIANT_WAVE3D, 0, 0, 0, 0, 0))   # partial-sum family
    assert st == _abi.ST_OK
    assert L.stencil_apply(h, fake, ctypes.c_void_p(0x2000), 2, ctypes.byref(wa(4, 0.5)), None, 0,
                           None) == _abi.ST_EUNSUPPORTED
    L.stencil_plan_destroy(h)


def test_packed_half_variant_needs_even_fp16_box(L):
    """The packed-half 3D box kernel takes fp16 boxes of radius 1 or 2 with
    an even nx only; other cases reject it as a plan option."""
    ok, keep = _prob(ndim=3, n=(64, 20, 10), shape=1, r=1, dtype=1)
    st, h = _plan(L, ok, _abi.StPlanOpts(_abi.ST_VARIANT_ZM3D_H2, 0, 16, 0, 0, 0))
    assert st == _abi.ST_OK
    v = ctypes.c_int32()
    L.stencil_plan_describe(h, ctypes.byref(v), None, None, None, None)
    assert v.value == _abi.ST_VARIANT_ZM3D_H2
    L.stencil_plan_destroy(h)
    r2, keep3 = _prob(ndim=3, n=(64, 20, 10), shape=1, r=2, dtype=1)
    st, h = _plan(L, r2, _abi.StPlanOpts(_abi.ST_VARIANT_ZM3D_H2, 0, 16, 0, 0, 0))
    assert st == _abi.ST_OK
    L.stencil_plan_destroy(h)
    assert _plan(L, r2, _abi.StPlanOpts(_abi.ST_VARIANT_ZM3D_H2, 0, 12, 0, 0, 0))[0] == _abi.ST_EINVAL
    for kw in (dict(n=(63, 20, 10), dtype=1), dict(n=(64, 20, 10), dtype=0), dict(n=(64, 20, 10), dtype=2, r=2)):
        p, keep2 = _prob(ndim=3, shape=1, **dict(dict(r=1), **kw))
        assert _plan(L, p, _abi.StPlanOpts(_abi.ST_VARIANT_ZM3D_H2, 0, 16, 0, 0, 0))[0] == _abi.ST_EINVAL, kw


def test_reverse_step_has_its_own_map_cell(tmp_path):
    """A wave plan's adjoint/gradient step reads the map cell of the reverse
    key (update value 3 next to the forward key's 1): a cache line for it
    changes the reverse configuration and leaves the forward one alone; an
    illegal line falls back to the compiled-in default."""
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    # 256^3 is size class 3; the forward key (update 1) is not in the file.
    cache.write_text("3 0 4 0 1 3 3 0 4 0 16 1 48\n")
    code = (
        "from paper_2609_06694_amd import stencil as st\n"
        "m=st.WaveModel((256,256,256)); f=m.describe(); r=m.describe_reverse()\n"
        "print(r['variant'], r['tile_y'], r['zchunk'], f['variant'])\n")
    env = dict(os.environ, STENCIL_TUNE_CACHE=str(cache), PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, cwd=ROOT)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["wave3d_lds", "16", "48", "wave3d_lds"]
    cache.write_text("3 0 4 0 1 3 3 0 4 0 12 1 48\n")   # 12-row tiles do not exist
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, cwd=ROOT)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split()[:2] == ["wave3d_lds", "32"]


def test_describe_reverse_needs_a_wave_plan(L):
    p, keep = _prob(ndim=3, n=(64, 40, 30), shape=0, r=1)
    st, h = _plan(L, p)
    assert st == _abi.ST_OK
    v = ctypes.c_int32()
    assert L.stencil_plan_describe_reverse(h, ctypes.byref(v), None, None, None, None) == _abi.ST_EINVAL
    assert b"wave" in L.stencil_last_error()
    L.stencil_plan_destroy(h)
    assert L.stencil_plan_describe_reverse(None, None, None, None, None, None) == _abi.ST_EINVAL


@pytest.mark.parametrize("tsteps", [0, 1, 3, 8, -1])
def test_batched_schedule_tables_check_out(tsteps):
    """The grouped launch's schedule (the same host code that builds and
    checks the apply's member tables): one launch per time block of the
    deepest-running member, a new table where the set of running members
    changes, every table's workgroup ranges contiguous (checked inside).
    Host only."""
    from paper_2609_06694_amd import stencil as st
    cases = wl.batch2d(count=40, lo=64, hi=1500, steps=4)
    spec = [dict(n=c.n[:2], shape=wl.SHAPE_NAMES[c.shape], radius=c.radius, coeffs=c.coeffs) for c in cases]
    bs = st.BatchedStencil(spec, **({"tsteps": tsteps} if tsteps else {}))
    for steps in (1, 5, 7, 32, 33):
        for cus in (1, 256):
            sc = bs.schedule(steps, cus)
            assert sc["launches"] >= 1 and sc["tables"] >= 1 and sc["workgroups"] >= sc["launches"]
            if tsteps > 0:
                assert sc["launches"] == -(-steps // tsteps)
            if tsteps == 1:
                assert sc["tables"] == 1
    if tsteps == -1:   # members at their own depths finish at different launches
        assert bs.schedule(32, 256)["tables"] > 1
    with pytest.raises(_abi.StencilError):
        bs.schedule(0, 256)


def test_box_slab_dispatch_marches_y_within_4gib():
    """A 125-point box on a slab with few z planes dispatches the march along
    y by default; a slab whose whole grid exceeds 4 GiB (the y march
    addresses x-z planes with 32-bit offsets) falls back to the z-march; an
    explicit y march is refused there and for stars."""
    from paper_2609_06694_amd import stencil as st
    c = wl.random_unit_sum_coeffs(np.random.default_rng(3), 3, wl.BOX, 2)
    assert st.Stencil((4096, 4096, 8), "box", 2, c).describe()["variant"] == "ym3d"
    assert st.Stencil((512, 512, 512), "box", 2, c).describe()["variant"] == "zm3d"
    assert st.Stencil((32768, 8192, 8), "box", 2, c).describe()["variant"] == "zm3d"
    with pytest.raises(_abi.StencilError):
        st.Stencil((32768, 8192, 8), "box", 2, c, variant=10)
    cs = wl.random_unit_sum_coeffs(np.random.default_rng(4), 3, wl.STAR, 1)
    with pytest.raises(_abi.StencilError):
        st.Stencil((300, 200, 9), "star", 1, cs, variant=10)
    c1 = wl.random_unit_sum_coeffs(np.random.default_rng(5), 3, wl.BOX, 1)
    d = st.Stencil((300, 200, 9), "box", 1, c1, variant=10, tile_y=16, zchunk=32).describe()
    assert d["variant"] == "ym3d" and d["tile_y"] == 16 and d["zchunk"] == 32
