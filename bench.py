#!/usr/bin/env python3
"""Throughput of the stencil hot path on one MI355X.

One "step" of this benchmark is one pass of the headline workload: 20
leapfrog time steps of the 3D acoustic wave model (radius-4, 25-point
eighth-order Laplacian star, f32, 512^3 cells, zero frame, kappa per cell)
over inputs already resident in HBM.  `value` is GCells/s = cells * time
steps / second.  The JSON line also carries the live roofline of the
dominant kernel (the fused leapfrog step), the FP64 oracle timed on a
bounded sample on the host, and the other workloads (2D Jacobi, the 7-point
star and the 27- and 125-point boxes in fp16/f32/f64, the 2D box, 64 uneven
grids, variable coefficients, the wave gradient) as `per_config`.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
WAVE_BYTES_PER_CELL = 16     # read u_t, u_{t-1}, kappa; write u_{t+1}
# FP32 vector peak without packed FP32 (the kernels are built without it):
# 256 CUs x 64 FMA lanes x 2 flop x 2.4 GHz.  The published 157.3 TFLOP/s
# counts packed (two-wide) FP32.
VALU_PEAK_TFLOPS = 78.6
VALU_F64_PEAK_TFLOPS = 78.6   # FP64 vector, published


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--only", default="", help="comma list of extra workloads to run")
    ap.add_argument("--pmc-target", action="store_true",
                    help="run only the profiler target: a 512 MiB device copy (counter calibration) "
                         "then one 2-step pass of the headline workload")
    ap.add_argument("--shapes", action="store_true",
                    help="also sweep the 7- and 27-point 3D sweeps over cubes and slabs (f16/f32/f64)")
    ap.add_argument("--stream-ceiling", action="store_true",
                    help="also measure plain streaming kernels (copy, read-3/write-1) as the "
                         "practical bandwidth ceiling")
    return ap.parse_args()


def pmc_target(dev, st, wl, torch):
    """Profiler target: a device copy of known size (its FETCH_SIZE/WRITE_SIZE
    calibrate the counters) followed by two leapfrog launches at 512^3."""
    a = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    case = wl.wave3d(n=512, steps=2)
    u0 = torch.from_numpy(case.u0).to(dev)
    prev = torch.from_numpy(case.u_prev).to(dev)
    kap = torch.from_numpy(case.kappa).to(dev)
    out = torch.empty_like(u0)
    model = st.WaveModel(case.n, radius=4, boundary="zero")
    model.forward(u0, prev, kap, 2, out=out, prev_inout=True)
    torch.cuda.synchronize()
    log("pmc target done: copy 512 MiB, 2 wave launches")


def stream_ceiling(dev, torch):
    """Practical HBM bandwidth of plain streaming kernels on this device."""
    n = 256 * 1024 * 1024
    a, b, c, d = (torch.rand(n, device=dev) for _ in range(4))
    res = {}
    ms = timed(lambda: b.copy_(a), 5, 2, torch.cuda.synchronize)
    res["copy_gbs"] = 2 * 4 * n / (ms * 1e-3) / 1e9
    ms = timed(lambda: torch.addcmul(a, b, c, out=d), 5, 2, torch.cuda.synchronize)
    res["read3_write1_gbs"] = 4 * 4 * n / (ms * 1e-3) / 1e9
    ms = timed(lambda: torch.add(a, b, out=c), 5, 2, torch.cuda.synchronize)
    res["read2_write1_gbs"] = 3 * 4 * n / (ms * 1e-3) / 1e9
    return res


WAVE_SOURCES = ["paper_2609_06694_amd/csrc/kernels_wave_ring.hip", "paper_2609_06694_amd/csrc/zmarch.h",
                "paper_2609_06694_amd/csrc/common.h"]
TRAFFIC_PROFILE = "profiles/wave3d_fwd_r4_512cube_pmc_traffic.md"


def ring_kernel_name(disp):
    """Instantiation of the LDS-ring leapfrog kernel a dispatch selects: two
    rows per thread, tile_y / 2 waves per workgroup."""
    if disp.get("variant") != "wave3d_lds":
        return disp.get("variant")
    return f"wave3d_ring_kernel<R=4,zero,RY=2,NW={disp['tile_y'] // 2},D=2,iso>"


def measured_traffic(kernel):
    """HBM bytes per launch of the leapfrog kernel from the committed PMC
    summary, or None when the kernel sources or the instantiation the
    dispatch selects changed since it was taken."""
    import hashlib
    try:
        src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in WAVE_SOURCES)
        h = hashlib.sha256(src).hexdigest()[:16]
        for line in open(os.path.join(ROOT, TRAFFIC_PROFILE)):
            if line.startswith("traffic_json:"):
                rec = json.loads(line.split(":", 1)[1])
                if rec.get("source_hash") == h and rec.get("kernel") == kernel:
                    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def timed(fn, reps, warmup, sync):
    """Median wall time (ms) of fn() over reps, bracketed by device syncs."""
    import torch
    for _ in range(warmup):
        fn()
    sync()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def timed_pair(fa, fb, reps, warmup, sync):
    """Median times (ms) of two variants measured in interleaved passes (a,
    b, a, b, ...), so drift of clocks or temperature affects both alike."""
    import torch
    for _ in range(warmup):
        fa()
        fb()
    sync()
    ta, tb = [], []
    for _ in range(reps):
        for fn, ts in ((fa, ta), (fb, tb)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
    return float(np.median(ta)), float(np.median(tb))


def gcells(cells, steps, ms):
    return cells * steps / (ms * 1e-3) / 1e9


def bench_wave(args, dev, st, wl, torch):
    case = wl.wave3d(n=512, steps=20)
    bufs = [torch.from_numpy(case.u0).to(dev), torch.empty(case.u0.shape, dtype=torch.float32, device=dev)]
    prev = torch.from_numpy(case.u_prev).to(dev)
    kap = torch.from_numpy(case.kappa).to(dev)
    model = st.WaveModel(case.n, radius=4, boundary="zero")
    state = {"i": 0}

    def one_pass():
        # Continue the simulation: u_T of this pass is u_0 of the next, and
        # u_prev is updated in place, so consecutive passes copy nothing.
        i = state["i"]
        model.forward(bufs[i], prev, kap, case.steps, out=bufs[1 - i], prev_inout=True)
        state["i"] = 1 - i

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        one_pass()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    ms_per_pass = e0.elapsed_time(e1) / args.steps
    launch_ms = ms_per_pass / case.steps
    finite = bool(torch.isfinite(bufs[state["i"]]).all().item())
    log(f"wave3d 512^3 x20: {ms_per_pass:.3f} ms/pass (events), wall {wall:.3f} ms/pass, "
        f"{launch_ms * 1e3:.1f} us/launch, finite={finite}")
    return case, ms_per_pass, launch_ms, model.describe(), finite


def bench_jacobi(dev, st, wl, torch):
    case = wl.jacobi2d()
    s = st.Stencil(case.n[:2], "star", 1, case.coeffs)
    u = torch.from_numpy(case.u0).to(dev)
    out = torch.empty_like(u)
    ms = timed(lambda: s.apply(u, case.steps, out=out), 20, 3, torch.cuda.synchronize)
    g = gcells(case.cells, case.steps, ms)
    # The 10-step sweep is a few microseconds of GPU work, so a single call
    # is bound by host launch latency, and so is a one-call graph replayed
    # again and again (each replay is one host submission).  A loop of such
    # sweeps is captured whole: 20 full calls in one HIP graph, one replay.
    reps = 20
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(reps):
            s.apply(u, case.steps, out=out)
    gms = timed(graph.replay, 5, 2, torch.cuda.synchronize) / reps
    one = torch.cuda.CUDAGraph()
    with torch.cuda.graph(one):
        s.apply(u, case.steps, out=out)
    oms = timed(lambda: [one.replay() for _ in range(reps)], 5, 2, torch.cuda.synchronize) / reps
    return {"workload": "jacobi2d_star1_512^2_10steps_f32", "ms": gms, "gcells_s": gcells(case.cells, case.steps, gms),
            "timing": "one HIP graph holding 20 full calls (10 steps each), replayed",
            "ms_one_call_graph_replays": oms, "ms_single_call": ms, "gcells_s_single_call": g,
            "hbm_frac": None, "note": "1 MiB grid is cache resident; not an HBM figure",
            "dispatch": s.describe()}


ESIZE = {"f16": 2, "f32": 4, "f64": 8}


def bench_linear(dev, st, wl, torch, case, reps=3):
    dt = wl.DTYPE_TAGS[case.dtype]
    shape = wl.SHAPE_NAMES[case.shape]
    s = st.Stencil(case.n[:case.ndim], shape, case.radius, case.coeffs, dtype=dt)
    u = torch.from_numpy(case.u0).to(dev)
    out = torch.empty_like(u)
    ms = timed(lambda: s.apply(u, case.steps, out=out), reps, 1, torch.cuda.synchronize)
    g = gcells(case.cells, case.steps, ms)
    bpc = 2 * ESIZE[dt]
    taps = (2 * case.radius + 1) ** case.ndim if case.shape == wl.BOX else 1 + 2 * case.ndim * case.radius
    fpc = 2 * taps   # one multiply-add per tap (f32 arithmetic; f64 for f64 storage)
    return {"workload": f"{case.name}_{'x'.join(str(v) for v in case.n[:case.ndim])}_{case.steps}steps",
            "ms": ms, "gcells_s": g, "eff_gbs": g * bpc, "hbm_frac": g * bpc / HBM_PEAK_GBS,
            "bytes_per_cell_update": bpc, "flop_per_cell_update": fpc, "valu_tflops": g * fpc / 1e3,
            "valu_frac": g * fpc / 1e3 / (VALU_F64_PEAK_TFLOPS if dt == "f64" else VALU_PEAK_TFLOPS),
            "dispatch": s.describe()}


def bench_varcoef(dev, st, torch, shape, r, n=512, steps=10, ndim=3):
    """Variable-coefficient sweep (f32, periodic) on n^ndim; fields and data
    are seeded device-side uniform draws, fields normalised per cell."""
    ntap = st.varcoef_taps(ndim, shape, r)
    g = torch.Generator(device=dev)
    g.manual_seed(99 + ntap)
    grid = (n,) * ndim
    f = torch.rand((ntap,) + grid, generator=g, device=dev)
    f /= f.sum(dim=0, keepdim=True)
    u = torch.rand(grid, generator=g, device=dev)
    out = torch.empty_like(u)
    s = st.VarCoefStencil(grid, shape, r)
    ms = timed(lambda: s.apply(u, f, steps, out=out), 3, 1, torch.cuda.synchronize)
    gc = gcells(n ** ndim, steps, ms)
    bpc = (ntap + 2) * 4
    return {"workload": f"varcoef_{shape}{r}_f32_{n}^{ndim}_{steps}steps", "ms": ms, "gcells_s": gc,
            "bytes_per_cell_update": bpc, "eff_gbs": gc * bpc, "hbm_frac": gc * bpc / HBM_PEAK_GBS,
            "dispatch": s.describe()}


# Cubes of the paper's kernel matrix and slab stand-ins (its slab sizes are
# not given): thin in z, thin in y, and a long narrow column.
SHAPES = [("cube128", (128, 128, 128)), ("cube256", (256, 256, 256)), ("cube512", (512, 512, 512)),
          ("cube1024", (1024, 1024, 1024)), ("slab_z", (4096, 4096, 8)), ("slab_y", (4096, 64, 512)),
          ("column_z", (64, 64, 32768))]


def bench_shapes(dev, st, wl, torch):
    """7- and 27-point 3D sweeps (10 steps) over cubes and slabs in each
    storage type, with the default dispatch; inputs are seeded device-side
    uniform draws (timing only: parity is covered by the tests)."""
    out = {}
    rng = np.random.default_rng(77)
    torch.manual_seed(77)
    for sname, r in (("star", 1), ("box", 1)):
        c = wl.random_unit_sum_coeffs(rng, 3, wl.STAR if sname == "star" else wl.BOX, r)
        for dt in ("f16", "f32", "f64"):
            tdt = {"f16": torch.float16, "f32": torch.float32, "f64": torch.float64}[dt]
            for tag, n in SHAPES:
                s = st.Stencil(n, sname, r, c, dtype=dt)
                u = torch.rand((n[2], n[1], n[0]), device=dev, dtype=tdt)
                o = torch.empty_like(u)
                ms = timed(lambda: s.apply(u, 10, out=o), 3, 1, torch.cuda.synchronize)
                cells = n[0] * n[1] * n[2]
                g = gcells(cells, 10, ms)
                out[f"{sname}1_{dt}_{tag}"] = {"grid": list(n), "ms": round(ms, 4), "gcells_s": round(g, 1),
                                               "hbm_frac": round(g * 2 * ESIZE[dt] / HBM_PEAK_GBS, 3),
                                               "dispatch": s.describe()}
                del u, o
                torch.cuda.empty_cache()
    return out


def bench_batch(dev, st, wl, torch):
    cases = wl.batch2d()
    plans = [st.Stencil(c.n[:2], wl.SHAPE_NAMES[c.shape], c.radius, c.coeffs) for c in cases]
    ins = [torch.from_numpy(c.u0).to(dev) for c in cases]
    outs = [torch.empty_like(u) for u in ins]
    cells = sum(c.cells for c in cases)

    def run():
        for p, u, o, c in zip(plans, ins, outs, cases):
            p.apply(u, c.steps, out=o)

    bs = st.BatchedStencil([dict(n=c.n[:2], shape=wl.SHAPE_NAMES[c.shape], radius=c.radius, coeffs=c.coeffs)
                            for c in cases])
    # Seven interleaved passes of the two variants, medians.
    ms, bms = timed_pair(run, lambda: bs.apply(ins, 32, outs=outs), 7, 2, torch.cuda.synchronize)
    g = gcells(cells, 32, ms)
    bg = gcells(cells, 32, bms)
    return {"workload": "batch64_2d_mixed_32steps_f32", "cells": cells, "ms": bms, "gcells_s": bg,
            "launches": "one per time block for all 64 grids", "eff_gbs": bg * 8,
            "ms_separate_launches": ms, "gcells_s_separate": g}


def bench_grad(dev, st, wl, torch):
    case = wl.wavegrad3d()
    n = case.n
    kap = torch.from_numpy(case.kappa).to(dev)
    kt = torch.from_numpy(case.kappa_true).to(dev)
    zeros = torch.zeros(n[::-1], dtype=torch.float32, device=dev)
    wav = torch.from_numpy(case.wavelet).to(dev)
    model = st.WaveModel(n, radius=4, boundary="zero", ckpt_every=case.ckpt_every)
    # Synthetic observed traces: the forward model at the perturbed kappa.
    _, _, target = model.forward(zeros, zeros, kt, case.steps, src=case.src, wavelet=wav,
                                 rec_z=case.rec_z, record=True)
    target = target.contiguous()
    res = {}

    def grad():
        res["g"] = model.gradient(zeros, zeros, kap, case.steps, case.src, wav, case.rec_z, target)

    # Forward and forward + backward in seven interleaved passes, medians.
    fwd_ms, g_ms = timed_pair(lambda: model.forward(zeros, zeros, kap, case.steps, src=case.src, wavelet=wav,
                                                    rec_z=case.rec_z, record=True), grad, 7, 1,
                              torch.cuda.synchronize)
    dk, loss = res["g"]
    return {"workload": "wavegrad3d_star4_256^3_200steps_ckpt20", "fwd_ms": fwd_ms, "fwd_bwd_ms": g_ms,
            "ratio_fwd_bwd_over_fwd": g_ms / fwd_ms,
            "fwd_gcells_s": gcells(case.cells, case.steps, fwd_ms),
            "loss": float(loss.item()), "grad_finite": bool(torch.isfinite(dk).all().item())}


def cpu_baseline(wl):
    """The FP64 oracle (unchanged, OpenMP over all host cores) on a bounded
    sample of the headline workload: a 288^3 grid, 20 leapfrog steps."""
    import oracle
    oracle.build(force=False)
    n = 288
    case = wl.wave3d(n=n, steps=20)
    t0 = time.perf_counter()
    oracle.wave_forward(case.u_prev, case.u0, case.kappa, case.steps, r=4, boundary=wl.ZERO)
    dt = time.perf_counter() - t0
    return {"value": gcells(n ** 3, case.steps, dt * 1e3), "unit": "GCells/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"wave leapfrog r=4, {n}^3 cells x 20 steps, FP64, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the stencil library runs on one GPU; run with --gpus 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    from paper_2609_06694_amd import stencil as st, workloads as wl
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.pmc_target:
        pmc_target(dev, st, wl, torch)
        return

    case, ms_pass, launch_ms, disp, finite = bench_wave(args, dev, st, wl, torch)
    cells = case.cells
    value = gcells(cells, case.steps, ms_pass)
    achieved = WAVE_BYTES_PER_CELL * cells / (launch_ms * 1e-3) / 1e9
    tbytes = measured_traffic(ring_kernel_name(disp))
    traffic = None if tbytes is None else round(tbytes / (launch_ms * 1e-3) / 1e9, 1)
    line = {
        "metric": "GCells/s", "value": round(value, 2), "unit": "GCells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_pass, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "wave3d_star4_512^3_20steps_zero_frame", "grid": [512, 512, 512],
                   "time_steps": case.steps, "radius": 4, "dispatch": disp},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_bytes_per_launch": tbytes, "traffic_source": TRAFFIC_PROFILE,
                     "kernel": ring_kernel_name(disp), "bytes_per_cell": WAVE_BYTES_PER_CELL,
                     "cells_per_launch": cells, "launch_ms": round(launch_ms, 5)},
    }
    extras = {}
    if not args.quick:
        only = set(filter(None, args.only.split(",")))
        todo = [
            ("jacobi2d", lambda: bench_jacobi(dev, st, wl, torch)),
            ("box3d_f16", lambda: bench_linear(dev, st, wl, torch, wl.box3d(dtype=wl.F16))),
            ("box3d_f32", lambda: bench_linear(dev, st, wl, torch, wl.box3d(dtype=wl.F32))),
            ("star3d_f16", lambda: bench_linear(dev, st, wl, torch, wl.star3d(dtype=wl.F16))),
            ("star3d_f32", lambda: bench_linear(dev, st, wl, torch, wl.star3d(dtype=wl.F32))),
            ("star3d_f64", lambda: bench_linear(dev, st, wl, torch, wl.star3d(dtype=wl.F64))),
            ("varcoef_star1", lambda: bench_varcoef(dev, st, torch, "star", 1)),
            ("varcoef_box1", lambda: bench_varcoef(dev, st, torch, "box", 1)),
            ("varcoef2d_star1", lambda: bench_varcoef(dev, st, torch, "star", 1, n=4096, steps=20, ndim=2)),
            ("box2d_f64", lambda: bench_linear(dev, st, wl, torch, wl.box2d(dtype=wl.F64))),
            ("box3d_r2_f16", lambda: bench_linear(dev, st, wl, torch, wl.box3d_r2(dtype=wl.F16))),
            ("box3d_r2_f32", lambda: bench_linear(dev, st, wl, torch, wl.box3d_r2(dtype=wl.F32))),
            ("box2d_f16", lambda: bench_linear(dev, st, wl, torch, wl.box2d(dtype=wl.F16))),
            ("box2d_f32", lambda: bench_linear(dev, st, wl, torch, wl.box2d(dtype=wl.F32))),
            ("batch64", lambda: bench_batch(dev, st, wl, torch)),
            ("wavegrad", lambda: bench_grad(dev, st, wl, torch)),
        ]
        for name, fn in todo:
            if only and name not in only:
                continue
            t0 = time.perf_counter()
            extras[name] = fn()
            log(f"{name}: {json.dumps(extras[name])} ({time.perf_counter() - t0:.1f} s)")
            torch.cuda.empty_cache()
        line["per_config"] = extras
    if args.shapes:
        t0 = time.perf_counter()
        line["shapes"] = bench_shapes(dev, st, wl, torch)
        log(f"shapes: {json.dumps(line['shapes'])} ({time.perf_counter() - t0:.1f} s)")
    if args.stream_ceiling:
        line["stream_ceiling"] = stream_ceiling(dev, torch)
        log(f"stream ceiling: {line['stream_ceiling']}")
    if not args.no_cpu:
        t0 = time.perf_counter()
        line["cpu_baseline"] = cpu_baseline(wl)
        log(f"cpu baseline: {line['cpu_baseline']} ({time.perf_counter() - t0:.1f} s)")
    if not finite:
        line["error"] = "non-finite wave field"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
