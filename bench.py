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
# FP32 vector peak, published: 157.3 TFLOP/s (256 CUs x 128 FMA lanes x 2 flop
# x 2.4 GHz).  The kernels are built without packed FP32, yet plain f32
# multiply-adds whose operands are all vector registers measured 22-23 lanes
# per SIMD cycle (a multiply-add with a scalar-register operand: 15.5; an
# add and a multiply-add from different waves together: 28), so the
# published figure, not the 16-lane rate, is the ceiling.
VALU_PEAK_TFLOPS = 157.3
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
    ap.add_argument("--pmc-target", nargs="?", const="wave", default="",
                    help="run only a profiler target: a 512 MiB device copy (counter calibration), then "
                         "a few launches of one workload: " + ", ".join(PMC_TARGETS))
    ap.add_argument("--summarize-counters", nargs="*", default=None,
                    help="instead of benchmarking: per-kernel means of rocprofv3 counter_collection.csv files")
    ap.add_argument("--shapes", action="store_true",
                    help="also sweep the 7- and 27-point 3D sweeps over cubes and slabs (f16/f32/f64)")
    ap.add_argument("--summarize-trace", default="",
                    help="instead of benchmarking: summarise a rocprofv3 kernel_trace.csv (durations of "
                         "the launches of --kernel after the first --skip of them)")
    ap.add_argument("--kernel", default="wave3d_ring_kernel", help="kernel name substring for --summarize-trace")
    ap.add_argument("--skip", type=int, default=0, help="launches to skip (warm-up) for --summarize-trace")
    ap.add_argument("--summarize-clock", default="",
                    help="instead of benchmarking: clock per dispatch (GRBM_COUNT / traced duration) from a "
                         "rocprofv3 --kernel-trace --pmc GRBM_COUNT output directory")
    ap.add_argument("--no-stream-ceiling", action="store_true",
                    help="skip the plain streaming kernels (copy, read-2/write-1, read-3/write-1) timed "
                         "after the headline as this device's practical bandwidth ceiling")
    return ap.parse_args()


PMC_TARGETS = ("wave", "wave_f64", "box3d_f16", "box3d_f16_zm", "box3d_f32", "box3d_f16_mfma", "star3d_f16", "box2d_f16",
               "box2d_f32", "box3d_r2_f16", "box3d_r2_f32", "batch64", "wavegrad", "clock")


def pmc_target(name, dev, st, wl, torch):
    """Profiler target: a device copy of known size (its FETCH_SIZE and
    WRITE_SIZE calibrate the counters) followed by a few launches of one
    workload at its full size."""
    a = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    if name == "wave":
        case = wl.wave3d(n=512, steps=2)
        u0 = torch.from_numpy(case.u0).to(dev)
        prev = torch.from_numpy(case.u_prev).to(dev)
        kap = torch.from_numpy(case.kappa).to(dev)
        out = torch.empty_like(u0)
        model = st.WaveModel(case.n, radius=4, boundary="zero")
        model.forward(u0, prev, kap, 2, out=out, prev_inout=True)
    elif name == "wave_f64":
        case = wl.wave3d(n=512, steps=2)
        u0 = torch.from_numpy(case.u0).to(dev).double()
        prev = torch.from_numpy(case.u_prev).to(dev).double()
        kap = torch.from_numpy(case.kappa).to(dev).double()
        model = st.WaveModel(case.n, radius=4, boundary="zero", dtype="f64")
        model.forward(u0, prev, kap, 2, out=torch.empty_like(u0), prev_inout=True)
    elif name in ("box3d_f16", "box3d_f16_zm", "box3d_f32", "box3d_f16_mfma", "star3d_f16", "box2d_f16",
                  "box2d_f32", "box3d_r2_f16", "box3d_r2_f32"):
        case = {"box3d_f16": lambda: wl.box3d(dtype=wl.F16), "box3d_f32": lambda: wl.box3d(dtype=wl.F32),
                "box3d_f16_zm": lambda: wl.box3d(dtype=wl.F16),
                "box3d_f16_mfma": lambda: wl.box3d(dtype=wl.F16), "star3d_f16": lambda: wl.star3d(dtype=wl.F16),
                "box2d_f16": lambda: wl.box2d(dtype=wl.F16), "box2d_f32": lambda: wl.box2d(dtype=wl.F32),
                "box3d_r2_f16": lambda: wl.box3d_r2(dtype=wl.F16),
                "box3d_r2_f32": lambda: wl.box3d_r2(dtype=wl.F32)}[name]()
        opts = {"variant": 6} if name.endswith("mfma") else \
            ({"variant": 2, "tile_y": 16, "zchunk": 64} if name.endswith("_zm") else {})
        s = st.Stencil(case.n[:case.ndim], wl.SHAPE_NAMES[case.shape], case.radius, case.coeffs,
                       dtype=wl.DTYPE_TAGS[case.dtype], **opts)
        u = torch.from_numpy(case.u0).to(dev)
        k = fused_depth(s.describe(), case.ndim)
        s.apply(u, 2 * k, out=torch.empty_like(u))   # two launches
    elif name == "batch64":
        cases = wl.batch2d()
        bs = st.BatchedStencil([dict(n=c.n[:2], shape=wl.SHAPE_NAMES[c.shape], radius=c.radius, coeffs=c.coeffs)
                                for c in cases])
        ins = [torch.from_numpy(c.u0).to(dev) for c in cases]
        bs.apply(ins, 2 * max(1, bs.describe()["tsteps"]))
    elif name == "clock":
        # Twelve launches each of the headline leapfrog, the fp16 27-point
        # box (VALU-bound) and torch's read-3/write-1 stream, for the clock
        # each keeps (GRBM_COUNT over the kernel trace's durations).
        case = wl.wave3d(n=512, steps=2)
        u0 = torch.from_numpy(case.u0).to(dev)
        prev = torch.from_numpy(case.u_prev).to(dev)
        kap = torch.from_numpy(case.kappa).to(dev)
        st.WaveModel(case.n, radius=4, boundary="zero").forward(u0, prev, kap, 12, out=torch.empty_like(u0),
                                                                  prev_inout=True)
        torch.cuda.synchronize()
        del u0, prev, kap
        c = wl.box3d(dtype=wl.F16)
        s = st.Stencil(c.n, wl.SHAPE_NAMES[c.shape], c.radius, c.coeffs, dtype=wl.DTYPE_TAGS[c.dtype])
        u = torch.from_numpy(c.u0).to(dev)
        s.apply(u, 12 * fused_depth(s.describe(), 3), out=torch.empty_like(u))
        torch.cuda.synchronize()
        del u
        n = 256 * 1024 * 1024
        a, b, cc, d = (torch.rand(n, device=dev) for _ in range(4))
        for _ in range(12):
            torch.addcmul(a, b, cc, out=d)
    elif name == "wavegrad":
        case = wl.wavegrad3d(steps=40)
        n = case.n
        z = torch.zeros(n[::-1], dtype=torch.float32, device=dev)
        wav = torch.from_numpy(case.wavelet).to(dev)
        model = st.WaveModel(n, ckpt_every=20)
        _, _, target = model.forward(z, z, torch.from_numpy(case.kappa_true).to(dev), case.steps, src=case.src,
                                     wavelet=wav, rec_z=case.rec_z, record=True)
        model.gradient(z, z, torch.from_numpy(case.kappa).to(dev), case.steps, case.src, wav, case.rec_z,
                       target.contiguous())
    else:
        raise SystemExit(f"unknown profiler target {name!r}; one of {PMC_TARGETS}")
    torch.cuda.synchronize()
    log(f"pmc target {name} done")


def summarize_clock(directory):
    """Clock kept by each kernel family of a `--pmc GRBM_COUNT --kernel-trace`
    run: GRBM_COUNT (GPU clock cycles, summed over the 8 XCDs) over each
    dispatch's traced duration.  Prints one JSON line."""
    import csv
    import glob
    kt = glob.glob(os.path.join(directory, "**", "*kernel_trace.csv"), recursive=True)[0]
    cc = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)[0]
    dur, name = {}, {}
    with open(kt, newline="") as f:
        for r in csv.DictReader(f):
            dur[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            name[r["Dispatch_Id"]] = r["Kernel_Name"]
    cyc = {}
    with open(cc, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == "GRBM_COUNT":
                cyc[r["Dispatch_Id"]] = cyc.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"] or 0)
    fam = {}
    for d in sorted(cyc, key=int):
        if d not in dur or dur[d] < 50:
            continue
        k = name[d].split("(")[0].replace("void ", "")[:80]
        fam.setdefault(k, []).append((dur[d], cyc[d] / 8 / (dur[d] * 1e3)))
    out = {k: {"launches": len(v), "us": [round(t, 1) for t, _ in v], "ghz": [round(g, 3) for _, g in v]}
           for k, v in fam.items()}
    print(json.dumps(out), flush=True)
    return out


def summarize_counters(paths):
    """Per-kernel means of the counters in rocprofv3 counter_collection.csv
    files (one row per dispatch and counter).  Prints one JSON line."""
    import csv
    acc = {}
    for path in paths:
        with open(path, newline="") as f:
            for rec in csv.DictReader(f):
                k = rec.get("Kernel_Name", "")
                c = rec.get("Counter_Name", "")
                v = float(rec.get("Counter_Value") or 0)
                d = rec.get("Dispatch_Id", "")
                acc.setdefault(k, {}).setdefault(c, {}).setdefault(d, 0.0)
                acc[k][c][d] += v   # counters reported per dimension instance are summed per dispatch
    out = {}
    for k, cs in acc.items():
        out[k] = {c: {"dispatches": len(ds), "mean": float(np.mean(list(ds.values()))),
                      "values": [round(v, 1) for v in ds.values()][:8]} for c, ds in cs.items()}
    print(json.dumps(out), flush=True)
    return out


def stream_ceiling(dev, torch):
    """Practical HBM bandwidth of plain streaming kernels on this device
    (torch elementwise kernels on 1 GiB f32 arrays, medians of 5)."""
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
    rows per thread, tile_y / 2 waves per workgroup, tile_x = 2: both
    planes of a march step staged per barrier."""
    if disp.get("variant") != "wave3d_lds":
        return disp.get("variant")
    pb = ",PB=2" if disp.get("tile_x") == 2 else ""
    return f"wave3d_ring_kernel<R=4,zero,RY=2,NW={disp['tile_y'] // 2},D=2,iso{pb}>"


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


SPONGE = (20, 0.5)   # absorbing layer of the sponge workload: width (cells), strength


def bench_wave_sponge(dev, st, wl, torch):
    """The headline wave workload with the absorbing layer fused into the
    leapfrog kernel, against the plain leapfrog, interleaved passes."""
    case = wl.wave3d(n=512, steps=20)
    u0 = torch.from_numpy(case.u0).to(dev)
    prev = torch.from_numpy(case.u_prev).to(dev)
    kap = torch.from_numpy(case.kappa).to(dev)
    out = torch.empty_like(u0)
    plain = st.WaveModel(case.n, radius=4, boundary="zero")
    damped = st.WaveModel(case.n, radius=4, boundary="zero", sponge=SPONGE)
    pp, pd = prev.clone(), prev.clone()
    ms_p, ms_d = timed_pair(lambda: plain.forward(u0, pp, kap, case.steps, out=out, prev_inout=True),
                            lambda: damped.forward(u0, pd, kap, case.steps, out=out, prev_inout=True),
                            REPS, 1, torch.cuda.synchronize)
    g = gcells(case.cells, case.steps, ms_d)
    return {"workload": f"wave3d_star4_512^3_20steps_sponge_w{SPONGE[0]}_s{SPONGE[1]}", "ms": ms_d,
            "gcells_s": g, "bytes_per_cell_update": WAVE_BYTES_PER_CELL,
            "hbm_frac": g * WAVE_BYTES_PER_CELL / HBM_PEAK_GBS, "ms_plain": ms_p,
            "overhead_vs_plain": ms_d / ms_p, "dispatch": damped.describe(),
            "timing": f"median of {REPS} passes interleaved with the plain leapfrog"}


WAVE_F64_BYTES_PER_CELL = 32   # the four operands of WAVE_BYTES_PER_CELL in binary64


def bench_wave_f64(dev, st, wl, torch):
    """The headline wave workload stored and computed in binary64 (fields
    converted from the f32 case), median of passes that continue the
    simulation from the previous pass's state."""
    case = wl.wave3d(n=512, steps=20)
    bufs = [torch.from_numpy(case.u0).to(dev).double(), torch.empty(case.u0.shape, dtype=torch.float64, device=dev)]
    prev = torch.from_numpy(case.u_prev).to(dev).double()
    kap = torch.from_numpy(case.kappa).to(dev).double()
    model = st.WaveModel(case.n, radius=4, boundary="zero", dtype="f64")
    state = {"i": 0}

    def one_pass():
        i = state["i"]
        model.forward(bufs[i], prev, kap, case.steps, out=bufs[1 - i], prev_inout=True)
        state["i"] = 1 - i

    ms = timed(one_pass, REPS, 2, torch.cuda.synchronize)
    g = gcells(case.cells, case.steps, ms)
    finite = bool(torch.isfinite(bufs[state["i"]]).all().item())
    return {"workload": "wave3d_star4_512^3_20steps_zero_frame_f64", "ms": ms, "gcells_s": g,
            "bytes_per_cell_update": WAVE_F64_BYTES_PER_CELL, "hbm_frac": g * WAVE_F64_BYTES_PER_CELL / HBM_PEAK_GBS,
            "flop_per_cell_update": 53, "valu_f64_frac": g * 53 / 1e3 / VALU_F64_PEAK_TFLOPS,
            "finite": finite, "dispatch": model.describe(),
            "timing": f"median of {REPS} passes (each continues the previous one's state)"}


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


def fused_depth(desc, ndim):
    """Time steps one launch of the dispatched kernel advances: the fused
    depth of the 2D families, two for the 3D two-step kernel, else one."""
    k = max(1, int(desc.get("tsteps") or 1))
    if ndim == 3:
        return 2 if k == 2 and desc.get("variant") == "zm3d" else 1
    return k


def linear_record(case, wl, desc, ms):
    """GCells/s and roofline fractions of a linear sweep.  `hbm_frac` counts
    the algorithmic HBM bytes of the launches as run: one read and one write
    of the grid per launch, i.e. 2b/k bytes per cell-update with k fused
    steps.  `equiv_frac_one_step` charges 2b per cell-update (what k
    single-step launches would move) and can exceed the HBM roof."""
    dt = wl.DTYPE_TAGS[case.dtype]
    g = gcells(case.cells, case.steps, ms)
    k = fused_depth(desc, case.ndim)
    bpc = 2 * ESIZE[dt] / k
    taps = (2 * case.radius + 1) ** case.ndim if case.shape == wl.BOX else 1 + 2 * case.ndim * case.radius
    fpc = 2 * taps   # one multiply-add per tap (f32 arithmetic; f64 for f64 storage)
    return {"workload": f"{case.name}_{'x'.join(str(v) for v in case.n[:case.ndim])}_{case.steps}steps",
            "ms": ms, "gcells_s": g, "fused_steps_per_launch": k, "bytes_per_cell_update": bpc,
            "eff_gbs": g * bpc, "hbm_frac": g * bpc / HBM_PEAK_GBS,
            "equiv_frac_one_step": g * 2 * ESIZE[dt] / HBM_PEAK_GBS,
            "flop_per_cell_update": fpc, "valu_tflops": g * fpc / 1e3,
            "valu_frac": g * fpc / 1e3 / (VALU_F64_PEAK_TFLOPS if dt == "f64" else VALU_PEAK_TFLOPS),
            "timing": f"median of {REPS} passes", "dispatch": desc}


REPS = 7   # timed passes per workload (medians); twins are interleaved


def bench_linear(dev, st, wl, torch, case):
    dt = wl.DTYPE_TAGS[case.dtype]
    s = st.Stencil(case.n[:case.ndim], wl.SHAPE_NAMES[case.shape], case.radius, case.coeffs, dtype=dt)
    u = torch.from_numpy(case.u0).to(dev)
    out = torch.empty_like(u)
    ms = timed(lambda: s.apply(u, case.steps, out=out), REPS, 1, torch.cuda.synchronize)
    return linear_record(case, wl, s.describe(), ms)


def bench_linear_twins(dev, st, wl, torch, case_a, case_b):
    """Two storage twins of one workload, timed in interleaved passes."""
    runs, plans = [], []
    for case in (case_a, case_b):
        dt = wl.DTYPE_TAGS[case.dtype]
        s = st.Stencil(case.n[:case.ndim], wl.SHAPE_NAMES[case.shape], case.radius, case.coeffs, dtype=dt)
        u = torch.from_numpy(case.u0).to(dev)
        out = torch.empty_like(u)
        runs.append(lambda s=s, u=u, out=out, c=case: s.apply(u, c.steps, out=out))
        plans.append(s)
    ma, mb = timed_pair(runs[0], runs[1], REPS, 1, torch.cuda.synchronize)
    ra = linear_record(case_a, wl, plans[0].describe(), ma)
    rb = linear_record(case_b, wl, plans[1].describe(), mb)
    ra["timing"] = rb["timing"] = f"median of {REPS} interleaved passes with its storage twin"
    return ra, rb


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
    ms = timed(lambda: s.apply(u, f, steps, out=out), REPS, 1, torch.cuda.synchronize)
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
    """7-, 27- and 125-point 3D sweeps (10 steps) over cubes and slabs in
    each storage type, with the default dispatch; inputs are seeded
    device-side uniform draws (timing only: parity is covered by the tests)."""
    out = {}
    rng = np.random.default_rng(77)
    torch.manual_seed(77)
    for sname, r in (("star", 1), ("box", 1), ("box", 2)):
        c = wl.random_unit_sum_coeffs(rng, 3, wl.STAR if sname == "star" else wl.BOX, r)
        for dt in ("f16", "f32", "f64"):
            tdt = {"f16": torch.float16, "f32": torch.float32, "f64": torch.float64}[dt]
            for tag, n in SHAPES:
                s = st.Stencil(n, sname, r, c, dtype=dt)
                u = torch.rand((n[2], n[1], n[0]), device=dev, dtype=tdt)
                o = torch.empty_like(u)
                ms = timed(lambda: s.apply(u, 10, out=o), REPS, 1, torch.cuda.synchronize)
                cells = n[0] * n[1] * n[2]
                g = gcells(cells, 10, ms)
                desc = s.describe()
                k = fused_depth(desc, 3)
                out[f"{sname}{r}_{dt}_{tag}"] = {"grid": list(n), "ms": round(ms, 4), "gcells_s": round(g, 1),
                                               "fused_steps_per_launch": k,
                                               "hbm_frac": round(g * 2 * ESIZE[dt] / k / HBM_PEAK_GBS, 3),
                                               "equiv_frac_one_step": round(g * 2 * ESIZE[dt] / HBM_PEAK_GBS, 3),
                                               "dispatch": desc}
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
    t0 = time.perf_counter()
    tune = bs.autotune(device=dev)
    tune_s = time.perf_counter() - t0
    desc = bs.describe()
    own = desc["tsteps"] == -1   # the tuner chose each member's own map depth
    # Seven interleaved passes of the two variants, medians.
    ms, bms = timed_pair(run, lambda: bs.apply(ins, 32, outs=outs), REPS, 2, torch.cuda.synchronize)
    g = gcells(cells, 32, ms)
    bg = gcells(cells, 32, bms)
    # The other grouping: each member at its own map depth (members finish
    # after different launch counts; later launches re-divide the device),
    # or the tuned uniform depth if the tuner chose the former.
    alt = st.BatchedStencil([dict(n=c.n[:2], shape=wl.SHAPE_NAMES[c.shape], radius=c.radius, coeffs=c.coeffs)
                             for c in cases], tsteps=3 if own else -1)
    bms2, ams = timed_pair(lambda: bs.apply(ins, 32, outs=outs), lambda: alt.apply(ins, 32, outs=outs), REPS, 2,
                           torch.cuda.synchronize)
    # Map depths the members of `alt` read (the tuner updated the map in process).
    depths = sorted(st.Stencil(c.n[:2], wl.SHAPE_NAMES[c.shape], c.radius, c.coeffs).describe()["tsteps"]
                    for c in cases)
    if own:
        launches = "one grouped launch per time block for the grids that have blocks left, each grid at its own map depth"
        bpc = None
    else:
        k = max(1, desc["tsteps"])
        launches = f"one grouped launch per time block of {k} fused steps for all 64 grids ({-(-32 // k)} launches)"
        bpc = 8 / k
    return {"workload": "batch64_2d_mixed_32steps_f32", "cells": cells, "ms": bms, "gcells_s": bg,
            "launches": launches + ", autotuned",
            "autotune": dict(tune, seconds=round(tune_s, 1)), "dispatch": desc,
            "bytes_per_cell_update": bpc, "hbm_frac": None if bpc is None else bg * bpc / HBM_PEAK_GBS,
            "equiv_frac_one_step": bg * 8 / HBM_PEAK_GBS,
            "ms_separate_launches": ms, "gcells_s_separate": g,
            "other_grouping": {"kind": "uniform batch depth 3" if own else "each grid at its own map depth",
                               "ms": ams, "gcells_s": gcells(cells, 32, ams), "ms_tuned_same_passes": bms2,
                               "member_map_depths": {str(d): depths.count(d) for d in sorted(set(depths))}},
            "timing": f"median of {REPS} passes interleaved with the 64 separate plain launches "
                      f"(and, separately, with the other grouping)"}


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
                                                    rec_z=case.rec_z, record=True), grad, REPS, 1,
                              torch.cuda.synchronize)
    dk, loss = res["g"]
    return {"workload": "wavegrad3d_star4_256^3_200steps_ckpt20", "fwd_ms": fwd_ms, "fwd_bwd_ms": g_ms,
            "ratio_fwd_bwd_over_fwd": g_ms / fwd_ms,
            "fwd_gcells_s": gcells(case.cells, case.steps, fwd_ms),
            "loss": float(loss.item()), "grad_finite": bool(torch.isfinite(dk).all().item())}


def host_info():
    """CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def _oracle_rate(fn, cell_updates):
    t0 = time.perf_counter()
    fn()
    dt = time.perf_counter() - t0
    return {"gcells_s": cell_updates / dt / 1e9, "seconds": round(dt, 2)}


def cpu_baseline(wl):
    """The FP64 oracle (unchanged, OpenMP over all host cores) on a bounded
    sample of the headline workload: a 384^3 grid, 20 leapfrog steps."""
    import oracle
    oracle.build(force=False)
    oracle.set_threads(0)
    n = 384
    case = wl.wave3d(n=n, steps=20)
    r = _oracle_rate(lambda: oracle.wave_forward(case.u_prev, case.u0, case.kappa, case.steps, r=4,
                                                 boundary=wl.ZERO), n ** 3 * case.steps)
    return dict({"value": r["gcells_s"], "unit": "GCells/s", "cores": oracle.max_threads(), "kind": "oracle",
                 "sample": f"wave leapfrog r=4, {n}^3 cells x 20 steps (same law as the 512^3 workload), "
                           f"FP64, {r['seconds']} s"}, **host_info())


def cpu_per_config(wl):
    """The FP64 oracle timed per workload on bounded samples of the same law
    (all host threads; one thread as well for the 2D Jacobi and 2D box)."""
    import oracle
    oracle.build(force=False)
    oracle.set_threads(0)
    allt = oracle.max_threads()
    res = {}

    def linear(tag, case, sample_desc, threads=(None,)):
        out = {"sample": sample_desc}
        for th in threads:
            oracle.set_threads(th or 0)
            rr = _oracle_rate(lambda: oracle.sweep(case.u0, case.coeffs, case.shape, case.radius, case.boundary,
                                                   case.steps), case.cells * case.steps)
            out["gcells_s" if th is None else f"gcells_s_{th}_thread"] = rr["gcells_s"]
        oracle.set_threads(0)
        out["threads"] = allt
        res[tag] = out

    linear("jacobi2d", wl.jacobi2d(), "the full workload: 512^2 x 10 steps", (None, 1))
    linear("box3d", wl.box3d(n=128, steps=5, dtype=wl.F16), "27-point box, 128^3 x 5 steps (fp16 inputs)")
    linear("star3d", wl.star3d(n=(256, 256, 256), steps=5), "7-point star, 256^3 x 5 steps")
    linear("box2d", wl.box2d(n=2048, steps=5, dtype=wl.F16), "25-point box, 2048^2 x 5 steps (fp16 inputs)",
           (None, 1))
    cases = wl.batch2d()[:8]
    for c in cases:
        c.steps = 4
    t0 = time.perf_counter()
    for c in cases:
        oracle.sweep(c.u0, c.coeffs, c.shape, c.radius, c.boundary, c.steps)
    dt = time.perf_counter() - t0
    res["batch64"] = {"sample": "the first 8 of the 64 grids x 4 steps", "threads": allt,
                      "gcells_s": sum(c.cells for c in cases) * 4 / dt / 1e9}
    g = wl.wavegrad3d(n=64)
    _, _, tg = oracle.wave_forward(g.u_prev, g.u0, g.kappa_true, g.steps, src=g.src, wavelet=g.wavelet,
                                   rec_z=g.rec_z)
    rr = _oracle_rate(lambda: oracle.wave_gradient(g.u_prev, g.u0, g.kappa, g.steps, g.src, g.wavelet, g.rec_z,
                                                   tg, ckpt_every=g.ckpt_every), g.cells * g.steps)
    res["wavegrad"] = {"sample": "gradient law at 64^3 x 200 steps, K = 20", "threads": allt,
                       "fwd_bwd_ms": rr["seconds"] * 1e3, "gcells_s_fwd_bwd": rr["gcells_s"]}
    # The oracle evaluates the leapfrog in FP64 whatever the storage, so the
    # f64 wave workload's CPU figure is the headline's cpu_baseline sample.
    res["wave3d_f64"] = {"sample": "the cpu_baseline sample (the FP64 oracle's leapfrog serves both storages)",
                         "threads": allt, "see": "cpu_baseline"}
    return res


def summarize_trace(path, kernel, skip):
    """Launch statistics of one kernel from a rocprofv3 kernel trace: the
    launches whose name contains `kernel`, in dispatch order, after the first
    `skip` (the warm-up passes).  Prints one JSON line (microseconds)."""
    import csv
    rows = []
    with open(path, newline="") as f:
        for rec in csv.DictReader(f):
            if kernel in rec.get("Kernel_Name", ""):
                rows.append((int(rec.get("Dispatch_Id") or 0), int(rec["Start_Timestamp"]),
                             int(rec["End_Timestamp"]), rec["Kernel_Name"]))
    rows.sort(key=lambda r: (r[1], r[0]))
    names = sorted({r[3] for r in rows})
    timed_rows = rows[skip:]
    d = np.array([(e - b) / 1e3 for _, b, e, _ in timed_rows], dtype=np.float64)
    out = {"trace": path, "kernel_filter": kernel, "kernels": names, "launches_total": len(rows),
           "skipped": skip, "launches": int(d.size)}
    if d.size:
        out.update({"mean_us": round(float(d.mean()), 2), "median_us": round(float(np.median(d)), 2),
                    "min_us": round(float(d.min()), 2), "max_us": round(float(d.max()), 2),
                    "sum_ms": round(float(d.sum()) / 1e3, 3)})
    print(json.dumps(out), flush=True)
    return out


def main():
    args = parse()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.kernel, args.skip)
        return
    if args.summarize_counters is not None:
        summarize_counters(args.summarize_counters)
        return
    if args.summarize_clock:
        summarize_clock(args.summarize_clock)
        return
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
        pmc_target(args.pmc_target, dev, st, wl, torch)
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
    if not args.no_stream_ceiling:
        # The same run's plain read-3/write-1 stream (the leapfrog's pointwise
        # traffic pattern): HBM rates differ from device to device, so the
        # kernel's share of this ceiling is the comparable figure.
        sc = stream_ceiling(dev, torch)
        line["roofline"]["stream_ceiling"] = {k: round(v, 1) for k, v in sc.items()}
        line["roofline"]["frac_of_stream"] = round(achieved / sc["read3_write1_gbs"], 4)
        torch.cuda.empty_cache()
    extras = {}
    if not args.quick:
        only = set(filter(None, args.only.split(",")))
        todo = [
            ("jacobi2d", lambda: {"jacobi2d": bench_jacobi(dev, st, wl, torch)}),
            ("box3d", lambda: dict(zip(("box3d_f16", "box3d_f32"), bench_linear_twins(
                dev, st, wl, torch, wl.box3d(dtype=wl.F16), wl.box3d(dtype=wl.F32))))),
            ("star3d", lambda: dict(zip(("star3d_f16", "star3d_f32"), bench_linear_twins(
                dev, st, wl, torch, wl.star3d(dtype=wl.F16), wl.star3d(dtype=wl.F32))))),
            ("star3d_f64", lambda: {"star3d_f64": bench_linear(dev, st, wl, torch, wl.star3d(dtype=wl.F64))}),
            ("varcoef_star1", lambda: {"varcoef_star1": bench_varcoef(dev, st, torch, "star", 1)}),
            ("varcoef_box1", lambda: {"varcoef_box1": bench_varcoef(dev, st, torch, "box", 1)}),
            ("varcoef2d_star1", lambda: {"varcoef2d_star1": bench_varcoef(dev, st, torch, "star", 1, n=4096,
                                                                          steps=20, ndim=2)}),
            ("box2d_f64", lambda: {"box2d_f64": bench_linear(dev, st, wl, torch, wl.box2d(dtype=wl.F64))}),
            ("box3d_r2", lambda: dict(zip(("box3d_r2_f16", "box3d_r2_f32"), bench_linear_twins(
                dev, st, wl, torch, wl.box3d_r2(dtype=wl.F16), wl.box3d_r2(dtype=wl.F32))))),
            ("box2d", lambda: dict(zip(("box2d_f16", "box2d_f32"), bench_linear_twins(
                dev, st, wl, torch, wl.box2d(dtype=wl.F16), wl.box2d(dtype=wl.F32))))),
            ("batch64", lambda: {"batch64": bench_batch(dev, st, wl, torch)}),
            ("wavegrad", lambda: {"wavegrad": bench_grad(dev, st, wl, torch)}),
            ("wave3d_sponge", lambda: {"wave3d_sponge": bench_wave_sponge(dev, st, wl, torch)}),
            ("wave3d_f64", lambda: {"wave3d_f64": bench_wave_f64(dev, st, wl, torch)}),
        ]
        for name, fn in todo:
            if only and name not in only:
                continue
            t0 = time.perf_counter()
            recs = fn()
            extras.update(recs)
            log(f"{name}: {json.dumps(recs)} ({time.perf_counter() - t0:.1f} s)")
            torch.cuda.empty_cache()
        line["per_config"] = extras
    if args.shapes:
        t0 = time.perf_counter()
        line["shapes"] = bench_shapes(dev, st, wl, torch)
        log(f"shapes: {json.dumps(line['shapes'])} ({time.perf_counter() - t0:.1f} s)")
    if not args.no_cpu:
        t0 = time.perf_counter()
        line["cpu_baseline"] = cpu_baseline(wl)
        log(f"cpu baseline: {line['cpu_baseline']} ({time.perf_counter() - t0:.1f} s)")
        if not args.quick:
            t0 = time.perf_counter()
            line["cpu_per_config"] = cpu_per_config(wl)
            log(f"cpu per config: {json.dumps(line['cpu_per_config'])} ({time.perf_counter() - t0:.1f} s)")
    if not finite:
        line["error"] = "non-finite wave field"
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
