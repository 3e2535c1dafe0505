"""Regenerate the shipped dispatch map (dispatch_mi355x.txt next to the
library) by running the autotuner on the benchmark workloads' cases.

Usage (on the GPU machine): python -m paper_2609_06694_amd.tune_defaults OUT [WORDS]
Each tuned case key is appended to OUT; copy OUT to the package directory as
dispatch_mi355x.txt to make it the default map.  WORDS (comma-separated)
tunes only the workloads whose name contains every word, for refreshing
some entries of the map.
"""
from __future__ import annotations

import os
import sys



def main(out: str, words: str = "") -> None:
    os.environ["STENCIL_TUNE_CACHE"] = out
    os.environ.pop("STENCIL_TUNE_FAULT", None)
    import torch  # noqa: F401  (device memory for the scratch buffers)
    from . import stencil as st, workloads as wl
    open(out, "w").write("# ndim shape r dtype boundary update size_class slab variant tile_x tile_y tsteps zchunk\n")
    plans = []
    c = wl.jacobi2d()
    plans.append(("jacobi2d 512^2", st.Stencil(c.n[:2], "star", 1, c.coeffs)))
    for dt in ("f16", "f32"):
        c = wl.box3d(n=16, dtype=wl.F16 if dt == "f16" else wl.F32)
        plans.append((f"box3d 512^3 {dt}", st.Stencil((512, 512, 512), "box", 1, c.coeffs, dtype=dt)))
        c = wl.box3d_r2(n=16, dtype=wl.F16 if dt == "f16" else wl.F32)
        plans.append((f"box3d r2 512^3 {dt}", st.Stencil((512, 512, 512), "box", 2, c.coeffs, dtype=dt)))
        c = wl.box2d(n=16, dtype=wl.F16 if dt == "f16" else wl.F32)
        plans.append((f"box2d 4096^2 {dt}", st.Stencil((4096, 4096), "box", 2, c.coeffs, dtype=dt)))
    for dt in ("f16", "f32", "f64"):
        c = wl.star3d(n=(16, 16, 16))
        plans.append((f"star3d 512^3 {dt}", st.Stencil((512, 512, 512), "star", 1, c.coeffs, dtype=dt)))
    c = wl.box3d(n=16, dtype=wl.F32)
    plans.append(("box3d 512^3 f64", st.Stencil((512, 512, 512), "box", 1, c.coeffs, dtype="f64")))
    # Slabs: few planes, a long column, thin across the march.
    for dt in ("f16", "f32"):
        for shp in ((4096, 4096, 8), (64, 64, 32768), (4096, 64, 512)):
            c = wl.star3d(n=(16, 16, 16))
            plans.append((f"star3d slab {shp} {dt}", st.Stencil(shp, "star", 1, c.coeffs, dtype=dt)))
            c = wl.box3d(n=16, dtype=wl.F32)
            plans.append((f"box3d slab {shp} {dt}", st.Stencil(shp, "box", 1, c.coeffs, dtype=dt)))
    # Smaller cubes fall in other size classes (fewer tiles: more plane chunks).
    for m in (128, 256):
        for dt in ("f16", "f32"):
            c = wl.star3d(n=(16, 16, 16))
            plans.append((f"star3d {m}^3 {dt}", st.Stencil((m, m, m), "star", 1, c.coeffs, dtype=dt)))
            c = wl.box3d(n=16, dtype=wl.F32)
            plans.append((f"box3d {m}^3 {dt}", st.Stencil((m, m, m), "box", 1, c.coeffs, dtype=dt)))
    # The 125-point box on small cubes and on slabs (the march along y and
    # the whole-block kernel are candidates there).
    for dt in ("f16", "f32"):
        c = wl.box3d_r2(n=16, dtype=wl.F16 if dt == "f16" else wl.F32)
        for shp in ((128, 128, 128), (256, 256, 256), (4096, 4096, 8), (4096, 64, 512), (64, 64, 32768)):
            plans.append((f"box3d r2 {shp} {dt}", st.Stencil(shp, "box", 2, c.coeffs, dtype=dt)))
    plans.append(("varcoef star1 512^3 f32", st.VarCoefStencil((512, 512, 512), "star", 1)))
    plans.append(("varcoef box1 512^3 f32", st.VarCoefStencil((512, 512, 512), "box", 1)))
    plans.append(("wave 512^3", st.WaveModel((512, 512, 512))))
    plans.append(("wave 256^3", st.WaveModel((256, 256, 256))))
    # One representative grid per case key of the 64-grid workload; the
    # 512^2 Jacobi grid keeps its own entry.
    seen = {(wl.STAR, 1, 0, False)}
    for g in wl.batch2d():
        cells = g.n[0] * g.n[1]
        size_class = sum(cells > 1 << b for b in (18, 20, 22, 25))
        lo, hi = min(g.n[:2]), max(g.n[:2])
        slab = 0 if hi < 4 * lo else (1 if g.n[1] == lo else (2 if g.n[1] == hi else 3))
        key = (g.shape, g.radius, size_class, slab)
        if key in seen:
            continue
        seen.add(key)
        plans.append((g.name, st.Stencil(g.n[:2], wl.SHAPE_NAMES[g.shape], g.radius, g.coeffs)))
    need = [w for w in words.split(",") if w]
    for name, p in plans:
        if not all(w in name for w in need):
            continue
        stats = p.autotune()
        print(f"{name}: {p.describe()} {stats}", flush=True)
        torch.cuda.empty_cache()
    # Two tuned workloads that share a case key overwrite each other's entry.
    keys = [tuple(line.split()[:8]) for line in open(out) if line.strip() and not line.startswith("#")]
    dup = sorted({k for k in keys if keys.count(k) > 1})
    if dup:
        print(f"warning: case keys tuned more than once (the last entry wins): {dup}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "dispatch_tuned.txt", sys.argv[2] if len(sys.argv) > 2 else "")
