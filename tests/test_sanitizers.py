"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle (plain C) is built with both sanitizers together with a driver
that calls every entry point on small grids, bad arguments included.  The
library's host side (plan creation and validation, option checks, dispatch
map and tuning-cache parsing, workspace sizes, coefficient reports, batched
plans and the argument checks that return before device work) is built with
the sanitizers on the host compilation only (device code is not
instrumented) and exercised by a second driver, without a GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(ROOT, "_build", "asan")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CSRC = os.path.join(ROOT, "paper_2609_06694_amd", "csrc")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-fopenmp", os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe])
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    r = _run([exe], env=env, timeout=300)
    assert r.stdout.strip().endswith("ok")


def _newer(target, sources):
    return os.path.exists(target) and all(os.path.getmtime(target) >= os.path.getmtime(s) for s in sources)


def _build_sanitized_library():
    from paper_2609_06694_amd import build as hb
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "libstencil_asan.so")
    srcs = [os.path.join(CSRC, f) for f in hb.SOURCES]
    deps = srcs + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")] + \
        [os.path.join(ROOT, "include", "stencil.h")]
    if _newer(lib, deps):
        return lib
    procs, objs = [], []
    for src in srcs:
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer"] + SAN_HOST + \
              [f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
        if src.endswith(".hip"):
            cmd += ["-x", "hip"] + hb.DEVICE_FLAGS
        cmd += ["-c", src, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(obj)
        while sum(p.poll() is None for _, p in procs) >= 8:
            procs[[p.poll() is None for _, p in procs].index(True)][1].wait()
    for src, p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, f"sanitized build of {src} failed:\n{err[-3000:]}"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + SAN_HOST + ["-o", lib] + objs + ["-ldl"])
    return lib


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc missing")
def test_runtime_host_paths_under_address_and_ub_sanitizers(tmp_path):
    lib = _build_sanitized_library()
    exe = str(tmp_path / "runtime_driver")
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer"] + SAN_HOST +
         [f"-I{os.path.join(ROOT, 'include')}", os.path.join(HERE, "runtime_driver.cpp"), "-o", exe,
          f"-L{OUT}", "-lstencil_asan", f"-Wl,-rpath,{OUT}"])
    cache = tmp_path / "tune.txt"
    cache.write_text("# tuning cache with malformed lines\n3 1 1 1 0 0 4 0 2 0 16 1 64\ngarbage\n"
                     "2 0 1 0 0 0 0 0 1 32 32 16\n9 9 9 9 9 9 9 9 9 9 9 9 9 9 9\n")
    r = _run([exe], env=dict(ENV, STENCIL_TUNE_CACHE=str(cache)), timeout=300)
    assert r.stdout.strip().endswith("ok")
