"""MI355X-native repeated stencil sweeps (2D/3D star and box, radius 1-4,
f32 or fp16 storage) with per-case HIP kernels behind a C ABI.

The compute path is ``libstencil.so`` (hand-written HIP for gfx950); this
package is the thin ctypes binding plus seeded input generators.  Importing
the package does not load the library; :func:`load_library` does, and fails
loudly if it has not been built.
"""
__all__ = ["workloads", "load_library"]


def load_library():
    from ._abi import lib
    return lib()
