// 2D row-march kernel (one grid per launch) and its launcher; the march
// itself is ym2d_run.
#include <algorithm>

#include "internal.h"
#include "ym2d_run.h"

namespace stk {

template <int R, int SHAPE, typename T, int BC, int NT, int RY, int D>
__global__ __launch_bounds__(NT) void ym2d_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                  int nx, int ny, int k, int ow, int ych, int strips,
                                                  Taps tp) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    ym2d_run<R, SHAPE, T, BC, NT, RY, D>(in, out, nx, ny, k, k, ow, ych, strips,
                                         xcd_remap(blockIdx.x, gridDim.x), tp,
                                         reinterpret_cast<acc_t<T>*>(lds_raw));
}

// esz: bytes of the arithmetic type (4, or 8 for f64 storage).
int ym2d_lds_bytes(int nt, int k, int R, int esz) {
    const int RY = ym2d_rows(nt, k, R, esz);
    return esz * k * ym2d_ring_rows(RY, R) * (nt + 2 * R);
}

int ym2d_rows(int nt, int k, int R, int esz) {
    // Eight rows per iteration unless the rings would outgrow 64 KiB.
    return esz * k * ym2d_ring_rows(8, R) * (nt + 2 * R) <= 64 * 1024 ? 8 : 4;
}

int ym2d_max_lds_bytes() { return 160 * 1024; }

// Rows per chunk when the configuration leaves it open: enough workgroups to
// give every CU about two, but chunks of at least 4kR rows, so the re-read
// and recomputed halo rows stay below half of the work.
int ym2d_auto_chunk(int nx, int ny, int nt, int k, int R) {
    const int ow = nt - 2 * k * R;
    const int strips = (nx + ow - 1) / ow;
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            cus = n;
    }
    const int target = 2 * cus * (nt == 256 ? 2 : 1);
    int chunks = std::max(1, target / std::max(1, strips));
    int ych = (ny + chunks - 1) / chunks;
    ych = std::max(ych, std::max(16, 4 * k * R));
    return std::min(ych, ny);
}

bool ym2d_supported(int r, int shape) {
    if (shape == kStar) return r >= 1 && r <= 4;
    return r >= 1 && r <= 2;
}

template <int R, int SHAPE, typename T, int BC, int NT, int RY>
static hipError_t go(const Geom& g, int k, int ych, const Taps& tp, const void* in, void* out,
                     hipStream_t s) {
    constexpr int D = 2;
    const int ow = NT - 2 * k * R;
    const int strips = (g.nx + ow - 1) / ow;
    const int chunks = (g.ny + ych - 1) / ych;
    const size_t lds = sizeof(acc_t<T>) * (size_t)k * ym2d_ring_rows(RY, R) * (NT + 2 * R);
    if (lds > 64 * 1024) {
        hipError_t e = allow_large_lds<ym2d_kernel<R, SHAPE, T, BC, NT, RY, D>>();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((ym2d_kernel<R, SHAPE, T, BC, NT, RY, D>), dim3(strips * chunks), dim3(NT), lds, s,
                       (const T*)in, (T*)out, g.nx, g.ny, k, ow, ych, strips, tp);
    return hipGetLastError();
}

template <int R, int SHAPE, typename T, int BC, int NT>
static hipError_t go_ry(const Geom& g, int k, int ych, const Taps& tp, const void* in, void* out,
                        hipStream_t s) {
    if (ym2d_rows(NT, k, R, (int)sizeof(acc_t<T>)) == 8) return go<R, SHAPE, T, BC, NT, 8>(g, k, ych, tp, in, out, s);
    return go<R, SHAPE, T, BC, NT, 4>(g, k, ych, tp, in, out, s);
}

template <int R, int SHAPE, typename T, int BC>
static hipError_t go_nt(const Geom& g, int nt, int k, int ych, const Taps& tp, const void* in,
                        void* out, hipStream_t s) {
    if (nt == 512) return go_ry<R, SHAPE, T, BC, 512>(g, k, ych, tp, in, out, s);
    return go_ry<R, SHAPE, T, BC, 256>(g, k, ych, tp, in, out, s);
}

template <int R, int SHAPE, typename T>
static hipError_t go_bc(const Geom& g, int nt, int k, int ych, const Taps& tp, const void* in,
                        void* out, hipStream_t s) {
    return g.boundary == kPeriodic ? go_nt<R, SHAPE, T, kPeriodic>(g, nt, k, ych, tp, in, out, s)
                                   : go_nt<R, SHAPE, T, kZero>(g, nt, k, ych, tp, in, out, s);
}

template <typename T>
static hipError_t go_t(const Geom& g, int nt, int k, int ych, const Taps& tp, const void* in,
                       void* out, hipStream_t s) {
    if (g.shape == kStar) {
        switch (g.r) {
            case 1: return go_bc<1, kStar, T>(g, nt, k, ych, tp, in, out, s);
            case 2: return go_bc<2, kStar, T>(g, nt, k, ych, tp, in, out, s);
            case 3: return go_bc<3, kStar, T>(g, nt, k, ych, tp, in, out, s);
            case 4: return go_bc<4, kStar, T>(g, nt, k, ych, tp, in, out, s);
        }
    } else {
        switch (g.r) {
            case 1: return go_bc<1, kBox, T>(g, nt, k, ych, tp, in, out, s);
            case 2: return go_bc<2, kBox, T>(g, nt, k, ych, tp, in, out, s);
        }
    }
    return hipErrorInvalidValue;
}

// cfg.tile_x: window width (threads per workgroup, 256 or 512); cfg.tile_y:
// rows per chunk (0: automatic); k fused steps.
hipError_t launch_ym2d(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                       void* out, int k, hipStream_t stream) {
    const int nt = cfg.tile_x == 512 ? 512 : 256;
    if (k < 1 || (cfg.tile_x != 256 && cfg.tile_x != 512) || nt - 2 * k * g.r < kWave) return hipErrorInvalidValue;
    const int esz = g.dtype == 2 ? 8 : 4;
    if (ym2d_lds_bytes(nt, k, g.r, esz) > ym2d_max_lds_bytes()) return hipErrorInvalidValue;
    const int ych = cfg.tile_y > 0 ? std::min(cfg.tile_y, g.ny)
                                   : ym2d_fill_chunk(ym2d_auto_chunk(g.nx, g.ny, nt, k, g.r), k * g.r,
                                                     ym2d_rows(nt, k, g.r, esz), g.ny);
    if (g.dtype == 0) return go_t<float>(g, nt, k, ych, taps, in, out, stream);
    if (g.dtype == 2) return go_t<double>(g, nt, k, ych, taps, in, out, stream);
    return go_t<_Float16>(g, nt, k, ych, taps, in, out, stream);
}

}  // namespace stk
