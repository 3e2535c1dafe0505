// 2D linear sweep: one workgroup per output tile, k time steps fused in LDS.
#include "internal.h"
#include "tb2d_tile.h"

namespace stk {

template <int R, int SHAPE, typename T, int BC>
__global__ __launch_bounds__(kThreads) void tb2d_kernel(const T* __restrict__ in,
                                                        T* __restrict__ out, int nx, int ny,
                                                        int BX, int BY, int k, int tiles_x,
                                                        Taps taps) {
    extern __shared__ float lds[];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tyi = b / tiles_x, txi = b - tyi * tiles_x;
    tb2d_tile<R, SHAPE, T, BC>(in, out, nx, ny, txi * BX, tyi * BY, BX, BY, k, taps, lds);
}

int tb2d_max_lds_bytes() { return 64 * 1024; }

int tb2d_lds_floats_host(int BX, int BY, int k, int R) { return tb2d_lds_floats(BX, BY, k, R); }

bool tb2d_supported(int r, int shape) {
    if (shape == kStar) return r >= 1 && r <= 4;
    return r >= 1 && r <= 2;
}

template <int R, int SHAPE, typename T, int BC>
static hipError_t go(const Geom& g, int BX, int BY, int k, const Taps& taps, const void* in,
                     void* out, hipStream_t s) {
    const int tiles_x = (g.nx + BX - 1) / BX, tiles_y = (g.ny + BY - 1) / BY;
    const size_t lds = sizeof(float) * (size_t)tb2d_lds_floats(BX, BY, k, R);
    hipLaunchKernelGGL((tb2d_kernel<R, SHAPE, T, BC>), dim3(tiles_x * tiles_y), dim3(kThreads),
                       lds, s, (const T*)in, (T*)out, g.nx, g.ny, BX, BY, k, tiles_x, taps);
    return hipGetLastError();
}

template <int R, int SHAPE, typename T>
static hipError_t go_bc(const Geom& g, int BX, int BY, int k, const Taps& taps, const void* in,
                        void* out, hipStream_t s) {
    return g.boundary == kPeriodic ? go<R, SHAPE, T, kPeriodic>(g, BX, BY, k, taps, in, out, s)
                                   : go<R, SHAPE, T, kZero>(g, BX, BY, k, taps, in, out, s);
}

template <typename T>
static hipError_t go_t(const Geom& g, int BX, int BY, int k, const Taps& taps, const void* in,
                       void* out, hipStream_t s) {
    if (g.shape == kStar) {
        switch (g.r) {
            case 1: return go_bc<1, kStar, T>(g, BX, BY, k, taps, in, out, s);
            case 2: return go_bc<2, kStar, T>(g, BX, BY, k, taps, in, out, s);
            case 3: return go_bc<3, kStar, T>(g, BX, BY, k, taps, in, out, s);
            case 4: return go_bc<4, kStar, T>(g, BX, BY, k, taps, in, out, s);
        }
    } else {
        switch (g.r) {
            case 1: return go_bc<1, kBox, T>(g, BX, BY, k, taps, in, out, s);
            case 2: return go_bc<2, kBox, T>(g, BX, BY, k, taps, in, out, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tb2d(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                       void* out, int k, hipStream_t stream) {
    if (k < 1 || cfg.tile_x < kWave || cfg.tile_x % kWave || cfg.tile_y < 1) return hipErrorInvalidValue;
    if (g.dtype != 0 && g.dtype != 1) return hipErrorInvalidValue;   // fp16 / f32 storage only
    if ((int)sizeof(float) * tb2d_lds_floats(cfg.tile_x, cfg.tile_y, k, g.r) > tb2d_max_lds_bytes())
        return hipErrorInvalidValue;
    if (g.dtype == 0) return go_t<float>(g, cfg.tile_x, cfg.tile_y, k, taps, in, out, stream);
    return go_t<_Float16>(g, cfg.tile_x, cfg.tile_y, k, taps, in, out, stream);
}

}  // namespace stk
