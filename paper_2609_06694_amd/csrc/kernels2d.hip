// 2D linear sweep: one workgroup per output tile, k time steps fused in LDS.
#include "internal.h"
#include "tb2d_tile.h"

namespace stk {

template <int R, int SHAPE, typename T, int BC, int NW>
__global__ __launch_bounds__(NW * kWave) void tb2d_kernel(const T* __restrict__ in,
                                                        T* __restrict__ out, int nx, int ny,
                                                        int BX, int BY, int k, int tiles_x,
                                                        Taps taps) {
    extern __shared__ float lds[];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tyi = b / tiles_x, txi = b - tyi * tiles_x;
    tb2d_tile<R, SHAPE, T, BC, NW>(in, out, nx, ny, txi * BX, tyi * BY, BX, BY, k, taps, lds);
}

int tb2d_max_lds_bytes() { return 64 * 1024; }

int tb2d_lds_floats_host(int BX, int BY, int k, int R) { return tb2d_lds_floats(BX, BY, k, R); }

bool tb2d_supported(int r, int shape) {
    if (shape == kStar) return r >= 1 && r <= 4;
    return r >= 1 && r <= 2;
}

template <int R, int SHAPE, typename T, int BC, int NW>
static hipError_t go(const Geom& g, int BX, int BY, int k, const Taps& taps, const void* in,
                     void* out, hipStream_t s) {
    const int tiles_x = (g.nx + BX - 1) / BX, tiles_y = (g.ny + BY - 1) / BY;
    const size_t lds = sizeof(float) * (size_t)tb2d_lds_floats(BX, BY, k, R);
    hipLaunchKernelGGL((tb2d_kernel<R, SHAPE, T, BC, NW>), dim3(tiles_x * tiles_y), dim3(NW * kWave),
                       lds, s, (const T*)in, (T*)out, g.nx, g.ny, BX, BY, k, tiles_x, taps);
    return hipGetLastError();
}

// g.waves: 4, 8 or 16 waves per workgroup.
template <int R, int SHAPE, typename T, int BC>
static hipError_t go_nw(const Geom& g, int BX, int BY, int k, const Taps& taps, const void* in,
                        void* out, int nw, hipStream_t s) {
    if (nw == 16) return go<R, SHAPE, T, BC, 16>(g, BX, BY, k, taps, in, out, s);
    if (nw == 8) return go<R, SHAPE, T, BC, 8>(g, BX, BY, k, taps, in, out, s);
    return go<R, SHAPE, T, BC, 4>(g, BX, BY, k, taps, in, out, s);
}

template <int R, int SHAPE, typename T>
static hipError_t go_bc(const Geom& g, int BX, int BY, int k, const Taps& taps, const void* in,
                        void* out, int nw, hipStream_t s) {
    return g.boundary == kPeriodic ? go_nw<R, SHAPE, T, kPeriodic>(g, BX, BY, k, taps, in, out, nw, s)
                                   : go_nw<R, SHAPE, T, kZero>(g, BX, BY, k, taps, in, out, nw, s);
}

template <typename T>
static hipError_t go_t(const Geom& g, int BX, int BY, int k, const Taps& taps, const void* in,
                       void* out, int nw, hipStream_t s) {
    if (g.shape == kStar) {
        switch (g.r) {
            case 1: return go_bc<1, kStar, T>(g, BX, BY, k, taps, in, out, nw, s);
            case 2: return go_bc<2, kStar, T>(g, BX, BY, k, taps, in, out, nw, s);
            case 3: return go_bc<3, kStar, T>(g, BX, BY, k, taps, in, out, nw, s);
            case 4: return go_bc<4, kStar, T>(g, BX, BY, k, taps, in, out, nw, s);
        }
    } else {
        switch (g.r) {
            case 1: return go_bc<1, kBox, T>(g, BX, BY, k, taps, in, out, nw, s);
            case 2: return go_bc<2, kBox, T>(g, BX, BY, k, taps, in, out, nw, s);
        }
    }
    return hipErrorInvalidValue;
}

// cfg.tile_x x cfg.tile_y outputs per workgroup; cfg.zchunk: waves per
// workgroup (0 = 4; 8 or 16).
hipError_t launch_tb2d(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                       void* out, int k, hipStream_t stream) {
    if (k < 1 || cfg.tile_x < 8 || cfg.tile_y < 1) return hipErrorInvalidValue;
    const int nw = cfg.zchunk == 0 ? 4 : cfg.zchunk;
    if (nw != 4 && nw != 8 && nw != 16) return hipErrorInvalidValue;
    if (g.dtype != 0 && g.dtype != 1) return hipErrorInvalidValue;   // fp16 / f32 storage only
    if ((int)sizeof(float) * tb2d_lds_floats(cfg.tile_x, cfg.tile_y, k, g.r) > tb2d_max_lds_bytes())
        return hipErrorInvalidValue;
    if (g.dtype == 0) return go_t<float>(g, cfg.tile_x, cfg.tile_y, k, taps, in, out, nw, stream);
    return go_t<_Float16>(g, cfg.tile_x, cfg.tile_y, k, taps, in, out, nw, stream);
}

}  // namespace stk
