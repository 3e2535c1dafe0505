// 2D linear sweep, k time steps per launch, by a row march (y-march).
//
// A workgroup of NT threads owns a window of NT columns and marches down a
// chunk of rows.  Thread x keeps window column x.  Each iteration brings RY
// new input rows (time level 0) into an LDS row ring; then, one stage per
// fused step s = 1..k, it computes RY rows of level s from the ring of level
// s-1, R rows behind the rows that level s-1 just produced, and puts them in
// the ring of level s (the last stage writes them to HBM).  Intermediate
// time levels never leave the chip (temporal blocking, Section 4.3), and
// because rows stream, the redundant halo computation of a fused step is
// paid in x only: level s is valid on window columns [sR, NT - sR), so the
// NT - 2kR middle columns are the workgroup's outputs.  A chunk of rows
// re-reads and recomputes kR rows above and below it.
//
// Each level's ring holds C = RY + 2R rows: stage s+1 reads exactly the C
// newest rows of level s, and the next iteration overwrites the RY oldest
// ones only after the barrier that follows stage s+1 (for k = 1 an extra
// barrier closes every iteration).  Rows of a level above its first valid
// row (Y + sR) are computed from rows not yet loaded; they feed only other
// such rows and are never written out.
//
// Input rows are loaded D iterations ahead into registers, every load
// unconditional (coordinates clamped or wrapped; cells outside a zero frame
// are masked when staged), so the compiler keeps all of them in flight.
// fp16 storage: every intermediate level is rounded to binary16, exactly as
// one launch per step would store it; arithmetic is FP32.  Zero frame: cells
// outside the grid are zero at every level.
#include <algorithm>

#include "internal.h"

namespace stk {

template <int BC>
__device__ __forceinline__ bool ym_fix(int& i, int n) {
    if (BC == kPeriodic) {
        i = wrap_index(i, n);
        return true;
    }
    const bool ok = (unsigned)i < (unsigned)n;
    i = min(max(i, 0), n - 1);
    return ok;
}

template <int R, int SHAPE, typename T, int BC, int NT, int RY, int D>
__global__ __launch_bounds__(NT) void ym2d_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                  int nx, int ny, int k, int ow, int ych, int strips,
                                                  Taps tp) {
    constexpr int C = RY + 2 * R;       // ring rows per level
    constexpr int RW = NT + 2 * R;      // ring row width: R pad columns on each side
    extern __shared__ float lds[];      // k rings of C x RW floats
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int si = b % strips, ci = b / strips;
    const int x = threadIdx.x;
    const int kr = k * R;
    const int wx0 = si * ow - kr;                 // window origin column
    const int oy0 = ci * ych, oy1 = min(oy0 + ych, ny);
    const int Y = oy0 - kr;                       // first level-0 row of the march
    const int iters = (oy1 - oy0 + 2 * kr + RY - 1) / RY;

    // This thread's column: load address (wrapped or clamped) and validity.
    int gxl = wx0 + x;
    const bool colin = ym_fix<BC>(gxl, nx);
    const int gx = wx0 + x;                        // unclamped grid column
    const bool out_col = x >= kr && x < kr + ow && gx < nx;

    T v[D][RY];
    uint32_t vm[D];
    auto issue = [&](int slot, int it) {
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            int gy = Y + it * RY + j;
            const bool ok = ym_fix<BC>(gy, ny) && colin;
            v[slot][j] = in[(size_t)gy * nx + gxl];
            m |= (uint32_t)ok << j;
        }
        vm[slot] = m;
    };
#pragma unroll
    for (int d = 0; d < D; ++d) issue(d, d);

    for (int i0 = 0; i0 < iters; i0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int i = i0 + d;   // iterations past `iters` compute rows no one reads
            // Uniform ring offset of this iteration: stage s+1 reads level-s
            // slots base+0 .. base+C-1 (mod C); stage s writes base+2R+j.
            int base = (i * RY - 2 * R) % C;
            base = base < 0 ? base + C : base;

            // Stage 0: stage the input rows of this iteration in ring 0.
            {
                float* r0 = lds;
#pragma unroll
                for (int j = 0; j < RY; ++j) {
                    int q = base + 2 * R + j;
                    q = q >= C ? q - C : q;
                    const float val = to_f32(v[d][j]);
                    r0[q * RW + R + x] = (BC == kPeriodic || ((vm[d] >> j) & 1u)) ? val : 0.f;
                }
            }
            issue(d, i + D);
            __syncthreads();

            for (int s = 1; s <= k; ++s) {
                const float* src = lds + (s - 1) * (C * RW);
                float acc[RY];
                if constexpr (SHAPE == kBox) {
#pragma unroll
                    for (int j = 0; j < RY; ++j) acc[j] = 0.f;
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        float col[C];
#pragma unroll
                        for (int j = 0; j < C; ++j) {
                            int q = base + j;
                            q = q >= C ? q - C : q;
                            col[j] = src[q * RW + R + x + dx];
                        }
#pragma unroll
                        for (int j = 0; j < RY; ++j)
#pragma unroll
                            for (int dy = -R; dy <= R; ++dy)
                                acc[j] = fmaf(tp.c[box2<R>(dy, dx)], col[j + R + dy], acc[j]);
                    }
                } else {
                    float col[C];
#pragma unroll
                    for (int j = 0; j < C; ++j) {
                        int q = base + j;
                        q = q >= C ? q - C : q;
                        col[j] = src[q * RW + R + x];
                    }
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        float a = tp.c[0] * col[j + R];
#pragma unroll
                        for (int e = 1; e <= R; ++e) {
                            a = fmaf(tp.c[star_y<R>(-e)], col[j + R - e], a);
                            a = fmaf(tp.c[star_y<R>(e)], col[j + R + e], a);
                        }
                        acc[j] = a;
                    }
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        int q = base + R + j;
                        q = q >= C ? q - C : q;
                        const float* row = src + q * RW + R + x;
#pragma unroll
                        for (int e = 1; e <= R; ++e) {
                            acc[j] = fmaf(tp.c[star_x<R>(-e)], row[-e], acc[j]);
                            acc[j] = fmaf(tp.c[star_x<R>(e)], row[e], acc[j]);
                        }
                    }
                }
                const int y0 = Y + i * RY - s * R;   // global row of acc[0]
                if (s < k) {
                    float* dst = lds + s * (C * RW);
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        int q = base + 2 * R + j;
                        q = q >= C ? q - C : q;
                        float val = round_to_storage<T>(acc[j]);
                        if (BC == kZero) {
                            const int gy = y0 + j;
                            if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) val = 0.f;
                        }
                        dst[q * RW + R + x] = val;
                    }
                    __syncthreads();
                } else if (out_col) {
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        const int gy = y0 + j;
                        if (gy >= oy0 && gy < oy1)
                            __builtin_nontemporal_store(from_f32<T>(acc[j]), &out[(size_t)gy * nx + gx]);
                    }
                }
            }
            if (k == 1) __syncthreads();
        }
    }
}

int ym2d_lds_bytes(int nt, int k, int R) {
    const int RY = ym2d_rows(nt, k, R);
    return (int)sizeof(float) * k * (RY + 2 * R) * (nt + 2 * R);
}

int ym2d_rows(int nt, int k, int R) {
    // Eight rows per iteration unless the rings would outgrow 64 KiB.
    return (int)sizeof(float) * k * (8 + 2 * R) * (nt + 2 * R) <= 64 * 1024 ? 8 : 4;
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
    const size_t lds = sizeof(float) * (size_t)k * (RY + 2 * R) * (NT + 2 * R);
    auto kern = ym2d_kernel<R, SHAPE, T, BC, NT, RY, D>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(strips * chunks), dim3(NT), lds, s, (const T*)in, (T*)out, g.nx, g.ny,
                       k, ow, ych, strips, tp);
    return hipGetLastError();
}

template <int R, int SHAPE, typename T, int BC, int NT>
static hipError_t go_ry(const Geom& g, int k, int ych, const Taps& tp, const void* in, void* out,
                        hipStream_t s) {
    if (ym2d_rows(NT, k, R) == 8) return go<R, SHAPE, T, BC, NT, 8>(g, k, ych, tp, in, out, s);
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
    if (ym2d_lds_bytes(nt, k, g.r) > ym2d_max_lds_bytes()) return hipErrorInvalidValue;
    const int ych = cfg.tile_y > 0 ? std::min(cfg.tile_y, g.ny) : ym2d_auto_chunk(g.nx, g.ny, nt, k, g.r);
    if (g.dtype == 0) return go_t<float>(g, nt, k, ych, taps, in, out, stream);
    return go_t<_Float16>(g, nt, k, ych, taps, in, out, stream);
}

}  // namespace stk
