// 3D 27-point box sweep with fp16 storage on the matrix cores (MFMA).
//
// With fp16 storage a 27-point box costs 27 FP32 multiply-adds per 4 bytes
// of traffic, so the vector-ALU z-march is compute-bound well below the HBM
// roofline.  Here the in-plane part is recast as a dense contraction
// (Section 7.2.3: box stencils mapped onto tensor cores): for one input
// plane, one row offset dy and one output plane offset dz,
//
//     D[x][y] += sum_k A[x][k] * B[k][y],   A[x][k] = c(dz, dy, k - 8 - x),
//                                           B[k][y] = u(x0 - 8 + k, y + dy)
//
// over a 16 x 16 output block and a 32-wide window of input columns, which is
// one v_mfma_f32_16x16x32_f16.  A is a banded Toeplitz matrix of coefficients
// (three nonzero diagonals), the same for every block, so it lives in
// registers for the whole launch; B is read straight from the LDS plane tile
// as 8 consecutive fp16 values per lane (16-byte reads).  Each B serves the
// three output planes the input plane feeds.  Products of fp16 values are
// exact in FP32 and the accumulation is FP32; the coefficients are split
// into fp16 high and low parts (c ~= hi + lo to ~2^-22 relative), so the
// result carries FP32 coefficients at twice the MFMA count.  Outputs are
// rounded to fp16 once per step, as on the vector path.
//
// A workgroup of four waves owns a 64 x 64 output tile (each wave 16 rows,
// four 16-column blocks) and marches z; each plane is staged once in LDS
// with one halo row above and below and eight columns on each side (keeping
// every 16-byte chunk aligned), loaded D planes ahead by unconditional 16-byte
// loads with a validity mask (grids need nx % 8 == 0).  The contributions of
// a plane go to a queue of three accumulator sets (output planes zp+1, zp,
// zp-1); the oldest is complete after the plane and is stored.
#include "internal.h"

namespace stk {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // native vector: stays in registers

constexpr int kMX = 64;               // tile width (output columns)
constexpr int kMY = 64;               // tile height: four waves x 16 rows
constexpr int kLW = 88;               // LDS row pitch in halves (80 used; pitch spreads banks)
constexpr int kLH = kMY + 2;          // rows staged: one halo row above and below
constexpr int kCH = (kMX + 16) / 8;   // 16-byte chunks per staged row
constexpr int kNCH = kCH * kLH;       // chunks per plane
constexpr int kCPT = (kNCH + kThreads - 1) / kThreads;   // chunks per thread
static_assert(kCPT <= 32, "validity mask holds 32 chunks");

template <int BC>
__device__ __forceinline__ bool mf_fix(int& i, int n) {
    if (BC == kPeriodic) {
        i = i < 0 ? i + n : (i >= n ? i - n : i);
        if ((unsigned)i >= (unsigned)n) i = wrap_index(i, n);   // grids smaller than the halo
        return true;
    }
    const bool ok = (unsigned)i < (unsigned)n;
    i = min(max(i, 0), n - 1);
    return ok;
}

// Issues the 16-byte loads of plane zp (this thread's kCPT chunks) and
// returns their validity mask.
template <int BC>
__device__ __forceinline__ uint32_t mf_load(const _Float16* __restrict__ in, int nx, int ny, int nz,
                                            int zp, int x0, int y0, u32x4 (&v)[kCPT]) {
    int gz = zp;
    const bool zin = mf_fix<BC>(gz, nz);
    const _Float16* pl = in + (size_t)gz * nx * ny;
    uint32_t m = 0;
#pragma unroll
    for (int t = 0; t < kCPT; ++t) {
        const int q0 = threadIdx.x + t * kThreads;
        const bool qv = q0 < kNCH;
        const int q = qv ? q0 : 0;
        const int row = q / kCH, cc = q - row * kCH;
        int gy = y0 - 1 + row, gx = x0 - 8 + 8 * cc;
        const bool oy = mf_fix<BC>(gy, ny);
        bool ox;
        if (BC == kPeriodic) {
            ox = mf_fix<BC>(gx, nx);   // stays a multiple of 8 (nx % 8 == 0)
        } else {
            ox = gx >= 0 && gx + 8 <= nx;
            gx = min(max(gx, 0), nx - 8);
        }
        v[t] = *(const u32x4*)(pl + (size_t)gy * nx + gx);
        m |= (uint32_t)(zin && oy && ox && qv) << t;
    }
    return m;
}

// Stages one loaded plane in LDS (zeros where the mask says outside).
__device__ __forceinline__ void mf_stage(_Float16* __restrict__ t, const u32x4 (&v)[kCPT], uint32_t m) {
#pragma unroll
    for (int c = 0; c < kCPT; ++c) {
        const int q = threadIdx.x + c * kThreads;
        if (q < kNCH) {
            const int row = q / kCH, cc = q - row * kCH;
            const u32x4 z = {0u, 0u, 0u, 0u};
            *(u32x4*)(t + row * kLW + 8 * cc) = ((m >> c) & 1u) ? v[c] : z;
        }
    }
}

// Adds the contributions of the staged plane to the accumulator queue
// (output plane zp - dz goes to slot 1 - dz), then stores output plane
// zo = zp - 1, which is complete, and advances the queue.
__device__ __forceinline__ void mf_plane(const _Float16* __restrict__ t, const half8 (&ahi)[3][3],
                                         const half8 (&alo)[3][3], float4v (&acc)[3][4],
                                         _Float16* __restrict__ out, int nx, int ny, int x0, int y0,
                                         int zo, int z0, int z1) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    // Consecutive MFMAs go to the four independent column blocks, so an
    // accumulator is reused only every fourth instruction (latency hidden).
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        half8 bv[4];
        const int row = 16 * wv + (lane & 15) + 1 + dy;
#pragma unroll
        for (int xb = 0; xb < 4; ++xb) bv[xb] = *(const half8*)(t + row * kLW + 16 * xb + 8 * (lane >> 4));
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
            for (int xb = 0; xb < 4; ++xb)
                acc[1 - dz][xb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi[dz + 1][dy + 1], bv[xb],
                                                                         acc[1 - dz][xb], 0, 0, 0);
#pragma unroll
            for (int xb = 0; xb < 4; ++xb)
                acc[1 - dz][xb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(alo[dz + 1][dy + 1], bv[xb],
                                                                         acc[1 - dz][xb], 0, 0, 0);
        }
    }
    const int gy = y0 + 16 * wv + (lane & 15);
    if (zo >= z0 && zo < z1 && gy < ny) {
        _Float16* orow = out + (size_t)zo * nx * ny + (size_t)gy * nx;
#pragma unroll
        for (int xb = 0; xb < 4; ++xb) {
            const int gx = x0 + 16 * xb + 4 * (lane >> 4);
            if (gx < nx) {   // nx % 8 == 0: the four columns are all inside or all outside
                typedef _Float16 half4 __attribute__((ext_vector_type(4)));
                half4 h;
                h[0] = (_Float16)acc[0][xb][0];
                h[1] = (_Float16)acc[0][xb][1];
                h[2] = (_Float16)acc[0][xb][2];
                h[3] = (_Float16)acc[0][xb][3];
                __builtin_nontemporal_store(h, (half4*)(orow + gx));
            }
        }
    }
#pragma unroll
    for (int xb = 0; xb < 4; ++xb) {
        acc[0][xb] = acc[1][xb];
        acc[1][xb] = acc[2][xb];
        acc[2][xb] = float4v{0.f, 0.f, 0.f, 0.f};
    }
}

// D planes in flight: plane zp's registers are refilled with plane zp + D
// as soon as zp is staged.  The march runs in groups of D; a plane past
// zend is a clamped reload of the last plane and emits nothing.
template <int BC, int D>
__global__ __launch_bounds__(kThreads, 2) void zm3d_mfma_kernel(const _Float16* __restrict__ in,
                                                                _Float16* __restrict__ out, int nx,
                                                                int ny, int nz, int zc, int tiles_x,
                                                                int tiles_y, Taps tp) {
    __shared__ __attribute__((aligned(16))) _Float16 tile[2][kLH * kLW];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % tiles_x;
    const int rest = b / tiles_x;
    const int tyi = rest % tiles_y, zci = rest / tiles_y;
    const int x0 = txi * kMX, y0 = tyi * kMY;
    const int z0 = zci * zc, z1 = min(z0 + zc, nz);
    const int lane = threadIdx.x & (kWave - 1);

    // Coefficient operands: lane holds A[m][kb..kb+7], m = lane % 16.
    half8 ahi[3][3], alo[3][3];
    {
        const int m = lane & 15, kb = 8 * (lane >> 4);
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int dx = kb + j - 8 - m;   // selects, not a runtime index into tp
                    const float c = dx == -1 ? tp.c[box3<1>(dz, dy, -1)]
                                  : dx == 0  ? tp.c[box3<1>(dz, dy, 0)]
                                  : dx == 1  ? tp.c[box3<1>(dz, dy, 1)] : 0.f;
                    const _Float16 h = (_Float16)c;
                    ahi[dz + 1][dy + 1][j] = h;
                    alo[dz + 1][dy + 1][j] = (_Float16)(c - (float)h);
                }
    }

    float4v acc[3][4];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int xb = 0; xb < 4; ++xb) acc[s][xb] = float4v{0.f, 0.f, 0.f, 0.f};

    const int zbeg = z0 - 1, zend = z1 + 1;   // planes z0-1 .. z1 feed outputs z0 .. z1-1
    u32x4 v[D][kCPT];
    uint32_t vm[D];
#pragma unroll
    for (int d = 0; d < D; ++d) vm[d] = mf_load<BC>(in, nx, ny, nz, min(zbeg + d, zend - 1), x0, y0, v[d]);
    for (int zb = zbeg; zb < zend; zb += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int zp = zb + d;
            _Float16* t = tile[d & 1];   // D is even: plane parity equals d parity
            mf_stage(t, v[d], vm[d]);
            vm[d] = mf_load<BC>(in, nx, ny, nz, min(zp + D, zend - 1), x0, y0, v[d]);
            __syncthreads();
            mf_plane(t, ahi, alo, acc, out, nx, ny, x0, y0, zp - 1, z0, z1);
        }
    }
}

bool zm3d_mfma_supported(const Geom& g) {
    return g.ndim == 3 && g.shape == kBox && g.r == 1 && g.dtype == 1 && g.nx % 8 == 0;
}

template <int BC>
static hipError_t go(const Geom& g, int zc, const Taps& tp, const void* in, void* out, hipStream_t s) {
    constexpr int D = 2;   // deeper prefetch (4, 6) measured no faster
    static_assert(D % 2 == 0, "the LDS double buffer alternates with the plane parity");
    const int tiles_x = (g.nx + kMX - 1) / kMX, tiles_y = (g.ny + kMY - 1) / kMY;
    const int nchunks = (g.nz + zc - 1) / zc;
    hipLaunchKernelGGL((zm3d_mfma_kernel<BC, D>), dim3(tiles_x * tiles_y * nchunks), dim3(kThreads), 0, s,
                       (const _Float16*)in, (_Float16*)out, g.nx, g.ny, g.nz, zc, tiles_x, tiles_y, tp);
    return hipGetLastError();
}

hipError_t launch_zm3d_mfma(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                            void* out, hipStream_t stream) {
    if (!zm3d_mfma_supported(g)) return hipErrorInvalidValue;
    const int zc = cfg.zchunk > 0 ? cfg.zchunk : g.nz;
    return g.boundary == kPeriodic ? go<kPeriodic>(g, zc, taps, in, out, stream)
                                   : go<kZero>(g, zc, taps, in, out, stream);
}

}  // namespace stk
