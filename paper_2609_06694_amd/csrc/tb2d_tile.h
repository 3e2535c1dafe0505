// One output tile of the 2D sweep with k time steps fused in LDS.
//
// The tile of BX x BY outputs is loaded once with a halo of k*R cells on
// every side; each fused step shrinks the valid region by R per side and
// ping-pongs between two LDS buffers, so the k-1 intermediate time levels
// never touch HBM (temporal blocking, Section 4.3: intermediate time planes
// stay on chip).  Arithmetic is FP32; with fp16 storage every intermediate
// level is rounded to binary16 exactly as a one-step-per-launch sweep would
// store it.  Zero boundary: cells outside the grid are forced to zero at
// every level.  Periodic boundary: the halo is loaded with wrapped indices.
//
// NW waves share a tile: lanes take columns, waves take strips of kRY2 rows.
// A 64-column window run by 16 waves covers the whole tile in one pass per
// fused step, which suits small grids, where the sweep is a chain of short
// dependent steps (latency) rather than a stream of bytes.
#pragma once

#include "common.h"

namespace stk {

// Rows each thread computes in one strip; columns map to the 64 lanes.
constexpr int kRY2 = 4;

// LDS floats needed for a tile (two buffers, RY spare rows for strip overrun).
__host__ __device__ inline int tb2d_lds_floats(int BX, int BY, int k, int R) {
    const int W = BX + 2 * k * R, H = BY + 2 * k * R;
    return 2 * W * (H + kRY2);
}

template <int R, int SHAPE>
__device__ __forceinline__ void strip2d(const float* __restrict__ src, int W, int x, int y0,
                                        const Taps& tp, float (&acc)[kRY2]) {
    constexpr int RY = kRY2;
    if constexpr (SHAPE == kBox) {
#pragma unroll
        for (int i = 0; i < RY; ++i) acc[i] = 0.f;
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            float col[RY + 2 * R];
#pragma unroll
            for (int j = 0; j < RY + 2 * R; ++j) col[j] = src[(y0 - R + j) * W + x + dx];
#pragma unroll
            for (int i = 0; i < RY; ++i)
#pragma unroll
                for (int dy = -R; dy <= R; ++dy)
                    acc[i] = fmaf(tp.c[box2<R>(dy, dx)], col[i + R + dy], acc[i]);
        }
    } else {
        float col[RY + 2 * R];
#pragma unroll
        for (int j = 0; j < RY + 2 * R; ++j) col[j] = src[(y0 - R + j) * W + x];
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            float a = tp.c[0] * col[i + R];
#pragma unroll
            for (int d = 1; d <= R; ++d) {
                a = fmaf(tp.c[star_y<R>(-d)], col[i + R - d], a);
                a = fmaf(tp.c[star_y<R>(d)], col[i + R + d], a);
            }
            acc[i] = a;
        }
#pragma unroll
        for (int d = 1; d <= R; ++d) {
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                acc[i] = fmaf(tp.c[star_x<R>(-d)], src[(y0 + i) * W + x - d], acc[i]);
                acc[i] = fmaf(tp.c[star_x<R>(d)], src[(y0 + i) * W + x + d], acc[i]);
            }
        }
    }
}

// Processes the tile whose first output is (gx0, gy0).  `lds` holds
// tb2d_lds_floats(BX, BY, k, R) floats.  Must be called by all NW * 64 threads.
template <int R, int SHAPE, typename T, int BC, int NW = 4>
__device__ void tb2d_tile(const T* __restrict__ in, T* __restrict__ out, int nx, int ny,
                          int gx0, int gy0, int BX, int BY, int k, const Taps& tp,
                          float* __restrict__ lds) {
    constexpr int RY = kRY2;
    const int W = BX + 2 * k * R, H = BY + 2 * k * R;
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    float* b0 = lds;
    float* b1 = lds + W * (H + RY);
    const int ox = gx0 - k * R, oy = gy0 - k * R;
    const bool interior = ox >= 0 && oy >= 0 && ox + W <= nx && oy + H <= ny;

    // Stage the input tile with its k*R halo, four rows per thread at a time:
    // the loads (rows clamped into the tile and the grid, so every address
    // is valid) are all issued before the first LDS store.
    constexpr int SB = 4;
    for (int lx = tx; lx < W; lx += kWave) {
        int gx = ox + lx;
        bool xin = true;
        if (!interior) {
            if (BC == kPeriodic) gx = wrap_index(gx, nx);
            else {
                xin = gx >= 0 && gx < nx;
                gx = min(max(gx, 0), nx - 1);
            }
        }
        for (int ly0 = ty; ly0 < H; ly0 += SB * NW) {
            T v[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                int gy = oy + min(ly0 + u * NW, H - 1);
                if (!interior) gy = BC == kPeriodic ? wrap_index(gy, ny) : min(max(gy, 0), ny - 1);
                v[u] = in[(size_t)gy * nx + gx];
            }
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int ly = ly0 + u * NW;
                if (ly >= H) break;
                const int gy = oy + ly;
                const bool yin = BC == kPeriodic || interior || (gy >= 0 && gy < ny);
                b0[ly * W + lx] = (yin && xin) ? to_f32(v[u]) : 0.f;
            }
        }
    }
    __syncthreads();

    for (int s = 1; s <= k; ++s) {
        const float* src = (s & 1) ? b0 : b1;
        float* dst = (s & 1) ? b1 : b0;
        const int lo = s * R;
        const int yhi = H - lo, xhi = W - lo;
        const bool last = (s == k);
        for (int y0 = lo + ty * RY; y0 < yhi; y0 += NW * RY) {
            for (int x = lo + tx; x < xhi; x += kWave) {
                float acc[RY];
                strip2d<R, SHAPE>(src, W, x, y0, tp, acc);
                const int gx = ox + x;
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int y = y0 + i;
                    if (y >= yhi) break;
                    const int gy = oy + y;
                    if (last) {
                        if (gx < nx && gy < ny) out[(size_t)gy * nx + gx] = from_f32<T>(acc[i]);
                    } else {
                        float v = round_to_storage<T>(acc[i]);
                        if (BC == kZero && (gx < 0 || gx >= nx || gy < 0 || gy >= ny)) v = 0.f;
                        dst[y * W + x] = v;
                    }
                }
            }
        }
        if (!last) __syncthreads();
    }
}

}  // namespace stk
