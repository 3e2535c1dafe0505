// Plane staging shared by the 3D z-march kernels.
//
// A workgroup owns a column of 64 x BY cells (BY = 4*RY) and marches along z.
// Each arriving plane is staged once into LDS with an R-cell halo in x and y;
// contributions of that plane to the 2R+1 output planes it touches are added
// into a register queue of partial sums, so every input plane is read from
// HBM once per workgroup and never re-read for its z-neighbours (register
// reuse along the streaming axis instead of per-update DRAM reads, Section
// 2.1: on-chip reuse is what raises arithmetic intensity).
#pragma once

#include "common.h"

namespace stk {

template <int R, int RY>
struct PlaneGeom {
    static constexpr int BX = kWave;
    static constexpr int BY = 4 * RY;
    static constexpr int W = BX + 2 * R;
    static constexpr int H = BY + 2 * R;
    static constexpr int NH = W * H - BX * BY;                 // halo cells per plane
    static constexpr int HT = (NH + kThreads - 1) / kThreads;  // halo cells per thread
};

// LDS coordinates of halo cell h (0 <= h < NH).
template <int R, int RY>
__device__ __forceinline__ void halo_coord(int h, int& ly, int& lx) {
    using G = PlaneGeom<R, RY>;
    if (h < 2 * R * G::W) {
        const int row = h / G::W;
        lx = h - row * G::W;
        ly = row < R ? row : G::BY + row;   // top R rows, then bottom R rows
    } else {
        const int q = h - 2 * R * G::W;
        const int row = q / (2 * R), c = q - row * (2 * R);
        ly = R + row;
        lx = c < R ? c : G::BX + c;
    }
}

// Maps an unclipped grid coordinate through the boundary rule; false = zero.
template <int BC>
__device__ __forceinline__ bool map_coord(int& i, int n) {
    if (BC == kPeriodic) {
        if (i < 0 || i >= n) i = wrap_index(i, n);
        return true;
    }
    return i >= 0 && i < n;
}

// Loads one plane of `f` (interior RY values and this thread's halo share)
// into registers, converted to f32.  Out-of-domain cells read as zero.  The
// loads are predicated rather than followed by a select: a select would
// consume each value as soon as it is loaded and force a wait right there,
// while predicated loads stay in flight until the plane is staged in LDS.
template <int R, int RY, int BC, typename T>
__device__ __forceinline__ void load_plane(const T* __restrict__ f, int nx, int ny, int nz, int zp,
                                           int x0, int y0, float (&in)[RY],
                                           float (&halo)[PlaneGeom<R, RY>::HT]) {
    using G = PlaneGeom<R, RY>;
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    int gz = zp;
    const bool zin = map_coord<BC>(gz, nz);
    const T* plane = f + (size_t)gz * nx * ny;
    const bool inner = x0 - R >= 0 && y0 - R >= 0 && x0 + G::BX + R <= nx && y0 + G::BY + R <= ny;
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        int gx = x0 + tx, gy = y0 + ty * RY + i;
        bool ok = zin;
        if (!inner) ok = ok && map_coord<BC>(gx, nx) && map_coord<BC>(gy, ny);
        in[i] = ok ? to_f32(plane[(uint32_t)(gy * nx + gx)]) : 0.f;
    }
#pragma unroll
    for (int j = 0; j < G::HT; ++j) {
        const int h = threadIdx.x + j * kThreads;
        float v = 0.f;
        if (h < G::NH) {
            int ly, lx;
            halo_coord<R, RY>(h, ly, lx);
            int gx = x0 - R + lx, gy = y0 - R + ly;
            bool ok = zin;
            if (!inner) ok = ok && map_coord<BC>(gx, nx) && map_coord<BC>(gy, ny);
            if (ok) v = to_f32(plane[(uint32_t)(gy * nx + gx)]);
        }
        halo[j] = v;
    }
}

// Writes a loaded plane into an LDS tile of H x W floats, scaling the values
// by `scale_in[i]` / `scale_halo[j]` when SCALED (used for kappa (.) lambda).
template <int R, int RY, bool SCALED>
__device__ __forceinline__ void store_plane(float* __restrict__ tile, const float (&in)[RY],
                                            const float (&halo)[PlaneGeom<R, RY>::HT],
                                            const float (&scale_in)[RY],
                                            const float (&scale_halo)[PlaneGeom<R, RY>::HT]) {
    using G = PlaneGeom<R, RY>;
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < RY; ++i)
        tile[(R + ty * RY + i) * G::W + R + tx] = SCALED ? in[i] * scale_in[i] : in[i];
#pragma unroll
    for (int j = 0; j < G::HT; ++j) {
        const int h = threadIdx.x + j * kThreads;
        if (h < G::NH) {
            int ly, lx;
            halo_coord<R, RY>(h, ly, lx);
            tile[ly * G::W + lx] = SCALED ? halo[j] * scale_halo[j] : halo[j];
        }
    }
}

// In-plane arms of a star in difference form, sum over the x and y arms of
// c_d (u(x+d) - u(x)), for this thread's RY rows; u0 receives u(x).  Adding
// (sum of all weights) * u(x) and the z arms later gives L(u) exactly in real
// arithmetic, while each difference of nearby values is formed with little
// rounding: a high-order Laplacian otherwise cancels terms of size ~8|u| to a
// result much smaller than u.
template <int R, int RY, bool ISO>
__device__ __forceinline__ void star_plane_diff(const float* __restrict__ tile, const Taps& tp,
                                                float (&p)[RY], float (&u0)[RY]) {
    using G = PlaneGeom<R, RY>;
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const float* base = tile + (ty * RY) * G::W + R + tx;
    float col[RY + 2 * R];
#pragma unroll
    for (int j = 0; j < RY + 2 * R; ++j) col[j] = base[j * G::W];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        const float* row = tile + (R + ty * RY + i) * G::W + R + tx;
        const float c = col[i + R];
        u0[i] = c;
        float a = 0.f;
#pragma unroll
        for (int d = 1; d <= R; ++d) {
            if constexpr (ISO) {
                a = fmaf(tp.c[star_x<R>(d)], ((col[i + R - d] - c) + (col[i + R + d] - c)) +
                                                 ((row[-d] - c) + (row[d] - c)), a);
            } else {
                a = fmaf(tp.c[star_y<R>(-d)], col[i + R - d] - c, a);
                a = fmaf(tp.c[star_y<R>(d)], col[i + R + d] - c, a);
                a = fmaf(tp.c[star_x<R>(-d)], row[-d] - c, a);
                a = fmaf(tp.c[star_x<R>(d)], row[d] - c, a);
            }
        }
        p[i] = a;
    }
}

// In-plane contribution of an isotropic star (one weight per distance, equal
// on every arm): c0 u + sum_d w_d (u(x-d) + u(x+d) + u(y-d) + u(y+d)).
// Taps: c[0] = centre, c[star_x<R>(d)] = w_d.
template <int R, int RY>
__device__ __forceinline__ void star_plane_iso(const float* __restrict__ tile, const Taps& tp,
                                               float (&p)[RY]) {
    using G = PlaneGeom<R, RY>;
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const float* base = tile + (ty * RY) * G::W + R + tx;
    float col[RY + 2 * R];
#pragma unroll
    for (int j = 0; j < RY + 2 * R; ++j) col[j] = base[j * G::W];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        const float* row = tile + (R + ty * RY + i) * G::W + R + tx;
        float a = tp.c[0] * col[i + R];
#pragma unroll
        for (int d = 1; d <= R; ++d)
            a = fmaf(tp.c[star_x<R>(d)], (col[i + R - d] + col[i + R + d]) + (row[-d] + row[d]), a);
        p[i] = a;
    }
}

// In-plane star contribution (centre, x and y arms) for this thread's RY rows.
template <int R, int RY>
__device__ __forceinline__ void star_plane(const float* __restrict__ tile, const Taps& tp,
                                           float (&p)[RY]) {
    using G = PlaneGeom<R, RY>;
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const float* base = tile + (ty * RY) * G::W + R + tx;   // row ty*RY - R + R, column tx
    float col[RY + 2 * R];
#pragma unroll
    for (int j = 0; j < RY + 2 * R; ++j) col[j] = base[j * G::W];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        float a = tp.c[0] * col[i + R];
#pragma unroll
        for (int d = 1; d <= R; ++d) {
            a = fmaf(tp.c[star_y<R>(-d)], col[i + R - d], a);
            a = fmaf(tp.c[star_y<R>(d)], col[i + R + d], a);
        }
        p[i] = a;
    }
#pragma unroll
    for (int d = 1; d <= R; ++d) {
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            const float* row = tile + (R + ty * RY + i) * G::W + R + tx;
            p[i] = fmaf(tp.c[star_x<R>(-d)], row[-d], p[i]);
            p[i] = fmaf(tp.c[star_x<R>(d)], row[d], p[i]);
        }
    }
}

}  // namespace stk
