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

template <int R, int RY, int NW = 4>
struct PlaneGeom {
    static constexpr int NT = NW * kWave;                      // threads per workgroup
    static constexpr int BX = kWave;
    static constexpr int BY = NW * RY;
    static constexpr int W = BX + 2 * R;
    static constexpr int H = BY + 2 * R;
    static constexpr int NH = W * H - BX * BY;                 // halo cells per plane
    static constexpr int HT = (NH + NT - 1) / NT;              // halo cells per thread
};

// LDS coordinates of halo cell h (0 <= h < NH).
template <int R, int RY, int NW = 4>
__device__ __forceinline__ void halo_coord(int h, int& ly, int& lx) {
    using G = PlaneGeom<R, RY, NW>;
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

// Moves a grid coordinate onto a cell whose address is always valid:
// periodic boundaries wrap; the zero frame clamps into the grid and reports
// whether the cell was inside (an outside cell is loaded from the clamped
// address and zeroed when the value is consumed).
template <int BC>
__device__ __forceinline__ bool fix_coord(int& i, int n) {
    if (BC == kPeriodic) {
        if (n >= kMaxRadius) {
            // Uniform branch.  Needed coordinates lie within R <= n of the
            // grid, so one period suffices; the clamp only keeps cells past
            // every neighbourhood (tile overhang of tiny grids) addressable.
            i = i < 0 ? i + n : (i >= n ? i - n : i);
            i = min(i, n - 1);
        } else {
            i = wrap_index(i, n);
        }
        return true;
    }
    const bool ok = (unsigned)i < (unsigned)n;
    i = min(max(i, 0), n - 1);
    return ok;
}

// A loaded value in its arithmetic type, or zero if mask bit `bit` says its
// cell lies outside the domain (zero frame only).
template <int BC, typename T>
__device__ __forceinline__ acc_t<T> masked(T v, uint32_t m, int bit) {
    const acc_t<T> f = to_acc<T>(v);
    if (BC == kPeriodic) return f;
    return ((m >> bit) & 1u) ? f : acc_t<T>(0);
}

// Issues the loads of one plane of `f` (this thread's RY interior values and
// its halo share) into registers, in storage precision, and returns the
// validity mask (bit i: interior value i, bit RY + j: halo value j).
// Every lane loads from a valid address and no load sits under a branch:
// the compiler can then count the loads still in flight and wait for exactly
// the plane it consumes, so D planes really are in flight at once; a load
// under a divergent branch (or a select right after it) makes it wait for
// every outstanding load instead.
template <int R, int RY, int BC, typename T, int NW = 4>
__device__ __forceinline__ uint32_t load_plane(const T* __restrict__ f, int nx, int ny, int nz, int zp,
                                               int x0, int y0, T (&in)[RY],
                                               T (&halo)[PlaneGeom<R, RY, NW>::HT]) {
    using G = PlaneGeom<R, RY, NW>;
    static_assert(RY + G::HT <= 32, "validity mask holds 32 cells");
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    int gz = zp;
    const bool zin = fix_coord<BC>(gz, nz);
    const T* plane = f + (size_t)gz * nx * ny;
    const bool inner = x0 - R >= 0 && y0 - R >= 0 && x0 + G::BX + R <= nx && y0 + G::BY + R <= ny;
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        int gx = x0 + tx, gy = y0 + ty * RY + i;
        bool ok = zin;
        if (!inner) {
            const bool okx = fix_coord<BC>(gx, nx), oky = fix_coord<BC>(gy, ny);
            ok = ok && okx && oky;
        }
        in[i] = plane[(uint32_t)(gy * nx + gx)];
        m |= (uint32_t)ok << i;
    }
#pragma unroll
    for (int j = 0; j < G::HT; ++j) {
        const int h = threadIdx.x + j * G::NT;
        const bool hv = h < G::NH;   // the last round of halo cells is partial
        int ly, lx;
        halo_coord<R, RY, NW>(hv ? h : 0, ly, lx);
        int gx = x0 - R + lx, gy = y0 - R + ly;
        bool ok = zin && hv;
        if (!inner) {
            const bool okx = fix_coord<BC>(gx, nx), oky = fix_coord<BC>(gy, ny);
            ok = ok && okx && oky;
        }
        halo[j] = plane[(uint32_t)(gy * nx + gx)];
        m |= (uint32_t)ok << (RY + j);
    }
    return m;
}

// The in-plane part of load_plane's addressing, which is the same for every
// plane of a march: byte offsets of this thread's cells within a plane
// (after the boundary rule) and their x/y validity bits.  Computed once per
// workgroup, it leaves one scalar plane base and unconditional loads per plane.
template <int R, int RY, int NW = 4>
struct PlaneIdx {
    uint32_t off[RY + PlaneGeom<R, RY, NW>::HT];
    uint32_t mxy;
};

// sy: element stride of the in-plane second axis (0: nx, a z-march plane).
template <int R, int RY, int BC, typename T, int NW = 4>
__device__ __forceinline__ PlaneIdx<R, RY, NW> plane_index(int nx, int ny, int x0, int y0, int sy = 0) {
    using G = PlaneGeom<R, RY, NW>;
    static_assert(RY + G::HT <= 32, "validity mask holds 32 cells");
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    PlaneIdx<R, RY, NW> pi;
    pi.mxy = 0;
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        int gx = x0 + tx, gy = y0 + ty * RY + i;
        const bool okx = fix_coord<BC>(gx, nx), oky = fix_coord<BC>(gy, ny);
        pi.off[i] = (sy > 0 ? (uint32_t)gy * (uint32_t)sy + (uint32_t)gx : (uint32_t)(gy * nx + gx)) *
                    (uint32_t)sizeof(T);
        pi.mxy |= (uint32_t)(okx && oky) << i;
    }
#pragma unroll
    for (int j = 0; j < G::HT; ++j) {
        const int h = threadIdx.x + j * G::NT;
        const bool hv = h < G::NH;
        int ly, lx;
        halo_coord<R, RY, NW>(hv ? h : 0, ly, lx);
        int gx = x0 - R + lx, gy = y0 - R + ly;
        const bool okx = fix_coord<BC>(gx, nx), oky = fix_coord<BC>(gy, ny);
        pi.off[RY + j] = (sy > 0 ? (uint32_t)gy * (uint32_t)sy + (uint32_t)gx : (uint32_t)(gy * nx + gx)) *
                         (uint32_t)sizeof(T);
        pi.mxy |= (uint32_t)(hv && okx && oky) << (RY + j);
    }
    return pi;
}

// Value at byte offset `off` from a uniform base.  The offset passes through
// an empty asm statement at the point of use so that its zero extension stays
// next to the load (PIN), and with SB the base passes through one that holds
// it in scalar registers as a global pointer: the load then takes the
// scalar-base + 32-bit-offset form instead of a 64-bit address built per lane
// (without SB the compiler still built those inside the wave kernel's march).
// Each pin costs a register copy per load.  Measured on the 512^3 leapfrog:
// 310 -> 335 GCells/s with SB (outputs the same bit for bit); the linear
// z-marches were unchanged and the reverse step 0.6 % slower, so SB is the
// forward leapfrog's.
template <typename T, bool PIN = true, bool SB = false>
__device__ __forceinline__ T load_at(const char* base, uint32_t off) {
    if constexpr (PIN) asm volatile("" : "+v"(off));
    if constexpr (SB) {
        using GP = const __attribute__((address_space(1))) char*;
        GP g = (GP)base;
        asm volatile("" : "+s"(g));
        return *reinterpret_cast<const __attribute__((address_space(1))) T*>(g + off);
    } else {
        return *reinterpret_cast<const T*>(base + off);
    }
}
template <typename T, bool SB = false>
__device__ __forceinline__ T load_at_nt(const char* base, uint32_t off) {
    asm volatile("" : "+v"(off));
    if constexpr (SB) {
        using GP = const __attribute__((address_space(1))) char*;
        GP g = (GP)base;
        asm volatile("" : "+s"(g));
        return __builtin_nontemporal_load(reinterpret_cast<const __attribute__((address_space(1))) T*>(g + off));
    } else {
        return __builtin_nontemporal_load(reinterpret_cast<const T*>(base + off));
    }
}

// Non-temporal store of v at byte offset off from a uniform base, in the
// scalar-base form of load_at<T, true, true>.
template <typename T>
__device__ __forceinline__ void store_at_nt(void* base, uint32_t off, T v) {
    asm volatile("" : "+v"(off));
    using GP = __attribute__((address_space(1))) char*;
    GP g = (GP)base;
    asm volatile("" : "+s"(g));
    __builtin_nontemporal_store(v, reinterpret_cast<__attribute__((address_space(1))) T*>(g + off));
}

// load_plane with the in-plane addressing taken from plane_index; plane zp
// starts zp * sz elements into f (sz = 0: nx * ny, a z-march plane).
template <int R, int RY, int BC, typename T, int NW = 4, bool PIN = true, bool SB = false>
__device__ __forceinline__ uint32_t load_plane_at(const T* __restrict__ f, int nx, int ny, int nz, int zp,
                                                  const PlaneIdx<R, RY, NW>& pi, T (&in)[RY],
                                                  T (&halo)[PlaneGeom<R, RY, NW>::HT], size_t sz = 0) {
    using G = PlaneGeom<R, RY, NW>;
    int gz = zp;
    const bool zin = fix_coord<BC>(gz, nz);
    const char* plane = reinterpret_cast<const char*>(f + (size_t)gz * (sz ? sz : (size_t)nx * ny));
#pragma unroll
    for (int i = 0; i < RY; ++i) in[i] = load_at<T, PIN, SB>(plane, pi.off[i]);
#pragma unroll
    for (int j = 0; j < G::HT; ++j) halo[j] = load_at<T, PIN, SB>(plane, pi.off[RY + j]);
    return zin ? pi.mxy : 0u;
}

// Writes a loaded plane (mask m from load_plane) into an LDS tile of H x W
// floats, multiplying by `scale_in[i]` / `scale_halo[j]` when SCALED (used
// for kappa (.) lambda; the scale is read at the same cells, so the mask of
// the plane also covers it).
template <int R, int RY, int BC, bool SCALED, typename T, int NW = 4, typename A = float>
__device__ __forceinline__ void store_plane(A* __restrict__ tile, const T (&in)[RY],
                                            const T (&halo)[PlaneGeom<R, RY, NW>::HT], uint32_t m,
                                            const A (&scale_in)[RY],
                                            const A (&scale_halo)[PlaneGeom<R, RY, NW>::HT]) {
    using G = PlaneGeom<R, RY, NW>;
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        const A v = masked<BC>(in[i], m, i);
        tile[(R + ty * RY + i) * G::W + R + tx] = SCALED ? v * scale_in[i] : v;
    }
#pragma unroll
    for (int j = 0; j < G::HT; ++j) {
        const int h = threadIdx.x + j * G::NT;
        if (h < G::NH) {
            int ly, lx;
            halo_coord<R, RY, NW>(h, ly, lx);
            const A v = masked<BC>(halo[j], m, RY + j);
            tile[ly * G::W + lx] = SCALED ? v * scale_halo[j] : v;
        }
    }
}

// Unscaled form of store_plane.
template <int R, int RY, int BC, typename T, int NW = 4, typename A = float>
__device__ __forceinline__ void store_plane(A* __restrict__ tile, const T (&in)[RY],
                                            const T (&halo)[PlaneGeom<R, RY, NW>::HT], uint32_t m) {
    const A one[RY] = {};
    const A oneh[PlaneGeom<R, RY, NW>::HT] = {};
    store_plane<R, RY, BC, false, T, NW, A>(tile, in, halo, m, one, oneh);
}

// In-plane arms of a star in difference form, sum over the x and y arms of
// c_d (u(x+d) - u(x)), for this thread's RY rows; u0 receives u(x).  Adding
// (sum of all weights) * u(x) and the z arms later gives L(u) exactly in real
// arithmetic, while each difference of nearby values is formed with little
// rounding: a high-order Laplacian otherwise cancels terms of size ~8|u| to a
// result much smaller than u.
template <int R, int RY, bool ISO, int NW = 4>
__device__ __forceinline__ void star_plane_diff(const float* __restrict__ tile, const Taps& tp,
                                                float (&p)[RY], float (&u0)[RY]) {
    using G = PlaneGeom<R, RY, NW>;
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
template <int R, int RY, int NW = 4>
__device__ __forceinline__ void star_plane_iso(const float* __restrict__ tile, const Taps& tp,
                                               float (&p)[RY]) {
    using G = PlaneGeom<R, RY, NW>;
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
template <int R, int RY, int NW = 4, typename A = float>
__device__ __forceinline__ void star_plane(const A* __restrict__ tile, const Taps& tp, A (&p)[RY]) {
    using G = PlaneGeom<R, RY, NW>;
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const A* base = tile + (ty * RY) * G::W + R + tx;   // row ty*RY - R + R, column tx
    A col[RY + 2 * R];
#pragma unroll
    for (int j = 0; j < RY + 2 * R; ++j) col[j] = base[j * G::W];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        A a = A(tp.c[0]) * col[i + R];
#pragma unroll
        for (int d = 1; d <= R; ++d) {
            a = fma_acc(A(tp.c[star_y<R>(-d)]), col[i + R - d], a);
            a = fma_acc(A(tp.c[star_y<R>(d)]), col[i + R + d], a);
        }
        p[i] = a;
    }
#pragma unroll
    for (int d = 1; d <= R; ++d) {
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            const A* row = tile + (R + ty * RY + i) * G::W + R + tx;
            p[i] = fma_acc(A(tp.c[star_x<R>(-d)]), row[-d], p[i]);
            p[i] = fma_acc(A(tp.c[star_x<R>(d)]), row[d], p[i]);
        }
    }
}

}  // namespace stk
