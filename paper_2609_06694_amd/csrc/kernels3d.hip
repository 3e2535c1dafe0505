// 3D linear sweep (star r = 1..4, box r = 1..2): plane-streaming z-march.
//
// The same kernel marches the y axis for slabs with few z planes (variant
// ST_VARIANT_YM3D, boxes): the host passes the grid as (x, z, y) with the
// strides of that order (in-plane second axis z: stride nx*ny; march axis
// y: stride nx) and the weights with dz and dy exchanged.  A march of 8
// planes re-reads 2R halo planes and computes partial sums for 2R output
// planes outside its chunk; marching the long axis instead keeps both
// below 2 % for a 4096 x 4096 x 8 slab.
#include "internal.h"
#include "zmarch.h"

namespace stk {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// D planes are kept in flight per workgroup: the register slot of plane zp
// is refilled with plane zp + D as soon as zp has been staged in LDS.
template <int R, int SHAPE, typename T, int BC, int RY, int NW, int D>
__global__ __launch_bounds__(NW * kWave) void zm3d_kernel(const T* __restrict__ in,
                                                          T* __restrict__ out, int nx, int ny,
                                                          int nz, int zc, int tiles_x, int tiles_y,
                                                          Taps tp, int sy, size_t sz) {
    using G = PlaneGeom<R, RY, NW>;
    using A = acc_t<T>;   // arithmetic type (f64 for f64 storage, else f32)
    __shared__ A tile[2][G::H * G::W];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % tiles_x;
    const int rest = b / tiles_x;
    const int tyi = rest % tiles_y, zci = rest / tiles_y;
    const int x0 = txi * G::BX, y0 = tyi * G::BY;
    const int z0 = zci * zc, z1 = min(z0 + zc, nz);
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const int gx = x0 + tx;
    const int zbeg = z0 - R, zend = z1 + R;

    constexpr int Q = 2 * R + 1;
    A acc[Q][RY];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < RY; ++i) acc[q][i] = A(0);

    // The 125 weights of the radius-2 box do not fit in scalar registers (the
    // compiler would park them in vector lanes and read each one back before
    // use).  They are kept in LDS instead, grouped by dx and padded to whole
    // 4-vectors, and read back as uniform vectors once per plane; the first
    // barrier of the march publishes them.
    constexpr bool kLdsTaps = SHAPE == kBox && R >= 2;
    constexpr int kPerDx = (Q * Q + 3) / 4 * 4;
    __shared__ f32x4 ctab[kLdsTaps ? Q * kPerDx / 4 : 1];
    if constexpr (kLdsTaps) {
        float* cf = reinterpret_cast<float*>(ctab);
        for (int i = threadIdx.x; i < Q * kPerDx; i += NW * kWave) {
            const int dxi = i / kPerDx, j = i % kPerDx;   // j = (dz+R)*Q + (dy+R)
            cf[i] = j < Q * Q ? tp.c[j * Q + dxi] : 0.f;
        }
    }

    // In-flight planes stay in storage precision until staged.  Plane
    // indices past the end of the march are clamped to its last plane (a
    // cache hit), keeping every load unconditional.
    T vin[D][RY], vhalo[D][G::HT];
    uint32_t vm[D];
    // Strides: sy of the in-plane second axis, sz of the march axis (0 for
    // the z-march's nx and nx * ny).
    const PlaneIdx<R, RY, NW> pidx = plane_index<R, RY, BC, T, NW>(nx, ny, x0, y0, sy);
#pragma unroll
    for (int d = 0; d < D; ++d)
        vm[d] = load_plane_at<R, RY, BC, T, NW>(in, nx, ny, nz, min(zbeg + d, zend - 1), pidx, vin[d], vhalo[d], sz);

    for (int zb = zbeg; zb < zend; zb += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int zp = zb + d;
            // The march runs in whole groups of D planes: up to D-1 planes
            // past zend are clamped loads that emit no output.  (A uniform
            // early exit here would let the compiler assume fewer loads in
            // flight at the loop head and wait for all of them.)
            A* t = tile[zp & 1];
            store_plane<R, RY, BC, T, NW>(t, vin[d], vhalo[d], vm[d]);
            A cen[RY];
#pragma unroll
            for (int i = 0; i < RY; ++i) cen[i] = masked<BC>(vin[d][i], vm[d], i);
            vm[d] = load_plane_at<R, RY, BC, T, NW>(in, nx, ny, nz, min(zp + D, zend - 1), pidx, vin[d], vhalo[d], sz);
            __syncthreads();

            if constexpr (SHAPE == kStar) {
                A p[RY];
                star_plane<R, RY, NW>(t, tp, p);
                // plane zp feeds output zo = zp - dz with weight c_z(dz); slot R - dz
#pragma unroll
                for (int i = 0; i < RY; ++i) acc[R][i] += p[i];
#pragma unroll
                for (int e = 1; e <= R; ++e) {
#pragma unroll
                    for (int i = 0; i < RY; ++i) {
                        acc[R - e][i] = fma_acc(A(tp.c[star_z<R>(e)]), cen[i], acc[R - e][i]);
                        acc[R + e][i] = fma_acc(A(tp.c[star_z<R>(-e)]), cen[i], acc[R + e][i]);
                    }
                }
            } else if constexpr (kLdsTaps) {
                // An offset the compiler cannot see through keeps the weight
                // reads inside the march (hoisted, they would need 125
                // registers).
                int cb = 0;
                asm volatile("" : "+v"(cb));
#pragma unroll
                for (int dx = -R; dx <= R; ++dx) {
                    A col[RY + 2 * R];
                    const A* base = t + (ty * RY) * G::W + R + tx + dx;
#pragma unroll
                    for (int j = 0; j < RY + 2 * R; ++j) col[j] = base[j * G::W];
                    A w[kPerDx];
#pragma unroll
                    for (int v = 0; v < kPerDx / 4; ++v) {
                        const f32x4 q = ctab[cb + (dx + R) * (kPerDx / 4) + v];
                        w[4 * v] = q.x;
                        w[4 * v + 1] = q.y;
                        w[4 * v + 2] = q.z;
                        w[4 * v + 3] = q.w;
                    }
#pragma unroll
                    for (int dz = -R; dz <= R; ++dz)
#pragma unroll
                        for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                            for (int i = 0; i < RY; ++i)
                                acc[R - dz][i] = fma_acc(w[(dz + R) * Q + dy + R], col[i + R + dy], acc[R - dz][i]);
                    // One dx group at a time: the scheduler would otherwise
                    // issue all weight reads of the plane at once.
                    __builtin_amdgcn_sched_barrier(0);
                }
                // Pin the sums here: the compiler would otherwise sink the
                // multiply-adds past the store branches, away from the weight
                // reads, leaving every weight live at once.
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int i = 0; i < RY; ++i) asm volatile("" : "+v"(acc[q][i]));
            } else {
#pragma unroll
                for (int dx = -R; dx <= R; ++dx) {
                    A col[RY + 2 * R];
                    const A* base = t + (ty * RY) * G::W + R + tx + dx;
#pragma unroll
                    for (int j = 0; j < RY + 2 * R; ++j) col[j] = base[j * G::W];
#pragma unroll
                    for (int dz = -R; dz <= R; ++dz)
#pragma unroll
                        for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                            for (int i = 0; i < RY; ++i)
                                acc[R - dz][i] = fma_acc(A(tp.c[box3<R>(dz, dy, dx)]), col[i + R + dy],
                                                      acc[R - dz][i]);
                }
            }

            // Output plane zp - R has received all 2R+1 planes.
            const int zo = zp - R;
            if (zo >= z0 && zo < z1 && gx < nx) {
                T* o = out + (size_t)zo * (sz ? sz : (size_t)nx * ny);
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int gy = y0 + ty * RY + i;
                    const uint32_t oi = sy > 0 ? (uint32_t)gy * (uint32_t)sy + (uint32_t)gx : (uint32_t)(gy * nx + gx);
                    if (gy < ny) __builtin_nontemporal_store(from_acc<T>(acc[0][i]), &o[oi]);
                }
            }
#pragma unroll
            for (int q = 0; q < Q - 1; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) acc[q][i] = acc[q + 1][i];
#pragma unroll
            for (int i = 0; i < RY; ++i) acc[Q - 1][i] = 0.f;
        }
    }
}

bool zm3d_supported(int r, int shape) {
    if (shape == kStar) return r >= 1 && r <= 4;
    return r >= 1 && r <= 2;
}

int zm3d_rows(const LaunchCfg& cfg) { return cfg.tile_y >= 32 ? 32 : (cfg.tile_y >= 16 ? 16 : 8); }

// Planes in flight per workgroup, chosen so the register ring stays within
// the budget of three to four waves per SIMD.
template <int R, int RY>
constexpr int zm3d_depth() {
    return RY >= 8 ? 1 : (RY >= 4 ? 2 : (R >= 3 ? 3 : 4));
}

// g.sy / g.sz: strides of a y-march view (0 for the z-march).
template <int R, int SHAPE, typename T, int BC, int RY, int NW>
static hipError_t go(const Geom& g, int zc, const Taps& tp, const void* in, void* out,
                     hipStream_t s) {
    using G = PlaneGeom<R, RY, NW>;
    const int tiles_x = (g.nx + G::BX - 1) / G::BX, tiles_y = (g.ny + G::BY - 1) / G::BY;
    const int nchunks = (g.nz + zc - 1) / zc;
    constexpr int D = zm3d_depth<R, RY>();
    hipLaunchKernelGGL((zm3d_kernel<R, SHAPE, T, BC, RY, NW, D>), dim3(tiles_x * tiles_y * nchunks),
                       dim3(G::NT), 0, s, (const T*)in, (T*)out, g.nx, g.ny, g.nz, zc, tiles_x,
                       tiles_y, tp, g.sy, g.sz);
    return hipGetLastError();
}

template <int R, int SHAPE, typename T, int BC>
static hipError_t go_ry(const Geom& g, const LaunchCfg& c, const Taps& tp, const void* in,
                        void* out, hipStream_t s) {
    const int zc = c.zchunk > 0 ? c.zchunk : g.nz;
    if constexpr (sizeof(T) == 8) {
        // f64: partial sums and tiles take twice the registers and LDS; 8- and
        // 16-row tiles only.
        if (zm3d_rows(c) == 8) return go<R, SHAPE, T, BC, 2, 4>(g, zc, tp, in, out, s);
        return go<R, SHAPE, T, BC, 4, 4>(g, zc, tp, in, out, s);
    } else {
        switch (zm3d_rows(c)) {
            case 8: return go<R, SHAPE, T, BC, 2, 4>(g, zc, tp, in, out, s);
            case 16: return go<R, SHAPE, T, BC, 4, 4>(g, zc, tp, in, out, s);
            default: return go<R, SHAPE, T, BC, 8, 4>(g, zc, tp, in, out, s);
        }
    }
}

template <int R, int SHAPE, typename T>
static hipError_t go_bc(const Geom& g, const LaunchCfg& c, const Taps& tp, const void* in,
                        void* out, hipStream_t s) {
    return g.boundary == kPeriodic ? go_ry<R, SHAPE, T, kPeriodic>(g, c, tp, in, out, s)
                                   : go_ry<R, SHAPE, T, kZero>(g, c, tp, in, out, s);
}

template <typename T>
static hipError_t go_t(const Geom& g, const LaunchCfg& c, const Taps& tp, const void* in,
                       void* out, hipStream_t s) {
    if (g.shape == kBox) {
        if (g.r == 1) return go_bc<1, kBox, T>(g, c, tp, in, out, s);
        if (g.r == 2) return go_bc<2, kBox, T>(g, c, tp, in, out, s);
        return hipErrorInvalidValue;
    }
    switch (g.r) {
        case 1: return go_bc<1, kStar, T>(g, c, tp, in, out, s);
        case 2: return go_bc<2, kStar, T>(g, c, tp, in, out, s);
        case 3: return go_bc<3, kStar, T>(g, c, tp, in, out, s);
        case 4: return go_bc<4, kStar, T>(g, c, tp, in, out, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_zm3d(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                       void* out, hipStream_t stream) {
    if (g.dtype == 0) return go_t<float>(g, cfg, taps, in, out, stream);
    if (g.dtype == 2) return go_t<double>(g, cfg, taps, in, out, stream);
    return go_t<_Float16>(g, cfg, taps, in, out, stream);
}

bool ym3d_supported(const Geom& g) {
    const size_t esz = g.dtype == 1 ? 2 : (g.dtype == 2 ? 8 : 4);
    return g.ndim == 3 && g.shape == kBox && (g.r == 1 || g.r == 2) &&
           (size_t)g.nx * g.ny * g.nz * esz <= 0xFFFFFFFFull;
}

// The march along y: the z-march kernel on the (x, z, y) view of the grid,
// with the weights' dz and dy exchanged.  cfg.tile_y: z rows per workgroup;
// cfg.zchunk: y rows per march chunk.
hipError_t launch_ym3d(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in, void* out,
                       hipStream_t stream) {
    if (!ym3d_supported(g)) return hipErrorInvalidValue;
    Geom v = g;
    v.ny = g.nz;
    v.nz = g.ny;
    v.sy = g.nx * g.ny;
    v.sz = (size_t)g.nx;
    Taps t = taps;
    const int w = 2 * g.r + 1;
    for (int a = 0; a < w; ++a)        // dz + r
        for (int b = 0; b < w; ++b)    // dy + r
            for (int c = 0; c < w; ++c) t.c[(b * w + a) * w + c] = taps.c[(a * w + b) * w + c];
    return launch_zm3d(v, cfg, t, in, out, stream);
}

}  // namespace stk
