// 2D and 3D sweeps with variable coefficients (Section 2.1: a coefficient
// that varies in space is one more array to read):
//   forward    out(x) = sum_k f_k(x)       in(B(x + d_k))
//   transpose  out(y) = sum_k f_k(y - d_k) in(B(y - d_k))
// f_k is the field of the k-th offset of the shape in (dz,dy,dx) order.
//
// A workgroup owns a 64 x 4*RY column of cells and marches z (a 2D grid is
// one plane: the march has no z halo).  Every input
// plane is staged once in LDS with its halo into a ring of 2R+2 tiles (2R+1
// planes in use, one being written, so one barrier per plane suffices); when
// plane zo+R has arrived, output plane zo is formed from the ring and from
// the coefficient fields of plane zo, which are streamed pointwise one plane
// ahead.  The fields have no reuse, so a launch moves (taps + 2) values per
// cell and the kernel is HBM-bound.
#include "internal.h"
#include "zmarch.h"

namespace stk {

namespace {

// Offsets of a shape in (dz,dy,dx) lexicographic order (dz = 0 in 2D).
template <int SHAPE, int R, int NDIM>
struct VcOffsets {
    static constexpr int RZ = NDIM == 3 ? R : 0;
    static constexpr int N = SHAPE == kBox ? (2 * R + 1) * (2 * R + 1) * (2 * RZ + 1) : 1 + 2 * NDIM * R;
    int d[N][3];
    constexpr VcOffsets() : d{} {
        int k = 0;
        for (int dz = -RZ; dz <= RZ; ++dz)
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx)
                    if (SHAPE == kBox || (dz != 0) + (dy != 0) + (dx != 0) <= 1) {
                        d[k][0] = dz;
                        d[k][1] = dy;
                        d[k][2] = dx;
                        ++k;
                    }
    }
};

}  // namespace

template <int R, int SHAPE, typename T, int BC, int RY, int NW, bool ADJ, int NDIM>
__global__ __launch_bounds__(NW * kWave) void vc3d_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                          const T* __restrict__ f, int nx, int ny, int nz,
                                                          int zc, int tiles_x, int tiles_y) {
    using G = PlaneGeom<R, RY, NW>;
    using A = acc_t<T>;
    constexpr VcOffsets<SHAPE, R, NDIM> kOff{};
    constexpr int NTAP = VcOffsets<SHAPE, R, NDIM>::N;
    constexpr int RZ = VcOffsets<SHAPE, R, NDIM>::RZ;   // z reach
    constexpr int NR = 2 * RZ + 2;
    __shared__ A ring[NR][G::H * G::W];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % tiles_x;
    const int rest = b / tiles_x;
    const int tyi = rest % tiles_y, zci = rest / tiles_y;
    const int x0 = txi * G::BX, y0 = tyi * G::BY;
    const int z0 = zci * zc, z1 = min(z0 + zc, nz);
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const int gx = x0 + tx;
    const size_t plane_sz = (size_t)nx * ny;
    const size_t cells = plane_sz * nz;
    const int zbeg = z0 - RZ, zend = z1 + RZ;
    const PlaneIdx<R, RY, NW> pidx = plane_index<R, RY, BC, T, NW>(nx, ny, x0, y0);

    // Coefficients of one output plane, loaded one plane ahead (streamed
    // once, so without keeping them in the caches: 5-9 % faster).  Every
    // address is valid: the plane is clamped to the chunk, forward loads use
    // the interior offsets of pidx (cells past the grid edge are never
    // stored), transposed loads map the shifted cell through the boundary
    // rule (a cell outside a zero frame is clamped; its product vanishes
    // because the staged value there is zero).
    T cv[NTAP][RY];
    auto load_coef = [&](int zo) __attribute__((always_inline)) {
        zo = min(max(zo, z0), z1 - 1);
#pragma unroll
        for (int k = 0; k < NTAP; ++k) {
            const T* fk = f + (size_t)k * cells;
            if constexpr (!ADJ) {
                const char* pl = reinterpret_cast<const char*>(fk + (size_t)zo * plane_sz);
#pragma unroll
                for (int i = 0; i < RY; ++i) cv[k][i] = load_at_nt<T, true>(pl, pidx.off[i]);
            } else {
                int gz = zo - kOff.d[k][0];
                fix_coord<BC>(gz, nz);
                const T* pl = fk + (size_t)gz * plane_sz;
                int sx = gx - kOff.d[k][2];
                fix_coord<BC>(sx, nx);
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    int sy = y0 + ty * RY + i - kOff.d[k][1];
                    fix_coord<BC>(sy, ny);
                    cv[k][i] = pl[(uint32_t)(sy * nx + sx)];
                }
            }
        }
    };

    T vin[RY], vhalo[G::HT];
    uint32_t vm = load_plane_at<R, RY, BC, T, NW, true, true>(in, nx, ny, nz, zbeg, pidx, vin, vhalo);
    load_coef(z0);

    int slot = 0;   // ring slot of plane zp
    for (int zp = zbeg; zp < zend; ++zp) {
        store_plane<R, RY, BC, T, NW>(ring[slot], vin, vhalo, vm);
        // A 2D grid is a single pass with nothing to prefetch.  In 3D the
        // last pass reloads a clamped plane: cheaper than a branch here.
        if constexpr (NDIM == 3)
            vm = load_plane_at<R, RY, BC, T, NW, true, true>(in, nx, ny, nz, min(zp + 1, zend - 1), pidx, vin, vhalo);
        __syncthreads();

        const int zo = zp - RZ;
        if (zo >= z0) {
            // ring slot of plane zo + s (|s| <= RZ): slot - RZ + s, modulo NR
            int sl[2 * RZ + 1];
#pragma unroll
            for (int s = 0; s <= 2 * RZ; ++s) {
                const int v = slot - 2 * RZ + s;
                sl[s] = v < 0 ? v + NR : v;
            }
            A acc[RY];
#pragma unroll
            for (int i = 0; i < RY; ++i) acc[i] = A(0);
#pragma unroll
            for (int k = 0; k < NTAP; ++k) {
                const int sz = ADJ ? -kOff.d[k][0] : kOff.d[k][0];
                const int sy = ADJ ? -kOff.d[k][1] : kOff.d[k][1];
                const int sx = ADJ ? -kOff.d[k][2] : kOff.d[k][2];
                const A* t = ring[sl[RZ + sz]] + (R + ty * RY + sy) * G::W + R + tx + sx;
#pragma unroll
                for (int i = 0; i < RY; ++i) acc[i] = fma_acc(to_acc<T>(cv[k][i]), t[i * G::W], acc[i]);
            }
            if (zo < z1 && gx < nx) {
                T* o = out + (size_t)zo * plane_sz;
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int gy = y0 + ty * RY + i;
                    if (gy < ny) store_at_nt(o, pidx.off[i], from_acc<T>(acc[i]));   // the cell's byte offset
                }
            }
            if constexpr (NDIM == 3) {
                // The box streams 27 fields: issuing them at raised wave
                // priority measured 3 % faster (the 7-point star 2 % slower).
                if constexpr (SHAPE == kBox) __builtin_amdgcn_s_setprio(3);
                load_coef(zo + 1);
                if constexpr (SHAPE == kBox) __builtin_amdgcn_s_setprio(0);
            }
        }
        slot = slot + 1 == NR ? 0 : slot + 1;
    }
}

bool vc3d_supported(int r, int shape) { return shape == kStar ? (r >= 1 && r <= 4) : r == 1; }

template <int R, int SHAPE, typename T, int BC, int RY, bool ADJ>
static hipError_t go(const Geom& g, int zc, const void* in, void* out, const void* fields, hipStream_t s) {
    constexpr int NW = 4;
    using G = PlaneGeom<R, RY, NW>;
    const int tiles_x = (g.nx + G::BX - 1) / G::BX, tiles_y = (g.ny + G::BY - 1) / G::BY;
    const int nchunks = (g.nz + zc - 1) / zc;
    if (g.ndim == 2) {
        hipLaunchKernelGGL((vc3d_kernel<R, SHAPE, T, BC, RY, NW, ADJ, 2>), dim3(tiles_x * tiles_y),
                           dim3(NW * kWave), 0, s, (const T*)in, (T*)out, (const T*)fields, g.nx, g.ny, 1, 1,
                           tiles_x, tiles_y);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((vc3d_kernel<R, SHAPE, T, BC, RY, NW, ADJ, 3>), dim3(tiles_x * tiles_y * nchunks),
                       dim3(NW * kWave), 0, s, (const T*)in, (T*)out, (const T*)fields, g.nx, g.ny, g.nz, zc,
                       tiles_x, tiles_y);
    return hipGetLastError();
}

// tile_y = rows per workgroup: 8 (two rows per thread) or, for stars of
// radius 1, 16 (four rows per thread).
template <int R, int SHAPE, typename T, bool ADJ>
static hipError_t go_ry(const Geom& g, const LaunchCfg& c, const void* in, void* out, const void* fields,
                        hipStream_t s) {
    const int zc = c.zchunk > 0 ? c.zchunk : g.nz;
    if constexpr (SHAPE == kStar && R == 1) {
        if (c.tile_y >= 16)
            return g.boundary == kPeriodic ? go<R, SHAPE, T, kPeriodic, 4, ADJ>(g, zc, in, out, fields, s)
                                           : go<R, SHAPE, T, kZero, 4, ADJ>(g, zc, in, out, fields, s);
    }
    return g.boundary == kPeriodic ? go<R, SHAPE, T, kPeriodic, 2, ADJ>(g, zc, in, out, fields, s)
                                   : go<R, SHAPE, T, kZero, 2, ADJ>(g, zc, in, out, fields, s);
}

template <typename T, bool ADJ>
static hipError_t go_t(const Geom& g, const LaunchCfg& c, const void* in, void* out, const void* fields,
                       hipStream_t s) {
    if (g.shape == kBox) return g.r == 1 ? go_ry<1, kBox, T, ADJ>(g, c, in, out, fields, s) : hipErrorInvalidValue;
    switch (g.r) {
        case 1: return go_ry<1, kStar, T, ADJ>(g, c, in, out, fields, s);
        case 2: return go_ry<2, kStar, T, ADJ>(g, c, in, out, fields, s);
        case 3: return go_ry<3, kStar, T, ADJ>(g, c, in, out, fields, s);
        case 4: return go_ry<4, kStar, T, ADJ>(g, c, in, out, fields, s);
    }
    return hipErrorInvalidValue;
}

// One variable-coefficient step (or its transpose) of a 2D or 3D grid.
hipError_t launch_vc3d(const Geom& g, const LaunchCfg& cfg, const void* in, void* out, const void* fields,
                       bool adjoint, hipStream_t stream) {
    if (!vc3d_supported(g.r, g.shape)) return hipErrorInvalidValue;
    switch (g.dtype) {
        case 0: return adjoint ? go_t<float, true>(g, cfg, in, out, fields, stream)
                               : go_t<float, false>(g, cfg, in, out, fields, stream);
        case 1: return adjoint ? go_t<_Float16, true>(g, cfg, in, out, fields, stream)
                               : go_t<_Float16, false>(g, cfg, in, out, fields, stream);
        case 2: return adjoint ? go_t<double, true>(g, cfg, in, out, fields, stream)
                               : go_t<double, false>(g, cfg, in, out, fields, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace stk
