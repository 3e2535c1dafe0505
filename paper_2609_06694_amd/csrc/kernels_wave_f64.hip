// Forward leapfrog with FP64 storage and arithmetic (the double-precision
// member of the case matrix, Section 7.2.1), fused with the source, the
// receiver plane and the absorbing layer like the f32 kernels (Section 4.3):
//
//   u_{t+1} = 2 u_t - u_{t-1} + kappa (.) L(u_t)                 (plain)
//   u_{t+1} = (2 u_t - (1 - gamma/2) u_{t-1} + kappa (.) L(u_t)) / (1 + gamma/2)
//
// then wavelet[t] added at the source cell.  L is the star of radius R with
// FP64 weights (the built-in Laplacian's exact rationals rounded once to
// binary64, or the caller's weights).  In binary64 the direct weighted sum
// loses about 3 decimal digits to cancellation against 16, so it needs no
// difference form: the z-march of the linear sweep (each plane staged once
// in LDS with its halo, contributions queued over 2R+1 planes) with the
// pointwise update at the output plane.  Eight bytes per value make it the
// 32-byte-per-cell-update member of the family.
#include "internal.h"
#include "zmarch.h"

namespace stk {

// In-plane part of the star (centre, x and y arms) at this thread's RY rows
// of a staged binary64 plane.
template <int R, int RY, int NW>
__device__ __forceinline__ void star_plane_f64(const double* __restrict__ tile, const TapsD& tp,
                                               double (&p)[RY]) {
    using G = PlaneGeom<R, RY, NW>;
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const double* base = tile + (ty * RY) * G::W + R + tx;
    double col[RY + 2 * R];
#pragma unroll
    for (int j = 0; j < RY + 2 * R; ++j) col[j] = base[j * G::W];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        const double* row = tile + (R + ty * RY + i) * G::W + R + tx;
        double a = tp.c[0] * col[i + R];
#pragma unroll
        for (int d = 1; d <= R; ++d) {
            a = fma(tp.c[star_y<R>(-d)], col[i + R - d], a);
            a = fma(tp.c[star_y<R>(d)], col[i + R + d], a);
            a = fma(tp.c[star_x<R>(-d)], row[-d], a);
            a = fma(tp.c[star_x<R>(d)], row[d], a);
        }
        p[i] = a;
    }
}

template <int R, int BC, int RY, int NW, int D, bool SP>
__global__ __launch_bounds__(NW * kWave) void wave3d_f64_kernel(WaveLaunchF64 w, int nx, int ny, int nz, int zc,
                                                                int tiles_x, int tiles_y, TapsD tp) {
    using G = PlaneGeom<R, RY, NW>;
    __shared__ double tile[2][G::H * G::W];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % tiles_x;
    const int rest = b / tiles_x;
    const int tyi = rest % tiles_y, zci = rest / tiles_y;
    const int x0 = txi * G::BX, y0 = tyi * G::BY;
    const int z0 = zci * zc, z1 = min(z0 + zc, nz);
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const int gx = x0 + tx;
    const size_t plane_sz = (size_t)nx * ny;
    const int zbeg = z0 - R, zend = z1 + R;

    constexpr int Q = 2 * R + 1;
    double acc[Q][RY];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < RY; ++i) acc[q][i] = 0.0;

    double vin[D][RY], vhalo[D][G::HT];
    uint32_t vm[D];
    double pv[D][RY], kv[D][RY], uq[R + 1][RY];   // u_{t-1}, kappa of the output plane; u_t queue
#pragma unroll
    for (int q = 0; q <= R; ++q)
#pragma unroll
        for (int i = 0; i < RY; ++i) uq[q][i] = 0.0;
    const double amp = w.src_x >= 0 ? *w.src_amp : 0.0;
    const PlaneIdx<R, RY, NW> pidx = plane_index<R, RY, BC, double, NW>(nx, ny, x0, y0);

    // Pointwise operands of output plane zo, clamped to the chunk (clamped
    // values are never used).
    auto issue_point = [&](int slot, int zo) {
        const size_t zoff = (size_t)min(max(zo, z0), z1 - 1) * plane_sz;
        const char* pp = reinterpret_cast<const char*>(w.prev + zoff);
        const char* kp = reinterpret_cast<const char*>(w.kappa + zoff);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            pv[slot][i] = load_at_nt<double>(pp, pidx.off[i]);
            kv[slot][i] = load_at_nt<double>(kp, pidx.off[i]);
        }
    };
#pragma unroll
    for (int d = 0; d < D; ++d) {
        vm[d] = load_plane_at<R, RY, BC, double, NW>(w.cur, nx, ny, nz, min(zbeg + d, zend - 1), pidx, vin[d],
                                                     vhalo[d]);
        issue_point(d, zbeg + d - R);
    }

    for (int zb = zbeg; zb < zend; zb += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int zp = zb + d;
            // Whole groups of D planes: up to D-1 planes past zend are clamped
            // loads that emit no output.
            double* t = tile[zp & 1];
            store_plane<R, RY, BC, double, NW, double>(t, vin[d], vhalo[d], vm[d]);
            double cen[RY];
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                cen[i] = masked<BC>(vin[d][i], vm[d], i);
                uq[R][i] = cen[i];
            }
            vm[d] = load_plane_at<R, RY, BC, double, NW>(w.cur, nx, ny, nz, min(zp + D, zend - 1), pidx, vin[d],
                                                         vhalo[d]);
            __syncthreads();

            double p[RY];
            star_plane_f64<R, RY, NW>(t, tp, p);
            // Plane zp feeds output zo = zp - e with the weight of offset +e.
#pragma unroll
            for (int i = 0; i < RY; ++i) acc[R][i] += p[i];
#pragma unroll
            for (int e = 1; e <= R; ++e)
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    acc[R - e][i] = fma(tp.c[star_z<R>(e)], cen[i], acc[R - e][i]);
                    acc[R + e][i] = fma(tp.c[star_z<R>(-e)], cen[i], acc[R + e][i]);
                }

            // Output plane zo = zp - R has received all 2R+1 planes.
            const int zo = zp - R;
            if (zo >= z0 && zo < z1 && gx < nx) {
                const size_t zoff = (size_t)zo * plane_sz;
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int gy = y0 + ty * RY + i;
                    if (gy >= ny) continue;
                    const double a = acc[0][i], uo = uq[0][i];
                    double v;
                    if constexpr (SP) {
                        const int idx[3] = {gx, gy, zo};
                        const int n3[3] = {nx, ny, nz};
                        double gm = 0.0;
#pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            const int e = min(idx[ax], n3[ax] - 1 - idx[ax]);
                            if (e < w.sp_w) {
                                const double q = (double)(w.sp_w - e) / (double)w.sp_w;
                                gm += w.sp_s * q * q;
                            }
                        }
                        v = (2.0 * uo - (1.0 - 0.5 * gm) * pv[d][i] + kv[d][i] * a) / (1.0 + 0.5 * gm);
                    } else {
                        v = 2.0 * uo - pv[d][i] + kv[d][i] * a;
                    }
                    if (zo == w.src_z && gy == w.src_y && gx == w.src_x) v += amp;
                    if (w.trace_t != nullptr && zo == w.rec_z) w.trace_t[(uint32_t)(gy * nx + gx)] = v;
                    double* np_ = w.next + zoff;
                    __builtin_nontemporal_store(v, reinterpret_cast<double*>(reinterpret_cast<char*>(np_) + pidx.off[i]));
                }
            }
            issue_point(d, zp + D - R);
#pragma unroll
            for (int q = 0; q < Q - 1; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) acc[q][i] = acc[q + 1][i];
#pragma unroll
            for (int i = 0; i < RY; ++i) acc[Q - 1][i] = 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) uq[q][i] = uq[q + 1][i];
        }
    }
}

// Two planes in flight, two rows per thread; 64 x 8 tiles of four waves or
// 64 x 16 of eight (the same registers per thread, a smaller halo share).
template <int R, int BC, int NW, bool SP>
static hipError_t go(const Geom& g, int zc, const TapsD& tp, const WaveLaunchF64& w, hipStream_t s) {
    constexpr int RY = 2, D = 2;
    using G = PlaneGeom<R, RY, NW>;
    const int tiles_x = (g.nx + G::BX - 1) / G::BX, tiles_y = (g.ny + G::BY - 1) / G::BY;
    const int nchunks = (g.nz + zc - 1) / zc;
    hipLaunchKernelGGL((wave3d_f64_kernel<R, BC, RY, NW, D, SP>), dim3(tiles_x * tiles_y * nchunks), dim3(G::NT),
                       0, s, w, g.nx, g.ny, g.nz, zc, tiles_x, tiles_y, tp);
    return hipGetLastError();
}

template <int R, int BC>
static hipError_t go_ry(const Geom& g, const LaunchCfg& c, const TapsD& tp, const WaveLaunchF64& w,
                        hipStream_t s) {
    const int zc = c.zchunk > 0 ? c.zchunk : g.nz;
    if constexpr (BC == kZero) {
        if (w.sp_w > 0)
            return c.tile_y >= 16 ? go<R, BC, 8, true>(g, zc, tp, w, s) : go<R, BC, 4, true>(g, zc, tp, w, s);
    } else {
        if (w.sp_w > 0) return hipErrorInvalidValue;   // the layer lines a zero frame only
    }
    return c.tile_y >= 16 ? go<R, BC, 8, false>(g, zc, tp, w, s) : go<R, BC, 4, false>(g, zc, tp, w, s);
}

template <int R>
static hipError_t go_bc(const Geom& g, const LaunchCfg& c, const TapsD& tp, const WaveLaunchF64& w,
                        hipStream_t s) {
    return g.boundary == kPeriodic ? go_ry<R, kPeriodic>(g, c, tp, w, s) : go_ry<R, kZero>(g, c, tp, w, s);
}

hipError_t launch_wave3d_f64(const Geom& g, const LaunchCfg& cfg, const TapsD& taps, const WaveLaunchF64& w,
                             hipStream_t stream) {
    switch (g.r) {
        case 1: return go_bc<1>(g, cfg, taps, w, stream);
        case 2: return go_bc<2>(g, cfg, taps, w, stream);
        case 3: return go_bc<3>(g, cfg, taps, w, stream);
        case 4: return go_bc<4>(g, cfg, taps, w, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace stk
