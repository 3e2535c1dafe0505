// Forward leapfrog with the z-neighbours held in an LDS ring.
//
// L(u) is evaluated in difference form, sum_{d != 0} c_d (u(x+d) - u(x)) plus
// (sum of weights) u(x): the same operator, with far less cancellation error
// than the direct weighted sum for high-order Laplacians.
//
// Each arriving plane is staged once: its halo tile feeds the in-plane (x, y)
// taps and its interior also enters a ring of 2R+2 interior planes in LDS.
// The in-plane partial sum of plane z waits R planes in a short register
// queue; when plane z+R has arrived, the z-taps of output z are read from the
// ring.  Keeping the z-neighbours in LDS instead of a (2R+1)-deep register
// queue of partial sums lowers the per-thread state to the in-plane partials,
// which lets several workgroups share a CU (the plane stream of one
// workgroup alone cannot cover HBM latency and the per-plane barrier).
#include "internal.h"
#include "zmarch.h"

namespace stk {

// PB planes are staged per barrier (1, or 2 = the D planes of one march
// step).  The next group's staging may run while slower waves still read
// the current group, so the halo tiles rotate over 2 PB buffers and the
// ring holds the 2R + PB planes the current group's outputs read plus the
// PB planes the next group writes: 2R+2 slots for PB = 1, 2R+4 for PB = 2.
template <int R, int BC, int RY, int NW, int D, bool ISO, bool LAP = false, bool SP = false, int PB = 1>
__global__ __launch_bounds__(NW * kWave) void wave3d_ring_kernel(WaveLaunch w, int nx, int ny, int nz,
                                                                 int zc, int tiles_x, int tiles_y,
                                                                 Taps tp) {
    static_assert(PB == 1 || PB == D, "one plane, or one march step of D planes, per barrier");
    using G = PlaneGeom<R, RY, NW>;
    constexpr int NR = 2 * R + 2 * PB;     // ring depth (see above)
    constexpr int IP = G::BX * G::BY;      // interior cells per plane
    __shared__ float tile[2 * PB][G::H * G::W];
    __shared__ float ring[NR][IP];
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

    float pq[R + 1][RY];                   // in-plane partials of planes zp-R..zp
    float vin[D][RY], vhalo[D][G::HT];
    uint32_t vm[D];
    float pv[D][RY], kv[D][RY];            // u_{t-1}, kappa of the output plane
    // The source amplitude is read once, up front: a load inside the
    // per-cell branch would make the wave wait for every load in flight.
    const float amp = w.src_x >= 0 ? *w.src_amp : 0.f;
#pragma unroll
    for (int q = 0; q <= R; ++q)
#pragma unroll
        for (int i = 0; i < RY; ++i) pq[q][i] = 0.f;

    // In-plane addressing, the same for every plane of the march.
    const PlaneIdx<R, RY, NW> pidx = plane_index<R, RY, BC, float, NW>(nx, ny, x0, y0);
    // Absorbing layer: the x and y part of the damping at this thread's
    // cells, fixed for the march (the z part is uniform per plane).
    float gxy[RY];
#pragma unroll
    for (int i = 0; i < RY; ++i)
        gxy[i] = SP ? sponge_ramp(gx, nx, w.sp_w, w.sp_s, w.sp_invw) +
                          sponge_ramp(y0 + ty * RY + i, ny, w.sp_w, w.sp_s, w.sp_invw)
                    : 0.f;

    // Unconditional loads (clamped to the chunk; the interior offsets of
    // pidx are valid addresses, and values at cells outside the grid are
    // never used), for the reason given at load_plane.
    auto issue_point = [&](int slot, int zo) {
        const size_t zoff = (size_t)min(max(zo, z0), z1 - 1) * plane_sz;
        const char* pp = reinterpret_cast<const char*>(w.prev + zoff);
        const char* kp = reinterpret_cast<const char*>(w.kappa + zoff);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            pv[slot][i] = load_at_nt<float, true>(pp, pidx.off[i]);
            kv[slot][i] = load_at_nt<float, true>(kp, pidx.off[i]);
        }
    };
#pragma unroll
    for (int d = 0; d < D; ++d) {
        vm[d] = load_plane_at<R, RY, BC, float, NW, true, true>(w.cur, nx, ny, nz, min(zbeg + d, zend - 1), pidx, vin[d], vhalo[d]);
        issue_point(d, zbeg + d - R);
    }

    // Stage plane zp (arrived in slot d of the prefetch) into halo tile t
    // and ring slot sl, then issue the loads of plane zp + D.  The wave
    // issues those loads at raised priority, so they leave before the other
    // waves' arithmetic (1 % faster on the 512^3 radius-4 workload; raising
    // it for the pointwise loads too gained less).
    auto stage = [&](int d, int zp, float* t, int sl) {
        store_plane<R, RY, BC, float, NW>(t, vin[d], vhalo[d], vm[d]);
#pragma unroll
        for (int i = 0; i < RY; ++i) ring[sl][(ty * RY + i) * G::BX + tx] = masked<BC>(vin[d][i], vm[d], i);
        __builtin_amdgcn_s_setprio(3);
        vm[d] = load_plane_at<R, RY, BC, float, NW, true, true>(w.cur, nx, ny, nz, min(zp + D, zend - 1), pidx, vin[d], vhalo[d]);
        __builtin_amdgcn_s_setprio(0);
    };

    int slot = 0;   // ring slot of plane zs
    for (int zs = zbeg; zs < zend; zs += D) {
        // The march runs in whole groups of D planes: up to D-1 planes past
        // zend are clamped loads that emit no output.  (A uniform early exit
        // here would let the compiler assume fewer loads in flight at the
        // loop head and wait for all of them.)
        if constexpr (PB == D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int sl = slot + d >= NR ? slot + d - NR : slot + d;
                stage(d, zs + d, tile[(zs - zbeg + d) & (2 * PB - 1)], sl);
            }
            __syncthreads();
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int zp = zs + d;
            const int sd = slot + d >= NR ? slot + d - NR : slot + d;   // ring slot of plane zp
            float* t = tile[(zp - zbeg) & (2 * PB - 1)];
            if constexpr (PB == 1) {
                stage(d, zp, t, sd);
                __syncthreads();
            }

            float p[RY], uc[RY];
            star_plane_diff<R, RY, ISO, NW>(t, tp, p, uc);
#pragma unroll
            for (int i = 0; i < RY; ++i) pq[R][i] = p[i];

            const int zo = zp - R;
            if (zo >= z0 && zo < z1 && gx < nx) {
                const size_t zoff = (size_t)zo * plane_sz;
                float* np_ = w.next + zoff;
                // ring slots of planes zo-R .. zo+R: slot(zp - 2R + j), j = 0..2R
                int sl[2 * R + 1];
#pragma unroll
                for (int j = 0; j <= 2 * R; ++j) {
                    const int s2 = sd - 2 * R + j;
                    sl[j] = s2 < 0 ? s2 + NR : s2;
                }
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int cell = (ty * RY + i) * G::BX + tx;
                    const float uo = ring[sl[R]][cell];
                    float a = pq[0][i];
#pragma unroll
                    for (int e = 1; e <= R; ++e) {
                        if constexpr (ISO) {
                            a = fmaf(tp.c[star_x<R>(e)], (ring[sl[R - e]][cell] - uo) + (ring[sl[R + e]][cell] - uo), a);
                        } else {
                            a = fmaf(tp.c[star_z<R>(-e)], ring[sl[R - e]][cell] - uo, a);
                            a = fmaf(tp.c[star_z<R>(e)], ring[sl[R + e]][cell] - uo, a);
                        }
                    }
                    a = fmaf(tp.sum, uo, a);
                    const int gy = y0 + ty * RY + i;
                    if (gy >= ny) continue;
                    const uint32_t o = (uint32_t)(gy * nx + gx);
                    // The state update.  With w.exact_update (the gradient's
                    // forward and recompute steps) it is evaluated in FP64 and
                    // rounded once: the misfit gradient is linear in the
                    // small residual P u - d and amplifies the state's error
                    // by about |d| / |r|, and f32 arithmetic would round
                    // 2u - u_prev and then the sum.  The source cell always
                    // takes that path: its large value radiates its rounding.
                    const bool at_src = zo == w.src_z && gy == w.src_y && gx == w.src_x;
                    float v;
                    if constexpr (SP) {
                        // Damped step A (2u + kappa L u) - B u_prev.
                        const float gm = gxy[i] + sponge_ramp(zo, nz, w.sp_w, w.sp_s, w.sp_invw);
                        const float A = __builtin_amdgcn_rcpf(1.f + 0.5f * gm);
                        const float B = (1.f - 0.5f * gm) * A;
                        if (w.exact_update || at_src) {
                            double vd = fma((double)A, fma((double)kv[d][i], (double)a, 2.0 * (double)uo),
                                            -(double)B * (double)pv[d][i]);
                            if (at_src) vd += (double)amp;
                            v = (float)vd;
                        } else {
                            v = fmaf(A, fmaf(kv[d][i], a, 2.f * uo), -B * pv[d][i]);
                        }
                    } else {
                        if (w.exact_update || at_src) {
                            double vd = fma((double)kv[d][i], (double)a, 2.0 * (double)uo - (double)pv[d][i]);
                            if (at_src) vd += (double)amp;
                            v = (float)vd;
                        } else {
                            v = fmaf(kv[d][i], a, 2.f * uo - pv[d][i]);
                        }
                    }
                    if (w.trace_t != nullptr && zo == w.rec_z) w.trace_t[o] = v;
                    // pidx.off[i] is this output cell's byte offset in its plane.
                    if constexpr (LAP) store_at_nt(w.lap_out + zoff, pidx.off[i], a);
                    store_at_nt(np_, pidx.off[i], v);
                }
            }
            issue_point(d, zp + D - R);
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) pq[q][i] = pq[q + 1][i];
        }
        slot = slot + D >= NR ? slot + D - NR : slot + D;
    }
}

bool wave3d_ring_supported(int r) { return r >= 1 && r <= 4; }

template <int R, int BC, int RY, int NW, bool SP, int PB>
static hipError_t go(const Geom& g, int zc, const Taps& tp, const WaveLaunch& w, hipStream_t s) {
    using G = PlaneGeom<R, RY, NW>;
    constexpr int D = 2;
    const int tiles_x = (g.nx + G::BX - 1) / G::BX, tiles_y = (g.ny + G::BY - 1) / G::BY;
    const int nchunks = (g.nz + zc - 1) / zc;
    const dim3 grid(tiles_x * tiles_y * nchunks), block(G::NT);
    if (w.lap_out) {   // also write L(u_t) (gradient recompute)
        if (g.iso)
            hipLaunchKernelGGL((wave3d_ring_kernel<R, BC, RY, NW, D, true, true, SP, PB>), grid, block, 0, s, w,
                               g.nx, g.ny, g.nz, zc, tiles_x, tiles_y, tp);
        else
            hipLaunchKernelGGL((wave3d_ring_kernel<R, BC, RY, NW, D, false, true, SP, PB>), grid, block, 0, s, w,
                               g.nx, g.ny, g.nz, zc, tiles_x, tiles_y, tp);
        return hipGetLastError();
    }
    if (g.iso)
        hipLaunchKernelGGL((wave3d_ring_kernel<R, BC, RY, NW, D, true, false, SP, PB>), grid, block, 0, s, w, g.nx,
                           g.ny, g.nz, zc, tiles_x, tiles_y, tp);
    else
        hipLaunchKernelGGL((wave3d_ring_kernel<R, BC, RY, NW, D, false, false, SP, PB>), grid, block, 0, s, w, g.nx,
                           g.ny, g.nz, zc, tiles_x, tiles_y, tp);
    return hipGetLastError();
}

// cfg.tile_x selects the planes staged per barrier: 2 = the two planes of a
// march step, else one.
template <int R, int BC, int RY, int NW, bool SP>
static hipError_t go_pb(const Geom& g, const LaunchCfg& c, int zc, const Taps& tp, const WaveLaunch& w,
                        hipStream_t s) {
    if (c.tile_x == 2) return go<R, BC, RY, NW, SP, 2>(g, zc, tp, w, s);
    return go<R, BC, RY, NW, SP, 1>(g, zc, tp, w, s);
}

// The absorbing layer is provided with the zero frame only (its damping band
// lines the faces of a bounded domain).
template <int R, int BC, int RY, int NW>
static hipError_t go_sp(const Geom& g, const LaunchCfg& c, int zc, const Taps& tp, const WaveLaunch& w,
                        hipStream_t s) {
    if constexpr (BC == kZero) {
        if (w.sp_w > 0) return go_pb<R, BC, RY, NW, true>(g, c, zc, tp, w, s);
    } else {
        if (w.sp_w > 0) return hipErrorInvalidValue;
    }
    return go_pb<R, BC, RY, NW, false>(g, c, zc, tp, w, s);
}

template <int R, int BC>
static hipError_t go_ry(const Geom& g, const LaunchCfg& c, const Taps& tp, const WaveLaunch& w,
                        hipStream_t s) {
    const int zc = c.zchunk > 0 ? c.zchunk : g.nz;
    // Two rows per thread at every tile height: taller tiles add waves (up
    // to 16, a 1024-thread workgroup) rather than registers, so occupancy
    // stays at four waves per SIMD while the halo share of each plane falls.
    if (c.tile_y >= 32) return go_sp<R, BC, 2, 16>(g, c, zc, tp, w, s);
    if (c.tile_y >= 16) return go_sp<R, BC, 2, 8>(g, c, zc, tp, w, s);
    return go_sp<R, BC, 2, 4>(g, c, zc, tp, w, s);
}

template <int R>
static hipError_t go_bc(const Geom& g, const LaunchCfg& c, const Taps& tp, const WaveLaunch& w,
                        hipStream_t s) {
    return g.boundary == kPeriodic ? go_ry<R, kPeriodic>(g, c, tp, w, s) : go_ry<R, kZero>(g, c, tp, w, s);
}

hipError_t launch_wave3d_ring(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                              const WaveLaunch& w, hipStream_t stream) {
    switch (g.r) {
        case 1: return go_bc<1>(g, cfg, taps, w, stream);
        case 2: return go_bc<2>(g, cfg, taps, w, stream);
        case 3: return go_bc<3>(g, cfg, taps, w, stream);
        case 4: return go_bc<4>(g, cfg, taps, w, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace stk
