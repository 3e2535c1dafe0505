// Adjoint and gradient steps of the 3D leapfrog in the LDS-ring design (the
// forward kernel's staging: halo tile for in-plane taps, ring of interior
// planes for z taps).
#include "internal.h"
#include "zmarch.h"

namespace stk {

// Adjoint (MODE = kWaveAdj) and gradient (MODE = kWaveGrad, kWaveGradPt)
// steps in the ring design:
//   adjoint : l_t = 2 l_{t+1} - s * l_{t+2} + L^T(kappa (.) l_{t+1})
//   gradient: the same with s = 1, plus l_t += [z = rec] (u_t - d_t) and
//             g += l_{t+1} (.) L(u_t).
// kWaveGrad stages u_t and applies L itself; kWaveGradPt reads L(u_t) as a
// pointwise field and u_t on the receiver plane from the recorded trace, so
// it stages one field like the adjoint (half the LDS, twice the waves).
// kappa (.) l_{t+1} (and, for the gradient, u_t) is staged once per plane:
// its halo tile gives the in-plane taps and its interior enters an LDS ring
// of 2R+2 planes for the z taps, as in the forward kernel.  The unscaled
// l_{t+1} of the output plane waits R planes in a register queue.  `tp` holds
// L^T (the flipped star), `tp2` holds L.  Both are applied in the forward
// kernel's difference form, sum_{d != 0} c_d (v(x+d) - v(x)) + (sum of
// weights) v(x), so the reverse sweep applies exactly the transpose of the
// operator the forward sweep applies (a direct weighted sum with an f32
// centre weight would differ from it by up to half an ulp of that weight).
//
// With the absorbing layer (SP) the step is u_{t+1} = A (2 u_t + kappa L u_t)
// - B u_{t-1}, and the transposed step becomes
//   l_t = 2 A l_{t+1} + L^T(kappa (.) A l_{t+1}) - B l_{t+2} (+ residual),
//   g  += (A l_{t+1}) (.) L(u_t):
// the staged field is kappa A l_{t+1} (A at every staged cell, halo included).
template <int MODE, int R, int BC, int RY, int NW, int D, bool ISO, bool SP = false>
__global__ __launch_bounds__(NW * kWave, (MODE == kWaveGradPt && NW == 8) ? 4 : 1) void wave3d_ring_adj_kernel(WaveLaunch w, int nx, int ny,
                                                                     int nz, int zc, int tiles_x,
                                                                     int tiles_y, Taps tp, Taps tp2) {
    using G = PlaneGeom<R, RY, NW>;
    constexpr bool TWO = (MODE == kWaveGrad);
    constexpr bool PT = (MODE == kWaveGradPt);
    constexpr bool GRAD = TWO || PT;
    constexpr int NR = 2 * R + 2;
    constexpr int IP = G::BX * G::BY;
    __shared__ float tile[TWO ? 2 : 1][2][G::H * G::W];
    __shared__ float ring[TWO ? 2 : 1][NR][IP];
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

    float pq[R + 1][RY], pq2[TWO ? R + 1 : 1][RY];   // in-plane partials, planes zp-R..zp
    float lq[R + 1][RY];                               // l_{t+1} at this thread's cells
#pragma unroll
    for (int q = 0; q <= R; ++q)
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            pq[q][i] = 0.f;
            lq[q][i] = 0.f;
            if constexpr (TWO) pq2[q][i] = 0.f;
        }
    float vin[D][RY], vhalo[D][G::HT], kin[D][RY], khalo[D][G::HT];
    float uin[TWO ? D : 1][RY], uhalo[TWO ? D : 1][G::HT];
    uint32_t vm[D];
    float p2v[D][RY], gv[GRAD ? D : 1][RY];   // l_{t+2}, g of the output plane
    float luv[PT ? D : 1][RY];                // L(u_t) of the output plane

    // In-plane addressing, the same for every plane and field of the march.
    const PlaneIdx<R, RY, NW> pidx = plane_index<R, RY, BC, float, NW>(nx, ny, x0, y0);
    // Absorbing layer: the x and y part of the damping at this thread's
    // interior and halo cells, fixed for the march.
    float gin[SP ? RY : 1], ghalo[SP ? G::HT : 1];
    if constexpr (SP) {
#pragma unroll
        for (int i = 0; i < RY; ++i)
            gin[i] = sponge_ramp(gx, nx, w.sp_w, w.sp_s, w.sp_invw) +
                     sponge_ramp(y0 + ty * RY + i, ny, w.sp_w, w.sp_s, w.sp_invw);
#pragma unroll
        for (int j = 0; j < G::HT; ++j) {
            const int h = threadIdx.x + j * G::NT;
            int ly, lx;
            halo_coord<R, RY, NW>(h < G::NH ? h : 0, ly, lx);
            ghalo[j] = sponge_ramp(x0 - R + lx, nx, w.sp_w, w.sp_s, w.sp_invw) +
                       sponge_ramp(y0 - R + ly, ny, w.sp_w, w.sp_s, w.sp_invw);
        }
    }
    auto issue_plane = [&](int slot, int zp) __attribute__((always_inline)) {
        zp = min(zp, zend - 1);
        vm[slot] = load_plane_at<R, RY, BC, float, NW>(w.cur, nx, ny, nz, zp, pidx, vin[slot], vhalo[slot]);
        load_plane_at<R, RY, BC, float, NW>(w.kappa, nx, ny, nz, zp, pidx, kin[slot], khalo[slot]);
        if constexpr (TWO) load_plane_at<R, RY, BC, float, NW>(w.u, nx, ny, nz, zp, pidx, uin[slot], uhalo[slot]);
    };
    // The interior offsets of pidx are valid addresses; values at cells
    // outside the grid are never used.
    auto issue_point = [&](int slot, int zo) __attribute__((always_inline)) {
        const size_t zoff = (size_t)min(max(zo, z0), z1 - 1) * plane_sz;
        const char* pp = reinterpret_cast<const char*>(w.prev + zoff);
        const char* gp = reinterpret_cast<const char*>(w.grad + zoff);
        // Without L(u_t) (no gradient term this step) the loads read l_{t+2}
        // instead, a valid address; their values are not used.
        const char* lp = reinterpret_cast<const char*>((PT && w.lap ? w.lap : w.prev) + zoff);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            p2v[slot][i] = load_at_nt<float>(pp, pidx.off[i]);
            if constexpr (GRAD) gv[slot][i] = load_at_nt<float>(gp, pidx.off[i]);
            if constexpr (PT) luv[slot][i] = load_at_nt<float>(lp, pidx.off[i]);
        }
    };
#pragma unroll
    for (int d = 0; d < D; ++d) {
        issue_plane(d, zbeg + d);
        issue_point(d, zbeg + d - R);
    }

    int slot = 0;
    for (int zs = zbeg; zs < zend; zs += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int zp = zs + d;   // planes past zend: clamped loads, no output
            if constexpr (SP) {   // kappa -> kappa A on plane zp
                const float gz = sponge_ramp(zp, nz, w.sp_w, w.sp_s, w.sp_invw);
#pragma unroll
                for (int i = 0; i < RY; ++i) kin[d][i] *= __builtin_amdgcn_rcpf(1.f + 0.5f * (gin[i] + gz));
#pragma unroll
                for (int j = 0; j < G::HT; ++j) khalo[d][j] *= __builtin_amdgcn_rcpf(1.f + 0.5f * (ghalo[j] + gz));
            }
            float* t1 = tile[0][zp & 1];
            store_plane<R, RY, BC, true, float, NW>(t1, vin[d], vhalo[d], vm[d], kin[d], khalo[d]);
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                const float l = masked<BC>(vin[d][i], vm[d], i);
                lq[R][i] = l;
                ring[0][slot][(ty * RY + i) * G::BX + tx] = l * kin[d][i];
            }
            float* t2 = nullptr;
            if constexpr (TWO) {
                t2 = tile[1][zp & 1];
                store_plane<R, RY, BC, float, NW>(t2, uin[d], uhalo[d], vm[d]);
#pragma unroll
                for (int i = 0; i < RY; ++i)
                    ring[1][slot][(ty * RY + i) * G::BX + tx] = masked<BC>(uin[d][i], vm[d], i);
            }
            issue_plane(d, zp + D);
            __syncthreads();

            {
                float p[RY], uc[RY];
                star_plane_diff<R, RY, ISO, NW>(t1, tp, p, uc);
#pragma unroll
                for (int i = 0; i < RY; ++i) pq[R][i] = p[i];
                if constexpr (TWO) {
                    star_plane_diff<R, RY, ISO, NW>(t2, tp2, p, uc);
#pragma unroll
                    for (int i = 0; i < RY; ++i) pq2[R][i] = p[i];
                }
            }

            const int zo = zp - R;
            if (zo >= z0 && zo < z1 && gx < nx) {
                int sl[2 * R + 1];
#pragma unroll
                for (int j = 0; j <= 2 * R; ++j) {
                    const int s2 = slot - 2 * R + j;
                    sl[j] = s2 < 0 ? s2 + NR : s2;
                }
                const size_t zoff = (size_t)zo * plane_sz;
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int cell = (ty * RY + i) * G::BX + tx;
                    const float ko = ring[0][sl[R]][cell];
                    float a = pq[0][i];
#pragma unroll
                    for (int e = 1; e <= R; ++e) {
                        if constexpr (ISO) {
                            a = fmaf(tp.c[star_x<R>(e)], (ring[0][sl[R - e]][cell] - ko) + (ring[0][sl[R + e]][cell] - ko), a);
                        } else {
                            a = fmaf(tp.c[star_z<R>(-e)], ring[0][sl[R - e]][cell] - ko, a);
                            a = fmaf(tp.c[star_z<R>(e)], ring[0][sl[R + e]][cell] - ko, a);
                        }
                    }
                    a = fmaf(tp.sum, ko, a);
                    const int gy = y0 + ty * RY + i;
                    if (gy >= ny) continue;
                    const uint32_t o = (uint32_t)(gy * nx + gx);
                    // Damping of the output cell: l_{t+1} enters as A l_{t+1}
                    // and l_{t+2} as B l_{t+2} (1 and 1 without the layer).
                    float Al = lq[0][i], Bp = p2v[d][i];
                    if constexpr (SP) {
                        const float gm = gin[i] + sponge_ramp(zo, nz, w.sp_w, w.sp_s, w.sp_invw);
                        const float A = __builtin_amdgcn_rcpf(1.f + 0.5f * gm);
                        Al *= A;
                        if (MODE != kWaveAdj || w.prev_damped) Bp *= (1.f - 0.5f * gm) * A;
                    }
                    float v;
                    if constexpr (MODE == kWaveAdj) {
                        v = 2.f * Al - w.prev_sign * Bp + a;
                    } else if constexpr (PT) {
                        v = 2.f * Al - Bp + a;
                        if (w.target_t != nullptr && zo == w.rec_z) v += w.trace_res[o] - w.target_t[o];
                        if (w.lap != nullptr)
                            __builtin_nontemporal_store(fmaf(Al, luv[d][i], gv[d][i]), &w.grad[zoff + o]);
                    } else {
                        const float uo = ring[1][sl[R]][cell];
                        float a2 = pq2[0][i];
#pragma unroll
                        for (int e = 1; e <= R; ++e) {
                            if constexpr (ISO) {
                                a2 = fmaf(tp2.c[star_x<R>(e)], (ring[1][sl[R - e]][cell] - uo) + (ring[1][sl[R + e]][cell] - uo), a2);
                            } else {
                                a2 = fmaf(tp2.c[star_z<R>(-e)], ring[1][sl[R - e]][cell] - uo, a2);
                                a2 = fmaf(tp2.c[star_z<R>(e)], ring[1][sl[R + e]][cell] - uo, a2);
                            }
                        }
                        a2 = fmaf(tp2.sum, uo, a2);
                        v = 2.f * Al - Bp + a;
                        if (w.target_t != nullptr && zo == w.rec_z) v += ring[1][sl[R]][cell] - w.target_t[o];
                        __builtin_nontemporal_store(fmaf(Al, a2, gv[d][i]), &w.grad[zoff + o]);
                    }
                    __builtin_nontemporal_store(v, &w.next[zoff + o]);
                }
            }
            issue_point(d, zp + D - R);
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    pq[q][i] = pq[q + 1][i];
                    lq[q][i] = lq[q + 1][i];
                    if constexpr (TWO) pq2[q][i] = pq2[q + 1][i];
                }
            slot = slot + 1 == NR ? 0 : slot + 1;
        }
    }
}

template <int MODE, int R, int BC, int NW>
static hipError_t go_adj(const Geom& g, int zc, const Taps& tp, const Taps& tp2, const WaveLaunch& w,
                         hipStream_t s) {
    using G = PlaneGeom<R, 2, NW>;
    const int tiles_x = (g.nx + G::BX - 1) / G::BX, tiles_y = (g.ny + G::BY - 1) / G::BY;
    const int nchunks = (g.nz + zc - 1) / zc;
    constexpr int D = MODE == kWaveGradPt ? 1 : 2;   // planes in flight (registers: see the kernel)
    const dim3 grid(tiles_x * tiles_y * nchunks), block(G::NT);
    // The absorbing layer lines the faces of a bounded domain: zero frame only.
    if (w.sp_w > 0) {
        if constexpr (BC == kZero && MODE != kWaveGrad) {
            if (g.iso)
                hipLaunchKernelGGL((wave3d_ring_adj_kernel<MODE, R, BC, 2, NW, D, true, true>), grid, block, 0, s, w,
                                   g.nx, g.ny, g.nz, zc, tiles_x, tiles_y, tp, tp2);
            else
                hipLaunchKernelGGL((wave3d_ring_adj_kernel<MODE, R, BC, 2, NW, D, false, true>), grid, block, 0, s, w,
                                   g.nx, g.ny, g.nz, zc, tiles_x, tiles_y, tp, tp2);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (g.iso)
        hipLaunchKernelGGL((wave3d_ring_adj_kernel<MODE, R, BC, 2, NW, D, true>), grid, block, 0, s, w, g.nx, g.ny,
                           g.nz, zc, tiles_x, tiles_y, tp, tp2);
    else
        hipLaunchKernelGGL((wave3d_ring_adj_kernel<MODE, R, BC, 2, NW, D, false>), grid, block, 0, s, w, g.nx, g.ny,
                           g.nz, zc, tiles_x, tiles_y, tp, tp2);
    return hipGetLastError();
}

template <int MODE, int R, int BC>
static hipError_t go_adj_ty(const Geom& g, const LaunchCfg& c, const Taps& tp, const Taps& tp2,
                            const WaveLaunch& w, hipStream_t s) {
    const int zc = c.zchunk > 0 ? c.zchunk : g.nz;
    // Two staged fields (gradient) need two rings: 32-row tiles would not fit in LDS.
    if constexpr (MODE != kWaveGrad)
        if (c.tile_y >= 32) return go_adj<MODE, R, BC, 16>(g, zc, tp, tp2, w, s);
    if (c.tile_y >= 16) return go_adj<MODE, R, BC, 8>(g, zc, tp, tp2, w, s);
    return go_adj<MODE, R, BC, 4>(g, zc, tp, tp2, w, s);
}

template <int MODE, int R>
static hipError_t go_adj_bc(const Geom& g, const LaunchCfg& c, const Taps& tp, const Taps& tp2,
                            const WaveLaunch& w, hipStream_t s) {
    return g.boundary == kPeriodic ? go_adj_ty<MODE, R, kPeriodic>(g, c, tp, tp2, w, s)
                                   : go_adj_ty<MODE, R, kZero>(g, c, tp, tp2, w, s);
}

template <int MODE>
static hipError_t go_adj_r(const Geom& g, const LaunchCfg& c, const Taps& tp, const Taps& tp2,
                           const WaveLaunch& w, hipStream_t s) {
    switch (g.r) {
        case 1: return go_adj_bc<MODE, 1>(g, c, tp, tp2, w, s);
        case 2: return go_adj_bc<MODE, 2>(g, c, tp, tp2, w, s);
        case 3: return go_adj_bc<MODE, 3>(g, c, tp, tp2, w, s);
        case 4: return go_adj_bc<MODE, 4>(g, c, tp, tp2, w, s);
    }
    return hipErrorInvalidValue;
}

// `taps` is L^T (applied to kappa (.) lambda), `taps_fwd` is L (applied to
// u_t in gradient mode).
hipError_t launch_wave3d_ring_adj(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                                  const Taps& taps_fwd, WaveMode mode, const WaveLaunch& w,
                                  hipStream_t stream) {
    if (mode == kWaveAdj) return go_adj_r<kWaveAdj>(g, cfg, taps, taps_fwd, w, stream);
    if (mode == kWaveGrad) return go_adj_r<kWaveGrad>(g, cfg, taps, taps_fwd, w, stream);
    if (mode == kWaveGradPt) return go_adj_r<kWaveGradPt>(g, cfg, taps, taps_fwd, w, stream);
    return hipErrorInvalidValue;
}

}  // namespace stk
