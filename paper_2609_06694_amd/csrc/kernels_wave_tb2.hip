// Two leapfrog steps per launch for the 3D acoustic wave (temporal blocking).
//
// Several time steps fused into one launch keep the intermediate time level
// on chip (Section 4.3, the temporal-blocking family), so a launch reads
// u_{t-1}, u_t and kappa once and writes u_{t+1} and u_{t+2}: about 10 B of
// HBM traffic per cell-update instead of 16.  A workgroup marches along z:
//  stage A computes u_{t+1} on its output tile plus an R-cell halo in x and y
//          (the single-step plane machinery on the extended tile), writes the
//          tile's own cells to HBM and stages the extended plane in LDS;
//  stage B applies the stencil to those staged planes and emits u_{t+2} on
//          the output tile, R planes behind stage A.
// Output tiles are (64 - 2R) x 4*RYB cells; the halo cells of stage A are
// recomputed by neighbouring workgroups instead of exchanged.
#include "internal.h"
#include "zmarch.h"

namespace stk {

template <int R, int BC, int RYB, int D>
__global__ __launch_bounds__(kThreads, 2) void wave3d_tb2_kernel(WaveTB2 w, int nx, int ny, int nz,
                                                              int zc, int tiles_x, int tiles_y,
                                                              Taps tp) {
    constexpr int RYA = RYB + R / 2;       // stage-A rows per wave (extended tile)
    using GA = PlaneGeom<R, RYA>;          // extended tile 64 x EY plus an R halo
    constexpr int EY = GA::BY;             // extended rows = BY + 2R
    constexpr int BY = 4 * RYB;            // output rows
    constexpr int OX = kWave - 2 * R;      // output columns
    static_assert(EY == BY + 2 * R, "stage A must cover the output tile plus R rows");
    __shared__ float tA[2][GA::H * GA::W];
    __shared__ float tB[2][EY * kWave];

    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % tiles_x;
    const int rest = b / tiles_x;
    const int tyi = rest % tiles_y, zci = rest / tiles_y;
    const int ex0 = txi * OX - R, ey0 = tyi * BY - R;   // extended-tile origin
    const int z0 = zci * zc, z1 = min(z0 + zc, nz);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
    const size_t plane_sz = (size_t)nx * ny;
    const int zbeg = z0 - 2 * R, zend = z1 + 2 * R;     // u_t planes staged
    constexpr int Q = 2 * R + 1;

    // Stage-A cells of this thread: column ex0+lane, rows ey0 + wv*RYA + i.
    // Stage-B cells: column ex0+lane (output if R <= lane < R+OX), rows
    // ey0 + R + wv*RYB + i.
    const int gxe = ex0 + lane;
    const bool lane_out = lane >= R && lane < R + OX && gxe < nx;

    float accA[Q][RYA], cqA[R + 1][RYA];
    float accB[Q][RYB], cqB[R + 1][RYB];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int i = 0; i < RYA; ++i) accA[q][i] = 0.f;
#pragma unroll
        for (int i = 0; i < RYB; ++i) accB[q][i] = 0.f;
    }
#pragma unroll
    for (int q = 0; q <= R; ++q) {
#pragma unroll
        for (int i = 0; i < RYA; ++i) cqA[q][i] = 0.f;
#pragma unroll
        for (int i = 0; i < RYB; ++i) cqB[q][i] = 0.f;
    }

    float vin[D][RYA], vhalo[D][GA::HT];
    uint32_t vm[D];
    float pA[D][RYA], kA[D][RYA];    // u_{t-1}, kappa at stage-A cells of plane za
    float uB[D][RYB], kB[D][RYB];    // u_t, kappa at stage-B cells of plane zb

    // Stage-A pointwise operands of plane za (boundary-mapped).
    auto issue_a = [&](int slot, int za) {
        if (za < z0 - R || za >= z1 + R) return;
        int gz = za;
        if (!map_coord<BC>(gz, nz)) return;
        const size_t zoff = (size_t)gz * plane_sz;
#pragma unroll
        for (int i = 0; i < RYA; ++i) {
            int gx = gxe, gy = ey0 + wv * RYA + i;
            const bool ok = map_coord<BC>(gx, nx) && map_coord<BC>(gy, ny);
            const uint32_t o = ok ? (uint32_t)(gy * nx + gx) : 0u;
            pA[slot][i] = __builtin_nontemporal_load(&w.prev[zoff + o]);
            kA[slot][i] = w.kappa[zoff + o];
        }
    };
    // Stage-B pointwise operands of output plane zb.
    auto issue_b = [&](int slot, int zb) {
        if (zb < z0 || zb >= z1 || !lane_out) return;
        const size_t zoff = (size_t)zb * plane_sz;
#pragma unroll
        for (int i = 0; i < RYB; ++i) {
            const int gy = ey0 + R + wv * RYB + i;
            const uint32_t o = (uint32_t)((gy < ny ? gy : 0) * nx + gxe);
            uB[slot][i] = w.cur[zoff + o];
            kB[slot][i] = w.kappa[zoff + o];
        }
    };

#pragma unroll
    for (int d = 0; d < D; ++d) {
        vm[d] = load_plane<R, RYA, BC>(w.cur, nx, ny, nz, min(zbeg + d, zend - 1), ex0, ey0, vin[d], vhalo[d]);
        issue_a(d, zbeg + d - R);
        issue_b(d, zbeg + d - 2 * R);
    }

    for (int zs = zbeg; zs < zend; zs += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int zp = zs + d;
            if (zp >= zend) break;
            // ---- stage A: accumulate u_t plane zp into u_{t+1} partial sums
            float* ta = tA[zp & 1];
            store_plane<R, RYA, BC>(ta, vin[d], vhalo[d], vm[d]);
            float cen[RYA];
#pragma unroll
            for (int i = 0; i < RYA; ++i) {
                cen[i] = masked<BC>(vin[d][i], vm[d], i);
                cqA[R][i] = cen[i];
            }
            vm[d] = load_plane<R, RYA, BC>(w.cur, nx, ny, nz, min(zp + D, zend - 1), ex0, ey0, vin[d], vhalo[d]);
            __syncthreads();
            {
                float p[RYA];
                star_plane<R, RYA>(ta, tp, p);
#pragma unroll
                for (int i = 0; i < RYA; ++i) accA[R][i] += p[i];
#pragma unroll
                for (int e = 1; e <= R; ++e)
#pragma unroll
                    for (int i = 0; i < RYA; ++i) {
                        accA[R - e][i] = fmaf(tp.c[star_z<R>(e)], cen[i], accA[R - e][i]);
                        accA[R + e][i] = fmaf(tp.c[star_z<R>(-e)], cen[i], accA[R + e][i]);
                    }
            }
            // ---- stage A emission: u_{t+1} on the extended plane za
            const int za = zp - R;
            const bool a_live = za >= z0 - R;
            float* tb = tB[za & 1];
            if (a_live) {
                int gz = za;
                const bool zin = map_coord<BC>(gz, nz);
#pragma unroll
                for (int i = 0; i < RYA; ++i) {
                    const int row = wv * RYA + i;
                    int gx = gxe, gy = ey0 + row;
                    const bool in = zin && map_coord<BC>(gx, nx) && map_coord<BC>(gy, ny);
                    float v = 2.f * cqA[0][i] - pA[d][i] + kA[d][i] * accA[0][i];
                    if (in && gz == w.src_z && gy == w.src_y && gx == w.src_x) v += *w.amp1;
                    if (!in) v = 0.f;   // zero boundary (periodic cells are always in)
                    tb[row * kWave + lane] = v;
                    if (za >= z0 && za < z1 && lane_out && row >= R && row < R + BY && gy < ny &&
                        ey0 + row == gy) {
                        const uint32_t o = (uint32_t)(gy * nx + gxe);
                        __builtin_nontemporal_store(v, &w.out1[(size_t)za * plane_sz + o]);
                        if (w.trace1 != nullptr && za == w.rec_z) w.trace1[o] = v;
                    }
                }
            }
            issue_a(d, zp + D - R);
#pragma unroll
            for (int q = 0; q < Q - 1; ++q)
#pragma unroll
                for (int i = 0; i < RYA; ++i) accA[q][i] = accA[q + 1][i];
#pragma unroll
            for (int i = 0; i < RYA; ++i) accA[Q - 1][i] = 0.f;
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int i = 0; i < RYA; ++i) cqA[q][i] = cqA[q + 1][i];
            __syncthreads();

            // ---- stage B: accumulate u_{t+1} plane za into u_{t+2} partial sums
            if (a_live) {
                float pb[RYB], cb[RYB];
                {
                    const float* base = tb + (wv * RYB) * kWave + lane;   // row wv*RYB (= R + wv*RYB - R)
                    float col[RYB + 2 * R];
#pragma unroll
                    for (int j = 0; j < RYB + 2 * R; ++j) col[j] = base[j * kWave];
#pragma unroll
                    for (int i = 0; i < RYB; ++i) {
                        cb[i] = col[i + R];
                        float a = tp.c[0] * col[i + R];
#pragma unroll
                        for (int e = 1; e <= R; ++e) {
                            a = fmaf(tp.c[star_y<R>(-e)], col[i + R - e], a);
                            a = fmaf(tp.c[star_y<R>(e)], col[i + R + e], a);
                        }
                        pb[i] = a;
                    }
                    // x arms; lanes within R of the tile edge read neighbouring
                    // LDS words and produce values that are never stored.
#pragma unroll
                    for (int e = 1; e <= R; ++e)
#pragma unroll
                        for (int i = 0; i < RYB; ++i) {
                            const float* row = tb + (R + wv * RYB + i) * kWave + lane;
                            pb[i] = fmaf(tp.c[star_x<R>(-e)], row[-e], pb[i]);
                            pb[i] = fmaf(tp.c[star_x<R>(e)], row[e], pb[i]);
                        }
                }
#pragma unroll
                for (int i = 0; i < RYB; ++i) {
                    accB[R][i] += pb[i];
                    cqB[R][i] = cb[i];
                }
#pragma unroll
                for (int e = 1; e <= R; ++e)
#pragma unroll
                    for (int i = 0; i < RYB; ++i) {
                        accB[R - e][i] = fmaf(tp.c[star_z<R>(e)], cb[i], accB[R - e][i]);
                        accB[R + e][i] = fmaf(tp.c[star_z<R>(-e)], cb[i], accB[R + e][i]);
                    }
                // ---- stage B emission: u_{t+2} on the output tile, plane zb
                const int zb = za - R;
                if (zb >= z0 && lane_out) {
                    const size_t zoff = (size_t)zb * plane_sz;
#pragma unroll
                    for (int i = 0; i < RYB; ++i) {
                        const int gy = ey0 + R + wv * RYB + i;
                        if (gy >= ny) continue;
                        const uint32_t o = (uint32_t)(gy * nx + gxe);
                        float v = 2.f * cqB[0][i] - uB[d][i] + kB[d][i] * accB[0][i];
                        if (zb == w.src_z && gy == w.src_y && gxe == w.src_x) v += *w.amp2;
                        if (w.trace2 != nullptr && zb == w.rec_z) w.trace2[o] = v;
                        __builtin_nontemporal_store(v, &w.out2[zoff + o]);
                    }
                }
#pragma unroll
                for (int q = 0; q < Q - 1; ++q)
#pragma unroll
                    for (int i = 0; i < RYB; ++i) accB[q][i] = accB[q + 1][i];
#pragma unroll
                for (int i = 0; i < RYB; ++i) accB[Q - 1][i] = 0.f;
#pragma unroll
                for (int q = 0; q < R; ++q)
#pragma unroll
                    for (int i = 0; i < RYB; ++i) cqB[q][i] = cqB[q + 1][i];
            }
            issue_b(d, zp + D - 2 * R);
        }
    }
}

bool wave3d_tb2_supported(int r) { return r == 2 || r == 4; }

template <int R, int BC, int RYB>
static hipError_t go(const Geom& g, int zc, const Taps& tp, const WaveTB2& w, hipStream_t s) {
    constexpr int OX = kWave - 2 * R;
    constexpr int BY = 4 * RYB;
    constexpr int D = 2;
    const int tiles_x = (g.nx + OX - 1) / OX, tiles_y = (g.ny + BY - 1) / BY;
    const int nchunks = (g.nz + zc - 1) / zc;
    hipLaunchKernelGGL((wave3d_tb2_kernel<R, BC, RYB, D>), dim3(tiles_x * tiles_y * nchunks),
                       dim3(kThreads), 0, s, w, g.nx, g.ny, g.nz, zc, tiles_x, tiles_y, tp);
    return hipGetLastError();
}

template <int R, int BC>
static hipError_t go_ry(const Geom& g, const LaunchCfg& c, const Taps& tp, const WaveTB2& w,
                        hipStream_t s) {
    const int zc = c.zchunk > 0 ? c.zchunk : g.nz;
    if (c.tile_y >= 16) return go<R, BC, 4>(g, zc, tp, w, s);
    return go<R, BC, 2>(g, zc, tp, w, s);
}

hipError_t launch_wave3d_tb2(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                             const WaveTB2& w, hipStream_t stream) {
    if (g.r == 4)
        return g.boundary == kPeriodic ? go_ry<4, kPeriodic>(g, cfg, taps, w, stream)
                                       : go_ry<4, kZero>(g, cfg, taps, w, stream);
    if (g.r == 2)
        return g.boundary == kPeriodic ? go_ry<2, kPeriodic>(g, cfg, taps, w, stream)
                                       : go_ry<2, kZero>(g, cfg, taps, w, stream);
    return hipErrorInvalidValue;
}

}  // namespace stk
