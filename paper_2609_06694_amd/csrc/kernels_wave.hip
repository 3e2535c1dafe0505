// 3D acoustic leapfrog and its adjoint, fused with source, receiver and the
// kappa-gradient accumulation (a stencil fused with the physics around it in
// one launch, Section 4.3).
//
//  forward : u_{t+1} = 2 u_t - u_{t-1} + kappa (.) L(u_t)   (+ source, trace)
//  adjoint : l_t = 2 l_{t+1} - s * l_{t+2} + L^T(kappa (.) l_{t+1})
//  gradient: the adjoint step plus the receiver residual injection
//            l_t += [z = rec] (u_t - d_t), and g += l_{t+1} (.) L(u_t)
//
// L is a star of radius R held in `tp` (transposed taps for the adjoint).
// Every field is f32; the output may alias the pointwise `prev` operand
// because each cell of prev is read only by the thread that writes it.
#include "internal.h"
#include "zmarch.h"

namespace stk {

// Each workgroup keeps D planes in flight: the slot of plane zp is refilled
// with plane zp + D as soon as it has been staged in LDS, and the pointwise
// operands of output plane zo are issued D planes before zo is emitted, so
// D HBM round trips overlap instead of one per plane.
template <int MODE, int R, int BC, int RY, int NW, int D>
__global__ __launch_bounds__(NW * kWave) void wave3d_kernel(WaveLaunch w, int nx, int ny, int nz,
                                                            int zc, int tiles_x, int tiles_y,
                                                            Taps tp, Taps tp2) {
    using G = PlaneGeom<R, RY, NW>;
    constexpr bool TWO = (MODE == kWaveGrad);       // second stencil field u_t
    constexpr bool SCALE = (MODE != kWaveFwd);      // first field is kappa (.) lambda
    __shared__ float tile[TWO ? 4 : 2][G::H * G::W];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % tiles_x;
    const int rest = b / tiles_x;
    const int tyi = rest % tiles_y, zci = rest / tiles_y;
    const int x0 = txi * G::BX, y0 = tyi * G::BY;
    const int z0 = zci * zc, z1 = min(z0 + zc, nz);
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const int gx = x0 + tx;
    const size_t plane_sz = (size_t)nx * ny;
    const int zbeg = z0 - R, zend = z1 + R;   // planes staged: zbeg .. zend-1

    constexpr int Q = 2 * R + 1;
    float acc[Q][RY], acc2[TWO ? Q : 1][RY];
    float cq[R + 1][RY];      // unscaled first field at planes zp-R..zp
    float cq2[TWO ? R + 1 : 1][RY];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            acc[q][i] = 0.f;
            if constexpr (TWO) acc2[q][i] = 0.f;
        }
#pragma unroll
    for (int q = 0; q <= R; ++q)
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            cq[q][i] = 0.f;
            if constexpr (TWO) cq2[q][i] = 0.f;
        }

    // Ring of D in-flight planes (first field, kappa when scaled, u_t when
    // two fields) and of D sets of pointwise operands.
    float vin[D][RY], vhalo[D][G::HT];
    float kin[SCALE ? D : 1][RY], khalo[SCALE ? D : 1][G::HT];
    float uin[TWO ? D : 1][RY], uhalo[TWO ? D : 1][G::HT];
    uint32_t vm[D];   // validity mask of the planes (same cells for all fields)
    float pq[D][RY], kq[MODE == kWaveFwd ? D : 1][RY], gq[TWO ? D : 1][RY];
    // Read once, up front: a load inside the per-cell branch would make the
    // wave wait for every load in flight.
    const float amp = (MODE == kWaveFwd && w.src_x >= 0) ? *w.src_amp : 0.f;

    // All loads are unconditional; plane indices past the end of the march
    // are clamped to its last plane (see load_plane).
    auto issue_plane = [&](int slot, int zp) {
        zp = min(zp, zend - 1);
        vm[slot] = load_plane<R, RY, BC, float, NW>(w.cur, nx, ny, nz, zp, x0, y0, vin[slot], vhalo[slot]);
        if constexpr (SCALE) load_plane<R, RY, BC, float, NW>(w.kappa, nx, ny, nz, zp, x0, y0, kin[slot], khalo[slot]);
        if constexpr (TWO) load_plane<R, RY, BC, float, NW>(w.u, nx, ny, nz, zp, x0, y0, uin[slot], uhalo[slot]);
    };
    // Pointwise operands of output plane zo (read by the thread that writes
    // it), clamped to the chunk and the grid; clamped values are never used.
    auto issue_point = [&](int slot, int zo) {
        const size_t zoff = (size_t)min(max(zo, z0), z1 - 1) * plane_sz;
        const float* pp = w.prev + zoff;
        const float* kp = w.kappa + zoff;
        const float* gp = w.grad + zoff;
        const int gxc = min(gx, nx - 1);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            const int gy = min(y0 + ty * RY + i, ny - 1);
            const uint32_t o = (uint32_t)(gy * nx + gxc);
            pq[slot][i] = __builtin_nontemporal_load(&pp[o]);
            if constexpr (MODE == kWaveFwd) kq[slot][i] = __builtin_nontemporal_load(&kp[o]);
            if constexpr (TWO) gq[slot][i] = __builtin_nontemporal_load(&gp[o]);
        }
    };

#pragma unroll
    for (int d = 0; d < D; ++d) {
        issue_plane(d, zbeg + d);
        issue_point(d, zbeg + d - R);
    }

    for (int zb = zbeg; zb < zend; zb += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int zp = zb + d;
            // The march runs in whole groups of D planes: up to D-1 planes
            // past zend are clamped loads that emit no output.  (A uniform
            // early exit here would let the compiler assume fewer loads in
            // flight at the loop head and wait for all of them.)
            float* t;
            float* t2 = nullptr;
            if constexpr (TWO) {
                t = tile[2 * (zp & 1)];
                t2 = tile[2 * (zp & 1) + 1];
            } else {
                t = tile[zp & 1];
            }
            if constexpr (SCALE) store_plane<R, RY, BC, true, float, NW>(t, vin[d], vhalo[d], vm[d], kin[d], khalo[d]);
            else store_plane<R, RY, BC, float, NW>(t, vin[d], vhalo[d], vm[d]);
            if constexpr (TWO) store_plane<R, RY, BC, float, NW>(t2, uin[d], uhalo[d], vm[d]);
            float cen[RY];
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                const float v = masked<BC>(vin[d][i], vm[d], i);
                cq[R][i] = v;
                if constexpr (SCALE) cen[i] = v * kin[d][i];
                else cen[i] = v;
                if constexpr (TWO) cq2[R][i] = masked<BC>(uin[d][i], vm[d], i);
            }
            issue_plane(d, zp + D);
            __syncthreads();

            {
                float p[RY];
                star_plane<R, RY, NW>(t, tp, p);
#pragma unroll
                for (int i = 0; i < RY; ++i) acc[R][i] += p[i];
#pragma unroll
                for (int e = 1; e <= R; ++e)
#pragma unroll
                    for (int i = 0; i < RY; ++i) {
                        acc[R - e][i] = fmaf(tp.c[star_z<R>(e)], cen[i], acc[R - e][i]);
                        acc[R + e][i] = fmaf(tp.c[star_z<R>(-e)], cen[i], acc[R + e][i]);
                    }
            }
            if constexpr (TWO) {
                float p[RY];
                star_plane<R, RY, NW>(t2, tp2, p);
#pragma unroll
                for (int i = 0; i < RY; ++i) acc2[R][i] += p[i];
#pragma unroll
                for (int e = 1; e <= R; ++e)
#pragma unroll
                    for (int i = 0; i < RY; ++i) {
                        acc2[R - e][i] = fmaf(tp2.c[star_z<R>(e)], cq2[R][i], acc2[R - e][i]);
                        acc2[R + e][i] = fmaf(tp2.c[star_z<R>(-e)], cq2[R][i], acc2[R + e][i]);
                    }
            }

            // Output plane zo = zp - R has received all 2R+1 planes.
            const int zo = zp - R;
            if (zo >= z0 && zo < z1 && gx < nx) {
                const size_t zoff = (size_t)zo * plane_sz;
                float* np_ = w.next + zoff;
                float* gp = w.grad + zoff;
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int gy = y0 + ty * RY + i;
                    if (gy >= ny) continue;
                    const uint32_t o = (uint32_t)(gy * nx + gx);
                    float v;
                    if constexpr (MODE == kWaveFwd) {
                        v = 2.f * cq[0][i] - pq[d][i] + kq[d][i] * acc[0][i];
                        if (zo == w.src_z && gy == w.src_y && gx == w.src_x) v += amp;
                        if (w.trace_t != nullptr && zo == w.rec_z) w.trace_t[o] = v;
                    } else if constexpr (MODE == kWaveAdj) {
                        v = 2.f * cq[0][i] - w.prev_sign * pq[d][i] + acc[0][i];
                    } else {
                        v = 2.f * cq[0][i] - pq[d][i] + acc[0][i];
                        if (w.target_t != nullptr && zo == w.rec_z) v += cq2[0][i] - w.target_t[o];
                        __builtin_nontemporal_store(fmaf(cq[0][i], acc2[0][i], gq[d][i]), &gp[o]);
                    }
                    __builtin_nontemporal_store(v, &np_[o]);
                }
            }
            issue_point(d, zp + D - R);
#pragma unroll
            for (int q = 0; q < Q - 1; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    acc[q][i] = acc[q + 1][i];
                    if constexpr (TWO) acc2[q][i] = acc2[q + 1][i];
                }
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                acc[Q - 1][i] = 0.f;
                if constexpr (TWO) acc2[Q - 1][i] = 0.f;
            }
#pragma unroll
            for (int q = 0; q < R; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    cq[q][i] = cq[q + 1][i];
                    if constexpr (TWO) cq2[q][i] = cq2[q + 1][i];
                }
        }
    }
}

bool wave3d_supported(int r) { return r >= 1 && r <= 4; }


// Planes in flight per workgroup: deeper for thin tiles (few registers per
// plane), shallower for the two-field gradient step.
template <int MODE, int RY>
constexpr int wave_depth() {
    return MODE == kWaveGrad ? (RY >= 4 ? 1 : 2) : (RY >= 8 ? 1 : (RY >= 4 ? 2 : 4));
}

template <int MODE, int R, int BC, int RY, int NW>
static hipError_t go(const Geom& g, int zc, const Taps& tp, const Taps& tp2, const WaveLaunch& w,
                     hipStream_t s) {
    using G = PlaneGeom<R, RY, NW>;
    const int tiles_x = (g.nx + G::BX - 1) / G::BX, tiles_y = (g.ny + G::BY - 1) / G::BY;
    const int nchunks = (g.nz + zc - 1) / zc;
    constexpr int D = wave_depth<MODE, RY>();
    hipLaunchKernelGGL((wave3d_kernel<MODE, R, BC, RY, NW, D>), dim3(tiles_x * tiles_y * nchunks),
                       dim3(G::NT), 0, s, w, g.nx, g.ny, g.nz, zc, tiles_x, tiles_y, tp, tp2);
    return hipGetLastError();
}

template <int MODE, int R, int BC>
static hipError_t go_ry(const Geom& g, const LaunchCfg& c, const Taps& tp, const Taps& tp2,
                        const WaveLaunch& w, hipStream_t s) {
    const int zc = c.zchunk > 0 ? c.zchunk : g.nz;
    switch (zm3d_rows(c)) {
        case 8: return go<MODE, R, BC, 2, 4>(g, zc, tp, tp2, w, s);
        case 16: return go<MODE, R, BC, 4, 4>(g, zc, tp, tp2, w, s);
        default: return go<MODE, R, BC, 4, 8>(g, zc, tp, tp2, w, s);
    }
}

template <int MODE, int R>
static hipError_t go_bc(const Geom& g, const LaunchCfg& c, const Taps& tp, const Taps& tp2,
                        const WaveLaunch& w, hipStream_t s) {
    return g.boundary == kPeriodic ? go_ry<MODE, R, kPeriodic>(g, c, tp, tp2, w, s)
                                   : go_ry<MODE, R, kZero>(g, c, tp, tp2, w, s);
}

template <int MODE>
static hipError_t go_r(const Geom& g, const LaunchCfg& c, const Taps& tp, const Taps& tp2,
                       const WaveLaunch& w, hipStream_t s) {
    switch (g.r) {
        case 1: return go_bc<MODE, 1>(g, c, tp, tp2, w, s);
        case 2: return go_bc<MODE, 2>(g, c, tp, tp2, w, s);
        case 3: return go_bc<MODE, 3>(g, c, tp, tp2, w, s);
        case 4: return go_bc<MODE, 4>(g, c, tp, tp2, w, s);
    }
    return hipErrorInvalidValue;
}

// `taps` is the stencil applied to the first field: L for the forward step,
// L^T for the adjoint and gradient steps.  `taps_fwd` (L) is applied to the
// second field u_t in gradient mode.
hipError_t launch_wave3d(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                              const Taps& taps_fwd, WaveMode mode, const WaveLaunch& w,
                              hipStream_t stream) {
    switch (mode) {
        case kWaveFwd: return go_r<kWaveFwd>(g, cfg, taps, taps_fwd, w, stream);
        case kWaveAdj: return go_r<kWaveAdj>(g, cfg, taps, taps_fwd, w, stream);
        case kWaveGrad: return go_r<kWaveGrad>(g, cfg, taps, taps_fwd, w, stream);
        case kWaveGradPt: break;   // the pointwise gradient step is the ring kernel's
    }
    return hipErrorInvalidValue;
}

__global__ void scale_kernel(float* dst, const float* src, float alpha, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t j = i; j < n; j += stride) dst[j] = alpha * src[j];
}

hipError_t launch_scale(float* dst, const float* src, float alpha, size_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, stream, dst, src,
                       alpha, n);
    return hipGetLastError();
}

// dst = alpha * B(x) * dst, B = (1 - gamma/2) / (1 + gamma/2) of the
// absorbing layer (one thread per cell of an x row; grid: rows).
__global__ void sponge_scale_kernel(float* dst, float alpha, int nx, int ny, int nz, int w, float s, float invw) {
    const int row = blockIdx.x;   // y + ny * z
    const int y = row % ny, z = row / ny;
    const float gyz = sponge_ramp(y, ny, w, s, invw) + sponge_ramp(z, nz, w, s, invw);
    float* p = dst + (size_t)row * nx;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
        const float gm = gyz + sponge_ramp(x, nx, w, s, invw);
        const float A = __builtin_amdgcn_rcpf(1.f + 0.5f * gm);
        p[x] = alpha * ((1.f - 0.5f * gm) * A) * p[x];
    }
}

hipError_t launch_sponge_scale(const Geom& g, float* dst, float alpha, int w, float s, hipStream_t stream) {
    const size_t rows = (size_t)g.ny * g.nz;
    if (rows == 0 || g.nx == 0) return hipSuccess;
    if (rows > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sponge_scale_kernel, dim3((unsigned)rows), dim3(kThreads), 0, stream, dst, alpha, g.nx,
                       g.ny, g.nz, w, s, w > 0 ? 1.f / (float)w : 0.f);
    return hipGetLastError();
}

__global__ void fill_kernel(float* dst, float v, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t j = i; j < n; j += stride) dst[j] = v;
}

hipError_t launch_fill(float* dst, float v, size_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, stream, dst, v, n);
    return hipGetLastError();
}

// Stage 1: workgroup b sums the squared misfit over a fixed strided subset.
__global__ __launch_bounds__(kThreads) void loss_part_kernel(const float* traces,
                                                              const float* target, size_t n,
                                                              double* parts) {
    __shared__ double red[kThreads];
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kThreads) {
        const double d = (double)traces[i] - (double)target[i];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

// Stage 2: one workgroup adds the partial sums in a fixed order.
__global__ __launch_bounds__(kThreads) void loss_final_kernel(const double* parts, int nparts,
                                                               double* loss) {
    __shared__ double red[kThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kThreads) s += parts[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = 0.5 * red[0];
}

hipError_t launch_trace_loss(const float* traces, const float* target, size_t n, double* parts,
                             double* loss, hipStream_t stream) {
    hipLaunchKernelGGL(loss_part_kernel, dim3(kLossParts), dim3(kThreads), 0, stream, traces,
                       target, n, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(kThreads), 0, stream, parts, kLossParts,
                       loss);
    return hipGetLastError();
}

}  // namespace stk
