// 3D linear sweep of radius 1 (27-point box, 7-point star), two time steps
// per launch (temporal blocking, Section 4.3).
//
// A workgroup of NW waves owns 64 extended columns x 4 NW extended rows
// (four rows per thread) and marches z.  Stage 1 computes the intermediate level u_{t+1} on that whole
// extended region (the output tile plus a one-cell ring) exactly as the
// one-step z-march does: each input plane is staged once in LDS with its
// halo and its contributions go to a register queue of partial sums.  When
// u_{t+1} of plane z1 is complete it is rounded to the storage precision,
// set to zero outside a zero frame, and staged in a second LDS tile; stage 2
// applies the stencil to it (a second register queue) and emits u_{t+2} on
// the inner 62 x (4 NW - 2) cells, one plane behind.  The intermediate level
// never leaves the chip, so a launch reads and writes each cell once for two
// steps; the ring of recomputed u_{t+1} costs 64*32/(62*30) - 1 = 10 % more
// arithmetic with eight waves.
#include "internal.h"
#include "zmarch.h"

namespace stk {

namespace {
constexpr int kR = 1;
constexpr int kRYA = 4;                 // extended rows per thread
constexpr int kOX = kWave - 2 * kR;     // 62 output columns
constexpr int kW1 = kWave + 2 * kR;     // pitch of the u_{t+1} tile (one pad column each side)
}  // namespace

template <int SHAPE, typename T, int BC, int NW, int D>
__global__ __launch_bounds__(NW * kWave) void zm3d_tb2_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                              int nx, int ny, int nz, int zc, int tiles_x,
                                                              int tiles_y, Taps tp) {
    constexpr int R = kR, RY = kRYA, Q = 2 * R + 1;
    using GA = PlaneGeom<R, RY, NW>;            // 64 x 4 NW extended region, one-cell halo
    constexpr int kEY = GA::BY;                 // extended rows
    constexpr int kOY = kEY - 2 * R;            // output rows
    __shared__ float t0[2][GA::H * GA::W];   // u_t planes with halo
    __shared__ float t1[2][kEY * kW1];       // u_{t+1} planes on the extended region
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % tiles_x;
    const int rest = b / tiles_x;
    const int tyi = rest % tiles_y, zci = rest / tiles_y;
    const int ex0 = txi * kOX - R, ey0 = tyi * kOY - R;   // extended-region origin
    const int z0 = zci * zc, z1e = min(z0 + zc, nz);
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const int gx = ex0 + tx;
    const bool col_in = gx >= 0 && gx < nx;
    const bool col_out = tx >= R && tx < R + kOX && gx < nx;
    const size_t plane_sz = (size_t)nx * ny;

    float acc1[Q][RY], acc2[Q][RY];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < RY; ++i) acc1[q][i] = acc2[q][i] = 0.f;

    // u_t planes zbeg .. zend-1 feed u_{t+1} on planes z0-R .. z1e+R-1,
    // which feed u_{t+2} on the chunk's planes z0 .. z1e-1.
    const int zbeg = z0 - 2 * R, zend = z1e + 2 * R;
    T vin[D][RY], vhalo[D][GA::HT];
    uint32_t vm[D];
    const PlaneIdx<R, RY, NW> pidx = plane_index<R, RY, BC, T, NW>(nx, ny, ex0, ey0);
#pragma unroll
    for (int d = 0; d < D; ++d)
        vm[d] = load_plane_at<R, RY, BC, T, NW>(in, nx, ny, nz, min(zbeg + d, zend - 1), pidx, vin[d], vhalo[d]);

    for (int zb = zbeg; zb < zend; zb += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int zp = zb + d;   // planes past zend: clamped reloads, no output
            float* ta = t0[zp & 1];
            store_plane<R, RY, BC, T, NW>(ta, vin[d], vhalo[d], vm[d]);
            float cen[RY];
#pragma unroll
            for (int i = 0; i < RY; ++i) cen[i] = masked<BC>(vin[d][i], vm[d], i);
            vm[d] = load_plane_at<R, RY, BC, T, NW>(in, nx, ny, nz, min(zp + D, zend - 1), pidx, vin[d], vhalo[d]);
            __syncthreads();

            // ---- stage 1: plane zp of u_t into the u_{t+1} queue
            if constexpr (SHAPE == kStar) {
                float p[RY];
                star_plane<R, RY, NW>(ta, tp, p);
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    acc1[R][i] += p[i];
                    acc1[0][i] = fmaf(tp.c[star_z<R>(1)], cen[i], acc1[0][i]);
                    acc1[2][i] = fmaf(tp.c[star_z<R>(-1)], cen[i], acc1[2][i]);
                }
            } else {
#pragma unroll
                for (int dx = -R; dx <= R; ++dx) {
                    float col[RY + 2 * R];
                    const float* base = ta + (ty * RY) * GA::W + R + tx + dx;
#pragma unroll
                    for (int j = 0; j < RY + 2 * R; ++j) col[j] = base[j * GA::W];
#pragma unroll
                    for (int dz = -R; dz <= R; ++dz)
#pragma unroll
                        for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                            for (int i = 0; i < RY; ++i)
                                acc1[R - dz][i] = fmaf(tp.c[box3<R>(dz, dy, dx)], col[i + R + dy], acc1[R - dz][i]);
                }
            }
            // u_{t+1} of plane za = zp - R is complete: storage rounding, zero
            // frame, staged for stage 2.
            const int za = zp - R;
            float* tb = t1[za & 1];
            {
                const bool zin = BC == kPeriodic || (za >= 0 && za < nz);
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int row = ty * RY + i;
                    const int gy = ey0 + row;
                    float v = round_to_storage<T>(acc1[0][i]);
                    if (BC == kZero && !(zin && col_in && gy >= 0 && gy < ny)) v = 0.f;
                    tb[row * kW1 + R + tx] = v;
                    cen[i] = v;
                }
            }
#pragma unroll
            for (int q = 0; q < Q - 1; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) acc1[q][i] = acc1[q + 1][i];
#pragma unroll
            for (int i = 0; i < RY; ++i) acc1[Q - 1][i] = 0.f;
            __syncthreads();

            // ---- stage 2: plane za of u_{t+1} into the u_{t+2} queue.  Lanes and
            // rows on the ring produce values that are never stored (the pad
            // columns of tb are never written, so their sums are discarded).
            if constexpr (SHAPE == kStar) {
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int row = ty * RY + i;
                    const float* c0 = tb + row * kW1 + R + tx;
                    const float up = row > 0 ? c0[-kW1] : 0.f;
                    const float dn = row < kEY - 1 ? c0[kW1] : 0.f;
                    float a = tp.c[0] * c0[0];
                    a = fmaf(tp.c[star_x<R>(-1)], c0[-1], a);
                    a = fmaf(tp.c[star_x<R>(1)], c0[1], a);
                    a = fmaf(tp.c[star_y<R>(-1)], up, a);
                    a = fmaf(tp.c[star_y<R>(1)], dn, a);
                    acc2[R][i] += a;
                    acc2[0][i] = fmaf(tp.c[star_z<R>(1)], cen[i], acc2[0][i]);
                    acc2[2][i] = fmaf(tp.c[star_z<R>(-1)], cen[i], acc2[2][i]);
                }
            } else {
#pragma unroll
                for (int dx = -R; dx <= R; ++dx) {
                    float col[RY + 2 * R];
#pragma unroll
                    for (int j = 0; j < RY + 2 * R; ++j) {
                        const int row = ty * RY - R + j;
                        col[j] = (row >= 0 && row < kEY) ? tb[row * kW1 + R + tx + dx] : 0.f;
                    }
#pragma unroll
                    for (int dz = -R; dz <= R; ++dz)
#pragma unroll
                        for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                            for (int i = 0; i < RY; ++i)
                                acc2[R - dz][i] = fmaf(tp.c[box3<R>(dz, dy, dx)], col[i + R + dy], acc2[R - dz][i]);
                }
            }
            // u_{t+2} of plane zo = za - R is complete.
            const int zo = za - R;
            if (zo >= z0 && zo < z1e && col_out) {
                T* o = out + (size_t)zo * plane_sz;
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int row = ty * RY + i;
                    const int gy = ey0 + row;
                    if (row >= R && row < R + kOY && gy < ny)
                        __builtin_nontemporal_store(from_f32<T>(acc2[0][i]), &o[(uint32_t)(gy * nx + gx)]);
                }
            }
#pragma unroll
            for (int q = 0; q < Q - 1; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) acc2[q][i] = acc2[q + 1][i];
#pragma unroll
            for (int i = 0; i < RY; ++i) acc2[Q - 1][i] = 0.f;
        }
    }
}

bool zm3d_tb2_supported(int r, int shape) { return r == 1 && (shape == kStar || shape == kBox); }

template <int SHAPE, typename T, int BC, int NW>
static hipError_t go(const Geom& g, int zc, const Taps& tp, const void* in, void* out, hipStream_t s) {
    constexpr int D = 2;
    constexpr int OY = 4 * NW - 2 * kR;
    const int tiles_x = (g.nx + kOX - 1) / kOX, tiles_y = (g.ny + OY - 1) / OY;
    const int nchunks = (g.nz + zc - 1) / zc;
    hipLaunchKernelGGL((zm3d_tb2_kernel<SHAPE, T, BC, NW, D>), dim3(tiles_x * tiles_y * nchunks),
                       dim3(NW * kWave), 0, s, (const T*)in, (T*)out, g.nx, g.ny, g.nz, zc, tiles_x, tiles_y, tp);
    return hipGetLastError();
}

// tile_y = extended rows: 16 (4 waves, 62 x 14 outputs) or 32 (8 waves, 62 x 30).
template <int SHAPE, typename T>
static hipError_t go_bc(const Geom& g, int ty, int zc, const Taps& tp, const void* in, void* out,
                        hipStream_t s) {
    if (ty >= 32)
        return g.boundary == kPeriodic ? go<SHAPE, T, kPeriodic, 8>(g, zc, tp, in, out, s)
                                       : go<SHAPE, T, kZero, 8>(g, zc, tp, in, out, s);
    return g.boundary == kPeriodic ? go<SHAPE, T, kPeriodic, 4>(g, zc, tp, in, out, s)
                                   : go<SHAPE, T, kZero, 4>(g, zc, tp, in, out, s);
}

// Two steps of a radius-1 3D linear sweep in one launch.
hipError_t launch_zm3d_tb2(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                           void* out, hipStream_t stream) {
    if (!zm3d_tb2_supported(g.r, g.shape) || (g.dtype != 0 && g.dtype != 1)) return hipErrorInvalidValue;
    const int zc = cfg.zchunk > 0 ? cfg.zchunk : g.nz;
    const int ty = cfg.tile_y;
    if (g.dtype == 0)
        return g.shape == kBox ? go_bc<kBox, float>(g, ty, zc, taps, in, out, stream)
                               : go_bc<kStar, float>(g, ty, zc, taps, in, out, stream);
    return g.shape == kBox ? go_bc<kBox, _Float16>(g, ty, zc, taps, in, out, stream)
                           : go_bc<kStar, _Float16>(g, ty, zc, taps, in, out, stream);
}

}  // namespace stk
