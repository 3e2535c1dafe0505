// 3D box sweep (radius 1) with fp16 storage on packed-half dot products.
//
// Each lane owns two adjacent cells of a row (one 32-bit pair of binary16
// values), so a wave moves 256 contiguous bytes per row and a plane enters
// LDS as 32-bit pairs.  The contraction uses v_dot2 (two binary16 products
// added to an f32 accumulator; the products are exact in f32) and the
// mixed-precision fma (binary16 operand, f32 weight and sum): for the output
// pair (x, x+1) and one (dz, dy) row of weights w_-1, w_0, w_1,
//   out(x)   += dot2((u_x, u_x+1), (w_0, w_1))  + w_-1 * u_x-1
//   out(x+1) += dot2((u_x, u_x+1), (w_-1, w_0)) + w_1  * u_x+2,
// four instructions for six multiply-adds.  Of the three rows of one dz,
// two end terms of each cell share a dot2: (u_x-1 of rows y-1, y) with
// (w_-1 of those rows), and (u_x+2 of rows y, y+1) with their w_1, the
// value pairs built by one v_perm per row and reused by the three dz; a
// cell's nine rows take 9 + 3 + 3 = 15 instructions per plane for its 27
// multiply-adds (18 unpaired).  The packed weights are the
// binary16 roundings w_hi of the f32 weights; their residuals w - w_hi (at
// most 2^-12 |w|) enter through one extra multiply-add per cell,
// (sum of residuals) * u(x): the part of the residual sum that acts on the
// local mean, so the sweep's action on slowly varying data (and its sum
// for a periodic grid) keeps the f32 weights' value.  What is left,
// sum (w - w_hi)(u(x+d) - u(x)), is below 2^-12 of the local variation and
// well under the binary16 rounding of every step.  Under a zero frame the
// taps that leave the grid read zero rather than the centre value, so there
// the residual sum runs over the taps inside the grid only.
//
// The 7-point star (radius 1) is the box with its off-axis weights zero; it
// runs the same code with the rows and terms those zeros would feed left
// out (the centre row keeps all four instructions, the four axis rows
// keep the two dot products), so it matches the box kernel given those
// zero weights, at a third of its arithmetic.
//
// Radius 2 (the 125-point box) uses the same pairs: for a row of weights
// w_-2..w_2,
//   out(x)   += dot2((u_x-2, u_x-1), (w_-2, w_-1)) + dot2((u_x, u_x+1), (w_0, w_1)) + w_2 u_x+2
//   out(x+1) += w_-2 u_x-1 + dot2((u_x, u_x+1), (w_-1, w_0)) + dot2((u_x+2, u_x+3), (w_1, w_2)),
// six instructions for ten multiply-adds; its 25 weight rows (six words
// each) are read per row through the scalar cache, five rows at a time.
//
// Layout and march follow the z-march of zmarch.h: a workgroup owns a
// column of 128 x BY cells, stages every plane once (with a one-pair halo
// in x and an R-row halo in y) and adds the plane's contributions to the
// 2R+1 output planes it touches into a register queue of partial sums.
// Requires an even nx (whole pairs in every row).
#include <string.h>

#include <type_traits>

#include "internal.h"
#include "zmarch.h"

namespace stk {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// Weights of a radius-1 box in the form the kernel consumes, per (dz, dy)
// row k = (dz+1)*3 + (dy+1): packed (w_0, w_1) and (w_-1, w_0) binary16
// pairs, the binary16 values of w_-1 and w_1 widened to f32, the sum of
// all residuals w - w_hi, and each residual in (dz, dy, dx) order.
struct H2Taps {
    uint32_t p01[9], pm0[9];
    float wm[9], wp[9];
    // Per dz: (w_-1 of row dy = -1, w_-1 of row dy = 0) and (w_1 of row
    // dy = 0, w_1 of row dy = 1) as binary16 pairs, so two end terms of a
    // cell take one dot2 (the pairs of values come from one v_perm).
    uint32_t wmp[3], wpp[3];
    float res;
    float rr[27];
};

// Radius 2: per (dz, dy) row k = (dz+2)*5 + (dy+2), words [8k .. 8k+5] of
// `row` hold (w_-2, w_-1), (w_0, w_1), (w_-1, w_0), (w_1, w_2) as binary16
// pairs and w_2, w_-2 as f32 bit patterns; for dy = -2 and 0, words 6 and 7
// hold (w_2 of rows k, k+1) and (w_-2 of rows k, k+1) as binary16 pairs; rr
// holds the 125 residuals in
// (dz, dy, dx) order.  A kernel argument (1.3 KB), read per row through
// the scalar cache.
struct H2Taps5 {
    uint32_t row[25 * 8];
    float rr[125];
    float res;
};

// Sum of the residuals rr ((2R+1)^3, in LDS) of the taps of cell (cx, cy, cz)
// that land inside an nx x ny x nz grid (with all_z, every plane counts as
// inside).  A rolled loop: it runs once per thread and on the two face
// planes only.
template <int R = 1>
__device__ __forceinline__ float h2_inner_res(const float* rr, int cx, int cy, int cz, int nx, int ny, int nz,
                                              bool all_z) {
    constexpr int Q = 2 * R + 1;
    float r = 0.f;
#pragma unroll 1
    for (int t = 0; t < Q * Q * Q; ++t) {
        const int dz = t / (Q * Q) - R, dy = (t / Q) % Q - R, dx = t % Q - R;
        const bool in = (all_z || (unsigned)(cz + dz) < (unsigned)nz) && (unsigned)(cy + dy) < (unsigned)ny &&
                        (unsigned)(cx + dx) < (unsigned)nx;
        r += in ? rr[t] : 0.f;
    }
    return r;
}

template <int RY, int NW, int R = 1>
struct H2Geom {
    static constexpr int NT = NW * kWave;
    static constexpr int BXP = kWave;          // pairs per tile row
    static constexpr int BY = NW * RY;
    static constexpr int WP = BXP + 2;         // one halo pair on each side (R <= 2 cells)
    static constexpr int H = BY + 2 * R;       // R halo rows above and below
    static constexpr int NH = WP * H - BXP * BY;
    static constexpr int HT = (NH + NT - 1) / NT;
};

__device__ __forceinline__ half2_t as_h2(uint32_t v) { return __builtin_bit_cast(half2_t, v); }

template <int R>
using H2TapsOf = std::conditional_t<R == 1, H2Taps, H2Taps5>;

template <int R, int SH, int BC, int RY, int NW, int D>
__global__ __launch_bounds__(NW * kWave) void zm3d_h2_kernel(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out, int nxp, int ny,
                                                             int nz, int zc, int tiles_x, int tiles_y,
                                                             H2TapsOf<R> tp) {
    using G = H2Geom<RY, NW, R>;
    constexpr int Q = 2 * R + 1;
    __shared__ uint32_t tile[2][G::H * G::WP];

    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % tiles_x;
    const int rest = b / tiles_x;
    const int tyi = rest % tiles_y, zci = rest / tiles_y;
    const int x0 = txi * G::BXP, y0 = tyi * G::BY;   // x0 in pairs
    const int z0 = zci * zc, z1 = min(z0 + zc, nz);
    const int tx = threadIdx.x & (kWave - 1), ty = threadIdx.x >> 6;
    const int gx = x0 + tx;
    const int zbeg = z0 - R, zend = z1 + R;

    // In-plane addressing (pair offsets after the boundary rule) and x/y
    // validity, the same for every plane.
    uint32_t off[RY + G::HT];
    uint32_t mxy = 0;
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        int px = gx, py = y0 + ty * RY + i;
        const bool okx = fix_coord<BC>(px, nxp), oky = fix_coord<BC>(py, ny);
        off[i] = (uint32_t)(py * nxp + px) * 4u;
        mxy |= (uint32_t)(okx && oky) << i;
    }
#pragma unroll
    for (int j = 0; j < G::HT; ++j) {
        const int h = threadIdx.x + j * G::NT;
        const bool hv = h < G::NH;
        const int hh = hv ? h : 0;
        int ly, lx;
        if (hh < 2 * R * G::WP) {   // the R top rows, then the R bottom rows
            const int row = hh / G::WP;
            ly = row < R ? row : G::BY + row;
            lx = hh - row * G::WP;
        } else {                    // side pairs of the interior rows
            const int q = hh - 2 * R * G::WP;
            ly = R + (q >> 1);
            lx = (q & 1) ? G::WP - 1 : 0;
        }
        int px = x0 - 1 + lx, py = y0 - R + ly;
        const bool okx = fix_coord<BC>(px, nxp), oky = fix_coord<BC>(py, ny);
        off[RY + j] = (uint32_t)(py * nxp + px) * 4u;
        mxy |= (uint32_t)(hv && okx && oky) << (RY + j);
    }

    // Zero frame: residual sums over the in-grid taps of each cell of the
    // thread's pairs, for planes away from the z faces (the face planes
    // recompute theirs).
    __shared__ float rrs[Q * Q * Q];
    float ria[RY], rib[RY];
    if constexpr (BC == kZero) {
        for (int i = threadIdx.x; i < Q * Q * Q; i += G::NT) rrs[i] = tp.rr[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            const int cy = y0 + ty * RY + i;
            ria[i] = h2_inner_res<R>(rrs, 2 * gx, cy, 0, 2 * nxp, ny, nz, true);
            rib[i] = h2_inner_res<R>(rrs, 2 * gx + 1, cy, 0, 2 * nxp, ny, nz, true);
        }
    }

    float ax[Q][RY], ay[Q][RY];   // partial sums of output planes zp-R .. zp+R (cells x, x+1)
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < RY; ++i) ax[q][i] = ay[q][i] = 0.f;

    uint32_t vin[D][RY + G::HT];
    uint32_t vm[D];
    const size_t plane_sz = (size_t)nxp * ny;
    auto load = [&](int slot, int zp) {
        int gz = min(zp, zend - 1);
        const bool zin = fix_coord<BC>(gz, nz);
        const char* base = reinterpret_cast<const char*>(in + (size_t)gz * plane_sz);
#pragma unroll
        for (int k = 0; k < RY + G::HT; ++k) vin[slot][k] = load_at<uint32_t>(base, off[k]);
        vm[slot] = zin ? mxy : 0u;
    };
#pragma unroll
    for (int d = 0; d < D; ++d) load(d, zbeg + d);

    for (int zb = zbeg; zb < zend; zb += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int zp = zb + d;
            uint32_t* t = tile[zp & 1];
            // Stage the plane (cells outside a zero frame are zero).
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                const uint32_t v = BC == kPeriodic || ((vm[d] >> i) & 1u) ? vin[d][i] : 0u;
                t[(R + ty * RY + i) * G::WP + 1 + tx] = v;
            }
#pragma unroll
            for (int j = 0; j < G::HT; ++j) {
                const int h = threadIdx.x + j * G::NT;
                if (h < G::NH) {
                    int ly, lx;
                    if (h < 2 * R * G::WP) {
                        const int row = h / G::WP;
                        ly = row < R ? row : G::BY + row;
                        lx = h - row * G::WP;
                    } else {
                        const int q = h - 2 * R * G::WP;
                        ly = R + (q >> 1);
                        lx = (q & 1) ? G::WP - 1 : 0;
                    }
                    const uint32_t v = BC == kPeriodic || ((vm[d] >> (RY + j)) & 1u) ? vin[d][RY + j] : 0u;
                    t[ly * G::WP + lx] = v;
                }
            }
            load(d, zp + D);
            __syncthreads();

            // Rows -R .. RY-1+R of this thread's column of pairs: the pair
            // to the left, its own pair and the pair to the right.
            const uint32_t* cp = t + (ty * RY) * G::WP + tx;
            if constexpr (R == 1) {
                uint32_t pm[RY + 2], p0[RY + 2], pp[RY + 2];
#pragma unroll
                for (int j = 0; j < RY + 2; ++j) {
                    pm[j] = cp[j * G::WP];
                    p0[j] = cp[j * G::WP + 1];
                    pp[j] = cp[j * G::WP + 2];
                }
                // End values of the box rows in pairs: (u_x-1 of rows i, i+1)
                // for out(x) and (u_x+2 of rows i+1, i+2) for out(x+1).
                uint32_t em[SH == kBox ? RY : 1], ep[SH == kBox ? RY : 1];
                if constexpr (SH == kBox) {
#pragma unroll
                    for (int i = 0; i < RY; ++i) {
                        em[i] = __builtin_amdgcn_perm(pm[i + 1], pm[i], 0x07060302u);
                        ep[i] = __builtin_amdgcn_perm(pp[i + 2], pp[i + 1], 0x05040100u);
                    }
                }
                // Plane zp feeds output plane zp - dz with the weights of dz:
                // the centre pairs of the dz rows, then the end terms.
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
                    const int q = 1 - dz;
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy) {
                        if (SH == kStar && dz != 0 && dy != 0) continue;   // an all-zero row
                        const int k = (dz + 1) * 3 + (dy + 1);
#pragma unroll
                        for (int i = 0; i < RY; ++i) {
                            const int j = i + 1 + dy;
                            ax[q][i] = __builtin_amdgcn_fdot2(as_h2(p0[j]), as_h2(tp.p01[k]), ax[q][i], false);
                            ay[q][i] = __builtin_amdgcn_fdot2(as_h2(p0[j]), as_h2(tp.pm0[k]), ay[q][i], false);
                        }
                    }
                    if constexpr (SH == kBox) {
                        const int k0 = (dz + 1) * 3;   // row dy = -1 of this dz
#pragma unroll
                        for (int i = 0; i < RY; ++i) {
                            ax[q][i] = __builtin_amdgcn_fdot2(as_h2(em[i]), as_h2(tp.wmp[dz + 1]), ax[q][i], false);
                            ax[q][i] = fmaf(tp.wm[k0 + 2], (float)as_h2(pm[i + 2]).y, ax[q][i]);
                            ay[q][i] = __builtin_amdgcn_fdot2(as_h2(ep[i]), as_h2(tp.wpp[dz + 1]), ay[q][i], false);
                            ay[q][i] = fmaf(tp.wp[k0], (float)as_h2(pp[i]).x, ay[q][i]);
                        }
                    } else if (dz == 0) {   // the star's only end terms: row (0, 0)
#pragma unroll
                        for (int i = 0; i < RY; ++i) {
                            ax[q][i] = fmaf(tp.wm[4], (float)as_h2(pm[i + 1]).y, ax[q][i]);
                            ay[q][i] = fmaf(tp.wp[4], (float)as_h2(pp[i + 1]).x, ay[q][i]);
                        }
                    }
                }
            } else {
                // Radius 2: rolled loops over dy (the weight rows and the
                // thread's rows at offset dy live at a time; unrolled, the
                // compiler would load all 25 weight rows, 150 registers, at
                // once), the dz groups unrolled so each sum stays in its
                // register.  Rows dy, dy + 1 go together (dy = -2, 0): their
                // end terms w_2 u_x+2 and w_-2 u_x-1 share one dot2 on values
                // paired by a v_perm; row 2 goes alone.
#pragma unroll 1
                for (int dy = -R; dy < R; dy += 2) {
                    uint32_t pm[RY], p0[RY], pp[RY], qm[RY], q0[RY], qp[RY], ex[RY], ey[RY];
#pragma unroll
                    for (int i = 0; i < RY; ++i) {
                        const uint32_t* r = cp + (i + R + dy) * G::WP;
                        pm[i] = r[0];
                        p0[i] = r[1];
                        pp[i] = r[2];
                        qm[i] = r[G::WP];
                        q0[i] = r[G::WP + 1];
                        qp[i] = r[G::WP + 2];
                        ex[i] = __builtin_amdgcn_perm(qp[i], pp[i], 0x05040100u);   // (u_x+2 of rows dy, dy+1)
                        ey[i] = __builtin_amdgcn_perm(qm[i], pm[i], 0x07060302u);   // (u_x-1 of rows dy, dy+1)
                    }
#pragma unroll
                    for (int dz = -R; dz <= R; ++dz) {
                        const int q = R - dz;
                        const int k = (dz + R) * Q + (dy + R);   // row dy; row dy + 1 is k + 1
                        // (w_-2, w_-1), (w_0, w_1), (w_-1, w_0), (w_1, w_2) of both
                        // rows and the two end pairs (scalar loads from the
                        // arguments: uniform, no LDS traffic)
                        const uint4 wa = {tp.row[8 * k], tp.row[8 * k + 1], tp.row[8 * k + 2], tp.row[8 * k + 3]};
                        const uint4 wb = {tp.row[8 * k + 8], tp.row[8 * k + 9], tp.row[8 * k + 10], tp.row[8 * k + 11]};
                        const uint32_t fap = tp.row[8 * k + 6], fbp = tp.row[8 * k + 7];
#pragma unroll
                        for (int i = 0; i < RY; ++i) {
                            ax[q][i] = __builtin_amdgcn_fdot2(as_h2(pm[i]), as_h2(wa.x), ax[q][i], false);
                            ax[q][i] = __builtin_amdgcn_fdot2(as_h2(p0[i]), as_h2(wa.y), ax[q][i], false);
                            ax[q][i] = __builtin_amdgcn_fdot2(as_h2(qm[i]), as_h2(wb.x), ax[q][i], false);
                            ax[q][i] = __builtin_amdgcn_fdot2(as_h2(q0[i]), as_h2(wb.y), ax[q][i], false);
                            ax[q][i] = __builtin_amdgcn_fdot2(as_h2(ex[i]), as_h2(fap), ax[q][i], false);
                            ay[q][i] = __builtin_amdgcn_fdot2(as_h2(p0[i]), as_h2(wa.z), ay[q][i], false);
                            ay[q][i] = __builtin_amdgcn_fdot2(as_h2(pp[i]), as_h2(wa.w), ay[q][i], false);
                            ay[q][i] = __builtin_amdgcn_fdot2(as_h2(q0[i]), as_h2(wb.z), ay[q][i], false);
                            ay[q][i] = __builtin_amdgcn_fdot2(as_h2(qp[i]), as_h2(wb.w), ay[q][i], false);
                            ay[q][i] = __builtin_amdgcn_fdot2(as_h2(ey[i]), as_h2(fbp), ay[q][i], false);
                        }
                    }
                }
                {
                    constexpr int dy = R;   // the last row, alone
                    uint32_t pm[RY], p0[RY], pp[RY];
#pragma unroll
                    for (int i = 0; i < RY; ++i) {
                        const uint32_t* r = cp + (i + R + dy) * G::WP;
                        pm[i] = r[0];
                        p0[i] = r[1];
                        pp[i] = r[2];
                    }
#pragma unroll
                    for (int dz = -R; dz <= R; ++dz) {
                        const int q = R - dz;
                        const int k = (dz + R) * Q + (dy + R);
                        // (w_-2, w_-1), (w_0, w_1), (w_-1, w_0), (w_1, w_2), w_2, w_-2
                        const uint4 wa = {tp.row[8 * k], tp.row[8 * k + 1], tp.row[8 * k + 2], tp.row[8 * k + 3]};
                        const float fa = __uint_as_float(tp.row[8 * k + 4]);
                        const float fb = __uint_as_float(tp.row[8 * k + 5]);
#pragma unroll
                        for (int i = 0; i < RY; ++i) {
                            ax[q][i] = __builtin_amdgcn_fdot2(as_h2(pm[i]), as_h2(wa.x), ax[q][i], false);
                            ax[q][i] = __builtin_amdgcn_fdot2(as_h2(p0[i]), as_h2(wa.y), ax[q][i], false);
                            ax[q][i] = fmaf(fa, (float)as_h2(pp[i]).x, ax[q][i]);
                            ay[q][i] = fmaf(fb, (float)as_h2(pm[i]).y, ay[q][i]);
                            ay[q][i] = __builtin_amdgcn_fdot2(as_h2(p0[i]), as_h2(wa.z), ay[q][i], false);
                            ay[q][i] = __builtin_amdgcn_fdot2(as_h2(pp[i]), as_h2(wa.w), ay[q][i], false);
                        }
                    }
                }
            }
            // The centre pairs of the thread's rows (for the residual term).
            uint32_t pc[RY];
#pragma unroll
            for (int i = 0; i < RY; ++i) pc[i] = cp[(i + R) * G::WP + 1];
            // The weight residuals, applied to the centre value.
            if constexpr (BC == kPeriodic) {
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    ax[R][i] = fmaf(tp.res, (float)as_h2(pc[i]).x, ax[R][i]);
                    ay[R][i] = fmaf(tp.res, (float)as_h2(pc[i]).y, ay[R][i]);
                }
            } else {
                const bool zface = zp < R || zp > nz - 1 - R;   // uniform over the workgroup
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    float ra = ria[i], rb = rib[i];
                    if (zface) {
                        const int cy = y0 + ty * RY + i;
                        ra = h2_inner_res<R>(rrs, 2 * gx, cy, zp, 2 * nxp, ny, nz, false);
                        rb = h2_inner_res<R>(rrs, 2 * gx + 1, cy, zp, 2 * nxp, ny, nz, false);
                    }
                    ax[R][i] = fmaf(ra, (float)as_h2(pc[i]).x, ax[R][i]);
                    ay[R][i] = fmaf(rb, (float)as_h2(pc[i]).y, ay[R][i]);
                }
            }

            // Output plane zp - R has received all 2R + 1 planes.
            const int zo = zp - R;
            if (zo >= z0 && zo < z1 && gx < nxp) {
                char* o = reinterpret_cast<char*>(out + (size_t)zo * plane_sz);
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    const int gy = y0 + ty * RY + i;
                    if (gy < ny) {
                        half2_t h;
                        h.x = (_Float16)ax[0][i];   // round to nearest even
                        h.y = (_Float16)ay[0][i];
                        __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, h),
                                                    reinterpret_cast<uint32_t*>(o + (uint32_t)(gy * nxp + gx) * 4u));
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < Q - 1; ++q)
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    ax[q][i] = ax[q + 1][i];
                    ay[q][i] = ay[q + 1][i];
                }
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                ax[Q - 1][i] = 0.f;
                ay[Q - 1][i] = 0.f;
            }
        }
    }
}

bool zm3d_h2_supported(const Geom& g) {
    const bool shape_ok = g.shape == kBox ? (g.r == 1 || g.r == 2) : g.r == 1;
    return g.ndim == 3 && shape_ok && g.dtype == 1 && g.nx % 2 == 0;
}

// The 7-point star's weights (centre, then the x, y and z arms) placed in
// the dense (dz, dy, dx) layout of the radius-1 box, zero off the axes.
static Taps star_as_box(const Taps& t) {
    Taps b;
    memset(&b, 0, sizeof b);
    auto at = [](int dz, int dy, int dx) { return ((dz + 1) * 3 + (dy + 1)) * 3 + (dx + 1); };
    b.c[at(0, 0, 0)] = t.c[0];
    for (int d = -1; d <= 1; d += 2) {
        b.c[at(0, 0, d)] = t.c[star_x<1>(d)];
        b.c[at(0, d, 0)] = t.c[star_y<1>(d)];
        b.c[at(d, 0, 0)] = t.c[star_z<1>(d)];
    }
    b.sum = t.sum;
    return b;
}

// Host-side weight preparation (dense (dz,dy,dx) box weights, f32).
static H2Taps pack_h2(const Taps& t) {
    H2Taps h;
    double res = 0.0;
    auto hi = [](float w) { return (_Float16)w; };
    for (int k = 0; k < 9; ++k) {
        const float wm = t.c[k * 3 + 0], w0 = t.c[k * 3 + 1], wp = t.c[k * 3 + 2];
        const _Float16 hm = hi(wm), h0 = hi(w0), hp = hi(wp);
        half2_t a, c;
        a.x = h0; a.y = hp;
        c.x = hm; c.y = h0;
        h.p01[k] = __builtin_bit_cast(uint32_t, a);
        h.pm0[k] = __builtin_bit_cast(uint32_t, c);
        h.wm[k] = (float)hm;
        h.wp[k] = (float)hp;
        const double rm = (double)wm - (double)(float)hm, r0 = (double)w0 - (double)(float)h0,
                     rp = (double)wp - (double)(float)hp;
        h.rr[k * 3 + 0] = (float)rm;
        h.rr[k * 3 + 1] = (float)r0;
        h.rr[k * 3 + 2] = (float)rp;
        res += rm + r0 + rp;
    }
    for (int z = 0; z < 3; ++z) {   // rows k = 3z + (dy + 1)
        half2_t a, c;
        a.x = hi(t.c[(3 * z + 0) * 3 + 0]);   // w_-1 of dy = -1
        a.y = hi(t.c[(3 * z + 1) * 3 + 0]);   // w_-1 of dy = 0
        c.x = hi(t.c[(3 * z + 1) * 3 + 2]);   // w_1 of dy = 0
        c.y = hi(t.c[(3 * z + 2) * 3 + 2]);   // w_1 of dy = 1
        h.wmp[z] = __builtin_bit_cast(uint32_t, a);
        h.wpp[z] = __builtin_bit_cast(uint32_t, c);
    }
    h.res = (float)res;
    return h;
}

// Radius 2: the 25 weight rows as binary16 pairs plus the two end weights,
// and the residuals (dense (dz,dy,dx) box weights, f32).
static H2Taps5 pack_h2_r2(const Taps& t) {
    H2Taps5 h;
    memset(&h, 0, sizeof h);
    double res = 0.0;
    auto pk = [](_Float16 a, _Float16 b) {
        half2_t v;
        v.x = a;
        v.y = b;
        return __builtin_bit_cast(uint32_t, v);
    };
    for (int k = 0; k < 25; ++k) {
        _Float16 c[5];
        for (int dx = 0; dx < 5; ++dx) {
            const float w = t.c[k * 5 + dx];
            c[dx] = (_Float16)w;
            const double r = (double)w - (double)(float)c[dx];
            h.rr[k * 5 + dx] = (float)r;
            res += r;
        }
        h.row[8 * k + 0] = pk(c[0], c[1]);
        h.row[8 * k + 1] = pk(c[2], c[3]);
        h.row[8 * k + 2] = pk(c[1], c[2]);
        h.row[8 * k + 3] = pk(c[3], c[4]);
        const float fa = (float)c[4], fb = (float)c[0];
        memcpy(&h.row[8 * k + 4], &fa, 4);
        memcpy(&h.row[8 * k + 5], &fb, 4);
    }
    // Rows k, k + 1 with dy = -2, 0: their end weights w_2 and w_-2 as
    // binary16 pairs in the row's spare words 6 and 7.
    for (int k = 0; k < 25; ++k)
        if (k % 5 == 0 || k % 5 == 2) {
            h.row[8 * k + 6] = pk((_Float16)t.c[k * 5 + 4], (_Float16)t.c[(k + 1) * 5 + 4]);
            h.row[8 * k + 7] = pk((_Float16)t.c[k * 5 + 0], (_Float16)t.c[(k + 1) * 5 + 0]);
        }
    h.res = (float)res;
    return h;
}

template <int R, int SH, int BC, int RY, int NW>
static hipError_t go(const Geom& g, int zc, const H2TapsOf<R>& tp, const void* in, void* out, hipStream_t s) {
    using G = H2Geom<RY, NW, R>;
    const int nxp = g.nx / 2;
    const int tiles_x = (nxp + G::BXP - 1) / G::BXP, tiles_y = (g.ny + G::BY - 1) / G::BY;
    const int nchunks = (g.nz + zc - 1) / zc;
    constexpr int D = 2;
    hipLaunchKernelGGL((zm3d_h2_kernel<R, SH, BC, RY, NW, D>), dim3(tiles_x * tiles_y * nchunks), dim3(G::NT), 0, s,
                       (const uint32_t*)in, (uint32_t*)out, nxp, g.ny, g.nz, zc, tiles_x, tiles_y, tp);
    return hipGetLastError();
}

template <int R, int SH, int BC>
static hipError_t go_rows(const Geom& g, int rows, int zc, const H2TapsOf<R>& tp, const void* in, void* out,
                          hipStream_t s) {
    if (rows == 8) return go<R, SH, BC, 2, 4>(g, zc, tp, in, out, s);
    if (rows == 16) return go<R, SH, BC, 4, 4>(g, zc, tp, in, out, s);
    return go<R, SH, BC, 8, 4>(g, zc, tp, in, out, s);
}

// tile_y: 8, 16 or 32 rows per workgroup (4 waves of 2, 4 or 8 rows).
hipError_t launch_zm3d_h2(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in, void* out,
                          hipStream_t s) {
    if (!zm3d_h2_supported(g)) return hipErrorInvalidValue;
    const int zc = cfg.zchunk > 0 ? cfg.zchunk : g.nz;
    const int rows = cfg.tile_y >= 32 ? 32 : (cfg.tile_y >= 16 ? 16 : 8);
    if (g.r == 2) {
        const H2Taps5 tp = pack_h2_r2(taps);
        return g.boundary == kPeriodic ? go_rows<2, kBox, kPeriodic>(g, rows, zc, tp, in, out, s)
                                       : go_rows<2, kBox, kZero>(g, rows, zc, tp, in, out, s);
    }
    if (g.shape == kStar) {
        const H2Taps tp = pack_h2(star_as_box(taps));
        return g.boundary == kPeriodic ? go_rows<1, kStar, kPeriodic>(g, rows, zc, tp, in, out, s)
                                       : go_rows<1, kStar, kZero>(g, rows, zc, tp, in, out, s);
    }
    const H2Taps tp = pack_h2(taps);
    return g.boundary == kPeriodic ? go_rows<1, kBox, kPeriodic>(g, rows, zc, tp, in, out, s)
                                   : go_rows<1, kBox, kZero>(g, rows, zc, tp, in, out, s);
}

}  // namespace stk
