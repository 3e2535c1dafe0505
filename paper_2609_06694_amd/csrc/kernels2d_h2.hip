// 2D box sweep (radius 1 or 2) with fp16 storage, k fused steps per launch,
// by the row march of ym2d_run.h on packed-half dot products.
//
// Thread x of a window owns a pair of adjacent cells (one 32-bit pair of
// binary16 values), so a 256-thread window spans 512 columns and every LDS
// row ring stores pairs.  Each fused step computes a row pair from the three
// pairs around it in each of the 2R+1 rows of the level below: for a row of
// weights w_-R..w_R (binary16 roundings; their residuals' sum enters once
// on the centre value, as in the 3D packed-half kernel)
//   radius 1: out(x)   = dot2((u_x, u_x+1), (w_0, w_1))  + w_-1 u_x-1,
//             out(x+1) = dot2((u_x, u_x+1), (w_-1, w_0)) + w_1 u_x+2;
//   radius 2: out(x)   = dot2((u_x-2, u_x-1), (w_-2, w_-1)) + dot2((u_x, u_x+1), (w_0, w_1)) + w_2 u_x+2,
//             out(x+1) = w_-2 u_x-1 + dot2((u_x, u_x+1), (w_-1, w_0)) + dot2((u_x+2, u_x+3), (w_1, w_2)),
// and at radius 2 the end terms w_2 u_x+2 and w_-2 u_x-1 of two adjacent
// rows share one dot2 on values paired by a v_perm: 13 instructions (15
// unpaired) for the 25 multiply-adds of a radius-2 cell.  The
// residuals w - w_hi enter as one multiply-add on the centre value, with
// their sum over the taps inside the grid (all taps under a periodic
// boundary; under a zero frame fewer at the edges).  A level
// stays valid one pair less on each side than the level below, so a window
// of NT pairs writes its NT - 2k middle pairs.  Every intermediate level is
// rounded to binary16 (the storage of one launch per step).  Requires an
// even nx.
#include <string.h>

#include <algorithm>

#include "internal.h"
#include "ym2d_run.h"

namespace stk {

typedef _Float16 h2v_t __attribute__((ext_vector_type(2)));

// Weights per row dy (index dy + R): radius 2: pa = (w_-2, w_-1),
// pb = (w_0, w_1), pc = (w_-1, w_0), pd = (w_1, w_2), fa = w_2, fb = w_-2;
// radius 1: pb = (w_0, w_1), pc = (w_-1, w_0), fa = w_-1, fb = w_1.
// res: the sum of the residuals w - w_hi; rr: each residual, (dy, dx)
// row-major over (2R+1)^2 (the zero frame sums only the taps inside).
struct H2Taps2 {
    uint32_t pa[5], pb[5], pc[5], pd[5];
    float fa[5], fb[5];
    // Radius 2: (w_2 of rows t, t+1) and (w_-2 of rows t, t+1) as binary16
    // pairs, t = 0..3, so two end terms of a cell take one dot2.
    uint32_t fap[4], fbp[4];
    float res;
    float rr[25];
};

__device__ __forceinline__ h2v_t h2v(uint32_t v) { return __builtin_bit_cast(h2v_t, v); }

__device__ __forceinline__ uint32_t pack_rne(float a, float b) {
    h2v_t h;
    h.x = (_Float16)a;   // round to nearest even
    h.y = (_Float16)b;
    return __builtin_bit_cast(uint32_t, h);
}

template <int R, int BC, int NT, int RY, int D>
__global__ __launch_bounds__(NT) void ym2d_h2_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                     int nxp, int ny, int k, int ow, int ych, int strips, H2Taps2 tp) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    uint32_t* lds = reinterpret_cast<uint32_t*>(lds_raw);
    constexpr int C = ym2d_ring_rows(RY, R);   // ring rows per level
    constexpr int U = C / RY;                  // iterations per ring period
    constexpr int NRD = RY + 2 * R;            // rows a stage reads from the level below
    constexpr int RW = NT + 2;                 // one pad pair on each side
    static_assert(U % D == 0, "the prefetch slots must repeat with the ring");
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int si = b % strips, ci = b / strips;
    const int x = threadIdx.x;
    const int kr = k * R;                       // halo rows of a chunk
    const int wx0 = si * ow - k;                // window origin pair (one halo pair per level and side)
    const int oy0 = ci * ych, oy1 = min(oy0 + ych, ny);
    const int Y = oy0 - kr;                     // first level-0 row of the march
    const int iters = (oy1 - oy0 + 2 * kr + RY - 1) / RY;

    int gxl = wx0 + x;
    const bool colin = ym_fix<BC>(gxl, nxp);
    const int gx = wx0 + x;                     // unclamped pair column
    const bool out_col = x >= k && x < k + ow && gx < nxp;

    // Residual weight on the centre value of each cell of the pair.  Under a
    // zero frame the taps that leave the grid read zero, not the centre
    // value, so the residual sum counts only the taps inside: rxa/rxb hold,
    // per row offset dy, the residuals of the in-grid x taps of the two
    // cells; rows within R of the top or bottom add only their in-grid dy.
    constexpr int W = 2 * R + 1;
    float rxa[W], rxb[W];
    float ria = tp.res, rib = tp.res;
    if constexpr (BC == kZero) {
        const int ca = 2 * gx, cb = ca + 1, ncx = 2 * nxp;
        ria = rib = 0.f;
#pragma unroll
        for (int t = 0; t < W; ++t) {
            rxa[t] = rxb[t] = 0.f;
#pragma unroll
            for (int dx = -R; dx <= R; ++dx) {
                const float w = tp.rr[t * W + dx + R];
                rxa[t] += (unsigned)(ca + dx) < (unsigned)ncx ? w : 0.f;
                rxb[t] += (unsigned)(cb + dx) < (unsigned)ncx ? w : 0.f;
            }
            ria += rxa[t];
            rib += rxb[t];
        }
    }

    uint32_t v[D][RY];
    uint32_t vm[D];
    auto issue = [&](int slot, int it) {
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            int gy = Y + it * RY + j;
            const bool ok = ym_fix<BC>(gy, ny) && colin;
            v[slot][j] = in[(size_t)gy * nxp + gxl];
            m |= (uint32_t)ok << j;
        }
        vm[slot] = m;
    };
#pragma unroll
    for (int d = 0; d < D; ++d) issue(d, d);

    for (int i0 = 0;; i0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            if (i >= iters) return;   // uniform: the whole workgroup leaves together
            const int d = u % D;
            const int base = ((u * RY - 2 * R) % C + C) % C;
            {
#pragma unroll
                for (int j = 0; j < RY; ++j) {
                    int q = base + 2 * R + j;
                    q = q >= C ? q - C : q;
                    lds[q * RW + 1 + x] = (BC == kPeriodic || ((vm[d] >> j) & 1u)) ? v[d][j] : 0u;
                }
            }
            issue(d, i + D);
            __syncthreads();

            for (int s = 1; s <= k; ++s) {
                const uint32_t* src = lds + (s - 1) * (C * RW);
                uint32_t pm[NRD], p0[NRD], pp[NRD];
#pragma unroll
                for (int j = 0; j < NRD; ++j) {
                    int q = base + j;
                    q = q >= C ? q - C : q;
                    pm[j] = src[q * RW + x];
                    p0[j] = src[q * RW + x + 1];
                    pp[j] = src[q * RW + x + 2];
                }
                const int y0 = Y + i * RY - s * R;   // global row of ax[0]
                float ax[RY], ay[RY];
#pragma unroll
                for (int j = 0; j < RY; ++j) {
                    float ra = ria, rb = rib;
                    if constexpr (BC == kZero) {
                        const int y = y0 + j;
                        if (y < R || y >= ny - R) {   // uniform over the workgroup
                            ra = rb = 0.f;
#pragma unroll
                            for (int t = 0; t < W; ++t)
                                if ((unsigned)(y + t - R) < (unsigned)ny) {
                                    ra += rxa[t];
                                    rb += rxb[t];
                                }
                        }
                    }
                    ax[j] = ra * (float)h2v(p0[j + R]).x;
                    ay[j] = rb * (float)h2v(p0[j + R]).y;
                }
#pragma unroll
                for (int dy = -R; dy <= R; ++dy) {
                    const int t = dy + R;
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        const int r = j + R + dy;
                        if constexpr (R == 1) {
                            ax[j] = __builtin_amdgcn_fdot2(h2v(p0[r]), h2v(tp.pb[t]), ax[j], false);
                            ax[j] = fmaf(tp.fa[t], (float)h2v(pm[r]).y, ax[j]);
                            ay[j] = __builtin_amdgcn_fdot2(h2v(p0[r]), h2v(tp.pc[t]), ay[j], false);
                            ay[j] = fmaf(tp.fb[t], (float)h2v(pp[r]).x, ay[j]);
                        } else {
                            ax[j] = __builtin_amdgcn_fdot2(h2v(pm[r]), h2v(tp.pa[t]), ax[j], false);
                            ax[j] = __builtin_amdgcn_fdot2(h2v(p0[r]), h2v(tp.pb[t]), ax[j], false);
                            ay[j] = __builtin_amdgcn_fdot2(h2v(p0[r]), h2v(tp.pc[t]), ay[j], false);
                            ay[j] = __builtin_amdgcn_fdot2(h2v(pp[r]), h2v(tp.pd[t]), ay[j], false);
                        }
                    }
                }
                if constexpr (R == 2) {
                    // The end terms w_2 u_x+2 (out x) and w_-2 u_x-1 (out x+1)
                    // of rows r, r+1 (r even) share one dot2: the value pairs
                    // come from one v_perm each; a row j takes the pairs that
                    // start at its even rows and one end term alone.
                    uint32_t ex[NRD / 2], ey[NRD / 2];
#pragma unroll
                    for (int h = 0; h < NRD / 2; ++h) {
                        ex[h] = __builtin_amdgcn_perm(pp[2 * h + 1], pp[2 * h], 0x05040100u);   // (u_x+2 of 2h, 2h+1)
                        ey[h] = __builtin_amdgcn_perm(pm[2 * h + 1], pm[2 * h], 0x07060302u);   // (u_x-1 of 2h, 2h+1)
                    }
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        if (j % 2 == 0) {   // rows j, j+1 | j+2, j+3 | j+4
                            ax[j] = __builtin_amdgcn_fdot2(h2v(ex[j / 2]), h2v(tp.fap[0]), ax[j], false);
                            ax[j] = __builtin_amdgcn_fdot2(h2v(ex[j / 2 + 1]), h2v(tp.fap[2]), ax[j], false);
                            ax[j] = fmaf(tp.fa[4], (float)h2v(pp[j + 4]).x, ax[j]);
                            ay[j] = __builtin_amdgcn_fdot2(h2v(ey[j / 2]), h2v(tp.fbp[0]), ay[j], false);
                            ay[j] = __builtin_amdgcn_fdot2(h2v(ey[j / 2 + 1]), h2v(tp.fbp[2]), ay[j], false);
                            ay[j] = fmaf(tp.fb[4], (float)h2v(pm[j + 4]).y, ay[j]);
                        } else {            // row j | j+1, j+2 | j+3, j+4
                            ax[j] = fmaf(tp.fa[0], (float)h2v(pp[j]).x, ax[j]);
                            ax[j] = __builtin_amdgcn_fdot2(h2v(ex[(j + 1) / 2]), h2v(tp.fap[1]), ax[j], false);
                            ax[j] = __builtin_amdgcn_fdot2(h2v(ex[(j + 3) / 2]), h2v(tp.fap[3]), ax[j], false);
                            ay[j] = fmaf(tp.fb[0], (float)h2v(pm[j]).y, ay[j]);
                            ay[j] = __builtin_amdgcn_fdot2(h2v(ey[(j + 1) / 2]), h2v(tp.fbp[1]), ay[j], false);
                            ay[j] = __builtin_amdgcn_fdot2(h2v(ey[(j + 3) / 2]), h2v(tp.fbp[3]), ay[j], false);
                        }
                    }
                }
                if (s < k) {
                    uint32_t* dst = lds + s * (C * RW);
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        int q = base + 2 * R + j;
                        q = q >= C ? q - C : q;
                        uint32_t val = pack_rne(ax[j], ay[j]);
                        if (BC == kZero) {
                            const int gy = y0 + j;
                            if (gx < 0 || gx >= nxp || gy < 0 || gy >= ny) val = 0u;
                        }
                        dst[q * RW + 1 + x] = val;
                    }
                    __syncthreads();
                } else if (out_col) {
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        const int gy = y0 + j;
                        if (gy >= oy0 && gy < oy1)
                            __builtin_nontemporal_store(pack_rne(ax[j], ay[j]), &out[(size_t)gy * nxp + gx]);
                    }
                }
            }
            if (k == 1) __syncthreads();
        }
    }
}

bool ym2d_h2_supported(const Geom& g) {
    return g.ndim == 2 && g.shape == kBox && (g.r == 1 || g.r == 2) && g.dtype == 1 && g.nx % 2 == 0;
}

static H2Taps2 pack_h2_2d(const Taps& t, int R) {
    H2Taps2 h;
    memset(&h, 0, sizeof h);
    const int w = 2 * R + 1;
    double res = 0.0;
    auto pk = [](_Float16 a, _Float16 b) {
        h2v_t v;
        v.x = a;
        v.y = b;
        return __builtin_bit_cast(uint32_t, v);
    };
    for (int dy = -R; dy <= R; ++dy) {
        const int tix = dy + R;
        _Float16 c[5];
        for (int dx = -R; dx <= R; ++dx) {
            const float wf = t.c[(dy + R) * w + (dx + R)];
            c[dx + R] = (_Float16)wf;
            const double r = (double)wf - (double)(float)c[dx + R];
            h.rr[tix * w + dx + R] = (float)r;
            res += r;
        }
        if (R == 1) {
            h.pb[tix] = pk(c[1], c[2]);
            h.pc[tix] = pk(c[0], c[1]);
            h.fa[tix] = (float)c[0];
            h.fb[tix] = (float)c[2];
        } else {
            h.pa[tix] = pk(c[0], c[1]);
            h.pb[tix] = pk(c[2], c[3]);
            h.pc[tix] = pk(c[1], c[2]);
            h.pd[tix] = pk(c[3], c[4]);
            h.fa[tix] = (float)c[4];
            h.fb[tix] = (float)c[0];
        }
    }
    if (R == 2)
        for (int r = 0; r < 4; ++r) {   // rows r and r + 1
            const _Float16 a0 = (_Float16)t.c[r * w + 4], a1 = (_Float16)t.c[(r + 1) * w + 4];
            const _Float16 b0 = (_Float16)t.c[r * w + 0], b1 = (_Float16)t.c[(r + 1) * w + 0];
            h.fap[r] = pk(a0, a1);
            h.fbp[r] = pk(b0, b1);
        }
    h.res = (float)res;
    return h;
}

// LDS bytes of a launch: k rings of ym2d_ring_rows(RY, R) rows of NT + 2 pairs.
static int h2_rows(int nt, int k, int R) {
    return 4 * k * ym2d_ring_rows(8, R) * (nt + 2) <= 64 * 1024 ? 8 : 4;
}
int ym2d_h2_lds_bytes(int nt, int k, int R) { return 4 * k * ym2d_ring_rows(h2_rows(nt, k, R), R) * (nt + 2); }

template <int R, int BC, int NT, int RY>
static hipError_t go(const Geom& g, int k, int ych, const H2Taps2& tp, const void* in, void* out, hipStream_t s) {
    constexpr int D = 2;
    const int nxp = g.nx / 2;
    const int ow = NT - 2 * k;
    const int strips = (nxp + ow - 1) / ow;
    const int chunks = (g.ny + ych - 1) / ych;
    const size_t lds = 4 * (size_t)k * ym2d_ring_rows(RY, R) * (NT + 2);
    if (lds > 64 * 1024) {
        hipError_t e = allow_large_lds<ym2d_h2_kernel<R, BC, NT, RY, D>>();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((ym2d_h2_kernel<R, BC, NT, RY, D>), dim3(strips * chunks), dim3(NT), lds, s,
                       (const uint32_t*)in, (uint32_t*)out, nxp, g.ny, k, ow, ych, strips, tp);
    return hipGetLastError();
}

template <int R, int BC, int NT>
static hipError_t go_ry(const Geom& g, int k, int ych, const H2Taps2& tp, const void* in, void* out,
                        hipStream_t s) {
    if (h2_rows(NT, k, R) == 8) return go<R, BC, NT, 8>(g, k, ych, tp, in, out, s);
    return go<R, BC, NT, 4>(g, k, ych, tp, in, out, s);
}

template <int R, int BC>
static hipError_t go_nt(const Geom& g, int nt, int k, int ych, const H2Taps2& tp, const void* in, void* out,
                        hipStream_t s) {
    if (nt == 512) return go_ry<R, BC, 512>(g, k, ych, tp, in, out, s);
    return go_ry<R, BC, 256>(g, k, ych, tp, in, out, s);
}

// Rows per chunk when left open: about four workgroups per CU, chunks of
// at least 4kR rows.
static int auto_chunk(const Geom& g, int nt, int k) {
    const int ow = nt - 2 * k;
    const int strips = (g.nx / 2 + ow - 1) / ow;
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) cus = n;
    }
    const int target = 4 * cus;
    const int chunks = std::max(1, target / std::max(1, strips));
    int ych = (g.ny + chunks - 1) / chunks;
    ych = std::max(ych, std::max(16, 4 * k * g.r));
    return std::min(ych, g.ny);
}

// cfg.tile_x: threads per window (256 or 512: 512 or 1024 columns);
// cfg.tile_y: rows per chunk (0: automatic); k fused steps.
hipError_t launch_ym2d_h2(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in, void* out,
                          int k, hipStream_t s) {
    if (!ym2d_h2_supported(g)) return hipErrorInvalidValue;
    const int nt = cfg.tile_x == 512 ? 512 : 256;
    if (k < 1 || k > 16 || nt - 2 * k < kWave || ym2d_h2_lds_bytes(nt, k, g.r) > ym2d_max_lds_bytes())
        return hipErrorInvalidValue;
    const H2Taps2 tp = pack_h2_2d(taps, g.r);
    const int ych = cfg.tile_y > 0 ? std::min(cfg.tile_y, g.ny)
                                   : ym2d_fill_chunk(auto_chunk(g, nt, k), k * g.r, h2_rows(nt, k, g.r), g.ny);
    if (g.r == 1)
        return g.boundary == kPeriodic ? go_nt<1, kPeriodic>(g, nt, k, ych, tp, in, out, s)
                                       : go_nt<1, kZero>(g, nt, k, ych, tp, in, out, s);
    return g.boundary == kPeriodic ? go_nt<2, kPeriodic>(g, nt, k, ych, tp, in, out, s)
                                   : go_nt<2, kZero>(g, nt, k, ych, tp, in, out, s);
}

}  // namespace stk
