// 2D linear sweep, k time steps per launch, by a row march (y-march).
//
// A workgroup of NT threads owns a window of NT columns and marches down a
// chunk of rows.  Thread x keeps window column x.  Each iteration brings RY
// new input rows (time level 0) into an LDS row ring; then, one stage per
// fused step s = 1..k, it computes RY rows of level s from the ring of level
// s-1, R rows behind the rows that level s-1 just produced, and puts them in
// the ring of level s (the last stage writes them to HBM).  Intermediate
// time levels never leave the chip (temporal blocking, Section 4.3), and
// because rows stream, the redundant halo computation of a fused step is
// paid in x only: level s is valid on window columns [sR, NT - sR), so the
// NT - 2kR middle columns are the workgroup's outputs.  A chunk of rows
// re-reads and recomputes kR rows above and below it.
//
// Each level's ring holds C rows, C = RY * 2^m >= RY + 2R: stage s+1 reads
// the RY + 2R newest rows of level s, and the next iteration overwrites the
// RY oldest ones only after the barrier that follows stage s+1 (for k = 1 an
// extra barrier closes every iteration).  Because C is a multiple of RY, the
// ring position of an iteration repeats every C / RY iterations; the march
// is unrolled by that period, so every ring slot is a compile-time constant
// and each LDS access is a fixed offset from one per-thread address.  Rows of a level above its first valid
// row (Y + sR) are computed from rows not yet loaded; they feed only other
// such rows and are never written out.
//
// Input rows are loaded D iterations ahead into registers, every load
// unconditional (coordinates clamped or wrapped; cells outside a zero frame
// are masked when staged), so the compiler keeps all of them in flight.
// fp16 storage: every intermediate level is rounded to binary16, exactly as
// one launch per step would store it; arithmetic is FP32.  Zero frame: cells
// outside the grid are zero at every level.
#pragma once

#include <type_traits>

#include "common.h"

namespace stk {

// Ring rows per level: the smallest RY * 2^m that holds RY + 2R rows.
__host__ __device__ constexpr int ym2d_ring_rows(int RY, int R) {
    int c = RY;
    while (c < RY + 2 * R) c *= 2;
    return c;
}

// A chunk of ych output rows marches ych + 2kR input rows in iterations of
// ry rows; an automatic chunk is lengthened to fill its last iteration (the
// rows past the chunk are computed either way).
inline int ym2d_fill_chunk(int ych, int kr, int ry, int ny) {
    const int rows = (ych + 2 * kr + ry - 1) / ry * ry;
    return rows - 2 * kr < ny ? rows - 2 * kr : ny;
}

template <int BC>
__device__ __forceinline__ bool ym_fix(int& i, int n) {
    if (BC == kPeriodic) {
        i = wrap_index(i, n);
        return true;
    }
    const bool ok = (unsigned)i < (unsigned)n;
    i = min(max(i, 0), n - 1);
    return ok;
}

// One workgroup's chunk: window strip b % strips, row chunk b / strips.
// The window geometry (output width ow = NT - 2 kgeo R, halo rows) is laid
// out for kgeo fused steps; klev <= kgeo levels are computed (a final,
// shorter time block keeps the geometry of the others).  `lds` holds
// klev rings of ym2d_ring_rows(RY, R) x (NT + 2R) values of the arithmetic type.  Called by all NT
// threads.
template <int R, int SHAPE, typename T, int BC, int NT, int RY, int D>
__device__ void ym2d_run(const T* __restrict__ in, T* __restrict__ out, int nx, int ny, int kgeo,
                         int klev, int ow, int ych, int strips, int b, const Taps& tp,
                         acc_t<T>* __restrict__ lds) {
    using A = acc_t<T>;   // arithmetic type (f64 for f64 storage, else f32)
    constexpr int C = ym2d_ring_rows(RY, R);   // ring rows per level
    constexpr int U = C / RY;                  // iterations per ring period
    constexpr int NRD = RY + 2 * R;            // rows a stage reads from the level below
    static_assert(U % D == 0, "the prefetch slots must repeat with the ring");
    constexpr int RW = NT + 2 * R;      // ring row width: R pad columns on each side
    const int k = klev;
    const int si = b % strips, ci = b / strips;
    const int x = threadIdx.x;
    const int kr = kgeo * R;
    const int wx0 = si * ow - kr;                 // window origin column
    const int oy0 = ci * ych, oy1 = min(oy0 + ych, ny);
    const int Y = oy0 - kr;                       // first level-0 row of the march
    const int iters = (oy1 - oy0 + 2 * kr + RY - 1) / RY;

    // This thread's column: load address (wrapped or clamped) and validity.
    int gxl = wx0 + x;
    const bool colin = ym_fix<BC>(gxl, nx);
    const int gx = wx0 + x;                        // unclamped grid column
    const bool out_col = x >= kr && x < kr + ow && gx < nx;

    T v[D][RY];
    uint32_t vm[D];
    auto issue = [&](int slot, int it) {
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            int gy = Y + it * RY + j;
            const bool ok = ym_fix<BC>(gy, ny) && colin;
            v[slot][j] = in[(size_t)gy * nx + gxl];
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
            // Ring offset of this iteration (a constant: i0 is a multiple of
            // the period U): stage s+1 reads level-s slots base+2R-(RY+2R)
            // .. base+2R+RY-1, stage s writes base+2R+j (all mod C).
            const int base = ((u * RY - 2 * R) % C + C) % C;

            // Stage 0: stage the input rows of this iteration in ring 0.
            {
                A* r0 = lds;
#pragma unroll
                for (int j = 0; j < RY; ++j) {
                    int q = base + 2 * R + j;
                    q = q >= C ? q - C : q;
                    const A val = to_acc<T>(v[d][j]);
                    r0[q * RW + R + x] = (BC == kPeriodic || ((vm[d] >> j) & 1u)) ? val : A(0);
                }
            }
            issue(d, i + D);
            __syncthreads();

            for (int s = 1; s <= k; ++s) {
                const A* src = lds + (s - 1) * (C * RW);
                A acc[RY];
                if constexpr (SHAPE == kBox) {
#pragma unroll
                    for (int j = 0; j < RY; ++j) acc[j] = A(0);
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        A col[NRD];
#pragma unroll
                        for (int j = 0; j < NRD; ++j) {
                            int q = base + j;
                            q = q >= C ? q - C : q;
                            col[j] = src[q * RW + R + x + dx];
                        }
                        // This column's weights in vector registers (f32: a
                        // multiply-add with all operands in vector registers
                        // issues faster than one taking a scalar register).
                        A w[2 * R + 1];
#pragma unroll
                        for (int dy = -R; dy <= R; ++dy) {
                            w[dy + R] = A(tp.c[box2<R>(dy, dx)]);
                            if constexpr (std::is_same_v<A, float>) asm volatile("" : "+v"(w[dy + R]));
                        }
#pragma unroll
                        for (int j = 0; j < RY; ++j)
#pragma unroll
                            for (int dy = -R; dy <= R; ++dy)
                                acc[j] = fma_acc(w[dy + R], col[j + R + dy], acc[j]);
                    }
                } else {
                    A col[NRD];
#pragma unroll
                    for (int j = 0; j < NRD; ++j) {
                        int q = base + j;
                        q = q >= C ? q - C : q;
                        col[j] = src[q * RW + R + x];
                    }
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        A a = A(tp.c[0]) * col[j + R];
#pragma unroll
                        for (int e = 1; e <= R; ++e) {
                            a = fma_acc(A(tp.c[star_y<R>(-e)]), col[j + R - e], a);
                            a = fma_acc(A(tp.c[star_y<R>(e)]), col[j + R + e], a);
                        }
                        acc[j] = a;
                    }
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        int q = base + R + j;
                        q = q >= C ? q - C : q;
                        const A* row = src + q * RW + R + x;
#pragma unroll
                        for (int e = 1; e <= R; ++e) {
                            acc[j] = fma_acc(A(tp.c[star_x<R>(-e)]), row[-e], acc[j]);
                            acc[j] = fma_acc(A(tp.c[star_x<R>(e)]), row[e], acc[j]);
                        }
                    }
                }
                const int y0 = Y + i * RY - s * R;   // global row of acc[0]
                if (s < k) {
                    A* dst = lds + s * (C * RW);
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        int q = base + 2 * R + j;
                        q = q >= C ? q - C : q;
                        A val = to_acc<T>(from_acc<T>(acc[j]));   // storage rounding
                        if (BC == kZero) {
                            const int gy = y0 + j;
                            if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) val = A(0);
                        }
                        dst[q * RW + R + x] = val;
                    }
                    __syncthreads();
                } else if (out_col) {
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        const int gy = y0 + j;
                        if (gy >= oy0 && gy < oy1)
                            __builtin_nontemporal_store(from_acc<T>(acc[j]), &out[(size_t)gy * nx + gx]);
                    }
                }
            }
            if (k == 1) __syncthreads();
        }
    }
}

}  // namespace stk
