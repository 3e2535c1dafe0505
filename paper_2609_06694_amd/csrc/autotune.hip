// Autotuner: fills the dispatch map by measurement.
//
// Numeric parameter sweeps run as a deterministic program outside the kernel
// code (Section 4.3).  For each distinct case of a plan the legal candidates
// (tile shape, fused time steps, rows per workgroup, plane chunk) are each
// checked against the plain single-step configuration on a probe grid; a
// candidate whose output differs is rejected before it is timed (an
// incorrect-but-faster result must never win, Section 6.2's correctness gate).
// Survivors are timed with HIP events (median of five) on the real extent and
// the fastest is written into the plan and the dispatch map.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "plan.h"

namespace stk {

__device__ __forceinline__ float hash_unit(uint32_t i, uint32_t seed) {
    uint32_t h = i * 0x9E3779B1u ^ (seed * 0x85EBCA77u + 0x165667B1u);
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return (float)(h >> 8) * (1.0f / 16777216.0f);
}

template <typename T>
__global__ void fill_random(T* p, size_t n, uint32_t seed, float lo, float hi) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = from_acc<T>(lo + (hi - lo) * hash_unit((uint32_t)i, seed));
}

// out[0] = max |a - b|, out[1] = max |b|, as f32 bit patterns (non-negative
// floats order like unsigned integers); differences are formed in the
// arithmetic type and rounded up to f32 at the end.
template <typename T>
__global__ void max_diff(const T* a, const T* b, size_t n, unsigned* out) {
    using A = acc_t<T>;
    A d = 0, m = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const A x = to_acc<T>(a[i]), y = to_acc<T>(b[i]);
        const A e = x > y ? x - y : y - x;
        d = (e > d || e != e) ? (e != e ? A(INFINITY) : e) : d;
        m = fmax(m, y < 0 ? -y : y);
    }
    float df = (float)d, mf = (float)m;
    if ((A)df < d) df = nextafterf(df, INFINITY);
    atomicMax(&out[0], __float_as_uint(df));
    atomicMax(&out[1], __float_as_uint(mf));
}

// Per-dtype launch of max_diff.
void launch_max_diff(int dtype, const void* a, const void* b, size_t n, unsigned* out, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<size_t>(4096, (n + 255) / 256);
    if (dtype == ST_F16)
        hipLaunchKernelGGL(max_diff<_Float16>, dim3(blocks), dim3(256), 0, s, (const _Float16*)a,
                           (const _Float16*)b, n, out);
    else if (dtype == ST_F64)
        hipLaunchKernelGGL(max_diff<double>, dim3(blocks), dim3(256), 0, s, (const double*)a, (const double*)b,
                           n, out);
    else
        hipLaunchKernelGGL(max_diff<float>, dim3(blocks), dim3(256), 0, s, (const float*)a, (const float*)b, n,
                           out);
}

// Relative tolerance of a candidate against the plain kernel, by dtype.
float parity_tol(int dtype) { return dtype == ST_F16 ? 2e-3f : (dtype == ST_F64 ? 1e-10f : 1e-5f); }

__global__ void zero_u32(unsigned* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

}  // namespace stk

using namespace stk;

namespace {

struct TuneStats {
    int tried = 0, rejected = 0;
};

size_t esize(int dtype) { return dtype == ST_F16 ? 2 : (dtype == ST_F64 ? 8 : 4); }

size_t grid_bytes_of(const st_problem& p) { return (size_t)p.n[0] * p.n[1] * p.n[2] * esize(p.dtype); }

hipError_t fill(void* p, const st_problem& pr, size_t cells, uint32_t seed, float lo, float hi,
                hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<size_t>(8192, (cells + 255) / 256);
    if (pr.dtype == ST_F16)
        hipLaunchKernelGGL(fill_random<_Float16>, dim3(blocks), dim3(256), 0, s, (_Float16*)p, cells, seed, lo, hi);
    else if (pr.dtype == ST_F64)
        hipLaunchKernelGGL(fill_random<double>, dim3(blocks), dim3(256), 0, s, (double*)p, cells, seed, lo, hi);
    else
        hipLaunchKernelGGL(fill_random<float>, dim3(blocks), dim3(256), 0, s, (float*)p, cells, seed, lo, hi);
    return hipGetLastError();
}

std::vector<LaunchCfg> candidates(const st_problem& p) {
    std::vector<LaunchCfg> out;
    if (p.update == ST_VARCOEF) {   // plane march: tile height and plane chunk
        for (int ty : {8, 16})
            for (int zc : {16, 32, 64, 128, 256, 0}) {
                if (zc != 0 && (p.ndim == 2 || zc >= p.n[2])) continue;
                LaunchCfg c{ST_VARIANT_VC3D, 0, ty, 1, zc};
                if (cfg_legal(p, c)) out.push_back(c);
            }
        return out;
    }
    if (p.update == ST_WAVE || p.ndim == 3) {
        std::vector<int> vars;
        // Forward wave candidates come from the difference-form (LDS ring)
        // family only: the direct weighted sum is faster by a few percent
        // but its f32 cancellation error, invisible over the short parity
        // probe, exceeds the 1e-5 gate after tens of steps.
        if (p.update == ST_WAVE) vars = {p.dtype == ST_F64 ? ST_VARIANT_WAVE3D : ST_VARIANT_WAVE3D_LDS};
        else vars = {ST_VARIANT_ZM3D};
        // Chunks of 8 planes only on small grids (up to 2^22 cells), where
        // they give enough workgroups to fill the chip.
        const bool small = (double)p.n[0] * p.n[1] * p.n[2] <= (double)(1 << 22);
        // Wave: one or two planes staged per barrier (tile_x 0 or 2).
        for (int var : vars)
            for (int pb : {0, 2})
                for (int ty : {8, 16, 32})
                    for (int zc : {8, 16, 32, 64, 128, 256, 0}) {
                        if (zc != 0 && zc >= p.n[2]) continue;
                        if (zc == 8 && !small) continue;
                        if (pb != 0 && p.update != ST_WAVE) continue;
                        LaunchCfg c{var, pb, ty, 1, zc};
                        if (cfg_legal(p, c)) out.push_back(c);
                    }
        // Two fused steps (radius 1: 62 x (tile_y - 2) output tiles).
        for (int ty : {16, 32})
            for (int zc : {8, 16, 32, 64, 128, 0}) {
                if (zc != 0 && zc >= p.n[2]) continue;
                if (zc == 8 && !small) continue;
                LaunchCfg c{ST_VARIANT_ZM3D, 0, ty, 2, zc};
                if (cfg_legal(p, c)) out.push_back(c);
            }
        // Packed-half form of the fp16 boxes and 7-point star (two cells per lane).
        for (int ty : {8, 16, 32})
            for (int zc : {8, 16, 32, 64, 128, 256, 0}) {
                if (zc != 0 && zc >= p.n[2]) continue;
                if (zc == 8 && !small) continue;
                LaunchCfg c{ST_VARIANT_ZM3D_H2, 0, ty, 1, zc};
                if (cfg_legal(p, c)) out.push_back(c);
            }
        // The march along y, where z is shorter than y.
        if (p.update == ST_LINEAR && p.n[2] < p.n[1])
            for (int ty : {8, 16, 32})
                for (int zc : {16, 32, 64, 128, 256, 0}) {
                    if (zc != 0 && zc >= p.n[1]) continue;
                    LaunchCfg c{ST_VARIANT_YM3D, 0, ty, 1, zc};
                    if (cfg_legal(p, c)) out.push_back(c);
                }
        // Matrix-core form of the fp16 27-point box (64 x 64 tiles).
        for (int zc : {16, 32, 64, 128, 0}) {
            if (zc != 0 && zc >= p.n[2]) continue;
            LaunchCfg c{ST_VARIANT_ZM3D_MFMA, 0, 64, 1, zc};
            if (cfg_legal(p, c)) out.push_back(c);
        }
        return out;
    }
    for (int tx : {64, 128, 256})
        for (int ty : {16, 32, 64})
            for (int k : {1, 2, 4, 8, 10, 16}) {
                if (tx > 2 * p.n[0] + 64 || ty > 2 * p.n[1] + 16) continue;
                LaunchCfg c{ST_VARIANT_TB2D, tx, ty, k, 0};
                if (cfg_legal(p, c)) out.push_back(c);
            }
    // Windows of 64 columns with their halo, one pass per fused step: 64 or
    // 32 rows run by 16 or 8 waves (small, latency-bound grids).
    for (int k : {1, 2, 4, 8, 10, 16})
        for (int h : {64, 32}) {
            const int bx = 64 - 2 * k * (int)p.radius, by = h - 2 * k * (int)p.radius;
            if (bx < 16 || by < 8 || bx > 2 * p.n[0] || by > 2 * p.n[1]) continue;
            LaunchCfg c{ST_VARIANT_TB2D, bx, by, k, h / 4};
            if (cfg_legal(p, c)) out.push_back(c);
        }
    // Packed-half row march (fp16 boxes, even nx).
    for (int nt : {256, 512})
        for (int k : {1, 2, 3, 4, 8})
            for (int ych : {0, 32, 64, 128}) {
                if (2 * nt > 2 * p.n[0] + 512 || (ych != 0 && ych >= p.n[1])) continue;
                LaunchCfg c{ST_VARIANT_YM2D_H2, nt, ych, k, 0};
                if (cfg_legal(p, c)) out.push_back(c);
            }
    // Row march: window width, fused depth, rows per chunk (0 = automatic).
    for (int nt : {256, 512})
        for (int k : {1, 2, 4, 8, 10, 16})
            for (int ych : {0, 32, 64, 128, 256}) {
                if (nt > 2 * p.n[0] + 256 || (ych != 0 && ych >= p.n[1])) continue;
                LaunchCfg c{ST_VARIANT_YM2D, nt, ych, k, 0};
                if (cfg_legal(p, c)) out.push_back(c);
            }
    return out;
}

// `steps` steps of configuration c (linear: ping-pong in/tmp ending in out;
// wave: forward leapfrog with prev = tmp).  Taps may be perturbed.  `aux` is
// kappa (wave) or the coefficient fields (variable coefficients).
hipError_t run_cfg(const st_problem& p, const st_plan* pl, const LaunchCfg& c, const Taps& taps,
                   const void* in, void* out, void* tmp, const void* aux, int steps,
                   hipStream_t s) {
    Geom g = plan_geom(pl);
    const float* kappa = (const float*)aux;
    if (p.update == ST_VARCOEF) {
        const void* cur = in;
        for (int j = 1; j <= steps; ++j) {
            void* dst = ((steps - j) % 2 == 0) ? out : tmp;
            hipError_t e = launch_vc3d(g, c, cur, dst, aux, false, s);
            if (e != hipSuccess) return e;
            cur = dst;
        }
        return hipSuccess;
    }
    if (p.update == ST_WAVE && p.dtype == ST_F64) {
        // FP64 leapfrog: its binary64 weights, with a planted fault carried
        // over from the perturbed f32 taps.
        TapsD t64 = pl->taps64;
        t64.c[0] += (double)taps.c[0] - (double)pl->taps.c[0];
        const double* prev = (const double*)tmp;
        const double* cur = (const double*)in;
        for (int t = 0; t < steps; ++t) {
            WaveLaunchF64 w;
            memset(&w, 0, sizeof w);
            w.src_x = -1;
            w.rec_z = -1;
            w.prev = prev;
            w.cur = cur;
            w.next = ((steps - t - 1) % 2 == 0) ? (double*)out : (double*)tmp;
            w.kappa = (const double*)aux;
            hipError_t e = launch_wave3d_f64(g, c, t64, w, s);
            if (e != hipSuccess) return e;
            prev = cur;
            cur = w.next;
        }
        return hipSuccess;
    }
    if (p.update == ST_WAVE) {
        const float* prev = (const float*)tmp;
        const float* cur = (const float*)in;
        for (int t = 0; t < steps; ++t) {
            WaveLaunch w;
            memset(&w, 0, sizeof w);
            w.src_x = -1;
            w.rec_z = -1;
            w.prev = prev;
            w.cur = cur;
            w.next = ((steps - t - 1) % 2 == 0) ? (float*)out : (float*)tmp;
            w.kappa = kappa;
            hipError_t e = c.variant == ST_VARIANT_WAVE3D_LDS ? launch_wave3d_ring(g, c, taps, w, s)
                                                              : launch_wave3d(g, c, taps, pl->taps, kWaveFwd, w, s);
            if (e != hipSuccess) return e;
            prev = cur;
            cur = w.next;
        }
        return hipSuccess;
    }
    const int k = p.ndim == 2 ? std::max(1, c.tsteps) : (c.tsteps == 2 ? 2 : 1);
    const int L = (steps + k - 1) / k;
    const void* cur = in;
    int done = 0;
    for (int j = 1; j <= L; ++j) {
        const int kj = std::min(k, steps - done);
        void* dst = ((L - j) % 2 == 0) ? out : tmp;
        hipError_t e = p.ndim == 2 ? launch_linear2d(g, c, taps, cur, dst, kj, s)
                                   : launch_linear3d(g, c, taps, cur, dst, kj, s);
        if (e != hipSuccess) return e;
        cur = dst;
        done += kj;
    }
    return hipSuccess;
}

bool faulty(const st_problem& p, const LaunchCfg& c) {
    const char* f = getenv("STENCIL_TUNE_FAULT");
    if (!f || f[0] != '1') return false;
    if (p.ndim == 2 && p.update == ST_LINEAR) return c.tsteps > 1;
    return c.tile_y == 16;
}

st_status tune_one(st_plan* pl, char* scratch, size_t bytes, hipStream_t s, TuneStats& st) {
    const st_problem& p = pl->prob;
    const size_t cells = (size_t)p.n[0] * p.n[1] * p.n[2];
    const size_t gb = (cells * esize(p.dtype) + 255) / 256 * 256;
    // Scratch: in, out, tmp, ref (each a full grid), kappa (wave) or the
    // coefficient fields (variable coefficients), 2 counters.
    const size_t kb = p.update == ST_WAVE ? gb : (p.update == ST_VARCOEF ? (size_t)(varcoef_taps(p) + 1) * gb : 0);
    if (bytes < 4 * gb + kb + 64) {
        set_error("autotune scratch of %zu bytes needed", 4 * gb + kb + 64);
        return ST_EWORKSPACE;
    }
    char* in = scratch;
    char* out = scratch + gb;
    char* tmp = scratch + 2 * gb;
    char* ref = scratch + 3 * gb;
    float* kappa = (float*)(scratch + 4 * gb);
    unsigned* cnt = (unsigned*)(scratch + 4 * gb + kb);
    // 2D probes run ten steps: depths that divide it need no remainder launch.
    const int steps = p.update == ST_WAVE ? 2 : (p.ndim == 2 ? 10 : 2);
    const float lo = p.update == ST_WAVE ? -1.f : 0.f;
#define T_TRY(e)                                                                         \
    do {                                                                                 \
        hipError_t e_ = (e);                                                             \
        if (e_ != hipSuccess) {                                                          \
            set_error("autotune: %s: %s", #e, hipGetErrorString(e_));                    \
            return ST_EHIP;                                                              \
        }                                                                                \
    } while (0)
    if (p.update == ST_WAVE) {
        st_problem kp = p;
        kp.dtype = p.dtype == ST_F64 ? ST_F64 : ST_F32;   // kappa in the storage type of the wave plan
        T_TRY(fill(kappa, kp, cells, 7u, 0.05f, 0.2f, s));
    }
    if (p.update == ST_VARCOEF) {   // fields near 1/taps: bounded repeated sweeps
        const int nt = varcoef_taps(p);
        for (int k = 0; k <= nt; ++k)   // one spare field for the planted fault
            T_TRY(fill((char*)kappa + (size_t)k * gb, p, cells, 11u + k, 0.f, 2.f / nt, s));
    }
    T_TRY(fill(in, p, cells, 1u, lo, 1.f, s));
    T_TRY(fill(tmp, p, cells, 2u, lo, 1.f, s));
    LaunchCfg plain = candidates(p).front();
    if (p.ndim == 2 && p.update == ST_LINEAR)   // one step per launch; f64 has the row march only
        plain = p.dtype == ST_F64 ? LaunchCfg{ST_VARIANT_YM2D, 256, 0, 1, 0} : LaunchCfg{ST_VARIANT_TB2D, 64, 32, 1, 0};
    else plain.zchunk = 0;
    T_TRY(run_cfg(p, pl, plain, pl->taps, in, ref, tmp, kappa, steps, s));

    hipEvent_t e0, e1;
    T_TRY(hipEventCreate(&e0));
    T_TRY(hipEventCreate(&e1));
    float best_ms = INFINITY;
    LaunchCfg best = pl->cfg;
    bool any = false;
    for (const LaunchCfg& c : candidates(p)) {
        ++st.tried;
        Taps taps = pl->taps;
        // A planted fault shifts the centre weight; the difference-form
        // kernels read the weight sum in its place, so shift both.
        if (faulty(p, c)) {
            taps.c[0] += 0.25f;
            taps.sum += 0.25f;
        }
        // A planted fault in a variable-coefficient candidate reads every
        // field one grid too far.
        const void* aux = kappa;
        if (p.update == ST_VARCOEF && faulty(p, c)) aux = (const char*)kappa + gb;
        // Parity: same inputs (tmp is the wave's u_{-1}; refill it each time).
        T_TRY(fill(tmp, p, cells, 2u, lo, 1.f, s));
        T_TRY(run_cfg(p, pl, c, taps, in, out, tmp, aux, steps, s));
        unsigned h[2] = {0u, 0u};
        hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, s, cnt, 2);
        launch_max_diff(p.dtype, out, ref, cells, cnt, s);
        T_TRY(hipGetLastError());
        T_TRY(hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
        T_TRY(hipStreamSynchronize(s));
        float dmax, rmax;
        memcpy(&dmax, &h[0], 4);
        memcpy(&rmax, &h[1], 4);
        const float tol = parity_tol(p.dtype) * std::max(rmax, 1e-30f);
        if (!(dmax <= tol)) {
            ++st.rejected;
            continue;
        }
        // Timing on the real extent, median of five.
        std::vector<float> ms;
        for (int rep = 0; rep < 6; ++rep) {
            T_TRY(hipEventRecord(e0, s));
            T_TRY(run_cfg(p, pl, c, taps, in, out, tmp, aux, steps, s));
            T_TRY(hipEventRecord(e1, s));
            T_TRY(hipEventSynchronize(e1));
            float t = 0.f;
            T_TRY(hipEventElapsedTime(&t, e0, e1));
            if (rep > 0) ms.push_back(t);
        }
        std::sort(ms.begin(), ms.end());
        const float med = ms[ms.size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best = c;
            any = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
#undef T_TRY
    if (!any) {
        set_error("autotune: no candidate passed parity");
        return ST_ETUNE;
    }
    pl->cfg = best;
    dispatch_store(classify(p), best, true);
    return ST_OK;
}

// Reverse-step candidates of a wave case: the LDS-ring kernel (the one the
// pointwise gradient step runs) by tile height and plane chunk.
std::vector<LaunchCfg> reverse_candidates(const st_problem& p) {
    std::vector<LaunchCfg> out;
    for (int ty : {32, 16, 8})
        for (int zc : {0, 16, 32, 64, 128, 256}) {
            if (zc != 0 && zc >= p.n[2]) continue;
            LaunchCfg c{ST_VARIANT_WAVE3D_LDS, 0, ty, 1, zc};
            if (adj_cfg_legal(p, c)) out.push_back(c);
        }
    return out;
}

size_t plane_bytes_of(const st_problem& p) { return ((size_t)p.n[0] * p.n[1] * 4 + 255) / 256 * 256; }

// Bytes tune_reverse needs beyond tune_one's scratch: L(u_t), the reference
// gradient, and two planes (the target and the recorded trace).
size_t reverse_extra_bytes(const st_problem& p) {
    const size_t gb = (grid_bytes_of(p) + 255) / 256 * 256;
    return 2 * gb + 2 * plane_bytes_of(p);
}

// Tunes the reverse step of a wave plan whose forward runs the LDS-ring
// kernel: the pointwise gradient step (lambda_t and the dkappa update from
// L(u_t), with the receiver-plane residual).  Every candidate's lambda_t and
// dkappa are checked against the 32-row, unchunked launch on random fields;
// the fastest passing candidate (median of five) goes into the plan and the
// map cell of the reverse key.
st_status tune_reverse(st_plan* pl, char* scratch, size_t bytes, hipStream_t s, TuneStats& st) {
    const st_problem& p = pl->prob;
    if (p.update != ST_WAVE || pl->cfg.variant != ST_VARIANT_WAVE3D_LDS) return ST_OK;
    const size_t cells = (size_t)p.n[0] * p.n[1] * p.n[2];
    const size_t plane = (size_t)p.n[0] * p.n[1];
    const size_t gb = (cells * 4 + 255) / 256 * 256;
    const size_t need = 5 * gb + 64 + reverse_extra_bytes(p);
    if (bytes < need) {
        set_error("autotune scratch of %zu bytes needed", need);
        return ST_EWORKSPACE;
    }
    // tune_one's layout (in, out, tmp, ref, kappa, counters), then the rest.
    float* lam1 = (float*)scratch;              // lambda_{t+1}
    float* grad = (float*)(scratch + gb);       // dkappa accumulator
    float* lam2 = (float*)(scratch + 2 * gb);   // lambda_{t+2}, overwritten by lambda_t
    float* ref = (float*)(scratch + 3 * gb);
    const float* kappa = (const float*)(scratch + 4 * gb);
    unsigned* cnt = (unsigned*)(scratch + 5 * gb);
    char* extra = scratch + 5 * gb + 64;
    float* lap = (float*)extra;
    float* ref_grad = (float*)(extra + gb);
    float* target = (float*)(extra + 2 * gb);
    float* trace = (float*)(extra + 2 * gb + plane_bytes_of(p));
#define R_TRY(e)                                                                         \
    do {                                                                                 \
        hipError_t e_ = (e);                                                             \
        if (e_ != hipSuccess) {                                                          \
            set_error("autotune: %s: %s", #e, hipGetErrorString(e_));                    \
            return ST_EHIP;                                                              \
        }                                                                                \
    } while (0)
    st_problem f32 = p;
    f32.dtype = ST_F32;
    R_TRY(fill(lam1, f32, cells, 21u, -1.f, 1.f, s));
    R_TRY(fill(lap, f32, cells, 22u, -1.f, 1.f, s));
    R_TRY(fill(target, f32, plane, 23u, -1.f, 1.f, s));
    R_TRY(fill(trace, f32, plane, 24u, -1.f, 1.f, s));
    const Geom g = plan_geom(pl);
    // A planted fault (16-row candidates) shifts the centre weight of L^T.
    Taps bad = pl->taps_t;
    bad.c[0] += 0.25f;
    bad.sum += 0.25f;
    auto run = [&](const LaunchCfg& c) -> hipError_t {
        WaveLaunch w;
        memset(&w, 0, sizeof w);
        w.src_x = -1;
        w.prev_sign = 1.f;
        w.prev_damped = true;
        w.prev = lam2;
        w.cur = lam1;
        w.next = lam2;
        w.kappa = kappa;
        w.grad = grad;
        w.lap = lap;
        w.rec_z = (int)(p.n[2] / 2);
        w.target_t = target;
        w.trace_res = trace;
        return launch_wave_adjoint(g, c, faulty(p, c) ? bad : pl->taps_t, pl->taps, kWaveGradPt, w, s);
    };
    auto reset = [&]() -> hipError_t {
        hipError_t e = fill(lam2, f32, cells, 25u, -1.f, 1.f, s);
        return e != hipSuccess ? e : fill(grad, f32, cells, 26u, -1.f, 1.f, s);
    };
    const LaunchCfg plain{ST_VARIANT_WAVE3D_LDS, 0, 32, 1, 0};
    R_TRY(reset());
    R_TRY(run(plain));
    R_TRY(hipMemcpyAsync(ref, lam2, cells * 4, hipMemcpyDeviceToDevice, s));
    R_TRY(hipMemcpyAsync(ref_grad, grad, cells * 4, hipMemcpyDeviceToDevice, s));

    hipEvent_t e0, e1;
    R_TRY(hipEventCreate(&e0));
    R_TRY(hipEventCreate(&e1));
    float best_ms = INFINITY;
    LaunchCfg best = pl->adj_cfg;
    bool any = false;
    for (const LaunchCfg& c : reverse_candidates(p)) {
        ++st.tried;
        R_TRY(reset());
        R_TRY(run(c));
        unsigned h[4] = {0u, 0u, 0u, 0u};
        hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, s, cnt, 4);
        launch_max_diff(ST_F32, lam2, ref, cells, cnt, s);
        launch_max_diff(ST_F32, grad, ref_grad, cells, cnt + 2, s);
        R_TRY(hipGetLastError());
        R_TRY(hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
        R_TRY(hipStreamSynchronize(s));
        float v[4];
        memcpy(v, h, sizeof v);
        const float tol = parity_tol(ST_F32);
        if (!(v[0] <= tol * std::max(v[1], 1e-30f)) || !(v[2] <= tol * std::max(v[3], 1e-30f))) {
            ++st.rejected;
            continue;
        }
        // Two launches per sample: lambda alternates between two states, so
        // the repeated in-place step stays bounded.
        std::vector<float> ms;
        for (int rep = 0; rep < 6; ++rep) {
            R_TRY(hipEventRecord(e0, s));
            R_TRY(run(c));
            R_TRY(run(c));
            R_TRY(hipEventRecord(e1, s));
            R_TRY(hipEventSynchronize(e1));
            float t = 0.f;
            R_TRY(hipEventElapsedTime(&t, e0, e1));
            if (rep > 0) ms.push_back(t);
        }
        std::sort(ms.begin(), ms.end());
        const float med = ms[ms.size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best = c;
            any = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
#undef R_TRY
    if (!any) {
        set_error("autotune: no reverse-step candidate passed parity");
        return ST_ETUNE;
    }
    pl->adj_cfg = best;
    dispatch_store(reverse_key(p), best, true);
    return ST_OK;
}

// Steps of the grouped-launch probe: a multiple of every candidate depth
// but 8, so most candidates run whole blocks.
constexpr int kBatchProbeSteps = 12;

// Batch depths the grouped launch is timed at (kMemberDepths: each member
// its own map depth).
constexpr int kBatchDepths[] = {1, 2, 3, 4, 6, 8, kMemberDepths};

// Workspace of a grouped launch of the probe at any candidate depth: the
// partner grids plus the largest member-table set.
size_t batch_probe_ws(const st_plan* plan) {
    size_t grids = 0, meta = 0;
    for (const st_plan* m : plan->members) grids += (grid_bytes_of(m->prob) + 255) / 256 * 256;
    for (int k : kBatchDepths) meta = std::max(meta, batched_meta_bytes(plan, kBatchProbeSteps, k));
    return grids + meta;
}


// Fused depth of the grouped batched launch, measured on the member grids:
// each candidate depth (one depth for all members, or each member's own map
// depth) runs the whole batch, every member's output is checked against
// depth 1, and the fastest passing candidate (median of five) becomes the
// plan's batch depth.
st_status tune_batch_depth(st_plan* plan, char* scratch, size_t bytes, hipStream_t s, TuneStats& st) {
    const size_t need = batch_tune_bytes(plan);
    if (bytes < need) {
        set_error("autotune scratch of %zu bytes needed", need);
        return ST_EWORKSPACE;
    }
#define B_TRY(e)                                                                         \
    do {                                                                                 \
        hipError_t e_ = (e);                                                             \
        if (e_ != hipSuccess) {                                                          \
            set_error("autotune: %s: %s", #e, hipGetErrorString(e_));                    \
            return ST_EHIP;                                                              \
        }                                                                                \
    } while (0)
    const int nm = (int)plan->members.size();
    std::vector<void*> in(nm), out(nm), ref(nm);
    std::vector<size_t> cells(nm);
    char* p = scratch;
    for (int g = 0; g < nm; ++g) {
        const st_problem& pr = plan->members[g]->prob;
        cells[g] = (size_t)pr.n[0] * pr.n[1];
        const size_t gb = (grid_bytes_of(pr) + 255) / 256 * 256;
        in[g] = p;
        out[g] = p + gb;
        ref[g] = p + 2 * gb;
        p += 3 * gb;
        B_TRY(fill(in[g], pr, cells[g], 11u + g, 0.f, 1.f, s));
    }
    const size_t wsb = batch_probe_ws(plan);
    void* ws = p;
    unsigned* cnt = (unsigned*)(p + (wsb + 255) / 256 * 256);
    const int keep = plan->cfg.tsteps;
    plan->cfg.tsteps = 1;
    st_status r = stencil_apply_batched(plan, in.data(), ref.data(), kBatchProbeSteps, ws, wsb, s);
    if (r != ST_OK) {
        plan->cfg.tsteps = keep;
        return r;
    }
    hipEvent_t e0, e1;
    B_TRY(hipEventCreate(&e0));
    B_TRY(hipEventCreate(&e1));
    float best_ms = INFINITY;
    int best = keep;
    for (int k : kBatchDepths) {
        ++st.tried;
        plan->cfg.tsteps = k;
        r = stencil_apply_batched(plan, in.data(), out.data(), kBatchProbeSteps, ws, wsb, s);
        if (r != ST_OK) break;
        bool ok = true;
        for (int g = 0; g < nm && ok; ++g) {
            const st_problem& pr = plan->members[g]->prob;
            unsigned h[2] = {0u, 0u};
            hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, s, cnt, 2);
            launch_max_diff(pr.dtype, out[g], ref[g], cells[g], cnt, s);
            B_TRY(hipGetLastError());
            B_TRY(hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, s));
            B_TRY(hipStreamSynchronize(s));
            float dmax, rmax;
            memcpy(&dmax, &h[0], 4);
            memcpy(&rmax, &h[1], 4);
            ok = dmax <= parity_tol(pr.dtype) * std::max(rmax, 1e-30f);
        }
        if (!ok) {
            ++st.rejected;
            continue;
        }
        std::vector<float> ms;
        for (int rep = 0; rep < 6 && r == ST_OK; ++rep) {
            B_TRY(hipEventRecord(e0, s));
            r = stencil_apply_batched(plan, in.data(), out.data(), kBatchProbeSteps, ws, wsb, s);
            B_TRY(hipEventRecord(e1, s));
            B_TRY(hipEventSynchronize(e1));
            float t = 0.f;
            B_TRY(hipEventElapsedTime(&t, e0, e1));
            if (rep > 0) ms.push_back(t);
        }
        if (r != ST_OK) break;
        std::sort(ms.begin(), ms.end());
        if (ms[ms.size() / 2] < best_ms) {
            best_ms = ms[ms.size() / 2];
            best = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
#undef B_TRY
    plan->cfg.tsteps = best;
    return r;
}

}  // namespace

namespace stk {

size_t reverse_tune_bytes(const st_problem& p) { return reverse_extra_bytes(p); }

size_t batch_tune_bytes(const st_plan* plan) {
    size_t g = 0;
    for (const st_plan* m : plan->members) g += 3 * ((grid_bytes_of(m->prob) + 255) / 256 * 256);
    return g + batch_probe_ws(plan) + 256;
}

}  // namespace stk

extern "C" {

st_status stencil_autotune(st_plan* plan, void* scratch, size_t scratch_bytes, void* stream) {
    set_error("%s", "");
    if (!plan) {
        set_error("plan is NULL");
        return ST_EINVAL;
    }
    if (!scratch) {
        set_error("scratch is NULL");
        return ST_EWORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    TuneStats st;
    if (!plan->batched) {
        st_status r = tune_one(plan, (char*)scratch, scratch_bytes, s, st);
        if (r == ST_OK) r = tune_reverse(plan, (char*)scratch, scratch_bytes, s, st);
        plan->tune_tried = st.tried;
        plan->tune_rejected = st.rejected;
        return r;
    }
    // One measurement per distinct case key; members of that key adopt it.
    std::vector<std::pair<CaseKey, LaunchCfg>> done;
    for (st_plan* m : plan->members) {
        const CaseKey k = classify(m->prob);
        bool found = false;
        for (auto& d : done)
            if (!memcmp(&d.first, &k, sizeof k)) {
                m->cfg = d.second;
                found = true;
                break;
            }
        if (found) continue;
        st_status r = tune_one(m, (char*)scratch, scratch_bytes, s, st);
        if (r != ST_OK) return r;
        done.push_back({k, m->cfg});
    }
    // Then the batch depth of the grouped launch.
    st_status r = tune_batch_depth(plan, (char*)scratch, scratch_bytes, s, st);
    plan->tune_tried = st.tried;
    plan->tune_rejected = st.rejected;
    return r;
}

st_status stencil_autotune_stats(const st_plan* plan, int32_t* tried, int32_t* rejected) {
    if (!plan) {
        set_error("plan is NULL");
        return ST_EINVAL;
    }
    if (tried) *tried = plan->tune_tried;
    if (rejected) *rejected = plan->tune_rejected;
    return ST_OK;
}

}  // extern "C"
