// Host-side internals shared by the runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <atomic>

#include "common.h"

namespace stk {

// Geometry and type of one case, as the launchers need it.
struct Geom {
    int ndim;
    int nx, ny, nz;
    int shape, r, dtype, boundary;
    bool iso;   // star with one weight per distance on every arm and sign
    // Element strides of the in-plane second axis and of the march axis for
    // a march along y (0: the z-march's nx and nx * ny).
    int sy = 0;
    size_t sz = 0;
};

// Launch parameters chosen by the dispatch map.
struct LaunchCfg {
    int variant;   // st_variant
    int tile_x;    // TB2D output tile width
    int tile_y;    // TB2D output tile height; ZM3D/WAVE3D rows per workgroup
    int tsteps;    // TB2D fused time steps
    int zchunk;    // ZM3D/WAVE3D planes per workgroup (0 = all)
};

// kWaveGrad stages u_t and applies L to it; kWaveGradPt takes L(u_t) as a
// pointwise field (written by a forward step with lap_out) and the residual
// plane from the recorded trace.
enum WaveMode { kWaveFwd = 0, kWaveAdj = 1, kWaveGrad = 2, kWaveGradPt = 3 };

struct WaveLaunch {
    const float* prev;      // u_{t-1} (fwd/adj) or lambda_{t+2} (grad)
    const float* cur;       // u_t (fwd) or lambda_{t+1} (adj, grad)
    float* next;            // u_{t+1} / lambda_t; may alias prev
    const float* kappa;
    const float* u;         // grad: u_t (second stencil field)
    float* grad;            // grad: dJ/dkappa accumulator
    const float* target_t;  // grad: d_t plane (ny*nx) or null
    int rec_z;              // grad: plane of the residual injection; fwd: receiver plane
    float* trace_t;         // fwd: plane written with u_{t+1}[rec_z] or null
    int src_x, src_y, src_z;  // fwd: source cell (src_x < 0 = none)
    const float* src_amp;   // fwd: device pointer to the amplitude added at the source
    float prev_sign;        // adj: next = 2 cur - prev_sign * prev (-1 on the first step, +1 after)
    float* lap_out;         // fwd (ring kernel): receives L(u_t) at every cell, or null
    const float* lap;       // gradPt: L(u_t), or null (no gradient update this step)
    const float* trace_res; // gradPt: u_t on plane rec_z (ny*nx), used with target_t
    // Absorbing layer (sp_w > 0): damping gamma(x) = sum over axes of
    // sp_s ((W - e) / W)^2 within W = sp_w cells of a face (e = distance to
    // the nearer face); step u_{t+1} = A (2 u_t + kappa L u_t) - B u_{t-1},
    // A = 1 / (1 + gamma/2), B = (1 - gamma/2) A.  Ring kernels only.
    int sp_w;
    float sp_s, sp_invw;
    bool prev_damped;       // adj: the prev term carries B (false on the first transposed step)
    bool exact_update;      // fwd (ring kernel): state update in FP64, rounded once
};

// Damping ramp of the absorbing layer along one axis at index i of n cells.
__device__ __forceinline__ float sponge_ramp(int i, int n, int w, float s, float invw) {
    const int e = min(i, n - 1 - i);
    const float q = (float)max(w - e, 0) * invw;
    return s * q * q;
}

// Operands of one FP64 forward leapfrog step (fields as in WaveLaunch, in
// binary64).
struct WaveLaunchF64 {
    const double* prev;     // u_{t-1}
    const double* cur;      // u_t
    double* next;           // u_{t+1}; may alias prev
    const double* kappa;
    int src_x, src_y, src_z;  // src_x < 0 = none
    const double* src_amp;  // device pointer to the amplitude added at the source
    int rec_z;
    double* trace_t;        // plane written with u_{t+1}[rec_z] or null
    int sp_w;               // absorbing layer width (0 = none) and strength
    double sp_s;
};

// Star weights in binary64, in the compact star layout of Taps (c[0] the
// centre, then the x, y and z arms by star_x / star_y / star_z).
struct TapsD {
    double c[6 * kMaxRadius + 1];
};

// Two fused forward leapfrog steps: (u_{t-1}, u_t) -> (u_{t+1}, u_{t+2}).
// out1/out2 must not alias prev/cur (other workgroups read their halos).
struct WaveTB2 {
    const float* prev;
    const float* cur;
    float* out1;
    float* out2;
    const float* kappa;
    int src_x, src_y, src_z;     // src_x < 0 = none
    const float* amp1;           // added at the source to u_{t+1}
    const float* amp2;           // added at the source to u_{t+2}
    int rec_z;
    float* trace1;               // plane for u_{t+1}[rec_z] or null
    float* trace2;               // plane for u_{t+2}[rec_z] or null
};

// Raises kernel KERN's dynamic-LDS ceiling to the 160 KiB of a gfx950 CU,
// once per device (the first launch on a device that needs more than the
// default 64 KiB), so later launches skip the runtime call.
template <auto KERN>
inline hipError_t allow_large_lds() {
    static std::atomic<unsigned long long> done{0};   // bit d: set on device d
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const unsigned long long bit = 1ull << (dev & 63);
    if (done.load(std::memory_order_acquire) & bit) return hipSuccess;
    e = hipFuncSetAttribute((const void*)KERN, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess) done.fetch_or(bit, std::memory_order_acq_rel);
    return e;
}

// Launchers (return the launch status; asynchronous on `stream`).
hipError_t launch_tb2d(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                       void* out, int k, hipStream_t stream);
hipError_t launch_ym2d(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                       void* out, int k, hipStream_t stream);
hipError_t launch_zm3d(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                       void* out, hipStream_t stream);
hipError_t launch_zm3d_mfma(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                            void* out, hipStream_t stream);
bool zm3d_mfma_supported(const Geom& g);
hipError_t launch_zm3d_h2(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in, void* out,
                          hipStream_t stream);
hipError_t launch_ym3d(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in, void* out,
                       hipStream_t stream);
bool ym3d_supported(const Geom& g);
bool zm3d_h2_supported(const Geom& g);
hipError_t launch_ym2d_h2(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in, void* out, int k,
                          hipStream_t stream);
bool ym2d_h2_supported(const Geom& g);
int ym2d_h2_lds_bytes(int nt, int k, int R);
hipError_t launch_zm3d_tb2(const Geom& g, const LaunchCfg& cfg, const Taps& taps, const void* in,
                           void* out, hipStream_t stream);
bool zm3d_tb2_supported(int r, int shape);
// One variable-coefficient step (adjoint = the transpose); fields as in
// stencil_apply_varcoef.
hipError_t launch_vc3d(const Geom& g, const LaunchCfg& cfg, const void* in, void* out, const void* fields,
                       bool adjoint, hipStream_t stream);
bool vc3d_supported(int r, int shape);
// One FP64 forward leapfrog step (cfg.tile_y: 8 or 16 rows per workgroup).
hipError_t launch_wave3d_f64(const Geom& g, const LaunchCfg& cfg, const TapsD& taps, const WaveLaunchF64& w,
                             hipStream_t stream);

// One launch of a 3D linear sweep (k = 1 or 2 fused steps) through the
// kernel family the configuration names.
inline hipError_t launch_linear3d(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                                  const void* in, void* out, int k, hipStream_t stream) {
    if (k == 2) return launch_zm3d_tb2(g, cfg, taps, in, out, stream);
    if (cfg.variant == 6) return launch_zm3d_mfma(g, cfg, taps, in, out, stream);
    if (cfg.variant == 8) return launch_zm3d_h2(g, cfg, taps, in, out, stream);
    if (cfg.variant == 10) return launch_ym3d(g, cfg, taps, in, out, stream);
    return launch_zm3d(g, cfg, taps, in, out, stream);
}
hipError_t launch_wave3d(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                         const Taps& taps_fwd, WaveMode mode, const WaveLaunch& w,
                         hipStream_t stream);
hipError_t launch_wave3d_tb2(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                             const WaveTB2& w, hipStream_t stream);
bool wave3d_tb2_supported(int r);
hipError_t launch_wave3d_ring(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                              const WaveLaunch& w, hipStream_t stream);
bool wave3d_ring_supported(int r);
hipError_t launch_wave3d_ring_adj(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                                  const Taps& taps_fwd, WaveMode mode, const WaveLaunch& w,
                                  hipStream_t stream);

// One adjoint or gradient step through the kernel family the configuration
// names (the LDS-ring kernel, or the partial-sum queue kernel).
inline hipError_t launch_wave_adjoint(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                                      const Taps& taps_fwd, WaveMode mode, const WaveLaunch& w,
                                      hipStream_t stream) {
    if (cfg.variant == 4) return launch_wave3d_ring_adj(g, cfg, taps, taps_fwd, mode, w, stream);
    return launch_wave3d(g, cfg, taps, taps_fwd, mode, w, stream);
}
hipError_t launch_scale(float* dst, const float* src, float alpha, size_t n, hipStream_t stream);
// dst = alpha * B(x) * dst with B the absorbing layer's damping of u_{t-1}.
hipError_t launch_sponge_scale(const Geom& g, float* dst, float alpha, int w, float s, hipStream_t stream);
hipError_t launch_fill(float* dst, float v, size_t n, hipStream_t stream);
// loss = 1/2 sum (traces - target)^2 in double, two fixed-order passes
// through `parts` (kLossParts doubles of scratch): deterministic.
constexpr int kLossParts = 512;
hipError_t launch_trace_loss(const float* traces, const float* target, size_t n, double* parts,
                             double* loss, hipStream_t stream);

bool tb2d_supported(int r, int shape);
bool zm3d_supported(int r, int shape);
bool wave3d_supported(int r);
int zm3d_rows(const LaunchCfg& cfg);    // rows per workgroup actually used
int tb2d_max_lds_bytes();
int tb2d_lds_floats_host(int BX, int BY, int k, int R);
bool ym2d_supported(int r, int shape);
int ym2d_rows(int nt, int k, int R, int esz = 4);        // input rows per march iteration
int ym2d_lds_bytes(int nt, int k, int R, int esz = 4);   // esz: 8 for f64 storage
int ym2d_max_lds_bytes();
int ym2d_auto_chunk(int nx, int ny, int nt, int k, int R);

// One launch of a 2D linear sweep (k fused steps) through the kernel family
// the configuration names.
inline hipError_t launch_linear2d(const Geom& g, const LaunchCfg& cfg, const Taps& taps,
                                  const void* in, void* out, int k, hipStream_t stream) {
    if (cfg.variant == 5) return launch_ym2d(g, cfg, taps, in, out, k, stream);
    if (cfg.variant == 9) return launch_ym2d_h2(g, cfg, taps, in, out, k, stream);
    return launch_tb2d(g, cfg, taps, in, out, k, stream);
}


}  // namespace stk
