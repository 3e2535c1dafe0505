// C ABI of libstencil: plan creation and validation, single-grid sweeps,
// transposed sweeps and the checkpointed wave gradient.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "plan.h"

using namespace stk;

namespace stk {
const char* last_error();
}

#define ST_FAIL(code, ...)            \
    do {                              \
        stk::set_error(__VA_ARGS__);  \
        return (code);                \
    } while (0)

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            ST_FAIL(ST_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));              \
    } while (0)

namespace {

constexpr int64_t kMaxExtent = int64_t(1) << 24;
constexpr double kMaxCells = 68719476736.0;   // 2^36

size_t elem_bytes(int dtype) { return dtype == ST_F16 ? 2 : (dtype == ST_F64 ? 8 : 4); }

size_t cells_of(const st_problem& p) { return (size_t)p.n[0] * (size_t)p.n[1] * (size_t)p.n[2]; }

size_t grid_bytes(const st_problem& p) { return cells_of(p) * elem_bytes(p.dtype); }

// The f32 views of a wave plan's operands (ST_F64 plans take run_wave_f64).
const float* wkappa(const st_wave_args* wa) { return static_cast<const float*>(wa->kappa); }
const float* wwavelet(const st_wave_args* wa) { return static_cast<const float*>(wa->wavelet); }
float* wtraces(const st_wave_args* wa) { return static_cast<float*>(wa->traces); }

bool in_shape(int ndim, int shape, int r, int idx) {
    const int w = 2 * r + 1;
    const int dx = idx % w - r;
    const int dy = (idx / w) % w - r;
    const int dz = ndim == 3 ? idx / (w * w) - r : 0;
    if (shape == ST_BOX) return true;
    return ((dz != 0) + (dy != 0) + (dx != 0)) <= 1;
}

// Central second-difference weights of accuracy order 2r (r = 1..4), the
// standard finite-difference table.
const double kFd2[4][5] = {
    {-2.0, 1.0, 0.0, 0.0, 0.0},
    {-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0, 0.0, 0.0},
    {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0, 0.0},
    {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0},
};

void builtin_laplacian(int r, std::vector<float>& dense) {
    const int w = 2 * r + 1;
    dense.assign((size_t)w * w * w, 0.f);
    const double* f = kFd2[r - 1];
    dense[(size_t)(r * w + r) * w + r] = (float)(3.0 * f[0]);
    for (int j = 1; j <= r; ++j)
        for (int s = -1; s <= 1; s += 2) {
            dense[(size_t)((r + s * j) * w + r) * w + r] = (float)f[j];
            dense[(size_t)(r * w + r + s * j) * w + r] = (float)f[j];
            dense[(size_t)(r * w + r) * w + r + s * j] = (float)f[j];
        }
}

// Dense (dz,dy,dx) array -> compact kernel taps (layout in common.h).
Taps pack_taps(int ndim, int shape, int r, const std::vector<float>& dense) {
    Taps t;
    memset(&t, 0, sizeof t);
    const int w = 2 * r + 1;
    const int rz = ndim == 3 ? r : 0;
    auto at = [&](int dz, int dy, int dx) {
        return dense[(size_t)((dz + rz) * w + (dy + r)) * w + (dx + r)];
    };
    double sum = 0.0;
    for (float v : dense) sum += (double)v;
    t.sum = (float)sum;
    if (shape == ST_BOX) {
        for (size_t i = 0; i < dense.size() && i < (size_t)kMaxTaps; ++i) t.c[i] = dense[i];
        return t;
    }
    t.c[0] = at(0, 0, 0);
    for (int d = -r; d <= r; ++d) {
        if (d == 0) continue;
        const int slot = d < 0 ? 1 + (d + r) : r + d;
        t.c[slot] = at(0, 0, d);
        t.c[2 * r + slot] = at(0, d, 0);
        if (ndim == 3) t.c[4 * r + slot] = at(d, 0, 0);
    }
    return t;
}

st_status validate(const st_problem* p) {
    if (!p) ST_FAIL(ST_EINVAL, "problem is NULL");
    if (p->ndim != 2 && p->ndim != 3) ST_FAIL(ST_EINVAL, "ndim must be 2 or 3 (got %d)", p->ndim);
    if (p->shape != ST_STAR && p->shape != ST_BOX) ST_FAIL(ST_EINVAL, "unknown shape %d", p->shape);
    if (p->dtype != ST_F32 && p->dtype != ST_F16 && p->dtype != ST_F64)
        ST_FAIL(ST_EINVAL, "unknown dtype %d", p->dtype);
    if (p->boundary != ST_PERIODIC && p->boundary != ST_ZERO)
        ST_FAIL(ST_EINVAL, "unknown boundary %d", p->boundary);
    if (p->update != ST_LINEAR && p->update != ST_WAVE && p->update != ST_VARCOEF)
        ST_FAIL(ST_EINVAL, "unknown update %d", p->update);
    if (p->radius < 1 || p->radius > 4) ST_FAIL(ST_EINVAL, "radius must be 1..4 (got %d)", p->radius);
    for (int a = 0; a < 3; ++a)
        if (p->n[a] < 1 || p->n[a] > kMaxExtent)
            ST_FAIL(ST_ESHAPE, "extent n[%d] = %lld outside 1..2^24", a, (long long)p->n[a]);
    if (p->ndim == 2 && p->n[2] != 1) ST_FAIL(ST_ESHAPE, "2D problem needs n[2] == 1");
    if ((double)p->n[0] * (double)p->n[1] * (double)p->n[2] > kMaxCells)
        ST_FAIL(ST_ESHAPE, "grid has more than 2^36 cells");
    if ((double)p->n[0] * (double)p->n[1] > 2147483647.0)
        ST_FAIL(ST_ESHAPE, "one plane must hold fewer than 2^31 cells");
    // The plane marches (every 3D kernel, and the variable-coefficient
    // kernel in 2D) address a plane by 32-bit byte offsets.
    if ((p->ndim == 3 || p->update == ST_VARCOEF) &&
        (double)p->n[0] * (double)p->n[1] * (double)elem_bytes(p->dtype) > 4294967295.0)
        ST_FAIL(ST_ESHAPE, "one x-y plane of a 3D or variable-coefficient grid must fit in 4 GiB");
    if (p->update == ST_VARCOEF) {
        if (!vc3d_supported(p->radius, p->shape))
            ST_FAIL(ST_EUNSUPPORTED, "variable-coefficient %s r=%d is not provided",
                    p->shape == ST_STAR ? "star" : "box", p->radius);
    } else if (p->update == ST_WAVE) {
        if (p->ndim != 3 || p->shape != ST_STAR)
            ST_FAIL(ST_EUNSUPPORTED, "the wave update needs a 3D star stencil");
        if (p->dtype != ST_F32 && p->dtype != ST_F64)
            ST_FAIL(ST_EUNSUPPORTED, "the wave update needs f32 or f64 storage");
    } else {
        if (!p->coeffs) ST_FAIL(ST_EINVAL, "coefficients are NULL");
        if (p->ndim == 2 && !tb2d_supported(p->radius, p->shape))
            ST_FAIL(ST_EUNSUPPORTED, "2D %s r=%d is not provided", p->shape == ST_STAR ? "star" : "box",
                    p->radius);
        if (p->ndim == 3 && !zm3d_supported(p->radius, p->shape))
            ST_FAIL(ST_EUNSUPPORTED, "3D %s r=%d is not provided", p->shape == ST_STAR ? "star" : "box",
                    p->radius);
    }
    if (p->coeffs && p->update != ST_VARCOEF) {
        const int w = 2 * p->radius + 1;
        const int count = p->ndim == 3 ? w * w * w : w * w;
        for (int i = 0; i < count; ++i) {
            if (!isfinite(p->coeffs[i])) ST_FAIL(ST_EINVAL, "coefficient %d is not finite", i);
            if (!in_shape(p->ndim, p->shape, p->radius, i) && p->coeffs[i] != 0.f)
                ST_FAIL(ST_EINVAL, "coefficient %d lies outside the star but is nonzero", i);
        }
    }
    return ST_OK;
}

st_status build_plan(const st_problem* p, const st_plan_opts* opts, st_plan** out) {
    st_status s = validate(p);
    if (s != ST_OK) return s;
    st_plan* pl = new (std::nothrow) st_plan();
    if (!pl) ST_FAIL(ST_ENOMEM, "out of host memory");
    pl->prob = *p;
    pl->prob.coeffs = nullptr;
    const int w = 2 * p->radius + 1;
    const int count = p->ndim == 3 ? w * w * w : w * w;
    if (p->update == ST_VARCOEF) pl->dense.assign(count, 0.f);   // the fields carry the weights
    else if (p->coeffs) pl->dense.assign(p->coeffs, p->coeffs + count);
    else builtin_laplacian(p->radius, pl->dense);
    std::vector<float> flipped(pl->dense.rbegin(), pl->dense.rend());
    pl->taps = pack_taps(p->ndim, p->shape, p->radius, pl->dense);
    pl->taps_t = pack_taps(p->ndim, p->shape, p->radius, flipped);
    if (p->update == ST_WAVE && !p->coeffs) {
        // The built-in Laplacian is a sum of per-axis second differences,
        // each of which annihilates constants: its weights sum to exactly 0.
        // The sum of the f32-rounded weights is not 0 (about -1.9e-7 for
        // r = 4), and the difference form's (sum) u(x) term would add that
        // spurious multiple of u to every evaluation.
        pl->taps.sum = 0.f;
        pl->taps_t.sum = 0.f;
    }
    memset(&pl->taps64, 0, sizeof pl->taps64);
    if (p->update == ST_WAVE && p->dtype == ST_F64) {
        // Binary64 star weights: the caller's (exact as doubles) or the
        // built-in Laplacian's rationals, each rounded once to binary64.
        const int r = p->radius;
        auto slot = [r](int d) { return d < 0 ? 1 + (d + r) : r + d; };
        if (p->coeffs) {
            pl->taps64.c[0] = (double)pl->taps.c[0];
            for (int i = 1; i <= 6 * r; ++i) pl->taps64.c[i] = (double)pl->taps.c[i];
        } else {
            const double* f = kFd2[r - 1];
            pl->taps64.c[0] = 3.0 * f[0];
            for (int d = -r; d <= r; ++d) {
                if (d == 0) continue;
                const double v = f[d < 0 ? -d : d];
                pl->taps64.c[slot(d)] = v;
                pl->taps64.c[2 * r + slot(d)] = v;
                pl->taps64.c[4 * r + slot(d)] = v;
            }
        }
    }
    pl->iso = false;
    if (p->shape == ST_STAR) {
        // One weight per distance on every arm and sign (e.g. a Laplacian).
        bool iso = true;
        const int arms = p->ndim == 3 ? 6 : 4;
        for (int d = 1; d <= p->radius && iso; ++d) {
            const float w = pl->taps.c[p->radius + d];   // +x arm at distance d
            for (int a = 0; a < arms / 2; ++a)
                for (int sgn = 0; sgn < 2; ++sgn) {
                    const int slot = 2 * p->radius * a + (sgn ? p->radius + d : 1 + (-d + p->radius));
                    iso = iso && pl->taps.c[slot] == w;
                }
        }
        pl->iso = iso;
    }
    pl->cfg = dispatch_lookup(classify(*p));
    if (pl->cfg.zchunk == kAutoChunk) pl->cfg.zchunk = auto_zchunk(*p, pl->cfg);
    if (!cfg_legal(pl->prob, pl->cfg)) {   // a stale map entry falls back to the default
        LaunchCfg d = default_dispatch(classify(*p));
        // (the y-march default of a few-plane slab needs the grid under 4 GiB)
        if (!cfg_legal(pl->prob, d) && p->ndim == 3 && p->update == ST_LINEAR)
            d = variant_default(*p, ST_VARIANT_ZM3D);
        if (d.zchunk == kAutoChunk) d.zchunk = auto_zchunk(*p, d);
        pl->cfg = d;
    }
    // The adjoint and gradient steps have a map cell of their own.
    if (p->update == ST_WAVE) {
        auto fix_chunk = [&](LaunchCfg& c) {
            if (c.zchunk == kAutoChunk) c.zchunk = auto_zchunk(*p, c, c.variant == ST_VARIANT_WAVE3D_LDS ? 1 : 0);
        };
        pl->adj_cfg = dispatch_lookup(reverse_key(*p));
        fix_chunk(pl->adj_cfg);
        if (!adj_cfg_legal(pl->prob, pl->adj_cfg)) {
            pl->adj_cfg = default_dispatch(reverse_key(*p));
            fix_chunk(pl->adj_cfg);
        }
    }
    pl->ckpt_every = 20;
    pl->batched = false;
    if (opts) {
        if (opts->ckpt_every < 0) {
            delete pl;
            ST_FAIL(ST_EINVAL, "ckpt_every must be >= 0");
        }
        if (opts->ckpt_every > 0) pl->ckpt_every = opts->ckpt_every;
        LaunchCfg c = pl->cfg;
        if (opts->variant != ST_VARIANT_AUTO && opts->variant != c.variant) {
            c = variant_default(*p, opts->variant);
            if (c.zchunk == kAutoChunk) c.zchunk = auto_zchunk(*p, c);
        }
        if (opts->tile_x > 0) c.tile_x = opts->tile_x;
        if (opts->tile_y > 0) c.tile_y = opts->tile_y;
        if (opts->tsteps > 0) c.tsteps = opts->tsteps;
        if (opts->zchunk > 0) c.zchunk = opts->zchunk;
        if (!cfg_legal(pl->prob, c)) {
            delete pl;
            ST_FAIL(ST_EINVAL, "plan options name an illegal variant/tile/depth for this case");
        }
        pl->cfg = c;
        // An explicit partial-sum family, tile height or chunk applies to the
        // adjoint kernel too.
        if (opts->variant == ST_VARIANT_WAVE3D) {
            pl->adj_cfg.variant = ST_VARIANT_WAVE3D;
            pl->adj_cfg.tile_y = 32;
        }
        if (opts->tile_y > 0) pl->adj_cfg.tile_y = opts->tile_y;
        if (opts->zchunk > 0) pl->adj_cfg.zchunk = opts->zchunk;
        else if (opts->tile_y > 0 || opts->variant == ST_VARIANT_WAVE3D)
            pl->adj_cfg.zchunk = auto_zchunk(*p, pl->adj_cfg, pl->adj_cfg.variant == ST_VARIANT_WAVE3D_LDS ? 1 : 0);
    }
    *out = pl;
    return ST_OK;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// One forward leapfrog step through the plan's forward kernel family.
hipError_t wave_forward_launch(const st_plan* pl, const WaveLaunch& w, hipStream_t s) {
    const Geom g = plan_geom(pl);
    if (pl->cfg.variant == ST_VARIANT_WAVE3D_LDS) return launch_wave3d_ring(g, pl->cfg, pl->taps, w, s);
    LaunchCfg c = pl->cfg;
    return launch_wave3d(g, c, pl->taps, pl->taps, kWaveFwd, w, s);
}

// One launch of the linear sweep, k fused steps (k = 1 for 3D).
hipError_t linear_launch(const st_plan* pl, const Taps& taps, const void* in, void* out, int k,
                         hipStream_t s) {
    const Geom g = geom_of(pl->prob);
    if (pl->prob.ndim == 2) return launch_linear2d(g, pl->cfg, taps, in, out, k, s);
    return launch_linear3d(g, pl->cfg, taps, in, out, k, s);
}

// Runs `steps` linear steps from u_in into u_out, rotating through the
// workspace so the last launch lands in u_out (see the buffer schedule in
// stencil_apply's documentation).
st_status run_linear(const st_plan* pl, const Taps& taps, const void* u_in, void* u_out, int steps,
                     void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t gb = grid_bytes(pl->prob);
    if (steps == 0) {
        if (u_in != u_out) HIP_TRY(hipMemcpyAsync(u_out, u_in, gb, hipMemcpyDeviceToDevice, s));
        return ST_OK;
    }
    if (!ws || ws_bytes < gb) ST_FAIL(ST_EWORKSPACE, "workspace of %zu bytes needed", gb);
    const int k = pl->prob.ndim == 2 ? std::max(1, pl->cfg.tsteps) : (pl->cfg.tsteps == 2 ? 2 : 1);
    const int L = (steps + k - 1) / k;
    const void* cur = u_in;
    if (u_in == u_out && (L % 2) == 1) {
        HIP_TRY(hipMemcpyAsync(ws, u_in, gb, hipMemcpyDeviceToDevice, s));
        cur = ws;
    }
    int done = 0;
    for (int j = 1; j <= L; ++j) {
        const int kj = std::min(k, steps - done);
        void* dst = ((L - j) % 2 == 0) ? u_out : ws;
        HIP_TRY(linear_launch(pl, taps, cur, dst, kj, s));
        cur = dst;
        done += kj;
    }
    return ST_OK;
}

WaveLaunch wave_base(const st_wave_args* wa = nullptr) {
    WaveLaunch w;
    memset(&w, 0, sizeof w);
    w.src_x = -1;
    w.rec_z = -1;
    w.prev_sign = 1.f;
    w.prev_damped = true;
    if (wa && wa->sponge_width > 0) {
        w.sp_w = wa->sponge_width;
        w.sp_s = wa->sponge_strength;
        w.sp_invw = 1.f / (float)wa->sponge_width;
    }
    return w;
}

bool has_sponge(const st_wave_args* wa) { return wa && wa->sponge_width > 0; }

bool use_tb2(const st_plan* pl) {
    return pl->cfg.variant == ST_VARIANT_WAVE3D && pl->cfg.tsteps == 2 &&
           wave3d_tb2_supported(pl->prob.radius);
}

// Forward leapfrog with two fused steps per launch.  A fused launch must not
// write either of its inputs (other workgroups read their halos), so its
// outputs rotate over three buffer pairs: A = (caller prev, caller out),
// B and C in the workspace.  The pairs are chosen backwards from the last
// launch (which writes A) as B, C, B, C, ...; the first launch therefore
// never writes A, whose prev buffer is one of its inputs.  An odd step count
// starts with one single-step launch done in place on the prev buffer.
st_status run_wave_tb2(const st_plan* pl, const void* u_in, void* u_out, int steps,
                       const st_wave_args* wa, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t cells = cells_of(pl->prob);
    const size_t gb = (cells * 4 + 255) / 256 * 256;
    if (!ws || ws_bytes < 4 * gb) ST_FAIL(ST_EWORKSPACE, "workspace of %zu bytes needed", 4 * gb);
    const Geom g = geom_of(pl->prob);
    const size_t plane = (size_t)pl->prob.n[0] * pl->prob.n[1];
    float* P = (float*)wa->u_prev;
    float* O = (float*)u_out;
    float* W[4] = {(float*)ws, (float*)((char*)ws + gb), (float*)((char*)ws + 2 * gb),
                   (float*)((char*)ws + 3 * gb)};
    const float* prev = P;
    const float* cur = (const float*)u_in;
    const bool has_src = wa->src[0] >= 0 && wwavelet(wa);
    const bool rec = wa->rec_z >= 0 && wtraces(wa);
    int t = 0;
    if (steps % 2 == 1) {
        // One single step in place on the prev buffer: (P, I) -> (I, P).
        WaveLaunch w = wave_base();
        w.prev = P;
        w.cur = cur;
        w.next = P;
        w.kappa = wkappa(wa);
        if (has_src) {
            w.src_x = (int)wa->src[0];
            w.src_y = (int)wa->src[1];
            w.src_z = (int)wa->src[2];
            w.src_amp = wwavelet(wa);
        }
        if (rec) {
            w.rec_z = (int)wa->rec_z;
            w.trace_t = wtraces(wa);
        }
        HIP_TRY(wave_forward_launch(pl, w, s));
        prev = cur;
        cur = P;
        t = 1;
    }
    const int L = (steps - t) / 2;
    if (L == 1 && (prev == P || cur == P || cur == O)) {
        // The only fused launch cannot write A; land in B and copy.
        WaveTB2 w{};
        w.prev = prev; w.cur = cur; w.out1 = W[0]; w.out2 = W[1]; w.kappa = wkappa(wa);
        w.src_x = has_src ? (int)wa->src[0] : -1; w.src_y = (int)wa->src[1]; w.src_z = (int)wa->src[2];
        w.amp1 = has_src ? wwavelet(wa) + t : nullptr; w.amp2 = has_src ? wwavelet(wa) + t + 1 : nullptr;
        w.rec_z = rec ? (int)wa->rec_z : -1;
        w.trace1 = rec ? wtraces(wa) + (size_t)t * plane : nullptr;
        w.trace2 = rec ? wtraces(wa) + (size_t)(t + 1) * plane : nullptr;
        HIP_TRY(launch_wave3d_tb2(g, pl->cfg, pl->taps, w, s));
        HIP_TRY(hipMemcpyAsync(P, W[0], cells * 4, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(O, W[1], cells * 4, hipMemcpyDeviceToDevice, s));
        return ST_OK;
    }
    for (int j = 1; j <= L; ++j) {
        float* o1;
        float* o2;
        const int back = L - j;          // launches after this one
        if (back == 0) { o1 = P; o2 = O; }
        else if (back % 2 == 1) { o1 = W[0]; o2 = W[1]; }
        else { o1 = W[2]; o2 = W[3]; }
        WaveTB2 w{};
        w.prev = prev; w.cur = cur; w.out1 = o1; w.out2 = o2; w.kappa = wkappa(wa);
        w.src_x = has_src ? (int)wa->src[0] : -1; w.src_y = (int)wa->src[1]; w.src_z = (int)wa->src[2];
        w.amp1 = has_src ? wwavelet(wa) + t : nullptr; w.amp2 = has_src ? wwavelet(wa) + t + 1 : nullptr;
        w.rec_z = rec ? (int)wa->rec_z : -1;
        w.trace1 = rec ? wtraces(wa) + (size_t)t * plane : nullptr;
        w.trace2 = rec ? wtraces(wa) + (size_t)(t + 1) * plane : nullptr;
        HIP_TRY(launch_wave3d_tb2(g, pl->cfg, pl->taps, w, s));
        prev = o1;
        cur = o2;
        t += 2;
    }
    return ST_OK;
}

// Leapfrog (forward or adjoint) over `steps` steps with the buffer schedule
// b_t = out if (T - t) even else prev_buf, so u_T ends in u_out and u_{T-1}
// in the caller's prev buffer.
st_status run_wave(const st_plan* pl, bool adjoint, const void* u_in, void* u_out, int steps,
                   const st_wave_args* wa, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t gb = grid_bytes(pl->prob);
    float* P = (float*)wa->u_prev;
    float* O = (float*)u_out;
    const float* cur = (const float*)u_in;
    if (steps == 0) {
        if (u_in != u_out) HIP_TRY(hipMemcpyAsync(u_out, u_in, gb, hipMemcpyDeviceToDevice, s));
        return ST_OK;
    }
    if (!adjoint && steps >= 2 && use_tb2(pl) && !has_sponge(wa))
        return run_wave_tb2(pl, u_in, u_out, steps, wa, ws, ws_bytes, s);
    if (u_in == u_out && (steps % 2) == 1) {
        if (!ws || ws_bytes < gb) ST_FAIL(ST_EWORKSPACE, "workspace of %zu bytes needed", gb);
        HIP_TRY(hipMemcpyAsync(ws, u_in, gb, hipMemcpyDeviceToDevice, s));
        cur = (const float*)ws;
    }
    const Geom g = plan_geom(pl);
    const float* prev = P;
    const size_t plane = (size_t)pl->prob.n[0] * pl->prob.n[1];
    for (int t = 0; t < steps; ++t) {
        float* next = ((steps - (t + 1)) % 2 == 0) ? O : P;
        WaveLaunch w = wave_base(wa);
        w.prev = prev;
        w.cur = cur;
        w.next = next;
        w.kappa = wkappa(wa);
        if (!adjoint) {
            if (wa->src[0] >= 0 && wwavelet(wa)) {
                w.src_x = (int)wa->src[0];
                w.src_y = (int)wa->src[1];
                w.src_z = (int)wa->src[2];
                w.src_amp = wwavelet(wa) + t;
            }
            if (wa->rec_z >= 0 && wtraces(wa)) {
                w.rec_z = (int)wa->rec_z;
                w.trace_t = wtraces(wa) + (size_t)t * plane;
            }
            HIP_TRY(wave_forward_launch(pl, w, s));
        } else {
            // The first transposed step takes the co-state of u_{T-1} as is;
            // later ones take B l_{t+2} (damped layer).
            w.prev_sign = t == 0 ? -1.f : 1.f;
            w.prev_damped = t != 0;
            HIP_TRY(launch_wave_adjoint(g, pl->adj_cfg, pl->taps_t, pl->taps, kWaveAdj, w, s));
        }
        prev = cur;
        cur = next;
    }
    // u_{T-1} (or lambda_1) must end in the caller's prev buffer.
    if (prev != P) HIP_TRY(hipMemcpyAsync(P, prev, gb, hipMemcpyDeviceToDevice, s));
    // Co-state of u_{-1}: -l_1, or -B l_1 with the absorbing layer.
    if (adjoint && has_sponge(wa))
        HIP_TRY(launch_sponge_scale(g, P, -1.f, wa->sponge_width, wa->sponge_strength, s));
    else if (adjoint)
        HIP_TRY(launch_scale(P, P, -1.f, cells_of(pl->prob), s));
    return ST_OK;
}

// FP64 forward leapfrog, with run_wave's buffer schedule (u_T ends in u_out,
// u_{T-1} in the caller's prev buffer).
st_status run_wave_f64(const st_plan* pl, const void* u_in, void* u_out, int steps, const st_wave_args* wa,
                       void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t gb = grid_bytes(pl->prob);
    double* P = static_cast<double*>(wa->u_prev);
    double* O = static_cast<double*>(u_out);
    const double* cur = static_cast<const double*>(u_in);
    if (steps == 0) {
        if (u_in != u_out) HIP_TRY(hipMemcpyAsync(u_out, u_in, gb, hipMemcpyDeviceToDevice, s));
        return ST_OK;
    }
    if (u_in == u_out && (steps % 2) == 1) {
        if (!ws || ws_bytes < gb) ST_FAIL(ST_EWORKSPACE, "workspace of %zu bytes needed", gb);
        HIP_TRY(hipMemcpyAsync(ws, u_in, gb, hipMemcpyDeviceToDevice, s));
        cur = static_cast<const double*>(ws);
    }
    const Geom g = plan_geom(pl);
    const double* prev = P;
    const size_t plane = (size_t)pl->prob.n[0] * pl->prob.n[1];
    for (int t = 0; t < steps; ++t) {
        double* next = ((steps - (t + 1)) % 2 == 0) ? O : P;
        WaveLaunchF64 w;
        memset(&w, 0, sizeof w);
        w.prev = prev;
        w.cur = cur;
        w.next = next;
        w.kappa = static_cast<const double*>(wa->kappa);
        w.src_x = -1;
        w.rec_z = -1;
        if (wa->src[0] >= 0 && wa->wavelet) {
            w.src_x = (int)wa->src[0];
            w.src_y = (int)wa->src[1];
            w.src_z = (int)wa->src[2];
            w.src_amp = static_cast<const double*>(wa->wavelet) + t;
        }
        if (wa->rec_z >= 0 && wa->traces) {
            w.rec_z = (int)wa->rec_z;
            w.trace_t = static_cast<double*>(wa->traces) + (size_t)t * plane;
        }
        if (wa->sponge_width > 0) {
            w.sp_w = wa->sponge_width;
            w.sp_s = (double)wa->sponge_strength;
        }
        HIP_TRY(launch_wave3d_f64(g, pl->cfg, pl->taps64, w, s));
        prev = cur;
        cur = next;
    }
    if (prev != P) HIP_TRY(hipMemcpyAsync(P, prev, gb, hipMemcpyDeviceToDevice, s));
    return ST_OK;
}

st_status check_wave_args(const st_plan* pl, const st_wave_args* wa, bool need_kappa) {
    if (!wa) ST_FAIL(ST_EINVAL, "wave plan needs st_wave_args");
    if (!wa->u_prev) ST_FAIL(ST_EINVAL, "wave->u_prev is NULL");
    if (need_kappa && !wkappa(wa)) ST_FAIL(ST_EINVAL, "wkappa(wave) is NULL");
    const st_problem& p = pl->prob;
    if (wa->src[0] >= 0) {
        for (int a = 0; a < 3; ++a)
            if (wa->src[a] < 0 || wa->src[a] >= p.n[a]) ST_FAIL(ST_EINVAL, "source outside the grid");
    }
    if (wa->rec_z >= p.n[2] || wa->rec_z < -1) ST_FAIL(ST_EINVAL, "receiver plane outside the grid");
    if (wa->sponge_width != 0 || wa->sponge_strength != 0.f) {
        const int64_t nmin = std::min(p.n[0], std::min(p.n[1], p.n[2]));
        if (wa->sponge_width < 0 || wa->sponge_width > nmin / 2)
            ST_FAIL(ST_EINVAL, "sponge_width must lie in 0..min(n)/2");
        if (!(wa->sponge_strength >= 0.f && wa->sponge_strength <= 4.f))
            ST_FAIL(ST_EINVAL, "sponge_strength must lie in [0, 4]");
    }
    if (wa->sponge_width > 0) {
        if (p.boundary != ST_ZERO) ST_FAIL(ST_EUNSUPPORTED, "the absorbing layer needs the zero frame");
        if (p.dtype != ST_F64 &&
            (pl->cfg.variant != ST_VARIANT_WAVE3D_LDS || pl->adj_cfg.variant != ST_VARIANT_WAVE3D_LDS))
            ST_FAIL(ST_EUNSUPPORTED, "the absorbing layer is fused into the LDS-ring kernels only");
    }
    return ST_OK;
}

}  // namespace

extern "C" {

const char* stencil_last_error(void) { return stk::last_error(); }

const char* stencil_version(void) { return "libstencil 0.1 (gfx950)"; }

st_status stencil_plan(const st_problem* problem, const st_plan_opts* opts, st_plan** out) {
    stk::set_error("%s", "");
    if (!out) ST_FAIL(ST_EINVAL, "out is NULL");
    *out = nullptr;
    return build_plan(problem, opts, out);
}

void stencil_plan_destroy(st_plan* plan) {
    if (!plan) return;
    for (st_plan* m : plan->members) stencil_plan_destroy(m);
    if (plan->stage_event) {
        (void)hipEventSynchronize(plan->stage_event);
        (void)hipEventDestroy(plan->stage_event);
    }
    if (plan->stage) (void)hipHostFree(plan->stage);
    delete plan;
}

st_status stencil_plan_describe(const st_plan* plan, int32_t* variant, int32_t* tile_x,
                                int32_t* tile_y, int32_t* tsteps, int32_t* zchunk) {
    if (!plan) ST_FAIL(ST_EINVAL, "plan is NULL");
    const LaunchCfg& c = plan->cfg;   // batched: the grouped launch (row march, batch depth)
    if (variant) *variant = c.variant;
    if (tile_x) *tile_x = c.tile_x;
    if (tile_y) *tile_y = c.tile_y;
    if (tsteps) *tsteps = c.tsteps;
    if (zchunk) *zchunk = c.zchunk;
    return ST_OK;
}

st_status stencil_plan_describe_reverse(const st_plan* plan, int32_t* variant, int32_t* tile_x,
                                        int32_t* tile_y, int32_t* tsteps, int32_t* zchunk) {
    stk::set_error("%s", "");
    if (!plan || plan->batched || plan->prob.update != ST_WAVE) ST_FAIL(ST_EINVAL, "needs a wave plan");
    const LaunchCfg& c = plan->adj_cfg;
    if (variant) *variant = c.variant;
    if (tile_x) *tile_x = c.tile_x;
    if (tile_y) *tile_y = c.tile_y;
    if (tsteps) *tsteps = c.tsteps;
    if (zchunk) *zchunk = c.zchunk;
    return ST_OK;
}

st_status stencil_plan_coefficients(const st_plan* plan, float* dense, int32_t count, double* weight_sum) {
    stk::set_error("%s", "");
    if (!plan || plan->batched) ST_FAIL(ST_EINVAL, "needs a single-grid plan");
    if (count < 0) ST_FAIL(ST_EINVAL, "count must be >= 0");
    if (dense) {
        const size_t m = std::min((size_t)count, plan->dense.size());
        for (size_t i = 0; i < m; ++i) dense[i] = plan->dense[i];
    }
    if (weight_sum) *weight_sum = (double)plan->taps.sum;
    return ST_OK;
}

size_t stencil_workspace_bytes(const st_plan* plan, int32_t steps, int32_t mode);

st_status stencil_apply(const st_plan* plan, const void* u_in, void* u_out, int32_t steps,
                        const st_wave_args* wave, void* workspace, size_t ws_bytes, void* stream) {
    stk::set_error("%s", "");
    if (!plan) ST_FAIL(ST_EINVAL, "plan is NULL");
    if (plan->batched) ST_FAIL(ST_EINVAL, "batched plan: use stencil_apply_batched");
    if (!u_in || !u_out) ST_FAIL(ST_EINVAL, "grid pointer is NULL");
    if (steps < 0) ST_FAIL(ST_EINVAL, "steps must be >= 0");
    if (plan->prob.update == ST_WAVE) {
        st_status s = check_wave_args(plan, wave, true);
        if (s != ST_OK) return s;
        if (wave->u_prev == u_in || wave->u_prev == u_out)
            ST_FAIL(ST_EINVAL, "wave->u_prev must not alias u_in or u_out");
        if (plan->prob.dtype == ST_F64)
            return run_wave_f64(plan, u_in, u_out, steps, wave, workspace, ws_bytes, as_stream(stream));
        return run_wave(plan, false, u_in, u_out, steps, wave, workspace, ws_bytes, as_stream(stream));
    }
    if (plan->prob.update == ST_VARCOEF) ST_FAIL(ST_EINVAL, "variable-coefficient plan: use stencil_apply_varcoef");
    if (wave) ST_FAIL(ST_EINVAL, "linear plan takes no wave arguments");
    return run_linear(plan, plan->taps, u_in, u_out, steps, workspace, ws_bytes, as_stream(stream));
}

namespace {
// `steps` variable-coefficient steps from u_in into u_out through the
// workspace, with run_linear's buffer schedule (one step per launch).
st_status run_varcoef(const st_plan* pl, bool adjoint, const void* u_in, void* u_out, const void* fields,
                      int steps, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t gb = grid_bytes(pl->prob);
    if (steps == 0) {
        if (u_in != u_out) HIP_TRY(hipMemcpyAsync(u_out, u_in, gb, hipMemcpyDeviceToDevice, s));
        return ST_OK;
    }
    if (!ws || ws_bytes < gb) ST_FAIL(ST_EWORKSPACE, "workspace of %zu bytes needed", gb);
    const Geom g = geom_of(pl->prob);
    const void* cur = u_in;
    if (u_in == u_out && (steps % 2) == 1) {
        HIP_TRY(hipMemcpyAsync(ws, u_in, gb, hipMemcpyDeviceToDevice, s));
        cur = ws;
    }
    for (int j = 1; j <= steps; ++j) {
        void* dst = ((steps - j) % 2 == 0) ? u_out : ws;
        HIP_TRY(launch_vc3d(g, pl->cfg, cur, dst, fields, adjoint, s));
        cur = dst;
    }
    return ST_OK;
}

st_status varcoef_entry(const st_plan* plan, bool adjoint, const void* u_in, void* u_out, const void* fields,
                        int32_t steps, void* workspace, size_t ws_bytes, void* stream) {
    stk::set_error("%s", "");
    if (!plan) ST_FAIL(ST_EINVAL, "plan is NULL");
    if (plan->batched || plan->prob.update != ST_VARCOEF)
        ST_FAIL(ST_EINVAL, "stencil_apply_varcoef needs an ST_VARCOEF plan");
    if (!u_in || !u_out || !fields) ST_FAIL(ST_EINVAL, "grid or field pointer is NULL");
    if (steps < 0) ST_FAIL(ST_EINVAL, "steps must be >= 0");
    return run_varcoef(plan, adjoint, u_in, u_out, fields, steps, workspace, ws_bytes, as_stream(stream));
}
}  // namespace

st_status stencil_apply_varcoef(const st_plan* plan, const void* u_in, void* u_out, const void* fields,
                                int32_t steps, void* workspace, size_t ws_bytes, void* stream) {
    return varcoef_entry(plan, false, u_in, u_out, fields, steps, workspace, ws_bytes, stream);
}

st_status stencil_apply_varcoef_adjoint(const st_plan* plan, const void* v_in, void* v_out, const void* fields,
                                        int32_t steps, void* workspace, size_t ws_bytes, void* stream) {
    return varcoef_entry(plan, true, v_in, v_out, fields, steps, workspace, ws_bytes, stream);
}

st_status stencil_apply_adjoint(const st_plan* plan, const void* v_in, void* v_out, int32_t steps,
                                const st_wave_args* wave, void* workspace, size_t ws_bytes,
                                void* stream) {
    stk::set_error("%s", "");
    if (!plan) ST_FAIL(ST_EINVAL, "plan is NULL");
    if (plan->batched) ST_FAIL(ST_EINVAL, "batched plans have no adjoint entry point");
    if (!v_in || !v_out) ST_FAIL(ST_EINVAL, "grid pointer is NULL");
    if (steps < 0) ST_FAIL(ST_EINVAL, "steps must be >= 0");
    if (plan->prob.update == ST_WAVE) {
        if (plan->prob.dtype == ST_F64) ST_FAIL(ST_EUNSUPPORTED, "the wave adjoint takes f32 plans");
        st_status s = check_wave_args(plan, wave, true);
        if (s != ST_OK) return s;
        if (wave->u_prev == v_in || wave->u_prev == v_out)
            ST_FAIL(ST_EINVAL, "wave->u_prev must not alias v_in or v_out");
        return run_wave(plan, true, v_in, v_out, steps, wave, workspace, ws_bytes, as_stream(stream));
    }
    if (plan->prob.update == ST_VARCOEF)
        ST_FAIL(ST_EINVAL, "variable-coefficient plan: use stencil_apply_varcoef_adjoint");
    if (wave) ST_FAIL(ST_EINVAL, "linear plan takes no wave arguments");
    return run_linear(plan, plan->taps_t, v_in, v_out, steps, workspace, ws_bytes, as_stream(stream));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Checkpointed gradient of the receiver misfit with respect to kappa.
// ---------------------------------------------------------------------------
namespace {

struct GradLayout {
    int T, K, S;
    size_t grid;        // bytes per f32 grid
    size_t ckpt_off;    // 2*(S-1) grids: checkpoints of segments 1..S-1
    size_t states_off;  // K grids of the segment being reversed: u_{t0+1}..u_{t0+K} (queue
                        // kernels) or L(u_{t0})..L(u_{t0+K-1}) (ring kernels)
    size_t scratch_off; // 3 grids: forward rotation
    size_t lam_off;     // 2 grids: adjoint ping-pong
    size_t traces_off;  // T planes
    size_t part_off;    // loss partial sums
    size_t total;
};

GradLayout grad_layout(const st_plan* pl, int steps) {
    GradLayout L;
    L.T = steps;
    L.K = std::max(1, std::min(pl->ckpt_every, std::max(1, steps)));
    L.S = (steps + L.K - 1) / L.K;
    const size_t align = 256;
    L.grid = (cells_of(pl->prob) * 4 + align - 1) / align * align;
    const size_t plane = (size_t)pl->prob.n[0] * pl->prob.n[1] * 4;
    size_t off = 0;
    L.ckpt_off = off;
    off += (size_t)2 * std::max(0, L.S - 1) * L.grid;
    L.states_off = off;
    off += (size_t)L.K * L.grid;
    L.scratch_off = off;
    off += 3 * L.grid;
    L.lam_off = off;
    off += 2 * L.grid;
    L.traces_off = off;
    off += ((size_t)steps * plane + align - 1) / align * align;
    L.part_off = off;
    off += sizeof(double) * kLossParts;
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

size_t stencil_workspace_bytes(const st_plan* plan, int32_t steps, int32_t mode) {
    if (!plan) return 0;
    if (plan->batched && mode == 2) {
        size_t m = batch_tune_bytes(plan);
        for (const st_plan* x : plan->members) m = std::max(m, stencil_workspace_bytes(x, 0, 2));
        return m;
    }
    if (plan->batched) {
        size_t total = 0;
        for (const st_plan* m : plan->members) total += (grid_bytes(m->prob) + 255) / 256 * 256;
        return total + batched_meta_bytes(plan, steps);
    }
    if (mode == 1) return plan->prob.update == ST_WAVE && steps > 0 ? grad_layout(plan, steps).total : 0;
    if (mode == 0 && plan->prob.update == ST_WAVE && use_tb2(plan))
        return 4 * ((grid_bytes(plan->prob) + 255) / 256 * 256);
    if (mode == 2) {
        const size_t gb = (grid_bytes(plan->prob) + 255) / 256 * 256;
        const size_t kb = plan->prob.update == ST_WAVE      ? gb
                          : plan->prob.update == ST_VARCOEF ? (size_t)(varcoef_taps(plan->prob) + 1) * gb
                                                            : 0;
        // A wave plan also tunes its reverse step (fields past tune_one's).
        return 4 * gb + kb + 64 + (plan->prob.update == ST_WAVE ? reverse_tune_bytes(plan->prob) : 0);
    }
    return grid_bytes(plan->prob);
}

st_status stencil_wave_gradient(const st_plan* plan, const void* u0, const st_wave_args* wave,
                                int32_t steps, float* dkappa, double* loss_dev, void* workspace,
                                size_t ws_bytes, void* stream) {
    stk::set_error("%s", "");
    if (!plan) ST_FAIL(ST_EINVAL, "plan is NULL");
    if (plan->prob.update != ST_WAVE) ST_FAIL(ST_EINVAL, "gradient needs a wave plan");
    if (plan->prob.dtype == ST_F64) ST_FAIL(ST_EUNSUPPORTED, "the wave gradient takes f32 plans");
    if (!u0 || !dkappa || !loss_dev) ST_FAIL(ST_EINVAL, "u0, dkappa and loss must be non-NULL");
    if (steps < 1) ST_FAIL(ST_EINVAL, "steps must be >= 1");
    st_status st = check_wave_args(plan, wave, true);
    if (st != ST_OK) return st;
    if (wave->rec_z < 0 || !wave->target) ST_FAIL(ST_EINVAL, "gradient needs rec_z >= 0 and target");
    const GradLayout L = grad_layout(plan, steps);
    if (!workspace || ws_bytes < L.total)
        ST_FAIL(ST_EWORKSPACE, "workspace of %zu bytes needed", L.total);
    hipStream_t s = as_stream(stream);
    char* ws = (char*)workspace;
    const Geom g = plan_geom(plan);
    const size_t plane = (size_t)plan->prob.n[0] * plan->prob.n[1];
    const int T = L.T, K = L.K, S = L.S;
    auto ckpt = [&](int seg, int which) -> float* {   // seg >= 1; which 0 = u_{sK-1}, 1 = u_{sK}
        return (float*)(ws + L.ckpt_off + (size_t)(2 * (seg - 1) + which) * L.grid);
    };
    float* scratch[3] = {(float*)(ws + L.scratch_off), (float*)(ws + L.scratch_off + L.grid),
                         (float*)(ws + L.scratch_off + 2 * L.grid)};
    float* traces = wtraces(wave) ? wtraces(wave) : (float*)(ws + L.traces_off);
    const bool has_src = wave->src[0] >= 0 && wwavelet(wave);

    auto fwd_step = [&](const float* prev, const float* cur, float* next, int t, bool record,
                        float* lap_out = nullptr) {
        WaveLaunch w = wave_base(wave);
        // The misfit gradient is linear in the small residual P u - d, which
        // amplifies the states' rounding by |d| / |r|: the gradient's forward
        // and recompute steps round each state once (FP64 update).
        w.exact_update = true;
        w.prev = prev;
        w.cur = cur;
        w.next = next;
        w.kappa = wkappa(wave);
        w.lap_out = lap_out;
        if (has_src) {
            w.src_x = (int)wave->src[0];
            w.src_y = (int)wave->src[1];
            w.src_z = (int)wave->src[2];
            w.src_amp = wwavelet(wave) + t;
        }
        if (record) {
            w.rec_z = (int)wave->rec_z;
            w.trace_t = traces + (size_t)t * plane;
        }
        return wave_forward_launch(plan, w, s);
    };
    auto pick = [&](const float* a, const float* b) -> float* {
        for (float* c : scratch)
            if (c != a && c != b) return c;
        return nullptr;
    };

    // With the LDS-ring kernels the recompute also writes L(u_t) (4 more
    // bytes per cell) and the reverse step takes it pointwise, with u_t on
    // the receiver plane from the recorded traces: the reverse kernel then
    // stages one field instead of two.  The queue kernels keep the states.
    const bool pointwise = plan->cfg.variant == ST_VARIANT_WAVE3D_LDS &&
                           plan->adj_cfg.variant == ST_VARIANT_WAVE3D_LDS;
    const int t_last = (S - 1) * K;   // first step of the last segment
    auto lap = [&](int t, int t0) { return (float*)(ws + L.states_off + (size_t)(t - t0) * L.grid); };

    // Forward: record traces, keep (u_{sK-1}, u_{sK}) for s = 1..S-1.  The
    // last segment is reversed first, right after this pass, so (pointwise
    // reverse) its steps write L(u_t) now and it needs no recompute.
    const float* prev = (const float*)wave->u_prev;
    const float* cur = (const float*)u0;
    for (int t = 0; t < T; ++t) {
        const int tn = t + 1;   // this step produces u_tn
        float* as_prev = nullptr;   // ckpt slot holding u_{sK-1}
        float* as_cur = nullptr;    // ckpt slot holding u_{sK}
        if ((tn + 1) % K == 0 && (tn + 1) / K >= 1 && (tn + 1) / K < S) as_prev = ckpt((tn + 1) / K, 0);
        if (tn % K == 0 && tn / K >= 1 && tn / K < S) as_cur = ckpt(tn / K, 1);
        float* next = as_cur ? as_cur : (as_prev ? as_prev : pick(prev, cur));
        HIP_TRY(fwd_step(prev, cur, next, t, true, pointwise && t >= t_last ? lap(t, t_last) : nullptr));
        if (as_cur && as_prev)   // K == 1: the same state opens two checkpoints
            HIP_TRY(hipMemcpyAsync(as_prev, as_cur, cells_of(plan->prob) * 4, hipMemcpyDeviceToDevice, s));
        prev = cur;
        cur = next;
    }
    HIP_TRY(launch_trace_loss(traces, wave->target, (size_t)T * plane, (double*)(ws + L.part_off),
                              loss_dev, s));

    // Backward, segment by segment.
    float* lam[2] = {(float*)(ws + L.lam_off), (float*)(ws + L.lam_off + L.grid)};
    HIP_TRY(launch_fill(lam[0], 0.f, cells_of(plan->prob), s));
    HIP_TRY(launch_fill(lam[1], 0.f, cells_of(plan->prob), s));
    HIP_TRY(launch_fill(dkappa, 0.f, cells_of(plan->prob), s));
    float* l_next = lam[0];   // lambda_{t+1}
    float* l_next2 = lam[1];  // lambda_{t+2}
    for (int seg = S - 1; seg >= 0 && pointwise; --seg) {
        const int t0 = seg * K;
        const int t1 = std::min(t0 + K, T);
        const float* p = seg == 0 ? (const float*)wave->u_prev : ckpt(seg, 0);
        const float* c = seg == 0 ? (const float*)u0 : ckpt(seg, 1);
        // Recompute u_{t+1} and L(u_t) for the segment (the last one has
        // them from the forward pass).
        for (int t = t0; t < t1 && seg < S - 1; ++t) {
            float* nx = pick(p, c);
            HIP_TRY(fwd_step(p, c, nx, t, false, lap(t, t0)));
            p = c;
            c = nx;
        }
        const int tstart = (seg == S - 1) ? T : t1 - 1;
        for (int t = tstart; t >= t0; --t) {
            WaveLaunch w = wave_base(wave);
            w.prev = l_next2;
            w.cur = l_next;
            w.next = l_next2;   // lambda_t overwrites lambda_{t+2} in place
            w.kappa = wkappa(wave);
            w.grad = dkappa;
            w.lap = t <= T - 1 ? lap(t, t0) : nullptr;   // lambda_{T+1} = 0: no term at t = T
            w.rec_z = (int)wave->rec_z;
            w.target_t = t >= 1 ? wave->target + (size_t)(t - 1) * plane : nullptr;
            w.trace_res = t >= 1 ? traces + (size_t)(t - 1) * plane : nullptr;   // u_t[rec_z]
            HIP_TRY(launch_wave_adjoint(g, plan->adj_cfg, plan->taps_t, plan->taps, kWaveGradPt, w, s));
            std::swap(l_next, l_next2);
        }
    }
    for (int seg = S - 1; seg >= 0 && !pointwise; --seg) {
        const int t0 = seg * K;
        const int t1 = std::min(t0 + K, T);
        const float* base_prev = seg == 0 ? (const float*)wave->u_prev : ckpt(seg, 0);
        const float* base_cur = seg == 0 ? (const float*)u0 : ckpt(seg, 1);
        auto state = [&](int t) -> const float* {   // u_t for t in [t0, t1]
            if (t == t0) return base_cur;
            return (const float*)(ws + L.states_off + (size_t)(t - t0 - 1) * L.grid);
        };
        const int tstart = (seg == S - 1) ? T : t1 - 1;
        // Recompute u_{t0+1}..u_{tstart}.
        const float* p = base_prev;
        const float* c = base_cur;
        for (int t = t0; t < tstart; ++t) {
            float* nx = (float*)state(t + 1);
            HIP_TRY(fwd_step(p, c, nx, t, false));
            p = c;
            c = nx;
        }
        for (int t = tstart; t >= t0; --t) {
            WaveLaunch w = wave_base();
            w.prev = l_next2;
            w.cur = l_next;
            w.next = l_next2;   // lambda_t overwrites lambda_{t+2} in place
            w.kappa = wkappa(wave);
            w.u = state(t);
            w.grad = dkappa;
            w.rec_z = (int)wave->rec_z;
            w.target_t = t >= 1 ? wave->target + (size_t)(t - 1) * plane : nullptr;
            HIP_TRY(launch_wave_adjoint(g, plan->adj_cfg, plan->taps_t, plan->taps, kWaveGrad, w, s));
            std::swap(l_next, l_next2);
        }
    }
    return ST_OK;
}

}  // extern "C"
