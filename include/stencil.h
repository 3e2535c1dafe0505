/*
 * stencil.h - C ABI of libstencil, repeated stencil sweeps on AMD MI355X.
 *
 * A case is the pair (offset geometry S, coefficients c_d) driving a
 * time-stepped sweep over a regular grid (Section 2.1, the linear
 * constant-coefficient form of the update rule):
 *
 *     u^{t+1}(x) = sum_{d in S} c_d u^t(B(x + d)),
 *
 * where S is a star (offsets along the axes) or a box (the full cube) of
 * order r = max |d|_inf (Section 2.1, stencil type), and B is the boundary
 * rule.  Each (dimension, shape, radius, storage precision, boundary, grid
 * class) case is served by its own specialised kernel chosen through a
 * dispatch map (Section 4.2, the operator map; Section 7.2.1, dispatch of
 * configurations to structurally distinct kernels).
 *
 * Conventions shared by every entry point
 *  - Layout: row-major, x unit-stride.  2D grids are [ny][nx], 3D grids are
 *    [nz][ny][nx]; n[0] = nx, n[1] = ny, n[2] = nz (n[2] = 1 in 2D).
 *  - Coefficients: a HOST array of (2r+1)^ndim floats ordered (dz, dy, dx)
 *    lexicographically with dx fastest.  Entries outside the shape must be
 *    zero.  The plan copies them; the caller keeps ownership.
 *  - Storage: ST_F32 or ST_F16 (IEEE binary16).  Arithmetic is always FP32;
 *    fp16 results are rounded to nearest even once per time step.
 *  - Device buffers: every pointer named "device" is memory the CALLER
 *    allocated on the current HIP device and still owns.  The library never
 *    allocates device memory; scratch space comes from the caller's
 *    workspace, sized by stencil_workspace_bytes().
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls are asynchronous on that stream unless stated.
 *  - Errors: every call returns a status.  Argument and shape errors are
 *    detected on the host before any HIP call.  Kernel faults surface at the
 *    caller's next synchronisation.  stencil_last_error() returns a
 *    thread-local message for the most recent failure.  The library never
 *    aborts the process.
 */
#ifndef STENCIL_H
#define STENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ST_OK = 0,
    ST_EINVAL = 1,        /* null pointer, bad enum, negative steps, bad opts */
    ST_ESHAPE = 2,        /* grid extent too small for the radius, or too large */
    ST_EUNSUPPORTED = 3,  /* legal but not provided (e.g. box r > 2, fp16 wave) */
    ST_EWORKSPACE = 4,    /* workspace missing or smaller than required */
    ST_EHIP = 5,          /* a HIP runtime call or kernel launch failed */
    ST_ENOMEM = 6,        /* host allocation failed */
    ST_ETUNE = 7          /* autotuning found no candidate that passed parity */
} st_status;

/* Storage type of the grid.  ST_F32 and ST_F16 (IEEE binary16, rounded to
 * nearest even on every store) compute in f32; ST_F64 computes in f64 with
 * the f32 coefficient values widened exactly (linear sweeps, single and
 * batched, and variable-coefficient sweeps; not the wave update).
 * Section 2.1 names f16/f32/f64 as the precision axis of a case. */
typedef enum { ST_F32 = 0, ST_F16 = 1, ST_F64 = 2 } st_dtype;
typedef enum { ST_PERIODIC = 0, ST_ZERO = 1 } st_boundary;
typedef enum { ST_STAR = 0, ST_BOX = 1 } st_shape;

/* ST_LINEAR:  the weighted-sum sweep above.
 * ST_WAVE:    acoustic leapfrog u_{t+1} = 2 u_t - u_{t-1} + kappa (.) L(u_t),
 *             L a star stencil, kappa a per-cell coefficient field (Section
 *             2.1: a spatially varying coefficient is one more array to read).
 * ST_VARCOEF: the sweep with one coefficient field per offset,
 *             u'(x) = sum_k f_k(x) u(B(x + d_k)) (Section 2.1, variable
 *             coefficients); applied by stencil_apply_varcoef.  2D or 3D,
 *             star r = 1..4 or box r = 1; `coeffs` is ignored (may be NULL). */
typedef enum { ST_LINEAR = 0, ST_WAVE = 1, ST_VARCOEF = 2 } st_update;

/* Kernel families a dispatch-map entry can name. */
typedef enum {
    ST_VARIANT_AUTO = 0,  /* let the dispatch map choose */
    ST_VARIANT_TB2D = 1,  /* 2D LDS tile, k fused time steps per launch */
    ST_VARIANT_ZM3D = 2,  /* 3D plane-streaming (z-march) with register queues */
    ST_VARIANT_WAVE3D = 3, /* 3D leapfrog z-march, fused source/receiver */
    ST_VARIANT_WAVE3D_LDS = 4, /* 3D leapfrog forward with z-neighbours in an LDS ring */
    ST_VARIANT_YM2D = 5,  /* 2D row march, k fused time steps held in LDS row rings */
    ST_VARIANT_ZM3D_MFMA = 6, /* 3D 27-point box, fp16 storage: in-plane contraction on MFMA */
    ST_VARIANT_VC3D = 7,  /* variable-coefficient plane march (ST_VARCOEF plans, 2D and 3D) */
    ST_VARIANT_ZM3D_H2 = 8, /* 3D box r = 1..2 or star r = 1, fp16 storage, even nx: two
                              cells per lane, packed-half dot products with f32 accumulation */
    ST_VARIANT_YM2D_H2 = 9, /* 2D box r = 1..2, fp16 storage, even nx: the row march on
                               packed-half dot products */
    ST_VARIANT_YM3D = 10  /* 3D box r = 1..2 marched along y (slabs with few z planes):
                             tile_y = z rows per workgroup, zchunk = y rows per chunk;
                             grids up to 4 GiB */
} st_variant;

typedef struct st_plan st_plan;   /* opaque; immutable after creation */

typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int64_t n[3];          /* nx, ny, nz: each 1..2^24, at most 2^36 cells, one
                              x-y plane under 2^31 cells; 3D and variable-
                              coefficient grids: one plane under 4 GiB */
    int32_t shape;         /* st_shape */
    int32_t radius;        /* 1..4; box: r <= 2 */
    const float *coeffs;   /* HOST, (2r+1)^ndim dense; for ST_WAVE may be NULL,
                              meaning the central second-difference Laplacian
                              of accuracy order 2r */
    int32_t dtype;         /* st_dtype (ST_WAVE: ST_F32, or ST_F64 for the forward
                              leapfrog of stencil_apply only) */
    int32_t boundary;      /* st_boundary */
    int32_t update;        /* st_update (ST_WAVE requires ndim 3, star) */
} st_problem;

/* Per-plan overrides.  Zero fields mean "dispatch map decides". */
typedef struct {
    int32_t variant;       /* st_variant */
    int32_t tile_x;        /* TB2D: output tile width (8..512);
                              YM2D: window width = threads per workgroup (256 or 512);
                              WAVE3D_LDS: planes staged per barrier (1, or 2 = the two
                              planes of a march step under one barrier) */
    int32_t tile_y;        /* TB2D: output tile height; YM2D: rows per chunk (0 = automatic);
                              ZM3D/WAVE3D: rows per workgroup */
    int32_t tsteps;        /* TB2D/YM2D: time steps fused per launch (1..16);
                              WAVE3D: 1, or 2 = two fused leapfrog steps (radius 2 or 4) */
    int32_t zchunk;        /* ZM3D/WAVE3D: planes per workgroup (0 = whole depth);
                              TB2D: waves per workgroup (0 = 4, or 8, 16) */
    int32_t ckpt_every;    /* wave gradient checkpoint interval (0 = 20) */
} st_plan_opts;

/* Extra operands of an ST_WAVE plan.  u_prev, kappa, wavelet and traces
 * hold values of the plan's storage type (float for ST_F32, double for
 * ST_F64); target is float (the gradient takes f32 plans only). */
typedef struct {
    void *u_prev;          /* device, cells: u_{-1} on entry, u_{T-1} on exit */
    const void *kappa;     /* device, cells */
    int64_t src[3];        /* point source (x, y, z); src[0] < 0 = none */
    const void *wavelet;   /* device, steps: wavelet[t] is added at src to u_{t+1} */
    int64_t rec_z;         /* receiver plane z index, -1 = none */
    void *traces;          /* device, steps*ny*nx or NULL: traces[t] = plane rec_z of u_{t+1} */
    const float *target;   /* device, steps*ny*nx: observed traces d (gradient only) */
    /* Absorbing layer (0 = none): a damping term gamma(x) u_t, from the
     * damped wave equation u_tt + gamma u_t = c^2 Lap u with central
     * differences in time, fused into the leapfrog (Section 4.3: stencils
     * fused with the application's physics):
     *   u_{t+1} = A (2 u_t + kappa L(u_t)) - B u_{t-1},
     *   A = 1 / (1 + gamma/2),  B = (1 - gamma/2) / (1 + gamma/2),
     * gamma(x) = sum over the three axes of s ((W - e) / W)^2 where the cell
     * lies within W cells of a face, e its distance to the nearer face (0
     * on a boundary cell), W = sponge_width, s = sponge_strength.  It needs
     * the zero frame and the LDS-ring kernels (ST_EUNSUPPORTED otherwise);
     * 0 <= W <= min(n) / 2 and 0 <= s <= 4, finite (ST_EINVAL otherwise).
     * An ST_F64 plan evaluates the layer in binary64 (its forward step only).
     * The same layer applies to stencil_apply, stencil_apply_adjoint (the
     * transpose of the damped state map) and stencil_wave_gradient. */
    int32_t sponge_width;
    float sponge_strength;
} st_wave_args;

/* Create a plan.  Validates the problem (ST_EINVAL / ST_ESHAPE /
 * ST_EUNSUPPORTED before any device work), classifies the case, looks up the
 * dispatch map (compiled-in defaults, then the tuning cache file named by the
 * STENCIL_TUNE_CACHE environment variable, then `opts`) and keeps a host copy
 * of the coefficients.  `opts` may be NULL.  On success *out owns the plan. */
st_status stencil_plan(const st_problem *problem, const st_plan_opts *opts, st_plan **out);

/* Release a plan.  NULL-safe. */
void stencil_plan_destroy(st_plan *plan);

/* Bytes of device workspace an operation needs for `steps` steps.
 * mode 0 = stencil_apply / stencil_apply_adjoint / stencil_apply_batched,
 * 1 = stencil_wave_gradient, 2 = stencil_autotune scratch.
 * Returns 0 for a NULL plan. */
size_t stencil_workspace_bytes(const st_plan *plan, int32_t steps, int32_t mode);

/* The variant, tile and temporal depth the plan dispatches to (any pointer
 * may be NULL).  Host only. */
st_status stencil_plan_describe(const st_plan *plan, int32_t *variant, int32_t *tile_x,
                                int32_t *tile_y, int32_t *tsteps, int32_t *zchunk);

/* The configuration of a wave plan's reverse step (the adjoint and gradient
 * launches of stencil_apply_adjoint and stencil_wave_gradient), which has a
 * dispatch-map cell of its own (Section 4.2's operator map, one more update
 * kind).  Any pointer may be NULL.  ST_EINVAL for a NULL, batched or non-wave
 * plan.  Host only. */
st_status stencil_plan_describe_reverse(const st_plan *plan, int32_t *variant, int32_t *tile_x,
                                        int32_t *tile_y, int32_t *tsteps, int32_t *zchunk);

/* The coefficients a plan applies (Section 2.1: the case's weights c_d).
 * `dense` (HOST, may be NULL) receives min(count, (2r+1)^ndim) floats in the
 * layout of st_problem.coeffs; for an ST_WAVE plan created without
 * coefficients these are the f32-rounded weights of the built-in Laplacian
 * (an ST_F64 wave plan applies its rationals rounded to binary64 instead).
 * *weight_sum (may be NULL) receives the weight sum the difference-form
 * kernels use, sum_{d != 0} c_d (u(x+d) - u(x)) + (weight sum) u(x): the
 * FP64 sum of the given weights, and exactly 0 for the built-in Laplacian
 * (its weights sum to 0 in real arithmetic; its rounded ones do not).
 * ST_EINVAL for a NULL or batched plan, or count < 0.  Host only. */
st_status stencil_plan_coefficients(const st_plan *plan, float *dense, int32_t count,
                                    double *weight_sum);

/* Forward sweep, `steps` time steps (Section 2.1 update rule, iterated).
 *  ST_LINEAR: u_out = A^steps u_in.  u_in == u_out is allowed; other overlap
 *             is not.  `wave` must be NULL.
 *  ST_WAVE:   u_in = u_0 and wave->u_prev = u_{-1}; on return u_out = u_T and
 *             wave->u_prev = u_{T-1}.  Source and receiver are optional.  An
 *             ST_F64 plan runs the leapfrog in binary64 with binary64 weights
 *             (the built-in Laplacian's rationals rounded once).
 * Device buffers hold n[0]*n[1]*n[2] values of the plan's storage type.
 * steps == 0 copies u_in to u_out. */
st_status stencil_apply(const st_plan *plan, const void *u_in, void *u_out, int32_t steps,
                        const st_wave_args *wave, void *workspace, size_t ws_bytes,
                        void *stream);

/* stencil_apply for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sweep, forward, for a single-grid ST_LINEAR or ST_WAVE plan, with the
 * workspace taken from a fixed device array of this library instead of the
 * caller.  The array holds stencil_noalloc_capacity() bytes (64 MiB) on each
 * GPU the library runs on, for the life of the process; a call whose
 * workspace (stencil_workspace_bytes(plan, steps, 0)) exceeds it returns
 * ST_EWORKSPACE before any device work.  No allocation of any kind is made.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other streams, other threads) race and must not be issued.
 * Arguments, buffer rules and results are those of stencil_apply; ST_EINVAL
 * for batched and variable-coefficient plans. */
st_status stencil_apply_noalloc(const st_plan *plan, const void *u_in, void *u_out, int32_t steps,
                                const st_wave_args *wave, void *stream);

/* Bytes of the fixed scratch array of stencil_apply_noalloc. */
size_t stencil_noalloc_capacity(void);

/* Transposed sweep.
 *  ST_LINEAR: v_out = (A^T)^steps v_in, (A^T v)(x) = sum_d c_d v(B(x - d)).
 *  ST_WAVE:   transpose of the linear state map (u_{-1}, u_0) -> (u_{T-1}, u_T)
 *             (no source): on entry v_in and wave->u_prev are the co-states of
 *             u_T and u_{T-1}; on return v_out and wave->u_prev are the
 *             co-states of u_0 and u_{-1}.
 * Same buffer rules as stencil_apply.  ST_EUNSUPPORTED for an ST_F64 wave plan. */
st_status stencil_apply_adjoint(const st_plan *plan, const void *v_in, void *v_out,
                                int32_t steps, const st_wave_args *wave, void *workspace,
                                size_t ws_bytes, void *stream);

/* Variable-coefficient sweep of an ST_VARCOEF plan, `steps` time steps:
 *   u_out = A^steps u_in,   (A u)(x) = sum_k f_k(x) u(B(x + d_k)).
 * `fields` (device, read only) holds one coefficient field per offset d_k of
 * the plan's shape, taken in (dz,dy,dx) lexicographic order of the in-shape
 * offsets (a star of radius r has 1 + 2*ndim*r, the radius-1 box 3^ndim),
 * each a full [nz][ny][nx] grid of the plan's storage type, stored one after
 * another.
 * `fields` must not overlap u_in, u_out or the workspace.
 * Buffer rules, workspace (mode 0) and steps == 0 as for stencil_apply.
 * A plan of another update kind returns ST_EINVAL. */
st_status stencil_apply_varcoef(const st_plan *plan, const void *u_in, void *u_out, const void *fields,
                                int32_t steps, void *workspace, size_t ws_bytes, void *stream);

/* Its transpose: v_out = (A^T)^steps v_in,
 *   (A^T v)(y) = sum_k f_k(y - d_k) v(B(y - d_k))   (periodic: y - d_k wraps;
 *   zero frame: terms with y - d_k outside the grid vanish).
 * Same arguments and rules as stencil_apply_varcoef. */
st_status stencil_apply_varcoef_adjoint(const st_plan *plan, const void *v_in, void *v_out,
                                        const void *fields, int32_t steps, void *workspace,
                                        size_t ws_bytes, void *stream);

/* Gradient of J = 1/2 sum_{t=1..T} || u_t[z = rec_z] - target[t-1] ||^2 with
 * respect to kappa for an ST_WAVE plan, by the discrete adjoint of the
 * leapfrog, recomputing states from (u_{t-1}, u_t) checkpoints taken every
 * ckpt_every steps.  u0 / wave->u_prev give u_0 / u_{-1} (not modified);
 * wave->src, wavelet, rec_z (required >= 0) and target are used; traces, if
 * non-NULL, receive the recorded traces.  dkappa (device, cells) is
 * overwritten; *loss_dev (device, one double) receives J.  Workspace from
 * stencil_workspace_bytes(plan, steps, 1).  ST_EUNSUPPORTED for an ST_F64 plan. */
st_status stencil_wave_gradient(const st_plan *plan, const void *u0, const st_wave_args *wave,
                                int32_t steps, float *dkappa, double *loss_dev,
                                void *workspace, size_t ws_bytes, void *stream);

/* Batched plan over `count` independent 2D ST_LINEAR problems of one storage
 * type and boundary rule (shapes, radii, extents and coefficients may
 * differ).  opts->tsteps (0 = 3) is the fused depth of the batch, the same
 * for every member (clamped per member to what its radius allows); -1 asks
 * for each member's own depth (the fused depth of its own map entry, within
 * the same limits); below -1 is ST_EINVAL.  The other option fields apply to
 * each member's own plan.  *out owns the plan. */
st_status stencil_plan_batched(const st_problem *problems, int32_t count,
                               const st_plan_opts *opts, st_plan **out);

/* All members advanced `steps` steps, one launch per time block for the
 * whole batch: each launch runs one block of k fused steps (the batch
 * depth, or the member's own) of every member that has blocks left,
 * max ceil(steps / k) launches in all instead of one series per member; a
 * launch divides the device among the members it carries (launch fusion,
 * one of the application-level wins of Section 5).  Workgroups never wait
 * on each other.  u_in / u_out are
 * HOST arrays of `count` device pointers (u_in[i] == u_out[i] allowed).
 * Workspace from stencil_workspace_bytes(batched_plan, steps, 0): a partner
 * grid per member plus the member tables (one per distinct set of running
 * members).  Asynchronous on `stream`; ST_EHIP
 * if a launch fails. */
st_status stencil_apply_batched(const st_plan *plan, const void *const *u_in,
                                void *const *u_out, int32_t steps, void *workspace,
                                size_t ws_bytes, void *stream);

/* The launch schedule stencil_apply_batched would run for `steps` (>= 1)
 * steps on a device of `cus` compute units (0: the current device's):
 * *launches grouped launches, *tables member tables (a new one wherever the
 * set of running members changes), *workgroups in all.  Builds and checks
 * the same tables as the apply (every running member's workgroup range
 * inside its launch, the ranges contiguous), with stand-in buffer
 * addresses; ST_EINVAL if a check fails.  Any output pointer may be NULL.
 * Host only (no device work unless cus is 0). */
st_status stencil_plan_describe_batched(const st_plan *plan, int32_t steps, int32_t cus,
                                        int32_t *launches, int32_t *tables, int64_t *workgroups);

/* Autotune: for every distinct case of the plan (one, or each batch
 * member), time the legal candidates (tile shape, fused time steps, rows per
 * workgroup, plane chunk), reject any candidate whose output differs from
 * the plain single-step kernel on a probe grid, keep the fastest, write it
 * into the plan and into the dispatch map, and append it to the tuning cache
 * file when STENCIL_TUNE_CACHE is set.  A wave plan whose forward step runs
 * the LDS-ring kernel then tunes its reverse step the same way (the
 * pointwise gradient step: lambda_t and the dkappa update, both checked).  `scratch` (device) must hold
 * stencil_workspace_bytes(plan, 0, 2) bytes.  Synchronises `stream`.
 * Setting STENCIL_TUNE_FAULT=1 deliberately perturbs the coefficients of part
 * of the candidates (fused-step or 32-row ones) so tests can check that the
 * parity filter rejects wrong-but-faster candidates.  An ST_F64 wave plan
 * tunes its forward step only (it has no reverse step). */
st_status stencil_autotune(st_plan *plan, void *scratch, size_t scratch_bytes, void *stream);

/* Counts from the plan's last stencil_autotune: candidates tried and
 * candidates rejected by the parity check.  Host only. */
st_status stencil_autotune_stats(const st_plan *plan, int32_t *tried, int32_t *rejected);

/* Message for the most recent failing call on this thread ("" if none). */
const char *stencil_last_error(void);

/* Library version string. */
const char *stencil_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STENCIL_H */
