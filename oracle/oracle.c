/*
 * FP64 CPU oracle for repeated stencil sweeps.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library: it is written directly
 * from the definitions and is deliberately slow and plain (one loop per
 * index, one term per offset, no blocking or fusion).
 *
 * What it computes
 *  - Linear constant-coefficient sweep (Section 2.1, the weighted-sum form
 *    of the update rule): u^{t+1}(x) = sum_{d in S} c_d u^t(B(x+d)), with S
 *    the star (offsets along the axes) or box (full cube) of radius r
 *    (Section 2.1, stencil type and order), and B the boundary rule.
 *  - Its transpose: (A^T v)(x) = sum_{d in S} c_d v(B(x-d)).
 *  - The acoustic leapfrog u_{t+1} = 2u_t - u_{t-1} + kappa (.) L(u_t), a
 *    linear stencil (L) with a per-cell coefficient field (Section 2.1:
 *    spatially varying coefficients are one more array to read), with an
 *    optional point source and a recorded receiver plane.
 *  - The transposed leapfrog state map and the gradient of the trace misfit
 *    with respect to kappa, by the discrete adjoint (Lagrangian) recursion,
 *    with its own checkpoint/recompute loop.
 *  - Central second-difference weights of order 2r from the Taylor moment
 *    conditions.
 *  - An absorbing layer for the leapfrog (a damping term gamma(x) u_t in a
 *    band of cells along the faces, the stencil fused with the boundary
 *    physics, Section 4.3), its transposed state map and its kappa-gradient.
 *  - A diagnostic of the numerical floor: the same sweeps with every stored
 *    state rounded to binary32 or binary16 (FP64 arithmetic otherwise), to
 *    set a storage format's measured error against the error that format
 *    alone must incur.
 *
 * Conventions: x is unit stride; a 3D array is [nz][ny][nx]; n[0]=nx,
 * n[1]=ny, n[2]=nz (nz=1 in 2D).  Coefficients are a dense (2r+1)^ndim
 * array ordered (dz,dy,dx) with dx fastest; only offsets inside the shape
 * are read.  Boundary 0 = periodic, 1 = zero outside the domain.
 * Every function returns 0 on success and a negative value on bad input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PERIODIC 0
#define OR_ZERO 1
#define OR_STAR 0
#define OR_BOX 1

static int g_threads = 0;

void oracle_set_threads(int nthreads) { g_threads = nthreads; }

int oracle_max_threads(void) {
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

static int offset_in_shape(int shape, int dz, int dy, int dx) {
    if (shape == OR_BOX) return 1;
    return ((dz != 0) + (dy != 0) + (dx != 0)) <= 1;
}

static int64_t wrap(int64_t i, int64_t n) { return ((i % n) + n) % n; }

/*
 * Storage-rounding diagnostic (not used by the gate results).  Storing a
 * value in a binary floating-point format with p significant bits, minimum
 * normal exponent emin and largest finite value maxfin keeps the multiple
 * of the format's spacing at that magnitude nearest to it, ties to the even
 * multiple (IEEE 754 round-to-nearest-even); below 2^emin the spacing stays
 * 2^(emin-p+1) (gradual underflow), and a result beyond maxfin overflows to
 * infinity.  binary32: p = 24, emin = -126; binary16: p = 11, emin = -14.
 * Running a sweep with every stored state rounded this way measures the
 * error floor that the storage format alone imposes (FP64 arithmetic
 * otherwise).
 */
#define OR_STORE_EXACT 0
#define OR_STORE_BINARY32 1
#define OR_STORE_BINARY16 2

static double round_to_format(double x, int p, int emin, double maxfin) {
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);                 /* |x| in [2^(e-1), 2^e) */
    int lead = e - 1;
    if (lead < emin) lead = emin;
    const double spacing = ldexp(1.0, lead - (p - 1));
    const double q = nearbyint(x / spacing) * spacing;   /* x / spacing is exact */
    if (fabs(q) > maxfin) return copysign(INFINITY, x);
    return q;
}

static double store_round(double x, int storage) {
    if (storage == OR_STORE_BINARY32) return round_to_format(x, 24, -126, 3.4028234663852886e38);
    if (storage == OR_STORE_BINARY16) return round_to_format(x, 11, -14, 65504.0);
    return x;
}

static void store_round_all(double *u, int64_t count, int storage) {
    if (storage == OR_STORE_EXACT) return;
    for (int64_t i = 0; i < count; ++i) u[i] = store_round(u[i], storage);
}

/* Rounds `count` values in place to the storage format (0 = unchanged). */
int oracle_round_storage(double *u, int64_t count, int storage) {
    if (storage < OR_STORE_EXACT || storage > OR_STORE_BINARY16 || count < 0) return -11;
    store_round_all(u, count, storage);
    return 0;
}

/* u at (z,y,x) under the boundary rule. */
static double fetch(const double *u, const int64_t n[3], int boundary,
                    int64_t z, int64_t y, int64_t x) {
    if (boundary == OR_PERIODIC) {
        x = wrap(x, n[0]);
        y = wrap(y, n[1]);
        z = wrap(z, n[2]);
    } else if (x < 0 || x >= n[0] || y < 0 || y >= n[1] || z < 0 || z >= n[2]) {
        return 0.0;
    }
    return u[(z * n[1] + y) * n[0] + x];
}

static int check_args(int ndim, const int64_t n[3], int shape, int r, int boundary) {
    if (ndim != 2 && ndim != 3) return -1;
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) return -2;
    if (ndim == 2 && n[2] != 1) return -2;
    if (shape != OR_STAR && shape != OR_BOX) return -3;
    if (r < 1 || r > 8) return -4;
    if (boundary != OR_PERIODIC && boundary != OR_ZERO) return -5;
    return 0;
}

/* out(x) = sum_{d in S} c_d in(B(x + sign*d)); sign = -1 gives the transpose.
 * The offsets of S are listed once, in (dz,dy,dx) lexicographic order, and
 * every cell sums its terms in that order. */
static void apply_once(int ndim, const int64_t n[3], int shape, int r,
                       const double *c, int boundary, int sign,
                       const double *in, double *out) {
    const int rz = (ndim == 3) ? r : 0;
    const int w = 2 * r + 1;
    const int64_t nz = n[2], ny = n[1], nx = n[0];
    int d[17 * 17 * 17][3];
    double cd[17 * 17 * 17];
    int nt = 0;
    for (int dz = -rz; dz <= rz; ++dz)
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
                if (!offset_in_shape(shape, dz, dy, dx)) continue;
                d[nt][0] = dz; d[nt][1] = dy; d[nt][2] = dx;
                cd[nt] = c[((dz + rz) * w + (dy + r)) * w + (dx + r)];
                ++nt;
            }
#pragma omp parallel for collapse(2) schedule(static) num_threads(oracle_max_threads())
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
                double acc = 0.0;
                for (int k = 0; k < nt; ++k)
                    acc += cd[k] * fetch(in, n, boundary, z + sign * d[k][0],
                                         y + sign * d[k][1], x + sign * d[k][2]);
                out[(z * ny + y) * nx + x] = acc;
            }
        }
    }
}

static int64_t cells_of(const int64_t n[3]) { return n[0] * n[1] * n[2]; }

/* `steps` forward (sign=+1) or transposed (sign=-1) sweeps of u_in into u_out. */
static int sweep_common(int ndim, const int64_t n[3], int shape, int r,
                        const double *c, int boundary, int steps, int sign, int storage,
                        const double *u_in, double *u_out) {
    int e = check_args(ndim, n, shape, r, boundary);
    if (e) return e;
    if (steps < 0) return -6;
    if (storage < OR_STORE_EXACT || storage > OR_STORE_BINARY16) return -11;
    const int64_t cells = cells_of(n);
    double *a = (double *)malloc(sizeof(double) * (size_t)cells);
    double *b = (double *)malloc(sizeof(double) * (size_t)cells);
    if (!a || !b) { free(a); free(b); return -7; }
    memcpy(a, u_in, sizeof(double) * (size_t)cells);
    for (int t = 0; t < steps; ++t) {
        apply_once(ndim, n, shape, r, c, boundary, sign, a, b);
        store_round_all(b, cells, storage);
        double *tmp = a; a = b; b = tmp;
    }
    memcpy(u_out, a, sizeof(double) * (size_t)cells);
    free(a);
    free(b);
    return 0;
}

int oracle_sweep(int ndim, const int64_t n[3], int shape, int r, const double *c,
                 int boundary, int steps, const double *u_in, double *u_out) {
    return sweep_common(ndim, n, shape, r, c, boundary, steps, +1, OR_STORE_EXACT, u_in, u_out);
}

int oracle_sweep_adjoint(int ndim, const int64_t n[3], int shape, int r, const double *c,
                         int boundary, int steps, const double *v_in, double *v_out) {
    return sweep_common(ndim, n, shape, r, c, boundary, steps, -1, OR_STORE_EXACT, v_in, v_out);
}

/* The forward sweep with every step's result rounded to the storage format
 * (diagnostic floor; storage 0 is oracle_sweep). */
int oracle_sweep_stored(int ndim, const int64_t n[3], int shape, int r, const double *c,
                        int boundary, int steps, int storage, const double *u_in, double *u_out) {
    return sweep_common(ndim, n, shape, r, c, boundary, steps, +1, storage, u_in, u_out);
}

/*
 * Central second-difference weights of accuracy order 2r on the unit grid:
 * w_{-j} = w_j, and sum_j w_j j^{2m} = 2 [m == 1] for m = 0..r (a symmetric
 * stencil annihilates odd moments).  Solved by Gaussian elimination with
 * partial pivoting.  Output: w[0..r] = (w_0, w_1, ..., w_r).
 */
/* ---- Variable coefficients (Section 2.1: a coefficient that varies in
 * space is one more array to read).  `f` holds one field per offset of the
 * shape, in (dz,dy,dx) lexicographic order of the in-shape offsets, each a
 * full grid: f[k][z][y][x].
 *   forward:   out(x) = sum_k f_k(x) in(B(x + d_k))
 *   transpose: out(y) = sum over (x, k) with B(x + d_k) = y of f_k(x) in(x),
 *              written as a scatter over x (zero boundary: terms whose
 *              target lies outside are dropped). */
static int taps_of(int ndim, int shape, int r, int (*d)[3]) {
    const int rz = (ndim == 3) ? r : 0;
    int k = 0;
    for (int dz = -rz; dz <= rz; ++dz)
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
                if (!offset_in_shape(shape, dz, dy, dx)) continue;
                if (d) { d[k][0] = dz; d[k][1] = dy; d[k][2] = dx; }
                ++k;
            }
    return k;
}

int oracle_varcoef_taps(int ndim, int shape, int r) {
    if (check_args(ndim, (const int64_t[3]){1, 1, 1}, shape, r, OR_PERIODIC)) return -1;
    return taps_of(ndim, shape, r, NULL);
}

static void varcoef_once(int ndim, const int64_t n[3], int shape, int r, const double *f,
                         int boundary, const double *in, double *out) {
    int d[729][3];
    const int nt = taps_of(ndim, shape, r, d);
    const int64_t nz = n[2], ny = n[1], nx = n[0], cells = nx * ny * nz;
#pragma omp parallel for collapse(2) schedule(static) num_threads(oracle_max_threads())
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t i = (z * ny + y) * nx + x;
                double acc = 0.0;
                for (int k = 0; k < nt; ++k)
                    acc += f[k * cells + i] * fetch(in, n, boundary, z + d[k][0], y + d[k][1], x + d[k][2]);
                out[i] = acc;
            }
}

static void varcoef_transpose_once(int ndim, const int64_t n[3], int shape, int r, const double *f,
                                   int boundary, const double *in, double *out) {
    int d[729][3];
    const int nt = taps_of(ndim, shape, r, d);
    const int64_t nz = n[2], ny = n[1], nx = n[0], cells = nx * ny * nz;
    memset(out, 0, sizeof(double) * (size_t)cells);
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t i = (z * ny + y) * nx + x;
                for (int k = 0; k < nt; ++k) {
                    int64_t tz = z + d[k][0], ty = y + d[k][1], tx = x + d[k][2];
                    if (boundary == OR_PERIODIC) {
                        tz = wrap(tz, nz);
                        ty = wrap(ty, ny);
                        tx = wrap(tx, nx);
                    } else if (tx < 0 || tx >= nx || ty < 0 || ty >= ny || tz < 0 || tz >= nz) {
                        continue;
                    }
                    out[(tz * ny + ty) * nx + tx] += f[k * cells + i] * in[i];
                }
            }
}

int oracle_varcoef_sweep(int ndim, const int64_t n[3], int shape, int r, const double *f,
                         int boundary, int steps, int transpose, const double *u_in, double *u_out) {
    int e = check_args(ndim, n, shape, r, boundary);
    if (e) return e;
    if (r > 4) return -4;
    if (steps < 0) return -6;
    const int64_t cells = cells_of(n);
    double *a = (double *)malloc(sizeof(double) * (size_t)cells);
    double *b = (double *)malloc(sizeof(double) * (size_t)cells);
    if (!a || !b) { free(a); free(b); return -7; }
    memcpy(a, u_in, sizeof(double) * (size_t)cells);
    for (int t = 0; t < steps; ++t) {
        if (transpose) varcoef_transpose_once(ndim, n, shape, r, f, boundary, a, b);
        else varcoef_once(ndim, n, shape, r, f, boundary, a, b);
        double *tmp = a; a = b; b = tmp;
    }
    memcpy(u_out, a, sizeof(double) * (size_t)cells);
    free(a);
    free(b);
    return 0;
}

int oracle_fd2_weights(int r, double *w) {
    if (r < 1 || r > 8) return -4;
    const int m = r + 1;
    double A[9][10];
    for (int row = 0; row < m; ++row) {
        for (int j = 0; j < m; ++j) {
            double mom = (j == 0) ? (row == 0 ? 1.0 : 0.0) : 2.0 * pow((double)j, 2.0 * row);
            A[row][j] = mom;
        }
        A[row][m] = (row == 1) ? 2.0 : 0.0;
    }
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int row = col + 1; row < m; ++row)
            if (fabs(A[row][col]) > fabs(A[piv][col])) piv = row;
        if (A[piv][col] == 0.0) return -8;
        if (piv != col)
            for (int k = 0; k <= m; ++k) { double t = A[col][k]; A[col][k] = A[piv][k]; A[piv][k] = t; }
        for (int row = 0; row < m; ++row) {
            if (row == col) continue;
            const double f = A[row][col] / A[col][col];
            for (int k = col; k <= m; ++k) A[row][k] -= f * A[col][k];
        }
    }
    for (int j = 0; j < m; ++j) w[j] = A[j][m] / A[j][j];
    return 0;
}

/* Dense (2r+1)^3 star coefficients of the 3D Laplacian of order 2r. */
int oracle_laplacian3d(int r, double *dense) {
    double w[9];
    int e = oracle_fd2_weights(r, w);
    if (e) return e;
    const int W = 2 * r + 1;
    memset(dense, 0, sizeof(double) * (size_t)(W * W * W));
    dense[(r * W + r) * W + r] = 3.0 * w[0];
    for (int j = 1; j <= r; ++j) {
        for (int s = -1; s <= 1; s += 2) {
            dense[((r + s * j) * W + r) * W + r] = w[j];
            dense[(r * W + (r + s * j)) * W + r] = w[j];
            dense[(r * W + r) * W + (r + s * j)] = w[j];
        }
    }
    return 0;
}

/*
 * Absorbing layer.  The damped wave equation u_tt + gamma u_t = c^2 Lap u,
 * with u_tt by the central second difference and u_t by the central first
 * difference (u_{t+1} - u_{t-1}) / 2, gives the step
 *     (1 + gamma/2) u_{t+1} = 2 u_t - (1 - gamma/2) u_{t-1} + kappa L(u_t),
 * i.e. u_{t+1} = A (2 u_t + kappa L(u_t)) - B u_{t-1} with
 * A = 1 / (1 + gamma/2), B = (1 - gamma/2) / (1 + gamma/2); gamma = 0 is the
 * plain leapfrog.  The damping field is a sum over the axes of a quadratic
 * ramp in the band of `width` cells along each face:
 *     gamma(x) = sum_a s ((W - e_a) / W)^2 over axes with e_a < W,
 * e_a = min(i_a, n_a - 1 - i_a) the distance of the cell from the nearer
 * face (0 on a boundary cell), W = width, s = strength.
 */
int oracle_sponge_profile(const int64_t n[3], int width, double strength, double *gamma) {
    if (n[0] < 1 || n[1] < 1 || n[2] < 1 || width < 0 || !(strength >= 0.0)) return -12;
    for (int64_t z = 0; z < n[2]; ++z)
        for (int64_t y = 0; y < n[1]; ++y)
            for (int64_t x = 0; x < n[0]; ++x) {
                const int64_t idx[3] = {x, y, z};
                double g = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const int64_t e = idx[a] < n[a] - 1 - idx[a] ? idx[a] : n[a] - 1 - idx[a];
                    if (e < width) {
                        const double q = (double)(width - e) / (double)width;
                        g += strength * q * q;
                    }
                }
                gamma[(z * n[1] + y) * n[0] + x] = g;
            }
    return 0;
}

/* One leapfrog step: next = 2 cur - prev + kappa * L(cur), or with a damping
 * field (gamma != NULL) next = (2 cur - (1 - gamma/2) prev + kappa L(cur)) /
 * (1 + gamma/2); then the source. */
static void wave_step(const int64_t n[3], int r, const double *lap, int boundary,
                      const double *kappa, const double *gamma, const double *prev,
                      const double *cur, double *next, double *scratch, const int64_t *src,
                      double amp, int storage) {
    const int64_t cells = cells_of(n);
    apply_once(3, n, OR_STAR, r, lap, boundary, +1, cur, scratch);
#pragma omp parallel for schedule(static) num_threads(oracle_max_threads())
    for (int64_t i = 0; i < cells; ++i) {
        if (gamma)
            next[i] = (2.0 * cur[i] - (1.0 - 0.5 * gamma[i]) * prev[i] + kappa[i] * scratch[i]) /
                      (1.0 + 0.5 * gamma[i]);
        else
            next[i] = 2.0 * cur[i] - prev[i] + kappa[i] * scratch[i];
    }
    if (src) next[(src[2] * n[1] + src[1]) * n[0] + src[0]] += amp;
    store_round_all(next, cells, storage);
}

static int check_wave(const int64_t n[3], int r, int boundary, const int64_t *src, int64_t rec_z) {
    int e = check_args(3, n, OR_STAR, r, boundary);
    if (e) return e;
    if (src && (src[0] < 0 || src[0] >= n[0] || src[1] < 0 || src[1] >= n[1] ||
                src[2] < 0 || src[2] >= n[2])) return -9;
    if (rec_z >= n[2]) return -10;
    return 0;
}

/*
 * Leapfrog forward.  On entry u_prev = u_{-1}, u_cur = u_0; on exit
 * u_prev = u_{T-1}, u_cur = u_T.  If src is given, wavelet[t] is added at
 * src after the update that produces u_{t+1}.  If rec_z >= 0, traces[t] is
 * the plane z = rec_z of u_{t+1} (after the source), t = 0..T-1.
 * lap is the dense (2r+1)^3 star coefficient array of L.
 */
static int wave_forward_common(const int64_t n[3], int r, const double *lap, int boundary,
                               int steps, const double *kappa, const double *gamma, double *u_prev,
                               double *u_cur, const int64_t *src, const double *wavelet, int64_t rec_z,
                               double *traces, int storage) {
    int e = check_wave(n, r, boundary, src, rec_z);
    if (e) return e;
    if (steps < 0) return -6;
    if (storage < OR_STORE_EXACT || storage > OR_STORE_BINARY16) return -11;
    const int64_t cells = cells_of(n), plane = n[0] * n[1];
    double *a = (double *)malloc(sizeof(double) * (size_t)cells);
    double *b = (double *)malloc(sizeof(double) * (size_t)cells);
    double *c = (double *)malloc(sizeof(double) * (size_t)cells);
    double *s = (double *)malloc(sizeof(double) * (size_t)cells);
    if (!a || !b || !c || !s) { free(a); free(b); free(c); free(s); return -7; }
    memcpy(a, u_prev, sizeof(double) * (size_t)cells);
    memcpy(b, u_cur, sizeof(double) * (size_t)cells);
    for (int t = 0; t < steps; ++t) {
        wave_step(n, r, lap, boundary, kappa, gamma, a, b, c, s, src, src ? wavelet[t] : 0.0, storage);
        if (rec_z >= 0) memcpy(traces + (int64_t)t * plane, c + rec_z * plane, sizeof(double) * (size_t)plane);
        double *tmp = a; a = b; b = c; c = tmp;
    }
    memcpy(u_prev, a, sizeof(double) * (size_t)cells);
    memcpy(u_cur, b, sizeof(double) * (size_t)cells);
    free(a); free(b); free(c); free(s);
    return 0;
}

int oracle_wave_forward(const int64_t n[3], int r, const double *lap, int boundary,
                        int steps, const double *kappa, double *u_prev, double *u_cur,
                        const int64_t *src, const double *wavelet, int64_t rec_z,
                        double *traces) {
    return wave_forward_common(n, r, lap, boundary, steps, kappa, NULL, u_prev, u_cur, src, wavelet,
                               rec_z, traces, OR_STORE_EXACT);
}

/* The leapfrog with the absorbing layer's damping field gamma (cells). */
int oracle_wave_forward_damped(const int64_t n[3], int r, const double *lap, int boundary,
                               int steps, const double *kappa, const double *gamma, double *u_prev,
                               double *u_cur, const int64_t *src, const double *wavelet, int64_t rec_z,
                               double *traces) {
    if (!gamma) return -12;
    return wave_forward_common(n, r, lap, boundary, steps, kappa, gamma, u_prev, u_cur, src, wavelet,
                               rec_z, traces, OR_STORE_EXACT);
}

/* The leapfrog with every new state rounded to the storage format
 * (diagnostic floor; storage 0 is oracle_wave_forward). */
int oracle_wave_forward_stored(const int64_t n[3], int r, const double *lap, int boundary,
                               int steps, const double *kappa, double *u_prev, double *u_cur,
                               const int64_t *src, const double *wavelet, int64_t rec_z,
                               double *traces, int storage) {
    return wave_forward_common(n, r, lap, boundary, steps, kappa, NULL, u_prev, u_cur, src, wavelet,
                               rec_z, traces, storage);
}

/*
 * Transpose of the linear leapfrog state map (u_{-1}, u_0) -> (u_{T-1}, u_T)
 * (no source).  Writing the forward step as the block matrix
 * [[0, I], [-I, 2I + K L]] on the pair (previous, current), with K = diag
 * kappa, its transpose is [[0, -I], [I, 2I + L^T K]].  With co-states
 * lambda_{T+1} = -a_in, lambda_T = b_in this is the recursion
 *     lambda_t = 2 lambda_{t+1} - lambda_{t+2} + L^T(kappa (.) lambda_{t+1}),
 * and the co-state of (u_{-1}, u_0) is (-lambda_1, lambda_0).
 * On entry a = co-state of u_{T-1}, b = co-state of u_T; on exit a = co-state
 * of u_{-1}, b = co-state of u_0.
 */
int oracle_wave_adjoint(const int64_t n[3], int r, const double *lap, int boundary,
                        int steps, const double *kappa, double *a, double *b) {
    int e = check_wave(n, r, boundary, NULL, -1);
    if (e) return e;
    if (steps < 0) return -6;
    const int64_t cells = cells_of(n);
    double *l2 = (double *)malloc(sizeof(double) * (size_t)cells);   /* lambda_{t+2} */
    double *l1 = (double *)malloc(sizeof(double) * (size_t)cells);   /* lambda_{t+1} */
    double *l0 = (double *)malloc(sizeof(double) * (size_t)cells);   /* lambda_t */
    double *kl = (double *)malloc(sizeof(double) * (size_t)cells);
    double *s = (double *)malloc(sizeof(double) * (size_t)cells);
    if (!l2 || !l1 || !l0 || !kl || !s) { free(l2); free(l1); free(l0); free(kl); free(s); return -7; }
    for (int64_t i = 0; i < cells; ++i) { l2[i] = -a[i]; l1[i] = b[i]; }
    for (int t = steps - 1; t >= 0; --t) {
        for (int64_t i = 0; i < cells; ++i) kl[i] = kappa[i] * l1[i];
        apply_once(3, n, OR_STAR, r, lap, boundary, -1, kl, s);
        for (int64_t i = 0; i < cells; ++i) l0[i] = 2.0 * l1[i] - l2[i] + s[i];
        double *tmp = l2; l2 = l1; l1 = l0; l0 = tmp;
    }
    /* now l1 = lambda_0, l2 = lambda_1 */
    for (int64_t i = 0; i < cells; ++i) { a[i] = -l2[i]; b[i] = l1[i]; }
    free(l2); free(l1); free(l0); free(kl); free(s);
    return 0;
}

/*
 * Transpose of the damped state map (u_{-1}, u_0) -> (u_{T-1}, u_T) (no
 * source).  One damped step is the block matrix [[0, I], [-B, A (2I + K L)]]
 * on (previous, current), A = diag(1 / (1 + gamma/2)), B = diag((1 - gamma/2)
 * / (1 + gamma/2)), K = diag(kappa); its transpose [[0, -B], [I,
 * (2I + L^T K) A]] maps the co-states (alpha, beta) of (u_t, u_{t+1}) to
 * those of (u_{t-1}, u_t):
 *     (alpha, beta) <- (-B beta, alpha + 2 A beta + L^T(kappa (.) A beta)),
 * applied T times.  On entry a, b are the co-states of u_{T-1}, u_T; on exit
 * those of u_{-1}, u_0.
 */
int oracle_wave_adjoint_damped(const int64_t n[3], int r, const double *lap, int boundary,
                               int steps, const double *kappa, const double *gamma, double *a,
                               double *b) {
    int e = check_wave(n, r, boundary, NULL, -1);
    if (e) return e;
    if (steps < 0) return -6;
    if (!gamma) return -12;
    const int64_t cells = cells_of(n);
    double *ab = (double *)malloc(sizeof(double) * (size_t)cells);   /* A beta */
    double *kab = (double *)malloc(sizeof(double) * (size_t)cells);  /* kappa A beta */
    double *s = (double *)malloc(sizeof(double) * (size_t)cells);
    double *na = (double *)malloc(sizeof(double) * (size_t)cells);
    if (!ab || !kab || !s || !na) { free(ab); free(kab); free(s); free(na); return -7; }
    for (int t = steps - 1; t >= 0; --t) {
        for (int64_t i = 0; i < cells; ++i) {
            const double A = 1.0 / (1.0 + 0.5 * gamma[i]);
            const double B = (1.0 - 0.5 * gamma[i]) / (1.0 + 0.5 * gamma[i]);
            ab[i] = A * b[i];
            kab[i] = kappa[i] * ab[i];
            na[i] = -B * b[i];
        }
        apply_once(3, n, OR_STAR, r, lap, boundary, -1, kab, s);
        for (int64_t i = 0; i < cells; ++i) {
            b[i] = a[i] + 2.0 * ab[i] + s[i];
            a[i] = na[i];
        }
    }
    free(ab); free(kab); free(s); free(na);
    return 0;
}

/*
 * Gradient of J(kappa) = 1/2 sum_{t=1..T} || P u_t - d_t ||^2, P = restriction
 * to the plane z = rec_z, d_t = target[t-1], with respect to kappa, at the
 * given (u_{-1}, u_0), source and wavelet.  Lagrangian of the leapfrog
 * constraints gives, with lambda_{T+1} = lambda_{T+2} = 0 and t = T..1,
 *     lambda_t = 2 lambda_{t+1} - lambda_{t+2} + L^T(kappa (.) lambda_{t+1})
 *                + P^T (P u_t - d_t),
 *     dJ/dkappa = sum_{t=0}^{T-1} lambda_{t+1} (.) L(u_t).
 * States are rebuilt segment by segment from (u_{t-1}, u_t) checkpoints kept
 * every `ckpt_every` steps (0 = keep every state).  Outputs grad (cells) and
 * *loss.
 */
static int wave_gradient_common(const int64_t n[3], int r, const double *lap, int boundary,
                                int steps, const double *kappa, const double *gamma,
                                const double *u_prev0,
                                const double *u0, const int64_t *src, const double *wavelet,
                                int64_t rec_z, const double *target, int ckpt_every,
                                double *grad, double *loss, int storage) {
    int e = check_wave(n, r, boundary, src, rec_z);
    if (e) return e;
    if (rec_z < 0) return -10;
    if (steps < 1) return -6;
    if (storage < OR_STORE_EXACT || storage > OR_STORE_BINARY16) return -11;
    const int64_t cells = cells_of(n), plane = n[0] * n[1];
    const int T = steps;
    const int K = (ckpt_every <= 0 || ckpt_every > T) ? T : ckpt_every;
    const int nseg = (T + K - 1) / K;
    /* checkpoint s holds (u_{sK-1}, u_{sK}) */
    double *ck = (double *)malloc(sizeof(double) * (size_t)cells * 2 * (size_t)nseg);
    /* states[j] = u_{sK + j}, j = 0..K, during the backward pass of segment s */
    double *states = (double *)malloc(sizeof(double) * (size_t)cells * (size_t)(K + 2));
    double *l2 = (double *)malloc(sizeof(double) * (size_t)cells);
    double *l1 = (double *)malloc(sizeof(double) * (size_t)cells);
    double *l0 = (double *)malloc(sizeof(double) * (size_t)cells);
    double *kl = (double *)malloc(sizeof(double) * (size_t)cells);
    double *s = (double *)malloc(sizeof(double) * (size_t)cells);
    double *p0 = (double *)malloc(sizeof(double) * (size_t)cells);
    double *p1 = (double *)malloc(sizeof(double) * (size_t)cells);
    double *p2 = (double *)malloc(sizeof(double) * (size_t)cells);
    if (!ck || !states || !l2 || !l1 || !l0 || !kl || !s || !p0 || !p1 || !p2) {
        free(ck); free(states); free(l2); free(l1); free(l0); free(kl); free(s);
        free(p0); free(p1); free(p2);
        return -7;
    }
    /* forward: loss and checkpoints */
    double J = 0.0;
    memcpy(p0, u_prev0, sizeof(double) * (size_t)cells);
    memcpy(p1, u0, sizeof(double) * (size_t)cells);
    for (int t = 0; t < T; ++t) {
        if (t % K == 0) {
            memcpy(ck + (size_t)cells * 2 * (size_t)(t / K), p0, sizeof(double) * (size_t)cells);
            memcpy(ck + (size_t)cells * (2 * (size_t)(t / K) + 1), p1, sizeof(double) * (size_t)cells);
        }
        wave_step(n, r, lap, boundary, kappa, gamma, p0, p1, p2, s, src, src ? wavelet[t] : 0.0, storage);
        const double *d = target + (int64_t)t * plane;
        const double *pl = p2 + rec_z * plane;
        for (int64_t i = 0; i < plane; ++i) J += 0.5 * (pl[i] - d[i]) * (pl[i] - d[i]);
        double *tmp = p0; p0 = p1; p1 = p2; p2 = tmp;
    }
    *loss = J;
    /* backward */
    memset(grad, 0, sizeof(double) * (size_t)cells);
    memset(l2, 0, sizeof(double) * (size_t)cells);   /* lambda_{T+2} */
    memset(l1, 0, sizeof(double) * (size_t)cells);   /* lambda_{T+1} */
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int t0 = seg * K;
        const int t1 = (t0 + K < T) ? t0 + K : T;    /* segment covers u_{t0}..u_{t1} */
        /* rebuild u_{t0-1}..u_{t1} into states[0..] with states[j+1] = u_{t0+j} */
        memcpy(states, ck + (size_t)cells * 2 * (size_t)seg, sizeof(double) * (size_t)cells);
        memcpy(states + cells, ck + (size_t)cells * (2 * (size_t)seg + 1), sizeof(double) * (size_t)cells);
        for (int t = t0; t < t1; ++t) {
            const int j = t - t0 + 1;
            wave_step(n, r, lap, boundary, kappa, gamma, states + (size_t)cells * (j - 1),
                      states + (size_t)cells * j, states + (size_t)cells * (j + 1), s,
                      src, src ? wavelet[t] : 0.0, storage);
        }
        const int tstart = (seg == nseg - 1) ? T : t1 - 1;
        for (int t = tstart; t >= t0; --t) {
            const double *ut = states + (size_t)cells * (t - t0 + 1);
            /* gradient term lambda_{t+1} (.) L(u_t); damped: (A lambda_{t+1}) (.) L(u_t) */
            apply_once(3, n, OR_STAR, r, lap, boundary, +1, ut, s);
            for (int64_t i = 0; i < cells; ++i) {
                const double w = gamma ? l1[i] / (1.0 + 0.5 * gamma[i]) : l1[i];
                grad[i] = store_round(grad[i] + w * s[i], storage);
            }
            if (t >= 1) {
                /* damped: lambda_t = 2 A lambda_{t+1} + L^T(kappa A lambda_{t+1}) - B lambda_{t+2} + ... */
                for (int64_t i = 0; i < cells; ++i)
                    kl[i] = kappa[i] * (gamma ? l1[i] / (1.0 + 0.5 * gamma[i]) : l1[i]);
                apply_once(3, n, OR_STAR, r, lap, boundary, -1, kl, s);
                for (int64_t i = 0; i < cells; ++i) {
                    if (gamma) {
                        const double A = 1.0 / (1.0 + 0.5 * gamma[i]);
                        const double B = (1.0 - 0.5 * gamma[i]) * A;
                        l0[i] = 2.0 * A * l1[i] - B * l2[i] + s[i];
                    } else {
                        l0[i] = 2.0 * l1[i] - l2[i] + s[i];
                    }
                }
                const double *d = target + (int64_t)(t - 1) * plane;
                const double *pl = ut + rec_z * plane;
                double *lp = l0 + rec_z * plane;
                for (int64_t i = 0; i < plane; ++i) lp[i] += pl[i] - d[i];
                store_round_all(l0, cells, storage);
                double *tmp = l2; l2 = l1; l1 = l0; l0 = tmp;
            }
        }
    }
    free(ck); free(states); free(l2); free(l1); free(l0); free(kl); free(s);
    free(p0); free(p1); free(p2);
    return 0;
}

int oracle_wave_gradient(const int64_t n[3], int r, const double *lap, int boundary,
                         int steps, const double *kappa, const double *u_prev0,
                         const double *u0, const int64_t *src, const double *wavelet,
                         int64_t rec_z, const double *target, int ckpt_every,
                         double *grad, double *loss) {
    return wave_gradient_common(n, r, lap, boundary, steps, kappa, NULL, u_prev0, u0, src, wavelet,
                                rec_z, target, ckpt_every, grad, loss, OR_STORE_EXACT);
}

/* The gradient of the misfit of the damped leapfrog (damping field gamma):
 * with the step u_{t+1} = A (2 u_t + kappa L(u_t)) - B u_{t-1} + source, the
 * Lagrangian gives lambda_t = 2 A lambda_{t+1} + L^T(kappa (.) A lambda_{t+1})
 * - B lambda_{t+2} + P^T (P u_t - d_t) and dJ/dkappa = sum_t (A lambda_{t+1})
 * (.) L(u_t). */
int oracle_wave_gradient_damped(const int64_t n[3], int r, const double *lap, int boundary,
                                int steps, const double *kappa, const double *gamma,
                                const double *u_prev0, const double *u0, const int64_t *src,
                                const double *wavelet, int64_t rec_z, const double *target,
                                int ckpt_every, double *grad, double *loss) {
    if (!gamma) return -12;
    return wave_gradient_common(n, r, lap, boundary, steps, kappa, gamma, u_prev0, u0, src, wavelet,
                                rec_z, target, ckpt_every, grad, loss, OR_STORE_EXACT);
}

/* The gradient with every stored state (u_t, lambda_t and the running
 * gradient) rounded to the storage format (diagnostic floor; storage 0 is
 * oracle_wave_gradient). */
int oracle_wave_gradient_stored(const int64_t n[3], int r, const double *lap, int boundary,
                                int steps, const double *kappa, const double *u_prev0,
                                const double *u0, const int64_t *src, const double *wavelet,
                                int64_t rec_z, const double *target, int ckpt_every,
                                double *grad, double *loss, int storage) {
    return wave_gradient_common(n, r, lap, boundary, steps, kappa, NULL, u_prev0, u0, src, wavelet,
                                rec_z, target, ckpt_every, grad, loss, storage);
}
