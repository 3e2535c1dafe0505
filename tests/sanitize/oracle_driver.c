/* Exercises every entry point of the FP64 oracle on small grids, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py: any out-of-bounds access, use of freed memory
 * or undefined operation aborts the run.  Bad-argument paths are included.
 * Prints "ok" on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_sweep(int, const int64_t *, int, int, const double *, int, int, const double *, double *);
int oracle_sweep_adjoint(int, const int64_t *, int, int, const double *, int, int, const double *, double *);
int oracle_sweep_stored(int, const int64_t *, int, int, const double *, int, int, int, const double *, double *);
int oracle_varcoef_taps(int, int, int);
int oracle_varcoef_sweep(int, const int64_t *, int, int, const double *, int, int, int, const double *, double *);
int oracle_fd2_weights(int, double *);
int oracle_laplacian3d(int, double *);
int oracle_round_storage(double *, int64_t, int);
int oracle_sponge_profile(const int64_t *, int, double, double *);
int oracle_wave_forward(const int64_t *, int, const double *, int, int, const double *, double *, double *,
                        const int64_t *, const double *, int64_t, double *);
int oracle_wave_forward_stored(const int64_t *, int, const double *, int, int, const double *, double *, double *,
                               const int64_t *, const double *, int64_t, double *, int);
int oracle_wave_forward_damped(const int64_t *, int, const double *, int, int, const double *, const double *,
                               double *, double *, const int64_t *, const double *, int64_t, double *);
int oracle_wave_adjoint(const int64_t *, int, const double *, int, int, const double *, double *, double *);
int oracle_wave_adjoint_damped(const int64_t *, int, const double *, int, int, const double *, const double *,
                               double *, double *);
int oracle_wave_gradient(const int64_t *, int, const double *, int, int, const double *, const double *,
                         const double *, const int64_t *, const double *, int64_t, const double *, int, double *,
                         double *);
int oracle_wave_gradient_stored(const int64_t *, int, const double *, int, int, const double *, const double *,
                                const double *, const int64_t *, const double *, int64_t, const double *, int,
                                double *, double *, int);
int oracle_wave_gradient_damped(const int64_t *, int, const double *, int, int, const double *, const double *,
                                const double *, const double *, const int64_t *, const double *, int64_t,
                                const double *, int, double *, double *);

static double *fill(size_t n, unsigned seed) {
    double *a = (double *)malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) {
        seed = seed * 1103515245u + 12345u;
        a[i] = (double)(seed >> 8) / 16777216.0;
    }
    return a;
}

#define CHECK(x)                                                           \
    do {                                                                   \
        if ((x) != 0) {                                                    \
            fprintf(stderr, "call failed: %s (line %d)\n", #x, __LINE__);  \
            return 1;                                                      \
        }                                                                  \
    } while (0)
#define REJECT(x)                                                          \
    do {                                                                   \
        if ((x) == 0) {                                                    \
            fprintf(stderr, "bad call accepted: %s (line %d)\n", #x, __LINE__); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

int main(void) {
    /* linear sweeps, every shape/radius, both boundaries, grids below 2r+1 */
    const int64_t shapes[4][3] = {{7, 5, 1}, {3, 4, 1}, {6, 5, 4}, {2, 3, 5}};
    for (int s = 0; s < 4; ++s) {
        const int ndim = shapes[s][2] == 1 ? 2 : 3;
        const size_t cells = (size_t)(shapes[s][0] * shapes[s][1] * shapes[s][2]);
        for (int shape = 0; shape < 2; ++shape)
            for (int r = 1; r <= (shape ? 2 : 4); ++r)
                for (int bc = 0; bc < 2; ++bc) {
                    const int w = 2 * r + 1;
                    const size_t nc = ndim == 3 ? (size_t)(w * w * w) : (size_t)(w * w);
                    double *c = fill(nc, 3u + (unsigned)r), *u = fill(cells, 7u), *o = fill(cells, 9u);
                    CHECK(oracle_sweep(ndim, shapes[s], shape, r, c, bc, 3, u, o));
                    CHECK(oracle_sweep_adjoint(ndim, shapes[s], shape, r, c, bc, 2, u, o));
                    CHECK(oracle_sweep_stored(ndim, shapes[s], shape, r, c, bc, 2, 2, u, o));
                    if (r <= 4 && (shape == 0 || r == 1)) {
                        const int nt = oracle_varcoef_taps(ndim, shape, r);
                        double *f = fill((size_t)nt * cells, 11u);
                        CHECK(oracle_varcoef_sweep(ndim, shapes[s], shape, r, f, bc, 2, 0, u, o));
                        CHECK(oracle_varcoef_sweep(ndim, shapes[s], shape, r, f, bc, 2, 1, u, o));
                        free(f);
                    }
                    free(c); free(u); free(o);
                }
    }
    double w[9], lap[729];
    for (int r = 1; r <= 8; ++r) CHECK(oracle_fd2_weights(r, w));
    CHECK(oracle_laplacian3d(4, lap));
    double v[5] = {1.0, 1e-9, 70000.0, -0.3, 1e-42};
    CHECK(oracle_round_storage(v, 5, 2));
    CHECK(oracle_round_storage(v, 5, 1));
    /* the wave family with source, receiver, checkpoints and the layer */
    const int64_t n[3] = {9, 8, 10};
    const size_t cells = 9 * 8 * 10, plane = 9 * 8;
    const int T = 6;
    const int64_t src[3] = {4, 3, 5};
    double *k = fill(cells, 13u), *a = fill(cells, 15u), *b = fill(cells, 17u), *g = fill(cells, 19u);
    double *wav = fill(T, 21u), *tr = fill(T * plane, 23u), *tg = fill(T * plane, 25u), *gm = fill(cells, 27u);
    for (size_t i = 0; i < cells; ++i) k[i] = 0.05 + 0.1 * k[i];
    double J = 0.0;
    CHECK(oracle_sponge_profile(n, 3, 0.8, gm));
    CHECK(oracle_wave_forward(n, 4, lap, 1, T, k, a, b, src, wav, 2, tr));
    CHECK(oracle_wave_forward_stored(n, 4, lap, 1, T, k, a, b, src, wav, 2, tr, 1));
    CHECK(oracle_wave_forward_damped(n, 4, lap, 1, T, k, gm, a, b, src, wav, 2, tr));
    CHECK(oracle_wave_adjoint(n, 4, lap, 0, T, k, a, b));
    CHECK(oracle_wave_adjoint_damped(n, 4, lap, 1, T, k, gm, a, b));
    for (int K = 0; K <= 4; K += 2) {
        CHECK(oracle_wave_gradient(n, 4, lap, 1, T, k, a, b, src, wav, 2, tg, K, g, &J));
        CHECK(oracle_wave_gradient_stored(n, 4, lap, 1, T, k, a, b, src, wav, 2, tg, K, g, &J, 1));
        CHECK(oracle_wave_gradient_damped(n, 4, lap, 1, T, k, gm, a, b, src, wav, 2, tg, K, g, &J));
    }
    /* rejected arguments */
    const int64_t bad[3] = {0, 4, 4};
    REJECT(oracle_sweep(3, bad, 0, 1, lap, 0, 1, a, b));
    REJECT(oracle_sweep(3, n, 0, 9, lap, 0, 1, a, b));
    REJECT(oracle_sweep_stored(3, n, 0, 1, lap, 0, 1, 5, a, b));
    REJECT(oracle_round_storage(v, 5, 3));
    const int64_t far[3] = {99, 0, 0};
    REJECT(oracle_wave_forward(n, 4, lap, 1, T, k, a, b, far, wav, 2, tr));
    REJECT(oracle_wave_gradient(n, 4, lap, 1, T, k, a, b, src, wav, -1, tg, 0, g, &J));
    REJECT(oracle_sponge_profile(n, -1, 0.5, gm));
    REJECT(oracle_wave_adjoint_damped(n, 4, lap, 1, T, k, NULL, a, b));
    free(k); free(a); free(b); free(g); free(wav); free(tr); free(tg); free(gm);
    if (!isfinite(J)) return 1;
    printf("ok\n");
    return 0;
}
