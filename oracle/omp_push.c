/*
 * Parallel driver of the oracle's particle step, for the benchmark's CPU
 * baseline only (test infrastructure, like the rest of this directory).
 *
 * The particles are split into one contiguous chunk per OpenMP thread; each
 * thread runs orc_push (gather, pusher, move, Esirkepov deposit; Secs.
 * II.C-E) on its chunk with current planes of its own, and the planes are
 * summed into J at the end.  The arithmetic is orc_push's; only the order
 * in which the per-thread currents are added differs from one serial call.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dim;
    int32_t order;
    int64_t n[3];
    double d[3];
    double dt;
    int32_t pusher;
    int32_t absorb_x;
    double laser[4];
    int32_t laser_circular;
} orc_grid;

void orc_push(const orc_grid *g, double q, double m, int64_t np, double *const *x, double *const *u, double *w,
              double w0, const double *const *F, double *const *J, double *diag);

/* Returns 0, or -1 when the per-thread planes cannot be allocated;
 * *threads receives the number of threads that ran. */
int orc_push_omp(const orc_grid *g, double q, double m, int64_t np, double *const *x, double *const *u,
                 double *w, double w0, const double *const *F, double *const *J, int *threads) {
    const int64_t nc = g->n[0] * g->n[1] * g->n[2];
    const int nt = omp_get_max_threads();
    double *priv = (double *)calloc((size_t)nt * 3 * (size_t)nc, sizeof(double));
    if (!priv) return -1;
    int used = 0;
#pragma omp parallel
    {
        const int t = omp_get_thread_num(), T = omp_get_num_threads();
#pragma omp single
        used = T;
        const int64_t a = np * t / T, b = np * (t + 1) / T;
        double *Jt[3] = {priv + ((size_t)t * 3 + 0) * nc, priv + ((size_t)t * 3 + 1) * nc,
                         priv + ((size_t)t * 3 + 2) * nc};
        double *xt[3] = {x[0] + a, x[1] + a, x[2] + a};
        double *ut[3] = {u[0] + a, u[1] + a, u[2] + a};
        orc_push(g, q, m, b - a, xt, ut, w ? w + a : NULL, w0, F, Jt, NULL);
    }
    for (int c = 0; c < 3; ++c)
#pragma omp parallel for
        for (int64_t i = 0; i < nc; ++i) {
            double s = 0.0;
            for (int t = 0; t < used; ++t) s += priv[((size_t)t * 3 + c) * nc + i];
            J[c][i] += s;
        }
    free(priv);
    *threads = used;
    return 0;
}
