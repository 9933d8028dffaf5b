/*
 * Drives every entry point of the FP64 CPU oracle (oracle/nbody_oracle.c) on
 * small seeded inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: any out-of-bounds access, use after free, leak
 * or undefined arithmetic in the oracle aborts the run. Beside that it checks
 * a few facts the oracle must meet whatever its build: the third law
 * (sum_i m_i a_i = 0), time reversibility of the leapfrog, and the
 * dot-product identity <J u, lam> = <u, J^T lam>. Prints "ok".
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_accel(int64_t ni, const double *xi, const int64_t *self_index, int64_t nj,
                  const double *xj, const double *mj, double eps, double G, double *acc,
                  double *pot);
void oracle_kdk(int64_t n, double *x, double *v, const double *m, double eps, double G,
                double dt, int64_t nsteps, double *acc, double *traj_x, double *traj_v);
void oracle_diag(int64_t n, const double *x, const double *v, const double *m, double eps,
                 double G, double *out);
void oracle_vjp(int64_t n, const double *x, const double *m, const double *lam, double eps,
                double G, double *jt, double *gt);
void oracle_vjp_sampled(int64_t n, int64_t ns, const int64_t *idx, const double *x,
                        const double *m, const double *lam, double eps, double G, double *jt,
                        double *gt);
void oracle_jvp(int64_t n, const double *x, const double *m, const double *u, double eps,
                double G, double *ju);
void oracle_diffusion3d(int64_t nx, int64_t ny, int64_t nz, double dx, double dy, double dz,
                        double dt, double kappa, const double *f, double *fn);
void oracle_adjoint(int64_t n, int64_t nsteps, const double *traj_x, const double *m,
                    double eps, double G, double dt, double *lamx, double *lamv, double *lamm);
int oracle_num_threads(void);
void oracle_set_num_threads(int k);

static uint64_t state = 88172645463325252ull;
static double urand(void) { /* xorshift64, in [-1, 1) */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 4503599627370496.0 - 1.0;
}

static void fail(const char *what, double a) {
    fprintf(stderr, "FAILED: %s (%g)\n", what, a);
    exit(1);
}

int main(void) {
    enum { N = 37, S = 5, NS = 4 };
    const double eps = 0.05, G = 1.3, dt = 0.01;
    double *x = malloc(3 * N * sizeof(double)), *v = malloc(3 * N * sizeof(double));
    double *m = malloc(N * sizeof(double)), *a = malloc(3 * N * sizeof(double));
    double *pot = malloc(N * sizeof(double)), *u = malloc(3 * N * sizeof(double));
    double *lam = malloc(3 * N * sizeof(double)), *jt = malloc(3 * N * sizeof(double));
    double *gt = malloc(N * sizeof(double)), *ju = malloc(3 * N * sizeof(double));
    int64_t *self = malloc(N * sizeof(int64_t));
    for (int i = 0; i < 3 * N; ++i) {
        x[i] = urand();
        v[i] = 0.1 * urand();
        u[i] = urand();
        lam[i] = urand();
    }
    for (int i = 0; i < N; ++i) {
        m[i] = 0.5 + 0.25 * (urand() + 1.0);
        self[i] = i;
    }
    oracle_set_num_threads(2);
    if (oracle_num_threads() < 1) fail("threads", 0);

    /* force with and without the potential, a set on itself and separate sets */
    oracle_accel(N, x, self, N, x, m, eps, G, a, pot);
    double tot[3] = {0, 0, 0}, scale = 0;
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < N; ++i) {
            tot[c] += m[i] * a[c * N + i];
            scale += fabs(m[i] * a[c * N + i]);
        }
    for (int c = 0; c < 3; ++c)
        if (fabs(tot[c]) > 1e-13 * scale) fail("third law", tot[c]);
    double *a2 = malloc(3 * 7 * sizeof(double));
    oracle_accel(7, x + 0, NULL, N, x, m, eps, G, a2, NULL);
    oracle_accel(N, x, self, N, x, m, 0.0, G, a, NULL); /* eps = 0 allowed on a set itself */
    for (int i = 0; i < 3 * N; ++i)
        if (!isfinite(a[i])) fail("eps = 0", a[i]);

    /* leapfrog with a stored trajectory, then back: reversible */
    double *tx = malloc((S + 1) * 3 * N * sizeof(double)), *tv = malloc((S + 1) * 3 * N * sizeof(double));
    double *x0 = malloc(3 * N * sizeof(double)), *v0 = malloc(3 * N * sizeof(double));
    memcpy(x0, x, 3 * N * sizeof(double));
    memcpy(v0, v, 3 * N * sizeof(double));
    oracle_kdk(N, x, v, m, eps, G, dt, S, a, tx, tv);
    for (int i = 0; i < 3 * N; ++i) v[i] = -v[i];
    oracle_kdk(N, x, v, m, eps, G, dt, S, a, NULL, NULL);
    for (int i = 0; i < 3 * N; ++i)
        if (fabs(x[i] - x0[i]) > 1e-12 || fabs(-v[i] - v0[i]) > 1e-12) fail("reversibility", x[i] - x0[i]);

    double out[13];
    oracle_diag(N, x, v, m, eps, G, out);
    if (!(out[0] > 0) || !(out[1] < 0)) fail("diagnostics", out[0]);

    /* transposed and forward Jacobians: <J u, lam> = <u, J^T lam> */
    oracle_vjp(N, x, m, lam, eps, G, jt, gt);
    oracle_jvp(N, x, m, u, eps, G, ju);
    double l = 0, r = 0, sl = 0;
    for (int i = 0; i < 3 * N; ++i) {
        l += ju[i] * lam[i];
        r += u[i] * jt[i];
        sl += fabs(ju[i] * lam[i]);
    }
    if (fabs(l - r) > 1e-12 * sl) fail("dot-product identity", l - r);
    int64_t idx[NS] = {0, 5, 17, N - 1};
    double jts[3 * NS], gts[NS];
    oracle_vjp_sampled(N, NS, idx, x, m, lam, eps, G, jts, gts);
    for (int q = 0; q < NS; ++q)
        if (jts[q] != jt[idx[q]] || gts[q] != gt[idx[q]]) fail("sampled rows", (double)q);

    /* reverse-mode walk over the stored trajectory */
    double *lx = calloc(3 * N, sizeof(double)), *lv = calloc(3 * N, sizeof(double));
    double *lm = calloc(N, sizeof(double));
    memcpy(lx, lam, 3 * N * sizeof(double));
    oracle_adjoint(N, S, tx, m, eps, G, dt, lx, lv, lm);
    for (int i = 0; i < N; ++i)
        if (!isfinite(lm[i])) fail("adjoint", lm[i]);

    /* the stencil on a ragged grid, edges clamped */
    const int nx = 5, ny = 4, nz = 3;
    double *f = malloc(nx * ny * nz * sizeof(double)), *fn = malloc(nx * ny * nz * sizeof(double));
    for (int i = 0; i < nx * ny * nz; ++i) f[i] = 2.5;
    oracle_diffusion3d(nx, ny, nz, 1.0, 1.0, 1.0, 0.1, 1.0, f, fn);
    for (int i = 0; i < nx * ny * nz; ++i)
        if (fabs(fn[i] - 2.5) > 1e-15) fail("stencil keeps a constant field", fn[i]);

    free(x); free(v); free(m); free(a); free(pot); free(u); free(lam); free(jt); free(gt);
    free(ju); free(self); free(a2); free(tx); free(tv); free(x0); free(v0); free(lx); free(lv);
    free(lm); free(f); free(fn);
    printf("ok\n");
    return 0;
}
