/*
 * FP64 CPU oracle for the direct-summation gravitational N-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the GPU library never links, loads or calls it,
 * and it shares no code, header or constant with the GPU library.
 *
 * Plain nested loops in double precision, built with
 * -O2 -fno-fast-math -ffp-contract=off, so every j-sum is a strictly
 * sequential left-to-right sum. The only parallelism is OpenMP over the sink
 * index i, so every result is independent of the thread count.
 *
 * Layout: structure of arrays. A position array of n particles holds
 * x[0..n), y[0..n), z[0..n) back to back (3n doubles); likewise velocities,
 * accelerations and adjoint vectors.
 *
 * What each function follows:
 *   oracle_accel   Eq. (1), the softened pairwise acceleration (section
 *                  "N-body simulation"), with G and the softening eps; the
 *                  potential is the one the listing's CALCULATE_POTENTIAL
 *                  branch accumulates, with the physical sign -G and with the
 *                  j = i term left out, as Eq. (1) leaves it out.
 *   oracle_kdk     second-order kick-drift-kick leapfrog (synchronised
 *                  Stormer-Verlet) around Eq. (1). Not in the paper: the
 *                  integrator of the N-body workloads.
 *   oracle_diag    kinetic, potential and total energy, linear and angular
 *                  momentum, centre of mass. Not in the paper.
 *   oracle_vjp,    the transposed Jacobian of Eq. (1) with respect to the
 *   oracle_jvp     positions and the masses applied to a vector, and the
 *                  Jacobian applied to a vector. Not in the paper.
 *                  oracle_vjp_sampled returns chosen rows of oracle_vjp.
 *   oracle_diffusion3d  one explicit step of the 3-D diffusion equation
 *                  (section "3D diffusion equation"), the paper's second demo.
 *   oracle_adjoint reverse-mode derivative of a KDK trajectory, one sub-step
 *                  (kick, drift, kick) at a time, read back from the stored
 *                  FP64 trajectory. Not in the paper.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later calls (k >= 1); the results do not depend on it. */
void oracle_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k >= 1) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/*
 * Eq. (1): a_i = G * sum_{j != i} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^(3/2)
 * for ni sinks at xi against nj sources at xj with masses mj.
 *
 * self_index: NULL when the sinks are a set of their own (every source term
 * is summed, as the listing does for separate sink and source sets);
 * otherwise self_index[i] is the source index of sink i itself, and that
 * term is skipped (so eps = 0 is allowed).
 * pot: NULL, or phi_i = -G * sum_{j != i} m_j / sqrt(|r_j - r_i|^2 + eps^2).
 */
void oracle_accel(int64_t ni, const double *xi, const int64_t *self_index,
                  int64_t nj, const double *xj, const double *mj,
                  double eps, double G, double *acc, double *pot)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ni; i++) {
        const double px = xi[i], py = xi[ni + i], pz = xi[2 * ni + i];
        const int64_t self = self_index ? self_index[i] : -1;
        double ax = 0.0, ay = 0.0, az = 0.0, phi = 0.0;
        for (int64_t j = 0; j < nj; j++) {
            if (j == self)
                continue;
            const double dx = xj[j] - px;
            const double dy = xj[nj + j] - py;
            const double dz = xj[2 * nj + j] - pz;
            const double s = dx * dx + dy * dy + dz * dz + eps2;
            const double r = sqrt(s);
            const double s32 = s * r; /* (|d|^2 + eps^2)^(3/2) */
            ax += mj[j] * dx / s32;
            ay += mj[j] * dy / s32;
            az += mj[j] * dz / s32;
            phi += mj[j] / r;
        }
        acc[i] = G * ax;
        acc[ni + i] = G * ay;
        acc[2 * ni + i] = G * az;
        if (pot)
            pot[i] = -G * phi;
    }
}

/* a(x) of one particle set against itself (j = i skipped). */
static void accel_self(int64_t n, const double *x, const double *m,
                       double eps, double G, double *acc)
{
    int64_t *self = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++)
        self[i] = i;
    oracle_accel(n, x, self, n, x, m, eps, G, acc, NULL);
    free(self);
}

/*
 * nsteps kick-drift-kick steps of size dt (h = dt/2), in place on x, v:
 *   a_0 = a(x_0)
 *   v_{n+1/2} = v_n + h a_n
 *   x_{n+1}   = x_n + dt v_{n+1/2}
 *   a_{n+1}   = a(x_{n+1})
 *   v_{n+1}   = v_{n+1/2} + h a_{n+1}
 * acc (3n) receives a(x_final). traj_x / traj_v (each (nsteps+1)*3n, may be
 * NULL) receive the state after every step, step 0 first.
 */
void oracle_kdk(int64_t n, double *x, double *v, const double *m,
                double eps, double G, double dt, int64_t nsteps,
                double *acc, double *traj_x, double *traj_v)
{
    const double h = 0.5 * dt;
    const size_t n3 = 3 * (size_t)n;
    accel_self(n, x, m, eps, G, acc);
    if (traj_x)
        memcpy(traj_x, x, n3 * sizeof(double));
    if (traj_v)
        memcpy(traj_v, v, n3 * sizeof(double));
    for (int64_t s = 0; s < nsteps; s++) {
        for (size_t k = 0; k < n3; k++)
            v[k] = v[k] + h * acc[k];
        for (size_t k = 0; k < n3; k++)
            x[k] = x[k] + dt * v[k];
        accel_self(n, x, m, eps, G, acc);
        for (size_t k = 0; k < n3; k++)
            v[k] = v[k] + h * acc[k];
        if (traj_x)
            memcpy(traj_x + (size_t)(s + 1) * n3, x, n3 * sizeof(double));
        if (traj_v)
            memcpy(traj_v + (size_t)(s + 1) * n3, v, n3 * sizeof(double));
    }
}

/*
 * Conserved quantities of a state. out[0..12]:
 *   0 KE = 1/2 sum m |v|^2
 *   1 PE = -G sum_{i<j} m_i m_j / sqrt(|r_j - r_i|^2 + eps^2)
 *   2 E  = KE + PE
 *   3..5  P = sum m v
 *   6..8  L = sum m (r x v)
 *   9..11 centre of mass sum m r / sum m
 *   12    total mass
 * The pair sum is split as PE = sum_i m_i * (sum_{j>i} m_j / sqrt(s_ij)):
 * the inner sums run in parallel, the outer one sequentially.
 */
void oracle_diag(int64_t n, const double *x, const double *v, const double *m,
                 double eps, double G, double *out)
{
    const double eps2 = eps * eps;
    double *row = (double *)malloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        double sum = 0.0;
        for (int64_t j = i + 1; j < n; j++) {
            const double dx = x[j] - x[i];
            const double dy = x[n + j] - x[n + i];
            const double dz = x[2 * n + j] - x[2 * n + i];
            sum += m[j] / sqrt(dx * dx + dy * dy + dz * dz + eps2);
        }
        row[i] = sum;
    }
    double ke = 0, pe = 0, p[3] = {0, 0, 0}, l[3] = {0, 0, 0}, c[3] = {0, 0, 0}, mt = 0;
    for (int64_t i = 0; i < n; i++) {
        const double rx = x[i], ry = x[n + i], rz = x[2 * n + i];
        const double vx = v[i], vy = v[n + i], vz = v[2 * n + i];
        ke += 0.5 * m[i] * (vx * vx + vy * vy + vz * vz);
        pe += m[i] * row[i];
        p[0] += m[i] * vx;
        p[1] += m[i] * vy;
        p[2] += m[i] * vz;
        l[0] += m[i] * (ry * vz - rz * vy);
        l[1] += m[i] * (rz * vx - rx * vz);
        l[2] += m[i] * (rx * vy - ry * vx);
        c[0] += m[i] * rx;
        c[1] += m[i] * ry;
        c[2] += m[i] * rz;
        mt += m[i];
    }
    free(row);
    out[0] = ke;
    out[1] = -G * pe;
    out[2] = out[0] + out[1];
    for (int k = 0; k < 3; k++) {
        out[3 + k] = p[k];
        out[6 + k] = l[k];
        out[9 + k] = c[k] / mt;
    }
    out[12] = mt;
}

/*
 * The derivative of f(d) = d / (|d|^2 + eps^2)^(3/2) is the symmetric 3x3
 * matrix T(d) = s^(-3/2) I - 3 s^(-5/2) d d^T with s = |d|^2 + eps^2; it is
 * even in d. Given s32 = s^(3/2) and s52 = s^(5/2): out += c * T(d) w.
 */
static void add_T_times(const double d[3], double s32, double s52,
                        double c, const double w[3], double out[3])
{
    const double dw = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
    out[0] += c * (w[0] / s32 - 3.0 * d[0] * dw / s52);
    out[1] += c * (w[1] / s32 - 3.0 * d[1] * dw / s52);
    out[2] += c * (w[2] / s32 - 3.0 * d[2] * dw / s52);
}

/*
 * Transposed Jacobians of a(x, m) (Eq. (1), j = i skipped) applied to lam:
 *   jt_k = sum_i (d a_i / d r_k)^T lam_i
 *   gt_k = sum_i (d a_i / d m_k)   . lam_i
 * with, for i != k,
 *   d a_i / d r_k = G m_k T(r_k - r_i),
 *   d a_k / d r_k = -G sum_{j != k} m_j T(r_j - r_k),
 *   d a_i / d m_k = G (r_k - r_i) / (|r_k - r_i|^2 + eps^2)^(3/2),
 *   d a_k / d m_k = 0.
 * T is symmetric, so the transposes drop out. gt may be NULL.
 */
static void vjp_row(int64_t n, int64_t k, const double *x, const double *m,
                    const double *lam, double eps2, double G, double jt[3], double *gt)
{
    const double rk[3] = {x[k], x[n + k], x[2 * n + k]};
    const double lk[3] = {lam[k], lam[n + k], lam[2 * n + k]};
    double off[3] = {0, 0, 0};  /* sum_{i != k} m_k T(r_k - r_i) lam_i */
    double diag[3] = {0, 0, 0}; /* sum_{j != k} m_j T(r_j - r_k) lam_k */
    double g = 0.0;
    for (int64_t i = 0; i < n; i++) {
        if (i == k)
            continue;
        const double li[3] = {lam[i], lam[n + i], lam[2 * n + i]};
        const double d[3] = {rk[0] - x[i], rk[1] - x[n + i], rk[2] - x[2 * n + i]};
        const double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
        const double s32 = s * sqrt(s);
        const double s52 = s32 * s;
        add_T_times(d, s32, s52, m[k], li, off);  /* T(r_k - r_i) */
        add_T_times(d, s32, s52, m[i], lk, diag); /* T(r_i - r_k) = T(r_k - r_i) */
        g += (li[0] * d[0] + li[1] * d[1] + li[2] * d[2]) / s32;
    }
    jt[0] = G * (off[0] - diag[0]);
    jt[1] = G * (off[1] - diag[1]);
    jt[2] = G * (off[2] - diag[2]);
    *gt = G * g;
}

void oracle_vjp(int64_t n, const double *x, const double *m, const double *lam,
                double eps, double G, double *jt, double *gt)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; k++) {
        double r[3], g;
        vjp_row(n, k, x, m, lam, eps2, G, r, &g);
        jt[k] = r[0];
        jt[n + k] = r[1];
        jt[2 * n + k] = r[2];
        if (gt)
            gt[k] = g;
    }
}

/* The rows idx[0 .. ns) of oracle_vjp: jt is 3 x ns (SoA), gt ns. */
void oracle_vjp_sampled(int64_t n, int64_t ns, const int64_t *idx, const double *x,
                        const double *m, const double *lam, double eps, double G,
                        double *jt, double *gt)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < ns; q++) {
        double r[3], g;
        vjp_row(n, idx[q], x, m, lam, eps2, G, r, &g);
        jt[q] = r[0];
        jt[ns + q] = r[1];
        jt[2 * ns + q] = r[2];
        gt[q] = g;
    }
}

/*
 * Jacobian of a(x) applied to u: (J u)_i = sum_k (d a_i / d r_k) u_k
 *   = G sum_{j != i} m_j T(r_j - r_i) (u_j - u_i).
 */
void oracle_jvp(int64_t n, const double *x, const double *m, const double *u,
                double eps, double G, double *ju)
{
    const double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double acc[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i)
                continue;
            const double du[3] = {u[j] - u[i], u[n + j] - u[n + i], u[2 * n + j] - u[2 * n + i]};
            const double d[3] = {x[j] - x[i], x[n + j] - x[n + i], x[2 * n + j] - x[2 * n + i]};
            const double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
            const double s32 = s * sqrt(s);
            add_T_times(d, s32, s32 * s, m[j], du, acc);
        }
        ju[i] = G * acc[0];
        ju[n + i] = G * acc[1];
        ju[2 * n + i] = G * acc[2];
    }
}

/*
 * One explicit step of the 3-D diffusion equation du/dt = kappa lap(u)
 * (section "3D diffusion equation"): on an nx x ny x nz grid stored with k
 * fastest, index (i, j, k) -> k + nz (j + ny i), every point becomes
 *   fn = cc f + ce f(i+1) + cw f(i-1) + cn f(j+1) + cs f(j-1) + ct f(k+1) + cb f(k-1)
 * with ce = cw = kappa dt / dx^2, cn = cs = kappa dt / dy^2,
 * ct = cb = kappa dt / dz^2, cc = 1 - (ce + cw + cn + cs + ct + cb), and a
 * neighbour index outside the grid replaced by the nearest one inside.
 */
void oracle_diffusion3d(int64_t nx, int64_t ny, int64_t nz, double dx, double dy,
                        double dz, double dt, double kappa, const double *f, double *fn)
{
    const double ce = kappa * dt / (dx * dx), cw = ce;
    const double cn = kappa * dt / (dy * dy), cs = cn;
    const double ct = kappa * dt / (dz * dz), cb = ct;
    const double cc = 1.0 - (ce + cw + cn + cs + ct + cb);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nx; i++) {
        const int64_t ip = i + 1 < nx ? i + 1 : nx - 1, im = i > 0 ? i - 1 : 0;
        for (int64_t j = 0; j < ny; j++) {
            const int64_t jp = j + 1 < ny ? j + 1 : ny - 1, jm = j > 0 ? j - 1 : 0;
            for (int64_t k = 0; k < nz; k++) {
                const int64_t kp = k + 1 < nz ? k + 1 : nz - 1, km = k > 0 ? k - 1 : 0;
#define AT(a, b, c) f[(c) + nz * ((b) + ny * (a))]
                fn[k + nz * (j + ny * i)] = cc * AT(i, j, k) + ce * AT(ip, j, k) + cw * AT(im, j, k) +
                                            cn * AT(i, jp, k) + cs * AT(i, jm, k) + ct * AT(i, j, kp) +
                                            cb * AT(i, j, km);
#undef AT
            }
        }
    }
}

/*
 * Reverse-mode derivative of nsteps KDK steps (as in oracle_kdk), read back
 * from the stored position trajectory traj_x ((nsteps+1)*3n, step 0 first).
 *
 * On entry lamx, lamv hold dL/dx, dL/dv at the last step and lamm (n) holds
 * whatever the caller accumulates into (normally zeros); on exit lamx, lamv
 * hold dL/dx_0, dL/dv_0 and lamm has dL/dm added.
 *
 * Each step s -> s+1 is undone one sub-step at a time, last first:
 *   kick    v_{s+1} = v_half + h a(x_{s+1}):
 *           lamx += h J(x_{s+1})^T lamv, lamm += h G(x_{s+1})^T lamv
 *   drift   x_{s+1} = x_s + dt v_half:      lamv += dt lamx
 *   kick    v_half = v_s + h a(x_s):
 *           lamx += h J(x_s)^T lamv,     lamm += h G(x_s)^T lamv
 */
void oracle_adjoint(int64_t n, int64_t nsteps, const double *traj_x,
                    const double *m, double eps, double G, double dt,
                    double *lamx, double *lamv, double *lamm)
{
    const double h = 0.5 * dt;
    const size_t n3 = 3 * (size_t)n;
    double *jt = (double *)malloc(n3 * sizeof(double));
    double *gt = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t s = nsteps - 1; s >= 0; s--) {
        const double *x1 = traj_x + (size_t)(s + 1) * n3;
        const double *x0 = traj_x + (size_t)s * n3;
        oracle_vjp(n, x1, m, lamv, eps, G, jt, gt);
        for (size_t k = 0; k < n3; k++)
            lamx[k] += h * jt[k];
        for (int64_t k = 0; k < n; k++)
            lamm[k] += h * gt[k];
        for (size_t k = 0; k < n3; k++)
            lamv[k] += dt * lamx[k];
        oracle_vjp(n, x0, m, lamv, eps, G, jt, gt);
        for (size_t k = 0; k < n3; k++)
            lamx[k] += h * jt[k];
        for (int64_t k = 0; k < n; k++)
            lamm[k] += h * gt[k];
    }
    free(jt);
    free(gt);
}
