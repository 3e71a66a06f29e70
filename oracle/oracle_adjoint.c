/*
 * FP64 CPU oracle for the adjoint of the Lennard-Jones forces (section 4.1)
 * and of velocity-Verlet trajectories built on them.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it shares no code with the HIP library.
 *
 * Definitions.  For a pair (i, j) in the force set, r = x_i - x_j (minimum
 * image), u = |r|^2 and, with the pair's eps and sig,
 *     s(u)    = 24 eps (2 sig^12 u^-7 - sig^6 u^-4)        (section 4.1)
 *     ds/du   = 24 eps (-14 sig^12 u^-8 + 4 sig^6 u^-5)
 *     ds/deps = 24 (2 sig^12 u^-7 - sig^6 u^-4)  (s is linear in eps: defined at eps = 0)
 *     ds/dsig = 24 eps (24 sig^11 u^-7 - 6 sig^5 u^-4).
 * The pair adds f = s r to F_i and -f to F_j.  For a scalar loss with
 * lam_i = dL/dF_i the pair contributes (lam_i - lam_j) . f, so with
 * dl = lam_i - lam_j and J = s I + 2 (ds/du) r r^T (= df/dr):
 *     dL/dx_i += J dl,   dL/dx_j -= J dl,   dL/dtheta += (ds/dtheta) r . dl.
 * The cut-off is a fixed set boundary and is not differentiated.
 *
 * Parameters are ordered (eps_AA, eps_AB, eps_BB, sig_AA, sig_AB, sig_BB); a
 * pair of types ti, tj uses entry ti + tj.  Every sum runs row by row in index
 * order (rows in parallel), so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int oracle_pair_f32(const float *pi, const float *pj, const float L[3], const int32_t per[3],
                    float R2, double r[3]);
void oracle_lj_forces_f64(int64_t n, const double *x, const int32_t *type, const double L[3],
                          const int32_t per[3], double rc, const double eps[3],
                          const double sig[3], double *F, double *U);

static int ptype(const int32_t *type, int64_t i, int64_t j)
{
    return type ? type[i] + type[j] : 0;
}

/* The pair's contribution to row i: g += J dl and th[0..5] += 1/2 dtheta terms
 * (each pair is visited from both of its rows). */
static void pair_terms(const double r[3], const double dl[3], double eps, double sig, int k,
                       double g[3], double th[6])
{
    double u = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double s2 = sig * sig, s6 = s2 * s2 * s2, s12 = s6 * s6;
    double s = 24.0 * eps * (2.0 * s12 / pow(u, 7.0) - s6 / pow(u, 4.0));
    double sp = 24.0 * eps * (-14.0 * s12 / pow(u, 8.0) + 4.0 * s6 / pow(u, 5.0));
    double dsdeps = 24.0 * (2.0 * s12 / pow(u, 7.0) - s6 / pow(u, 4.0));
    double dsdsig = 24.0 * eps * (24.0 * s12 / sig / pow(u, 7.0) - 6.0 * s6 / sig / pow(u, 4.0));
    double rdl = r[0] * dl[0] + r[1] * dl[1] + r[2] * dl[2];
    for (int a = 0; a < 3; a++) g[a] += s * dl[a] + 2.0 * sp * rdl * r[a];
    th[k] += 0.5 * dsdeps * rdl;
    th[3 + k] += 0.5 * dsdsig * rdl;
}

static void sum_theta(int64_t n, const double *rows, double gtheta[6])
{
    for (int p = 0; p < 6; p++) gtheta[p] = 0.0;
    for (int64_t i = 0; i < n; i++)
        for (int p = 0; p < 6; p++) gtheta[p] += rows[6 * i + p];
}

/* Vector-Jacobian product of the forces at FP32 positions, on the FP32 pair set
 * of squared radius rc2 (the set the forces use).  lam, gx: (n, 3). */
void oracle_lj_vjp(int64_t n, const float *pos, const int32_t *type, const float L[3],
                   const int32_t per[3], float rc2, const double eps[3], const double sig[3],
                   const double *lam, double *gx, double gtheta[6])
{
    double *th = (double *)calloc((size_t)n * 6, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double g[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; j++) {
            double r[3];
            if (j == i || !oracle_pair_f32(pos + 3 * i, pos + 3 * j, L, per, rc2, r)) continue;
            double dl[3] = {lam[3 * i] - lam[3 * j], lam[3 * i + 1] - lam[3 * j + 1],
                            lam[3 * i + 2] - lam[3 * j + 2]};
            int k = ptype(type, i, j);
            pair_terms(r, dl, eps[k], sig[k], k, g, th + 6 * i);
        }
        for (int a = 0; a < 3; a++) gx[3 * i + a] = g[a];
    }
    sum_theta(n, th, gtheta);
    free(th);
}

/* The same at FP64 positions with the FP64 minimum image and the FP64 cut-off
 * test u <= rc^2 (the set of the oracle's FP64 trajectories). */
static void vjp_f64(int64_t n, const double *x, const int32_t *type, const double L[3],
                    const int32_t per[3], double rc, const double eps[3], const double sig[3],
                    const double *lam, double *gx, double gtheta[6])
{
    double rc2 = rc * rc;
    double *th = (double *)calloc((size_t)n * 6, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double g[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double r[3];
            for (int a = 0; a < 3; a++) {
                double t = x[3 * i + a] - x[3 * j + a];
                if (per[a]) t -= L[a] * nearbyint(t / L[a]);
                r[a] = t;
            }
            if (r[0] * r[0] + r[1] * r[1] + r[2] * r[2] > rc2) continue;
            double dl[3] = {lam[3 * i] - lam[3 * j], lam[3 * i + 1] - lam[3 * j + 1],
                            lam[3 * i + 2] - lam[3 * j + 2]};
            int k = ptype(type, i, j);
            pair_terms(r, dl, eps[k], sig[k], k, g, th + 6 * i);
        }
        for (int a = 0; a < 3; a++) gx[3 * i + a] = g[a];
    }
    sum_theta(n, th, gtheta);
    free(th);
}

void oracle_lj_vjp_f64(int64_t n, const double *x, const int32_t *type, const double L[3],
                       const int32_t per[3], double rc, const double eps[3], const double sig[3],
                       const double *lam, double *gx, double gtheta[6])
{
    vjp_f64(n, x, type, L, per, rc, eps, sig, lam, gx, gtheta);
}

/* ------------------------------------------------------------------------- */
/* Trajectories.  Velocity Verlet with unit mass (section 4.1):               */
/*   v' = v_n + dt/2 F_n;  x_{n+1} = wrap(x_n + dt v');  F_{n+1} = F(x_{n+1});  */
/*   v_{n+1} = v' + dt/2 F_{n+1}.                                              */
/* xs, Fs: (nsteps + 1, n, 3), state 0 first.                                  */
/* ------------------------------------------------------------------------- */

void oracle_lj_traj(int64_t n, const double *x0, const double *v0, const int32_t *type,
                    const double L[3], const int32_t per[3], double rc, const double eps[3],
                    const double sig[3], double dt, int32_t nsteps, double *xs, double *Fs,
                    double *vs)
{
    const size_t m = (size_t)n * 3;
    double *v = (double *)malloc(sizeof(double) * m);
    double U;
    memcpy(xs, x0, sizeof(double) * m);
    memcpy(v, v0, sizeof(double) * m);
    oracle_lj_forces_f64(n, xs, type, L, per, rc, eps, sig, Fs, &U);
    if (vs) memcpy(vs, v, sizeof(double) * m);
    for (int32_t k = 0; k < nsteps; k++) {
        const double *x = xs + k * m, *F = Fs + k * m;
        double *xn = xs + (k + 1) * m, *Fn = Fs + (k + 1) * m;
        for (size_t q = 0; q < m; q++) {
            v[q] += 0.5 * dt * F[q];
            xn[q] = x[q] + dt * v[q];
        }
        for (int64_t i = 0; i < n; i++)
            for (int a = 0; a < 3; a++) {
                if (!per[a]) continue;
                double t = xn[3 * i + a];
                t -= L[a] * floor(t / L[a]);
                if (t >= L[a]) t -= L[a];
                xn[3 * i + a] = t;
            }
        oracle_lj_forces_f64(n, xn, type, L, per, rc, eps, sig, Fn, &U);
        for (size_t q = 0; q < m; q++) v[q] += 0.5 * dt * Fn[q];
        if (vs) memcpy(vs + (k + 1) * m, v, sizeof(double) * m);
    }
    free(v);
}

/* Reverse-mode derivative of a loss L(F_0, ..., F_K) through the trajectory
 * above, given the states xs (K + 1, n, 3) and fbar = dL/dF_k (K + 1, n, 3).
 * Walking the step n -> n + 1 backwards (bars are cotangents):
 *   v_{n+1} = v' + dt/2 F_{n+1}   : Fbar_{n+1} += dt/2 vbar
 *   F_{n+1} = F(x_{n+1})          : xbar += VJP_x(Fbar_{n+1}), thbar += VJP_theta
 *   x_{n+1} = x_n + dt v'          : vbar += dt xbar
 *   v' = v_n + dt/2 F_n           : Fbar_n = dt/2 vbar + fbar_n
 * and finally xbar += VJP_x(Fbar_0) at x_0 (the periodic wrap is a
 * translation and passes cotangents through).  Outputs dL/dx_0, dL/dv_0 and
 * dL/dtheta (6).  `vjp(k, lam, g, th)` evaluates the force VJP at state k. */
typedef void (*vjp_at_fn)(const void *ctx, int32_t k, const double *lam, double *g, double th[6]);

static void traj_adjoint(int64_t n, int32_t nsteps, double dt, const double *fbar, vjp_at_fn vjp,
                         const void *ctx, double *xbar, double *vbar, double gtheta[6])
{
    const size_t m = (size_t)n * 3;
    double *Fb = (double *)malloc(sizeof(double) * m);
    double *g = (double *)malloc(sizeof(double) * m);
    double th[6];
    for (int p = 0; p < 6; p++) gtheta[p] = 0.0;
    memset(xbar, 0, sizeof(double) * m);
    memset(vbar, 0, sizeof(double) * m);
    memcpy(Fb, fbar + (size_t)nsteps * m, sizeof(double) * m);
    for (int32_t k = nsteps - 1; k >= 0; k--) {
        for (size_t q = 0; q < m; q++) Fb[q] += 0.5 * dt * vbar[q];
        vjp(ctx, k + 1, Fb, g, th);
        for (int p = 0; p < 6; p++) gtheta[p] += th[p];
        for (size_t q = 0; q < m; q++) {
            xbar[q] += g[q];
            vbar[q] += dt * xbar[q];
            Fb[q] = 0.5 * dt * vbar[q] + fbar[(size_t)k * m + q];
        }
    }
    vjp(ctx, 0, Fb, g, th);
    for (int p = 0; p < 6; p++) gtheta[p] += th[p];
    for (size_t q = 0; q < m; q++) xbar[q] += g[q];
    free(Fb);
    free(g);
}

struct traj64 {
    int64_t n;
    const double *xs;
    const int32_t *type;
    const double *L;
    const int32_t *per;
    double rc;
    const double *eps, *sig;
};

static void vjp_at64(const void *c, int32_t k, const double *lam, double *g, double th[6])
{
    const struct traj64 *t = (const struct traj64 *)c;
    vjp_f64(t->n, t->xs + (size_t)k * t->n * 3, t->type, t->L, t->per, t->rc, t->eps, t->sig,
            lam, g, th);
}

void oracle_lj_traj_adjoint(int64_t n, const double *xs, const int32_t *type, const double L[3],
                            const int32_t per[3], double rc, const double eps[3],
                            const double sig[3], double dt, int32_t nsteps, const double *fbar,
                            double *xbar, double *vbar, double gtheta[6])
{
    struct traj64 t = {n, xs, type, L, per, rc, eps, sig};
    traj_adjoint(n, nsteps, dt, fbar, vjp_at64, &t, xbar, vbar, gtheta);
}

/* ------------------------------------------------------------------------- */
/* Trajectories with FP32 particle state.  The same velocity-Verlet step, but  */
/* x, v and F are stored in FP32 and each update rounds after every multiply   */
/* and add (h = dt/2 in FP32):  v = v + h F;  x = x + dt v.  Forces are the     */
/* FP64 sums on the FP32 pair set (squared radius rc2), rounded to FP32.       */
/* Positions are wrapped into the box only when the neighbour structures are  */
/* rebuilt: after a drift whose largest squared displacement since the last   */
/* rebuild (FP32 predicate arithmetic) exceeds disp2_thr, and, when            */
/* rebuild_every > 0, after every rebuild_every-th full step.  Wrap: x >= L:   */
/* x - L; x < 0: x + L; a result equal to L becomes 0.  xs, vs, Fs: (K+1, n, 3) */
/* FP32, state 0 first (x0 wrapped).                                           */
/* ------------------------------------------------------------------------- */

void oracle_lj_rows(int64_t n, const float *pos, const int32_t *type, const float L[3],
                    const int32_t per[3], float rc2, const double eps[3], const double sig[3],
                    const int64_t *rows, int64_t nrows, double *F, double *U, double *W);
float oracle_max_disp2(int64_t n, const float *pos, const float *ref, const float L[3],
                       const int32_t per[3]);

static void wrap_all_f32(int64_t n, float *x, const float L[3], const int32_t per[3])
{
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            if (!per[a]) continue;
            float t = x[3 * i + a];
            if (t >= L[a]) t = t - L[a];
            if (t < 0.0f) t = t + L[a];
            if (t >= L[a]) t = 0.0f;
            x[3 * i + a] = t;
        }
}

static void forces_f32(int64_t n, const float *x, const int32_t *type, const float L[3],
                       const int32_t per[3], float rc2, const double eps[3], const double sig[3],
                       double *tmp, float *F)
{
    oracle_lj_rows(n, x, type, L, per, rc2, eps, sig, NULL, n, tmp, NULL, NULL);
    for (int64_t q = 0; q < 3 * n; q++) F[q] = (float)tmp[q];
}

int32_t oracle_lj_traj_f32(int64_t n, const float *x0, const float *v0, const int32_t *type,
                           const float L[3], const int32_t per[3], float rc2, const double eps[3],
                           const double sig[3], float dt, float disp2_thr, int32_t rebuild_every,
                           int32_t nsteps, float *xs, float *vs, float *Fs)
{
    const size_t m = (size_t)n * 3;
    double *tmp = (double *)malloc(sizeof(double) * m);
    float *xb = (float *)malloc(sizeof(float) * m);
    float *v = (float *)malloc(sizeof(float) * m);
    const float h = 0.5f * dt;
    int32_t rebuilds = 1;
    memcpy(xs, x0, sizeof(float) * m);
    wrap_all_f32(n, xs, L, per);
    memcpy(xb, xs, sizeof(float) * m);
    memcpy(v, v0, sizeof(float) * m);
    forces_f32(n, xs, type, L, per, rc2, eps, sig, tmp, Fs);
    memcpy(vs, v, sizeof(float) * m);
    for (int32_t k = 0; k < nsteps; k++) {
        const float *F = Fs + k * m;
        float *x = xs + (k + 1) * m, *Fn = Fs + (k + 1) * m;
        memcpy(x, xs + k * m, sizeof(float) * m);
        for (size_t q = 0; q < m; q++) {
            float kick = h * F[q];
            v[q] = v[q] + kick;
            float drift = dt * v[q];
            x[q] = x[q] + drift;
        }
        if (oracle_max_disp2(n, x, xb, L, per) > disp2_thr) {
            wrap_all_f32(n, x, L, per);
            memcpy(xb, x, sizeof(float) * m);
            rebuilds++;
        }
        forces_f32(n, x, type, L, per, rc2, eps, sig, tmp, Fn);
        for (size_t q = 0; q < m; q++) {
            float kick = h * Fn[q];
            v[q] = v[q] + kick;
        }
        if (rebuild_every > 0 && (k + 1) % rebuild_every == 0 && k + 1 < nsteps) {
            wrap_all_f32(n, x, L, per);
            memcpy(xb, x, sizeof(float) * m);
            rebuilds++;
        }
        memcpy(vs + (k + 1) * m, v, sizeof(float) * m);
    }
    free(tmp);
    free(xb);
    free(v);
    return rebuilds;
}

struct traj32 {
    int64_t n;
    const float *xs;
    const int32_t *type;
    const float *L;
    const int32_t *per;
    float rc2;
    const double *eps, *sig;
};

static void vjp_at32(const void *c, int32_t k, const double *lam, double *g, double th[6])
{
    const struct traj32 *t = (const struct traj32 *)c;
    oracle_lj_vjp(t->n, t->xs + (size_t)k * t->n * 3, t->type, t->L, t->per, t->rc2, t->eps,
                  t->sig, lam, g, th);
}

/* The reverse recursion of oracle_lj_traj_adjoint over FP32 states, with the
 * force VJP on the FP32 pair set of each state. */
void oracle_lj_traj_adjoint_f32(int64_t n, const float *xs, const int32_t *type, const float L[3],
                                const int32_t per[3], float rc2, const double eps[3],
                                const double sig[3], double dt, int32_t nsteps,
                                const double *fbar, double *xbar, double *vbar, double gtheta[6])
{
    struct traj32 t = {n, xs, type, L, per, rc2, eps, sig};
    traj_adjoint(n, nsteps, dt, fbar, vjp_at32, &t, xbar, vbar, gtheta);
}
