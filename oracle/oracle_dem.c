/*
 * FP64 CPU oracle for the discrete-element grains of OpenFPM's DEM client
 * (section 4.5: the Silbert grain model with Hertzian contacts, Eqs. 9-13).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it shares no code with the HIP library.
 *
 * State: positions x, velocities v, angular velocities w (FP64), all grains of
 * radius R, mass m, moment of inertia I.  prm = {R, m, I, kn, kt, gn, gt, mu,
 * gx, gy, gz, dt, walls}.  A pair (p, q) is in contact when the minimum-image
 * separation r_pq = x_p - x_q has |r_pq| < 2R (FP64).  Readings taken where
 * the paper is silent:
 *  - n = r_pq / |r_pq|, delta = 2R - |r_pq| (Eq. 9), m_eff = m / 2;
 *  - the contact point lies midway between the centres, at arm a = |r_pq| / 2
 *    from each (so the pair's torques balance its tangential forces exactly
 *    and angular momentum is conserved); its relative velocity is
 *        v_pq = v_p - v_q - a (w_p + w_q) x n,
 *    v_n = (v_pq . n) n, v_t = v_pq - v_n;
 *  - tangential history u_t of the pair, kept by p under q's id (and by q
 *    under p's, with the opposite sign): u_t <- u_t + v_t dt (Eq. 10), then
 *    its normal component is removed so that it stays in the contact plane;
 *    a pair that loses contact forgets it;
 *  - F_n = s (kn delta n - gn m_eff v_n), F_t = s (-kt u_t - gt m_eff v_t),
 *    s = sqrt(delta / 2R) (Eqs. 11-12);
 *  - Coulomb's law: when |F_t| > mu |F_n|, F_t is scaled down to mu |F_n| and
 *    u_t is set to the value that gives that force, -(F_t / s + gt m_eff v_t) / kt;
 *  - torque on p: (-a n) x F_t;
 *  - walls (bit 1: planes x = 0 and x = L_x; bit 2: floor z = 0): a grain
 *    closer than R to a wall gets the normal force of Eq. 11 with the wall's
 *    normal, delta = R - distance and m_eff = m, and no tangential force;
 *  - gravity m g; the leapfrog of Eq. 13: v += dt F / m, x += dt v (new v),
 *    w += dt T / I.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/*
 * Force f and torque t on grain p at the state (x, v, w), its contact
 * history (hid_p, hu_p: C slots of partner id, -1 empty, and u_t) and the
 * updated history of its current contacts in ascending partner order
 * (hid_o, hu_o); returns its number of contacts (only the first C stored).
 */
static int dem_grain(int64_t p, int64_t n, const double *x, const double *v, const double *w,
                     const float L[3], const int32_t per[3], const double *prm, int C,
                     const int64_t *hid_p, const double *hu_p, double f[3], double t[3],
                     int64_t *hid_o, double *hu_o)
{
    const double R = prm[0], m = prm[1], kn = prm[3], kt = prm[4];
    const double gn = prm[5], gt = prm[6], mu = prm[7], dt = prm[11];
    const int walls = (int)prm[12];
    const double meff = 0.5 * m, d2max = 4.0 * R * R;
    f[0] = m * prm[8], f[1] = m * prm[9], f[2] = m * prm[10];
    t[0] = t[1] = t[2] = 0.0;
    int nc = 0;
    for (int c = 0; c < C; c++) hid_o[c] = -1;
    for (int64_t q = 0; q < n; q++) {
        if (q == p) continue;
        double r[3];
        for (int k = 0; k < 3; k++) {
            double d = x[3 * p + k] - x[3 * q + k];
            if (per[k]) {
                if (d > 0.5 * L[k]) d -= L[k];
                else if (d < -0.5 * L[k]) d += L[k];
            }
            r[k] = d;
        }
        const double rr2 = dot(r, r);
        if (!(rr2 < d2max)) continue;
        const double rr = sqrt(rr2);
        const double nv[3] = {r[0] / rr, r[1] / rr, r[2] / rr};
        const double a = 0.5 * rr;
        const double delta = 2.0 * R - rr;
        double ws[3] = {w[3 * p] + w[3 * q], w[3 * p + 1] + w[3 * q + 1],
                        w[3 * p + 2] + w[3 * q + 2]}, rot[3];
        cross(ws, nv, rot);
        double vr[3];
        for (int k = 0; k < 3; k++) vr[k] = v[3 * p + k] - v[3 * q + k] - a * rot[k];
        const double vn = dot(vr, nv);
        double vt[3];
        for (int k = 0; k < 3; k++) vt[k] = vr[k] - vn * nv[k];
        double u[3] = {0, 0, 0};
        for (int c = 0; c < C; c++)
            if (hid_p[c] == q) {
                for (int k = 0; k < 3; k++) u[k] = hu_p[c * 3 + k];
                break;
            }
        for (int k = 0; k < 3; k++) u[k] += vt[k] * dt;
        const double un = dot(u, nv);
        for (int k = 0; k < 3; k++) u[k] -= un * nv[k];
        const double s = sqrt(delta / (2.0 * R));
        double fn[3], ft[3];
        for (int k = 0; k < 3; k++) {
            fn[k] = s * (kn * delta * nv[k] - gn * meff * vn * nv[k]);
            ft[k] = s * (-kt * u[k] - gt * meff * vt[k]);
        }
        const double fnm = sqrt(dot(fn, fn)), ftm = sqrt(dot(ft, ft));
        if (ftm > mu * fnm) {
            const double sc = mu * fnm / ftm;
            for (int k = 0; k < 3; k++) ft[k] *= sc;
            if (kt > 0.0)
                for (int k = 0; k < 3; k++) u[k] = -(ft[k] / s + gt * meff * vt[k]) / kt;
        }
        double arm[3] = {-a * nv[0], -a * nv[1], -a * nv[2]}, tq[3];
        cross(arm, ft, tq);
        for (int k = 0; k < 3; k++) {
            f[k] += fn[k] + ft[k];
            t[k] += tq[k];
        }
        if (nc < C) {
            hid_o[nc] = q;
            for (int k = 0; k < 3; k++) hu_o[nc * 3 + k] = u[k];
        }
        nc++;
    }
    /* walls: normal force only */
    for (int wall = 0; wall < 3; wall++) {
        double nw[3] = {0, 0, 0}, dist;
        if (wall == 0) {
            if (!(walls & 1)) continue;
            dist = x[3 * p];
            nw[0] = 1.0;
        } else if (wall == 1) {
            if (!(walls & 1)) continue;
            dist = L[0] - x[3 * p];
            nw[0] = -1.0;
        } else {
            if (!(walls & 2)) continue;
            dist = x[3 * p + 2];
            nw[2] = 1.0;
        }
        if (!(dist < R)) continue;
        const double delta = R - dist;
        const double s = sqrt(delta / (2.0 * R));
        const double vn = dot(v + 3 * p, nw);
        for (int k = 0; k < 3; k++) f[k] += s * (kn * delta * nw[k] - gn * m * vn * nw[k]);
    }
    return nc;
}

/*
 * Forces F (n x 3) and torques T (n x 3) at the state (x, v, w) with the
 * history (hid_in, hu_in): for grain p, slots c < C hold a partner id
 * (-1: empty) and its u_t.  The updated history of the current contacts goes
 * to (hid_out, hu_out) in ascending partner order; ncontact[p] counts them
 * (it may exceed C: only the first C are stored).  Returns the largest count.
 */
int oracle_dem_forces(int64_t n, const double *x, const double *v, const double *w,
                      const float L[3], const int32_t per[3], const double *prm, int C,
                      const int64_t *hid_in, const double *hu_in, double *F, double *T,
                      int64_t *hid_out, double *hu_out, int32_t *ncontact)
{
    int worst = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : worst)
    for (int64_t p = 0; p < n; p++) {
        const int nc = dem_grain(p, n, x, v, w, L, per, prm, C, hid_in + p * C,
                                 hu_in + p * C * 3, F + 3 * p, T + 3 * p, hid_out + p * C,
                                 hu_out + p * C * 3);
        ncontact[p] = nc;
        if (nc > worst) worst = nc;
    }
    return worst;
}

/*
 * The same evaluation for the grains rows[0 .. nrows) only, with no contact
 * history (every pair starts from u_t = 0): force and torque of row r in
 * F[3 r], T[3 r], its contact count in ncontact[r].
 */
void oracle_dem_forces_rows(int64_t n, const double *x, const double *v, const double *w,
                            const float L[3], const int32_t per[3], const double *prm,
                            const int64_t *rows, int64_t nrows, double *F, double *T,
                            int32_t *ncontact)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t hid_p[1] = {-1}, hid_o[1];
        double hu_p[3] = {0, 0, 0}, hu_o[3];
        ncontact[r] = dem_grain(rows[r], n, x, v, w, L, per, prm, 1, hid_p, hu_p, F + 3 * r,
                                T + 3 * r, hid_o, hu_o);
    }
}

/* One leapfrog step of Eq. 13 with the forces and torques given. */
void oracle_dem_leapfrog(int64_t n, double *x, double *v, double *w, const double *F,
                         const double *T, const double *prm)
{
    const double m = prm[1], I = prm[2], dt = prm[11];
    for (int64_t p = 0; p < 3 * n; p++) {
        v[p] += dt * F[p] / m;
        x[p] += dt * v[p];
        w[p] += dt * T[p] / I;
    }
}
