/*
 * FP64 CPU oracle for the particle hot path of OpenFPM (arXiv 1804.07598).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the bench's CPU
 * baseline do.  It shares no code, header, table or constant with the HIP
 * library: every formula below is written out again from the paper.
 *
 * Everything is plain O(N^2) loops over all particle pairs with minimum-image
 * periodicity.  Work is split over rows (particles) with OpenMP; each row is
 * summed sequentially in index order, so results do not depend on the thread
 * count.
 *
 * Conventions shared with the callers (argument layouts, not code):
 *   positions / velocities : float or double, (n, 3) row-major;
 *   box                    : L[3] (side lengths, origin 0), per[3] (1 = periodic);
 *   pair tables            : 3 entries in upper-triangular order AA, AB, BB;
 *   virial                 : 6 entries xx, yy, zz, xy, xz, yz.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * -ffp-contract=off matters: the FP32 geometry predicate below must round
 * every product and sum separately.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Geometry in FP32: the predicate that defines every neighbour set.          */
/*                                                                           */
/* Cell lists and Verlet lists (section 2, refs [45, 46]) only decide which    */
/* pairs are candidates; the set of interacting pairs is "all j != i within    */
/* distance R" (the cut-off test returns zero beyond r_cut, section 4.1        */
/* listing).  The set is defined in FP32 so that it can be reproduced bit for  */
/* bit: per axis t = xj - xi; if t > L/2 the separation is (xj - L) - xi, if   */
/* t < -L/2 it is xj - (xi - L): the periodic image (section 3.1's ghost      */
/* copies) is taken by moving whichever of the two lies in the upper half of  */
/* the box down by one period.  That subtraction is exact (Sterbenz), so the  */
/* separation is rounded once, and swapping i and j negates it exactly: the   */
/* sets are symmetric.  Then d2 = (dx*dx + dy*dy) + dz*dz, each operation      */
/* rounded to nearest, no fused multiply-add; a pair is in the set iff         */
/* d2 <= R^2 (the listing rejects only rn > r_cut2).                           */
/* ------------------------------------------------------------------------- */

static float img_delta_f32(float xi, float xj, float L, int periodic)
{
    float t = xj - xi;
    if (!periodic) return t;
    float half = L * 0.5f;
    if (t > half) {
        float xs = xj - L;
        return xs - xi;
    }
    if (t < -half) {
        float xs = xi - L;
        return xj - xs;
    }
    return t;
}

/* Returns the branch taken: 0 = direct, +1 = xj shifted by -L, -1 = xj shifted by +L. */
static int img_branch_f32(float xi, float xj, float L, int periodic)
{
    float t = xj - xi;
    if (!periodic) return 0;
    float half = L * 0.5f;
    if (t > half) return 1;
    if (t < -half) return -1;
    return 0;
}

static float dist2_f32(const float *pi, const float *pj, const float *L, const int *per)
{
    float dx = img_delta_f32(pi[0], pj[0], L[0], per[0]);
    float dy = img_delta_f32(pi[1], pj[1], L[1], per[1]);
    float dz = img_delta_f32(pi[2], pj[2], L[2], per[2]);
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

/* Exact FP64 separation xi - xj for the image chosen by the FP32 predicate.
 * The difference of two floats is exact in double. */
static void sep_f64(const float *pi, const float *pj, const float *L, const int *per, double r[3])
{
    for (int a = 0; a < 3; a++) {
        int b = img_branch_f32(pi[a], pj[a], L[a], per[a]);
        double d = (double)pi[a] - (double)pj[a];
        if (b == 1) d += (double)L[a];       /* xj was replaced by xj - L */
        else if (b == -1) d -= (double)L[a]; /* xj was replaced by xj + L */
        r[a] = d;
    }
}

/* Pair (i, j) of FP32 positions: 1 when j is in i's set of squared radius R2
 * (the FP32 predicate above), with r = x_i - x_j in FP64 for that image.  Used
 * by the other oracle files; j == i is the caller's to exclude. */
int oracle_pair_f32(const float *pi, const float *pj, const float L[3], const int32_t per[3],
                    float R2, double r[3])
{
    int perv[3] = {per[0], per[1], per[2]};
    if (!(dist2_f32(pi, pj, L, perv) <= R2)) return 0;
    sep_f64(pi, pj, L, perv, r);
    return 1;
}

/* Squared radius of a set, R^2 rounded once to FP32 from (r_cut + skin) in FP64. */
float oracle_radius2_f32(float r_cut, float skin)
{
    double R = (double)r_cut + (double)skin;
    return (float)(R * R);
}

/* ------------------------------------------------------------------------- */
/* Cell list (section 2, ref [45]): cells of side >= R on a regular grid.      */
/* ------------------------------------------------------------------------- */

/* Number of cells per axis: the largest n with L/n >= R (with a 1e-6 relative
 * margin so that FP32 rounding of the cell index can never separate two
 * candidates by more than one cell), at least 1. */
void oracle_cell_grid(const float L[3], float r_cut, float skin, int32_t ncell[3])
{
    double R = (double)r_cut + (double)skin;
    for (int a = 0; a < 3; a++) {
        double m = floor((double)L[a] / (R * 1.000001));
        ncell[a] = m < 1.0 ? 1 : (int32_t)m;
    }
}

static int32_t cell_coord_f32(float x, float L, int32_t n)
{
    float inv = (float)n / L;
    float f = x * inv;
    if (f < 1.0f) return 0;
    if (f >= (float)n) return n - 1;
    int32_t i = (int32_t)f;
    return i > n - 1 ? n - 1 : i;
}

/* Linear cell index c = (ix * ny + iy) * nz + iz. */
void oracle_cell_index(int64_t n, const float *pos, const float L[3], const int32_t ncell[3],
                       int32_t *cid)
{
    for (int64_t i = 0; i < n; i++) {
        int32_t ix = cell_coord_f32(pos[3 * i + 0], L[0], ncell[0]);
        int32_t iy = cell_coord_f32(pos[3 * i + 1], L[1], ncell[1]);
        int32_t iz = cell_coord_f32(pos[3 * i + 2], L[2], ncell[2]);
        cid[i] = (ix * ncell[1] + iy) * ncell[2] + iz;
    }
}

/* Counting sort by cell: counts per cell, their exclusive prefix sum (offsets,
 * ncells + 1 entries) and the resulting order (order[slot] = particle index).
 * This is the cache-friendly reordering of particles by cell (section 3.6).
 * Inside a cell particles are ordered by z ascending (FP32 values as given),
 * ties by particle index; with z == NULL by particle index alone. */
static const float *g_sort_z; /* key of the comparison below (single-threaded use) */

static int cmp_z_then_index(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    if (g_sort_z[i] < g_sort_z[j]) return -1;
    if (g_sort_z[i] > g_sort_z[j]) return 1;
    return (i > j) - (i < j);
}

void oracle_cell_sort(int64_t n, const int32_t *cid, const float *z, int32_t ncells,
                      int32_t *counts, int32_t *offsets, int32_t *order)
{
    memset(counts, 0, sizeof(int32_t) * (size_t)ncells);
    for (int64_t i = 0; i < n; i++) counts[cid[i]]++;
    offsets[0] = 0;
    for (int32_t c = 0; c < ncells; c++) offsets[c + 1] = offsets[c] + counts[c];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncells);
    memcpy(fill, offsets, sizeof(int32_t) * (size_t)ncells);
    for (int64_t i = 0; i < n; i++) order[fill[cid[i]]++] = (int32_t)i;
    free(fill);
    if (z) {
        g_sort_z = z;
        for (int32_t c = 0; c < ncells; c++)
            qsort(order + offsets[c], (size_t)counts[c], sizeof(int32_t), cmp_z_then_index);
        g_sort_z = NULL;
    }
}

/* ------------------------------------------------------------------------- */
/* Brute-force neighbour sets.                                                */
/* For each requested row i (all rows when rows == NULL), every j != i with    */
/* dist2_f32 <= R2, in ascending j.  counts[r], cols[r * cap + k].             */
/* Returns 0, or -1 if some row has more than cap neighbours (its count is     */
/* still exact; only the first cap columns are stored).                        */
/* ------------------------------------------------------------------------- */
int oracle_neighbors(int64_t n, const float *pos, const float L[3], const int32_t per[3],
                     float R2, const int64_t *rows, int64_t nrows, int32_t *counts,
                     int32_t *cols, int64_t cap)
{
    int overflow = 0;
    int64_t nr = rows ? nrows : n;
    int perv[3] = {per[0], per[1], per[2]};
#pragma omp parallel for schedule(dynamic, 16) reduction(| : overflow)
    for (int64_t r = 0; r < nr; r++) {
        int64_t i = rows ? rows[r] : r;
        int32_t c = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            if (dist2_f32(pos + 3 * i, pos + 3 * j, L, perv) <= R2) {
                if (c < cap) cols[r * cap + c] = (int32_t)j;
                c++;
            }
        }
        counts[r] = c;
        if (c > cap) overflow = 1;
    }
    return overflow ? -1 : 0;
}

/* Maximum over particles of the minimum-image squared displacement from a
 * reference configuration, in the same FP32 arithmetic (Verlet-list rebuild
 * test: rebuild iff this exceeds (skin/2)^2). */
float oracle_max_disp2(int64_t n, const float *pos, const float *ref, const float L[3],
                       const int32_t per[3])
{
    float m = 0.0f;
    int perv[3] = {per[0], per[1], per[2]};
    for (int64_t i = 0; i < n; i++) {
        float d2 = dist2_f32(ref + 3 * i, pos + 3 * i, L, perv);
        if (d2 > m) m = d2;
    }
    return m;
}

/* ------------------------------------------------------------------------- */
/* Lennard-Jones (section 4.1): V(r) = 4 eps ((sig/r)^12 - (sig/r)^6); the     */
/* force on p from q is 24 eps (2 sig^12 / rn^7 - sig^6 / rn^4) (xp - xq) with  */
/* rn = |xp - xq|^2, and zero when rn > r_cut^2 (truncated, not shifted).      */
/* ------------------------------------------------------------------------- */

static int pair_index(int32_t ti, int32_t tj)
{
    return ti + tj; /* 0 = AA, 1 = AB, 2 = BB for two types */
}

static double lj_s(double u, double eps, double sig)
{
    double s2 = sig * sig, s6 = s2 * s2 * s2, s12 = s6 * s6;
    return 24.0 * eps * (2.0 * s12 / pow(u, 7.0) - s6 / pow(u, 4.0));
}

static double lj_v(double u, double eps, double sig)
{
    double s2 = sig * sig, s6 = s2 * s2 * s2, s12 = s6 * s6;
    return 4.0 * eps * (s12 / pow(u, 6.0) - s6 / pow(u, 3.0));
}

/* Per requested row i: F_i = sum_j s(u) r_ij (r_ij = x_i - x_j, exact FP64 image
 * of the FP32 predicate's choice), U_i = 1/2 sum_j V(u), W_i = 1/2 sum_j r (x) F.
 * Pairs are those with dist2_f32 <= rc2.  Totals are sums over rows. */
void oracle_lj_rows(int64_t n, const float *pos, const int32_t *type, const float L[3],
                    const int32_t per[3], float rc2, const double eps[3], const double sig[3],
                    const int64_t *rows, int64_t nrows, double *F, double *U, double *W)
{
    int64_t nr = rows ? nrows : n;
    int perv[3] = {per[0], per[1], per[2]};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; r++) {
        int64_t i = rows ? rows[r] : r;
        double f[3] = {0, 0, 0}, u = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            if (!(dist2_f32(pos + 3 * i, pos + 3 * j, L, perv) <= rc2)) continue;
            double d[3];
            sep_f64(pos + 3 * i, pos + 3 * j, L, perv, d);
            double rn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            int k = type ? pair_index(type[i], type[j]) : 0;
            double s = lj_s(rn, eps[k], sig[k]);
            for (int a = 0; a < 3; a++) f[a] += s * d[a];
            u += 0.5 * lj_v(rn, eps[k], sig[k]);
            w[0] += 0.5 * d[0] * s * d[0];
            w[1] += 0.5 * d[1] * s * d[1];
            w[2] += 0.5 * d[2] * s * d[2];
            w[3] += 0.5 * d[0] * s * d[1];
            w[4] += 0.5 * d[0] * s * d[2];
            w[5] += 0.5 * d[1] * s * d[2];
        }
        for (int a = 0; a < 3; a++) F[3 * r + a] = f[a];
        if (U) U[r] = u;
        if (W) for (int a = 0; a < 6; a++) W[6 * r + a] = w[a];
    }
}

/* Sum of |r . F_pair| over pairs (each pair once), the scale for virial errors. */
double oracle_lj_virial_scale(int64_t n, const float *pos, const int32_t *type, const float L[3],
                              const int32_t per[3], float rc2, const double eps[3],
                              const double sig[3])
{
    double total = 0.0;
    int perv[3] = {per[0], per[1], per[2]};
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t i = 0; i < n; i++) {
        double acc = 0.0;
        for (int64_t j = i + 1; j < n; j++) {
            if (!(dist2_f32(pos + 3 * i, pos + 3 * j, L, perv) <= rc2)) continue;
            double d[3];
            sep_f64(pos + 3 * i, pos + 3 * j, L, perv, d);
            double rn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            int k = type ? pair_index(type[i], type[j]) : 0;
            acc += fabs(lj_s(rn, eps[k], sig[k]) * rn);
        }
        total += acc;
    }
    return total;
}

/* ------------------------------------------------------------------------- */
/* Velocity Verlet (section 4.1): v += dt/2 F/m; x += dt v; wrap into the box  */
/* (on one address space the "map" of particles that left the domain is the    */
/* periodic wrap); F = F(x); v += dt/2 F/m.  All in FP64 with an FP64 cut-off  */
/* test and FP64 minimum image; this is the oracle's own trajectory.           */
/* thermo[(s) * 2 + 0] = U, thermo[s * 2 + 1] = KE for s = 0..nsteps.          */
/* ------------------------------------------------------------------------- */

static void lj_forces_f64(int64_t n, const double *x, const int32_t *type, const double L[3],
                          const int32_t per[3], double rc, const double eps[3], const double sig[3],
                          double *F, double *Uout)
{
    double rc2 = rc * rc, Utot = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : Utot)
    for (int64_t i = 0; i < n; i++) {
        double f[3] = {0, 0, 0}, u = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double d[3];
            for (int a = 0; a < 3; a++) {
                double t = x[3 * i + a] - x[3 * j + a];
                if (per[a]) t -= L[a] * nearbyint(t / L[a]);
                d[a] = t;
            }
            double rn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (rn > rc2) continue;
            int k = type ? pair_index(type[i], type[j]) : 0;
            double s = lj_s(rn, eps[k], sig[k]);
            for (int a = 0; a < 3; a++) f[a] += s * d[a];
            u += 0.5 * lj_v(rn, eps[k], sig[k]);
        }
        for (int a = 0; a < 3; a++) F[3 * i + a] = f[a];
        Utot += u;
    }
    *Uout = Utot;
}

static void wrap_f64(int64_t n, double *x, const double L[3], const int32_t per[3])
{
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            if (!per[a]) continue;
            double v = x[3 * i + a];
            v -= L[a] * floor(v / L[a]);
            if (v >= L[a]) v -= L[a];
            x[3 * i + a] = v;
        }
}

static double kinetic_f64(int64_t n, const double *v, double mass)
{
    double k = 0.0;
    for (int64_t i = 0; i < 3 * n; i++) k += v[i] * v[i];
    return 0.5 * mass * k;
}

void oracle_vv(int64_t n, double *x, double *v, const int32_t *type, const double L[3],
               const int32_t per[3], double rc, const double eps[3], const double sig[3],
               double mass, double dt, int32_t nsteps, double *thermo)
{
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double U;
    lj_forces_f64(n, x, type, L, per, rc, eps, sig, F, &U);
    if (thermo) { thermo[0] = U; thermo[1] = kinetic_f64(n, v, mass); }
    for (int32_t s = 1; s <= nsteps; s++) {
        for (int64_t i = 0; i < 3 * n; i++) {
            v[i] += 0.5 * dt * F[i] / mass;
            x[i] += dt * v[i];
        }
        wrap_f64(n, x, L, per);
        lj_forces_f64(n, x, type, L, per, rc, eps, sig, F, &U);
        for (int64_t i = 0; i < 3 * n; i++) v[i] += 0.5 * dt * F[i] / mass;
        if (thermo) { thermo[2 * s] = U; thermo[2 * s + 1] = kinetic_f64(n, v, mass); }
    }
    free(F);
}

/* Forces of the FP64 trajectory code, exposed for the adjoint tests. */
void oracle_lj_forces_f64(int64_t n, const double *x, const int32_t *type, const double L[3],
                          const int32_t per[3], double rc, const double eps[3],
                          const double sig[3], double *F, double *U)
{
    lj_forces_f64(n, x, type, L, per, rc, eps, sig, F, U);
}

/* Number of OpenMP threads the oracle's loops use. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
