/*
 * FP64 CPU oracle for the weakly compressible SPH sums of OpenFPM's section
 * 4.2 (Eqs. 1-5).  TEST INFRASTRUCTURE ONLY (see oracle.c).
 *
 * Readings taken where the paper is silent or garbled:
 *  - kernel (prm[10]): 0 = Wendland C2 with support 2h,
 *    W(r) = aD (1 - q/2)^4 (2q + 1), q = r/h, aD = 21 / (16 pi h^3);
 *    1 = the classic cubic spline the paper names, support 2h,
 *    W = aD (1 - 3q^2/2 + 3q^3/4) for q < 1, aD (2 - q)^3 / 4 for 1 <= q < 2,
 *    aD = 1 / (pi h^3); the paper's cutoff 2 sqrt(3) dp is h = sqrt(3) dp;
 *  - gradient: grad_a W_ab = dW/dr (x_a - x_b) / r, so a compressed pair repels;
 *  - Eq. 4: B = c0^2 rho0 / gamma with c0 given directly;
 *  - Eq. 5: Pi_ab = -alpha cbar mu_ab / rhobar_ab for approaching pairs
 *    (v_ab . x_ab < 0), zero otherwise; mu_ab = h v_ab.x_ab / (r^2 + eta^2);
 *    rhobar_ab = (rho_a + rho_b) / 2; cbar = prm[11] when positive (the
 *    paper's sqrt(g h_swl)), else c0;
 *  - boundary particles (kind 1) enter every sum and get a density rate, but
 *    no acceleration.
 * The pair set is the FP32 predicate of oracle.c with R = 2h.
 */
#include <math.h>
#include <stdint.h>

static const double PI = 3.14159265358979323846;

static int branch_f32(float xi, float xj, float L, int periodic)
{
    float t = xj - xi;
    if (!periodic) return 0;
    float half = L * 0.5f;
    if (t > half) return 1;
    if (t < -half) return -1;
    return 0;
}

static float delta_f32(float xi, float xj, float L, int periodic)
{
    float t = xj - xi;
    int b = branch_f32(xi, xj, L, periodic);
    if (b == 1) {
        float s = xj - L;
        return s - xi;
    }
    if (b == -1) {
        float s = xi - L;
        return xj - s;
    }
    return t;
}

static float d2_f32(const float *pi, const float *pj, const float *L, const int32_t *per)
{
    float dx = delta_f32(pi[0], pj[0], L[0], per[0]);
    float dy = delta_f32(pi[1], pj[1], L[1], per[1]);
    float dz = delta_f32(pi[2], pj[2], L[2], per[2]);
    float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

/* Wendland C2 kernel value at distance r (3-D normalisation). */
double oracle_sph_kernel_w(double r, double h)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    double aD = 21.0 / (16.0 * PI * h * h * h);
    double t = 1.0 - 0.5 * q;
    return aD * t * t * t * t * (2.0 * q + 1.0);
}

/* Cubic spline kernel value at distance r (3-D normalisation). */
double oracle_sph_cubic_w(double r, double h)
{
    double q = r / h;
    double aD = 1.0 / (PI * h * h * h);
    if (q >= 2.0) return 0.0;
    if (q < 1.0) return aD * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
    double t = 2.0 - q;
    return aD * 0.25 * t * t * t;
}

/* dW/dr of the kernel selected by `kernel` (0 Wendland C2, 1 cubic spline). */
double oracle_sph_kernel_dwdr(double r, double h, int kernel)
{
    double q = r / h;
    if (q >= 2.0) return 0.0;
    if (kernel == 1) {
        double aD = 1.0 / (PI * h * h * h);
        if (q < 1.0) return aD * (-3.0 * q + 2.25 * q * q) / h;
        double t = 2.0 - q;
        return aD * (-0.75 * t * t) / h;
    }
    double aD = 21.0 / (16.0 * PI * h * h * h);
    double t = 1.0 - 0.5 * q;
    /* d/dq [t^4 (2q + 1)] = -2 t^3 (2q + 1) + 2 t^4 = -5 q t^3 */
    return aD * (-5.0 * q * t * t * t) / h;
}

static double pressure(double rho, double rho0, double c0, double gamma)
{
    double B = c0 * c0 * rho0 / gamma;
    return B * (pow(rho / rho0, gamma) - 1.0);
}

/*
 * prm = {h, m, rho0, c0, gamma, alpha, eta2, gx, gy, gz, kernel, cbar}.
 * For each requested row a: acc (3), drho, mumax = max over its pairs of |mu_ab|.
 */
void oracle_sph_rows(int64_t n, const float *pos, const float *vel, const float *rho,
                     const int32_t *kind, const float L[3], const int32_t per[3], float R2,
                     const double *prm, const int64_t *rows, int64_t nrows, double *acc,
                     double *drho, double *mumax)
{
    const double h = prm[0], m = prm[1], rho0 = prm[2], c0 = prm[3], gamma = prm[4];
    const double alpha = prm[5], eta2 = prm[6];
    const int kernel = (int)prm[10];
    const double cbar = prm[11] > 0.0 ? prm[11] : c0;
    int64_t nr = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nr; r++) {
        int64_t a = rows ? rows[r] : r;
        double ax = 0, ay = 0, az = 0, dr = 0, mu_max = 0;
        double ra = rho[a];
        double Pa = pressure(ra, rho0, c0, gamma);
        for (int64_t b = 0; b < n; b++) {
            if (b == a) continue;
            if (!(d2_f32(pos + 3 * a, pos + 3 * b, L, per) <= R2)) continue;
            double x[3];
            for (int k = 0; k < 3; k++) {
                int br = branch_f32(pos[3 * a + k], pos[3 * b + k], L[k], per[k]);
                double d = (double)pos[3 * a + k] - (double)pos[3 * b + k];
                if (br == 1) d += (double)L[k];
                else if (br == -1) d -= (double)L[k];
                x[k] = d; /* x_a - x_b */
            }
            double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
            double rr = sqrt(r2);
            double gfac = oracle_sph_kernel_dwdr(rr, h, kernel) / rr; /* grad_a W_ab = gfac x_ab */
            double v[3];
            for (int k = 0; k < 3; k++) v[k] = (double)vel[3 * a + k] - (double)vel[3 * b + k];
            double vx = v[0] * x[0] + v[1] * x[1] + v[2] * x[2];
            dr += m * vx * gfac;
            double rb = rho[b];
            double Pb = pressure(rb, rho0, c0, gamma);
            double mu = h * vx / (r2 + eta2);
            double Pi = 0.0;
            if (vx < 0.0) Pi = -alpha * cbar * mu / (0.5 * (ra + rb));
            if (fabs(mu) > mu_max) mu_max = fabs(mu);
            double coef = -m * ((Pa + Pb) / (ra * rb) + Pi) * gfac;
            ax += coef * x[0];
            ay += coef * x[1];
            az += coef * x[2];
        }
        if (kind[a] == 0) {
            acc[3 * r + 0] = ax + prm[7];
            acc[3 * r + 1] = ay + prm[8];
            acc[3 * r + 2] = az + prm[9];
        } else {
            acc[3 * r + 0] = 0.0;
            acc[3 * r + 1] = 0.0;
            acc[3 * r + 2] = 0.0;
        }
        drho[r] = dr;
        mumax[r] = mu_max;
    }
}
