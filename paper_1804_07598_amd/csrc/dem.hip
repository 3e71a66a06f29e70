// Discrete-element grains (section 4.5): the Silbert model with Hertzian
// contacts (Eqs. 9-12) and the leapfrog of Eq. 13, over the Verlet list at
// radius 2R + skin.
//
// Per grain p and each neighbour q with |r_pq| < 2R (FP64 from the exact
// separation of the FP32 coordinates), n = r_pq / |r_pq|, delta = 2R - |r_pq|,
// s = sqrt(delta / 2R), m_eff = m / 2 and the contact point midway between
// the centres (arm a = |r_pq| / 2):
//   v_pq = v_p - v_q - a (w_p + w_q) x n,  v_n = (v_pq . n) n, v_t = v_pq - v_n
//   u_t <- u_t + v_t dt, minus its normal component       (Eq. 10)
//   F_n = s (kn delta n - gn m_eff v_n), F_t = s (-kt u_t - gt m_eff v_t)
//   if |F_t| > mu |F_n|: F_t scaled to mu |F_n|, u_t = -(F_t / s + gt m_eff v_t) / kt
//   F_p += F_n + F_t, T_p += (-a n) x F_t.
// Walls (bit 1: x = 0 and x = L_x, bit 2: z = 0) push with Eq. 11's normal
// force (delta = R - distance, m_eff = m).  Gravity m g.
//
// Contact history: for each grain, by caller index, up to C (partner caller
// index, u_t) slots; p and q each keep their own copy (u_t of (q, p) is minus
// that of (p, q), and both update with exactly negated arithmetic).  A step
// reads one buffer and writes the current contacts to the other, so grains
// never share a write.  Angular velocity lives in the per-slot buffer the
// cell sort carries along; torques in the per-slot scratch.
#include "geom.h"

namespace fpm {
namespace {

struct DemCoef {
    double R, m, inv_m, inv_I, kn, kt, gn, gt, mu, dt, meff, inv_2R, d2max;
    double g[3];
    float dtf, g32[3];
    int walls;
    int C;
};

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Forces and torques of the grains; history read from buffer rb, the current
// contacts written to buffer 1 - rb.
__global__ __launch_bounds__(kBlock) void k_dem_forces(State st, DemCoef k, int rb, int cap4) {
    const SysDesc &d = st.sys[block_system(st)];
    const Box b = d.box;
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
    const float4 *__restrict__ pos = st.pos[0];
    const float4 *__restrict__ vel = st.vel[0];
    const float4 *__restrict__ om = st.old[0];
    const int32_t *__restrict__ id = st.id[0];
    const int C = k.C;
    const int64_t me = id[i];
    const int32_t *hid_in = st.hid[rb] + me * C;
    const float4 *hu_in = st.hu[rb] + me * C;
    int32_t *hid_out = st.hid[1 - rb] + me * C;
    float4 *hu_out = st.hu[1 - rb] + me * C;
    const float4 pi4 = pos[i], vi4 = vel[i], wi4 = om[i];
    const float3 pi = xyz(pi4);
    double f[3] = {k.m * k.g[0], k.m * k.g[1], k.m * k.g[2]}, t[3] = {0.0, 0.0, 0.0};
    int nc = 0;
    const int cnt = (int)(st.nnb[i] & ~kWrapBit);
    for (int e = 0; e < cnt; e++) {
        const int j = st.nbr[nbr_index(i, e, cap4)];
        const float4 q4 = pos[j];
        double r[3] = {sep_axis(pi.x, q4.x, b.L[0], b.half[0], b.per[0]),
                       sep_axis(pi.y, q4.y, b.L[1], b.half[1], b.per[1]),
                       sep_axis(pi.z, q4.z, b.L[2], b.half[2], b.per[2])};
        const double rr2 = dot3(r, r);
        if (!(rr2 < k.d2max)) continue;
        const float4 vj4 = vel[j], wj4 = om[j];
        const int64_t qid = id[j];
        const double rr = sqrt(rr2);
        const double nv[3] = {r[0] / rr, r[1] / rr, r[2] / rr};
        const double a = 0.5 * rr;
        const double delta = 2.0 * k.R - rr;
        const double ws[3] = {(double)wi4.x + (double)wj4.x, (double)wi4.y + (double)wj4.y,
                              (double)wi4.z + (double)wj4.z};
        double rot[3];
        cross3(ws, nv, rot);
        const double vr[3] = {(double)vi4.x - (double)vj4.x - a * rot[0],
                              (double)vi4.y - (double)vj4.y - a * rot[1],
                              (double)vi4.z - (double)vj4.z - a * rot[2]};
        const double vn = dot3(vr, nv);
        const double vt[3] = {vr[0] - vn * nv[0], vr[1] - vn * nv[1], vr[2] - vn * nv[2]};
        double u[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < C; c++)
            if (hid_in[c] == qid) {
                const float4 h = hu_in[c];
                u[0] = h.x, u[1] = h.y, u[2] = h.z;
                break;
            }
        for (int c3 = 0; c3 < 3; c3++) u[c3] += vt[c3] * k.dt;
        const double un = dot3(u, nv);
        for (int c3 = 0; c3 < 3; c3++) u[c3] -= un * nv[c3];
        const double s = sqrt(delta * k.inv_2R);
        double fn[3], ft[3];
        for (int c3 = 0; c3 < 3; c3++) {
            fn[c3] = s * (k.kn * delta * nv[c3] - k.gn * k.meff * vn * nv[c3]);
            ft[c3] = s * (-k.kt * u[c3] - k.gt * k.meff * vt[c3]);
        }
        const double fnm = sqrt(dot3(fn, fn)), ftm = sqrt(dot3(ft, ft));
        if (ftm > k.mu * fnm) {
            const double sc = k.mu * fnm / ftm;
            for (int c3 = 0; c3 < 3; c3++) ft[c3] *= sc;
            if (k.kt > 0.0)
                for (int c3 = 0; c3 < 3; c3++) u[c3] = -(ft[c3] / s + k.gt * k.meff * vt[c3]) / k.kt;
        }
        const double arm[3] = {-a * nv[0], -a * nv[1], -a * nv[2]};
        double tq[3];
        cross3(arm, ft, tq);
        for (int c3 = 0; c3 < 3; c3++) {
            f[c3] += fn[c3] + ft[c3];
            t[c3] += tq[c3];
        }
        if (nc < C) {
            hid_out[nc] = (int32_t)qid;
            hu_out[nc] = make_float4((float)u[0], (float)u[1], (float)u[2], 0.f);
        }
        nc++;
    }
    for (int c = nc; c < C; c++) hid_out[c] = -1;
    // walls: normal force only
    for (int wall = 0; wall < 3; wall++) {
        double nw[3] = {0.0, 0.0, 0.0}, dist;
        if (wall == 0) {
            if (!(k.walls & 1)) continue;
            dist = (double)pi.x;
            nw[0] = 1.0;
        } else if (wall == 1) {
            if (!(k.walls & 1)) continue;
            dist = (double)b.L[0] - (double)pi.x;
            nw[0] = -1.0;
        } else {
            if (!(k.walls & 2)) continue;
            dist = (double)pi.z;
            nw[2] = 1.0;
        }
        if (!(dist < k.R)) continue;
        const double delta = k.R - dist;
        const double s = sqrt(delta * k.inv_2R);
        const double vv[3] = {vi4.x, vi4.y, vi4.z};
        const double vn = dot3(vv, nw);
        for (int c3 = 0; c3 < 3; c3++) f[c3] += s * (k.kn * delta * nw[c3] - k.gn * k.m * vn * nw[c3]);
    }
    st.frc[i] = make_float4((float)f[0], (float)f[1], (float)f[2], 0.f);
    st.aux[i] = make_float4((float)t[0], (float)t[1], (float)t[2], 0.f);
    st.ncon[me] = nc;
    if (nc > C) st.ctl->overflow = nc;
    if (!isfinite(f[0]) || !isfinite(f[1]) || !isfinite(f[2])) st.ctl->nonfinite = 1;
}

// The leapfrog of Eq. 13 in FP32: v += dt F / m, x += dt v, w += dt T / I,
// and the displacement since the last rebuild for the rebuild decision.
__global__ __launch_bounds__(kBlock) void k_dem_integrate(State st, DemCoef k) {
#pragma clang fp contract(off)
    const SysDesc &d = st.sys[block_system(st)];
    const Box b = d.box;
    const int64_t i = global_slot();
    double dsp = 0.0;
    if (i - d.slot_base < d.n) {
        const float dt = k.dtf;
        const float im = (float)k.inv_m, iI = (float)k.inv_I;
        float4 v = st.vel[0][i], p = st.pos[0][i], w = st.old[0][i];
        const float4 f = st.frc[i], tq = st.aux[i];
        v.x = v.x + dt * (f.x * im);
        v.y = v.y + dt * (f.y * im);
        v.z = v.z + dt * (f.z * im);
        p.x = p.x + dt * v.x;
        p.y = p.y + dt * v.y;
        p.z = p.z + dt * v.z;
        w.x = w.x + dt * (tq.x * iI);
        w.y = w.y + dt * (tq.y * iI);
        w.z = w.z + dt * (tq.z * iI);
        st.vel[0][i] = v;
        st.pos[0][i] = p;
        st.old[0][i] = w;
        if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z)) st.ctl->nonfinite = 1;
        dsp = dist2_pred(xyz(st.xbuild[i]), xyz(p), b);
    }
    double v1[1] = {dsp};
    const int slot[1] = {kSlotDisp};
    const int op[1] = {1};
    block_partials<1>(v1, slot, op, st.part, st.pstride);
}

// Angular velocities from the caller's order; contact history cleared.
__global__ void k_dem_set_omega(State st, const float *w) {
    const SysDesc &d = st.sys[block_system(st)];
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
    const int64_t r = st.id[0][i];
    st.old[0][i] = w ? make_float4(w[3 * r], w[3 * r + 1], w[3 * r + 2], 0.f)
                     : make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_dem_clear(State st, int64_t n, int C) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * C) {
        st.hid[0][t] = -1;
        st.hid[1][t] = -1;
    }
    if (t < n) st.ncon[t] = 0;
}

__global__ void k_dem_out(State st, float *w, float *tq) {
    const SysDesc &d = st.sys[block_system(st)];
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
    const int64_t r = st.id[0][i];
    const float4 a = st.old[0][i], b = st.aux[i];
    if (w) w[3 * r] = a.x, w[3 * r + 1] = a.y, w[3 * r + 2] = a.z;
    if (tq) tq[3 * r] = b.x, tq[3 * r + 1] = b.y, tq[3 * r + 2] = b.z;
}

__global__ void k_dem_contacts_out(State st, int rb, int64_t n, int C, int32_t *ids, float *ut,
                                   int32_t *ncon) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * C) {
        if (ids) ids[t] = st.hid[rb][t];
        if (ut) {
            const float4 h = st.hu[rb][t];
            ut[3 * t] = h.x, ut[3 * t + 1] = h.y, ut[3 * t + 2] = h.z;
        }
    }
    if (ncon && t < n) ncon[t] = st.ncon[t];
}

DemCoef make_coef(const fpm_ctx *c, const fpm_dem_params &p) {
    DemCoef k;
    k.R = p.R;
    k.m = p.mass;
    k.inv_m = 1.0 / (double)p.mass;
    k.inv_I = 1.0 / (double)p.inertia;
    k.kn = p.kn;
    k.kt = p.kt;
    k.gn = p.gn;
    k.gt = p.gt;
    k.mu = p.mu;
    k.dt = p.dt;
    k.dtf = p.dt;
    k.meff = 0.5 * (double)p.mass;
    k.inv_2R = 1.0 / (2.0 * (double)p.R);
    k.d2max = 4.0 * (double)p.R * (double)p.R;
    for (int a = 0; a < 3; a++) k.g[a] = p.g[a], k.g32[a] = p.g[a];
    k.walls = p.walls;
    k.C = c->dem_cap;
    return k;
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_dem_forces(fpm_ctx *c, const fpm_dem_params &p) {
    hipLaunchKernelGGL(k_dem_forces, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st,
                       make_coef(c, p), c->dem_rb, c->cap4);
    return hipGetLastError();
}

hipError_t launch_dem_integrate(fpm_ctx *c, const fpm_dem_params &p) {
    hipLaunchKernelGGL(k_dem_integrate, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st,
                       make_coef(c, p));
    return hipGetLastError();
}

hipError_t launch_dem_set_omega(fpm_ctx *c, const float *w) {
    hipLaunchKernelGGL(k_dem_set_omega, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, w);
    hipLaunchKernelGGL(k_dem_clear, dim3(grid_for(c->n * c->dem_cap, 256)), dim3(256), 0,
                       c->stream, c->st, c->n, c->dem_cap);
    return hipGetLastError();
}

hipError_t launch_dem_out(fpm_ctx *c, float *w, float *tq, int32_t *ids, float *ut,
                          int32_t *ncon) {
    if (w || tq)
        hipLaunchKernelGGL(k_dem_out, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, w, tq);
    if (ids || ut || ncon)
        hipLaunchKernelGGL(k_dem_contacts_out, dim3(grid_for(c->n * c->dem_cap, 256)), dim3(256),
                           0, c->stream, c->st, c->dem_rb, c->n, c->dem_cap, ids, ut, ncon);
    return hipGetLastError();
}

}  // namespace fpm
