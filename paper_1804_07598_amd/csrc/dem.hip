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
// Contact history: the u_t of a grain's pairs sits beside its Verlet list,
// one float4 (u_t, in-contact flag) per list entry, in the list's order and
// slot blocking, so the step reads it with the list and each lane updates only
// its own entries.  The lists and slots change only at a rebuild: the gated
// export kernel then copies the history of the pairs in contact to rows keyed
// by caller index (partner caller index, u_t; up to C per grain) before the
// cell sort, and the gated import kernel moves it to the new list positions
// after the build.  A pair keeps its history as long as it stays in contact;
// p and q each keep their own copy (u_t of (q, p) is minus that of (p, q), and
// both update with exactly negated arithmetic).  Angular velocity lives in the
// per-slot buffer the cell sort carries along; torques in the per-slot
// scratch.
#include "geom.h"

namespace fpm {
namespace {

struct DemCoef {
    double R, m, inv_m, inv_I, kn, kt, gn, gt, mu, dt, meff, inv_2R, d2max, inv_kt;
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

struct DemAcc {
    double f[3], t[3];
};

// One contact at separation r (|r|^2 = rr2 < 4R^2) of a grain with velocity vi
// and angular velocity wi and a partner with vj, wj; u holds the pair's
// tangential history on entry and its update on exit.  Both grains of a pair
// evaluate it with negated r, velocities and history, so their histories stay
// exact negatives and their torques equal.
__device__ __forceinline__ void contact(DemAcc &a, const DemCoef &k, const double r[3],
                                        double rr2, const float4 vi, const float4 wi,
                                        const float4 vj, const float4 wj, double u[3]) {
    const double rr = sqrt(rr2);
    const double inv = 1.0 / rr;
    const double nv[3] = {r[0] * inv, r[1] * inv, r[2] * inv};
    const double arm = 0.5 * rr;
    const double delta = 2.0 * k.R - rr;
    const double ws[3] = {(double)wi.x + (double)wj.x, (double)wi.y + (double)wj.y,
                          (double)wi.z + (double)wj.z};
    double rot[3];
    cross3(ws, nv, rot);
    const double vr[3] = {(double)vi.x - (double)vj.x - arm * rot[0],
                          (double)vi.y - (double)vj.y - arm * rot[1],
                          (double)vi.z - (double)vj.z - arm * rot[2]};
    const double vn = dot3(vr, nv);
    const double vt[3] = {vr[0] - vn * nv[0], vr[1] - vn * nv[1], vr[2] - vn * nv[2]};
    for (int c = 0; c < 3; c++) u[c] += vt[c] * k.dt;
    const double un = dot3(u, nv);
    for (int c = 0; c < 3; c++) u[c] -= un * nv[c];
    const double s = sqrt(delta * k.inv_2R);
    const double fnm = s * (k.kn * delta - k.gn * k.meff * vn);  // F_n = fnm n
    double ft[3];
    for (int c = 0; c < 3; c++) ft[c] = s * (-k.kt * u[c] - k.gt * k.meff * vt[c]);
    const double ft2 = dot3(ft, ft);
    const double cap = k.mu * fabs(fnm);
    if (ft2 > cap * cap) {  // Coulomb: |F_t| <= mu |F_n|
        const double sc = cap / sqrt(ft2);
        for (int c = 0; c < 3; c++) ft[c] *= sc;
        if (k.kt > 0.0) {
            const double is = 1.0 / s;
            for (int c = 0; c < 3; c++) u[c] = -(ft[c] * is + k.gt * k.meff * vt[c]) * k.inv_kt;
        }
    }
    const double am[3] = {-arm * nv[0], -arm * nv[1], -arm * nv[2]};
    double tq[3];
    cross3(am, ft, tq);
    for (int c = 0; c < 3; c++) {
        a.f[c] += fnm * nv[c] + ft[c];
        a.t[c] += tq[c];
    }
}

// History of list entry e of slot i: entry-major within each 64-slot block,
// so one entry of a wavefront's 64 slots is one 1 KiB load.
__device__ __forceinline__ int64_t hist_base(int64_t i, int cap4) {
    return (i >> 6) * (int64_t)cap4 * 4 * 64 + (i & 63);
}


// Before a rebuild: the pairs in contact with their u_t, from list positions
// to rows keyed by caller index, in list order.  CR > 0: the row capacity is
// CR (a multiple of four, at most 16) and the row of partner ids is assembled
// in registers and stored 16 bytes at a time.
template <int CR>
__device__ __forceinline__ void export_slot(const State &st, const SysDesc &d, int64_t i, int cap4,
                                            int C, int64_t ns) {
    constexpr int NR = CR > 0 ? CR : 1;
    if (i - d.slot_base >= d.n) return;
    const int32_t *__restrict__ id = st.id[0];
    const int64_t me = id[i];
    int cnt = (int)(st.nnb[i] & ~kWrapBit);
    if (cnt > 4 * cap4) cnt = 4 * cap4;
    const float4 *hrow = st.hl + hist_base(i, cap4);
    int32_t *hid = st.hid + me * C;
    float4 *hu = st.hu + me * C;
    int row[NR];
#pragma unroll
    for (int c = 0; c < NR; c++) row[c] = -1;
    int nc = 0;
    for (int e = 0; e < cnt; e++) {
        const float4 h = hrow[e * 64];
        if (h.w == 0.f) continue;
        const int j = st.nbr[nbr_index(i, e, cap4)];
        if ((uint64_t)j >= (uint64_t)ns) continue;
        if (nc < C) {
            const int pid = id[j];
            if (CR > 0) {
#pragma unroll
                for (int c = 0; c < NR; c++) row[c] = c == nc ? pid : row[c];
            } else {
                hid[nc] = pid;
            }
            hu[nc] = h;
        }
        nc++;
    }
    if (CR > 0) {
        int4 *h4 = reinterpret_cast<int4 *>(hid);
#pragma unroll
        for (int g = 0; g < NR / 4; g++)
            h4[g] = make_int4(row[4 * g], row[4 * g + 1], row[4 * g + 2], row[4 * g + 3]);
    } else {
        for (int c = nc; c < C; c++) hid[c] = -1;
    }
    if (nc > C) st.ctl->overflow = nc;
}

// The export fused with the first kernel of the cell build (gated on the
// flag): the export reads the old lists, ids and history, the cell
// assignment the positions, so neither sees the other's writes.
template <int CR>
__global__ __launch_bounds__(kBlock) void k_dem_export_assign(State st, int cap4, int C,
                                                              int64_t ns) {
    const int s = block_system(st);
    if (!rebuilding(st, s)) return;
    const int64_t i = global_slot();
    export_slot<CR>(st, st.sys[s], i, cap4, C, ns);
    cell_assign_slot(st, s, i);
}

// After a rebuild: each entry of the new lists takes the u_t its partner had
// in the exported row, or none.  Run by the gated import kernel after an eager
// rebuild, and inside a captured step by the force kernel that follows the
// rebuild.  CR > 0: the row capacity is CR (a multiple of four, at most 16)
// and its partner ids are loaded into registers at once; CR = 0: any
// capacity, searched in memory.
template <int CR>
__device__ __forceinline__ void import_slot(const State &st, int64_t i, int cap4, int C) {
    constexpr int NR = CR > 0 ? CR : 1;
    const int32_t *__restrict__ id = st.id[0];
    const int64_t me = id[i];
    const int cnt = (int)(st.nnb[i] & ~kWrapBit);
    const int32_t *hid = st.hid + me * C;
    const float4 *hu = st.hu + me * C;
    int hrow[NR];
    int stored = 0;
    if (CR > 0) {
        const int4 *h4 = reinterpret_cast<const int4 *>(hid);
#pragma unroll
        for (int g = 0; g < NR / 4; g++) {
            const int4 t = h4[g];
            hrow[4 * g] = t.x, hrow[4 * g + 1] = t.y, hrow[4 * g + 2] = t.z, hrow[4 * g + 3] = t.w;
        }
#pragma unroll
        for (int c = 0; c < NR; c++) stored += hrow[c] >= 0;  // rows are filled from the front
    } else {
        while (stored < C && hid[stored] >= 0) stored++;
    }
    float4 *hrow_l = st.hl + hist_base(i, cap4);
    for (int e = 0; e < cnt; e++) {
        float4 h = make_float4(0.f, 0.f, 0.f, 0.f);
        const int pid = stored > 0 ? id[st.nbr[nbr_index(i, e, cap4)]] : -1;
        if (pid >= 0) {  // padding entries name a slot whose id is -1, like an empty row entry
            int m = -1;
            if (CR > 0) {
#pragma unroll
                for (int c = 0; c < NR; c++) m = hrow[c] == pid ? c : m;
            } else {
                for (int c = 0; c < stored; c++)
                    if (hid[c] == pid) {
                        m = c;
                        break;
                    }
            }
            if (m >= 0) {
                h = hu[m];
                h.w = 1.f;
            }
        }
        hrow_l[e * 64] = h;
    }
}

template <int CR>
__global__ __launch_bounds__(kBlock) void k_dem_import(State st, int cap4, int C) {
    const int s = block_system(st);
    if (!rebuilding(st, s)) return;
    const SysDesc &d = st.sys[s];
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
    import_slot<CR>(st, i, cap4, C);
}

// Forces and torques of the grains, advancing the history in place.  The list
// is walked four entries at a time: their list indices and history entries
// with one request, then the four partners' position, velocity and angular
// velocity with the next.  With imp set, a grain whose system has just been
// rebuilt (flag still set) first imports its history into the new list; the
// same thread then reads it back.
template <int CR>
__global__ __launch_bounds__(kBlock) void k_dem_forces(State st, DemCoef k, int cap4, int imp) {
    const int sy = block_system(st);
    const SysDesc &d = st.sys[sy];
    const Box b = d.box;
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
    if (imp && rebuilding(st, sy)) import_slot<CR>(st, i, cap4, k.C);  // lists just rebuilt
    const float4 *__restrict__ pos = st.pos[0];
    const float4 *__restrict__ vel = st.vel[0];
    const float4 *__restrict__ om = st.old[0];
    const float4 pi4 = pos[i], vi = vel[i], wi = om[i];
    const float3 pi = xyz(pi4);
    DemAcc a;
    for (int c = 0; c < 3; c++) a.f[c] = k.m * k.g[c], a.t[c] = 0.0;
    int nc = 0;
    const int cnt = (int)(st.nnb[i] & ~kWrapBit);
    const int4 *lst = reinterpret_cast<const int4 *>(st.nbr) + ((i >> 6) * (int64_t)cap4) * 64 +
                      (i & 63);
    float4 *hrow = st.hl + hist_base(i, cap4);
    int4 e = cnt > 0 ? lst[0] : make_int4(0, 0, 0, 0);
    for (int k0 = 0; k0 < cnt; k0 += 4) {  // lists are padded to a multiple of eight
        const int j[4] = {e.x, e.y, e.z, e.w};
        e = lst[((k0 + 4 < cnt ? k0 + 4 : k0) >> 2) * 64];  // the next group, ahead of time
        float4 h[4];
#pragma unroll
        for (int u = 0; u < 4; u++) h[u] = hrow[(k0 + u) * 64];
        float4 q[4], vj[4], wj[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            q[u] = pos[j[u]];
            vj[u] = vel[j[u]];
            wj[u] = om[j[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const bool live = k0 + u < cnt;
            const double r[3] = {sep_axis(pi.x, q[u].x, b.L[0], b.half[0], b.per[0]),
                                 sep_axis(pi.y, q[u].y, b.L[1], b.half[1], b.per[1]),
                                 sep_axis(pi.z, q[u].z, b.L[2], b.half[2], b.per[2])};
            const double rr2 = dot3(r, r);
            if (live && rr2 < k.d2max) {
                const bool had = h[u].w != 0.f;
                double uu[3] = {had ? (double)h[u].x : 0.0, had ? (double)h[u].y : 0.0,
                                had ? (double)h[u].z : 0.0};
                contact(a, k, r, rr2, vi, wi, vj[u], wj[u], uu);
                hrow[(k0 + u) * 64] = make_float4((float)uu[0], (float)uu[1], (float)uu[2], 1.f);
                nc++;
            } else if (live && h[u].w != 0.f) {
                hrow[(k0 + u) * 64] = make_float4(0.f, 0.f, 0.f, 0.f);  // contact lost
            }
        }
    }
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
        const double vv[3] = {vi.x, vi.y, vi.z};
        const double vn = dot3(vv, nw);
        for (int c = 0; c < 3; c++) a.f[c] += s * (k.kn * delta * nw[c] - k.gn * k.m * vn * nw[c]);
    }
    st.frc[i] = make_float4((float)a.f[0], (float)a.f[1], (float)a.f[2], 0.f);
    st.aux[i] = make_float4((float)a.t[0], (float)a.t[1], (float)a.t[2], 0.f);
    st.ncon[st.id[0][i]] = nc;
    if (nc > k.C) st.ctl->overflow = nc;
    if (!isfinite(a.f[0]) || !isfinite(a.f[1]) || !isfinite(a.f[2])) st.ctl->nonfinite = 1;
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

__global__ void k_dem_clear(State st, int64_t n, int C, int64_t nh) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * C) st.hid[t] = -1;
    if (t < n) st.ncon[t] = 0;
    if (t < nh) st.hl[t] = make_float4(0.f, 0.f, 0.f, 0.f);
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

// The pairs in contact at the last evaluation, per grain in caller order (in
// list order, up to C), with their u_t; the rest of each row -1 and zero.
__global__ void k_dem_contacts_out(State st, int cap4, int C, int32_t *ids, float *ut) {
    const SysDesc &d = st.sys[block_system(st)];
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
    const int32_t *__restrict__ id = st.id[0];
    const int64_t me = id[i];
    const int cnt = (int)(st.nnb[i] & ~kWrapBit);
    const float4 *hrow = st.hl + hist_base(i, cap4);
    int nc = 0;
    for (int e = 0; e < cnt && nc < C; e++) {
        const float4 h = hrow[e * 64];
        if (h.w == 0.f) continue;
        const int64_t o = me * C + nc;
        if (ids) ids[o] = id[st.nbr[nbr_index(i, e, cap4)]];
        if (ut) ut[3 * o] = h.x, ut[3 * o + 1] = h.y, ut[3 * o + 2] = h.z;
        nc++;
    }
    for (int c = nc; c < C; c++) {
        const int64_t o = me * C + c;
        if (ids) ids[o] = -1;
        if (ut) ut[3 * o] = 0.f, ut[3 * o + 1] = 0.f, ut[3 * o + 2] = 0.f;
    }
}

__global__ void k_ncon_out(State st, int64_t n, int32_t *ncon) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) ncon[t] = st.ncon[t];
}

DemCoef make_coef(const fpm_ctx *c, const fpm_dem_params &p) {
    DemCoef k;
    k.R = p.R;
    k.m = p.mass;
    k.inv_m = 1.0 / (double)p.mass;
    k.inv_I = 1.0 / (double)p.inertia;
    k.kn = p.kn;
    k.kt = p.kt;
    k.inv_kt = p.kt > 0.f ? 1.0 / (double)p.kt : 0.0;
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

hipError_t launch_dem_forces(fpm_ctx *c, const fpm_dem_params &p, bool imp) {
    const dim3 g(c->nblk), blk(kBlock);
    const DemCoef k = make_coef(c, p);
    const int m = imp ? 1 : 0;
    switch (c->dem_cap) {
    case 4: hipLaunchKernelGGL(k_dem_forces<4>, g, blk, 0, c->stream, c->st, k, c->cap4, m); break;
    case 8: hipLaunchKernelGGL(k_dem_forces<8>, g, blk, 0, c->stream, c->st, k, c->cap4, m); break;
    case 12: hipLaunchKernelGGL(k_dem_forces<12>, g, blk, 0, c->stream, c->st, k, c->cap4, m); break;
    case 16: hipLaunchKernelGGL(k_dem_forces<16>, g, blk, 0, c->stream, c->st, k, c->cap4, m); break;
    default: hipLaunchKernelGGL(k_dem_forces<0>, g, blk, 0, c->stream, c->st, k, c->cap4, m);
    }
    return hipGetLastError();
}

hipError_t launch_dem_integrate(fpm_ctx *c, const fpm_dem_params &p) {
    hipLaunchKernelGGL(k_dem_integrate, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st,
                       make_coef(c, p));
    return hipGetLastError();
}

hipError_t launch_dem_export_assign(fpm_ctx *c) {
    const dim3 g(c->nblk), blk(kBlock);
    const int64_t ns = (int64_t)c->nblk * kBlock;
    switch (c->dem_cap) {
    case 4:
        hipLaunchKernelGGL(k_dem_export_assign<4>, g, blk, 0, c->stream, c->st, c->cap4, 4, ns);
        break;
    case 8:
        hipLaunchKernelGGL(k_dem_export_assign<8>, g, blk, 0, c->stream, c->st, c->cap4, 8, ns);
        break;
    case 12:
        hipLaunchKernelGGL(k_dem_export_assign<12>, g, blk, 0, c->stream, c->st, c->cap4, 12, ns);
        break;
    case 16:
        hipLaunchKernelGGL(k_dem_export_assign<16>, g, blk, 0, c->stream, c->st, c->cap4, 16, ns);
        break;
    default:
        hipLaunchKernelGGL(k_dem_export_assign<0>, g, blk, 0, c->stream, c->st, c->cap4,
                           c->dem_cap, ns);
    }
    return hipGetLastError();
}

hipError_t launch_dem_import(fpm_ctx *c) {
    const dim3 g(c->nblk), blk(kBlock);
    switch (c->dem_cap) {
    case 4: hipLaunchKernelGGL(k_dem_import<4>, g, blk, 0, c->stream, c->st, c->cap4, 4); break;
    case 8: hipLaunchKernelGGL(k_dem_import<8>, g, blk, 0, c->stream, c->st, c->cap4, 8); break;
    case 12: hipLaunchKernelGGL(k_dem_import<12>, g, blk, 0, c->stream, c->st, c->cap4, 12); break;
    case 16: hipLaunchKernelGGL(k_dem_import<16>, g, blk, 0, c->stream, c->st, c->cap4, 16); break;
    default:
        hipLaunchKernelGGL(k_dem_import<0>, g, blk, 0, c->stream, c->st, c->cap4, c->dem_cap);
    }
    return hipGetLastError();
}

hipError_t launch_dem_set_omega(fpm_ctx *c, const float *w) {
    hipLaunchKernelGGL(k_dem_set_omega, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, w);
    return launch_dem_clear(c);
}

hipError_t launch_dem_clear(fpm_ctx *c) {
    const int64_t nh = (int64_t)c->nblk * kBlock * c->cap4 * 4;
    int64_t m = c->n * c->dem_cap;
    if (nh > m) m = nh;
    hipLaunchKernelGGL(k_dem_clear, dim3(grid_for(m, 256)), dim3(256), 0, c->stream, c->st, c->n,
                       c->dem_cap, nh);
    return hipGetLastError();
}

hipError_t launch_dem_out(fpm_ctx *c, float *w, float *tq, int32_t *ids, float *ut,
                          int32_t *ncon) {
    if (w || tq)
        hipLaunchKernelGGL(k_dem_out, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, w, tq);
    if (ids || ut)
        hipLaunchKernelGGL(k_dem_contacts_out, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st,
                           c->cap4, c->dem_cap, ids, ut);
    if (ncon)
        hipLaunchKernelGGL(k_ncon_out, dim3(grid_for(c->n, 256)), dim3(256), 0, c->stream, c->st,
                           c->n, ncon);
    return hipGetLastError();
}

}  // namespace fpm
