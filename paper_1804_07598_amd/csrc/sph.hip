// Weakly compressible SPH (section 4.2, Eqs. 1-5) over the Verlet list.
//
// Per particle a and each neighbour b within 2h (FP32 predicate, as for LJ):
//   dv_a/dt   = -sum_b m ((P_a + P_b)/(rho_a rho_b) + Pi_ab) gradW_ab + g     (Eq. 1)
//   drho_a/dt =  sum_b m v_ab . gradW_ab                                     (Eq. 2)
//   P = B ((rho/rho0)^gamma - 1), B = c0^2 rho0 / gamma                      (Eqs. 3-4)
//   Pi_ab = -alpha cbar mu_ab / rhobar_ab when v_ab . x_ab < 0, else 0,
//   mu_ab = h v_ab . x_ab / (|x_ab|^2 + eta^2), rhobar_ab = (rho_a + rho_b)/2 (Eq. 5)
// with x_ab = x_a - x_b, v_ab = v_a - v_b, cbar the viscosity's sound speed
// (c0 unless given) and a kernel of support 2h, q = r/h:
//   Wendland C2  W = a_D (1 - q/2)^4 (2q + 1), a_D = 21 / (16 pi h^3),
//                gradW_ab = -(5 a_D / h^2) (1 - q/2)^3 x_ab;
//   cubic spline W = a_D (1 - 3q^2/2 + 3q^3/4) (q < 1), a_D (2 - q)^3 / 4
//                (1 <= q < 2), a_D = 1 / (pi h^3),
//                gradW_ab = (a_D / h^2) (-3 + 9q/4) x_ab (q < 1),
//                           -(3 a_D / (4 h)) (2 - q)^2 / r x_ab (1 <= q < 2).
// Boundary particles (kind 1) take part in every sum and evolve their density
// by Eq. 2, but carry no acceleration.  Pair terms are evaluated in FP64 from
// exact FP32 separations (the pressure terms cancel to within a few percent of
// gravity in a resting column, which FP32 pair terms cannot resolve to 1e-5).
//
// Time stepping is kick-drift-kick on (v, rho), or the Verlet scheme (ref.
// [46] of section 4.2) with periodic Euler-form steps, with the time step
// chosen on the device from the CFL terms of the latest rates:
//   dt = cfl * min(min_a sqrt(h / |a_a|), h / (c0 + max_ab |mu_ab|)).
#include "geom.h"

namespace fpm {
namespace {

struct SphCoef {
    double h, m, rho0, inv_rho0, B, gamma, alpha_c0, eta2, kgrad;  // alpha_c0 = alpha cbar
    double half_inv_h;  // 1 / (2 h)
    double inv_h, cin, cout;  // cubic spline: 1/h, a_D / h^2, 3 a_D / (4 h)
    double rc2lo, rc2hi;
    float g[3];
    int gamma7;
};

// 1/x and sqrt(x) in FP64 from the hardware estimates (about 2^-26 relative)
// refined by one Newton step each (error squared: below 1e-14 relative),
// without the cost of IEEE division and square root.
__device__ __forceinline__ double rcp64(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

__device__ __forceinline__ double sqrt64(double x) {
    const double y = __builtin_amdgcn_rsq(x);  // ~ 1/sqrt(x)
    const double s = x * y;                    // ~ sqrt(x)
    return fma(0.5 * s, fma(-s, y, 1.0), s);   // one Newton step on sqrt
}

// Tait's equation of state.  G7: gamma is 7 (x^7 by multiplications);
// otherwise k.gamma7 decides between that and pow(x, gamma).  The rates
// kernels take G7 as a template argument, so that with gamma = 7 their pair
// loop holds no pow.
template <bool G7 = false>
__device__ __forceinline__ double tait(double rho, const SphCoef &k) {
    const double x = rho * k.inv_rho0;
    double xg;
    if (G7 || k.gamma7) {
        const double x2 = x * x, x4 = x2 * x2;
        xg = x4 * x2 * x;
    } else {
        xg = pow(x, k.gamma);
    }
    return k.B * (xg - 1.0);
}

struct SphAcc {
    double ax = 0.0, ay = 0.0, az = 0.0, dr = 0.0, mu = 0.0;
};

// gradW_ab / x_ab at distance r (KER 0 Wendland C2, 1 cubic spline).
template <int KER>
__device__ __forceinline__ double grad_factor(double r, const SphCoef &k) {
    if (KER == 0) {
        const double t = fma(-r, k.half_inv_h, 1.0);
        return -k.kgrad * t * t * t;  // kgrad = 5 a_D / h^2
    }
    const double q = r * k.inv_h;
    const double t = 2.0 - q;
    const double outer = -k.cout * t * t * rcp64(r);
    const double inner = k.cin * fma(2.25, q, -3.0);
    return q < 1.0 ? inner : outer;
}

template <bool IMG, int KER, bool G7>
__device__ __forceinline__ void sph_pair(SphAcc &s, float3 pi, double xi, double yi, double zi,
                                         float4 vi, double Pa_over, float4 q, float4 w,
                                         const Box &b, float rc2, const SphCoef &k) {
    double dx, dy, dz;
    if (IMG) {
        dx = sep_axis(pi.x, q.x, b.L[0], b.half[0], b.per[0]);
        dy = sep_axis(pi.y, q.y, b.L[1], b.half[1], b.per[1]);
        dz = sep_axis(pi.z, q.z, b.L[2], b.half[2], b.per[2]);
    } else {
        dx = xi - (double)q.x;
        dy = yi - (double)q.y;
        dz = zi - (double)q.z;
    }
    const double r2 = dx * dx + dy * dy + dz * dz;
    bool in = r2 <= k.rc2lo;
    // the band is narrow: the FP32 predicate only when some lane of the wavefront is in it
    if (__builtin_expect(__ballot(!in && r2 <= k.rc2hi) != 0, 0)) {
        if (!in && r2 <= k.rc2hi)
            in = (IMG ? dist2_pred(pi, xyz(q), b) : dist2_direct(pi, xyz(q))) <= rc2;
    }
    if (in) {
        const double gw = grad_factor<KER>(sqrt64(r2), k);  // gradW = gw * x_ab
        const double rho_b = (double)w.w;
        const double vx = (double)vi.x - (double)w.x, vy = (double)vi.y - (double)w.y,
                     vz = (double)vi.z - (double)w.z;
        const double vr = vx * dx + vy * dy + vz * dz;
        // continuity, Eq. 2
        s.dr += k.m * gw * vr;
        // momentum, Eq. 1 (pressure part uses (P_a + P_b) / (rho_a rho_b))
        const double Pb = tait<G7>(rho_b, k);
        const double rho_a = (double)vi.w;
        double term = (Pa_over + Pb) * rcp64(rho_a * rho_b);
        const double mu = k.h * vr * rcp64(r2 + k.eta2);
        if (vr < 0.0) term += -2.0 * k.alpha_c0 * mu * rcp64(rho_a + rho_b);
        s.mu = fmax(s.mu, fabs(mu));
        const double f = -k.m * term * gw;
        s.ax += f * dx;
        s.ay += f * dy;
        s.az += f * dz;
    }
}

// Positions and velocities of the four neighbours of one list group.
__device__ __forceinline__ void sph_gather(const char *pb, const char *vb, int4 e, float4 (&q)[4],
                                           float4 (&w)[4]) {
    const uint32_t jj[4] = {(uint32_t)e.x << 4, (uint32_t)e.y << 4, (uint32_t)e.z << 4,
                            (uint32_t)e.w << 4};
#pragma unroll
    for (int u = 0; u < 4; u++) {
        q[u] = *reinterpret_cast<const float4 *>(pb + jj[u]);
        w[u] = *reinterpret_cast<const float4 *>(vb + jj[u]);
    }
}

// Walks a list padded to a multiple of eight entries four at a time,
// software-pipelined: the neighbours of the next group are requested before
// the current group's pairs are evaluated (two register sets take turns; a
// group past the end of the list re-reads one in range, which is harmless).
template <bool IMG, int KER, bool G7>
__device__ __forceinline__ void sph_walk(SphAcc &s, const float4 *__restrict__ pos,
                                         const float4 *__restrict__ vel,
                                         const int4 *__restrict__ lst, int cnt, int self,
                                         float4 pi4, float4 vi, double Pa, const Box &b,
                                         float rc2, const SphCoef &k) {
    const float3 pi = xyz(pi4);
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    const char *pb = reinterpret_cast<const char *>(pos);
    const char *vb = reinterpret_cast<const char *>(vel);
    (void)self;
    if (cnt <= 0) return;
    float4 q0[4], w0[4], q1[4], w1[4];
    sph_gather(pb, vb, lst[0], q0, w0);
    int4 nxt = lst[(4 < cnt ? 4 : 0) >> 2 << 6];
    for (int kk = 0; kk < cnt; kk += 8) {
        sph_gather(pb, vb, nxt, q1, w1);
        nxt = lst[((kk + 8 < cnt ? kk + 8 : kk) >> 2) * 64];
#pragma unroll
        for (int u = 0; u < 4; u++)
            sph_pair<IMG, KER, G7>(s, pi, xi, yi, zi, vi, Pa, q0[u], w0[u], b, rc2, k);
        if (kk + 4 >= cnt) break;
        sph_gather(pb, vb, nxt, q0, w0);
        nxt = lst[((kk + 12 < cnt ? kk + 12 : kk) >> 2) * 64];
#pragma unroll
        for (int u = 0; u < 4; u++)
            sph_pair<IMG, KER, G7>(s, pi, xi, yi, zi, vi, Pa, q1[u], w1[u], b, rc2, k);
    }
}

template <int KER, bool G7>
__global__ __launch_bounds__(kBlock) void k_sph_rates(State st, float rc2, SphCoef k,
                                                      int cap4) {
    const int sys = block_system(st);
    const SysDesc &d = st.sys[sys];
    if (threadIdx.x == 0 && pblock() == d.blk_base) {
        // a rebuild that preceded this launch is complete: account it and
        // clear its flag (nothing in this launch reads the flag)
        SysCtl *sc = st.sctl + sys;
        if (sc->rebuild[0]) {
            sc->n_rebuilds += 1;
            sc->rebuild[0] = 0;
        }
    }
    const Box b = d.box;
    const float4 *__restrict__ pos = st.pos[0];
    const float4 *__restrict__ vel = st.vel[0];
    const int64_t i = global_slot();
    const bool active = i - d.slot_base < d.n;
    uint32_t nn = 0;
    float4 pi4 = make_float4(0.f, 0.f, 0.f, 0.f), vi = make_float4(0.f, 0.f, 0.f, 1.f);
    if (active) {
        nn = st.nnb[i];
        pi4 = pos[i];
        vi = vel[i];
    }
    const bool img_wave = __ballot((nn & kWrapBit) != 0) != 0;
    const int cnt = (int)(nn & ~kWrapBit);
    const int4 *lst = reinterpret_cast<const int4 *>(st.nbr) +
                      ((i >> 6) * (int64_t)cap4) * 64 + (i & 63);
    const double Pa = tait<G7>((double)vi.w, k);
    SphAcc s;
    if (img_wave)
        sph_walk<true, KER, G7>(s, pos, vel, lst, cnt, (int)i, pi4, vi, Pa, b, rc2, k);
    else
        sph_walk<false, KER, G7>(s, pos, vel, lst, cnt, (int)i, pi4, vi, Pa, b, rc2, k);
    const bool fluid = __float_as_int(pi4.w) == 0;
    double accmin = 1e300;
    if (active) {
        float4 out;
        if (fluid) {
            out = make_float4((float)(s.ax + k.g[0]), (float)(s.ay + k.g[1]),
                              (float)(s.az + k.g[2]), (float)s.dr);
            const double ax = s.ax + k.g[0], ay = s.ay + k.g[1], az = s.az + k.g[2];
            const double am = sqrt(ax * ax + ay * ay + az * az);
            accmin = am > 0.0 ? k.h / am : 1e300;
        } else {
            out = make_float4(0.f, 0.f, 0.f, (float)s.dr);
        }
        st.frc[i] = out;
        if (!isfinite(out.x) || !isfinite(out.y) || !isfinite(out.z) || !isfinite(out.w))
            st.ctl->nonfinite = 1;
    }
    double v[2] = {s.mu, accmin};
    const int slot[2] = {kSlotMu, kSlotAcc};
    const int op[2] = {1, 2};
    block_partials<2>(v, slot, op, st.part, st.pstride);
}

// Kick-drift-kick on (v, rho): the closing half kick of the previous step and
// the opening half kick of this one are fused; boundary particles keep x and v.
// Both step kernels raise the system's rebuild flag from a wavefront with a
// particle moved by more than half the skin since the last build (one lane,
// as the LJ step kernel does; thr: (skin/2)^2); the rates kernel that follows
// the gated rebuild accounts it and clears the flag.
__device__ __forceinline__ void raise_rebuild(const State &st, int sys, bool over) {
    const uint64_t m = __ballot(over);
    if (m && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1) st.sctl[sys].rebuild[0] = 1;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_sph_integrate(State st, float thr) {
    const int sys = block_system(st);
    const SysDesc &d = st.sys[sys];
    const Box b = d.box;
    const int64_t i = global_slot();
    const Ctl *ctl = st.ctl;
    const float dt = ctl->sph_dt, dtl = ctl->sph_dt_last;
    const float hk = MODE == kKickDriftFirst ? 0.5f * dt
                                             : (MODE == kKickOnly ? 0.5f * dtl : 0.5f * (dtl + dt));
    double ke = 0.0, vmax = 0.0;
    bool over = false;
    if (i - d.slot_base < d.n) {
        float4 v = st.vel[0][i];
        const float4 f = st.frc[i];
        float4 p = st.pos[0][i];
        const bool fluid = __float_as_int(p.w) == 0;
        v.w += hk * f.w;
        if (fluid) {
            v.x += hk * f.x;
            v.y += hk * f.y;
            v.z += hk * f.z;
            if (MODE != kKickOnly) {
                p.x += dt * v.x;
                p.y += dt * v.y;
                p.z += dt * v.z;
                st.pos[0][i] = p;
                if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z)) st.ctl->nonfinite = 1;
            }
        }
        st.vel[0][i] = v;
        const double v2 = (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z;
        ke = 0.5 * v2;  // per unit mass; the finalize multiplies by m
        vmax = sqrt(v2);
        if (MODE != kKickOnly) over = dist2_pred(xyz(st.xbuild[i]), xyz(p), b) > thr;
    }
    raise_rebuild(st, sys, over);
    double v2[2] = {ke, vmax};
    const int slot[2] = {kSlotKE, kSlotVmax};
    const int op[2] = {0, 1};
    block_partials<2>(v2, slot, op, st.part, st.pstride);
}

// One step of the Verlet scheme on (x, v, rho) with rates (a, D) of the
// current state and the step dt of those rates:
//   x' = x + dt v + dt^2/2 a (fluid), v' = v_prev + 2 dt a (fluid),
//   rho' = rho_prev + 2 dt D,
// or on every `every`-th step since the state was set (the first one
// included) the Euler form v' = v + dt a, rho' = rho + dt D.  The state
// before the step becomes the previous one.  Boundary particles keep x, v.
__global__ __launch_bounds__(kBlock) void k_sph_verlet(State st, int every, float thr) {
    const int sys = block_system(st);
    const SysDesc &d = st.sys[sys];
    const Box b = d.box;
    const int64_t i = global_slot();
    const Ctl *ctl = st.ctl;
    const float dt = ctl->sph_dt;
    const bool euler = ctl->sph_nstep % every == 0;
    const float f2 = euler ? dt : 2.0f * dt;
    const float hdt2 = 0.5f * dt * dt;
    double ke = 0.0, vmax = 0.0;
    bool over = false;
    if (i - d.slot_base < d.n) {
        const float4 v = st.vel[0][i];  // (v, rho) now
        const float4 o = st.old[0][i];  // (v, rho) one step before
        const float4 f = st.frc[i];     // (a, D)
        const float4 base = euler ? v : o;
        float4 p = st.pos[0][i];
        float4 nv = v;
        nv.w = base.w + f2 * f.w;
        if (__float_as_int(p.w) == 0) {
            nv.x = base.x + f2 * f.x;
            nv.y = base.y + f2 * f.y;
            nv.z = base.z + f2 * f.z;
            p.x = (p.x + dt * v.x) + hdt2 * f.x;
            p.y = (p.y + dt * v.y) + hdt2 * f.y;
            p.z = (p.z + dt * v.z) + hdt2 * f.z;
            st.pos[0][i] = p;
            if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z)) st.ctl->nonfinite = 1;
        }
        st.old[0][i] = v;
        st.vel[0][i] = nv;
        const double v2 = (double)nv.x * nv.x + (double)nv.y * nv.y + (double)nv.z * nv.z;
        ke = 0.5 * v2;  // per unit mass; the finalize multiplies by m
        vmax = sqrt(v2);
        over = dist2_pred(xyz(st.xbuild[i]), xyz(p), b) > thr;
    }
    raise_rebuild(st, sys, over);
    double v2[2] = {ke, vmax};
    const int slot[2] = {kSlotKE, kSlotVmax};
    const int op[2] = {0, 1};
    block_partials<2>(v2, slot, op, st.part, st.pstride);
}

__global__ void k_sph_restart(Ctl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->sph_nstep = 0;
}

// Reduces the CFL terms of the last rates into the next time step; with
// `advance`, first moves the current step into the history (time, dt, kinetic
// energy and largest speed of the last integrate).
__global__ __launch_bounds__(1024) void k_sph_finalize(State st, int nblk, SphCoef k, float cfl,
                                                       float c0, int advance, float *dt_out,
                                                       double *hist) {
    __shared__ double red[16][4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    double mu = 0.0, acc = 1e300, ke = 0.0, vmax = 0.0;
    const double *P = st.part;
    const int64_t S = st.pstride;
    for (int r = t; r < nblk; r += 1024) {
        mu = fmax(mu, P[kSlotMu * S + r]);
        acc = fmin(acc, P[kSlotAcc * S + r]);
        if (advance) {
            ke += P[kSlotKE * S + r];
            vmax = fmax(vmax, P[kSlotVmax * S + r]);
        }
    }
    mu = wave_max(mu);
    acc = wave_min(acc);
    ke = wave_sum(ke);
    vmax = wave_max(vmax);
    if (lane == 0) {
        red[w][0] = mu;
        red[w][1] = acc;
        red[w][2] = ke;
        red[w][3] = vmax;
    }
    __syncthreads();
    if (t != 0) return;
    for (int q = 1; q < 16; q++) {
        mu = fmax(red[0][0], red[q][0]);
        red[0][0] = mu;
        red[0][1] = fmin(red[0][1], red[q][1]);
        red[0][2] += red[q][2];
        red[0][3] = fmax(red[0][3], red[q][3]);
    }
    mu = red[0][0];
    acc = red[0][1];
    ke = red[0][2];
    vmax = red[0][3];
    Ctl *ctl = st.ctl;
    if (advance) {
        const float dtu = ctl->sph_dt;
        ctl->sph_dt_last = dtu;
        ctl->sph_time += (double)dtu;
        const int row = st.sctl[0].step;
        if (hist) {
            hist[(int64_t)row * 4 + 0] = ctl->sph_time;
            hist[(int64_t)row * 4 + 1] = (double)dtu;
            hist[(int64_t)row * 4 + 2] = ke * k.m;
            hist[(int64_t)row * 4 + 3] = vmax;
        }
        st.sctl[0].step = row + 1;
        ctl->sph_nstep += 1;
    }
    const double dt = (double)cfl * fmin(sqrt(acc), k.h / ((double)c0 + mu));
    ctl->sph_dt = (float)dt;
    if (dt_out) *dt_out = (float)dt;
}

SphCoef make_coef(const fpm_ctx *c, const fpm_sph_params &p) {
    SphCoef k;
    k.h = p.h;
    k.m = p.mass;
    k.rho0 = p.rho0;
    k.inv_rho0 = 1.0 / (double)p.rho0;
    k.gamma = p.gamma;
    k.gamma7 = p.gamma == 7.0f;
    k.B = (double)p.c0 * (double)p.c0 * (double)p.rho0 / (double)p.gamma;
    k.alpha_c0 = (double)p.alpha * (double)(p.cbar > 0.f ? p.cbar : p.c0);
    k.eta2 = p.eta2;
    const double h = p.h;
    const double aD = 21.0 / (16.0 * 3.14159265358979323846 * h * h * h);
    k.kgrad = 5.0 * aD / (h * h);
    k.half_inv_h = 0.5 / h;
    const double aDc = 1.0 / (3.14159265358979323846 * h * h * h);
    k.inv_h = 1.0 / h;
    k.cin = aDc / (h * h);
    k.cout = 0.75 * aDc / h;
    const double band = predicate_band(c);
    k.rc2lo = (double)c->rc2 * (1.0 - band);
    k.rc2hi = (double)c->rc2 * (1.0 + band);
    for (int a = 0; a < 3; a++) k.g[a] = p.g[a];
    return k;
}

}  // namespace

hipError_t launch_sph_rates(fpm_ctx *c, const fpm_sph_params &p) {
    const SphCoef k = make_coef(c, p);
    const dim3 g((unsigned)c->nblk), t(kBlock);
    if (p.kernel == 1 && k.gamma7)
        hipLaunchKernelGGL((k_sph_rates<1, true>), g, t, 0, c->stream, c->st, c->rc2, k, c->cap4);
    else if (p.kernel == 1)
        hipLaunchKernelGGL((k_sph_rates<1, false>), g, t, 0, c->stream, c->st, c->rc2, k, c->cap4);
    else if (k.gamma7)
        hipLaunchKernelGGL((k_sph_rates<0, true>), g, t, 0, c->stream, c->st, c->rc2, k, c->cap4);
    else
        hipLaunchKernelGGL((k_sph_rates<0, false>), g, t, 0, c->stream, c->st, c->rc2, k, c->cap4);
    return hipGetLastError();
}

hipError_t launch_sph_verlet(fpm_ctx *c, const fpm_sph_params &p) {
    hipLaunchKernelGGL(k_sph_verlet, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st,
                       p.verlet_every, c->disp2_thr);
    return hipGetLastError();
}

hipError_t launch_sph_restart(fpm_ctx *c) {
    hipLaunchKernelGGL(k_sph_restart, dim3(1), dim3(64), 0, c->stream, c->st.ctl);
    return hipGetLastError();
}

hipError_t launch_sph_integrate(fpm_ctx *c, const fpm_sph_params &p, int mode) {
    (void)p;
    const dim3 g((unsigned)c->nblk), t(kBlock);
    if (mode == kKickDriftFirst)
        hipLaunchKernelGGL(k_sph_integrate<kKickDriftFirst>, g, t, 0, c->stream, c->st,
                           c->disp2_thr);
    else if (mode == kKickKickDrift)
        hipLaunchKernelGGL(k_sph_integrate<kKickKickDrift>, g, t, 0, c->stream, c->st,
                           c->disp2_thr);
    else
        hipLaunchKernelGGL(k_sph_integrate<kKickOnly>, g, t, 0, c->stream, c->st, c->disp2_thr);
    return hipGetLastError();
}

hipError_t launch_sph_finalize(fpm_ctx *c, const fpm_sph_params &p, int advance, float *dt_out,
                               double *hist) {
    const SphCoef k = make_coef(c, p);
    hipLaunchKernelGGL(k_sph_finalize, dim3(1), dim3(1024), 0, c->stream, c->st, c->nblk, k, p.cfl,
                       p.c0, advance, dt_out, hist);
    return hipGetLastError();
}

}  // namespace fpm
