// Lennard-Jones forces, potential energy and virial over the Verlet list
// (section 4.1: V(r) = 4 eps ((sig/r)^12 - (sig/r)^6); the force on p from q is
// 24 eps (2 sig^12 / rn^7 - sig^6 / rn^4) (xp - xq), rn = |xp - xq|^2, and the
// pair is dropped when rn > r_cut^2), and the vector-Jacobian product of the
// forces for the adjoint.
//
// One lane per cell-sorted particle walks its full list (every pair is seen
// from both sides, so there are no scattered writes).  The list is read UNR
// entries at a time (16-byte loads) and the UNR neighbour positions are
// gathered before any is used, so each lane keeps UNR loads in flight.
//
// Set membership follows the FP32 predicate exactly; the pair physics is
// evaluated in FP64 from the exact separation of the FP32 coordinates and
// accumulated per lane in FP64.  The FP64 squared distance decides membership
// directly unless it lies in a narrow band around r_cut^2 (predicate_band),
// where the FP32 predicate is evaluated.  Partials go to one row per
// workgroup; the finalize kernel sums them per system in a fixed order.
#include "geom.h"

namespace fpm {
namespace {

struct LJCoef {
    double c12[3];  // 4 eps sig^12
    double c6[3];   // 4 eps sig^6
    double a12[3];  // 4 sig^12: c12 at unit eps (the pair force is linear in eps)
    double a6[3];   // 4 sig^6
    double inv_sig[3];
    float side_margin;  // half the skin, widened: see Sided
    float side_wide;    // half box lengths above this take Sided on every lane
};

// 1/x in FP64: the hardware estimate (relative error up to 5e-8) refined by
// one Newton step.  The step matters: without it the FP32 forces differ from
// correctly rounded ones in many last bits, and trajectories then drift away
// from their reference.
__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Image handling of a lane whose particle lies more than half the skin
// (widened) from the box's mid-plane on every periodic axis.  Every particle
// is within half the skin of its build position, which lies in [0, L)
// (larger displacements rebuild the lists first), so a partner of a particle
// in the lower half of an axis can only have t = x_j - x_i > -L/2, and one of
// a particle in the upper half only t < L/2: each lane meets images across
// one face per axis.  The predicate's image test then takes one compare
// (sg t > L/2) and the shifted separation (x_i +- L) - x_j, exact in FP64 like
// the unshifted one, so the results are those of the general form bit for
// bit.  sg is 0 on closed axes.  A lane nearer the mid-plane can meet a
// partner across the other face too, but only at a separation along that axis
// above L/2 - skin/2: where that exceeds r_cut (L/2 > r_cut + skin/2, widened:
// every box of at least two cells per axis) such a pair lies outside the force
// set under either image, so the one-face form holds for every lane.
struct Sided {
    float sg[3];
    double xs[3];  // x_i + sg L
};

__device__ __forceinline__ Sided make_sided(float3 pi, double xi, double yi, double zi,
                                            const Box &b, float margin, float wide, bool &ok) {
    Sided sd;
    const float p[3] = {pi.x, pi.y, pi.z};
    const double x[3] = {xi, yi, zi};
    ok = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const bool lo = p[a] < b.half[a];
        sd.sg[a] = b.per[a] ? (lo ? 1.f : -1.f) : 0.f;
        sd.xs[a] = x[a] + (double)(sd.sg[a] * b.L[a]);
        ok = ok && (!b.per[a] || b.half[a] > wide ||
                    fabsf(p[a] - b.half[a]) > margin + 4e-7f * b.L[a]);
    }
    return sd;
}

// Separation x_i - x_j (exact FP64, image as chosen by the predicate), its
// periodic shift, and membership of the pair in the force set.  IMG 0: no
// lane of the wavefront has image partners; 1: the general form; 2: the
// one-face form of Sided.
template <int IMG>
__device__ __forceinline__ bool separation(float3 pi, double xi, double yi, double zi, float4 q,
                                           const Box &b, float rc2, double rc2lo, double rc2hi,
                                           double &dx, double &dy, double &dz, double &sx,
                                           double &sy, double &sz, const Sided *sd = nullptr) {
    if (IMG == 2) {
        const float tx = q.x - pi.x, ty = q.y - pi.y, tz = q.z - pi.z;
        const double bx = sd->sg[0] * tx > b.half[0] ? sd->xs[0] : xi;
        const double by = sd->sg[1] * ty > b.half[1] ? sd->xs[1] : yi;
        const double bz = sd->sg[2] * tz > b.half[2] ? sd->xs[2] : zi;
        dx = bx - (double)q.x;
        dy = by - (double)q.y;
        dz = bz - (double)q.z;
        sx = bx - xi;
        sy = by - yi;
        sz = bz - zi;
    } else {
        dx = xi - (double)q.x;
        dy = yi - (double)q.y;
        dz = zi - (double)q.z;
        sx = sy = sz = 0.0;
    }
    if (IMG == 1) {
        // the image as chosen by the predicate, with selects rather than branches
        const float tx = q.x - pi.x, ty = q.y - pi.y, tz = q.z - pi.z;
        const double Lx = b.per[0] ? (double)b.L[0] : 0.0, Ly = b.per[1] ? (double)b.L[1] : 0.0,
                     Lz = b.per[2] ? (double)b.L[2] : 0.0;
        sx = tx > b.half[0] ? Lx : (tx < -b.half[0] ? -Lx : 0.0);
        sy = ty > b.half[1] ? Ly : (ty < -b.half[1] ? -Ly : 0.0);
        sz = tz > b.half[2] ? Lz : (tz < -b.half[2] ? -Lz : 0.0);
        dx += sx;
        dy += sy;
        dz += sz;
    }
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    bool in = r2 <= rc2hi;
    const bool band = r2 > rc2lo;  // together with `in`: inside the band
    // the band is narrow: a wavefront rarely has a lane in it, and only then
    // is the FP32 predicate evaluated
    if (__builtin_expect(__ballot(in && band) != 0, 0)) {
        if (in && band)
            in = (IMG ? dist2_pred(pi, xyz(q), b) : dist2_direct(pi, xyz(q))) <= rc2;
    }
    return in;
}

// The coefficients a particle of type ti (0 or 1) can meet: pair type ti + tj
// for a neighbour of type tj, so entry [tj] holds those of pair type ti + tj
// (one type: both entries are pair type 0).  Selected once per lane, so a
// pair needs a two-way select only.
struct LaneCoef {
    double c12[2], c6[2], a12[2], a6[2];
};

template <int NT>
__device__ __forceinline__ LaneCoef lane_coef(const LJCoef &cf, int ti) {
    LaneCoef l;
    for (int t = 0; t < 2; t++) {
        const int k = NT == 2 ? ti + t : 0;
        l.c12[t] = k == 0 ? cf.c12[0] : (k == 1 ? cf.c12[1] : cf.c12[2]);
        l.c6[t] = k == 0 ? cf.c6[0] : (k == 1 ? cf.c6[1] : cf.c6[2]);
        l.a12[t] = k == 0 ? cf.a12[0] : (k == 1 ? cf.a12[1] : cf.a12[2]);
        l.a6[t] = k == 0 ? cf.a6[0] : (k == 1 ? cf.a6[1] : cf.a6[2]);
    }
    return l;
}

// Neighbour type (0 or 1; always 0 with one type).
template <int NT>
__device__ __forceinline__ int nbr_type(float4 q) {
    return NT == 2 ? __float_as_int(q.w) : 0;
}

template <int NT>
__device__ __forceinline__ void coef(const LaneCoef &lc, int tj, double &c12, double &c6) {
    c12 = NT == 2 && tj ? lc.c12[1] : lc.c12[0];
    c6 = NT == 2 && tj ? lc.c6[1] : lc.c6[0];
}

// Per-lane accumulators.  The virial needs no per-pair work: summed over all
// particles, 1/2 sum_ij r_ij (x) f_ij with r_ij = x_i - x_j + s_ij (s_ij the
// periodic shift, f_ji = -f_ij, s_ji = -s_ij) equals
// sum_i x_i (x) F_i + 1/2 sum_ij s_ij (x) f_ij, so each lane adds x_i (x) F_i
// once and only image pairs add a shift term (w*).
struct Acc {
    double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0;
    double wxx = 0.0, wyy = 0.0, wzz = 0.0, wxy = 0.0, wxz = 0.0, wyz = 0.0;
};

template <int NT, int IMG>
__device__ __forceinline__ void pair(Acc &a, float3 pi, double xi, double yi, double zi,
                                     const LaneCoef &cf, float4 q, const Box &b, float rc2,
                                     double rc2lo, double rc2hi, const Sided &sd) {
    double dx, dy, dz, sx, sy, sz;
    if (separation<IMG>(pi, xi, yi, zi, q, b, rc2, rc2lo, rc2hi, dx, dy, dz, sx, sy, sz,
                        &sd)) {
        double c12, c6;
        coef<NT>(cf, nbr_type<NT>(q), c12, c6);
        const double r2i = recip(fma(dx, dx, fma(dy, dy, dz * dz)));
        const double r6i = r2i * r2i * r2i;
        const double s = r6i * r2i * fma(12.0 * c12, r6i, -6.0 * c6);
        a.u = fma(r6i, fma(c12, r6i, -c6), a.u);
        a.fx = fma(s, dx, a.fx);
        a.fy = fma(s, dy, a.fy);
        a.fz = fma(s, dz, a.fz);
        if (IMG) {
            const double hx = 0.5 * s * sx, hy = 0.5 * s * sy, hz = 0.5 * s * sz;
            a.wxx = fma(hx, dx, a.wxx);
            a.wyy = fma(hy, dy, a.wyy);
            a.wzz = fma(hz, dz, a.wzz);
            a.wxy = fma(hx, dy, a.wxy);
            a.wxz = fma(hx, dz, a.wxz);
            a.wyz = fma(hy, dz, a.wyz);
        }
    }
}

// UNR list entries starting at entry k (k a multiple of UNR; groups of four
// entries are one 16-byte load per lane).
template <int UNR>
struct Entries {
    int4 e[UNR / 4];
};

template <int UNR>
__device__ __forceinline__ Entries<UNR> list_group(const int4 *__restrict__ lst, int k) {
    Entries<UNR> r;
#pragma unroll
    for (int g = 0; g < UNR / 4; g++) r.e[g] = lst[((k >> 2) + g) * 64];
    return r;
}

// Neighbour positions of a group of entries.  Slots are below 2^27, so the
// byte offset fits 32 bits and each gather is one shift plus one load with a
// scalar base.
template <int UNR>
__device__ __forceinline__ void gather(const float4 *__restrict__ pos, const Entries<UNR> &en,
                                       float4 (&q)[UNR], const SlotRange &sr) {
    const char *base = reinterpret_cast<const char *>(pos);
#pragma unroll
    for (int g = 0; g < UNR / 4; g++) {
        const int j[4] = {checked(sr, en.e[g].x), checked(sr, en.e[g].y),
                          checked(sr, en.e[g].z), checked(sr, en.e[g].w)};
#pragma unroll
        for (int u = 0; u < 4; u++)
            q[4 * g + u] = *reinterpret_cast<const float4 *>(base + ((uint32_t)j[u] << 4));
    }
}

// Walks a list padded to a multiple of eight entries, UNR (4 or 8) at a time,
// software-pipelined: the neighbour positions of the next group and the list
// entries of the one after are requested before the current group is
// computed, so their latency overlaps the pair arithmetic.
template <int NT, int IMG, int UNR>
__device__ __forceinline__ void walk(Acc &a, const float4 *__restrict__ pos,
                                     const int4 *__restrict__ lst, int cnt, float4 pi4,
                                     const Box &b, float rc2, double rc2lo, double rc2hi,
                                     const LJCoef &cf, const Sided &sd, const SlotRange &sr) {
    if (cnt <= 0) return;
    const float3 pi = xyz(pi4);
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    const LaneCoef lc = lane_coef<NT>(cf, __float_as_int(pi4.w));
    // two register sets take turns (no copies between rounds); a round past
    // the end of the list re-reads a group in range, which is harmless
    float4 q0[UNR], q1[UNR];
    gather<UNR>(pos, list_group<UNR>(lst, 0), q0, sr);
    Entries<UNR> nxt = list_group<UNR>(lst, UNR < cnt ? UNR : 0);
    for (int k = 0; k < cnt; k += 2 * UNR) {
        gather<UNR>(pos, nxt, q1, sr);
        nxt = list_group<UNR>(lst, k + 2 * UNR < cnt ? k + 2 * UNR : k);
#pragma unroll
        for (int u = 0; u < UNR; u++)
            pair<NT, IMG>(a, pi, xi, yi, zi, lc, q0[u], b, rc2, rc2lo, rc2hi, sd);
        if (k + UNR >= cnt) break;
        gather<UNR>(pos, nxt, q0, sr);
        nxt = list_group<UNR>(lst, k + 3 * UNR < cnt ? k + 3 * UNR : k);
#pragma unroll
        for (int u = 0; u < UNR; u++)
            pair<NT, IMG>(a, pi, xi, yi, zi, lc, q1[u], b, rc2, rc2lo, rc2hi, sd);
    }
}

// The velocity-Verlet updates that follow the force evaluation of a step
// (kLjStep, kLjLast): the closing half kick of this step with the new force
// (rounded to FP32, as stored), the kinetic energy of the full-step velocity,
// and for kLjStep the opening half kick and the drift of the next step, whose
// positions go to the other position buffer (neighbour gathers of this launch
// still read the current one), with the test of their displacement since the
// last build against (skin/2)^2.  Every FP32 update rounds after each multiply
// and add, as in the stand-alone integrate kernel, so trajectories do not
// depend on whether the updates are fused.
template <int MODE>
__device__ __forceinline__ double kick_drift(const State &st, const SysDesc &d, int64_t i,
                                             float4 f, float4 p, float4 v, float4 xb, float dt,
                                             float thr, bool &over) {
#pragma clang fp contract(off)
    const float h = 0.5f * dt;
    v.x += h * f.x;
    v.y += h * f.y;
    v.z += h * f.z;
    const double ke = (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z;
    if (MODE == kLjStep) {
        v.x += h * f.x;
        v.y += h * f.y;
        v.z += h * f.z;
        p.x += dt * v.x;
        p.y += dt * v.y;
        p.z += dt * v.z;
        st.pos[1][i] = p;
        over = dist2_pred(xyz(xb), xyz(p), d.box) > thr;
        if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z)) st.ctl->nonfinite = 1;
    } else if (st.par) {
        st.pos[1][i] = p;  // odd step: buffer 1 of this launch is the caller-visible one
    }
    st.vel[0][i] = v;
    return ke;
}

template <int NT, int UNR, int MODE>
__global__ __launch_bounds__(kBlock) void k_lj(State st, float rc2, double rc2lo, double rc2hi,
                                               LJCoef cf, int cap4, StepArgs sa) {
    const int sys = block_system(st);
    const SysDesc &d = st.sys[sys];
    const Box b = d.box;
    const float4 *__restrict__ pos = st.pos[0];
    const int64_t i = global_slot();
    const bool active = i - d.slot_base < d.n;
    uint32_t nn = 0;
    float4 pi4 = make_float4(0.f, 0.f, 0.f, 0.f);
    // the step modes read the velocity and build position at the start, so
    // that their latency hides behind the pair loop
    float4 v4 = pi4, xb4 = pi4;
    if (active) {
        nn = st.nnb[i];
        pi4 = pos[i];
        if (MODE != kLjForce) v4 = st.vel[0][i];
        if (MODE == kLjStep) xb4 = st.xbuild[i];
    }
    const bool img_wave = __ballot((nn & kWrapBit) != 0) != 0;
    const int cnt = (int)(nn & ~kWrapBit);
    const int4 *lst = reinterpret_cast<const int4 *>(st.nbr) +
                      ((i >> 6) * (int64_t)cap4) * 64 + (i & 63);
    Acc a;
    bool side_ok = true;
    const Sided sd = make_sided(xyz(pi4), pi4.x, pi4.y, pi4.z, b, cf.side_margin, cf.side_wide,
                                 side_ok);
    const SlotRange sr = slot_range(st, d);
    // wavefronts with image partners (a minority) keep at most four entries in
    // flight: their walks need more registers per entry, and the kernel's
    // register count, hence every wavefront's occupancy, is set by the largest
    constexpr int UI = UNR < 4 ? UNR : 4;
    if (img_wave && __ballot(active && !side_ok) == 0)
        walk<NT, 2, UI>(a, pos, lst, cnt, pi4, b, rc2, rc2lo, rc2hi, cf, sd, sr);
    else if (img_wave)
        walk<NT, 1, UI>(a, pos, lst, cnt, pi4, b, rc2, rc2lo, rc2hi, cf, sd, sr);
    else
        walk<NT, 0, UNR>(a, pos, lst, cnt, pi4, b, rc2, rc2lo, rc2hi, cf, sd, sr);
    double ke = 0.0;
    bool over = false;
    if (active) {
        const float4 f = make_float4((float)a.fx, (float)a.fy, (float)a.fz, (float)(0.5 * a.u));
        // inside a step loop the stored force is read by nobody (the next
        // step's kernel computes its own, and the last step of a loop stores it)
        if (MODE != kLjStep) st.frc[i] = f;
        if (!isfinite(a.fx) || !isfinite(a.fy) || !isfinite(a.fz)) st.ctl->nonfinite = 1;
        if (MODE != kLjForce)
            ke = kick_drift<MODE>(st, d, i, f, pi4, v4, xb4, sa.dt, sa.thr, over);
    }
    if (MODE != kLjForce) {
        SysCtl *sc = st.sctl + sys;
        if (MODE == kLjStep) {
            // the next step's rebuild flag, raised by one lane of a wavefront that needs it
            const uint64_t m = __ballot(over);
            if (m && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1)
                sc->rebuild[st.par ^ 1] = 1;
        }
        if (threadIdx.x == 0 && pblock() == d.blk_base) {
            // this step's rebuild (if any) is complete: account it and clear its flag
            if (sc->rebuild[st.par]) {
                sc->n_rebuilds += 1;
                sc->rebuild[st.par] = 0;
            }
            sc->step += 1;
        }
    }
    const double xi = pi4.x, yi = pi4.y, zi = pi4.z;
    if (MODE == kLjForce) {
        double v[7] = {0.5 * a.u,
                       fma(xi, a.fx, a.wxx),
                       fma(yi, a.fy, a.wyy),
                       fma(zi, a.fz, a.wzz),
                       fma(xi, a.fy, a.wxy),
                       fma(xi, a.fz, a.wxz),
                       fma(yi, a.fz, a.wyz)};
        const int slot[7] = {kSlotU, kSlotW, kSlotW + 1, kSlotW + 2, kSlotW + 3, kSlotW + 4,
                             kSlotW + 5};
        const int op[7] = {0, 0, 0, 0, 0, 0, 0};
        block_partials<7>(v, slot, op, st.part, st.pstride);
    } else {
        // one row of the step loop's ring: U, W6, KE
        double v[8] = {0.5 * a.u,
                       fma(xi, a.fx, a.wxx),
                       fma(yi, a.fy, a.wyy),
                       fma(zi, a.fz, a.wzz),
                       fma(xi, a.fy, a.wxy),
                       fma(xi, a.fz, a.wxz),
                       fma(yi, a.fz, a.wyz),
                       ke};
        const int slot[8] = {0, 1, 2, 3, 4, 5, 6, 7};
        const int op[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        block_partials<8>(v, slot, op, sa.ring, st.pstride);
    }
}

// ---------------------------------------------------------------------------
// Vector-Jacobian product of the forces.  With F_i = sum_j s(u_ij) r_ij,
// r_ij = x_i - x_j, u = |r|^2 and a cotangent lam (dL/dF):
//   dL/dx_k = sum_j [ s (lam_k - lam_j) + 2 s'(u) r_kj (r_kj . (lam_k - lam_j)) ],
//   dL/dtheta = 1/2 sum_i sum_j (ds/dtheta) r_ij . (lam_i - lam_j)
// (each pair is visited from both sides, hence the 1/2), with
// s = 12 c12 u^-7 - 6 c6 u^-4, s' = -84 c12 u^-8 + 24 c6 u^-5,
// ds/deps = 12 a12 u^-7 - 6 a6 u^-4 (s at unit eps, a12 = 4 sig^12,
// a6 = 4 sig^6; defined at eps = 0 too), ds/dsig = (144 c12 u^-7 - 36 c6 u^-4) / sig.
// The pair set is the force set; the cut-off itself is not differentiated.

// ge, gs: the eps and sig terms by neighbour type (pair type ti + index).
struct VjpAcc {
    double gx = 0.0, gy = 0.0, gz = 0.0;
    double ge[2] = {0.0, 0.0}, gs[2] = {0.0, 0.0};
};

template <int NT, int IMG>
__device__ __forceinline__ void vjp_pair(VjpAcc &a, float3 pi, double xi, double yi, double zi,
                                         const LaneCoef &cf, float4 li, float4 q, float4 lj,
                                         const Box &b, float rc2, double rc2lo, double rc2hi,
                                         const Sided &sd) {
    double dx, dy, dz, sx, sy, sz;
    if (separation<IMG>(pi, xi, yi, zi, q, b, rc2, rc2lo, rc2hi, dx, dy, dz, sx, sy, sz,
                        &sd)) {
        const int tj = nbr_type<NT>(q);
        double c12, c6;
        coef<NT>(cf, tj, c12, c6);
        const double r2i = recip(fma(dx, dx, fma(dy, dy, dz * dz)));
        const double r6i = r2i * r2i * r2i;
        const double s = r6i * r2i * fma(12.0 * c12, r6i, -6.0 * c6);
        const double sp = r6i * r2i * r2i * fma(-84.0 * c12, r6i, 24.0 * c6);
        const double lx = (double)li.x - (double)lj.x, ly = (double)li.y - (double)lj.y,
                     lz = (double)li.z - (double)lj.z;
        const double rl = fma(dx, lx, fma(dy, ly, dz * lz));
        const double t = 2.0 * sp * rl;
        a.gx = fma(s, lx, fma(t, dx, a.gx));
        a.gy = fma(s, ly, fma(t, dy, a.gy));
        a.gz = fma(s, lz, fma(t, dz, a.gz));
        const double a12 = NT == 2 && tj ? cf.a12[1] : cf.a12[0];
        const double a6 = NT == 2 && tj ? cf.a6[1] : cf.a6[0];
        const double de = 0.5 * r6i * r2i * fma(12.0 * a12, r6i, -6.0 * a6) * rl;
        const double ds = 0.5 * r6i * r2i * fma(144.0 * c12, r6i, -36.0 * c6) * rl;  // / sig
        if (NT == 1) {
            a.ge[0] += de;
            a.gs[0] += ds;
        } else {
            a.ge[0] += tj ? 0.0 : de;
            a.ge[1] += tj ? de : 0.0;
            a.gs[0] += tj ? 0.0 : ds;
            a.gs[1] += tj ? ds : 0.0;
        }
    }
}

// Positions and cotangents of the four neighbours of one list group.
__device__ __forceinline__ void vjp_gather(const float4 *__restrict__ pos,
                                           const float4 *__restrict__ lam, int4 e, float4 (&q)[4],
                                           float4 (&l)[4], const SlotRange &sr) {
    const int jj[4] = {checked(sr, e.x), checked(sr, e.y), checked(sr, e.z), checked(sr, e.w)};
#pragma unroll
    for (int u = 0; u < 4; u++) {
        q[u] = pos[jj[u]];
        l[u] = lam[jj[u]];
    }
}

// Walks a list padded to a multiple of eight entries four at a time,
// software-pipelined as the force walk: the next group's gathers are issued
// before the current group's pairs (two register sets take turns; a group
// past the end of the list re-reads one in range, which is harmless).  The
// pairs are taken in list order, as without the pipeline.
template <int NT, int IMG>
__device__ __forceinline__ void vjp_walk(VjpAcc &a, const float4 *__restrict__ pos,
                                         const float4 *__restrict__ lam,
                                         const int4 *__restrict__ lst, int cnt, float4 pi4,
                                         float4 li, const Box &b, float rc2, double rc2lo,
                                         double rc2hi, const LJCoef &cf, const Sided &sd,
                                         const SlotRange &sr) {
    const float3 pi = xyz(pi4);
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    const LaneCoef lc = lane_coef<NT>(cf, __float_as_int(pi4.w));
    if (cnt <= 0) return;
    float4 q0[4], l0[4], q1[4], l1[4];
    vjp_gather(pos, lam, lst[0], q0, l0, sr);
    int4 nxt = lst[(4 < cnt ? 4 : 0) >> 2 << 6];
    for (int k = 0; k < cnt; k += 8) {
        vjp_gather(pos, lam, nxt, q1, l1, sr);
        nxt = lst[((k + 8 < cnt ? k + 8 : k) >> 2) * 64];
#pragma unroll
        for (int u = 0; u < 4; u++)
            vjp_pair<NT, IMG>(a, pi, xi, yi, zi, lc, li, q0[u], l0[u], b, rc2, rc2lo, rc2hi, sd);
        if (k + 4 >= cnt) break;
        vjp_gather(pos, lam, nxt, q0, l0, sr);
        nxt = lst[((k + 12 < cnt ? k + 12 : k) >> 2) * 64];
#pragma unroll
        for (int u = 0; u < 4; u++)
            vjp_pair<NT, IMG>(a, pi, xi, yi, zi, lc, li, q1[u], l1[u], b, rc2, rc2lo, rc2hi, sd);
    }
}

// Cotangent in cell-sorted order (padding slots get zero): lam + h * vbar
// (vbar may be null).
__global__ void k_gather_lam(State st, const double *lam, const double *vbar, double h) {
    const SysDesc &d = st.sys[block_system(st)];
    const int64_t i = global_slot();
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i - d.slot_base < d.n) {
        const int64_t r = st.id[0][i];
        double l[3] = {lam[3 * r], lam[3 * r + 1], lam[3 * r + 2]};
        if (vbar)
            for (int a = 0; a < 3; a++) l[a] = fma(h, vbar[3 * r + a], l[a]);
        v = make_float4((float)l[0], (float)l[1], (float)l[2], 0.f);
    }
    st.aux[i] = v;
}

template <int NT>
__global__ __launch_bounds__(kBlock) void k_lj_vjp(State st, float rc2, double rc2lo,
                                                   double rc2hi, LJCoef cf, int cap4,
                                                   AdjOut o) {
    const int sys = block_system(st);
    const SysDesc &d = st.sys[sys];
    const Box b = d.box;
    const float4 *__restrict__ pos = st.pos[0];
    const int64_t i = global_slot();
    const bool active = i - d.slot_base < d.n;
    if (threadIdx.x == 0 && pblock() == d.blk_base) {
        // a rebuild that preceded this launch is complete: account it and
        // clear its flag (nothing in this launch reads the flag)
        SysCtl *sc = st.sctl + sys;
        if (sc->rebuild[0]) {
            sc->n_rebuilds += 1;
            sc->rebuild[0] = 0;
        }
    }
    uint32_t nn = 0;
    float4 pi4 = make_float4(0.f, 0.f, 0.f, 0.f), li = pi4;
    if (active) {
        nn = st.nnb[i];
        pi4 = pos[i];
        li = st.aux[i];
    }
    const bool img_wave = __ballot((nn & kWrapBit) != 0) != 0;
    const int cnt = (int)(nn & ~kWrapBit);
    const int4 *lst = reinterpret_cast<const int4 *>(st.nbr) +
                      ((i >> 6) * (int64_t)cap4) * 64 + (i & 63);
    VjpAcc a;
    bool side_ok = true;
    const Sided sd = make_sided(xyz(pi4), pi4.x, pi4.y, pi4.z, b, cf.side_margin, cf.side_wide,
                                 side_ok);
    const SlotRange sr = slot_range(st, d);
    if (img_wave && __ballot(active && !side_ok) == 0)
        vjp_walk<NT, 2>(a, pos, st.aux, lst, cnt, pi4, li, b, rc2, rc2lo, rc2hi, cf, sd, sr);
    else if (img_wave)
        vjp_walk<NT, 1>(a, pos, st.aux, lst, cnt, pi4, li, b, rc2, rc2lo, rc2hi, cf, sd, sr);
    else
        vjp_walk<NT, 0>(a, pos, st.aux, lst, cnt, pi4, li, b, rc2, rc2lo, rc2hi, cf, sd, sr);
    if (active) {
        const int64_t r = st.id[0][i];
        const double g[3] = {a.gx, a.gy, a.gz};
        for (int c = 0; c < 3; c++) {
            const int64_t q = 3 * r + c;
            if (o.mode == kVjpPlain) {
                o.gx[q] = g[c];
            } else if (o.mode == kVjpLast) {
                o.gx[q] += g[c];
            } else {
                // one reverse velocity-Verlet step (see fpm_lj_adjoint_step)
                const double xb = o.gx[q] + g[c];
                const double vb = fma(o.dt, xb, o.vbar[q]);
                o.gx[q] = xb;
                o.vbar[q] = vb;
                o.fbar[q] = fma(0.5 * o.dt, vb, o.floss ? o.floss[q] : 0.0);
            }
        }
    }
    // by pair type: ti + neighbour type (one type: pair type 0 only)
    const bool t1 = NT == 2 && __float_as_int(pi4.w) != 0;
    double ge[3] = {a.ge[0], 0.0, 0.0}, gs[3] = {a.gs[0], 0.0, 0.0};
    if (NT == 2) {
        ge[0] = t1 ? 0.0 : a.ge[0];
        ge[1] = t1 ? a.ge[0] : a.ge[1];
        ge[2] = t1 ? a.ge[1] : 0.0;
        gs[0] = t1 ? 0.0 : a.gs[0];
        gs[1] = t1 ? a.gs[0] : a.gs[1];
        gs[2] = t1 ? a.gs[1] : 0.0;
    }
    double v[6];
    for (int p = 0; p < 3; p++) {
        v[p] = ge[p];
        v[3 + p] = gs[p] * cf.inv_sig[p];
    }
    const int slot[6] = {0, 1, 2, 3, 4, 5};
    const int op[6] = {0, 0, 0, 0, 0, 0};
    block_partials<6>(v, slot, op, st.part, st.pstride);
}

// ---------------------------------------------------------------------------
// Symmetric half lists (the section 4.1 listing's getCellListSym and
// applyKernel_in_sym: every pair evaluated once, its reaction given to the
// partner, the ghost_put of section 3.4).  Lists hold every neighbour in
// ascending slot order, so the partners above slot i are its entries from
// plo[i] on and those below it the first plo[i].  At a rebuild k_sym_index
// finds, for each lower entry m of slot j (partner i < j), the position of j
// in i's list, by bisection of that sorted list (the four entries of a group
// searched together, so that their loads overlap).  Pass 1 evaluates each
// pair once, at its lower slot i: s (x_i - x_j) goes into i's own sum, the
// pair energy and virial into the partials, and the force factor s (0 off
// the force set) beside i's own list entry.  Pass 2 adds to every slot j the
// reactions s (x_j - x_i) of its lower partners in list order, the factors
// gathered from the partners' entries through the recorded positions, and
// applies the step's velocity-Verlet updates.  There are no atomics and every
// sum has a fixed order, so results repeat bit for bit.  Both passes walk
// whole groups of four entries in wavefront lockstep (from the first to the
// last group any lane of the wavefront needs), so list and factor stores stay
// coalesced; the factor gathers of pass 2 are the transposition the method
// needs, one random 8-byte read per pair.

__device__ __forceinline__ int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__global__ __launch_bounds__(kBlock) void k_sym_index(State st, int cap, int cap4) {
    const int s = block_system(st);
    if (!rebuilding(st, s)) return;
    const SysDesc &d = st.sys[s];
    const int64_t i64 = global_slot();
    const int i = (int)i64;
    const bool active = i64 - d.slot_base < d.n;
    const int32_t *__restrict__ nbr = st.nbr;
    const int cnt = active ? min((int)(st.nnb[i64] & ~kWrapBit), cap) : 0;
    int lo = 0, hi = cnt;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (nbr[nbr_index(i64, mid, cap4)] < i) lo = mid + 1;
        else hi = mid;
    }
    st.plo[i64] = lo;
    const int4 *lst = reinterpret_cast<const int4 *>(nbr) + ((i64 >> 6) * (int64_t)cap4) * 64 +
                      (i64 & 63);
    ushort4 *tl = reinterpret_cast<ushort4 *>(st.tsym) + ((i64 >> 6) * (int64_t)cap4) * 64 +
                  (i64 & 63);
    bool miss = false;
    const int g1 = wave_max((lo + 3) >> 2);
    for (int g = 0; g < g1; g++) {
        const int4 e = lst[g * 64];
        const int jj[4] = {e.x, e.y, e.z, e.w};
        int j[4], a[4], b[4];
        bool eq[4], on[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            on[t] = 4 * g + t < lo;
            j[t] = on[t] ? jj[t] : i;
            a[t] = 0;
            eq[t] = false;
        }
#pragma unroll
        for (int t = 0; t < 4; t++) b[t] = on[t] ? min((int)(st.nnb[j[t]] & ~kWrapBit), cap) : 0;
        // lower-bound searches for i in the lower partners' lists; eq records
        // whether the last probe that moved b found i itself
        while (__ballot(a[0] < b[0] || a[1] < b[1] || a[2] < b[2] || a[3] < b[3]) != 0) {
            int v[4];
#pragma unroll
            for (int t = 0; t < 4; t++)
                v[t] = a[t] < b[t] ? nbr[nbr_index(j[t], (a[t] + b[t]) >> 1, cap4)] : 0;
#pragma unroll
            for (int t = 0; t < 4; t++) {
                if (a[t] >= b[t]) continue;
                const int mid = (a[t] + b[t]) >> 1;
                if (v[t] < i) {
                    a[t] = mid + 1;
                } else {
                    b[t] = mid;
                    eq[t] = v[t] == i;
                }
            }
        }
        ushort4 o;
        o.x = (uint16_t)(on[0] ? a[0] : 0);
        o.y = (uint16_t)(on[1] ? a[1] : 0);
        o.z = (uint16_t)(on[2] ? a[2] : 0);
        o.w = (uint16_t)(on[3] ? a[3] : 0);
#pragma unroll
        for (int t = 0; t < 4; t++) miss |= on[t] && !eq[t];
        if (on[0] || on[1] || on[2] || on[3]) tl[g * 64] = o;
    }
    if (miss) st.ctl->sym_miss = 1;
}

// Exact FP64 separation x_i - x_j for the image the FP32 predicate takes
// (IMG as in separation).
template <int IMG>
__device__ __forceinline__ void pair_sep(float3 pi, double xi, double yi, double zi, float4 q,
                                         const Box &b, double &dx, double &dy, double &dz,
                                         const Sided &sd) {
    if (IMG == 2) {
        const float tx = q.x - pi.x, ty = q.y - pi.y, tz = q.z - pi.z;
        dx = (sd.sg[0] * tx > b.half[0] ? sd.xs[0] : xi) - (double)q.x;
        dy = (sd.sg[1] * ty > b.half[1] ? sd.xs[1] : yi) - (double)q.y;
        dz = (sd.sg[2] * tz > b.half[2] ? sd.xs[2] : zi) - (double)q.z;
        return;
    }
    dx = xi - (double)q.x;
    dy = yi - (double)q.y;
    dz = zi - (double)q.z;
    if (IMG == 1) {
        const float tx = q.x - pi.x, ty = q.y - pi.y, tz = q.z - pi.z;
        const double Lx = b.per[0] ? (double)b.L[0] : 0.0, Ly = b.per[1] ? (double)b.L[1] : 0.0,
                     Lz = b.per[2] ? (double)b.L[2] : 0.0;
        dx += tx > b.half[0] ? Lx : (tx < -b.half[0] ? -Lx : 0.0);
        dy += ty > b.half[1] ? Ly : (ty < -b.half[1] ? -Ly : 0.0);
        dz += tz > b.half[2] ? Lz : (tz < -b.half[2] ? -Lz : 0.0);
    }
}

template <int NT, int IMG>
__device__ __forceinline__ void sym_upper(const State &st, int64_t i, int p0, int cnt, float4 pi4,
                                          const Box &b, float rc2, double rc2lo, double rc2hi,
                                          const LJCoef &cf, int cap4, double (&f)[3], double &u,
                                          double (&w)[6], const Sided &sd) {
    const float3 pi = xyz(pi4);
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    const LaneCoef lc = lane_coef<NT>(cf, __float_as_int(pi4.w));
    const float4 *__restrict__ pos = st.pos[0];
    const int4 *lst = reinterpret_cast<const int4 *>(st.nbr) + ((i >> 6) * (int64_t)cap4) * 64 +
                      (i & 63);
    double2 *fac = reinterpret_cast<double2 *>(st.sbuf) +
                   (((i >> 6) * (int64_t)cap4) * 64 + (i & 63)) * 2;
    const int g0 = wave_min(p0 >> 2), g1 = wave_max((cnt + 3) >> 2);
    if (g0 >= g1) return;
    int4 e = lst[g0 * 64];
    for (int g = g0; g < g1; g++) {
        const int jj[4] = {e.x, e.y, e.z, e.w};
        double sv[4] = {0.0, 0.0, 0.0, 0.0};
        bool on[4];
        float4 q[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int k = 4 * g + t;
            on[t] = k >= p0 && k < cnt;
            q[t] = pos[on[t] ? jj[t] : (int)i];
        }
        if (g + 1 < g1) e = lst[(g + 1) * 64];  // the next group's entries, requested early
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (!on[t]) continue;
            double dx, dy, dz, sx, sy, sz;
            if (separation<IMG>(pi, xi, yi, zi, q[t], b, rc2, rc2lo, rc2hi, dx, dy, dz, sx, sy,
                                sz, &sd)) {
                double c12, c6;
                coef<NT>(lc, nbr_type<NT>(q[t]), c12, c6);
                const double r2i = recip(fma(dx, dx, fma(dy, dy, dz * dz)));
                const double r6i = r2i * r2i * r2i;
                sv[t] = r6i * r2i * fma(12.0 * c12, r6i, -6.0 * c6);
                u = fma(r6i, fma(c12, r6i, -c6), u);
                const double fx = sv[t] * dx, fy = sv[t] * dy, fz = sv[t] * dz;
                f[0] += fx;
                f[1] += fy;
                f[2] += fz;
                w[0] = fma(dx, fx, w[0]);
                w[1] = fma(dy, fy, w[1]);
                w[2] = fma(dz, fz, w[2]);
                w[3] = fma(dx, fy, w[3]);
                w[4] = fma(dx, fz, w[4]);
                w[5] = fma(dy, fz, w[5]);
            }
        }
        // the group's factors, at the lane's own entries (lower entries: 0, unused)
        if (on[0] || on[1] || on[2] || on[3]) {
            fac[g * 128] = make_double2(sv[0], sv[1]);
            fac[g * 128 + 1] = make_double2(sv[2], sv[3]);
        }
    }
}

// Pass 1 (see above): each pair at its lower slot.
template <int NT>
__global__ __launch_bounds__(kBlock) void k_lj_sym1(State st, float rc2, double rc2lo,
                                                    double rc2hi, LJCoef cf, int cap, int cap4,
                                                    double *part) {
    const SysDesc &d = st.sys[block_system(st)];
    const Box b = d.box;
    const int64_t i = global_slot();
    const bool active = i - d.slot_base < d.n;
    uint32_t nn = 0;
    int p0 = 0;
    float4 pi4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (active) {
        nn = st.nnb[i];
        p0 = st.plo[i];
        pi4 = st.pos[0][i];
    }
    const bool img_wave = __ballot((nn & kWrapBit) != 0) != 0;
    const int cnt = min((int)(nn & ~kWrapBit), cap);
    double f[3] = {0.0, 0.0, 0.0}, u = 0.0, w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool side_ok = true;
    const Sided sd = make_sided(xyz(pi4), pi4.x, pi4.y, pi4.z, b, cf.side_margin, cf.side_wide,
                                 side_ok);
    if (img_wave && __ballot(active && !side_ok) == 0)
        sym_upper<NT, 2>(st, i, p0, cnt, pi4, b, rc2, rc2lo, rc2hi, cf, cap4, f, u, w, sd);
    else if (img_wave)
        sym_upper<NT, 1>(st, i, p0, cnt, pi4, b, rc2, rc2lo, rc2hi, cf, cap4, f, u, w, sd);
    else
        sym_upper<NT, 0>(st, i, p0, cnt, pi4, b, rc2, rc2lo, rc2hi, cf, cap4, f, u, w, sd);
    if (active)
        for (int c = 0; c < 3; c++) st.fown[3 * i + c] = f[c];
    double v[7] = {u, w[0], w[1], w[2], w[3], w[4], w[5]};
    const int slot[7] = {0, 1, 2, 3, 4, 5, 6};
    const int op[7] = {0, 0, 0, 0, 0, 0, 0};
    block_partials<7>(v, slot, op, part, st.pstride);
}

template <int IMG>
__device__ __forceinline__ void sym_lower(const State &st, int64_t j, int p, float4 pj4,
                                          const Box &b, int cap4, double (&f)[3],
                                          const Sided &sd) {
    const float3 pj = xyz(pj4);
    const double xj = pj.x, yj = pj.y, zj = pj.z;
    const float4 *__restrict__ pos = st.pos[0];
    const int4 *lst = reinterpret_cast<const int4 *>(st.nbr) + ((j >> 6) * (int64_t)cap4) * 64 +
                      (j & 63);
    const ushort4 *tl = reinterpret_cast<const ushort4 *>(st.tsym) +
                        ((j >> 6) * (int64_t)cap4) * 64 + (j & 63);
    const int g1 = wave_max((p + 3) >> 2);
    if (g1 <= 0) return;
    int4 e = lst[0];
    ushort4 tm = tl[0];
    for (int g = 0; g < g1; g++) {
        const int ii[4] = {e.x, e.y, e.z, e.w};
        const int kk[4] = {tm.x, tm.y, tm.z, tm.w};
        float4 q[4];
        double sv[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const bool ok = 4 * g + t < p;
            q[t] = pos[ok ? ii[t] : (int)j];
            sv[t] = ok ? st.sbuf[nbr_index(ii[t], kk[t], cap4)] : 0.0;
        }
        if (g + 1 < g1) {
            e = lst[(g + 1) * 64];
            tm = tl[(g + 1) * 64];
        }
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (4 * g + t >= p) continue;
            double dx, dy, dz;
            pair_sep<IMG>(pj, xj, yj, zj, q[t], b, dx, dy, dz, sd);
            f[0] = fma(sv[t], dx, f[0]);
            f[1] = fma(sv[t], dy, f[1]);
            f[2] = fma(sv[t], dz, f[2]);
        }
    }
}

// Pass 2 (see above): reactions from the lower partners, then the forces and
// (MODE kLjStep, kLjLast) the step's updates as in k_lj.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_lj_sym2(State st, int cap4, StepArgs sa,
                                                    float side_margin, float side_wide) {
    const int sys = block_system(st);
    const SysDesc &d = st.sys[sys];
    const Box b = d.box;
    const int64_t i = global_slot();
    const bool active = i - d.slot_base < d.n;
    uint32_t nn = 0;
    int p = 0;
    float4 pi4 = make_float4(0.f, 0.f, 0.f, 0.f), v4 = pi4, xb4 = pi4;
    double f[3] = {0.0, 0.0, 0.0};
    if (active) {
        nn = st.nnb[i];
        p = st.plo[i];
        pi4 = st.pos[0][i];
        if (MODE != kLjForce) v4 = st.vel[0][i];
        if (MODE == kLjStep) xb4 = st.xbuild[i];
        for (int c = 0; c < 3; c++) f[c] = st.fown[3 * i + c];
    }
    bool side_ok = true;
    const Sided sd =
        make_sided(xyz(pi4), pi4.x, pi4.y, pi4.z, b, side_margin, side_wide, side_ok);
    const bool img_wave = __ballot((nn & kWrapBit) != 0) != 0;
    if (img_wave && __ballot(active && !side_ok) == 0)
        sym_lower<2>(st, i, p, pi4, b, cap4, f, sd);
    else if (img_wave)
        sym_lower<1>(st, i, p, pi4, b, cap4, f, sd);
    else
        sym_lower<0>(st, i, p, pi4, b, cap4, f, sd);
    double ke = 0.0;
    bool over = false;
    if (active) {
        const float4 fo = make_float4((float)f[0], (float)f[1], (float)f[2], 0.f);
        if (MODE != kLjStep) st.frc[i] = fo;
        if (!isfinite(f[0]) || !isfinite(f[1]) || !isfinite(f[2])) st.ctl->nonfinite = 1;
        if (MODE != kLjForce)
            ke = kick_drift<MODE>(st, d, i, fo, pi4, v4, xb4, sa.dt, sa.thr, over);
    }
    if (MODE != kLjForce) {
        SysCtl *sc = st.sctl + sys;
        if (MODE == kLjStep) {
            const uint64_t m = __ballot(over);
            if (m && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1)
                sc->rebuild[st.par ^ 1] = 1;
        }
        if (threadIdx.x == 0 && pblock() == d.blk_base) {
            if (sc->rebuild[st.par]) {
                sc->n_rebuilds += 1;
                sc->rebuild[st.par] = 0;
            }
            sc->step += 1;
        }
        double v1[1] = {ke};
        const int s1[1] = {7}, o1[1] = {0};
        block_partials<1>(v1, s1, o1, sa.ring, st.pstride);
    }
}

// Margin of the one-face image form (Sided): particles stay within half the
// skin of their build positions; above half box lengths of side_wide every
// lane takes the form.
float side_margin(const fpm_ctx *c) { return 0.5f * c->skin * 1.001f + 1e-4f; }
float side_wide(const fpm_ctx *c) { return c->r_cut * 1.00001f + side_margin(c); }

LJCoef make_coef(const fpm_ctx *c, const fpm_lj_params &p) {
    LJCoef cf;
    for (int k = 0; k < 3; k++) {
        const double e = (double)p.eps[k], s = (double)p.sig[k];
        const double s6 = s * s * s * s * s * s;
        cf.c12[k] = 4.0 * e * s6 * s6;
        cf.c6[k] = 4.0 * e * s6;
        cf.a12[k] = 4.0 * s6 * s6;
        cf.a6[k] = 4.0 * s6;
        cf.inv_sig[k] = 1.0 / s;
    }
    cf.side_margin = side_margin(c);
    cf.side_wide = side_wide(c);
    return cf;
}

}  // namespace

namespace {

template <int MODE>
void launch_lj_mode(fpm_ctx *c, const fpm_lj_params &p, const StepArgs &sa) {
    const LJCoef cf = make_coef(c, p);
    const double band = predicate_band(c);
    const double rc2lo = (double)c->rc2 * (1.0 - band), rc2hi = (double)c->rc2 * (1.0 + band);
    const dim3 g((unsigned)c->nblk), t(kBlock);
    const bool u4 = c->tune_unroll == 4;
    if (p.n_types == 2) {
        if (u4)
            hipLaunchKernelGGL((k_lj<2, 4, MODE>), g, t, 0, c->stream, c->st, c->rc2, rc2lo,
                               rc2hi, cf, c->cap4, sa);
        else
            hipLaunchKernelGGL((k_lj<2, 8, MODE>), g, t, 0, c->stream, c->st, c->rc2, rc2lo,
                               rc2hi, cf, c->cap4, sa);
    } else {
        if (u4)
            hipLaunchKernelGGL((k_lj<1, 4, MODE>), g, t, 0, c->stream, c->st, c->rc2, rc2lo,
                               rc2hi, cf, c->cap4, sa);
        else
            hipLaunchKernelGGL((k_lj<1, 8, MODE>), g, t, 0, c->stream, c->st, c->rc2, rc2lo,
                               rc2hi, cf, c->cap4, sa);
    }
}

}  // namespace

namespace {

// The two passes over symmetric half lists; pass 1's partials go to `part`
// (the force partials, or the step's ring row).
template <int MODE>
void launch_sym_mode(fpm_ctx *c, const fpm_lj_params &p, const StepArgs &sa, double *part) {
    const LJCoef cf = make_coef(c, p);
    const double band = predicate_band(c);
    const double rc2lo = (double)c->rc2 * (1.0 - band), rc2hi = (double)c->rc2 * (1.0 + band);
    const dim3 g((unsigned)c->nblk), t(kBlock);
    if (p.n_types == 2)
        hipLaunchKernelGGL(k_lj_sym1<2>, g, t, 0, c->stream, c->st, c->rc2, rc2lo, rc2hi, cf,
                           c->cap, c->cap4, part);
    else
        hipLaunchKernelGGL(k_lj_sym1<1>, g, t, 0, c->stream, c->st, c->rc2, rc2lo, rc2hi, cf,
                           c->cap, c->cap4, part);
    hipLaunchKernelGGL(k_lj_sym2<MODE>, g, t, 0, c->stream, c->st, c->cap4, sa,
                       side_margin(c), side_wide(c));
}

}  // namespace

hipError_t launch_lj_forces(fpm_ctx *c, const fpm_lj_params &p) {
    if (c->sym)
        launch_sym_mode<kLjForce>(c, p, StepArgs{0.f, 0.f, nullptr}, c->st.part);
    else
        launch_lj_mode<kLjForce>(c, p, StepArgs{0.f, 0.f, nullptr});
    return hipGetLastError();
}

hipError_t launch_lj_step(fpm_ctx *c, const fpm_lj_params &p, float dt, bool last, int row) {
    const StepArgs sa{dt, c->disp2_thr, c->st.ring + (size_t)row * 8 * c->st.pstride};
    if (c->sym) {
        if (last)
            launch_sym_mode<kLjLast>(c, p, sa, sa.ring);
        else
            launch_sym_mode<kLjStep>(c, p, sa, sa.ring);
    } else if (last) {
        launch_lj_mode<kLjLast>(c, p, sa);
    } else {
        launch_lj_mode<kLjStep>(c, p, sa);
    }
    return hipGetLastError();
}

hipError_t launch_sym_index(fpm_ctx *c) {
    hipLaunchKernelGGL(k_sym_index, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, c->cap,
                       c->cap4);
    return hipGetLastError();
}

hipError_t launch_lj_vjp(fpm_ctx *c, const fpm_lj_params &p, const double *lam,
                         const double *vbar, const AdjOut &o) {
    const LJCoef cf = make_coef(c, p);
    const double band = predicate_band(c);
    const double rc2lo = (double)c->rc2 * (1.0 - band), rc2hi = (double)c->rc2 * (1.0 + band);
    const dim3 g((unsigned)c->nblk), t(kBlock);
    hipLaunchKernelGGL(k_gather_lam, g, t, 0, c->stream, c->st, lam, vbar, 0.5 * o.dt);
    if (p.n_types == 2)
        hipLaunchKernelGGL(k_lj_vjp<2>, g, t, 0, c->stream, c->st, c->rc2, rc2lo, rc2hi, cf,
                           c->cap4, o);
    else
        hipLaunchKernelGGL(k_lj_vjp<1>, g, t, 0, c->stream, c->st, c->rc2, rc2lo, rc2hi, cf,
                           c->cap4, o);
    return hipGetLastError();
}

}  // namespace fpm
