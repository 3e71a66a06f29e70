// Lennard-Jones forces, potential energy and virial over the Verlet list
// (section 4.1: V(r) = 4 eps ((sig/r)^12 - (sig/r)^6); the force on p from q is
// 24 eps (2 sig^12 / rn^7 - sig^6 / rn^4) (xp - xq), rn = |xp - xq|^2, and the
// pair is dropped when rn > r_cut^2).
//
// One lane per cell-sorted particle walks its full list (every pair is seen
// from both sides, so there are no scattered writes).  The list is read eight
// entries at a time (two 16-byte loads per lane) and the eight neighbour
// positions are gathered before any is used, so each lane keeps eight loads in
// flight instead of waiting on every entry.
//
// Set membership follows the FP32 predicate exactly; the pair physics is
// evaluated in FP64 from the exact separation of the FP32 coordinates and
// accumulated per lane in FP64.  The FP64 squared distance decides membership
// directly unless it lies within a relative 1e-6 of r_cut^2, where the FP32
// predicate (whose error is below 5 ulp, about 3e-7 relative) is evaluated.
// Energy and virial partials go to one row per workgroup; the finalize kernel
// sums them in a fixed order.
#include "geom.h"

namespace fpm {
namespace {

struct LJCoef {
    double c12[3];  // 4 eps sig^12
    double c6[3];   // 4 eps sig^6
};

// 1/x in FP64: the hardware estimate refined by one Newton step.
__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Per-lane accumulators.  The virial needs no per-pair work: summed over all
// particles, 1/2 sum_ij r_ij (x) f_ij with r_ij = x_i - x_j + s_ij (s_ij the
// periodic shift, f_ji = -f_ij, s_ji = -s_ij) equals
// sum_i x_i (x) F_i + 1/2 sum_ij s_ij (x) f_ij, so each lane adds x_i (x) F_i
// once and only image pairs add a shift term (wx*).
struct Acc {
    double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0;
    double wxx = 0.0, wyy = 0.0, wzz = 0.0, wxy = 0.0, wxz = 0.0, wyz = 0.0;
};

// One list entry.  Padding entries point at a particle far away, so every
// entry can be processed without a bounds test.
template <int NT, bool IMG>
__device__ __forceinline__ void pair(Acc &a, float3 pi, double xi, double yi, double zi, int ti,
                                     float4 q, const Box &b, float rc2, double rc2lo,
                                     double rc2hi, const LJCoef &cf) {
    double dx = xi - (double)q.x, dy = yi - (double)q.y, dz = zi - (double)q.z;
    double sx = 0.0, sy = 0.0, sz = 0.0;  // periodic shift of this pair
    if (IMG) {
        sx = -(double)img_shift(pi.x, q.x, b.half[0], b.per[0]) * (double)b.L[0];
        sy = -(double)img_shift(pi.y, q.y, b.half[1], b.per[1]) * (double)b.L[1];
        sz = -(double)img_shift(pi.z, q.z, b.half[2], b.per[2]) * (double)b.L[2];
        dx += sx;
        dy += sy;
        dz += sz;
    }
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    bool in = r2 <= rc2lo;
    if (!in && r2 <= rc2hi)
        in = (IMG ? dist2_pred(pi, xyz(q), b) : dist2_direct(pi, xyz(q))) <= rc2;
    if (in) {
        double c12 = cf.c12[0], c6 = cf.c6[0];
        if (NT == 2) {
            const int tp = ti + __float_as_int(q.w);
            c12 = tp == 0 ? cf.c12[0] : (tp == 1 ? cf.c12[1] : cf.c12[2]);
            c6 = tp == 0 ? cf.c6[0] : (tp == 1 ? cf.c6[1] : cf.c6[2]);
        }
        const double r2i = recip(r2);
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

// Walks a list padded to a multiple of eight entries.
template <int NT, bool IMG>
__device__ __forceinline__ void walk(Acc &a, const float4 *__restrict__ pos,
                                     const int4 *__restrict__ lst, int cnt, float4 pi4,
                                     const Box &b, float rc2, double rc2lo, double rc2hi,
                                     const LJCoef &cf) {
    const float3 pi = xyz(pi4);
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    const int ti = __float_as_int(pi4.w);
    for (int k = 0; k < cnt; k += 8) {
        const int4 e0 = lst[(k >> 2) * 64];
        const int4 e1 = lst[((k >> 2) + 1) * 64];
        const int jj[8] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
        float4 q[8];
#pragma unroll
        for (int u = 0; u < 8; u++) q[u] = pos[jj[u]];
#pragma unroll
        for (int u = 0; u < 8; u++)
            pair<NT, IMG>(a, pi, xi, yi, zi, ti, q[u], b, rc2, rc2lo, rc2hi, cf);
    }
}

template <int NT>
__global__ __launch_bounds__(kBlock) void k_lj(State st, Box b, int64_t n, float rc2,
                                               double rc2lo, double rc2hi, LJCoef cf, int cap4) {
    const float4 *__restrict__ pos = st.pos[0];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t nn = 0;
    float4 pi4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < n) {
        nn = st.nnb[i];
        pi4 = pos[i];
    }
    const bool img_wave = __ballot((nn & kWrapBit) != 0) != 0;
    const int cnt = (int)(nn & ~kWrapBit);
    const int4 *lst = reinterpret_cast<const int4 *>(st.nbr) +
                      ((i >> 6) * (int64_t)cap4) * 64 + (i & 63);
    Acc a;
    if (img_wave)
        walk<NT, true>(a, pos, lst, cnt, pi4, b, rc2, rc2lo, rc2hi, cf);
    else
        walk<NT, false>(a, pos, lst, cnt, pi4, b, rc2, rc2lo, rc2hi, cf);
    if (i < n) {
        st.frc[i] = make_float4((float)a.fx, (float)a.fy, (float)a.fz, (float)(0.5 * a.u));
        if (!isfinite(a.fx) || !isfinite(a.fy) || !isfinite(a.fz)) st.ctl->nonfinite = 1;
    }
    const double xi = pi4.x, yi = pi4.y, zi = pi4.z;
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
}

}  // namespace

hipError_t launch_lj_forces(fpm_ctx *c, const fpm_lj_params &p) {
    LJCoef cf;
    for (int k = 0; k < 3; k++) {
        const double e = (double)p.eps[k], s = (double)p.sig[k];
        const double s6 = s * s * s * s * s * s;
        cf.c12[k] = 4.0 * e * s6 * s6;
        cf.c6[k] = 4.0 * e * s6;
    }
    const double band = predicate_band(c);
    const double rc2lo = (double)c->rc2 * (1.0 - band), rc2hi = (double)c->rc2 * (1.0 + band);
    const unsigned g = (unsigned)((c->n_pad + kBlock - 1) / kBlock);
    if (p.n_types == 2)
        hipLaunchKernelGGL(k_lj<2>, dim3(g), dim3(kBlock), 0, c->stream, c->st, c->box, c->n,
                           c->rc2, rc2lo, rc2hi, cf, c->cap4);
    else
        hipLaunchKernelGGL(k_lj<1>, dim3(g), dim3(kBlock), 0, c->stream, c->st, c->box, c->n,
                           c->rc2, rc2lo, rc2hi, cf, c->cap4);
    return hipGetLastError();
}

}  // namespace fpm
