// Lennard-Jones forces, potential energy and virial over the Verlet list
// (section 4.1: V(r) = 4 eps ((sig/r)^12 - (sig/r)^6); the force on p from q is
// 24 eps (2 sig^12 / rn^7 - sig^6 / rn^4) (xp - xq), rn = |xp - xq|^2, and the
// pair is dropped when rn > r_cut^2).
//
// One lane per cell-sorted particle walks its list (full list: every pair is
// seen from both sides, so no scattered writes).  Set membership follows the
// FP32 predicate exactly; the pair physics is evaluated in FP64 from the exact
// separation of the FP32 coordinates and accumulated per lane in FP64.  The
// FP64 squared distance r2 decides membership directly unless it lies within
// a relative 1e-6 of r_cut^2, where the FP32 predicate (whose error is below
// 5 ulp, i.e. 3e-7 relative) is evaluated instead.  Energy and virial are
// reduced per wavefront with shuffles, per workgroup through LDS, and across
// workgroups by the last workgroup in a fixed order, so the totals do not
// depend on scheduling.
#include "geom.h"

namespace fpm {
namespace {

struct LJCoef {
    double c12[3];  // 4 eps sig^12
    double c6[3];   // 4 eps sig^6
};

// 1/x in FP64 from the hardware estimate refined by two Newton steps.
__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Block-wide fixed-order sum of NV doubles per thread; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[NV]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NV; c++) v[c] = wave_sum(v[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; c++) lds[w][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
#pragma unroll
        for (int c = 0; c < NV; c++) {
            double s = 0.0;
            for (int k = 0; k < nw; k++) s += lds[k][c];
            v[c] = s;
        }
    }
}

// Sum of part[b * 8 + c] over all blocks b, by one block, in a fixed order.
template <int NV>
__device__ void reduce_partials(const double *part, int nblocks, double (&tot)[NV]) {
    __shared__ double red[kBlock][NV];
    const int t = threadIdx.x;
    double acc[NV];
#pragma unroll
    for (int c = 0; c < NV; c++) acc[c] = 0.0;
    for (int bidx = t; bidx < nblocks; bidx += blockDim.x)
#pragma unroll
        for (int c = 0; c < NV; c++) acc[c] += part[(int64_t)bidx * 8 + c];
#pragma unroll
    for (int c = 0; c < NV; c++) red[t][c] = acc[c];
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int c = 0; c < NV; c++) red[t][c] += red[t + s][c];
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < NV; c++) tot[c] = red[0][c];
}

template <int NT>
__global__ __launch_bounds__(kBlock) void k_lj(State st, Box b, int64_t n, float rc2,
                                               double rc2lo, double rc2hi, LJCoef cf, int cap,
                                               double *out, double *thermo, int rows,
                                               int count_step) {
    Ctl *ctl = st.ctl;
    const int cur = ctl->cur;
    const float4 *__restrict__ pos = st.pos[cur];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;

    double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0;
    double wxx = 0.0, wyy = 0.0, wzz = 0.0, wxy = 0.0, wxz = 0.0, wyz = 0.0;
    uint32_t nn = 0;
    float4 pi4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < n) {
        nn = st.nnb[i];
        pi4 = pos[i];
    }
    const bool img_wave = __ballot((nn & kWrapBit) != 0) != 0;
    const int cnt = (int)(nn & ~kWrapBit);
    const float3 pi = xyz(pi4);
    const double xi = pi.x, yi = pi.y, zi = pi.z;
    const int ti = __float_as_int(pi4.w);
    const int32_t *__restrict__ lst = st.nbr + ((i >> 6) * (int64_t)cap) * 64 + (i & 63);

    for (int k = 0; k < cnt; k++) {
        const int j = lst[(int64_t)k * 64];
        const float4 q = pos[j];
        double dx, dy, dz;
        if (img_wave) {
            dx = sep_axis(pi.x, q.x, b.L[0], b.half[0], b.per[0]);
            dy = sep_axis(pi.y, q.y, b.L[1], b.half[1], b.per[1]);
            dz = sep_axis(pi.z, q.z, b.L[2], b.half[2], b.per[2]);
        } else {
            dx = xi - (double)q.x;
            dy = yi - (double)q.y;
            dz = zi - (double)q.z;
        }
        const double r2 = dx * dx + dy * dy + dz * dz;
        bool in = r2 <= rc2lo;
        if (!in && r2 <= rc2hi) in = dist2_pred(pi, xyz(q), b) <= rc2;
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
            u = fma(r6i, fma(c12, r6i, -c6), u);
            const double sx = s * dx, sy = s * dy, sz = s * dz;
            fx += sx;
            fy += sy;
            fz += sz;
            wxx = fma(sx, dx, wxx);
            wyy = fma(sy, dy, wyy);
            wzz = fma(sz, dz, wzz);
            wxy = fma(sx, dy, wxy);
            wxz = fma(sx, dz, wxz);
            wyz = fma(sy, dz, wyz);
        }
    }
    if (i < n) {
        st.frc[i] = make_float4((float)fx, (float)fy, (float)fz, 0.f);
        if (!isfinite(fx) || !isfinite(fy) || !isfinite(fz)) atomicOr(&ctl->nonfinite, 1);
    }

    __shared__ double lds[kBlock / 64][7];
    double v[7] = {0.5 * u, 0.5 * wxx, 0.5 * wyy, 0.5 * wzz, 0.5 * wxy, 0.5 * wxz, 0.5 * wyz};
    block_sum<7>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < 7; c++) st.part[(int64_t)blockIdx.x * 8 + c] = v[c];
    if (last_block(&ctl->done[2])) {
        double tot[7];
        reduce_partials<7>(st.part, gridDim.x, tot);
        if (threadIdx.x == 0) {
            ctl->thermo[0] = tot[0];
            for (int c = 1; c < 7; c++) ctl->thermo[c + 1] = tot[c];
            if (out) {
                out[0] = tot[0];
                out[1] = 0.0;
                for (int c = 1; c < 7; c++) out[c + 1] = tot[c];
            }
            if (count_step) {
                const int row = ctl->step;
                if (thermo && row < rows) {
                    thermo[(int64_t)row * 8 + 0] = tot[0];
                    for (int c = 1; c < 7; c++) thermo[(int64_t)row * 8 + c + 1] = tot[c];
                }
                ctl->step = row + 1;
            }
        }
    }
}

}  // namespace

hipError_t launch_lj_forces(fpm_ctx *c, const fpm_lj_params &p, double *out, double *thermo,
                            int32_t rows, int count_step) {
    LJCoef cf;
    for (int k = 0; k < 3; k++) {
        const double e = (double)p.eps[k], s = (double)p.sig[k];
        const double s6 = s * s * s * s * s * s;
        cf.c12[k] = 4.0 * e * s6 * s6;
        cf.c6[k] = 4.0 * e * s6;
    }
    const double rc2lo = (double)c->rc2 * (1.0 - 1e-6), rc2hi = (double)c->rc2 * (1.0 + 1e-6);
    const unsigned g = (unsigned)((c->n_pad + kBlock - 1) / kBlock);
    if (p.n_types == 2)
        hipLaunchKernelGGL(k_lj<2>, dim3(g), dim3(kBlock), 0, c->stream, c->st, c->box, c->n,
                           c->rc2, rc2lo, rc2hi, cf, c->cap, out, thermo, rows, count_step);
    else
        hipLaunchKernelGGL(k_lj<1>, dim3(g), dim3(kBlock), 0, c->stream, c->st, c->box, c->n,
                           c->rc2, rc2lo, rc2hi, cf, c->cap, out, thermo, rows, count_step);
    return hipGetLastError();
}

}  // namespace fpm
