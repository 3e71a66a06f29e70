// Velocity Verlet (section 4.1 listing: v += dt/2 F; x += dt v; new forces;
// v += dt/2 F), unit mass, fused per step into one pass over the particles:
// the closing half kick of step n and the opening half kick + drift of step
// n + 1 touch the same arrays, so they run together, and the kinetic energy of
// step n is taken from the full-step velocity on the way.  The drift also
// measures the displacement since the last neighbour-list build; the finalize
// kernel turns the largest one into the device rebuild flag (the
// updateCellListSym of the listing, decided on the device).
#include "geom.h"

namespace fpm {
namespace {

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_integrate(State st, Box b, int64_t n, float dt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float h = 0.5f * dt;
    double ke = 0.0, d2 = 0.0;
    if (i < n) {
        float4 v = st.vel[0][i];
        const float4 f = st.frc[i];
        v.x += h * f.x;
        v.y += h * f.y;
        v.z += h * f.z;
        if (MODE != kKickDriftFirst)
            ke = (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z;
        if (MODE == kKickKickDrift) {
            v.x += h * f.x;
            v.y += h * f.y;
            v.z += h * f.z;
        }
        st.vel[0][i] = v;
        if (MODE != kKickOnly) {
            float4 p = st.pos[0][i];
            p.x += dt * v.x;
            p.y += dt * v.y;
            p.z += dt * v.z;
            st.pos[0][i] = p;
            d2 = dist2_pred(xyz(st.xbuild[i]), xyz(p), b);
            if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z)) st.ctl->nonfinite = 1;
        }
    }
    if (MODE == kKickDriftFirst) {
        double v1[1] = {d2};
        const int s1[1] = {kSlotDisp}, o1[1] = {1};
        block_partials<1>(v1, s1, o1, st.part, st.pstride);
    } else if (MODE == kKickKickDrift) {
        double v2[2] = {ke, d2};
        const int s2[2] = {kSlotKE, kSlotDisp}, o2[2] = {0, 1};
        block_partials<2>(v2, s2, o2, st.part, st.pstride);
    } else {
        double v1[1] = {ke};
        const int s1[1] = {kSlotKE}, o1[1] = {0};
        block_partials<1>(v1, s1, o1, st.part, st.pstride);
    }
}

// One workgroup of 1024 threads reduces the per-block partials in a fixed
// order (thread t takes blocks t, t + 1024, ... of the slots it needs, all
// loads issued before any is summed; then wavefront shuffles, and one thread
// per slot adds the 16 wavefront results in order) and applies the step's
// control logic (see the kFin* modes).
constexpr int kFinRowsPerThread = 4;  // blocks per thread and pass (4096 workgroups per pass)

__global__ __launch_bounds__(1024) void k_finalize(State st, int nblk, int mode, float thr,
                                                   double *out, double *rows) {
    constexpr int NS = 9;  // U, W6, KE, displacement
    __shared__ double red[16][NS];
    __shared__ double tot[NS];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const bool want_f = mode & kFinForce, want_k = mode & kFinKE, want_d = mode & kFinDisp;
    const double *P = st.part;
    const int64_t S = st.pstride;
    double acc[NS];
#pragma unroll
    for (int c = 0; c < NS; c++) acc[c] = 0.0;
    for (int r0 = t; r0 < nblk; r0 += 1024 * kFinRowsPerThread) {
        double v[kFinRowsPerThread][NS];
#pragma unroll
        for (int q = 0; q < kFinRowsPerThread; q++) {
            const int r = r0 + q * 1024;
            const bool ok = r < nblk;
#pragma unroll
            for (int c = 0; c < 7; c++) v[q][c] = (want_f && ok) ? P[c * S + r] : 0.0;
            v[q][7] = (want_k && ok) ? P[kSlotKE * S + r] : 0.0;
            v[q][8] = (want_d && ok) ? P[kSlotDisp * S + r] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kFinRowsPerThread; q++) {
#pragma unroll
            for (int c = 0; c < 8; c++) acc[c] += v[q][c];
            acc[8] = fmax(acc[8], v[q][8]);
        }
    }
#pragma unroll
    for (int c = 0; c < 8; c++) acc[c] = wave_sum(acc[c]);
    acc[8] = wave_max(acc[8]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NS; c++) red[w][c] = acc[c];
    __syncthreads();
    if (t < NS) {
        double s = red[0][t];
        for (int k = 1; k < 16; k++) s = t == 8 ? fmax(s, red[k][t]) : s + red[k][t];
        tot[t] = s;
    }
    __syncthreads();
    if (t != 0) return;
    Ctl *ctl = st.ctl;
    if ((mode & kFinBuild) && ctl->rebuild) {
        ctl->n_rebuilds += 1;
        ctl->rebuild = 0;
    }
    if (want_f) {
        ctl->thermo[0] = tot[kSlotU];
        for (int c = 0; c < 6; c++) ctl->thermo[2 + c] = tot[kSlotW + c];
        if (out) {
            out[0] = tot[kSlotU];
            out[1] = 0.0;
            for (int c = 0; c < 6; c++) out[2 + c] = tot[kSlotW + c];
        }
    }
    if (want_k) ctl->thermo[1] = 0.5 * tot[kSlotKE];
    if (mode & kFinRow) {
        const int row = ctl->step;
        if (rows)
            for (int c = 0; c < 8; c++) rows[(int64_t)row * 8 + c] = ctl->thermo[c];
        ctl->step = row + 1;
    }
    if (want_d && tot[8] > (double)thr) ctl->rebuild = 1;
}

__global__ void k_reset_step(Ctl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->step = 0;
}

// State back in caller order.
__global__ void k_gather_out(State st, int64_t n, float *pos, float *vel, float *frc, float *rho,
                             float *drho) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = st.id[0][i];
    const float4 p = st.pos[0][i], v = st.vel[0][i], f = st.frc[i];
    if (pos) {
        pos[3 * r] = p.x;
        pos[3 * r + 1] = p.y;
        pos[3 * r + 2] = p.z;
    }
    if (vel) {
        vel[3 * r] = v.x;
        vel[3 * r + 1] = v.y;
        vel[3 * r + 2] = v.z;
    }
    if (frc) {
        frc[3 * r] = f.x;
        frc[3 * r + 1] = f.y;
        frc[3 * r + 2] = f.z;
    }
    if (rho) rho[r] = v.w;
    if (drho) drho[r] = f.w;
}

}  // namespace

hipError_t launch_integrate(fpm_ctx *c, float dt, int mode) {
    const unsigned g = (unsigned)c->nblk;
    if (mode == kKickDriftFirst)
        hipLaunchKernelGGL(k_integrate<kKickDriftFirst>, dim3(g), dim3(kBlock), 0, c->stream,
                           c->st, c->box, c->n, dt);
    else if (mode == kKickKickDrift)
        hipLaunchKernelGGL(k_integrate<kKickKickDrift>, dim3(g), dim3(kBlock), 0, c->stream,
                           c->st, c->box, c->n, dt);
    else
        hipLaunchKernelGGL(k_integrate<kKickOnly>, dim3(g), dim3(kBlock), 0, c->stream, c->st,
                           c->box, c->n, dt);
    return hipGetLastError();
}

hipError_t launch_finalize(fpm_ctx *c, int mode, double *out, double *rows) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, c->stream, c->st, c->nblk, mode,
                       c->disp2_thr, out, rows);
    return hipGetLastError();
}

hipError_t launch_reset_step(fpm_ctx *c) {
    hipLaunchKernelGGL(k_reset_step, dim3(1), dim3(64), 0, c->stream, c->st.ctl);
    return hipGetLastError();
}

hipError_t launch_gather_out(fpm_ctx *c, float *pos, float *vel, float *frc, float *rho,
                             float *drho) {
    const unsigned g = (unsigned)((c->n + 255) / 256);
    hipLaunchKernelGGL(k_gather_out, dim3(g), dim3(256), 0, c->stream, c->st, c->n, pos, vel, frc,
                       rho, drho);
    return hipGetLastError();
}

}  // namespace fpm
