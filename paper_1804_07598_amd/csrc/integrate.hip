// Velocity Verlet (section 4.1 listing: v += dt/2 F; x += dt v; new forces;
// v += dt/2 F), unit mass, fused per step into one pass over the particles:
// the closing half kick of step n and the opening half kick + drift of step
// n + 1 touch the same arrays, so they run together, and the kinetic energy of
// step n is taken from the full-step velocity on the way.  The drift also
// measures the displacement since the last neighbour-list build and raises the
// device rebuild flag when the largest one exceeds skin/2 (the
// updateCellListSym of the listing, decided on the device).
#include "geom.h"

namespace fpm {
namespace {

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_integrate(State st, Box b, int64_t n, float dt,
                                                      float thr, double *thermo, int rows) {
    Ctl *ctl = st.ctl;
    const int cur = ctl->cur;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float h = 0.5f * dt;
    double ke = 0.0;
    float d2 = 0.0f;
    if (i < n) {
        float4 v = st.vel[cur][i];
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
        st.vel[cur][i] = v;
        if (MODE != kKickOnly) {
            float4 p = st.pos[cur][i];
            p.x += dt * v.x;
            p.y += dt * v.y;
            p.z += dt * v.z;
            st.pos[cur][i] = p;
            d2 = dist2_pred(xyz(st.xbuild[i]), xyz(p), b);
            if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z)) atomicOr(&ctl->nonfinite, 1);
        }
    }
    if (MODE != kKickOnly) {
        // non-negative floats order like their bit patterns
        const float m = wave_max(d2);
        if ((threadIdx.x & 63) == 0 && m > 0.0f) atomicMax(&ctl->maxdisp2, __float_as_uint(m));
    }
    if (MODE != kKickDriftFirst) {
        __shared__ double lds[kBlock / 64];
        const double w = wave_sum(ke);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int k = 0; k < kBlock / 64; k++) s += lds[k];
            st.part[(int64_t)blockIdx.x * 8 + 7] = s;
        }
    }
    if (last_block(&ctl->done[3])) {
        if (MODE != kKickDriftFirst) {
            __shared__ double red[kBlock];
            double acc = 0.0;
            for (int k = threadIdx.x; k < (int)gridDim.x; k += blockDim.x)
                acc += st.part[(int64_t)k * 8 + 7];
            red[threadIdx.x] = acc;
            __syncthreads();
            for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
                if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                const double kin = 0.5 * red[0];
                ctl->thermo[1] = kin;
                const int row = ctl->step - 1;
                if (thermo && row >= 0 && row < rows) thermo[(int64_t)row * 8 + 1] = kin;
            }
        }
        if (MODE != kKickOnly && threadIdx.x == 0) {
            const uint32_t bits = atomicExch(&ctl->maxdisp2, 0u);
            if (__uint_as_float(bits) > thr) ctl->rebuild = 1;
        }
    }
}

__global__ void k_reset_step(Ctl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->step = 0;
}

// State back in caller order.
__global__ void k_gather_out(State st, int64_t n, float *pos, float *vel, float *frc, float *rho,
                             float *drho) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cur = st.ctl->cur;
    const int64_t r = st.id[cur][i];
    const float4 p = st.pos[cur][i], v = st.vel[cur][i], f = st.frc[i];
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

hipError_t launch_integrate(fpm_ctx *c, float dt, int mode, double *thermo, int32_t rows) {
    const unsigned g = (unsigned)((c->n_pad + kBlock - 1) / kBlock);
    if (mode == kKickDriftFirst)
        hipLaunchKernelGGL(k_integrate<kKickDriftFirst>, dim3(g), dim3(kBlock), 0, c->stream,
                           c->st, c->box, c->n, dt, c->disp2_thr, thermo, rows);
    else if (mode == kKickKickDrift)
        hipLaunchKernelGGL(k_integrate<kKickKickDrift>, dim3(g), dim3(kBlock), 0, c->stream,
                           c->st, c->box, c->n, dt, c->disp2_thr, thermo, rows);
    else
        hipLaunchKernelGGL(k_integrate<kKickOnly>, dim3(g), dim3(kBlock), 0, c->stream, c->st,
                           c->box, c->n, dt, c->disp2_thr, thermo, rows);
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
