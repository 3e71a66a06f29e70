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

// The FP32 updates round after every multiply and add (no fused multiply-add),
// so a trajectory is reproducible from its definition operation by operation.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_integrate(State st, float dt) {
#pragma clang fp contract(off)
    const SysDesc &d = st.sys[block_system(st)];
    const int64_t i = global_slot();
    const float h = 0.5f * dt;
    double ke = 0.0, d2 = 0.0;
    if (i - d.slot_base < d.n) {
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
            d2 = dist2_pred(xyz(st.xbuild[i]), xyz(p), d.box);
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

// One workgroup per system reduces that system's per-block partials in a
// fixed order (thread t takes blocks t, t + NT, ... of the slots it needs, all
// loads issued before any is summed; then wavefront shuffles, and one thread
// per slot adds the wavefront results in order) and applies the step's
// control logic (see the kFin* modes).
constexpr int kFinRowsPerThread = 4;

template <int NT>
__global__ __launch_bounds__(NT) void k_finalize(State st, int mode, float thr, double *out,
                                                 double *rows) {
    constexpr int NS = 9;  // U (or VJP 0), W6 (VJP 1..5), KE, displacement
    constexpr int NW = NT / 64;
    __shared__ double red[NW][NS];
    __shared__ double tot[NS];
    const int s = blockIdx.x;
    const SysDesc &d = st.sys[s];
    const int b0 = d.blk_base, nb = d.n_pad / kBlock;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const bool want_f = mode & (kFinForce | kFinVjp), want_k = mode & kFinKE,
               want_d = mode & kFinDisp;
    const double *P = st.part;
    const int64_t S = st.pstride;
    double acc[NS];
#pragma unroll
    for (int c = 0; c < NS; c++) acc[c] = 0.0;
    for (int r0 = t; r0 < nb; r0 += NT * kFinRowsPerThread) {
        double v[kFinRowsPerThread][NS];
#pragma unroll
        for (int q = 0; q < kFinRowsPerThread; q++) {
            const int r = r0 + q * NT;
            const bool ok = r < nb;
#pragma unroll
            for (int c = 0; c < 7; c++) v[q][c] = (want_f && ok) ? P[c * S + b0 + r] : 0.0;
            v[q][7] = (want_k && ok) ? P[kSlotKE * S + b0 + r] : 0.0;
            v[q][8] = (want_d && ok) ? P[kSlotDisp * S + b0 + r] : 0.0;
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
        double x = red[0][t];
        for (int k = 1; k < NW; k++) x = t == 8 ? fmax(x, red[k][t]) : x + red[k][t];
        tot[t] = x;
    }
    __syncthreads();
    if (t != 0) return;
    SysCtl *sc = st.sctl + s;
    if ((mode & kFinBuild) && sc->rebuild[0]) {
        sc->n_rebuilds += 1;
        sc->rebuild[0] = 0;
    }
    if (mode & kFinVjp) {
        if (out)
            for (int c = 0; c < 6; c++) out[(int64_t)s * 6 + c] += tot[c];
        return;
    }
    if (want_f) {
        sc->thermo[0] = tot[kSlotU];
        for (int c = 0; c < 6; c++) sc->thermo[2 + c] = tot[kSlotW + c];
        if (out) {
            out[(int64_t)s * 8] = tot[kSlotU];
            out[(int64_t)s * 8 + 1] = 0.0;
            for (int c = 0; c < 6; c++) out[(int64_t)s * 8 + 2 + c] = tot[kSlotW + c];
        }
    }
    if (want_k) sc->thermo[1] = 0.5 * tot[kSlotKE];
    if (mode & kFinRow) {
        const int row = sc->step;
        if (rows)
            for (int c = 0; c < 8; c++)
                rows[((int64_t)row * st.nsys + s) * 8 + c] = sc->thermo[c];
        sc->step = row + 1;
    }
    if (want_d && tot[8] > (double)thr) sc->rebuild[0] = 1;
}

// Thermo rows of a step loop: workgroup (r, s) reduces ring row r of system s
// (U, W6, KE, per-workgroup partials in block order, then wavefront shuffles
// and the wavefront results in order) into thermo row step - nrows + r, where
// step is the system's step counter after the loop's force kernels (each
// advanced it by one); the last row also becomes the system's thermo.
template <int NT>
__global__ __launch_bounds__(NT) void k_finalize_rows(State st, int nrows, double *rows) {
    constexpr int NS = 8;
    constexpr int NW = NT / 64;
    __shared__ double red[NW][NS];
    const int r = blockIdx.x, s = blockIdx.y;
    const SysDesc &d = st.sys[s];
    const int b0 = d.blk_base, nb = d.n_pad / kBlock;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t S = st.pstride;
    const double *P = st.ring + (int64_t)r * NS * S;
    double acc[NS];
#pragma unroll
    for (int c = 0; c < NS; c++) acc[c] = 0.0;
    for (int r0 = t; r0 < nb; r0 += NT * kFinRowsPerThread) {
        double v[kFinRowsPerThread][NS];
#pragma unroll
        for (int q = 0; q < kFinRowsPerThread; q++) {
            const int k = r0 + q * NT;
#pragma unroll
            for (int c = 0; c < NS; c++) v[q][c] = k < nb ? P[c * S + b0 + k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kFinRowsPerThread; q++)
#pragma unroll
            for (int c = 0; c < NS; c++) acc[c] += v[q][c];
    }
#pragma unroll
    for (int c = 0; c < NS; c++) acc[c] = wave_sum(acc[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NS; c++) red[w][c] = acc[c];
    __syncthreads();
    if (t != 0) return;
    double tot[NS];
    for (int c = 0; c < NS; c++) {
        double x = red[0][c];
        for (int k = 1; k < NW; k++) x += red[k][c];
        tot[c] = x;
    }
    SysCtl *sc = st.sctl + s;
    const double th[8] = {tot[0], 0.5 * tot[7], tot[1], tot[2], tot[3], tot[4], tot[5], tot[6]};
    const int row = sc->step - nrows + r;
    if (rows)
        for (int c = 0; c < 8; c++) rows[((int64_t)row * st.nsys + s) * 8 + c] = th[c];
    if (r == nrows - 1)
        for (int c = 0; c < 8; c++) sc->thermo[c] = th[c];
}

__global__ void k_reset_step(SysCtl *sctl, int nsys) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nsys) sctl[s].step = 0;
}

// New positions in caller order for the current sorted state (type bits and
// the neighbour structures are kept); the displacement since the last build
// decides, as after a drift, whether they must be rebuilt: a wavefront with a
// particle moved by more than half the skin raises the system's rebuild flag
// (one lane, as the step kernel does).  hs: half the skin; thr: its square.
__global__ __launch_bounds__(kBlock) void k_set_positions(State st, const float *pos, float hs,
                                                          float thr) {
    const int sys = block_system(st);
    const SysDesc &d = st.sys[sys];
    const int64_t i = global_slot();
    bool over = false;
    if (i - d.slot_base < d.n) {
        const int64_t r = st.id[0][i];
        float4 p = st.pos[0][i];
        p.x = pos[3 * r];
        p.y = pos[3 * r + 1];
        p.z = pos[3 * r + 2];
        st.pos[0][i] = p;
        const Box &b = d.box;
        over = dist2_pred(xyz(st.xbuild[i]), xyz(p), b) > thr;
        // a position more than half the skin outside [0, L) on a periodic axis
        // (moved by whole periods) forces the rebuild, which wraps it back: the
        // force kernels rely on every position lying within half the skin of
        // [0, L)
        const float c[3] = {p.x, p.y, p.z};
        for (int a = 0; a < 3; a++)
            if (b.per[a] && !(c[a] >= -hs && c[a] < b.L[a] + hs)) over = true;
        if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z)) st.ctl->nonfinite = 1;
    }
    const uint64_t m = __ballot(over);
    if (m && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1) st.sctl[sys].rebuild[0] = 1;
}

// State back in caller order.
__global__ void k_gather_out(State st, float *pos, float *vel, float *frc, float *rho,
                             float *drho) {
    const SysDesc &d = st.sys[block_system(st)];
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
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
    const dim3 g((unsigned)c->nblk), t(kBlock);
    if (mode == kKickDriftFirst)
        hipLaunchKernelGGL(k_integrate<kKickDriftFirst>, g, t, 0, c->stream, c->st, dt);
    else if (mode == kKickKickDrift)
        hipLaunchKernelGGL(k_integrate<kKickKickDrift>, g, t, 0, c->stream, c->st, dt);
    else
        hipLaunchKernelGGL(k_integrate<kKickOnly>, g, t, 0, c->stream, c->st, dt);
    return hipGetLastError();
}

// Largest systems get a full 1024-thread workgroup; batches of small systems
// one wavefront-quad each.
hipError_t launch_finalize(fpm_ctx *c, int mode, double *out, double *rows) {
    if (c->max_sys_blocks > 1024)
        hipLaunchKernelGGL(k_finalize<1024>, dim3(c->nsys), dim3(1024), 0, c->stream, c->st,
                           mode, c->disp2_thr, out, rows);
    else
        hipLaunchKernelGGL(k_finalize<256>, dim3(c->nsys), dim3(256), 0, c->stream, c->st, mode,
                           c->disp2_thr, out, rows);
    return hipGetLastError();
}

hipError_t launch_finalize_rows(fpm_ctx *c, int nrows, double *rows) {
    const dim3 g((unsigned)nrows, (unsigned)c->nsys);
    if (c->max_sys_blocks > 1024)
        hipLaunchKernelGGL(k_finalize_rows<1024>, g, dim3(1024), 0, c->stream, c->st, nrows,
                           rows);
    else
        hipLaunchKernelGGL(k_finalize_rows<256>, g, dim3(256), 0, c->stream, c->st, nrows, rows);
    return hipGetLastError();
}

hipError_t launch_reset_step(fpm_ctx *c) {
    hipLaunchKernelGGL(k_reset_step, dim3((c->nsys + 255) / 256), dim3(256), 0, c->stream,
                       c->st.sctl, c->nsys);
    return hipGetLastError();
}

hipError_t launch_set_positions(fpm_ctx *c, const float *pos) {
    hipLaunchKernelGGL(k_set_positions, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, pos,
                       0.5f * c->skin, c->disp2_thr);
    return hipGetLastError();
}

hipError_t launch_gather_out(fpm_ctx *c, float *pos, float *vel, float *frc, float *rho,
                             float *drho) {
    hipLaunchKernelGGL(k_gather_out, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, pos, vel,
                       frc, rho, drho);
    return hipGetLastError();
}

}  // namespace fpm
