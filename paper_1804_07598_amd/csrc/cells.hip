// Cell list by counting sort (section 2, ref [45]; the cache-friendly particle
// reordering of section 3.6): cell index -> per-cell histogram -> exclusive
// prefix scan -> scatter -> stable in-cell order -> gather into the other
// ping-pong buffer.  Every kernel reads the device rebuild flag first and
// returns at once when it is clear, so the chain can sit in a static graph.
#include "geom.h"

namespace fpm {
namespace {

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_force_rebuild(Ctl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->rebuild = 1;
}

// Copy the caller's arrays into buffer 0 in caller order, identity ids, and
// zero the control block.
__global__ void k_init_state(State st, int64_t n, int64_t n_pad, const float *pos,
                             const float *vel, const int32_t *type) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        Ctl z = {};
        *st.ctl = z;
    }
    if (i >= n_pad) return;
    float4 p = make_float4(0.f, 0.f, 0.f, 0.f), v = p;
    int32_t t = 0;
    if (i < n) {
        p = make_float4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0.f);
        if (vel) v = make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f);
        if (type) t = type[i];
    }
    p.w = __int_as_float(t);
    st.pos[0][i] = p;
    st.vel[0][i] = v;
    st.pos[1][i] = p;
    st.vel[1][i] = v;
    st.id[0][i] = (int32_t)i;
    st.id[1][i] = (int32_t)i;
    st.frc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    st.xbuild[i] = p;
}

// Density lives in vel.w (caller order before the first build).
__global__ void k_set_density(State st, int64_t n, const float *rho) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cur = st.ctl->cur;
    // slot i holds caller particle id[i]
    int32_t id = st.id[cur][i];
    st.vel[cur][i].w = rho[id];
}

// a2 + a3: wrap, cell index, histogram with the arrival rank kept per particle.
__global__ void k_cell_assign(State st, Box b, int64_t n) {
    const Ctl *ctl = st.ctl;
    if (!ctl->rebuild) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cur = ctl->cur;
    float4 p = st.pos[cur][i];
    if (b.per[0]) p.x = wrap_coord(p.x, b.L[0]);
    if (b.per[1]) p.y = wrap_coord(p.y, b.L[1]);
    if (b.per[2]) p.z = wrap_coord(p.z, b.L[2]);
    st.pos[cur][i] = p;
    int c = cell_of(xyz(p), b);
    st.cid[i] = c;
    st.rnk[i] = atomicAdd(&st.cnt[c], 1);
}

// a4: exclusive scan of the per-cell counts by one workgroup of 1024 threads
// (16 wavefronts).  Each thread owns a contiguous chunk; chunk sums are
// scanned with wavefront shuffles, then across wavefronts through LDS.  The
// counts are cleared on the way for the next rebuild.
__global__ __launch_bounds__(1024) void k_scan(State st, int64_t ncells) {
    Ctl *ctl = st.ctl;
    if (!ctl->rebuild) return;
    __shared__ int32_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t chunk = (ncells + 1023) / 1024;
    const int64_t beg = min((int64_t)t * chunk, ncells), end = min(beg + chunk, ncells);
    int32_t s = 0;
    for (int64_t k = beg; k < end; k++) s += st.cnt[k];
    int32_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    if (w == 0) {
        int32_t v = lane < 16 ? wsum[lane] : 0;
        int32_t x = v;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            int32_t u = __shfl_up(x, o, 64);
            if (lane >= o) x += u;
        }
        if (lane < 16) wsum[lane] = x - v;  // exclusive over wavefronts
    }
    __syncthreads();
    int32_t run = wsum[w] + incl - s;
    for (int64_t k = beg; k < end; k++) {
        int32_t v = st.cnt[k];
        st.off[k] = run;
        run += v;
        st.cnt[k] = 0;
    }
    if (t == 1023) st.off[ncells] = run;
    if (t == 0) {
        ctl->max_count = 0;
        ctl->total_count = 0;
        ctl->overflow = 0;
    }
}

// a5 (first half): scatter (caller id, source slot) to off[c] + arrival rank.
__global__ void k_scatter(State st, int64_t n) {
    const Ctl *ctl = st.ctl;
    if (!ctl->rebuild) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cur = ctl->cur;
    int c = st.cid[i];
    int s = st.off[c] + st.rnk[i];
    st.tmp[s] = make_int2(st.id[cur][i], (int32_t)i);
}

// a5 (second half): the final slot inside the cell is the number of cell
// members with a smaller caller index, which makes the order independent of
// the atomics' arrival order.  Gathers position, velocity and id into the
// other buffer, records the build positions, and flips the buffers.
__global__ void k_rank_gather(State st, int64_t n, int64_t n_pad) {
    Ctl *ctl = st.ctl;
    if (!ctl->rebuild) return;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int cur = ctl->cur, nxt = cur ^ 1;
    if (s < n) {
        int2 me = st.tmp[s];
        int c = st.cid[me.y];
        int beg = st.off[c], end = st.off[c + 1];
        int r = 0;
        for (int k = beg; k < end; k++) r += st.tmp[k].x < me.x;
        int f = beg + r;
        float4 p = st.pos[cur][me.y];
        st.pos[nxt][f] = p;
        st.vel[nxt][f] = st.vel[cur][me.y];
        st.id[nxt][f] = me.x;
        st.xbuild[f] = p;
    } else if (s < n_pad) {
        st.pos[nxt][s] = st.pos[cur][s];
        st.vel[nxt][s] = st.vel[cur][s];
        st.xbuild[s] = st.pos[cur][s];
    }
    if (last_block(&ctl->done[0])) {
        if (threadIdx.x == 0) {
            ctl->cur = nxt;
            ctl->n_rebuilds += 1;
        }
    }
}

// Caller-order cell list for inspection: offsets as is, order = ids.
__global__ void k_cells_out(State st, int64_t n, int64_t ncells, int32_t *offsets,
                            int32_t *order) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int cur = st.ctl->cur;
    if (offsets && i <= ncells) offsets[i] = st.off[i];
    if (order && i < n) order[i] = st.id[cur][i];
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_init_state(fpm_ctx *c, const float *pos, const float *vel, const int32_t *type) {
    hipLaunchKernelGGL(k_init_state, dim3(grid_for(c->n_pad, kBlock)), dim3(kBlock), 0, c->stream,
                       c->st, c->n, c->n_pad, pos, vel, type);
    return hipGetLastError();
}

hipError_t launch_set_density(fpm_ctx *c, const float *rho) {
    hipLaunchKernelGGL(k_set_density, dim3(grid_for(c->n, kBlock)), dim3(kBlock), 0, c->stream,
                       c->st, c->n, rho);
    return hipGetLastError();
}

hipError_t launch_force_rebuild(fpm_ctx *c) {
    hipLaunchKernelGGL(k_force_rebuild, dim3(1), dim3(64), 0, c->stream, c->st.ctl);
    return hipGetLastError();
}

hipError_t launch_cell_build(fpm_ctx *c) {
    const unsigned g = grid_for(c->n_pad, kBlock);
    hipLaunchKernelGGL(k_cell_assign, dim3(g), dim3(kBlock), 0, c->stream, c->st, c->box, c->n);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, c->stream, c->st, c->ncells);
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(kBlock), 0, c->stream, c->st, c->n);
    hipLaunchKernelGGL(k_rank_gather, dim3(g), dim3(kBlock), 0, c->stream, c->st, c->n, c->n_pad);
    return hipGetLastError();
}

hipError_t launch_cells_out(fpm_ctx *c, int32_t *offsets, int32_t *order) {
    int64_t m = c->n > c->ncells + 1 ? c->n : c->ncells + 1;
    hipLaunchKernelGGL(k_cells_out, dim3(grid_for(m, 256)), dim3(256), 0, c->stream, c->st, c->n,
                       c->ncells, offsets, order);
    return hipGetLastError();
}

}  // namespace fpm
