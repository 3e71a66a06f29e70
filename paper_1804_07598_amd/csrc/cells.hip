// Cell list by counting sort (section 2, ref [45]; the cache-friendly particle
// reordering of section 3.6): cell index -> per-cell histogram -> exclusive
// prefix scan -> scatter -> stable in-cell order -> gather into buffer 1.
// Every kernel reads the device rebuild flag first and returns at once when it
// is clear, so the chain can sit in a static graph and run only when needed.
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

// Copy the caller's arrays into both buffers in caller order, identity ids,
// and zero the control block.
__global__ void k_init_state(State st, int64_t n, int64_t n_pad, const float *pos,
                             const float *vel, const int32_t *type) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        Ctl z = {};
        *st.ctl = z;
    }
    if (i >= n_pad) return;
    float4 p = make_float4(kFarAway, kFarAway, kFarAway, 0.f);
    float4 v = make_float4(0.f, 0.f, 0.f, 1.f);
    int32_t t = 0;
    if (i < n) {
        p = make_float4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0.f);
        v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (vel) v = make_float4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.f);
        if (type) t = type[i];
    }
    p.w = __int_as_float(t);
    for (int b = 0; b < 2; b++) {
        st.pos[b][i] = p;
        st.vel[b][i] = v;
        st.id[b][i] = (int32_t)i;
    }
    st.frc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    st.xbuild[i] = p;
    st.nnb[i] = 0;
}

// Density lives in vel.w; slot i holds caller particle id[i].
__global__ void k_set_density(State st, int64_t n, const float *rho) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    st.vel[0][i].w = rho[st.id[0][i]];
}

// Wrap, cell index and histogram, keeping each particle's arrival rank.
// Particles are still nearly in cell order from the previous build, so
// neighbouring lanes mostly share a cell: each run of equal cells inside a
// wavefront issues one atomic add for the whole run.
__global__ __launch_bounds__(kBlock) void k_cell_assign(State st, Box b, int64_t n) {
    if (!st.ctl->rebuild) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int c = -1;
    if (i < n) {
        float4 p = st.pos[0][i];
        if (b.per[0]) p.x = wrap_coord(p.x, b.L[0]);
        if (b.per[1]) p.y = wrap_coord(p.y, b.L[1]);
        if (b.per[2]) p.z = wrap_coord(p.z, b.L[2]);
        st.pos[0][i] = p;
        c = cell_of(xyz(p), b);
        st.cid[i] = c;
    }
    const int prev = __shfl_up(c, 1, 64);
    const bool head = lane == 0 || c != prev;
    const uint64_t heads = __ballot(head);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);  // lanes 0..lane
    const int hl = 63 - __clzll(heads & upto);                       // head of my run
    const uint64_t after = heads & ~upto;
    const int next = after ? __ffsll((long long)after) - 1 : 64;     // first head after me
    int base = 0;
    if (head && c >= 0) base = atomicAdd(&st.cnt[c], next - lane);
    base = __shfl(base, hl, 64);
    if (i < n) st.rnk[i] = base + (lane - hl);
}

// Exclusive prefix scan of the per-cell counts by one workgroup of 1024
// threads, in tiles of 4096 cells loaded as int4 (coalesced).  Inside a tile:
// per-thread sums, wavefront inclusive scan with shuffles, scan of the 16
// wavefront totals, then the carry to the next tile.  Counts are cleared on
// the way for the next rebuild.
__global__ __launch_bounds__(1024) void k_scan(State st, int64_t ncells) {
    if (!st.ctl->rebuild) return;
    __shared__ int32_t wsum[16];
    __shared__ int32_t carry_s;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int32_t carry = 0;
    for (int64_t base = 0; base < ncells; base += 4096) {
        const int64_t k0 = base + 4 * (int64_t)t;
        int4 v = make_int4(0, 0, 0, 0);
        if (k0 + 3 < ncells) {
            v = *reinterpret_cast<const int4 *>(st.cnt + k0);
        } else {
            if (k0 < ncells) v.x = st.cnt[k0];
            if (k0 + 1 < ncells) v.y = st.cnt[k0 + 1];
            if (k0 + 2 < ncells) v.z = st.cnt[k0 + 2];
        }
        const int32_t s = v.x + v.y + v.z + v.w;
        int32_t incl = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int32_t u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        if (w == 0) {
            int32_t x = lane < 16 ? wsum[lane] : 0;
            int32_t y = x;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                int32_t u = __shfl_up(y, o, 64);
                if (lane >= o) y += u;
            }
            if (lane < 16) wsum[lane] = y - x;
            if (lane == 15) carry_s = y;
        }
        __syncthreads();
        int32_t e = carry + wsum[w] + incl - s;
        const int32_t o0 = e, o1 = e + v.x, o2 = o1 + v.y, o3 = o2 + v.z;
        if (k0 + 3 < ncells) {
            *reinterpret_cast<int4 *>(st.off + k0) = make_int4(o0, o1, o2, o3);
            *reinterpret_cast<int4 *>(st.cnt + k0) = make_int4(0, 0, 0, 0);
        } else {
            if (k0 < ncells) { st.off[k0] = o0; st.cnt[k0] = 0; }
            if (k0 + 1 < ncells) { st.off[k0 + 1] = o1; st.cnt[k0 + 1] = 0; }
            if (k0 + 2 < ncells) { st.off[k0 + 2] = o2; st.cnt[k0 + 2] = 0; }
        }
        carry += carry_s;
        __syncthreads();
    }
    if (t == 0) st.off[ncells] = carry;
}

// Scatter (caller id, source slot) to off[c] + arrival rank.
__global__ void k_scatter(State st, int64_t n) {
    if (!st.ctl->rebuild) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = st.cid[i];
    int s = st.off[c] + st.rnk[i];
    st.tmp[s] = make_int2(st.id[0][i], (int32_t)i);
}

// The final slot inside the cell is the number of cell members with a smaller
// caller index, which makes the order independent of the atomics' arrival
// order.  Gathers position, velocity and id into buffer 1 and records the
// build positions.
__global__ void k_rank_gather(State st, int64_t n, int64_t n_pad) {
    if (!st.ctl->rebuild) return;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) {
        int2 me = st.tmp[s];
        int c = st.cid[me.y];
        int beg = st.off[c], end = st.off[c + 1];
        int r = 0;
        for (int k = beg; k < end; k++) r += st.tmp[k].x < me.x;
        int f = beg + r;
        float4 p = st.pos[0][me.y];
        st.pos[1][f] = p;
        st.vel[1][f] = st.vel[0][me.y];
        st.id[1][f] = me.x;
        st.xbuild[f] = p;
    } else if (s < n_pad) {
        st.pos[1][s] = st.pos[0][s];
        st.vel[1][s] = st.vel[0][s];
        st.id[1][s] = st.id[0][s];
        st.xbuild[s] = st.pos[0][s];
    }
}

// Buffer 1 -> buffer 0 (used when the cell list is rebuilt on its own).
__global__ void k_copy_back(State st, int64_t n_pad) {
    if (!st.ctl->rebuild) return;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_pad) return;
    st.pos[0][s] = st.pos[1][s];
    st.vel[0][s] = st.vel[1][s];
    st.id[0][s] = st.id[1][s];
}

// Caller-order view of the cell list: offsets as is, order = ids.
__global__ void k_cells_out(State st, int64_t n, int64_t ncells, int32_t *offsets,
                            int32_t *order) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (offsets && i <= ncells) offsets[i] = st.off[i];
    if (order && i < n) order[i] = st.id[0][i];
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

hipError_t launch_copy_back(fpm_ctx *c) {
    hipLaunchKernelGGL(k_copy_back, dim3(grid_for(c->n_pad, kBlock)), dim3(kBlock), 0, c->stream,
                       c->st, c->n_pad);
    return hipGetLastError();
}

hipError_t launch_cells_out(fpm_ctx *c, int32_t *offsets, int32_t *order) {
    int64_t m = c->n > c->ncells + 1 ? c->n : c->ncells + 1;
    hipLaunchKernelGGL(k_cells_out, dim3(grid_for(m, 256)), dim3(256), 0, c->stream, c->st, c->n,
                       c->ncells, offsets, order);
    return hipGetLastError();
}

}  // namespace fpm
