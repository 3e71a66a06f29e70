// Verlet list build (section 2, ref [46]; section 4.1 uses Verlet lists for
// the MD client).  One thread per cell-sorted particle scans the de-duplicated
// 27-cell stencil around its cell and keeps every j != i that passes the FP32
// predicate at the list radius r_cut + skin.  Entries are stored in blocked ELL
// order so that the force kernel reads them coalesced.
#include "geom.h"

namespace fpm {
namespace {

// Neighbour cell coordinates of cell coordinate c along one axis, without
// repeats (grids of one or two cells) and without crossing a closed face.
__device__ __forceinline__ int stencil_axis(int c, int n, int per, int out[3]) {
    int m = 0;
    for (int d = -1; d <= 1; d++) {
        int x = c + d;
        if (per) {
            x = x < 0 ? x + n : (x >= n ? x - n : x);
        } else if (x < 0 || x >= n) {
            continue;
        }
        bool dup = false;
        for (int k = 0; k < m; k++) dup |= (out[k] == x);
        if (!dup) out[m++] = x;
    }
    return m;
}

__global__ __launch_bounds__(kBlock) void k_verlet(State st, Box b, int64_t n, float R2,
                                                   int cap) {
    Ctl *ctl = st.ctl;
    if (!ctl->rebuild) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int cur = ctl->cur;
    const float4 *pos = st.pos[cur];
    int count = 0;
    bool img = false;
    if (i < n) {
        const float3 pi = xyz(pos[i]);
        int cx[3], cy[3], cz[3];
        const int mx = stencil_axis(cell_coord(pi.x, b.inv[0], b.nc[0]), b.nc[0], b.per[0], cx);
        const int my = stencil_axis(cell_coord(pi.y, b.inv[1], b.nc[1]), b.nc[1], b.per[1], cy);
        const int mz = stencil_axis(cell_coord(pi.z, b.inv[2], b.nc[2]), b.nc[2], b.per[2], cz);
        for (int a = 0; a < mx; a++)
            for (int q = 0; q < my; q++)
                for (int r = 0; r < mz; r++) {
                    const int cell = (cx[a] * b.nc[1] + cy[q]) * b.nc[2] + cz[r];
                    const int beg = st.off[cell], end = st.off[cell + 1];
                    for (int j = beg; j < end; j++) {
                        if (j == i) continue;
                        const float3 pj = xyz(pos[j]);
                        if (dist2_pred(pi, pj, b) <= R2) {
                            if (count < cap) st.nbr[ell_index(i, count, cap)] = j;
                            img |= uses_image(pi, pj, b);
                            count++;
                        }
                    }
                }
        st.nnb[i] = (uint32_t)min(count, cap) | (img ? kWrapBit : 0u);
    }
    // list statistics and overflow flag
    int wmax = wave_max_i(count);
    double wsum = wave_sum((double)count);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&ctl->max_count, wmax);
        if (wmax > cap) atomicMax(&ctl->overflow, wmax);
        atomicAdd((unsigned long long *)&ctl->total_count, (unsigned long long)wsum);
    }
    if (last_block(&ctl->done[1])) {
        if (threadIdx.x == 0) ctl->rebuild = 0;
    }
}

// Verlet list in caller indices, row = caller index of the particle.
__global__ void k_neighbors_out(State st, int64_t n, int cap, int32_t *counts, int32_t *cols) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cur = st.ctl->cur;
    const int32_t *id = st.id[cur];
    const int row = id[i];
    const int cnt = (int)(st.nnb[i] & ~kWrapBit);
    counts[row] = cnt;
    for (int k = 0; k < cnt; k++) cols[(int64_t)row * cap + k] = id[st.nbr[ell_index(i, k, cap)]];
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_verlet_build(fpm_ctx *c) {
    hipLaunchKernelGGL(k_verlet, dim3(grid_for(c->n_pad, kBlock)), dim3(kBlock), 0, c->stream,
                       c->st, c->box, c->n, c->R2, c->cap);
    return hipGetLastError();
}

hipError_t launch_neighbors_out(fpm_ctx *c, int32_t *counts, int32_t *cols) {
    hipLaunchKernelGGL(k_neighbors_out, dim3(grid_for(c->n, 256)), dim3(256), 0, c->stream, c->st,
                       c->n, c->cap, counts, cols);
    return hipGetLastError();
}

}  // namespace fpm
