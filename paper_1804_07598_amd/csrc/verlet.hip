// Verlet list build (section 2, ref [46]; section 4.1 uses Verlet lists for
// the MD client).  A particle's list holds every j != i that passes the FP32
// predicate at the list radius r_cut + skin; candidates are the particles of
// the 27 (de-duplicated) cells around its cell.
//
// Main path: a workgroup takes one (x, y) column of cells and a block of zb
// consecutive z-cells.  The z-runs (z0 - 1 .. z1) of the 3 x 3 neighbouring
// columns are staged in LDS, each column contiguous and in z order, with the
// global slot kept in w, so that a particle's stencil is nine contiguous LDS
// ranges.  Candidates are tested in chunks of 32; hits are collected in a bit
// mask and written after the chunk, which takes far fewer store instructions
// than storing inside the test loop.  The kernel also moves the freshly
// sorted state from buffer 1 back to buffer 0.
//
// Fallback: grids with fewer than three cells along an axis (and workgroups
// whose staged region would not fit) read candidates from global memory.
#include "geom.h"

namespace fpm {
namespace {

constexpr int kColThreads = 128;  // threads of a column workgroup
constexpr int kLdsAtoms = 2048;   // staged positions per column workgroup (32 KiB)
constexpr int kMaxZb = 32;        // z-cells per workgroup, at most

// Neighbour cell coordinates of c along one axis, ascending, without repeats
// (grids of one or two cells) and without crossing a closed face.
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
    for (int a = 0; a < m; a++)
        for (int k = a + 1; k < m; k++)
            if (out[k] < out[a]) {
                int t = out[a];
                out[a] = out[k];
                out[k] = t;
            }
    return m;
}

// Branch-free form of the predicate's image choice on one axis (same
// arithmetic as img_delta: each candidate's operations round identically).
__device__ __forceinline__ float img_delta_sel(float xi, float xj, float L, float half, int per) {
#pragma clang fp contract(off)
    const float t = xj - xi;
    const float s1 = xj - L;
    const float s2 = xi - L;
    const float a1 = s1 - xi;  // t > L/2: (xj - L) - xi
    const float a2 = xj - s2;  // t < -L/2: xj - (xi - L)
    const float r = t > half ? a1 : (t < -half ? a2 : t);
    return per ? r : t;
}

template <bool IMG>
__device__ __forceinline__ float cand_d2(float3 pi, float3 pj, const Box &b) {
#pragma clang fp contract(off)
    if (!IMG) return dist2_direct(pi, pj);
    const float dx = img_delta_sel(pi.x, pj.x, b.L[0], b.half[0], b.per[0]);
    const float dy = img_delta_sel(pi.y, pj.y, b.L[1], b.half[1], b.per[1]);
    const float dz = img_delta_sel(pi.z, pj.z, b.L[2], b.half[2], b.per[2]);
    const float xx = dx * dx;
    const float yy = dy * dy;
    const float zz = dz * dz;
    const float s = xx + yy;
    return s + zz;
}

// Where list entry k of a slot goes, relative to the slot's entry 0.
__device__ __forceinline__ int ell_off(int k) { return ((k & ~3) << 6) | (k & 3); }

// Fills entries count .. (count rounded up to 8) with the far-away padding
// slot, so that list readers can consume whole groups of eight.
__device__ __forceinline__ void pad_list(int32_t *__restrict__ wp, int count, int cap,
                                         int dummy) {
    const int c = min(count, cap);
    const int c8 = (c + 7) & ~7;
    for (int k = c; k < c8; k++) wp[ell_off(k)] = dummy;
}

// Tests candidates [beg, end) of `src` (global slots) or of the LDS stage
// (global slot in w, lower-face images already shifted) against particle i and
// appends the hits.
template <bool IMG, bool LDS>
__device__ __forceinline__ void scan_range(const float4 *__restrict__ src, int beg, int end,
                                           int i, float3 pi, const Box &b, float R2,
                                           int32_t *__restrict__ wp, int cap, int &count,
                                           bool &img) {
    for (int c0 = beg; c0 < end; c0 += 32) {
        const int len = min(32, end - c0);
        uint32_t mask = 0;
#pragma unroll 4
        for (int u = 0; u < len; u++) {
            const float4 q = src[c0 + u];
            const int gj = LDS ? __float_as_int(q.w) : c0 + u;
            const bool hit = cand_d2<IMG>(pi, xyz(q), b) <= R2 && gj != i;
            mask |= (uint32_t)hit << u;
            if (IMG) img |= hit && uses_image(pi, xyz(q), b);
        }
        while (mask) {
            const int u = __ffs(mask) - 1;
            mask &= mask - 1;
            const int gj = LDS ? __float_as_int(src[c0 + u].w) : c0 + u;
            if (count < cap) wp[ell_off(count)] = gj;
            count++;
        }
    }
}

// True when some stencil cell of cell (ix, iy, iz) lies across a periodic face.
__device__ __forceinline__ bool near_face(int ix, int iy, int iz, const Box &b) {
    return (b.per[0] && (ix == 0 || ix == b.nc[0] - 1)) ||
           (b.per[1] && (iy == 0 || iy == b.nc[1] - 1)) ||
           (b.per[2] && (iz == 0 || iz == b.nc[2] - 1));
}

// List of slot i from global memory through the cell offsets.
template <bool IMG>
__device__ void verlet_atom_global(const State &st, const SysDesc &d, int i, float3 pi,
                                   float R2, int cap, int cap4, int &count, bool &img) {
    const Box &b = d.box;
    const float4 *__restrict__ pos = st.pos[1];
    const int32_t *__restrict__ off = st.off + d.off_base;
    int32_t *wp = st.nbr + nbr_index(i, 0, cap4);
    const int ix = cell_coord(pi.x, b.inv[0], b.nc[0]);
    const int iy = cell_coord(pi.y, b.inv[1], b.nc[1]);
    const int iz = cell_coord(pi.z, b.inv[2], b.nc[2]);
    int cx[3], cy[3], cz[3];
    const int mx = stencil_axis(ix, b.nc[0], b.per[0], cx);
    const int my = stencil_axis(iy, b.nc[1], b.per[1], cy);
    const int mz = stencil_axis(iz, b.nc[2], b.per[2], cz);
    for (int a = 0; a < mx; a++)
        for (int q = 0; q < my; q++) {
            const int col = (cx[a] * b.nc[1] + cy[q]) * b.nc[2];
            int r = 0;
            while (r < mz) {
                int r1 = r;
                while (r1 + 1 < mz && cz[r1 + 1] == cz[r1] + 1) r1++;
                const int beg = off[col + cz[r]], end = off[col + cz[r1] + 1];
                scan_range<IMG, false>(pos, beg, end, i, pi, b, R2, wp, cap, count, img);
                r = r1 + 1;
            }
        }
    pad_list(wp, count, cap, d.dummy);
}

// A list longer than the capacity raises the sticky overflow flag (any of the
// overflowing lengths is kept; the lists are invalid until rebuilt).
__device__ __forceinline__ void note_overflow(const State &st, int count, int cap) {
    if (count > cap) st.ctl->overflow = count;
}

__device__ __forceinline__ void copy_back(const State &st, int64_t s) {
    st.pos[0][s] = st.pos[1][s];
    st.vel[0][s] = st.vel[1][s];
    st.id[0][s] = st.id[1][s];
}

// One thread per particle, candidates read from global memory.  The grid
// runs over the list of particle workgroups of the systems built this way.
__global__ __launch_bounds__(kBlock) void k_verlet(State st, const int32_t *blocks, float R2,
                                                   int cap, int cap4) {
    const int blk = blocks[blockIdx.x];
    const int s = st.blk2sys[blk];
    if (!st.sctl[s].rebuild) return;
    const SysDesc &d = st.sys[s];
    const Box b = d.box;
    const int64_t i = (int64_t)blk * kBlock + threadIdx.x;
    const bool active = i - d.slot_base < d.n;
    int count = 0;
    bool img = false, face = false;
    float3 pi = make_float3(0.f, 0.f, 0.f);
    if (active) {
        pi = xyz(st.pos[1][i]);
        face = near_face(cell_coord(pi.x, b.inv[0], b.nc[0]), cell_coord(pi.y, b.inv[1], b.nc[1]),
                         cell_coord(pi.z, b.inv[2], b.nc[2]), b);
    }
    const bool face_wave = __ballot(face) != 0;
    if (active) {
        if (face_wave)
            verlet_atom_global<true>(st, d, (int)i, pi, R2, cap, cap4, count, img);
        else
            verlet_atom_global<false>(st, d, (int)i, pi, R2, cap, cap4, count, img);
        st.nnb[i] = (uint32_t)min(count, cap) | (img ? kWrapBit : 0u);
        note_overflow(st, count, cap);
    }
    copy_back(st, i);
}

// Column workgroups (see the file comment); one work item per (system,
// column, z-block).
__global__ __launch_bounds__(kColThreads) void k_verlet_cols(State st, float R2, int cap,
                                                             int cap4) {
    const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);  // consecutive columns per XCD
    const int s = st.item2sys[lb];
    if (!st.sctl[s].rebuild) return;
    const SysDesc &d = st.sys[s];
    const Box b = d.box;
    const int zb = d.zb, nzb = d.nzb;
    const int32_t *__restrict__ off = st.off + d.off_base;
    __shared__ float4 sp[kLdsAtoms];
    __shared__ int cs[9][kMaxZb + 3];  // column-relative LDS start of run cell m (m = nrun: end)
    __shared__ int seg[9][3][2];       // (global start, length) of the three run segments
    __shared__ float sh[9][3][3];      // image shift (x, y, z) of each segment
    __shared__ int colbase[10];
    const float4 *__restrict__ pos = st.pos[1];
    const int nx = b.nc[0], ny = b.nc[1], nz = b.nc[2];
    const int item = lb - d.item_base;
    const int zblk = item % nzb, colid = item / nzb;
    const int ix = colid / ny, iy = colid % ny;
    const int z0 = zblk * zb, z1 = min(z0 + zb, nz);
    const int nrun = z1 - z0 + 2;
    const int cell0 = (ix * ny + iy) * nz;
    const int abeg = off[cell0 + z0], aend = off[cell0 + z1];

    if (threadIdx.x < 9) {
        const int k = threadIdx.x;
        int cx = ix + k / 3 - 1, cy = iy + k % 3 - 1;
        float sx = 0.f, sy = 0.f;  // shift of a column across a periodic face
        bool ok = true;
        if (cx < 0 || cx >= nx) {
            if (b.per[0]) {
                sx = cx < 0 ? -b.L[0] : b.L[0];
                cx = cx < 0 ? cx + nx : cx - nx;
            } else {
                ok = false;
            }
        }
        if (cy < 0 || cy >= ny) {
            if (b.per[1]) {
                sy = cy < 0 ? -b.L[1] : b.L[1];
                cy = cy < 0 ? cy + ny : cy - ny;
            } else {
                ok = false;
            }
        }
        const int col = (cx * ny + cy) * nz;
        int acc = 0;
        for (int sg = 0; sg < 3; sg++) {
            seg[k][sg][1] = 0;
            sh[k][sg][0] = sx;
            sh[k][sg][1] = sy;
            sh[k][sg][2] = 0.f;
        }
        for (int m = 0; m < nrun; m++) {
            int z = z0 - 1 + m;
            bool okz = ok;
            float sz = 0.f;
            if (z < 0 || z >= nz) {
                if (b.per[2]) {
                    sz = z < 0 ? -b.L[2] : b.L[2];
                    z = z < 0 ? z + nz : z - nz;
                } else {
                    okz = false;
                }
            }
            int gs = 0, len = 0;
            if (okz) {
                gs = off[col + z];
                len = off[col + z + 1] - gs;
            }
            cs[k][m] = acc;
            const int sg = m == 0 ? 0 : (m == nrun - 1 ? 2 : 1);
            if (m <= 1 || m == nrun - 1) {  // the middle segment starts at its first cell
                seg[k][sg][0] = gs;
                sh[k][sg][2] = sz;
            }
            seg[k][sg][1] += len;
            acc += len;
        }
        cs[k][nrun] = acc;
        colbase[k + 1] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        colbase[0] = 0;
        for (int k = 0; k < 9; k++) colbase[k + 1] += colbase[k];
    }
    __syncthreads();
    const bool use_lds = colbase[9] <= kLdsAtoms;
    if (use_lds) {
        // Periodic images as the predicate takes them: the coordinate in the
        // upper half of the box moves down one period (exact).  Cells staged
        // from across the lower face lie at the top of the box and are stored
        // shifted down; cells from across the upper face are stored as they
        // are, and the scan shifts particle i down instead.
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int q = w; q < 27; q += kColThreads / 64) {
            const int k = q / 3, sg = q % 3;
            const int gs = seg[k][sg][0], len = seg[k][sg][1];
            const int ls = colbase[k] + (sg == 0 ? 0 : (sg == 1 ? cs[k][1] : cs[k][nrun - 1]));
            const float sx = fminf(sh[k][sg][0], 0.f), sy = fminf(sh[k][sg][1], 0.f),
                        sz = fminf(sh[k][sg][2], 0.f);
            for (int t = lane; t < len; t += 64) {
                float4 p = pos[gs + t];
                p.x = p.x + sx;
                p.y = p.y + sy;
                p.z = p.z + sz;
                p.w = __int_as_float(gs + t);
                sp[ls + t] = p;
            }
        }
    }
    __syncthreads();

    for (int base = abeg; base < aend; base += kColThreads) {
        const int i = base + (int)threadIdx.x;
        const bool active = i < aend;
        int count = 0;
        bool img = false, face = false;
        int m = 1;
        float3 pi = make_float3(0.f, 0.f, 0.f);
        if (active) {
            pi = xyz(pos[i]);
            const int iz = cell_coord(pi.z, b.inv[2], nz);
            m = min(max(iz - z0 + 1, 1), nrun - 2);  // iz lies in [z0, z1) by construction
            face = near_face(ix, iy, iz, b);
        }
        const bool face_wave = __ballot(face) != 0;
        if (active) {
            int32_t *wp = st.nbr + nbr_index(i, 0, cap4);
            if (use_lds) {
                // the run's last cell is cell 0 one period up when z1 wraps; only
                // particles of the top z-cell (m + 2 == nrun) reach it
                const bool top_img = b.per[2] && z1 == nz;
                for (int k = 0; k < 9; k++) {
                    float3 pk = pi;  // i moved down one period where column k lies across
                    if (sh[k][1][0] > 0.f) pk.x = pi.x - b.L[0];  // the upper face (exact:
                    if (sh[k][1][1] > 0.f) pk.y = pi.y - b.L[1];  // i is in the top cell)
                    const int beg = colbase[k] + cs[k][m - 1], end = colbase[k] + cs[k][m + 2];
                    const int mid = m + 2 == nrun ? colbase[k] + cs[k][nrun - 1] : end;
                    scan_range<false, true>(sp, beg, mid, i, pk, b, R2, wp, cap, count, img);
                    if (top_img) pk.z = pi.z - b.L[2];
                    scan_range<false, true>(sp, mid, end, i, pk, b, R2, wp, cap, count, img);
                }
                pad_list(wp, count, cap, d.dummy);
                img = face;  // its stencil reaches across a periodic face
            } else if (face_wave) {
                verlet_atom_global<true>(st, d, i, pi, R2, cap, cap4, count, img);
            } else {
                verlet_atom_global<false>(st, d, i, pi, R2, cap, cap4, count, img);
            }
            st.nnb[i] = (uint32_t)min(count, cap) | (img ? kWrapBit : 0u);
            note_overflow(st, count, cap);
            copy_back(st, i);
        }
    }
    // padding slots are in no cell: the system's first work item moves them back
    if (item == 0)
        for (int64_t q = d.slot_base + d.n + threadIdx.x; q < d.slot_base + d.n_pad;
             q += kColThreads)
            copy_back(st, q);
}

// Longest list and total entries of the current lists (on request only).
__global__ void k_list_stats(State st, int64_t nslots) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int c = i < nslots ? (int)(st.nnb[i] & ~kWrapBit) : 0;
    int mx = c;
    unsigned long long sm = (unsigned long long)c;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, __shfl_xor(mx, o, 64));
        sm += __shfl_xor(sm, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&st.ctl->max_count, mx);
        atomicAdd((unsigned long long *)&st.ctl->total_count, sm);
    }
}

__global__ void k_zero_stats(Ctl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->max_count = 0;
        ctl->total_count = 0;
    }
}

// Verlet lists in caller indices, row = caller index of the particle.
__global__ void k_neighbors_out(State st, int cap, int cap4, int32_t *counts, int32_t *cols) {
    const SysDesc &d = st.sys[block_system(st)];
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
    const int32_t *id = st.id[0];
    const int row = id[i];
    const int cnt = (int)(st.nnb[i] & ~kWrapBit);
    counts[row] = cnt;
    for (int k = 0; k < cnt; k++) cols[(int64_t)row * cap + k] = id[st.nbr[nbr_index(i, k, cap4)]];
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_verlet_build(fpm_ctx *c) {
    if (c->nitems > 0)
        hipLaunchKernelGGL(k_verlet_cols, dim3(c->nitems), dim3(kColThreads), 0, c->stream,
                           c->st, c->R2, c->cap, c->cap4);
    if (c->n_pa_blocks > 0)
        hipLaunchKernelGGL(k_verlet, dim3(c->n_pa_blocks), dim3(kBlock), 0, c->stream, c->st,
                           c->pa_blocks, c->R2, c->cap, c->cap4);
    return hipGetLastError();
}

hipError_t launch_list_stats(fpm_ctx *c) {
    hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(64), 0, c->stream, c->st.ctl);
    hipLaunchKernelGGL(k_list_stats, dim3(grid_for(c->n_slots, 256)), dim3(256), 0, c->stream,
                       c->st, c->n_slots);
    return hipGetLastError();
}

hipError_t launch_neighbors_out(fpm_ctx *c, int32_t *counts, int32_t *cols) {
    hipLaunchKernelGGL(k_neighbors_out, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, c->cap,
                       c->cap4, counts, cols);
    return hipGetLastError();
}

int verlet_zblock(int64_t n, int64_t ncells, const int nc[3], int tune_zb) {
    if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3) return 0;
    if (tune_zb > 0) return tune_zb > kMaxZb ? kMaxZb : (tune_zb > nc[2] - 2 ? nc[2] - 2 : tune_zb);
    const double avg = (double)n / (double)ncells;
    // aim at ~1400 staged particles (70% of the LDS stage) and ~100 per workgroup
    int zb = (int)(1400.0 / (9.0 * (avg > 0.05 ? avg : 0.05))) - 2;
    zb = zb < 1 ? 1 : zb;
    zb = zb > kMaxZb ? kMaxZb : zb;
    zb = zb > nc[2] - 2 ? nc[2] - 2 : zb;
    return zb;
}

}  // namespace fpm
