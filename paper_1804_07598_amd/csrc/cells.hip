// Cell list by counting sort (section 2, ref [45]; the cache-friendly particle
// reordering of section 3.6): cell index -> per-cell histogram -> exclusive
// prefix scan -> scatter -> stable in-cell order -> gather into buffer 1.
// Every kernel reads its system's rebuild flag first and returns at once when
// it is clear, so the chain can sit in a static graph and run only when and
// where needed.
#include "geom.h"

namespace fpm {
namespace {

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_force_rebuild(SysCtl *sctl, int nsys) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nsys) sctl[s].rebuild[0] = 1;
}

__global__ void k_init_ctl(Ctl *ctl, SysCtl *sctl, int nsys) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) {
        Ctl z = {};
        *ctl = z;
    }
    if (s < nsys) {
        SysCtl z = {};
        sctl[s] = z;
    }
}

// Copy the caller's arrays into both buffers in caller order (system by
// system), identity ids; padding slots are parked far away.
__global__ void k_init_state(State st, const float *pos, const float *vel, const int32_t *type) {
    const SysDesc &d = st.sys[block_system(st)];
    const int64_t i = global_slot();
    const int64_t local = i - d.slot_base;
    float4 p = make_float4(kFarAway, kFarAway, kFarAway, 0.f);
    float4 v = make_float4(0.f, 0.f, 0.f, 1.f);
    int32_t t = 0, id = -1;
    if (local < d.n) {
        const int64_t r = d.caller_base + local;
        p = make_float4(pos[3 * r], pos[3 * r + 1], pos[3 * r + 2], 0.f);
        v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (vel) v = make_float4(vel[3 * r], vel[3 * r + 1], vel[3 * r + 2], 0.f);
        if (type) t = type[r];
        id = (int32_t)r;
    }
    p.w = __int_as_float(t);
    for (int b = 0; b < 2; b++) {
        st.pos[b][i] = p;
        st.vel[b][i] = v;
        st.id[b][i] = id;
    }
    st.frc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    st.xbuild[i] = p;
    st.nnb[i] = 0;
}

// Density lives in vel.w; slot i holds caller particle id[i].
__global__ void k_set_density(State st, const float *rho) {
    const SysDesc &d = st.sys[block_system(st)];
    const int64_t i = global_slot();
    if (i - d.slot_base < d.n) st.vel[0][i].w = rho[st.id[0][i]];
}

// Wrap, cell index and histogram (gated).
__global__ __launch_bounds__(kBlock) void k_cell_assign(State st) {
    const int s = block_system(st);
    if (!rebuilding(st, s)) return;
    cell_assign_slot(st, s, global_slot());
}

// Exclusive scan of one tile of kScanTile values in[base ..) (n values in
// all) into out[] with `carry` added, by a workgroup of 1024 threads:
// per-thread sums of four, wavefront inclusive scan with shuffles, scan of the
// 16 wavefront totals.  `in` may alias `out`; with `clear` the inputs are
// zeroed.  Returns the tile's total to every thread.
constexpr int kScanTile = 4096;

// The eighth-of-cell table of system d, which only the lockstep Verlet build
// reads (null for systems built another way).
__device__ __forceinline__ int32_t *eighths(const State &st, const SysDesc &d) {
    return d.zb == -4 || d.zb == -5 ? st.sub + (int64_t)d.cell_base * 8 : nullptr;
}
constexpr int64_t kScanDeviceCells = 16384;  // a single system with more cells scans device-wide

__device__ __forceinline__ int32_t scan_tile(int32_t *in, int32_t *out, int64_t base, int64_t n,
                                             int32_t carry, bool clear, int32_t *sub) {
    __shared__ int32_t wsum[16];
    __shared__ int32_t total;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t k0 = base + 4 * (int64_t)t;
    int32_t v[4];
#pragma unroll
    for (int q = 0; q < 4; q++) v[q] = k0 + q < n ? in[k0 + q] : 0;
    const int32_t sum = v[0] + v[1] + v[2] + v[3];
    int32_t incl = sum;
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
        if (lane == 15) total = y;
    }
    __syncthreads();
    int32_t e = carry + wsum[w] + incl - sum;
#pragma unroll
    for (int q = 0; q < 4; q++)
        if (k0 + q < n) {
            out[k0 + q] = e;
            // an empty cell's eighths all start at its offset (the gather writes
            // the table of every other cell)
            if (sub && v[q] == 0)
                for (int h = 0; h < 8; h++) sub[(k0 + q) * 8 + h] = e;
            e += v[q];
            if (clear) in[k0 + q] = 0;
        }
    const int32_t tot = total;
    __syncthreads();  // wsum and total are reused by the next tile
    return tot;
}

// Exclusive prefix scan of each system's cell counts, one workgroup per
// system walking its tiles in order.  Offsets are global slots.  Counts are
// cleared on the way for the next rebuild.
__global__ __launch_bounds__(1024) void k_scan(State st) {
    const int s = blockIdx.x;
    if (!rebuilding(st, s)) return;
    const SysDesc &d = st.sys[s];
    int32_t *cnt = st.cnt + d.cell_base;
    int32_t *off = st.off + d.off_base;
    const int64_t ncells = d.ncells;
    int32_t carry = d.slot_base;
    for (int64_t base = 0; base < ncells; base += kScanTile)
        carry += scan_tile(cnt, off, base, ncells, carry, true, eighths(st, d));
    if (threadIdx.x == 0) off[ncells] = carry;
}

// The same scan for a single system with many cells, over the whole device:
// tile totals (one workgroup per tile), then each tile's scan from its carry.
__global__ __launch_bounds__(1024) void k_scan_sums(State st) {
    if (!rebuilding(st, 0)) return;
    const SysDesc &d = st.sys[0];
    const int32_t *cnt = st.cnt + d.cell_base;
    const int64_t k0 = (int64_t)blockIdx.x * kScanTile + 4 * (int64_t)threadIdx.x;
    int32_t v = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) v += k0 + q < d.ncells ? cnt[k0 + q] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __shared__ int32_t wsum[16];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < 16; w++) t += wsum[w];
        st.tsum[blockIdx.x] = t;
    }
}

// Each tile's workgroup adds up the totals of the tiles before it for its
// carry (integer sums, so the order does not matter); the last tile also
// writes the end offset.
__global__ __launch_bounds__(1024) void k_scan_tiles(State st) {
    if (!rebuilding(st, 0)) return;
    const SysDesc &d = st.sys[0];
    const int b = blockIdx.x, t = threadIdx.x;
    __shared__ int32_t part[16];
    int32_t v = 0;
    for (int k = t; k < b; k += 1024) v += st.tsum[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((t & 63) == 0) part[t >> 6] = v;
    __syncthreads();
    int32_t carry = d.slot_base;
#pragma unroll
    for (int w = 0; w < 16; w++) carry += part[w];
    const int32_t tot = scan_tile(st.cnt + d.cell_base, st.off + d.off_base,
                                  (int64_t)b * kScanTile, d.ncells, carry, true, eighths(st, d));
    if (b == (int)gridDim.x - 1 && t == 0) st.off[d.off_base + d.ncells] = carry + tot;
}

// Scatter (caller id, source slot, z, cell) to the cell's offset + arrival rank.
__global__ void k_scatter(State st) {
    const int s = block_system(st);
    if (!rebuilding(st, s)) return;
    const SysDesc &d = st.sys[s];
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
    const int c = st.cid[i];
    const int slot = st.off[off_index(d, c)] + st.rnk[i];
    st.tmp[slot] = make_int4(st.id[0][i], (int32_t)i, __float_as_int(st.pos[0][i].z), c);
}

// The final slot inside the cell is the number of cell members that come
// before it in (z, caller index) order, which makes the order independent of
// the atomics' arrival order and every column of cells one run sorted by z.
// Gathers position, velocity and id into buffer 1 and records the build
// positions.  Each member also writes the eighth-of-cell table entries that
// start at its slot (the eighths after its predecessor's, up to its own; the
// last member closes the cell).  The members that lie in the workgroup's
// own slots are read from LDS.
__global__ __launch_bounds__(kBlock) void k_rank_gather(State st) {
    __shared__ int4 stage[kBlock];
    const int s = block_system(st);
    if (!rebuilding(st, s)) return;  // the whole workgroup
    const SysDesc &d = st.sys[s];
    const int64_t i = global_slot();
    const int lo = (int)(i - threadIdx.x);  // the workgroup's first slot
    const bool member = i - d.slot_base < d.n;
    const int4 me = member ? st.tmp[i] : make_int4(0, 0, 0, 0);
    stage[threadIdx.x] = me;
    __syncthreads();
    if (member) {
        const float mz = __int_as_float(me.z);
        const int c = me.w;
        const int beg = st.off[off_index(d, c)], end = st.off[off_index(d, c) + 1];
        int r = 0;
        float zprev = -INFINITY;
        auto count = [&](int4 o) {
            const float oz = __int_as_float(o.z);
            const bool before = oz < mz || (oz == mz && o.x < me.x);
            r += before;
            zprev = before ? fmaxf(zprev, oz) : zprev;
        };
        // [sb, se): the cell's members among this workgroup's slots (i is one)
        const int sb = max(beg, lo), se = min(end, lo + kBlock);
        for (int k = beg; k < sb; k++) count(st.tmp[k]);
        for (int k = sb; k < se; k++) count(stage[k - lo]);
        for (int k = se; k < end; k++) count(st.tmp[k]);
        const int f = beg + r;
        if (d.zb == -4 || d.zb == -5) {
            const int nz = d.box.nc[2];
            const int iz = (c - d.cell_base) % nz;
            const float inv = d.box.inv[2];
            const int e = z_eighth(mz, inv, iz);
            const int e0 = r == 0 ? 0 : z_eighth(zprev, inv, iz) + 1;
            int32_t *sub = st.sub + (int64_t)c * 8;
            for (int h = e0; h <= e; h++) sub[h] = f;
            if (f == end - 1)
                for (int h = e + 1; h < 8; h++) sub[h] = end;
        }
        const float4 p = st.pos[0][me.y];
        st.pos[1][f] = p;
        st.vel[1][f] = st.vel[0][me.y];
        st.id[1][f] = me.x;
        st.xbuild[f] = p;
        if (st.keep_old) st.old[1][f] = st.old[0][me.y];
    } else {
        st.pos[1][i] = st.pos[0][i];
        st.vel[1][i] = st.vel[0][i];
        st.id[1][i] = st.id[0][i];
        st.xbuild[i] = st.pos[0][i];
        if (st.keep_old) st.old[1][i] = st.old[0][i];
    }
}

// Debug builds: after a cell build every sorted slot of a system lies in the
// offset range of the cell its position falls in, and the system's offsets
// run from its first slot to its first slot plus its particle count.
__global__ __launch_bounds__(kBlock) void k_check_cells(State st) {
    const int s = block_system(st);
    if (!rebuilding(st, s)) return;
    const SysDesc &d = st.sys[s];
    const int64_t f = global_slot();
    if (f - d.slot_base >= d.n) return;
    const int c = d.cell_base + cell_of(xyz(st.pos[1][f]), d.box);
    const int lo = st.off[off_index(d, c)], hi = st.off[off_index(d, c) + 1];
    bool bad = f < lo || f >= hi;
    if (f == d.slot_base)
        bad = bad || st.off[d.off_base] != d.slot_base ||
              st.off[d.off_base + d.ncells] != d.slot_base + d.n;
    if (bad) st.ctl->bad_index = 1;
}

// Buffer 1 -> buffer 0 (used when the cell list is rebuilt on its own).
__global__ void k_copy_back(State st) {
    if (!rebuilding(st, block_system(st))) return;
    const int64_t i = global_slot();
    st.pos[0][i] = st.pos[1][i];
    st.vel[0][i] = st.vel[1][i];
    st.id[0][i] = st.id[1][i];
    if (st.keep_old) st.old[0][i] = st.old[1][i];
}

// Caller-order view of the cell lists: offsets renumbered into the packed
// caller numbering (no padding slots), order[k] = caller index at packed k.
__global__ void k_cells_out(State st, int32_t *offsets, int32_t *order) {
    const int s = block_system(st);
    const SysDesc &d = st.sys[s];
    const int64_t i = global_slot();
    const int64_t local = i - d.slot_base;
    if (order && local < d.n) order[d.caller_base + local] = st.id[0][i];
    if (offsets) {
        // the system's first workgroup writes its ncells + 1 offsets
        if (pblock() != d.blk_base) return;
        for (int c = threadIdx.x; c <= d.ncells; c += blockDim.x)
            offsets[d.off_base + c] = st.off[d.off_base + c] - d.slot_base + d.caller_base;
    }
}

inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_init_state(fpm_ctx *c, const float *pos, const float *vel, const int32_t *type) {
    hipLaunchKernelGGL(k_init_ctl, dim3(grid_for(c->nsys, 256)), dim3(256), 0, c->stream,
                       c->st.ctl, c->st.sctl, c->nsys);
    hipLaunchKernelGGL(k_init_state, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, pos, vel,
                       type);
    return hipGetLastError();
}

hipError_t launch_set_density(fpm_ctx *c, const float *rho) {
    hipLaunchKernelGGL(k_set_density, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, rho);
    return hipGetLastError();
}

hipError_t launch_force_rebuild(fpm_ctx *c) {
    hipLaunchKernelGGL(k_force_rebuild, dim3(grid_for(c->nsys, 256)), dim3(256), 0, c->stream,
                       c->st.sctl, c->nsys);
    return hipGetLastError();
}

hipError_t launch_cell_build(fpm_ctx *c, bool dem_export) {
    const unsigned g = (unsigned)c->nblk;
    if (dem_export) {
        const hipError_t e = launch_dem_export_assign(c);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_cell_assign, dim3(g), dim3(kBlock), 0, c->stream, c->st);
    }
    const int64_t nc0 = c->sys[0].d.ncells;
    if (c->nsys == 1 && nc0 > kScanDeviceCells) {
        const unsigned nt = (unsigned)((nc0 + kScanTile - 1) / kScanTile);
        hipLaunchKernelGGL(k_scan_sums, dim3(nt), dim3(1024), 0, c->stream, c->st);
        hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(1024), 0, c->stream, c->st);
    } else {
        hipLaunchKernelGGL(k_scan, dim3(c->nsys), dim3(1024), 0, c->stream, c->st);
    }
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(kBlock), 0, c->stream, c->st);
    hipLaunchKernelGGL(k_rank_gather, dim3(g), dim3(kBlock), 0, c->stream, c->st);
    if (kChecked) return launch_check_cells(c);
    return hipGetLastError();
}

hipError_t launch_check_cells(fpm_ctx *c) {
    hipLaunchKernelGGL(k_check_cells, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st);
    return hipGetLastError();
}

hipError_t launch_copy_back(fpm_ctx *c) {
    hipLaunchKernelGGL(k_copy_back, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st);
    return hipGetLastError();
}

hipError_t launch_cells_out(fpm_ctx *c, int32_t *offsets, int32_t *order) {
    hipLaunchKernelGGL(k_cells_out, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, offsets,
                       order);
    return hipGetLastError();
}

}  // namespace fpm
