// Device helpers shared by the kernels: the FP32 neighbour predicate, periodic
// images, cell coordinates, and wavefront/workgroup reductions.
#pragma once

#include "fpm_internal.h"

namespace fpm {

// One coordinate difference of the FP32 neighbour predicate (header of fpm.h):
// t = xj - xi; on a periodic axis t > L/2 selects the image (xj - L) - xi and
// t < -L/2 the image xj - (xi - L): the coordinate in the upper half of the
// box moves down one period, which is exact, so the image separation is
// rounded once and is the exact negative of the (j, i) separation.  Every
// operation rounds separately.
__device__ __forceinline__ float img_delta(float xi, float xj, float L, float half, int per) {
#pragma clang fp contract(off)
    float t = xj - xi;
    if (per) {
        if (t > half) {
            float s = xj - L;
            t = s - xi;
        } else if (t < -half) {
            float s = xi - L;
            t = xj - s;
        }
    }
    return t;
}

// Image shift of j as seen from i on one axis: -1, 0 or +1 periods.
__device__ __forceinline__ int img_shift(float xi, float xj, float half, int per) {
    const float t = xj - xi;
    return per ? (t > half ? -1 : (t < -half ? 1 : 0)) : 0;
}

// d2 = (dx*dx + dy*dy) + dz*dz without contraction.
__device__ __forceinline__ float dist2_pred(float3 pi, float3 pj, const Box &b) {
#pragma clang fp contract(off)
    float dx = img_delta(pi.x, pj.x, b.L[0], b.half[0], b.per[0]);
    float dy = img_delta(pi.y, pj.y, b.L[1], b.half[1], b.per[1]);
    float dz = img_delta(pi.z, pj.z, b.L[2], b.half[2], b.per[2]);
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

// The same predicate when no periodic image can be involved.
__device__ __forceinline__ float dist2_direct(float3 pi, float3 pj) {
#pragma clang fp contract(off)
    float dx = pj.x - pi.x;
    float dy = pj.y - pi.y;
    float dz = pj.z - pi.z;
    float xx = dx * dx;
    float yy = dy * dy;
    float zz = dz * dz;
    float s = xx + yy;
    return s + zz;
}

// True when the predicate would use a shifted image on some axis.
__device__ __forceinline__ bool uses_image(float3 pi, float3 pj, const Box &b) {
    float tx = pj.x - pi.x, ty = pj.y - pi.y, tz = pj.z - pi.z;
    return (b.per[0] && fabsf(tx) > b.half[0]) || (b.per[1] && fabsf(ty) > b.half[1]) ||
           (b.per[2] && fabsf(tz) > b.half[2]);
}

// Exact FP64 separation xi - xj for the image chosen by the FP32 predicate.
__device__ __forceinline__ double sep_axis(float xi, float xj, float L, float half, int per) {
    return (double)xi - (double)xj - (double)img_shift(xi, xj, half, per) * (double)L;
}

// Wrap a coordinate into [0, L) after less than one box length of travel.
__device__ __forceinline__ float wrap_coord(float x, float L) {
#pragma clang fp contract(off)
    if (x >= L) x = x - L;
    if (x < 0.f) x = x + L;
    if (x >= L) x = 0.f;  // x slightly below 0 can round up to L
    return x;
}

// Cell coordinate along one axis: floor(x * (n / L)) clamped to [0, n-1],
// with the product taken in FP32.
__device__ __forceinline__ int cell_coord(float x, float inv, int n) {
#pragma clang fp contract(off)
    float f = x * inv;
    if (f < 1.0f) return 0;
    if (f >= (float)n) return n - 1;
    int i = (int)f;
    return i > n - 1 ? n - 1 : i;
}

// Eighth of cell iz (its cell_coord) in which coordinate z lies:
// floor((z * inv - iz) * 8) clamped to [0, 7], in FP32.  z * inv - iz is exact
// (Sterbenz) inside the cell, so (iz, eighth) never decreases as z grows; the
// cell sort tabulates where each eighth of a cell starts, and the Verlet build
// bounds its candidate windows with that table.
__device__ __forceinline__ int z_eighth(float z, float inv, int iz) {
#pragma clang fp contract(off)
    const float f = z * inv;
    const float t = (f - (float)iz) * 8.f;
    if (!(t >= 0.f)) return 0;
    return t >= 7.f ? 7 : (int)t;
}

__device__ __forceinline__ int cell_of(float3 p, const Box &b) {
    int ix = cell_coord(p.x, b.inv[0], b.nc[0]);
    int iy = cell_coord(p.y, b.inv[1], b.nc[1]);
    int iz = cell_coord(p.z, b.inv[2], b.nc[2]);
    return (ix * b.nc[1] + iy) * b.nc[2] + iz;
}

__device__ __forceinline__ float3 xyz(float4 v) { return make_float3(v.x, v.y, v.z); }

// Workgroups of a launch are dealt to the 8 XCDs in turn (workgroup b runs on
// XCD b % 8), and each XCD has its own L2.  This maps b to a logical index so
// that every XCD works through one contiguous range: neighbouring particles,
// whose positions the neighbour gathers share, then meet in the same L2.
// A bijection of [0, nb) for any nb.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, q = b >> 3;
    const int full = nb >> 3, rem = nb & 7;
    return x * full + min(x, rem) + q;
}

// Logical particle workgroup of the current workgroup.
__device__ __forceinline__ int pblock() { return xcd_block((int)blockIdx.x, (int)gridDim.x); }

// The system of the current particle workgroup (uniform over the workgroup).
// (a single system needs no table load: kernels then start their loads of
// the system's description at once)
__device__ __forceinline__ int block_system(const State &st) {
    return st.nsys == 1 ? 0 : st.blk2sys[pblock()];
}

// Global slot of this thread in a particle kernel (systems are block aligned).
__device__ __forceinline__ int64_t global_slot() {
    return (int64_t)pblock() * kBlock + threadIdx.x;
}

// Offsets entry of global cell c of system d.
__device__ __forceinline__ int off_index(const SysDesc &d, int c) {
    return d.off_base + (c - d.cell_base);
}

// Wrap, cell index and histogram for slot i of system s, keeping each
// particle's arrival rank.  Particles are still nearly in cell order from the
// previous build, so neighbouring lanes mostly share a cell: each run of equal
// cells inside a wavefront issues one atomic add for the whole run.  Every
// lane of the wavefront takes part (shuffles and a ballot).
__device__ __forceinline__ void cell_assign_slot(const State &st, int s, int64_t i) {
    const SysDesc &d = st.sys[s];
    const Box b = d.box;
    const int lane = threadIdx.x & 63;
    int c = -1;
    if (i - d.slot_base < d.n) {
        float4 p = st.pos[0][i];
        if (b.per[0]) p.x = wrap_coord(p.x, b.L[0]);
        if (b.per[1]) p.y = wrap_coord(p.y, b.L[1]);
        if (b.per[2]) p.z = wrap_coord(p.z, b.L[2]);
        st.pos[0][i] = p;
        c = d.cell_base + cell_of(xyz(p), b);
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
    if (c >= 0) st.rnk[i] = base + (lane - hl);
}

// Slots of a system, for the entry checks of debug builds.
struct SlotRange {
    int base, n_pad, dummy;
    int32_t *flag;  // Ctl::bad_index
};

__device__ __forceinline__ SlotRange slot_range(const State &st, const SysDesc &d) {
    return SlotRange{d.slot_base, d.n_pad, d.dummy, &st.ctl->bad_index};
}

// A list entry as read by a kernel: in debug builds one outside the system's
// slots is reported and replaced by the far-away slot; otherwise unchanged.
__device__ __forceinline__ int checked(const SlotRange &r, int j) {
    if (kChecked && (unsigned)(j - r.base) >= (unsigned)r.n_pad) {
        *r.flag = 1;
        return r.dummy;
    }
    return j;
}

// True when system s must rebuild its neighbour structures in this launch.
__device__ __forceinline__ bool rebuilding(const State &st, int s) {
    return st.sctl[s].rebuild[st.par] != 0;
}

// Wavefront reductions (64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Workgroup reduction of NV values (op 0 = sum, 1 = max, 2 = min) in a fixed
// order; thread 0 writes the results to part[slot[k] * pstride + pblock()]
// (one array per slot, so the finalize kernel reads them coalesced).
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], const int (&slot)[NV],
                                               const int (&op)[NV], double *part,
                                               int pstride) {
    __shared__ double lds[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NV; c++)
        v[c] = op[c] == 0 ? wave_sum(v[c]) : (op[c] == 1 ? wave_max(v[c]) : wave_min(v[c]));
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; c++) lds[w][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
#pragma unroll
        for (int c = 0; c < NV; c++) {
            double s = lds[0][c];
            for (int k = 1; k < nw; k++)
                s = op[c] == 0 ? s + lds[k][c] : (op[c] == 1 ? fmax(s, lds[k][c]) : fmin(s, lds[k][c]));
            part[(int64_t)slot[c] * pstride + pblock()] = s;
        }
    }
}

}  // namespace fpm
