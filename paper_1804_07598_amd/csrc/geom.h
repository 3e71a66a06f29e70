// Device geometry shared by the neighbour-search and interaction kernels:
// the FP32 neighbour predicate, periodic images, cell coordinates.
#pragma once

#include "fpm_internal.h"

namespace fpm {

// One coordinate difference of the FP32 neighbour predicate (header of fpm.h):
// t = xj - xi; on a periodic axis t > L/2 selects (xj - L) - xi and
// t < -L/2 selects xj - (xi - L).  Every operation rounds separately.
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

// True when the predicate would use a shifted image on some axis.
__device__ __forceinline__ bool uses_image(float3 pi, float3 pj, const Box &b) {
    float tx = pj.x - pi.x, ty = pj.y - pi.y, tz = pj.z - pi.z;
    return (b.per[0] && fabsf(tx) > b.half[0]) || (b.per[1] && fabsf(ty) > b.half[1]) ||
           (b.per[2] && fabsf(tz) > b.half[2]);
}

// Exact FP64 separation xi - xj for the image chosen by the FP32 predicate.
__device__ __forceinline__ double sep_axis(float xi, float xj, float L, float half, int per) {
    double d = (double)xi - (double)xj;
    if (per) {
        float t = xj - xi;
        if (t > half) d += (double)L;
        else if (t < -half) d -= (double)L;
    }
    return d;
}

// Wrap a coordinate into [0, L) after at most one box length of travel.
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

__device__ __forceinline__ int cell_of(float3 p, const Box &b) {
    int ix = cell_coord(p.x, b.inv[0], b.nc[0]);
    int iy = cell_coord(p.y, b.inv[1], b.nc[1]);
    int iz = cell_coord(p.z, b.inv[2], b.nc[2]);
    return (ix * b.nc[1] + iy) * b.nc[2] + iz;
}

// Blocked-ELL index of list entry k of slot i.
__device__ __forceinline__ int64_t ell_index(int64_t i, int k, int cap) {
    return ((i >> 6) * (int64_t)cap + k) * 64 + (i & 63);
}

__device__ __forceinline__ float3 xyz(float4 v) { return make_float3(v.x, v.y, v.z); }

// Wavefront reductions (64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Last-block-done protocol: every block calls this once after publishing its
// partial results; it returns true in exactly one block (the last to arrive),
// after which that block may read every block's partials.  The counter is
// reset by the last block.
__device__ __forceinline__ bool last_block(uint32_t *counter) {
    __shared__ bool is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        uint32_t t = atomicAdd(counter, 1u);
        is_last = (t == gridDim.x - 1);
        if (is_last) {
            __threadfence();
            atomicExch(counter, 0u);
        }
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last;
}

}  // namespace fpm
