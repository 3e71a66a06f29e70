// Verlet list build (section 2, ref [46]; section 4.1 uses Verlet lists for
// the MD client).  A particle's list holds every j != i that passes the FP32
// predicate at the list radius r_cut + skin; candidates are the particles of
// the 27 (de-duplicated) cells around its cell.  Every build also moves the
// freshly sorted state from buffer 1 back to buffer 0.
//
// Four builds produce the same sets (the choice is a launch shape):
//  - lockstep windows (k_verlet_ls, the default for contexts of at least
//    131,072 particles): one lane per particle; each lane's candidates in a
//    neighbour column are one z-window of slots, and the wavefront's lanes
//    walk their windows in step, hits staged in LDS rows;
//  - lane groups (k_verlet_grp, the default below that): G lanes per
//    particle over the same windows (or over whole cells for grids of fewer
//    than three cells along an axis), each 64-slot row of lists staged in
//    LDS and stored whole;
//  - one lane per particle without staging (k_verlet: windows, or whole
//    cells read from global memory), the default for short lists;
//  - column workgroups (k_verlet_cols): a workgroup stages the z-runs of the
//    3 x 3 columns around a block of z-cells in LDS and tests candidates in
//    chunks of 32.
#include "geom.h"

namespace fpm {
namespace {

constexpr int kColThreads = 128;  // threads of a column workgroup
constexpr int kLdsAtoms = 2048;   // staged positions per column workgroup (32 KiB)
constexpr int kMaxZb = 32;        // z-cells per workgroup, at most
constexpr int kRowGroups = 32;    // groups of four entries per slot kept in LDS by the lane-group build

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

// One particle's list being written.  Entries are collected four at a time
// and stored as one 16-byte group (the list layout's unit), which takes a
// quarter of the store instructions of entry-by-entry writes and never leaves
// a group half written.
struct ListOut {
    int4 *g0;    // the slot's group 0; group q is at g0[64 q]
    int cap;     // capacity in entries
    int count;   // entries found so far (may exceed cap: overflow)
    int4 buf;    // the group being filled
};

__device__ __forceinline__ ListOut list_out(const State &st, int64_t i, int cap, int cap4) {
    ListOut o;
    o.g0 = reinterpret_cast<int4 *>(st.nbr) + ((i >> 6) * (int64_t)cap4) * 64 + (i & 63);
    o.cap = cap;
    o.count = 0;
    o.buf = make_int4(0, 0, 0, 0);
    return o;
}

__device__ __forceinline__ void push(ListOut &o, int gj) {
    const int k = o.count & 3;
    o.buf.x = k == 0 ? gj : o.buf.x;
    o.buf.y = k == 1 ? gj : o.buf.y;
    o.buf.z = k == 2 ? gj : o.buf.z;
    o.buf.w = k == 3 ? gj : o.buf.w;
    if (k == 3 && o.count < o.cap) o.g0[(o.count >> 2) * 64] = o.buf;
    o.count++;
}

// Completes the list with the far-away padding slot up to a multiple of eight
// entries, so that list readers can consume whole groups of eight.
__device__ __forceinline__ void finish(ListOut &o, int dummy) {
    const int c = min(o.count, o.cap);
    const int c8 = (c + 7) & ~7;
    int g = c >> 2;
    if (c & 3) {
        const int k = c & 3;
        int4 v = o.buf;
        v.y = k <= 1 ? dummy : v.y;
        v.z = k <= 2 ? dummy : v.z;
        v.w = dummy;
        o.g0[g * 64] = v;
        g++;
    }
    for (; g * 4 < c8; g++) o.g0[g * 64] = make_int4(dummy, dummy, dummy, dummy);
}

// Tests candidates [beg, end) of `src` (global slots) or of the LDS stage
// (global slot in w, lower-face images already shifted) against particle i and
// appends the hits.
template <bool IMG, bool LDS>
__device__ __forceinline__ void scan_range(const float4 *__restrict__ src, int beg, int end,
                                           int i, float3 pi, const Box &b, float R2,
                                           ListOut &o, bool &img) {
    for (int c0 = beg; c0 < end; c0 += 32) {
        const int len = min(32, end - c0);
        uint32_t mask = 0;
#pragma unroll 4
        for (int u = 0; u < len; u++) {
            const float4 q = src[c0 + u];
            const bool hit = cand_d2<IMG>(pi, xyz(q), b) <= R2;
            mask |= (uint32_t)hit << u;
            if (IMG) img |= hit && uses_image(pi, xyz(q), b) && c0 + u != i;
        }
        while (mask) {
            const int u = __ffs(mask) - 1;
            mask &= mask - 1;
            const int gj = LDS ? __float_as_int(src[c0 + u].w) : c0 + u;
            if (gj != i) push(o, gj);  // i itself is always a hit
        }
    }
}

// First index of the z-sorted stage range [lo, hi) whose z is >= z (or > z
// with STRICT), hi if there is none.
template <bool STRICT>
__device__ __forceinline__ int z_bound(const float4 *sp, int lo, int hi, float z) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const float zm = sp[mid].z;
        if (STRICT ? zm <= z : zm < z)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
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
                                   float R2, ListOut &o, bool &img) {
    const Box &b = d.box;
    const float4 *__restrict__ pos = st.pos[1];
    const int32_t *__restrict__ off = st.off + d.off_base;
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
                scan_range<IMG, false>(pos, beg, end, i, pi, b, R2, o, img);
                r = r1 + 1;
            }
        }
    finish(o, d.dummy);
}

// One z-run of a neighbouring column, [beg, end) of the sorted buffer, whose
// z (after subtracting the image shift a.z) ascends.  Candidates below zlo are
// skipped and the scan stops above zhi; the rest are tested with the exact
// predicate: separation (q - a) - pk per axis, where a holds the shift of
// candidates moved down one period and pk the particle itself moved down for
// runs across the upper face (both subtractions exact).  Hits are appended.
__device__ __forceinline__ void scan_window(const float4 *__restrict__ pos, int beg, int end,
                                            float3 a, float3 pk, float zlo, float zhi, int i,
                                            float R2, ListOut &o, bool &hit_any) {
#pragma clang fp contract(off)
    constexpr int B = 8;  // candidates requested together (latency is the cost here)
    int c = beg;
    // skip to the window: z only, B at a time (the run is sorted)
    while (c < end) {
        int below = 0;
#pragma unroll
        for (int u = 0; u < B; u++) {
            const float z = c + u < end ? pos[c + u].z - a.z : INFINITY;
            below += z < zlo;
        }
        c += below;
        if (below < B) break;
    }
    // scan the window, B at a time
    while (c < end) {
        float4 q[B];
#pragma unroll
        for (int u = 0; u < B; u++) q[u] = pos[min(c + u, end - 1)];
        bool past = false;
#pragma unroll
        for (int u = 0; u < B; u++) {
            const int j = c + u;
            const float qz = q[u].z - a.z;
            past |= qz > zhi;
            const float dx = (q[u].x - a.x) - pk.x, dy = (q[u].y - a.y) - pk.y, dz = qz - pk.z;
            const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
            const float s = xx + yy;
            if (j < end && qz <= zhi && s + zz <= R2 && j != i) {
                push(o, j);
                hit_any = true;
            }
        }
        if (past) break;
        c += B;
    }
}

// List of slot i from global memory with candidate windows, for grids of at
// least three cells per axis.  Column (ox, oy) is at least dxy from i
// horizontally (the distance to the face of i's cell that faces it), so only
// |dz| <= sqrt(R^2 - dxy^2) can pass and columns beyond R are skipped; cells
// are ordered by z inside a column, so the window is found by a short skip.
// Bounds are widened (R^2 by 1e-4, cell faces by 1e-5 L) so that rounding
// can only add candidates; the predicate decides exactly.
__device__ void verlet_atom_window(const State &st, const SysDesc &d, int i, float3 pi,
                                   float R2, ListOut &o, bool &img) {
    const Box &b = d.box;
    const float4 *__restrict__ pos = st.pos[1];
    const int32_t *__restrict__ off = st.off + d.off_base;
    const int nx = b.nc[0], ny = b.nc[1], nz = b.nc[2];
    const int ix = cell_coord(pi.x, b.inv[0], nx);
    const int iy = cell_coord(pi.y, b.inv[1], ny);
    const int iz = cell_coord(pi.z, b.inv[2], nz);
    const float marg = 1e-5f * fmaxf(b.L[0], fmaxf(b.L[1], b.L[2]));
    const float dxl = fmaxf(pi.x - (float)ix / b.inv[0] - marg, 0.f);
    const float dxh = fmaxf((float)(ix + 1) / b.inv[0] - pi.x - marg, 0.f);
    const float dyl = fmaxf(pi.y - (float)iy / b.inv[1] - marg, 0.f);
    const float dyh = fmaxf((float)(iy + 1) / b.inv[1] - pi.y - marg, 0.f);
    const float Rw2 = R2 * 1.0001f;
    // z-runs: cells iz-1 .. iz+1 as at most two contiguous pieces
    int zc0[2], zc1[2];
    float azs[2], pks[2];
    int nseg = 0;
    if (iz == 0) {
        if (b.per[2]) {  // cell nz-1, one period down
            zc0[nseg] = nz - 1, zc1[nseg] = nz - 1, azs[nseg] = b.L[2], pks[nseg] = pi.z;
            nseg++;
        }
        zc0[nseg] = 0, zc1[nseg] = 1, azs[nseg] = 0.f, pks[nseg] = pi.z;
        nseg++;
    } else if (iz == nz - 1) {
        zc0[nseg] = nz - 2, zc1[nseg] = nz - 1, azs[nseg] = 0.f, pks[nseg] = pi.z;
        nseg++;
        if (b.per[2]) {  // cell 0, particle i moved down one period
            zc0[nseg] = 0, zc1[nseg] = 0, azs[nseg] = 0.f, pks[nseg] = pi.z - b.L[2];
            nseg++;
        }
    } else {
        zc0[nseg] = iz - 1, zc1[nseg] = iz + 1, azs[nseg] = 0.f, pks[nseg] = pi.z;
        nseg++;
    }
    for (int ox = -1; ox <= 1; ox++) {
        int cx = ix + ox;
        float ax = 0.f, px = pi.x;
        if (cx < 0 || cx >= nx) {
            if (!b.per[0]) continue;
            if (cx < 0) cx += nx, ax = b.L[0];
            else cx -= nx, px = pi.x - b.L[0];
        }
        const float ddx = ox < 0 ? dxl : (ox > 0 ? dxh : 0.f);
        for (int oy = -1; oy <= 1; oy++) {
            int cy = iy + oy;
            float ay = 0.f, py = pi.y;
            if (cy < 0 || cy >= ny) {
                if (!b.per[1]) continue;
                if (cy < 0) cy += ny, ay = b.L[1];
                else cy -= ny, py = pi.y - b.L[1];
            }
            const float ddy = oy < 0 ? dyl : (oy > 0 ? dyh : 0.f);
            const float h2 = Rw2 - ddx * ddx - ddy * ddy;
            if (h2 < 0.f) continue;
            const float hz = sqrtf(h2);
            const int col = (cx * ny + cy) * nz;
            for (int g = 0; g < nseg; g++) {
                bool hit = false;
                const float3 a = make_float3(ax, ay, azs[g]);
                const float3 pk = make_float3(px, py, pks[g]);
                scan_window(pos, off[col + zc0[g]], off[col + zc1[g] + 1], a, pk, pk.z - hz,
                            pk.z + hz, i, R2, o, hit);
                img |= hit && (ax != 0.f || px != pi.x || ay != 0.f || py != pi.y ||
                               azs[g] != 0.f || pks[g] != pi.z);
            }
        }
    }
    finish(o, d.dummy);
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
    if (st.keep_old) st.old[0][s] = st.old[1][s];
}

// ---------------------------------------------------------------------------
// Cooperative build: G lanes per particle.  A workgroup of 64 G threads owns
// one 64-slot row of the list layout.  A particle's G lanes walk each
// candidate run 32 consecutive candidates at a time (32 / G loads per lane in
// flight, coalesced, no divergence inside the run), hits are compacted with
// ballots and written to the row's lists in LDS, in list layout, and the
// whole row is stored with contiguous 16-byte writes at the end.  The run
// bounds of all nine columns are fetched at once, spread over the group's
// lanes and broadcast by shuffles.  Runs, windows and image shifts are those
// of verlet_atom_window (grids of at least three cells per axis) or the whole
// cells of verlet_atom_global (smaller grids), so the lists are identical
// entry for entry to those of the particle-by-particle builds.

// The G-lane group of this thread inside its wavefront: bit offset of the
// group in the ballot mask and this lane's index in the group.
template <int G>
struct Group {
    int base, l;
    __device__ __forceinline__ Group() {
        const int lane = (int)(threadIdx.x & 63);
        base = lane & ~(G - 1);
        l = lane & (G - 1);
    }
    // this group's bits of a wavefront ballot
    __device__ __forceinline__ uint32_t bits(uint64_t m) const {
        return (uint32_t)(m >> base) & (uint32_t)((1ull << G) - 1);
    }
};

// LDS row of lists: entry k of row position p, as in the global list layout.
__device__ __forceinline__ int row_entry(int p, int k) { return ((k >> 2) * 64 + p) * 4 + (k & 3); }

// One z-run [beg, end), shifts as in scan_window (SH: some shift is nonzero;
// without, the subtractions of zero are left out, which rounds identically);
// hits are appended at row[p][cnt..] for entries below lcap and straight to
// the slot's list in global memory (gl, list layout) from there up to the
// capacity.  Returns true when some hit was found.  The scan
// stops after the first batch reaching above zhi; every candidate tested is
// decided by the predicate alone.  The hit test has no short-circuit, so no
// branch splits a batch and all of its loads stay in flight together.
template <int G, bool SH>
__device__ __forceinline__ bool scan_run_group(const Group<G> &gr, const float4 *__restrict__ pos,
                                               int beg, int end, float3 a, float3 pk, float zhi,
                                               int i, float R2, int *row, int p, int lcap,
                                               int *gl, int cap, int &cnt) {
#pragma clang fp contract(off)
    constexpr int U = 32 / G;  // loads in flight per lane
    const char *base = reinterpret_cast<const char *>(pos);  // slots < 2^26: 32-bit offsets
    bool any = false;
    for (int c = beg; c < end; c += U * G) {
        float4 q[U];
#pragma unroll
        for (int u = 0; u < U; u++)
            q[u] = *reinterpret_cast<const float4 *>(
                base + ((uint32_t)min(c + u * G + gr.l, end - 1) << 4));
        bool past = false;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int j = c + u * G + gr.l;
            const float qx = SH ? q[u].x - a.x : q[u].x;
            const float qy = SH ? q[u].y - a.y : q[u].y;
            const float qz = SH ? q[u].z - a.z : q[u].z;
            past |= qz > zhi;
            const float dx = qx - pk.x, dy = qy - pk.y, dz = qz - pk.z;
            const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
            const float sxy = xx + yy;
            const bool hit = (j < end) & (sxy + zz <= R2) & (j != i);
            const uint32_t hm = gr.bits(__ballot(hit));
            const int k = cnt + __popc(hm & ((1u << gr.l) - 1));
            if (hit) {
                if (k < lcap)
                    row[row_entry(p, k)] = j;
                else if (k < cap)
                    gl[(k >> 2) * 256 + (k & 3)] = j;
            }
            cnt += __popc(hm);
            any |= hm != 0;
        }
        if (gr.bits(__ballot(past))) break;
    }
    return any;
}

// Whole cells (grids with fewer than three cells along some axis): one run of
// the de-duplicated stencil, every candidate tested with the full predicate
// (image chosen per axis), as in verlet_atom_global.  Returns true when a hit
// uses a periodic image.
template <int G>
__device__ __forceinline__ bool scan_cells_group(const Group<G> &gr, const float4 *__restrict__ pos,
                                                 int beg, int end, float3 pi, const Box &b, int i,
                                                 float R2, int *row, int p, int lcap, int *gl,
                                                 int cap, int &cnt) {
    constexpr int U = 32 / G;
    const char *base = reinterpret_cast<const char *>(pos);
    bool img = false;
    for (int c = beg; c < end; c += U * G) {
        float4 q[U];
#pragma unroll
        for (int u = 0; u < U; u++)
            q[u] = *reinterpret_cast<const float4 *>(
                base + ((uint32_t)min(c + u * G + gr.l, end - 1) << 4));
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int j = c + u * G + gr.l;
            const bool hit = (j < end) & (cand_d2<true>(pi, xyz(q[u]), b) <= R2) & (j != i);
            const uint32_t hm = gr.bits(__ballot(hit));
            const int k = cnt + __popc(hm & ((1u << gr.l) - 1));
            if (hit) {
                if (k < lcap)
                    row[row_entry(p, k)] = j;
                else if (k < cap)
                    gl[(k >> 2) * 256 + (k & 3)] = j;
            }
            cnt += __popc(hm);
            img |= gr.bits(__ballot(hit && uses_image(pi, xyz(q[u]), b))) != 0;
        }
    }
    return img;
}

// Eight and sixteen lanes per particle: registers held to 64 per lane, so
// that the LDS budget (four 512-lane workgroups per CU) sets the occupancy;
// the few values this spills are reloaded between runs, not inside them.
template <int G>
__global__ __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(G == 4 ? 1 : 8)))
void k_verlet_grp(State st, const int32_t *blocks, float R2, int cap, int cap4, int lcap4) {
    constexpr int NC = (9 + G - 1) / G;  // neighbour columns held per lane
    extern __shared__ int4 lrow[];       // lcap4 * 64 int4: the row's first lcap4 groups
    __shared__ int rowc8[64];            // padded list lengths of the row
    if (st.nsys == 1 && !rebuilding(st, 0)) return;  // a single system: no table loads first
    const int r = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int blk = blocks[r >> 2];
    const int s = st.nsys == 1 ? 0 : st.blk2sys[blk];
    if (!rebuilding(st, s)) return;
    const SysDesc &d = st.sys[s];
    const Box &b = d.box;
    const Group<G> gr;
    const int p = (int)threadIdx.x / G;
    const int64_t row0 = (int64_t)blk * kBlock + (r & 3) * 64;
    const int64_t i = row0 + p;
    int *row = reinterpret_cast<int *>(lrow);
    const int lcap = 4 * lcap4;
    int *gl = st.nbr + ((row0 >> 6) * (int64_t)cap4 * 64 + p) * 4;  // the slot's list
    const float4 *__restrict__ pos = st.pos[1];
    const int32_t *__restrict__ off = st.off + d.off_base;
    int cnt = 0;
    bool img = false;
    if (i - d.slot_base < d.n) {
        const float3 pi = xyz(pos[i]);
        const int nx = b.nc[0], ny = b.nc[1], nz = b.nc[2];
        const int ix = cell_coord(pi.x, b.inv[0], nx);
        const int iy = cell_coord(pi.y, b.inv[1], ny);
        const int iz = cell_coord(pi.z, b.inv[2], nz);
        if (d.zb == -3) {
            // whole cells of the de-duplicated stencil, z pieces merged
            int sx[3], sy[3], sz[3];
            const int mx = stencil_axis(ix, nx, b.per[0], sx);
            const int my = stencil_axis(iy, ny, b.per[1], sy);
            const int mz = stencil_axis(iz, nz, b.per[2], sz);
            for (int a = 0; a < mx; a++)
                for (int q = 0; q < my; q++) {
                    const int col = (sx[a] * ny + sy[q]) * nz;
                    int z = 0;
                    while (z < mz) {
                        int z1 = z;
                        while (z1 + 1 < mz && sz[z1 + 1] == sz[z1] + 1) z1++;
                        img |= scan_cells_group<G>(gr, pos, off[col + sz[z]], off[col + sz[z1] + 1],
                                                   pi, b, (int)i, R2, row, p, lcap, gl, cap, cnt);
                        z = z1 + 1;
                    }
                }
        } else {
            // z-runs: cells iz-1 .. iz+1 as at most two contiguous pieces
            // (first and last cell, shift of the candidates, particle's own z)
            int zc0[2], zc1[2];
            float azs[2], pks[2];
            int nseg = 1;
            azs[0] = azs[1] = 0.f, pks[0] = pks[1] = pi.z;
            zc0[1] = zc1[1] = 0;
            if (iz == 0 && b.per[2]) {  // cell nz-1 one period down, then cells 0, 1
                zc0[0] = zc1[0] = nz - 1, azs[0] = b.L[2];
                zc0[1] = 0, zc1[1] = 1, nseg = 2;
            } else if (iz == 0) {
                zc0[0] = 0, zc1[0] = 1;
            } else if (iz == nz - 1) {  // cells nz-2, nz-1, then cell 0 with i moved down
                zc0[0] = nz - 2, zc1[0] = nz - 1;
                if (b.per[2]) zc0[1] = zc1[1] = 0, pks[1] = pi.z - b.L[2], nseg = 2;
            } else {
                zc0[0] = iz - 1, zc1[0] = iz + 1;
            }
            // run bounds: this lane fetches those of columns l, l + G, ...
            int rb[NC][2], re[NC][2];
    #pragma unroll
            for (int m = 0; m < NC; m++) {
                const int k = gr.l + m * G;
                int cx = ix + k / 3 - 1, cy = iy + k % 3 - 1;
                const bool ok = k < 9 && (b.per[0] || (cx >= 0 && cx < nx)) &&
                                (b.per[1] || (cy >= 0 && cy < ny));
                cx = cx < 0 ? cx + nx : (cx >= nx ? cx - nx : cx);
                cy = cy < 0 ? cy + ny : (cy >= ny ? cy - ny : cy);
                const int col = ok ? (cx * ny + cy) * nz : 0;
    #pragma unroll
                for (int g = 0; g < 2; g++) {
                    const bool okg = ok && g < nseg;
                    const int e0 = off[okg ? col + zc0[g] : 0], e1 = off[okg ? col + zc1[g] + 1 : 0];
                    rb[m][g] = okg ? e0 : 0;
                    re[m][g] = okg ? e1 : 0;
                }
            }
            const float marg = 1e-5f * fmaxf(b.L[0], fmaxf(b.L[1], b.L[2]));
            const float dxl = fmaxf(pi.x - (float)ix / b.inv[0] - marg, 0.f);
            const float dxh = fmaxf((float)(ix + 1) / b.inv[0] - pi.x - marg, 0.f);
            const float dyl = fmaxf(pi.y - (float)iy / b.inv[1] - marg, 0.f);
            const float dyh = fmaxf((float)(iy + 1) / b.inv[1] - pi.y - marg, 0.f);
            const float Rw2 = R2 * 1.0001f;
            for (int k = 0; k < 9; k++) {
                const int ox = k / 3 - 1, oy = k % 3 - 1;
                const int cx = ix + ox, cy = iy + oy;
                const float ax = cx < 0 ? b.L[0] : 0.f, px = cx >= nx ? pi.x - b.L[0] : pi.x;
                const float ay = cy < 0 ? b.L[1] : 0.f, py = cy >= ny ? pi.y - b.L[1] : pi.y;
                const float ddx = ox < 0 ? dxl : (ox > 0 ? dxh : 0.f);
                const float ddy = oy < 0 ? dyl : (oy > 0 ? dyh : 0.f);
                const float h2 = Rw2 - ddx * ddx - ddy * ddy;
                // bounds of column k from lane k % G of the group (empty runs where
                // the column lies across a closed face)
                int kb[2], ke[2];
    #pragma unroll
                for (int g = 0; g < 2; g++) {
                    int vb = rb[0][g], ve = re[0][g];
    #pragma unroll
                    for (int m = 1; m < NC; m++) {
                        vb = k / G == m ? rb[m][g] : vb;
                        ve = k / G == m ? re[m][g] : ve;
                    }
                    kb[g] = __shfl(vb, k % G, G);
                    ke[g] = __shfl(ve, k % G, G);
                }
                if (h2 < 0.f) continue;
                const float hz = sqrtf(h2);
    #pragma unroll
                for (int g = 0; g < 2; g++) {
                    if (kb[g] >= ke[g]) continue;
                    const float3 a = make_float3(ax, ay, azs[g]);
                    const float3 pk = make_float3(px, py, pks[g]);
                    const bool sh = ax != 0.f || px != pi.x || ay != 0.f || py != pi.y ||
                                    azs[g] != 0.f || pks[g] != pi.z;
                    const bool hit =
                        sh ? scan_run_group<G, true>(gr, pos, kb[g], ke[g], a, pk, pk.z + hz, (int)i,
                                                     R2, row, p, lcap, gl, cap, cnt)
                           : scan_run_group<G, false>(gr, pos, kb[g], ke[g], a, pk, pk.z + hz, (int)i,
                                                      R2, row, p, lcap, gl, cap, cnt);
                    img |= hit && sh;
                }
            }
        }
        const int c = min(cnt, cap);
        const int c8 = (c + 7) & ~7;
        for (int k = c + gr.l; k < c8; k += G) {
            if (k < lcap)
                row[row_entry(p, k)] = d.dummy;
            else
                gl[(k >> 2) * 256 + (k & 3)] = d.dummy;
        }
        if (gr.l == 0) {
            st.nnb[i] = (uint32_t)c | (img ? kWrapBit : 0u);
            note_overflow(st, cnt, cap);
        }
        rowc8[p] = c8;
    } else {
        rowc8[p] = 0;
    }
    if (gr.l == 0) copy_back(st, i);
    __syncthreads();
    // the row's lists, in list layout, written group by group over the row
    int4 *dst = reinterpret_cast<int4 *>(st.nbr) + (row0 >> 6) * (int64_t)cap4 * 64;
    for (int t = (int)threadIdx.x; t < lcap4 * 64; t += 64 * G)
        if ((t >> 6) * 4 < rowc8[t & 63]) dst[t] = lrow[t];
}

// One thread per particle, candidates read from global memory.  The grid
// runs over the list of particle workgroups of the systems built this way.
__global__ __launch_bounds__(kBlock) void k_verlet(State st, const int32_t *blocks, float R2,
                                                   int cap, int cap4) {
    if (st.nsys == 1 && !rebuilding(st, 0)) return;  // a single system: no table loads first
    const int blk = blocks[blockIdx.x];
    const int s = st.nsys == 1 ? 0 : st.blk2sys[blk];
    if (!rebuilding(st, s)) return;
    const SysDesc &d = st.sys[s];
    const Box b = d.box;
    const int64_t i = (int64_t)blk * kBlock + threadIdx.x;
    const bool active = i - d.slot_base < d.n;
    ListOut o = list_out(st, i, cap, cap4);
    bool img = false, face = false;
    float3 pi = make_float3(0.f, 0.f, 0.f);
    if (active) {
        pi = xyz(st.pos[1][i]);
        face = near_face(cell_coord(pi.x, b.inv[0], b.nc[0]), cell_coord(pi.y, b.inv[1], b.nc[1]),
                         cell_coord(pi.z, b.inv[2], b.nc[2]), b);
    }
    const bool face_wave = __ballot(face) != 0;
    if (active) {
        if (d.zb < 0)
            verlet_atom_window(st, d, (int)i, pi, R2, o, img);
        else if (face_wave)
            verlet_atom_global<true>(st, d, (int)i, pi, R2, o, img);
        else
            verlet_atom_global<false>(st, d, (int)i, pi, R2, o, img);
        st.nnb[i] = (uint32_t)min(o.count, cap) | (img ? kWrapBit : 0u);
        note_overflow(st, o.count, cap);
    }
    copy_back(st, i);
}

// Column workgroups (see the file comment); one work item per (system,
// column, z-block).
__global__ __launch_bounds__(kColThreads) void k_verlet_cols(State st, float R2, int cap,
                                                             int cap4) {
    const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);  // consecutive columns per XCD
    const int s = st.item2sys[lb];
    if (!rebuilding(st, s)) return;
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
    // faces of the column's cells (FP32, within a few ulp of the cell test)
    const float xlo = (float)ix / b.inv[0], xhi = (float)(ix + 1) / b.inv[0];
    const float ylo = (float)iy / b.inv[1], yhi = (float)(iy + 1) / b.inv[1];
    const float marg = 1e-5f * fmaxf(b.L[0], fmaxf(b.L[1], b.L[2]));

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
            ListOut o = list_out(st, i, cap, cap4);
            if (use_lds) {
                // The run's last cell is cell 0 one period up when z1 wraps; only
                // particles of the top z-cell (m + 2 == nrun) reach it.
                const bool top_img = b.per[2] && z1 == nz;
                // Candidate windows: column k is at least dxy from i horizontally
                // (distance to the side of i's cell that faces it), so only
                // |dz| <= sqrt(R^2 - dxy^2) can pass; each stage range is sorted by
                // z, so that window is a subrange found by bisection.  Bounds are
                // widened (R^2 by 1e-4, cell faces by 1e-5 L) so that rounding
                // can only add candidates; the predicate then decides exactly.
                const float Rw2 = R2 * 1.0001f;
                const float dxl = fmaxf(pi.x - xlo - marg, 0.f), dxh = fmaxf(xhi - pi.x - marg, 0.f);
                const float dyl = fmaxf(pi.y - ylo - marg, 0.f), dyh = fmaxf(yhi - pi.y - marg, 0.f);
                for (int k = 0; k < 9; k++) {
                    const int ox = k / 3 - 1, oy = k % 3 - 1;
                    const float ddx = ox < 0 ? dxl : (ox > 0 ? dxh : 0.f);
                    const float ddy = oy < 0 ? dyl : (oy > 0 ? dyh : 0.f);
                    const float h2 = Rw2 - ddx * ddx - ddy * ddy;
                    if (h2 < 0.f) continue;
                    const float hz = sqrtf(h2);
                    float3 pk = pi;  // i moved down one period where column k lies across
                    if (sh[k][1][0] > 0.f) pk.x = pi.x - b.L[0];  // the upper face (exact:
                    if (sh[k][1][1] > 0.f) pk.y = pi.y - b.L[1];  // i is in the top cell)
                    const int beg = colbase[k] + cs[k][m - 1], end = colbase[k] + cs[k][m + 2];
                    const int mid = m + 2 == nrun ? colbase[k] + cs[k][nrun - 1] : end;
                    int lo = z_bound<false>(sp, beg, mid, pk.z - hz);
                    int hi = z_bound<true>(sp, lo, mid, pk.z + hz);
                    scan_range<false, true>(sp, lo, hi, i, pk, b, R2, o, img);
                    if (top_img) pk.z = pi.z - b.L[2];
                    lo = z_bound<false>(sp, mid, end, pk.z - hz);
                    hi = z_bound<true>(sp, lo, end, pk.z + hz);
                    scan_range<false, true>(sp, lo, hi, i, pk, b, R2, o, img);
                }
                finish(o, d.dummy);
                img = face;  // its stencil reaches across a periodic face
            } else if (face_wave) {
                verlet_atom_global<true>(st, d, i, pi, R2, o, img);
            } else {
                verlet_atom_global<false>(st, d, i, pi, R2, o, img);
            }
            st.nnb[i] = (uint32_t)min(o.count, cap) | (img ? kWrapBit : 0u);
            note_overflow(st, o.count, cap);
            copy_back(st, i);
        }
    }
    // padding slots are in no cell: the system's first work item moves them back
    if (item == 0)
        for (int64_t q = d.slot_base + d.n + threadIdx.x; q < d.slot_base + d.n_pad;
             q += kColThreads)
            copy_back(st, q);
}

// ---------------------------------------------------------------------------
// Lockstep window build (grids of at least three cells per axis): one lane per
// particle, and the lanes of a wavefront walk their candidate windows in step,
// candidate m of every lane's window of the same neighbour column at a time,
// so that the wavefront's loads fall on a few cache lines (the lanes are
// consecutive slots of one column, and their windows in a neighbour column
// are short z-shifted ranges of the same sorted run).  A particle's window in
// column k holds the run of cells iz-1 .. iz+1 restricted to
// |z - z_i| <= sqrt(R^2 - d_k^2), d_k its horizontal distance to the column
// (as in verlet_atom_window: bounds widened so that rounding only adds
// candidates); the window ends are found by bisection on the z-sorted run.
// Opposite columns are walked as one sequence (window of column k, then of
// column 8 - k): a particle close to one side of its cell has a long window on
// that side and a short one on the other, so the pair's total varies much less
// between the lanes than either window, and the wavefront waits less for its
// longest lane.  Wavefronts with a particle in the first or last z-cell of a
// periodic box take the general form (each window in up to two pieces, one of
// them across the z face, walked piece by piece).  Hits are stored straight
// into the list layout.  Lists are identical as sets to those of the other
// builds; entries are in column order, z ascending within a column.

// One window piece of one column: candidates [lo, lo + len) of the sorted
// buffer, shifted by -a (candidates across the lower face) and tested against
// the particle at pk (moved down one period across the upper face).
struct Piece {
    int lo, len;
};

// Slot bounds of the candidates of one window piece: cells zc0 .. zc1 of the
// column starting at cell `col`, whose (unshifted) z lies in [zlo, zhi].
// The bounds come from the eighth-of-cell table of the cell sort: a particle
// with z >= zlo has (cell, eighth) >= those of zlo, so every such particle is
// at or after lo, and likewise every particle with z <= zhi is before hi; the
// piece holds at most an eighth of a cell of extra candidates at either end,
// which the predicate rejects.
__device__ __forceinline__ void window_bounds(const int32_t *__restrict__ off,
                                              const int32_t *__restrict__ sub, const Box &b,
                                              int col, int zc0, int zc1, float zlo, float zhi,
                                              int &lo, int &hi) {
    const int nz = b.nc[2];
    const float inv = b.inv[2];
    const int c0 = cell_coord(zlo, inv, nz), c1 = cell_coord(zhi, inv, nz);
    const int e0 = z_eighth(zlo, inv, c0), e1 = z_eighth(zhi, inv, c1);
    lo = c0 < zc0 ? off[col + zc0] : (c0 > zc1 ? off[col + zc1 + 1] : sub[(col + c0) * 8 + e0]);
    hi = c1 > zc1 ? off[col + zc1 + 1]
                  : (c1 < zc0 ? off[col + zc0]
                              : (e1 == 7 ? off[col + c1 + 1] : sub[(col + c1) * 8 + e1 + 1]));
}

// Shifts of column k for a particle in cell (ix, iy): candidate shift (ax, ay)
// for columns across the lower face, particle coordinate (px, py) moved down
// across the upper face, and the column's first cell; false when the column
// lies across a closed face.
__device__ __forceinline__ bool column_of(const Box &b, int ix, int iy, float x, float y, int k,
                                          float &ax, float &ay, float &px, float &py, int &col) {
    const int nx = b.nc[0], ny = b.nc[1], nz = b.nc[2];
    int cx = ix + k / 3 - 1, cy = iy + k % 3 - 1;
    ax = ay = 0.f;
    px = x;
    py = y;
    if (cx < 0 || cx >= nx) {
        if (!b.per[0]) return false;
        if (cx < 0) cx += nx, ax = b.L[0];
        else cx -= nx, px = x - b.L[0];
    }
    if (cy < 0 || cy >= ny) {
        if (!b.per[1]) return false;
        if (cy < 0) cy += ny, ay = b.L[1];
        else cy -= ny, py = y - b.L[1];
    }
    col = (cx * ny + cy) * nz;
    return true;
}

// Hits of the lockstep build collect in a per-lane LDS row, unwritten ones
// at its front.  A store inside the candidate loop makes the wavefront's next
// loads wait for it (loads and stores share one completion counter), so
// stores are issued at few, wavefront-uniform points: after a round of
// candidates in which some lane holds kFlushAt unwritten entries, every lane
// writes its complete groups of four (16-byte stores into the list layout)
// and moves the rest, at most three, to the front of its row.  A round adds
// at most eight entries, so a row never holds more than kFlushAt + 7 and the
// final padding to eight fits as well.
constexpr int kRowInts = 40;  // ints per lane (16-byte aligned rows)
constexpr int kFlushAt = 28;
static_assert(kFlushAt + 7 + 4 <= kRowInts, "a lane's row must hold a round and a group read");

// Entries are held as byte offsets into the position buffer (slot * 16, the
// form the candidate loads use) and written to the list as slots.
__device__ __forceinline__ int4 slots_of(int4 o) {
    return make_int4(o.x >> 4, o.y >> 4, o.z >> 4, o.w >> 4);
}

struct HitRow {
    int *r;         // this lane's row
    int loc = 0;    // unwritten entries, at r[0, loc)
    int done = 0;   // entries written to the list
    int lost = 0;   // hits dropped past the capacity

    // Appends the slot at byte offset o when `hit`.  Called for every
    // candidate, without a branch: a miss writes the first free word, which
    // the next hit reuses.
    __device__ __forceinline__ void put(int o, bool hit) {
        r[loc] = o;
        loc += hit;
    }

    // Writes the complete groups of four below the capacity to the list (gl:
    // this lane's list, groups 256 ints apart) and keeps the rest.  Hits past
    // the capacity are dropped and counted, so that the list is reported as
    // overflowed (FPM_EOVERFLOW, lists invalid); nothing is written beyond
    // the capacity.
    __device__ __forceinline__ void flush(int *gl, int cap) {
        const int keep = min(done + loc, cap);
        const int upto = keep & ~3;
        for (int k = done; k < upto; k += 4)
            *reinterpret_cast<int4 *>(gl + (k >> 2) * 256) =
                slots_of(*reinterpret_cast<const int4 *>(r + (k - done)));
        // the remaining 0 to 3 entries to the front (upto - done is a
        // multiple of four, at most kFlushAt + 7 - 3)
        *reinterpret_cast<int4 *>(r) = *reinterpret_cast<const int4 *>(r + (upto - done));
        lost += done + loc - keep;
        loc = keep - upto;
        done = upto;
    }

    __device__ __forceinline__ void flush_if_due(int *gl, int cap) {
        if (__ballot(loc >= kFlushAt) != 0) flush(gl, cap);
    }

    // Hits found, including any dropped.
    __device__ __forceinline__ int found() const { return done + loc + lost; }

    // Writes the remaining entries, padded with slot `pad` to a multiple of
    // eight, and returns the list length (at most cap).
    __device__ __forceinline__ int finish(int *gl, int cap, int pad) {
        const int keep = min(done + loc, cap);
        const int c8 = (keep + 7) & ~7;
        for (int k = keep; k < c8; k++) r[k - done] = pad << 4;
        for (int k = done; k < c8; k += 4)
            *reinterpret_cast<int4 *>(gl + (k >> 2) * 256) =
                slots_of(*reinterpret_cast<const int4 *>(r + (k - done)));
        return keep;
    }
};

template <bool SH>
__device__ __forceinline__ bool test_cand(float4 q, float3 a, float3 pk, float R2) {
#pragma clang fp contract(off)
    const float qx = SH ? q.x - a.x : q.x, qy = SH ? q.y - a.y : q.y, qz = SH ? q.z - a.z : q.z;
    const float dx = qx - pk.x, dy = qy - pk.y, dz = qz - pk.z;
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float sxy = xx + yy;
    return sxy + zz <= R2;
}

// Lockstep build of a system whose grid has at most two cells per axis: the
// stencil holds every cell, so the candidates of every particle are the whole
// system, walked by all lanes together (each load serves the whole wavefront)
// and tested with the whole-cell predicate (image chosen per axis).  The sets
// are those of the other builds; hits come in slot order.
__device__ __forceinline__ void lockstep_whole_system(const State &st, const SysDesc &d,
                                                      int64_t i, bool active, float R2, int cap,
                                                      int cap4, int *row) {
    const Box &b = d.box;
    const float4 *__restrict__ pos = st.pos[1];
    const float3 pi = active ? xyz(pos[i]) : make_float3(0.f, 0.f, 0.f);
    int *gl = st.nbr + (((i >> 6) * (int64_t)cap4 * 64 + (i & 63)) << 2);
    HitRow hr{row};
    bool img = false;
    const int end = d.slot_base + d.n;
    const char *pbase = reinterpret_cast<const char *>(pos);
    constexpr int U = 8;
    for (int m = d.slot_base; m < end; m += U) {  // the same range for every lane
        float4 q[U];
#pragma unroll
        for (int u = 0; u < U; u++)
            q[u] = *reinterpret_cast<const float4 *>(pbase + ((uint32_t)(m + u) << 4));
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int j = m + u;
            const bool hit = active & (j < end) & (j != (int)i) &
                             (cand_d2<true>(pi, xyz(q[u]), b) <= R2);
            hr.put(j << 4, hit);
            img |= hit & uses_image(pi, xyz(q[u]), b);
        }
        hr.flush_if_due(gl, cap);
    }
    if (active) {
        const int c = hr.finish(gl, cap, d.dummy);
        st.nnb[i] = (uint32_t)c | (img ? kWrapBit : 0u);
        note_overflow(st, hr.found(), cap);
    }
    copy_back(st, i);
}

// One wavefront per workgroup (a quarter of a particle workgroup's slots):
// small systems spread over every CU.  Registers held to 128 per lane: four
// waves per SIMD, without spills.
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_verlet_ls(State st, const int32_t *blocks, float R2, int cap, int cap4) {
#pragma clang fp contract(off)
    if (st.nsys == 1 && !rebuilding(st, 0)) return;  // a single system: no table loads first
    // one system: each XCD takes one contiguous range of its columns (shared
    // candidates in one L2); a batch: workgroups in turn over the XCDs, so that
    // the systems rebuilding in a step are spread evenly over them
    const int r = st.nsys == 1 ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const int blk = blocks[r >> 2];
    const int s = st.nsys == 1 ? 0 : st.blk2sys[blk];
    if (!rebuilding(st, s)) return;
    const SysDesc &d = st.sys[s];
    const Box &b = d.box;
    const int64_t i = (int64_t)blk * kBlock + (r & 3) * kWave + threadIdx.x;
    const bool active = i - d.slot_base < d.n;
    __shared__ __align__(16) int rows[kWave * kRowInts];
    int *row = rows + threadIdx.x * kRowInts;
    if (d.zb == -3) {  // the whole workgroup: a grid of at most two cells per axis
        lockstep_whole_system(st, d, i, active, R2, cap, cap4, row);
        return;
    }
    const float4 *__restrict__ pos = st.pos[1];
    const int32_t *__restrict__ off = st.off + d.off_base;
    const int nx = b.nc[0], ny = b.nc[1], nz = b.nc[2];
    float3 pi = make_float3(0.f, 0.f, 0.f);
    int ix = 0, iy = 0, iz = 1;
    if (active) {
        pi = xyz(pos[i]);
        ix = cell_coord(pi.x, b.inv[0], nx);
        iy = cell_coord(pi.y, b.inv[1], ny);
        iz = cell_coord(pi.z, b.inv[2], nz);
    }
    // z-pieces of the runs: cells zc0[g] .. zc1[g], candidate z shift azs[g],
    // particle z pks[g] (as in the lane-group build)
    int zc0[2] = {iz - 1, 0}, zc1[2] = {iz + 1, -1};
    float azs[2] = {0.f, 0.f}, pks[2] = {pi.z, pi.z};
    if (iz == 0) {
        if (b.per[2]) zc0[0] = zc1[0] = nz - 1, azs[0] = b.L[2], zc0[1] = 0, zc1[1] = 1;
        else zc0[0] = 0, zc1[0] = 1;
    } else if (iz == nz - 1) {
        zc0[0] = nz - 2, zc1[0] = nz - 1;
        if (b.per[2]) zc0[1] = zc1[1] = 0, pks[1] = pi.z - b.L[2];
    }
    const bool zwrap = __ballot(active && zc1[1] >= zc0[1]) != 0;  // some lane has two pieces
    // horizontal distances to the four sides of the particle's cell
    const float marg = 1e-5f * fmaxf(b.L[0], fmaxf(b.L[1], b.L[2]));
    const float dxl = fmaxf(pi.x - (float)ix / b.inv[0] - marg, 0.f);
    const float dxh = fmaxf((float)(ix + 1) / b.inv[0] - pi.x - marg, 0.f);
    const float dyl = fmaxf(pi.y - (float)iy / b.inv[1] - marg, 0.f);
    const float dyh = fmaxf((float)(iy + 1) / b.inv[1] - pi.y - marg, 0.f);
    const float Rw2 = R2 * 1.0001f;
    // windows of every piece (independent table loads)
    const int32_t *__restrict__ sub = st.sub;
    Piece w[9][2];
    bool shx[9];  // column k lies across an x or y face for this particle
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const int ox = k / 3 - 1, oy = k % 3 - 1;
        float ax, ay, px, py;
        int col = 0;
        bool ok = active && column_of(b, ix, iy, pi.x, pi.y, k, ax, ay, px, py, col);
        shx[k] = ax != 0.f || ay != 0.f || px != pi.x || py != pi.y;
        const float ddx = ox < 0 ? dxl : (ox > 0 ? dxh : 0.f);
        const float ddy = oy < 0 ? dyl : (oy > 0 ? dyh : 0.f);
        const float h2 = Rw2 - ddx * ddx - ddy * ddy;
        ok = ok && h2 >= 0.f;
        const float hz = ok ? sqrtf(h2) : 0.f;
        col += d.cell_base;  // global cell numbering of the table
#pragma unroll
        for (int g = 0; g < 2; g++) {
            int lo = 0, hi = 0;
            if (ok && zc1[g] >= zc0[g])
                window_bounds(off - d.cell_base, sub, b, col, zc0[g], zc1[g],
                              pks[g] - hz + azs[g], pks[g] + hz + azs[g], lo, hi);
            w[k][g].lo = lo;
            w[k][g].len = hi > lo ? hi - lo : 0;
        }
    }
    // shifts of a column for this particle
    auto shifts = [&](int k, int g, float3 &a, float3 &pk) {
        float ax, ay, px, py;
        int col;
        column_of(b, ix, iy, pi.x, pi.y, k, ax, ay, px, py, col);
        a = make_float3(ax, ay, azs[g]);
        pk = make_float3(px, py, pks[g]);
    };
    int *gl = st.nbr + (((i >> 6) * (int64_t)cap4 * 64 + (i & 63)) << 2);
    HitRow hr{row};
    bool img = false;
    // one walk over window A followed by window B, all lanes in step, eight
    // candidates per round (their loads issued together); indices past the
    // end of a lane's walk run up to seven slots past its last window (into
    // the position buffer's slack at most) and are not tested.  `own`
    // (std::true_type) when a window is the particle's own column, the only
    // one that holds the particle itself.
    const char *pbase = reinterpret_cast<const char *>(pos);  // slots < 2^26: 32-bit offsets
    const int io = (int)i << 4;  // this particle's byte offset
    auto walk = [&](Piece A, Piece B, int ka, int kb, bool shA, bool shB, int gA, int gB,
                    auto own) {
        constexpr int U = 8;
        constexpr bool kOwn = decltype(own)::value;
        const int tot = A.len + B.len;
        const bool sh = __ballot(active && (shA || shB)) != 0;
        float3 aA = make_float3(0.f, 0.f, 0.f), pA = pi, aB = aA, pB = pi;
        if (sh) {
            shifts(ka, gA, aA, pA);
            shifts(kb, gB, aB, pB);
        }
        // one loop for wavefronts with shifted candidates, one without (the
        // choice is uniform, so it is taken once per walk)
        auto rounds = [&](auto shifted) {
            constexpr bool kSh = decltype(shifted)::value;
            for (int m = 0; __ballot(m < tot) != 0; m += U) {
                // byte offsets of the round's first candidate in A and in B
                const int oA = (A.lo + m) << 4, oB = (B.lo - A.len + m) << 4;
                int jj[U];  // byte offsets of the candidates (slot * 16)
                float4 q[U];
#pragma unroll
                for (int u = 0; u < U; u++) jj[u] = (m + u < A.len ? oA : oB) + 16 * u;
#pragma unroll
                for (int u = 0; u < U; u++)
                    q[u] = *reinterpret_cast<const float4 *>(pbase + (uint32_t)jj[u]);
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int mu = m + u;
                    const bool other = !kOwn || jj[u] != io;
                    if (kSh) {
                        const bool inA = mu < A.len;
                        const bool hit = (mu < tot) & other &
                                         test_cand<true>(q[u], inA ? aA : aB, inA ? pA : pB, R2);
                        hr.put(jj[u], hit);
                        img |= hit & (inA ? shA : shB);
                    } else {
                        const bool hit = (mu < tot) & other & test_cand<false>(q[u], aA, pi, R2);
                        hr.put(jj[u], hit);
                    }
                }
                hr.flush_if_due(gl, cap);
            }
        };
        if (sh)
            rounds(std::true_type{});
        else
            rounds(std::false_type{});
    };
    // the same over four pieces: both z-pieces of column ka, then both of
    // column kb (lanes whose column wraps in z have two)
    auto walk4 = [&](const Piece *P, int ka, int kb, bool sxa, bool sxb, bool sz0, bool sz1) {
        constexpr int U = 8;
        const int c1 = P[0].len, c2 = c1 + P[1].len, c3 = c2 + P[2].len, tot = c3 + P[3].len;
        float axa, aya, pxa, pya, axb, ayb, pxb, pyb;
        int col;
        column_of(b, ix, iy, pi.x, pi.y, ka, axa, aya, pxa, pya, col);
        column_of(b, ix, iy, pi.x, pi.y, kb, axb, ayb, pxb, pyb, col);
        for (int m = 0; __ballot(m < tot) != 0; m += U) {
            const int o0 = (P[0].lo + m) << 4, o1 = (P[1].lo - c1 + m) << 4,
                      o2 = (P[2].lo - c2 + m) << 4, o3 = (P[3].lo - c3 + m) << 4;
            int jj[U];  // byte offsets; past the last piece: into the slack at most
            float4 q[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int mu = m + u;
                jj[u] = (mu < c1 ? o0 : mu < c2 ? o1 : mu < c3 ? o2 : o3) + 16 * u;
            }
#pragma unroll
            for (int u = 0; u < U; u++)
                q[u] = *reinterpret_cast<const float4 *>(pbase + (uint32_t)jj[u]);
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int mu = m + u;
                const bool inb = mu >= c2;
                const bool g1 = inb ? mu >= c3 : mu >= c1;
                const float3 a = make_float3(inb ? axb : axa, inb ? ayb : aya, g1 ? azs[1] : azs[0]);
                const float3 pk = make_float3(inb ? pxb : pxa, inb ? pyb : pya, g1 ? pks[1] : pks[0]);
                const bool hit = (mu < tot) & (jj[u] != io) & test_cand<true>(q[u], a, pk, R2);
                hr.put(jj[u], hit);
                img |= hit & ((inb ? sxb : sxa) | (g1 ? sz1 : sz0));
            }
            hr.flush_if_due(gl, cap);
        }
    };
    const Piece none{0, 0};
    // symmetric-list systems need every list in ascending slot order: each
    // lane walks its pieces sorted by their first slot (a window is one
    // ascending slot range and windows do not overlap)
    const bool sorted = d.zb == -5;
    int ord[18];
#pragma unroll
    for (int t = 0; t < 18; t++) ord[t] = t;
    if (sorted) {
        int key[18];
#pragma unroll
        for (int t = 0; t < 18; t++) key[t] = w[t / 2][t % 2].len > 0 ? w[t / 2][t % 2].lo : INT_MAX;
        // odd-even transposition sort of (key, piece) pairs
#pragma unroll
        for (int r = 0; r < 18; r++)
#pragma unroll
            for (int t = r & 1; t + 1 < 18; t += 2) {
                const bool sw = key[t + 1] < key[t];
                const int k0 = key[t], o0 = ord[t];
                key[t] = sw ? key[t + 1] : k0;
                ord[t] = sw ? ord[t + 1] : o0;
                key[t + 1] = sw ? k0 : key[t + 1];
                ord[t + 1] = sw ? o0 : ord[t + 1];
            }
    }
    if (!zwrap && !sorted) {
        // pairs of opposite columns, then the particle's own column
#pragma unroll
        for (int pr = 0; pr < 4; pr++)
            walk(w[pr][0], w[8 - pr][0], pr, 8 - pr, shx[pr], shx[8 - pr], 0, 0,
                 std::false_type{});
        walk(w[4][0], none, 4, 4, shx[4], false, 0, 0, std::true_type{});
    } else if (!sorted) {
        // some lane's column wraps in z: pairs of opposite columns with both
        // z-pieces of each (together a column's pieces span the z-range of an
        // unwrapped window), then the particle's own column
        const bool sz0 = azs[0] != 0.f || pks[0] != pi.z, sz1 = azs[1] != 0.f || pks[1] != pi.z;
#pragma unroll 1
        for (int pr = 0; pr < 5; pr++) {
            Piece P[4] = {none, none, none, none};
            bool sxa = false, sxb = false;
#pragma unroll
            for (int t = 0; t < 5; t++) {
                P[0] = t == pr ? w[t][0] : P[0];
                P[1] = t == pr ? w[t][1] : P[1];
                sxa = t == pr ? shx[t] : sxa;
                if (t < 4) {
                    P[2] = t == pr ? w[8 - t][0] : P[2];
                    P[3] = t == pr ? w[8 - t][1] : P[3];
                    sxb = t == pr ? shx[8 - t] : sxb;
                }
            }
            walk4(P, pr, 8 - pr, sxa, sxb, sz0, sz1);
        }
    } else {
        // ascending slot order: every piece of every column on its own (one
        // copy of the walk; the piece is picked from registers by a select
        // chain)
#pragma unroll 1
        for (int q = 0; q < 18; q++) {
            int kg = 0;
#pragma unroll
            for (int t = 0; t < 18; t++) kg = t == q ? ord[t] : kg;
            Piece P = none;
            bool shk = false;
#pragma unroll
            for (int t = 0; t < 18; t++) {
                P = t == kg ? w[t / 2][t % 2] : P;
                shk = t == kg ? shx[t / 2] : shk;
            }
            const int k = kg >> 1, g = kg & 1;
            const float az = g ? azs[1] : azs[0], pz = g ? pks[1] : pks[0];
            walk(P, none, k, k, shk || az != 0.f || pz != pi.z, false, g, g, std::true_type{});
        }
    }
    if (active) {
        // the unwritten entries, padded with the far-away slot to a multiple of
        // eight (a list that overflowed ends at the capacity)
        const int c = hr.finish(gl, cap, d.dummy);
        st.nnb[i] = (uint32_t)c | (img ? kWrapBit : 0u);
        note_overflow(st, hr.found(), cap);
    }
    copy_back(st, i);
}

// Debug builds: every list just built holds at most cap entries, all slots of
// its own system, none of them the particle itself and none twice, followed
// by the far-away slot up to a multiple of eight.
__global__ __launch_bounds__(kBlock) void k_check_lists(State st, int cap, int cap4) {
    const int s = block_system(st);
    if (!rebuilding(st, s)) return;
    const SysDesc &d = st.sys[s];
    const int64_t i = global_slot();
    if (i - d.slot_base >= d.n) return;
    const int c = (int)(st.nnb[i] & ~kWrapBit);
    bool bad = c < 0 || c > cap;
    const int c8 = bad ? 0 : min((c + 7) & ~7, 4 * cap4);
    for (int k = 0; k < c8 && !bad; k++) {
        const int j = st.nbr[nbr_index(i, k, cap4)];
        if (k < c) {
            bad = (unsigned)(j - d.slot_base) >= (unsigned)d.n || j == (int)i;
            for (int k2 = 0; k2 < k && !bad; k2++) bad = st.nbr[nbr_index(i, k2, cap4)] == j;
        } else {
            bad = j != d.dummy;
        }
    }
    if (bad) st.ctl->bad_index = 1;
}

// Longest list and total entries of the current lists (on request only): a
// grid-stride pass, reduced per workgroup, one pair of atomics per workgroup.
__global__ __launch_bounds__(256) void k_list_stats(State st, int64_t nslots) {
    __shared__ int smx[4];
    __shared__ unsigned long long ssm[4];
    int mx = 0;
    unsigned long long sm = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nslots;
         i += (int64_t)gridDim.x * 256) {
        const int c = (int)(st.nnb[i] & ~kWrapBit);
        mx = max(mx, c);
        sm += (unsigned long long)c;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, __shfl_xor(mx, o, 64));
        sm += __shfl_xor(sm, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) smx[w] = mx, ssm[w] = sm;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; k++) mx = max(mx, smx[k]), sm += ssm[k];
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
    if (c->n_ls_blocks > 0)  // four one-wavefront workgroups per particle workgroup
        hipLaunchKernelGGL(k_verlet_ls, dim3(4 * c->n_ls_blocks), dim3(kWave), 0, c->stream,
                           c->st, c->pa_blocks + c->n_pa_blocks + c->n_grp_blocks, c->R2, c->cap,
                           c->cap4);
    if (c->n_grp_blocks > 0) {
        // four 64-slot rows per particle workgroup
        const dim3 grid(4 * c->n_grp_blocks);
        const int lcap4 = c->cap4 < kRowGroups ? c->cap4 : kRowGroups;
        const size_t lds = (size_t)lcap4 * 64 * sizeof(int4);
        const int32_t *blocks = c->pa_blocks + c->n_pa_blocks;
        switch (c->tune_zb) {
        case 4:
            hipLaunchKernelGGL(k_verlet_grp<4>, grid, dim3(256), lds, c->stream, c->st, blocks,
                               c->R2, c->cap, c->cap4, lcap4);
            break;
        case 16:
            hipLaunchKernelGGL(k_verlet_grp<16>, grid, dim3(1024), lds, c->stream, c->st, blocks,
                               c->R2, c->cap, c->cap4, lcap4);
            break;
        default:
            hipLaunchKernelGGL(k_verlet_grp<8>, grid, dim3(512), lds, c->stream, c->st, blocks,
                               c->R2, c->cap, c->cap4, lcap4);
        }
    }
    if (kChecked) return launch_check_lists(c);
    return hipGetLastError();
}

hipError_t launch_check_lists(fpm_ctx *c) {
    hipLaunchKernelGGL(k_check_lists, dim3(c->nblk), dim3(kBlock), 0, c->stream, c->st, c->cap,
                       c->cap4);
    return hipGetLastError();
}

hipError_t launch_list_stats(fpm_ctx *c) {
    hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(64), 0, c->stream, c->st.ctl);
    const unsigned g = grid_for(c->n_slots, 256);
    hipLaunchKernelGGL(k_list_stats, dim3(g < 512 ? g : 512), dim3(256), 0, c->stream, c->st,
                       c->n_slots);
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
