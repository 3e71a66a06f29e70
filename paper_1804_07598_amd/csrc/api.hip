// Host side of the C ABI declared in include/fpm.h: argument checks, the
// workspace layout, the order of kernel launches and the graphs of the step
// loops.
#include <math.h>
#include <string.h>

#include <new>

#include "fpm_internal.h"

using namespace fpm;

namespace {

int fail(fpm_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(fpm_ctx *c, hipError_t e, const char *where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(c, FPM_EHIP, m);
}

#define HIPCHK(c, expr)                                      \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int cap4_for(int cap) { return (cap + 7) / 8 * 2; }

// Launch geometry and device tables of a batch holding n particles in total.
struct Plan {
    std::vector<SysHost> sys;
    std::vector<SysDesc> desc;
    std::vector<int32_t> blk2sys, item2sys, pa_blocks, grp_blocks, ls_blocks;
    int64_t n_slots = 0;
    int nblk = 0, ncells_total = 0, noff_total = 0, nitems = 0, max_ncells = 0;
    int max_sys_blocks = 0;
};

// Particles per system: the batch counts, or all n in the single box.
bool system_counts(const fpm_ctx *c, int64_t n, std::vector<int64_t> &cnt) {
    if (c->counts.empty()) {
        cnt.assign(1, n);
        return c->boxes.size() == 1;
    }
    int64_t tot = 0;
    for (int64_t k : c->counts) tot += k;
    cnt = c->counts;
    return tot == n;
}

constexpr int kShortListCap = 48;
constexpr int64_t kLockstepMinSlots = 131072;  // 2048 wavefronts: two per SIMD

Plan make_plan(const fpm_ctx *c, const std::vector<int64_t> &cnt) {
    Plan P;
    const int nsys = (int)cnt.size();
    int64_t slot = 0, caller = 0;
    int blk = 0, cell = 0, offb = 0, item = 0;
    int64_t total = 0;
    for (int64_t v : cnt) total += v;
    // contexts built by lockstep windows build grids of at most two cells per
    // axis in the same launch (every particle's candidates: the whole system)
    const bool ls_ctx = !c->sym && (c->tune_verlet_path == 5 ||
                                    (c->tune_verlet_path == 0 && c->cap > kShortListCap &&
                                     total >= kLockstepMinSlots));
    for (int s = 0; s < nsys; s++) {
        SysHost h{};
        SysDesc &d = h.d;
        d.box = c->boxes[s];
        d.n = (int32_t)cnt[s];
        d.n_pad = (int32_t)((cnt[s] + 1 + kBlock - 1) / kBlock * kBlock);  // >= 1 padding slot
        d.slot_base = (int32_t)slot;
        d.blk_base = blk;
        d.ncells = d.box.nc[0] * d.box.nc[1] * d.box.nc[2];
        d.cell_base = cell;
        d.off_base = offb;
        // Verlet build of the system (zb): > 0 column workgroups, 0 particle by
        // particle over whole cells, -1 particle by particle over candidate
        // windows, -2 lane groups over candidate windows, -3 lane groups over
        // whole cells, -4 lockstep windows, -5 lockstep windows in ascending
        // slot order (symmetric half lists).  Automatic choice, with the list
        // capacity standing in for the list length (unknown before the first
        // build): capacities up to kShortListCap take -1 (short lists come
        // from column runs of a few candidates, which would leave most lanes
        // of a group idle: 688,380 grains, about 6 entries, 89 us against
        // 206 us); longer lists take -4 for contexts of at least
        // kLockstepMinSlots particles, all systems together (1M LJ atoms, 76
        // entries: 452 against 518 us; 512 boxes of 256..8192 atoms, 2.2M in
        // all: 658 against 724 us per step) and -2 below that, where the
        // lockstep build's one wavefront per 64 particles leaves the SIMDs
        // short of waves (32,768-atom mixture: 130 against 55 us); grids of
        // fewer than three cells per axis take
        // -3 (built in the lockstep launch when -4 is the context's choice and
        // the grid has at most two cells per axis).
        const bool big = d.box.nc[0] >= 3 && d.box.nc[1] >= 3 && d.box.nc[2] >= 3;
        const bool auto_groups = c->tune_verlet_path == 0 && c->cap > kShortListCap;
        const bool many = total >= kLockstepMinSlots;
        if (c->sym)  // symmetric half lists need lists in ascending slot order
            d.zb = big ? -5 : 0;
        else if (c->tune_verlet_path == 1)
            d.zb = 0;
        else if (c->tune_verlet_path == 5 || (auto_groups && big && many))
            d.zb = big ? -4 : -3;
        else if (c->tune_verlet_path == 4 || auto_groups)
            d.zb = big ? -2 : -3;
        else if (c->tune_verlet_path == 3 || c->tune_verlet_path == 0)
            d.zb = big ? -1 : 0;
        else
            d.zb = verlet_zblock(cnt[s], d.ncells, d.box.nc, c->tune_zb);
        d.nzb = d.zb > 0 ? (d.box.nc[2] + d.zb - 1) / d.zb : 0;
        d.item_base = item;
        d.dummy = (int32_t)(slot + cnt[s]);
        d.caller_base = (int32_t)caller;
        h.nblk = d.n_pad / kBlock;
        h.nitems = d.zb > 0 ? d.box.nc[0] * d.box.nc[1] * d.nzb : 0;
        const bool tiny = d.box.nc[0] <= 2 && d.box.nc[1] <= 2 && d.box.nc[2] <= 2;
        const bool ls = d.zb == -4 || d.zb == -5 || (d.zb == -3 && ls_ctx && tiny);
        for (int b = 0; b < h.nblk; b++) {
            P.blk2sys.push_back(s);
            if (d.zb == 0 || d.zb == -1) P.pa_blocks.push_back(blk + b);
            if ((d.zb == -2 || d.zb == -3) && !ls) P.grp_blocks.push_back(blk + b);
            if (ls) P.ls_blocks.push_back(blk + b);
        }
        for (int q = 0; q < h.nitems; q++) P.item2sys.push_back(s);
        slot += d.n_pad;
        caller += cnt[s];
        blk += h.nblk;
        cell += d.ncells;
        offb += d.ncells + 1;
        item += h.nitems;
        if (d.ncells > P.max_ncells) P.max_ncells = d.ncells;
        if (h.nblk > P.max_sys_blocks) P.max_sys_blocks = h.nblk;
        P.sys.push_back(h);
        P.desc.push_back(d);
    }
    P.n_slots = slot;
    P.nblk = blk;
    P.ncells_total = cell;
    P.noff_total = offb;
    P.nitems = item;
    return P;
}

// Workspace layout of a plan; with base == nullptr only the size is computed.
size_t layout(const fpm_ctx *c, const Plan &P, char *base, State *st,
              int32_t **pa_blocks = nullptr) {
    const int64_t ns = P.n_slots;
    const int nsys = (int)P.sys.size();
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    State s{};
    // positions: kPosSlack slots past the end, which the lockstep build's
    // walks may read (and never test) beyond a lane's last window
    for (int k = 0; k < 2; k++) s.pos[k] = (float4 *)take((ns + kPosSlack) * sizeof(float4));
    for (int k = 0; k < 2; k++) s.vel[k] = (float4 *)take(ns * sizeof(float4));
    for (int k = 0; k < 2; k++) s.id[k] = (int32_t *)take(ns * sizeof(int32_t));
    s.frc = (float4 *)take(ns * sizeof(float4));
    s.xbuild = (float4 *)take(ns * sizeof(float4));
    s.cid = (int32_t *)take(ns * sizeof(int32_t));
    s.rnk = (int32_t *)take(ns * sizeof(int32_t));
    s.tmp = (int4 *)take(ns * sizeof(int4));
    s.cnt = (int32_t *)take(((size_t)P.ncells_total + 4) * sizeof(int32_t));
    s.off = (int32_t *)take(((size_t)P.noff_total + 4) * sizeof(int32_t));
    s.sub = (int32_t *)take(((size_t)P.ncells_total * 8 + 4) * sizeof(int32_t));
    s.tsum = (int32_t *)take(((size_t)P.ncells_total / 4096 + 4) * sizeof(int32_t));
    s.nbr = (int32_t *)take((size_t)ns * cap4_for(c->cap) * 4 * sizeof(int32_t));
    s.nnb = (uint32_t *)take(ns * sizeof(uint32_t));
    s.part = (double *)take((size_t)P.nblk * kSlots * sizeof(double));
    s.ring = (double *)take((size_t)P.nblk * kRingRows * 8 * sizeof(double));
    if (c->sym) {
        const size_t ent = (size_t)ns * cap4_for(c->cap) * 4;
        s.sbuf = (double *)take(ent * sizeof(double));
        s.tsym = (uint16_t *)take(ent * sizeof(uint16_t));
        s.plo = (int32_t *)take(ns * sizeof(int32_t));
        s.fown = (double *)take((size_t)ns * 3 * sizeof(double));
    }
    s.aux = (float4 *)take(ns * sizeof(float4));
    for (int k = 0; k < 2; k++) s.old[k] = (float4 *)take(ns * sizeof(float4));
    if (c->dem_cap > 0) {
        int64_t ncall = 0;
        for (const SysDesc &d : P.desc) ncall += d.n;
        const size_t hslots = (size_t)ncall * c->dem_cap;
        s.hl = (float4 *)take((size_t)ns * cap4_for(c->cap) * 4 * sizeof(float4));
        s.hid = (int32_t *)take(hslots * sizeof(int32_t));
        s.hu = (float4 *)take(hslots * sizeof(float4));
        s.ncon = (int32_t *)take((size_t)ncall * sizeof(int32_t));
        s.keep_old = 1;
    }
    s.ctl = (Ctl *)take(sizeof(Ctl));
    s.sctl = (SysCtl *)take(nsys * sizeof(SysCtl));
    s.sys = (const SysDesc *)take(nsys * sizeof(SysDesc));
    s.blk2sys = (const int32_t *)take(P.blk2sys.size() * sizeof(int32_t));
    s.item2sys = (const int32_t *)take((P.item2sys.size() + 1) * sizeof(int32_t));
    char *pa = take((P.pa_blocks.size() + P.grp_blocks.size() + P.ls_blocks.size() + 1) *
                    sizeof(int32_t));
    s.nsys = nsys;
    s.pstride = P.nblk;
    if (st) *st = s;
    if (pa_blocks) *pa_blocks = (int32_t *)pa;
    return off;
}

void drop_graphs(fpm_ctx *c) {
    for (hipGraphExec_t *g :
         {&c->g_pow[0], &c->g_pow[1], &c->g_pow[2], &c->g_pow[3], &c->g_one, &c->g_last[0],
          &c->g_last[1], &c->s_first, &c->s_chunk, &c->s_one, &c->d_chunk, &c->d_one}) {
        if (*g) (void)hipGraphExecDestroy(*g);
        *g = nullptr;
    }
}

int ready(fpm_ctx *c) {
    if (!c) return FPM_EINVAL;
    if (!c->have_particles) return fail(c, FPM_EINVAL, "no particles set");
    return FPM_OK;
}

// Brackets an eager launch with two events when profiling is on (never while
// a graph is being captured).
template <class F>
hipError_t timed(fpm_ctx *c, const char *name, F &&launch) {
    if (!c->profiling || (c->cap_stream && c->stream == c->cap_stream)) return launch();
    fpm_ctx::Timed t{name, nullptr, nullptr};
    hipError_t e = hipEventCreate(&t.start);
    if (e == hipSuccess) e = hipEventCreate(&t.stop);
    if (e == hipSuccess) e = hipEventRecord(t.start, c->stream);
    if (e != hipSuccess) return e;
    e = launch();
    hipError_t e2 = hipEventRecord(t.stop, c->stream);
    c->timed.push_back(t);
    return e != hipSuccess ? e : e2;
}

void drop_timers(fpm_ctx *c) {
    for (auto &t : c->timed) {
        if (t.start) (void)hipEventDestroy(t.start);
        if (t.stop) (void)hipEventDestroy(t.stop);
    }
    c->timed.clear();
}

// Gated neighbour-structure refresh: every kernel returns at once unless the
// device rebuild flag is set.  The flag is cleared (and the build accounted)
// by the next finalize with kFinBuild.
// With DEM on, the contact history follows the lists: exported to caller-keyed
// rows before the cell sort, imported into the new lists after the build.
// defer_import: the DEM force kernel that follows imports the history.
hipError_t refresh_lists(fpm_ctx *c, bool defer_import = false) {
    hipError_t e = hipSuccess;
    const bool exp = c->dem_cap > 0 && !c->dem_exported;
    e = timed(c, "cell_build", [&] { return launch_cell_build(c, exp); });
    if (e == hipSuccess) e = timed(c, "verlet_build", [&] { return launch_verlet_build(c); });
    if (e == hipSuccess && c->sym) e = launch_sym_index(c);
    if (e == hipSuccess && c->dem_cap > 0) {
        if (!defer_import) e = launch_dem_import(c);
        c->dem_exported = false;
    }
    return e;
}

// Eager refresh that leaves the flag clear.
hipError_t refresh_and_account(fpm_ctx *c) {
    hipError_t e = refresh_lists(c);
    if (e == hipSuccess) e = launch_finalize(c, kFinBuild, nullptr, nullptr);
    if (e == hipSuccess) c->build_pending = false;
    return e;
}

constexpr int kChunk = 25;  // steps per captured graph (SPH and DEM loops)
constexpr int kPowSteps[4] = {16, 8, 4, 2};  // LJ loops: steps of the even graphs
static_assert(kPowSteps[0] <= kRingRows, "a graph's steps must fit the partials ring");

template <class F>
int capture(fpm_ctx *c, F &&body, hipGraphExec_t *out) {
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) e = body();
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = user;
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(c, e, "graph capture");
    }
    if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
    return FPM_OK;
}

// Launches recorded by `body` see the state of step parity `par`: the rebuild
// flag copy par, and for odd steps the two position buffers exchanged, so that
// every step reads its positions from buffer 0 of its own view and writes the
// drifted ones to buffer 1 (the caller-visible buffer 0 holds the positions of
// even steps).
template <class F>
hipError_t with_parity(fpm_ctx *c, int par, F &&body) {
    const State keep = c->st;
    c->st.par = par;
    if (par) {
        c->st.pos[0] = keep.pos[1];
        c->st.pos[1] = keep.pos[0];
    }
    hipError_t e = body();
    c->st = keep;
    return e;
}

// `count` LJ velocity-Verlet steps from a step of parity par0: per step the
// gated rebuild, then the force kernel with the closing half kick and (but for
// a last step) the next step's opening half kick and drift; then the thermo
// rows of these steps.  The first opening half kick and drift of a loop run
// before it (fpm_step).  With `rec`, step k's positions (those its force
// kernel reads: the positions after step k) go to rec + 3 n k in caller order.
hipError_t lj_steps_body(fpm_ctx *c, const fpm_lj_params &p, float dt, double *thermo, int par0,
                         int count, bool last, float *rec = nullptr) {
    hipError_t e = hipSuccess;
    for (int k = 0; k < count && e == hipSuccess; k++)
        e = with_parity(c, (par0 + k) & 1, [&] {
            hipError_t x = refresh_lists(c);
            if (x == hipSuccess && rec)
                x = launch_gather_out(c, rec + (size_t)k * 3 * (size_t)c->n, nullptr, nullptr,
                                      nullptr, nullptr);
            if (x == hipSuccess) x = launch_lj_step(c, p, dt, last && k == count - 1, k);
            return x;
        });
    if (e == hipSuccess) e = launch_finalize_rows(c, count, thermo);
    return e;
}

// One SPH step with the device time step: kick-drift-kick (the closing half
// kick of the previous step fused with this step's opening one) or Verlet.
hipError_t sph_step_body(fpm_ctx *c, const fpm_sph_params &p, double *hist, bool first) {
    hipError_t e = p.scheme == 1
                       ? launch_sph_verlet(c, p)
                       : launch_sph_integrate(c, p, first ? kKickDriftFirst : kKickKickDrift);
    // the step kernel raised the rebuild flag if needed; the rates kernel
    // accounts the rebuild and clears the flag
    if (e == hipSuccess) e = refresh_lists(c);
    if (e == hipSuccess) e = launch_sph_rates(c, p);
    if (e == hipSuccess) e = launch_sph_finalize(c, p, 1, nullptr, hist);
    return e;
}

bool valid_lj(const fpm_lj_params *p) {
    if (!p || (p->n_types != 1 && p->n_types != 2)) return false;
    for (int k = 0; k < 3; k++)
        if (!(isfinite(p->eps[k]) && isfinite(p->sig[k]) && p->sig[k] > 0.f)) return false;
    return true;
}

bool valid_sph(const fpm_sph_params *p) {
    if (!p) return false;
    const float v[] = {p->h, p->mass, p->rho0, p->c0, p->gamma, p->cfl};
    for (float x : v)
        if (!(isfinite(x) && x > 0.f)) return false;
    return isfinite(p->alpha) && p->alpha >= 0.f && isfinite(p->eta2) && p->eta2 >= 0.f &&
           isfinite(p->g[0]) && isfinite(p->g[1]) && isfinite(p->g[2]) && isfinite(p->cbar) &&
           (p->kernel == 0 || p->kernel == 1) && (p->scheme == 0 || p->scheme == 1) &&
           (p->scheme == 0 || p->verlet_every >= 1);
}

int dem_ready(fpm_ctx *c, const fpm_dem_params *p) {
    int r = ready(c);
    if (r) return r;
    if (c->dem_cap <= 0) return fail(c, FPM_EINVAL, "DEM storage not set (fpm_set_dem)");
    if (!p) return fail(c, FPM_EINVAL, "null DEM params");
    const float v[] = {p->R, p->mass, p->inertia, p->dt};
    for (float x : v)
        if (!(isfinite(x) && x > 0.f)) return fail(c, FPM_EINVAL, "bad DEM params");
    const float w[] = {p->kn, p->kt, p->gn, p->gt, p->mu};
    for (float x : w)
        if (!(isfinite(x) && x >= 0.f)) return fail(c, FPM_EINVAL, "bad DEM params");
    if (!(isfinite(p->g[0]) && isfinite(p->g[1]) && isfinite(p->g[2])) || p->walls < 0 ||
        p->walls > 3)
        return fail(c, FPM_EINVAL, "bad DEM params");
    if ((double)c->r_cut + (double)c->skin < 2.0 * (double)p->R)
        return fail(c, FPM_EINVAL, "the list radius must cover 2R");
    return FPM_OK;
}

}  // namespace

extern "C" {

int fpm_create(fpm_ctx **out, void *stream) {
    if (!out) return FPM_EINVAL;
    fpm_ctx *c = new (std::nothrow) fpm_ctx();
    if (!c) return FPM_EINVAL;
    c->stream = (hipStream_t)stream;
    *out = c;
    return FPM_OK;
}

int fpm_destroy(fpm_ctx *c) {
    if (!c) return FPM_OK;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    drop_timers(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return FPM_OK;
}

const char *fpm_last_error(const fpm_ctx *c) { return c ? c->err.c_str() : "null context"; }

int fpm_set_systems(fpm_ctx *c, int32_t nsys, const float *L, const int32_t *per,
                    const int64_t *counts) {
    if (!c) return FPM_EINVAL;
    if (nsys < 1 || nsys > kMaxSystems) return fail(c, FPM_EINVAL, "system count out of range");
    if (!L || !per) return fail(c, FPM_EINVAL, "null box argument");
    int64_t tot = 0;
    for (int s = 0; s < nsys; s++) {
        for (int a = 0; a < 3; a++) {
            const float x = L[3 * s + a];
            if (!(isfinite(x) && x > 0.f)) return fail(c, FPM_EINVAL, "box side must be > 0");
            if (per[3 * s + a] != 0 && per[3 * s + a] != 1)
                return fail(c, FPM_EINVAL, "periodic flag must be 0/1");
        }
        if (counts) {
            if (counts[s] < 1) return fail(c, FPM_EINVAL, "every system needs a particle");
            tot += counts[s];
            if (tot > kMaxParticles) return fail(c, FPM_EINVAL, "particle count out of range");
        }
    }
    if (!counts && nsys != 1) return fail(c, FPM_EINVAL, "a batch needs its particle counts");
    c->boxes.assign(nsys, Box{});
    for (int s = 0; s < nsys; s++)
        for (int a = 0; a < 3; a++) {
            Box &b = c->boxes[s];
            b.L[a] = L[3 * s + a];
            b.half[a] = L[3 * s + a] * 0.5f;
            b.per[a] = per[3 * s + a];
        }
    c->counts.clear();
    if (counts) c->counts.assign(counts, counts + nsys);
    c->box_set = true;
    c->nbr_set = false;
    c->have_particles = false;
    drop_graphs(c);
    return FPM_OK;
}

int fpm_set_box(fpm_ctx *c, const float L[3], const int32_t per[3]) {
    return fpm_set_systems(c, 1, L, per, nullptr);
}

int fpm_set_neighbor_params(fpm_ctx *c, float r_cut, float skin, int32_t max_nbr) {
    if (!c) return FPM_EINVAL;
    if (!c->box_set) return fail(c, FPM_EINVAL, "set the box first");
    if (!(isfinite(r_cut) && r_cut > 0.f && isfinite(skin) && skin >= 0.f))
        return fail(c, FPM_EINVAL, "r_cut must be > 0 and skin >= 0");
    if (max_nbr < 1 || max_nbr > kMaxNbrCap) return fail(c, FPM_EINVAL, "max_nbr out of range");
    const double R = (double)r_cut + (double)skin;
    std::vector<Box> boxes = c->boxes;
    int64_t total = 0;
    for (Box &b : boxes) {
        int64_t ncells = 1;
        for (int a = 0; a < 3; a++) {
            if (b.per[a] && !(R < 0.5 * (double)b.L[a] * (1.0 - 1e-6)))
                return fail(c, FPM_ECUTOFF, "r_cut + skin must be below half the periodic box");
            const double m = floor((double)b.L[a] / (R * 1.000001));
            b.nc[a] = m < 1.0 ? 1 : (m > (1 << 20) ? (1 << 20) : (int)m);
            b.inv[a] = (float)b.nc[a] / b.L[a];
            ncells *= b.nc[a];
            if (ncells > ((int64_t)1 << 30)) return fail(c, FPM_EINVAL, "too many cells");
        }
        total += ncells + 1;
        if (total > ((int64_t)1 << 30)) return fail(c, FPM_EINVAL, "too many cells");
    }
    c->boxes = boxes;
    c->r_cut = r_cut;
    c->skin = skin;
    c->cap = max_nbr;
    c->cap4 = cap4_for(max_nbr);
    c->R2 = (float)(R * R);
    c->rc2 = (float)((double)r_cut * (double)r_cut);
    const double hs = 0.5 * (double)skin;
    c->disp2_thr = (float)(hs * hs);
    c->nbr_set = true;
    c->have_particles = false;
    drop_graphs(c);
    return FPM_OK;
}

int fpm_set_tuning(fpm_ctx *c, int32_t verlet_path, int32_t zblock, int32_t unroll) {
    if (!c) return FPM_EINVAL;
    if (verlet_path < 0 || verlet_path > 5) return fail(c, FPM_EINVAL, "verlet_path is 0..5");
    if (zblock < 0 || zblock > 64) return fail(c, FPM_EINVAL, "zblock out of range");
    if (verlet_path == 4 && zblock != 0 && zblock != 4 && zblock != 8 && zblock != 16)
        return fail(c, FPM_EINVAL, "lanes per particle (zblock of path 4) is 0, 4, 8 or 16");
    if (unroll != 0 && unroll != 4 && unroll != 8) return fail(c, FPM_EINVAL, "unroll is 0, 4 or 8");
    if (verlet_path != c->tune_verlet_path || zblock != c->tune_zb) c->have_particles = false;
    c->tune_verlet_path = verlet_path;
    c->tune_zb = zblock;
    c->tune_unroll = unroll;
    drop_graphs(c);
    return FPM_OK;
}

int fpm_workspace_size(fpm_ctx *c, int64_t n, size_t *bytes) {
    if (!c) return FPM_EINVAL;
    if (!bytes) return fail(c, FPM_EINVAL, "null size pointer");
    if (!c->nbr_set) return fail(c, FPM_EINVAL, "set box and neighbour parameters first");
    if (n < 1 || n > kMaxParticles) return fail(c, FPM_EINVAL, "particle count out of range");
    std::vector<int64_t> cnt;
    if (!system_counts(c, n, cnt)) return fail(c, FPM_EINVAL, "n differs from the batch total");
    *bytes = layout(c, make_plan(c, cnt), nullptr, nullptr);
    return FPM_OK;
}

int fpm_set_workspace(fpm_ctx *c, void *ws, size_t bytes) {
    if (!c) return FPM_EINVAL;
    if (!ws || ((uintptr_t)ws % kAlign) != 0)
        return fail(c, FPM_EINVAL, "workspace must be a 256-byte aligned device pointer");
    (void)hipStreamSynchronize(c->stream);
    c->ws = ws;
    c->ws_bytes = bytes;
    c->have_particles = false;
    drop_graphs(c);
    return FPM_OK;
}

// The bytes that fix a plan's device tables and workspace layout.
std::vector<char> plan_key(const fpm_ctx *c, const Plan &P) {
    std::vector<char> k;
    auto put = [&](const void *p, size_t bytes) {
        const char *b = static_cast<const char *>(p);
        k.insert(k.end(), b, b + bytes);
    };
    const void *ws = c->ws;
    put(&ws, sizeof(ws));
    put(&P.n_slots, sizeof(P.n_slots));
    put(P.desc.data(), P.desc.size() * sizeof(SysDesc));
    for (const std::vector<int32_t> *v :
         {&P.blk2sys, &P.item2sys, &P.pa_blocks, &P.grp_blocks, &P.ls_blocks}) {
        const size_t m = v->size();
        put(&m, sizeof(m));
        put(v->data(), m * sizeof(int32_t));
    }
    return k;
}

// Lays out the workspace for plan P (n particles) and uploads its tables;
// waits for the copies.
hipError_t upload_plan(fpm_ctx *c, const Plan &P, int64_t n) {
    layout(c, P, (char *)c->ws, &c->st, &c->pa_blocks);
    c->sys = P.sys;
    c->nsys = (int)P.sys.size();
    c->n = n;
    c->n_slots = P.n_slots;
    c->nblk = P.nblk;
    c->ncells_total = P.ncells_total;
    c->noff_total = P.noff_total;
    c->nitems = P.nitems;
    c->n_pa_blocks = (int)P.pa_blocks.size();
    c->n_grp_blocks = (int)P.grp_blocks.size();
    c->n_ls_blocks = (int)P.ls_blocks.size();
    c->max_ncells = P.max_ncells;
    c->max_sys_blocks = P.max_sys_blocks;
    // the tables are small; the copies finish before the host vectors go away
    const struct {
        void *dst;
        const std::vector<int32_t> *src;
    } tables[] = {{(void *)c->st.blk2sys, &P.blk2sys},
                  {(void *)c->st.item2sys, &P.item2sys},
                  {c->pa_blocks, &P.pa_blocks},  // then the lane-group and lockstep blocks
                  {c->pa_blocks + P.pa_blocks.size(), &P.grp_blocks},
                  {c->pa_blocks + P.pa_blocks.size() + P.grp_blocks.size(), &P.ls_blocks}};
    hipError_t e = hipMemcpyAsync((void *)c->st.sys, P.desc.data(),
                                  P.desc.size() * sizeof(SysDesc), hipMemcpyHostToDevice,
                                  c->stream);
    for (const auto &t : tables)
        if (e == hipSuccess && !t.src->empty())
            e = hipMemcpyAsync(t.dst, t.src->data(), t.src->size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

int fpm_set_particles(fpm_ctx *c, int64_t n, const float *pos, const float *vel,
                      const int32_t *type) {
    if (!c) return FPM_EINVAL;
    if (!c->nbr_set) return fail(c, FPM_EINVAL, "set box and neighbour parameters first");
    if (n < 1 || n > kMaxParticles) return fail(c, FPM_EINVAL, "particle count out of range");
    if (!pos) return fail(c, FPM_EINVAL, "null positions");
    std::vector<int64_t> cnt;
    if (!system_counts(c, n, cnt)) return fail(c, FPM_EINVAL, "n differs from the batch total");
    Plan P = make_plan(c, cnt);
    const size_t need = layout(c, P, nullptr, nullptr);
    if (!c->ws || c->ws_bytes < need) return fail(c, FPM_ENOWS, "workspace missing or too small");
    std::vector<char> key = plan_key(c, P);
    if (!(c->have_particles && key == c->plan_key)) {
        // a new layout: tables uploaded, captured graphs dropped
        c->have_particles = false;
        drop_graphs(c);
        HIPCHK(c, upload_plan(c, P, n));
        c->plan_key = std::move(key);
    }  // else the same layout and tables: the state is re-initialised in place
    HIPCHK(c, launch_fill_i32(c->stream, c->st.cnt, c->ncells_total, 0));
    HIPCHK(c, launch_init_state(c, pos, vel, type));
    HIPCHK(c, launch_force_rebuild(c));
    if (c->dem_cap > 0) {  // no history yet: nothing to export before the first build
        HIPCHK(c, launch_dem_clear(c));
        c->dem_exported = true;
    }
    HIPCHK(c, refresh_and_account(c));
    if (c->dem_cap > 0) HIPCHK(c, launch_dem_set_omega(c, nullptr));
    c->have_particles = true;
    c->forces_valid = false;
    c->sph_restart = true;
    return FPM_OK;
}

int fpm_system_info(fpm_ctx *c, int32_t s, int64_t out[8]) {
    int r = ready(c);
    if (r) return r;
    if (!out || s < 0 || s >= c->nsys) return fail(c, FPM_EINVAL, "bad system index or output");
    const SysHost &h = c->sys[s];
    out[0] = h.d.n;
    out[1] = h.d.caller_base;
    out[2] = h.d.ncells;
    out[3] = h.d.off_base;
    for (int a = 0; a < 3; a++) out[4 + a] = h.d.box.nc[a];
    out[7] = h.d.zb;
    return FPM_OK;
}

int fpm_set_positions(fpm_ctx *c, const float *pos) {
    int r = ready(c);
    if (r) return r;
    if (!pos) return fail(c, FPM_EINVAL, "null positions");
    HIPCHK(c, launch_set_positions(c, pos));  // raises the rebuild flag if needed
    c->forces_valid = false;
    c->sph_restart = true;
    return FPM_OK;
}

int fpm_set_density(fpm_ctx *c, const float *rho) {
    int r = ready(c);
    if (r) return r;
    if (!rho) return fail(c, FPM_EINVAL, "null density");
    HIPCHK(c, launch_set_density(c, rho));
    c->forces_valid = false;
    c->sph_restart = true;
    return FPM_OK;
}

int fpm_get_particles(fpm_ctx *c, float *pos, float *vel, float *frc) {
    int r = ready(c);
    if (r) return r;
    HIPCHK(c, launch_gather_out(c, pos, vel, frc, nullptr, nullptr));
    return FPM_OK;
}

int fpm_get_sph(fpm_ctx *c, float *rho, float *drho) {
    int r = ready(c);
    if (r) return r;
    HIPCHK(c, launch_gather_out(c, nullptr, nullptr, nullptr, rho, drho));
    return FPM_OK;
}

int fpm_build_cell_list(fpm_ctx *c) {
    int r = ready(c);
    if (r) return r;
    HIPCHK(c, launch_force_rebuild(c));
    const bool exp = c->dem_cap > 0 && !c->dem_exported;  // the sort invalidates the list history
    HIPCHK(c, timed(c, "cell_build", [&] { return launch_cell_build(c, exp); }));
    if (exp) c->dem_exported = true;
    HIPCHK(c, launch_copy_back(c));
    c->build_pending = true;  // flags stay set: the Verlet lists are rebuilt on next use
    c->forces_valid = false;
    return FPM_OK;
}

int fpm_get_cell_list(fpm_ctx *c, int32_t ncell[3], int32_t *offsets, int32_t *order) {
    int r = ready(c);
    if (r) return r;
    if (ncell)
        for (int a = 0; a < 3; a++) ncell[a] = c->sys[0].d.box.nc[a];
    if (offsets || order) HIPCHK(c, launch_cells_out(c, offsets, order));
    return FPM_OK;
}

int fpm_build_verlet(fpm_ctx *c) {
    int r = ready(c);
    if (r) return r;
    HIPCHK(c, launch_force_rebuild(c));
    HIPCHK(c, refresh_and_account(c));
    c->forces_valid = false;
    return FPM_OK;
}

int fpm_get_neighbors(fpm_ctx *c, int32_t *counts, int32_t *cols) {
    int r = ready(c);
    if (r) return r;
    if (!counts || !cols) return fail(c, FPM_EINVAL, "null output");
    HIPCHK(c, refresh_and_account(c));
    HIPCHK(c, launch_neighbors_out(c, counts, cols));
    Ctl h;
    HIPCHK(c, hipMemcpyAsync(&h, c->st.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h.overflow) return fail(c, FPM_EOVERFLOW, "Verlet list exceeded max_nbr");
    return FPM_OK;
}

int fpm_lj_forces(fpm_ctx *c, const fpm_lj_params *p, double *out) {
    int r = ready(c);
    if (r) return r;
    if (!valid_lj(p)) return fail(c, FPM_EINVAL, "bad LJ params");
    HIPCHK(c, refresh_and_account(c));
    HIPCHK(c, timed(c, "lj_force", [&] { return launch_lj_forces(c, *p); }));
    HIPCHK(c, launch_finalize(c, kFinForce, out, nullptr));
    c->forces_valid = true;
    c->sph = false;
    return FPM_OK;
}

int fpm_lj_force_vjp(fpm_ctx *c, const fpm_lj_params *p, const double *lam, double *gx,
                     double *gtheta) {
    int r = ready(c);
    if (r) return r;
    if (!valid_lj(p)) return fail(c, FPM_EINVAL, "bad LJ params");
    if (!lam || !gx) return fail(c, FPM_EINVAL, "null cotangent or output");
    HIPCHK(c, refresh_and_account(c));
    const AdjOut o{gx, nullptr, nullptr, nullptr, 0.0, kVjpPlain};
    HIPCHK(c, timed(c, "lj_vjp", [&] { return launch_lj_vjp(c, *p, lam, nullptr, o); }));
    if (gtheta) HIPCHK(c, launch_finalize(c, kFinVjp, gtheta, nullptr));
    return FPM_OK;
}

int fpm_lj_adjoint_step(fpm_ctx *c, const fpm_lj_params *p, float dt, const double *floss,
                        double *xbar, double *vbar, double *fbar, double *gtheta, int32_t last) {
    int r = ready(c);
    if (r) return r;
    if (!valid_lj(p)) return fail(c, FPM_EINVAL, "bad LJ params");
    if (!isfinite(dt)) return fail(c, FPM_EINVAL, "dt must be finite");
    if (!xbar || !vbar || !fbar) return fail(c, FPM_EINVAL, "null adjoint array");
    if (last != 0 && last != 1) return fail(c, FPM_EINVAL, "last must be 0 or 1");
    HIPCHK(c, refresh_and_account(c));
    const AdjOut o{xbar, vbar, fbar, floss, (double)dt, last ? kVjpLast : kVjpStep};
    HIPCHK(c, timed(c, "lj_vjp", [&] {
        return launch_lj_vjp(c, *p, fbar, last ? nullptr : vbar, o);
    }));
    if (gtheta) HIPCHK(c, launch_finalize(c, kFinVjp, gtheta, nullptr));
    return FPM_OK;
}

int fpm_lj_adjoint_sweep(fpm_ctx *c, const fpm_lj_params *p, float dt, int32_t nsteps,
                         const float *xs, const double *const *floss, double *xbar,
                         double *vbar, double *fbar, double *gtheta) {
    int r = ready(c);
    if (r) return r;
    if (!valid_lj(p)) return fail(c, FPM_EINVAL, "bad LJ params");
    if (!isfinite(dt) || nsteps < 0) return fail(c, FPM_EINVAL, "bad dt or step count");
    if (nsteps > 0 && (!xs || !floss)) return fail(c, FPM_EINVAL, "null positions or loss table");
    if (!xbar || !vbar || !fbar) return fail(c, FPM_EINVAL, "null adjoint array");
    // step k (latest first) at the positions reached after it, x_{k+1}: the
    // launches of fpm_set_positions followed by fpm_lj_adjoint_step, queued
    // without host synchronisation (the VJP kernel accounts a rebuild and
    // clears its flag)
    for (int32_t k = nsteps - 1; k >= 0; k--) {
        HIPCHK(c, launch_set_positions(c, xs + (size_t)k * 3 * (size_t)c->n));
        HIPCHK(c, refresh_lists(c));
        c->build_pending = false;
        const AdjOut o{xbar, vbar, fbar, floss[k], (double)dt, kVjpStep};
        HIPCHK(c, timed(c, "lj_vjp", [&] { return launch_lj_vjp(c, *p, fbar, vbar, o); }));
        if (gtheta) HIPCHK(c, launch_finalize(c, kFinVjp, gtheta, nullptr));
    }
    c->forces_valid = false;
    c->sph_restart = true;
    return FPM_OK;
}

int fpm_integrate(fpm_ctx *c, float dt, int32_t half) {
    int r = ready(c);
    if (r) return r;
    if (!isfinite(dt)) return fail(c, FPM_EINVAL, "dt must be finite");
    if (half != 0 && half != 1) return fail(c, FPM_EINVAL, "half must be 0 or 1");
    HIPCHK(c, timed(c, "integrate", [&] {
        return launch_integrate(c, dt, half ? kKickOnly : kKickDriftFirst);
    }));
    if (!half) {
        HIPCHK(c, launch_finalize(c, kFinDisp, nullptr, nullptr));
        c->forces_valid = false;
    }
    return FPM_OK;
}

int fpm_step(fpm_ctx *c, const fpm_lj_params *p, float dt, int32_t nsteps, double *thermo) {
    int r = ready(c);
    if (r) return r;
    if (!valid_lj(p)) return fail(c, FPM_EINVAL, "bad LJ params");
    if (!isfinite(dt) || nsteps < 0) return fail(c, FPM_EINVAL, "bad dt or step count");
    if (nsteps == 0) return FPM_OK;
    if (!c->forces_valid || c->build_pending || c->sph) {
        HIPCHK(c, refresh_and_account(c));
        HIPCHK(c, launch_lj_forces(c, *p));
        c->forces_valid = true;
    }
    c->sph = false;
    const bool same = c->g_one && c->g_dt == dt && c->g_thermo == thermo &&
                      memcmp(&c->g_prm, p, sizeof(*p)) == 0 && c->g_unroll == c->tune_unroll;
    if (!same) {
        drop_graphs(c);
        int e;
        const fpm_lj_params prm = *p;
        for (int g = 0; g < 4; g++) {
            e = capture(c, [&] { return lj_steps_body(c, prm, dt, thermo, 0, kPowSteps[g], false); },
                        &c->g_pow[g]);
            if (e) return e;
        }
        e = capture(c, [&] { return lj_steps_body(c, prm, dt, thermo, 0, 1, false); }, &c->g_one);
        if (e) return e;
        for (int par = 0; par < 2; par++) {
            e = capture(c, [&] { return lj_steps_body(c, prm, dt, thermo, par, 1, true); },
                        &c->g_last[par]);
            if (e) return e;
        }
        c->g_dt = dt;
        c->g_thermo = thermo;
        c->g_prm = *p;
        c->g_unroll = c->tune_unroll;
    }
    HIPCHK(c, launch_reset_step(c));
    // opening half kick and drift of the first step, its rebuild decision
    HIPCHK(c, launch_integrate(c, dt, kKickDriftFirst));
    HIPCHK(c, launch_finalize(c, kFinDisp, nullptr, nullptr));
    if (c->profiling) {
        // the same launches without graphs, each step's force kernel timed
        // ("lj_step") and its rebuild kernels too ("cell_build", "verlet_build")
        const fpm_lj_params prm = *p;
        for (int k = 0; k < nsteps; k++) {
            const bool last = k == nsteps - 1;
            HIPCHK(c, with_parity(c, k & 1, [&] {
                hipError_t x = refresh_lists(c);
                if (x == hipSuccess)
                    x = timed(c, "lj_step", [&] { return launch_lj_step(c, prm, dt, last, 0); });
                return x;
            }));
            HIPCHK(c, launch_finalize_rows(c, 1, thermo));
        }
        return FPM_OK;
    }
    // steps 0 .. nsteps-2 fused with the next step's opening, then the last step
    int left = nsteps - 1, step = 0;
    for (int g = 0; g < 4; g++)
        for (; left >= kPowSteps[g]; left -= kPowSteps[g], step += kPowSteps[g])
            HIPCHK(c, hipGraphLaunch(c->g_pow[g], c->stream));
    if (left == 1) {
        HIPCHK(c, hipGraphLaunch(c->g_one, c->stream));
        step += 1;
    }
    HIPCHK(c, hipGraphLaunch(c->g_last[step & 1], c->stream));
    return FPM_OK;
}

int fpm_step_record(fpm_ctx *c, const fpm_lj_params *p, float dt, int32_t nsteps, float *xs) {
    int r = ready(c);
    if (r) return r;
    if (!valid_lj(p)) return fail(c, FPM_EINVAL, "bad LJ params");
    if (!isfinite(dt) || nsteps < 0) return fail(c, FPM_EINVAL, "bad dt or step count");
    if (nsteps > 0 && !xs) return fail(c, FPM_EINVAL, "null position record");
    if (nsteps == 0) return FPM_OK;
    if (!c->forces_valid || c->build_pending || c->sph) {
        HIPCHK(c, refresh_and_account(c));
        HIPCHK(c, launch_lj_forces(c, *p));
        c->forces_valid = true;
    }
    c->sph = false;
    HIPCHK(c, launch_reset_step(c));
    HIPCHK(c, launch_integrate(c, dt, kKickDriftFirst));
    HIPCHK(c, launch_finalize(c, kFinDisp, nullptr, nullptr));
    // the launches of fpm_step's loop (steps fused with the next one's opening
    // half kick and drift, as bit for bit as separate calls), without graphs,
    // each step's positions recorded
    for (int32_t k0 = 0; k0 < nsteps; k0 += kPowSteps[0]) {
        const int cnt = nsteps - k0 < kPowSteps[0] ? nsteps - k0 : kPowSteps[0];
        HIPCHK(c, lj_steps_body(c, *p, dt, nullptr, k0 & 1, cnt, k0 + cnt == nsteps,
                                xs + (size_t)k0 * 3 * (size_t)c->n));
    }
    return FPM_OK;
}

int fpm_sph_rates(fpm_ctx *c, const fpm_sph_params *p, float *dt_out) {
    int r = ready(c);
    if (r) return r;
    if (!valid_sph(p)) return fail(c, FPM_EINVAL, "bad SPH params");
    if (c->nsys != 1) return fail(c, FPM_EINVAL, "SPH runs on a single system");
    HIPCHK(c, refresh_and_account(c));
    HIPCHK(c, timed(c, "sph_rates", [&] { return launch_sph_rates(c, *p); }));
    HIPCHK(c, launch_sph_finalize(c, *p, 0, dt_out, nullptr));
    c->sph = true;
    c->forces_valid = true;
    return FPM_OK;
}

int fpm_sph_step(fpm_ctx *c, const fpm_sph_params *p, int32_t nsteps, double *hist) {
    int r = ready(c);
    if (r) return r;
    if (!valid_sph(p)) return fail(c, FPM_EINVAL, "bad SPH params");
    if (c->nsys != 1) return fail(c, FPM_EINVAL, "SPH runs on a single system");
    if (nsteps < 0) return fail(c, FPM_EINVAL, "bad step count");
    if (nsteps == 0) return FPM_OK;
    // the Verlet scheme keeps the previous step's (v, rho), which the cell
    // sort must carry along; a switch of scheme restarts its step count
    const int keep = p->scheme == 1;
    if (c->st.keep_old != keep) {
        c->st.keep_old = keep;
        c->sph_restart = true;
        drop_graphs(c);
    }
    if (!keep) {
        c->sph_restart = true;
    } else if (c->sph_restart) {
        HIPCHK(c, launch_sph_restart(c));
        c->sph_restart = false;
    }
    if (!c->forces_valid || !c->sph || c->build_pending) {
        HIPCHK(c, refresh_and_account(c));
        HIPCHK(c, launch_sph_rates(c, *p));
        HIPCHK(c, launch_sph_finalize(c, *p, 0, nullptr, nullptr));
        c->forces_valid = true;
        c->sph = true;
    }
    const bool same = c->s_first && c->s_hist == hist && memcmp(&c->s_prm, p, sizeof(*p)) == 0;
    if (!same) {
        drop_graphs(c);
        const fpm_sph_params prm = *p;
        int e = capture(c, [&] { return sph_step_body(c, prm, hist, true); }, &c->s_first);
        if (e) return e;
        e = capture(c,
                    [&] {
                        hipError_t x = hipSuccess;
                        for (int s = 0; s < kChunk && x == hipSuccess; s++)
                            x = sph_step_body(c, prm, hist, false);
                        return x;
                    },
                    &c->s_chunk);
        if (e) return e;
        e = capture(c, [&] { return sph_step_body(c, prm, hist, false); }, &c->s_one);
        if (e) return e;
        c->s_hist = hist;
        c->s_prm = *p;
    }
    HIPCHK(c, launch_reset_step(c));
    HIPCHK(c, hipGraphLaunch(c->s_first, c->stream));
    int left = nsteps - 1;
    for (; left >= kChunk; left -= kChunk) HIPCHK(c, hipGraphLaunch(c->s_chunk, c->stream));
    for (; left > 0; left--) HIPCHK(c, hipGraphLaunch(c->s_one, c->stream));
    if (p->scheme == 0) HIPCHK(c, launch_sph_integrate(c, *p, kKickOnly));
    HIPCHK(c, launch_finalize(c, kFinBuild, nullptr, nullptr));
    return FPM_OK;
}

int fpm_set_symmetric(fpm_ctx *c, int32_t on) {
    if (!c) return FPM_EINVAL;
    if (on != 0 && on != 1) return fail(c, FPM_EINVAL, "on must be 0 or 1");
    if (on && c->dem_cap > 0) return fail(c, FPM_EINVAL, "symmetric lists are for LJ, not DEM");
    if (on && c->cap > 4096) return fail(c, FPM_EINVAL, "list capacity too large");
    c->sym = on != 0;
    c->have_particles = false;
    drop_graphs(c);
    return FPM_OK;
}

int fpm_set_dem(fpm_ctx *c, int32_t max_contacts) {
    if (!c) return FPM_EINVAL;
    if (max_contacts < 1 || max_contacts > 64) return fail(c, FPM_EINVAL, "max_contacts is 1..64");
    if (c->nsys > 1 || !c->counts.empty())
        return fail(c, FPM_EINVAL, "DEM runs on a single system");
    c->dem_cap = max_contacts;
    c->have_particles = false;
    drop_graphs(c);
    return FPM_OK;
}


int fpm_set_omega(fpm_ctx *c, const float *w) {
    int r = ready(c);
    if (r) return r;
    if (c->dem_cap <= 0) return fail(c, FPM_EINVAL, "DEM storage not set (fpm_set_dem)");
    HIPCHK(c, launch_dem_set_omega(c, w));
    return FPM_OK;
}

int fpm_dem_forces(fpm_ctx *c, const fpm_dem_params *p) {
    int r = dem_ready(c, p);
    if (r) return r;
    HIPCHK(c, refresh_and_account(c));
    HIPCHK(c, timed(c, "dem_forces", [&] { return launch_dem_forces(c, *p); }));
    c->forces_valid = false;
    return FPM_OK;
}

// One DEM step: gated rebuild (with the history export and import), forces
// and torques, leapfrog, finalize (accounts a rebuild, decides the next).
hipError_t dem_step_body(fpm_ctx *c, const fpm_dem_params &p) {
    hipError_t e = refresh_lists(c, true);
    if (e == hipSuccess) e = timed(c, "dem_forces", [&] { return launch_dem_forces(c, p, true); });
    if (e == hipSuccess) e = launch_dem_integrate(c, p);
    if (e == hipSuccess) e = launch_finalize(c, kFinBuild | kFinDisp, nullptr, nullptr);
    return e;
}

int fpm_dem_step(fpm_ctx *c, const fpm_dem_params *p, int32_t nsteps) {
    int r = dem_ready(c, p);
    if (r) return r;
    if (nsteps < 0) return fail(c, FPM_EINVAL, "bad step count");
    if (c->build_pending) HIPCHK(c, refresh_and_account(c));
    c->forces_valid = false;
    if (nsteps == 0) return FPM_OK;
    if (!(c->d_chunk && memcmp(&c->d_prm, p, sizeof(*p)) == 0)) {
        drop_graphs(c);
        const fpm_dem_params prm = *p;
        c->dem_exported = false;  // the captured steps always carry the export
        int e = capture(c,
                        [&] {
                            hipError_t x = hipSuccess;
                            for (int s = 0; s < kChunk && x == hipSuccess; s++)
                                x = dem_step_body(c, prm);
                            return x;
                        },
                        &c->d_chunk);
        if (e) return e;
        e = capture(c, [&] { return dem_step_body(c, prm); }, &c->d_one);
        if (e) return e;
        c->d_prm = *p;
    }
    int left = nsteps;
    for (; left >= kChunk; left -= kChunk) HIPCHK(c, hipGraphLaunch(c->d_chunk, c->stream));
    for (; left > 0; left--) HIPCHK(c, hipGraphLaunch(c->d_one, c->stream));
    return FPM_OK;
}

int fpm_get_dem(fpm_ctx *c, float *w, float *tq, int32_t *ncon) {
    int r = ready(c);
    if (r) return r;
    if (c->dem_cap <= 0) return fail(c, FPM_EINVAL, "DEM storage not set (fpm_set_dem)");
    HIPCHK(c, launch_dem_out(c, w, tq, nullptr, nullptr, ncon));
    return FPM_OK;
}

int fpm_get_contacts(fpm_ctx *c, int32_t *ids, float *ut) {
    int r = ready(c);
    if (r) return r;
    if (c->dem_cap <= 0) return fail(c, FPM_EINVAL, "DEM storage not set (fpm_set_dem)");
    HIPCHK(c, launch_dem_out(c, nullptr, nullptr, ids, ut, nullptr));
    return FPM_OK;
}

int fpm_check(fpm_ctx *c) {
    int r = ready(c);
    if (r) return r;
    Ctl h;
    HIPCHK(c, hipMemcpyAsync(&h, c->st.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h.overflow) return fail(c, FPM_EOVERFLOW, "Verlet list exceeded max_nbr");
    if (h.sym_miss) return fail(c, FPM_EOVERFLOW, "symmetric lists: a pair missing from one side");
    if (h.nonfinite) return fail(c, FPM_ENONFINITE, "non-finite position or force");
    if (h.bad_index) return fail(c, FPM_EBADINDEX, "a list or cell-list entry out of range");
    return FPM_OK;
}

int fpm_read_counters(fpm_ctx *c, int64_t out[3]) {
    int r = ready(c);
    if (r) return r;
    if (!out) return fail(c, FPM_EINVAL, "null output");
    HIPCHK(c, launch_list_stats(c));
    Ctl h;
    std::vector<SysCtl> sc(c->nsys);
    HIPCHK(c, hipMemcpyAsync(&h, c->st.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(sc.data(), c->st.sctl, sc.size() * sizeof(SysCtl),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out[0] = 0;
    for (const SysCtl &x : sc) out[0] += x.n_rebuilds;
    out[1] = h.max_count;
    out[2] = h.total_count;
    return FPM_OK;
}

int fpm_set_profiling(fpm_ctx *c, int32_t on) {
    if (!c) return FPM_EINVAL;
    if (!on) {
        (void)hipStreamSynchronize(c->stream);
        drop_timers(c);
    }
    c->profiling = on != 0;
    return FPM_OK;
}

int fpm_kernel_time(fpm_ctx *c, const char *kernel, double *ms, int64_t *count) {
    if (!c) return FPM_EINVAL;
    if (!kernel || !ms || !count) return fail(c, FPM_EINVAL, "null argument");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    int64_t k = 0;
    hipError_t err = hipSuccess;
    std::vector<fpm_ctx::Timed> keep;
    for (auto &t : c->timed) {
        if (t.name != kernel) {
            keep.push_back(t);
            continue;
        }
        float m = 0.f;
        hipError_t e = hipEventElapsedTime(&m, t.start, t.stop);
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
        if (e != hipSuccess) err = e;
        tot += m;
        k++;
    }
    c->timed.swap(keep);
    if (err != hipSuccess) return hip_fail(c, err, "hipEventElapsedTime");
    *ms = k ? tot / (double)k : 0.0;
    *count = k;
    return FPM_OK;
}

}  // extern "C"
