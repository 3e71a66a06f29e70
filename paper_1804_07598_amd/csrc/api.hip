// Host side of the C ABI declared in include/fpm.h: argument checks, the
// workspace layout, the order of kernel launches and the graphs of fpm_step.
#include <math.h>
#include <string.h>

#include <climits>
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

#define HIPCHK(c, expr)                                   \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout for n particles; with base == nullptr only the size is computed.
size_t layout(fpm_ctx *c, int64_t n, char *base, State *st) {
    const int64_t n_pad = (n + kBlock - 1) / kBlock * kBlock;
    const int64_t nblk = n_pad / kBlock;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    State s{};
    for (int k = 0; k < 2; k++) s.pos[k] = (float4 *)take(n_pad * sizeof(float4));
    for (int k = 0; k < 2; k++) s.vel[k] = (float4 *)take(n_pad * sizeof(float4));
    for (int k = 0; k < 2; k++) s.id[k] = (int32_t *)take(n_pad * sizeof(int32_t));
    s.frc = (float4 *)take(n_pad * sizeof(float4));
    s.xbuild = (float4 *)take(n_pad * sizeof(float4));
    s.cid = (int32_t *)take(n_pad * sizeof(int32_t));
    s.rnk = (int32_t *)take(n_pad * sizeof(int32_t));
    s.tmp = (int2 *)take(n_pad * sizeof(int2));
    s.cnt = (int32_t *)take(c->ncells * sizeof(int32_t));
    s.off = (int32_t *)take((c->ncells + 1) * sizeof(int32_t));
    s.nbr = (int32_t *)take((size_t)n_pad * c->cap * sizeof(int32_t));
    s.nnb = (uint32_t *)take(n_pad * sizeof(uint32_t));
    s.part = (double *)take((size_t)(nblk + 1) * 8 * sizeof(double));
    s.ctl = (Ctl *)take(sizeof(Ctl));
    if (st) *st = s;
    return off;
}

bool finite3(const float *v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

void drop_graphs(fpm_ctx *c) {
    for (hipGraphExec_t *g : {&c->g_first, &c->g_chunk, &c->g_one, &c->s_one}) {
        if (*g) (void)hipGraphExecDestroy(*g);
        *g = nullptr;
    }
}

int ready(fpm_ctx *c) {
    if (!c) return FPM_EINVAL;
    if (!c->have_particles) return fail(c, FPM_EINVAL, "no particles set");
    return FPM_OK;
}

// Gated neighbour-structure refresh: both kernels return at once unless the
// device rebuild flag is set.
hipError_t refresh_lists(fpm_ctx *c) {
    hipError_t e = launch_cell_build(c);
    if (e != hipSuccess) return e;
    return launch_verlet_build(c);
}

constexpr int kChunk = 25;  // steps per captured graph

// Captures `steps` velocity-Verlet steps into an executable graph.
int capture_steps(fpm_ctx *c, const fpm_lj_params &p, float dt, double *thermo, int steps,
                  bool first, hipGraphExec_t *out) {
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
    for (int s = 0; s < steps && e == hipSuccess; s++) {
        e = launch_integrate(c, dt, (first && s == 0) ? kKickDriftFirst : kKickKickDrift, thermo,
                             INT_MAX);
        if (e == hipSuccess) e = refresh_lists(c);
        if (e == hipSuccess) e = launch_lj_forces(c, p, nullptr, thermo, INT_MAX, 1);
    }
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
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return FPM_OK;
}

const char *fpm_last_error(const fpm_ctx *c) { return c ? c->err.c_str() : "null context"; }

int fpm_set_box(fpm_ctx *c, const float L[3], const int32_t per[3]) {
    if (!c) return FPM_EINVAL;
    if (!L || !per) return fail(c, FPM_EINVAL, "null box argument");
    for (int a = 0; a < 3; a++) {
        if (!(isfinite(L[a]) && L[a] > 0.f)) return fail(c, FPM_EINVAL, "box side must be > 0");
        if (per[a] != 0 && per[a] != 1) return fail(c, FPM_EINVAL, "periodic flag must be 0/1");
        c->box.L[a] = L[a];
        c->box.half[a] = L[a] * 0.5f;
        c->box.per[a] = per[a];
    }
    c->box_set = true;
    c->nbr_set = false;
    c->have_particles = false;
    drop_graphs(c);
    return FPM_OK;
}

int fpm_set_neighbor_params(fpm_ctx *c, float r_cut, float skin, int32_t max_nbr) {
    if (!c) return FPM_EINVAL;
    if (!c->box_set) return fail(c, FPM_EINVAL, "set the box first");
    if (!(isfinite(r_cut) && r_cut > 0.f && isfinite(skin) && skin >= 0.f))
        return fail(c, FPM_EINVAL, "r_cut must be > 0 and skin >= 0");
    if (max_nbr < 1 || max_nbr > kMaxNbrCap) return fail(c, FPM_EINVAL, "max_nbr out of range");
    const double R = (double)r_cut + (double)skin;
    int64_t ncells = 1;
    for (int a = 0; a < 3; a++) {
        if (c->box.per[a] && !(R < 0.5 * (double)c->box.L[a] * (1.0 - 1e-6)))
            return fail(c, FPM_ECUTOFF, "r_cut + skin must be below half the periodic box");
        double m = floor((double)c->box.L[a] / (R * 1.000001));
        int nc = m < 1.0 ? 1 : (m > 1 << 20 ? 1 << 20 : (int)m);
        c->box.nc[a] = nc;
        c->box.inv[a] = (float)nc / c->box.L[a];
        ncells *= nc;
    }
    if (ncells > (int64_t)1 << 30) return fail(c, FPM_EINVAL, "too many cells");
    c->ncells = ncells;
    c->r_cut = r_cut;
    c->skin = skin;
    c->cap = max_nbr;
    c->R2 = (float)(R * R);
    c->rc2 = (float)((double)r_cut * (double)r_cut);
    const double hs = 0.5 * (double)skin;
    c->disp2_thr = (float)(hs * hs);
    c->nbr_set = true;
    c->have_particles = false;
    drop_graphs(c);
    return FPM_OK;
}

int fpm_workspace_size(fpm_ctx *c, int64_t n, size_t *bytes) {
    if (!c) return FPM_EINVAL;
    if (!bytes) return fail(c, FPM_EINVAL, "null size pointer");
    if (!c->nbr_set) return fail(c, FPM_EINVAL, "set box and neighbour parameters first");
    if (n < 1 || n > kMaxParticles) return fail(c, FPM_EINVAL, "particle count out of range");
    *bytes = layout(c, n, nullptr, nullptr);
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

int fpm_set_particles(fpm_ctx *c, int64_t n, const float *pos, const float *vel,
                      const int32_t *type) {
    if (!c) return FPM_EINVAL;
    if (!c->nbr_set) return fail(c, FPM_EINVAL, "set box and neighbour parameters first");
    if (n < 1 || n > kMaxParticles) return fail(c, FPM_EINVAL, "particle count out of range");
    if (!pos) return fail(c, FPM_EINVAL, "null positions");
    const size_t need = layout(c, n, nullptr, nullptr);
    if (!c->ws || c->ws_bytes < need) return fail(c, FPM_ENOWS, "workspace missing or too small");
    layout(c, n, (char *)c->ws, &c->st);
    c->n = n;
    c->n_pad = (n + kBlock - 1) / kBlock * kBlock;
    c->nblk = (int)(c->n_pad / kBlock);
    drop_graphs(c);
    HIPCHK(c, launch_fill_i32(c->stream, c->st.cnt, c->ncells, 0));
    HIPCHK(c, launch_init_state(c, pos, vel, type));
    HIPCHK(c, launch_force_rebuild(c));
    HIPCHK(c, refresh_lists(c));
    c->have_particles = true;
    c->forces_valid = false;
    return FPM_OK;
}

int fpm_get_particles(fpm_ctx *c, float *pos, float *vel, float *frc) {
    int r = ready(c);
    if (r) return r;
    HIPCHK(c, launch_gather_out(c, pos, vel, frc, nullptr, nullptr));
    return FPM_OK;
}

int fpm_build_cell_list(fpm_ctx *c) {
    int r = ready(c);
    if (r) return r;
    HIPCHK(c, launch_force_rebuild(c));
    HIPCHK(c, launch_cell_build(c));
    return FPM_OK;
}

int fpm_get_cell_list(fpm_ctx *c, int32_t ncell[3], int32_t *offsets, int32_t *order) {
    int r = ready(c);
    if (r) return r;
    if (ncell)
        for (int a = 0; a < 3; a++) ncell[a] = c->box.nc[a];
    HIPCHK(c, launch_cells_out(c, offsets, order));
    return FPM_OK;
}

int fpm_build_verlet(fpm_ctx *c) {
    int r = ready(c);
    if (r) return r;
    HIPCHK(c, launch_force_rebuild(c));
    HIPCHK(c, refresh_lists(c));
    return FPM_OK;
}

int fpm_get_neighbors(fpm_ctx *c, int32_t *counts, int32_t *cols) {
    int r = ready(c);
    if (r) return r;
    if (!counts || !cols) return fail(c, FPM_EINVAL, "null output");
    HIPCHK(c, refresh_lists(c));
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
    if (!p || (p->n_types != 1 && p->n_types != 2)) return fail(c, FPM_EINVAL, "bad LJ params");
    HIPCHK(c, refresh_lists(c));
    HIPCHK(c, launch_lj_forces(c, *p, out, nullptr, 0, 0));
    c->forces_valid = true;
    return FPM_OK;
}

int fpm_integrate(fpm_ctx *c, float dt, int32_t half) {
    int r = ready(c);
    if (r) return r;
    if (!isfinite(dt)) return fail(c, FPM_EINVAL, "dt must be finite");
    if (half != 0 && half != 1) return fail(c, FPM_EINVAL, "half must be 0 or 1");
    HIPCHK(c, launch_integrate(c, dt, half ? kKickOnly : kKickDriftFirst, nullptr, 0));
    return FPM_OK;
}

int fpm_step(fpm_ctx *c, const fpm_lj_params *p, float dt, int32_t nsteps, double *thermo) {
    int r = ready(c);
    if (r) return r;
    if (!p || (p->n_types != 1 && p->n_types != 2)) return fail(c, FPM_EINVAL, "bad LJ params");
    if (!isfinite(dt) || nsteps < 0) return fail(c, FPM_EINVAL, "bad dt or step count");
    if (nsteps == 0) return FPM_OK;
    if (!c->forces_valid) {
        HIPCHK(c, refresh_lists(c));
        HIPCHK(c, launch_lj_forces(c, *p, nullptr, nullptr, 0, 0));
        c->forces_valid = true;
    }
    const bool same = c->g_first && c->g_dt == dt && c->g_thermo == thermo &&
                      memcmp(&c->g_prm, p, sizeof(*p)) == 0;
    if (!same) {
        drop_graphs(c);
        int e;
        if ((e = capture_steps(c, *p, dt, thermo, 1, true, &c->g_first))) return e;
        if ((e = capture_steps(c, *p, dt, thermo, kChunk, false, &c->g_chunk))) return e;
        if ((e = capture_steps(c, *p, dt, thermo, 1, false, &c->g_one))) return e;
        c->g_dt = dt;
        c->g_thermo = thermo;
        c->g_prm = *p;
    }
    HIPCHK(c, launch_reset_step(c));
    HIPCHK(c, hipGraphLaunch(c->g_first, c->stream));
    int left = nsteps - 1;
    for (; left >= kChunk; left -= kChunk) HIPCHK(c, hipGraphLaunch(c->g_chunk, c->stream));
    for (; left > 0; left--) HIPCHK(c, hipGraphLaunch(c->g_one, c->stream));
    HIPCHK(c, launch_integrate(c, dt, kKickOnly, thermo, INT_MAX));
    return FPM_OK;
}

int fpm_check(fpm_ctx *c) {
    int r = ready(c);
    if (r) return r;
    Ctl h;
    HIPCHK(c, hipMemcpyAsync(&h, c->st.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h.overflow) return fail(c, FPM_EOVERFLOW, "Verlet list exceeded max_nbr");
    if (h.nonfinite) return fail(c, FPM_ENONFINITE, "non-finite position or force");
    return FPM_OK;
}

int fpm_read_counters(fpm_ctx *c, int64_t out[3]) {
    int r = ready(c);
    if (r) return r;
    if (!out) return fail(c, FPM_EINVAL, "null output");
    Ctl h;
    HIPCHK(c, hipMemcpyAsync(&h, c->st.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out[0] = h.n_rebuilds;
    out[1] = h.max_count;
    out[2] = h.total_count;
    return FPM_OK;
}

}  // extern "C"
