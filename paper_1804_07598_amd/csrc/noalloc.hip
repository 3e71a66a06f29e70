// Allocation-free Lennard-Jones forces: the computation of fpm_lj_forces for a
// particle set given in one call, with every array it needs (cell-sorted
// state, cell list, Verlet lists, per-workgroup partial sums) laid out in a
// static device array instead of a caller workspace.  Nothing here or in the
// calls it makes allocates device memory.
//
// The array is one per GPU (each device that loads the library holds its own
// copy until the process ends).  Its address is taken once per device with
// hipGetSymbolAddress while that device is current; host code passes only
// that address on, never the array's name, which in host code is a host-side
// stand-in.  Every call on a GPU reuses the same array, so the computation
// clears what it reads before writing it (cell counts, control words) and
// calls that overlap on one GPU race.
#include <mutex>

#include "fpm_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[FPM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices];  // address of `scratch` on each device, once taken
std::mutex g_mu;

int fail(fpm_ctx *c, int code, const std::string &msg) {
    c->err = msg;
    return code;
}

// Address of the current device's copy of the array.
int device_scratch(fpm_ctx *c, void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(c, FPM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(c, FPM_EHIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(c, FPM_EHIP,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return FPM_OK;
}

// A context that takes over the box, neighbour parameters, launch shapes and
// stream of `c` and nothing else.
void copy_config(const fpm_ctx *c, fpm_ctx *t) {
    t->stream = c->stream;
    t->boxes = c->boxes;
    t->box_set = true;
    t->r_cut = c->r_cut;
    t->skin = c->skin;
    t->R2 = c->R2;
    t->rc2 = c->rc2;
    t->disp2_thr = c->disp2_thr;
    t->cap = c->cap;
    t->cap4 = c->cap4;
    t->nbr_set = true;
    t->tune_verlet_path = c->tune_verlet_path;
    t->tune_zb = c->tune_zb;
    t->tune_unroll = c->tune_unroll;
}

}  // namespace

extern "C" int fpm_lj_forces_static(fpm_ctx *c, const fpm_lj_params *prm, int64_t n,
                                    const float *pos, const int32_t *type, float *frc,
                                    double *out) {
    if (!c) return FPM_EINVAL;
    if (!c->box_set || !c->nbr_set)
        return fail(c, FPM_EINVAL, "set the box and the neighbour parameters first");
    if (c->boxes.size() != 1 || !c->counts.empty())
        return fail(c, FPM_EINVAL, "fpm_lj_forces_static takes a single system");
    if (c->dem_cap > 0) return fail(c, FPM_EINVAL, "fpm_lj_forces_static takes no DEM storage");
    if (!pos || !frc) return fail(c, FPM_EINVAL, "null positions or force output");
    if (n < 1) return fail(c, FPM_EINVAL, "particle count out of range");
    fpm_ctx t;
    copy_config(c, &t);
    size_t need = 0;
    int r = fpm_workspace_size(&t, n, &need);
    if (r) return fail(c, r, t.err);
    if (need > (size_t)FPM_STATIC_SCRATCH_BYTES)
        return fail(c, FPM_ENOWS,
                    "fpm_lj_forces_static: " + std::to_string(n) + " particles need " +
                        std::to_string(need) + " bytes of scratch, more than the static " +
                        std::to_string((size_t)FPM_STATIC_SCRATCH_BYTES) + " bytes");
    void *ws = nullptr;
    r = device_scratch(c, &ws);
    if (r) return r;
    r = fpm_set_workspace(&t, ws, (size_t)FPM_STATIC_SCRATCH_BYTES);
    if (!r) r = fpm_set_particles(&t, n, pos, nullptr, type);
    if (!r) r = fpm_lj_forces(&t, prm, out);
    if (!r) r = fpm_get_particles(&t, nullptr, nullptr, frc);
    if (r) return fail(c, r, t.err);
    return FPM_OK;
}
