// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fpm.h"

namespace fpm {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kBlock = 256;        // threads per workgroup for particle kernels
constexpr int kMaxNbrCap = 4096;   // largest accepted Verlet-list capacity
constexpr int64_t kMaxParticles = (int64_t(1) << 26) - 1;
constexpr uint32_t kWrapBit = 0x80000000u;  // "list holds periodic images" flag in counts

// Per-block partial results (for each slot an array with one double per
// workgroup of the particle kernels), reduced in a fixed order by the
// finalize kernels.
enum Slot {
    kSlotU = 0,        // potential energy (LJ)
    kSlotW = 1,        // virial xx, yy, zz, xy, xz, yz (1..6)
    kSlotKE = 7,       // kinetic energy
    kSlotDisp = 8,     // largest squared displacement since the last build
    kSlotMaxCnt = 9,   // longest Verlet list of the build
    kSlotTotCnt = 10,  // total Verlet-list entries of the build
    kSlotOvf = 11,     // longest list if it exceeded the capacity, else 0
    kSlotMu = 12,      // SPH: largest |mu_ab|
    kSlotAcc = 13,     // SPH: smallest h / |a|
    kSlotVmax = 14,    // SPH: largest |v|
    kSlots = 16
};

// Finalize modes (bit mask).
enum {
    kFinBuild = 1,   // account a finished rebuild (stats, counter) and clear the flag
    kFinForce = 2,   // reduce U and W into ctl->thermo (and the optional output)
    kFinKE = 4,      // reduce the kinetic energy into ctl->thermo[1]
    kFinRow = 8,     // append ctl->thermo as row ctl->step of the thermo output
    kFinDisp = 16,   // reduce the displacement and raise the rebuild flag
    kFinSph = 32     // SPH: time step from the CFL terms, time and history row
};

// Device-resident control block.  One per context, inside the workspace.
struct Ctl {
    int32_t rebuild;        // 1: the neighbour structures must be rebuilt
    int32_t overflow;       // longest list of the last build if above capacity, else 0
    int32_t nonfinite;      // 1 once a non-finite value was seen
    int32_t step;           // rows written in the current fpm_step call
    int64_t n_rebuilds;     // rebuilds since fpm_set_particles
    int32_t max_count;      // longest list of the last build
    int32_t pad0;
    int64_t total_count;    // total list entries of the last build
    double thermo[8];       // last U, KE, W6
    float sph_dt;           // SPH time step of the next step (from the latest rates)
    float sph_dt_last;      // SPH time step of the last completed step
    double sph_time;        // simulated SPH time
};

// Device view of the box.
struct Box {
    float L[3];
    float half[3];
    int32_t per[3];
    int32_t nc[3];          // cells per axis
    float inv[3];           // nc / L in FP32
};

// Pointers into the workspace.  Buffer 0 holds the cell-sorted state between
// rebuilds; a rebuild gathers into buffer 1 and the Verlet build copies it back.
struct State {
    float4 *pos[2];         // x, y, z, type bits
    float4 *vel[2];         // vx, vy, vz, (SPH: rho)
    int32_t *id[2];         // slot -> caller index
    float4 *frc;            // fx, fy, fz, (LJ: atom energy / SPH: drho/dt)
    float4 *xbuild;         // positions at the last rebuild
    int32_t *cid;           // cell of each slot
    int32_t *rnk;           // arrival rank inside the cell
    int2 *tmp;              // (caller id, source slot) after the scatter
    int32_t *cnt;           // per-cell counts (kept at zero between rebuilds)
    int32_t *off;           // exclusive scan of counts, ncells + 1
    int32_t *nbr;           // Verlet list, see nbr_index()
    uint32_t *nnb;          // list length | kWrapBit
    double *part;           // per-block partials, part[slot * pstride + block]
    Ctl *ctl;
    int32_t pstride;        // >= the grid of every kernel that writes partials
    int32_t dummy;          // padding slot (index n): a particle far outside every box;
                            // lists are padded with it to a multiple of 8 entries
};

// Position of the padding slot: far enough that no pair with it is ever in
// range, small enough that squared FP32 distances stay finite.
constexpr float kFarAway = 1.0e18f;

// Verlet-list storage: per group of 64 slots, per group of 4 entries, 64 int4
// (one per slot), so a wavefront reads 4 entries per lane in one 1 KiB load.
// `cap4` is the capacity in groups of four.
__host__ __device__ __forceinline__ int64_t nbr_index(int64_t i, int k, int cap4) {
    return (((i >> 6) * (int64_t)cap4 + (k >> 2)) * 64 + (i & 63)) * 4 + (k & 3);
}

}  // namespace fpm

struct fpm_ctx {
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    std::string err;
    bool box_set = false, nbr_set = false, have_particles = false, forces_valid = false;
    bool build_pending = false;        // cell list rebuilt without the Verlet list
    bool sph = false;                  // the kept rates are SPH rates (not LJ forces)
    fpm::Box box{};
    float r_cut = 0.f, skin = 0.f;
    float R2 = 0.f;          // (r_cut + skin)^2 rounded to FP32
    float rc2 = 0.f;         // r_cut^2 rounded to FP32
    float disp2_thr = 0.f;   // (skin/2)^2 rounded to FP32
    int32_t cap = 0;         // list capacity asked for
    int32_t cap4 = 0;        // allocated capacity in groups of 4 (>= cap, multiple of 2)
    int64_t ncells = 0;
    int64_t n = 0, n_pad = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    fpm::State st{};
    int nblk = 0;            // workgroups of the particle kernels
    int nblk_build = 0;      // workgroups of the Verlet-list build
    int zb = 0;              // z-cells per workgroup of the column build (0: per-particle build)
    int nzb = 0;             // z-blocks per column
    // graphs of fpm_step, keyed by their parameters
    hipGraphExec_t g_first = nullptr, g_chunk = nullptr, g_one = nullptr;
    double *g_thermo = nullptr;
    float g_dt = 0.f;
    fpm_lj_params g_prm{};
    hipGraphExec_t s_first = nullptr, s_chunk = nullptr, s_one = nullptr;  // SPH graphs
    fpm_sph_params s_prm{};
    double *s_hist = nullptr;
    // event timing of eager launches (fpm_set_profiling)
    struct Timed {
        std::string name;
        hipEvent_t start, stop;
    };
    bool profiling = false;
    std::vector<Timed> timed;
};

namespace fpm {

// Launchers implemented in the .hip files.  All enqueue on ctx->stream.
hipError_t launch_fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v);
hipError_t launch_init_state(fpm_ctx *c, const float *pos, const float *vel, const int32_t *type);
hipError_t launch_set_density(fpm_ctx *c, const float *rho);
hipError_t launch_force_rebuild(fpm_ctx *c);
hipError_t launch_cell_build(fpm_ctx *c);
hipError_t launch_copy_back(fpm_ctx *c);
hipError_t launch_verlet_build(fpm_ctx *c);
hipError_t launch_list_stats(fpm_ctx *c);  // fills ctl->max_count and ctl->total_count
// z-cells per workgroup of the column Verlet build, 0 when the grid is too
// small for it (fewer than three cells along an axis).
int verlet_zblock(int64_t n, int64_t ncells, const int nc[3]);
hipError_t launch_lj_forces(fpm_ctx *c, const fpm_lj_params &p);
hipError_t launch_integrate(fpm_ctx *c, float dt, int mode);
hipError_t launch_finalize(fpm_ctx *c, int mode, double *out, double *rows);
hipError_t launch_gather_out(fpm_ctx *c, float *pos, float *vel, float *frc, float *rho,
                             float *drho);
hipError_t launch_cells_out(fpm_ctx *c, int32_t *offsets, int32_t *order);
hipError_t launch_neighbors_out(fpm_ctx *c, int32_t *counts, int32_t *cols);
hipError_t launch_reset_step(fpm_ctx *c);
hipError_t launch_sph_rates(fpm_ctx *c, const fpm_sph_params &p);
hipError_t launch_sph_integrate(fpm_ctx *c, const fpm_sph_params &p, int mode);
hipError_t launch_sph_finalize(fpm_ctx *c, const fpm_sph_params &p, int mode, float *dt_out,
                               double *hist);

// Integrate modes.
enum { kKickDriftFirst = 0, kKickKickDrift = 1, kKickOnly = 2 };

// Relative half-width of the band around r_cut^2 inside which the interaction
// kernels evaluate the FP32 predicate instead of trusting the exact FP64
// squared distance.  Outside it both agree: the FP32 squared distance differs
// from the exact one by at most 3 L |d| 2^-23 (the once-rounded ghost
// coordinate xj +- L) plus 5 ulp of d^2, which the band covers twice over.
inline double predicate_band(const fpm_ctx *c) {
    double lmax = 0.0;
    for (int a = 0; a < 3; a++)
        if (c->box.per[a] && (double)c->box.L[a] > lmax) lmax = (double)c->box.L[a];
    return 6.0 * lmax / (double)c->r_cut * 0x1p-23 + 1e-6;
}

}  // namespace fpm
