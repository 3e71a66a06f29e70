// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/fpm.h"

namespace fpm {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kBlock = 256;        // threads per workgroup for particle kernels
constexpr int kMaxNbrCap = 4096;   // largest accepted Verlet-list capacity
constexpr int64_t kMaxParticles = (int64_t(1) << 26) - 1;
constexpr uint32_t kWrapBit = 0x80000000u;  // "list holds periodic images" flag in counts

// Device-resident control block.  One per context, inside the workspace.
struct Ctl {
    int32_t cur;            // ping-pong buffer holding the sorted state (0/1)
    int32_t rebuild;        // 1: the neighbour structures must be rebuilt this step
    uint32_t maxdisp2;      // FP32 bits of the largest squared displacement since build
    int32_t overflow;       // largest list length seen if above capacity, else 0
    int32_t nonfinite;      // 1 once a non-finite value was seen
    int32_t step;           // step counter inside the current fpm_step call
    uint32_t done[4];       // last-block counters of the reduction kernels
    int64_t n_rebuilds;     // rebuilds since fpm_set_particles
    int32_t max_count;      // largest list length of the last build
    int32_t pad0;
    int64_t total_count;    // total list entries of the last build
    double thermo[8];       // last U, KE, W6
    float sph_dt;           // current SPH time step
    float sph_pad;
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

// Pointers into the workspace.
struct State {
    float4 *pos[2];         // x, y, z, type bits (sorted, ping-pong)
    float4 *vel[2];         // vx, vy, vz, (SPH: rho)
    int32_t *id[2];         // slot -> caller index
    float4 *frc;            // fx, fy, fz, (SPH: drho/dt)
    float4 *xbuild;         // positions at the last rebuild
    int32_t *cid;           // cell of each slot (current order)
    int32_t *rnk;           // arrival rank inside the cell
    int2 *tmp;              // (caller id, source slot) after the scatter
    int32_t *cnt;           // per-cell counts (kept at zero between rebuilds)
    int32_t *off;           // exclusive scan of counts, ncells + 1
    int32_t *nbr;           // Verlet list, blocked ELL: [(i/64)*cap + k]*64 + i%64
    uint32_t *nnb;          // list length | kWrapBit
    double *part;           // per-block FP64 partial sums
    Ctl *ctl;
};

}  // namespace fpm

struct fpm_ctx {
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    std::string err;
    bool box_set = false, nbr_set = false, have_particles = false, forces_valid = false;
    bool sph = false;
    fpm::Box box{};
    float r_cut = 0.f, skin = 0.f;
    float R2 = 0.f;          // (r_cut + skin)^2 rounded to FP32
    float rc2 = 0.f;         // r_cut^2 rounded to FP32
    float disp2_thr = 0.f;   // (skin/2)^2 rounded to FP32
    int32_t cap = 0;
    int64_t ncells = 0;
    int64_t n = 0, n_pad = 0, n_alloc = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    fpm::State st{};
    int nblk = 0;            // blocks of the particle kernels
    // graphs of fpm_step, keyed by their parameters
    hipGraphExec_t g_first = nullptr, g_chunk = nullptr, g_one = nullptr;
    int g_chunk_len = 0;
    double *g_thermo = nullptr;
    float g_dt = 0.f;
    fpm_lj_params g_prm{};
    hipGraphExec_t s_one = nullptr;  // SPH step graph
    fpm_sph_params s_prm{};
    double *s_hist = nullptr;
};

namespace fpm {

// Launchers implemented in the .hip files.  All enqueue on ctx->stream.
hipError_t launch_fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v);
hipError_t launch_init_state(fpm_ctx *c, const float *pos, const float *vel, const int32_t *type);
hipError_t launch_set_density(fpm_ctx *c, const float *rho);
hipError_t launch_force_rebuild(fpm_ctx *c);
hipError_t launch_cell_build(fpm_ctx *c);
hipError_t launch_verlet_build(fpm_ctx *c);
hipError_t launch_lj_forces(fpm_ctx *c, const fpm_lj_params &p, double *out, double *thermo,
                            int32_t thermo_rows, int count_step);
hipError_t launch_integrate(fpm_ctx *c, float dt, int mode, double *thermo, int32_t thermo_rows);
hipError_t launch_gather_out(fpm_ctx *c, float *pos, float *vel, float *frc, float *rho,
                             float *drho);
hipError_t launch_cells_out(fpm_ctx *c, int32_t *offsets, int32_t *order);
hipError_t launch_neighbors_out(fpm_ctx *c, int32_t *counts, int32_t *cols);
hipError_t launch_reset_step(fpm_ctx *c);
hipError_t launch_sph_rates(fpm_ctx *c, const fpm_sph_params &p);
hipError_t launch_sph_kick_drift(fpm_ctx *c, const fpm_sph_params &p, int first);
hipError_t launch_sph_kick(fpm_ctx *c, const fpm_sph_params &p, double *hist, int32_t rows);

// Integrate modes.
enum { kKickDriftFirst = 0, kKickKickDrift = 1, kKickOnly = 2 };

}  // namespace fpm
