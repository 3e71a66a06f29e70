// Internal declarations shared by the HIP translation units of the library.
//
// A context holds one or more independent systems ("batch").  Every system
// owns a contiguous range of particle slots padded to whole workgroups, its
// own cell grid and its own control words, so every workgroup of a particle
// kernel belongs to exactly one system and reads that system's description
// with scalar loads.  A single simulation is a batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fpm.h"

#ifndef FPM_CHECKED
#define FPM_CHECKED 0
#endif

namespace fpm {

// Debug builds (compiled with FPM_CHECKED=1 as libfpm_checked.so): the cell
// list and the Verlet lists are validated after every rebuild, and every list
// entry the LJ force and VJP kernels read is range-checked; a violation sets
// Ctl::bad_index, which fpm_check reports.
constexpr bool kChecked = FPM_CHECKED != 0;

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kBlock = 256;        // threads per workgroup of the particle kernels
constexpr int kMaxNbrCap = 4096;   // largest accepted Verlet-list capacity
constexpr int64_t kMaxParticles = (int64_t(1) << 26) - 1;
constexpr int kMaxSystems = 1 << 16;
constexpr uint32_t kWrapBit = 0x80000000u;  // "list holds periodic images" flag in counts
constexpr int kPosSlack = 8;       // readable slots after each position buffer

// Per-block partial results: for each slot one double per particle workgroup
// (part[slot * pstride + block]), reduced per system in a fixed order by the
// finalize kernels.
enum Slot {
    kSlotU = 0,        // potential energy (LJ)
    kSlotW = 1,        // virial xx, yy, zz, xy, xz, yz (1..6)
    kSlotKE = 7,       // kinetic energy
    kSlotDisp = 8,     // largest squared displacement since the last build
    kSlotMu = 9,       // SPH: largest |mu_ab|
    kSlotAcc = 10,     // SPH: smallest h / |a|
    kSlotVmax = 11,    // SPH: largest |v|
    kSlots = 12
};

// Finalize modes (bit mask).
enum {
    kFinBuild = 1,   // account a finished rebuild and clear the system's flag
    kFinForce = 2,   // reduce U and W into the system's thermo (and the optional output)
    kFinKE = 4,      // reduce the kinetic energy into thermo[1]
    kFinRow = 8,     // append the system's thermo as row `step` of the thermo output
    kFinDisp = 16,   // reduce the displacement and raise the rebuild flag
    kFinVjp = 32     // add the parameter gradient (slots 0..5) to the output
};

// Device view of one periodic (or partly closed) box and its cell grid.
struct Box {
    float L[3];
    float half[3];
    int32_t per[3];
    int32_t nc[3];          // cells per axis
    float inv[3];           // nc / L in FP32
};

// One system of the batch (device table, read with scalar loads).
struct SysDesc {
    Box box;
    int32_t n;              // particles
    int32_t slot_base;      // first slot (a multiple of kBlock)
    int32_t n_pad;          // slots (a multiple of kBlock, >= n + 1)
    int32_t blk_base;       // first particle workgroup
    int32_t cell_base;      // first cell of the global cell numbering
    int32_t ncells;
    int32_t off_base;       // first entry of the offsets array (ncells + 1 entries)
    int32_t zb, nzb;        // column Verlet build: z-cells per workgroup, z-blocks (0: none)
    int32_t item_base;      // first work item of the column build
    int32_t dummy;          // padding slot slot_base + n: far outside every box
    int32_t caller_base;    // first caller index of this system
};

// Per-system control words.
// The rebuild flag comes in two copies so that a captured LJ step can consume
// one (its force kernel accounts the rebuild and clears it) while its drift
// raises the other for the next step: step t of a step loop reads copy t & 1
// (State::par); every call outside a step loop uses copy 0.
struct SysCtl {
    int32_t rebuild[2];     // 1: this system's neighbour structures must be rebuilt
    int32_t step;           // rows written in the current fpm_step call
    int32_t pad;
    int64_t n_rebuilds;     // rebuilds since fpm_set_particles
    double thermo[8];       // last U, KE, W6
};

// Context-wide control block.
struct Ctl {
    int32_t overflow;       // a list length above the capacity (sticky), else 0
    int32_t nonfinite;      // 1 once a non-finite value was seen (sticky)
    int32_t max_count;      // longest list (filled on request)
    int32_t sym_miss;       // symmetric lists: a partner's list lacked the pair (sticky)
    int64_t total_count;    // total list entries (filled on request)
    float sph_dt;           // SPH time step of the next step (from the latest rates)
    float sph_dt_last;      // SPH time step of the last completed step
    double sph_time;        // simulated SPH time
    int32_t sph_nstep;      // SPH steps since the state was set (Verlet/Euler choice)
    int32_t bad_index;      // debug builds: a list or cell-list entry out of range (sticky)
};

// Pointers into the workspace.  Buffer 0 holds the cell-sorted state between
// rebuilds; a rebuild gathers into buffer 1 and the Verlet build copies it back.
struct State {
    float4 *pos[2];         // x, y, z, type bits
    float4 *vel[2];         // vx, vy, vz, (SPH: rho)
    int32_t *id[2];         // slot -> caller index (global over the batch)
    float4 *frc;            // fx, fy, fz, (LJ: atom energy / SPH: drho/dt)
    float4 *xbuild;         // positions at the last rebuild
    int32_t *cid;           // global cell of each slot
    int32_t *rnk;           // arrival rank inside the cell
    int4 *tmp;              // (caller id, source slot, z bits, cell) after the scatter
    int32_t *cnt;           // per-cell counts (kept at zero between rebuilds)
    int32_t *off;           // per system: exclusive scan of counts (global slots), ncells + 1
    int32_t *sub;           // per cell, 8 entries: first slot whose z lies in eighth q of the
                            // cell or above (see z_eighth); entry 0 is the cell's offset
    int32_t *tsum;          // device-wide scan: totals of the 4096-cell tiles
    int32_t *nbr;           // Verlet lists, see nbr_index()
    uint32_t *nnb;          // list length | kWrapBit
    double *part;           // per-block partials, part[slot * pstride + block]
    float4 *aux;            // per-slot scratch (adjoint input, sorted)
    float4 *old[2];         // SPH Verlet: previous step's (v, rho); DEM: angular velocity;
                            // double buffered like pos
    int32_t keep_old;       // 1: the cell sort carries old[] along
    float4 *hl;             // DEM: (u_t, in contact) per Verlet-list entry, entry-major per 64 slots
    int32_t *hid;           // DEM: partners in contact by caller index, C per grain (at rebuilds)
    float4 *hu;             // DEM: their u_t
    int32_t *ncon;          // DEM: contacts per grain (caller index)
    Ctl *ctl;
    SysCtl *sctl;           // per system
    const SysDesc *sys;     // per system
    const int32_t *blk2sys; // particle workgroup -> system
    const int32_t *item2sys;  // column-build work item -> system
    double *ring;           // step loops: per-step partials U, W6, KE, ring[(row * 8 + k) * pstride + block]
    double *sbuf;           // symmetric lists: pair force factor per list entry
    uint16_t *tsym;         // symmetric lists: per lower entry, the pair's position in the partner's list
    int32_t *plo;           // symmetric lists: entries below the slot itself (lists ascend)
    double *fown;           // symmetric lists: each slot's own pair sum (3 per slot)
    int32_t nsys;
    int32_t pstride;        // number of particle workgroups
    int32_t par;            // rebuild flag copy this launch reads (see SysCtl)
};

// Rows of per-step partial sums kept by a step loop before they are reduced.
constexpr int kRingRows = 16;

// Position of the padding slots: far enough that no pair with them is ever in
// range, small enough that squared FP32 distances stay finite.
constexpr float kFarAway = 1.0e18f;

// Verlet-list storage: per group of 64 slots, per group of 4 entries, 64 int4
// (one per slot), so a wavefront reads 4 entries per lane in one 1 KiB load.
// `cap4` is the capacity in groups of four.
__host__ __device__ __forceinline__ int64_t nbr_index(int64_t i, int k, int cap4) {
    return (((i >> 6) * (int64_t)cap4 + (k >> 2)) * 64 + (i & 63)) * 4 + (k & 3);
}

// Host copy of one system's layout.
struct SysHost {
    SysDesc d;
    int nblk;               // particle workgroups
    int nitems;             // column-build work items
};

}  // namespace fpm

struct fpm_ctx {
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    std::string err;
    bool box_set = false, nbr_set = false, have_particles = false, forces_valid = false;
    bool build_pending = false;        // cell list rebuilt without the Verlet list
    bool sph = false;                  // the kept rates are SPH rates (not LJ forces)
    // systems: boxes and particle counts (a single box is a batch of one)
    std::vector<fpm::Box> boxes;
    std::vector<int64_t> counts;       // particles per system (batch set-up), empty otherwise
    float r_cut = 0.f, skin = 0.f;
    float R2 = 0.f;          // (r_cut + skin)^2 rounded to FP32
    float rc2 = 0.f;         // r_cut^2 rounded to FP32
    float disp2_thr = 0.f;   // (skin/2)^2 rounded to FP32
    int32_t cap = 0;         // list capacity asked for
    int32_t cap4 = 0;        // allocated capacity in groups of 4 (>= cap, multiple of 2)
    int64_t n = 0;           // particles of the whole batch
    int64_t n_slots = 0;     // slots of the whole batch
    void *ws = nullptr;
    size_t ws_bytes = 0;
    fpm::State st{};
    std::vector<fpm::SysHost> sys;
    std::vector<char> plan_key;  // tables and layout of the last fpm_set_particles
    int nsys = 0;
    int nblk = 0;            // particle workgroups of the batch
    int ncells_total = 0;
    int noff_total = 0;
    int nitems = 0;          // column-build work items
    int n_pa_blocks = 0;     // workgroups of systems built particle by particle
    int n_grp_blocks = 0;    // workgroups of systems built by lane groups
    int n_ls_blocks = 0;     // workgroups of systems built by the lockstep window build
    int32_t *pa_blocks = nullptr;  // device list of those workgroups, then of these
    int max_ncells = 0;
    int max_sys_blocks = 0;  // particle workgroups of the largest system
    // tuning (fpm_set_tuning); 0 = automatic
    int tune_verlet_path = 0;   // 1: whole cells, 2: column blocks, 3: windows, 4: lane groups,
                                // 5: lockstep windows
    int tune_zb = 0;            // z-cells per column workgroup (path 4: lanes per particle)
    int tune_unroll = 0;        // force kernel: entries in flight per lane (4 or 8)
    // graphs of fpm_step, keyed by their parameters
    // LJ step loops: 16, 8, 4 and 2 steps from an even step; one step from an
    // even step; the last step from an even or an odd step
    hipGraphExec_t g_pow[4] = {nullptr, nullptr, nullptr, nullptr};
    hipGraphExec_t g_one = nullptr;
    hipGraphExec_t g_last[2] = {nullptr, nullptr};
    double *g_thermo = nullptr;
    float g_dt = 0.f;
    fpm_lj_params g_prm{};
    int g_unroll = 0;
    hipGraphExec_t s_first = nullptr, s_chunk = nullptr, s_one = nullptr;  // SPH graphs
    fpm_sph_params s_prm{};
    double *s_hist = nullptr;
    bool sph_restart = true;           // the SPH step count restarts at the next step call
    int dem_cap = 0;                   // DEM contact slots per grain (0: DEM off)
    bool sym = false;                  // LJ forces from symmetric half lists (fpm_set_symmetric)
    bool dem_exported = false;         // DEM: the caller-keyed rows already hold the history
    hipGraphExec_t d_chunk = nullptr, d_one = nullptr;  // DEM step graphs
    fpm_dem_params d_prm{};
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
hipError_t launch_cell_build(fpm_ctx *c, bool dem_export);  // dem_export: history out first
hipError_t launch_copy_back(fpm_ctx *c);
hipError_t launch_verlet_build(fpm_ctx *c);
hipError_t launch_list_stats(fpm_ctx *c);  // fills ctl->max_count and ctl->total_count
hipError_t launch_check_cells(fpm_ctx *c);  // debug builds (gated): cell-list validation
hipError_t launch_check_lists(fpm_ctx *c);  // debug builds (gated): Verlet-list validation
// z-cells per workgroup of the column Verlet build for one system, 0 when the
// grid is too small for it (fewer than three cells along an axis).
int verlet_zblock(int64_t n, int64_t ncells, const int nc[3], int tune_zb);
hipError_t launch_lj_forces(fpm_ctx *c, const fpm_lj_params &p);
// Force kernel modes: forces only; forces fused with the closing half kick of
// the step and the next step's opening half kick and drift; the same for the
// last step of a loop (closing kick only).
enum { kLjForce = 0, kLjStep = 1, kLjLast = 2 };
struct StepArgs {
    float dt;       // time step
    float thr;      // (skin/2)^2 in FP32: a larger displacement since the build rebuilds
    double *ring;   // this step's row of per-step partials (U, W6, KE)
};
// One step of a step loop (see kLjStep / kLjLast); its partials go to ring row `row`.
hipError_t launch_lj_step(fpm_ctx *c, const fpm_lj_params &p, float dt, bool last, int row);
// Reduces ring rows 0 .. nrows-1 of every system into thermo rows (rows may be
// null) ending at the system's step counter.
hipError_t launch_finalize_rows(fpm_ctx *c, int nrows, double *rows);
// Symmetric half lists: transpose positions at a rebuild (gated).
hipError_t launch_sym_index(fpm_ctx *c);
// Output of the force VJP kernel.  kVjpPlain: gx = g.  kVjpLast: gx += g.
// kVjpStep: one reverse velocity-Verlet step on caller-order FP64 arrays:
// gx (= xbar) += g; vbar += dt xbar; fbar = dt/2 vbar + floss (floss may be null).
enum { kVjpPlain = 0, kVjpStep = 1, kVjpLast = 2 };
struct AdjOut {
    double *gx, *vbar, *fbar;
    const double *floss;
    double dt;
    int mode;
};
hipError_t launch_lj_vjp(fpm_ctx *c, const fpm_lj_params &p, const double *lam,
                         const double *vbar, const AdjOut &o);
hipError_t launch_set_positions(fpm_ctx *c, const float *pos);
hipError_t launch_integrate(fpm_ctx *c, float dt, int mode);
hipError_t launch_finalize(fpm_ctx *c, int mode, double *out, double *rows);
hipError_t launch_gather_out(fpm_ctx *c, float *pos, float *vel, float *frc, float *rho,
                             float *drho);
hipError_t launch_cells_out(fpm_ctx *c, int32_t *offsets, int32_t *order);
hipError_t launch_neighbors_out(fpm_ctx *c, int32_t *counts, int32_t *cols);
hipError_t launch_reset_step(fpm_ctx *c);
hipError_t launch_sph_rates(fpm_ctx *c, const fpm_sph_params &p);
hipError_t launch_sph_integrate(fpm_ctx *c, const fpm_sph_params &p, int mode);
hipError_t launch_sph_verlet(fpm_ctx *c, const fpm_sph_params &p);
hipError_t launch_sph_restart(fpm_ctx *c);  // the next SPH step counts as the first
hipError_t launch_dem_forces(fpm_ctx *c, const fpm_dem_params &p, bool imp = false);  // imp: import after a rebuild
hipError_t launch_dem_integrate(fpm_ctx *c, const fpm_dem_params &p);
hipError_t launch_dem_set_omega(fpm_ctx *c, const float *w);  // also clears the history
hipError_t launch_dem_clear(fpm_ctx *c);                      // empty history
hipError_t launch_dem_export_assign(fpm_ctx *c);  // gated: list history -> caller-keyed rows, then cell assign
hipError_t launch_dem_import(fpm_ctx *c);  // gated: caller-keyed rows -> new list positions
hipError_t launch_dem_out(fpm_ctx *c, float *w, float *tq, int32_t *ids, float *ut,
                          int32_t *ncon);
hipError_t launch_sph_finalize(fpm_ctx *c, const fpm_sph_params &p, int mode, float *dt_out,
                               double *hist);

// Integrate modes.
enum { kKickDriftFirst = 0, kKickKickDrift = 1, kKickOnly = 2 };

// Relative half-width of the band around r_cut^2 inside which the interaction
// kernels evaluate the FP32 predicate instead of trusting the exact FP64
// squared distance.  Outside it both agree: every FP32 separation component is
// the exact one rounded once (pairs within the list radius satisfy the
// exactness condition of the image shift even between rebuilds, as
// r_cut + skin < L/2), so with u = 2^-24 the FP32 squared distance is within
// 5u (3e-7) relative of the exact one; the band is 2e-6.
inline double predicate_band(const fpm_ctx *) { return 2e-6; }

}  // namespace fpm
