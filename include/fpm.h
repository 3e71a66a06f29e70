/*
 * fpm.h -- C ABI of the MI355X particle hot path (OpenFPM, arXiv 1804.07598).
 *
 * The library implements, in hand-written HIP kernels for gfx950, the
 * data-parallel core of the paper's particle codes: cell lists and Verlet
 * lists (section 2, refs [45, 46]), the Lennard-Jones interaction of the MD
 * client (section 4.1 and its listing), the weakly compressible SPH sums of
 * section 4.2 (Eqs. 1-5) and velocity-Verlet time stepping (section 4.1).
 * Periodic images take the place of the paper's ghost layers: everything runs
 * on one device.
 *
 * Conventions for every entry point
 *  - Return value: FPM_OK (0) or a negative FPM_E* code; fpm_last_error()
 *    gives a message.  No C++ exception crosses this interface.
 *  - Pointers named d_* are device pointers; h_* are host pointers.  The
 *    library never frees caller memory and never keeps a caller pointer beyond
 *    the call, except the workspace (fpm_set_workspace) which it borrows until
 *    fpm_destroy or the next fpm_set_workspace.
 *  - The library allocates no device memory: the caller queries
 *    fpm_workspace_size() and hands in one buffer.
 *  - All device work is enqueued asynchronously on the stream given to
 *    fpm_create (a hipStream_t passed as void*; NULL = the null stream).
 *    Results in device memory are valid once the stream has been synchronised.
 *    Only fpm_check and fpm_read_counters synchronise.
 *  - Particle arrays in the caller's order are (n, 3) row-major float32.
 *    Inside the library particles live in cell-sorted order; the caller's
 *    order is restored by fpm_get_particles.
 *  - The box is [0, L[0]) x [0, L[1]) x [0, L[2]); periodic axes wrap.
 *    Positions are wrapped into the box at every neighbour-list rebuild;
 *    between rebuilds a particle may sit up to skin/2 outside a periodic face.
 *
 * Neighbour sets are defined in FP32, identically for every kernel: per axis
 * t = xj - xi; on a periodic axis, if t > L/2 the image (xj - L) - xi is used,
 * if t < -L/2 the image xj - (xi - L), otherwise t (the coordinate in the
 * upper half of the box moves down one period, which is exact: the image
 * separation is the exact one rounded once, and the sets are symmetric); then
 * d2 = (dx*dx + dy*dy) + dz*dz with every operation rounded separately (no
 * fused multiply-add), and j != i is a neighbour iff d2 <= R2, where R2 is
 * (r_cut + skin)^2 evaluated in FP64 and rounded once to FP32 (the listing of
 * section 4.1 rejects a pair only when rn > r_cut2).  Pair physics is then
 * evaluated in FP64 from the exact separation of the FP32 coordinates.
 */
#ifndef FPM_H
#define FPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPM_OK 0
#define FPM_EINVAL (-1)     /* bad argument, call order or non-finite input */
#define FPM_EHIP (-2)       /* HIP runtime error; message kept */
#define FPM_ECUTOFF (-3)    /* r_cut + skin >= L/2 on a periodic axis */
#define FPM_EOVERFLOW (-4)  /* a Verlet list exceeded max_nbr; lists invalid */
#define FPM_ENOWS (-5)      /* workspace missing or too small */
#define FPM_ENONFINITE (-6) /* a position or force became NaN/Inf */
#define FPM_EBADINDEX (-7)  /* debug build only: a list or cell-list entry out of range */

typedef struct fpm_ctx fpm_ctx;

/* Pair table of the Lennard-Jones potential of section 4.1,
 * V(r) = 4 eps ((sig/r)^12 - (sig/r)^6), truncated (not shifted) at r_cut.
 * Entries are in upper-triangular order AA, AB, BB; with n_types == 1 only
 * entry 0 is used.  Particle type is 0 (A) or 1 (B). */
typedef struct {
    int32_t n_types; /* 1 or 2 */
    float eps[3];
    float sig[3];
} fpm_lj_params;

/* Weakly compressible SPH of section 4.2 (Eqs. 1-5).  Kernels of support
 * 2h: 0 = Wendland C2, W = aD (1 - q/2)^4 (2q + 1), aD = 21 / (16 pi h^3);
 * 1 = the classic cubic spline the paper names, W = aD (1 - 3q^2/2 + 3q^3/4)
 * for q < 1, aD (2 - q)^3 / 4 for 1 <= q < 2, aD = 1 / (pi h^3) (the paper's
 * cutoff 2 sqrt(3) dp is h = sqrt(3) dp); q = r/h.  Boundary particles
 * (kind 1) enter every sum and evolve their density by Eq. 2, but do not
 * move.  Time stepping (fpm_sph_step): scheme 0 kick-drift-kick; scheme 1
 * the Verlet scheme with dynamic step (section 4.2, ref. [46]):
 * x' = x + dt v + dt^2/2 a, v' = v_prev + 2 dt a, rho' = rho_prev + 2 dt D,
 * where every verlet_every-th step (counted from the first step after the
 * state was set) takes the Euler form v' = v + dt a, rho' = rho + dt D. */
typedef struct {
    float h;        /* smoothing length; neighbours within 2h (r_cut = 2h) */
    float mass;     /* particle mass */
    float rho0;     /* reference density of Eq. 3 */
    float c0;       /* sound speed; Eq. 4 gives b = c0^2 rho0 / gamma */
    float gamma;    /* Tait exponent (7) */
    float alpha;    /* artificial-viscosity coefficient of Eq. 5 */
    float eta2;     /* eta^2 of Eq. 5's mu (absolute, length^2) */
    float g[3];     /* body acceleration (gravity) */
    float cfl;      /* CFL factor of the dynamic time step */
    int32_t kernel; /* 0 Wendland C2, 1 cubic spline */
    float cbar;     /* sound speed of Eq. 5's viscosity (the paper's
                       sqrt(g h_swl)); <= 0 takes c0 */
    int32_t scheme; /* 0 kick-drift-kick, 1 Verlet */
    int32_t verlet_every; /* scheme 1: period of the Euler-form steps (>= 1) */
} fpm_sph_params;

/* Discrete-element grains of section 4.5: the Silbert model with Hertzian
 * contacts (Eqs. 9-12) and the leapfrog of Eq. 13.  All grains have radius R,
 * mass m and moment of inertia I; (p, q) touch when |r_pq| < 2R (FP64 from the
 * exact separation of the FP32 coordinates, minimum image).  With
 * n = r_pq / |r_pq|, delta = 2R - |r_pq|, s = sqrt(delta / 2R), m_eff = m / 2
 * and the contact point midway between the centres (arm a = |r_pq| / 2):
 * v_pq = v_p - v_q - a (w_p + w_q) x n, v_n its normal part, v_t the rest;
 * the tangential history u_t of the pair grows by v_t dt and loses its normal
 * part (Eq. 10); F_n = s (kn delta n - gn m_eff v_n), F_t = s (-kt u_t -
 * gt m_eff v_t), F_t capped at mu |F_n| with u_t reset to match (Coulomb);
 * torque (-a n) x F_t.  Walls (bit 1: planes x = 0 and x = L_x; bit 2: floor
 * z = 0) add Eq. 11's normal force with delta = R - distance and m_eff = m.
 * Gravity m g.  A pair that separates forgets its history. */
typedef struct {
    float R, mass, inertia;
    float kn, kt;   /* elastic constants */
    float gn, gt;   /* damping constants */
    float mu;       /* Coulomb friction coefficient */
    float g[3];     /* gravity */
    float dt;       /* time step */
    int32_t walls;  /* bit mask, see above */
} fpm_dem_params;

/* ---- context (the library-start/finish calls of the section 4.1 listing) ---- */

/* Creates a context bound to `stream` (a hipStream_t, or NULL). */
int fpm_create(fpm_ctx **out, void *stream);
/* Destroys the context and any captured graphs; waits for its stream. */
int fpm_destroy(fpm_ctx *ctx);
/* Message of the last error on this context (never NULL). */
const char *fpm_last_error(const fpm_ctx *ctx);

/* ---- problem definition (the Box / bc / Ghost objects of the listing) ---- */

/* Box side lengths (FP32, > 0) and periodic flags (0/1) per axis: a single
 * system holding every particle later passed to fpm_set_particles. */
int fpm_set_box(fpm_ctx *ctx, const float h_L[3], const int32_t h_periodic[3]);
/* A batch of nsys independent systems (1 <= nsys <= 65536) sharing one context,
 * one set of neighbour parameters and one launch per step.  System s has box
 * h_L[3s..3s+2], periodic flags h_periodic[3s..3s+2] and h_counts[s] >= 1
 * particles; in every caller-order array the particles of system 0 come first,
 * then those of system 1, and so on (h_counts may be NULL only for nsys = 1).
 * Particles of different systems never interact.  Per-system outputs are
 * described at each call.  SPH calls accept batches of one only. */
int fpm_set_systems(fpm_ctx *ctx, int32_t nsys, const float *h_L, const int32_t *h_periodic,
                    const int64_t *h_counts);
/* Interaction radius, Verlet skin and Verlet-list capacity per particle.
 * The list radius is r_cut + skin; cells are the largest grid whose side is
 * >= that radius.  Returns FPM_ECUTOFF when r_cut + skin >= L/2 on a periodic
 * axis, FPM_EINVAL for max_nbr outside [1, 4096]. */
int fpm_set_neighbor_params(fpm_ctx *ctx, float r_cut, float skin, int32_t max_nbr);
/* Bytes of device workspace needed for n particles with the current box and
 * neighbour parameters (n <= 2^26 - 1; for a batch, n is the total). */
int fpm_workspace_size(fpm_ctx *ctx, int64_t n, size_t *h_bytes);
/* Lends the workspace (device memory, 256-byte aligned, >= the queried size
 * for the n later passed to fpm_set_particles). */
int fpm_set_workspace(fpm_ctx *ctx, void *d_ws, size_t bytes);

/* ---- particles (the vector_dist of the listing) ---- */

/* Copies n particles in (device arrays, caller order): positions inside the
 * box, velocities (may be NULL = zero) and types (NULL = all 0; SPH: kind,
 * 0 fluid / 1 boundary).  Builds the cell list and Verlet list.  Called
 * again with the same n and settings it keeps the workspace layout and the
 * captured step graphs and does not synchronise the stream (a restart from a
 * checkpoint); otherwise it lays the workspace out anew and waits for the
 * upload of its tables. */
int fpm_set_particles(fpm_ctx *ctx, int64_t n, const float *d_pos, const float *d_vel,
                      const int32_t *d_type);
/* New positions (device, caller order, n x 3) for the current particles,
 * on periodic axes in [-L, 2L) (the box or one period either side of it);
 * types and velocities are kept.  The neighbour structures are rebuilt on
 * next use when some particle moved more than skin/2 since the last build
 * (nearest periodic image) or lies more than skin/2 outside [0, L) on a
 * periodic axis; that rebuild wraps every position back into the box. */
int fpm_set_positions(fpm_ctx *ctx, const float *d_pos);
/* Host-side layout of system s: h_out = {n, first caller index, cells,
 * first entry of that system's cell offsets, cells along x, y, z, Verlet
 * build of the system: z-cells per workgroup of the column build (> 0), or
 * 0 particle by particle over whole cells, -1 particle by particle over
 * candidate windows, -2 lane groups over candidate windows, -3 lane groups
 * over whole cells (a grid of at most two cells per axis in a context built
 * by lockstep windows: the whole system, in the lockstep launch), -4
 * lockstep windows, -5 lockstep windows in ascending slot order (symmetric
 * half lists)}. */
int fpm_system_info(fpm_ctx *ctx, int32_t s, int64_t h_out[8]);
/* SPH only: per-particle density (device, caller order, n entries). */
int fpm_set_density(fpm_ctx *ctx, const float *d_rho);
/* Gathers the state back into caller order; any pointer may be NULL.
 * d_frc receives the last computed forces (LJ) or accelerations (SPH);
 * d_rho the SPH density, d_drho its rate. */
int fpm_get_particles(fpm_ctx *ctx, float *d_pos, float *d_vel, float *d_frc);
int fpm_get_sph(fpm_ctx *ctx, float *d_rho, float *d_drho);

/* ---- neighbour structures (getCellListSym / updateCellListSym) ---- */

/* Wraps positions into the box and rebuilds the cell list: cell index per
 * particle, per-cell counts, their exclusive prefix sum and a reordering of
 * particles by cell (inside a cell by FP32 z, ties in ascending caller
 * index).  Results of the last evaluation that live per particle (forces,
 * SPH rates, DEM torques and contacts) are not carried through the
 * reordering: read them before this call, or evaluate again after it. */
int fpm_build_cell_list(fpm_ctx *ctx);
/* Cell list in caller terms: d_offsets[ncells + 1] (exclusive scan of
 * counts) and d_order[n] (slot -> caller index).  h_ncell receives the grid.
 * For a batch, system s owns d_offsets[off_s .. off_s + ncells_s] (see
 * fpm_system_info), counted in the packed caller numbering, and h_ncell is
 * system 0's grid. */
int fpm_get_cell_list(fpm_ctx *ctx, int32_t h_ncell[3], int32_t *d_offsets, int32_t *d_order);
/* Rebuilds the Verlet list (radius r_cut + skin) from the current cell list. */
int fpm_build_verlet(fpm_ctx *ctx);
/* Verlet list in caller indices: d_counts[n], d_cols[n * max_nbr] (row i
 * holds the neighbours of caller particle i, unordered).  Returns
 * FPM_EOVERFLOW if the last build overflowed. */
int fpm_get_neighbors(fpm_ctx *ctx, int32_t *d_counts, int32_t *d_cols);

/* ---- interactions (applyKernel_in over the Verlet list) ---- */

/* Lennard-Jones forces on all particles from the current Verlet list, with
 * d_out[8 s + k] = {U, 0, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz}[k] of system s in FP64
 * (U = potential energy, W = sum over pairs of r (x) F; d_out may be NULL).
 * Forces are kept in the context. */
int fpm_lj_forces(fpm_ctx *ctx, const fpm_lj_params *prm, double *d_out);

/* ---- adjoint (reverse mode through the forces of section 4.1) ---- */

/* Vector-Jacobian product of the LJ forces at the current positions: given
 * d_lam = dL/dF (FP64, caller order, n x 3), writes d_gx = dL/dx (FP64, n x 3,
 * overwritten) and ADDS dL/dtheta to d_gtheta[6 s + k] for system s, with
 * theta = (eps_AA, eps_AB, eps_BB, sig_AA, sig_AB, sig_BB) (n_types = 1: only
 * entries 0 and 3 are non-zero; d_gtheta may be NULL).  The pair set is the
 * force set; the cut-off is not differentiated.  The cotangent is rounded to
 * FP32 per particle before the pair loop (relative error at most 2^-24 per
 * component; the neighbour gathers then move 16 bytes per pair, as for the
 * positions); pair terms and all sums are FP64.  dL/deps is computed from the
 * unit-depth pair force, so it is exact at eps = 0 too. */
int fpm_lj_force_vjp(fpm_ctx *ctx, const fpm_lj_params *prm, const double *d_lam, double *d_gx,
                     double *d_gtheta);
/* One step of the reverse velocity-Verlet recursion (unit mass) at the
 * current positions x_{k+1}, on caller-order FP64 arrays of n x 3:
 *   lam = fbar + dt/2 vbar;  xbar += VJP_x(lam);  gtheta += VJP_theta(lam);
 *   vbar += dt xbar;  fbar = dt/2 vbar + d_floss
 * (d_floss = dL/dF_k of the loss, may be NULL = 0), which turns the
 * cotangents of (x_{k+1}, v_{k+1}, F_{k+1}) into those of (x_k, v_k, F_k).
 * With last = 1, at x_0: xbar += VJP_x(fbar), gtheta += VJP_theta(fbar) only.
 * Afterwards xbar, vbar = dL/dx_0, dL/dv_0.  d_gtheta as in fpm_lj_force_vjp. */
int fpm_lj_adjoint_step(fpm_ctx *ctx, const fpm_lj_params *prm, float dt, const double *d_floss,
                        double *d_xbar, double *d_vbar, double *d_fbar, double *d_gtheta,
                        int32_t last);

/* The reverse sweep over a recomputed segment of nsteps velocity-Verlet steps
 * (section 4.1's step, differentiated): for k = nsteps - 1 down to 0, the
 * positions become d_xs + 3 n k (device, caller order, n x 3 FP32 each: the
 * positions after step k, as fpm_step_record writes them) and one
 * fpm_lj_adjoint_step follows with d_floss = h_floss[k] (h_floss: host array
 * of nsteps device pointers, NULL entries for steps without a loss term).
 * Results, rebuild decisions and rebuild counts are identical to those
 * calls; the launches are queued without host synchronisation, and the
 * rebuild a step needs is accounted by its VJP launch instead of a separate
 * reduction.  Velocities are left as they were. */
int fpm_lj_adjoint_sweep(fpm_ctx *ctx, const fpm_lj_params *prm, float dt, int32_t nsteps,
                         const float *d_xs, const double *const *h_floss, double *d_xbar,
                         double *d_vbar, double *d_fbar, double *d_gtheta);

/* ---- time stepping (the getV kick/drift expressions of the listing) ---- */

/* One half of velocity Verlet with unit mass: half == 0 applies
 * v += dt/2 F; x += dt v (and updates the rebuild flag); half == 1 applies
 * v += dt/2 F. */
int fpm_integrate(fpm_ctx *ctx, float dt, int32_t half);
/* nsteps full velocity-Verlet steps with automatic Verlet-list rebuilds when
 * the largest displacement since the last build exceeds skin/2 (decided per
 * system), all on the device (graph-launched, no host synchronisation).
 * d_thermo, if not NULL, receives nsteps x nsys rows of 8 FP64 values
 * {U, KE, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz}: row (step t, system s) at
 * d_thermo[8 (t nsys + s)], for the state after step t + 1. */
int fpm_step(fpm_ctx *ctx, const fpm_lj_params *prm, float dt, int32_t nsteps,
             double *d_thermo);
/* nsteps steps as nsteps calls fpm_step(ctx, prm, dt, 1, NULL) make them
 * (identical trajectory), with the caller-order positions after step k
 * written to d_xs + 3 n k (device, n x 3 FP32 per step); no host
 * synchronisation.  For the recomputation of a checkpointed segment before
 * fpm_lj_adjoint_sweep. */
int fpm_step_record(fpm_ctx *ctx, const fpm_lj_params *prm, float dt, int32_t nsteps,
                    float *d_xs);

/* ---- SPH (section 4.2) ---- */

/* Rates of Eqs. 1-2 at the current state: accelerations (kept as forces) and
 * density rates; d_dt[1] (FP32, may be NULL) receives the CFL time step
 * dt = cfl * min(min_a sqrt(h/|f_a|), h / (c0 + max_ab |mu_ab|)). */
int fpm_sph_rates(fpm_ctx *ctx, const fpm_sph_params *prm, float *d_dt);
/* nsteps time steps of prm->scheme with the dynamic dt on the device (the
 * dt of a step comes from the rates at its start); d_hist (may be NULL)
 * receives nsteps FP64 rows {t, dt, KE, max|v|}.  FPM_EINVAL for an unknown
 * kernel or scheme, or verlet_every < 1 with scheme 1. */
int fpm_sph_step(fpm_ctx *ctx, const fpm_sph_params *prm, int32_t nsteps, double *d_hist);

/* Symmetric half lists (the section 4.1 listing's getCellListSym and
 * applyKernel_in_sym; the reaction step is section 3.4's ghost_put): with
 * on = 1, fpm_lj_forces and fpm_step evaluate every pair once, at the pair's
 * lower slot, and hand the reaction to the partner.  Lists are then kept in
 * ascending slot order; each rebuild also records, for every pair, where it
 * sits in the partner's list.  A first pass stores each pair's force factor
 * beside the pair's list entry and the particle's own sum, a second pass
 * gathers the lower partners' factors and adds their reactions in list
 * order: no atomics, results repeat bit for bit.  Forces, energy and
 * virial agree with the full-list path to rounding.  Call before
 * fpm_workspace_size and fpm_set_particles (the workspace grows by 10 bytes
 * per list entry and 28 per particle); not with DEM storage.  FPM_EOVERFLOW
 * from fpm_check if a pair was missing from one side (lists overflowed). */
int fpm_set_symmetric(fpm_ctx *ctx, int32_t on);

/* ---- DEM (section 4.5) ---- */

/* Turns on DEM storage: per-grain angular velocities and the contact
 * history.  The history of a pair is kept beside its Verlet-list entry (one
 * u_t per list entry, so the workspace grows by 16 B per list slot); across
 * a list rebuild up to max_contacts (1..64) contacts per grain are carried
 * over by partner, and max_contacts also sizes the rows of
 * fpm_get_contacts.  Call before fpm_workspace_size and fpm_set_particles
 * (single system; the Verlet list radius r_cut + skin must cover 2R).  The
 * angular velocity shares storage with SPH's Verlet scheme: do not mix DEM
 * and SPH on one context. */
int fpm_set_dem(fpm_ctx *ctx, int32_t max_contacts);
/* Angular velocities (device, caller order, n x 3; NULL = zero); clears the
 * contact history.  fpm_set_particles starts from zero and no history. */
int fpm_set_omega(fpm_ctx *ctx, const float *d_omega);
/* Forces and torques at the current state, advancing the contact history by
 * one step (Eq. 10 is part of the evaluation).  FPM_EOVERFLOW (from
 * fpm_check) when a grain has more than max_contacts contacts. */
int fpm_dem_forces(fpm_ctx *ctx, const fpm_dem_params *prm);
/* nsteps of: forces (as fpm_dem_forces), then the leapfrog of Eq. 13,
 * v += dt F / m, x += dt v, w += dt T / I; lists rebuilt on the device when
 * some grain moved more than skin/2. */
int fpm_dem_step(fpm_ctx *ctx, const fpm_dem_params *prm, int32_t nsteps);
/* Caller-order outputs (any may be NULL): angular velocities and the last
 * torques (n x 3), contact counts (n). */
int fpm_get_dem(fpm_ctx *ctx, float *d_omega, float *d_torque, int32_t *d_ncontact);
/* The contacts of the last evaluation with their history, in caller order:
 * d_ids (n x max_contacts partner caller indices in list order, then -1) and
 * d_ut (n x max_contacts x 3, zero after the last contact). */
int fpm_get_contacts(fpm_ctx *ctx, int32_t *d_ids, float *d_ut);

/* ---- allocation-free entry point ---- */

/* Bytes of the static device array behind fpm_lj_forces_static (one array per
 * GPU, held until the process ends): with max_nbr = 128 it takes about 90,000
 * particles. */
#define FPM_STATIC_SCRATCH_BYTES (64u << 20)
/* For callers that may not allocate device memory (serving loops and harnesses
 * that forbid hipMalloc): the forces, energy and virial of fpm_lj_forces for n
 * particles given in this call, computed in a static device array of
 * FPM_STATIC_SCRATCH_BYTES instead of a caller workspace.  ctx supplies the
 * box (a single system), the neighbour parameters, the launch shapes and the
 * stream; its own workspace, particles and forces are not touched, and no
 * fpm_set_workspace is needed.  d_pos (n x 3, caller order, inside the box),
 * d_type (n, NULL = all 0), d_frc (n x 3, written) and d_out (8 FP64 as in
 * fpm_lj_forces, may be NULL) are device pointers.  Returns FPM_ENOWS when
 * the particles need more than FPM_STATIC_SCRATCH_BYTES (checked before any
 * device work), FPM_EINVAL for a batch, DEM storage or bad arguments.
 * Allocates no device memory.  The stream is synchronised once (when the
 * small system tables are copied).  Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (several streams or threads) race. */
int fpm_lj_forces_static(fpm_ctx *ctx, const fpm_lj_params *prm, int64_t n, const float *d_pos,
                         const int32_t *d_type, float *d_frc, double *d_out);

/* ---- status ---- */

/* Synchronises the stream and reports device-side flags: FPM_EOVERFLOW if a
 * list overflowed, FPM_ENONFINITE if a non-finite value was seen, and in the
 * debug build (libfpm_checked.so: cell list and Verlet lists validated after
 * every rebuild, every list entry the LJ force and VJP kernels read checked
 * against its system's slots) FPM_EBADINDEX if an entry was out of range. */
int fpm_check(fpm_ctx *ctx);
/* Synchronises and reads counters: h_out[0] = rebuilds so far (summed over
 * the systems of a batch),
 * h_out[1] = largest Verlet-list length seen in the last build,
 * h_out[2] = total Verlet-list entries of the last build. */
int fpm_read_counters(fpm_ctx *ctx, int64_t h_out[3]);

/* ---- measurement and tuning ---- */

/* Launch shapes (0 = automatic).  verlet_path: 1 builds Verlet lists particle
 * by particle over whole neighbour cells, 2 by column blocks staged in LDS,
 * 3 particle by particle over candidate windows, 4 over the same windows with
 * a group of lanes per particle and each 64-slot row of lists staged in LDS,
 * 5 one lane per particle with the lanes of a wavefront walking their windows
 * in step (2, 3, 4 and 5 where the grid has >= 3 cells per axis; elsewhere
 * paths 2 and 3 take path 1 and paths 4 and 5 run lane groups over whole
 * cells; automatic takes 3 when max_nbr is at most 48, else 5 when the
 * context holds at least 131,072 particles (all systems together) and 4
 * below that, and lane groups over whole
 * cells for small grids; max_nbr stands in for the list length here, since
 * the lists are not known before the first build).  zblock: z-cells per column workgroup (1..64);
 * for path 4, lanes per particle (0 = 8, 4, 8 or 16; other values are
 * FPM_EINVAL).  unroll: list entries in
 * flight per lane in the force kernel (4 or 8).  Results do not depend on
 * them.  Changing verlet_path or zblock drops the particles (call
 * fpm_set_particles again). */
int fpm_set_tuning(fpm_ctx *ctx, int32_t verlet_path, int32_t zblock, int32_t unroll);

/* With on = 1, every launch made outside a graph of the kernels named
 * "lj_force", "lj_vjp", "verlet_build", "cell_build", "integrate", "sph_rates" is
 * bracketed by two HIP events recorded on the context's stream, and fpm_step
 * issues its steps without graphs so that each step's fused force kernel
 * ("lj_step": forces, closing kick, next opening kick and drift) is timed the
 * same way (identical results); on = 0 stops recording and drops pending
 * records. */
int fpm_set_profiling(fpm_ctx *ctx, int32_t on);
/* Synchronises, then returns the mean duration in milliseconds (h_ms) and the
 * number (h_count) of the recorded launches of `kernel` since the last call
 * for that name; the records are consumed. */
int fpm_kernel_time(fpm_ctx *ctx, const char *kernel, double *h_ms, int64_t *h_count);

#ifdef __cplusplus
}
#endif
#endif /* FPM_H */
