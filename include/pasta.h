/*
 * pasta.h -- C ABI of libpasta, an MI355X (gfx950) implementation of the
 * molecular-dynamics hot path of the semiclassical nuclear-pasta model of
 * Caplan, Schneider, Horowitz and Berry, "Pasta Nucleosynthesis: Molecular
 * dynamics simulations of nuclear statistical equilibrium" (arXiv:1412.8502).
 *
 * The model (Sec. II.A): N point nucleons of mass M in a periodic cube of
 * side L(t); neutrons and protons interact through the two-body potentials
 * of Eq. (1a-c) with the constants of Table I; the nuclear part is cut at
 * r_nuc, the screened Coulomb part between protons is not cut; only the
 * nearest periodic image interacts.  Positions and velocities advance by
 * velocity Verlet; after each step the box grows as l(t) = l(0)(1 + xi_dot t)
 * (Eq. 3a) without moving the particles; every 100 steps the velocities are
 * rescaled to <KE> = (3/2) kT.  The cluster algorithm of Sec. II.C links
 * protons closer than r_pp and attaches neutrons closer than r_np.
 *
 * Conventions for every entry point:
 *  - Units: MeV, fm, fm/c; velocities in units of c; k_B = 1.
 *  - d_* arguments are device pointers (HIP device memory of the current
 *    device), h_* are host pointers.  Every buffer is owned by the caller;
 *    the library never allocates or frees device memory.  Scratch memory is
 *    passed in as a caller-owned workspace of at least the size the matching
 *    *_workspace query returns (256-byte aligned).
 *  - Particle arrays keep the caller's order: pos and vel are [n][3] FP64
 *    (x, y, z interleaved), species is [n] uint8 (1 = proton, 0 = neutron).
 *    Positions must lie in [0, L).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *    asynchronously on it; only calls that fill h_* outputs synchronise.
 *  - Every call returns PASTA_OK (0) or a negative PASTA_E* code;
 *    pasta_last_error() then describes the failure (thread-local string).
 *    No C++ exception crosses the ABI.  Device-side checks (non-finite
 *    forces or velocities, a particle moving more than a cell per step) set
 *    an error word that the next synchronising call reports as
 *    PASTA_EDEVICE.
 */
#ifndef PASTA_H
#define PASTA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PASTA_OK 0
#define PASTA_EINVAL (-1)     /* bad argument: null pointer, n < 0, bad mode  */
#define PASTA_EBOX (-2)       /* L < 2 r_cut: the nearest image is ambiguous  */
#define PASTA_EWORKSPACE (-3) /* workspace too small or misaligned           */
#define PASTA_EHIP (-4)       /* a HIP runtime call failed (message has it)   */
#define PASTA_EDEVICE (-5)    /* device error word set (see pasta_last_error) */
#define PASTA_ENOMEM (-6)     /* host allocation failed                       */

/* Precision of the pair arithmetic.
 * PASTA_FP64:  positions, pair arithmetic (differences, exp, sqrt) and
 *              accumulation in IEEE double.
 * PASTA_MIXED: pair differences formed exactly from 32-bit fixed-point
 *              coordinates (x/L * 2^32, so the nearest image is the
 *              two's-complement wrap of the difference), pair arithmetic
 *              (Gaussians, screened Coulomb, exp, rsqrt) in FP32, each
 *              thread's FP32 sum over at most one source tile added into
 *              FP64 per-particle accumulators.  Positions, velocities, the
 *              box and the Verlet update stay FP64. */
#define PASTA_FP64 0
#define PASTA_MIXED 1

/* Which terms a force call evaluates (bit mask). */
#define PASTA_TERM_NUCLEAR 1 /* Eq. (1a,b), cut at r_nuc           */
#define PASTA_TERM_COULOMB 2 /* Eq. (1c) screened Coulomb (r_coul)  */
#define PASTA_TERM_ALL 3

/* Interaction parameters (Eq. 1, Table I, Sec. II.A). */
typedef struct pasta_potential {
    double a;           /* MeV, short-range repulsion (Table I: 110)        */
    double b;           /* MeV, intermediate-range attraction (Table I: -26) */
    double c;           /* MeV, isospin term (Table I: 24); b - c for n-p,
                           b + c for n-n and p-p                            */
    double Lambda;      /* fm^2, range of the Gaussians (Table I: 1.25)     */
    double lambda_s;    /* fm, Coulomb screening length (fixed to 10 fm)    */
    double alpha_hbarc; /* MeV fm, alpha hbar c = 1.4399645                 */
    double mass;        /* MeV, nucleon mass (939)                          */
    double r_nuc;       /* fm, nuclear cutoff (11.5)                        */
    double r_coul;      /* fm, Coulomb cutoff: INFINITY = uncut, the paper's
                           model (Sec. II.A cuts only the nuclear part); a
                           finite value keeps the proton pairs with
                           r^2 < r_coul^2 (the include test is decided on the
                           FP64 r^2 in both precisions) and requires
                           L >= 2 r_coul.  The batched path takes INFINITY
                           only.                                           */
} pasta_potential;

/* Integration parameters (Sec. II.A: velocity Verlet, Eq. 3 box growth,
 * velocity rescale every 100 steps). */
typedef struct pasta_integrator {
    double dt;               /* fm/c time step (the paper: 2)               */
    double xi_dot;           /* c/fm box expansion rate (0 = fixed box)     */
    double T;                /* MeV thermostat temperature                  */
    int32_t rescale_every;   /* rescale v to KE = 1.5 N T after every step
                                whose index is a multiple of this; 0 = off  */
    int32_t scale_positions; /* 0: positions not moved by the box growth
                                (the paper); 1: x *= L_{n+1}/L_n (variant) */
} pasta_integrator;

/* Kernel choices, process-wide; read at every launch (the list settings:
 * when a workspace is sized and when a simulation is created).
 * nuclear_variant: 0 = dense cell tiles (every candidate pair through the
 *   full pair arithmetic); 1 = screened + compacted (a conservative 16-bit
 *   screen, survivors listed in LDS, exact arithmetic on listed pairs only;
 *   the default); 2 = neighbour lists with a halo (Sec. II.B.1): each target
 *   lists the sources within r_nuc + list_skin, built from cells at least
 *   that wide; the forces read only the lists; a simulation rebuilds cells
 *   and lists, all at once, only in steps where
 *       2 max_i |u_i| + sqrt(3) |L - L_build| >= list_skin
 *   (u_i = nearest-image displacement since the last build), the condition
 *   under which a pair now inside r_nuc may have been outside r_nuc +
 *   list_skin at the build.  The decision is taken on the device.  If the
 *   list memory runs out, the forces fall back to the screened cell sweep
 *   over the cells of the last build until the next build.  One-shot
 *   pasta_forces builds and uses the lists once; 3 = as 1 with 8 lanes per
 *   target and 32 targets per work item (smaller target boxes, so fewer
 *   staged sources).  Cells are binned by octant inside, so the targets of
 *   a work item are spatially compact; 4 = Newton's third law: each item
 *   stages the half stencil (its cell and the 13 neighbours with a
 *   lexicographically positive offset), every unordered pair inside r_nuc
 *   is evaluated once, the reaction on the source is accumulated in 64-bit
 *   fixed point (2^-43 MeV/fm; order-independent sums, so results are
 *   deterministic) and added by the combine kernel; always the fused form;
 *   grids of fewer than 3 cells per side run as 3.  The batched path runs
 *   2 and 4 as 3 (it rebuilds its cells every step) and reads the variant
 *   at creation.  A simulation keeps the variant it was created with.  All
 *   variants give the same forces to rounding.
 * coulomb_splits: number of source ranges per Coulomb target tile, 1..32;
 *   0 = automatic (about 2^19 / Z, at most 32).
 * fused_forces: 0 = the Coulomb kernel, then the nuclear kernel whose
 *   epilogue adds the Coulomb partials and applies the half kick; 1 = one
 *   launch holding both kinds of work items (they share the GPU) followed by
 *   a small combine + kick kernel.
 * coulomb_form: 0 = gather tiles (every ordered proton pair, summed per
 *   target; coulomb_splits applies); 1 = pairwise: every unordered pair once
 *   (Newton's third law), the reaction carried along the wavefront by a
 *   lane rotation; 256-proton super-blocks, one partial per super-block and
 *   proton (used when those partials fit the workspace's partial buffer,
 *   else the gather form); 2 = pairwise, each item adding its per-proton
 *   sums into 64-bit fixed-point accumulators (2^-43 MeV/fm, integer
 *   atomics: order-independent, deterministic sums; no partials, no size
 *   limit; a proton sum outside +-2^19 MeV/fm sets the device error word);
 *   only in the fused form in mixed precision, elsewhere it runs as 1.  The
 *   batched path reads it at creation and plans each system's Coulomb term
 *   the same way (form 2 in mixed precision only).
 * list_skin: the halo delta_r of variant 2, fm, in (0, 64] (default 2).
 * batch_wgs_per_cu: workgroups per compute unit of the persistent batched
 *   kernel (mode 0), 1..8, capped at what fits; 0 = as many as fit.  Read
 *   when a batch is created.
 * list_pool_scale: list memory relative to the default sizing, in (0, 1000]
 *   (default 1; the default holds 1.5 x the expected entries per lane at the
 *   starting density plus a Poisson margin).
 * nuclear_tile: sources per LDS tile of variant 3's items: 0 or 512 (the
 *   default), 256 (more workgroups fit per CU, more end-of-tile drains) or
 *   1024 (fewer drains, fewer workgroups per CU); a length other than the
 *   default always runs in the fused form.  The other variants and the
 *   batched path use their default tiles. */
typedef struct pasta_tuning {
    int32_t nuclear_variant;
    int32_t coulomb_splits;
    int32_t fused_forces;
    int32_t coulomb_form;
    double list_skin;
    double list_pool_scale;
    int32_t batch_wgs_per_cu;
    int32_t nuclear_tile;
} pasta_tuning;
int pasta_set_tuning(const pasta_tuning* t);
int pasta_get_tuning(pasta_tuning* out);
/* Autotuner: builds the cell list of the given state once, then times the
 * Coulomb + nuclear kernels (reps evaluations of the forces each, without
 * energies as in a simulation step; HIP events; the list of candidates is
 * timed twice and each keeps its faster pass) for every
 * candidate setting -- nuclear variant {0, 1, 3, 4 (fused only), 3 with
 * 256- and 1024-source tiles (fused only)} x Coulomb
 * {gather with splits S/2, S, 2S around the automatic S, pairwise,
 * pairwise into fixed-point accumulators (fused, mixed precision)} x
 * fused_forces {0, 1}
 * -- and returns the fastest
 * in *h_best (the list fields copied from the current setting; the list
 * form's cost depends on how often the lists are rebuilt, which a single
 * state does not tell, so it is not a candidate).  Optional
 * outputs: h_cands[] / h_ms[] (capacity *h_ncand on entry, count on exit).
 * Does not change the process-wide setting.  Synchronises. */
int pasta_autotune_workspace(const pasta_potential* pot, int32_t precision, int64_t n, double L,
                             size_t* h_bytes);
int pasta_autotune(const pasta_potential* pot, int32_t precision, int64_t n, double L,
                   const double* d_pos, const uint8_t* d_species, void* d_work,
                   size_t work_bytes, void* stream, int32_t reps, pasta_tuning* h_best,
                   double* h_ms, pasta_tuning* h_cands, int32_t* h_ncand);

/* Fills *out with the paper's values (Table I, lambda = 10 fm, M = 939 MeV,
 * r_nuc = 11.5 fm, alpha hbar c = 1.4399645 MeV fm, r_coul = INFINITY). */
void pasta_potential_paper(pasta_potential* out);

/* Thread-local description of the last error (never NULL). */
const char* pasta_last_error(void);

/* Library version string. */
const char* pasta_version(void);

/* ------------------------------------------------------------------ a1 --
 * Cell list (Sec. II.B.2 bins the volume into cubic cells no narrower than
 * the interaction range).  ncell = the largest integer with L/ncell >= r_cut.
 * A particle's cell along an axis is floor(x * (ncell/L)) clamped to
 * ncell-1; the linear cell index is (cz*ncell + cy)*ncell + cx.  Protons
 * come first: bin = cell for a proton, ncell^3 + cell for a neutron.
 * Outputs: d_perm[n] = particle indices in increasing (bin, index) order;
 * d_cell_start[2*ncell^3 + 1] = first position of each bin in d_perm (the
 * last entry is n); *h_ncell = ncell.  Requires L >= 2 r_cut. */
int pasta_cell_list_workspace(int64_t n, double L, double r_cut, size_t* h_bytes);
/* Sizing query: *h_ncell = the ncell a cell list of box side L and cutoff
 * r_cut uses (so d_cell_start needs 2 ncell^3 + 1 entries). */
int pasta_cell_dims(double L, double r_cut, int32_t* h_ncell);
int pasta_cell_list(int64_t n, double L, double r_cut, const double* d_pos,
                    const uint8_t* d_species, int32_t* d_cell_start, int32_t* d_perm,
                    int32_t* h_ncell, void* d_work, size_t work_bytes, void* stream);

/* -------------------------------------------------------------- a2 + a3 --
 * One force evaluation (Eq. 1a-c): for every particle i,
 *   F_i = sum_{j != i} -dV_ij/dr (x_i - x_j)/r   (nearest image),
 *   E_i = (1/2) sum_{j != i} V_ij               (sum_i E_i = total energy).
 * `terms` selects the nuclear and/or Coulomb parts.  d_force is [n][3]
 * MeV/fm, d_epot is [n] MeV (may be NULL).  Requires L >= 2 r_nuc (and
 * L >= 2 r_coul for a finite Coulomb cutoff, which uses the gather form).
 * Internally: a1 cell list with r_cut = r_nuc (r_nuc + list_skin and the
 * neighbour lists in the list form), the nuclear kernel, and the all-pairs
 * screened-Coulomb tile kernel.  The workspace query and the call must see
 * the same process-wide setting. */
int pasta_forces_workspace(const pasta_potential* pot, int32_t precision, int64_t n,
                           double L, size_t* h_bytes);
int pasta_forces(const pasta_potential* pot, int32_t precision, int32_t terms, int64_t n,
                 double L, const double* d_pos, const uint8_t* d_species, double* d_force,
                 double* d_epot, void* d_work, size_t work_bytes, void* stream);

/* ------------------------------------------- forces without allocation --
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc, code that must not grow its footprint):
 * the same force evaluation as pasta_forces, with the same arguments minus
 * the workspace.  Its scratch memory is a static device array of
 * PASTA_NOALLOC_SCRATCH_BYTES inside the library, which each device the
 * library runs on holds until the process ends; the call itself allocates
 * nothing.  The array's device address is looked up on the first call on
 * each device.  Returns PASTA_EWORKSPACE, without touching the outputs, when
 * the workspace pasta_forces_workspace reports for these arguments (under
 * the current tuning) exceeds PASTA_NOALLOC_SCRATCH_BYTES.  Every call on a
 * device shares that device's array: calls that overlap in time on one
 * device (several host threads or streams) race and corrupt each other's
 * results, so serialise them.  Like pasta_forces, it synchronises the
 * stream once (to size the Coulomb launch). */
#define PASTA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int pasta_forces_noalloc(const pasta_potential* pot, int32_t precision, int32_t terms,
                         int64_t n, double L, const double* d_pos, const uint8_t* d_species,
                         double* d_force, double* d_epot, void* stream);

/* ------------------------------------------------------------------ a4 --
 * Simulation handle: velocity Verlet in an expanding periodic box.
 * Step n -> n+1 (global step index n):
 *   v += (dt/2M) F_n;  x += dt v;
 *   L_{n+1} = L0 (1 + xi_dot (n+1) dt)   (Eq. 3a, from the index, never
 *                                          accumulated);
 *   [scale_positions: x *= L_{n+1}/L_n];  wrap x into [0, L_{n+1});
 *   F_{n+1} = F(x, L_{n+1});  v += (dt/2M) F_{n+1};
 *   if rescale_every > 0 and (n+1) % rescale_every == 0:
 *       v *= sqrt(1.5 N T / KE),  KE = sum (1/2) M v^2.
 * The simulation keeps its own copy of the state, in the sorted order of
 * its cell list.  It reads the caller's d_pos and d_vel (caller order) in
 * pasta_sim_create and pasta_sim_set_state, and writes the current state
 * back into them at the end of every pasta_sim_step call (in stream order);
 * changing them in between has no effect on the run.  d_species must stay
 * valid and unchanged.  L_max bounds the largest box the run will
 * reach (it sizes the cell grid); a step that would exceed it fails with
 * PASTA_EBOX.  L_start (workspace query) is the box side at the starting
 * step: with the list form it sets the density the list memory is sized for
 * (a simulation gives the list memory whatever the workspace holds beyond
 * the rest, so a larger workspace means more list memory).
 * pasta_sim_create evaluates F at the starting state. */
typedef struct pasta_sim pasta_sim;
int pasta_sim_workspace(const pasta_potential* pot, const pasta_integrator* integ,
                        int32_t precision, int64_t n, double L_start, double L_max,
                        size_t* h_bytes);
int pasta_sim_create(const pasta_potential* pot, const pasta_integrator* integ,
                     int32_t precision, int64_t n, double L0, int64_t step0, double L_max,
                     double* d_pos, double* d_vel, const uint8_t* d_species, void* d_work,
                     size_t work_bytes, void* stream, pasta_sim** out);
/* Advances nsteps steps (asynchronous). */
int pasta_sim_step(pasta_sim* sim, int64_t nsteps);
/* Synchronises; returns kinetic and potential energy (MeV), the box side and
 * the global step index of the current state.  Any pointer may be NULL.
 * Steps evaluate forces only; the potential energy (and the energy shares of
 * pasta_sim_forces) of the current state is evaluated when first asked for,
 * with one more force evaluation that rewrites the same forces. */
int pasta_sim_energies(pasta_sim* sim, double* h_ekin, double* h_epot, double* h_L,
                       int64_t* h_step);
/* Copies the current forces ([n][3], caller order) and energy shares ([n])
 * to caller buffers (asynchronous; either pointer may be NULL). */
int pasta_sim_forces(pasta_sim* sim, double* d_force, double* d_epot);
/* Synchronises; counts unordered pairs inside r_nuc and proton pairs whose
 * Coulomb term is evaluated, at the current state. */
int pasta_sim_pair_counts(pasta_sim* sim, int64_t* h_nuclear, int64_t* h_coulomb);
/* Checkpoint/restart: the state is (d_pos, d_vel, step); L follows from the
 * step index.  set_state re-evaluates the forces. */
int pasta_sim_get_step(pasta_sim* sim, int64_t* h_step);
/* Copies the current state into caller buffers (d_pos, d_vel: [n][3],
 * caller order; either may be NULL) and returns its global step index in
 * *h_step (may be NULL).  Asynchronous for the copies. */
int pasta_sim_get_state(pasta_sim* sim, double* d_pos, double* d_vel, int64_t* h_step);
int pasta_sim_set_state(pasta_sim* sim, const double* d_pos, const double* d_vel,
                        int64_t step);
/* Per-kernel timing with HIP events on the simulation's stream.  When on,
 * every launch is bracketed by events; pasta_sim_kernel_times synchronises
 * and returns, per kernel class, the summed milliseconds and launch counts
 * since timing was switched on (arrays of PASTA_KERNEL_CLASSES entries). */
#define PASTA_KERNEL_CLASSES 9
int pasta_sim_set_timing(pasta_sim* sim, int32_t on);
int pasta_sim_kernel_times(pasta_sim* sim, double* h_ms, int64_t* h_launches);
const char* pasta_kernel_class_name(int32_t k);
/* Neighbour-list statistics (zeros unless the simulation uses the list
 * form).  Synchronises.  builds: list builds so far (the initial one
 * included); overflows: builds that ran out of list memory; max_disp: max
 * |u| (fm) at the last rebuild decision; rows_used / rows_capacity: list
 * memory rows (256 entries each) taken by the last build / available. */
int pasta_sim_list_stats(pasta_sim* sim, int64_t* h_builds, int64_t* h_overflows,
                         double* h_max_disp, int64_t* h_rows_used, int64_t* h_rows_capacity);
void pasta_sim_destroy(pasta_sim* sim);

/* ------------------------------------------------------------------ a5 --
 * Cluster algorithm (Sec. II.C).  Protons i, j are linked when their
 * nearest-image distance satisfies |d|^2 <= r_pp^2; proton clusters are the
 * connected components (an isolated proton is its own cluster).  A neutron
 * joins the cluster of its nearest proton with |d|^2 <= r_np^2 (ties go to
 * the lower proton index); otherwise it is free.  Distances are computed in
 * FP64 as d = x_i - x_j, d -= L if d > L/2, d += L if d < -L/2,
 * |d|^2 = (dx*dx + dy*dy) + dz*dz, without fused multiply-add.
 * Outputs: d_label[n] = canonical cluster label (clusters numbered 0..K-1 in
 * increasing order of their smallest proton index; -1 = free neutron);
 * d_hist_A[n+1] and d_hist_Z[n+1]: number of clusters with mass number A and
 * charge Z; *h_nclusters = K, *h_nfree = free neutrons.  Synchronises.
 * Requires L >= 2 max(r_pp, r_np). */
int pasta_cluster_workspace(int64_t n, double L, double r_pp, double r_np, size_t* h_bytes);
int pasta_cluster(int64_t n, double L, const double* d_pos, const uint8_t* d_species,
                  double r_pp, double r_np, int32_t* d_label, int32_t* d_hist_A,
                  int32_t* d_hist_Z, int32_t* h_nclusters, int32_t* h_nfree, void* d_work,
                  size_t work_bytes, void* stream);

/* ------------------------------------------------------------------ a6 --
 * Batched systems: nsys independent boxes (the paper's grid of runs over Y_P
 * and T, Sec. III.B), each with its own n, L0 and integrator, advanced
 * together.  Particle arrays are the concatenation of the systems' arrays
 * (system s occupies rows [sum_{k<s} n_k, ... + n_s)); each system follows
 * exactly the pasta_sim_step definition above.  Z per system is counted from
 * d_species at creation.
 * mode 0: one persistent kernel launch per step whose phases are separated by
 *         device-wide barriers (the grid is sized to be resident; a barrier
 *         wait is bounded and reports PASTA_EDEVICE instead of hanging);
 * mode 1: the same phases as one kernel launch each.
 * Steps are captured once into a hipGraph of steps_per_graph steps and
 * replayed; the batch works on an internal stream joined to `stream` by
 * events.  The batch keeps the state in its workspace, in the sorted order of
 * its cell lists: d_pos and d_vel are read at creation and hold the state of
 * every system after each pasta_batch_step call (stream-ordered); writes to
 * them between calls are not seen.  h_L_max[s] bounds system s's box. */
typedef struct pasta_batch pasta_batch;
int pasta_batch_workspace(const pasta_potential* pot, int32_t precision, int32_t nsys,
                          const int64_t* h_n, const double* h_L_max, size_t* h_bytes);
int pasta_batch_create(const pasta_potential* pot, int32_t precision, int32_t nsys,
                       const int64_t* h_n, const double* h_L0, const pasta_integrator* h_integ,
                       int64_t step0, const double* h_L_max, double* d_pos, double* d_vel,
                       const uint8_t* d_species, void* d_work, size_t work_bytes, int32_t mode,
                       int32_t steps_per_graph, void* stream, pasta_batch** out);
/* Advances every system nsteps steps, then synchronises and checks the
 * device error word: PASTA_EDEVICE if a device check failed (a non-finite
 * force, or, in mode 0, a barrier wait that hit its bound -- the persistent
 * kernel then stops advancing, and this call and every later step, forces
 * and energies call fail the same way). */
int pasta_batch_step(pasta_batch* b, int64_t nsteps);
/* Bound of one device-wide barrier wait of mode 0, in polls of about a
 * microsecond each (default 2^22).  A wait that reaches it sets the device
 * error word and every workgroup leaves the kernel instead of waiting on.
 * polls = 0 makes every wait but the last arriver's fail at once (this is
 * how the failure path is tested).  Synchronises; the captured steps are
 * re-captured at the next pasta_batch_step. */
int pasta_batch_set_wait_limit(pasta_batch* b, int64_t polls);
/* Synchronises; per-system kinetic and potential energies and box sides
 * (arrays of nsys; any may be NULL) and the global step index.  As for a
 * simulation, steps compute forces only and the energy shares of the
 * current state are evaluated when first asked for (here or by
 * pasta_batch_forces). */
int pasta_batch_energies(pasta_batch* b, double* h_ekin, double* h_epot, double* h_L,
                         int64_t* h_step);
/* Copies forces ([sum n][3]) and energy shares ([sum n]) of the current
 * state; synchronises and returns PASTA_EDEVICE, as pasta_batch_step does,
 * when the device error word is set. */
int pasta_batch_forces(pasta_batch* b, double* d_force, double* d_epot);
/* Synchronises; per-system unordered nuclear pairs inside r_nuc and Coulomb
 * pairs at the current state. */
int pasta_batch_pair_counts(pasta_batch* b, int64_t* h_nuclear, int64_t* h_coulomb);
/* Grid size of the persistent (or per-phase) launches and the mode. */
int pasta_batch_info(pasta_batch* b, int32_t* h_grid, int32_t* h_mode);
void pasta_batch_destroy(pasta_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* PASTA_H */
