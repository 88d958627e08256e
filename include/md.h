/*
 * md.h -- C ABI of the MI355X short-range molecular-dynamics hot path.
 *
 * The library computes, on one GPU, the steps of the cell-task method of
 * R. Meyer, "Efficient Parallelization of Short-Range Molecular Dynamics
 * Simulations on Many-Core Systems" (arXiv:1305.4196):
 *   - particles binned into linked cells of width >= cutoff (Sec. II.A);
 *   - Verlet neighbor lists generated cell by cell, each cell's work writing
 *     only its own particles' lists (Sec. II.A, II.C);
 *   - pair (Lennard-Jones) and many-body (Finnis-Sinclair-type EAM, the
 *     potential family of Sec. II.C) forces, with no particle updated by two
 *     workers at once (the invariant of Sec. II.A);
 *   - the equations of motion as a per-particle loop (Sec. II.A), here
 *     velocity Verlet;
 *   - adjoints of forces and energy, and replica batches (the replica-carrying
 *     functor of Sec. II.C).
 *
 * Conventions (all calls):
 *   - Pointers are DEVICE pointers unless marked [host].
 *   - Per-atom arrays are structure-of-arrays double[3][N]: all x, then all y,
 *     then all z, in the caller's ("user") atom order.  The caller owns every
 *     buffer it passes; the library never frees caller memory.
 *   - Atoms of replica r are user indices [offsets[r], offsets[r+1]).  Each
 *     replica is an orthorhombic periodic box with origin 0.
 *   - Every call enqueues work on `stream` (a hipStream_t, passed as void*) and
 *     returns without synchronising, except where marked "synchronises".
 *   - Return values: MD_OK or a negative md_status.  Argument errors are found
 *     on the host before anything is enqueued.  Conditions found on the device
 *     (neighbor-list overflow, non-finite forces) set sticky flags that
 *     md_get_status reports.
 *   - One context per stream; contexts share no state.
 */
#ifndef MD_H
#define MD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MD_OK = 0,
    MD_ERR_ARG = -1,        /* bad argument (null pointer, n <= 0, non-finite or non-positive size) */
    MD_ERR_BOX = -2,        /* some box edge is shorter than 2 (rc + skin): minimum image not unique */
    MD_ERR_CAPACITY = -3,   /* neighbor list overflowed its per-atom capacity (see md_get_status) */
    MD_ERR_NONFINITE = -4,  /* a force or position became NaN/Inf on the device */
    MD_ERR_HIP = -5,        /* a HIP runtime call failed */
    MD_ERR_STATE = -6,      /* call out of order (e.g. forces before cells/list) */
    MD_ERR_TIMEOUT = -7     /* a task of the dependent schedule waited past its limit (see md_get_status) */
} md_status;

typedef enum { MD_FP64 = 0, MD_MIXED = 1 } md_precision;
/* MD_FP64: every operation in binary64.
 * MD_MIXED: displacement, squared distance and every cutoff test in binary64;
 *           pair arithmetic (potential, force magnitude, tables) in binary32;
 *           per-atom accumulation, integration and global sums in binary64. */

typedef enum { MD_LIST_FULL = 0, MD_LIST_HALF = 1, MD_LIST_WAVES = 2, MD_LIST_DEPS = 3 } md_list_kind;
/* MD_LIST_FULL: every pair is stored with both atoms; each atom's force is
 *               written only by the worker that owns the atom (no atomics).
 * MD_LIST_HALF: Newton-3 list, each pair once (Sec. II.D.3), held by the atom
 *               that comes first in the cell-sorted order; the partner's force
 *               is accumulated with binary64 atomics (order not deterministic).
 * MD_LIST_WAVES: the same half list, its brick tasks run in waves of tasks
 *               whose write sets (a brick and one cell around it) are disjoint
 *               (Sec. II.B and the appendix: index sets per axis, Cartesian
 *               products, inner loops not reset), one launch per wave.  A task
 *               sums partner forces in on-chip memory and adds them to the
 *               partners with plain stores: no global atomics while the halo
 *               fits the LDS stage.  LJ only; the order of the on-chip sums
 *               is not deterministic.
 * MD_LIST_DEPS: the same tasks in one persistent launch that runs them in
 *               dependence order instead of wave by wave (Sec. II.B): a task
 *               starts as soon as the last earlier task, in wave order, that
 *               writes each of its cells has finished (its direct
 *               predecessors, found by the backward method).  Workgroups take
 *               ready tasks from a device queue; finished tasks count their
 *               successors down.  Each wait for a ready task is bounded
 *               (md_set_tuning key 5); past the bound the launch ends early
 *               and md_get_status reports MD_ERR_TIMEOUT.  LJ only. */

typedef enum { MD_POT_LJ = 0, MD_POT_EAM = 1 } md_pot_kind;

/* Uniform-knot cubic table: on interval k (x in [x0 + k h, x0 + (k+1) h)),
 * f(x) = a0 + a1 t + a2 t^2 + a3 t^3 with u = (x - x0)/h, k = min(floor(u), n_knots-2),
 * t = u - k.  coef: DEVICE pointer to (n_knots - 1) x 4 doubles, row k = (a0..a3). */
typedef struct {
    int32_t n_knots;
    double x0;
    double h;
    const double *coef;
} md_spline;

/* Potential description.
 * LJ:  V(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] for r < rc, else 0 (unshifted);
 *      lj_params is a DEVICE pointer to {eps, sigma}.
 * EAM: E = sum_i F(rho_i) + sum_{i<j} phi(r_ij), rho_i = sum_{j!=i} rho(r_ij);
 *      phi is zero for r >= rc_phi, rho zero for r >= rc_rho; F beyond its last
 *      knot continues linearly.  rc must equal max(rc_phi, rc_rho). */
typedef struct {
    int32_t kind;             /* md_pot_kind */
    double rc;                /* interaction cutoff; must equal the rc given to md_build_cells */
    const double *lj_params;  /* LJ: device {eps, sigma} */
    md_spline phi, rho, embed;/* EAM tables */
    double rc_phi, rc_rho;    /* EAM cutoffs */
} md_potential;

typedef struct md_ctx md_ctx;

/* Create a context for n_atoms_total atoms in n_replicas replicas,
 * 1 <= n_atoms_total <= 2^26 (67,108,864: a list entry holds a 26-bit atom
 * index).  replica_offsets [host]: n_replicas + 1 int64, offsets[0] = 0,
 * offsets[n_replicas] = n_atoms_total, non-decreasing with every replica
 * non-empty.  Allocates the per-atom workspace on the current device.
 * Errors: MD_ERR_ARG (including n_atoms_total out of range), MD_ERR_HIP. */
int md_create(md_ctx **ctx, int64_t n_atoms_total, int32_t n_replicas,
              const int64_t *replica_offsets);

/* Free the context and all its workspace (synchronises the device). */
void md_destroy(md_ctx *ctx);

/* Linked cells (Sec. II.A).  pos: [3][N] user order (need not be wrapped).
 * boxes [host]: n_replicas x 3 edge lengths.  Positions are wrapped into
 * [0, L) (x - L floor(x/L); x >= L -> x - L; x < 0 -> 0), each replica gets
 * n_c = floor(L_d / (rc + skin)) cells per dimension (width >= rc + skin),
 * cell index x fastest, and the context's internal copy of the atoms is
 * sorted by (cell, user index).  The cell grid is re-planned only when a box,
 * rc or skin changes.  A non-finite position (here or at a rebuild inside
 * md_verlet_step) raises the device's non-finite flag (md_get_status) and the
 * atom is placed in cell i mod (its replica's cell count), where it has no
 * partners; results involving it are invalid.  Errors: MD_ERR_ARG (rc <= 0,
 * skin < 0, non-finite or non-positive L), MD_ERR_BOX (L_d < 2 (rc + skin)),
 * MD_ERR_HIP. */
int md_build_cells(md_ctx *ctx, const double *pos, const double *boxes_host, double rc,
                   double skin, void *stream);

/* Verlet lists from the cells (Sec. II.A): for each atom, the distinct cells
 * of its 3x3x3 neighbourhood are scanned and every other atom with
 * r2 < (rc + skin)^2 is kept, where d = minimum image of x_i - x_j
 * (d > L/2 -> d - L, d < -L/2 -> d + L) and r2 = (dx*dx + dy*dy) + dz*dz, all in
 * binary64 without contraction, so the pair set equals the exhaustive one
 * bit for bit.  The first call sizes the per-atom capacity (synchronises);
 * later calls regrow it if md_get_status reported an overflow.
 * Errors: MD_ERR_STATE (no cells), MD_ERR_HIP. */
int md_build_neighbor_list(md_ctx *ctx, int32_t list_kind, void *stream);

/* Forces at the current cells/list: the force calculation over the Verlet
 * lists, the per-cell work of Sec. II.A (pair potential, or the many-body
 * potential of Sec. II.C in two passes, density then force).  The list of
 * md_build_neighbor_list decides which pairs are candidates; the r < rc test
 * runs in binary64 on r2 formed with fused multiply-adds (and, in bricks
 * staged through their cell images, from the pre-shifted partner position),
 * so a pair whose r2 lies within a few roundings of rc^2 may be counted where
 * the exhaustive definition would not, or the other way round; every other
 * pair is decided exactly as there.  forces: [3][N] out, user order.
 * energy, virial: [n_replicas] out (DEVICE), per replica E and scalar virial
 * W = sum_{i<j} d_ij . f_ij; either may be NULL.  Sums are taken in a fixed
 * order (bitwise repeatable for the full list).
 * Errors: MD_ERR_ARG, MD_ERR_STATE (no list, or rc differs), MD_ERR_HIP. */
int md_compute_forces(md_ctx *ctx, const md_potential *pot, int32_t precision, double *forces,
                      double *energy, double *virial, void *stream);

/* md_compute_forces for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, but every scratch
 * buffer the call's kernels use -- sorted forces, block partials, the brick
 * queue, EAM densities and staged tables, per-atom energies of a
 * multi-replica context -- lies in one static device array of the library,
 * MD_NOALLOC_BYTES = 48 MiB per device (md_query key 16), held by every device
 * the library runs on until the process ends.  The call allocates nothing and
 * calls no allocating routine; the context, cells and list must already exist
 * (md_create, md_build_cells, md_build_neighbor_list with MD_LIST_FULL).
 * It needs 24 bytes per atom, 16 more for EAM, 16 more for energies of a
 * multi-replica context, and about 130 KiB besides (LJ up to about 2.0M atoms,
 * EAM up to about 1.2M); a larger system is rejected with MD_ERR_ARG before
 * anything is enqueued.  Every call on a device shares that device's array
 * (the queue counters it needs zeroed are cleared at the start of each call), so
 * calls that overlap in time on one device -- on different streams or from
 * different threads -- race and give wrong results; serialise them.
 * Errors: as md_compute_forces, plus MD_ERR_STATE (list kind other than full). */
int md_compute_forces_noalloc(md_ctx *ctx, const md_potential *pot, int32_t precision,
                              double *forces, double *energy, double *virial, void *stream);

/* n_steps of velocity Verlet (the per-particle integration loop of Sec. II.A):
 * cells and list are rebuilt from pos, forces F(x0) computed; then per step
 * v += dt/(2m) F; x += dt v; wrap; if max_i |minimage(x_i - x_i^ref)|^2 >
 * (skin/2)^2 rebuild cells and list (decided on the device, no host sync);
 * F <- F(x); v += dt/(2m) F.  pos, vel: [3][N] in/out; forces: [3][N] out
 * (forces at the final positions).  energy_hist: ceil(n_steps / hist_every)
 * x 3 doubles (E_pot, KE, W), summed over replicas, after steps hist_every,
 * 2 hist_every, ... and after the last step (row r: step min((r+1) hist_every,
 * n_steps)), or NULL; the steps in between skip the energy terms of the pair
 * loops.  hist_every >= 1 (ignored when energy_hist is NULL).  rebuilds: 1 int32 out
 * (DEVICE, number of rebuilds after the initial one) or NULL.  Uses the rc and
 * skin of the last md_build_cells.  If md_get_status then reports
 * MD_ERR_CAPACITY, the outputs are invalid: the context has grown its
 * capacity and the caller repeats the call from its saved inputs.
 * Errors: MD_ERR_ARG (n_steps < 1, dt or mass not finite/positive,
 * hist_every < 1), MD_ERR_STATE, MD_ERR_BOX, MD_ERR_HIP. */
int md_verlet_step(md_ctx *ctx, const md_potential *pot, int32_t precision, int32_t list_kind,
                   double *pos, double *vel, double *forces, double dt, double mass,
                   int32_t n_steps, double *energy_hist, int32_t hist_every,
                   int32_t *rebuilds, void *stream);

/* Adjoint (vector-Jacobian product) of (F, E) at positions pos with the
 * current cells/list (pos must lie within skin/2 of the positions the list was
 * built from; pos == NULL means exactly those positions).  Inputs: cotangent
 * u_forces [3][N] on the forces and v_energy [n_replicas] on the energies.
 * Outputs: g_pos [3][N] = d(sum_r v_r E_r + u.F)/dx = -v F - H u (user order),
 * g_params = d(...)/d(parameters) summed over replicas: LJ {d/deps, d/dsigma}
 * (2 doubles); EAM the three tables' shapes back to back, phi then rho then
 * embed ((n_knots-1) x 4 each).  Either output may be NULL.  Parameter
 * histograms use binary64 atomics (last-bit order not deterministic).
 * The adjoint always evaluates in binary64: precision is checked (MD_FP64 or
 * MD_MIXED) but both give the binary64 result, the derivative of the FP64
 * forces.  The adjoint is not in the paper; it differentiates the forces of
 * Sec. II.A/II.C through the same lists.
 * Errors: MD_ERR_ARG, MD_ERR_STATE, MD_ERR_HIP. */
int md_force_vjp(md_ctx *ctx, const md_potential *pot, int32_t precision, const double *pos,
                 const double *u_forces, const double *v_energy, double *g_pos,
                 double *g_params, void *stream);

/* Device status (synchronises the context's last stream).  device_flags
 * [host]: bit 0 list overflow, bit 1 non-finite force or position, bit 2 a dependent-
 * schedule wait past its limit; cleared after reading.
 * required_capacity [host]: per-atom list capacity now allocated or required.
 * Returns MD_ERR_CAPACITY / MD_ERR_NONFINITE / MD_ERR_TIMEOUT if the flag is
 * set, else MD_OK. */
int md_get_status(md_ctx *ctx, int32_t *device_flags, int64_t *required_capacity);

/* Export the current neighbor list as CSR over user indices (for checking).
 * start [host]: N+1 int64 out; nbr [host]: capacity ints out (unordered within
 * an atom); returns the number of entries (which may exceed capacity: then
 * nothing is written to nbr) or a negative md_status.  Synchronises. */
int64_t md_get_neighbor_list(md_ctx *ctx, int64_t *start, int32_t *nbr, int64_t capacity);

/* Export the cells (for checking) [host]: cell_start (n_cells_total + 1 int32),
 * order (N int32: user index of each sorted slot), n_cells_total (1 int64).
 * Pass NULL arrays to query n_cells_total only.  Synchronises. */
int md_get_cells(md_ctx *ctx, int32_t *cell_start, int32_t *order, int64_t *n_cells_total);

/* The wave schedule of the last MD_LIST_WAVES build (for checking) [host]:
 * colour (n_bricks int32 out, capacity entries available): the wave of each
 * brick, bricks numbered replica by replica, x fastest within a replica's brick
 * grid; n_bricks (1 int64 out, may be NULL).  Pass colour = NULL to query the
 * size.  Returns the number of waves (>= 1), or MD_ERR_STATE (no schedule),
 * MD_ERR_ARG (capacity too small). */
int md_get_waves(md_ctx *ctx, int32_t *colour, int64_t capacity, int64_t *n_bricks);

/* The task graph of the last MD_LIST_DEPS build (for checking) [host], tasks
 * numbered as the bricks of md_get_waves: succ_off (n_bricks + 1 int32 out,
 * may be NULL) and succ (capacity int32 out, may be NULL): the direct
 * successors of task t are succ[succ_off[t] .. succ_off[t+1]), ascending.
 * Returns the number of edges, or MD_ERR_STATE (no graph), MD_ERR_ARG
 * (capacity too small). */
int64_t md_get_task_graph(md_ctx *ctx, int32_t *succ_off, int32_t *succ, int64_t capacity);

/* Tuning knobs (used by the autotuner).  The kernels run one workgroup per
 * brick of bx x by x bz cells (the cell-task blocking of Sec. II.D.2).
 * key 0 = candidates staged in LDS per brick task (64..4096, a multiple of 64,
 *   within the device's LDS; by default the first list build picks one from
 *   the largest brick halo, and candidates beyond it are read from global
 *   memory); drops the current list;
 * key 1 = most workgroups per CU in the brick-task grids (1..8);
 * key 2 = fixed per-atom list capacity (1..4096, rounded up to a multiple of 8;
 *   reallocates, synchronises the device and drops the current list -- a small
 *   value forces the overflow path);
 * key 3 = brick shape bx | by << 8 | bz << 16 (1..8 cells per axis, at most 64
 *   cells, (bx+2)(by+2)(bz+2) <= 512), or 0 to choose it from the mean
 *   occupancy of the non-empty cells; drops the current list;
 * key 4 = threads per brick task (128..512, a multiple of 64), or 0 to choose
 *   them with the shape; drops the current list;
 * key 5 = longest wait of a dependent-schedule workgroup for a ready task, in
 *   microseconds (default 2,000,000; 0 ends a launch at the first wait, the
 *   way the failure path is tested);
 * key 6 = which atom of a pair holds it in the half lists (MD_LIST_HALF,
 *   MD_LIST_WAVES, MD_LIST_DEPS): 0 (default) the one that comes first in the
 *   cell-sorted order; 1 the half list over 14 of the 27 cells (Sec. II.D.3):
 *   the atom that sees the partner's cell, through the pair's minimum image,
 *   above its own in z, else above in y, else above in x, else (same cell)
 *   the one first in the sorted order.  Partners then lie in the atom's cell
 *   and the layer above, so a task writes a 3 x 3 x 2 block of cells per cell
 *   and the waves and task graphs use that stricter overlap.  The list is
 *   built full and filtered.  Drops the current list;
 * key 7 = how the force and adjoint kernels share the bricks among their
 *   workgroups: 1 static cost-balanced ranges; 2 a queue from which
 *   workgroups take one brick at a time (better where empty regions leave the
 *   static ranges uneven); 0 (default) the queue when more than 5 % of the
 *   cells were empty at the last brick plan, else the static ranges.  Forces
 *   do not depend on it; energy and virial sums may differ in the last bits;
 * key 8 = most intervals of each EAM table whose parameter gradient a
 *   workgroup of md_force_vjp sums in LDS before adding it to g_params: -1
 *   (default) as many as fit beside the stage (the last intervals of the phi
 *   and rho tables, where the pairs fall, and the embedding table when it
 *   fits whole); 0 none (every term a global atomic).  The gradient does not
 *   depend on it beyond the summation order;
 * key 9 = whether the adjoint kernels stage each candidate's cotangent (and,
 *   for EAM pass B, its F' and F'' rho-dot) in LDS beside its position: 1
 *   when that larger stage fits a workgroup's LDS without costing resident
 *   workgroups (LJ, EAM pass A) or LDS room of the parameter sums (EAM pass
 *   B), 0 (default) never: every pair gathers them from global memory, which
 *   measured as fast on the replica batches.  The result does not depend on it.
 * Returns MD_OK or MD_ERR_ARG. */
int md_set_tuning(md_ctx *ctx, int32_t key, int32_t value);

/* Current configuration [host out]: key 0 LDS stage of the force and adjoint
 * tasks (candidates; unless set with md_set_tuning, sized at the first list
 * build from the largest halo, and for LJ grown to the largest stage that
 * keeps as many workgroups resident per CU, so that halos that grow later stay
 * in LDS), 1 workgroups
 * per CU, 2 per-atom list capacity, 3 brick shape (bx | by << 8 | bz << 16 of
 * replica 0), 4 threads per brick task, 5 bricks in total, 6 largest brick halo
 * (candidates) and 7 largest brick (atoms) seen by the list builds since the
 * sizing pass (both synchronise), 8 LDS bytes a workgroup may use, 9 workgroups
 * of the LJ force grid, 10 entries of the current list (synchronises), 11
 * waves of the current wave schedule (0 if none), 12 edges of the current
 * task graph (0 if none), 13 the half-list rule (key 6), 14 the brick
 * schedule in use (1 static ranges, 2 queue), 15 entries of the current list
 * stored as 16-bit candidate indices (bricks on axes of at least 4 cells
 * whose whole halo fits the LDS stage; the others store 32-bit entries with
 * an image code; synchronises), 16 bytes of the static scratch array of
 * md_compute_forces_noalloc, 17 candidates the list build stages per brick
 * (at most key 0: its own static LDS is larger than the force tasks'; a halo
 * between the two is listed with its last candidates read from global memory
 * and still gets 16-bit entries).
 * Returns MD_OK, MD_ERR_ARG, MD_ERR_STATE (keys 10 and 15 without a list) or MD_ERR_HIP. */
int md_query(md_ctx *ctx, int32_t key, int64_t *value);

/* Kernel timing with HIP events on the stream of the timed calls.
 * enable = 1: clear the counters and, from the next call on, record an event
 * pair around every force launch (LJ kernel, or EAM density + force pair, or
 * half-list kernel + integration) and every neighbour-list launch, and one
 * event at each end of md_verlet_step's setup and step loop.
 * enable = 2: as 1, but only the setup and loop events (md_profile_detail's
 * [0..2]); the loop then runs without the per-launch event pairs, which cost
 * their stream a few microseconds per step.
 * enable = 0: stop, synchronise, and return [host] the summed durations and
 * launch counts (any pointer may be NULL).  List launches include those that
 * exit at once because no rebuild was due. */
int md_profile(md_ctx *ctx, int32_t enable, double *force_ms, int64_t *force_launches,
               double *list_ms, int64_t *list_launches);

/* Timings of the md_verlet_step calls made while md_profile was enabled, taken
 * when md_profile(ctx, 0, ...) stopped it (HIP events on the calls' stream).
 * Entries [3..7] are zero after md_profile(ctx, 2, ...).
 * out [host]: n_out (at most 8) doubles:
 *   [0] ms of the step loops (from the end of the setup to the last step's
 *       last launch: every rebuild test, list rebuild, force and integration
 *       launch of the steps), [1] steps in those loops,
 *   [2] ms of their setup (user order to sorted, cells, list, F(x0)),
 *   [3] ms of the force launches of steps that record no energies, [4] their
 *       number, [5] ms of the force launches of recorded steps, [6] their
 *       number, [7] ms of the setup's F(x0) launches.
 * Errors: MD_ERR_ARG. */
int md_profile_detail(md_ctx *ctx, double *out, int32_t n_out);

/* Human-readable description of the last error on this context (static storage). */
const char *md_last_error(md_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MD_H */
