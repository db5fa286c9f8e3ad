/*
 * afmm.h -- C ABI of the MI355X adaptive fast multipole Poisson solver.
 *
 * Problem (Lee & Teyssier, Sec. 1 and Sec. 3): cell masses on a graded AMR
 * octree in, gravitational potential and acceleration of every leaf cell out.
 * Level l has 2^l cells per dimension over the box [0, boxlen)^3 and cell
 * (i, j, k) has centre ((i, j, k) + 1/2) * boxlen / 2^l.  Only leaves carry
 * mass and only leaves are targets.  Isolated boundaries.
 *
 * Method: one FMM tree per AMR level and a merged tree over finer levels
 * (Sec. 3.1), upward pass by P2M and M2M (Sec. 2, Eqs. eqn:multipole and
 * eq:M2M_general), downward pass by M2L over the 189-cell interaction list and
 * L2L (Sec. 2, Eqs. eq:M2L and eq:L2L; Alg. 3), and at the leaves far (L2P),
 * intermediate (M2P/P2P), near (P2P/M2P) and nearest (coarse-fine P2P) fields
 * (Sec. 3.2, Alg. 4).  Adaptive time stepping follows Alg. 1 and Alg. 2.
 *
 * Conventions: g(R) = -G/|R| with R = target - source; phi = sum g m;
 * acceleration a = -grad phi.  Expansions are truncated at total order p
 * (|alpha| + |beta| <= p in Eq. eq:M2L).
 *
 * Errors: every entry point returns an afmm_status; nothing throws across the
 * ABI.  afmm_last_error() gives a thread-local message for the last failure.
 * A device (HIP) error makes the plan unusable (sticky AFMM_E_DEVICE).
 */
#ifndef AFMM_H
#define AFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t afmm_status;
#define AFMM_OK 0
#define AFMM_E_INVALID_ARG (-1)    /* null pointer, bad size, out-of-range coordinate, duplicate cell */
#define AFMM_E_NOT_GRADED (-2)     /* refinement breaks the graded-octree rule of Sec. 3.2 */
#define AFMM_E_INCOMPLETE_OCT (-3) /* a refined cell without its 8 children, or an orphan cell */
#define AFMM_E_UNSUPPORTED (-4)    /* p outside 1..8, unknown precision or flag, tap_split outside 0..21 */
#define AFMM_E_OUT_OF_MEMORY (-5)  /* device or host allocation failed, or max_device_bytes exceeded */
#define AFMM_E_DEVICE (-6)         /* HIP runtime error; sticky on the plan */
#define AFMM_E_ATS_ORDER (-7)      /* solve(l, icount) needs trees that were never built */
#define AFMM_E_NONFINITE (-8)      /* non-finite mass seen (only with AFMM_CHECK_INPUT) */

#define AFMM_FP64 0          /* every step in FP64 */
#define AFMM_FP32_MIXED 1    /* M2L, M2P, L2L, L2P and P2P in FP32; P2M, M2M, FMM levels
                                f <= fp64_levels and the per-cell output in FP64 */

#define AFMM_CHECK_INPUT 1u  /* before a solve, scan the leaf masses that it reads (every leaf slot
                                for a full solve; the leaf slots of levels >= l when solve(l, .)
                                rebuilds trees; none otherwise) for NaN/Inf; one host sync, no
                                allocation (the flag lives in the plan) */
#define AFMM_SERIAL 2u       /* every launch of a solve on the caller's stream (the default; wins
                                over AFMM_OVERLAP) */
#define AFMM_OVERLAP 4u      /* run the intermediate-field M2P on an internal second stream,
                                concurrently with the M2L/L2L chain on the caller's stream.
                                Results are identical either way; measured on MI355X the overlap
                                does not pay (both launches fill the GPU), so it is off by default */

#define AFMM_GRAPH 32u       /* replay solves from hipGraphs: the launches of one afmm_solve are
                                captured (on an internal stream, on first use) once per distinct
                                (level, rebuild or not, trees kept or not, d_mass, d_phi, d_acc)
                                and replayed as one graph launch on the caller's stream; results
                                are identical to eager solves.  Up to 32 graphs are cached per plan
                                (least recently used evicted); the autotuner drops them.  Profiled
                                solves run eagerly.  Callers that change I/O buffers every call get
                                a capture per call: keep the buffers, update them in place. */
#define AFMM_PAPER_QUAD_CAP 8u
                             /* the paper's expansion setting (Sec. 2: local expansions to order p,
                                multipoles only up to the quadrupole at p = 3): every multipole that
                                enters M2L, M2P or the near-field M2P is truncated at order p - 1.
                                Accelerations only use multipoles of order <= p - 1 (the gradient
                                lowers the admissible order by one), so they are unchanged bit for
                                bit; potentials lose the order-p terms. */
#define AFMM_SELF_POTENTIAL 16u
                             /* add each leaf's own contribution to its potential, the potential at
                                the centre of a uniform cube of the leaf's mass m and side h:
                                phi_self = -G m C / h, C = integral of 1/|r| over the unit cube
                                centred at the origin (about 2.38, computed numerically by the
                                library).  The pair sums exclude the self pair (1/r is singular);
                                the acceleration of a uniform cube at its centre is zero, so only
                                the potential changes. */

#define AFMM_PERIODIC 64u    /* periodic box (an extension: the paper's Sec. 5 names periodic domains as
                                future work): the box is a torus and phi the potential of the masses
                                with a uniform neutralising background, zero on average over the box
                                (the Ewald sum).  Neighbour lists wrap around the box; the images
                                beyond the 3^3 block of boxes and the block's level-1 interaction
                                list enter the 64 level-2 cells through one Ewald-summed operator.
                                Needs levelmin >= 3 and a hierarchy graded on the torus (the
                                grading rule with wrapped neighbours), else AFMM_E_UNSUPPORTED /
                                AFMM_E_NOT_GRADED.  Full and ATS solves, drifted solves, re-planning,
                                graph replay, the adjoint and batches (of periodic plans only) work
                                as for isolated boxes.  The first plan of each order p computes the
                                operator table on the host (about a second at p = 6). */

#define AFMM_ALL_LEVELS (-1) /* synchronous solve: all trees rebuilt, every leaf evaluated */

typedef struct afmm_options {
  int32_t p;                 /* expansion order, 1..8 (the paper's own setting is p = 3) */
  int32_t precision;         /* AFMM_FP64 or AFMM_FP32_MIXED */
  double G;                  /* gravitational constant */
  double boxlen;             /* box side */
  uint32_t flags;            /* AFMM_CHECK_INPUT | AFMM_SERIAL | AFMM_OVERLAP | AFMM_GRAPH |
                                AFMM_PAPER_QUAD_CAP | AFMM_SELF_POTENTIAL | AFMM_PERIODIC */
  int32_t fp64_levels;       /* mixed form: FMM levels <= this stay FP64 (default 3) */
  int32_t tap_split;         /* M2L and M2P blocks per tile: the 189 source offsets of a tile are
                                split over this many blocks and their partial sums reduced in a
                                fixed order; 0 = automatic (enough blocks to fill the GPU), else
                                1..21.  Results depend on it only through FP rounding order. */
  size_t max_device_bytes;   /* cap on the plan's device memory; 0 = no cap */
  int32_t m2p_shape;         /* tile shape of the intermediate-field (M2P) launch: 0 = one
                                16-group tile per wave with each lane loading its own B
                                fragments (default), 1 = the same tile with the source rows
                                loaded row by row and staged through LDS, 2 = as 1 with two
                                16-group tiles of one parity class per wave (p <= 5), 3 = as 0
                                with the source rows loaded row by row and each lane's
                                fragments taken from other lanes over the cross-lane crossbar
                                (no LDS staging).  FP64 launches run shapes 0 and 3 (3 up to p = 7); a shape
                                the order or precision does not support falls back to 0.  The
                                autotuner chooses it by timing.  Results do not depend on it:
                                every shape runs the same products in the same order. */
} afmm_options;

/* Defaults: p = 4, FP64, G = 1, boxlen = 1, no flags, fp64_levels = 3, tap_split = 0 (automatic),
   no cap. */
void afmm_options_default(afmm_options* opt);

/*
 * An AMR hierarchy, host memory, read only during plan creation (the caller
 * keeps ownership).  Flat level-major arrays over all cells of levels
 * levelmin..levelmax; the caller's order inside each level is arbitrary and
 * is kept for the mass/phi/acc slots.
 *   ncell[l - levelmin]   number of cells at level l; ncell[0] must be 8^levelmin
 *   ijk[3 * i + d]        integer coordinate d of cell i, in [0, 2^l)
 *   refined[i]            1 if the cell's 8 children are present at level l + 1
 * Requirements: 1 <= levelmin <= levelmax <= 20; complete octs; the strong
 * grading rule (a refined level-l cell needs the 27 level-(l-1) neighbours of
 * its father refined, clipped to the box); fewer than 2^31 cells in total.
 */
typedef struct afmm_hierarchy {
  int32_t levelmin;
  int32_t levelmax;
  const int64_t* ncell;
  const int32_t* ijk;
  const uint8_t* refined;
} afmm_hierarchy;

typedef struct afmm_plan afmm_plan;
typedef struct afmm_batch afmm_batch;

/* Counts and algorithmic work of one synchronous solve (AFMM_ALL_LEVELS). */
typedef struct afmm_plan_info {
  int32_t levelmin, levelmax, p, K, precision, nhier;
  int64_t ncell, nleaves, nrefined;
  int64_t leaves_per_level[21];     /* indexed by absolute level */
  int64_t m2l_targets;              /* FMM cells that receive a local expansion */
  int64_t m2l_pairs;                /* (target cell, source cell) M2L pairs */
  int64_t m2p_pairs;                /* intermediate-field M2P pairs (refined sources) */
  int64_t p2p_pairs;                /* leaf-leaf pairs: intermediate, near and nearest */
  int64_t near_m2p_pairs;           /* near-field M2P pairs from refined level-l cells */
  int64_t nearest_pairs;            /* of p2p_pairs, those from the nearest field */
  double flops_m2l, flops_m2p, flops_p2p, flops_updown; /* algorithmic (useful) flops */
  double bytes_min;                 /* algorithmic HBM bytes of one solve */
  size_t device_bytes;              /* device memory held by the plan */
} afmm_plan_info;

/*
 * Build a plan: validate the hierarchy, order cells along a Morton curve per
 * level, build neighbour tables and group lists (the merged topology that all
 * per-level trees share, Sec. 3.1), translation tables, and allocate device
 * memory.  hip_stream (hipStream_t, may be NULL) orders the uploads.
 * Returns AFMM_E_INVALID_ARG / NOT_GRADED / INCOMPLETE_OCT for bad input.
 */
afmm_status afmm_plan_create(const afmm_hierarchy* h, const afmm_options* opt, void* hip_stream,
                             afmm_plan** out);
/*
 * Destroying a plan (or a batch) waits for its device, then keeps its device
 * buffers for later plans on that device, up to 2 GiB per device (the oldest
 * are freed first); plans created with max_device_bytes free theirs.
 * afmm_release_cached_memory frees every kept buffer; the library also does so
 * by itself before it reports an allocation failure.  Call it before a device
 * reset (hipDeviceReset), which would leave the kept buffers dangling.
 * Thread-safe.
 */
afmm_status afmm_plan_destroy(afmm_plan* plan);
afmm_status afmm_release_cached_memory(void);
/* The counts are taken on the first call (or when profiling is switched on),
 * not by afmm_plan_create: host time of the order of the topology build. */
afmm_status afmm_plan_get_info(const afmm_plan* plan, afmm_plan_info* out);

/*
 * Re-plan between adaptive time steps (Sec. 3.2, Alg. 1): the AMR of levels
 * >= level has changed since `old` was built, the levels below it have not.
 * Builds a plan for `h` with the options of `old` (which the caller keeps and
 * may destroy afterwards) and hands over the tree state of the stale levels:
 * the leaf masses of levels < level that the last rebuild of `old` took stay
 * those of the new plan's trees, while the trees of levels >= level are new
 * and take their masses from d_mass at the next afmm_solve, whatever that
 * call's level and icount (it then counts as a rebuild of levels >= min(its
 * own level, `level`), for the input check and the adjoint alike).  If `old`
 * holds no tree snapshot yet, the new plan holds none either.
 *   level       in [levelmin + 1, levelmax(h) + 1]
 * Requirements: same levelmin; levels below `level` identical in `h` and in the
 * hierarchy of `old` (same cells, same caller order, same refined flags).
 * Synchronous on hip_stream (the snapshot copy).  Errors: AFMM_E_INVALID_ARG
 * (null pointer, a level out of range, differing coarse levels, a batched
 * plan), AFMM_E_DEVICE (a dead `old`), and the errors of afmm_plan_create.
 */
afmm_status afmm_plan_replan(const afmm_plan* old, const afmm_hierarchy* h, int32_t level, void* hip_stream,
                             afmm_plan** out);

/*
 * Solve (Alg. 1).  d_mass, d_phi, d_acc are device pointers, FP64, one slot per
 * cell in the hierarchy's flat order (d_acc is [ncell][3]).  Masses of refined
 * cells are ignored.  Only leaves of the solved level(s) are written; other
 * entries are left untouched.  Stream-ordered and asynchronous (no host sync
 * unless AFMM_CHECK_INPUT).
 *   level == AFMM_ALL_LEVELS: synchronous solve, every tree rebuilt from d_mass.
 *   level == l, icount >= 1:  Alg. 1 Solve(l, icount): trees j >= l are rebuilt
 *                             from d_mass iff l == levelmin or icount > 1; stale
 *                             trees keep their multipoles and leaf masses; only
 *                             level-l leaves are written, and only the local
 *                             expansions of their ancestors are computed (Alg. 2).
 *                             A solve that rebuilds no tree reuses the device
 *                             multipoles of the previous solve.  Returns
 *                             AFMM_E_ATS_ORDER if no tree snapshot exists yet,
 *                             AFMM_E_INVALID_ARG for icount < 1 or a level
 *                             outside [levelmin, levelmax].
 * Plans are not thread-safe; one plan per stream.
 */
afmm_status afmm_solve(afmm_plan* plan, int32_t level, int32_t icount, const double* d_mass,
                       double* d_phi, double* d_acc, void* hip_stream);

/*
 * Adaptive time step with drifted stale trees.  During a sub-cycle of Alg. 1
 * the trees of the inactive coarser levels keep the masses of their last
 * rebuild, an error of first order in the time since then (Sec. 4 discussion of
 * the binary orbit under adaptive time steps: the inactive multipoles are not
 * drifted).  This call is afmm_solve plus a first-order drift of those trees:
 *   - the trees it rebuilds (as afmm_solve decides) record `time` and the mass
 *     rate d_mass_rate (dm/dt, FP64, one slot per cell in the order of d_mass,
 *     device memory; read for the levels rebuilt) of their leaves;
 *   - every stale tree whose last rebuild recorded rates is evaluated with its
 *     masses advanced linearly to `time`: m + (time - t_rebuild) dm/dt.  Trees
 *     last rebuilt by afmm_solve (no rates) stay as they were.
 * A mass field that changes linearly in time is therefore solved exactly at
 * every sub-step.  Costs a pass over all slots and the whole upward pass at
 * every call (stale multipoles change with time, so no call reuses the
 * previous trees) plus 16 bytes per cell of device memory, allocated by the
 * first call; the call runs eagerly (AFMM_GRAPH does not capture it).  With
 * level == AFMM_ALL_LEVELS every tree is rebuilt at `time` with its rates.
 * The adjoint of a drifted solve is that of afmm_solve (the drifted stale
 * masses are not an input).  Errors as afmm_solve, plus AFMM_E_INVALID_ARG for
 * a null d_mass_rate or a non-finite time; with AFMM_CHECK_INPUT the rates of
 * the leaves the call reads are checked as the masses are.
 */
afmm_status afmm_solve_drift(afmm_plan* plan, int32_t level, int32_t icount, double time,
                             const double* d_mass, const double* d_mass_rate, double* d_phi, double* d_acc,
                             void* hip_stream);

/*
 * Adjoint of the last solve's linear map m -> (phi, a): d_mass_bar = A^T
 * (d_phi_bar, d_acc_bar) over the same trees and lists (transposed kernels,
 * gather form, no atomics).  Inputs are indexed like d_phi / d_acc and only
 * their leaf entries of the solved level(s) are read; every leaf of d_mass_bar
 * is written (refined entries are set to 0).  After an adaptive-time-step
 * solve(l, .), entries of levels whose trees were stale are 0: their snapshot
 * masses are not an input of that solve.
 */
afmm_status afmm_solve_adjoint(afmm_plan* plan, int32_t level, const double* d_phi_bar,
                               const double* d_acc_bar, double* d_mass_bar, void* hip_stream);

/*
 * Allocation-free adjoint, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc (afmm_solve_adjoint allocates its workspace on its first call).
 * Same arguments, semantics and results as afmm_solve_adjoint, bit for bit,
 * but the call allocates nothing: its scratch (target and mass bars, the
 * multipole and local-expansion bars, the B staging of the transposed M2P and
 * M2L, their tap-split partial sums) lives in one static device array of the
 * library, 64 MiB per GPU, which each GPU the library runs on holds until the
 * process ends.  The adjoint's topology (its source tiles) is built at plan
 * creation for every plan whose scratch fits that bound; a plan whose scratch
 * exceeds it is refused with AFMM_E_OUT_OF_MEMORY before anything runs (about
 * 10^5 cells at p = 6 fit).  Every call on one GPU shares the array: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller; calls on one stream are ordered.  Each call writes
 * every scratch byte it reads, so no call depends on what an earlier one left.
 * Errors as afmm_solve_adjoint, plus AFMM_E_OUT_OF_MEMORY for oversized plans.
 */
afmm_status afmm_solve_adjoint_noalloc(afmm_plan* plan, int32_t level, const double* d_phi_bar,
                                       const double* d_acc_bar, double* d_mass_bar, void* hip_stream);

/*
 * Batch of independent hierarchies of uneven size and depth, solved together
 * (synchronous solves, Alg. 1 with every tree rebuilt).  The batch is one plan
 * over the forest of all hierarchies: level l of the forest is the union of the
 * level-l cells of every hierarchy (Morton order inside each), so every kernel
 * of a solve runs once over all hierarchies.  The whole solve -- mass gather
 * from the n caller arrays, upward pass, M2L/L2L chain, leaf fields and the
 * scatter of the results -- is captured once into a hipGraph at creation and
 * replayed by afmm_batch_solve as one graph launch.
 *   plans[i]       plans built by afmm_plan_create (one hierarchy each); all must
 *                  share p, precision, G, boxlen, fp64_levels, tap_split and the
 *                  AFMM_PAPER_QUAD_CAP / AFMM_SELF_POTENTIAL flags (the batch solves
 *                  with them; the scheduling flags of the members are ignored, the M2P
 *                  tile shape is that of plans[0]).  The
 *                  batch copies their topology: they may be destroyed afterwards.
 *   hip_stream     orders the uploads and the graph capture.
 * afmm_batch_solve: d_mass[i], d_phi[i], d_acc[i] are device pointers laid out as
 * for afmm_solve on plans[i] (host arrays of n pointers, read at the call).  Only
 * leaf entries of the outputs are written.  A solve of the batch gives the same
 * bits as afmm_solve on each plan (same tap_split, no atomics anywhere).
 * Errors: AFMM_E_INVALID_ARG (null pointer, n < 1, an options mismatch),
 * AFMM_E_DEVICE (capture or launch failure), AFMM_E_OUT_OF_MEMORY.
 */
afmm_status afmm_batch_create(afmm_plan* const* plans, int32_t n, void* hip_stream, afmm_batch** out);
afmm_status afmm_batch_solve(afmm_batch* batch, const double* const* d_mass, double* const* d_phi,
                             double* const* d_acc, void* hip_stream);
afmm_status afmm_batch_get_info(const afmm_batch* batch, afmm_plan_info* out);
afmm_status afmm_batch_destroy(afmm_batch* batch);

/*
 * Host-only validation (no device memory touched): fills counts of `out`
 * (ncell, leaves, refined, pair counts, flops) or returns the error a plan
 * creation would return.
 */
afmm_status afmm_hierarchy_check(const afmm_hierarchy* h, const afmm_options* opt,
                                 afmm_plan_info* out);

/*
 * Per-launch timing (instrumentation, no effect on results).  While enabled,
 * every kernel launch of a solve is bracketed by hipEvents recorded on the
 * solve's stream, and the solve runs serially (as with AFMM_SERIAL) so that
 * each interval times one launch alone.  afmm_plan_get_profile synchronises on those events, sums
 * them per kernel family and resets the records; `out` receives up to `cap`
 * families and *n_out their number.  flops/bytes are the algorithmic work of
 * the timed launches (useful terms only, as in afmm_plan_info).
 */
typedef struct afmm_stage_time {
  char name[24];      /* "gather", "upward", "m2l_f64", "m2l_f32", "leaf_f64", "leaf_f32" */
  int32_t launches;
  double ms;          /* summed event time */
  double flops;       /* summed algorithmic flops */
  double bytes;       /* summed algorithmic HBM bytes */
} afmm_stage_time;
afmm_status afmm_plan_set_profiling(afmm_plan* plan, int32_t enable);
afmm_status afmm_plan_get_profile(afmm_plan* plan, afmm_stage_time* out, int32_t cap, int32_t* n_out);
/* The same for a batch.  While profiling is enabled, afmm_batch_solve runs the
   captured launches eagerly (not as a graph) so that each can be timed. */
afmm_status afmm_batch_set_profiling(afmm_batch* batch, int32_t enable);
afmm_status afmm_batch_get_profile(afmm_batch* batch, afmm_stage_time* out, int32_t cap, int32_t* n_out);

/*
 * Autotuner of the work granularity.  The tap split of M2L and of M2P (how
 * many blocks share the 189 source offsets of one tile, see tap_split) trades
 * parallelism against partial-sum traffic and per-block setup; the best value
 * depends on the hierarchy's shape.  afmm_plan_autotune times candidate splits
 * (per-launch events, serial launches; each candidate's time is the minimum
 * over 5 full solves of the caller's data after one warm-up) and keeps, per
 * precision, the fastest M2L split and the fastest M2P (tile shape, split)
 * pair (the shapes of afmm_options.m2p_shape that the order and precision
 * support); it leaves phi/acc holding a full solve and counts as one
 * (AFMM_ALL_LEVELS).
 * afmm_batch_autotune does the same on a batch and re-captures its graph.
 * Results of later solves change only through FP rounding order.  Takes a few
 * dozen solves; no host-visible allocation beyond the partial-sum buffers.
 */
typedef struct afmm_tune_result {
  int32_t m2l_split[2];   /* chosen splits, [0] FP64 kernels, [1] FP32 kernels */
  int32_t m2p_split[2];
  double ms_before;       /* summed launch time of one solve before / after */
  double ms_after;
  int32_t candidates;     /* candidate configurations timed */
  int32_t m2p_shape[2];   /* chosen M2P tile shapes (see afmm_options.m2p_shape) */
} afmm_tune_result;
afmm_status afmm_plan_autotune(afmm_plan* plan, const double* d_mass, double* d_phi, double* d_acc,
                               void* hip_stream, afmm_tune_result* out);
afmm_status afmm_batch_autotune(afmm_batch* batch, const double* const* d_mass, double* const* d_phi,
                                double* const* d_acc, void* hip_stream, afmm_tune_result* out);

/*
 * Particle-mesh coupling for time loops.  The paper's solver works on cell
 * masses obtained by depositing particle masses onto the AMR cells with a
 * cloud-in-cell scheme (Sec. 1), and its binary-orbit test (Sec. 4, Fig.
 * fig:binary) advances two point masses with a fixed-step leapfrog on a grid
 * refined around them.  These calls provide the pieces of such a loop.
 *
 * afmm_particle_hierarchy_create: host only.  A graded hierarchy over levels
 * levelmin..levelmax (levelmin complete): at every level l < levelmax each
 * cell within `nexpand` cells (Chebyshev distance, clipped to the box) of the
 * 2x2x2 cloud of a particle at level l is refined, then the strong grading
 * rule (Sec. 3.2) is closed; levelmax of the result is the deepest level that
 * has cells.  Cells come level by level, each level in Morton order (bit b
 * of i, j, k at key bits 3b, 3b + 1, 3b + 2), the order a plan keeps its
 * levels in.  pos: host [np][3], inside [0, boxlen).  The result is owned by
 * the library: afmm_particle_hierarchy_view fills an afmm_hierarchy that
 * points into it (valid until afmm_particle_hierarchy_destroy).
 */
typedef struct afmm_particle_hierarchy afmm_particle_hierarchy;
afmm_status afmm_particle_hierarchy_create(int32_t levelmin, int32_t levelmax, int32_t nexpand, int64_t np,
                                           const double* pos, double boxlen, afmm_particle_hierarchy** out);
afmm_status afmm_particle_hierarchy_view(const afmm_particle_hierarchy* h, afmm_hierarchy* out);
afmm_status afmm_particle_hierarchy_destroy(afmm_particle_hierarchy* h);

/*
 * afmm_cic_deposit: cell masses from particle masses by cloud-in-cell at one
 * level: particle p (device d_pos[np][3], d_pmass[np]) gives the 8 cells of
 * that level around it (centres within one cell size) the weights
 * prod_d (1 - |x_d / h - 1/2 - c_d|).  d_cell_mass (device, one slot per cell
 * of the plan's hierarchy, as for afmm_solve) is cleared first, then
 * accumulated with atomic additions (the rounding of a sum depends on the
 * order in which particles land).  Every cloud cell must be a leaf of `level`:
 * otherwise (or if a cloud leaves the box) AFMM_E_INVALID_ARG after the call.
 * One host sync.  The plan builds a key table of the level on first use
 * (8 bytes per cell of the level, counted in its device memory).
 * afmm_cic_interpolate: the inverse map with the same weights: d_acc[np][3] =
 * sum of the cloud cells' d_cell_acc (and d_phi[np] of d_cell_phi when both
 * are non-null); same requirements.  With deposition and interpolation at one
 * level and the solver's antisymmetric near-field pairs, a particle exerts no
 * force on itself.
 * afmm_particles_update: d_state[i] += dt * d_rate[i] for i < n3 (the leapfrog
 * kick v += dt a and drift x += dt v on [np][3] arrays, n3 = 3 np).
 */
afmm_status afmm_cic_deposit(afmm_plan* plan, int32_t level, int64_t np, const double* d_pos, const double* d_pmass,
                             double* d_cell_mass, void* hip_stream);
afmm_status afmm_cic_interpolate(afmm_plan* plan, int32_t level, int64_t np, const double* d_pos,
                                 const double* d_cell_acc, const double* d_cell_phi, double* d_acc, double* d_phi,
                                 void* hip_stream);
afmm_status afmm_particles_update(int64_t n3, double dt, const double* d_rate, double* d_state, void* hip_stream);

const char* afmm_status_string(afmm_status s);
const char* afmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AFMM_H */
