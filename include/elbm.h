/*
 * elbm.h -- C ABI of the MI355X grid-refined entropic lattice Boltzmann library.
 *
 * Method: Dorschner, Frapolli, Chikatamarla, Karlin, "Grid refinement for entropic
 * lattice Boltzmann models" (arXiv:1608.06915).  Per level, the KBC stream-collide of
 * Sec. II.A (Eq. f_equations with the mirror state Eq. f_mirr, the product-form
 * equilibrium Eq. feq_iso and the entropic stabiliser Eq. gamma_min_approx); between
 * levels, the multi-domain coupling of Sec. III (non-equilibrium rescaling
 * Eq. f_neq_rescaling_iso at twin nodes, four-point reconstruction Eq. interp at
 * hanging nodes) and the five-step algorithm of Sec. III.C with two fine substeps per
 * coarse step and no time interpolation, applied recursively over any number of
 * levels with refinement ratio r = 2.
 *
 * Conventions
 *   - Status: every call returns elbm_status; no exception or exit crosses the ABI.
 *     On failure elbm_last_error(ctx) holds a message.
 *   - Lattices: D2Q9 (dim 2) and D3Q27 (dim 3).  Velocity index
 *     i = (cx+1) + 3(cy+1) [+ 9(cz+1)]; the opposite of i is Q-1-i.
 *   - Units: lattice units of level 0 (the coarsest) at the boundary.  Level l has
 *     spacing and time step 2^-l of level 0; its viscosity is 2^l nu0 (convective
 *     scaling, Sec. III.A); body forces are force densities in level-0 units.
 *   - Coordinates: level-l node coordinates are integers in level-l spacing.  A
 *     periodic axis with N coarse nodes has period N 2^l at level l; a non-periodic
 *     axis has nodes 0 .. (N-1) 2^l and its faces carry walls (default), an inlet or an
 *     outflow.  Walls sit half a spacing of the level that resolves them outside
 *     the last node (halfway bounce-back).
 *   - Level index box: level 0 covers the domain; level l > 0 covers, per axis, the
 *     hull of its blocks, or the whole period when a block spans or wraps it.  Dense
 *     per-level arrays (fields, masks) cover that box, x fastest; vector fields are
 *     [component][box]; population arrays are [Q][box].
 *   - Memory: "_host" pointers are host memory, "_dev" pointers device memory.  The
 *     caller owns both; the library keeps no caller pointer after a call returns,
 *     except the bound workspace and stream.
 *   - Threading: one context per stream; a context is not thread-safe.
 */
#ifndef ELBM_H
#define ELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ELBM_OK = 0,
  ELBM_EINVAL = 1,    /* bad argument or geometry (not nested, misaligned, missing margin) */
  ELBM_ESTATE = 2,    /* call out of order (e.g. advance before bind) */
  ELBM_ESMALL = 3,    /* workspace smaller than elbm_finalize reported */
  ELBM_EDEVICE = 4,   /* HIP runtime error; message in elbm_last_error */
  ELBM_EUNSTABLE = 5, /* a node is non-finite, has rho <= 0 or |u_a| >= 1 */
  ELBM_ENOMEM = 6     /* host allocation failed */
} elbm_status;

typedef enum {
  ELBM_STORE_F64 = 0,  /* FP64 populations, FP64 arithmetic */
  ELBM_STORE_F32 = 1,  /* FP32 populations, FP32 arithmetic */
  ELBM_STORE_F16S = 2, /* FP16 of f_i - W_i (round to nearest even), FP32 arithmetic */
  ELBM_STORE_BF16S = 3 /* BF16 of f_i - W_i (round to nearest even), FP32 arithmetic */
} elbm_storage;

typedef enum { ELBM_FACE_WALL = 1, ELBM_FACE_INLET = 2, ELBM_FACE_OUTFLOW = 3 } elbm_face_kind;

typedef struct elbm_ctx elbm_ctx;

typedef struct {
  int32_t dim;         /* 2 or 3 */
  int32_t storage;     /* elbm_storage */
  int64_t extent[3];   /* coarse nodes per axis (unused axes: 1) */
  int32_t periodic[3]; /* nonzero: periodic axis */
  double nu0;          /* kinematic viscosity of level 0, lattice units (Eq. visc) */
  int32_t n_levels;    /* 1 .. 8; refinement ratio 2 between consecutive levels */
} elbm_desc;

/* Create a lattice (Sec. II.A, Sec. III.A for the level parameters). */
elbm_status elbm_create(const elbm_desc *desc, elbm_ctx **out);
/* Release host state and graphs; the caller's workspace is not freed. */
elbm_status elbm_destroy(elbm_ctx *ctx);
const char *elbm_status_string(elbm_status s);
const char *elbm_last_error(const elbm_ctx *ctx);

/* Boundary kind of a non-periodic face (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z).  u: inlet
 * velocity (level-invariant); incoming populations at inlet nodes are set to the
 * equilibrium at (rho=1, u); an outflow copies incoming populations from one node
 * upstream.  Before elbm_finalize. */
elbm_status elbm_set_face(elbm_ctx *ctx, int face, int kind, const double u[3]);

/* Add a refinement block to level 1..L-1: the closed node box [lo, hi] in level
 * coordinates.  The level's region is the union of its blocks (Sec. III: the
 * overlapping region where both grids are present).  Faces that are not on a wall
 * or spanning a periodic axis are interfaces and must lie on parent nodes (even
 * coordinates).  A block spanning a periodic axis uses lo = 0, hi = period-1.
 * Before elbm_finalize. */
elbm_status elbm_add_block(elbm_ctx *ctx, int level, const int64_t lo[3], const int64_t hi[3]);

/* Mark solid nodes of a level from a host uint8 mask over the box [lo, lo+n).
 * Solid nodes reflect populations (halfway bounce-back); momentum exchanged with
 * them is accumulated as drag.  Before elbm_finalize. */
elbm_status elbm_set_solid(elbm_ctx *ctx, int level, const int64_t lo[3], const int64_t n[3],
                           const uint8_t *mask_host);

/* Uniform body-force density F (level-0 units), applied by the exact-difference
 * method of Sec. III.A with du = F_l / rho and F_l = F / 2^l. */
elbm_status elbm_set_force_uniform(elbm_ctx *ctx, const double F[3]);

/* Validate the geometry (nesting, alignment, margins, boundary combinations) and
 * build the node classes, interface lists and tick schedule on the host.  Returns
 * the device workspace size the caller must provide to elbm_bind. */
elbm_status elbm_finalize(elbm_ctx *ctx, size_t *workspace_bytes);

elbm_status elbm_level_box(const elbm_ctx *ctx, int level, int64_t lo[3], int64_t n[3]);
/* Node counts: n_nodes (stored nodes incl. solid), n_fluid (nodes that collide every
 * level step, interface layers included), relaxation parameter beta_l (Eq. visc),
 * number of bricks. */
elbm_status elbm_level_info(const elbm_ctx *ctx, int level, int64_t *n_nodes, int64_t *n_fluid, double *beta,
                            int64_t *n_bricks);
/* Node classes over the level index box (int32): -1 absent, else bit0 solid, bit1
 * parent ring (coalesced from the child), bits 2-3 distance to the own parent
 * interface (0 outer layer, 1 inner layer, 3 bulk or level 0). */
elbm_status elbm_node_class(const elbm_ctx *ctx, int level, int32_t *out_host);
/* Owned-volume weights (level-0 volume units) over the level index box. */
elbm_status elbm_weights(const elbm_ctx *ctx, int level, double *out_host);

/* Bind the caller-owned device workspace (>= elbm_finalize bytes, 256-byte aligned)
 * and HIP stream (hipStream_t; NULL = default stream).  Uploads tables. */
elbm_status elbm_bind(elbm_ctx *ctx, void *workspace_dev, size_t bytes, void *hip_stream);

/* Initial state of a level: f_i = f_i^eq(rho, u) (1 + noise_i) at every fluid node
 * (Eq. feq_iso), from host arrays over the level index box (rho, u [D][box],
 * noise [Q][box] or NULL).  Synchronous. */
elbm_status elbm_init_fields(elbm_ctx *ctx, int level, const double *rho_host, const double *u_host,
                             const double *noise_host);

/* For callers that cannot allocate device memory (code running under a HIP graph
 * capture of its own, tight serving loops, harnesses that forbid hipMalloc):
 * elbm_init_fields with the host arrays staged through a static device buffer of
 * 32 MiB instead of memory allocated per call, the same initial state bit for bit.
 * Each GPU the library runs on holds one such buffer from the first elbm_bind on it
 * until the process ends; every call on that GPU shares it, so calls that overlap on
 * one GPU (other threads or contexts) race.  The level needs n (1 + D + Q) 8 bytes of
 * staging (n = nodes of the level index box; without noise n (1 + D) 8): ELBM_EINVAL
 * beyond 32 MiB, nothing written.  Synchronous. */
elbm_status elbm_init_fields_static(elbm_ctx *ctx, int level, const double *rho_host, const double *u_host,
                                    const double *noise_host);

/* Per-node body-force density field of a level (device, [D][box], level-0 units),
 * added to the uniform force; NULL removes it.  Asynchronous on the bound stream. */
elbm_status elbm_set_force_field(elbm_ctx *ctx, int level, const double *F_dev);

/* Advance n coarse steps (Sec. III.C): each is 2^(L-1) finest ticks, captured as one
 * HIP graph unless graphs are disabled.  Asynchronous on the bound stream. */
elbm_status elbm_advance(elbm_ctx *ctx, int n_coarse_steps);

/* Macroscopic fields from the stored post-collision state: rho = sum f,
 * u = sum c f / rho - du/2 (the mid-step velocity of the forcing scheme), gamma of the
 * last collision (needs elbm_set_gamma_output).  Device arrays over the level box;
 * absent and solid nodes are NaN.  Any pointer may be NULL.  Asynchronous. */
elbm_status elbm_read_moments(elbm_ctx *ctx, int level, double *rho_dev, double *u_dev, double *gamma_dev);
/* Post-collision populations f_i, device [Q][box], NaN at absent/solid nodes. */
elbm_status elbm_read_populations(elbm_ctx *ctx, int level, double *f_dev);
/* Populations at n level coordinates (host int64 [n][3]) into host double [n][Q];
 * NaN where no fluid node exists.  Synchronous. */
elbm_status elbm_sample_populations(elbm_ctx *ctx, int level, int64_t n, const int64_t *coords_host,
                                    double *out_host);

/* Mass and momentum over owned volumes (FP64 deterministic reduction) and the count
 * of unstable nodes.  Synchronous. */
elbm_status elbm_reduce(elbm_ctx *ctx, double *mass, double mom[3], int64_t *n_unstable);
/* ELBM_EUNSTABLE if any node is non-finite, has rho <= 0 or |u_a| >= 1.  Synchronous. */
elbm_status elbm_check(elbm_ctx *ctx);
/* Momentum exchanged with solid nodes of a level (sum over its steps since the last
 * reset of sum over links 2 c_i f'_i, level-l units) and the number of level steps.
 * Synchronous. */
elbm_status elbm_drag(elbm_ctx *ctx, int level, double F[3], int64_t *steps, int reset);

/* Write gamma (Eq. gamma_min_approx) of every collision to a per-node buffer. */
elbm_status elbm_set_gamma_output(elbm_ctx *ctx, int enable);

/* Nodes per brick along x, y, z for dimension D (2 or 3; z is 1 in 2-D): the tiling of
 * each level box that elbm_gamma_indicator reports on, from the level box origin.
 * ELBM_EINVAL for another D or a NULL dims. */
elbm_status elbm_brick_dims(int D, int64_t dims[3]);

/* Under-resolution indicator from the entropic stabiliser.  Resolved flow drives gamma
 * to its LBGK value 2, so its deviation measures under-resolution (Sec. IV, turbulent
 * channel flow); the conclusion (Sec. V) names it as the refinement criterion of an
 * adaptive scheme.  Writes, per brick of `level` (elbm_brick_dims), the largest
 * |gamma - 2| over the brick's fluid nodes, gamma being that of each node's last
 * collision, into out_dev: device float array [grid[2]][grid[1]][grid[0]] (x fastest),
 * -1 where a brick holds no fluid node or no brick exists.  grid (host, always written)
 * receives the brick-grid extent; out_dev may be NULL to query only that (needs a
 * finalized context).  Caller owns out_dev.  ELBM_ESTATE before bind or when gamma
 * output is off (elbm_set_gamma_output); ELBM_EINVAL for a bad level.  Asynchronous on
 * the bound stream. */
elbm_status elbm_gamma_indicator(elbm_ctx *ctx, int level, float *out_dev, int64_t grid[3]);

/* Re-meshing: take over the current state of `src` in `dst`, a lattice of the same
 * domain, levels, storage, viscosity, boundaries and forcing whose refinement blocks
 * differ (the adaptive refinement the conclusion, Sec. V, proposes, e.g. driven by
 * elbm_gamma_indicator).  Call at a coarse-step boundary, both lattices bound on the
 * same device.  Per fluid node of dst: the stored values of src's node at the same
 * level and position; else coalescence of src's node one level finer at the same
 * position; else the four-point reconstruction of Eq. interp from src values at the
 * parent positions (src nodes of the node's own level where present, src parent nodes
 * elsewhere).  Density and velocity pass unchanged (or interpolated); the
 * non-equilibrium part of the post-collision state scales by
 * beta_c (1 - 2 beta_f) / (2 beta_f (1 - 2 beta_c)) from coarse to fine and by its
 * inverse from fine to coarse (Eq. f_neq_rescaling_iso with f' - f^eq =
 * (1 - 2 beta)(f - f^eq) at gamma = 2).  dst's drag accumulators restart.  ELBM_EINVAL
 * if the lattices differ otherwise, or a dst node has no source (a newly refined
 * region must lie where src has the parent level).  Synchronous; src is unchanged. */
elbm_status elbm_transfer_state(elbm_ctx *dst, const elbm_ctx *src);

/* Launch configuration: use_graph (0: eager launches; 1: one graph per coarse step;
 * G in 2..64: graphs of G coarse steps, single-step graphs for the remainder of an
 * elbm_advance), workgroups per CU
 * for the persistent stream-collide grid (0: one workgroup per brick), XCD-aware
 * brick-to-workgroup mapping (0: none; 1: each XCD takes the bricks of its slab of each
 * level along the slowest brick axis, by a table built at finalize; B in 2..4096: runs of
 * B consecutive bricks per XCD, dealt round-robin), threads per workgroup (64, 128 or 256; each thread
 * covers 256/threads nodes of its brick), register-budget variant of the
 * stream-collide kernel (1: uncapped, 4: at most 128 VGPRs for 4 waves per SIMD),
 * pipeline (plain bricks -- every node fluid with bulk links only -- in a kernel of
 * their own and the other bricks in the general kernel with 256 threads: 1: persistent
 * software-pipelined, wg_per_cu workgroups per CU, default 2; 2: one node per thread
 * within 128 registers, one workgroup per brick unless wg_per_cu is set; threads and
 * occupancy then do not apply to the plain bricks).  Every configuration gives
 * bitwise identical populations. */
elbm_status elbm_set_launch(elbm_ctx *ctx, int use_graph, int wg_per_cu, int xcd_remap, int threads,
                            int occupancy, int pipeline);
/* Current launch configuration: {use_graph, wg_per_cu, xcd_remap, threads, occupancy,
 * pipeline}. */
elbm_status elbm_get_launch(const elbm_ctx *ctx, int32_t cfg[6]);
/* Launch configuration from a tuning cache: cache_path holds one
 *   "key": [graph, wg_per_cu, xcd, threads, occupancy, pipeline]
 * line per workload shape, key = "d<dim>s<storage>_<bricks of level 0>_<bricks of
 * level 1>...".  On a hit the configuration is applied (as elbm_set_launch) and the
 * state is untouched.  A miss (or a missing file) returns ELBM_ESTATE with the key in
 * the error text and leaves the configuration unchanged.  The cache is written by the
 * launch tuner (paper_1608_06915_amd/tune.py, every candidate timed in a process of its
 * own); `steps` is reserved and ignored. */
elbm_status elbm_tune(elbm_ctx *ctx, const char *cache_path, int steps);
/* Advance `steps` coarse steps eagerly (no graphs), timing every tick's stream-collide
 * with HIP events on the bound stream: a tick of one launch passes the events to
 * hipExtLaunchKernel, which stamps them with the kernel's own start and end; a tick split
 * into two launches (pipeline modes) records them around both.  Returns the total
 * milliseconds, the summed stream-collide milliseconds and the number of timed ticks;
 * the state advances exactly as elbm_advance would.  Synchronous. */
elbm_status elbm_profile(elbm_ctx *ctx, int steps, double *ms_total, double *ms_stream_collide,
                         int64_t *n_launches);
/* Measurement aid, not part of the method: a plain streaming copy of `bytes` (a
 * multiple of 16) from src_dev to dst_dev (caller-owned, 16-byte aligned, not
 * overlapping) with `grid` workgroups of 256 threads (0: four per compute unit),
 * 16-byte loads and non-temporal stores, on the given HIP stream (NULL: default).
 * Timing it gives the read + write bandwidth HBM sustains for a pure stream, against
 * which the stream-collide's traffic is compared.  ELBM_EINVAL for a bad argument.
 * Asynchronous. */
elbm_status elbm_stream_copy(void *dst_dev, const void *src_dev, size_t bytes, int grid, void *hip_stream);

/* Wait for the bound stream. */
elbm_status elbm_synchronize(elbm_ctx *ctx);

/* Checkpoint: state bytes, copy state to/from caller device memory (async). */
elbm_status elbm_state_bytes(const elbm_ctx *ctx, size_t *bytes);
elbm_status elbm_save_state(elbm_ctx *ctx, void *dev_dst);
elbm_status elbm_load_state(elbm_ctx *ctx, const void *dev_src);

/* ---- Discrete adjoint.  The paper has no adjoint: this is the exact transpose of the
 * linearised coarse step that elbm_advance computes (collision of Sec. II.A with the
 * stabiliser of Eq. gamma_min_approx and the exact-difference forcing of Sec. III.A,
 * the rescaling Eq. f_neq_rescaling_iso and reconstruction Eq. interp of Sec. III, and
 * streaming, in the order of the Sec. III.C schedule).  Where <dh|dh> = 0 the
 * stabiliser is the constant 2 and is not differentiated; the collision is not
 * differentiable at equilibrium, so gradients are meaningful at non-equilibrium
 * states.  Half-precision storage is differentiated as if rounding were the
 * identity.  Adjoint arithmetic uses the compute type of the storage (FP64 for
 * ELBM_F64, else FP32).
 *
 * Objectives:
 *   ELBM_OBJ_DRAG  J = dir . (sum over the run's substeps of level body_level of the
 *                  momentum exchange 2 c_i f'_i on solid links) / number of substeps;
 *   ELBM_OBJ_KE    J = 1/2 sum_l sum_x w |j - F/2|^2 / rho at the final state, w the
 *                  owned-volume weights of elbm_weights. */
typedef enum { ELBM_OBJ_DRAG = 0, ELBM_OBJ_KE = 1 } elbm_objective;

/* Device workspace for runs of up to n_max coarse steps with a checkpoint every K
 * coarse steps: ceil(n_max/K) checkpointed states, two tapes of K 2^l + 1 states per
 * level l (the recomputation of one segment fills one while the reverse sweep of the
 * next segment reads the other), and the adjoint fields.  After elbm_finalize. */
elbm_status elbm_adjoint_bytes(elbm_ctx *ctx, int n_max, int K, size_t *bytes);
/* Bind the caller-owned adjoint workspace (256-byte aligned, at least the size above;
 * never freed by the library).  After elbm_bind. */
elbm_status elbm_adjoint_bind(elbm_ctx *ctx, void *workspace_dev, size_t bytes, int n_max, int K);
/* Advance n coarse steps (1 <= n <= n_max) from the current state as elbm_advance
 * does, checkpointing every K steps, and evaluate J (written to *J).  The state
 * afterwards is the final state.  For ELBM_OBJ_DRAG the drag accumulators of
 * body_level are reset before and after.  Synchronous. */
elbm_status elbm_adjoint_forward(elbm_ctx *ctx, int n, int objective, int body_level, const double dir[3],
                                 double *J);
/* Reverse sweep of the preceding elbm_adjoint_forward: segment by segment the forward
 * is recomputed from its checkpoint, then its ticks are reversed.  The state, force
 * fields and geometry must not change in between (not checked).  The forward state is
 * left unchanged.  Synchronous. */
elbm_status elbm_adjoint_backward(elbm_ctx *ctx);
/* Results of elbm_adjoint_backward for one level, device arrays over the level box:
 * lam [Q][box] = dJ/df of the state at the start of the forward run, dJdF [D][box] =
 * dJ/dF for the per-node force field of elbm_set_force_field (level-0 units).  Zero
 * at absent and solid nodes.  Either pointer may be NULL.  Asynchronous. */
elbm_status elbm_adjoint_read(elbm_ctx *ctx, int level, double *lam_dev, double *dJdF_dev);
/* dJ/du0 [D][box] (host) through the initialisation f = f^eq(rho0, u0) (1 + noise) of
 * elbm_init_fields, given the same host arrays that initialised the level.
 * Synchronous. */
elbm_status elbm_adjoint_velocity(elbm_ctx *ctx, int level, const double *rho_host, const double *u_host,
                                  const double *noise_host, double *out_host);
/* Milliseconds of the last adjoint run: [0] forward with checkpoints, [1] recomputation
 * (summed over segments), [2] reverse ticks (summed), [3] the whole backward pass
 * (the recomputation of a segment overlaps the reverse sweep of the next one, so
 * [3] < [1] + [2] when there are several segments). */
elbm_status elbm_adjoint_timing(const elbm_ctx *ctx, double ms[4]);

#ifdef __cplusplus
}
#endif
#endif
