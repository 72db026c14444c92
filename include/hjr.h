/*
 * hjr.h -- C ABI of libhjr: grid-based Hamilton-Jacobi reachability safe-set
 * solves on AMD Instinct MI355X (gfx950).
 *
 * What is computed (Herbert, Choi et al., "Scalable Learning of Safety
 * Guarantees for Autonomous Systems using Hamilton-Jacobi Reachability"):
 *
 *   - Sec. II-A, eq. (1)-(2): the value function of the safety problem is
 *     found by iterating the HJI variational inequality backwards in time
 *     from the constraint function until it stops changing; its converged
 *     sign gives the safe set.  This library stores the negated quantities
 *     (l = -c, V = -V_paper), so one iteration of time step dt is
 *         Vhat = V + dt L(V),  Vtil = Vhat + dt L(Vhat),
 *         V'   = min(l, (V + Vtil) / 2),
 *     with L(V) = H(x, (p+ + p-)/2) + sum_i alpha_i (p+_i - p-_i)/2,
 *     H(x, p) = max_u min_d p . f(x, u, d), p+- the second-order ENO
 *     one-sided derivatives (two linear-extrapolation ghost nodes per side),
 *     alpha_i = max over the grid and the control/disturbance box vertices of
 *     |f_i| (global Lax-Friedrichs), dt = cfl / sum_i alpha_i / dx_i.  The
 *     iteration stops after the first step whose residual max |V' - V| is
 *     < tol; the residual runs over all nodes, or, with a band b > 0, over
 *     the nodes where |V| < b or |V'| < b (the safe set { V >= 0 } depends
 *     on the values near V = 0 only; the paper asks for convergence without
 *     fixing a norm).
 *   - Sec. III-A: a decomposable system is solved as independent subsystem
 *     problems (hjr_solve_batch solves many in one device pass).
 *   - Sec. III-B: warm start -- pass a previous converged V as V0.
 *   - Sec. III-C: coarse approximations -- converge on a coarse grid, carry
 *     V to a finer grid by multilinear interpolation, continue
 *     (hjr_interp, hjr_solve_levels, hjr_problem.nlev).
 *
 * Conventions for every entry point:
 *   - Arrays are dense, row-major, last grid axis fastest, element type
 *     float (HJR_F32) or double (HJR_F64) as chosen by hjr_opts.dtype.
 *   - Every array pointer is a DEVICE pointer owned by the caller, unless
 *     stated otherwise; scalars reported back (iterations, residual, stats)
 *     are written through HOST pointers.
 *   - Work is enqueued on opts->stream (a hipStream_t; NULL = the null
 *     stream).  Solves synchronise that stream before returning, because
 *     the host decides how many iterations to launch; hjr_interp and
 *     hjr_refine_mask return without synchronising unless stated.
 *   - No exception crosses the ABI and the library never aborts; errors are
 *     reported as hjr_status.  The only process-wide state is a mutex-guarded
 *     pool of idle solver engines (device tables, pinned staging buffers, a
 *     stream and captured graphs), reused by later calls; every call is
 *     thread-safe.
 *   - A grid is valid if 1 <= ndim <= 4, n_i >= 3, lo_i < hi_i; node j of
 *     axis i sits at lo_i + j (hi_i - lo_i)/(n_i - 1) (both ends are nodes).
 */
#ifndef HJR_H
#define HJR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hjr_status {
    HJR_OK = 0,
    HJR_EINVAL = 1,         /* invalid argument; nothing was enqueued */
    HJR_ENOMEM = 2,         /* device/host allocation failed, workspace too small,
                               or a request exceeds a server's memory budget */
    HJR_NOT_CONVERGED = 3,  /* max_iter reached; outputs hold the last iterate */
    HJR_EDEVICE = 4,        /* a HIP runtime call failed */
    HJR_EBUSY = 5,          /* server: ticket still running / queue full */
    HJR_ENOTFOUND = 6       /* server: unknown ticket */
} hjr_status;

enum hjr_dtype { HJR_F32 = 0, HJR_F64 = 1 };

/* Dynamics kinds and their parameter vectors hjr_dyn.p[]:
 *  HJR_QUAD_Z2D  vertical quadcopter / z-subsystem (paper Sec. V, and the
 *                z rows of eq. (3)); state (z, vz):
 *                z' = vz, vz' = k u - g + d,  u in [u_lo, u_hi].
 *                p = {k, g, u_lo, u_hi}; disturbance channel 0.
 *  HJR_QUAD_X4D  x-subsystem of the near-hover quadcopter (eq. (3));
 *                state (x, vx, theta, omega):
 *                x' = vx + d, vx' = g tan(theta), theta' = -d1 theta + omega,
 *                omega' = -d0 theta + n0 S,  |S| <= s_max.
 *                p = {g, d1, d0, n0, s_max}; disturbance channel 0.
 *  HJR_QUAD_X4DV the x-subsystem as the 10-D model of Sec. IV, eq. (3)
 *                writes it, with the disturbance on the velocity rate:
 *                x' = vx, vx' = g tan(theta) + d, theta' = -d1 theta + omega,
 *                omega' = -d0 theta + n0 S,  |S| <= s_max.
 *                p = {g, d1, d0, n0, s_max}; disturbance channel 0.
 *  HJR_DI2X2     test model: two independent QUAD_Z2D systems a, b on one
 *                4-D grid; p = {k_a, g_a, ulo_a, uhi_a, k_b, g_b, ulo_b,
 *                uhi_b, axis(z_a), axis(v_a), axis(z_b), axis(v_b)} (axes as
 *                doubles, a permutation of 0..3); channel 0 acts on a, 1 on b.
 */
enum hjr_dyn_kind { HJR_QUAD_Z2D = 0, HJR_QUAD_X4D = 1, HJR_DI2X2 = 2, HJR_QUAD_X4DV = 3 };

typedef struct hjr_grid {
    int32_t ndim;
    int32_t n[4];
    double lo[4];
    double hi[4];
} hjr_grid;

typedef struct hjr_dyn {
    int32_t kind;
    int32_t reserved;
    double p[16];
} hjr_dyn;

/* Disturbance bound d in [lo, hi] of one channel (paper Sec. II-C: learned
 * bounds arrive as new D; here a constant box per channel). */
typedef struct hjr_dstb {
    double lo;
    double hi;
} hjr_dstb;

typedef struct hjr_opts {
    int32_t dtype;          /* HJR_F32 (default) or HJR_F64 */
    int32_t order;          /* 2 = ENO2 (default), 1 = first-order upwind */
    double cfl;             /* 0 < cfl <= 1, default 0.8 */
    int64_t max_iter;       /* >= 1, default 100000 (per level) */
    void* stream;           /* hipStream_t, NULL = null stream */
    void* workspace;        /* device scratch from the caller, or NULL to let
                               the library allocate (and free) its own */
    size_t workspace_bytes; /* size of workspace; >= hjr_*_workspace_bytes */
    int32_t chunk;          /* iterations enqueued between host convergence
                               checks; 0 = library default */
    int32_t flags;          /* HJR_FLAG_* */
    int32_t tile_rows;      /* rows of the two fastest axes per LDS tile (a
                               tuning knob, see paper_2101_05916_amd/autotune.py);
                               0 = library default.  Clamped to what fits. */
    int32_t walk;           /* 4-D problems on narrow LDS planes (last axis
                               <= 64 nodes, no per-node bounds): consecutive
                               axis-0 planes one workgroup walks through per
                               tile (a tuning knob; results do not depend on
                               it); 0 (default) or -1 = none (plane tiles one
                               by one), k >= 1 = k */
    double band;            /* residual band of the stop test (see above);
                               0 (default) = every node; must be >= 0 */
} hjr_opts;

/* flags */
#define HJR_FLAG_NO_GRAPH 1     /* launch chunks kernel by kernel, no hipGraph */
#define HJR_FLAG_NO_PIPELINE 2  /* wait for each chunk before enqueuing the next */
#define HJR_FLAG_PROFILE 4      /* time the RK-stage launches of one chunk in
                                   eight with HIP events stamped at each
                                   stage's first kernel start and last kernel
                                   end (implies HJR_FLAG_NO_GRAPH) */
#define HJR_FLAG_FLAT_TILES 8   /* use the shape-agnostic flat tiles only (the
                                   LDS plane tiles are the default where the
                                   last axis has <= 204 nodes) */

typedef struct hjr_stats {
    int64_t iterations;     /* RK2 steps taken (sum over levels for multi-level jobs) */
    double residual;        /* max |V' - V| of the last step (last level) */
    double dt;              /* time step of the last level */
    double alpha[4];        /* Lax-Friedrichs bounds of the last level */
    int32_t status;         /* hjr_status of this solve */
    int32_t levels;         /* levels completed */
    int64_t level_iterations[4]; /* steps per level */
    int64_t cell_updates;   /* sum over levels of (nodes x steps) */
    double device_ms;       /* device time from the first enqueue to completion */
    double kernel_ms[2];    /* with HJR_FLAG_PROFILE: summed device time of the
                               timed RK stage-1 and stage-2 launches (one chunk
                               in eight; a stage's launches of all tile families
                               count as one; steps past every problem's stop
                               step are left out) */
    int64_t kernel_launches[2]; /* with HJR_FLAG_PROFILE: number of timed stages */
    int64_t kernel_cell_updates; /* with HJR_FLAG_PROFILE: cell-updates those timed
                                    launches performed */
} hjr_stats;

/* Fill *o with the defaults listed in hjr_opts.  Never fails for o != NULL. */
hjr_status hjr_opts_default(hjr_opts* o);

/* Static text for a status code. */
const char* hjr_strerror(hjr_status s);

/* Bytes of device workspace hjr_solve / hjr_solve_ex needs for one problem on
 * grid g with options o: the stage-1 array, a per-axis table and the per-
 * tile flags of a localized update.  (The
 * library also keeps small per-engine tables -- problem descriptors, residual
 * words, pinned staging, captured graphs -- which it allocates on first use
 * and reuses across calls.)  EINVAL for an invalid grid or dtype. */
hjr_status hjr_workspace_bytes(const hjr_grid* g, const hjr_opts* o, size_t* out);

/* One safe-set computation (paper Sec. II-A, eq. (2); warm start Sec. III-B).
 *   dyn, grid   model and grid (host structs, copied before return)
 *   l           constraint function on the grid (N = prod n_i elements);
 *               l > 0 inside the constraint set
 *   V0          initial value, or NULL for the cold start V0 = l; the first
 *               iterate is min(l, V0).  May alias V_out (in-place update).
 *   d           host array of disturbance bounds, one per channel of dyn
 *   tol         > 0; stop after the first step whose residual (max |V' - V|
 *               over the nodes selected by o->band) is < tol
 *   o           options (NULL = defaults)
 *   V_out       result (N elements); holds the last iterate on NOT_CONVERGED
 *   iterations, residual   host outputs (nullable)
 * Returns OK, NOT_CONVERGED, EINVAL (nothing enqueued), ENOMEM, EDEVICE.
 * Synchronises o->stream. */
hjr_status hjr_solve(const hjr_dyn* dyn, const hjr_grid* grid, const void* l,
                     const void* V0, const hjr_dstb* d, double tol,
                     const hjr_opts* o, void* V_out, int64_t* iterations,
                     double* residual);

/* hjr_solve that also reports dt, alpha and timing in *stats (host, nullable). */
hjr_status hjr_solve_ex(const hjr_dyn* dyn, const hjr_grid* grid, const void* l,
                        const void* V0, const hjr_dstb* d, double tol,
                        const hjr_opts* o, void* V_out, hjr_stats* stats);

/* Device scratch bytes available to hjr_solve_noalloc per device. */
#define HJR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* hjr_solve_ex for callers that cannot allocate memory: code that must not
 * call hipMalloc (tight serving loops, harnesses that forbid allocation).
 * The stage-1 array, the per-axis table and the iteration tables live in a
 * statically sized device array of HJR_NOALLOC_SCRATCH_BYTES per device
 * (loaded with the library, held until the process ends); the host staging
 * is on the caller's stack.  The call allocates no device or pinned host
 * memory and creates no stream, event or graph: it runs on o->stream
 * itself, launching kernel by kernel (hjr_opts.flags other than
 * HJR_FLAG_FLAT_TILES and hjr_opts.workspace are ignored) and synchronising
 * that stream after every chunk of o->chunk iterations.  Arguments, results
 * and statuses as for hjr_solve_ex (stats->device_ms is the call's wall
 * time); results are bit-identical to hjr_solve_ex's.  ENOMEM, with nothing
 * enqueued, if the grid needs more scratch than HJR_NOALLOC_SCRATCH_BYTES
 * (about N elements of the dtype: up to ~16.7e6 FP32 or ~8.3e6 FP64 nodes).
 * Every call on one device shares that device's scratch: calls that overlap
 * on one device (from several threads or streams) race and must not be
 * issued; sequential calls are independent (nothing is carried over). */
hjr_status hjr_solve_noalloc(const hjr_dyn* dyn, const hjr_grid* grid, const void* l,
                             const void* V0, const hjr_dstb* d, double tol,
                             const hjr_opts* o, void* V_out, hjr_stats* stats);

/* Level transition of the coarse-to-fine scheme (paper Sec. III-C): sample
 * V_src (grid src) onto grid dst by multilinear interpolation.  For
 * destination index j of axis i: num = j (n_src - 1), q = num div
 * (n_dst - 1), t = (num mod (n_dst - 1)) / (n_dst - 1) in double (q = n_src - 2,
 * t = 1 at the last node); the 2^D corner weights are products of t and 1 - t
 * in double, summed in double in row-major corner order, rounded once to the
 * element type.  If l_dst != NULL the result is then min(l_dst, .).  Works in
 * both directions (refine or restrict).  src and dst must share ndim, lo and
 * hi exactly (else EINVAL).  V_dst must not overlap V_src.  Asynchronous. */
hjr_status hjr_interp(const hjr_grid* src, const void* V_src, const hjr_grid* dst,
                      void* V_dst, const void* l_dst, const hjr_opts* o);

/* Refinement mask of a level (cells straddling the zero level set, which
 * bounds the safe set of Sec. II-A): for each cell c in [0, n-2]^D (row-major,
 * (n-1)^D bytes), mask[c] = 1 iff among its 2^D corner nodes one has V >= 0
 * and another V < 0, else 0.  mask is a device pointer; *count (host,
 * nullable) receives the number of marked cells, in which case the call
 * synchronises o->stream. */
hjr_status hjr_refine_mask(const hjr_grid* g, const void* V, uint8_t* mask,
                           int64_t* count, const hjr_opts* o);

/* Coarse-to-fine solve of one subsystem (paper Sec. III-C): level 0 starts
 * from V0 (NULL = cold, V0 = l[0]); level k > 0 starts from
 * min(l[k], interp(V*_{k-1})).  grids[k] share one box.  V_levels[k] (device,
 * N_k elements each) receive every level's converged value; masks[k]
 * (nullable array, nullable entries, (n_k - 1)^D bytes) receive each level's
 * refinement mask and mask_counts[k] (host, nullable) its count.  stats
 * (host, nullable) gets per-level iterations in level_iterations.  nlev in
 * 1..4.  Synchronises o->stream. */
hjr_status hjr_solve_levels(const hjr_dyn* dyn, int32_t nlev, const hjr_grid* grids,
                            const void* const* l, const void* V0, const hjr_dstb* d,
                            double tol, const hjr_opts* o, void* const* V_levels,
                            uint8_t* const* masks, int64_t* mask_counts,
                            hjr_stats* stats);

/* Safe-set computation with state-dependent disturbance bounds (paper
 * Sec. II-A: the disturbance ranges over a set D(x) that depends on the
 * state; Sec. II-C: the learned bound is a confidence interval at every
 * state).  As hjr_solve_levels, except that level k's disturbance box at
 * node i comes from the device array dfield[k] of 2 * nch * N_k elements of
 * the solve's dtype (nch = 1 for QUAD_Z2D and QUAD_X4D, 2 for DI2X2):
 * dfield[k][2c N_k + i] is the lower and dfield[k][(2c + 1) N_k + i] the
 * upper bound of channel c at node i.  The Hamiltonian at a node takes its
 * min over that node's box; the Lax-Friedrichs bound alpha_i is the max of
 * |f_i| over every node and the vertices of its box.  Every pair must be
 * two finite numbers with lower <= upper: the fields are checked on the
 * device before anything else is enqueued, and the call returns EINVAL if
 * one is not.  The fields are only read and must stay valid until the call
 * returns.  nlev in 1..4, grids as for hjr_solve_levels; no refinement
 * masks.  Synchronises o->stream. */
hjr_status hjr_solve_field(const hjr_dyn* dyn, int32_t nlev, const hjr_grid* grids,
                           const void* const* l, const void* const* dfield, const void* V0,
                           double tol, const hjr_opts* o, void* const* V_levels,
                           hjr_stats* stats);

/* Localized warm start (Sec. VI names localized warm starting as a further
 * speed-up): the band of a previous value V on grid g -- node i is in it iff
 * a cell straddling V = 0 (the cells of hjr_refine_mask) lies within k cells
 * of it, i.e. for every axis the cell's index range [c_a, c_a + 1] is at
 * most k nodes from i_a.  node_mask: DEVICE, N bytes (1 in the band, else
 * 0); *count (host, nullable): nodes in the band.  k >= 0.  Allocates two N-
 * byte scratch arrays for the call and synchronises o->stream. */
hjr_status hjr_band_mask(const hjr_grid* g, const void* V, int32_t k, uint8_t* node_mask,
                         int64_t* count, const hjr_opts* o);

/* Localized update: hjr_solve_ex (d: constant boxes, or dfield: per-node
 * boxes as in hjr_solve_field, nullable) in which only the nodes with
 * node_mask[i] != 0 (DEVICE, N bytes) are updated; every other node keeps
 * its initial value min(l, V0) throughout and serves as boundary data, and
 * the residual runs over the masked nodes (an empty mask stops after one
 * step).  The 4-D x-subsystem with ENO2 and constant boxes runs on plane
 * tiles, over the list of the tiles that hold a masked node (built once per
 * solve, with a device-to-host copy of one flag per tile); every other case
 * runs on the flat tiles and skips tiles without a masked node.
 * stats->cell_updates counts masked nodes x steps.  Synchronises o->stream. */
hjr_status hjr_solve_local(const hjr_dyn* dyn, const hjr_grid* grid, const void* l, const void* V0,
                           const hjr_dstb* d, const void* dfield, const uint8_t* node_mask,
                           double tol, const hjr_opts* o, void* V_out, hjr_stats* stats);

/* One independent subsystem problem of a batch (decomposition, Sec. III-A). */
typedef struct hjr_problem {
    hjr_dyn dyn;
    int32_t nlev;           /* 1..4 grid levels, coarse to fine */
    int32_t reserved;
    hjr_grid grids[4];
    const void* l[4];       /* constraint per level (device) */
    void* V[4];             /* converged value per level (device, output) */
    const void* V0;         /* start on level 0, NULL = cold */
    hjr_dstb d[2];
    double tol;
    int32_t tile_rows[4];   /* per level, 0 = hjr_opts.tile_rows / default */
    double band;            /* residual band of this problem's stop test,
                               0 = every node (hjr_opts.band is not used) */
    const void* dfield[4];  /* per level: per-node disturbance boxes (device,
                               layout of hjr_solve_field), or NULL = the
                               constant boxes d (then d must be valid) */
    int32_t order[4];       /* per level: spatial derivative order (1 =
                               one-sided first order, 2 = ENO2), 0 =
                               hjr_opts.order; any other value is EINVAL.
                               Sec. III-C: a coarse level with cheap gradient
                               approximations (order 1) starts the finer
                               level's ENO2 solve. */
} hjr_problem;

/* Bytes of device workspace hjr_solve_batch needs for these problems. */
hjr_status hjr_batch_workspace_bytes(int32_t n, const hjr_problem* probs,
                                     const hjr_opts* o, size_t* out);

/* Solve n independent problems together: every device pass advances all
 * unfinished problems by one RK2 step, so per-launch cost is shared and the
 * chip stays full.  Each problem's result is bit-identical to solving it
 * alone (no arithmetic crosses problems).  Disturbance fields
 * (hjr_problem.dfield) are checked as in hjr_solve_field before anything is
 * solved (EINVAL if one is invalid).  results (host, n entries, nullable)
 * receive per-problem stats.  Returns OK if every problem
 * converged, NOT_CONVERGED if any did not (see results[i].status), or an
 * error.  Synchronises o->stream. */
hjr_status hjr_solve_batch(int32_t n, const hjr_problem* probs, const hjr_opts* o,
                           hjr_stats* results);

/* ------------------------------------------------------------------------ */
/* Safety queries on a converged value function (paper Sec. II-A: the        */
/* gradient of the converged value gives the optimal safety controller;     */
/* Sec. II-B: it overrides the learned policy near the safe set's boundary) */
/* ------------------------------------------------------------------------ */

/* Controls per model: QUAD_Z2D {u}, QUAD_X4D and QUAD_X4DV {S}, DI2X2 {u_a, u_b}. */
typedef struct hjr_query {
    int64_t n;              /* states queried (0: nothing to do) */
    const double* x;        /* DEVICE, n x ndim, state-major (x[i ndim + a]) */
    double* value;          /* DEVICE, n, or NULL: V at x, multilinear
                               interpolation of the grid values (corner
                               weights products of t and 1 - t in double, t
                               the fraction of x in its cell, corners in
                               row-major order of their offsets) */
    double* grad;           /* DEVICE, n x ndim, or NULL: the same
                               interpolation of the node gradients
                               (p+ + p-)/2 the solver evaluates H with
                               (hjr_opts.order: 2 = ENO2, 1 = first order) */
    double* u_star;         /* DEVICE, n x nctrl, or NULL: the optimal safety
                               control, the control-box vertex maximising
                               min over d of grad . f(x, u, d): each input at
                               the bound picked by the sign of its
                               coefficient in grad . f, the upper bound when
                               that coefficient is 0 */
    const double* u_perf;   /* DEVICE, n x nctrl, or NULL: a performance
                               control to filter */
    double* u_out;          /* DEVICE, n x nctrl, or NULL (needs u_perf): the
                               least-restrictive filter, u_perf where
                               value >= level, else u_star */
    double level;           /* filter threshold on the value (0 = the safe
                               set's boundary; a positive level overrides
                               earlier) */
} hjr_query;

/* Safety query at n states on the value V (N elements of o->dtype, e.g. the
 * output of a solve) over grid with model dyn.  Computed in double after
 * the loads of V.  A state outside the grid box, or with a NaN coordinate,
 * gets NaN in every output (and u_out = u_star = NaN).  EINVAL for an
 * invalid model, grid, order or dtype, n < 0, missing x or V with n > 0,
 * u_out without u_perf, or a NaN level; nothing is enqueued then.
 * Asynchronous on o->stream. */
hjr_status hjr_safety_query(const hjr_dyn* dyn, const hjr_grid* grid, const void* V,
                            const hjr_query* q, const hjr_opts* o);

/* Decomposed system (paper Sec. III-A): subsystems that share no state and
 * no input have the product of their safe sets, so the full value is the
 * minimum of theirs, and each subsystem's safety controller drives its own
 * inputs.  A subsystem's axis a is component state_index[a] of the full
 * state; its controls start at component control_index of the full control
 * vector (e.g. the near-hover quadcopter: x on (px, vx, thx, wx) = (0, 1, 2,
 * 3) and control 0, y on (4, 5, 6, 7) and control 1, z on (8, 9) and
 * control 2). */
typedef struct hjr_subsystem {
    hjr_dyn dyn;
    hjr_grid grid;
    const void* V;            /* DEVICE, its converged value (hjr_opts.dtype) */
    int32_t state_index[4];   /* full-state component of each axis; distinct
                                 across subsystems */
    int32_t control_index;
    int32_t reserved;
} hjr_subsystem;

typedef struct hjr_query_decomposed {
    int64_t n;                /* states queried */
    int32_t state_dim;        /* full state dimension (<= 32) */
    int32_t control_dim;      /* full control dimension */
    const double* x;          /* DEVICE, n x state_dim */
    double* sub_value;        /* DEVICE, n x nsub: each subsystem's value
                                 (required: also the scratch of the min) */
    double* value;            /* DEVICE, n, or NULL: min over subsystems (NaN
                                 if a part of the state is outside its box) */
    int32_t* active;          /* DEVICE, n, or NULL: the first subsystem
                                 attaining the min, -1 with a NaN value */
    double* grad;             /* DEVICE, n x state_dim, or NULL: each
                                 subsystem's gradient at its components */
    double* u_star;           /* DEVICE, n x control_dim, or NULL */
    const double* u_perf;     /* DEVICE, n x control_dim, or NULL */
    double* u_out;            /* DEVICE, n x control_dim, or NULL (needs
                                 u_perf): per subsystem, its inputs from u_perf
                                 where its own value >= level, else its u_star */
    double level;
} hjr_query_decomposed;

/* hjr_safety_query per subsystem at its part of each state, then the
 * minimum.  Components of the state and control vectors that belong to no
 * subsystem are left untouched.  EINVAL (nothing enqueued) for nsub outside
 * 1..16, an invalid subsystem, overlapping or out-of-range state components,
 * controls past control_dim, or the conditions of hjr_safety_query.
 * Asynchronous on o->stream (nsub + 1 kernel launches). */
hjr_status hjr_safety_query_decomposed(int32_t nsub, const hjr_subsystem* subs,
                                       const hjr_query_decomposed* q, const hjr_opts* o);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of safe-set update requests (a request is a  */
/* new disturbance bound for a subsystem instance, paper Sec. II-C/III-B).   */
/* ------------------------------------------------------------------------ */

typedef struct hjr_server hjr_server;

typedef struct hjr_server_cfg {
    size_t hbm_budget_bytes;  /* device bytes the server may hold for resident
                                 values, constraints and scratch; requests wait
                                 until they fit; 0 = 8 GiB */
    int32_t max_active;       /* problems advanced together, 0 = 256 */
    int32_t dtype;            /* HJR_F32 or HJR_F64 */
    int32_t order;            /* 2 or 1 */
    int32_t chunk;            /* iterations per device pass group, 0 = default */
    double cfl;               /* 0 = 0.8 */
    int64_t max_iter;         /* per request, 0 = 100000 */
    int32_t device;           /* HIP device ordinal */
    int32_t flags;            /* HJR_FLAG_* */
} hjr_server_cfg;

typedef struct hjr_request {
    uint64_t instance_id;     /* subsystem instance; its converged V stays
                                 resident and warm-starts its next request */
    hjr_dyn dyn;
    hjr_grid grid;            /* must not change between requests of one instance */
    const void* l;            /* HOST array, N elements of the server dtype;
                                 copied before hjr_server_submit returns; may be
                                 NULL for later requests of a known instance */
    hjr_dstb d[2];
    double tol;
    int32_t cold;             /* 1 = ignore the resident value, start from l */
    int32_t reserved;
    double band;              /* residual band of the stop test, 0 = every node */
    const void* dfield;       /* HOST array: per-node disturbance boxes of this
                                 request (layout of hjr_solve_field, server
                                 dtype), copied before hjr_server_submit
                                 returns, or NULL = the constant boxes d */
} hjr_request;

typedef struct hjr_reply {
    int32_t status;           /* hjr_status of the solve */
    int32_t reserved;
    int64_t iterations;
    double residual;
    double latency_ms;        /* submit -> result resident */
    double queue_ms;          /* submit -> admitted */
    int32_t warm;             /* 1 if warm-started from the resident value */
    int32_t reserved2;
} hjr_reply;

/* Create a server bound to cfg->device; it owns a worker thread and a
 * stream.  cfg may be NULL for defaults. */
hjr_status hjr_server_create(const hjr_server_cfg* cfg, hjr_server** out);

/* Queue a request; *ticket (host) identifies it.  Requests for one instance
 * run in submission order.  ENOMEM if the instance alone exceeds the budget,
 * EINVAL for invalid input. */
hjr_status hjr_server_submit(hjr_server* s, const hjr_request* req, uint64_t* ticket);

/* Non-blocking: OK and *reply filled if the ticket finished, EBUSY if it
 * has not, ENOTFOUND for an unknown ticket. */
hjr_status hjr_server_poll(hjr_server* s, uint64_t ticket, hjr_reply* reply);

/* Blocking version of poll; timeout_ms < 0 waits forever.  EBUSY on timeout. */
hjr_status hjr_server_wait(hjr_server* s, uint64_t ticket, double timeout_ms,
                           hjr_reply* reply);

/* Copy an instance's resident converged value (last successful request) to
 * the HOST buffer dst of bytes size.  ENOTFOUND if the instance has none. */
hjr_status hjr_server_read_value(hjr_server* s, uint64_t instance_id, void* dst,
                                 size_t bytes);

/* Device bytes currently held by the server. */
hjr_status hjr_server_memory(hjr_server* s, size_t* used, size_t* budget);

/* Finish queued work, stop the worker, free everything. */
hjr_status hjr_server_destroy(hjr_server* s);

#ifdef __cplusplus
}
#endif

#endif
