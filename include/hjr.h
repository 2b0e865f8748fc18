/*
 * hjr.h -- C ABI of libhjr, the gfx950 (AMD Instinct MI355X) solver for the grid update of the
 * HJI variational inequality used by warm-start reachability.
 *
 * Method: Herbert, Ghosh, Bansal, Tomlin, "Reachability-Based Safety Guarantees using Efficient
 * Initializations".  Given dynamics x' = f(x, u, d) with compact control and disturbance sets
 * (Sec. II-A, eq. (1)) and a target function l whose zero sublevel set is the unsafe set
 * (Sec. II-B.1), the library marches the variational inequality min{D_t V + H, l - V} = 0
 * (eq. (7)), H = max_u min_d <grad V, f> (eq. (6)), backwards in time on a grid until V stops
 * changing.  It starts from V = l (standard reachability, eq. (12)) or from a caller-supplied
 * warm-start function k (eqs. (13)-(14)); a warm start is applied as min(k, l), the effective
 * initial value used in the proof of Theorem 1 (case b).  The result is the converged value
 * function V*; the unsafe set (backward reachable tube) is {V* <= 0} (Sec. II-B.1).
 *
 * Discrete scheme (the paper leaves it to a level-set toolbox):
 *   derivatives   HJR_UPWIND1: one-sided first differences; HJR_WENO5: fifth-order WENO of Jiang
 *                 and Peng.  Non-periodic dims extend the grid by linear extrapolation (so a
 *                 first difference beyond an edge equals the nearest interior one); periodic
 *                 dims wrap.
 *   Hamiltonian   Lax-Friedrichs: L(V) = H(x, (D-V + D+V)/2) + sum_i alpha_i(x) (D+_i V - D-_i V)/2
 *                 with alpha_i(x) = max over (u, d) of |f_i(x, u, d)|.
 *   time          backward time s = -t; HJR_EULER: V + dt L(V); HJR_TVDRK3: the three-stage
 *                 Shu-Osher scheme.  dt = cfl / max_x sum_i alpha_i(x)/dx_i (fixed per solve).
 *   projection    V <- min(l, V) after every full step (eq. (7)).  Variants, all options of the
 *                 same solver: none at all (brs: the backward reachable set, Sec. II); the step's
 *                 result times a discount factor before it (discounted reachability, Sec. II-C);
 *                 max(g, .) after it (reach-avoid with a constraint function g).
 *   local updates optional exact skipping of node blocks whose neighbourhood did not change
 *                 (the local updating of Sec. VII); results are bitwise those of full updates.
 *   stopping      HJR_CONV_PER_STEP: stop when max_x |V^{n+1} - V^n| < tol.
 *                 HJR_CONV_PER_INTERVAL: steps are cut to end on multiples of dt_report and the
 *                 change across a whole interval is tested (the rule of Sec. IV: interval 0.01,
 *                 threshold 0.001).  Also stop at max_iter steps or at t_max (t_max > 0).
 *   precision     HJR_FP64: everything in FP64.  HJR_FP32: stencil, Hamiltonian and RK in FP32
 *                 (time, dt and the convergence test in FP64).  HJR_FP32_POLISH64: FP32 until
 *                 the change is below tol_fp32, then FP64 from min(l, V32 + polish_shift) until
 *                 it is below tol; starting above the FP64 solution makes the polish exact by
 *                 Theorem 2.
 *
 * Memory layout: every grid array is dense, C order (the last dimension is contiguous), one
 * double per node.  Node j of dim i is at lo[i] + j*dx[i]; dx = (hi-lo)/(n-1) for a non-periodic
 * dim (both ends are nodes) and (hi-lo)/n for a periodic dim (hi excluded).
 *
 * Errors: every entry point returns an hjr_status.  Negative values are errors (nothing was
 * written to the outputs), positive values are warnings with valid outputs.  hjr_last_error()
 * returns a thread-local description of the last error on the calling thread.  Arguments are
 * validated before any device work; a non-finite l or k is reported as HJR_ERR_NONFINITE.
 *
 * Ownership: the library never keeps a caller pointer beyond the call, except on the submit
 * path, where l_dev, k_dev and V_dev must stay valid until hjr_poll reports the ticket done.
 * Host pointers may be pageable memory.
 *
 * Threads: hjr_solve, hjr_solve_device, hjr_batch_solve and the kernel-level entry points may be
 * called from several threads.  One hjr_ctx must be used from one thread at a time.
 */
#ifndef HJR_H
#define HJR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HJR_ABI_VERSION 5
#define HJR_MAX_DIM 6
#define HJR_MAX_PARAMS 16

typedef int32_t hjr_status;
enum {
    HJR_OK = 0,
    HJR_NOT_CONVERGED = 1,   /* max_iter reached; V is the last iterate */
    HJR_PENDING = 2,         /* hjr_poll: the ticket is still running */
    HJR_HORIZON = 3,         /* t_max reached (finite-horizon solve); V is V(., -t_max) */
    HJR_ERR_INVALID_ARG = -1,
    HJR_ERR_UNSUPPORTED = -2,
    HJR_ERR_NONFINITE = -3,
    HJR_ERR_OOM = -4,
    HJR_ERR_DEVICE = -5,
    HJR_ERR_BUDGET = -6,     /* a request can never fit the context's memory budget */
    HJR_ERR_UNKNOWN_TICKET = -7
};

/* Grid.  ndim in 1..6 and equal to the model's state dimension; n[i] >= 3 (>= 7 with WENO5);
 * lo[i] < hi[i]; the product of n must stay below 2^29 (an FP64 field stays below 4 GiB). */
typedef struct {
    int32_t ndim;
    int32_t n[HJR_MAX_DIM];
    double lo[HJR_MAX_DIM];
    double hi[HJR_MAX_DIM];
    uint32_t periodic_mask;  /* bit i set: dim i is periodic */
} hjr_grid;

/* Models (state order in brackets) and parameter layouts:
 *  HJR_DYN_DOUBLE_INTEGRATOR [x1, x2]: x1' = x2 + d, x2' = b u; |u| <= ubar, |d| <= dbar
 *      (the running example of Sec. II-A, eq. (2)).       params = {ubar, b, dbar}
 *  HJR_DYN_DUBINS3 [x, y, theta]: x' = v cos(theta) + d1, y' = v sin(theta) + d2, theta' = u;
 *      |u| <= ubar, |d_i| <= dbar_i.                        params = {v, ubar, dbar1, dbar2}
 *  HJR_DYN_UNICYCLE4 [x, y, theta, v]: x' = v cos(theta) + d1, y' = v sin(theta) + d2,
 *      theta' = u1, v' = u2; |u1| <= ubar1, |u2| <= ubar2; (d1, d2) in the disk of radius dbar
 *      (shape 0) or the box |d_i| <= dbar (shape 1).       params = {ubar1, ubar2, dbar, shape}
 *  HJR_DYN_QUAD6 [px, py, pz, vx, vy, vz]: p' = v, vx' = g tan(theta) + dx,
 *      vy' = -g tan(phi) + dy, vz' = T/m - g + dz; |theta| <= theta_max, |phi| <= phi_max,
 *      T in [Tmin, Tmax], |d_i| <= dbar_i.
 *      params = {g, m, phi_max, theta_max, Tmin, Tmax, dbar_x, dbar_y, dbar_z}
 *  HJR_DYN_QUAD10_XY [p, v, theta, omega]: one horizontal subsystem of the 10-D near-hover
 *      quadrotor (Sec. VI, eq. (Quad10D_dyn)): p' = v + d, v' = g tan(theta),
 *      theta' = -d1 theta + omega, omega' = -d0 theta + n0 S; |S| <= S_max, |d| <= dbar; the
 *      theta range of the grid must lie inside (-pi/2, pi/2).
 *      params = {g, d0, d1, n0, S_max, dbar}
 *  HJR_DYN_QUAD10_Z [p_z, v_z]: its vertical subsystem: p_z' = v_z + d, v_z' = (k_T/m) T - g;
 *      T in [T_min, T_max], |d| <= dbar.                    params = {g, k_T, m, T_min, T_max, dbar} */
enum {
    HJR_DYN_DOUBLE_INTEGRATOR = 1,
    HJR_DYN_DUBINS3 = 2,
    HJR_DYN_UNICYCLE4 = 3,
    HJR_DYN_QUAD6 = 4,
    HJR_DYN_QUAD10_XY = 5,
    HJR_DYN_QUAD10_Z = 6
};

typedef struct {
    int32_t id;
    int32_t n_params;
    double params[HJR_MAX_PARAMS];
} hjr_dynamics;

enum { HJR_AVOID = 0, HJR_REACH = 1 };      /* AVOID: control maximises, disturbance minimises */
enum { HJR_UPWIND1 = 1, HJR_WENO5 = 5 };
enum { HJR_EULER = 1, HJR_TVDRK3 = 3 };
enum { HJR_FP64 = 0, HJR_FP32 = 1, HJR_FP32_POLISH64 = 2 };
enum { HJR_CONV_PER_STEP = 0, HJR_CONV_PER_INTERVAL = 1 };

typedef struct {
    int32_t game;           /* HJR_AVOID (default) | HJR_REACH */
    int32_t spatial;        /* HJR_UPWIND1 | HJR_WENO5 (default) */
    int32_t temporal;       /* HJR_EULER | HJR_TVDRK3 (default) */
    int32_t precision;      /* HJR_FP64 | HJR_FP32 | HJR_FP32_POLISH64 (default) */
    int32_t conv_mode;      /* HJR_CONV_PER_STEP (default) | HJR_CONV_PER_INTERVAL */
    int32_t steps_per_sync; /* time steps launched between host checks; 0 = adaptive */
    double cfl;             /* in (0, 1]; default 0.5 */
    double tol;             /* > 0; default 1e-6 */
    double tol_fp32;        /* FP32-phase threshold; 0 = max(tol, k ulp_fp32(max |l|)), k = 3 before the
                               FP64 polish, 8 for HJR_FP32 alone */
    double polish_shift;    /* < 0 = auto (2 * tol_fp32); the FP64 polish starts at min(l, V32 + shift) */
    double dt_report;       /* interval length of HJR_CONV_PER_INTERVAL; default 0.01 */
    double t_max;           /* > 0: stop at this backward time (finite horizon); default 0 */
    double dt_max;          /* > 0: cap on dt; default 0 (a vanishing flow field uses dt = 1) */
    int64_t max_iter;       /* cap on time steps per phase; default 100000 */
    int64_t stall_window;   /* HJR_FP32 and HJR_FP32_POLISH64: after this many steps without the
                               change dropping 1% below its smallest value in the phase (16 times
                               as many while the change is above 64 tol), the phase ends as
                               stalled.  A stalled FP32 phase hands over to the polish; a
                               stalled final phase returns HJR_NOT_CONVERGED with converged = 3.
                               The polish waits 8 times as long (its stall is final).
                               0 = 128; < 0 disables.  HJR_FP64 solves never stop this way. */
    int32_t brs;            /* 0 (default): the backward reachable tube of the VI, eq. (7): every step
                               ends with V <- min(l, V).  1: the backward reachable set of Sec. II
                               at time t_max: the HJ PDE, eq. (5), with no projection.  Needs
                               t_max > 0, precision HJR_FP64 or HJR_FP32 and no warm start k. */
    int32_t local_updates;  /* 0 (default) or 1: update locally (the direction Sec. VII proposes for
                               local changes of the environment), exactly.  The grid is cut into
                               blocks of 1024 consecutive nodes; a step recomputes a block only if
                               a block within its stencils' reach over one step (3 nodes per stage
                               with WENO5, 1 with upwind, in every dimension) changed in the
                               previous step, or if the step size, the discount or the phase just
                               changed.  Otherwise the step would reproduce the block bit for bit,
                               so results are identical to a full update; only the time differs.
                               Costs 16 bytes per block and a dependency list per block (built
                               on the host); where a list would be too long (high dimensions with
                               WENO5) the solve runs without it. */
    double discount;        /* 0 (default) or 1: none.  In (0, 1): discounted reachability (Sec. II-C):
                               each step ends with V <- min(l, discount * V_step), V_step the
                               result of the time integrator, which makes the step a contraction
                               whatever the start; once the change falls below the threshold (or
                               stalls), the factor is annealed to 1 and the solve goes on as
                               usual.  Applies to the first phase (rounded to FP32 there when
                               the precision is HJR_FP32 or HJR_FP32_POLISH64); the FP64 polish is
                               never discounted.  Not with brs. */
} hjr_options;

typedef struct {
    int64_t iterations;         /* time steps of the first phase (FP32, or FP64 for HJR_FP64) */
    int64_t polish_iterations;  /* FP64 polish time steps */
    int64_t intervals;          /* completed report intervals (interval mode) */
    double t_final;             /* backward time marched */
    double last_delta;          /* last change tested against the threshold */
    double dt;                  /* nominal CFL time step */
    double max_abs_l;           /* max |l| over the grid */
    double seconds;             /* wall-clock time of the device work */
    int32_t converged;          /* 1 converged, 0 max_iter reached, 2 horizon reached,
                                   3 stalled: the change stopped decreasing above tol */
    int32_t pad;
    int64_t discounted_iterations;  /* steps of the first phase taken with a discount < 1 */
    int64_t node_updates;   /* grid points advanced one step, summed over all steps: steps x nodes,
                               or fewer with local_updates (the blocks each step computed) */
} hjr_result;

/* Library information and defaults. */
int32_t hjr_abi_version(void);
/* Identity of this build: a hash of the library's sources and compiler flags, fixed at compile
 * time (a NUL-terminated string owned by the library).  Lets a caller check that a prebuilt
 * library matches the sources it was shipped with. */
const char *hjr_build_id(void);
hjr_status hjr_default_options(hjr_options *opts);
const char *hjr_status_string(hjr_status status);
const char *hjr_last_error(void);
/* Number of visible devices (0 when no GPU is usable). */
int32_t hjr_device_count(void);

/* Synchronous solve with host arrays.  l: prod(n) doubles; k: prod(n) doubles or NULL (cold
 * start); V_out: prod(n) doubles written on success or HJR_NOT_CONVERGED / HJR_HORIZON. */
hjr_status hjr_solve(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l,
                     const double *k, const hjr_options *opts, double *V_out, hjr_result *result);

/* Same, with device arrays (l_dev, k_dev nullable, V_dev) on the current device.  Work is
 * issued on `stream` (a hipStream_t, NULL = a stream the library owns); returns when done. */
hjr_status hjr_solve_device(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l_dev,
                            const double *k_dev, const hjr_options *opts, double *V_dev,
                            void *stream, hjr_result *result);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): hjr_solve_device without any allocation.  Same
 * arguments, semantics and results (bitwise) as hjr_solve_device.  Every device buffer the
 * solve needs (its FP32 and FP64 working arrays, tables, state and tile lists) is taken from a
 * static 64 MiB block that each GPU holds from the library's load until the process ends, so
 * no hipMalloc, hipFree, pinned host allocation, event, graph or stream is created; the caller
 * still provides l_dev, k_dev and V_dev.  Limit: about 2 million grid points with TVD-RK3 and
 * the FP64 polish (32 bytes per point), about 3 million with Euler; larger problems return
 * HJR_ERR_BUDGET before any device work.  The block is shared by all calls on one GPU: calls
 * from several host threads on the same GPU are serialised (one waits for the other), and
 * nothing left in it by an earlier call is relied on.  No autotuning and no kernel profile run
 * on this path (the tuner's earlier choices still apply).  `stream`: a hipStream_t, or NULL for
 * the null stream. */
hjr_status hjr_solve_device_noalloc(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l_dev,
                                    const double *k_dev, const hjr_options *opts, double *V_dev,
                                    void *stream, hjr_result *result);

/* Reach-avoid solve (the reach-avoid problems that Sec. II names beside reach and avoid): a
 * constraint function g (prod(n) doubles, finite, same layout as l) marks where the state may
 * not go (g > 0).  Every step ends with V <- max(g, min(l, V_step)) and the start is
 * max(g, l), or max(g, min(k, l)) with a warm start.  With HJR_REACH, {V <= 0} is the set of
 * states that can reach {l <= 0} while keeping g <= 0 on the way, whatever the disturbance.
 * Every option applies as in hjr_solve except brs (refused).  The library keeps an FP32 copy of
 * g in FP32 phases (4 more bytes per node).  g NULL is HJR_ERR_INVALID_ARG.  The device variant
 * takes device arrays on `stream` as hjr_solve_device does. */
hjr_status hjr_solve_reach_avoid(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l,
                                 const double *g, const double *k, const hjr_options *opts,
                                 double *V_out, hjr_result *result);
hjr_status hjr_solve_reach_avoid_device(const hjr_grid *grid, const hjr_dynamics *dyn,
                                        const double *l_dev, const double *g_dev,
                                        const double *k_dev, const hjr_options *opts,
                                        double *V_dev, void *stream, hjr_result *result);

/* Local updates (hjr_options.local_updates): the block dependency lists the solver builds for a
 * grid and a reach (grid steps per dimension: 9 for WENO5 + TVD-RK3, 3 for WENO5 + Euler or
 * upwind + TVD-RK3, 1 for upwind + Euler).  Blocks are 1024 consecutive nodes of the flattened
 * grid (last dimension fastest); block b depends on dep[off[b] .. off[b+1]-1], a sorted list that
 * holds every block with a node within `reach` steps of one of b's nodes (wrapping in periodic
 * dimensions).  Host arrays: off needs nblocks + 1 entries, dep ndeps; pass NULL for both to
 * learn the sizes first.  HJR_ERR_UNSUPPORTED when the lists would be too long to be worth it
 * (a local-updates solve of that grid then updates every block). */
hjr_status hjr_local_dependencies(const hjr_grid *grid, int32_t reach, int64_t *nblocks, int64_t *ndeps,
                                  uint32_t *off, uint32_t *dep);

/* Batched solve: `count` independent problems (host arrays) advanced together, every stage of
 * every instance in one launch per stage.  Each problem's status and result are filled in; the
 * return value is HJR_OK if every problem converged, else the first non-OK status. */
typedef struct {
    hjr_grid grid;
    hjr_dynamics dyn;
    hjr_options opts;
    const double *l;
    const double *k;       /* NULL: cold */
    double *V_out;
    hjr_result result;     /* out */
    hjr_status status;     /* out */
    int32_t pad;
} hjr_problem;
hjr_status hjr_batch_solve(int32_t count, hjr_problem *problems);

/* Kernel-level entry points (device arrays, element type FP32 when precision == HJR_FP32, else
 * FP64).  They run exactly the kernels the solvers run (the stage kernel specialised to the
 * model and scheme, with the nodes-per-thread the autotuner chose for this size class in this
 * process, else 4).
 *   hjr_cfl_dt: dt = cfl / max_x sum_i alpha_i(x)/dx_i (1 when that maximum is 0), capped by
 *     dt_max > 0; computed by a device reduction.
 *   hjr_stage_device: one time-integrator stage at every node.  Vs is the field the stencil is
 *     applied to, Vn the field at the start of the step, l the target function, out the result:
 *       Euler (stage 1 only): out = min(l, Vs + dt L(Vs))
 *       TVD-RK3 stage 1: out = Vn + dt L(Vn) (Vs must equal Vn)
 *               stage 2: out = 3/4 Vn + 1/4 (Vs + dt L(Vs))
 *               stage 3: out = min(l, 1/3 Vn + 2/3 (Vs + dt L(Vs)))
 *     If delta_out is not NULL and the stage ends the step, *delta_out = max |out - Vn|.
 *     out must not alias Vs. */
hjr_status hjr_cfl_dt(const hjr_grid *grid, const hjr_dynamics *dyn, double cfl, double dt_max,
                      double *dt_out);
hjr_status hjr_stage_device(const hjr_grid *grid, const hjr_dynamics *dyn, int32_t game,
                            int32_t spatial, int32_t temporal, int32_t stage, int32_t precision,
                            double dt, const void *Vs, const void *Vn, const void *l, void *out,
                            double *delta_out, void *stream);

/* Kernel timing: while enabled (process-wide), the solvers launch every stage kernel with a
 * pair of HIP events that the launch itself stamps with the kernel's start and end (so gaps in
 * the stream are not counted) and accumulate the durations; hjr_profile_read returns the totals
 * since the last reset.  `launches` counts kernel launches (one per model/scheme group and
 * stage); `nodes` counts grid nodes covered by their tile lists (including nodes of instances
 * that had already finished).  `working_launches` and `working_ms` count only the launches of
 * steps that at least one instance of the launch's group was still taking (in the other launches
 * every workgroup returns at once, after convergence); roofline figures use these. */
typedef struct {
    int64_t launches;
    int64_t nodes;
    double ms;
    int64_t working_launches;
    double working_ms;
} hjr_kernel_time;
typedef struct {
    hjr_kernel_time stage32[3];   /* FP32 stage kernels, by RK stage (Euler uses [0]) */
    hjr_kernel_time stage64[3];   /* FP64 stage kernels */
} hjr_profile;
hjr_status hjr_profile_enable(int32_t on);
hjr_status hjr_profile_read(hjr_profile *out, int32_t reset);

/* Launch plan (host only, touches no device): the tiles the plane-march kernels take for one
 * grid under launch configuration `config`, in launch order (workgroup t takes tile t and runs
 * on XCD t mod 8).  config: -1 whole dim-0 lines; -2, -4, -8 runs of that many planes; -16 the
 * brick variant (6-D grids whose periodic dims among dims 1..3 have even lengths).  Tile t goes
 * to out[5t .. 5t+4]: its first column (flat index within a dim-0 plane), first plane, number of
 * planes, number of columns (0: a padding tile that does nothing), and number of rows (1; 8 for a
 * brick, whose rows are 2k, 2k+1 along each of dims 1..3 from the first column's row, those
 * beyond a dim's end left out).  Writes at most `cap` tiles (out may be NULL when cap is 0);
 * returns the number of tiles, or a negative hjr_status (HJR_ERR_INVALID_ARG for a bad grid or
 * configuration). */
int64_t hjr_march_plan(const hjr_grid *grid, int32_t config, int64_t *out, int64_t cap);

/* ---------------------------------------------------------------------------------------------
 * Safe control (Sec. II-B.2, eq. (uOpt)): online, the system applies
 * u*(x) = argmax_u min_d <grad V(x), f(x, u, d)> with V the converged value function (avoid game;
 * argmin_u max_d for the reach game).  Two calls on device arrays, both asynchronous on `stream`
 * (NULL: the null stream), neither allocating nor synchronising; the caller owns every array
 * and must keep it alive until the stream has run the call.
 * ------------------------------------------------------------------------------------------- */

/* Number of control inputs of a model: 1 (double integrator: u), 1 (Dubins car: turn rate),
 * 2 (unicycle: turn rate, acceleration), 3 (quadrotor: theta, phi, T), 1 (near-hover
 * horizontal subsystem: S), 1 (near-hover vertical subsystem: T); 0 for an unknown id. */
int32_t hjr_num_controls(int32_t dyn_id);

/* Query table of a value function: for V (FP64 device array, C order, grid->n nodes) writes
 * table (FP64 device array, npts x (ndim + 1), node-major): table[node * (ndim + 1) + d] =
 * (D-_d V + D+_d V) / 2 for d < ndim, with the solver's one-sided derivatives (spatial =
 * HJR_UPWIND1 or HJR_WENO5, the same edge rule), and table[node * (ndim + 1) + ndim] = V at the
 * node.  One record per node, so a query reads one contiguous record per cell corner.
 * Errors: HJR_ERR_INVALID_ARG (bad grid or scheme, NULL array), HJR_ERR_UNSUPPORTED (2^29
 * nodes or more), HJR_ERR_DEVICE (launch failure). */
hjr_status hjr_gradient_device(const hjr_grid *grid, int32_t spatial, const double *V, double *table,
                               void *stream);

/* Safe-control queries for nq states x (FP64 device array, nq x ndim, row-major).  For each
 * state, p = grad V(x) and V(x) by multilinear interpolation of `table` (from
 * hjr_gradient_device) over the grid cell holding x (a non-periodic coordinate is clamped into
 * [lo, hi], a periodic one reduced into one period), and u*(x) in closed form: each control
 * takes the bound that the sign of its coefficient in <p, f> selects (the upper bound when the
 * coefficient is zero).  Outputs (FP64 device arrays): u (nq x hjr_num_controls), p (nq x ndim;
 * may be NULL) and v (nq; may be NULL).  A state with a non-finite coordinate gets NaN in every
 * output.  nq = 0 does nothing.  Errors: HJR_ERR_INVALID_ARG (bad grid, model or game, nq < 0 or
 * above 2^38, NULL table, x or u), HJR_ERR_DEVICE (launch failure). */
hjr_status hjr_safe_control_device(const hjr_grid *grid, const hjr_dynamics *dyn, int32_t game,
                                   const double *table, const double *x, int64_t nq, double *u,
                                   double *p, double *v, void *stream);

/* Serving context: requests with device arrays are admitted while their working memory fits
 * `hbm_budget_bytes` (0 = 90% of free device memory) and advance together, in the same batched
 * launches, with requests already running; a request that arrives while others run joins at the
 * next step boundary.  A worker thread owned by the context drives the device. */
typedef struct hjr_ctx hjr_ctx;
hjr_status hjr_ctx_create(int32_t device, size_t hbm_budget_bytes, hjr_ctx **out);
hjr_status hjr_submit(hjr_ctx *ctx, const hjr_grid *grid, const hjr_dynamics *dyn,
                      const double *l_dev, const double *k_dev, const hjr_options *opts,
                      double *V_dev, int64_t *ticket);
/* HJR_PENDING while running; otherwise the request's final status (and result).  A finished
 * ticket is forgotten after it has been polled once. */
hjr_status hjr_poll(hjr_ctx *ctx, int64_t ticket, hjr_result *result);
/* Block until every submitted request has finished. */
hjr_status hjr_ctx_drain(hjr_ctx *ctx);
/* Counters: requests admitted/finished, peak bytes in use, batched steps launched. */
typedef struct {
    int64_t admitted, finished, queued, running;
    int64_t bytes_in_use, bytes_peak, budget;
    int64_t chunks, launches;
} hjr_ctx_stats;
hjr_status hjr_ctx_get_stats(hjr_ctx *ctx, hjr_ctx_stats *stats);
hjr_status hjr_ctx_destroy(hjr_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* HJR_H */
