/*
 * hjr_oracle.h -- interface of the plain FP64 CPU reference solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this code.  The GPU library neither includes this header nor links this code,
 * and this code includes nothing from the GPU library.
 *
 * The method is the grid solution of the infinite-horizon avoid problem of Herbert, Ghosh,
 * Bansal and Tomlin, "Reachability-Based Safety Guarantees using Efficient Initializations":
 * the HJI variational inequality of Sec. II-B.2, eq. (7), marched backwards in time from V = l
 * (standard, eqs. (11)-(12)) or from a warm-start function k (eqs. (13)-(14)) until the value
 * function stops changing (Sec. IV, first paragraph).
 */
#ifndef HJR_ORACLE_H
#define HJR_ORACLE_H

#include <stdint.h>

#define OR_MAXD 6

/* Uniform Cartesian grid, row-major (C order: the last dimension is contiguous).
 * Non-periodic dim i: n[i] nodes, both ends are nodes, dx = (hi-lo)/(n-1).
 * Periodic dim i (bit i of `periodic`): n[i] nodes, hi excluded, dx = (hi-lo)/n. */
typedef struct {
    int32_t ndim;
    int32_t n[OR_MAXD];
    double lo[OR_MAXD];
    double hi[OR_MAXD];
    uint32_t periodic;
} or_grid;

/* Dynamics ids and parameter layouts (state order in brackets):
 *  1 double integrator [x1, x2]: x1' = x2 + d, x2' = b u; |u| <= ubar, |d| <= dbar.
 *      params = {ubar, b, dbar}                       (Sec. II-A, eq. (2))
 *  2 Dubins car [x, y, theta]: x' = v cos(theta) + d1, y' = v sin(theta) + d2, theta' = u;
 *      |u| <= ubar, |d1| <= dbar1, |d2| <= dbar2.  params = {v, ubar, dbar1, dbar2}
 *  3 unicycle [x, y, theta, v]: x' = v cos(theta) + d1, y' = v sin(theta) + d2,
 *      theta' = u1, v' = u2; |u1| <= ubar1, |u2| <= ubar2; (d1, d2) in a Euclidean ball of
 *      radius dbar (shape 0) or the box |d_i| <= dbar (shape 1).
 *      params = {ubar1, ubar2, dbar, shape}
 *  4 planar-attitude quadrotor [px, py, pz, vx, vy, vz]: p' = v, vx' = g tan(theta) + dx,
 *      vy' = -g tan(phi) + dy, vz' = T/m - g + dz; |theta| <= theta_max, |phi| <= phi_max,
 *      T in [Tmin, Tmax], |d_i| <= dbar_i.
 *      params = {g, m, phi_max, theta_max, Tmin, Tmax, dbar_x, dbar_y, dbar_z}
 *  5 near-hover quadrotor of Sec. VI (eq. (Quad10D_dyn)), one horizontal subsystem
 *      [p, v, theta, omega]: p' = v + d, v' = g tan(theta), theta' = -d1 theta + omega,
 *      omega' = -d0 theta + n0 S; |S| <= S_max, |d| <= dbar.
 *      params = {g, d0, d1, n0, S_max, dbar}
 *  6 near-hover quadrotor, vertical subsystem [p_z, v_z]: p_z' = v_z + d, v_z' = (k_T/m) T - g;
 *      T in [T_min, T_max], |d| <= dbar.   params = {g, k_T, m, T_min, T_max, dbar}           */
typedef struct {
    int32_t id;
    int32_t n_params;
    double p[16];
} or_dyn;

enum { OR_AVOID = 0, OR_REACH = 1 };
enum { OR_UPWIND1 = 1, OR_WENO5 = 5 };
enum { OR_EULER = 1, OR_RK3 = 3 };
enum { OR_CONV_STEP = 0, OR_CONV_INTERVAL = 1 };

typedef struct {
    int32_t game;           /* OR_AVOID: control maximises, disturbance minimises (eq. (6)) */
    int32_t spatial;        /* OR_UPWIND1 | OR_WENO5 */
    int32_t temporal;       /* OR_EULER | OR_RK3 */
    int32_t conv_mode;      /* OR_CONV_STEP | OR_CONV_INTERVAL */
    int32_t min_each_stage; /* 0: project onto V <= l after the full step only */
    int32_t brs;            /* 1: no projection at all (the backward reachable set of Sec. II,
                               i.e. the HJ PDE of eq. (5) without the min with l of eq. (7)) */
    double cfl;
    double tol;
    double dt_report;       /* interval length in OR_CONV_INTERVAL mode */
    double t_max;           /* 0: infinite horizon */
    double dt_max;          /* 0: no cap (a zero flow field uses dt = 1) */
    int64_t max_iter;
    double discount;        /* discounted reachability (Sec. II-C): in (0, 1) every step ends with
                               min(l, discount * V_step); or_solve anneals it to 1 once the change
                               falls below tol.  0 or 1: none */
} or_opts;

typedef struct {
    int64_t steps;          /* time steps taken */
    int64_t intervals;      /* completed report intervals (interval mode) */
    double t;               /* accumulated backward time */
    double last_delta;      /* last max-norm change that was tested against tol */
    double dt;              /* nominal CFL time step */
    int32_t converged;      /* 1 converged, 0 max_iter hit, 2 horizon t_max reached */
    int32_t pad;
    int64_t discounted_steps;  /* steps taken before the discount was annealed to 1 */
} or_result;

/* All functions return 0 on success and a negative value on bad arguments. */
int or_hamiltonian(const or_dyn *dyn, int game, const double *x, const double *p,
                   double *H, double *alpha);
int or_flow(const or_dyn *dyn, const double *x, const double *u, const double *d, double *f);
double or_weno5(double v1, double v2, double v3, double v4, double v5);
int or_derivatives(const or_grid *g, int spatial, const double *V, int64_t node, int dim,
                   double *dminus, double *dplus);
int or_operator(const or_grid *g, const or_dyn *dyn, int game, int spatial, const double *V,
                double *L);
int or_operator_at(const or_grid *g, const or_dyn *dyn, int game, int spatial, const double *V,
                   const int64_t *nodes, int64_t count, double *L);
int or_stage_at(const or_grid *g, const or_dyn *dyn, const or_opts *o, int stage, double dt,
                const double *Vs, const double *Vn, const double *l, const int64_t *nodes,
                int64_t count, double *out);
double or_cfl_dt(const or_grid *g, const or_dyn *dyn, double cfl, double dt_max);
int or_step(const or_grid *g, const or_dyn *dyn, const or_opts *o, const double *l,
            const double *V, double dt, double *Vout, double *delta);
int or_solve(const or_grid *g, const or_dyn *dyn, const double *l, const double *k,
             const or_opts *o, double *V, or_result *res);
/* Reach-avoid variants: gc is a constraint function (the state must keep gc <= 0); each step
 * ends with max(gc, min(l, V_step)) and the start is max(gc, min(k, l)).  gc NULL: as above. */
int or_step_ra(const or_grid *g, const or_dyn *dyn, const or_opts *o, const double *l,
               const double *gc, const double *V, double dt, double *Vout, double *delta);
int or_solve_ra(const or_grid *g, const or_dyn *dyn, const double *l, const double *gc,
                const double *k, const or_opts *o, double *V, or_result *res);
int or_threads(void);

/* Safe control (Sec. II-B.2, eq. (uOpt)).  or_num_controls: number of control inputs of a model
 * (1, 1, 2, 3, 1, 1 for ids 1-6; -1 otherwise).  or_gradient_at: p = (D- + D+)/2 at a node.
 * or_interp_at: p and V at a state x by multilinear interpolation of the nodal values over x's
 * cell (non-periodic coordinates clamped into [lo, hi], periodic ones wrapped).
 * or_optimal_control: u* = argmax_u min_d <p, f> (avoid) / argmin_u max_d (reach) by
 * enumerating the corners of the control box; on ties the later corner wins.
 * or_safe_control: both for nq states (x: nq x ndim; u: nq x nu; p: nq x ndim; v: nq); a state
 * with a non-finite coordinate gets NaN in every output (or_interp_at rejects it). */
int or_num_controls(int id);
int or_gradient_at(const or_grid *g, int spatial, const double *V, int64_t node, double *p);
int or_interp_at(const or_grid *g, int spatial, const double *V, const double *x, double *p,
                 double *v);
int or_optimal_control(const or_dyn *dyn, int game, const double *x, const double *p, double *u);
int or_safe_control(const or_grid *g, const or_dyn *dyn, int game, int spatial, const double *V,
                    const double *x, int64_t nq, double *u, double *p, double *v);

#endif
