/*
 * hjr_oracle.c -- plain FP64 CPU reference for the HJI variational-inequality grid update.
 *
 * TEST INFRASTRUCTURE ONLY: it checks the GPU library and is never called by it.  It is written
 * for reading, not for speed: one node at a time, every quantity straight from its definition,
 * no blocking, no fusion, no reuse between neighbouring nodes.  Build with -ffp-contract=off so
 * every operation is a single IEEE round-to-nearest operation.
 *
 * Source: Herbert, Ghosh, Bansal, Tomlin, "Reachability-Based Safety Guarantees using Efficient
 * Initializations".  The paper fixes the continuous problem -- the dynamics (eq. (1)), the target
 * function l (Sec. II-B.1), the Hamiltonian max_u min_d <grad V, f> (eq. (6)), the variational
 * inequality min{D_t V + H, l - V} = 0 (eq. (7)), the standard initial value V(x,0) = l
 * (eq. (12)), the warm initial value k whose effective form is min(k, l) (proof of Theorem 1,
 * case b) and the stopping rule "largest change of V over one step is below a threshold"
 * (Sec. IV).  It leaves the discretisation to a level-set toolbox, so the discrete scheme below
 * is the standard one for this equation, with every choice the paper is silent on stated where
 * it is made:
 *   - derivatives: first-order one-sided differences, or fifth-order WENO (Jiang and Peng),
 *   - numerical Hamiltonian: Lax-Friedrichs with per-node dissipation alpha_i(x) = max |f_i|,
 *   - time: forward Euler or the three-stage TVD Runge-Kutta scheme of Shu and Osher,
 *   - the projection V <- min(l, V) after every full step,
 *   - time step dt = cfl / max_x sum_i alpha_i(x)/dx_i.
 * Time runs backwards (s = -t >= 0), so eq. (5) becomes dV/ds = H and one step adds dt * L(V).
 */
#include "hjr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------------ */
/* Grid                                                                                        */
/* ------------------------------------------------------------------------------------------ */

static int is_periodic(const or_grid *g, int d) { return (int)((g->periodic >> d) & 1u); }

static double grid_dx(const or_grid *g, int d)
{
    if (is_periodic(g, d)) return (g->hi[d] - g->lo[d]) / (double)g->n[d];
    return (g->hi[d] - g->lo[d]) / (double)(g->n[d] - 1);
}

static double grid_coord(const or_grid *g, int d, int j) { return g->lo[d] + (double)j * grid_dx(g, d); }

static int64_t grid_points(const or_grid *g)
{
    int64_t N = 1;
    for (int d = 0; d < g->ndim; ++d) N *= g->n[d];
    return N;
}

static int64_t grid_stride(const or_grid *g, int d)
{
    int64_t s = 1;
    for (int e = g->ndim - 1; e > d; --e) s *= g->n[e];
    return s;
}

static void unflatten(const or_grid *g, int64_t node, int *idx)
{
    for (int d = g->ndim - 1; d >= 0; --d) {
        idx[d] = (int)(node % g->n[d]);
        node /= g->n[d];
    }
}

static int grid_ok(const or_grid *g)
{
    if (!g || g->ndim < 1 || g->ndim > OR_MAXD) return 0;
    for (int d = 0; d < g->ndim; ++d) {
        if (g->n[d] < 2 || !(g->hi[d] > g->lo[d])) return 0;
        if (is_periodic(g, d) && g->n[d] < 3) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------------------------ */
/* Dynamics f(x, u, d), eq. (1), and the Hamiltonian of eq. (6)                               */
/* ------------------------------------------------------------------------------------------ */

static int dyn_ndim(int id)
{
    switch (id) {
    case 1: return 2;
    case 2: return 3;
    case 3: return 4;
    case 4: return 6;
    case 5: return 4;
    case 6: return 2;
    default: return -1;
    }
}

static int dyn_nparams(int id)
{
    switch (id) {
    case 1: return 3;
    case 2: return 4;
    case 3: return 4;
    case 4: return 9;
    case 5: return 6;
    case 6: return 6;
    default: return -1;
    }
}

/* The flow field written out exactly as the model equations read. */
int or_flow(const or_dyn *dyn, const double *x, const double *u, const double *d, double *f)
{
    const double *q = dyn->p;
    switch (dyn->id) {
    case 1: /* double integrator, eq. (2): p' = v + d, v' = b u */
        f[0] = x[1] + d[0];
        f[1] = q[1] * u[0];
        return 0;
    case 2: /* Dubins car */
        f[0] = q[0] * cos(x[2]) + d[0];
        f[1] = q[0] * sin(x[2]) + d[1];
        f[2] = u[0];
        return 0;
    case 3: /* unicycle with speed as a state */
        f[0] = x[3] * cos(x[2]) + d[0];
        f[1] = x[3] * sin(x[2]) + d[1];
        f[2] = u[0];
        f[3] = u[1];
        return 0;
    case 4: /* quadrotor translation: u = (theta, phi, T) */
        f[0] = x[3];
        f[1] = x[4];
        f[2] = x[5];
        f[3] = q[0] * tan(u[0]) + d[0];
        f[4] = -q[0] * tan(u[1]) + d[1];
        f[5] = u[2] / q[1] - q[0] + d[2];
        return 0;
    case 5: /* near-hover quadrotor (Sec. VI, eq. (Quad10D_dyn)), one horizontal subsystem:
             * (p, v, theta, omega), u = S, q = {g, d0, d1, n0, S_max, dbar} */
        f[0] = x[1] + d[0];
        f[1] = q[0] * tan(x[2]);
        f[2] = -q[2] * x[2] + x[3];
        f[3] = -q[1] * x[2] + q[3] * u[0];
        return 0;
    case 6: /* near-hover quadrotor, vertical subsystem: (p_z, v_z), u = T_z,
             * q = {g, k_T, m, T_min, T_max, dbar_z} */
        f[0] = x[1] + d[0];
        f[1] = q[1] / q[2] * u[0] - q[0];
        return 0;
    default:
        return -1;
    }
}

/* Corners of the control box.  Every model above is affine in each control input, or (for the
 * quadrotor angles) monotone in it, so max_u and min_u of <p, f> over the box are attained at a
 * corner. */
static int control_corners(const or_dyn *dyn, double u[][3])
{
    const double *q = dyn->p;
    switch (dyn->id) {
    case 1:
        u[0][0] = -q[0];
        u[1][0] = q[0];
        return 2;
    case 2:
        u[0][0] = -q[1];
        u[1][0] = q[1];
        return 2;
    case 3: {
        int c = 0;
        for (int a = -1; a <= 1; a += 2)
            for (int b = -1; b <= 1; b += 2) {
                u[c][0] = a * q[0];
                u[c][1] = b * q[1];
                ++c;
            }
        return c;
    }
    case 4: {
        int c = 0;
        for (int a = -1; a <= 1; a += 2)
            for (int b = -1; b <= 1; b += 2)
                for (int t = 0; t < 2; ++t) {
                    u[c][0] = a * q[3];          /* theta */
                    u[c][1] = b * q[2];          /* phi   */
                    u[c][2] = t ? q[5] : q[4];   /* T     */
                    ++c;
                }
        return c;
    }
    case 5:
        u[0][0] = -q[4];
        u[1][0] = q[4];
        return 2;
    case 6:
        u[0][0] = q[3];
        u[1][0] = q[4];
        return 2;
    default:
        return 0;
    }
}

/* Corners of the disturbance box (all models enter d additively and affinely). */
static int disturbance_corners(const or_dyn *dyn, double d[][3])
{
    const double *q = dyn->p;
    switch (dyn->id) {
    case 1:
        d[0][0] = -q[2];
        d[1][0] = q[2];
        return 2;
    case 5:
    case 6:
        d[0][0] = -q[5];
        d[1][0] = q[5];
        return 2;
    case 2:
    case 3: {
        double b1 = q[2];                       /* Dubins dbar1; unicycle box dbar */
        double b2 = dyn->id == 2 ? q[3] : q[2]; /* Dubins dbar2; unicycle box dbar */
        int c = 0;
        for (int a = -1; a <= 1; a += 2)
            for (int b = -1; b <= 1; b += 2) {
                d[c][0] = a * b1;
                d[c][1] = b * b2;
                ++c;
            }
        return c;
    }
    case 4: {
        int c = 0;
        for (int a = -1; a <= 1; a += 2)
            for (int b = -1; b <= 1; b += 2)
                for (int e = -1; e <= 1; e += 2) {
                    d[c][0] = a * q[6];
                    d[c][1] = b * q[7];
                    d[c][2] = e * q[8];
                    ++c;
                }
        return c;
    }
    default:
        return 0;
    }
}

static int ball_disturbance(const or_dyn *dyn) { return dyn->id == 3 && dyn->p[3] == 0.0; }

/* H(x, p) = max_u min_d <p, f(x,u,d)> for the avoid game (eq. (6)); min_u max_d for the reach
 * game.  alpha_i(x) = max over (u, d) of |f_i(x,u,d)|, the Lax-Friedrichs dissipation
 * coefficient (a bound on |dH/dp_i| for every p).
 *
 * Box sets: both extrema of an affine (or monotone) function over a box are at corners, so the
 * corners are enumerated.  Ball disturbance (unicycle, shape 0): d enters x' and y' additively,
 * so <p, f(x,u,d)> = <p, f(x,u,0)> + p1 d1 + p2 d2, and by Cauchy-Schwarz the extrema of
 * p1 d1 + p2 d2 over |d| <= r are -/+ r |(p1, p2)|; the maximisers of |f_1| and |f_2| over the
 * ball are the axis points (+-r, 0) and (0, +-r), which are enumerated for alpha. */
int or_hamiltonian(const or_dyn *dyn, int game, const double *x, const double *p, double *H,
                   double *alpha)
{
    int nd = dyn_ndim(dyn->id);
    if (nd < 0) return -1;
    double U[8][3], D[8][3];
    memset(U, 0, sizeof U);
    memset(D, 0, sizeof D);
    int nu = control_corners(dyn, U);
    int ball = ball_disturbance(dyn);
    int ndist;
    if (ball) {
        double r = dyn->p[2];
        double axis[4][2] = {{r, 0.0}, {-r, 0.0}, {0.0, r}, {0.0, -r}};
        for (int c = 0; c < 4; ++c) {
            D[c][0] = axis[c][0];
            D[c][1] = axis[c][1];
        }
        ndist = 4;
    } else {
        ndist = disturbance_corners(dyn, D);
    }
    double f[OR_MAXD];
    double zero[3] = {0.0, 0.0, 0.0};

    if (H) {
        double best = game == OR_AVOID ? -INFINITY : INFINITY;
        for (int a = 0; a < nu; ++a) {
            double inner;
            if (ball) {
                or_flow(dyn, x, U[a], zero, f);
                double s = 0.0;
                for (int i = 0; i < nd; ++i) s += p[i] * f[i];
                double pn = sqrt(p[0] * p[0] + p[1] * p[1]);
                inner = game == OR_AVOID ? s - dyn->p[2] * pn : s + dyn->p[2] * pn;
            } else {
                inner = game == OR_AVOID ? INFINITY : -INFINITY;
                for (int b = 0; b < ndist; ++b) {
                    or_flow(dyn, x, U[a], D[b], f);
                    double s = 0.0;
                    for (int i = 0; i < nd; ++i) s += p[i] * f[i];
                    if (game == OR_AVOID) inner = s < inner ? s : inner;
                    else inner = s > inner ? s : inner;
                }
            }
            if (game == OR_AVOID) best = inner > best ? inner : best;
            else best = inner < best ? inner : best;
        }
        *H = best;
    }
    if (alpha) {
        for (int i = 0; i < nd; ++i) alpha[i] = 0.0;
        for (int a = 0; a < nu; ++a)
            for (int b = 0; b < ndist; ++b) {
                or_flow(dyn, x, U[a], D[b], f);
                for (int i = 0; i < nd; ++i) {
                    double m = fabs(f[i]);
                    if (m > alpha[i]) alpha[i] = m;
                }
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Spatial derivatives                                                                         */
/* ------------------------------------------------------------------------------------------ */

/* Fifth-order WENO approximation of a one-sided derivative from five consecutive first
 * differences v1..v5 (Jiang and Peng 2000; Osher and Fedkiw 2003, Sec. 3.4): three third-order
 * candidates, weighted by smoothness indicators, with ideal weights 0.1, 0.6, 0.3 and
 * eps = 1e-6 * max(v_k^2) + 1e-18. */
double or_weno5(double v1, double v2, double v3, double v4, double v5)
{
    double phi1 = v1 / 3.0 - 7.0 * v2 / 6.0 + 11.0 * v3 / 6.0;
    double phi2 = -v2 / 6.0 + 5.0 * v3 / 6.0 + v4 / 3.0;
    double phi3 = v3 / 3.0 + 5.0 * v4 / 6.0 - v5 / 6.0;

    double S1 = 13.0 / 12.0 * (v1 - 2.0 * v2 + v3) * (v1 - 2.0 * v2 + v3)
              + 0.25 * (v1 - 4.0 * v2 + 3.0 * v3) * (v1 - 4.0 * v2 + 3.0 * v3);
    double S2 = 13.0 / 12.0 * (v2 - 2.0 * v3 + v4) * (v2 - 2.0 * v3 + v4)
              + 0.25 * (v2 - v4) * (v2 - v4);
    double S3 = 13.0 / 12.0 * (v3 - 2.0 * v4 + v5) * (v3 - 2.0 * v4 + v5)
              + 0.25 * (3.0 * v3 - 4.0 * v4 + v5) * (3.0 * v3 - 4.0 * v4 + v5);

    double m = v1 * v1;
    if (v2 * v2 > m) m = v2 * v2;
    if (v3 * v3 > m) m = v3 * v3;
    if (v4 * v4 > m) m = v4 * v4;
    if (v5 * v5 > m) m = v5 * v5;
    double eps = 1e-6 * m + 1e-18;

    double a1 = 0.1 / ((S1 + eps) * (S1 + eps));
    double a2 = 0.6 / ((S2 + eps) * (S2 + eps));
    double a3 = 0.3 / ((S3 + eps) * (S3 + eps));
    double sum = a1 + a2 + a3;
    return (a1 / sum) * phi1 + (a2 / sum) * phi2 + (a3 / sum) * phi3;
}

/* Value of V at node position j + o along dimension `dim` of the line through `node`.
 * Periodic dims wrap around.  Non-periodic dims use ghost nodes filled by linear extrapolation
 * of the two nearest grid nodes: V_{-m} = V_0 + m (V_0 - V_1) and
 * V_{n-1+m} = V_{n-1} + m (V_{n-1} - V_{n-2}). */
static double line_value(const or_grid *g, const double *V, int64_t line_base, int dim, int j, int o)
{
    int n = g->n[dim];
    int64_t s = grid_stride(g, dim);
    int m = j + o;
    if (is_periodic(g, dim)) {
        int w = ((m % n) + n) % n;
        return V[line_base + (int64_t)w * s];
    }
    if (m < 0) {
        double v0 = V[line_base], v1 = V[line_base + s];
        return v0 + (double)(-m) * (v0 - v1);
    }
    if (m > n - 1) {
        double vn = V[line_base + (int64_t)(n - 1) * s], vm = V[line_base + (int64_t)(n - 2) * s];
        return vn + (double)(m - (n - 1)) * (vn - vm);
    }
    return V[line_base + (int64_t)m * s];
}

/* Left and right derivative approximations D-V and D+V at `node` along `dim`. */
int or_derivatives(const or_grid *g, int spatial, const double *V, int64_t node, int dim,
                   double *dminus, double *dplus)
{
    int idx[OR_MAXD];
    unflatten(g, node, idx);
    int j = idx[dim];
    int64_t base = node - (int64_t)j * grid_stride(g, dim);
    double dx = grid_dx(g, dim);
    if (spatial == OR_UPWIND1) {
        double um = line_value(g, V, base, dim, j, -1);
        double u0 = line_value(g, V, base, dim, j, 0);
        double up = line_value(g, V, base, dim, j, 1);
        *dminus = (u0 - um) / dx;
        *dplus = (up - u0) / dx;
        return 0;
    }
    if (spatial == OR_WENO5) {
        /* first differences D_m = (V_m - V_{m-1}) / dx for m = j-2 .. j+3 */
        double D[6];
        for (int o = -2; o <= 3; ++o)
            D[o + 2] = (line_value(g, V, base, dim, j, o) - line_value(g, V, base, dim, j, o - 1)) / dx;
        /* D-: differences at j-2..j+2; D+: at j+3..j-1, i.e. the mirrored stencil */
        *dminus = or_weno5(D[0], D[1], D[2], D[3], D[4]);
        *dplus = or_weno5(D[5], D[4], D[3], D[2], D[1]);
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------------------------------ */
/* Lax-Friedrichs operator L(V) = H(x, (D- + D+)/2) + sum_i alpha_i (D+_i - D-_i) / 2         */
/* ------------------------------------------------------------------------------------------ */

static double lf_at(const or_grid *g, const or_dyn *dyn, int game, int spatial, const double *V,
                    int64_t node)
{
    int idx[OR_MAXD];
    unflatten(g, node, idx);
    double x[OR_MAXD], p[OR_MAXD], diff[OR_MAXD], alpha[OR_MAXD];
    for (int d = 0; d < g->ndim; ++d) {
        double dm, dp;
        or_derivatives(g, spatial, V, node, d, &dm, &dp);
        x[d] = grid_coord(g, d, idx[d]);
        p[d] = 0.5 * (dm + dp);
        diff[d] = 0.5 * (dp - dm);
    }
    double H;
    or_hamiltonian(dyn, game, x, p, &H, alpha);
    double L = H;
    for (int d = 0; d < g->ndim; ++d) L += alpha[d] * diff[d];
    return L;
}

static int problem_ok(const or_grid *g, const or_dyn *dyn, int spatial)
{
    if (!grid_ok(g) || !dyn) return 0;
    if (dyn_ndim(dyn->id) != g->ndim || dyn->n_params != dyn_nparams(dyn->id)) return 0;
    if (spatial != OR_UPWIND1 && spatial != OR_WENO5) return 0;
    return 1;
}

int or_operator(const or_grid *g, const or_dyn *dyn, int game, int spatial, const double *V,
                double *L)
{
    if (!problem_ok(g, dyn, spatial)) return -1;
    int64_t N = grid_points(g);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) L[i] = lf_at(g, dyn, game, spatial, V, i);
    return 0;
}

int or_operator_at(const or_grid *g, const or_dyn *dyn, int game, int spatial, const double *V,
                   const int64_t *nodes, int64_t count, double *L)
{
    if (!problem_ok(g, dyn, spatial)) return -1;
    int64_t N = grid_points(g);
    for (int64_t c = 0; c < count; ++c)
        if (nodes[c] < 0 || nodes[c] >= N) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < count; ++c) L[c] = lf_at(g, dyn, game, spatial, V, nodes[c]);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Time step                                                                                   */
/* ------------------------------------------------------------------------------------------ */

/* dt = cfl / max_x sum_i alpha_i(x) / dx_i.  alpha does not depend on V, so dt is fixed for a
 * solve.  A flow field that vanishes everywhere gives dt = 1; dt_max > 0 caps dt. */
double or_cfl_dt(const or_grid *g, const or_dyn *dyn, double cfl, double dt_max)
{
    if (!problem_ok(g, dyn, OR_UPWIND1)) return -1.0;
    int64_t N = grid_points(g);
    double rate = 0.0;
#pragma omp parallel for reduction(max : rate) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int idx[OR_MAXD];
        unflatten(g, i, idx);
        double x[OR_MAXD], alpha[OR_MAXD];
        for (int d = 0; d < g->ndim; ++d) x[d] = grid_coord(g, d, idx[d]);
        or_hamiltonian(dyn, OR_AVOID, x, x, NULL, alpha);
        double r = 0.0;
        for (int d = 0; d < g->ndim; ++d) r += alpha[d] / grid_dx(g, d);
        if (r > rate) rate = r;
    }
    double dt = rate > 0.0 ? cfl / rate : 1.0;
    if (dt_max > 0.0 && dt > dt_max) dt = dt_max;
    return dt;
}

/* One stage of the time integrator at one node.  Vs is the field the stencil is applied to,
 * Vn the field at the start of the step.
 *   Euler        : out = min(l, Vs + dt L(Vs))                      (Vs = Vn)
 *   TVD-RK3 (Shu and Osher), stage 1: V1 = Vn + dt L(Vn)
 *                          stage 2: V2 = 3/4 Vn + 1/4 (V1 + dt L(V1))
 *                          stage 3: out = min(l, 1/3 Vn + 2/3 (V2 + dt L(V2)))
 * With min_each_stage the projection onto V <= l is also applied after stages 1 and 2; with brs
 * it is never applied.  With a discount factor gamma in (0, 1) (discounted reachability,
 * Sec. II-C: the value one step later enters the dynamic programming principle multiplied by the
 * per-step factor, the target term not) the value of the full step is multiplied by gamma before
 * the projection.  With a constraint function gc (reach-avoid: the state must also stay where
 * gc <= 0) the full step ends with max(gc, .) after the projection. */
static double stage_value(const or_grid *g, const or_dyn *dyn, const or_opts *o, int stage,
                          double dt, const double *Vs, const double *Vn, const double *l,
                          const double *gc, int64_t i)
{
    double L = lf_at(g, dyn, o->game, o->spatial, Vs, i);
    double gamma = (o->discount > 0.0 && o->discount < 1.0) ? o->discount : 1.0;
    double v;
    if (o->temporal == OR_EULER) {
        v = gamma * (Vs[i] + dt * L);
        if (!o->brs && l[i] < v) v = l[i];
        return (gc && gc[i] > v) ? gc[i] : v;
    }
    if (stage == 1) {
        v = Vs[i] + dt * L;
        if (o->min_each_stage && l[i] < v) v = l[i];
        return v;
    }
    if (stage == 2) {
        v = 0.75 * Vn[i] + 0.25 * (Vs[i] + dt * L);
        if (o->min_each_stage && l[i] < v) v = l[i];
        return v;
    }
    v = gamma * (Vn[i] / 3.0 + 2.0 / 3.0 * (Vs[i] + dt * L));
    if (!o->brs && l[i] < v) v = l[i];
    return (gc && gc[i] > v) ? gc[i] : v;
}

static int opts_ok(const or_opts *o)
{
    if (!o) return 0;
    if (o->spatial != OR_UPWIND1 && o->spatial != OR_WENO5) return 0;
    if (o->temporal != OR_EULER && o->temporal != OR_RK3) return 0;
    if (o->game != OR_AVOID && o->game != OR_REACH) return 0;
    return 1;
}

int or_stage_at(const or_grid *g, const or_dyn *dyn, const or_opts *o, int stage, double dt,
                const double *Vs, const double *Vn, const double *l, const int64_t *nodes,
                int64_t count, double *out)
{
    if (!problem_ok(g, dyn, o ? o->spatial : 0) || !opts_ok(o)) return -1;
    if (stage < 1 || stage > (o->temporal == OR_RK3 ? 3 : 1)) return -1;
    int64_t N = grid_points(g);
    for (int64_t c = 0; c < count; ++c)
        if (nodes[c] < 0 || nodes[c] >= N) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < count; ++c)
        out[c] = stage_value(g, dyn, o, stage, dt, Vs, Vn, l, NULL, nodes[c]);
    return 0;
}

/* One full time step V -> Vout = min(l, step(V)) (then max(gc, .) when gc is given), and
 * delta = max_x |Vout - V|. */
int or_step_ra(const or_grid *g, const or_dyn *dyn, const or_opts *o, const double *l,
               const double *gc, const double *V, double dt, double *Vout, double *delta)
{
    if (!problem_ok(g, dyn, o ? o->spatial : 0) || !opts_ok(o)) return -1;
    int64_t N = grid_points(g);
    if (o->temporal == OR_EULER) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) Vout[i] = stage_value(g, dyn, o, 1, dt, V, V, l, gc, i);
    } else {
        double *V1 = (double *)malloc(sizeof(double) * (size_t)N);
        double *V2 = (double *)malloc(sizeof(double) * (size_t)N);
        if (!V1 || !V2) {
            free(V1);
            free(V2);
            return -2;
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) V1[i] = stage_value(g, dyn, o, 1, dt, V, V, l, gc, i);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) V2[i] = stage_value(g, dyn, o, 2, dt, V1, V, l, gc, i);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) Vout[i] = stage_value(g, dyn, o, 3, dt, V2, V, l, gc, i);
        free(V1);
        free(V2);
    }
    double m = 0.0;
#pragma omp parallel for reduction(max : m) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double c = fabs(Vout[i] - V[i]);
        if (c > m) m = c;
    }
    *delta = m;
    return 0;
}

int or_step(const or_grid *g, const or_dyn *dyn, const or_opts *o, const double *l,
            const double *V, double dt, double *Vout, double *delta)
{
    return or_step_ra(g, dyn, o, l, NULL, V, dt, Vout, delta);
}

/* ------------------------------------------------------------------------------------------ */
/* Solve: march the variational inequality backwards in time until V stops changing           */
/* ------------------------------------------------------------------------------------------ */

/* V0 = l (standard, eq. (12)) or min(k, l) (warm start; the proof of Theorem 1, case b, shows
 * the warm solve behaves as if started from min(k, l)).  Each iteration takes one time step.
 * Per-step mode stops when max |V^{n+1} - V^n| < tol.  Interval mode (the rule of Sec. IV)
 * takes CFL steps whose sizes are cut so that they end exactly on multiples of dt_report and
 * stops when the largest change of V across one whole interval is below tol.  Both modes also
 * stop at max_iter steps or when t reaches t_max (t_max > 0).  Discounted reachability (a
 * discount in (0, 1)) runs the same loop with the discounted step; the first time the test
 * passes, the discount is set to 1 (annealed) and the loop goes on instead of stopping.
 * Reach-avoid (gc given): V0 = max(gc, l) or max(gc, min(k, l)), and every step ends with
 * max(gc, .); the set {V <= 0} is then the set of states that can reach {l <= 0} while keeping
 * gc <= 0 on the way. */
int or_solve_ra(const or_grid *g, const or_dyn *dyn, const double *l, const double *gc,
                const double *k, const or_opts *o, double *V, or_result *res)
{
    if (!problem_ok(g, dyn, o ? o->spatial : 0) || !opts_ok(o) || !(o->cfl > 0.0) ||
        !(o->tol > 0.0) || !res)
        return -1;
    if (o->conv_mode == OR_CONV_INTERVAL && !(o->dt_report > 0.0)) return -1;
    or_opts cur = *o;  /* its discount drops to 1 at the anneal */
    int discounted = o->discount > 0.0 && o->discount < 1.0;
    int64_t disc_steps = 0;
    int64_t N = grid_points(g);
    for (int64_t i = 0; i < N; ++i) {
        if (!isfinite(l[i]) || (k && !isfinite(k[i])) || (gc && !isfinite(gc[i]))) return -3;
        V[i] = (k && k[i] < l[i]) ? k[i] : l[i];
        if (gc && gc[i] > V[i]) V[i] = gc[i];
    }
    double *Vnext = (double *)malloc(sizeof(double) * (size_t)N);
    double *Vstart = o->conv_mode == OR_CONV_INTERVAL ? (double *)malloc(sizeof(double) * (size_t)N) : NULL;
    if (!Vnext || (o->conv_mode == OR_CONV_INTERVAL && !Vstart)) {
        free(Vnext);
        free(Vstart);
        return -2;
    }
    if (Vstart) memcpy(Vstart, V, sizeof(double) * (size_t)N);

    double dt_nom = or_cfl_dt(g, dyn, o->cfl, o->dt_max);
    double t = 0.0, t_int = 0.0, last = INFINITY;
    int64_t steps = 0, intervals = 0;
    int converged = 0;
    for (;;) {
        if (o->max_iter > 0 && steps >= o->max_iter) break;
        if (o->t_max > 0.0 && t >= o->t_max * (1.0 - 1e-12)) {
            converged = 2;
            break;
        }
        double dt = dt_nom;
        if (o->t_max > 0.0 && o->t_max - t < dt) dt = o->t_max - t;
        if (o->conv_mode == OR_CONV_INTERVAL && o->dt_report - t_int < dt) dt = o->dt_report - t_int;
        double delta;
        or_step_ra(g, dyn, &cur, l, gc, V, dt, Vnext, &delta);
        memcpy(V, Vnext, sizeof(double) * (size_t)N);
        steps += 1;
        t += dt;
        if (o->conv_mode == OR_CONV_STEP) {
            last = delta;
            if (delta < o->tol) {
                if (discounted) {
                    discounted = 0;
                    disc_steps = steps;
                    cur.discount = 1.0;
                    continue;
                }
                converged = 1;
                break;
            }
        } else {
            t_int += dt;
            if (t_int >= o->dt_report * (1.0 - 1e-12)) {
                double m = 0.0;
                for (int64_t i = 0; i < N; ++i) {
                    double c = fabs(V[i] - Vstart[i]);
                    if (c > m) m = c;
                }
                intervals += 1;
                last = m;
                memcpy(Vstart, V, sizeof(double) * (size_t)N);
                t_int = 0.0;
                if (m < o->tol) {
                    if (discounted) {
                        discounted = 0;
                        disc_steps = steps;
                        cur.discount = 1.0;
                        continue;
                    }
                    converged = 1;
                    break;
                }
            }
        }
    }
    res->steps = steps;
    res->intervals = intervals;
    res->t = t;
    res->last_delta = last;
    res->dt = dt_nom;
    res->converged = converged;
    res->discounted_steps = discounted ? steps : disc_steps;
    free(Vnext);
    free(Vstart);
    return 0;
}

int or_solve(const or_grid *g, const or_dyn *dyn, const double *l, const double *k,
             const or_opts *o, double *V, or_result *res)
{
    return or_solve_ra(g, dyn, l, NULL, k, o, V, res);
}

/* ------------------------------------------------------------------------------------------ */
/* Safe control (Sec. II-B.2, eq. (uOpt)): at a state x, with p the gradient of the converged   */
/* value function there, the safe controller applies u* = argmax_u min_d <p, f(x, u, d)> (avoid */
/* game; argmin_u max_d for the reach game).                                                   */
/* ------------------------------------------------------------------------------------------ */

int or_num_controls(int id)
{
    switch (id) {
    case 1: return 1;
    case 2: return 1;
    case 3: return 2;
    case 4: return 3;
    case 5: return 1;
    case 6: return 1;
    default: return -1;
    }
}

/* Gradient at a grid node: the average (D- + D+)/2 of the solver's one-sided derivatives (the
 * same p the Hamiltonian is evaluated at in the Lax-Friedrichs operator). */
int or_gradient_at(const or_grid *g, int spatial, const double *V, int64_t node, double *p)
{
    for (int d = 0; d < g->ndim; ++d) {
        double dm, dp;
        if (or_derivatives(g, spatial, V, node, d, &dm, &dp) != 0) return -1;
        p[d] = 0.5 * (dm + dp);
    }
    return 0;
}

/* The grid cell holding coordinate x along dim d: lower node j, upper node jn and the weight w
 * of the upper node (linear interpolation).  Non-periodic dims clamp x into [lo, hi]; periodic
 * dims reduce it into one period. */
static void cell_of(const or_grid *g, int d, double x, int *j, int *jn, double *w)
{
    int n = g->n[d];
    double s = (x - g->lo[d]) / grid_dx(g, d);
    if (is_periodic(g, d)) {
        s = s - (double)n * floor(s / (double)n);
        int k = (int)floor(s);
        if (k > n - 1) k = n - 1;
        if (k < 0) k = 0;
        *j = k;
        *jn = k + 1 == n ? 0 : k + 1;
        *w = s - (double)k;
    } else {
        if (s < 0.0) s = 0.0;
        if (s > (double)(n - 1)) s = (double)(n - 1);
        int k = (int)floor(s);
        if (k > n - 2) k = n - 2;
        *j = k;
        *jn = k + 1;
        *w = s - (double)k;
    }
}

/* Multilinear interpolation at x of the nodal gradient (p, ndim values) and of V (*v), over
 * the 2^ndim corners of x's cell; corner c takes the upper node along dim d when bit d of c is
 * set, with weight prod_d (bit ? w_d : 1 - w_d). */
int or_interp_at(const or_grid *g, int spatial, const double *V, const double *x, double *p,
                 double *v)
{
    if (!grid_ok(g)) return -1;
    int nd = g->ndim;
    for (int d = 0; d < nd; ++d)
        if (!isfinite(x[d])) return -1;
    int j[OR_MAXD], jn[OR_MAXD];
    double w[OR_MAXD];
    for (int d = 0; d < nd; ++d) cell_of(g, d, x[d], &j[d], &jn[d], &w[d]);
    for (int d = 0; d < nd; ++d) p[d] = 0.0;
    double acc = 0.0;
    for (int c = 0; c < (1 << nd); ++c) {
        double wt = 1.0;
        int64_t node = 0;
        for (int d = 0; d < nd; ++d) {
            int up = (c >> d) & 1;
            wt *= up ? w[d] : 1.0 - w[d];
            node += (int64_t)(up ? jn[d] : j[d]) * grid_stride(g, d);
        }
        double pc[OR_MAXD];
        if (or_gradient_at(g, spatial, V, node, pc) != 0) return -1;
        for (int d = 0; d < nd; ++d) p[d] += wt * pc[d];
        acc += wt * V[node];
    }
    if (v) *v = acc;
    return 0;
}

/* min over the disturbance set (avoid) or max (reach) of <p, f(x, u, d)> for one control u. */
static double inner_value(const or_dyn *dyn, int game, const double *x, const double *p,
                          const double *u)
{
    int nd = dyn_ndim(dyn->id);
    double f[OR_MAXD];
    double zero[3] = {0.0, 0.0, 0.0};
    if (ball_disturbance(dyn)) {
        or_flow(dyn, x, u, zero, f);
        double s = 0.0;
        for (int i = 0; i < nd; ++i) s += p[i] * f[i];
        double pn = sqrt(p[0] * p[0] + p[1] * p[1]);
        return game == OR_AVOID ? s - dyn->p[2] * pn : s + dyn->p[2] * pn;
    }
    double D[8][3];
    memset(D, 0, sizeof D);
    int ndist = disturbance_corners(dyn, D);
    double best = game == OR_AVOID ? INFINITY : -INFINITY;
    for (int b = 0; b < ndist; ++b) {
        or_flow(dyn, x, u, D[b], f);
        double s = 0.0;
        for (int i = 0; i < nd; ++i) s += p[i] * f[i];
        if (game == OR_AVOID) best = s < best ? s : best;
        else best = s > best ? s : best;
    }
    return best;
}

/* u* at state x for gradient p: the corner of the control box that maximises (avoid) or
 * minimises (reach) the inner value; the objective is affine (or monotone) in each control, so
 * a corner attains the optimum.  Corners are visited in the order of control_corners and a
 * later corner that ties the best so far replaces it, so a control whose coefficient in the
 * objective is zero ends at its upper bound. */
int or_optimal_control(const or_dyn *dyn, int game, const double *x, const double *p, double *u)
{
    int nu = or_num_controls(dyn->id);
    if (nu < 0) return -1;
    double U[8][3];
    memset(U, 0, sizeof U);
    int nc = control_corners(dyn, U);
    int best_c = -1;
    double best = 0.0;
    for (int c = 0; c < nc; ++c) {
        double val = inner_value(dyn, game, x, p, U[c]);
        if (best_c < 0 || (game == OR_AVOID ? val >= best : val <= best)) {
            best = val;
            best_c = c;
        }
    }
    for (int i = 0; i < nu; ++i) u[i] = U[best_c][i];
    return 0;
}

/* The whole query: for each of the nq states x (row-major, nq x ndim) the interpolated
 * gradient p (nq x ndim), value v (nq) and safe control u (nq x nu).  p and v may be NULL. */
int or_safe_control(const or_grid *g, const or_dyn *dyn, int game, int spatial, const double *V,
                    const double *x, int64_t nq, double *u, double *p, double *v)
{
    int nd = dyn_ndim(dyn->id);
    int nu = or_num_controls(dyn->id);
    if (!grid_ok(g) || nd != g->ndim || nu < 0 || nq < 0) return -1;
    if (spatial != OR_UPWIND1 && spatial != OR_WENO5) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t q = 0; q < nq; ++q) {
        double pq[OR_MAXD], vq;
        int finite = 1;
        for (int d = 0; d < nd; ++d) finite &= isfinite(x[q * nd + d]) ? 1 : 0;
        if (!finite) {  /* a state with a non-finite coordinate gets NaN outputs */
            for (int i = 0; i < nu; ++i) u[q * nu + i] = NAN;
            if (p)
                for (int d = 0; d < nd; ++d) p[q * nd + d] = NAN;
            if (v) v[q] = NAN;
            continue;
        }
        if (or_interp_at(g, spatial, V, x + q * nd, pq, &vq) != 0) {
            bad = 1;
            continue;
        }
        if (or_optimal_control(dyn, game, x + q * nd, pq, u + q * nu) != 0) bad = 1;
        if (p)
            for (int d = 0; d < nd; ++d) p[q * nd + d] = pq[d];
        if (v) v[q] = vq;
    }
    return bad ? -1 : 0;
}
