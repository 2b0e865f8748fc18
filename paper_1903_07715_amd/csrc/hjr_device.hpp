// hjr_device.hpp -- device-side data structures and per-node arithmetic of the HJI VI update.
//
// Layout of one solve instance on the device (all arrays dense, C order, last dim contiguous):
//   FP32 phase : V (current iterate), A (RK stage 1 / Euler ping-pong), B (RK stage 2), l32
//   FP64 phase : V64, A64, B64, l64 (l64 and V64 may be caller memory)
//   tables     : node coordinates per dim and cos/sin of the heading dim, FP32 and FP64 copies
//   state      : SolveState (time, step counter, convergence flag, max-change accumulator)
// A stage kernel reads the stencil field S and the step-start field Vn and writes O:
//   Euler : S = cur, O = other (ping-pong by state parity), O = min(l, S + dt L(S))
//   RK3   : stage 0: S = V -> A; stage 1: S = A, Vn = V -> B; stage 2: S = B, Vn = V -> V
//           (in place: every node reads only its own V, so the overwrite is race-free).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hjr {

constexpr int kMaxDim = 6;
constexpr int kBlock = 256;        // threads per workgroup = nodes per tile

enum : int { kDynDI = 1, kDynDubins = 2, kDynUnicycle = 3, kDynQuad = 4 };
enum : int { kUpwind1 = 1, kWeno5 = 5 };
enum : int { kEuler = 1, kRK3 = 3 };

// state->done codes
enum : int { kRunning = 0, kConverged = 1, kMaxIter = 2, kHorizon = 3, kNonFinite = 4, kStalled = 5 };

struct SolveState {
    double t;            // backward time marched (all phases)
    double t_int;        // time since the start of the current report interval
    double dt_nom;       // CFL step
    double dt_cur;       // step used by the next step (cut at t_max / interval ends)
    double tol;          // threshold of the current phase
    double tol_final;    // FP64 threshold
    double tol32_req;    // requested FP32 threshold (0 = automatic)
    double t_max;
    double dt_report;
    double dt_max;
    double cfl;
    double last_delta;
    double max_abs_l;
    unsigned long long delta_bits;   // max |V^{n+1} - V^n| as FP64 bits (non-negative => ordered)
    unsigned long long idelta_bits;  // max change across the current interval
    unsigned long long rate_bits;    // max_x sum alpha_i/dx_i (CFL reduction)
    unsigned long long lmax_bits;    // max |l|
    double best_delta;    // smallest change seen in this phase (stall detection)
    long long n_best;     // step at which best_delta last dropped by 1%
    long long stall_window;  // > 0: stop the phase after this many steps without such a drop
    long long n;          // steps in the current phase
    long long max_iter;
    long long intervals;
    unsigned int nonfinite;
    int done;
    int parity;           // Euler ping-pong: 0 => current iterate in V, 1 => in A
    int conv_mode;        // 0 per step, 1 per interval
    int check_interval;   // the step just taken closed a report interval
    int phase;            // 0 first phase, 1 FP64 polish
};

// Division by a runtime constant: q = (x * mul) >> (32 + shift), exact for 0 <= x < 2^31.
struct FastDiv {
    uint32_t mul;
    uint32_t shift;
    uint32_t d;
};

__host__ __device__ inline uint32_t fdiv(uint32_t x, const FastDiv &f)
{
#ifdef __HIP_DEVICE_COMPILE__
    return __umulhi(x, f.mul) >> f.shift;
#else
    return (uint32_t)(((uint64_t)x * f.mul) >> 32) >> f.shift;
#endif
}

// Everything a kernel needs to know about one instance.  Built on the host, copied to device
// memory once per change of the active set, read with uniform (scalar) loads.
struct Inst {
    int ndim;
    int dyn;
    int spatial;
    int temporal;
    int game;
    int nstages;
    uint32_t npts;
    uint32_t periodic;
    int n[kMaxDim];
    uint32_t stride[kMaxDim];
    FastDiv div[kMaxDim];
    float inv_dx32[kMaxDim];
    double inv_dx64[kMaxDim];
    float c32[8];        // model constants (see make_constants on the host)
    double c64[8];
    int coord_off[kMaxDim];  // offset of each dim's coordinate table in tab32/tab64
    int trig_off;            // offset of cos table (sin follows); -1 if unused
    const float *tab32;
    const double *tab64;
    // fields
    float *V32, *A32, *B32;
    const float *l32;
    double *V64, *A64, *B64;
    const double *l64;
    float *Vs32;             // interval-mode snapshot (FP32 phase)
    double *Vs64;            // interval-mode snapshot (FP64 phase)
    SolveState *state;
};

struct Tile {
    int inst;
    uint32_t start;
};

template <typename T> struct Fields;
template <> struct Fields<float> {
    __device__ static float *V(const Inst &I) { return I.V32; }
    __device__ static float *A(const Inst &I) { return I.A32; }
    __device__ static float *B(const Inst &I) { return I.B32; }
    __device__ static const float *l(const Inst &I) { return I.l32; }
    __device__ static float *snap(const Inst &I) { return I.Vs32; }
    __device__ static float inv_dx(const Inst &I, int d) { return I.inv_dx32[d]; }
    __device__ static float c(const Inst &I, int k) { return I.c32[k]; }
    __device__ static const float *tab(const Inst &I) { return I.tab32; }
};
template <> struct Fields<double> {
    __device__ static double *V(const Inst &I) { return I.V64; }
    __device__ static double *A(const Inst &I) { return I.A64; }
    __device__ static double *B(const Inst &I) { return I.B64; }
    __device__ static const double *l(const Inst &I) { return I.l64; }
    __device__ static double *snap(const Inst &I) { return I.Vs64; }
    __device__ static double inv_dx(const Inst &I, int d) { return I.inv_dx64[d]; }
    __device__ static double c(const Inst &I, int k) { return I.c64[k]; }
    __device__ static const double *tab(const Inst &I) { return I.tab64; }
};

__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip(double x) { return 1.0 / x; }

// ---------------------------------------------------------------------------------------------
// WENO5 one-sided derivative from five first differences (Jiang-Peng smoothness indicators,
// ideal weights 0.1/0.6/0.3, eps = 1e-6 max v^2 + 1e-18).  The weights a_k = g_k / (S_k + eps)^2
// are normalised without forming them: with t_k = S_k/eps + 1 in [1, 3.4e7], the ratio
// a_k / sum a equals b_k / sum b for b_k = g_k prod_{j != k} t_j^2, which stays inside the FP32
// range and needs a single reciprocal per derivative.
// ---------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T weno5(T v1, T v2, T v3, T v4, T v5)
{
    const T c13_12 = T(13.0 / 12.0);
    T phi1 = v1 * T(1.0 / 3.0) - v2 * T(7.0 / 6.0) + v3 * T(11.0 / 6.0);
    T phi2 = -v2 * T(1.0 / 6.0) + v3 * T(5.0 / 6.0) + v4 * T(1.0 / 3.0);
    T phi3 = v3 * T(1.0 / 3.0) + v4 * T(5.0 / 6.0) - v5 * T(1.0 / 6.0);
    T q1 = v1 - T(2) * v2 + v3;
    T q2 = v2 - T(2) * v3 + v4;
    T q3 = v3 - T(2) * v4 + v5;
    T r1 = v1 - T(4) * v2 + T(3) * v3;
    T r2 = v2 - v4;
    T r3 = T(3) * v3 - T(4) * v4 + v5;
    T S1 = c13_12 * q1 * q1 + T(0.25) * r1 * r1;
    T S2 = c13_12 * q2 * q2 + T(0.25) * r2 * r2;
    T S3 = c13_12 * q3 * q3 + T(0.25) * r3 * r3;
    T m = fmax(fmax(fmax(v1 * v1, v2 * v2), fmax(v3 * v3, v4 * v4)), v5 * v5);
    T eps = T(1e-6) * m + T(1e-18);
    T ie = recip(eps);
    T t1 = S1 * ie + T(1);
    T t2 = S2 * ie + T(1);
    T t3 = S3 * ie + T(1);
    T s1 = t1 * t1, s2 = t2 * t2, s3 = t3 * t3;
    T b1 = T(0.1) * (s2 * s3);
    T b2 = T(0.6) * (s1 * s3);
    T b3 = T(0.3) * (s1 * s2);
    return (b1 * phi1 + b2 * phi2 + b3 * phi3) * recip(b1 + b2 + b3);
}

// First differences along one dim around node j, with the edge rule applied:
// d[k] = (S[j+k-2] - S[j+k-3]) / dx for k = 0..5 (WENO5) or k = 0..1 = (j, j+1) (upwind).
// Non-periodic: the difference index m is clamped to [1, n-1] (linear extrapolation).
template <typename T, int SPATIAL>
__device__ __forceinline__ void line_derivs(const T *__restrict__ S, uint32_t node, int j, int n,
                                            uint32_t stride, bool periodic, T inv_dx, T &dm, T &dp)
{
    constexpr int H = SPATIAL == kWeno5 ? 3 : 1;  // half width of the value stencil
    T u[2 * H + 1];
#pragma unroll
    for (int o = -H; o <= H; ++o) {
        int jj = j + o;
        if (periodic) {
            jj += jj < 0 ? n : 0;
            jj -= jj >= n ? n : 0;
        } else {
            jj = jj < 0 ? 0 : (jj > n - 1 ? n - 1 : jj);
        }
        u[o + H] = S[node + (int)((jj - j) * (int)stride)];
    }
    // raw differences r[o] = u[o] - u[o-1] for o = -H+1 .. H
    T r[2 * H];
#pragma unroll
    for (int o = -H + 1; o <= H; ++o) r[o + H - 1] = u[o + H] - u[o + H - 1];
    if (!periodic) {
        const int lo = 1 - j, hi = n - 1 - j;  // valid difference offsets
        T rlo = r[0], rhi = r[2 * H - 1];
#pragma unroll
        for (int o = -H + 1; o <= H; ++o) {
            rlo = (o == lo) ? r[o + H - 1] : rlo;
            rhi = (o == hi) ? r[o + H - 1] : rhi;
        }
#pragma unroll
        for (int o = -H + 1; o <= H; ++o) {
            T v = r[o + H - 1];
            v = (o < lo) ? rlo : v;
            v = (o > hi) ? rhi : v;
            r[o + H - 1] = v;
        }
    }
#pragma unroll
    for (int k = 0; k < 2 * H; ++k) r[k] *= inv_dx;
    if constexpr (SPATIAL == kWeno5) {
        // r[k] is the difference at offset k-2 (k = 0..5): D- uses offsets -2..2, D+ 3..-1
        dm = weno5<T>(r[0], r[1], r[2], r[3], r[4]);
        dp = weno5<T>(r[5], r[4], r[3], r[2], r[1]);
    } else {
        dm = r[0];
        dp = r[1];
    }
}

// ---------------------------------------------------------------------------------------------
// Hamiltonians H(x, p) = max_u min_d <p, f> (avoid) or min_u max_d (reach), in closed form, and
// alpha_i(x) = max |f_i|.  Model constants c[] (host make_constants):
//   DI      : c0 = |b| ubar, c1 = dbar
//   Dubins  : c0 = v, c1 = ubar, c2 = dbar1, c3 = dbar2
//   Unicycle: c0 = ubar1, c1 = ubar2, c2 = dbar, c3 = shape (0 disk, 1 box)
//   Quad    : c0 = g tan(theta_max), c1 = g tan(phi_max), c2 = Tmax/m - g, c3 = Tmin/m - g,
//             c4..c6 = dbar_x..z, c7 = max(|c2|, |c3|)
// sgn = +1 for the avoid game, -1 for reach: control terms enter as +sgn*|.|, disturbance
// terms as -sgn*|.|.
// ---------------------------------------------------------------------------------------------
template <typename T, int DYN>
__device__ __forceinline__ T hamiltonian(const Inst &I, const T *__restrict__ tab, const int *idx,
                                         const T *p, T *alpha, T sgn)
{
    using F = Fields<T>;
    if constexpr (DYN == kDynDI) {
        T x2 = tab[I.coord_off[1] + idx[1]];
        T cu = F::c(I, 0), dd = F::c(I, 1);
        alpha[0] = fabs(x2) + dd;
        alpha[1] = cu;
        return p[0] * x2 + sgn * (cu * fabs(p[1]) - dd * fabs(p[0]));
    } else if constexpr (DYN == kDynDubins) {
        T cs = tab[I.trig_off + idx[2]];
        T sn = tab[I.trig_off + I.n[2] + idx[2]];
        T v = F::c(I, 0), ub = F::c(I, 1), d1 = F::c(I, 2), d2 = F::c(I, 3);
        alpha[0] = fabs(v * cs) + d1;
        alpha[1] = fabs(v * sn) + d2;
        alpha[2] = ub;
        return v * (p[0] * cs + p[1] * sn) + sgn * (ub * fabs(p[2]) - d1 * fabs(p[0]) - d2 * fabs(p[1]));
    } else if constexpr (DYN == kDynUnicycle) {
        T cs = tab[I.trig_off + idx[2]];
        T sn = tab[I.trig_off + I.n[2] + idx[2]];
        T v = tab[I.coord_off[3] + idx[3]];
        T u1 = F::c(I, 0), u2 = F::c(I, 1), dd = F::c(I, 2);
        alpha[0] = fabs(v * cs) + dd;
        alpha[1] = fabs(v * sn) + dd;
        alpha[2] = u1;
        alpha[3] = u2;
        T dist = F::c(I, 3) != T(0) ? dd * (fabs(p[0]) + fabs(p[1])) : dd * sqrt(p[0] * p[0] + p[1] * p[1]);
        return v * (p[0] * cs + p[1] * sn) + sgn * (u1 * fabs(p[2]) + u2 * fabs(p[3]) - dist);
    } else {
        T vx = tab[I.coord_off[3] + idx[3]];
        T vy = tab[I.coord_off[4] + idx[4]];
        T vz = tab[I.coord_off[5] + idx[5]];
        T ax = F::c(I, 0), ay = F::c(I, 1), tmax = F::c(I, 2), tmin = F::c(I, 3);
        T dx = F::c(I, 4), dy = F::c(I, 5), dz = F::c(I, 6);
        alpha[0] = fabs(vx);
        alpha[1] = fabs(vy);
        alpha[2] = fabs(vz);
        alpha[3] = ax + dx;
        alpha[4] = ay + dy;
        alpha[5] = F::c(I, 7) + dz;
        // thrust: the control picks Tmax or Tmin by the sign of p_vz (avoid: maximise)
        T pz = p[5];
        T thrust = (sgn * pz > T(0)) ? pz * tmax : pz * tmin;
        return p[0] * vx + p[1] * vy + p[2] * vz + thrust +
               sgn * (ax * fabs(p[3]) + ay * fabs(p[4]) - dx * fabs(p[3]) - dy * fabs(p[4]) - dz * fabs(pz));
    }
}

template <int DYN> struct DynDim;
template <> struct DynDim<kDynDI> { static constexpr int value = 2; };
template <> struct DynDim<kDynDubins> { static constexpr int value = 3; };
template <> struct DynDim<kDynUnicycle> { static constexpr int value = 4; };
template <> struct DynDim<kDynQuad> { static constexpr int value = 6; };

template <int NDIM>
__device__ __forceinline__ void unflatten(const Inst &I, uint32_t node, int *idx)
{
    uint32_t rem = node;
#pragma unroll
    for (int d = NDIM - 1; d >= 1; --d) {
        uint32_t q = fdiv(rem, I.div[d]);
        idx[d] = (int)(rem - q * (uint32_t)I.n[d]);
        rem = q;
    }
    idx[0] = (int)rem;
}

// L(S) at one node.
template <typename T, int DYN, int SPATIAL>
__device__ __forceinline__ T lf_operator(const Inst &I, const T *__restrict__ S, uint32_t node)
{
    constexpr int N = DynDim<DYN>::value;
    using F = Fields<T>;
    int idx[N];
    unflatten<N>(I, node, idx);
    T p[N], diff[N], alpha[N];
#pragma unroll
    for (int d = 0; d < N; ++d) {
        T dm, dp;
        line_derivs<T, SPATIAL>(S, node, idx[d], I.n[d], I.stride[d], (I.periodic >> d) & 1u,
                                F::inv_dx(I, d), dm, dp);
        p[d] = T(0.5) * (dm + dp);
        diff[d] = T(0.5) * (dp - dm);
    }
    const T sgn = I.game == 0 ? T(1) : T(-1);
    T L = hamiltonian<T, DYN>(I, F::tab(I), idx, p, alpha, sgn);
#pragma unroll
    for (int d = 0; d < N; ++d) L += alpha[d] * diff[d];
    return L;
}

// sum_i alpha_i(x) / dx_i at one node, in FP64 (for the CFL reduction).
template <int DYN>
__device__ __forceinline__ double cfl_rate(const Inst &I, uint32_t node)
{
    constexpr int N = DynDim<DYN>::value;
    int idx[N];
    unflatten<N>(I, node, idx);
    double p[N], alpha[N];
#pragma unroll
    for (int d = 0; d < N; ++d) p[d] = 0.0;
    (void)hamiltonian<double, DYN>(I, I.tab64, idx, p, alpha, 1.0);
    double r = 0.0;
#pragma unroll
    for (int d = 0; d < N; ++d) r += alpha[d] * I.inv_dx64[d];
    return r;
}

}  // namespace hjr
