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
constexpr int kBlock = 256;        // threads per workgroup
constexpr int kLocalShift = 10;    // local updates: activity is tracked per block of 2^10 nodes
constexpr int kFusedNpt = 4;       // nodes per thread of the fused (all-model) stage kernel

enum : int { kDynDI = 1, kDynDubins = 2, kDynUnicycle = 3, kDynQuad = 4, kDynQ10XY = 5, kDynQ10Z = 6 };
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
    double gamma;         // discount factor of the current step (1 = none, always after the anneal)
    long long n_disc;     // steps of the first phase taken with gamma < 1 (set at the anneal)
    int epoch;            // steps taken in all phases (local updates: the current step's number)
    int full_epoch;       // local updates: steps up to this epoch compute every block
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
    int brs;              // 1: no projection onto V <= l (backward reachable set)
    int nstages;
    uint32_t npts;
    uint32_t periodic;
    int n[kMaxDim];
    uint32_t stride[kMaxDim];
    FastDiv div[kMaxDim];
    float inv_dx32[kMaxDim];
    double inv_dx64[kMaxDim];
    float hinv_dx32[kMaxDim];    // 1 / (2 dx)
    double hinv_dx64[kMaxDim];
    float eps0_32[kMaxDim];      // WENO5 epsilon floor for undivided differences: 4e-18 dx^2
    double eps0_64[kMaxDim];
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
    const float *g32;        // reach-avoid constraint function (nullptr: none)
    const double *g64;
    int *act;                // local updates (nullptr: off): two arrays of nblocks; act[e & 1][b]
                             // == e marks block b for step e
    uint32_t nblocks;        // node blocks of 2^kLocalShift nodes
    unsigned long long *cnt; // per node block: grid points computed in all steps so far
    const uint32_t *dep_off; // per node block, its range in dep: the blocks within the reach of
    const uint32_t *dep;     // one full step's stencils (itself included)
    float *Vs32;             // interval-mode snapshot (FP32 phase)
    double *Vs64;            // interval-mode snapshot (FP64 phase)
    SolveState *state;
};

// A tile is npt * kBlock consecutive nodes of one instance's flattened grid (npt nodes per
// thread, kBlock apart).
struct Tile {
    int inst;
    uint32_t start;
    int npt;
};

// A march tile: cn <= kBlock consecutive columns (flat positions within a dim-0 plane, starting
// at c0) of one instance, each advanced through the dim-0 planes i0 .. i0 + len - 1 by one
// thread (cn = 0: a padding tile that does nothing).
struct MTile {
    int inst;
    uint32_t c0;
    int i0;
    int len;
    uint32_t cn;
};

template <typename T> struct Fields;
template <> struct Fields<float> {
    __device__ static float *V(const Inst &I) { return I.V32; }
    __device__ static float *A(const Inst &I) { return I.A32; }
    __device__ static float *B(const Inst &I) { return I.B32; }
    __device__ static const float *l(const Inst &I) { return I.l32; }
    __device__ static const float *g(const Inst &I) { return I.g32; }
    __device__ static float *snap(const Inst &I) { return I.Vs32; }
    __device__ static float hinv_dx(const Inst &I, int d) { return I.hinv_dx32[d]; }
    __device__ static float eps0(const Inst &I, int d) { return I.eps0_32[d]; }
    __device__ static float c(const Inst &I, int k) { return I.c32[k]; }
    __device__ static const float *tab(const Inst &I) { return I.tab32; }
};
template <> struct Fields<double> {
    __device__ static double *V(const Inst &I) { return I.V64; }
    __device__ static double *A(const Inst &I) { return I.A64; }
    __device__ static double *B(const Inst &I) { return I.B64; }
    __device__ static const double *l(const Inst &I) { return I.l64; }
    __device__ static const double *g(const Inst &I) { return I.g64; }
    __device__ static double *snap(const Inst &I) { return I.Vs64; }
    __device__ static double hinv_dx(const Inst &I, int d) { return I.hinv_dx64[d]; }
    __device__ static double eps0(const Inst &I, int d) { return I.eps0_64[d]; }
    __device__ static double c(const Inst &I, int k) { return I.c64[k]; }
    __device__ static const double *tab(const Inst &I) { return I.tab64; }
};

__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
// FP64: the hardware reciprocal estimate refined by two Newton steps r <- r + r(1 - x r), each
// of which squares the relative error, so the result is within an ulp of 1/x; this replaces
// the longer scaled IEEE division sequence.  Only used on positive normal arguments.
__device__ inline double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
}

// 2^-floor(log2 x) for a positive normal x, from the exponent bits (no division).
__device__ inline float pow2_recip(float x)
{
    return __uint_as_float(0x7f000000u - (__float_as_uint(x) & 0x7f800000u));
}
__device__ inline double pow2_recip(double x)
{
    return __longlong_as_double((long long)(0x7fe0000000000000ull -
                                            ((unsigned long long)__double_as_longlong(x) & 0x7ff0000000000000ull)));
}

// Loads and stores through the global address space (the field pointers come from device
// memory, so without the cast the compiler would use generic "flat" accesses).  The element
// offset is turned into a 32-bit byte offset (every array is below 4 GiB), so the access is a
// uniform 64-bit base plus one 32-bit per-lane offset.
template <typename T>
__device__ __forceinline__ T ldg(const T *p, uint32_t i)
{
    const uint32_t b = i * (uint32_t)sizeof(T);
    return *(const __attribute__((address_space(1))) T *)((const __attribute__((address_space(1))) char *)p + b);
}
template <typename T>
__device__ __forceinline__ void stg(T *p, uint32_t i, T v)
{
    const uint32_t b = i * (uint32_t)sizeof(T);
    *(__attribute__((address_space(1))) T *)((__attribute__((address_space(1))) char *)p + b) = v;
}

// ---------------------------------------------------------------------------------------------
// WENO5 one-sided derivatives (Jiang-Peng smoothness indicators, ideal weights 0.1/0.6/0.3,
// eps = 1e-6 max v^2 + 1e-18 over the five differences v of the stencil), formed per interface.
// The interface between nodes j and j+1 has the five undivided first differences
// e1..e5 = u(j-1) - u(j-2), ..., u(j+3) - u(j+2).  D- at node j+1 takes v = (e1..e5) and D+ at
// node j the mirrored v = (e5..e1); the mirrored stencil has the same three indicators in reverse
// order (A, B, C over (e1,e2,e3), (e2,e3,e4), (e3,e4,e5)) and the same eps, so everything but
// the candidate values is computed once per interface and serves both derivatives.  Both come
// out multiplied by dx.
// The weights depend only on the ratios of the (S_k + eps), so every S_k and eps may carry one
// common factor: with undivided differences and a factor 4 the indicators are
// S_k = (13/3) c_k^2 + r_k^2 and eps = 4e-6 max e^2 + 4e-18 dx^2 (eps0).  With
// a_k = g_k / (S_k + eps)^2, the normalised combination sum a_k phi_k / sum a_k is formed without
// the a_k: t_k = (S_k + eps) 2^-x (x the exponent of eps) lies in [1, 7e7], and a_k is
// proportional to g_k prod_{i != k} t_i^2, which stays inside the FP32 range; so the interface
// keeps the three pair products of the t_k^2.  The ideal weights are folded in as
// 0.1 : 0.6 : 0.3 = 1 : 6 : 3, with 6 phi_2 and 3 phi_3 formed directly, so one reciprocal
// finishes each derivative.
// ---------------------------------------------------------------------------------------------
template <typename T> struct WenoIf {
    T ab, ac, bc;  // t_A^2 t_B^2, t_A^2 t_C^2, t_B^2 t_C^2
};

// The WENO5 arithmetic below is written with explicit fused multiply-adds and contraction off,
// so its rounding is fixed by the source alone: the flat kernel (both interfaces of every node)
// and the march kernel (each interface once, shared by two nodes) produce the same bits.
// m: the largest of e1^2 .. e5^2 (a maximum is exact, so any grouping gives the same value; the
// flat kernel shares the middle four squares between a node's two interfaces).  The second
// differences and their (13/3) c^2 terms are the same expressions in both interfaces of a node,
// so the flat kernel computes the shared ones once.
template <typename T>
__device__ __forceinline__ WenoIf<T> weno5_interface_m(T e1, T e2, T e3, T e4, T e5, T m, T eps0)
{
#pragma clang fp contract(off)
    const T k = T(13.0 / 3.0);
    const T cA = fma(T(-2), e2, e1) + e3;
    const T cB = fma(T(-2), e3, e2) + e4;
    const T cC = fma(T(-2), e4, e3) + e5;
    const T rA = fma(T(3), e3, fma(T(-4), e2, e1));
    const T rB = e2 - e4;
    const T rC = fma(T(3), e3, fma(T(-4), e4, e5));
    const T SA = fma(rA, rA, (k * cA) * cA);
    const T SB = fma(rB, rB, (k * cB) * cB);
    const T SC = fma(rC, rC, (k * cC) * cC);
    const T eps = fma(T(4e-6), m, eps0);
    const T sc = pow2_recip(eps);
    const T e = eps * sc;
    const T tA = fma(SA, sc, e), tB = fma(SB, sc, e), tC = fma(SC, sc, e);
    const T sA = tA * tA, sB = tB * tB, sC = tC * tC;
    return WenoIf<T>{sA * sB, sA * sC, sB * sC};
}

template <typename T>
__device__ __forceinline__ WenoIf<T> weno5_interface(T e1, T e2, T e3, T e4, T e5, T eps0)
{
#pragma clang fp contract(off)
    const T m = fmax(fmax(fmax(e2 * e2, e3 * e3), e4 * e4), fmax(e1 * e1, e5 * e5));
    return weno5_interface_m(e1, e2, e3, e4, e5, m, eps0);
}

// D- at the node right of the interface: v = (e1..e5), weights 1 : 6 : 3 on A, B, C.
template <typename T>
__device__ __forceinline__ T weno5_left(const WenoIf<T> &w, T e1, T e2, T e3, T e4, T e5)
{
#pragma clang fp contract(off)
    const T f1 = fma(e3, T(11.0 / 6.0), fma(e2, T(-7.0 / 6.0), e1 * T(1.0 / 3.0)));
    const T f6 = fma(T(2), e4, fma(T(5), e3, -e2));
    const T f3 = fma(T(-0.5), e5, fma(T(2.5), e4, e3));
    const T num = fma(w.ab, f3, fma(w.ac, f6, w.bc * f1));
    const T den = fma(T(3), w.ab, fma(T(6), w.ac, w.bc));
    return num * recip(den);
}

// D+ at the node left of the interface: v = (e5..e1), weights 1 : 6 : 3 on C, B, A.
template <typename T>
__device__ __forceinline__ T weno5_right(const WenoIf<T> &w, T e1, T e2, T e3, T e4, T e5)
{
#pragma clang fp contract(off)
    const T f1 = fma(e3, T(11.0 / 6.0), fma(e4, T(-7.0 / 6.0), e5 * T(1.0 / 3.0)));
    const T f6 = fma(T(2), e2, fma(T(5), e3, -e4));
    const T f3 = fma(T(-0.5), e1, fma(T(2.5), e2, e3));
    const T num = fma(w.bc, f3, fma(w.ac, f6, w.ab * f1));
    const T den = fma(T(3), w.bc, fma(T(6), w.ac, w.ab));
    return num * recip(den);
}

// D- and D+ at a node from its six differences d[k] = u(k-2) - u(k-3): D- from the interface on
// its left (d0..d4), D+ from the one on its right (d1..d5).
template <typename T>
__device__ __forceinline__ void weno5_pair(const T *d, T eps0, T &dm, T &dp)
{
#pragma clang fp contract(off)
    const T mid = fmax(fmax(d[1] * d[1], d[2] * d[2]), fmax(d[3] * d[3], d[4] * d[4]));
    const WenoIf<T> wl = weno5_interface_m(d[0], d[1], d[2], d[3], d[4], fmax(mid, d[0] * d[0]), eps0);
    const WenoIf<T> wr = weno5_interface_m(d[1], d[2], d[3], d[4], d[5], fmax(mid, d[5] * d[5]), eps0);
    dm = weno5_left(wl, d[0], d[1], d[2], d[3], d[4]);
    dp = weno5_right(wr, d[1], d[2], d[3], d[4], d[5]);
}

// The Lax-Friedrichs operator's dissipation sum_d alpha_d (D+ - D-)_d / 2 added to the Hamiltonian
// term, and the integrator's stage value from the stage input s, the step-start value vn and the
// operator L (forward Euler, or stage 1, 2, 3 of TVD-RK3 with the discount gm on the step's last
// stage).  The fused multiply-adds are written out, so the rounding is fixed by the source and
// every stage kernel (flat tiles, plane march, brick, WENO5 march) produces the same bits.
template <typename T, int N>
__device__ __forceinline__ T add_dissipation(T L, const T *alpha, const T *diff)
{
#pragma unroll
    for (int d = 0; d < N; ++d) L = fma(alpha[d], diff[d], L);
    return L;
}
template <typename T>
__device__ __forceinline__ T stage_value(bool euler, int stage, T gm, T s, T vn, T dt, T L)
{
#pragma clang fp contract(off)
    const T e = fma(dt, L, s);
    if (euler) return gm * e;
    if (stage == 0) return e;
    if (stage == 1) return fma(T(0.75), vn, T(0.25) * e);
    return gm * fma(vn, T(1.0 / 3.0), T(2.0 / 3.0) * e);
}

// Every lane of a block works on one tile of one instance, so the instance's array pointers are
// wave-uniform.  Saying so (readfirstlane of both halves) puts them in scalar registers, and
// each stencil load then becomes a scalar base plus one shared per-lane byte offset instead of
// a per-lane 64-bit address computation.
template <typename P>
__device__ __forceinline__ P *uniform_ptr(P *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P *)(((uint64_t)hi << 32) | lo);
}

// Stencil values along one dim: u[o + H] = S at line position j + o, o = -H..H (H = 3 for WENO5,
// 1 for upwind); the centre value is shared by every dim and is not loaded here.
// inner: every lane of the wave has j in [H, n - H), so no offset leaves the line and the loads
// use the wave-uniform offsets o * stride.  Otherwise, per lane: on a periodic dim an offset
// past an end wraps once (n >= 2H + 1, so one wrap is enough); on a non-periodic dim a position
// off the line loads the centre instead, because line_derivs replaces every difference that
// involves such a position (any finite in-line value will do).
template <typename T, int SPATIAL>
__device__ __forceinline__ void line_load(const T *__restrict__ S, uint32_t node, int j, int n, uint32_t stride,
                                          bool periodic, bool inner, T *u)
{
    constexpr int H = SPATIAL == kWeno5 ? 3 : 1;
    if (inner) {
#pragma unroll
        for (int o = -H; o <= H; ++o)
            if (o != 0) u[o + H] = ldg(S, node + (uint32_t)(o * (int)stride));
        return;
    }
#pragma unroll
    for (int o = -H; o <= H; ++o) {
        if (o == 0) continue;
        int off;
        if (periodic)
            off = o < 0 ? (j + o < 0 ? o + n : o) : (j + o >= n ? o - n : o);
        else
            off = (o < 0 ? j + o >= 0 : j + o < n) ? o : 0;
        u[o + H] = ldg(S, node + (uint32_t)(off * (int)stride));
    }
}

// Undivided first differences along a line at node j from its stencil values u[0..2H]
// (positions j-H..j+H): r[k] = u[k+1] - u[k] (WENO5: the differences entering at offsets -2..3;
// upwind: 0..1).  On a non-periodic dim a difference beyond an edge equals the nearest interior
// one (linear extrapolation of V), so the differences of a line form one extended sequence
// that does not depend on the node: Delta_m = u(m) - u(m-1) for 1 <= m <= n-1, Delta_1 below,
// Delta_{n-1} above.  Waves whose nodes are all at least H nodes from both ends (inner, a
// per-wave vote, so the branch never diverges) skip that rule.
template <typename T, int SPATIAL>
__device__ __forceinline__ void line_diffs(const T *u, int j, int n, bool periodic, bool inner, T *r)
{
    constexpr int H = SPATIAL == kWeno5 ? 3 : 1;
#pragma unroll
    for (int o = -H + 1; o <= H; ++o) r[o + H - 1] = u[o + H] - u[o + H - 1];
    if constexpr (SPATIAL == kUpwind1) {
        // two differences: at the first node the one before the edge takes the one after it,
        // at the last node the reverse (n >= 3, so both cannot apply)
        if (!periodic && !inner) {
            const T r0 = r[0], r1 = r[1];
            r[0] = j == 0 ? r1 : r0;
            r[1] = j == n - 1 ? r0 : r1;
        }
    } else if (!periodic && !inner) {
        const int lo = 1 - j, hi = n - 1 - j;  // offsets of the first and last valid difference
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
}

// Left and right derivatives D-V, D+V at node j of a line of n nodes from its stencil values,
// both multiplied by dx.
template <typename T, int SPATIAL>
__device__ __forceinline__ void line_derivs(const T *u, int j, int n, bool periodic, bool inner, T eps0, T &dm,
                                            T &dp)
{
    constexpr int H = SPATIAL == kWeno5 ? 3 : 1;
    T r[2 * H];
    line_diffs<T, SPATIAL>(u, j, n, periodic, inner, r);
    if constexpr (SPATIAL == kWeno5) {
        weno5_pair<T>(r, eps0, dm, dp);
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
//   Q10 XY  : c0 = g, c1 = d0, c2 = d1, c3 = n0 S_max, c4 = dbar (near-hover horizontal)
//   Q10 Z   : c0 = (k_T/m) T_max - g, c1 = (k_T/m) T_min - g, c2 = dbar, c3 = max(|c0|, |c1|)
// sgn = +1 for the avoid game, -1 for reach: control terms enter as +sgn*|.|, disturbance
// terms as -sgn*|.|.
// ---------------------------------------------------------------------------------------------
// The per-node values a model's flow takes from the node's coordinates (read from the tables):
// heading cosine and sine, speed or velocity coordinates.  No model's flow depends on the dim-0
// coordinate, so along a dim-0 line these are fixed.
template <typename T> struct HamCoef {
    T a, b, c, d;
};

template <typename T, int DYN>
__device__ __forceinline__ HamCoef<T> ham_coef(const Inst &I, const T *__restrict__ tab, const int *idx)
{
    HamCoef<T> k{};
    if constexpr (DYN == kDynDI) {
        k.a = ldg(tab, I.coord_off[1] + idx[1]);                  // x2
    } else if constexpr (DYN == kDynDubins) {
        k.a = ldg(tab, I.trig_off + idx[2]);                      // cos theta
        k.b = ldg(tab, I.trig_off + I.n[2] + idx[2]);             // sin theta
    } else if constexpr (DYN == kDynUnicycle) {
        k.a = ldg(tab, I.trig_off + idx[2]);
        k.b = ldg(tab, I.trig_off + I.n[2] + idx[2]);
        k.c = ldg(tab, I.coord_off[3] + idx[3]);                  // speed
    } else if constexpr (DYN == kDynQ10XY) {
        k.a = ldg(tab, I.coord_off[1] + idx[1]);                  // v
        k.b = ldg(tab, I.coord_off[2] + idx[2]);                  // theta
        k.c = ldg(tab, I.trig_off + idx[2]);                      // tan theta
        k.d = ldg(tab, I.coord_off[3] + idx[3]);                  // omega
    } else if constexpr (DYN == kDynQ10Z) {
        k.a = ldg(tab, I.coord_off[1] + idx[1]);                  // v_z
    } else {
        k.a = ldg(tab, I.coord_off[3] + idx[3]);                  // v_x, v_y, v_z
        k.b = ldg(tab, I.coord_off[4] + idx[4]);
        k.c = ldg(tab, I.coord_off[5] + idx[5]);
    }
    return k;
}

template <typename T, int DYN>
__device__ __forceinline__ T ham_eval(const Inst &I, const HamCoef<T> &k, const T *p, T *alpha, T sgn)
{
    using F = Fields<T>;
    if constexpr (DYN == kDynDI) {
        T x2 = k.a;
        T cu = F::c(I, 0), dd = F::c(I, 1);
        alpha[0] = fabs(x2) + dd;
        alpha[1] = cu;
        return p[0] * x2 + sgn * (cu * fabs(p[1]) - dd * fabs(p[0]));
    } else if constexpr (DYN == kDynDubins) {
        T cs = k.a, sn = k.b;
        T v = F::c(I, 0), ub = F::c(I, 1), d1 = F::c(I, 2), d2 = F::c(I, 3);
        alpha[0] = fabs(v * cs) + d1;
        alpha[1] = fabs(v * sn) + d2;
        alpha[2] = ub;
        return v * (p[0] * cs + p[1] * sn) + sgn * (ub * fabs(p[2]) - d1 * fabs(p[0]) - d2 * fabs(p[1]));
    } else if constexpr (DYN == kDynUnicycle) {
        T cs = k.a, sn = k.b, v = k.c;
        T u1 = F::c(I, 0), u2 = F::c(I, 1), dd = F::c(I, 2);
        alpha[0] = fabs(v * cs) + dd;
        alpha[1] = fabs(v * sn) + dd;
        alpha[2] = u1;
        alpha[3] = u2;
        T dist = F::c(I, 3) != T(0) ? dd * (fabs(p[0]) + fabs(p[1])) : dd * sqrt(p[0] * p[0] + p[1] * p[1]);
        return v * (p[0] * cs + p[1] * sn) + sgn * (u1 * fabs(p[2]) + u2 * fabs(p[3]) - dist);
    } else if constexpr (DYN == kDynQ10XY) {
        // c0 = g, c1 = d0, c2 = d1, c3 = n0 S_max, c4 = dbar; the table holds tan(theta)
        T v = k.a, th = k.b, tn = k.c, om = k.d;
        T f1 = F::c(I, 0) * tn, f2 = om - F::c(I, 2) * th, f3 = -F::c(I, 1) * th;
        T ns = F::c(I, 3), dd = F::c(I, 4);
        alpha[0] = fabs(v) + dd;
        alpha[1] = fabs(f1);
        alpha[2] = fabs(f2);
        alpha[3] = fabs(f3) + ns;
        return p[0] * v + p[1] * f1 + p[2] * f2 + p[3] * f3 + sgn * (ns * fabs(p[3]) - dd * fabs(p[0]));
    } else if constexpr (DYN == kDynQ10Z) {
        // c0 = (k_T/m) T_max - g, c1 = (k_T/m) T_min - g, c2 = dbar, c3 = max(|c0|, |c1|)
        T vz = k.a;
        alpha[0] = fabs(vz) + F::c(I, 2);
        alpha[1] = F::c(I, 3);
        // the thrust picks T_max or T_min by the sign of p_vz (avoid: maximise)
        T thrust = (sgn * p[1] > T(0)) ? p[1] * F::c(I, 0) : p[1] * F::c(I, 1);
        return p[0] * vz + thrust - sgn * F::c(I, 2) * fabs(p[0]);
    } else {
        T vx = k.a, vy = k.b, vz = k.c;
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

template <typename T, int DYN>
__device__ __forceinline__ T hamiltonian(const Inst &I, const T *__restrict__ tab, const int *idx,
                                         const T *p, T *alpha, T sgn)
{
    return ham_eval<T, DYN>(I, ham_coef<T, DYN>(I, tab, idx), p, alpha, sgn);
}

template <int DYN> struct DynDim;
template <> struct DynDim<kDynDI> { static constexpr int value = 2; };
template <> struct DynDim<kDynDubins> { static constexpr int value = 3; };
template <> struct DynDim<kDynUnicycle> { static constexpr int value = 4; };
template <> struct DynDim<kDynQuad> { static constexpr int value = 6; };
template <> struct DynDim<kDynQ10XY> { static constexpr int value = 4; };
template <> struct DynDim<kDynQ10Z> { static constexpr int value = 2; };

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

// L(S) at one node.  Every stencil value of every dim is loaded before any arithmetic, so a
// wave has all its loads in flight at once.  Returns the centre value through *centre.
template <typename T, int DYN, int SPATIAL>
__device__ __forceinline__ T lf_operator(const Inst &I, const T *__restrict__ S, uint32_t node, T *centre)
{
    constexpr int N = DynDim<DYN>::value;
    constexpr int W = SPATIAL == kWeno5 ? 7 : 3;
    using F = Fields<T>;
    constexpr int H = W / 2;
    int idx[N];
    bool inner[N];
    unflatten<N>(I, node, idx);
    T u[N][W];
    const T c = ldg(S, node);
#pragma unroll
    for (int d = 0; d < N; ++d) {
        // the last dim is the contiguous one (stride 1 is then a compile-time constant)
        const uint32_t stride = d == N - 1 ? 1u : I.stride[d];
        inner[d] = __all(idx[d] >= H && idx[d] < I.n[d] - H);
        line_load<T, SPATIAL>(S, node, idx[d], I.n[d], stride, (I.periodic >> d) & 1u, inner[d], u[d]);
        u[d][H] = c;
    }
    T p[N], diff[N], alpha[N];
#pragma unroll
    for (int d = 0; d < N; ++d) {
        T dm, dp;
        line_derivs<T, SPATIAL>(u[d], idx[d], I.n[d], (I.periodic >> d) & 1u, inner[d], F::eps0(I, d), dm, dp);
        const T h = F::hinv_dx(I, d);
        p[d] = h * (dm + dp);
        diff[d] = h * (dp - dm);
    }
    const T sgn = I.game == 0 ? T(1) : T(-1);
    T L = hamiltonian<T, DYN>(I, uniform_ptr(F::tab(I)), idx, p, alpha, sgn);
    L = add_dissipation<T, N>(L, alpha, diff);
    *centre = c;
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
