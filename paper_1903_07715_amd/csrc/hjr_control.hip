// Safe-control queries on a resident value function (Sec. II-B.2, eq. (uOpt)).
//
// gradient_kernel: one thread per node writes p = (D- + D+)/2 along every dim, with the same
// stencil loads and one-sided derivatives as the stage kernels (so p is the gradient the
// Lax-Friedrichs Hamiltonian sees), into a node-major table: the ndim components followed by
// V itself, so a query reads one contiguous record per cell corner.  control_kernel: one thread
// per query state interpolates p and V multilinearly over the state's grid cell and applies the
// model's optimal control in closed form.  Every model is affine in each control input (the quadrotor's attitude enters
// through tan, which is increasing), and the disturbance enters additively, so
// argmax_u min_d <p, f(x, u, d)> picks each control's bound by the sign of its coefficient in
// <p, f>; a zero coefficient picks the upper bound.  The reach game flips every choice.
#include "hjr_control.hpp"

namespace hjr {

template <int N, int SPATIAL>
__global__ __launch_bounds__(kBlock) void gradient_kernel(const Inst I, const double *__restrict__ V,
                                                          double *__restrict__ table)
{
    constexpr int W = SPATIAL == kWeno5 ? 7 : 3;
    constexpr int H = W / 2;
    const uint32_t node = blockIdx.x * kBlock + threadIdx.x;
    if (node >= I.npts) return;
    const double *Vu = uniform_ptr(V);
    int idx[N];
    unflatten<N>(I, node, idx);
    const double c = ldg(Vu, node);
#pragma unroll
    for (int d = 0; d < N; ++d) {
        const uint32_t stride = d == N - 1 ? 1u : I.stride[d];
        const bool periodic = (I.periodic >> d) & 1u;
        const bool inner = __all(idx[d] >= H && idx[d] < I.n[d] - H);
        double u[W];
        line_load<double, SPATIAL>(Vu, node, idx[d], I.n[d], stride, periodic, inner, u);
        u[H] = c;
        double dm, dp;
        line_derivs<double, SPATIAL>(u, idx[d], I.n[d], periodic, inner, I.eps0_64[d], dm, dp);
        table[(size_t)node * (N + 1) + d] = I.hinv_dx64[d] * (dm + dp);
    }
    table[(size_t)node * (N + 1) + N] = c;
}

// Cell of coordinate x along dim d: lower node j, upper node jn, weight w of the upper node.
// Non-periodic: x clamped into [lo, hi]; periodic: reduced into one period.  x is finite.
__device__ __forceinline__ void cell_of(const CtlGrid &G, int d, double x, int &j, int &jn, double &w)
{
#pragma clang fp contract(off)
    const int n = G.n[d];
    double s = (x - G.lo[d]) / G.dx[d];
    if ((G.periodic >> d) & 1u) {
        s = s - (double)n * floor(s / (double)n);
        int k = (int)floor(s);
        k = k > n - 1 ? n - 1 : (k < 0 ? 0 : k);
        j = k;
        jn = k + 1 == n ? 0 : k + 1;
        w = s - (double)k;
    } else {
        if (!(s >= 0.0)) s = 0.0;
        if (s > (double)(n - 1)) s = (double)(n - 1);
        int k = (int)floor(s);
        if (k > n - 2) k = n - 2;
        j = k;
        jn = k + 1;
        w = s - (double)k;
    }
}

template <int DYN> struct NumControls;
template <> struct NumControls<kDynDI> { static constexpr int value = 1; };
template <> struct NumControls<kDynDubins> { static constexpr int value = 1; };
template <> struct NumControls<kDynUnicycle> { static constexpr int value = 2; };
template <> struct NumControls<kDynQuad> { static constexpr int value = 3; };
template <> struct NumControls<kDynQ10XY> { static constexpr int value = 1; };
template <> struct NumControls<kDynQ10Z> { static constexpr int value = 1; };

// u* for gradient p.  sg = +1 (avoid: maximise) or -1 (reach: minimise); a control's bound
// follows the sign of sg times its coefficient in <p, f>, the upper bound when that is zero.
template <int DYN>
__device__ __forceinline__ void optimal_control(const CtlModel &M, const double *p, double *u)
{
    const double sg = M.game == 0 ? 1.0 : -1.0;
    const double *q = M.q;
    if constexpr (DYN == kDynDI) {  // x2' = b u, |u| <= ubar; q = {ubar, b, dbar}
        u[0] = sg * (q[1] * p[1]) >= 0.0 ? q[0] : -q[0];
    } else if constexpr (DYN == kDynDubins) {  // theta' = u, |u| <= ubar; q = {v, ubar, ...}
        u[0] = sg * p[2] >= 0.0 ? q[1] : -q[1];
    } else if constexpr (DYN == kDynUnicycle) {  // theta' = u1, v' = u2; q = {ubar1, ubar2, ...}
        u[0] = sg * p[2] >= 0.0 ? q[0] : -q[0];
        u[1] = sg * p[3] >= 0.0 ? q[1] : -q[1];
    } else if constexpr (DYN == kDynQ10XY) {  // omega' = -d0 theta + n0 S; q = {g, d0, d1, n0, S_max, dbar}
        u[0] = sg * (q[3] * p[3]) >= 0.0 ? q[4] : -q[4];
    } else if constexpr (DYN == kDynQ10Z) {  // v_z' = (k_T/m) T - g; q = {g, k_T, m, T_min, T_max, dbar}
        u[0] = sg * (q[1] / q[2] * p[1]) >= 0.0 ? q[4] : q[3];
    } else {  // vx' = g tan(theta), vy' = -g tan(phi), vz' = T/m - g; q = {g, m, phi_max, theta_max, Tmin, Tmax, ...}
        u[0] = sg * (q[0] * p[3]) >= 0.0 ? q[3] : -q[3];
        u[1] = sg * -(q[0] * p[4]) >= 0.0 ? q[2] : -q[2];
        u[2] = sg * p[5] >= 0.0 ? q[5] : q[4];
    }
}

template <int DYN>
__global__ __launch_bounds__(kBlock) void control_kernel(const CtlGrid G, const CtlModel M,
                                                         const double *__restrict__ table,
                                                         const double *__restrict__ x, int64_t nq,
                                                         double *__restrict__ u, double *__restrict__ p,
                                                         double *__restrict__ v)
{
#pragma clang fp contract(off)
    constexpr int N = DynDim<DYN>::value;
    constexpr int NU = NumControls<DYN>::value;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= nq) return;
    double xq[N];
    bool finite = true;
#pragma unroll
    for (int d = 0; d < N; ++d) {
        xq[d] = x[q * N + d];
        finite = finite && isfinite(xq[d]);
    }
    if (!finite) {  // NaN in every output of this query
        const double nan = __builtin_nan("");
#pragma unroll
        for (int i = 0; i < NU; ++i) u[q * NU + i] = nan;
        if (p)
#pragma unroll
            for (int d = 0; d < N; ++d) p[q * N + d] = nan;
        if (v) v[q] = nan;
        return;
    }
    int j[N], jn[N];
    double w[N];
#pragma unroll
    for (int d = 0; d < N; ++d) cell_of(G, d, xq[d], j[d], jn[d], w[d]);
    double pq[N];
#pragma unroll
    for (int d = 0; d < N; ++d) pq[d] = 0.0;
    double vq = 0.0;
    // corner c takes the upper node along dim d when bit d of c is set
#pragma unroll 4
    for (int c = 0; c < (1 << N); ++c) {
        double wt = 1.0;
        uint32_t node = 0;
#pragma unroll
        for (int d = 0; d < N; ++d) {
            const bool up = (c >> d) & 1;
            wt *= up ? w[d] : 1.0 - w[d];
            node += (uint32_t)(up ? jn[d] : j[d]) * G.stride[d];
        }
        const double *rec = table + (size_t)node * (N + 1);
#pragma unroll
        for (int d = 0; d < N; ++d) pq[d] += wt * rec[d];
        vq += wt * rec[N];
    }
    double uq[NU];
    optimal_control<DYN>(M, pq, uq);
#pragma unroll
    for (int i = 0; i < NU; ++i) u[q * NU + i] = uq[i];
    if (p)
#pragma unroll
        for (int d = 0; d < N; ++d) p[q * N + d] = pq[d];
    if (v) v[q] = vq;
}

template <int N>
static void launch_gradient_n(const Inst &I, int spatial, const double *V, double *table, dim3 g, hipStream_t s)
{
    if (spatial == kWeno5)
        hipLaunchKernelGGL((gradient_kernel<N, kWeno5>), g, dim3(kBlock), 0, s, I, V, table);
    else
        hipLaunchKernelGGL((gradient_kernel<N, kUpwind1>), g, dim3(kBlock), 0, s, I, V, table);
}

hipError_t launch_gradient(const Inst &I, int spatial, const double *V, double *table, hipStream_t s)
{
    if (I.npts == 0) return hipSuccess;
    const dim3 g((I.npts + kBlock - 1) / kBlock);
    switch (I.ndim) {
    case 1: launch_gradient_n<1>(I, spatial, V, table, g, s); break;
    case 2: launch_gradient_n<2>(I, spatial, V, table, g, s); break;
    case 3: launch_gradient_n<3>(I, spatial, V, table, g, s); break;
    case 4: launch_gradient_n<4>(I, spatial, V, table, g, s); break;
    case 5: launch_gradient_n<5>(I, spatial, V, table, g, s); break;
    case 6: launch_gradient_n<6>(I, spatial, V, table, g, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_control(const CtlGrid &G, const CtlModel &M, int dyn, const double *table, const double *x,
                          int64_t nq, double *u, double *p, double *v, hipStream_t s)
{
    if (nq <= 0) return hipSuccess;
    const dim3 g((unsigned)((nq + kBlock - 1) / kBlock));
    switch (dyn) {
    case kDynDI:
        hipLaunchKernelGGL(control_kernel<kDynDI>, g, dim3(kBlock), 0, s, G, M, table, x, nq, u, p, v);
        break;
    case kDynDubins:
        hipLaunchKernelGGL(control_kernel<kDynDubins>, g, dim3(kBlock), 0, s, G, M, table, x, nq, u, p, v);
        break;
    case kDynUnicycle:
        hipLaunchKernelGGL(control_kernel<kDynUnicycle>, g, dim3(kBlock), 0, s, G, M, table, x, nq, u, p, v);
        break;
    case kDynQuad:
        hipLaunchKernelGGL(control_kernel<kDynQuad>, g, dim3(kBlock), 0, s, G, M, table, x, nq, u, p, v);
        break;
    case kDynQ10XY:
        hipLaunchKernelGGL(control_kernel<kDynQ10XY>, g, dim3(kBlock), 0, s, G, M, table, x, nq, u, p, v);
        break;
    case kDynQ10Z:
        hipLaunchKernelGGL(control_kernel<kDynQ10Z>, g, dim3(kBlock), 0, s, G, M, table, x, nq, u, p, v);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hjr
