// hjr_kernels.hip -- gfx950 kernels of the HJI VI grid update and their launch wrappers.
//
// Work is described by a list of tiles (instance, first node, nodes per thread); a tile is
// npt * kBlock consecutive nodes of one instance's flattened grid.  One launch of a stage kernel advances every tile of
// every instance in its list, so a batch of grids of different size and dimension moves in one
// launch per stage.  Workgroups are mapped to tiles so that each XCD (workgroups are dealt to
// the eight XCDs round-robin) takes one contiguous run of tiles: the stencil halo of a tile is
// then mostly in the same XCD's L2.  A grid smaller than the tile count makes each workgroup
// loop over its XCD's run (persistent mode).
#include <hip/hip_ext.h>

#include <algorithm>
#include <vector>

#include "hjr_kernels.hpp"

namespace hjr {

// --------------------------------------------------------------------------------------------
// Reductions
// --------------------------------------------------------------------------------------------

// max that propagates NaN (fmax would drop it and let a blown-up field look converged)
template <typename T>
__device__ __forceinline__ T nanmax(T a, T b) { return (a != a || a > b) ? a : b; }

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ unsigned wave_sum(unsigned v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide max of a non-negative value, then an atomic max into *dst (FP64 bits).  Thousands
// of workgroups update the same word, so each first reads the word (from L2, relaxed) and
// issues the atomic only if its value is larger: the word only grows during a launch, so a
// skipped update was never needed.
template <int W = kBlock / 64>
__device__ __forceinline__ double block_max_to(double v, unsigned long long *dst, double *red)
{
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0) {
        m = red[0];
#pragma unroll
        for (int w = 1; w < W; ++w) m = nanmax(m, red[w]);
        const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
        if (m > 0.0 || m != m) {
            const unsigned long long cur = __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (bits > cur) atomicMax(dst, bits);
        }
    }
    __syncthreads();
    return m;  // the workgroup's maximum, in thread 0
}

// --------------------------------------------------------------------------------------------
// Local updates (exact): a step's result on a block of nodes depends only on V within the
// reach of its stencils (nstages x stencil half-width), so when none of those blocks changed
// in the previous step (and dt, the discount and the phase did not change either), the step
// would reproduce the block's values bit for bit, and its RK intermediates are the ones still
// in memory from the last step that computed it.  Such blocks are skipped.
// --------------------------------------------------------------------------------------------

// Whether the tile [start, start + span) takes part in this step: a full step, or one of its
// blocks was marked for this step by a block that changed in the previous one.  The marks of
// step e live in act[e & 1] (act holds two arrays of nblocks), which no stage of step e
// writes, so every stage of the step takes the same decision.
__device__ __forceinline__ bool tile_active(const Inst &I, const SolveState *st, uint32_t start, uint32_t span)
{
    const int epoch = st->epoch;
    if (epoch <= st->full_epoch) return true;
    const int *act = I.act + ((epoch & 1) ? I.nblocks : 0u);
    const uint32_t b1 = (min(start + span, I.npts) - 1u) >> kLocalShift;
    bool a = false;
    for (uint32_t b = start >> kLocalShift; b <= b1; ++b) a |= act[b] == epoch;
    return a;
}

// After the last stage of a tile whose values changed: mark every block whose next step
// depends on the tile's blocks (the dependency relation is symmetric; the lists are supersets
// of it) for the next step.  All threads of the workgroup share the stores.
__device__ __forceinline__ void mark_dependents(const Inst &I, const SolveState *st, uint32_t start, uint32_t span)
{
    const int next = st->epoch + 1;
    int *act = I.act + ((next & 1) ? I.nblocks : 0u);
    const uint32_t b0 = start >> kLocalShift;
    const uint32_t b1 = (min(start + span, I.npts) - 1u) >> kLocalShift;
    const uint32_t j1 = I.dep_off[b1 + 1];
    for (uint32_t j = I.dep_off[b0] + threadIdx.x; j < j1; j += kBlock) act[I.dep[j]] = next;
}

// --------------------------------------------------------------------------------------------
// Tile mapping
// --------------------------------------------------------------------------------------------

struct TileRange {
    int first, count, step;
};

__device__ __forceinline__ TileRange xcd_range(int ntiles)
{
    // X groups of workgroups: with 8 or more workgroups, group x is the workgroups that land on
    // XCD x; each group owns one contiguous run of tiles and deals it out round-robin.
    // These are scalar integer divisions, which the scalar unit runs as long instruction
    // sequences once per wave; with 8 groups (any launch of 8 or more workgroups) they are
    // shifts and masks, and with one workgroup per tile every group's count is 0 or 1.
    const int G = gridDim.x, b = blockIdx.x;
    int x, k, bx, tn, t0;
    if (G >= 8) {
        x = b & 7;
        k = b >> 3;
        bx = (G >> 3) + (x < (G & 7) ? 1 : 0);            // workgroups in group x
        tn = (ntiles >> 3) + (x < (ntiles & 7) ? 1 : 0);  // tiles of group x
        t0 = x * (ntiles >> 3) + min(x, ntiles & 7);
    } else {
        x = b;
        k = 0;
        bx = 1;
        tn = ntiles / G + (x < ntiles % G ? 1 : 0);
        t0 = x * (ntiles / G) + min(x, ntiles % G);
    }
    TileRange r;
    r.first = t0 + k;
    r.count = k >= tn ? 0 : (bx == tn ? 1 : (tn - k + bx - 1) / bx);
    r.step = bx;
    return r;
}

// --------------------------------------------------------------------------------------------
// Stage kernel
// --------------------------------------------------------------------------------------------

// LOCAL: the instance may use local updates (its changes are then recorded per block).
template <typename T, int DYN, int SPATIAL, int NPT, bool LOCAL>
__device__ __forceinline__ void stage_tile(const Inst &I, uint32_t start, int stage, T dt, double *red)
{
    using F = Fields<T>;
    SolveState *st = I.state;
    const bool euler = I.temporal == kEuler;
    const int par = euler ? st->parity : 0;
    T *V = F::V(I), *A = F::A(I), *B = F::B(I);
    const T *S, *Vn;
    T *O;
    if (euler) {
        S = par ? A : V;
        Vn = S;
        O = par ? V : A;
    } else if (stage == 0) {
        S = V; Vn = V; O = A;
    } else if (stage == 1) {
        S = A; Vn = V; O = B;
    } else {
        S = B; Vn = V; O = V;
    }
    const bool last = euler || stage == 2;
    S = uniform_ptr(S);
    Vn = uniform_ptr(Vn);
    O = uniform_ptr(O);
    const T *l = uniform_ptr(F::l(I));
    const T *G = uniform_ptr(F::g(I));  // reach-avoid constraint, or nullptr
    const T gm = (T)st->gamma;  // discount (1 outside discounted reachability: x * 1 == x exactly)
    T delta = T(0);  // in the field's precision: the max of exact differences is exact
    // NPT nodes per thread, kBlock apart: independent work the scheduler can interleave
    auto one = [&](uint32_t node) {
        T s;
        T L = lf_operator<T, DYN, SPATIAL>(I, S, node, &s);
        T vn = ldg(Vn, node);
        T out = stage_value<T>(euler, stage, gm, s, vn, dt, L);
        if (last) {
            if (!I.brs) out = fmin(ldg(l, node), out);
            if (G) out = fmax(ldg(G, node), out);
        }
        stg(O, node, out);
        if (last) delta = nanmax(delta, T(fabs(out - vn)));
    };
    if (start + (uint32_t)(NPT * kBlock) <= I.npts) {
#pragma unroll
        for (int k = 0; k < NPT; ++k) one(start + k * kBlock + threadIdx.x);
    } else {
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const uint32_t node = start + k * kBlock + threadIdx.x;
            if (node < I.npts) one(node);
        }
    }
    if (last) {
        block_max_to((double)delta, &st->delta_bits, red);
        if (LOCAL && I.act) {
            // every thread reads the per-wave maxima block_max_to left in red
            double m = red[0];
#pragma unroll
            for (int w = 1; w < kBlock / 64; ++w) m = nanmax(m, red[w]);
            __syncthreads();  // red is rewritten by the next tile of a persistent grid
            const uint32_t span = (uint32_t)(NPT * kBlock);
            if (m > 0.0 || m != m) mark_dependents(I, st, start, span);
            // grid points computed, per block (one counter per block: no contention)
            const uint32_t end = min(start + span, I.npts);
            const uint32_t b = (start >> kLocalShift) + threadIdx.x;
            if (b <= ((end - 1u) >> kLocalShift)) {
                const uint32_t lo = max(start, b << kLocalShift), hi = min(end, (b + 1u) << kLocalShift);
                atomicAdd(&I.cnt[b], (unsigned long long)(hi - lo));
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void stage_kernel(const Inst *__restrict__ insts,
                                                       const Tile *__restrict__ tiles, int ntiles,
                                                       int stage)
{
    __shared__ double red[kBlock / 64];
    const TileRange r = xcd_range(ntiles);
    for (int c = 0; c < r.count; ++c) {
        const Tile tl = tiles[r.first + c * r.step];
        const Inst &I = insts[tl.inst];
        SolveState *st = I.state;
        if (st->done != kRunning || stage >= I.nstages) continue;
        if (I.act && !tile_active(I, st, tl.start, (uint32_t)(kFusedNpt * kBlock))) continue;
        const T dt = (T)st->dt_cur;
        const int key = I.dyn * 8 + I.spatial;
        switch (key) {
        case kDynDI * 8 + kUpwind1: stage_tile<T, kDynDI, kUpwind1, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynDI * 8 + kWeno5: stage_tile<T, kDynDI, kWeno5, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynDubins * 8 + kUpwind1: stage_tile<T, kDynDubins, kUpwind1, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynDubins * 8 + kWeno5: stage_tile<T, kDynDubins, kWeno5, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynUnicycle * 8 + kUpwind1: stage_tile<T, kDynUnicycle, kUpwind1, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynUnicycle * 8 + kWeno5: stage_tile<T, kDynUnicycle, kWeno5, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynQuad * 8 + kUpwind1: stage_tile<T, kDynQuad, kUpwind1, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynQuad * 8 + kWeno5: stage_tile<T, kDynQuad, kWeno5, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynQ10XY * 8 + kUpwind1: stage_tile<T, kDynQ10XY, kUpwind1, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynQ10XY * 8 + kWeno5: stage_tile<T, kDynQ10XY, kWeno5, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynQ10Z * 8 + kUpwind1: stage_tile<T, kDynQ10Z, kUpwind1, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        case kDynQ10Z * 8 + kWeno5: stage_tile<T, kDynQ10Z, kWeno5, kFusedNpt, true>(I, tl.start, stage, dt, red); break;
        default: break;
        }
    }
}

// One model and one scheme per kernel: register allocation (and so occupancy) follows that
// variant alone instead of the largest variant of the fused kernel.  LOCAL variants serve the
// instances that use local updates (so the others' kernels carry none of that code).
template <typename T, int DYN, int SPATIAL, int NPT, bool LOCAL>
__global__ __launch_bounds__(kBlock) void stage_kernel_one(const Inst *__restrict__ insts,
                                                           const Tile *__restrict__ tiles, int ntiles,
                                                           int stage)
{
    __shared__ double red[kBlock / 64];
    const TileRange r = xcd_range(ntiles);
    for (int c = 0; c < r.count; ++c) {
        const Tile tl = tiles[r.first + c * r.step];
        const Inst &I = insts[tl.inst];
        SolveState *st = I.state;
        if (st->done != kRunning || stage >= I.nstages) continue;
        if (LOCAL && !tile_active(I, st, tl.start, (uint32_t)(NPT * kBlock))) continue;
        stage_tile<T, DYN, SPATIAL, NPT, LOCAL>(I, tl.start, stage, (T)st->dt_cur, red);
    }
}

// --------------------------------------------------------------------------------------------
// Plane-march stage kernel (first-order upwind stencils)
//
// Each thread owns one column of the grid (a position within a dim-0 plane) and advances it
// through a run of consecutive dim-0 planes.  The column's indices in dims 1.., its stencil
// offsets, its edge rule and the model's coordinate values are worked out once, not per node,
// and the dim-0 neighbours are carried from one plane to the next in registers, so per node
// the thread loads the next plane's value, the 2 (ndim - 1) neighbours within the plane and
// l, and writes one value.  Consecutive lanes hold consecutive columns, so every load and
// store of a wave is one contiguous run.  The per-node arithmetic is that of stage_tile
// (bitwise the same results).
// --------------------------------------------------------------------------------------------

// Buffer accesses: a resource descriptor (a field's base address and size, in scalar registers)
// plus a per-lane 32-bit byte offset and a uniform 32-bit byte offset.  A column's offsets stay
// fixed from plane to plane and only the uniform plane offset moves, so a load or store needs no
// per-lane address arithmetic and one scalar add per plane.  The host only hands the kernel
// fields below 4 GiB; offsets at or beyond the field's size would read zero and drop writes
// instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void *base, size_t bytes)
{
    const uint32_t n = bytes > 0xffffffffull ? 0xffffffffu : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n, 0x00020000);
}
template <typename T> __device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff);
template <> __device__ __forceinline__ float bld<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
template <> __device__ __forceinline__ double bld<double>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, soff, 0);
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, double v)
{
    using u2 = unsigned int __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, soff, 0);
}

// The fields a plane-march stage reads and writes: S the stage's input, Vn the step-start value
// (RK3 stages 2 and 3), O the output.  Euler steps alternate between V and A by the step's parity.
template <typename T> struct MarchFields {
    const T *S, *Vn;
    T *O;
};
template <typename T>
__device__ __forceinline__ MarchFields<T> march_fields(const Inst &I, int stage, bool euler)
{
    using F = Fields<T>;
    T *V = F::V(I), *A = F::A(I), *B = F::B(I);
    if (euler) return I.state->parity ? MarchFields<T>{A, A, V} : MarchFields<T>{V, V, A};
    if (stage == 0) return MarchFields<T>{V, V, A};
    if (stage == 1) return MarchFields<T>{A, V, B};
    return MarchFields<T>{B, V, V};
}

// The update of one node by the plane-march kernels, in the expressions and order of
// stage_tile: one-sided differences along dim 0 from the column's previous, current and next
// values (at a non-periodic end the interior difference stands in for the missing one), along
// dims 1.. from the loaded neighbours and the edge-rule signs sm, sp; the Hamiltonian with its
// dissipation; the integrator stage with its projection.  vn is the step-start value (u0 for
// Euler).
template <typename T, int DYN, bool EP> struct MarchUpdate {
    static constexpr int N = DynDim<DYN>::value;
    const Inst &I;
    HamCoef<T> kc;
    T sgn, gm, dt;
    int n0, stage;
    bool per0, euler, hasg;
    T sm[N], sp[N];

    __device__ __forceinline__ T operator()(int i, T um, T u0, T up, const T *un, const T *unp, T lv, T gv,
                                            T vn) const
    {
        using F = Fields<T>;
        T p[N], diff[N], alpha[N];
        {
            T dm = u0 - um, dq = up - u0;
            if (!per0) {
                const T r0 = dm, r1 = dq;
                dm = i == 0 ? r1 : r0;
                dq = i == n0 - 1 ? r0 : r1;
            }
            const T h = F::hinv_dx(I, 0);
            p[0] = h * (dm + dq);
            diff[0] = h * (dq - dm);
        }
#pragma unroll
        for (int d = 1; d < N; ++d) {
            const T dm = sm[d] * (u0 - un[d]);
            const T dq = sp[d] * (unp[d] - u0);
            const T h = F::hinv_dx(I, d);
            p[d] = h * (dm + dq);
            diff[d] = h * (dq - dm);
        }
        const T L = add_dissipation<T, N>(ham_eval<T, DYN>(I, kc, p, alpha, sgn), alpha, diff);
        if (EP) return fmin(lv, stage_value<T>(true, 0, gm, u0, vn, dt, L));
        T out = stage_value<T>(euler, stage, gm, u0, vn, dt, L);
        if (euler || stage == 2) {
            if (!I.brs) out = fmin(lv, out);
            if (hasg) out = fmax(gv, out);
        }
        return out;
    }
};

// The byte offsets of a node's -/+ neighbours along dim d within the plane (s: the dim's stride
// in columns) and the signs that apply the edge rule: at a non-periodic end the missing
// neighbour is replaced by the one on the other side and the difference negated, which gives
// the interior difference exactly (the rule of line_derivs); periodic dims wrap.
template <typename T>
__device__ __forceinline__ void edge_offsets(const Inst &I, int d, int j, uint32_t c, int s, uint32_t &om,
                                             uint32_t &op, T &sm, T &sp)
{
    const int n = I.n[d];
    int m, q;
    T a, b;
    if ((I.periodic >> d) & 1u) {
        m = j > 0 ? -1 : n - 1;
        q = j < n - 1 ? 1 : 1 - n;
        a = b = T(1);
    } else {
        m = j > 0 ? -1 : 1;
        q = j < n - 1 ? 1 : -1;
        a = j > 0 ? T(1) : T(-1);
        b = j < n - 1 ? T(1) : T(-1);
    }
    om = (uint32_t)((int)c + m * s) * (uint32_t)sizeof(T);
    op = (uint32_t)((int)c + q * s) * (uint32_t)sizeof(T);
    sm = a;
    sp = b;
}

// EP: the instance takes forward Euler steps projected on l with no constraint function (the
// common case), so every node makes the same loads; the compiler can then keep the next plane's
// loads in flight across this plane's arithmetic (a load under a branch makes it wait for all).
template <typename T, int DYN, bool EP>
__device__ __forceinline__ void march_tile(const Inst &I, const MTile &tl, int stage, T dt, double *red)
{
    constexpr int N = DynDim<DYN>::value;
    using F = Fields<T>;
    SolveState *st = I.state;
    const bool euler = EP || I.temporal == kEuler;
    const MarchFields<T> f = march_fields<T>(I, stage, euler);
    const bool last = euler || stage == 2;
    const T *G = EP ? nullptr : uniform_ptr(F::g(I));  // reach-avoid constraint, or nullptr
    const size_t fbytes = (size_t)I.npts * sizeof(T);
    const __amdgpu_buffer_rsrc_t rS = buf(uniform_ptr(f.S), fbytes), rVn = buf(uniform_ptr(f.Vn), fbytes);
    const __amdgpu_buffer_rsrc_t rO = buf(uniform_ptr(f.O), fbytes), rl = buf(uniform_ptr(F::l(I)), fbytes);
    const __amdgpu_buffer_rsrc_t rG = buf(G, fbytes);
    const uint32_t P = I.stride[0];                       // columns (nodes per dim-0 plane)
    const uint32_t pb = P * (uint32_t)sizeof(T);          // bytes per plane
    const int n0 = I.n[0];
    const bool per0 = I.periodic & 1u;
    const uint32_t c = tl.c0 + threadIdx.x;
    T delta = T(0);
    if (threadIdx.x < tl.cn) {
        int idx[N];
        idx[0] = 0;
        uint32_t rem = c;
#pragma unroll
        for (int d = N - 1; d >= 2; --d) {
            const uint32_t q = fdiv(rem, I.div[d]);
            idx[d] = (int)(rem - q * (uint32_t)I.n[d]);
            rem = q;
        }
        if (N >= 2) idx[1] = (int)rem;
        MarchUpdate<T, DYN, EP> mu{I, {}, I.game == 0 ? T(1) : T(-1), (T)st->gamma, dt, n0, stage, per0, euler,
                                   G != nullptr, {}, {}};
        uint32_t om[N], op[N];
#pragma unroll
        for (int d = 1; d < N; ++d)
            edge_offsets<T>(I, d, idx[d], c, d == N - 1 ? 1 : (int)I.stride[d], om[d], op[d], mu.sm[d], mu.sp[d]);
        mu.kc = ham_coef<T, DYN>(I, uniform_ptr(F::tab(I)), idx);
        const uint32_t cb = c * (uint32_t)sizeof(T);
        const int i0 = tl.i0, i1 = tl.i0 + tl.len;
        const bool proj = EP || (last && !I.brs);
        const bool useg = !EP && last && G != nullptr;
        // values of S at planes i - 1 and i; at a non-periodic end the centre stands in for the
        // missing neighbour (its difference is replaced in the update)
        const int im = i0 > 0 ? i0 - 1 : (per0 ? n0 - 1 : 0);
        T um = bld<T>(rS, cb, (uint32_t)im * pb);
        T u0 = bld<T>(rS, cb, (uint32_t)i0 * pb);
        // every load a node needs (the next plane's value, the neighbours within the plane, l,
        // the constraint, the step-start value), issued together
        struct Cur {
            T up, un[N], unp[N], lv, gv, vn;
        };
        auto load_plane = [&](int i, uint32_t so) {
            Cur c;
            const uint32_t sp1 = i + 1 < n0 ? so + pb : (per0 ? 0u : so);
            c.up = bld<T>(rS, cb, sp1);
#pragma unroll
            for (int d = 1; d < N; ++d) {
                c.un[d] = bld<T>(rS, om[d], so);
                c.unp[d] = bld<T>(rS, op[d], so);
            }
            c.lv = proj ? bld<T>(rl, cb, so) : T(0);
            c.gv = useg ? bld<T>(rG, cb, so) : T(0);
            c.vn = euler ? T(0) : bld<T>(rVn, cb, so);
            return c;
        };
        // the node at plane i from its loads c (so is the same in every lane; saying so keeps the
        // store's offset in a scalar register)
        auto node = [&](int i, uint32_t so, const Cur &c) {
            so = __builtin_amdgcn_readfirstlane(so);
            const T vn = euler ? u0 : c.vn;
            const T out = mu(i, um, u0, c.up, c.un, c.unp, c.lv, c.gv, vn);
            bst(rO, cb, so, out);
            if (last) delta = nanmax(delta, T(fabs(out - vn)));
            um = u0;
            u0 = c.up;
        };
        // Two planes per trip, with two sets of load registers used in turn: the next plane's
        // loads go out before this plane's arithmetic, so the loads of two planes are in flight
        // at once, and no register copy waits for a load (the last plane of a run reloads
        // itself, unused).
        uint32_t so = (uint32_t)i0 * pb;  // byte offset of plane i
        Cur ca = load_plane(i0, so);
        // (the scheduling barriers keep the compiler from moving the loads after the arithmetic)
        for (int i = i0; i < i1; i += 2, so += 2 * pb) {
            const int ib = i + 1 < i1 ? i + 1 : i;
            const Cur cn = load_plane(ib, (uint32_t)ib * pb);
            asm volatile("" ::: "memory");
            node(i, so, ca);
            if (i + 1 >= i1) break;
            const int ia = i + 2 < i1 ? i + 2 : i + 1;
            ca = load_plane(ia, (uint32_t)ia * pb);
            asm volatile("" ::: "memory");
            node(i + 1, so + pb, cn);
        }
    }
    if (last) block_max_to((double)delta, &st->delta_bits, red);
}

// One workgroup per tile, in list order: workgroups are dealt to the 8 XCDs round-robin
// (workgroup b to XCD b mod 8), and the host interleaves the list so that each XCD receives
// compact blocks of neighbouring tiles.
template <typename T, int DYN>
__global__ __launch_bounds__(kBlock) void march_kernel(const Inst *__restrict__ insts, const MTile *__restrict__ tiles,
                                                       int ntiles, int stage)
{
    __shared__ double red[kBlock / 64];
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const MTile tl = tiles[t];
    if (tl.cn == 0) return;  // padding
    const Inst &I = insts[tl.inst];
    const SolveState *st = I.state;
    if (st->done != kRunning || stage >= I.nstages) return;
    if (I.temporal == kEuler && !I.brs && Fields<T>::g(I) == nullptr)
        march_tile<T, DYN, true>(I, tl, stage, (T)st->dt_cur, red);
    else
        march_tile<T, DYN, false>(I, tl, stage, (T)st->dt_cur, red);
}

// --------------------------------------------------------------------------------------------
// Brick variant of the plane-march kernel (6-D grids, first-order upwind)
//
// In the march kernel the loads that cost time are those of the far neighbours, along dims 1..3
// of a 6-D grid (a row of dims 4..5 or more away): they miss the L1 cache and the vector memory
// pipeline waits on their round trips to L2 and beyond.  Here a workgroup takes a brick of
// 2 x 2 x 2 rows over dims 1..3 (rows 2k and 2k+1 of each of the three dims) and a segment of
// kBrickSeg consecutive columns of those rows, and walks its dim-0 line as the march kernel
// does.  Each plane's centre values also go to LDS, and along each far dim a node takes the
// neighbour inside its pair of rows from there, so only the neighbour on the other side is
// loaded from memory: three far loads per node instead of six.  At an end of a dim the edge
// rule picks the same values as in the march kernel (the partner or the loaded neighbour, and
// the same sign flips), and the update is MarchUpdate, so the results are the march kernel's
// bit for bit.  A dim of odd length leaves its last row without a partner; that row loads both
// of its neighbours from memory (one load: without a partner the row is the dim's last, so a
// non-periodic end replaces the missing neighbour by the loaded one; the host does not give
// this kernel a periodic dim of odd length among dims 1..3).  Lanes past the end of a segment
// work on the segment's last column and rows past the end of a dim on the brick's first column;
// neither stores, and every lane passes every barrier.
// --------------------------------------------------------------------------------------------
constexpr int kBrickSeg = 128;                          // columns per row segment
constexpr int kBrickRows = 8;                           // 2 x 2 x 2 rows over dims 1..3
constexpr int kBrickThreads = kBrickSeg * kBrickRows;   // threads per workgroup

// Workgroup barrier for LDS traffic only: the LDS writes before it are complete and visible to
// the reads after it; loads and stores of global memory still in flight are not waited for.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T, int DYN, bool EP>
__device__ __forceinline__ void march_brick_tile(const Inst &I, const MTile &tl, int stage, T dt, double *red,
                                                 T (*lds)[kBrickRows][kBrickSeg])
{
    constexpr int N = DynDim<DYN>::value;
    static_assert(N == 6, "bricks pair the rows of dims 1..3 of a 6-D grid");
    using F = Fields<T>;
    SolveState *st = I.state;
    const bool euler = EP || I.temporal == kEuler;
    const MarchFields<T> f = march_fields<T>(I, stage, euler);
    const bool last = euler || stage == 2;
    const T *G = EP ? nullptr : uniform_ptr(F::g(I));
    const size_t fbytes = (size_t)I.npts * sizeof(T);
    const __amdgpu_buffer_rsrc_t rS = buf(uniform_ptr(f.S), fbytes), rVn = buf(uniform_ptr(f.Vn), fbytes);
    const __amdgpu_buffer_rsrc_t rO = buf(uniform_ptr(f.O), fbytes), rl = buf(uniform_ptr(F::l(I)), fbytes);
    const __amdgpu_buffer_rsrc_t rG = buf(G, fbytes);
    const uint32_t pb = I.stride[0] * (uint32_t)sizeof(T);  // bytes per plane
    const int n0 = I.n[0];
    const bool per0 = I.periodic & 1u;
    // the row is the same in a wave (a wave is 64 columns of one row); saying so keeps everything
    // that depends only on the row (its indices along dims 1..3, edge rule, partner) scalar
    const int row = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kBrickSeg);
    const int sx = (int)threadIdx.x % kBrickSeg;
    // indices of the brick's first column (the same in every lane)
    int base[N];
    {
        uint32_t rem = tl.c0;
#pragma unroll
        for (int d = N - 1; d >= 2; --d) {
            const uint32_t q = fdiv(rem, I.div[d]);
            base[d] = (int)(rem - q * (uint32_t)I.n[d]);
            rem = q;
        }
        base[1] = (int)rem;
    }
    int e[4];  // this row's place in its pair along dims 1..3
    e[1] = (row >> 2) & 1;
    e[2] = (row >> 1) & 1;
    e[3] = row & 1;
    bool rowok = true;
#pragma unroll
    for (int d = 1; d <= 3; ++d) rowok = rowok && base[d] + e[d] < I.n[d];
    // lanes past the segment's end work on its last column; a row past a dim's end on the
    // brick's first column (valid addresses either way; neither stores)
    const bool active = rowok && sx < (int)tl.cn;
    const int sc = sx < (int)tl.cn ? sx : (int)tl.cn - 1;
    int idx[N];
    uint32_t c = tl.c0;
    idx[0] = 0;
#pragma unroll
    for (int d = 1; d < N; ++d) idx[d] = base[d];
    if (rowok) {
        c += (uint32_t)(e[1] * (int)I.stride[1] + e[2] * (int)I.stride[2] + e[3] * (int)I.stride[3] + sc);
#pragma unroll
        for (int d = 1; d <= 3; ++d) idx[d] += e[d];
        const uint32_t r = (uint32_t)(base[4] * I.n[5] + base[5] + sc);  // position within the row
        const uint32_t q = fdiv(r, I.div[5]);
        idx[4] = (int)q;
        idx[5] = (int)(r - q * (uint32_t)I.n[5]);
    }
    MarchUpdate<T, DYN, EP> mu{I, {}, I.game == 0 ? T(1) : T(-1), (T)st->gamma, dt, n0, stage, per0, euler,
                               G != nullptr, {}, {}};
    // far dims: the byte offset of the neighbour loaded from memory, and which sides take the
    // partner row's value from LDS instead (all of it the same across a wave)
    uint32_t og[4];
    bool ml[4], pl[4];
#pragma unroll
    for (int d = 1; d <= 3; ++d) {
        const int j = idx[d], n = I.n[d];
        const bool per = (I.periodic >> d) & 1u;
        int q = 0;
        bool m = false, p = false;
        T a = T(1), b = T(1);
        if (!rowok) {
            // a row past a dim's end: its values are never used
        } else if (e[d]) {  // the partner is j - 1
            m = true;
            if (j + 1 < n) q = 1;
            else if (per) q = 1 - n;
            else { p = true; b = T(-1); }
        } else if (j + 1 < n) {  // the partner is j + 1
            p = true;
            if (j > 0) q = -1;
            else if (per) q = n - 1;
            else { m = true; a = T(-1); }
        } else {  // the dim's last row, without a partner (non-periodic)
            q = -1;
            b = T(-1);
        }
        og[d] = (uint32_t)((int)c + q * (int)I.stride[d]) * (uint32_t)sizeof(T);
        ml[d] = m;
        pl[d] = p;
        mu.sm[d] = a;
        mu.sp[d] = b;
    }
    uint32_t om[N], op[N];
#pragma unroll
    for (int d = 4; d < N; ++d)
        edge_offsets<T>(I, d, idx[d], c, d == N - 1 ? 1 : (int)I.stride[d], om[d], op[d], mu.sm[d], mu.sp[d]);
    mu.kc = ham_coef<T, DYN>(I, uniform_ptr(F::tab(I)), idx);
    const uint32_t cb = c * (uint32_t)sizeof(T);
    const int i0 = tl.i0, i1 = tl.i0 + tl.len;
    const bool proj = EP || (last && !I.brs);
    const bool useg = !EP && last && G != nullptr;
    const int im = i0 > 0 ? i0 - 1 : (per0 ? n0 - 1 : 0);
    T um = bld<T>(rS, cb, (uint32_t)im * pb);
    T u0 = bld<T>(rS, cb, (uint32_t)i0 * pb);
    T delta = T(0);
    struct Cur {
        T up, g[4], un[N], unp[N], lv, gv, vn;
    };
    auto load_plane = [&](int i, uint32_t so) {
        Cur c;
        const uint32_t sp1 = i + 1 < n0 ? so + pb : (per0 ? 0u : so);
        c.up = bld<T>(rS, cb, sp1);
#pragma unroll
        for (int d = 1; d <= 3; ++d) c.g[d] = bld<T>(rS, og[d], so);
#pragma unroll
        for (int d = 4; d < N; ++d) {
            c.un[d] = bld<T>(rS, om[d], so);
            c.unp[d] = bld<T>(rS, op[d], so);
        }
        c.lv = proj ? bld<T>(rl, cb, so) : T(0);
        c.gv = useg ? bld<T>(rG, cb, so) : T(0);
        c.vn = euler ? T(0) : bld<T>(rVn, cb, so);
        return c;
    };
    // the node at plane i: its centre value goes to the plane's LDS buffer (two buffers, used by
    // alternate planes, so one barrier per plane suffices), then the partner rows' values come back
    auto node = [&](int i, uint32_t so, Cur &c) {
        so = __builtin_amdgcn_readfirstlane(so);
        T(*b)[kBrickSeg] = lds[i & 1];
        b[row][sx] = u0;
        lds_barrier();
#pragma unroll
        for (int d = 1; d <= 3; ++d) {
            const T v = b[row ^ (4 >> (d - 1))][sx];
            c.un[d] = ml[d] ? v : c.g[d];
            c.unp[d] = pl[d] ? v : c.g[d];
        }
        const T vn = euler ? u0 : c.vn;
        const T out = mu(i, um, u0, c.up, c.un, c.unp, c.lv, c.gv, vn);
        if (active) {
            bst(rO, cb, so, out);
            if (last) delta = nanmax(delta, T(fabs(out - vn)));
        }
        um = u0;
        u0 = c.up;
    };
    // two planes per trip with two sets of load registers, as in march_tile; every lane makes the
    // same number of trips, so the barriers match
    uint32_t so = (uint32_t)i0 * pb;
    Cur ca = load_plane(i0, so);
    for (int i = i0; i < i1; i += 2, so += 2 * pb) {
        const int ib = i + 1 < i1 ? i + 1 : i;
        Cur cn = load_plane(ib, (uint32_t)ib * pb);
        asm volatile("" ::: "memory");
        node(i, so, ca);
        if (i + 1 >= i1) break;
        const int ia = i + 2 < i1 ? i + 2 : i + 1;
        ca = load_plane(ia, (uint32_t)ia * pb);
        asm volatile("" ::: "memory");
        node(i + 1, so + pb, cn);
    }
    if (last) block_max_to<kBrickThreads / 64>((double)delta, &st->delta_bits, red);
}

// FP32: at most 64 VGPRs, so that two workgroups (8 waves per SIMD) fit on a CU
template <typename T, int DYN>
__global__ __launch_bounds__(kBrickThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 4)))
void march_brick_kernel(const Inst *__restrict__ insts,
                                                                    const MTile *__restrict__ tiles, int ntiles,
                                                                    int stage)
{
    __shared__ double red[kBrickThreads / 64];
    __shared__ T lds[2][kBrickRows][kBrickSeg];
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const MTile tl = tiles[t];
    if (tl.cn == 0) return;  // padding
    const Inst &I = insts[tl.inst];
    const SolveState *st = I.state;
    if (st->done != kRunning || stage >= I.nstages) return;
    if (I.temporal == kEuler && !I.brs && Fields<T>::g(I) == nullptr)
        march_brick_tile<T, DYN, true>(I, tl, stage, (T)st->dt_cur, red, lds);
    else
        march_brick_tile<T, DYN, false>(I, tl, stage, (T)st->dt_cur, red, lds);
}

// --------------------------------------------------------------------------------------------
// Plane-march stage kernel for WENO5 stencils
//
// As march_tile: one thread per column, walking a run of dim-0 planes.  Along dim 0 the thread
// keeps the column's six edge-extended differences around the current plane in registers and
// computes each WENO5 interface once: the interface between planes i and i+1 gives D+ at i and
// D- at i+1, so per node the dim-0 stencil costs one interface and two candidate combinations
// where the flat kernel computes two interfaces, and one new load where the flat kernel makes
// six.  Within the plane each dim takes its six neighbours at offsets fixed per column
// (periodic ends wrapped, positions off the line replaced by the centre, as line_load does) and
// the flat kernel's line_derivs.  The per-node arithmetic is that of stage_tile, so the results
// are bitwise the same.
// --------------------------------------------------------------------------------------------
template <typename T, int DYN>
__device__ __forceinline__ void march_tile_w5(const Inst &I, const MTile &tl, int stage, T dt, double *red)
{
    constexpr int N = DynDim<DYN>::value;
    using F = Fields<T>;
    SolveState *st = I.state;
    const bool euler = I.temporal == kEuler;
    const int par = euler ? st->parity : 0;
    T *V = F::V(I), *A = F::A(I), *B = F::B(I);
    const T *S, *Vn;
    T *O;
    if (euler) {
        S = par ? A : V;
        Vn = S;
        O = par ? V : A;
    } else if (stage == 0) {
        S = V; Vn = V; O = A;
    } else if (stage == 1) {
        S = A; Vn = V; O = B;
    } else {
        S = B; Vn = V; O = V;
    }
    const bool last = euler || stage == 2;
    const T *G = uniform_ptr(F::g(I));
    const size_t fbytes = (size_t)I.npts * sizeof(T);
    const __amdgpu_buffer_rsrc_t rS = buf(uniform_ptr(S), fbytes), rVn = buf(uniform_ptr(Vn), fbytes);
    const __amdgpu_buffer_rsrc_t rO = buf(uniform_ptr(O), fbytes), rl = buf(uniform_ptr(F::l(I)), fbytes);
    const __amdgpu_buffer_rsrc_t rG = buf(G, fbytes);
    const T gm = (T)st->gamma;
    const uint32_t P = I.stride[0];
    const uint32_t pb = P * (uint32_t)sizeof(T);
    const int n0 = I.n[0];
    const bool per0 = I.periodic & 1u;
    const uint32_t c = tl.c0 + threadIdx.x;
    T delta = T(0);
    if (threadIdx.x < tl.cn) {
        int idx[N];
        idx[0] = 0;
        uint32_t rem = c;
#pragma unroll
        for (int d = N - 1; d >= 2; --d) {
            const uint32_t q = fdiv(rem, I.div[d]);
            idx[d] = (int)(rem - q * (uint32_t)I.n[d]);
            rem = q;
        }
        if (N >= 2) idx[1] = (int)rem;
        // byte offsets of the neighbours at -3, -2, -1, +1, +2, +3 along each dim of the plane
        uint32_t off[N][6];
        bool inner[N];
#pragma unroll
        for (int d = 1; d < N; ++d) {
            const int j = idx[d], n = I.n[d];
            const bool per = (I.periodic >> d) & 1u;
            const int s = d == N - 1 ? 1 : (int)I.stride[d];
            inner[d] = __all(j >= 3 && j < n - 3);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const int o = k < 3 ? k - 3 : k - 2;
                int q;
                if (per)
                    q = o < 0 ? (j + o < 0 ? o + n : o) : (j + o >= n ? o - n : o);
                else
                    q = (o < 0 ? j + o >= 0 : j + o < n) ? o : 0;
                off[d][k] = (uint32_t)((int)c + q * s) * (uint32_t)sizeof(T);
            }
        }
        const HamCoef<T> kc = ham_coef<T, DYN>(I, uniform_ptr(F::tab(I)), idx);
        const T sgn = I.game == 0 ? T(1) : T(-1);
        const uint32_t cb = c * (uint32_t)sizeof(T);
        const int i0 = tl.i0, i1 = tl.i0 + tl.len;
        const bool proj = last && !I.brs;
        const bool useg = last && G != nullptr;
        const T eps00 = F::eps0(I, 0);
        // planes i0-3 .. i0+3 (wrapped on a periodic dim 0; off the line the centre stands in)
        // and the differences Delta_{i0-2} .. Delta_{i0+3} of the extended sequence
        T D[6];
        T u0, u1, u2, u3;  // S at planes i, i+1, i+2, i+3
        {
            T w[7];
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                int q = i0 + k - 3;
                if (per0)
                    q = q < 0 ? q + n0 : (q >= n0 ? q - n0 : q);
                else
                    q = (q < 0 || q >= n0) ? i0 : q;
                w[k] = bld<T>(rS, cb, (uint32_t)q * pb);
            }
            line_diffs<T, kWeno5>(w, i0, n0, per0, false, D);
            u0 = w[3];
            u1 = w[4];
            u2 = w[5];
            u3 = w[6];
        }
        // D- at the current plane, from the interface on its left
        T dmn;
        {
            const WenoIf<T> wl = weno5_interface(D[0], D[1], D[2], D[3], D[4], eps00);
            dmn = weno5_left(wl, D[0], D[1], D[2], D[3], D[4]);
        }
        uint32_t so = (uint32_t)i0 * pb;
        for (int i = i0; i < i1; ++i, so += pb) {
            struct {
                T u4, un[N][6], lv, gv, vn;
            } cur;
            {
                // plane i+4 (its difference enters at the next plane); past a non-periodic end,
                // or after the last plane of the run, plane i is read instead and not used
                int q4 = i + 4;
                if (per0) q4 = q4 >= n0 ? q4 - n0 : q4;
                const bool need4 = i + 1 < i1 && (per0 || q4 < n0);
                cur.u4 = bld<T>(rS, cb, need4 ? (uint32_t)q4 * pb : so);
#pragma unroll
                for (int d = 1; d < N; ++d)
#pragma unroll
                    for (int k = 0; k < 6; ++k) cur.un[d][k] = bld<T>(rS, off[d][k], so);
                cur.lv = proj ? bld<T>(rl, cb, so) : T(0);
                cur.gv = useg ? bld<T>(rG, cb, so) : T(0);
                cur.vn = euler ? T(0) : bld<T>(rVn, cb, so);
            }
            T p[N], diff[N], alpha[N];
            {
                const WenoIf<T> wr = weno5_interface(D[1], D[2], D[3], D[4], D[5], eps00);
                const T dm = dmn;
                const T dq = weno5_right(wr, D[1], D[2], D[3], D[4], D[5]);
                dmn = weno5_left(wr, D[1], D[2], D[3], D[4], D[5]);
                const T h = F::hinv_dx(I, 0);
                p[0] = h * (dm + dq);
                diff[0] = h * (dq - dm);
            }
#pragma unroll
            for (int d = 1; d < N; ++d) {
                const T uu[7] = {cur.un[d][0], cur.un[d][1], cur.un[d][2], u0,
                                 cur.un[d][3], cur.un[d][4], cur.un[d][5]};
                T dm, dq;
                line_derivs<T, kWeno5>(uu, idx[d], I.n[d], (I.periodic >> d) & 1u, inner[d], F::eps0(I, d), dm, dq);
                const T h = F::hinv_dx(I, d);
                p[d] = h * (dm + dq);
                diff[d] = h * (dq - dm);
            }
            const T L = add_dissipation<T, N>(ham_eval<T, DYN>(I, kc, p, alpha, sgn), alpha, diff);
            const T vn = euler ? u0 : cur.vn;
            T out = stage_value<T>(euler, stage, gm, u0, vn, dt, L);
            if (last) {
                if (!I.brs) out = fmin(cur.lv, out);
                if (G) out = fmax(cur.gv, out);
            }
            bst(rO, cb, so, out);
            if (last) delta = nanmax(delta, T(fabs(out - vn)));
            // slide: the difference Delta_{i+4} enters (past a non-periodic end it repeats the
            // last interior one)
            const T dnew = (per0 || i + 4 < n0) ? cur.u4 - u3 : D[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) D[k] = D[k + 1];
            D[5] = dnew;
            u0 = u1;
            u1 = u2;
            u2 = u3;
            u3 = cur.u4;
        }
    }
    if (last) block_max_to((double)delta, &st->delta_bits, red);
}

template <typename T, int DYN>
__global__ __launch_bounds__(kBlock) void march_kernel_w5(const Inst *__restrict__ insts,
                                                          const MTile *__restrict__ tiles, int ntiles, int stage)
{
    __shared__ double red[kBlock / 64];
    const int t = blockIdx.x;
    if (t >= ntiles) return;
    const MTile tl = tiles[t];
    if (tl.cn == 0) return;  // padding
    const Inst &I = insts[tl.inst];
    const SolveState *st = I.state;
    if (st->done != kRunning || stage >= I.nstages) return;
    march_tile_w5<T, DYN>(I, tl, stage, (T)st->dt_cur, red);
}

// --------------------------------------------------------------------------------------------
// Step bookkeeping (one thread per instance)
// --------------------------------------------------------------------------------------------

// Step size for the next step: the CFL step, cut so the step ends exactly at t_max and, in
// interval mode, at the end of the current report interval.
__device__ __forceinline__ double next_dt(const SolveState *st)
{
    double dt = st->dt_nom;
    if (st->t_max > 0.0 && st->t_max - st->t < dt) dt = st->t_max - st->t;
    if (st->conv_mode == 1 && st->dt_report - st->t_int < dt) dt = st->dt_report - st->t_int;
    return dt;
}

__device__ __forceinline__ void apply_limits(SolveState *st)
{
    if (st->done != kRunning) return;
    if (st->max_iter > 0 && st->n >= st->max_iter) {
        st->done = kMaxIter;
    } else if (st->t_max > 0.0 && st->t >= st->t_max * (1.0 - 1e-12)) {
        st->done = kHorizon;
    } else {
        const double dt = next_dt(st);
        if (dt != st->dt_cur) st->full_epoch = st->epoch;  // another step size: compute in full
        st->dt_cur = dt;
    }
}

// Stall rule: no new 1% low of the change for stall_window steps (or intervals) while the
// change is within 64x of the threshold, or for 16 stall_windows at any level, means the iterate
// has reached its floor (FP32 rounding, or a limit cycle of the scheme).  Far from the threshold
// the change may plateau or grow for a while as fronts develop, hence the longer window there.
__device__ __forceinline__ void note_delta(SolveState *st, double delta, long long count)
{
    if (st->stall_window <= 0 || st->done != kRunning) return;
    if (delta < 0.99 * st->best_delta) {
        st->best_delta = delta;
        st->n_best = count;
        return;
    }
    const long long window = delta < 64.0 * st->tol ? st->stall_window : 16 * st->stall_window;
    if (count - st->n_best >= window) st->done = kStalled;
}

// Discounted reachability: a first phase that has converged (or stalled) with gamma < 1 goes on
// undiscounted instead of ending.
__device__ __forceinline__ void anneal(SolveState *st, long long count)
{
    if (st->gamma == 1.0 || (st->done != kConverged && st->done != kStalled)) return;
    st->gamma = 1.0;
    st->n_disc = st->n;
    st->full_epoch = st->epoch;  // another step function: the next step is computed in full
    st->done = kRunning;
    st->best_delta = INFINITY;
    st->n_best = count;
}

__global__ void step_end_kernel(const Inst *__restrict__ insts, int ninst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    const Inst &I = insts[i];
    SolveState *st = I.state;
    if (st->done != kRunning) return;
    const double dt = st->dt_cur;
    st->n += 1;
    st->epoch += 1;
    st->t += dt;
    const double delta = __longlong_as_double((long long)st->delta_bits);
    st->delta_bits = 0ull;
    if (I.temporal == kEuler) st->parity ^= 1;
    if (st->conv_mode == 0) {
        st->last_delta = delta;
        if (delta < st->tol) st->done = kConverged;
        note_delta(st, delta, st->n);
        anneal(st, st->n);
        apply_limits(st);
    } else {
        st->t_int += dt;
        st->check_interval = st->t_int >= st->dt_report * (1.0 - 1e-12) ? 1 : 0;
        if (!st->check_interval) apply_limits(st);
    }
}

// Interval mode: change across the interval that just closed, and new snapshot.
template <typename T>
__global__ __launch_bounds__(kBlock) void interval_kernel(const Inst *__restrict__ insts,
                                                          const Tile *__restrict__ tiles, int ntiles)
{
    using F = Fields<T>;
    __shared__ double red[kBlock / 64];
    const TileRange r = xcd_range(ntiles);
    for (int c = 0; c < r.count; ++c) {
        const Tile tl = tiles[r.first + c * r.step];
        const Inst &I = insts[tl.inst];
        SolveState *st = I.state;
        if (st->done != kRunning || !st->check_interval) continue;
        const T *cur = (I.temporal == kEuler && st->parity) ? F::A(I) : F::V(I);
        T *snap = F::snap(I);
        double d = 0.0;
        for (int k = 0; k < tl.npt; ++k) {
            const uint32_t node = tl.start + k * kBlock + threadIdx.x;
            if (node < I.npts) {
                T v = cur[node];
                d = nanmax(d, (double)fabs(v - snap[node]));
                snap[node] = v;
            }
        }
        block_max_to(d, &st->idelta_bits, red);
    }
}

__global__ void interval_end_kernel(const Inst *__restrict__ insts, int ninst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    SolveState *st = insts[i].state;
    if (st->done != kRunning || !st->check_interval) return;
    const double d = __longlong_as_double((long long)st->idelta_bits);
    st->idelta_bits = 0ull;
    st->check_interval = 0;
    st->intervals += 1;
    st->t_int = 0.0;
    st->last_delta = d;
    if (d < st->tol) st->done = kConverged;
    note_delta(st, d, st->intervals);
    anneal(st, st->intervals);
    apply_limits(st);
}

// --------------------------------------------------------------------------------------------
// Solve set-up: initial value, input checks, max |l|, CFL rate (one pass over the grid)
// --------------------------------------------------------------------------------------------

template <int DYN>
__device__ __forceinline__ double rate_of(const Inst &I, uint32_t node) { return cfl_rate<DYN>(I, node); }

__global__ __launch_bounds__(kBlock) void init_kernel(const Inst *__restrict__ insts, int inst,
                                                      const double *__restrict__ l64,
                                                      const double *__restrict__ k64, int fp32)
{
    __shared__ double red[kBlock / 64];
    __shared__ unsigned cnt[kBlock / 64];
    const Inst &I = insts[inst];
    SolveState *st = I.state;
    const uint32_t node = blockIdx.x * kBlock + threadIdx.x;
    double lmax = 0.0, rate = 0.0;
    unsigned bad = 0;
    if (node < I.npts) {
        double l = l64[node];
        double v = l;
        bad = isfinite(l) ? 0u : 1u;
        if (k64) {
            double k = k64[node];
            bad |= isfinite(k) ? 0u : 1u;
            v = k < l ? k : l;
        }
        if (I.g64) {  // reach-avoid: start from max(g, .)
            const double gv = I.g64[node];
            bad |= isfinite(gv) ? 0u : 1u;
            v = gv > v ? gv : v;
            if (fp32) const_cast<float *>(I.g32)[node] = (float)gv;
        }
        lmax = fabs(l);
        if (I.act && (node & ((1u << kLocalShift) - 1u)) == 0u) {  // local updates: no marks yet
            I.act[node >> kLocalShift] = -(1 << 30);
            I.act[I.nblocks + (node >> kLocalShift)] = -(1 << 30);
            I.cnt[node >> kLocalShift] = 0ull;
        }
        if (fp32) {
            I.V32[node] = (float)v;
            const_cast<float *>(I.l32)[node] = (float)l;
            if (I.Vs32) I.Vs32[node] = (float)v;
        } else {
            I.V64[node] = v;
            if (I.Vs64) I.Vs64[node] = v;
        }
        switch (I.dyn) {
        case kDynDI: rate = rate_of<kDynDI>(I, node); break;
        case kDynDubins: rate = rate_of<kDynDubins>(I, node); break;
        case kDynUnicycle: rate = rate_of<kDynUnicycle>(I, node); break;
        case kDynQ10XY: rate = rate_of<kDynQ10XY>(I, node); break;
        case kDynQ10Z: rate = rate_of<kDynQ10Z>(I, node); break;
        default: rate = rate_of<kDynQuad>(I, node); break;
        }
    }
    unsigned b = wave_sum(bad);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = b;
    block_max_to(lmax, &st->lmax_bits, red);
    block_max_to(rate, &st->rate_bits, red);
    if (threadIdx.x == 0) {
        unsigned s = 0;
        for (int w = 0; w < kBlock / 64; ++w) s += cnt[w];
        if (s) atomicAdd(&st->nonfinite, s);
    }
}

// dt, phase threshold and first step size, after init_kernel.
// fp32_ulps: 0 for an FP64 phase; otherwise an FP32 phase whose default threshold is that many
// FP32 spacings at max |l| (or tol, whichever is larger)
__global__ void setup_kernel(const Inst *__restrict__ insts, int inst, int fp32_ulps)
{
    if (threadIdx.x != 0) return;
    SolveState *st = insts[inst].state;
    const double rate = __longlong_as_double((long long)st->rate_bits);
    st->max_abs_l = __longlong_as_double((long long)st->lmax_bits);
    double dt = rate > 0.0 ? st->cfl / rate : 1.0;
    if (st->dt_max > 0.0 && dt > st->dt_max) dt = st->dt_max;
    st->dt_nom = dt;
    double tol = st->tol_final;
    const bool fp32_phase = fp32_ulps > 0;
    if (fp32_phase) {
        if (st->tol32_req > 0.0) {
            tol = st->tol32_req;
        } else if (st->max_abs_l > 0.0) {
            int e;
            (void)frexp(st->max_abs_l, &e);
            const double ulp = ldexp(1.0, e - 24);  // FP32 spacing at max |l|
            tol = fmax(tol, (double)fp32_ulps * ulp);
        }
    }
    st->tol = tol;
    if (!fp32_phase) st->stall_window = 0;
    st->best_delta = INFINITY;
    st->n_best = 0;
    st->done = st->nonfinite ? kNonFinite : kRunning;
    st->dt_cur = next_dt(st);
    if (st->max_iter > 0 && st->n >= st->max_iter) st->done = kMaxIter;
}

// --------------------------------------------------------------------------------------------
// FP32 -> FP64 polish hand-over and result extraction
// --------------------------------------------------------------------------------------------

// Reset the per-phase counters for the polish; remembers where the FP32 iterate is.
__global__ void polish_switch_kernel(const Inst *__restrict__ insts, int inst, double shift_req)
{
    if (threadIdx.x != 0) return;
    SolveState *st = insts[inst].state;
    st->tol32_req = shift_req >= 0.0 ? shift_req : 2.0 * st->tol;  // reused: the shift
    if (st->gamma != 1.0) {  // the FP32 phase ended still discounted: the polish is not
        st->n_disc = st->n;
        st->gamma = 1.0;
    }
    st->phase = 1;
    st->full_epoch = st->epoch;  // new arrays: the first FP64 step is computed in full
    st->parity = 0;
    st->done = kRunning;
    st->n = 0;
    st->delta_bits = 0ull;
    st->idelta_bits = 0ull;
    st->check_interval = 0;
    st->t_int = 0.0;
    st->tol = st->tol_final;
    st->best_delta = INFINITY;  // stall detection restarts for the polish
    st->n_best = 0;
    // a stalled polish ends the solve unconverged, so it waits 8 times as long as the FP32 phase
    // (slow tails, where the change creeps towards the threshold, are not stalls)
    if (st->stall_window > 0) st->stall_window = st->stall_window < (1ll << 40) ? 8 * st->stall_window : st->stall_window;
    st->dt_cur = next_dt(st);
}

__global__ __launch_bounds__(kBlock) void polish_init_kernel(const Inst *__restrict__ insts, int inst,
                                                             int parity32)
{
    const Inst &I = insts[inst];
    const uint32_t node = blockIdx.x * kBlock + threadIdx.x;
    if (node >= I.npts) return;
    const float *cur = parity32 ? I.A32 : I.V32;
    const double shift = I.state->tol32_req;
    const double l = I.l64[node];
    const double v = (double)cur[node] + shift;
    double v0 = v < l ? v : l;
    if (I.g64 && I.g64[node] > v0) v0 = I.g64[node];
    I.V64[node] = v0;
    if (I.Vs64) I.Vs64[node] = v0;
}

// Final iterate into the FP64 output array.
__global__ __launch_bounds__(kBlock) void output_kernel(const Inst *__restrict__ insts, int inst,
                                                        int from32, int parity, double *out)
{
    const Inst &I = insts[inst];
    const uint32_t node = blockIdx.x * kBlock + threadIdx.x;
    if (node >= I.npts) return;
    if (from32) {
        const float *cur = parity ? I.A32 : I.V32;
        out[node] = (double)cur[node];
    } else {
        out[node] = parity ? I.A64[node] : I.V64[node];
    }
}

// --------------------------------------------------------------------------------------------
// Launch wrappers
// --------------------------------------------------------------------------------------------

static inline int grid_for(int ntiles, int max_blocks)
{
    if (max_blocks > 0 && ntiles > max_blocks) return max_blocks;
    return ntiles;
}

hipError_t launch_stage(bool fp64, const Inst *insts, const Tile *tiles, int ntiles, int stage,
                        int max_blocks, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const int g = grid_for(ntiles, max_blocks);
    if (fp64)
        hipLaunchKernelGGL(stage_kernel<double>, dim3(g), dim3(kBlock), 0, s, insts, tiles, ntiles, stage);
    else
        hipLaunchKernelGGL(stage_kernel<float>, dim3(g), dim3(kBlock), 0, s, insts, tiles, ntiles, stage);
    return hipGetLastError();
}

// With ev0/ev1 the launch goes through hipExtLaunchKernel, which stamps the two events with the
// kernel's own start and end (so their interval is the kernel's duration, without queue gaps).
template <typename T, int NPT, bool LOCAL>
static void launch_one_npt(int dyn, int spatial, dim3 g, hipStream_t s, const Inst *insts, const Tile *tiles,
                           int ntiles, int stage, hipEvent_t ev0, hipEvent_t ev1)
{
#define HJR_ONE(D, SP)                                                                                         \
    do {                                                                                                       \
        if (ev0 || ev1)                                                                                        \
            hipExtLaunchKernelGGL((stage_kernel_one<T, D, SP, NPT, LOCAL>), g, dim3(kBlock), 0, s, ev0, ev1, 0u, insts, \
                                  tiles, ntiles, stage);                                                       \
        else                                                                                                   \
            hipLaunchKernelGGL((stage_kernel_one<T, D, SP, NPT, LOCAL>), g, dim3(kBlock), 0, s, insts, tiles, ntiles, \
                               stage);                                                                         \
    } while (0)
    const int key = dyn * 8 + spatial;
    switch (key) {
    case kDynDI * 8 + kUpwind1: HJR_ONE(kDynDI, kUpwind1); break;
    case kDynDI * 8 + kWeno5: HJR_ONE(kDynDI, kWeno5); break;
    case kDynDubins * 8 + kUpwind1: HJR_ONE(kDynDubins, kUpwind1); break;
    case kDynDubins * 8 + kWeno5: HJR_ONE(kDynDubins, kWeno5); break;
    case kDynUnicycle * 8 + kUpwind1: HJR_ONE(kDynUnicycle, kUpwind1); break;
    case kDynUnicycle * 8 + kWeno5: HJR_ONE(kDynUnicycle, kWeno5); break;
    case kDynQuad * 8 + kUpwind1: HJR_ONE(kDynQuad, kUpwind1); break;
    case kDynQuad * 8 + kWeno5: HJR_ONE(kDynQuad, kWeno5); break;
    case kDynQ10XY * 8 + kUpwind1: HJR_ONE(kDynQ10XY, kUpwind1); break;
    case kDynQ10XY * 8 + kWeno5: HJR_ONE(kDynQ10XY, kWeno5); break;
    case kDynQ10Z * 8 + kUpwind1: HJR_ONE(kDynQ10Z, kUpwind1); break;
    case kDynQ10Z * 8 + kWeno5: HJR_ONE(kDynQ10Z, kWeno5); break;
    default: break;
    }
#undef HJR_ONE
}

template <typename T>
static void launch_one(int dyn, int spatial, int npt, bool local, dim3 g, hipStream_t s, const Inst *insts,
                       const Tile *tiles, int ntiles, int stage, hipEvent_t ev0, hipEvent_t ev1)
{
    if (local) {  // local-update groups always use 4 nodes per thread
        launch_one_npt<T, 4, true>(dyn, spatial, g, s, insts, tiles, ntiles, stage, ev0, ev1);
        return;
    }
    switch (npt) {
    case 1: launch_one_npt<T, 1, false>(dyn, spatial, g, s, insts, tiles, ntiles, stage, ev0, ev1); break;
    case 2: launch_one_npt<T, 2, false>(dyn, spatial, g, s, insts, tiles, ntiles, stage, ev0, ev1); break;
    case 8: launch_one_npt<T, 8, false>(dyn, spatial, g, s, insts, tiles, ntiles, stage, ev0, ev1); break;
    default: launch_one_npt<T, 4, false>(dyn, spatial, g, s, insts, tiles, ntiles, stage, ev0, ev1); break;
    }
}

hipError_t launch_stage_one(bool fp64, int dyn, int spatial, int npt, const Inst *insts, const Tile *tiles, int ntiles,
                            int stage, int max_blocks, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, bool local)
{
    if (ntiles <= 0) return hipSuccess;
    const dim3 g(grid_for(ntiles, max_blocks));
    if (fp64)
        launch_one<double>(dyn, spatial, npt, local, g, s, insts, tiles, ntiles, stage, ev0, ev1);
    else
        launch_one<float>(dyn, spatial, npt, local, g, s, insts, tiles, ntiles, stage, ev0, ev1);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_march_t(int dyn, int spatial, bool brick, dim3 g, hipStream_t s, const Inst *insts,
                                 const MTile *tiles, int ntiles, int stage, hipEvent_t ev0, hipEvent_t ev1)
{
#define HJR_MARCH_KB(K, B)                                                                                     \
    do {                                                                                                       \
        if (ev0 || ev1)                                                                                        \
            hipExtLaunchKernelGGL((K), g, dim3(B), 0, s, ev0, ev1, 0u, insts, tiles, ntiles, stage);           \
        else                                                                                                   \
            hipLaunchKernelGGL((K), g, dim3(B), 0, s, insts, tiles, ntiles, stage);                            \
    } while (0)
#define HJR_MARCH_K(K) HJR_MARCH_KB(K, kBlock)
    if (brick) {
        // bricks exist for the 6-D model with the upwind stencil only
        if (dyn != kDynQuad || spatial != kUpwind1) return hipErrorInvalidValue;
        HJR_MARCH_KB((march_brick_kernel<T, kDynQuad>), kBrickThreads);
        return hipSuccess;
    }
#define HJR_MARCH(D)                                                                                           \
    do {                                                                                                       \
        if (spatial == kWeno5)                                                                                 \
            HJR_MARCH_K((march_kernel_w5<T, D>));                                                              \
        else                                                                                                   \
            HJR_MARCH_K((march_kernel<T, D>));                                                                 \
    } while (0)
    switch (dyn) {
    case kDynDI: HJR_MARCH(kDynDI); break;
    case kDynDubins: HJR_MARCH(kDynDubins); break;
    case kDynUnicycle: HJR_MARCH(kDynUnicycle); break;
    case kDynQuad: HJR_MARCH(kDynQuad); break;
    case kDynQ10XY: HJR_MARCH(kDynQ10XY); break;
    case kDynQ10Z: HJR_MARCH(kDynQ10Z); break;
    default: break;
    }
#undef HJR_MARCH
#undef HJR_MARCH_K
#undef HJR_MARCH_KB
    return hipSuccess;
}

// Rounds of 8 blocks, one per XCD, interleaved workgroup by workgroup; the blocks are taken
// largest first (the blocks at the high ends of the index ranges are smaller) so that the
// blocks of a round are of about the same size and little padding is needed; a last round of
// fewer blocks is appended in plain order.
static void interleave_blocks(int inst, std::vector<std::vector<MTile>> &blocks, std::vector<MTile> &out)
{
    std::stable_sort(blocks.begin(), blocks.end(),
                     [](const std::vector<MTile> &a, const std::vector<MTile> &b) { return a.size() > b.size(); });
    const size_t nb8 = blocks.size() / 8 * 8;
    for (size_t r = 0; r < nb8; r += 8) {
        size_t m = 0;
        for (size_t x = 0; x < 8; ++x) m = std::max(m, blocks[r + x].size());
        for (size_t k = 0; k < m; ++k)
            for (size_t x = 0; x < 8; ++x)
                out.push_back(k < blocks[r + x].size() ? blocks[r + x][k] : MTile{inst, 0u, 0, 0, 0u});
    }
    for (size_t r = nb8; r < blocks.size(); ++r) out.insert(out.end(), blocks[r].begin(), blocks[r].end());
}

void march_tiles(int inst, int ndim, const int *n, int len, std::vector<MTile> &out)
{
    const int n0 = n[0];
    const int L = len > 0 ? std::min(len, n0) : n0;
    uint64_t P = 1;
    for (int d = 1; d < ndim; ++d) P *= (uint64_t)n[d];
    // rows of consecutive columns: over dims 1 and 2 when the dims after them hold at least
    // 4 kBlock columns, else over dim 1 when the dims after it do, else one row
    const uint64_t minrow = 4 * (uint64_t)kBlock;
    uint64_t na = 1, nb = 1;
    if (ndim >= 4 && P / ((uint64_t)n[1] * n[2]) >= minrow) {
        na = (uint64_t)n[1];
        nb = (uint64_t)n[2];
    } else if (ndim >= 3 && P / (uint64_t)n[1] >= minrow) {
        na = (uint64_t)n[1];
    }
    const uint64_t R = P / (na * nb);                     // columns per row
    const uint64_t tr = (R + kBlock - 1) / kBlock;        // tiles per row
    // blocks of about 256 column tiles: Bt neighbouring tiles of Ba x Bb neighbouring rows
    const uint64_t Bt = std::min<uint64_t>(tr, 16);
    uint64_t Ba = 1, Bb = 1;
    const uint64_t rest = std::max<uint64_t>(1, 256 / Bt);
    if (nb > 1) {
        while ((Ba + 1) * (Ba + 1) <= rest) ++Ba;
        Bb = Ba;
    } else {
        Ba = rest;
    }
    Ba = std::min(Ba, na);
    Bb = std::min(Bb, nb);
    std::vector<std::vector<MTile>> blocks;
    for (uint64_t a0 = 0; a0 < na; a0 += Ba)
        for (uint64_t b0 = 0; b0 < nb; b0 += Bb)
            for (uint64_t t0 = 0; t0 < tr; t0 += Bt) {
                std::vector<MTile> blk;
                for (uint64_t a = a0; a < std::min(na, a0 + Ba); ++a)
                    for (uint64_t b = b0; b < std::min(nb, b0 + Bb); ++b)
                        for (uint64_t t = t0; t < std::min(tr, t0 + Bt); ++t) {
                            const uint64_t c0 = (a * nb + b) * R + t * kBlock;
                            const uint32_t cn = (uint32_t)std::min<uint64_t>(kBlock, R - t * kBlock);
                            for (int i0 = 0; i0 < n0; i0 += L)
                                blk.push_back(MTile{inst, (uint32_t)c0, i0, std::min(L, n0 - i0), cn});
                        }
                blocks.push_back(std::move(blk));
            }
    interleave_blocks(inst, blocks, out);
}

void march_brick_tiles(int inst, int ndim, const int *n, std::vector<MTile> &out)
{
    if (ndim != 6) return;
    const uint64_t R = (uint64_t)n[4] * n[5];            // columns per row
    const uint64_t s3 = R, s2 = (uint64_t)n[3] * s3, s1 = (uint64_t)n[2] * s2;
    const uint64_t segs = (R + kBrickSeg - 1) / kBrickSeg;
    const uint64_t q1 = (n[1] + 1) / 2, q2 = (n[2] + 1) / 2, q3 = (n[3] + 1) / 2;  // row pairs per dim
    // blocks of about 64 bricks (the workgroups an XCD holds at two per CU): all segments of
    // 2 x 2 x B3 neighbouring bricks
    const uint64_t B1 = std::min<uint64_t>(2, q1), B2 = std::min<uint64_t>(2, q2);
    const uint64_t k = B1 * B2 * segs;
    const uint64_t B3 = std::min<uint64_t>(q3, std::max<uint64_t>(1, (64 + k / 2) / k));
    std::vector<std::vector<MTile>> blocks;
    for (uint64_t a0 = 0; a0 < q1; a0 += B1)
        for (uint64_t b0 = 0; b0 < q2; b0 += B2)
            for (uint64_t c0 = 0; c0 < q3; c0 += B3) {
                std::vector<MTile> blk;
                for (uint64_t a = a0; a < std::min(q1, a0 + B1); ++a)
                    for (uint64_t b = b0; b < std::min(q2, b0 + B2); ++b)
                        for (uint64_t c = c0; c < std::min(q3, c0 + B3); ++c)
                            for (uint64_t g = 0; g < segs; ++g) {
                                const uint64_t col = 2 * a * s1 + 2 * b * s2 + 2 * c * s3 + g * kBrickSeg;
                                const uint32_t cn = (uint32_t)std::min<uint64_t>(kBrickSeg, R - g * kBrickSeg);
                                blk.push_back(MTile{inst, (uint32_t)col, 0, n[0], cn});
                            }
                blocks.push_back(std::move(blk));
            }
    interleave_blocks(inst, blocks, out);
}

hipError_t launch_march(bool fp64, int dyn, int spatial, bool brick, const Inst *insts, const MTile *tiles,
                        int ntiles, int stage, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (ntiles <= 0) return hipSuccess;
    const dim3 g(ntiles);
    const hipError_t e = fp64 ? launch_march_t<double>(dyn, spatial, brick, g, s, insts, tiles, ntiles, stage, ev0, ev1)
                              : launch_march_t<float>(dyn, spatial, brick, g, s, insts, tiles, ntiles, stage, ev0, ev1);
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_step_end(const Inst *insts, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(step_end_kernel, dim3((ninst + 63) / 64), dim3(64), 0, s, insts, ninst);
    return hipGetLastError();
}

hipError_t launch_interval(bool fp64, const Inst *insts, const Tile *tiles, int ntiles, int max_blocks,
                           hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    const int g = grid_for(ntiles, max_blocks);
    if (fp64)
        hipLaunchKernelGGL(interval_kernel<double>, dim3(g), dim3(kBlock), 0, s, insts, tiles, ntiles);
    else
        hipLaunchKernelGGL(interval_kernel<float>, dim3(g), dim3(kBlock), 0, s, insts, tiles, ntiles);
    return hipGetLastError();
}

hipError_t launch_interval_end(const Inst *insts, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(interval_end_kernel, dim3((ninst + 63) / 64), dim3(64), 0, s, insts, ninst);
    return hipGetLastError();
}

hipError_t launch_init(const Inst *insts, int inst, uint32_t npts, const double *l64, const double *k64,
                       int fp32_ulps, hipStream_t s)
{
    const int g = (int)((npts + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(init_kernel, dim3(g), dim3(kBlock), 0, s, insts, inst, l64, k64, fp32_ulps > 0 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(64), 0, s, insts, inst, fp32_ulps);
    return hipGetLastError();
}

hipError_t launch_polish(const Inst *insts, int inst, uint32_t npts, int parity32, double shift_req,
                         hipStream_t s)
{
    hipLaunchKernelGGL(polish_switch_kernel, dim3(1), dim3(64), 0, s, insts, inst, shift_req);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int g = (int)((npts + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(polish_init_kernel, dim3(g), dim3(kBlock), 0, s, insts, inst, parity32);
    return hipGetLastError();
}

hipError_t launch_output(const Inst *insts, int inst, uint32_t npts, bool from32, int parity, double *out,
                         hipStream_t s)
{
    const int g = (int)((npts + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(output_kernel, dim3(g), dim3(kBlock), 0, s, insts, inst, from32 ? 1 : 0, parity, out);
    return hipGetLastError();
}

}  // namespace hjr
