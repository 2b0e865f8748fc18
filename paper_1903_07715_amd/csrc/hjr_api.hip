// hjr_api.hip -- host side of libhjr: validation, device memory, the batched step engine, the
// C ABI declared in include/hjr.h and the serving context.
//
// One Engine advances a set of solve instances together.  Each instance owns its device
// buffers and a SolveState slot; the engine keeps the Inst descriptors and the tile lists of the
// FP32-phase and FP64-phase instances in device memory.  A chunk is m time steps issued without
// host round trips: per step, one launch per RK stage and precision over all tiles, then one
// bookkeeping launch that advances every instance's clock, tests its convergence and freezes it
// when done (frozen instances make every later kernel return at once).  After a chunk the host
// reads all states back with one copy, hands converged FP32 instances over to the FP64 polish,
// finishes completed instances, admits waiting ones and rebuilds the tile lists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/hjr.h"
#include "fastdiv.hpp"
#include "hjr_control.hpp"
#include "hjr_kernels.hpp"

namespace hjr {

// --------------------------------------------------------------------------------------------
// Errors
// --------------------------------------------------------------------------------------------

static thread_local std::string g_last_error;

static hjr_status fail(hjr_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HJR_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(HJR_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));        \
    } while (0)

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// --------------------------------------------------------------------------------------------
// Kernel timing (process-wide)
// --------------------------------------------------------------------------------------------

static std::atomic<int> g_profile_on{0};
static std::mutex g_profile_mu;
static hjr_profile g_profile{};

// --------------------------------------------------------------------------------------------
// Validation
// --------------------------------------------------------------------------------------------

static int dyn_ndim(int id)
{
    switch (id) {
    case HJR_DYN_DOUBLE_INTEGRATOR: return 2;
    case HJR_DYN_DUBINS3: return 3;
    case HJR_DYN_UNICYCLE4: return 4;
    case HJR_DYN_QUAD6: return 6;
    case HJR_DYN_QUAD10_XY: return 4;
    case HJR_DYN_QUAD10_Z: return 2;
    default: return -1;
    }
}

static int dyn_nparams(int id)
{
    switch (id) {
    case HJR_DYN_DOUBLE_INTEGRATOR: return 3;
    case HJR_DYN_DUBINS3: return 4;
    case HJR_DYN_UNICYCLE4: return 4;
    case HJR_DYN_QUAD6: return 9;
    case HJR_DYN_QUAD10_XY: return 6;
    case HJR_DYN_QUAD10_Z: return 6;
    default: return -1;
    }
}

static hjr_status validate_grid(const hjr_grid *g, int spatial, uint64_t *npts_out);

static hjr_status validate(const hjr_grid *g, const hjr_dynamics *dy, int spatial, uint64_t *npts_out)
{
    if (!g || !dy) return fail(HJR_ERR_INVALID_ARG, "grid and dynamics must not be NULL");
    if (g->ndim < 1 || g->ndim > HJR_MAX_DIM) return fail(HJR_ERR_INVALID_ARG, "ndim %d out of range", g->ndim);
    const int nd = dyn_ndim(dy->id);
    if (nd < 0) return fail(HJR_ERR_UNSUPPORTED, "unknown dynamics id %d", dy->id);
    if (nd != g->ndim)
        return fail(HJR_ERR_INVALID_ARG, "dynamics %d has %d states but the grid has %d dims", dy->id, nd, g->ndim);
    if (dy->n_params != dyn_nparams(dy->id))
        return fail(HJR_ERR_INVALID_ARG, "dynamics %d takes %d parameters, got %d", dy->id, dyn_nparams(dy->id),
                    dy->n_params);
    for (int i = 0; i < dy->n_params; ++i)
        if (!std::isfinite(dy->params[i])) return fail(HJR_ERR_INVALID_ARG, "parameter %d is not finite", i);
    const double *q = dy->params;
    switch (dy->id) {
    case HJR_DYN_DOUBLE_INTEGRATOR:
        if (q[0] < 0 || q[2] < 0) return fail(HJR_ERR_INVALID_ARG, "bounds must be non-negative");
        break;
    case HJR_DYN_DUBINS3:
        if (q[1] < 0 || q[2] < 0 || q[3] < 0) return fail(HJR_ERR_INVALID_ARG, "bounds must be non-negative");
        break;
    case HJR_DYN_UNICYCLE4:
        if (q[0] < 0 || q[1] < 0 || q[2] < 0 || (q[3] != 0.0 && q[3] != 1.0))
            return fail(HJR_ERR_INVALID_ARG, "bad unicycle parameters");
        break;
    case HJR_DYN_QUAD6:
        if (!(q[1] > 0) || q[2] < 0 || q[3] < 0 || q[2] >= 1.5 || q[3] >= 1.5 || q[4] > q[5] || q[6] < 0 ||
            q[7] < 0 || q[8] < 0)
            return fail(HJR_ERR_INVALID_ARG, "bad quadrotor parameters");
        break;
    case HJR_DYN_QUAD10_XY: {
        if (q[3] < 0 || q[4] < 0 || q[5] < 0) return fail(HJR_ERR_INVALID_ARG, "n0, S_max and dbar must be non-negative");
        const double half_pi = 1.5707963267948966;
        if (!(g->lo[2] > -half_pi) || !(g->hi[2] < half_pi) || ((g->periodic_mask >> 2) & 1u))
            return fail(HJR_ERR_INVALID_ARG, "the pitch/roll range must lie inside (-pi/2, pi/2) and not wrap");
        break;
    }
    case HJR_DYN_QUAD10_Z:
        if (q[1] < 0 || !(q[2] > 0) || q[3] > q[4] || q[5] < 0)
            return fail(HJR_ERR_INVALID_ARG, "need k_T >= 0, m > 0, T_min <= T_max, dbar >= 0");
        break;
    }
    return validate_grid(g, spatial, npts_out);
}

static hjr_status validate_grid(const hjr_grid *g, int spatial, uint64_t *npts_out)
{
    if (!g) return fail(HJR_ERR_INVALID_ARG, "grid must not be NULL");
    if (g->ndim < 1 || g->ndim > HJR_MAX_DIM) return fail(HJR_ERR_INVALID_ARG, "ndim %d out of range", g->ndim);
    if (spatial != HJR_UPWIND1 && spatial != HJR_WENO5)
        return fail(HJR_ERR_INVALID_ARG, "bad spatial scheme %d", spatial);
    uint64_t N = 1;
    for (int d = 0; d < g->ndim; ++d) {
        const int minn = spatial == HJR_WENO5 ? 7 : 3;
        if (g->n[d] < minn) return fail(HJR_ERR_INVALID_ARG, "dim %d has %d nodes (< %d)", d, g->n[d], minn);
        if (!std::isfinite(g->lo[d]) || !std::isfinite(g->hi[d]) || !(g->hi[d] > g->lo[d]))
            return fail(HJR_ERR_INVALID_ARG, "dim %d: need lo < hi", d);
        N *= (uint64_t)g->n[d];
        if (N >= (1ull << 29)) return fail(HJR_ERR_UNSUPPORTED, "grid has 2^29 or more nodes");
    }
    if (g->periodic_mask >> g->ndim) return fail(HJR_ERR_INVALID_ARG, "periodic_mask names a missing dim");
    *npts_out = N;
    return HJR_OK;
}

static hjr_status validate_opts(const hjr_options *o)
{
    if (!o) return fail(HJR_ERR_INVALID_ARG, "options must not be NULL");
    if (o->game != HJR_AVOID && o->game != HJR_REACH) return fail(HJR_ERR_INVALID_ARG, "bad game %d", o->game);
    if (o->spatial != HJR_UPWIND1 && o->spatial != HJR_WENO5)
        return fail(HJR_ERR_INVALID_ARG, "bad spatial scheme %d", o->spatial);
    if (o->temporal != HJR_EULER && o->temporal != HJR_TVDRK3)
        return fail(HJR_ERR_INVALID_ARG, "bad temporal scheme %d", o->temporal);
    if (o->precision < HJR_FP64 || o->precision > HJR_FP32_POLISH64)
        return fail(HJR_ERR_INVALID_ARG, "bad precision %d", o->precision);
    if (o->conv_mode != HJR_CONV_PER_STEP && o->conv_mode != HJR_CONV_PER_INTERVAL)
        return fail(HJR_ERR_INVALID_ARG, "bad conv_mode %d", o->conv_mode);
    if (!(o->cfl > 0.0) || !(o->cfl <= 1.0)) return fail(HJR_ERR_INVALID_ARG, "cfl must be in (0, 1]");
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(HJR_ERR_INVALID_ARG, "tol must be > 0");
    if (!(o->tol_fp32 >= 0.0)) return fail(HJR_ERR_INVALID_ARG, "tol_fp32 must be >= 0");
    if (o->conv_mode == HJR_CONV_PER_INTERVAL && !(o->dt_report > 0.0))
        return fail(HJR_ERR_INVALID_ARG, "interval mode needs dt_report > 0");
    if (!(o->t_max >= 0.0) || !(o->dt_max >= 0.0)) return fail(HJR_ERR_INVALID_ARG, "t_max, dt_max must be >= 0");
    if (o->max_iter < 0) return fail(HJR_ERR_INVALID_ARG, "max_iter must be >= 0");
    if (o->steps_per_sync < 0) return fail(HJR_ERR_INVALID_ARG, "steps_per_sync must be >= 0");
    return HJR_OK;
}

// --------------------------------------------------------------------------------------------
// Device memory: a process-wide caching pool (allocation is slow next to a solve of a small grid)
// --------------------------------------------------------------------------------------------

class Pool {
public:
    static Pool &get()
    {
        static Pool *p = new Pool();  // never destroyed: cached blocks live until process exit
        return *p;
    }
    hipError_t alloc(void **ptr, size_t bytes)
    {
        bytes = round(bytes);
        int dev = 0;
        (void)hipGetDevice(&dev);
        {
            std::lock_guard<std::mutex> g(mu_);
            auto &fl = free_[key(dev, bytes)];
            if (!fl.empty()) {
                *ptr = fl.back();
                fl.pop_back();
                size_[*ptr] = bytes;
                return hipSuccess;
            }
        }
        hipError_t e = hipMalloc(ptr, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim(dev);
            e = hipMalloc(ptr, bytes);
        }
        if (e == hipSuccess) {
            std::lock_guard<std::mutex> g(mu_);
            size_[*ptr] = bytes;
            dev_[*ptr] = dev;
        }
        return e;
    }
    void release(void *ptr)
    {
        if (!ptr) return;
        std::lock_guard<std::mutex> g(mu_);
        auto it = size_.find(ptr);
        if (it == size_.end()) return;
        free_[key(dev_[ptr], it->second)].push_back(ptr);
        size_.erase(it);
    }

private:
    static size_t round(size_t b)
    {
        size_t r = 1 << 20;
        while (r < b) r <<= 1;
        return r;
    }
    static uint64_t key(int dev, size_t b) { return ((uint64_t)dev << 56) | (uint64_t)b; }
    void trim(int dev)
    {
        std::lock_guard<std::mutex> g(mu_);
        for (auto &kv : free_) {
            if ((int)(kv.first >> 56) != dev) continue;
            for (void *p : kv.second) {
                (void)hipFree(p);
                dev_.erase(p);
            }
            kv.second.clear();
        }
    }
    std::mutex mu_;
    std::map<uint64_t, std::vector<void *>> free_;
    std::unordered_map<void *, size_t> size_;
    std::unordered_map<void *, int> dev_;
};

// --------------------------------------------------------------------------------------------
// One solve instance
// --------------------------------------------------------------------------------------------

struct Request {
    hjr_grid grid;
    hjr_dynamics dyn;
    hjr_options opts;
    const double *l_dev = nullptr;   // FP64 target function (caller or owned)
    const double *k_dev = nullptr;
    const double *g_dev = nullptr;   // reach-avoid constraint function (caller or owned), or null
    double *V_dev = nullptr;         // FP64 output (caller or owned)
    std::vector<uint32_t> dep_off, dep;  // local updates: block dependency lists (empty: off)
    uint64_t npts = 0;
    size_t bytes = 0;                // working memory
    void *mem = nullptr;             // owned working buffer
    Inst inst{};
    int slot = -1;
    int phase = 0;                   // 0 first phase, 1 polish
    bool fp32_first = false;
    int64_t iters0 = 0;
    hjr_result result{};
    hjr_status status = HJR_PENDING;
    int64_t ticket = 0;
    double t_submit = 0.0, t_start = 0.0;
    bool done = false;
    // march tiles of this request in its slot for launch configuration mtiles_cfg (0: none
    // built); kept across engine rebuilds, which happen at every admission, hand-over and
    // completion
    std::vector<MTile> mtiles;
    int mtiles_cfg = 0;
};

static void make_constants(const hjr_dynamics &dy, double c[8])
{
    for (int i = 0; i < 8; ++i) c[i] = 0.0;
    const double *q = dy.params;
    switch (dy.id) {
    case HJR_DYN_DOUBLE_INTEGRATOR:
        c[0] = std::fabs(q[1]) * q[0];
        c[1] = q[2];
        break;
    case HJR_DYN_DUBINS3:
    case HJR_DYN_UNICYCLE4:
        for (int i = 0; i < 4; ++i) c[i] = q[i];
        break;
    case HJR_DYN_QUAD6: {
        const double g = q[0], m = q[1];
        c[0] = g * std::tan(q[3]);
        c[1] = g * std::tan(q[2]);
        c[2] = q[5] / m - g;
        c[3] = q[4] / m - g;
        c[4] = q[6];
        c[5] = q[7];
        c[6] = q[8];
        c[7] = std::max(std::fabs(c[2]), std::fabs(c[3]));
        break;
    }
    case HJR_DYN_QUAD10_XY:
        c[0] = q[0];          // g
        c[1] = q[1];          // d0
        c[2] = q[2];          // d1
        c[3] = q[3] * q[4];   // n0 S_max
        c[4] = q[5];          // dbar
        break;
    case HJR_DYN_QUAD10_Z: {
        const double g = q[0], a = q[1] / q[2];
        c[0] = a * q[4] - g;
        c[1] = a * q[3] - g;
        c[2] = q[5];
        c[3] = std::max(std::fabs(c[0]), std::fabs(c[1]));
        break;
    }
    }
}

static double grid_dx(const hjr_grid &g, int d)
{
    return ((g.periodic_mask >> d) & 1u) ? (g.hi[d] - g.lo[d]) / g.n[d] : (g.hi[d] - g.lo[d]) / (g.n[d] - 1);
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Working memory of one request, carved from one pool block.
struct Layout {
    size_t V32, A32, B32, l32, g32, Vs32, A64, B64, Vs64, V64, l64, k64, g64, act, cnt, dep_off, dep, tab32, tab64,
        total;
    int ntab;
};

static Layout plan_layout(const Request &r, bool own_io, bool has_g)
{
    Layout L{};
    const size_t N = r.npts;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    const bool fp32 = r.opts.precision != HJR_FP64;
    const bool fp64 = r.opts.precision != HJR_FP32;
    const bool interval = r.opts.conv_mode == HJR_CONV_PER_INTERVAL;
    const size_t none = (size_t)-1;
    L.V32 = fp32 ? take(N * 4) : none;
    L.A32 = fp32 ? take(N * 4) : none;
    L.B32 = fp32 && r.opts.temporal == HJR_TVDRK3 ? take(N * 4) : none;
    L.l32 = fp32 ? take(N * 4) : none;
    L.g32 = fp32 && has_g ? take(N * 4) : none;
    L.Vs32 = fp32 && interval ? take(N * 4) : none;
    L.A64 = fp64 ? take(N * 8) : none;
    L.B64 = fp64 && r.opts.temporal == HJR_TVDRK3 ? take(N * 8) : none;
    L.Vs64 = fp64 && interval ? take(N * 8) : none;
    L.V64 = own_io ? take(N * 8) : none;
    L.l64 = own_io ? take(N * 8) : none;
    L.k64 = own_io ? take(N * 8) : none;
    L.g64 = own_io && has_g ? take(N * 8) : none;
    const bool local = !r.dep_off.empty();
    const size_t nb = local ? r.dep_off.size() - 1 : 0;
    L.act = local ? take(2 * nb * 4) : none;
    L.cnt = local ? take(nb * 8) : none;
    L.dep_off = local ? take(r.dep_off.size() * 4) : none;
    L.dep = local ? take(r.dep.size() * 4) : none;
    int nt = 0;
    for (int d = 0; d < r.grid.ndim; ++d) nt += r.grid.n[d];
    nt += 2 * r.grid.n[std::min(2, r.grid.ndim - 1)];
    L.ntab = nt;
    L.tab32 = take((size_t)nt * 4);
    L.tab64 = take((size_t)nt * 8);
    L.total = off;
    return L;
}

static size_t request_bytes(const Request &r, bool own_io) { return plan_layout(r, own_io, r.g_dev != nullptr).total; }

// Grid part of an instance descriptor: sizes, strides, division constants, spacings.
static void fill_grid(const hjr_grid &g, uint64_t npts, Inst &I)
{
    I.ndim = g.ndim;
    I.npts = (uint32_t)npts;
    I.periodic = g.periodic_mask;
    uint32_t s = 1;
    for (int d = g.ndim - 1; d >= 0; --d) {
        I.n[d] = g.n[d];
        I.stride[d] = s;
        s *= (uint32_t)g.n[d];
        FastDivParams p = fastdiv_params((uint32_t)g.n[d]);
        I.div[d].mul = p.mul;
        I.div[d].shift = p.shift;
        I.div[d].d = (uint32_t)g.n[d];
        const double dx = grid_dx(g, d);
        I.inv_dx64[d] = 1.0 / dx;
        I.inv_dx32[d] = (float)(1.0 / dx);
        I.hinv_dx64[d] = 0.5 / dx;
        I.hinv_dx32[d] = (float)(0.5 / dx);
        I.eps0_64[d] = 4e-18 * dx * dx;
        I.eps0_32[d] = std::max((float)I.eps0_64[d], FLT_MIN);  // kept normal in FP32
    }
}

// Fill the Inst descriptor and the coordinate tables (host staging `tab64`, `tab32`).
static void build_inst(Request &r, char *base, const Layout &L, std::vector<double> &tab64,
                       std::vector<float> &tab32, SolveState *state_dev)
{
    Inst &I = r.inst;
    std::memset(&I, 0, sizeof I);
    const hjr_grid &g = r.grid;
    I.ndim = g.ndim;
    I.dyn = r.dyn.id;
    I.spatial = r.opts.spatial;
    I.temporal = r.opts.temporal;
    I.game = r.opts.game;
    I.brs = r.opts.brs;
    I.nstages = r.opts.temporal == HJR_TVDRK3 ? 3 : 1;
    fill_grid(g, r.npts, I);
    double c[8];
    make_constants(r.dyn, c);
    for (int i = 0; i < 8; ++i) {
        I.c64[i] = c[i];
        I.c32[i] = (float)c[i];
    }
    tab64.assign((size_t)L.ntab, 0.0);
    int off = 0;
    for (int d = 0; d < g.ndim; ++d) {
        I.coord_off[d] = off;
        const double dx = grid_dx(g, d);
        for (int j = 0; j < g.n[d]; ++j) tab64[off + j] = g.lo[d] + (double)j * dx;
        off += g.n[d];
    }
    I.trig_off = -1;
    if (r.dyn.id == HJR_DYN_DUBINS3 || r.dyn.id == HJR_DYN_UNICYCLE4) {
        I.trig_off = off;
        const int nt = g.n[2];
        for (int j = 0; j < nt; ++j) {
            const double th = tab64[I.coord_off[2] + j];
            tab64[off + j] = std::cos(th);
            tab64[off + nt + j] = std::sin(th);
        }
    } else if (r.dyn.id == HJR_DYN_QUAD10_XY) {
        I.trig_off = off;  // tan of the pitch/roll coordinate
        for (int j = 0; j < g.n[2]; ++j) tab64[off + j] = std::tan(tab64[I.coord_off[2] + j]);
    }
    tab32.resize(tab64.size());
    for (size_t i = 0; i < tab64.size(); ++i) tab32[i] = (float)tab64[i];
    auto at = [&](size_t o) -> char * { return o == (size_t)-1 ? nullptr : base + o; };
    I.tab32 = (const float *)at(L.tab32);
    I.tab64 = (const double *)at(L.tab64);
    I.V32 = (float *)at(L.V32);
    I.A32 = (float *)at(L.A32);
    I.B32 = (float *)at(L.B32);
    I.l32 = (const float *)at(L.l32);
    I.g32 = (const float *)at(L.g32);
    I.Vs32 = (float *)at(L.Vs32);
    I.A64 = (double *)at(L.A64);
    I.B64 = (double *)at(L.B64);
    I.Vs64 = (double *)at(L.Vs64);
    I.V64 = r.V_dev;
    I.l64 = r.l_dev;
    I.g64 = r.g_dev;
    I.act = (int *)at(L.act);
    I.cnt = (unsigned long long *)at(L.cnt);
    I.nblocks = r.dep_off.empty() ? 0u : (uint32_t)(r.dep_off.size() - 1);
    I.dep_off = (const uint32_t *)at(L.dep_off);
    I.dep = (const uint32_t *)at(L.dep);
    I.state = state_dev;
}

static SolveState initial_state(const Request &r)
{
    SolveState st;
    std::memset(&st, 0, sizeof st);
    st.tol_final = r.opts.tol;
    st.tol = r.opts.tol;
    st.tol32_req = r.opts.tol_fp32;
    st.t_max = r.opts.t_max;
    st.dt_report = r.opts.dt_report;
    st.dt_max = r.opts.dt_max;
    st.cfl = r.opts.cfl;
    st.max_iter = r.opts.max_iter;
    st.conv_mode = r.opts.conv_mode;
    st.stall_window = r.opts.stall_window == 0 ? 128 : (r.opts.stall_window < 0 ? 0 : r.opts.stall_window);
    st.last_delta = INFINITY;
    st.gamma = r.opts.discount > 0.0 ? r.opts.discount : 1.0;
    st.done = kRunning;  // set properly by setup_kernel
    return st;
}

// --------------------------------------------------------------------------------------------
// Autotuner: nodes per thread of the stage kernels, per (precision, model, scheme, size class).
// The per-node arithmetic is identical for every candidate (results are bitwise equal), so the
// tuner explores on the real solve: successive chunks of steps run with successive candidates,
// the median duration of each candidate's stage launches is recorded, and once every candidate
// has been timed the fastest is used from then on, for the rest of the process.  The default is
// timed first and again last (its best time counts), so a clock that is still rising during the
// first chunks does not count against it.  With
// HJR_TUNE_CACHE=<file> the choices are also kept in a small JSON file for later processes.
// --------------------------------------------------------------------------------------------

// Launch configurations: 1, 2, 4, 8 = flat tiles with that many nodes per thread; kMarchFull =
// the plane-march kernel over whole dim-0 lines, -8, -4, -2 = the same in runs of that many
// planes (more threads; per run, the planes before and after it are read again: two extra loads
// for upwind, six and one extra dim-0 interface for WENO5).  The march kernels serve groups whose
// dim-0 planes hold enough columns to fill the device at one thread per column.  kMarchBrick =
// the brick variant over whole lines (6-D grids, upwind: pairs of rows of dims 1..3 share their
// far neighbours through LDS).
static const int kMarchFull = -1;
static const int kMarch8 = -8;
static const int kMarchBrick = -16;
static const int kFlatSchedule[] = {4, 2, 8, 1, 4};
static const int kMarchSchedule[] = {4, kMarchFull, 2, 8, 1, kMarch8, 4};
// 6-D groups: the flat kernels at 1 and 2 nodes per thread are left out (on the 25^6 grid they
// are 2.5-3x slower than the brick kernel in both precisions), so that the few FP64 polish
// steps of a solve finish the search sooner
static const int kMarchBrickSchedule[] = {4, kMarchBrick, kMarchFull, 8, kMarch8, 4};
// WENO5: runs of 4 or 8 planes (whole lines leave too few threads, runs of 2 pay the run start
// too often: both measured slower everywhere)
static const int kMarchW5Schedule[] = {4, -4, 2, 8, kMarch8, 1, 4};
static const uint64_t kMarchMinColumns = 8192;

static bool valid_config(int c)
{
    return c == 1 || c == 2 || c == 4 || c == 8 || c == kMarchFull || c == -2 || c == -4 || c == kMarch8 ||
           c == kMarchBrick;
}
static bool is_march(int c) { return c < 0; }

// Whether the brick kernel serves a grid: 6-D, upwind, and every periodic dim among dims 1..3
// of even length (the last row of an odd dim has no partner and loads its neighbours itself,
// which a periodic wrap would need twice).
static bool brick_ok(const hjr_grid &g, int spatial)
{
    if (g.ndim != 6 || spatial != HJR_UPWIND1) return false;
    for (int d = 1; d <= 3; ++d)
        if (((g.periodic_mask >> d) & 1u) && (g.n[d] & 1)) return false;
    return true;
}

class Tuner {
public:
    static Tuner &get()
    {
        static Tuner *t = new Tuner();
        return *t;
    }
    // march: the group may use the plane-march kernel (its candidates are then timed too);
    // brick: also the brick variant
    static std::string key(int prec, int dyn, int spatial, uint64_t nodes, bool march = false, bool brick = false)
    {
        int b = 0;
        while ((2ull << b) <= nodes) ++b;
        char buf[64];
        snprintf(buf, sizeof buf, "fp%d_dyn%d_sp%d_n2^%d%s", prec ? 64 : 32, dyn, spatial, b,
                 march ? (brick ? "_mb" : "_m") : "");
        return buf;
    }
    static bool ends_with(const std::string &k, const char *x)
    {
        const size_t n = strlen(x);
        return k.size() > n && k.compare(k.size() - n, n, x) == 0;
    }
    static bool march_key(const std::string &k) { return ends_with(k, "_m") || ends_with(k, "_mb"); }
    static const int *schedule(const std::string &k, int *len)
    {
        if (ends_with(k, "_mb")) {
            *len = (int)(sizeof kMarchBrickSchedule / sizeof kMarchBrickSchedule[0]);
            return kMarchBrickSchedule;
        }
        if (march_key(k) && k.find("_sp5_") != std::string::npos) {
            *len = (int)(sizeof kMarchW5Schedule / sizeof kMarchW5Schedule[0]);
            return kMarchW5Schedule;
        }
        if (march_key(k)) {
            *len = (int)(sizeof kMarchSchedule / sizeof kMarchSchedule[0]);
            return kMarchSchedule;
        }
        *len = (int)(sizeof kFlatSchedule / sizeof kFlatSchedule[0]);
        return kFlatSchedule;
    }
    // The chosen nodes-per-thread, or 0 while candidates remain untimed.
    int choice(const std::string &k)
    {
        std::lock_guard<std::mutex> g(mu_);
        load_file();
        auto it = chosen_.find(k);
        return it == chosen_.end() ? 0 : it->second;
    }
    // The next candidate to time for k.
    int next_candidate(const std::string &k)
    {
        std::lock_guard<std::mutex> g(mu_);
        int len;
        const int *sch = schedule(k, &len);
        const int n = count_[k];
        return n < len ? sch[n] : sch[0];
    }
    void record(const std::string &k, int config, double us)
    {
        std::lock_guard<std::mutex> g(mu_);
        int len;
        const int *sch = schedule(k, &len);
        auto &m = timed_[k];
        m[config] = m.count(config) ? std::min(m[config], us) : us;
        if (++count_[k] < len) return;
        for (int i = 0; i < len; ++i)
            if (!m.count(sch[i])) return;
        // another candidate must beat the default by 8% (and the best so far by 2%): near-ties
        // keep the default, so the choice does not flip with timing noise from run to run
        const int def = sch[0];
        int best = def;
        for (int i = 0; i < len; ++i) {
            const int c = sch[i];
            if (m[c] < 0.92 * m[def] && m[c] < 0.98 * m[best]) best = c;
        }
        chosen_[k] = best;
        save_file();
    }

private:
    void save_file()
    {
        const char *path = getenv("HJR_TUNE_CACHE");
        if (!path || !*path) return;
        FILE *f = fopen(path, "w");
        if (!f) return;
        fprintf(f, "{\n");
        size_t i = 0;
        for (auto &kv : chosen_)
            fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < chosen_.size() ? "," : "");
        fprintf(f, "}\n");
        fclose(f);
    }
    void load_file()
    {
        if (loaded_) return;
        loaded_ = true;
        const char *path = getenv("HJR_TUNE_CACHE");
        if (!path || !*path) return;
        FILE *f = fopen(path, "r");
        if (!f) return;
        char line[256];
        while (fgets(line, sizeof line, f)) {
            char k[128];
            int v = 0;
            if (sscanf(line, " \"%127[^\"]\" : %d", k, &v) == 2 && valid_config(v))
                chosen_[k] = v;
        }
        fclose(f);
    }
    std::mutex mu_;
    std::map<std::string, int> chosen_;
    std::map<std::string, std::map<int, double>> timed_;
    std::map<std::string, int> count_;  // timings recorded per key
    bool loaded_ = false;
};

// --------------------------------------------------------------------------------------------
// Arena: device memory carved from one caller-provided block (a bump allocator that never
// frees; the allocation-free entry point hands the engine its static scratch array this way).
// --------------------------------------------------------------------------------------------

struct Arena {
    char *base = nullptr;
    size_t size = 0;
    size_t used = 0;
    hipError_t alloc(void **ptr, size_t bytes)
    {
        const size_t b = align256(bytes);
        if (used + b > size) return hipErrorOutOfMemory;
        *ptr = base + used;
        used += b;
        return hipSuccess;
    }
};

// --------------------------------------------------------------------------------------------
// Engine
// --------------------------------------------------------------------------------------------

class Engine {
public:
    // arena: take every device buffer from this block instead of the pool, keep host staging in
    // pageable memory, and make no allocating call at all: no graphs, no events (so no profile
    // and no autotuning; the tuner's earlier choices still apply), no stream of its own.
    explicit Engine(int capacity, Arena *arena = nullptr) : cap_(capacity), arena_(arena) {}
    ~Engine() { release(); }

    hjr_status init(hipStream_t stream)
    {
        HJR_HIP(hipGetDevice(&device_));
        if (stream || arena_) {
            stream_ = stream;
        } else {
            HJR_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
            own_stream_ = true;
        }
        HJR_HIP(dalloc((void **)&d_states_, sizeof(SolveState) * cap_));
        HJR_HIP(dalloc((void **)&d_insts_, sizeof(Inst) * cap_));
        HJR_HIP(halloc((void **)&h_states_, sizeof(SolveState) * cap_));
        HJR_HIP(halloc((void **)&h_insts_, sizeof(Inst) * cap_));
        std::memset(h_insts_, 0, sizeof(Inst) * cap_);
        // idle slots: a frozen state so step_end skips them
        for (int i = 0; i < cap_; ++i) {
            std::memset(&h_states_[i], 0, sizeof(SolveState));
            h_states_[i].done = 99;
            h_insts_[i].state = d_states_ + i;
        }
        HJR_HIP(hipMemcpyAsync(d_states_, h_states_, sizeof(SolveState) * cap_, hipMemcpyHostToDevice, stream_));
        HJR_HIP(hipMemcpyAsync(d_insts_, h_insts_, sizeof(Inst) * cap_, hipMemcpyHostToDevice, stream_));
        HJR_HIP(hipStreamSynchronize(stream_));
        slots_.assign(cap_, nullptr);
        hist_.assign(cap_, Hist{});
        HJR_HIP(hipDeviceGetAttribute(&cus_, hipDeviceAttributeMultiprocessorCount, device_));
        if (const char *mb = getenv("HJR_MAX_BLOCKS")) max_blocks_ = atoi(mb);
        if (const char *fu = getenv("HJR_FUSED")) fused_ = atoi(fu) != 0;
        if (const char *np = getenv("HJR_NPT")) npt_override_ = atoi(np);
        if (!valid_config(npt_override_)) npt_override_ = 0;
        if (const char *at = getenv("HJR_AUTOTUNE")) autotune_ = atoi(at) != 0;
        if (const char *gr = getenv("HJR_GRAPHS")) graphs_ = atoi(gr) != 0;
        if (const char *pb = getenv("HJR_PLANE_BLOCK_BYTES")) plane_block_bytes_ = strtoull(pb, nullptr, 10);
        if (arena_) {
            graphs_ = false;
            autotune_ = false;
        }
        return HJR_OK;
    }

    void release()
    {
        if (stream_) (void)hipStreamSynchronize(stream_);
        for (EvRec &e : evs_) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        evs_.clear();
        drop_graphs();
        for (Request *r : slots_)
            if (r) drop(r);
        dfree(d_states_);
        dfree(d_insts_);
        dfree(d_tiles32_);
        dfree(d_tiles64_);
        dfree(d_mtiles_[0]);
        dfree(d_mtiles_[1]);
        d_states_ = nullptr;
        d_insts_ = nullptr;
        d_tiles32_ = d_tiles64_ = nullptr;
        d_mtiles_[0] = d_mtiles_[1] = nullptr;
        mtiles_cap_[0] = mtiles_cap_[1] = 0;
        hfree(h_states_);
        hfree(h_insts_);
        hfree(h_tiles_);
        h_states_ = nullptr;
        h_insts_ = nullptr;
        h_tiles_ = nullptr;
        if (own_stream_ && stream_) (void)hipStreamDestroy(stream_);
        stream_ = nullptr;
    }

    hipStream_t stream() const { return stream_; }
    // Replay captured HIP graphs of whole chunks (worth it for engines that live across many
    // chunks of the same length; HJR_GRAPHS=0/1 overrides).
    void prefer_graphs(bool on)
    {
        const char *gr = getenv("HJR_GRAPHS");
        graphs_ = gr ? atoi(gr) != 0 : on;
    }
    int active() const { return nactive_; }
    bool has_free_slot() const { return nactive_ < cap_; }
    int64_t launches() const { return launches_; }
    int64_t chunks() const { return chunks_; }
    void set_max_blocks(int b) { max_blocks_ = b; }

    // Start a request: allocate, upload descriptors and tables, launch init + setup.
    // own_io: the library owns l/k/V device copies (host-pointer path); host arrays given.
    hjr_status admit(Request *r, bool own_io, const double *l_host, const double *k_host,
                     const double *g_host = nullptr)
    {
        int slot = -1;
        for (int i = 0; i < cap_; ++i)
            if (!slots_[i]) {
                slot = i;
                break;
            }
        if (slot < 0) return fail(HJR_ERR_INVALID_ARG, "engine is full");
        Layout L = plan_layout(*r, own_io, own_io ? g_host != nullptr : r->g_dev != nullptr);
        r->bytes = L.total;
        HJR_HIP(dalloc(&r->mem, L.total));
        char *base = (char *)r->mem;
        if (own_io) {
            r->V_dev = (double *)(base + L.V64);
            r->l_dev = (const double *)(base + L.l64);
            r->k_dev = k_host ? (const double *)(base + L.k64) : nullptr;
            HJR_HIP(hipMemcpyAsync((void *)r->l_dev, l_host, r->npts * 8, hipMemcpyHostToDevice, stream_));
            if (k_host)
                HJR_HIP(hipMemcpyAsync((void *)r->k_dev, k_host, r->npts * 8, hipMemcpyHostToDevice, stream_));
            r->g_dev = g_host ? (const double *)(base + L.g64) : nullptr;
            if (g_host)
                HJR_HIP(hipMemcpyAsync((void *)r->g_dev, g_host, r->npts * 8, hipMemcpyHostToDevice, stream_));
        }
        std::vector<double> t64;
        std::vector<float> t32;
        build_inst(*r, base, L, t64, t32, d_states_ + slot);
        if (r->inst.act) {
            HJR_HIP(hipMemcpyAsync((void *)r->inst.dep_off, r->dep_off.data(), r->dep_off.size() * 4,
                                   hipMemcpyHostToDevice, stream_));
            HJR_HIP(hipMemcpyAsync((void *)r->inst.dep, r->dep.data(), r->dep.size() * 4, hipMemcpyHostToDevice,
                                   stream_));
        }
        HJR_HIP(hipMemcpyAsync((void *)r->inst.tab64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice, stream_));
        HJR_HIP(hipMemcpyAsync((void *)r->inst.tab32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, stream_));
        // the host vectors must outlive the copies
        HJR_HIP(hipStreamSynchronize(stream_));
        r->slot = slot;
        r->phase = 0;
        hist_[slot] = Hist{};
        r->fp32_first = r->opts.precision != HJR_FP64;
        slots_[slot] = r;
        ++nactive_;
        h_insts_[slot] = r->inst;
        h_states_[slot] = initial_state(*r);
        HJR_HIP(hipMemcpyAsync(d_insts_ + slot, &h_insts_[slot], sizeof(Inst), hipMemcpyHostToDevice, stream_));
        HJR_HIP(hipMemcpyAsync(d_states_ + slot, &h_states_[slot], sizeof(SolveState), hipMemcpyHostToDevice,
                               stream_));
        // FP32 followed by the FP64 polish: the FP32 phase runs down to 3 spacings, leaving the
        // polish little to do; FP32 alone stops at 8, clear of its rounding noise
        const int ulps = !r->fp32_first ? 0 : (r->opts.precision == HJR_FP32_POLISH64 ? 3 : 8);
        HJR_HIP(launch_init(d_insts_, slot, (uint32_t)r->npts, r->l_dev, r->k_dev, ulps, stream_));
        r->t_start = now_s();
        dirty_ = true;
        return HJR_OK;
    }

    // Enqueue m steps for every running instance.
    hjr_status enqueue_steps(int m, bool prof)
    {
        const int ninst = top_slot_ + 1;
        for (int step = 0; step < m; ++step) {
            cur_step_ = step;
            for (int stage = 0; stage < max_stages_; ++stage) {
                for (int prec = 0; prec < 2; ++prec) {
                    hjr_status s = launch_stage_all(prec, stage, prof);
                    if (s != HJR_OK) return s;
                }
            }
            HJR_HIP(launch_step_end(d_insts_, ninst, stream_));
            ++launches_;
            if (any_interval_) {
                HJR_HIP(launch_interval(false, d_insts_, d_tiles32_, n32_, max_blocks_, stream_));
                HJR_HIP(launch_interval(true, d_insts_, d_tiles64_, n64_, max_blocks_, stream_));
                HJR_HIP(launch_interval_end(d_insts_, ninst, stream_));
                launches_ += 3;
            }
        }
        return HJR_OK;
    }

    // Issue m steps (replaying a captured HIP graph of them when graphs are on), then read the
    // states back.
    hjr_status run_chunk(int m)
    {
        if (dirty_) {
            hjr_status s = rebuild();
            if (s != HJR_OK) return s;
        }
        const int ninst = top_slot_ + 1;
        const bool prof = g_profile_on.load() != 0 && !arena_;
        nev_ = 0;
        // where each instance stood before the chunk, to tell working launches from the ones
        // issued after it finished (profile accounting)
        before_.resize(ninst);
        for (int i = 0; i < ninst; ++i) before_[i] = {h_states_[i].phase, h_states_[i].n, h_states_[i].done};
        bool done = false;
        bool exploring = false;
        for (int p = 0; p < 2; ++p)
            for (const Seg &g : segs_[p]) exploring |= !g.tune_key.empty();
        if (graphs_ && !prof && !exploring) {
            hipGraphExec_t exec = nullptr;
            auto it = graphs_by_m_.find(m);
            if (it != graphs_by_m_.end()) {
                exec = it->second;
            } else {
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    const int64_t l0 = launches_;
                    hjr_status s = enqueue_steps(m, false);
                    launches_ = l0;
                    e = hipStreamEndCapture(stream_, &g);
                    if (s != HJR_OK && e == hipSuccess) e = hipErrorUnknown;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
                if (g) (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    graphs_ = false;  // fall back to direct launches for this engine
                    exec = nullptr;
                } else {
                    graphs_by_m_[m] = exec;
                }
            }
            if (exec) {
                HJR_HIP(hipGraphLaunch(exec, stream_));
                launches_ += (int64_t)m * (max_stages_ * ((int)segs_[0].size() + (int)segs_[1].size()) + 1);
                done = true;
            }
        }
        if (!done) {
            hjr_status s = enqueue_steps(m, prof);
            if (s != HJR_OK) return s;
        }
        ++chunks_;
        HJR_HIP(hipMemcpyAsync(h_states_, d_states_, sizeof(SolveState) * ninst, hipMemcpyDeviceToHost, stream_));
        HJR_HIP(hipStreamSynchronize(stream_));
        if (nev_ > 0) {
            std::map<std::pair<int, int>, std::vector<float>> tuned;  // (prec, group) -> launch ms
            std::lock_guard<std::mutex> g(g_profile_mu);
            for (int i = 0; i < nev_; ++i) {
                EvRec &e = evs_[i];
                float ms = 0.f;
                HJR_HIP(hipEventElapsedTime(&ms, e.a, e.b));
                if (e.group >= 0) {
                    // only launches of steps every instance of the group was taking: after an
                    // instance finishes, its tiles return at once and the launch says nothing
                    // about the candidate
                    auto &v = tuned[{e.prec, e.group}];
                    if (launch_full(e)) v.push_back(ms);
                    continue;
                }
                hjr_kernel_time &kt = e.prec ? g_profile.stage64[e.stage] : g_profile.stage32[e.stage];
                kt.launches += 1;
                kt.nodes += e.nodes;
                kt.ms += ms;
                if (launch_worked(e)) {
                    kt.working_launches += 1;
                    kt.working_ms += ms;
                }
            }
            // the median of the chunk's full launches; a chunk in which one of the group's
            // instances changed phase is not used (its launches before or after the change
            // returned at once).  A chunk in which an instance finished still counts: a solve's
            // few FP64 polish steps often end inside their first chunk.
            for (auto &kv : tuned) {
                auto &v = kv.second;
                std::sort(v.begin(), v.end());
                const Seg &sg = segs_[kv.first.first][kv.first.second];
                bool same_phase = true;
                for (int i : sg.slots)
                    same_phase = same_phase && i < (int)before_.size() && h_states_[i].phase == before_[i].phase;
                if (same_phase && v.size() >= 3) {
                    Tuner::get().record(sg.tune_key, sg.npt, 1e3 * v[v.size() / 2]);
                    if (getenv("HJR_TUNE_VERBOSE"))
                        fprintf(stderr, "[hjr tune] %s npt=%d launches=%zu min=%.1fus median=%.1fus max=%.1fus\n",
                                sg.tune_key.c_str(), sg.npt, v.size(), 1e3 * v.front(), 1e3 * v[v.size() / 2],
                                1e3 * v.back());
                }
            }
            if (!tuned.empty()) dirty_ = true;  // next chunk: next candidate, or the choice
        }
        return HJR_OK;
    }

    void drop_graphs()
    {
        for (auto &kv : graphs_by_m_) (void)hipGraphExecDestroy(kv.second);
        graphs_by_m_.clear();
    }

    // Steps until the first running instance is expected to meet its threshold, from the decay
    // of its max-change between the last two read-backs (geometric model); 0 if unknown.
    int predict_steps()
    {
        double best = 0.0;
        bool any = false;
        for (int i = 0; i <= top_slot_; ++i) {
            Request *r = slots_[i];
            if (!r) continue;
            const SolveState &st = h_states_[i];
            Hist &h = hist_[i];
            if (st.done != kRunning || st.phase != h.phase || st.n <= h.n || !(h.delta > 0.0)) {
                h = Hist{st.phase, st.n, st.last_delta};
                continue;
            }
            const double d = st.last_delta;
            if (d > 0.0 && d < h.delta && st.tol > 0.0) {
                const double rho = std::pow(d / h.delta, 1.0 / (double)(st.n - h.n));
                const double rem = d <= st.tol ? 1.0 : std::log(st.tol / d) / std::log(rho);
                if (!any || rem < best) best = rem;
                any = true;
            }
            h = Hist{st.phase, st.n, st.last_delta};
        }
        if (!any) return 0;
        return (int)std::min(1e6, std::ceil(best));
    }

    // Advance the phase machine of every instance after a chunk.  Finished requests are
    // appended to `finished` (their slots are freed).
    hjr_status update(std::vector<Request *> &finished)
    {
        for (int i = 0; i <= top_slot_; ++i) {
            Request *r = slots_[i];
            if (!r) continue;
            const SolveState &st = h_states_[i];
            if (st.done == kRunning) continue;
            if (st.done == kNonFinite) {
                r->status = fail(HJR_ERR_NONFINITE, "l or k holds a NaN or an infinity");
                finish(r, finished, false);
                continue;
            }
            const bool polish = r->phase == 0 && r->opts.precision == HJR_FP32_POLISH64 && st.done != kHorizon;
            if (polish) {
                r->iters0 = st.n;
                r->phase = 1;
                HJR_HIP(launch_polish(d_insts_, i, (uint32_t)r->npts, st.parity, r->opts.polish_shift, stream_));
                h_states_[i].done = kRunning;  // until the next read-back
                dirty_ = true;
                continue;
            }
            // final phase done
            hjr_result &res = r->result;
            std::memset(&res, 0, sizeof res);
            if (r->phase == 0) {
                res.iterations = st.n;
            } else {
                res.iterations = r->iters0;
                res.polish_iterations = st.n;
            }
            res.discounted_iterations = (r->phase == 0 && st.gamma != 1.0) ? st.n : st.n_disc;
            res.node_updates = (int64_t)st.epoch * (int64_t)r->npts;
            if (r->inst.act) {  // the per-block counts of computed grid points
                std::vector<unsigned long long> c(r->inst.nblocks);
                HJR_HIP(hipMemcpyAsync(c.data(), r->inst.cnt, c.size() * 8, hipMemcpyDeviceToHost, stream_));
                HJR_HIP(hipStreamSynchronize(stream_));
                res.node_updates = 0;
                for (unsigned long long v : c) res.node_updates += (int64_t)v;
            }
            res.intervals = st.intervals;
            res.t_final = st.t;
            res.last_delta = st.last_delta;
            res.dt = st.dt_nom;
            res.max_abs_l = st.max_abs_l;
            res.converged = st.done == kConverged ? 1 : (st.done == kHorizon ? 2 : (st.done == kStalled ? 3 : 0));
            r->status = st.done == kConverged ? HJR_OK : (st.done == kHorizon ? HJR_HORIZON : HJR_NOT_CONVERGED);
            const bool from32 = r->phase == 0 && r->fp32_first;
            const int parity = (r->opts.temporal == HJR_EULER) ? st.parity : 0;
            if (from32 || parity) {
                HJR_HIP(launch_output(d_insts_, i, (uint32_t)r->npts, from32, parity, r->V_dev, stream_));
            }
            finish(r, finished, true);
        }
        return HJR_OK;
    }

    // Free the slot of a finished request (its output stays in V_dev).
    void finish(Request *r, std::vector<Request *> &finished, bool ok)
    {
        (void)ok;
        const int i = r->slot;
        h_states_[i].done = 99;
        (void)hipMemcpyAsync(d_states_ + i, &h_states_[i], sizeof(SolveState), hipMemcpyHostToDevice, stream_);
        slots_[i] = nullptr;
        --nactive_;
        r->result.seconds = now_s() - r->t_start;
        finished.push_back(r);
        dirty_ = true;
    }

    // Return a request's working memory to the pool (after its output has been consumed).
    void drop(Request *r)
    {
        dfree(r->mem);
        r->mem = nullptr;
    }

private:
    // device and host buffers: the pool and pinned host memory, or the arena and plain host
    // memory (an arena never frees; its block is reused by the next engine)
    hipError_t dalloc(void **p, size_t bytes) { return arena_ ? arena_->alloc(p, bytes) : Pool::get().alloc(p, bytes); }
    void dfree(void *p)
    {
        if (!arena_) Pool::get().release(p);
    }
    hipError_t halloc(void **p, size_t bytes)
    {
        if (!arena_) return hipHostMalloc(p, bytes, hipHostMallocDefault);
        *p = ::operator new(bytes, std::nothrow);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    void hfree(void *p)
    {
        if (!p) return;
        if (arena_)
            ::operator delete(p);
        else
            (void)hipHostFree(p);
    }

    struct EvRec {
        hipEvent_t a, b;
        int prec, stage;
        int64_t nodes;
        int group;  // >= 0: autotuner timing of segs_[prec][group]; -1: kernel profile
        int seg;    // the launch's group in segs_[prec] (-1: the fused kernel)
        int step;   // the step of the chunk the launch belongs to
    };
    struct Hist {
        int phase = -1;
        long long n = 0;
        double delta = 0.0;
    };
    struct Before {
        int phase;
        long long n;
        int done;
    };

    // Steps of the last chunk that instance i took (in the phase it ended the chunk in).
    long long steps_taken(int i) const
    {
        const SolveState &a = h_states_[i];
        const Before &b = before_[i];
        if (b.done != kRunning && a.phase == b.phase) return 0;  // already finished, or idle slot
        return a.phase != b.phase ? a.n : a.n - b.n;
    }
    // Whether some instance of the launch's group (every instance, for the fused kernel) was
    // still taking the launch's step.
    // Whether every instance of the launch's group was still taking the launch's step.
    bool launch_full(const EvRec &e) const
    {
        if (e.seg < 0) return false;
        for (int i : segs_[e.prec][e.seg].slots)
            if (i >= (int)before_.size() || steps_taken(i) <= e.step) return false;
        return true;
    }
    bool launch_worked(const EvRec &e) const
    {
        if (e.seg < 0) {
            for (int i = 0; i <= top_slot_ && i < (int)before_.size(); ++i)
                if (slots_[i] && steps_taken(i) > e.step) return true;
            return false;
        }
        for (int i : segs_[e.prec][e.seg].slots)
            if (i < (int)before_.size() && steps_taken(i) > e.step) return true;
        return false;
    }


    hjr_status event_pair(hipEvent_t *a, hipEvent_t *b, int prec, int stage, int64_t nodes, int group, int seg = -1)
    {
        if (nev_ == (int)evs_.size()) {
            EvRec e{};
            HJR_HIP(hipEventCreate(&e.a));
            HJR_HIP(hipEventCreate(&e.b));
            evs_.push_back(e);
        }
        EvRec &e = evs_[nev_++];
        e.prec = prec;
        e.stage = stage;
        e.nodes = nodes;
        e.group = group;
        e.seg = seg;
        e.step = cur_step_;
        *a = e.a;
        *b = e.b;
        return HJR_OK;
    }

    hjr_status rebuild()
    {
        // tiles grouped by (precision, model, scheme); each group is a contiguous segment
        struct G {
            std::vector<int> slots;
            uint64_t nodes = 0;
            uint64_t largest = 0;  // size class for the tuner: the group's largest instance
            uint64_t min_cols = ~0ull;  // the fewest columns (nodes per dim-0 plane) of its grids
            bool march_ok = true;
            bool brick_ok = true;
        };
        std::map<int, G> groups[2];
        top_slot_ = -1;
        max_stages_ = 1;
        any_interval_ = false;
        for (int i = 0; i < cap_; ++i) {
            Request *r = slots_[i];
            if (!r) continue;
            top_slot_ = i;
            if (r->opts.temporal == HJR_TVDRK3) max_stages_ = 3;
            if (r->opts.conv_mode == HJR_CONV_PER_INTERVAL) any_interval_ = true;
            const int fp64 = !(r->phase == 0 && r->fp32_first) ? 1 : 0;
            G &g = groups[fp64][r->dyn.id * 8 + r->opts.spatial + (r->inst.act ? kLocalKey : 0)];
            g.slots.push_back(i);
            g.nodes += r->npts;
            g.largest = std::max(g.largest, r->npts);
            g.min_cols = std::min(g.min_cols, r->npts / (uint64_t)r->grid.n[0]);
            g.march_ok = g.march_ok && (r->opts.spatial == HJR_UPWIND1 || r->opts.spatial == HJR_WENO5) &&
                         r->grid.ndim >= 2 && !r->inst.act;
            g.brick_ok = g.brick_ok && brick_ok(r->grid, r->opts.spatial);
        }
        if (top_slot_ < 0) top_slot_ = 0;
        std::vector<Tile> t[2];
        std::vector<MTile> mt[2];
        for (int p = 0; p < 2; ++p) {
            segs_[p].clear();
            for (auto &kv : groups[p]) {
                const bool local = kv.first >= kLocalKey;
                const int dyn = (kv.first % kLocalKey) / 8, sp = kv.first % 8;
                // the march kernel addresses each field with 32-bit byte offsets
                const bool march_ok = kv.second.march_ok && kv.second.min_cols >= kMarchMinColumns &&
                                      kv.second.largest * (p ? 8ull : 4ull) <= 0xffffffffull;
                const bool brick = march_ok && kv.second.brick_ok;
                int cfg = kFusedNpt;
                std::string tkey;
                if (local && !fused_) {
                    cfg = 4;  // the local-update kernels exist for 4 nodes per thread only
                } else if (!fused_) {
                    cfg = npt_override_;
                    if (cfg && is_march(cfg) && !march_ok) cfg = 4;
                    if (cfg == kMarchBrick && !brick) cfg = kMarchFull;
                    if (!cfg) {
                        const std::string k = Tuner::key(p, dyn, sp, kv.second.largest, march_ok, brick);
                        cfg = Tuner::get().choice(k);
                        if (!cfg && autotune_) {
                            cfg = Tuner::get().next_candidate(k);
                            tkey = k;  // this group's launches are timed this chunk
                        }
                        if (!cfg) cfg = kFusedNpt;
                    }
                }
                // flat tiles of the groups launched with them, and of every group when the
                // interval kernel (which walks them) runs; march groups get their march tiles
                const int off = (int)t[p].size();
                if (!is_march(cfg) || any_interval_) append_tiles(kv.second.slots, is_march(cfg) ? 4 : cfg, t[p]);
                const int moff = (int)mt[p].size();
                if (is_march(cfg)) append_march_tiles(kv.second.slots, cfg, mt[p]);
                segs_[p].push_back(Seg{dyn, sp, cfg, off, (int)t[p].size() - off, moff, (int)mt[p].size() - moff,
                                       (int64_t)kv.second.nodes, tkey, local, kv.second.slots});
            }
        }
        n32_ = (int)t[0].size();
        n64_ = (int)t[1].size();
        for (int p = 0; p < 2; ++p) {
            nodes_[p] = 0;
            for (auto &kv : groups[p]) nodes_[p] += (int64_t)kv.second.nodes;
        }
        hjr_status s = upload_tiles(t[0], t[1]);
        if (s != HJR_OK) return s;
        for (int p = 0; p < 2; ++p) {
            s = upload_march_tiles(p, mt[p]);
            if (s != HJR_OK) return s;
        }
        drop_graphs();
        dirty_ = false;
        return HJR_OK;
    }

    // Tiles of each instance, in the order the workgroups of one XCD will sweep them.  In flat
    // order a node's neighbours along dim 0 are a whole dim-0 plane away, so on a grid whose
    // planes are larger than plane_block_bytes_ (FP32 field bytes) they have left the caches
    // before they are read again.  Such grids are visited in chunks of the inner (dims 1..)
    // index range, two dim-1 strides long, with dim 0 innermost: a node's dim-0 neighbours are
    // then one chunk away and its dim-1 neighbours inside the chunk.  Every tile start falls in
    // exactly one (chunk, plane) range, so this is a permutation of the flat-order tiles and
    // the results do not change.
    void append_tiles(const std::vector<int> &slots, int npt, std::vector<Tile> &out)
    {
        const uint64_t T = (uint64_t)npt * kBlock;
        for (int i : slots) {
            const Request *r = slots_[i];
            const uint64_t N = r->npts;
            const int n0 = r->grid.n[0];
            const uint64_t P = N / (uint64_t)n0;  // nodes per dim-0 plane
            if (r->grid.ndim < 2 || P * 4 <= plane_block_bytes_ || N < 16 * T) {
                for (uint64_t s = 0; s < N; s += T) out.push_back(Tile{i, (uint32_t)s, npt});
                continue;
            }
            const uint64_t C = std::max<uint64_t>(T, 2 * (P / (uint64_t)r->grid.n[1]));
            for (uint64_t c0 = 0; c0 < P; c0 += C) {
                const uint64_t c1 = std::min(P, c0 + C);
                for (int i0 = 0; i0 < n0; ++i0) {
                    const uint64_t a = (uint64_t)i0 * P + c0, b = (uint64_t)i0 * P + c1;
                    for (uint64_t t = (a + T - 1) / T; t * T < b; ++t) out.push_back(Tile{i, (uint32_t)(t * T), npt});
                }
            }
        }
    }

    // March tiles of each instance for configuration cfg (runs of -cfg dim-0 planes, kMarchFull
    // the whole line), in XCD order.
    void append_march_tiles(const std::vector<int> &slots, int cfg, std::vector<MTile> &out)
    {
        for (int i : slots) {
            Request *r = slots_[i];
            if (r->mtiles_cfg != cfg) {
                r->mtiles.clear();
                if (cfg == kMarchBrick)
                    march_brick_tiles(i, r->grid.ndim, r->grid.n, r->mtiles);
                else
                    march_tiles(i, r->grid.ndim, r->grid.n, cfg == kMarchFull ? 0 : -cfg, r->mtiles);
                r->mtiles_cfg = cfg;
            }
            out.insert(out.end(), r->mtiles.begin(), r->mtiles.end());
        }
    }

    hjr_status upload_march_tiles(int p, const std::vector<MTile> &m)
    {
        if (m.empty()) return HJR_OK;
        const size_t need = m.size() * sizeof(MTile);
        // earlier copies from the staging buffer, and kernels reading the old list, must be done
        HJR_HIP(hipStreamSynchronize(stream_));
        if (need > mtiles_cap_[p]) {
            dfree(d_mtiles_[p]);
            d_mtiles_[p] = nullptr;
            mtiles_cap_[p] = std::max(need * 2, (size_t)4096);
            HJR_HIP(dalloc((void **)&d_mtiles_[p], mtiles_cap_[p]));
        }
        HJR_HIP(hipMemcpy(d_mtiles_[p], m.data(), need, hipMemcpyHostToDevice));
        return HJR_OK;
    }

    hjr_status upload_tiles(const std::vector<Tile> &a, const std::vector<Tile> &b)
    {
        const size_t need = (a.size() + b.size() + 2) * sizeof(Tile);
        if (need > tiles_cap_) {
            HJR_HIP(hipStreamSynchronize(stream_));
            dfree(d_tiles32_);
            dfree(d_tiles64_);
            hfree(h_tiles_);
            tiles_cap_ = std::max(need * 2, (size_t)4096);
            HJR_HIP(dalloc((void **)&d_tiles32_, tiles_cap_));
            HJR_HIP(dalloc((void **)&d_tiles64_, tiles_cap_));
            HJR_HIP(halloc((void **)&h_tiles_, tiles_cap_ * 2));
        }
        // staging is reused: earlier copies from it must have completed
        HJR_HIP(hipStreamSynchronize(stream_));
        std::memcpy(h_tiles_, a.data(), a.size() * sizeof(Tile));
        std::memcpy((char *)h_tiles_ + tiles_cap_, b.data(), b.size() * sizeof(Tile));
        if (!a.empty())
            HJR_HIP(hipMemcpyAsync(d_tiles32_, h_tiles_, a.size() * sizeof(Tile), hipMemcpyHostToDevice, stream_));
        if (!b.empty())
            HJR_HIP(hipMemcpyAsync(d_tiles64_, (char *)h_tiles_ + tiles_cap_, b.size() * sizeof(Tile),
                                   hipMemcpyHostToDevice, stream_));
        return HJR_OK;
    }

    // One stage over every tile of one precision: a single fused launch, or one launch per
    // (model, scheme) group with the kernel specialised to it.
    hjr_status launch_stage_all(int prec, int stage, bool prof)
    {
        const int nt = prec ? n64_ : n32_;
        const Tile *tl = prec ? d_tiles64_ : d_tiles32_;
        if (fused_) {
            if (nt <= 0) return HJR_OK;
            hipEvent_t a = nullptr, b = nullptr;
            if (prof) {
                hjr_status s = event_pair(&a, &b, prec, stage, nodes_[prec], -1);
                if (s != HJR_OK) return s;
                HJR_HIP(hipEventRecord(a, stream_));
            }
            HJR_HIP(launch_stage(prec != 0, d_insts_, tl, nt, stage, max_blocks_, stream_));
            if (prof) HJR_HIP(hipEventRecord(b, stream_));
            ++launches_;
            return HJR_OK;
        }
        // per-group kernel durations (profile, or the autotuner's timing of a candidate) come
        // from events stamped by the launch itself with the kernel's start and end
        // (march groups have no flat tiles unless the interval kernel needs them)
        for (int gi = 0; gi < (int)segs_[prec].size(); ++gi) {
            const Seg &g = segs_[prec][gi];
            if ((is_march(g.npt) ? g.mcount : g.count) <= 0) continue;
            const bool explore = !g.tune_key.empty() && !prof;
            hipEvent_t ga = nullptr, gb = nullptr;
            if (prof || explore) {
                hjr_status s = event_pair(&ga, &gb, prec, stage, prof ? g.nodes : 0, prof ? -1 : gi, gi);
                if (s != HJR_OK) return s;
            }
            if (is_march(g.npt))
                HJR_HIP(launch_march(prec != 0, g.dyn, g.spatial, g.npt == kMarchBrick, d_insts_, d_mtiles_[prec] + g.moff,
                                     g.mcount, stage, stream_, ga, gb));
            else
                HJR_HIP(launch_stage_one(prec != 0, g.dyn, g.spatial, g.npt, d_insts_, tl + g.off, g.count, stage,
                                         max_blocks_, stream_, ga, gb, g.local));
            ++launches_;
        }
        return HJR_OK;
    }

    struct Seg {
        int dyn, spatial;
        int npt;               // launch configuration: nodes per thread, or a march run length (< 0)
        int off, count;        // flat tiles
        int moff, mcount;      // march tiles
        int64_t nodes;         // nodes of the group's instances
        std::string tune_key;  // non-empty: this group is being timed for the autotuner
        bool local;            // instances with local updates (their own kernel variant)
        std::vector<int> slots;  // the group's instances
    };
    static constexpr int kLocalKey = 1024;  // group key offset of local-update instances
    std::vector<Seg> segs_[2];
    std::map<int, hipGraphExec_t> graphs_by_m_;
    bool graphs_ = false;
    int64_t nodes_[2] = {0, 0};
    bool fused_ = false;
    bool autotune_ = true;
    int npt_override_ = 0;

    int cap_;
    Arena *arena_ = nullptr;
    int device_ = 0;
    int cus_ = 256;
    hipStream_t stream_ = nullptr;
    bool own_stream_ = false;
    SolveState *d_states_ = nullptr, *h_states_ = nullptr;
    Inst *d_insts_ = nullptr, *h_insts_ = nullptr;
    Tile *d_tiles32_ = nullptr, *d_tiles64_ = nullptr;
    Tile *h_tiles_ = nullptr;
    size_t tiles_cap_ = 0;
    MTile *d_mtiles_[2] = {nullptr, nullptr};
    size_t mtiles_cap_[2] = {0, 0};
    int n32_ = 0, n64_ = 0;
    int top_slot_ = 0, max_stages_ = 1;
    bool any_interval_ = false;
    bool dirty_ = true;
    int max_blocks_ = 0;
    uint64_t plane_block_bytes_ = 16ull << 20;  // larger dim-0 planes: blocked tile order
    std::vector<Request *> slots_;
    std::vector<Hist> hist_;
    std::vector<EvRec> evs_;
    int nev_ = 0;
    std::vector<Before> before_;
    int cur_step_ = 0;
    int nactive_ = 0;
    int64_t launches_ = 0, chunks_ = 0;
};

// Chunk-size policy.  Every step launched after an instance has converged is a launch that
// returns at once; to keep those few, the next chunk is sized from the predicted number of steps
// to convergence, and otherwise grows geometrically while nothing finishes.
struct ChunkPolicy {
    int fixed, cur;
    explicit ChunkPolicy(int steps_per_sync) : fixed(steps_per_sync), cur(steps_per_sync > 0 ? steps_per_sync : 4) {}
    int next() const { return cur; }
    void after(bool something_finished, int predicted)
    {
        if (fixed > 0) return;
        int grow = something_finished ? 4 : std::min(cur * 2, 64);
        if (predicted > 0) grow = std::max(1, std::min(grow, predicted));
        cur = grow;
    }
};

// Local updates: for every block of 2^kLocalShift consecutive nodes, the blocks holding a node
// within `reach` grid steps (per dimension; wrapping in periodic dims) of one of its nodes.  The
// block's rows (runs along the last dimension) are bounded by a box in the other dimensions,
// the box is widened by `reach`, and every row in it is taken whole, so the list is a superset
// of the exact one (which only costs a few extra blocks).  Gives up (lists left empty, local
// updates off) when a list would be long enough to make the check cost more than it saves.
static void block_dependencies(const hjr_grid &g, uint64_t N, int reach, std::vector<uint32_t> &off,
                               std::vector<uint32_t> &dep)
{
    const int d = g.ndim, m = d - 1;                // row space: dims 0 .. d-2
    const uint64_t B = 1ull << kLocalShift, rowlen = (uint64_t)g.n[d - 1];
    const uint64_t nb = (N + B - 1) / B;
    const size_t kMaxPerBlock = 256;
    off.assign(1, 0);
    dep.clear();
    std::vector<uint32_t> cur;
    std::vector<uint32_t> seen(nb, UINT32_MAX);
    for (uint64_t b = 0; b < nb; ++b) {
        cur.clear();
        if (m == 0) {  // 1-D: the block's neighbours along the only dimension
            const int64_t lo = (int64_t)(b * B) - reach, hi = (int64_t)std::min(N, (b + 1) * B) - 1 + reach;
            const bool per = g.periodic_mask & 1u;
            if (per && (lo < 0 || hi >= (int64_t)N)) {
                for (uint64_t c = 0; c < nb; ++c) cur.push_back((uint32_t)c);
            } else {
                for (int64_t c = std::max<int64_t>(lo, 0) / (int64_t)B; c <= std::min<int64_t>(hi, N - 1) / (int64_t)B; ++c)
                    cur.push_back((uint32_t)c);
            }
        } else {
            // rows of the block and their index box
            const uint64_t r0 = (b * B) / rowlen, r1 = (std::min(N, (b + 1) * B) - 1) / rowlen;
            int a0[HJR_MAX_DIM], a1[HJR_MAX_DIM];
            uint64_t t0 = r0, t1 = r1;
            for (int j = m - 1; j >= 0; --j) {
                a0[j] = (int)(t0 % (uint64_t)g.n[j]);
                a1[j] = (int)(t1 % (uint64_t)g.n[j]);
                t0 /= (uint64_t)g.n[j];
                t1 /= (uint64_t)g.n[j];
            }
            int lo[HJR_MAX_DIM], hi[HJR_MAX_DIM];
            bool split = false;
            for (int j = 0; j < m; ++j) {
                if (split) {
                    lo[j] = 0;
                    hi[j] = g.n[j] - 1;
                } else {
                    lo[j] = a0[j];
                    hi[j] = a1[j];
                    if (a0[j] != a1[j]) split = true;
                }
            }
            // widen by the reach: per dim a list of index ranges (two when a periodic one wraps)
            std::vector<std::pair<int, int>> rng[HJR_MAX_DIM];
            uint64_t combos = 1;
            for (int j = 0; j < m; ++j) {
                const int n = g.n[j];
                const bool per = (g.periodic_mask >> j) & 1u;
                int l = lo[j] - reach, h = hi[j] + reach;
                if (per) {
                    if (h - l + 1 >= n) {
                        rng[j].push_back({0, n - 1});
                    } else if (l < 0) {
                        rng[j].push_back({0, h});
                        rng[j].push_back({l + n, n - 1});
                    } else if (h >= n) {
                        rng[j].push_back({l, n - 1});
                        rng[j].push_back({0, h - n});
                    } else {
                        rng[j].push_back({l, h});
                    }
                } else {
                    rng[j].push_back({std::max(l, 0), std::min(h, n - 1)});
                }
                if (j < m - 1) {
                    uint64_t e = 0;
                    for (auto &p : rng[j]) e += (uint64_t)(p.second - p.first + 1);
                    combos *= e;
                }
            }
            if (combos * 2 > kMaxPerBlock * 8) {
                off.clear();
                dep.clear();
                return;
            }
            // every combination of the outer dims, then the last row dim's ranges: runs of rows
            int idx[HJR_MAX_DIM] = {0};
            std::vector<int> outer_vals[HJR_MAX_DIM];
            for (int j = 0; j < m - 1; ++j)
                for (auto &p : rng[j])
                    for (int v = p.first; v <= p.second; ++v) outer_vals[j].push_back(v);
            int pos[HJR_MAX_DIM] = {0};
            for (;;) {
                uint64_t base = 0;
                for (int j = 0; j < m - 1; ++j) {
                    idx[j] = outer_vals[j][pos[j]];
                    base = base * (uint64_t)g.n[j] + (uint64_t)idx[j];
                }
                for (auto &p : rng[m - 1]) {
                    const uint64_t rs = base * (uint64_t)g.n[m - 1] + (uint64_t)p.first;
                    const uint64_t re = base * (uint64_t)g.n[m - 1] + (uint64_t)p.second;
                    const uint64_t f = rs * rowlen / B, l = ((re + 1) * rowlen - 1) / B;
                    for (uint64_t c = f; c <= l; ++c)
                        if (seen[c] != (uint32_t)b) {
                            seen[c] = (uint32_t)b;
                            cur.push_back((uint32_t)c);
                        }
                }
                int j = m - 2;
                while (j >= 0 && ++pos[j] == (int)outer_vals[j].size()) pos[j--] = 0;
                if (j < 0) break;
            }
        }
        if (cur.size() > kMaxPerBlock) {
            off.clear();
            dep.clear();
            return;
        }
        std::sort(cur.begin(), cur.end());
        dep.insert(dep.end(), cur.begin(), cur.end());
        off.push_back((uint32_t)dep.size());
    }
}

static hjr_status prepare(Request &r, const hjr_grid *g, const hjr_dynamics *dy, const hjr_options *o,
                          const void *k)
{
    hjr_status s = validate_opts(o);
    if (s != HJR_OK) return s;
    if (o->brs != 0 && o->brs != 1) return fail(HJR_ERR_INVALID_ARG, "brs must be 0 or 1");
    if (o->brs) {
        if (!(o->t_max > 0.0)) return fail(HJR_ERR_INVALID_ARG, "the reachable-set mode needs t_max > 0");
        if (o->precision == HJR_FP32_POLISH64)
            return fail(HJR_ERR_INVALID_ARG, "the reachable-set mode needs precision HJR_FP64 or HJR_FP32");
        if (k) return fail(HJR_ERR_INVALID_ARG, "the reachable-set mode takes no warm start");
    }
    if (!(o->discount >= 0.0 && o->discount <= 1.0))
        return fail(HJR_ERR_INVALID_ARG, "discount must lie in [0, 1]");
    if (o->brs && o->discount > 0.0 && o->discount < 1.0)
        return fail(HJR_ERR_INVALID_ARG, "the reachable-set mode is not discounted");
    if (o->local_updates != 0 && o->local_updates != 1) return fail(HJR_ERR_INVALID_ARG, "local_updates must be 0 or 1");
    uint64_t N = 0;
    s = validate(g, dy, o->spatial, &N);
    if (s != HJR_OK) return s;
    r.grid = *g;
    r.dyn = *dy;
    r.opts = *o;
    r.npts = N;
    r.dep_off.clear();
    r.dep.clear();
    if (o->local_updates) {
        const int reach = (o->temporal == HJR_TVDRK3 ? 3 : 1) * (o->spatial == HJR_WENO5 ? 3 : 1);
        block_dependencies(*g, N, reach, r.dep_off, r.dep);
    }
    return HJR_OK;
}

// Run a set of requests to completion on one engine (used by the synchronous entry points).
static hjr_status run_all(Engine &E, std::vector<Request *> &reqs, bool own_io, const std::vector<const double *> &lh,
                          const std::vector<const double *> &kh, int steps_per_sync,
                          const double *g_host = nullptr)
{
    size_t next = 0;
    ChunkPolicy pol(steps_per_sync);
    std::vector<Request *> fin;
    while (next < reqs.size() || E.active() > 0) {
        while (next < reqs.size() && E.has_free_slot()) {
            Request *r = reqs[next];
            hjr_status s = E.admit(r, own_io, own_io ? lh[next] : nullptr, own_io ? kh[next] : nullptr,
                                   own_io && next == 0 ? g_host : nullptr);
            if (s != HJR_OK) return s;
            ++next;
        }
        hjr_status s = E.run_chunk(pol.next());
        if (s != HJR_OK) return s;
        const size_t before = fin.size();
        s = E.update(fin);
        if (s != HJR_OK) return s;
        pol.after(fin.size() > before, E.predict_steps());
    }
    HJR_HIP(hipStreamSynchronize(E.stream()));
    return HJR_OK;
}

}  // namespace hjr

// ============================================================================================
// C ABI
// ============================================================================================

using namespace hjr;

extern "C" {

int32_t hjr_abi_version(void) { return HJR_ABI_VERSION; }

#ifndef HJR_SOURCE_HASH
#define HJR_SOURCE_HASH "unknown"
#endif
const char *hjr_build_id(void) { return HJR_SOURCE_HASH; }

hjr_status hjr_default_options(hjr_options *o)
{
    if (!o) return fail(HJR_ERR_INVALID_ARG, "options must not be NULL");
    std::memset(o, 0, sizeof *o);
    o->game = HJR_AVOID;
    o->spatial = HJR_WENO5;
    o->temporal = HJR_TVDRK3;
    o->precision = HJR_FP32_POLISH64;
    o->conv_mode = HJR_CONV_PER_STEP;
    o->steps_per_sync = 0;
    o->cfl = 0.5;
    o->tol = 1e-6;
    o->tol_fp32 = 0.0;
    o->polish_shift = -1.0;
    o->dt_report = 0.01;
    o->t_max = 0.0;
    o->dt_max = 0.0;
    o->max_iter = 100000;
    o->stall_window = 0;
    o->brs = 0;
    o->local_updates = 0;
    o->discount = 0.0;
    return HJR_OK;
}

const char *hjr_status_string(hjr_status s)
{
    switch (s) {
    case HJR_OK: return "ok";
    case HJR_NOT_CONVERGED: return "not converged (max_iter reached)";
    case HJR_PENDING: return "pending";
    case HJR_HORIZON: return "horizon reached";
    case HJR_ERR_INVALID_ARG: return "invalid argument";
    case HJR_ERR_UNSUPPORTED: return "unsupported";
    case HJR_ERR_NONFINITE: return "non-finite input";
    case HJR_ERR_OOM: return "out of device memory";
    case HJR_ERR_DEVICE: return "device error";
    case HJR_ERR_BUDGET: return "request exceeds the memory budget";
    case HJR_ERR_UNKNOWN_TICKET: return "unknown ticket";
    default: return "unknown status";
    }
}

const char *hjr_last_error(void) { return g_last_error.c_str(); }

int32_t hjr_device_count(void)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

static hjr_status solve_host(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l, const double *g,
                             const double *k, const hjr_options *opts, double *V_out, hjr_result *result)
{
    Request r;
    hjr_status s = prepare(r, grid, dyn, opts, k);
    if (s != HJR_OK) return s;
    if (!l || !V_out) return fail(HJR_ERR_INVALID_ARG, "l and V_out must not be NULL");
    if (g && opts->brs) return fail(HJR_ERR_INVALID_ARG, "the reachable-set mode takes no constraint function");
    Engine E(1);
    s = E.init(nullptr);
    if (s != HJR_OK) return s;
    std::vector<Request *> reqs{&r};
    s = run_all(E, reqs, true, {l}, {k}, opts->steps_per_sync, g);
    if (s == HJR_OK && r.status >= 0) {
        hipError_t e = hipMemcpy(V_out, r.V_dev, r.npts * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) s = fail(HJR_ERR_DEVICE, "copy of V failed: %s", hipGetErrorString(e));
    }
    E.drop(&r);
    if (s != HJR_OK) return s;
    if (result) *result = r.result;
    return r.status;
}

static hjr_status solve_dev(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l_dev, const double *g_dev,
                            const double *k_dev, const hjr_options *opts, double *V_dev, void *stream,
                            hjr_result *result)
{
    Request r;
    hjr_status s = prepare(r, grid, dyn, opts, k_dev);
    if (s != HJR_OK) return s;
    if (!l_dev || !V_dev) return fail(HJR_ERR_INVALID_ARG, "l_dev and V_dev must not be NULL");
    if (g_dev && opts->brs) return fail(HJR_ERR_INVALID_ARG, "the reachable-set mode takes no constraint function");
    r.l_dev = l_dev;
    r.k_dev = k_dev;
    r.g_dev = g_dev;
    r.V_dev = V_dev;
    Engine E(1);
    s = E.init((hipStream_t)stream);
    if (s != HJR_OK) return s;
    std::vector<Request *> reqs{&r};
    s = run_all(E, reqs, false, {}, {}, opts->steps_per_sync);
    E.drop(&r);
    if (s != HJR_OK) return s;
    if (result) *result = r.result;
    return r.status;
}

// ---------------------------------------------------------------------------------------------
// Allocation-free solve.  Its engine takes every device buffer from `scratch`, a file-scope
// device array of kScratchBytes that each GPU holds from the library's load until the process
// ends.  In host code the array's name is only a stand-in: the device address of each GPU's
// copy comes from hipGetSymbolAddress with that GPU current, once, and is kept per device.
// Calls on one GPU share its copy, so they are serialised by a per-device mutex; the contents
// left by the last call are never relied on (every buffer is written before it is read).
// ---------------------------------------------------------------------------------------------

namespace hjr {
constexpr size_t kScratchBytes = 64ull << 20;
constexpr int kMaxScratchDevices = 64;
}  // namespace hjr
static __device__ __align__(256) unsigned char scratch[hjr::kScratchBytes];
namespace hjr {
static std::mutex g_scratch_mu[kMaxScratchDevices];
static void *g_scratch_ptr[kMaxScratchDevices];

// The current device's scratch address (the caller holds g_scratch_mu[dev]).
static hjr_status scratch_address(int dev, void **out)
{
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(HJR_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HJR_OK;
}

// Scratch bytes a single solve's engine may take: the state and descriptor, the request's
// working arrays, and the flat and march tile lists of both precisions (the engine keeps room
// for twice the tiles it lists; the bound takes one tile per 256 nodes, the most the flat and
// march configurations list, plus padding of the march order, or the brick plan's own length
// where that is longer: its padding depends on how the grid's row pairs fall into blocks).
static size_t noalloc_bytes(const Request &r)
{
    size_t tiles = (size_t)((r.npts + kBlock - 1) / kBlock) + 8 * kBlock;
    if (brick_ok(r.grid, r.opts.spatial)) {
        std::vector<MTile> m;
        march_brick_tiles(0, r.grid.ndim, r.grid.n, m);
        tiles = std::max(tiles, m.size());
    }
    const size_t list = align256(std::max(2 * tiles * sizeof(MTile), (size_t)4096));
    return align256(sizeof(SolveState)) + align256(sizeof(Inst)) + request_bytes(r, false) + 4 * list;
}
}  // namespace hjr

hjr_status hjr_solve_device_noalloc(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l_dev,
                                    const double *k_dev, const hjr_options *opts, double *V_dev, void *stream,
                                    hjr_result *result)
{
    Request r;
    hjr_status s = prepare(r, grid, dyn, opts, k_dev);
    if (s != HJR_OK) return s;
    if (!l_dev || !V_dev) return fail(HJR_ERR_INVALID_ARG, "l_dev and V_dev must not be NULL");
    const size_t need = noalloc_bytes(r);
    if (need > kScratchBytes)
        return fail(HJR_ERR_BUDGET, "the problem needs %zu bytes of scratch memory; the allocation-free entry point "
                    "has %zu (use hjr_solve_device)", need, kScratchBytes);
    int dev = 0;
    HJR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(HJR_ERR_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> guard(g_scratch_mu[dev]);
    void *base = nullptr;
    s = scratch_address(dev, &base);
    if (s != HJR_OK) return s;
    r.l_dev = l_dev;
    r.k_dev = k_dev;
    r.V_dev = V_dev;
    Arena arena{(char *)base, kScratchBytes, 0};
    Engine E(1, &arena);
    s = E.init((hipStream_t)stream);
    if (s != HJR_OK) return s;
    std::vector<Request *> reqs{&r};
    s = run_all(E, reqs, false, {}, {}, opts->steps_per_sync);
    E.drop(&r);
    if (s != HJR_OK) return s;
    if (result) *result = r.result;
    return r.status;
}

hjr_status hjr_solve(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l, const double *k,
                     const hjr_options *opts, double *V_out, hjr_result *result)
{
    return solve_host(grid, dyn, l, nullptr, k, opts, V_out, result);
}

hjr_status hjr_solve_device(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l_dev, const double *k_dev,
                            const hjr_options *opts, double *V_dev, void *stream, hjr_result *result)
{
    return solve_dev(grid, dyn, l_dev, nullptr, k_dev, opts, V_dev, stream, result);
}

hjr_status hjr_local_dependencies(const hjr_grid *grid, int32_t reach, int64_t *nblocks, int64_t *ndeps,
                                  uint32_t *off, uint32_t *dep)
{
    uint64_t N = 0;
    hjr_status s = validate_grid(grid, HJR_UPWIND1, &N);
    if (s != HJR_OK) return s;
    if (reach < 1 || reach > 64) return fail(HJR_ERR_INVALID_ARG, "reach must lie in 1..64");
    if (!nblocks || !ndeps) return fail(HJR_ERR_INVALID_ARG, "nblocks and ndeps must not be NULL");
    std::vector<uint32_t> o, d;
    block_dependencies(*grid, N, reach, o, d);
    if (o.empty()) return fail(HJR_ERR_UNSUPPORTED, "the dependency lists would be too long");
    *nblocks = (int64_t)o.size() - 1;
    *ndeps = (int64_t)d.size();
    if (off) std::memcpy(off, o.data(), o.size() * 4);
    if (dep) std::memcpy(dep, d.data(), d.size() * 4);
    return HJR_OK;
}

hjr_status hjr_solve_reach_avoid(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l, const double *g,
                                 const double *k, const hjr_options *opts, double *V_out, hjr_result *result)
{
    if (!g) return fail(HJR_ERR_INVALID_ARG, "g must not be NULL");
    return solve_host(grid, dyn, l, g, k, opts, V_out, result);
}

hjr_status hjr_solve_reach_avoid_device(const hjr_grid *grid, const hjr_dynamics *dyn, const double *l_dev,
                                        const double *g_dev, const double *k_dev, const hjr_options *opts,
                                        double *V_dev, void *stream, hjr_result *result)
{
    if (!g_dev) return fail(HJR_ERR_INVALID_ARG, "g_dev must not be NULL");
    return solve_dev(grid, dyn, l_dev, g_dev, k_dev, opts, V_dev, stream, result);
}

hjr_status hjr_batch_solve(int32_t count, hjr_problem *problems)
{
    if (count < 0 || (count > 0 && !problems)) return fail(HJR_ERR_INVALID_ARG, "bad problem list");
    if (count == 0) return HJR_OK;
    std::vector<Request> rs(count);
    std::vector<Request *> reqs;
    std::vector<const double *> lh, kh;
    int sps = 0;
    for (int i = 0; i < count; ++i) {
        hjr_problem &p = problems[i];
        hjr_status s = prepare(rs[i], &p.grid, &p.dyn, &p.opts, p.k);
        if (s == HJR_OK && (!p.l || !p.V_out)) s = fail(HJR_ERR_INVALID_ARG, "problem %d: NULL array", i);
        if (s != HJR_OK) {
            p.status = s;
            return fail(s, "problem %d: %s", i, g_last_error.c_str());
        }
        reqs.push_back(&rs[i]);
        lh.push_back(p.l);
        kh.push_back(p.k);
        sps = std::max(sps, p.opts.steps_per_sync);
    }
    Engine E(count);
    hjr_status s = E.init(nullptr);
    if (s != HJR_OK) return s;
    E.prefer_graphs(true);
    s = run_all(E, reqs, true, lh, kh, sps);
    hjr_status first = HJR_OK;
    for (int i = 0; i < count; ++i) {
        Request &r = rs[i];
        if (s == HJR_OK && r.status >= 0) {
            hipError_t e = hipMemcpy(problems[i].V_out, r.V_dev, r.npts * 8, hipMemcpyDeviceToHost);
            if (e != hipSuccess) r.status = fail(HJR_ERR_DEVICE, "copy failed: %s", hipGetErrorString(e));
        }
        problems[i].status = s == HJR_OK ? r.status : s;
        problems[i].result = r.result;
        if (first == HJR_OK && problems[i].status != HJR_OK) first = problems[i].status;
        E.drop(&r);
    }
    return s != HJR_OK ? s : first;
}

// ---------------------------------------------------------------------------------------------
// Kernel timing
// ---------------------------------------------------------------------------------------------

hjr_status hjr_profile_enable(int32_t on)
{
    g_profile_on.store(on ? 1 : 0);
    return HJR_OK;
}

hjr_status hjr_profile_read(hjr_profile *out, int32_t reset)
{
    std::lock_guard<std::mutex> g(g_profile_mu);
    if (out) *out = g_profile;
    if (reset) std::memset(&g_profile, 0, sizeof g_profile);
    return HJR_OK;
}

int64_t hjr_march_plan(const hjr_grid *grid, int32_t config, int64_t *out, int64_t cap)
{
    uint64_t npts = 0;
    hjr_status st = validate_grid(grid, HJR_UPWIND1, &npts);
    if (st != HJR_OK) return st;
    if (!is_march(config) || !valid_config(config) || grid->ndim < 2 || cap < 0 || (cap > 0 && !out))
        return fail(HJR_ERR_INVALID_ARG, "bad march configuration %d, ndim %d or output", config, grid->ndim);
    std::vector<MTile> m;
    if (config == kMarchBrick) {
        if (!brick_ok(*grid, HJR_UPWIND1))
            return fail(HJR_ERR_INVALID_ARG, "bricks need a 6-D grid whose periodic dims among 1..3 have even lengths");
        march_brick_tiles(0, grid->ndim, grid->n, m);
    } else {
        march_tiles(0, grid->ndim, grid->n, config == kMarchFull ? 0 : -config, m);
    }
    const int64_t rows = config == kMarchBrick ? 8 : 1;
    for (int64_t t = 0; t < (int64_t)m.size() && t < cap; ++t) {
        out[5 * t + 0] = m[t].c0;
        out[5 * t + 1] = m[t].i0;
        out[5 * t + 2] = m[t].len;
        out[5 * t + 3] = m[t].cn;
        out[5 * t + 4] = rows;
    }
    return (int64_t)m.size();
}

// ---------------------------------------------------------------------------------------------
// Kernel-level entry points
// ---------------------------------------------------------------------------------------------

hjr_status hjr_cfl_dt(const hjr_grid *grid, const hjr_dynamics *dyn, double cfl, double dt_max, double *dt_out)
{
    if (!dt_out) return fail(HJR_ERR_INVALID_ARG, "dt_out must not be NULL");
    hjr_options o;
    hjr_default_options(&o);
    o.spatial = HJR_UPWIND1;
    o.precision = HJR_FP64;
    o.cfl = cfl;
    o.dt_max = dt_max;
    Request r;
    hjr_status s = prepare(r, grid, dyn, &o, nullptr);
    if (s != HJR_OK) return s;
    std::vector<double> zeros(r.npts, 0.0);
    Engine E(1);
    s = E.init(nullptr);
    if (s != HJR_OK) return s;
    s = E.admit(&r, true, zeros.data(), nullptr);
    if (s == HJR_OK) {
        SolveState st;
        hipError_t e = hipStreamSynchronize(E.stream());
        if (e == hipSuccess) e = hipMemcpy(&st, r.inst.state, sizeof st, hipMemcpyDeviceToHost);
        if (e != hipSuccess) s = fail(HJR_ERR_DEVICE, "state copy failed: %s", hipGetErrorString(e));
        else *dt_out = st.dt_nom;
    }
    std::vector<Request *> fin;
    E.finish(&r, fin, false);
    (void)hipStreamSynchronize(E.stream());
    E.drop(&r);
    return s;
}

hjr_status hjr_stage_device(const hjr_grid *grid, const hjr_dynamics *dyn, int32_t game, int32_t spatial,
                            int32_t temporal, int32_t stage, int32_t precision, double dt, const void *Vs,
                            const void *Vn, const void *l, void *out, double *delta_out, void *stream)
{
    hjr_options o;
    hjr_default_options(&o);
    o.game = game;
    o.spatial = spatial;
    o.temporal = temporal;
    o.precision = precision == HJR_FP32 ? HJR_FP32 : HJR_FP64;
    Request r;
    hjr_status s = prepare(r, grid, dyn, &o, nullptr);
    if (s != HJR_OK) return s;
    const int nst = temporal == HJR_TVDRK3 ? 3 : 1;
    if (stage < 1 || stage > nst) return fail(HJR_ERR_INVALID_ARG, "stage %d out of range 1..%d", stage, nst);
    if (!Vs || !Vn || !l || !out) return fail(HJR_ERR_INVALID_ARG, "NULL array");
    if (out == Vs) return fail(HJR_ERR_INVALID_ARG, "out must not alias Vs");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HJR_ERR_INVALID_ARG, "dt must be > 0");
    hipStream_t st = (hipStream_t)stream;
    const bool f32 = precision == HJR_FP32;
    const size_t esz = f32 ? 4 : 8;
    // descriptor with the caller's arrays in the roles the kernel expects for this stage
    Layout L = plan_layout(r, false, false);
    void *mem = nullptr;
    HJR_HIP(Pool::get().alloc(&mem, L.total + align256(sizeof(SolveState)) + align256(sizeof(Inst))));
    char *base = (char *)mem;
    SolveState *dstate = (SolveState *)(base + align256(L.total));
    Inst *dinst = (Inst *)((char *)dstate + align256(sizeof(SolveState)));
    std::vector<double> t64;
    std::vector<float> t32;
    build_inst(r, base, L, t64, t32, dstate);
    Inst I = r.inst;
    void *Vfield = (void *)Vn, *Afield = nullptr, *Bfield = nullptr;
    const int k = stage - 1;
    hipError_t e = hipSuccess;
    if (temporal == HJR_EULER) {
        Vfield = (void *)Vs;
        Afield = out;
    } else if (k == 0) {
        Vfield = (void *)Vs;
        Afield = out;
    } else if (k == 1) {
        Vfield = (void *)Vn;
        Afield = (void *)Vs;
        Bfield = out;
    } else {
        e = hipMemcpyAsync(out, Vn, r.npts * esz, hipMemcpyDeviceToDevice, st);
        Vfield = out;
        Bfield = (void *)Vs;
    }
    if (f32) {
        I.V32 = (float *)Vfield;
        I.A32 = (float *)Afield;
        I.B32 = (float *)Bfield;
        I.l32 = (const float *)l;
    } else {
        I.V64 = (double *)Vfield;
        I.A64 = (double *)Afield;
        I.B64 = (double *)Bfield;
        I.l64 = (const double *)l;
    }
    SolveState hs = initial_state(r);
    hs.dt_cur = dt;
    hs.dt_nom = dt;
    hs.done = kRunning;
    // the kernel variant the solvers use: the specialised kernel with the nodes-per-thread the
    // tuner chose for this size class (HJR_NPT overrides; HJR_FUSED=1 selects the fused kernel)
    bool fused = false;
    if (const char *fu = getenv("HJR_FUSED")) fused = atoi(fu) != 0;
    int npt = 0;
    if (const char *np = getenv("HJR_NPT")) npt = atoi(np);
    if (!valid_config(npt)) npt = 0;
    const uint64_t cols = r.npts / (uint64_t)grid->n[0];
    const bool march_ok = (spatial == HJR_UPWIND1 || spatial == HJR_WENO5) && grid->ndim >= 2 && cols >= kMarchMinColumns &&
                          r.npts * (f32 ? 4ull : 8ull) <= 0xffffffffull;
    if (is_march(npt) && !march_ok) npt = 0;
    const bool bricks = march_ok && brick_ok(*grid, spatial);
    if (npt == kMarchBrick && !bricks) npt = kMarchFull;
    if (!npt) npt = Tuner::get().choice(Tuner::key(f32 ? 0 : 1, dyn->id, spatial, r.npts, march_ok, bricks));
    if (!npt || fused) npt = kFusedNpt;
    std::vector<Tile> tiles;
    std::vector<MTile> mtiles;
    if (npt == kMarchBrick) {
        march_brick_tiles(0, grid->ndim, grid->n, mtiles);
    } else if (is_march(npt)) {
        march_tiles(0, grid->ndim, grid->n, npt == kMarchFull ? 0 : -npt, mtiles);
    } else {
        for (uint64_t s0 = 0; s0 < r.npts; s0 += (uint64_t)npt * kBlock) tiles.push_back(Tile{0, (uint32_t)s0, npt});
    }
    const size_t tl_bytes = is_march(npt) ? mtiles.size() * sizeof(MTile) : tiles.size() * sizeof(Tile);
    const void *tl_host = is_march(npt) ? (const void *)mtiles.data() : (const void *)tiles.data();
    void *dtl = nullptr;
    if (e == hipSuccess) e = Pool::get().alloc(&dtl, tl_bytes);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)I.tab64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync((void *)I.tab32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dstate, &hs, sizeof hs, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dinst, &I, sizeof I, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dtl, tl_host, tl_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        if (is_march(npt))
            e = launch_march(!f32, dyn->id, spatial, npt == kMarchBrick, dinst, (const MTile *)dtl, (int)mtiles.size(),
                             k, st);
        else if (fused)
            e = launch_stage(!f32, dinst, (const Tile *)dtl, (int)tiles.size(), k, 0, st);
        else
            e = launch_stage_one(!f32, dyn->id, spatial, npt, dinst, (const Tile *)dtl, (int)tiles.size(), k, 0, st);
    }
    SolveState after;
    if (e == hipSuccess) e = hipMemcpyAsync(&after, dstate, sizeof after, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    Pool::get().release(dtl);
    Pool::get().release(mem);
    if (e != hipSuccess) return fail(HJR_ERR_DEVICE, "stage launch failed: %s", hipGetErrorString(e));
    const bool last = temporal == HJR_EULER || k == 2;
    if (delta_out && last) *delta_out = __builtin_bit_cast(double, after.delta_bits);
    return HJR_OK;
}

int32_t hjr_num_controls(int32_t dyn_id)
{
    switch (dyn_id) {
    case HJR_DYN_DOUBLE_INTEGRATOR: return 1;
    case HJR_DYN_DUBINS3: return 1;
    case HJR_DYN_UNICYCLE4: return 2;
    case HJR_DYN_QUAD6: return 3;
    case HJR_DYN_QUAD10_XY: return 1;
    case HJR_DYN_QUAD10_Z: return 1;
    default: return 0;
    }
}

hjr_status hjr_gradient_device(const hjr_grid *grid, int32_t spatial, const double *V, double *table, void *stream)
{
    uint64_t N = 0;
    hjr_status s = validate_grid(grid, spatial, &N);
    if (s != HJR_OK) return s;
    if (!V || !table) return fail(HJR_ERR_INVALID_ARG, "NULL array");
    Inst I;
    std::memset(&I, 0, sizeof I);
    fill_grid(*grid, N, I);
    hipError_t e = launch_gradient(I, spatial, V, table, (hipStream_t)stream);
    if (e != hipSuccess) return fail(HJR_ERR_DEVICE, "gradient launch failed: %s", hipGetErrorString(e));
    return HJR_OK;
}

hjr_status hjr_safe_control_device(const hjr_grid *grid, const hjr_dynamics *dyn, int32_t game, const double *table,
                                   const double *x, int64_t nq, double *u, double *p, double *v, void *stream)
{
    uint64_t N = 0;
    hjr_status s = validate(grid, dyn, HJR_UPWIND1, &N);
    if (s != HJR_OK) return s;
    if (game != HJR_AVOID && game != HJR_REACH) return fail(HJR_ERR_INVALID_ARG, "bad game %d", game);
    if (nq < 0 || nq > ((int64_t)1 << 38)) return fail(HJR_ERR_INVALID_ARG, "query count %lld out of range", (long long)nq);
    if (nq == 0) return HJR_OK;
    if (!table || !x || !u) return fail(HJR_ERR_INVALID_ARG, "NULL array");
    CtlGrid G;
    std::memset(&G, 0, sizeof G);
    G.ndim = grid->ndim;
    G.npts = (uint32_t)N;
    G.periodic = grid->periodic_mask;
    uint32_t st = 1;
    for (int d = grid->ndim - 1; d >= 0; --d) {
        G.n[d] = grid->n[d];
        G.stride[d] = st;
        st *= (uint32_t)grid->n[d];
        G.lo[d] = grid->lo[d];
        G.dx[d] = grid_dx(*grid, d);
    }
    CtlModel M;
    std::memset(&M, 0, sizeof M);
    M.game = game;
    for (int i = 0; i < dyn->n_params && i < 16; ++i) M.q[i] = dyn->params[i];
    hipError_t e = launch_control(G, M, dyn->id, table, x, nq, u, p, v, (hipStream_t)stream);
    if (e != hipSuccess) return fail(HJR_ERR_DEVICE, "control launch failed: %s", hipGetErrorString(e));
    return HJR_OK;
}

}  // extern "C"

// ============================================================================================
// Serving context
// ============================================================================================

struct hjr_ctx {
    int device = 0;
    size_t budget = 0;
    std::unique_ptr<Engine> engine;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<int64_t, std::unique_ptr<Request>> all;
    int64_t next_ticket = 1;
    size_t in_use = 0, peak = 0;
    int64_t admitted = 0, finished = 0;
    bool stop = false;
    hjr_status fatal = HJR_OK;
    std::string fatal_msg;
    std::thread worker;
    ChunkPolicy policy{0};
    int max_chunk = 32;

    void loop()
    {
        (void)hipSetDevice(device);
        std::vector<Request *> fin;
        while (true) {
            {
                std::unique_lock<std::mutex> g(mu);
                cv.wait(g, [&] { return stop || !queue.empty() || engine->active() > 0; });
                if (stop && queue.empty() && engine->active() == 0) return;
                // admit in arrival order while memory and slots allow
                while (!queue.empty() && engine->has_free_slot()) {
                    Request *r = queue.front();
                    const size_t b = request_bytes(*r, false);
                    if (in_use + b > budget) break;
                    queue.pop_front();
                    in_use += b;
                    peak = std::max(peak, in_use);
                    g.unlock();
                    hjr_status s = engine->admit(r, false, nullptr, nullptr);
                    g.lock();
                    ++admitted;
                    if (s != HJR_OK) {
                        r->status = s;
                        r->done = true;
                        in_use -= b;
                        cv_done.notify_all();
                    }
                }
            }
            if (engine->active() == 0) continue;
            // adaptive chunk, capped so that waiting requests join within max_chunk steps
            hjr_status s = engine->run_chunk(std::min(policy.next(), max_chunk));
            fin.clear();
            if (s == HJR_OK) s = engine->update(fin);
            if (s == HJR_OK) policy.after(!fin.empty(), engine->predict_steps());
            if (s == HJR_OK && !fin.empty()) {
                hipError_t e = hipStreamSynchronize(engine->stream());
                if (e != hipSuccess) s = fail(HJR_ERR_DEVICE, "sync failed: %s", hipGetErrorString(e));
            }
            std::lock_guard<std::mutex> g(mu);
            if (s != HJR_OK) {
                fatal = s;
                fatal_msg = g_last_error;
                for (auto &kv : all)
                    if (!kv.second->done) {
                        kv.second->status = s;
                        kv.second->done = true;
                    }
                queue.clear();
                cv_done.notify_all();
                return;
            }
            for (Request *r : fin) {
                in_use -= r->bytes;
                engine->drop(r);
                r->done = true;
                ++finished;
            }
            if (!fin.empty()) cv_done.notify_all();
        }
    }
};

extern "C" {

hjr_status hjr_ctx_create(int32_t device, size_t hbm_budget_bytes, hjr_ctx **out)
{
    if (!out) return fail(HJR_ERR_INVALID_ARG, "out must not be NULL");
    int n = 0;
    HJR_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(HJR_ERR_INVALID_ARG, "device %d out of range", device);
    HJR_HIP(hipSetDevice(device));
    auto c = std::make_unique<hjr_ctx>();
    c->device = device;
    size_t fr = 0, tot = 0;
    HJR_HIP(hipMemGetInfo(&fr, &tot));
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
    c->engine = std::make_unique<Engine>(256);
    hjr_status s = c->engine->init(nullptr);
    if (s != HJR_OK) return s;
    c->engine->prefer_graphs(true);
    hjr_ctx *p = c.release();
    p->worker = std::thread([p] { p->loop(); });
    *out = p;
    return HJR_OK;
}

hjr_status hjr_submit(hjr_ctx *ctx, const hjr_grid *grid, const hjr_dynamics *dyn, const double *l_dev,
                      const double *k_dev, const hjr_options *opts, double *V_dev, int64_t *ticket)
{
    if (!ctx || !ticket) return fail(HJR_ERR_INVALID_ARG, "ctx and ticket must not be NULL");
    auto r = std::make_unique<Request>();
    hjr_status s = prepare(*r, grid, dyn, opts, k_dev);
    if (s != HJR_OK) return s;
    if (!l_dev || !V_dev) return fail(HJR_ERR_INVALID_ARG, "l_dev and V_dev must not be NULL");
    r->l_dev = l_dev;
    r->k_dev = k_dev;
    r->V_dev = V_dev;
    if (request_bytes(*r, false) > ctx->budget)
        return fail(HJR_ERR_BUDGET, "request needs %zu bytes, budget is %zu", request_bytes(*r, false), ctx->budget);
    std::lock_guard<std::mutex> g(ctx->mu);
    if (ctx->fatal != HJR_OK) return fail(ctx->fatal, "context failed: %s", ctx->fatal_msg.c_str());
    r->ticket = ctx->next_ticket++;
    r->t_submit = now_s();
    *ticket = r->ticket;
    ctx->queue.push_back(r.get());
    ctx->all[r->ticket] = std::move(r);
    ctx->cv.notify_all();
    return HJR_OK;
}

hjr_status hjr_poll(hjr_ctx *ctx, int64_t ticket, hjr_result *result)
{
    if (!ctx) return fail(HJR_ERR_INVALID_ARG, "ctx must not be NULL");
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->all.find(ticket);
    if (it == ctx->all.end()) return fail(HJR_ERR_UNKNOWN_TICKET, "unknown ticket %lld", (long long)ticket);
    Request *r = it->second.get();
    if (!r->done) return HJR_PENDING;
    hjr_status s = r->status;
    if (result) *result = r->result;
    if (s < 0) fail(s, "request %lld failed", (long long)ticket);
    ctx->all.erase(it);
    return s;
}

hjr_status hjr_ctx_drain(hjr_ctx *ctx)
{
    if (!ctx) return fail(HJR_ERR_INVALID_ARG, "ctx must not be NULL");
    std::unique_lock<std::mutex> g(ctx->mu);
    ctx->cv_done.wait(g, [&] {
        for (auto &kv : ctx->all)
            if (!kv.second->done) return false;
        return true;
    });
    return ctx->fatal;
}

hjr_status hjr_ctx_get_stats(hjr_ctx *ctx, hjr_ctx_stats *st)
{
    if (!ctx || !st) return fail(HJR_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(ctx->mu);
    st->admitted = ctx->admitted;
    st->finished = ctx->finished;
    st->queued = (int64_t)ctx->queue.size();
    st->running = ctx->engine->active();
    st->bytes_in_use = (int64_t)ctx->in_use;
    st->bytes_peak = (int64_t)ctx->peak;
    st->budget = (int64_t)ctx->budget;
    st->chunks = ctx->engine->chunks();
    st->launches = ctx->engine->launches();
    return HJR_OK;
}

hjr_status hjr_ctx_destroy(hjr_ctx *ctx)
{
    if (!ctx) return HJR_OK;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->stop = true;
        ctx->queue.clear();
        ctx->cv.notify_all();
    }
    if (ctx->worker.joinable()) ctx->worker.join();
    hjr_status s = ctx->fatal;
    delete ctx;
    return s;
}

}  // extern "C"
