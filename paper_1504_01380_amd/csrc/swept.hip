// swept.hip -- host runtime and C ABI of libswept.so (declared in swept.h).
//
// Planning, scratch management, stream handling and the launch sequences of
// the swept and naive schedules.  All arithmetic runs in the kernels of
// kernels.hpp; this file only validates, plans and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "swept.h"
#include "kernels.hpp"

namespace {

using namespace swept;

struct Context {
    bool ready = false;
    int device = -1;
    hipStream_t stream = nullptr;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    int tile_w = 0;   // 0 = automatic
    int ppl = 0;      // pairs per lane, 0 = automatic
    int mode = SWEPT_MODE_AUTO;
    bool profiling = false;
    std::vector<hipEvent_t> events;   // events[i] before stage i, events[i+1] after it
    std::vector<int32_t> kinds;       // kernel used by each recorded stage
    int64_t recorded = 0;             // stages recorded by the last swept run
};

Context g_ctx;
thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(SWEPT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                        \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
    } while (0)

void batch_release();

int ensure_scratch(size_t bytes)
{
    if (bytes <= g_ctx.scratch_bytes)
        return SWEPT_OK;
    if (g_ctx.scratch) {
        HIP_TRY(hipStreamSynchronize(g_ctx.stream));
        batch_release();
        HIP_TRY(hipFree(g_ctx.scratch));
        g_ctx.scratch = nullptr;
        g_ctx.scratch_bytes = 0;
    }
    hipError_t e = hipMalloc(&g_ctx.scratch, bytes);
    if (e != hipSuccess) {
        g_ctx.scratch = nullptr;
        (void)hipGetLastError();
        return fail(SWEPT_ENOMEM, "hipMalloc of %zu bytes of scratch failed: %s", bytes,
                    hipGetErrorString(e));
    }
    g_ctx.scratch_bytes = bytes;
    return SWEPT_OK;
}

// ------------------------------------------------------------------ stencils

int substeps_of(int id) { return id == SWEPT_KS_F64 ? 4 : 1; }

size_t pt_bytes(int id)
{
    switch (id) {
    case SWEPT_HEAT_F64: return sizeof(HeatF64::Pt);
    case SWEPT_HEAT_F32: return sizeof(HeatF32::Pt);
    default: return sizeof(KSF64::Pt);
    }
}

int check_common(const void* u, int64_t nx, int64_t nsteps, int32_t id, const double* params,
                 int32_t nparams)
{
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    if (!u)
        return fail(SWEPT_EINVAL, "u is NULL");
    if (nx < 3)
        return fail(SWEPT_EINVAL, "nx = %lld: need at least 3 points", (long long)nx);
    if (nsteps < 0)
        return fail(SWEPT_EINVAL, "nsteps = %lld is negative", (long long)nsteps);
    if (id != SWEPT_HEAT_F64 && id != SWEPT_HEAT_F32 && id != SWEPT_KS_F64)
        return fail(SWEPT_EINVAL, "unknown stencil id %d", id);
    const int need = id == SWEPT_KS_F64 ? 2 : 1;
    if (!params || nparams < need)
        return fail(SWEPT_EINVAL, "stencil %d needs %d parameter(s)", id, need);
    for (int i = 0; i < need; ++i)
        if (!std::isfinite(params[i]))
            return fail(SWEPT_EINVAL, "parameter %d is not finite", i);
    if (id == SWEPT_KS_F64 && !(params[1] > 0.0))
        return fail(SWEPT_EINVAL, "KS needs dx > 0");
    return SWEPT_OK;
}

HeatF64::Consts heat64_consts(const double* p) { return HeatF64::Consts{p[0]}; }
HeatF32::Consts heat32_consts(const double* p) { return HeatF32::Consts{(float)p[0]}; }
KSF64::Consts ks_consts(const double* p)
{
    const double dt = p[0], dx = p[1];
    return KSF64::Consts{dt, 0.5 * dt, 1.0 / (2.0 * dx), 1.0 / (dx * dx)};
}

// --------------------------------------------------------------------- plan

struct Plan {
    int64_t W = 0, k = 0, tiles = 0, stages = 0;
    int P = 1;
    int mode = SWEPT_MODE_NAIVE;
};

constexpr size_t kMaxLds = 64 * 1024;

// Measured on MI355X (20,000-step heat at N = 2^24, binary64 and binary32;
// KS at N = 2^20; heat at N = 4096): W = 1024 is fastest for every stencil on
// large grids (a 2k-entry LDS edge chain small enough for ~10 workgroups per
// CU); small grids keep at least 16 tiles so that more CUs take part.
int64_t target_tile(int /*id*/) { return 1024; }

int auto_ppl(int /*id*/, int64_t k) { return k >= 512 ? 4 : (k >= 128 ? 2 : 1); }

bool tile_fits(int id, int64_t nx, int64_t W)
{
    return W >= 2 && W % 2 == 0 && nx % W == 0 && (size_t)W * pt_bytes(id) <= kMaxLds;
}

// Tiles of W = 2k points (paper, Section 3: each node owns an even number of
// points); stages 0..ceil(L/k).
int make_plan(int64_t nx, int64_t nsteps, int32_t id, Plan* p)
{
    *p = Plan{};
    const int64_t L = nsteps * substeps_of(id);
    if (g_ctx.mode == SWEPT_MODE_NAIVE) {
        p->mode = SWEPT_MODE_NAIVE;
        return SWEPT_OK;
    }
    int64_t W = 0;
    if (g_ctx.tile_w > 0) {
        if (!tile_fits(id, nx, g_ctx.tile_w))
            return fail(SWEPT_EINVAL,
                        "tile width %d must be even, divide nx = %lld and fit 64 KB of LDS",
                        g_ctx.tile_w, (long long)nx);
        W = g_ctx.tile_w;
    } else {
        const int64_t cap = std::min(target_tile(id), std::max<int64_t>(2, nx / 16));
        for (int64_t w = cap - (cap & 1); w >= 2; w -= 2)
            if (tile_fits(id, nx, w)) {
                W = w;
                break;
            }
    }
    if (W == 0) {
        if (g_ctx.mode == SWEPT_MODE_STAGE || g_ctx.mode == SWEPT_MODE_STAGE_BANDED)
            return fail(SWEPT_EUNSUPPORTED, "nx = %lld has no even tile width", (long long)nx);
        p->mode = SWEPT_MODE_NAIVE;
        return SWEPT_OK;
    }
    p->W = W;
    p->k = W / 2;
    p->tiles = nx / W;
    p->stages = L == 0 ? 0 : 1 + (L + p->k - 1) / p->k;
    p->P = g_ctx.ppl > 0 ? g_ctx.ppl : auto_ppl(id, p->k);
    p->mode = SWEPT_MODE_STAGE;
    return SWEPT_OK;
}

// ------------------------------------------------------------- swept launch

template <class S, int P>
void launch_stage(const StageArgs<S>& a, size_t lds, hipStream_t st, int tiles, bool cont)
{
    if (cont)
        hipLaunchKernelGGL((swept_diamond_cont_kernel<S, P>), dim3(tiles), dim3(64), lds, st, a);
    else
        hipLaunchKernelGGL((swept_stage_kernel<S, P>), dim3(tiles), dim3(64), lds, st, a);
}

// Full diamonds (below the target level, k a multiple of the band 64P) run
// on the continuous kernel; the triangle and capped stages on the banded one.
bool use_continuous(const Plan& p, int64_t s, int64_t L)
{
    const int64_t b = (s - 1) * p.k;
    return g_ctx.mode != SWEPT_MODE_STAGE_BANDED && s > 0 && b + 2 * p.k - 1 <= L &&
           p.k % (64 * p.P) == 0;
}

int reserve_events(int64_t stages)
{
    g_ctx.recorded = 0;
    while ((int64_t)g_ctx.events.size() < stages + 1) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        g_ctx.events.push_back(e);
    }
    g_ctx.kinds.assign((size_t)stages, 0);
    return SWEPT_OK;
}

void release_events()
{
    for (hipEvent_t e : g_ctx.events)
        (void)hipEventDestroy(e);
    g_ctx.events.clear();
    g_ctx.kinds.clear();
    g_ctx.recorded = 0;
}

template <class S>
int run_swept(void* u, int64_t nx, int64_t L, const typename S::Consts& c, const Plan& p)
{
    using Pt = typename S::Pt;
    const size_t edge = (size_t)nx * sizeof(Pt);  // tiles * k * 2 points
    int rc = ensure_scratch(3 * edge);
    if (rc)
        return rc;
    Pt* re = static_cast<Pt*>(g_ctx.scratch);
    Pt* le[2] = {re + nx, re + 2 * nx};
    const size_t lds = (size_t)p.W * sizeof(Pt);

    StageArgs<S> a{};
    a.u = static_cast<typename S::T*>(u);
    a.re = re;
    a.re_out = re;
    a.n = nx;
    a.L = L;
    a.k = (int)p.k;
    a.tiles = (int)p.tiles;
    a.c = c;
    if (g_ctx.profiling) {
        rc = reserve_events(p.stages);
        if (rc)
            return rc;
        HIP_TRY(hipEventRecord(g_ctx.events[0], g_ctx.stream));
    }
    for (int64_t s = 0; s < p.stages; ++s) {
        a.tri = s == 0;
        a.b = (s - 1) * p.k;
        a.J0 = (p.k + s * p.k) % nx;
        a.le_in = le[(s + 1) & 1];
        a.le_out = le[s & 1];
        const bool cont = use_continuous(p, s, L);
        switch (p.P) {
        case 1: launch_stage<S, 1>(a, lds, g_ctx.stream, (int)p.tiles, cont); break;
        case 2: launch_stage<S, 2>(a, lds, g_ctx.stream, (int)p.tiles, cont); break;
        case 4: launch_stage<S, 4>(a, lds, g_ctx.stream, (int)p.tiles, cont); break;
        case 8: launch_stage<S, 8>(a, lds, g_ctx.stream, (int)p.tiles, cont); break;
        default: return fail(SWEPT_EINVAL, "pairs per lane %d not in {1,2,4,8}", p.P);
        }
        if (g_ctx.profiling) {
            g_ctx.kinds[(size_t)s] = cont ? 1 : 0;
            HIP_TRY(hipEventRecord(g_ctx.events[(size_t)s + 1], g_ctx.stream));
        }
    }
    HIP_TRY(hipGetLastError());
    if (g_ctx.profiling)
        g_ctx.recorded = p.stages;
    return SWEPT_OK;
}

unsigned grid_for(int64_t n, int block)
{
    const int64_t b = (n + block - 1) / block;
    return (unsigned)std::min<int64_t>(b, 1 << 20);
}

// ----------------------------------------------------------- swept adjoint

// Tile for the adjoint: one lane per point of a level (2k <= 64) and the
// region's forward and cotangent values in 64 KB of LDS.
template <class S>
size_t adjoint_lds(int64_t k)
{
    return (size_t)(2 * k + 1) * (size_t)(2 * k + 4) *
           (sizeof(typename S::Pt) + sizeof(typename S::Ad));
}

template <class S>
int64_t adjoint_depth(int64_t nx, int64_t want)
{
    for (int64_t k = std::min<int64_t>(32, want > 0 ? want : 32); k >= 1; --k)
        if (nx % (2 * k) == 0 && adjoint_lds<S>(k) <= kMaxLds)
            return k;
    return 0;
}

template <class S>
int run_adjoint(const void* u0v, void* gradv, int64_t nx, int64_t nsteps, const double* params,
                const typename S::Consts& c, int64_t win_first, double wgt, const void* cotv)
{
    using Pt = typename S::Pt;
    using Ad = typename S::Ad;
    using T = typename S::T;
    const T* u0 = static_cast<const T*>(u0v);
    T* grad = static_cast<T*>(gradv);
    const T* cot = static_cast<const T*>(cotv);
    const T two_w = (T)(2.0 * wgt);
    const int64_t L = nsteps * S::NPHASE;
    if (L == 0) {
        hipLaunchKernelGGL((adjoint_seed_kernel<S>), dim3(grid_for(nx, 256)), dim3(256), 0,
                           g_ctx.stream, u0, cot, grad, nx, two_w, win_first <= 0 ? 1 : 0);
        HIP_TRY(hipGetLastError());
        return SWEPT_OK;
    }
    const int64_t k = adjoint_depth<S>(nx, g_ctx.tile_w > 0 ? g_ctx.tile_w / 2 : 0);
    if (k == 0)
        return fail(SWEPT_EUNSUPPORTED, "nx = %lld has no even tile width for the adjoint",
                    (long long)nx);
    const int64_t tiles = nx / (2 * k);
    const int64_t stages = 1 + (L + k - 1) / k;
    // checkpoints: right and left edges of every stage; cotangent hand-over buffers
    const size_t ck = (size_t)stages * nx * sizeof(Pt);
    const size_t ae = 2 * (size_t)nx * sizeof(Ad);        // tiles * 2 sides * k * 2
    const size_t fh = (size_t)nx * sizeof(Pt);            // tiles * 2 sides * k
    const size_t uf = ((size_t)nx * sizeof(T) + 255) / 256 * 256;
    int rc = ensure_scratch(2 * ck + 2 * ae + 2 * fh + uf);
    if (rc)
        return rc;
    unsigned char* base = static_cast<unsigned char*>(g_ctx.scratch);
    Pt* ck_re = reinterpret_cast<Pt*>(base);
    Pt* ck_le = reinterpret_cast<Pt*>(base + ck);
    Ad* aeb[2] = {reinterpret_cast<Ad*>(base + 2 * ck), reinterpret_cast<Ad*>(base + 2 * ck + ae)};
    Pt* fhb[2] = {reinterpret_cast<Pt*>(base + 2 * ck + 2 * ae),
                  reinterpret_cast<Pt*>(base + 2 * ck + 2 * ae + fh)};

    // forward pass on a copy of u0, keeping the edges of every stage
    T* ufwd = reinterpret_cast<T*>(base + 2 * ck + 2 * ae + 2 * fh);
    HIP_TRY(hipMemcpyAsync(ufwd, u0, nx * sizeof(T), hipMemcpyDeviceToDevice, g_ctx.stream));
    StageArgs<S> a{};
    a.u = ufwd;
    a.n = nx;
    a.L = L;
    a.k = (int)k;
    a.tiles = (int)tiles;
    a.c = c;
    const size_t lds_fwd = (size_t)2 * k * sizeof(Pt);
    for (int64_t s = 0; s < stages; ++s) {
        a.tri = s == 0;
        a.b = (s - 1) * k;
        a.J0 = (k + s * k) % nx;
        a.re = s > 0 ? ck_re + (s - 1) * nx : ck_re;
        a.re_out = ck_re + s * nx;
        a.le_in = s > 0 ? ck_le + (s - 1) * nx : ck_le;
        a.le_out = ck_le + s * nx;
        hipLaunchKernelGGL((swept_stage_kernel<S, 1>), dim3(tiles), dim3(64), lds_fwd,
                           g_ctx.stream, a);
    }
    HIP_TRY(hipGetLastError());

    // reverse pass
    AdjArgs<S> g{};
    g.u0 = u0;
    g.grad = grad;
    g.cot = cot;
    g.n = nx;
    g.L = L;
    g.win_first = win_first;
    g.two_w = two_w;
    g.k = (int)k;
    g.tiles = (int)tiles;
    g.c = c;
    const size_t lds_adj = adjoint_lds<S>(k);
    for (int64_t s = stages - 1; s >= 0; --s) {
        g.tri = s == 0;
        g.b = (s - 1) * k;
        g.J0 = (k + s * k) % nx;
        g.re_in = s > 0 ? ck_re + (s - 1) * nx : ck_re;
        g.le_in = s > 0 ? ck_le + (s - 1) * nx : ck_le;
        g.has_later = s + 1 < stages;
        g.ae_in = aeb[(s + 1) & 1];
        g.fh_in = fhb[(s + 1) & 1];
        g.ae_out = aeb[s & 1];
        g.fh_out = fhb[s & 1];
        hipLaunchKernelGGL((swept_adjoint_kernel<S>), dim3(tiles), dim3(64), lds_adj,
                           g_ctx.stream, g);
    }
    HIP_TRY(hipGetLastError());
    (void)params;
    return SWEPT_OK;
}

// -------------------------------------------------------------------- batch

// Per-instance tiling for the batch: tiles of width 2k_t, k_t in {base,
// base+1}, summing to the ring length; odd rings run on their two-fold cover
// (the same bits: the scheme is translation-equivariant, so a field repeated
// twice stays repeated).
struct BatchPlanInst {
    int64_t n_user, n_ring, L, x_off, e_off, f_off, stages;
    int tiles, kmax, stencil;
};

struct BatchCache {
    std::vector<int64_t> key;       // the batch's defining numbers and pointers
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
BatchCache g_batch;

void batch_release()
{
    if (g_batch.exec)
        (void)hipGraphExecDestroy(g_batch.exec);
    if (g_batch.graph)
        (void)hipGraphDestroy(g_batch.graph);
    g_batch = BatchCache{};
}

int64_t batch_depth(int id, int64_t nring, int64_t want)
{
    // target depth k; tiles never exceed the LDS chain budget
    const int64_t lim = (int64_t)(kMaxLds / (2 * pt_bytes(id))) - 1;
    const int64_t k = std::min<int64_t>(want, lim);
    return std::max<int64_t>(1, std::min<int64_t>(k, nring / 2));
}

template <class S>
int launch_batch_stage(const BatchInst<S>* inst, const BatchTask* tasks, const int64_t* X,
                       typename S::Pt* re, typename S::Pt* le0, typename S::Pt* le1, int stage,
                       int64_t ntasks, int kmax, hipStream_t st)
{
    if (ntasks <= 0)
        return SWEPT_OK;
    BatchArgs<S> a{};
    a.inst = inst;
    a.tasks = tasks;
    a.X = X;
    a.re = re;
    a.le[0] = le0;
    a.le[1] = le1;
    a.stage = stage;
    const size_t lds = (size_t)2 * kmax * sizeof(typename S::Pt);
    hipLaunchKernelGGL((swept_batch_kernel<S, 2>), dim3((unsigned)ntasks), dim3(64), lds, st, a);
    return SWEPT_OK;
}

int run_batch(void* const* u, const int64_t* nx, const int64_t* nsteps, const int32_t* ids,
              const double* params, int64_t count)
{
    using PtH = HeatF64::Pt;
    using PtK = KSF64::Pt;
    // ---- plan
    std::vector<BatchPlanInst> P((size_t)count);
    std::vector<int64_t> X;
    int64_t e_heat = 0, e_ks = 0, f_tot = 0;
    for (int64_t j = 0; j < count; ++j) {
        BatchPlanInst& p = P[(size_t)j];
        p.stencil = ids[j];
        p.n_user = nx[j];
        p.n_ring = (nx[j] % 2 == 0) ? nx[j] : 2 * nx[j];
        p.L = nsteps[j] * substeps_of(ids[j]);
        const int64_t want = g_ctx.tile_w > 0 ? g_ctx.tile_w / 2 : 256;
        const int64_t k = batch_depth(ids[j], p.n_ring, want);
        const int64_t half = p.n_ring / 2;
        const int64_t T = std::max<int64_t>(1, half / k);
        const int64_t base = half / T, rem = half % T;
        p.tiles = (int)T;
        p.kmax = (int)(base + (rem ? 1 : 0));
        p.x_off = (int64_t)X.size();
        X.push_back(0);
        for (int64_t t = 0; t < T; ++t)
            X.push_back(X.back() + 2 * (base + (t < rem ? 1 : 0)));
        // stage s >= 1 of tile t starts at level (X_{t+s} - X_{t+1})/2 >= (s-1)*base
        p.stages = p.L == 0 ? 0 : 2 + (p.L + base - 1) / base;
        if (p.stencil == SWEPT_KS_F64) {
            p.e_off = e_ks;
            e_ks += p.n_ring;
        } else {
            p.e_off = e_heat;
            e_heat += p.n_ring;
        }
        p.f_off = -1;
        if (p.n_ring != p.n_user) {
            p.f_off = f_tot;
            f_tot += p.n_ring;
        }
    }
    // tasks of each stencil, sorted by the instance's stage count (descending),
    // so that the tasks of stage g are a prefix of the list
    std::vector<int64_t> order((size_t)count);
    for (int64_t j = 0; j < count; ++j)
        order[(size_t)j] = j;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return P[(size_t)a].stages > P[(size_t)b].stages; });
    std::vector<BatchTask> th, tk;
    std::vector<int64_t> sh, sk;  // stage count of the instance of each task
    int kmax_h = 1, kmax_k = 1;
    for (int64_t j : order) {
        const BatchPlanInst& p = P[(size_t)j];
        if (p.L == 0)
            continue;
        auto& tv = p.stencil == SWEPT_KS_F64 ? tk : th;
        auto& sv = p.stencil == SWEPT_KS_F64 ? sk : sh;
        for (int t = 0; t < p.tiles; ++t) {
            tv.push_back(BatchTask{(int)j, t});
            sv.push_back(p.stages);
        }
        int& km = p.stencil == SWEPT_KS_F64 ? kmax_k : kmax_h;
        km = std::max(km, p.kmax);
    }
    int64_t smax = 0;
    for (const auto& p : P)
        smax = std::max(smax, p.stages);

    // ---- device memory: [inst heat][inst ks][X][tasks h][tasks k][edges h][edges k][fields]
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_ih = al(sizeof(BatchInst<HeatF64>) * (size_t)count);
    const size_t b_ik = al(sizeof(BatchInst<KSF64>) * (size_t)count);
    const size_t b_x = al(sizeof(int64_t) * X.size());
    const size_t b_th = al(sizeof(BatchTask) * std::max<size_t>(1, th.size()));
    const size_t b_tk = al(sizeof(BatchTask) * std::max<size_t>(1, tk.size()));
    const size_t b_eh = al(3 * (size_t)e_heat * sizeof(PtH));
    const size_t b_ek = al(3 * (size_t)e_ks * sizeof(PtK));
    const size_t b_f = al((size_t)f_tot * sizeof(double));
    int rc = ensure_scratch(b_ih + b_ik + b_x + b_th + b_tk + b_eh + b_ek + b_f);
    if (rc)
        return rc;
    unsigned char* base = static_cast<unsigned char*>(g_ctx.scratch);
    auto* d_ih = reinterpret_cast<BatchInst<HeatF64>*>(base);
    auto* d_ik = reinterpret_cast<BatchInst<KSF64>*>(base + b_ih);
    auto* d_x = reinterpret_cast<int64_t*>(base + b_ih + b_ik);
    auto* d_th = reinterpret_cast<BatchTask*>(base + b_ih + b_ik + b_x);
    auto* d_tk = reinterpret_cast<BatchTask*>(base + b_ih + b_ik + b_x + b_th);
    auto* d_eh = reinterpret_cast<PtH*>(base + b_ih + b_ik + b_x + b_th + b_tk);
    auto* d_ek = reinterpret_cast<PtK*>(base + b_ih + b_ik + b_x + b_th + b_tk + b_eh);
    auto* d_f = reinterpret_cast<double*>(base + b_ih + b_ik + b_x + b_th + b_tk + b_eh + b_ek);

    std::vector<BatchInst<HeatF64>> ih((size_t)count);
    std::vector<BatchInst<KSF64>> ik((size_t)count);
    for (int64_t j = 0; j < count; ++j) {
        const BatchPlanInst& p = P[(size_t)j];
        double* field = p.f_off >= 0 ? d_f + p.f_off : static_cast<double*>(u[j]);
        if (p.stencil == SWEPT_KS_F64)
            ik[(size_t)j] = BatchInst<KSF64>{field, p.n_ring, p.L, p.x_off, p.e_off, p.tiles, 0,
                                            ks_consts(params + 2 * j)};
        else
            ih[(size_t)j] = BatchInst<HeatF64>{field, p.n_ring, p.L, p.x_off, p.e_off, p.tiles, 0,
                                              heat64_consts(params + 2 * j)};
    }
    HIP_TRY(hipStreamSynchronize(g_ctx.stream));
    HIP_TRY(hipMemcpy(d_ih, ih.data(), sizeof(BatchInst<HeatF64>) * (size_t)count, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_ik, ik.data(), sizeof(BatchInst<KSF64>) * (size_t)count, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_x, X.data(), sizeof(int64_t) * X.size(), hipMemcpyHostToDevice));
    if (!th.empty())
        HIP_TRY(hipMemcpy(d_th, th.data(), sizeof(BatchTask) * th.size(), hipMemcpyHostToDevice));
    if (!tk.empty())
        HIP_TRY(hipMemcpy(d_tk, tk.data(), sizeof(BatchTask) * tk.size(), hipMemcpyHostToDevice));

    // ---- the launch sequence (captured once into a graph per batch)
    std::vector<int64_t> key;
    key.push_back(count);
    for (int64_t j = 0; j < count; ++j) {
        key.push_back(nx[j]);
        key.push_back(nsteps[j]);
        key.push_back(ids[j]);
        key.push_back((int64_t)(intptr_t)u[j]);
        int64_t pb[2];
        std::memcpy(pb, params + 2 * j, sizeof pb);
        key.push_back(pb[0]);
        key.push_back(pb[1]);
    }
    key.push_back((int64_t)(intptr_t)g_ctx.scratch);
    key.push_back(g_ctx.tile_w);
    if (g_batch.exec && key == g_batch.key) {
        HIP_TRY(hipGraphLaunch(g_batch.exec, g_ctx.stream));
        return SWEPT_OK;
    }
    batch_release();
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    for (int64_t j = 0; j < count; ++j) {      // odd rings: build the two-fold cover
        const BatchPlanInst& p = P[(size_t)j];
        if (p.f_off >= 0)
            hipLaunchKernelGGL((batch_cover_kernel<HeatF64>), dim3(grid_for(p.n_ring, 256)),
                               dim3(256), 0, cs, static_cast<const double*>(u[j]), d_f + p.f_off,
                               p.n_user, 2);
    }
    size_t ph = 0, pk = 0;
    for (int64_t g = 0; g < smax; ++g) {
        while (ph < sh.size() && sh[ph] > g) ++ph;
        while (pk < sk.size() && sk[pk] > g) ++pk;
        launch_batch_stage<HeatF64>(d_ih, d_th, d_x, d_eh, d_eh + e_heat, d_eh + 2 * e_heat,
                                    (int)g, (int64_t)ph, kmax_h, cs);
        launch_batch_stage<KSF64>(d_ik, d_tk, d_x, d_ek, d_ek + e_ks, d_ek + 2 * e_ks, (int)g,
                                  (int64_t)pk, kmax_k, cs);
    }
    for (int64_t j = 0; j < count; ++j) {      // odd rings: copy one period back
        const BatchPlanInst& p = P[(size_t)j];
        if (p.f_off >= 0)
            hipLaunchKernelGGL((batch_cover_kernel<HeatF64>), dim3(grid_for(p.n_user, 256)),
                               dim3(256), 0, cs, d_f + p.f_off, static_cast<double*>(u[j]),
                               p.n_user, 1);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess)
        return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    g_batch.key = std::move(key);
    g_batch.graph = graph;
    g_batch.exec = exec;
    HIP_TRY(hipGraphLaunch(exec, g_ctx.stream));
    return SWEPT_OK;
}

// ------------------------------------------------------------- naive launch

template <class S>
int run_naive_single(void* u, int64_t nx, int64_t nsteps, const typename S::Consts& c)
{
    using T = typename S::T;
    int rc = ensure_scratch((size_t)nx * sizeof(T));
    if (rc)
        return rc;
    T* a = static_cast<T*>(u);
    T* b = static_cast<T*>(g_ctx.scratch);
    const unsigned grid = grid_for(nx, 256);
    for (int64_t s = 0; s < nsteps; ++s) {
        hipLaunchKernelGGL((naive_step_kernel<S>), dim3(grid), dim3(256), 0, g_ctx.stream, a, b,
                           nx, c);
        std::swap(a, b);
    }
    if (a != u)
        HIP_TRY(hipMemcpyAsync(u, a, (size_t)nx * sizeof(T), hipMemcpyDeviceToDevice,
                               g_ctx.stream));
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

int run_naive_ks_fused(void* u, int64_t nx, int64_t nsteps, const KSF64::Consts& c)
{
    int rc = ensure_scratch((size_t)nx * sizeof(double));
    if (rc)
        return rc;
    double* a = static_cast<double*>(u);
    double* b = static_cast<double*>(g_ctx.scratch);
    constexpr int NB = 256;
    const unsigned grid = (unsigned)((nx + NB - 1) / NB);
    for (int64_t s = 0; s < nsteps; ++s) {
        hipLaunchKernelGGL((naive_fused_kernel<KSF64, NB>), dim3(grid), dim3(NB), 0,
                           g_ctx.stream, a, b, nx, c);
        std::swap(a, b);
    }
    if (a != u)
        HIP_TRY(hipMemcpyAsync(u, a, (size_t)nx * sizeof(double), hipMemcpyDeviceToDevice,
                               g_ctx.stream));
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

int run_naive_ks_substep(void* u, int64_t nx, int64_t nsteps, const KSF64::Consts& c)
{
    using Pt = KSF64::Pt;
    int rc = ensure_scratch(2 * (size_t)nx * sizeof(Pt));
    if (rc)
        return rc;
    Pt* a = static_cast<Pt*>(g_ctx.scratch);
    Pt* b = a + nx;
    const unsigned grid = grid_for(nx, 256);
    double* uf = static_cast<double*>(u);
    hipLaunchKernelGGL((field_to_pt_kernel<KSF64>), dim3(grid), dim3(256), 0, g_ctx.stream, uf,
                       a, nx);
    for (int64_t s = 0; s < nsteps; ++s) {
        hipLaunchKernelGGL((naive_substep_kernel<KSF64, 0>), dim3(grid), dim3(256), 0,
                           g_ctx.stream, a, b, nx, c);
        hipLaunchKernelGGL((naive_substep_kernel<KSF64, 1>), dim3(grid), dim3(256), 0,
                           g_ctx.stream, b, a, nx, c);
        hipLaunchKernelGGL((naive_substep_kernel<KSF64, 2>), dim3(grid), dim3(256), 0,
                           g_ctx.stream, a, b, nx, c);
        hipLaunchKernelGGL((naive_substep_kernel<KSF64, 3>), dim3(grid), dim3(256), 0,
                           g_ctx.stream, b, a, nx, c);
    }
    hipLaunchKernelGGL((pt_to_field_kernel<KSF64>), dim3(grid), dim3(256), 0, g_ctx.stream, a,
                       uf, nx);
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

int naive_dispatch(void* u, int64_t nx, int64_t nsteps, int32_t id, const double* params)
{
    switch (id) {
    case SWEPT_HEAT_F64: return run_naive_single<HeatF64>(u, nx, nsteps, heat64_consts(params));
    case SWEPT_HEAT_F32: return run_naive_single<HeatF32>(u, nx, nsteps, heat32_consts(params));
    default: return run_naive_ks_fused(u, nx, nsteps, ks_consts(params));
    }
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

int swept_init(int device)
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(SWEPT_EINVAL, "device %d out of range [0, %d)", device, count);
    if (g_ctx.ready && g_ctx.device != device)
        swept_finalize();
    HIP_TRY(hipSetDevice(device));
    g_ctx.ready = true;
    g_ctx.device = device;
    g_ctx.stream = nullptr;
    g_err.clear();
    return SWEPT_OK;
}

int swept_set_stream(void* hip_stream)
{
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    g_ctx.stream = static_cast<hipStream_t>(hip_stream);
    return SWEPT_OK;
}

int swept_set_tuning(int32_t tile_w, int32_t pairs_per_lane, int32_t mode)
{
    if (tile_w < 0 || (tile_w != 0 && (tile_w % 2 != 0 || tile_w < 2)))
        return fail(SWEPT_EINVAL, "tile width %d must be 0 or even and >= 2", tile_w);
    if (pairs_per_lane != 0 && pairs_per_lane != 1 && pairs_per_lane != 2 && pairs_per_lane != 4 &&
        pairs_per_lane != 8)
        return fail(SWEPT_EINVAL, "pairs per lane %d not in {0,1,2,4,8}", pairs_per_lane);
    if (mode != SWEPT_MODE_AUTO && mode != SWEPT_MODE_STAGE && mode != SWEPT_MODE_NAIVE &&
        mode != SWEPT_MODE_STAGE_BANDED)
        return fail(SWEPT_EINVAL, "unknown mode %d", mode);
    g_ctx.tile_w = tile_w;
    g_ctx.ppl = pairs_per_lane;
    g_ctx.mode = mode;
    return SWEPT_OK;
}

int swept_plan(int64_t nx, int64_t nsteps, int32_t stencil_id, int64_t* out)
{
    if (!out || nx < 3 || nsteps < 0 ||
        (stencil_id != SWEPT_HEAT_F64 && stencil_id != SWEPT_HEAT_F32 &&
         stencil_id != SWEPT_KS_F64))
        return fail(SWEPT_EINVAL, "invalid plan request");
    Plan p;
    int rc = make_plan(nx, nsteps, stencil_id, &p);
    if (rc)
        return rc;
    out[0] = p.W;
    out[1] = p.k;
    out[2] = p.tiles;
    out[3] = p.stages;
    out[4] = p.P;
    out[5] = p.mode;
    return SWEPT_OK;
}

int swept_advance(void* u, int64_t nx, int64_t nsteps, int32_t stencil_id, const double* params,
                  int32_t nparams)
{
    int rc = check_common(u, nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    if (nsteps == 0)
        return SWEPT_OK;
    Plan p;
    rc = make_plan(nx, nsteps, stencil_id, &p);
    if (rc)
        return rc;
    if (p.mode == SWEPT_MODE_NAIVE)
        return naive_dispatch(u, nx, nsteps, stencil_id, params);
    const int64_t L = nsteps * substeps_of(stencil_id);
    switch (stencil_id) {
    case SWEPT_HEAT_F64: return run_swept<HeatF64>(u, nx, L, heat64_consts(params), p);
    case SWEPT_HEAT_F32: return run_swept<HeatF32>(u, nx, L, heat32_consts(params), p);
    default: return run_swept<KSF64>(u, nx, L, ks_consts(params), p);
    }
}

int swept_naive_advance(void* u, int64_t nx, int64_t nsteps, int32_t stencil_id,
                        const double* params, int32_t nparams)
{
    int rc = check_common(u, nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    if (nsteps == 0)
        return SWEPT_OK;
    return naive_dispatch(u, nx, nsteps, stencil_id, params);
}

int swept_naive_substep_advance(void* u, int64_t nx, int64_t nsteps, int32_t stencil_id,
                                const double* params, int32_t nparams)
{
    int rc = check_common(u, nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    if (stencil_id != SWEPT_KS_F64)
        return fail(SWEPT_EINVAL, "per-sub-timestep launches exist for the KS stencil only");
    if (nsteps == 0)
        return SWEPT_OK;
    return run_naive_ks_substep(u, nx, nsteps, ks_consts(params));
}

int swept_advance_batch(void* const* u, const int64_t* nx, const int64_t* nsteps,
                        const int32_t* stencil_id, const double* params, int64_t count)
{
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    if (count < 0 || (count > 0 && (!u || !nx || !nsteps || !stencil_id || !params)))
        return fail(SWEPT_EINVAL, "bad batch arrays");
    for (int64_t j = 0; j < count; ++j) {
        int rc = check_common(u[j], nx[j], nsteps[j], stencil_id[j], params + 2 * j, 2);
        if (rc)
            return fail(rc, "instance %lld: %s", (long long)j, g_err.c_str());
        if (stencil_id[j] != SWEPT_HEAT_F64 && stencil_id[j] != SWEPT_KS_F64)
            return fail(SWEPT_EUNSUPPORTED, "instance %lld: the batch takes binary64 stencils",
                        (long long)j);
    }
    if (count == 0)
        return SWEPT_OK;
    int rc = run_batch(u, nx, nsteps, stencil_id, params, count);
    if (rc)
        return rc;
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

int swept_set_profiling(int enable)
{
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    g_ctx.profiling = enable != 0;
    g_ctx.recorded = 0;
    return SWEPT_OK;
}

int swept_stage_times(double* ms_out, int32_t* kind_out, int64_t cap, int64_t* count)
{
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    if (!g_ctx.profiling || g_ctx.recorded == 0)
        return fail(SWEPT_EINVAL, "no profiled swept run recorded");
    if (cap < 0)
        return fail(SWEPT_EINVAL, "negative capacity");
    const int64_t n = g_ctx.recorded;
    HIP_TRY(hipEventSynchronize(g_ctx.events[(size_t)n]));
    for (int64_t i = 0; i < n && i < cap; ++i) {
        if (ms_out) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, g_ctx.events[(size_t)i], g_ctx.events[(size_t)i + 1]));
            ms_out[i] = ms;
        }
        if (kind_out)
            kind_out[i] = g_ctx.kinds[(size_t)i];
    }
    if (count)
        *count = n;
    return SWEPT_OK;
}

int swept_adjoint(const void* u0, void* grad_u0, int64_t nx, int64_t nsteps, int32_t stencil_id,
                  const double* params, int32_t nparams, int64_t window_first,
                  double window_weight, const void* cot_final)
{
    int rc = check_common(u0, nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    if (!grad_u0)
        return fail(SWEPT_EINVAL, "grad_u0 is NULL");
    if (!std::isfinite(window_weight))
        return fail(SWEPT_EINVAL, "window weight is not finite");
    switch (stencil_id) {
    case SWEPT_HEAT_F64:
        return run_adjoint<HeatF64>(u0, grad_u0, nx, nsteps, params, heat64_consts(params),
                                    window_first, window_weight, cot_final);
    case SWEPT_KS_F64:
        return run_adjoint<KSF64>(u0, grad_u0, nx, nsteps, params, ks_consts(params), window_first,
                                  window_weight, cot_final);
    default:
        return fail(SWEPT_EUNSUPPORTED, "the adjoint exists for the binary64 stencils only");
    }
}

int swept_sync(void)
{
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    HIP_TRY(hipStreamSynchronize(g_ctx.stream));
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

const char* swept_last_error(void) { return g_err.c_str(); }

void swept_finalize(void)
{
    if (g_ctx.ready)
        (void)hipDeviceSynchronize();
    if (g_ctx.scratch)
        (void)hipFree(g_ctx.scratch);
    release_events();
    batch_release();
    g_ctx = Context{};
}

}  // extern "C"
