// swept.hip -- host runtime and C ABI of libswept.so (declared in swept.h).
//
// Planning, scratch management, stream handling and the launch sequences of
// the swept and naive schedules.  All arithmetic runs in the kernels of
// kernels.hpp; this file only validates, plans and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "swept.h"
#include "swept_debug.h"
#include "kernels.hpp"

// Scratch of swept_advance_noalloc: a fixed array that every GPU the library
// runs on holds until the process ends.  Host code never uses its name as an
// address (in host code the name is only a stand-in); it uses the per-device
// address from hipGetSymbolAddress, taken in swept_init.
static __device__ __align__(256) unsigned char scratch[SWEPT_NOALLOC_SCRATCH_BYTES];

namespace {

using namespace swept;

struct Context {
    bool ready = false;
    int device = -1;
    hipStream_t stream = nullptr;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    void* obj = nullptr;              // swept_window_objective: field copy and sums
    size_t obj_bytes = 0;
    int tile_w = 0;   // 0 = automatic
    int ppl = 0;      // pairs per lane, 0 = automatic
    int mode = SWEPT_MODE_AUTO;
    bool profiling = false;
    std::vector<hipEvent_t> events;   // events[i] before stage i, events[i+1] after it
    std::vector<int32_t> kinds;       // kernel used by each recorded stage
    int64_t recorded = 0;             // stages recorded by the last swept run
    int* fault = nullptr;             // persistent batch: set by a wait that gave up
    bool fault_unread = false;        // a persistent batch ran since swept_sync last looked
    int heat_form = SWEPT_FORM_AUTO;  // swept_set_heat_form
    int last_form = 0;                // last heat call: SWEPT_FORM_* (0: none yet)
    unsigned long long last_guard = 0;  // its range check's call id (0: none)
    bool last_batch = false;          // the last heat call was a batch (its flag: g_batch_form_bad)
};

Context g_ctx;
thread_local std::string g_err;

// Device address of `scratch` on each device swept_init has selected.
std::map<int, void*> g_noalloc_ptr;
// While swept_advance_noalloc runs: the fixed array stands in for the
// library's growing scratch (nullptr otherwise).
void* g_fixed = nullptr;

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
    if (g_fixed) {
        if (bytes > (size_t)SWEPT_NOALLOC_SCRATCH_BYTES)
            return fail(SWEPT_EINVAL,
                        "swept_advance_noalloc: this call needs %zu bytes of scratch, the fixed "
                        "array holds %zu (SWEPT_NOALLOC_SCRATCH_BYTES)",
                        bytes, (size_t)SWEPT_NOALLOC_SCRATCH_BYTES);
        return SWEPT_OK;
    }
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

// The scratch the current call works in: the fixed array during
// swept_advance_noalloc, else the library's allocation.
void* scratch_base() { return g_fixed ? g_fixed : g_ctx.scratch; }

// ------------------------------------------------------------------ stencils

// the canonical stencil an id shares its point layout and sizes with (the
// contraction-on ids differ from theirs only in rounding)
int base_id(int id)
{
    switch (id) {
    case SWEPT_HEAT_F64_FMA: return SWEPT_HEAT_F64;
    case SWEPT_HEAT_F32_FMA: return SWEPT_HEAT_F32;
    case SWEPT_KS_F64_FMA: return SWEPT_KS_F64;
    default: return id;
    }
}

bool known_id(int id) { return id >= SWEPT_HEAT_F64 && id <= SWEPT_KS_F64_FMA; }

int substeps_of(int id)
{
    const int b = base_id(id);
    return (b == SWEPT_KS_F64 || b == SWEPT_EULER_F64) ? 4 : 1;
}

size_t pt_bytes(int id)
{
    switch (base_id(id)) {
    case SWEPT_HEAT_F64: return sizeof(HeatF64::Pt);
    case SWEPT_HEAT_F32: return sizeof(HeatF32::Pt);
    case SWEPT_EULER_F64: return sizeof(EulerF64::Pt);
    default: return sizeof(KSF64::Pt);
    }
}

int check_problem(int64_t nx, int64_t nsteps, int32_t id, const double* params, int32_t nparams)
{
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    if (nx < 3)
        return fail(SWEPT_EINVAL, "nx = %lld: need at least 3 points", (long long)nx);
    if (nsteps < 0)
        return fail(SWEPT_EINVAL, "nsteps = %lld is negative", (long long)nsteps);
    if (!known_id(id))
        return fail(SWEPT_EINVAL, "unknown stencil id %d", id);
    const int bid = base_id(id);
    const int need = bid == SWEPT_EULER_F64 ? 3 : (bid == SWEPT_KS_F64 ? 2 : 1);
    if (!params || nparams < need)
        return fail(SWEPT_EINVAL, "stencil %d needs %d parameter(s)", id, need);
    for (int i = 0; i < need; ++i)
        if (!std::isfinite(params[i]))
            return fail(SWEPT_EINVAL, "parameter %d is not finite", i);
    if ((bid == SWEPT_KS_F64 || bid == SWEPT_EULER_F64) && !(params[1] > 0.0))
        return fail(SWEPT_EINVAL, "stencil %d needs dx > 0", id);
    if (id == SWEPT_EULER_F64 && !(params[2] > 1.0))
        return fail(SWEPT_EINVAL, "Euler needs gamma > 1");
    return SWEPT_OK;
}

int check_common(const void* u, int64_t nx, int64_t nsteps, int32_t id, const double* params,
                 int32_t nparams)
{
    if (g_ctx.ready && !u)
        return fail(SWEPT_EINVAL, "u is NULL");
    return check_problem(nx, nsteps, id, params, nparams);
}

HeatF64::Consts heat64_consts(const double* p) { return HeatF64::Consts{p[0]}; }
HeatF32::Consts heat32_consts(const double* p) { return HeatF32::Consts{(float)p[0]}; }
EulerF64::Consts euler_consts(const double* p)
{
    const double dt = p[0], dx = p[1], gamma = p[2];
    return EulerF64::Consts{gamma - 1.0, (0.5 * dt) / dx, dt / dx};
}
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
    int64_t ring = 0;   // SWEPT_MODE_STAGE_RAGGED: the tiled ring (nx, or 2nx for odd nx)
};

constexpr size_t kMaxLds = 64 * 1024;
// the lane-frame kernel holds a region and its V edges in one wavefront
constexpr int64_t kLaneMaxK = 32;
// the unequal tiling is used automatically from this depth up (shallower
// regions would hardly beat one launch per step)
constexpr int64_t kRaggedMinK = 4;

// Measured on MI355X (20,000-step heat at N = 2^24, binary64 and binary32;
// KS at N = 2^20; heat at N = 4096): W = 1024 is fastest for every stencil on
// large grids (a 2k-entry LDS edge chain small enough for ~10 workgroups per
// CU); small grids keep at least 16 tiles so that more CUs take part.
int64_t target_tile(int /*id*/) { return 1024; }

// Pairs per lane a stencil's point fits in registers with: heat 8; KS
// (three values a point) 4; Euler (nine values a point) 2.
template <class S>
constexpr int pmax_of()
{
    return S::NPHASE == 1 ? 8 : (sizeof(typename S::Pt) <= 3 * sizeof(double) ? 4 : 2);
}

int pmax(int id)
{
    switch (base_id(id)) {
    case SWEPT_KS_F64: return pmax_of<KSF64>();
    case SWEPT_EULER_F64: return pmax_of<EulerF64>();
    default: return 8;
    }
}

int auto_ppl(int id, int64_t k)
{
    return std::min(pmax(id) == 2 ? 1 : 4, k >= 512 ? 4 : (k >= 128 ? 2 : 1));
}

// LDS of the stage kernels: the 2k-point edge chain (with one more entry on
// the continuous kernel of a stencil that prefetches it, see
// cont_chain_points) and, on the continuous kernel of a stencil that shares
// face fluxes (Euler), the face chain (k/2 faces).  LDS sets how many
// workgroups share a CU: Euler at W = 256 takes 19,968 bytes, eight per CU.
size_t stage_lds_bytes(int id, int64_t W)
{
    const bool euler = base_id(id) == SWEPT_EULER_F64;
    const size_t face = euler ? sizeof(EulerF64::Face) : 0;
    return (size_t)(W + (euler ? 0 : 2)) * pt_bytes(id) + (size_t)(W / 4) * face;
}

template <class S>
size_t stage_lds(int64_t W, bool cont)
{
    size_t bytes = (size_t)(cont ? cont_chain_points<S>(W / 2) : W) * sizeof(typename S::Pt);
    if constexpr (has_faces<S>::value)
        if (cont)
            bytes += (size_t)(W / 4) * sizeof(typename S::Face);
    return bytes;
}

bool tile_fits(int id, int64_t nx, int64_t W)
{
    return W >= 2 && W % 2 == 0 && nx % W == 0 && stage_lds_bytes(id, W) <= kMaxLds;
}

// the lane-frame kernel: k <= 32 and the rows from the middle level up
// (k^2 + 3k + 3 points) in LDS
size_t lane_lds_bytes(int id, int64_t k)
{
    return (size_t)(k * k + 3 * k + 3) * pt_bytes(id);
}

bool lane_fits(int id, int64_t k)
{
    return k >= 1 && k <= kLaneMaxK && lane_lds_bytes(id, k) <= kMaxLds;
}

// Tilings chosen by swept_autotune, per stencil and size class floor(log2 nx).
struct Tuned {
    int64_t W;
    int P;                 // pairs per lane; 0: the lane-frame kernel
    bool ragged = false;   // the unequal tiling of depth W/2 (SWEPT_MODE_STAGE_RAGGED)
};
std::map<std::pair<int, int>, Tuned> g_tuned;
// Batch depth per stencil id chosen by swept_autotune_batch (0 = default).
int64_t g_batch_want[3] = {0, 0, 0};
constexpr int64_t kBatchWantDefault = 256;
// swept_set_batch_schedule
int g_batch_sched = SWEPT_BATCH_PERSISTENT;
int64_t g_spin_limit = 0;               // microseconds; 0: kSpinDefault
constexpr int64_t kSpinDefault = 60 * 1000 * 1000;
// task numbers a workgroup of the persistent batch takes per claim
constexpr int kChunkDefault = 2;
int g_chunk = 0;                        // 0: kChunkDefault
// independent queues of the persistent batch per stencil
constexpr int kQueuesDefault = 32;
int g_queues = 0;                       // 0: kQueuesDefault
// the persistent batch runs only when its most loaded queue carries at most
// this multiple of the mean work (else one launch per stage)
constexpr double kQueueImbalance = 1.25;

std::pair<int, int> tune_key(int id, int64_t nx)
{
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= nx)
        ++b;
    return {id, b};
}

// The unequal tiling of swept_advance (SWEPT_MODE_STAGE_RAGGED), that of
// one batch instance: a ring of 2h points (h = nx/2 for even nx; odd nx runs
// on its two-fold cover, h = nx) in T = ceil(h/k) tiles, T-1 of 2k points and
// the last of the remainder.  Regions between two full tiles are k x k
// squares (on the continuous-band schedule below the target level when k is
// a multiple of the band 64P), the others rectangles on the banded one.
int ragged_plan(int64_t nx, int64_t L, int32_t id, int64_t want_k, int want_P, Plan* p)
{
    *p = Plan{};
    const int64_t ring = nx % 2 == 0 ? nx : 2 * nx;
    const int64_t h = ring / 2;
    int64_t k = std::max<int64_t>(1, std::min(want_k > 0 ? want_k : target_tile(id) / 2, h));
    while (k > 1 && stage_lds_bytes(id, 2 * k) > kMaxLds)
        --k;
    int P = want_P > 0 ? want_P : (g_ctx.ppl > 0 ? g_ctx.ppl : auto_ppl(id, k));
    if (P > pmax(id))
        return fail(SWEPT_EUNSUPPORTED, "this stencil takes at most %d pairs per lane", pmax(id));
    if (k >= 2 * 64 * P && want_k <= 0)
        k -= k % (64 * P);   // full squares a multiple of the band
    const int64_t T = (h + k - 1) / k;
    const int64_t rem = h - (T - 1) * k;
    p->W = 2 * k;
    p->k = k;
    p->tiles = T;
    p->P = P;
    p->ring = ring;
    // stage s >= 1 of tile t starts at level (X_{t+s} - X_{t+1})/2, the sum of
    // s-1 consecutive half-widths, which hold the short tile at most
    // ceil((s-1)/T) times; a tile's regions end once that level reaches L
    p->stages = L == 0 ? 0 : 2 + (L + k - rem) * T / h;
    p->mode = SWEPT_MODE_STAGE_RAGGED;
    return SWEPT_OK;
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
    int tunedP = 0;
    bool lane = g_ctx.mode == SWEPT_MODE_STAGE_LANE;
    if (g_ctx.tile_w == 0 && g_ctx.ppl == 0 && g_ctx.mode == SWEPT_MODE_AUTO) {
        const auto it = g_tuned.find(tune_key(id, nx));
        if (it != g_tuned.end() && it->second.W < 0) {
            p->mode = SWEPT_MODE_NAIVE;   // the naive schedule was fastest
            return SWEPT_OK;
        }
        if (it != g_tuned.end() && it->second.ragged)
            return ragged_plan(nx, L, id, it->second.W / 2, it->second.P, p);
        if (it != g_tuned.end() && tile_fits(id, nx, it->second.W) &&
            (it->second.P > 0 || lane_fits(id, it->second.W / 2))) {
            W = it->second.W;
            tunedP = it->second.P;
            lane = it->second.P == 0;
        }
    }
    if (g_ctx.mode == SWEPT_MODE_STAGE_RAGGED)
        return ragged_plan(nx, L, id, g_ctx.tile_w / 2, 0, p);
    if (W > 0) {
        // tuned for this stencil and size class
    } else if (g_ctx.tile_w > 0) {
        if (!tile_fits(id, nx, g_ctx.tile_w))
            return fail(SWEPT_EINVAL,
                        "tile width %d must be even, divide nx = %lld and fit 64 KB of LDS",
                        g_ctx.tile_w, (long long)nx);
        if (lane && !lane_fits(id, g_ctx.tile_w / 2))
            return fail(SWEPT_EINVAL,
                        "the lane-frame kernel takes tiles of at most %d points whose upper "
                        "half fits 64 KB of LDS", (int)(2 * kLaneMaxK));
        W = g_ctx.tile_w;
    } else {
        const int64_t cap = lane ? std::min<int64_t>(2 * kLaneMaxK, nx)
                                 : std::min(target_tile(id), std::max<int64_t>(2, nx / 16));
        for (int64_t w = cap - (cap & 1); w >= 2; w -= 2)
            if (tile_fits(id, nx, w) && (!lane || lane_fits(id, w / 2))) {
                W = w;
                break;
            }
        // One tiling rule for every nx: when no even width within a factor
        // of two of the target divides nx (odd nx, or an awkward even one),
        // tile the ring unequally at the target depth instead.
        if (!lane && g_ctx.mode == SWEPT_MODE_AUTO && 2 * W < cap && cap / 2 >= kRaggedMinK)
            return ragged_plan(nx, L, id, cap / 2, 0, p);
    }
    if (W == 0) {
        if (g_ctx.mode == SWEPT_MODE_STAGE || g_ctx.mode == SWEPT_MODE_STAGE_BANDED || lane)
            return fail(SWEPT_EUNSUPPORTED, "nx = %lld has no even tile width", (long long)nx);
        p->mode = SWEPT_MODE_NAIVE;
        return SWEPT_OK;
    }
    p->W = W;
    p->k = W / 2;
    p->tiles = nx / W;
    p->stages = L == 0 ? 0 : 1 + (L + p->k - 1) / p->k;
    // pairs per lane: 0 on the lane-frame kernel (one point per lane)
    p->P = lane ? 0 : (g_ctx.ppl > 0 ? g_ctx.ppl : (tunedP > 0 ? tunedP : auto_ppl(id, p->k)));
    p->mode = lane ? SWEPT_MODE_STAGE_LANE : SWEPT_MODE_STAGE;
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
// The continuous kernel writes no field value, so it takes only the stages
// whose diamond lies strictly below the target level (its apex, level
// b + 2k - 1, below L); a stage whose apex reaches L goes to the banded
// kernel, which writes the points that reach L.
bool use_continuous(const Plan& p, int64_t s, int64_t L)
{
    const int64_t b = (s - 1) * p.k;
    return g_ctx.mode != SWEPT_MODE_STAGE_BANDED && s > 0 && b + 2 * p.k - 1 < L &&
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

// LDS of the lane-frame kernel: the full points of the rows from the middle
// level up (k^2 + 3k + 2, and one spare)
template <class S>
size_t lane_lds(int64_t k)
{
    return (size_t)(k * k + 3 * k + 3) * sizeof(typename S::Pt);
}

unsigned grid_for(int64_t n, int block);

// Call ids of the range check; the device marks only ever rise to them.
std::atomic<unsigned long long> g_call_id{0};
// Longest run (in levels) the fused form's bound covers with room to spare
// (the argument at HeatLap: about 2e15 in binary64, 4e6 in binary32).
template <class T>
constexpr int64_t kFusedMaxLevels = sizeof(T) == 8 ? 1000000000000000LL : 1000000LL;

// The fused heat form's preconditions: the host checks r and the run length
// and, if they hold, enqueues the check of the initial field (heat_range_kernel),
// whose result the stage kernels read on the device.  Returns the call id
// for the stage kernels (0: the canonical form).  Stencils without a fused
// form return 0 and leave the record of the last heat call alone.
template <class S>
unsigned long long range_check(const void* u, int64_t n, const typename S::Consts& c, int64_t L)
{
    if constexpr (!has_fused_form<S>) {
        return 0;
    } else {
        using T = typename S::T;
        g_ctx.last_guard = 0;
        g_ctx.last_batch = false;
        g_ctx.last_form = SWEPT_FORM_CANONICAL;
        if (g_ctx.heat_form == SWEPT_FORM_CANONICAL || !(c.r >= 0 && c.r <= 0.5) ||
            L > kFusedMaxLevels<T>)
            return 0;
        const unsigned long long id = ++g_call_id;
        hipLaunchKernelGGL(heat_range_kernel<T>, dim3(grid_for(n, 256)), dim3(256), 0,
                           g_ctx.stream, static_cast<const T*>(u), n,
                           std::numeric_limits<T>::max() / 16, id);
        g_ctx.last_guard = id;
        g_ctx.last_form = SWEPT_FORM_FUSED;   // until the mark says otherwise
        return id;
    }
}

template <class S>
int run_swept(void* u, int64_t nx, int64_t L, const typename S::Consts& c, const Plan& p)
{
    using Pt = typename S::Pt;
    const size_t edge = (size_t)nx * sizeof(Pt);  // tiles * k * 2 points
    int rc = ensure_scratch(3 * edge);
    if (rc)
        return rc;
    Pt* re = static_cast<Pt*>(scratch_base());
    Pt* le[2] = {re + nx, re + 2 * nx};
    const size_t lds_band = stage_lds<S>(p.W, false), lds_cont = stage_lds<S>(p.W, true);

    StageArgs<S> a{};
    a.u = static_cast<typename S::T*>(u);
    a.re = re;
    a.re_out = re;
    a.n = nx;
    a.L = L;
    a.k = (int)p.k;
    a.tiles = (int)p.tiles;
    a.c = c;
    a.guard = range_check<S>(u, nx, c, L);
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
        if (p.mode == SWEPT_MODE_STAGE_LANE) {
            hipLaunchKernelGGL((swept_lane_kernel<S, true>), dim3((unsigned)p.tiles), dim3(64),
                               lane_lds<S>(p.k), g_ctx.stream, a);
            if (g_ctx.profiling) {
                g_ctx.kinds[(size_t)s] = 2;
                HIP_TRY(hipEventRecord(g_ctx.events[(size_t)s + 1], g_ctx.stream));
            }
            continue;
        }
        const bool cont = use_continuous(p, s, L);
        const size_t lds = cont ? lds_cont : lds_band;
        // pairs per lane beyond the register budget of a point are not built
        constexpr int PMAX = pmax_of<S>();
        switch (p.P) {
        case 1: launch_stage<S, 1>(a, lds, g_ctx.stream, (int)p.tiles, cont); break;
        case 2: launch_stage<S, 2>(a, lds, g_ctx.stream, (int)p.tiles, cont); break;
        case 4:
            if constexpr (PMAX >= 4)
                launch_stage<S, 4>(a, lds, g_ctx.stream, (int)p.tiles, cont);
            else
                return fail(SWEPT_EUNSUPPORTED, "this stencil takes at most %d pairs per lane",
                            PMAX);
            break;
        case 8:
            if constexpr (PMAX >= 8)
                launch_stage<S, 8>(a, lds, g_ctx.stream, (int)p.tiles, cont);
            else
                return fail(SWEPT_EUNSUPPORTED, "this stencil takes at most %d pairs per lane",
                            PMAX);
            break;
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

unsigned grid_for(int64_t n, int block);

template <class S, int P>
void launch_ragged(const RaggedArgs<S>& a, size_t lds, hipStream_t st, int tiles)
{
    hipLaunchKernelGGL((swept_ragged_kernel<S, P>), dim3(tiles), dim3(64), lds, st, a);
}

// The unequal tiling of one field (ragged_plan): the stages of its T tiles,
// one launch each, on the field itself or, for odd nx, on its two-fold cover
// in the scratch (the scheme commutes with the translation by nx, so the
// cover stays nx-periodic and its first nx points are the field's result).
template <class S>
int run_ragged(void* u, int64_t nx, int64_t L, const typename S::Consts& c, const Plan& p)
{
    using Pt = typename S::Pt;
    using T = typename S::T;
    const int64_t ring = p.ring;
    const bool cover = ring != nx;
    const size_t cov_b = cover ? ((size_t)ring * sizeof(T) + 255) / 256 * 256 : 0;
    const size_t edge = (size_t)ring * sizeof(Pt);
    int rc = ensure_scratch(cov_b + 3 * edge);
    if (rc)
        return rc;
    unsigned char* base = static_cast<unsigned char*>(scratch_base());
    T* field = cover ? reinterpret_cast<T*>(base) : static_cast<T*>(u);
    Pt* re = reinterpret_cast<Pt*>(base + cov_b);
    if (cover)
        hipLaunchKernelGGL((batch_cover_kernel<S>), dim3(grid_for(ring, 256)), dim3(256), 0,
                           g_ctx.stream, static_cast<const T*>(u), field, nx, 2);
    RaggedArgs<S> a{};
    a.guard = range_check<S>(u, nx, c, L);
    a.u = field;
    a.re = re;
    a.le[0] = re + ring;
    a.le[1] = re + 2 * ring;
    a.n = ring;
    a.L = L;
    a.k = (int)p.k;
    a.tiles = (int)p.tiles;
    a.c = c;
    const size_t lds = stage_lds<S>(2 * p.k, true);
    if (g_ctx.profiling) {
        rc = reserve_events(p.stages);
        if (rc)
            return rc;
        HIP_TRY(hipEventRecord(g_ctx.events[0], g_ctx.stream));
    }
    constexpr int PMAX = pmax_of<S>();
    for (int64_t st = 0; st < p.stages; ++st) {
        a.stage = (int)st;
        switch (p.P) {
        case 1: launch_ragged<S, 1>(a, lds, g_ctx.stream, (int)p.tiles); break;
        case 2: launch_ragged<S, 2>(a, lds, g_ctx.stream, (int)p.tiles); break;
        case 4:
            if constexpr (PMAX >= 4)
                launch_ragged<S, 4>(a, lds, g_ctx.stream, (int)p.tiles);
            else
                return fail(SWEPT_EUNSUPPORTED, "this stencil takes at most %d pairs per lane",
                            PMAX);
            break;
        default: return fail(SWEPT_EUNSUPPORTED, "the unequal tiling takes 1, 2 or 4 pairs per lane");
        }
        if (g_ctx.profiling) {
            g_ctx.kinds[(size_t)st] = 3;
            HIP_TRY(hipEventRecord(g_ctx.events[(size_t)st + 1], g_ctx.stream));
        }
    }
    if (cover)
        hipLaunchKernelGGL((batch_cover_kernel<S>), dim3(grid_for(nx, 256)), dim3(256), 0,
                           g_ctx.stream, static_cast<const T*>(field), static_cast<T*>(u), nx, 1);
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

// Tile for the adjoint: one wavefront per region, whose lanes are the
// columns of the region and its V edges (the two outermost ones excepted at
// k = 32).  LDS of the reverse kernel: one kept forward value per point of
// the region's layout (2k^2 + 6k + 2, and one spare); of the checkpoint
// kernel: the full points of the rows from the middle level up (k^2 + 3k + 2,
// and one spare).
template <class S>
size_t adjoint_lds(int64_t k)
{
    return (size_t)(2 * k * k + 6 * k + 3) * sizeof(typename S::Kept);
}

// Depth: the largest k <= want (32 by default: a stage costs a launch and
// its edge traffic plus a chain of about 4k dependent levels, so deeper
// stages are cheaper per level up to the lane frame's k <= 32) dividing nx/2,
// with both kernels' LDS in budget.
template <class S>
int64_t adjoint_depth(int64_t nx, int64_t want)
{
    for (int64_t k = std::min<int64_t>(32, want > 0 ? want : 32); k >= 1; --k)
        if (nx % (2 * k) == 0 && adjoint_lds<S>(k) <= kMaxLds && lane_lds<S>(k) <= kMaxLds)
            return k;
    return 0;
}

template <class S>
int run_adjoint(const void* u0v, void* gradv, int64_t nx, int64_t nsteps, const double* params,
                const typename S::Consts& c, int64_t win_first, double wgt, const void* cotv)
{
    using Pt = typename S::Pt;
    using Ad = typename S::Ad;
    using Kept = typename S::Kept;
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
    const size_t fh = (size_t)nx * sizeof(Kept);          // tiles * 2 sides * k
    int rc = ensure_scratch(2 * ck + 2 * ae + 2 * fh);
    if (rc)
        return rc;
    unsigned char* base = static_cast<unsigned char*>(g_ctx.scratch);
    Pt* ck_re = reinterpret_cast<Pt*>(base);
    Pt* ck_le = reinterpret_cast<Pt*>(base + ck);
    Ad* aeb[2] = {reinterpret_cast<Ad*>(base + 2 * ck), reinterpret_cast<Ad*>(base + 2 * ck + ae)};
    Kept* fhb[2] = {reinterpret_cast<Kept*>(base + 2 * ck + 2 * ae),
                    reinterpret_cast<Kept*>(base + 2 * ck + 2 * ae + fh)};

    // forward pass, keeping the V edges of every stage (the field is not written)
    StageArgs<S> a{};
    a.u = const_cast<T*>(u0);   // read only, by the triangle
    a.n = nx;
    a.L = L;
    a.k = (int)k;
    a.tiles = (int)tiles;
    a.c = c;
    const size_t lds_ck = lane_lds<S>(k);
    for (int64_t s = 0; s < stages; ++s) {
        a.tri = s == 0;
        a.b = (s - 1) * k;
        a.J0 = (k + s * k) % nx;
        a.re = s > 0 ? ck_re + (s - 1) * nx : ck_re;
        a.re_out = ck_re + s * nx;
        a.le_in = s > 0 ? ck_le + (s - 1) * nx : ck_le;
        a.le_out = ck_le + s * nx;
        hipLaunchKernelGGL((swept_lane_kernel<S, false>), dim3(tiles), dim3(64), lds_ck,
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

// Per-instance tiling for the batch: T = ceil(h/k) tiles, the first T-1 of
// half-width k and the last of the remainder r = h - (T-1)k in [1, k], h the
// half ring length (no tile exceeds the target k, which sets every
// workgroup's LDS, and every region between two full tiles is a k x k square
// that the continuous-band schedule can take).  Odd rings run on their
// two-fold cover (the same bits: the scheme is translation-equivariant, so a
// field repeated twice stays repeated).
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

int64_t batch_want(int id)
{
    return g_batch_want[id] > 0 ? g_batch_want[id] : kBatchWantDefault;
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
                       int64_t ntasks, int kmax, int fusable, hipStream_t st)
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
    a.fusable = fusable;
    const size_t lds = (size_t)cont_chain_points<S>(kmax) * sizeof(typename S::Pt);
    hipLaunchKernelGGL((swept_batch_kernel<S, 2>), dim3((unsigned)ntasks), dim3(64), lds, st, a);
    return SWEPT_OK;
}

// One stencil's persistent launch in a batch (swept_batch_persistent_kernel):
// its instances split into Q queues by a greedy longest-first assignment of
// their work (tiles x stages x k^2) to the least loaded queue; each queue's
// tile list holds its instances in order of decreasing stage count, so
// stage g's tasks are a prefix of it, numbered first[g] .. first[g+1]-1.
struct PersistPlan {
    std::vector<BatchTask> tasks;   // the queues' tile lists, one after another
    std::vector<int64_t> toff;      // Q + 1 offsets into tasks
    std::vector<int64_t> first;     // Q x (smax + 1)
    int64_t max_total = 0;
    double load_max = 0.0, load_mean = 0.0;   // work per queue
};

PersistPlan persist_plan(const std::vector<BatchPlanInst>& P, bool ks, int64_t smax, int Q,
                         std::vector<int>& tpos)
{
    PersistPlan pp;
    std::vector<int64_t> ids;
    auto work = [&](int64_t j) {
        const BatchPlanInst& p = P[(size_t)j];
        return (double)p.tiles * (double)p.stages * (double)p.kmax * (double)p.kmax;
    };
    for (int64_t j = 0; j < (int64_t)P.size(); ++j)
        if ((P[(size_t)j].stencil == SWEPT_KS_F64) == ks && P[(size_t)j].L > 0)
            ids.push_back(j);
    std::stable_sort(ids.begin(), ids.end(), [&](int64_t x, int64_t y) { return work(x) > work(y); });
    std::vector<std::vector<int64_t>> qi((size_t)Q);
    std::vector<double> load((size_t)Q, 0.0);
    for (int64_t j : ids) {
        const size_t q = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
        qi[q].push_back(j);
        load[q] += work(j);
    }
    for (double l : load) {
        pp.load_max = std::max(pp.load_max, l);
        pp.load_mean += l / Q;
    }
    pp.toff.push_back(0);
    pp.first.assign((size_t)Q * (size_t)(smax + 1), 0);
    for (int q = 0; q < Q; ++q) {
        auto& v = qi[(size_t)q];
        std::stable_sort(v.begin(), v.end(), [&](int64_t x, int64_t y) {
            return P[(size_t)x].stages > P[(size_t)y].stages;
        });
        const int64_t base = (int64_t)pp.tasks.size();
        for (int64_t j : v) {
            tpos[(size_t)j] = (int)pp.tasks.size();
            for (int t = 0; t < P[(size_t)j].tiles; ++t)
                pp.tasks.push_back(BatchTask{(int)j, t});
        }
        pp.toff.push_back((int64_t)pp.tasks.size());
        int64_t* f = pp.first.data() + (size_t)q * (size_t)(smax + 1);
        size_t ptr = 0;
        int64_t tiles_in = 0;    // tiles of the instances with more than g stages
        for (int64_t g = 0; g < smax; ++g) {
            while (ptr < v.size() && P[(size_t)v[ptr]].stages > g)
                tiles_in += P[(size_t)v[ptr++]].tiles;
            f[g + 1] = f[g] + tiles_in;
        }
        pp.max_total = std::max(pp.max_total, f[smax]);
        (void)base;
    }
    return pp;
}

// The XCDs of the current device as the persistent batch sees them: m if
// the XCC_ID values of 4096 one-wave workgroups are exactly 0..m-1 (the
// hardware spreads workgroups over all XCDs), else 0 (agent-scope queues).
std::map<int, int> g_xcds;

int probe_xcds(int* m)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto it = g_xcds.find(dev);
    if (it != g_xcds.end()) {
        *m = it->second;
        return SWEPT_OK;
    }
    constexpr int kBlocks = 4096;
    int* d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(int) * kBlocks));
    std::vector<int> h(kBlocks, -1);
    hipLaunchKernelGGL(xcc_probe_kernel, dim3(kBlocks), dim3(64), 0, g_ctx.stream, d);
    hipError_t e = hipMemcpyAsync(h.data(), d, sizeof(int) * kBlocks, hipMemcpyDeviceToHost,
                                  g_ctx.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(g_ctx.stream);
    (void)hipFree(d);
    if (e != hipSuccess)
        return hip_fail(e, "XCD probe");
    int hi = -1;
    bool ok = true;
    std::vector<int> seen(16, 0);
    for (int x : h) {
        ok = ok && x >= 0 && x < 16;
        if (x >= 0 && x < 16) {
            seen[(size_t)x] = 1;
            hi = std::max(hi, x);
        }
    }
    for (int x = 0; x <= hi; ++x)
        ok = ok && seen[(size_t)x];
    *m = ok ? hi + 1 : 0;
    g_xcds[dev] = *m;
    return SWEPT_OK;
}

template <class S>
struct PersistLaunch {
    PersistArgs<S> a{};
    size_t lds = 0;
    unsigned grid = 0;
    int64_t tiles = 0;
    bool xl = false;

    int setup(const PersistPlan& pp, const BatchInst<S>* inst, const BatchTask* tasks,
              const int64_t* toff, const int64_t* first, const int64_t* X,
              typename S::Pt* edges, int64_t ering, int* done, unsigned* counter, int64_t smax,
              int Q, bool xcd_local, int kmax, int64_t spin_limit)
    {
        tiles = (int64_t)pp.tasks.size();
        if (pp.max_total <= 0)
            return SWEPT_OK;
        lds = (size_t)cont_chain_points<S>(kmax) * sizeof(typename S::Pt);
        int per_cu = 0, dev = 0;
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        xl = xcd_local;
        const void* fn = xl ? reinterpret_cast<const void*>(&swept_batch_persistent_kernel<S, 2, true>)
                            : reinterpret_cast<const void*>(&swept_batch_persistent_kernel<S, 2, false>);
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds));
        // workgroup w serves queue w mod Q: at least one per queue
        const int64_t resident = (int64_t)std::max(1, per_cu) * prop.multiProcessorCount;
        grid = (unsigned)std::max<int64_t>(Q, resident / Q * Q);
        a.inst = inst;
        a.tasks = tasks;
        a.toff = toff;
        a.first = first;
        a.X = X;
        a.re = edges;
        a.le[0] = edges + ering;
        a.le[1] = edges + 2 * ering;
        a.done = done;
        a.counter = counter;
        a.fault = g_ctx.fault;
        a.smax = (int)smax;
        a.queues = Q;
        a.spin_ticks = (uint64_t)spin_limit * 100;   // the real-time counter runs at 100 MHz
        a.chunk = g_chunk > 0 ? g_chunk : kChunkDefault;
        return SWEPT_OK;
    }

    void launch(hipStream_t st) const
    {
        if (grid == 0)
            return;
        hipLaunchKernelGGL(persist_clear_kernel, dim3(grid_for(std::max<int64_t>(1, tiles), 256)),
                           dim3(256), 0, st, a.done, tiles, a.counter, a.queues);
        if (xl)
            hipLaunchKernelGGL((swept_batch_persistent_kernel<S, 2, true>), dim3(grid), dim3(64),
                               lds, st, a);
        else
            hipLaunchKernelGGL((swept_batch_persistent_kernel<S, 2, false>), dim3(grid), dim3(64),
                               lds, st, a);
        hipLaunchKernelGGL(persist_check_kernel, dim3(1), dim3(64), 0, st, a.counter, a.first,
                           a.smax, a.queues, a.fault);
    }
};

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
        const int64_t want = g_ctx.tile_w > 0 ? g_ctx.tile_w / 2 : batch_want(ids[j]);
        const int64_t k = batch_depth(ids[j], p.n_ring, want);
        const int64_t half = p.n_ring / 2;
        const int64_t T = std::max<int64_t>(1, (half + k - 1) / k);   // half-widths <= k
        const int64_t kt = T > 1 ? k : half, rem = half - (T - 1) * kt;
        p.tiles = (int)T;
        p.kmax = (int)kt;
        p.x_off = (int64_t)X.size();
        X.push_back(0);
        for (int64_t t = 0; t < T; ++t)
            X.push_back(X.back() + 2 * (t + 1 < T ? kt : rem));
        // stage s >= 1 of tile t starts at level b = (X_{t+s} - X_{t+1})/2, the
        // sum of s-1 consecutive half-widths, which hold the short tile at
        // most ceil((s-1)/T) times: b >= (s-1)h/T - (kt - rem).  A tile's
        // regions end once b >= L, so s <= 1 + (L + kt - rem)T/h.
        p.stages = p.L == 0 ? 0 : 2 + (p.L + kt - rem) * T / half;
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
    // the fused heat form: one decision for all heat instances of the batch,
    // on the same conditions as a single field's (r and run length here,
    // the range of every heat field on the device, heat_range_batch_kernel)
    bool any_heat = false, fusable = g_ctx.heat_form == SWEPT_FORM_AUTO;
    int64_t nmax_heat = 0;
    for (int64_t j = 0; j < count; ++j) {
        const BatchPlanInst& p = P[(size_t)j];
        if (p.stencil != SWEPT_HEAT_F64)
            continue;
        any_heat = true;
        nmax_heat = std::max(nmax_heat, p.n_ring);
        const double r = heat64_consts(params + 2 * j).r;
        fusable = fusable && r >= 0 && r <= 0.5 && p.L <= kFusedMaxLevels<double>;
    }
    fusable = fusable && any_heat;
    // record of the last heat call, once the batch has been enqueued
    auto record_form = [&]() {
        if (!any_heat)
            return;
        g_ctx.last_guard = 0;
        g_ctx.last_batch = fusable;
        g_ctx.last_form = fusable ? SWEPT_FORM_FUSED : SWEPT_FORM_CANONICAL;
    };
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
    std::vector<int> tpos((size_t)count, 0);
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
    // persistent launches: each stencil's instances in Q queues, one per XCD
    // unless a number of queues was set (or the XCDs could not be told apart).
    // A queue holds whole instances, so a batch whose instances cannot be
    // spread evenly (a few large ones) would leave XCDs idle: such a batch
    // takes one launch per stage instead.
    bool persist = g_batch_sched == SWEPT_BATCH_PERSISTENT;
    int nxcd = 0;
    if (persist && g_queues == 0) {
        int rc0 = probe_xcds(&nxcd);
        if (rc0)
            return rc0;
    }
    const bool xcd_local = nxcd > 0;
    const int Q = xcd_local ? nxcd : (g_queues > 0 ? g_queues : kQueuesDefault);
    PersistPlan pph, ppk;
    if (persist) {
        pph = persist_plan(P, false, smax, Q, tpos);
        ppk = persist_plan(P, true, smax, Q, tpos);
        auto uneven = [](const PersistPlan& pp) {
            return pp.load_max > kQueueImbalance * pp.load_mean;
        };
        if (g_queues == 0 && (uneven(pph) || uneven(ppk))) {
            persist = false;
            pph = PersistPlan{};
            ppk = PersistPlan{};
        }
    }
    if (persist) {
        if (std::max(pph.max_total, ppk.max_total) >= (int64_t(1) << 31))
            return fail(SWEPT_EUNSUPPORTED,
                        "swept_advance_batch: %lld regions in one queue exceed the persistent "
                        "launch's 2^31 task numbers (use SWEPT_BATCH_STAGED)",
                        (long long)std::max(pph.max_total, ppk.max_total));
    }

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
    // persistent: [tasks h][tasks k][toff h, k][first h, k][done h, k][counters h, k]
    const size_t b_pt = al(sizeof(BatchTask) * (pph.tasks.size() + ppk.tasks.size() + 1));
    const size_t b_toff = al(sizeof(int64_t) * 2 * (size_t)(Q + 1));
    const size_t b_first = al(sizeof(int64_t) * (pph.first.size() + ppk.first.size()));
    const size_t b_done = al(sizeof(int) * (pph.tasks.size() + ppk.tasks.size() + 1));
    const size_t b_cnt = al(sizeof(unsigned) * 2 * (size_t)Q * kCounterStride);
    int ncover = 0;
    for (const auto& p : P)
        ncover += p.f_off >= 0;
    const size_t b_cov = al(sizeof(CoverEntry) * 2 * (size_t)std::max(1, ncover));
    const size_t b_main = b_ih + b_ik + b_x + b_th + b_tk + b_eh + b_ek + b_f + b_cov;
    int rc = ensure_scratch(b_main + (persist ? b_pt + b_toff + b_first + b_done + b_cnt : 0));
    if (rc)
        return rc;
    if (persist && !g_ctx.fault) {
        HIP_TRY(hipMalloc(&g_ctx.fault, sizeof(int)));
        HIP_TRY(hipMemset(g_ctx.fault, 0, sizeof(int)));
    }
    unsigned char* base = static_cast<unsigned char*>(g_ctx.scratch);
    auto* d_ih = reinterpret_cast<BatchInst<HeatF64>*>(base);
    auto* d_ik = reinterpret_cast<BatchInst<KSF64>*>(base + b_ih);
    auto* d_x = reinterpret_cast<int64_t*>(base + b_ih + b_ik);
    auto* d_th = reinterpret_cast<BatchTask*>(base + b_ih + b_ik + b_x);
    auto* d_tk = reinterpret_cast<BatchTask*>(base + b_ih + b_ik + b_x + b_th);
    auto* d_eh = reinterpret_cast<PtH*>(base + b_ih + b_ik + b_x + b_th + b_tk);
    auto* d_ek = reinterpret_cast<PtK*>(base + b_ih + b_ik + b_x + b_th + b_tk + b_eh);
    auto* d_f = reinterpret_cast<double*>(base + b_ih + b_ik + b_x + b_th + b_tk + b_eh + b_ek);
    auto* d_cov = reinterpret_cast<CoverEntry*>(base + b_main - b_cov);   // in, then out
    auto* d_pt = reinterpret_cast<BatchTask*>(base + b_main);
    auto* d_toff = reinterpret_cast<int64_t*>(base + b_main + b_pt);
    auto* d_first = reinterpret_cast<int64_t*>(base + b_main + b_pt + b_toff);
    auto* d_done = reinterpret_cast<int*>(base + b_main + b_pt + b_toff + b_first);
    auto* d_cnt = reinterpret_cast<unsigned*>(base + b_main + b_pt + b_toff + b_first + b_done);

    std::vector<BatchInst<HeatF64>> ih((size_t)count);
    std::vector<BatchInst<KSF64>> ik((size_t)count);
    for (int64_t j = 0; j < count; ++j) {
        const BatchPlanInst& p = P[(size_t)j];
        double* field = p.f_off >= 0 ? d_f + p.f_off : static_cast<double*>(u[j]);
        if (p.stencil == SWEPT_KS_F64)
            ik[(size_t)j] = BatchInst<KSF64>{field, p.n_ring, p.L, p.x_off, p.e_off, p.tiles,
                                            tpos[(size_t)j], ks_consts(params + 2 * j)};
        else
            ih[(size_t)j] = BatchInst<HeatF64>{field, p.n_ring, p.L, p.x_off, p.e_off, p.tiles,
                                              tpos[(size_t)j], heat64_consts(params + 2 * j)};
    }
    HIP_TRY(hipStreamSynchronize(g_ctx.stream));
    HIP_TRY(hipMemcpy(d_ih, ih.data(), sizeof(BatchInst<HeatF64>) * (size_t)count, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_ik, ik.data(), sizeof(BatchInst<KSF64>) * (size_t)count, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(d_x, X.data(), sizeof(int64_t) * X.size(), hipMemcpyHostToDevice));
    if (!th.empty())
        HIP_TRY(hipMemcpy(d_th, th.data(), sizeof(BatchTask) * th.size(), hipMemcpyHostToDevice));
    if (!tk.empty())
        HIP_TRY(hipMemcpy(d_tk, tk.data(), sizeof(BatchTask) * tk.size(), hipMemcpyHostToDevice));
    if (ncover > 0) {
        std::vector<CoverEntry> cov(2 * (size_t)ncover);
        size_t c = 0;
        for (int64_t j = 0; j < count; ++j) {
            const BatchPlanInst& p = P[(size_t)j];
            if (p.f_off < 0)
                continue;
            cov[c] = CoverEntry{static_cast<const double*>(u[j]), d_f + p.f_off, p.n_user, 2};
            cov[(size_t)ncover + c] =
                CoverEntry{d_f + p.f_off, static_cast<double*>(u[j]), p.n_user, 1};
            ++c;
        }
        HIP_TRY(hipMemcpy(d_cov, cov.data(), sizeof(CoverEntry) * cov.size(),
                          hipMemcpyHostToDevice));
    }
    if (persist) {
        std::vector<BatchTask> pt(pph.tasks);
        pt.insert(pt.end(), ppk.tasks.begin(), ppk.tasks.end());
        std::vector<int64_t> toff(pph.toff), first(pph.first);
        toff.insert(toff.end(), ppk.toff.begin(), ppk.toff.end());
        first.insert(first.end(), ppk.first.begin(), ppk.first.end());
        if (!pt.empty())
            HIP_TRY(hipMemcpy(d_pt, pt.data(), sizeof(BatchTask) * pt.size(),
                              hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_toff, toff.data(), sizeof(int64_t) * toff.size(),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_first, first.data(), sizeof(int64_t) * first.size(),
                          hipMemcpyHostToDevice));
    }

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
    key.push_back(g_batch_sched);
    key.push_back(g_spin_limit);
    key.push_back(g_chunk);
    key.push_back(g_queues);
    key.push_back(g_ctx.heat_form);
    for (int64_t w : g_batch_want)
        key.push_back(w);
    if (g_batch.exec && key == g_batch.key) {
        HIP_TRY(hipGraphLaunch(g_batch.exec, g_ctx.stream));
        g_ctx.fault_unread |= persist;
        record_form();
        return SWEPT_OK;
    }
    batch_release();
    // persistent launches: as many workgroups as can be resident at once
    PersistLaunch<HeatF64> plh;
    PersistLaunch<KSF64> plk;
    if (persist) {
        const int64_t lim = g_spin_limit > 0 ? g_spin_limit : kSpinDefault;
        int rc2 = plh.setup(pph, d_ih, d_pt, d_toff, d_first, d_x, d_eh, e_heat, d_done, d_cnt,
                            smax, Q, xcd_local, kmax_h, lim);
        if (!rc2)
            rc2 = plk.setup(ppk, d_ik, d_pt + pph.tasks.size(), d_toff + (Q + 1),
                            d_first + pph.first.size(), d_x, d_ek, e_ks,
                            d_done + pph.tasks.size(), d_cnt + (size_t)Q * kCounterStride, smax,
                            Q, xcd_local, kmax_k, lim);
        if (rc2)
            return rc2;
        plh.a.fusable = fusable;
    }
    // the two persistent launches run side by side on a forked branch of the
    // graph (each waits only on its own regions, so either may start first)
    const bool fork = persist && plh.grid > 0 && plk.grid > 0;
    hipStream_t cs, cs2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    auto release_capture_objects = [&]() {
        (void)hipStreamDestroy(cs);
        if (cs2)
            (void)hipStreamDestroy(cs2);
        if (ev_fork)
            (void)hipEventDestroy(ev_fork);
        if (ev_join)
            (void)hipEventDestroy(ev_join);
    };
    if (fork) {
        hipError_t e0 = hipStreamCreateWithFlags(&cs2, hipStreamNonBlocking);
        if (e0 == hipSuccess)
            e0 = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming);
        if (e0 == hipSuccess)
            e0 = hipEventCreateWithFlags(&ev_join, hipEventDisableTiming);
        if (e0 != hipSuccess) {
            release_capture_objects();
            return hip_fail(e0, "batch graph streams");
        }
    }
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        release_capture_objects();
        return hip_fail(e, "hipStreamBeginCapture");
    }
    if (ncover > 0)          // odd rings: build the two-fold covers
        hipLaunchKernelGGL(batch_cover_all_kernel, dim3((unsigned)(ncover * kCoverBlocks)),
                           dim3(256), 0, cs, d_cov, ncover);
    // the heat fields' range check, after the covers (which it reads for odd
    // rings) and before both stencils' regions, while it has the GPU to itself
    if (fusable) {
        const unsigned rows = (unsigned)std::min<int64_t>(64, std::max<int64_t>(1, nmax_heat / 8192));
        hipLaunchKernelGGL(batch_form_clear_kernel, dim3(1), dim3(64), 0, cs);
        hipLaunchKernelGGL(heat_range_batch_kernel<HeatF64>, dim3((unsigned)count, rows), dim3(256),
                           0, cs, d_ih, std::numeric_limits<double>::max() / 16);
    }
    if (persist) {
        if (fork) {
            (void)hipEventRecord(ev_fork, cs);
            (void)hipStreamWaitEvent(cs2, ev_fork, 0);
            plk.launch(cs2);
            (void)hipEventRecord(ev_join, cs2);
        }
        plh.launch(cs);
        if (fork)
            (void)hipStreamWaitEvent(cs, ev_join, 0);
        else
            plk.launch(cs);
    } else {
        size_t ph = 0, pk = 0;
        for (int64_t g = 0; g < smax; ++g) {
            while (ph < sh.size() && sh[ph] > g) ++ph;
            while (pk < sk.size() && sk[pk] > g) ++pk;
            launch_batch_stage<HeatF64>(d_ih, d_th, d_x, d_eh, d_eh + e_heat, d_eh + 2 * e_heat,
                                        (int)g, (int64_t)ph, kmax_h, fusable, cs);
            launch_batch_stage<KSF64>(d_ik, d_tk, d_x, d_ek, d_ek + e_ks, d_ek + 2 * e_ks, (int)g,
                                      (int64_t)pk, kmax_k, 0, cs);
        }
    }
    if (ncover > 0)          // odd rings: copy one period back
        hipLaunchKernelGGL(batch_cover_all_kernel, dim3((unsigned)(ncover * kCoverBlocks)),
                           dim3(256), 0, cs, d_cov + ncover, ncover);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    release_capture_objects();
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
    g_ctx.fault_unread |= persist;
    record_form();
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
    T* b = static_cast<T*>(scratch_base());
    // 16 bytes of points per thread where the length and the field allow
    constexpr int V = 16 / sizeof(T);
    const bool vec = nx % V == 0 && reinterpret_cast<uintptr_t>(u) % 16 == 0;
    const unsigned grid = grid_for(vec ? nx / V : nx, 256);
    for (int64_t s = 0; s < nsteps; ++s) {
        if (vec)
            hipLaunchKernelGGL((naive_step_vec_kernel<S>), dim3(grid), dim3(256), 0, g_ctx.stream,
                               a, b, nx, c);
        else
            hipLaunchKernelGGL((naive_step_kernel<S>), dim3(grid), dim3(256), 0, g_ctx.stream, a,
                               b, nx, c);
        std::swap(a, b);
    }
    if (a != u)
        HIP_TRY(hipMemcpyAsync(u, a, (size_t)nx * sizeof(T), hipMemcpyDeviceToDevice,
                               g_ctx.stream));
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

template <class S, int NB, int NT>
int run_naive_fused(void* u, int64_t nx, int64_t nsteps, const typename S::Consts& c)
{
    using T = typename S::T;
    int rc = ensure_scratch((size_t)nx * sizeof(T));
    if (rc)
        return rc;
    T* a = static_cast<T*>(u);
    T* b = static_cast<T*>(scratch_base());
    const unsigned grid = (unsigned)((nx + NB - 1) / NB);
    for (int64_t s = 0; s < nsteps; ++s) {
        hipLaunchKernelGGL((naive_fused_kernel<S, NB, NT>), dim3(grid), dim3(NT), 0, g_ctx.stream,
                           a, b, nx, c);
        std::swap(a, b);
    }
    if (a != u)
        HIP_TRY(hipMemcpyAsync(u, a, (size_t)nx * sizeof(T), hipMemcpyDeviceToDevice,
                               g_ctx.stream));
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

template <class S>
int run_naive_substep(void* u, int64_t nx, int64_t nsteps, const typename S::Consts& c)
{
    using Pt = typename S::Pt;
    using T = typename S::T;
    int rc = ensure_scratch(2 * (size_t)nx * sizeof(Pt));
    if (rc)
        return rc;
    Pt* a = static_cast<Pt*>(scratch_base());
    Pt* b = a + nx;
    const unsigned grid = grid_for(nx, 256);
    T* uf = static_cast<T*>(u);
    hipLaunchKernelGGL((field_to_pt_kernel<S>), dim3(grid), dim3(256), 0, g_ctx.stream, uf, a, nx);
    for (int64_t s = 0; s < nsteps; ++s) {
        hipLaunchKernelGGL((naive_substep_kernel<S, 0>), dim3(grid), dim3(256), 0, g_ctx.stream,
                           a, b, nx, c);
        hipLaunchKernelGGL((naive_substep_kernel<S, 1>), dim3(grid), dim3(256), 0, g_ctx.stream,
                           b, a, nx, c);
        hipLaunchKernelGGL((naive_substep_kernel<S, 2>), dim3(grid), dim3(256), 0, g_ctx.stream,
                           a, b, nx, c);
        hipLaunchKernelGGL((naive_substep_kernel<S, 3>), dim3(grid), dim3(256), 0, g_ctx.stream,
                           b, a, nx, c);
    }
    hipLaunchKernelGGL((pt_to_field_kernel<S>), dim3(grid), dim3(256), 0, g_ctx.stream, a, uf,
                       nx);
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

int naive_dispatch(void* u, int64_t nx, int64_t nsteps, int32_t id, const double* params)
{
    switch (id) {
    case SWEPT_HEAT_F64: return run_naive_single<HeatF64>(u, nx, nsteps, heat64_consts(params));
    case SWEPT_HEAT_F32: return run_naive_single<HeatF32>(u, nx, nsteps, heat32_consts(params));
    case SWEPT_HEAT_F64_FMA:
        return run_naive_single<HeatFmaF64>(u, nx, nsteps, heat64_consts(params));
    case SWEPT_HEAT_F32_FMA:
        return run_naive_single<HeatFmaF32>(u, nx, nsteps, heat32_consts(params));
    case SWEPT_KS_F64_FMA:
        return nx >= 1024 * 512
                   ? run_naive_fused<KSFmaF64, 1024, 512>(u, nx, nsteps, ks_consts(params))
                   : run_naive_fused<KSFmaF64, 256, 256>(u, nx, nsteps, ks_consts(params));
    // large blocks where the grid still has at least 512 of them (two per CU)
    case SWEPT_EULER_F64:
        return nx >= 256 * 512
                   ? run_naive_fused<EulerF64, 256, 256>(u, nx, nsteps, euler_consts(params))
                   : run_naive_fused<EulerF64, 128, 128>(u, nx, nsteps, euler_consts(params));
    default:
        return nx >= 1024 * 512
                   ? run_naive_fused<KSF64, 1024, 512>(u, nx, nsteps, ks_consts(params))
                   : run_naive_fused<KSF64, 256, 256>(u, nx, nsteps, ks_consts(params));
    }
}

// The naive schedule for a batch: per time step, one launch per stencil over
// the blocks of the instances that still have steps to go (instances sorted
// by step count, so those blocks are a prefix of the block list).
template <class S, int NB>
void naive_batch_tables(const std::vector<int64_t>& order, void* const* u, const int64_t* nx,
                        const int64_t* nsteps, const int32_t* ids, const double* params,
                        int32_t id, typename S::T* spare, const std::vector<int64_t>& spare_off,
                        typename S::Consts (*consts)(const double*),
                        std::vector<NaiveInst<S>>& inst, std::vector<NaiveBlock<S>>& blocks,
                        std::vector<int64_t>& block_steps)
{
    for (int64_t j : order) {
        if (ids[j] != id || nsteps[j] == 0)
            continue;
        const int64_t q = (int64_t)inst.size();
        inst.push_back(NaiveInst<S>{consts(params + 2 * j)});
        for (int64_t x0 = 0; x0 < nx[j]; x0 += NB) {
            NaiveBlock<S> b{};
            b.buf[0] = static_cast<typename S::T*>(u[j]);
            b.buf[1] = spare + spare_off[(size_t)j];
            b.n = nx[j];
            b.x0 = x0;
            b.inst = q;
            blocks.push_back(b);
            block_steps.push_back(nsteps[j]);
        }
    }
}

int run_naive_batch(void* const* u, const int64_t* nx, const int64_t* nsteps, const int32_t* ids,
                    const double* params, int64_t count)
{
    constexpr int NBH = 1024, NBK = 256;
    std::vector<int64_t> order((size_t)count), spare_off((size_t)count);
    size_t total = 0;
    int64_t smax = 0;
    for (int64_t j = 0; j < count; ++j) {
        order[(size_t)j] = j;
        spare_off[(size_t)j] = (int64_t)total;
        total += (size_t)nx[j];
        smax = std::max(smax, nsteps[j]);
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return nsteps[a] > nsteps[b]; });
    std::vector<NaiveInst<HeatF64>> ih;
    std::vector<NaiveInst<KSF64>> ik;
    std::vector<NaiveBlock<HeatF64>> bh;
    std::vector<NaiveBlock<KSF64>> bk;
    std::vector<int64_t> sh, sk;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_f = al(total * sizeof(double));
    const size_t cap_i = al(sizeof(NaiveInst<KSF64>) * (size_t)std::max<int64_t>(1, count));
    size_t nblocks = 0;
    for (int64_t j = 0; j < count; ++j)
        nblocks += (size_t)((nx[j] + NBK - 1) / NBK);
    const size_t b_b = al(sizeof(NaiveBlock<KSF64>) * std::max<size_t>(1, nblocks));
    int rc = ensure_scratch(b_f + 2 * cap_i + 2 * b_b);
    if (rc)
        return rc;
    unsigned char* base = static_cast<unsigned char*>(g_ctx.scratch);
    double* spare = reinterpret_cast<double*>(base);
    auto* d_ih = reinterpret_cast<NaiveInst<HeatF64>*>(base + b_f);
    auto* d_ik = reinterpret_cast<NaiveInst<KSF64>*>(base + b_f + cap_i);
    auto* d_bh = reinterpret_cast<NaiveBlock<HeatF64>*>(base + b_f + 2 * cap_i);
    auto* d_bk = reinterpret_cast<NaiveBlock<KSF64>*>(base + b_f + 2 * cap_i + b_b);
    naive_batch_tables<HeatF64, NBH>(order, u, nx, nsteps, ids, params, SWEPT_HEAT_F64, spare,
                                     spare_off, heat64_consts, ih, bh, sh);
    naive_batch_tables<KSF64, NBK>(order, u, nx, nsteps, ids, params, SWEPT_KS_F64, spare,
                                   spare_off, ks_consts, ik, bk, sk);
    HIP_TRY(hipStreamSynchronize(g_ctx.stream));
    if (!ih.empty()) {
        HIP_TRY(hipMemcpy(d_ih, ih.data(), sizeof(ih[0]) * ih.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_bh, bh.data(), sizeof(bh[0]) * bh.size(), hipMemcpyHostToDevice));
    }
    if (!ik.empty()) {
        HIP_TRY(hipMemcpy(d_ik, ik.data(), sizeof(ik[0]) * ik.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(d_bk, bk.data(), sizeof(bk[0]) * bk.size(), hipMemcpyHostToDevice));
    }
    size_t ph = bh.size(), pk = bk.size();
    for (int64_t s = 0; s < smax; ++s) {
        while (ph > 0 && sh[ph - 1] <= s) --ph;
        while (pk > 0 && sk[pk - 1] <= s) --pk;
        if (ph)
            hipLaunchKernelGGL((naive_batch_kernel<HeatF64, NBH>), dim3((unsigned)ph), dim3(256),
                               0, g_ctx.stream, d_ih, d_bh, (int)(s & 1));
        if (pk)
            hipLaunchKernelGGL((naive_batch_kernel<KSF64, NBK>), dim3((unsigned)pk), dim3(256), 0,
                               g_ctx.stream, d_ik, d_bk, (int)(s & 1));
    }
    // an odd step count leaves the result in the spare buffer
    for (int64_t j = 0; j < count; ++j)
        if (nsteps[j] % 2 == 1)
            HIP_TRY(hipMemcpyAsync(u[j], spare + spare_off[(size_t)j], (size_t)nx[j] * sizeof(double),
                                   hipMemcpyDeviceToDevice, g_ctx.stream));
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

// The straight decomposition of the discrete adjoint: a forward pass of one
// launch per step that keeps every step's field, then one launch per step
// backwards.  Scratch: (nsteps + 1) fields and two cotangent fields.
template <class S, int NB, class StepFn>
int run_naive_adjoint(const void* u0v, void* gradv, int64_t nx, int64_t nsteps,
                      const typename S::Consts& c, int64_t win_first, double wgt,
                      const void* cotv, StepFn forward_step)
{
    using T = typename S::T;
    const T* u0 = static_cast<const T*>(u0v);
    T* grad = static_cast<T*>(gradv);
    const T* cot = static_cast<const T*>(cotv);
    const T two_w = (T)(2.0 * wgt);
    const size_t field = ((size_t)nx * sizeof(T) + 255) / 256 * 256;
    if ((double)(nsteps + 3) * (double)field > 1.5e14)
        return fail(SWEPT_ENOMEM, "the naive adjoint would keep %lld fields", (long long)nsteps + 1);
    int rc = ensure_scratch((size_t)(nsteps + 3) * field);
    if (rc)
        return rc;
    unsigned char* base = static_cast<unsigned char*>(g_ctx.scratch);
    auto slot = [&](int64_t j) { return reinterpret_cast<T*>(base + (size_t)j * field); };
    T* ub[2] = {reinterpret_cast<T*>(base + (size_t)(nsteps + 1) * field),
                reinterpret_cast<T*>(base + (size_t)(nsteps + 2) * field)};
    HIP_TRY(hipMemcpyAsync(slot(0), u0, (size_t)nx * sizeof(T), hipMemcpyDeviceToDevice,
                           g_ctx.stream));
    for (int64_t j = 0; j < nsteps; ++j)
        forward_step(slot(j), slot(j + 1));
    T* out = nsteps == 0 ? grad : ub[0];
    hipLaunchKernelGGL((adjoint_seed_kernel<S>), dim3(grid_for(nx, 256)), dim3(256), 0,
                       g_ctx.stream, slot(nsteps), cot, out, nx, two_w,
                       nsteps >= win_first ? 1 : 0);
    const unsigned grid = (unsigned)((nx + NB - 1) / NB);
    for (int64_t j = nsteps - 1; j >= 0; --j) {
        const int in = (int)((nsteps - 1 - j) & 1);
        T* dst = j == 0 ? grad : ub[in ^ 1];
        hipLaunchKernelGGL((naive_adjoint_kernel<S, NB>), dim3(grid), dim3(NB), 0, g_ctx.stream,
                           slot(j), ub[in], dst, nx, c, two_w, j >= win_first ? 1 : 0);
    }
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

// swept_advance after validation: plan, then the swept or the naive schedule
int advance_dispatch(void* u, int64_t nx, int64_t nsteps, int32_t id, const double* params)
{
    if (nsteps == 0)
        return SWEPT_OK;
    Plan p;
    int rc = make_plan(nx, nsteps, id, &p);
    if (rc)
        return rc;
    if (p.mode == SWEPT_MODE_NAIVE) {
        if (id == SWEPT_HEAT_F64 || id == SWEPT_HEAT_F32) {
            g_ctx.last_guard = 0;
            g_ctx.last_batch = false;
            g_ctx.last_form = SWEPT_FORM_CANONICAL;
        }
        return naive_dispatch(u, nx, nsteps, id, params);
    }
    const int64_t L = nsteps * substeps_of(id);
    if (p.mode == SWEPT_MODE_STAGE_RAGGED) {
        switch (id) {
        case SWEPT_HEAT_F64: return run_ragged<HeatF64>(u, nx, L, heat64_consts(params), p);
        case SWEPT_HEAT_F32: return run_ragged<HeatF32>(u, nx, L, heat32_consts(params), p);
        case SWEPT_EULER_F64: return run_ragged<EulerF64>(u, nx, L, euler_consts(params), p);
        case SWEPT_HEAT_F64_FMA:
            return run_ragged<HeatFmaF64>(u, nx, L, heat64_consts(params), p);
        case SWEPT_HEAT_F32_FMA:
            return run_ragged<HeatFmaF32>(u, nx, L, heat32_consts(params), p);
        case SWEPT_KS_F64_FMA: return run_ragged<KSFmaF64>(u, nx, L, ks_consts(params), p);
        default: return run_ragged<KSF64>(u, nx, L, ks_consts(params), p);
        }
    }
    switch (id) {
    case SWEPT_HEAT_F64: return run_swept<HeatF64>(u, nx, L, heat64_consts(params), p);
    case SWEPT_HEAT_F32: return run_swept<HeatF32>(u, nx, L, heat32_consts(params), p);
    case SWEPT_EULER_F64: return run_swept<EulerF64>(u, nx, L, euler_consts(params), p);
    case SWEPT_HEAT_F64_FMA: return run_swept<HeatFmaF64>(u, nx, L, heat64_consts(params), p);
    case SWEPT_HEAT_F32_FMA: return run_swept<HeatFmaF32>(u, nx, L, heat32_consts(params), p);
    case SWEPT_KS_F64_FMA: return run_swept<KSFmaF64>(u, nx, L, ks_consts(params), p);
    default: return run_swept<KSF64>(u, nx, L, ks_consts(params), p);
    }
}

// ----------------------------------------------------------------- objective

int ensure_obj(size_t bytes)
{
    if (bytes <= g_ctx.obj_bytes)
        return SWEPT_OK;
    if (g_ctx.obj) {
        HIP_TRY(hipStreamSynchronize(g_ctx.stream));
        HIP_TRY(hipFree(g_ctx.obj));
        g_ctx.obj = nullptr;
        g_ctx.obj_bytes = 0;
    }
    hipError_t e = hipMalloc(&g_ctx.obj, bytes);
    if (e != hipSuccess) {
        g_ctx.obj = nullptr;
        (void)hipGetLastError();
        return fail(SWEPT_ENOMEM, "hipMalloc of %zu bytes for the objective failed: %s", bytes,
                    hipGetErrorString(e));
    }
    g_ctx.obj_bytes = bytes;
    return SWEPT_OK;
}

// J = w * sum_{j = max(first, 0)}^{nsteps} |u^j|^2 + <cot, u^nsteps>: a copy of
// u0 advanced by the swept schedule to the step before the window, then one
// naive step at a time, each step's field summed on the device.
int run_objective(const void* u0, int64_t nx, int64_t nsteps, int32_t id, const double* params,
                  int64_t first, double wgt, const void* cot, double* J)
{
    const size_t field = ((size_t)nx * sizeof(double) + 255) / 256 * 256;
    int rc = ensure_obj(field + 4 * kObjBlocks * sizeof(double));
    if (rc)
        return rc;
    double* f = static_cast<double*>(g_ctx.obj);
    double* acc_sq = reinterpret_cast<double*>(static_cast<unsigned char*>(g_ctx.obj) + field);
    double* acc_dot = acc_sq + 2 * kObjBlocks;
    HIP_TRY(hipMemcpyAsync(f, u0, (size_t)nx * sizeof(double), hipMemcpyDeviceToDevice,
                           g_ctx.stream));
    hipLaunchKernelGGL(objective_clear_kernel, dim3(1), dim3(256), 0, g_ctx.stream, acc_sq,
                       4 * kObjBlocks);
    auto sum_squares = [&] {
        hipLaunchKernelGGL(objective_accumulate_kernel, dim3(kObjBlocks), dim3(kObjThreads), 0,
                           g_ctx.stream, f, f, nx, acc_sq);
    };
    first = std::max<int64_t>(first, 0);
    if (first > nsteps) {
        rc = advance_dispatch(f, nx, nsteps, id, params);
    } else {
        if (first == 0)
            sum_squares();
        const int64_t pre = std::max<int64_t>(first - 1, 0);
        rc = advance_dispatch(f, nx, pre, id, params);
        for (int64_t j = pre + 1; j <= nsteps && rc == SWEPT_OK; ++j) {
            rc = naive_dispatch(f, nx, 1, id, params);
            if (rc == SWEPT_OK)
                sum_squares();
        }
    }
    if (rc)
        return rc;
    if (cot)
        hipLaunchKernelGGL(objective_accumulate_kernel, dim3(kObjBlocks), dim3(kObjThreads), 0,
                           g_ctx.stream, static_cast<const double*>(cot), f, nx, acc_dot);
    hipLaunchKernelGGL(objective_final_kernel, dim3(1), dim3(64), 0, g_ctx.stream, acc_sq, acc_dot,
                       wgt, J);
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

// ----------------------------------------------------------------- autotuner
//
// The paper's model (Section 4, Eq. (1)): with n points per node, a swept
// cycle computes for n^2 s and communicates twice, for 2 tau, while it
// advances n sub-timesteps, so a sub-timestep costs n s + 2 tau / n, least at
// n* = sqrt(2 tau / s).  On one GPU a node is a workgroup and tau is the cost
// of a stage boundary: the end of one launch, the edge round trip through
// memory, the start of the next.  s1 is the time one wavefront spends per
// point-substep when it runs alone.  Because the tiles share the chip, a
// sub-timestep also takes at least N s_full, s_full being the whole GPU's
// time per point-substep, so with W-point tiles
//     t(W) = max(W s1, N s_full) + 2 tau / W,
// least at W0 = max(N s_full / s1, sqrt(2 tau / s1)).  W0 centres the
// candidates; short timed runs choose among them.

struct DeviceBuffer {
    void* p = nullptr;
    ~DeviceBuffer()
    {
        if (p)
            (void)hipFree(p);
    }
    int alloc(size_t bytes)
    {
        hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(SWEPT_ENOMEM, "hipMalloc of %zu bytes for the tuner failed", bytes);
        }
        e = hipMemsetAsync(p, 0, bytes, g_ctx.stream);
        return e == hipSuccess ? SWEPT_OK : hip_fail(e, "hipMemsetAsync");
    }
};

// Probe fields hold zeros; Euler probes need a physical state (rho = 1,
// u = 0, p = 1 at gamma = 1.4: E = 2.5) so that no flux divides by zero.
int fill_probe_field(int id, void* p, size_t cells)
{
    if (id != SWEPT_EULER_F64)
        return SWEPT_OK;
    std::vector<Cons> h(cells, Cons{1.0, 0.0, 2.5});
    HIP_TRY(hipMemcpyAsync(p, h.data(), cells * sizeof(Cons), hipMemcpyHostToDevice, g_ctx.stream));
    HIP_TRY(hipStreamSynchronize(g_ctx.stream));
    return SWEPT_OK;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a)
            (void)hipEventDestroy(a);
        if (b)
            (void)hipEventDestroy(b);
    }
};

// Saves the tuning knobs and restores them on scope exit.
struct KnobGuard {
    int tile_w = g_ctx.tile_w, ppl = g_ctx.ppl, mode = g_ctx.mode;
    bool profiling = g_ctx.profiling;
    KnobGuard() { g_ctx.profiling = false; }
    ~KnobGuard()
    {
        g_ctx.tile_w = tile_w;
        g_ctx.ppl = ppl;
        g_ctx.mode = mode;
        g_ctx.profiling = profiling;
    }
};

// Best of `reps` timings (seconds) of fn() on the stream, after one untimed call.
template <class F>
int time_best(F&& fn, int reps, double* sec)
{
    int rc = fn();
    if (rc)
        return rc;
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    double best = 1e30;
    for (int r = 0; r < reps; ++r) {
        HIP_TRY(hipEventRecord(ev.a, g_ctx.stream));
        rc = fn();
        if (rc)
            return rc;
        HIP_TRY(hipEventRecord(ev.b, g_ctx.stream));
        HIP_TRY(hipEventSynchronize(ev.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
        best = std::min(best, 1e-3 * (double)ms);
    }
    *sec = best;
    return SWEPT_OK;
}

size_t field_bytes(int id)
{
    switch (base_id(id)) {
    case SWEPT_HEAT_F32: return sizeof(float);
    case SWEPT_EULER_F64: return sizeof(Cons);
    default: return sizeof(double);
    }
}

// One swept run of `nsteps` steps on the zero field f with the given tiling;
// returns its time and its number of stages.
// P = 0: the lane-frame kernel
int timed_swept(void* f, int64_t nx, int64_t nsteps, int id, const double* params, int64_t W,
                int P, int reps, double* sec, int64_t* stages, bool ragged = false)
{
    g_ctx.tile_w = (int)W;
    g_ctx.ppl = P;
    g_ctx.mode = ragged ? SWEPT_MODE_STAGE_RAGGED
                        : (P == 0 ? SWEPT_MODE_STAGE_LANE : SWEPT_MODE_STAGE);
    Plan p;
    int rc = make_plan(nx, nsteps, id, &p);
    if (rc)
        return rc;
    if (stages)
        *stages = p.stages;
    return time_best([&] { return advance_dispatch(f, nx, nsteps, id, params); }, reps, sec);
}

// tau, s1 and s_full of the stencil on this GPU
int measure_model(int id, const double* params, double* tau, double* s1, double* sfull)
{
    const int S = substeps_of(id);
    const int64_t nbig = int64_t(1) << 20;
    DeviceBuffer f;
    int rc = f.alloc((size_t)nbig * field_bytes(id));
    if (!rc)
        rc = fill_probe_field(id, f.p, (size_t)nbig);
    if (rc)
        return rc;
    double t;
    int64_t st;
    // tau: 64 tiles of 4 points over 64 stages with next to no work in them
    rc = timed_swept(f.p, 256, 128 / S, id, params, 4, 1, 3, &t, &st);
    if (rc)
        return rc;
    *tau = t / (double)st;
    // s1: a single 512-point tile, 2048 sub-timesteps, one workgroup
    const int64_t Ls = 2048;
    rc = timed_swept(f.p, 512, Ls / S, id, params, 512, 2, 2, &t, &st);
    if (rc)
        return rc;
    *s1 = std::max(1e-15, (t - (double)st * *tau) / (512.0 * (double)Ls));
    // s_full: 2^20 points in 512-point tiles
    rc = timed_swept(f.p, nbig, Ls / S, id, params, 512, 2, 2, &t, &st);
    if (rc)
        return rc;
    *sfull = std::max(1e-18, (t - (double)st * *tau) / ((double)nbig * (double)Ls));
    return SWEPT_OK;
}

// Even tile widths that divide nx and fit the LDS budget, nearest (in ratio)
// to each of the targets.
std::vector<int64_t> tile_candidates(int id, int64_t nx, const std::vector<double>& targets)
{
    std::vector<int64_t> valid;
    for (int64_t d = 1; d * d <= nx; ++d)
        if (nx % d == 0)
            for (int64_t w : {d, nx / d})
                if (w >= 4 && tile_fits(id, nx, w))
                    valid.push_back(w);
    std::vector<int64_t> out;
    for (double tg : targets) {
        int64_t best = 0;
        double bd = 1e30;
        for (int64_t w : valid) {
            const double dist = std::fabs(std::log((double)w / tg));
            if (dist < bd) {
                bd = dist;
                best = w;
            }
        }
        if (best && std::find(out.begin(), out.end(), best) == out.end())
            out.push_back(best);
    }
    std::sort(out.begin(), out.end());
    return out;
}

int autotune(int64_t nx, int64_t nsteps, int id, const double* params, double* report)
{
    KnobGuard guard;
    double tau = 0, s1 = 0, sfull = 0;
    int rc = measure_model(id, params, &tau, &s1, &sfull);
    if (rc)
        return rc;
    const double nstar = std::sqrt(2.0 * tau / s1);
    const double w0 = std::max((double)nx * sfull / s1, nstar);
    // The model leaves out that wider tiles hold more LDS, so fewer of them
    // share a CU to hide latency: the candidates reach well below W0.
    std::vector<int64_t> Ws =
        tile_candidates(id, nx, {w0 / 8, w0 / 4, w0 / 2, w0, 2 * w0, 4 * w0});
    {   // the untuned plan's width is always among the candidates
        g_ctx.tile_w = 0;
        g_ctx.ppl = 0;
        g_ctx.mode = SWEPT_MODE_STAGE;
        Plan dflt;
        if (make_plan(nx, nsteps, id, &dflt) == SWEPT_OK && dflt.W >= 4 &&
            std::find(Ws.begin(), Ws.end(), dflt.W) == Ws.end())
            Ws.push_back(dflt.W);
        g_err.clear();
    }
    const int S = substeps_of(id);
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g_ctx.device));
    DeviceBuffer f;
    rc = f.alloc((size_t)nx * field_bytes(id));
    if (!rc)
        rc = fill_probe_field(id, f.p, (size_t)nx);
    if (rc)
        return rc;
    // the naive schedule costs the same every step: time a few
    const int64_t nn = std::min<int64_t>(nsteps, 256);
    double t;
    g_ctx.mode = SWEPT_MODE_NAIVE;
    rc = time_best([&] { return naive_dispatch(f.p, nx, nn, id, params); }, 2, &t);
    if (rc)
        return rc;
    double best_rate = (double)nx * (double)nn / t;
    Tuned best{-1, 0};
    // the lane-frame kernel, for tilings whose regions are latency-bound:
    // the two widest widths it takes
    std::vector<int64_t> lane_Ws;
    for (int64_t w = 2 * kLaneMaxK; w >= 4 && lane_Ws.size() < 2; w -= 2)
        if (tile_fits(id, nx, w) && lane_fits(id, w / 2))
            lane_Ws.push_back(w);
    for (int64_t W : lane_Ws) {
        const int64_t per_cu = std::max<int64_t>(
            1, std::min<int64_t>(32, (160 * 1024) / (int64_t)lane_lds_bytes(id, W / 2)));
        const int64_t npts = W * std::min(nx / W, 4 * (int64_t)cus * per_cu);
        const int64_t Lp = std::min(nsteps * S, std::max<int64_t>(16 * (W / 2), 64));
        const int64_t np = std::max<int64_t>(1, (Lp + S - 1) / S);
        rc = timed_swept(f.p, npts, np, id, params, W, 0, 3, &t, nullptr);
        if (rc)
            return rc;
        const double rate = (double)npts * (double)np / t;
        if (rate > best_rate) {
            best_rate = rate;
            best = Tuned{W, 0};
        }
    }
    for (int64_t W : Ws) {
        // Once the tiles fill the chip the rate per point no longer depends
        // on their number: time four rounds of the workgroups that fit at
        // once (64-lane workgroups, at most 32 per CU, LDS of W points
        // each), over sixteen stages.
        const int64_t per_cu =
            std::max<int64_t>(1, std::min<int64_t>(32, (int64_t)((160 * 1024) /
                                                                 stage_lds_bytes(id, W))));
        const int64_t npts = W * std::min(nx / W, 4 * (int64_t)cus * per_cu);
        const int64_t Lp = std::min(nsteps * S, std::max<int64_t>(16 * (W / 2), 64));
        const int64_t np = std::max<int64_t>(1, (Lp + S - 1) / S);
        for (int P : {1, 2, 4}) {
            if ((P > 1 && 64 * P > W / 2) || P > pmax(id))
                continue;
            rc = timed_swept(f.p, npts, np, id, params, W, P, 3, &t, nullptr);
            if (rc)
                return rc;
            const double rate = (double)npts * (double)np / t;
            if (rate > best_rate) {
                best_rate = rate;
                best = Tuned{W, P};
            }
        }
    }
    {   // the unequal tiling, which the untuned plan takes where no good even
        // width divides nx: timed on the whole grid over sixteen of its stages
        g_tuned.erase(tune_key(id, nx));
        g_ctx.tile_w = 0;
        g_ctx.ppl = 0;
        g_ctx.mode = SWEPT_MODE_AUTO;
        Plan rg;
        const bool have = make_plan(nx, nsteps, id, &rg) == SWEPT_OK &&
                          rg.mode == SWEPT_MODE_STAGE_RAGGED;
        g_err.clear();
        if (have) {
            const int64_t Lp = std::min(nsteps * S, std::max<int64_t>(16 * rg.k, 64));
            const int64_t np = std::max<int64_t>(1, (Lp + S - 1) / S);
            rc = timed_swept(f.p, nx, np, id, params, rg.W, rg.P, 3, &t, nullptr, true);
            if (rc)
                return rc;
            const double rate = (double)nx * (double)np / t;
            if (rate > best_rate) {
                best_rate = rate;
                best = Tuned{rg.W, rg.P, true};
            }
        }
    }
    g_tuned[tune_key(id, nx)] = best;
    if (report) {
        const double r[8] = {tau, s1, sfull, nstar, w0, (double)std::max<int64_t>(best.W, 0),
                             (double)best.P, best_rate};
        std::memcpy(report, r, sizeof r);
    }
    return SWEPT_OK;
}

// The batch runs all its instances at once, so the chip is always full and
// the depth only trades the fill and drain of each region against its LDS
// and the stage count: time the batch's own shapes (one stencil at a time, zero
// fields, steps cut to a few stages) at each candidate depth.
int autotune_batch(const int64_t* nx, const int64_t* nsteps, const int32_t* ids,
                   const double* params, int64_t count, int64_t* want_out)
{
    KnobGuard guard;
    g_ctx.tile_w = 0;
    // the probe: the batch's binary64 instances on zero fields, every step
    // count scaled by one factor so that the longest instance runs
    // kTuneSubsteps sub-timesteps (the others keep their proportion, so the
    // spread of stage counts the schedule sees is the batch's)
    constexpr double kTuneSubsteps = 6144.0;
    std::vector<int64_t> sel;
    size_t total = 0;
    double lmax = 0.0;
    bool has[3] = {false, false, false};
    for (int64_t j = 0; j < count; ++j)
        if ((ids[j] == SWEPT_HEAT_F64 || ids[j] == SWEPT_KS_F64) && nsteps[j] > 0) {
            sel.push_back(j);
            total += (size_t)nx[j];
            lmax = std::max(lmax, (double)nsteps[j] * substeps_of(ids[j]));
            has[ids[j]] = true;
        }
    for (int id : {SWEPT_HEAT_F64, SWEPT_KS_F64})
        want_out[id] = 0;
    if (sel.empty())
        return SWEPT_OK;
    const double scale = std::min(1.0, kTuneSubsteps / lmax);
    DeviceBuffer f;
    int rc = f.alloc(total * sizeof(double));
    if (rc)
        return rc;
    std::vector<void*> up;
    std::vector<int64_t> nxs, ns;
    std::vector<int32_t> is;
    std::vector<double> ps;
    size_t off = 0;
    for (int64_t j : sel) {
        up.push_back(static_cast<double*>(f.p) + off);
        off += (size_t)nx[j];
        nxs.push_back(nx[j]);
        ns.push_back(std::max<int64_t>(1, std::llround((double)nsteps[j] * scale)));
        is.push_back(ids[j]);
        ps.push_back(params[2 * j]);
        ps.push_back(params[2 * j + 1]);
    }
    // coordinate descent over the two depths, the whole probe timed (the two
    // stencils' launches overlap, so each depth is judged beside the other):
    // KS first (most of the work), then heat.  Depths are multiples of the
    // band size 128 (two pairs per lane), so that the square regions can take
    // the continuous-band schedule.
    for (int id : {SWEPT_HEAT_F64, SWEPT_KS_F64})
        g_batch_want[id] = kBatchWantDefault;
    for (int id : {SWEPT_KS_F64, SWEPT_HEAT_F64}) {
        if (!has[id])
            continue;
        double best_t = 1e30;
        int64_t best = kBatchWantDefault;
        for (int64_t want : {128, 256, 384, 512}) {
            g_batch_want[id] = want;
            double t;
            rc = time_best([&] {
                return run_batch(up.data(), nxs.data(), ns.data(), is.data(), ps.data(),
                                 (int64_t)sel.size());
            }, 2, &t);
            if (rc)
                break;
            if (t < best_t) {
                best_t = t;
                best = want;
            }
        }
        g_batch_want[id] = best;
        want_out[id] = best;
        if (rc)
            break;
    }
    HIP_TRY(hipStreamSynchronize(g_ctx.stream));
    batch_release();  // its graph points at the probe fields
    if (rc) {
        for (int id : {SWEPT_HEAT_F64, SWEPT_KS_F64})
            g_batch_want[id] = 0;
        return rc;
    }
    return SWEPT_OK;
}

}  // namespace

// A roctx range around each entry point (visible to rocprofv3 --marker-trace;
// a no-op when no profiler is attached).
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

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
    if (g_noalloc_ptr.find(device) == g_noalloc_ptr.end()) {
        // the fixed scratch array's address on this device (each GPU holds
        // its own copy); host code uses only this address
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_noalloc_ptr[device] = p;
    }
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
        mode != SWEPT_MODE_STAGE_BANDED && mode != SWEPT_MODE_STAGE_LANE &&
        mode != SWEPT_MODE_STAGE_RAGGED)
        return fail(SWEPT_EINVAL, "unknown mode %d", mode);
    g_ctx.tile_w = tile_w;
    g_ctx.ppl = pairs_per_lane;
    g_ctx.mode = mode;
    return SWEPT_OK;
}

int swept_set_heat_form(int32_t form)
{
    if (form != SWEPT_FORM_AUTO && form != SWEPT_FORM_CANONICAL)
        return fail(SWEPT_EINVAL, "heat form %d is neither SWEPT_FORM_AUTO nor "
                                  "SWEPT_FORM_CANONICAL", form);
    g_ctx.heat_form = form;
    return SWEPT_OK;
}

int swept_last_heat_form(int32_t* form)
{
    if (!form)
        return fail(SWEPT_EINVAL, "form is null");
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    *form = g_ctx.last_form;
    if (g_ctx.last_form == SWEPT_FORM_FUSED) {
        HIP_TRY(hipStreamSynchronize(g_ctx.stream));
        if (g_ctx.last_batch) {
            int bad = 0;
            HIP_TRY(hipMemcpyFromSymbol(&bad, HIP_SYMBOL(g_batch_form_bad), sizeof(bad), 0,
                                        hipMemcpyDeviceToHost));
            if (bad != 0)
                *form = SWEPT_FORM_CANONICAL;
        } else {
            unsigned long long mark = 0;
            HIP_TRY(hipMemcpyFromSymbol(&mark, HIP_SYMBOL(g_form_mark), sizeof(mark), 0,
                                        hipMemcpyDeviceToHost));
            if (mark >= g_ctx.last_guard)
                *form = SWEPT_FORM_CANONICAL;
        }
    }
    return SWEPT_OK;
}

int swept_plan(int64_t nx, int64_t nsteps, int32_t stencil_id, int64_t* out)
{
    if (!out || nx < 3 || nsteps < 0 || !known_id(stencil_id))
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
    TraceRange trace_range("swept_advance");
    int rc = check_common(u, nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    return advance_dispatch(u, nx, nsteps, stencil_id, params);
}

int swept_advance_noalloc(void* u, int64_t nx, int64_t nsteps, int32_t stencil_id,
                          const double* params, int32_t nparams)
{
    int rc = check_common(u, nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    const auto it = g_noalloc_ptr.find(g_ctx.device);
    if (it == g_noalloc_ptr.end() || !it->second)
        return fail(SWEPT_ENOTINIT, "no fixed scratch address for device %d", g_ctx.device);
    // the fixed array replaces the growing scratch for this call; stage
    // profiling (which creates events) is off during it
    struct Fixed {
        bool prof = g_ctx.profiling;
        explicit Fixed(void* p)
        {
            g_fixed = p;
            g_ctx.profiling = false;
        }
        ~Fixed()
        {
            g_fixed = nullptr;
            g_ctx.profiling = prof;
        }
    } fixed(it->second);
    return advance_dispatch(u, nx, nsteps, stencil_id, params);
}

int swept_naive_advance(void* u, int64_t nx, int64_t nsteps, int32_t stencil_id,
                        const double* params, int32_t nparams)
{
    TraceRange trace_range("swept_naive_advance");
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
    TraceRange trace_range("swept_naive_substep_advance");
    int rc = check_common(u, nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    if (stencil_id != SWEPT_KS_F64 && stencil_id != SWEPT_EULER_F64)
        return fail(SWEPT_EINVAL,
                    "per-sub-timestep launches exist for the four-sub-timestep stencils only");
    if (nsteps == 0)
        return SWEPT_OK;
    if (stencil_id == SWEPT_EULER_F64)
        return run_naive_substep<EulerF64>(u, nx, nsteps, euler_consts(params));
    return run_naive_substep<KSF64>(u, nx, nsteps, ks_consts(params));
}

int swept_advance_batch(void* const* u, const int64_t* nx, const int64_t* nsteps,
                        const int32_t* stencil_id, const double* params, int64_t count)
{
    TraceRange trace_range("swept_advance_batch");
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

int swept_naive_advance_batch(void* const* u, const int64_t* nx, const int64_t* nsteps,
                              const int32_t* stencil_id, const double* params, int64_t count)
{
    TraceRange trace_range("swept_naive_advance_batch");
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
        if (nx[j] > (int64_t(1) << 40))
            return fail(SWEPT_EINVAL, "instance %lld is too long", (long long)j);
    }
    if (count == 0)
        return SWEPT_OK;
    return run_naive_batch(u, nx, nsteps, stencil_id, params, count);
}

int swept_autotune(int64_t nx, int64_t nsteps, int32_t stencil_id, const double* params,
                   int32_t nparams, double* report)
{
    TraceRange trace_range("swept_autotune");
    int rc = check_problem(nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    if (nsteps == 0)
        return fail(SWEPT_EINVAL, "nothing to tune for zero steps");
    rc = autotune(nx, nsteps, stencil_id, params, report);
    if (rc)
        return rc;
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

int swept_autotune_batch(const int64_t* nx, const int64_t* nsteps, const int32_t* stencil_id,
                         const double* params, int64_t count, int64_t* depth_out)
{
    TraceRange trace_range("swept_autotune_batch");
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    if (count < 0 || !depth_out || (count > 0 && (!nx || !nsteps || !stencil_id || !params)))
        return fail(SWEPT_EINVAL, "bad batch arrays");
    for (int64_t j = 0; j < count; ++j) {
        int rc = check_problem(nx[j], nsteps[j], stencil_id[j], params + 2 * j, 2);
        if (rc)
            return fail(rc, "instance %lld: %s", (long long)j, g_err.c_str());
        if (stencil_id[j] != SWEPT_HEAT_F64 && stencil_id[j] != SWEPT_KS_F64)
            return fail(SWEPT_EUNSUPPORTED, "instance %lld: the batch takes binary64 stencils",
                        (long long)j);
    }
    depth_out[0] = depth_out[1] = depth_out[2] = 0;
    int rc = autotune_batch(nx, nsteps, stencil_id, params, count, depth_out);
    if (rc)
        return rc;
    HIP_TRY(hipGetLastError());
    return SWEPT_OK;
}

int swept_clear_tuning(void)
{
    g_tuned.clear();
    for (int64_t& w : g_batch_want)
        w = 0;
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
    TraceRange trace_range("swept_adjoint");
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
        return fail(SWEPT_EUNSUPPORTED, "the adjoint exists for the heat and KS binary64 stencils only");
    }
}

int swept_window_objective(const void* u0, int64_t nx, int64_t nsteps, int32_t stencil_id,
                           const double* params, int32_t nparams, int64_t window_first,
                           double window_weight, const void* cot_final, void* J_out)
{
    TraceRange trace_range("swept_window_objective");
    int rc = check_common(u0, nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    if (!J_out)
        return fail(SWEPT_EINVAL, "J_out is NULL");
    if (!std::isfinite(window_weight))
        return fail(SWEPT_EINVAL, "window weight is not finite");
    if (stencil_id != SWEPT_HEAT_F64 && stencil_id != SWEPT_KS_F64 &&
        stencil_id != SWEPT_HEAT_F64_FMA && stencil_id != SWEPT_KS_F64_FMA)
        return fail(SWEPT_EUNSUPPORTED, "the objective takes single-value binary64 stencils");
    return run_objective(u0, nx, nsteps, stencil_id, params, window_first, window_weight,
                         cot_final, static_cast<double*>(J_out));
}

int swept_naive_adjoint(const void* u0, void* grad_u0, int64_t nx, int64_t nsteps,
                        int32_t stencil_id, const double* params, int32_t nparams,
                        int64_t window_first, double window_weight, const void* cot_final)
{
    TraceRange trace_range("swept_naive_adjoint");
    int rc = check_common(u0, nx, nsteps, stencil_id, params, nparams);
    if (rc)
        return rc;
    if (!grad_u0)
        return fail(SWEPT_EINVAL, "grad_u0 is NULL");
    if (!std::isfinite(window_weight))
        return fail(SWEPT_EINVAL, "window weight is not finite");
    switch (stencil_id) {
    case SWEPT_HEAT_F64: {
        const HeatF64::Consts c = heat64_consts(params);
        const unsigned grid = grid_for(nx, 256);
        return run_naive_adjoint<HeatF64, 256>(
            u0, grad_u0, nx, nsteps, c, window_first, window_weight, cot_final,
            [&](const double* a, double* b) {
                hipLaunchKernelGGL((naive_step_kernel<HeatF64>), dim3(grid), dim3(256), 0,
                                   g_ctx.stream, a, b, nx, c);
            });
    }
    case SWEPT_KS_F64: {
        const KSF64::Consts c = ks_consts(params);
        const bool big = nx >= 1024 * 512;   // as in the forward naive path
        const unsigned grid = (unsigned)(big ? (nx + 1023) / 1024 : (nx + 255) / 256);
        return run_naive_adjoint<KSF64, 128>(
            u0, grad_u0, nx, nsteps, c, window_first, window_weight, cot_final,
            [&](const double* a, double* b) {
                if (big)
                    hipLaunchKernelGGL((naive_fused_kernel<KSF64, 1024, 512>), dim3(grid),
                                       dim3(512), 0, g_ctx.stream, a, b, nx, c);
                else
                    hipLaunchKernelGGL((naive_fused_kernel<KSF64, 256, 256>), dim3(grid),
                                       dim3(256), 0, g_ctx.stream, a, b, nx, c);
            });
    }
    default:
        return fail(SWEPT_EUNSUPPORTED, "the adjoint exists for the heat and KS binary64 stencils only");
    }
}

int swept_sync(void)
{
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    HIP_TRY(hipStreamSynchronize(g_ctx.stream));
    HIP_TRY(hipGetLastError());
    if (g_ctx.fault_unread && g_ctx.fault) {
        int f = 0;
        HIP_TRY(hipMemcpy(&f, g_ctx.fault, sizeof f, hipMemcpyDeviceToHost));
        g_ctx.fault_unread = false;
        if (f) {
            HIP_TRY(hipMemset(g_ctx.fault, 0, sizeof f));
            if (f == 1)
                return fail(SWEPT_ETIMEOUT,
                            "swept_advance_batch: a persistent launch gave up waiting for a "
                            "region (spin limit %lld us); its fields are not valid",
                            (long long)(g_spin_limit > 0 ? g_spin_limit : kSpinDefault));
            return fail(SWEPT_EHIP,
                        "swept_advance_batch: a persistent launch left a queue unserved (%s); "
                        "its fields are not valid",
                        f == 3 ? "a workgroup ran on an XCD the probe did not see"
                               : "no workgroup took its last tasks");
        }
    }
    return SWEPT_OK;
}

int swept_set_batch_schedule(int32_t schedule, int64_t spin_limit, int32_t chunk,
                             int32_t queues)
{
    if (schedule != SWEPT_BATCH_PERSISTENT && schedule != SWEPT_BATCH_STAGED)
        return fail(SWEPT_EINVAL, "swept_set_batch_schedule: unknown schedule %d", schedule);
    if (spin_limit < 0)
        return fail(SWEPT_EINVAL, "swept_set_batch_schedule: spin_limit %lld < 0",
                    (long long)spin_limit);
    if (chunk < 0 || chunk > 32)
        return fail(SWEPT_EINVAL, "swept_set_batch_schedule: chunk %d outside [0, 32]", chunk);
    if (spin_limit > (int64_t(1) << 40))
        return fail(SWEPT_EINVAL, "swept_set_batch_schedule: spin_limit %lld us is too long",
                    (long long)spin_limit);
    if (queues < 0 || queues > 1024)
        return fail(SWEPT_EINVAL, "swept_set_batch_schedule: queues %d outside [0, 1024]",
                    queues);
    g_batch_sched = schedule;
    g_spin_limit = spin_limit;
    g_chunk = chunk;
    g_queues = queues;
    return SWEPT_OK;
}

const char* swept_last_error(void) { return g_err.c_str(); }

#ifdef SWEPT_COUNT_UPDATES
int swept_debug_update_count(uint64_t* count, int32_t reset)
{
    if (!g_ctx.ready)
        return fail(SWEPT_ENOTINIT, "swept_init has not been called");
    if (!count)
        return fail(SWEPT_EINVAL, "swept_debug_update_count: count is null");
    HIP_TRY(hipStreamSynchronize(g_ctx.stream));
    unsigned long long c = 0;
    HIP_TRY(hipMemcpyFromSymbol(&c, HIP_SYMBOL(g_update_count), sizeof c, 0,
                                hipMemcpyDeviceToHost));
    *count = (uint64_t)c;
    if (reset) {
        c = 0;
        HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(g_update_count), &c, sizeof c, 0,
                                  hipMemcpyHostToDevice));
    }
    return SWEPT_OK;
}
#endif

void swept_finalize(void)
{
    if (g_ctx.ready)
        (void)hipDeviceSynchronize();
    if (g_ctx.scratch)
        (void)hipFree(g_ctx.scratch);
    if (g_ctx.obj)
        (void)hipFree(g_ctx.obj);
    if (g_ctx.fault)
        (void)hipFree(g_ctx.fault);
    release_events();
    batch_release();
    swept_clear_tuning();
    g_batch_sched = SWEPT_BATCH_PERSISTENT;
    g_spin_limit = 0;
    g_chunk = 0;
    g_queues = 0;
    g_ctx = Context{};
}

}  // extern "C"
