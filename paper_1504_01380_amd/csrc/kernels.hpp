// kernels.hpp -- the "global code" of the swept rule on gfx950 (paper,
// Sections 3 and 5): which point advances which sub-timestep, where and when.
//
// Geometry of one stage.  A stage s is computed region by region; region t is
// owned by one workgroup (the paper's node).  With tile width W = 2k:
//   stage 0   (Section 3, 1st local computation): the triangle over tile
//             [tW, tW+W): levels 1..k-1 on [tW+l, tW+W-1-l].
//   stage s>0 (Section 3, 2nd and later local computations): the diamond
//             centred at J = tW + k + s*k with base level b = (s-1)k; at
//             relative level j (level b+j) it covers [J-j, J+j-1] for j <= k
//             and [J-2k+j, J+2k-1-j] for k < j < 2k.
// Every stage is capped at the target level L; points that reach level L are
// written to u.  The region of stage s+1 for workgroup t sits k points to the
// right of its stage-s region, so the V it needs is its own right leading
// edge (the "kept" edge, buffer RE) and the left leading edge of workgroup
// t+1 (the "sent" edge, buffer LE) -- the paper's rule of keeping one swept
// edge and receiving the other (Section 3, Fig. 3c/3e), with the tiles
// drifting right instead of alternating, which is the same schedule relabelled.
//
// Inside a region.  Rotated by 45 degrees a diamond is a k x k square of
// point pairs: pair d at step m (0 <= d, m < k) holds A at x = J+m-d and B at
// x-1, both at relative level m+d+1.  Its inputs are its own state at step
// m-1 and pair d-1 at step m; pair -1 is the right V edge, the state of pair
// d at step -1 is the left V edge at level d, pair k-1 traces the new left
// edge and the final states (m = k-1) are the new right edge.
//
// A wavefront sweeps this square in bands of 64*P pairs: lane r owns pairs
// e = rP..rP+P-1 of the band and pair e works on step m = tau - e at wave
// step tau.  At a given tau the whole band therefore sits on one level, a
// contiguous run of 128P points that slides up-right one point per level.
// Per wave step every lane updates its 2P points in registers and passes its
// last pair to the next lane with one DPP row shift per 32-bit word; lane 0
// receives pair -1 from LDS (the right V edge for the first band, the last
// pair of the previous band otherwise).  All points of a band are at the
// same sub-timestep, so multi-substep schemes need no divergence.
#pragma once

#include <type_traits>

#include "stencils.hpp"

namespace swept {

template <class S>
struct StageArgs {
    using Pt = typename S::Pt;
    typename S::T* u;        // the field, n points
    const Pt* re;            // [tiles][k][2]: kept right edge of stage s-1, own region only
    Pt* re_out;              // [tiles][k][2]: kept right edge of this stage (may equal re)
    const Pt* le_in;         // [tiles][k][2]: left edges written by stage s-1
    Pt* le_out;              // [tiles][k][2]: left edges of this stage
    int64_t n;               // grid points
    int64_t L;               // target level (sub-timesteps)
    int64_t b;               // base level of this stage: (s-1)k
    int64_t J0;              // centre of region 0: (k + s*k) mod n
    int k;                   // sweep depth; tile width W = 2k
    int tiles;               // n / W
    int tri;                 // 1 for stage 0
    typename S::Consts c;
    unsigned long long guard;  // call id of the range check (0: the canonical form only)
};

// The stencil a kernel runs once the call's range check has passed: the
// fused-Laplacian form of heat (HeatLap), which gives the canonical bits from
// fewer operations; void where there is none.
template <class S>
struct fused_form {
    using type = void;
};
template <>
struct fused_form<HeatF64> {
    using type = HeatLapF64;
};
template <>
struct fused_form<HeatF32> {
    using type = HeatLapF32;
};
template <class S>
constexpr bool has_fused_form = !std::is_void_v<typename fused_form<S>::type>;
// a stencil type as a value, for the kernels' generic lambdas
template <class S>
struct stencil_tag {
    using type = S;
};

// The largest call id whose initial field failed the range check, per
// device (calls are numbered from 1 by the host and only ever raise it).  A
// stage kernel of call `guard` takes the fused form while the mark is below
// its id: a call whose own check failed has raised the mark to at least its
// id (in an earlier launch on the same stream), so it never does.
__device__ unsigned long long g_form_mark;

__device__ __forceinline__ bool fused_ok(unsigned long long guard)
{
    return guard != 0 && g_form_mark < guard;
}

// The same decision for a batch, whose launch sequence is captured once and
// launched again with the same arguments: nonzero once the range check of
// the current launch found a heat instance out of range.  Each launch of the
// sequence clears it (batch_form_clear_kernel) and checks its heat instances
// (heat_range_batch_kernel) before their first region reads it.
__device__ int g_batch_form_bad;

__device__ __forceinline__ bool batch_fused_ok(int fusable)
{
    return fusable != 0 && g_batch_form_bad == 0;
}

// The range check of the fused heat form: any finite |u| above `bound`
// (a sixteenth of the largest finite value) marks the call.
template <class T>
__global__ __launch_bounds__(256) void heat_range_kernel(const T* __restrict__ u, int64_t n,
                                                         T bound, unsigned long long id)
{
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const T v = u[i];
        bad = bad || (__builtin_isfinite(v) && __builtin_fabs(v) > bound);
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0)
        atomicMax(&g_form_mark, id);
}

__device__ __forceinline__ int64_t wrapn(int64_t x, int64_t n)
{
    // callers keep x in (-n, 2n)
    return x < 0 ? x + n : (x >= n ? x - n : x);
}

template <int NPH>
__device__ __forceinline__ int phase_of(int64_t level)
{
    if constexpr (NPH == 1) {
        return 0;
    } else {
        const int64_t m = level % NPH;
        return int(m < 0 ? m + NPH : m);
    }
}

// A stencil may set kChainPrefetch = false: lane 0 then reads pair -1 from
// the LDS chain at the step that uses it instead of one step ahead, which
// frees the registers of two points (for every lane) where a wave step is
// long enough to cover the LDS latency.
template <class S, class = void>
struct chain_prefetch : std::true_type {};
template <class S>
struct chain_prefetch<S, std::void_t<decltype(S::kChainPrefetch)>>
    : std::integral_constant<bool, S::kChainPrefetch> {};

// A stencil may set kChainStore: the continuous kernel's last slot then
// stores into the LDS chain only the components of its pair that the next
// sub-timestep reads (S::chain_store<PH>), instead of the whole points.
template <class S, class = void>
struct has_chain_store : std::false_type {};
template <class S>
struct has_chain_store<S, std::void_t<decltype(S::kChainStore)>>
    : std::integral_constant<bool, S::kChainStore> {};

// A stencil may set kUnmaskedEnds: the continuous kernel's pipeline fill
// and drain then run unmasked (MASK 4 and 3 of cont_step): a slot computes
// before it has taken its first state and after it has stored its final
// one, which saves the per-pair masking where a step is long (KS).
// Otherwise a slot idles until its start and after its end, and all slots
// store at the end (MASK 1 and 2).
template <class S, class = void>
struct unmasked_ends : std::false_type {};
template <class S>
struct unmasked_ends<S, std::void_t<decltype(S::kUnmaskedEnds)>>
    : std::integral_constant<bool, S::kUnmaskedEnds> {};

// A stencil may set kFaces: its flux sub-timesteps then come as face fluxes
// (face_of, step_faces), and the continuous kernel computes each face once.
template <class S, class = void>
struct has_faces : std::false_type {};
template <class S>
struct has_faces<S, std::void_t<decltype(S::kFaces)>> : std::integral_constant<bool, S::kFaces> {};
struct NoFace {};
template <class S, bool = has_faces<S>::value>
struct face_type {
    using type = NoFace;
};
template <class S>
struct face_type<S, true> {
    using type = typename S::Face;
};
template <class S>
using face_t = typename face_type<S>::type;
template <class S, int PH>
constexpr bool face_phase()
{
    if constexpr (has_faces<S>::value)
        return S::template flux_phase<PH>;
    else
        return false;
}

// One wave step of a band: every active pair advances one level.  Pairs are
// visited from the last to the first so that pair q still reads pair q-1's
// state from the previous step.
// Debug build (SWEPT_COUNT_UPDATES): the stage kernels count every point
// update they compute, two per active pair and wave step, so that a test
// can check that a run computes each (point, sub-timestep level) once and no
// more -- the swept rule's "no redundant computation" (Section 3) -- on the
// GPU itself.  A no-op in the normal build.
#ifdef SWEPT_COUNT_UPDATES
__device__ unsigned long long g_update_count;
__device__ __forceinline__ void count_pairs(bool act)
{
    const unsigned long long m = __ballot(act);
    if ((threadIdx.x & 63) == 0)
        atomicAdd(&g_update_count, 2ull * (unsigned long long)__popcll(m));
}
#else
__device__ __forceinline__ void count_pairs(bool) {}
#endif

template <class S, int P, int PH>
__device__ __forceinline__ void band_update(typename S::Pt (&A)[P], typename S::Pt (&B)[P],
                                            const typename S::Pt& inA,
                                            const typename S::Pt& inB, int mlane, int elane,
                                            int nvalid, int k, const typename S::Consts& c)
{
    using Pt = typename S::Pt;
#pragma unroll
    for (int q = P - 1; q >= 0; --q) {
        const int m = mlane - q;
        const bool act = (unsigned)m < (unsigned)k && elane + q < nvalid;
        count_pairs(act);
        if (act) {
            const Pt rA = (q == 0) ? inA : A[q - 1];
            const Pt cB = (q == 0) ? inB : B[q - 1];
            const Pt nA = S::template step<PH>(A[q], cB, rA, c);
            const Pt nB = S::template step<PH>(B[q], A[q], cB, c);
            A[q] = nA;
            B[q] = nB;
        }
    }
}

// One region on the banded schedule.  The region is kp pairs by ks steps
// (kp = ks for equal tiles; tiles of unequal width make it rectangular):
// pair d at step m holds A at x = J+m-d and B at x-1, level b+m+d+1.  Inputs:
// re[2d], re[2d+1] = (B, A) of pair d at step -1 (the left V edge) and
// le_in[2m], le_in[2m+1] = pair -1 at step m (the right V edge); for the
// triangle (tri) the pairs start from level 0 of u instead.  Outputs: the
// final state of every pair (re_out, the new right edge) and the last
// pair's state at every step (le_out, the new left edge); points that reach
// level L are written to u.  chain is 2*ks points of LDS.
// An edge value another workgroup may have written in the same launch.
// COH (the persistent batch on XCD-local queues): a device-scope load, which
// skips this CU's L1 (it may hold the value from an earlier region) and is
// served by the XCD's L2, where the writer's stores land -- so the reader
// needs no cache invalidation.  Otherwise an ordinary load (a kernel
// boundary or an agent-scope acquire orders it).
template <class S, bool COH>
__device__ __forceinline__ typename S::Pt ld_edge(const typename S::Pt* p)
{
    if constexpr (!COH) {
        return *p;
    } else {
        using T = typename S::T;
        using Pt = typename S::Pt;
        static_assert(sizeof(Pt) % sizeof(T) == 0, "a point is a whole number of values");
        constexpr int NW = (int)(sizeof(Pt) / sizeof(T));
        Pt v;
        T* dst = reinterpret_cast<T*>(&v);
        const T* src = reinterpret_cast<const T*>(p);
#pragma unroll
        for (int i = 0; i < NW; ++i)
            dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return v;
    }
}

template <class S, int P, bool COH = false>
__device__ __forceinline__ void banded_region(typename S::T* u, const typename S::Pt* re,
                                              typename S::Pt* re_out,
                                              const typename S::Pt* le_in,
                                              typename S::Pt* le_out, typename S::Pt* chain,
                                              int64_t n, int64_t L, int64_t b, int64_t J, int kp,
                                              int ks, bool tri, const typename S::Consts& cst)
{
    using Pt = typename S::Pt;
    using T = typename S::T;
    const int lane = threadIdx.x;

    // right V edge of this region = left edge of the next tile's region of the previous stage
    if (!tri) {
        for (int i = lane; i < 2 * ks; i += 64)
            chain[i] = ld_edge<S, COH>(le_in + i);
    }
    __syncthreads();

    const int64_t top = L - b;  // highest relative level of this stage that is <= L

    for (int base = 0; base < kp; base += 64 * P) {
        const int nvalid = min(64 * P, kp - base);
        const int elane = lane * P;
        const int tau_first = tri ? (ks - base) : 0;
        const int64_t tau_cap = top - base - 1;  // wave step at which the band reaches level L
        const int64_t tau_end = min((int64_t)(nvalid + ks - 2), tau_cap);
        if (tau_end < tau_first && !tri)
            continue;  // the whole band lies above level L (a triangle band
                       // with no step still hands on its level-0 edges)

        Pt A[P], B[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int d = base + elane + q;
            if (elane + q < nvalid) {
                if (tri) {    // level 0 of the tile: pair d starts at step ks-1-d
                    const int64_t xa = J + ks - 1 - 2 * (int64_t)d;
                    A[q] = S::from_field(u[xa]);
                    B[q] = S::from_field(u[xa - 1]);
                } else {      // left V edge at relative level d
                    B[q] = ld_edge<S, COH>(re + 2 * d);
                    A[q] = ld_edge<S, COH>(re + 2 * d + 1);
                }
            } else {
                A[q] = S::from_field(T{});
                B[q] = S::from_field(T{});
            }
        }

        const int eL = nvalid - 1;       // last valid pair of the band
        const int rL = eL / P, qL = eL - rL * P;
        if (tri && lane == rL) {         // its level-0 state is part of the new left edge
#pragma unroll
            for (int q = 0; q < P; ++q)
                if (q == qL) {
                    const int m = ks - 1 - (base + eL);
                    chain[2 * m] = B[q];
                    chain[2 * m + 1] = A[q];
                }
        }

        int slot = min(tau_first, ks - 1);
        Pt cA = chain[2 * slot + 1], cB = chain[2 * slot];
        const int mbase = -elane;
        // one wave step at sub-timestep phase PH
        auto wave_step = [&](int tau, auto phc) {
            constexpr int PH = decltype(phc)::value;
            Pt inA, inB, nA, nB;
            if constexpr (chain_prefetch<S>::value) {
                inA = S::shr1(A[P - 1], cA);
                inB = S::shr1(B[P - 1], cB);
                const int nslot = min(tau + 1, ks - 1);  // prefetch pair -1 for the next step
                nA = chain[2 * nslot + 1];
                nB = chain[2 * nslot];
            } else {
                const int cslot = min(tau, ks - 1);
                inA = S::shr1(A[P - 1], chain[2 * cslot + 1]);
                inB = S::shr1(B[P - 1], chain[2 * cslot]);
            }
            const int mlane = tau + mbase;
            band_update<S, P, PH>(A, B, inA, inB, mlane, elane, nvalid, ks, cst);
            if (tau == tau_cap) {  // the band is at level L: write it out
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const int m = mlane - q;
                    if ((unsigned)m < (unsigned)ks && elane + q < nvalid) {
                        const int d = base + elane + q;
                        const int64_t xa = wrapn(J + m - d, n);
                        u[xa] = S::to_field(A[q]);
                        u[xa == 0 ? n - 1 : xa - 1] = S::to_field(B[q]);
                    }
                }
            }
            if (lane == rL) {      // the last pair traces the band's left edge
#pragma unroll
                for (int q = 0; q < P; ++q)
                    if (q == qL) {
                        const int m = tau - eL;
                        if ((unsigned)m < (unsigned)ks) {
                            chain[2 * m] = B[q];
                            chain[2 * m + 1] = A[q];
                        }
                    }
            }
            if constexpr (chain_prefetch<S>::value) {
                cA = nA;
                cB = nB;
            }
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        int tau = tau_first;
        const int tend = (int)tau_end;
        if constexpr (S::NPHASE == 1) {
            for (; tau <= tend; ++tau)
                wave_step(tau, I0{});
        } else {
            static_assert(S::NPHASE == 4, "multi-phase stencils have four sub-timesteps");
            // the band sits on level b+base+tau+1 at step tau, so the phase of
            // step tau is (b+base+tau) mod 4: run whole RK2 steps with the
            // phase known at compile time, the partial ones around them by case
            auto any_step = [&](int tau) {
                switch (phase_of<S::NPHASE>(b + base + tau)) {
                case 0: wave_step(tau, I0{}); break;
                case 1: wave_step(tau, I1{}); break;
                case 2: wave_step(tau, I2{}); break;
                default: wave_step(tau, I3{}); break;
                }
            };
            for (; tau <= tend && phase_of<S::NPHASE>(b + base + tau) != 0; ++tau)
                any_step(tau);
            for (; tau + 3 <= tend; tau += 4) {
                wave_step(tau, I0{});
                wave_step(tau + 1, I1{});
                wave_step(tau + 2, I2{});
                wave_step(tau + 3, I3{});
            }
            for (; tau <= tend; ++tau)
                any_step(tau);
        }

        // final states = new right edge (levels above L are never read)
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int d = base + elane + q;
            if (elane + q < nvalid) {
                re_out[2 * d] = B[q];
                re_out[2 * d + 1] = A[q];
            }
        }
    }

    __syncthreads();
    for (int i = lane; i < 2 * ks; i += 64)
        le_out[i] = chain[i];
}

// Equal tiles: workgroup t, stage s; the region is k x k, centred at
// J = tW + k + s*k (the tiles drift right by k per stage).
template <class S, int P>
__global__ __launch_bounds__(64) void swept_stage_kernel(StageArgs<S> g)
{
    using Pt = typename S::Pt;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int t = blockIdx.x;
    const int k = g.k;
    const int tn = (t + 1 == g.tiles) ? 0 : t + 1;
    const int64_t J = wrapn((int64_t)t * (2 * (int64_t)k) + g.J0, g.n);
    auto run = [&](auto sx) {
        using SX = typename decltype(sx)::type;
        banded_region<SX, P>(g.u, g.re + (size_t)t * k * 2, g.re_out + (size_t)t * k * 2,
                             g.le_in + (size_t)tn * k * 2, g.le_out + (size_t)t * k * 2,
                             reinterpret_cast<Pt*>(smem_raw), g.n, g.L, g.b, J, k, k,
                             g.tri != 0, g.c);
    };
    if constexpr (has_fused_form<S>) {
        if (fused_ok(g.guard)) {
            run(stencil_tag<typename fused_form<S>::type>{});
            return;
        }
    }
    run(stencil_tag<S>{});
}

// ------------------------------------------------- continuous diamond stage
// The same diamond, for stages that lie entirely below the target level and
// whose k is a multiple of the band size 64*P.  Instead of draining and
// refilling the pipeline at every band, each of the wavefront's 64*P pair
// slots moves on to the next band as soon as it finishes the last step of
// the current one: slot e works on band (sigma-e) div k, step (sigma-e) mod k
// at wave step sigma.  A slot changes band at sigma = beta*k + e; it then
// stores its final state (right edge) and takes the next band's left-edge
// state, which it fetched from HBM one band earlier.  Only the first and the
// last 64P-1 wave steps of the whole stage have idle slots.  Because 64P and
// k are multiples of 4, all slots are at the same sub-timestep modulo 4.

// MASK: 0 = all slots active; 1 = pipeline fill (slot e active iff e <= j);
// 2 = pipeline drain (slot e active iff e > j); 3 = the drain unmasked:
// slot e has finished at step e, where it stores its final state, and from
// then on computes values that no active slot reads (slot e+1 reads slot
// e's state of the step before, its last one; a finished slot's values
// reach only slots that have finished too); 4 = the fill unmasked: slot e
// takes its first state at step e and computes before that values that no
// active slot reads (an active slot reads only lower slots, all active).
// QS >= 0: slot (rs, QS) stores its state before it computes (MASK 0, 3)
// and takes its next one (MASK 0, 4).
//
// Face sharing (stencils with kFaces, flux sub-timesteps).  Pair e's update
// needs three faces: F[e] between its B and A, G between its A and pair
// e-1's B, and pair e-1's F.  So F is computed for every pair first, from
// the states before the step, and reaches pair e+1 in the same lane or, for
// the last pair, the next lane by a DPP shift; slot 0 takes the face of
// pair -1 from the face chain.  The face chain holds the right V edge's
// faces at first; the last slot then leaves there the face of the chain
// entry it wrote one step before (fslot), which slot 0 reads k - 64P steps
// later, at the same sub-timestep.  Flux steps are the odd sub-timesteps
// and k, 64P are even, so a chain index m is a flux one for one parity of m
// only: entry m of the face chain sits at fch[m / 2].  A slot that changes
// band takes the face of its new state from Fn, computed before the
// cycle's head.
template <class S, int P, int PH, int MASK, int QS>
__device__ __forceinline__ void cont_step(typename S::Pt (&A)[P], typename S::Pt (&B)[P],
                                          typename S::Pt (&An)[P], typename S::Pt (&Bn)[P],
                                          typename S::Pt& cA, typename S::Pt& cB,
                                          typename S::Pt* chain, int lane, int j, int rs,
                                          int next_slot, int wslot, bool wlast,
                                          typename S::Pt* re_store,
                                          const typename S::Consts& c, face_t<S> (&Fn)[P],
                                          void* fch, int fslot, bool wmirror, int k)
{
    using Pt = typename S::Pt;
    if constexpr (face_phase<S, PH>()) {
        using Face = typename S::Face;
        static_assert(!chain_prefetch<S>::value, "face sharing reads the chain at its step");
        Face* fchain = static_cast<Face*>(fch);
        const Pt inB = S::shr1(B[P - 1], chain[2 * j]);
        Face F[P];
#pragma unroll
        for (int q = 0; q < P; ++q)
            F[q] = S::template face_of<PH>(B[q], A[q], c);
        const Face H0 = S::shr1(F[P - 1], fchain[j >> 1]);
        if (MASK != 1 && lane == 63)
            fchain[fslot >> 1] = F[P - 1];
#pragma unroll
        for (int q = P - 1; q >= 0; --q) {
            if (QS == q) {
                if (lane == rs) {
                    if constexpr (MASK != 4) {
                        re_store[0] = B[q];
                        re_store[1] = A[q];
                    }
                    if constexpr (MASK != 3) {
                        A[q] = An[q];
                        B[q] = Bn[q];
                        F[q] = Fn[q];
                    }
                }
            }
            const Pt cBq = (q == 0) ? inB : B[q - 1];
            bool act = true;
            if constexpr (MASK == 1)
                act = lane * P + q <= j;
            if constexpr (MASK == 2)
                act = lane * P + q > j;
            count_pairs(MASK == 3 ? lane * P + q > j : (MASK == 4 ? lane * P + q <= j : act));
            if (act) {
                const Face G = S::template face_of<PH>(A[q], cBq, c);
                const Face H = (q == 0) ? H0 : F[q - 1];
                B[q] = S::template step_faces<PH>(A[q], F[q], G, c);
                A[q] = S::template step_faces<PH>(cBq, G, H, c);
            }
        }
    } else {
        Pt inA, inB, nA, nB;
        if constexpr (chain_prefetch<S>::value) {
            inA = S::shr1(A[P - 1], cA);
            inB = S::shr1(B[P - 1], cB);
            nA = chain[2 * next_slot + 1];
            nB = chain[2 * next_slot];
        } else {   // slot 0 is at step j of its band: pair -1 of step j
            inA = S::shr1(A[P - 1], chain[2 * j + 1]);
            inB = S::shr1(B[P - 1], chain[2 * j]);
        }
#pragma unroll
        for (int q = P - 1; q >= 0; --q) {
            if (QS == q) {     // folded at compile time after unrolling
                if (lane == rs) {  // this slot enters the next band (MASK 3: ends)
                    if constexpr (MASK != 4) {
                        re_store[0] = B[q];
                        re_store[1] = A[q];
                    }
                    if constexpr (MASK != 3) {
                        A[q] = An[q];
                        B[q] = Bn[q];
                    }
                }
            }
            const Pt rA = (q == 0) ? inA : A[q - 1];
            const Pt cBq = (q == 0) ? inB : B[q - 1];
            bool act = true;
            if constexpr (MASK == 1)
                act = lane * P + q <= j;
            if constexpr (MASK == 2)
                act = lane * P + q > j;
            count_pairs(MASK == 3 ? lane * P + q > j : (MASK == 4 ? lane * P + q <= j : act));
            if (act) {
                B[q] = S::template step<PH>(B[q], A[q], cBq, c);
                A[q] = S::template step<PH>(A[q], cBq, rA, c);
            }
        }
        if constexpr (chain_prefetch<S>::value) {
            cA = nA;
            cB = nB;
        }
    }
    if (wlast && lane == 63) {  // the last slot traces the band's left edge
        if constexpr (has_chain_store<S>::value) {
            S::template chain_store<PH>(&chain[2 * wslot], &chain[2 * wslot + 1], B[P - 1],
                                        A[P - 1]);
            if (chain_prefetch<S>::value && wmirror)
                S::template chain_store<PH>(&chain[2 * k], &chain[2 * k + 1], B[P - 1],
                                            A[P - 1]);
        } else {
            chain[2 * wslot] = B[P - 1];
            chain[2 * wslot + 1] = A[P - 1];
            if (chain_prefetch<S>::value && wmirror) {
                chain[2 * k] = B[P - 1];
                chain[2 * k + 1] = A[P - 1];
            }
        }
    }
}

// Wave steps are issued in statically unrolled groups.  Every cycle starts at
// a step sigma = cyc*k with b + sigma = b mod 4 (k and 64P are multiples of
// 4), so inside a group the sub-timestep of step i is (PH0 + i) mod NPHASE
// with PH0 = b mod NPHASE, known at compile time.

// Head of a cycle, steps j = j0 .. j0+G-1 (G = max(P, NPHASE) divides 64P):
// step j = rs*P + QS is the one at which slot j changes band (cycles
// 1..nb-1), starts (the fill, cycle 0) or ends (the drain after the last
// band).
template <class S, int P, int PH0, int MASK, bool TRANS, int I, int G>
__device__ __forceinline__ void cont_head_group(int j0, int k, int nb, int cyc,
                                                typename S::Pt (&A)[P], typename S::Pt (&B)[P],
                                                typename S::Pt (&An)[P],
                                                typename S::Pt (&Bn)[P], typename S::Pt& cA,
                                                typename S::Pt& cB, typename S::Pt* chain,
                                                const typename S::Pt* re,
                                                typename S::Pt* re_out, int lane,
                                                const typename S::Consts& c,
                                                face_t<S> (&Fn)[P], void* fch)
{
    if constexpr (I < G) {
        constexpr int NB = 64 * P;
        constexpr int QS = I % P;
        constexpr int PH = (PH0 + I) % S::NPHASE;
        const int j = j0 + I;
        const int rs = j / P;
        const int next_slot = j + 1;   // entry k mirrors entry 0 (read at j = k - 1)
        // last slot: step m = sigma - (NB-1) mod k of its band (j < NB here,
        // so j + k - (NB-1) lies in [k - NB + 1, k])
        const int wraw = j + k - (NB - 1);
        const int wslot = wraw == k ? 0 : wraw;
        // it is active from step NB-1 of the fill to step NB-2 of the drain
        const bool wlast = (MASK == 1 || MASK == 4) ? (j == NB - 1)
                                                    : (MASK >= 2 ? (j < NB - 1) : true);
        typename S::Pt* re_store = nullptr;
        if constexpr (TRANS)
            re_store = re_out + 2 * ((cyc - 1) * NB + j);
        // the chain entry the last slot wrote one step before (j < 64P here)
        const int fslot = j + k - NB;
        cont_step<S, P, PH, MASK, (TRANS || MASK == 4) ? QS : -1>(A, B, An, Bn, cA, cB, chain,
                                                                 lane, j, rs,
                                                   next_slot, wslot, wlast, re_store, c, Fn, fch,
                                                   fslot, wraw == k, k);
        cont_head_group<S, P, PH0, MASK, TRANS, I + 1, G>(j0, k, nb, cyc, A, B, An, Bn, cA, cB,
                                                          chain, re, re_out, lane, c, Fn, fch);
    }
}

// Body of a cycle, steps j = j0 .. j0+U-1 with 64P <= j < k: no slot changes
// band and every slot is active.
template <class S, int P, int PH0, int I, int U>
__device__ __forceinline__ void cont_body_group(int j0, int k, typename S::Pt (&A)[P],
                                                typename S::Pt (&B)[P], typename S::Pt (&An)[P],
                                                typename S::Pt (&Bn)[P], typename S::Pt& cA,
                                                typename S::Pt& cB, typename S::Pt* chain,
                                                int lane, const typename S::Consts& c,
                                                face_t<S> (&Fn)[P], void* fch)
{
    if constexpr (I < U) {
        constexpr int NB = 64 * P;
        const int j = j0 + I;
        cont_step<S, P, (PH0 + I) % S::NPHASE, 0, -1>(A, B, An, Bn, cA, cB, chain, lane, j, 0,
                                                      j + 1, j - (NB - 1), true, nullptr, c,
                                                      Fn, fch, j - NB, false, k);
        cont_body_group<S, P, PH0, I + 1, U>(j0, k, A, B, An, Bn, cA, cB, chain, lane, c, Fn,
                                             fch);
    }
}

// Points of cont_region's LDS chain at depth k (the face chain not included):
// k entries of two, and for stencils that prefetch a copy of entry 0.
template <class S>
constexpr int64_t cont_chain_points(int64_t k)
{
    return 2 * k + (chain_prefetch<S>::value ? 2 : 0);
}

// One full diamond region (k x k pairs, every level below the target) on
// the continuous-band schedule.  re: the left V edge (pair d at step -1),
// read and then overwritten in place by re_out when they are the same
// buffer; le_in: the right V edge (pair -1 at step m); le_out: the new left
// edge; chain: k entries of two points in LDS (cont_chain_points), followed
// for stencils that prefetch by a copy of entry 0 as entry k, so that slot 0
// reads entry j + 1 at every step j without a wrap, and for stencils with
// kFaces by the face chain (k/2 faces).  PH0 = b mod NPHASE.
template <class S, int P, int PH0, bool COH = false>
__device__ __forceinline__ void cont_region(const typename S::Pt* re, typename S::Pt* re_out,
                                            const typename S::Pt* le_in, typename S::Pt* le_out,
                                            typename S::Pt* chain, int k,
                                            const typename S::Consts& cst)
{
    using Pt = typename S::Pt;
    constexpr int NB = 64 * P;
    constexpr int G = P > S::NPHASE ? P : S::NPHASE;  // head group: QS and phase static
    constexpr int U = 4;                               // body group; k - NB is a multiple of 4
    const int lane = threadIdx.x;
    const int nb = k / NB;
    for (int i = lane; i < 2 * k; i += 64)
        chain[i] = ld_edge<S, COH>(le_in + i);
    if (chain_prefetch<S>::value && lane < 2)
        chain[2 * k + lane] = ld_edge<S, COH>(le_in + lane);
    __syncthreads();
    void* fch = nullptr;
    face_t<S> Fn[P];
    if constexpr (has_faces<S>::value) {
        // faces of the right V edge: slot 0 meets pair -1 of step m at
        // sub-timestep (PH0 + m) mod 4, a flux one for m = 2i + 1 - PH0 mod 2
        using Face = typename S::Face;
        Face* fchain = reinterpret_cast<Face*>(chain + 2 * k);
        for (int i = lane; i < k / 2; i += 64) {
            const int m = 2 * i + ((PH0 + 1) & 1);
            fchain[i] = S::face_sel(chain[2 * m], chain[2 * m + 1], ((PH0 + m) & 3) == 3, cst);
        }
        fch = fchain;
        __syncthreads();
    }

    Pt A[P], B[P], An[P], Bn[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int e = lane * P + q;
        B[q] = ld_edge<S, COH>(re + 2 * e);
        A[q] = ld_edge<S, COH>(re + 2 * e + 1);
        if constexpr (unmasked_ends<S>::value) {  // taken at the slot's fill step
            An[q] = A[q];
            Bn[q] = B[q];
        } else if (nb > 1) {
            Bn[q] = ld_edge<S, COH>(re + 2 * (NB + e));
            An[q] = ld_edge<S, COH>(re + 2 * (NB + e) + 1);
        } else {
            An[q] = A[q];
            Bn[q] = B[q];
        }
    }
    Pt cA = chain[1], cB = chain[0];
    {   // the chain's address in a VGPR (an opaque per-lane zero, in units of
        // two points so the 16-byte alignment stays known): the per-step LDS
        // accesses then take their offsets from it instead of a copy of a
        // scalar address in every step
        int vz;
        asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
        chain += 2 * vz;
    }

    for (int cyc = 0;; ++cyc) {
        if (cyc == 0) {
            if constexpr (unmasked_ends<S>::value) {
                for (int j0 = 0; j0 < NB; j0 += G)
                    cont_head_group<S, P, PH0, 4, false, 0, G>(j0, k, nb, cyc, A, B, An, Bn, cA,
                                                               cB, chain, re, re_out, lane, cst,
                                                               Fn, fch);
                if (nb > 1) {   // every slot has started: band 1's left-edge states
#pragma unroll
                    for (int q = 0; q < P; ++q) {
                        const int e = lane * P + q;
                        Bn[q] = ld_edge<S, COH>(re + 2 * (NB + e));
                        An[q] = ld_edge<S, COH>(re + 2 * (NB + e) + 1);
                    }
                }
            } else {
                for (int j0 = 0; j0 < NB; j0 += G)
                    cont_head_group<S, P, PH0, 1, false, 0, G>(j0, k, nb, cyc, A, B, An, Bn, cA,
                                                               cB, chain, re, re_out, lane, cst,
                                                               Fn, fch);
            }
        } else if (cyc == nb) {
            if constexpr (unmasked_ends<S>::value) {  // each slot stores at its own step
                for (int j0 = 0; j0 < NB; j0 += G)
                    cont_head_group<S, P, PH0, 3, true, 0, G>(j0, k, nb, cyc, A, B, An, Bn, cA,
                                                              cB, chain, re, re_out, lane, cst,
                                                              Fn, fch);
            } else {
                for (int j0 = 0; j0 < NB; j0 += G)
                    cont_head_group<S, P, PH0, 2, false, 0, G>(j0, k, nb, cyc, A, B, An, Bn, cA,
                                                               cB, chain, re, re_out, lane, cst,
                                                               Fn, fch);
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const int e = lane * P + q;
                    re_out[2 * ((nb - 1) * NB + e)] = B[q];
                    re_out[2 * ((nb - 1) * NB + e) + 1] = A[q];
                }
            }
            break;
        } else {
            if constexpr (has_faces<S>::value) {
                // slot e takes its next state at cycle step e, sub-timestep
                // (PH0 + e) mod 4 (read only when that is a flux one)
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const int e = lane * P + q;
                    Fn[q] = S::face_sel(Bn[q], An[q], ((PH0 + e) & 3) == 3, cst);
                }
            }
            for (int j0 = 0; j0 < NB; j0 += G)
                cont_head_group<S, P, PH0, 0, true, 0, G>(j0, k, nb, cyc, A, B, An, Bn, cA, cB,
                                                          chain, re, re_out, lane, cst, Fn, fch);
            // every slot has entered band cyc: fetch band cyc+1's left-edge
            // states for all of them at once (used k - 64P steps or more
            // later, at the next cycle's head)
            if (cyc + 1 < nb) {
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const int e = lane * P + q;
                    Bn[q] = ld_edge<S, COH>(re + 2 * ((cyc + 1) * NB + e));
                    An[q] = ld_edge<S, COH>(re + 2 * ((cyc + 1) * NB + e) + 1);
                }
            }
        }
        for (int j0 = NB; j0 < k; j0 += U)
            cont_body_group<S, P, PH0, 0, U>(j0, k, A, B, An, Bn, cA, cB, chain, lane, cst, Fn,
                                             fch);
    }

    __syncthreads();
    for (int i = lane; i < 2 * k; i += 64)
        le_out[i] = chain[i];
}

template <class S, int P>
__global__ __launch_bounds__(64) void swept_diamond_cont_kernel(StageArgs<S> g)
{
    using Pt = typename S::Pt;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int t = blockIdx.x;
    const int k = g.k;
    const int tn = (t + 1 == g.tiles) ? 0 : t + 1;
    auto run = [&](auto sx) {
        using SX = typename decltype(sx)::type;
        cont_region<SX, P, 0>(g.re + (size_t)t * k * 2, g.re_out + (size_t)t * k * 2,
                              g.le_in + (size_t)tn * k * 2, g.le_out + (size_t)t * k * 2,
                              reinterpret_cast<Pt*>(smem_raw), k, g.c);
    };
    if constexpr (has_fused_form<S>) {
        if (fused_ok(g.guard)) {
            run(stencil_tag<typename fused_form<S>::type>{});
            return;
        }
    }
    run(stencil_tag<S>{});
}

// ------------------------------------------------------------------ batch
// Many independent periodic instances, each tiled by even widths 2k_t that
// need not be equal (full tiles of k and one shorter tile the remainder, so
// any even length tiles).  Workgroup t of
// an instance keeps k_t pairs; at stage s its region is k_t pairs by
// k_{t+s} steps, centred at J = (X_{t+s} + X_{t+1})/2 with base level
// b = (X_{t+s} - X_{t+1})/2, where X_t = 2 sum_{t'<t} k_t' is extended
// periodically (X_{t+T} = X_t + n).  Stage 0 is each tile's triangle; every
// later region lies above level 0.  Right edges of tile t live at offset
// X_t of the instance's edge buffer, left edges at offset X_{(t+s) mod T}.
// A region between two full tiles is a k x k square; below the target level
// it runs on the continuous-band schedule (cont_region), the others on the
// banded one.

template <class S>
struct BatchInst {
    typename S::T* u;    // the instance's field (n points; the two-fold cover for odd rings)
    int64_t n, L;        // ring length, target level
    int64_t x_off;       // offset of X_0..X_T in the tile-boundary array
    int64_t e_off;       // offset of the instance's edges in the edge buffers (n points)
    int tiles;
    int tpos;            // persistent launch: index of tile 0 in the stencil's tile list
    typename S::Consts c;
};

struct BatchTask {
    int inst, tile;
};

template <class S>
struct BatchArgs {
    const BatchInst<S>* inst;
    const BatchTask* tasks;     // this stage's tasks are tasks[0 .. gridDim.x)
    const int64_t* X;           // tile boundaries, per instance X_0 = 0 .. X_T = n
    typename S::Pt* re;         // right edges, all instances
    typename S::Pt* le[2];      // left edges, by stage parity
    int stage;
    int fusable;                // heat: the batch's range check decides the form (0: canonical)
};

__global__ __launch_bounds__(64) void batch_form_clear_kernel()
{
    if (threadIdx.x == 0)
        g_batch_form_bad = 0;
}

// The fused heat form's range check over every instance of a batch's heat
// table (block row x: instance x; entries of other stencils have n = 0):
// any finite |u| above `bound` raises the batch's flag.
template <class S>
__global__ __launch_bounds__(256) void heat_range_batch_kernel(const BatchInst<S>* __restrict__ inst,
                                                               typename S::T bound)
{
    const typename S::T* u = inst[blockIdx.x].u;
    const int64_t n = inst[blockIdx.x].n;
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.y * 256;
    for (int64_t i = (int64_t)blockIdx.y * 256 + threadIdx.x; i < n; i += stride) {
        const typename S::T v = u[i];
        bad = bad || (__builtin_isfinite(v) && __builtin_fabs(v) > bound);
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0)
        __hip_atomic_store(&g_batch_form_bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Stage s of tile t of one ring of n points tiled at the even boundaries
// Xp(0) = 0 < Xp(1) < ... < Xp(T) = n, extended periodically
// (Xp(i + T) = Xp(i) + n).  re: the ring's right-edge buffer (tile t's
// entries at offset Xp(t)); le_in / le_out: its left-edge buffers of the
// previous and this stage parity (region i's entries at offset Xp(i)).
template <class S, int P, bool COH = false, class XF>
__device__ __forceinline__ void tiled_region(typename S::T* u, int64_t n, int64_t L, int T,
                                             const XF& Xp, int t, int s, typename S::Pt* re_ring,
                                             const typename S::Pt* le_in_ring,
                                             typename S::Pt* le_out_ring,
                                             const typename S::Consts& c,
                                             typename S::Pt* chain)
{
    using Pt = typename S::Pt;
    const int64_t xs = Xp((int64_t)t + s), x1 = Xp((int64_t)t + 1);
    const int64_t b = (xs - x1) / 2;
    if (s > 0 && b >= L)
        return;                  // this tile's regions are all above the target level
    const int kp = (int)((x1 - Xp(t)) / 2);
    const int i = (int)(((int64_t)t + s) % T);
    const int ks = (int)((Xp((int64_t)i + 1) - Xp(i)) / 2);
    const int64_t J = ((xs + x1) / 2) % n;
    Pt* re = re_ring + Xp(t);
    const Pt* le_in = le_in_ring + Xp(i);
    Pt* le_out = le_out_ring + Xp(i);
    if (s > 0 && kp == ks && kp % (64 * P) == 0 && b + 2 * (int64_t)kp - 1 < L) {
        // a full square diamond strictly below the target level: the
        // continuous-band schedule, whose cycles start at phase b mod NPHASE
        if constexpr (S::NPHASE == 1) {
            cont_region<S, P, 0, COH>(re, re, le_in, le_out, chain, kp, c);
        } else {
            static_assert(S::NPHASE == 4, "one or four sub-timesteps per step");
            switch ((int)(b % 4)) {
            case 0: cont_region<S, P, 0, COH>(re, re, le_in, le_out, chain, kp, c); break;
            case 1: cont_region<S, P, 1, COH>(re, re, le_in, le_out, chain, kp, c); break;
            case 2: cont_region<S, P, 2, COH>(re, re, le_in, le_out, chain, kp, c); break;
            default: cont_region<S, P, 3, COH>(re, re, le_in, le_out, chain, kp, c); break;
            }
        }
        return;
    }
    banded_region<S, P, COH>(u, re, re, le_in, le_out, chain, n, L, b, J, kp, ks, s == 0, c);
}

template <class S, int P>
__global__ __launch_bounds__(64) void swept_batch_kernel(BatchArgs<S> g)
{
    using Pt = typename S::Pt;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const BatchTask task = g.tasks[blockIdx.x];
    const BatchInst<S> I = g.inst[task.inst];
    const int64_t* X = g.X + I.x_off;
    const int T = I.tiles;
    const int64_t n = I.n;
    auto Xp = [&](int64_t i) { return X[i % T] + (i / T) * n; };
    auto run = [&](auto sx) {
        using SX = typename decltype(sx)::type;
        tiled_region<SX, P>(I.u, n, I.L, T, Xp, task.tile, g.stage, g.re + I.e_off,
                            g.le[(g.stage + 1) & 1] + I.e_off, g.le[g.stage & 1] + I.e_off, I.c,
                            reinterpret_cast<Pt*>(smem_raw));
    };
    if constexpr (has_fused_form<S>) {
        if (batch_fused_ok(g.fusable)) {
            run(stencil_tag<typename fused_form<S>::type>{});
            return;
        }
    }
    run(stencil_tag<S>{});
}

// ----------------------------------------------------- persistent batch
// One launch runs every stage of every instance of one stencil in a batch.
// Tiles synchronise pairwise, as the paper's nodes do (Section 3: a node's
// next stage needs only the edge it kept and the one its neighbour sent),
// instead of all at once at a kernel boundary.
// Its tasks (one region each) are numbered stage-major: all regions of stage
// 0, then all of stage 1, and so on; inside a stage in order of decreasing
// stage count of their instance (the longest instances start first).  A
// workgroup takes the next few numbers from a counter and, for each run of
// them inside one stage, waits until stage s-1 of every task's own tile and
// next tile have been published, runs the regions and publishes their tiles
// at stage s.  Every task that a claimed task waits for has a smaller
// number and belongs to an earlier stage, so a workgroup that is already
// running claimed it earlier and reaches it without waiting on anything
// later: by induction over the numbers, the waits end.  They are bounded
// all the same: after spin_ticks of waiting, or as soon as another
// workgroup has given up, a workgroup sets `fault` and leaves (the host
// reports a timeout).
//
// Those two waits give every ordering the stage-by-stage launches give.
// Region (t, s) reads and rewrites tile t's right edge, which (t, s-1)
// wrote; it reads the left edge at X_{t+s} of stage parity s-1, which
// (t+1, s-1) wrote, and writes the one of parity s at the same place, which
// only (t+1, s-1) reads.  Only stage 0 reads the field, and a region writes
// its final level into tiles whose stage 0 it depends on.
// The instances are split into `queues` independent schedules (balanced by
// work), each with its own tile list, stage offsets and counter.  Two ways
// to map workgroups to queues:
//  - XCD-local (XL): queue j is served only by the workgroups running on
//    XCD j (read from the hardware's XCC_ID register), so every region of an
//    instance runs under one L2.  A region's edges reach the other
//    workgroups of its queue once its stores have completed (the L1 is
//    write-through), and they read edges with device-scope loads, which skip
//    their own L1 (ld_edge): neither side touches the cache as a whole,
//    where an agent-scope release writes back, and an acquire invalidates,
//    the XCD's entire L2 at microseconds a time;
//  - otherwise workgroup w serves queue w mod queues, and the release and
//    acquire are at agent scope.
template <class S>
struct PersistArgs {
    using Pt = typename S::Pt;
    const BatchInst<S>* inst;
    const BatchTask* tasks;      // per queue, the tiles; instance by instance, most stages first
    const int64_t* toff;         // toff[j]: queue j's first entry in tasks
    const int64_t* first;        // first[j*(smax+1) + s]: number of queue j's first task of
                                 // stage s (within the queue); first[j*(smax+1) + smax] = its total
    const int64_t* X;            // tile boundaries, as for swept_batch_kernel
    Pt* re;
    Pt* le[2];
    int* done;                   // stages published, per tile (index tpos + t)
    unsigned* counter;           // queue j's next task number at counter[j * kCounterStride]
    int* fault;                  // set when a workgroup gives up waiting
    int smax;
    int queues;
    uint64_t spin_ticks;         // 100 MHz ticks after which a wait gives up
    int chunk;                   // task numbers taken per claim (1..32)
    int fusable;                 // as for swept_batch_kernel
};

// The XCD this wave runs on (XCC_ID register, low four bits).
__device__ __forceinline__ unsigned xcc_id()
{
    unsigned x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & 0xfu;
}

__global__ __launch_bounds__(64) void xcc_probe_kernel(int* __restrict__ out)
{
    if (threadIdx.x == 0)
        out[blockIdx.x] = (int)xcc_id();
}
constexpr int kCounterStride = 64;   // 256 bytes between the queues' counters

// Wait until every lane's *p >= want (lanes with p == nullptr have nothing
// to wait for); false if the wait gave up.  The bound is wall-clock time on
// the 100 MHz real-time counter.
__device__ __forceinline__ bool persist_wait(const int* p, int want, int* fault,
                                             uint64_t limit_ticks)
{
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        const bool ok =
            p == nullptr || __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want;
        if (__all(ok))
            return true;
        if (__hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            __builtin_amdgcn_s_memrealtime() - t0 > limit_ticks) {
            __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// SX: the stencil whose sub-timesteps the regions compute (S or its fused form)
template <class S, class SX, int P, bool XL>
__device__ __forceinline__ void batch_persistent(const PersistArgs<S>& g)
{
    using Pt = typename S::Pt;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x;
    const int j = XL ? (int)xcc_id() : (int)(blockIdx.x % (unsigned)g.queues);
    if (j >= g.queues) {     // an XCD the host's probe did not see: report, run nothing
        __hip_atomic_store(g.fault, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const BatchTask* tasks = g.tasks + g.toff[j];
    const int64_t* first = g.first + (int64_t)j * (g.smax + 1);
    unsigned* counter = g.counter + (int64_t)j * kCounterStride;
    const int64_t total = first[g.smax];
    int s = 0;    // this workgroup's stage; its task numbers only grow
    for (;;) {
        // claim `chunk` (<= 32) consecutive numbers; each run of them inside
        // one stage waits for all its inputs (lane 2i: task i's own tile,
        // lane 2i+1: its next tile) with one acquire, then runs them and
        // publishes each (XL) or the whole run (one agent release)
        unsigned q0 = 0;
        if (lane == 0)
            q0 = atomicAdd(counter, (unsigned)g.chunk);
        q0 = __builtin_amdgcn_readfirstlane(q0);
        if ((int64_t)q0 >= total)
            return;
        const int64_t qe = (int64_t)q0 + g.chunk < total ? (int64_t)q0 + g.chunk : total;
        for (int64_t q = q0; q < qe;) {
            while (first[s + 1] <= q)
                ++s;
            const int64_t qs = qe < first[s + 1] ? qe : first[s + 1];
            // the flag of lane 2i + side: task q+i's own tile (side 0) or next tile
            int* flag = nullptr;
            if (lane < 2 * (qs - q)) {
                const BatchTask task = tasks[q + (lane >> 1) - first[s]];
                const int tpos = g.inst[task.inst].tpos, T = g.inst[task.inst].tiles;
                const int t = (lane & 1) ? (task.tile + 1 == T ? 0 : task.tile + 1) : task.tile;
                flag = g.done + tpos + t;
            }
            if (s > 0) {
                if (!persist_wait(flag, s, g.fault, g.spin_ticks))
                    return;
                if constexpr (XL)    // the edges are read with device-scope loads;
                    asm volatile("" ::: "memory");   // keep them after the wait
                else
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            for (int64_t x = q; x < qs; ++x) {
                const BatchTask task = tasks[x - first[s]];
                const BatchInst<S> I = g.inst[task.inst];
                const int T = I.tiles;
                const int64_t* X = g.X + I.x_off;
                const int64_t n = I.n;
                auto Xp = [&](int64_t i) { return X[i % T] + (i / T) * n; };
                tiled_region<SX, P, XL>(I.u, n, I.L, T, Xp, task.tile, s, g.re + I.e_off,
                                       g.le[(s + 1) & 1] + I.e_off, g.le[s & 1] + I.e_off, I.c,
                                       reinterpret_cast<Pt*>(smem_raw));
                if constexpr (XL) {
                    // publish at once: the release is only this wave's
                    // stores reaching the shared L2
                    __syncthreads();
                    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                    if (lane == 2 * (x - q))
                        __hip_atomic_store(flag, s + 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            if constexpr (!XL) {
                // one agent-scope release (an L2 write-back) for the whole run
                __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                if (flag != nullptr && (lane & 1) == 0)
                    __hip_atomic_store(flag, s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            q = qs;
        }
    }
}

// The task loop keeps a few more values live than one region does; the
// bounds hold each stencil to the occupancy its regions reach anyway: heat
// 8 waves per SIMD (its LDS chain allows more), KS 3 (at depth 256 its LDS
// chain of 24-byte points fits 13 workgroups per CU).
template <class S, int P, bool XL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(S::kPersistWaves)))
void swept_batch_persistent_kernel(PersistArgs<S> g)
{
    if constexpr (has_fused_form<S>) {
        if (batch_fused_ok(g.fusable)) {
            batch_persistent<S, typename fused_form<S>::type, P, XL>(g);
            return;
        }
    }
    batch_persistent<S, S, P, XL>(g);
}

// After a persistent launch: every queue must have handed out all its task
// numbers (a queue that no workgroup served would leave its instances
// unfinished); fault = 2 otherwise, unless a wait already gave up (1).
__global__ __launch_bounds__(64) void persist_check_kernel(const unsigned* __restrict__ counter,
                                                           const int64_t* __restrict__ first,
                                                           int smax, int queues,
                                                           int* __restrict__ fault)
{
    for (int j = threadIdx.x; j < queues; j += blockDim.x)
        if ((int64_t)counter[(int64_t)j * kCounterStride] < first[(int64_t)j * (smax + 1) + smax])
            atomicCAS(fault, 0, 2);
}

// Zero the stage flags and the queues' counters before a persistent launch.
__global__ __launch_bounds__(256) void persist_clear_kernel(int* __restrict__ done, int64_t n,
                                                            unsigned* __restrict__ counter,
                                                            int queues)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < n; i += stride)
        done[i] = 0;
    for (int64_t j = i0; j < queues; j += stride)
        counter[j * kCounterStride] = 0;
}

// One field on the same tiling, its boundaries computed instead of read from a
// table: T - 1 tiles of 2k points and a last one of the remainder,
// X_t = 2kt for t < T and X_T = n.  Workgroup t runs tile t.
template <class S>
struct RaggedArgs {
    using Pt = typename S::Pt;
    typename S::T* u;        // the field (n points; the two-fold cover for an odd field)
    Pt* re;                  // right edges, n points
    Pt* le[2];               // left edges by stage parity, n points each
    int64_t n, L;
    int k, tiles, stage;
    typename S::Consts c;
    unsigned long long guard;  // call id of the range check (0: the canonical form only)
};

template <class S, int P>
__global__ __launch_bounds__(64) void swept_ragged_kernel(RaggedArgs<S> g)
{
    using Pt = typename S::Pt;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int T = g.tiles;
    const int64_t n = g.n, w = 2 * (int64_t)g.k;
    auto Xp = [&](int64_t i) { return (i % T) * w + (i / T) * n; };
    auto run = [&](auto sx) {
        using SX = typename decltype(sx)::type;
        tiled_region<SX, P>(g.u, n, g.L, T, Xp, (int)blockIdx.x, g.stage, g.re,
                            g.le[(g.stage + 1) & 1], g.le[g.stage & 1], g.c,
                            reinterpret_cast<Pt*>(smem_raw));
    };
    if constexpr (has_fused_form<S>) {
        if (fused_ok(g.guard)) {
            run(stencil_tag<typename fused_form<S>::type>{});
            return;
        }
    }
    run(stencil_tag<S>{});
}

// The two-fold covers of a batch's odd rings in one launch: entry i copies
// dst[j] = src[j mod n] for j < copies * n, with kCoverBlocks workgroups per
// entry.
struct CoverEntry {
    const double* src;
    double* dst;
    int64_t n;
    int64_t copies;
};
constexpr int kCoverBlocks = 8;

__global__ __launch_bounds__(256) void batch_cover_all_kernel(const CoverEntry* __restrict__ tab,
                                                             int count)
{
    const int i = (int)(blockIdx.x / kCoverBlocks);
    if (i >= count)
        return;
    const CoverEntry e = tab[i];
    const int64_t total = e.copies * e.n;
    const int64_t stride = (int64_t)kCoverBlocks * blockDim.x;
    for (int64_t j = (int64_t)(blockIdx.x % kCoverBlocks) * blockDim.x + threadIdx.x; j < total;
         j += stride)
        e.dst[j] = e.src[j % e.n];
}

template <class S>
__global__ __launch_bounds__(256) void batch_cover_kernel(const typename S::T* __restrict__ src,
                                                         typename S::T* __restrict__ dst,
                                                         int64_t n, int copies)
{
    // dst[i] = src[i mod n] for i < copies * n
    const int64_t total = (int64_t)copies * n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
        dst[i] = src[i % n];
}

// ------------------------------------------------------------ swept adjoint
// The stages in reverse order, on the same regions as the forward pass
// (stage s, region t: centre J, base b, tile width 2k; relative level j
// spans [J-j, J+j-1] for j <= k and [J-2k+j, J+2k-1-j] above; stage 0 is the
// triangle, whose relative level k is level 0).  A region
//   1. recomputes its forward values from its checkpoint -- the V kept by the
//      forward pass for that stage (or u0 for the triangle);
//   2. takes from the later regions above it (stage s+1: centred at J-k and
//      J+k) the cotangents of their two outermost points and the forward
//      value of their outermost point, at each level of their lower half;
//   3. forms the cotangent of each of its points from the top level down,
//      each from the three cotangents of the level above and the forward
//      values of its level (seeded at the target level L, plus the objective
//      source at step levels in the window);
//   4. hands the same kind of data to the earlier regions below it, or, for
//      the triangle, writes the gradient with respect to u0.
//
// One wavefront per region, in a fixed frame: lane l holds column dx = l - o.
// The region and its V edges span dx in [-k-1, k]; o = k + 1 covers them for
// k <= 31.  For k = 32, o = 32 and the two outermost columns lie outside the
// wave; only row k reads them (the V edge of row k-1 on the way up, the later
// regions' cotangents of row k+1 on the way down), and there they enter the
// boundary lanes' DPP moves as the value a lane keeps when it has no source.
// Both sweeps keep one level per lane in registers and take the neighbours'
// values with one DPP wave shift per 32-bit word, so a level costs a few VALU
// operations and no LDS round trip.  Values that enter from outside the
// region -- the V edges on the way up, the later regions' cotangents on the
// way down -- each reach a column at two consecutive levels, so every lane
// holds its two in registers and selects them at those levels.  LDS keeps,
// per point, the one forward value the reverse sweep reads there (S::keep),
// with the later regions' forward halo at the ends of the upper levels.

template <class S>
struct AdjArgs {
    using Pt = typename S::Pt;
    using Ad = typename S::Ad;
    using Kept = typename S::Kept;
    const typename S::T* u0;   // initial field (triangle)
    typename S::T* grad;       // d J / d u0 (triangle)
    const typename S::T* cot;  // cotangent of the final field, or null
    const Pt* re_in;           // checkpoint: right edges of stage s-1 (own region)
    const Pt* le_in;           // checkpoint: left edges of stage s-1
    const Ad* ae_in;           // from stage s+1: [tiles][2 sides][k][2] cotangents
    const Kept* fh_in;         // from stage s+1: [tiles][2 sides][k] kept forward values
    Ad* ae_out;                // to stage s-1
    Kept* fh_out;
    int64_t n, L, b, J0;
    int64_t win_first;         // first time step of the objective window
    typename S::T two_w;       // 2 * objective weight
    int k, tiles, tri, has_later;
    typename S::Consts c;
};

// LDS layout of a region's forward values.  Row j (relative level) holds the
// columns the reverse sweep reads, dx in [-j-2, j+1] below the middle level
// (the V edges sit at -j-2, -j-1, j, j+1) and [j-2k-1, 2k-j] from it up (the
// later regions' forward halo at both ends): 2k^2 + 6k + 2 values, the
// k^2 + 3k rows below the middle level first.
struct AdjLayout {
    int k;
    __device__ __forceinline__ int frow(int j) const
    {
        return j < k ? j * j + 3 * j : k * k + 3 * k + (j - k) * (3 * k + 3 - j);
    }
    __device__ __forceinline__ int lo(int j) const { return j < k ? -j - 2 : j - 2 * k - 1; }
    __device__ __forceinline__ int fidx(int j, int dx) const { return frow(j) + dx - lo(j); }
    __device__ __forceinline__ int fsize() const { return 2 * k * k + 6 * k + 2; }
    __device__ __forceinline__ int lower_size() const { return k * k + 3 * k; }
    // the same per half, without a branch: index of (j, dx) = base + dx
    template <bool UP>
    __device__ __forceinline__ int lo_h(int j) const { return UP ? j - 2 * k - 1 : -j - 2; }
    template <bool UP>
    __device__ __forceinline__ int hi_h(int j) const { return UP ? 2 * k - j : j + 1; }
    template <bool UP>
    __device__ __forceinline__ int base_h(int j) const
    {
        return UP ? k * k + 3 * k + (j - k) * (3 * k + 3 - j) - (j - 2 * k - 1) : j * j + 4 * j + 2;
    }
};

// lane frame: lane l holds column l - adj_frame(k)
__device__ __forceinline__ int adj_frame(int k) { return k + 1 < 32 ? k + 1 : 32; }

// DPP wave shifts of a whole record, one v_mov_b32_dpp per 32-bit word:
// kWaveShr1 -- lane i receives lane i-1; kWaveShl1 -- lane i receives lane
// i+1.  dpp_record: the lane with no source receives 0; dpp_record_keep: it
// receives `old`.
constexpr int kWaveShl1 = 0x130;
constexpr int kWaveShr1 = 0x138;
template <int CTRL, class V>
__device__ __forceinline__ V dpp_record(const V& src)
{
    static_assert(sizeof(V) % 4 == 0, "records of 32-bit words");
    constexpr int NW = (int)(sizeof(V) / 4);
    int w[NW];
    __builtin_memcpy(w, &src, sizeof(V));
#pragma unroll
    for (int i = 0; i < NW; ++i)
        w[i] = __builtin_amdgcn_mov_dpp(w[i], CTRL, 0xF, 0xF, true);
    V out;
    __builtin_memcpy(&out, w, sizeof(V));
    return out;
}
template <int CTRL, class V>
__device__ __forceinline__ V dpp_record_keep(const V& src, const V& old)
{
    static_assert(sizeof(V) % 4 == 0, "records of 32-bit words");
    constexpr int NW = (int)(sizeof(V) / 4);
    int w[NW], o[NW];
    __builtin_memcpy(w, &src, sizeof(V));
    __builtin_memcpy(o, &old, sizeof(V));
#pragma unroll
    for (int i = 0; i < NW; ++i)
        w[i] = __builtin_amdgcn_update_dpp(o[i], w[i], CTRL, 0xF, 0xF, false);
    V out;
    __builtin_memcpy(&out, w, sizeof(V));
    return out;
}

// c ? x : y for a whole record, word by word (a select between the records
// themselves would make the compiler keep them in scratch memory).
template <class V>
__device__ __forceinline__ V pick(bool c, const V& x, const V& y)
{
    constexpr int NW = (int)(sizeof(V) / 4);
    int wx[NW], wy[NW];
    __builtin_memcpy(wx, &x, sizeof(V));
    __builtin_memcpy(wy, &y, sizeof(V));
#pragma unroll
    for (int i = 0; i < NW; ++i)
        wx[i] = c ? wx[i] : wy[i];
    V out;
    __builtin_memcpy(&out, wx, sizeof(V));
    return out;
}

template <int N>
using Phase = std::integral_constant<int, N>;

// fn(j, Phase<p>) for j = j_first, j_first+1, ..., j_last with
// p = phase_of(base + j): single levels until the phase is 0, then groups of
// NPHASE levels whose phases are compile-time constants, then single levels.
template <int NPH, class Fn>
__device__ __forceinline__ void levels_up(int64_t base, int j_first, int j_last, Fn&& fn)
{
    static_assert(NPH == 1 || NPH == 4, "one or four sub-timesteps per step");
    int j = j_first;
    if constexpr (NPH == 1) {
        for (; j <= j_last; ++j)
            fn(j, Phase<0>{});
    } else {
        auto one = [&](int jj) {
            switch (phase_of<4>(base + jj)) {
            case 0: fn(jj, Phase<0>{}); break;
            case 1: fn(jj, Phase<1>{}); break;
            case 2: fn(jj, Phase<2>{}); break;
            default: fn(jj, Phase<3>{}); break;
            }
        };
        for (; j <= j_last && phase_of<4>(base + j) != 0; ++j)
            one(j);
        for (; j + 3 <= j_last; j += 4) {
            fn(j, Phase<0>{});
            fn(j + 1, Phase<1>{});
            fn(j + 2, Phase<2>{});
            fn(j + 3, Phase<3>{});
        }
        for (; j <= j_last; ++j)
            one(j);
    }
}

// The same for j = j_first, j_first-1, ..., j_last (j_first >= j_last).
template <int NPH, class Fn>
__device__ __forceinline__ void levels_down(int64_t base, int j_first, int j_last, Fn&& fn)
{
    static_assert(NPH == 1 || NPH == 4, "one or four sub-timesteps per step");
    int j = j_first;
    if constexpr (NPH == 1) {
        for (; j >= j_last; --j)
            fn(j, Phase<0>{});
    } else {
        auto one = [&](int jj) {
            switch (phase_of<4>(base + jj)) {
            case 0: fn(jj, Phase<0>{}); break;
            case 1: fn(jj, Phase<1>{}); break;
            case 2: fn(jj, Phase<2>{}); break;
            default: fn(jj, Phase<3>{}); break;
            }
        };
        for (; j >= j_last && phase_of<4>(base + j) != 3; --j)
            one(j);
        for (; j - 3 >= j_last; j -= 4) {
            fn(j, Phase<3>{});
            fn(j - 1, Phase<2>{});
            fn(j - 2, Phase<1>{});
            fn(j - 3, Phase<0>{});
        }
        for (; j >= j_last; --j)
            one(j);
    }
}

// S::keep for a phase known at run time
template <class S>
__device__ __forceinline__ typename S::Kept keep_at(int64_t level, const typename S::Pt& p)
{
    if constexpr (S::NPHASE == 1) {
        return S::template keep<0>(p);
    } else {
        switch (phase_of<4>(level)) {
        case 0: return S::template keep<0>(p);
        case 1: return S::template keep<1>(p);
        case 2: return S::template keep<2>(p);
        default: return S::template keep<3>(p);
        }
    }
}

template <class S>
__global__ __launch_bounds__(64) void swept_adjoint_kernel(AdjArgs<S> g)
{
    using Pt = typename S::Pt;
    using Ad = typename S::Ad;
    using Kept = typename S::Kept;
    using T = typename S::T;
    constexpr int NPH = S::NPHASE;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int k = g.k;
    const AdjLayout ly{k};
    const int dx = (int)threadIdx.x - adj_frame(k);   // this lane's column
    const bool wide = adj_frame(k) == k;              // columns -k-1 and k outside the wave
    const int t = blockIdx.x;
    const int64_t n = g.n;
    const int64_t J = wrapn((int64_t)t * (2 * (int64_t)k) + g.J0, n);
    const int jtop = (int)min((int64_t)(2 * k - 1), g.L - g.b);
    const bool act_k = dx >= -k && dx <= k - 1;   // the middle level's points
    // LDS byte addresses in 32 bits: a per-row offset plus the lane's column
    constexpr unsigned KB = sizeof(Kept);
    unsigned char* const Fb = smem_raw;
    const unsigned dump_b = (unsigned)ly.fsize() * KB;   // a spare slot for lanes with nothing to store
    auto F = [&](int idx) -> Kept& { return *reinterpret_cast<Kept*>(Fb + (unsigned)idx * KB); };

    // 1. checkpoint, the later regions' data, and the forward recompute.
    // The V edge reaches this column at rows iA and iB: -dx-2 and -dx-1 on
    // the left (the kept right edge of the stage before), dx and dx-1 on the
    // right (the left edge of the next region of the stage before).  The
    // stored forward value of row j is the one read by the sub-timestep that
    // leaves level b + j.
    Pt v{}, eA{}, eB{}, oL{}, oR{};
    const int iA = dx < 0 ? -dx - 2 : dx, iB = dx < 0 ? -dx - 1 : dx - 1;
    int j0 = k;
    if (g.tri) {
        if (act_k) {
            v = S::from_field(g.u0[J + dx]);
            F(ly.fidx(k, dx)) = keep_at<S>(g.b + k, v);
        }
    } else {
        j0 = 0;
        const Pt* re = g.re_in + (size_t)t * k * 2;
        const int tn = (t + 1 == g.tiles) ? 0 : t + 1;
        const Pt* le = g.le_in + (size_t)tn * k * 2;
        if (iA >= 0 && iA < k)
            eA = dx < 0 ? re[2 * iA] : le[2 * iA];
        if (iB >= 0 && iB < k)
            eB = dx < 0 ? re[2 * iB + 1] : le[2 * iB + 1];
        if (wide) {   // columns -k-1 and k of row k-1
            oL = re[2 * (k - 1)];
            oR = le[2 * (k - 1) + 1];
        }
        v = pick(iA == 0, eA, eB);   // row 0 holds only edges
        if (dx >= -2 && dx <= 1)
            F(ly.fidx(0, dx)) = keep_at<S>(g.b, v);
    }
    if (g.has_later) {   // their relative level jj is our level jj + k
        const int tl = (t == 0) ? g.tiles - 1 : t - 1;
        const Kept* fhR = g.fh_in + ((size_t)tl * 2 + 1) * k;   // upper-left region, right side
        const Kept* fhL = g.fh_in + ((size_t)t * 2 + 0) * k;    // upper-right region, left side
        for (int jj = threadIdx.x; jj < k; jj += 64) {         // forward halo at their levels 0..k-1
            if (jj + k <= jtop) {
                F(ly.fidx(jj + k, -k + jj - 1)) = fhR[jj];
                F(ly.fidx(jj + k, k - jj)) = fhL[jj];
            }
        }
    }
    // (issued early) The later regions' cotangents reach this column at rows
    // rA and rB (their levels 1..k are our rows k+1..2k): dx+2k+2 and dx+2k+1
    // on the left (the upper-left region's right side), 2k-dx and 2k-dx+1 on
    // the right (the upper-right region's left side).
    Ad inA{}, inB{}, iL{}, iR{};
    const int rA = dx < 0 ? dx + 2 * k + 2 : 2 * k - dx;
    const int rB = dx < 0 ? dx + 2 * k + 1 : 2 * k - dx + 1;
    if (g.has_later) {
        const int tl = (t == 0) ? g.tiles - 1 : t - 1;
        const Ad* inl = g.ae_in + ((size_t)tl * 2 + 1) * k * 2;
        const Ad* inr = g.ae_in + ((size_t)t * 2 + 0) * k * 2;
        const Ad* in = dx < 0 ? inl : inr;
        if (rA > k && rA <= 2 * k)
            inA = in[2 * (rA - k - 1)];
        if (rB > k && rB <= 2 * k)
            inB = in[2 * (rB - k - 1) + 1];
        if (wide) {   // columns -k-1 and k of row k+1
            iL = inl[0];
            iR = inr[1];
        }
    }

    // rows below the middle: the V edge enters at rows iA and iB; every row
    // is stored with its edges (dx in [-j-2, j+1])
    levels_up<NPH>(g.b - 1, j0 + 1, min(k - 1, jtop), [&](int j, auto ph) {
        constexpr int PH = decltype(ph)::value;
        const Pt l = dpp_record<kWaveShr1>(v), r = dpp_record<kWaveShl1>(v);
        v = pick(iA == j, eA, pick(iB == j, eB, S::template step<PH>(l, v, r, g.c)));
        const bool in_row = (unsigned)(dx + j + 2) <= (unsigned)(2 * j + 3);
        const unsigned at = (unsigned)(ly.template base_h<false>(j) + dx) * KB;
        *reinterpret_cast<Kept*>(Fb + (in_row ? at : dump_b)) =
            S::template keep<(PH + 1) % NPH>(v);
    });
    // from the middle row up: only the region's own points are stored
    // (dx in [j-2k, 2k-1-j]; the ends of these rows hold the later regions'
    // forward halo).  The middle row of a diamond reads columns -k-1 and k.
    auto up_level = [&](int j, auto ph, auto outer) {
        constexpr int PH = decltype(ph)::value;
        Pt l, r;
        if constexpr (decltype(outer)::value) {
            l = dpp_record_keep<kWaveShr1>(v, oL);
            r = dpp_record_keep<kWaveShl1>(v, oR);
        } else {
            l = dpp_record<kWaveShr1>(v);
            r = dpp_record<kWaveShl1>(v);
        }
        v = S::template step<PH>(l, v, r, g.c);
        const bool own = (unsigned)(dx - (j - 2 * k)) <= (unsigned)(4 * k - 1 - 2 * j);
        const unsigned at = (unsigned)(ly.template base_h<true>(j) + dx) * KB;
        *reinterpret_cast<Kept*>(Fb + (own ? at : dump_b)) = S::template keep<(PH + 1) % NPH>(v);
    };
    if (!g.tri && jtop >= k)
        levels_up<NPH>(g.b - 1, k, k, [&](int j, auto ph) { up_level(j, ph, std::true_type{}); });
    levels_up<NPH>(g.b - 1, k + 1, jtop, [&](int j, auto ph) { up_level(j, ph, std::false_type{}); });
    __syncthreads();

    // 2. cotangents from the top level down
    Ad a = pick(rA == jtop + 1, inA, inB);
    // the cotangents this column hands down (rows 1..k): it is one of the
    // four outermost columns of rows -dx and 1-dx (left) or dx+1 and dx+2
    // (right); row cA's value is kept in capA, row cB's in capB
    const int cA = dx < 0 ? -dx : dx + 1, cB = cA + 1;
    Ad capA{}, capB{};
    const int jbot = g.tri ? k : 1;
    // the objective's source enters at step levels from row jw up
    const int jw = (int)max((int64_t)-1, min((int64_t)(2 * k + 1), g.win_first * NPH - g.b));
    // kept forward values of row j at dx-1, dx, dx+1, the column clamped
    // into the row for the lanes outside it (whose results are never used)
    auto fwd3 = [&](int j, auto up) {
        constexpr bool UP = decltype(up)::value;
        const int col = min(max(dx, ly.template lo_h<UP>(j) + 1), ly.template hi_h<UP>(j) - 1);
        return reinterpret_cast<const Kept*>(Fb + (unsigned)(ly.template base_h<UP>(j) + col - 1) * KB);
    };
    // one level: UP selects the layout half (rows >= k), MERGE takes the
    // later regions' cotangents (rows > k), otherwise the hand-down rows are
    // captured; OUTER (the middle row) reads columns -k-1 and k of row k+1
    auto level = [&](int j, auto ph, auto up, auto merge, auto outer) {
        constexpr int PH = decltype(ph)::value;
        const Kept* fr = fwd3(j, up);
        Ad al, ar;
        if constexpr (decltype(outer)::value) {
            al = dpp_record_keep<kWaveShr1>(a, iL);
            ar = dpp_record_keep<kWaveShl1>(a, iR);
        } else {
            al = dpp_record<kWaveShr1>(a);
            ar = dpp_record<kWaveShl1>(a);
        }
        Ad o = S::template adj<PH>(al, a, ar, fr[0], fr[1], fr[2], g.c);
        if (PH == 0 && j >= jw)
            o = S::source(o, fr[1], g.two_w);
        if constexpr (decltype(merge)::value) {
            a = pick(rA == j, inA, pick(rB == j, inB, o));
        } else {
            a = o;
            capA = pick(cA == j, a, capA);
            capB = pick(cB == j, a, capB);
        }
    };
    using Yes = std::true_type;
    using No = std::false_type;
    int jstart = jtop;
    if (g.b + jtop == g.L) {   // the target level: the seed
        const Kept* fr = jtop >= k ? fwd3(jtop, Yes{}) : fwd3(jtop, No{});
        T c0 = T(0);
        if (g.cot && (jtop <= k ? (dx >= -jtop && dx <= jtop - 1)
                                : (dx >= jtop - 2 * k && dx <= 2 * k - 1 - jtop)))
            c0 = g.cot[wrapn(J + dx, n)];
        const Ad o = S::seed(c0, g.two_w, fr[1], g.L / NPH >= g.win_first);
        if (jtop > k) {
            a = pick(rA == jtop, inA, pick(rB == jtop, inB, o));
        } else {
            a = o;
            capA = pick(cA == jtop, a, capA);
            capB = pick(cB == jtop, a, capB);
        }
        --jstart;
    }
    levels_down<NPH>(g.b, jstart, max(k + 1, jbot),
                     [&](int j, auto ph) { level(j, ph, Yes{}, Yes{}, No{}); });
    if (jstart >= k && k >= jbot)   // the middle row: upper layout, lower cotangent rule
        levels_down<NPH>(g.b, k, k, [&](int j, auto ph) { level(j, ph, Yes{}, No{}, Yes{}); });
    levels_down<NPH>(g.b, min(jstart, k - 1), jbot,
                     [&](int j, auto ph) { level(j, ph, No{}, No{}, No{}); });

    // 3. the gradient, or the hand-down to the earlier regions
    if (g.tri) {
        if (act_k)
            g.grad[J + dx] = S::grad(a);
        return;
    }
    Ad* aeLo = g.ae_out + ((size_t)t * 2 + 0) * k * 2;
    Ad* aeRo = g.ae_out + ((size_t)t * 2 + 1) * k * 2;
    auto hand_down = [&](int j, const Ad& val) {
        if (j < 1 || j > k || j > jtop)
            return;
        if (dx == -j) aeLo[2 * (j - 1)] = val;
        if (dx == -j + 1) aeLo[2 * (j - 1) + 1] = val;
        if (dx == j - 2) aeRo[2 * (j - 1)] = val;
        if (dx == j - 1) aeRo[2 * (j - 1) + 1] = val;
    };
    hand_down(cA, capA);
    hand_down(cB, capB);
    Kept* fhL = g.fh_out + ((size_t)t * 2 + 0) * k;
    Kept* fhR = g.fh_out + ((size_t)t * 2 + 1) * k;
    for (int j = threadIdx.x; j < k && j <= jtop; j += 64) {
        fhL[j] = F(ly.fidx(j, -j));
        fhR[j] = F(ly.fidx(j, j - 1));
    }
}

// One stage in the lane frame of the adjoint kernels (lane = column, k <= 32,
// neighbours by DPP): the region's levels row by row, with the same edge
// buffers and formats as the banded and continuous kernels -- the new V
// edges, the two outermost points on each side of rows k..2k-1.  A row is a
// handful of VALU operations on the critical path, against about two wave
// steps of the pair-banded schedule per level, so this is the kernel for
// regions that are latency-bound (few tiles).  FIELD: write the points that
// reach level L to g.u (the stage kernel of swept_advance); without it, g.u
// is only read, by the triangle (the forward pass of the swept adjoint,
// which keeps the edges of every stage as its checkpoint).  LDS holds the
// rows from the middle level up (the upper half of the adjoint layout).
// One row of the lane frame: every column advances one level from its
// neighbours in the lanes beside it.  A stencil with face fluxes computes,
// in a flux sub-timestep, the face to its right once and takes the face to
// its left from the lane before (lane 0's is never read: it lies outside
// the region on every row that comes here).
template <class S, int PH>
__device__ __forceinline__ typename S::Pt lane_row(const typename S::Pt& v,
                                                   const typename S::Consts& c)
{
    using Pt = typename S::Pt;
    if constexpr (face_phase<S, PH>()) {
        const Pt r = dpp_record<kWaveShl1>(v);
        const typename S::Face F = S::template face_of<PH>(v, r, c);
        return S::template step_faces<PH>(v, dpp_record<kWaveShr1>(F), F, c);
    } else {
        const Pt l = dpp_record<kWaveShr1>(v), r = dpp_record<kWaveShl1>(v);
        return S::template step<PH>(l, v, r, c);
    }
}

// SX: the stencil whose sub-timesteps the rows compute (S or its fused form)
template <class S, class SX, bool FIELD>
__device__ __forceinline__ void lane_stage(const StageArgs<S>& g)
{
    using Pt = typename S::Pt;
    constexpr int NPH = S::NPHASE;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int k = g.k;
    const AdjLayout ly{k};
    const int dx = (int)threadIdx.x - adj_frame(k);
    const bool wide = adj_frame(k) == k;
    const int t = blockIdx.x;
    const int64_t J = wrapn((int64_t)t * (2 * (int64_t)k) + g.J0, g.n);
    const int jtop = (int)min((int64_t)(2 * k - 1), g.L - g.b);
    constexpr unsigned PB = sizeof(Pt);
    unsigned char* const Fb = smem_raw;
    const int low = ly.lower_size();
    const unsigned dump_b = (unsigned)(ly.fsize() - low) * PB;
    auto U = [&](int j, int col) -> Pt& {
        return *reinterpret_cast<Pt*>(Fb + (unsigned)(ly.fidx(j, col) - low) * PB);
    };

    Pt v{}, eA{}, eB{}, oL{}, oR{};
    const int iA = dx < 0 ? -dx - 2 : dx, iB = dx < 0 ? -dx - 1 : dx - 1;
    int j0 = k;
    if (g.tri) {
        if (dx >= -k && dx <= k - 1) {
            v = S::from_field(g.u[J + dx]);
            U(k, dx) = v;
        }
    } else {
        j0 = 0;
        const Pt* re = g.re + (size_t)t * k * 2;
        const int tn = (t + 1 == g.tiles) ? 0 : t + 1;
        const Pt* le = g.le_in + (size_t)tn * k * 2;
        if (iA >= 0 && iA < k)
            eA = dx < 0 ? re[2 * iA] : le[2 * iA];
        if (iB >= 0 && iB < k)
            eB = dx < 0 ? re[2 * iB + 1] : le[2 * iB + 1];
        if (wide) {
            oL = re[2 * (k - 1)];
            oR = le[2 * (k - 1) + 1];
        }
        v = pick(iA == 0, eA, eB);
    }
    levels_up<NPH>(g.b - 1, j0 + 1, min(k - 1, jtop), [&](int j, auto ph) {
        constexpr int PH = decltype(ph)::value;
        v = pick(iA == j, eA, pick(iB == j, eB, lane_row<SX, PH>(v, g.c)));
    });
    auto up_level = [&](int j, auto ph, auto outer) {
        constexpr int PH = decltype(ph)::value;
        if constexpr (decltype(outer)::value) {   // k = 32: the outermost columns' neighbours
            const Pt l = dpp_record_keep<kWaveShr1>(v, oL);
            const Pt r = dpp_record_keep<kWaveShl1>(v, oR);
            v = SX::template step<PH>(l, v, r, g.c);
        } else {
            v = lane_row<SX, PH>(v, g.c);
        }
        const bool own = (unsigned)(dx - (j - 2 * k)) <= (unsigned)(4 * k - 1 - 2 * j);
        const unsigned at = (unsigned)(ly.template base_h<true>(j) + dx - low) * PB;
        *reinterpret_cast<Pt*>(Fb + (own ? at : dump_b)) = v;
    };
    if (!g.tri && jtop >= k)
        levels_up<NPH>(g.b - 1, k, k, [&](int j, auto ph) { up_level(j, ph, std::true_type{}); });
    levels_up<NPH>(g.b - 1, k + 1, jtop, [&](int j, auto ph) { up_level(j, ph, std::false_type{}); });
    if constexpr (FIELD) {
        // the top row reached is the target level: its points are the result
        const bool own = jtop <= k ? (dx >= -jtop && dx <= jtop - 1)
                                   : (dx >= jtop - 2 * k && dx <= 2 * k - 1 - jtop);
        if (g.b + jtop == g.L && jtop > j0 && own)
            g.u[wrapn(J + dx, g.n)] = S::to_field(v);
    }
    __syncthreads();
    Pt* re_out = g.re_out + (size_t)t * k * 2;
    Pt* le_out = g.le_out + (size_t)t * k * 2;
    for (int j = k + (int)threadIdx.x; j <= jtop; j += 64) {
        const int i = j - k;
        re_out[2 * i] = U(j, 2 * k - 2 - j);
        re_out[2 * i + 1] = U(j, 2 * k - 1 - j);
        le_out[2 * i] = U(j, j - 2 * k);
        le_out[2 * i + 1] = U(j, j - 2 * k + 1);
    }
}

template <class S, bool FIELD>
__global__ __launch_bounds__(64) void swept_lane_kernel(StageArgs<S> g)
{
    if constexpr (FIELD && has_fused_form<S>) {
        if (fused_ok(g.guard)) {
            lane_stage<S, typename fused_form<S>::type, FIELD>(g);
            return;
        }
    }
    lane_stage<S, S, FIELD>(g);
}

// Zero time steps: the gradient is the seed at level 0.
template <class S>
__global__ __launch_bounds__(256) void adjoint_seed_kernel(const typename S::T* __restrict__ u0,
                                                          const typename S::T* __restrict__ cot,
                                                          typename S::T* __restrict__ grad,
                                                          int64_t n, typename S::T two_w, int src)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        grad[i] = S::grad(S::seed(cot ? cot[i] : typename S::T(0), two_w,
                                  S::template keep<0>(S::from_field(u0[i])), src != 0));
}

// Naive adjoint (the straight decomposition run backwards): one launch per
// time step turns the cotangent of step j+1 into that of step j, from the
// forward field of step j kept by the forward pass.  A block of NB points
// recomputes the step's forward levels on a halo of 7 (KS: levels 4j..4j+3
// over [i0-7+l, i0+NB+7-l)), applies the transposed sub-timesteps 3, 2, 1, 0
// (each one point narrower), and adds the window source at the step level.
template <class S, int NB>
__global__ __launch_bounds__(NB) void naive_adjoint_kernel(const typename S::T* __restrict__ uj,
                                                          const typename S::T* __restrict__ ub_in,
                                                          typename S::T* __restrict__ ub_out,
                                                          int64_t n, typename S::Consts c,
                                                          typename S::T two_w, int src)
{
    using Pt = typename S::Pt;
    using Ad = typename S::Ad;
    using T = typename S::T;
    const int64_t i0 = (int64_t)blockIdx.x * NB;
    const int tid = threadIdx.x;
    auto at = [&](int64_t x) {
        x %= n;
        return x < 0 ? x + n : x;
    };
    auto cot = [&](int64_t x) { return S::seed(ub_in[at(x)], T(0), typename S::Kept{}, false); };
    if constexpr (S::NPHASE == 1) {
        const int64_t i = i0 + tid;
        if (i < n) {
            const Pt fl = S::from_field(uj[at(i - 1)]), fc = S::from_field(uj[i]),
                     fr = S::from_field(uj[at(i + 1)]);
            Ad a = S::template adj<0>(cot(i - 1), cot(i), cot(i + 1), S::template keep<0>(fl),
                                      S::template keep<0>(fc), S::template keep<0>(fr), c);
            if (src)
                a = S::source(a, S::template keep<0>(fc), two_w);
            ub_out[i] = S::grad(a);
        }
    } else {
        static_assert(S::NPHASE == 4, "one or four sub-timesteps");
        __shared__ Pt f0[NB + 14], f1[NB + 12], f2[NB + 10], f3[NB + 8];
        __shared__ Ad a4[NB + 8], a3[NB + 6], a2[NB + 4], a1[NB + 2];
        for (int j = tid; j < NB + 14; j += NB)
            f0[j] = S::from_field(uj[at(i0 - 7 + j)]);          // x = i0-7+j
        for (int j = tid; j < NB + 8; j += NB)
            a4[j] = cot(i0 - 4 + j);                            // x = i0-4+j
        __syncthreads();
        for (int j = tid; j < NB + 12; j += NB)                 // x = i0-6+j
            f1[j] = S::template step<0>(f0[j], f0[j + 1], f0[j + 2], c);
        __syncthreads();
        for (int j = tid; j < NB + 10; j += NB)                 // x = i0-5+j
            f2[j] = S::template step<1>(f1[j], f1[j + 1], f1[j + 2], c);
        __syncthreads();
        for (int j = tid; j < NB + 8; j += NB)                  // x = i0-4+j
            f3[j] = S::template step<2>(f2[j], f2[j + 1], f2[j + 2], c);
        __syncthreads();
        for (int j = tid; j < NB + 6; j += NB)                  // x = i0-3+j
            a3[j] = S::template adj<3>(a4[j], a4[j + 1], a4[j + 2], S::template keep<3>(f3[j]),
                                       S::template keep<3>(f3[j + 1]), S::template keep<3>(f3[j + 2]), c);
        __syncthreads();
        for (int j = tid; j < NB + 4; j += NB)                  // x = i0-2+j
            a2[j] = S::template adj<2>(a3[j], a3[j + 1], a3[j + 2], S::template keep<2>(f2[j + 2]),
                                       S::template keep<2>(f2[j + 3]), S::template keep<2>(f2[j + 4]), c);
        __syncthreads();
        for (int j = tid; j < NB + 2; j += NB)                  // x = i0-1+j
            a1[j] = S::template adj<1>(a2[j], a2[j + 1], a2[j + 2], S::template keep<1>(f1[j + 4]),
                                       S::template keep<1>(f1[j + 5]), S::template keep<1>(f1[j + 6]), c);
        __syncthreads();
        const int64_t i = i0 + tid;                             // x = i0+tid
        if (i < n) {
            Ad a = S::template adj<0>(a1[tid], a1[tid + 1], a1[tid + 2], S::template keep<0>(f0[tid + 6]),
                                      S::template keep<0>(f0[tid + 7]), S::template keep<0>(f0[tid + 8]), c);
            if (src)
                a = S::source(a, S::template keep<0>(f0[tid + 7]), two_w);
            ub_out[i] = S::grad(a);
        }
    }
}

// ------------------------------------------------------------- naive paths
// The straight decomposition: every sub-timestep of every point, one launch
// per time step, from two full fields.

template <class S>
__global__ __launch_bounds__(256) void naive_step_kernel(const typename S::T* __restrict__ in,
                                                        typename S::T* __restrict__ out,
                                                        int64_t n, typename S::Consts c)
{
    static_assert(S::NPHASE == 1, "single-substep schemes only");
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t il = i == 0 ? n - 1 : i - 1;
        const int64_t ir = i == n - 1 ? 0 : i + 1;
        out[i] = S::to_field(S::template step<0>(S::from_field(in[il]), S::from_field(in[i]),
                                                 S::from_field(in[ir]), c));
    }
}

// The same step, V = 16 / sizeof(T) consecutive points per thread: one
// aligned 16-byte load and store of the thread's points plus its two outer
// neighbours (nx a multiple of V, 16-byte aligned fields).
template <class S>
__global__ __launch_bounds__(256) void naive_step_vec_kernel(const typename S::T* __restrict__ in,
                                                            typename S::T* __restrict__ out,
                                                            int64_t n, typename S::Consts c)
{
    static_assert(S::NPHASE == 1, "single-substep schemes only");
    using T = typename S::T;
    constexpr int V = 16 / sizeof(T);
    struct alignas(16) Vec {
        T v[V];
    };
    const int64_t nv = n / V;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        const Vec x = reinterpret_cast<const Vec*>(in)[i];
        const T l = in[i == 0 ? n - 1 : i * V - 1];
        const T r = in[i == nv - 1 ? 0 : i * V + V];
        Vec y;
#pragma unroll
        for (int q = 0; q < V; ++q) {
            const T xl = q == 0 ? l : x.v[q - 1];
            const T xr = q == V - 1 ? r : x.v[q + 1];
            y.v[q] = S::to_field(S::template step<0>(S::from_field(xl), S::from_field(x.v[q]),
                                                     S::from_field(xr), c));
        }
        reinterpret_cast<Vec*>(out)[i] = y;
    }
}

// Four-sub-timestep schemes (KS, Euler): one RK2 step in one launch.  Each
// block of NB points (NT threads) stages u on [i0-4, i0+NB+4) in LDS and
// recomputes the intermediate levels on its halo (the same per-point
// operations, so the same bits).  Measured on MI355X: NB = 1024 on 512
// threads for KS, 256 on 256 for Euler.
template <class S, int NB, int NT>
__device__ __forceinline__ void fused_block(const typename S::T* __restrict__ in,
                                            typename S::T* __restrict__ out, int64_t n,
                                            int64_t i0, const typename S::Consts& c)
{
    using Pt = typename S::Pt;
    static_assert(S::NPHASE == 4, "four-substep schemes only");
    // NB points on NT threads; the levels alternate between two buffers:
    // level l of the step holds points i0-4+l+j at index j
    __shared__ Pt b0[NB + 8], b1[NB + 8];
    const int tid = threadIdx.x;
    for (int j = tid; j < NB + 8; j += NT) {
        int64_t x = (i0 - 4 + j) % n;
        if (x < 0) x += n;
        b0[j] = S::from_field(in[x]);
    }
    __syncthreads();
    for (int j = tid; j < NB + 6; j += NT)
        b1[j] = S::template step<0>(b0[j], b0[j + 1], b0[j + 2], c);
    __syncthreads();
    for (int j = tid; j < NB + 4; j += NT)
        b0[j] = S::template step<1>(b1[j], b1[j + 1], b1[j + 2], c);
    __syncthreads();
    for (int j = tid; j < NB + 2; j += NT)
        b1[j] = S::template step<2>(b0[j], b0[j + 1], b0[j + 2], c);
    __syncthreads();
    for (int j = tid; j < NB; j += NT) {
        const int64_t i = i0 + j;
        if (i < n)
            out[i] = S::to_field(S::template step<3>(b1[j], b1[j + 1], b1[j + 2], c));
    }
}

template <class S, int NB, int NT>
__global__ __launch_bounds__(NT) void naive_fused_kernel(const typename S::T* __restrict__ in,
                                                        typename S::T* __restrict__ out,
                                                        int64_t n, typename S::Consts c)
{
    fused_block<S, NB, NT>(in, out, n, (int64_t)blockIdx.x * NB, c);
}

// Naive batch: one launch per time step advances every block of NB points
// (heat: NB = 4 x 256, four points per thread; KS: NB = 256, the fused step
// above) of every instance that still has steps to go.  Blocks never
// straddle two instances; an instance's field alternates between buf[0] and
// buf[1].  A block's record holds all it needs besides the constants, so its
// loads of field values wait on one table read only.
template <class S>
struct NaiveInst {
    typename S::Consts c;
};

template <class S>
struct NaiveBlock {
    typename S::T* buf[2];
    int64_t n, x0;
    int64_t inst;
};

template <class S, int NB>
__global__ __launch_bounds__(256) void naive_batch_kernel(const NaiveInst<S>* __restrict__ inst,
                                                         const NaiveBlock<S>* __restrict__ blocks,
                                                         int parity)
{
    const NaiveBlock<S> bk = blocks[blockIdx.x];
    const typename S::Consts c = inst[bk.inst].c;
    // a select, not bk.buf[parity]: an indexed record would live in memory
    const typename S::T* in = parity ? bk.buf[1] : bk.buf[0];
    typename S::T* out = parity ? bk.buf[0] : bk.buf[1];
    if constexpr (S::NPHASE == 1) {
        static_assert(NB % 256 == 0, "whole points per thread");
        constexpr int PER = NB / 256;
        typename S::T v[PER];
        int64_t xs[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int64_t i = bk.x0 + threadIdx.x + 256 * q;
            xs[q] = i;
            if (i < bk.n) {
                const int64_t il = i == 0 ? bk.n - 1 : i - 1;
                const int64_t ir = i == bk.n - 1 ? 0 : i + 1;
                v[q] = S::to_field(S::template step<0>(S::from_field(in[il]), S::from_field(in[i]),
                                                       S::from_field(in[ir]), c));
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (xs[q] < bk.n)
                out[xs[q]] = v[q];
    } else {
        static_assert(NB == 256, "one point per thread");
        fused_block<S, NB, NB>(in, out, bk.n, bk.x0, c);
    }
}

// KS: one launch per sub-timestep (the paper's straight decomposition that
// communicates every sub-timestep).  Fields of per-point inputs Pt.
template <class S, int PH>
__global__ __launch_bounds__(256) void naive_substep_kernel(const typename S::Pt* __restrict__ in,
                                                           typename S::Pt* __restrict__ out,
                                                           int64_t n, typename S::Consts c)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t il = i == 0 ? n - 1 : i - 1;
        const int64_t ir = i == n - 1 ? 0 : i + 1;
        out[i] = S::template step<PH>(in[il], in[i], in[ir], c);
    }
}

template <class S>
__global__ __launch_bounds__(256) void field_to_pt_kernel(const typename S::T* __restrict__ in,
                                                         typename S::Pt* __restrict__ out,
                                                         int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = S::from_field(in[i]);
}

template <class S>
__global__ __launch_bounds__(256) void pt_to_field_kernel(const typename S::Pt* __restrict__ in,
                                                         typename S::T* __restrict__ out,
                                                         int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = S::to_field(in[i]);
}

// ------------------------------------------------------------- objective
// The objective of the adjoint, J = w * sum over the window's steps of
// sum_i u_i^2 + sum_i c_i u_i^nsteps, summed on the device in a fixed order:
// a fixed grid of kObjBlocks blocks, each thread adding its points
// (i = tid, tid + stride, ...) in order, a fixed tree over the block, and a
// per-block (sum, compensation) pair that accumulates the successive calls
// by an error-free two-sum.  The result does not depend on timing and
// carries a few roundings of relative error, not one per step.
constexpr int kObjBlocks = 256;
constexpr int kObjThreads = 256;

__device__ __forceinline__ void two_sum_into(double* slot, double b)
{
    const double a = slot[0];
    const double t = a + b;
    const double bp = t - a;
    const double e = (a - (t - bp)) + (b - bp);
    slot[0] = t;
    slot[1] = slot[1] + e;
}

// acc[2*blockIdx.x .. +1] += sum_i x_i * y_i over this block's points
__global__ __launch_bounds__(kObjThreads) void objective_accumulate_kernel(
    const double* __restrict__ x, const double* __restrict__ y, int64_t n, double* acc)
{
    __shared__ double part[kObjThreads];
    const int64_t stride = (int64_t)kObjBlocks * kObjThreads;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kObjThreads + threadIdx.x; i < n; i += stride)
        s = s + x[i] * y[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kObjThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] = part[threadIdx.x] + part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        two_sum_into(acc + 2 * blockIdx.x, part[0]);
}

__global__ __launch_bounds__(256) void objective_clear_kernel(double* acc, int count)
{
    for (int i = threadIdx.x; i < count; i += blockDim.x)
        acc[i] = 0.0;
}

// J = w * (window sums) + (final cotangent term), each set of block slots
// combined in block order by the same two-sum
__global__ __launch_bounds__(64) void objective_final_kernel(const double* __restrict__ acc_sq,
                                                            const double* __restrict__ acc_dot,
                                                            double w, double* J)
{
    if (threadIdx.x != 0)
        return;
    double sq[2] = {0.0, 0.0}, dt[2] = {0.0, 0.0};
    for (int b = 0; b < kObjBlocks; ++b) {
        two_sum_into(sq, acc_sq[2 * b]);
        two_sum_into(sq, acc_sq[2 * b + 1]);
        two_sum_into(dt, acc_dot[2 * b]);
        two_sum_into(dt, acc_dot[2 * b + 1]);
    }
    J[0] = w * (sq[0] + sq[1]) + (dt[0] + dt[1]);
}

}  // namespace swept
