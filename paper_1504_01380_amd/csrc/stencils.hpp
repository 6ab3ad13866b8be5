// stencils.hpp -- the "local code" of the swept rule (paper, Section 5): what
// one sub-timestep does to one spatial point, given the inputs of the point
// and of its two neighbours (Section 2).  The global code (kernels.hpp) calls
// these in swept order and never looks inside.
//
// Every stencil S provides:
//   T        storage type of the field u
//   Pt       the per-point input variables of a sub-timestep
//   Consts   per-run constants, rounded once on the host
//   NPHASE   sub-timesteps per time step
//   step<PH>(L, C, R, k): the outputs at the centre point after sub-timestep
//            PH, from the inputs at its left, centre and right neighbours
//   from_field / to_field: Pt at a time-step boundary <-> field value
//   shr1(src, old): the Pt of lane i-1 in lane i, `old` in lane 0
//
// Arithmetic is written in the exact association the scheme defines and the
// library is compiled with -ffp-contract=off: no multiply-add is fused, so
// every path that evaluates these functions produces the same bits.  The
// contraction-on variants (HeatFma, KSFmaF64) fuse theirs explicitly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swept {

// DPP "wave_shr:1": lane i receives lane i-1's value; lane 0 keeps `old`
// (bound_ctrl off).  One v_mov_b32_dpp per 32-bit half.
__device__ __forceinline__ int dpp_shr1_i32(int src, int old)
{
    return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xF, 0xF, false);
}

__device__ __forceinline__ double dpp_shr1(double src, double old)
{
    const int lo = dpp_shr1_i32(__double2loint(src), __double2loint(old));
    const int hi = dpp_shr1_i32(__double2hiint(src), __double2hiint(old));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float dpp_shr1(float src, float old)
{
    return __int_as_float(dpp_shr1_i32(__float_as_int(src), __float_as_int(old)));
}

// ----------------------------------------------------------------- heat
// u_t = u_xx, 3-point forward Euler, one sub-timestep per step (paper,
// Section 4):  u' = u + r*((u[i-1] + u[i+1]) - 2u).
template <class TT>
struct Heat {
    using T = TT;
    struct Pt {
        T u;
    };
    struct Consts {
        T r;
    };
    static constexpr int NPHASE = 1;
    static constexpr int kPersistWaves = 8;   // waves per SIMD of the persistent batch kernel

    __device__ __forceinline__ static Pt from_field(T v) { return Pt{v}; }
    __device__ __forceinline__ static T to_field(const Pt& p) { return p.u; }
    __device__ __forceinline__ static Pt shr1(const Pt& s, const Pt& old)
    {
        return Pt{dpp_shr1(s.u, old.u)};
    }
    template <int PH>
    __device__ __forceinline__ static Pt step(const Pt& l, const Pt& c, const Pt& r,
                                              const Consts& k)
    {
        const T lap = (l.u + r.u) - T(2) * c.u;
        return Pt{c.u + k.r * lap};
    }

    // Discrete adjoint.  The heat step matrix is symmetric, so the cotangent
    // of a level is the same 3-point update applied to the cotangents of the
    // level above it.
    struct Ad {
        T u;
    };
    // the forward value the reverse sweep reads at a level (the objective's
    // source needs u; the update itself needs none)
    using Kept = T;
    template <int PH>
    __device__ __forceinline__ static Kept keep(const Pt& p)
    {
        return p.u;
    }
    template <int PH>
    __device__ __forceinline__ static Ad adj(const Ad& l, const Ad& c, const Ad& r, Kept, Kept,
                                             Kept, const Consts& k)
    {
        const T lap = (l.u + r.u) - T(2) * c.u;
        return Ad{c.u + k.r * lap};
    }
    // cotangent at the target level: cot (+ 2w u when that level is in the window)
    __device__ __forceinline__ static Ad seed(T cot, T two_w, Kept u, bool src)
    {
        return Ad{src ? cot + two_w * u : cot};
    }
    __device__ __forceinline__ static Ad source(const Ad& a, Kept u, T two_w)
    {
        return Ad{a.u + two_w * u};
    }
    __device__ __forceinline__ static T grad(const Ad& a) { return a.u; }
};

using HeatF64 = Heat<double>;
using HeatF32 = Heat<float>;

// ------------------------------------------------- Kuramoto-Sivashinsky
// u_t = -u u_x - u_xx - u_xxxx, central differences, RK2 midpoint as four
// radius-1 sub-timesteps (paper, Sections 2 and 6):
//   sub0  w  = D2(u)            sub1  v  = u + h*F(u, w)
//   sub2  z  = D2(v)            sub3  u' = u + dt*F(v, z)
// D2(a) = ((a[i-1]+a[i+1]) - 2a)*c2, D1(a) = (a[i+1]-a[i-1])*c1,
// F(a,b) = -(((a*D1(a)) + b) + D2(b)).
// A point carries (u, a, b): at a step boundary a = u; after sub0 b = w;
// after sub1 a = v; after sub2 b = z; sub3 writes u' into u and a.  The
// unused slot holds a stale value that no sub-timestep reads.  Since a = u
// (the same bits) until sub1 writes v, sub0 and sub1 read u wherever the
// scheme reads a: their neighbours' a need not be moved between lanes or
// kept in the LDS chain.
struct KSF64 {
    using T = double;
    struct Pt {
        double u, a, b;
    };
    struct Consts {
        double dt, h, c1, c2;
    };
    static constexpr int NPHASE = 4;
    static constexpr int kPersistWaves = 3;   // waves per SIMD of the persistent batch kernel
    // the continuous kernel's fill and drain run unmasked: a KS wave step is
    // long enough that masking the idle slots costs more than their updates
    static constexpr bool kUnmaskedEnds = true;

    __device__ __forceinline__ static Pt from_field(double v) { return Pt{v, v, 0.0}; }
    __device__ __forceinline__ static double to_field(const Pt& p) { return p.u; }
    __device__ __forceinline__ static Pt shr1(const Pt& s, const Pt& old)
    {
        return Pt{dpp_shr1(s.u, old.u), dpp_shr1(s.a, old.a), dpp_shr1(s.b, old.b)};
    }
    // F(a, b) at a point from the a and b of it and its two neighbours
    __device__ __forceinline__ static double rhs(double la, double ca, double ra, double lb,
                                                 double cb, double rb, const Consts& k)
    {
        const double d1a = (ra - la) * k.c1;
        const double d2b = ((lb + rb) - 2.0 * cb) * k.c2;
        return -(((ca * d1a) + cb) + d2b);
    }
    template <int PH>
    __device__ __forceinline__ static Pt step(const Pt& l, const Pt& c, const Pt& r,
                                              const Consts& k)
    {
        if constexpr (PH == 0) {          // a = u here
            return Pt{c.u, c.u, ((l.u + r.u) - 2.0 * c.u) * k.c2};
        } else if constexpr (PH == 2) {
            return Pt{c.u, c.a, ((l.a + r.a) - 2.0 * c.a) * k.c2};
        } else if constexpr (PH == 1) {   // a = u here
            return Pt{c.u, c.u + k.h * rhs(l.u, c.u, r.u, l.b, c.b, r.b, k), c.b};
        } else {
            const double un = c.u + k.dt * rhs(l.a, c.a, r.a, l.b, c.b, r.b, k);
            return Pt{un, un, c.b};
        }
    }

    // A pair's state after sub-timestep PH is read only by sub-timestep PH+1
    // (of the pair beside it), whose centre point is B: sub0 reads u of both
    // points; sub1 u and b of both; sub2 u and a of B and a of A; sub3 u, a,
    // b of B and a, b of A.  The continuous kernel's LDS chain keeps only
    // those components.
    static constexpr bool kChainStore = true;
    template <int PH>
    __device__ __forceinline__ static void chain_store(Pt* dB, Pt* dA, const Pt& B, const Pt& A)
    {
        dB->u = B.u;
        if constexpr (PH == 3 || PH == 0) {
            dA->u = A.u;
        } else {
            dB->a = B.a;
            dA->a = A.a;
        }
        if constexpr (PH == 0 || PH == 2) {
            dB->b = B.b;
            dA->b = A.b;
        }
    }

    // Discrete adjoint: the transposed Jacobian of each sub-timestep, in the
    // pull form (the cotangent of a point from the cotangents of the three
    // points of the level above that read it).  A cotangent carries
    // (ub, xb, yb): the cotangents of (u, w) after sub0, (u, v) after sub1,
    // (u, v, z) after sub2.  PH is the sub-timestep that leaves the level.
    struct Ad {
        double u, x, y;
    };
    // The one forward value each transposed sub-timestep reads at a point:
    // v (held in a) for sub3, u for sub1 and for the objective's source at
    // step levels; sub2 reads none.  PH is the sub-timestep that leaves the
    // level.
    using Kept = double;
    template <int PH>
    __device__ __forceinline__ static Kept keep(const Pt& p)
    {
        return PH == 3 ? p.a : p.u;
    }
    __device__ __forceinline__ static double d2(double l, double m, double r, const Consts& k)
    {
        return ((l + r) - 2.0 * m) * k.c2;
    }
    template <int PH>
    __device__ __forceinline__ static Ad adj(const Ad& al, const Ad& ac, const Ad& ar, Kept fl,
                                             Kept, Kept fr, const Consts& k)
    {
        if constexpr (PH == 3) {        // reverse of u' = u + dt*F(v, z), g = dt*ub'; fl, fr = v
            const double gl = k.dt * al.u, gm = k.dt * ac.u, gr = k.dt * ar.u;
            const double vb = (k.c1 * ((gr * fr) - (gl * fl))) - (gm * ((fr - fl) * k.c1));
            const double zb = -(gm + d2(gl, gm, gr, k));
            return Ad{ac.u, vb, zb};
        } else if constexpr (PH == 2) { // reverse of z = D2(v)
            return Ad{ac.u, ac.x + d2(al.y, ac.y, ar.y, k), 0.0};
        } else if constexpr (PH == 1) { // reverse of v = u + h*F(u, w), q = h*vb; fl, fr = u
            const double ql = k.h * al.x, qm = k.h * ac.x, qr = k.h * ar.x;
            const double ub = (ac.u + ac.x) +
                              ((k.c1 * ((qr * fr) - (ql * fl))) - (qm * ((fr - fl) * k.c1)));
            const double wb = -(qm + d2(ql, qm, qr, k));
            return Ad{ub, wb, 0.0};
        } else {                        // reverse of w = D2(u)
            return Ad{ac.u + d2(al.x, ac.x, ar.x, k), 0.0, 0.0};
        }
    }
    __device__ __forceinline__ static Ad seed(double cot, double two_w, Kept u, bool src)
    {
        return Ad{src ? cot + two_w * u : cot, 0.0, 0.0};
    }
    __device__ __forceinline__ static Ad source(const Ad& a, Kept u, double two_w)
    {
        return Ad{a.u + two_w * u, a.x, a.y};
    }
    __device__ __forceinline__ static double grad(const Ad& a) { return a.u; }
};

// ------------------------------------------------ contraction-on variants
// The same schemes with the multiply-adds fused, the form in which the
// paper's Section 4 counts the heat sub-timestep as 3 FLOPs.  Each fused
// multiply-add rounds once instead of twice, so these results differ from
// the canonical (unfused) ones by rounding only; they are a separate
// stencil id, never mixed with the bit-exact ones.
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// heat: s = u[i-1] + u[i+1];  lap = fma(-2, u, s);  u' = fma(r, lap, u)
template <class TT>
struct HeatFma : Heat<TT> {
    using Base = Heat<TT>;
    using typename Base::Pt;
    using typename Base::Consts;
    template <int PH>
    __device__ __forceinline__ static Pt step(const Pt& l, const Pt& c, const Pt& r,
                                              const Consts& k)
    {
        const TT lap = fmad(TT(-2), c.u, l.u + r.u);
        return Pt{fmad(k.r, lap, c.u)};
    }
};

using HeatFmaF64 = HeatFma<double>;
using HeatFmaF32 = HeatFma<float>;

// The canonical heat step (not a separate scheme): the same bits as Heat's
// five operations from four.  2u is exact whenever it is finite, so
// (u[i-1] + u[i+1]) - 2u is the exact difference s - 2u rounded once, which
// is what fma(-2, u, s) computes.  The two differ only where |u| exceeds
// half the largest finite value (2u overflows, the fused form does not).
// The kernels take this form only after the library has checked, for the
// call at hand, that 0 <= r <= 1/2, the run is not too long, and every
// finite |u0| is at most a sixteenth of the largest finite value: for such
// r the update is a convex combination of the three inputs, so each level
// exceeds the previous level's largest magnitude by at most 7 units of
// roundoff relative, and growing 8x takes more than 2e15 steps in binary64
// and 4e6 in binary32 (the library allows 1e15 and 1e6).  A non-finite input
// yields non-finite outputs in both forms alike.
template <class TT>
struct HeatLap : Heat<TT> {
    using Base = Heat<TT>;
    using typename Base::Pt;
    using typename Base::Consts;
    template <int PH>
    __device__ __forceinline__ static Pt step(const Pt& l, const Pt& c, const Pt& r,
                                              const Consts& k)
    {
        const TT lap = fmad(TT(-2), c.u, l.u + r.u);
        return Pt{c.u + k.r * lap};
    }
};

using HeatLapF64 = HeatLap<double>;
using HeatLapF32 = HeatLap<float>;

// KS: D2(a) = fma(-2, a, a[i-1] + a[i+1]) * c2,
//     F(a,b) = -(fma(a, D1(a), b) + D2(b)),  v = fma(h, F, u),  u' = fma(dt, F, u)
struct KSFmaF64 : KSF64 {
    __device__ __forceinline__ static double rhs(double la, double ca, double ra, double lb,
                                                 double cb, double rb, const Consts& k)
    {
        const double d1a = (ra - la) * k.c1;
        const double d2b = fmad(-2.0, cb, lb + rb) * k.c2;
        return -(fmad(ca, d1a, cb) + d2b);
    }
    // as KSF64, sub0 and sub1 read u where the scheme reads a (equal there)
    template <int PH>
    __device__ __forceinline__ static Pt step(const Pt& l, const Pt& c, const Pt& r,
                                              const Consts& k)
    {
        if constexpr (PH == 0) {
            return Pt{c.u, c.u, fmad(-2.0, c.u, l.u + r.u) * k.c2};
        } else if constexpr (PH == 2) {
            return Pt{c.u, c.a, fmad(-2.0, c.a, l.a + r.a) * k.c2};
        } else if constexpr (PH == 1) {
            return Pt{c.u, fmad(k.h, rhs(l.u, c.u, r.u, l.b, c.b, r.b, k), c.u), c.b};
        } else {
            const double un = fmad(k.dt, rhs(l.a, c.a, r.a, l.b, c.b, r.b, k), c.u);
            return Pt{un, un, c.b};
        }
    }
};

// ---------------------------------------------------------------- Euler
// 1D Euler equations of gas dynamics (paper, Section 7): second-order
// finite volume with the minmod limiter, interface flux with scalar
// dissipation proportional to the spectral radius of the Roe matrix, and the
// midpoint Runge-Kutta rule; as in Section 2, each Runge-Kutta stage is a
// slope sub-timestep and a flux-difference sub-timestep:
//   sub0  s = slope(q)               sub1  r  = q - ch*dF(q, s)
//   sub2  s = slope(r)               sub3  q' = q - cf*dF(r, s)
// slope = minmod of the one-sided differences, per conserved variable;
// dF(v, s) = F[i+1/2] - F[i-1/2], each face flux from the states
// reconstructed on its two sides, F = (f(qL) + f(qR))/2 - (lam/2)(qR - qL),
// lam = |u| + c at the Roe average.  ch = (dt/2)/dx, cf = dt/dx.  A cell's
// field value is (rho, m = rho u, E); a point carries q, r and s.
struct Cons {
    double r, m, e;
};

struct EulerF64 {
    // a nine-value point: lane 0 reads pair -1 when it needs it, which keeps
    // two points' registers free for occupancy (measured: +6% at W = 256)
    static constexpr bool kChainPrefetch = false;
    using T = Cons;
    struct Pt {
        double q[3], r[3], s[3];
    };
    struct Consts {
        double gm1, ch, cf;
    };
    static constexpr int NPHASE = 4;

    __device__ __forceinline__ static Pt from_field(const Cons& v)
    {
        return Pt{{v.r, v.m, v.e}, {v.r, v.m, v.e}, {0.0, 0.0, 0.0}};
    }
    __device__ __forceinline__ static Cons to_field(const Pt& p)
    {
        return Cons{p.q[0], p.q[1], p.q[2]};
    }
    __device__ __forceinline__ static Pt shr1(const Pt& v, const Pt& old)
    {
        Pt o;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o.q[c] = dpp_shr1(v.q[c], old.q[c]);
            o.r[c] = dpp_shr1(v.r[c], old.r[c]);
            o.s[c] = dpp_shr1(v.s[c], old.s[c]);
        }
        return o;
    }
    __device__ __forceinline__ static double minmod(double a, double b)
    {
        if (a > 0.0 && b > 0.0)
            return a < b ? a : b;
        if (a < 0.0 && b < 0.0)
            return a > b ? a : b;
        return 0.0;
    }
    // physical flux f(q); returns the total enthalpy (E + p)/rho
    __device__ __forceinline__ static double flux(const double (&q)[3], double gm1, double (&f)[3])
    {
        const double u = q[1] / q[0];
        const double p = gm1 * (q[2] - (0.5 * (q[1] * u)));
        f[0] = q[1];
        f[1] = (q[1] * u) + p;
        f[2] = (q[2] + p) * u;
        return (q[2] + p) / q[0];
    }
    // the face flux from the values v and slopes s of the cells on its two sides
    __device__ __forceinline__ static void face(const double (&vl)[3], const double (&sl)[3],
                                                const double (&vr)[3], const double (&sr)[3],
                                                double gm1, double (&F)[3])
    {
        double qL[3], qR[3], fL[3], fR[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            qL[c] = vl[c] + (0.5 * sl[c]);
            qR[c] = vr[c] - (0.5 * sr[c]);
        }
        const double HL = flux(qL, gm1, fL);
        const double HR = flux(qR, gm1, fR);
        const double a = sqrt(qL[0]), b = sqrt(qR[0]);
        const double uL = qL[1] / qL[0], uR = qR[1] / qR[0];
        const double ur = ((a * uL) + (b * uR)) / (a + b);
        const double Hr = ((a * HL) + (b * HR)) / (a + b);
        const double cr2 = gm1 * (Hr - (0.5 * (ur * ur)));
        const double lam = fabs(ur) + (cr2 > 0.0 ? sqrt(cr2) : 0.0);
        const double hl = 0.5 * lam;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            F[c] = (0.5 * (fL[c] + fR[c])) - (hl * (qR[c] - qL[c]));
    }
    // The flux sub-timesteps (1 and 3) split into face fluxes and their
    // difference, so that a kernel can compute the face between two cells
    // once and hand it to both (the face of cell pair (l, r) is the same
    // value for the update of l and of r).
    static constexpr bool kFaces = true;
    struct Face {
        double f[3];
    };
    template <int PH>
    static constexpr bool flux_phase = PH == 1 || PH == 3;
    // the face between cells l and r for flux sub-timestep PH
    template <int PH>
    __device__ __forceinline__ static Face face_of(const Pt& l, const Pt& r, const Consts& k)
    {
        Face F;
        if constexpr (PH == 1)
            face(l.q, l.s, r.q, r.s, k.gm1, F.f);
        else
            face(l.r, l.s, r.r, r.s, k.gm1, F.f);
        return F;
    }
    // the same with the sub-timestep chosen per lane: 3 if r3, else 1
    __device__ __forceinline__ static Face face_sel(const Pt& l, const Pt& r, bool r3,
                                                    const Consts& k)
    {
        double vl[3], vr[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vl[c] = r3 ? l.r[c] : l.q[c];
            vr[c] = r3 ? r.r[c] : r.q[c];
        }
        Face F;
        face(vl, l.s, vr, r.s, k.gm1, F.f);
        return F;
    }
    __device__ __forceinline__ static Face shr1(const Face& v, const Face& old)
    {
        Face o;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            o.f[c] = dpp_shr1(v.f[c], old.f[c]);
        return o;
    }
    // cell c after flux sub-timestep PH, from its left and right face fluxes
    template <int PH>
    __device__ __forceinline__ static Pt step_faces(const Pt& c, const Face& FL, const Face& FR,
                                                    const Consts& k)
    {
        Pt o = c;
        const double coef = PH == 1 ? k.ch : k.cf;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double v = c.q[j] - (coef * (FR.f[j] - FL.f[j]));
            if constexpr (PH == 1)
                o.r[j] = v;
            else
                o.q[j] = o.r[j] = v;
        }
        return o;
    }
    template <int PH>
    __device__ __forceinline__ static Pt step(const Pt& l, const Pt& c, const Pt& r,
                                              const Consts& k)
    {
        if constexpr (PH == 0 || PH == 2) {   // limited slopes of q (sub0) or r (sub2)
            Pt o = c;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double vl = PH == 0 ? l.q[j] : l.r[j];
                const double vc = PH == 0 ? c.q[j] : c.r[j];
                const double vr = PH == 0 ? r.q[j] : r.r[j];
                o.s[j] = minmod(vc - vl, vr - vc);
            }
            return o;
        } else {                              // flux differences of (q, s) or (r, s)
            return step_faces<PH>(c, face_of<PH>(l, c, k), face_of<PH>(c, r, k), k);
        }
    }
};

}  // namespace swept
