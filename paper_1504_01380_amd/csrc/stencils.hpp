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
// every path that evaluates these functions produces the same bits.
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
    template <int PH>
    __device__ __forceinline__ static Ad adj(const Ad& l, const Ad& c, const Ad& r, const Pt&,
                                             const Pt&, const Pt&, const Consts& k)
    {
        const T lap = (l.u + r.u) - T(2) * c.u;
        return Ad{c.u + k.r * lap};
    }
    // cotangent at the target level: cot (+ 2w u when that level is in the window)
    __device__ __forceinline__ static Ad seed(T cot, T two_w, const Pt& f, bool src)
    {
        return Ad{src ? cot + two_w * f.u : cot};
    }
    __device__ __forceinline__ static Ad source(const Ad& a, const Pt& f, T two_w)
    {
        return Ad{a.u + two_w * f.u};
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
// unused slot holds a stale value that no sub-timestep reads.
struct KSF64 {
    using T = double;
    struct Pt {
        double u, a, b;
    };
    struct Consts {
        double dt, h, c1, c2;
    };
    static constexpr int NPHASE = 4;

    __device__ __forceinline__ static Pt from_field(double v) { return Pt{v, v, 0.0}; }
    __device__ __forceinline__ static double to_field(const Pt& p) { return p.u; }
    __device__ __forceinline__ static Pt shr1(const Pt& s, const Pt& old)
    {
        return Pt{dpp_shr1(s.u, old.u), dpp_shr1(s.a, old.a), dpp_shr1(s.b, old.b)};
    }
    __device__ __forceinline__ static double rhs(const Pt& l, const Pt& c, const Pt& r,
                                                 const Consts& k)
    {
        const double d1a = (r.a - l.a) * k.c1;
        const double d2b = ((l.b + r.b) - 2.0 * c.b) * k.c2;
        return -(((c.a * d1a) + c.b) + d2b);
    }
    template <int PH>
    __device__ __forceinline__ static Pt step(const Pt& l, const Pt& c, const Pt& r,
                                              const Consts& k)
    {
        if constexpr (PH == 0 || PH == 2) {
            return Pt{c.u, c.a, ((l.a + r.a) - 2.0 * c.a) * k.c2};
        } else if constexpr (PH == 1) {
            return Pt{c.u, c.u + k.h * rhs(l, c, r, k), c.b};
        } else {
            const double un = c.u + k.dt * rhs(l, c, r, k);
            return Pt{un, un, c.b};
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
    __device__ __forceinline__ static double d2(double l, double m, double r, const Consts& k)
    {
        return ((l + r) - 2.0 * m) * k.c2;
    }
    template <int PH>
    __device__ __forceinline__ static Ad adj(const Ad& al, const Ad& ac, const Ad& ar,
                                             const Pt& fl, const Pt&, const Pt& fr,
                                             const Consts& k)
    {
        if constexpr (PH == 3) {        // reverse of u' = u + dt*F(v, z), g = dt*ub'
            const double gl = k.dt * al.u, gm = k.dt * ac.u, gr = k.dt * ar.u;
            const double vb = (k.c1 * ((gr * fr.a) - (gl * fl.a))) - (gm * ((fr.a - fl.a) * k.c1));
            const double zb = -(gm + d2(gl, gm, gr, k));
            return Ad{ac.u, vb, zb};
        } else if constexpr (PH == 2) { // reverse of z = D2(v)
            return Ad{ac.u, ac.x + d2(al.y, ac.y, ar.y, k), 0.0};
        } else if constexpr (PH == 1) { // reverse of v = u + h*F(u, w), q = h*vb
            const double ql = k.h * al.x, qm = k.h * ac.x, qr = k.h * ar.x;
            const double ub = (ac.u + ac.x) +
                              ((k.c1 * ((qr * fr.u) - (ql * fl.u))) - (qm * ((fr.u - fl.u) * k.c1)));
            const double wb = -(qm + d2(ql, qm, qr, k));
            return Ad{ub, wb, 0.0};
        } else {                        // reverse of w = D2(u)
            return Ad{ac.u + d2(al.x, ac.x, ar.x, k), 0.0, 0.0};
        }
    }
    __device__ __forceinline__ static Ad seed(double cot, double two_w, const Pt& f, bool src)
    {
        return Ad{src ? cot + two_w * f.u : cot, 0.0, 0.0};
    }
    __device__ __forceinline__ static Ad source(const Ad& a, const Pt& f, double two_w)
    {
        return Ad{a.u + two_w * f.u, a.x, a.y};
    }
    __device__ __forceinline__ static double grad(const Ad& a) { return a.u; }
};

}  // namespace swept
