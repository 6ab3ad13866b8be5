"""CPU emulation of the swept adjoint schedule (tests only).

Mirrors what the HIP adjoint path does: a forward swept pass that keeps the
V edges of every stage (one checkpoint per sweep), then the stages in
reverse order.  Each region recomputes its forward values from its
checkpoint, receives from the two later regions above it the cotangents of
their two boundary points and the forward value of their boundary point at
each level of their lower half, pulls the cotangents of its own points level
by level from the top, and hands the same kind of data to the two earlier
regions below it.  Values must equal the oracle's discrete adjoint bit for
bit.

Region geometry (stage s, region t, tile width W = 2k): centre
J = tW + k + s*k, base level b = (s-1)k; at relative level j it covers
[J-j, J+j-1] for j <= k and [J-2k+j, J+2k-1-j] above; stage 0 is the
triangle (relative levels k..2k-1, level 0 = relative k).
"""
from __future__ import annotations


def heat_local(r):
    def fwd(ph, l, c, rr):
        return c + r * ((l + rr) - 2.0 * c)

    def adj(ph, al, ac, ar, fl, fc, fr):
        return ac + r * ((al + ar) - 2.0 * ac)

    def seed(cot, two_w, fc, src):
        return cot + two_w * fc if src else cot

    def source(a, fc, two_w):
        return a + two_w * fc
    return dict(fwd=fwd, adj=adj, seed=seed, source=source, nph=1,
                from_field=lambda v: v, to_field=lambda p: p, grad=lambda a: a)


def ks_local(dt, dx):
    h, c1, c2 = 0.5 * dt, 1.0 / (2.0 * dx), 1.0 / (dx * dx)

    def d2(l, m, r):
        return ((l + r) - 2.0 * m) * c2

    def rhs(l, c, r):
        d1a = (r[1] - l[1]) * c1
        d2b = ((l[2] + r[2]) - 2.0 * c[2]) * c2
        return -(((c[1] * d1a) + c[2]) + d2b)

    def fwd(ph, l, c, r):
        if ph in (0, 2):
            return (c[0], c[1], d2(l[1], c[1], r[1]))
        if ph == 1:
            return (c[0], c[0] + h * rhs(l, c, r), c[2])
        un = c[0] + dt * rhs(l, c, r)
        return (un, un, c[2])

    # adjoint state (ub, xb, yb); forward state (u, a, b); ph = phase of the
    # level whose cotangent is formed (its forward sub-timestep is ph)
    def adj(ph, al, ac, ar, fl, fc, fr):
        if ph == 3:
            gl, gm, gr = dt * al[0], dt * ac[0], dt * ar[0]
            vl, vr = fl[1], fr[1]
            vb = (c1 * ((gr * vr) - (gl * vl))) - (gm * ((vr - vl) * c1))
            zb = -(gm + d2(gl, gm, gr))
            return (ac[0], vb, zb)
        if ph == 2:
            return (ac[0], ac[1] + d2(al[2], ac[2], ar[2]), 0.0)
        if ph == 1:
            ql, qm, qr = h * al[1], h * ac[1], h * ar[1]
            ul, ur = fl[0], fr[0]
            ub = (ac[0] + ac[1]) + ((c1 * ((qr * ur) - (ql * ul))) - (qm * ((ur - ul) * c1)))
            wb = -(qm + d2(ql, qm, qr))
            return (ub, wb, 0.0)
        return (ac[0] + d2(al[1], ac[1], ar[1]), 0.0, 0.0)

    def seed(cot, two_w, fc, src):
        return ((cot + two_w * fc[0]) if src else cot, 0.0, 0.0)

    def source(a, fc, two_w):
        return (a[0] + two_w * fc[0], a[1], a[2])
    return dict(fwd=fwd, adj=adj, seed=seed, source=source, nph=4,
                from_field=lambda v: (v, v, 0.0), to_field=lambda p: p[0], grad=lambda a: a[0])


def adjoint(u0, nsteps, k, loc, n0, wgt, cot=None):
    """Gradient of J = wgt*sum_{j=n0}^{nsteps}|u^j|^2 + <cot, u^nsteps>."""
    n = len(u0)
    W = 2 * k
    assert n % W == 0
    T = n // W
    nph = loc["nph"]
    L = nsteps * nph
    two_w = 2.0 * wgt
    fwd, adj = loc["fwd"], loc["adj"]
    if L == 0:
        return [loc["seed"](0.0 if cot is None else cot[x], two_w, loc["from_field"](u0[x]),
                            nsteps >= n0)[0] if nph == 4 else
                loc["seed"](0.0 if cot is None else cot[x], two_w, u0[x], nsteps >= n0)
                for x in range(n)]
    S = 1 + (L + k - 1) // k

    def geom(s, t):
        J = (t * W + k + s * k) % n
        b = (s - 1) * k
        jlo = k if s == 0 else 1          # lowest computed relative level (tri: abs 1 = rel k+1)
        jtop = min(2 * k - 1, L - b)
        return J, b, jlo, jtop

    def span(j):
        return (-j, j - 1) if j <= k else (-2 * k + j, 2 * k - 1 - j)

    # ---- forward pass with one checkpoint (the V of every region) per stage
    V = {}       # (s, t) -> {(x_rel, j): value} inputs of region (s, t)
    F = {}       # forward value of every (x, level) by region, rebuilt per region below
    field = {}   # global forward values (x, level) -> value (only to build V's)
    for x in range(n):
        field[(x, 0)] = loc["from_field"](u0[x])
    for s in range(S):
        for t in range(T):
            J, b, jlo, jtop = geom(s, t)
            Vst = {}
            if s == 0:
                for dx in range(-k, k):
                    Vst[(dx, k)] = field[((J + dx) % n, 0)]
            else:
                for i in range(k):                  # left and right arms at rel level i
                    for dx in (-i - 2, -i - 1, i, i + 1):
                        if b + i <= L:
                            Vst[(dx, i)] = field[((J + dx) % n, b + i)]
            V[(s, t)] = Vst
        for t in range(T):
            J, b, jlo, jtop = geom(s, t)
            for j in range(jlo + (1 if s == 0 else 0), jtop + 1):
                lo, hi = span(j)
                ph = (b + j - 1) % nph
                for dx in range(lo, hi + 1):
                    x = (J + dx) % n
                    field[(x, b + j)] = fwd(ph, field[((x - 1) % n, b + j - 1)],
                                            field[(x, b + j - 1)], field[((x + 1) % n, b + j - 1)])

    # ---- reverse pass
    AE = {}   # (s, t, side) -> {j: (a_first, a_second)}   cotangents handed down
    FH = {}   # (s, t, side) -> {j: forward value}           forward halo handed down
    grad = [None] * n
    for s in range(S - 1, -1, -1):
        for t in range(T):
            J, b, jlo, jtop = geom(s, t)
            # recompute this region's forward values from its checkpoint only
            Fr = dict(V[(s, t)])
            j0 = k if s == 0 else 0
            for j in range(j0 + 1, jtop + 1):
                lo, hi = span(j)
                ph = (b + j - 1) % nph
                for dx in range(lo, hi + 1):
                    Fr[(dx, j)] = fwd(ph, Fr[(dx - 1, j - 1)], Fr[(dx, j - 1)], Fr[(dx + 1, j - 1)])
            # data from the later regions: upper-left (s+1, t-1), upper-right (s+1, t)
            A = {}
            if s + 1 < S:
                ul, ur = (s + 1, (t - 1) % T), (s + 1, t)
                # the later regions are centred at J-k and J+k with base b+k:
                # their relative level jj is our relative level jj+k
                for jj, (a1, a2) in AE[ul + ("R",)].items():
                    A[(-k + jj - 2, jj + k)] = a1
                    A[(-k + jj - 1, jj + k)] = a2
                for jj, f in FH[ul + ("R",)].items():
                    Fr[(-k + jj - 1, jj + k)] = f
                for jj, (a1, a2) in AE[ur + ("L",)].items():
                    A[(k - jj, jj + k)] = a1
                    A[(k - jj + 1, jj + k)] = a2
                for jj, f in FH[ur + ("L",)].items():
                    Fr[(k - jj, jj + k)] = f
            # cotangents, from the top level down
            jbot = k if s == 0 else 1
            for j in range(jtop, jbot - 1, -1):
                lo, hi = span(j)
                lev = b + j
                ph = lev % nph
                for dx in range(lo, hi + 1):
                    x = (J + dx) % n
                    if lev == L:
                        a = loc["seed"](0.0 if cot is None else cot[x], two_w, Fr[(dx, j)],
                                        nsteps >= n0)
                    else:
                        a = adj(ph, A[(dx - 1, j + 1)], A[(dx, j + 1)], A[(dx + 1, j + 1)],
                                Fr[(dx - 1, j)], Fr[(dx, j)], Fr[(dx + 1, j)])
                        if ph == 0 and lev // nph >= n0:
                            a = loc["source"](a, Fr[(dx, j)], two_w)
                    A[(dx, j)] = a
            # hand down: boundary cotangents at levels 1..k, boundary forward at 0..k-1
            if s > 0:
                AE[(s, t, "L")] = {j: (A[(-j, j)], A[(-j + 1, j)]) for j in range(1, min(k, jtop) + 1)}
                AE[(s, t, "R")] = {j: (A[(j - 2, j)], A[(j - 1, j)]) for j in range(1, min(k, jtop) + 1)}
                FH[(s, t, "L")] = {j: Fr[(-j, j)] for j in range(0, min(k - 1, jtop) + 1)}
                FH[(s, t, "R")] = {j: Fr[(j - 1, j)] for j in range(0, min(k - 1, jtop) + 1)}
            else:
                for dx in range(-k, k):
                    grad[(J + dx) % n] = loc["grad"](A[(dx, k)])
    return grad
