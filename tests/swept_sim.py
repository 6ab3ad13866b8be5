"""CPU emulation of the swept stage kernel's schedule (tests only).

Re-expresses, index for index, what swept_stage_kernel in
paper_1504_01380_amd/csrc/kernels.hpp does -- tiles, stages, bands of 64*P
pairs, wave steps, the lane-to-lane shift, the LDS chain and the RE/LE edge
buffers -- on plain Python values, so the schedule can be checked on a CPU:
every (point, level) must be computed exactly once, after its inputs, and the
values must equal the oracle's bit for bit.  The per-point update is passed
in (the scheme's local code), so the same emulation serves every stencil.
"""
from __future__ import annotations

import math
import random


def heat_step(r):
    def f(ph, l, c, rr):
        return c + r * ((l + rr) - 2.0 * c)
    return f, 1, (lambda v: v), (lambda p: p)


def ks_step(dt, dx):
    h, c1, c2 = 0.5 * dt, 1.0 / (2.0 * dx), 1.0 / (dx * dx)

    def rhs(l, c, r, ia):
        d1a = (r[ia] - l[ia]) * c1
        d2b = ((l[2] + r[2]) - 2.0 * c[2]) * c2
        return -(((c[ia] * d1a) + c[2]) + d2b)

    # as the kernel: a = u until sub1 writes v, so sub0 and sub1 read u
    # (index 0) where the scheme reads a (index 1)
    def f(ph, l, c, r):
        if ph == 0:
            return (c[0], c[0], ((l[0] + r[0]) - 2.0 * c[0]) * c2)
        if ph == 2:
            return (c[0], c[1], ((l[1] + r[1]) - 2.0 * c[1]) * c2)
        if ph == 1:
            return (c[0], c[0] + h * rhs(l, c, r, 0), c[2])
        un = c[0] + dt * rhs(l, c, r, 1)
        return (un, un, c[2])
    f.unmasked_ends = True   # as the KS continuous kernel (kUnmaskedEnds)
    return f, 4, (lambda v: (v, v, 0.0)), (lambda p: p[0])


NAN = float("nan")


def _chain_store(ph, B, A, oldB, oldA):
    """What the continuous kernel's last slot leaves in the LDS chain after
    sub-timestep ph: whole points for one-value stencils; for KS points
    (u, a, b) only what sub-timestep ph+1 reads (sub0: u of both; sub1: u
    and b of both; sub2: B's u and a, A's a; sub3: B's u, a and b, A's a and
    b) -- here the other components become NaN, so a read of one of them
    would show in the result."""
    if not isinstance(B, tuple):
        return B, A
    if ph == 3:
        return (B[0], NAN, NAN), (A[0], NAN, NAN)
    if ph == 0:
        return (B[0], NAN, B[2]), (A[0], NAN, A[2])
    if ph == 1:
        return (B[0], B[1], NAN), (NAN, A[1], NAN)
    return (B[0], B[1], B[2]), (NAN, A[1], A[2])


def _poison(p):
    """A point of the same kind as p whose every component is NaN."""
    return tuple(NAN for _ in p) if isinstance(p, tuple) else NAN


def _cont_stage(t, J, b, k, P, lanes, RE, chain, step, nph, n, visits):
    """One full diamond on the continuous-band schedule of
    swept_diamond_cont_kernel: slot e works on band (sigma-e) div k, step
    (sigma-e) mod k at wave step sigma and changes band at sigma = beta*k+e.
    In the pipeline fill and drain the slots that have not started or have
    finished are idle; for a stencil whose step function has unmasked_ends
    (KS, as in the kernel) they keep computing: slot e takes its first state
    at fill step e and stores its final one at drain step e.  Here a slot's
    state is NaN before its start and after its end, so a read of it by an
    active slot would show in the result.  As in the kernel, the chain holds
    a copy of entry 0 as entry k, which the last slot updates with entry 0,
    and slot 0 prefetches entry j + 1 at every step j (no wrap at j = k - 1)."""
    NB = lanes * P
    nb = k // NB
    chain.extend([chain[0], chain[1]])
    unmasked = getattr(step, "unmasked_ends", False)
    A = [RE[t][2 * e + 1] for e in range(NB)]
    B = [RE[t][2 * e] for e in range(NB)]
    if unmasked:   # taken at each slot's fill step
        An, Bn = A, B
        A = [_poison(p) for p in An]
        B = [_poison(p) for p in Bn]
    else:
        An = [RE[t][2 * (NB + e) + 1] if nb > 1 else None for e in range(NB)]
        Bn = [RE[t][2 * (NB + e)] if nb > 1 else None for e in range(NB)]
    cA, cB = chain[1], chain[0]
    fill, drain = (4, 3) if unmasked else (1, 2)
    for cyc in range(nb + 1):
        steps = range(NB) if cyc == nb else range(k)
        for j in steps:
            sigma = cyc * k + j
            mask = fill if (cyc == 0 and j < NB) else (drain if cyc == nb else 0)
            trans = 0 < cyc < nb and j < NB
            inA = [cA] + [A[(r - 1) * P + P - 1] for r in range(1, lanes)]
            inB = [cB] + [B[(r - 1) * P + P - 1] for r in range(1, lanes)]
            ns = j + 1
            nA, nB = chain[2 * ns + 1], chain[2 * ns]
            ph = (b + sigma) % nph
            for r in range(lanes):
                for q in range(P - 1, -1, -1):
                    e = r * P + q
                    if (trans or mask in (3, 4)) and e == j:
                        if mask != 4:
                            RE[t][2 * ((cyc - 1) * NB + j)] = B[e]
                            RE[t][2 * ((cyc - 1) * NB + j) + 1] = A[e]
                        if mask == 3:
                            A[e] = B[e] = _poison(A[e])
                        else:
                            A[e], B[e] = An[e], Bn[e]
                    if (mask == 1 and e > j) or (mask == 2 and e <= j):
                        continue
                    rA = inA[r] if q == 0 else A[e - 1]
                    cBv = inB[r] if q == 0 else B[e - 1]
                    B[e] = step(ph, B[e], A[e], cBv)
                    A[e] = step(ph, A[e], cBv, rA)
                    if visits is not None and not ((mask == 3 and e <= j) or
                                                   (mask == 4 and e > j)):
                        beta, m = divmod(sigma - e, k)
                        d = beta * NB + e
                        lvl = b + m + d + 1
                        xa = (J + m - d) % n
                        for x in (xa, (xa - 1) % n):
                            visits[(x, lvl)] = visits.get((x, lvl), 0) + 1
            wlast = (j == NB - 1) if mask in (1, 4) else ((j < NB - 1) if mask >= 2 else True)
            if wlast:
                ws = (j + k - (NB - 1)) % k
                chain[2 * ws], chain[2 * ws + 1] = _chain_store(ph, B[NB - 1], A[NB - 1],
                                                                chain[2 * ws], chain[2 * ws + 1])
                if ws == 0:
                    chain[2 * k], chain[2 * k + 1] = _chain_store(ph, B[NB - 1], A[NB - 1],
                                                                  chain[2 * k],
                                                                  chain[2 * k + 1])
            cA, cB = nA, nB
            if (trans or mask == 4) and j == NB - 1 and cyc + 1 < nb:
                # every slot has entered band cyc: band cyc+1's left-edge
                # states, for all slots at once
                for e in range(NB):
                    Bn[e] = RE[t][2 * ((cyc + 1) * NB + e)]
                    An[e] = RE[t][2 * ((cyc + 1) * NB + e) + 1]
    if drain == 2:
        for e in range(NB):
            RE[t][2 * ((nb - 1) * NB + e)] = B[e]
            RE[t][2 * ((nb - 1) * NB + e) + 1] = A[e]
    del chain[2 * k:]                     # the copy of entry 0 is not part of the edge


def cont_faces_symbolic(k, P, b, lanes=64):
    """The face-sharing bookkeeping of the continuous kernel for a stencil
    whose flux sub-timesteps (1 and 3 of 4) split into face fluxes, on
    symbolic values: a point is (x, level) and a face is ('F', x, level,
    phase), the face between x and x+1.  Every update asserts that it gets
    exactly the neighbours and the two faces it needs; returns the final
    right edge and the chain (the new left edge) for a check of the
    geometry.  Mirrors the kernel: F[e] = face of pair e (B, A) before the
    step; pair e's right face is F[e-1], slot 0's comes from the face chain
    (the right V edge's faces, then those the last slot leaves one step
    after each chain entry), entry m at index m // 2 (the flux entries are
    those of one parity of m); a slot that changes band takes the face of
    its new state computed before the cycle's head."""
    NB = lanes * P
    assert k % NB == 0 and NB % 4 == 0   # as 64P in the kernel
    nb = k // NB

    def step(ph, l, c, r):
        assert l == (c[0] - 1, c[1]) and r == (c[0] + 1, c[1]) and ph == c[1] % 4, (l, c, r, ph)
        return (c[0], c[1] + 1)

    def face(ph, l, r):
        assert r == (l[0] + 1, l[1]) and ph == l[1] % 4, (l, r, ph)
        return ('F', l[0], l[1], ph)

    def step_f(ph, c, FL, FR):
        assert FL == ('F', c[0] - 1, c[1], ph) and FR == ('F', c[0], c[1], ph), (c, FL, FR, ph)
        return (c[0], c[1] + 1)

    J = 0
    # left V edge: pair d at step -1; right V edge (chain): pair -1 at step m
    RE = []
    for d in range(k):
        RE += [(J - 2 - d, b + d), (J - 1 - d, b + d)]
    chain = []
    for m in range(k):
        chain += [(J + m, b + m), (J + m + 1, b + m)]
    flux = (1, 3)
    fchain = [None] * (k // 2)
    for i in range(k // 2):
        m = 2 * i + (b + 1) % 2
        assert (b + m) % 4 in flux
        fchain[i] = face((b + m) % 4, chain[2 * m], chain[2 * m + 1])
    fnext = [None] * NB
    A = [RE[2 * e + 1] for e in range(NB)]
    B = [RE[2 * e] for e in range(NB)]
    An = [RE[2 * (NB + e) + 1] if nb > 1 else None for e in range(NB)]
    Bn = [RE[2 * (NB + e)] if nb > 1 else None for e in range(NB)]
    out = list(RE)
    for cyc in range(nb + 1):
        if 0 < cyc < nb:   # faces of the states the slots take at this cycle's head
            for e in range(NB):
                ph = (b + cyc * k + e) % 4
                fnext[e] = face(ph, Bn[e], An[e]) if ph in flux else None
        for j in (range(NB) if cyc == nb else range(k)):
            mask = 1 if (cyc == 0 and j < NB) else (2 if cyc == nb else 0)
            trans = 0 < cyc < nb and j < NB
            ph = (b + cyc * k + j) % 4
            inA = [chain[2 * j + 1]] + [A[(r - 1) * P + P - 1] for r in range(1, lanes)]
            inB = [chain[2 * j]] + [B[(r - 1) * P + P - 1] for r in range(1, lanes)]
            fl = ph in flux
            if fl:
                def own_face(e):
                    try:
                        return face(ph, B[e], A[e])
                    except AssertionError:
                        return None   # a slot outside its band: never read
                F = [own_face(e) for e in range(NB)]
                H0 = [fchain[j >> 1]] + [F[(r - 1) * P + P - 1] for r in range(1, lanes)]
                if mask != 1:
                    fs = j + k - NB if j < NB else j - NB
                    assert fs % 2 == j % 2
                    fchain[fs >> 1] = F[NB - 1]
            for r in range(lanes):
                for q in range(P - 1, -1, -1):
                    e = r * P + q
                    if trans and e == j:
                        out[2 * ((cyc - 1) * NB + j)] = B[e]
                        out[2 * ((cyc - 1) * NB + j) + 1] = A[e]
                        A[e], B[e] = An[e], Bn[e]
                        if cyc + 1 < nb:
                            Bn[e] = RE[2 * ((cyc + 1) * NB + j)]
                            An[e] = RE[2 * ((cyc + 1) * NB + j) + 1]
                        if fl:
                            F[e] = fnext[e]
                    act = (e <= j) if mask == 1 else ((e > j) if mask == 2 else True)
                    if not act:
                        continue
                    rA = inA[r] if q == 0 else A[e - 1]
                    cBv = inB[r] if q == 0 else B[e - 1]
                    if fl:
                        G = face(ph, A[e], cBv)
                        H = H0[r] if q == 0 else F[e - 1]
                        B[e] = step_f(ph, A[e], F[e], G)
                        A[e] = step_f(ph, cBv, G, H)
                    else:
                        B[e] = step(ph, B[e], A[e], cBv)
                        A[e] = step(ph, A[e], cBv, rA)
            wlast = (j == NB - 1) if mask == 1 else ((j < NB - 1) if mask == 2 else True)
            if wlast:
                ws = (j + k - (NB - 1)) % k
                chain[2 * ws], chain[2 * ws + 1] = B[NB - 1], A[NB - 1]
    for e in range(NB):
        out[2 * ((nb - 1) * NB + e)] = B[e]
        out[2 * ((nb - 1) * NB + e) + 1] = A[e]
    return out, chain


def simulate(u0, nsteps, k, P, stencil, lanes=64, track=False, cont=False):
    """Run the swept schedule on a Python list; returns (u, visits) where
    visits maps (x, level) -> number of times it was computed (if track)."""
    step, nph, from_field, to_field = stencil
    n = len(u0)
    W = 2 * k
    assert n % W == 0
    T = n // W
    L = nsteps * nph
    u = list(u0)
    visits = {} if track else None
    if L == 0:
        return u, visits
    stages = 1 + (L + k - 1) // k
    RE = [[None] * (2 * k) for _ in range(T)]
    LE = [[[None] * (2 * k) for _ in range(T)] for _ in range(2)]
    band = lanes * P
    for s in range(stages):
        tri = s == 0
        b = (s - 1) * k
        J0 = (k + s * k) % n
        le_in, le_out = LE[(s + 1) % 2], LE[s % 2]
        for t in range(T):
            J = (t * W + J0) % n
            chain = list(le_in[(t + 1) % T]) if not tri else [None] * (2 * k)
            top = L - b
            if cont and not tri and b + 2 * k - 1 < L and k % (lanes * P) == 0:
                _cont_stage(t, J, b, k, P, lanes, RE, chain, step, nph, n, visits)
                le_out[t] = chain
                continue
            for base in range(0, k, band):
                nvalid = min(band, k - base)
                tau_first = (k - base) if tri else 0
                tau_cap = top - base - 1
                tau_end = min(nvalid + k - 2, tau_cap)
                if tau_end < tau_first and not tri:
                    continue
                A = [None] * band
                B = [None] * band
                for e in range(nvalid):
                    d = base + e
                    if tri:
                        xa = J + k - 1 - 2 * d
                        A[e], B[e] = from_field(u[xa]), from_field(u[xa - 1])
                    else:
                        B[e], A[e] = RE[t][2 * d], RE[t][2 * d + 1]
                eL = nvalid - 1
                if tri:
                    m = k - 1 - (base + eL)
                    chain[2 * m], chain[2 * m + 1] = B[eL], A[eL]
                slot = min(tau_first, k - 1)
                cA, cB = chain[2 * slot + 1], chain[2 * slot]
                for tau in range(tau_first, tau_end + 1):
                    # lane r receives lane r-1's last pair; lane 0 the chain
                    inA = [cA] + [A[(r - 1) * P + P - 1] for r in range(1, lanes)]
                    inB = [cB] + [B[(r - 1) * P + P - 1] for r in range(1, lanes)]
                    slot = min(tau + 1, k - 1)
                    nA, nB = chain[2 * slot + 1], chain[2 * slot]
                    ph = (b + base + tau) % nph
                    for r in range(lanes):
                        for q in range(P - 1, -1, -1):
                            e = r * P + q
                            m = tau - e
                            if not (0 <= m < k and e < nvalid):
                                continue
                            rA = inA[r] if q == 0 else A[e - 1]
                            cBv = inB[r] if q == 0 else B[e - 1]
                            nAv = step(ph, A[e], cBv, rA)
                            nBv = step(ph, B[e], A[e], cBv)
                            A[e], B[e] = nAv, nBv
                            if track:
                                d = base + e
                                lvl = b + m + d + 1
                                xa = (J + m - d) % n
                                for x in (xa, (xa - 1) % n):
                                    visits[(x, lvl)] = visits.get((x, lvl), 0) + 1
                    if tau == tau_cap:
                        for e in range(nvalid):
                            m = tau - e
                            if 0 <= m < k:
                                d = base + e
                                xa = (J + m - d) % n
                                u[xa] = to_field(A[e])
                                u[(xa - 1) % n] = to_field(B[e])
                    m = tau - eL
                    if 0 <= m < k:
                        chain[2 * m], chain[2 * m + 1] = B[eL], A[eL]
                    cA, cB = nA, nB
                for e in range(nvalid):
                    d = base + e
                    RE[t][2 * d], RE[t][2 * d + 1] = B[e], A[e]
            le_out[t] = chain
    return u, visits


def levels_complete(visits, n, L, k):
    """Every (x, 1..L) computed exactly once (levels above L may appear: a
    band stops at L, so nothing above it is computed either)."""
    for x in range(n):
        for lvl in range(1, L + 1):
            if visits.get((x, lvl), 0) != 1:
                return False, (x, lvl, visits.get((x, lvl), 0))
    extra = [key for key in visits if key[1] > L]
    if extra:
        return False, ("above L", extra[:3])
    return True, None


class _Recorded(list):
    """A list that logs (name, index, "r" or "w") for every element read or
    written, into log[0] (a list, or None while not recording)."""

    def __init__(self, data, name, log):
        super().__init__(data)
        self.name, self.log = name, log

    def _note(self, i, kind):
        if self.log[0] is None:
            return
        idx = range(*i.indices(len(self))) if isinstance(i, slice) else [i % len(self)]
        self.log[0].extend((self.name, j, kind) for j in idx)

    def __getitem__(self, i):
        self._note(i, "r")
        return super().__getitem__(i)

    def __setitem__(self, i, v):
        self._note(i, "w")
        super().__setitem__(i, v)


class _Offset:
    """A window of a flat list starting at `off` (a tile's slice of the edge
    buffer)."""

    def __init__(self, data, off):
        self.data, self.off = data, off

    def __getitem__(self, i):
        return self.data[self.off + i]

    def __setitem__(self, i, v):
        self.data[self.off + i] = v


def simulate_tiles(u0, nsteps, ks_list, P, stencil, lanes=64, track=False, cont=False,
                   order="stage", seed=0, inplace=False, waits=("own", "next"),
                   footprints=None, stages=None):
    """The swept schedule on tiles of unequal even widths 2*k_t (sum = N).
    Workgroup t keeps k_t pairs; at stage s its region is the rectangle of
    k_t pairs by k_{t+s} steps centred at J = (X_{t+s} + X_{t+1}) / 2 with
    base level b = (X_{t+s} - X_{t+1}) / 2 (X_t = 2*sum_{t'<t} k_t', taken
    periodically with period N).  Stage 0 is the triangle of each tile.
    Right edges live at offset X_t, left edges at offset X_{(t+s) mod T}.
    With cont, a square k x k region strictly below level L whose k is a
    multiple of lanes*P runs on the continuous-band schedule (as in
    swept_batch_kernel), its cycles starting at phase b mod nph.

    order="stage" runs the regions stage by stage (the per-stage launches).
    order="random" runs them in a random order (seeded) in which region
    (t, s) only waits for what the persistent batch kernel waits for:
    `waits` names "own" (stage s-1 of tile t) and "next" (stage s-1 of tile
    t+1); a region whose wait is not met is never run early, and one that
    is met may run at once.  Every tile runs `stages` regions (default: up
    to the first stage whose regions all lie above the target level; the
    batch host passes its bound 2 + (L + k - rem) T / h).  inplace=True
    reads stage 0 from, and writes the final level into, one array, as the
    kernels do.  With a dict
    `footprints`, every region's reads and writes of the field and the edge
    buffers are stored there under (t, s) as a set of (buffer, index,
    "r"/"w")."""
    step, nph, from_field, to_field = stencil
    n = len(u0)
    T = len(ks_list)
    X = [0]
    for kt in ks_list:
        X.append(X[-1] + 2 * kt)
    assert X[-1] == n

    def Xp(i):  # periodic extension
        q, r = divmod(i, T)
        return X[r] + q * n

    L = nsteps * nph
    log = [None]
    u = _Recorded(u0, "u", log)
    out = u if inplace else _Recorded(u0, "out", log)
    visits = {} if track else None
    if L == 0:
        return list(u), visits
    RE = _Recorded([None] * n, "re", log)
    LE = [_Recorded([None] * n, "le0", log), _Recorded([None] * n, "le1", log)]
    band = lanes * P

    def region(t, s):
        if footprints is None:
            return region_body(t, s)
        log[0] = []
        ran = region_body(t, s)
        footprints[(t, s)] = set(log[0])
        log[0] = None
        return ran

    def region_body(t, s):
        """Run region (t, s); False if it lies above the target level."""
        le_in, le_out = LE[(s + 1) % 2], LE[s % 2]
        if True:
            kp, ks = ks_list[t], ks_list[(t + s) % T]
            J2 = Xp(t + s) + Xp(t + 1)
            assert J2 % 2 == 0
            J = (J2 // 2) % n
            b = (Xp(t + s) - Xp(t + 1)) // 2
            tri = s == 0
            if not tri and b >= L:
                return False
            re_off = X[t]
            le_off_out = X[(t + s) % T]
            le_off_in = X[(t + s) % T]   # written by workgroup t+1 at stage s-1
            chain = [None] * (2 * ks) if tri else list(le_in[le_off_in:le_off_in + 2 * ks])
            top = L - b
            if cont and not tri and kp == ks and kp % band == 0 and b + 2 * kp - 1 < L:
                _cont_stage(0, J, b, kp, P, lanes, [_Offset(RE, re_off)], chain, step, nph, n,
                            visits)
                le_out[le_off_out:le_off_out + 2 * ks] = chain
                return True
            for base in range(0, kp, band):
                nvalid = min(band, kp - base)
                tau_first = (ks - base) if tri else 0
                tau_cap = top - base - 1
                tau_end = min(nvalid + ks - 2, tau_cap)
                if tau_end < tau_first and not tri:
                    continue
                A = [None] * band
                B = [None] * band
                for e in range(nvalid):
                    d = base + e
                    if tri:
                        xa = J + ks - 1 - 2 * d
                        A[e], B[e] = from_field(u[xa % n]), from_field(u[(xa - 1) % n])
                    else:
                        B[e], A[e] = RE[re_off + 2 * d], RE[re_off + 2 * d + 1]
                eL = nvalid - 1
                if tri:
                    m = ks - 1 - (base + eL)
                    chain[2 * m], chain[2 * m + 1] = B[eL], A[eL]
                slot = min(tau_first, ks - 1)
                cA, cB = chain[2 * slot + 1], chain[2 * slot]
                for tau in range(tau_first, tau_end + 1):
                    inA = [cA] + [A[(r - 1) * P + P - 1] for r in range(1, lanes)]
                    inB = [cB] + [B[(r - 1) * P + P - 1] for r in range(1, lanes)]
                    slot = min(tau + 1, ks - 1)
                    nA, nB = chain[2 * slot + 1], chain[2 * slot]
                    ph = (b + base + tau) % nph
                    for r in range(lanes):
                        for q in range(P - 1, -1, -1):
                            e = r * P + q
                            m = tau - e
                            if not (0 <= m < ks and e < nvalid):
                                continue
                            rA = inA[r] if q == 0 else A[e - 1]
                            cBv = inB[r] if q == 0 else B[e - 1]
                            nAv = step(ph, A[e], cBv, rA)
                            nBv = step(ph, B[e], A[e], cBv)
                            A[e], B[e] = nAv, nBv
                            if track:
                                d = base + e
                                lvl = b + m + d + 1
                                xa = (J + m - d) % n
                                for x in (xa, (xa - 1) % n):
                                    visits[(x, lvl)] = visits.get((x, lvl), 0) + 1
                    if tau == tau_cap:
                        for e in range(nvalid):
                            m = tau - e
                            if 0 <= m < ks:
                                d = base + e
                                xa = (J + m - d) % n
                                out[xa] = to_field(A[e])
                                out[(xa - 1) % n] = to_field(B[e])
                    m = tau - eL
                    if 0 <= m < ks:
                        chain[2 * m], chain[2 * m + 1] = B[eL], A[eL]
                    cA, cB = nA, nB
                for e in range(nvalid):
                    d = base + e
                    RE[re_off + 2 * d], RE[re_off + 2 * d + 1] = B[e], A[e]
            le_out[le_off_out:le_off_out + 2 * ks] = chain
            return True

    if order == "stage":
        s = 0
        while any([region(t, s) for t in range(T)]):
            s += 1
        return list(out), visits
    assert order == "random"
    if stages is None:     # every tile runs to the first stage at which all are above L
        stages = 1
        while any((Xp(t + stages) - Xp(t + 1)) // 2 < L for t in range(T)):
            stages += 1
    rng = random.Random(seed)
    done = [0] * T                      # stages run, per tile
    ready = lambda t: done[t] < stages and (  # noqa: E731
        done[t] == 0 or "next" not in waits or done[(t + 1) % T] >= done[t])
    while True:
        cand = [t for t in range(T) if ready(t)]
        if not cand:
            break
        t = rng.choice(cand)
        region(t, done[t])
        done[t] += 1
    assert all(d == stages for d in done)
    return list(out), visits


def unordered_conflicts(footprints, T, waits=("own", "next")):
    """Pairs of regions that the persistent kernel's two waits leave
    unordered (neither reaches the other through (t, s-1) -> (t, s) and
    (t+1, s-1) -> (t, s)) although one writes an element the other reads or
    writes.  Empty when the waits order every conflicting access."""
    stages = 1 + max(s for (_, s) in footprints)
    # below[(t, s)]: every region that (t, s) waits for, directly or not
    below = {}
    for s in range(stages):
        for t in range(T):
            b = set()
            if s > 0:
                pre = ([(t, s - 1)] if "own" in waits else []) + \
                    ([((t + 1) % T, s - 1)] if "next" in waits else [])
                for p in pre:
                    b.add(p)
                    b |= below[p]
            below[(t, s)] = b
    writes = {r: {(a, i) for (a, i, k) in f if k == "w"} for r, f in footprints.items()}
    touches = {r: {(a, i) for (a, i, _) in f} for r, f in footprints.items()}
    bad = []
    regions = sorted(footprints)
    for x in regions:
        for y in regions:
            if x >= y or x in below[y] or y in below[x]:
                continue
            if writes[x] & touches[y] or writes[y] & touches[x]:
                bad.append((x, y))
    return bad
