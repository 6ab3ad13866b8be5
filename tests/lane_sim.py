"""CPU emulation of the lane-frame stage kernel (tests only).

Mirrors swept_lane_kernel with field writes: one 64-lane wavefront per
region, lane l holding column dx = l - o (o = k + 1 for k <= 31, o = 32 for
k = 32); a row's neighbours come from wave shifts by one lane (the lane with
no source receives zero, or, for the middle row at k = 32, the V-edge value
of the column outside the wave); the V edges enter at two rows per column;
the rows from the middle level up keep their own points for the edge
copy-out; the top row writes the field when it is the target level.  The
stage geometry (drifting regions, edge buffers RE and LE) is the one of
tests/swept_sim.py.
"""
from __future__ import annotations

LANES = 64


def _frame(k):
    return k + 1 if k + 1 < 32 else 32


def _zero(v):
    return tuple(0.0 for _ in v) if isinstance(v, tuple) else 0.0


def _shr(v, old=None):
    """lane i receives lane i-1; lane 0 receives `old` (zero if None)."""
    return [old if old is not None else _zero(v[0])] + v[:-1]


def _shl(v, old=None):
    """lane i receives lane i+1; lane 63 receives `old` (zero if None)."""
    return v[1:] + [old if old is not None else _zero(v[0])]


def simulate_lane(u0, nsteps, k, stencil, track=False):
    step, nph, from_field, to_field = stencil
    n = len(u0)
    W = 2 * k
    assert n % W == 0 and 1 <= k <= 32
    T = n // W
    L = nsteps * nph
    u = list(u0)
    visits = {} if track else None
    if L == 0:
        return u, visits
    stages = 1 + (L + k - 1) // k
    o = _frame(k)
    wide = o == k
    RE = [[None] * (2 * k) for _ in range(T)]
    LE = [[[None] * (2 * k) for _ in range(T)] for _ in range(2)]
    for s in range(stages):
        tri = s == 0
        b = (s - 1) * k
        J0 = (k + s * k) % n
        le_in, le_out = LE[(s + 1) % 2], LE[s % 2]
        new_re = [None] * T
        for t in range(T):
            J = (t * W + J0) % n
            jtop = min(2 * k - 1, L - b)
            dxs = [lane - o for lane in range(LANES)]
            iA = [(-dx - 2) if dx < 0 else dx for dx in dxs]
            iB = [(-dx - 1) if dx < 0 else dx - 1 for dx in dxs]
            v = [0.0] * LANES
            eA = [None] * LANES
            eB = [None] * LANES
            oL = oR = None
            U = {}   # (row, column) -> point, rows from the middle level up
            if tri:
                j0 = k
                z = from_field(0.0)
                v = [from_field(u[J + dx]) if -k <= dx <= k - 1 else z for dx in dxs]
                for lane, dx in enumerate(dxs):
                    if -k <= dx <= k - 1:
                        U[(k, dx)] = v[lane]
            else:
                j0 = 0
                re = RE[t]
                le = le_in[(t + 1) % T]
                for lane, dx in enumerate(dxs):
                    if 0 <= iA[lane] < k:
                        eA[lane] = re[2 * iA[lane]] if dx < 0 else le[2 * iA[lane]]
                    if 0 <= iB[lane] < k:
                        eB[lane] = re[2 * iB[lane] + 1] if dx < 0 else le[2 * iB[lane] + 1]
                if wide:
                    oL, oR = re[2 * (k - 1)], le[2 * (k - 1) + 1]
                v = [eA[i] if iA[i] == 0 else eB[i] for i in range(LANES)]
                z = from_field(0.0)
                v = [z if x is None else x for x in v]

            def row(j, old_l=None, old_r=None):
                nonlocal v
                ph = (b + j - 1) % nph
                lv, rv = _shr(v, old_l), _shl(v, old_r)
                out = []
                for i in range(LANES):
                    try:
                        out.append(step(ph, lv[i], v[i], rv[i]))
                    except (OverflowError, ZeroDivisionError):
                        out.append(v[i])   # a lane outside the region: never read
                return out

            for j in range(j0 + 1, min(k - 1, jtop) + 1):         # below the middle
                o_row = row(j)
                v = [eA[i] if iA[i] == j else (eB[i] if iB[i] == j else o_row[i])
                     for i in range(LANES)]
                if track:
                    for i, dx in enumerate(dxs):
                        if -j <= dx <= j - 1:
                            key = ((J + dx) % n, b + j)
                            visits[key] = visits.get(key, 0) + 1
            for j in range(max(k, j0 + 1), jtop + 1):               # the middle row up
                if j == k:
                    v = row(j, oL if wide else None, oR if wide else None)
                else:
                    v = row(j)
                for i, dx in enumerate(dxs):
                    if j - 2 * k <= dx <= 2 * k - 1 - j:
                        U[(j, dx)] = v[i]
                        if track:
                            key = ((J + dx) % n, b + j)
                            visits[key] = visits.get(key, 0) + 1
            if b + jtop == L and jtop > j0:                         # the target level
                for i, dx in enumerate(dxs):
                    own = (-jtop <= dx <= jtop - 1) if jtop <= k else \
                        (jtop - 2 * k <= dx <= 2 * k - 1 - jtop)
                    if own:
                        u[(J + dx) % n] = to_field(v[i])
            re_out = list(RE[t])
            lo = list(le_out[t])
            for j in range(k, jtop + 1):
                i = j - k
                re_out[2 * i] = U[(j, 2 * k - 2 - j)]
                re_out[2 * i + 1] = U[(j, 2 * k - 1 - j)]
                lo[2 * i] = U[(j, j - 2 * k)]
                lo[2 * i + 1] = U[(j, j - 2 * k + 1)]
            new_re[t] = re_out
            le_out[t] = lo
        for t in range(T):
            RE[t] = new_re[t]
    return u, visits
