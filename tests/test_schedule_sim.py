"""The swept stage kernel's schedule, emulated on the CPU (tests/swept_sim.py),
must compute every (point, level) up to the target exactly once and give the
oracle's bits (paper, Section 3: the swept decomposition computes everything
exactly once, without redundancy; Section 2: the result is that of plain
stepping).  Covers the triangle, diamonds, the cap at an arbitrary level,
bands of 64*P pairs including a partial last band, one tile (T = 1), and the
four-sub-timestep KS scheme."""
import numpy as np
import pytest

import workloads
from tests import swept_sim
from tests.conftest import same_bits


@pytest.mark.parametrize("n,k,P,nsteps", [
    (16, 4, 1, 1), (16, 4, 1, 3), (16, 4, 1, 4), (16, 4, 1, 7), (16, 4, 1, 8),
    (16, 4, 1, 9), (16, 4, 1, 29), (48, 8, 1, 50), (32, 16, 1, 33), (12, 6, 1, 40),
    (20, 1, 1, 5), (40, 2, 2, 13), (24, 3, 1, 17),
])
def test_heat_exactly_once_and_bitwise(oracle_mod, n, k, P, nsteps):
    u0 = workloads.white_noise(n, seed=n + k)
    got, visits = swept_sim.simulate(list(u0), nsteps, k, P, swept_sim.heat_step(0.25),
                                     lanes=64, track=True)
    ok, why = swept_sim.levels_complete(visits, n, nsteps, k)
    assert ok, why
    want = oracle_mod.heat(u0, nsteps, 0.25)
    assert same_bits(np.array(got), want)


@pytest.mark.parametrize("lanes,P,k,nsteps", [
    (4, 1, 10, 37),   # bands of 4 pairs, partial last band (10 = 4+4+2)
    (4, 2, 12, 40),   # bands of 8 pairs, partial last band
    (2, 2, 8, 21),    # full bands
    (3, 1, 7, 30),    # odd band size
])
def test_heat_multiband(oracle_mod, lanes, P, k, nsteps):
    n = 4 * k
    u0 = workloads.white_noise(n, seed=lanes * 100 + k)
    got, visits = swept_sim.simulate(list(u0), nsteps, k, P, swept_sim.heat_step(0.3),
                                     lanes=lanes, track=True)
    ok, why = swept_sim.levels_complete(visits, n, nsteps, k)
    assert ok, why
    assert same_bits(np.array(got), oracle_mod.heat(u0, nsteps, 0.3))


@pytest.mark.parametrize("lanes,P,k,nsteps", [(64, 1, 8, 9), (4, 2, 12, 11), (64, 2, 6, 5)])
def test_ks_bitwise(oracle_mod, lanes, P, k, nsteps):
    n = 4 * k
    u0 = workloads.smoothed_noise(n, seed=k)
    got, visits = swept_sim.simulate(list(u0), nsteps, k, P, swept_sim.ks_step(0.005, 0.5),
                                     lanes=lanes, track=True)
    ok, why = swept_sim.levels_complete(visits, n, 4 * nsteps, k)
    assert ok, why
    assert same_bits(np.array(got), oracle_mod.ks(u0, nsteps, 0.005, 0.5))


def test_dropped_update_is_caught(oracle_mod):
    """A schedule that skips one wave step must fail the exactly-once check."""
    n, k, nsteps = 16, 4, 9
    u0 = workloads.white_noise(n, seed=1)
    step, nph, ff, tf = swept_sim.heat_step(0.25)
    calls = {"n": 0}

    def skipping(ph, l, c, r):
        calls["n"] += 1
        return c if calls["n"] == 37 else step(ph, l, c, r)

    got, _ = swept_sim.simulate(list(u0), nsteps, k, 1, (skipping, nph, ff, tf), track=True)
    assert not same_bits(np.array(got), oracle_mod.heat(u0, nsteps, 0.25))


@pytest.mark.parametrize("lanes,P,k,nsteps,stencil", [
    (2, 1, 2, 20, "heat"),     # one band (k = 64P)
    (2, 1, 4, 30, "heat"),     # two bands
    (2, 2, 12, 61, "heat"),    # three bands of 4 pairs
    (4, 1, 16, 100, "heat"),   # four bands
    (3, 1, 9, 40, "heat"),     # odd band size
    (2, 2, 8, 30, "ks"),       # KS: k and 64P multiples of 4 in the kernel; here 4 | k, 4 | NB
    (4, 1, 8, 25, "ks"),
])
def test_continuous_schedule(oracle_mod, lanes, P, k, nsteps, stencil):
    """Full diamonds on the continuous-band schedule: exactly once, bitwise."""
    n = 3 * 2 * k
    if stencil == "heat":
        u0 = workloads.white_noise(n, seed=k * 10 + P)
        st, L, want = swept_sim.heat_step(0.3), nsteps, oracle_mod.heat(u0, nsteps, 0.3)
    else:
        u0 = workloads.smoothed_noise(n, seed=k)
        st, L, want = swept_sim.ks_step(0.005, 0.5), 4 * nsteps, oracle_mod.ks(u0, nsteps, 0.005, 0.5)
    got, visits = swept_sim.simulate(list(u0), nsteps, k, P, st, lanes=lanes, track=True,
                                     cont=True)
    ok, why = swept_sim.levels_complete(visits, n, L, k)
    assert ok, why
    assert same_bits(np.array(got), want)


@pytest.mark.parametrize("ks_list,lanes,P,nsteps,stencil", [
    ([4, 4, 4, 2], 2, 2, 30, "heat"),    # the batch split: full tiles and a remainder
    ([8, 8, 3], 2, 1, 41, "heat"),       # two bands per full square
    ([4, 4, 4, 4, 1], 1, 4, 27, "heat"),
    ([8, 8, 8, 5], 4, 1, 19, "ks"),      # b mod 4 = 1 once the short tile is below
                                         # (KS: 4 | k and 4 | lanes*P, as in the kernel)
    ([8, 8, 6], 1, 4, 23, "ks"),         # b mod 4 = 2
    ([8, 8, 8, 8, 7], 2, 2, 17, "ks"),   # b mod 4 = 3
    ([8, 8], 2, 2, 15, "ks"),            # every region a full square
])
def test_batch_continuous_schedule(oracle_mod, ks_list, lanes, P, nsteps, stencil):
    """The batch schedule with its square regions on the continuous-band
    schedule (the others banded): exactly once, the oracle's bits, for every
    phase of the regions' base level."""
    n = 2 * sum(ks_list)
    if stencil == "heat":
        u0 = workloads.white_noise(n, seed=n + nsteps)
        st, L, want = swept_sim.heat_step(0.3), nsteps, oracle_mod.heat(u0, nsteps, 0.3)
    else:
        u0 = workloads.smoothed_noise(n, seed=n + nsteps)
        st, L = swept_sim.ks_step(0.005, 0.5), 4 * nsteps
        want = oracle_mod.ks(u0, nsteps, 0.005, 0.5)
    got, visits = swept_sim.simulate_tiles(list(u0), nsteps, ks_list, P, st, lanes=lanes,
                                           track=True, cont=True)
    ok, why = swept_sim.levels_complete(visits, n, L, max(ks_list))
    assert ok, why
    assert same_bits(np.array(got), want)


@pytest.mark.parametrize("k,T,nsteps,stencil", [
    (1, 5, 7, "heat"), (2, 3, 9, "heat"), (3, 2, 11, "heat"), (8, 3, 15, "heat"),
    (8, 2, 16, "heat"), (31, 1, 61, "heat"), (32, 2, 63, "heat"), (32, 1, 100, "heat"),
    (32, 2, 31, "heat"), (4, 3, 5, "ks"), (8, 2, 7, "ks"), (32, 2, 9, "ks"), (31, 1, 16, "ks"),
])
def test_lane_kernel_schedule(oracle_mod, k, T, nsteps, stencil):
    """The lane-frame stage kernel (every stage, field writes at the target
    level; k = 32 takes the outermost columns as DPP fallback values):
    exactly once, the oracle's bits."""
    from tests import lane_sim
    n = 2 * k * T
    if stencil == "heat":
        u0 = workloads.white_noise(n, seed=n + nsteps)
        st, L, want = swept_sim.heat_step(0.3), nsteps, oracle_mod.heat(u0, nsteps, 0.3)
    else:
        u0 = workloads.smoothed_noise(n, seed=n + nsteps)
        st, L = swept_sim.ks_step(0.005, 0.5), 4 * nsteps
        want = oracle_mod.ks(u0, nsteps, 0.005, 0.5)
    got, visits = lane_sim.simulate_lane(list(u0), nsteps, k, st, track=True)
    ok, why = swept_sim.levels_complete(visits, n, L, k)
    assert ok, why
    assert same_bits(np.array(got), want)


@pytest.mark.parametrize("nsteps", range(1, 26))
def test_continuous_schedule_every_cap(oracle_mod, nsteps):
    """The continuous schedule at every target level modulo k (k = 4): a
    diamond whose apex reaches the target level writes that level, so it
    must not run on the continuous kernel, which writes no field value
    (nsteps = 7, 11, ... once failed here)."""
    k, n = 4, 16
    u0 = workloads.white_noise(n, seed=nsteps)
    got, visits = swept_sim.simulate(list(u0), nsteps, k, 4, swept_sim.heat_step(0.3), lanes=1,
                                     track=True, cont=True)
    ok, why = swept_sim.levels_complete(visits, n, nsteps, k)
    assert ok, why
    assert same_bits(np.array(got), oracle_mod.heat(u0, nsteps, 0.3))


@pytest.mark.parametrize("stencil,n,k,nsteps,n0,cot", [
    ("heat", 16, 4, 3, 0, True), ("heat", 32, 8, 33, 20, False), ("heat", 8, 4, 13, 3, True),
    ("heat", 12, 1, 9, 2, True), ("ks", 16, 4, 5, 2, True), ("ks", 32, 4, 9, 6, False),
    ("ks", 24, 6, 7, 1, True), ("ks", 16, 2, 5, 5, True),
])
def test_adjoint_schedule(oracle_mod, stencil, n, k, nsteps, n0, cot):
    """The swept adjoint schedule (reverse stages, per-region recompute from
    one checkpoint per stage, boundary hand-over) gives the oracle's discrete
    adjoint bit for bit."""
    from tests import swept_adj_sim
    w = 1.0 / (7 * n)
    c = workloads.white_noise(n, seed=99) if cot else None
    if stencil == "heat":
        u0 = workloads.white_noise(n, seed=n + k)
        loc, want = swept_adj_sim.heat_local(0.3), oracle_mod.heat_adjoint(u0, nsteps, 0.3, n0, w, c)
    else:
        u0 = 3 * workloads.smoothed_noise(n, seed=n + k)
        loc = swept_adj_sim.ks_local(0.005, 0.5)
        want = oracle_mod.ks_adjoint(u0, nsteps, 0.005, 0.5, n0, w, c)
    got = swept_adj_sim.adjoint(list(u0), nsteps, k, loc, n0, w, None if c is None else list(c))
    assert same_bits(np.array(got), want)


def _split(half, k):
    """The batch plan's tiling of a ring of 2*half points: T = ceil(half/k)
    tiles, T-1 of half-width k and the last of the remainder."""
    T = max(1, -(-half // k))
    if T == 1:
        return [half]
    return [k] * (T - 1) + [half - (T - 1) * k]


@pytest.mark.parametrize("ks_list,nsteps,stencil", [
    ([4, 5, 4, 5], 23, "heat"),       # alternating widths
    ([3, 7, 2, 5, 6], 40, "heat"),    # arbitrary widths
    ([6], 30, "heat"),                # one tile
    ([1, 1, 2], 9, "heat"),           # k = 1 tiles
    (_split(50, 8), 61, "heat"),      # the plan's split: 6 tiles of 8 and one of 2
    ([4, 5, 4], 7, "ks"),
    (_split(21, 4), 6, "ks"),
])
def test_unequal_tiles(oracle_mod, ks_list, nsteps, stencil):
    """Tiles of unequal even widths (the batch path): every (point, level)
    exactly once, the oracle's bits."""
    n = 2 * sum(ks_list)
    if stencil == "heat":
        u0 = workloads.white_noise(n, seed=n)
        st, L, want = swept_sim.heat_step(0.25), nsteps, oracle_mod.heat(u0, nsteps, 0.25)
    else:
        u0 = workloads.smoothed_noise(n, seed=n)
        st, L, want = swept_sim.ks_step(0.005, 0.5), 4 * nsteps, oracle_mod.ks(u0, nsteps, 0.005, 0.5)
    got, visits = swept_sim.simulate_tiles(list(u0), nsteps, ks_list, 1, st, lanes=2, track=True)
    ok, why = swept_sim.levels_complete(visits, n, L, 0)
    assert ok, why
    assert same_bits(np.array(got), want)


@pytest.mark.parametrize("n,k,nsteps", [(17, 4, 30), (9, 2, 11), (3, 8, 5), (101, 16, 70)])
def test_odd_ring_on_two_fold_cover(oracle_mod, n, k, nsteps):
    """An odd ring of n points run on its 2n-point cover: the first period of
    the result is the n-point run (the scheme commutes with translation)."""
    u0 = workloads.white_noise(n, seed=n)
    cover = list(u0) + list(u0)
    got, _ = swept_sim.simulate_tiles(cover, nsteps, _split(n, k), 1, swept_sim.heat_step(0.25),
                                      lanes=4)
    want = oracle_mod.heat(u0, nsteps, 0.25)
    assert same_bits(np.array(got[:n]), want)
    assert same_bits(np.array(got[n:]), want)


@pytest.mark.parametrize("k,P,lanes", [(8, 1, 4), (16, 2, 2), (16, 1, 4), (24, 2, 2), (32, 4, 2),
                                       (64, 1, 64), (128, 1, 64), (256, 2, 64), (128, 2, 64)])
@pytest.mark.parametrize("b", [0, 1, 2, 3])
def test_continuous_face_sharing(k, P, lanes, b):
    """The continuous kernel's face sharing (Euler): each pair's update gets
    exactly the neighbours and faces it needs, and the stage leaves the
    right and left edges of the diamond."""
    out, chain = swept_sim.cont_faces_symbolic(k, P, b, lanes)
    for d in range(k):   # final states: pair d at step k-1
        assert out[2 * d] == (k - 1 - d - 1, b + k - 1 + d + 1)
        assert out[2 * d + 1] == (k - 1 - d, b + k - 1 + d + 1)
    for m in range(k):   # last pair (k-1) at step m
        assert chain[2 * m] == (m - (k - 1) - 1, b + m + k)
        assert chain[2 * m + 1] == (m - (k - 1), b + m + k)


@pytest.mark.parametrize("n,nsteps,stencil", [
    (130, 30, "heat"),    # even, no even divisor near the target: unequal tiles
    (131, 23, "heat"),    # odd: unequal tiles of the two-fold cover
    (258, 41, "heat"),
    (8198, 3, "heat"),    # the grid whose equal tiling was 2 points wide
    (129, 9, "ks"),
    (194, 7, "ks"),
])
def test_single_field_unequal_plan(oracle_mod, n, nsteps, stencil):
    """The unequal tiling the library plans for a single field without a good
    even divisor (swept_plan, host logic): T-1 tiles of half-width k and the
    remainder, of the ring or its two-fold cover; its emulated schedule
    computes every (point, level) once and gives the oracle's bits."""
    import paper_1504_01380_amd as swept
    swept.lib().swept_set_tuning(0, 0, 0)
    p = swept.plan(n, nsteps, stencil)
    assert p["mode"] == swept.MODE_STAGE_RAGGED
    ring = n if n % 2 == 0 else 2 * n
    k, T = p["depth_k"], p["tiles"]
    ks_list = _split(ring // 2, k)
    assert len(ks_list) == T and p["tile_w"] == 2 * k
    if stencil == "heat":
        u0 = workloads.white_noise(n, seed=n)
        st, L, want = swept_sim.heat_step(0.3), nsteps, oracle_mod.heat(u0, nsteps, 0.3)
    else:
        u0 = workloads.smoothed_noise(n, seed=n)
        st, L = swept_sim.ks_step(0.005, 0.5), 4 * nsteps
        want = oracle_mod.ks(u0, nsteps, 0.005, 0.5)
    field = list(u0) if ring == n else list(u0) + list(u0)
    # KS phases need the band (lanes x pairs) a multiple of 4, as 64P is on the GPU
    got, visits = swept_sim.simulate_tiles(field, nsteps, ks_list, 1, st,
                                           lanes=2 if stencil == "heat" else 4, track=True,
                                           cont=True)
    ok, why = swept_sim.levels_complete(visits, ring, L, 0)
    assert ok, why
    assert same_bits(np.array(got[:n]), want)
    # the plan launches every stage in which some tile still has a region
    # below the target level: stage s of tile t starts at (X_{t+s} - X_{t+1})/2
    X = [0]
    for kt in ks_list:
        X.append(X[-1] + 2 * kt)

    def Xp(i):
        return X[i % T] + (i // T) * ring

    last = max(s for s in range(1, 4 * L + 4)
               if any((Xp(t + s) - Xp(t + 1)) // 2 < L for t in range(T)))
    assert last + 1 <= p["stages"] <= last + 3


def _lanes(stencil):
    """Emulated lanes per band: the KS band must hold a multiple of four pairs
    (its cycles start at a fixed phase of the four sub-timesteps)."""
    return 4 if stencil == "ks" else 2


def _case(oracle_mod, stencil, n, nsteps):
    if stencil == "heat":
        u0 = workloads.white_noise(n, seed=n)
        return u0, swept_sim.heat_step(0.25), nsteps, oracle_mod.heat(u0, nsteps, 0.25)
    u0 = workloads.smoothed_noise(n, seed=n)
    return (u0, swept_sim.ks_step(0.005, 0.5), 4 * nsteps,
            oracle_mod.ks(u0, nsteps, 0.005, 0.5))


PERSIST_CASES = [
    ([3, 7, 2, 5, 6], 40, "heat", False), (_split(50, 8), 61, "heat", False),
    ([6], 30, "heat", False), ([4, 4], 19, "heat", False), ([1, 1, 2], 9, "heat", False),
    ([4, 5, 4], 7, "ks", False), (_split(21, 4), 6, "ks", False),
    ([8, 8, 8], 11, "heat", True), ([8, 8, 8, 2], 9, "ks", True),
]


@pytest.mark.parametrize("ks_list,nsteps,stencil,cont", PERSIST_CASES)
def test_persistent_waits_order_every_conflict(oracle_mod, ks_list, nsteps, stencil, cont):
    """The persistent batch kernel lets region (t, s) run as soon as stage s-1
    of tiles t and t+1 is published.  Every pair of regions those two waits
    leave unordered must touch disjoint data: no element of the field or of
    the edge buffers that one writes is read or written by the other, so
    any interleaving of concurrent regions gives the stage-by-stage bits."""
    n = 2 * sum(ks_list)
    u0, st, _, want = _case(oracle_mod, stencil, n, nsteps)
    fp = {}
    got, _ = swept_sim.simulate_tiles(list(u0), nsteps, ks_list, 1, st, lanes=_lanes(stencil),
                                      cont=cont, inplace=True, footprints=fp)
    assert same_bits(np.array(got), want)
    assert swept_sim.unordered_conflicts(fp, len(ks_list)) == []


@pytest.mark.parametrize("ks_list,nsteps,stencil,cont", PERSIST_CASES)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_persistent_orders_bitwise(oracle_mod, ks_list, nsteps, stencil, cont, seed):
    """Regions run in random orders that respect only the two waits, on one
    in-place field: every (point, level) exactly once, the oracle's bits."""
    n = 2 * sum(ks_list)
    u0, st, L, want = _case(oracle_mod, stencil, n, nsteps)
    got, visits = swept_sim.simulate_tiles(list(u0), nsteps, ks_list, 1, st,
                                           lanes=_lanes(stencil), track=True, cont=cont,
                                           order="random", seed=seed, inplace=True)
    ok, why = swept_sim.levels_complete(visits, n, L, 0)
    assert ok, why
    assert same_bits(np.array(got), want)


@pytest.mark.parametrize("n,k,nsteps,stencil", [(100, 8, 61, "heat"), (42, 4, 6, "ks"),
                                                (34, 17, 20, "heat")])
def test_persistent_host_stage_bound(oracle_mod, n, k, nsteps, stencil):
    """The batch host's stage count 2 + (L + k - rem) T / h, run by every tile
    of the plan's split in a random order, completes the instance."""
    ks_list = _split(n // 2, k)
    u0, st, L, want = _case(oracle_mod, stencil, n, nsteps)
    T, h, rem = len(ks_list), n // 2, ks_list[-1]
    kt = ks_list[0] if T > 1 else h
    stages = 2 + (L + kt - rem) * T // h
    got, visits = swept_sim.simulate_tiles(list(u0), nsteps, ks_list, 1, st,
                                           lanes=_lanes(stencil), track=True, order="random",
                                           seed=n, inplace=True, stages=stages)
    ok, why = swept_sim.levels_complete(visits, n, L, 0)
    assert ok, why
    assert same_bits(np.array(got), want)


def test_persistent_without_the_next_wait_is_caught(oracle_mod):
    """Planted in the emulation: with only the own-tile wait, regions that
    read a neighbour's edge are left unordered against the region that
    writes it -- the footprint check names them, and a random order gives
    wrong bits or runs a region before its input exists."""
    ks_list, nsteps = [4, 4, 4], 20
    n = 2 * sum(ks_list)
    u0, st, _, want = _case(oracle_mod, "heat", n, nsteps)
    fp = {}
    swept_sim.simulate_tiles(list(u0), nsteps, ks_list, 1, st, lanes=2, inplace=True,
                             footprints=fp)
    assert swept_sim.unordered_conflicts(fp, len(ks_list), waits=("own",))
    wrong = 0
    for seed in range(5):
        try:
            got, _ = swept_sim.simulate_tiles(list(u0), nsteps, ks_list, 1, st, lanes=2,
                                              order="random", seed=seed, inplace=True,
                                              waits=("own",))
            wrong += not same_bits(np.array(got), want)
        except TypeError:      # an edge read before any region wrote it (None)
            wrong += 1
    assert wrong > 0
