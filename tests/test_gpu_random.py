"""Randomised GPU parity: seeded random launch configurations (tile width,
pairs per lane, schedule mode, step count) for every stencil, the batch and
the adjoint, each against the CPU oracle bit for bit.

The step counts are drawn around multiples of the sweep depth k (k-1, k,
k+1, 2k-1, ...), where the stage structure changes: the triangle alone, a
last stage capped inside its lower half, a full diamond whose apex is the
target level.  The configurations are fixed by the seed, so a failure names
a reproducible case in its test id."""
import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

HEAT_R = 0.3
KS_P = [workloads.KS_DT, workloads.KS_DX]


def _steps_near(g, k, per_step, top):
    """A step count whose sub-timestep count lies near a multiple of k."""
    m = int(g.integers(0, 4))
    d = int(g.choice([-1, 0, 1]))
    levels = max(0, m * k + d)
    if g.random() < 0.25:
        levels = int(g.integers(0, 4 * k + 2))
    return min(top, -(-levels // per_step))


def _cases(stencil, count, seed, ks, ps, nmax, top, modes=(1, 3, 0)):
    # modes: stage, stage with the banded kernel only, automatic (4: the
    # lane-frame kernel, k <= 32)
    g = np.random.default_rng(seed)
    per_step = 1 if stencil.startswith("heat") else 4
    out = []
    for _ in range(count):
        k = int(g.choice(ks))
        T = int(g.integers(1, max(2, nmax // (2 * k)) + 1))
        T = max(1, min(T, nmax // (2 * k)))
        out.append((2 * k * T, 2 * k, int(g.choice(ps)), int(g.choice(modes)),
                    _steps_near(g, k, per_step, top)))
    return out


def _ids(cases):
    return ["n%d-W%d-P%d-m%d-s%d" % c for c in cases]


@pytest.fixture(scope="module")
def sw():
    import paper_1504_01380_amd as swept
    swept.init(0)
    yield swept
    swept.set_tuning(0, 0, swept.MODE_AUTO)


def _run(sw, u0, nsteps, stencil, params):
    import torch
    u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    sw.advance(u, nsteps, stencil, params)
    torch.cuda.synchronize()
    sw.sync()
    return u.cpu().numpy()


def _same(a, b):
    return a.dtype == b.dtype and a.shape == b.shape and \
        np.array_equal(a.view(np.uint8), b.view(np.uint8))


HEAT = _cases("heat", 40, 2024, [1, 2, 3, 5, 8, 16, 32, 64, 96, 128, 256], [1, 2, 4, 8], 8192, 1100)
HEAT32 = _cases("heat32", 12, 2025, [4, 16, 64, 128, 256], [1, 2, 4, 8], 8192, 1100)
KS = _cases("ks", 24, 2026, [1, 2, 4, 8, 12, 16, 64, 128, 256], [1, 2, 4], 4096, 300)
EULER = _cases("euler", 12, 2027, [2, 4, 8, 16, 64, 128], [1, 2], 2048, 70)
LANE = ([("heat",) + c for c in _cases("heat", 16, 2030, [1, 2, 3, 5, 8, 16, 31, 32], [1], 4096,
                                        400, modes=(4,))] +
        [("ks",) + c for c in _cases("ks", 12, 2031, [1, 2, 4, 8, 13, 16, 32], [1], 4096, 100,
                                      modes=(4,))] +
        [("euler",) + c for c in _cases("euler", 6, 2032, [2, 4, 8, 16, 28], [1], 2048, 40,
                                         modes=(4,))])


@pytest.mark.parametrize("n,W,P,mode,nsteps", HEAT, ids=_ids(HEAT))
def test_random_heat_f64(sw, oracle_mod, n, W, P, mode, nsteps):
    sw.set_tuning(W, P, mode)
    try:
        u0 = workloads.white_noise(n, seed=n + W + nsteps)
        assert _same(_run(sw, u0, nsteps, "heat", [HEAT_R]), oracle_mod.heat(u0, nsteps, HEAT_R))
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)


@pytest.mark.parametrize("n,W,P,mode,nsteps", HEAT32, ids=_ids(HEAT32))
def test_random_heat_f32(sw, oracle_mod, n, W, P, mode, nsteps):
    sw.set_tuning(W, P, mode)
    try:
        u0 = workloads.white_noise(n, seed=n + W + nsteps, dtype=np.float32)
        assert _same(_run(sw, u0, nsteps, "heat", [HEAT_R]), oracle_mod.heat(u0, nsteps, HEAT_R))
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)


@pytest.mark.parametrize("n,W,P,mode,nsteps", KS, ids=_ids(KS))
def test_random_ks(sw, oracle_mod, n, W, P, mode, nsteps):
    sw.set_tuning(W, P, mode)
    try:
        u0 = workloads.smoothed_noise(n, seed=n + W + nsteps)
        assert _same(_run(sw, u0, nsteps, "ks", KS_P), oracle_mod.ks(u0, nsteps, *KS_P))
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)


@pytest.mark.parametrize("n,W,P,mode,nsteps", EULER, ids=_ids(EULER))
def test_random_euler(sw, oracle_mod, n, W, P, mode, nsteps):
    sw.set_tuning(W, P, mode)
    try:
        q0 = workloads.euler_smooth(n, seed=n + nsteps)
        dx = 1.0 / n
        par = [workloads.EULER_CFL * dx, dx, workloads.EULER_GAMMA]
        want = oracle_mod.euler(q0, nsteps, par[0], dx, par[2])
        assert _same(_run(sw, q0, nsteps, "euler", par), want)
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)


@pytest.mark.parametrize("stencil,n,W,P,mode,nsteps", LANE,
                         ids=["%s-n%d-W%d-P%d-m%d-s%d" % c for c in LANE])
def test_random_lane_kernel(sw, oracle_mod, stencil, n, W, P, mode, nsteps):
    """Every stage on the lane-frame kernel (mode 4)."""
    sw.set_tuning(W, 0, mode)
    try:
        assert sw.plan(n, nsteps, stencil)["mode"] == sw.MODE_STAGE_LANE
        if stencil == "heat":
            u0 = workloads.white_noise(n, seed=n + W + nsteps)
            want = oracle_mod.heat(u0, nsteps, HEAT_R)
            par = [HEAT_R]
        elif stencil == "ks":
            u0 = workloads.smoothed_noise(n, seed=n + W + nsteps)
            want = oracle_mod.ks(u0, nsteps, *KS_P)
            par = KS_P
        else:
            u0 = workloads.euler_smooth(n, seed=n + nsteps)
            dx = 1.0 / n
            par = [workloads.EULER_CFL * dx, dx, workloads.EULER_GAMMA]
            want = oracle_mod.euler(u0, nsteps, par[0], dx, par[2])
        assert _same(_run(sw, u0, nsteps, stencil, par), want)
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)


def _batch_case(seed):
    g = np.random.default_rng(seed)
    count = int(g.integers(5, 16))
    insts = []
    for q in range(count):
        kind = "heat" if g.random() < 0.5 else "ks"
        n = int(g.integers(3, 3000))
        steps = int(g.integers(0, 260 if kind == "heat" else 90))
        insts.append((kind, n, steps, seed * 100 + q))
    tile = int(g.choice([0, 0, 64, 256, 512]))
    return insts, tile


BATCHES = [_batch_case(s) for s in (31, 32, 33, 34, 35, 36)]


@pytest.mark.parametrize("insts,tile", BATCHES, ids=["batch%d" % i for i in range(len(BATCHES))])
def test_random_batch(sw, oracle_mod, insts, tile):
    import torch
    sw.set_tuning(tile, 0, sw.MODE_AUTO)
    try:
        u0 = [workloads.white_noise(n, seed=sd) if kind == "heat" else
              workloads.smoothed_noise(n, seed=sd) for kind, n, _, sd in insts]
        us = [torch.from_numpy(u).cuda() for u in u0]
        pars = [[HEAT_R] if kind == "heat" else KS_P for kind, _, _, _ in insts]
        sw.advance_batch(us, [s for _, _, s, _ in insts], [k for k, _, _, _ in insts], pars)
        torch.cuda.synchronize()
        sw.sync()
        for (kind, n, steps, _), u, x in zip(insts, u0, us):
            want = oracle_mod.heat(u, steps, HEAT_R) if kind == "heat" else \
                oracle_mod.ks(u, steps, *KS_P)
            assert _same(x.cpu().numpy(), want), (kind, n, steps)
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)


def _adjoint_cases(seed, count):
    g = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kind = "heat" if g.random() < 0.4 else "ks"
        k = int(g.choice([1, 2, 3, 5, 8, 13, 16, 24, 31, 32]))
        T = int(g.integers(1, 5))
        per = 1 if kind == "heat" else 4
        steps = _steps_near(g, k, per, 120)
        first = int(g.integers(0, steps + 2))
        out.append((kind, 2 * k * T, 2 * k, steps, first, bool(g.random() < 0.5)))
    return out


ADJ = _adjoint_cases(2028, 16)


@pytest.mark.parametrize("kind,n,W,nsteps,first,with_cot", ADJ,
                         ids=["%s-n%d-W%d-s%d-f%d-c%d" % c for c in ADJ])
def test_random_adjoint(sw, oracle_mod, kind, n, W, nsteps, first, with_cot):
    import torch
    sw.set_tuning(W, 0, sw.MODE_AUTO)
    try:
        u0 = workloads.white_noise(n, seed=n + nsteps) if kind == "heat" else \
            3 * workloads.smoothed_noise(n, seed=n + nsteps)
        cot = workloads.white_noise(n, seed=n) if with_cot else None
        w = 1.0 / (5 * n)
        par = [HEAT_R] if kind == "heat" else KS_P
        c = None if cot is None else torch.from_numpy(cot).cuda()
        got = sw.adjoint(torch.from_numpy(u0).cuda(), nsteps, kind, par, window_first=first,
                         window_weight=w, cot_final=c)
        torch.cuda.synchronize()
        sw.sync()
        want = oracle_mod.heat_adjoint(u0, nsteps, HEAT_R, first, w, cot) if kind == "heat" else \
            oracle_mod.ks_adjoint(u0, nsteps, *KS_P, first, w, cot)
        assert _same(got.cpu().numpy(), want)
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)
