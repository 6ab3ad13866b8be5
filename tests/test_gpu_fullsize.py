"""Parity at the benchmark sizes, in the launch configuration bench.py times
(automatic tuning): outputs the oracle can evaluate one at a time from their
cone of dependence (paper, Section 2: after n sub-timesteps a point depends
only on the points within n edges), plus whole-field bitwise agreement of the
swept and the naive GPU schedules, whose own parity with the oracle the
smaller tests establish."""
import math

import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def sw():
    import paper_1504_01380_amd as swept
    swept.init(0)
    swept.set_tuning(0, 0, swept.MODE_AUTO)
    return swept


def gpu_run(sw, fn, u0, nsteps, stencil, params):
    import torch
    u = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda")
    fn(u, nsteps, stencil, params)
    torch.cuda.synchronize()
    sw.sync()
    return u.cpu().numpy()


def sample_indices(n, tile, seed):
    g = workloads.rng(seed)
    picks = [0, 1, tile - 1, tile, n // 2 + tile // 2, n - 1]
    return np.array(sorted(set(picks + list(g.integers(0, n, size=2)))), dtype=np.int64)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_heat_large_full_size(sw, oracle_mod, dtype):
    w = workloads.WORKLOADS["heat_large"]
    n, nsteps = w["n"], w["nsteps"]
    u0 = workloads.initial("heat_large", dtype=dtype)
    plan = sw.plan(n, nsteps, "heat", None if dtype == np.float64 else __import__("torch").float32)
    print("heat N=%d steps=%d %s plan=%s" % (n, nsteps, np.dtype(dtype).name, plan), flush=True)
    swept = gpu_run(sw, sw.advance, u0, nsteps, "heat", [w["r"]])
    idx = sample_indices(n, plan["tile_w"], 77)
    want = oracle_mod.heat_points(u0, nsteps, w["r"], idx)
    assert np.array_equal(swept[idx].view(np.uint8), want.view(np.uint8))
    naive = gpu_run(sw, sw.naive_advance, u0, nsteps, "heat", [w["r"]])
    assert np.array_equal(swept.view(np.uint8), naive.view(np.uint8))


@pytest.mark.parametrize("tile_w,ppl", [(0, 0), (512, 2)])   # default; the tuned bench tiling
def test_ks_full_size(sw, oracle_mod, tile_w, ppl):
    w = workloads.WORKLOADS["ks"]
    n, nsteps, par = w["n"], w["nsteps"], [w["dt"], w["dx"]]
    u0 = workloads.initial("ks")
    sw.set_tuning(tile_w, ppl, sw.MODE_AUTO)
    plan = sw.plan(n, nsteps, "ks")
    print("ks N=%d steps=%d plan=%s" % (n, nsteps, plan), flush=True)
    swept = gpu_run(sw, sw.advance, u0, nsteps, "ks", par)
    naive = gpu_run(sw, sw.naive_advance, u0, nsteps, "ks", par)
    assert np.array_equal(swept.view(np.uint8), naive.view(np.uint8))
    assert np.all(np.isfinite(swept))
    # the grid sum is conserved up to rounding (both D1 and D2 telescope)
    assert abs(math.fsum(swept) - math.fsum(u0)) < 1e-6
    # oracle, one output at a time, on a shorter horizon of the same run
    short = 2000
    got = gpu_run(sw, sw.advance, u0, short, "ks", par)
    idx = sample_indices(n, plan["tile_w"], 78)
    want = oracle_mod.ks_points(u0, short, *par, idx)
    assert np.array_equal(got[idx].view(np.uint8), want.view(np.uint8))
    sw.set_tuning(0, 0, sw.MODE_AUTO)


def test_ks_adjoint_full_grid(sw, oracle_mod):
    """The KS adjoint workload's grid (N = 2^16) on a shorter horizon: the
    swept adjoint equals the oracle's discrete adjoint bit for bit."""
    import torch
    w = workloads.WORKLOADS["ks_adjoint"]
    n, par = w["n"], [w["dt"], w["dx"]]
    nsteps, window = 600, 100
    u0 = workloads.initial("ks_adjoint")
    wgt = 1.0 / (window * n)
    first = nsteps - window + 1
    print("ks adjoint N=%d steps=%d" % (n, nsteps), flush=True)
    g = sw.adjoint(torch.from_numpy(u0).cuda(), nsteps, "ks", par, window_first=first,
                   window_weight=wgt)
    torch.cuda.synchronize()
    want = oracle_mod.ks_adjoint(u0, nsteps, *par, first, wgt)
    assert np.array_equal(g.cpu().numpy().view(np.uint8), want.view(np.uint8))


def test_ks_adjoint_workload_matches_oracle(sw, oracle_mod):
    """The full adjoint workload: N = 2^16, 20,000 KS steps, J = mean of u^2
    over the final 2,000 steps.  The swept adjoint's gradient equals the
    oracle's discrete adjoint bit for bit."""
    import torch
    w = workloads.WORKLOADS["ks_adjoint"]
    n, nsteps, par, window = w["n"], w["nsteps"], [w["dt"], w["dx"]], 2000
    u0 = workloads.initial("ks_adjoint")
    wgt = 1.0 / (window * n)
    first = nsteps - window + 1
    print("ks adjoint N=%d steps=%d window=%d" % (n, nsteps, window), flush=True)
    g = sw.adjoint(torch.from_numpy(u0).cuda(), nsteps, "ks", par, window_first=first,
                   window_weight=wgt)
    torch.cuda.synchronize()
    want = oracle_mod.ks_adjoint(u0, nsteps, *par, first, wgt)
    assert np.array_equal(g.cpu().numpy().view(np.uint8), want.view(np.uint8))


def _device_equal(a, b):
    import torch
    return bool(torch.equal(a.view(torch.int64), b.view(torch.int64)))


def test_heat_maximum_size(sw, oracle_mod):
    """2^28 points (2 GiB binary64, 262,144 tiles at W = 1024), 256 steps:
    sampled outputs against the oracle's cones of dependence (tile edges, the
    wrap-around, random points) and the whole field against the naive
    schedule, compared on the device."""
    import torch
    n, nsteps = 1 << 28, 256
    u0 = workloads.white_noise(n, seed=2028)
    plan = sw.plan(n, nsteps, "heat")
    print("heat N=2^28 plan=%s" % (plan,), flush=True)
    a = torch.from_numpy(u0).cuda()
    b = a.clone()
    sw.advance(a, nsteps, "heat", [0.25])
    sw.naive_advance(b, nsteps, "heat", [0.25])
    torch.cuda.synchronize()
    sw.sync()
    assert _device_equal(a, b)
    idx = sample_indices(n, plan["tile_w"], 88)
    want = oracle_mod.heat_points(u0, nsteps, 0.25, idx)
    got = a[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.array_equal(got.view(np.uint8), want.view(np.uint8))


def test_ks_maximum_size(sw, oracle_mod):
    """KS at 2^26 points (512 MiB), 100 steps: sampled outputs against the
    oracle and the whole field against the naive schedule."""
    import torch
    n, nsteps, par = 1 << 26, 100, [workloads.KS_DT, workloads.KS_DX]
    u0 = workloads.smoothed_noise(n, seed=2026)
    plan = sw.plan(n, nsteps, "ks")
    print("ks N=2^26 plan=%s" % (plan,), flush=True)
    a = torch.from_numpy(u0).cuda()
    b = a.clone()
    sw.advance(a, nsteps, "ks", par)
    sw.naive_advance(b, nsteps, "ks", par)
    torch.cuda.synchronize()
    sw.sync()
    assert _device_equal(a, b)
    idx = sample_indices(n, plan["tile_w"], 89)
    want = oracle_mod.ks_points(u0, nsteps, *par, idx)
    got = a[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.array_equal(got.view(np.uint8), want.view(np.uint8))


def test_euler_large_size(sw):
    """Euler at 2^24 cells (400 MB of state), 50 steps from the periodic Sod
    problem: the swept and naive schedules agree bit for bit and the totals
    of mass, momentum and energy are conserved to rounding (the oracle's
    parity is established at the smaller sizes and the full workload)."""
    import torch
    n, nsteps = 1 << 24, 50
    par = [workloads.EULER_CFL / n, 1.0 / n, workloads.EULER_GAMMA]
    q0 = torch.from_numpy(workloads.euler_mirrored_sod(n)).cuda()
    a = q0.clone()
    b = q0.clone()
    sw.advance(a, nsteps, "euler", par)
    sw.naive_advance(b, nsteps, "euler", par)
    torch.cuda.synchronize()
    sw.sync()
    assert _device_equal(a, b)
    s0, s1 = q0.sum(dim=0), a.sum(dim=0)
    assert torch.allclose(s1, s0, rtol=1e-12, atol=1e-9)
