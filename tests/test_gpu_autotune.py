"""The autotuner (Eq. (1) prior plus timed probes): the model it measures is
consistent, the choice it keeps is used by later automatic advances, and
results never depend on it (every tuned run equals the oracle bit for bit)."""
import math

import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available, same_bits

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

KS_P = [workloads.KS_DT, workloads.KS_DX]


@pytest.fixture()
def sw():
    import paper_1504_01380_amd as swept
    swept.init(0)
    swept.set_tuning(0, 0, swept.MODE_AUTO)
    swept.clear_tuning()
    yield swept
    swept.clear_tuning()
    swept.set_tuning(0, 0, swept.MODE_AUTO)


@pytest.mark.parametrize("stencil,n,nsteps", [("heat", 4096, 3000), ("ks", 8192, 700),
                                              ("heat", 3 * 2048, 500)])
def test_autotune_choice_is_used_and_exact(sw, oracle_mod, stencil, n, nsteps):
    import torch
    par = [0.25] if stencil == "heat" else KS_P
    rep = sw.autotune(n, nsteps, stencil, par)
    print(rep, flush=True)
    assert rep["tau"] > 0 and rep["s1"] > 0 and rep["s_full"] > 0
    assert rep["s_full"] < rep["s1"]          # the chip is faster than one wavefront
    assert math.isclose(rep["n_star"], math.sqrt(2 * rep["tau"] / rep["s1"]), rel_tol=1e-12)
    assert rep["w0"] >= rep["n_star"] * (1 - 1e-12)
    p = sw.plan(n, nsteps, stencil, torch.float64)
    if rep["tile_w"] == 0:
        assert p["mode"] == sw.MODE_NAIVE
    else:
        assert n % rep["tile_w"] == 0
        assert (p["tile_w"], p["pairs_per_lane"]) == (rep["tile_w"], rep["pairs_per_lane"])
        # pairs per lane 0: the lane-frame kernel was fastest
        assert p["mode"] == (sw.MODE_STAGE_LANE if rep["pairs_per_lane"] == 0 else sw.MODE_STAGE)
    u0 = workloads.white_noise(n, seed=n) if stencil == "heat" else \
        workloads.smoothed_noise(n, seed=n)
    u = torch.from_numpy(u0).cuda()
    sw.advance(u, nsteps, stencil, par)
    want = oracle_mod.heat(u0, nsteps, 0.25) if stencil == "heat" else \
        oracle_mod.ks(u0, nsteps, *KS_P)
    assert same_bits(u.cpu().numpy(), want)
    sw.clear_tuning()
    assert sw.plan(n, nsteps, stencil, torch.float64)["mode"] == sw.MODE_STAGE


def test_autotune_batch(sw, oracle_mod):
    import torch
    insts = workloads.batch(count=40, seed=11, nmin=64, nmax=2000, smin=20, smax=200)
    sizes = [i.n for i in insts]
    steps = [i.nsteps for i in insts]
    kinds = [i.stencil for i in insts]
    pars = [[0.25] if k == "heat" else KS_P for k in kinds]
    depth = sw.autotune_batch(sizes, steps, kinds, pars)
    print(depth, flush=True)
    assert set(depth) == set(kinds)
    assert all(k in (128, 256, 384, 512) for k in depth.values())
    us = [torch.from_numpy(i.u0).cuda() for i in insts]
    sw.advance_batch(us, steps, kinds, pars)
    torch.cuda.synchronize()
    for i, u in zip(insts, us):
        want = oracle_mod.heat(i.u0, i.nsteps, 0.25) if i.stencil == "heat" else \
            oracle_mod.ks(i.u0, i.nsteps, *KS_P)
        assert same_bits(u.cpu().numpy(), want)
