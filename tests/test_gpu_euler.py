"""The Euler finite-volume stencil (three conserved variables, four
sub-timesteps) on the swept and naive paths: bit for bit the oracle's
result, on the periodic Sod problem and on smooth random states."""
import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available, same_bits

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

GAMMA = workloads.EULER_GAMMA


@pytest.fixture(scope="module")
def sw():
    import paper_1504_01380_amd as swept
    swept.init(0)
    swept.set_tuning(0, 0, swept.MODE_AUTO)
    yield swept
    swept.set_tuning(0, 0, swept.MODE_AUTO)


def params(n):
    dx = 1.0 / n
    return [workloads.EULER_CFL * dx, dx, GAMMA]


def run(sw, fn, q0, nsteps):
    import torch
    q = torch.from_numpy(q0.copy()).cuda()
    fn(q, nsteps, "euler", params(q0.shape[0]))
    torch.cuda.synchronize()
    sw.sync()
    return q.cpu().numpy()


def want(oracle_mod, q0, nsteps):
    dt, dx, gamma = params(q0.shape[0])      # the very parameters the GPU run gets
    return oracle_mod.euler(q0, nsteps, dt, dx, gamma)


@pytest.mark.parametrize("n,W,P,nsteps,ic", [
    (64, 16, 1, 1, "sod"), (64, 16, 1, 3, "smooth"), (64, 8, 1, 17, "sod"),
    (256, 64, 1, 40, "smooth"), (512, 256, 2, 70, "sod"), (1024, 512, 1, 130, "smooth"),
    (1024, 256, 2, 257, "sod"), (600, 200, 1, 77, "smooth"), (4096, 512, 2, 300, "sod"),
    (2048, 128, 1, 1000, "smooth"),
])
@pytest.mark.parametrize("mode", ["stage", "banded"])
def test_euler_swept_bitwise(sw, oracle_mod, n, W, P, nsteps, ic, mode):
    sw.set_tuning(W, P, sw.MODE_STAGE if mode == "stage" else sw.MODE_STAGE_BANDED)
    q0 = workloads.euler_mirrored_sod(n) if ic == "sod" else workloads.euler_smooth(n, seed=n + W)
    got = run(sw, sw.advance, q0, nsteps)
    assert np.array_equal(got.view(np.uint8), want(oracle_mod, q0, nsteps).view(np.uint8))
    sw.set_tuning(0, 0, sw.MODE_AUTO)


@pytest.mark.parametrize("n,nsteps", [(64, 30), (1000, 25), (5, 3), (4096, 200)])
def test_euler_naive_bitwise(sw, oracle_mod, n, nsteps):
    q0 = workloads.euler_smooth(n, seed=n)
    w = want(oracle_mod, q0, nsteps)
    assert same_bits(run(sw, sw.naive_advance, q0, nsteps), w)
    assert same_bits(run(sw, sw.naive_substep_advance, q0, nsteps), w)


def test_euler_auto_plan_and_odd_grid(sw, oracle_mod):
    import torch
    p = sw.plan(1 << 20, 100, "euler", torch.float64)
    assert p["mode"] == sw.MODE_STAGE and p["tile_w"] * 72 <= 64 * 1024
    q0 = workloads.euler_mirrored_sod(1001)            # odd: unequal tiles of the cover
    assert same_bits(run(sw, sw.advance, q0, 60), want(oracle_mod, q0, 60))


def test_euler_rejects_bad_shapes_and_params(sw):
    import torch
    import paper_1504_01380_amd as swmod
    with pytest.raises(ValueError):
        sw.advance(torch.zeros(300, dtype=torch.float64, device="cuda"), 3, "euler", params(100))
    q = torch.from_numpy(workloads.euler_mirrored_sod(64)).cuda()
    with pytest.raises(swmod.SweptError):
        sw.advance(q, 3, "euler", [1e-3, 1 / 64, 1.0])      # gamma must exceed 1
    with pytest.raises(swmod.SweptError):
        sw.advance(q, 3, "euler", [1e-3, 1 / 64])           # three parameters
    sw.set_tuning(64, 4, sw.MODE_STAGE)
    with pytest.raises(swmod.SweptError):
        sw.advance(q, 3, "euler", params(64))               # at most two pairs per lane
    sw.set_tuning(0, 0, sw.MODE_AUTO)


def test_euler_workload_full_size(sw, oracle_mod):
    """The Euler workload (periodic Sod, 2^20 cells, 10,000 steps) in the
    automatic launch configuration against the full oracle run."""
    w = workloads.WORKLOADS["euler"]
    n, nsteps = w["n"], w["nsteps"]
    q0 = workloads.initial("euler")
    got = run(sw, sw.advance, q0, nsteps)
    dt, dx, gamma = params(n)
    ref = oracle_mod.euler(q0, nsteps, dt, dx, gamma, threads=oracle_mod.max_threads())
    assert same_bits(got, ref)
    # the tiling the benchmark's autotuner picks (W = 256, one pair per lane)
    sw.set_tuning(256, 1, sw.MODE_STAGE)
    try:
        assert same_bits(run(sw, sw.advance, q0, nsteps), ref)
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)


def test_euler_small_workload_full_size(sw, oracle_mod):
    """The small Euler workload (periodic Sod, 4096 cells, 10,000 steps)
    against the full oracle run, in the automatic configuration and on the
    lane-frame kernel at the tilings the autotuner weighs for it (W = 32 and
    16: each face flux computed once and handed to the next lane)."""
    w = workloads.WORKLOADS["euler_small"]
    n, nsteps = w["n"], w["nsteps"]
    q0 = workloads.initial("euler_small")
    dt, dx, gamma = params(n)
    ref = oracle_mod.euler(q0, nsteps, dt, dx, gamma, threads=oracle_mod.max_threads())
    assert same_bits(run(sw, sw.advance, q0, nsteps), ref)
    try:
        for W in (32, 16):
            sw.set_tuning(W, 0, sw.MODE_STAGE_LANE)
            assert same_bits(run(sw, sw.advance, q0, nsteps), ref), W
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)
