"""GPU parity: the HIP paths, called through the C ABI, against the CPU oracle.

Bar: bit-exact.  All paths evaluate the same per-point operations on the same
operands in binary64 / binary32 with no fused multiply-add, so the swept
schedule, the naive schedules and the oracle must agree bit for bit (paper,
Section 3: the swept rule only reorders the computation)."""
import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

HEAT_P = [0.25]
KS_P = [workloads.KS_DT, workloads.KS_DX]


@pytest.fixture(scope="module")
def sw():
    import paper_1504_01380_amd as swept
    swept.init(0)
    yield swept
    swept.set_tuning(0, 0, swept.MODE_AUTO)


@pytest.fixture(autouse=True)
def _reset_tuning(sw):
    sw.set_tuning(0, 0, sw.MODE_AUTO)
    yield
    sw.set_tuning(0, 0, sw.MODE_AUTO)


def run(sw, fn, u0, nsteps, stencil, params):
    import torch
    u = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda")
    fn(u, nsteps, stencil, params)
    torch.cuda.synchronize()
    sw.sync()
    return u.cpu().numpy()


def same_bits(a, b):
    return a.dtype == b.dtype and a.shape == b.shape and \
        np.array_equal(a.view(np.uint8), b.view(np.uint8))


# ---------------------------------------------------------------- heat f64

@pytest.mark.parametrize("n,W,P,nsteps", [
    (64, 16, 1, 1), (64, 16, 1, 7), (64, 16, 1, 8), (64, 16, 1, 9), (64, 16, 1, 100),
    (96, 32, 1, 333), (256, 64, 1, 129), (512, 128, 1, 500), (512, 256, 2, 257),
    (2048, 512, 4, 1000), (4096, 1024, 4, 700), (4096, 2048, 8, 2049), (4096, 4096, 4, 3000),
    (640, 320, 2, 777),     # k = 160: partial last band with P = 2
    (1000, 200, 1, 401),    # k = 100 > 64: two bands, the second partial
    (40, 2, 1, 23),         # k = 1
    (30, 10, 1, 60),
    # the apex of a full diamond at the target level (nsteps = k - 1 mod k):
    # that stage must write the field, so it is not a continuous-kernel stage
    (512, 128, 1, 127), (512, 128, 1, 191), (2048, 512, 4, 767), (4096, 1024, 4, 1535),
])
def test_heat_f64_swept_bitwise(sw, oracle_mod, n, W, P, nsteps):
    sw.set_tuning(W, P, sw.MODE_STAGE)
    u0 = workloads.white_noise(n, seed=n * 7 + W)
    got = run(sw, sw.advance, u0, nsteps, "heat", HEAT_P)
    assert same_bits(got, oracle_mod.heat(u0, nsteps, 0.25))


@pytest.mark.parametrize("P", [1, 2, 4, 8])
def test_heat_f64_pairs_per_lane(sw, oracle_mod, P):
    n, W, nsteps = 8192, 2048, 1500
    sw.set_tuning(W, P, sw.MODE_STAGE)
    u0 = workloads.white_noise(n, seed=P)
    got = run(sw, sw.advance, u0, nsteps, "heat", [0.3])
    assert same_bits(got, oracle_mod.heat(u0, nsteps, 0.3))


@pytest.mark.parametrize("n,nsteps", [(64, 50), (1000, 37), (4096, 300), (3, 10), (5, 4)])
def test_heat_f64_naive_bitwise(sw, oracle_mod, n, nsteps):
    u0 = workloads.white_noise(n, seed=n)
    got = run(sw, sw.naive_advance, u0, nsteps, "heat", HEAT_P)
    assert same_bits(got, oracle_mod.heat(u0, nsteps, 0.25))


def test_heat_small_workload_full(sw, oracle_mod):
    """The 4096-point, 10,000-step sine-mode workload in the default launch
    configuration, against the full oracle run."""
    w = workloads.WORKLOADS["heat_small"]
    u0 = workloads.initial("heat_small")
    want = oracle_mod.heat(u0, w["nsteps"], w["r"])
    assert same_bits(run(sw, sw.advance, u0, w["nsteps"], "heat", [w["r"]]), want)
    assert same_bits(run(sw, sw.naive_advance, u0, w["nsteps"], "heat", [w["r"]]), want)
    # the tiling the benchmark's autotuner picks: W = 64 on the lane-frame kernel
    sw.set_tuning(64, 0, sw.MODE_STAGE_LANE)
    assert same_bits(run(sw, sw.advance, u0, w["nsteps"], "heat", [w["r"]]), want)


# ---------------------------------------------------------------- heat f32

@pytest.mark.parametrize("n,W,P,nsteps", [(64, 16, 1, 9), (1024, 256, 2, 600),
                                          (8192, 4096, 4, 2500), (8192, 1024, 8, 999),
                                          (1024, 256, 2, 383)])
def test_heat_f32_swept_bitwise(sw, oracle_mod, n, W, P, nsteps):
    sw.set_tuning(W, P, sw.MODE_STAGE)
    u0 = workloads.white_noise(n, seed=W, dtype=np.float32)
    got = run(sw, sw.advance, u0, nsteps, "heat", [0.3])
    assert same_bits(got, oracle_mod.heat(u0, nsteps, 0.3))
    got = run(sw, sw.naive_advance, u0, nsteps, "heat", [0.3])
    assert same_bits(got, oracle_mod.heat(u0, nsteps, 0.3))


# ---------------------------------------------------------------------- KS

@pytest.mark.parametrize("n,W,P,nsteps", [
    (64, 16, 1, 1), (64, 16, 1, 2), (64, 16, 1, 5), (256, 64, 1, 40),
    (1024, 256, 2, 130), (2048, 1024, 2, 300), (2048, 512, 4, 257), (4096, 2048, 1, 100),
    (600, 200, 1, 77),
])
def test_ks_swept_bitwise(sw, oracle_mod, n, W, P, nsteps):
    sw.set_tuning(W, P, sw.MODE_STAGE)
    u0 = workloads.smoothed_noise(n, seed=n + W)
    got = run(sw, sw.advance, u0, nsteps, "ks", KS_P)
    assert same_bits(got, oracle_mod.ks(u0, nsteps, *KS_P))


@pytest.mark.parametrize("n,nsteps", [(64, 30), (1000, 25), (5, 3)])
def test_ks_naive_bitwise(sw, oracle_mod, n, nsteps):
    u0 = workloads.smoothed_noise(n, seed=n)
    want = oracle_mod.ks(u0, nsteps, *KS_P)
    assert same_bits(run(sw, sw.naive_advance, u0, nsteps, "ks", KS_P), want)
    assert same_bits(run(sw, sw.naive_substep_advance, u0, nsteps, "ks", KS_P), want)


# ------------------------------------------------------- edge cases, API

def test_zero_steps_is_noop(sw):
    u0 = workloads.white_noise(128, seed=1)
    assert same_bits(run(sw, sw.advance, u0, 0, "heat", HEAT_P), u0)
    assert same_bits(run(sw, sw.naive_advance, u0, 0, "heat", HEAT_P), u0)


def test_odd_grid_runs_on_its_cover(sw, oracle_mod):
    u0 = workloads.white_noise(1001, seed=3)
    assert sw.plan(1001, 50, "heat")["mode"] == sw.MODE_STAGE_RAGGED
    assert same_bits(run(sw, sw.advance, u0, 50, "heat", HEAT_P), oracle_mod.heat(u0, 50, 0.25))


def test_translation_equivariance(sw):
    n, nsteps = 4096, 1234
    u0 = workloads.white_noise(n, seed=5)
    base = run(sw, sw.advance, u0, nsteps, "heat", HEAT_P)
    for shift in (1, 77, 1000):
        got = run(sw, sw.advance, np.roll(u0, shift), nsteps, "heat", HEAT_P)
        assert same_bits(got, np.roll(base, shift))


def test_composition(sw):
    """advance(n1) then advance(n2) == advance(n1 + n2), bit for bit."""
    u0 = workloads.smoothed_noise(2048, seed=6)
    whole = run(sw, sw.advance, u0, 300, "ks", KS_P)
    part = run(sw, sw.advance, u0, 123, "ks", KS_P)
    part = run(sw, sw.advance, part, 177, "ks", KS_P)
    assert same_bits(part, whole)


def test_bad_arguments_raise(sw):
    import torch
    u = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(sw.SweptError):
        sw.advance(u, -1, "heat", HEAT_P)
    with pytest.raises(sw.SweptError):
        sw.advance(u, 1, "ks", [0.005, 0.0])
    with pytest.raises(sw.SweptError):
        sw.advance(u, 1, "heat", [float("nan")])
    with pytest.raises(TypeError):
        sw.advance(u.float(), 1, "ks", KS_P)
    sw.set_tuning(48, 0, sw.MODE_STAGE)
    with pytest.raises(sw.SweptError):
        sw.advance(u, 1, "heat", HEAT_P)


@pytest.mark.parametrize("stencil,n,W,P,nsteps", [
    ("heat", 8192, 2048, 4, 3000), ("heat", 4096, 512, 2, 1500), ("ks", 4096, 1024, 2, 400),
    ("ks", 2048, 512, 1, 300),
])
def test_banded_and_continuous_kernels_agree(sw, oracle_mod, stencil, n, W, P, nsteps):
    """Full diamonds run on the continuous-band kernel by default; the banded
    kernel must give the same bits (and both the oracle's)."""
    if stencil == "heat":
        u0, par = workloads.white_noise(n, seed=W + P), [0.3]
        want = oracle_mod.heat(u0, nsteps, 0.3)
    else:
        u0, par = workloads.smoothed_noise(n, seed=W + P), KS_P
        want = oracle_mod.ks(u0, nsteps, *KS_P)
    sw.set_tuning(W, P, sw.MODE_STAGE)
    assert same_bits(run(sw, sw.advance, u0, nsteps, stencil, par), want)
    sw.set_tuning(W, P, sw.MODE_STAGE_BANDED)
    assert same_bits(run(sw, sw.advance, u0, nsteps, stencil, par), want)


def test_ks_rejects_eight_pairs_per_lane(sw):
    import paper_1504_01380_amd as swmod
    sw.set_tuning(2048, 8, sw.MODE_STAGE)
    u = __import__("torch").zeros(4096, dtype=__import__("torch").float64, device="cuda")
    with pytest.raises(swmod.SweptError):
        sw.advance(u, 10, "ks", KS_P)
    sw.set_tuning(0, 0, sw.MODE_AUTO)
