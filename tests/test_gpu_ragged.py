"""One tiling rule for every grid: swept_advance on grids without a good even
tile width (odd nx, run on the two-fold cover; even nx whose even divisors are
far below the target, such as 8198 = 2 x 4099) takes the unequal tiling --
T-1 tiles of 2k points and one remainder -- and must give the oracle's bits,
for every stencil (paper, Section 3: the swept rule only reorders the
per-point updates)."""
import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available, same_bits

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

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


def case(oracle_mod, stencil, n, nsteps):
    """(u0, stencil name, params, the oracle's result)."""
    if stencil in ("heat", "heat_fma"):
        u0 = workloads.white_noise(n, seed=n)
        f = oracle_mod.heat if stencil == "heat" else oracle_mod.heat_fma
        return u0, [0.3], f(u0, nsteps, 0.3)
    if stencil == "heat_f32":
        u0 = workloads.white_noise(n, seed=n, dtype=np.float32)
        return u0, [0.3], oracle_mod.heat(u0, nsteps, 0.3)
    if stencil in ("ks", "ks_fma"):
        u0 = workloads.smoothed_noise(n, seed=n)
        f = oracle_mod.ks if stencil == "ks" else oracle_mod.ks_fma
        return u0, KS_P, f(u0, nsteps, *KS_P)
    q0 = workloads.euler_smooth(n, seed=n)
    par = [workloads.EULER_CFL / n, 1.0 / n, workloads.EULER_GAMMA]
    return q0, par, oracle_mod.euler(q0, nsteps, *par)


@pytest.mark.parametrize("stencil,n,nsteps", [
    ("heat", 1001, 333), ("heat", 8198, 1000), ("heat", 8186, 777), ("heat", 6126, 1500),
    ("heat", 65537, 1200), ("heat", 129, 41), ("heat", 131, 500), ("heat", 2 * 65537, 1025),
    ("heat_f32", 1001, 400), ("heat_f32", 8198, 900), ("heat_fma", 4099, 700),
    ("ks", 1001, 120), ("ks", 8198, 250), ("ks", 4099, 301), ("ks", 65537, 100),
    ("ks_fma", 8198, 150), ("euler", 1001, 60), ("euler", 8198, 41), ("euler", 4097, 33),
])
def test_unequal_tiling_bitwise(sw, oracle_mod, stencil, n, nsteps):
    import torch
    name = "heat" if stencil == "heat_f32" else stencil
    u0, par, want = case(oracle_mod, stencil, n, nsteps)
    p = sw.plan(n, nsteps, name, torch.float32 if u0.dtype == np.float32 else torch.float64)
    print("%s n=%d steps=%d plan=%s" % (stencil, n, nsteps, p), flush=True)
    assert p["mode"] == sw.MODE_STAGE_RAGGED
    got = run(sw, sw.advance, u0, nsteps, name, par)
    assert same_bits(got, want)


@pytest.mark.parametrize("stencil,n,W,P,nsteps", [
    ("heat", 4096, 600, 1, 500), ("heat", 4096, 1024, 4, 2000), ("heat", 3000, 256, 2, 1111),
    ("ks", 2048, 256, 2, 300), ("ks", 4097, 128, 1, 150), ("euler", 1000, 64, 1, 50),
    ("heat", 5, 2, 1, 9), ("heat", 7, 0, 0, 30),
])
def test_forced_unequal_tiling(sw, oracle_mod, stencil, n, W, P, nsteps):
    u0, par, want = case(oracle_mod, stencil, n, nsteps)
    sw.set_tuning(W, P, sw.MODE_STAGE_RAGGED)
    p = sw.plan(n, nsteps, stencil)
    print("%s n=%d W=%d P=%d steps=%d plan=%s" % (stencil, n, W, P, nsteps, p), flush=True)
    got = run(sw, sw.advance, u0, nsteps, stencil, par)
    assert same_bits(got, want)


def test_large_awkward_grid(sw, oracle_mod):
    """2^24 + 2 points (= 2 x 3 x 2796203): 16,385 tiles, the last of 2
    points; whole field against the naive schedule, sampled points against
    the oracle's cones."""
    n, nsteps = (1 << 24) + 2, 3000
    u0 = workloads.white_noise(n, seed=77)
    p = sw.plan(n, nsteps, "heat")
    print("heat n=%d steps=%d plan=%s" % (n, nsteps, p), flush=True)
    assert p["mode"] == sw.MODE_STAGE_RAGGED and p["depth_k"] >= 256
    got = run(sw, sw.advance, u0, nsteps, "heat", [0.25])
    assert same_bits(got, run(sw, sw.naive_advance, u0, nsteps, "heat", [0.25]))
    idx = np.array([0, 1, 1023, 1024, n // 2, n - 3, n - 2, n - 1], dtype=np.int64)
    assert same_bits(got[idx], oracle_mod.heat_points(u0, nsteps, 0.25, idx))


def test_noalloc_on_an_odd_grid(sw):
    """The allocation-free entry point takes the same unequal tiling."""
    u0 = workloads.white_noise(100001, seed=3)
    a = run(sw, sw.advance_noalloc, u0, 500, "heat", [0.25])
    assert same_bits(a, run(sw, sw.advance, u0, 500, "heat", [0.25]))
