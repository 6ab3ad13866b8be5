"""The contraction-on stencils (multiply-adds fused, the 3-FLOP form of the
heat sub-timestep in the paper's Section 4) on the GPU, through the C ABI.

Two bars:
 - bit-exact against the oracle's fused forms (heat_fma, ks_fma), whose every
   operation is pinned by a per-operation rational brute force;
 - within 1e-12 relative (max norm) of the canonical, unfused oracle -- for
   heat at any horizon, for KS up to 1,000 steps (a chaotic scheme amplifies
   the one-rounding differences exponentially beyond that).
The swept and naive schedules of a fused stencil give the same bits."""
import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available, same_bits

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

REL_TOL = 1e-12
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


def rel_err(a, b):
    return float(np.abs(a.astype(np.float64) - b.astype(np.float64)).max() /
                 np.abs(b.astype(np.float64)).max())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,W,P,nsteps,r,mode", [
    (64, 16, 1, 9, 0.3, "stage"), (512, 128, 1, 500, 0.3, "stage"),
    (2048, 512, 4, 1000, 0.3, "stage"), (4096, 1024, 4, 1535, 0.25, "stage"),
    (8192, 2048, 8, 1500, 0.1, "stage"), (1000, 200, 1, 401, 0.3, "banded"),
    (4096, 64, 0, 700, 0.3, "lane"), (4096, 0, 0, 3000, 0.3, "auto"),
])
def test_heat_fma_swept(sw, oracle_mod, dtype, n, W, P, nsteps, r, mode):
    modes = {"stage": sw.MODE_STAGE, "banded": sw.MODE_STAGE_BANDED,
             "lane": sw.MODE_STAGE_LANE, "auto": sw.MODE_AUTO}
    sw.set_tuning(W, P, modes[mode])
    u0 = workloads.white_noise(n, seed=n + W, dtype=dtype)
    got = run(sw, sw.advance, u0, nsteps, "heat_fma", [r])
    assert same_bits(got, oracle_mod.heat_fma(u0, nsteps, r))
    canon = oracle_mod.heat(u0, nsteps, r)
    assert rel_err(got, canon) <= (REL_TOL if dtype == np.float64 else 1e-5)
    if dtype == np.float64 and r != 0.25:
        # the fused and unfused forms really differ here (at r = 1/4 every
        # product r*lap is exact and the two forms agree bit for bit)
        assert not same_bits(got, canon)


@pytest.mark.parametrize("n,nsteps,r", [(4096, 300, 0.3), (1000, 77, 0.25), (5, 9, 0.3)])
def test_heat_fma_naive_equals_swept(sw, oracle_mod, n, nsteps, r):
    u0 = workloads.white_noise(n, seed=n)
    naive = run(sw, sw.naive_advance, u0, nsteps, "heat_fma", [r])
    assert same_bits(naive, oracle_mod.heat_fma(u0, nsteps, r))
    assert same_bits(naive, run(sw, sw.advance, u0, nsteps, "heat_fma", [r]))


@pytest.mark.parametrize("n,W,P,nsteps", [
    (256, 64, 1, 33), (1024, 256, 2, 250), (4096, 1024, 4, 300), (2048, 512, 2, 1000),
    (4096, 64, 0, 200),
])
def test_ks_fma_swept(sw, oracle_mod, n, W, P, nsteps):
    sw.set_tuning(W, P, sw.MODE_STAGE_LANE if P == 0 else sw.MODE_STAGE)
    u0 = workloads.smoothed_noise(n, seed=n + W)
    got = run(sw, sw.advance, u0, nsteps, "ks_fma", KS_P)
    assert same_bits(got, oracle_mod.ks_fma(u0, nsteps, *KS_P))
    canon = oracle_mod.ks(u0, nsteps, *KS_P)
    assert 0 < rel_err(got, canon) <= REL_TOL


@pytest.mark.parametrize("n,nsteps", [(1 << 14, 1000), (1 << 20, 1000)])
def test_ks_fma_within_tolerance_of_the_canonical_oracle(sw, oracle_mod, n, nsteps):
    """The KS workload's grid (2^20 points, default plan) over the 1,000-step
    horizon on which the 1e-12 bar applies."""
    u0 = workloads.smoothed_noise(n, seed=1002)
    print("ks_fma N=%d steps=%d plan=%s" % (n, nsteps, sw.plan(n, nsteps, "ks_fma")), flush=True)
    got = run(sw, sw.advance, u0, nsteps, "ks_fma", KS_P)
    canon = oracle_mod.ks(u0, nsteps, *KS_P)
    assert 0 < rel_err(got, canon) <= REL_TOL
    assert same_bits(got, run(sw, sw.naive_advance, u0, nsteps, "ks_fma", KS_P))
