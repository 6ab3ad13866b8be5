"""swept_advance_noalloc, the entry point that allocates nothing (its scratch
is a fixed array the library holds per GPU), called through the C ABI:
bit for bit the result of swept_advance on the same input, for two calls in
a row (the second smaller, so the array holds the first call's leftovers),
and a clear error for a request beyond the array."""
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
    swept.set_tuning(0, 0, swept.MODE_AUTO)
    yield swept
    swept.set_tuning(0, 0, swept.MODE_AUTO)


def run(sw, fn, u0, nsteps, stencil, params):
    import torch
    u = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda")
    fn(u, nsteps, stencil, params)
    torch.cuda.synchronize()
    sw.sync()
    return u.cpu().numpy()


# (first call, second smaller call): stencil, n, nsteps, params
PAIRS = [
    (("heat", 1 << 20, 500, [0.25]), ("heat", 4096, 300, [0.25])),
    (("ks", 1 << 16, 120, KS_P), ("ks", 2048, 77, KS_P)),
    (("heat", 5_592_404, 40, [0.3]), ("heat", 1001, 55, [0.3])),   # near the limit; odd n (naive)
    (("heat_f32", 1 << 18, 333, [0.25]), ("heat_f32", 640, 129, [0.25])),
    (("euler", 1 << 14, 50, None), ("euler", 600, 21, None)),
]


def make(case):
    st, n, nsteps, par = case
    if st == "heat_f32":
        return "heat", workloads.white_noise(n, seed=n, dtype=np.float32), nsteps, par
    if st == "heat":
        return st, workloads.white_noise(n, seed=n), nsteps, par
    if st == "ks":
        return st, workloads.smoothed_noise(n, seed=n), nsteps, par
    return st, workloads.euler_smooth(n, seed=n), nsteps, \
        [workloads.EULER_CFL / n, 1.0 / n, workloads.EULER_GAMMA]


@pytest.mark.parametrize("first,second", PAIRS)
def test_noalloc_equals_swept_advance(sw, first, second):
    for case in (first, second):
        st, u0, nsteps, par = make(case)
        print("noalloc %s n=%d steps=%d" % (st, u0.shape[0], nsteps), flush=True)
        got = run(sw, sw.advance_noalloc, u0, nsteps, st, par)
        want = run(sw, sw.advance, u0, nsteps, st, par)
        assert same_bits(got, want), case


def test_noalloc_matches_the_oracle(sw, oracle_mod):
    u0 = workloads.white_noise(8192, seed=5)
    got = run(sw, sw.advance_noalloc, u0, 700, "heat", [0.25])
    assert same_bits(got, oracle_mod.heat(u0, 700, 0.25))


def test_noalloc_rejects_sizes_beyond_the_array(sw):
    import torch
    n = 5_592_406            # 3 * n * 8 bytes > SWEPT_NOALLOC_SCRATCH_BYTES (even n: swept path)
    assert 3 * n * 8 > sw.NOALLOC_SCRATCH_BYTES
    u0 = workloads.white_noise(n, seed=1)
    u = torch.from_numpy(u0).cuda()
    with pytest.raises(sw.SweptError) as err:
        sw.advance_noalloc(u, 10, "heat", [0.25])
    assert err.value.code == -1 and "SWEPT_NOALLOC_SCRATCH_BYTES" in str(err.value)
    torch.cuda.synchronize()
    assert same_bits(u.cpu().numpy(), u0)      # nothing was enqueued
