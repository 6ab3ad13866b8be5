"""GPU swept adjoint, through the C ABI, against the CPU oracle's discrete
adjoint (bit for bit: both evaluate the same transposed sub-timestep
Jacobians in the same order) and against central finite differences of the
forward map."""
import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available

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


def gpu_adjoint(sw, u0, nsteps, stencil, params, first, wgt, cot=None, tile=0):
    import torch
    sw.set_tuning(tile, 0, sw.MODE_AUTO)
    u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    c = None if cot is None else torch.from_numpy(np.ascontiguousarray(cot)).cuda()
    g = sw.adjoint(u, nsteps, stencil, params, window_first=first, window_weight=wgt,
                   cot_final=c)
    torch.cuda.synchronize()
    sw.sync()
    sw.set_tuning(0, 0, sw.MODE_AUTO)
    return g.cpu().numpy()


@pytest.mark.parametrize("n,nsteps,first,tile,with_cot", [
    (64, 1, 0, 0, True), (64, 37, 20, 0, True), (128, 100, 1, 0, False), (96, 50, 51, 32, True),
    (1024, 333, 300, 0, True), (64, 0, 0, 0, True), (4096, 1000, 900, 64, False),
    (64, 37, 20, 64, True), (640, 45, 44, 64, False),
])
def test_heat_adjoint_bitwise(sw, oracle_mod, n, nsteps, first, tile, with_cot):
    u0 = workloads.white_noise(n, seed=n + nsteps)
    cot = workloads.white_noise(n, seed=5) if with_cot else None
    w = 1.0 / (n * 10)
    got = gpu_adjoint(sw, u0, nsteps, "heat", [0.3], first, w, cot, tile)
    want = oracle_mod.heat_adjoint(u0, nsteps, 0.3, first, w, cot)
    assert np.array_equal(got.view(np.uint8), want.view(np.uint8))


@pytest.mark.parametrize("n,nsteps,first,tile,with_cot", [
    (64, 1, 0, 0, True), (64, 9, 5, 0, True), (128, 40, 1, 0, False), (96, 25, 20, 8, True),
    (1024, 120, 100, 0, True), (4096, 300, 250, 16, False), (256, 50, 51, 4, True),
    (4096, 300, 250, 64, True), (128, 77, 30, 64, False), (64, 21, 1, 64, True),
    (192, 33, 7, 64, True),
])
def test_ks_adjoint_bitwise(sw, oracle_mod, n, nsteps, first, tile, with_cot):
    u0 = workloads.smoothed_noise(n, seed=n + nsteps) * 5
    cot = workloads.white_noise(n, seed=6) if with_cot else None
    w = 1.0 / (n * 10)
    got = gpu_adjoint(sw, u0, nsteps, "ks", KS_P, first, w, cot, tile)
    want = oracle_mod.ks_adjoint(u0, nsteps, *KS_P, first, w, cot)
    assert np.array_equal(got.view(np.uint8), want.view(np.uint8))


def test_autograd_function(sw, oracle_mod):
    import torch
    n, nsteps = 512, 80
    u0 = torch.from_numpy(workloads.smoothed_noise(n, seed=3)).cuda().requires_grad_(True)
    u = sw.SweptAdvance.apply(u0, nsteps, "ks", KS_P)
    weights = torch.from_numpy(workloads.white_noise(n, seed=4)).cuda()
    (u * weights).sum().backward()
    want = oracle_mod.ks_adjoint(u0.detach().cpu().numpy(), nsteps, *KS_P, nsteps + 1, 0.0,
                                 weights.cpu().numpy())
    assert np.array_equal(u0.grad.cpu().numpy().view(np.uint8), want.view(np.uint8))


def test_window_objective_fd(sw):
    """J = mean u^2 over the final steps; <dJ/du0, v> against central finite
    differences along random unit directions (short horizon, eps = 1e-6)."""
    import torch
    n, nsteps, window = 2048, 400, 40
    u0 = torch.from_numpy(workloads.smoothed_noise(n, seed=9)).cuda().requires_grad_(True)
    J = sw.WindowMeanSquare.apply(u0, nsteps, "ks", KS_P, window)
    J.backward()
    g = u0.grad.double()
    rng = workloads.rng(77)
    eps = 1e-6
    for _ in range(4):
        v = torch.from_numpy(rng.standard_normal(n)).cuda()
        v /= torch.linalg.norm(v)
        jp = sw.window_mean_square_value(u0.detach() + eps * v, nsteps, "ks", KS_P, window)
        jm = sw.window_mean_square_value(u0.detach() - eps * v, nsteps, "ks", KS_P, window)
        fd = float((jp - jm) / (2 * eps))
        ad = float(torch.dot(g, v))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-12


@pytest.mark.parametrize("stencil,n,nsteps,first,with_cot", [
    ("heat", 64, 37, 20, True), ("heat", 1001, 50, 0, False), ("heat", 5, 9, 3, True),
    ("heat", 128, 0, 0, True), ("ks", 64, 9, 5, True), ("ks", 1000, 40, 1, False),
    ("ks", 7, 6, 2, True), ("ks", 4096, 120, 100, True), ("ks", 300, 25, 26, True),
])
def test_naive_adjoint_bitwise(sw, oracle_mod, stencil, n, nsteps, first, with_cot):
    """The straight-decomposition adjoint (the baseline) gives the oracle's
    bits too, on any grid (it needs no tiling: odd and tiny n included)."""
    import torch
    if stencil == "heat":
        u0, par = workloads.white_noise(n, seed=n + 1), [0.3]
        want = lambda c: oracle_mod.heat_adjoint(u0, nsteps, 0.3, first, w, c)
    else:
        u0, par = workloads.smoothed_noise(n, seed=n + 1) * 5, KS_P
        want = lambda c: oracle_mod.ks_adjoint(u0, nsteps, *KS_P, first, w, c)
    w = 1.0 / (n * 10)
    cot = workloads.white_noise(n, seed=9) if with_cot else None
    u = torch.from_numpy(u0).cuda()
    c = None if cot is None else torch.from_numpy(cot).cuda()
    g = sw.naive_adjoint(u, nsteps, stencil, par, window_first=first, window_weight=w,
                         cot_final=c)
    torch.cuda.synchronize()
    assert np.array_equal(g.cpu().numpy().view(np.uint8), want(cot).view(np.uint8))
