"""No redundant computation, on the GPU (paper, Section 3: every variable is
computed once, by the node that owns its domain of dependence).  The counting
build libswept_count.so (SWEPT_COUNT_UPDATES) counts every point update of
the stage kernels; a swept run of nsteps steps on a ring of n points (the
two-fold cover of an odd field) must add exactly n x nsteps x sub-timesteps,
and give the bits of the normal library.  Covers equal tiles on the
continuous-band and banded schedules (heat f64/f32, the contraction-on heat,
KS, Euler), the unequal tiling (odd and awkward N) and batches on both
schedules."""
import ctypes
import os

import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available, same_bits

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_COUNT = os.path.join(ROOT, "paper_1504_01380_amd", "libswept_count.so")
KS_P = [workloads.KS_DT, workloads.KS_DX]


@pytest.fixture(scope="module")
def sw():
    import paper_1504_01380_amd as swept
    swept.init(0)
    yield swept
    swept.set_tuning(0, 0, swept.MODE_AUTO)


@pytest.fixture(scope="module")
def cl():
    """The counting build, through ctypes (argument marshalling only)."""
    if not os.path.exists(LIB_COUNT):
        pytest.fail("libswept_count.so is not built (python paper_1504_01380_amd/build.py)")
    L = ctypes.CDLL(LIB_COUNT)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.swept_init.argtypes = [ctypes.c_int]
    L.swept_set_stream.argtypes = [vp]
    L.swept_set_tuning.argtypes = [i32, i32, i32]
    L.swept_advance.argtypes = [vp, i64, i64, i32, dp, i32]
    L.swept_advance_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64), ctypes.POINTER(i32), dp, i64]
    L.swept_set_batch_schedule.argtypes = [i32, i64, i32, i32]
    L.swept_debug_update_count.argtypes = [ctypes.POINTER(ctypes.c_uint64), i32]
    L.swept_last_error.restype = ctypes.c_char_p
    L.swept_finalize.restype = None
    assert L.swept_init(0) == 0
    yield L
    L.swept_finalize()


def _ok(L, rc):
    assert rc == 0, L.swept_last_error().decode()


def _count(L):
    import torch
    torch.cuda.synchronize()
    c = ctypes.c_uint64()
    _ok(L, L.swept_debug_update_count(ctypes.byref(c), 1))
    return c.value


def _bind_stream(L):
    import torch
    _ok(L, L.swept_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


STENCILS = {"heat": (0, 1, [0.3]), "heat_f32": (1, 1, [0.3]), "ks": (2, 4, KS_P),
            "heat_fma": (4, 1, [0.25])}


def _field(stencil, n):
    if stencil == "heat_f32":
        return workloads.white_noise(n, seed=n, dtype=np.float32)
    if stencil == "ks":
        return workloads.smoothed_noise(n, seed=n)
    if stencil == "euler":
        return workloads.euler_smooth(n, seed=n)
    return workloads.white_noise(n, seed=n)


@pytest.mark.parametrize("stencil,n,nsteps,W,P,mode", [
    ("heat", 4096, 1000, 512, 2, 1), ("heat", 65536, 2500, 1024, 4, 1),
    ("heat", 4096, 777, 512, 2, 3), ("heat_f32", 8192, 700, 512, 2, 1),
    ("heat_fma", 8192, 600, 1024, 4, 1), ("ks", 8192, 300, 512, 2, 1),
    ("ks", 4096, 211, 256, 1, 3), ("euler", 2048, 60, 256, 1, 1),
    ("heat", 1001, 333, 0, 0, 0), ("ks", 8198, 250, 0, 0, 0), ("heat", 6126, 900, 0, 0, 5),
])
def test_each_point_level_once(sw, cl, stencil, n, nsteps, W, P, mode):
    """n x L updates (2n x L for an odd n, run on its cover), and the normal
    library's bits."""
    import torch
    if stencil == "euler":
        sid, S, par = 3, 4, [workloads.EULER_CFL / n, 1.0 / n, workloads.EULER_GAMMA]
    else:
        sid, S, par = STENCILS[stencil]
    u0 = _field(stencil, n)
    ring = n if n % 2 == 0 else 2 * n
    u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    _bind_stream(cl)
    _ok(cl, cl.swept_set_tuning(W, P, mode))
    _count(cl)
    arr = (ctypes.c_double * len(par))(*par)
    _ok(cl, cl.swept_advance(ctypes.c_void_p(u.data_ptr()), n, nsteps, sid, arr, len(par)))
    got = _count(cl)
    _ok(cl, cl.swept_set_tuning(0, 0, 0))
    print("%s n=%d steps=%d W=%d P=%d mode=%d: %d updates, %d expected"
          % (stencil, n, nsteps, W, P, mode, got, ring * nsteps * S), flush=True)
    assert got == ring * nsteps * S
    v = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    sw.set_tuning(W, P, mode)
    sw.advance(v, nsteps, {"heat_f32": "heat"}.get(stencil, stencil), par)
    sw.set_tuning(0, 0, 0)
    torch.cuda.synchronize()
    assert same_bits(u.cpu().numpy(), v.cpu().numpy())


@pytest.mark.parametrize("schedule", [0, 1])
def test_batch_each_point_level_once(cl, schedule):
    """A mixed batch (odd and even N, heat and KS, 128 instances): the sum of
    ring x L over its instances, on the persistent launch and per stage."""
    import torch
    insts = workloads.batch(count=128, seed=21, smin=50, smax=400)
    us = [torch.from_numpy(i.u0).cuda() for i in insts]
    _bind_stream(cl)
    _ok(cl, cl.swept_set_batch_schedule(schedule, 0, 0, 0))
    _count(cl)
    n = len(insts)
    ptrs = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
    nx = (ctypes.c_int64 * n)(*[i.n for i in insts])
    ns = (ctypes.c_int64 * n)(*[i.nsteps for i in insts])
    ids = (ctypes.c_int32 * n)(*[0 if i.stencil == "heat" else 2 for i in insts])
    par = []
    for i in insts:
        par += [0.25, 0.0] if i.stencil == "heat" else KS_P
    pa = (ctypes.c_double * len(par))(*par)
    _ok(cl, cl.swept_advance_batch(ptrs, nx, ns, ids, pa, n))
    got = _count(cl)
    want = sum((i.n if i.n % 2 == 0 else 2 * i.n) * i.nsteps * (1 if i.stencil == "heat" else 4)
               for i in insts)
    print("batch schedule %d: %d updates, %d expected" % (schedule, got, want), flush=True)
    _ok(cl, cl.swept_set_batch_schedule(0, 0, 0, 0))
    assert got == want
