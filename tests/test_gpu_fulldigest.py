"""Whole-field parity at the full benchmark sizes: every point of the GPU's
result against the oracle's full run, through the SHA-256 digests that
tests/golden/make_full_digests.py wrote from the oracle alone.  Covered: the
heat workload (2^24 points, 20,000 steps) in binary64 and binary32 and the KS
workload (2^20 points, 50,000 steps), each on the swept schedule in the
automatic plan and in the tiling the benchmark's autotuner picks, and on the
naive schedule (including the fused KS step with 1024-point blocks that grids
of 2^19 points and more use).

The contraction-on heat stencil is held to the same digest: at r = 1/4 every
product r * lap is exact, so fusing the multiply-adds changes no bit."""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_digests.json")


def golden(name):
    with open(GOLDEN) as fh:
        return json.load(fh)[name]


@pytest.fixture(scope="module")
def sw():
    import paper_1504_01380_amd as swept
    swept.init(0)
    swept.set_tuning(0, 0, swept.MODE_AUTO)
    yield swept
    swept.set_tuning(0, 0, swept.MODE_AUTO)


def digest_of_run(sw, fn, u0, nsteps, stencil, params, tuning=(0, 0, 0)):
    import torch
    sw.set_tuning(*tuning)
    try:
        u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
        fn(u, nsteps, stencil, params)
        torch.cuda.synchronize()
        sw.sync()
    finally:
        sw.set_tuning(0, 0, sw.MODE_AUTO)
    return hashlib.sha256(u.cpu().numpy().tobytes()).hexdigest()


HEAT_RUNS = [("swept", "auto", (0, 0, 0)), ("swept", "W1024P4", (1024, 4, 1)),
             ("swept", "W512P2", (512, 2, 1)), ("naive", "naive", (0, 0, 0))]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("schedule,label,tuning", HEAT_RUNS)
def test_heat_large_whole_field(sw, dtype, schedule, label, tuning):
    w = workloads.WORKLOADS["heat_large"]
    ref = golden("heat_large_f64" if dtype == np.float64 else "heat_large_f32")
    u0 = workloads.initial("heat_large", dtype=dtype)
    print("heat_large %s %s %s" % (np.dtype(dtype).name, schedule, label), flush=True)
    fn = sw.advance if schedule == "swept" else sw.naive_advance
    assert digest_of_run(sw, fn, u0, w["nsteps"], "heat", [w["r"]], tuning) == ref["sha256"]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_heat_large_fma_whole_field(sw, dtype):
    w = workloads.WORKLOADS["heat_large"]
    ref = golden("heat_large_f64" if dtype == np.float64 else "heat_large_f32")
    u0 = workloads.initial("heat_large", dtype=dtype)
    assert digest_of_run(sw, sw.advance, u0, w["nsteps"], "heat_fma", [w["r"]]) == ref["sha256"]


@pytest.mark.parametrize("schedule,label,tuning", [
    ("swept", "auto", (0, 0, 0)), ("swept", "W512P2", (512, 2, 1)),
    ("swept", "W1024P4", (1024, 4, 1)), ("naive", "naive", (0, 0, 0))])
def test_ks_whole_field(sw, schedule, label, tuning):
    w = workloads.WORKLOADS["ks"]
    ref = golden("ks")
    u0 = workloads.initial("ks")
    print("ks %s %s" % (schedule, label), flush=True)
    fn = sw.advance if schedule == "swept" else sw.naive_advance
    assert digest_of_run(sw, fn, u0, w["nsteps"], "ks", [w["dt"], w["dx"]], tuning) == \
        ref["sha256"]
