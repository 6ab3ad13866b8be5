"""swept_advance inside a captured HIP graph: once the library's scratch
exists (a warm-up call of the same size), a call only enqueues kernels, so a
caller can capture it and replay it.  Every replay, with eager work and
synchronisations between the replays, must equal the eager result."""
import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.mark.parametrize("stencil,n,nsteps", [("heat", 1 << 16, 700), ("ks", 1 << 14, 150)])
def test_captured_advance_replays(stencil, n, nsteps):
    import torch
    import paper_1504_01380_amd as sw
    sw.init(0)
    sw.set_tuning(0, 0, sw.MODE_AUTO)
    par = [0.25] if stencil == "heat" else [workloads.KS_DT, workloads.KS_DX]
    u0 = workloads.white_noise(n, seed=5) if stencil == "heat" else \
        workloads.smoothed_noise(n, seed=5)
    ref = torch.from_numpy(u0).cuda()
    sw.advance(ref, nsteps, stencil, par)          # eager result; sizes the scratch
    torch.cuda.synchronize()
    want = ref.cpu().numpy()

    u = torch.from_numpy(u0).cuda()
    src = u.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            sw.advance(u, nsteps, stencil, par)
    torch.cuda.synchronize()
    for rep in range(3):
        u.copy_(src)                               # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = u.cpu().numpy()
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), rep
        junk = torch.randn(1 << 16, device="cuda").sum()   # unrelated eager work
        torch.cuda.synchronize()
        del junk
