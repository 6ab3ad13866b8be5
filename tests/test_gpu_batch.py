"""Batched swept runs: every instance of a batch equals its own oracle run
bit for bit (odd and even lengths, heat and KS, different step counts, tiles
of unequal width), also when the captured graph is launched again, on both
schedules (one persistent launch, and one launch per stage); a persistent
wait that gives up is reported, and the next batch is whole again."""
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
    swept.set_batch_schedule(swept.BATCH_PERSISTENT, 0)


@pytest.fixture(autouse=True)
def _default_schedule(sw):
    sw.set_batch_schedule(sw.BATCH_PERSISTENT, 0)
    yield
    sw.set_batch_schedule(sw.BATCH_PERSISTENT, 0)


def oracle_run(oracle_mod, stencil, u0, nsteps):
    if stencil == "heat":
        return oracle_mod.heat(u0, nsteps, 0.25)
    return oracle_mod.ks(u0, nsteps, *KS_P)


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("tile", [0, 64, 16])
def test_mixed_batch_bitwise(sw, oracle_mod, tile, schedule):
    import torch
    sw.set_tuning(tile, 0, sw.MODE_AUTO)
    sw.set_batch_schedule(schedule, 0)
    g = workloads.rng(2024 + tile)
    sizes = [256, 257, 300, 1001, 2048, 3, 4, 999, 4096, 777, 513, 64]
    insts = []
    for q, n in enumerate(sizes):
        stencil = "heat" if q % 2 == 0 else "ks"
        nsteps = int(g.integers(1, 120 if stencil == "ks" else 400))
        u0 = g.uniform(-1, 1, size=n)
        insts.append((stencil, nsteps, u0))
    insts.append(("ks", 0, g.uniform(-1, 1, size=100)))        # zero steps
    us = [torch.from_numpy(u0.copy()).cuda() for _, _, u0 in insts]
    sw.advance_batch(us, [ns for _, ns, _ in insts], [st for st, _, _ in insts],
                     [[0.25] if st == "heat" else KS_P for st, _, _ in insts])
    torch.cuda.synchronize()
    sw.sync()
    for (st, ns, u0), u in zip(insts, us):
        want = oracle_run(oracle_mod, st, u0, ns)
        print(st, u0.size, ns, flush=True)
        assert np.array_equal(u.cpu().numpy().view(np.uint8), want.view(np.uint8))
    # the same batch again: the cached graph is launched a second time
    for (_, _, u0), u in zip(insts, us):
        u.copy_(torch.from_numpy(u0))
    sw.advance_batch(us, [ns for _, ns, _ in insts], [st for st, _, _ in insts],
                     [[0.25] if st == "heat" else KS_P for st, _, _ in insts])
    torch.cuda.synchronize()
    for (st, ns, u0), u in zip(insts, us):
        want = oracle_run(oracle_mod, st, u0, ns)
        assert np.array_equal(u.cpu().numpy().view(np.uint8), want.view(np.uint8))
    sw.set_tuning(0, 0, sw.MODE_AUTO)


def test_batch_equals_solo_runs(sw):
    """A sample of the ensemble workload (log-uniform sizes, odd sizes
    included): each batched instance equals its own swept_advance."""
    import torch
    insts = workloads.batch(count=48, seed=7, smin=50, smax=300)
    us = [torch.from_numpy(i.u0).cuda() for i in insts]
    solo = []
    for i in insts:
        u = torch.from_numpy(i.u0).cuda()
        sw.advance(u, i.nsteps, i.stencil, [0.25] if i.stencil == "heat" else KS_P)
        solo.append(u)
    sw.advance_batch(us, [i.nsteps for i in insts], [i.stencil for i in insts],
                     [[0.25] if i.stencil == "heat" else KS_P for i in insts])
    torch.cuda.synchronize()
    for a, b in zip(us, solo):
        assert torch.equal(a.view(torch.int64), b.view(torch.int64))


def test_naive_batch_bitwise(sw, oracle_mod):
    """The naive batch baseline gives the oracle's bits too (odd step counts
    end in the spare buffer and are copied back; zero steps leave u alone)."""
    import torch
    g = workloads.rng(77)
    insts = []
    for q, n in enumerate([3, 4, 5, 255, 256, 257, 1000, 513, 2048, 99]):
        stencil = "heat" if q % 2 else "ks"
        insts.append((stencil, int(g.integers(0, 60)), g.uniform(-1, 1, size=n)))
    us = [torch.from_numpy(u0.copy()).cuda() for _, _, u0 in insts]
    sw.naive_advance_batch(us, [ns for _, ns, _ in insts], [st for st, _, _ in insts],
                           [[0.25] if st == "heat" else KS_P for st, _, _ in insts])
    torch.cuda.synchronize()
    for (st, ns, u0), u in zip(insts, us):
        want = oracle_run(oracle_mod, st, u0, ns)
        assert same_bits(u.cpu().numpy(), want), (st, u0.size, ns)


def test_full_ensemble(sw, oracle_mod):
    """The ensemble workload at full size (4096 instances, N log-uniform in
    [256, 65536], 1,000-20,000 steps): the swept batch equals the naive batch
    on every instance bit for bit, and the oracle on a sample of instances
    (the shortest-running ones of each stencil and parity, which the oracle
    finishes in seconds)."""
    import torch
    insts = workloads.batch()
    ns = [i.nsteps for i in insts]
    kinds = [i.stencil for i in insts]
    pars = [[0.25] if k == "heat" else KS_P for k in kinds]
    us = [torch.from_numpy(i.u0).cuda() for i in insts]
    vs = [u.clone() for u in us]
    print("swept batch", flush=True)
    sw.advance_batch(us, ns, kinds, pars)
    print("naive batch", flush=True)
    sw.naive_advance_batch(vs, ns, kinds, pars)
    torch.cuda.synchronize()
    for q, (a, b) in enumerate(zip(us, vs)):
        assert torch.equal(a.view(torch.int64), b.view(torch.int64)), q
    cost = sorted(range(len(insts)), key=lambda q: insts[q].n * insts[q].nsteps *
                  (4 if insts[q].stencil == "ks" else 1))
    picked = {}
    for q in cost:
        key = (insts[q].stencil, insts[q].n % 2)
        picked.setdefault(key, q)
    threads = oracle_mod.max_threads()
    for key, q in sorted(picked.items()):
        i = insts[q]
        want = (oracle_mod.heat(i.u0, i.nsteps, 0.25, threads=threads) if i.stencil == "heat"
                else oracle_mod.ks(i.u0, i.nsteps, *KS_P, threads=threads))
        print(key, i.n, i.nsteps, flush=True)
        assert same_bits(us[q].cpu().numpy(), want)


def _ensemble_sample(count, seed, smin, smax):
    insts = workloads.batch(count=count, seed=seed, smin=smin, smax=smax)
    return (insts, [i.nsteps for i in insts], [i.stencil for i in insts],
            [[0.25] if i.stencil == "heat" else KS_P for i in insts])


@pytest.mark.parametrize("chunk,queues", [(1, 0), (3, 0), (0, 0), (32, 0), (1, 1), (3, 7),
                                          (32, 64), (2, 1024)])
def test_persistent_equals_staged(sw, chunk, queues):
    """The two schedules run the same regions: the same bits on a sample of
    the ensemble (sizes log-uniform in [256, 65536], odd ones included), for
    claims of one task, of a few (runs that often cross a stage), the
    default and many; on one queue per XCD (the default), and on one queue,
    a few and more queues than instances with agent-scope hand-over."""
    import torch
    insts, ns, kinds, pars = _ensemble_sample(256, 11, 200, 2000)
    got = {}
    for sched in (sw.BATCH_STAGED, sw.BATCH_PERSISTENT):
        sw.set_batch_schedule(sched, 0, chunk, queues)
        us = [torch.from_numpy(i.u0).cuda() for i in insts]
        print("schedule", sched, flush=True)
        sw.advance_batch(us, ns, kinds, pars)
        torch.cuda.synchronize()
        sw.sync()
        got[sched] = us
    for q, (a, b) in enumerate(zip(got[0], got[1])):
        assert torch.equal(a.view(torch.int64), b.view(torch.int64)), q


@pytest.mark.parametrize("count,queues", [(64, 0), (1, 1)])
def test_persistent_wait_that_gives_up_is_reported(sw, oracle_mod, count, queues):
    """A spin limit of one microsecond, set from the host: the regions of
    later stages give up waiting, every workgroup leaves, and swept_sync
    reports SWEPT_ETIMEOUT once; with the default limit the same batch is
    whole.  On one queue per XCD (64 instances, which spread evenly) and on
    one agent-scope queue (one instance)."""
    import torch
    g = workloads.rng(5)
    u0s = [g.uniform(-1, 1, size=8192 + 2 * q) for q in range(count)]
    us = [torch.from_numpy(u0.copy()).cuda() for u0 in u0s]
    args = ([3000] * count, ["heat"] * count, [[0.25]] * count)
    sw.set_batch_schedule(sw.BATCH_PERSISTENT, 1, 0, queues)
    sw.advance_batch(us, *args)
    torch.cuda.synchronize()
    with pytest.raises(sw.SweptError) as err:
        sw.sync()
    assert err.value.code == -6 and "gave up" in str(err.value)
    sw.sync()                                  # reported once
    sw.set_batch_schedule(sw.BATCH_PERSISTENT, 0, 0, queues)
    for u, u0 in zip(us, u0s):
        u.copy_(torch.from_numpy(u0))
    sw.advance_batch(us, *args)
    torch.cuda.synchronize()
    sw.sync()
    for q in (0, count - 1):
        assert same_bits(us[q].cpu().numpy(), oracle_mod.heat(u0s[q], 3000, 0.25))


def test_few_large_instances(sw):
    """A batch of a few large instances (which one queue per XCD cannot spread
    evenly, so it runs one launch per stage) equals the instances' own
    swept_advance runs."""
    import torch
    g = workloads.rng(8)
    insts = [("heat", 1 << 20, 700), ("ks", 1 << 18, 150), ("heat", 3 * 65536 + 2, 301)]
    us, solo = [], []
    for st, n, ns in insts:
        u0 = g.uniform(-1, 1, size=n) if st == "heat" else workloads.smoothed_noise(n, seed=n)
        us.append(torch.from_numpy(u0).cuda())
        v = torch.from_numpy(u0).cuda()
        sw.advance(v, ns, st, [0.25] if st == "heat" else KS_P)
        solo.append(v)
    sw.advance_batch(us, [ns for _, _, ns in insts], [st for st, _, _ in insts],
                     [[0.25] if st == "heat" else KS_P for st, _, _ in insts])
    torch.cuda.synchronize()
    sw.sync()
    for q, (a, b) in enumerate(zip(us, solo)):
        assert torch.equal(a.view(torch.int64), b.view(torch.int64)), q
