"""The fused-Laplacian evaluation of heat (binary64 and binary32) in
swept_advance and swept_advance_batch.

(u[i-1] + u[i+1]) - 2u equals fma(-2, u, u[i-1] + u[i+1]) bit for bit while
2u is finite; the library takes the fused form only after its range check
(0 <= r <= 1/2, every finite |u0| <= MAX/16 for the type's largest finite
value MAX), which keeps every point far from MAX/2 (paper, Section 4: the
heat sub-timestep).  Both forms must
give the oracle's bits; the checks here also make sure the fused form is the
one taken where it is allowed, that data or parameters outside the allowed
range take the five operations as written, and that one call's failed check
does not stick to later calls.  A batch takes one decision for all its heat
instances and checks its fields again at every launch of its captured
graph."""
import numpy as np
import pytest

import workloads
from tests.conftest import gpu_available, same_bits

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

DMAX = np.finfo(np.float64).max
FMAX = np.finfo(np.float32).max


@pytest.fixture(scope="module")
def sw():
    import paper_1504_01380_amd as swept
    swept.init(0)
    yield swept
    swept.set_tuning(0, 0, swept.MODE_AUTO)
    swept.set_heat_form(swept.FORM_AUTO)


@pytest.fixture(autouse=True)
def _reset(sw):
    sw.set_tuning(0, 0, sw.MODE_AUTO)
    sw.set_heat_form(sw.FORM_AUTO)
    yield
    sw.set_tuning(0, 0, sw.MODE_AUTO)
    sw.set_heat_form(sw.FORM_AUTO)


def run(sw, u0, nsteps, r, fn=None):
    import torch
    u = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda")
    (fn or sw.advance)(u, nsteps, "heat", [r])
    torch.cuda.synchronize()
    sw.sync()
    return u.cpu().numpy()


def same_bits_up_to_nan(a, b):
    """Byte equality except that any two NaNs match (the payload a NaN
    carries is not part of the scheme)."""
    na, nb = np.isnan(a), np.isnan(b)
    return np.array_equal(na, nb) and same_bits(a[~na], b[~nb])


# (label, nx, nsteps, tuning): the continuous and banded kernels (equal
# tiles), the lane-frame kernel (few tiles) and the unequal tiling (odd nx on
# its two-fold cover, and an even nx with no good even divisor)
PLANS = [("cont_W1024_P4", 1 << 16, 1500, (1024, 4, 1)),
         ("cont_W512_P2", 3 << 12, 777, (512, 2, 1)),
         ("banded", 1 << 14, 600, (256, 1, 3)),
         ("lane", 4096, 1000, (64, 0, 4)),
         ("ragged_odd", 1001, 700, (0, 0, 0)),
         ("ragged_8198", 8198, 513, (0, 0, 0)),
         ("auto", 5000, 300, (0, 0, 0))]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("label,nx,nsteps,tuning", PLANS)
def test_fused_form_is_taken_and_exact(sw, oracle_mod, label, nx, nsteps, tuning, dtype):
    u0 = workloads.white_noise(nx, seed=nx + 3, dtype=dtype)
    want = oracle_mod.heat(u0, nsteps, 0.25)
    sw.set_tuning(*tuning)
    got = run(sw, u0, nsteps, 0.25)
    assert sw.last_heat_form() == sw.FORM_FUSED
    assert same_bits(got, want)
    sw.set_heat_form(sw.FORM_CANONICAL)
    got = run(sw, u0, nsteps, 0.25)
    assert sw.last_heat_form() == sw.FORM_CANONICAL
    assert same_bits(got, want)


@pytest.mark.parametrize("dtype,r", [(dt, r) for dt in (np.float64, np.float32)
                                     for r in (0.0, 0.1, 0.3, 0.5)] +
                         [(np.float32, 0.5000000000000001)])
def test_fused_form_over_the_allowed_r(sw, oracle_mod, r, dtype):
    """0 <= r <= 1/2 as the field's type rounds it (the double just above
    1/2 rounds to 1/2 in binary32)."""
    u0 = workloads.white_noise(1 << 14, seed=77, dtype=dtype)
    sw.set_tuning(256, 2, 1)
    got = run(sw, u0, 900, r)
    assert sw.last_heat_form() == sw.FORM_FUSED
    assert same_bits(got, oracle_mod.heat(u0, 900, r))


@pytest.mark.parametrize("dtype,r", [(np.float64, -0.05), (np.float64, 0.5000000000000001),
                                     (np.float64, 0.6), (np.float64, 1.0),
                                     (np.float32, -0.05), (np.float32, 0.50000006),
                                     (np.float32, 0.6)])
def test_r_outside_the_range_takes_the_canonical_form(sw, oracle_mod, dtype, r):
    u0 = workloads.white_noise(1 << 14, seed=78, dtype=dtype)
    sw.set_tuning(256, 2, 1)
    got = run(sw, u0, 120, r)
    assert sw.last_heat_form() == sw.FORM_CANONICAL
    assert same_bits_up_to_nan(got, oracle_mod.heat(u0, 120, r))


@pytest.mark.parametrize("dtype,big", [(np.float64, DMAX), (np.float32, FMAX)])
def test_values_near_the_overflow_take_the_canonical_form(sw, oracle_mod, dtype, big):
    """Values of 0.4..0.6 MAX: 2u overflows for half of them, so the
    oracle's run fills with infinities and NaNs, which the fused form would
    not produce.  The range check must send the call to the canonical form."""
    rng = np.random.default_rng(5)
    u0 = (big * (0.5 + 0.1 * rng.uniform(-1.0, 1.0, 1 << 14))).astype(dtype)
    want = oracle_mod.heat(u0, 40, 0.25)
    assert not np.all(np.isfinite(want))        # the case separates the two forms
    sw.set_tuning(256, 2, 1)
    got = run(sw, u0, 40, 0.25)
    assert sw.last_heat_form() == sw.FORM_CANONICAL
    assert same_bits_up_to_nan(got, want)


@pytest.mark.parametrize("dtype,big", [(np.float64, DMAX), (np.float32, FMAX)])
def test_the_bound_is_a_sixteenth_of_the_largest_value(sw, oracle_mod, dtype, big):
    u0 = workloads.white_noise(1 << 14, seed=79, dtype=dtype)
    sw.set_tuning(256, 2, 1)
    lim = dtype(big / 16)
    for scale, form in ((lim, sw.FORM_FUSED),
                        (np.nextafter(lim, dtype(np.inf)), sw.FORM_CANONICAL)):
        v = u0.copy()
        v[123] = scale
        got = run(sw, v, 200, 0.25)
        assert sw.last_heat_form() == form
        assert same_bits(got, oracle_mod.heat(v, 200, 0.25))


def test_non_finite_values_pass_the_check(sw, oracle_mod):
    """Infinities in the field allow the fused form: a non-finite input only
    makes non-finite outputs, the same in both forms."""
    u0 = workloads.white_noise(1 << 14, seed=80)
    u0[[10, 5000]] = [np.inf, -np.inf]
    sw.set_tuning(256, 2, 1)
    got = run(sw, u0, 300, 0.25)
    assert sw.last_heat_form() == sw.FORM_FUSED
    want = oracle_mod.heat(u0, 300, 0.25)
    assert same_bits_up_to_nan(got, want)
    assert np.isnan(want).any() and np.isfinite(want).any()


def test_a_failed_check_does_not_stick(sw, oracle_mod):
    good = workloads.white_noise(1 << 14, seed=81)
    bad = good.copy()
    bad[7] = DMAX / 4
    sw.set_tuning(256, 2, 1)
    for u0, form in ((good, sw.FORM_FUSED), (bad, sw.FORM_CANONICAL),
                     (good, sw.FORM_FUSED), (bad, sw.FORM_CANONICAL)):
        got = run(sw, u0, 250, 0.25)
        assert sw.last_heat_form() == form
        assert same_bits_up_to_nan(got, oracle_mod.heat(u0, 250, 0.25))


def test_naive_and_noalloc_report_their_forms(sw, oracle_mod):
    u0 = workloads.white_noise(1 << 14, seed=82)
    want = oracle_mod.heat(u0, 300, 0.25)
    got = run(sw, u0, 300, 0.25, fn=sw.advance_noalloc)
    assert sw.last_heat_form() == sw.FORM_FUSED
    assert same_bits(got, want)
    sw.set_tuning(0, 0, sw.MODE_NAIVE)
    got = run(sw, u0, 300, 0.25)
    assert sw.last_heat_form() == sw.FORM_CANONICAL
    assert same_bits(got, want)


# ------------------------------------------------------------------ batches
KS_P = [workloads.KS_DT, workloads.KS_DX]
BATCH_SIZES = [256, 257, 1001, 2048, 4096, 777, 6000, 100]


def mixed_batch(seed, r=0.25):
    """(stencil, nsteps, u0, params): heat and KS alternately, odd and even
    lengths (the odd heat ring runs on its two-fold cover)."""
    g = workloads.rng(seed)
    insts = []
    for q, n in enumerate(BATCH_SIZES):
        st = "heat" if q % 2 == 0 else "ks"
        ns = int(g.integers(1, 400 if st == "heat" else 100))
        insts.append((st, ns, g.uniform(-1, 1, n), [r] if st == "heat" else KS_P))
    return insts


def batch_oracle(oracle_mod, insts):
    return [oracle_mod.heat(u0, ns, p[0]) if st == "heat" else oracle_mod.ks(u0, ns, *p)
            for st, ns, u0, p in insts]


def run_batch(sw, insts, us=None):
    """Advance the batch; with `us`, refill those tensors (same pointers, so
    the captured graph is launched again)."""
    import torch
    if us is None:
        us = [torch.from_numpy(u0.copy()).cuda() for _, _, u0, _ in insts]
    else:
        for (_, _, u0, _), u in zip(insts, us):
            u.copy_(torch.from_numpy(u0))
    sw.advance_batch(us, [ns for _, ns, _, _ in insts], [st for st, _, _, _ in insts],
                     [p for _, _, _, p in insts])
    torch.cuda.synchronize()
    sw.sync()
    return us


def assert_batch(us, want):
    for u, w in zip(us, want):
        assert same_bits_up_to_nan(u.cpu().numpy(), w)


@pytest.fixture
def batch_schedule(sw):
    yield
    sw.set_batch_schedule(sw.BATCH_PERSISTENT, 0)


@pytest.mark.parametrize("schedule", ["persistent", "staged"])
def test_batch_takes_the_fused_form(sw, oracle_mod, batch_schedule, schedule):
    sw.set_batch_schedule(sw.BATCH_PERSISTENT if schedule == "persistent" else sw.BATCH_STAGED, 0)
    insts = mixed_batch(31)
    want = batch_oracle(oracle_mod, insts)
    assert_batch(run_batch(sw, insts), want)
    assert sw.last_heat_form() == sw.FORM_FUSED
    sw.set_heat_form(sw.FORM_CANONICAL)
    assert_batch(run_batch(sw, insts), want)
    assert sw.last_heat_form() == sw.FORM_CANONICAL


@pytest.mark.parametrize("schedule", ["persistent", "staged"])
def test_batch_checks_its_fields_at_every_launch(sw, oracle_mod, batch_schedule, schedule):
    """The same batch (same pointers: the captured graph runs again) with a
    heat field of values near MAX/2 in the second launch, whose oracle run
    overflows where the fused form would not: that launch must take the five
    operations, and the next good launch the fused form again."""
    sw.set_batch_schedule(sw.BATCH_PERSISTENT if schedule == "persistent" else sw.BATCH_STAGED, 0)
    good = mixed_batch(32)
    bad = list(good)
    rng = np.random.default_rng(6)
    st, ns, u0, p = bad[2]
    bad[2] = (st, ns, DMAX * (0.5 + 0.1 * rng.uniform(-1.0, 1.0, u0.size)), p)
    want_bad = batch_oracle(oracle_mod, bad)
    assert not np.all(np.isfinite(want_bad[2]))     # the case separates the two forms
    want_good = batch_oracle(oracle_mod, good)
    us = run_batch(sw, good)
    assert sw.last_heat_form() == sw.FORM_FUSED
    assert_batch(us, want_good)
    for insts, want, form in ((bad, want_bad, sw.FORM_CANONICAL),
                              (good, want_good, sw.FORM_FUSED),
                              (bad, want_bad, sw.FORM_CANONICAL)):
        run_batch(sw, insts, us)
        assert sw.last_heat_form() == form
        assert_batch(us, want)


def test_batch_r_outside_the_range_takes_the_canonical_form(sw, oracle_mod):
    insts = mixed_batch(33)
    st, ns, u0, _ = insts[4]
    insts[4] = (st, min(ns, 100), u0, [0.6])
    assert_batch(run_batch(sw, insts), batch_oracle(oracle_mod, insts))
    assert sw.last_heat_form() == sw.FORM_CANONICAL


def test_a_batch_without_heat_leaves_the_record(sw, oracle_mod):
    u0 = workloads.white_noise(1 << 14, seed=83)
    sw.set_tuning(256, 2, 1)
    run(sw, u0, 100, 0.25)
    assert sw.last_heat_form() == sw.FORM_FUSED
    sw.set_tuning(0, 0, sw.MODE_AUTO)
    insts = [i for i in mixed_batch(34) if i[0] == "ks"]
    assert_batch(run_batch(sw, insts), batch_oracle(oracle_mod, insts))
    assert sw.last_heat_form() == sw.FORM_FUSED
