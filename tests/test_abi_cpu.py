"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/swept.h declares, and rejects bad calls with the
documented status codes instead of aborting."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swept.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swept_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def swept():
    import paper_1504_01380_amd as swept
    return swept


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ("swept_init", "swept_advance", "swept_naive_advance", "swept_plan",
                 "swept_set_stream", "swept_set_tuning", "swept_sync", "swept_last_error",
                 "swept_finalize", "swept_naive_substep_advance"):
        assert must in names


def test_library_exports_every_declared_symbol(swept):
    lib = ctypes.CDLL(swept.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(swept.EXPORTS) == declared_functions()


def test_calls_before_init_fail_cleanly(swept):
    lib = swept.lib()
    lib.swept_finalize()
    par = (ctypes.c_double * 1)(0.25)
    rc = lib.swept_advance(ctypes.c_void_p(1), 64, 1, 0, par, 1)
    assert rc == -2  # SWEPT_ENOTINIT
    assert "swept_init" in swept.last_error()
    assert lib.swept_sync() == -2
    assert lib.swept_set_stream(None) == -2
    form = ctypes.c_int32(7)
    assert lib.swept_last_heat_form(ctypes.byref(form)) == -2


def test_heat_form_validation(swept):
    lib = swept.lib()
    assert lib.swept_set_heat_form(2) == -1     # FUSED is reported, not requested
    assert lib.swept_set_heat_form(-1) == -1
    assert lib.swept_last_heat_form(None) == -1
    assert lib.swept_set_heat_form(swept.FORM_CANONICAL) == 0
    assert lib.swept_set_heat_form(swept.FORM_AUTO) == 0


def test_tuning_validation(swept):
    lib = swept.lib()
    assert lib.swept_set_tuning(3, 0, 0) == -1      # odd tile
    assert lib.swept_set_tuning(0, 3, 0) == -1      # bad pairs per lane
    assert lib.swept_set_tuning(0, 0, 9) == -1      # bad mode
    assert lib.swept_set_tuning(0, 0, 6) == -1
    assert lib.swept_set_tuning(0, 0, 5) == 0       # unequal tiles
    assert lib.swept_set_tuning(0, 0, 4) == 0       # the lane-frame kernel
    assert lib.swept_set_tuning(0, 0, 0) == 0
    assert lib.swept_set_tuning(128, 2, 1) == 0
    assert lib.swept_set_tuning(0, 0, 0) == 0


def test_plan_geometry(swept):
    """The planner (host logic, no device needed): tiles of W = 2k points that
    divide the grid, ceil(L/k)+1 stages; unequal tiles for odd grids."""
    lib = swept.lib()
    lib.swept_set_tuning(0, 0, 0)
    p = swept.plan(1 << 24, 20000, "heat")
    assert p["tile_w"] == 1024 and p["depth_k"] == 512 and p["tiles"] == 16384
    assert p["stages"] == 1 + (20000 + 511) // 512 and p["mode"] == swept.MODE_STAGE
    assert p["pairs_per_lane"] == 4
    p = swept.plan(4096, 10000, "heat")
    assert (1 << 24) % p["tile_w"] == 0 and p["tiles"] * p["tile_w"] == 4096
    p = swept.plan(1 << 20, 50000, "ks")
    assert p["stages"] == 1 + (4 * 50000 + p["depth_k"] - 1) // p["depth_k"]
    # odd: unequal tiles of the two-fold cover; tiny odd grids: naive
    assert swept.plan(1001, 5, "heat")["mode"] == swept.MODE_STAGE_RAGGED
    assert swept.plan(127, 5, "heat")["mode"] == swept.MODE_NAIVE
    lib.swept_set_tuning(0, 0, swept.MODE_STAGE)
    out = (ctypes.c_int64 * 6)()
    assert lib.swept_plan(1001, 5, 0, out) == -5                    # SWEPT_EUNSUPPORTED
    lib.swept_set_tuning(48, 0, swept.MODE_STAGE)
    assert swept.plan(96, 5, "heat")["depth_k"] == 24
    assert lib.swept_plan(100, 5, 0, out) == -1                     # 48 does not divide 100
    lib.swept_set_tuning(0, 0, 0)
    assert lib.swept_plan(2, 5, 0, out) == -1                       # nx < 3
    assert lib.swept_plan(64, -1, 0, out) == -1
    assert lib.swept_plan(64, 1, 7, out) == -1


def test_plan_lane_frame(swept):
    """The lane-frame schedule plans tiles of at most 64 points (k <= 32)
    whose rows from the middle level up fit the LDS budget, and reports 0
    pairs per lane."""
    lib = swept.lib()
    try:
        lib.swept_set_tuning(0, 0, swept.MODE_STAGE_LANE)
        p = swept.plan(4096, 100, "heat")
        assert (p["tile_w"], p["depth_k"], p["pairs_per_lane"], p["mode"]) == \
            (64, 32, 0, swept.MODE_STAGE_LANE)
        assert p["stages"] == 1 + (100 + 31) // 32
        p = swept.plan(96, 10, "ks")
        assert p["tile_w"] == 48 and p["mode"] == swept.MODE_STAGE_LANE
        # Euler points are 72 bytes: k = 32 would need 79 KB, so the plan
        # falls back to the widest dividing tile that fits (k = 16 for 4096)
        p = swept.plan(4096, 10, "euler")
        assert p["tile_w"] == 32 and p["mode"] == swept.MODE_STAGE_LANE
        out = (ctypes.c_int64 * 6)()
        lib.swept_set_tuning(128, 0, swept.MODE_STAGE_LANE)
        assert lib.swept_plan(4096, 10, 0, out) == -1          # W = 128 > 64
        lib.swept_set_tuning(0, 0, swept.MODE_STAGE_LANE)
        assert lib.swept_plan(1001, 10, 0, out) == -5          # odd: no even tile
    finally:
        lib.swept_set_tuning(0, 0, 0)


def test_tuner_rejects_bad_requests_without_a_gpu():
    """Validation happens before any device work."""
    import paper_1504_01380_amd as sw
    L = sw.lib()
    import ctypes
    par = (ctypes.c_double * 2)(0.25, 0.0)
    rep = (ctypes.c_double * 8)()
    # not initialised, or invalid: an error code, never a crash
    assert L.swept_autotune(2, 10, 0, par, 1, rep) != 0
    assert L.swept_autotune(4096, 10, 7, par, 1, rep) != 0
    out = (ctypes.c_int64 * 3)()
    assert L.swept_autotune_batch(None, None, None, None, -1, out) != 0
    assert L.swept_clear_tuning() == 0


def test_mean_square_window_bounds_are_checked(swept):
    """A window outside 1..nsteps is rejected before anything runs (J would
    otherwise sum the wrong steps, and the gradient would not match it)."""
    import torch
    u = torch.zeros(16, dtype=torch.float64)
    for bad in (0, -3, 11):
        with pytest.raises(ValueError):
            swept.window_mean_square_value(u, 10, "ks", [0.005, 0.5], bad)
        with pytest.raises(ValueError):
            swept.WindowMeanSquare.apply(u, 10, "ks", [0.005, 0.5], bad)


def test_plan_has_no_cliff_for_awkward_grids(swept):
    """Grids whose even divisors are all far below the target tile (8198 =
    2 x 4099, 8186, 6126, 2^24 + 2) and odd grids get tiles near the target
    depth (the unequal tiling), never 2-point tiles with a stage per step."""
    swept.lib().swept_set_tuning(0, 0, 0)
    for n in (8198, 8186, 6126, (1 << 24) + 2, 1001, (1 << 20) + 1):
        for st in ("heat", "ks", "euler"):
            p = swept.plan(n, 10000, st)
            target = min(1024, n // 16) // 2
            assert p["mode"] == swept.MODE_STAGE_RAGGED, (n, st, p)
            assert p["depth_k"] >= min(target, 128) // 2, (n, st, p)
            L = 10000 * (4 if st != "heat" else 1)
            h = n // 2 if n % 2 == 0 else n          # half the tiled ring
            assert p["stages"] <= (L + p["depth_k"]) * p["tiles"] // h + 2, (n, st, p)
    # a forced unequal tiling of a divisible grid: T - 1 tiles of 600 points
    swept.lib().swept_set_tuning(600, 0, swept.MODE_STAGE_RAGGED)
    p = swept.plan(4096, 100, "heat")
    assert (p["tile_w"], p["tiles"], p["mode"]) == (600, 7, swept.MODE_STAGE_RAGGED)
    swept.lib().swept_set_tuning(0, 0, 0)


def test_batch_schedule_validation(swept):
    """swept_set_batch_schedule needs no device and rejects unknown
    schedules and negative spin limits."""
    lib = swept.lib()
    assert lib.swept_set_batch_schedule(2, 0, 0, 0) == -1
    assert lib.swept_set_batch_schedule(-1, 0, 0, 0) == -1
    assert lib.swept_set_batch_schedule(0, -5, 0, 0) == -1
    assert "spin_limit" in swept.last_error()
    assert lib.swept_set_batch_schedule(0, 0, -1, 0) == -1
    assert lib.swept_set_batch_schedule(0, 0, 33, 0) == -1
    assert "chunk" in swept.last_error()
    assert lib.swept_set_batch_schedule(0, 0, 0, 1025) == -1
    assert "queues" in swept.last_error()
    assert lib.swept_set_batch_schedule(swept.BATCH_STAGED, 100, 4, 8) == 0
    assert lib.swept_set_batch_schedule(swept.BATCH_PERSISTENT, 0, 0, 0) == 0


def test_counting_build_exports(swept):
    """The counting build (SWEPT_COUNT_UPDATES) exports every entry point of
    swept.h and the one of swept_debug.h; the normal library does not export
    the debug one."""
    count_lib = os.path.join(os.path.dirname(swept.LIB_PATH), "libswept_count.so")
    if not os.path.exists(count_lib):
        pytest.skip("libswept_count.so not built")
    lib = ctypes.CDLL(count_lib)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert hasattr(lib, "swept_debug_update_count")
    assert not hasattr(ctypes.CDLL(swept.LIB_PATH), "swept_debug_update_count")
    c = ctypes.c_uint64()
    lib.swept_finalize()
    assert lib.swept_debug_update_count(ctypes.byref(c), 0) == -2    # before swept_init
