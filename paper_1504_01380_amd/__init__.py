"""Python binding of libswept.so, the MI355X swept-rule stencil library.

Argument marshalling only: every sub-timestep of every point runs in the HIP
kernels behind the C ABI declared in include/swept.h.  PyTorch supplies device
memory and the stream.  If the library has not been built this module raises
at import time -- there is no other implementation to fall back to.

    import torch, paper_1504_01380_amd as swept
    u = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
    swept.advance(u, 1000, "heat", [0.25])          # in place, on torch's stream
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswept.so")

HEAT_F64, HEAT_F32, KS_F64, EULER_F64 = 0, 1, 2, 3
# the same schemes with their multiply-adds fused (results equal the above to rounding)
HEAT_F64_FMA, HEAT_F32_FMA, KS_F64_FMA = 4, 5, 6
NOALLOC_SCRATCH_BYTES = 128 << 20   # SWEPT_NOALLOC_SCRATCH_BYTES
MODE_AUTO, MODE_STAGE, MODE_NAIVE, MODE_STAGE_BANDED, MODE_STAGE_LANE, MODE_STAGE_RAGGED = \
    0, 1, 2, 3, 4, 5
BATCH_PERSISTENT, BATCH_STAGED = 0, 1
# how swept_advance evaluates binary64 heat (both give the canonical bits)
FORM_AUTO, FORM_CANONICAL, FORM_FUSED = 0, 1, 2

_STATUS = {0: "SWEPT_OK", -1: "SWEPT_EINVAL", -2: "SWEPT_ENOTINIT", -3: "SWEPT_ENOMEM",
           -4: "SWEPT_EHIP", -5: "SWEPT_EUNSUPPORTED", -6: "SWEPT_ETIMEOUT"}

EXPORTS = ("swept_init", "swept_set_stream", "swept_set_tuning", "swept_set_heat_form",
           "swept_last_heat_form", "swept_plan",
           "swept_advance", "swept_advance_noalloc", "swept_naive_advance",
           "swept_naive_substep_advance",
           "swept_set_profiling", "swept_stage_times", "swept_adjoint", "swept_naive_adjoint",
           "swept_advance_batch", "swept_window_objective",
           "swept_naive_advance_batch", "swept_set_batch_schedule", "swept_autotune",
           "swept_autotune_batch", "swept_clear_tuning",
           "swept_sync", "swept_last_error", "swept_finalize")


class SweptError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__("%s failed: %s (%s)" % (what, msg, _STATUS.get(code, code)))
        self.code = code


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libswept.so is not built (expected at %s); run "
                          "__graft_entry__.build() or python paper_1504_01380_amd/build.py"
                          % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.swept_init.argtypes = [ctypes.c_int]
    L.swept_set_stream.argtypes = [vp]
    L.swept_set_tuning.argtypes = [i32, i32, i32]
    L.swept_set_heat_form.argtypes = [i32]
    L.swept_last_heat_form.argtypes = [ctypes.POINTER(i32)]
    L.swept_plan.argtypes = [i64, i64, i32, ctypes.POINTER(i64)]
    for f in (L.swept_advance, L.swept_advance_noalloc, L.swept_naive_advance,
              L.swept_naive_substep_advance):
        f.argtypes = [vp, i64, i64, i32, dp, i32]
    L.swept_adjoint.argtypes = [vp, vp, i64, i64, i32, dp, i32, i64, ctypes.c_double, vp]
    L.swept_naive_adjoint.argtypes = L.swept_adjoint.argtypes
    L.swept_window_objective.argtypes = [vp, i64, i64, i32, dp, i32, i64, ctypes.c_double, vp, vp]
    L.swept_advance_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                      ctypes.POINTER(i32), dp, i64]
    L.swept_naive_advance_batch.argtypes = L.swept_advance_batch.argtypes
    L.swept_set_batch_schedule.argtypes = [i32, i64, i32, i32]
    L.swept_autotune.argtypes = [i64, i64, i32, dp, i32, dp]
    L.swept_autotune_batch.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                       dp, i64, ctypes.POINTER(i64)]
    L.swept_clear_tuning.argtypes = []
    L.swept_set_profiling.argtypes = [ctypes.c_int]
    L.swept_stage_times.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), i64,
                                    ctypes.POINTER(i64)]
    L.swept_sync.argtypes = []
    L.swept_last_error.argtypes = []
    L.swept_last_error.restype = ctypes.c_char_p
    L.swept_finalize.argtypes = []
    L.swept_finalize.restype = None
    for name in EXPORTS:
        if name not in ("swept_last_error", "swept_finalize"):
            getattr(L, name).restype = ctypes.c_int
    return L


_lib = _load()
_device = None


def lib() -> ctypes.CDLL:
    return _lib


def last_error() -> str:
    return _lib.swept_last_error().decode()


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise SweptError(rc, what, last_error())


def stencil_id(stencil, dtype: torch.dtype | None = None) -> int:
    """'heat' (float64 or float32 by dtype), 'ks', 'euler', their
    contraction-on forms 'heat_fma' and 'ks_fma', or an integer id."""
    if isinstance(stencil, int):
        return stencil
    s = stencil.lower()
    if s == "heat":
        return HEAT_F32 if dtype == torch.float32 else HEAT_F64
    if s == "heat_fma":
        return HEAT_F32_FMA if dtype == torch.float32 else HEAT_F64_FMA
    if s == "ks":
        return KS_F64
    if s == "ks_fma":
        return KS_F64_FMA
    if s == "euler":
        return EULER_F64
    raise ValueError("unknown stencil %r" % (stencil,))


def dtype_of(sid: int) -> torch.dtype:
    return torch.float32 if sid in (HEAT_F32, HEAT_F32_FMA) else torch.float64


def substeps(sid: int) -> int:
    return 4 if sid in (KS_F64, EULER_F64, KS_F64_FMA) else 1


def init(device: int = 0) -> None:
    global _device
    _check(_lib.swept_init(int(device)), "swept_init")
    _device = int(device)


def _prepare(u: torch.Tensor, sid: int) -> int:
    """Check u for the stencil, bind the library to u's device and torch's
    current stream; returns the number of grid points (cells)."""
    if not u.is_cuda:
        raise ValueError("u must be a device tensor")
    if u.dtype != dtype_of(sid):
        raise TypeError("stencil %d needs %s, got %s" % (sid, dtype_of(sid), u.dtype))
    if sid == EULER_F64:
        if not u.is_contiguous() or u.dim() != 2 or u.shape[1] != 3:
            raise ValueError("Euler fields are contiguous (N, 3) tensors of (rho, m, E)")
    elif not u.is_contiguous() or u.dim() != 1:
        raise ValueError("u must be a contiguous 1-D tensor")
    if _device != u.device.index:
        init(u.device.index)
    _check(_lib.swept_set_stream(ctypes.c_void_p(torch.cuda.current_stream(u.device).cuda_stream)),
           "swept_set_stream")
    return u.shape[0]


def _params(params: Sequence[float]):
    arr = (ctypes.c_double * max(1, len(params)))(*[float(p) for p in params])
    return arr, len(params)


def set_tuning(tile_w: int = 0, pairs_per_lane: int = 0, mode: int = MODE_AUTO) -> None:
    _check(_lib.swept_set_tuning(int(tile_w), int(pairs_per_lane), int(mode)), "swept_set_tuning")


def set_heat_form(form: int = FORM_AUTO) -> None:
    """FORM_AUTO (the fused Laplacian where the library's range check allows
    it) or FORM_CANONICAL (the five operations as written) for heat in
    advance() and advance_batch(); both give the same bits."""
    _check(_lib.swept_set_heat_form(int(form)), "swept_set_heat_form")


def last_heat_form() -> int:
    """FORM_FUSED or FORM_CANONICAL: how the last heat advance(), or the
    last advance_batch() with a heat instance, evaluated its updates (0
    before any); synchronises the library's stream."""
    out = ctypes.c_int32(0)
    _check(_lib.swept_last_heat_form(ctypes.byref(out)), "swept_last_heat_form")
    return int(out.value)


def set_batch_schedule(schedule: int = BATCH_PERSISTENT, spin_limit: int = 0,
                       chunk: int = 0, queues: int = 0) -> None:
    """BATCH_PERSISTENT (one launch per stencil for the whole batch) or
    BATCH_STAGED (one launch per stage); for the persistent one, the wait
    limit in microseconds, the task numbers per claim and the number of
    queues (0: the library's defaults)."""
    _check(_lib.swept_set_batch_schedule(int(schedule), int(spin_limit), int(chunk),
                                         int(queues)), "swept_set_batch_schedule")


def plan(nx: int, nsteps: int, stencil, dtype: torch.dtype | None = None) -> dict:
    out = (ctypes.c_int64 * 6)()
    _check(_lib.swept_plan(int(nx), int(nsteps), stencil_id(stencil, dtype), out), "swept_plan")
    keys = ("tile_w", "depth_k", "tiles", "stages", "pairs_per_lane", "mode")
    return dict(zip(keys, [int(v) for v in out]))


def advance(u: torch.Tensor, nsteps: int, stencil, params: Sequence[float]) -> torch.Tensor:
    """Advance u in place by nsteps time steps with the swept rule."""
    sid = stencil_id(stencil, u.dtype)
    nx = _prepare(u, sid)
    p, npar = _params(params)
    _check(_lib.swept_advance(ctypes.c_void_p(u.data_ptr()), nx, int(nsteps), sid, p, npar),
           "swept_advance")
    return u


def advance_noalloc(u: torch.Tensor, nsteps: int, stencil, params: Sequence[float]) -> torch.Tensor:
    """advance() with the library's fixed scratch array: the call allocates no
    device memory (for graph capture and serving loops); sizes beyond
    NOALLOC_SCRATCH_BYTES of scratch raise SweptError."""
    sid = stencil_id(stencil, u.dtype)
    nx = _prepare(u, sid)
    p, npar = _params(params)
    _check(_lib.swept_advance_noalloc(ctypes.c_void_p(u.data_ptr()), nx, int(nsteps), sid, p,
                                      npar), "swept_advance_noalloc")
    return u


def naive_advance(u: torch.Tensor, nsteps: int, stencil, params: Sequence[float]) -> torch.Tensor:
    """Advance u in place with one kernel launch per time step."""
    sid = stencil_id(stencil, u.dtype)
    nx = _prepare(u, sid)
    p, npar = _params(params)
    _check(_lib.swept_naive_advance(ctypes.c_void_p(u.data_ptr()), nx, int(nsteps), sid,
                                    p, npar), "swept_naive_advance")
    return u


def naive_substep_advance(u: torch.Tensor, nsteps: int, stencil, params: Sequence[float]):
    """KS and Euler: one kernel launch per sub-timestep."""
    sid = stencil_id(stencil, u.dtype)
    nx = _prepare(u, sid)
    p, npar = _params(params)
    _check(_lib.swept_naive_substep_advance(ctypes.c_void_p(u.data_ptr()), nx, int(nsteps),
                                            sid, p, npar), "swept_naive_substep_advance")
    return u


def _batch_args(us, nsteps, stencils, params):
    count = len(us)
    if not (len(nsteps) == len(stencils) == len(params) == count):
        raise ValueError("batch arrays differ in length")
    for u in us:
        if u.dtype != torch.float64:
            raise TypeError("the batch takes float64 fields")
    _prepare(us[0], HEAT_F64)
    for u in us:
        if not u.is_cuda or not u.is_contiguous() or u.dim() != 1 or u.device != us[0].device:
            raise ValueError("batch fields must be contiguous 1-D tensors on one device")
    ptrs = (ctypes.c_void_p * count)(*[u.data_ptr() for u in us])
    nx = (ctypes.c_int64 * count)(*[u.numel() for u in us])
    ns = (ctypes.c_int64 * count)(*[int(n) for n in nsteps])
    ids = (ctypes.c_int32 * count)(*[stencil_id(st, torch.float64) for st in stencils])
    flat = []
    for p in params:
        flat += (list(p) + [0.0, 0.0])[:2]
    par = (ctypes.c_double * (2 * count))(*flat)
    return ptrs, nx, ns, ids, par, count


def advance_batch(us: Sequence[torch.Tensor], nsteps: Sequence[int], stencils,
                  params: Sequence[Sequence[float]]) -> None:
    """Advance independent float64 fields in place, instance j by nsteps[j]
    steps of stencils[j] ("heat" or "ks") with params[j], in one batched
    swept run (one HIP graph)."""
    if len(us) == 0:
        return
    _check(_lib.swept_advance_batch(*_batch_args(us, nsteps, stencils, params)),
           "swept_advance_batch")


def naive_advance_batch(us: Sequence[torch.Tensor], nsteps: Sequence[int], stencils,
                        params: Sequence[Sequence[float]]) -> None:
    """The same as advance_batch with the naive schedule (one launch per time
    step over all instances still running)."""
    if len(us) == 0:
        return
    _check(_lib.swept_naive_advance_batch(*_batch_args(us, nsteps, stencils, params)),
           "swept_naive_advance_batch")


def autotune(nx: int, nsteps: int, stencil, params: Sequence[float],
             dtype: torch.dtype | None = None) -> dict:
    """Measure tau, s1 and s_full, form the prior tile width of Eq. (1) and
    keep the fastest of the timed candidates for later automatic advances of
    this stencil and size class.  Returns the model and the choice."""
    arr, npar = _params(params)
    rep = (ctypes.c_double * 8)()
    _check(_lib.swept_autotune(int(nx), int(nsteps), stencil_id(stencil, dtype), arr, npar, rep),
           "swept_autotune")
    keys = ("tau", "s1", "s_full", "n_star", "w0", "tile_w", "pairs_per_lane", "probe_rate")
    out = dict(zip(keys, list(rep)))
    out["tile_w"] = int(out["tile_w"])
    out["pairs_per_lane"] = int(out["pairs_per_lane"])
    return out


def autotune_batch(sizes: Sequence[int], nsteps: Sequence[int], stencils,
                   params: Sequence[Sequence[float]]) -> dict:
    """Choose the batch depth per stencil from timed probes of this batch's
    shapes; returns {"heat": k, "ks": k} for the stencils present."""
    count = len(sizes)
    nx = (ctypes.c_int64 * max(1, count))(*[int(n) for n in sizes])
    ns = (ctypes.c_int64 * max(1, count))(*[int(n) for n in nsteps])
    ids = (ctypes.c_int32 * max(1, count))(*[stencil_id(st, torch.float64) for st in stencils])
    flat = []
    for p in params:
        flat += (list(p) + [0.0, 0.0])[:2]
    par = (ctypes.c_double * max(2, len(flat)))(*flat)
    out = (ctypes.c_int64 * 3)()
    _check(_lib.swept_autotune_batch(nx, ns, ids, par, count, out), "swept_autotune_batch")
    res = {}
    if out[HEAT_F64]:
        res["heat"] = int(out[HEAT_F64])
    if out[KS_F64]:
        res["ks"] = int(out[KS_F64])
    return res


def clear_tuning() -> None:
    _check(_lib.swept_clear_tuning(), "swept_clear_tuning")


def set_profiling(enable: bool) -> None:
    _check(_lib.swept_set_profiling(1 if enable else 0), "swept_set_profiling")


def stage_times():
    """(ms, kind) per stage launch of the most recent profiled swept_advance;
    kind 0 = banded kernel (triangle or capped stage), 1 = continuous kernel."""
    count = ctypes.c_int64(0)
    _check(_lib.swept_stage_times(None, None, 0, ctypes.byref(count)), "swept_stage_times")
    n = count.value
    ms = (ctypes.c_double * max(1, n))()
    kind = (ctypes.c_int32 * max(1, n))()
    _check(_lib.swept_stage_times(ms, kind, n, ctypes.byref(count)), "swept_stage_times")
    return [float(ms[i]) for i in range(n)], [int(kind[i]) for i in range(n)]


def _adjoint_call(fn, what, u0, nsteps, stencil, params, window_first, window_weight, cot_final):
    sid = stencil_id(stencil, u0.dtype)
    nx = _prepare(u0, sid)
    grad = torch.empty_like(u0)
    cot = None
    if cot_final is not None:
        cot = cot_final.contiguous()
        if cot.shape != u0.shape or cot.dtype != u0.dtype or cot.device != u0.device:
            raise ValueError("cot_final must match u0")
    first = nsteps + 1 if window_first is None else int(window_first)
    p, npar = _params(params)
    _check(fn(ctypes.c_void_p(u0.data_ptr()), ctypes.c_void_p(grad.data_ptr()), nx, int(nsteps),
              sid, p, npar, first, float(window_weight),
              None if cot is None else ctypes.c_void_p(cot.data_ptr())), what)
    return grad


def adjoint(u0: torch.Tensor, nsteps: int, stencil, params: Sequence[float], *,
            window_first: int | None = None, window_weight: float = 0.0,
            cot_final: torch.Tensor | None = None) -> torch.Tensor:
    """dJ/du0 by the swept discrete adjoint, for
    J = window_weight * sum_{j=window_first}^{nsteps} |u^j|^2 + <cot_final, u^nsteps>."""
    return _adjoint_call(_lib.swept_adjoint, "swept_adjoint", u0, nsteps, stencil, params,
                         window_first, window_weight, cot_final)


def naive_adjoint(u0: torch.Tensor, nsteps: int, stencil, params: Sequence[float], *,
                  window_first: int | None = None, window_weight: float = 0.0,
                  cot_final: torch.Tensor | None = None) -> torch.Tensor:
    """The same gradient by the straight decomposition (one launch per step
    forward, keeping every step, and one per step backward)."""
    return _adjoint_call(_lib.swept_naive_adjoint, "swept_naive_adjoint", u0, nsteps, stencil,
                         params, window_first, window_weight, cot_final)


class SweptAdvance(torch.autograd.Function):
    """u = advance(u0, nsteps); backward by the swept adjoint."""

    @staticmethod
    def forward(ctx, u0, nsteps, stencil, params):
        u = u0.detach().clone()
        advance(u, nsteps, stencil, params)
        ctx.save_for_backward(u0.detach())
        ctx.args = (nsteps, stencil, tuple(params))
        return u

    @staticmethod
    def backward(ctx, grad_out):
        (u0,) = ctx.saved_tensors
        nsteps, stencil, params = ctx.args
        g = adjoint(u0, nsteps, stencil, params, cot_final=grad_out.contiguous())
        return g, None, None, None


def _check_window(nsteps: int, window: int) -> None:
    if not 1 <= int(window) <= int(nsteps):
        raise ValueError("window = %r must satisfy 1 <= window <= nsteps = %r" % (window, nsteps))


def objective(u0: torch.Tensor, nsteps: int, stencil, params: Sequence[float], *,
              window_first: int | None = None, window_weight: float = 0.0,
              cot_final: torch.Tensor | None = None) -> torch.Tensor:
    """J = window_weight * sum_{j=window_first}^{nsteps} |u^j|^2 + <cot_final, u^nsteps>,
    the objective of adjoint(), computed by the library; a 0-d float64 device
    tensor (the call is asynchronous on torch's stream)."""
    sid = stencil_id(stencil, u0.dtype)
    nx = _prepare(u0, sid)
    cot = None
    if cot_final is not None:
        cot = cot_final.contiguous()
        if cot.shape != u0.shape or cot.dtype != u0.dtype or cot.device != u0.device:
            raise ValueError("cot_final must match u0")
    J = torch.empty((), dtype=torch.float64, device=u0.device)
    first = nsteps + 1 if window_first is None else int(window_first)
    p, npar = _params(params)
    _check(_lib.swept_window_objective(ctypes.c_void_p(u0.data_ptr()), nx, int(nsteps), sid, p,
                                       npar, first, float(window_weight),
                                       None if cot is None else ctypes.c_void_p(cot.data_ptr()),
                                       ctypes.c_void_p(J.data_ptr())), "swept_window_objective")
    return J


def window_mean_square_value(u0: torch.Tensor, nsteps: int, stencil, params, window: int):
    """J = mean of u^2 over all points and the last `window` time steps
    (steps nsteps-window+1 .. nsteps), computed by the library."""
    _check_window(nsteps, window)
    return objective(u0.detach(), nsteps, stencil, params, window_first=nsteps - window + 1,
                     window_weight=1.0 / (window * u0.numel()))


class WindowMeanSquare(torch.autograd.Function):
    """J(u0) = mean of u^2 over the final `window` steps; gradient by the
    swept adjoint with one checkpoint per sweep."""

    @staticmethod
    def forward(ctx, u0, nsteps, stencil, params, window):
        _check_window(nsteps, window)
        ctx.save_for_backward(u0.detach())
        ctx.args = (nsteps, stencil, tuple(params), window)
        return window_mean_square_value(u0, nsteps, stencil, params, window)

    @staticmethod
    def backward(ctx, grad_out):
        (u0,) = ctx.saved_tensors
        nsteps, stencil, params, window = ctx.args
        g = adjoint(u0, nsteps, stencil, params, window_first=nsteps - window + 1,
                    window_weight=1.0 / (window * u0.numel()))
        return g * grad_out, None, None, None, None


def sync() -> None:
    _check(_lib.swept_sync(), "swept_sync")


def finalize() -> None:
    global _device
    _lib.swept_finalize()
    _device = None
