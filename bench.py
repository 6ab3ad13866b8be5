"""Benchmark: point-updates/s of the swept rule vs naive per-step stepping on
one MI355X, with the roofline fraction of the dominant kernel and the CPU
oracle timed beside it.

Workload (one bench "step" = one whole run of it, inputs resident in HBM):
heat equation u_t = u_xx, periodic, N = 2^24 points, 3-point forward Euler,
r = 0.25, 20,000 time steps, u0 ~ U[-1, 1] (seed 1001), binary64.  The same
run in binary32 and the naive one-launch-per-step schedule are reported
beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published figures; VALU issue rate derived from the unit counts.
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_HZ = 256, 4, 16, 2.4e9
VALU_LANE_OPS = CUS * SIMDS_PER_CU * LANES_PER_SIMD * CLOCK_HZ   # 39.3e12 FP64 ops per second
# 32-bit VALU operations issue at twice that rate on CDNA4 (the published
# 157.3 TFLOP/s FP32 vector peak = 78.6e12 non-fused FP32 ops/s x 2 for FMA).
VALU_LANE_OPS_F32 = 2 * VALU_LANE_OPS
HBM_PEAK = 8.0e12
HEAT_OPS_PER_UPDATE = 5           # add, mul, sub, mul, add (no fused multiply-add)
# the same bits in four: add, fma(-2, u, s), mul, add (the fused-Laplacian form the
# library takes for binary64 heat once its range check passes); an FMA issues once
HEAT_FUSED_LAP_OPS = 4
HEAT_FMA_OPS_PER_UPDATE = 3       # add, fma, fma (the contraction-on stencil)
KS_FMA_OPS_PER_STEP = 22          # 3 + 8 + 3 + 8 instructions per point-step, fused
# LDS: 128 bytes per clock per CU (the CDNA3 ISA figure; the CDNA4 LDS is
# 160 KB per CU, its rate taken as the same)
LDS_PEAK = CUS * 128 * CLOCK_HZ
HEAT_NAIVE_BYTES = {8: 16, 4: 8}  # read u, write u' per point-update


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--nsteps", type=int, default=20_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-naive", action="store_true", help="skip the naive and f32 legs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the untuned plans (no autotuner in the warm-up)")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: a plain copy of u (calibration), the "
                         "timed swept runs, then 50 naive steps")
    ap.add_argument("--sweep", action="store_true",
                    help="the headline workload at every tile width W in {512, ..., 4096} and "
                         "pairs per lane, one JSON line each (instead of the benchmark line)")
    ap.add_argument("--size-sweep", action="store_true",
                    help="heat (10,000 steps) and KS (2,000 steps) at N = 2^12 ... 2^24 / 2^20, "
                         "autotuned swept against naive, one JSON line each (instead of the "
                         "benchmark line)")
    ap.add_argument("--profile-mix", action="store_true",
                    help="short run for rocprofv3 instruction counters: one swept run each of "
                         "heat (2^24, 2,000 steps, W=1024 P=4), KS (2^20, 1,000 steps, W=1024 "
                         "P=4) and Euler (2^20 cells, 300 steps, W=256 P=1)")
    return ap.parse_args()


def progress(msg: str) -> None:
    """One line on stderr per finished leg (the JSON result goes to stdout)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def timed_runs(sw, torch, fn, u0, nsteps, params, reps, warmup, after=None, stencil="heat"):
    """Run fn `reps` times on copies of u0; HIP events on the stream the
    library launches on (torch's current stream) bracket each run.  `after`
    runs once the closing event of a timed run has completed."""
    stream = torch.cuda.current_stream()
    u = u0.clone()
    for _ in range(warmup):
        u.copy_(u0)
        fn(u, nsteps, stencil, params)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        u.copy_(u0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(u, nsteps, stencil, params)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
        if after is not None:
            after()
    sw.sync()
    return times, u


KERNEL_SOURCES = [os.path.join(ROOT, "paper_1504_01380_amd", "csrc", f)
                  for f in ("kernels.hpp", "stencils.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_heat_f64.json")


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None if
    there is none or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha") != kernel_source_sha() or rec.get("kernel") != kernel:
        return None
    return rec.get("bytes_per_launch")


def host_cpu():
    """The host CPU's model name, and the physical cores and sockets behind
    the CPUs this process may run on (from /proc/cpuinfo and the affinity
    mask)."""
    usable = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    model, cores, sockets = "", set(), set()
    try:
        with open("/proc/cpuinfo") as fh:
            blocks = fh.read().strip().split("\n\n")
        for b in blocks:
            kv = {}
            for ln in b.split("\n"):
                if ":" in ln:
                    a, v = ln.split(":", 1)
                    kv[a.strip()] = v.strip()
            cpu = int(kv.get("processor", -1))
            if usable and cpu not in usable:
                continue
            model = model or kv.get("model name", "")
            phys = kv.get("physical id", "0")
            sockets.add(phys)
            cores.add((phys, kv.get("core id", str(cpu))))
    except (OSError, ValueError):
        pass
    return {"model": model, "physical_cores": len(cores) or None,
            "sockets": len(sockets) or None, "usable_cpus": len(usable) or os.cpu_count()}


def cpu_baseline(u0_np, nsteps_full, seconds):
    """The oracle as it stands, on the host cores, on the first few steps of
    the same workload (all N points), sized to about `seconds` of work."""
    import oracle
    oracle.build(force=False)
    n = u0_np.size
    threads = oracle.max_threads()
    oracle.heat(u0_np, 2, 0.25, threads=threads)      # first touch, thread start-up
    t0 = time.perf_counter()
    oracle.heat(u0_np, 20, 0.25, threads=threads)
    per_step = max((time.perf_counter() - t0) / 20, 1e-6)
    # step on from the field reached, in chunks sized by the rate so far,
    # until about `seconds` of work (or all steps) are done
    u, k, dt = u0_np, 0, 0.0
    while k < nsteps_full and dt < 0.9 * seconds:
        chunk = int(max(2, min(nsteps_full - k, (seconds - dt) / per_step)))
        t0 = time.perf_counter()
        u = oracle.heat(u, chunk, 0.25, threads=threads)
        dt += time.perf_counter() - t0
        k += chunk
        per_step = dt / k
    # one thread, on a few steps of the same field (a fifth of the time)
    per1 = (dt / k) * threads
    k1 = int(max(2, min(nsteps_full, 0.2 * seconds / per1)))
    t0 = time.perf_counter()
    oracle.heat(u0_np, k1, 0.25, threads=1)
    dt1 = time.perf_counter() - t0
    host = host_cpu()
    return {"value": n * k / dt, "unit": "point-updates/s", "cores": threads, "kind": "oracle",
            "sample": "heat f64 N=%d, first %d of %d steps, all points, OpenMP %d threads, "
                      "%.1f s" % (n, k, nsteps_full, threads, dt),
            "single_thread": {"value": n * k1 / dt1, "sample": "first %d steps, 1 thread, %.1f s"
                              % (k1, dt1)},
            "cpu": host["model"], "physical_cores": host["physical_cores"],
            "sockets": host["sockets"], "usable_cpus": host["usable_cpus"],
            "host_cpus": os.cpu_count()}


KS_OPS_PER_STEP = 30  # per point-step: 4 sub-timesteps (4 + 11 + 4 + 11 flops, no FMA)
# Euler, per cell-step: two slope sub-timesteps (9 each) and two flux-difference
# sub-timesteps (151 each: two faces of 71 and the 9-flop update), counting a
# division, a square root, |x| and a min/max as one flop each.
EULER_OPS_PER_STEP = 320


def heat_ops(sw) -> int:
    """VALU instructions per heat update of the last swept_advance call: 4
    in the fused-Laplacian form, 5 in the canonical one."""
    return HEAT_FUSED_LAP_OPS if sw.last_heat_form() == sw.FORM_FUSED else HEAT_OPS_PER_UPDATE


def other_workloads(sw, torch, workloads, tune=True):
    """The other single-field workloads: heat N=4096 (launch-latency bound
    when stepped naively), KS N=2^20 and Euler N=2^20 cells (four
    sub-timesteps per step), each after the autotuner has chosen its
    tiling."""
    out = {}
    we, wes = workloads.WORKLOADS["euler"], workloads.WORKLOADS["euler_small"]
    cases = [("heat_small", "heat", workloads.WORKLOADS["heat_small"], [0.25],
              HEAT_OPS_PER_UPDATE, 16),
             ("ks", "ks", workloads.WORKLOADS["ks"],
              [workloads.KS_DT, workloads.KS_DX], KS_OPS_PER_STEP, 16),
             ("euler", "euler", we, [we["cfl"] / we["n"], 1.0 / we["n"], we["gamma"]],
              EULER_OPS_PER_STEP, 48),
             ("euler_small", "euler", wes, [wes["cfl"] / wes["n"], 1.0 / wes["n"], wes["gamma"]],
              EULER_OPS_PER_STEP, 48)]
    for name, st, w, par, ops, naive_bytes in cases:
        u0 = torch.from_numpy(workloads.initial(name)).cuda()
        n, nsteps = u0.shape[0], w["nsteps"]
        tuned = sw.autotune(n, nsteps, st, par) if tune else None
        plan = sw.plan(n, nsteps, st)
        rec = {"n": n, "time_steps": nsteps, "tile_w": plan["tile_w"],
               "pairs_per_lane": plan["pairs_per_lane"], "stages": plan["stages"],
               "mode": plan["mode"], "tuning": tuned}
        for label, fn, reps in (("swept", sw.advance, 3), ("naive", sw.naive_advance, 1)):
            u = u0.clone()
            fn(u, nsteps, st, par)           # warm-up
            ts = []
            for _ in range(reps):
                u.copy_(u0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fn(u, nsteps, st, par)
                e1.record()
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) / 1e3)
            t = sum(ts) / len(ts)
            rec[label] = n * nsteps / t
            rec[label + "_ms"] = t * 1e3
            if label == "swept" and st == "heat":
                ops = heat_ops(sw)
                rec["ops_per_update"] = ops
        rec["speedup_vs_naive"] = rec["swept"] / rec["naive"]
        rec["swept_frac_alu"] = ops * rec["swept"] / VALU_LANE_OPS
        rec["naive_GBps"] = naive_bytes * rec["naive"] / 1e9
        if st in ("ks", "euler"):
            u = u0.clone()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            sw.naive_substep_advance(u, nsteps, st, par)
            e1.record()
            e1.synchronize()
            t = e0.elapsed_time(e1) / 1e3
            rec["naive_substep"] = n * nsteps / t
            rec["speedup_vs_naive_substep"] = rec["swept"] / rec["naive_substep"]
        sw.sync()
        out[name] = rec
        progress("%s done" % name)
    return out


def batch_workload(sw, torch, workloads, tune=True):
    """The ensemble: 4096 independent instances (half heat, half KS, N
    log-uniform in [256, 65536], 1,000-20,000 steps) in one batched swept
    run, against the batched naive schedule (one launch per time step over
    all instances still running).  Rates count each instance's own N x steps
    (the two-fold cover of an odd ring is overhead, not work)."""
    insts = workloads.batch()
    ns = [i.nsteps for i in insts]
    kinds = [i.stencil for i in insts]
    pars = [[0.25] if k == "heat" else [workloads.KS_DT, workloads.KS_DX] for k in kinds]
    u0 = [torch.from_numpy(i.u0).cuda() for i in insts]
    us = [u.clone() for u in u0]
    work = float(sum(i.n * i.nsteps for i in insts))
    rec = {"instances": len(insts), "total_points": sum(i.n for i in insts),
           "point_steps": work, "odd_instances": sum(i.n % 2 for i in insts)}
    if tune:
        t0 = time.perf_counter()
        rec["tuned_depth"] = sw.autotune_batch([i.n for i in insts], ns, kinds, pars)
        rec["tune_s"] = time.perf_counter() - t0

    def restore():
        for a, b in zip(us, u0):
            a.copy_(b)
        torch.cuda.synchronize()

    def timed(schedule):
        sw.set_batch_schedule(schedule, 0)
        t0 = time.perf_counter()
        sw.advance_batch(us, ns, kinds, pars)     # warm-up: plan, capture the graph
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        ts = []
        for _ in range(3):
            restore()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sw.advance_batch(us, ns, kinds, pars)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        sw.sync()
        return sorted(ts)[1], first

    # one launch per stage first, then the default: one persistent launch
    ts_, _ = timed(sw.BATCH_STAGED)
    rec["staged"] = work / ts_
    rec["staged_ms"] = ts_ * 1e3
    t, rec["first_call_s"] = timed(sw.BATCH_PERSISTENT)
    rec["schedule"] = "persistent (one launch, per-tile stage flags)"
    rec["swept"] = work / t
    rec["swept_ms"] = t * 1e3
    rec["persistent_vs_staged"] = ts_ / t
    rec["heat_form"] = "fused-Laplacian" if sw.last_heat_form() == sw.FORM_FUSED else "canonical"
    sw.naive_advance_batch(us[:64], [min(x, 4) for x in ns[:64]], kinds[:64], pars[:64])
    restore()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sw.naive_advance_batch(us, ns, kinds, pars)
    e1.record()
    e1.synchronize()
    tn = e0.elapsed_time(e1) / 1e3
    rec["naive"] = work / tn
    rec["naive_ms"] = tn * 1e3
    rec["speedup_vs_naive"] = rec["swept"] / rec["naive"]
    sw.sync()
    return rec


def ks_adjoint_workload(sw, torch, workloads, directions=16):
    """Gradient of J = mean of u^2 over the final 2,000 of 20,000 KS steps
    (N = 2^16) by the swept adjoint, timed, and checked along the 16 seeded
    unit directions of workloads.adjoint_directions:
      - against the oracle's tangent-linear derivatives (forward mode, no
        truncation error; tests/golden/ks_adjoint_tlm.json, written from the
        oracle alone);
      - against central finite differences of J (computed by the library) at
        several eps, with one and two levels of Richardson extrapolation, so
        that the finite-difference error can be split into truncation (falls
        as eps^2) and round-off (grows as 1/eps)."""
    import math
    w = workloads.WORKLOADS["ks_adjoint"]
    window = workloads.KS_ADJOINT_WINDOW
    n, nsteps, par = w["n"], w["nsteps"], [w["dt"], w["dx"]]
    u0 = torch.from_numpy(workloads.initial("ks_adjoint")).cuda()
    wgt = 1.0 / (window * n)
    first = nsteps - window + 1
    sw.adjoint(u0, nsteps, "ks", par, window_first=first, window_weight=wgt)   # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g = sw.adjoint(u0, nsteps, "ks", par, window_first=first, window_weight=wgt)
    e1.record()
    e1.synchronize()
    t_adj = e0.elapsed_time(e1) / 1e3

    def J(u):
        return float(sw.window_mean_square_value(u, nsteps, "ks", par, window))

    # the straight-decomposition adjoint (one launch per step each way,
    # every step's field kept) on the same objective
    gn = sw.naive_adjoint(u0, nsteps, "ks", par, window_first=first, window_weight=wgt)
    torch.cuda.synchronize()
    e0.record()
    gn = sw.naive_adjoint(u0, nsteps, "ks", par, window_first=first, window_weight=wgt)
    e1.record()
    e1.synchronize()
    t_naive = e0.elapsed_time(e1) / 1e3
    same = bool(torch.equal(gn.view(torch.int64), g.view(torch.int64)))
    del gn
    torch.cuda.empty_cache()

    dirs = workloads.adjoint_directions(n, directions)
    g_np = g.cpu().numpy()
    gv = [math.fsum(g_np * dirs[q]) for q in range(directions)]
    rec = {"n": n, "time_steps": nsteps, "window": window, "adjoint_ms": t_adj * 1e3,
           "gradient_point_steps_per_s": n * nsteps / t_adj,
           "naive_adjoint_ms": t_naive * 1e3,
           "naive_gradient_point_steps_per_s": n * nsteps / t_naive,
           "speedup_vs_naive": t_naive / t_adj, "naive_equals_swept_bitwise": same,
           "directions": directions}
    t0 = time.perf_counter()
    J0 = J(u0)
    rec["J"] = J0
    rec["objective_ms"] = (time.perf_counter() - t0) * 1e3
    golden = os.path.join(ROOT, "tests", "golden", "ks_adjoint_tlm.json")
    ref = gv
    if os.path.exists(golden):
        with open(golden) as fh:
            gold = json.load(fh)
        tlm = [float.fromhex(x) for x in gold["dJ"]][:directions]
        ref = tlm
        terr = [abs(a - b) / abs(b) for a, b in zip(gv, tlm)]
        rec["tlm_rel_err_max"] = max(terr)
        rec["tlm_rel_err_median"] = sorted(terr)[len(terr) // 2]
        rec["J_rel_err_vs_oracle"] = abs(J0 - float.fromhex(gold["J"])) / abs(float.fromhex(gold["J"]))
    rec["reference"] = "oracle tangent-linear" if ref is not gv else "<g, v>"

    def rel(vals):
        e = sorted(abs(a - b) / abs(b) for a, b in zip(vals, ref))
        return {"max": e[-1], "median": e[len(e) // 2], "within_1e-6": sum(x <= 1e-6 for x in e)}

    fd = {}
    for eps in (1e-6, 5e-7, 2.5e-7, 1.25e-7, 1e-7, 1e-8):
        vals = []
        for q in range(directions):
            v = torch.from_numpy(dirs[q]).cuda()
            vals.append((J(u0 + eps * v) - J(u0 - eps * v)) / (2 * eps))
        fd[eps] = vals
    rich1 = [(4 * b - a) / 3 for a, b in zip(fd[1e-6], fd[5e-7])]
    rich1b = [(4 * b - a) / 3 for a, b in zip(fd[5e-7], fd[2.5e-7])]
    rich1c = [(4 * b - a) / 3 for a, b in zip(fd[2.5e-7], fd[1.25e-7])]
    rich2 = [(16 * b - a) / 15 for a, b in zip(rich1, rich1b)]
    rich2b = [(16 * b - a) / 15 for a, b in zip(rich1b, rich1c)]
    rich3 = [(64 * b - a) / 63 for a, b in zip(rich2, rich2b)]
    rec["fd"] = {"%g" % e: rel(v) for e, v in fd.items()}
    rec["fd_richardson_1e-6_5e-7"] = rel(rich1)
    rec["fd_richardson2_1e-6_5e-7_2.5e-7"] = rel(rich2)
    rec["fd_richardson3_1e-6_to_1.25e-7"] = rel(rich3)
    # the literal check: eps = 1e-6, against the adjoint's <g, v>
    lit = sorted(abs(a - b) / abs(b) for a, b in zip(fd[1e-6], gv))
    rec.update({"fd_eps": 1e-6, "fd_directions": directions, "fd_rel_err_max": lit[-1],
                "fd_rel_err_median": lit[len(lit) // 2],
                "fd_within_1e-6": sum(x <= 1e-6 for x in lit)})
    sw.sync()
    return rec


def fma_legs(sw, torch, workloads, u0, u_canonical, nsteps, updates, tune=True):
    """The contraction-on stencils beside the bit-exact headline, never in
    its place: heat f64 on the headline workload (3 instructions per update:
    add, fma, fma) and KS on its workload (22 per point-step), each swept
    (autotuned) and naive.  At r = 1/4 every product r*lap is exact, so the
    fused heat run must give the canonical run's bits."""
    out = {}
    tune_h = sw.autotune(u0.numel(), nsteps, "heat_fma", [0.25], torch.float64) if tune else None
    plan = sw.plan(u0.numel(), nsteps, "heat_fma", torch.float64)
    st, uf = timed_runs(sw, torch, sw.advance, u0, nsteps, [0.25], 2, 1, stencil="heat_fma")
    nt, _ = timed_runs(sw, torch, sw.naive_advance, u0, nsteps, [0.25], 1, 1, stencil="heat_fma")
    v = updates / (sum(st) / len(st))
    nv = updates / nt[0]
    out["heat_f64"] = {"swept": v, "naive": nv, "speedup_vs_naive": v / nv,
                       "ops_per_update": HEAT_FMA_OPS_PER_UPDATE,
                       "swept_frac_alu": HEAT_FMA_OPS_PER_UPDATE * v / VALU_LANE_OPS,
                       "bits_equal_canonical": bool(torch.equal(uf.view(torch.int64),
                                                                u_canonical.view(torch.int64))),
                       "tile_w": plan["tile_w"], "pairs_per_lane": plan["pairs_per_lane"],
                       "tuning": tune_h}
    del uf
    wk = workloads.WORKLOADS["ks"]
    par = [wk["dt"], wk["dx"]]
    k0 = torch.from_numpy(workloads.initial("ks")).cuda()
    n, ns = k0.numel(), wk["nsteps"]
    tune_k = sw.autotune(n, ns, "ks_fma", par) if tune else None
    plan = sw.plan(n, ns, "ks_fma")
    st, _ = timed_runs(sw, torch, sw.advance, k0, ns, par, 3, 1, stencil="ks_fma")
    nt, _ = timed_runs(sw, torch, sw.naive_advance, k0, ns, par, 1, 1, stencil="ks_fma")
    v = n * ns / (sum(st) / len(st))
    nv = n * ns / nt[0]
    out["ks"] = {"swept": v, "naive": nv, "speedup_vs_naive": v / nv,
                 "ops_per_point_step": KS_FMA_OPS_PER_STEP,
                 "swept_frac_alu": KS_FMA_OPS_PER_STEP * v / VALU_LANE_OPS,
                 "tile_w": plan["tile_w"], "pairs_per_lane": plan["pairs_per_lane"],
                 "tuning": tune_k}
    sw.sync()
    return out


def profile_mix(sw, torch, workloads):
    """One swept run of each single-field stencil in its tuned launch shape,
    for counter collection (nothing is timed or printed but progress)."""
    we, wk = workloads.WORKLOADS["euler"], workloads.WORKLOADS["ks"]
    for name, st, nsteps, par, W, P in (
            ("heat_large", "heat", 2000, [0.25], 1024, 4),
            ("ks", "ks", 1000, [wk["dt"], wk["dx"]], 1024, 4),
            ("euler", "euler", 300, [we["cfl"] / we["n"], 1.0 / we["n"], we["gamma"]], 256, 1)):
        sw.set_tuning(W, P, sw.MODE_AUTO)
        u = torch.from_numpy(workloads.initial(name)).cuda()
        sw.advance(u, nsteps, st, par)
        torch.cuda.synchronize()
        progress("%s done" % name)
    sw.set_tuning(0, 0, sw.MODE_AUTO)


def tile_sweep(sw, torch, workloads, args):
    """The headline heat workload (2^24 points, 20,000 steps, f64) on each
    tiling W x pairs per lane, timed like the benchmark (best of two runs
    after one warm-up): one JSON line per tiling."""
    n, nsteps = args.n, args.nsteps
    u0 = torch.from_numpy(workloads.white_noise(
        n, seed=workloads.WORKLOADS["heat_large"]["seed"])).cuda()
    for W in (512, 1024, 2048, 4096):
        for P in (1, 2, 4, 8):
            if 64 * P > W // 2:
                continue
            sw.set_tuning(W, P, sw.MODE_STAGE)
            plan = sw.plan(n, nsteps, "heat", torch.float64)
            times, _ = timed_runs(sw, torch, sw.advance, u0, nsteps, [0.25], 2, 1)
            t = min(times)
            ops = heat_ops(sw)
            print(json.dumps({"tile_w": W, "pairs_per_lane": P, "stages": plan["stages"],
                              "ms": t * 1e3, "value": n * nsteps / t, "ops_per_update": ops,
                              "frac_alu": ops * n * nsteps / t / VALU_LANE_OPS}),
                  flush=True)
    sw.set_tuning(0, 0, sw.MODE_AUTO)


def size_sweep(sw, torch, workloads):
    """Swept against naive as the grid grows (the paper's speedup against
    points per node): heat f64 at N = 2^12 ... 2^24 over 10,000 steps and KS
    at N = 2^12 ... 2^20 over 2,000 steps, each after the autotuner, median
    of three runs.  One JSON line per size."""
    def timed(fn, u0, nsteps, st, par):
        u = u0.clone()
        fn(u, nsteps, st, par)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            u.copy_(u0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn(u, nsteps, st, par)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        return sorted(ts)[1]
    cases = [("heat", lg, 10_000, [0.25]) for lg in range(12, 25, 2)] + \
            [("ks", lg, 2_000, [workloads.KS_DT, workloads.KS_DX]) for lg in range(12, 21, 2)]
    for st, lg, nsteps, par in cases:
        n = 1 << lg
        u0 = torch.from_numpy(workloads.white_noise(n, seed=lg) if st == "heat" else
                              workloads.smoothed_noise(n, seed=lg)).cuda()
        sw.clear_tuning()
        tuned = sw.autotune(n, nsteps, st, par)
        plan = sw.plan(n, nsteps, st)
        ts = timed(sw.advance, u0, nsteps, st, par)
        tn = timed(sw.naive_advance, u0, nsteps, st, par)
        print(json.dumps({"stencil": st, "n": n, "time_steps": nsteps, "tile_w": plan["tile_w"],
                          "pairs_per_lane": plan["pairs_per_lane"], "mode": plan["mode"],
                          "swept": n * nsteps / ts, "naive": n * nsteps / tn,
                          "speedup_vs_naive": tn / ts, "naive_us_per_step": tn / nsteps * 1e6,
                          "tune_probe_rate": tuned["probe_rate"]}), flush=True)
    sw.clear_tuning()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads
    import paper_1504_01380_amd as sw

    sw.init(0)
    sw.set_tuning(0, 0, sw.MODE_AUTO)
    sw.clear_tuning()
    if args.profile_mix:
        profile_mix(sw, torch, workloads)
        return
    if args.sweep:
        tile_sweep(sw, torch, workloads, args)
        return
    if args.size_sweep:
        size_sweep(sw, torch, workloads)
        return
    n, nsteps = args.n, args.nsteps
    u0_np = workloads.white_noise(n, seed=workloads.WORKLOADS["heat_large"]["seed"])
    u0 = torch.from_numpy(u0_np).cuda()
    tuning = None
    if not args.no_tune:
        # warm-up: the autotuner (Eq. (1) prior + timed probes) picks the tiling
        t0 = time.perf_counter()
        tuning = sw.autotune(n, nsteps, "heat", [0.25], torch.float64)
        tuning["tune_s"] = time.perf_counter() - t0
    plan = sw.plan(n, nsteps, "heat", torch.float64)
    progress("tuned: %s" % (plan,))

    if args.profile:
        # a plain device copy of known size, for scaling the HBM counters
        dst = torch.empty_like(u0)
        dst.copy_(u0)
        torch.cuda.synchronize()

    # The stage launches of every timed run are bracketed by HIP events on
    # the library's stream (torch's current stream).
    sw.set_profiling(True)
    k = plan["depth_k"]
    # the full diamonds strictly below the target level (the continuous
    # kernel's stages; a diamond whose apex is the target level is banded)
    full = [s for s in range(1, plan["stages"]) if (s - 1) * k + 2 * k - 1 < nsteps]
    diamond_ms, stage_ms, kinds = [], [], set()

    def record():
        ms, kind = sw.stage_times()
        stage_ms.append(sum(ms))
        diamond_ms.extend(ms[s] for s in full)
        kinds.update(kind[s] for s in full)

    times, u_swept = timed_runs(sw, torch, sw.advance, u0, nsteps, [0.25], args.steps,
                                args.warmup, after=record)
    sw.set_profiling(False)
    ops = heat_ops(sw)     # the form the timed runs took (both give the same bits)
    progress("heat f64 swept runs done (%d VALU instructions per update)" % ops)
    t = sum(times) / len(times)
    updates = float(n) * nsteps
    value = updates / t

    # Dominant kernel: the one that runs the full diamond stages (the
    # continuous-band kernel when k is a multiple of its band), one launch per
    # stage; each launch computes 2k^2 point-updates per tile.
    tiles = plan["tiles"]
    kname = ("swept_diamond_cont_kernel<Heat<double>,%d>" if kinds == {1} else
             "swept_stage_kernel<Heat<double>,%d>") % plan["pairs_per_lane"]
    updates_per_launch = float(tiles) * 2 * k * k
    flops_per_launch = ops * updates_per_launch
    avg_launch = (sum(diamond_ms) / len(diamond_ms) / 1e3) if diamond_ms else float("nan")
    achieved = flops_per_launch / avg_launch
    edge_bytes = float(tiles) * 4 * 2 * k * 8   # RE in/out + LE in/out, 2k values each
    # LDS per region and stage of the continuous kernel: the right V edge
    # in (2k points), the new left edge out (2k), and per wave step (nb*k + NB
    # of them, NB = 64P) slot 0's read of pair -1 and the last slot's write
    # of its pair (4 points)
    NB = 64 * plan["pairs_per_lane"]
    lds_bytes = float(tiles) * 8 * (4 * k + 4 * ((k // max(NB, 1)) * k + NB))
    lds = {"achieved_GBps": lds_bytes / avg_launch / 1e9, "peak_GBps": LDS_PEAK / 1e9,
           "frac": lds_bytes / avg_launch / LDS_PEAK, "bytes_per_launch": lds_bytes,
           "kernel": kname}
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_LANE_OPS / 1e12,
                "unit": "TFLOP/s", "frac": achieved / VALU_LANE_OPS,
                "traffic": measured_traffic(kname),
                "kernel": kname, "launches_per_step": len(diamond_ms) // max(1, args.steps),
                "stages_per_step": plan["stages"], "avg_launch_ms": avg_launch * 1e3,
                "flops_per_launch": flops_per_launch, "ops_per_update": ops,
                "heat_form": "fused Laplacian" if ops == HEAT_FUSED_LAP_OPS else "canonical",
                "counting": "FP64 VALU instructions issued per update (a fused multiply-add "
                            "issues once)",
                "stage_sum_ms": sum(stage_ms) / max(1, len(stage_ms)),
                "algorithmic_bytes_per_launch": edge_bytes,
                "whole_run_frac": ops * value / VALU_LANE_OPS}

    out = {
        "metric": "point-updates/sec swept vs naive per-step (1 MI355X), % of VALU/HBM peak",
        "value": value, "unit": "point-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "heat N=2^24 f64 r=0.25 20000 steps, u0~U[-1,1] seed 1001",
                   "n": n, "time_steps": nsteps, "tile_w": plan["tile_w"],
                   "depth_k": plan["depth_k"], "tiles": plan["tiles"], "stages": plan["stages"],
                   "pairs_per_lane": plan["pairs_per_lane"], "tuning": tuning},
        "roofline": roofline,
        "lds": lds,
    }

    if args.profile:
        # a few naive steps, for the naive kernel's HBM counters
        u = u0.clone()
        sw.naive_advance(u, 50, "heat", [0.25])
        torch.cuda.synchronize()
        args.no_naive = args.no_cpu = True
    if not args.no_naive:
        nt, _ = timed_runs(sw, torch, sw.naive_advance, u0, nsteps, [0.25], 1, 1)
        naive = updates / nt[0]
        out["naive"] = {"value": naive, "ms": nt[0] * 1e3,
                        "hbm_GBps": naive * HEAT_NAIVE_BYTES[8] / 1e9,
                        "hbm_frac": naive * HEAT_NAIVE_BYTES[8] / HBM_PEAK}
        out["speedup_vs_naive"] = value / naive
        progress("heat f64 naive done")
        # the same swept runs evaluating the five operations as written
        sw.set_heat_form(sw.FORM_CANONICAL)
        ct, uc = timed_runs(sw, torch, sw.advance, u0, nsteps, [0.25], 2, 1)
        sw.set_heat_form(sw.FORM_AUTO)
        canon = updates / (sum(ct) / len(ct))
        out["canonical_form"] = {
            "swept": canon, "ms": sum(ct) / len(ct) * 1e3, "ops_per_update": HEAT_OPS_PER_UPDATE,
            "swept_frac_alu": HEAT_OPS_PER_UPDATE * canon / VALU_LANE_OPS,
            "speedup_vs_naive": canon / naive,
            "bits_equal_default": bool(torch.equal(uc.view(torch.int64),
                                                   u_swept.view(torch.int64)))}
        progress("heat f64 canonical form done")
        u32 = u0.float()
        tune32 = None if args.no_tune else sw.autotune(n, nsteps, "heat", [0.25], torch.float32)
        plan32 = sw.plan(n, nsteps, "heat", torch.float32)
        st, _ = timed_runs(sw, torch, sw.advance, u32, nsteps, [0.25], 2, 1)
        ops32 = heat_ops(sw)
        nt32, _ = timed_runs(sw, torch, sw.naive_advance, u32, nsteps, [0.25], 1, 1)
        s32 = updates / (sum(st) / len(st))
        n32 = updates / nt32[0]
        out["f32"] = {"swept": s32, "naive": n32, "speedup_vs_naive": s32 / n32,
                      "ops_per_update": ops32,
                      "swept_frac_alu": ops32 * s32 / VALU_LANE_OPS_F32,
                      "naive_hbm_frac": n32 * HEAT_NAIVE_BYTES[4] / HBM_PEAK,
                      "tile_w": plan32["tile_w"], "pairs_per_lane": plan32["pairs_per_lane"],
                      "tuning": tune32}

    if not args.no_naive:
        progress("heat f32 done")
        out["fma"] = fma_legs(sw, torch, workloads, u0, u_swept, nsteps, updates,
                              tune=not args.no_tune)
        progress("contraction-on legs done")
        out["workloads"] = other_workloads(sw, torch, workloads, tune=not args.no_tune)
        out["workloads"]["batch"] = batch_workload(sw, torch, workloads, tune=not args.no_tune)
        progress("batch done")
        out["workloads"]["ks_adjoint"] = ks_adjoint_workload(sw, torch, workloads)
        progress("ks adjoint done")

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(u0_np, nsteps, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
