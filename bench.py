"""Benchmark of the FP32 shallow-water step on one MI355X.

Main line (``value``): cell-RK3-updates/s on the single large synthetic
coastline: 4096 x 4096 cells, dx = 5 m, linear beach + 32 seeded bumps + a
2 m plane hump, Manning n = 0.025, h_dry = 1e-3, CFL 0.4.  Inputs are
resident in HBM before timing.  One bench "step" is one full TVD-RK3 step
(three stage kernels: halo staging, WENO5/LF faces in x and y, sources, RK
combination, wave-speed and runup reductions, device-side dt) over the grid.

Extra objects on the same JSON line:
  roofline      stage kernel: algorithmic flops (and bytes) per launch over
                its mean device duration, HIP events on the kernels' stream;
  cpu_baseline  the FP64 reference checker on a bounded sample;
  small_grid    the 128 x 64 dam break: ms per step with graph replays;
  outputs       the same grid with six snapshots at output times streamed to
                the host and the maximum-depth map kept: cost per step and
                how long after the run the last snapshot is on the host;
  batched       the mitigation ensemble (64 x 1024^2, dx 2 m, 3000 steps,
                Carrier's N-wave on a beach with seeded hills and Manning
                patches) in one batch: scenarios/hour batched vs the plain
                single-scenario solver, per-member runup;
  uneven        200 scenarios of {256^2, 512x1024, 1024^2, 2048x1024} cells
                and U{1000..4000} steps in one batch: scenarios/hour against
                the plain solver one scenario at a time;
  serving       Poisson arrivals of 500 requests with the uneven batch's size
                and step mix at 0.7x and 1.0x of its measured batched
                capacity, under a device-memory budget: p50/p99
                time-to-result, scenarios/hour, memory high-water mark;
  valu_calibration  the vector-ALU issue ceiling for unpacked FP32 code,
                measured on the same GPU (the stage kernel's roofline).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The server overlaps its segments (compute stream) with request uploads and
# result read-backs on two more streams.  HIP maps a process's streams onto
# at most GPU_MAX_HW_QUEUES hardware queues (4 by default); after the earlier
# lines' contexts and batches, the server's streams shared queues and its
# uploads serialized with the segments (serving p50 at 0.7x load 1.44 s
# against 0.90 s with 8 queues, same run otherwise).  Raised (never lowered)
# before HIP starts.
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _hwq = 4
if _hwq < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

METRIC = "cell-RK3-updates/s FP32 (1 GPU); scenarios/hour + p50/p99 latency batched"
UNIT = "cell-RK3-updates/s"
# Algorithmic HBM bytes per cell per stage launch (FP32): stage 1 reads
# u^n (3 planes) + b + g n^2 and writes u^(1) (3); stages 2 and 3 also read
# u^n (3) for the RK combination: 32, 44, 44 bytes.
BYTES_STAGE = (32.0, 44.0, 44.0)
# Algorithmic flops per cell per stage: 2.8e3 per cell-RK3-update (twelve
# WENO5 reconstructions of ~65 flops per cell and stage, four bed-face
# reuses, fluxes, splits, divergence, sources and the RK combination), a
# third of it per stage launch.  A count on the definition (each add, mul,
# div, sqrt, pow once) gives 1050 per stage, FLOPS_STAGE_DEF; the roofline
# uses the smaller figure.
FLOPS_STAGE = 2.8e3 / 3.0
FLOPS_STAGE_DEF = 2 * 25 + 2 * (6 * 70 + 3 + 48 + 10) + 16 + 15 + 7
HBM_PEAK = 8.0e12        # B/s
# FP32 vector peak as published: 256 CU x 2.4 GHz x 128 FMA lanes per CU
# and clock x 2 flops; the 128 lanes count packed FP32 (two FMAs per lane in
# one v_pk_fma_f32).  All device code here is built with packed FP32
# disabled, so the ceiling for the code that runs is half of it: 64 FMA lanes
# per CU and clock, one wave64 VALU instruction per CU and clock, 78.6
# TFLOP/s (the valu_calibration object measures it live; transcendental
# instructions such as v_rcp_f32 take two issue cycles).
FP32_PEAK = 157.3e12
FP32_UNPACKED_PEAK = 256 * 2.4e9 * 64 * 2


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def valu_calibration(iters=4096):
    """Vector-ALU issue ceiling of the GPU for the code this library builds
    (libswe_calib.so): wave64 VALU instructions per CU and clock, at the
    nominal 2.4 GHz, of 16 independent chains per thread of two FMAs
    ("fma"), one v_rcp_f32 and one FMA ("rcp_fma") and one v_rcp_f32 and
    seven FMAs ("rcp_7fma"), at 1, 2, 4 and 8 waves per SIMD."""
    import ctypes
    path = os.path.join(ROOT, "paper_2301_12010_amd", "libswe_calib.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    lib.swe_calib_valu.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)]
    lib.swe_calib_valu.restype = ctypes.c_int
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"clock_ghz_assumed": 2.4, "cus": cus}
    for op, name in enumerate(("fma", "rcp_fma", "rcp_7fma")):
        rates = {}
        for w in (1, 2, 4, 8):
            ms, wi = ctypes.c_float(), ctypes.c_double()
            rc = lib.swe_calib_valu(op, w, iters, ctypes.byref(ms), ctypes.byref(wi))
            if rc != 0:
                raise RuntimeError(f"swe_calib_valu({op}, {w}) failed: {rc}")
            rates[str(w)] = wi.value / (cus * ms.value * 1e-3 * 2.4e9)
        out[name] = rates
    # issue cycles of one v_rcp_f32 in units of one FMA's, from the 8-wave rates
    f, r1 = out["fma"]["8"], out["rcp_fma"]["8"]
    out["rcp_issue_cycles_per_fma"] = (2.0 / r1 - 1.0 / f) * f
    log(f"VALU calibration: fma {f:.3f}, rcp+fma {r1:.3f} wave64 instr per CU per clock at 8 waves/SIMD")
    return out


def kernel_source_digest(text=None):
    """Digest of the stage kernel's code (its body and launch wrapper) with
    comments and whitespace removed: counters taken on the kernel stay
    attributed to it until its code changes."""
    if text is None:
        with open(os.path.join(ROOT, "paper_2301_12010_amd", "csrc", "swe_stage.hpp")) as fh:
            text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return hashlib.sha256("".join(text.split()).encode()).hexdigest()[:16]


def measured_traffic(workload, tile):
    """HBM bytes per stage launch from committed rocprofv3 counter runs, if
    they were taken on the current kernel source with the same tile shape."""
    p = os.path.join(ROOT, "profiles", "stage_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if (d.get("kernel_digest") != kernel_source_digest() or d.get("workload") != workload
            or list(d.get("tile", [])) != list(tile)):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(sc, budget_s=15.0):
    import oracle
    o = oracle.Oracle.from_scenario(sc)
    t0 = time.perf_counter()
    steps = 0
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 50 or el * (steps + 1) / steps > 2 * budget_s:
            break
    rate = sc.cells * steps / el
    o.close()
    out = {"value": rate, "unit": UNIT, "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"FP64 checker, {sc.params.nx}x{sc.params.ny} large coastline, first {steps} "
                     f"RK3 step(s) from the same initial state ({el:.1f} s)",
           "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    one = _cpu_one_thread(sc)
    if one is not None:
        out["one_thread"] = one
    out["per_config"] = _cpu_per_config()
    return out


def _cpu_per_config():
    """The checker (all threads) on the other workloads' truncated samples:
    the dam break in full, three ensemble members for 50 steps, one uneven
    member per size class for 20 steps."""
    import oracle
    from paper_2301_12010_amd import inputs

    def rate(scens, steps):
        cells, t = 0, 0.0
        for sc in scens:
            o = oracle.Oracle.from_scenario(sc)
            t0 = time.perf_counter()
            o.step(steps)
            t += time.perf_counter() - t0
            o.close()
            cells += sc.cells * steps
        return {"value": cells / t, "unit": UNIT, "seconds": t}

    plan = inputs.uneven_plan()
    picks = [next(i for i, (sz, _) in enumerate(plan) if sz == size) for size in inputs.UNEVEN_SIZES]
    return {
        "dam_break_128x64_200_steps": rate([inputs.dam_break()], 200),
        "ensemble_3_members_1024x1024_50_steps":
            rate([inputs.mitigation_coast(1024, 1024, 2.0, seed=1000 + k) for k in range(3)], 50),
        "uneven_one_per_size_20_steps": rate([inputs.uneven_scenario(i, plan) for i in picks], 20),
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _cpu_one_thread(sc):
    """The checker on one thread: its first step of the same grid, in a child
    process (the OpenMP thread count is fixed when the runtime starts)."""
    import subprocess
    code = ("import sys, time, json; sys.path.insert(0, %r); import oracle; "
            "from paper_2301_12010_amd import inputs; "
            "sc = inputs.large_coast(%d, %d, %r, seed=2); o = oracle.Oracle.from_scenario(sc); "
            "t = time.perf_counter(); o.step(1); el = time.perf_counter() - t; "
            "print(json.dumps({'value': sc.cells / el, 'seconds': el, 'threads': oracle.num_threads()}))"
            % (ROOT, sc.params.nx, sc.params.ny, sc.params.dx))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        res = json.loads(r.stdout.strip().splitlines()[-1])
        res.update({"unit": UNIT, "sample": "FP64 checker, first RK3 step of the same grid, one thread"})
        return res
    except Exception as exc:  # the baseline is a report; its absence is stated
        log(f"one-thread baseline skipped: {exc}")
        return None


def run_large(args, torch, inputs, swe):
    t_gen = time.perf_counter()
    sc = inputs.large_coast(args.nx, args.ny, 5.0 * 4096 / args.nx, seed=2, nsteps=2000)
    log(f"generated {sc.name} in {time.perf_counter() - t_gen:.1f}s")
    tile = args.tile
    if tile < 0:
        tile, _ = swe.autotune(sc.params.nx, sc.params.ny)
        log(f"autotuned tile variant {tile}")
    stream = torch.cuda.Stream()  # default priority; the solver's kernels run here
    s = swe.Solver.from_scenario(sc, stream=stream)
    s.set_option(swe.OPT_TILE, tile)
    s.set_option(swe.OPT_GRAPH_STEPS, args.graph_steps)
    s.set_option(swe.OPT_COMPENSATED, int(args.compensated))
    s.set_option(swe.OPT_FRICTION_IMPLICIT, int(args.friction_implicit))
    s.set_option(swe.OPT_LOCAL_SPLIT, int(args.local_split))
    s.step(args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    s.step(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    st = s.stats()
    if st["rc"] != 0:
        raise RuntimeError(f"solver state non-finite after timing: {st}")
    value = sc.cells * args.steps / (ms * 1e-3)
    log(f"timed {args.steps} steps: {ms:.1f} ms, t={st['t']:.2f}s, {value:.3e} {UNIT}")

    # stage-kernel durations with HIP events around each launch (plain launches)
    kms = s.time_stages(20)
    avg_ms = sum(kms) / 3.0
    n = sc.cells
    # the compensated level reads and writes its residual planes too
    bytes_cell = (sum(BYTES_STAGE) + (8 + 12 + 12 if args.compensated else 0)) / 3.0
    bytes_launch = n * bytes_cell
    flops_launch = n * FLOPS_STAGE
    ach_bw = bytes_launch / (avg_ms * 1e-3)
    ach_fl = flops_launch / (avg_ms * 1e-3)
    tv = swe.tile_variants()[tile]
    # counters were taken for the default kernels only
    plain = not (args.compensated or args.friction_implicit or args.local_split)
    traffic = measured_traffic(sc.name, (tv["tx"], tv["ty"], tv["r"])) if plain else None
    roof_alu = {"bound": "alu", "achieved": ach_fl / 1e12, "peak": FP32_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": ach_fl / FP32_PEAK, "traffic": traffic,
                "kernel": "k_stage (3 stage launches per step)", "kernel_ms": kms,
                "flops_per_cell_launch": FLOPS_STAGE,
                "frac_with_definition_count": n * FLOPS_STAGE_DEF / (avg_ms * 1e-3) / FP32_PEAK,
                "peak_unpacked": FP32_UNPACKED_PEAK / 1e12, "frac_unpacked": ach_fl / FP32_UNPACKED_PEAK}
    roof_hbm = {"bound": "hbm", "achieved": ach_bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": ach_bw / HBM_PEAK, "traffic": traffic,
                "bytes_per_cell_launch": bytes_cell}
    roofline = roof_alu if roof_alu["frac"] >= roof_hbm["frac"] else roof_hbm
    other = roof_hbm if roofline is roof_alu else roof_alu
    outputs = None if args.no_outputs else measure_outputs(s, torch, stream, sc)
    s.close()
    e2e = None if args.no_end_to_end else measure_end_to_end(swe, stream, sc, tile, args)
    return sc, value, ms, roofline, other, tv, outputs, e2e


def measure_end_to_end(swe, stream, sc, tile, args):
    """The same job from host arrays to host arrays: swe_create from the host
    fields (validation, ghosts, upload over PCIe), the timed steps, and
    swe_read of h, hu, hv into host memory.  Reported beside `value`, never
    as it: `value` starts with the state resident in HBM."""
    import time as _t
    t0 = _t.perf_counter()
    s = swe.Solver.from_scenario(sc, stream=stream)
    s.set_option(swe.OPT_TILE, tile)
    s.set_option(swe.OPT_GRAPH_STEPS, args.graph_steps)
    s.stats()  # upload complete
    t1 = _t.perf_counter()
    s.step(args.steps)
    s.stats()
    t2 = _t.perf_counter()
    h, hu, hv, st = s.read()
    t3 = _t.perf_counter()
    s.close()
    if st["status"] != 0:
        raise RuntimeError(f"end-to-end run non-finite: {st}")
    rate = sc.cells * args.steps / (t3 - t0)
    log(f"end to end: create {t1 - t0:.3f}s, steps {t2 - t1:.3f}s, read {t3 - t2:.3f}s -> {rate:.3e}")
    return {"value": rate, "unit": UNIT, "create_s": t1 - t0, "steps_s": t2 - t1, "read_s": t3 - t2,
            "steps": args.steps,
            "note": "host fields -> swe_create -> steps -> swe_read to host; host clock"}


def measure_small_grid(torch, inputs, swe, steps=200, reps=5):
    """The 128 x 64 dam break (Section 2.1): ms per step with the autotuned
    tile, graph replays of all its steps, median of reps runs after one
    untimed run."""
    sc = inputs.dam_break()
    tile, _ = swe.autotune(sc.params.nx, sc.params.ny)
    stream = torch.cuda.Stream()
    times = []
    for r in range(reps + 1):
        s = swe.Solver.from_scenario(sc, stream=stream)
        s.set_option(swe.OPT_TILE, tile)
        s.set_option(swe.OPT_GRAPH_STEPS, steps)
        s.step(steps)  # builds and runs the graph once
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s.step(steps)
        b.record(stream)
        b.synchronize()
        if r:
            times.append(a.elapsed_time(b) / steps)
        s.close()
    times.sort()
    ms = times[len(times) // 2]
    tv = swe.tile_variants()[tile]
    res = {"workload": f"dam_break {sc.params.nx}x{sc.params.ny}", "steps": steps,
           "tile": [tv["tx"], tv["ty"], tv["r"]], "ms_per_step": ms,
           "cell_updates_per_s": sc.cells / (ms * 1e-3)}
    log(f"small grid: {res}")
    return res


def measure_outputs(s, torch, stream, sc, steps=300, chunk=25, n_out=6):
    """Snapshots at output times plus the maximum-depth map during a run.

    The host drives the run in chunks of `chunk` steps and keeps at most two
    chunks ahead of the GPU, polling the outputs between chunks, as a caller
    streaming results would.  The same loop without outputs is the
    reference.  Reports the per-step cost of the outputs and how long after
    the last step the last snapshot reaches the host.
    """
    import time as _t

    def run(with_outputs):
        if with_outputs:
            st = s.stats()
            # about every steps / n_out steps, between step ends
            times = [st["t"] + (j * steps / n_out - 0.5) * st["dt"] for j in range(1, n_out + 1)]
            s.set_outputs(times)
            s.track_max_depth(True)
        torch.cuda.synchronize()
        evs = []
        ready = [False] * (n_out if with_outputs else 0)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for i in range(steps // chunk):
            s.step(chunk)
            e = torch.cuda.Event()
            e.record(stream)
            evs.append(e)
            if i >= 2:
                evs[i - 2].synchronize()
            for k in range(len(ready)):
                ready[k] = ready[k] or s.output_ready(k)
        stop.record(stream)
        stop.synchronize()
        t_end = _t.perf_counter()
        ms = start.elapsed_time(stop)
        on_host_early = sum(ready)
        for k in range(len(ready)):
            ready[k] = ready[k] or s.output_ready(k, wait=True)
        drain_ms = (_t.perf_counter() - t_end) * 1e3
        if with_outputs:
            for k in range(n_out):  # hand-out into caller arrays (not timed)
                assert s.output(k) is not None
            s.max_depth()
            s.set_outputs([])
            s.track_max_depth(False)
        return ms / steps, sum(ready), on_host_early, drain_ms

    base, _, _, _ = run(False)
    with_o, taken, early, drain = run(True)
    res = {"steps": steps, "chunk_steps": chunk, "snapshots": taken,
           "snapshots_on_host_before_run_end": early, "snapshot_mb": 12 * sc.cells / 1e6,
           "max_depth_map": True, "ms_per_step": with_o, "ms_per_step_without": base,
           "overhead": with_o / base - 1.0, "last_snapshot_ms_after_run_end": drain}
    log(f"outputs: {res}")
    return res


def run_batched(args, torch, inputs, swe):
    """Mitigation ensemble: scenarios/hour batched vs the plain solver."""
    t0 = time.perf_counter()
    members = inputs.mitigation_ensemble(args.ens_count, 1024, 1024, args.ens_steps)
    log(f"generated {len(members)} ensemble members in {time.perf_counter() - t0:.1f}s")
    cells = 1024 * 1024
    out = {"workload": f"mitigation_ensemble_{len(members)}x1024x1024_dx2", "scenarios": len(members),
           "steps_per_scenario": args.ens_steps}
    known = {"rounds_graph": (swe.BATCH_ROUNDS, True), "rounds": (swe.BATCH_ROUNDS, False),
             "persistent": (swe.BATCH_PERSISTENT, False)}
    modes = [(m,) + known[m] for m in args.ens_modes]
    for name, mode, graph in modes:
        bt = swe.Batch()
        bt.set_mode(mode, graph)
        for sc in members:
            bt.add_scenario(sc)
        steps = args.ens_steps if name == "rounds_graph" else min(args.ens_steps, args.ens_other_steps)
        torch.cuda.synchronize()
        t = time.perf_counter()
        bt.run(steps)
        st0 = bt.stats(0)
        dt = time.perf_counter() - t
        rate = len(members) * cells * steps / dt
        out[name] = {"steps": steps, "seconds": dt, "cell_updates_per_s": rate}
        if name == "rounds_graph":
            runups = [bt.stats(i)["runup"] for i in range(len(members))]
            assert all(bt.stats(i)["rc"] == 0 for i in range(len(members)))
            out["scenarios_per_hour"] = len(members) / dt * 3600.0
            out["runup_m"] = {"min": min(runups), "median": sorted(runups)[len(runups) // 2],
                              "max": max(runups)}
        log(f"batched {name}: {steps} steps in {dt:.2f}s, {rate:.3e} cell-updates/s")
        bt.close()
    if "scenarios_per_hour" not in out:
        return out, members
    # plain single-scenario solver, one scenario at a time (same inputs, same steps)
    k = min(2, len(members))
    t = time.perf_counter()
    for sc in members[:k]:
        s = swe.Solver.from_scenario(sc)
        s.step(args.ens_steps)
        s.stats()
        s.close()
    dt = (time.perf_counter() - t) / k
    out["plain_solver_scenarios_per_hour"] = 3600.0 / dt
    out["plain_solver_cell_updates_per_s"] = cells * args.ens_steps / dt
    out["batched_over_plain"] = out["scenarios_per_hour"] / out["plain_solver_scenarios_per_hour"]
    log(f"plain solver {dt:.2f}s per scenario")
    return out, members


def run_serving(swe, scens, steps, rate, budget_bytes, max_slots, seed=5, label=""):
    """Poisson arrivals at `rate` requests/s; request i is scenario
    scens[i % len(scens)] run for steps[i] steps.  Returns time-to-result
    percentiles, scenarios/hour and the memory high-water mark."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(steps)
    gaps = rng.exponential(1.0 / rate, size=n)
    sv = swe.Server(mem_budget=budget_bytes, max_slots=max_slots, segment_steps=100)
    sv.set_mode(swe.BATCH_ROUNDS)
    t_start = time.perf_counter()
    t_next = t_start
    pending, results = {}, []
    t_log = t_start

    def drain():
        for tk in list(pending):
            r, _ = sv.poll(tk, want_state=False)
            if r["status"] != swe.PENDING:
                results.append(r)
                del pending[tk]

    for i in range(n):
        t_next += gaps[i]
        while time.perf_counter() < t_next:
            drain()
            time.sleep(0.001)
        sc = scens[i % len(scens)]
        pending[sv.submit_scenario(sc, int(steps[i]))] = i
        if time.perf_counter() - t_log > 20.0:
            t_log = time.perf_counter()
            log(f"serving {label}: {i + 1}/{n} submitted, {len(results)} done")
    while pending:
        drain()
        time.sleep(0.002)
    st = sv.stats()
    sv.close()
    ok = [r for r in results if r["status"] == swe.DONE]
    ttr = np.array([r["t_done"] - r["t_submit"] for r in ok])
    wait = np.array([r["t_admit"] - r["t_submit"] for r in ok])
    span = max(r["t_done"] for r in ok) - min(r["t_submit"] for r in ok)
    return {"requests": n, "completed": len(ok), "arrival_rate_per_s": rate,
            "steps_per_request": [int(min(steps)), int(max(steps))],
            "p50_time_to_result_s": float(np.percentile(ttr, 50)),
            "p99_time_to_result_s": float(np.percentile(ttr, 99)),
            "p50_admission_wait_s": float(np.percentile(wait, 50)),
            "p99_admission_wait_s": float(np.percentile(wait, 99)),
            "scenarios_per_hour": len(ok) / span * 3600.0,
            "mem_budget_bytes": st["mem_budget"], "mem_high_water_bytes": st["mem_high_water"],
            "budget_binds": bool(st["mem_high_water"] >= 0.9 * st["mem_budget"]),
            "max_slots": max_slots, "segments": st["segments"]}


def run_serving_mix(args, swe, scens, plan, capacity_per_s):
    """Serving with the uneven batch's size and step mix: Poisson arrivals
    at each of args.serve_loads times the measured batched capacity."""
    n = args.serve_requests
    steps = [plan[i % len(plan)][1] for i in range(n)]
    out = {"workload": f"poisson_requests_uneven_mix_{n}", "capacity_scenarios_per_s": capacity_per_s,
           "mix": "sizes and steps of the uneven batch, request i = scenario i mod %d" % len(plan)}
    for frac in args.serve_loads:
        res = run_serving(swe, scens, steps, frac * capacity_per_s, args.serve_budget_gb << 30,
                          args.serve_slots, label=f"{frac}x")
        res["load_fraction"] = frac
        out[f"load_{frac}"] = res
        log(f"serving at {frac}x capacity: p50 {res['p50_time_to_result_s']:.2f}s "
            f"p99 {res['p99_time_to_result_s']:.2f}s, {res['scenarios_per_hour']:.0f} scenarios/hour, "
            f"high water {res['mem_high_water_bytes'] / 1e9:.2f} GB")
    return out


def run_uneven(args, torch, inputs, swe):
    """Uneven batch: 200 scenarios of four grid sizes and U{1000..4000} steps,
    the autotuner run per size class (the batch launches the tile tuned for
    its largest class; the plain solver uses each class's); per-round
    launches and the persistent kernel, each captured as a graph, against
    the plain solver."""
    plan = inputs.uneven_plan(args.uneven_count)
    t0 = time.perf_counter()
    scens, by_size, cells_steps = [], {}, 0
    for s_idx, ((nx, ny), steps) in enumerate(plan):
        scens.append(inputs.uneven_scenario(s_idx, plan))
        cells_steps += nx * ny * steps
        by_size.setdefault((nx, ny), []).append((s_idx, steps))
        if s_idx % 20 == 0:
            log(f"uneven: generated {s_idx + 1}/{len(plan)}")
    tiles = {}
    for (nx, ny) in by_size:
        tiles[f"{nx}x{ny}"] = swe.autotune(nx, ny)[0]
    log(f"uneven: {len(plan)} scenarios ready in {time.perf_counter() - t0:.1f}s, tuned tiles {tiles}")
    out = {"workload": f"uneven_batch_{len(plan)}", "scenarios": len(plan), "cell_updates": cells_steps,
           "tile_forced": args.uneven_tile, "compensated": bool(args.uneven_compensated),
           "local_split": bool(args.uneven_local_split),
           "sizes": {f"{nx}x{ny}": len(v) for (nx, ny), v in by_size.items()},
           "tuned_tile_variants": tiles}
    modes = [("rounds_graph", swe.BATCH_ROUNDS)]
    if args.uneven_persistent:
        modes.append(("persistent_graph", swe.BATCH_PERSISTENT))
    for name, mode in modes:
        bt = swe.Batch()
        bt.set_mode(mode, True)
        if args.uneven_tile >= 0:
            bt.set_tile(args.uneven_tile)
        if args.uneven_compensated:
            bt.set_option(swe.OPT_COMPENSATED, 1)
        if args.uneven_local_split:
            bt.set_option(swe.OPT_LOCAL_SPLIT, 1)
        for sc in scens:
            bt.add_scenario(sc)
        torch.cuda.synchronize()
        t = time.perf_counter()
        bt.run()
        for i in range(len(plan)):
            st = bt.stats(i)
            assert st["rc"] == 0 and st["step"] == plan[i][1], (i, st)
        dt = time.perf_counter() - t
        bt.close()
        out[name] = {"seconds": dt, "cell_updates_per_s": cells_steps / dt,
                     "scenarios_per_hour": len(plan) / dt * 3600.0}
        log(f"uneven {name}: {dt:.1f}s, {cells_steps / dt:.3e} cell-updates/s")
    best = max([m for m, _ in modes], key=lambda k: out[k]["scenarios_per_hour"])
    out["mode"] = best
    out["seconds"] = out[best]["seconds"]
    out["cell_updates_per_s"] = out[best]["cell_updates_per_s"]
    out["scenarios_per_hour"] = out[best]["scenarios_per_hour"]
    # plain solver, one scenario at a time with its size's tuned tile and the
    # batch's options: the first member of each size class, the class's
    # per-cell-update rate applied to all of its members
    plain_s = 0.0
    for (nx, ny), members in by_size.items():
        rates = []
        for s_idx, steps in members[:1]:
            sol = swe.Solver.from_scenario(scens[s_idx])
            sol.set_option(swe.OPT_COMPENSATED, int(args.uneven_compensated))
            sol.set_option(swe.OPT_LOCAL_SPLIT, int(args.uneven_local_split))
            sol.stats()
            t = time.perf_counter()
            sol.step(steps)
            sol.stats()
            rates.append(nx * ny * steps / (time.perf_counter() - t))
            sol.close()
        rate = sum(rates) / len(rates)
        plain_s += sum(nx * ny * st / rate for _, st in members)
        out.setdefault("plain_rate_by_size", {})[f"{nx}x{ny}"] = rate
    out["plain_solver_seconds_est"] = plain_s
    out["plain_solver_scenarios_per_hour"] = len(plan) / plain_s * 3600.0
    out["batched_over_plain"] = out["scenarios_per_hour"] / out["plain_solver_scenarios_per_hour"]
    return out, scens, plan


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nx", type=int, default=4096)
    ap.add_argument("--ny", type=int, default=4096)
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--graph-steps", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-batched", action="store_true", help="skip the ensemble run")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven batch (and the serving run)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--uneven-persistent", action="store_true",
                    help="also run the uneven batch with the persistent kernel")
    ap.add_argument("--no-outputs", action="store_true", help="skip the snapshot/max-depth measurement")
    ap.add_argument("--no-end-to-end", action="store_true",
                    help="skip the host-to-host run (create from host fields, steps, read to host)")
    ap.add_argument("--no-small-grid", action="store_true", help="skip the 128 x 64 latency measurement")
    ap.add_argument("--ens-count", type=int, default=64)
    ap.add_argument("--ens-steps", type=int, default=3000)
    ap.add_argument("--ens-modes", nargs="+", default=["rounds_graph", "persistent"],
                    choices=["rounds_graph", "rounds", "persistent"],
                    help="launch modes of the ensemble run (rounds_graph gives scenarios/hour)")
    ap.add_argument("--ens-other-steps", type=int, default=300,
                    help="steps of the ensemble run in modes other than rounds_graph")
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--serve-budget-gb", type=int, default=2)
    ap.add_argument("--serve-slots", type=int, default=64,
                    help="requests resident and stepped together (the server's max_slots)")
    ap.add_argument("--workload", choices=("coast", "uneven", "serving", "serving-ensemble"), default="coast",
                    help="coast: every line (default); uneven: the 200-scenario uneven batch alone; "
                         "serving: the uneven batch, then Poisson serving at --serve-loads of its capacity; "
                         "serving-ensemble: the same on the ensemble's all-1024^2 mix")
    ap.add_argument("--uneven-count", type=int, default=200)
    ap.add_argument("--uneven-tile", type=int, default=-1,
                    help="tile variant of the uneven batch's launches (-1: the one tuned for its largest size)")
    ap.add_argument("--uneven-compensated", action="store_true",
                    help="the uneven batch with the compensated level (SWE_OPT_COMPENSATED)")
    ap.add_argument("--uneven-local-split", action="store_true",
                    help="the uneven batch with local Lax-Friedrichs splitting (SWE_OPT_LOCAL_SPLIT)")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.7, 1.0])
    ap.add_argument("--compensated", action="store_true",
                    help="main line with the compensated level (SWE_OPT_COMPENSATED)")
    ap.add_argument("--friction-implicit", action="store_true",
                    help="main line with point-implicit friction (SWE_OPT_FRICTION_IMPLICIT)")
    ap.add_argument("--local-split", action="store_true",
                    help="main line with local Lax-Friedrichs splitting (SWE_OPT_LOCAL_SPLIT)")
    ap.add_argument("--no-valu-calibration", action="store_true",
                    help="skip the vector-ALU issue calibration (libswe_calib.so)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path; "
              "every scenario and batch runs on a single device", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2301_12010_amd import inputs, swe

    torch.cuda.set_device(0)
    if args.workload == "serving-ensemble":
        # the same serving measurement on the ensemble's mix: every request a
        # 1024^2 N-wave member (request i = member i mod count) of ens_steps
        # steps, at the loads of the ensemble's batched capacity
        args.ens_modes = ["rounds_graph"]
        batched, members = run_batched(args, torch, inputs, swe)
        cap = batched["scenarios_per_hour"] / 3600.0
        n = args.serve_requests
        out = {"batched": batched,
               "serving": {"workload": f"poisson_requests_ensemble_mix_{n}", "capacity_scenarios_per_s": cap,
                           "mix": "the ensemble members, %d steps each" % args.ens_steps}}
        for frac in args.serve_loads:
            res = run_serving(swe, members, [args.ens_steps] * n, frac * cap, args.serve_budget_gb << 30,
                              args.serve_slots, label=f"{frac}x")
            res["load_fraction"] = frac
            out["serving"][f"load_{frac}"] = res
            log(f"serving (ensemble mix) at {frac}x capacity: p50 {res['p50_time_to_result_s']:.2f}s "
                f"p99 {res['p99_time_to_result_s']:.2f}s, {res['scenarios_per_hour']:.0f} scenarios/hour, "
                f"high water {res['mem_high_water_bytes'] / 1e9:.2f} GB")
        print(json.dumps(out), flush=True)
        return
    if args.workload in ("uneven", "serving"):
        res, scens, plan = run_uneven(args, torch, inputs, swe)
        out = {"uneven": res}
        if args.workload == "serving":
            out["serving"] = run_serving_mix(args, swe, scens, plan, res["scenarios_per_hour"] / 3600.0)
        print(json.dumps(out), flush=True)
        return
    sc, value, ms, roofline, other, tv, outputs, e2e = run_large(args, torch, inputs, swe)
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": sc.name, "nx": sc.params.nx, "ny": sc.params.ny,
                   "dx": sc.params.dx, "cells": sc.cells, "cfl": sc.params.cfl,
                   "tile": [tv["tx"], tv["ty"], tv["r"]], "graph_steps": args.graph_steps},
        "roofline": roofline, "roofline_other": other,
    }
    if args.compensated or args.friction_implicit or args.local_split:
        out["config"]["options"] = {"compensated": bool(args.compensated),
                                    "friction": "implicit" if args.friction_implicit else "explicit",
                                    "split": "local" if args.local_split else "global"}
    if e2e is not None:
        out["end_to_end"] = e2e
    if outputs is not None:
        out["outputs"] = outputs
    if not args.no_small_grid:
        out["small_grid"] = measure_small_grid(torch, inputs, swe)
    if not args.no_batched:
        batched, members = run_batched(args, torch, inputs, swe)
        out["batched"] = batched
        del members
    if not args.no_uneven:
        uneven, scens, plan = run_uneven(args, torch, inputs, swe)
        out["uneven"] = uneven
        if not args.no_serving:
            log(f"serving {args.serve_requests} requests at {args.serve_loads} of the uneven capacity ...")
            out["serving"] = run_serving_mix(args, swe, scens, plan, uneven["scenarios_per_hour"] / 3600.0)
        del scens
    if not args.no_valu_calibration:
        out["valu_calibration"] = valu_calibration()
    if args.calibrate_copy_mb > 0:
        n = args.calibrate_copy_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 4 * n
        del a, b
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
