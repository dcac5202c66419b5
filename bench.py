#!/usr/bin/env python3
"""Race-check throughput on one MI355X.

Workload: a 5-point Jacobi stencil over a 4096 x 4096 fp32 grid, 16 x 16
thread blocks staging an 18 x 18 LDS tile, 20 launches ping-ponging two
arrays (a launch boundary orders every launch after the previous one), with
0.1 % of the blocks (66) seeded to also write one neighbour-owned halo cell
(a cross-block race).  Every global and LDS access is checked by the HIP
hook.  One step is one whole checking job on resident inputs: reset the
shadow, 20 instrumented launches with their launch boundaries, and the
report (device-to-host copy of the flagged set).

The timed jobs record one pair of HIP events around each job's launches
(the mean launch time of the roofline) and none between them; the per-launch
latency percentiles come from the same number of jobs run right after, with
a pair around every launch.

Prints one JSON line: checks/s, slowdown against the same kernel without
hooks, p50/p99 per-launch latency, the roofline of the instrumented kernel,
measured device peaks, and the CPU oracle timed on the same records (launch
0 of the job by default, the whole job with --cpu-full-job) on the host
threads available (at most 16), and on one core.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NY = NX = 4096
LAUNCHES = 20
HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth


def jacobi_check_counts(ny: int, nx: int, seeded_writes: int):
    """Instrumented accesses of one sweep: (global checks, LDS checks)."""
    cells = ny * nx
    halo = 2 * nx * (((ny + 15) // 16) - 1) + 2 * ny * (((nx + 15) // 16) - 1)
    g_read, l_write = cells + halo, cells + halo
    l_read = 5 * cells - 2 * nx - 2 * ny
    g_write = cells + seeded_writes
    return g_read + g_write, l_write + l_read


def algorithmic_bytes_per_launch(ny: int, nx: int) -> int:
    """HBM bytes the checking method must move in one sweep: for each of the
    two monitored arrays, every 8-byte shadow word is read and written back
    once (each word changes state at least once per launch, and streaming
    it costs its line's read and write-back), 16 bytes per monitored word."""
    return 2 * ny * nx * (8 + 8)


def data_bytes_per_launch(ny: int, nx: int) -> int:
    """HBM bytes of the stencil's own data in one sweep: a 4-byte read of
    u_old and a 4-byte write of u_new per cell."""
    return ny * nx * (4 + 4)


def counter_record(kernel: str, summary: str):
    """The machine-readable record of a committed counter summary under
    profiles/ for `kernel`, or None when the kernel's built assembly
    fingerprint differs from the recorded one."""
    import re as _re
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    m = _re.search(r"```json\n(.*?)\n```", open(path).read(), flags=_re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    fp_path = os.path.join(ROOT, "paper_2401_04701_amd", "libhr_kernels.json")
    if rec.get("kernel") != kernel or not os.path.exists(fp_path):
        return None
    with open(fp_path) as f:
        if json.load(f).get(rec["isa_symbol"]) != rec["isa_sha256"]:
            return None
    return rec


def counter_traffic(kernel: str, summary: str = "k_jacobi_check_4096x4096_hbm_counters.md"):
    """HBM bytes per launch of `kernel` from its committed counter summary
    under profiles/, or None when the kernel changed since the counters were
    taken: its built assembly fingerprint differs from the recorded one, and
    so does the hash of the sources it compiles from."""
    import hashlib
    import re as _re
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    m = _re.search(r"```json\n(.*?)\n```", open(path).read(), flags=_re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec["kernel"] != kernel:
        return None
    fp_path = os.path.join(ROOT, "paper_2401_04701_amd", "libhr_kernels.json")
    if rec.get("isa_sha256") and os.path.exists(fp_path):
        with open(fp_path) as f:
            if json.load(f).get(rec["isa_symbol"]) == rec["isa_sha256"]:
                return rec["traffic_bytes_per_launch"]
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q))


def host_cpu():
    """The host's CPU model and the threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(),
            "threads_available": len(os.sched_getaffinity(0))}


def cpu_baseline(gpu_keys, full_job=False):
    """The oracle on the same records the GPU checks: the access log of the
    4096 x 4096 job modelled and checked piece by piece (one launch, one band
    of 16 block rows with its neighbour rows; oracle/goldens.py), over worker
    processes on the host threads available (at most 16).  By default the
    sample is launch 0 of the job's 20; full_job runs all 20 launches.  Its
    flagged set is compared with the GPU's keys of the launch's output array
    (region 1 for launch 0).  Also one band of launch 0 on one core."""
    import oracle
    import synth_inputs as si
    from oracle import goldens
    oracle.build(force=False)
    seeds = si.jacobi_seeds(NY, NX, si.master_seed(1))
    tab = si.jacobi_seed_table(NY, NX, seeds)
    launches = list(range(LAUNCHES)) if full_job else [0]
    keys, checks, dt, workers = goldens.jacobi_streamed(NY, NX, LAUNCHES, tab,
                                                        launch_list=launches)
    want = gpu_keys if full_job else {k for k in gpu_keys if k[1] == 1}
    t0 = time.perf_counter()
    goldens._JAC.update(ny=NY, nx=NX, tab=tab)
    _, one_checks = goldens._jacobi_piece((0, 0, 16))
    one_dt = time.perf_counter() - t0
    what = "the whole job (20 launches)" if full_job else "launch 0 of the job's 20"
    return {"value": checks / dt, "unit": "checks/s", "cores": workers, "kind": "oracle",
            "sample": f"{what} on the full {NY}x{NX} grid, the same records the GPU checks: "
                      f"{checks} checks in {dt:.1f} s over {workers} worker processes, "
                      f"{len(keys)} flagged",
            "seconds": dt, "checks": checks, "flagged": len(keys),
            "same_flagged_set_as_gpu": keys == want,
            "single_core": {"value": one_checks / one_dt, "unit": "checks/s", "cores": 1,
                            "sample": f"launch 0, block rows 0-15 (with row 16): {one_checks} "
                                      f"checks in {one_dt:.1f} s"},
            "host": host_cpu()}


def _best_ms(torch, stream, fn, reps=6):
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def measure_peaks(torch, hr, stream):
    """Measured agent-scope atomic, coherent-load and copy peaks (best of 6)."""
    out = {}
    n = 1 << 25                                     # 256 MiB of 8-byte words
    words = torch.zeros(n, dtype=torch.int64, device="cuda")
    fails = torch.zeros(1, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    rnd = [0]
    for op, opname in ((0, "cas"), (1, "xchg")):
        for scatter, pat in ((0, "coalesced"), (1, "scattered")):
            # the best over grid sizes: fewer, longer-running blocks keep more
            # operations in flight per wave
            best_rate, best_blocks = 0.0, 0
            for blocks in ((0, 1024, 2048, 4096, 8192) if scatter == 0 else (0,)):
                def run(op=op, scatter=scatter, blocks=blocks):
                    hr.peak_atomic(words, op, rnd[0], scatter, fails, blocks)
                    rnd[0] += 1
                rate = n / (_best_ms(torch, stream, run) * 1e-3)
                if rate > best_rate:
                    best_rate, best_blocks = rate, blocks
            out[f"{opname}_{pat}_per_s"] = best_rate
            if scatter == 0:
                out[f"{opname}_{pat}_blocks"] = best_blocks or min((n + 255) // 256, 65536)
    # spread over a 32 MiB array (the label-propagation shadow size)
    nr = 1 << 22
    for op, opname in ((0, "cas"), (1, "xchg")):
        def run(op=op):
            hr.peak_atomic(words[:nr], op, rnd[0], 2, fails)
            rnd[0] += 1
        words[:nr].fill_(rnd[0])
        torch.cuda.synchronize()
        out[f"{opname}_random32MiB_per_s"] = nr / (_best_ms(torch, stream, run) * 1e-3)
    out["atomic_failures"] = int(fails.item())
    blocks, iters = 4096, 256
    for op, name in ((0, "lds_cas_per_s"), (1, "lds_load_cas_per_s")):
        ms = _best_ms(torch, stream, lambda op=op: hr.peak_lds(blocks, iters, op, fails))
        out[name] = blocks * 1024 * iters / (ms * 1e-3)
    out["lds_failures"] = int(fails.item()) - out["atomic_failures"]
    for scatter, pat in ((0, "coalesced"), (1, "scattered")):
        ms = _best_ms(torch, stream, lambda scatter=scatter: hr.peak_load(words, scatter, sink))
        out[f"load_{pat}_per_s"] = n / (ms * 1e-3)
    src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda").random_(0, 255)
    dst = torch.empty_like(src)
    ms = _best_ms(torch, stream, lambda: hr.peak_copy(src, dst))
    out["copy_gbs"] = 2 * src.numel() / (ms * 1e-3) / 1e9
    del words, src, dst
    return out


class Timing:
    """HIP events on the launch stream.  per_launch: a pair around every
    launch, for the per-launch latency percentiles; each pair leaves the
    device idle for a few microseconds between launches.  Otherwise one pair
    around all the launches of a job (end() after its last launch), so that
    the timed jobs run their launches back to back as a caller's would."""

    def __init__(self, torch, stream, per_launch):
        self.torch, self.stream, self.per_launch = torch, stream, per_launch
        self.pairs, self.counts = [], []
        self._first, self._n = None, 0

    def _event(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        return e

    def launch(self, fn):
        if self.per_launch:
            e0 = self._event()
            fn()
            self.pairs.append((e0, self._event()))
            self.counts.append(1)
            return
        if self._first is None:
            self._first = self._event()
        fn()
        self._n += 1

    def end(self):
        if self._first is not None:
            self.pairs.append((self._first, self._event()))
            self.counts.append(self._n)
            self._first, self._n = None, 0

    def ms(self):
        """Per pair: one launch (per_launch), or one job's launches."""
        return [a.elapsed_time(b) for a, b in self.pairs]

    def mean_launch_ms(self):
        return sum(self.ms()) / max(1, sum(self.counts))


def _timed_launch(timing, fn):
    if timing is None:
        fn()
    else:
        timing.launch(fn)


def _end_launches(timing):
    if timing is not None:
        timing.end()


def _timed_job(args, torch, stream, job):
    """Warm up, then time `steps` whole jobs with one event pair around each
    job's launches; then run `steps` more with a pair around every launch for
    the latency percentiles.  Returns (seconds per job, mean launch ms of the
    timed jobs, per-launch ms, the last timed job's result)."""
    for _ in range(args.warmup):
        job(None)
    torch.cuda.synchronize()
    span = Timing(torch, stream, per_launch=False)
    t0 = time.perf_counter()
    out = None
    for _ in range(args.steps):
        out = job(span)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / args.steps
    each = Timing(torch, stream, per_launch=True)
    for _ in range(args.steps):
        job(each)
    torch.cuda.synchronize()
    return step_s, span.mean_launch_ms(), each.ms(), out


def _common(args, metric_value, step_s, launch_ms, plain_ms, plain_step_s, workload, extra):
    return {
        "metric": "instrumented accesses checked/sec + slowdown vs uninstrumented; p50/p99 check latency",
        "value": metric_value, "unit": "checks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": workload, **extra, "parallelism": "single GPU"},
        "slowdown": float(np.median(launch_ms) / np.median(plain_ms)),
        "slowdown_step": step_s / plain_step_s,
        "p50_launch_ms": pct(launch_ms, 50), "p99_launch_ms": pct(launch_ms, 99),
        "plain_p50_launch_ms": pct(plain_ms, 50)}


def bench_labelprop(args, torch, si, hr, stream):
    """R-MAT scale 22, 2^25 edges, 1 % seeded edges, 10 launches per job."""
    scale, edges, launches, tpb = 22, 1 << 25, 10, 256
    rp, col, mask = si.labelprop_graph(scale, edges, si.master_seed(2), 0.01)
    n = 1 << scale
    checks_per_launch = n + edges + int(mask.sum())
    label = torch.arange(n, dtype=torch.int32, device="cuda")
    init = label.clone()
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    mask_d = torch.from_numpy(mask).cuda()
    ctx = hr.Context(ring_capacity=1 << 21)
    r_lab = ctx.shadow_alloc(label)

    def job(ev):
        ctx.reset()
        label.copy_(init)
        for _ in range(launches):
            _timed_launch(ev, lambda: ctx.labelprop_check(
                r_lab, label, rp_d, col_d, mask_d, tpb=tpb))
            ctx.kernel_end()
        _end_launches(ev)
        return ctx.report()

    def plain(ev):
        label.copy_(init)
        for _ in range(launches):
            _timed_launch(ev, lambda: hr.labelprop_plain(label, rp_d, col_d, mask_d, tpb))
        _end_launches(ev)

    step_s, avg_ms, launch_ms, (recs, st) = _timed_job(args, torch, stream, job)
    pstep_s, _, plain_ms, _ = _timed_job(args, torch, stream, plain)
    ctx.close()
    assert st == 0
    res = _common(args, checks_per_launch * launches / step_s, step_s, launch_ms, plain_ms,
                  pstep_s, "labelprop_rmat22_2p25edges_seeded1pct_10launches",
                  {"vertices": n, "edges": edges, "launches": launches,
                   "checks_per_step": checks_per_launch * launches})
    # algorithmic bytes: the sweep's own data (row_ptr and the label load per
    # vertex, col + mask + label min per edge) plus one 8-byte shadow load per
    # check; the shadow words themselves change only a few times per launch
    alg = n * (8 + 4) + edges * (4 + 1 + 4) + checks_per_launch * 8 + n * 16
    avg = avg_ms * 1e-3
    res["flagged"] = int(len(recs))
    res["roofline"] = {"bound": "hbm", "achieved": alg / avg / 1e9, "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": alg / avg / 1e9 / HBM_PEAK_GBS,
                       "traffic": counter_traffic(
                           "k_labelprop<1>", "k_labelprop_check_rmat22_hbm_counters.md"),
                       "kernel": "k_labelprop<1>", "alg_bytes_per_launch": alg,
                       "avg_launch_ms": avg * 1e3}
    print(json.dumps(res), flush=True)


def bench_reduce(args, torch, si, hr, stream):
    """One block, 256 threads, LDS int32[512] tree reduction (latency)."""
    x = torch.from_numpy(si.reduce_input(si.master_seed(0))).cuda()
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    ctx = hr.Context()
    r_in, r_out = ctx.shadow_alloc(x), ctx.shadow_alloc(out)
    reps = 50

    def job(ev):
        ctx.reset()
        for _ in range(reps):
            _timed_launch(ev, lambda: ctx.reduce_check(r_in, r_out, x, out, 3))
            ctx.kernel_end()
        _end_launches(ev)
        return ctx.report()

    def plain(ev):
        for _ in range(reps):
            _timed_launch(ev, lambda: hr.reduce_plain(x, out, 3))
        _end_launches(ev)

    step_s, _, launch_ms, (recs, st) = _timed_job(args, torch, stream, job)
    pstep_s, _, plain_ms, _ = _timed_job(args, torch, stream, plain)
    ctx.close()
    res = _common(args, 3069 * reps / step_s, step_s, launch_ms, plain_ms, pstep_s,
                  "reduce_lds_int32x512_1block256_drop3", {"launches_per_step": reps,
                                                          "checks_per_launch": 3069})
    res["flagged"] = int(len(recs))
    res["p50_launch_us"] = pct(launch_ms, 50) * 1e3
    res["p99_launch_us"] = pct(launch_ms, 99) * 1e3
    print(json.dumps(res), flush=True)


def bench_batched(args, torch, si, hr, stream):
    """1000 checked jobs (reduce / jacobi / labelprop, blocks 1-512, threads
    64-1024, LDS 1-64 KiB, 10 % seeded) in one persistent launch, against the
    serial path running the same jobs one at a time (context, shadow, one
    launch per phase, report, free)."""
    from paper_2401_04701_amd import jobs, tune

    def note(*a):
        print("[batched]", *a, file=sys.stderr, flush=True)
    note("building 1000 job inputs")
    specs = si.batched_manifest(si.master_seed(3))
    arrays = [si.instance_inputs(s) for s in specs]
    js = [jobs.Job(s, a) for s, a in zip(specs, arrays)]
    checks = sum(jobs.check_count_arrays(s, a) for s, a in zip(specs, arrays))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = hr.Context(ring_capacity=1 << 20)
    batch = hr.Batch(ctx, [j.inst for j in js])
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    note("autotuning")
    best, trials = tune.autotune(ctx, batch)
    note("timed batched runs with", best)

    def job(ev):
        ctx.reset()
        _timed_launch(ev, lambda: batch.run(**best))
        _end_launches(ev)
        return ctx.report()

    step_s, _, launch_ms, (recs, st) = _timed_job(args, torch, stream, job)
    assert st == 0
    per_batch = batch.split({(int(r["space"]), int(r["region"]),
                              int(r["block"]) if r["space"] == hr.HR_LDS else 0, int(r["index"]))
                             for r in recs})
    # the serial path over the same jobs (timed once, whole)
    note("serial path")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_serial = [j.serial(ring_capacity=1 << 20) for j in js]
    serial_s = time.perf_counter() - t0
    equal = all(st2 == 0 and a == b for (a, st2), b in zip(per_serial, per_batch))
    items = batch.info(0)[1]
    batch.close()
    ctx.close()
    res = {
        "metric": "instrumented accesses checked/sec + slowdown vs uninstrumented; p50/p99 check latency",
        "value": checks / step_s, "unit": "checks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batched_1000_mixed_jobs_one_persistent_launch", "jobs": len(js),
                   "checks_per_step": int(checks), "work_items": items,
                   "parallelism": "single GPU"},
        "jobs_per_s": len(js) / step_s,
        "serial_jobs_per_s": len(js) / serial_s,
        "serial_checks_per_s": checks / serial_s,
        "batched_vs_serial": serial_s / step_s,
        "equal_results": bool(equal),
        "flagged": int(len(recs)),
        "tuning": best, "tuning_trials_ms": trials, "batch_create_ms": create_ms,
        "p50_launch_ms": pct(launch_ms, 50), "p99_launch_ms": pct(launch_ms, 99)}
    print(json.dumps(res), flush=True)


def bench_serving(args, torch, si, hr, stream):
    """Poisson streams of check jobs (95 % the batched mix, 5 % full 4096^2
    stencil jobs, 20 launches, 0.1 % of blocks seeded) at each arrival rate,
    served with continuous batching against a 64 GiB shadow budget, and the
    serial plain path (context, shadow, launches, report, free; one job at a
    time) replaying the same arrival trace.  Latency = finish - arrival."""
    from paper_2401_04701_amd import jobs

    def note(*a):
        print("[serving]", *a, file=sys.stderr, flush=True)
    rates = [float(r) for r in args.rates.split(",")]
    specs = si.serving_stream(si.master_seed(4), n_jobs=args.serve_jobs)
    note("building", len(specs), "job inputs")
    js, checks = [], 0
    for i, spec in enumerate(specs):
        a = si.instance_inputs(spec)
        checks += jobs.check_count_arrays(spec, a)
        js.append(jobs.Job(spec, a))
        del a
        if (i + 1) % 250 == 0:
            note("  built", i + 1)
    torch.cuda.synchronize()
    insts = [j.inst for j in js]
    ctx = hr.Context(ring_capacity=1 << 20)
    note("warm-up")
    hr.serve(ctx, insts[:64], np.zeros(64), stream=stream)
    hr.serve(ctx, insts[:16], np.zeros(16), serial=True, stream=stream)
    pat = np.array([s["pattern"] for s in specs])
    big = np.array([bool(s.get("big")) for s in specs])
    classes = {"reduce": pat == si.PAT_REDUCE,
               "stencil_small": (pat == si.PAT_JACOBI) & ~big,
               "stencil_4096sq": big,
               "labelprop": pat == si.PAT_LABELPROP}
    out, equal = [], True
    for rate in rates:
        arr = si.poisson_arrivals(si.master_seed(4) + int(rate), len(js), rate)
        row, sets = {"rate_per_s": rate}, {}
        for mode in ("served", "serial"):
            note("rate", rate, mode)
            sets[mode], times = hr.serve(ctx, insts, arr, serial=(mode == "serial"),
                                         large_burst=args.serve_large_burst,
                                         lane_burst=args.serve_lane_burst, stream=stream)
            fin = np.array([t.finish_s for t in times])
            lat = fin - arr
            span = float(fin.max())
            row[mode] = {"jobs_per_s": len(js) / span, "checks_per_s": checks / span,
                         "makespan_s": span, "p50_ms": pct(lat, 50) * 1e3,
                         "p99_ms": pct(lat, 99) * 1e3,
                         "clean_status": all(t.status == 0 for t in times),
                         "flagged": int(sum(t.flagged for t in times)),
                         "by_class": {c: {"jobs": int(m.sum()), "p50_ms": pct(lat[m], 50) * 1e3,
                                          "p99_ms": pct(lat[m], 99) * 1e3}
                                      for c, m in classes.items() if m.any()}}
            note("  %.0f jobs/s, p50 %.2f ms, p99 %.2f ms; p50 by class %s"
                 % (row[mode]["jobs_per_s"], row[mode]["p50_ms"], row[mode]["p99_ms"],
                    {c: round(v["p50_ms"], 3) for c, v in row[mode]["by_class"].items()}))
        # every job's flagged set served in the mix equals its set run alone
        row["equal_results"] = (sets["served"] == sets["serial"]
                                and row["served"]["clean_status"]
                                and row["serial"]["clean_status"])
        equal &= row["equal_results"]
        row["served_vs_serial_jobs_per_s"] = (row["served"]["jobs_per_s"]
                                              / row["serial"]["jobs_per_s"])
        out.append(row)
    ctx.close()
    top = out[-1]
    res = {
        "metric": "instrumented accesses checked/sec + slowdown vs uninstrumented; p50/p99 check latency",
        "value": top["served"]["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1,
        "steps": len(rates), "warmup": 1, "ms_per_step": top["served"]["makespan_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "serving_poisson_stream_%d_jobs_5pct_4096sq_stencil" % len(js),
                   "jobs": len(js), "full_size_jobs": sum(bool(s.get("big")) for s in specs),
                   "checks_per_stream": int(checks), "shadow_budget_bytes": 64 << 30,
                   "large_burst": args.serve_large_burst or "all phases",
                   "lane_burst": args.serve_lane_burst or "library default",
                   "parallelism": "single GPU"},
        "p50_ms": top["served"]["p50_ms"], "p99_ms": top["served"]["p99_ms"],
        "p50_ms_by_class": {c: v["p50_ms"] for c, v in top["served"]["by_class"].items()},
        "served_vs_serial": top["served_vs_serial_jobs_per_s"],
        "equal_results": bool(equal), "rates": out}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full-job", action="store_true",
                    help="time the oracle on all 20 launches of the job (a few minutes of "
                         "host time) instead of launch 0")
    ap.add_argument("--no-peaks", action="store_true")
    ap.add_argument("--verify-count", action="store_true",
                    help="first run one job with the device access counter (untimed)")
    ap.add_argument("--workload", default="jacobi",
                    choices=["jacobi", "labelprop", "reduce", "batched", "serving"],
                    help="jacobi: the headline 4096^2 stencil job; labelprop: R-MAT scale-22 "
                         "label propagation job; reduce: one-block LDS reduction latency; "
                         "batched: 1000 mixed jobs in one persistent launch vs one at a time; "
                         "serving: Poisson job streams, continuous batching vs one at a time")
    ap.add_argument("--rates", default="100,250,500,1000,2500,5000",
                    help="serving: arrival rates in jobs/s")
    ap.add_argument("--serve-jobs", type=int, default=2000, help="serving: jobs per stream")
    ap.add_argument("--serve-large-burst", type=int, default=0,
                    help="serving: phases of a large stencil job per iteration (0: all)")
    ap.add_argument("--serve-lane-burst", type=int, default=0,
                    help="serving: phases per iteration of the short-job lane (0: the library's)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first copy 256 MiB once with the library's copy kernel, the "
                         "calibration of the HBM byte counters of a counter run")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the checker runs each job on a single device "
              "(jobs shard across GPUs with no exchange); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth_inputs as si
    from paper_2401_04701_amd import hr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.calibration_copy:
        src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda").random_(0, 255)
        dst = torch.empty_like(src)
        hr.peak_copy(src, dst)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "labelprop":
        return bench_labelprop(args, torch, si, hr, stream)
    if args.workload == "reduce":
        return bench_reduce(args, torch, si, hr, stream)
    if args.workload == "batched":
        return bench_batched(args, torch, si, hr, stream)
    if args.workload == "serving":
        return bench_serving(args, torch, si, hr, stream)

    seeds = si.jacobi_seeds(NY, NX, si.master_seed(1))
    tab = torch.from_numpy(si.jacobi_seed_table(NY, NX, seeds)).cuda()
    u0 = torch.from_numpy(si.jacobi_grid(NY, NX, si.master_seed(1))).cuda()
    u = [u0.clone(), torch.zeros_like(u0)]
    n_g, n_l = jacobi_check_counts(NY, NX, len(seeds))
    checks_per_launch = n_g + n_l
    checks_per_step = checks_per_launch * LAUNCHES

    if args.verify_count:
        # the access count from the device counter (untimed, slower kernel)
        with hr.Context(count_checks=True) as cctx:
            regs = [cctx.shadow_alloc(u[0]), cctx.shadow_alloc(u[1])]
            for L in range(LAUNCHES):
                cctx.jacobi_check(regs[L % 2], regs[(L + 1) % 2], u[L % 2], u[(L + 1) % 2], tab)
                cctx.kernel_end()
            counted = cctx.check_count()
        assert counted == checks_per_step, (counted, checks_per_step)

    ctx = hr.Context()
    regs = [ctx.shadow_alloc(u[0]), ctx.shadow_alloc(u[1])]

    def checked_step(timing, c=ctx, rg=regs, clears=None):
        c.reset()
        for L in range(LAUNCHES):
            _timed_launch(timing, lambda: c.jacobi_check(rg[L % 2], rg[(L + 1) % 2], u[L % 2],
                                                         u[(L + 1) % 2], tab))
            if clears is None:
                c.kernel_end()
            else:
                clears.launch(c.kernel_end)      # the 4-byte words' boundary clears
        _end_launches(timing)
        return c.report()

    def plain_step(timing):
        for L in range(LAUNCHES):
            _timed_launch(timing, lambda: hr.jacobi_plain(u[L % 2], u[(L + 1) % 2], tab))
        _end_launches(timing)

    step_s, avg_launch_ms, launch_ms, (recs, st) = _timed_job(args, torch, stream, checked_step)
    flagged_count = len(recs)
    assert st == 0 and flagged_count > 0
    pstep_s, _, plain_ms, _ = _timed_job(args, torch, stream, plain_step)
    ctx.close()

    # The same job with 4-byte shadow words (default widths: 16-bit block
    # field, exact for these 65,536 blocks); the launch-boundary clear of
    # its shadow is timed on its own.
    ctx4 = hr.Context(word4=True)
    regs4 = [ctx4.shadow_alloc(u[0]), ctx4.shadow_alloc(u[1])]
    step4_s, _, launch4_ms, (recs4, st4) = _timed_job(
        args, torch, stream, lambda t: checked_step(t, ctx4, regs4))
    clears = Timing(torch, stream, per_launch=True)
    for _ in range(2):
        checked_step(None, ctx4, regs4, clears)
    torch.cuda.synchronize()
    clear4_ms = clears.ms()
    del clears
    ctx4.close()

    def keys(rs):
        return {(int(r["space"]), int(r["region"]), int(r["block"]) if r["space"] else 0,
                 int(r["index"])) for r in rs}
    assert st4 == 0 and keys(recs4) == keys(recs)

    # The same job under each shadow map and transition encoding the
    # autotuner knows (tune.autotune_stencil): per-launch time and the
    # flagged set, which must not change (and must be the headline's).
    from paper_2401_04701_amd import tune
    tuned, trials, tuned_set = tune.autotune_stencil(hr, u, tab, LAUNCHES, stream=stream)
    map_ms = {k[len("map_"):]: v for k, v in trials.items() if k.startswith("map_")}
    fsm_ms = {k[len("fsm_"):]: v for k, v in trials.items() if k.startswith("fsm_")}
    remap = {regs[0]: 0, regs[1]: 1}
    head_set = {(sp, remap[rg] if sp == 0 else rg, lb, ix) for sp, rg, lb, ix in keys(recs)}
    map_same = fsm_same = tuned_set == head_set

    avg_launch_s = avg_launch_ms * 1e-3
    alg = algorithmic_bytes_per_launch(NY, NX)
    achieved = alg / avg_launch_s / 1e9
    with_data = alg + data_bytes_per_launch(NY, NX)
    result = {
        "metric": "instrumented accesses checked/sec + slowdown vs uninstrumented; p50/p99 check latency",
        "value": checks_per_step / step_s,
        "unit": "checks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "jacobi5pt_fp32_4096x4096_b16x16_lds18x18_20launches_seeded66",
                   "grid": [NY, NX], "launches": LAUNCHES, "seeded_blocks": int(len(seeds)),
                   "checks_per_step": int(checks_per_step),
                   "global_checks_per_launch": int(n_g), "lds_checks_per_launch": int(n_l),
                   "parallelism": "single GPU"},
        "slowdown": float(np.median(launch_ms) / np.median(plain_ms)),
        "slowdown_step": step_s / pstep_s,
        "p50_launch_ms": pct(launch_ms, 50),
        "p99_launch_ms": pct(launch_ms, 99),
        "plain_p50_launch_ms": pct(plain_ms, 50),
        "flagged": int(flagged_count),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic("k_jacobi<1>"),
                     "kernel": "k_jacobi<1>", "alg_bytes_per_launch": alg,
                     "alg_bytes": "16 B per monitored shadow word (8 B read, 8 B written "
                                  "back), 2 x 4096 x 4096 words",
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "with_stencil_data": {
                         "bytes_per_launch": with_data,
                         "achieved": with_data / avg_launch_s / 1e9,
                         "frac": with_data / avg_launch_s / 1e9 / HBM_PEAK_GBS}},
    }
    result["word4"] = {"value": checks_per_step / step4_s, "unit": "checks/s",
                       "ms_per_step": step4_s * 1e3,
                       "p50_launch_ms": pct(launch4_ms, 50), "p99_launch_ms": pct(launch4_ms, 99),
                       "p50_clear_ms": pct(clear4_ms, 50),
                       "shadow_bytes": 2 * NY * NX * 4, "shadow_bytes_8byte": 2 * NY * NX * 8,
                       "flagged": len(recs4), "same_flagged_set": True}
    result["shadow_map"] = {"headline_map": "rowmajor", "p50_launch_ms": map_ms,
                            "fastest": min(map_ms, key=map_ms.get),
                            "same_flagged_set": bool(map_same)}
    result["fsm_encoding"] = {"headline": "bits", "p50_launch_ms": fsm_ms,
                              "fastest": min(fsm_ms, key=fsm_ms.get),
                              "same_flagged_set": bool(fsm_same)}
    result["stencil_autotune"] = {"best": {"tile": tune.tile_name(tuned["tile"]),
                                           "fsm": tuned["fsm"]},
                                  "trials_p50_launch_ms": trials}
    if not args.no_peaks:
        peaks = measure_peaks(torch, hr, stream)
        g_rate = n_g / avg_launch_s
        result["atomic"] = {"global_checks_per_s": g_rate,
                            "peak_xchg_per_s": peaks["xchg_coalesced_per_s"],
                            "frac": g_rate / peaks["xchg_coalesced_per_s"], **peaks}
        # the memory-side atomic requests the kernel actually issues (its
        # exchanges and fold compare-and-swaps, 8 lanes of 8-byte words per
        # request; hooks whose word does not change issue none), from the
        # committed L2 counters while the kernel is the one they measured
        rec = counter_record("k_jacobi<1>", "k_jacobi_check_4096x4096_l2_counters.md")
        if rec:
            req_s = rec["ea_atomic_requests_per_launch"] / avg_launch_s
            peak_req = peaks["xchg_coalesced_per_s"] / rec["lanes_per_request"]
            result["atomic"].update(ea_requests_per_launch=rec["ea_atomic_requests_per_launch"],
                                    ea_requests_per_s=req_s, peak_requests_per_s=peak_req,
                                    requests_frac=req_s / peak_req)
    if not args.no_cpu_baseline:
        remap = {regs[0]: 0, regs[1]: 1}
        gpu_keys = {(int(r["space"]),
                     int(r["region"]) if r["space"] else remap[int(r["region"])],
                     int(r["block"]) if r["space"] else 0, int(r["index"])) for r in recs}
        result["cpu_baseline"] = cpu_baseline(gpu_keys, full_job=args.cpu_full_job)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
