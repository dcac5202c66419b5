"""Oracle-derived expected sets at full size -- test infrastructure.

Writes the golden files under tests/golden/ that the full-size GPU tests
compare against.  It calls only the oracle (``oracle.model_*`` and
``oracle.flagged``, the plain pairwise check) and the seeded input
generators of ``synth_inputs``; nothing here comes from the HIP checker.

A full-size access log does not fit in memory (the 4096 x 4096 stencil makes
2.85e9 records over its 20 launches), so it is streamed in pieces whose
flagged sets are exactly those of the whole log restricted to the piece's
own locations:

* Launches are independent: a launch boundary orders every pair of accesses
  in different launches (Sec. II-B), so no race spans two launches and the
  flagged set of a job is the union of its launches' sets.
* Stencil: within a launch, the accesses to a cell come from its owner
  block and from the blocks next to it (halo reads, seeded writes).  A band
  of block rows together with the block row above and below it therefore
  holds every access to the band's own cells, and each block's LDS words are
  touched by that block alone.  A band's result keeps only the keys its own
  blocks own.
* Label propagation: the log is split by the label index an access touches
  (the model's ``keep`` mask), so every access to a kept label is in its
  part.

Usage: python -m oracle.goldens [jacobi] [labelprop] [batched] [serving]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth_inputs as si  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")


def workers() -> int:
    """Host threads this process may use (at most 16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def key_digest(keys) -> str:
    """SHA-256 of a flagged set: its keys sorted, one 'space,region,block,index'
    line each."""
    text = "".join("%d,%d,%d,%d\n" % k for k in sorted(keys))
    return hashlib.sha256(text.encode()).hexdigest()


# --------------------------------------------------------------------------
# Stencil: one (launch, band of block rows) piece at a time.
# --------------------------------------------------------------------------
_JAC = {}


def _jacobi_piece(args):
    launch, by0, by1 = args
    ny, nx, tab = _JAC["ny"], _JAC["nx"], _JAC["tab"]
    nby, nbx = si.jacobi_blocks(ny, nx)
    win = (0, nbx, max(by0 - 1, 0), min(by1 + 1, nby))
    recs = oracle.model_jacobi(ny, nx, 1, tab, window=win, launch0=launch)
    flagged = oracle.flagged(recs)
    own = set()
    for k in flagged:
        sp, rg, lb, ix = k
        by = lb // nbx if sp == 1 else (ix // nx) // 16
        if by0 <= by < by1:
            own.add(k)
    # checks of the piece's own blocks: the records of its band's blocks
    lo, hi = by0 * nbx, by1 * nbx
    checks = int(np.count_nonzero((recs["block"] >= lo) & (recs["block"] < hi)))
    return own, checks


def jacobi_streamed(ny: int, nx: int, launches: int, seed_tab, band: int = 16,
                    n_workers: int | None = None, launch_list=None):
    """Flagged set of the stencil job (every launch, or those of
    launch_list) and its number of checked accesses, from the oracle run
    piece by piece over worker processes.  Returns (keys, checks, seconds,
    workers)."""
    nby, _ = si.jacobi_blocks(ny, nx)
    _JAC.update(ny=ny, nx=nx, tab=None if seed_tab is None else np.asarray(seed_tab, np.int32))
    launch_list = list(range(launches)) if launch_list is None else list(launch_list)
    pieces = [(L, b, min(b + band, nby)) for L in launch_list for b in range(0, nby, band)]
    n_workers = n_workers or workers()
    t0 = time.perf_counter()
    keys, checks = set(), 0
    if n_workers == 1:
        results = map(_jacobi_piece, pieces)
    else:
        pool = ProcessPoolExecutor(n_workers, mp_context=_fork())
        results = pool.map(_jacobi_piece, pieces)
    for own, c in results:
        keys |= own
        checks += c
    if n_workers != 1:
        pool.shutdown()
    return keys, checks, time.perf_counter() - t0, n_workers


# --------------------------------------------------------------------------
# Label propagation: one (launch, part of the labels) piece at a time.
# --------------------------------------------------------------------------
_LP = {}


def _labelprop_piece(args):
    launch, part, parts = args
    rp, col, mask, tpb = _LP["rp"], _LP["col"], _LP["mask"], _LP["tpb"]
    n = rp.shape[0] - 1
    keep = (np.arange(n, dtype=np.int64) % parts == part).astype(np.uint8)
    recs = oracle.model_labelprop(rp, col, mask, 1, tpb, keep=keep, launch0=launch)
    return oracle.flagged(recs), int(recs.shape[0])


def labelprop_streamed(rp, col, mask, launches: int, tpb: int = 256, parts: int = 16,
                       n_workers: int | None = None):
    """Flagged set of the label-propagation job and its number of checked
    accesses, from the oracle run per launch and per part of the labels
    (label u belongs to part u mod parts).  Returns (keys, checks, seconds,
    workers)."""
    _LP.update(rp=np.asarray(rp, np.int32), col=np.asarray(col, np.int32),
               mask=np.asarray(mask, np.uint8), tpb=tpb)
    pieces = [(L, p, parts) for L in range(launches) for p in range(parts)]
    n_workers = n_workers or workers()
    t0 = time.perf_counter()
    keys, checks = set(), 0
    with ProcessPoolExecutor(n_workers, mp_context=_fork()) as pool:
        for f, c in pool.map(_labelprop_piece, pieces):
            keys |= f
            checks += c
    return keys, checks, time.perf_counter() - t0, n_workers


def _fork():
    import multiprocessing
    return multiprocessing.get_context("fork")


# --------------------------------------------------------------------------
# Whole jobs of the batched manifest and of the serving stream.
# --------------------------------------------------------------------------
def job_flagged(spec, arrays) -> set:
    """Flagged set of one job (job-local regions 0 and 1), launch by launch."""
    p, phases = spec["pattern"], spec["phases"]
    if p == si.PAT_REDUCE:
        return oracle.flagged(oracle.model_reduce_n(spec["n"], spec["threads"], spec["blocks"],
                                                    spec["drop"]))
    if p == si.PAT_JACOBI:
        ny, nx = spec["ny"], spec["nx"]
        if ny * nx > 1 << 20:
            return jacobi_streamed(ny, nx, phases, arrays["seed_tab"])[0]
        out = set()
        for L in range(phases):
            out |= oracle.flagged(oracle.model_jacobi(ny, nx, 1, arrays["seed_tab"], launch0=L))
        return out
    out = set()
    for L in range(phases):
        out |= oracle.flagged(oracle.model_labelprop(arrays["row_ptr"], arrays["col"],
                                                     arrays["mask"], 1, spec["threads"],
                                                     launch0=L))
    return out


def _entry(spec, keys):
    return {"index": spec["index"], "pattern": spec["pattern"], "flagged": len(keys),
            "sha256": key_digest(keys)}


def _job_entry(spec):
    return _entry(spec, job_flagged(spec, si.instance_inputs(spec)))


def _is_big(spec):
    return spec["pattern"] == si.PAT_JACOBI and spec["ny"] * spec["nx"] > 1 << 20


def jobs_golden(specs, n_workers=None):
    """Golden entry of every job: the small jobs one per worker, the
    full-size stencils each spread over all workers."""
    entries = {}
    small = [s for s in specs if not _is_big(s)]
    with ProcessPoolExecutor(n_workers or workers(), mp_context=_fork()) as pool:
        for s, e in zip(small, pool.map(_job_entry, small, chunksize=1)):
            entries[s["index"]] = e
    for s in specs:
        if _is_big(s):
            a = si.instance_inputs(s)
            keys = jacobi_streamed(s["ny"], s["nx"], s["phases"], a["seed_tab"],
                                   n_workers=n_workers)[0]
            entries[s["index"]] = _entry(s, keys)
    return [entries[s["index"]] for s in specs]


# --------------------------------------------------------------------------
# The workloads whose goldens are committed.
# --------------------------------------------------------------------------
def jacobi_full_workload():
    ny = nx = 4096
    seeds = si.jacobi_seeds(ny, nx, si.master_seed(1))
    return ny, nx, 20, seeds, si.jacobi_seed_table(ny, nx, seeds)


def labelprop_full_workload():
    scale, edges, launches = 22, 1 << 25, 10
    rp, col, mask = si.labelprop_graph(scale, edges, si.master_seed(2), 0.01)
    return rp, col, mask, launches


def serving_test_stream():
    """The job stream of the serving GPU tests: 40 jobs of the batched mix at
    reduced sizes plus two full-size 4096 x 4096 stencil jobs."""
    return si.serving_stream(si.master_seed(4), n_jobs=40, max_blocks=12, max_threads=512,
                             max_lds_kib=8.0, seeded_frac=0.5, jacobi_phases=4,
                             labelprop_phases=3)


def write_json(name, obj):
    path = os.path.join(GOLDEN, name)
    with open(path + ".tmp", "w") as f:
        json.dump(obj, f, indent=1)
        f.write("\n")
    os.replace(path + ".tmp", path)
    return path


def main(argv):
    what = set(argv) or {"jacobi", "labelprop", "batched", "serving"}
    oracle.build(force=False)
    if "jacobi" in what:
        ny, nx, launches, seeds, tab = jacobi_full_workload()
        keys, checks, sec, w = jacobi_streamed(ny, nx, launches, tab)
        print("jacobi %dx%d x %d launches: %d flagged, %d checks, %.1f s on %d workers"
              % (ny, nx, launches, len(keys), checks, sec, w), flush=True)
        write_json("jacobi_4096x4096_20launches.json", {
            "workload": "5-point Jacobi, fp32 4096 x 4096, 16 x 16 blocks, 20 launches, "
                        "66 seeded blocks (master seed 0x24010471)",
            "generated_by": "python -m oracle.goldens jacobi",
            "checks": checks, "flagged": len(keys), "sha256": key_digest(keys),
            "keys": [list(k) for k in sorted(keys)]})
    if "labelprop" in what:
        rp, col, mask, launches = labelprop_full_workload()
        keys, checks, sec, w = labelprop_streamed(rp, col, mask, launches)
        print("labelprop rmat22: %d flagged, %d checks, %.1f s on %d workers"
              % (len(keys), checks, sec, w), flush=True)
        ks = sorted(keys)
        write_json("labelprop_rmat22_10launches.json", {
            "workload": "label propagation, R-MAT scale 22, 2^25 edges, 1 % seeded edges, "
                        "10 launches, 256 threads per block (master seed 0x24010472)",
            "generated_by": "python -m oracle.goldens labelprop",
            "checks": checks, "flagged": len(keys), "sha256": key_digest(keys),
            "first_keys": [list(k) for k in ks[:16]], "last_keys": [list(k) for k in ks[-16:]]})
    if "batched" in what:
        specs = si.batched_manifest(si.master_seed(3))
        t0 = time.perf_counter()
        entries = jobs_golden(specs)
        print("batched manifest: %d jobs, %d flagged in all, %.1f s"
              % (len(entries), sum(e["flagged"] for e in entries), time.perf_counter() - t0),
              flush=True)
        write_json("batched_manifest_1000.json", {
            "workload": "1000-job batched manifest (master seed 0x24010473)",
            "generated_by": "python -m oracle.goldens batched", "jobs": entries})
    if "serving" in what:
        specs = serving_test_stream()
        t0 = time.perf_counter()
        entries = jobs_golden(specs)
        print("serving test stream: %d jobs, %d flagged in all, %.1f s"
              % (len(entries), sum(e["flagged"] for e in entries), time.perf_counter() - t0),
              flush=True)
        write_json("serving_stream_40.json", {
            "workload": "serving test stream: 40 jobs, 2 of them full-size 4096 x 4096 "
                        "stencils (master seed 0x24010474)",
            "generated_by": "python -m oracle.goldens serving", "jobs": entries})


if __name__ == "__main__":
    main(sys.argv[1:])
