"""Batched checking on the GPU: many jobs in one persistent launch must give,
job by job, the same flagged set as running the job alone (serial path) and
as the oracle; tolerance zero.  Different worker counts, queue orders and
executor variants change the schedule, never the result."""
import numpy as np
import pytest

import json
import os

import oracle
import synth_inputs as si
from oracle import closed_forms as cf
from oracle.goldens import key_digest

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_04701_amd import hr, jobs
    torch.cuda.set_device(0)
    return torch, hr, jobs


def say(*a):
    print("[case]", *a, flush=True)


def expected(spec, arrays, use_oracle):
    """Flagged keys of one job with job-local regions (0, 1)."""
    p = spec["pattern"]
    if p == si.PAT_REDUCE:
        want = cf.reduce_n_flagged(spec["n"], spec["threads"], spec["blocks"], spec["drop"])
        if use_oracle:
            got = oracle.flagged(oracle.model_reduce_n(spec["n"], spec["threads"], spec["blocks"],
                                                       spec["drop"]))
            assert got == want
        return want
    if p == si.PAT_JACOBI:
        want = cf.jacobi_flagged(spec["ny"], spec["nx"], spec["phases"], arrays["seeds"])
        if use_oracle:
            got = oracle.flagged(oracle.model_jacobi(spec["ny"], spec["nx"], spec["phases"],
                                                     arrays["seed_tab"]))
            assert got == want
        return want
    want = cf.labelprop_flagged(arrays["row_ptr"], arrays["col"], arrays["mask"])
    if use_oracle:
        got = oracle.flagged(oracle.model_labelprop(arrays["row_ptr"], arrays["col"],
                                                    arrays["mask"], spec["phases"],
                                                    spec["threads"]))
        assert got == want
    return want


def small_manifest(n=36, seed=11):
    specs = si.batched_manifest(seed, n_instances=n, max_blocks=12, max_threads=512,
                                max_lds_kib=8.0, seeded_frac=0.5, jacobi_phases=4,
                                labelprop_phases=3)
    return specs, [si.instance_inputs(s) for s in specs]


def test_batch_small_matches_serial_and_oracle(env):
    torch, hr, jobs = env
    specs, arrays = small_manifest()
    want = [expected(s, a, use_oracle=True) for s, a in zip(specs, arrays)]
    assert sum(bool(w) for w in want) >= 5
    js = [jobs.Job(s, a) for s, a in zip(specs, arrays)]
    say("serial path", len(js), "jobs")
    for i, (j, w) in enumerate(zip(js, want)):
        got, st = j.serial()
        assert st == 0 and got == w, j.spec
    say("serial path done")
    with hr.Context(count_checks=True) as ctx:
        with hr.Batch(ctx, [j.inst for j in js]) as b:
            for variant in (0, 1):
                max_w, items = b.info(variant)
                assert max_w > 0 and items > 0
                for order, workers in ((0, 0), (1, 0), (0, 3), (1, 1)):
                    say("batch variant", variant, "order", order, "workers", workers)
                    ctx.reset()
                    b.run(workers=workers, order=order, variant=variant, spin_limit=1 << 16)
                    keys = ctx.flagged()
                    say("  status", ctx.status, "flagged", len(keys))
                    assert ctx.status == 0
                    per = b.split(keys)
                    for i, (w, p) in enumerate(zip(want, per)):
                        assert p == w, (i, specs[i])
            n = ctx.check_count()
    expect = sum(jobs.check_count_arrays(s, a) for s, a in zip(specs, arrays))
    assert n == expect                            # the last run (reset clears the counter)
    say("batch with wave grouping")
    with hr.Context(wave_grouping=True) as ctx:
        with hr.Batch(ctx, [j.inst for j in js]) as b:
            b.run(spin_limit=1 << 16)
            per = b.split(ctx.flagged())
            assert ctx.status == 0
            # the run's own choice over the context's: off, or a coalescing
            # width; and the stencil jobs' shadow map (tiles of 4 x 4, 2 x 8,
            # 16 x 1, then row-major again)
            for coalesce, tile in ((1, None), (2, (2, 2)), (16, (1, 3)), (64, (4, 0)),
                                   (8, None)):
                say("  coalesce", coalesce, "tile", tile)
                ctx.reset()
                b.run(spin_limit=1 << 16, coalesce=coalesce, tile=tile)
                assert ctx.status == 0 and b.split(ctx.flagged()) == per
            ctx.reset()
            with pytest.raises(hr.HRError):
                b.run(coalesce=3)
            with pytest.raises(hr.HRError):
                b.run(tile=(5, 0))
    for i, (w, p) in enumerate(zip(want, per)):
        assert p == w, (i, specs[i])


def test_batch_full_manifest(env):
    """The 1000-job manifest (blocks 1-512, threads 64-1024, LDS 1-64 KiB,
    10 % seeded) in one persistent launch against the oracle's sets of the
    whole jobs (tests/golden/batched_manifest_1000.json) and the closed
    forms, and a sample of jobs against the serial path."""
    torch, hr, jobs = env
    specs = si.batched_manifest(si.master_seed(3))
    golden = load_golden("batched_manifest_1000.json")["jobs"]
    assert [g["index"] for g in golden] == [s["index"] for s in specs]
    say("building 1000 job inputs")
    arrays = [si.instance_inputs(s) for s in specs]
    want = [expected(s, a, use_oracle=False) for s, a in zip(specs, arrays)]
    js = [jobs.Job(s, a) for s, a in zip(specs, arrays)]
    say("batch run")
    with hr.Context(ring_capacity=1 << 20) as ctx:
        with hr.Batch(ctx, [j.inst for j in js]) as b:
            say("  workers", b.info(0), b.info(1))
            for tile in (None, (2, 2), (1, 3)):       # the stencil jobs' shadow maps
                say("  shadow map", tile)
                ctx.reset()
                b.run(spin_limit=1 << 18, tile=tile)
                per = b.split(ctx.flagged())
                say("  status", ctx.status)
                assert ctx.status == 0
                for i, (w, p) in enumerate(zip(want, per)):
                    assert p == w, (i, specs[i], tile)
                # every job's set against the oracle's, run on the whole
                # job by oracle/goldens.py
                for i, (g, p) in enumerate(zip(golden, per)):
                    assert (len(p), key_digest(p)) == (g["flagged"], g["sha256"]), (i, tile)
    rng = np.random.default_rng(1)
    for i in rng.choice(len(js), 12, replace=False):
        got, st = js[int(i)].serial(ring_capacity=1 << 20)
        assert st == 0 and got == want[int(i)]
