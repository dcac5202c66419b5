"""Serving on the GPU: a Poisson stream of jobs checked with continuous
batching must give, job by job, the same flagged set as each job alone (the
serial path) and as the oracle, whatever the admission pressure (shadow
budget, job slots); tolerance zero.  The stream mixes the batched job mix
with full-size 4096 x 4096 stencil jobs."""
import numpy as np
import pytest

import json
import os

import oracle
import synth_inputs as si
from oracle import closed_forms as cf
from oracle.goldens import key_digest, serving_test_stream

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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
            assert oracle.flagged(oracle.model_reduce_n(spec["n"], spec["threads"],
                                                        spec["blocks"], spec["drop"])) == want
        return want
    if p == si.PAT_JACOBI:
        want = cf.jacobi_flagged(spec["ny"], spec["nx"], spec["phases"], arrays["seeds"])
        if use_oracle and not spec.get("big"):
            assert oracle.flagged(oracle.model_jacobi(spec["ny"], spec["nx"], spec["phases"],
                                                      arrays["seed_tab"])) == want
        return want
    want = cf.labelprop_flagged(arrays["row_ptr"], arrays["col"], arrays["mask"])
    if use_oracle:
        assert oracle.flagged(oracle.model_labelprop(arrays["row_ptr"], arrays["col"],
                                                     arrays["mask"], spec["phases"],
                                                     spec["threads"])) == want
    return want


def shadow_bytes(spec):
    """Shadow bytes the serving executor reserves for a job (256-byte
    granules, one spare)."""
    p = spec["pattern"]
    if p == si.PAT_REDUCE:
        words = spec["blocks"] * (spec["n"] + spec["threads"])
    elif p == si.PAT_JACOBI:
        words = 2 * spec["nx"] * spec["ny"]
    else:
        words = spec["vertices"]
    return ((words + 31) // 32 + 1) * 256


def items_of(spec):
    """Work items (1024-thread blocks) of one phase of a job: its blocks
    packed 1024 / threads to an item."""
    p = spec["pattern"]
    if p == si.PAT_REDUCE:
        blocks, threads = spec["blocks"], spec["threads"]
    elif p == si.PAT_JACOBI:
        blocks, threads = -(-spec["ny"] // 16) * -(-spec["nx"] // 16), 256
    else:
        threads = spec["threads"]
        blocks = -(-spec["vertices"] // threads)
    pack = 1024 // threads
    return -(-blocks // pack)


@pytest.fixture(scope="module")
def stream(env):
    torch, hr, jobs = env
    specs = serving_test_stream()
    say("stream of", len(specs), "jobs,", sum(bool(s.get("big")) for s in specs), "full-size")
    arrays = [si.instance_inputs(s) for s in specs]
    want = [expected(s, a, use_oracle=True) for s, a in zip(specs, arrays)]
    assert sum(bool(w) for w in want) >= 8
    # every job's expected set is the oracle's on the whole job, the
    # full-size stencils included (streamed by oracle/goldens.py)
    with open(os.path.join(GOLDEN, "serving_stream_40.json")) as f:
        golden = json.load(f)["jobs"]
    assert [g["index"] for g in golden] == [s["index"] for s in specs]
    for i, (g, w) in enumerate(zip(golden, want)):
        assert (len(w), key_digest(w)) == (g["flagged"], g["sha256"]), (i, specs[i])
    js = [jobs.Job(s, a) for s, a in zip(specs, arrays)]
    return specs, js, want


def test_serving_each_job_alone_equals_oracle(env, stream):
    torch, hr, jobs = env
    specs, js, want = stream
    for i, (j, w) in enumerate(zip(js, want)):
        got, st = j.serial()
        assert st == 0 and got == w, (i, specs[i])
    say("every job alone matches the oracle")


@pytest.mark.parametrize("budget_jobs,slots,rate", [(0, 0, 2000.0), (3, 4, 5000.0),
                                                    (1, 0, 20000.0), (0, 1, 1000.0)])
def test_serving_mix_equals_alone(env, stream, budget_jobs, slots, rate):
    """Continuous batching under admission pressure: budget_jobs times the
    largest job's shadow (0: the default budget), `slots` resident jobs at
    most (0: default)."""
    torch, hr, jobs = env
    specs, js, want = stream
    big = max(shadow_bytes(s) for s in specs)
    budget = budget_jobs * big
    arrivals = si.poisson_arrivals(7, len(js), rate)
    say("serve budget", budget, "slots", slots, "rate", rate)
    with hr.Context(ring_capacity=1 << 16) as ctx:
        per, times = hr.serve(ctx, [j.inst for j in js], arrivals, shadow_budget=budget,
                              max_slots=slots)
    for i, (w, p) in enumerate(zip(want, per)):
        assert p == w, (i, specs[i])
        t = times[i]
        assert t.status == 0 and t.flagged == len(w)
        assert t.admit_s >= t.arrival_s - 1e-6 and t.finish_s >= t.admit_s
    # admission is in arrival order
    admits = np.array([t.admit_s for t in times])
    assert np.all(np.diff(admits) >= 0)
    lat = np.array([t.finish_s - t.arrival_s for t in times])
    say("  p50 %.3f ms p99 %.3f ms" % (1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99)))


@pytest.mark.parametrize("burst,lane", [(1, 1), (3, 2), (0, 5), (2, 64)])
def test_serving_bursts(env, stream, burst, lane):
    """The large lane runs its stencil jobs one at a time, `burst` phases per
    iteration (0: all of a job's phases in one); the other lanes run `lane`
    phases of their jobs per iteration: the sets do not depend on either,
    and the large jobs finish in admission order."""
    torch, hr, jobs = env
    specs, js, want = stream
    arrivals = si.poisson_arrivals(9, len(js), 5000.0)
    say("serve with large-lane bursts of", burst, "and lane bursts of", lane)
    with hr.Context(ring_capacity=1 << 16) as ctx:
        per, times = hr.serve(ctx, [j.inst for j in js], arrivals, large_burst=burst,
                              lane_burst=lane)
    for i, (w, p) in enumerate(zip(want, per)):
        assert p == w, (i, specs[i])
        assert times[i].status == 0 and times[i].flagged == len(w)
    big = [i for i, s in enumerate(specs) if s.get("big")]
    assert len(big) >= 2
    fin = np.array([times[i].finish_s for i in big])
    assert np.all(np.diff(fin) > 0)


def test_serving_serial_replay(env, stream):
    torch, hr, jobs = env
    specs, js, want = stream
    arrivals = si.poisson_arrivals(8, len(js), 2000.0)
    with hr.Context() as ctx:
        per, times = hr.serve(ctx, [j.inst for j in js], arrivals, serial=True)
    for i, (w, p) in enumerate(zip(want, per)):
        assert p == w, (i, specs[i])
        assert times[i].status == 0 and times[i].flagged == len(w)
    fin = np.array([t.finish_s for t in times])
    assert np.all(np.diff(fin) > 0)                 # one job at a time, in order


def test_serving_rejects_job_over_budget(env, stream):
    torch, hr, jobs = env
    specs, js, want = stream
    small = min(shadow_bytes(s) for s in specs)
    arrivals = np.zeros(len(js))
    with hr.Context() as ctx:
        with pytest.raises(hr.HRError) as e:
            hr.serve(ctx, [j.inst for j in js], arrivals, shadow_budget=small)
        assert e.value.status == hr.HR_E_NOMEM
        arrivals[3], arrivals[2] = 1.0, 2.0         # unsorted arrivals
        with pytest.raises(hr.HRError) as e:
            hr.serve(ctx, [j.inst for j in js], arrivals)
        assert e.value.status == hr.HR_E_INVAL


def test_serving_item_cap(env, stream):
    """An iteration holds at most max_items work items: with the cap at the
    largest job's items, jobs wait for room, the results stay those of each
    job alone, and no two jobs whose items together exceed the cap are ever
    resident together."""
    torch, hr, jobs = env
    specs, js, want = stream
    items = [items_of(s) for s in specs]
    cap = max(items)
    arrivals = si.poisson_arrivals(9, len(js), 5000.0)
    say("serve with item cap", cap, "items per job", sorted(items)[-5:])
    with hr.Context(ring_capacity=1 << 16) as ctx:
        per, times = hr.serve(ctx, [j.inst for j in js], arrivals, max_items=cap)
    for i, (w, p) in enumerate(zip(want, per)):
        assert p == w, (i, specs[i])
        assert times[i].status == 0
    # resident intervals [admit, finish): the items of the jobs resident at
    # any admission never exceed the cap
    iv = [(t.admit_s, t.finish_s) for t in times]
    for i, (a, _) in enumerate(iv):
        resident = sum(items[k] for k, (b, f) in enumerate(iv) if b <= a < f)
        assert resident <= cap, (i, resident)
    say("  item cap held")


def test_serving_item_cap_arguments(env, stream):
    torch, hr, jobs = env
    specs, js, want = stream
    items = [items_of(s) for s in specs]
    arrivals = np.zeros(len(js))
    with hr.Context() as ctx:
        with pytest.raises(hr.HRError) as e:        # a job that can never fit
            hr.serve(ctx, [j.inst for j in js], arrivals, max_items=max(items) - 1)
        assert e.value.status == hr.HR_E_INVAL
        with pytest.raises(hr.HRError) as e:        # above the launch limit
            hr.serve(ctx, [j.inst for j in js], arrivals, max_items=hr.SERVE_MAX_ITEMS + 1)
        assert e.value.status == hr.HR_E_INVAL
        with pytest.raises(hr.HRError) as e:        # more than 64 phases per iteration
            hr.serve(ctx, [j.inst for j in js], arrivals, lane_burst=65)
        assert e.value.status == hr.HR_E_INVAL


@pytest.mark.parametrize("pattern", [si.PAT_LABELPROP, si.PAT_REDUCE, si.PAT_JACOBI])
def test_serving_single_class_stream(env, stream, pattern):
    """A stream of one job class runs in one or two lanes; results equal each
    job alone."""
    torch, hr, jobs = env
    specs, js, want = stream
    pick = [i for i, s in enumerate(specs) if s["pattern"] == pattern]
    assert pick
    arrivals = si.poisson_arrivals(10 + pattern, len(pick), 3000.0)
    say("single-class stream", pattern, len(pick), "jobs")
    with hr.Context(ring_capacity=1 << 16) as ctx:
        per, times = hr.serve(ctx, [js[i].inst for i in pick], arrivals)
    for k, i in enumerate(pick):
        assert per[k] == want[i], (i, specs[i])
        assert times[k].status == 0
