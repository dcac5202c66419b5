"""Randomized serving on the GPU: streams of random size and mix (reductions,
small stencils, label propagation, and mid-size stencils that take the
large-job lane), random arrival rates, shadow budgets, slot limits and
bursts; every job's served set must equal its workload's closed form (the
forms the oracle's goldens pin), with a clean status.  Fixed seeds."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_04701_amd import hr, jobs
    torch.cuda.set_device(0)
    return torch, hr, jobs


def expected(spec, a):
    p = spec["pattern"]
    if p == si.PAT_REDUCE:
        return cf.reduce_n_flagged(spec["n"], spec["threads"], spec["blocks"], spec["drop"])
    if p == si.PAT_JACOBI:
        return cf.jacobi_flagged(spec["ny"], spec["nx"], spec["phases"], a["seeds"])
    return cf.labelprop_flagged(a["row_ptr"], a["col"], a["mask"])


@pytest.mark.parametrize("chunk", range(3))
def test_random_streams(env, chunk):
    torch, hr, jobs = env
    served = 0
    for i in range(10):
        seed = 0x24010474 + 100 * chunk + i
        r = np.random.default_rng(seed)
        nj = int(r.integers(5, 40))
        side = int(r.choice([1040, 1296]))
        specs = si.serving_stream(seed, n_jobs=nj, big_frac=float(r.choice([0.0, 0.1, 0.2])),
                                  big_side=side, big_phases=int(r.integers(1, 6)),
                                  max_blocks=int(r.choice([4, 32, 300])),
                                  max_threads=int(r.choice([256, 1024])), max_lds_kib=8.0,
                                  seeded_frac=0.5, jacobi_phases=int(r.integers(1, 9)),
                                  labelprop_phases=int(r.integers(1, 5)))
        arrays = [si.instance_inputs(s) for s in specs]
        want = [expected(s, a) for s, a in zip(specs, arrays)]
        js = [jobs.Job(s, a) for s, a in zip(specs, arrays)]
        arrivals = si.poisson_arrivals(seed, nj, float(r.choice([100.0, 2000.0, 50000.0])))
        big = 2 * side * side * 8 + 4096
        opts = dict(shadow_budget=int(r.choice([3 * big, 64 << 30])),
                    max_slots=int(r.choice([0, 1, 3])), large_burst=int(r.integers(0, 4)),
                    lane_burst=int(r.integers(0, 6)))
        print("[case] stream", seed, nj, "jobs", opts, flush=True)
        with hr.Context(ring_capacity=1 << 16) as ctx:
            per, times = hr.serve(ctx, [j.inst for j in js], arrivals, **opts)
        for k, (w, p) in enumerate(zip(want, per)):
            assert p == w and times[k].status == 0, (seed, k, specs[k], opts)
        served += nj
    assert served > 0
