"""Randomized batched launches on the GPU: manifests of random size and mix,
each run once under a random tuning (kernel variant, queue order, worker
count, shadow map of the stencil jobs, coalescing width); every job's set
must equal its workload's closed form (the forms the oracle's goldens pin),
with a clean status.  Fixed seeds."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu

TILES = (None, (2, 2), (3, 1), (1, 3), (4, 0))


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


@pytest.mark.parametrize("chunk", range(2))
def test_random_batches(env, chunk):
    torch, hr, jobs = env
    for i in range(10):
        seed = 0x24010473 + 100 * chunk + i
        r = np.random.default_rng(seed)
        specs = si.batched_manifest(seed, n_instances=int(r.integers(1, 80)),
                                    max_blocks=int(r.choice([4, 64, 512])),
                                    max_threads=int(r.choice([128, 1024])), max_lds_kib=16.0,
                                    seeded_frac=0.5, jacobi_phases=int(r.integers(1, 9)),
                                    labelprop_phases=int(r.integers(1, 5)))
        arrays = [si.instance_inputs(s) for s in specs]
        want = [expected(s, a) for s, a in zip(specs, arrays)]
        js = [jobs.Job(s, a) for s, a in zip(specs, arrays)]
        grouping = bool(r.random() < 0.5)
        with hr.Context(ring_capacity=1 << 18, wave_grouping=grouping) as ctx:
            with hr.Batch(ctx, [j.inst for j in js]) as b:
                variant = int(r.integers(0, 2))
                max_w, _ = b.info(variant)
                tuning = dict(variant=variant, order=int(r.integers(0, 2)),
                              workers=int(r.integers(1, max_w + 1)),
                              coalesce=int(r.choice([0, 1, 2, 8, 64])),
                              tile=TILES[int(r.integers(0, len(TILES)))])
                print("[case] batch", seed, len(specs), "jobs", tuning, flush=True)
                b.run(spin_limit=1 << 20, **tuning)
                per = b.split(ctx.flagged())
                assert ctx.status == 0, (seed, tuning)
        for k, (w, p) in enumerate(zip(want, per)):
            assert p == w, (seed, k, specs[k], tuning)
