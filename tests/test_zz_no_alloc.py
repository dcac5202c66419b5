"""hr_job_run_static, the allocation-free serial path, against hr_job_run
(the existing entry point) and the oracle: the same flagged keys and warning
bits, called several times in a row on the one static scratch array, each
later call with a smaller input than the one before it, so that anything a
call leaves behind in the array would show up as a spurious race."""
import ctypes

import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_04701_amd import hr
    torch.cuda.set_device(0)
    return torch, hr


def say(*a):
    print("[case]", *a, flush=True)


def jacobi_job(torch, hr, ny, nx, phases, n_seeds, seed):
    seeds = si.jacobi_seeds(ny, nx, seed, count=n_seeds) if n_seeds else np.zeros((0, 3), np.int32)
    tab = si.jacobi_seed_table(ny, nx, seeds) if len(seeds) else None
    tens = [torch.from_numpy(si.jacobi_grid(ny, nx, seed)).cuda(),
            torch.zeros((ny, nx), dtype=torch.float32, device="cuda"),
            None if tab is None else torch.from_numpy(tab).cuda()]
    inst = hr.Instance()
    inst.pattern, inst.phases, inst.n, inst.ny, inst.drop = hr.HR_PAT_JACOBI, phases, nx, ny, -1
    for i, t in enumerate(tens):
        inst.data[i] = None if t is None else t.data_ptr()
    want = oracle.flagged(oracle.model_jacobi(ny, nx, phases, tab))
    return inst, tens, want


def reduce_job(torch, hr, n, threads, blocks, drop, seed):
    rng = np.random.default_rng(seed)
    tens = [torch.from_numpy(rng.integers(0, 1 << 20, n * blocks).astype(np.int32)).cuda(),
            torch.zeros(threads * blocks, dtype=torch.int32, device="cuda")]
    inst = hr.Instance()
    inst.pattern, inst.phases, inst.n, inst.threads, inst.blocks = hr.HR_PAT_REDUCE, 1, n, \
        threads, blocks
    inst.drop = drop
    inst.data[0], inst.data[1] = tens[0].data_ptr(), tens[1].data_ptr()
    want = oracle.flagged(oracle.model_reduce_n(n, threads, blocks, drop))
    return inst, tens, want


def labelprop_job(torch, hr, v, e, phases, seed):
    src, dst = si.rmat_folded(v, e, seed)
    row_ptr, col = si.csr_by_source(src, dst, v)
    mask = si.seeded_edge_mask(e, 0.02, seed)
    tens = [torch.arange(v, dtype=torch.int32, device="cuda"), torch.from_numpy(row_ptr).cuda(),
            torch.from_numpy(col).cuda(), torch.from_numpy(mask).cuda()]
    inst = hr.Instance()
    inst.pattern, inst.phases, inst.n, inst.threads, inst.drop = hr.HR_PAT_LABELPROP, phases, v, \
        256, -1
    for i, t in enumerate(tens):
        inst.data[i] = t.data_ptr()
    want = oracle.flagged(oracle.model_labelprop(row_ptr, col, mask, phases, 256))
    return inst, tens, want


def run_both(hr, inst, want, **kw):
    """Static path == allocating path == oracle, keys and warning bits."""
    got_s, st_s = hr.job_run(inst, static=True, **kw)
    got_a, st_a = hr.job_run(inst, **kw)
    assert got_s == got_a and st_s == st_a, (len(got_s), len(got_a), st_s, st_a)
    assert got_s == want, (len(got_s), len(want))
    return st_s


def test_static_job_matches_allocating_path(env):
    torch, hr = env
    # larger seeded stencil first, then smaller jobs on the same array
    say("static: jacobi 200x168 x4 seeded")
    inst, keep, want = jacobi_job(torch, hr, 200, 168, 4, 9, 101)
    assert len(want) > 0
    assert run_both(hr, inst, want) == 0
    say("static: jacobi 72x40 x3 race-free after the seeded one")
    inst, keep, want = jacobi_job(torch, hr, 72, 40, 3, 0, 102)
    assert want == set()
    assert run_both(hr, inst, want) == 0
    say("static: reduce n=256 t=128 b=5 drop 2")
    inst, keep, want = reduce_job(torch, hr, 256, 128, 5, 2, 103)
    assert len(want) > 0
    assert run_both(hr, inst, want) == 0
    say("static: labelprop 2000 vertices x2")
    inst, keep, want = labelprop_job(torch, hr, 2000, 16000, 2, 104)
    assert len(want) > 0
    assert run_both(hr, inst, want) == 0
    torch.cuda.synchronize()


def test_static_job_recovers_dropped_records(env):
    """A tiny ring and a site limit: the global part of the set comes back
    from the race words, in ring-sized chunks, as in hr_report."""
    torch, hr = env
    say("static: jacobi 64x56 x2 seeded, ring 4")
    inst, keep, want = jacobi_job(torch, hr, 64, 56, 2, 6, 105)
    assert len(want) > 4
    st = run_both(hr, inst, want, ring_capacity=4)
    assert st & hr.HR_W_RING_OVERFLOW
    say("static: jacobi 48x40 x2 seeded, site limit 1")
    inst, keep, want = jacobi_job(torch, hr, 48, 40, 2, 4, 106)
    st = run_both(hr, inst, want, site_limit=1)
    assert st & hr.HR_W_REPORT_LIMITED
    torch.cuda.synchronize()


def test_static_job_rejects_what_does_not_fit(env):
    torch, hr = env
    dummy = torch.zeros(16, dtype=torch.int32, device="cuda")
    inst = hr.Instance()
    inst.pattern, inst.phases, inst.n, inst.ny = hr.HR_PAT_JACOBI, 1, 4096, 4096
    inst.data[0] = inst.data[1] = dummy.data_ptr()     # never touched: rejected on the host
    n = ctypes.c_size_t(0)
    out = np.zeros(4, dtype=hr.RACE_DTYPE)
    cfg = hr._Config(0, 0, 0, 0, 0, 0, 0)
    st = hr.lib().hr_job_run_static(ctypes.byref(inst), ctypes.byref(cfg),
                                    out.ctypes.data_as(ctypes.c_void_p), 4, ctypes.byref(n), None)
    assert st == hr.HR_E_NOMEM
    assert 2 * 4096 * 4096 > hr.HR_STATIC_SHADOW_WORDS
    cfg = hr._Config(0, 0, 0, hr.HR_CFG_WORD4, 0, 0, 0)
    inst.n = inst.ny = 32
    st = hr.lib().hr_job_run_static(ctypes.byref(inst), ctypes.byref(cfg),
                                    out.ctypes.data_as(ctypes.c_void_p), 4, ctypes.byref(n), None)
    assert st == hr.HR_E_INVAL
