"""Selective monitoring on the GPU: threads switched off at run time (device
hr_thread_enable, driven by switch operations of the access interpreter) and
regions switched off from the host (hr_region_enable).  The checker must
flag exactly the races among the monitored accesses: the oracle's set on the
log without the unmonitored accesses, bit for bit."""
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


def run(torch, hr, prog, off_from=None):
    """off_from: {program region: first launch in which it is unmonitored}."""
    data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
    with hr.Context() as ctx:
        regs = [ctx.shadow_alloc(d) for d in data]
        for L, launch in enumerate(prog.launches):
            for pr, first in (off_from or {}).items():
                if L == first:
                    ctx.region_enable(regs[pr], False)
            ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words)
            ctx.kernel_end()
        return ctx.flagged(), ctx.status


@pytest.mark.parametrize("seed,threads,p_switch", [(41, 128, 0.1), (42, 256, 0.3), (43, 64, 0.05)])
def test_switched_off_threads(env, seed, threads, p_switch):
    torch, hr = env
    prog = si.random_program(seed, launches=2, blocks=6, threads=threads, phases=4, max_ops=3,
                             global_regions=2, global_words=128, lds_words=64,
                             p_switch=p_switch)
    want = oracle.flagged_program(prog)
    say("switch ops", seed, threads, p_switch, "oracle flags", len(want))
    got, st = run(torch, hr, prog)
    assert st == 0 and got == want


def test_unmonitored_region(env):
    torch, hr = env
    prog = si.random_program(44, launches=3, blocks=4, threads=128, phases=4, max_ops=2,
                             global_regions=3, global_words=96, lds_words=32)
    log = oracle.model_program(prog)
    full = oracle.flagged(log.copy())
    say("region switched off for the whole job")
    got, st = run(torch, hr, prog, off_from={1: 0})
    assert st == 0
    assert got == {k for k in full if not (k[0] == 0 and k[1] == 1)}
    assert any(k[0] == 0 and k[1] == 1 for k in full)
    say("region switched off from the second launch")
    got, st = run(torch, hr, prog, off_from={2: 1})
    keep = ~((log["space"] == 0) & (log["region"] == 2) & (log["launch"] >= 1))
    assert st == 0 and got == oracle.flagged(np.ascontiguousarray(log[keep]))
