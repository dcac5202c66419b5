"""Autotuner of the batched launch: times candidate tunings of one batch
(kernel variant, queue order, worker count, then coalescing of same-word
lanes for the best of those) on the device and keeps the fastest.  Each
trial is a full run of the batch (the results are the same for every
tuning; only the schedule and the number of atomics differ)."""
from __future__ import annotations

import itertools


def candidates(batch):
    out = []
    for variant in (0, 1):
        max_w, _ = batch.info(variant)
        for order, frac in itertools.product((0, 1), (1.0, 0.5)):
            out.append({"variant": variant, "order": order, "workers": max(1, int(max_w * frac))})
    return out


def autotune(ctx, batch, reps: int = 2, cands=None):
    """Return (best tuning dict, {tuning key: best ms})."""
    import torch
    stream = torch.cuda.current_stream()
    timings = {}

    def trial(cand):
        ms = None
        for _ in range(reps):
            ctx.reset()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            batch.run(**cand)
            e1.record(stream)
            e1.synchronize()
            t = e0.elapsed_time(e1)
            ms = t if ms is None else min(ms, t)
        key = "v{variant}_o{order}_w{workers}".format(**cand)
        if cand.get("coalesce"):
            key += "_c{coalesce}".format(**cand)
        timings[key] = ms
        return ms

    best, best_ms = None, None
    for cand in cands or candidates(batch):
        ms = trial(cand)
        if best_ms is None or ms < best_ms:
            best, best_ms = cand, ms
    # coalescing of same-word lanes, off and on, for the best schedule
    for c in (1, 2):
        cand = dict(best, coalesce=c)
        ms = trial(cand)
        if ms < best_ms:
            best, best_ms = cand, ms
    return best, timings
