"""Autotuners: of the batched launch (autotune) and of a standalone stencil
job (autotune_stencil).  The batched one times candidate tunings of one
batch on the device and keeps the fastest.  It picks, in turn, the schedule (kernel
variant, queue order, worker count), the shadow map of the stencil jobs'
grids (row-major, or tiles of 4 x 4, 8 x 2, 2 x 8 or 16 x 1 elements) and
the coalescing width of same-word lanes (grouping off, or within segments
of 8, 16 or 64 lanes).  Each trial is a full run of the batch; the results
are the same for every tuning, only the schedule, the shadow lines touched
and the number of atomics differ."""
from __future__ import annotations

import itertools

# shadow maps: (tw, th) = log2 of the tile's width and height; None: row-major
TILES = (None, (2, 2), (3, 1), (1, 3), (4, 0))
# coalescing widths: 1 = grouping off, else lanes per grouping segment
WIDTHS = (1, 8, 16, 64)


def tile_name(tile) -> str:
    return "rowmajor" if tile is None else f"{1 << tile[0]}x{1 << tile[1]}"


def candidates(batch):
    out = []
    for variant in (0, 1):
        max_w, _ = batch.info(variant)
        for order, frac in itertools.product((0, 1), (1.0, 0.5)):
            out.append({"variant": variant, "order": order, "workers": max(1, int(max_w * frac))})
    return out


def key_of(cand) -> str:
    key = "v{variant}_o{order}_w{workers}".format(**cand)
    if "tile" in cand:
        key += "_t" + tile_name(cand["tile"])
    if cand.get("coalesce"):
        key += "_c{coalesce}".format(**cand)
    return key


def autotune(ctx, batch, reps: int = 2, cands=None, tiles=TILES, widths=WIDTHS):
    """Return (best tuning dict, {tuning key: best ms}).  The schedule is
    chosen first over `cands`, then the shadow map for it, then the
    coalescing width for both."""
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
        timings[key_of(cand)] = ms
        return ms

    def best_of(options, base):
        best, best_ms = None, None
        for cand in options:
            ms = trial(dict(base, **cand))
            if best_ms is None or ms < best_ms:
                best, best_ms = dict(base, **cand), ms
        return best, best_ms

    best, best_ms = best_of(cands or candidates(batch), {})
    best, best_ms = best_of([{"tile": t} for t in tiles], best)
    best, best_ms = best_of([{"coalesce": c} for c in widths], best)
    return best, timings


# encodings of the state machine's transition (hr_config flags)
ENCODINGS = (("bits", False), ("table", True), ("table_lds", "lds"))


def autotune_stencil(hr, u, seed_tab, launches, tiles=TILES, encodings=ENCODINGS, reps=3,
                     stream=None):
    """Time one checked stencil job (the grids u[0], u[1], `launches`
    launches, seeded blocks `seed_tab`) under every shadow map in `tiles`
    with the bit-logic transition, and under every transition encoding in
    `encodings` with the row-major map; each trial is `reps` runs of the
    whole job, timed per launch.  Returns (best tuning dict, {tuning key:
    p50 ms per launch}, the flagged set with the grids as regions 0 and 1
    when every trial flagged that same set with a clean status, else None)."""
    import numpy as np
    import torch
    stream = stream or torch.cuda.current_stream()
    timings, sets = {}, []

    def trial(key, ctx_kw, tile):
        with hr.Context(**ctx_kw) as ctx:
            regs = [ctx.shadow_alloc(u[0], tile=tile), ctx.shadow_alloc(u[1], tile=tile)]
            ms = []
            for rep in range(reps + 1):               # the first run warms up
                ctx.reset()
                for L in range(launches):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    ctx.jacobi_check(regs[L % 2], regs[(L + 1) % 2], u[L % 2], u[(L + 1) % 2],
                                     seed_tab)
                    e1.record(stream)
                    ctx.kernel_end()
                    if rep:
                        ms.append((e0, e1))
                recs, st = ctx.report()
            torch.cuda.synchronize()
            timings[key] = float(np.percentile([a.elapsed_time(b) for a, b in ms], 50))
            remap = {regs[0]: 0, regs[1]: 1}
            sets.append((st, {(int(r["space"]),
                               int(r["region"]) if r["space"] else remap[int(r["region"])],
                               int(r["block"]) if r["space"] else 0, int(r["index"]))
                              for r in recs}))

    for tile in tiles:
        trial("map_" + tile_name(tile), {}, tile)
    for name, mode in encodings:
        if mode:
            trial("fsm_" + name, {"fsm_table": mode}, None)
    timings["fsm_bits"] = timings.get("map_rowmajor", timings.get("fsm_bits"))
    best_map = min((k for k in timings if k.startswith("map_")), key=timings.get)
    best_fsm = min((k for k in timings if k.startswith("fsm_") and timings[k] is not None),
                   key=timings.get)
    same = all(st == 0 for st, _ in sets) and all(k == sets[0][1] for _, k in sets)
    best = {"tile": next(t for t in tiles if "map_" + tile_name(t) == best_map),
            "fsm": best_fsm[len("fsm_"):]}
    return best, timings, (sets[0][1] if same else None)
