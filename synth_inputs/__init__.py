"""Seeded synthetic inputs shared by the oracle and the HIP race checker.

This module holds no part of the race-check arithmetic.  It only draws
random numbers and lays out workload inputs as plain arrays: the data of the
three workloads (tree reduction, Jacobi stencil, label propagation), the
seeded race-injection tables, R-MAT graphs in CSR form, and tiny barrier
programs for the access-program interpreter.  Both sides read these arrays
and interpret them independently.

Master seed of workload configuration c is ``0x24010470 + c``.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

MASTER_SEED_BASE = 0x24010470


def master_seed(config: int) -> int:
    return MASTER_SEED_BASE + int(config)


# --------------------------------------------------------------------------
# Workload 0: one-block LDS tree reduction of 512 int32 over 9 barrier steps.
# --------------------------------------------------------------------------
REDUCE_N = 512
REDUCE_THREADS = 256
REDUCE_STEPS = 9


def reduce_input(seed: int) -> np.ndarray:
    """int32[512] drawn uniformly from [0, 2^20)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << 20, size=REDUCE_N, dtype=np.int64).astype(np.int32)


# --------------------------------------------------------------------------
# Workload 1: 5-point Jacobi stencil on an ny x nx fp32 grid, 16x16 blocks.
# --------------------------------------------------------------------------
JACOBI_BS = 16
SIDE_N, SIDE_S, SIDE_W, SIDE_E = 0, 1, 2, 3


def jacobi_grid(ny: int, nx: int, seed: int) -> np.ndarray:
    """fp32 (ny, nx) grid drawn uniformly from [0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.random((ny, nx), dtype=np.float32)


def jacobi_blocks(ny: int, nx: int):
    bs = JACOBI_BS
    return (ny + bs - 1) // bs, (nx + bs - 1) // bs


def _seed_options(ny: int, nx: int, bx: int, by: int):
    """(side, offset) pairs whose writer thread and target cell lie in the grid."""
    bs = JACOBI_BS
    y0, x0 = by * bs, bx * bs
    out = []
    for o in range(bs):
        # north: writer (ty=0, tx=o) at (y0, x0+o); target (y0-1, x0+o)
        if y0 - 1 >= 0 and y0 < ny and x0 + o < nx:
            out.append((SIDE_N, o))
        # south: writer (ty=15, tx=o) at (y0+15, x0+o); target (y0+16, x0+o)
        if y0 + bs < ny and x0 + o < nx:
            out.append((SIDE_S, o))
        # west: writer (ty=o, tx=0) at (y0+o, x0); target (y0+o, x0-1)
        if x0 - 1 >= 0 and x0 < nx and y0 + o < ny:
            out.append((SIDE_W, o))
        # east: writer (ty=o, tx=15) at (y0+o, x0+15); target (y0+o, x0+16)
        if x0 + bs < nx and y0 + o < ny:
            out.append((SIDE_E, o))
    return out


def jacobi_seeds(ny: int, nx: int, seed: int, frac: float = 0.001,
                 count: int | None = None) -> np.ndarray:
    """Seeded race injection for the stencil.

    Returns int32 (k, 3) rows ``(block_linear, side, offset)``: block
    ``block_linear = by * nbx + bx`` also writes the neighbour-owned halo cell
    on ``side`` at position ``offset`` along that side, every launch.
    ``k = round(frac * nblocks)`` unless ``count`` is given.
    """
    nby, nbx = jacobi_blocks(ny, nx)
    nb = nby * nbx
    k = int(round(frac * nb)) if count is None else int(count)
    rng = np.random.default_rng(seed ^ 0x5EED)
    rows = []
    if k <= 0:
        return np.zeros((0, 3), dtype=np.int32)
    order = rng.permutation(nb)
    for b in order:
        by, bx = divmod(int(b), nbx)
        opts = _seed_options(ny, nx, bx, by)
        if not opts:
            continue
        side, off = opts[int(rng.integers(0, len(opts)))]
        rows.append((int(b), side, off))
        if len(rows) == k:
            break
    rows.sort()
    return np.asarray(rows, dtype=np.int32).reshape(-1, 3)


def jacobi_seed_table(ny: int, nx: int, seeds: np.ndarray) -> np.ndarray:
    """Per-block int32 table: -1, or ``side << 8 | offset`` for seeded blocks."""
    nby, nbx = jacobi_blocks(ny, nx)
    tab = np.full(nby * nbx, -1, dtype=np.int32)
    for b, side, off in np.asarray(seeds).reshape(-1, 3):
        tab[int(b)] = (int(side) << 8) | int(off)
    return tab


# --------------------------------------------------------------------------
# Workload 2: label propagation over an R-MAT graph in CSR form.
# --------------------------------------------------------------------------
RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def rmat_edges(scale: int, n_edges: int, seed: int,
               abc=(0.57, 0.19, 0.19)):
    """Directed R-MAT edges (no noise, no permutation; self loops and
    duplicates kept).  Returns (src, dst) uint32 arrays."""
    a, b, c = abc
    rng = np.random.default_rng(seed)
    src = np.zeros(n_edges, dtype=np.uint32)
    dst = np.zeros(n_edges, dtype=np.uint32)
    t_ab = np.float32(a + b)
    t_a = np.float32(a)
    t_abc = np.float32(a + b + c)
    for level in range(scale):
        u = rng.random(n_edges, dtype=np.float32)
        sbit = (u >= t_ab).astype(np.uint32)                 # quadrants c, d
        dbit = (((u >= t_a) & (u < t_ab)) | (u >= t_abc)).astype(np.uint32)  # b, d
        shift = np.uint32(scale - 1 - level)
        src |= sbit << shift
        dst |= dbit << shift
    return src, dst


def csr_by_source(src: np.ndarray, dst: np.ndarray, n_vertices: int):
    """Stable CSR by source vertex: (row_ptr int32[n+1], col int32[m])."""
    order = np.argsort(src, kind="stable")
    col = dst[order].astype(np.int32)
    counts = np.bincount(src, minlength=n_vertices).astype(np.int64)
    row_ptr = np.zeros(n_vertices + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    return row_ptr.astype(np.int32), col


def seeded_edge_mask(n_edges: int, p: float, seed: int) -> np.ndarray:
    """uint8 Bernoulli(p) mask over CSR edge positions."""
    rng = np.random.default_rng(seed ^ 0xED6E)
    return (rng.random(n_edges, dtype=np.float64) < p).astype(np.uint8)


def labelprop_graph(scale: int, n_edges: int, seed: int, p_seed: float):
    """R-MAT graph in CSR plus its seeded-edge mask."""
    src, dst = rmat_edges(scale, n_edges, seed)
    row_ptr, col = csr_by_source(src, dst, 1 << scale)
    mask = seeded_edge_mask(n_edges, p_seed, seed)
    return row_ptr, col, mask


# --------------------------------------------------------------------------
# Barrier programs for the access-program interpreter.
#
# A program is a list of launches.  A launch has ``blocks`` blocks of
# ``threads`` threads and a list of phases.  In each phase every thread runs
# its own list of memory operations, then the phase ends with
#   scope 0: nothing,
#   scope 1: a wave-scope barrier in the waves whose bit is set in wave_mask,
#   scope 2: a block-scope barrier in every thread of the block.
# Operation word (uint32):
#   bits  0..23  element index
#   bits 24..26  region (global regions 0..7; LDS uses region 0)
#   bits 27..28  kind: 0 plain read, 1 plain write, 2 atomic, 3 switch the
#                thread's monitoring off (bit 0 clear) or on (bit 0 set)
#   bit  29      space: 0 global, 1 LDS
# op_off has phases*blocks*threads+1 entries; the operations of
# (phase p, block b, thread t) are ops[op_off[i]:op_off[i+1]] with
# i = (p * blocks + b) * threads + t.
# --------------------------------------------------------------------------
KIND_R, KIND_W, KIND_A = 0, 1, 2
KIND_SWITCH = 3          # not an access: switches the thread's monitoring off / on
SPACE_GLOBAL, SPACE_LDS = 0, 1
SCOPE_NONE, SCOPE_WAVE, SCOPE_BLOCK = 0, 1, 2
SCOPE_TILE = 3           # a tile barrier, in the tiles whose bit is set in wave_mask


def op_word(space: int, region: int, kind: int, index: int) -> int:
    assert 0 <= index < (1 << 24) and 0 <= region < 8 and kind in (0, 1, 2)
    return (index | (region << 24) | (kind << 27) | (space << 29)) & 0xFFFFFFFF


def switch_word(on: bool) -> int:
    """Operation that switches the thread's monitoring off or on."""
    return (int(bool(on)) | (KIND_SWITCH << 27)) & 0xFFFFFFFF


def op_fields(word: int):
    """(space, region, kind, index) of an operation word."""
    w = int(word)
    return (w >> 29) & 1, (w >> 24) & 7, (w >> 27) & 3, w & 0xFFFFFF


@dataclasses.dataclass
class Launch:
    blocks: int
    threads: int
    scope: np.ndarray       # uint8[phases]
    wave_mask: np.ndarray   # uint64[phases]
    op_off: np.ndarray      # int32[phases*blocks*threads + 1]
    ops: np.ndarray         # uint32[...]

    @property
    def phases(self) -> int:
        return int(self.scope.shape[0])

    def thread_ops(self, phase: int, block: int, thread: int) -> np.ndarray:
        i = (phase * self.blocks + block) * self.threads + thread
        return self.ops[self.op_off[i]:self.op_off[i + 1]]


@dataclasses.dataclass
class Program:
    launches: List[Launch]
    global_words: List[int]   # element count of each global region
    lds_words: int            # element count of the LDS array


def build_launch(blocks, threads, scopes, wave_masks, per_thread_ops) -> Launch:
    """per_thread_ops[p][b][t] is a list of operation words."""
    offs = [0]
    flat = []
    for p in range(len(scopes)):
        for b in range(blocks):
            for t in range(threads):
                lst = per_thread_ops[p][b][t]
                flat.extend(lst)
                offs.append(len(flat))
    return Launch(blocks=blocks, threads=threads,
                  scope=np.asarray(scopes, dtype=np.uint8),
                  wave_mask=np.asarray(wave_masks, dtype=np.uint64),
                  op_off=np.asarray(offs, dtype=np.int32),
                  ops=np.asarray(flat, dtype=np.uint32))


def random_program(seed: int, launches: int = 2, blocks: int = 2,
                   threads: int = 128, phases: int = 3, max_ops: int = 2,
                   global_regions: int = 2, global_words: int = 64,
                   lds_words: int = 64, p_lds: float = 0.3,
                   kind_p=(0.5, 0.25, 0.25), scope_p=(0.3, 0.3, 0.4),
                   p_active: float = 1.0, wave_width: int = 64,
                   p_switch: float = 0.0, tile_width: int = 0) -> Program:
    """Random barrier program.  Addresses are drawn from small ranges so that
    conflicting accesses from different threads are common.  Every thread of
    a block sees the same phase structure, so barriers are uniform.
    wave_width only shapes the wave masks of wave-barrier phases.  A share
    p_switch of the operations switch the thread's monitoring off or on.
    tile_width > 0: scope_p has a fourth entry, the share of phases ending
    with a tile barrier (tiles of tile_width lanes nested in the waves), whose
    mask selects tiles."""
    rng = np.random.default_rng(seed)
    waves = min(64, (threads + wave_width - 1) // wave_width)
    tiles = min(64, (threads + tile_width - 1) // tile_width) if tile_width else 0
    out = []
    kind_p = np.asarray(kind_p, dtype=np.float64)
    for _ in range(launches):
        scopes = rng.choice(4 if tile_width else 3, size=phases, p=scope_p).astype(np.uint8)
        masks = np.zeros(phases, dtype=np.uint64)
        for p in range(phases):
            if scopes[p] in (SCOPE_WAVE, SCOPE_TILE):
                groups = waves if scopes[p] == SCOPE_WAVE else tiles
                bits = rng.random(groups) < 0.7
                m = 0
                for w in np.nonzero(bits)[0]:
                    m |= 1 << int(w)
                masks[p] = m
        n_slots = phases * blocks * threads
        counts = rng.integers(0, max_ops + 1, size=n_slots)
        counts[rng.random(n_slots) >= p_active] = 0
        total = int(counts.sum())
        kinds = rng.choice(3, size=total, p=kind_p).astype(np.uint32)
        lds = rng.random(total) < p_lds
        regions = rng.integers(0, global_regions, size=total).astype(np.uint32)
        gidx = rng.integers(0, global_words, size=total).astype(np.uint32)
        lidx = rng.integers(0, lds_words, size=total).astype(np.uint32)
        index = np.where(lds, lidx, gidx)
        regions = np.where(lds, 0, regions).astype(np.uint32)
        ops = (index | (regions << 24) | (kinds << 27)
               | (lds.astype(np.uint32) << 29)).astype(np.uint32)
        if p_switch > 0:
            sw = rng.random(total) < p_switch
            on = rng.integers(0, 2, size=total).astype(np.uint32)
            ops = np.where(sw, on | np.uint32(KIND_SWITCH << 27), ops).astype(np.uint32)
        op_off = np.zeros(n_slots + 1, dtype=np.int64)
        np.cumsum(counts, out=op_off[1:])
        out.append(Launch(blocks=blocks, threads=threads, scope=scopes,
                          wave_mask=masks, op_off=op_off.astype(np.int32),
                          ops=ops))
    return Program(launches=out, global_words=[global_words] * global_regions,
                   lds_words=lds_words)


def tile_reduce_program(tile: int, blocks: int, threads: int, drop: int = -1) -> Program:
    """Wave-synchronous (sub-wave) tree reduction as an access program.

    Every tile of `tile` lanes (a power of two) owns an LDS segment of
    n = 2 * tile int32 words at tile_index * n.  Lane l of a tile reads the
    global input words l and l + tile of its segment (region 0, laid out
    like the LDS) and stores them to the segment, then runs log2(n) halving
    steps: in step s lanes l < h = n >> (s+1) read seg[l] and seg[l+h] and
    write seg[l], and each step ends with a tile barrier (a wave-scope barrier
    in every tile, with tiles as the synchronization groups) unless s ==
    drop.  Finally every lane reads seg[0] and writes global out[b*threads +
    t] (region 1).  One launch."""
    assert tile >= 2 and tile & (tile - 1) == 0 and threads % tile == 0
    tiles = threads // tile
    assert tiles <= 64, "the wave mask holds 64 groups"
    n = 2 * tile
    steps = n.bit_length() - 1
    mask = (1 << tiles) - 1
    per = [[[[] for _ in range(threads)] for _ in range(blocks)] for _ in range(steps + 1)]
    for b in range(blocks):
        for t in range(threads):
            l, base = t % tile, (t // tile) * n
            gbase = b * threads * 2 + base
            ops0 = per[0][b][t]
            for j in (l, l + tile):
                ops0.append(op_word(SPACE_GLOBAL, 0, KIND_R, gbase + j))
                ops0.append(op_word(SPACE_LDS, 0, KIND_W, base + j))
            for st in range(steps):
                h = n >> (st + 1)
                if l < h:
                    per[st][b][t] += [op_word(SPACE_LDS, 0, KIND_R, base + l),
                                      op_word(SPACE_LDS, 0, KIND_R, base + l + h),
                                      op_word(SPACE_LDS, 0, KIND_W, base + l)]
            per[steps][b][t] += [op_word(SPACE_LDS, 0, KIND_R, base),
                                 op_word(SPACE_GLOBAL, 1, KIND_W, b * threads + t)]
    scopes = [SCOPE_NONE if st == drop else SCOPE_WAVE for st in range(steps)] + [SCOPE_NONE]
    masks = [mask if sc == SCOPE_WAVE else 0 for sc in scopes]
    launch = build_launch(blocks, threads, scopes, masks, per)
    return Program([launch], [blocks * threads * 2, blocks * threads], 2 * threads)


def nested_reduce_program(tile: int, waves: int, blocks: int, drop_tile: int = -1,
                          drop_wave: int = -1, wave: int = 64) -> Program:
    """Two-level wave-synchronous reduction with tiles nested in waves, as an
    access program (tile barriers: scope 3; wave barriers: scope 1).

    Stage 1, per tile of `tile` lanes (a power of two): lane l reads global
    input words l and l + tile of its tile's segment (region 0) and stores
    them to its LDS segment of 2 * tile words, then log2(2 * tile) halving
    steps (lanes l < h read seg[l] and seg[l + h], write seg[l]), each ended
    by a tile barrier in every tile unless step == drop_tile.  Stage 2, per
    wave of `wave` lanes: lane 0 of each tile reads its segment's seg[0] and
    writes it to the wave's slot array (T = wave / tile slots, after all
    segments), then a wave barrier; log2(T) halving steps over the slots
    (lanes l < h read slot[l], slot[l + h], write slot[l]), each ended by a
    wave barrier unless step == drop_wave.  Finally every lane reads slot 0
    of its wave and writes global out[b * threads + t] (region 1).  One
    launch; threads = waves * wave."""
    assert tile >= 2 and tile & (tile - 1) == 0 and wave % tile == 0 and wave <= 64
    T = wave // tile
    assert T >= 2 and T & (T - 1) == 0
    threads = waves * wave
    tiles = threads // tile
    assert tiles <= 64, "the barrier mask holds 64 groups"
    n = 2 * tile
    s1 = n.bit_length() - 1
    s2 = T.bit_length() - 1
    seg_words = tiles * n
    phases = 1 + s1 + 1 + s2 + 1
    per = [[[[] for _ in range(threads)] for _ in range(blocks)] for _ in range(phases)]
    for b in range(blocks):
        for t in range(threads):
            l, g = t % tile, t // tile
            base, gbase = g * n, b * threads * 2 + g * n
            w, lw = t // wave, t % wave
            slots = seg_words + w * T
            ph = per[0][b][t]
            for j in (l, l + tile):
                ph.append(op_word(SPACE_GLOBAL, 0, KIND_R, gbase + j))
                ph.append(op_word(SPACE_LDS, 0, KIND_W, base + j))
            for st in range(s1):
                h = n >> (st + 1)
                if l < h:
                    per[1 + st][b][t] += [op_word(SPACE_LDS, 0, KIND_R, base + l),
                                          op_word(SPACE_LDS, 0, KIND_R, base + l + h),
                                          op_word(SPACE_LDS, 0, KIND_W, base + l)]
            if l == 0:
                per[1 + s1][b][t] += [op_word(SPACE_LDS, 0, KIND_R, base),
                                      op_word(SPACE_LDS, 0, KIND_W, slots + (g % T))]
            for st in range(s2):
                h = T >> (st + 1)
                if lw < h:
                    per[2 + s1 + st][b][t] += [op_word(SPACE_LDS, 0, KIND_R, slots + lw),
                                               op_word(SPACE_LDS, 0, KIND_R, slots + lw + h),
                                               op_word(SPACE_LDS, 0, KIND_W, slots + lw)]
            per[phases - 1][b][t] += [op_word(SPACE_LDS, 0, KIND_R, slots),
                                      op_word(SPACE_GLOBAL, 1, KIND_W, b * threads + t)]
    all_tiles, all_waves = (1 << tiles) - 1, (1 << waves) - 1
    # the loads end with a tile barrier, each tile step with one (unless
    # dropped), the slot writes with a wave barrier, each wave step with one
    # (unless dropped); the final reads and writes end with nothing
    scopes = ([SCOPE_TILE] + [SCOPE_NONE if st == drop_tile else SCOPE_TILE for st in range(s1)] +
              [SCOPE_WAVE] + [SCOPE_NONE if st == drop_wave else SCOPE_WAVE for st in range(s2)] +
              [SCOPE_NONE])
    masks = [all_tiles if sc == SCOPE_TILE else (all_waves if sc == SCOPE_WAVE else 0)
             for sc in scopes]
    assert len(scopes) == phases
    launch = build_launch(blocks, threads, scopes, masks, per)
    return Program([launch], [blocks * threads * 2, blocks * threads], seg_words + waves * T)


# --------------------------------------------------------------------------
# Batched jobs: a manifest of independent checked jobs of mixed patterns.
# --------------------------------------------------------------------------
PAT_REDUCE, PAT_JACOBI, PAT_LABELPROP = 0, 1, 2


def _log_uniform(rng, lo: float, hi: float) -> float:
    return float(np.exp(rng.uniform(np.log(lo), np.log(hi))))


def batched_manifest(seed: int, n_instances: int = 1000, max_blocks: int = 512,
                     min_threads: int = 64, max_threads: int = 1024, max_lds_kib: float = 64.0,
                     seeded_frac: float = 0.1, jacobi_phases: int = 20,
                     labelprop_phases: int = 10):
    """Job specs: pattern uniform over (reduce, jacobi, labelprop); blocks
    log-uniform in [1, max_blocks]; threads log-uniform in [min_threads,
    max_threads] rounded to a multiple of 64; LDS log-uniform in [1,
    max_lds_kib] KiB; a seeded_frac share of jobs carries its pattern's
    seeded race.  Scaled sizes:
      reduce:    n = largest power of two <= min(LDS words, 2 * threads);
                 the seeded variant drops one step's barrier;
      jacobi:    a square grid of side 16 * ceil(sqrt(blocks)), 256-thread
                 blocks, `jacobi_phases` launches, one seeded block;
      labelprop: V = blocks * threads vertices, 8 V edges, `labelprop_phases`
                 launches, 1 % of the edges seeded.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_instances):
        pattern = int(rng.integers(0, 3))
        blocks = max(1, int(round(_log_uniform(rng, 1, max_blocks))))
        threads = 64 * max(1, int(round(_log_uniform(rng, min_threads, max_threads) / 64)))
        lds_kib = _log_uniform(rng, 1.0, max_lds_kib)
        seeded = bool(rng.random() < seeded_frac)
        iseed = int(rng.integers(0, 2 ** 31 - 1))
        spec = {"index": i, "pattern": pattern, "blocks": blocks, "threads": threads,
                "lds_kib": lds_kib, "seeded": seeded, "seed": iseed}
        if pattern == PAT_REDUCE:
            words = int(lds_kib * 1024) // 4
            n = 1 << int(np.floor(np.log2(max(2, min(words, 2 * threads)))))
            steps = n.bit_length() - 1
            drop = int(np.random.default_rng(iseed).integers(0, steps)) if seeded else -1
            spec.update(n=n, drop=drop, phases=1)
        elif pattern == PAT_JACOBI:
            g = int(np.ceil(np.sqrt(blocks)))
            spec.update(ny=16 * g, nx=16 * g, phases=jacobi_phases, threads=256, blocks=g * g)
        else:
            v = blocks * threads
            spec.update(vertices=v, edges=8 * v, phases=labelprop_phases,
                        p_seed=0.01 if seeded else 0.0)
        specs.append(spec)
    return specs


def rmat_folded(n_vertices: int, n_edges: int, seed: int):
    """R-MAT edges at scale ceil(log2 n_vertices), vertex ids folded into
    [0, n_vertices) modulo n_vertices."""
    scale = max(1, int(np.ceil(np.log2(n_vertices))))
    src, dst = rmat_edges(scale, n_edges, seed)
    return (src % np.uint32(n_vertices)).astype(np.uint32), \
           (dst % np.uint32(n_vertices)).astype(np.uint32)


def instance_inputs(spec):
    """Host arrays of one job of a batched manifest."""
    seed = spec["seed"]
    if spec["pattern"] == PAT_REDUCE:
        rng = np.random.default_rng(seed)
        n, b, t = spec["n"], spec["blocks"], spec["threads"]
        return {"in": rng.integers(0, 1 << 20, size=n * b, dtype=np.int64).astype(np.int32),
                "out": np.zeros(b * t, dtype=np.int32)}
    if spec["pattern"] == PAT_JACOBI:
        ny, nx = spec["ny"], spec["nx"]
        if not spec["seeded"]:
            seeds = np.zeros((0, 3), np.int32)
        elif "seed_frac" in spec:
            seeds = jacobi_seeds(ny, nx, seed, frac=spec["seed_frac"])
        else:
            seeds = jacobi_seeds(ny, nx, seed, count=1)
        return {"u0": jacobi_grid(ny, nx, seed), "u1": np.zeros((ny, nx), np.float32),
                "seeds": seeds,
                "seed_tab": jacobi_seed_table(ny, nx, seeds) if len(seeds) else None}
    v, e = spec["vertices"], spec["edges"]
    src, dst = rmat_folded(v, e, seed)
    row_ptr, col = csr_by_source(src, dst, v)
    mask = seeded_edge_mask(e, spec["p_seed"], seed) if spec["seeded"] else np.zeros(e, np.uint8)
    return {"label": np.arange(v, dtype=np.int32), "row_ptr": row_ptr, "col": col, "mask": mask}


# --------------------------------------------------------------------------
# Serving stream: the batched mix plus a share of full-size stencil jobs,
# arriving as a Poisson process.
# --------------------------------------------------------------------------
def serving_stream(seed: int, n_jobs: int = 2000, big_frac: float = 0.05, big_side: int = 4096,
                   big_phases: int = 20, big_seed_frac: float = 0.001, **manifest_kw):
    """Job specs in arrival order: round(big_frac * n_jobs) full-size Jacobi
    jobs (big_side^2 grid, big_phases launches, big_seed_frac of the blocks
    seeded) at seeded random positions; every other job is drawn as in
    batched_manifest (keyword arguments are passed on to it)."""
    rng = np.random.default_rng(seed)
    n_big = int(round(big_frac * n_jobs))
    big_at = set(int(i) for i in rng.choice(n_jobs, n_big, replace=False)) if n_big else set()
    small = iter(batched_manifest(seed ^ 0x5E2F, n_instances=n_jobs - n_big, **manifest_kw))
    g = (big_side + JACOBI_BS - 1) // JACOBI_BS
    specs = []
    for i in range(n_jobs):
        if i in big_at:
            spec = {"pattern": PAT_JACOBI, "ny": big_side, "nx": big_side, "phases": big_phases,
                    "threads": 256, "blocks": g * g, "lds_kib": 0.0, "seeded": True,
                    "seed": int(rng.integers(0, 2 ** 31 - 1)), "seed_frac": big_seed_frac,
                    "big": True}
        else:
            spec = dict(next(small))
        spec["index"] = i
        specs.append(spec)
    return specs


def poisson_arrivals(seed: int, n: int, rate: float) -> np.ndarray:
    """Arrival times (seconds, from 0) of n jobs of a Poisson process."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    gaps[0] = 0.0
    return np.cumsum(gaps)
