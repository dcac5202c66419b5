"""Access programs of the example kernels that the source instrumenter
rewrites (paper_2401_04701_amd/examples/), written from the kernels' source
text: which element each thread reads, writes or updates atomically, in
which block-barrier phase.  The oracle's flagged set of such a program is
the expected set of the instrumented kernel.  Test infrastructure: nothing
here is used by the checker.

Program regions: global region 0 is the kernel's first pointer parameter,
region 1 its second; LDS array 0 is its first __shared__ array.
"""
from __future__ import annotations

import numpy as np

import oracle
import synth_inputs as si

R, W, A = si.KIND_R, si.KIND_W, si.KIND_A
G, L = si.SPACE_GLOBAL, si.SPACE_LDS


def histogram_program(keys: np.ndarray, blocks: int, threads: int, plain: int) -> si.Program:
    """histogram(keys, bins, n, plain): thread i < n reads keys[i], then
    increments bins[keys[i]], with a plain read-modify-write (a read and a
    write of the bin) when plain is set, else with an atomic add."""
    n = int(keys.shape[0])
    per = [[[[] for _ in range(threads)] for _ in range(blocks)]]
    for b in range(blocks):
        for t in range(threads):
            i = b * threads + t
            if i >= n:
                continue
            k = int(keys[i])
            ops = [si.op_word(G, 0, R, i)]
            if plain:
                ops += [si.op_word(G, 1, R, k), si.op_word(G, 1, W, k)]
            else:
                ops.append(si.op_word(G, 1, A, k))
            per[0][b][t] = ops
    launch = si.build_launch(blocks, threads, [si.SCOPE_NONE], [0], per)
    return si.Program([launch], [n, int(keys.max()) + 1 if n else 1], 0)


def stencil3_program(n: int, blocks: int, seeded_block: int) -> si.Program:
    """stencil3(u, v, n, seeded_block), 256 threads per block and a 258-word
    LDS tile: thread l of block b (cell g = 256 b + l) stages u[g] into
    tile[l + 1] when g < n, lane 0 also u[g - 1] into tile[0] when g > 0,
    lane 255 also u[g + 1] into tile[257] when g + 1 < n; a block barrier;
    then, when g < n, it reads tile[l + 1], tile[l] when g > 0 and tile[l + 2]
    when g + 1 < n, and writes v[g]; lane 255 of the seeded block also writes
    v[g + 1] when g + 1 < n."""
    T = 256
    per = [[[[] for _ in range(T)] for _ in range(blocks)] for _ in range(2)]
    for b in range(blocks):
        for l in range(T):
            g = b * T + l
            p0, p1 = per[0][b][l], per[1][b][l]
            if g < n:
                p0 += [si.op_word(G, 0, R, g), si.op_word(L, 0, W, l + 1)]
            if l == 0 and g > 0:
                p0 += [si.op_word(G, 0, R, g - 1), si.op_word(L, 0, W, 0)]
            if l == 255 and g + 1 < n:
                p0 += [si.op_word(G, 0, R, g + 1), si.op_word(L, 0, W, 257)]
            if g < n:
                p1.append(si.op_word(L, 0, R, l + 1))
                if g > 0:
                    p1.append(si.op_word(L, 0, R, l))
                if g + 1 < n:
                    p1.append(si.op_word(L, 0, R, l + 2))
                p1.append(si.op_word(G, 1, W, g))
                if b == seeded_block and l == 255 and g + 1 < n:
                    p1.append(si.op_word(G, 1, W, g + 1))
    launch = si.build_launch(blocks, T, [si.SCOPE_BLOCK, si.SCOPE_NONE], [0, 0], per)
    return si.Program([launch], [n, n], 258)


def flagged_as(program: si.Program, regions, wave_width: int = 64, tile_width: int = 0) -> set:
    """Oracle flagged set of a program with its global regions renamed to the
    context regions `regions` (program region j -> regions[j]); LDS keys keep
    array id 0."""
    out = set()
    for sp, rg, lb, ix in oracle.flagged_program(program, wave_width, tile_width):
        out.add((sp, regions[rg] if sp == 0 else rg, lb, ix))
    return out


def _rescope(program: si.Program, fn) -> si.Program:
    launches = []
    for l in program.launches:
        scope, mask = zip(*(fn(int(sc), int(m), l.threads) for sc, m in zip(l.scope, l.wave_mask)))
        launches.append(si.Launch(l.blocks, l.threads, np.array(scope, dtype=np.uint8),
                                  np.array(mask, dtype=np.uint64), l.op_off, l.ops))
    return si.Program(launches, program.global_words, program.lds_words)


def as_tile_groups(program: si.Program, tile: int) -> si.Program:
    """A program with tile barriers (scope 3) and wave barriers as a checker
    whose only groups below the block are tiles of `tile` lanes sees it (to
    be evaluated with wave width `tile`): a tile barrier stays a barrier of
    its tiles, and a wave barrier becomes a barrier of every tile of the
    waves it names, each tile on its own."""
    per = 64 // tile

    def fn(sc, m, threads):
        if sc == si.SCOPE_TILE:
            return si.SCOPE_WAVE, m
        if sc == si.SCOPE_WAVE:
            tiles = 0
            for w in range(64):
                if (m >> w) & 1:
                    for g in range(w * per, min(64, (w + 1) * per)):
                        tiles |= 1 << g
            return si.SCOPE_WAVE, tiles
        return sc, m
    return _rescope(program, fn)


def without_tile_barriers(program: si.Program) -> si.Program:
    """The program as a checker of whole waves sees it when the tile
    barriers' masks are narrower than its groups: no ordering at all."""
    return _rescope(program, lambda sc, m, threads: (si.SCOPE_NONE, 0) if sc == si.SCOPE_TILE
                    else (sc, m))


def insert_block_barrier(program: si.Program, before: int) -> si.Program:
    """The program with an empty phase ending in a block barrier inserted
    before phase `before` of every launch (a block-wide sync between two
    phases)."""
    launches = []
    for l in program.launches:
        cut = before * l.blocks * l.threads
        op_off = np.concatenate([l.op_off[:cut],
                                 np.full(l.blocks * l.threads, l.op_off[cut], l.op_off.dtype),
                                 l.op_off[cut:]])
        scope = np.insert(l.scope, before, si.SCOPE_BLOCK).astype(np.uint8)
        mask = np.insert(l.wave_mask, before, 0).astype(np.uint64)
        launches.append(si.Launch(l.blocks, l.threads, scope, mask, op_off, l.ops))
    return si.Program(launches, program.global_words, program.lds_words)
