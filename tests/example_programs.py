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


def flagged_as(program: si.Program, regions, wave_width: int = 64) -> set:
    """Oracle flagged set of a program with its global regions renamed to the
    context regions `regions` (program region j -> regions[j]); LDS keys keep
    array id 0."""
    out = set()
    for sp, rg, lb, ix in oracle.flagged_program(program, wave_width):
        out.add((sp, regions[rg] if sp == 0 else rg, lb, ix))
    return out
