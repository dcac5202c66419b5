"""Closed-form flagged sets of the workloads -- test infrastructure.

Each function states, from the workload's definition and the race
definition of the paper (Sec. II-A, II-B), which locations race, without
walking an access log.  They pin the pairwise oracle at small sizes and stand
in for it at full size.  Keys are (space, region, lds_block, index).
"""
from __future__ import annotations

import numpy as np


def reduce_flagged(drop: int) -> set:
    """One-block LDS tree reduction with the barrier after step `drop` removed.

    Step s (h = 256 >> s) has thread t < h read a[t] and a[t+h] and write a[t].
    Without the barrier after step k < 8, step k+1 reads a[t + h'] (h' = 128 >> k)
    in the same block epoch in which thread t + h' wrote it during step k:
    the words [128 >> k, 256 >> k) race.  Without the last barrier, every
    thread's final read of a[0] meets thread 0's last write: {a[0]}.
    """
    if drop is None or drop < 0 or drop > 8:
        return set()
    if drop == 8:
        return {(1, 0, 0, 0)}
    return {(1, 0, 0, i) for i in range(128 >> drop, 256 >> drop)}


def reduce_n_flagged(n: int, threads: int, blocks: int, drop: int) -> set:
    """Scaled reduction (n words per block, n a power of two <= 2 * threads).

    Step s halves h = n >> (s+1).  Without the barrier after step k (not the
    last), step k+1 reads a[t + h'] (h' = n >> (k+2)) in the block epoch in
    which thread t + h' wrote it: words [n >> (k+2), n >> (k+1)) race in every
    block.  Without the last step's barrier, the final reads of a[0] meet
    thread 0's last write.  The load barrier (n != 2 * threads) is never
    dropped, so the loads race with nothing.
    """
    steps = n.bit_length() - 1
    if drop is None or drop < 0 or drop >= steps:
        return set()
    if drop == steps - 1:
        words = [0]
    else:
        words = range(n >> (drop + 2), n >> (drop + 1))
    return {(1, 0, b, i) for b in range(blocks) for i in words}


def jacobi_flagged(ny: int, nx: int, launches: int, seeds, launch0: int = 0) -> set:
    """Jacobi sweeps with seeded neighbour-cell writes.

    In a launch each output cell is written by its owner thread only, and the
    input array is only read, so the only racy cells are the seeded halo
    cells of the output array: the owner's write and the seeded writer's
    write come from different blocks in the same launch.  Launch L writes
    array (L+1) % 2.
    """
    out = set()
    nbx = (nx + 15) // 16
    for b, side, off in np.asarray(seeds, dtype=np.int64).reshape(-1, 3):
        by, bx = divmod(int(b), nbx)
        y0, x0 = by * 16, bx * 16
        if side == 0:
            y, x = y0 - 1, x0 + off
        elif side == 1:
            y, x = y0 + 16, x0 + off
        elif side == 2:
            y, x = y0 + off, x0 - 1
        else:
            y, x = y0 + off, x0 + 16
        assert 0 <= y < ny and 0 <= x < nx
        for L in range(launch0, launch0 + launches):
            out.add((0, (L + 1) % 2, 0, y * nx + x))
    return out


def labelprop_flagged(row_ptr, col, mask) -> set:
    """Label propagation with seeded plain read+write edges.

    All unseeded accesses to label[] are atomics, which never race with each
    other.  A seeded edge (v, u) reads and writes label[u] plainly; it races
    with thread u's own atomic load of label[u] when v != u.  A seeded self
    loop (u, u) races only when some other thread w != u touches label[u],
    i.e. there is an edge (w, u) with w != u.
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    mask = np.asarray(mask).astype(bool)
    n = row_ptr.shape[0] - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    seeded_nonloop = mask & (src != col)
    flagged = np.zeros(n, dtype=bool)
    flagged[col[seeded_nonloop]] = True
    has_foreign_in = np.zeros(n, dtype=bool)
    has_foreign_in[col[src != col]] = True
    seeded_loop = mask & (src == col)
    loop_targets = np.zeros(n, dtype=bool)
    loop_targets[col[seeded_loop]] = True
    flagged |= loop_targets & has_foreign_in
    return {(0, 0, 0, int(u)) for u in np.nonzero(flagged)[0]}


def tile_reduce_flagged(tile: int, blocks: int, threads: int, drop: int) -> set:
    """Sub-wave tree reduction (tiles of `tile` lanes, each over its own LDS
    segment of n = 2 * tile words, tile barriers after each step).

    The segments are disjoint and each is touched only by its tile's lanes,
    so each tile is the scaled block reduction with n = 2 * tile: without the
    barrier after step k (not the last), step k+1 reads seg[l + h'] (h' =
    n >> (k+2)) in the tile epoch in which lane l + h' wrote it: words
    [n >> (k+2), n >> (k+1)) of every segment race.  Without the last step's
    barrier, every lane's final read of seg[0] meets lane 0's last write.
    """
    n = 2 * tile
    steps = n.bit_length() - 1
    if drop is None or drop < 0 or drop >= steps:
        return set()
    words = [0] if drop == steps - 1 else range(n >> (drop + 2), n >> (drop + 1))
    return {(1, 0, b, seg * n + w) for b in range(blocks) for seg in range(threads // tile)
            for w in words}
