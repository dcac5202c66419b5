"""Replay an access log through the checker's transition function (host
evaluation via hr_fsm_step) in a chosen happens-before-consistent order.

Test helper: the GPU applies shadow updates in some order consistent with
program order, barriers and launches; these helpers generate such orders
(random or exhaustive) so the CPU tests can show the flagged set does not
depend on which one the hardware picks."""
from __future__ import annotations

import numpy as np

from paper_2401_04701_amd import hr


def random_orders(log: np.ndarray, n_orders: int, seed: int, wave_width: int = 64):
    """Yield index orders of `log` (records grouped by launch; within a thread
    in program order as emitted) that respect program order and barriers."""
    rng = np.random.default_rng(seed)
    launches = sorted(set(int(x) for x in log["launch"]))
    for _ in range(n_orders):
        order = []
        for L in launches:
            idx = np.nonzero(log["launch"] == L)[0]
            order.extend(_one_launch_order(log, idx, rng, wave_width))
        yield order


def _one_launch_order(log, idx, rng, wave_width):
    threads = {}
    for i in idx:
        key = (int(log["block"][i]), int(log["thread"][i]))
        threads.setdefault(key, []).append(int(i))
    keys = list(threads)
    pos = {k: 0 for k in keys}
    # pending records per (block, bc) and per (block, wave, bc, wc)
    pend_b = {}
    pend_w = {}
    for k in keys:
        for i in threads[k]:
            b, t = k
            bc, wc = int(log["bc"][i]), int(log["wc"][i])
            pend_b[(b, bc)] = pend_b.get((b, bc), 0) + 1
            pend_w[(b, t // wave_width, bc, wc)] = pend_w.get((b, t // wave_width, bc, wc), 0) + 1
    out = []
    remaining = len(idx)
    while remaining:
        cand = []
        for k in keys:
            if pos[k] >= len(threads[k]):
                continue
            i = threads[k][pos[k]]
            b, t = k
            bc, wc = int(log["bc"][i]), int(log["wc"][i])
            if any(pend_b.get((b, e), 0) for e in range(bc)):
                continue
            if any(pend_w.get((b, t // wave_width, bc, e), 0) for e in range(wc)):
                continue
            cand.append(k)
        assert cand, "no enabled record: log is not barrier-consistent"
        k = cand[int(rng.integers(0, len(cand)))]
        i = threads[k][pos[k]]
        pos[k] += 1
        b, t = k
        bc, wc = int(log["bc"][i]), int(log["wc"][i])
        pend_b[(b, bc)] -= 1
        pend_w[(b, t // wave_width, bc, wc)] -= 1
        out.append(i)
        remaining -= 1
    return out


def replay(log: np.ndarray, order, wave_bits: int = 6, word4=None) -> set:
    """Apply the transition function in `order`; return the keys that reached
    the race state.  LDS shadow starts fresh for every block and launch.
    word4 = (wc_bits, bc_bits, thread_bits) replays global words as 4-byte
    words of those widths, which start fresh at every launch."""
    words = {}
    racy = set()
    for i in order:
        r = log[i]
        sp, rg, ix = int(r["space"]), int(r["region"]), int(r["index"])
        b, t, L = int(r["block"]), int(r["thread"]), int(r["launch"])
        if sp == hr.HR_LDS:
            wkey = (1, rg, b, ix, L)
            key = (1, rg, b, ix)
        elif word4 is not None:
            wkey = (0, rg, 0, ix, L)
            key = (0, rg, 0, ix)
        else:
            wkey = (0, rg, 0, ix)
            key = wkey
        old = words.get(wkey, 0)
        if sp == hr.HR_GLOBAL and word4 is not None:
            new = hr.fsm_step_word4(old, int(r["kind"]), b, t, int(r["bc"]), int(r["wc"]),
                                    wave_bits, *word4)
            raced = new == hr.T_RACE
        else:
            new = hr.fsm_step(sp, old, int(r["kind"]), L & 511, b, t, int(r["bc"]),
                              int(r["wc"]), wave_bits)
            raced = (new & 7) == hr.T_RACE
        words[wkey] = new
        if raced:
            racy.add(key)
    return racy


def random_orders_nested(log: np.ndarray, n_orders: int, seed: int, tile_width: int):
    """As random_orders, for tiles of tile_width lanes nested in 64-lane waves:
    a record also waits for every record of its tile in an earlier tile epoch
    of the same wave epoch."""
    rng = np.random.default_rng(seed)
    launches = sorted(set(int(x) for x in log["launch"]))
    for _ in range(n_orders):
        order = []
        for L in launches:
            idx = np.nonzero(log["launch"] == L)[0]
            order.extend(_one_launch_order_nested(log, idx, rng, tile_width))
        yield order


def _one_launch_order_nested(log, idx, rng, tw):
    threads = {}
    for i in idx:
        threads.setdefault((int(log["block"][i]), int(log["thread"][i])), []).append(int(i))
    keys = list(threads)
    pos = {k: 0 for k in keys}
    pend = {}

    def scopes(i, b, t):
        bc, wc, tc = int(log["bc"][i]), int(log["wc"][i]), int(log["tc"][i])
        return [("b", b, bc), ("w", b, t // 64, bc, wc), ("t", b, t // tw, bc, wc, tc)]
    for k in keys:
        for i in threads[k]:
            for sc in scopes(i, *k):
                pend[sc] = pend.get(sc, 0) + 1
    out = []
    for _ in range(len(idx)):
        cand = []
        for k in keys:
            if pos[k] >= len(threads[k]):
                continue
            i = threads[k][pos[k]]
            b, t = k
            bc, wc, tc = int(log["bc"][i]), int(log["wc"][i]), int(log["tc"][i])
            if any(pend.get(("b", b, e), 0) for e in range(bc)):
                continue
            if any(pend.get(("w", b, t // 64, bc, e), 0) for e in range(wc)):
                continue
            if any(pend.get(("t", b, t // tw, bc, wc, e), 0) for e in range(tc)):
                continue
            cand.append(k)
        assert cand, "no enabled record: log is not barrier-consistent"
        k = cand[int(rng.integers(0, len(cand)))]
        i = threads[k][pos[k]]
        pos[k] += 1
        for sc in scopes(i, *k):
            pend[sc] -= 1
        out.append(i)
    return out


def replay_nested(log: np.ndarray, order, tile_bits: int) -> set:
    """Apply the nested-tile machine's transition in `order`; return the keys
    that reached the race state."""
    words, racy = {}, set()
    for i in order:
        r = log[i]
        sp, rg, ix = int(r["space"]), int(r["region"]), int(r["index"])
        b, t, L = int(r["block"]), int(r["thread"]), int(r["launch"])
        wkey = (1, rg, b, ix, L) if sp == hr.HR_LDS else (0, rg, 0, ix)
        new = hr.fsm_step_nested(sp, words.get(wkey, 0), int(r["kind"]), L & 511, b, t,
                                 int(r["bc"]), int(r["wc"]), int(r["tc"]), tile_bits)
        words[wkey] = new
        if (new & 7) == hr.T_RACE:
            racy.add(wkey[:4])
    return racy
