"""CPU model of the device hooks as the tuned kernels issue them, under
adversarial interleavings.  Test helper.

protocol_sim.py models each hook as load -> exchange -> fold, one hook of a
thread at a time.  The kernels go further, in three ways this model adds:

* preloaded words (depth D): the shadow word of a later global access of
  the thread is loaded before the thread's earlier hooks have settled (the
  label-propagation loop prefetches the next edges' words), so it may miss
  the thread's own earlier updates (consecutive duplicate edges);
* split issue and settle (S pending): a global hook publishes its exchange
  and the thread goes on to its next accesses (LDS hooks, or another global
  hook's load and exchange) before the fold of the first is done (the
  stencil settles after the next LDS hook, the edge-pair loop settles both
  edges after issuing both); folds settle in program order, all before the
  thread's next barrier;
* wave grouping (coalescing width W): lanes of one hardware wave whose k-th
  operation of a phase is a global access of the same kind to the same word
  form one hook: an owner lane applies its own access and one partner's in
  one update, the other members skip theirs and go on only once the owner's
  hook is done (the lanes run the hook together).  Owner and partner are
  drawn at random, and a member may be left to update alone (a hash bucket
  taken by another word).

Every step on a shadow word is atomic on its own; a random scheduler picks
the next step of any thread.  Barriers release a group once every member
has arrived with nothing pending.  The transition and merge are the
library's (hr_fsm_step, hr_fsm_merge), evaluated on the host.
"""
from __future__ import annotations

import numpy as np

import synth_inputs as si
from paper_2401_04701_amd import hr

RACE = hr.T_RACE
STATS = {"folds": 0, "stale_own": 0, "split_overlaps": 0, "grouped": 0, "partners": 0}


class _T:
    __slots__ = ("block", "thread", "wave", "ops", "pc", "bc", "wc", "hook", "pending",
                 "pre", "pre_next", "done", "xlog")

    def __init__(self, block, thread, wave, ops):
        self.block, self.thread, self.wave, self.ops = block, thread, wave, ops
        self.pc, self.bc, self.wc = 0, 0, 0
        self.hook = None        # the hook being started (load / exchange / LDS loop)
        self.pending = []       # published global hooks not yet settled (folds)
        self.pre = {}           # op index -> (preloaded word, own exchanges made by then)
        self.pre_next = 0       # next op index a preload may consider
        self.done = set()       # op indices whose hooks have completed (folds included)
        self.xlog = []          # keys of the thread's own exchanges, in order


def _expand(launch, narrow, group_width, rng):
    """Per-thread op lists with grouping applied.  Ops: ('A', space, region,
    index, kind, ids) where ids lists the (thread, wave) identities the
    update applies, ('S', owner_key) a grouped member's skipped access, or
    ('B',) / ('W',) barriers."""
    ths, ops_of = [], {}
    for b in range(launch.blocks):
        for t in range(launch.threads):
            w = t // narrow
            thread = w * 64 + t % narrow        # narrow waves relabelled onto 64-lane waves
            th = _T(b, thread, w, [])
            ths.append(th)
            ops_of[(b, t)] = th
    # instruction slots: (block, phase, k) -> lanes with their k-th access
    for p in range(launch.phases):
        slot = {}
        for b in range(launch.blocks):
            for t in range(launch.threads):
                th = ops_of[(b, t)]
                for k, word in enumerate(launch.thread_ops(p, b, t)):
                    space, region, kind, index = si.op_fields(word)
                    pos = len(th.ops)
                    th.ops.append(["A", space, region, index, kind, [(th.thread, th.wave)]])
                    if group_width and space == si.SPACE_GLOBAL:
                        seg = (t % narrow) // group_width if narrow > group_width else 0
                        slot.setdefault((b, th.wave, seg, k, kind, region, index), []).append(
                            (th, pos))
                sc = int(launch.scope[p])
                w = t // narrow
                if sc == si.SCOPE_BLOCK:
                    th.ops.append(["B"])
                elif sc == si.SCOPE_WAVE and (int(launch.wave_mask[p]) >> w) & 1:
                    th.ops.append(["W"])
        for lanes in slot.values():
            if len(lanes) < 2:
                continue
            order = rng.permutation(len(lanes))
            owner, opos = lanes[order[0]]
            members = [lanes[i] for i in order[1:]]
            # some members update alone (their bucket went to another word)
            alone = [m for m in members if rng.random() < 0.2]
            joined = [m for m in members if m not in alone]
            if not joined:
                continue
            STATS["grouped"] += 1
            partner = joined[int(rng.integers(0, len(joined)))]
            owner.ops[opos][5] = [(owner.thread, owner.wave), (partner[0].thread, partner[0].wave)]
            STATS["partners"] += 1
            for th, pos in joined:
                th.ops[pos] = ["S", (id(owner), opos)]
    return ths


def simulate(program, narrow: int, seed: int, preload: int = 0, split: int = 0,
             group_width: int = 0):
    """Run every launch under a random schedule.  Returns (pushed keys,
    final global shadow words)."""
    rng = np.random.default_rng(seed)
    gwords, pushed = {}, []
    for L, launch in enumerate(program.launches):
        lwords = {}
        ths = _expand(launch, narrow, group_width, rng)
        by_id = {id(th): th for th in ths}
        groups = {}
        for th in ths:
            groups.setdefault(("B", th.block), []).append(th)
            groups.setdefault(("W", th.block, th.wave), []).append(th)
        while True:
            _release(groups)
            acts = []
            for th in ths:
                acts.extend(_actions(th, by_id, preload, split))
            if not acts:
                assert all(th.pc == len(th.ops) and not th.pending for th in ths), "deadlock"
                break
            th, act = acts[int(rng.integers(0, len(acts)))]
            _step(th, act, L, gwords, lwords, pushed)
    return pushed, gwords


def _release(groups):
    released = True
    while released:
        released = False
        for (kind, *_), members in groups.items():
            if all(m.hook is None and not m.pending and m.pc < len(m.ops) and
                   m.ops[m.pc][0] == kind for m in members):
                released = True
                for m in members:
                    m.done.add(m.pc)
                    m.pc += 1
                    m.pre_next = max(m.pre_next, m.pc)
                    if kind == "B":
                        m.bc += 1
                        m.wc = 0
                    else:
                        m.wc += 1


def _actions(th, by_id, preload, split):
    acts = []
    if th.hook is not None:
        acts.append((th, "hook"))
    elif th.pc < len(th.ops):
        op = th.ops[th.pc]
        if op[0] == "S":
            owner = by_id[op[1][0]]
            if op[1][1] in owner.done:          # the owner's hook (and fold) is done
                acts.append((th, "skip"))
        elif op[0] == "A":
            # without split, a hook starts only once the previous one settled;
            # with it, LDS hooks run beside pending folds and at most `split`
            # global hooks are in flight
            if not th.pending or (split and (op[1] == si.SPACE_LDS or len(th.pending) < split)):
                acts.append((th, "start"))
    if th.pending:
        acts.append((th, "settle"))
    if preload and (th.hook is None or th.hook["stage"] == "xchg"):
        q = _preload_target(th, preload)
        if q is not None:
            acts.append((th, ("preload", q)))
    return acts


def _preload_target(th, depth):
    """The next global access whose word may be loaded now, in program order:
    within the current barrier interval, at most `depth` global accesses
    after the one in progress."""
    seen = 0
    for q in range(th.pc, len(th.ops)):
        op = th.ops[q]
        if op[0] in ("B", "W"):
            return None
        if op[0] != "A" or op[1] != si.SPACE_GLOBAL:
            continue
        if seen > depth:
            return None
        seen += 1
        busy = th.hook is not None and th.hook["pos"] == q
        if q >= th.pre_next and q not in th.pre and not busy:
            return q
    return None


def _step(th, act, L, gwords, lwords, pushed):
    if act == "skip":
        th.done.add(th.pc)
        th.pc += 1
        return
    if isinstance(act, tuple):                  # preload the word of op q
        q = act[1]
        _, space, region, index, kind, ids = th.ops[q]
        th.pre[q] = (gwords.get((0, region, 0, index), 0), len(th.xlog))
        th.pre_next = q + 1
        return
    if act == "settle":
        _fold_step(th, th.pending[0], gwords, pushed)
        return
    if act == "start":
        _, space, region, index, kind, ids = th.ops[th.pc]
        th.hook = {"space": space, "region": region, "index": index, "kind": kind, "ids": ids,
                   "pos": th.pc, "stage": "load"}
        if space == si.SPACE_GLOBAL and th.pc in th.pre:
            word, since = th.pre.pop(th.pc)
            th.hook.update(stage="xchg", old=word, since=since)
        if th.pending:
            STATS["split_overlaps"] += 1
        return
    h = th.hook
    if h["space"] == si.SPACE_GLOBAL:
        key = (0, h["region"], 0, h["index"])
        if h["stage"] == "load":
            h.update(stage="xchg", old=gwords.get(key, 0), since=None)
            return
        # exchange: the new word from the loaded one, published atomically
        # (an unchanged word publishes nothing)
        nw = h["old"]
        for thread, _wave in h["ids"]:
            nw = hr.fsm_step(hr.HR_GLOBAL, nw, h["kind"], L & 511, th.block, thread, th.bc,
                             th.wc, 6)
        th.hook = None
        th.pc = max(th.pc, h["pos"] + 1)
        th.pre_next = max(th.pre_next, th.pc)
        if nw == h["old"]:
            th.done.add(h["pos"])
            return
        r = gwords.get(key, 0)
        gwords[key] = nw
        if h["since"] is not None and key in th.xlog[h["since"]:]:
            STATS["stale_own"] += 1             # the preload missed the thread's own update
        th.xlog.append(key)
        if nw == RACE or r == h["old"]:
            if nw == RACE and r != RACE:
                pushed.append(key)
            th.done.add(h["pos"])
            return
        STATS["folds"] += 1
        th.pending.append({"key": key, "cur": nw, "lost": r, "pos": h["pos"]})
        if len(th.pending) > 1:
            STATS["split_overlaps"] += 1
        return
    # LDS: load, then compare-and-swap until it holds
    wkey = (th.block, h["region"], h["index"])
    if h["stage"] == "load":
        h.update(stage="cas", old=lwords.get(wkey, 0))
        return
    nw = hr.fsm_step(hr.HR_LDS, h["old"], h["kind"], 0, 0, th.thread, th.bc, th.wc, 6)
    seen = lwords.get(wkey, 0)
    if nw == h["old"] or seen == h["old"]:
        if nw != h["old"]:
            lwords[wkey] = nw
            if nw == RACE:
                pushed.append((1, h["region"], th.block, h["index"]))
        th.hook = None
        th.done.add(h["pos"])
        th.pc = max(th.pc, h["pos"] + 1)
        return
    h["old"] = seen


def _fold_step(th, f, gwords, pushed):
    """One round of the fold: merge the overwritten summary into the word
    the thread believes is there, and compare-and-swap it in."""
    m = hr.fsm_merge(f["cur"], f["lost"], 6)
    if m == f["cur"]:
        th.done.add(th.pending.pop(0)["pos"])
        return
    seen = gwords.get(f["key"], 0)
    if seen == f["cur"]:
        gwords[f["key"]] = m
        if m == RACE and f["lost"] != RACE:
            pushed.append(f["key"])
        th.done.add(th.pending.pop(0)["pos"])
        return
    f["cur"] = seen
