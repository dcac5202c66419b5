"""Validity of the enriched race records against the oracle's access log.

Test helper.  A record names two shadow summaries, `before` and `with`,
whose access sets hold a racing pair.  Which pair the device reports depends
on the interleaving, so the check is that the record is *valid*: some access
of the log at the record's key that `before` may stand for races (by the
oracle's pairwise definition) with some access that `with` may stand for,
and, for a record made by the hook of the completing access, `with` is that
access alone (its thread, block and class).
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2401_04701_amd import hr

NONE = 0xFFFFFFFF
CLASS = {hr.HR_READ: 1, hr.HR_WRITE: 3, hr.HR_ATOMIC: 2}


def _within(c_acc: int, c_sum: int) -> bool:
    return c_sum != 0 and (c_acc | c_sum) == c_sum


def stands_for(acc, s: dict, space: int, launch: int, wave_bits: int = 6) -> bool:
    """Whether summary `s` (decoded) may include access `acc`; groups are
    waves (wave_bits 6) or tiles of 2**wave_bits lanes."""
    if space == hr.HR_GLOBAL:
        if (int(acc["launch"]) & 511) != s["launch"]:
            return False
    elif int(acc["launch"]) != launch:
        return False
    c = CLASS[int(acc["kind"])]
    if s["state"] == hr.HR_S_BLOCKS:
        return _within(c, s["class_block"])
    if s["state"] not in (hr.HR_S_WAVES, hr.HR_S_THREADS, hr.HR_S_THREAD):
        return False
    if space == hr.HR_GLOBAL and int(acc["block"]) != s["block"]:
        return False
    if space == hr.HR_GLOBAL and _within(c, s["class_launch"]):
        return True                      # an access of the block earlier in the launch
    if int(acc["bc"]) != s["bc"]:
        return False
    if _within(c, s["class_block"]):
        return True                      # the block's latest epoch
    if s["state"] == hr.HR_S_WAVES:
        return False
    if (int(acc["thread"]) >> wave_bits) != s["wave"] or int(acc["wc"]) != s["wc"]:
        return False
    if s["state"] == hr.HR_S_THREAD and int(acc["thread"]) != s["thread"]:
        return False
    return _within(c, s["class_wave"])


def stands_for_nested(acc, s: dict, space: int, launch: int, tile_bits: int) -> bool:
    """As stands_for, for a summary of the nested-tile machine (decoded by
    hr_describe_nested): waves of 64 lanes, tiles of 2**tile_bits lanes with
    their own epochs (the access's tc) inside them."""
    if space == hr.HR_GLOBAL:
        if (int(acc["launch"]) & 511) != s["launch"]:
            return False
    elif int(acc["launch"]) != launch:
        return False
    c = CLASS[int(acc["kind"])]
    if s["state"] == hr.HR_S_BLOCKS:
        return _within(c, s["class_block"])
    if s["state"] not in (hr.HR_S_WAVES, hr.HR_S_TILES, hr.HR_S_THREADS, hr.HR_S_THREAD):
        return False
    if space == hr.HR_GLOBAL and int(acc["block"]) != s["block"]:
        return False
    if space == hr.HR_GLOBAL and _within(c, s["class_launch"]):
        return True                      # an access of the block earlier in the launch
    if int(acc["bc"]) != s["bc"]:
        return False
    if _within(c, s["class_block"]):
        return True                      # the block's latest epoch
    if s["state"] == hr.HR_S_WAVES:
        return False
    if (int(acc["thread"]) >> 6) != s["wave"] or int(acc["wc"]) != s["wc"]:
        return False
    if _within(c, s["class_wave"]):
        return True                      # the wave's latest epoch
    if s["state"] == hr.HR_S_TILES:
        return False
    if (int(acc["thread"]) >> tile_bits) != s["tile"] or int(acc["tc"]) != s["tc"]:
        return False
    if s["state"] == hr.HR_S_THREAD and int(acc["thread"]) != s["thread"]:
        return False
    return _within(c, s["class_tile"])


def record_problem(rec, log_at_key: np.ndarray, strict_with: bool = True, wave_bits: int = 6,
                   nested: bool = False):
    """None if the record is valid for the accesses at its key, else a reason.
    nested: a record of a context with tiles of 2**wave_bits lanes nested in
    64-lane waves (its words decode with hr_describe_nested)."""
    space = int(rec["space"])
    if int(rec["flags"]) & hr.HR_RACE_SCANNED:
        return None                      # only the key is reported
    launch = int(rec["launch"])
    if nested:
        b = hr.describe_nested(space, int(rec["before"]), wave_bits)
        w = hr.describe_nested(space, int(rec["with"]), wave_bits)
        covers = lambda a, s: stands_for_nested(a, s, space, launch, wave_bits)  # noqa: E731
        races = lambda p, q: oracle.race_pair(p, q, 64, 1 << wave_bits)  # noqa: E731
        finest = "class_tile"
    else:
        b = hr.describe(space, int(rec["before"]), wave_bits)
        w = hr.describe(space, int(rec["with"]), wave_bits)
        covers = lambda a, s: stands_for(a, s, space, launch, wave_bits)  # noqa: E731
        races = lambda p, q: oracle.race_pair(p, q, 1 << wave_bits)  # noqa: E731
        finest = "class_wave"
    fold = bool(int(rec["flags"]) & hr.HR_RACE_FOLD)
    if not fold and strict_with:
        if w["state"] != hr.HR_S_THREAD or w["thread"] != int(rec["tid"]):
            return "with is not the completing access alone"
        if w[finest] != CLASS[int(rec["kind"])]:
            return "with has another class than the record's kind"
        if space == hr.HR_GLOBAL and w["block"] != int(rec["block"]):
            return "with names another block"
    ps = [a for a in log_at_key if covers(a, b)]
    qs = [a for a in log_at_key if covers(a, w)]
    if not ps:
        return "no access of the log matches before"
    if not qs:
        return "no access of the log matches with"
    for p in ps:
        for q in qs:
            if races(p, q):
                return None
    return "no racing pair between before and with"


def by_key(log: np.ndarray):
    out = {}
    for a in log:
        lb = int(a["lds_block"]) if int(a["space"]) == hr.HR_LDS else 0
        out.setdefault((int(a["space"]), int(a["region"]), lb, int(a["index"])), []).append(a)
    return out


def record_key(rec, region_map=None):
    sp = int(rec["space"])
    rg = int(rec["region"])
    if region_map is not None and sp == hr.HR_GLOBAL:
        rg = region_map[rg]
    return (sp, rg, int(rec["block"]) if sp == hr.HR_LDS else 0, int(rec["index"]))
