"""The full-size goldens written by oracle/goldens.py (the oracle streamed
over the whole access log of a job) agree with what the workloads'
definitions fix in closed form, and with the oracle's own record counts.
The GPU tests compare the checker against these files."""
import json
import os

import numpy as np

import oracle
import synth_inputs as si
from oracle import closed_forms as cf
from oracle import goldens

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_jacobi_full_golden_matches_closed_form():
    g = load("jacobi_4096x4096_20launches.json")
    ny, nx, launches, seeds, tab = goldens.jacobi_full_workload()
    keys = {tuple(k) for k in g["keys"]}
    assert len(seeds) == 66 and len(keys) == g["flagged"] == 2 * 66
    assert keys == cf.jacobi_flagged(ny, nx, launches, seeds)
    assert goldens.key_digest(keys) == g["sha256"]
    lib = oracle._lib()
    per_launch = lib.orc_model_jacobi(ny, nx, 0, 1, tab.ctypes.data, 0, 256, 0, 256, None, 0)
    assert g["checks"] == per_launch * launches == 2851145000


def test_labelprop_full_golden_matches_closed_form():
    g = load("labelprop_rmat22_10launches.json")
    rp, col, mask, launches = goldens.labelprop_full_workload()
    want = cf.labelprop_flagged(rp, col, mask)
    assert len(want) == g["flagged"] and goldens.key_digest(want) == g["sha256"]
    ks = sorted(want)
    assert [list(k) for k in ks[:16]] == g["first_keys"]
    assert [list(k) for k in ks[-16:]] == g["last_keys"]
    n = rp.shape[0] - 1
    assert g["checks"] == launches * (n + col.shape[0] + int(mask.sum()))


def test_streamed_oracle_equals_whole_log_oracle():
    """Streaming (per launch, per band of block rows with their neighbours;
    per part of the labels) gives the oracle's set on the whole log."""
    ny, nx = 200, 168
    seeds = si.jacobi_seeds(ny, nx, 17, count=9)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    whole = oracle.flagged(oracle.model_jacobi(ny, nx, 3, tab))
    for band in (1, 2, 5):
        keys, checks, _, _ = goldens.jacobi_streamed(ny, nx, 3, tab, band=band, n_workers=1)
        assert keys == whole and checks == oracle.model_jacobi(ny, nx, 3, tab).shape[0]
    rp, col, mask = si.labelprop_graph(9, 4096, 5, 0.05)
    whole = oracle.flagged(oracle.model_labelprop(rp, col, mask, 2, 64))
    keys, checks, _, _ = goldens.labelprop_streamed(rp, col, mask, 2, tpb=64, parts=5,
                                                    n_workers=2)
    assert keys == whole and len(whole) > 10
    assert checks == oracle.model_labelprop(rp, col, mask, 2, 64).shape[0]


def _closed_form(spec, a):
    p = spec["pattern"]
    if p == si.PAT_REDUCE:
        return cf.reduce_n_flagged(spec["n"], spec["threads"], spec["blocks"], spec["drop"])
    if p == si.PAT_JACOBI:
        return cf.jacobi_flagged(spec["ny"], spec["nx"], spec["phases"], a["seeds"])
    return cf.labelprop_flagged(a["row_ptr"], a["col"], a["mask"])


def test_batched_and_serving_goldens_match_closed_forms():
    """Every job's oracle set in the batched-manifest and serving-stream
    goldens (whole jobs, the full-size stencils streamed) equals what the
    job's workload definition fixes in closed form."""
    for name, specs in (("batched_manifest_1000.json", si.batched_manifest(si.master_seed(3))),
                        ("serving_stream_40.json", goldens.serving_test_stream())):
        g = load(name)["jobs"]
        assert [e["index"] for e in g] == [s["index"] for s in specs]
        flagged = 0
        for e, s in zip(g, specs):
            want = _closed_form(s, si.instance_inputs(s))
            assert (e["pattern"], e["flagged"], e["sha256"]) == \
                (s["pattern"], len(want), goldens.key_digest(want)), (name, s["index"])
            flagged += len(want)
        assert flagged > 0
