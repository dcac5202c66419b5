"""Checked jobs on the device: upload a job's arrays and describe it as an
hr_instance for the batched launch or the serial path."""
from __future__ import annotations

import numpy as np

from . import hr

PATTERN = {"reduce": hr.HR_PAT_REDUCE, "jacobi": hr.HR_PAT_JACOBI,
           "labelprop": hr.HR_PAT_LABELPROP}


class Job:
    """One job: its device tensors and its hr_instance."""

    def __init__(self, spec, arrays, device="cuda"):
        import torch
        self.spec = spec
        t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)
        inst = hr.Instance()
        inst.pattern = spec["pattern"]
        inst.phases = spec["phases"]
        inst.drop = -1
        inst.region[0] = inst.region[1] = hr.NO_REGION
        if spec["pattern"] == hr.HR_PAT_REDUCE:
            self.tensors = [t(arrays["in"]), t(arrays["out"])]
            inst.n, inst.threads, inst.blocks = spec["n"], spec["threads"], spec["blocks"]
            inst.drop = spec["drop"]
        elif spec["pattern"] == hr.HR_PAT_JACOBI:
            self.tensors = [t(arrays["u0"]), t(arrays["u1"]), t(arrays["seed_tab"])]
            inst.n, inst.ny = spec["nx"], spec["ny"]
        else:
            self.tensors = [t(arrays["label"]), t(arrays["row_ptr"]), t(arrays["col"]),
                            t(arrays["mask"])]
            inst.n, inst.threads = spec["vertices"], spec["threads"]
        for i, x in enumerate(self.tensors):
            inst.data[i] = None if x is None else x.data_ptr()
        self.inst = inst

    def serial(self, ring_capacity=0):
        """The serial path: (flagged keys with job-local regions, warnings)."""
        return hr.job_run(self.inst, ring_capacity=ring_capacity)


def check_count(spec) -> int:
    """Instrumented accesses of a whole job (every phase)."""
    if spec["pattern"] == hr.HR_PAT_REDUCE:
        n, t, b = spec["n"], spec["threads"], spec["blocks"]
        return b * (2 * n + 3 * (n - 1) + 2 * t)
    if spec["pattern"] == hr.HR_PAT_JACOBI:
        ny, nx = spec["ny"], spec["nx"]
        cells = ny * nx
        halo = 2 * nx * (((ny + 15) // 16) - 1) + 2 * ny * (((nx + 15) // 16) - 1)
        seeded = 1 if spec["seeded"] else 0
        per = 2 * (cells + halo) + cells + seeded + 5 * cells - 2 * nx - 2 * ny
        return per * spec["phases"]
    return None  # label propagation depends on the seeded edges: use check_count_arrays


def check_count_arrays(spec, arrays) -> int:
    c = check_count(spec)
    if c is not None:
        if spec["pattern"] == hr.HR_PAT_JACOBI and spec["seeded"] and len(arrays["seeds"]) == 0:
            c -= spec["phases"]
        return c
    return (spec["vertices"] + spec["edges"] + int(arrays["mask"].sum())) * spec["phases"]
