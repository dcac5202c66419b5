"""Build the race checker's shared library (libhr.so) for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhr.so")
SOURCES = ["hr_runtime.hip", "hr_workloads.hip", "hr_batch.hip", "hr_serve.hip", "hr_peaks.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed-fp32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libhr.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", INCLUDE, "-I", CSRC]
    cmd += [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libhr.so")
    os.replace(tmp, LIB)
    return LIB


EXAMPLES = ["reduce_block.hip", "stencil3.hip", "histogram.hip"]
EXAMPLES_LIB = os.path.join(PKG, "libhr_examples.so")


def build_examples(verbose: bool = False) -> str:
    """Instrument the example kernels with the source instrumenter and
    compile them, with their launchers, into libhr_examples.so (linked to
    libhr.so).  The instrumented sources go to _gen/."""
    from . import instrument
    gen = os.path.join(PKG, "_gen")
    os.makedirs(gen, exist_ok=True)
    outs = []
    for name in EXAMPLES:
        text, _ = instrument.instrument(os.path.join(PKG, "examples", name))
        out = os.path.join(gen, name.replace(".hip", ".inst.hip"))
        with open(out, "w") as f:
            f.write(text)
        outs.append(out)
    tmp = EXAMPLES_LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", INCLUDE, "-I", CSRC] + outs + [
        "-L", PKG, "-lhr", "-Wl,-rpath,$ORIGIN", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libhr_examples.so")
    os.replace(tmp, EXAMPLES_LIB)
    return EXAMPLES_LIB


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_examples(verbose=True))
