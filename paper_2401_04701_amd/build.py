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
SOURCES = ["hr_runtime.hip", "hr_workloads.hip", "hr_batch.hip", "hr_serve.hip", "hr_peaks.hip",
           "hr_static.hip"]

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


KERNELS_JSON = os.path.join(PKG, "libhr_kernels.json")
FINGERPRINTED = ["hr_workloads.hip", "hr_serve.hip"]


def _kernel_bodies(asm: str) -> dict:
    """Each kernel of a device assembly listing: its instructions and labels,
    without comments, line records and directives.  Local labels lose the
    function number the assembler gives them (.LBB<function>_<block>), which
    changes when other functions are added to the module."""
    import re
    local = re.compile(r"\.LBB\d+_(\d+)")
    out, cur, lines = {}, None, []
    kernels = set()
    for ln in asm.splitlines():
        t = ln.strip()
        if t.startswith(".amdhsa_kernel "):
            kernels.add(t.split()[1])
    for ln in asm.splitlines():
        t = ln.split(";", 1)[0].rstrip()
        if cur is None:
            if t.endswith(":") and t[:-1] in kernels:
                cur, lines = t[:-1], []
            continue
        if t.startswith(".Lfunc_end"):
            out[cur] = "\n".join(lines)
            cur = None
            continue
        t = t.strip()
        if not t or (t.startswith(".") and not t.endswith(":")):   # directives
            continue
        lines.append(local.sub(r".LBB_\1", t))
    return out


def kernel_fingerprints(verbose: bool = False) -> str:
    """SHA-256 of each kernel's gfx950 assembly (instructions and labels
    only), written next to libhr.so.  A counter summary under profiles/
    records the fingerprint of the kernel it measured, so a changed kernel
    is recognised whatever else changed in its source files."""
    import hashlib
    import json
    import tempfile
    fp = {}
    with tempfile.TemporaryDirectory() as tmp:
        for src in FINGERPRINTED:
            out = os.path.join(tmp, src + ".s")
            cmd = [hipcc()] + [f for f in HIPCC_FLAGS if f != "-shared"] + [
                "--cuda-device-only", "-S", "-I", INCLUDE, "-I", CSRC,
                os.path.join(CSRC, src), "-o", out]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed producing the assembly of {src}")
            with open(out) as f:
                for name, body in _kernel_bodies(f.read()).items():
                    fp[name] = hashlib.sha256(body.encode()).hexdigest()
    with open(KERNELS_JSON + ".tmp", "w") as f:
        json.dump(fp, f, indent=1, sort_keys=True)
    os.replace(KERNELS_JSON + ".tmp", KERNELS_JSON)
    return KERNELS_JSON


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libhr.so (always recompiles), and write
    the kernels' assembly fingerprints."""
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
    kernel_fingerprints(verbose)
    return LIB


EXAMPLES = ["reduce_block.hip", "stencil3.hip", "histogram.hip", "wave_reduce.hip",
            "tile_reduce.hip", "cg_reduce.hip"]
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
