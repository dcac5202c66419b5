"""Race-check oracle -- test infrastructure, not part of the checker.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  It shares no code with the HIP checker: the plain C
pairwise check and workload access models live in ``oracle.c`` (built with
gcc into ``liboracle.so``), the schedule brute force in ``brute.py`` and the
closed-form flagged sets in ``closed_forms.py``.

A flagged key is ``(space, region, lds_block, index)``: space 0 is global
memory and 1 is LDS; ``lds_block`` is the owning block of an LDS location and
0 for global memory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib_handle = None

REC_DTYPE = np.dtype([
    ("index", np.uint64), ("space", np.uint32), ("region", np.uint32),
    ("lds_block", np.uint32), ("kind", np.uint32), ("launch", np.uint32),
    ("block", np.uint32), ("thread", np.uint32), ("bc", np.uint32),
    ("wc", np.uint32), ("tc", np.uint32)])
KEY_DTYPE = np.dtype([("index", np.uint64), ("space", np.uint32),
                      ("region", np.uint32), ("lds_block", np.uint32),
                      ("pad", np.uint32)])
assert REC_DTYPE.itemsize == 48 and KEY_DTYPE.itemsize == 24


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        u32, u64, sz, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
        lib.orc_flagged.argtypes = [P, sz, u32, P, sz, ctypes.POINTER(sz)]
        lib.orc_flagged.restype = i32
        lib.orc_race_pair.argtypes = [P, P, u32]
        lib.orc_race_pair.restype = i32
        lib.orc_model_reduce.argtypes = [i32, u32, P, sz]
        lib.orc_model_reduce.restype = sz
        lib.orc_model_reduce_n.argtypes = [u32, u32, u32, i32, u32, P, sz]
        lib.orc_model_reduce_n.restype = sz
        lib.orc_model_jacobi.argtypes = [u32, u32, u32, u32, P, u32, u32, u32, u32, P, sz]
        lib.orc_model_jacobi.restype = sz
        lib.orc_model_labelprop.argtypes = [u32, P, P, P, u32, u32, u32, i32, P, P, sz]
        lib.orc_model_labelprop.restype = sz
        lib.orc_model_launch.argtypes = [u32, u32, u32, u32, P, P, P, P, u32, P, sz]
        lib.orc_model_launch.restype = sz
        lib.orc_flagged_nested.argtypes = [P, sz, u32, u32, P, sz, ctypes.POINTER(sz)]
        lib.orc_flagged_nested.restype = i32
        lib.orc_race_pair_nested.argtypes = [P, P, u32, u32]
        lib.orc_race_pair_nested.restype = i32
        lib.orc_model_launch_nested.argtypes = [u32, u32, u32, u32, P, P, P, P, u32, u32, P, sz]
        lib.orc_model_launch_nested.restype = sz
        _lib_handle = lib
    return _lib_handle


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
def flagged(recs: np.ndarray, wave_width: int = 64, tile_width: int = 0) -> set:
    """Set of racy keys of an access log (REC_DTYPE array; sorted in place).
    tile_width: tiles of that many lanes nested in the waves, with their own
    barriers and tile epochs (the records' tc); 0: none."""
    recs = np.ascontiguousarray(recs, dtype=REC_DTYPE)
    lib = _lib()
    n_out = ctypes.c_size_t(0)
    cap = 1024
    while True:
        out = np.zeros(cap, dtype=KEY_DTYPE)
        rc = lib.orc_flagged_nested(_ptr(recs), recs.shape[0], wave_width, tile_width,
                                    _ptr(out), cap, ctypes.byref(n_out))
        if rc == 0:
            break
        cap = int(n_out.value)
    out = out[:n_out.value]
    return {(int(k["space"]), int(k["region"]), int(k["lds_block"]), int(k["index"]))
            for k in out}


def race_pair(p: np.ndarray, c: np.ndarray, wave_width: int = 64, tile_width: int = 0) -> bool:
    p = np.ascontiguousarray(p, dtype=REC_DTYPE).reshape(1)
    c = np.ascontiguousarray(c, dtype=REC_DTYPE).reshape(1)
    return bool(_lib().orc_race_pair_nested(_ptr(p), _ptr(c), wave_width, tile_width))


def make_records(rows) -> np.ndarray:
    """Records from tuples (space, region, index, kind, launch, block, thread,
    bc, wc); the LDS owning block is the accessing block."""
    recs = np.zeros(len(rows), dtype=REC_DTYPE)
    for i, (sp, rg, ix, kd, la, bl, th, bc, wc) in enumerate(rows):
        recs[i] = (ix, sp, rg, bl if sp == 1 else 0, kd, la, bl, th, bc, wc, 0)
    return recs


# --------------------------------------------------------------------------
def _run_model(fn, *args):
    n = fn(*args, None, 0)
    out = np.zeros(n, dtype=REC_DTYPE)
    m = fn(*args, _ptr(out), n)
    assert m == n
    return out


def model_reduce(drop: int = -1, launch: int = 0) -> np.ndarray:
    """Access log of the one-block LDS tree reduction (drop: barrier removed)."""
    return _run_model(_lib().orc_model_reduce, int(drop), int(launch))


def model_reduce_n(n: int, threads: int, blocks: int, drop: int = -1,
                   launch: int = 0) -> np.ndarray:
    """Access log of the scaled LDS tree reduction (n words per block)."""
    return _run_model(_lib().orc_model_reduce_n, n, threads, blocks, int(drop), int(launch))


def model_jacobi(ny: int, nx: int, launches: int, seed_tab=None, window=None,
                 launch0: int = 0) -> np.ndarray:
    """Access log of the Jacobi sweeps; window = (bx0, bx1, by0, by1)."""
    nby, nbx = (ny + 15) // 16, (nx + 15) // 16
    bx0, bx1, by0, by1 = window if window is not None else (0, nbx, 0, nby)
    tab = None if seed_tab is None else np.ascontiguousarray(seed_tab, dtype=np.int32)
    return _run_model(_lib().orc_model_jacobi, ny, nx, launch0, launches, _ptr(tab),
                      bx0, bx1, by0, by1)


def model_labelprop(row_ptr, col, mask, launches: int, tpb: int = 256,
                    monitor_csr: bool = False, keep=None, launch0: int = 0) -> np.ndarray:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    keep = None if keep is None else np.ascontiguousarray(keep, dtype=np.uint8)
    n = row_ptr.shape[0] - 1
    return _run_model(_lib().orc_model_labelprop, n, _ptr(row_ptr), _ptr(col), _ptr(mask),
                      launch0, launches, tpb, int(monitor_csr), _ptr(keep))


def model_launch(launch, index: int, wave_width: int = 64, tile_width: int = 0) -> np.ndarray:
    """Access log of one launch of an interpreted barrier program (tile
    barriers, scope 3, advance the tile epochs of tile_width-lane tiles)."""
    scope = np.ascontiguousarray(launch.scope, dtype=np.uint8)
    wm = np.ascontiguousarray(launch.wave_mask, dtype=np.uint64)
    off = np.ascontiguousarray(launch.op_off, dtype=np.int32)
    ops = np.ascontiguousarray(launch.ops, dtype=np.uint32)
    return _run_model(_lib().orc_model_launch_nested, index, launch.blocks, launch.threads,
                      launch.phases, _ptr(scope), _ptr(wm), _ptr(off), _ptr(ops),
                      wave_width, tile_width)


def model_program(program, wave_width: int = 64, tile_width: int = 0) -> np.ndarray:
    logs = [model_launch(l, i, wave_width, tile_width) for i, l in enumerate(program.launches)]
    return np.concatenate(logs) if logs else np.zeros(0, dtype=REC_DTYPE)


def flagged_program(program, wave_width: int = 64, tile_width: int = 0) -> set:
    return flagged(model_program(program, wave_width, tile_width), wave_width, tile_width)
