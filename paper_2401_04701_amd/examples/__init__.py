"""Example kernels rewritten by the source instrumenter (see instrument.py),
compiled by build.build_examples into libhr_examples.so, and a ctypes binding
of their launchers: hr_launch_<kernel>(ctx, regions, n_regions, grid, block,
lds_bytes, stream, <kernel parameters>)."""
from __future__ import annotations

import ctypes
import os

from .. import hr

LIB_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "libhr_examples.so")
_lib = None

P, u32, i32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32, ctypes.c_size_t
_COMMON = [P, P, u32, u32, u32, u32, u32, u32, u32, sz, P]
_PARAMS = {
    "reduce_block": [P, P, i32],
    "stencil3": [P, P, i32, i32],
    "histogram": [P, P, i32, i32],
    "wave_reduce": [P, P, i32],
    "tile_reduce": [P, P, i32, i32, i32],
    "cg_reduce": [P, P, i32, i32],
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        _lib = ctypes.CDLL(LIB_PATH)     # libhr.so is loaded first, by the hr import
        for name, extra in _PARAMS.items():
            fn = getattr(_lib, f"hr_launch_{name}")
            fn.argtypes = _COMMON + extra
            fn.restype = ctypes.c_int
    return _lib


def launch(name: str, ctx: hr.Context, regions, grid, block, *args, lds=0, stream=None):
    """Launch instrumented kernel `name`; regions: context region of each of
    its pointer parameters, in order; args: its parameters (tensors are
    passed as device pointers)."""
    regs = (ctypes.c_uint32 * max(1, len(regions)))(*regions)
    g = tuple(grid) + (1,) * (3 - len(grid))
    b = tuple(block) + (1,) * (3 - len(block))
    conv = [hr._dptr(a) if hasattr(a, "data_ptr") else a for a in args]
    st = getattr(lib(), f"hr_launch_{name}")(ctx.handle, regs, len(regions), *g, *b, lds,
                                              hr._stream_ptr(stream), *conv)
    hr._check(f"hr_launch_{name}", st)
