"""ctypes binding of libhr.so (the C ABI in include/hr.h).

Argument marshalling only: every step of the checking path runs in the HIP
kernels of the library.  PyTorch supplies device memory and streams.  There
is no fallback: if libhr.so is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhr.so")

HR_OK = 0
HR_W_CLOCK_OVERFLOW = 1
HR_W_RING_OVERFLOW = 2
HR_W_OUT_OF_RANGE = 4
HR_W_STALLED = 8
HR_W_REPORT_LIMITED = 16
HR_W_FOLDED = 32
HR_W_LOG_TRUNCATED = 64
HR_W_PARTIAL_BARRIER = 128
HR_RACE_FOLD, HR_RACE_SCANNED = 1, 2
HR_S_INIT, HR_S_RACE, HR_S_BLOCKS, HR_S_WAVES, HR_S_THREADS, HR_S_THREAD, HR_S_TILES = range(7)
HR_E_INVAL, HR_E_NOMEM, HR_E_HIP, HR_E_STATE = -1, -2, -3, -4
HR_GLOBAL, HR_LDS = 0, 1
HR_READ, HR_WRITE, HR_ATOMIC = 0, 1, 2
HR_CFG_COUNT_CHECKS = 1
HR_CFG_WAVE_GROUPING = 2
HR_CFG_WORD4 = 4
HR_CFG_ACCESS_LOG = 8
HR_CFG_NESTED_TILES = 16
HR_CFG_FSM_TABLE = 32
HR_CFG_FSM_TABLE_LDS = 64
NO_REGION = 0xFFFFFFFF
HR_PAT_REDUCE, HR_PAT_JACOBI, HR_PAT_LABELPROP = 0, 1, 2
HR_SITES = 256
HR_TILE_LOG2_MAX = 4
# the static scratch array of hr_job_run_static
HR_STATIC_SCRATCH_BYTES = 64 << 20
HR_STATIC_RING_RECORDS = 16384
HR_STATIC_SHADOW_WORDS = 8289280
# call-site ids of the workloads' race records (the enum in hr.h)
SITES = {
    "HR_SITE_REDUCE_LOAD": 1, "HR_SITE_REDUCE_STAGE": 2, "HR_SITE_REDUCE_LEFT": 3,
    "HR_SITE_REDUCE_RIGHT": 4, "HR_SITE_REDUCE_SUM": 5, "HR_SITE_REDUCE_TOTAL": 6,
    "HR_SITE_REDUCE_OUT": 7,
    "HR_SITE_JACOBI_CENTRE": 16, "HR_SITE_JACOBI_HALO": 17, "HR_SITE_JACOBI_STAGE": 18,
    "HR_SITE_JACOBI_TILE": 19, "HR_SITE_JACOBI_OUT": 20, "HR_SITE_JACOBI_SEED": 21,
    "HR_SITE_LP_OWN": 32, "HR_SITE_LP_CSR": 33, "HR_SITE_LP_MIN": 34,
    "HR_SITE_LP_SEED_READ": 35, "HR_SITE_LP_SEED_WRITE": 36,
}
globals().update(SITES)

# Global shadow-word fields (see csrc/hr_fsm.h), for decoding in tests.
T_INIT, T_RACE, T_MB, T_MW, T_MT, T_ST = 0, 1, 2, 3, 4, 5

RACE_DTYPE = np.dtype([("space", np.uint8), ("kind", np.uint8), ("site", np.uint16),
                       ("region", np.uint32), ("block", np.uint32), ("launch", np.uint32),
                       ("index", np.uint64), ("before", np.uint64), ("with", np.uint64),
                       ("tid", np.uint32), ("flags", np.uint32)])
assert RACE_DTYPE.itemsize == 48
# hr_access_rec: one checked access of the debug access log
ACCESS_DTYPE = np.dtype([("index", np.uint64), ("region", np.uint32), ("block", np.uint32),
                         ("launch", np.uint32), ("thread", np.uint16), ("space", np.uint8),
                         ("kind", np.uint8), ("bc", np.uint8), ("wc", np.uint8),
                         ("site", np.uint16), ("tc", np.uint32)])
assert ACCESS_DTYPE.itemsize == 32


class HRError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed with status {status}")
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [("ring_capacity", ctypes.c_uint32), ("bc_bits", ctypes.c_uint32),
                ("wc_bits", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("shadow_budget", ctypes.c_uint64), ("site_limit", ctypes.c_uint32),
                ("wave_bits", ctypes.c_uint32), ("thread_bits", ctypes.c_uint32),
                ("coalesce_width", ctypes.c_uint32), ("log_capacity", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class Summary(ctypes.Structure):
    """hr_summary: a decoded shadow summary (UINT32_MAX: field not kept)."""
    _fields_ = [(f, ctypes.c_uint32) for f in
                ("state", "class_launch", "class_block", "class_wave", "launch", "block", "bc",
                 "wave", "wc", "thread")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SummaryNested(ctypes.Structure):
    """hr_summary_nested: a decoded summary of a context with tiles nested
    in waves (UINT32_MAX: field not kept)."""
    _fields_ = [(f, ctypes.c_uint32) for f in
                ("state", "class_launch", "class_block", "class_wave", "class_tile", "launch",
                 "block", "bc", "wave", "wc", "tile", "tc", "thread")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Instance(ctypes.Structure):
    """hr_instance: one checked job of a batch (see include/hr.h)."""
    _fields_ = [("pattern", ctypes.c_uint32), ("blocks", ctypes.c_uint32),
                ("threads", ctypes.c_uint32), ("phases", ctypes.c_uint32),
                ("n", ctypes.c_uint32), ("ny", ctypes.c_uint32), ("drop", ctypes.c_int32),
                ("region", ctypes.c_uint32 * 2), ("pad", ctypes.c_uint32),
                ("data", ctypes.c_void_p * 4)]


class _Tuning(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_uint32), ("order", ctypes.c_uint32),
                ("spin_limit", ctypes.c_uint32), ("variant", ctypes.c_uint32),
                ("coalesce", ctypes.c_uint32), ("tile", ctypes.c_uint32)]


class ServeJob(ctypes.Structure):
    """hr_serve_job: arrival time in, admission/finish times and counts out."""
    _fields_ = [("arrival_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("finish_s", ctypes.c_double), ("flagged", ctypes.c_uint32),
                ("status", ctypes.c_int32)]


class _ServeConfig(ctypes.Structure):
    _fields_ = [("shadow_budget", ctypes.c_uint64), ("max_slots", ctypes.c_uint32),
                ("serial", ctypes.c_uint32), ("max_items", ctypes.c_uint32),
                ("large_burst", ctypes.c_uint32), ("lane_burst", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


SERVE_MAX_ITEMS = (1 << 22) - 1    # work items of one serving iteration (one launch)

assert ctypes.sizeof(Instance) == 72
assert ctypes.sizeof(ServeJob) == 32
assert ctypes.sizeof(_ServeConfig) == 32


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # Load PyTorch's HIP runtime first: libhr.so then binds to that same
    # libamdhip64.so.7 (matched by soname), so device pointers and streams
    # handed over by PyTorch are valid in the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, u32, u64, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                            ctypes.c_size_t)
    sigs = {
        "hr_ctx_create": [P, P, P],
        "hr_ctx_destroy": [P],
        "hr_shadow_alloc": [P, P, sz, u32, P],
        "hr_shadow_alloc_2d": [P, P, u32, u32, u32, u32, u32, P],
        "hr_shadow_free": [P, u32],
        "hr_region_enable": [P, u32, u32],
        "hr_dev_args": [P, P, sz, P],
        "hr_kernel_end": [P, P],
        "hr_reset": [P, P],
        "hr_report": [P, P, sz, P, P],
        "hr_check_count": [P, P, P],
        "hr_access_log": [P, P, sz, P, P],
        "hr_fsm_step": [u32, u64, u32, u32, u32, u32, u32, u32, u32, P],
        "hr_fsm_step_table": [u32, u64, u32, u32, u32, u32, u32, u32, u32, P],
        "hr_fsm_merge": [u64, u64, u32, P],
        "hr_fsm_step_nested": [u32, u64, u32, u32, u32, u32, u32, u32, u32, u32, P],
        "hr_fsm_merge_nested": [u64, u64, u32, P],
        "hr_describe": [u32, u64, u32, P],
        "hr_describe_nested": [u32, u64, u32, P],
        "hr_fsm_step_word4": [u32, u32, u32, u32, u32, u32, u32, u32, u32, u32, P],
        "hr_word4_widen": [u32, u32, u32, u32, P],
        "hr_reduce_check": [P, u32, u32, P, P, u32, u32, u32, ctypes.c_int32, P],
        "hr_reduce_plain": [P, P, u32, u32, u32, ctypes.c_int32, P],
        "hr_jacobi_check": [P, u32, u32, P, P, u32, u32, P, P],
        "hr_jacobi_plain": [P, P, u32, u32, P, P],
        "hr_labelprop_check": [P, u32, u32, u32, P, P, P, P, u32, u32, P],
        "hr_labelprop_plain": [P, P, P, P, u32, u32, P],
        "hr_program_check": [P, P, u32, u32, u32, u32, P, P, P, sz, P, sz, P, u32, P],
        "hr_batch_create": [P, P, u32, P],
        "hr_batch_run": [P, P, P],
        "hr_batch_info": [P, u32, P, P],
        "hr_batch_destroy": [P],
        "hr_job_run": [P, P, P, sz, P, P],
        "hr_job_run_static": [P, P, P, sz, P, P],
        "hr_serve": [P, P, P, u32, P, P, sz, P, P],
        "hr_peak_copy": [P, P, sz, P],
        "hr_peak_atomic": [P, sz, u32, u32, u32, P, u32, P],
        "hr_peak_load": [P, sz, u32, P, P],
        "hr_peak_lds": [u32, u32, u32, P, P],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = i32
    return lib


_lib = _load()
EXPORTED = ("hr_ctx_create", "hr_ctx_destroy", "hr_shadow_alloc", "hr_shadow_alloc_2d",
            "hr_shadow_free",
            "hr_region_enable",
            "hr_dev_args", "hr_batch_create", "hr_batch_run", "hr_batch_info",
            "hr_batch_destroy", "hr_job_run", "hr_job_run_static", "hr_serve",
            "hr_kernel_end", "hr_reset", "hr_report", "hr_check_count", "hr_access_log",
            "hr_fsm_step", "hr_fsm_step_table", "hr_fsm_merge", "hr_fsm_step_nested",
            "hr_fsm_merge_nested",
            "hr_describe", "hr_describe_nested", "hr_fsm_step_word4", "hr_word4_widen",
            "hr_reduce_check", "hr_reduce_plain", "hr_jacobi_check", "hr_jacobi_plain",
            "hr_labelprop_check", "hr_labelprop_plain", "hr_program_check",
            "hr_peak_copy", "hr_peak_atomic", "hr_peak_load", "hr_peak_lds")


def lib():
    return _lib


def _check(fn: str, st: int) -> int:
    if st < 0:
        raise HRError(fn, st)
    return st


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def fsm_step(space: int, old: int, kind: int, launch: int, block: int, thread: int,
             bc: int, wc: int, wave_bits: int = 6) -> int:
    """Host evaluation of the device transition function (verification aid);
    wave_bits < 6 makes tiles of 2**wave_bits lanes the synchronization
    groups (wc then counts tile barriers)."""
    out = ctypes.c_uint64(0)
    _check("hr_fsm_step", _lib.hr_fsm_step(space, old, kind, launch, block, thread, bc, wc,
                                           wave_bits, ctypes.byref(out)))
    return int(out.value)


def fsm_step_table(old: int, kind: int, launch: int, block: int, thread: int, bc: int, wc: int,
                   wave_bits: int = 6) -> int:
    """The global-word transition through the flat table (HR_CFG_FSM_TABLE);
    it must equal fsm_step(HR_GLOBAL, ...) on every input."""
    out = ctypes.c_uint64(0)
    _check("hr_fsm_step_table", _lib.hr_fsm_step_table(HR_GLOBAL, old, kind, launch, block,
                                                       thread, bc, wc, wave_bits,
                                                       ctypes.byref(out)))
    return int(out.value)


def fsm_step_nested(space: int, old: int, kind: int, launch: int, block: int, thread: int,
                    bc: int, wc: int, tc: int, tile_bits: int) -> int:
    """Host evaluation of the nested-tile machine's transition (verification)."""
    out = ctypes.c_uint64(0)
    _check("hr_fsm_step_nested", _lib.hr_fsm_step_nested(space, old, kind, launch, block, thread,
                                                         bc, wc, tc, tile_bits, ctypes.byref(out)))
    return int(out.value)


def fsm_merge_nested(x: int, y: int, tile_bits: int) -> int:
    out = ctypes.c_uint64(0)
    _check("hr_fsm_merge_nested", _lib.hr_fsm_merge_nested(x, y, tile_bits, ctypes.byref(out)))
    return int(out.value)


def describe(space: int, word: int, wave_bits: int = 6) -> dict:
    """Decode a shadow summary word (a race record's `before` or `with`)."""
    out = Summary()
    _check("hr_describe", _lib.hr_describe(space, word, wave_bits, ctypes.byref(out)))
    return out.as_dict()


def describe_nested(space: int, word: int, tile_bits: int) -> dict:
    """Decode a shadow summary word of a context with tiles of 2**tile_bits
    lanes nested in waves."""
    out = SummaryNested()
    _check("hr_describe_nested", _lib.hr_describe_nested(space, word, tile_bits,
                                                         ctypes.byref(out)))
    return out.as_dict()


def fsm_step_word4(old: int, kind: int, block: int, thread: int, bc: int, wc: int,
                   wave_bits: int = 6, wc_bits: int = 0, bc_bits: int = 0,
                   thread_bits: int = 0) -> int:
    """Host evaluation of the device transition on a 4-byte global word with
    the given field widths (0: the defaults 1, 2, 8)."""
    out = ctypes.c_uint32(0)
    _check("hr_fsm_step_word4", _lib.hr_fsm_step_word4(old, kind, block, thread, bc, wc,
                                                       wave_bits, wc_bits, bc_bits, thread_bits,
                                                       ctypes.byref(out)))
    return int(out.value)


def word4_widen(word: int, wc_bits: int = 0, bc_bits: int = 0, thread_bits: int = 0) -> int:
    """The 8-byte word of the summary a 4-byte word holds (launch 0)."""
    out = ctypes.c_uint64(0)
    _check("hr_word4_widen", _lib.hr_word4_widen(word, wc_bits, bc_bits, thread_bits,
                                                 ctypes.byref(out)))
    return int(out.value)


def fsm_merge(x: int, y: int, wave_bits: int = 6) -> int:
    """Host evaluation of the device summary merge (verification aid)."""
    out = ctypes.c_uint64(0)
    _check("hr_fsm_merge", _lib.hr_fsm_merge(x, y, wave_bits, ctypes.byref(out)))
    return int(out.value)


# ---------------------------------------------------------------- plain runs
def reduce_plain(inp, out, drop=-1, n=512, threads=256, blocks=1, stream=None):
    _check("hr_reduce_plain", _lib.hr_reduce_plain(_dptr(inp), _dptr(out), n, threads, blocks,
                                                   int(drop), _stream_ptr(stream)))


def jacobi_plain(u_old, u_new, seeds=None, stream=None):
    ny, nx = u_old.shape
    _check("hr_jacobi_plain", _lib.hr_jacobi_plain(_dptr(u_old), _dptr(u_new), ny, nx,
                                                   _dptr(seeds), _stream_ptr(stream)))


def labelprop_plain(label, row_ptr, col, mask, tpb=256, stream=None):
    n = label.shape[0]
    _check("hr_labelprop_plain", _lib.hr_labelprop_plain(_dptr(label), _dptr(row_ptr), _dptr(col),
                                                         _dptr(mask), n, tpb, _stream_ptr(stream)))


def peak_copy(src, dst, stream=None):
    _check("hr_peak_copy", _lib.hr_peak_copy(_dptr(src), _dptr(dst), src.numel() * src.element_size(),
                                             _stream_ptr(stream)))


def peak_atomic(words, op, rnd, scatter, fails, blocks=0, stream=None):
    _check("hr_peak_atomic", _lib.hr_peak_atomic(_dptr(words), words.numel(), op, rnd, scatter,
                                                 _dptr(fails), blocks, _stream_ptr(stream)))


def peak_lds(blocks, iters, op, fails, stream=None):
    _check("hr_peak_lds", _lib.hr_peak_lds(blocks, iters, op, _dptr(fails), _stream_ptr(stream)))


def peak_load(words, scatter, sink, stream=None):
    _check("hr_peak_load", _lib.hr_peak_load(_dptr(words), words.numel(), scatter, _dptr(sink),
                                             _stream_ptr(stream)))


class DeviceProgram:
    """One launch of an access program, uploaded to device memory."""

    def __init__(self, launch, device="cuda"):
        import torch
        self.blocks, self.threads, self.phases = launch.blocks, launch.threads, launch.phases
        self.scope = torch.from_numpy(np.ascontiguousarray(launch.scope, np.uint8)).to(device)
        self.wmask = torch.from_numpy(
            np.ascontiguousarray(launch.wave_mask, np.uint64).view(np.int64)).to(device)
        self.op_off = torch.from_numpy(np.ascontiguousarray(launch.op_off, np.int32)).to(device)
        ops = np.ascontiguousarray(launch.ops, np.uint32)
        if ops.size == 0:
            ops = np.zeros(1, np.uint32)
            self.n_ops = 0
        else:
            self.n_ops = ops.size
        self.ops = torch.from_numpy(ops.view(np.int32)).to(device)


class Context:
    """A checking job: shadow regions, report ring, launch epochs.  The
    arguments are the fields of hr_config; word4=True selects 4-byte global
    shadow words (HR_CFG_WORD4), whose thread field is thread_bits wide;
    nested_tiles=True (HR_CFG_NESTED_TILES) makes tiles of 2**wave_bits
    lanes with their own barriers nested in whole waves; fsm_table=True
    (HR_CFG_FSM_TABLE) reads the global-word transitions from the machine's
    flat table in device memory, fsm_table="lds" (HR_CFG_FSM_TABLE_LDS) from
    a copy in each block's LDS in the stencil kernel."""

    def __init__(self, ring_capacity=0, bc_bits=0, wc_bits=0, count_checks=False,
                 shadow_budget=0, wave_grouping=False, site_limit=0, wave_bits=0,
                 word4=False, thread_bits=0, coalesce_width=0, access_log=False,
                 log_capacity=0, nested_tiles=False, fsm_table=False, stream=None):
        flags = (HR_CFG_COUNT_CHECKS if count_checks else 0) | \
                (HR_CFG_WAVE_GROUPING if wave_grouping else 0) | \
                (HR_CFG_WORD4 if word4 else 0) | \
                (HR_CFG_ACCESS_LOG if access_log else 0) | \
                (HR_CFG_NESTED_TILES if nested_tiles else 0) | \
                (HR_CFG_FSM_TABLE if fsm_table else 0) | \
                (HR_CFG_FSM_TABLE_LDS if fsm_table == "lds" else 0)
        cfg = _Config(ring_capacity, bc_bits, wc_bits, flags, shadow_budget, site_limit,
                      wave_bits, thread_bits, coalesce_width, log_capacity, 0)
        self.wave_bits = wave_bits or 6
        self._c = ctypes.c_void_p(0)
        self._stream = _stream_ptr(stream)
        _check("hr_ctx_create", _lib.hr_ctx_create(ctypes.byref(self._c), ctypes.byref(cfg),
                                                   self._stream))
        self.status = 0

    def close(self):
        if self._c:
            _check("hr_ctx_destroy", _lib.hr_ctx_destroy(self._c))
            self._c = ctypes.c_void_p(0)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._c

    def shadow_alloc(self, tensor, tile=None) -> int:
        """Monitor `tensor`.  tile=(tw, th): a 2-D tensor's shadow words in
        tiles of 2**tw columns by 2**th rows (hr_shadow_alloc_2d); None or
        (0, 0) keeps the row-major map."""
        if not (tensor.is_cuda and tensor.element_size() == 4 and tensor.is_contiguous()):
            raise ValueError("shadow_alloc needs a contiguous device tensor of 4-byte elements")
        r = ctypes.c_uint32(0)
        if tile is not None:
            if tensor.dim() != 2:
                raise ValueError("a tiled shadow map needs a 2-D tensor")
            rows, cols = tensor.shape
            _check("hr_shadow_alloc_2d", _lib.hr_shadow_alloc_2d(
                self._c, _dptr(tensor), rows, cols, 4, tile[0], tile[1], ctypes.byref(r)))
            return int(r.value)
        _check("hr_shadow_alloc", _lib.hr_shadow_alloc(self._c, _dptr(tensor),
                                                       tensor.numel() * 4, 4, ctypes.byref(r)))
        return int(r.value)

    def dev_args(self) -> bytes:
        size = ctypes.c_size_t(0)
        _lib.hr_dev_args(self._c, None, 0, ctypes.byref(size))
        buf = ctypes.create_string_buffer(size.value)
        _check("hr_dev_args", _lib.hr_dev_args(self._c, buf, size.value, ctypes.byref(size)))
        return buf.raw

    def kernel_end(self, stream=None):
        _check("hr_kernel_end", _lib.hr_kernel_end(self._c, _stream_ptr(stream)))

    def reset(self, stream=None):
        _check("hr_reset", _lib.hr_reset(self._c, _stream_ptr(stream)))

    def report(self, stream=None):
        """Flagged records (RACE_DTYPE array) and the warning bits."""
        n = ctypes.c_size_t(0)
        cap = 4096
        while True:
            out = np.zeros(cap, dtype=RACE_DTYPE)
            st = _lib.hr_report(self._c, out.ctypes.data_as(ctypes.c_void_p), cap,
                                ctypes.byref(n), _stream_ptr(stream))
            if st == HR_E_INVAL and n.value > cap:
                cap = int(n.value)
                continue
            _check("hr_report", st)
            self.status = st
            return out[:n.value], st

    def flagged(self, stream=None) -> set:
        recs, _ = self.report(stream)
        return {(int(r["space"]), int(r["region"]),
                 int(r["block"]) if r["space"] == HR_LDS else 0, int(r["index"]))
                for r in recs}

    def check_count(self, stream=None) -> int:
        out = ctypes.c_uint64(0)
        _check("hr_check_count", _lib.hr_check_count(self._c, ctypes.byref(out),
                                                     _stream_ptr(stream)))
        return int(out.value)

    # ------------------------------------------------------- workloads
    def access_log(self, stream=None):
        """The debug access log (a context made with access_log=True): one
        ACCESS_DTYPE record per checked access, unordered.  Returns
        (records, warning bits)."""
        n = ctypes.c_size_t(0)
        st = _lib.hr_access_log(self._c, None, 0, ctypes.byref(n), _stream_ptr(stream))
        if st == HR_E_INVAL and n.value == 0:
            _check("hr_access_log", st)
        out = np.zeros(n.value, dtype=ACCESS_DTYPE)
        st = _lib.hr_access_log(self._c, out.ctypes.data_as(ctypes.c_void_p), n.value,
                                ctypes.byref(n), _stream_ptr(stream))
        _check("hr_access_log", st)
        return out[:n.value], st

    def shadow_free(self, region: int):
        _check("hr_shadow_free", _lib.hr_shadow_free(self._c, region))

    def region_enable(self, region: int, on: bool):
        """Monitor a region (on) or not, for the kernels launched afterwards."""
        _check("hr_region_enable", _lib.hr_region_enable(self._c, region, int(bool(on))))

    def reduce_check(self, r_in, r_out, inp, out, drop=-1, n=512, threads=256, blocks=1,
                     stream=None):
        _check("hr_reduce_check", _lib.hr_reduce_check(self._c, r_in, r_out, _dptr(inp),
                                                       _dptr(out), n, threads, blocks, int(drop),
                                                       _stream_ptr(stream)))

    def jacobi_check(self, r_old, r_new, u_old, u_new, seeds=None, stream=None):
        ny, nx = u_old.shape
        _check("hr_jacobi_check", _lib.hr_jacobi_check(self._c, r_old, r_new, _dptr(u_old),
                                                       _dptr(u_new), ny, nx, _dptr(seeds),
                                                       _stream_ptr(stream)))

    def labelprop_check(self, r_label, label, row_ptr, col, mask, tpb=256,
                        r_row_ptr=NO_REGION, r_col=NO_REGION, stream=None):
        n = label.shape[0]
        _check("hr_labelprop_check", _lib.hr_labelprop_check(
            self._c, r_label, r_row_ptr, r_col, _dptr(label), _dptr(row_ptr), _dptr(col),
            _dptr(mask), n, tpb, _stream_ptr(stream)))

    def program_check(self, prog: DeviceProgram, regions, lds_words, block_map=None,
                      stream=None):
        regs = (ctypes.c_uint32 * max(1, len(regions)))(*regions)
        _check("hr_program_check", _lib.hr_program_check(
            self._c, regs, len(regions), prog.blocks, prog.threads, prog.phases,
            _dptr(prog.scope), _dptr(prog.wmask), _dptr(prog.op_off), prog.op_off.numel(),
            _dptr(prog.ops), prog.n_ops, _dptr(block_map), lds_words, _stream_ptr(stream)))


def _races_to_keys(recs):
    return {(int(r["space"]), int(r["region"]),
             int(r["block"]) if r["space"] == HR_LDS else 0, int(r["index"])) for r in recs}


def job_run(inst: Instance, ring_capacity=0, stream=None, static=False, site_limit=0,
            records=False):
    """The serial path for one job (own context and shadow, synchronous), or
    with static=True its variant over the library's static scratch array
    (hr_job_run_static, no allocation).  Returns (flagged keys with region
    ids 0/1, warning bits), or (race records, warning bits) with records."""
    cfg = _Config(ring_capacity, 0, 0, 0, 0, site_limit, 0)
    fn_name = "hr_job_run_static" if static else "hr_job_run"
    fn = getattr(_lib, fn_name)
    n = ctypes.c_size_t(0)
    cap = 4096
    while True:
        out = np.zeros(cap, dtype=RACE_DTYPE)
        st = fn(ctypes.byref(inst), ctypes.byref(cfg), out.ctypes.data_as(ctypes.c_void_p), cap,
                ctypes.byref(n), _stream_ptr(stream))
        if st == HR_E_INVAL and n.value > cap:
            cap = int(n.value)
            continue
        _check(fn_name, st)
        if records:
            return out[:n.value].copy(), st
        return _races_to_keys(out[:n.value]), st


def serve(ctx: Context, instances, arrivals, shadow_budget=0, max_slots=0, serial=False,
          max_items=0, large_burst=0, lane_burst=0, stream=None):
    """Check a stream of jobs arriving at `arrivals` (seconds from the call,
    non-decreasing) with continuous batching, or one at a time (serial).
    max_items caps the work items (1024-thread blocks) of one iteration
    (0: SERVE_MAX_ITEMS); large_burst: phases of a large stencil job per
    iteration of the large-job lane (0: all remaining); lane_burst: phases
    per iteration of the short-job lane (0: 2).  Returns (per-job flagged keys with job-local
    region ids 0/1, ServeJob array with admission/finish times, flagged
    counts and warning bits)."""
    n = len(instances)
    inst = (Instance * n)(*instances)
    times = (ServeJob * n)()
    for j, a in enumerate(arrivals):
        times[j].arrival_s = float(a)
    cfg = _ServeConfig(int(shadow_budget), int(max_slots), int(bool(serial)), int(max_items),
                       int(large_burst), int(lane_burst), 0)
    cnt = ctypes.c_size_t(0)
    cap = 1 << 20          # a larger count re-runs the whole stream
    while True:
        out = np.zeros(cap, dtype=RACE_DTYPE)
        st = _lib.hr_serve(ctx.handle, inst, times, n, ctypes.byref(cfg),
                           out.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(cnt),
                           _stream_ptr(stream))
        if st == HR_E_INVAL and cnt.value > cap:
            cap = int(cnt.value)
            continue
        _check("hr_serve", st)
        break
    per = [set() for _ in range(n)]
    for r in out[:cnt.value]:
        j, k = divmod(int(r["region"]), 2)
        lds = r["space"] == HR_LDS
        per[j].add((int(r["space"]), 0 if lds else k, int(r["block"]) if lds else 0,
                    int(r["index"])))
    return per, times


class Batch:
    """Many checked jobs run to completion in one persistent launch."""

    def __init__(self, ctx: Context, instances):
        self.ctx = ctx
        self.n = len(instances)
        self.inst = (Instance * self.n)(*instances)
        self._b = ctypes.c_void_p(0)
        _check("hr_batch_create", _lib.hr_batch_create(ctx.handle, self.inst, self.n,
                                                       ctypes.byref(self._b)))

    def regions(self, i):
        return tuple(self.inst[i].region)

    def info(self, variant=0):
        w, it = ctypes.c_uint32(0), ctypes.c_uint64(0)
        _check("hr_batch_info", _lib.hr_batch_info(self._b, variant, ctypes.byref(w),
                                                   ctypes.byref(it)))
        return int(w.value), int(it.value)

    def run(self, workers=0, order=0, variant=0, spin_limit=0, coalesce=0, tile=None,
            stream=None):
        """coalesce: wave grouping at data-dependent sites, 0 the context's
        setting, 1 off, else the coalescing width (2..64 lanes).  tile=(tw,
        th): the stencil jobs' shadow map (None: row-major)."""
        t = _Tuning(workers, order, spin_limit, variant, coalesce,
                    0 if tile is None else (tile[0] | tile[1] << 4))
        _check("hr_batch_run", _lib.hr_batch_run(self._b, ctypes.byref(t), _stream_ptr(stream)))

    def split(self, keys):
        """Per-job flagged keys, with job-local region ids (0 and 1, as the
        serial path reports them)."""
        owner = {}
        for i in range(self.n):
            for k, r in enumerate(self.inst[i].region):
                if r != NO_REGION:
                    owner[r] = (i, k)
        per = [set() for _ in range(self.n)]
        for sp, rg, blk, ix in keys:
            i, k = owner[rg]
            per[i].add((sp, k if sp == HR_GLOBAL else 0, blk, ix))
        return per

    def close(self):
        if self._b:
            _check("hr_batch_destroy", _lib.hr_batch_destroy(self._b))
            self._b = ctypes.c_void_p(0)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
