"""ctypes binding of libpms.so (include/pms.h).  Argument marshalling only.

Every computation runs in the library's GPU kernels.  If libpms.so has not
been built this module raises ImportError; there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpms.so")

PMS_OK, PMS_ERR_INVALID, PMS_ERR_OVERFLOW, PMS_ERR_NOMEM, PMS_ERR_DEVICE = range(5)
PMS_MAX_L, PMS_MAX_N, PMS_MAX_T = 16, 64, 1 << 17

SYMBOLS = ["pms_solve", "pms_solve_ex", "pms_solve_intersect", "pms_solve_many", "pms_decode", "pms_status_string", "pms_last_error",
           "pms_set_config", "pms_get_config", "pms_autotune", "pms_last_stats",
           "pms_window_stride", "pms_build_windows", "pms_step_launch", "pms_solve_dev",
           "pms_valu_probe", "pms_solve_dev_noalloc", "pms_shutdown",
           "pms_sort_codes", "pms_autotune_many", "pms_fill_work_items"]
PROBE_OPS = {"xor": 0, "bcnt": 1, "min3": 2, "or_sdwa": 3, "add": 4, "fma_f32": 5, "xor_vv": 6,
             "compare": 7, "mov_s": 8, "mov64_s": 9}


class PmsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)} ({status}): {message}")
        self.status = status
        self.message = message


class Instance(ctypes.Structure):
    _fields_ = [("seqs", ctypes.POINTER(ctypes.c_char_p)), ("n", ctypes.c_int32),
                ("t", ctypes.c_int32), ("l", ctypes.c_int32), ("d", ctypes.c_int32),
                ("out_motifs", ctypes.POINTER(ctypes.c_uint32)), ("capacity", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("count", ctypes.c_uint64), ("latency_ms", ctypes.c_double)]


def _record_dtype(struct) -> np.dtype:
    """The numpy record layout of a ctypes structure (same offsets and size),
    so that arrays of them can be filled and read without per-field calls."""
    kinds = {ctypes.c_int32: np.int32, ctypes.c_uint64: np.uint64, ctypes.c_double: np.float64}
    names, formats, offsets = [], [], []
    for name, ct in struct._fields_:
        names.append(name)
        formats.append(kinds.get(ct, np.uint64))   # pointers as addresses
        offsets.append(getattr(struct, name).offset)
    return np.dtype({"names": names, "formats": formats, "offsets": offsets,
                     "itemsize": ctypes.sizeof(struct)})


_INSTANCE_DT = _record_dtype(Instance)
_RESULT_DT = _record_dtype(Result)

VARIANT_AUTO, VARIANT_LANE, VARIANT_GROUP, VARIANT_GROUP64 = 0, 1, 2, 3
FILTER_DEFAULT, FILTER_ON, FILTER_OFF = 0, 1, 2
INPUT_MASK_N, INPUT_BOTH_STRANDS = 1, 2
VARIANT_NAMES = {1: "lane", 2: "group16", 3: "group64"}
LAYOUT_PLANES, LAYOUT_BITSLICED = 0, 1


class Config(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint32), ("wg_waves", ctypes.c_uint32),
                ("wgs_per_cu", ctypes.c_uint32), ("tail_split", ctypes.c_uint32),
                ("variant", ctypes.c_uint32), ("filter", ctypes.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("windows_ms", ctypes.c_double),
                ("seq_visits", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("window_compares", ctypes.c_uint64), ("candidate_slots", ctypes.c_uint64),
                ("grid", ctypes.c_uint32), ("wg_waves", ctypes.c_uint32),
                ("chunk", ctypes.c_uint32), ("reruns", ctypes.c_uint32),
                ("variant", ctypes.c_uint32), ("work_items", ctypes.c_uint32),
                ("host_prep_ms", ctypes.c_double), ("host_finish_ms", ctypes.c_double),
                ("single_batches", ctypes.c_uint64), ("filtered_batches", ctypes.c_uint64),
                ("filtered_groups", ctypes.c_uint64)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is ctypes.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


class ProbeResult(ctypes.Structure):
    _fields_ = [("lane_ops_per_s", ctypes.c_double), ("ms", ctypes.c_double),
                ("sclk_mhz", ctypes.c_double), ("lane_ops_per_clk_per_cu", ctypes.c_double),
                ("compute_units", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class DevInstance(ctypes.Structure):
    _fields_ = [("windows", ctypes.c_uint64), ("out", ctypes.c_uint64), ("out_cap", ctypes.c_uint64),
                ("n", ctypes.c_int32), ("nw_stride", ctypes.c_int32), ("l", ctypes.c_int32),
                ("d", ctypes.c_int32)]


class WorkItem(ctypes.Structure):
    _fields_ = [("begin", ctypes.c_uint64), ("len", ctypes.c_uint32), ("inst", ctypes.c_uint32)]


class DevState(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("visits", ctypes.c_uint64), ("t_done", ctypes.c_uint64),
                ("items_left", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class DevCounters(ctypes.Structure):
    _fields_ = [("next_item", ctypes.c_uint32), ("error", ctypes.c_uint32),
                ("batches", ctypes.c_uint64), ("t_start", ctypes.c_uint64),
                ("single_batches", ctypes.c_uint64), ("filtered_batches", ctypes.c_uint64),
                ("filtered_groups", ctypes.c_uint64)]


def _load():
    # torch ships its own HIP runtime and its libraries ask for it by the
    # name libamdhip64.so.  Loading torch first makes libpms.so bind to that
    # same runtime (matched by SONAME) instead of a second copy from
    # /opt/rocm, which would then see no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'` "
                          "or `python paper_1403_1313_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    u32p, u64p, vp = P(ctypes.c_uint32), P(ctypes.c_uint64), ctypes.c_void_p
    i32 = ctypes.c_int32
    sig = {
        "pms_solve": ([P(ctypes.c_char_p), i32, i32, i32, i32, u32p, u64p], ctypes.c_int),
        "pms_solve_ex": ([P(ctypes.c_char_p), i32, P(i32), i32, i32, ctypes.c_uint32, u32p, u64p],
                         ctypes.c_int),
        "pms_solve_intersect": ([P(ctypes.c_char_p), i32, i32, i32, i32, u32p, u64p], ctypes.c_int),
        "pms_solve_many": ([P(Instance), i32, P(Result)], ctypes.c_int),
        "pms_decode": ([ctypes.c_uint32, i32, ctypes.c_char_p], None),
        "pms_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "pms_last_error": ([], ctypes.c_char_p),
        "pms_set_config": ([P(Config)], ctypes.c_int),
        "pms_get_config": ([P(Config)], ctypes.c_int),
        "pms_autotune": ([i32, i32, i32, i32, ctypes.c_char_p, P(Config)], ctypes.c_int),
        "pms_last_stats": ([P(Stats)], ctypes.c_int),
        "pms_window_stride": ([i32, i32, i32], i32),
        "pms_build_windows": ([vp, i32, i32, i32, i32, vp, vp, vp], ctypes.c_int),
        "pms_step_launch": ([vp, i32, i32, vp, i32, vp, vp, P(Config), vp], ctypes.c_int),
        "pms_solve_dev": ([vp, i32, i32, i32, i32, vp, ctypes.c_uint64, vp, vp], ctypes.c_int),
        "pms_valu_probe": ([ctypes.c_int, i32, i32, P(ProbeResult)], ctypes.c_int),
        "pms_solve_dev_noalloc": ([vp, i32, i32, i32, i32, vp, ctypes.c_uint64, vp, vp], ctypes.c_int),
        "pms_shutdown": ([], ctypes.c_int),
        "pms_sort_codes": ([u32p, ctypes.c_uint64, i32], ctypes.c_int),
        "pms_autotune_many": ([P(Instance), i32, ctypes.c_char_p, P(Config)], ctypes.c_int),
        "pms_fill_work_items": ([ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                 vp, i32], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def shutdown() -> int:
    """pms_shutdown: releases the library's device resources (status code;
    a later call creates them again)."""
    return int(_lib.pms_shutdown())


# The library's streams, events, graph and buffers are released before the
# interpreter exits, so none of them outlives the HIP runtime's own teardown.
atexit.register(shutdown)


def lib():
    return _lib


def status_string(status: int) -> str:
    return _lib.pms_status_string(int(status)).decode()


def last_error() -> str:
    return _lib.pms_last_error().decode()


def _check(status: int, allow=(PMS_OK,)):
    if status not in allow:
        raise PmsError(status, last_error())
    return status


def _rows(seqs) -> Tuple[ctypes.Array, object, int, int]:
    """char* array for n rows (list of str/bytes or an (n, t) uint8 array).

    For an array the pointers address its rows directly; the second element
    returned keeps the memory they point into alive."""
    if isinstance(seqs, np.ndarray):
        m = np.ascontiguousarray(seqs, dtype=np.uint8)
        if m.ndim != 2:
            raise ValueError("sequence array must be 2-D (n, t)")
        n, t = int(m.shape[0]), int(m.shape[1])
        base = m.ctypes.data
        arr = (ctypes.c_char_p * max(n, 1))(*[base + i * t for i in range(n)])
        return arr, m, n, t
    rows = [s.encode() if isinstance(s, str) else bytes(s) for s in seqs]
    n = len(rows)
    t = len(rows[0]) if rows else 0
    arr = (ctypes.c_char_p * max(n, 1))(*rows) if n else (ctypes.c_char_p * 1)()
    return arr, rows, n, t


_tls = threading.local()


def _out_buffer(words: int) -> np.ndarray:
    """Per-thread output scratch reused across calls: results are copied out
    of it, so a call's buffer only has to outlive the call."""
    buf = getattr(_tls, "out", None)
    if buf is None or buf.size < words:
        buf = np.empty(max(words, 1), dtype=np.uint32)
        _tls.out = buf
    return buf


def solve_raw(seqs, l: int, d: int, capacity: Optional[int] = None, t: Optional[int] = None):
    """pms_solve: (status, count, motifs[:min(count, capacity)])."""
    arr, keep, n, t0 = _rows(seqs)
    t = t0 if t is None else t
    if capacity is None:
        capacity = 1 << 20
    out = _out_buffer(capacity)
    cnt = ctypes.c_uint64(capacity)
    st = _lib.pms_solve(arr, n, t, l, d, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
                        if capacity > 0 else None, ctypes.byref(cnt))
    del keep
    k = min(int(cnt.value), capacity)
    return st, int(cnt.value), out[:k].copy()


def solve(seqs, l: int, d: int) -> np.ndarray:
    """Sorted uint32 motif codes of one instance (regrows on overflow)."""
    st, cnt, res = solve_raw(seqs, l, d, capacity=1 << 16)
    if st == PMS_ERR_OVERFLOW:
        st, cnt, res = solve_raw(seqs, l, d, capacity=cnt)
    _check(st)
    return res


def solve_ex_raw(rows, l: int, d: int, mask_n: bool = False, both: bool = False,
                 capacity: Optional[int] = None):
    """pms_solve_ex over rows of their own lengths (list of str/bytes or 1-D
    uint8 arrays): (status, count, motifs[:min(count, capacity)])."""
    data = [r.encode() if isinstance(r, str) else
            (np.ascontiguousarray(r, dtype=np.uint8).tobytes() if isinstance(r, np.ndarray)
             else bytes(r)) for r in rows]
    n = len(data)
    arr = (ctypes.c_char_p * max(n, 1))(*data)
    lens = (ctypes.c_int32 * max(n, 1))(*[len(r) for r in data])
    if capacity is None:
        capacity = 1 << 20
    out = _out_buffer(capacity)
    cnt = ctypes.c_uint64(capacity)
    flags = (INPUT_MASK_N if mask_n else 0) | (INPUT_BOTH_STRANDS if both else 0)
    st = _lib.pms_solve_ex(arr, n, lens, l, d, flags,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if capacity > 0
                           else None, ctypes.byref(cnt))
    k = min(int(cnt.value), capacity)
    return st, int(cnt.value), out[:k].copy()


def solve_ex(rows, l: int, d: int, mask_n: bool = False, both: bool = False) -> np.ndarray:
    """Sorted uint32 motif codes of pms_solve_ex (regrows on overflow)."""
    st, cnt, res = solve_ex_raw(rows, l, d, mask_n, both, capacity=1 << 16)
    if st == PMS_ERR_OVERFLOW:
        st, cnt, res = solve_ex_raw(rows, l, d, mask_n, both, capacity=cnt)
    _check(st)
    return res


def solve_intersect_raw(seqs, l: int, d: int, capacity: Optional[int] = None):
    """pms_solve_intersect: (status, count, motifs[:min(count, capacity)])."""
    arr, keep, n, t = _rows(seqs)
    if capacity is None:
        capacity = 1 << 20
    out = _out_buffer(capacity)
    cnt = ctypes.c_uint64(capacity)
    st = _lib.pms_solve_intersect(arr, n, t, l, d,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
                                  if capacity > 0 else None, ctypes.byref(cnt))
    del keep
    k = min(int(cnt.value), capacity)
    return st, int(cnt.value), out[:k].copy()


def solve_intersect(seqs, l: int, d: int) -> np.ndarray:
    """Sorted uint32 motif codes by the neighbourhood-intersection method."""
    st, cnt, res = solve_intersect_raw(seqs, l, d, capacity=1 << 16)
    if st == PMS_ERR_OVERFLOW:
        st, cnt, res = solve_intersect_raw(seqs, l, d, capacity=cnt)
    _check(st)
    return res


def _row_pointers(seqs):
    """(address of n row pointers, object keeping them alive, n, t)."""
    if isinstance(seqs, np.ndarray):
        m = np.ascontiguousarray(seqs, dtype=np.uint8)
        if m.ndim != 2:
            raise ValueError("sequence array must be 2-D (n, t)")
        n, t = int(m.shape[0]), int(m.shape[1])
        ptrs = m.ctypes.data + np.arange(max(n, 1), dtype=np.uint64) * np.uint64(t)
        return ptrs.ctypes.data, (m, ptrs), n, t
    arr, rows, n, t = _rows(seqs)
    return ctypes.addressof(arr), (arr, rows), n, t


def _instance_records(instances, caps, outs):
    """pms_instance records for [(seqs, l, d), ...] with output addresses
    `outs` and capacities `caps`, and the objects that keep the row pointer
    arrays they address alive."""
    m = len(instances)
    rec = np.zeros(max(m, 1), dtype=_INSTANCE_DT)
    keep = []
    if m and all(isinstance(x[0], np.ndarray) and x[0].dtype == np.uint8 and x[0].ndim == 2
                 and x[0].flags["C_CONTIGUOUS"] and min(x[0].shape) >= 1 for x in instances):
        # Row pointers of every instance in one array, filled column-wise.
        arrs = [x[0] for x in instances]
        ns = np.fromiter((a.shape[0] for a in arrs), dtype=np.int64, count=m)
        ts = np.fromiter((a.shape[1] for a in arrs), dtype=np.int64, count=m)
        addrs = np.fromiter((a.__array_interface__["data"][0] for a in arrs), dtype=np.uint64,
                            count=m)
        first = np.zeros(m, dtype=np.int64)
        np.cumsum(ns[:-1], out=first[1:])
        within = np.arange(int(ns.sum()), dtype=np.int64) - np.repeat(first, ns)
        ptrs = np.repeat(addrs, ns) + (within * np.repeat(ts, ns)).astype(np.uint64)
        keep.append((arrs, ptrs))
        rec["seqs"] = np.uint64(ptrs.ctypes.data) + 8 * first.astype(np.uint64)
        rec["n"][:m], rec["t"][:m] = ns, ts
        rec["l"][:m] = np.fromiter((x[1] for x in instances), dtype=np.int32, count=m)
        rec["d"][:m] = np.fromiter((x[2] for x in instances), dtype=np.int32, count=m)
        rec["out_motifs"][:m] = np.where(caps > 0, outs, np.uint64(0))
        rec["capacity"][:m] = caps
    else:
        for i, (seqs, l, d) in enumerate(instances):
            addr, k, n, t = _row_pointers(seqs)
            keep.append(k)
            rec[i] = (addr, n, t, l, d, int(outs[i]) if caps[i] else 0, caps[i])
    return rec, keep


def solve_many(instances: Sequence[Tuple[object, int, int]], capacities=None):
    """pms_solve_many over [(seqs, l, d), ...]: (status, [motifs], [Result])."""
    m = len(instances)
    caps = (np.full(m, 1 << 16, dtype=np.uint64) if capacities is None
            else np.asarray([int(c) for c in capacities[:m]], dtype=np.uint64))
    offs = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.maximum(caps, 1).astype(np.int64), out=offs[1:])
    pool = _out_buffer(int(offs[m]))
    base = pool.ctypes.data
    rec, keep = _instance_records(instances, caps, base + 4 * offs[:m].astype(np.uint64))
    res = (Result * max(m, 1))()
    st = _lib.pms_solve_many(ctypes.cast(rec.ctypes.data, ctypes.POINTER(Instance)), m, res)
    del keep
    counts = np.frombuffer(res, dtype=_RESULT_DT, count=m)["count"]
    take = np.minimum(counts, caps).astype(np.int64)
    motifs = [pool[offs[i]:offs[i] + take[i]].copy() for i in range(m)]
    return st, motifs, [res[i] for i in range(m)]


def sort_codes(codes: np.ndarray, l: int) -> np.ndarray:
    """pms_sort_codes: sorts a contiguous uint32 array of motif codes in place
    and returns it."""
    if codes.dtype != np.uint32 or not codes.flags["C_CONTIGUOUS"] or not codes.flags["WRITEABLE"]:
        raise ValueError("codes must be a writable contiguous uint32 array")
    _check(_lib.pms_sort_codes(codes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                               int(codes.size), int(l)))
    return codes


def fill_work_items(begin: int, count: int, item_len: int, inst: int, out_ptr: int,
                    max_items: int) -> int:
    """pms_fill_work_items into host memory at out_ptr (16-byte records):
    the number of items written (-1 for invalid arguments)."""
    return int(_lib.pms_fill_work_items(int(begin), int(count), int(item_len), int(inst),
                                        ctypes.c_void_p(int(out_ptr)), int(max_items)))


def decode(code: int, l: int) -> str:
    buf = ctypes.create_string_buffer(l)
    _lib.pms_decode(int(code), int(l), buf)
    return buf.raw[:l].decode()


def set_config(chunk=0, wg_waves=0, wgs_per_cu=0, tail_split=0, variant=0, filter=0, reset=False):
    if reset:
        return _check(_lib.pms_set_config(None))
    cfg = Config(chunk, wg_waves, wgs_per_cu, tail_split, variant, filter)
    return _check(_lib.pms_set_config(ctypes.byref(cfg)))


def get_config() -> dict:
    cfg = Config()
    _check(_lib.pms_get_config(ctypes.byref(cfg)))
    return cfg.as_dict()


def autotune(n: int, t: int, l: int, d: int, cache_path: Optional[str] = None) -> dict:
    cfg = Config()
    _check(_lib.pms_autotune(n, t, l, d, cache_path.encode() if cache_path else None,
                             ctypes.byref(cfg)))
    return cfg.as_dict()


def autotune_many(instances: Sequence[Tuple[object, int, int]],
                  cache_path: Optional[str] = None) -> dict:
    """pms_autotune_many on [(seqs, l, d), ...]: tunes the launch on the batch
    itself and makes the result the current configuration."""
    m = len(instances)
    rec, keep = _instance_records(instances, np.zeros(m, dtype=np.uint64),
                                  np.zeros(m, dtype=np.uint64))
    cfg = Config()
    st = _lib.pms_autotune_many(ctypes.cast(rec.ctypes.data, ctypes.POINTER(Instance)), m,
                                cache_path.encode() if cache_path else None, ctypes.byref(cfg))
    del keep
    _check(st)
    return cfg.as_dict()


def last_stats() -> dict:
    s = Stats()
    _check(_lib.pms_last_stats(ctypes.byref(s)))
    return s.as_dict()


def valu_probe(op: str, waves_per_simd: int = 0, iters: int = 0) -> dict:
    """Issue rate of one VALU instruction kind (see pms_valu_probe)."""
    r = ProbeResult()
    _check(_lib.pms_valu_probe(PROBE_OPS[op], waves_per_simd, iters, ctypes.byref(r)))
    return {k: float(getattr(r, k)) for k, _ in r._fields_ if k != "reserved"}


def window_stride(t: int, l: int, layout: int = LAYOUT_BITSLICED) -> int:
    return int(_lib.pms_window_stride(t, l, layout))


# ---------------------------------------------------------------------------
# Device level (torch tensors supply device memory and the stream).
# ---------------------------------------------------------------------------
def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def build_windows(dev_seqs, n: int, t: int, l: int, dev_windows, dev_bad=None, stream=None,
                  layout: int = LAYOUT_BITSLICED):
    return _check(_lib.pms_build_windows(
        dev_seqs.data_ptr(), n, t, l, layout, dev_windows.data_ptr(),
        dev_bad.data_ptr() if dev_bad is not None else None, _stream_handle(stream)))


def solve_dev(dev_seqs, n: int, t: int, l: int, d: int, dev_out, capacity: int, dev_count,
              stream=None):
    return _check(_lib.pms_solve_dev(
        dev_seqs.data_ptr(), n, t, l, d, dev_out.data_ptr() if capacity else None, capacity,
        dev_count.data_ptr(), _stream_handle(stream)))


def solve_dev_noalloc(dev_seqs, n: int, t: int, l: int, d: int, dev_out, capacity: int,
                      dev_count, stream=None):
    """pms_solve_dev_noalloc: pms_solve_dev with the library's fixed scratch."""
    return _check(_lib.pms_solve_dev_noalloc(
        dev_seqs.data_ptr(), n, t, l, d, dev_out.data_ptr() if capacity else None, capacity,
        dev_count.data_ptr(), _stream_handle(stream)))


def step_launch(dev_instances, n_inst: int, max_n: int, dev_work, n_work: int, dev_state,
                dev_counters, config: Optional[dict] = None, stream=None):
    cfg = Config(**config) if config else None
    return _check(_lib.pms_step_launch(
        dev_instances.data_ptr(), n_inst, max_n, dev_work.data_ptr() if n_work else None, n_work,
        dev_state.data_ptr(), dev_counters.data_ptr(),
        ctypes.byref(cfg) if cfg is not None else None, _stream_handle(stream)))
