"""CPU oracle for the planted (l, d) motif set -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product library never
calls it, and it shares no code with the GPU path.

The arithmetic lives in ``pms_oracle.c`` (plain C, character compares):
M = { x in {A,C,G,T}^l : every sequence has a window within Hamming distance
d of x } (Section I.A; Section III.A), ``brute`` mode unpruned, ``skip`` mode
with the enhanced early rejection of Section III.A.  Results are candidate
numbers: base p of the l-mer (p = 0 leftmost) is base-4 digit l-1-p, with
A=0, C=1, G=2, T=3, so ascending numbers are ascending strings.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

from . import build as _build

BRUTE = 0
SKIP = 1
MASK_N = 1   # oracle_solve_ex flags
BOTH = 2
_MODES = {"brute": BRUTE, "skip": SKIP}


def as_matrix(seqs) -> np.ndarray:
    """(n, t) uint8 matrix from a 2-D array or a list of equal-length str/bytes."""
    if isinstance(seqs, np.ndarray):
        m = np.ascontiguousarray(seqs, dtype=np.uint8)
        if m.ndim != 2:
            raise ValueError("sequence matrix must be 2-D")
        return m
    rows = [s.encode() if isinstance(s, str) else bytes(s) for s in seqs]
    if not rows or len({len(r) for r in rows}) != 1:
        raise ValueError("sequences must be non-empty and of equal length")
    return np.frombuffer(b"".join(rows), dtype=np.uint8).reshape(len(rows), len(rows[0])).copy()


class OracleLib:
    """ctypes view of one build of ``pms_oracle.c``."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_solve.argtypes = [
            ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
            ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint64, u64p, u64p]
        lib.oracle_solve.restype = ctypes.c_int
        lib.oracle_candidate_distances.argtypes = [
            ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_candidate_distances.restype = ctypes.c_int
        lib.oracle_solve_ex.argtypes = [
            ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_int), ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
            ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint64,
            u64p, u64p]
        lib.oracle_solve_ex.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def solve(self, seqs, l: int, d: int, mode: str = "brute",
              threads: Optional[int] = None, k_range: Optional[Tuple[int, int]] = None,
              cap: Optional[int] = None, return_visits: bool = False):
        """Sorted uint32 array of motif numbers among candidates ``k_range`` (default all).

        With ``return_visits`` also returns the number of (candidate, sequence)
        scans performed.  ``cap`` bounds the stored motifs; a larger result raises.
        """
        m = as_matrix(seqs)
        n, t = m.shape
        total = 1 << (2 * l)
        k0, k1 = (0, total) if k_range is None else (int(k_range[0]), int(k_range[1]))
        if threads is None:
            threads = os.cpu_count() or 1
        if cap is None:
            cap = min(max(k1 - k0, 0), 1 << 24)
        out = np.empty(max(cap, 1), dtype=np.uint32)
        count = ctypes.c_uint64(0)
        visits = ctypes.c_uint64(0)
        rc = self.lib.oracle_solve(
            m.tobytes(), n, t, l, d, k0, k1, _MODES[mode], int(threads),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), cap,
            ctypes.byref(count), ctypes.byref(visits))
        if rc != 0:
            raise ValueError(f"oracle_solve failed with code {rc}")
        if count.value > cap:
            raise OverflowError(f"{count.value} motifs exceed cap {cap}")
        res = out[:count.value].copy()
        return (res, int(visits.value)) if return_visits else res

    def solve_ex(self, rows, l: int, d: int, mask_n: bool = False, both: bool = False,
                 mode: str = "brute", threads: Optional[int] = None,
                 k_range: Optional[Tuple[int, int]] = None, cap: Optional[int] = None,
                 return_visits: bool = False):
        """``solve`` for rows of their own lengths, with N masking and/or both
        strands (``oracle_solve_ex``).  ``rows``: list of str/bytes."""
        data = [r.encode() if isinstance(r, str) else bytes(r) for r in rows]
        n = len(data)
        arr = (ctypes.c_char_p * max(n, 1))(*data)
        lens = (ctypes.c_int * max(n, 1))(*[len(r) for r in data])
        total = 1 << (2 * l)
        k0, k1 = (0, total) if k_range is None else (int(k_range[0]), int(k_range[1]))
        if threads is None:
            threads = os.cpu_count() or 1
        if cap is None:
            cap = min(max(k1 - k0, 0), 1 << 24)
        out = np.empty(max(cap, 1), dtype=np.uint32)
        count = ctypes.c_uint64(0)
        visits = ctypes.c_uint64(0)
        flags = (MASK_N if mask_n else 0) | (BOTH if both else 0)
        rc = self.lib.oracle_solve_ex(
            arr, lens, n, l, d, flags, k0, k1, _MODES[mode], int(threads),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), cap,
            ctypes.byref(count), ctypes.byref(visits))
        if rc != 0:
            raise ValueError(f"oracle_solve_ex failed with code {rc}")
        if count.value > cap:
            raise OverflowError(f"{count.value} motifs exceed cap {cap}")
        res = out[:count.value].copy()
        return (res, int(visits.value)) if return_visits else res

    def candidate_distances(self, seqs, l: int, k: int) -> np.ndarray:
        """Per sequence, the smallest Hamming distance of candidate ``k`` to a window."""
        m = as_matrix(seqs)
        n, t = m.shape
        per = (ctypes.c_int32 * n)()
        rc = self.lib.oracle_candidate_distances(m.tobytes(), n, t, l, int(k), per)
        if rc != 0:
            raise ValueError(f"oracle_candidate_distances failed with code {rc}")
        return np.frombuffer(per, dtype=np.int32).copy()

    def is_motif(self, seqs, l: int, d: int, k: int) -> bool:
        return bool(self.candidate_distances(seqs, l, k).max() <= d)


_DEFAULT: Optional[OracleLib] = None


def default() -> OracleLib:
    """The oracle built from ``pms_oracle.c`` (rebuilt when the source is newer)."""
    global _DEFAULT
    if _DEFAULT is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        _DEFAULT = OracleLib(_build.LIB)
    return _DEFAULT


def solve(seqs, l: int, d: int, **kw):
    return default().solve(seqs, l, d, **kw)


def solve_ex(rows, l: int, d: int, **kw):
    return default().solve_ex(rows, l, d, **kw)


def candidate_distances(seqs, l: int, k: int) -> np.ndarray:
    return default().candidate_distances(seqs, l, k)


def is_motif(seqs, l: int, d: int, k: int) -> bool:
    return default().is_motif(seqs, l, d, k)


def number_to_lmer(k: int, l: int) -> str:
    """The l-mer whose base p is base-4 digit l-1-p of k (A=0, C=1, G=2, T=3)."""
    return "".join("ACGT"[(k >> (2 * (l - 1 - p))) & 3] for p in range(l))


def lmer_to_number(s: str) -> int:
    k = 0
    for ch in s.upper():
        k = 4 * k + "ACGT".index(ch)
    return k
