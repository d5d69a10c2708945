"""CPU oracle for Triple State QuickSort (arXiv 1505.00558).

TEST INFRASTRUCTURE ONLY.  This package wraps ``liboracle_tsqs.so`` (plain C,
single-threaded, built with gcc from ``tsqs_oracle.c``), the slow and obviously
correct reference that the GPU library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the GPU path (``paper_1505_00558_amd``) and
neither imports the other.

What it computes: the array-based Triple State QuickSort of the paper (SIII
partition state machine, SIII.H/SIII.I pivot tiers and presorted handlers, SIV
insertion sort, SV.C sample jitter), with comparison / copy counters (SV.A).
Readings of the parts the paper does not print are listed in the design doc and
named in ``tsqs_stage.inc`` where they are used.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_tsqs.so")
_SOURCES = ["tsqs_oracle.c", "tsqs_stage.inc", "tsqs_oracle.h"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2).  Returns the library path."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           os.path.join(_HERE, "tsqs_oracle.c"), "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("ins_max", ctypes.c_int32),
        ("med3_below", ctypes.c_int32),
        ("med5_below", ctypes.c_int32),
        ("ninther_below", ctypes.c_int32),
        ("medof3_small", ctypes.c_int32),
        ("random_samples", ctypes.c_int32),
        ("handlers", ctypes.c_int32),
        ("reverse_tolerance", ctypes.c_int32),
        ("analysis_random_pivot", ctypes.c_int32),
        ("debug_checks", ctypes.c_int32),
        ("seed", ctypes.c_uint32),
        ("reserved", ctypes.c_int32),
    ]


class Counters(ctypes.Structure):
    _fields_ = [
        ("comparisons", ctypes.c_uint64),
        ("copies", ctypes.c_uint64),
        ("pivot_copies", ctypes.c_uint64),
        ("literal_swaps", ctypes.c_uint64),
        ("stages", ctypes.c_uint64),
        ("insertion_stages", ctypes.c_uint64),
        ("max_depth", ctypes.c_uint64),
        ("tar_peak", ctypes.c_uint64),
        ("hole_errors", ctypes.c_uint64),
        ("revisit_errors", ctypes.c_uint64),
        ("internal_errors", ctypes.c_uint64),
        ("post_errors", ctypes.c_uint64),
        ("events", ctypes.c_uint64 * 32),
    ]

    def as_dict(self) -> dict:
        d = {f: int(getattr(self, f)) for f, _ in self._fields_ if f != "events"}
        d["events"] = [int(x) for x in self.events]
        return d


# indices of oracle_counters_t.events (OE_* of tsqs_oracle.h): the states of
# SIII.B-F and the outcomes of the handlers of SIII.I
EVENTS = [
    "STATE1", "CLOSE_BY_SIDE", "CLOSE_BY_ZONE", "STATE2L", "STATE2R", "STATE3L",
    "STATE3R", "ROLL", "RUN_FITS", "RUN_FILLS", "COPY_BACK", "EXIT2", "BYPASS",
    "R_AT_MID", "SORTED", "SORTED_CONFIRMED", "SORTED_FALLBACK", "REVERSED",
    "REV_SWAP", "REV_CONFIRMED", "REV_FALLBACK",
]


class Entry(ctypes.Structure):
    """oracle_entry_t: a stage entered in the middle (States 2/3, exit2)."""
    _fields_ = [
        ("a", ctypes.c_int64), ("b", ctypes.c_int64), ("l", ctypes.c_int64),
        ("r", ctypes.c_int64), ("m", ctypes.c_int64), ("ml", ctypes.c_int64),
        ("mr", ctypes.c_int64), ("hole0", ctypes.c_int64), ("hole1", ctypes.c_int64),
        ("entry", ctypes.c_int32), ("open_side", ctypes.c_int32), ("lc", ctypes.c_int32),
        ("p", ctypes.c_int32), ("temp", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


ENTRY_STATE2, ENTRY_STATE3, ENTRY_EXIT2 = 0, 1, 2

_lib = None
_SUFFIX = {
    np.dtype(np.int32): ("i32", ctypes.c_int32),
    np.dtype(np.uint32): ("u32", ctypes.c_uint32),
    np.dtype(np.int64): ("i64", ctypes.c_int64),
    np.dtype(np.uint64): ("u64", ctypes.c_uint64),
    np.dtype(np.float32): ("f32", ctypes.c_uint32),
}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    for suf, ct in _SUFFIX.values():
        f = getattr(lib, "oracle_tsqs_sort_" + suf)
        f.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(Params),
                      ctypes.POINTER(Counters)]
        f.restype = ctypes.c_int
        g = getattr(lib, "oracle_tsqs_sort_pairs_" + suf)
        g.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                      ctypes.POINTER(Params), ctypes.POINTER(Counters)]
        g.restype = ctypes.c_int
    lib.oracle_default_params.argtypes = [ctypes.POINTER(Params)]
    lib.oracle_default_params.restype = None
    lib.oracle_free_storage.argtypes = []
    lib.oracle_free_storage.restype = None
    lib.oracle_median3_i32.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(Counters)]
    lib.oracle_median3_i32.restype = ctypes.c_int
    lib.oracle_insertion_i32.argtypes = [ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.POINTER(Counters)]
    lib.oracle_insertion_i32.restype = ctypes.c_int
    lib.oracle_median5_i32.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(Counters)]
    lib.oracle_median5_i32.restype = ctypes.c_int
    lib.oracle_choose_pivot_i32.argtypes = [ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.POINTER(Params),
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(Counters)]
    lib.oracle_choose_pivot_i32.restype = ctypes.c_int
    lib.oracle_run_entry_i32.argtypes = [ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.POINTER(Entry), ctypes.POINTER(Counters)]
    lib.oracle_run_entry_i32.restype = ctypes.c_int
    _lib = lib
    return lib


def default_params(**overrides) -> Params:
    p = Params()
    _load().oracle_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def free_storage() -> None:
    _load().oracle_free_storage()


def _check_rc(rc: int) -> None:
    if rc == -1:
        raise ValueError("oracle: invalid parameters")
    if rc == -2:
        raise RuntimeError("oracle: internal error (watchdog or invariant)")
    if rc != 0:
        raise MemoryError("oracle: allocation failed (%d)" % rc)


def sort(keys: np.ndarray, params: Params | None = None, counters: bool = False):
    """Return a sorted copy of ``keys`` (int32/uint32/int64/uint64/float32).

    float32 keys are ordered by IEEE 754-2008 totalOrder on their bits.
    With ``counters=True`` returns ``(sorted, Counters)``.
    """
    keys = np.asarray(keys)
    suf, _ = _SUFFIX[keys.dtype]
    out = np.ascontiguousarray(keys).copy()
    buf = out.view(np.uint32) if keys.dtype == np.float32 else out
    c = Counters()
    p = params if params is not None else default_params()
    rc = getattr(_load(), "oracle_tsqs_sort_" + suf)(
        buf.ctypes.data if out.size else None, out.size, ctypes.byref(p), ctypes.byref(c))
    _check_rc(rc)
    return (out, c) if counters else out


def sort_pairs(keys: np.ndarray, vals: np.ndarray, params: Params | None = None,
               counters: bool = False):
    """Sort (key, uint32 payload) elements by key; returns sorted copies."""
    keys = np.asarray(keys)
    suf, _ = _SUFFIX[keys.dtype]
    ko = np.ascontiguousarray(keys).copy()
    vo = np.ascontiguousarray(vals, dtype=np.uint32).copy()
    if ko.shape != vo.shape:
        raise ValueError("keys and vals differ in shape")
    kb = ko.view(np.uint32) if keys.dtype == np.float32 else ko
    c = Counters()
    p = params if params is not None else default_params()
    rc = getattr(_load(), "oracle_tsqs_sort_pairs_" + suf)(
        kb.ctypes.data if ko.size else None, vo.ctypes.data if vo.size else None,
        ko.size, ctypes.byref(p), ctypes.byref(c))
    _check_rc(rc)
    return (ko, vo, c) if counters else (ko, vo)


def median3(three) -> tuple:
    """MedianOf3S of SIII.I on three int32 keys.

    Returns (flag, result_list, pivot, Counters)."""
    a = np.array(three, dtype=np.int32)
    piv = ctypes.c_int32(0)
    c = Counters()
    flag = _load().oracle_median3_i32(a.ctypes.data, ctypes.byref(piv), ctypes.byref(c))
    return flag, a.tolist(), int(piv.value), c


def insertion(arr) -> tuple:
    """Insertion sort of SIV on int32 keys.  Returns (sorted_list, Counters)."""
    a = np.array(arr, dtype=np.int32)
    c = Counters()
    _load().oracle_insertion_i32(a.ctypes.data, a.size, ctypes.byref(c))
    return a.tolist(), c


def median5(five) -> tuple:
    """Median of five (SIII.H, reading R4) on five int32 keys.

    Returns (flag, result_list, pivot, Counters)."""
    a = np.array(five, dtype=np.int32)
    piv = ctypes.c_int32(0)
    c = Counters()
    flag = _load().oracle_median5_i32(a.ctypes.data, ctypes.byref(piv), ctypes.byref(c))
    return flag, a.tolist(), int(piv.value), c


def choose_pivot(arr, params: Params | None = None) -> tuple:
    """The size-tiered pivot choice (SIII.H, SV.C) on int32 ar[0..n-1].

    Returns (flag, array_after, pivot, Counters)."""
    a = np.array(arr, dtype=np.int32)
    piv = ctypes.c_int32(0)
    c = Counters()
    p = params if params is not None else default_params()
    flag = _load().oracle_choose_pivot_i32(a.ctypes.data, a.size, ctypes.byref(p),
                                           ctypes.byref(piv), ctypes.byref(c))
    if flag == -2:
        raise ValueError("choose_pivot needs n >= 3")
    return flag, a.tolist(), int(piv.value), c


def run_entry(arr, **fields) -> tuple:
    """Run a stage from an entry state (oracle_entry_t fields as keywords) on
    int32 keys.  Returns (array_after, Entry_after, Counters)."""
    a = np.array(arr, dtype=np.int32)
    e = Entry()
    for k, v in fields.items():
        setattr(e, k, v)
    c = Counters()
    rc = _load().oracle_run_entry_i32(a.ctypes.data, a.size, ctypes.byref(e), ctypes.byref(c))
    _check_rc(rc)
    return a.tolist(), e, c


def total_order_key(bits: np.ndarray) -> np.ndarray:
    """Sort key (uint64) realising totalOrder for float32 bit patterns.

    Test helper used to compare against library sorts: negative patterns map
    below 2^31 in reverse magnitude order, positive ones above it."""
    b = np.asarray(bits, dtype=np.uint32).astype(np.uint64)
    neg = (b >> np.uint64(31)) == 1
    mag = b & np.uint64(0x7FFFFFFF)
    return np.where(neg, np.uint64(0x7FFFFFFF) - mag, np.uint64(0x80000000) + mag)
