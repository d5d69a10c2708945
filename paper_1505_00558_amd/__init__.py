"""Three-way partition sort for AMD MI355X (gfx950).

Thin ctypes binding of ``libtsqs.so`` (C ABI in ``include/tsqs.h``).  Every step
of the sort runs in the library's HIP kernels; this module only marshals torch
tensors (device memory) and the current HIP stream.  There is no CPU fallback:
if the library is missing or no GPU is present the calls raise.

The method is Triple State QuickSort's (Muqaddas, arXiv 1505.00558, SIII):
recursive partitioning around a sampled pivot into < / == / > parts, the == part
being final and never compared again.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsqs.so")

INT32, UINT32, INT64, UINT64, FLOAT32 = 0, 1, 2, 3, 4
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EINTERNAL, EAGAIN, ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
NOALLOC_MAX_KEYS = 1 << 20
NOALLOC_SCRATCH_BYTES = 32 << 20
OPT_SMALL_MAX, OPT_SAMPLES, OPT_DEPTH_FACTOR, OPT_PIVOT_MODE = 1, 2, 3, 4
OPT_SEED, OPT_TIMING, OPT_PART_GRID, OPT_FINISH_GRID, OPT_FINISH_ALGO = 5, 6, 7, 8, 9
OPT_PRESORT, OPT_SCHEDULE, OPT_ITER_CAP, OPT_QUEUE_DIRECT = 10, 11, 12, 13
OPT_PART_THREADS1, OPT_PART_THREADS2, OPT_WORKSPACE_CAP, OPT_DEBUG = 14, 15, 16, 17
ERR_SHADOW = 128
SCHEDULE_LEVELS, SCHEDULE_PERSISTENT = 0, 1
MAX_LEVELS = 192

SYMBOLS = ["tsqs_sort", "tsqs_sort_pairs", "tsqs_sort_noalloc", "tsqs_sort_records", "tsqs_sort_batch", "tsqs_autotune",
           "tsqs_free_storage", "tsqs_set_option", "tsqs_get_option", "tsqs_get_stats",
           "tsqs_strerror", "tsqs_version", "tsqs_graph_create", "tsqs_graph_launch",
           "tsqs_graph_stats", "tsqs_graph_destroy"]
QUEUE_SYMBOLS = ["tsqs_queue_open", "tsqs_queue_submit", "tsqs_queue_step", "tsqs_queue_poll",
                 "tsqs_queue_result", "tsqs_queue_reap", "tsqs_queue_release",
                 "tsqs_queue_cancel", "tsqs_queue_info", "tsqs_queue_close"]


class Stats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_uint32),
        ("max_depth", ctypes.c_uint32),
        ("n", ctypes.c_uint64),
        ("key_bytes", ctypes.c_uint32),
        ("payload_bytes", ctypes.c_uint32),
        ("fallback_parts", ctypes.c_uint64),
        ("small_parts", ctypes.c_uint64),
        ("small_keys", ctypes.c_uint64),
        ("band_keys", ctypes.c_uint64),
        ("level_keys", ctypes.c_uint64 * MAX_LEVELS),
        ("level_parts", ctypes.c_uint32 * MAX_LEVELS),
        ("level_ms", ctypes.c_float * MAX_LEVELS),
        ("partition_ms", ctypes.c_double),
        ("partition_bytes", ctypes.c_uint64),
        ("partition_launches", ctypes.c_uint32),
        ("presorted", ctypes.c_uint32),
        ("tail_parts", ctypes.c_uint64),
        ("tail_keys", ctypes.c_uint64),
        ("tail_bytes", ctypes.c_uint64),
        ("select_rounds", ctypes.c_uint64),
        ("error_flags", ctypes.c_uint32),
        ("schedule", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        lv = int(self.levels)
        return {
            "levels": lv, "max_depth": int(self.max_depth), "n": int(self.n),
            "key_bytes": int(self.key_bytes), "payload_bytes": int(self.payload_bytes),
            "fallback_parts": int(self.fallback_parts), "small_parts": int(self.small_parts),
            "small_keys": int(self.small_keys), "band_keys": int(self.band_keys),
            "level_keys": [int(x) for x in self.level_keys[:lv]],
            "level_parts": [int(x) for x in self.level_parts[:lv]],
            "level_ms": [float(x) for x in self.level_ms[:lv]],
            "partition_ms": float(self.partition_ms),
            "partition_bytes": int(self.partition_bytes),
            "partition_launches": int(self.partition_launches),
            "presorted": int(self.presorted),
            "tail_parts": int(self.tail_parts), "tail_keys": int(self.tail_keys),
            "tail_bytes": int(self.tail_bytes), "select_rounds": int(self.select_rounds),
            "error_flags": int(self.error_flags), "schedule": int(self.schedule),
        }


class Tune(ctypes.Structure):
    _fields_ = [
        ("small_max", ctypes.c_int64),
        ("samples", ctypes.c_int64),
        ("part_grid", ctypes.c_int64),
        ("finish_grid", ctypes.c_int64),
        ("finish_algo", ctypes.c_int64),
        ("ms_default", ctypes.c_double),
        ("ms_best", ctypes.c_double),
        ("trials", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("part_threads1", ctypes.c_int64),
        ("part_threads2", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {k: (getattr(self, k) if isinstance(getattr(self, k), float) else int(getattr(self, k)))
                for k, _ in self._fields_ if k != "reserved"}


class TsqsError(RuntimeError):
    pass


_lib = None


def load_library():
    """Load libtsqs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtsqs.so is not built; run paper_1505_00558_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.tsqs_sort.argtypes = [vp, sz, ctypes.c_int, vp]
    lib.tsqs_sort.restype = ctypes.c_int
    lib.tsqs_sort_pairs.argtypes = [vp, vp, sz, ctypes.c_int, vp]
    lib.tsqs_sort_pairs.restype = ctypes.c_int
    lib.tsqs_sort_noalloc.argtypes = [vp, vp, sz, ctypes.c_int, vp]
    lib.tsqs_sort_noalloc.restype = ctypes.c_int
    lib.tsqs_sort_records.argtypes = [vp, vp, sz, vp, sz, ctypes.c_int, vp]
    lib.tsqs_sort_records.restype = ctypes.c_int
    lib.tsqs_sort_batch.argtypes = [vp, vp, vp, sz, ctypes.c_int, vp]
    lib.tsqs_sort_batch.restype = ctypes.c_int
    lib.tsqs_autotune.argtypes = [ctypes.c_int, ctypes.c_int, sz, vp, sz, vp, ctypes.POINTER(Tune)]
    lib.tsqs_autotune.restype = ctypes.c_int
    lib.tsqs_free_storage.argtypes = []
    lib.tsqs_free_storage.restype = None
    lib.tsqs_set_option.argtypes = [ctypes.c_int, ctypes.c_int64]
    lib.tsqs_set_option.restype = ctypes.c_int
    lib.tsqs_get_option.argtypes = [ctypes.c_int]
    lib.tsqs_get_option.restype = ctypes.c_int64
    lib.tsqs_get_stats.argtypes = [ctypes.POINTER(Stats)]
    lib.tsqs_get_stats.restype = ctypes.c_int
    lib.tsqs_strerror.argtypes = [ctypes.c_int]
    lib.tsqs_strerror.restype = ctypes.c_char_p
    lib.tsqs_version.argtypes = []
    lib.tsqs_version.restype = ctypes.c_int
    lib.tsqs_graph_create.argtypes = [vp, vp, sz, vp, sz, ctypes.c_int, ctypes.POINTER(vp)]
    lib.tsqs_graph_create.restype = ctypes.c_int
    lib.tsqs_graph_launch.argtypes = [vp, vp]
    lib.tsqs_graph_launch.restype = ctypes.c_int
    lib.tsqs_graph_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.tsqs_graph_stats.restype = ctypes.c_int
    lib.tsqs_graph_destroy.argtypes = [vp]
    lib.tsqs_graph_destroy.restype = ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.tsqs_queue_open.argtypes = [sz, vp, ctypes.POINTER(vp)]
    lib.tsqs_queue_submit.argtypes = [vp, vp, sz, ctypes.c_int, u64p]
    lib.tsqs_queue_step.argtypes = [vp]
    lib.tsqs_queue_poll.argtypes = [vp, ctypes.c_uint64]
    lib.tsqs_queue_result.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp),
                                      ctypes.POINTER(sz)]
    lib.tsqs_queue_reap.argtypes = [vp, vp, sz, ctypes.POINTER(sz)]
    lib.tsqs_queue_release.argtypes = [vp, ctypes.c_uint64]
    lib.tsqs_queue_cancel.argtypes = [vp, ctypes.c_uint64]
    lib.tsqs_queue_info.argtypes = [vp, u64p, u64p, u64p, u64p, u64p]
    lib.tsqs_queue_close.argtypes = [vp]
    for name in QUEUE_SYMBOLS:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load_library().tsqs_strerror(int(code)).decode()


def _check(rc: int) -> None:
    if rc != OK:
        raise TsqsError("tsqs error %d: %s" % (rc, strerror(rc)))


def _dtype_code(t) -> int:
    import torch
    m = {torch.int32: INT32, torch.int64: INT64, torch.float32: FLOAT32}
    if hasattr(torch, "uint32"):
        m[torch.uint32] = UINT32
    if hasattr(torch, "uint64"):
        m[torch.uint64] = UINT64
    if t.dtype not in m:
        raise TypeError("unsupported key dtype %s" % t.dtype)
    return m[t.dtype]


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_tensor(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def sort(keys, dtype_code: int | None = None):
    """Sort a 1-D device tensor of keys in place (ascending; float32 by totalOrder)."""
    _check_tensor(keys, "keys")
    dt = _dtype_code(keys) if dtype_code is None else dtype_code
    _check(load_library().tsqs_sort(ctypes.c_void_p(keys.data_ptr()), keys.numel(), dt,
                                    _stream_handle()))
    return keys


def sort_pairs(keys, vals, dtype_code: int | None = None):
    """Sort keys in place, moving the uint32 payload ``vals`` (int32 or uint32 tensor) along."""
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals")
    if vals.numel() != keys.numel() or vals.element_size() != 4:
        raise ValueError("vals must hold one 4-byte payload per key")
    dt = _dtype_code(keys) if dtype_code is None else dtype_code
    _check(load_library().tsqs_sort_pairs(ctypes.c_void_p(keys.data_ptr()),
                                          ctypes.c_void_p(vals.data_ptr()), keys.numel(), dt,
                                          _stream_handle()))
    return keys, vals


def sort_noalloc(keys, vals=None, dtype_code: int | None = None):
    """As ``sort`` / ``sort_pairs`` through ``tsqs_sort_noalloc``: every device
    buffer of the call comes from the library's fixed per-GPU array (at most
    NOALLOC_MAX_KEYS keys; larger requests raise with ESCRATCH)."""
    _check_tensor(keys, "keys")
    vp = None
    if vals is not None:
        _check_tensor(vals, "vals")
        if vals.numel() != keys.numel() or vals.element_size() != 4:
            raise ValueError("vals must hold one 4-byte payload per key")
        vp = ctypes.c_void_p(vals.data_ptr())
    dt = _dtype_code(keys) if dtype_code is None else dtype_code
    _check(load_library().tsqs_sort_noalloc(ctypes.c_void_p(keys.data_ptr()), vp, keys.numel(), dt,
                                            _stream_handle()))
    return keys if vals is None else (keys, vals)


def sort_records(keys, records, out=None, dtype_code: int | None = None):
    """Sort keys in place and put ``records`` (a contiguous tensor whose first
    dimension is the key count; each row is one record of any size) in key order:
    into ``out`` (same shape and byte size), or in place when ``out`` is None."""
    _check_tensor(keys, "keys")
    _check_tensor(records, "records")
    n = keys.numel()
    if records.dim() < 1 or records.shape[0] != n:
        raise ValueError("records needs one row per key")
    rec_bytes = records.numel() * records.element_size() // n if n else 0
    op = None
    if out is not None:
        _check_tensor(out, "out")
        if out.numel() * out.element_size() != records.numel() * records.element_size():
            raise ValueError("out must have the byte size of records")
        op = ctypes.c_void_p(out.data_ptr())
    dt = _dtype_code(keys) if dtype_code is None else dtype_code
    if n == 0:
        return keys, (records if out is None else out)
    _check(load_library().tsqs_sort_records(ctypes.c_void_p(keys.data_ptr()),
                                            ctypes.c_void_p(records.data_ptr()), rec_bytes, op,
                                            n, dt, _stream_handle()))
    return keys, (records if out is None else out)


def sort_batch(keys, offsets, vals=None, dtype_code: int | None = None):
    """Sort len(offsets)-1 arrays stored back to back in ``keys``.

    ``offsets`` is a host sequence / numpy array of nseg+1 non-decreasing uint64
    values starting at 0."""
    import numpy as np
    _check_tensor(keys, "keys")
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    nseg = offs.size - 1
    if nseg < 0:
        raise ValueError("offsets needs at least one value")
    vp = None
    if vals is not None:
        _check_tensor(vals, "vals")
        if vals.numel() != keys.numel() or vals.element_size() != 4:
            raise ValueError("vals must hold one 4-byte payload per key")
        vp = ctypes.c_void_p(vals.data_ptr())
    dt = _dtype_code(keys) if dtype_code is None else dtype_code
    _check(load_library().tsqs_sort_batch(ctypes.c_void_p(keys.data_ptr()), vp,
                                          offs.ctypes.data_as(ctypes.c_void_p), nseg, dt,
                                          _stream_handle()))
    return keys


class Graph:
    """One sort of fixed buffers and shape captured into a HIP graph
    (tsqs_graph_*): ``launch()`` replays it on the current stream, sorting
    whatever the buffers hold then.  ``offsets`` as for ``sort_batch``, or None
    for one array."""

    def __init__(self, keys, offsets=None, vals=None, dtype_code: int | None = None):
        import numpy as np
        _check_tensor(keys, "keys")
        vp = None
        if vals is not None:
            _check_tensor(vals, "vals")
            if vals.numel() != keys.numel() or vals.element_size() != 4:
                raise ValueError("vals must hold one 4-byte payload per key")
            vp = ctypes.c_void_p(vals.data_ptr())
        offs, nseg = None, 0
        if offsets is not None:
            offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
            nseg = offs.size - 1
        dt = _dtype_code(keys) if dtype_code is None else dtype_code
        self._lib = load_library()
        self._g = ctypes.c_void_p()
        self._keep = (keys, vals)        # the buffers the graph sorts stay alive with it
        _check(self._lib.tsqs_graph_create(
            ctypes.c_void_p(keys.data_ptr()), vp, keys.numel(),
            offs.ctypes.data_as(ctypes.c_void_p) if offs is not None else None, nseg, dt,
            ctypes.byref(self._g)))

    def launch(self) -> None:
        _check(self._lib.tsqs_graph_launch(self._g, _stream_handle()))

    def stats(self) -> dict:
        s = Stats()
        _check(self._lib.tsqs_graph_stats(self._g, ctypes.byref(s)))
        return s.as_dict()

    def destroy(self) -> None:
        if self._g:
            g, self._g = self._g, ctypes.c_void_p()
            _check(self._lib.tsqs_graph_destroy(g))

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def autotune(dtype_code: int, n: int, with_payload: bool = False, offsets=None) -> dict:
    """Time candidate options on seeded keys shaped like the work (one array of n
    keys, or the arrays of ``offsets``), set the fastest, and return them."""
    import numpy as np
    t = Tune()
    offs = None
    nseg = 0
    if offsets is not None:
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
        nseg = offs.size - 1
        n = int(offs[-1])
    _check(load_library().tsqs_autotune(int(dtype_code), 1 if with_payload else 0, int(n),
                                        offs.ctypes.data_as(ctypes.c_void_p) if offs is not None
                                        else None, nseg, _stream_handle(), ctypes.byref(t)))
    return t.as_dict()


def free_storage() -> None:
    load_library().tsqs_free_storage()


def set_option(key: int, value: int) -> None:
    _check(load_library().tsqs_set_option(int(key), int(value)))


def get_option(key: int) -> int:
    return int(load_library().tsqs_get_option(int(key)))


def get_stats() -> dict:
    """Statistics of the last call (waits for its device work; raises if the
    device reported an error for it)."""
    s = Stats()
    _check(load_library().tsqs_get_stats(ctypes.byref(s)))
    return s.as_dict()


def last_call_status() -> tuple:
    """(return code, statistics) of the last call, without raising."""
    s = Stats()
    rc = load_library().tsqs_get_stats(ctypes.byref(s))
    return int(rc), s.as_dict()


class _DeviceView:
    """__cuda_array_interface__ of a device buffer the library owns (no copy)."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr,
                                         "data": (ptr, False), "version": 2}


_TYPESTR = {INT32: "<i4", UINT32: "<i4", INT64: "<i8", UINT64: "<i8", FLOAT32: "<f4"}


class Queue:
    """Serving queue (``include/tsqs_queue.h``): requests are copied into a
    device arena held within ``budget_bytes`` and sorted by ticks that batch every
    live request of a key type into the same launches."""

    QUEUED, RUNNING, DONE = 0, 1, 2

    def __init__(self, budget_bytes: int):
        self._lib = load_library()
        self._q = ctypes.c_void_p()
        _check(self._lib.tsqs_queue_open(int(budget_bytes), _stream_handle(),
                                         ctypes.byref(self._q)))
        self._keep = {}

    def submit(self, keys, dtype_code: int | None = None) -> int:
        """Queue a sort of the device tensor ``keys`` (left unchanged; it must stay
        valid until the request is admitted).  Returns a ticket."""
        _check_tensor(keys, "keys")
        dt = _dtype_code(keys) if dtype_code is None else dtype_code
        t = ctypes.c_uint64()
        _check(self._lib.tsqs_queue_submit(self._q, ctypes.c_void_p(keys.data_ptr()),
                                           keys.numel(), dt, ctypes.byref(t)))
        self._keep[t.value] = (keys, dt)
        return t.value

    def step(self) -> None:
        _check(self._lib.tsqs_queue_step(self._q))

    def poll(self, ticket: int) -> int:
        rc = self._lib.tsqs_queue_poll(self._q, int(ticket))
        if rc < 0:
            _check(rc)
        return rc

    def result(self, ticket: int):
        """The sorted keys of a done request, as a tensor viewing the arena
        (valid until ``release``)."""
        import torch
        ptr, n = ctypes.c_void_p(), ctypes.c_size_t()
        _check(self._lib.tsqs_queue_result(self._q, int(ticket), ctypes.byref(ptr),
                                           ctypes.byref(n)))
        src, dt = self._keep[int(ticket)]
        view = torch.as_tensor(_DeviceView(int(ptr.value), int(n.value), _TYPESTR[dt]),
                               device=src.device)
        return view

    def reap(self, cap: int = 4096) -> list:
        """Tickets found done since the previous call."""
        buf = (ctypes.c_uint64 * cap)()
        n = ctypes.c_size_t()
        _check(self._lib.tsqs_queue_reap(self._q, buf, cap, ctypes.byref(n)))
        return list(buf[:n.value])

    def release(self, ticket: int) -> None:
        _check(self._lib.tsqs_queue_release(self._q, int(ticket)))
        self._keep.pop(int(ticket), None)

    def cancel(self, ticket: int) -> bool:
        """Drop a queued request (or release a done one): True; False if it is
        running (release it when done)."""
        rc = self._lib.tsqs_queue_cancel(self._q, int(ticket))
        if rc == EAGAIN:
            return False
        _check(rc)
        self._keep.pop(int(ticket), None)
        return True

    def info(self) -> dict:
        v = [ctypes.c_uint64() for _ in range(5)]
        _check(self._lib.tsqs_queue_info(self._q, *[ctypes.byref(x) for x in v]))
        return dict(zip(["queued", "running", "done", "arena_used", "arena_bytes"],
                        [x.value for x in v]))

    def close(self) -> None:
        if self._q:
            _check(self._lib.tsqs_queue_close(self._q))
            self._q = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
