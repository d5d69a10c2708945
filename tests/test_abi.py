"""The C ABI library loads, exports every function include/tsqs.h declares, and
rejects bad arguments before making any HIP call (so this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_1505_00558_amd as tsqs
    if not os.path.exists(tsqs.LIB_PATH):
        from paper_1505_00558_amd import build
        build.build()
    return tsqs.load_library()


def _declared(header="tsqs.h"):
    with open(os.path.join(ROOT, "include", header)) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(tsqs_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_api():
    names = _declared()
    for n in ("tsqs_sort", "tsqs_sort_pairs", "tsqs_sort_batch", "tsqs_autotune", "tsqs_free_storage",
              "tsqs_set_option", "tsqs_get_option", "tsqs_get_stats", "tsqs_strerror"):
        assert n in names


def test_exports_every_declared_symbol(lib):
    import paper_1505_00558_amd as tsqs
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(tsqs.SYMBOLS) == _declared()
    for n in _declared("tsqs_queue.h"):
        assert hasattr(lib, n), n
    assert sorted(tsqs.QUEUE_SYMBOLS) == _declared("tsqs_queue.h")


def test_version_and_strerror(lib):
    assert lib.tsqs_version() == 3
    import paper_1505_00558_amd as tsqs
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert tsqs.strerror(code) and tsqs.strerror(code) != "unknown error code"
    assert tsqs.strerror(-99) == "unknown error code"


def test_sort_argument_errors(lib):
    fake = ctypes.c_void_p(0x1000)
    assert lib.tsqs_sort(None, 5, 0, None) == -1
    assert lib.tsqs_sort(None, 0, 0, None) == 0
    assert lib.tsqs_sort(None, 1, 0, None) == 0
    assert lib.tsqs_sort(fake, 5, 9, None) == -4
    assert lib.tsqs_sort(fake, 5, -1, None) == -4
    assert lib.tsqs_sort(fake, 1 << 32, 0, None) == -1
    assert lib.tsqs_sort_pairs(fake, None, 5, 0, None) == -1
    assert lib.tsqs_sort_pairs(None, fake, 5, 0, None) == -1
    assert lib.tsqs_sort_pairs(fake, fake, 1 << 32, 2, None) == -1
    assert lib.tsqs_sort_pairs(None, None, 1, 4, None) == 0


def _offs(vals):
    arr = (ctypes.c_uint64 * len(vals))(*vals)
    return ctypes.cast(arr, ctypes.c_void_p), arr


def test_batch_argument_errors(lib):
    fake = ctypes.c_void_p(0x1000)
    p, keep = _offs([1, 5])
    assert lib.tsqs_sort_batch(fake, None, p, 1, 0, None) == -1        # offsets[0] != 0
    p, keep = _offs([0, 5, 3])
    assert lib.tsqs_sort_batch(fake, None, p, 2, 0, None) == -1        # decreasing
    p, keep = _offs([0, 1 << 32])
    assert lib.tsqs_sort_batch(fake, None, p, 1, 0, None) == -1        # array too long
    assert lib.tsqs_sort_batch(fake, None, None, 3, 0, None) == -1     # no offsets
    p, keep = _offs([0, 1, 2, 2])
    assert lib.tsqs_sort_batch(None, None, p, 3, 0, None) == 0         # all arrays <= 1
    assert lib.tsqs_sort_batch(fake, None, None, 0, 0, None) == 0      # no arrays
    p, keep = _offs([0, 5])
    assert lib.tsqs_sort_batch(None, None, p, 1, 0, None) == -1        # null keys
    assert lib.tsqs_sort_batch(fake, None, p, 1, 7, None) == -4


def test_graph_argument_errors(lib):
    """tsqs_graph_*: every argument error returns before any HIP call."""
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p()
    ref = ctypes.byref(out)
    assert lib.tsqs_graph_create(fake, None, 100, None, 0, 0, None) == -1      # no out
    assert lib.tsqs_graph_create(fake, None, 100, None, 0, 7, ref) == -4       # dtype
    assert lib.tsqs_graph_create(None, None, 100, None, 0, 0, ref) == -1       # no keys
    assert lib.tsqs_graph_create(fake, None, 1, None, 0, 0, ref) == -1         # nothing to sort
    assert lib.tsqs_graph_create(fake, None, 1 << 32, None, 0, 0, ref) == -1   # too long
    assert lib.tsqs_graph_create(ctypes.c_void_p(0x1002), None, 100, None, 0, 0, ref) == -1  # alignment
    p, keep = _offs([0, 5, 3])
    assert lib.tsqs_graph_create(fake, None, 3, p, 2, 0, ref) == -1            # decreasing
    p, keep = _offs([0, 5, 9])
    assert lib.tsqs_graph_create(fake, None, 10, p, 2, 0, ref) == -1           # total != nmemb
    p, keep = _offs([0, 1, 2])
    assert lib.tsqs_graph_create(fake, None, 2, p, 2, 0, ref) == -1            # arrays <= 1
    assert not out.value
    assert lib.tsqs_graph_launch(None, None) == -1
    assert lib.tsqs_graph_stats(None, None) == -1
    assert lib.tsqs_graph_destroy(None) == -1


def test_options(lib):
    import paper_1505_00558_amd as tsqs
    old = tsqs.get_option(tsqs.OPT_SMALL_MAX)
    try:
        assert lib.tsqs_set_option(tsqs.OPT_SMALL_MAX, 8) == -1
        assert lib.tsqs_set_option(tsqs.OPT_SMALL_MAX, 1 << 20) == -1
        assert lib.tsqs_set_option(tsqs.OPT_SMALL_MAX, 1024) == 0
        assert tsqs.get_option(tsqs.OPT_SMALL_MAX) == 1024
        assert lib.tsqs_set_option(tsqs.OPT_SAMPLES, 4) == -1          # must be odd
        assert lib.tsqs_set_option(tsqs.OPT_SAMPLES, 65) == -1
        assert lib.tsqs_set_option(tsqs.OPT_PIVOT_MODE, 2) == -1
        assert lib.tsqs_set_option(tsqs.OPT_FINISH_ALGO, 4) == -1
        assert tsqs.get_option(tsqs.OPT_FINISH_ALGO) == 3
        assert tsqs.get_option(tsqs.OPT_PRESORT) == 1
        assert lib.tsqs_set_option(tsqs.OPT_PRESORT, 0) == 0
        assert tsqs.get_option(tsqs.OPT_PRESORT) == 0
        assert lib.tsqs_set_option(tsqs.OPT_PRESORT, 1) == 0
        assert tsqs.get_option(tsqs.OPT_SCHEDULE) == 0
        assert lib.tsqs_set_option(tsqs.OPT_SCHEDULE, 2) == -1
        assert lib.tsqs_set_option(tsqs.OPT_SCHEDULE, 1) == 0
        assert tsqs.get_option(tsqs.OPT_SCHEDULE) == 1
        assert lib.tsqs_set_option(tsqs.OPT_SCHEDULE, 0) == 0
        assert tsqs.get_option(tsqs.OPT_ITER_CAP) == 0
        assert lib.tsqs_set_option(tsqs.OPT_ITER_CAP, -1) == -1
        assert lib.tsqs_set_option(tsqs.OPT_ITER_CAP, 0) == 0
        assert tsqs.get_option(tsqs.OPT_QUEUE_DIRECT) == 1 << 22
        assert lib.tsqs_set_option(tsqs.OPT_QUEUE_DIRECT, -1) == -1
        assert lib.tsqs_set_option(tsqs.OPT_QUEUE_DIRECT, 1 << 32) == -1
        assert lib.tsqs_set_option(tsqs.OPT_QUEUE_DIRECT, 0) == 0
        assert tsqs.get_option(tsqs.OPT_QUEUE_DIRECT) == 0
        assert lib.tsqs_set_option(tsqs.OPT_QUEUE_DIRECT, 1 << 22) == 0
        for key, ok, bad in ((tsqs.OPT_PART_THREADS1, (512, 1024), (256, 768, 2048)),
                             (tsqs.OPT_PART_THREADS2, (256, 512), (128, 384, 1024))):
            assert tsqs.get_option(key) == ok[0]
            for v in bad:
                assert lib.tsqs_set_option(key, v) == -1
            for v in ok[::-1]:
                assert lib.tsqs_set_option(key, v) == 0
                assert tsqs.get_option(key) == v
        assert tsqs.get_option(tsqs.OPT_WORKSPACE_CAP) == 0
        assert lib.tsqs_set_option(tsqs.OPT_WORKSPACE_CAP, -1) == -1
        assert lib.tsqs_set_option(tsqs.OPT_WORKSPACE_CAP, 1 << 20) == 0
        assert tsqs.get_option(tsqs.OPT_WORKSPACE_CAP) == 1 << 20
        assert lib.tsqs_set_option(tsqs.OPT_WORKSPACE_CAP, 0) == 0
        assert tsqs.get_option(tsqs.OPT_DEBUG) == 0
        assert lib.tsqs_set_option(tsqs.OPT_DEBUG, 1) == 0 and tsqs.get_option(tsqs.OPT_DEBUG) == 1
        assert lib.tsqs_set_option(tsqs.OPT_DEBUG, 4) == -1
        assert lib.tsqs_set_option(tsqs.OPT_DEBUG, -1) == -1
        assert lib.tsqs_set_option(tsqs.OPT_DEBUG, 0) == 0
        assert lib.tsqs_set_option(999, 1) == -4
        assert tsqs.get_option(999) == -(1 << 63)
    finally:
        tsqs.set_option(tsqs.OPT_SMALL_MAX, old)


def test_stats_before_any_sort(lib):
    import paper_1505_00558_amd as tsqs
    s = tsqs.Stats()
    assert lib.tsqs_get_stats(None) == -1
    # no successful call yet in this process: nothing to report
    assert lib.tsqs_get_stats(ctypes.byref(s)) in (0, -1)


def test_product_path_has_no_oracle_import():
    """The library package neither imports the oracle nor carries a CPU sort."""
    pkg = os.path.join(ROOT, "paper_1505_00558_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                with open(os.path.join(dirpath, fn)) as f:
                    txt = f.read()
                assert "oracle" not in txt, fn


def test_queue_argument_errors(lib):
    """Queue calls reject bad arguments before any HIP call."""
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p()
    t = ctypes.c_uint64()
    assert lib.tsqs_queue_open(1 << 30, None, None) == -1
    assert lib.tsqs_queue_open(1 << 20, None, ctypes.byref(out)) == -1     # below 64 MiB
    assert lib.tsqs_queue_submit(None, fake, 5, 0, ctypes.byref(t)) == -1
    assert lib.tsqs_queue_step(None) == -1
    assert lib.tsqs_queue_poll(None, 1) == -1
    assert lib.tsqs_queue_result(None, 1, None, None) == -1
    assert lib.tsqs_queue_release(None, 1) == -1
    assert lib.tsqs_queue_cancel(None, 1) == -1
    assert lib.tsqs_queue_reap(None, None, 0, None) == -1
    assert lib.tsqs_queue_info(None, None, None, None, None, None) == -1
    assert lib.tsqs_queue_close(None) == -1


def test_autotune_argument_errors(lib):
    import paper_1505_00558_amd as tsqs
    t = tsqs.Tune()
    assert lib.tsqs_autotune(9, 0, 1000, None, 0, None, ctypes.byref(t)) == -4
    assert lib.tsqs_autotune(0, 0, 1, None, 0, None, ctypes.byref(t)) == -1
    assert lib.tsqs_autotune(0, 0, 1 << 32, None, 0, None, ctypes.byref(t)) == -1
    p, keep = _offs([0, 5, 3])
    assert lib.tsqs_autotune(0, 0, 3, p, 2, None, ctypes.byref(t)) == -1     # decreasing
    p, keep = _offs([0, 5, 9])
    assert lib.tsqs_autotune(0, 0, 10, p, 2, None, ctypes.byref(t)) == -1    # n != last offset


def test_sort_records_argument_checks(lib):
    """Argument errors of tsqs_sort_records, all detected before any device work."""
    fake, fake2 = ctypes.c_void_p(0x10000000), ctypes.c_void_p(0x10000100)
    assert lib.tsqs_sort_records(fake, fake, 8, None, 0, 0, None) == 0           # nothing to do
    assert lib.tsqs_sort_records(None, fake, 8, None, 10, 0, None) == -1         # null keys
    assert lib.tsqs_sort_records(fake, None, 8, None, 10, 0, None) == -1         # null records
    assert lib.tsqs_sort_records(fake, fake, 0, None, 10, 0, None) == -1         # empty records
    assert lib.tsqs_sort_records(fake, fake, 65537, None, 10, 0, None) == -1     # too large
    assert lib.tsqs_sort_records(fake, fake, 8, None, 1 << 32, 0, None) == -1    # n >= 2^32
    assert lib.tsqs_sort_records(fake, fake, 64, fake2, 10, 0, None) == -1       # overlapping out
    assert lib.tsqs_sort_records(fake, fake, 8, None, 10, 9, None) == -4         # bad dtype


def test_noalloc_argument_errors(lib):
    """tsqs_sort_noalloc refuses bad arguments and requests above its fixed
    maximum before any device work (no GPU needed)."""
    import paper_1505_00558_amd as tsqs
    assert lib.tsqs_sort_noalloc(None, None, 0, tsqs.INT32, None) == tsqs.OK
    assert lib.tsqs_sort_noalloc(None, None, 1, tsqs.INT32, None) == tsqs.OK
    assert lib.tsqs_sort_noalloc(None, None, 10, tsqs.INT32, None) == tsqs.EINVAL
    assert lib.tsqs_sort_noalloc(None, None, 10, 9, None) == tsqs.EUNSUPPORTED
    big = tsqs.NOALLOC_MAX_KEYS + 1
    assert lib.tsqs_sort_noalloc(ctypes.c_void_p(256), None, big, tsqs.INT32, None) == tsqs.ESCRATCH
    assert "scratch" in tsqs.strerror(tsqs.ESCRATCH)
