"""The persistent schedule and the non-blocking boundary, through the C ABI.

* A call only enqueues: right after tsqs_sort of 2^28 keys returns, the stream
  still has work; after synchronising, the keys equal the oracle's.
* TSQS_OPT_SCHEDULE 1 (every part in the persistent kernel, one launch):
  bit-identical to the oracle for every key type and family, pairs and
  batches (arrays alone vs together).
* The exact-minimum test mode at 2^26 int32: every large part's exact pivot is
  selected by the whole grid (select rounds counted), keys bit-identical to
  the oracle.
* The iteration cap: a cap of one iteration stops the persistent kernel with
  an error flag (reported by tsqs_get_stats) instead of running on; the next
  call with the default cap is correct.
* Calls on two streams one after the other without a host wait share the
  workspace correctly.
"""
import time

import numpy as np
import pytest

import tsqs_inputs as ti
from gpu_util import CODES, device_ok, from_dev, gpu_sort, gpu_sort_pairs, payload_valid, same_bits, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    yield
    tsqs.set_option(tsqs.OPT_SCHEDULE, 0)
    tsqs.set_option(tsqs.OPT_ITER_CAP, 0)
    tsqs.set_option(tsqs.OPT_PIVOT_MODE, 0)


@pytest.fixture
def persistent():
    import paper_1505_00558_amd as tsqs
    tsqs.set_option(tsqs.OPT_SCHEDULE, tsqs.SCHEDULE_PERSISTENT)
    yield
    tsqs.set_option(tsqs.OPT_SCHEDULE, tsqs.SCHEDULE_LEVELS)


def test_call_returns_before_the_work_is_done(oracle_mod):
    import paper_1505_00558_amd as tsqs
    import torch
    n = 1 << 28
    print("case: non-blocking 2^28 int32 uniform", flush=True)
    k = ti.family("uniform", n, "int32", seed=ti.seed_for(2, "uniform"))
    t = to_dev(k)
    torch.cuda.synchronize()
    tsqs.sort(t)
    pending = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    st = device_ok()
    assert pending, "tsqs_sort waited for its device work"
    assert st["levels"] > 0
    assert same_bits(from_dev(t, np.int32), oracle_mod.sort(k))


@pytest.mark.parametrize("dtype", list(ti.DTYPES))
@pytest.mark.parametrize("fam", ti.FAMILIES)
def test_persistent_families(oracle_mod, persistent, dtype, fam):
    n = (1 << 20) + 37
    print("case: persistent", dtype, fam, n, flush=True)
    k = ti.family(fam, n, dtype, seed=ti.seed_for(2, fam) + 9)
    got = gpu_sort(k)
    assert same_bits(got, oracle_mod.sort(k))


@pytest.mark.parametrize("dtype", list(ti.DTYPES))
def test_persistent_pairs(oracle_mod, persistent, dtype):
    n = 300007
    print("case: persistent pairs", dtype, n, flush=True)
    k = ti.family("uniform", n, dtype, seed=77)
    v = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort_pairs(k, v)
    assert same_bits(gk, oracle_mod.sort(k))
    assert payload_valid(k, gk, gv)


@pytest.mark.parametrize("with_vals", [False, True])
def test_persistent_batch(oracle_mod, persistent, with_vals):
    import paper_1505_00558_amd as tsqs
    import torch
    print("case: persistent batch", with_vals, flush=True)
    sizes = [0, 1, 5, 16, 300, 8192, 8193, 70000, 200003, 3, 1 << 18]
    arrays = [ti.family(ti.FAMILIES[j % len(ti.FAMILIES)], s, "int32", seed=100 + j)
              for j, s in enumerate(sizes)]
    keys = np.concatenate(arrays)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    t = to_dev(keys)
    tv = to_dev(np.arange(keys.size, dtype=np.uint32)) if with_vals else None
    tsqs.sort_batch(t, offs, tv)
    torch.cuda.synchronize()
    device_ok()
    out = from_dev(t, np.int32)
    for j, a in enumerate(arrays):
        seg = out[offs[j]:offs[j + 1]]
        assert same_bits(seg, oracle_mod.sort(a)), j
    if with_vals:
        vo = from_dev(tv, np.uint32)
        assert payload_valid(keys, out, vo)


def test_min_pivot_grid_select_2e26(oracle_mod):
    """Exact-minimum pivots (the depth-limit test mode) at 2^26 int32: the first
    split keeps nearly every key, so the part's subtree takes exact-median
    pivots at once; those of large parts come from grid-wide selection rounds,
    and the whole sort stays within a few times a normal sort's time."""
    import paper_1505_00558_amd as tsqs
    import torch
    n = 1 << 26
    print("case: min pivot 2^26 int32", flush=True)
    k = ti.family("uniform", n, "int32", seed=ti.seed_for(2, "uniform") + 3)
    t = to_dev(k)
    tsqs.set_option(tsqs.OPT_PIVOT_MODE, 1)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tsqs.sort(t)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        st = device_ok()
    finally:
        tsqs.set_option(tsqs.OPT_PIVOT_MODE, 0)
    print("min-pivot sort: %.1f ms, tail parts %d, tail keys %d, select rounds %d, fallbacks %d"
          % (ms, st["tail_parts"], st["tail_keys"], st["select_rounds"], st["fallback_parts"]),
          flush=True)
    assert st["select_rounds"] > 0 and st["fallback_parts"] > 0
    assert same_bits(from_dev(t, np.int32), oracle_mod.sort(k))
    assert ms < 100.0        # a 2^26 sort takes about 2 ms; 52 peeling passes took 130 ms


def test_iteration_cap_reports_instead_of_running_on(oracle_mod, persistent):
    import paper_1505_00558_amd as tsqs
    import torch
    n = 1 << 20
    print("case: iteration cap", flush=True)
    k = ti.family("uniform", n, "int32", seed=4)
    t = to_dev(k)
    tsqs.set_option(tsqs.OPT_ITER_CAP, 1)
    try:
        tsqs.sort(t)
        torch.cuda.synchronize()
        rc, st = tsqs.last_call_status()
    finally:
        tsqs.set_option(tsqs.OPT_ITER_CAP, 0)
    assert rc == tsqs.EINTERNAL and (st["error_flags"] & 32), (rc, st["error_flags"])
    # the next call, with the default cap, is whole
    assert same_bits(gpu_sort(k), oracle_mod.sort(k))


def test_two_streams_share_the_workspace(oracle_mod):
    import paper_1505_00558_amd as tsqs
    import torch
    print("case: two streams", flush=True)
    a = ti.family("uniform", 3000017, "int64", seed=1)
    b = ti.family("organ_pipe", 2000003, "int64", seed=2)
    ta, tb = to_dev(a), to_dev(b)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(sa):
        tsqs.sort(ta)
    with torch.cuda.stream(sb):
        tsqs.sort(tb)
    torch.cuda.synchronize()
    device_ok()
    assert same_bits(from_dev(ta, np.int64), oracle_mod.sort(a))
    assert same_bits(from_dev(tb, np.int64), oracle_mod.sort(b))


def test_level_schedule_tail_with_three_samples(oracle_mod):
    """Three pivot samples leave parts after the launched levels; the
    persistent kernel finishes them."""
    import paper_1505_00558_amd as tsqs
    tsqs.set_option(tsqs.OPT_SAMPLES, 3)
    tails = 0
    try:
        for fam in ti.FAMILIES:
            print("case: 3 samples", fam, flush=True)
            k = ti.family(fam, 1 << 21, "int32", seed=ti.seed_for(2, fam) + 11)
            assert same_bits(gpu_sort(k), oracle_mod.sort(k)), fam
            tails += tsqs.get_stats()["tail_parts"]
    finally:
        tsqs.set_option(tsqs.OPT_SAMPLES, 63)
    print("parts finished by the persistent kernel:", tails, flush=True)
