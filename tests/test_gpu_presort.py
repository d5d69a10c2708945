"""GPU parity of the presortedness check (the sorted / reversed handlers of
SIII.I, done once per single array before its first pass).

Keys must be bit-identical to the oracle's output.  Which way the check
decided is read from the call's statistics (presorted: 0 = partitioned as
usual, 1 = found non-decreasing, 2 = found non-increasing and reversed): a
single adjacent pair out of order anywhere (at a wave, chunk or array edge,
or between two of the probe's sampled keys) must send the array to the
partition passes, and the answer must be the oracle's either way.
"""
import numpy as np
import pytest

import tsqs_inputs as ti
from gpu_util import CODES, from_dev, gpu_sort, gpu_sort_pairs, payload_valid, same_bits, to_dev

pytestmark = pytest.mark.gpu

N = (1 << 20) + 37          # a ragged last chunk (4096 keys per chunk)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    # the cases are sized around the default small-part size (an earlier test may
    # have left the autotuner's choice in place)
    before = tsqs.get_option(tsqs.OPT_SMALL_MAX)
    tsqs.set_option(tsqs.OPT_SMALL_MAX, 8192)
    yield
    tsqs.set_option(tsqs.OPT_PRESORT, 1)
    tsqs.set_option(tsqs.OPT_SMALL_MAX, before)


def _check(oracle_mod, k, want):
    import paper_1505_00558_amd as tsqs
    got = gpu_sort(k)
    st = tsqs.get_stats()
    assert same_bits(got, oracle_mod.sort(k))
    assert st["presorted"] == want
    if want:
        assert sum(st["level_keys"]) == 0 and st["small_keys"] == 0


def _oracle_sorted(oracle_mod, fam, n, dtype, seed):
    return oracle_mod.sort(ti.family(fam, n, dtype, seed=seed))


@pytest.mark.parametrize("dtype", list(ti.DTYPES))
def test_sorted_and_reversed(oracle_mod, dtype):
    print("case: presort sorted/reversed", dtype, flush=True)
    asc = _oracle_sorted(oracle_mod, "uniform", N, dtype, 11)
    _check(oracle_mod, asc, 1)
    _check(oracle_mod, np.ascontiguousarray(asc[::-1]), 2)


@pytest.mark.parametrize("dtype", ["int32", "uint64", "float32"])
def test_ties(oracle_mod, dtype):
    """Runs of equal keys: non-decreasing / non-increasing, and all keys equal."""
    print("case: presort ties", dtype, flush=True)
    asc = _oracle_sorted(oracle_mod, "many_equals", N, dtype, 12)
    _check(oracle_mod, asc, 1)
    _check(oracle_mod, np.ascontiguousarray(asc[::-1]), 2)
    _check(oracle_mod, np.full(N, asc[N // 2], dtype=asc.dtype), 1)


def test_float32_specials_reversed(oracle_mod):
    """NaNs of both signs, infinities, -0.0 and +0.0 under totalOrder, reversed."""
    print("case: presort float32 specials", flush=True)
    asc = oracle_mod.sort(ti.special_float32(13, N))
    _check(oracle_mod, asc, 1)
    _check(oracle_mod, np.ascontiguousarray(asc[::-1]), 2)


# one adjacent pair out of order: first pair, a wave edge (lane 63 / 64), a chunk
# edge (4095 / 4096), between two probe samples, the last pair
BREAKS = [0, 63, 4095, N // 126, N // 2, N - 2]


@pytest.mark.parametrize("where", BREAKS)
@pytest.mark.parametrize("direction", ["ascending", "descending"])
def test_one_pair_out_of_order(oracle_mod, where, direction):
    print("case: presort one pair out of order", direction, where, flush=True)
    k = (np.arange(N, dtype=np.int64) * 3 - 3 * (N // 2)).astype(np.int32)   # strictly increasing
    if direction == "descending":
        k = np.ascontiguousarray(k[::-1])
    k = k.copy()
    k[where], k[where + 1] = k[where + 1], k[where]
    _check(oracle_mod, k, 0)


def _order(k):
    """1 if non-decreasing, 2 if non-increasing (and not constant), else 0."""
    if np.all(k[1:] >= k[:-1]):
        return 1
    return 2 if np.all(k[1:] <= k[:-1]) else 0


@pytest.mark.parametrize("fam", ti.FAMILIES)
def test_families(oracle_mod, fam):
    """Every input family: the check decides exactly as the input's order says
    (nearly sorted: a probe that may pass and a scan that must fail)."""
    print("case: presort family", fam, flush=True)
    k = ti.family(fam, N, "int32", seed=15)
    _check(oracle_mod, k, _order(k))


@pytest.mark.parametrize("n", [8193, 8194, 65537])
def test_small_edges(oracle_mod, n):
    """The smallest arrays that get a pass (at most small_max keys never do)."""
    print("case: presort small", n, flush=True)
    asc = _oracle_sorted(oracle_mod, "uniform", n, "uint32", 16)
    _check(oracle_mod, asc, 1)
    _check(oracle_mod, np.ascontiguousarray(asc[::-1]), 2)


@pytest.mark.parametrize("dtype", ["int32", "uint64"])
def test_pairs(oracle_mod, dtype):
    """Payloads: untouched for a sorted array, reversed with a reversed one."""
    print("case: presort pairs", dtype, flush=True)
    import paper_1505_00558_amd as tsqs
    asc = np.unique(_oracle_sorted(oracle_mod, "uniform", N, dtype, 17))
    n = asc.size
    v = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort_pairs(asc, v)
    assert tsqs.get_stats()["presorted"] == 1
    assert same_bits(gk, asc) and np.array_equal(gv, v)
    desc = np.ascontiguousarray(asc[::-1])
    gk, gv = gpu_sort_pairs(desc, v)
    assert tsqs.get_stats()["presorted"] == 2
    assert same_bits(gk, asc) and np.array_equal(gv, v[::-1])
    ties = np.ascontiguousarray(_oracle_sorted(oracle_mod, "many_equals", N, dtype, 18)[::-1])
    v = np.arange(N, dtype=np.uint32)
    gk, gv = gpu_sort_pairs(ties, v)
    assert tsqs.get_stats()["presorted"] == 2
    assert same_bits(gk, oracle_mod.sort(ties)) and payload_valid(ties, gk, gv)


def test_option_off(oracle_mod):
    """TSQS_OPT_PRESORT 0: sorted and reversed arrays take the partition passes."""
    import paper_1505_00558_amd as tsqs
    asc = _oracle_sorted(oracle_mod, "uniform", N, "int32", 19)
    tsqs.set_option(tsqs.OPT_PRESORT, 0)
    try:
        for k in (asc, np.ascontiguousarray(asc[::-1])):
            got = gpu_sort(k)
            st = tsqs.get_stats()
            assert same_bits(got, asc)
            assert st["presorted"] == 0 and st["level_keys"][0] == k.size
    finally:
        tsqs.set_option(tsqs.OPT_PRESORT, 1)


def _as_dtype(x, dtype):
    """The int32 pattern x as keys of another type, order kept."""
    x = x.astype(np.int64)
    if dtype == "int32":
        return x.astype(np.int32)
    if dtype == "uint32":
        return (x + (1 << 31)).astype(np.uint32)
    if dtype == "int64":
        return x * 3 - (1 << 40)
    if dtype == "uint64":
        return (x + (1 << 40)).astype(np.uint64)
    return x.astype(np.float32)      # |x| < 2^24: exact


@pytest.mark.parametrize("with_vals", [False, True], ids=["keys", "pairs"])
@pytest.mark.parametrize("dtype", list(ti.DTYPES))
def test_batch_arrays(oracle_mod, dtype, with_vals):
    """Batches: each array that needs a pass, up to 2^16 keys, is checked by its own
    wave; arrays found in order (here: sorted, reversed, all equal) take no pass, the
    others do.  Every key type, keys alone and with payloads."""
    import paper_1505_00558_amd as tsqs
    import torch
    asc = (np.arange(N, dtype=np.int64) * 5 - 5 * (N // 2)).astype(np.int32)
    uni = ti.family("uniform", N, "int32", seed=40) >> 8
    near = asc.copy()
    near[1000], near[1001] = near[1001], near[1000]
    parts = [asc[:60000], asc[60000:120000][::-1], np.full(20000, 7, np.int32), uni[:200000],
             near[:50000], asc[:3000][::-1], uni[:9000][::-1].copy(), asc[200000:400000]]
    parts = [_as_dtype(p, dtype) for p in parts]
    if dtype == "float32":
        # a descending run through +0.0 and -0.0 (strictly decreasing in
        # totalOrder, so it is reversed, -0.0 before +0.0)
        parts[1] = np.concatenate([np.arange(30000, 0, -1) + 0.5, [0.0, -0.0],
                                   -(np.arange(1, 30000) + 0.5)]).astype(np.float32)
    offs = np.cumsum([0] + [p.size for p in parts]).astype(np.uint64)
    keys = np.concatenate(parts)
    # small-part size of the type: 8192 4-byte records, 4096 8-byte, 2048 16-byte
    # (8-byte keys with a payload); the 3000 reversed keys are a small part (no
    # pass, no check) unless the records are 16 bytes
    rec = keys.dtype.itemsize + (4 if with_vals else 0)
    rec = 16 if rec > 8 else rec
    small_max = 8192 * 4 // rec
    found = 3 + (1 if 3000 > small_max else 0)
    for presort, want in ((1, found), (0, 0)):
        print("case: batch presort", dtype, with_vals, presort, flush=True)
        tsqs.set_option(tsqs.OPT_PRESORT, presort)
        try:
            t = to_dev(keys.copy())
            v = torch.arange(keys.size, dtype=torch.int32, device="cuda:0") if with_vals else None
            tsqs.sort_batch(t, offs, vals=v, dtype_code=CODES[keys.dtype])
            torch.cuda.synchronize()
            st = tsqs.get_stats()
        finally:
            tsqs.set_option(tsqs.OPT_PRESORT, 1)
        got = from_dev(t, keys.dtype)
        # found in order: 60000 sorted, 60000 reversed, 20000 equal keys (and the
        # 3000 reversed keys when they are not a small part); the 200000 sorted
        # keys are above the size a wave checks: they take the passes
        assert st["presorted"] == want
        for a, b in zip(offs[:-1].tolist(), offs[1:].tolist()):
            assert same_bits(got[a:b], oracle_mod.sort(keys[a:b]))
        if with_vals:
            gv = v.cpu().numpy().astype(np.int64)
            for a, b in zip(offs[:-1].tolist(), offs[1:].tolist()):
                assert np.all((gv[a:b] >= a) & (gv[a:b] < b))
            assert np.array_equal(np.sort(gv), np.arange(keys.size))
            assert same_bits(keys[gv], got)


def test_large_arrays_skip_the_passes(oracle_mod):
    """A large array found in order partitions nothing (its levels are launched
    without waiting for the check's answer, and find no part); one pair out of
    order still takes every pass."""
    import paper_1505_00558_amd as tsqs
    n = (1 << 24) + 5
    print("case: presort large", n, flush=True)
    asc = (np.arange(n, dtype=np.int64) * 7 - 7 * (n // 2)).astype(np.int32)
    for k, want in ((asc, 1), (np.ascontiguousarray(asc[::-1]), 2)):
        got = gpu_sort(k)
        st = tsqs.get_stats()
        assert np.array_equal(got, asc)
        assert st["presorted"] == want
        assert sum(st["level_parts"]) == 0 and st["tail_parts"] == 0
    k = asc.copy()
    k[n - 3], k[n - 2] = k[n - 2], k[n - 3]
    got = gpu_sort(k)
    st = tsqs.get_stats()
    assert same_bits(got, oracle_mod.sort(k))
    assert st["presorted"] == 0 and sum(st["level_parts"]) > 0
