"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Keys must be bit-identical to the oracle's output (the unique sorted
arrangement under the stated order); payloads must be a permutation that stays
with its keys (the sort is unstable, so payload order among equal keys is not
compared).
"""
import numpy as np
import pytest

import tsqs_inputs as ti
from gpu_util import CODES, from_dev, gpu_sort, gpu_sort_pairs, payload_valid, same_bits, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    yield
    tsqs.set_option(tsqs.OPT_FINISH_ALGO, 3)
    tsqs.set_option(tsqs.OPT_PART_GRID, 0)
    tsqs.set_option(tsqs.OPT_FINISH_GRID, 0)
    tsqs.set_option(tsqs.OPT_SMALL_MAX, 8192)
    tsqs.set_option(tsqs.OPT_SAMPLES, 63)
    tsqs.set_option(tsqs.OPT_PIVOT_MODE, 0)
    tsqs.set_option(tsqs.OPT_PRESORT, 1)
    tsqs.set_option(tsqs.OPT_PART_THREADS1, 512)
    tsqs.set_option(tsqs.OPT_PART_THREADS2, 256)


def test_config1_one_million_int32(oracle_mod):
    print("case: 1e6 int32 uniform", flush=True)
    k = ti.family("uniform", 1000000, "int32", seed=ti.seed_for(1, "uniform"))
    assert same_bits(gpu_sort(k), oracle_mod.sort(k))


@pytest.mark.parametrize("dtype", list(ti.DTYPES))
@pytest.mark.parametrize("fam", ti.FAMILIES)
def test_families_dtypes(oracle_mod, dtype, fam):
    n = (1 << 20) + 37
    print("case:", dtype, fam, n, flush=True)
    k = ti.family(fam, n, dtype, seed=ti.seed_for(2, fam) + 5)
    ref = oracle_mod.sort(k)
    assert same_bits(gpu_sort(k), ref)
    if fam in ("sorted", "reversed", "stair_steps"):
        # found in order by the presortedness check: also through the passes
        import paper_1505_00558_amd as tsqs
        tsqs.set_option(tsqs.OPT_PRESORT, 0)
        try:
            assert same_bits(gpu_sort(k), ref)
        finally:
            tsqs.set_option(tsqs.OPT_PRESORT, 1)


@pytest.mark.parametrize("dtype", list(ti.DTYPES))
@pytest.mark.parametrize("fam", ["uniform", "many_equals", "organ_pipe"])
def test_pairs(oracle_mod, dtype, fam):
    n = 300007
    print("case: pairs", dtype, fam, n, flush=True)
    k = ti.family(fam, n, dtype, seed=ti.seed_for(3, fam) + 1)
    v = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort_pairs(k, v)
    rk, _ = oracle_mod.sort_pairs(k, v)
    assert same_bits(gk, rk)
    assert payload_valid(k, gk, gv)


def test_distinct10_u64_pairs(oracle_mod):
    n = 500009
    k = ti.distinct10_u64(123, n)
    v = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort_pairs(k, v)
    assert same_bits(gk, oracle_mod.sort(k))
    assert payload_valid(k, gk, gv)


EDGE_N = [0, 1, 2, 3, 15, 16, 17, 255, 4095, 4096, 4097, 8191, 8192, 8193, 8194, 12289,
          65537, 131071]


@pytest.mark.parametrize("n", EDGE_N)
@pytest.mark.parametrize("fam", ["uniform", "many_equals", "sorted", "reversed"])
def test_edge_sizes(oracle_mod, n, fam):
    print("case: edge", fam, n, flush=True)
    k = ti.family(fam, n, "int32", seed=n + 1)
    assert same_bits(gpu_sort(k), oracle_mod.sort(k))
    v = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort_pairs(k, v)
    assert same_bits(gk, oracle_mod.sort(k))
    assert payload_valid(k, gk, gv)


@pytest.mark.parametrize("n", [2, 100, 9000, 300000])
def test_all_equal_and_two_values(oracle_mod, n):
    a = np.full(n, -7, dtype=np.int32)
    assert same_bits(gpu_sort(a), a)
    b = (ti.splitmix64(9, n) % np.uint64(2)).astype(np.int64) * (1 << 40)
    assert same_bits(gpu_sort(b), oracle_mod.sort(b))


def test_extreme_values(oracle_mod):
    n = 100003
    for dt, lo, hi in [(np.int32, -(1 << 31), (1 << 31) - 1), (np.uint32, 0, (1 << 32) - 1),
                       (np.int64, -(1 << 63), (1 << 63) - 1), (np.uint64, 0, (1 << 64) - 1)]:
        sel = ti.splitmix64(31, n) % np.uint64(3)
        k = np.where(sel == 0, lo, np.where(sel == 1, hi, 0)).astype(dt)
        assert same_bits(gpu_sort(k), oracle_mod.sort(k)), dt


def test_float_specials_and_payload_nans(oracle_mod):
    n = 400009
    f = ti.special_float32(5, n).view(np.uint32).copy()
    sel = ti.splitmix64(6, n) % np.uint64(500)
    f[sel == 0] = 0xFFC00000          # negative quiet NaN
    f[sel == 1] = 0x7FC00123          # NaN with a payload
    f[sel == 2] = 0x7F800001          # signaling NaN bits
    f[sel == 3] = 0x00000001          # subnormal
    f = f.view(np.float32)
    assert same_bits(gpu_sort(f), oracle_mod.sort(f))


@pytest.mark.parametrize("small_max", [16, 100, 1024])
def test_small_threshold_variants(oracle_mod, small_max):
    import paper_1505_00558_amd as tsqs
    tsqs.set_option(tsqs.OPT_SMALL_MAX, small_max)
    try:
        for fam in ("uniform", "stair_steps", "organ_pipe"):
            k = ti.family(fam, 200003, "int64", seed=small_max)
            assert same_bits(gpu_sort(k), oracle_mod.sort(k)), fam
            v = np.arange(k.size, dtype=np.uint32)
            gk, gv = gpu_sort_pairs(k, v)
            assert payload_valid(k, gk, gv)
    finally:
        tsqs.set_option(tsqs.OPT_SMALL_MAX, 8192)


def test_three_samples(oracle_mod):
    import paper_1505_00558_amd as tsqs
    tsqs.set_option(tsqs.OPT_SAMPLES, 3)
    try:
        for fam in ti.FAMILIES:
            k = ti.family(fam, 500000, "uint32")
            assert same_bits(gpu_sort(k), oracle_mod.sort(k)), fam
    finally:
        tsqs.set_option(tsqs.OPT_SAMPLES, 63)


@pytest.mark.parametrize("fam", ["uniform", "many_equals", "sorted"])
def test_min_pivot_forces_depth_fallback(oracle_mod, fam):
    """Exact-minimum pivots peel one value off a part; a child that keeps more
    than 15/16 of its part's keys takes the depth limit at once, and the
    exact-median fallback must then finish within log2(n) more levels."""
    import paper_1505_00558_amd as tsqs
    n = 60001
    k = ti.family(fam, n, "int32", seed=3)
    tsqs.set_option(tsqs.OPT_PIVOT_MODE, 1)
    tsqs.set_option(tsqs.OPT_PRESORT, 0)     # a sorted array must take the passes here
    try:
        got = gpu_sort(k)
        st = tsqs.get_stats()
    finally:
        tsqs.set_option(tsqs.OPT_PIVOT_MODE, 0)
        tsqs.set_option(tsqs.OPT_PRESORT, 1)
    assert same_bits(got, oracle_mod.sort(k))
    lg = int(np.ceil(np.log2(n)))
    if fam != "many_equals":
        assert st["fallback_parts"] > 0
    assert st["levels"] <= 2 * lg + lg + 2


def test_stats_and_timing():
    import paper_1505_00558_amd as tsqs
    import torch
    n = 1 << 22
    k = ti.family("uniform", n, "int32", seed=1)
    tsqs.set_option(tsqs.OPT_TIMING, 1)
    try:
        t = to_dev(k)
        tsqs.sort(t)
        st = tsqs.get_stats()
    finally:
        tsqs.set_option(tsqs.OPT_TIMING, 0)
    assert st["n"] == n and st["levels"] >= 1
    assert st["level_keys"][0] == n
    assert st["partition_bytes"] == 2 * 4 * sum(st["level_keys"])
    assert st["partition_ms"] > 0
    assert st["small_keys"] + st["band_keys"] == n
    assert bool((t[1:] >= t[:-1]).all().item())


@pytest.mark.parametrize("with_vals", [False, True])
def test_batch_each_array_alone(oracle_mod, with_vals):
    import paper_1505_00558_amd as tsqs
    import torch
    keys, offs, fams = ti.batch(2024, 300, lo_log2=4, hi_log2=16)
    print("case: batch", with_vals, keys.size, flush=True)
    t = to_dev(keys)
    tv = to_dev(np.arange(keys.size, dtype=np.uint32)) if with_vals else None
    tsqs.sort_batch(t, offs, tv, CODES[keys.dtype])
    torch.cuda.synchronize()
    got = from_dev(t, keys.dtype)
    gv = from_dev(tv, np.uint32) if with_vals else None
    for j in range(len(offs) - 1):
        a, b = int(offs[j]), int(offs[j + 1])
        assert same_bits(got[a:b], oracle_mod.sort(keys[a:b])), (j, fams[j])
        if with_vals:
            assert np.all((gv[a:b] >= a) & (gv[a:b] < b))
    if with_vals:
        assert payload_valid(keys, got, gv)


def test_batch_float_and_int64(oracle_mod):
    import paper_1505_00558_amd as tsqs
    import torch
    for dt in ("float32", "int64"):
        keys, offs, _ = ti.batch(77, 120, lo_log2=1, hi_log2=15, dtype=dt)
        t = to_dev(keys)
        tsqs.sort_batch(t, offs, None, CODES[keys.dtype])
        torch.cuda.synchronize()
        got = from_dev(t, keys.dtype)
        for j in range(len(offs) - 1):
            a, b = int(offs[j]), int(offs[j + 1])
            assert same_bits(got[a:b], oracle_mod.sort(keys[a:b])), (dt, j)


def test_full_size_int32_properties():
    """2^28 int32 uniform keys in the bench's launch configuration: sorted,
    equal to torch.sort of the input (an independent library sort), and
    order statistics at sampled ranks equal to numpy's selection."""
    import paper_1505_00558_amd as tsqs
    import torch
    n = 1 << 28
    print("case: full-size 2^28 int32", flush=True)
    k = ti.family("uniform", n, "int32", seed=ti.seed_for(2, "uniform"))
    t = to_dev(k)
    ref = torch.sort(t).values
    tsqs.sort(t)
    torch.cuda.synchronize()
    assert bool(torch.equal(t, ref))
    ranks = [0, 1, n // 3, n // 2, n - 2, n - 1]
    part = np.partition(k, ranks)
    got = t[torch.tensor(ranks, device="cuda:0")].cpu().numpy()
    assert np.array_equal(got, part[ranks])
    del ref
    torch.cuda.empty_cache()


@pytest.mark.parametrize("algo", [0, 1, 2])
@pytest.mark.parametrize("dtype", list(ti.DTYPES))
def test_finish_variants(oracle_mod, dtype, algo):
    """The alternative small-part sorts (TSQS_OPT_FINISH_ALGO 0: the bitonic
    network; 1: merge-path merging one output at a time; 2: cross-lane bitonic
    merging within a wave, then merge-path merging with register merge
    networks): keys and payloads as for the default (cross-lane bitonic merging
    within a wave, then merge-path merging one output at a time)."""
    import paper_1505_00558_amd as tsqs
    before = tsqs.get_option(tsqs.OPT_FINISH_ALGO)
    tsqs.set_option(tsqs.OPT_FINISH_ALGO, algo)
    try:
        for fam, n in (("uniform", 300007), ("many_equals", 70001), ("organ_pipe", 8191),
                       ("reversed", 4097), ("uniform", 333), ("sorted", 65)):
            k = ti.family(fam, n, dtype, seed=ti.seed_for(3, fam) + 7)
            assert same_bits(gpu_sort(k), oracle_mod.sort(k)), (fam, n)
            v = np.arange(n, dtype=np.uint32)
            gk, gv = gpu_sort_pairs(k, v)
            assert same_bits(gk, oracle_mod.sort(k)) and payload_valid(k, gk, gv), (fam, n)
    finally:
        tsqs.set_option(tsqs.OPT_FINISH_ALGO, before)


def test_autotune_chooses_valid_options_and_sorts(oracle_mod):
    """The autotuner measures candidate options, sets the fastest, and sorts
    under them still agree with the oracle (options restored afterwards)."""
    import paper_1505_00558_amd as tsqs
    before = {k: tsqs.get_option(k) for k in (tsqs.OPT_SMALL_MAX, tsqs.OPT_SAMPLES,
                                               tsqs.OPT_PART_GRID, tsqs.OPT_FINISH_GRID,
                                               tsqs.OPT_FINISH_ALGO, tsqs.OPT_PART_THREADS1,
                                               tsqs.OPT_PART_THREADS2)}
    try:
        r = tsqs.autotune(tsqs.INT32, 1 << 22)
        print("case: autotune", r, flush=True)
        assert r["trials"] >= 5 and r["ms_best"] <= r["ms_default"]
        assert tsqs.get_option(tsqs.OPT_SMALL_MAX) == r["small_max"]
        assert tsqs.get_option(tsqs.OPT_SAMPLES) == r["samples"]
        assert tsqs.get_option(tsqs.OPT_FINISH_ALGO) == r["finish_algo"]
        assert tsqs.get_option(tsqs.OPT_PART_THREADS1) == r["part_threads1"] in (512, 1024)
        assert tsqs.get_option(tsqs.OPT_PART_THREADS2) == r["part_threads2"] in (256, 512)
        for fam in ("uniform", "organ_pipe", "many_equals"):
            k = ti.family(fam, 1 << 20, "int32", seed=ti.seed_for(2, fam) + 3)
            assert same_bits(gpu_sort(k), oracle_mod.sort(k)), fam
        offs = np.array([0, 1000, 1000, 70000, 70001, 200000], dtype=np.uint64)
        r2 = tsqs.autotune(tsqs.UINT64, 0, with_payload=True, offsets=offs)
        assert r2["trials"] >= 5
    finally:
        for k, v in before.items():
            tsqs.set_option(k, v)


@pytest.mark.parametrize("dtype", ["int32", "uint64"])
def test_batch_empty_and_one_key_arrays(oracle_mod, dtype):
    """Batches whose arrays include empty and one-key arrays between larger
    ones, keys only and with payloads: each array equals the oracle's sort and
    payloads stay within their array."""
    import paper_1505_00558_amd as tsqs
    import torch
    sizes = [0, 1, 0, 2, 5000, 0, 1, 70001, 0, 8193, 1]
    arrs = [ti.family("uniform" if j % 2 else "many_equals", n, dtype, seed=300 + j)
            for j, n in enumerate(sizes)]
    keys = np.concatenate(arrs)
    offs = np.cumsum([0] + sizes).astype(np.uint64)
    for with_vals in (False, True):
        print("case: batch with empty arrays", dtype, with_vals, flush=True)
        t = to_dev(keys)
        tv = to_dev(np.arange(keys.size, dtype=np.uint32)) if with_vals else None
        tsqs.sort_batch(t, offs, tv, CODES[keys.dtype])
        torch.cuda.synchronize()
        got = from_dev(t, keys.dtype)
        gv = from_dev(tv, np.uint32) if with_vals else None
        for j, a in enumerate(arrs):
            lo, hi = int(offs[j]), int(offs[j + 1])
            assert same_bits(got[lo:hi], oracle_mod.sort(a)), (j, sizes[j])
            if with_vals:
                assert np.all((gv[lo:hi] >= lo) & (gv[lo:hi] < hi)), j
        if with_vals:
            assert payload_valid(keys, got, gv)


@pytest.mark.parametrize("algo", [2, 3])
@pytest.mark.parametrize("dtype", list(ti.DTYPES))
def test_small_part_sizes(oracle_mod, dtype, algo):
    """Arrays the small-part sort takes whole, sized so that the last waves of
    the workgroup hold only padding (they skip the register phase) or a few
    keys and padding, for every key type, keys alone and with payloads."""
    import paper_1505_00558_amd as tsqs
    before = tsqs.get_option(tsqs.OPT_FINISH_ALGO)
    tsqs.set_option(tsqs.OPT_FINISH_ALGO, algo)
    try:
        for n in (1025, 2049, 2100, 3000, 4095, 4097, 5000, 6145, 8191, 8192):
            print("case: small part", dtype, algo, n, flush=True)
            k = ti.family("uniform", n, dtype, seed=n)
            assert same_bits(gpu_sort(k), oracle_mod.sort(k)), n
            v = np.arange(n, dtype=np.uint32)
            gk, gv = gpu_sort_pairs(k, v)
            assert same_bits(gk, oracle_mod.sort(k)) and payload_valid(k, gk, gv), n
    finally:
        tsqs.set_option(tsqs.OPT_FINISH_ALGO, before)


@pytest.mark.parametrize("threads", [(1024, 256), (512, 512), (1024, 512)])
@pytest.mark.parametrize("dtype", list(ti.DTYPES))
def test_partition_workgroup_sizes(oracle_mod, dtype, threads):
    """The partition kernels at twice the threads with half the keys per thread
    (TSQS_OPT_PART_THREADS1 / 2): keys and payloads as for the default sizes."""
    import paper_1505_00558_amd as tsqs
    tsqs.set_option(tsqs.OPT_PART_THREADS1, threads[0])
    tsqs.set_option(tsqs.OPT_PART_THREADS2, threads[1])
    try:
        for fam, n in (("uniform", 300007), ("many_equals", 70001), ("organ_pipe", 200003),
                       ("stair_steps", 123457)):
            print("case: partition threads", threads, dtype, fam, n, flush=True)
            k = ti.family(fam, n, dtype, seed=ti.seed_for(3, fam) + 11)
            assert same_bits(gpu_sort(k), oracle_mod.sort(k)), (fam, n)
            v = np.arange(n, dtype=np.uint32)
            gk, gv = gpu_sort_pairs(k, v)
            assert same_bits(gk, oracle_mod.sort(k)) and payload_valid(k, gk, gv), (fam, n)
    finally:
        tsqs.set_option(tsqs.OPT_PART_THREADS1, 512)
        tsqs.set_option(tsqs.OPT_PART_THREADS2, 256)


def test_tune_cache(tmp_path, monkeypatch):
    """TSQS_TUNE_CACHE: the first tuning of a shape times candidates and appends
    one line (this device's architecture and the shape); the same shape again
    takes that line without timing anything and sets the same options; another
    shape tunes and appends."""
    import paper_1505_00558_amd as tsqs
    keys = (tsqs.OPT_SMALL_MAX, tsqs.OPT_SAMPLES, tsqs.OPT_PART_GRID, tsqs.OPT_FINISH_GRID,
            tsqs.OPT_FINISH_ALGO, tsqs.OPT_PART_THREADS1, tsqs.OPT_PART_THREADS2)
    names = ("small_max", "samples", "part_grid", "finish_grid", "finish_algo", "part_threads1",
             "part_threads2")
    before = {k: tsqs.get_option(k) for k in keys}
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("TSQS_TUNE_CACHE", str(path))
    try:
        r1 = tsqs.autotune(tsqs.INT32, 1 << 20)
        assert r1["trials"] >= 5
        lines = path.read_text().splitlines()
        assert len(lines) == 1 and lines[0].startswith("gfx") and " dt=0 v=0 b=0 lg=20 | " in lines[0]
        tsqs.set_option(tsqs.OPT_SMALL_MAX, 1024)
        tsqs.set_option(tsqs.OPT_FINISH_ALGO, 0)
        r2 = tsqs.autotune(tsqs.INT32, (1 << 20) - 5)     # the same ceil(log2 n)
        assert r2["trials"] == 0
        for k, nm in zip(keys, names):
            assert r2[nm] == r1[nm] and tsqs.get_option(k) == r1[nm], nm
        assert len(path.read_text().splitlines()) == 1
        r3 = tsqs.autotune(tsqs.INT32, 1 << 18, with_payload=True)
        assert r3["trials"] >= 5
        assert len(path.read_text().splitlines()) == 2
    finally:
        for k, v in before.items():
            tsqs.set_option(k, v)
