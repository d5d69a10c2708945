"""The seeded generators: pinned to the published SplitMix64 outputs and to the
family definitions."""
import os

import numpy as np
import pytest

import tsqs_inputs as ti

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_splitmix64_reference_outputs():
    ref = []
    with open(os.path.join(GOLD, "splitmix64_seed0.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                ref.append(int(line, 16))
    got = [int(x) for x in ti.splitmix64(0, len(ref))]
    assert got == ref


def test_counter_based_offsets():
    a = ti.splitmix64(77, 1000)
    b = ti.splitmix64(77, 10, start=500)
    assert np.array_equal(a[500:510], b)


def test_family_shapes():
    n = 10
    assert ti.family("sorted", n).tolist() == list(range(10))
    assert ti.family("reversed", n).tolist() == list(range(9, -1, -1))
    assert ti.family("organ_pipe", n).tolist() == [1, 2, 3, 4, 5, 5, 4, 3, 2, 1]
    st = ti.family("stair_steps", 3500)
    assert st[999] == 0 and st[1000] == 1 and st[3499] == 3
    me = ti.family("many_equals", 100000)
    assert me.min() >= 0 and me.max() < 100 and len(np.unique(me)) == 100
    ns = ti.family("nearly_sorted", 100000)
    assert np.array_equal(np.sort(ns), np.arange(100000))
    moved = np.count_nonzero(ns != np.arange(100000))
    assert 0 < moved <= 2 * (100000 // 200)


def test_uniform_int32_full_range():
    u = ti.family("uniform", 1 << 16, "int32")
    assert u.dtype == np.int32 and u.min() < -(1 << 30) and u.max() > (1 << 30)


def test_special_floats():
    n = 1 << 18
    f = ti.family("uniform", n, "float32").view(np.uint32)
    for bits in ti.SPECIAL_F32_BITS:
        frac = np.count_nonzero(f == np.uint32(bits)) / n
        assert 0.0005 < frac < 0.0015
    g = ti.normal_float32(3, n)
    assert abs(float(g.mean())) < 0.02 and abs(float(g.std()) - 1.0) < 0.02


def test_distinct10():
    k = ti.distinct10_u64(5, 100000)
    assert len(np.unique(k)) <= 10000


def test_batch_layout():
    keys, offs, fams = ti.batch(11, 200, lo_log2=4, hi_log2=12)
    sizes = np.diff(offs.astype(np.int64))
    assert len(sizes) == 200 and sizes.min() >= 16 and sizes.max() <= 4096
    assert int(offs[-1]) == keys.size
    j = 17
    alone = ti.family(fams[j], int(sizes[j]), "int32", seed=11 + 0x100000 + j)
    assert np.array_equal(keys[int(offs[j]):int(offs[j + 1])], alone)
    k2, o2, _ = ti.batch(11, 200, lo_log2=4, hi_log2=12, max_total=50000)
    assert int(o2[-1]) <= 50000


def test_batch_plan_matches_batch():
    keys, offs, fams = ti.batch(4242, 50, 4, 12)
    sizes, poffs, pfams, seeds = ti.batch_plan(4242, 50, 4, 12)
    assert np.array_equal(offs, poffs) and fams == pfams
    assert np.array_equal(np.diff(poffs).astype(np.int64), sizes)
    for j in (0, 17, 49):
        a, b = int(offs[j]), int(offs[j + 1])
        assert np.array_equal(keys[a:b], ti.family(fams[j], b - a, "int32", seed=int(seeds[j])))
    _, coffs, _, _ = ti.batch_plan(4242, 50, 4, 12, max_total=5000)
    assert int(coffs[-1]) <= 5000


def test_device_generator_library_exports():
    import ctypes
    path = os.path.join(os.path.dirname(ti.__file__), "libtsqs_inputs.so")
    if not os.path.exists(path):
        pytest.skip("libtsqs_inputs.so not built")
    lib = ctypes.CDLL(path)
    assert hasattr(lib, "tsqs_inputs_generate")
    lib.tsqs_inputs_generate.restype = ctypes.c_int
    # argument errors are reported before any device work
    assert lib.tsqs_inputs_generate(None, 0, None, None, None, 1, None) == -1


def test_paper_types_closed_forms():
    """SVI input types at n = 10, m = 3 (hill from its definition; sawtooth,
    stagger and plateau from their published definitions)."""
    assert ti.paper_type("hill", 10, 3).tolist() == [0, 1, 2, 3, 3, 3, 3, 3, 2, 1]
    assert ti.paper_type("hill", 9, 100).tolist() == [0, 1, 2, 3, 5, 4, 3, 2, 1]
    assert ti.paper_type("sawtooth", 10, 3).tolist() == [0, 1, 2, 0, 1, 2, 0, 1, 2, 0]
    assert ti.paper_type("stagger", 10, 3).tolist() == [0, 4, 8, 2, 6, 0, 4, 8, 2, 6]
    assert ti.paper_type("plateau", 10, 3).tolist() == [0, 1, 2, 3, 3, 3, 3, 3, 3, 3]
    r = ti.paper_type("random", 100000, 50, seed=4)
    assert r.min() == 0 and r.max() == 49
    s = ti.paper_type("shuffle", 100000, 4, seed=5)
    ev, od = s[s % 2 == 0], s[s % 2 == 1]
    # two interleaved runs: the evens 0, 2, 4, ... and the odds 1, 3, 5, ... in order
    assert np.array_equal(ev, 2 * np.arange(ev.size)) and np.array_equal(od, 2 * np.arange(od.size) + 1)
    assert 0.2 < od.size / s.size < 0.3                   # one in m = 4 picks the odd run
    o = ti.paper_type("organ_pipes", 200000, 1000, seed=6)
    assert o.min() >= 1 and o.max() <= 1000
    assert np.abs(np.diff(o)).max() <= 1000


def test_paper_fort_by_hand():
    """Fort of 0..7 with ranges longer than 2 split: reverse all, then each half, then
    each quarter (worked out by hand)."""
    assert ti.fort(np.arange(8), 2).tolist() == [5, 4, 7, 6, 1, 0, 3, 2]
    assert ti.fort(np.arange(5), 100).tolist() == [4, 3, 2, 1, 0]        # one reversal
    # 0..6, ranges longer than 1 split: [0,6] reversed: 6 5 4 3 2 1 0; [0,3] reversed:
    # 3 4 5 6, then [0,1] and [2,3]: 4 3 6 5; [4,6] reversed: 0 1 2, then [4,5]: 1 0
    assert ti.fort(np.arange(7), 1).tolist() == [4, 3, 6, 5, 1, 0, 2]


def test_paper_orders():
    n, m = 11, 1000
    v = ti.paper_type("random", n, m, seed=9)
    get = lambda o: ti.paper_input("random", o, n, m, dtype="int64", seed=9)
    assert np.array_equal(get("as_is"), v)
    assert np.array_equal(get("sorted"), np.sort(v))
    assert np.array_equal(get("reversed"), v[::-1])
    assert np.array_equal(get("front_half_reversed"), np.r_[v[:5][::-1], v[5:]])
    assert np.array_equal(get("back_half_reversed"), np.r_[v[:5], v[5:][::-1]])
    assert np.array_equal(get("dither"), v + np.arange(n) % 5)
    f = ti.paper_input("random", "fort", 4096, m, dtype="int64", seed=9)
    assert np.array_equal(np.sort(f), np.sort(ti.paper_type("random", 4096, m, seed=9)))
