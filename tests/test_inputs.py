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
