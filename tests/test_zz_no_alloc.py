"""tsqs_sort_noalloc (the entry point that allocates nothing) against tsqs_sort
and tsqs_sort_pairs, through the C ABI.

Two calls in a row on every key type, the second with a smaller input of
another family, each compared bit for bit with the allocating entry point on
the same input and with the oracle; payloads follow their keys.  A request
above the fixed maximum is refused before any device work.
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


def _noalloc(a, v=None):
    import paper_1505_00558_amd as tsqs
    import torch
    t = to_dev(a)
    tv = None if v is None else to_dev(np.asarray(v, dtype=np.uint32))
    tsqs.sort_noalloc(t, tv, CODES[np.dtype(a.dtype)])
    torch.cuda.synchronize()
    return from_dev(t, a.dtype), (None if tv is None else from_dev(tv, np.uint32))


@pytest.mark.parametrize("dtype", list(ti.DTYPES))
def test_noalloc_keys_two_calls(oracle_mod, dtype):
    import paper_1505_00558_amd as tsqs
    for n, fam, seed in ((tsqs.NOALLOC_MAX_KEYS, "uniform", 11), (50003, "many_equals", 12)):
        print("case: noalloc keys", dtype, fam, n, flush=True)
        k = ti.family(fam, n, dtype, seed=ti.seed_for(9, fam) + seed)
        got, _ = _noalloc(k)
        assert same_bits(got, gpu_sort(k))
        assert same_bits(got, oracle_mod.sort(k))


@pytest.mark.parametrize("dtype", list(ti.DTYPES))
def test_noalloc_pairs_two_calls(oracle_mod, dtype):
    for n, fam, seed in ((300007, "organ_pipe", 21), (1000, "uniform", 22)):
        print("case: noalloc pairs", dtype, fam, n, flush=True)
        k = ti.family(fam, n, dtype, seed=ti.seed_for(9, fam) + seed)
        v = np.arange(n, dtype=np.uint32)
        gk, gv = _noalloc(k, v)
        rk, _ = gpu_sort_pairs(k, v)
        assert same_bits(gk, rk)
        assert same_bits(gk, oracle_mod.sort(k))
        assert payload_valid(k, gk, gv)


def test_noalloc_refuses_above_maximum():
    import paper_1505_00558_amd as tsqs
    import torch
    n = tsqs.NOALLOC_MAX_KEYS + 1
    print("case: noalloc refuses", n, flush=True)
    k = ti.family("uniform", n, "int32", seed=5)
    t = to_dev(k)
    with pytest.raises(tsqs.TsqsError) as e:
        tsqs.sort_noalloc(t)
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert same_bits(from_dev(t, np.int32), k)
