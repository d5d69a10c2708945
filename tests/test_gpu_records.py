"""GPU parity of records sorted by their keys (late swapping, SVIII.H).

Keys must be bit-identical to the oracle's output.  Each record carries the
index of its key in the input, so the records are checked to be a permutation
of the input records in which record i belongs to output key i (records with
equal keys may come out in any order)."""
import numpy as np
import pytest

import tsqs_inputs as ti
from gpu_util import from_dev, same_bits, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    yield


def _records(n, rec_bytes, seed):
    """n records: bytes 0..3 the record's index (when there is room), the rest seeded."""
    body = (ti.splitmix64(seed, n * rec_bytes) & np.uint64(0xFF)).astype(np.uint8).reshape(n, rec_bytes)
    if rec_bytes >= 4:
        body[:, :4] = np.arange(n, dtype=np.uint32).view(np.uint8).reshape(n, 4)
    return body


def _check(oracle_mod, keys, recs, gk, gr):
    n, rb = recs.shape
    assert same_bits(gk, oracle_mod.sort(keys))
    assert rb >= 4
    idx = gr[:, :4].copy().view(np.uint32).reshape(n).astype(np.int64)
    assert np.array_equal(np.sort(idx), np.arange(n))
    assert np.array_equal(gr, recs[idx])
    assert same_bits(keys[idx], gk)


def _run(keys, recs, out_of_place, out_offset=0):
    import paper_1505_00558_amd as tsqs
    import torch
    from gpu_util import CODES
    tk = to_dev(keys)
    n, rb = recs.shape
    raw = torch.from_numpy(recs.reshape(-1).copy()).to("cuda:0")
    if out_of_place:
        big = torch.zeros(n * rb + out_offset, dtype=torch.uint8, device="cuda:0")
        out = big[out_offset:]
        tsqs.sort_records(tk, raw.view(n, rb), out=out.view(n, rb), dtype_code=CODES[keys.dtype])
        torch.cuda.synchronize()
        assert bool(torch.equal(raw.cpu(), torch.from_numpy(recs.reshape(-1))))   # input untouched
        res = out
    else:
        tsqs.sort_records(tk, raw.view(n, rb), dtype_code=CODES[keys.dtype])
        torch.cuda.synchronize()
        res = raw
    return from_dev(tk, keys.dtype), res.cpu().numpy().reshape(n, rb)


@pytest.mark.parametrize("rec_bytes", [4, 8, 12, 16, 56, 320, 1000])
@pytest.mark.parametrize("out_of_place", [False, True])
def test_record_sizes(oracle_mod, rec_bytes, out_of_place):
    n = 300007
    print("case: records", rec_bytes, "out" if out_of_place else "in place", flush=True)
    keys = ti.family("uniform", n, "int32", seed=31)
    recs = _records(n, rec_bytes, 32)
    gk, gr = _run(keys, recs, out_of_place)
    _check(oracle_mod, keys, recs, gk, gr)


@pytest.mark.parametrize("fam", ["many_equals", "reversed", "sorted", "organ_pipe"])
@pytest.mark.parametrize("dtype", ["int64", "float32", "uint32"])
def test_record_families(oracle_mod, fam, dtype):
    n = (1 << 18) + 11
    print("case: records family", fam, dtype, flush=True)
    keys = ti.family(fam, n, dtype, seed=33)
    recs = _records(n, 56, 34)
    gk, gr = _run(keys, recs, True)
    _check(oracle_mod, keys, recs, gk, gr)


@pytest.mark.parametrize("offset", [1, 2, 4, 8])
def test_unaligned_output(oracle_mod, offset):
    """An output buffer at an odd offset: the gather falls back to narrower words."""
    n = 70001
    print("case: records unaligned out", offset, flush=True)
    keys = ti.family("uniform", n, "int32", seed=35)
    recs = _records(n, 24, 36)
    gk, gr = _run(keys, recs, True, out_offset=offset)
    _check(oracle_mod, keys, recs, gk, gr)


@pytest.mark.parametrize("n", [1, 2, 3, 8193, 8194])
def test_small_counts(oracle_mod, n):
    print("case: records small", n, flush=True)
    keys = ti.family("uniform", n, "int32", seed=37)
    recs = _records(n, 56, 38)
    for oop in (False, True):
        gk, gr = _run(keys, recs, oop)
        _check(oracle_mod, keys, recs, gk, gr)


def test_one_byte_records(oracle_mod):
    """Records smaller than a word (byte copies); keys with their record byte equal."""
    n = 100003
    keys = ti.family("uniform", n, "int32", seed=39)
    recs = (keys.view(np.uint32) & np.uint32(0xFF)).astype(np.uint8).reshape(n, 1)
    gk, gr = _run(keys, recs, False)
    assert same_bits(gk, oracle_mod.sort(keys))
    assert np.array_equal(gr.reshape(n), (gk.view(np.uint32) & np.uint32(0xFF)).astype(np.uint8))
