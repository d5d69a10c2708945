"""GPU parity at the benchmark's full sizes, in the launch configuration that
bench.py times (default options): every 2^28 int32 family, the two 2^27 uint64
arrays with their uint32 payload, and the 2^27 float32 array with specials.

At these sizes the keys are compared bit for bit with the CPU oracle's output
on the same input (every 2^28 int32 family, the 2^27 float32 array, the
uniform 2^27 uint64 keys), and with torch.sort of the same input (an
independent library sort); payloads are checked to be a permutation that
carries its keys."""
import numpy as np
import pytest

import tsqs_inputs as ti

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    yield
    torch.cuda.empty_cache()


def _ranks(n):
    return [0, 1, n // 3, n // 2, n - 2, n - 1]


@pytest.mark.parametrize("fam", ti.FAMILIES)
def test_full_size_int32_family(oracle_mod, fam):
    import paper_1505_00558_amd as tsqs
    import torch
    n = 1 << 28
    print("case: full size 2^28 int32", fam, flush=True)
    t = ti.device_family(fam, n, "int32", seed=ti.seed_for(2, fam))
    host = t.cpu().numpy()
    ref = torch.sort(t).values
    tsqs.sort(t)
    torch.cuda.synchronize()
    assert bool(torch.equal(t, ref))
    del ref
    got = t.cpu().numpy()
    assert np.array_equal(got, oracle_mod.sort(host))
    del t
    torch.cuda.empty_cache()


@pytest.mark.parametrize("variant", ["uniform", "distinct10"])
def test_full_size_uint64_pairs(oracle_mod, variant):
    import paper_1505_00558_amd as tsqs
    import torch
    n = 1 << 27
    print("case: full size 2^27 uint64 + payload", variant, flush=True)
    if variant == "uniform":
        k = ti.family("uniform", n, "uint64", seed=ti.seed_for(3, 0))
    else:
        k = ti.distinct10_u64(ti.seed_for(3, 1), n)
    orig = torch.from_numpy(k.view(np.int64)).to("cuda:0")
    t = orig.clone()
    v = torch.arange(n, dtype=torch.int32, device=t.device)
    tsqs.sort_pairs(t, v, tsqs.UINT64)
    torch.cuda.synchronize()
    # uint64 order = int64 order of the keys with the top bit flipped
    flip = torch.tensor(-(1 << 63), dtype=torch.int64, device=t.device)
    ref = torch.sort(orig ^ flip).values ^ flip
    assert bool(torch.equal(t, ref))
    del ref
    vv = v.to(torch.int64)
    assert bool(torch.equal(torch.sort(vv).values, torch.arange(n, dtype=torch.int64, device=t.device)))
    assert bool(torch.equal(orig[vv], t))
    got = t.cpu().numpy().view(np.uint64)
    if variant == "uniform":
        assert np.array_equal(got, oracle_mod.sort(k))
    else:
        r = _ranks(n)
        assert np.array_equal(got[r], np.partition(k, r)[r])
    del orig, t, v, vv
    torch.cuda.empty_cache()


def test_full_size_float32_specials(oracle_mod):
    import paper_1505_00558_amd as tsqs
    import torch
    n = 1 << 27
    print("case: full size 2^27 float32 with specials", flush=True)
    k = ti.special_float32(ti.seed_for(3, 2), n)
    t = torch.from_numpy(k).to("cuda:0")

    def codes(x):
        # IEEE totalOrder as unsigned 32-bit codes (negatives reversed), in int64
        b = x.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        return torch.where(b >= (1 << 31), 0xFFFFFFFF - b, b + (1 << 31))

    ref = torch.sort(codes(t)).values
    tsqs.sort(t, tsqs.FLOAT32)
    torch.cuda.synchronize()
    assert bool(torch.equal(codes(t), ref))
    del ref
    got = t.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle_mod.sort(k).view(np.uint32))
    del t
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fam", ["uniform", "many_equals"])
def test_wide_int32_part(fam):
    """A single array of more than 4 GiB of keys (the partition's 64-bit
    addressing variant, and bands longer than a band chunk for many equals)."""
    import paper_1505_00558_amd as tsqs
    import torch
    n = (1 << 30) + 4097
    print("case: wide int32", fam, n, flush=True)
    t = ti.device_family(fam, n, "int32", seed=ti.seed_for(2, fam) + 5)
    ref = torch.sort(t).values
    tsqs.sort(t)
    torch.cuda.synchronize()
    assert bool(torch.equal(t, ref))
    del t, ref
    torch.cuda.empty_cache()


def test_wide_uint64_pairs():
    """More than 4 GiB of uint64 keys with a uint32 payload in one array."""
    import paper_1505_00558_amd as tsqs
    import torch
    n = (1 << 29) + 333
    print("case: wide uint64 pairs", n, flush=True)
    orig = ti.device_family("uniform", n, "uint64", seed=ti.seed_for(3, 0) + 9)
    t = orig.clone()
    v = torch.arange(n, dtype=torch.int32, device=t.device)
    tsqs.sort_pairs(t, v, tsqs.UINT64)
    torch.cuda.synchronize()
    flip = torch.tensor(-(1 << 63), dtype=torch.int64, device=t.device)
    ref = torch.sort(orig ^ flip).values ^ flip
    assert bool(torch.equal(t, ref))
    del ref
    vv = v.to(torch.int64)
    assert bool(torch.equal(torch.sort(vv).values, torch.arange(n, dtype=torch.int64, device=t.device)))
    assert bool(torch.equal(orig[vv], t))
    del orig, t, v, vv
    torch.cuda.empty_cache()
