"""GPU tests of the batched segmented sort (many independent arrays, one call)
and of the device-side input generator it is benchmarked with.

Keys of sampled arrays are compared bit for bit with the CPU oracle (the arrays
regenerated alone on the host from their sub-seeds); the full-size batch of
100,000 arrays is checked on every array through properties that hold at any
size: each array non-decreasing, and its key multiset unchanged (two
order-independent per-array sums, modulo 2^64).
"""
import numpy as np
import pytest

import tsqs_inputs as ti
from gpu_util import device_ok, CODES, from_dev, same_bits

pytestmark = pytest.mark.gpu

BATCH_SEED = ti.seed_for(4, 0)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    yield


def _ulp_close_f32(a, b):
    """Equal bits, or finite values one float32 ulp apart (Box-Muller goes
    through log/cos, whose last bit may differ between host and device libm)."""
    ab, bb = a.view(np.uint32), b.view(np.uint32)
    same = ab == bb
    fin = np.isfinite(a) & np.isfinite(b) & (np.sign(a) == np.sign(b))
    near = fin & (np.abs(ab.astype(np.int64) - bb.astype(np.int64)) <= 1)
    return bool(np.all(same | near))


@pytest.mark.parametrize("dtype", list(ti.DTYPES))
@pytest.mark.parametrize("fam", ti.FAMILIES)
def test_device_generator_matches_host(dtype, fam):
    for n in (1, 37, 1000, 70001):
        seed = 1000 + n
        host = ti.family(fam, n, dtype, seed=seed)
        dev = from_dev(ti.device_family(fam, n, dtype, seed=seed), dtype)
        if dtype == "float32" and fam == "uniform":
            assert _ulp_close_f32(dev, host), (fam, dtype, n)
        else:
            assert same_bits(dev, host), (fam, dtype, n)


def test_device_batch_matches_host():
    keys, offs, fams = ti.batch(BATCH_SEED, 300, 4, 14)
    t, doffs, dfams = ti.device_batch(BATCH_SEED, 300, 4, 14)
    assert np.array_equal(offs, doffs) and fams == dfams
    assert same_bits(from_dev(t, np.int32), keys)


def test_batch_100000_arrays_full_size(oracle_mod):
    """The batched workload at full size in the benchmark's launch configuration:
    100,000 int32 arrays, log-uniform sizes in [16, 2^20], one tsqs_sort_batch."""
    import paper_1505_00558_amd as tsqs
    import torch
    sizes, offs, fams, seeds = ti.batch_plan(BATCH_SEED, 100000, 4, 20)
    print("case: batch 100000 arrays, %d keys" % int(offs[-1]), flush=True)
    t, doffs, _ = ti.device_batch(BATCH_SEED, 100000, 4, 20)
    t0 = t.clone()
    tsqs.sort_batch(t, offs)
    torch.cuda.synchronize()
    device_ok()
    # every array element by element against an independent sort: torch.sort of
    # (array index << 32 | key code) over groups of arrays of up to 2^28 keys
    nseg = offs.size - 1
    j0 = 0
    while j0 < nseg:
        j1 = j0 + 1
        while j1 < nseg and int(offs[j1 + 1] - offs[j0]) <= (1 << 28):
            j1 += 1
        a, b = int(offs[j0]), int(offs[j1])
        lens = torch.from_numpy((offs[j0 + 1:j1 + 1] - offs[j0:j1]).astype(np.int64)).to(t.device)
        ids = torch.repeat_interleave(torch.arange(j1 - j0, dtype=torch.int64, device=t.device), lens)
        comp = (ids << 32) | (t0[a:b].to(torch.int64) + (1 << 31))
        exp = (torch.sort(comp).values & 0xFFFFFFFF) - (1 << 31)
        assert bool(torch.equal(t[a:b].to(torch.int64), exp)), (j0, j1)
        del lens, ids, comp, exp
        j0 = j1
    del t0
    # sampled arrays against the oracle: the largest, the smallest, and a spread
    pick = set(np.linspace(0, len(sizes) - 1, 24).astype(int).tolist())
    pick |= {int(np.argmax(sizes)), int(np.argmin(sizes))}
    for j in sorted(pick):
        a, b = int(offs[j]), int(offs[j + 1])
        host = ti.family(fams[j], b - a, "int32", seed=int(seeds[j]))
        got = t[a:b].cpu().numpy()
        assert same_bits(got, oracle_mod.sort(host)), (j, fams[j], b - a)
    del t
    torch.cuda.empty_cache()


def test_batch_equals_one_call_per_array():
    """Capped batch (arrays drawn until 2^24 keys): the batched result equals
    sorting every array with its own tsqs_sort call."""
    import paper_1505_00558_amd as tsqs
    import torch
    t0, offs, fams = ti.device_batch(BATCH_SEED + 1, 100000, 4, 20, max_total=1 << 24)
    print("case: batch vs plain, %d arrays" % (offs.size - 1), flush=True)
    t1 = t0.clone()
    tsqs.sort_batch(t0, offs)
    for j in range(offs.size - 1):
        tsqs.sort(t1[int(offs[j]):int(offs[j + 1])])
    torch.cuda.synchronize()
    assert bool(torch.equal(t0, t1))
