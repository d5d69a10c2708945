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
from gpu_util import CODES, from_dev, same_bits

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


def _array_sums(t, offs):
    """Per-array (sum of x, sum of x*x + 0x9E3779B97F4A7C15*x) modulo 2^64, on the
    device, in slices (int64 arithmetic wraps)."""
    import torch
    n = int(offs[-1])
    o = torch.from_numpy(offs.astype(np.int64)).to(t.device)
    c1 = torch.zeros(offs.size, dtype=torch.int64, device=t.device)
    c2 = torch.zeros_like(c1)
    step = 1 << 27
    carry1 = torch.zeros((), dtype=torch.int64, device=t.device)
    carry2 = torch.zeros_like(carry1)
    golden = -7046029254386353131  # 0x9E3779B97F4A7C15 as int64
    for a in range(0, n, step):
        b = min(n, a + step)
        x = t[a:b].to(torch.int64)
        s1 = torch.cumsum(x, 0) + carry1
        s2 = torch.cumsum(x * x + x * golden, 0) + carry2
        # prefix sums at the offsets that fall in (a, b]
        sel = (o > a) & (o <= b)
        idx = o[sel] - a - 1
        c1[sel] = s1[idx]
        c2[sel] = s2[idx]
        carry1, carry2 = s1[-1], s2[-1]
        del x, s1, s2
    return (c1[1:] - c1[:-1]).cpu().numpy(), (c2[1:] - c2[:-1]).cpu().numpy()


def _sorted_each(t, offs):
    import torch
    n = int(offs[-1])
    starts = torch.from_numpy(offs[1:-1].astype(np.int64)).to(t.device)
    step = 1 << 28
    for a in range(0, n - 1, step):
        b = min(n - 1, a + step)
        desc = torch.nonzero(t[a:b] > t[a + 1:b + 1]).flatten() + (a + 1)
        if desc.numel() and not bool(torch.isin(desc, starts).all()):
            return False
    return True


def test_batch_100000_arrays_full_size(oracle_mod):
    """The batched workload at full size in the benchmark's launch configuration:
    100,000 int32 arrays, log-uniform sizes in [16, 2^20], one tsqs_sort_batch."""
    import paper_1505_00558_amd as tsqs
    import torch
    sizes, offs, fams, seeds = ti.batch_plan(BATCH_SEED, 100000, 4, 20)
    print("case: batch 100000 arrays, %d keys" % int(offs[-1]), flush=True)
    t, doffs, _ = ti.device_batch(BATCH_SEED, 100000, 4, 20)
    before = _array_sums(t, offs)
    tsqs.sort_batch(t, offs)
    torch.cuda.synchronize()
    assert _sorted_each(t, offs)
    after = _array_sums(t, offs)
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
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
