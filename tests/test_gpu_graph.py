"""GPU tests of captured sorts (tsqs_graph_*): every replay of a graph sorts
what its buffers hold at that moment exactly like the eager call, with the
program's own eager sorts (which grow and reuse the library's workspace) and
synchronisations between the replays; replays on two streams are ordered."""
import numpy as np
import pytest

import tsqs_inputs as ti
from gpu_util import CODES, from_dev, payload_valid, same_bits, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    yield


@pytest.mark.parametrize("dtype", ["int32", "uint64", "float32"])
def test_graph_single_array_replays(oracle_mod, dtype):
    import paper_1505_00558_amd as tsqs
    import torch
    n = (1 << 20) + 37
    inputs = [ti.family(f, n, dtype, seed=50 + j) for j, f in
              enumerate(["uniform", "organ_pipe", "many_equals", "sorted"])]
    work = to_dev(inputs[0])
    g = tsqs.Graph(work, dtype_code=CODES[np.dtype(dtype)])
    try:
        for r, a in enumerate(inputs):
            print("case: graph replay", dtype, r, flush=True)
            work.copy_(to_dev(a))
            # eager work between replays: a larger sort grows the library's workspace
            other = ti.device_family("uniform", (1 << 21) + r, "int32", seed=90 + r)
            tsqs.sort(other)
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            assert g.stats()["error_flags"] == 0
            assert same_bits(from_dev(work, a.dtype), oracle_mod.sort(a)), r
            assert bool(torch.equal(other, torch.sort(ti.device_family(
                "uniform", (1 << 21) + r, "int32", seed=90 + r)).values))
    finally:
        g.destroy()


def test_graph_batch_with_payloads_replays(oracle_mod):
    import paper_1505_00558_amd as tsqs
    import torch
    sizes = [1, 0, 17, 5000, 8193, 70000, 300001, 2]
    offs = np.cumsum([0] + sizes).astype(np.uint64)
    n = int(offs[-1])
    work = torch.empty(n, dtype=torch.int64, device="cuda:0")
    vals = torch.empty(n, dtype=torch.int32, device="cuda:0")
    g = tsqs.Graph(work, offsets=offs, vals=vals, dtype_code=tsqs.INT64)
    s2 = torch.cuda.Stream()
    try:
        for r in range(4):
            print("case: graph batch replay", r, flush=True)
            keys = np.concatenate([ti.family(ti.FAMILIES[(r + j) % 7], m, "int64", seed=200 + 10 * r + j)
                                   for j, m in enumerate(sizes)])
            work.copy_(to_dev(keys))
            vals.copy_(torch.arange(n, dtype=torch.int32, device="cuda:0"))
            tsqs.sort_pairs(to_dev(keys), to_dev(np.arange(n, dtype=np.uint32)), tsqs.INT64)
            torch.cuda.synchronize()
            if r % 2:
                with torch.cuda.stream(s2):      # a replay on another stream
                    g.launch()
            else:
                g.launch()
            torch.cuda.synchronize()
            got = from_dev(work, np.int64)
            gv = from_dev(vals, np.uint32)
            for a, b in zip(offs[:-1].tolist(), offs[1:].tolist()):
                assert same_bits(got[a:b], oracle_mod.sort(keys[a:b])), (r, a, b)
                assert np.all((gv[a:b] >= a) & (gv[a:b] < b))
            assert payload_valid(keys, got, gv)
    finally:
        g.destroy()
