"""GPU tests of the serving queue (include/tsqs_queue.h): continuously batched
requests of mixed key types give the same keys as each request sorted alone,
and as the CPU oracle; admission respects the arena; completion flags are
raised exactly for the requests whose keys are all final."""
import time

import numpy as np
import pytest

import tsqs_inputs as ti
from gpu_util import from_dev, same_bits, to_dev

pytestmark = pytest.mark.gpu

DTYPES = ["int32", "float32", "int64"]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    yield


def _requests(seed, count, lo_log2, hi_log2):
    """Host arrays of a request mix: sizes log-uniform, key type and family drawn
    per request from the seeded stream."""
    sizes = ti.batch_sizes(seed, count, lo_log2, hi_log2)
    x = ti.splitmix64(seed + 3, count)
    out = []
    for j, n in enumerate(sizes.tolist()):
        dt = DTYPES[int(x[j] % np.uint64(3))]
        fam = ti.FAMILIES[int((x[j] >> np.uint64(8)) % np.uint64(7))]
        out.append((dt, fam, ti.family(fam, n, dt, seed=seed + 0x100000 + j)))
    return out


def _drain(q, tickets, limit_s=120.0):
    """Step the queue until every ticket is done (bounded wait)."""
    t0 = time.time()
    left = set(tickets)
    while left:
        q.step()
        left = {t for t in left if q.poll(t) != q.DONE}
        assert time.time() - t0 < limit_s, "queue did not finish in %.0f s" % limit_s


def test_queue_mix_equals_alone_and_oracle(oracle_mod):
    import paper_1505_00558_amd as tsqs
    import torch
    reqs = _requests(0x5E12, 48, 10, 20)
    srcs = [to_dev(a) for _, _, a in reqs]
    print("case: queue mix of %d requests, %d keys" % (len(reqs), sum(a.size for *_, a in reqs)),
          flush=True)
    q = tsqs.Queue(4 << 30)
    # alone: one request in the queue at a time
    alone = []
    for (dt, fam, a), t in zip(reqs, srcs):
        tk = q.submit(t)
        _drain(q, [tk])
        alone.append(from_dev(q.result(tk).clone(), a.dtype))
        q.release(tk)
    # mix: submissions spread over the ticks of earlier requests
    tickets = []
    for i, t in enumerate(srcs):
        tickets.append(q.submit(t))
        if i % 5 == 4:
            for _ in range(3):
                q.step()
    _drain(q, tickets)
    torch.cuda.synchronize()
    for (dt, fam, a), tk, al in zip(reqs, tickets, alone):
        got = from_dev(q.result(tk).clone(), a.dtype)
        assert same_bits(got, al), (dt, fam, a.size)
        assert same_bits(got, oracle_mod.sort(a)), (dt, fam, a.size)
        q.release(tk)
    info = q.info()
    assert info["queued"] == 0 and info["running"] == 0 and info["done"] == 0
    assert info["arena_used"] == 0
    q.close()


def test_queue_source_unchanged_and_tiny_requests(oracle_mod):
    import paper_1505_00558_amd as tsqs
    q = tsqs.Queue(256 << 20)
    arrs = [np.array([7], dtype=np.int32), np.array([3, -1], dtype=np.int32),
            ti.family("uniform", 16, "int64", seed=5), ti.family("organ_pipe", 1000, "float32"),
            ti.family("many_equals", 8193, "int32", seed=9)]
    srcs = [to_dev(a) for a in arrs]
    tks = [q.submit(t) for t in srcs]
    _drain(q, tks)
    for a, t, tk in zip(arrs, srcs, tks):
        assert same_bits(from_dev(q.result(tk).clone(), a.dtype), oracle_mod.sort(a))
        assert same_bits(from_dev(t, a.dtype), a)      # the source is not sorted in place
        q.release(tk)
    q.close()


def test_queue_admission_waits_for_space(oracle_mod):
    """With an arena that holds only a few requests, later ones stay queued (first
    in, first out) until earlier results are released, then complete."""
    import paper_1505_00558_amd as tsqs
    q = tsqs.Queue(256 << 20)
    cap = q.info()["arena_bytes"]
    n = (cap // 4) // 3 - 64                            # three int32 requests fill the arena
    arrs = [ti.family(f, n, "int32", seed=40 + j) for j, f in
            enumerate(["uniform", "reversed", "many_equals", "stair_steps", "uniform"])]
    srcs = [to_dev(a) for a in arrs]
    tks = [q.submit(t) for t in srcs]
    q.step()
    states = [q.poll(t) for t in tks]
    assert states[3] == q.QUEUED and states[4] == q.QUEUED
    _drain(q, tks[:3])
    assert q.poll(tks[3]) == q.QUEUED                   # no room until a release
    for tk, a in zip(tks[:3], arrs[:3]):
        assert same_bits(from_dev(q.result(tk).clone(), np.int32), oracle_mod.sort(a))
        q.release(tk)
    _drain(q, tks[3:])
    for tk, a in zip(tks[3:], arrs[3:]):
        assert same_bits(from_dev(q.result(tk).clone(), np.int32), oracle_mod.sort(a))
        q.release(tk)
    assert q.info()["arena_used"] == 0
    q.close()


def test_queue_largest_requests():
    """The largest request size of the serving workload (2^24 keys) for each key
    type, together in one queue; checked against an independent library sort
    (torch.sort; for float32 on the totalOrder integer codes)."""
    import paper_1505_00558_amd as tsqs
    import torch
    n = 1 << 24
    q = tsqs.Queue(8 << 30)
    items = []
    for dt in DTYPES:
        t = ti.device_family("uniform", n, dt, seed=ti.seed_for(5, 0))
        items.append((dt, t, q.submit(t)))
    print("case: queue 3 x 2^24", flush=True)
    _drain(q, [tk for *_, tk in items])
    for dt, t, tk in items:
        got = q.result(tk)
        if dt == "float32":
            # totalOrder: compare the order-preserving integer codes
            b = t.view(torch.int32)
            code = torch.where(b < 0, ~b, b | torch.tensor(-2**31, dtype=torch.int32,
                                                             device=b.device))
            ref_code = torch.sort(code.to(torch.int64) & 0xFFFFFFFF).values
            gb = got.view(torch.int32)
            gcode = torch.where(gb < 0, ~gb, gb | torch.tensor(-2**31, dtype=torch.int32,
                                                                device=gb.device))
            assert bool(torch.equal(gcode.to(torch.int64) & 0xFFFFFFFF, ref_code))
        else:
            assert bool(torch.equal(got, torch.sort(t).values))
        q.release(tk)
    q.close()
