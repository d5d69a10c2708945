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


@pytest.fixture
def direct_min(request):
    """TSQS_OPT_QUEUE_DIRECT for the queues a test opens (restored after)."""
    import paper_1505_00558_amd as tsqs
    before = tsqs.get_option(tsqs.OPT_QUEUE_DIRECT)
    tsqs.set_option(tsqs.OPT_QUEUE_DIRECT, request.param)
    yield request.param
    tsqs.set_option(tsqs.OPT_QUEUE_DIRECT, before)


# 0: every request through the ticks; 1 << 19: the largest of these requests by
# the single-array schedule; 20000: most of them
@pytest.mark.parametrize("direct_min", [0, 1 << 19, 20000], indirect=True)
def test_queue_mix_equals_alone_and_oracle(oracle_mod, direct_min):
    import paper_1505_00558_amd as tsqs
    import torch
    reqs = _requests(0x5E12, 48, 10, 20)
    srcs = [to_dev(a) for _, _, a in reqs]
    print("case: queue mix of %d requests, %d keys, direct from %d" % (
        len(reqs), sum(a.size for *_, a in reqs), direct_min), flush=True)
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


@pytest.mark.parametrize("direct_min", [0, 1 << 22], indirect=True)
def test_queue_largest_requests(direct_min):
    """The largest request size of the serving workload (2^24 keys) for each key
    type, together in one queue, through the ticks and by the single-array
    schedule; checked against an independent library sort (torch.sort; for
    float32 on the totalOrder integer codes)."""
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


@pytest.mark.parametrize("direct_min", [4096], indirect=True)
def test_queue_direct_keeps_caller_stats(direct_min):
    """Requests sorted by the single-array schedule inside the queue leave the
    statistics of the caller's own last tsqs_sort in place, and a tsqs_sort on
    the caller's stream after them sees its keys sorted."""
    import paper_1505_00558_amd as tsqs
    import torch
    mine = ti.device_family("uniform", 100003, "int32", seed=77)
    ref = torch.sort(mine).values
    tsqs.sort(mine)
    st = tsqs.get_stats()
    assert st["n"] == 100003
    q = tsqs.Queue(1 << 30)
    srcs = [ti.device_family(f, 50000 + 17 * j, "int64", seed=j) for j, f in enumerate(ti.FAMILIES)]
    tks = [q.submit(t) for t in srcs]
    _drain(q, tks)
    assert tsqs.get_stats()["n"] == 100003
    for t, tk in zip(srcs, tks):
        assert bool(torch.equal(q.result(tk), torch.sort(t).values))
        q.release(tk)
    again = ti.device_family("organ_pipe", 70001, "int32", seed=78)
    tsqs.sort(again)
    torch.cuda.synchronize()
    assert bool(torch.equal(again, torch.sort(ti.device_family("organ_pipe", 70001, "int32", seed=78)).values))
    assert bool(torch.equal(mine, ref))
    q.close()


@pytest.mark.parametrize("direct_min", [0], indirect=True)
def test_queue_cancel(oracle_mod, direct_min):
    """A queued request can be cancelled (never admitted; the rest of the queue
    completes as before); a running one cannot (TSQS_EAGAIN); a done one is
    released; a cancelled ticket is unknown afterwards.  Every request goes
    through the ticks (one level per step), so a request admitted by one step
    is still running after it: by the single-array schedule it could finish
    before the poll."""
    import paper_1505_00558_amd as tsqs
    q = tsqs.Queue(256 << 20)
    cap = q.info()["arena_bytes"]
    n = (cap // 4) // 3 - 64                            # three int32 requests fill the arena
    arrs = [ti.family(f, n, "int32", seed=60 + j) for j, f in
            enumerate(["uniform", "organ_pipe", "many_equals", "stair_steps", "uniform"])]
    srcs = [to_dev(a) for a in arrs]
    tks = [q.submit(t) for t in srcs]
    q.step()
    assert q.poll(tks[3]) == q.QUEUED and q.poll(tks[0]) == q.RUNNING
    assert q.cancel(tks[3])                             # queued: dropped
    with pytest.raises(tsqs.TsqsError):
        q.poll(tks[3])
    assert not q.cancel(tks[0])                         # running: not cancelled
    _drain(q, tks[:3])
    assert q.cancel(tks[2])                             # done: released
    for tk, a in zip(tks[:2], arrs[:2]):
        assert same_bits(from_dev(q.result(tk).clone(), np.int32), oracle_mod.sort(a))
        q.release(tk)
    _drain(q, [tks[4]])
    assert same_bits(from_dev(q.result(tks[4]).clone(), np.int32), oracle_mod.sort(arrs[4]))
    q.release(tks[4])
    info = q.info()
    assert info["queued"] == 0 and info["running"] == 0 and info["arena_used"] == 0
    q.close()


def test_workspace_cap_reports_enomem(oracle_mod):
    """TSQS_OPT_WORKSPACE_CAP: a sort that would grow the workspace past the cap
    returns TSQS_ENOMEM without touching the keys; under the cap, or with it
    lifted, the same sort succeeds."""
    import paper_1505_00558_amd as tsqs
    import torch
    tsqs.free_storage()                                 # start from an empty workspace
    k = ti.family("uniform", 1 << 22, "int32", seed=71)
    t = to_dev(k)
    tsqs.set_option(tsqs.OPT_WORKSPACE_CAP, 4 << 20)    # far below the 16 MiB scratch copy
    try:
        with pytest.raises(tsqs.TsqsError) as e:
            tsqs.sort(t)
        assert "-2" in str(e.value)
        torch.cuda.synchronize()
        assert same_bits(from_dev(t, np.int32), k)      # untouched
        tsqs.set_option(tsqs.OPT_WORKSPACE_CAP, 256 << 20)
        tsqs.sort(t)
        torch.cuda.synchronize()
        assert same_bits(from_dev(t, np.int32), oracle_mod.sort(k))
    finally:
        tsqs.set_option(tsqs.OPT_WORKSPACE_CAP, 0)
