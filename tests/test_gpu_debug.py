"""GPU runs with the debug shadows on (TSQS_OPT_DEBUG): every store of every
partition pass lands on a slot no other key of the same part's pass took (the
atomic chunk reservations are disjoint) and that is not final yet; every slot
of the keys receives its final key exactly once (a band fill, a small part, a
part of one key), and all of them do.  Each case must sort exactly like the
oracle and report no shadow error, over every key type, keys alone and with
payloads, batches, both schedules, the depth-limit fallback, records and a
captured graph."""
import numpy as np
import pytest

import tsqs_inputs as ti
from gpu_util import CODES, from_dev, gpu_sort, gpu_sort_pairs, payload_valid, same_bits, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def debug_on():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1505_00558_amd as tsqs
    tsqs.load_library()
    tsqs.set_option(tsqs.OPT_DEBUG, 1)
    yield
    tsqs.set_option(tsqs.OPT_DEBUG, 0)
    tsqs.set_option(tsqs.OPT_SCHEDULE, tsqs.SCHEDULE_LEVELS)
    tsqs.set_option(tsqs.OPT_PIVOT_MODE, 0)


def _no_shadow_error():
    import paper_1505_00558_amd as tsqs
    rc, st = tsqs.last_call_status()
    assert rc == tsqs.OK and st["error_flags"] == 0, (rc, st["error_flags"])


@pytest.mark.parametrize("schedule", [0, 1], ids=["levels", "persistent"])
@pytest.mark.parametrize("dtype", list(ti.DTYPES))
def test_shadows_single_arrays(oracle_mod, dtype, schedule):
    import paper_1505_00558_amd as tsqs
    tsqs.set_option(tsqs.OPT_SCHEDULE, schedule)
    try:
        for fam, n in (("uniform", 300007), ("many_equals", 200003), ("organ_pipe", 70001),
                       ("sorted", 100000), ("reversed", 65537), ("stair_steps", 150001),
                       ("uniform", 8193), ("uniform", 3), ("uniform", 2)):
            print("case: shadows", dtype, schedule, fam, n, flush=True)
            k = ti.family(fam, n, dtype, seed=ti.seed_for(3, fam) + n)
            assert same_bits(gpu_sort(k), oracle_mod.sort(k)), (fam, n)
            _no_shadow_error()
            v = np.arange(n, dtype=np.uint32)
            gk, gv = gpu_sort_pairs(k, v)
            _no_shadow_error()
            assert same_bits(gk, oracle_mod.sort(k)) and payload_valid(k, gk, gv), (fam, n)
    finally:
        tsqs.set_option(tsqs.OPT_SCHEDULE, tsqs.SCHEDULE_LEVELS)


def test_shadows_large_and_fallback(oracle_mod):
    """2^24 keys (many levels, long bands), and exact-minimum pivots (the
    depth-limit fallback, grid-wide selection in the persistent kernel)."""
    import paper_1505_00558_amd as tsqs
    import torch
    n = (1 << 24) + 11
    t = ti.device_family("uniform", n, "int32", seed=5)
    ref = torch.sort(t).values
    tsqs.sort(t)
    torch.cuda.synchronize()
    _no_shadow_error()
    assert bool(torch.equal(t, ref))
    k = ti.family("uniform", (1 << 20) + 3, "int32", seed=6)
    tsqs.set_option(tsqs.OPT_PIVOT_MODE, 1)
    try:
        got = gpu_sort(k)
        _no_shadow_error()
        assert tsqs.get_stats()["fallback_parts"] > 0
    finally:
        tsqs.set_option(tsqs.OPT_PIVOT_MODE, 0)
    assert same_bits(got, oracle_mod.sort(k))


def test_shadows_batch_records_graph(oracle_mod):
    import paper_1505_00558_amd as tsqs
    import torch
    sizes = [1, 0, 5, 9000, 70001, 2, 300000]
    offs = np.cumsum([0] + sizes).astype(np.uint64)
    keys = np.concatenate([ti.family(ti.FAMILIES[j % 7], m, "uint64", seed=300 + j)
                           for j, m in enumerate(sizes)])
    t = to_dev(keys)
    v = torch.arange(keys.size, dtype=torch.int32, device="cuda:0")
    tsqs.sort_batch(t, offs, vals=v, dtype_code=CODES[keys.dtype])
    torch.cuda.synchronize()
    _no_shadow_error()
    got = from_dev(t, np.uint64)
    for a, b in zip(offs[:-1].tolist(), offs[1:].tolist()):
        assert same_bits(got[a:b], oracle_mod.sort(keys[a:b]))
    # records: 24-byte records moved with their int32 keys
    n = 50001
    rk = ti.family("many_equals", n, "int32", seed=8)
    rec = np.random.default_rng(8).integers(0, 256, size=(n, 24), dtype=np.uint8)
    rec[:, :4] = rk.view(np.uint8).reshape(n, 4)
    dk, dr = to_dev(rk), torch.from_numpy(rec.copy()).to("cuda:0")
    out = torch.empty_like(dr)
    tsqs.sort_records(dk, dr, out)
    torch.cuda.synchronize()
    _no_shadow_error()
    o = out.cpu().numpy().reshape(n, 24)
    assert same_bits(o[:, :4].copy().view(np.int32).reshape(-1), oracle_mod.sort(rk))
    # a graph created with the shadows on, replayed twice
    work = to_dev(keys)
    g = tsqs.Graph(work, offsets=offs, dtype_code=CODES[keys.dtype])
    try:
        for r in range(2):
            work.copy_(to_dev(keys))
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            assert g.stats()["error_flags"] == 0
            got = from_dev(work, np.uint64)
            for a, b in zip(offs[:-1].tolist(), offs[1:].tolist()):
                assert same_bits(got[a:b], oracle_mod.sort(keys[a:b]))
    finally:
        g.destroy()


@pytest.mark.parametrize("mode", [2, 3], ids=["planted_final", "planted_stamp"])
def test_shadow_checks_see_a_planted_entry(oracle_mod, mode):
    """The checks are not vacuous: with one shadow entry planted before the sort
    (slot 0 of the keys marked final, or slot 0 of the scratch copy marked as
    stored by the root's pass), the same correct sort reports TSQS_ERR_SHADOW;
    the keys are still sorted (the checks only observe)."""
    import paper_1505_00558_amd as tsqs
    k = ti.family("uniform", 100003, "int32", seed=12)
    tsqs.set_option(tsqs.OPT_DEBUG, mode)
    try:
        t = to_dev(k)
        tsqs.sort(t)
        rc, st = tsqs.last_call_status()
    finally:
        tsqs.set_option(tsqs.OPT_DEBUG, 1)
    assert rc == tsqs.EINTERNAL and st["error_flags"] & tsqs.ERR_SHADOW
    assert same_bits(from_dev(t, np.int32), oracle_mod.sort(k))
    # and with the plain mode again, no error
    assert same_bits(gpu_sort(k), oracle_mod.sort(k))
    _no_shadow_error()
