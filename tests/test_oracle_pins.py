"""Pins of the oracle's pivot choice and of the states entered after SIII.C.

* Median of five (SIII.H; reading R4): for every permutation and every weak
  ordering of five keys, the samples end sorted in place, the pivot is the
  third smallest, and the flag is 1 exactly for non-decreasing input and -1
  exactly for strictly decreasing input.
* Ninther / fifteenther and the median-of-five tier inside the tiered choice
  (SIII.H, SV.C; reading R5): sample positions worked out by hand, with and
  without the per-call jitter (tests/golden/pivot_samples.txt).  Every other
  slot holds a distinct background value, so a sample taken from a wrong
  position, or a wrong slot written, changes the array.
* States 2L, 2R, 3L, 3R and exit2 (SIII.D-F): hand-traced runs from hand-built
  entry states (tests/golden/stage_traces.txt), compared slot for slot, with
  the final l and r, the comparison and copy counts and the tar[] fill.
* A mistake planted in the inputs of a trace is seen (the check is not
  vacuous).
"""
import itertools
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _weak_orderings(k):
    """Every weak ordering of k keys, as rank vectors (values 0..)."""
    seen = set()
    for t in itertools.product(range(k), repeat=k):
        vals = sorted(set(t))
        canon = tuple(vals.index(x) for x in t)
        seen.add(canon)
    return sorted(seen)


def test_weak_ordering_count():
    # ordered Bell (Fubini) numbers: 1, 3, 13, 75, 541
    assert [len(_weak_orderings(k)) for k in range(1, 6)] == [1, 3, 13, 75, 541]


@pytest.mark.parametrize("kind", ["permutations", "weak_orderings"])
def test_median5_all_orderings(oracle_mod, kind):
    cases = (list(itertools.permutations(range(5))) if kind == "permutations"
             else _weak_orderings(5))
    assert len(cases) == (120 if kind == "permutations" else 541)
    for t in cases:
        vals = [10 * x + 3 for x in t]
        flag, out, piv, c = oracle_mod.median5(vals)
        assert out == sorted(vals), t
        assert piv == sorted(vals)[2], t
        nondec = all(vals[i] <= vals[i + 1] for i in range(4))
        strict_dec = all(vals[i] > vals[i + 1] for i in range(4))
        assert flag == (1 if nondec else (-1 if strict_dec else 0)), t
        assert c.comparisons <= 10


def _pivot_cases():
    cases = []
    with open(os.path.join(GOLD, "pivot_samples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, pos, before, after, tail = [x.split() for x in line.split("|")]
            name, tier, n, seed, rnd = head
            cases.append(dict(name=name, tier=tier, n=int(n), seed=int(seed), random=int(rnd),
                              pos=[int(x) for x in pos], before=[int(x) for x in before],
                              after=[int(x) for x in after], p=int(tail[0]), flag=int(tail[1])))
    return cases


PIVOT_CASES = _pivot_cases()


@pytest.mark.parametrize("case", PIVOT_CASES, ids=[c["name"] for c in PIVOT_CASES])
def test_pivot_sample_positions(oracle_mod, case):
    n = case["n"]
    tiers = {"med5": dict(),
             "ninther": dict(),
             "fifteenther": dict(med5_below=800, ninther_below=900)}
    prm = oracle_mod.default_params(seed=case["seed"], random_samples=case["random"],
                                    **tiers[case["tier"]])
    arr = 100000 + np.arange(n)
    arr[case["pos"]] = case["before"]
    expected = arr.copy()
    expected[case["pos"]] = case["after"]
    flag, out, piv, _ = oracle_mod.choose_pivot(arr, prm)
    assert out == expected.tolist()
    assert piv == case["p"]
    assert out[(n - 1) >> 1] == case["p"]
    assert flag == case["flag"]


def _trace_cases():
    cases, cur = [], None
    with open(os.path.join(GOLD, "stage_traces.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = line.split()
            if w[0] == "case":
                cur = {"name": w[1]}
                cases.append(cur)
            elif w[0] == "entry":
                cur["entry"] = w[1]
                kv = dict(zip(w[2::2], w[3::2]))
                cur["open"] = kv.pop("open")
                holes = line.split("holes")[1].split()[:2]
                cur["holes"] = [int(x) for x in holes]
                for k in ("p", "temp", "a", "b", "l", "r", "m", "ml", "mr", "lc"):
                    cur[k] = int(line.split(" " + k + " ")[1].split()[0])
            elif w[0] in ("before", "after"):
                cur[w[0]] = [0 if x == "_" else int(x) for x in w[1:]]
            elif w[0] == "result":
                kv = dict(zip(w[1::2], w[2::2]))
                cur["result"] = {k: int(v) for k, v in kv.items()}
    return cases


TRACE_CASES = _trace_cases()


def _run_trace(oracle_mod, case, before=None):
    entry = {"STATE2": oracle_mod.ENTRY_STATE2, "STATE3": oracle_mod.ENTRY_STATE3,
             "EXIT2": oracle_mod.ENTRY_EXIT2}[case["entry"]]
    return oracle_mod.run_entry(
        before if before is not None else case["before"],
        a=case["a"], b=case["b"], l=case["l"], r=case["r"], m=case["m"], ml=case["ml"],
        mr=case["mr"], hole0=case["holes"][0], hole1=case["holes"][1], entry=entry,
        open_side=0 if case["open"] == "LO" else 1, lc=case["lc"], p=case["p"],
        temp=case["temp"])


def test_trace_file_covers_every_state():
    kinds = {(c["entry"], c["open"]) for c in TRACE_CASES}
    assert {("STATE2", "LO"), ("STATE2", "HI"), ("STATE3", "LO"), ("STATE3", "HI"),
            ("EXIT2", "LO")} <= kinds
    assert len(TRACE_CASES) >= 14


@pytest.mark.parametrize("case", TRACE_CASES, ids=[c["name"] for c in TRACE_CASES])
def test_stage_trace(oracle_mod, case):
    out, e, c = _run_trace(oracle_mod, case)
    res = case["result"]
    assert out == case["after"]
    assert (e.l, e.r) == (res["l"], res["r"])
    assert c.comparisons == res["comparisons"]
    assert c.copies == res["copies"]
    assert c.tar_peak == res["tar_peak"]
    assert c.hole_errors == 0 and c.internal_errors == 0
    # the result is the three-way partition of the keys it was given
    p = case["p"]
    assert all(x < p for x in out[case["a"]:e.l + 1])
    assert all(x == p for x in out[e.l + 1:e.r])
    assert all(x > p for x in out[e.r:case["b"] + 1])


def test_stage_trace_detects_planted_change(oracle_mod):
    """A key changed in an entry state changes the traced result."""
    case = next(c for c in TRACE_CASES if c["name"] == "3L-run-fits")
    before = list(case["before"])
    before[4] = 4                       # a key of the run now below p
    out, _, _ = _run_trace(oracle_mod, case, before)
    assert out != case["after"]
