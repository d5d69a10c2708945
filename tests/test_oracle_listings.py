"""Pins of the oracle against the paper's complete listings and its analysis.

* MedianOf3S (SIII.I): exact comparisons, copies, result and flag for the 13
  weak orderings of three keys, traced by hand (tests/golden/median3_counts.txt).
* Insertion sort (SIV): comparisons and copies equal a closed form in the
  input's inversion table that the listing implies: for element k with d_k
  strictly larger predecessors, 1 comparison if d_k = 0, otherwise
  d_k + [k - d_k > 0] comparisons and d_k + 2 copies.
* Sorted input performs no element copies other than loading the pivot
  (caption of Fig. 31 in Appendix B).
* Analysis mode (SV.A assumptions: random pivot, distinct keys, random order):
  mean comparisons (less the one exit2 comparison per stage) within 2% of eq.
  (3)'s 2(n+1)H_n - 4n, and mean virtual swaps (copies / 3, less the per-stage
  pivot / temp loads the model omits) within 15% of eq. (8).
"""
import os

import numpy as np
import pytest

import tsqs_inputs as ti

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _median3_rows():
    rows = []
    with open(os.path.join(GOLD, "median3_counts.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = [p.strip() for p in line.split("|")]
            rows.append(([int(x) for x in parts[0].split()], [int(x) for x in parts[1].split()],
                         int(parts[2]), int(parts[3]), int(parts[4])))
    return rows


def test_median3_golden_has_13_weak_orderings():
    rows = _median3_rows()
    assert len(rows) == 13
    pats = set()
    for inp, *_ in rows:
        ranks = tuple(sorted(set(inp)).index(x) for x in inp)
        pats.add(ranks)
    assert len(pats) == 13


@pytest.mark.parametrize("row", _median3_rows(), ids=lambda r: "".join(map(str, r[0])))
def test_median3_listing(oracle_mod, row):
    inp, out, flag, comps, copies = row
    f, res, piv, c = oracle_mod.median3(inp)
    assert res == out
    assert f == flag
    assert c.comparisons == comps
    assert c.copies - c.pivot_copies == copies
    assert c.pivot_copies == 1
    assert piv == out[1]


def _insertion_expected(a):
    comps = copies = 0
    for k in range(1, len(a)):
        d = sum(1 for j in range(k) if a[j] > a[k])
        if d == 0:
            comps += 1
        else:
            comps += d + (1 if k - d > 0 else 0)
            copies += d + 2
    return comps, copies


@pytest.mark.parametrize("seed", range(40))
def test_insertion_counts_closed_form(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 48))
    hi = int(rng.choice([3, n, 1000]))
    a = rng.integers(0, hi, size=n).astype(np.int32).tolist()
    out, c = oracle_mod.insertion(a)
    assert out == sorted(a)
    comps, copies = _insertion_expected(a)
    assert c.comparisons == comps
    assert c.copies == copies


@pytest.mark.parametrize("fam,n", [("sorted", 100000), ("sorted", 777), ("stair_steps", 200000),
                                   ("sorted", 31), ("stair_steps", 5001)])
def test_sorted_input_copies_only_pivots(oracle_mod, fam, n):
    k = ti.family(fam, n, "int32")
    out, c = oracle_mod.sort(k, counters=True)
    assert np.array_equal(out, k)
    assert c.copies == c.pivot_copies
    assert c.literal_swaps == 0


def _harmonic(n):
    return float(np.sum(1.0 / np.arange(1, n + 1)))


def test_analysis_mode_matches_eq3_and_eq8(oracle_mod):
    """SV.A under its own assumptions (random pivot, distinct keys, no cutoff).

    Classical quicksort compares each of the n'-1 non-pivot keys once per stage;
    the triple-state stage does the same plus the one comparison of temp with p
    in exit2 (SIII.F), so comparisons - stages must follow eq. (3)'s exact form
    2(n+1)H_n - 4n.  Eq. (5)-(8) count two copies per Hoare swap plus one for
    temp; the stage also copies the pivot into p, the mid element into the
    pivot's slot and the first element into temp (SIII.A), three copies per
    stage the model leaves out, so (copies - 3*stages)/3 is compared with eq.
    (8) (within 15%: the model is of Hoare swaps, not of this copy pattern)."""
    n, trials = 2000, 300
    p = oracle_mod.default_params(analysis_random_pivot=1, ins_max=2, handlers=0)
    comps, raw_vs, model_vs = [], [], []
    for t in range(trials):
        perm = np.random.default_rng(1000 + t).permutation(n).astype(np.int32)
        p.seed = 2 * t + 1
        out, c = oracle_mod.sort(perm, p, counters=True)
        assert np.array_equal(out, np.arange(n, dtype=np.int32))
        comps.append(c.comparisons - c.stages)
        raw_vs.append(c.copies / 3.0)
        model_vs.append((c.copies - 3.0 * c.stages) / 3.0)
    h = _harmonic(n)
    eq3 = 2 * (n + 1) * h - 4 * n
    eq8 = 2.0 / 9.0 * (n + 1) * h - (n + 1) / 6.0
    mc = float(np.mean(comps))
    assert abs(mc - eq3) / eq3 < 0.02, (mc, eq3)
    mv = float(np.mean(model_vs))
    assert abs(mv - eq8) / eq8 < 0.15, (mv, eq8)
    assert 1.0 < float(np.mean(raw_vs)) / eq8 < 1.5


def test_eq8_closed_form_satisfies_its_recurrence():
    # S_n = (1 + 1/n)(2/9 + S_{n-1}), S_2 = 1/2 (SV.A); closed form (8)
    def closed(n):
        return 2.0 / 9.0 * (n + 1) * _harmonic(n) - (n + 1) / 6.0
    s = 0.5
    assert abs(closed(2) - s) < 1e-12
    for n in range(3, 200):
        s = (1 + 1.0 / n) * (2.0 / 9.0 + s)
        assert abs(closed(n) - s) < 1e-9
