"""Brute-force pin of the oracle: every sequence of length <= 8 over {0..n-1}.

The expected output is the plain definition of the result (the counting sort of
the input multiset), computed inside tests/native/exhaustive.c independently of
the oracle.  Profiles lower the size thresholds so that tiny inputs reach every
state of the paper's partition (SIII.B-F), both presorted handlers (SIII.I) and
the median-of-five tier (SIII.H, SV.C).
"""
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (nmax, ins_max, med3_below, medof3_small, handlers, reverse_tolerance, seed, keys_only)
PROFILES = [
    (8, 2, 1000, 1, 1, 3, 7, 0),     # median of 3 for every part >= 3, handlers on
    (7, 4, 5, 0, 1, 3, 99, 0),       # MEDOF3_SMALL off: median of 5 from 5 keys, jitter
    (7, 4, 5, 0, 1, 3, 123457, 0),   # another per-call random factor
    (7, 2, 1000, 1, 1, 0, 7, 0),     # zero reverse tolerance: handler fall-backs
    (7, 2, 1000, 1, 0, 3, 7, 0),     # handlers off: main path only
    (7, 2, 1000, 1, 1, 3, 7, 1),     # keys-only instantiation
]


@pytest.fixture(scope="module")
def exhaustive_bin(tmp_path_factory, oracle_mod):
    out = str(tmp_path_factory.mktemp("exh") / "exhaustive")
    subprocess.run(["gcc", "-O2", "-std=c11", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "tests", "native", "exhaustive.c"),
                    os.path.join(ROOT, "oracle", "tsqs_oracle.c"), "-o", out], check=True)
    return out


_RESULTS = {}


def _run(exhaustive_bin, prof):
    """One run per profile, shared by the tests of this module."""
    if prof not in _RESULTS:
        res = subprocess.run([exhaustive_bin] + [str(x) for x in prof], check=True,
                             capture_output=True, text=True, timeout=300)
        _RESULTS[prof] = (json.loads(res.stdout.strip().splitlines()[-1]), res.stderr)
    return _RESULTS[prof]


@pytest.mark.parametrize("prof", PROFILES, ids=lambda p: "n%d-ins%d-m3b%d-m3s%d-h%d-tol%d-s%d-k%d" % p)
def test_exhaustive(exhaustive_bin, prof):
    r, err = _run(exhaustive_bin, prof)
    expected_arrays = sum(n ** n for n in range(1, prof[0] + 1))
    assert r["arrays"] == expected_arrays
    for key in ("bad_keys", "bad_ids", "hole_errors", "revisit_errors", "internal_errors",
                "tar_over", "rc_bad", "post_errors"):
        assert r[key] == 0, (key, r[key], err[:2000])


def test_exhaustive_sum_is_known():
    # sum_{n=1..8} n^n, the count of arrays the full profile checks
    assert sum(n ** n for n in range(1, 9)) == 17650828


def test_exhaustive_reaches_every_state(exhaustive_bin):
    """The full profile reaches every state and handler outcome on n <= 8."""
    import oracle
    hits = _run(exhaustive_bin, PROFILES[0])[0]["hits"]
    hits2 = _run(exhaustive_bin, PROFILES[3])[0]["hits"]
    missing = [nm for i, nm in enumerate(oracle.EVENTS) if hits[i] + hits2[i] == 0]
    assert not missing, missing
