"""Pins for the oracle's AHP on the difference scale of section V-B's
pairwise rule (reading: a(i, j) = v_i - v_j when v_i > v_j, 1 when equal,
and 1 / (v_j - v_i) otherwise, so that a(j, i) = 1 / a(i, j)).  Hand cases
in exact fractions, a closed form, and invariants; CPU only."""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _diff_def(p, q):
    if p == q:
        return Fraction(1)
    return Fraction(p - q) if p > q else 1 / Fraction(q - p)


def _ahp_exact(v):
    """Local rank of one criterion from the definition: column sums, then
    the row means of the column-normalised matrix (Eqs. (9)-(10))."""
    n = len(v)
    A = [[_diff_def(v[i], v[j]) for j in range(n)] for i in range(n)]
    col = [sum(A[i][j] for i in range(n)) for j in range(n)]
    return [sum(A[i][j] / col[j] for j in range(n)) / n for i in range(n)]


def test_diff_rule_table(oracle_lib):
    for p in range(0, 40):
        for q in range(0, 40):
            assert O.diff(p, q) == float(_diff_def(p, q))
            assert O.diff(p, q) * O.diff(q, p) == pytest.approx(1.0, rel=1e-15)


def test_three_servers_by_hand(oracle_lib):
    """Values 0, 2, 5: columns sum to 8, 9/2 and 23/15, so the priorities are
    (1/8 + 1/9 + 3/23) / 3, (1/4 + 2/9 + 5/23) / 3 and
    (5/8 + 2/3 + 15/23) / 3."""
    want = [(Fraction(1, 8) + Fraction(1, 9) + Fraction(3, 23)) / 3,
            (Fraction(1, 4) + Fraction(2, 9) + Fraction(5, 23)) / 3,
            (Fraction(5, 8) + Fraction(2, 3) + Fraction(15, 23)) / 3]
    assert sum(want) == 1
    got = O.ahp(np.array([[0.0, 2.0, 5.0]]), [1.0], scale=O.DIFF)
    np.testing.assert_allclose(got, [float(x) for x in want], rtol=1e-15)
    # a cost criterion compares the other way round: the same as reversed values
    got_c = O.ahp(np.array([[0.0, 2.0, 5.0]]), [1.0], cost=[1], scale=O.DIFF)
    want_c = _ahp_exact([5, 3, 0])
    np.testing.assert_allclose(got_c, [float(x) for x in want_c], rtol=1e-15)


def test_two_servers_closed_form(oracle_lib):
    """Two servers d apart: the larger gets d / (d + 1), the smaller
    1 / (d + 1)."""
    for a, b in [(0, 1), (3, 10), (100, 40000), (7, 7)]:
        d = abs(a - b)
        got = O.ahp(np.array([[float(a), float(b)]]), [1.0], scale=O.DIFF)
        hi, lo = (d / (d + 1), 1 / (d + 1)) if d else (0.5, 0.5)
        want = [hi, lo] if a >= b else [lo, hi]
        np.testing.assert_allclose(got, want, rtol=1e-14)


def test_random_against_exact_and_invariants(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(25):
        C, N = int(rng.integers(1, 4)), int(rng.integers(2, 12))
        X = rng.integers(0, 60, size=(C, N))
        w = rng.uniform(0.1, 1.0, C)
        w /= w.sum()
        cost = rng.integers(0, 2, C).astype(np.int32)
        pg, p1, p2 = O.ahp(X.astype(float), w, cost, scale=O.DIFF, return_levels=True)
        for c in range(C):
            v = (-X[c]).tolist() if cost[c] else X[c].tolist()
            np.testing.assert_allclose(p2[c], [float(x) for x in _ahp_exact(v)], rtol=1e-13)
        np.testing.assert_allclose(p2.sum(axis=1), 1.0, rtol=1e-13)
        np.testing.assert_allclose(pg, p1 @ p2, rtol=1e-13)
        perm = rng.permutation(N)
        np.testing.assert_allclose(O.ahp(X[:, perm].astype(float), w, cost, scale=O.DIFF), pg[perm], rtol=1e-13)
    # a 0/1 criterion (f_u): differences of at most 1 compare as equal
    np.testing.assert_allclose(O.ahp(np.array([[0.0, 1.0, 1.0, 0.0]]), [1.0], scale=O.DIFF), 0.25, rtol=1e-15)
