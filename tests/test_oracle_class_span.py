"""Pins of the weight-class span of the LSH index (Section 3, weight classes).

J(x, y) = sum min / sum max <= min(|x|, |y|) / max(|x|, |y|), so J >= j1 keeps
the norms within a factor 1/j1 and the classes floor(log2 |x|) within
ceil(log2(1/j1)) of each other.  These tests check that bound on random pairs,
plant neighbours exactly that many classes away (in both directions) with J
just above j1, and require the oracle's query to return them, equal to brute
force; a span one class narrower than the bound must miss some of them.
"""
import math

import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

SEED = WL.HASH_SEED


def reach(j1: float) -> int:
    """The farthest class distance a pair with J >= j1 can have."""
    return int(math.ceil(math.log2(1.0 / j1)))


def test_class_distance_bound_on_random_pairs():
    rng = np.random.default_rng(17)
    seen = 0
    for _ in range(3000):
        j1 = float(rng.choice([0.2, 0.3, 0.5]))
        ia = np.sort(rng.choice(60, size=int(rng.integers(1, 20)), replace=False))
        wa = rng.random(len(ia)) + 0.05
        # b: most of a's ids with perturbed weights, a few new ids, then a global scale
        keep = ia[rng.random(len(ia)) < 0.8]
        new = rng.choice(np.setdiff1d(np.arange(60), ia), size=int(rng.integers(0, 4)), replace=False)
        ib = np.sort(np.concatenate([keep, new]))
        wb = np.array([wa[np.searchsorted(ia, i)] if i in set(ia.tolist()) else rng.random() for i in ib.tolist()])
        wb = wb * rng.uniform(0.5, 2.0, size=len(ib)) * 2.0 ** rng.uniform(-2.5, 2.5)
        if not (O.row_ok_for_index(ia, wa) and O.row_ok_for_index(ib, wb)):
            continue
        if O.weighted_jaccard_merge(ia, wa, ib, wb) >= j1:
            seen += 1
            assert abs(O.weight_class(wa) - O.weight_class(wb)) <= reach(j1)
            assert abs(O.weight_class(wa) - O.weight_class(wb)) <= O.class_span(j1)
    assert seen > 100


def _planted(j1: float, rng, n_pairs: int = 8, n_noise: int = 16):
    """Pairs (small, large): large = small plus new ids, |large| / |small| just
    below 1/j1, so J = |small| / |large| is just above j1 and the classes are
    reach(j1) apart.  Returns the rows and the pairs' positions."""
    rows, pairs = [], []
    for _ in range(n_pairs):
        ids = rng.choice(1 << 20, size=60, replace=False)
        small_i = np.sort(ids[:30]).astype(np.int32)
        small_w = rng.random(30) + 0.5
        small_w *= 1.9 / O.seq_sum(small_w)  # class 0, near its top
        target = 1.0 / (j1 * 1.02)            # J = j1 * 1.02
        extra_i = ids[30:].astype(np.int32)
        extra_w = rng.random(30) + 0.5
        extra_w *= (target - 1.0) * 1.9 / O.seq_sum(extra_w)
        big_i = np.concatenate([small_i, extra_i])
        big_w = np.concatenate([small_w, extra_w])
        o = np.argsort(big_i)
        big_i, big_w = big_i[o], big_w[o]
        J = O.weighted_jaccard_merge(small_i, small_w, big_i, big_w)
        assert j1 <= J < j1 * 1.05
        assert O.weight_class(big_w) - O.weight_class(small_w) == reach(j1)
        pairs.append((len(rows), len(rows) + 1))
        rows += [(small_i, small_w), (big_i, big_w)]
    for _ in range(n_noise):
        ii = np.sort(rng.choice(1 << 20, size=30, replace=False)).astype(np.int32)
        rows.append((ii, (rng.random(30) + 0.5) * 2.0 ** rng.uniform(-2, 4)))
    return rows, pairs


def _brute(rows, qi, qw, j1, topn):
    res = [(O.weighted_jaccard_merge(qi, qw, *rows[x]), x) for x in range(len(rows))]
    res = sorted((t for t in res if t[0] >= j1), key=lambda t: (-t[0], t[1]))
    return res[:topn]


@pytest.mark.parametrize("j1", [0.2, 0.3])
def test_neighbours_at_the_farthest_class_are_found(j1):
    rng = np.random.default_rng(int(j1 * 100))
    rows, pairs = _planted(j1, rng)
    # K = 1: a table's keys agree with probability J, so one of 64 tables holds
    # a pair at J ~ j1 with probability 1 - (1 - J)^64 (above 1 - 1e-6)
    index = O.lsh_index_build(*WL.csr_from_rows(rows), 64, 1, SEED)
    for a, b in pairs:
        for q, other in ((a, b), (b, a)):  # the neighbour above, then below the query's class
            _, res = O.lsh_index_query(index, *rows[q], j1, 50)
            assert res == _brute(rows, *rows[q], j1, 50)
            assert other in [x for _, x in res]


@pytest.mark.parametrize("j1", [0.2, 0.3])
def test_a_narrower_span_misses_them(j1, monkeypatch):
    # the check above bites: searching one class fewer than the bound loses
    # the planted neighbours of the farthest class
    rng = np.random.default_rng(int(j1 * 100))
    rows, pairs = _planted(j1, rng)
    index = O.lsh_index_build(*WL.csr_from_rows(rows), 64, 1, SEED)
    monkeypatch.setattr(O, "class_span", lambda j: reach(j) - 1)
    missed = 0
    for a, b in pairs:
        _, res = O.lsh_index_query(index, *rows[a], j1, 50)
        missed += b not in [x for _, x in res]
    assert missed == len(pairs)
