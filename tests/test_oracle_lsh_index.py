"""Pins of the oracle's weight classes, exact weighted Jaccard and LSH index
(Section 3, approximate near neighbour search)."""
import math

import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

SEED = WL.HASH_SEED


@pytest.mark.parametrize("w,c", [([0.5, 0.5], 0), ([1.5], 0), ([2.0], 1), ([0.75, 0.25], 0),
                                 ([1.0, 1.0, 1.0, 1.0], 2), ([0.3, 0.0, 0.2], -1), ([2.0 ** -700], -700),
                                 ([2.0 ** 600, 2.0 ** 600], 601), ([1.9999999999999998], 0)])
def test_weight_class_closed_forms(w, c):
    assert O.weight_class(w) == c


def test_weight_class_invariant_and_exact_normalisation():
    rng = np.random.default_rng(2)
    for _ in range(200):
        w = rng.lognormal(rng.normal(0, 8), 1.0, size=int(rng.integers(1, 50)))
        c = O.weight_class(w)
        s = O.seq_sum(w)
        assert 2.0 ** c <= s < 2.0 ** (c + 1)
        wn = np.ldexp(w, -c)
        assert 1.0 <= O.seq_sum(wn) < 2.0
        assert np.array_equal(np.ldexp(wn, c), w)  # scaling by 2^-c lost nothing


def _j_union(ia, wa, ib, wb):
    ids = np.union1d(ia, ib)
    da, db = dict(zip(ia.tolist(), wa.tolist())), dict(zip(ib.tolist(), wb.tolist()))
    a = np.array([da.get(i, 0.0) for i in ids.tolist()])
    b = np.array([db.get(i, 0.0) for i in ids.tolist()])
    return np.minimum(a, b).sum() / np.maximum(a, b).sum()


def test_merge_jaccard():
    rng = np.random.default_rng(4)
    for _ in range(100):
        ia = np.sort(rng.choice(200, size=int(rng.integers(1, 40)), replace=False))
        ib = np.sort(rng.choice(200, size=int(rng.integers(1, 40)), replace=False))
        wa, wb = rng.random(len(ia)) + 0.01, rng.random(len(ib)) + 0.01
        assert abs(O.weighted_jaccard_merge(ia, wa, ib, wb) - _j_union(ia, wa, ib, wb)) < 1e-14
    ia = np.array([1, 5, 9])
    assert O.weighted_jaccard_merge(ia, [1.0, 2.0, 3.0], ia, [1.0, 2.0, 3.0]) == 1.0
    assert O.weighted_jaccard_merge(ia, [1.0, 2.0, 3.0], np.array([2, 6]), [1.0, 1.0]) == 0.0
    assert O.weighted_jaccard_merge(ia, [1.0, 2.0, 3.0], ia, [0.5, 1.0, 1.5]) == 0.5


def test_row_rules():
    assert O.row_ok_for_index([1, 4, 9], [1.0, 0.0, 2.0])
    assert not O.row_ok_for_index([1, 4, 4], [1.0, 1.0, 2.0])   # repeated id
    assert not O.row_ok_for_index([4, 1], [1.0, 1.0])           # not ascending
    assert not O.row_ok_for_index([1, 2], [0.0, 0.0])           # empty
    assert not O.row_ok_for_index([1, 2], [np.nan, 1.0])
    assert not O.row_ok_for_index([1], [2.0 ** 800])
    assert O.class_span(0.5) == 2 and O.class_span(0.9) == 2 and O.class_span(0.2) == 4


@pytest.fixture(scope="module")
def planted():
    """400 indexed sets, 40 queries that are near-duplicates (J = 0.9) of
    indexed sets at another scale, 20 unrelated queries."""
    rng = np.random.default_rng(8)
    rp, idx, w = WL.lsh_L64K8(seed=9, n_sets=400)
    rows = [(idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]] * 2.0 ** int(rng.integers(-6, 7))) for q in range(400)]
    data = WL.csr_from_rows(rows)
    queries, truth = [], []
    for q in rng.choice(400, size=40, replace=False).tolist():
        qi, qw = WL.near_duplicate(rng, *rows[q], J=0.9)
        queries.append((qi, qw))
        truth.append(q)
    qrp, qidx, qw = WL.lsh_L64K8(seed=10, n_sets=20)
    queries += [(qidx[qrp[q]:qrp[q + 1]], qw[qrp[q]:qrp[q + 1]]) for q in range(20)]
    index = O.lsh_index_build(*data, 16, 4, SEED)
    return data, index, queries, truth


def test_every_indexed_set_finds_itself(planted):
    (rp, idx, w), index, _, _ = planted
    for q in range(0, 400, 37):
        n, res = O.lsh_index_query(index, idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]], 0.5, 3)
        assert res[0] == (1.0, q)


def test_planted_neighbours_are_found_and_results_are_exact(planted):
    (rp, idx, w), index, queries, truth = planted
    for qn, (qi, qw) in enumerate(queries):
        n, res = O.lsh_index_query(index, qi, qw, 0.5, 10)
        brute = sorted(((O.weighted_jaccard_merge(qi, qw, idx[rp[x]:rp[x + 1]], w[rp[x]:rp[x + 1]]), x)
                        for x in range(400)), key=lambda t: (-t[0], t[1]))
        brute = [t for t in brute if t[0] >= 0.5][:10]
        if qn < len(truth):
            # J = 0.9 pairs collide in a table with probability 0.9^4, so in one of 16 tables almost surely
            assert res and res[0][1] == truth[qn] and abs(res[0][0] - 0.9) < 1e-12
            assert res == brute
        else:
            assert res == brute == []


def test_key_agreement_rate_is_j_to_the_k(planted):
    # the fraction of tables in which a pair's keys agree estimates J^K
    (rp, idx, w), index, queries, truth = planted
    agree = total = 0
    for qn, q in enumerate(truth):
        qi, qw = queries[qn]
        c = int(index["class"][q])
        st, keys, _, _, _ = O.lsh_set(qi, np.ldexp(qw, -c), 16, 4, SEED)
        agree += int((keys == index["keys"][q]).sum())
        total += 16
    p = 0.9 ** 4
    assert abs(agree / total - p) < 5 * math.sqrt(p * (1 - p) / total)
