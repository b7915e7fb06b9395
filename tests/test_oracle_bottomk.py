"""Pins of the oracle's bottom-k sketch (Section 3, bottom-k minhash) and its
Jaccard estimate against facts that do not come from that code."""
import math

import numpy as np
import pytest

import workloads as WL
from jaccard import weighted_jaccard
from oracle import oracle as O
from test_oracle_bruteforce import IDS, R_BOX, SEED, T, W_BOX, stream

HASH = WL.HASH_SEED


@pytest.fixture(scope="module")
def darts():
    return stream(IDS, T, SEED, 5, 4)


@pytest.mark.parametrize("trial", range(6))
def test_bottomk_equals_first_darts_of_the_brute_force_stream(darts, trial):
    # with t = k = T the bottom-k sketch is the T first darts hitting x
    rng = np.random.default_rng(trial)
    x = {i: float(rng.uniform(0.05, W_BOX)) for i in IDS if rng.random() < 0.8} or {IDS[0]: 1.0}
    hits = [d for d in darts if d["weight"] <= x.get(d["i"], 0.0)]
    assert len(hits) >= T and hits[T - 1]["rank"] < R_BOX  # the box holds the answer
    ids = np.array(sorted(x), dtype=np.int32)
    st, s, r, phi = O.bottomk_set(ids, np.array([x[i] for i in ids]), T, SEED)
    assert st == 0
    assert [(float(d["rank"]), int(d["s"])) for d in hits[:T]] == list(zip(r.tolist(), [int(v) for v in s]))


def _rows(seed, n):
    rp, idx, w = WL.batch_k256(seed=seed, n_sets=n)
    return [(idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]]) for q in range(n)]


@pytest.mark.parametrize("k", [1, 8, 64, 200])
def test_bottomk_is_lsh_with_one_table(k):
    # the (L,K) LSH oracle keeps the K smallest darts of each table; with L = 1
    # every dart lands in table 0 and t = L*K = k
    for ids, w in _rows(31 + k, 6):
        st, s, r, _ = O.bottomk_set(ids, w, k, HASH)
        st2, keys, s2, r2, _ = O.lsh_set(ids, w, 1, k, HASH)
        assert st == st2 == 0
        assert np.array_equal(s, s2[0]) and np.array_equal(r, r2[0])


def test_bottom_1_is_the_k1_minhash():
    # t(1) = 1, so the first dart is the single bucket's minimum
    for ids, w in _rows(41, 10):
        st, s, r, _ = O.bottomk_set(ids, w, 1, HASH)
        st2, s2, r2, _, _ = O.minhash_set(ids, w, 1, HASH)
        assert st == st2 == 0 and s[0] == s2[0] and r[0] == r2[0]


def test_schedule_independence():
    for ids, w in _rows(43, 5):
        ref = O.bottomk_set(ids, w, 100, HASH)
        for phi0, sched in ((2.0 ** -6, O.SCHED_DOUBLE), (5.0, O.SCHED_DOUBLE), (1.0, O.SCHED_PLUS_ONE)):
            got = O.bottomk_set(ids, w, 100, HASH, phi0=phi0, schedule=sched)
            assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])


def test_repeated_ids_act_as_the_max_weight():
    ids = np.array([5, 9, 5, 12, 9], dtype=np.int32)
    w = np.array([0.3, 2.0, 1.1, 0.7, 0.4])
    st, s, r, _ = O.bottomk_set(ids, w, 50, HASH)
    st2, s2, r2, _ = O.bottomk_set(np.array([5, 9, 12], np.int32), np.array([1.1, 2.0, 0.7]), 50, HASH)
    assert st == st2 == 0 and np.array_equal(s, s2) and np.array_equal(r, r2)
    assert len(set(zip(r.tolist(), s.tolist()))) == 50  # distinct darts


def test_sketch_is_sorted_and_rows_agree_with_single_sets():
    rp, idx, w = WL.batch_k256(seed=47, n_sets=8)
    out = O.bottomk_csr(rp, idx, w, 64, HASH)
    assert (np.diff(out["rank"], axis=1) >= 0).all()
    for q in range(8):
        st, s, r, _ = O.bottomk_set(idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]], 64, HASH)
        assert np.array_equal(out["s"][q], s)


def test_estimator_identity_and_disjoint_sets():
    rp, idx, w = WL.csr_from_rows([([1, 2, 3], [1.0, 2.0, 0.5]), ([1, 2, 3], [1.0, 2.0, 0.5]),
                                   ([7, 8], [1.0, 1.0])])
    out = O.bottomk_csr(rp, idx, w, 32, HASH)
    r, s = out["rank"], out["s"]
    assert O.jaccard_est_bottomk(r[:1], s[:1], r[1:2], s[1:2])[0] == 1.0
    assert O.jaccard_est_bottomk(r[:1], s[:1], r[2:3], s[2:3])[0] == 0.0


def test_estimator_is_unbiased_on_planted_pairs():
    rng = np.random.default_rng(19)
    rows, js = [], []
    for i in range(120):
        (xi, xw), (yi, yw) = WL.paired_sets(rng, 40, 1.0, (0.2, 0.5, 0.8)[i % 3])
        rows += [(xi, xw), (yi, yw)]
        js.append(weighted_jaccard(xi, xw, yi, yw))
    js = np.array(js)
    k = 128
    rp, idx, w = WL.csr_from_rows(rows)
    out = O.bottomk_csr(rp, idx, w, k, HASH)
    est = O.jaccard_est_bottomk(out["rank"][0::2], out["s"][0::2], out["rank"][1::2], out["s"][1::2])
    se = math.sqrt((js * (1 - js)).sum() / k) / len(js)
    assert abs(est.mean() - js.mean()) < 5 * se, (est.mean(), js.mean(), se)
