"""Pins of the oracle's Hamming top-k search over 1-bit sketches (the serving
loop's near-neighbour scan): its popcount against Python's own bit count, the
search against a plain double loop on small inputs, and the cases whose answer
is known in closed form."""
import numpy as np
import pytest

from oracle import oracle as O


def test_popcount_matches_python_bit_count():
    rng = np.random.default_rng(1)
    v = rng.integers(0, 2 ** 63, size=2000, dtype=np.int64).view(np.uint64) ^ \
        (rng.integers(0, 2, size=2000, dtype=np.int64).view(np.uint64) << np.uint64(63))
    v = np.concatenate([v, np.array([0, 1, 2 ** 63, 2 ** 64 - 1], dtype=np.uint64)])
    got = O.popcount64(v)
    ref = [bin(int(x)).count("1") for x in v.tolist()]
    assert got.tolist() == ref


def _brute(db, q, topk):
    rows = []
    for qi in range(q.shape[0]):
        d = [(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(db[r].tolist(), q[qi].tolist())), r)
             for r in range(db.shape[0])]
        d.sort()
        rows.append(d[:topk])
    return rows


@pytest.mark.parametrize("words,n_db,n_q,topk", [(1, 40, 5, 3), (3, 25, 4, 25), (16, 60, 3, 10), (2, 7, 2, 10)])
def test_search_matches_a_plain_double_loop(words, n_db, n_q, topk):
    rng = np.random.default_rng(words * 100 + n_db)
    db = rng.integers(0, 2 ** 63, size=(n_db, words), dtype=np.int64).view(np.uint64)
    db[3] = db[1]                               # equal rows: the smaller id comes first
    q = rng.integers(0, 2 ** 63, size=(n_q, words), dtype=np.int64).view(np.uint64)
    ids, dist = O.hamming_topk(db, q, topk)
    ref = _brute(db, q, topk)
    for qi in range(n_q):
        m = min(topk, n_db)
        assert [int(x) for x in ids[qi, :m]] == [r for _, r in ref[qi]]
        assert [int(x) for x in dist[qi, :m]] == [d for d, _ in ref[qi]]


def test_known_answers():
    rng = np.random.default_rng(5)
    words = 4
    db = rng.integers(0, 2 ** 63, size=(30, words), dtype=np.int64).view(np.uint64)
    q = np.stack([db[7], ~db[12]])
    ids, dist = O.hamming_topk(db, q, 30)
    assert ids[0, 0] == 7 and dist[0, 0] == 0           # an exact copy is at distance 0
    assert ids[1, -1] == 12 and dist[1, -1] == 64 * words  # the complement is farthest
    assert (np.diff(dist, axis=1) >= 0).all()            # distances ascend
