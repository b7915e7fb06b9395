"""GPU parity of the weight-class LSH index (dms_index_*) against the oracle:
classes, statuses, candidate counts, neighbour ids and exact Jaccard values."""
import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu

SEED = WL.HASH_SEED


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2005_11547_amd import Context
    c = Context(SEED)
    yield c
    c.close()


def _dev(torch, rp, idx, w):
    from paper_2005_11547_amd import to_device
    return to_device(np.ascontiguousarray(rp), np.ascontiguousarray(idx), np.ascontiguousarray(w))


@pytest.fixture(scope="module")
def data():
    """Indexed sets at scales 2^-6..2^6 plus rows the index must refuse, and
    queries: near-duplicates (J = 0.9, 0.7), exact copies, unrelated sets and
    bad rows."""
    rng = np.random.default_rng(12)
    rp, idx, w = WL.lsh_L64K8(seed=13, n_sets=500)
    rows = [(idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]] * 2.0 ** int(rng.integers(-6, 7))) for q in range(500)]
    rows += [([], []), ([3, 3, 5], [1.0, 1.0, 1.0]), ([9, 4], [1.0, 1.0]), ([1, 2], [np.nan, 1.0]),
             ([1, 2], [0.0, 0.0]), ([7], [2.0 ** 800]), ([2 ** 31 - 1, -2 ** 31], [1.0, 1.0])]
    queries = []
    for q in rng.choice(500, size=30, replace=False).tolist():
        queries.append(WL.near_duplicate(rng, *rows[q], J=0.9))
        queries.append(WL.near_duplicate(rng, *rows[q], J=0.7))
    queries += [rows[q] for q in (0, 17, 499)]
    qrp, qidx, qw = WL.lsh_L64K8(seed=14, n_sets=15)
    queries += [(qidx[qrp[q]:qrp[q + 1]], qw[qrp[q]:qrp[q + 1]]) for q in range(15)]
    queries += [([], []), ([4, 2], [1.0, 1.0]), ([5], [-1.0])]
    return WL.csr_from_rows(rows), WL.csr_from_rows(queries)


@pytest.mark.parametrize("L,K,j1", [(16, 4, 0.5), (8, 2, 0.3), (32, 6, 0.85), (1, 1, 0.2)])
def test_index_matches_oracle(torch, ctx, data, L, K, j1):
    from paper_2005_11547_amd import LshIndex
    (rp, idx, w), (qrp, qidx, qw) = data
    print(f"[index] L={L} K={K} j1={j1}", flush=True)
    ix = LshIndex(ctx, *_dev(torch, rp, idx, w), L, K)
    ref = O.lsh_index_build(rp, idx, w, L, K, SEED)
    cls, st = ix.sets()
    st = st.cpu().numpy()
    assert np.array_equal(st == 0, ref["ok"])
    assert np.array_equal(cls.cpu().numpy()[ref["ok"]], ref["class"][ref["ok"]])
    topn = 12
    out = ix.query(*_dev(torch, qrp, qidx, qw), j1, topn)
    torch.cuda.synchronize()
    ids, jv = out["ids"].cpu().numpy(), out["j"].cpu().numpy()
    cnt, cand, qst = out["count"].cpu().numpy(), out["candidates"].cpu().numpy(), out["status"].cpu().numpy()
    for q in range(len(qrp) - 1):
        qi, qwv = qidx[qrp[q]:qrp[q + 1]], qw[qrp[q]:qrp[q + 1]]
        n_c, res = O.lsh_index_query(ref, qi, qwv, j1, topn)
        assert (qst[q] == 0) == O.row_ok_for_index(qi, qwv), q
        assert cand[q] == n_c, (q, cand[q], n_c)
        assert cnt[q] == len(res), q
        assert [int(v) for v in ids[q, :len(res)]] == [x for _, x in res], q
        assert np.array_equal(jv[q, :len(res)], np.array([J for J, _ in res])), q
        assert (ids[q, len(res):] == -1).all()
    ix.close()


def test_status_codes(torch, ctx, data):
    from paper_2005_11547_amd import LshIndex
    (rp, idx, w), _ = data
    ix = LshIndex(ctx, *_dev(torch, rp, idx, w), 4, 2)
    _, st = ix.sets()
    assert st.cpu().numpy()[500:].tolist() == [1, 3, 3, 3, 1, 2, 0]
    ix.close()


def test_full_size_properties(torch, ctx):
    # 1M indexed sets (L = 64, K = 8); queries are near-duplicates of sampled
    # sets: each result is checked with the oracle's exact Jaccard, and the
    # planted neighbour must come first
    from paper_2005_11547_amd import LshIndex
    rp, idx, w = WL.lsh_L64K8()
    ix = LshIndex(ctx, *_dev(torch, rp, idx, w), 64, 8)
    rng = np.random.default_rng(21)
    picks = rng.choice(len(rp) - 1, size=200, replace=False)
    queries = [WL.near_duplicate(rng, idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]], J=0.9) for q in picks]
    out = ix.query(*_dev(torch, *WL.csr_from_rows(queries)), 0.5, 5)
    torch.cuda.synchronize()
    ids, jv, qst = out["ids"].cpu().numpy(), out["j"].cpu().numpy(), out["status"].cpu().numpy()
    assert (qst == 0).all()
    for n, q in enumerate(picks.tolist()):
        assert ids[n, 0] == q
        for r in range(5):
            x = int(ids[n, r])
            if x < 0:
                break
            J = O.weighted_jaccard_merge(*queries[n], idx[rp[x]:rp[x + 1]], w[rp[x]:rp[x + 1]])
            assert J == jv[n, r] and J >= 0.5
    ix.close()


def test_invalid_arguments(torch, ctx, data):
    from paper_2005_11547_amd import DMSError, LshIndex
    (rp, idx, w), (qrp, qidx, qw) = data
    with pytest.raises(DMSError):
        LshIndex(ctx, *_dev(torch, rp, idx, w), 0, 4)
    ix = LshIndex(ctx, *_dev(torch, rp, idx, w), 4, 2)
    for j1 in (0.0, 1.5):
        with pytest.raises(DMSError):
            ix.query(*_dev(torch, qrp, qidx, qw), j1, 5)
    ix.close()
