"""Oracle: the validate option (repeated element ids) only changes the status of
rows that list an id twice; every other row's outputs are unchanged."""
import numpy as np

import workloads as WL
from oracle import oracle as O

SEED = WL.HASH_SEED


def test_validate_marks_repeats_only():
    rp, idx, w = WL.batch_k256(n_sets=60)
    rows = []
    for i in range(60):
        ii, ww = idx[rp[i]:rp[i + 1]], w[rp[i]:rp[i + 1]]
        if i % 4 == 1:
            j = len(ii) // 2
            ii, ww = np.append(ii, ii[j]), np.append(ww, 0.5 * ww[j])  # same id, another weight
        rows.append((ii, ww))
    rp, idx, w = WL.csr_from_rows(rows)
    plain = O.sketch_csr(rp, idx, w, 64, SEED)
    val = O.sketch_csr(rp, idx, w, 64, SEED, validate=True)
    rep = np.arange(60) % 4 == 1
    assert (val["status"][rep] == 3).all()
    assert (val["u32"][rep] == 0xFFFFFFFF).all() and (val["bits"][rep] == 0).all()
    assert np.array_equal(val["u32"][~rep], plain["u32"][~rep])
    assert np.array_equal(val["status"][~rep], plain["status"][~rep])
    # without validation a repeat with a smaller weight is the row without it
    # (the same darts again, min is idempotent: reading of duplicate ids)
    base = O.sketch_csr(*WL.csr_from_rows([(idx[rp[i]:rp[i + 1] - 1], w[rp[i]:rp[i + 1] - 1]) if rep[i]
                                          else (idx[rp[i]:rp[i + 1]], w[rp[i]:rp[i + 1]]) for i in range(60)]),
                        64, SEED)
    assert np.array_equal(plain["u32"], base["u32"])
    lv = O.lsh_csr(rp, idx, w, 8, 4, SEED, validate=True)
    bv = O.bottomk_csr(rp, idx, w, 32, SEED, validate=True)
    assert (lv["status"][rep] == 3).all() and (lv["keys"][rep] == 0).all()
    assert (bv["status"][rep] == 3).all()
    assert (lv["status"][~rep] == 0).all() and (bv["status"][~rep] == 0).all()


def test_repeated_id_as_uint32():
    """Ids are compared as uint32: -1 and 2^32 - 1 are the same id."""
    idx = np.array([5, -1, 7, -1], dtype=np.int32)
    w = np.ones(4)
    r = O.sketch_csr(np.array([0, 4]), idx, w, 16, SEED, validate=True)
    assert r["status"][0] == 3
    r = O.sketch_csr(np.array([0, 3]), idx[:3], w[:3], 16, SEED, validate=True)
    assert r["status"][0] == 0
