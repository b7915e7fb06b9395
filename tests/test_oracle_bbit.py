"""Pins of the oracle's b-bit fingerprints, packing, estimator and unary map
(Section 1.1) against facts that do not come from the functions themselves."""
import math

import numpy as np
import pytest

import workloads as WL
from jaccard import weighted_jaccard
from oracle import oracle as O

SEED = WL.HASH_SEED


def _pack_bigint(values, b):
    """Brute force: the row's bit stream as one Python integer, cut into words."""
    k = len(values)
    stream = 0
    for j, v in enumerate(values):
        stream |= (int(v) & ((1 << b) - 1)) << (j * b)
    words = (k * b + 63) // 64
    return [(stream >> (64 * q)) & ((1 << 64) - 1) for q in range(words)]


@pytest.mark.parametrize("b", [1, 2, 3, 5, 7, 8, 13, 16, 31, 32])
@pytest.mark.parametrize("k", [1, 63, 64, 100, 257])
def test_pack_equals_bigint_stream(b, k):
    rng = np.random.default_rng(b * 1000 + k)
    v = rng.integers(0, 2 ** 32, size=(3, k), dtype=np.uint64).astype(np.uint32)
    got = O.bbit_pack(v, b)
    assert got.shape == (3, (k * b + 63) // 64)
    for r in range(3):
        assert [int(x) for x in got[r]] == _pack_bigint(v[r], b)
    assert np.array_equal(O.bbit_unpack(got, k, b), v.astype(np.uint64) & np.uint64((1 << b) - 1))


def test_pack_32_8_16_are_plain_reinterpretations():
    rng = np.random.default_rng(5)
    v = rng.integers(0, 2 ** 32, size=(4, 128), dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(O.bbit_pack(v, 32), v.astype("<u4").view("<u8"))
    assert np.array_equal(O.bbit_pack(v, 16), (v & 0xFFFF).astype("<u2").view("<u8"))
    assert np.array_equal(O.bbit_pack(v, 8), (v & 0xFF).astype("<u1").view("<u8"))


@pytest.fixture(scope="module")
def planted():
    """Oracle sketches (k = 256) of planted pairs with known weighted Jaccard."""
    rng = np.random.default_rng(17)
    rows, js = [], []
    for i in range(150):
        beta = (0.2, 0.5, 0.8)[i % 3]
        (xi, xw), (yi, yw) = WL.paired_sets(rng, 48, 1.0, beta)
        rows += [(xi, xw), (yi, yw)]
        js.append(weighted_jaccard(xi, xw, yi, yw))
    rp, idx, w = WL.csr_from_rows(rows)
    ref = O.sketch_csr(rp, idx, w, 256, SEED)
    assert (ref["status"] == 0).all()
    return ref, np.array(js)


def test_one_bit_pack_equals_the_oracle_bit_sketch(planted):
    ref, _ = planted
    assert np.array_equal(O.bbit_pack(ref["u32"], 1), ref["bits"])


def test_bbit_estimator_at_b1_is_the_one_bit_estimator(planted):
    ref, _ = planted
    u = ref["u32"]
    a, b = O.bbit_pack(u[0::2], 1), O.bbit_pack(u[1::2], 1)
    e1 = O.jaccard_est_1bit(ref["bits"][0::2], ref["bits"][1::2], 256)
    assert np.allclose(O.jaccard_est_bbit(a, b, 256, 1), e1, rtol=0, atol=1e-15)


@pytest.mark.parametrize("b", [1, 2, 4, 8])
def test_bbit_estimator_is_unbiased_on_planted_pairs(planted, b):
    # agreement probability is J + (1 - J) 2^-b per bucket; the corrected mean
    # over 150 pairs x 256 buckets must sit within 5 standard errors of mean J
    ref, js = planted
    u = ref["u32"]
    est = O.jaccard_est_bbit(O.bbit_pack(u[0::2], b), O.bbit_pack(u[1::2], b), 256, b)
    c = 2.0 ** -b
    p = js + (1 - js) * c
    se = math.sqrt((p * (1 - p)).sum() / 256) / len(js) / (1 - c)
    assert abs(est.mean() - js.mean()) < 5 * se, (est.mean(), js.mean(), se)
    # without the correction the estimate is visibly biased for small b
    raw = (O.bbit_unpack(O.bbit_pack(u[0::2], b), 256, b) ==
           O.bbit_unpack(O.bbit_pack(u[1::2], b), 256, b)).mean(axis=1)
    if b <= 2:
        assert abs(raw.mean() - js.mean()) > 10 * se


@pytest.mark.parametrize("b", [1, 3, 8])
def test_unary_map_inner_products(planted, b):
    ref, _ = planted
    u = ref["u32"][:20]
    k = u.shape[1]
    idx, val = O.unary_map(u, b)
    assert val == 1.0 / math.sqrt(k)
    # each coordinate lies in its own block of 2^b, so rows are strictly ascending
    j = np.arange(k)
    assert ((idx >> b) == j[None, :]).all()
    assert (np.diff(idx, axis=1) > 0).all()
    dense = np.zeros((u.shape[0], k << b))
    np.put_along_axis(dense, idx.astype(np.int64), val, axis=1)
    gram = dense @ dense.T
    fp = u.astype(np.uint64) & np.uint64((1 << b) - 1)
    agree = (fp[:, None, :] == fp[None, :, :]).sum(axis=2) / k
    assert np.allclose(np.diag(gram), 1.0)
    assert np.allclose(gram, agree, rtol=0, atol=1e-12)
