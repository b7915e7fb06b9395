"""Pins of the oracle against the laws the paper proves or states.

* Lemma 1: DartHash_t(x, phi) returns Poisson(phi t) darts, uniform over the
  part of weight-rank space under x (Section 2).
* Darts hashed to k buckets form k independent Poisson processes of rate
  phi t / k (Section 3).
* Eq. (1): Pr[h(x) = h(y)] = J(x, y); k J-hat ~ Bin(k, J) (Section 1.1);
  a 1-bit minhash collides with probability (1+J)/2; an (L,K) LSH key collides
  with probability J^K, independently across tables (Section 1.2, Section 3).
* The collision criterion of Section 1: x and y share a minhash exactly when
  the first dart hitting x or y lands in both.
* Theorem 1's output does not depend on the phi schedule.
* The estimation experiment of Section 4.1: estimates fall inside the 95%
  binomial interval about 95% of the time.
"""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as WL
from jaccard import weighted_jaccard
from oracle import oracle as O

SEED = WL.HASH_SEED


def _set(rng, n, d=1 << 20, scale=1.0):
    ids = np.sort(rng.choice(d, size=n, replace=False)).astype(np.int32)
    w = rng.standard_exponential(n) * scale
    return ids, w


def _minhash(ids, w, k, seed=SEED, **kw):
    st, s, r, phi, c = O.minhash_set(ids, w, k, seed, **kw)
    assert st == 0
    return s, r


# -------------------------------------------------------------------- Lemma 1
def test_lemma1_dart_count_is_poisson_phi_t():
    rng = np.random.default_rng(1)
    ids, w = _set(rng, 40)
    S = float(w.sum())
    t, phi = 331, 1.0
    counts = []
    for seed in range(400):
        st, D, c = O.darthash(ids, w, phi / S, t, 1000 + seed)
        assert st == 0
        counts.append(len(D))
    counts = np.array(counts)
    lam = phi * t
    assert abs(counts.mean() - lam) < 5 * math.sqrt(lam / len(counts))
    assert abs(counts.var(ddof=1) / lam - 1.0) < 5 * math.sqrt(2.0 / len(counts))


def test_lemma1_darts_are_uniform_under_x():
    rng = np.random.default_rng(2)
    ids, w = _set(rng, 30, scale=0.5)
    S = float(w.sum())
    tau = 2.0 / S
    wfrac, rfrac, elem = [], [], []
    xi = dict(zip(ids.tolist(), w.tolist()))
    for seed in range(60):
        st, D, c = O.darthash(ids, w, tau, 331, 5000 + seed)
        for d in D:
            wfrac.append(d["weight"] / xi[int(d["i"])])
            rfrac.append(d["rank"] / tau)
            elem.append(int(d["i"]))
    assert stats.kstest(wfrac, "uniform").pvalue > 1e-4
    assert stats.kstest(rfrac, "uniform").pvalue > 1e-4
    # darts per element proportional to x_i
    cnt = np.array([elem.count(int(i)) for i in ids], dtype=float)
    exp = w / w.sum() * len(elem)
    assert stats.chisquare(cnt, exp).pvalue > 1e-4


def test_bucket_occupancy_is_poisson():
    rng = np.random.default_rng(3)
    ids, w = _set(rng, 64)
    S = float(w.sum())
    k, t = 64, 331
    occ = []
    for seed in range(100):
        st, D, c = O.darthash(ids, w, 1.0 / S, t, 9000 + seed)
        b = ((D["s"] >> np.uint64(32)) * np.uint64(k)) >> np.uint64(32)
        occ.extend(np.bincount(b.astype(np.int64), minlength=k).tolist())
    occ = np.array(occ)
    lam = t / k
    top = 12
    obs = np.array([(occ == j).sum() for j in range(top)] + [(occ >= top).sum()], dtype=float)
    pm = stats.poisson.pmf(np.arange(top), lam)
    exp = np.concatenate([pm, [1 - pm.sum()]]) * len(occ)
    assert stats.chisquare(obs, exp).pvalue > 1e-4


# ------------------------------------------------------- Theorem 1 schedules
def test_output_independent_of_schedule_and_order():
    rng = np.random.default_rng(4)
    for case in range(12):
        ids, w = _set(rng, int(rng.integers(1, 200)), scale=10.0 ** rng.uniform(-3, 3))
        base = _minhash(ids, w, 64)
        for phi0, sched in [(2.0 ** -10, O.SCHED_DOUBLE), (2.0 ** -10, O.SCHED_PLUS_ONE),
                            (3.0, O.SCHED_DOUBLE), (17.0, O.SCHED_PLUS_ONE)]:
            s, r = _minhash(ids, w, 64, phi0=phi0, schedule=sched)
            assert np.array_equal(s, base[0]) and np.array_equal(r, base[1])
        p = rng.permutation(len(ids))  # another order, another rounding of ||x||_1
        s, r = _minhash(ids[p], w[p], 64)
        assert np.array_equal(s, base[0]) and np.array_equal(r, base[1])


# -------------------------------------------------- collision criterion (Sec 1)
def test_union_intersection_algebra():
    rng = np.random.default_rng(5)
    k = 128
    for case in range(10):
        n = int(rng.integers(5, 60))
        ids = np.sort(rng.choice(5000, size=n, replace=False)).astype(np.int32)
        x = rng.standard_exponential(n) * (rng.random(n) < 0.8)
        y = rng.standard_exponential(n) * (rng.random(n) < 0.8)
        if not (np.minimum(x, y) > 0).any():
            continue
        hx, hy = _minhash(ids, x, k), _minhash(ids, y, k)
        hu, hi = _minhash(ids, np.maximum(x, y), k), _minhash(ids, np.minimum(x, y), k)
        for j in range(k):
            px, py = (hx[0][j], hx[1][j]), (hy[0][j], hy[1][j])
            pu, pi = (hu[0][j], hu[1][j]), (hi[0][j], hi[1][j])
            assert pu in (px, py)
            assert (px == py) == (pu == pi)
            assert pu[1] <= min(px[1], py[1])      # union dominates: smaller rank
            assert pi[1] >= max(px[1], py[1])      # intersection is dominated


def test_special_cases():
    rng = np.random.default_rng(6)
    ids, w = _set(rng, 50)
    # identical sets
    a = _minhash(ids, w, 256)
    p = rng.permutation(len(ids))
    b = _minhash(ids[p], w[p], 256)
    assert np.array_equal(a[0], b[0])
    # disjoint supports never share a dart
    ids2 = np.setdiff1d(np.arange(2000, 2100), ids).astype(np.int32)[:50]
    c = _minhash(ids2, rng.standard_exponential(len(ids2)), 256)
    assert not np.intersect1d(a[0], c[0]).size
    # k = 1 uses t = 1
    assert O.t_of_k(1) == 1
    st, s, r, phi, cnt = O.minhash_set(ids, w, 1, SEED)
    assert st == 0 and len(s) == 1
    # statuses
    assert O.minhash_set(ids, np.zeros(len(ids)), 8, SEED)[0] == O.STATUS["empty"]
    assert O.minhash_set(ids[:0], w[:0], 8, SEED)[0] == O.STATUS["empty"]
    bad = w.copy(); bad[3] = -1.0
    assert O.minhash_set(ids, bad, 8, SEED)[0] == O.STATUS["invalid"]
    bad[3] = np.nan
    assert O.minhash_set(ids, bad, 8, SEED)[0] == O.STATUS["invalid"]
    bad[3] = np.inf
    assert O.minhash_set(ids, bad, 8, SEED)[0] == O.STATUS["invalid"]
    big = w.copy(); big[0] = 2.0 ** 800
    assert O.minhash_set(ids, big, 8, SEED)[0] == O.STATUS["range"]
    big[0] = 2.0 ** 700          # extreme but inside the supported domain
    assert O.minhash_set(ids, big, 8, SEED)[0] == O.STATUS["ok"]
    tiny = np.array([2.0 ** -800])
    assert O.minhash_set(ids[:1], tiny, 8, SEED)[0] == O.STATUS["range"]
    # zero weights are skipped: same sketch as without the element
    z = w.copy(); z[7] = 0.0
    keep = np.arange(len(ids)) != 7
    assert np.array_equal(_minhash(ids, z, 64)[0], _minhash(ids[keep], w[keep], 64)[0])


def _binom_z(matches, trials, probs):
    mean = float(np.sum(trials * probs))
    var = float(np.sum(trials * probs * (1 - probs)))
    return (float(np.sum(matches)) - mean) / math.sqrt(var)


def test_collision_rate_equals_weighted_jaccard_planted_pairs():
    rp, idx, w, meta = WL.plain_k64(n_sets=0, n_pairs=120)
    k = 64
    out = O.sketch_csr(rp, idx, w, k, SEED)
    assert (out["status"] == 0).all()
    m, J, bits_agree = [], [], []
    for p in range(len(rp) // 2):
        a, b = 2 * p, 2 * p + 1
        Jp = weighted_jaccard(idx[rp[a]:rp[a + 1]], w[rp[a]:rp[a + 1]],
                                 idx[rp[b]:rp[b + 1]], w[rp[b]:rp[b + 1]])
        J.append(Jp)
        m.append(int((out["u32"][a] == out["u32"][b]).sum()))
        bits_agree.append(k - int(O.popcount64(out["bits"][a] ^ out["bits"][b]).sum()))
    J, m, bits_agree = np.array(J), np.array(m), np.array(bits_agree)
    assert abs(_binom_z(m, k, J)) < 4.5
    assert abs(_binom_z(bits_agree, k, (1 + J) / 2)) < 4.5
    # no over-dispersion: per-pair standardised squares average about 1
    var = k * J * (1 - J)
    ok = var > 0
    disp = np.mean((m[ok] - k * J[ok]) ** 2 / var[ok])
    assert 0.6 < disp < 1.6
    # estimator wrapper
    est = O.jaccard_est_u32(out["u32"][0::2], out["u32"][1::2])
    assert np.allclose(est, m / k)


def test_special_jaccard_laws():
    rng = np.random.default_rng(7)
    k = 1024
    # one element, weights c < c': J = c/c'
    ids = np.array([42], dtype=np.int32)
    a = _minhash(ids, np.array([0.3]), k)
    b = _minhash(ids, np.array([0.75]), k)
    assert abs(_binom_z(np.sum(a[0] == b[0]), k, np.array(0.4))) < 4.5
    # x <= y: J = |x|_1 / |y|_1
    ids, y = _set(rng, 80)
    x = y * rng.uniform(0.2, 1.0, size=len(y))
    J = x.sum() / y.sum()
    assert abs(_binom_z(np.sum(_minhash(ids, x, k)[0] == _minhash(ids, y, k)[0]), k, np.array(J))) < 4.5
    # 0/1 weights: classic Jaccard |A n B| / |A u B|
    A = np.arange(0, 120, dtype=np.int32)
    B = np.arange(60, 200, dtype=np.int32)
    J = 60 / 200
    sa = _minhash(A, np.ones(len(A)), k)[0]
    sb = _minhash(B, np.ones(len(B)), k)[0]
    assert abs(_binom_z(np.sum(sa == sb), k, np.array(J))) < 4.5


def test_lsh_key_collision_is_J_to_the_K():
    rng = np.random.default_rng(8)
    L, K = 64, 4
    hits, probs = [], []
    for p in range(25):
        Jt = [0.5, 0.8, 0.95][p % 3]
        (xi, xw), (yi, yw) = WL.paired_sets(rng, int(rng.integers(20, 200)), 1.0, 2 * Jt / (1 + Jt))
        J = weighted_jaccard(xi, xw, yi, yw)
        st1, k1, *_ = O.lsh_set(xi, xw, L, K, SEED)
        st2, k2, *_ = O.lsh_set(yi, yw, L, K, SEED)
        assert st1 == 0 and st2 == 0
        hits.append(int((k1 == k2).sum()))
        probs.append(J ** K)
    assert abs(_binom_z(np.array(hits), L, np.array(probs))) < 4.5


def test_estimation_experiment_coverage():
    # Section 4.1: for k = 1..100 and J in {0.25, 0.5, 0.75}, a fresh pair and
    # fresh hash seeds; k J-hat must land in the central 95% binomial interval
    # about 95% of the time.
    rng = np.random.default_rng(9)
    inside = total = 0
    for k in range(1, 101, 3):
        for Jt in (0.25, 0.5, 0.75):
            (xi, xw), (yi, yw) = WL.paired_sets(rng, 256, 1.0, 2 * Jt / (1 + Jt))
            J = weighted_jaccard(xi, xw, yi, yw)
            seed = int(rng.integers(1, 2 ** 63))
            a = _minhash(xi, xw, k, seed=seed)[0]
            b = _minhash(yi, yw, k, seed=seed)[0]
            m = int(np.sum(a == b))
            lo, hi = stats.binom.ppf(0.025, k, J), stats.binom.ppf(0.975, k, J)
            inside += lo <= m <= hi
            total += 1
    assert inside / total > 0.9
