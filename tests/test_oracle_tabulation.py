"""Pins of the oracle's tabulation-hash variant (the paper's randomness source,
Section 4): the tables are the Mersenne Twister outputs after the six keys,
the enumeration with this hash equals rejection sampling of its dart stream,
and the minhash laws hold.  The hash values themselves have no external
reference: simple tabulation is its definition."""
import math

import numpy as np
import pytest

import workloads as WL
from jaccard import weighted_jaccard
from oracle import oracle as O
from test_oracle_bruteforce import IDS, NU, R_BOX, RHO, SEED, T, hitting, key, random_sets, stream

TAB = O.HASH_TAB


def tab_hash(seed):
    T8 = O.mt19937_64(seed, 6 + 2048)[6:]
    return lambda z: T8[z & 0xFF] ^ T8[256 + ((z >> 8) & 0xFF)] ^ T8[512 + ((z >> 16) & 0xFF)] ^ \
        T8[768 + ((z >> 24) & 0xFF)] ^ T8[1024 + ((z >> 32) & 0xFF)] ^ T8[1280 + ((z >> 40) & 0xFF)] ^ \
        T8[1536 + ((z >> 48) & 0xFF)] ^ T8[1792 + ((z >> 56) & 0xFF)]


def test_tables_follow_the_six_keys():
    mt = O.mt19937_64(SEED, 6 + 2048)
    tabs = O.tab_tables(SEED)
    assert len(tabs) == 2048 and list(tabs) == mt[6:]
    assert list(O.hash_keys(SEED).values()) == mt[:6]


@pytest.fixture(scope="module")
def tdarts():
    return stream(IDS, T, SEED, NU, RHO, mix=tab_hash(SEED))


@pytest.mark.parametrize("case", range(8))
def test_darthash_with_tabulation_equals_rejection_sampling(tdarts, case):
    x = random_sets(25)[case]
    S = sum(x.values())
    for phi in (0.5, 2.0):
        tau = phi / S
        if tau >= R_BOX:
            continue
        ids = np.array(sorted(x), dtype=np.int32)
        st, D, cnt = O.darthash(ids, np.array([x[i] for i in ids]), tau, T, SEED, hash=TAB)
        assert st == 0
        assert sorted(key(d) for d in D) == sorted(key(d) for d in hitting(tdarts, x, tau))


def test_minhash_with_tabulation_is_first_hitting_dart(tdarts):
    for x in random_sets(12):
        if sum(x.values()) < 0.3:
            continue
        ids = np.array(sorted(x), dtype=np.int32)
        st, s, r, _, _ = O.minhash_set(ids, np.array([x[i] for i in ids]), 2, SEED, t=T, hash=TAB)
        assert st == 0 and r.max() < R_BOX
        hit = hitting(tdarts, x)
        for b in range(2):
            first = next(d for d in hit if ((d["s"] >> 32) * 2) >> 32 == b)
            assert (int(s[b]), float(r[b])) == (first["s"], first["rank"])


def test_collision_law_and_schedule_independence():
    rng = np.random.default_rng(41)
    rows, js = [], []
    for i in range(90):
        (xi, xw), (yi, yw) = WL.paired_sets(rng, 40, 1.0, (0.2, 0.5, 0.8)[i % 3])
        rows += [(xi, xw), (yi, yw)]
        js.append(weighted_jaccard(xi, xw, yi, yw))
    js = np.array(js)
    rp, idx, w = WL.csr_from_rows(rows)
    k = 256
    out = O.sketch_csr(rp, idx, w, k, SEED, hash=TAB)
    agree = (out["u32"][0::2] == out["u32"][1::2]).mean(axis=1)
    se = math.sqrt((js * (1 - js)).sum() / k) / len(js)
    assert abs(agree.mean() - js.mean()) < 5 * se
    late = O.sketch_csr(rp[:21], idx[:rp[20]], w[:rp[20]], k, SEED, phi0=2.0 ** -5,
                        schedule=O.SCHED_DOUBLE, hash=TAB)
    assert np.array_equal(late["u32"], out["u32"][:20])
