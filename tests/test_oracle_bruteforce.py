"""Pin of the oracle's DartHash enumeration against plain rejection sampling.

The paper defines the weighted minhash as the first dart of an infinite stream
that hits x (Section 1, and eq. 1).  Here the stream is generated without any
reference to a set: every area of every region of a bounded box of the
weight-rank space, for every element of a tiny universe, is visited with no
early exits; the darts are ordered by (rank, id hash).  The darts hitting x are
then found by scanning the stream.  The oracle, which walks Algorithm 1's loops
with their breaks, must return exactly the same darts and bucket minima.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

M64 = (1 << 64) - 1


def mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def stream(ids, t, seed, NU, RHO, mix=mix):
    """All darts with element in ids, nu <= NU, rho <= RHO, as a list of
    dicts sorted by (rank, s); `mix` is the hash function of every step."""
    K = O.hash_keys(seed)
    C = O.poisson_thresholds()
    u = 1.0 / t
    out = []
    for i in ids:
        for nu in range(NU + 1):
            Wn = float(2 ** nu - 1) / t
            for rho in range(RHO + 1):
                Rr = float(2 ** rho - 1)
                dnu = math.ldexp(u, nu - rho)
                drho = math.ldexp(1.0, rho - nu)
                g = mix(K["key_r"] ^ ((i << 32) | (nu << 16) | rho))
                for w in range(2 ** rho):
                    for r in range(2 ** nu):
                        a = mix(g ^ K["key_a"] ^ ((w << 32) | r))
                        X = sum(1 for c in C if a >= c)
                        for j in range(X):
                            U = (mix(a ^ K["key_u"] ^ j) >> 11) * 2.0 ** -53
                            V = (mix(a ^ K["key_v"] ^ j) >> 11) * 2.0 ** -53
                            out.append(dict(i=i, nu=nu, rho=rho, w=w, r=r, j=j,
                                            weight=Wn + (w + V) * dnu,
                                            rank=Rr + (r + U) * drho,
                                            s=mix(a ^ K["key_s"] ^ j)))
    out.sort(key=lambda d: (d["rank"], d["s"]))
    return out


T, NU, RHO, SEED = 10, 5, 4, 77
IDS = [3, 17, 1000, 123456]
W_BOX = float(2 ** (NU + 1) - 1) / T      # every dart of region NU+1 weighs at least this
R_BOX = float(2 ** (RHO + 1) - 1)         # every dart of region RHO+1 ranks at least this


@pytest.fixture(scope="module")
def darts():
    return stream(IDS, T, SEED, NU, RHO)


def hitting(darts, x, tau=None):
    return [d for d in darts if d["weight"] <= x.get(d["i"], 0.0) and (tau is None or d["rank"] <= tau)]


def key(d):
    return (int(d["i"]), int(d["nu"]), int(d["rho"]), int(d["w"]), int(d["r"]), int(d["j"]),
            float(d["rank"]), float(d["weight"]), int(d["s"]))


def oracle_darts(x, tau):
    ids = np.array(sorted(x), dtype=np.int32)
    w = np.array([x[i] for i in ids])
    st, D, cnt = O.darthash(ids, w, tau, T, SEED)
    assert st == 0
    return sorted(key(d) for d in D), cnt


def random_sets(n):
    rng = np.random.default_rng(11)
    out = []
    for _ in range(n):
        m = int(rng.integers(1, len(IDS) + 1))
        sub = rng.choice(IDS, size=m, replace=False)
        x = {int(i): float(rng.uniform(0.0, W_BOX * 0.999)) for i in sub}
        if rng.random() < 0.3:
            x[int(sub[0])] = float(rng.uniform(0, 0.05))
        out.append(x)
    return out


def test_stream_is_nonempty(darts):
    assert 3000 < len(darts) < 12000   # about 1953 areas per element, Poisson(1) each


@pytest.mark.parametrize("case", range(25))
def test_darthash_equals_rejection_sampling(darts, case):
    x = random_sets(25)[case]
    S = sum(x.values())
    for phi in (0.5, 1.0, 2.0, 5.0):
        tau = phi / S
        if tau >= R_BOX:
            continue
        got, cnt = oracle_darts(x, tau)
        want = sorted(key(d) for d in hitting(darts, x, tau))
        assert got == want
        assert cnt["accepted"] == len(want)


def test_boundaries_are_inclusive(darts):
    # A weight equal to a dart's weight, and a threshold equal to its rank,
    # both include the dart (Algorithm 1 accepts weight <= x_i and rank <= phi/||x||_1).
    d = next(d for d in darts if d["rank"] < 10.0 and d["nu"] >= 1 and d["weight"] < W_BOX)
    x = {d["i"]: d["weight"]}
    got, _ = oracle_darts(x, d["rank"])
    assert key(d) in got
    want = sorted(key(e) for e in hitting(darts, x, d["rank"]))
    assert got == want
    # a weight equal to a column boundary W + w * delta_nu, visited with its area
    for e in darts[:400]:
        if e["w"] > 0:
            b = float(2 ** e["nu"] - 1) / T + e["w"] * math.ldexp(1.0 / T, e["nu"] - e["rho"])
            x = {e["i"]: b}
            got, _ = oracle_darts(x, 20.0)
            assert got == sorted(key(f) for f in hitting(darts, x, 20.0))
            break


@pytest.mark.parametrize("k", [1, 2, 4])
def test_minhash_is_first_hitting_dart(darts, k):
    for x in random_sets(20):
        if sum(x.values()) < 0.3:
            continue
        ids = np.array(sorted(x), dtype=np.int32)
        w = np.array([x[i] for i in ids])
        st, s, r, phi, _ = O.minhash_set(ids, w, k, SEED, t=T)
        assert st == 0
        assert r.max() < R_BOX
        hit = hitting(darts, x)
        for b in range(k):
            first = next(d for d in hit if ((d["s"] >> 32) * k) >> 32 == b)
            assert (int(s[b]), float(r[b])) == (first["s"], first["rank"])


def test_lsh_is_first_K_darts_per_table(darts):
    L, K = 2, 2
    for x in random_sets(15):
        if sum(x.values()) < 0.5:
            continue
        ids = np.array(sorted(x), dtype=np.int32)
        w = np.array([x[i] for i in ids])
        # t = L*K = 4 differs from T, so use a dedicated stream
        st, keys, s, r, phi = O.lsh_set(ids, w, L, K, SEED)
        assert st == 0
        if r.max() >= R_BOX:
            continue
        box = stream(sorted(x), L * K, SEED, NU, RHO)
        hit = [d for d in box if d["weight"] <= x[d["i"]]]
        assert max(x.values()) < float(2 ** (NU + 1) - 1) / (L * K)
        for l in range(L):
            firsts = [d for d in hit if ((d["s"] >> 32) * L) >> 32 == l][:K]
            assert [f["s"] for f in firsts] == [int(v) for v in s[l]]
            h = mix(O.hash_keys(SEED)["key_l"] ^ l)
            for f in firsts:
                h = mix(h ^ f["s"])
            assert int(keys[l]) == h
