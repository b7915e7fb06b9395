"""Pins of the oracle's enumeration counts, which price the GPU's work in the
bench: the region count against the closed form of Algorithm 1's two outer
loops (nu while W[nu] <= x_i, rho while R[rho] <= tau), the accepted count
against the number of darts DartHash returns, the ordering of the counts, and
the per-schedule sums of the minhash, bottom-k and LSH loops against single
DartHash passes at phi = 1, 2, ... (the schedule of Theorem 1's proof)."""
import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

SEED = WL.HASH_SEED
FIELDS = ("regions", "areas", "generated", "rank_pass", "accepted")


def _rows(seed, n):
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n):
        m = int(rng.integers(1, 60))
        ids = np.sort(rng.choice(1 << 20, size=m, replace=False)).astype(np.int64)
        rows.append((ids, rng.exponential(1.0, size=m) * 2.0 ** float(rng.uniform(-6, 6))))
    return rows


def _pass(idx, w, phi, t):
    st, darts, c = O.darthash(idx, w, phi / O.seq_sum(w), t, SEED)
    assert st == 0
    return np.array([c[f] for f in FIELDS], np.int64), len(darts)


def test_region_count_is_the_loop_closed_form_and_counts_are_ordered():
    for ids, w in _rows(1, 12):
        t = O.t_of_k(64)
        W, R, _ = O.tables(t)
        S = O.seq_sum(w)
        for phi in (1.0, 2.0, 5.0):
            tau = phi / S
            c, n_darts = _pass(ids, w, phi, t)
            A = sum(sum(1 for v in W if v <= x) for x in w)
            B = sum(1 for r in R if r <= tau)
            assert c[0] == A * B
            assert c[4] == n_darts                        # every accepted dart is returned
            assert c[1] >= c[0] and c[2] >= c[3] >= c[4]  # one first area per region; filters shrink


@pytest.mark.parametrize("kind", ["minhash", "bottomk", "lsh"])
def test_schedule_sums_equal_single_passes(kind):
    rows = _rows(2, 10)
    rp, idx, w = WL.csr_from_rows(rows)
    if kind == "minhash":
        k, t = 64, O.t_of_k(64)
        r = O.sketch_csr(rp, idx, w, k, SEED, full=True)
        tot = np.stack([[c[f] for f in FIELDS] for c in r["counters"]])
        last = np.stack([[c[f] for f in FIELDS] for c in r["counters_last"]])
        phis = r["phi"]
    elif kind == "bottomk":
        k = t = 32
        r = O.bottomk_csr(rp, idx, w, k, SEED, counters=True)
        tot = np.stack([[c[f] for f in FIELDS] for c in r["counters"][:, 0]])
        last = np.stack([[c[f] for f in FIELDS] for c in r["counters"][:, 1]])
        phis = [O.bottomk_set(ids, ww, k, SEED)[3] for ids, ww in rows]
    else:
        L, K = 8, 4
        t = L * K
        r = O.lsh_csr(rp, idx, w, L, K, SEED, counters=True)
        tot = np.stack([[c[f] for f in FIELDS] for c in r["counters"][:, 0]])
        last = np.stack([[c[f] for f in FIELDS] for c in r["counters"][:, 1]])
        phis = [O.lsh_set(ids, ww, L, K, SEED)[4] for ids, ww in rows]
    assert (r["status"] == 0).all()
    for q, (ids, ww) in enumerate(rows):
        final = int(round(phis[q]))
        assert final >= 1 and float(final) == phis[q]   # phi = 1, 2, 3, ...
        passes = [_pass(ids, ww, float(p), t)[0] for p in range(1, final + 1)]
        assert np.array_equal(tot[q], np.sum(passes, axis=0)), (kind, q)
        assert np.array_equal(last[q], passes[-1]), (kind, q)


@pytest.mark.parametrize("kind", ["minhash", "bottomk", "lsh"])
@pytest.mark.parametrize("phi0", [1.0, 1.3])
def test_new_darts_of_a_doubling_schedule(kind, phi0):
    # Lemma 1: a pass at tau returns every dart of rank <= tau, so the bands
    # (tau_prev, tau] of the passes partition the darts of the last pass: the
    # new counts sum to the last pass's counts, and a pass's accepted new darts
    # are exactly its returned darts above the previous tau
    rows = _rows(3, 10)
    rp, idx, w = WL.csr_from_rows(rows)
    sched = O.SCHED_DOUBLE
    if kind == "minhash":
        k, t = 64, O.t_of_k(64)
        r = O.sketch_csr(rp, idx, w, k, SEED, phi0=phi0, schedule=sched, full=True)
        tot, last, phis = r["counters"], r["counters_last"], r["phi"]
    elif kind == "bottomk":
        k = t = 32
        r = O.bottomk_csr(rp, idx, w, k, SEED, phi0=phi0, schedule=sched, counters=True)
        tot, last = r["counters"][:, 0], r["counters"][:, 1]
        phis = [O.bottomk_set(ids, ww, k, SEED, phi0=phi0, schedule=sched)[3] for ids, ww in rows]
    else:
        L, K = 8, 4
        t = L * K
        r = O.lsh_csr(rp, idx, w, L, K, SEED, phi0=phi0, schedule=sched, counters=True)
        tot, last = r["counters"][:, 0], r["counters"][:, 1]
        phis = [O.lsh_set(ids, ww, L, K, SEED, phi0=phi0, schedule=sched)[4] for ids, ww in rows]
    assert (r["status"] == 0).all()
    for q, (ids, ww) in enumerate(rows):
        assert tot[q]["rank_new"] == last[q]["rank_pass"]
        assert tot[q]["accepted_new"] == last[q]["accepted"]
        S = O.seq_sum(ww)
        phi, tau_prev, acc_new = phi0, -1.0, 0
        while phi <= phis[q]:
            st, darts, c = O.darthash(ids, ww, phi / S, t, SEED)
            acc_new += int(np.count_nonzero(darts["rank"] > tau_prev))
            tau_prev = phi / S
            phi *= 2.0
        assert acc_new == tot[q]["accepted_new"]
        if phis[q] == phi0:  # one pass: every dart is new
            assert tot[q]["rank_new"] == tot[q]["rank_pass"] and tot[q]["accepted_new"] == tot[q]["accepted"]
