"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers; it contains none of the sketching
arithmetic.  Every generator returns a CSR matrix ``(row_ptr int64[n+1],
idx int32[nnz], w float64[nnz])`` with distinct, ascending element ids inside
each row.  The shapes follow the synthetic data of the paper's experiments
(Section 4, "Synthetic data") and the five benchmark workloads:

* ``plain_k64``      1,000 sets, nnz ~ U{16..128}, ids from [0, 10^4),
                     weights Uniform(0,1], plus 200 planted pairs at
                     J in {0.1, 0.5, 0.9} (400 extra rows);
* ``batch_k256``     1,000,000 sets, nnz = clip(round(LogNormal(ln 256, 1)), 1, 4096),
                     ids from [0, 2^20), weights Exponential(1);
* ``uneven_k1024``   100,000 sets, nnz ~ Zipf(1.5) on [1, 65536], ids from [0, 2^24),
                     weights LogNormal(0,1) rescaled so that ||x||_1 = 10^U(-3,3);
* ``lsh_L64K8``      1,000,000 sets, nnz = max(1, round(LogNormal(ln 128, 0.8))),
                     ids from [0, 2^22), weights LogNormal(1, 0.7);
* ``serving``        nnz = round(exp(U(0, ln 4096))), ids from [0, 2^22),
                     weights LogNormal(0, 1).
"""
from __future__ import annotations

import numpy as np

HASH_SEED = 2005_11547


def _rng(seed: int):
    return np.random.Generator(np.random.PCG64(seed))


def _row_ptr(nnz: np.ndarray) -> np.ndarray:
    rp = np.zeros(len(nnz) + 1, dtype=np.int64)
    np.cumsum(nnz, out=rp[1:])
    return rp


def distinct_ids(rng, nnz: np.ndarray, d: int) -> np.ndarray:
    """For every row, nnz[r] distinct ids drawn uniformly from [0, d), ascending.

    Sorted uniform reals come from normalised exponential spacings and are
    floored; a row whose floors collide is redrawn, so each accepted row is a
    uniformly random subset of [0, d)."""
    nnz = np.asarray(nnz, dtype=np.int64)
    if np.any(nnz > d):
        raise ValueError("row longer than the universe")
    rp = _row_ptr(nnz)
    out = np.empty(int(rp[-1]), dtype=np.int64)
    # rows long enough that floors would often collide are drawn one by one
    dense = nnz * nnz > d // 8
    for r in np.nonzero(dense)[0]:
        out[rp[r]:rp[r + 1]] = np.sort(rng.choice(d, size=int(nnz[r]), replace=False))
    todo = np.nonzero(~dense)[0]
    while len(todo):
        # bounded chunks keep the running sums small and the temporaries modest
        cum = np.cumsum(nnz[todo])
        cut = int(np.searchsorted(cum, 1 << 22, side="right"))
        chunk, todo = todo[:max(cut, 1)], todo[max(cut, 1):]
        redo = _draw_rows(rng, chunk, nnz, rp, d, out)
        todo = np.concatenate([redo, todo])
    return out.astype(np.int32)


def _draw_rows(rng, rows_g, nnz, rp, d, out):
    cnt = nnz[rows_g]
    tot = int(cnt.sum())
    n = len(rows_g)
    seg = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt + 1, out=seg[1:])
    cs = np.cumsum(rng.standard_exponential(int(seg[-1])))
    base = np.zeros(n)
    base[1:] = cs[seg[1:-1] - 1]
    total = cs[seg[1:] - 1] - base
    rows = np.repeat(np.arange(n), cnt)
    start = np.cumsum(cnt) - cnt
    flat = seg[:-1][rows] + (np.arange(tot) - start[rows])
    u = (cs[flat] - base[rows]) / total[rows]
    ids = np.minimum(np.floor(u * d).astype(np.int64), d - 1)
    dup = np.zeros(n, dtype=bool)
    if tot > 1:
        same = (ids[1:] == ids[:-1]) & (rows[1:] == rows[:-1])
        dup[rows[1:][same]] = True
    good = np.nonzero(~dup)[0]
    if len(good):
        out[_gather_ranges(rp[rows_g[good]], cnt[good])] = ids[_gather_ranges(start[good], cnt[good])]
    return rows_g[dup]


def _gather_ranges(starts: np.ndarray, lens: np.ndarray) -> np.ndarray:
    lens = np.asarray(lens, dtype=np.int64)
    tot = int(lens.sum())
    off = np.cumsum(lens) - lens
    return np.repeat(np.asarray(starts, dtype=np.int64) - off, lens) + np.arange(tot)


# --------------------------------------------------------------------------
def plain_k64(seed: int = 1, n_sets: int = 1000, n_pairs: int = 200):
    """Uniform(0,1] weights; planted pairs share m = round(2nJ/(1+J)) ids with
    identical weights and have n - m private ids each, so E[J] is the target."""
    rng = _rng(seed)
    d = 10_000
    nnz = rng.integers(16, 129, size=n_sets)
    idx = distinct_ids(rng, nnz, d)
    w = 1.0 - rng.random(int(nnz.sum()))
    rows_rp = [_row_ptr(nnz)]
    targets = np.array([0.1] * (n_pairs - 2 * (n_pairs // 3)) + [0.5] * (n_pairs // 3) +
                       [0.9] * (n_pairs // 3))[:n_pairs]
    p_idx, p_w, p_nnz = [], [], []
    for J in targets:
        n = int(rng.integers(16, 129))
        m = int(round(2 * n * J / (1 + J)))
        ids = rng.choice(d, size=2 * n - m, replace=False)
        shared, px, py = ids[:m], ids[m:n], ids[n:]
        ws = 1.0 - rng.random(m)
        wx = 1.0 - rng.random(n - m)
        wy = 1.0 - rng.random(n - m)
        for own, wo in ((px, wx), (py, wy)):
            ii = np.concatenate([shared, own])
            ww = np.concatenate([ws, wo])
            o = np.argsort(ii)
            p_idx.append(ii[o])
            p_w.append(ww[o])
            p_nnz.append(len(ii))
    all_nnz = np.concatenate([nnz, np.array(p_nnz, dtype=np.int64)])
    idx = np.concatenate([idx] + [a.astype(np.int32) for a in p_idx])
    w = np.concatenate([w] + p_w)
    return _row_ptr(all_nnz), idx, w, dict(n_sets=n_sets, pair_rows=(n_sets, n_sets + 2 * n_pairs),
                                           pair_targets=targets)


def batch_k256(seed: int = 2, n_sets: int = 1_000_000):
    rng = _rng(seed)
    nnz = np.clip(np.round(rng.lognormal(np.log(256.0), 1.0, size=n_sets)), 1, 4096).astype(np.int64)
    idx = distinct_ids(rng, nnz, 1 << 20)
    w = rng.standard_exponential(int(nnz.sum()))
    while True:
        z = w == 0.0
        if not z.any():
            break
        w[z] = rng.standard_exponential(int(z.sum()))
    return _row_ptr(nnz), idx, w


def zipf_lengths(rng, n: int, alpha: float = 1.5, hi: int = 65536) -> np.ndarray:
    """Row lengths with P(n) proportional to n^-alpha on [1, hi], by inverse CDF."""
    v = np.arange(1, hi + 1, dtype=np.float64)
    cdf = np.cumsum(v ** -alpha)
    cdf /= cdf[-1]
    return (np.searchsorted(cdf, rng.random(n), side="right") + 1).clip(1, hi).astype(np.int64)


def uneven_k1024(seed: int = 3, n_sets: int = 100_000):
    rng = _rng(seed)
    nnz = zipf_lengths(rng, n_sets)
    idx = distinct_ids(rng, nnz, 1 << 24)
    w = rng.lognormal(0.0, 1.0, size=int(nnz.sum()))
    target = 10.0 ** rng.uniform(-3.0, 3.0, size=n_sets)
    rp = _row_ptr(nnz)
    rows = np.repeat(np.arange(n_sets), nnz)
    sums = np.add.reduceat(w, rp[:-1])
    w = w * (target / sums)[rows]
    return rp, idx, w


def lsh_L64K8(seed: int = 4, n_sets: int = 1_000_000):
    rng = _rng(seed)
    nnz = np.maximum(1, np.round(rng.lognormal(np.log(128.0), 0.8, size=n_sets))).astype(np.int64)
    idx = distinct_ids(rng, nnz, 1 << 22)
    w = rng.lognormal(1.0, 0.7, size=int(nnz.sum()))
    return _row_ptr(nnz), idx, w


def serving_sets(rng, n_sets: int):
    """Request-shaped sets for the serving loop."""
    nnz = np.round(np.exp(rng.uniform(0.0, np.log(4096.0), size=n_sets))).astype(np.int64)
    nnz = np.clip(nnz, 1, 4096)
    idx = distinct_ids(rng, nnz, 1 << 22)
    w = rng.lognormal(0.0, 1.0, size=int(nnz.sum()))
    return _row_ptr(nnz), idx, w


def near_duplicate(rng, idx, w, J: float = 0.9):
    """A set close to (idx, w): every weight kept, plus new ids carrying
    (1/J - 1) * ||x||_1 of weight, so that J(x, y) = ||x||_1/||y||_1 = J."""
    n_new = max(1, len(idx) // 10)
    extra = rng.choice(1 << 22, size=n_new + len(idx), replace=False)
    extra = np.setdiff1d(extra, idx)[:n_new]
    ew = rng.random(len(extra)) + 0.5
    ew *= (1.0 / J - 1.0) * float(np.sum(w)) / float(np.sum(ew))
    ii = np.concatenate([idx, extra]).astype(np.int32)
    ww = np.concatenate([w, ew])
    o = np.argsort(ii)
    return ii[o], ww[o]


def simplex_sets(seed: int, n_sets: int, l0: int, l1: float, d: int = 1 << 31):
    """The paper's generator (Section 4, "Synthetic data"): support of size l0 with
    random ids, weights uniform on the probability simplex scaled to ||x||_1 = l1."""
    rng = _rng(seed)
    nnz = np.full(n_sets, l0, dtype=np.int64)
    idx = distinct_ids(rng, nnz, d)
    e = rng.standard_exponential(n_sets * l0).reshape(n_sets, l0)
    w = (e / e.sum(axis=1, keepdims=True) * l1).reshape(-1)
    return _row_ptr(nnz), idx, w


def paired_sets(rng, n: int, l1: float, b: float, d: int = 1 << 30):
    """A pair (x, y) in the manner of the paper's estimation experiment: y keeps
    b * x_i on x's support and adds one new element of weight (1 - b) * ||x||_1,
    so ||y||_1 = ||x||_1 (the general reading of the construction)."""
    ids = rng.choice(d, size=n + 1, replace=False)
    e = rng.standard_exponential(n)
    x = e / e.sum() * l1
    xi = ids[:n]
    yi = ids
    yw = np.concatenate([b * x, [(1.0 - b) * l1]])
    ox, oy = np.argsort(xi), np.argsort(yi)
    return (xi[ox].astype(np.int32), x[ox]), (yi[oy].astype(np.int32), yw[oy])


def csr_from_rows(rows):
    """Stack a list of (idx, w) rows into CSR."""
    nnz = np.array([len(r[0]) for r in rows], dtype=np.int64)
    idx = np.concatenate([np.asarray(r[0], dtype=np.int32) for r in rows]) if rows else np.zeros(0, np.int32)
    w = np.concatenate([np.asarray(r[1], dtype=np.float64) for r in rows]) if rows else np.zeros(0)
    return _row_ptr(nnz), idx, w
