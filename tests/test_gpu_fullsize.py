"""Parity at the full workload sizes, in the launch configuration bench.py times:
the whole batch runs on the GPU; sampled rows (spread over the batch, plus the
first, the last and the largest ones) are recomputed one by one by the oracle
and must match bit for bit; properties that hold for every row are checked on
all of them."""
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


def _sample_rows(rp, n, rng, extra_heavy=3):
    sizes = np.diff(rp)
    rows = set(np.linspace(0, len(sizes) - 1, n).astype(np.int64).tolist())
    rows |= {0, len(sizes) - 1}
    rows |= set(np.argsort(sizes)[-extra_heavy:].tolist())
    rows |= set(rng.choice(len(sizes), size=n // 2, replace=False).tolist())
    return np.array(sorted(rows), dtype=np.int64)


def _sub(rp, idx, w, rows):
    sub_rp = np.concatenate([[0], np.cumsum(rp[rows + 1] - rp[rows])]).astype(np.int64)
    sub_idx = np.concatenate([idx[rp[r]:rp[r + 1]] for r in rows])
    sub_w = np.concatenate([w[rp[r]:rp[r + 1]] for r in rows])
    return sub_rp, sub_idx, sub_w


def _run_sketch(torch, rp, idx, w, k, label, n_sample, heavy=3):
    from paper_2005_11547_amd import Context, to_device
    print(f"[fullsize] {label}: {len(rp) - 1} sets, {rp[-1]} nnz, k={k}", flush=True)
    ctx = Context(SEED)
    out = ctx.sketch(*to_device(rp, idx, w), k, bits=True)
    torch.cuda.synchronize()
    u32 = out["u32"].cpu().numpy().view(np.uint32)
    bits = out["bits"].cpu().numpy().view(np.uint64)
    status = out["status"].cpu().numpy()
    ctx.close()
    # every row: status OK for these workloads (positive finite weights in range)
    assert (status == 0).all()
    assert not (u32 == 0xFFFFFFFF).all(axis=1).any()
    # the 1-bit sketch is bit 0 of the minhash, packed little-endian
    words = (k + 63) // 64
    lowbits = (u32 & 1).astype(np.uint64)
    pad = np.zeros((len(u32), words * 64 - k), np.uint64)
    packed = np.concatenate([lowbits, pad], axis=1).reshape(len(u32), words, 64)
    assert np.array_equal((packed << np.arange(64, dtype=np.uint64)).sum(axis=2, dtype=np.uint64), bits)
    rows = _sample_rows(rp, n_sample, np.random.default_rng(1), heavy)
    ref = O.sketch_csr(*_sub(rp, idx, w, rows), k, SEED)
    assert np.array_equal(u32[rows], ref["u32"]), label
    assert np.array_equal(bits[rows], ref["bits"]), label
    assert np.array_equal(status[rows], ref["status"]), label


def test_batch_k256_full(torch):
    rp, idx, w = WL.batch_k256()
    _run_sketch(torch, rp, idx, w, 256, "batch k=256", 300)


def test_uneven_k1024_full(torch):
    rp, idx, w = WL.uneven_k1024()
    _run_sketch(torch, rp, idx, w, 1024, "uneven k=1024", 150, heavy=2)


def test_lsh_L64K8_full(torch):
    from paper_2005_11547_amd import Context, to_device
    rp, idx, w = WL.lsh_L64K8()
    print(f"[fullsize] lsh: {len(rp) - 1} sets, {rp[-1]} nnz", flush=True)
    ctx = Context(SEED)
    out = ctx.lsh(*to_device(rp, idx, w), 64, 8)
    torch.cuda.synchronize()
    keys = out["keys"].cpu().numpy().view(np.uint64)
    status = out["status"].cpu().numpy()
    ctx.close()
    assert (status == 0).all() and (keys != 0).all()
    rows = _sample_rows(rp, 300, np.random.default_rng(2))
    ref = O.lsh_csr(*_sub(rp, idx, w, rows), 64, 8, SEED)
    assert np.array_equal(keys[rows], ref["keys"])
