"""dms_sketch_csr_noalloc, the entry point for callers that cannot allocate:
its outputs equal dms_sketch_csr's bit for bit, on two calls in a row (the
second with a smaller batch, so stale scratch from the first would show), and
it refuses batches beyond its maximum and k whose tables are not prepared."""
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


def _batch(n_small, n_uneven, seed):
    rp, idx, w = WL.batch_k256(seed=seed, n_sets=n_small)
    rp2, idx2, w2 = WL.uneven_k1024(seed=seed, n_sets=n_uneven)
    rows = [(idx[rp[i]:rp[i + 1]], w[rp[i]:rp[i + 1]]) for i in range(n_small)]
    rows += [(idx2[rp2[i]:rp2[i + 1]], w2[rp2[i]:rp2[i + 1]]) for i in range(n_uneven)]
    return WL.csr_from_rows(rows)


def _outs(torch, n, k):
    return (torch.full((n, k), -1, dtype=torch.int32, device="cuda"),
            torch.full((n, (k + 63) // 64), -1, dtype=torch.int64, device="cuda"),
            torch.full((n,), -1, dtype=torch.int8, device="cuda"))


@pytest.mark.parametrize("engine,k", [("fast", 256), ("fast", 64), ("plain", 256), ("fast", 4096)])
def test_noalloc_equals_sketch_csr(torch, engine, k):
    from paper_2005_11547_amd import Context, dms, to_device
    c = Context(SEED, engine=dms.ENGINE_PLAIN if engine == "plain" else dms.ENGINE_FAST)
    c.dms_prepare(k)
    for call, (n_small, n_uneven, seed) in enumerate(((1500, 500, 41), (300, 100, 42))):
        if k == 4096:
            n_small, n_uneven = n_small // 10, n_uneven // 10
        rp, idx, w = _batch(n_small, n_uneven, seed)
        n = len(rp) - 1
        print(f"[no-alloc] engine={engine} k={k} call {call}: {n} sets", flush=True)
        d = to_device(rp, idx, w)
        a = _outs(torch, n, k)
        b = _outs(torch, n, k)
        c.dms_sketch_csr_noalloc(n, *d, k, *a)
        c.dms_sketch_csr(n, *d, k, *b)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y), (call, k)
        rows = np.linspace(0, n - 1, 40).astype(np.int64)
        sub = WL.csr_from_rows([(idx[rp[r]:rp[r + 1]], w[rp[r]:rp[r + 1]]) for r in rows])
        ref = O.sketch_csr(*sub, k, SEED)
        assert np.array_equal(a[0].cpu().numpy()[rows].view(np.uint32), ref["u32"])
        assert np.array_equal(a[2].cpu().numpy()[rows], ref["status"])
    c.close()


def test_noalloc_limits(torch):
    from paper_2005_11547_amd import Context, dms, to_device
    c = Context(SEED)
    rp, idx, w = WL.batch_k256(n_sets=8)
    d = to_device(rp, idx, w)
    out = _outs(torch, 8, 64)
    with pytest.raises(dms.DMSError):  # k = 64's tables are not made yet
        c.dms_sketch_csr_noalloc(8, *d, 64, *out)
    c.dms_prepare(64)
    with pytest.raises(dms.DMSError):  # beyond the maximum batch
        c.dms_sketch_csr_noalloc((1 << 20) + 1, *d, 64, *out)
    c.dms_sketch_csr_noalloc(8, *d, 64, *out)
    torch.cuda.synchronize()
    ref = O.sketch_csr(rp, idx, w, 64, SEED)
    assert np.array_equal(out[0].cpu().numpy().view(np.uint32), ref["u32"])
    c.close()
