"""Sketch, LSH and bottom-k calls captured into a HIP graph (torch.cuda.graph)
and replayed: a call enqueues only kernels (the device plan of heavy sets, the
size order's sort, the cursor reset and the persistent launch), so after one
eager call has sized the context's scratch it can be captured -- with the
default options, with splitting off, and with a split threshold that cuts many
sets into parts.  Every replay, with eager work and synchronizations in
between, must equal the eager result."""
import numpy as np
import pytest

import workloads as WL

pytestmark = pytest.mark.gpu

SEED = WL.HASH_SEED


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def batch(torch):
    from paper_2005_11547_amd import to_device
    rp, idx, w = WL.uneven_k1024(seed=81, n_sets=4000)
    return len(rp) - 1, to_device(rp, idx, w)


@pytest.mark.parametrize("split,order,L,K", [(None, 1, 64, 8), (0, 1, 16, 4), (0, 0, 16, 4), (0, 1, 64, 8),
                                             (512, 1, 16, 4)])
def test_captured_calls_replay_like_eager(torch, batch, split, order, L, K):
    # (64,8) LSH keeps its tables in registers, (16,4) in LDS; split None keeps the default
    from paper_2005_11547_amd import Context, dms
    n, d = batch
    c = Context(SEED)
    if split is not None:
        c.set_option(dms.OPT_SPLIT_NNZ, split)
    c.set_option(dms.OPT_ORDER, order)
    k, kb = 256, 64
    words = (k + 63) // 64
    u32 = torch.empty((n, k), dtype=torch.int32, device="cuda")
    bits = torch.empty((n, words), dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int8, device="cuda")
    keys = torch.empty((n, L), dtype=torch.int64, device="cuda")
    lst = torch.empty(n, dtype=torch.int8, device="cuda")
    bs = torch.empty((n, kb), dtype=torch.int64, device="cuda")
    br = torch.empty((n, kb), dtype=torch.float64, device="cuda")
    bst = torch.empty(n, dtype=torch.int8, device="cuda")
    outs = (u32, bits, st, keys, lst, bs, br, bst)

    def calls():
        c.dms_sketch_csr(n, *d, k, u32, bits, st)
        c.dms_lsh_keys(n, *d, L, K, keys, lst)
        c.dms_bottomk(n, *d, kb, bs, br, bst)

    print(f"[graph] eager split={split} order={order} L={L} K={K}", flush=True)
    calls()  # sizes the tables and scratch outside the capture
    torch.cuda.synchronize()
    ref = [t.cpu().clone() for t in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        calls()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in outs:
            t.fill_(-1 if t.dtype != torch.float64 else -1.0)
        calls()  # eager work between replays
        torch.cuda.synchronize()
        for t in outs:
            t.fill_(-1 if t.dtype != torch.float64 else -1.0)
        torch.cuda.synchronize()
        print(f"[graph] replay {rep}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a.cpu(), b), rep
    del g
    c.close()
