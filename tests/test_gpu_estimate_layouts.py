"""GPU parity of the memory-bound kernels across row widths and buffer
alignments: the estimators (u32, 1-bit, b-bit), the b-bit packing and the unary
map have a grouped-lane form for rows of a power of two of 16-byte vectors on
16-byte aligned buffers and a general form for everything else.  Both must
equal the oracle bit for bit."""
import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2005_11547_amd import Context
    c = Context(WL.HASH_SEED)
    yield c
    c.close()


def _dev(torch, a, offset=0):
    """Device copy of a 2-D array whose first element lies `offset` elements
    past a 256-byte aligned allocation (offset 1 breaks 16-byte alignment)."""
    a = np.ascontiguousarray(a)
    flat = torch.zeros(a.size + offset, dtype=torch.from_numpy(a[:0].copy()).dtype, device="cuda")
    flat[offset:] = torch.from_numpy(a.reshape(-1)).cuda()
    return flat[offset:].view(a.shape)


def _pairs(rng, n, k, share):
    a = rng.integers(0, 2 ** 32, size=(n, k), dtype=np.uint64).astype(np.uint32)
    b = a.copy()
    flip = rng.random((n, k)) >= share
    b[flip] = rng.integers(0, 2 ** 32, size=int(flip.sum()), dtype=np.uint64).astype(np.uint32)
    return a, b


@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("k", [4, 8, 12, 128, 512, 2048, 4096])
def test_u32_and_1bit_estimates(torch, ctx, k, offset):
    from paper_2005_11547_amd import dms
    rng = np.random.default_rng(k + offset)
    n = 131
    a, b = _pairs(rng, n, k, 0.6)
    print(f"[estimate] u32 k={k} offset={offset}", flush=True)
    got = ctx.jaccard(_dev(torch, a.view(np.int32), offset), _dev(torch, b.view(np.int32), offset), k, dms.FMT_U32)
    assert np.array_equal(got.cpu().numpy(), O.jaccard_est_u32(a, b)), k
    A, B = O.bbit_pack(a, 1), O.bbit_pack(b, 1)
    print(f"[estimate] 1-bit k={k} offset={offset}", flush=True)
    got = ctx.jaccard(_dev(torch, A.view(np.int64), offset), _dev(torch, B.view(np.int64), offset), k,
                      dms.FMT_1BIT)
    assert np.array_equal(got.cpu().numpy(), O.jaccard_est_1bit(A, B, k)), k


@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("k,bits", [(256, 8), (64, 1), (128, 2), (96, 4), (100, 16), (36, 32), (1024, 8),
                                    (256, 3), (2048, 1)])
def test_pack_estimate_unary(torch, ctx, k, bits, offset):
    rng = np.random.default_rng(7 * k + bits + offset)
    n = 77
    a, b = _pairs(rng, n, k, 0.5)
    print(f"[bbit] k={k} bits={bits} offset={offset}", flush=True)
    ga, gb = _dev(torch, a.view(np.int32), offset), _dev(torch, b.view(np.int32), offset)
    pa, pb = ctx.bbit_pack(ga, bits), ctx.bbit_pack(gb, bits)
    torch.cuda.synchronize()
    ra, rb = O.bbit_pack(a, bits), O.bbit_pack(b, bits)
    assert np.array_equal(pa.cpu().numpy().view(np.uint64), ra)
    assert np.array_equal(pb.cpu().numpy().view(np.uint64), rb)
    ea, eb = _dev(torch, ra.view(np.int64), offset), _dev(torch, rb.view(np.int64), offset)
    est = ctx.jaccard_bbit(ea, eb, k, bits).cpu().numpy()
    assert np.array_equal(est.view(np.uint64), O.jaccard_est_bbit(ra, rb, k, bits).view(np.uint64))
    if bits <= 16:
        idx, _ = ctx.unary_map(ga, bits)
        torch.cuda.synchronize()
        assert np.array_equal(idx.cpu().numpy(), O.unary_map(a, bits)[0])


def test_unary_map_many_rows(torch, ctx):
    # more 16-byte vectors than the grid has lanes (16384 blocks of 256), so
    # lanes advance their column across iterations and wrap past row ends
    rng = np.random.default_rng(5)
    for k, n in ((4, 4_500_000), (12, 1_600_000), (100, 200_000)):
        print(f"[unary] k={k} rows={n}", flush=True)
        a = rng.integers(0, 2 ** 32, size=(n, k), dtype=np.uint64).astype(np.uint32)
        idx, _ = ctx.unary_map(_dev(torch, a.view(np.int32)), 5)
        torch.cuda.synchronize()
        assert np.array_equal(idx.cpu().numpy(), O.unary_map(a, 5)[0]), k
