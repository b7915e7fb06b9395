"""GPU parity of the b-bit fingerprint kernels (pack, estimate, unary map)
against the oracle, on seeded inputs and on oracle sketches.  Integers must be
identical and the f64 estimates bit-identical."""
import numpy as np
import pytest

import workloads as WL
from oracle import oracle as O

pytestmark = pytest.mark.gpu

SEED = WL.HASH_SEED
BITS = [1, 2, 3, 5, 8, 13, 16, 31, 32]
KS = [1, 63, 64, 100, 257, 1024]


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2005_11547_amd import Context
    c = Context(SEED)
    yield c
    c.close()


def _u32(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


@pytest.mark.parametrize("k", KS)
def test_pack_estimate_unary_random(torch, ctx, k):
    rng = np.random.default_rng(k)
    n = 97
    a = rng.integers(0, 2 ** 32, size=(n, k), dtype=np.uint64).astype(np.uint32)
    # pairs that agree on a random subset of positions
    b = a.copy()
    flip = rng.random((n, k)) < rng.random((n, 1))
    b[flip] = rng.integers(0, 2 ** 32, size=int(flip.sum()), dtype=np.uint64).astype(np.uint32)
    ga, gb = _u32(torch, a), _u32(torch, b)
    for bits in BITS:
        print(f"[bbit] k={k} bits={bits}", flush=True)
        pa, pb = ctx.bbit_pack(ga, bits), ctx.bbit_pack(gb, bits)
        torch.cuda.synchronize()
        ra, rb = O.bbit_pack(a, bits), O.bbit_pack(b, bits)
        assert np.array_equal(pa.cpu().numpy().view(np.uint64), ra), (k, bits)
        assert np.array_equal(pb.cpu().numpy().view(np.uint64), rb), (k, bits)
        est = ctx.jaccard_bbit(pa, pb, k, bits).cpu().numpy()
        ref = O.jaccard_est_bbit(ra, rb, k, bits)
        assert np.array_equal(est.view(np.uint64), ref.view(np.uint64)), (k, bits)
        if bits <= 16 and (k << bits) <= 2 ** 31:
            idx, scale = ctx.unary_map(ga, bits)
            torch.cuda.synchronize()
            ridx, rscale = O.unary_map(a, bits)
            assert scale == rscale
            assert np.array_equal(idx.cpu().numpy(), ridx), (k, bits)


def test_estimate_ignores_padding_bits(torch, ctx):
    # bits past k*bits in the last word do not count
    rng = np.random.default_rng(9)
    k, bits = 100, 3
    a = rng.integers(0, 2 ** 32, size=(8, k), dtype=np.uint64).astype(np.uint32)
    pa = O.bbit_pack(a, bits)
    pb = pa.copy()
    pb[:, -1] |= np.uint64(1) << np.uint64(63)  # bit 300 + ... is padding (k*bits = 300)
    ga = torch.from_numpy(pa.view(np.int64)).cuda()
    gb = torch.from_numpy(pb.view(np.int64)).cuda()
    est = ctx.jaccard_bbit(ga, gb, k, bits).cpu().numpy()
    assert (est == 1.0).all()
    for bits2 in (4, 32):  # aligned path
        pa2 = O.bbit_pack(a, bits2)
        pb2 = pa2.copy()
        if (k * bits2) % 64:
            pb2[:, -1] |= np.uint64(1) << np.uint64(63)
        est = ctx.jaccard_bbit(torch.from_numpy(pa2.view(np.int64)).cuda(),
                               torch.from_numpy(pb2.view(np.int64)).cuda(), k, bits2).cpu().numpy()
        assert (est == 1.0).all(), bits2


def test_on_oracle_sketches_of_planted_pairs(torch, ctx):
    rng = np.random.default_rng(23)
    rows = []
    for i in range(60):
        (xi, xw), (yi, yw) = WL.paired_sets(rng, 40, 1.0, (0.2, 0.5, 0.8)[i % 3])
        rows += [(xi, xw), (yi, yw)]
    rp, idx, w = WL.csr_from_rows(rows)
    ref = O.sketch_csr(rp, idx, w, 256, SEED)
    u = ref["u32"]
    g = _u32(torch, u)
    p1 = ctx.bbit_pack(g, 1).cpu().numpy().view(np.uint64)
    assert np.array_equal(p1, ref["bits"])  # 1-bit pack is the 1-bit sketch
    for bits in (2, 4, 8):
        p = ctx.bbit_pack(g, bits)
        est = ctx.jaccard_bbit(p[0::2].contiguous(), p[1::2].contiguous(), 256, bits).cpu().numpy()
        r = O.jaccard_est_bbit(O.bbit_pack(u[0::2], bits), O.bbit_pack(u[1::2], bits), 256, bits)
        assert np.array_equal(est, r), bits


def test_full_size_pack_sampled(torch, ctx):
    # a 1M x 256 batch in the launch shape the bench uses; sampled rows against the oracle
    n, k, bits = 1_000_000, 256, 8
    g = torch.randint(-2 ** 31, 2 ** 31, (n, k), dtype=torch.int32, device="cuda",
                      generator=torch.Generator(device="cuda").manual_seed(5))
    p = ctx.bbit_pack(g, bits)
    idx, _ = ctx.unary_map(g, bits)
    torch.cuda.synchronize()
    rows = np.random.default_rng(1).choice(n, 300, replace=False)
    a = g[rows].cpu().numpy().view(np.uint32)
    assert np.array_equal(p[rows].cpu().numpy().view(np.uint64), O.bbit_pack(a, bits))
    assert np.array_equal(idx[rows].cpu().numpy(), O.unary_map(a, bits)[0])


def test_invalid_arguments(torch, ctx):
    from paper_2005_11547_amd import DMSError
    g = _u32(torch, np.zeros((2, 64), np.uint32))
    for bits in (0, 33):
        with pytest.raises(DMSError):
            ctx.bbit_pack(g, bits)
    with pytest.raises(DMSError):
        ctx.unary_map(g, 17)
    with pytest.raises(DMSError):
        ctx.unary_map(_u32(torch, np.zeros((1, 40000), np.uint32)), 16)  # k * 2^16 > 2^31
