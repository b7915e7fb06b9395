"""GPU parity: the HIP path, called through the C ABI, against the oracle on the
same seeded inputs.  Integer outputs and ranks must be bit-identical."""
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


@pytest.fixture(scope="module", params=["plain", "fast"])
def ctx(request, torch):
    from paper_2005_11547_amd import Context, dms
    engine = dms.ENGINE_PLAIN if request.param == "plain" else dms.ENGINE_FAST
    c = Context(SEED, engine=engine)
    yield c
    c.close()


def _dev(torch, rp, idx, w):
    from paper_2005_11547_amd import to_device
    return to_device(np.ascontiguousarray(rp), np.ascontiguousarray(idx), np.ascontiguousarray(w))


def _check_sketch(torch, ctx, rp, idx, w, k, label):
    print(f"[parity] {label}: {len(rp) - 1} sets, k={k}", flush=True)
    out = ctx.sketch(*_dev(torch, rp, idx, w), k, bits=True, full=True)
    torch.cuda.synchronize()
    ref = O.sketch_csr(rp, idx, w, k, SEED, full=True)
    st = out["status"].cpu().numpy()
    assert np.array_equal(st, ref["status"]), label
    assert np.array_equal(out["u32"].cpu().numpy().view(np.uint32), ref["u32"]), label
    assert np.array_equal(out["bits"].cpu().numpy().view(np.uint64), ref["bits"]), label
    ok = ref["status"] == 0
    assert np.array_equal(out["s"].cpu().numpy().view(np.uint64)[ok], ref["s"][ok]), label
    assert np.array_equal(out["rank"].cpu().numpy().view(np.uint64)[ok], ref["rank"].view(np.uint64)[ok]), label


def test_plain_k64_config(torch, ctx):
    rp, idx, w, meta = WL.plain_k64()
    _check_sketch(torch, ctx, rp, idx, w, 64, "plain k=64, 1000 sets + 200 planted pairs")


def test_batch_k256_sample(torch, ctx):
    rp, idx, w = WL.batch_k256(n_sets=1500)
    _check_sketch(torch, ctx, rp, idx, w, 256, "batch k=256, 1500 sets")


def test_uneven_k1024_sample(torch, ctx):
    rp, idx, w = WL.uneven_k1024(n_sets=400)
    _check_sketch(torch, ctx, rp, idx, w, 1024, "uneven k=1024, 400 sets")


@pytest.mark.parametrize("k", [1, 2, 63, 65, 100, 4096])
def test_odd_k(torch, ctx, k):
    rp, idx, w = WL.batch_k256(seed=11, n_sets=40 if k < 4096 else 8)
    _check_sketch(torch, ctx, rp, idx, w, k, f"odd k={k}")


def test_edge_rows(torch, ctx):
    rows = [
        ([], []),                                   # empty row
        ([5, 9], [0.0, 0.0]),                       # all-zero weights
        ([1, 2, 3], [0.5, -1.0, 2.0]),              # negative weight
        ([1, 2], [np.nan, 1.0]),                    # NaN
        ([1, 2], [np.inf, 1.0]),                    # infinity
        ([7], [2.0 ** 800]),                        # beyond the supported range
        ([7], [2.0 ** -800]),                       # below it
        ([7], [2.0 ** 700]),                        # huge but inside
        ([7], [2.0 ** -700]),                       # tiny but inside
        ([7, 8], [2.0 ** 512, 3.0]),                # the paper's largest ||x||_1
        ([7, 8], [2.0 ** -513, 2.0 ** -513]),       # and its smallest
        ([123], [1.0]),                             # single element
        ([1, 2, 3], [1e-300, 1.0, 0.0]),            # denormal-scale element
        ([4, 4, 9], [0.3, 0.7, 1.0]),               # repeated id (acts as the max weight)
        (list(range(200)), [1.0] * 200),            # 0/1 weights
        ([2 ** 31 - 1, 0], [0.25, 0.75]),           # extreme ids
        ([3, 1], [1.5, 0.5]),                       # unsorted ids
    ]
    rp, idx, w = WL.csr_from_rows(rows)
    for k in (1, 64, 256):
        _check_sketch(torch, ctx, rp, idx, w, k, f"edge rows k={k}")


def test_retry_path_many_doublings(torch):
    # phi0 = 2^-10 forces about ten doublings; the output may not change (Theorem 1
    # is schedule-independent).
    from paper_2005_11547_amd import Context, dms
    rp, idx, w = WL.batch_k256(seed=12, n_sets=60)
    for engine in (dms.ENGINE_PLAIN, dms.ENGINE_FAST):
        c = Context(SEED, engine=engine)
        c.set_option(dms.OPT_PHI0, 2.0 ** -10)
        _check_sketch(torch, c, rp, idx, w, 128, f"phi0=2^-10 engine {engine}")
        c.close()


def test_lsh_keys(torch, ctx):
    rp, idx, w = WL.lsh_L64K8(n_sets=800)
    L, K = 64, 8
    print(f"[parity] lsh: {len(rp) - 1} sets, L={L} K={K}", flush=True)
    out = ctx.lsh(*_dev(torch, rp, idx, w), L, K)
    torch.cuda.synchronize()
    ref = O.lsh_csr(rp, idx, w, L, K, SEED)
    assert np.array_equal(out["status"].cpu().numpy(), ref["status"])
    assert np.array_equal(out["keys"].cpu().numpy().view(np.uint64), ref["keys"])


def test_lsh_edge_rows(torch, ctx):
    rows = [([], []), ([4, 4, 9], [0.3, 0.7, 1.0]), ([1], [3.0]), ([1, 2], [-1.0, 1.0]),
            (list(range(50)), list(np.linspace(0.1, 5.0, 50)))]
    rp, idx, w = WL.csr_from_rows(rows)
    for L, K in ((64, 8), (3, 5), (1, 1), (16, 16)):
        out = ctx.lsh(*_dev(torch, rp, idx, w), L, K)
        torch.cuda.synchronize()
        ref = O.lsh_csr(rp, idx, w, L, K, SEED)
        assert np.array_equal(out["status"].cpu().numpy(), ref["status"])
        assert np.array_equal(out["keys"].cpu().numpy().view(np.uint64), ref["keys"]), (L, K)


def test_lsh_more_than_64_tables(torch, ctx):
    # past 64 tables the insertion-election slots live after the table counts
    # instead of sharing the expansion marks
    rp, idx, w = WL.lsh_L64K8(seed=91, n_sets=300)
    rows = [(idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]]) for q in range(len(rp) - 1)]
    rows += [([], []), ([4, 4, 9], [0.3, 0.7, 1.0]), ([1], [3.0])]
    rp, idx, w = WL.csr_from_rows(rows)
    for L, K in ((64, 3), (65, 2), (128, 4), (200, 3), (1024, 1)):
        print(f"[parity] lsh L={L} K={K}", flush=True)
        out = ctx.lsh(*_dev(torch, rp, idx, w), L, K)
        torch.cuda.synchronize()
        ref = O.lsh_csr(rp, idx, w, L, K, SEED)
        assert np.array_equal(out["status"].cpu().numpy(), ref["status"]), (L, K)
        assert np.array_equal(out["keys"].cpu().numpy().view(np.uint64), ref["keys"]), (L, K)


def test_lsh_wide_tables(torch, ctx):
    # darts enter a table through a group of lanes as wide as K rounded up to a
    # power of two: up to one group of all 64 lanes at K = 64
    rp, idx, w = WL.lsh_L64K8(seed=92, n_sets=200)
    rows = [(idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]]) for q in range(len(rp) - 1)]
    rows += [([], []), ([4, 4, 9], [0.3, 0.7, 1.0]), ([1], [3.0]), ([7] * 3, [1.0, 2.0, 0.5])]
    rp, idx, w = WL.csr_from_rows(rows)
    # K = 8 with L <= 64 keeps each table in one lane's registers
    for L, K in ((2, 64), (3, 33), (4, 32), (8, 20), (16, 9), (24, 16), (1, 8), (37, 8), (64, 8), (65, 8)):
        print(f"[parity] lsh L={L} K={K}", flush=True)
        out = ctx.lsh(*_dev(torch, rp, idx, w), L, K)
        torch.cuda.synchronize()
        ref = O.lsh_csr(rp, idx, w, L, K, SEED)
        assert np.array_equal(out["status"].cpu().numpy(), ref["status"]), (L, K)
        assert np.array_equal(out["keys"].cpu().numpy().view(np.uint64), ref["keys"]), (L, K)


def test_jaccard_estimates(torch, ctx):
    from paper_2005_11547_amd import dms
    rng = np.random.default_rng(3)
    for k in (1, 64, 100, 256, 1024):
        n = 500
        a = rng.integers(0, 4, size=(n, k), dtype=np.uint32)
        b = rng.integers(0, 4, size=(n, k), dtype=np.uint32)
        got = ctx.jaccard(torch.from_numpy(a.view(np.int32)).cuda(), torch.from_numpy(b.view(np.int32)).cuda(),
                          k, dms.FMT_U32)
        assert np.array_equal(got.cpu().numpy(), O.jaccard_est_u32(a, b))
        words = (k + 63) // 64
        A = rng.integers(0, 2 ** 63, size=(n, words), dtype=np.int64).view(np.uint64)
        B = rng.integers(0, 2 ** 63, size=(n, words), dtype=np.int64).view(np.uint64)
        if k % 64:  # bits beyond k are zero in packed sketches
            mask = np.uint64((1 << (k % 64)) - 1)
            A[:, -1] &= mask
            B[:, -1] &= mask
        got = ctx.jaccard(torch.from_numpy(A.view(np.int64)).cuda(), torch.from_numpy(B.view(np.int64)).cuda(),
                          k, dms.FMT_1BIT)
        assert np.array_equal(got.cpu().numpy(), O.jaccard_est_1bit(A, B, k))


def test_invalid_arguments(torch, ctx):
    from paper_2005_11547_amd import DMSError
    rp, idx, w = _dev(torch, *WL.csr_from_rows([([1], [1.0])]))
    with pytest.raises(DMSError):
        ctx.sketch(rp, idx, w, 0)
    with pytest.raises(DMSError):
        ctx.sketch(rp, idx, w, 5000)
    with pytest.raises(DMSError):
        ctx.lsh(rp, idx, w, 0, 8)


@pytest.mark.parametrize("split", [1, 7, 64, 300])
def test_heavy_sets_cut_into_parts(torch, split):
    # Sets above the split threshold are shared by several wavefronts and merged
    # by the last one; the result may not depend on the cut.
    from paper_2005_11547_amd import Context, dms
    rp, idx, w = WL.batch_k256(seed=21, n_sets=30)
    extra = [([5, 9], [0.0, 0.0]), ([1, 2, 3], [0.5, -1.0, 2.0]), ([7], [2.0 ** 800]),
             ([4, 4, 9, 9, 11], [0.3, 0.7, 1.0, 0.2, 0.5]),
             (list(range(1000)), [0.0] * 500 + [1.0] * 500)]
    rows = [(idx[rp[r]:rp[r + 1]], w[rp[r]:rp[r + 1]]) for r in range(len(rp) - 1)] + extra
    rp2, idx2, w2 = WL.csr_from_rows(rows)
    for phi0 in (1.0, 2.0 ** -10):
        c = Context(SEED, engine=dms.ENGINE_FAST)
        c.set_option(dms.OPT_SPLIT_NNZ, split)
        c.set_option(dms.OPT_PHI0, phi0)
        for k in (1, 100, 256):
            _check_sketch(torch, c, rp2, idx2, w2, k, f"split={split} phi0={phi0} k={k}")
        c.close()


def test_autotune_picks_a_candidate_and_changes_no_output(torch):
    # the tuner times schedules on a prefix of the batch and sets them on the
    # context; the sketches must stay bit-exact (Theorem 1's output does not
    # depend on the schedule, and split parts merge exactly)
    from paper_2005_11547_amd import Context, dms
    rp, idx, w = WL.batch_k256(seed=61, n_sets=3000)
    c = Context(SEED)
    d = _dev(torch, rp, idx, w)
    phi0, split = c.autotune(*d, 256)
    assert phi0 in (1.0, 1.15, 1.3, 1.5, 1.8) and split in (0.0, 1024.0, 4096.0, 16384.0)
    assert c.get_option(dms.OPT_PHI0) == phi0 and c.get_option(dms.OPT_SPLIT_NNZ) == split
    assert c.get_option(dms.OPT_ORDER) in (0.0, 1.0)
    assert c.get_option(dms.OPT_WAVES) in (0.0, 1.0, 2.0, 3.0, 4.0)
    assert c.get_option(dms.OPT_TILE) in (0.0, 128.0)
    _check_sketch(torch, c, rp[:401], idx[:rp[400]], w[:rp[400]], 256, f"after autotune phi0={phi0} split={split}")
    c.close()


@pytest.mark.parametrize("k,tile,waves", [(256, 0, 1), (256, 0, 2), (256, 0, 4), (256, 128, 0), (256, 64, 4),
                                          (1024, 0, 1), (1024, 512, 0), (1024, 512, 2), (1024, 256, 4),
                                          (64, 0, 3)])
def test_block_shape_options(torch, k, tile, waves):
    # waves per block and buckets per tile change the launch, never an output
    from paper_2005_11547_amd import Context, dms
    rp, idx, w = WL.uneven_k1024(seed=62, n_sets=300)
    c = Context(SEED)
    c.set_option(dms.OPT_TILE, tile)
    c.set_option(dms.OPT_WAVES, waves)
    _check_sketch(torch, c, rp, idx, w, k, f"k={k} tile={tile} waves={waves}")
    c.close()


def test_block_shape_that_does_not_fit_is_refused(torch):
    from paper_2005_11547_amd import Context, dms
    rp, idx, w = WL.batch_k256(seed=63, n_sets=8)
    c = Context(SEED)
    c.set_option(dms.OPT_WAVES, 4)  # four waves of 1024 buckets each exceed 64 KiB
    with pytest.raises(dms.DMSError):
        c.sketch(*_dev(torch, rp, idx, w), 1024)
    with pytest.raises(dms.DMSError):
        c.set_option(dms.OPT_TILE, 100)  # not a multiple of 64
    c.close()


@pytest.mark.parametrize("k", [3392, 3456, 4000, 4096])
def test_tiled_buckets_fast_engine(torch, k):
    """k whose buckets do not fit next to the queues: the fast engine keeps them
    in tiles of whole words and repeats the schedule per tile; every output
    equals the oracle's (Table 1's k = 4096 rows), with the 1-bit words of
    every tile in place, on sets of mixed sizes and norms (retries per tile)."""
    from paper_2005_11547_amd import Context
    c = Context(SEED)
    rows = []
    rp, idx, w = WL.batch_k256(seed=12, n_sets=12)
    rows += [(idx[rp[i]:rp[i + 1]], w[rp[i]:rp[i + 1]]) for i in range(12)]
    for i, (l0, l1) in enumerate(((256, 1.0), (4096, 1.0), (1024, 2.0 ** 64), (1024, 2.0 ** -64), (1, 1.0))):
        r2, i2, w2 = WL.simplex_sets(70 + i, 1, l0, l1)
        rows.append((i2, w2))
    rows.append((np.array([3, 9], np.int32), np.array([0.0, 0.0])))  # empty
    rp, idx, w = WL.csr_from_rows(rows)
    _check_sketch(torch, c, rp, idx, w, k, f"tiled k={k}")
    c.close()
