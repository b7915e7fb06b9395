"""GPU parity of the bottom-k sketch (dms_bottomk) and its estimate against the
oracle: id hashes and ranks bit-identical, statuses identical."""
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


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2005_11547_amd import Context
    c = Context(SEED)
    yield c
    c.close()


def _check(torch, ctx, rp, idx, w, k, label):
    from paper_2005_11547_amd import to_device
    print(f"[bottomk] {label}: {len(rp) - 1} sets, k={k}", flush=True)
    out = ctx.bottomk(*to_device(rp, idx, w), k)
    torch.cuda.synchronize()
    ref = O.bottomk_csr(rp, idx, w, k, SEED)
    assert np.array_equal(out["status"].cpu().numpy(), ref["status"]), label
    assert np.array_equal(out["s"].cpu().numpy().view(np.uint64), ref["s"]), label
    assert np.array_equal(out["rank"].cpu().numpy().view(np.uint64), ref["rank"].view(np.uint64)), label
    return out, ref


@pytest.mark.parametrize("k", [1, 7, 64, 256, 1024])
def test_batch_sample(torch, ctx, k):
    rp, idx, w = WL.batch_k256(seed=51, n_sets=600 if k < 1024 else 150)
    _check(torch, ctx, rp, idx, w, k, "batch")


def test_uneven_sample(torch, ctx):
    rp, idx, w = WL.uneven_k1024(seed=52, n_sets=200)
    _check(torch, ctx, rp, idx, w, 256, "uneven")


def test_edge_rows(torch, ctx):
    rows = [
        ([], []), ([5, 9], [0.0, 0.0]), ([1, 2, 3], [0.5, -1.0, 2.0]), ([1, 2], [np.nan, 1.0]),
        ([1, 2], [np.inf, 1.0]), ([7], [2.0 ** 800]), ([7], [2.0 ** -800]), ([7], [2.0 ** 700]),
        ([7], [2.0 ** -700]), ([123], [1.0]), ([1, 2, 3], [1e-300, 1.0, 0.0]),
        ([4, 4, 9], [0.3, 0.7, 1.0]), (list(range(200)), [1.0] * 200), ([2 ** 31 - 1, 0], [0.25, 0.75]),
        # ten ids each repeated 60 times: every dart arrives many times over
        ([i % 10 for i in range(600)], [0.5 + (i % 7) * 0.25 for i in range(600)]),
    ]
    rp, idx, w = WL.csr_from_rows(rows)
    for k in (1, 50, 300):
        _check(torch, ctx, rp, idx, w, k, f"edge rows k={k}")


@pytest.mark.parametrize("phi0", [2.0 ** -8, 8.0])
def test_schedules_that_force_retries_and_compactions(torch, phi0):
    # phi0 = 2^-8 needs many doublings; phi0 = 8 brings about 8k darts, several
    # times the buffer, so the buffer is compacted and cut during the pass
    from paper_2005_11547_amd import Context, dms
    c = Context(SEED)
    c.set_option(dms.OPT_BOTTOMK_PHI0, phi0)
    rp, idx, w = WL.batch_k256(seed=53, n_sets=120)
    rows = [(idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]]) for q in range(len(rp) - 1)]
    rows.append(([i % 10 for i in range(600)], [0.5 + (i % 7) * 0.25 for i in range(600)]))
    rp2, idx2, w2 = WL.csr_from_rows(rows)
    for k in (1, 64, 256):
        _check(torch, c, rp2, idx2, w2, k, f"phi0={phi0}")
    c.close()


def test_estimate_on_oracle_sketches(torch, ctx):
    rng = np.random.default_rng(29)
    rows = []
    for i in range(80):
        (xi, xw), (yi, yw) = WL.paired_sets(rng, 40, 1.0, (0.2, 0.5, 0.8)[i % 3])
        rows += [(xi, xw), (yi, yw)]
    rp, idx, w = WL.csr_from_rows(rows)
    for k in (1, 100, 256):
        ref = O.bottomk_csr(rp, idx, w, k, SEED)
        r, s = ref["rank"], ref["s"]
        est = O.jaccard_est_bottomk(r[0::2], s[0::2], r[1::2], s[1::2])
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        got = ctx.jaccard_bottomk(t(r[0::2]), t(s[0::2].view(np.int64)), t(r[1::2]), t(s[1::2].view(np.int64)))
        assert np.array_equal(got.cpu().numpy(), est), k


def test_full_size_sampled(torch, ctx):
    from paper_2005_11547_amd import to_device
    rp, idx, w = WL.batch_k256()
    n = len(rp) - 1
    out = ctx.bottomk(*to_device(rp, idx, w), 256)
    torch.cuda.synchronize()
    rows = np.linspace(0, n - 1, 120).astype(np.int64)
    sub = WL.csr_from_rows([(idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]]) for q in rows])
    ref = O.bottomk_csr(*sub, 256, SEED)
    sel = torch.from_numpy(rows).cuda()
    assert np.array_equal(out["s"][sel].cpu().numpy().view(np.uint64), ref["s"])
    assert np.array_equal(out["rank"][sel].cpu().numpy(), ref["rank"])
    assert (out["status"].cpu().numpy() == 0).all()


def test_invalid_arguments(torch, ctx):
    from paper_2005_11547_amd import DMSError, to_device
    d = to_device(*WL.csr_from_rows([([1], [1.0])]))
    for k in (0, 1025):
        with pytest.raises(DMSError):
            ctx.bottomk(*d, k)
