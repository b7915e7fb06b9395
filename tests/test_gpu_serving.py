"""GPU tests of the search kernel and the continuous-batching serving loop,
through the C ABI, against the oracle (all expected values come from oracle/)."""
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


def _bits(rng, n, words):
    return rng.integers(0, 2 ** 63, size=(n, words), dtype=np.int64).view(np.uint64) ^ \
        (rng.integers(0, 2, size=(n, words), dtype=np.int64).view(np.uint64) << np.uint64(63))


@pytest.mark.parametrize("words,n_db,n_q,topk", [(16, 50_000, 40, 10), (1, 3000, 17, 10),
                                                  (4, 20_000, 33, 64), (16, 5, 3, 10),
                                                  (16, 1, 1, 1), (7, 9000, 16, 5),
                                                  # the full grid of row slices: 512 partial
                                                  # top-k lists per query to merge
                                                  (16, 600_000, 4, 10), (16, 600_000, 3, 16),
                                                  (16, 600_000, 2, 17)])
def test_hamming_topk_matches_brute_force(torch, ctx, words, n_db, n_q, topk):
    print(f"[search] words={words} n_db={n_db} n_q={n_q} topk={topk}", flush=True)
    rng = np.random.default_rng(words * 1000 + n_db)
    db = _bits(rng, n_db, words)
    if n_db > 100:
        db[50:70] = db[10]       # exact duplicates: ties broken by the smaller row id
        db[80] = ~db[10]
    q = _bits(rng, n_q, words)
    q[0] = db[min(10, n_db - 1)]  # a query equal to a database row
    if n_q > 2 and n_db > 3:
        q[1] = db[3] ^ np.uint64(1)
    ids, dist = ctx.hamming_topk(torch.from_numpy(db.view(np.int64)).cuda(),
                                 torch.from_numpy(q.view(np.int64)).cuda(), topk)
    torch.cuda.synchronize()
    ref_ids, ref_dist = O.hamming_topk(db, q, topk)
    got_ids, got_dist = ids.cpu().numpy(), dist.cpu().numpy()
    m = min(topk, n_db)
    assert np.array_equal(got_ids[:, :m], ref_ids[:, :m])
    assert np.array_equal(got_dist[:, :m], ref_dist[:, :m])
    assert (got_ids[:, m:] == -1).all() and (got_dist[:, m:] == -1).all()


def _trace(rng, n_req, rate):
    rp, idx, w = WL.serving_sets(rng, n_req)
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    kind = (rng.random(n_req) < 0.5).astype(np.int32)  # 1 = search
    k = np.where(kind == 1, 1024, rng.choice([64, 256, 1024], size=n_req)).astype(np.int32)
    return arrival, kind, k, rp, idx, w


@pytest.fixture(scope="module")
def served(torch, ctx):
    from paper_2005_11547_amd import Server, SketchDB, SketchInfo, dms
    rng = np.random.default_rng(55)
    n_db = 1500
    db_rp, db_idx, db_w = WL.serving_sets(rng, n_db)
    db_bits = O.sketch_csr(db_rp, db_idx, db_w, 1024, SEED)["bits"]   # the oracle builds the database
    db = SketchDB(ctx, 1024, n_db)
    # the oracle's sketches follow specification version 1 with the mixer and SEED
    db.append_bits(torch.from_numpy(db_bits.view(np.int64)).cuda(), SketchInfo(1, dms.HASH_MIX, SEED, 1024, 0))
    arrival, kind, k, rp, idx, w = _trace(rng, 240, 20_000.0)
    srv = Server(ctx, db, topk=10, max_batch=64, max_inflight=3)
    out = srv.replay(arrival, kind, k, rp, idx, w)
    yield dict(db_bits=db_bits, db=db, trace=(arrival, kind, k, rp, idx, w), out=out, srv=srv)
    srv.close()  # a server goes before its context


def test_served_results_equal_oracle(served):
    arrival, kind, k, rp, idx, w = served["trace"]
    out = served["out"]
    print(f"[serve] stats {out['stats']}", flush=True)
    for r in range(len(arrival)):
        ii, ww = idx[rp[r]:rp[r + 1]], w[rp[r]:rp[r + 1]]
        ref = O.sketch_csr(np.array([0, len(ii)]), ii, ww, int(k[r]), SEED)
        assert out["status"][r] == ref["status"][0]
        assert np.array_equal(out["sketch"][r], ref["u32"][0]), r
        if kind[r] == 1:
            rid, rdist = O.hamming_topk(served["db_bits"], ref["bits"], 10)
            assert np.array_equal(out["ids"][r], rid[0]) and np.array_equal(out["dist"][r], rdist[0]), r
        else:
            assert (out["ids"][r] == -2).all()   # untouched: no search for a sketch request
    assert out["stats"]["batches"] >= 1 and out["stats"]["p99_s"] >= out["stats"]["p50_s"] > 0


def test_each_result_same_alone_and_in_the_mix(served):
    arrival, kind, k, rp, idx, w = served["trace"]
    out = served["out"]
    for r in range(0, len(arrival), 6):
        sub_rp = np.array([0, rp[r + 1] - rp[r]], np.int64)
        alone = served["srv"].replay(np.zeros(1), kind[r:r + 1], k[r:r + 1], sub_rp,
                                     idx[rp[r]:rp[r + 1]], w[rp[r]:rp[r + 1]])
        assert np.array_equal(alone["sketch"][0], out["sketch"][r])
        assert alone["status"][0] == out["status"][r]
        assert np.array_equal(alone["ids"][0], out["ids"][r])
        assert np.array_equal(alone["dist"][0], out["dist"][r])


def test_admission_under_a_tiny_arena(torch, ctx, served):
    from paper_2005_11547_amd import Server
    arrival, kind, k, rp, idx, w = served["trace"]
    n = 60
    srv = Server(ctx, served["db"], topk=10, max_batch=3, max_inflight=2, max_batch_nnz=4096,
                 max_set_nnz=4096)
    small = srv.replay(arrival[:n] * 0.0, kind[:n], k[:n], rp[:n + 1], idx[:rp[n]], w[:rp[n]])
    srv.close()
    for r in range(n):
        assert np.array_equal(small["sketch"][r], served["out"]["sketch"][r])
        assert np.array_equal(small["ids"][r], served["out"]["ids"][r])
    assert small["stats"]["batches"] >= n / 3


def test_server_rejects_bad_requests(torch, ctx, served):
    from paper_2005_11547_amd import DMSError
    arrival, kind, k, rp, idx, w = served["trace"]
    bad_k = k[:2].copy()
    bad_k[0] = 128
    with pytest.raises(DMSError):
        served["srv"].replay(arrival[:2], kind[:2], bad_k, rp[:3], idx[:rp[2]], w[:rp[2]])
    bad_kind = kind[:2].copy()
    bad_kind[:] = 1
    bad_k2 = np.array([64, 64], np.int32)
    with pytest.raises(DMSError):
        served["srv"].replay(arrival[:2], bad_kind, bad_k2, rp[:3], idx[:rp[2]], w[:rp[2]])


@pytest.mark.parametrize("split", [0, 16, 100])
def test_split_threshold_does_not_change_results(torch, ctx, served, split):
    # sets above the threshold are cut into parts run by several wavefronts
    # (at 16, nearly every set); the served results may not change
    from paper_2005_11547_amd import Server
    arrival, kind, k, rp, idx, w = served["trace"]
    n = 120
    srv = Server(ctx, served["db"], topk=10, max_batch=40, max_inflight=2, split_nnz=split)
    got = srv.replay(arrival[:n] * 0.0, kind[:n], k[:n], rp[:n + 1], idx[:rp[n]], w[:rp[n]])
    srv.close()
    for r in range(n):
        assert np.array_equal(got["sketch"][r], served["out"]["sketch"][r]), (split, r)
        assert got["status"][r] == served["out"]["status"][r]
        assert np.array_equal(got["ids"][r], served["out"]["ids"][r])


def _serve_online(srv, kind, k, rp, idx, w, burst):
    # submit in bursts, polling between them, then drain
    ids, got = [], {}
    n = len(kind)
    for b0 in range(0, n, burst):
        for r in range(b0, min(n, b0 + burst)):
            ids.append(srv.submit(kind[r], k[r], idx[rp[r]:rp[r + 1]], w[rp[r]:rp[r + 1]]))
        for a in srv.poll(wait_ms=0):
            got[a["id"]] = a
    for _ in range(2000):
        if len(got) == n:
            break
        for a in srv.poll(wait_ms=20, max_out=64):
            assert a["id"] not in got
            got[a["id"]] = a
    return ids, got


@pytest.mark.parametrize("burst,max_batch", [(1, 64), (17, 8), (240, 64)])
def test_online_submit_poll_equals_replay_and_oracle(torch, ctx, served, burst, max_batch):
    # requests handed in one by one (dms_server_submit) and collected as they
    # finish (dms_server_poll) get the answers the trace replay gave, which
    # equal the oracle's
    from paper_2005_11547_amd import Server
    arrival, kind, k, rp, idx, w = served["trace"]
    srv = Server(ctx, served["db"], topk=10, max_batch=max_batch, max_inflight=3)
    print(f"[online] burst={burst} max_batch={max_batch}", flush=True)
    ids, got = _serve_online(srv, kind, k, rp, idx, w, burst)
    assert ids == list(range(len(kind)))              # ids are handed out in order
    assert len(got) == len(kind)
    assert srv.poll(wait_ms=0) == []                   # nothing left over
    ref = served["out"]
    for r, rid in enumerate(ids):
        a = got[rid]
        assert a["status"] == ref["status"][r]
        assert np.array_equal(a["sketch"][:k[r]], ref["sketch"][r]), r
        if kind[r] == 1:
            assert np.array_equal(a["ids"], ref["ids"][r]) and np.array_equal(a["dist"], ref["dist"][r]), r
        else:
            assert (a["ids"] == -2).all()
        assert a["latency"] > 0
    for r in range(0, len(kind), 40):                  # a sample straight against the oracle
        ii, ww = idx[rp[r]:rp[r + 1]], w[rp[r]:rp[r + 1]]
        o = O.sketch_csr(np.array([0, len(ii)]), ii, ww, int(k[r]), SEED)
        assert np.array_equal(got[ids[r]]["sketch"][:k[r]], o["u32"][0])
    srv.close()


def test_online_requests_block_a_replay_and_bad_requests_are_refused(torch, ctx, served):
    from paper_2005_11547_amd import DMSError, Server
    arrival, kind, k, rp, idx, w = served["trace"]
    srv = Server(ctx, served["db"], topk=10, max_batch=8, max_inflight=1, max_set_nnz=4096)
    with pytest.raises(DMSError):
        srv.submit(1, 64, idx[:3], w[:3])              # a search needs k = 1024
    with pytest.raises(DMSError):
        srv.submit(0, 128, idx[:3], w[:3])             # k outside 64, 256, 1024
    with pytest.raises(DMSError):
        srv.submit(0, 64, np.zeros(5000, np.int32), np.ones(5000))  # above max_set_nnz
    rid = srv.submit(0, 64, idx[rp[0]:rp[1]], w[rp[0]:rp[1]])
    with pytest.raises(DMSError):                      # a replay may not overtake pending requests
        srv.replay(arrival[:1], kind[:1], k[:1], rp[:2], idx[:rp[1]], w[:rp[1]])
    got = []
    for _ in range(500):
        got += srv.poll(wait_ms=20)
        if got:
            break
    assert [a["id"] for a in got] == [rid]
    out = srv.replay(arrival[:1] * 0.0, np.zeros(1, np.int32), np.array([64], np.int32), rp[:2],
                     idx[:rp[1]], w[:rp[1]])
    assert np.array_equal(out["sketch"][0], got[0]["sketch"][:64])
    assert out["status"][0] == got[0]["status"]
    srv.close()


def test_closing_a_context_closes_its_server_and_index_first(torch, ctx, served):
    # the C ABI needs servers and indexes destroyed before their context; the
    # binding does it, and no stale HIP error reaches later calls
    from paper_2005_11547_amd import Context, LshIndex, Server, to_device
    c2 = Context(SEED)
    srv = Server(c2, served["db"], topk=10, max_batch=8, max_inflight=1)
    rp, idx, w = WL.csr_from_rows([([1, 5, 9], [1.0, 2.0, 0.5]), ([2, 3], [1.0, 1.0])])
    ix = LshIndex(c2, *to_device(rp, idx, w), 4, 2)
    c2.close()
    assert not srv._h and not ix._h
    out = ctx.sketch(*to_device(rp, idx, w), 64)
    torch.cuda.synchronize()
    assert np.array_equal(out["u32"].cpu().numpy().view(np.uint32), O.sketch_csr(rp, idx, w, 64, SEED)["u32"])


def test_database_provenance_is_checked(torch, ctx, served):
    """A database, its appends and its queries carry the (specification version,
    hash, seed, k) they were made under: mismatches are refused, matching
    sketches from the library and from the oracle are interchangeable."""
    from paper_2005_11547_amd import Context, Server, SketchDB, SketchInfo, dms, to_device
    rng = np.random.default_rng(56)
    rp, idx, w = WL.serving_sets(rng, 50)
    d = to_device(rp, idx, w)
    ref = O.sketch_csr(rp, idx, w, 1024, SEED)
    mine = ctx.sketch_info(1024)
    assert mine.as_tuple() == (dms.SPEC_VERSION, dms.HASH_MIX, SEED, 1024)
    db = SketchDB(ctx, 1024, 200)
    first, st = db.append_sets(*d)
    db.append_bits(torch.from_numpy(ref["bits"].view(np.int64)).cuda(), mine)
    info, n, rows = db.info()
    assert first == 0 and n == 100 and info.as_tuple() == mine.as_tuple()
    torch.cuda.synchronize()
    assert np.array_equal(st.cpu().numpy(), ref["status"])
    q = torch.from_numpy(ref["bits"][:7].view(np.int64)).cuda()
    ids, dist = db.topk(q, 3, mine)
    torch.cuda.synchronize()
    assert (dist.cpu().numpy()[:, 0] == 0).all()  # each query finds its own two copies at distance 0
    assert (ids.cpu().numpy()[:, :2] == np.stack([np.arange(7), np.arange(7) + 50], 1)).all()
    for bad in (SketchInfo(2, dms.HASH_MIX, SEED, 1024, 0), SketchInfo(1, dms.HASH_TAB, SEED, 1024, 0),
                SketchInfo(1, dms.HASH_MIX, SEED + 1, 1024, 0), SketchInfo(1, dms.HASH_MIX, SEED, 256, 0)):
        with pytest.raises(dms.DMSError) as e:
            db.append_bits(q, bad)
        assert e.value.code == dms.DMS_EMISMATCH
        with pytest.raises(dms.DMSError):
            db.topk(q, 3, bad)
    with pytest.raises(dms.DMSError):  # past the capacity
        db.append_bits(torch.zeros((101, 16), dtype=torch.int64, device="cuda"), mine)
    # a server accepts only a database of its context's sketches at k = 1024
    other = Context(SEED + 1)
    with pytest.raises(dms.DMSError) as e:
        Server(other, db, topk=10, max_batch=8, max_inflight=1)
    assert e.value.code == dms.DMS_EMISMATCH
    small = SketchDB(ctx, 256, 4)
    with pytest.raises(dms.DMSError):
        Server(ctx, small, topk=10, max_batch=8, max_inflight=1)
    tab = Context(SEED)
    tab.set_option(dms.OPT_HASH, dms.HASH_TAB)
    with pytest.raises(dms.DMSError):
        Server(tab, db, topk=10, max_batch=8, max_inflight=1)
    # a database made before the context's hash changed refuses further appends
    ctx2 = Context(SEED)
    db2 = SketchDB(ctx2, 1024, 60)
    ctx2.set_option(dms.OPT_HASH, dms.HASH_TAB)
    with pytest.raises(dms.DMSError) as e:
        db2.append_sets(*d)
    assert e.value.code == dms.DMS_EMISMATCH
    srv = Server(ctx, db, topk=10, max_batch=8, max_inflight=1)
    srv.close()
    for c in (other, tab, ctx2):
        c.close()
    small.close()
    db.close()
