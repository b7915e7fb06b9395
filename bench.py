"""Throughput benchmark of the DartMinHash hot path on one MI355X.

One step = one dms_sketch_csr call over the whole batch (all sets, k minhashes
plus 1-bit sketches), inputs resident in HBM.  Prints one JSON line.

`roofline` prices the main kernel against the int-VALU peak: algorithmic work
is one mixer evaluation per region, area, generated dart, rank-passing dart and
accepted dart, as the GPU itself counts them over the whole batch
(DMS_FLAG_COUNTERS, one extra untimed call), at the chip's measured lane-op
cost of a mixer, divided by the main kernel's average duration over the timed
steps (HIP events around that kernel on its stream, DMS_OPT_TIMING).  The
oracle, run on a sample of the sets at the same schedule, must report the same
counts for them; `frac_paper_schedule` prices the paper's retry schedule
(phi = 1, 2, ...) from the oracle's counts instead.  The secondary lines (other
workloads, estimators, fingerprints, the LSH index and the serving loop, which
--serving-seconds 0 skips) follow the same pattern; each checks a sample of its
outputs against the oracle.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch_k256]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as WL  # noqa: E402

PEAK_INT_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 39.32 T full-rate 32-bit lane-ops/s
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "batch_k256": dict(gen=lambda: WL.batch_k256(), k=256,
                       desc="1,000,000 sets, nnz=clip(round(LogNormal(ln 256,1)),1,4096), d=2^20, "
                            "w~Exp(1), k=256, uint32 minhashes + 1-bit sketches"),
    "uneven_k1024": dict(gen=lambda: WL.uneven_k1024(), k=1024,
                         desc="100,000 sets, nnz~Zipf(1.5) on [1,65536], d=2^24, w~LogNormal(0,1) "
                              "rescaled to ||x||_1=10^U(-3,3), k=1024, uint32 + 1-bit"),
    "plain_k64": dict(gen=lambda: WL.plain_k64()[:3], k=64,
                      desc="1,000 sets + 200 planted pairs, nnz~U{16..128}, d=10^4, "
                           "w~U(0,1], k=64, uint32 + 1-bit"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_work(counters, c_mix, band=False):
    """Lane-op equivalents per set, from exact enumeration counts (the oracle's
    counter records, or the GPU's int64 [n, 8] rows): one mixer per region,
    area, generated dart (rank uniform), rank-passing dart (weight uniform) and
    accepted dart (id hash), each costing c_mix, plus 8 lane-ops per dart
    uniform (53-bit conversion and the three FP64 operations of the rank or
    weight formula, and its compare).  With `band` the oracle's rank and
    acceptance counts of each pass's new band are used (what a retry that keeps
    its darts needs)."""
    if isinstance(counters, np.ndarray) and counters.dtype.names is None:
        c = counters.astype(np.float64)
        reg, area, gen, rank, acc = c[:, 0], c[:, 1], c[:, 2], c[:, 3], c[:, 4]
    else:
        reg, area, gen = (counters[f].astype(np.float64) for f in ("regions", "areas", "generated"))
        rank = counters["rank_new" if band else "rank_pass"].astype(np.float64)
        acc = counters["accepted_new" if band else "accepted"].astype(np.float64)
    H = reg + area + gen + rank + acc
    extra = 8.0 * (gen + rank)
    return H, c_mix * H + extra


def gpu_counts(run_with_counters, n, torch):
    """int64 [n, 8] enumeration counts of one untimed call with DMS_FLAG_COUNTERS."""
    cnt = torch.empty((n, 8), dtype=torch.int64, device="cuda")
    run_with_counters(cnt)
    torch.cuda.synchronize()
    out = cnt.cpu().numpy()
    del cnt
    return out


def cpu_info():
    """CPU model and logical cores of this host (lscpu)."""
    import subprocess
    info = {"model": None, "logical_cpus": os.cpu_count()}
    try:
        text = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in text.splitlines():
            if line.startswith("Model name:"):
                info["model"] = line.split(":", 1)[1].strip()
            elif line.startswith("Socket(s):"):
                info["sockets"] = int(line.split(":", 1)[1])
            elif line.startswith("Core(s) per socket:"):
                info["cores_per_socket"] = int(line.split(":", 1)[1])
    except Exception:
        pass
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    return info


def _oracle_shard(args):
    """One worker of the all-core baseline: the oracle over its rows."""
    from oracle import oracle as O
    rp, idx, w, k = args
    t0 = time.perf_counter()
    O.sketch_csr(rp, idx, w, k, WL.HASH_SEED)
    return len(rp) - 1, time.perf_counter() - t0


def _rows(rp, idx, w, rows):
    sub_rp = np.concatenate([[0], np.cumsum(rp[rows + 1] - rp[rows])]).astype(np.int64)
    sub_idx = np.concatenate([idx[rp[r]:rp[r + 1]] for r in rows]) if len(rows) else idx[:0]
    sub_w = np.concatenate([w[rp[r]:rp[r + 1]] for r in rows]) if len(rows) else w[:0]
    return sub_rp, sub_idx, sub_w


def cpu_all_cores(rp, idx, w, k, stride, workers):
    """The oracle on every `stride`-th set, as `workers` processes over
    contiguous shards of about equal nonzeros (forked before the GPU is used).
    Returns (sets/s of the whole sample, sets, workers, wall seconds)."""
    import multiprocessing as mp
    rows = np.arange(0, len(rp) - 1, stride)
    sub_rp, sub_idx, sub_w = _rows(rp, idx, w, rows)
    cuts = np.searchsorted(sub_rp, np.linspace(0, sub_rp[-1], workers + 1)[1:-1])
    bounds = [0] + [int(c) for c in cuts] + [len(rows)]
    shards = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        if b > a:
            shards.append((sub_rp[a:b + 1] - sub_rp[a], sub_idx[sub_rp[a]:sub_rp[b]],
                           sub_w[sub_rp[a]:sub_rp[b]], k))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(len(shards)) as pool:
        done = pool.map(_oracle_shard, shards)
    wall = time.perf_counter() - t0
    n = sum(d[0] for d in done)
    return n / wall, n, len(shards), wall


def cpu_configs(seconds_each=4.0):
    """Single-core oracle sets/s on the other configurations (row samples, each
    under a time budget): plain_k64 (all 1,400 rows), uneven_k1024 (every
    100th set), lsh_L64K8 ((64,8) keys; 10,000 sets drawn from the same
    generator)."""
    from oracle import oracle as O
    out = {}
    cases = (("plain_k64", lambda: WL.plain_k64()[:3], 1, "sketch", 64),
             ("uneven_k1024", lambda: WL.uneven_k1024(), 100, "sketch", 1024),
             ("lsh_L64K8", lambda: WL.lsh_L64K8(n_sets=10_000), 1, "lsh", None))
    for name, gen, stride, kind, k in cases:
        rp, idx, w = gen()
        rows = np.arange(0, len(rp) - 1, stride)
        got, t_cpu, chunk = 0, 0.0, 32
        while got < len(rows) and t_cpu < seconds_each:
            sel = rows[got:got + chunk]
            c_rp, c_idx, c_w = _rows(rp, idx, w, sel)
            t0 = time.perf_counter()
            if kind == "sketch":
                O.sketch_csr(c_rp, c_idx, c_w, k, WL.HASH_SEED)
            else:
                O.lsh_csr(c_rp, c_idx, c_w, 64, 8, WL.HASH_SEED)
            t_cpu += time.perf_counter() - t0
            got += len(sel)
        out[name] = {"sets_per_s": got / t_cpu, "sets": int(got), "seconds": t_cpu,
                     "sample": f"every {stride}th set" if stride > 1 else "all sets"}
        log(f"cpu baseline {name}: {out[name]}")
    return out


def calibrate_mixer(ctx, torch, n_cu):
    """Mixer evaluations per second at full occupancy (8 chains per thread)."""
    buf = torch.zeros(8, dtype=torch.int64, device="cuda")
    blocks, iters = n_cu * 8, 4096
    ctx.calibrate(0, 64, blocks, buf)  # warm-up
    ms = min(ctx.calibrate(0, iters, blocks, buf) for _ in range(3))
    mixers = blocks * 256 * iters * 8
    return mixers / (ms * 1e-3)


def serving_run(ctx, torch, seconds, n_db, rate=50_000.0, warm=1.0, split_nnz=128):
    """The serving workload: Poisson arrivals at `rate`, half sketch-only requests
    (k uniform in {64, 256, 1024}), half 1-bit k = 1024 sketch + top-10 Hamming
    search against a device-resident database of n_db sketched sets; 1% of the
    searches are near-duplicates (J = 0.9) of database rows.  The first `warm`
    seconds of the trace are excluded from the latency figures."""
    from paper_2005_11547_amd import Server, SketchDB
    rng = np.random.Generator(np.random.PCG64(5))
    t0 = time.time()
    db_rp, db_idx, db_w = WL.serving_sets(rng, n_db)
    log(f"serving: database of {n_db} sets generated in {time.time() - t0:.1f}s")
    d = [torch.from_numpy(a).cuda() for a in (db_rp, db_idx, db_w)]
    db = SketchDB(ctx, 1024, n_db)  # 1-bit k = 1024 rows that record the context's provenance
    torch.cuda.synchronize()
    t0 = time.time()
    db.append_sets(*d)
    torch.cuda.synchronize()
    log(f"serving: database sketched (k=1024, 1-bit) in {time.time() - t0:.2f}s")
    del d
    n_req = int(rate * (seconds + warm))
    rp, idx, w = WL.serving_sets(rng, n_req)
    arrival = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    kind = (rng.random(n_req) < 0.5).astype(np.int32)
    k = np.where(kind == 1, 1024, rng.choice([64, 256, 1024], size=n_req)).astype(np.int32)
    # plant near-duplicates of database rows among the searches
    planted = np.nonzero(kind == 1)[0]
    planted = planted[rng.random(len(planted)) < 0.01]
    targets = rng.integers(0, n_db, size=len(planted))
    rows = [(idx[rp[r]:rp[r + 1]], w[rp[r]:rp[r + 1]]) for r in range(n_req)]
    for r, tgt in zip(planted, targets):
        rows[r] = WL.near_duplicate(rng, db_idx[db_rp[tgt]:db_rp[tgt + 1]], db_w[db_rp[tgt]:db_rp[tgt + 1]], 0.9)
    rp, idx, w = WL.csr_from_rows(rows)
    srv = Server(ctx, db, topk=10, max_batch=512, max_inflight=4, max_batch_nnz=1 << 21,
                 max_set_nnz=8192, split_nnz=split_nnz)
    log(f"serving: replaying {n_req} requests at {rate:.0f}/s")
    out = srv.replay(arrival, kind, k, rp, idx, w)
    srv.close()
    db.close()
    steady = arrival >= warm
    lat = np.sort(out["latency"][steady])
    top1 = float(np.mean(out["ids"][planted, 0] == targets)) if len(planted) else None
    res = {"rate_req_s": rate, "requests": int(n_req), "completed_req_s": out["stats"]["req_per_s"],
           "p50_ms": float(lat[int(0.50 * (len(lat) - 1))] * 1e3),
           "p99_ms": float(lat[int(0.99 * (len(lat) - 1))] * 1e3),
           "max_ms": float(lat[-1] * 1e3), "batches": out["stats"]["batches"],
           "mean_batch": out["stats"]["mean_batch"], "db_rows": n_db,
           "search_share": float(kind.mean()), "planted_top1": top1,
           "trace": f"{seconds:.0f}s after {warm:.0f}s warm-up", "split_nnz": split_nnz}
    log(f"serving: {res}")
    return res


def plain_engine_run(torch, d, k, out_u32, out_bits, steps=2):
    """The same batch through the plain engine (one launch, one wave per set,
    one lane per nonzero): its time per batch, and whether all of its outputs
    equal the persistent engine's."""
    from paper_2005_11547_amd import Context, dms
    n = out_u32.shape[0]
    c = Context(WL.HASH_SEED, engine=dms.ENGINE_PLAIN)
    u32 = torch.empty_like(out_u32)
    bits = torch.empty_like(out_bits)
    st = torch.empty(n, dtype=torch.int8, device="cuda")
    c.dms_sketch_csr(n, d[0], d[1], d[2], k, u32, bits, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        c.dms_sketch_csr(n, d[0], d[1], d[2], k, u32, bits, st)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    same = bool(torch.equal(u32, out_u32) and torch.equal(bits, out_bits))
    c.close()
    res = {"ms_per_step": ms, "sets_per_s": n / (ms * 1e-3), "identical_to_persistent_engine": same}
    log(f"plain engine: {res}")
    del u32, bits, st
    return res


def secondary_runs(ctx, torch, steps=3, main=None, c_mix=None):
    """Throughput of the other batch workloads (k = 1024 uneven batching,
    (L,K) = (64,8) LSH keys, bottom-k sketches with k = 256 of the main batch,
    and the main batch under the tabulation-hash variant), each checked bit for
    bit on a row sample; for the uneven batch, the LSH keys and bottom-k also
    the fraction of the int-VALU peak, priced on the GPU's own enumeration
    counts over the whole batch and the main kernel's event-timed duration (the
    oracle's counts at the same schedule must equal the GPU's on the sample)."""
    from oracle import oracle as O
    from paper_2005_11547_amd import Context, dms, to_device
    res = {}
    for name, gen, kind in (("uneven_k1024", WL.uneven_k1024, "sketch"),
                            ("lsh_L64K8", WL.lsh_L64K8, "lsh"),
                            ("bottomk_k256", WL.batch_k256, "bottomk"),
                            ("tabulation_k256", WL.batch_k256, "tabulation")):
        # the main batch is reused rather than generated again
        rp, idx, w = main if (main is not None and gen is WL.batch_k256) else gen()
        n = len(rp) - 1
        d = to_device(rp, idx, w)
        run_ctx = ctx
        if kind == "tabulation":
            # the main batch with the tabulation-hash variant of the specification
            run_ctx = Context(WL.HASH_SEED)
            run_ctx.set_option(dms.OPT_HASH, dms.HASH_TAB)
            out = torch.empty((n, 256), dtype=torch.int32, device="cuda")
            st = torch.empty(n, dtype=torch.int8, device="cuda")
            run = lambda f=0, c=None: run_ctx.dms_sketch_csr(n, d[0], d[1], d[2], 256, out, None, st, flags=f,
                                                            out_counters=c)
        elif kind == "sketch":
            out = torch.empty((n, 1024), dtype=torch.int32, device="cuda")
            bits = torch.empty((n, 16), dtype=torch.int64, device="cuda")
            st = torch.empty(n, dtype=torch.int8, device="cuda")
            run = lambda f=0, c=None: ctx.dms_sketch_csr(n, d[0], d[1], d[2], 1024, out, bits, st, flags=f,
                                                        out_counters=c)
        elif kind == "lsh":
            out = torch.empty((n, 64), dtype=torch.int64, device="cuda")
            st = torch.empty(n, dtype=torch.int8, device="cuda")
            run = lambda f=0, c=None: ctx.dms_lsh_keys(n, d[0], d[1], d[2], 64, 8, out, st, flags=f, out_counters=c)
        else:
            out = torch.empty((n, 256), dtype=torch.int64, device="cuda")
            rk = torch.empty((n, 256), dtype=torch.float64, device="cuda")
            st = torch.empty(n, dtype=torch.int8, device="cuda")
            run = lambda f=0, c=None: ctx.dms_bottomk(n, d[0], d[1], d[2], 256, out, rk, st, flags=f, out_counters=c)
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        run_ctx.set_option(dms.OPT_TIMING, 1)
        run_ctx.kernel_time()
        e0.record()
        for _ in range(steps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        k_total, k_n = run_ctx.kernel_time()
        run_ctx.set_option(dms.OPT_TIMING, 0)
        kernel_ms = k_total / max(k_n, 1)
        rows = np.linspace(0, n - 1, 200).astype(np.int64)
        sub_rp, sub_idx, sub_w = _rows(rp, idx, w, rows)
        got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
        if kind == "tabulation":
            ref = O.sketch_csr(sub_rp, sub_idx, sub_w, 256, WL.HASH_SEED, hash=O.HASH_TAB)["u32"]
            exact = bool(np.array_equal(got.view(np.uint32), ref))
        elif kind == "sketch":
            ref = O.sketch_csr(sub_rp, sub_idx, sub_w, 1024, WL.HASH_SEED)["u32"]
            exact = bool(np.array_equal(got.view(np.uint32), ref))
        elif kind == "lsh":
            ref = O.lsh_csr(sub_rp, sub_idx, sub_w, 64, 8, WL.HASH_SEED)["keys"]
            exact = bool(np.array_equal(got.view(np.uint64), ref))
        else:
            ref = O.bottomk_csr(sub_rp, sub_idx, sub_w, 256, WL.HASH_SEED)
            exact = bool(np.array_equal(got.view(np.uint64), ref["s"]) and
                         np.array_equal(rk[torch.from_numpy(rows).cuda()].cpu().numpy(), ref["rank"]))
        res[name] = {"sets_per_s": n / (ms * 1e-3), "nnz_per_s": float(rp[-1]) / (ms * 1e-3),
                     "ms_per_step": ms, "kernel_ms": kernel_ms, "n_sets": n,
                     "bit_exact_sample": {"sets_checked": 200, "exact": exact}}
        if kind != "tabulation" and c_mix is not None:
            # the GPU's own counts over the whole batch; the oracle at the same
            # schedule on every 50th set must count the same
            g_cnt = gpu_counts(lambda c: run(dms.FLAG_COUNTERS, c), n, torch)
            srows = np.arange(0, n, 50)
            s_rp, s_idx, s_w = _rows(rp, idx, w, srows)
            if kind == "sketch":
                r = O.sketch_csr(s_rp, s_idx, s_w, 1024, WL.HASH_SEED, phi0=ctx.get_option(dms.OPT_PHI0),
                                 schedule=O.SCHED_DOUBLE, full=True)
                rc, paper = r["counters"], O.sketch_csr(s_rp, s_idx, s_w, 1024, WL.HASH_SEED, full=True)["counters"]
                fold = 0
            elif kind == "lsh":
                r = O.lsh_csr(s_rp, s_idx, s_w, 64, 8, WL.HASH_SEED, phi0=ctx.get_option(dms.OPT_LSH_PHI0),
                              schedule=O.SCHED_DOUBLE, counters=True)
                rc, paper = r["counters"][:, 0], O.lsh_csr(s_rp, s_idx, s_w, 64, 8, WL.HASH_SEED,
                                                            counters=True)["counters"][:, 0]
                fold = 64 * (8 + 1)  # the key of each table folds its K ids, one mixer each, plus its seed
            else:
                r = O.bottomk_csr(s_rp, s_idx, s_w, 256, WL.HASH_SEED, phi0=1.0 + 3.0 / 16.0,
                                  schedule=O.SCHED_DOUBLE, counters=True)
                rc, paper = r["counters"][:, 0], O.bottomk_csr(s_rp, s_idx, s_w, 256, WL.HASH_SEED,
                                                                counters=True)["counters"][:, 0]
                fold = 0
            okr = r["status"] == 0
            names = ("regions", "areas", "generated", "rank_new", "accepted_new")
            same = bool(all(np.array_equal(g_cnt[srows][okr, q], rc[nm][okr]) for q, nm in enumerate(names)))
            ok_all = st.cpu().numpy() == 0
            H, ops = algorithmic_work(g_cnt[ok_all], c_mix)
            total = float(ops.sum()) + c_mix * fold * float(ok_all.sum())
            achieved = total / (kernel_ms * 1e-3) / 1e12
            Hp, opsp = algorithmic_work(paper[okr], c_mix)
            res[name]["roofline"] = {
                "bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS, "unit": "T int32 lane-op/s",
                "frac": achieved / PEAK_INT_TOPS, "work": "the GPU's own enumeration counts over the whole batch",
                "mixers_per_set": float(H.mean()) + fold,
                "counts_equal_oracle_sample": same,
                "frac_paper_schedule": (float(opsp.mean()) + c_mix * fold) * float(ok_all.sum())
                / (kernel_ms * 1e-3) / 1e12 / PEAK_INT_TOPS,
                "mixers_per_set_paper_schedule": float(Hp.mean()) + fold,
                "sample": f"oracle counts on every 50th set ({len(srows)} sets)"}
        log(f"{name}: {res[name]}")
        if run_ctx is not ctx:
            run_ctx.close()
        del d, out
    return res


def fingerprint_runs(ctx, torch, out_u32, out_bits, k, bits=8, steps=5, big_pairs_1bit=1 << 24,
                     big_pairs_bbit=1 << 21):
    """Estimates and fingerprints, all HBM bound, each moving about 1 GB or
    more per call: the u32 estimate over the main batch's row pairs (2i, 2i+1),
    b-bit packing and the unary map of the main batch's minhashes, and the
    1-bit and b-bit estimates over 2^24 and 2^21 pairs of random rows (their
    cost does not depend on the values).  GB/s of each call's algorithmic bytes
    against the 8 TB/s peak, each checked bit for bit on a sample."""
    from paper_2005_11547_amd import dms
    from oracle import oracle as O
    n = out_u32.shape[0]
    words = (k * bits + 63) // 64
    packed = torch.empty((n, words), dtype=torch.int64, device="cuda")
    n_pairs = n // 2
    uidx = torch.empty((n, k), dtype=torch.int32, device="cuda")
    ua_all, ub_all = out_u32[0:2 * n_pairs:2].contiguous(), out_u32[1:2 * n_pairs:2].contiguous()
    est_u32 = torch.empty(n_pairs, dtype=torch.float64, device="cuda")
    bwords = (k + 63) // 64
    g = torch.Generator(device="cuda")
    g.manual_seed(2005_11547)

    def rand_rows(m, w):
        return torch.randint(-2 ** 63, 2 ** 63 - 1, (m, w), dtype=torch.int64, device="cuda", generator=g)

    ba, bb = rand_rows(big_pairs_1bit, bwords), rand_rows(big_pairs_1bit, bwords)
    pa, pb = rand_rows(big_pairs_bbit, words), rand_rows(big_pairs_bbit, words)
    est_1bit = torch.empty(big_pairs_1bit, dtype=torch.float64, device="cuda")
    est = torch.empty(big_pairs_bbit, dtype=torch.float64, device="cuda")
    runs = {
        "estimate_u32": (lambda: ctx.dms_jaccard_est(n_pairs, ua_all, ub_all, k, dms.FMT_U32, est_u32),
                         n_pairs * (8.0 * k + 8.0)),
        "estimate_1bit": (lambda: ctx.dms_jaccard_est(big_pairs_1bit, ba, bb, k, dms.FMT_1BIT, est_1bit),
                          big_pairs_1bit * (16.0 * bwords + 8.0)),
        "pack": (lambda: ctx.dms_bbit_pack(n, out_u32, k, bits, packed), n * (4.0 * k + 8.0 * words)),
        "estimate": (lambda: ctx.dms_jaccard_est_bbit(big_pairs_bbit, pa, pb, k, bits, est),
                     big_pairs_bbit * (16.0 * words + 8.0)),
        "unary_map": (lambda: ctx.dms_unary_map(n, out_u32, k, bits, uidx), n * 8.0 * k),
    }
    res = {"bits": bits, "n_sets": n, "k": k,
           "pairs": f"u32: rows (2i, 2i + 1) of the batch; 1-bit: {big_pairs_1bit} and b-bit: {big_pairs_bbit} "
                    f"pairs of random rows"}
    # each timed call starts after 512 MiB of unrelated writes, so its inputs come
    # from HBM, not from the 256 MB last-level cache
    flush = torch.empty(512 * 2 ** 20 // 8, dtype=torch.int64, device="cuda")
    for name, (fn, nbytes) in runs.items():
        fn()
        torch.cuda.synchronize()
        ms = 0.0
        for rep in range(steps):
            flush.fill_(rep)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1) / steps
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"ms": ms, "gbs": gbs, "frac_hbm": gbs / PEAK_HBM_GBS, "bytes": nbytes}
    rows = np.linspace(0, n_pairs - 1, 200).astype(np.int64)
    sel = torch.from_numpy(rows).cuda()
    ra = torch.from_numpy(2 * rows).cuda()
    ua = out_u32[ra].cpu().numpy().view(np.uint32)
    ub = out_u32[ra + 1].cpu().numpy().view(np.uint32)
    ok = np.array_equal(packed[ra].cpu().numpy().view(np.uint64), O.bbit_pack(ua, bits))
    ok &= np.array_equal(uidx[ra].cpu().numpy(), O.unary_map(ua, bits)[0])
    ok &= np.array_equal(est_u32[sel].cpu().numpy(), O.jaccard_est_u32(ua, ub))
    r1 = torch.from_numpy(np.linspace(0, big_pairs_1bit - 1, 200).astype(np.int64)).cuda()
    ok &= np.array_equal(est_1bit[r1].cpu().numpy(), O.jaccard_est_1bit(ba[r1].cpu().numpy().view(np.uint64),
                                                                        bb[r1].cpu().numpy().view(np.uint64), k))
    r2 = torch.from_numpy(np.linspace(0, big_pairs_bbit - 1, 200).astype(np.int64)).cuda()
    ok &= np.array_equal(est[r2].cpu().numpy(), O.jaccard_est_bbit(pa[r2].cpu().numpy().view(np.uint64),
                                                                    pb[r2].cpu().numpy().view(np.uint64), k, bits))
    res["bit_exact_sample"] = {"rows_checked": 200, "exact": bool(ok)}
    log(f"fingerprints: {res}")
    del packed, est, uidx, ua_all, ub_all, ba, bb, pa, pb, est_u32, est_1bit, flush
    return res


def index_run(ctx, torch, n_queries=10_000, j1=0.5, topn=10):
    """Weight-class LSH index over the (L,K) = (64,8) workload's 1M sets at
    scales 2^-8..2^8: build time, query throughput for near-duplicate queries
    (J = 0.9 of a random indexed set, at its own scale), the share whose planted
    set comes first, and the exact Jaccard of returned pairs re-checked by the
    oracle on a sample."""
    from oracle import oracle as O
    from paper_2005_11547_amd import LshIndex, to_device
    rp, idx, w = WL.lsh_L64K8()
    rng = np.random.default_rng(31)
    n = len(rp) - 1
    scale = np.repeat(2.0 ** rng.integers(-8, 9, size=n), np.diff(rp))
    w = w * scale
    d = to_device(rp, idx, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ix = LshIndex(ctx, *d, 64, 8)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    picks = rng.choice(n, size=n_queries, replace=False)
    queries = [WL.near_duplicate(rng, idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]], J=0.9) for q in picks]
    qd = to_device(*WL.csr_from_rows(queries))
    ix.query(*qd, j1, topn)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out = ix.query(*qd, j1, topn)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ids, jv = out["ids"].cpu().numpy(), out["j"].cpu().numpy()
    cand = out["candidates"].cpu().numpy()
    ok = True
    for m in range(0, n_queries, n_queries // 50):
        for r in range(topn):
            x = int(ids[m, r])
            if x < 0:
                break
            ok &= O.weighted_jaccard_merge(*queries[m], idx[rp[x]:rp[x + 1]], w[rp[x]:rp[x + 1]]) == jv[m, r]
    res = {"n_sets": n, "L": 64, "K": 8, "j1": j1, "build_s": build_s, "queries": n_queries,
           "query_ms": ms, "queries_per_s": n_queries / (ms * 1e-3),
           "planted_top1": float(np.mean(ids[:, 0] == picks)), "mean_candidates": float(cand.mean()),
           "exact_j_sample": {"queries_checked": 50, "exact": bool(ok)}}
    log(f"lsh_index: {res}")
    ix.close()
    del d, qd
    return res


# The paper's Table 1 (DartMinHash column, mean ms per set on an Intel i7-10510U,
# one core): (k, ||x||_0, ||x||_1, ms).
TABLE1 = [(1, 256, 1.0, 0.02), (256, 256, 1.0, 0.17), (4096, 256, 1.0, 2.67), (1, 4096, 1.0, 0.30),
          (256, 4096, 1.0, 0.49), (4096, 4096, 1.0, 3.64), (64, 64, 1.0, 0.04), (64, 1024, 1.0, 0.10),
          (64, 16384, 1.0, 1.37), (1024, 64, 1.0, 0.58), (1024, 1024, 1.0, 0.78),
          (1024, 16384, 1.0, 2.06), (256, 1024, 1.0, 0.26), (256, 1024, 2.0 ** 64, 2.47),
          (256, 1024, 2.0 ** -64, 2.25), (256, 1024, 2.0 ** 512, 18.58), (256, 1024, 2.0 ** -512, 17.10)]


def table1_run(ctx, torch, cpu_seconds=2.0):
    """The paper's Table 1 shapes: weights uniform on the simplex scaled to ||x||_1,
    random ids (Section 4, "Synthetic data").  GPU: sets/s on a batch of each
    shape; oracle: ms per set on one host core; paper: its ms per set (context)."""
    from oracle import oracle as O
    from paper_2005_11547_amd import to_device
    rows = []
    for i, (k, l0, l1, paper_ms) in enumerate(TABLE1):
        n = max(200, min(20000, 4_000_000 // l0))
        rp, idx, w = WL.simplex_sets(100 + i, n, l0, l1)
        d = to_device(rp, idx, w)
        out = torch.empty((n, k), dtype=torch.int32, device="cuda")
        st = torch.empty(n, dtype=torch.int8, device="cuda")
        ctx.dms_sketch_csr(n, d[0], d[1], d[2], k, out, None, st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.dms_sketch_csr(n, d[0], d[1], d[2], k, out, None, st)
        e1.record()
        torch.cuda.synchronize()
        gpu_ms = e0.elapsed_time(e1)
        # oracle: sets one by one until the time budget, checked against the GPU
        t0 = time.perf_counter()
        m = 0
        exact = True
        got = out.cpu().numpy().view(np.uint32)
        while m < n and time.perf_counter() - t0 < cpu_seconds:
            r = O.sketch_csr(np.array([0, l0]), idx[rp[m]:rp[m + 1]], w[rp[m]:rp[m + 1]], k, WL.HASH_SEED)
            exact &= bool(np.array_equal(r["u32"][0], got[m]))
            m += 1
        cpu_ms = (time.perf_counter() - t0) / max(m, 1) * 1e3
        row = {"k": k, "l0": l0, "l1": "2^%d" % round(np.log2(l1)) if l1 != 1.0 else 1,
               "gpu_sets_per_s": n / (gpu_ms * 1e-3), "gpu_us_per_set": gpu_ms * 1e3 / n,
               "oracle_ms_per_set": cpu_ms, "paper_ms_per_set": paper_ms,
               "gpu_batch": n, "bit_exact_sets": m, "exact": exact,
               "status_ok": bool((st.cpu().numpy() == 0).all())}
        log(f"table1: {row}")
        rows.append(row)
        del d, out
    return rows


def cached(name, gen, cache_dir):
    """A workload's CSR arrays, generated once and kept in cache_dir (if given)."""
    if not cache_dir:
        return gen()
    os.makedirs(cache_dir, exist_ok=True)
    path = os.path.join(cache_dir, name + ".npz")
    if not os.path.exists(path):
        rp, idx, w = gen()
        np.savez(path, rp=rp, idx=idx, w=w)
    z = np.load(path)
    return z["rp"], z["idx"], z["w"]


def kernels_once(cache_dir):
    """Every benched kernel once at its benched size, nothing else (for counter
    runs under rocprofv3): the k = 256 batch sketch, the uneven k = 1024
    sketch, the (64,8) LSH keys, bottom-k (k = 256), the estimators, b-bit pack,
    unary map and both copy calibration kernels."""
    import torch
    from paper_2005_11547_amd import Context, dms, to_device
    ctx = Context(WL.HASH_SEED)
    done = []
    rp, idx, w = cached("batch_k256", WL.batch_k256, cache_dir)
    n = len(rp) - 1
    d = to_device(rp, idx, w)
    u32 = torch.empty((n, 256), dtype=torch.int32, device="cuda")
    bits = torch.empty((n, 4), dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int8, device="cuda")
    ctx.dms_sketch_csr(n, *d, 256, u32, bits, st)
    bs = torch.empty((n, 256), dtype=torch.int64, device="cuda")
    br = torch.empty((n, 256), dtype=torch.float64, device="cuda")
    ctx.dms_bottomk(n, *d, 256, bs, br, st)
    torch.cuda.synchronize()
    done += ["sketch batch_k256", "bottomk batch_k256"]
    del bs, br, d
    fp = fingerprint_runs(ctx, torch, u32, bits, 256, steps=1)
    done += [k for k in fp if isinstance(fp[k], dict) and "gbs" in fp[k]]
    del u32, bits
    rp, idx, w = cached("lsh_L64K8", WL.lsh_L64K8, cache_dir)
    n = len(rp) - 1
    d = to_device(rp, idx, w)
    keys = torch.empty((n, 64), dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int8, device="cuda")
    ctx.dms_lsh_keys(n, *d, 64, 8, keys, st)
    torch.cuda.synchronize()
    done.append("lsh_keys lsh_L64K8")
    del d, keys
    rp, idx, w = cached("uneven_k1024", WL.uneven_k1024, cache_dir)
    n = len(rp) - 1
    d = to_device(rp, idx, w)
    u32 = torch.empty((n, 1024), dtype=torch.int32, device="cuda")
    bits = torch.empty((n, 16), dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int8, device="cuda")
    ctx.dms_sketch_csr(n, *d, 1024, u32, bits, st)
    torch.cuda.synchronize()
    done.append("sketch uneven_k1024")
    nb = 1 << 30
    src = torch.ones(nb // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    ctx.calibrate(2, 1, n_cu * 8, src, dst, nb)
    ctx.calibrate(3, 1, n_cu * 8, src, dst, nb)
    done.append("copy calibration (plain, four in flight), 1 GiB")
    print(json.dumps({"kernels_once": done}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--autotune", type=int, default=0,
                    help="pick the schedule with dms_autotune before timing (1) or time the context's "
                         "defaults (0, the default: they are the measured optimum for batch_k256; the "
                         "tuner's own choice is then reported under secondary.autotune)")
    ap.add_argument("--workload", default="batch_k256", choices=sorted(WORKLOADS))
    ap.add_argument("--engine", default="fast", choices=["fast", "plain"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="time budget of the oracle CPU baseline (0 disables it)")
    ap.add_argument("--cpu-stride", type=int, default=25,
                    help="oracle sample: every n-th set")
    ap.add_argument("--cpu-all-stride", type=int, default=10,
                    help="all-core oracle baseline: every n-th set")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="all-core oracle baseline: at most this many processes")
    ap.add_argument("--serving-seconds", type=float, default=5.0,
                    help="length of the served trace at 50k requests/s (0 disables serving)")
    ap.add_argument("--serving-db", type=int, default=1_000_000, help="database rows")
    ap.add_argument("--serving-split", type=int, default=128,
                    help="serving: sets with more nonzeros are shared by several wavefronts (0: never)")
    ap.add_argument("--table1", action="store_true",
                    help="time the paper's Table 1 shapes instead (GPU, oracle, paper) and exit")
    ap.add_argument("--secondary", type=int, default=1,
                    help="also time the k=1024 and LSH workloads (0 disables)")
    ap.add_argument("--copy-calibration", type=int, default=1 << 30,
                    help="bytes moved by the stream-copy calibration kernel (0 disables it)")
    ap.add_argument("--kernels-once", action="store_true",
                    help="run every benched kernel once at its benched size and exit (for counter runs)")
    ap.add_argument("--data-cache", default="",
                    help="directory that keeps generated workloads between runs (--kernels-once)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the sets of a batch "
              "are independent, so the path shards by rows with no exchange; multi-GPU runs are "
              "not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_11547_amd import Context, dms, to_device

    if args.kernels_once:
        kernels_once(args.data_cache)
        return

    if args.table1:
        ctx = Context(WL.HASH_SEED)
        print(json.dumps({"table1": table1_run(ctx, torch)}), flush=True)
        return

    wl = WORKLOADS[args.workload]
    k = wl["k"]
    t0 = time.time()
    rp, idx, w = wl["gen"]()
    n_sets = len(rp) - 1
    nnz = int(rp[-1])
    log(f"{args.workload}: {n_sets} sets, {nnz} nnz generated in {time.time() - t0:.1f}s")

    # CPU baselines first: the all-core run forks worker processes, which must
    # happen before this process touches the GPU
    host = cpu_info()
    all_core = None
    if args.cpu_seconds > 0:
        workers = max(1, min(args.cpu_workers, host.get("affinity_cpus") or os.cpu_count() or 1))
        rate, n_all, used, wall = cpu_all_cores(rp, idx, w, k, args.cpu_all_stride, workers)
        all_core = {"value": rate, "unit": "sets/s", "cores": used, "kind": "oracle",
                    "sample": f"every {args.cpu_all_stride}th set ({n_all} sets) in {used} processes over "
                              f"shards of equal nonzeros, {wall:.1f}s wall"}
        log(f"cpu baseline all cores: {all_core}")
    other_cfgs = cpu_configs() if args.cpu_seconds > 0 else None

    d_rp, d_idx, d_w = to_device(rp, idx, w)
    out_u32 = torch.empty((n_sets, k), dtype=torch.int32, device="cuda")
    words = (k + 63) // 64
    out_bits = torch.empty((n_sets, words), dtype=torch.int64, device="cuda")
    out_status = torch.empty(n_sets, dtype=torch.int8, device="cuda")
    engine = dms.ENGINE_FAST if args.engine == "fast" else dms.ENGINE_PLAIN
    ctx = Context(WL.HASH_SEED, engine=engine)
    tuned = None
    if args.autotune:
        # the schedule (first phi, split threshold) is picked on a prefix of this
        # batch before any timing; outputs do not depend on it
        t0 = time.perf_counter()
        phi0, split = ctx.autotune(d_rp, d_idx, d_w, k)
        tuned = {"phi0": phi0, "split_nnz": split, "order": ctx.get_option(dms.OPT_ORDER),
                 "seconds": time.perf_counter() - t0}
        log(f"autotune: {tuned}")
    schedule = {"phi0": ctx.get_option(dms.OPT_PHI0), "split_nnz": ctx.get_option(dms.OPT_SPLIT_NNZ),
                "largest_first": bool(ctx.get_option(dms.OPT_ORDER)), "autotuned": tuned is not None}

    def step():
        ctx.dms_sketch_csr(n_sets, d_rp, d_idx, d_w, k, out_u32, out_bits, out_status)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.set_option(dms.OPT_TIMING, 1)  # events around the main kernel of each step
    ctx.kernel_time()
    wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1) / args.steps
    k_total, k_launches = ctx.kernel_time()
    ctx.set_option(dms.OPT_TIMING, 0)
    kernel_ms = k_total / max(k_launches, 1)
    log(f"{args.steps} steps: {ms:.3f} ms/step (events), {wall / args.steps * 1e3:.3f} ms/step (wall), "
        f"main kernel {kernel_ms:.3f} ms ({k_launches} launches)")

    sets_per_s = n_sets / (ms * 1e-3)
    nnz_per_s = nnz / (ms * 1e-3)
    status = out_status.cpu().numpy()

    # the GPU's own enumeration counts over the whole batch (one untimed call)
    g_cnt = gpu_counts(lambda c: ctx.dms_sketch_csr(n_sets, d_rp, d_idx, d_w, k, out_u32, out_bits, out_status,
                                                    flags=dms.FLAG_COUNTERS, out_counters=c), n_sets, torch)

    # roofline: algorithmic integer work per launch / launch duration
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    mix_rate = calibrate_mixer(ctx, torch, n_cu)
    c_mix = PEAK_INT_TOPS * 1e12 / mix_rate
    log(f"mixer calibration: {mix_rate / 1e12:.3f} T mixers/s -> {c_mix:.1f} lane-op slots per mixer")

    from oracle import oracle as O
    stride = max(1, args.cpu_stride)
    sample = np.arange(0, n_sets, stride)
    sub_rp, sub_idx, sub_w = _rows(rp, idx, w, sample)
    # the oracle at the GPU's schedule (first phi, doubling) on the sample under
    # a time budget: the single-core CPU baseline, the outputs and the counts
    got = 0
    t_cpu = 0.0
    chunk = 64
    ref_u32, ref_bits, ref_st, cnts = [], [], [], []
    while got < len(sample) and (t_cpu < max(args.cpu_seconds, 1.0)):
        hi = min(len(sample), got + chunk)
        c_rp = sub_rp[got:hi + 1] - sub_rp[got]
        c_idx = sub_idx[sub_rp[got]:sub_rp[hi]]
        c_w = sub_w[sub_rp[got]:sub_rp[hi]]
        tc = time.perf_counter()
        r = O.sketch_csr(c_rp, c_idx, c_w, k, WL.HASH_SEED, phi0=schedule["phi0"], schedule=O.SCHED_DOUBLE,
                         full=True)
        t_cpu += time.perf_counter() - tc
        ref_u32.append(r["u32"]); ref_bits.append(r["bits"]); ref_st.append(r["status"])
        cnts.append(r["counters"])
        got = hi
    rows = sample[:got]
    ref_u32 = np.concatenate(ref_u32); ref_bits = np.concatenate(ref_bits)
    ref_st = np.concatenate(ref_st); cnts = np.concatenate(cnts)
    gpu_u32 = out_u32[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint32)
    gpu_bits = out_bits[torch.from_numpy(rows).cuda()].cpu().numpy().view(np.uint64)
    exact = bool(np.array_equal(gpu_u32, ref_u32) and np.array_equal(gpu_bits, ref_bits)
                 and np.array_equal(status[rows], ref_st))
    okr = ref_st == 0
    names = ("regions", "areas", "generated", "rank_new", "accepted_new")
    counts_equal = bool(all(np.array_equal(g_cnt[rows][okr, q], cnts[name][okr]) for q, name in enumerate(names)))
    log(f"oracle sample: {got} sets in {t_cpu:.1f}s; GPU bit-exact on them: {exact}; counts equal: {counts_equal}")
    # the paper's schedule (phi = 1, 2, 3, ...) on a smaller sample, for context
    p_rows = np.arange(0, n_sets, stride * 10)
    pr = O.sketch_csr(*_rows(rp, idx, w, p_rows), k, WL.HASH_SEED, full=True)
    Hp, opsp = algorithmic_work(pr["counters"], c_mix)

    ok_all = status == 0
    H, ops = algorithmic_work(g_cnt[ok_all], c_mix)
    ops_launch = float(ops.sum())
    achieved = ops_launch / (kernel_ms * 1e-3) / 1e12
    okp = pr["status"] == 0
    hbm_bytes = 8.0 * (n_sets + 1) + 12.0 * nnz + n_sets * (4.0 * k + 8.0 * words + 1.0)

    traffic = None
    if args.workload == "batch_k256" and args.engine == "fast":
        from paper_2005_11547_amd import profiling
        traffic = profiling.read_traffic(os.path.join(ROOT, "profiles", "traffic_all_benched_kernels.txt"))
    result = {
        "metric": "sketches/sec",
        "value": sets_per_s,
        "unit": "sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 hashing, f64 ranks",
        "data": "synthetic",
        "nnz_per_s": nnz_per_s,
        "bit_exact_vs_oracle": {"sets_checked": int(got), "exact": exact},
        "config": {"workload": f"{args.workload}: {wl['desc']}", "n_sets": n_sets, "nnz": nnz,
                   "k": k, "engine": args.engine, "parallelism": "one GPU",
                   "schedule": schedule},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS,
                     "unit": "T int32 lane-op/s", "frac": achieved / PEAK_INT_TOPS,
                     "traffic": traffic,
                     "work": "the GPU's own enumeration counts over the whole batch",
                     "kernel_ms": kernel_ms,
                     "mixers_per_set": float(H.mean()) if len(H) else 0.0,
                     "counts_equal_oracle_sample": counts_equal,
                     "frac_step": ops_launch / (ms * 1e-3) / 1e12 / PEAK_INT_TOPS,
                     "frac_paper_schedule": (float(opsp[okp].mean()) * n_sets / (kernel_ms * 1e-3) / 1e12
                                             / PEAK_INT_TOPS if okp.any() else 0.0),
                     "mixers_per_set_paper_schedule": float(Hp[okp].mean()) if okp.any() else 0.0,
                     "lane_ops_per_mixer": c_mix,
                     "hbm_gbs_algorithmic": hbm_bytes / (kernel_ms * 1e-3) / 1e9},
        "cpu_baseline": {"value": got / t_cpu if t_cpu > 0 else None, "unit": "sets/s",
                         "cores": 1, "kind": "oracle",
                         "sample": f"every {stride}th set of the same batch, first {got} of them "
                                   f"({t_cpu:.1f}s of single-thread CPU work, the GPU's schedule)",
                         "host": host, "all_cores": all_core, "other_configs": other_cfgs},
    }
    if args.copy_calibration > 0:
        nb = (args.copy_calibration // 16) * 16
        src = torch.empty(nb // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1)
        copy = {}
        for kind, name in ((2, "plain"), (3, "four_in_flight_streaming")):
            for blocks in (n_cu * 8, n_cu * 32):
                ctx.calibrate(kind, 1, blocks, src, dst, nb)  # warm-up
                ms_copy = min(ctx.calibrate(kind, 1, blocks, src, dst, nb) for _ in range(3))
                copy[f"{name}_{blocks}_blocks"] = 2.0 * nb / (ms_copy * 1e-3) / 1e9
        result["roofline"]["hbm_copy_gbs"] = max(copy.values())
        result["roofline"]["hbm_copy_variants_gbs"] = copy
        log(f"stream copy of {nb} bytes (read+write GB/s): {copy}")
        del src, dst
    if args.secondary and args.workload == "batch_k256":
        fp = fingerprint_runs(ctx, torch, out_u32, out_bits, k)
        plain = plain_engine_run(torch, (d_rp, d_idx, d_w), k, out_u32, out_bits)
        result["secondary"] = secondary_runs(ctx, torch, main=(rp, idx, w), c_mix=c_mix)
        result["secondary"]["bbit_b8"] = fp
        result["secondary"]["plain_engine_batch_k256"] = plain
        result["secondary"]["lsh_index_L64K8"] = index_run(ctx, torch)
        if not args.autotune:
            # what the autotuner picks for this batch (on a context of its own)
            t0 = time.perf_counter()
            tctx = Context(WL.HASH_SEED, engine=engine)
            phi0, split = tctx.autotune(d_rp, d_idx, d_w, k)
            order = tctx.get_option(dms.OPT_ORDER)
            tctx.close()
            result["secondary"]["autotune"] = {"phi0": phi0, "split_nnz": split, "order": order,
                                               "seconds": time.perf_counter() - t0}
            log(f"autotune: {result['secondary']['autotune']}")
    if args.serving_seconds > 0:
        result["serving"] = serving_run(ctx, torch, args.serving_seconds, args.serving_db,
                                        split_nnz=args.serving_split)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
