"""Python binding of the DartMinHash C ABI (include/dms.h).

Argument marshalling only: every step of the sketching path runs in the HIP
kernels of ``libdms.so``.  PyTorch provides device memory and the stream.
The binding raises if the library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdms.so")

DMS_OK, DMS_EINVAL, DMS_EHIP, DMS_ENOMEM, DMS_ESPEC, DMS_EMISMATCH = 0, -1, -2, -3, -4, -5
SPEC_VERSION = 1
SET_OK, SET_EMPTY, SET_RANGE, SET_INVALID = 0, 1, 2, 3
ENGINE_FAST, ENGINE_PLAIN = 0, 1
OPT_ENGINE, OPT_PHI0, OPT_LSH_PHI0, OPT_PHI_MAX, OPT_SPLIT_NNZ, OPT_BOTTOMK_PHI0, OPT_HASH, OPT_ORDER = (
    0, 1, 2, 3, 4, 5, 6, 7)
OPT_TIMING = 8
OPT_WAVES, OPT_TILE = 9, 10
HASH_MIX, HASH_TAB = 0, 1
FMT_U32, FMT_1BIT = 0, 1
FLAG_VALIDATE, FLAG_COUNTERS = 1, 2
COUNTER_WORDS = 8  # regions, areas, generated, rank passed, accepted, passes, last phi (bits), 0

EXPORTS = ["dms_create", "dms_destroy", "dms_set_stream", "dms_set_option", "dms_get_option",
           "dms_sketch_csr", "dms_lsh_keys", "dms_jaccard_est", "dms_hamming_topk", "dms_sync",
           "dms_last_error", "dms_status_str", "dms_t_of_k", "dms_spec_constants", "dms_calibrate",
           "dms_server_create", "dms_server_destroy", "dms_server_replay", "dms_server_submit",
           "dms_server_poll", "dms_bbit_pack",
           "dms_jaccard_est_bbit", "dms_unary_map", "dms_bottomk", "dms_jaccard_est_bottomk",
           "dms_index_build", "dms_index_sets", "dms_index_query", "dms_index_destroy", "dms_autotune",
           "dms_spec_tabulation", "dms_kernel_time", "dms_prepare", "dms_sketch_csr_noalloc",
           "dms_sketch_info_of", "dms_db_create", "dms_db_append_sets", "dms_db_append_bits", "dms_db_info",
           "dms_db_topk", "dms_db_destroy"]

REQ_SKETCH, REQ_SEARCH = 0, 1

_lib = None


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch_nnz", ctypes.c_int64), ("max_set_nnz", ctypes.c_int32),
                ("db_words", ctypes.c_int32), ("topk", ctypes.c_int32), ("split_nnz", ctypes.c_int32)]


class SketchInfo(ctypes.Structure):
    """Provenance of sketches (dms_sketch_info): comparable only when equal."""
    _fields_ = [("spec_version", ctypes.c_int32), ("hash", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("k", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_tuple(self):
        return (self.spec_version, self.hash, self.seed, self.k)


class DMSError(RuntimeError):
    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


def lib():
    """Load libdms.so (built by paper_2005_11547_amd/build_lib.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise DMSError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double)
    P = ctypes.POINTER
    sig = {
        "dms_create": ([P(vp), ctypes.c_int, u64], i32),
        "dms_destroy": ([vp], i32),
        "dms_set_stream": ([vp, vp], i32),
        "dms_set_option": ([vp, i32, f64], i32),
        "dms_get_option": ([vp, i32, P(f64)], i32),
        "dms_sketch_csr": ([vp, i64, vp, vp, vp, i32, vp, vp, vp, vp, vp, u32, vp], i32),
        "dms_lsh_keys": ([vp, i64, vp, vp, vp, i32, i32, vp, vp, u32, vp], i32),
        "dms_jaccard_est": ([vp, i64, vp, vp, i32, i32, vp], i32),
        "dms_bbit_pack": ([vp, i64, vp, i32, i32, vp], i32),
        "dms_bottomk": ([vp, i64, vp, vp, vp, i32, vp, vp, vp, u32, vp], i32),
        "dms_index_build": ([vp, i64, vp, vp, vp, i32, i32, ctypes.POINTER(vp)], i32),
        "dms_index_sets": ([vp, vp, vp], i32),
        "dms_index_query": ([vp, i64, vp, vp, vp, f64, i32, vp, vp, vp, vp, vp], i32),
        "dms_index_destroy": ([vp], i32),
        "dms_spec_tabulation": ([u64, vp], i32),
        "dms_autotune": ([vp, i64, vp, vp, vp, i32, ctypes.POINTER(f64), ctypes.POINTER(f64)], i32),
        "dms_jaccard_est_bottomk": ([vp, i64, vp, vp, vp, vp, i32, vp], i32),
        "dms_jaccard_est_bbit": ([vp, i64, vp, vp, i32, i32, vp], i32),
        "dms_unary_map": ([vp, i64, vp, i32, i32, vp, ctypes.POINTER(ctypes.c_double)], i32),
        "dms_hamming_topk": ([vp, vp, i64, i32, vp, i64, i32, vp, vp], i32),
        "dms_sync": ([vp], i32),
        "dms_kernel_time": ([vp, P(f64), P(i64)], i32),
        "dms_prepare": ([vp, i32], i32),
        "dms_sketch_csr_noalloc": ([vp, i64, vp, vp, vp, i32, vp, vp, vp], i32),
        "dms_last_error": ([vp], ctypes.c_char_p),
        "dms_status_str": ([i32], ctypes.c_char_p),
        "dms_t_of_k": ([i32, P(u32)], i32),
        "dms_spec_constants": ([u64, u32, vp, vp, vp, vp, vp], i32),
        "dms_calibrate": ([vp, i32, i32, i64, i32, vp, vp, P(f64)], i32),
        "dms_server_create": ([vp, P(ServerConfig), vp, P(vp)], i32),
        "dms_sketch_info_of": ([vp, i32, P(SketchInfo)], i32),
        "dms_db_create": ([vp, i32, i64, P(vp)], i32),
        "dms_db_append_sets": ([vp, i64, vp, vp, vp, vp, P(i64)], i32),
        "dms_db_append_bits": ([vp, i64, vp, P(SketchInfo), P(i64)], i32),
        "dms_db_info": ([vp, P(SketchInfo), P(i64), P(vp)], i32),
        "dms_db_topk": ([vp, vp, i64, P(SketchInfo), i32, vp, vp], i32),
        "dms_db_destroy": ([vp], i32),
        "dms_server_destroy": ([vp], i32),
        "dms_server_replay": ([vp, i64] + [vp] * 13, i32),
        "dms_server_submit": ([vp, i32, i32, i64, vp, vp, P(i64)], i32),
        "dms_server_poll": ([vp, i32, i64] + [vp] * 7, i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(t):
    """Device (or host) address of a tensor / numpy array, or None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ctypes.c_void_p(t.data_ptr())
    return t.ctypes.data_as(ctypes.c_void_p)


def t_of_k(k: int) -> int:
    t = ctypes.c_uint32(0)
    st = lib().dms_t_of_k(k, ctypes.byref(t))
    if st != DMS_OK:
        raise DMSError(f"dms_t_of_k({k}) -> {st}")
    return t.value


def spec_constants(seed: int, t: int) -> dict:
    """The library's own derivation of the specification constants (host only)."""
    import numpy as np
    keys = np.zeros(6, np.uint64)
    pois = np.zeros(20, np.uint64)
    W = np.zeros(1024, np.float64)
    R = np.zeros(1024, np.float64)
    u = ctypes.c_double(0.0)
    st = lib().dms_spec_constants(seed, t, _ptr(keys), _ptr(pois), _ptr(W), _ptr(R), ctypes.byref(u))
    if st != DMS_OK:
        raise DMSError(f"dms_spec_constants -> {st}")
    return dict(keys=keys, pois=pois, W=W, R=R, u=u.value)


def spec_tabulation(seed: int):
    """The library's simple-tabulation tables for the seed (host only)."""
    import numpy as np
    out = np.zeros(8 * 256, np.uint64)
    st = lib().dms_spec_tabulation(seed, _ptr(out))
    if st != DMS_OK:
        raise DMSError(f"dms_spec_tabulation -> {st}")
    return out


class Context:
    """One dms_ctx on a GPU; calls run on torch's current stream of that device."""

    def __init__(self, seed: int, device: int = 0, engine: int | None = None):
        import torch
        import weakref
        self.device = device
        self._h = ctypes.c_void_p()
        self._dependents = weakref.WeakSet()  # servers and indexes built on this context
        self._check(lib().dms_create(ctypes.byref(self._h), device, seed), "dms_create")
        self.seed = seed
        if engine is not None:
            self.set_option(OPT_ENGINE, engine)
        self._torch = torch

    def _check(self, st, what):
        if st != DMS_OK:
            msg = lib().dms_last_error(self._h).decode() if getattr(self, "_h", None) else ""
            raise DMSError(f"{what}: {lib().dms_status_str(st).decode()} {msg}", st)

    def sketch_info(self, k: int) -> SketchInfo:
        """Provenance of this context's sketches at k."""
        info = SketchInfo()
        self._check(lib().dms_sketch_info_of(self._h, k, ctypes.byref(info)), "dms_sketch_info_of")
        return info

    def close(self):
        """Destroy the context, and first every server, index and sketch
        database built on it (the C ABI requires them to go before their
        context)."""
        if self._h:
            # servers first: they read the databases
            for dep in sorted(self._dependents, key=lambda d: not isinstance(d, Server)):
                dep.close()
            lib().dms_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        s = self._torch.cuda.current_stream(self.device).cuda_stream
        self._check(lib().dms_set_stream(self._h, ctypes.c_void_p(s)), "dms_set_stream")

    def set_option(self, opt: int, value: float):
        self._check(lib().dms_set_option(self._h, opt, float(value)), "dms_set_option")

    def get_option(self, opt: int) -> float:
        v = ctypes.c_double(0.0)
        self._check(lib().dms_get_option(self._h, opt, ctypes.byref(v)), "dms_get_option")
        return v.value

    # -- raw C-ABI calls on device tensors -----------------------------------
    def dms_sketch_csr(self, n_sets, row_ptr, idx, w, k, out_u32=None, out_bits=None,
                       out_status=None, out_s=None, out_rank=None, flags=0, out_counters=None):
        self._stream()
        self._check(lib().dms_sketch_csr(self._h, n_sets, _ptr(row_ptr), _ptr(idx), _ptr(w), k,
                                         _ptr(out_u32), _ptr(out_bits), _ptr(out_status),
                                         _ptr(out_s), _ptr(out_rank), flags, _ptr(out_counters)),
                    "dms_sketch_csr")

    def dms_prepare(self, k):
        self._stream()
        self._check(lib().dms_prepare(self._h, k), "dms_prepare")

    def dms_sketch_csr_noalloc(self, n_sets, row_ptr, idx, w, k, out_u32=None, out_bits=None, out_status=None):
        self._stream()
        self._check(lib().dms_sketch_csr_noalloc(self._h, n_sets, _ptr(row_ptr), _ptr(idx), _ptr(w), k,
                                                 _ptr(out_u32), _ptr(out_bits), _ptr(out_status)),
                    "dms_sketch_csr_noalloc")

    def dms_lsh_keys(self, n_sets, row_ptr, idx, w, L, K, out_keys, out_status=None, flags=0,
                     out_counters=None):
        self._stream()
        self._check(lib().dms_lsh_keys(self._h, n_sets, _ptr(row_ptr), _ptr(idx), _ptr(w), L, K,
                                       _ptr(out_keys), _ptr(out_status), flags, _ptr(out_counters)),
                    "dms_lsh_keys")

    def dms_jaccard_est(self, n_pairs, a, b, k, fmt, out):
        self._stream()
        self._check(lib().dms_jaccard_est(self._h, n_pairs, _ptr(a), _ptr(b), k, fmt, _ptr(out)),
                    "dms_jaccard_est")

    def autotune(self, row_ptr, idx, w, k):
        """Pick the fastest first phi and split threshold for this batch and k
        (sets them on the context); returns (phi0, split)."""
        self._stream()
        phi0, split = ctypes.c_double(0.0), ctypes.c_double(0.0)
        self._check(lib().dms_autotune(self._h, row_ptr.numel() - 1, _ptr(row_ptr), _ptr(idx), _ptr(w), k,
                                       ctypes.byref(phi0), ctypes.byref(split)), "dms_autotune")
        return phi0.value, split.value

    def dms_bottomk(self, n_sets, row_ptr, idx, w, k, out_s, out_rank=None, out_status=None, flags=0,
                    out_counters=None):
        self._stream()
        self._check(lib().dms_bottomk(self._h, n_sets, _ptr(row_ptr), _ptr(idx), _ptr(w), k, _ptr(out_s),
                                      _ptr(out_rank), _ptr(out_status), flags, _ptr(out_counters)),
                    "dms_bottomk")

    def dms_jaccard_est_bottomk(self, n_pairs, rank_a, s_a, rank_b, s_b, k, out):
        self._stream()
        self._check(lib().dms_jaccard_est_bottomk(self._h, n_pairs, _ptr(rank_a), _ptr(s_a), _ptr(rank_b),
                                                  _ptr(s_b), k, _ptr(out)), "dms_jaccard_est_bottomk")

    def dms_bbit_pack(self, n_sets, minhash, k, bits, out):
        self._stream()
        self._check(lib().dms_bbit_pack(self._h, n_sets, _ptr(minhash), k, bits, _ptr(out)), "dms_bbit_pack")

    def dms_jaccard_est_bbit(self, n_pairs, a, b, k, bits, out):
        self._stream()
        self._check(lib().dms_jaccard_est_bbit(self._h, n_pairs, _ptr(a), _ptr(b), k, bits, _ptr(out)),
                    "dms_jaccard_est_bbit")

    def dms_unary_map(self, n_sets, minhash, k, bits, out_index):
        self._stream()
        scale = ctypes.c_double(0.0)
        self._check(lib().dms_unary_map(self._h, n_sets, _ptr(minhash), k, bits, _ptr(out_index),
                                        ctypes.byref(scale)), "dms_unary_map")
        return scale.value

    def dms_hamming_topk(self, db, n_db, words, queries, n_q, topk, out_ids, out_dist):
        self._stream()
        self._check(lib().dms_hamming_topk(self._h, _ptr(db), n_db, words, _ptr(queries), n_q, topk,
                                           _ptr(out_ids), _ptr(out_dist)), "dms_hamming_topk")

    def calibrate(self, kind, iters, blocks, a, b=None, nbytes=0):
        """Run one calibration kernel (see dms_calibrate); returns its duration in ms."""
        self._stream()
        ms = ctypes.c_double(0.0)
        self._check(lib().dms_calibrate(self._h, kind, iters, nbytes, blocks, _ptr(a), _ptr(b),
                                        ctypes.byref(ms)), "dms_calibrate")
        return ms.value

    def sync(self):
        self._check(lib().dms_sync(self._h), "dms_sync")

    def kernel_time(self):
        """(summed ms, launches) of the main kernels timed since the last call
        (needs OPT_TIMING = 1); waits for them."""
        ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
        self._check(lib().dms_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)), "dms_kernel_time")
        return ms.value, n.value

    # -- conveniences that allocate outputs ----------------------------------
    def _flags(self, n, dev, counters, validate):
        """(flags, counter tensor or None) for the sketching calls."""
        flags = (FLAG_COUNTERS if counters else 0) | (FLAG_VALIDATE if validate else 0)
        cnt = (self._torch.empty((n, COUNTER_WORDS), dtype=self._torch.int64, device=dev)
               if counters else None)
        return flags, cnt

    def sketch(self, row_ptr, idx, w, k, bits=True, full=False, counters=False, validate=False):
        """Sketch a CSR batch already on the GPU; returns a dict of device tensors
        (with ``counters`` also the int64 [n, 8] enumeration counts)."""
        torch = self._torch
        n = row_ptr.numel() - 1
        dev = row_ptr.device
        out = dict(u32=torch.empty((n, k), dtype=torch.int32, device=dev),
                   status=torch.empty(n, dtype=torch.int8, device=dev))
        if bits:
            out["bits"] = torch.empty((n, (k + 63) // 64), dtype=torch.int64, device=dev)
        if full:
            out["s"] = torch.empty((n, k), dtype=torch.int64, device=dev)
            out["rank"] = torch.empty((n, k), dtype=torch.float64, device=dev)
        flags, cnt = self._flags(n, dev, counters, validate)
        self.dms_sketch_csr(n, row_ptr, idx, w, k, out["u32"], out.get("bits"), out["status"],
                            out.get("s"), out.get("rank"), flags, cnt)
        if counters:
            out["counters"] = cnt
        return out

    def lsh(self, row_ptr, idx, w, L, K, counters=False, validate=False):
        torch = self._torch
        n = row_ptr.numel() - 1
        dev = row_ptr.device
        out = dict(keys=torch.empty((n, L), dtype=torch.int64, device=dev),
                   status=torch.empty(n, dtype=torch.int8, device=dev))
        flags, cnt = self._flags(n, dev, counters, validate)
        self.dms_lsh_keys(n, row_ptr, idx, w, L, K, out["keys"], out["status"], flags, cnt)
        if counters:
            out["counters"] = cnt
        return out

    def jaccard(self, a, b, k, fmt):
        torch = self._torch
        out = torch.empty(a.shape[0], dtype=torch.float64, device=a.device)
        self.dms_jaccard_est(a.shape[0], a, b, k, fmt, out)
        return out

    def bottomk(self, row_ptr, idx, w, k, counters=False, validate=False):
        """Bottom-k sketches: dict s (int64 [n, k], uint64 bits), rank (float64
        [n, k]) and status (int8 [n])."""
        torch = self._torch
        n = row_ptr.numel() - 1
        dev = row_ptr.device
        out = dict(s=torch.empty((n, k), dtype=torch.int64, device=dev),
                   rank=torch.empty((n, k), dtype=torch.float64, device=dev),
                   status=torch.empty(n, dtype=torch.int8, device=dev))
        flags, cnt = self._flags(n, dev, counters, validate)
        self.dms_bottomk(n, row_ptr, idx, w, k, out["s"], out["rank"], out["status"], flags, cnt)
        if counters:
            out["counters"] = cnt
        return out

    def jaccard_bottomk(self, rank_a, s_a, rank_b, s_b):
        torch = self._torch
        n, k = rank_a.shape
        out = torch.empty(n, dtype=torch.float64, device=rank_a.device)
        self.dms_jaccard_est_bottomk(n, rank_a, s_a, rank_b, s_b, k, out)
        return out

    def bbit_pack(self, minhash, bits):
        """Packed b-bit fingerprints of [n, k] uint32 minhashes (stored as int32):
        int64 [n, ceil(k*bits/64)]."""
        torch = self._torch
        n, k = minhash.shape
        out = torch.empty((n, (k * bits + 63) // 64), dtype=torch.int64, device=minhash.device)
        self.dms_bbit_pack(n, minhash, k, bits, out)
        return out

    def jaccard_bbit(self, a, b, k, bits):
        torch = self._torch
        out = torch.empty(a.shape[0], dtype=torch.float64, device=a.device)
        self.dms_jaccard_est_bbit(a.shape[0], a, b, k, bits, out)
        return out

    def unary_map(self, minhash, bits):
        """(int32 [n, k] coordinates, common value 1/sqrt(k))."""
        torch = self._torch
        n, k = minhash.shape
        out = torch.empty((n, k), dtype=torch.int32, device=minhash.device)
        scale = self.dms_unary_map(n, minhash, k, bits, out)
        return out, scale

    def hamming_topk(self, db, queries, topk):
        torch = self._torch
        nq, words = queries.shape
        ids = torch.empty((nq, topk), dtype=torch.int64, device=db.device)
        dist = torch.empty((nq, topk), dtype=torch.int32, device=db.device)
        self.dms_hamming_topk(db, db.shape[0], words, queries, nq, topk, ids, dist)
        return ids, dist


class LshIndex:
    """Weight-class (L,K) LSH index over a CSR batch of sets (dms_index_*).
    The index reads the given device tensors during queries and keeps them."""

    def __init__(self, ctx: Context, row_ptr, idx, w, L: int, K: int):
        self.ctx, self._keep = ctx, (row_ptr, idx, w)
        self.n = row_ptr.numel() - 1
        self._h = ctypes.c_void_p()
        ctx._stream()
        ctx._check(lib().dms_index_build(ctx._h, self.n, _ptr(row_ptr), _ptr(idx), _ptr(w), L, K,
                                         ctypes.byref(self._h)), "dms_index_build")
        ctx._dependents.add(self)

    def sets(self):
        """(class int32 [n], status int8 [n]) of the indexed sets."""
        torch = self.ctx._torch
        dev = self._keep[0].device
        cls = torch.empty(self.n, dtype=torch.int32, device=dev)
        st = torch.empty(self.n, dtype=torch.int8, device=dev)
        self.ctx._check(lib().dms_index_sets(self._h, _ptr(cls), _ptr(st)), "dms_index_sets")
        return cls, st

    def query(self, q_row_ptr, q_idx, q_w, j1: float, topn: int):
        torch = self.ctx._torch
        nq = q_row_ptr.numel() - 1
        dev = q_row_ptr.device
        out = dict(ids=torch.empty((nq, topn), dtype=torch.int64, device=dev),
                   j=torch.empty((nq, topn), dtype=torch.float64, device=dev),
                   count=torch.empty(nq, dtype=torch.int32, device=dev),
                   candidates=torch.empty(nq, dtype=torch.int32, device=dev),
                   status=torch.empty(nq, dtype=torch.int8, device=dev))
        self.ctx._stream()
        self.ctx._check(lib().dms_index_query(self._h, nq, _ptr(q_row_ptr), _ptr(q_idx), _ptr(q_w), float(j1),
                                              topn, _ptr(out["ids"]), _ptr(out["j"]), _ptr(out["count"]),
                                              _ptr(out["candidates"]), _ptr(out["status"])), "dms_index_query")
        return out

    def close(self):
        if self._h:
            lib().dms_index_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SketchDB:
    """Device-resident database of 1-bit sketches that records their provenance
    (dms_db_*); appends and searches check it."""

    def __init__(self, ctx: Context, k: int, capacity: int):
        self.ctx, self.k = ctx, k
        self.words = (k + 63) // 64
        self._h = ctypes.c_void_p()
        self._check(lib().dms_db_create(ctx._h, k, capacity, ctypes.byref(self._h)), "dms_db_create")
        ctx._dependents.add(self)

    def _check(self, st, what):
        if st != DMS_OK:
            raise DMSError(f"{what}: {lib().dms_status_str(st).decode()}", st)

    def info(self):
        """(SketchInfo, rows held, device address of the rows)."""
        info, n, rows = SketchInfo(), ctypes.c_int64(0), ctypes.c_void_p()
        self._check(lib().dms_db_info(self._h, ctypes.byref(info), ctypes.byref(n), ctypes.byref(rows)),
                    "dms_db_info")
        return info, n.value, rows.value

    def append_sets(self, row_ptr, idx, w):
        """Sketch a CSR batch (device tensors) into the next rows; returns
        (first row, int8 status tensor)."""
        torch = self.ctx._torch
        n = row_ptr.numel() - 1
        st = torch.empty(n, dtype=torch.int8, device=row_ptr.device)
        first = ctypes.c_int64(0)
        self.ctx._stream()
        self._check(lib().dms_db_append_sets(self._h, n, _ptr(row_ptr), _ptr(idx), _ptr(w), _ptr(st),
                                             ctypes.byref(first)), "dms_db_append_sets")
        return first.value, st

    def append_bits(self, bits, info: SketchInfo):
        """Copy rows of 1-bit sketches (uint64 words as int64, device or host)
        made under `info`; returns the first row."""
        first = ctypes.c_int64(0)
        self.ctx._stream()
        self._check(lib().dms_db_append_bits(self._h, bits.shape[0], _ptr(bits), ctypes.byref(info),
                                             ctypes.byref(first)), "dms_db_append_bits")
        return first.value

    def topk(self, queries, topk: int, info: SketchInfo):
        torch = self.ctx._torch
        nq = queries.shape[0]
        ids = torch.empty((nq, topk), dtype=torch.int64, device=queries.device)
        dist = torch.empty((nq, topk), dtype=torch.int32, device=queries.device)
        self.ctx._stream()
        self._check(lib().dms_db_topk(self._h, _ptr(queries), nq, ctypes.byref(info), topk, _ptr(ids),
                                      _ptr(dist)), "dms_db_topk")
        return ids, dist

    def close(self):
        if self._h:
            lib().dms_db_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching serving loop (dms_server_*) over a SketchDB of 1-bit
    k = 1024 sketches made under the context's provenance."""

    def __init__(self, ctx: Context, db: SketchDB, topk=10, max_batch=256, max_inflight=4,
                 max_batch_nnz=1 << 20, max_set_nnz=4096, split_nnz=128):
        import numpy as np
        self.ctx, self.db, self.topk = ctx, db, topk
        cfg = ServerConfig(max_batch, max_inflight, max_batch_nnz, max_set_nnz, 16, topk, split_nnz)
        self._h = ctypes.c_void_p()
        st = lib().dms_server_create(ctx._h, ctypes.byref(cfg), db._h, ctypes.byref(self._h))
        if st != DMS_OK:
            raise DMSError(f"dms_server_create: {lib().dms_status_str(st).decode()}", st)
        ctx._dependents.add(self)
        self._np = np

    def close(self):
        if self._h:
            lib().dms_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def replay(self, arrival_s, kind, k, row_ptr, idx, w):
        """Serve a trace; returns dict of per-request results and summary stats."""
        np = self._np
        n = len(arrival_s)
        arrival_s = np.ascontiguousarray(arrival_s, np.float64)
        kind = np.ascontiguousarray(kind, np.int32)
        k = np.ascontiguousarray(k, np.int32)
        row_ptr = np.ascontiguousarray(row_ptr, np.int64)
        idx = np.ascontiguousarray(idx, np.int32)
        w = np.ascontiguousarray(w, np.float64)
        off = np.zeros(n, np.int64)
        if n:
            off[1:] = np.cumsum(k[:-1].astype(np.int64))
        sk = np.zeros(int(k.astype(np.int64).sum()), np.uint32)
        status = np.zeros(n, np.int8)
        ids = np.full((n, self.topk), -2, np.int64)
        dist = np.full((n, self.topk), -2, np.int32)
        lat = np.zeros(n, np.float64)
        stats = np.zeros(7, np.float64)
        st = lib().dms_server_replay(self._h, n, _ptr(arrival_s), _ptr(kind), _ptr(k), _ptr(row_ptr),
                                     _ptr(idx), _ptr(w), _ptr(off), _ptr(sk), _ptr(status), _ptr(ids),
                                     _ptr(dist), _ptr(lat), _ptr(stats))
        if st != DMS_OK:
            raise DMSError(f"dms_server_replay: {lib().dms_status_str(st).decode()}")
        sketches = [sk[off[i]:off[i] + k[i]] for i in range(n)]
        return dict(sketch=sketches, status=status, ids=ids, dist=dist, latency=lat,
                    stats=dict(req_per_s=stats[0], p50_s=stats[1], p99_s=stats[2], max_s=stats[3],
                               batches=int(stats[4]), mean_batch=stats[5], elapsed_s=stats[6]))

    def submit(self, kind, k, idx, w):
        """Submit one request (host arrays); returns its id."""
        np = self._np
        idx = np.ascontiguousarray(idx, np.int32)
        w = np.ascontiguousarray(w, np.float64)
        rid = ctypes.c_int64(0)
        st = lib().dms_server_submit(self._h, int(kind), int(k), len(idx), _ptr(idx), _ptr(w),
                                     ctypes.byref(rid))
        if st != DMS_OK:
            raise DMSError(f"dms_server_submit: {lib().dms_status_str(st).decode()}")
        return rid.value

    def poll(self, wait_ms=0, max_out=1024):
        """Answers finished so far: list of dicts (id, status, sketch, and for
        search requests ids and dist), in completion order."""
        np = self._np
        out_id = np.zeros(max_out, np.int64)
        status = np.zeros(max_out, np.int8)
        sk = np.zeros((max_out, 1024), np.uint32)
        ids = np.full((max_out, self.topk), -2, np.int64)
        dist = np.full((max_out, self.topk), -2, np.int32)
        lat = np.zeros(max_out, np.float64)
        n = ctypes.c_int64(0)
        st = lib().dms_server_poll(self._h, int(wait_ms), max_out, _ptr(out_id), _ptr(status), _ptr(sk),
                                   _ptr(ids), _ptr(dist), _ptr(lat), ctypes.byref(n))
        if st != DMS_OK:
            raise DMSError(f"dms_server_poll: {lib().dms_status_str(st).decode()}")
        return [dict(id=int(out_id[i]), status=int(status[i]), sketch=sk[i], ids=ids[i], dist=dist[i],
                     latency=float(lat[i])) for i in range(n.value)]


def to_device(row_ptr, idx, w, device="cuda"):
    """Copy a host CSR batch (numpy) to device tensors."""
    import torch
    return (torch.from_numpy(row_ptr).to(device), torch.from_numpy(idx).to(device),
            torch.from_numpy(w).to(device))
