"""DartMinHash CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path (the HIP library and its
binding) never touches it.

Layout:

* constants of the method, derived here from their mathematical definitions
  with exact arithmetic (``fractions``/``decimal``) and IEEE binary64 division;
* a ctypes wrapper around ``dms_oracle.c`` (the single-threaded DartHash,
  DartMinHash and LSH loops);
* the estimators, the b-bit fingerprints and their packing, the unary
  feature map and the Hamming top-k scan, written directly with numpy.

Paper references are to Christiani, "DartMinHash: Fast Sketching for Weighted
Sets" (arXiv 2005.11547).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from decimal import Decimal, getcontext
from fractions import Fraction
from functools import lru_cache
import math
from math import factorial

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dms_oracle.c")
LIB = os.path.join(HERE, "libdms_oracle.so")

TABLE = 1024
NPOIS = 20
STATUS = {"ok": 0, "empty": 1, "range": 2, "invalid": 3}
SCHED_PLUS_ONE = 0   # phi = 1, 2, 3, ... (proof of Theorem 1)
SCHED_DOUBLE = 1     # phi = phi0, 2 phi0, 4 phi0, ...
HASH_MIX = 0         # SplitMix64 output function keyed by the six keys
HASH_TAB = 1         # simple tabulation, tables from the Mersenne Twister
TAB_WORDS = 8 * 256
MASK64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# Constants
# --------------------------------------------------------------------------
def t_of_k(k: int) -> int:
    """t = ceil(k ln k) + k (proof of Theorem 1), with a 60-digit logarithm."""
    if k < 1:
        raise ValueError("k must be positive")
    getcontext().prec = 60
    v = Decimal(k) * Decimal(k).ln()
    c = int(v.to_integral_value(rounding="ROUND_CEILING"))
    return c + k


@lru_cache(maxsize=None)
def poisson_thresholds() -> tuple:
    """C[n] = floor(2^64 * P[Poisson(1) <= n]) for n = 0..19, exactly.

    P[Poi(1) <= n] = e^-1 * sum_{m<=n} 1/m!.  e^-1 is bracketed by two partial
    sums of its alternating series; the floor must agree at both ends.
    """
    lo = sum(Fraction((-1) ** m, factorial(m)) for m in range(0, 42))  # odd last term: below
    hi = sum(Fraction((-1) ** m, factorial(m)) for m in range(0, 41))  # even last term: above
    assert lo < hi
    out = []
    for n in range(NPOIS):
        s = sum(Fraction(1, factorial(m)) for m in range(n + 1))
        a = (lo * s * 2 ** 64).__floor__()
        b = (hi * s * 2 ** 64).__floor__()
        assert a == b, n
        out.append(int(a))
    return tuple(out)


def mt19937_64(seed: int, n: int) -> list[int]:
    """First n outputs of MT19937-64 (Matsumoto and Nishimura), seeded the
    standard way (init_genrand64)."""
    NN, MM = 312, 156
    MATRIX_A = 0xB5026F5AA96619E9
    UM, LM = 0xFFFFFFFF80000000, 0x7FFFFFFF
    mt = [0] * NN
    mt[0] = seed & MASK64
    for i in range(1, NN):
        mt[i] = (6364136223846793005 * (mt[i - 1] ^ (mt[i - 1] >> 62)) + i) & MASK64
    idx = NN
    out = []
    for _ in range(n):
        if idx >= NN:
            for i in range(NN):
                x = (mt[i] & UM) | (mt[(i + 1) % NN] & LM)
                xa = x >> 1
                if x & 1:
                    xa ^= MATRIX_A
                mt[i] = mt[(i + MM) % NN] ^ xa
            idx = 0
        x = mt[idx]
        idx += 1
        x ^= (x >> 29) & 0x5555555555555555
        x ^= (x << 17) & 0x71D67FFFEDA60000
        x ^= (x << 37) & 0xFFF7EEE000000000
        x ^= x >> 43
        out.append(x & MASK64)
    return out


@lru_cache(maxsize=4096)
def _keys(seed: int) -> tuple:
    return tuple(mt19937_64(seed, 6))


def hash_keys(seed: int) -> dict:
    """The six hash keys: the first six MT19937-64 outputs for the seed."""
    k = _keys(seed)
    return dict(key_r=k[0], key_a=k[1], key_u=k[2], key_v=k[3], key_s=k[4], key_l=k[5])


def tables(t: int):
    """W[nu] = RN(RN(2^nu - 1)/t), R[rho] = RN(2^rho - 1), u = RN(1/t): the lower
    corners of the weight and rank regions (Section 2) and the unit column width."""
    W = [float(2 ** nu - 1) / float(t) for nu in range(TABLE)]
    R = [float(2 ** rho - 1) for rho in range(TABLE)]
    return W, R, 1.0 / float(t)


# --------------------------------------------------------------------------
# ctypes
# --------------------------------------------------------------------------
class Params(ctypes.Structure):
    _fields_ = [
        ("key_r", ctypes.c_uint64), ("key_a", ctypes.c_uint64), ("key_u", ctypes.c_uint64),
        ("key_v", ctypes.c_uint64), ("key_s", ctypes.c_uint64), ("key_l", ctypes.c_uint64),
        ("pois", ctypes.c_uint64 * NPOIS),
        ("W", ctypes.c_double * TABLE),
        ("R", ctypes.c_double * TABLE),
        ("u", ctypes.c_double),
        ("t", ctypes.c_uint32),
        ("phi0", ctypes.c_double),
        ("schedule", ctypes.c_int32),
        ("phi_max", ctypes.c_double),
        ("hash", ctypes.c_int32),
        ("tab", ctypes.c_uint64 * TAB_WORDS),
        ("validate", ctypes.c_int32),
    ]


class Counters(ctypes.Structure):
    _fields_ = [("regions", ctypes.c_int64), ("areas", ctypes.c_int64),
                ("generated", ctypes.c_int64), ("rank_pass", ctypes.c_int64),
                ("accepted", ctypes.c_int64), ("rank_new", ctypes.c_int64),
                ("accepted_new", ctypes.c_int64)]


DART_DTYPE = np.dtype([("i", "<u4"), ("nu", "<u2"), ("rho", "<u2"), ("w", "<u4"), ("r", "<u4"),
                       ("j", "<u4"), ("pad", "<u4"), ("rank", "<f8"), ("weight", "<f8"),
                       ("s", "<u8")])
COUNTER_DTYPE = np.dtype([("regions", "<i8"), ("areas", "<i8"), ("generated", "<i8"),
                          ("rank_pass", "<i8"), ("accepted", "<i8"), ("rank_new", "<i8"),
                          ("accepted_new", "<i8")])


SAN_LIB = os.path.join(HERE, "libdms_oracle_san.so")


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile dms_oracle.c with strict IEEE binary64 semantics.  With
    `sanitize`, a second build of the same source under AddressSanitizer and
    UndefinedBehaviorSanitizer (loaded only by the sanitizer test)."""
    out = SAN_LIB if sanitize else LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        tmp = out + ".tmp%d" % os.getpid()
        extra = (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                  "-fno-omit-frame-pointer", "-g"] if sanitize else [])
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fno-finite-math-only", "-mfpmath=sse", "-msse2", "-fPIC",
                               "-shared", "-Wall"] + extra + ["-o", tmp, SRC, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        # DMS_ORACLE_LIB selects another build of the same source (the sanitizer build)
        L = ctypes.CDLL(os.environ.get("DMS_ORACLE_LIB") or build())
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.dmso_mix64.argtypes = [ctypes.c_uint64]
        L.dmso_mix64.restype = ctypes.c_uint64
        L.dmso_darthash.argtypes = [P(Params), ctypes.c_int64, vp, vp, ctypes.c_double, vp,
                                    ctypes.c_int64, P(ctypes.c_int64), vp]
        L.dmso_minhash_set.argtypes = [P(Params), ctypes.c_int32, ctypes.c_int64, vp, vp, vp, vp,
                                       P(ctypes.c_double), vp]
        L.dmso_sketch_csr.argtypes = [P(Params), ctypes.c_int64, vp, vp, vp, ctypes.c_int32,
                                      vp, vp, vp, vp, vp, vp, vp]
        L.dmso_lsh_set.argtypes = [P(Params), ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                   vp, vp, vp, vp, vp, P(ctypes.c_double), vp]
        L.dmso_lsh_csr.argtypes = [P(Params), ctypes.c_int64, vp, vp, vp, ctypes.c_int32,
                                   ctypes.c_int32, vp, vp, vp]
        L.dmso_bottomk_set.argtypes = [P(Params), ctypes.c_int32, ctypes.c_int64, vp, vp, vp, vp, vp, vp]
        L.dmso_bottomk_csr.argtypes = [P(Params), ctypes.c_int64, vp, vp, vp, ctypes.c_int32, vp, vp, vp,
                                       vp]
        for f in ("dmso_bottomk_set", "dmso_bottomk_csr"):
            getattr(L, f).restype = ctypes.c_int
        for f in ("dmso_darthash", "dmso_minhash_set", "dmso_sketch_csr", "dmso_lsh_set",
                  "dmso_lsh_csr"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def mix64(z: int) -> int:
    return int(lib().dmso_mix64(z & MASK64))


@lru_cache(maxsize=8)
def tab_tables(seed: int) -> tuple:
    """Simple-tabulation tables: the MT19937-64 outputs that follow the six
    keys; table b (for byte b of the hashed word) is outputs 7 + 256 b onwards."""
    return tuple(mt19937_64(seed, 6 + TAB_WORDS)[6:])


def make_params(seed: int, t: int, phi0: float = 1.0, schedule: int = SCHED_PLUS_ONE,
                phi_max: float = 2.0 ** 20, hash: int = HASH_MIX, validate: bool = False) -> Params:
    p = Params()
    p.hash = hash
    p.validate = 1 if validate else 0
    if hash == HASH_TAB:
        for i, v in enumerate(tab_tables(seed)):
            p.tab[i] = v
    for name, v in hash_keys(seed).items():
        setattr(p, name, v)
    for n, c in enumerate(poisson_thresholds()):
        p.pois[n] = c
    W, R, u = tables(t)
    for i in range(TABLE):
        p.W[i] = W[i]
        p.R[i] = R[i]
    p.u = u
    p.t = t
    p.phi0 = phi0
    p.schedule = schedule
    p.phi_max = phi_max
    return p


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _csr(row_ptr, idx, w):
    return (np.ascontiguousarray(row_ptr, dtype=np.int64),
            np.ascontiguousarray(idx, dtype=np.int32),
            np.ascontiguousarray(w, dtype=np.float64))


# --------------------------------------------------------------------------
# Method
# --------------------------------------------------------------------------
def darthash(idx, w, tau: float, t: int, seed: int, hash: int = HASH_MIX):
    """DartHash_t(x, phi) with tau = phi/||x||_1 given explicitly (Algorithm 1).
    Returns (status, structured array of darts, counters dict)."""
    P = make_params(seed, t, hash=hash)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = ctypes.c_int64(0)
    cnt = Counters()
    st = lib().dmso_darthash(ctypes.byref(P), len(idx), _ptr(idx), _ptr(w), tau, None, 0,
                             ctypes.byref(n), ctypes.byref(cnt))
    out = np.zeros(n.value, dtype=DART_DTYPE)
    st = lib().dmso_darthash(ctypes.byref(P), len(idx), _ptr(idx), _ptr(w), tau, _ptr(out),
                             n.value, ctypes.byref(n), ctypes.byref(cnt))
    return st, out, {f: getattr(cnt, f) for f, _ in Counters._fields_}


def minhash_set(idx, w, k: int, seed: int, t: int | None = None, phi0: float = 1.0,
                schedule: int = SCHED_PLUS_ONE, hash: int = HASH_MIX):
    """DartMinHash of one set (Theorem 1).  Returns (status, s[k] uint64,
    rank[k] float64, phi_final, counters)."""
    t = t_of_k(k) if t is None else t
    P = make_params(seed, t, phi0, schedule, hash=hash)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    s = np.zeros(k, dtype=np.uint64)
    r = np.zeros(k, dtype=np.float64)
    phi = ctypes.c_double(0.0)
    cnt = (Counters * 2)()
    st = lib().dmso_minhash_set(ctypes.byref(P), k, len(idx), _ptr(idx), _ptr(w), _ptr(s),
                                _ptr(r), ctypes.byref(phi), cnt)
    return st, s, r, phi.value, {f: getattr(cnt[0], f) for f, _ in Counters._fields_}


def sketch_csr(row_ptr, idx, w, k: int, seed: int, t: int | None = None, phi0: float = 1.0,
               schedule: int = SCHED_PLUS_ONE, full: bool = False, hash: int = HASH_MIX,
               validate: bool = False):
    """DartMinHash of every row of a CSR matrix.

    Returns dict with u32 [n,k], bits [n, ceil(k/64)] (uint64), status [n] (int8),
    and with ``full`` also s [n,k], rank [n,k], phi [n], counters [n] (every pass
    summed) and counters_last [n] (the last pass).  With ``validate`` a row
    listing an id twice gets status INVALID."""
    t = t_of_k(k) if t is None else t
    P = make_params(seed, t, phi0, schedule, hash=hash, validate=validate)
    row_ptr, idx, w = _csr(row_ptr, idx, w)
    n = len(row_ptr) - 1
    words = (k + 63) // 64
    u32 = np.zeros((n, k), dtype=np.uint32)
    bits = np.zeros((n, words), dtype=np.uint64)
    status = np.zeros(n, dtype=np.int8)
    s = np.zeros((n, k), dtype=np.uint64) if full else None
    rk = np.zeros((n, k), dtype=np.float64) if full else None
    phi = np.zeros(n, dtype=np.float64) if full else None
    cnt = np.zeros((n, 2), dtype=COUNTER_DTYPE) if full else None
    st = lib().dmso_sketch_csr(ctypes.byref(P), n, _ptr(row_ptr), _ptr(idx), _ptr(w), k,
                               _ptr(u32), _ptr(bits), _ptr(status), _ptr(s), _ptr(rk),
                               _ptr(phi), _ptr(cnt))
    if st != 0:
        raise MemoryError("oracle out of memory")
    out = dict(u32=u32, bits=bits, status=status)
    if full:
        out.update(s=s, rank=rk, phi=phi, counters=cnt[:, 0].copy(), counters_last=cnt[:, 1].copy())
    return out


def lsh_set(idx, w, L: int, K: int, seed: int, phi0: float = 1.0,
            schedule: int = SCHED_PLUS_ONE, hash: int = HASH_MIX):
    """(L,K) LSH values of one set.  Returns (status, keys[L], s[L,K], rank[L,K], phi)."""
    P = make_params(seed, L * K, phi0, schedule, hash=hash)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    keys = np.zeros(L, dtype=np.uint64)
    s = np.zeros((L, K), dtype=np.uint64)
    r = np.zeros((L, K), dtype=np.float64)
    phi = ctypes.c_double(0.0)
    st = lib().dmso_lsh_set(ctypes.byref(P), L, K, len(idx), _ptr(idx), _ptr(w), _ptr(keys),
                            _ptr(s), _ptr(r), ctypes.byref(phi), None)
    return st, keys, s, r, phi.value


def lsh_csr(row_ptr, idx, w, L: int, K: int, seed: int, phi0: float = 1.0,
            schedule: int = SCHED_PLUS_ONE, hash: int = HASH_MIX, counters: bool = False,
            validate: bool = False):
    """(L,K) LSH keys of every row: dict keys [n,L] uint64, status [n] int8, and
    with ``counters`` the enumeration counts [n,2] (every pass summed, last pass)."""
    P = make_params(seed, L * K, phi0, schedule, hash=hash, validate=validate)
    row_ptr, idx, w = _csr(row_ptr, idx, w)
    n = len(row_ptr) - 1
    keys = np.zeros((n, L), dtype=np.uint64)
    status = np.zeros(n, dtype=np.int8)
    cnt = np.zeros((n, 2), dtype=COUNTER_DTYPE) if counters else None
    st = lib().dmso_lsh_csr(ctypes.byref(P), n, _ptr(row_ptr), _ptr(idx), _ptr(w), L, K,
                            _ptr(keys), _ptr(status), _ptr(cnt))
    if st != 0:
        raise MemoryError("oracle out of memory")
    out = dict(keys=keys, status=status)
    if counters:
        out["counters"] = cnt
    return out


def bottomk_set(idx, w, k: int, seed: int, phi0: float = 1.0, schedule: int = SCHED_PLUS_ONE,
                hash: int = HASH_MIX):
    """Bottom-k sketch of one set (Section 3): the k first darts hitting x, with
    DartHash at t = k.  Returns (status, s[k] uint64, rank[k] float64, phi)."""
    P = make_params(seed, k, phi0, schedule, hash=hash)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    s = np.zeros(k, dtype=np.uint64)
    r = np.zeros(k, dtype=np.float64)
    phi = ctypes.c_double(0.0)
    st = lib().dmso_bottomk_set(ctypes.byref(P), k, len(idx), _ptr(idx), _ptr(w), _ptr(s), _ptr(r),
                                ctypes.byref(phi), None)
    return st, s, r, phi.value


def bottomk_csr(row_ptr, idx, w, k: int, seed: int, phi0: float = 1.0,
                schedule: int = SCHED_PLUS_ONE, hash: int = HASH_MIX, counters: bool = False,
                validate: bool = False):
    """Bottom-k sketches of every row: dict s [n,k] uint64, rank [n,k] float64,
    u32 [n,k] (low 32 bits of s), status [n] int8, and with ``counters`` the
    enumeration counts [n,2] (every pass summed, last pass)."""
    rp, idx, w = _csr(row_ptr, idx, w)
    n = len(rp) - 1
    P = make_params(seed, k, phi0, schedule, hash=hash, validate=validate)
    s = np.zeros((n, k), dtype=np.uint64)
    r = np.zeros((n, k), dtype=np.float64)
    st = np.zeros(n, dtype=np.int8)
    cnt = np.zeros((n, 2), dtype=COUNTER_DTYPE) if counters else None
    rc = lib().dmso_bottomk_csr(ctypes.byref(P), n, _ptr(rp), _ptr(idx), _ptr(w), k, _ptr(s), _ptr(r),
                                _ptr(st), _ptr(cnt))
    if rc != 0:
        raise MemoryError("dmso_bottomk_csr")
    out = {"s": s, "rank": r, "u32": (s & np.uint64(0xFFFFFFFF)).astype(np.uint32), "status": st}
    if counters:
        out["counters"] = cnt
    return out


def jaccard_est_bottomk(rank_a, s_a, rank_b, s_b):
    """Bottom-k estimate (the bottom-k sketch estimator of the paper's reference
    for it): among the k smallest darts of the union of the two sketches, the
    fraction that lies in both.  Darts are (rank, s) pairs; rows are pairs."""
    rank_a, rank_b = np.asarray(rank_a, np.float64), np.asarray(rank_b, np.float64)
    s_a, s_b = np.asarray(s_a, np.uint64), np.asarray(s_b, np.uint64)
    n, k = rank_a.shape
    out = np.zeros(n, dtype=np.float64)
    for p in range(n):
        A = set(zip(rank_a[p].tolist(), s_a[p].tolist()))
        B = set(zip(rank_b[p].tolist(), s_b[p].tolist()))
        union = sorted(A | B)[:k]
        out[p] = sum(1 for d in union if d in A and d in B) / k
    return out


# --------------------------------------------------------------------------
# Estimators and search (Section 1.1)
# --------------------------------------------------------------------------
def jaccard_est_u32(a, b):
    """J-hat = (1/k) * #{j : h_j(x) = h_j(y)} for each row pair."""
    a = np.asarray(a, dtype=np.uint32)
    b = np.asarray(b, dtype=np.uint32)
    return (a == b).sum(axis=-1) / a.shape[-1]


def popcount64(v):
    v = np.asarray(v, dtype=np.uint64)
    out = np.zeros(v.shape, dtype=np.int64)
    for sh in range(0, 64, 8):
        byte = ((v >> np.uint64(sh)) & np.uint64(0xFF)).astype(np.int64)
        out += _POP8[byte]
    return out


_POP8 = np.array([bin(i).count("1") for i in range(256)], dtype=np.int64)


def jaccard_est_1bit(a, b, k: int):
    """1-bit sketches: each bit agrees with probability (1+J)/2, so
    J-hat = 1 - 2 * (#disagreeing bits)/k (unclamped)."""
    d = popcount64(np.bitwise_xor(np.asarray(a, np.uint64), np.asarray(b, np.uint64))).sum(axis=-1)
    return 1.0 - 2.0 * d / k


def hamming_topk(db_bits, q_bits, topk: int):
    """For every query row, the topk database rows of smallest Hamming distance,
    ties broken by the smaller row id.  Returns (ids [nq, topk] int64,
    dist [nq, topk] int32)."""
    db = np.asarray(db_bits, dtype=np.uint64)
    q = np.asarray(q_bits, dtype=np.uint64)
    ids = np.zeros((q.shape[0], topk), dtype=np.int64)
    dist = np.zeros((q.shape[0], topk), dtype=np.int32)
    for qi in range(q.shape[0]):
        d = popcount64(np.bitwise_xor(db, q[qi][None, :])).sum(axis=1)
        order = np.lexsort((np.arange(db.shape[0]), d))[:topk]
        ids[qi, :len(order)] = order
        dist[qi, :len(order)] = d[order]
    return ids, dist


# --------------------------------------------------------------------------
# b-bit fingerprints and the unary feature map (Section 1.1)
# --------------------------------------------------------------------------
def bbit_values(minhash_u32, b: int):
    """The b-bit fingerprint of each minhash: its lowest b bits (bits of the
    dart-id hash s, independent of the bucket bits; b = 1 is the 1-bit sketch)."""
    v = np.asarray(minhash_u32, dtype=np.uint64)
    return v & np.uint64((1 << b) - 1)


def bbit_words(k: int, b: int) -> int:
    return (k * b + 63) // 64


def bbit_pack(minhash_u32, b: int):
    """Pack the k fingerprints of each row into ceil(k*b/64) little-endian
    uint64 words: fingerprint j occupies stream bits [j*b, j*b + b), stream
    bit p is bit p % 64 of word p // 64, unused high bits are zero."""
    v = bbit_values(minhash_u32, b)
    n, k = v.shape
    words = bbit_words(k, b)
    stream = np.zeros((n, words * 64), dtype=np.uint8)
    for i in range(b):  # bit i of every fingerprint
        stream[:, np.arange(k) * b + i] = ((v >> np.uint64(i)) & np.uint64(1)).astype(np.uint8)
    packed = np.packbits(stream, axis=1, bitorder="little")  # byte q holds stream bits 8q..8q+7
    return packed.view("<u8").reshape(n, words).astype(np.uint64)


def bbit_unpack(words, k: int, b: int):
    """Inverse of bbit_pack: the k fingerprints of each row."""
    w = np.ascontiguousarray(np.asarray(words, dtype="<u8"))
    n = w.shape[0]
    stream = np.unpackbits(w.view(np.uint8).reshape(n, -1), axis=1, bitorder="little")
    out = np.zeros((n, k), dtype=np.uint64)
    for i in range(b):
        out |= stream[:, np.arange(k) * b + i].astype(np.uint64) << np.uint64(i)
    return out


def jaccard_est_bbit(a_words, b_words, k: int, b: int):
    """b-bit sketches: fingerprints of one bucket agree with probability
    J + (1 - J) 2^-b, so J-hat = (m/k - 2^-b) / (1 - 2^-b) with m the number of
    agreeing fingerprints (unclamped)."""
    m = (bbit_unpack(a_words, k, b) == bbit_unpack(b_words, k, b)).sum(axis=-1)
    c = 2.0 ** -b
    return (m / k - c) / (1.0 - c)


def unary_map(minhash_u32, b: int):
    """Linearisation of the Jaccard kernel: minhash j with fingerprint v maps to
    the unit vector of coordinate j*2^b + v, and the row is scaled by 1/sqrt(k),
    so <u(x), u(y)> = (agreeing fingerprints)/k.  Returns (indices [n, k] int32,
    ascending within a row, and the common value 1/sqrt(k))."""
    v = bbit_values(minhash_u32, b).astype(np.int64)
    n, k = v.shape
    idx = (np.arange(k, dtype=np.int64) << b)[None, :] + v
    return idx.astype(np.int32), 1.0 / math.sqrt(k)


# --------------------------------------------------------------------------
# Weight classes and the LSH index (Section 3, approximate near neighbours)
# --------------------------------------------------------------------------
def seq_sum(w) -> float:
    """||x||_1 summed left to right in binary64 (the order both sides use)."""
    s = 0.0
    for v in np.asarray(w, dtype=np.float64).tolist():
        if v > 0.0:
            s += v
    return s


def weight_class(w) -> int:
    """c with ||x||_1 in [2^c, 2^(c+1)) (the paper's weight classes)."""
    m, e = math.frexp(seq_sum(w))
    return e - 1


def row_ok_for_index(idx, w) -> bool:
    """Index rows must list strictly increasing ids with finite weights >= 0
    and some positive weight, inside the supported range."""
    idx = np.asarray(idx).astype(np.int64) & 0xFFFFFFFF  # ids are read as uint32
    w = np.asarray(w, dtype=np.float64)
    if len(idx) == 0 or np.any(np.diff(idx) <= 0):
        return False
    if not np.all(np.isfinite(w)) or np.any(w < 0) or not np.any(w > 0):
        return False
    return 2.0 ** -768 <= w.max() <= 2.0 ** 768


def weighted_jaccard_merge(ia, wa, ib, wb) -> float:
    """J(x, y) = sum min / sum max over the union of the two (id-sorted) rows,
    both sums taken in ascending id order."""
    ia = (np.asarray(ia).astype(np.int64) & 0xFFFFFFFF).tolist()  # ids are read as uint32
    ib = (np.asarray(ib).astype(np.int64) & 0xFFFFFFFF).tolist()
    wa, wb = np.asarray(wa, np.float64).tolist(), np.asarray(wb, np.float64).tolist()
    i = j = 0
    smin = smax = 0.0
    while i < len(ia) or j < len(ib):
        if j >= len(ib) or (i < len(ia) and ia[i] < ib[j]):
            smax += wa[i]
            i += 1
        elif i >= len(ia) or ib[j] < ia[i]:
            smax += wb[j]
            j += 1
        else:
            smin += min(wa[i], wb[j])
            smax += max(wa[i], wb[j])
            i += 1
            j += 1
    return smin / smax if smax > 0 else 0.0


def class_span(j1: float) -> int:
    """Classes searched on each side of the query's: J >= j1 bounds the norm
    ratio by 1/j1, i.e. ceil(log2(1/j1)) classes, plus one for the floors."""
    return int(math.ceil(math.log2(1.0 / j1))) + 1


def lsh_index_build(row_ptr, idx, w, L: int, K: int, seed: int, hash: int = HASH_MIX):
    """The index: per set its class and status, and per table l a dict from
    (class, key of the normalised set) to the ascending ids of the sets there."""
    rp, idx, w = _csr(row_ptr, idx, w)
    n = len(rp) - 1
    cls = np.zeros(n, dtype=np.int32)
    ok = np.zeros(n, dtype=bool)
    rows = []
    for q in range(n):
        ii, ww = idx[rp[q]:rp[q + 1]], w[rp[q]:rp[q + 1]]
        ok[q] = row_ok_for_index(ii, ww)
        if ok[q]:
            cls[q] = weight_class(ww)
            rows.append((ii, np.ldexp(ww, -int(cls[q]))))
        else:
            rows.append((ii[:0], ww[:0]))
    nrp = np.zeros(n + 1, dtype=np.int64)
    nrp[1:] = np.cumsum([len(r[0]) for r in rows])
    nidx = np.concatenate([r[0] for r in rows]) if n else np.zeros(0, np.int32)
    nw = np.concatenate([r[1] for r in rows]) if n else np.zeros(0)
    keys = lsh_csr(nrp, nidx, nw, L, K, seed, hash=hash)["keys"]
    tables = [dict() for _ in range(L)]
    for q in range(n):
        if not ok[q]:
            continue
        for l in range(L):
            tables[l].setdefault((int(cls[q]), int(keys[q, l])), []).append(q)
    return {"class": cls, "ok": ok, "keys": keys, "tables": tables, "L": L, "K": K, "seed": seed, "hash": hash,
            "rows": (rp, idx, w)}


def lsh_index_query(index, q_idx, q_w, j1: float, topn: int):
    """Near neighbours of one query set: for every class within class_span(j1)
    of the query's, the query scaled into that class is hashed to its L keys;
    the union of the matching buckets is verified with the exact weighted
    Jaccard.  Returns (candidates, [(J, id), ...] of J >= j1, by J descending
    then id ascending, at most topn)."""
    if not row_ok_for_index(q_idx, q_w):
        return 0, []
    rp, idx, w = index["rows"]
    cq = weight_class(q_w)
    span = class_span(j1)
    cands = set()
    for c in range(cq - span, cq + span + 1):
        qs = np.ldexp(np.asarray(q_w, np.float64), -c)
        st, keys, _, _, _ = lsh_set(q_idx, qs, index["L"], index["K"], index["seed"], hash=index["hash"])
        if st != 0:
            continue
        for l in range(index["L"]):
            cands.update(index["tables"][l].get((c, int(keys[l])), []))
    res = []
    for x in sorted(cands):
        J = weighted_jaccard_merge(q_idx, q_w, idx[rp[x]:rp[x + 1]], w[rp[x]:rp[x + 1]])
        if J >= j1:
            res.append((J, x))
    res.sort(key=lambda t: (-t[0], t[1]))
    return len(cands), res[:topn]
