/*
 * dms.h -- C ABI of the DartMinHash library for AMD Instinct MI355X (gfx950).
 *
 * Christiani, "DartMinHash: Fast Sketching for Weighted Sets" (arXiv 2005.11547).
 *
 * Conventions for every call:
 *  - Weighted sets arrive as one CSR matrix: row_ptr (int64, n_sets+1 entries,
 *    non-decreasing, row_ptr[0] = 0), idx (int32 element ids, read as uint32),
 *    w (float64 weights).  A row lists the nonzeros of one set x in R^d_{>=0};
 *    zero weights are skipped, as Algorithm 1 iterates over {i : x_i > 0}.
 *  - Pointers marked "device" must be device memory of the context's GPU;
 *    the caller allocates, owns and frees every input and output buffer.  The
 *    context owns only its internal tables and scratch space.
 *  - Calls are asynchronous on the context's stream (dms_set_stream): they only
 *    enqueue work, except that (a) the first call for a value of t copies that
 *    t's specification tables to the device and waits for the copy, and (b) a
 *    call needing more scratch space than the context holds waits for the
 *    stream before replacing it.  Once an eager call of the same shape has run,
 *    dms_sketch_csr, dms_lsh_keys and dms_bottomk therefore only enqueue
 *    kernels and can be captured into a HIP graph.  Calls that say they
 *    synchronize (index build, autotune, calibration, serving) do so always.
 *    Argument errors are reported synchronously by the return value, per-set
 *    data problems by out_status.  dms_sync waits for the stream.
 *  - A context is not thread safe; use one per host thread.
 *  - Return value: DMS_OK (0) or a negative DMS_E* code; dms_last_error gives
 *    the message of the last failure on that context.
 */
#ifndef DMS_H
#define DMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dms_status;
#define DMS_OK 0
#define DMS_EINVAL (-1) /* an argument is out of range or a pointer is NULL */
#define DMS_EHIP (-2)   /* the HIP runtime reported an error */
#define DMS_ENOMEM (-3) /* the context could not allocate its scratch space */
#define DMS_ESPEC (-4)  /* a specification constant could not be derived exactly */
#define DMS_EMISMATCH (-5) /* sketches made under another specification version, hash, seed or k */

/* Per-set status codes written to out_status arrays. */
#define DMS_SET_OK 0      /* sketch computed */
#define DMS_SET_EMPTY 1   /* no positive weight: the minhash is undefined (J = 0/0) */
#define DMS_SET_RANGE 2   /* largest weight outside [2^-768, 2^768], or phi beyond its cap */
#define DMS_SET_INVALID 3 /* a negative, NaN or infinite weight; with DMS_FLAG_VALIDATE also a
                             repeated element id */
#define DMS_QUERY_OVERFLOW 4 /* dms_index_query: the query's buckets hold more than 2048 entries */

/* Engines for the sketch and LSH calls (dms_set_option DMS_OPT_ENGINE). */
#define DMS_ENGINE_FAST 0  /* flattened wave pipeline, work-stealing persistent grid */
#define DMS_ENGINE_PLAIN 1 /* one wave per set, one lane per nonzero, one launch */

/* Options (dms_set_option / dms_get_option).  None but DMS_OPT_HASH changes any
 * output: Theorem 1's output is independent of the phi schedule. */
#define DMS_OPT_ENGINE 0    /* DMS_ENGINE_* */
#define DMS_OPT_PHI0 1      /* first phi of the minhash schedule (default 1.3) */
#define DMS_OPT_LSH_PHI0 2  /* first phi of the LSH schedule (default 2.5) */
#define DMS_OPT_PHI_MAX 3   /* give up with DMS_SET_RANGE beyond this phi (default 2^20) */
#define DMS_OPT_SPLIT_NNZ 4 /* fast engine: sets with more nonzeros are shared by several
                               wavefronts, one part of at most this many nonzeros each
                               (default 4096; 0 disables, and then every set must have fewer
                               than 2^32 nonzeros: queues name elements by 32-bit offsets within
                               the set or part).  The parts are planned on the device into
                               scratch of fixed capacity (twice the batch's sets, at least 1024
                               parts, at most 256 MiB of partial buckets); a heavy set that no
                               longer fits is sketched whole by one wave (same outputs). */
#define DMS_OPT_BOTTOMK_PHI0 5 /* first phi of the bottom-k schedule (default 0: 1 + 3/sqrt(k)) */
#define DMS_OPT_HASH 6      /* DMS_HASH_*: the hash of every hashing step (default DMS_HASH_MIX).
                               Unlike the other options it changes the outputs: sketches made
                               with different hashes are not comparable. */
#define DMS_OPT_ORDER 7     /* fast engine: 1 (default) hands sets to wavefronts largest first
                               (by a log-scale class of the nonzero count, a stable sort on the
                               device before the main launch), 0 in input order.  Batches of
                               2^31 sets or more always run in input order. */

#define DMS_OPT_WAVES 9     /* dms_sketch_csr, fast engine: waves per block, 1..4 (0, the default:
                               the count that keeps the most waves resident in a CU's LDS) */
#define DMS_OPT_TILE 10     /* dms_sketch_csr, fast engine: buckets a wave holds at once, a multiple
                               of 64 below k; the schedule then runs once per tile of buckets (same
                               outputs, more passes, less LDS per wave).  0 (default): all k when
                               they fit next to the queues in 64 KiB, else the fewest equal tiles.
                               A call whose choice of tile and waves does not fit 64 KiB of LDS
                               returns DMS_EINVAL. */
#define DMS_OPT_TIMING 8    /* 1: bracket the main kernel of every dms_sketch_csr, dms_lsh_keys and
                               dms_bottomk call with HIP events on the context's stream (read
                               and reset by dms_kernel_time); 0 (default): no events */

/* Hash functions (DMS_OPT_HASH). */
#define DMS_HASH_MIX 0 /* SplitMix64's output function of (key XOR input) */
#define DMS_HASH_TAB 1 /* simple tabulation of (key XOR input): XOR of one 64-bit word per input
                          byte, table b = MT19937-64 outputs 7 + 256 b .. 262 + 256 b for the seed
                          (the paper's randomness source, Section 4 "Implementation") */

/* Flags of dms_sketch_csr, dms_lsh_keys and dms_bottomk. */
#define DMS_FLAG_VALIDATE 1u /* a set listing an element id more than once gets DMS_SET_INVALID
                                (without it, a repeated id behaves as one element of the larger
                                weight: the same darts are met twice) */
#define DMS_FLAG_COUNTERS 2u /* write the per-set enumeration counts to out_counters (must be
                                non-NULL exactly when this flag is set): int64[n_sets*8] at
                                [s*8 + q], q = 0 regions, 1 areas, 2 darts generated, 3 darts
                                whose rank passed, 4 darts accepted (rank and weight), 5 phi
                                passes run, 6 the last pass's phi (bit pattern of a double),
                                7 zero.  Algorithm 1 visits the regions, areas and darts counted
                                by 0..2.  The fast engine counts a retry pass's darts of 3 and 4
                                only in its new rank band (tau_prev, tau] (it keeps the earlier
                                ones), the plain engine every dart of rank <= tau.  All zero for a
                                set whose row scan fails (empty, invalid, range). */

/* Formats of dms_jaccard_est. */
#define DMS_FMT_U32 0  /* k uint32 minhash values per set */
#define DMS_FMT_1BIT 1 /* ceil(k/64) uint64 words per set, bit j at bit j%64 of word j/64 */

typedef struct dms_ctx_s* dms_ctx;

/* Version of the specification the sketches follow (constants, hash, float
 * derivation); a database of sketches records it (dms_db_*). */
#define DMS_SPEC_VERSION 1

/* Create a context on HIP device `device`.  `seed` selects the hash functions:
 * the six 64-bit keys are the first six outputs of MT19937-64 seeded with it
 * (the paper seeds its hashing with a Mersenne Twister, Section 4
 * "Implementation").  Sketches made with different seeds are not comparable.
 * On success *out receives the context.  Errors: DMS_EINVAL (out NULL, bad
 * device), DMS_EHIP. */
dms_status dms_create(dms_ctx* out, int device, uint64_t seed);

/* Destroy a context and free what it owns (not the caller's buffers). */
dms_status dms_destroy(dms_ctx ctx);

/* Use `hip_stream` (a hipStream_t, or NULL for the null stream) for all later
 * calls on this context.  The context's scratch is shared by its calls, so
 * work queued on the new stream waits for what is queued on the old one (an
 * event recorded on the old stream) -- except while either stream is being
 * captured into a graph, when the caller orders the work (a capture cannot
 * wait for work outside it).  Errors: DMS_EINVAL, DMS_EHIP. */
dms_status dms_set_stream(dms_ctx ctx, void* hip_stream);

/* Set / read one DMS_OPT_* option.  Errors: DMS_EINVAL for an unknown option
 * or a value outside its range (phi0 and phi_max must be positive and finite). */
dms_status dms_set_option(dms_ctx ctx, int32_t option, double value);
dms_status dms_get_option(dms_ctx ctx, int32_t option, double* value);

/*
 * DartMinHash (Theorem 1, Section 3; DartHash is Algorithm 1, Section 2): for
 * every row s of the CSR matrix, k independent weighted minhashes.
 * t = ceil(k ln k) + k darts per unit of phi are hashed to k buckets; bucket j
 * keeps its dart of smallest rank (ties: smaller id hash); phi doubles until no
 * bucket is empty.
 *   row_ptr  device int64[n_sets+1]
 *   idx      device int32[row_ptr[n_sets]]
 *   w        device float64[row_ptr[n_sets]]
 *   k        1 .. 4096
 *   out_u32  device uint32[n_sets*k] or NULL: low 32 bits of bucket j's dart
 *            id hash at [s*k + j]; 0xFFFFFFFF for a set whose status is not OK
 *   out_bits device uint64[n_sets*ceil(k/64)] or NULL: the 1-bit sketch
 *            (Section 1.1), bit j = bit 0 of that hash, at bit j%64 of word
 *            s*ceil(k/64) + j/64; all zero for a set whose status is not OK
 *   out_status device int8[n_sets] or NULL: DMS_SET_*
 *   out_s    device uint64[n_sets*k] or NULL: the full 64-bit dart id hash
 *   out_rank device float64[n_sets*k] or NULL: the dart's rank (+inf if not OK)
 *   flags    DMS_FLAG_* (0 for none)
 *   out_counters device int64[n_sets*8] when flags has DMS_FLAG_COUNTERS, else NULL
 * Errors: DMS_EINVAL (k out of range, n_sets < 0, a required pointer NULL,
 * unknown flag bits, out_counters given without DMS_FLAG_COUNTERS or missing
 * with it), DMS_EHIP, DMS_ENOMEM.
 */
dms_status dms_sketch_csr(dms_ctx ctx, int64_t n_sets, const int64_t* row_ptr,
                          const int32_t* idx, const double* w, int32_t k, uint32_t* out_u32,
                          uint64_t* out_bits, int8_t* out_status, uint64_t* out_s,
                          double* out_rank, uint32_t flags, int64_t* out_counters);

/*
 * Autotuner for dms_sketch_csr: times the sketch of a prefix of the batch
 * (its first min(n_sets, 2^28/k) rows, so the rows should be in no particular
 * order) under candidate schedules -- first phi in {1, 1.15, 1.3, 1.5, 1.8},
 * then split thresholds in {0, 1024, 4096, 16384}, then both DMS_OPT_ORDER
 * values, then waves per block 1..4 and half the automatic bucket tile -- and
 * sets DMS_OPT_PHI0, DMS_OPT_SPLIT_NNZ, DMS_OPT_ORDER, DMS_OPT_WAVES and
 * DMS_OPT_TILE on the context to the fastest.  Outputs never depend on
 * either (Theorem 1's output is independent of the schedule; parts merge
 * exactly).  Synchronizes the stream; allocates and frees its own buffers.
 *   out_phi0, out_split: host double* or NULL, receive the chosen values
 * Errors: DMS_EINVAL, DMS_EHIP, DMS_ENOMEM.
 */
dms_status dms_autotune(dms_ctx ctx, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                        const double* w, int32_t k, double* out_phi0, double* out_split);

/*
 * (L,K) LSH values (Section 1.2 "Fast similarity search" and Section 3
 * "Bottom-k minhash and fast approximate near neighbor search"): DartHash with
 * t = L*K, darts hashed to L tables, each table's K darts of smallest rank in
 * ascending order (a repeated dart counts once), phi doubling until every
 * table holds K darts; table l's key folds the ordered dart id hashes:
 * h = mix(K_L ^ l), h = mix(h ^ s_m) for m < K.  Two sets share table l's key
 * with probability J^K, independently across tables.
 *   L 1..1024, K 1..64, L*K <= 65536
 *   out_keys device uint64[n_sets*L] at [s*L + l]; 0 for a set not OK
 *   out_status device int8[n_sets] or NULL
 *   flags, out_counters  as for dms_sketch_csr
 * Errors: DMS_EINVAL, DMS_EHIP, DMS_ENOMEM.
 */
dms_status dms_lsh_keys(dms_ctx ctx, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                        const double* w, int32_t L, int32_t K, uint64_t* out_keys,
                        int8_t* out_status, uint32_t flags, int64_t* out_counters);

/*
 * Weighted Jaccard estimates from sketches (Section 1.1): for pair p, with a
 * and b holding n_pairs sketches each (row p of a against row p of b):
 *   DMS_FMT_U32:  out[p] = (#j with a[p*k+j] == b[p*k+j]) / k
 *   DMS_FMT_1BIT: out[p] = 1 - 2 * popcount((a ^ b) restricted to k bits) / k
 *                 (each bit agrees with probability (1+J)/2; not clamped)
 *   a, b device arrays in the format's layout; out device float64[n_pairs].
 * Errors: DMS_EINVAL, DMS_EHIP.
 */
dms_status dms_jaccard_est(dms_ctx ctx, int64_t n_pairs, const void* a, const void* b, int32_t k,
                           int32_t format, double* out);

/*
 * Weight-class LSH index for approximate near neighbour search (Section 3):
 * set s belongs to weight class c = floor(log2 ||x||_1), with ||x||_1 summed
 * left to right, and is indexed by the (L,K) LSH keys (dms_lsh_keys) of
 * x * 2^-c, whose ||.||_1 lies in [1, 2) (the scaling is exact).  Indexed rows
 * must list strictly increasing ids (as uint32) with finite weights >= 0;
 * other rows get a non-OK status and are left out.  The index keeps the
 * caller's row_ptr, idx and w (device) for verification: they must stay valid
 * and unchanged until dms_index_destroy.  The build synchronizes the stream.
 * Errors: DMS_EINVAL, DMS_EHIP, DMS_ENOMEM.
 */
typedef struct dms_index_s* dms_index;
dms_status dms_index_build(dms_ctx ctx, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                           const double* w, int32_t L, int32_t K, dms_index* out);

/* Per indexed set: its weight class and DMS_SET_* status (device int32[n],
 * int8[n]; either may be NULL). */
dms_status dms_index_sets(dms_index ix, int32_t* out_class, int8_t* out_status);

/*
 * Near neighbours of n_q query sets (CSR, device; rows under the same rules as
 * indexed rows).  For every class c within span = ceil(log2(1/j1)) + 1 of the
 * query's own, the query scaled by 2^-c (Jaccard is unchanged when both sets
 * are scaled alike) is hashed to its L keys; every indexed set of class c
 * sharing one of them is a candidate; candidates are verified with the exact
 * weighted Jaccard J = sum min / sum max (both sums in ascending id order).
 *   out_ids    device int64[n_q*topn]  sets with J >= j1, by J descending then
 *                                      set ascending; -1 past the last
 *   out_j      device float64[n_q*topn] their J (0 past the last)
 *   out_count  device int32[n_q]  results written
 *   out_candidates device int32[n_q]  distinct candidates verified
 *   out_status device int8[n_q]   DMS_SET_* of the query, or DMS_QUERY_OVERFLOW
 *   j1 in (0, 1], topn 1..1024
 * Errors: DMS_EINVAL, DMS_EHIP, DMS_ENOMEM.
 */
dms_status dms_index_query(dms_index ix, int64_t n_q, const int64_t* q_row_ptr, const int32_t* q_idx,
                           const double* q_w, double j1, int32_t topn, int64_t* out_ids, double* out_j,
                           int32_t* out_count, int32_t* out_candidates, int8_t* out_status);

/* Free the index (waits for the context's stream). */
dms_status dms_index_destroy(dms_index ix);

/*
 * Bottom-k sketch (Section 3, bottom-k minhash): DartHash with t = k, phi
 * doubling from DMS_OPT_BOTTOMK_PHI0 until the darts of rank <= tau hold at
 * least k distinct ones; row s's sketch is its k darts of smallest (rank, id
 * hash), ascending.  A dart met twice (a repeated element id) counts once.
 *   row_ptr, idx, w  as for dms_sketch_csr
 *   out_s      device uint64[n_sets*k]  id hashes (~0 for a set whose status is not OK)
 *   out_rank   device float64[n_sets*k] or NULL (+inf for such a set)
 *   out_status device int8[n_sets] or NULL
 *   k 1..1024
 *   flags, out_counters  as for dms_sketch_csr (the rank and acceptance
 *   counts are those of each pass's new rank band)
 * Errors: DMS_EINVAL, DMS_EHIP, DMS_ENOMEM.
 */
dms_status dms_bottomk(dms_ctx ctx, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                       const double* w, int32_t k, uint64_t* out_s, double* out_rank,
                       int8_t* out_status, uint32_t flags, int64_t* out_counters);

/*
 * Jaccard estimate from two bottom-k sketches (dms_bottomk layout, both with
 * status OK): out[p] = (number of the k first darts of the union of the two
 * sketches that lie in both) / k.  Darts are equal when rank and id hash are.
 *   rank_a, rank_b device float64[n_pairs*k]; s_a, s_b device uint64[n_pairs*k]
 *   out device float64[n_pairs]; k 1..1024
 * Errors: DMS_EINVAL, DMS_EHIP.
 */
dms_status dms_jaccard_est_bottomk(dms_ctx ctx, int64_t n_pairs, const double* rank_a, const uint64_t* s_a,
                                   const double* rank_b, const uint64_t* s_b, int32_t k, double* out);

/*
 * b-bit fingerprints (Section 1.1, similarity estimation): the fingerprint of
 * a minhash is its lowest `bits` bits (bits of the dart-id hash, independent of
 * the bucket bits; bits = 1 gives the 1-bit sketch of dms_sketch_csr).  Row s's
 * k fingerprints are packed into words = ceil(k*bits/64) uint64 words:
 * fingerprint j occupies stream bits [j*bits, j*bits + bits), stream bit p is
 * bit p%64 of word p/64, and the unused high bits of the last word are zero.
 *   minhash device uint32[n_sets*k]     (out_u32 of dms_sketch_csr)
 *   out     device uint64[n_sets*words]
 *   k 1..2^20, bits 1..32
 * Errors: DMS_EINVAL, DMS_EHIP.
 */
dms_status dms_bbit_pack(dms_ctx ctx, int64_t n_sets, const uint32_t* minhash, int32_t k,
                         int32_t bits, uint64_t* out);

/*
 * Weighted Jaccard estimate from two packed b-bit sketches (layout of
 * dms_bbit_pack).  Fingerprints of one bucket agree with probability
 * J + (1 - J) 2^-bits, so out[p] = (m/k - 2^-bits) / (1 - 2^-bits) with m the
 * number of agreeing fingerprints of pair p (not clamped).  Bits past k*bits
 * in the last word are ignored.
 *   a, b device uint64[n_pairs*words]; out device float64[n_pairs]
 *   k 1..2^20, bits 1..32
 * Errors: DMS_EINVAL, DMS_EHIP.
 */
dms_status dms_jaccard_est_bbit(dms_ctx ctx, int64_t n_pairs, const uint64_t* a, const uint64_t* b,
                                int32_t k, int32_t bits, double* out);

/*
 * Unary feature map of b-bit minhashes (Section 1.1, large-scale kernel
 * machines): row s becomes the k*2^bits dimensional vector with value
 * 1/sqrt(k) at the k coordinates j*2^bits + fingerprint_j and zero elsewhere,
 * so the inner product of two rows is the fraction of agreeing fingerprints.
 *   minhash   device uint32[n_sets*k]
 *   out_index device int32[n_sets*k]   (ascending within a row)
 *   out_scale host double* or NULL     (receives 1/sqrt(k))
 *   k >= 1, bits 1..16, k*2^bits <= 2^31
 * Errors: DMS_EINVAL, DMS_EHIP.
 */
dms_status dms_unary_map(dms_ctx ctx, int64_t n_sets, const uint32_t* minhash, int32_t k,
                         int32_t bits, int32_t* out_index, double* out_scale);

/*
 * Provenance of sketches.  Two sketches can be compared (Section 1.1: the
 * estimators compare minhashes of the same hash functions) only if they were
 * made under the same specification version, hash kind, seed and k.
 */
typedef struct {
    int32_t spec_version; /* DMS_SPEC_VERSION */
    int32_t hash;         /* DMS_HASH_* */
    uint64_t seed;        /* seed of the hash keys */
    int32_t k;            /* minhashes per sketch (bits per 1-bit row) */
    int32_t reserved;     /* 0 */
} dms_sketch_info;

/* The provenance of the sketches this context makes at k (its seed and
 * DMS_OPT_HASH at the time of the call).  Errors: DMS_EINVAL. */
dms_status dms_sketch_info_of(dms_ctx ctx, int32_t k, dms_sketch_info* out);

/*
 * A device-resident database of 1-bit sketches (k bits per row, ceil(k/64)
 * uint64 words, row id = position) that records its provenance, taken from
 * the context at creation.  It owns its rows; the context must outlive it.
 * dms_db_create: room for `capacity` rows (k 1..4096, capacity < 2^31).
 *   Errors: DMS_EINVAL, DMS_ENOMEM.
 * dms_db_append_sets: sketches n_sets CSR sets (device, as for dms_sketch_csr)
 *   with the database's context into the next rows; out_status device int8
 *   [n_sets] or NULL; *out_first (host, or NULL) receives the first row.
 *   Errors: DMS_EMISMATCH (the context's hash changed since creation),
 *   DMS_ENOMEM (capacity), and those of dms_sketch_csr.
 * dms_db_append_bits: copies n rows of 1-bit sketches (device or host memory)
 *   that were made under *info; DMS_EMISMATCH unless *info equals the
 *   database's provenance; DMS_ENOMEM beyond the capacity.
 * dms_db_info: provenance, rows held, and the device address of the rows
 *   (any output may be NULL).
 * dms_db_topk: dms_hamming_topk of queries (device uint64[n_q*words]) made
 *   under *q_info against the rows held; DMS_EMISMATCH unless *q_info equals
 *   the database's provenance.
 * dms_db_destroy: waits for the context's stream and frees the rows.
 * Appends and searches run on the context's stream.
 */
typedef struct dms_db_s* dms_db;
dms_status dms_db_create(dms_ctx ctx, int32_t k, int64_t capacity, dms_db* out);
dms_status dms_db_append_sets(dms_db db, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                              const double* w, int8_t* out_status, int64_t* out_first);
dms_status dms_db_append_bits(dms_db db, int64_t n, const uint64_t* bits, const dms_sketch_info* info,
                              int64_t* out_first);
dms_status dms_db_info(dms_db db, dms_sketch_info* info, int64_t* n_rows, const uint64_t** rows);
dms_status dms_db_topk(dms_db db, const uint64_t* queries, int64_t n_q, const dms_sketch_info* q_info,
                       int32_t topk, int64_t* out_ids, int32_t* out_dist);
dms_status dms_db_destroy(dms_db db);

/*
 * Hamming top-k search over 1-bit sketches (the similarity-search use of
 * Section 1.1), without provenance checks (dms_db_topk checks them): for
 * every query row q, the `topk` database rows with the
 * smallest Hamming distance, ascending by (distance, row id).
 *   db      device uint64[n_db*words]       (1-bit sketches, `words` words each)
 *   queries device uint64[n_q*words]
 *   out_ids device int64[n_q*topk]   (-1 where n_db < topk)
 *   out_dist device int32[n_q*topk]  (-1 where n_db < topk)
 *   words 1..64, n_q 0..4096, topk 1..64, n_db < 2^31
 * Errors: DMS_EINVAL, DMS_EHIP, DMS_ENOMEM.
 */
dms_status dms_hamming_topk(dms_ctx ctx, const uint64_t* db, int64_t n_db, int32_t words,
                            const uint64_t* queries, int64_t n_q, int32_t topk, int64_t* out_ids,
                            int32_t* out_dist);

/*
 * Measurement support (roofline calibration; not part of the sketching path).
 * kind 0: 8 independent chains of the specification's 64-bit mixer per thread,
 *         `iters` steps each (blocks*256 threads): the chip's hashing rate.
 * kind 1: 8 chains of 32-bit xor/add per thread: full-rate integer issue.
 * kind 2: copy `bytes` (multiple of 16) from device buffer a to device buffer b
 *         with a grid-stride loop: HBM bandwidth and the reference for scaling
 *         the FETCH_SIZE / WRITE_SIZE counters.
 * kind 3: the same copy with four 16-byte loads in flight per thread and
 *         streaming (non-temporal) stores.
 * a must hold at least 8 bytes for kinds 0 and 1.  Blocks until the kernel
 * is done and stores its duration in *out_ms (HIP events on the context's
 * stream).  Errors: DMS_EINVAL, DMS_EHIP.
 */
dms_status dms_calibrate(dms_ctx ctx, int32_t kind, int32_t iters, int64_t bytes, int32_t blocks,
                         void* a, void* b, double* out_ms);

/*
 * Serving loop (continuous batching).  A server owns, per batch slot, a HIP
 * stream, a device arena and pinned staging buffers, and scans a sketch
 * database (dms_db, k = 1024, 16 words per row, row id = position) whose
 * provenance must equal the context's sketches at k = 1024.  Requests are either DMS_REQ_SKETCH (k minhashes of the
 * request's set, k in {64, 256, 1024}) or DMS_REQ_SEARCH (the set's 1-bit
 * k = 1024 sketch, then the topk database rows nearest in Hamming distance,
 * ascending by (distance, row)).  While a slot is free, the requests that have
 * arrived are admitted in arrival order as long as the slot's memory budget
 * (max_batch rows, max_batch_nnz nonzeros) allows; batches of different slots
 * overlap on the GPU.  A request's result depends only on its own set.
 */
#define DMS_REQ_SKETCH 0
#define DMS_REQ_SEARCH 1

typedef struct {
    int32_t max_batch;     /* requests per batch slot, 1..4096 */
    int32_t max_inflight;  /* batch slots (streams) in flight, 1..16 */
    int64_t max_batch_nnz; /* nonzeros a slot holds (its input arena) */
    int32_t max_set_nnz;   /* largest request set accepted, <= max_batch_nnz */
    int32_t db_words;      /* words per database row: 16 */
    int32_t topk;          /* neighbours per search, 1..64 */
    int32_t split_nnz;     /* sets with more nonzeros are shared by several wavefronts,
                              parts of at most this many each (0: never); 16.. */
} dms_server_config;

typedef struct dms_server_s* dms_server;

/* Create a server on ctx (the context must outlive it) over the rows db holds
 * now; the database must not be appended to or destroyed while the server
 * lives.  Errors: DMS_EINVAL, DMS_EMISMATCH (the database was made under
 * another specification version, hash, seed, or not at k = 1024), DMS_ENOMEM,
 * DMS_EHIP, DMS_ESPEC. */
dms_status dms_server_create(dms_ctx ctx, const dms_server_config* cfg, dms_db db, dms_server* out);
dms_status dms_server_destroy(dms_server s);

/*
 * Serve n_req requests whose arrival times (seconds after the call starts,
 * non-decreasing) are given: an open-loop trace replayed in real time; returns
 * when every request is answered.  All pointers are host memory.
 *   kind[n_req], k[n_req]               request kind and sketch size
 *   row_ptr[n_req+1], idx, w            the request sets (CSR)
 *   sketch_off[n_req], out_sketch       request r's k minhashes go to
 *                                       out_sketch[sketch_off[r] ...] (NULL: none)
 *   out_status[n_req]                   DMS_SET_* per request (or NULL)
 *   out_ids[n_req*topk], out_dist[...]  search results of search requests (or NULL)
 *   out_latency_s[n_req]                completion minus arrival (or NULL)
 *   out_stats[7]                        requests/s, p50 s, p99 s, max s, batches,
 *                                       mean requests per batch, elapsed s (or NULL)
 * Errors: DMS_EINVAL (a request outside the configured limits, an arrival out
 * of order), DMS_EHIP, DMS_ESPEC.
 */
dms_status dms_server_replay(dms_server s, int64_t n_req, const double* arrival_s,
                             const int32_t* kind, const int32_t* k, const int64_t* row_ptr,
                             const int32_t* idx, const double* w, const int64_t* sketch_off,
                             uint32_t* out_sketch, int8_t* out_status, int64_t* out_ids,
                             int32_t* out_dist, double* out_latency_s, double* out_stats);

/*
 * Online use of the same server: requests are submitted as they come and the
 * answers collected by polling.  A server serves either replays or online
 * requests at a time (dms_server_replay returns DMS_EINVAL while online
 * requests are pending).  Not thread-safe: one thread drives a server.
 *
 * dms_server_submit copies the request's set (host idx[nnz], w[nnz]) into the
 * server and returns its id (0, 1, 2, ... in submission order).  Errors:
 * DMS_EINVAL (kind, k or nnz outside the configured limits).
 *
 * dms_server_poll collects finished batches, admits waiting requests into free
 * slots (in submission order, within each slot's memory budget) and returns up
 * to max_out answers in completion order.  With wait_ms > 0 it waits up to that
 * long for a first answer while requests are in flight.  Host outputs, row n for
 * the n-th answer (each may be NULL but out_id):
 *   out_id[max_out]                    request id
 *   out_status[max_out]                DMS_SET_*
 *   out_sketch[max_out*1024]           the request's k minhashes at out_sketch[n*1024 ...]
 *   out_ids, out_dist[max_out*topk]    search answers (rows of search requests only)
 *   out_latency_s[max_out]             answer time minus submission time
 *   *n_out                             answers written
 * Errors: DMS_EINVAL, DMS_EHIP, DMS_ESPEC.
 */
dms_status dms_server_submit(dms_server s, int32_t kind, int32_t k, int64_t nnz, const int32_t* idx,
                             const double* w, int64_t* out_id);
dms_status dms_server_poll(dms_server s, int32_t wait_ms, int64_t max_out, int64_t* out_id,
                           int8_t* out_status, uint32_t* out_sketch, int64_t* out_ids, int32_t* out_dist,
                           double* out_latency_s, int64_t* n_out);

/* Make the context's device tables for k (t = ceil(k ln k) + k) now, so that
 * later calls with this k need no allocation (dms_sketch_csr makes them on
 * first use).  Synchronizes the stream.  Errors: DMS_EINVAL, DMS_ESPEC,
 * DMS_ENOMEM, DMS_EHIP. */
dms_status dms_prepare(dms_ctx ctx, int32_t k);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * dms_sketch_csr computation (same outputs, bit for bit) that calls no
 * hipMalloc or hipFree and no allocating library routine.  Its scratch (the
 * persistent kernel's work cursor and the largest-first size order) lives in a
 * 16 MiB device array of the library, one per GPU, held from the library's load
 * until the process ends.  Limits: n_sets <= 2^20 (DMS_EINVAL above); sets are
 * not split across wavefronts (as with DMS_OPT_SPLIT_NNZ = 0, so every set must
 * have fewer than 2^32 nonzeros).  The context's tables for k must exist
 * (dms_prepare, or an earlier dms_sketch_csr with this k), else DMS_EINVAL.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (on other streams or other contexts) race and must be ordered by the caller.
 *   arguments as for dms_sketch_csr (out_u32, out_bits, out_status may be NULL)
 * Errors: DMS_EINVAL, DMS_EHIP.
 */
dms_status dms_sketch_csr_noalloc(dms_ctx ctx, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                                  const double* w, int32_t k, uint32_t* out_u32, uint64_t* out_bits,
                                  int8_t* out_status);

/* Measurement support (DMS_OPT_TIMING): waits for the timed calls since the
 * last dms_kernel_time and returns the summed duration of their main kernels
 * (the persistent sketching kernel with its one-thread cursor reset, or the
 * plain engine's kernel) in *out_ms and their number in *out_launches (may be
 * NULL); then starts a new tally.  Errors: DMS_EINVAL, DMS_EHIP. */
dms_status dms_kernel_time(dms_ctx ctx, double* out_ms, int64_t* out_launches);

/* Wait until all work queued on the context's stream is done. */
dms_status dms_sync(dms_ctx ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next call. */
const char* dms_last_error(dms_ctx ctx);

/* Name of a return or per-set status code. */
const char* dms_status_str(dms_status s);

/*
 * Host-only queries of the specification (no GPU needed).
 * dms_t_of_k: t = ceil(k ln k) + k (proof of Theorem 1).
 * dms_spec_constants: for `seed` and t, the six hash keys (K_R, K_A, K_U, K_V,
 * K_S, K_L), the 20 Poisson(1) thresholds floor(2^64 P[Poi(1) <= n]), the
 * region corners W[1024] = RN(RN(2^nu-1)/t) and R[1024] = RN(2^rho-1), and
 * u = RN(1/t).  Any output pointer may be NULL.  Errors: DMS_EINVAL (t = 0),
 * DMS_ESPEC.
 */
dms_status dms_t_of_k(int32_t k, uint32_t* t);
dms_status dms_spec_constants(uint64_t seed, uint32_t t, uint64_t keys[6], uint64_t pois[20],
                              double* W, double* R, double* u);

/* The 8 x 256 simple-tabulation words of DMS_HASH_TAB for a seed (host array,
 * table-major).  Errors: DMS_EINVAL (out NULL). */
dms_status dms_spec_tabulation(uint64_t seed, uint64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* DMS_H */
