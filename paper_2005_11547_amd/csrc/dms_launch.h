// Host-side launchers of the library's kernels (defined in the .hip files)
// and the few context accessors the serving loop uses (defined in dms_api.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/dms.h"
#include "dms_internal.h"

namespace dms {
// Optional outputs and checks of a sketching launch (DMS_FLAG_*): per-set
// enumeration counts (kCounterWords int64 per set) and per-set flags of rows
// whose element ids repeat (those sets get DMS_SET_INVALID).
struct LaunchExtras {
    int64_t* counters = nullptr;
    const uint8_t* repeated = nullptr;
};

hipError_t launch_sketch_plain(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                               const int32_t* idx, const double* w, int k, uint32_t* out_u32,
                               uint64_t* out_bits, int8_t* out_status, uint64_t* out_s,
                               double* out_rank, double phi0, double phi_max, int hash,
                               const LaunchExtras& x, hipStream_t st);
hipError_t launch_lsh_plain(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                            const int32_t* idx, const double* w, int L, int K, uint64_t* out_keys,
                            int8_t* out_status, double phi0, double phi_max, int hash,
                            const LaunchExtras& x, hipStream_t st);
hipError_t launch_sketch_fast(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                              const int32_t* idx, const double* w, int k, uint32_t* out_u32,
                              uint64_t* out_bits, int8_t* out_status, uint64_t* out_s,
                              double* out_rank, double phi0, double phi_max,
                              unsigned long long* counter, int blocks, int hash, const LaunchExtras& x,
                              hipStream_t st);
int fast_waves(int mode, int k, int K);
int fast_blocks_per_cu(int mode, int k, int K, int waves);
size_t fast_lds(int mode, int k, int K, int waves);
const void* fast_kernel_address(int mode, int hash);
// The fast engine's LSH variant for L tables of K darts (kModeLshReg or kModeLsh).
int lsh_fast_mode(int L, int K);
hipError_t launch_bottomk_fast(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                               const int32_t* idx, const double* w, int k, uint64_t* out_s,
                               double* out_rank, int8_t* out_status, double phi0, double phi_max,
                               unsigned long long* counter, int blocks, const uint32_t* order, int hash,
                               const LaunchExtras& x, hipStream_t st);
hipError_t launch_bottomk_jaccard(int64_t n_pairs, const double* ra, const uint64_t* sa, const double* rb,
                                  const uint64_t* sb, int k, double* out, hipStream_t st);
hipError_t launch_index_prep(int64_t n, const int64_t* rp, const int32_t* idx, const double* w, double* wn,
                             int32_t* cls, int8_t* status, hipStream_t st);
size_t index_sort_scratch(int64_t n);
hipError_t launch_index_order(int64_t n, const int32_t* cls, const int8_t* status, uint64_t* okey,
                              uint64_t* okey2, int64_t* ord, unsigned long long* n_ok_dev, void* scratch,
                              size_t scratch_bytes, hipStream_t st);
hipError_t launch_index_table(int64_t n_ok, const int64_t* ord, const uint64_t* keys, const int32_t* cls, int L,
                              int l, uint64_t* tmp_k, uint64_t* tmp_v, uint64_t* out_k, uint64_t* out_v,
                              void* scratch, size_t scratch_bytes, hipStream_t st);
hipError_t launch_query_prep(int64_t n_q, const int64_t* rp, const int32_t* idx, const double* w, int span,
                             int64_t* xrp, int32_t* xidx, double* xw, int32_t* qcls, int8_t* qstatus,
                             hipStream_t st);
hipError_t launch_index_query(int64_t n_q, int span, int L, const uint64_t* qkeys, const int8_t* xstatus,
                              const int32_t* qcls, const int8_t* qstatus, const uint64_t* tkeys,
                              const uint64_t* tvals, int64_t n_ok, const int64_t* q_rp, const int32_t* q_idx,
                              const double* q_w, const int64_t* d_rp, const int32_t* d_idx, const double* d_w,
                              double j1, int topn, int64_t* out_ids, double* out_j, int32_t* out_count,
                              int32_t* out_cand, int8_t* out_status, int n_cu, hipStream_t st);
hipError_t launch_sketch_fast_split(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                                    const int32_t* idx, const double* w, int k, uint32_t* out_u32,
                                    uint64_t* out_bits, int8_t* out_status, uint64_t* out_s,
                                    double* out_rank, double phi0, double phi_max,
                                    unsigned long long* counter, int blocks, const void* parts,
                                    int64_t n_parts, void* heavy, uint64_t* partial, int64_t split,
                                    const uint32_t* order, int hash, const LaunchExtras& x,
                                    const unsigned long long* plan_dev, const uint8_t* planned, int kt_opt,
                                    int waves_opt, hipStream_t st);
size_t plan_part_bytes();
size_t plan_heavy_bytes();
// Device-side plan of the heavy sets for launch_sketch_fast_split: resets
// plan[0..7], writes at most part_cap parts (plan[1] of them, for plan[0] heavy
// sets), their row scans, and planned[n_sets] (1 for a set served by parts);
// zeroes the counters of planned sets when out_cnt is given.
hipError_t launch_plan(int64_t n_sets, const int64_t* rp, const double* w, int64_t split, int64_t part_cap,
                       unsigned long long* plan, void* parts, void* heavy, uint8_t* planned, int64_t* out_cnt,
                       hipStream_t st);
hipError_t launch_lsh_fast(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                           const int32_t* idx, const double* w, int L, int K, uint64_t* out_keys,
                           int8_t* out_status, double phi0, double phi_max,
                           unsigned long long* counter, int blocks, const uint32_t* order, int hash,
                           const LaunchExtras& x, hipStream_t st);
size_t hamming_partial_bytes(int64_t n_q, int n_blocks, int topk);
int hamming_blocks(int64_t n_db, int n_cu);
hipError_t launch_hamming(const uint64_t* db, int64_t n_db, int words, const uint64_t* queries,
                          int64_t n_q, int topk, int64_t* out_ids, int32_t* out_dist,
                          uint64_t* partial, int n_blocks, hipStream_t st);
hipError_t calib_run(int kind, int iters, void* a, void* b, int64_t bytes, int blocks,
                     hipStream_t st);
hipError_t launch_bbit_pack(int64_t n_sets, const uint32_t* v, int k, int b, uint64_t* out,
                            hipStream_t st);
hipError_t launch_bbit_jaccard(int64_t n_pairs, const uint64_t* a, const uint64_t* b_, int k, int b,
                               double* out, hipStream_t st);
hipError_t launch_unary_map(int64_t n_sets, const uint32_t* v, int k, int b, int32_t* out,
                            hipStream_t st);
hipError_t launch_jaccard(int64_t n_pairs, const void* a, const void* b, int k, int format,
                          double* out, hipStream_t st);
size_t fast_lds_bytes(int k, int waves);
// Buckets a minhash wave of the fast engine holds at once (k, or tiles of whole
// 64-bucket words when k buckets do not fit next to the queues).
int minhash_tile(int k);
// Tile and waves per block for the DMS_OPT_TILE / DMS_OPT_WAVES values (0:
// automatic); 0 when the choice does not fit a block's 64 KiB of LDS.
int minhash_tile_for(int k, int t);
int minhash_waves_for(int k, int kt, int waves);
hipError_t launch_heavy_scan(int64_t n_heavy, const int64_t* rp, const double* w, HeavySet* heavy,
                             hipStream_t st);
size_t size_order_bytes(int64_t n_sets);
// Per-set flags (1 = some element id occurs twice in the row) for DMS_FLAG_VALIDATE.
hipError_t launch_repeated_ids(int64_t n_sets, const int64_t* rp, const int32_t* idx, uint8_t* out,
                               hipStream_t st);
hipError_t launch_size_order(int64_t n_sets, const int64_t* rp, void* scratch, size_t scratch_bytes,
                             const uint32_t** order, hipStream_t st);

// The context's device tables for t, its device, its number of compute units
// and its options.
int ctx_spec(dms_ctx c, uint32_t t, const SpecTables** out);
int ctx_device(dms_ctx c);
int ctx_n_cu(dms_ctx c);
double ctx_phi0(dms_ctx c);
double ctx_phi_max(dms_ctx c);
int ctx_hash(dms_ctx c);
uint64_t ctx_seed(dms_ctx c);
// Read access to a sketch database for the serving loop.
const uint64_t* db_rows(dms_db db);
int64_t db_count(dms_db db);
const dms_sketch_info* db_info(dms_db db);
// Accessors for the entry points defined outside dms_api.cpp.
const SpecTables* ctx_spec_cached(dms_ctx c, uint32_t t);  // nullptr if t's tables are not made yet
hipStream_t ctx_stream(dms_ctx c);
int ctx_engine(dms_ctx c);
int ctx_order(dms_ctx c);
int ctx_resident_blocks(dms_ctx c, int mode, int k, int K);
int ctx_fail(dms_ctx c, int code, const char* msg);
void ctx_clear_error(dms_ctx c);
// Looks up, once per device, the device address of dms_sketch_csr_noalloc's
// scratch (the device must be current).
hipError_t noalloc_setup(int device);
}  // namespace dms
