// A device-resident database of 1-bit sketches that records how they were made
// (specification version, hash kind, seed, k): sketches are comparable only
// under one hash function and one k (the similarity estimators of Section 1.1
// compare minhashes of the same hash functions), so every way in checks the
// provenance, and the search and the serving loop refuse a database or queries
// made otherwise.
#include <hip/hip_runtime.h>

#include "../../include/dms.h"
#include "dms_internal.h"
#include "dms_launch.h"

struct dms_db_s {
    dms_ctx ctx = nullptr;
    dms_sketch_info info{};
    int32_t words = 0;         // uint64 words per row: ceil(k / 64)
    int64_t capacity = 0, n = 0;
    uint64_t* rows = nullptr;  // device, capacity * words
    int8_t* status = nullptr;  // device scratch for appended sets' statuses
    int64_t status_cap = 0;
};

namespace {

bool same(const dms_sketch_info& a, const dms_sketch_info& b)
{
    return a.spec_version == b.spec_version && a.hash == b.hash && a.seed == b.seed && a.k == b.k;
}

struct Device {
    int prev = -1;
    explicit Device(int dev)
    {
        (void)hipGetLastError();
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~Device()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace dms {
// Read access for the serving loop.
const uint64_t* db_rows(dms_db db) { return db->rows; }
int64_t db_count(dms_db db) { return db->n; }
const dms_sketch_info* db_info(dms_db db) { return &db->info; }
}  // namespace dms

extern "C" {

dms_status dms_sketch_info_of(dms_ctx ctx, int32_t k, dms_sketch_info* out)
{
    if (!ctx || !out || k < 1 || k > 4096) return DMS_EINVAL;
    out->spec_version = DMS_SPEC_VERSION;
    out->hash = dms::ctx_hash(ctx);
    out->seed = dms::ctx_seed(ctx);
    out->k = k;
    out->reserved = 0;
    return DMS_OK;
}

dms_status dms_db_create(dms_ctx ctx, int32_t k, int64_t capacity, dms_db* out)
{
    if (!ctx || !out || k < 1 || k > 4096 || capacity < 0 || capacity > ((int64_t)1 << 31) - 1) return DMS_EINVAL;
    *out = nullptr;
    Device g(dms::ctx_device(ctx));
    auto* db = new dms_db_s;
    db->ctx = ctx;
    (void)dms_sketch_info_of(ctx, k, &db->info);
    db->words = (k + 63) / 64;
    db->capacity = capacity;
    const size_t bytes = (size_t)(capacity > 0 ? capacity : 1) * (size_t)db->words * sizeof(uint64_t);
    if (hipMalloc((void**)&db->rows, bytes) != hipSuccess) {
        delete db;
        return DMS_ENOMEM;
    }
    *out = db;
    return DMS_OK;
}

dms_status dms_db_destroy(dms_db db)
{
    if (!db) return DMS_EINVAL;
    Device g(dms::ctx_device(db->ctx));
    (void)hipStreamSynchronize(dms::ctx_stream(db->ctx));
    (void)hipFree(db->rows);
    (void)hipFree(db->status);
    delete db;
    return DMS_OK;
}

dms_status dms_db_info(dms_db db, dms_sketch_info* info, int64_t* n_rows, const uint64_t** rows)
{
    if (!db) return DMS_EINVAL;
    if (info) *info = db->info;
    if (n_rows) *n_rows = db->n;
    if (rows) *rows = db->rows;
    return DMS_OK;
}

dms_status dms_db_append_sets(dms_db db, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                              const double* w, int8_t* out_status, int64_t* out_first)
{
    if (!db || n_sets < 0) return DMS_EINVAL;
    dms_ctx c = db->ctx;
    dms_sketch_info now{};
    (void)dms_sketch_info_of(c, db->info.k, &now);
    if (!same(now, db->info)) return DMS_EMISMATCH;  // the context's hash changed since the database was made
    if (n_sets > db->capacity - db->n) return DMS_ENOMEM;
    if (out_first) *out_first = db->n;
    if (n_sets == 0) return DMS_OK;
    const dms_status st = dms_sketch_csr(c, n_sets, row_ptr, idx, w, db->info.k, nullptr,
                                         db->rows + (size_t)db->n * db->words, out_status, nullptr, nullptr, 0,
                                         nullptr);
    if (st != DMS_OK) return st;
    db->n += n_sets;
    return DMS_OK;
}

dms_status dms_db_append_bits(dms_db db, int64_t n, const uint64_t* bits, const dms_sketch_info* info,
                              int64_t* out_first)
{
    if (!db || n < 0 || !info || (n > 0 && !bits)) return DMS_EINVAL;
    if (!same(*info, db->info)) return DMS_EMISMATCH;
    if (n > db->capacity - db->n) return DMS_ENOMEM;
    if (out_first) *out_first = db->n;
    if (n == 0) return DMS_OK;
    Device g(dms::ctx_device(db->ctx));
    const hipError_t e = hipMemcpyAsync(db->rows + (size_t)db->n * db->words, bits,
                                        (size_t)n * db->words * sizeof(uint64_t), hipMemcpyDefault,
                                        dms::ctx_stream(db->ctx));
    if (e != hipSuccess) return DMS_EHIP;
    db->n += n;
    return DMS_OK;
}

dms_status dms_db_topk(dms_db db, const uint64_t* queries, int64_t n_q, const dms_sketch_info* q_info,
                       int32_t topk, int64_t* out_ids, int32_t* out_dist)
{
    if (!db || !q_info) return DMS_EINVAL;
    if (!same(*q_info, db->info)) return DMS_EMISMATCH;
    return dms_hamming_topk(db->ctx, db->rows, db->n, db->words, queries, n_q, topk, out_ids, out_dist);
}

}  // extern "C"
