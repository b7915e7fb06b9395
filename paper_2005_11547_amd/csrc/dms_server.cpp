// Serving loop: continuous batching of sketch and near-neighbour requests.
//
// Requests arrive over time (an open-loop trace replayed in real time).  The
// loop keeps up to `max_inflight` batches on the GPU, each on its own stream
// with its own device arena and pinned staging buffers.  Whenever a slot is
// free, the requests that have arrived are admitted in arrival order while the
// slot's memory budget (nonzeros, output words, queries) allows; the rest wait
// for the next slot.  A batch is packed host-side into one CSR grouped by k
// (search requests first inside the k = 1024 group, so their 1-bit sketches
// are contiguous), copied to the device, sketched by one launch per k, the
// search requests' sketches are scanned against the device-resident database,
// and the results come back to pinned memory.  Batches overlap on the device;
// completion is observed with events.  Each request's result depends only on
// its own set, never on its batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <unordered_map>
#include <thread>
#include <vector>

#include "../../include/dms.h"
#include "dms_internal.h"
#include "dms_launch.h"


namespace {

constexpr int kKinds[3] = {64, 256, 1024};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    // device arena
    int64_t* d_rp = nullptr;
    int32_t* d_idx = nullptr;
    double* d_w = nullptr;
    uint32_t* d_u32 = nullptr;
    uint64_t* d_bits = nullptr;
    int8_t* d_status = nullptr;
    int64_t* d_ids = nullptr;
    int32_t* d_dist = nullptr;
    uint64_t* d_partial = nullptr;
    unsigned long long* d_counter = nullptr;
    dms::Part* d_parts = nullptr;          // heavy-set plan of the batch
    dms::HeavySet* d_heavy = nullptr;
    uint64_t* d_part_buckets = nullptr;    // 2k words per part
    dms::Part* h_parts = nullptr;
    dms::HeavySet* h_heavy = nullptr;
    // pinned host staging
    int64_t* h_rp = nullptr;
    int32_t* h_idx = nullptr;
    double* h_w = nullptr;
    uint32_t* h_u32 = nullptr;
    int8_t* h_status = nullptr;
    int64_t* h_ids = nullptr;
    int32_t* h_dist = nullptr;
    // batch bookkeeping
    bool busy = false;
    std::vector<int64_t> reqs;       // request index per batch row, in row order
    std::vector<int64_t> out_off;    // offset of each row's minhashes in d_u32
    std::vector<int64_t> query_row;  // batch row of each search query
    int64_t n_u32 = 0, n_q = 0;
    // online batches: the request id and k of each batch-local request index
    std::vector<int64_t> online_id;
    std::vector<int32_t> online_k;
};

// A request submitted online, waiting for a slot or in flight.
struct OnlineReq {
    int32_t kind = 0, k = 0;
    std::vector<int32_t> idx;
    std::vector<double> w;
    double t_submit = 0.0;
};

// An answer waiting to be polled.
struct OnlineDone {
    int64_t id = 0;
    int32_t k = 0;
    int8_t status = 0;
    bool search = false;
    std::vector<uint32_t> sketch;
    std::vector<int64_t> ids;
    std::vector<int32_t> dist;
    double latency = 0.0;
};

}  // namespace

struct dms_server_s {
    dms_ctx ctx = nullptr;
    dms_server_config cfg{};
    const uint64_t* db = nullptr;
    int64_t n_db = 0;
    int hamming_blocks = 1;
    std::vector<Slot> slots;
    // online use (dms_server_submit / dms_server_poll)
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    int64_t next_id = 0;
    std::deque<int64_t> waiting;                      // submitted, not yet in a batch
    std::unordered_map<int64_t, OnlineReq> requests;  // submitted, not yet answered
    std::deque<OnlineDone> answers;                   // answered, not yet polled
    int64_t in_flight = 0;                            // online requests on the GPU
};

namespace {

template <class T>
hipError_t dev_alloc(T** p, size_t n)
{
    return hipMalloc((void**)p, n * sizeof(T) + 16);
}
template <class T>
hipError_t host_alloc(T** p, size_t n)
{
    return hipHostMalloc((void**)p, n * sizeof(T) + 16, hipHostMallocDefault);
}

void free_slot(Slot& s)
{
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    (void)hipFree(s.d_rp); (void)hipFree(s.d_idx); (void)hipFree(s.d_w); (void)hipFree(s.d_u32);
    (void)hipFree(s.d_bits); (void)hipFree(s.d_status); (void)hipFree(s.d_ids);
    (void)hipFree(s.d_dist); (void)hipFree(s.d_partial); (void)hipFree(s.d_counter);
    (void)hipFree(s.d_parts); (void)hipFree(s.d_heavy); (void)hipFree(s.d_part_buckets);
    (void)hipHostFree(s.h_parts); (void)hipHostFree(s.h_heavy);
    (void)hipHostFree(s.h_rp); (void)hipHostFree(s.h_idx); (void)hipHostFree(s.h_w);
    (void)hipHostFree(s.h_u32); (void)hipHostFree(s.h_status); (void)hipHostFree(s.h_ids);
    (void)hipHostFree(s.h_dist);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    s = Slot();
}

// Launch one batch on slot s.  Rows are the requests in `take`.
dms_status launch_batch(dms_server_s* S, Slot& s, const std::vector<int64_t>& take,
                        const int32_t* kind, const int32_t* kval, const int64_t* row_ptr,
                        const int32_t* idx, const double* w)
{
    const dms_server_config& C = S->cfg;
    // order rows: by k group, search requests first inside the k = 1024 group
    std::vector<int64_t> order;
    order.reserve(take.size());
    for (int g = 0; g < 3; ++g) {
        if (kKinds[g] == 1024) {
            for (int64_t r : take) if (kval[r] == 1024 && kind[r] == DMS_REQ_SEARCH) order.push_back(r);
            for (int64_t r : take) if (kval[r] == 1024 && kind[r] != DMS_REQ_SEARCH) order.push_back(r);
        } else {
            for (int64_t r : take) if (kval[r] == kKinds[g]) order.push_back(r);
        }
    }
    s.reqs = order;
    s.out_off.assign(order.size(), 0);
    s.query_row.clear();
    // pack the CSR and the output offsets
    int64_t nnz = 0, u32 = 0;
    s.h_rp[0] = 0;
    for (size_t i = 0; i < order.size(); ++i) {
        const int64_t r = order[i];
        const int64_t b0 = row_ptr[r], n = row_ptr[r + 1] - b0;
        std::memcpy(s.h_idx + nnz, idx + b0, (size_t)n * sizeof(int32_t));
        std::memcpy(s.h_w + nnz, w + b0, (size_t)n * sizeof(double));
        nnz += n;
        s.h_rp[i + 1] = nnz;
        s.out_off[i] = u32;
        u32 += kval[r];
        if (kind[r] == DMS_REQ_SEARCH) s.query_row.push_back((int64_t)i);
    }
    s.n_u32 = u32;
    s.n_q = (int64_t)s.query_row.size();
    const int64_t rows = (int64_t)order.size();
    hipStream_t st = s.stream;
    (void)hipGetLastError();  // the launches below report their own errors only
    hipError_t e = hipMemcpyAsync(s.d_rp, s.h_rp, (rows + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nnz)
        e = hipMemcpyAsync(s.d_idx, s.h_idx, nnz * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nnz)
        e = hipMemcpyAsync(s.d_w, s.h_w, nnz * sizeof(double), hipMemcpyHostToDevice, st);
    // one sketch launch per k group
    int64_t row0 = 0;
    int64_t part_base = 0, part_heavy = 0, bucket_base = 0;  // plan space used by earlier groups
    for (int g = 0; g < 3 && e == hipSuccess; ++g) {
        const int k = kKinds[g];
        int64_t n = 0;
        while (row0 + n < rows && kval[order[row0 + n]] == k) ++n;
        if (n == 0) continue;
        const dms::SpecTables* sp = nullptr;
        if (dms::ctx_spec(S->ctx, dms::t_of_k(k), &sp) != DMS_OK) return DMS_ESPEC;
        uint32_t* o32 = s.d_u32 + s.out_off[row0];
        // 1-bit sketches are needed only for the search queries (k = 1024)
        uint64_t* obits = k == 1024 ? s.d_bits : nullptr;
        if (dms::fast_lds_bytes(k, 1) <= 65536) {
            // sets above the split threshold are shared by several waves: the
            // plan is made here from the host copy of the batch
            const int64_t split = C.split_nnz;
            int64_t n_parts = 0, n_heavy = 0;
            if (split > 0) {
                for (int64_t i = row0; i < row0 + n; ++i) {
                    const int64_t len = s.h_rp[i + 1] - s.h_rp[i];
                    if (len <= split) continue;
                    dms::HeavySet& h = s.h_heavy[part_heavy + n_heavy];
                    h.sum = 0.0;
                    h.set = i - row0;
                    h.base = n_parts;
                    h.parts = (int32_t)((len + split - 1) / split);
                    h.done = 0;
                    h.range = 0;
                    h.status = 0;
                    for (int32_t q = 0; q < h.parts; ++q) {
                        dms::Part& pt = s.h_parts[part_base + n_parts + q];
                        pt.set = i - row0;
                        pt.heavy = (int32_t)n_heavy;
                        pt.index = q;
                    }
                    n_parts += h.parts;
                    ++n_heavy;
                }
            }
            dms::Part* dp = s.d_parts + part_base;
            dms::HeavySet* dh = s.d_heavy + part_heavy;
            uint64_t* db = s.d_part_buckets + bucket_base;
            if (n_parts > 0) {
                e = hipMemcpyAsync(dp, s.h_parts + part_base, n_parts * sizeof(dms::Part), hipMemcpyHostToDevice, st);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(dh, s.h_heavy + part_heavy, n_heavy * sizeof(dms::HeavySet),
                                       hipMemcpyHostToDevice, st);
                if (e == hipSuccess) e = dms::launch_heavy_scan(n_heavy, s.d_rp + row0, s.d_w, dh, st);
            }
            if (e == hipSuccess)
                e = dms::launch_sketch_fast_split(sp, n, s.d_rp + row0, s.d_idx, s.d_w, k, o32, obits,
                                                  s.d_status + row0, nullptr, nullptr, dms::ctx_phi0(S->ctx),
                                                  dms::ctx_phi_max(S->ctx), s.d_counter + g,
                                                  2 * dms::ctx_n_cu(S->ctx), dp, n_parts, dh, db,
                                                  n_parts > 0 ? split : 0, nullptr, dms::ctx_hash(S->ctx),
                                                  dms::LaunchExtras{}, nullptr, nullptr, 0, 0, st);
            part_base += n_parts;
            part_heavy += n_heavy;
            bucket_base += n_parts * 2 * (int64_t)k;
        } else {
            e = dms::launch_sketch_plain(sp, n, s.d_rp + row0, s.d_idx, s.d_w, k, o32, obits,
                                         s.d_status + row0, nullptr, nullptr, dms::ctx_phi0(S->ctx),
                                         dms::ctx_phi_max(S->ctx), dms::ctx_hash(S->ctx), dms::LaunchExtras{}, st);
        }
        row0 += n;
    }
    // the search queries are the first rows of the k = 1024 group
    if (e == hipSuccess && s.n_q > 0) {
        e = dms::launch_hamming(S->db, S->n_db, C.db_words, s.d_bits, s.n_q, C.topk, s.d_ids,
                                s.d_dist, s.d_partial, S->hamming_blocks, st);
    }
    if (e == hipSuccess && u32)
        e = hipMemcpyAsync(s.h_u32, s.d_u32, u32 * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.h_status, s.d_status, rows, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && s.n_q) {
        e = hipMemcpyAsync(s.h_ids, s.d_ids, s.n_q * C.topk * sizeof(int64_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s.h_dist, s.d_dist, s.n_q * C.topk * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipEventRecord(s.done, st);
    if (e != hipSuccess) return DMS_EHIP;
    s.busy = true;
    return DMS_OK;
}

}  // namespace

extern "C" {

dms_status dms_server_create(dms_ctx ctx, const dms_server_config* cfg, dms_db database, dms_server* out)
{
    if (!ctx || !cfg || !out || !database) return DMS_EINVAL;
    {
        dms_sketch_info mine{};
        (void)dms_sketch_info_of(ctx, 1024, &mine);
        const dms_sketch_info& theirs = *dms::db_info(database);
        if (theirs.spec_version != mine.spec_version || theirs.hash != mine.hash || theirs.seed != mine.seed ||
            theirs.k != mine.k)
            return DMS_EMISMATCH;
    }
    const uint64_t* db = dms::db_rows(database);
    const int64_t n_db = dms::db_count(database);
    const dms_server_config& C = *cfg;
    if (C.max_batch < 1 || C.max_batch > 4096 || C.max_inflight < 1 || C.max_inflight > 16 ||
        C.max_batch_nnz < 1 || C.db_words != 16 || C.topk < 1 || C.topk > 64 || C.max_set_nnz < 1 ||
        C.max_set_nnz > C.max_batch_nnz || C.split_nnz < 0 || (C.split_nnz > 0 && C.split_nnz < 16))
        return DMS_EINVAL;
    hipError_t e = hipSetDevice(dms::ctx_device(ctx));
    if (e != hipSuccess) return DMS_EHIP;
    auto* S = new dms_server_s;
    S->ctx = ctx;
    S->cfg = C;
    S->db = db;
    S->n_db = n_db;
    S->hamming_blocks = dms::hamming_blocks(n_db, dms::ctx_n_cu(ctx));
    S->slots.resize(C.max_inflight);
    const size_t rows = C.max_batch, nnz = C.max_batch_nnz, u32 = (size_t)C.max_batch * 1024;
    const size_t q = C.max_batch, tk = (size_t)C.topk;
    for (Slot& s : S->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess) e = dev_alloc(&s.d_rp, rows + 1);
        if (e == hipSuccess) e = dev_alloc(&s.d_idx, nnz);
        if (e == hipSuccess) e = dev_alloc(&s.d_w, nnz);
        if (e == hipSuccess) e = dev_alloc(&s.d_u32, u32);
        if (e == hipSuccess) e = dev_alloc(&s.d_bits, rows * 16);
        if (e == hipSuccess) e = dev_alloc(&s.d_status, rows);
        if (e == hipSuccess) e = dev_alloc(&s.d_ids, q * tk);
        if (e == hipSuccess) e = dev_alloc(&s.d_dist, q * tk);
        if (e == hipSuccess)
            e = hipMalloc((void**)&s.d_partial, dms::hamming_partial_bytes((int64_t)q, S->hamming_blocks, C.topk) + 16);
        if (e == hipSuccess) e = dev_alloc(&s.d_counter, 4);
        // the heavy-set plan: at most max_batch heavy sets and nnz/split + max_batch parts
        const size_t max_parts = C.split_nnz > 0 ? (size_t)(C.max_batch_nnz / C.split_nnz) + rows : 1;
        const size_t max_heavy = C.split_nnz > 0 ? rows : 1;
        if (e == hipSuccess) e = dev_alloc(&s.d_parts, max_parts);
        if (e == hipSuccess) e = dev_alloc(&s.d_heavy, max_heavy);
        if (e == hipSuccess) e = dev_alloc(&s.d_part_buckets, max_parts * 2 * 1024);
        if (e == hipSuccess) e = host_alloc(&s.h_parts, max_parts);
        if (e == hipSuccess) e = host_alloc(&s.h_heavy, max_heavy);
        if (e == hipSuccess) e = host_alloc(&s.h_rp, rows + 1);
        if (e == hipSuccess) e = host_alloc(&s.h_idx, nnz);
        if (e == hipSuccess) e = host_alloc(&s.h_w, nnz);
        if (e == hipSuccess) e = host_alloc(&s.h_u32, u32);
        if (e == hipSuccess) e = host_alloc(&s.h_status, rows);
        if (e == hipSuccess) e = host_alloc(&s.h_ids, q * tk);
        if (e == hipSuccess) e = host_alloc(&s.h_dist, q * tk);
    }
    if (e != hipSuccess) {
        for (Slot& s : S->slots) free_slot(s);
        delete S;
        return e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? DMS_ENOMEM : DMS_EHIP;
    }
    // make sure every k's tables exist before the first batch (no allocation in the loop)
    for (int k : kKinds) {
        const dms::SpecTables* sp = nullptr;
        if (dms::ctx_spec(ctx, dms::t_of_k(k), &sp) != DMS_OK) {
            for (Slot& s : S->slots) free_slot(s);
            delete S;
            return DMS_ESPEC;
        }
    }
    *out = S;
    return DMS_OK;
}

dms_status dms_server_destroy(dms_server S)
{
    if (!S) return DMS_EINVAL;
    (void)hipSetDevice(dms::ctx_device(S->ctx));
    for (Slot& s : S->slots) free_slot(s);
    delete S;
    return DMS_OK;
}

dms_status dms_server_replay(dms_server S, int64_t n_req, const double* arrival_s,
                             const int32_t* kind, const int32_t* kval, const int64_t* row_ptr,
                             const int32_t* idx, const double* w, const int64_t* sketch_off,
                             uint32_t* out_sketch, int8_t* out_status, int64_t* out_ids,
                             int32_t* out_dist, double* out_latency_s, double* out_stats)
{
    if (!S || n_req < 0 || (n_req > 0 && (!arrival_s || !kind || !kval || !row_ptr || !idx || !w)))
        return DMS_EINVAL;
    if (!S->requests.empty()) return DMS_EINVAL;  // online requests are still pending
    const dms_server_config& C = S->cfg;
    for (int64_t r = 0; r < n_req; ++r) {
        const int64_t n = row_ptr[r + 1] - row_ptr[r];
        if ((kval[r] != 64 && kval[r] != 256 && kval[r] != 1024) || n < 0 || n > C.max_set_nnz ||
            (kind[r] != DMS_REQ_SKETCH && kind[r] != DMS_REQ_SEARCH) ||
            (kind[r] == DMS_REQ_SEARCH && kval[r] != 1024) || (r > 0 && arrival_s[r] < arrival_s[r - 1]))
            return DMS_EINVAL;
    }
    if (hipSetDevice(dms::ctx_device(S->ctx)) != hipSuccess) return DMS_EHIP;
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    auto now = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };
    std::deque<int64_t> pending;
    int64_t next = 0, completed = 0, batches = 0, batch_rows = 0;
    dms_status status = DMS_OK;
    while (completed < n_req && status == DMS_OK) {
        const double t = now();
        while (next < n_req && arrival_s[next] <= t) pending.push_back(next++);
        bool progress = false;
        // completions
        for (Slot& s : S->slots) {
            if (!s.busy) continue;
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) { status = DMS_EHIP; break; }
            const double tc = now();
            for (size_t i = 0; i < s.reqs.size(); ++i) {
                const int64_t r = s.reqs[i];
                if (out_sketch && sketch_off)
                    std::memcpy(out_sketch + sketch_off[r], s.h_u32 + s.out_off[i], (size_t)kval[r] * sizeof(uint32_t));
                if (out_status) out_status[r] = s.h_status[i];
                if (out_latency_s) out_latency_s[r] = tc - arrival_s[r];
            }
            for (int64_t qi = 0; qi < s.n_q; ++qi) {
                const int64_t r = s.reqs[s.query_row[qi]];
                if (out_ids) std::memcpy(out_ids + r * C.topk, s.h_ids + qi * C.topk, C.topk * sizeof(int64_t));
                if (out_dist) std::memcpy(out_dist + r * C.topk, s.h_dist + qi * C.topk, C.topk * sizeof(int32_t));
            }
            completed += (int64_t)s.reqs.size();
            s.busy = false;
            progress = true;
        }
        if (status != DMS_OK) break;  // a failed slot: launch nothing more
        // admission into a free slot, in arrival order, within the slot's memory
        if (!pending.empty()) {
            for (Slot& s : S->slots) {
                if (s.busy || pending.empty()) continue;
                std::vector<int64_t> take;
                int64_t nnz = 0;
                while (!pending.empty() && (int64_t)take.size() < C.max_batch) {
                    const int64_t r = pending.front();
                    const int64_t n = row_ptr[r + 1] - row_ptr[r];
                    if (nnz + n > C.max_batch_nnz) break;  // waits for the next slot
                    nnz += n;
                    take.push_back(r);
                    pending.pop_front();
                }
                status = launch_batch(S, s, take, kind, kval, row_ptr, idx, w);
                if (status != DMS_OK) break;
                ++batches;
                batch_rows += (int64_t)take.size();
                progress = true;
            }
        }
        if (!progress && completed < n_req) {
            // nothing to do: wait a little for arrivals or completions
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    const double total = now();
    if (status != DMS_OK) {
        for (Slot& s : S->slots) (void)hipStreamSynchronize(s.stream);
        for (Slot& s : S->slots) s.busy = false;
        return status;
    }
    if (out_stats) {
        std::vector<double> lat;
        if (out_latency_s) lat.assign(out_latency_s, out_latency_s + n_req);
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            if (lat.empty()) return 0.0;
            size_t i = (size_t)(p * (double)(lat.size() - 1) + 0.5);
            return lat[i];
        };
        out_stats[0] = total > 0 ? (double)n_req / total : 0.0;  // completed requests per second
        out_stats[1] = pct(0.50);
        out_stats[2] = pct(0.99);
        out_stats[3] = lat.empty() ? 0.0 : lat.back();
        out_stats[4] = (double)batches;
        out_stats[5] = batches ? (double)batch_rows / (double)batches : 0.0;
        out_stats[6] = total;
    }
    return DMS_OK;
}

dms_status dms_server_submit(dms_server S, int32_t kind, int32_t k, int64_t nnz, const int32_t* idx,
                             const double* w, int64_t* out_id)
{
    if (!S || !out_id || nnz < 0 || (nnz > 0 && (!idx || !w))) return DMS_EINVAL;
    const dms_server_config& C = S->cfg;
    if ((k != 64 && k != 256 && k != 1024) || nnz > C.max_set_nnz ||
        (kind != DMS_REQ_SKETCH && kind != DMS_REQ_SEARCH) || (kind == DMS_REQ_SEARCH && k != 1024))
        return DMS_EINVAL;
    OnlineReq r;
    r.kind = kind;
    r.k = k;
    r.idx.assign(idx, idx + nnz);
    r.w.assign(w, w + nnz);
    r.t_submit = std::chrono::duration<double>(std::chrono::steady_clock::now() - S->t0).count();
    const int64_t id = S->next_id++;
    S->requests.emplace(id, std::move(r));
    S->waiting.push_back(id);
    *out_id = id;
    return DMS_OK;
}

dms_status dms_server_poll(dms_server S, int32_t wait_ms, int64_t max_out, int64_t* out_id,
                           int8_t* out_status, uint32_t* out_sketch, int64_t* out_ids, int32_t* out_dist,
                           double* out_latency_s, int64_t* n_out)
{
    if (!S || !n_out || max_out < 0 || (max_out > 0 && !out_id)) return DMS_EINVAL;
    *n_out = 0;
    const dms_server_config& C = S->cfg;
    if (hipSetDevice(dms::ctx_device(S->ctx)) != hipSuccess) return DMS_EHIP;
    using clk = std::chrono::steady_clock;
    const auto until = clk::now() + std::chrono::milliseconds(wait_ms > 0 ? wait_ms : 0);
    for (;;) {
        // completions
        for (Slot& s : S->slots) {
            if (!s.busy || s.online_id.empty()) continue;
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return DMS_EHIP;
            const double tc = std::chrono::duration<double>(clk::now() - S->t0).count();
            std::vector<int64_t> search_row(s.reqs.size(), -1);
            for (int64_t qi = 0; qi < s.n_q; ++qi) search_row[(size_t)s.query_row[qi]] = qi;
            for (size_t i = 0; i < s.reqs.size(); ++i) {
                const int64_t local = s.reqs[i];
                OnlineDone d;
                d.id = s.online_id[(size_t)local];
                d.k = s.online_k[(size_t)local];
                d.status = s.h_status[i];
                d.sketch.assign(s.h_u32 + s.out_off[i], s.h_u32 + s.out_off[i] + d.k);
                if (search_row[i] >= 0) {
                    const int64_t qi = search_row[i];
                    d.search = true;
                    d.ids.assign(s.h_ids + qi * C.topk, s.h_ids + (qi + 1) * C.topk);
                    d.dist.assign(s.h_dist + qi * C.topk, s.h_dist + (qi + 1) * C.topk);
                }
                auto it = S->requests.find(d.id);
                d.latency = tc - it->second.t_submit;
                S->requests.erase(it);
                S->answers.push_back(std::move(d));
            }
            S->in_flight -= (int64_t)s.reqs.size();
            s.online_id.clear();
            s.online_k.clear();
            s.busy = false;
        }
        // admission into free slots, in submission order, within each slot's memory
        for (Slot& s : S->slots) {
            if (s.busy || S->waiting.empty()) continue;
            std::vector<int32_t> kind_b, k_b, idx_b;
            std::vector<double> w_b;
            std::vector<int64_t> rp_b(1, 0), take;
            int64_t nnz = 0;
            while (!S->waiting.empty() && (int64_t)take.size() < C.max_batch) {
                const OnlineReq& r = S->requests.at(S->waiting.front());
                const int64_t n = (int64_t)r.idx.size();
                if (nnz + n > C.max_batch_nnz) break;  // waits for the next slot
                kind_b.push_back(r.kind);
                k_b.push_back(r.k);
                idx_b.insert(idx_b.end(), r.idx.begin(), r.idx.end());
                w_b.insert(w_b.end(), r.w.begin(), r.w.end());
                nnz += n;
                rp_b.push_back(nnz);
                s.online_id.push_back(S->waiting.front());
                s.online_k.push_back(r.k);
                take.push_back((int64_t)take.size());
                S->waiting.pop_front();
            }
            const dms_status st = launch_batch(S, s, take, kind_b.data(), k_b.data(), rp_b.data(),
                                               idx_b.data(), w_b.data());
            if (st != DMS_OK) {
                // the batch never ran: its requests go back to the head of the queue
                for (auto it = s.online_id.rbegin(); it != s.online_id.rend(); ++it) S->waiting.push_front(*it);
                s.online_id.clear();
                s.online_k.clear();
                return st;
            }
            S->in_flight += (int64_t)take.size();
        }
        if (!S->answers.empty() || S->in_flight == 0 || clk::now() >= until) break;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    int64_t n = 0;
    while (n < max_out && !S->answers.empty()) {
        const OnlineDone& d = S->answers.front();
        out_id[n] = d.id;
        if (out_status) out_status[n] = d.status;
        if (out_sketch) std::memcpy(out_sketch + n * 1024, d.sketch.data(), (size_t)d.k * sizeof(uint32_t));
        if (d.search) {
            if (out_ids) std::memcpy(out_ids + n * C.topk, d.ids.data(), (size_t)C.topk * sizeof(int64_t));
            if (out_dist) std::memcpy(out_dist + n * C.topk, d.dist.data(), (size_t)C.topk * sizeof(int32_t));
        }
        if (out_latency_s) out_latency_s[n] = d.latency;
        S->answers.pop_front();
        ++n;
    }
    *n_out = n;
    return DMS_OK;
}

}  // extern "C"
