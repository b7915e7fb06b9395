// C ABI of the DartMinHash library: argument checking, per-t device tables,
// engine dispatch.  Kernels live in the .hip files.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/dms.h"
#include "dms_internal.h"
#include "dms_launch.h"


struct dms_ctx_s {
    int device = 0;
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    hipEvent_t switch_event = nullptr;  // orders work across dms_set_stream
    int engine = DMS_ENGINE_FAST;
    int n_cu = 0;
    unsigned long long* counter = nullptr;  // work-stealing cursor of the fast engine
    void* scratch = nullptr;                 // search partial results, grown on demand
    size_t scratch_bytes = 0;
    double split_nnz = 4096;                 // sets with more nonzeros are cut into parts
    unsigned long long* plan = nullptr;      // planning counters of the fast engine
    void* parts = nullptr;                   // part descriptors, heavy sets, partial buckets
    size_t parts_bytes = 0;
    void* heavy = nullptr;
    size_t heavy_bytes = 0;
    uint64_t* partial = nullptr;
    size_t partial_bytes = 0;
    void* planned = nullptr;                 // per set: served by parts of the device plan
    size_t planned_bytes = 0;
    void* repeated = nullptr;                // per set: repeated ids (DMS_FLAG_VALIDATE)
    size_t repeated_bytes = 0;
    // first phi of the minhash schedule: at 1.3 a second pass is needed with
    // probability about k^(1-phi) e^(-phi) (0.07 at k = 256), which costs less
    // than the larger first pass saves (Theorem 1's retry argument)
    double phi0 = 1.3;
    double lsh_phi0 = 2.5;  // (64,8) LSH: fastest of 2, 2.5, 3, 3.5, 4 on 1M sets
    double bottomk_phi0 = 0.0;  // 0: 1 + 3/sqrt(k)
    int hash = dms::kHashMix;   // DMS_HASH_*
    int order = 1;              // DMS_OPT_ORDER: largest sets first
    int waves = 0;              // DMS_OPT_WAVES: waves per block of the minhash kernel (0: automatic)
    int tile = 0;               // DMS_OPT_TILE: buckets per tile of the minhash kernel (0: automatic)
    void* order_buf = nullptr;  // its keys, values and sort scratch
    size_t order_bytes = 0;
    double phi_max = 1048576.0;
    std::map<uint32_t, dms::SpecTables*> spec;  // device copies, keyed by t
    std::string err;
    // DMS_OPT_TIMING: event pairs around the main kernel of each sketching
    // call since the last dms_kernel_time (the pool is reused)
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
    size_t n_timed = 0;
};

namespace {

dms_status fail(dms_ctx c, dms_status code, const char* fmt, ...)
    __attribute__((format(printf, 3, 4)));

dms_status fail(dms_ctx c, dms_status code, const char* fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

dms_status hip_fail(dms_ctx c, hipError_t e, const char* what)
{
    return fail(c, DMS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Device copy of the specification tables for t, created on first use.
dms_status spec_for(dms_ctx c, uint32_t t, const dms::SpecTables** out)
{
    auto it = c->spec.find(t);
    if (it != c->spec.end()) {
        *out = it->second;
        return DMS_OK;
    }
    dms::SpecTables host;
    if (!dms::make_spec(c->seed, t, &host))
        return fail(c, DMS_ESPEC, "Poisson thresholds could not be derived exactly");
    dms::SpecTables* dev = nullptr;
    hipError_t e = hipMalloc((void**)&dev, sizeof host);
    if (e != hipSuccess) return fail(c, DMS_ENOMEM, "hipMalloc(spec tables): %s", hipGetErrorString(e));
    e = hipMemcpyAsync(dev, &host, sizeof host, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(c, e, "copy of spec tables");
    }
    c->spec[t] = dev;
    *out = dev;
    return DMS_OK;
}

// Make *buf hold at least `need` bytes of device memory (contents not kept).
// Replacing a buffer first waits for the stream, whose queued work may still
// use the old one.
dms_status grow(dms_ctx c, void** buf, size_t* have, size_t need)
{
    if (need <= *have) return DMS_OK;
    if (*buf) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
        (void)hipFree(*buf);
    }
    *buf = nullptr;
    *have = 0;
    const size_t bytes = need + need / 4 + 256;
    hipError_t e = hipMalloc(buf, bytes);
    if (e != hipSuccess) return fail(c, DMS_ENOMEM, "hipMalloc(%zu bytes of sketch scratch): %s", bytes, hipGetErrorString(e));
    *have = bytes;
    return DMS_OK;
}

// Blocks of the persistent kernel that fit on the device at once (blocks of
// `waves` waves, or of the automatic choice when 0).
int resident_blocks(dms_ctx c, int mode, int k, int K, int waves = 0)
{
    if (waves <= 0) waves = dms::fast_waves(mode, k, K);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dms::fast_kernel_address(mode, c->hash), 64 * waves,
                                                     dms::fast_lds(mode, k, K, waves)) != hipSuccess)
        per_cu = 1;
    // the query ignores the LDS allocation granule; take the smaller count
    const int by_lds = dms::fast_blocks_per_cu(mode, k, K, waves);
    if (by_lds < per_cu) per_cu = by_lds;
    if (per_cu < 1) per_cu = 1;
    return per_cu * c->n_cu;
}

// Largest-first order of the batch for the fast engine's cursor (DMS_OPT_ORDER),
// or nullptr for input order.
dms_status size_order(dms_ctx c, int64_t n_sets, const int64_t* row_ptr, const uint32_t** order)
{
    *order = nullptr;
    if (!c->order || n_sets < 2 || n_sets >= ((int64_t)1 << 31)) return DMS_OK;
    const size_t need = dms::size_order_bytes(n_sets);
    if (dms_status g = grow(c, &c->order_buf, &c->order_bytes, need); g != DMS_OK) return g;
    hipError_t e = dms::launch_size_order(n_sets, row_ptr, c->order_buf, c->order_bytes, order, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "size order");
    return DMS_OK;
}

// Checks flags and out_counters of a sketching call and, for DMS_FLAG_VALIDATE,
// flags the rows whose ids repeat; fills the launch extras.
dms_status prepare_extras(dms_ctx c, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                          uint32_t flags, int64_t* out_counters, dms::LaunchExtras* x)
{
    if (flags & ~(uint32_t)(DMS_FLAG_VALIDATE | DMS_FLAG_COUNTERS))
        return fail(c, DMS_EINVAL, "unknown flag bits 0x%x", flags);
    if (((flags & DMS_FLAG_COUNTERS) != 0) != (out_counters != nullptr))
        return fail(c, DMS_EINVAL, "out_counters must be given exactly when DMS_FLAG_COUNTERS is set");
    x->counters = out_counters;
    x->repeated = nullptr;
    if (flags & DMS_FLAG_VALIDATE) {
        if (dms_status g = grow(c, &c->repeated, &c->repeated_bytes, (size_t)n_sets); g != DMS_OK) return g;
        hipError_t e = dms::launch_repeated_ids(n_sets, row_ptr, idx, (uint8_t*)c->repeated, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "row validation");
        x->repeated = (const uint8_t*)c->repeated;
    }
    return DMS_OK;
}

// Parts a device plan may hold for a batch of n sets with k buckets: twice the
// sets (at least 1024), within 256 MiB of partial buckets.  Heavy sets beyond
// the capacity are sketched whole; the outputs are the same.
int64_t plan_capacity(int64_t n_sets, int32_t k)
{
    const int64_t by_bytes = ((int64_t)256 << 20) / (16 * (int64_t)k);
    int64_t cap = 2 * n_sets < 1024 ? 1024 : 2 * n_sets;
    if (cap > by_bytes) cap = by_bytes;
    return cap < 64 ? 64 : cap;
}

// Brackets the main kernel of a sketching call with events (DMS_OPT_TIMING).
struct KernelTimer {
    dms_ctx c;
    bool on = false;
    explicit KernelTimer(dms_ctx ctx) : c(ctx)
    {
        if (!c->timing) return;
        if (c->n_timed == c->timed.size()) {
            hipEvent_t a = nullptr, b = nullptr;
            if (hipEventCreate(&a) != hipSuccess) return;
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return;
            }
            c->timed.emplace_back(a, b);
        }
        on = hipEventRecord(c->timed[c->n_timed].first, c->stream) == hipSuccess;
    }
    void done()
    {
        if (on && hipEventRecord(c->timed[c->n_timed].second, c->stream) == hipSuccess) ++c->n_timed;
        on = false;
    }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        (void)hipGetLastError();  // a launch below reports its own error, not an earlier one
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace dms {
int ctx_spec(dms_ctx c, uint32_t t, const SpecTables** out) { return spec_for(c, t, out); }
const SpecTables* ctx_spec_cached(dms_ctx c, uint32_t t)
{
    auto it = c->spec.find(t);
    return it == c->spec.end() ? nullptr : it->second;
}
hipStream_t ctx_stream(dms_ctx c) { return c->stream; }
int ctx_engine(dms_ctx c) { return c->engine; }
int ctx_order(dms_ctx c) { return c->order; }
int ctx_resident_blocks(dms_ctx c, int mode, int k, int K) { return resident_blocks(c, mode, k, K); }
int ctx_fail(dms_ctx c, int code, const char* msg) { return fail(c, code, "%s", msg); }
void ctx_clear_error(dms_ctx c) { c->err.clear(); }
int ctx_device(dms_ctx c) { return c->device; }
int ctx_n_cu(dms_ctx c) { return c->n_cu; }
double ctx_phi0(dms_ctx c) { return c->phi0; }
double ctx_phi_max(dms_ctx c) { return c->phi_max; }
int ctx_hash(dms_ctx c) { return c->hash; }
uint64_t ctx_seed(dms_ctx c) { return c->seed; }
}  // namespace dms

extern "C" {

dms_status dms_create(dms_ctx* out, int device, uint64_t seed)
{
    if (!out) return DMS_EINVAL;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return DMS_EHIP;
    if (device < 0 || device >= n) return DMS_EINVAL;
    dms_ctx c = new dms_ctx_s;
    c->device = device;
    c->seed = seed;
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess ||
        hipMalloc((void**)&c->counter, 64) != hipSuccess ||
        hipMalloc((void**)&c->plan, 64) != hipSuccess ||
        hipEventCreateWithFlags(&c->switch_event, hipEventDisableTiming) != hipSuccess) {
        if (c->counter) (void)hipFree(c->counter);
        if (c->plan) (void)hipFree(c->plan);
        delete c;
        return DMS_EHIP;
    }
    c->n_cu = prop.multiProcessorCount;
    // the device's scratch of dms_sketch_csr_noalloc, looked up once per device
    if (dms::noalloc_setup(device) != hipSuccess) {
        (void)hipFree(c->counter);
        (void)hipFree(c->plan);
        (void)hipEventDestroy(c->switch_event);
        delete c;
        return DMS_EHIP;
    }
    *out = c;
    return DMS_OK;
}

dms_status dms_destroy(dms_ctx c)
{
    if (!c) return DMS_EINVAL;
    DeviceGuard g(c->device);
    for (auto& kv : c->spec) (void)hipFree(kv.second);
    if (c->counter) (void)hipFree(c->counter);
    if (c->scratch) (void)hipFree(c->scratch);
    if (c->plan) (void)hipFree(c->plan);
    if (c->parts) (void)hipFree(c->parts);
    if (c->heavy) (void)hipFree(c->heavy);
    if (c->partial) (void)hipFree(c->partial);
    if (c->order_buf) (void)hipFree(c->order_buf);
    if (c->planned) (void)hipFree(c->planned);
    if (c->repeated) (void)hipFree(c->repeated);
    if (c->switch_event) (void)hipEventDestroy(c->switch_event);
    for (auto& pr : c->timed) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    delete c;
    return DMS_OK;
}

dms_status dms_set_stream(dms_ctx c, void* s)
{
    if (!c) return DMS_EINVAL;
    hipStream_t next = (hipStream_t)s;
    if (next == c->stream) return DMS_OK;
    // The context's scratch (work cursor, plan, size order) is shared by its
    // calls: work queued on the new stream starts after the old stream's.  A
    // stream being captured into a graph cannot wait for work outside the
    // capture; then the switch adds no ordering.
    DeviceGuard g(c->device);
    // The new stream is asked first: while it captures, the old one (often the
    // null stream, which must not be touched during a capture) is left alone.
    hipStreamCaptureStatus a = hipStreamCaptureStatusActive, b = hipStreamCaptureStatusActive;
    bool plain = hipStreamIsCapturing(next, &b) == hipSuccess && b == hipStreamCaptureStatusNone;
    plain = plain && hipStreamIsCapturing(c->stream, &a) == hipSuccess && a == hipStreamCaptureStatusNone;
    (void)hipGetLastError();  // a refused capture query leaves no error behind
    if (plain) {
        hipError_t e = hipEventRecord(c->switch_event, c->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(next, c->switch_event, 0);
        if (e != hipSuccess) return hip_fail(c, e, "stream switch");
    }
    c->stream = next;
    return DMS_OK;
}

dms_status dms_set_option(dms_ctx c, int32_t opt, double v)
{
    if (!c) return DMS_EINVAL;
    switch (opt) {
    case DMS_OPT_ENGINE:
        if (v != DMS_ENGINE_FAST && v != DMS_ENGINE_PLAIN)
            return fail(c, DMS_EINVAL, "unknown engine %g", v);
        c->engine = (int)v;
        return DMS_OK;
    case DMS_OPT_HASH:
        if (v != DMS_HASH_MIX && v != DMS_HASH_TAB) return fail(c, DMS_EINVAL, "unknown hash %g", v);
        c->hash = (int)v;
        return DMS_OK;
    case DMS_OPT_ORDER:
        if (v != 0.0 && v != 1.0) return fail(c, DMS_EINVAL, "order must be 0 or 1");
        c->order = (int)v;
        return DMS_OK;
    case DMS_OPT_TIMING:
        if (v != 0.0 && v != 1.0) return fail(c, DMS_EINVAL, "timing must be 0 or 1");
        c->timing = v != 0.0;
        return DMS_OK;
    case DMS_OPT_WAVES:
        if (v != 0.0 && v != 1.0 && v != 2.0 && v != 3.0 && v != 4.0)
            return fail(c, DMS_EINVAL, "waves per block must be 0 (automatic) or 1..4");
        c->waves = (int)v;
        return DMS_OK;
    case DMS_OPT_TILE:
        if (!(v >= 0.0) || v > 4096.0 || v != (double)(int)v || ((int)v % 64 != 0))
            return fail(c, DMS_EINVAL, "buckets per tile must be 0 (automatic) or a multiple of 64 up to 4096");
        c->tile = (int)v;
        return DMS_OK;
    case DMS_OPT_SPLIT_NNZ:
        if (!(v >= 0.0) || v > 1e12 || v != (double)(int64_t)v)
            return fail(c, DMS_EINVAL, "split threshold must be a non-negative integer");
        c->split_nnz = v;
        return DMS_OK;
    case DMS_OPT_PHI0:
    case DMS_OPT_LSH_PHI0:
    case DMS_OPT_BOTTOMK_PHI0:
    case DMS_OPT_PHI_MAX:
        if (!(v > 0.0) || std::isinf(v)) return fail(c, DMS_EINVAL, "phi must be positive and finite");
        if (opt == DMS_OPT_PHI0) c->phi0 = v;
        else if (opt == DMS_OPT_LSH_PHI0) c->lsh_phi0 = v;
        else if (opt == DMS_OPT_BOTTOMK_PHI0) c->bottomk_phi0 = v;
        else c->phi_max = v;
        return DMS_OK;
    default:
        return fail(c, DMS_EINVAL, "unknown option %d", opt);
    }
}

dms_status dms_get_option(dms_ctx c, int32_t opt, double* v)
{
    if (!c || !v) return DMS_EINVAL;
    switch (opt) {
    case DMS_OPT_ENGINE: *v = c->engine; return DMS_OK;
    case DMS_OPT_PHI0: *v = c->phi0; return DMS_OK;
    case DMS_OPT_LSH_PHI0: *v = c->lsh_phi0; return DMS_OK;
    case DMS_OPT_BOTTOMK_PHI0: *v = c->bottomk_phi0; return DMS_OK;
    case DMS_OPT_PHI_MAX: *v = c->phi_max; return DMS_OK;
    case DMS_OPT_SPLIT_NNZ: *v = c->split_nnz; return DMS_OK;
    case DMS_OPT_HASH: *v = c->hash; return DMS_OK;
    case DMS_OPT_ORDER: *v = c->order; return DMS_OK;
    case DMS_OPT_TIMING: *v = c->timing ? 1.0 : 0.0; return DMS_OK;
    case DMS_OPT_WAVES: *v = c->waves; return DMS_OK;
    case DMS_OPT_TILE: *v = c->tile; return DMS_OK;
    default: return fail(c, DMS_EINVAL, "unknown option %d", opt);
    }
}

dms_status dms_sketch_csr(dms_ctx c, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                          const double* w, int32_t k, uint32_t* out_u32, uint64_t* out_bits,
                          int8_t* out_status, uint64_t* out_s, double* out_rank, uint32_t flags,
                          int64_t* out_counters)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (n_sets < 0) return fail(c, DMS_EINVAL, "n_sets < 0");
    if (k < 1 || k > 4096) return fail(c, DMS_EINVAL, "k = %d outside 1..4096", k);
    if (n_sets == 0) return DMS_OK;
    if (!row_ptr || !idx || !w) return fail(c, DMS_EINVAL, "NULL input pointer");
    DeviceGuard g(c->device);
    const dms::SpecTables* sp = nullptr;
    dms_status st = spec_for(c, dms::t_of_k(k), &sp);
    if (st != DMS_OK) return st;
    dms::LaunchExtras x;
    if ((st = prepare_extras(c, n_sets, row_ptr, idx, flags, out_counters, &x)) != DMS_OK) return st;
    hipError_t e;
    // the flattened engine keeps its queues and k buckets in one block's LDS;
    // beyond 64 KiB the plain engine serves the call
    const int kt = dms::minhash_tile_for(k, c->tile);  // buckets a wave holds at once (k unless k is large)
    const int waves = kt > 0 ? dms::minhash_waves_for(k, kt, c->waves) : 0;
    if (c->engine != DMS_ENGINE_PLAIN && (kt <= 0 || waves <= 0))
        return fail(c, DMS_EINVAL, "DMS_OPT_TILE / DMS_OPT_WAVES do not fit a block's 64 KiB of LDS at k = %d", k);
    if (c->engine == DMS_ENGINE_PLAIN) {
        KernelTimer tm(c);
        e = dms::launch_sketch_plain(sp, n_sets, row_ptr, idx, w, k, out_u32, out_bits,
                                     out_status, out_s, out_rank, c->phi0, c->phi_max, c->hash, x, c->stream);
        tm.done();
    } else {
        const int64_t split = kt < k ? 0 : (int64_t)c->split_nnz;  // tiled buckets: sets are not split
        int64_t part_cap = 0;
        if (split > 0) {
            // the heavy sets are planned on the device into scratch of a fixed
            // capacity, so the call only enqueues kernels
            part_cap = plan_capacity(n_sets, k);
            dms_status g2 = grow(c, &c->parts, &c->parts_bytes, (size_t)part_cap * dms::plan_part_bytes());
            if (g2 == DMS_OK)
                g2 = grow(c, &c->heavy, &c->heavy_bytes, (size_t)(part_cap / 2) * dms::plan_heavy_bytes());
            if (g2 == DMS_OK)
                g2 = grow(c, (void**)&c->partial, &c->partial_bytes, (size_t)part_cap * 16 * (size_t)k);
            if (g2 == DMS_OK) g2 = grow(c, &c->planned, &c->planned_bytes, (size_t)n_sets);
            if (g2 != DMS_OK) return g2;
            e = dms::launch_plan(n_sets, row_ptr, w, split, part_cap, c->plan, c->parts, c->heavy,
                                 (uint8_t*)c->planned, out_counters, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "sketch planning");
        }
        const uint32_t* order = nullptr;
        if (dms_status so = size_order(c, n_sets, row_ptr, &order); so != DMS_OK) return so;
        KernelTimer tm(c);
        e = dms::launch_sketch_fast_split(sp, n_sets, row_ptr, idx, w, k, out_u32, out_bits,
                                          out_status, out_s, out_rank, c->phi0, c->phi_max,
                                          c->counter, resident_blocks(c, dms::kModeMinhash, k, kt, waves), c->parts,
                                          part_cap, c->heavy, c->partial, split, order, c->hash, x,
                                          split > 0 ? c->plan : nullptr,
                                          split > 0 ? (const uint8_t*)c->planned : nullptr, kt, waves, c->stream);
        tm.done();
    }
    if (e != hipSuccess) return hip_fail(c, e, "sketch launch");
    return DMS_OK;
}

dms_status dms_bottomk(dms_ctx c, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                       const double* w, int32_t k, uint64_t* out_s, double* out_rank, int8_t* out_status,
                       uint32_t flags, int64_t* out_counters)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (n_sets < 0) return fail(c, DMS_EINVAL, "n_sets < 0");
    if (k < 1 || k > 1024) return fail(c, DMS_EINVAL, "k = %d outside 1..1024", k);
    if (n_sets == 0) return DMS_OK;
    if (!row_ptr || !idx || !w || !out_s) return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    const dms::SpecTables* sp = nullptr;
    dms_status st = spec_for(c, (uint32_t)k, &sp);  // t = k
    if (st != DMS_OK) return st;
    dms::LaunchExtras x;
    if ((st = prepare_extras(c, n_sets, row_ptr, idx, flags, out_counters, &x)) != DMS_OK) return st;
    // phi0 = 1 + 3/sqrt(k) finds k darts in the first pass but for a shortfall of about
    // 3 standard deviations (measured fastest at k = 256: 1.15-1.2 against 1.25 and 1.3)
    const double phi0 = c->bottomk_phi0 > 0.0 ? c->bottomk_phi0 : 1.0 + 3.0 / std::sqrt((double)k);
    const uint32_t* order = nullptr;
    if (dms_status so = size_order(c, n_sets, row_ptr, &order); so != DMS_OK) return so;
    KernelTimer tm(c);
    hipError_t e = dms::launch_bottomk_fast(sp, n_sets, row_ptr, idx, w, k, out_s, out_rank, out_status,
                                            phi0, c->phi_max, c->counter,
                                            resident_blocks(c, dms::kModeBottomK, k, 1), order, c->hash, x,
                                            c->stream);
    tm.done();
    if (e != hipSuccess) return hip_fail(c, e, "bottom-k launch");
    return DMS_OK;
}

dms_status dms_jaccard_est_bottomk(dms_ctx c, int64_t n_pairs, const double* rank_a, const uint64_t* s_a,
                                   const double* rank_b, const uint64_t* s_b, int32_t k, double* out)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (n_pairs < 0 || k < 1 || k > 1024) return fail(c, DMS_EINVAL, "bad n_pairs or k");
    if (n_pairs == 0) return DMS_OK;
    if (!rank_a || !s_a || !rank_b || !s_b || !out) return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    hipError_t e = dms::launch_bottomk_jaccard(n_pairs, rank_a, s_a, rank_b, s_b, k, out, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "bottom-k jaccard launch");
    return DMS_OK;
}

dms_status dms_lsh_keys(dms_ctx c, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                        const double* w, int32_t L, int32_t K, uint64_t* out_keys,
                        int8_t* out_status, uint32_t flags, int64_t* out_counters)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (n_sets < 0) return fail(c, DMS_EINVAL, "n_sets < 0");
    if (L < 1 || L > 1024 || K < 1 || K > 64 || (int64_t)L * K > 65536)
        return fail(c, DMS_EINVAL, "L = %d, K = %d out of range", L, K);
    if (n_sets == 0) return DMS_OK;
    if (!row_ptr || !idx || !w || !out_keys) return fail(c, DMS_EINVAL, "NULL pointer");
    if ((size_t)L * K * 16 + (size_t)L * 8 > 65536)
        return fail(c, DMS_EINVAL, "L*K too large for one wave's tables");
    DeviceGuard g(c->device);
    const dms::SpecTables* sp = nullptr;
    dms_status st = spec_for(c, (uint32_t)(L * K), &sp);
    if (st != DMS_OK) return st;
    dms::LaunchExtras x;
    if ((st = prepare_extras(c, n_sets, row_ptr, idx, flags, out_counters, &x)) != DMS_OK) return st;
    hipError_t e;
    if (c->engine == DMS_ENGINE_PLAIN || dms::fast_lds(dms::kModeLsh, L, K, 1) > 65536) {
        KernelTimer tm(c);
        e = dms::launch_lsh_plain(sp, n_sets, row_ptr, idx, w, L, K, out_keys, out_status,
                                  c->lsh_phi0, c->phi_max, c->hash, x, c->stream);
        tm.done();
    } else {
        const uint32_t* order = nullptr;
        if (dms_status so = size_order(c, n_sets, row_ptr, &order); so != DMS_OK) return so;
        KernelTimer tm(c);
        e = dms::launch_lsh_fast(sp, n_sets, row_ptr, idx, w, L, K, out_keys, out_status,
                                 c->lsh_phi0, c->phi_max, c->counter, resident_blocks(c, dms::lsh_fast_mode(L, K), L, K),
                                 order, c->hash, x, c->stream);
        tm.done();
    }
    if (e != hipSuccess) return hip_fail(c, e, "lsh launch");
    return DMS_OK;
}

dms_status dms_jaccard_est(dms_ctx c, int64_t n_pairs, const void* a, const void* b, int32_t k,
                           int32_t format, double* out)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (n_pairs < 0 || k < 1 || k > (1 << 20)) return fail(c, DMS_EINVAL, "bad n_pairs or k");
    if (format != DMS_FMT_U32 && format != DMS_FMT_1BIT) return fail(c, DMS_EINVAL, "bad format");
    if (n_pairs == 0) return DMS_OK;
    if (!a || !b || !out) return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    hipError_t e = dms::launch_jaccard(n_pairs, a, b, k, format, out, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "jaccard launch");
    return DMS_OK;
}

dms_status dms_bbit_pack(dms_ctx c, int64_t n_sets, const uint32_t* minhash, int32_t k, int32_t bits,
                         uint64_t* out)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (n_sets < 0 || k < 1 || k > (1 << 20) || bits < 1 || bits > 32)
        return fail(c, DMS_EINVAL, "bad n_sets, k or bits");
    if (n_sets == 0) return DMS_OK;
    if (!minhash || !out) return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    hipError_t e = dms::launch_bbit_pack(n_sets, minhash, k, bits, out, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "b-bit pack launch");
    return DMS_OK;
}

dms_status dms_jaccard_est_bbit(dms_ctx c, int64_t n_pairs, const uint64_t* a, const uint64_t* b,
                                int32_t k, int32_t bits, double* out)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (n_pairs < 0 || k < 1 || k > (1 << 20) || bits < 1 || bits > 32)
        return fail(c, DMS_EINVAL, "bad n_pairs, k or bits");
    if (n_pairs == 0) return DMS_OK;
    if (!a || !b || !out) return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    hipError_t e = dms::launch_bbit_jaccard(n_pairs, a, b, k, bits, out, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "b-bit jaccard launch");
    return DMS_OK;
}

dms_status dms_unary_map(dms_ctx c, int64_t n_sets, const uint32_t* minhash, int32_t k, int32_t bits,
                         int32_t* out_index, double* out_scale)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (n_sets < 0 || k < 1 || bits < 1 || bits > 16 || ((int64_t)k << bits) > (int64_t(1) << 31))
        return fail(c, DMS_EINVAL, "bad n_sets, k or bits");
    if (out_scale) *out_scale = 1.0 / std::sqrt((double)k);
    if (n_sets == 0) return DMS_OK;
    if (!minhash || !out_index) return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    hipError_t e = dms::launch_unary_map(n_sets, minhash, k, bits, out_index, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "unary map launch");
    return DMS_OK;
}

dms_status dms_hamming_topk(dms_ctx c, const uint64_t* db, int64_t n_db, int32_t words,
                            const uint64_t* queries, int64_t n_q, int32_t topk, int64_t* out_ids,
                            int32_t* out_dist)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (words < 1 || words > 64 || topk < 1 || topk > 64 || n_q < 0 || n_q > 4096 || n_db < 0 ||
        n_db >= 2147483648LL)
        return fail(c, DMS_EINVAL, "bad hamming arguments");
    if (n_q == 0) return DMS_OK;
    if (!queries || !out_ids || !out_dist || (n_db > 0 && !db)) return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    const int blocks = dms::hamming_blocks(n_db, c->n_cu);
    const size_t need = dms::hamming_partial_bytes(n_q, blocks, topk);
    if (need > c->scratch_bytes) {
        // the previous scratch may still be read by queued work on this stream
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
        if (c->scratch) (void)hipFree(c->scratch);
        c->scratch = nullptr;
        c->scratch_bytes = 0;
        e = hipMalloc(&c->scratch, need);
        if (e != hipSuccess) return fail(c, DMS_ENOMEM, "hipMalloc(search scratch): %s", hipGetErrorString(e));
        c->scratch_bytes = need;
    }
    hipError_t e = dms::launch_hamming(db, n_db, words, queries, n_q, topk, out_ids, out_dist,
                                       (uint64_t*)c->scratch, blocks, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hamming launch");
    return DMS_OK;
}

dms_status dms_calibrate(dms_ctx c, int32_t kind, int32_t iters, int64_t bytes, int32_t blocks,
                         void* a, void* b, double* out_ms)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (kind < 0 || kind > 3 || iters < 1 || blocks < 1 || !a || !out_ms ||
        (kind >= 2 && (!b || bytes < 16 || bytes % 16)))
        return fail(c, DMS_EINVAL, "bad calibration arguments");
    DeviceGuard g(c->device);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(c, DMS_EHIP, "event");
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(c, DMS_EHIP, "event"); }
    hipError_t e = hipEventRecord(e0, c->stream);
    if (e == hipSuccess) e = dms::calib_run(kind, iters, a, b, bytes, blocks, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(c, e, "calibration");
    *out_ms = ms;
    return DMS_OK;
}

dms_status dms_prepare(dms_ctx c, int32_t k)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (k < 1 || k > 4096) return fail(c, DMS_EINVAL, "k = %d outside 1..4096", k);
    DeviceGuard g(c->device);
    const dms::SpecTables* sp = nullptr;
    return spec_for(c, dms::t_of_k(k), &sp);
}

dms_status dms_kernel_time(dms_ctx c, double* out_ms, int64_t* out_launches)
{
    if (!c || !out_ms) return DMS_EINVAL;
    c->err.clear();
    DeviceGuard g(c->device);
    double total = 0.0;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < c->n_timed && e == hipSuccess; ++i) {
        e = hipEventSynchronize(c->timed[i].second);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->timed[i].first, c->timed[i].second);
        total += ms;
    }
    const int64_t n = (int64_t)c->n_timed;
    c->n_timed = 0;
    if (e != hipSuccess) return hip_fail(c, e, "kernel timing");
    *out_ms = total;
    if (out_launches) *out_launches = n;
    return DMS_OK;
}

dms_status dms_sync(dms_ctx c)
{
    if (!c) return DMS_EINVAL;
    DeviceGuard g(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
    return DMS_OK;
}

const char* dms_last_error(dms_ctx c) { return c ? c->err.c_str() : "null context"; }

const char* dms_status_str(dms_status s)
{
    switch (s) {
    case DMS_OK: return "DMS_OK";
    case DMS_EINVAL: return "DMS_EINVAL";
    case DMS_EHIP: return "DMS_EHIP";
    case DMS_ENOMEM: return "DMS_ENOMEM";
    case DMS_ESPEC: return "DMS_ESPEC";
    case DMS_EMISMATCH: return "DMS_EMISMATCH";
    default: return "unknown status";
    }
}

dms_status dms_t_of_k(int32_t k, uint32_t* t)
{
    if (k < 1 || k > (1 << 20) || !t) return DMS_EINVAL;
    *t = dms::t_of_k(k);
    return DMS_OK;
}

dms_status dms_spec_constants(uint64_t seed, uint32_t t, uint64_t keys[6], uint64_t pois[20],
                              double* W, double* R, double* u)
{
    if (t == 0) return DMS_EINVAL;
    dms::SpecTables sp;
    if (!dms::make_spec(seed, t, &sp)) return DMS_ESPEC;
    if (keys) {
        keys[0] = sp.key_r; keys[1] = sp.key_a; keys[2] = sp.key_u;
        keys[3] = sp.key_v; keys[4] = sp.key_s; keys[5] = sp.key_l;
    }
    if (pois) std::memcpy(pois, sp.pois, sizeof sp.pois);
    for (int i = 0; i < dms::kMaxIndex; ++i) {
        if (W) W[i] = dms::corner_w(sp, i);
        if (R) R[i] = dms::corner_r(sp, i);
    }
    if (u) *u = sp.u;
    return DMS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Weight-class LSH index

struct dms_index_s {
    dms_ctx ctx = nullptr;
    int64_t n = 0, n_ok = 0;
    int L = 0, K = 0;
    const int64_t* rp = nullptr;  // the caller's sets (read by verification)
    const int32_t* idx = nullptr;
    const double* w = nullptr;
    int32_t* cls = nullptr;       // per set: weight class and status
    int8_t* status = nullptr;
    uint64_t* tkeys = nullptr;    // L tables of n_ok sorted (key, value) pairs
    uint64_t* tvals = nullptr;
    void* q = nullptr;            // query scratch, grown on demand
    size_t q_bytes = 0;
};

namespace {

template <class T>
hipError_t ix_alloc(T** p, size_t n)
{
    *p = nullptr;
    return hipMalloc((void**)p, (n ? n : 1) * sizeof(T));
}

void ix_free(dms_index ix)
{
    (void)hipFree(ix->cls);
    (void)hipFree(ix->status);
    (void)hipFree(ix->tkeys);
    (void)hipFree(ix->tvals);
    (void)hipFree(ix->q);
    delete ix;
}

// ceil(log2(1/j1)) + 1 classes on each side of the query's
int class_span(double j1) { return (int)std::ceil(std::log2(1.0 / j1)) + 1; }

}  // namespace

dms_status dms_index_build(dms_ctx c, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx,
                           const double* w, int32_t L, int32_t K, dms_index* out)
{
    if (!c || !out) return DMS_EINVAL;
    c->err.clear();
    *out = nullptr;
    if (n_sets < 0 || n_sets >= (int64_t(1) << 31)) return fail(c, DMS_EINVAL, "n_sets outside 0..2^31-1");
    if (L < 1 || L > 1024 || K < 1 || K > 64 || (int64_t)L * K > 65536)
        return fail(c, DMS_EINVAL, "L = %d, K = %d out of range", L, K);
    if (n_sets > 0 && (!row_ptr || !idx || !w)) return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    hipStream_t st = c->stream;
    auto* ix = new dms_index_s;
    ix->ctx = c;
    ix->n = n_sets;
    ix->L = L;
    ix->K = K;
    ix->rp = row_ptr;
    ix->idx = idx;
    ix->w = w;
    int64_t nnz = 0;
    hipError_t e = hipSuccess;
    if (n_sets > 0) {
        e = hipMemcpyAsync(&nnz, row_ptr + n_sets, sizeof nnz, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    double* wn = nullptr;
    uint64_t *keys = nullptr, *okey = nullptr, *okey2 = nullptr, *tmp_k = nullptr, *tmp_v = nullptr;
    int64_t* ord = nullptr;
    int8_t* kst = nullptr;
    unsigned long long* n_ok_dev = nullptr;
    void* scratch = nullptr;
    const size_t scratch_bytes = dms::index_sort_scratch(n_sets > 0 ? n_sets : 1);
    if (e == hipSuccess) e = ix_alloc(&ix->cls, (size_t)n_sets);
    if (e == hipSuccess) e = ix_alloc(&ix->status, (size_t)n_sets);
    if (e == hipSuccess) e = ix_alloc(&wn, (size_t)nnz);
    if (e == hipSuccess) e = ix_alloc(&keys, (size_t)n_sets * L);
    if (e == hipSuccess) e = ix_alloc(&kst, (size_t)n_sets);
    if (e == hipSuccess) e = ix_alloc(&okey, (size_t)n_sets);
    if (e == hipSuccess) e = ix_alloc(&okey2, (size_t)n_sets);
    if (e == hipSuccess) e = ix_alloc(&ord, (size_t)n_sets);
    if (e == hipSuccess) e = ix_alloc(&tmp_k, (size_t)n_sets);
    if (e == hipSuccess) e = ix_alloc(&tmp_v, (size_t)n_sets);
    if (e == hipSuccess) e = ix_alloc(&n_ok_dev, 1);
    if (e == hipSuccess) e = hipMalloc(&scratch, scratch_bytes ? scratch_bytes : 1);
    dms_status rc = DMS_OK;
    if (e != hipSuccess) rc = fail(c, DMS_ENOMEM, "index allocation: %s", hipGetErrorString(e));
    if (rc == DMS_OK && n_sets > 0) {
        // classes and normalised weights, then the (L,K) keys of the normalised sets
        e = dms::launch_index_prep(n_sets, row_ptr, idx, w, wn, ix->cls, ix->status, st);
        if (e != hipSuccess) rc = hip_fail(c, e, "index prep");
        if (rc == DMS_OK) rc = dms_lsh_keys(c, n_sets, row_ptr, idx, wn, L, K, keys, kst, 0, nullptr);
        if (rc == DMS_OK) {
            e = dms::launch_index_order(n_sets, ix->cls, ix->status, okey, okey2, ord, n_ok_dev, scratch,
                                        scratch_bytes, st);
            unsigned long long n_ok = 0;
            if (e == hipSuccess) e = hipMemcpyAsync(&n_ok, n_ok_dev, sizeof n_ok, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            ix->n_ok = (int64_t)n_ok;
            if (e != hipSuccess) rc = hip_fail(c, e, "index order");
        }
        if (rc == DMS_OK) {
            e = ix_alloc(&ix->tkeys, (size_t)ix->n_ok * L);
            if (e == hipSuccess) e = ix_alloc(&ix->tvals, (size_t)ix->n_ok * L);
            if (e != hipSuccess) rc = fail(c, DMS_ENOMEM, "index tables: %s", hipGetErrorString(e));
        }
        for (int l = 0; rc == DMS_OK && l < L; ++l) {
            e = dms::launch_index_table(ix->n_ok, ord, keys, ix->cls, L, l, tmp_k, tmp_v,
                                        ix->tkeys + (size_t)l * ix->n_ok, ix->tvals + (size_t)l * ix->n_ok,
                                        scratch, scratch_bytes, st);
            if (e != hipSuccess) rc = hip_fail(c, e, "index table");
        }
        if (rc == DMS_OK) {
            e = hipStreamSynchronize(st);  // the temporaries below are freed next
            if (e != hipSuccess) rc = hip_fail(c, e, "index build");
        }
    }
    (void)hipFree(wn); (void)hipFree(keys); (void)hipFree(kst); (void)hipFree(okey); (void)hipFree(okey2);
    (void)hipFree(ord); (void)hipFree(tmp_k); (void)hipFree(tmp_v); (void)hipFree(n_ok_dev); (void)hipFree(scratch);
    if (rc != DMS_OK) {
        ix_free(ix);
        return rc;
    }
    *out = ix;
    return DMS_OK;
}

dms_status dms_index_sets(dms_index ix, int32_t* out_class, int8_t* out_status)
{
    if (!ix) return DMS_EINVAL;
    dms_ctx c = ix->ctx;
    c->err.clear();
    DeviceGuard g(c->device);
    hipError_t e = hipSuccess;
    if (out_class && ix->n)
        e = hipMemcpyAsync(out_class, ix->cls, (size_t)ix->n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && out_status && ix->n)
        e = hipMemcpyAsync(out_status, ix->status, (size_t)ix->n, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "index sets");
    return DMS_OK;
}

dms_status dms_index_query(dms_index ix, int64_t n_q, const int64_t* q_row_ptr, const int32_t* q_idx,
                           const double* q_w, double j1, int32_t topn, int64_t* out_ids, double* out_j,
                           int32_t* out_count, int32_t* out_candidates, int8_t* out_status)
{
    if (!ix) return DMS_EINVAL;
    dms_ctx c = ix->ctx;
    c->err.clear();
    if (n_q < 0 || !(j1 > 0.0 && j1 <= 1.0) || topn < 1 || topn > 1024)
        return fail(c, DMS_EINVAL, "bad n_q, j1 or topn");
    if (n_q == 0) return DMS_OK;
    if (!q_row_ptr || !q_idx || !q_w || !out_ids || !out_j || !out_count || !out_candidates || !out_status)
        return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    hipStream_t st = c->stream;
    const int span = class_span(j1), span2 = 2 * span + 1;
    int64_t q_nnz = 0;
    hipError_t e = hipMemcpyAsync(&q_nnz, q_row_ptr + n_q, sizeof q_nnz, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(c, e, "query size");
    // scratch: expanded CSR, its keys and statuses, per-query class and status
    const size_t rows = (size_t)n_q * span2;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_rp = 0, o_idx = o_rp + up((rows + 1) * 8), o_w = o_idx + up((size_t)q_nnz * span2 * 4);
    const size_t o_keys = o_w + up((size_t)q_nnz * span2 * 8), o_xst = o_keys + up(rows * ix->L * 8);
    const size_t o_qc = o_xst + up(rows), o_qs = o_qc + up((size_t)n_q * 4), total = o_qs + up((size_t)n_q);
    if (total > ix->q_bytes) {
        e = hipStreamSynchronize(st);  // earlier queries may still read the old scratch
        if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
        (void)hipFree(ix->q);
        ix->q = nullptr;
        ix->q_bytes = 0;
        e = hipMalloc(&ix->q, total);
        if (e != hipSuccess) return fail(c, DMS_ENOMEM, "query scratch: %s", hipGetErrorString(e));
        ix->q_bytes = total;
    }
    char* b = (char*)ix->q;
    int64_t* xrp = (int64_t*)(b + o_rp);
    int32_t* xidx = (int32_t*)(b + o_idx);
    double* xw = (double*)(b + o_w);
    uint64_t* qkeys = (uint64_t*)(b + o_keys);
    int8_t* xst = (int8_t*)(b + o_xst);
    int32_t* qcls = (int32_t*)(b + o_qc);
    int8_t* qst = (int8_t*)(b + o_qs);
    e = dms::launch_query_prep(n_q, q_row_ptr, q_idx, q_w, span, xrp, xidx, xw, qcls, qst, st);
    if (e != hipSuccess) return hip_fail(c, e, "query prep");
    dms_status rc = dms_lsh_keys(c, (int64_t)rows, xrp, xidx, xw, ix->L, ix->K, qkeys, xst, 0, nullptr);
    if (rc != DMS_OK) return rc;
    e = dms::launch_index_query(n_q, span, ix->L, qkeys, xst, qcls, qst, ix->tkeys, ix->tvals, ix->n_ok,
                                q_row_ptr, q_idx, q_w, ix->rp, ix->idx, ix->w, j1, topn, out_ids, out_j,
                                out_count, out_candidates, out_status, c->n_cu, st);
    if (e != hipSuccess) return hip_fail(c, e, "query launch");
    return DMS_OK;
}

dms_status dms_index_destroy(dms_index ix)
{
    if (!ix) return DMS_EINVAL;
    DeviceGuard g(ix->ctx->device);
    (void)hipStreamSynchronize(ix->ctx->stream);
    ix_free(ix);
    return DMS_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate schedules on a prefix of the caller's batch.

dms_status dms_autotune(dms_ctx c, int64_t n_sets, const int64_t* row_ptr, const int32_t* idx, const double* w,
                        int32_t k, double* out_phi0, double* out_split)
{
    if (!c) return DMS_EINVAL;
    c->err.clear();
    if (n_sets < 1 || k < 1 || k > 4096) return fail(c, DMS_EINVAL, "bad n_sets or k");
    if (!row_ptr || !idx || !w) return fail(c, DMS_EINVAL, "NULL pointer");
    DeviceGuard g(c->device);
    // a sample large enough that the last sets to finish weigh little in each
    // trial (shorter prefixes favour a large first phi, which trims the tail)
    const int64_t n = n_sets < ((int64_t)1 << 28) / k ? n_sets : ((int64_t)1 << 28) / k;
    uint32_t* out = nullptr;
    int8_t* st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void**)&out, (size_t)n * k * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&st, (size_t)n);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    dms_status rc = e == hipSuccess ? DMS_OK : fail(c, DMS_ENOMEM, "autotune buffers: %s", hipGetErrorString(e));
    // best of two timed launches after one warm-up; +inf on failure
    auto trial = [&](double phi0, double split) -> float {
        c->phi0 = phi0;
        c->split_nnz = split;
        float best = INFINITY;
        for (int r = 0; r < 3 && rc == DMS_OK; ++r) {
            hipError_t x = hipEventRecord(e0, c->stream);
            if (x != hipSuccess) { rc = hip_fail(c, x, "autotune event"); break; }
            rc = dms_sketch_csr(c, n, row_ptr, idx, w, k, out, nullptr, st, nullptr, nullptr, 0, nullptr);
            if (rc != DMS_OK) break;
            x = hipEventRecord(e1, c->stream);
            if (x == hipSuccess) x = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
            if (x != hipSuccess) { rc = hip_fail(c, x, "autotune timing"); break; }
            if (r > 0 && ms < best) best = ms;
        }
        return best;
    };
    const double keep_phi0 = c->phi0, keep_split = c->split_nnz;
    const int keep_order = c->order, keep_waves = c->waves, keep_tile = c->tile;
    double best_phi0 = keep_phi0, best_split = keep_split;
    int best_order = keep_order, best_waves = keep_waves, best_tile = keep_tile;
    if (rc == DMS_OK) {
        // coordinate search: the first phi, then the split threshold
        const double phis[] = {1.0, 1.15, 1.3, 1.5, 1.8};
        float best = INFINITY;
        for (double p : phis) {
            const float ms = trial(p, keep_split);
            if (ms < best) { best = ms; best_phi0 = p; }
        }
        const double splits[] = {0.0, 1024.0, 4096.0, 16384.0};
        best = trial(best_phi0, keep_split);
        for (double sp : splits) {
            if (sp == keep_split) continue;
            const float ms = trial(best_phi0, sp);
            if (ms < best) { best = ms; best_split = sp; }
        }
        // then the order in which waves take the sets
        c->order = 1 - keep_order;
        const float ms = trial(best_phi0, best_split);
        if (ms < best) {
            best = ms;
            best_order = c->order;
        }
        c->order = best_order;
        // then the block shape: waves per block, and buckets per tile (half the
        // automatic tile, twice the passes, more waves resident)
        const int auto_tile = dms::minhash_tile(k);
        const int tiles[2] = {0, auto_tile >= 128 ? (auto_tile / 2 + 63) / 64 * 64 : 0};
        for (int ti = 0; ti < 2 && rc == DMS_OK; ++ti) {
            if (ti == 1 && (tiles[1] == 0 || dms::minhash_tile_for(k, tiles[1]) <= 0)) continue;
            for (int wv = 0; wv <= 4 && rc == DMS_OK; ++wv) {
                if (ti == 0 && wv == 0) continue;  // the automatic shape, timed above
                const int kt = dms::minhash_tile_for(k, tiles[ti]);
                if (wv > 0 && dms::minhash_waves_for(k, kt, wv) <= 0) continue;
                c->tile = tiles[ti];
                c->waves = wv;
                const float mt = trial(best_phi0, best_split);
                if (mt < best) {
                    best = mt;
                    best_tile = tiles[ti];
                    best_waves = wv;
                }
            }
        }
    }
    (void)hipFree(out);
    (void)hipFree(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->phi0 = rc == DMS_OK ? best_phi0 : keep_phi0;
    c->split_nnz = rc == DMS_OK ? best_split : keep_split;
    c->order = rc == DMS_OK ? best_order : keep_order;
    c->waves = rc == DMS_OK ? best_waves : keep_waves;
    c->tile = rc == DMS_OK ? best_tile : keep_tile;
    if (rc != DMS_OK) return rc;
    if (out_phi0) *out_phi0 = best_phi0;
    if (out_split) *out_split = best_split;
    return DMS_OK;
}

dms_status dms_spec_tabulation(uint64_t seed, uint64_t* out)
{
    if (!out) return DMS_EINVAL;
    dms::hash_tables(seed, out);
    return DMS_OK;
}
