// dms_sketch_csr_noalloc: the DartMinHash batch call for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).
// Its scratch -- the persistent kernel's work cursor and the size order's keys,
// values and sort space -- lives in a file-scope device array that every GPU
// holds from module load until the process ends; the call itself allocates
// nothing.  Calls on one GPU share that array, so calls that overlap on one GPU
// (other streams, other contexts) race; each call clears what must start at zero.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/dms.h"
#include "dms_internal.h"
#include "dms_launch.h"

namespace dms {

namespace {

constexpr int64_t kNoAllocMaxSets = (int64_t)1 << 20;  // largest batch of the call
constexpr size_t kCursorBytes = 256;                   // work cursor, then the size order
constexpr size_t kScratchBytes = (size_t)16 << 20;     // 16 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};  // the array's address on each device (host side)
bool g_fits = false;            // the size order of kNoAllocMaxSets sets fits behind the cursor

}  // namespace

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = ptr;
    g_fits = kCursorBytes + size_order_bytes(kNoAllocMaxSets) <= kScratchBytes;
    return hipSuccess;
}

}  // namespace dms

extern "C" dms_status dms_sketch_csr_noalloc(dms_ctx c, int64_t n_sets, const int64_t* row_ptr,
                                             const int32_t* idx, const double* w, int32_t k, uint32_t* out_u32,
                                             uint64_t* out_bits, int8_t* out_status)
{
    using namespace dms;
    if (!c) return DMS_EINVAL;
    ctx_clear_error(c);
    if (n_sets < 0) return ctx_fail(c, DMS_EINVAL, "n_sets < 0");
    if (n_sets > kNoAllocMaxSets)
        return ctx_fail(c, DMS_EINVAL, "n_sets above the no-alloc maximum of 2^20 sets per call");
    if (k < 1 || k > 4096) return ctx_fail(c, DMS_EINVAL, "k outside 1..4096");
    if (n_sets == 0) return DMS_OK;
    if (!row_ptr || !idx || !w) return ctx_fail(c, DMS_EINVAL, "NULL input pointer");
    const SpecTables* sp = ctx_spec_cached(c, t_of_k(k));
    if (!sp) return ctx_fail(c, DMS_EINVAL, "the context holds no tables for this k: call dms_prepare first");
    const int device = ctx_device(c);
    int prev = -1;
    (void)hipGetLastError();  // a launch below reports its own error, not an earlier one
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != device) (void)hipSetDevice(device);
    void* ptr = nullptr;
    bool fits = false;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        ptr = device < kMaxDevices ? g_ptr[device] : nullptr;
        fits = g_fits;
    }
    hipError_t e = hipSuccess;
    dms_status rc = DMS_OK;
    const hipStream_t st = ctx_stream(c);
    if (!ptr || !fits) {
        rc = ctx_fail(c, DMS_EHIP, "no-alloc scratch unavailable on this device");
    } else if (ctx_engine(c) == DMS_ENGINE_PLAIN) {
        // the plain engine needs no scratch
        e = launch_sketch_plain(sp, n_sets, row_ptr, idx, w, k, out_u32, out_bits, out_status, nullptr, nullptr,
                                ctx_phi0(c), ctx_phi_max(c), ctx_hash(c), LaunchExtras{}, st);
    } else {
        unsigned char* base = (unsigned char*)ptr;
        unsigned long long* cursor = (unsigned long long*)base;  // zeroed by the launch's reset kernel
        const uint32_t* order = nullptr;
        if (ctx_order(c) && n_sets >= 2)
            e = launch_size_order(n_sets, row_ptr, base + kCursorBytes, kScratchBytes - kCursorBytes, &order, st);
        // heavy sets are not split (as with DMS_OPT_SPLIT_NNZ = 0)
        if (e == hipSuccess)
            e = launch_sketch_fast_split(sp, n_sets, row_ptr, idx, w, k, out_u32, out_bits, out_status, nullptr,
                                         nullptr, ctx_phi0(c), ctx_phi_max(c), cursor,
                                         ctx_resident_blocks(c, kModeMinhash, k, minhash_tile(k)), nullptr, 0,
                                         nullptr, nullptr, 0,
                                         order, ctx_hash(c), LaunchExtras{}, nullptr, nullptr, 0, 0, st);
    }
    if (rc == DMS_OK && e != hipSuccess) rc = ctx_fail(c, DMS_EHIP, hipGetErrorString(e));
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    return rc;
}
