// Largest-first order of a batch for the work-stealing cursor of the fast
// engine.  Waves take sets in this order, so the longest sets start early and
// the launch ends on short ones (longest-processing-time-first scheduling).
// The key is a log-scale class of the set's nonzero count (eight classes per
// doubling); a stable one-pass radix sort keeps input order within a class.
// Only the order of work changes, never a result.
#include <hipcub/hipcub.hpp>

#include "dms_device.h"

namespace dms {

namespace {

__global__ void __launch_bounds__(256)
order_keys_kernel(int64_t n, const int64_t* __restrict__ rp, uint8_t* __restrict__ keys,
                  uint32_t* __restrict__ vals)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t c = rp[i + 1] - rp[i];
        uint32_t key = 0;
        if (c > 0) {
            const uint64_t v = (uint64_t)c;
            const int l = 63 - __builtin_clzll(v);  // floor(log2 c)
            const uint32_t m = l >= 3 ? (uint32_t)(v >> (l - 3)) & 7u : (uint32_t)(v << (3 - l)) & 7u;
            key = 8u * (uint32_t)l + m + 1u;
            if (key > 255u) key = 255u;
        }
        keys[i] = (uint8_t)key;
        vals[i] = (uint32_t)i;
    }
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t cub_bytes(int64_t n)
{
    size_t temp = 0;
    (void)hipcub::DeviceRadixSort::SortPairsDescending(nullptr, temp, (const uint8_t*)nullptr,
                                                       (uint8_t*)nullptr, (const uint32_t*)nullptr,
                                                       (uint32_t*)nullptr, (int)n, 0, 8);
    return temp;
}

}  // namespace

// Scratch for launch_size_order: keys and values twice, then the sort's own.
size_t size_order_bytes(int64_t n_sets)
{
    return 2 * align256((size_t)n_sets) + 2 * align256(4 * (size_t)n_sets) + align256(cub_bytes(n_sets));
}

// Writes the order into `scratch` (size_order_bytes(n_sets) bytes, n_sets < 2^31)
// and points *order at it.
hipError_t launch_size_order(int64_t n_sets, const int64_t* rp, void* scratch, size_t scratch_bytes,
                             const uint32_t** order, hipStream_t st)
{
    *order = nullptr;
    if (n_sets <= 0) return hipSuccess;
    if (scratch_bytes < size_order_bytes(n_sets)) return hipErrorInvalidValue;
    unsigned char* p = (unsigned char*)scratch;
    uint8_t* k_in = (uint8_t*)p;
    p += align256((size_t)n_sets);
    uint8_t* k_out = (uint8_t*)p;
    p += align256((size_t)n_sets);
    uint32_t* v_in = (uint32_t*)p;
    p += align256(4 * (size_t)n_sets);
    uint32_t* v_out = (uint32_t*)p;
    p += align256(4 * (size_t)n_sets);
    size_t temp = cub_bytes(n_sets);
    int64_t blocks = (n_sets + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(order_keys_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_sets, rp, k_in, v_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipcub::DeviceRadixSort::SortPairsDescending(p, temp, k_in, k_out, v_in, v_out, (int)n_sets, 0, 8, st);
    if (e == hipSuccess) *order = v_out;
    return e;
}

}  // namespace dms
