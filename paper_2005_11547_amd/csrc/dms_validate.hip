// Row validation for DMS_FLAG_VALIDATE: flags the sets that list an element id
// more than once.  Repeated ids are well defined for the method (the same
// darts are met twice) but usually signal malformed input, so callers may ask
// for them to be rejected.
#include "dms_device.h"
#include "dms_launch.h"

namespace dms {

namespace {

constexpr int kSlots = 2048;   // open-addressing slots per wave (load factor <= 1/2)
constexpr int kChunk = 1024;   // ids inserted per round
constexpr uint64_t kFree = ~0ull;  // never equal to a stored id (ids are 32-bit)

__device__ __forceinline__ uint32_t slot_of(uint32_t id)
{
    return (id * 0x9E3779B1u) >> (32 - 11);  // multiplicative hashing into 2^11 slots
}

}  // namespace

// One wave per row.  The row's ids enter a table in LDS a chunk at a time; an
// id meeting itself while its chunk is inserted, or found by a later id of the
// row looking the chunk up, marks the row.
__global__ void __launch_bounds__(256)
repeated_ids_kernel(int64_t n_sets, const int64_t* __restrict__ rp, const int32_t* __restrict__ idx,
                    uint8_t* out)
{
    __shared__ uint64_t table[4][kSlots];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t set = (int64_t)blockIdx.x * 4 + wave;
    if (set >= n_sets) return;  // whole wave leaves; no block barrier follows
    uint64_t* tab = table[wave];
    const int64_t b0 = rp[set], b1 = rp[set + 1];
    bool dup = false;
    for (int64_t c0 = b0; c0 < b1 && !wave_any(dup); c0 += kChunk) {
        const int64_t c1 = c0 + kChunk < b1 ? c0 + kChunk : b1;
        for (int i = lane; i < kSlots; i += kWave) tab[i] = kFree;
        wave_sync();
        for (int64_t e = c0 + lane; e < c1; e += kWave) {
            const uint32_t id = (uint32_t)idx[e];
            uint32_t h = slot_of(id);
            for (;;) {
                const uint64_t old = atomicCAS((unsigned long long*)&tab[h], (unsigned long long)kFree,
                                               (unsigned long long)id);
                if (old == kFree) break;
                if (old == (uint64_t)id) { dup = true; break; }
                h = (h + 1) & (kSlots - 1);
            }
        }
        wave_sync();
        for (int64_t e = c1 + lane; e < b1 && !dup; e += kWave) {
            const uint32_t id = (uint32_t)idx[e];
            for (uint32_t h = slot_of(id);; h = (h + 1) & (kSlots - 1)) {
                const uint64_t v = tab[h];
                if (v == kFree) break;
                if (v == (uint64_t)id) { dup = true; break; }
            }
        }
        wave_sync();  // the next chunk rewrites the table
    }
    const bool any = wave_any(dup);
    if (lane == 0) out[set] = any ? 1 : 0;
}

hipError_t launch_repeated_ids(int64_t n_sets, const int64_t* rp, const int32_t* idx, uint8_t* out,
                               hipStream_t st)
{
    if (n_sets <= 0) return hipSuccess;
    hipLaunchKernelGGL(repeated_ids_kernel, dim3((unsigned)((n_sets + 3) / 4)), dim3(256), 0, st, n_sets, rp,
                       idx, out);
    return hipGetLastError();
}

}  // namespace dms
