// Measurement support: microbenchmarks that calibrate the roofline
// denominators on the running GPU.
//   - mixer throughput: independent chains of the specification's 64-bit mixer
//     (the unit of work of every hashing stage);
//   - full-rate integer throughput: chains of 32-bit xor/add (v_xor_b32,
//     v_add_u32), the chip's integer VALU issue peak;
//   - stream copy: HBM read+write bandwidth, and the reference for scaling the
//     FETCH_SIZE / WRITE_SIZE counters (plain, and with four loads in flight
//     per thread and streaming stores).
#include "dms_device.h"

namespace dms {

constexpr int kChains = 8;

__global__ void __launch_bounds__(256) calib_mix_kernel(uint64_t* out, int iters)
{
    uint64_t z[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) z[c] = (uint64_t)(blockIdx.x * 256 + threadIdx.x) * 131 + c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) z[c] = mix64(z[c] ^ (uint64_t)i);
    }
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= z[c];
    if (acc == 0x123456789abcdefull) out[0] = acc;  // keeps the chains alive
}

__global__ void __launch_bounds__(256) calib_int_kernel(uint32_t* out, int iters)
{
    uint32_t z[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) z[c] = blockIdx.x * 256 + threadIdx.x + c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            z[c] ^= (uint32_t)i;
            z[c] += 0x9e3779b9u;
            z[c] ^= z[(c + 1) % kChains];
            z[c] += (uint32_t)c;
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= z[c];
    if (acc == 0x12345678u) out[0] = acc;
}

__global__ void __launch_bounds__(256) calib_copy_kernel(const uint4* __restrict__ src,
                                                         uint4* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

// The same copy with four 16-byte loads in flight per thread before its four
// stores (each of the four coalesced across the block), loads and stores both
// marked non-temporal (streamed past the caches); the tail is copied one vector
// at a time.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) calib_copy4_kernel(const u32x4* __restrict__ src,
                                                          u32x4* __restrict__ dst, int64_t n)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x * 4;
    const int64_t full = n / step * step;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x * 4 + threadIdx.x; base < full; base += step) {
        u32x4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = __builtin_nontemporal_load(&src[base + j * blockDim.x]);
#pragma unroll
        for (int j = 0; j < 4; ++j) __builtin_nontemporal_store(v[j], &dst[base + j * blockDim.x]);
    }
    for (int64_t i = full + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t calib_run(int kind, int iters, void* a, void* b, int64_t bytes, int blocks, hipStream_t st)
{
    switch (kind) {
    case 0:
        hipLaunchKernelGGL(calib_mix_kernel, dim3(blocks), dim3(256), 0, st, (uint64_t*)a, iters);
        break;
    case 1:
        hipLaunchKernelGGL(calib_int_kernel, dim3(blocks), dim3(256), 0, st, (uint32_t*)a, iters);
        break;
    case 2:
        hipLaunchKernelGGL(calib_copy_kernel, dim3(blocks), dim3(256), 0, st, (const uint4*)a,
                           (uint4*)b, bytes / 16);
        break;
    default:
        hipLaunchKernelGGL(calib_copy4_kernel, dim3(blocks), dim3(256), 0, st, (const u32x4*)a,
                           (u32x4*)b, bytes / 16);
        break;
    }
    return hipGetLastError();
}

}  // namespace dms
