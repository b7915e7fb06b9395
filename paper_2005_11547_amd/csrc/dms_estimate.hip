// Weighted Jaccard estimates from sketches (Section 1.1): the fraction of equal
// minhashes, 1 - 2 * (disagreeing bits)/k for 1-bit sketches, and for bottom-k
// sketches (Section 3) the share of the union's k first darts found in both.
// Memory bound: one wavefront per pair, lanes over the sketch, coalesced loads.
#include "dms_device.h"

namespace dms {

__global__ void __launch_bounds__(256)
jaccard_u32_kernel(int64_t n_pairs, const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                   int k, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < n_pairs;
         p += waves) {
        const uint32_t* pa = a + p * k;
        const uint32_t* pb = b + p * k;
        uint32_t m = 0;
        for (int j = lane; j < k; j += kWave) m += pa[j] == pb[j] ? 1u : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, kWave);
        if (lane == 0) out[p] = (double)m / (double)k;
    }
}

__global__ void __launch_bounds__(256)
jaccard_1bit_kernel(int64_t n_pairs, const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                    int k, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int words = (k + 63) / 64;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < n_pairs;
         p += waves) {
        const uint64_t* pa = a + p * words;
        const uint64_t* pb = b + p * words;
        uint32_t d = 0;
        for (int j = lane; j < words; j += kWave) {
            uint64_t x = pa[j] ^ pb[j];
            const int valid = k - j * 64;
            if (valid < 64) x &= (1ull << valid) - 1ull;
            d += (uint32_t)__popcll(x);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, kWave);
        if (lane == 0) out[p] = 1.0 - (2.0 * (double)d) / (double)k;
    }
}

hipError_t launch_jaccard(int64_t n_pairs, const void* a, const void* b, int k, int format,
                          double* out, hipStream_t st)
{
    if (n_pairs <= 0) return hipSuccess;
    int64_t blocks = (n_pairs + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    if (format == 0)
        hipLaunchKernelGGL(jaccard_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_pairs,
                           (const uint32_t*)a, (const uint32_t*)b, k, out);
    else
        hipLaunchKernelGGL(jaccard_1bit_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_pairs,
                           (const uint64_t*)a, (const uint64_t*)b, k, out);
    return hipGetLastError();
}

// Bottom-k estimate, one wave per pair.  Dart i of sketch a has
// i + lo - c darts of the union below it, with lo the darts of b below it and c
// the darts below it that both sketches hold (the earlier darts of a that are
// in b, counted by a running ballot); it counts when it is in b and that
// number is below k.  Ranks compare by their bits (they are >= +0).
__global__ void __launch_bounds__(256)
bottomk_jaccard_kernel(int64_t n_pairs, const double* __restrict__ ra, const uint64_t* __restrict__ sa,
                       const double* __restrict__ rb, const uint64_t* __restrict__ sb, int k,
                       double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < n_pairs;
         p += waves) {
        const int64_t base = p * k;
        uint32_t m = 0, shared_before = 0;
        for (int i0 = 0; i0 < k; i0 += kWave) {
            const int i = i0 + lane;
            int lo = 0;
            bool both = false;
            if (i < k) {
                const uint64_t r = (uint64_t)__double_as_longlong(ra[base + i]);
                const uint64_t s = sa[base + i];
                int hi = k;  // first dart of b that is not below (r, s)
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const uint64_t r2 = (uint64_t)__double_as_longlong(rb[base + mid]);
                    const uint64_t s2 = sb[base + mid];
                    if (r2 < r || (r2 == r && s2 < s)) lo = mid + 1;
                    else hi = mid;
                }
                both = lo < k && (uint64_t)__double_as_longlong(rb[base + lo]) == r && sb[base + lo] == s;
            }
            const uint64_t bb = __ballot(both);
            const uint32_t c = shared_before + (uint32_t)__builtin_amdgcn_mbcnt_hi(
                                   (uint32_t)(bb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0u));
            m += (both && (uint32_t)(i + lo) - c < (uint32_t)k) ? 1u : 0u;
            shared_before += (uint32_t)__popcll(bb);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, kWave);
        if (lane == 0) out[p] = (double)m / (double)k;
    }
}

hipError_t launch_bottomk_jaccard(int64_t n_pairs, const double* ra, const uint64_t* sa, const double* rb,
                                  const uint64_t* sb, int k, double* out, hipStream_t st)
{
    if (n_pairs <= 0) return hipSuccess;
    int64_t blocks = (n_pairs + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(bottomk_jaccard_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_pairs, ra, sa, rb,
                       sb, k, out);
    return hipGetLastError();
}

}  // namespace dms
