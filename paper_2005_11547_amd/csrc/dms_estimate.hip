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

// Pairs whose rows are a power-of-two number of 16-byte vectors (four u32
// minhashes or two 64-bit words): G = min(vectors, 64) lanes share a pair, each
// loading whole vectors of a and b, and 64 / G pairs share a wave; the group's
// count is summed by butterflies within the group.  FMT 0: u32 minhashes;
// 1: 1-bit sketches; 2: packed fingerprints of `bits` bits, `bits` dividing 64.
// Bits past k * bits in a row's last word are ignored.
template <int FMT>  // 0: u32 minhashes, 1: 1-bit sketch, 2: b-bit fingerprints
__global__ void __launch_bounds__(256)
pair_vec_kernel(int64_t n_pairs, const uint4* __restrict__ a, const uint4* __restrict__ b, int k, int bits,
                int vecs, int g_log, double* __restrict__ out)
{
    const int G = 1 << g_log;
    const int64_t slots = n_pairs << g_log;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;  // a multiple of 64: groups stay whole
    const int64_t nbits = (int64_t)k * (FMT == 0 ? 32 : bits);
    uint64_t low = 0;  // the lowest bit of every field of a word
    if (FMT == 2)
        for (int i = 0; i < 64; i += bits) low |= 1ull << i;
    for (int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; slot < slots; slot += stride) {
        const int64_t p = slot >> g_log;
        const int r = (int)(slot & (G - 1));
        uint32_t c = 0;
#pragma unroll 4
        for (int v = r; v < vecs; v += G) {
            const uint4 x = load_stream(a + p * vecs + v), y = load_stream(b + p * vecs + v);
            if (FMT == 0) {
                c += (x.x == y.x) + (x.y == y.y) + (x.z == y.z) + (x.w == y.w);
            } else {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    uint64_t d = h == 0 ? (((uint64_t)x.y << 32) | x.x) ^ (((uint64_t)y.y << 32) | y.x)
                                        : (((uint64_t)x.w << 32) | x.z) ^ (((uint64_t)y.w << 32) | y.z);
                    const int64_t valid = nbits - (int64_t)(2 * v + h) * 64;
                    if (valid < 64) d &= valid > 0 ? (1ull << valid) - 1ull : 0ull;
                    if (FMT == 2) {
                        for (int s = 1; s < bits; s <<= 1) d |= d >> s;
                        d &= low;
                    }
                    c += (uint32_t)__popcll(d);
                }
            }
        }
        for (int o = G >> 1; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
        if (r == 0) {
            if (FMT == 0) {
                out[p] = (double)c / (double)k;
            } else if (FMT == 1) {
                out[p] = 1.0 - (2.0 * (double)c) / (double)k;
            } else {
                const double cc = ldexp(1.0, -bits);
                out[p] = ((double)(k - (int)c) / (double)k - cc) / (1.0 - cc);
            }
        }
    }
}

// Lanes per pair (log2) for rows of `vecs` 16-byte vectors, or -1 when the
// rows are not a power of two of whole vectors or a pointer is not 16-aligned.
int pair_vec_glog(int64_t row_bytes, const void* a, const void* b)
{
    if (row_bytes <= 0 || row_bytes % 16 || ((uintptr_t)a | (uintptr_t)b) % 16) return -1;
    const int64_t vecs = row_bytes / 16;
    if (vecs & (vecs - 1)) return -1;
    // long rows (u32 minhashes, k >= 128): four vectors per lane, so that each
    // lane has more loads in flight (measured +18% at k = 256); shorter rows: one
    int g = 0;
    const int64_t per_lane = vecs >= 32 ? 4 : 1;
    while (((int64_t)1 << g) * per_lane < vecs && g < 6) ++g;
    return g;
}

template <int FMT>
void launch_pair_vec(int64_t n_pairs, const void* a, const void* b, int k, int bits, int64_t row_bytes,
                     int g_log, double* out, hipStream_t st)
{
    const int64_t slots = n_pairs << g_log;
    int64_t blocks = (slots + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(pair_vec_kernel<FMT>, dim3((unsigned)blocks), dim3(256), 0, st, n_pairs,
                       (const uint4*)a, (const uint4*)b, k, bits, (int)(row_bytes / 16), g_log, out);
}

hipError_t launch_jaccard(int64_t n_pairs, const void* a, const void* b, int k, int format,
                          double* out, hipStream_t st)
{
    if (n_pairs <= 0) return hipSuccess;
    const int64_t row_bytes = format == 0 ? 4 * (int64_t)k : 8 * (int64_t)((k + 63) / 64);
    const int g_log = pair_vec_glog(row_bytes, a, b);
    if (g_log >= 0) {
        if (format == 0) launch_pair_vec<0>(n_pairs, a, b, k, 32, row_bytes, g_log, out, st);
        else launch_pair_vec<1>(n_pairs, a, b, k, 1, row_bytes, g_log, out, st);
        return hipGetLastError();
    }
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

hipError_t launch_bbit_jaccard_vec(int64_t n_pairs, const uint64_t* a, const uint64_t* b, int k, int bits,
                                   double* out, hipStream_t st, bool* done)
{
    *done = false;
    if (64 % bits) return hipSuccess;
    const int64_t row_bytes = 8 * (((int64_t)k * bits + 63) / 64);
    const int g_log = pair_vec_glog(row_bytes, a, b);
    if (g_log < 0) return hipSuccess;
    launch_pair_vec<2>(n_pairs, a, b, k, bits, row_bytes, g_log, out, st);
    *done = true;
    return hipGetLastError();
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
