// b-bit fingerprints of minhash sketches and the unary feature map (Section
// 1.1): each minhash is cut to its lowest b bits (bits of the dart-id hash,
// independent of the bucket bits; b = 1 is the 1-bit sketch), the k
// fingerprints of a set are packed into a little-endian bit stream, pairs of
// packed sketches give the corrected agreement estimate of J, and the unary map
// turns the fingerprints into the k nonzero coordinates of a k * 2^b
// dimensional vector whose inner products estimate J.  All three are memory
// bound and read each input once.
#include "dms_device.h"

namespace dms {

hipError_t launch_bbit_jaccard_vec(int64_t n_pairs, const uint64_t* a, const uint64_t* b, int k, int bits,
                                   double* out, hipStream_t st, bool* done);

namespace {
constexpr int kPackWaves = 4;  // waves per block of the pack kernel

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
}

// Rows that are whole words (k * b divisible by 64, k divisible by 4) with b a
// power of two: the input is one stream of 16-byte vectors (four minhashes,
// 4b fingerprint bits) and the output one stream of words, G = 16 / b vectors
// per word.  Each lane packs its vector, the G lanes of a word OR their parts
// together by butterflies, and the first writes the word (b = 32: each vector
// is two words).
__global__ void __launch_bounds__(256)
bbit_pack_vec_kernel(int64_t n_vecs, const uint4* __restrict__ v, int b, int g_log,
                     uint64_t* __restrict__ out)
{
    const uint32_t mask = b == 32 ? 0xffffffffu : (1u << b) - 1u;
    const int G = 1 << g_log;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;  // a multiple of 64: groups stay whole
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_vecs; q += stride) {
        const uint4 x = load_stream(v + q);
        if (b == 32) {
            reinterpret_cast<uint4*>(out)[q] = x;  // two words: minhash 2i low, 2i + 1 high
            continue;
        }
        uint64_t part = (uint64_t)(x.x & mask) | ((uint64_t)(x.y & mask) << b) |
                        ((uint64_t)(x.z & mask) << (2 * b)) | ((uint64_t)(x.w & mask) << (3 * b));
        const int r = (int)(q & (G - 1));
        part <<= 4 * b * r;
        for (int o = G >> 1; o > 0; o >>= 1) part |= (uint64_t)__shfl_xor((long long)part, o, kWave);
        if (r == 0) out[q >> g_log] = part;
    }
}

// Unary map over 16-byte vectors (k divisible by 4): the column j of the
// vector's first minhash advances by a fixed step per grid-stride iteration.
__global__ void __launch_bounds__(256)
unary_map_vec_kernel(int64_t n_vecs, const uint4* __restrict__ v, int k, int b, uint4* __restrict__ out)
{
    const uint32_t mask = (uint32_t)((1ull << b) - 1ull);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t j = (uint32_t)((4 * q) % k);
    const uint32_t step = (uint32_t)((4 * stride) % k);
    for (; q < n_vecs; q += stride) {
        const uint4 x = load_stream(v + q);
        uint4 y;
        y.x = (j << b) + (x.x & mask);
        y.y = ((j + 1) << b) + (x.y & mask);
        y.z = ((j + 2) << b) + (x.z & mask);
        y.w = ((j + 3) << b) + (x.w & mask);
        out[q] = y;
        j += step;
        if (j >= (uint32_t)k) j -= (uint32_t)k;
    }
}

// One wave per (row, chunk of 64 fingerprints).  The chunk's 64 * b bits are
// exactly words [chunk * b, chunk * b + b) of the row, assembled in LDS with
// atomic ORs (a fingerprint may straddle two words) and written by b lanes.
__global__ void __launch_bounds__(64 * kPackWaves)
bbit_pack_kernel(int64_t n_sets, const uint32_t* __restrict__ v, int k, int b, int words,
                 int chunks, uint64_t* __restrict__ out)
{
    __shared__ unsigned long long stage[kPackWaves][32];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint64_t mask = (1ull << b) - 1ull;
    const int64_t total = n_sets * (int64_t)chunks;
    const int64_t step = (int64_t)gridDim.x * kPackWaves;
    for (int64_t task = (int64_t)blockIdx.x * kPackWaves + wave; task < total; task += step) {
        const int64_t row = task / chunks;
        const int c = (int)(task - row * chunks);
        const int f = c * 64 + lane;
        const uint64_t x = f < k ? (uint64_t)v[row * k + f] & mask : 0ull;
        if (lane < 32) stage[wave][lane] = 0ull;
        wave_sync();
        // chunk-local bit offset: lane * b < 64 * b, so the words are 0 .. b - 1
        const int p = lane * b;
        const int q = p >> 6, sh = p & 63;
        if (x) {
            atomicOr(&stage[wave][q], x << sh);
            if (sh + b > 64) atomicOr(&stage[wave][q + 1], x >> (64 - sh));
        }
        wave_sync();
        const int word = c * b + lane;
        if (lane < b && word < words) out[row * words + word] = stage[wave][lane];
        wave_sync();  // the stage is cleared for the next task only after these reads
    }
}

// One wave per pair.  When b divides 64 the fields never straddle words:
// XOR the words, fold each field onto its lowest bit and count the fields that
// differ.  Otherwise each lane extracts whole fingerprints.
__global__ void __launch_bounds__(256)
bbit_jaccard_kernel(int64_t n_pairs, const uint64_t* __restrict__ a, const uint64_t* __restrict__ bb,
                    int k, int b, int words, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t mask = (1ull << b) - 1ull;
    const bool aligned = (64 % b) == 0;
    uint64_t low = 0;  // the lowest bit of every field of a word
    for (int i = 0; i < 64; i += b) low |= 1ull << i;
    const int64_t bits = (int64_t)k * b;
    for (int64_t pr = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); pr < n_pairs;
         pr += waves) {
        const uint64_t* pa = a + pr * words;
        const uint64_t* pb = bb + pr * words;
        uint32_t diff = 0;
        if (aligned) {
            for (int q = lane; q < words; q += kWave) {
                uint64_t x = pa[q] ^ pb[q];
                const int64_t valid = bits - (int64_t)q * 64;
                if (valid < 64) x &= (1ull << valid) - 1ull;
                for (int s = 1; s < b; s <<= 1) x |= x >> s;
                diff += (uint32_t)__popcll(x & low);
            }
        } else {
            for (int j = lane; j < k; j += kWave) {
                const int64_t p = (int64_t)j * b;
                const int64_t q = p >> 6;
                const int sh = (int)(p & 63);
                uint64_t fa = pa[q] >> sh, fb = pb[q] >> sh;
                if (sh + b > 64) {
                    fa |= pa[q + 1] << (64 - sh);
                    fb |= pb[q + 1] << (64 - sh);
                }
                diff += ((fa ^ fb) & mask) ? 1u : 0u;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) diff += __shfl_xor(diff, o, kWave);
        if (lane == 0) {
            const double c = ldexp(1.0, -b);
            out[pr] = ((double)(k - (int)diff) / (double)k - c) / (1.0 - c);
        }
    }
}

// Coordinate of minhash j of a row: j * 2^b + (its b-bit fingerprint).
__global__ void __launch_bounds__(256)
unary_map_kernel(int64_t n_sets, const uint32_t* __restrict__ v, int k, int b,
                 int32_t* __restrict__ out)
{
    const uint32_t mask = (uint32_t)((1ull << b) - 1ull);
    for (int64_t row = blockIdx.x; row < n_sets; row += gridDim.x) {
        const uint32_t* src = v + row * k;
        int32_t* dst = out + row * k;
        for (int j = threadIdx.x; j < k; j += blockDim.x)
            dst[j] = (int32_t)(((uint32_t)j << b) + (src[j] & mask));
    }
}

hipError_t launch_bbit_pack(int64_t n_sets, const uint32_t* v, int k, int b, uint64_t* out,
                            hipStream_t st)
{
    if (n_sets <= 0) return hipSuccess;
    if ((b & (b - 1)) == 0 && k % 4 == 0 && ((int64_t)k * b) % 64 == 0 && aligned16(v) && aligned16(out)) {
        const int64_t n_vecs = n_sets * (int64_t)(k / 4);
        const int g_log = b == 32 ? 0 : (b == 16 ? 0 : b == 8 ? 1 : b == 4 ? 2 : b == 2 ? 3 : 4);
        int64_t blocks = (n_vecs + 255) / 256;
        if (blocks > 16384) blocks = 16384;
        hipLaunchKernelGGL(bbit_pack_vec_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_vecs,
                           (const uint4*)v, b, g_log, out);
        return hipGetLastError();
    }
    const int words = (int)(((int64_t)k * b + 63) / 64);
    const int chunks = (k + 63) / 64;
    int64_t blocks = (n_sets * chunks + kPackWaves - 1) / kPackWaves;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(bbit_pack_kernel, dim3((unsigned)blocks), dim3(64 * kPackWaves), 0, st, n_sets,
                       v, k, b, words, chunks, out);
    return hipGetLastError();
}

hipError_t launch_bbit_jaccard(int64_t n_pairs, const uint64_t* a, const uint64_t* b_, int k, int b,
                               double* out, hipStream_t st)
{
    if (n_pairs <= 0) return hipSuccess;
    bool done = false;
    hipError_t e = launch_bbit_jaccard_vec(n_pairs, a, b_, k, b, out, st, &done);
    if (done || e != hipSuccess) return e;
    const int words = (int)(((int64_t)k * b + 63) / 64);
    int64_t blocks = (n_pairs + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(bbit_jaccard_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_pairs, a, b_, k,
                       b, words, out);
    return hipGetLastError();
}

hipError_t launch_unary_map(int64_t n_sets, const uint32_t* v, int k, int b, int32_t* out,
                            hipStream_t st)
{
    if (n_sets <= 0) return hipSuccess;
    if (k % 4 == 0 && aligned16(v) && aligned16(out)) {
        const int64_t n_vecs = n_sets * (int64_t)(k / 4);
        int64_t blocks = (n_vecs + 255) / 256;
        if (blocks > 16384) blocks = 16384;
        hipLaunchKernelGGL(unary_map_vec_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_vecs,
                           (const uint4*)v, k, b, (uint4*)out);
        return hipGetLastError();
    }
    int64_t blocks = n_sets < 65536 ? n_sets : 65536;
    hipLaunchKernelGGL(unary_map_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n_sets, v, k, b, out);
    return hipGetLastError();
}

}  // namespace dms
