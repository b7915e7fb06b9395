// Hamming top-k search over 1-bit sketches held in HBM.
//
// scan kernel : block b owns a contiguous slice of database rows and a group of
//               up to kQG queries.  Each thread holds one row's words in
//               registers and compares it with every query of the group (query
//               words are read through the scalar cache, so the xor takes a
//               scalar operand); popcounts accumulate into the distance.  A row
//               whose key (distance << 32 | row) beats the block's running
//               k-th best for that query is appended to a per-query candidate
//               list in LDS; after every tile of rows the lists are folded into
//               each query's sorted top-k.  The block writes its top-k per query.
// merge kernel: one block per query selects the k smallest keys of all blocks:
//               for k <= 16 each thread keeps the 16 smallest of its share of
//               the keys in registers and one wave selects from those in LDS;
//               larger k: one wave selects directly from global memory.
// Keys are unique (row ids differ), so (distance, id) order is total.
#include "dms_device.h"

namespace dms {

namespace {
constexpr int kQG = 16;           // queries per block
constexpr int kTile = 256;        // rows per tile (one per thread)
constexpr int kCand = kTile + 64; // candidate slots per query (a tile plus the top-k)
constexpr int kMaxTopk = 64;
constexpr uint64_t kNoKey = ~0ull;
}  // namespace

// Select the `topk` smallest of n keys held in LDS `keys`, by one wave, into
// out[0..topk) ascending (kNoKey fills).  Keys are distinct or kNoKey.
__device__ __forceinline__ void wave_select(const uint64_t* keys, int n, int topk, uint64_t* out,
                                            int lane)
{
    uint64_t last = 0;
    bool first = true;
    for (int r = 0; r < topk; ++r) {
        uint64_t best = kNoKey;
        for (int i = lane; i < n; i += kWave) {
            const uint64_t v = keys[i];
            if ((first || v > last) && v < best) best = v;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t t = __shfl_xor(best, o, kWave);
            best = t < best ? t : best;
        }
        if (lane == 0) out[r] = best;
        if (best == kNoKey) {
            for (int q = r + 1 + lane; q < topk; q += kWave) out[q] = kNoKey;
            break;
        }
        last = best;
        first = false;
    }
}

// grid: (n_blocks, ceil(n_q / kQG)); 256 threads.  WMAX >= words bounds the
// per-thread row registers (fully unrolled, so the row stays in registers).
template <int WMAX>
__global__ void __launch_bounds__(256)
hamming_scan_kernel(const uint64_t* __restrict__ db, int64_t n_db, int words,
                    const uint64_t* __restrict__ queries, int64_t n_q, int topk,
                    int64_t rows_per_block, uint64_t* __restrict__ partial)
{
    __shared__ uint64_t cand[kQG][kCand];
    __shared__ uint64_t best[kQG][kMaxTopk];
    __shared__ uint64_t merged[kQG][kMaxTopk];
    __shared__ uint32_t ncand[kQG];
    __shared__ uint64_t thr[kQG];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool vec16 = (words % 2) == 0 && ((uintptr_t)db & 15) == 0;
    const int64_t q0 = (int64_t)blockIdx.y * kQG;
    const int nq = (int)((n_q - q0) < kQG ? (n_q - q0) : kQG);
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_block;
    int64_t r_end = r_begin + rows_per_block;
    if (r_end > n_db) r_end = n_db;

    for (int i = tid; i < kQG * kMaxTopk; i += blockDim.x) best[i / kMaxTopk][i % kMaxTopk] = kNoKey;
    if (tid < kQG) {
        ncand[tid] = 0;
        thr[tid] = kNoKey;
    }
    __syncthreads();

    for (int64_t base = r_begin; base < r_end; base += kTile) {
        const int64_t row = base + tid;
        const bool have = row < r_end;
        uint64_t w[WMAX];
        if (vec16) {  // even words on a 16-byte aligned database: 16-byte loads
            const uint4* r4 = reinterpret_cast<const uint4*>(db + (have ? row : 0) * words);
#pragma unroll
            for (int j = 0; j < WMAX; j += 2) {
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (have && j < words) v = r4[j / 2];
                w[j] = ((uint64_t)v.y << 32) | v.x;
                if (j + 1 < WMAX) w[j + 1] = ((uint64_t)v.w << 32) | v.z;
            }
        } else {
#pragma unroll
            for (int j = 0; j < WMAX; ++j) w[j] = (have && j < words) ? db[row * words + j] : 0ull;
        }
        for (int q = 0; q < nq; ++q) {
            const uint64_t* qw = queries + (q0 + q) * words;
            uint32_t d = 0;
#pragma unroll
            for (int j = 0; j < WMAX; ++j)
                if (j < words) d += (uint32_t)__popcll(w[j] ^ qw[j]);
            const uint64_t key = ((uint64_t)d << 32) | (uint64_t)row;
            if (have && key < thr[q]) {
                const uint32_t slot = atomicAdd(&ncand[q], 1u);
                cand[q][slot] = key;  // slot < ncand before the tile + kTile <= kCand - topk
            }
        }
        __syncthreads();
        // fold candidates into each query's top-k (one wave per query) once the
        // list could not take another tile, and after the last tile; until then
        // the threshold stays that of the last fold (looser, still exact)
        const bool last = base + kTile >= r_end;
        for (int q = wave; q < nq; q += blockDim.x / 64) {
            const int n = (int)ncand[q];
            if (n == 0 || (!last && n + kTile + topk <= kCand)) continue;
            for (int i = lane; i < topk; i += kWave) cand[q][n + i] = best[q][i];
            wave_sync();
            wave_select(cand[q], n + topk, topk, merged[q], lane);
            wave_sync();
            for (int i = lane; i < topk; i += kWave) best[q][i] = merged[q][i];
            if (lane == 0) {
                ncand[q] = 0;
                thr[q] = merged[q][topk - 1];
            }
        }
        __syncthreads();
    }
    // write this block's top-k for each query of the group
    for (int i = tid; i < nq * topk; i += blockDim.x) {
        const int q = i / topk, r = i % topk;
        partial[((q0 + q) * gridDim.x + blockIdx.x) * (int64_t)topk + r] = best[q][r];
    }
}

// grid: n_q blocks of 256 threads; topk <= kSmallTopk.
constexpr int kSmallTopk = 16;
__global__ void __launch_bounds__(256)
hamming_merge_small_kernel(const uint64_t* __restrict__ partial, int n_blocks, int topk,
                           int64_t* __restrict__ out_ids, int32_t* __restrict__ out_dist)
{
    __shared__ uint64_t pool[256 * kSmallTopk];
    __shared__ uint64_t res[kSmallTopk];
    const int64_t q = blockIdx.x;
    const int n = n_blocks * topk;
    const uint64_t* keys = partial + q * (int64_t)n;
    uint64_t best[kSmallTopk];  // ascending
#pragma unroll
    for (int j = 0; j < kSmallTopk; ++j) best[j] = kNoKey;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        uint64_t v = keys[i];
#pragma unroll
        for (int j = 0; j < kSmallTopk; ++j) {  // one pass of insertion: best stays sorted
            const uint64_t lo = v < best[j] ? v : best[j];
            v = v < best[j] ? best[j] : v;
            best[j] = lo;
        }
    }
#pragma unroll
    for (int j = 0; j < kSmallTopk; ++j) pool[threadIdx.x * kSmallTopk + j] = best[j];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        wave_select(pool, 256 * kSmallTopk, topk, res, lane);
        wave_sync();
        for (int r = lane; r < topk; r += kWave) {
            const uint64_t v = res[r];
            out_ids[q * topk + r] = v == kNoKey ? -1 : (int64_t)(uint32_t)v;
            out_dist[q * topk + r] = v == kNoKey ? -1 : (int32_t)(v >> 32);
        }
    }
}

// grid: n_q blocks of 64 threads.
__global__ void __launch_bounds__(64)
hamming_merge_kernel(const uint64_t* __restrict__ partial, int n_blocks, int topk,
                     int64_t* __restrict__ out_ids, int32_t* __restrict__ out_dist)
{
    __shared__ uint64_t res[kMaxTopk];
    const int64_t q = blockIdx.x;
    const uint64_t* keys = partial + q * (int64_t)n_blocks * topk;
    const int lane = threadIdx.x;
    uint64_t last = 0;
    bool first = true;
    for (int r = 0; r < topk; ++r) {
        uint64_t b = kNoKey;
        for (int i = lane; i < n_blocks * topk; i += kWave) {
            const uint64_t v = keys[i];
            if ((first || v > last) && v < b) b = v;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t t = __shfl_xor(b, o, kWave);
            b = t < b ? t : b;
        }
        if (lane == 0) res[r] = b;
        last = b;
        first = false;
        if (b == kNoKey) {
            for (int s = r + 1 + lane; s < topk; s += kWave) res[s] = kNoKey;
            break;
        }
    }
    wave_sync();
    for (int r = lane; r < topk; r += kWave) {
        const uint64_t v = res[r];
        out_ids[q * topk + r] = v == kNoKey ? -1 : (int64_t)(uint32_t)v;
        out_dist[q * topk + r] = v == kNoKey ? -1 : (int32_t)(v >> 32);
    }
}

size_t hamming_partial_bytes(int64_t n_q, int n_blocks, int topk)
{
    return (size_t)n_q * n_blocks * topk * sizeof(uint64_t);
}

int hamming_blocks(int64_t n_db, int n_cu)
{
    // enough row slices to fill the chip, each at least a few tiles long
    int64_t b = (n_db + 4 * kTile - 1) / (4 * kTile);
    const int64_t cap = 2 * (int64_t)n_cu;
    if (b > cap) b = cap;
    return b < 1 ? 1 : (int)b;
}

hipError_t launch_hamming(const uint64_t* db, int64_t n_db, int words, const uint64_t* queries,
                          int64_t n_q, int topk, int64_t* out_ids, int32_t* out_dist,
                          uint64_t* partial, int n_blocks, hipStream_t st)
{
    if (n_q <= 0) return hipSuccess;
    const int64_t per = (n_db + n_blocks - 1) / n_blocks;
    const int64_t rows_per_block = ((per + kTile - 1) / kTile) * kTile;
    const int64_t groups = (n_q + kQG - 1) / kQG;
    const int64_t rpb = rows_per_block < kTile ? (int64_t)kTile : rows_per_block;
    const dim3 grid((unsigned)n_blocks, (unsigned)groups);
    if (words <= 4)
        hipLaunchKernelGGL(hamming_scan_kernel<4>, grid, dim3(256), 0, st, db, n_db, words, queries,
                           n_q, topk, rpb, partial);
    else if (words <= 16)
        hipLaunchKernelGGL(hamming_scan_kernel<16>, grid, dim3(256), 0, st, db, n_db, words, queries,
                           n_q, topk, rpb, partial);
    else
        hipLaunchKernelGGL(hamming_scan_kernel<64>, grid, dim3(256), 0, st, db, n_db, words, queries,
                           n_q, topk, rpb, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (topk <= kSmallTopk)
        hipLaunchKernelGGL(hamming_merge_small_kernel, dim3((unsigned)n_q), dim3(256), 0, st, partial,
                           n_blocks, topk, out_ids, out_dist);
    else
        hipLaunchKernelGGL(hamming_merge_kernel, dim3((unsigned)n_q), dim3(64), 0, st, partial, n_blocks,
                           topk, out_ids, out_dist);
    return hipGetLastError();
}

}  // namespace dms
