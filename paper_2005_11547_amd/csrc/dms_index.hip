// Weight-class LSH index for approximate near neighbour search under weighted
// Jaccard (Section 3): sets are split into weight classes by ||x||_1 in
// [2^c, 2^(c+1)) and scaled by 2^-c (exactly) into [1, 2); each of L tables
// holds the (L,K) LSH key of every indexed set.  A query searches the classes
// within a span of its own, scaled into each of them (Jaccard does not change
// when both sets are scaled alike), gathers the sets that share a key, and
// verifies them with the exact weighted Jaccard.
//
// Layout of a table: n_ok (key, value) pairs sorted by key, then value; value
// = (class + kBias) << 32 | set.  A bucket is the run of one (key, class).
#include "dms_device.h"

#include <hipcub/hipcub.hpp>

namespace dms {

namespace {

constexpr int kBias = 1024;      // class + kBias lies in (0, 2^11) for ||x||_1 within 2^+-800
constexpr int kQueryCap = 2048;  // bucket hits one query may gather

__device__ __forceinline__ double lane_double(double v, int i)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, i);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), i);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Checks row [b0, b1) for the index (ids strictly increasing as uint32, weights
// finite and >= 0, some positive, the largest within [2^-768, 2^768]) and sums
// its positive weights left to right.  Called by all 64 lanes; returns the
// status and, when it is OK, the weight class floor(log2 ||x||_1) in *cls.
__device__ int8_t row_class(const int32_t* __restrict__ idx, const double* __restrict__ w, int64_t b0,
                            int64_t b1, int lane, int* cls)
{
    bool bad = false, pos = false;
    double mx = 0.0, s = 0.0;
    for (int64_t base = b0; base < b1; base += kWave) {
        const int64_t e = base + lane;
        double add = 0.0;
        if (e < b1) {
            const double v = w[e];
            if (e > b0 && (uint32_t)idx[e - 1] >= (uint32_t)idx[e]) bad = true;
            if (!(v >= 0.0) || isinf(v)) bad = true;  // NaN fails v >= 0
            if (v > 0.0) {
                pos = true;
                mx = v > mx ? v : mx;
                add = v;
            }
        }
        const int cnt = (int)(b1 - base < kWave ? b1 - base : kWave);
        for (int i = 0; i < cnt; ++i) s += lane_double(add, i);  // the same order on every lane
    }
    if (wave_any(bad)) return kSetInvalid;
    if (!wave_any(pos)) return kSetEmpty;
    mx = wave_max(mx);
    if (mx > 0x1.0p768 || mx < 0x1.0p-768) return kSetRange;
    *cls = ilogb(s);
    return kSetOk;
}

}  // namespace

// One wave per set: status, class, and the weights scaled by 2^-class (zero
// for a set that is not OK, so that the key pass reports it empty).
__global__ void __launch_bounds__(256)
index_prep_kernel(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ idx,
                  const double* __restrict__ w, double* __restrict__ wn, int32_t* __restrict__ cls,
                  int8_t* __restrict__ status)
{
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (s >= n) return;
    const int64_t b0 = rp[s], b1 = rp[s + 1];
    int c = 0;
    const int8_t st = row_class(idx, w, b0, b1, lane, &c);
    for (int64_t e = b0 + lane; e < b1; e += kWave) wn[e] = st == kSetOk ? ldexp(w[e], -c) : 0.0;
    if (lane == 0) {
        cls[s] = st == kSetOk ? c : 0;
        status[s] = st;
    }
}

// Entries of the OK sets, in (class, set) order: the set list is ordered by
// class first (ord), and entry i of table l takes key keys[ord[i] * L + l].
__global__ void __launch_bounds__(256)
index_entries_kernel(int64_t n_ok, const int64_t* __restrict__ ord, const uint64_t* __restrict__ keys,
                     const int32_t* __restrict__ cls, int L, int l, uint64_t* __restrict__ k_out,
                     uint64_t* __restrict__ v_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ok) return;
    const int64_t s = ord[i];
    k_out[i] = keys[s * L + l];
    v_out[i] = ((uint64_t)(uint32_t)(cls[s] + kBias) << 32) | (uint64_t)(uint32_t)s;
}

// Sort keys of the OK sets by (class, set): (class + kBias) << 32 | set, and
// the count of OK sets.
__global__ void __launch_bounds__(256)
index_order_keys_kernel(int64_t n, const int32_t* __restrict__ cls, const int8_t* __restrict__ status,
                        uint64_t* __restrict__ okey, unsigned long long* __restrict__ n_ok)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const bool ok = status[s] == kSetOk;
    okey[s] = ok ? ((uint64_t)(uint32_t)(cls[s] + kBias) << 32) | (uint64_t)(uint32_t)s : ~0ull;
    if (ok) atomicAdd(n_ok, 1ull);
}

__global__ void index_zero_kernel(unsigned long long* c) { *c = 0ull; }

__global__ void __launch_bounds__(256)
index_order_ids_kernel(int64_t n, const uint64_t* __restrict__ okey, int64_t* __restrict__ ord)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ord[i] = (int64_t)(uint32_t)okey[i];
}

// Query expansion: row q * span2 + j is query q scaled into class
// cls_q - span + j (span2 = 2 span + 1 rows per query).
__global__ void __launch_bounds__(256)
query_prep_kernel(int64_t n_q, const int64_t* __restrict__ rp, const int32_t* __restrict__ idx,
                  const double* __restrict__ w, int span, int64_t* __restrict__ xrp,
                  int32_t* __restrict__ xidx, double* __restrict__ xw, int32_t* __restrict__ qcls,
                  int8_t* __restrict__ qstatus)
{
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (q >= n_q) return;
    const int span2 = 2 * span + 1;
    const int64_t b0 = rp[q], b1 = rp[q + 1], len = b1 - b0;
    int c = 0;
    const int8_t st = row_class(idx, w, b0, b1, lane, &c);
    for (int j = 0; j < span2; ++j) {
        const int64_t o = (int64_t)span2 * b0 + (int64_t)j * len;
        if (lane == 0) xrp[q * span2 + j] = o;
        for (int64_t e = lane; e < len; e += kWave) {
            xidx[o + e] = idx[b0 + e];
            xw[o + e] = st == kSetOk ? ldexp(w[b0 + e], -(c - span + j)) : 0.0;
        }
    }
    if (q == n_q - 1 && lane == 0) xrp[n_q * span2] = (int64_t)span2 * b1;
    if (lane == 0) {
        qcls[q] = st == kSetOk ? c : 0;
        qstatus[q] = st;
    }
}

namespace {

// First position in table [0, n) whose (key, value) is not below (k, v).
__device__ __forceinline__ int64_t lower_pair(const uint64_t* __restrict__ tk, const uint64_t* __restrict__ tv,
                                              int64_t n, uint64_t k, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const uint64_t a = tk[mid];
        if (a < k || (a == k && tv[mid] < v)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Exact weighted Jaccard of two id-sorted rows, both sums in ascending id order.
__device__ double jaccard_merge(const int32_t* ia, const double* wa, int64_t na, const int32_t* ib,
                                const double* wb, int64_t nb)
{
    int64_t i = 0, j = 0;
    double smin = 0.0, smax = 0.0;
    while (i < na || j < nb) {
        const uint32_t a = i < na ? (uint32_t)ia[i] : 0u, b = j < nb ? (uint32_t)ib[j] : 0u;
        if (j >= nb || (i < na && a < b)) {
            smax += wa[i++];
        } else if (i >= na || b < a) {
            smax += wb[j++];
        } else {
            const double x = wa[i++], y = wb[j++];
            smin += x < y ? x : y;
            smax += x < y ? y : x;
        }
    }
    return smax > 0.0 ? smin / smax : 0.0;
}

}  // namespace

// One wave per query: gather the buckets of its (class, table) pairs, drop
// repeated sets, verify each with the exact Jaccard, keep J >= j1 and write
// the topn best by (J descending, set ascending).
__global__ void __launch_bounds__(64)
query_kernel(int64_t n_q, int span, int L, const uint64_t* __restrict__ qkeys,
             const int8_t* __restrict__ xstatus, const int32_t* __restrict__ qcls,
             const int8_t* __restrict__ qstatus,
             const uint64_t* __restrict__ tkeys, const uint64_t* __restrict__ tvals, int64_t n_ok,
             const int64_t* __restrict__ q_rp, const int32_t* __restrict__ q_idx,
             const double* __restrict__ q_w, const int64_t* __restrict__ d_rp,
             const int32_t* __restrict__ d_idx, const double* __restrict__ d_w, double j1, int topn,
             int64_t* __restrict__ out_ids, double* __restrict__ out_j, int32_t* __restrict__ out_count,
             int32_t* __restrict__ out_cand, int8_t* __restrict__ out_status)
{
    __shared__ uint32_t cid[kQueryCap];  // candidate sets
    __shared__ uint64_t cj[kQueryCap];   // their Jaccard bits (kept ones), ~0 otherwise
    const int lane = threadIdx.x;
    const int span2 = 2 * span + 1;
    for (int64_t q = blockIdx.x; q < n_q; q += gridDim.x) {
        int8_t st = qstatus[q];
        uint32_t total = 0;
        if (st == kSetOk) {
            // gather: lanes over (class j, table l) pairs
            const int P = span2 * L;
            for (int p0 = 0; p0 < P; p0 += kWave) {
                const int p = p0 + lane;
                int64_t lo = 0, hi = 0;
                // a class copy whose keys are not OK (scaled out of range) is skipped
                if (p < P && xstatus[q * span2 + p / L] == kSetOk) {
                    const int j = p / L, l = p - j * L;
                    const uint64_t key = qkeys[(q * span2 + j) * L + l];
                    const uint64_t c = (uint64_t)(uint32_t)(qcls[q] - span + j + kBias);
                    const uint64_t* tk = tkeys + (int64_t)l * n_ok;
                    const uint64_t* tv = tvals + (int64_t)l * n_ok;
                    lo = lower_pair(tk, tv, n_ok, key, c << 32);
                    hi = lower_pair(tk, tv, n_ok, key, (c + 1) << 32);
                }
                const uint32_t cnt = (uint32_t)(hi - lo);
                uint32_t incl = cnt;
                for (int o = 1; o < kWave; o <<= 1) {
                    const uint32_t y = (uint32_t)__shfl_up((int)incl, o, kWave);
                    if (lane >= o) incl += y;
                }
                const uint32_t round_total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
                if (total + round_total <= (uint32_t)kQueryCap) {
                    const uint32_t off = total + incl - cnt;
                    const uint64_t* tv = p < P ? tvals + (int64_t)(p % L) * n_ok : tvals;
                    for (uint32_t i = 0; i < cnt; ++i) cid[off + i] = (uint32_t)tv[lo + i];
                }
                total += round_total;
            }
            if (total > (uint32_t)kQueryCap) st = kQueryOverflow;
        }
        wave_sync();
        uint32_t U = 0, kept = 0;
        if (st == kSetOk && total > 0) {
            // sort the hits (bitonic over a power of two, padded) and drop repeats
            uint32_t N = 1;
            while (N < total) N <<= 1;
            for (uint32_t i = total + lane; i < N; i += kWave) cid[i] = 0xFFFFFFFFu;
            wave_sync();
            for (uint32_t size = 2; size <= N; size <<= 1) {
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t i = lane; i < N / 2; i += kWave) {
                        const uint32_t a = 2 * i - (i & (stride - 1)), b = a + stride;
                        const uint32_t x = cid[a], y = cid[b];
                        if ((x > y) == ((a & size) == 0)) {
                            cid[a] = y;
                            cid[b] = x;
                        }
                    }
                    wave_sync();
                }
            }
            uint32_t prev = 0;
            for (uint32_t base = 0; base < total; base += kWave) {
                const uint32_t i = base + lane;
                uint32_t v = 0xFFFFFFFFu;
                bool keep = false;
                if (i < total) {
                    v = cid[i];
                    keep = i == 0 || v != (lane == 0 ? prev : cid[i - 1]);
                }
                const int last = (int)((total - base < (uint32_t)kWave ? total - base : (uint32_t)kWave) - 1);
                prev = (uint32_t)__shfl((int)v, last, kWave);
                const uint64_t bm = __ballot(keep);
                wave_sync();
                if (keep)
                    cid[U + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u))] = v;
                U += (uint32_t)__popcll(bm);
                wave_sync();
            }
            // verify: exact Jaccard, kept when >= j1; order key ~J bits (descending J)
            const int64_t qb = q_rp[q], qn = q_rp[q + 1] - qb;
            for (uint32_t i = lane; i < U; i += kWave) {
                const int64_t x = cid[i];
                const double J = jaccard_merge(q_idx + qb, q_w + qb, qn, d_idx + d_rp[x], d_w + d_rp[x],
                                               d_rp[x + 1] - d_rp[x]);
                cj[i] = J >= j1 ? ~(uint64_t)__double_as_longlong(J) : ~0ull;
                kept += J >= j1 ? 1u : 0u;
            }
            for (int o = 32; o > 0; o >>= 1) kept += (uint32_t)__shfl_xor((int)kept, o, kWave);
            wave_sync();
            // order by (~J bits, set): the kept ones first, best J first, ties by set
            uint32_t N2 = 1;
            while (N2 < U) N2 <<= 1;
            for (uint32_t i = U + lane; i < N2; i += kWave) {
                cj[i] = ~0ull;
                cid[i] = 0xFFFFFFFFu;
            }
            wave_sync();
            for (uint32_t size = 2; size <= N2; size <<= 1) {
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t i = lane; i < N2 / 2; i += kWave) {
                        const uint32_t a = 2 * i - (i & (stride - 1)), b = a + stride;
                        const uint64_t ja = cj[a], jb = cj[b];
                        const uint32_t ia = cid[a], ib = cid[b];
                        const bool gt = ja > jb || (ja == jb && ia > ib);
                        if (gt == ((a & size) == 0)) {
                            cj[a] = jb;
                            cj[b] = ja;
                            cid[a] = ib;
                            cid[b] = ia;
                        }
                    }
                    wave_sync();
                }
            }
        }
        const uint32_t nout = kept < (uint32_t)topn ? kept : (uint32_t)topn;
        for (int i = lane; i < topn; i += kWave) {
            const bool has = (uint32_t)i < nout;
            out_ids[q * topn + i] = has ? (int64_t)cid[i] : -1;
            out_j[q * topn + i] = has ? __longlong_as_double((long long)~cj[i]) : 0.0;
        }
        if (lane == 0) {
            out_count[q] = (int32_t)nout;
            out_cand[q] = (int32_t)U;
            out_status[q] = st;
        }
        wave_sync();  // the next query reuses the LDS arrays
    }
}

// ---------------------------------------------------------------------------
// Host side

hipError_t launch_index_prep(int64_t n, const int64_t* rp, const int32_t* idx, const double* w, double* wn,
                             int32_t* cls, int8_t* status, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(index_prep_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, n, rp, idx, w, wn,
                       cls, status);
    return hipGetLastError();
}

// Bytes of hipCUB scratch for sorting n (u64, u64) pairs.
size_t index_sort_scratch(int64_t n)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                             (const uint64_t*)nullptr, (uint64_t*)nullptr, (int)n);
    size_t b2 = 0;
    (void)hipcub::DeviceRadixSort::SortKeys(nullptr, b2, (const uint64_t*)nullptr, (uint64_t*)nullptr, (int)n);
    return bytes > b2 ? bytes : b2;
}

// Order of the OK sets by (class, set) into ord[0, n_ok); the count goes to
// *n_ok_dev (the caller reads it back).  okey and okey2 hold n words each.
hipError_t launch_index_order(int64_t n, const int32_t* cls, const int8_t* status, uint64_t* okey,
                              uint64_t* okey2, int64_t* ord, unsigned long long* n_ok_dev, void* scratch,
                              size_t scratch_bytes, hipStream_t st)
{
    hipLaunchKernelGGL(index_zero_kernel, dim3(1), dim3(1), 0, st, n_ok_dev);
    hipLaunchKernelGGL(index_order_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, cls,
                       status, okey, n_ok_dev);
    size_t b = scratch_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortKeys(scratch, b, okey, okey2, (int)n, 0, 64, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(index_order_ids_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, okey2,
                       ord);
    return hipGetLastError();
}

// Table l: entries of the OK sets in (class, set) order, then a stable sort
// by key gives (key, class, set) order.
hipError_t launch_index_table(int64_t n_ok, const int64_t* ord, const uint64_t* keys, const int32_t* cls, int L,
                              int l, uint64_t* tmp_k, uint64_t* tmp_v, uint64_t* out_k, uint64_t* out_v,
                              void* scratch, size_t scratch_bytes, hipStream_t st)
{
    if (n_ok <= 0) return hipSuccess;
    hipLaunchKernelGGL(index_entries_kernel, dim3((unsigned)((n_ok + 255) / 256)), dim3(256), 0, st, n_ok, ord,
                       keys, cls, L, l, tmp_k, tmp_v);
    size_t b = scratch_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(scratch, b, tmp_k, out_k, tmp_v, out_v, (int)n_ok, 0, 64, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_query_prep(int64_t n_q, const int64_t* rp, const int32_t* idx, const double* w, int span,
                             int64_t* xrp, int32_t* xidx, double* xw, int32_t* qcls, int8_t* qstatus,
                             hipStream_t st)
{
    if (n_q <= 0) return hipSuccess;
    hipLaunchKernelGGL(query_prep_kernel, dim3((unsigned)((n_q + 3) / 4)), dim3(256), 0, st, n_q, rp, idx, w,
                       span, xrp, xidx, xw, qcls, qstatus);
    return hipGetLastError();
}

hipError_t launch_index_query(int64_t n_q, int span, int L, const uint64_t* qkeys, const int8_t* xstatus,
                              const int32_t* qcls,
                              const int8_t* qstatus, const uint64_t* tkeys, const uint64_t* tvals, int64_t n_ok,
                              const int64_t* q_rp, const int32_t* q_idx, const double* q_w, const int64_t* d_rp,
                              const int32_t* d_idx, const double* d_w, double j1, int topn, int64_t* out_ids,
                              double* out_j, int32_t* out_count, int32_t* out_cand, int8_t* out_status,
                              int n_cu, hipStream_t st)
{
    if (n_q <= 0) return hipSuccess;
    int64_t blocks = n_q < (int64_t)n_cu * 16 ? n_q : (int64_t)n_cu * 16;
    hipLaunchKernelGGL(query_kernel, dim3((unsigned)blocks), dim3(64), 0, st, n_q, span, L, qkeys, xstatus, qcls,
                       qstatus,
                       tkeys, tvals, n_ok, q_rp, q_idx, q_w, d_rp, d_idx, d_w, j1, topn, out_ids, out_j,
                       out_count, out_cand, out_status);
    return hipGetLastError();
}

}  // namespace dms
