// "Plain" DartMinHash and (L,K) LSH kernels: one wavefront per set, one lane
// per nonzero, each lane walking the regions of its elements one after another
// and the areas of each region column by column.  One launch covers the whole
// batch.  These kernels are the simple comparator for the flattened kernels in
// dms_sketch.hip.
#include "dms_device.h"
#include "dms_launch.h"

namespace dms {

// Enumeration counts of one lane: regions, areas, darts generated, darts of
// rank <= tau, darts accepted (every pass re-inserts every dart it meets).
struct LaneCounts {
    uint64_t reg = 0, area = 0, gen = 0, rank = 0, acc = 0;
};

// The darts of the hashed Poisson process hitting the elements owned by one
// lane below rank tau (Section 2, "Poisson darts"): the weight-rank plane
// above element i is cut into the dyadic regions (nu, rho) of Algorithm 1,
// each into a grid of 2^rho columns by 2^nu rows of area 1/t.  A region is
// visited when its lower corner lies under (x_i, tau); within it, the columns
// whose left edge is at most x_i and the rows whose lower edge is at most tau
// form prefixes (the edges grow with the index), whose lengths are counted
// first; every area of that grid is hashed and its darts tested against both
// bounds.  Every accepted dart goes to `sink(rank, s)`.  Sets *range when an
// index leaves the supported domain.
template <int HK, bool CNT, class Sink>
__device__ __forceinline__ void lane_darthash(const SpecTables* __restrict__ sp,
                                              const int32_t* __restrict__ idx,
                                              const double* __restrict__ w, int64_t b0,
                                              int64_t b1, int lane, double tau, bool* range,
                                              LaneCounts& cnt, Sink&& sink)
{
    const Hasher<HK> H(sp);
    for (int64_t e = b0 + lane; e < b1; e += kWave) {
        const double xi = w[e];
        if (!(xi > 0.0)) continue;
        const uint64_t id = (uint32_t)idx[e];
        for (int nu = 0; w_corner(sp->W, sp->u, nu) <= xi && !*range; ++nu) {
            if (nu + 1 >= kMaxIndex) { *range = true; break; }
            const double Wn = w_corner(sp->W, sp->u, nu);
            for (int rho = 0; r_corner(sp->R, rho) <= tau; ++rho) {
                if (rho + 1 >= kMaxIndex) { *range = true; break; }
                const double Rr = r_corner(sp->R, rho);
                const double dnu = ldexp(sp->u, nu - rho);   // column width 2^nu / (t 2^rho)
                const double drho = ldexp(1.0, rho - nu);    // row height 2^rho / 2^nu
                // columns w with Wn + w dnu <= x_i, rows r with Rr + r drho <= tau
                // real-number estimates of the counts (1/dnu ~ t 2^(rho-nu), 1/drho = 2^(nu-rho)),
                // made exact by prefix_count
                const double td = (double)sp->t;
                const double n_col = prefix_count(Wn, dnu, xi, ldexp(1.0, rho),
                                                  floor((xi - Wn) * td * ldexp(1.0, rho - nu)) + 1.0);
                const double n_row = prefix_count(Rr, drho, tau, ldexp(1.0, nu),
                                                  floor((tau - Rr) * ldexp(1.0, nu - rho)) + 1.0);
                if (n_col > 4294967296.0 || n_row > 4294967296.0) { *range = true; break; }
                const uint64_t g =
                    H(sp->key_r ^ ((id << 32) | ((uint64_t)nu << 16) | (uint64_t)rho));
                if (CNT) cnt.reg += 1;
                const uint64_t nc = (uint64_t)n_col, nr = (uint64_t)n_row;
                for (uint64_t wc = 0; wc < nc; ++wc) {
                    const double wd = (double)wc;
                    for (uint64_t rc = 0; rc < nr; ++rc) {
                        const double rd = (double)rc;
                        const uint64_t a = H(g ^ sp->key_a ^ ((wc << 32) | rc));
                        const uint32_t X = poisson_count(sp->pois, a);
                        if (CNT) {
                            cnt.area += 1;
                            cnt.gen += X;
                        }
                        for (uint32_t j = 0; j < X; ++j) {
                            const double U = unit53(H(a ^ sp->key_u ^ (uint64_t)j));
                            const double rank = Rr + (rd + U) * drho;
                            if (!(rank <= tau)) continue;
                            if (CNT) cnt.rank += 1;
                            const double V = unit53(H(a ^ sp->key_v ^ (uint64_t)j));
                            const double weight = Wn + (wd + V) * dnu;
                            if (!(weight <= xi)) continue;
                            if (CNT) cnt.acc += 1;
                            sink(rank, H(a ^ sp->key_s ^ (uint64_t)j));
                        }
                    }
                }
            }
        }
    }
}

// Wave totals of the lanes' counts, written by lane 0 (layout of kCounterWords).
__device__ __forceinline__ void write_counts(int64_t* out_cnt, int64_t set, int lane, const LaneCounts& c,
                                             uint64_t passes, double phi_end)
{
    const uint64_t v[5] = {c.reg, c.area, c.gen, c.rank, c.acc};
    uint64_t tot[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        uint64_t x = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
        tot[q] = x;
    }
    if (lane == 0) {
        int64_t* oc = out_cnt + set * kCounterWords;
        for (int q = 0; q < 5; ++q) oc[q] = (int64_t)tot[q];
        oc[5] = (int64_t)passes;
        oc[6] = __double_as_longlong(phi_end);
        oc[7] = 0;
    }
}

__device__ __forceinline__ void write_minhash(int64_t set, int k, int lane, int8_t status,
                                              const uint64_t* rank_bits, const uint64_t* sval,
                                              uint32_t* out_u32, uint64_t* out_bits,
                                              int8_t* out_status, uint64_t* out_s,
                                              double* out_rank)
{
    const bool ok = status == kSetOk;
    for (int j = lane; j < k; j += kWave) {
        const uint64_t s = ok ? sval[j] : ~0ull;
        const uint64_t rb = ok ? rank_bits[j] : kRankEmpty;
        if (out_u32) out_u32[set * k + j] = ok ? (uint32_t)s : 0xFFFFFFFFu;
        if (out_s) out_s[set * k + j] = s;
        if (out_rank) out_rank[set * k + j] = __longlong_as_double((long long)rb);
    }
    if (out_bits) {
        const int words = (k + 63) / 64;
        for (int wd = 0; wd < words; ++wd) {
            const int j = wd * 64 + lane;
            const bool bit = ok && j < k && (sval[j] & 1ull);
            const uint64_t word = __ballot(bit);
            if (lane == 0) out_bits[(int64_t)set * words + wd] = word;
        }
    }
    if (out_status && lane == 0) out_status[set] = status;
}

// grid: ceil(n_sets / waves) blocks of 64*waves threads; LDS: waves * 16 k bytes.
template <int HK, bool CNT>
__global__ void __launch_bounds__(256)
sketch_plain_kernel(const SpecTables* __restrict__ sp, int64_t n_sets,
                    const int64_t* __restrict__ rp, const int32_t* __restrict__ idx,
                    const double* __restrict__ w, int k, uint32_t* out_u32, uint64_t* out_bits,
                    int8_t* out_status, uint64_t* out_s, double* out_rank, double phi0,
                    double phi_max, int64_t* out_cnt, const uint8_t* __restrict__ repeated)
{
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int64_t set = (int64_t)blockIdx.x * waves + wave;
    if (set >= n_sets) return;  // whole wave leaves; no block barrier follows
    uint64_t* rank_bits = lds + (size_t)wave * 2 * k;
    uint64_t* sval = rank_bits + k;

    const int64_t b0 = rp[set], b1 = rp[set + 1];
    const RowInfo ri = scan_row(w, b0, b1, lane);
    int8_t status = ri.status;
    if (status == kSetOk && repeated && repeated[set]) status = kSetInvalid;
    LaneCounts cnt;
    uint64_t passes = 0;
    double phi_end = 0.0;
    if (status == kSetOk) {
        for (int j = lane; j < k; j += kWave) {
            rank_bits[j] = kRankEmpty;
            sval[j] = ~0ull;
        }
        double phi = phi0;
        for (;;) {
            if (phi > phi_max) { status = kSetRange; break; }
            const double tau = phi / ri.sum;
            bool range = false;
            passes += 1;
            phi_end = phi;
            lane_darthash<HK, CNT>(sp, idx, w, b0, b1, lane, tau, &range, cnt, [&](double rank, uint64_t s) {
                bucket_min(rank_bits, sval, bucket_of(s, (uint32_t)k),
                           (uint64_t)__double_as_longlong(rank), s);
            });
            if (wave_any(range)) { status = kSetRange; break; }
            wave_sync();
            bool filled = true;
            for (int j = lane; j < k; j += kWave) filled &= rank_bits[j] != kRankEmpty;
            if (wave_all(filled)) break;
            phi *= 2.0;
        }
    }
    wave_sync();
    write_minhash(set, k, lane, status, rank_bits, sval, out_u32, out_bits, out_status, out_s,
                  out_rank);
    if (CNT && out_cnt) write_counts(out_cnt, set, lane, cnt, passes, phi_end);
}

// ---------------------------------------------------------------------------
// (L,K) LSH.  Each table keeps its K smallest (rank, s) in ascending order in
// LDS; lanes holding a dart at the same time insert one after another.
struct LshLds {
    uint64_t* rank;   // [L*K]
    uint64_t* sval;   // [L*K]
    int32_t* cnt;     // [L]
};

__device__ __forceinline__ void lsh_insert(const LshLds& T, int K, uint32_t l, uint64_t rb,
                                           uint64_t s)
{
    uint64_t* r = T.rank + (size_t)l * K;
    uint64_t* v = T.sval + (size_t)l * K;
    const int c = T.cnt[l];
    int pos = 0;
    for (int m = 0; m < c; ++m) {
        if (r[m] == rb && v[m] == s) return;  // already held (repeated element id)
        pos += (r[m] < rb || (r[m] == rb && v[m] < s)) ? 1 : 0;
    }
    if (pos >= K) return;
    const int last = c < K ? c : K - 1;
    for (int m = last; m > pos; --m) {
        r[m] = r[m - 1];
        v[m] = v[m - 1];
    }
    r[pos] = rb;
    v[pos] = s;
    if (c < K) T.cnt[l] = c + 1;
}

// LDS per wave: L*K*16 + L*8 bytes.
template <int HK, bool CNT>
__global__ void __launch_bounds__(256)
lsh_plain_kernel(const SpecTables* __restrict__ sp, int64_t n_sets,
                 const int64_t* __restrict__ rp, const int32_t* __restrict__ idx,
                 const double* __restrict__ w, int L, int K, uint64_t* out_keys,
                 int8_t* out_status, double phi0, double phi_max, int64_t* out_cnt,
                 const uint8_t* __restrict__ repeated)
{
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int64_t set = (int64_t)blockIdx.x * waves + wave;
    if (set >= n_sets) return;
    const size_t per_wave = (size_t)2 * L * K + L;  // in 8-byte words
    uint64_t* base = lds + (size_t)wave * per_wave;
    LshLds T;
    T.rank = base;
    T.sval = base + (size_t)L * K;
    T.cnt = (int32_t*)(base + (size_t)2 * L * K);

    const int64_t b0 = rp[set], b1 = rp[set + 1];
    const RowInfo ri = scan_row(w, b0, b1, lane);
    int8_t status = ri.status;
    if (status == kSetOk && repeated && repeated[set]) status = kSetInvalid;
    LaneCounts cnt;
    uint64_t passes = 0;
    double phi_end = 0.0;
    if (status == kSetOk) {
        for (int l = lane; l < L; l += kWave) T.cnt[l] = 0;
        double phi = phi0;
        for (;;) {
            if (phi > phi_max) { status = kSetRange; break; }
            const double tau = phi / ri.sum;
            bool range = false;
            passes += 1;
            phi_end = phi;
            lane_darthash<HK, CNT>(sp, idx, w, b0, b1, lane, tau, &range, cnt, [&](double rank, uint64_t s) {
                const uint32_t l = bucket_of(s, (uint32_t)L);
                const uint64_t rb = (uint64_t)__double_as_longlong(rank);
                // lanes reaching this point together may target the same table:
                // they insert one after another, lowest lane first
                uint64_t active = __ballot(true);
                while (active) {
                    const int ln = __ffsll((unsigned long long)active) - 1;
                    if (lane == ln) lsh_insert(T, K, l, rb, s);
                    active &= active - 1;
                }
            });
            if (wave_any(range)) { status = kSetRange; break; }
            wave_sync();
            bool full = true;
            for (int l = lane; l < L; l += kWave) full &= T.cnt[l] >= K;
            if (wave_all(full)) break;
            phi *= 2.0;
        }
    }
    wave_sync();
    for (int l = lane; l < L; l += kWave) {
        uint64_t h = 0;
        if (status == kSetOk) {
            const Hasher<HK> H(sp);
            h = H(sp->key_l ^ (uint64_t)l);
            for (int m = 0; m < K; ++m) h = H(h ^ T.sval[(size_t)l * K + m]);
        }
        out_keys[set * L + l] = h;
    }
    if (out_status && lane == 0) out_status[set] = status;
    if (CNT && out_cnt) write_counts(out_cnt, set, lane, cnt, passes, phi_end);
}

}  // namespace dms

namespace dms {

int plain_waves_per_block(int k)
{
    int w = 65536 / (16 * k);
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}

hipError_t launch_sketch_plain(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                               const int32_t* idx, const double* w, int k, uint32_t* out_u32,
                               uint64_t* out_bits, int8_t* out_status, uint64_t* out_s,
                               double* out_rank, double phi0, double phi_max, int hash,
                               const LaunchExtras& x, hipStream_t st)
{
    if (n_sets <= 0) return hipSuccess;
    const int waves = plain_waves_per_block(k);
    const int64_t blocks = (n_sets + waves - 1) / waves;
    const size_t lds = (size_t)waves * 16 * k;
    const bool cnt = x.counters != nullptr;
    auto kern = hash == kHashTab ? (cnt ? sketch_plain_kernel<kHashTab, true> : sketch_plain_kernel<kHashTab, false>)
                                 : (cnt ? sketch_plain_kernel<kHashMix, true> : sketch_plain_kernel<kHashMix, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), lds, st, sp,
                       n_sets, rp, idx, w, k, out_u32, out_bits, out_status, out_s, out_rank,
                       phi0, phi_max, x.counters, x.repeated);
    return hipGetLastError();
}

hipError_t launch_lsh_plain(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                            const int32_t* idx, const double* w, int L, int K, uint64_t* out_keys,
                            int8_t* out_status, double phi0, double phi_max, int hash,
                            const LaunchExtras& x, hipStream_t st)
{
    if (n_sets <= 0) return hipSuccess;
    const size_t per_wave = ((size_t)2 * L * K + L) * 8;
    int waves = (int)(65536 / per_wave);
    waves = waves < 1 ? 1 : (waves > 4 ? 4 : waves);
    const int64_t blocks = (n_sets + waves - 1) / waves;
    const bool cnt = x.counters != nullptr;
    auto kern = hash == kHashTab ? (cnt ? lsh_plain_kernel<kHashTab, true> : lsh_plain_kernel<kHashTab, false>)
                                 : (cnt ? lsh_plain_kernel<kHashMix, true> : lsh_plain_kernel<kHashMix, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves),
                       per_wave * waves, st, sp, n_sets, rp, idx, w, L, K, out_keys, out_status,
                       phi0, phi_max, x.counters, x.repeated);
    return hipGetLastError();
}

}  // namespace dms
