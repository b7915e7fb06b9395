// Flattened DartMinHash kernel for gfx950.
//
// One wavefront sketches one set at a time, pulling set indices from a global
// counter until the batch is exhausted (persistent grid, work stealing).  The
// five nested loops of Algorithm 1 are flattened into four stages that always
// run 64 lanes wide, connected by queues in LDS:
//
//   elements --region round-->  region queue  (g, x_i, row count, area count)
//            --area round---->  dart queue    (area hash a, x_i, w, r, nu, rho, j)
//            --dart round---->  pass queue    (darts with rank <= tau)
//            --accept round-->  buckets       (weight <= x_i: id hash, bucket minimum)
//
// A region round expands elements into their (nu, rho) regions, an area round
// expands regions into areas and draws each area's Poisson(1) dart count, a
// dart round draws the rank uniform of 64 darts and compacts the survivors, an
// accept round draws the weight uniform, filters and inserts into the
// buckets.  The per-region column and row counts are computed in closed form
// and corrected with the exact loop-exit predicate, so the set of visited
// areas is exactly the one of Algorithm 1's loops (see dms_plain.hip).
#include "dms_device.h"

namespace dms {

namespace {

constexpr int kCapR = 128;  // region queue (items)
constexpr int kCapD = 256;  // dart queue
constexpr int kCapP = 128;  // pass queue

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint32_t scan_add(uint32_t v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, (unsigned)o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Inclusive prefix maximum over the 64 lanes.
__device__ __forceinline__ int32_t scan_max(int32_t v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(v, (unsigned)o, kWave);
        if (lane >= o) v = v > t ? v : t;
    }
    return v;
}

__device__ __forceinline__ uint32_t poisson_fast(const uint64_t* __restrict__ pois, uint64_t a)
{
    uint32_t x = (a >= pois[0]) + (a >= pois[1]) + (a >= pois[2]) + (a >= pois[3]) +
                 (a >= pois[4]) + (a >= pois[5]) + (a >= pois[6]) + (a >= pois[7]);
    if (x == 8) {
        while (x < (uint32_t)kNumPoisson && a >= pois[x]) ++x;
    }
    return x;
}

struct Queues {
    // buckets
    uint64_t* rank_bits;
    uint64_t* sval;
    // region queue
    uint64_t* rq_g;
    double* rq_x;
    uint32_t* rq_rc;
    uint32_t* rq_na;
    uint32_t* rq_m;
    // dart queue
    uint64_t* dq_a;
    double* dq_x;
    uint32_t* dq_r;
    uint32_t* dq_w;
    uint32_t* dq_m;
    // pass queue
    uint64_t* pq_a;
    double* pq_x;
    uint64_t* pq_rank;
    uint32_t* pq_w;
    uint32_t* pq_m;
    // expansion marks
    int32_t* mark;
};

// bytes of LDS per wave for k buckets
__host__ __device__ constexpr size_t wave_lds_bytes(int k)
{
    return (size_t)16 * k + (size_t)kCapR * 28 + (size_t)kCapD * 28 + (size_t)kCapP * 32 + 64 * 4;
}

__device__ __forceinline__ Queues carve(unsigned char* p, int k)
{
    Queues q;
    q.rank_bits = (uint64_t*)p; p += 8 * (size_t)k;
    q.sval = (uint64_t*)p; p += 8 * (size_t)k;
    q.rq_g = (uint64_t*)p; p += 8 * kCapR;
    q.rq_x = (double*)p; p += 8 * kCapR;
    q.dq_a = (uint64_t*)p; p += 8 * kCapD;
    q.dq_x = (double*)p; p += 8 * kCapD;
    q.pq_a = (uint64_t*)p; p += 8 * kCapP;
    q.pq_x = (double*)p; p += 8 * kCapP;
    q.pq_rank = (uint64_t*)p; p += 8 * kCapP;
    q.rq_rc = (uint32_t*)p; p += 4 * kCapR;
    q.rq_na = (uint32_t*)p; p += 4 * kCapR;
    q.rq_m = (uint32_t*)p; p += 4 * kCapR;
    q.dq_r = (uint32_t*)p; p += 4 * kCapD;
    q.dq_w = (uint32_t*)p; p += 4 * kCapD;
    q.dq_m = (uint32_t*)p; p += 4 * kCapD;
    q.pq_w = (uint32_t*)p; p += 4 * kCapP;
    q.pq_m = (uint32_t*)p; p += 4 * kCapP;
    q.mark = (int32_t*)p;
    return q;
}

// Number of c in [0, cap) with base + c * step <= bound, for a predicate that
// is monotone in c and true at c = 0.  `est` is a closed-form guess; the
// exact predicate corrects it.  Counts are exact below 2^53.
__device__ __forceinline__ double exact_count(double base, double step_scale_exp_base,
                                              int step_exp, double bound, double cap, double est)
{
    // step = ldexp(step_scale_exp_base, step_exp)
    double c = est;
    if (!(c >= 1.0)) c = 1.0;
    if (c > cap) c = cap;
    while (c < cap && base + c * ldexp(step_scale_exp_base, step_exp) <= bound) c += 1.0;
    while (c > 1.0 && !(base + (c - 1.0) * ldexp(step_scale_exp_base, step_exp) <= bound)) c -= 1.0;
    return c;
}

}  // namespace

// Persistent flattened DartMinHash.  grid * (blockDim/64) waves; each wave
// repeatedly takes the next set index from *next_set.
__global__ void __launch_bounds__(256)
sketch_fast_kernel(const SpecTables* __restrict__ sp, int64_t n_sets,
                   const int64_t* __restrict__ rp, const int32_t* __restrict__ idx,
                   const double* __restrict__ wts, int k, uint32_t* out_u32, uint64_t* out_bits,
                   int8_t* out_status, uint64_t* out_s, double* out_rank, double phi0,
                   double phi_max, unsigned long long* next_set)
{
    extern __shared__ unsigned char smem[];
    double* sW = (double*)smem;
    double* sR = sW + kTable;
    for (int i = threadIdx.x; i < kTable; i += blockDim.x) {
        sW[i] = sp->W[i];
        sR[i] = sp->R[i];
    }
    __syncthreads();  // the only block barrier

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    Queues Q = carve(smem + 16 * kTable + (size_t)wave * wave_lds_bytes(k), k);

    const uint64_t KR = sp->key_r, KA = sp->key_a, KU = sp->key_u, KV = sp->key_v, KS = sp->key_s;
    const double u = sp->u;
    const double td = (double)sp->t;

    for (;;) {
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(next_set, 1ull);
        const int64_t set = (int64_t)__shfl(got, 0, kWave);
        if (set >= n_sets) break;

        const int64_t b0 = rp[set], b1 = rp[set + 1];
        const RowInfo ri = scan_row(wts, b0, b1, lane);
        int8_t status = ri.status;
        if (status == kSetOk) {
            for (int j = lane; j < k; j += kWave) {
                Q.rank_bits[j] = kRankEmpty;
                Q.sval[j] = ~0ull;
            }
            double phi = phi0;
            double tau_prev = -1.0;  // darts of rank <= tau_prev are already in the buckets
            for (;;) {
                if (phi > phi_max) { status = kSetRange; break; }
                const double tau = phi / ri.sum;
                // rho runs over 0 .. B1-1: the rows whose lower corner is <= tau
                int B1 = 0;
                while (B1 < kTable && sR[B1] <= tau) ++B1;
                bool range = B1 >= kTable;

                // ---- pipeline state (wave-uniform) ----
                int64_t chunk = b0;          // first element of the current chunk
                uint32_t chunk_total = 0;    // regions in the current chunk
                uint32_t reg_done = 0;       // regions of the chunk already queued
                double ex = 0.0;             // this lane's element weight
                uint32_t eid = 0;            // this lane's element id
                uint32_t nreg_incl = 0;      // inclusive prefix of region counts
                uint32_t nreg = 0;
                uint32_t rq_head = 0, rq_count = 0, rq_consumed = 0;
                double rq_pending = 0.0;     // areas left in the region queue
                uint32_t dq_head = 0, dq_count = 0;
                uint32_t pq_head = 0, pq_count = 0;
                bool have_chunk = false;

                auto load_chunk = [&]() {
                    // advance to the next chunk holding at least one region
                    have_chunk = false;
                    while (!have_chunk && chunk < b1) {
                        const int64_t e = chunk + lane;
                        ex = 0.0;
                        eid = 0;
                        nreg = 0;
                        if (e < b1) {
                            ex = wts[e];
                            eid = (uint32_t)idx[e];
                        }
                        if (ex > 0.0) {
                            // weight rows: nu with W[nu] <= x (W[0] = 0)
                            int A = ilogb(1.0 + td * ex) + 1;
                            if (A < 1) A = 1;
                            if (A > kTable) A = kTable;
                            while (A < kTable && sW[A] <= ex) ++A;
                            while (A > 1 && sW[A - 1] > ex) --A;
                            if (A >= kTable) range = true;
                            nreg = (uint32_t)A * (uint32_t)B1;
                        }
                        nreg_incl = scan_add(nreg, lane);
                        chunk_total = uni((uint32_t)__shfl(nreg_incl, 63, kWave));
                        reg_done = 0;
                        have_chunk = chunk_total > 0;
                        if (!have_chunk) chunk += kWave;
                    }
                };
                load_chunk();

                for (;;) {
                    wave_sync();
                    if (wave_any(range)) break;
                    if (pq_count >= 64 || (pq_count > 0 && dq_count == 0 && rq_pending == 0.0 && !have_chunk)) {
                        // ---- accept round ----
                        const uint32_t m = pq_count < 64 ? pq_count : 64;
                        if ((uint32_t)lane < m) {
                            const uint32_t pos = (pq_head + lane) & (kCapP - 1);
                            const uint64_t a = Q.pq_a[pos];
                            const double xi = Q.pq_x[pos];
                            const uint32_t wv = Q.pq_w[pos];
                            const uint32_t meta = Q.pq_m[pos];
                            const int nu = meta & 511, rho = (meta >> 9) & 511;
                            const uint64_t j = meta >> 18;
                            const double V = unit53(mix64(a ^ KV ^ j));
                            const double weight = sW[nu] + ((double)wv + V) * ldexp(u, nu - rho);
                            if (weight <= xi) {
                                const uint64_t s = mix64(a ^ KS ^ j);
                                bucket_min(Q.rank_bits, Q.sval, bucket_of(s, (uint32_t)k),
                                           Q.pq_rank[pos], s);
                            }
                        }
                        pq_head = (pq_head + m) & (kCapP - 1);
                        pq_count -= m;
                    } else if (dq_count >= 64 || (dq_count > 0 && rq_pending == 0.0 && !have_chunk)) {
                        // ---- dart round ----
                        const uint32_t m = dq_count < 64 ? dq_count : 64;
                        bool pass = false;
                        uint64_t a = 0, rbits = 0;
                        double xi = 0.0;
                        uint32_t wv = 0, meta = 0;
                        if ((uint32_t)lane < m) {
                            const uint32_t pos = (dq_head + lane) & (kCapD - 1);
                            a = Q.dq_a[pos];
                            xi = Q.dq_x[pos];
                            const uint32_t rv = Q.dq_r[pos];
                            wv = Q.dq_w[pos];
                            meta = Q.dq_m[pos];
                            const int nu = meta & 511, rho = (meta >> 9) & 511;
                            const uint64_t j = meta >> 18;
                            const double U = unit53(mix64(a ^ KU ^ j));
                            const double rank = sR[rho] + ((double)rv + U) * ldexp(1.0, rho - nu);
                            pass = rank <= tau && rank > tau_prev;
                            rbits = (uint64_t)__double_as_longlong(rank);
                        }
                        const uint64_t bal = __ballot(pass);
                        if (pass) {
                            const uint32_t before = (uint32_t)__builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                            const uint32_t pos = (pq_head + pq_count + before) & (kCapP - 1);
                            Q.pq_a[pos] = a;
                            Q.pq_x[pos] = xi;
                            Q.pq_rank[pos] = rbits;
                            Q.pq_w[pos] = wv;
                            Q.pq_m[pos] = meta;
                        }
                        pq_count += (uint32_t)__popcll(bal);
                        dq_head = (dq_head + m) & (kCapD - 1);
                        dq_count -= m;
                    } else if (rq_pending >= 64.0 || (rq_pending > 0.0 && !have_chunk)) {
                        // ---- area round ----
                        const uint32_t n_items = rq_count < 64 ? rq_count : 64;
                        uint32_t na = 0, c = 0;
                        if ((uint32_t)lane < n_items) {
                            na = Q.rq_na[(rq_head + lane) & (kCapR - 1)];
                            c = na - (lane == 0 ? rq_consumed : 0u);
                        }
                        const uint32_t cc = c < 64 ? c : 64;
                        const uint32_t incl = scan_add(cc, lane);
                        const uint32_t excl = incl - cc;
                        const uint32_t total = uni((uint32_t)__shfl(incl, 63, kWave));
                        uint32_t m = total < 64 ? total : 64;
                        if (m == 0) {  // bookkeeping guard: never spin without progress
                            range = true;
                            continue;
                        }
                        // owner of each of the m positions
                        Q.mark[lane] = 0;
                        wave_sync();
                        if (cc > 0 && excl < 64) Q.mark[excl] = lane;
                        wave_sync();
                        const int32_t src = scan_max(Q.mark[lane], lane);
                        const uint32_t s_excl = (uint32_t)__shfl(excl, src, kWave);
                        const uint32_t local = (uint32_t)lane - s_excl + (src == 0 ? rq_consumed : 0u);
                        uint32_t X = 0;
                        uint64_t a = 0;
                        double xi = 0.0;
                        uint32_t wv = 0, rv = 0, meta = 0;
                        if ((uint32_t)lane < m) {
                            const uint32_t ip = (rq_head + (uint32_t)src) & (kCapR - 1);
                            const uint64_t g = Q.rq_g[ip];
                            xi = Q.rq_x[ip];
                            const uint32_t rc = Q.rq_rc[ip];
                            const uint32_t nai = Q.rq_na[ip];
                            meta = Q.rq_m[ip];
                            if (rc == 1) {
                                wv = local;
                                rv = 0;
                            } else if (nai == rc) {
                                wv = 0;
                                rv = local;
                            } else {
                                wv = local / rc;
                                rv = local - wv * rc;
                            }
                            a = mix64(g ^ KA ^ (((uint64_t)wv << 32) | rv));
                            X = poisson_fast(sp->pois, a);
                        }
                        // keep only a prefix of areas whose darts fit in the dart queue
                        uint32_t xincl = scan_add(X, lane);
                        const uint32_t room = kCapD - dq_count;
                        const uint64_t fit = __ballot((uint32_t)lane < m && xincl <= room);
                        const uint32_t m2 = (uint32_t)__popcll(fit);  // a prefix, xincl grows
                        if ((uint32_t)lane < m2 && X > 0) {
                            const uint32_t first = dq_head + dq_count + xincl - X;
                            for (uint32_t j = 0; j < X; ++j) {
                                const uint32_t pos = (first + j) & (kCapD - 1);
                                Q.dq_a[pos] = a;
                                Q.dq_x[pos] = xi;
                                Q.dq_r[pos] = rv;
                                Q.dq_w[pos] = wv;
                                Q.dq_m[pos] = meta | (j << 18);
                            }
                        }
                        dq_count += uni((uint32_t)__shfl(xincl, (int)m2 - 1, kWave));
                        // advance the region queue by m2 areas
                        const int32_t last_src = __shfl(src, (int)m2 - 1, kWave);
                        const uint32_t last_local = (uint32_t)__shfl(local, (int)m2 - 1, kWave);
                        const uint32_t last_na = (uint32_t)__shfl(na, last_src, kWave);
                        if (last_local + 1 == last_na) {
                            rq_head = (rq_head + (uint32_t)last_src + 1) & (kCapR - 1);
                            rq_count -= (uint32_t)last_src + 1;
                            rq_consumed = 0;
                        } else {
                            rq_head = (rq_head + (uint32_t)last_src) & (kCapR - 1);
                            rq_count -= (uint32_t)last_src;
                            rq_consumed = last_local + 1;
                        }
                        rq_pending -= (double)m2;
                    } else if (have_chunk) {
                        // ---- region round ----
                        const uint32_t left = chunk_total - reg_done;
                        const uint32_t m = left < 64 ? left : 64;
                        const uint32_t excl = nreg_incl - nreg;
                        Q.mark[lane] = 0;
                        wave_sync();
                        if (nreg > 0 && excl + nreg > reg_done && excl < reg_done + 64)
                            Q.mark[excl > reg_done ? excl - reg_done : 0] = lane;
                        wave_sync();
                        const int32_t src = scan_max(Q.mark[lane], lane);
                        const double x = __shfl(ex, src, kWave);
                        const uint32_t id = (uint32_t)__shfl(eid, src, kWave);
                        const uint32_t s_excl = (uint32_t)__shfl(excl, src, kWave);
                        uint32_t na = 0;
                        if ((uint32_t)lane < m) {
                            const uint32_t local = reg_done + (uint32_t)lane - s_excl;
                            uint32_t nu = (uint32_t)((float)local / (float)B1);
                            while (nu * (uint32_t)B1 > local) --nu;
                            while ((nu + 1) * (uint32_t)B1 <= local) ++nu;
                            const uint32_t rho = local - nu * (uint32_t)B1;
                            const double Wn = sW[nu], Rr = sR[rho];
                            const uint64_t g = mix64(KR ^ (((uint64_t)id << 32) | ((uint64_t)nu << 16) | rho));
                            // columns: w < 2^rho with W + w * dnu <= x
                            const double wcap = ldexp(1.0, (int)rho);
                            const double west = floor((x - Wn) * td * ldexp(1.0, (int)rho - (int)nu)) + 1.0;
                            const double wc = exact_count(Wn, u, (int)nu - (int)rho, x, wcap, west);
                            // rows: r < 2^nu with R + r * drho <= tau
                            const double rcap = ldexp(1.0, (int)nu);
                            const double rest = floor((tau - Rr) * ldexp(1.0, (int)nu - (int)rho)) + 1.0;
                            const double rcn = exact_count(Rr, 1.0, (int)rho - (int)nu, tau, rcap, rest);
                            const double nad = wc * rcn;
                            if (wc > 4294967296.0 || rcn > 4294967296.0 || nad >= 2147483648.0)
                                range = true;
                            na = range ? 1u : (uint32_t)nad;
                            const uint32_t qp = (rq_head + rq_count + (uint32_t)lane) & (kCapR - 1);
                            Q.rq_g[qp] = g;
                            Q.rq_x[qp] = x;
                            Q.rq_rc[qp] = range ? 1u : (uint32_t)rcn;
                            Q.rq_na[qp] = na;
                            Q.rq_m[qp] = nu | (rho << 9);
                        }
                        rq_pending += wave_sum((double)na);
                        rq_count += m;
                        reg_done += m;
                        if (reg_done == chunk_total) {
                            chunk += kWave;
                            load_chunk();
                        }
                    } else {
                        break;  // every queue drained, every element visited
                    }
                }
                if (wave_any(range)) { status = kSetRange; break; }
                wave_sync();
                bool filled = true;
                for (int j = lane; j < k; j += kWave) filled &= Q.rank_bits[j] != kRankEmpty;
                if (wave_all(filled)) break;
                tau_prev = tau;
                phi *= 2.0;
            }
        }
        // outputs
        wave_sync();
        const bool ok = status == kSetOk;
        for (int j = lane; j < k; j += kWave) {
            const uint64_t s = ok ? Q.sval[j] : ~0ull;
            const uint64_t rb = ok ? Q.rank_bits[j] : kRankEmpty;
            if (out_u32) out_u32[set * k + j] = ok ? (uint32_t)s : 0xFFFFFFFFu;
            if (out_s) out_s[set * k + j] = s;
            if (out_rank) out_rank[set * k + j] = __longlong_as_double((long long)rb);
        }
        if (out_bits) {
            const int words = (k + 63) / 64;
            for (int wd = 0; wd < words; ++wd) {
                const int j = wd * 64 + lane;
                const bool bit = ok && j < k && (Q.sval[j] & 1ull);
                const uint64_t word = __ballot(bit);
                if (lane == 0) out_bits[(int64_t)set * words + wd] = word;
            }
        }
        if (out_status && lane == 0) out_status[set] = status;
    }
}

__global__ void reset_counter_kernel(unsigned long long* c) { *c = 0ull; }

int fast_waves_per_block(int k)
{
    const size_t per = wave_lds_bytes(k);
    int w = (int)((65536 - 16 * kTable) / per);
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}

size_t fast_lds_bytes(int k, int waves) { return 16 * kTable + (size_t)waves * wave_lds_bytes(k); }

hipError_t launch_sketch_fast(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                              const int32_t* idx, const double* w, int k, uint32_t* out_u32,
                              uint64_t* out_bits, int8_t* out_status, uint64_t* out_s,
                              double* out_rank, double phi0, double phi_max,
                              unsigned long long* counter, int blocks, hipStream_t st)
{
    if (n_sets <= 0) return hipSuccess;
    const int waves = fast_waves_per_block(k);
    const size_t lds = fast_lds_bytes(k, waves);
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    const int64_t need = (n_sets + waves - 1) / waves;
    if (blocks <= 0 || blocks > need) blocks = (int)(need < 1 ? 1 : need);
    hipLaunchKernelGGL(sketch_fast_kernel, dim3((unsigned)blocks), dim3(64 * waves), lds, st, sp,
                       n_sets, rp, idx, w, k, out_u32, out_bits, out_status, out_s, out_rank, phi0,
                       phi_max, counter);
    return hipGetLastError();
}

}  // namespace dms
