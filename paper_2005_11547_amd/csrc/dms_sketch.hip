// Flattened DartMinHash kernel for gfx950.
//
// One wavefront sketches one set at a time, pulling set indices from a global
// counter until the batch is exhausted (persistent grid, work stealing).  The
// five nested loops of Algorithm 1 are flattened into four kinds of rounds
// that run 64 lanes wide, connected by small queues in LDS:
//
//   region round : expands elements into their (nu, rho) regions, hashes the
//                  region (g) and its first area (a), draws that area's
//                  Poisson(1) dart count; regions with more areas go to the
//                  region queue, areas with darts to the dart queue.
//   area round   : expands queued regions into their remaining areas, hashes
//                  them and draws their dart counts.
//   dart round   : draws the rank uniform of one dart per queued area; darts
//                  with rank <= tau go to the pass queue; an area with more
//                  darts goes back to the dart queue.
//   accept round : draws the weight uniform; darts with weight <= x_i get their
//                  id hash and enter the bucket minima.
//
// Column and row counts of a region come from a closed form corrected with the
// exact loop-exit predicate, so the visited areas are exactly those of
// Algorithm 1's loops with their early exits (the plain kernel in
// dms_plain.hip walks those loops literally).
#include "dms_device.h"

namespace dms {

namespace {

constexpr int kCapR = 128;  // region queue (regions with areas left)
constexpr int kCapD = 128;  // dart queue (areas with darts left)
constexpr int kCapP = 128;  // pass queue (darts with rank <= tau)

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Inclusive prefix sum over the 64 lanes (DPP row shifts and row broadcasts).
// Must be called with all 64 lanes active.
__device__ __forceinline__ uint32_t scan_add(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Inclusive prefix maximum of non-negative values over the 64 lanes.
__device__ __forceinline__ int32_t scan_max(int32_t v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));
    return v;
}

__device__ __forceinline__ uint32_t lane63(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Number of lanes below this one whose bit is set in `mask`.
__device__ __forceinline__ uint32_t rank_in(uint64_t mask)
{
    return (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
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

// LDS of one wave.
struct Queues {
    uint64_t* rank_bits;  // [k] bucket minima
    uint64_t* sval;       // [k]
    uint64_t* rq_g;       // region queue
    double* rq_x;
    uint32_t* rq_rc;      // rows of the region
    uint32_t* rq_na;      // areas of the region
    uint32_t* rq_first;   // areas already taken
    uint32_t* rq_m;       // nu | rho << 9
    uint64_t* dq_a;       // dart queue: area hash
    double* dq_x;
    uint32_t* dq_r;
    uint32_t* dq_w;
    uint32_t* dq_m;       // nu | rho << 9 | j << 18 | X << 23
    uint64_t* pq_a;       // pass queue
    double* pq_x;
    uint64_t* pq_rank;
    uint32_t* pq_w;
    uint32_t* pq_m;       // nu | rho << 9 | j << 18
    int32_t* mark;        // [64]
};

__host__ __device__ constexpr size_t wave_lds_bytes(int k)
{
    return (size_t)16 * k + (size_t)kCapR * 32 + (size_t)kCapD * 28 + (size_t)kCapP * 32 + 64 * 4;
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
    q.rq_first = (uint32_t*)p; p += 4 * kCapR;
    q.rq_m = (uint32_t*)p; p += 4 * kCapR;
    q.dq_r = (uint32_t*)p; p += 4 * kCapD;
    q.dq_w = (uint32_t*)p; p += 4 * kCapD;
    q.dq_m = (uint32_t*)p; p += 4 * kCapD;
    q.pq_w = (uint32_t*)p; p += 4 * kCapP;
    q.pq_m = (uint32_t*)p; p += 4 * kCapP;
    q.mark = (int32_t*)p;
    return q;
}

// Number of c in [0, cap) with base + c * step <= bound (an exit predicate
// that is monotone in c and true at c = 0), starting from the estimate est.
__device__ __forceinline__ double exact_count(double base, double step, double bound, double cap,
                                              double est)
{
    double c = est;
    if (!(c >= 1.0)) c = 1.0;
    if (c > cap) c = cap;
    while (c < cap && base + c * step <= bound) c += 1.0;
    while (c > 1.0 && !(base + (c - 1.0) * step <= bound)) c -= 1.0;
    return c;
}

}  // namespace

// Persistent flattened DartMinHash; each wave repeatedly takes the next set
// index from *next_set.
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
    const uint64_t* pois = sp->pois;

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
                const float inv_b1 = 1.0f / (float)B1;

                int64_t chunk = b0;        // first element of the current chunk
                uint32_t chunk_total = 0;  // regions of the chunk
                uint32_t reg_done = 0;     // regions of the chunk already expanded
                double ex = 0.0;           // this lane's element weight
                uint32_t eid = 0;          // this lane's element id
                uint32_t nreg = 0, nreg_excl = 0;
                bool have_chunk = false;
                uint32_t rq_head = 0, rq_count = 0, dq_head = 0, dq_count = 0;
                uint32_t pq_head = 0, pq_count = 0;
                uint64_t rq_pending = 0;   // areas left in the region queue

                auto load_chunk = [&]() {
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
                            A = A < 1 ? 1 : (A > kTable ? kTable : A);
                            while (A < kTable && sW[A] <= ex) ++A;
                            while (A > 1 && sW[A - 1] > ex) --A;
                            if (A >= kTable) range = true;
                            nreg = (uint32_t)A * (uint32_t)B1;
                        }
                        const uint32_t incl = scan_add(nreg);
                        nreg_excl = incl - nreg;
                        chunk_total = uni(lane63(incl));
                        reg_done = 0;
                        have_chunk = chunk_total > 0;
                        if (!have_chunk) chunk += kWave;
                    }
                };
                load_chunk();

                for (;;) {
                    wave_sync();
                    if (pq_count >= 64 || (pq_count > 0 && dq_count == 0 && rq_count == 0 && !have_chunk)) {
                        // ---------------- accept round ----------------
                        const uint32_t m = pq_count < 64 ? pq_count : 64;
                        if ((uint32_t)lane < m) {
                            const uint32_t pos = (pq_head + lane) & (kCapP - 1);
                            const uint64_t a = Q.pq_a[pos];
                            const double xi = Q.pq_x[pos];
                            const uint32_t wv = Q.pq_w[pos];
                            const uint32_t meta = Q.pq_m[pos];
                            const uint64_t rb = Q.pq_rank[pos];
                            const int nu = meta & 511, rho = (meta >> 9) & 511;
                            const uint64_t j = (meta >> 18) & 31;
                            const double V = unit53(mix64(a ^ KV ^ j));
                            const double weight = sW[nu] + ((double)wv + V) * ldexp(u, nu - rho);
                            if (weight <= xi) {
                                const uint64_t s = mix64(a ^ KS ^ j);
                                bucket_min(Q.rank_bits, Q.sval, bucket_of(s, (uint32_t)k), rb, s);
                            }
                        }
                        pq_head = (pq_head + m) & (kCapP - 1);
                        pq_count -= m;
                    } else if (dq_count >= 64 || (dq_count > 0 && rq_count == 0 && !have_chunk)) {
                        // ---------------- dart round ----------------
                        const uint32_t m = dq_count < 64 ? dq_count : 64;
                        const bool act = (uint32_t)lane < m;
                        uint64_t a = 0;
                        double xi = 0.0;
                        uint32_t rv = 0, wv = 0, meta = 0;
                        if (act) {
                            const uint32_t pos = (dq_head + lane) & (kCapD - 1);
                            a = Q.dq_a[pos];
                            xi = Q.dq_x[pos];
                            rv = Q.dq_r[pos];
                            wv = Q.dq_w[pos];
                            meta = Q.dq_m[pos];
                        }
                        const int nu = meta & 511, rho = (meta >> 9) & 511;
                        const uint32_t j = (meta >> 18) & 31, X = meta >> 23;
                        const double U = unit53(mix64(a ^ KU ^ (uint64_t)j));
                        const double rank = sR[rho] + ((double)rv + U) * ldexp(1.0, rho - nu);
                        const bool pass = act && rank <= tau && rank > tau_prev;
                        const bool more = act && j + 1 < X;
                        const uint64_t bp = __ballot(pass);
                        const uint64_t bm = __ballot(more);
                        wave_sync();  // every entry of the round is read before any write
                        if (pass) {
                            const uint32_t pos = (pq_head + pq_count + rank_in(bp)) & (kCapP - 1);
                            Q.pq_a[pos] = a;
                            Q.pq_x[pos] = xi;
                            Q.pq_rank[pos] = (uint64_t)__double_as_longlong(rank);
                            Q.pq_w[pos] = wv;
                            Q.pq_m[pos] = meta & ((1u << 23) - 1);
                        }
                        const uint32_t dq_left = dq_count - m;
                        if (more) {
                            const uint32_t pos = (dq_head + m + dq_left + rank_in(bm)) & (kCapD - 1);
                            Q.dq_a[pos] = a;
                            Q.dq_x[pos] = xi;
                            Q.dq_r[pos] = rv;
                            Q.dq_w[pos] = wv;
                            Q.dq_m[pos] = meta + (1u << 18);
                        }
                        pq_count += (uint32_t)__popcll(bp);
                        dq_head = (dq_head + m) & (kCapD - 1);
                        dq_count = dq_left + (uint32_t)__popcll(bm);
                    } else if (rq_pending >= 64 || (rq_count > 0 && !have_chunk)) {
                        // ---------------- area round ----------------
                        const uint32_t n_items = rq_count < 64 ? rq_count : 64;
                        uint32_t na = 0, first = 0, c = 0;
                        if ((uint32_t)lane < n_items) {
                            const uint32_t ip = (rq_head + lane) & (kCapR - 1);
                            na = Q.rq_na[ip];
                            first = Q.rq_first[ip];
                            c = na - first;
                        }
                        const uint32_t cc = c < 64 ? c : 64;
                        const uint32_t incl = scan_add(cc);
                        const uint32_t excl = incl - cc;
                        const uint32_t total = uni(lane63(incl));
                        const uint32_t m = total < 64 ? total : 64;
                        if (m == 0) {  // bookkeeping guard: never spin without progress
                            range = true;
                            break;
                        }
                        Q.mark[lane] = 0;
                        wave_sync();
                        if (cc > 0 && excl < 64) Q.mark[excl] = lane;
                        wave_sync();
                        const int32_t src = scan_max(Q.mark[lane]);
                        const uint32_t s_excl = (uint32_t)__shfl(excl, src, kWave);
                        const uint32_t s_first = (uint32_t)__shfl(first, src, kWave);
                        const uint32_t local = s_first + (uint32_t)lane - s_excl;
                        const bool act = (uint32_t)lane < m;
                        uint32_t X = 0, wv = 0, rv = 0, meta = 0;
                        uint64_t a = 0;
                        double xi = 0.0;
                        if (act) {
                            const uint32_t ip = (rq_head + (uint32_t)src) & (kCapR - 1);
                            const uint64_t g = Q.rq_g[ip];
                            xi = Q.rq_x[ip];
                            const uint32_t rc = Q.rq_rc[ip];
                            const uint32_t nai = Q.rq_na[ip];
                            meta = Q.rq_m[ip];
                            if (rc == 1) {
                                wv = local;
                            } else if (nai == rc) {
                                rv = local;
                            } else {
                                wv = local / rc;
                                rv = local - wv * rc;
                            }
                            a = mix64(g ^ KA ^ (((uint64_t)wv << 32) | rv));
                            X = poisson_fast(pois, a);
                        }
                        const bool push = act && X > 0;
                        const uint64_t bpush = __ballot(push);
                        if (push) {
                            const uint32_t pos = (dq_head + dq_count + rank_in(bpush)) & (kCapD - 1);
                            Q.dq_a[pos] = a;
                            Q.dq_x[pos] = xi;
                            Q.dq_r[pos] = rv;
                            Q.dq_w[pos] = wv;
                            Q.dq_m[pos] = meta | (X << 23);
                        }
                        dq_count += (uint32_t)__popcll(bpush);
                        // advance the region queue by m areas
                        const uint32_t last_src = (uint32_t)__builtin_amdgcn_readlane(src, (int)m - 1);
                        const uint32_t last_local = (uint32_t)__builtin_amdgcn_readlane((int)local, (int)m - 1);
                        const uint32_t last_na = (uint32_t)__builtin_amdgcn_readlane((int)na, (int)last_src);
                        if (last_local + 1 == last_na) {
                            rq_head = (rq_head + last_src + 1) & (kCapR - 1);
                            rq_count -= last_src + 1;
                        } else {
                            if (lane == 0) Q.rq_first[(rq_head + last_src) & (kCapR - 1)] = last_local + 1;
                            rq_head = (rq_head + last_src) & (kCapR - 1);
                            rq_count -= last_src;
                        }
                        rq_pending -= m;
                    } else if (have_chunk) {
                        // ---------------- region round ----------------
                        const uint32_t left = chunk_total - reg_done;
                        const uint32_t m = left < 64 ? left : 64;
                        Q.mark[lane] = 0;
                        wave_sync();
                        if (nreg > 0 && nreg_excl + nreg > reg_done && nreg_excl < reg_done + 64)
                            Q.mark[nreg_excl > reg_done ? nreg_excl - reg_done : 0] = lane;
                        wave_sync();
                        const int32_t src = scan_max(Q.mark[lane]);
                        const double x = __shfl(ex, src, kWave);
                        const uint32_t id = (uint32_t)__shfl(eid, src, kWave);
                        const uint32_t s_excl = (uint32_t)__shfl(nreg_excl, src, kWave);
                        const bool act = (uint32_t)lane < m;
                        uint32_t X = 0, rest = 0, meta = 0, rcu = 1, nau = 1;
                        uint64_t a = 0, g = 0;
                        if (act) {
                            const uint32_t local = reg_done + (uint32_t)lane - s_excl;
                            uint32_t nu = local, rho = 0;
                            if (B1 > 1) {
                                nu = (uint32_t)((float)local * inv_b1);
                                while (nu * (uint32_t)B1 > local) --nu;
                                while ((nu + 1) * (uint32_t)B1 <= local) ++nu;
                                rho = local - nu * (uint32_t)B1;
                            }
                            meta = nu | (rho << 9);
                            g = mix64(KR ^ (((uint64_t)id << 32) | ((uint64_t)nu << 16) | rho));
                            double wc = 1.0, rcn;
                            if (rho == 0) {
                                // R[0] = 0 and r * 2^-nu is exact: r <= tau * 2^nu
                                const double rcap = ldexp(1.0, (int)nu);
                                rcn = floor(ldexp(tau, (int)nu)) + 1.0;
                                rcn = rcn < rcap ? rcn : rcap;
                            } else {
                                const double Wn = sW[nu], Rr = sR[rho];
                                const double dnu = ldexp(u, (int)nu - (int)rho);
                                const double drho = ldexp(1.0, (int)rho - (int)nu);
                                const double wcap = ldexp(1.0, (int)rho);
                                wc = exact_count(Wn, dnu, x, wcap,
                                                 floor((x - Wn) * td * ldexp(1.0, (int)rho - (int)nu)) + 1.0);
                                const double rcap = ldexp(1.0, (int)nu);
                                rcn = exact_count(Rr, drho, tau, rcap,
                                                  floor((tau - Rr) * ldexp(1.0, (int)nu - (int)rho)) + 1.0);
                            }
                            const double nad = wc * rcn;
                            if (wc > 4294967296.0 || rcn > 4294967296.0 || nad >= 2147483648.0) {
                                range = true;
                            } else {
                                rcu = (uint32_t)rcn;
                                nau = (uint32_t)nad;
                            }
                            // the region's first area (w = 0, r = 0)
                            a = mix64(g ^ KA);
                            X = poisson_fast(pois, a);
                            rest = nau - 1;
                        }
                        const bool push_d = act && X > 0;
                        const bool push_r = act && rest > 0;
                        const uint64_t bd = __ballot(push_d);
                        const uint64_t br = __ballot(push_r);
                        if (push_d) {
                            const uint32_t pos = (dq_head + dq_count + rank_in(bd)) & (kCapD - 1);
                            Q.dq_a[pos] = a;
                            Q.dq_x[pos] = x;
                            Q.dq_r[pos] = 0;
                            Q.dq_w[pos] = 0;
                            Q.dq_m[pos] = meta | (X << 23);
                        }
                        if (push_r) {
                            const uint32_t pos = (rq_head + rq_count + rank_in(br)) & (kCapR - 1);
                            Q.rq_g[pos] = g;
                            Q.rq_x[pos] = x;
                            Q.rq_rc[pos] = rcu;
                            Q.rq_na[pos] = nau;
                            Q.rq_first[pos] = 1;
                            Q.rq_m[pos] = meta;
                        }
                        dq_count += (uint32_t)__popcll(bd);
                        rq_count += (uint32_t)__popcll(br);
                        // areas added to the region queue: sum of rest in two 16-bit halves
                        const uint32_t lo = scan_add(rest & 0xffffu), hi = scan_add(rest >> 16);
                        rq_pending += (uint64_t)uni(lane63(lo)) + ((uint64_t)uni(lane63(hi)) << 16);
                        reg_done += m;
                        if (wave_any(range)) break;
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
        wave_sync();  // the next set reuses this wave's LDS
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
