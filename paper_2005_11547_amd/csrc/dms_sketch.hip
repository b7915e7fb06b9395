// Flattened DartMinHash kernel for gfx950.
//
// One wavefront sketches one set at a time, pulling set indices from a global
// counter until the batch is exhausted (persistent grid, work stealing).  The
// five nested loops of Algorithm 1 are flattened into five kinds of rounds
// that run 64 lanes wide, connected by small queues in LDS:
//
//   low-band round : in a pass with tau < 1, the regions of an element below
//                  nu = -ilogb(tau) hold one area each; one lane per element
//                  hashes such a region, its area and its first dart's rank,
//                  up to three levels nu per round as independent hash chains.
//   region round : expands elements into their (nu, rho) regions, hashes the
//                  region (g) and its first area (a), tells from a whether the
//                  area holds no dart, one, or more, and draws its first
//                  dart's rank; regions with more areas go to the region queue,
//                  passing darts to the pass queue, areas with more darts to
//                  the dart queue.
//   area round   : expands queued regions into their remaining areas, hashes
//                  them and draws their first ranks (as above), up to 128 areas
//                  per round as two halves of independent hash chains.
//   dart round   : draws the rank uniform of the next dart of each queued
//                  area; darts with rank <= tau go to the pass queue; an area
//                  with more darts (one more Poisson threshold reached) goes
//                  back to the dart queue.
//   accept round : draws the weight uniform; darts with weight <= x_i get their
//                  id hash and enter the sink (bucket minima, LSH tables or the
//                  bottom-k buffer).
//
// Every decision about which round runs is wave-uniform, and the compiler
// sees it (scalar branches and registers); inside a round, lanes without work
// are masked by their flags rather than branched around.
//
// Column and row counts of a region come from a closed form corrected with the
// exact loop-exit predicate (prefix_count), so the visited areas are exactly
// those of Algorithm 1's loops with their early exits.
#include "dms_device.h"
#include "dms_launch.h"

namespace dms {

namespace {

// Every queue is a ring.  A round consumes up to 64 entries and pushes at most
// 64 into each queue it feeds, and it runs only while every queue it feeds
// holds at most cap - 64 entries (its consumer takes priority above that), so
// no ring overflows; a round that makes a second level or half pushes it only
// after checking that the queues still have room for it.  The region ring is the smaller one: its rounds are the
// costliest, and region entries come from few rounds; the dart and pass rings
// hold two rounds so that their (cheaper) consumers always run 64 lanes wide.
// With these sizes three waves of k = 256 fit 40,960 bytes, so twelve waves
// share a CU.
#ifndef DMS_CAP_R
#define DMS_CAP_R 80
#endif
#ifndef DMS_CAP_D
#define DMS_CAP_D 128
#endif
#ifndef DMS_CAP_P
#define DMS_CAP_P 128
#endif
constexpr uint32_t kCapR = DMS_CAP_R;  // region queue (regions with areas left)
constexpr uint32_t kCapD = DMS_CAP_D;  // dart queue (areas with darts left)
constexpr uint32_t kCapP = DMS_CAP_P;  // pass queue (darts with rank <= tau)
static_assert(kCapR >= 64 && kCapD >= 64 && kCapP >= 64, "a round moves up to 64 entries");
constexpr uint32_t kTrigR = kCapR - 64, kTrigD = kCapD - 64, kTrigP = kCapP - 64;
// Low-band levels made per round (independent hash chains between LDS round trips).
constexpr int kLowLevels = 3;

// Ring slot of a position below 3 * cap (a head below cap plus two counts).
template <uint32_t CAP>
__device__ __forceinline__ uint32_t ring(uint32_t p)
{
    if ((CAP & (CAP - 1)) == 0) return p & (CAP - 1);
    p = min(p, p - 2u * CAP);  // unsigned: wraps to a large value when p < 2 * CAP
    return min(p, p - CAP);
}
__device__ __forceinline__ uint32_t ring_r(uint32_t p) { return ring<kCapR>(p); }
// Ring slot of a position below 2 * cap (a head plus at most 64 entries).
__device__ __forceinline__ uint32_t ring_r1(uint32_t p)
{
    return (kCapR & (kCapR - 1)) == 0 ? p & (kCapR - 1) : min(p, p - kCapR);
}
__device__ __forceinline__ uint32_t ring_d(uint32_t p) { return ring<kCapD>(p); }
__device__ __forceinline__ uint32_t ring_p(uint32_t p) { return ring<kCapP>(p); }

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

// min(X, 2) for the Poisson(1) count X of an area hash: enough to tell an
// empty area, a one-dart area and an area with more darts apart.
__device__ __forceinline__ uint32_t poisson_head(uint64_t C0, uint64_t C1, uint64_t a)
{
    return (uint32_t)(a >= C0) + (uint32_t)(a >= C1);
}

// LDS of one wave: queues at fixed offsets from the wave's base, then the k
// bucket minima.  Offsets are compile-time constants so that every access is
// one base register plus an immediate.
// Entries name their element by its offset e from the first element of the
// pass (the weight itself is read back from the CSR only by the accept round).
constexpr uint32_t kOffRqG = 0;                              // u64[kCapR] region hash
constexpr uint32_t kOffDqA = kOffRqG + 8 * kCapR;            // u64[kCapD] area hash
constexpr uint32_t kOffPqA = kOffDqA + 8 * kCapD;            // u64[kCapP] area hash
constexpr uint32_t kOffPqRank = kOffPqA + 8 * kCapP;         // u64[kCapP] rank bits
constexpr uint32_t kOffRqE = kOffPqRank + 8 * kCapP;         // u32[kCapR] element offset
constexpr uint32_t kOffRqRc = kOffRqE + 4 * kCapR;           // u32[kCapR] rows
constexpr uint32_t kOffRqNa = kOffRqRc + 4 * kCapR;          // u32[kCapR] areas
constexpr uint32_t kOffRqFirst = kOffRqNa + 4 * kCapR;       // u32[kCapR] areas taken
constexpr uint32_t kOffRqM = kOffRqFirst + 4 * kCapR;        // u32[kCapR] nu | rho << 10
constexpr uint32_t kOffDqE = kOffRqM + 4 * kCapR;            // u32[kCapD]
constexpr uint32_t kOffDqR = kOffDqE + 4 * kCapD;            // u32[kCapD]
constexpr uint32_t kOffDqW = kOffDqR + 4 * kCapD;            // u32[kCapD]
constexpr uint32_t kOffDqM = kOffDqW + 4 * kCapD;            // u32[kCapD] nu|rho<<10|j<<20
constexpr uint32_t kOffPqE = kOffDqM + 4 * kCapD;            // u32[kCapP]
constexpr uint32_t kOffPqW = kOffPqE + 4 * kCapP;            // u32[kCapP]
constexpr uint32_t kOffPqM = kOffPqW + 4 * kCapP;            // u32[kCapP] nu|rho<<10|j<<20
constexpr uint32_t kOffMark = kOffPqM + 4 * kCapP;           // i32[64]
constexpr uint32_t kOffBins = kOffMark + 4 * 64;             // u64[k] rank bits, u64[k] ids
constexpr uint32_t kQueueBytes = kOffBins;
constexpr uint32_t kTablesBytes = 16 * kTable + 8 * kNumPoisson;  // W, R, Poisson thresholds

// Dart buffer of a bottom-k wave: at least k + 64 entries, so that after a
// compaction (at most k entries kept) a whole round of accepted darts always
// fits.  Up to k = 384 it is k + 128 rounded up to whole 64-entry slots (at most
// 512: always sorted in registers; at k = 256 it holds a first pass's darts
// with room to spare, and 10 waves fit a CU instead of 9 with 512 entries);
// beyond, a power of two of at least 2k entries for the bitonic network over LDS.
__host__ __device__ constexpr uint32_t bk_cap(int k)
{
    if (k <= 384) return (uint32_t)(k + 128 + 63) / 64 * 64;
    uint32_t need = (uint32_t)(2 * k > k + 64 ? 2 * k : k + 64), c = 64;
    while (c < need) c <<= 1;
    return c;
}

// LSH table bookkeeping after the L sorted lists: one count byte per table
// (K <= 64), padded to 8 bytes, then -- only past 64 tables -- the tables'
// ticket counters; up to 64 tables borrow the expansion marks for them, which
// are never live during an accept round.
__host__ __device__ constexpr size_t lsh_aux_bytes(int L)
{
    return (size_t)((L + 7) / 8) * 8 + (L > 64 ? (size_t)4 * L : 0);
}

// Bytes of the result area after the queues: the minima of K buckets (minhash:
// K is the tile of buckets a wave holds at once, k when untiled), L sorted
// lists of K darts plus their bookkeeping (LSH), nothing (register-table LSH:
// the tables are in registers, their mailboxes in the pass queue's slots that
// the accept round has just read), or the dart buffer (bottom-k).
__host__ __device__ constexpr size_t sink_bytes(int mode, int k, int K)
{
    return mode == kModeLshReg ? (size_t)0
         : mode == kModeLsh ? (size_t)16 * k * K + lsh_aux_bytes(k)
         : mode == kModeBottomK ? (size_t)16 * bk_cap(k)
                                : (size_t)16 * K;
}
__host__ __device__ constexpr size_t wave_lds_bytes(int mode, int k, int K)
{
    return kQueueBytes + sink_bytes(mode, k, K);
}

// (L,K) LSH tables of one wave: table l holds cnt[l] <= K darts sorted by
// (rank, id hash); ticket[l] is the table's ticket counter.
struct LshTables {
    uint64_t* rank;
    uint64_t* sval;
    uint8_t* cnt;
    int32_t* ticket;
    // staging of the darts of one ticket: the accept round's consumed
    // pass-queue slots (rank bits, id hash, table), which it no longer reads
    uint64_t* stage_r;
    uint64_t* stage_s;
    uint32_t* stage_l;
    int K;

    // Called by all 64 lanes of an accept round whose pass-queue head is
    // `head`; lanes with `has` insert their dart into table l.  A dart above a
    // full table's largest is dropped at once (later insertions only lower that
    // bound).  The others draw tickets from their table's counter, and the
    // darts holding ticket i (at most one per table) are inserted together by
    // groups of G >= K lanes, one dart per group: lane j of a group holds entry
    // j of the dart's table, the group counts the entries below the dart, and
    // the entries from that position on move up by one.  Tickets are taken in
    // ascending order, so a table is written by one group at a time.  The order
    // of insertions does not change a table's final K smallest darts; a dart
    // equal to an entry (a repeated element id) is dropped.
    __device__ void insert(bool has, uint32_t l, uint64_t rb, uint64_t s, uint32_t head, int lane) const
    {
        bool pending = has;
        if (pending && cnt[l] >= K) {
            const uint64_t mr = rank[(size_t)l * K + K - 1], ms = sval[(size_t)l * K + K - 1];
            pending = rb < mr || (rb == mr && s <= ms);
        }
        if (!wave_any(pending)) return;
        if (pending) __hip_atomic_store(&ticket[l], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        wave_sync();  // also: every lane has read its pass-queue entry
        int mine = 0;
        if (pending)
            mine = __hip_atomic_fetch_add(&ticket[l], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const uint32_t gsh = K <= 1 ? 0u : 32u - (uint32_t)__clz(K - 1);  // G = 2^gsh
        const uint32_t j = (uint32_t)lane & ((1u << gsh) - 1u);
        const uint32_t g = (uint32_t)lane >> gsh;
        const uint32_t groups = 64u >> gsh;
        const uint64_t gmask = gsh == 6 ? ~0ull : (1ull << (1u << gsh)) - 1ull;
        const uint32_t uK = (uint32_t)K;
        for (int level = 0; wave_any(pending); ++level) {
            const bool here = pending && mine == level;
            const uint64_t b = __ballot(here);
            const uint32_t n = (uint32_t)__popcll(b);
            if (here) {
                const uint32_t q = ring_p(head + rank_in(b));
                stage_r[q] = rb;
                stage_s[q] = s;
                stage_l[q] = l;
                pending = false;
            }
            wave_sync();
            for (uint32_t base = 0; base < n; base += groups) {
                const uint32_t q = base + g;
                const bool act = q < n;
                uint32_t tl = 0;
                uint64_t dr = 0, dsv = 0;
                if (act) {
                    const uint32_t p = ring_p(head + q);
                    tl = stage_l[p];
                    dr = stage_r[p];
                    dsv = stage_s[p];
                }
                const uint32_t c = act ? (uint32_t)cnt[tl] : 0u;
                const bool in = j < c;
                uint64_t R = 0, V = 0;
                if (in) {
                    R = rank[(size_t)tl * K + j];
                    V = sval[(size_t)tl * K + j];
                }
                const uint64_t bl = __ballot(in && (R < dr || (R == dr && V < dsv)));
                const uint64_t bd = __ballot(in && R == dr && V == dsv);
                const uint32_t pos = (uint32_t)__popcll((bl >> (g << gsh)) & gmask);
                const bool dup = ((bd >> (g << gsh)) & gmask) != 0;
                // entry j - 1 of the same group (lane - 1); used only when j > pos >= 0
                const uint64_t Rp = __shfl(R, lane - 1, kWave), Vp = __shfl(V, lane - 1, kWave);
                const bool put = act && !dup && pos < uK;
                if (put && j < uK && j >= pos && j <= c) {
                    rank[(size_t)tl * K + j] = j == pos ? dr : Rp;
                    sval[(size_t)tl * K + j] = j == pos ? dsv : Vp;
                }
                if (put && j == 0 && c < uK) cnt[tl] = (uint8_t)(c + 1);
            }
            wave_sync();  // the next ticket may use the same tables and staging slots
        }
    }
};

template <class T>
__device__ __forceinline__ T& at(unsigned char* base, uint32_t off, uint32_t i)
{
    return reinterpret_cast<T*>(base + off)[i];
}

}  // namespace

// Persistent flattened DartHash with one of three sinks: DartMinHash (k
// buckets keep their minimum), (L,K) LSH (k = L tables keep their K smallest
// darts) or the bottom-k sketch (a buffer of darts, sorted and cut to the k
// smallest).  Each wave repeatedly takes the next set index from *next_set.
template <int MODE, int HK, bool DBG>
__global__ void __launch_bounds__(256)
fast_kernel(const SpecTables* __restrict__ sp, int64_t n_sets, const int64_t* __restrict__ rp,
            const int32_t* __restrict__ idx, const double* __restrict__ wts, int k, int K,
            uint32_t* out_u32, uint64_t* out_bits, int8_t* out_status, uint64_t* out_s,
            double* out_rank, uint64_t* out_keys, double phi0, double phi_max,
            unsigned long long* next_set, const Part* __restrict__ parts, int64_t n_parts,
            HeavySet* heavy, uint64_t* partial, int64_t split, const uint32_t* __restrict__ order,
            int64_t* out_cnt, const uint8_t* __restrict__ repeated, const unsigned long long* plan_dev,
            const uint8_t* __restrict__ planned)
{
    constexpr bool RT = MODE == kModeLshReg;  // K = 8 tables in registers, one per lane
    constexpr bool LSH = MODE == kModeLsh || RT;
    constexpr bool BK = MODE == kModeBottomK;
    // Region and area rounds only need to know whether an area holds no dart,
    // one, or more (poisson_head); the dart round, which sees only areas with
    // two or more, tests one further threshold per dart: X > j + 1 iff the
    // area hash is at least threshold j + 1, so the count itself is never formed.
    extern __shared__ unsigned char smem[];
    double* sW = (double*)smem;
    double* sR = sW + kTable;
    uint64_t* sPois = (uint64_t*)(sR + kTable);
    for (int i = threadIdx.x; i < kTable; i += blockDim.x) {
        sW[i] = sp->W[i];
        sR[i] = sp->R[i];
    }
    if (threadIdx.x < kNumPoisson) sPois[threadIdx.x] = sp->pois[threadIdx.x];
    __syncthreads();  // the only block barrier
    // per-lane copies of the first two thresholds keep scalar registers free
    const uint64_t C0 = sPois[0], C1 = sPois[1];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    unsigned char* wb = smem + kTablesBytes + (uint32_t)wave * (uint32_t)wave_lds_bytes(MODE, k, K);
    uint64_t* const bin_rank = reinterpret_cast<uint64_t*>(wb + kOffBins);
    // minhash: the wave holds the minima of buckets [tile_lo, tile_lo + K) at a
    // time (K = k unless the buckets do not fit next to the queues)
    uint64_t* const bin_s = bin_rank + (LSH ? k * K : BK ? (int)bk_cap(k) : K);
    uint32_t tile_lo = 0;                       // first bucket of the current tile
    uint32_t tile_n = MODE == kModeMinhash ? (uint32_t)K : (uint32_t)k;  // its buckets
    LshTables T;
    T.rank = bin_rank;
    T.sval = bin_s;
    T.cnt = reinterpret_cast<uint8_t*>(bin_s + k * K);
    T.ticket = k <= kWave ? &at<int32_t>(wb, kOffMark, 0)
                         : reinterpret_cast<int32_t*>(T.cnt + ((k + 7) / 8) * 8);
    T.stage_r = &at<uint64_t>(wb, kOffPqRank, 0);
    T.stage_s = &at<uint64_t>(wb, kOffPqA, 0);
    T.stage_l = &at<uint32_t>(wb, kOffPqE, 0);
    T.K = K;
    // Register tables: lane l holds table l (l < L), its darts sorted by (rank
    // bits, id hash) in tr/ts; unused entries hold rank bits ~0, above every
    // rank (ranks are finite), so the table is full once tr[7] != ~0.  A dart
    // reaches its table's lane through the table's mailbox: during an accept
    // round, the pass-queue slot pq_head + l, whose entry the round has read,
    // holds table l's rank bits, id hash and a flag (1 while it holds a dart).
    constexpr uint64_t kNoRank = ~0ull;
    uint64_t tr[8], ts[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        tr[m] = kNoRank;
        ts[m] = 0;
    }
    // Inserts (r, v) into this lane's sorted table unless it is already there.
    // Entries ordering below the dart form a prefix, so from the top down each
    // entry is kept, replaced by the dart, or replaced by the entry below it,
    // by selects without branches (two comparisons live at a time).  The
    // order is taken on the rank bits alone; only a lane whose rank equals an
    // entry's takes the path that also compares id hashes (and may find the
    // same dart, which then changes nothing).
    auto reg_insert = [&](uint64_t r, uint64_t v) {
        bool tie = false;
#pragma unroll
        for (int m = 0; m < 8; ++m) tie |= tr[m] == r;
        if (!tie) {
            bool below = tr[7] < r;
#pragma unroll
            for (int m = 7; m >= 1; --m) {
                const bool below_prev = tr[m - 1] < r;
                tr[m] = below ? tr[m] : (below_prev ? r : tr[m - 1]);
                ts[m] = below ? ts[m] : (below_prev ? v : ts[m - 1]);
                below = below_prev;
            }
            tr[0] = below ? tr[0] : r;
            ts[0] = below ? ts[0] : v;
        } else {
            uint32_t pos = 0;
            bool dup = false;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                dup |= tr[m] == r && ts[m] == v;
                pos += (tr[m] < r || (tr[m] == r && ts[m] < v)) ? 1u : 0u;
            }
            if (!dup && pos < 8) {
#pragma unroll
                for (int m = 7; m >= 1; --m) {
                    if ((uint32_t)m > pos) {
                        tr[m] = tr[m - 1];
                        ts[m] = ts[m - 1];
                    }
                }
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    if ((uint32_t)m == pos) {
                        tr[m] = r;
                        ts[m] = v;
                    }
                }
            }
        }
    };

    const uint64_t KR = sp->key_r, KA = sp->key_a, KU = sp->key_u, KV = sp->key_v, KS = sp->key_s;
    const Hasher<HK> H(sp);
    // Hash of z for the lanes that use it (`live`).  The mixer runs on every
    // lane without a branch (masked-out lanes cost no extra instructions);
    // table lookups are issued only by the lanes that need them.
    auto HL = [&](bool live, uint64_t z) -> uint64_t {
        if (HK == kHashMix) return H(z);
        uint64_t h = 0;
        if (live) h = H(z);
        return h;
    };
    const double u = sp->u;
    const double td = (double)sp->t;

    // Bottom-k buffer: bk_count darts (rank bits, id hash) in bin_rank/bin_s,
    // and a cutoff: darts at or above it are never needed (k smaller ones are
    // held) and are not stored.
    uint32_t bk_count = 0;
    uint64_t cut_r = ~0ull, cut_s = ~0ull;
    // Sort the buffer by (rank, id hash), drop repeated darts and keep at most
    // the k smallest (the k-th becomes the cutoff).  All 64 lanes call it.
    // Up to 512 darts are sorted in registers (below); fuller buffers (only at
    // k > 384, where the buffer is a power of two that the padded network
    // stays within) by a bitonic network over LDS.
    auto bk_compact_lds = [&]() __attribute__((always_inline)) {
        const uint32_t n = bk_count;
        uint32_t N = 64;
        while (N < n) N <<= 1;
        for (uint32_t p = n + lane; p < N; p += kWave) {
            bin_rank[p] = ~0ull;
            bin_s[p] = ~0ull;
        }
        wave_sync();
        // bitonic sorting network over N entries, ascending
        for (uint32_t size = 2; size <= N; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (uint32_t i = lane; i < N / 2; i += kWave) {
                    const uint32_t lo = 2 * i - (i & (stride - 1));
                    const uint32_t hi = lo + stride;
                    const uint64_t r0 = bin_rank[lo], s0 = bin_s[lo];
                    const uint64_t r1 = bin_rank[hi], s1 = bin_s[hi];
                    const bool gt = r0 > r1 || (r0 == r1 && s0 > s1);
                    const bool lt = r0 < r1 || (r0 == r1 && s0 < s1);
                    if ((lo & size) == 0 ? gt : lt) {
                        bin_rank[lo] = r1;
                        bin_s[lo] = s1;
                        bin_rank[hi] = r0;
                        bin_s[hi] = s0;
                    }
                }
                wave_sync();
            }
        }
        // in-place removal of repeats, 64 entries at a time; an entry moves
        // only towards the front, to a slot whose entry is already read
        uint32_t D = 0;
        uint64_t prev_r = 0, prev_s = 0;
        for (uint32_t base = 0; base < n; base += kWave) {
            const uint32_t p = base + lane;
            uint64_t r = ~0ull, sv = ~0ull;
            bool keep = false;
            if (p < n) {
                r = bin_rank[p];
                sv = bin_s[p];
                const uint64_t pr = lane == 0 ? prev_r : bin_rank[p - 1];
                const uint64_t ps = lane == 0 ? prev_s : bin_s[p - 1];
                keep = p == 0 || r != pr || sv != ps;
            }
            const int last = (int)((n - base < (uint32_t)kWave ? n - base : (uint32_t)kWave) - 1);
            prev_r = __shfl(r, last, kWave);
            prev_s = __shfl(sv, last, kWave);
            const uint64_t bm = __ballot(keep);
            wave_sync();
            if (keep) {
                const uint32_t q = D + rank_in(bm);
                bin_rank[q] = r;
                bin_s[q] = sv;
            }
            D = uni(D + (uint32_t)__popcll(bm));
            wave_sync();
        }
        if (D > (uint32_t)k) {
            D = (uint32_t)k;
            cut_r = bin_rank[k - 1];
            cut_s = bin_s[k - 1];
        }
        bk_count = D;
        wave_sync();
    };
    // The same for n <= 64 NR darts held in registers: element e = 64 i + lane
    // sits in slot i of its lane, entries past n are empty (all ones).  The
    // bitonic network is the form without directions: each merge of two
    // sorted runs of size/2 first compares e with its mirror e ^ (size - 1),
    // then halves with every pair in ascending order, so an empty entry never
    // moves and a step whose upper element lies in a slot past n is skipped.
    // Exchanges between lanes go through lane permutes, those between slots
    // stay in the lane: no LDS round trip per step.  The repeats are then
    // dropped on the sorted registers and the distinct darts written to the
    // front of the buffer.
    auto bk_compact_reg = [&](auto slots) __attribute__((always_inline)) {
        constexpr int NR = decltype(slots)::value;
        const uint32_t n = bk_count;
        uint64_t R[NR], V[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const uint32_t e = 64u * i + (uint32_t)lane;
            R[i] = ~0ull;
            V[i] = ~0ull;
            if (e < n) {
                R[i] = bin_rank[e];
                V[i] = bin_s[e];
            }
        }
        // The network orders by the rank bits alone (FULL = false) or by (rank,
        // id hash).  Distinct darts of equal rank are rare: the rank order is
        // taken when no two neighbours share a rank, else the network runs
        // again on the full order (repeated darts always take that path).
        auto sort_slots = [&](auto fullc) __attribute__((always_inline)) {
            constexpr bool FULL = decltype(fullc)::value;
            auto less = [&](uint64_t ar, uint64_t av, uint64_t br, uint64_t bv) {
                return FULL ? ar < br || (ar == br && av < bv) : ar < br;
            };
            // one step between lanes of each occupied slot: partner lane ^ mask;
            // the lane for which `lower` holds keeps the smaller entry
            auto lane_step = [&](int mask, bool lower) __attribute__((always_inline)) {
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    if (64u * i >= n) continue;
                    const uint64_t pr = __shfl_xor(R[i], mask, kWave);
                    const uint64_t pv = __shfl_xor(V[i], mask, kWave);
                    const bool own_less = less(R[i], V[i], pr, pv);
                    const bool take = lower ? !own_less : own_less;
                    R[i] = take ? pr : R[i];
                    V[i] = take ? pv : V[i];
                }
            };
            // one step between slots i (lower) and i ^ MS of the same lane (flip =
            // false, MS a power of two) or of lane ^ 63 (the mirror step of a merge
            // of size > 64)
            auto slot_step = [&](auto msc, auto flipc) __attribute__((always_inline)) {
                constexpr int MS = decltype(msc)::value;
                constexpr bool flip = decltype(flipc)::value;
                constexpr int HB = flip ? (MS + 1) >> 1 : MS;  // the slot bit that tells lower from upper
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    const int j = i ^ MS;
                    if ((i & HB) != 0 || j >= NR) continue;
                    if (64u * j >= n) continue;  // the upper slot is empty
                    uint64_t ar = R[j], av = V[j], br = R[i], bv = V[i];
                    if constexpr (flip) {
                        ar = __shfl_xor(ar, 63, kWave);
                        av = __shfl_xor(av, 63, kWave);
                        br = __shfl_xor(br, 63, kWave);
                        bv = __shfl_xor(bv, 63, kWave);
                    }
                    const bool i_less = less(R[i], V[i], ar, av);
                    const bool j_less = less(R[j], V[j], br, bv);
                    R[i] = i_less ? R[i] : ar;
                    V[i] = i_less ? V[i] : av;
                    R[j] = j_less ? br : R[j];
                    V[j] = j_less ? bv : V[j];
                }
            };
            for (uint32_t size = 2; size <= 64u * NR; size <<= 1) {
                if (size <= 64u) lane_step((int)size - 1, ((uint32_t)lane & (size >> 1)) == 0);
                else if (size == 128u) slot_step(std::integral_constant<int, 1>{}, std::true_type{});
                else if (size == 256u) slot_step(std::integral_constant<int, 3>{}, std::true_type{});
                else slot_step(std::integral_constant<int, 7>{}, std::true_type{});
                for (uint32_t stride = size >> 2; stride > 0; stride >>= 1) {
                    if (stride < 64u) lane_step((int)stride, ((uint32_t)lane & stride) == 0);
                    else if (stride == 64u) slot_step(std::integral_constant<int, 1>{}, std::false_type{});
                    else if (stride == 128u) slot_step(std::integral_constant<int, 2>{}, std::false_type{});
                    else slot_step(std::integral_constant<int, 4>{}, std::false_type{});
                }
            }
        };
        sort_slots(std::false_type{});
        bool tie = false;  // some entry has its predecessor's rank
        {
            uint64_t last = ~0ull;  // rank of element 64 i - 1
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                if (64u * i >= n) continue;
                const uint32_t e = 64u * i + (uint32_t)lane;
                uint64_t pr = __shfl(R[i], lane == 0 ? 0 : lane - 1, kWave);
                if (lane == 0) pr = last;
                tie = tie || (e < n && e > 0 && R[i] == pr);
                last = uni64(__shfl(R[i], 63, kWave));
            }
        }
        if (wave_any(tie)) sort_slots(std::true_type{});
        wave_sync();  // every entry is read before the front is rewritten
        uint32_t D = 0;
        uint64_t last_r = 0, last_v = 0;  // element 64 i - 1 (lane 63 of slot i - 1)
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (64u * i >= n) continue;  // empty slots come last
            const uint32_t e = 64u * i + (uint32_t)lane;
            const int from = lane == 0 ? 0 : lane - 1;
            uint64_t pr = __shfl(R[i], from, kWave), pv = __shfl(V[i], from, kWave);
            if (lane == 0) {
                pr = last_r;
                pv = last_v;
            }
            const bool keep = e < n && (e == 0 || R[i] != pr || V[i] != pv);
            const uint64_t bm = __ballot(keep);
            if (keep) {
                const uint32_t q = D + rank_in(bm);
                bin_rank[q] = R[i];
                bin_s[q] = V[i];
            }
            D = uni(D + (uint32_t)__popcll(bm));
            last_r = uni64(__shfl(R[i], 63, kWave));
            last_v = uni64(__shfl(V[i], 63, kWave));
        }
        wave_sync();
        if (D > (uint32_t)k) {
            D = (uint32_t)k;
            cut_r = bin_rank[k - 1];
            cut_s = bin_s[k - 1];
        }
        bk_count = D;
        wave_sync();
    };
    auto bk_compact = [&]() __attribute__((always_inline)) {
        if (bk_count <= 64u) bk_compact_reg(std::integral_constant<int, 1>{});
        else if (bk_count <= 128u) bk_compact_reg(std::integral_constant<int, 2>{});
        else if (bk_count <= 256u) bk_compact_reg(std::integral_constant<int, 4>{});
        else if (bk_count <= 512u) bk_compact_reg(std::integral_constant<int, 8>{});
        else bk_compact_lds();
    };

    // Enumeration counts of the current set or part (wave-uniform): regions,
    // areas, darts generated, darts with rank in (tau_prev, tau], those of them
    // accepted, and phi passes run; phi_end is the last pass's phi.
    uint64_t n_reg = 0, n_area = 0, n_gen = 0, n_rank = 0, n_acc = 0, n_pass = 0;
    double phi_end = 0.0;

    // Runs phi passes over the elements [lo, hi) of a row with ||x||_1 = S,
    // starting at phi (darts of rank <= tau_prev are already in the buckets),
    // until no bucket is empty -- or just one pass when `single`.  Returns the
    // set's status (kSetOk or kSetRange).
    auto run = [&](int64_t lo, int64_t hi, double S, double phi, double tau_prev, bool single) -> int8_t {
        int8_t status = kSetOk;
            for (;;) {
                if (phi > phi_max) { status = kSetRange; break; }
                const double tau = phi / S;
                if (DBG) {
                    n_pass += 1;
                    phi_end = phi;
                }
                // rho runs over 0 .. B1-1: the rows whose lower corner is <= tau
                int B1 = 0;
                while (B1 < kMaxIndex && r_corner(sR, B1) <= tau) ++B1;
                bool range = B1 >= kMaxIndex;
                const float inv_b1 = 1.0f / (float)B1;
                // With tau < 1 every region lies in rank row 0 and has one column;
                // region nu has floor(tau 2^nu) + 1 rows (at most 2^nu), so the
                // regions below nu_split (tau 2^nu < 1, i.e. nu < -ilogb(tau)) are a
                // single area each: the "low band", walked by lockstep rounds over
                // nu with one element per lane and no expansion.
                const int nu_split = B1 == 1 ? max(0, -ilogb(tau)) : 0;

                const int64_t b1 = hi;
                int64_t chunk = lo;        // first element of the current chunk
                uint32_t chunk_total = 0;  // regions of the chunk
                uint32_t reg_done = 0;     // regions of the chunk already expanded
                double ex = 0.0;           // this lane's element weight
                uint32_t eid = 0;          // this lane's element id
                uint32_t nreg = 0, nreg_excl = 0;
                uint32_t n_low = 0;     // this lane's element: low-band regions
                uint32_t low_nu = 0;    // next low-band nu of the chunk (wave-uniform)
                bool low_left = false;  // some lane still has low-band regions
                bool have_chunk = false;
                uint32_t rq_head = 0, rq_count = 0, dq_head = 0, dq_count = 0;
                uint32_t pq_head = 0, pq_count = 0;

                auto load_chunk = [&]() {
                    have_chunk = false;
                    while (!have_chunk && chunk < b1) {
                        const int64_t e = chunk + lane;
                        ex = 0.0;
                        eid = 0;
                        nreg = 0;
                        n_low = 0;
                        if (e < b1) {
                            ex = wts[e];
                            eid = (uint32_t)idx[e];
                        }
                        if (ex > 0.0) {
                            // weight rows: nu with W[nu] <= x (W[0] = 0)
                            int A = ilogb(1.0 + td * ex) + 1;
                            A = A < 1 ? 1 : (A > kMaxIndex ? kMaxIndex : A);
                            while (A < kMaxIndex && w_corner(sW, u, A) <= ex) ++A;
                            while (A > 1 && w_corner(sW, u, A - 1) > ex) --A;
                            if (A >= kMaxIndex) range = true;
                            n_low = (uint32_t)min(A, nu_split);
                            nreg = (uint32_t)A;
                        }
                        if (nu_split > 0) {
                            // lockstep rounds pay for 64 lanes each: they serve the
                            // chunk only while they stay at least 3/4 full; otherwise
                            // its regions are all expanded
                            const uint32_t low_sum = uni(lane63(scan_add(n_low)));
                            const uint32_t low_max = uni(lane63((uint32_t)scan_max((int32_t)n_low)));
                            if (4 * low_sum < 3 * 64 * low_max) n_low = 0;
                        }
                        nreg = (nreg - n_low) * (uint32_t)B1;
                        const uint32_t incl = scan_add(nreg);
                        nreg_excl = incl - nreg;
                        chunk_total = uni(lane63(incl));
                        reg_done = 0;
                        low_nu = 0;
                        low_left = wave_any(n_low > 0);
                        have_chunk = chunk_total > 0 || low_left;
                        if (!have_chunk) chunk += kWave;
                    }
                };
                load_chunk();

                // An area that holds X > 0 darts: the rank uniform of its first dart
                // is drawn at once; a dart inside (tau_prev, tau] enters the pass
                // queue, and an area with more darts enters the dart queue at j = 1.
                // Called by all 64 lanes; the `act` lanes carry an area.  Region
                // and area rounds run only while both queues hold fewer than 64
                // entries, so neither can overflow.
                // `corner` marks a region's first area in rank row 0 (rho = 0,
                // r = 0): its rank R[0] + (0 + U) 2^-nu is U 2^-nu exactly (R[0] = 0,
                // and scaling by a power of two is exact while ranks stay normal,
                // as they do for every weight in the supported domain).
                struct FirstDart {
                    double rank;
                    bool has, pass, more;
                };
                auto first_dart = [&](bool act, uint64_t a, uint32_t rv, uint32_t meta, uint32_t X,
                                      bool corner) -> FirstDart {
                    // lanes without a dart are masked out of both tests by `has`
                    FirstDart f;
                    f.has = act && X > 0;
                    const int nu = meta & 1023, rho = (meta >> 10) & 1023;
                    const uint64_t hu = HL(f.has, a ^ KU);
                    if (corner) {
                        // U 2^-nu = (hu >> 11) 2^(-53-nu): one exact scaling
                        f.rank = ldexp((double)(hu >> 11), -53 - nu);
                    } else {
                        f.rank = r_corner(sR, rho) + ((double)rv + unit53(hu)) * ldexp(1.0, rho - nu);
                    }
                    f.pass = f.has && f.rank <= tau && f.rank > tau_prev;
                    f.more = f.has && X > 1;
                    return f;
                };
                auto push_area = [&](const FirstDart& f, uint64_t a, uint32_t ei, uint32_t rv, uint32_t wv,
                                     uint32_t meta) {
                    const uint64_t bp = __ballot(f.pass);
                    const uint64_t bm = __ballot(f.more);
                    if (DBG) {
                        n_gen += (uint64_t)__popcll(__ballot(f.has));
                        n_rank += (uint64_t)__popcll(bp);
                    }
                    if (f.pass) {
                        const uint32_t pos = ring_p(pq_head + pq_count + rank_in(bp));
                        at<uint64_t>(wb, kOffPqA, pos) = a;
                        at<uint32_t>(wb, kOffPqE, pos) = ei;
                        at<uint64_t>(wb, kOffPqRank, pos) = (uint64_t)__double_as_longlong(f.rank);
                        at<uint32_t>(wb, kOffPqW, pos) = wv;
                        at<uint32_t>(wb, kOffPqM, pos) = meta;
                    }
                    if (f.more) {
                        const uint32_t pos = ring_d(dq_head + dq_count + rank_in(bm));
                        at<uint64_t>(wb, kOffDqA, pos) = a;
                        at<uint32_t>(wb, kOffDqE, pos) = ei;
                        at<uint32_t>(wb, kOffDqR, pos) = rv;
                        at<uint32_t>(wb, kOffDqW, pos) = wv;
                        at<uint32_t>(wb, kOffDqM, pos) = meta | (1u << 20);
                    }
                    pq_count = uni(pq_count + (uint32_t)__popcll(bp));
                    dq_count = uni(dq_count + (uint32_t)__popcll(bm));
                };
                auto emit_area = [&](bool act, uint64_t a, uint32_t ei, uint32_t rv, uint32_t wv,
                                     uint32_t meta, uint32_t X, bool corner) {
                    push_area(first_dart(act, a, rv, meta, X, corner), a, ei, rv, wv, meta);
                };

                for (;;) {
                    wave_sync();
                    if (pq_count > kTrigP || (pq_count > 0 && dq_count == 0 && rq_count == 0 && !have_chunk)) {
                        // ---------------- accept round ----------------
                        const uint32_t m = pq_count < 64 ? pq_count : 64;
                        // lanes past m reread the last entry and stay inactive
                        const uint32_t pos = ring_p(pq_head + ((uint32_t)lane < m ? (uint32_t)lane : m - 1));
                        const uint64_t a = at<uint64_t>(wb, kOffPqA, pos);
                        const double xi = wts[lo + at<uint32_t>(wb, kOffPqE, pos)];
                        const uint32_t wv = at<uint32_t>(wb, kOffPqW, pos);
                        const uint32_t meta = at<uint32_t>(wb, kOffPqM, pos);
                        const uint64_t rb = at<uint64_t>(wb, kOffPqRank, pos);
                        const int nu = meta & 1023, rho = (meta >> 10) & 1023;
                        const uint64_t j = (meta >> 20) & 31;
                        // the id hash does not depend on the weight test: with the mixer
                        // it is drawn first, so both hash chains cover the wait for x_i
                        uint64_t s = HK == kHashMix ? H(a ^ KS ^ j) : 0ull;  // used only where acc
                        const double V = unit53(H(a ^ KV ^ j));
                        const double weight = w_corner(sW, u, nu) + ((double)wv + V) * ldexp(u, nu - rho);
                        const bool acc = (uint32_t)lane < m && weight <= xi;
                        if (DBG) n_acc += (uint64_t)__popcll(__ballot(acc));
                        if (HK != kHashMix) s = HL(acc, a ^ KS ^ j);
                        if (RT) {
                            // a dart ranked above its full table's largest is dropped at
                            // once (one of equal rank goes on: the insertion compares id
                            // hashes); the others go to their table's lane through its
                            // mailbox, one dart per table at a time (tickets in ascending order)
                            const uint32_t l = bucket_of(s, (uint32_t)k);
                            const int src = acc ? (int)l : lane;
                            const uint64_t omr = __shfl(tr[7], src, kWave);
                            bool pending = acc && rb <= omr;
                            if (wave_any(pending)) {
                                int32_t* const ticket = &at<int32_t>(wb, kOffMark, 0);
                                if (pending)
                                    __hip_atomic_store(&ticket[l], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                                // the mailboxes: the 64 slots from pq_head, all read above
                                // (a round of m < 64 darts takes the whole queue)
                                const uint32_t mb_in = ring_p(pq_head + (uint32_t)lane);
                                const uint32_t mb_out = ring_p(pq_head + l);
                                at<uint32_t>(wb, kOffPqM, mb_in) = 0;
                                wave_sync();
                                int mine = 0;
                                if (pending)
                                    mine = __hip_atomic_fetch_add(&ticket[l], 1, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
                                for (int level = 0; wave_any(pending); ++level) {
                                    if (pending && mine == level) {
                                        at<uint64_t>(wb, kOffPqA, mb_out) = rb;
                                        at<uint64_t>(wb, kOffPqRank, mb_out) = s;
                                        at<uint32_t>(wb, kOffPqM, mb_out) = 1;
                                        pending = false;
                                    }
                                    wave_sync();
                                    // flag and dart are read together (one LDS round trip)
                                    const uint32_t got = at<uint32_t>(wb, kOffPqM, mb_in);
                                    const uint64_t r2 = at<uint64_t>(wb, kOffPqA, mb_in);
                                    const uint64_t v2 = at<uint64_t>(wb, kOffPqRank, mb_in);
                                    if (got) {
                                        at<uint32_t>(wb, kOffPqM, mb_in) = 0;
                                        reg_insert(r2, v2);
                                    }
                                    wave_sync();
                                }
                            }
                        } else if (LSH) {
                            T.insert(acc, bucket_of(s, (uint32_t)k), rb, s, pq_head, lane);
                        } else if (BK) {
                            bool keep = acc && (rb < cut_r || (rb == cut_r && s < cut_s));
                            uint64_t bk = __ballot(keep);
                            if (bk_count + (uint32_t)__popcll(bk) > bk_cap(k)) {
                                bk_compact();  // at most k stay, so the round fits afterwards
                                keep = keep && (rb < cut_r || (rb == cut_r && s < cut_s));
                                bk = __ballot(keep);
                            }
                            if (keep) {
                                const uint32_t q = bk_count + rank_in(bk);
                                bin_rank[q] = rb;
                                bin_s[q] = s;
                            }
                            bk_count = uni(bk_count + (uint32_t)__popcll(bk));
                        } else {
                            const uint32_t b = bucket_of(s, (uint32_t)k) - tile_lo;
                            if (acc && b < tile_n) bucket_min(bin_rank, bin_s, b, rb, s);
                        }
                        pq_head = uni(ring_p(pq_head + m));
                        pq_count = uni(pq_count - m);
                    } else if (dq_count > kTrigD || (dq_count > 0 && rq_count == 0 && !have_chunk)) {
                        // ---------------- dart round ----------------
                        const uint32_t m = dq_count < 64 ? dq_count : 64;
                        const bool act = (uint32_t)lane < m;
                        const uint32_t rpos = ring_d(dq_head + (act ? (uint32_t)lane : m - 1));
                        const uint64_t a = at<uint64_t>(wb, kOffDqA, rpos);
                        const uint32_t ei = at<uint32_t>(wb, kOffDqE, rpos);
                        const uint32_t rv = at<uint32_t>(wb, kOffDqR, rpos);
                        const uint32_t wv = at<uint32_t>(wb, kOffDqW, rpos);
                        const uint32_t meta = at<uint32_t>(wb, kOffDqM, rpos);
                        const int nu = meta & 1023, rho = (meta >> 10) & 1023;
                        const uint32_t j = (meta >> 20) & 31;
                        const double U = unit53(H(a ^ KU ^ (uint64_t)j));
                        const double rank = r_corner(sR, rho) + ((double)rv + U) * ldexp(1.0, rho - nu);
                        const bool pass = act && rank <= tau && rank > tau_prev;
                        // dart j + 1 exists iff X > j + 1, i.e. the area hash reaches
                        // threshold j + 1 (X counts the thresholds at or below it)
                        const bool more = act && j + 1 < (uint32_t)kNumPoisson && a >= sPois[j + 1];
                        const uint64_t bp = __ballot(pass);
                        const uint64_t bm = __ballot(more);
                        if (DBG) {
                            n_gen += m;
                            n_rank += (uint64_t)__popcll(bp);
                        }
                        wave_sync();  // every entry of the round is read before any write
                        if (pass) {
                            const uint32_t pos = ring_p(pq_head + pq_count + rank_in(bp));
                            at<uint64_t>(wb, kOffPqA, pos) = a;
                            at<uint32_t>(wb, kOffPqE, pos) = ei;
                            at<uint64_t>(wb, kOffPqRank, pos) = (uint64_t)__double_as_longlong(rank);
                            at<uint32_t>(wb, kOffPqW, pos) = wv;
                            at<uint32_t>(wb, kOffPqM, pos) = meta;
                        }
                        const uint32_t dq_left = dq_count - m;
                        if (more) {
                            const uint32_t pos = ring_d(dq_head + m + dq_left + rank_in(bm));
                            at<uint64_t>(wb, kOffDqA, pos) = a;
                            at<uint32_t>(wb, kOffDqE, pos) = ei;
                            at<uint32_t>(wb, kOffDqR, pos) = rv;
                            at<uint32_t>(wb, kOffDqW, pos) = wv;
                            at<uint32_t>(wb, kOffDqM, pos) = meta + (1u << 20);
                        }
                        pq_count = uni(pq_count + (uint32_t)__popcll(bp));
                        dq_head = uni(ring_d(dq_head + m));
                        dq_count = uni(dq_left + (uint32_t)__popcll(bm));
                    } else if (rq_count > kTrigR || (rq_count > 0 && !have_chunk)) {
                        // ---------------- area round ----------------
                        // the queue's next areas, up to 64 per half: two halves (two
                        // independent hash chains per lane) while more than 64 areas wait.
                        // The second half is kept only while both queues still have room
                        // for its darts; otherwise its areas are made again next round.
                        const uint32_t n_items = rq_count < 64 ? rq_count : 64;
                        uint32_t na = 0, first = 0, c = 0;
                        if ((uint32_t)lane < n_items) {
                            const uint32_t ip = ring_r1(rq_head + lane);
                            na = at<uint32_t>(wb, kOffRqNa, ip);
                            first = at<uint32_t>(wb, kOffRqFirst, ip);
                            c = na - first;
                        }
                        const uint32_t cc = c < 128 ? c : 128;
                        const uint32_t incl = scan_add(cc);
                        const uint32_t excl = incl - cc;
                        const uint32_t total = uni(lane63(incl));
                        if (total == 0) {  // bookkeeping guard: never spin without progress
                            range = true;
                            break;
                        }
                        auto area_halves = [&](auto halves) {
                            constexpr int NH = decltype(halves)::value;
                            const uint32_t m = total < 64u * NH ? total : 64u * NH;
                            int32_t src[NH];
                            uint32_t local[NH];
                            int32_t carry = 0;  // entry holding the first area of the half
#pragma unroll
                            for (int h = 0; h < NH; ++h) {
                                // entry of each area: the last entry whose areas start at or
                                // before it (marks at the starts, then a prefix maximum)
                                at<int32_t>(wb, kOffMark, lane) = 0;
                                wave_sync();
                                if (cc > 0 && excl >= 64u * h && excl < 64u * (h + 1))
                                    at<int32_t>(wb, kOffMark, excl - 64u * h) = lane;
                                wave_sync();
                                int32_t v = at<int32_t>(wb, kOffMark, lane);
                                if (lane == 0) v = max(v, carry);
                                src[h] = scan_max(v);
                                carry = __builtin_amdgcn_readlane(src[h], 63);
                                const uint32_t s_excl = (uint32_t)__shfl(excl, src[h], kWave);
                                const uint32_t s_first = (uint32_t)__shfl(first, src[h], kWave);
                                local[h] = s_first + (64u * h + (uint32_t)lane) - s_excl;
                            }
                            bool actv[NH];
                            uint32_t eiv[NH], metav[NH], wvv[NH], rvv[NH];
                            uint64_t av[NH];
                            FirstDart fv[NH];
#pragma unroll
                            for (int h = 0; h < NH; ++h) {
                                actv[h] = 64u * h + (uint32_t)lane < m;
                                // every lane reads an entry of the queue's first 64 (src < 64);
                                // lanes past m are masked out by `act`
                                const uint32_t ip = ring_r1(rq_head + (uint32_t)src[h]);
                                const uint64_t g = at<uint64_t>(wb, kOffRqG, ip);
                                eiv[h] = at<uint32_t>(wb, kOffRqE, ip);
                                metav[h] = at<uint32_t>(wb, kOffRqM, ip);
                                wvv[h] = 0;
                                rvv[h] = local[h];  // tau < 1: one column, area = row
                                if (B1 > 1) {
                                    const uint32_t rc = at<uint32_t>(wb, kOffRqRc, ip);
                                    const uint32_t nas = (uint32_t)__shfl(na, src[h], kWave);
                                    if (actv[h] && rc != nas) {
                                        wvv[h] = rc == 1 ? local[h] : local[h] / rc;
                                        rvv[h] = local[h] - wvv[h] * rc;
                                    }
                                }
                                av[h] = HL(actv[h], g ^ KA ^ (((uint64_t)wvv[h] << 32) | rvv[h]));
                            }
#pragma unroll
                            for (int h = 0; h < NH; ++h)
                                fv[h] = first_dart(actv[h], av[h], rvv[h], metav[h], poisson_head(C0, C1, av[h]), false);
                            uint32_t done = 0;  // areas made this round
                            bool go = true;
#pragma unroll
                            for (int h = 0; h < NH; ++h) {
                                if (h > 0) {
                                    const uint32_t np = (uint32_t)__popcll(__ballot(fv[h].pass));
                                    const uint32_t nm = (uint32_t)__popcll(__ballot(fv[h].more));
                                    go = go && pq_count + np <= kCapP && dq_count + nm <= kCapD;
                                }
                                if (go) {
                                    push_area(fv[h], av[h], eiv[h], rvv[h], wvv[h], metav[h]);
                                    done = m < 64u * (h + 1) ? m : 64u * (h + 1);
                                }
                            }
                            if (DBG) n_area += done;
                            // advance the region queue by `done` areas
                            const int pl = (int)((done - 1) & 63u);  // last area: lane pl of half hl
                            const uint32_t hl = (done - 1) >> 6;
                            int32_t s_last = __builtin_amdgcn_readlane(src[0], pl);
                            uint32_t l_last = (uint32_t)__builtin_amdgcn_readlane((int)local[0], pl);
#pragma unroll
                            for (int h = 1; h < NH; ++h) {
                                if (hl == (uint32_t)h) {
                                    s_last = __builtin_amdgcn_readlane(src[h], pl);
                                    l_last = (uint32_t)__builtin_amdgcn_readlane((int)local[h], pl);
                                }
                            }
                            const uint32_t last_src = (uint32_t)s_last;
                            const uint32_t last_na = (uint32_t)__builtin_amdgcn_readlane((int)na, (int)last_src);
                            if (l_last + 1 == last_na) {
                                rq_head = uni(ring_r(rq_head + last_src + 1));
                                rq_count = uni(rq_count - (last_src + 1));
                            } else {
                                if (lane == 0) at<uint32_t>(wb, kOffRqFirst, ring_r(rq_head + last_src)) = l_last + 1;
                                rq_head = uni(ring_r(rq_head + last_src));
                                rq_count = uni(rq_count - last_src);
                            }
                        };
                        if (total > 64)
                            area_halves(std::integral_constant<int, 2>{});
                        else
                            area_halves(std::integral_constant<int, 1>{});
                    } else if (have_chunk && low_left) {
                        // ---------------- low-band round ----------------
                        // regions (low_nu + i, 0), i < n (n <= kLowLevels: the levels some lane
                        // still has), of every lane's element: one area each (w = r = 0),
                        // made as independent hash chains.  Level i > 0 is kept only while
                        // both queues still have room for its darts; otherwise it is made
                        // again next round.
                        const uint32_t e_lane = (uint32_t)(chunk - lo) + (uint32_t)lane;
                        auto low_levels = [&](auto levels) {
                            constexpr int N = decltype(levels)::value;
                            bool actl[N];
                            uint64_t gl[N], al[N];
                            FirstDart fl[N];
                            // stage by stage across the levels, so the chains interleave
#pragma unroll
                            for (int i = 0; i < N; ++i) {
                                // lanes without a region are masked by `act`
                                actl[i] = low_nu + (uint32_t)i < n_low;
                                gl[i] = HL(actl[i], KR ^ (((uint64_t)eid << 32) | ((uint64_t)(low_nu + i) << 16)));
                            }
#pragma unroll
                            for (int i = 0; i < N; ++i) al[i] = HL(actl[i], gl[i] ^ KA);
#pragma unroll
                            for (int i = 0; i < N; ++i)
                                fl[i] = first_dart(actl[i], al[i], 0u, low_nu + i, poisson_head(C0, C1, al[i]), true);
                            bool go = true;
#pragma unroll
                            for (int i = 0; i < N; ++i) {
                                if (i > 0) {
                                    const uint32_t np = (uint32_t)__popcll(__ballot(fl[i].pass));
                                    const uint32_t nm = (uint32_t)__popcll(__ballot(fl[i].more));
                                    go = go && pq_count + np <= kCapP && dq_count + nm <= kCapD;
                                }
                                if (go) {
                                    if (DBG) {
                                        const uint64_t nb = (uint64_t)__popcll(__ballot(actl[i]));
                                        n_reg += nb;
                                        n_area += nb;
                                    }
                                    push_area(fl[i], al[i], e_lane, 0u, 0u, low_nu);
                                    low_nu = uni(low_nu + 1);
                                }
                            }
                        };
                        static_assert(kLowLevels == 3, "the dispatch below makes one to three levels");
                        if (wave_any(low_nu + 2 < n_low))
                            low_levels(std::integral_constant<int, 3>{});
                        else if (wave_any(low_nu + 1 < n_low))
                            low_levels(std::integral_constant<int, 2>{});
                        else
                            low_levels(std::integral_constant<int, 1>{});
                        low_left = wave_any(low_nu < n_low);
                        if (!low_left && chunk_total == 0) {
                            chunk += kWave;
                            load_chunk();
                        }
                    } else if (have_chunk) {
                        // ---------------- region round ----------------
                        const uint32_t left = chunk_total - reg_done;
                        // tau < R[1] = 1: every region lies in rank row 0 and has one column;
                        // its rows are r <= tau 2^nu (R[0] = 0, r 2^-nu exact).  Up to 128
                        // regions as two halves of independent hash chains while more than
                        // 64 are left; the second half is kept only while the three queues
                        // have room for what it adds, else it is made again next round.
                        auto region_halves = [&](auto halves) {
                            constexpr int NH = decltype(halves)::value;
                            const uint32_t m = left < 64u * NH ? left : 64u * NH;
                            bool actv[NH];
                            uint32_t ev[NH], metav[NH], rcv[NH], restv[NH];
                            uint64_t gv[NH], av[NH];
                            FirstDart fv[NH];
#pragma unroll
                            for (int h = 0; h < NH; ++h) {
                                // element of each region: marks where an element's regions
                                // start in the window (at 0 for one started before it)
                                const uint32_t base = reg_done + 64u * h;
                                at<int32_t>(wb, kOffMark, lane) = 0;
                                wave_sync();
                                if (nreg > 0 && nreg_excl + nreg > base && nreg_excl < base + 64)
                                    at<int32_t>(wb, kOffMark, nreg_excl > base ? nreg_excl - base : 0) = lane;
                                wave_sync();
                                const int32_t src = scan_max(at<int32_t>(wb, kOffMark, lane));
                                const uint32_t id = (uint32_t)__shfl(eid, src, kWave);
                                const uint32_t s_excl = (uint32_t)__shfl(nreg_excl, src, kWave);
                                const uint32_t nu_base = (uint32_t)__shfl(n_low, src, kWave);
                                actv[h] = 64u * h + (uint32_t)lane < m;
                                ev[h] = (uint32_t)(chunk - lo) + (uint32_t)src;
                                // the element's regions above its low band; lanes past m are
                                // masked by `act`
                                const uint32_t nu = (nu_base + base + (uint32_t)lane - s_excl) & 1023u;
                                metav[h] = nu;
                                gv[h] = HL(actv[h], KR ^ (((uint64_t)id << 32) | ((uint64_t)nu << 16)));
                                const double rcn = fmin(floor(ldexp(tau, (int)nu)) + 1.0, ldexp(1.0, (int)nu));
                                rcv[h] = 1;
                                if (rcn >= 2147483648.0) {
                                    if (actv[h]) range = true;
                                } else {
                                    rcv[h] = (uint32_t)rcn;
                                }
                                restv[h] = actv[h] ? rcv[h] - 1 : 0u;
                            }
#pragma unroll
                            for (int h = 0; h < NH; ++h) av[h] = HL(actv[h], gv[h] ^ KA);
#pragma unroll
                            for (int h = 0; h < NH; ++h)
                                fv[h] = first_dart(actv[h], av[h], 0u, metav[h], poisson_head(C0, C1, av[h]), true);
                            uint32_t done = 0;
                            bool go = true;
#pragma unroll
                            for (int h = 0; h < NH; ++h) {
                                const bool push_r = restv[h] > 0;
                                const uint64_t br = __ballot(push_r);
                                if (h > 0) {
                                    const uint32_t np = (uint32_t)__popcll(__ballot(fv[h].pass));
                                    const uint32_t nm = (uint32_t)__popcll(__ballot(fv[h].more));
                                    go = go && pq_count + np <= kCapP && dq_count + nm <= kCapD &&
                                         rq_count + (uint32_t)__popcll(br) <= kCapR;
                                }
                                if (go) {
                                    push_area(fv[h], av[h], ev[h], 0u, 0u, metav[h]);
                                    if (push_r) {
                                        const uint32_t pos = ring_r(rq_head + rq_count + rank_in(br));
                                        at<uint64_t>(wb, kOffRqG, pos) = gv[h];
                                        at<uint32_t>(wb, kOffRqE, pos) = ev[h];
                                        at<uint32_t>(wb, kOffRqRc, pos) = rcv[h];
                                        at<uint32_t>(wb, kOffRqNa, pos) = rcv[h];
                                        at<uint32_t>(wb, kOffRqFirst, pos) = 1;
                                        at<uint32_t>(wb, kOffRqM, pos) = metav[h];
                                    }
                                    rq_count = uni(rq_count + (uint32_t)__popcll(br));
                                    done = m < 64u * (h + 1) ? m : 64u * (h + 1);
                                }
                            }
                            if (DBG) {
                                n_reg += done;
                                n_area += done;  // every region's first area (w = r = 0)
                            }
                            reg_done = uni(reg_done + done);
                        };
                        if (B1 == 1) {
                            // (two halves pay off where region rounds dominate, as for
                            // bottom-k; measured slower for the others)
                            if (BK && left > 64)
                                region_halves(std::integral_constant<int, 2>{});
                            else
                                region_halves(std::integral_constant<int, 1>{});
                        } else {
                            const uint32_t m = left < 64 ? left : 64;
                            if (DBG) {
                                n_reg += m;
                                n_area += m;  // every region's first area (w = r = 0)
                            }
                            at<int32_t>(wb, kOffMark, lane) = 0;
                            wave_sync();
                            if (nreg > 0 && nreg_excl + nreg > reg_done && nreg_excl < reg_done + 64)
                                at<int32_t>(wb, kOffMark, nreg_excl > reg_done ? nreg_excl - reg_done : 0) = lane;
                            wave_sync();
                            const int32_t src = scan_max(at<int32_t>(wb, kOffMark, lane));
                            const uint32_t id = (uint32_t)__shfl(eid, src, kWave);
                            const uint32_t s_excl = (uint32_t)__shfl(nreg_excl, src, kWave);
                            const bool act = (uint32_t)lane < m;
                            const uint32_t e = (uint32_t)(chunk - lo) + (uint32_t)src;
                            uint32_t X = 0, rest = 0, meta = 0, rcu = 1, nau = 1;
                            uint64_t a = 0, g = 0;
                            const double x = __shfl(ex, src, kWave);
                            if (act) {
                                // region `local` of the element: nu = local / B1, rho = local % B1
                                const uint32_t local = reg_done + (uint32_t)lane - s_excl;
                                uint32_t nu = (uint32_t)((float)local * inv_b1);
                                while (nu * (uint32_t)B1 > local) --nu;
                                while ((nu + 1) * (uint32_t)B1 <= local) ++nu;
                                const uint32_t rho = local - nu * (uint32_t)B1;
                                meta = nu | (rho << 10);
                                g = H(KR ^ (((uint64_t)id << 32) | ((uint64_t)nu << 16) | rho));
                                double wc = 1.0, rcn;
                                if (rho == 0) {
                                    // R[0] = 0 and r * 2^-nu is exact: r <= tau * 2^nu
                                    const double rcap = ldexp(1.0, (int)nu);
                                    rcn = floor(ldexp(tau, (int)nu)) + 1.0;
                                    rcn = rcn < rcap ? rcn : rcap;
                                } else {
                                    const double Wn = w_corner(sW, u, (int)nu), Rr = r_corner(sR, (int)rho);
                                    const double dnu = ldexp(u, (int)nu - (int)rho);
                                    const double drho = ldexp(1.0, (int)rho - (int)nu);
                                    const double wcap = ldexp(1.0, (int)rho);
                                    wc = prefix_count(Wn, dnu, x, wcap,
                                                     floor((x - Wn) * td * ldexp(1.0, (int)rho - (int)nu)) + 1.0);
                                    const double rcap = ldexp(1.0, (int)nu);
                                    rcn = prefix_count(Rr, drho, tau, rcap,
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
                                a = H(g ^ KA);
                                X = poisson_head(C0, C1, a);
                                rest = nau - 1;
                            }
                            emit_area(act, a, e, 0u, 0u, meta, X, false);
                            const bool push_r = act && rest > 0;
                            const uint64_t br = __ballot(push_r);
                            if (push_r) {
                                const uint32_t pos = ring_r(rq_head + rq_count + rank_in(br));
                                at<uint64_t>(wb, kOffRqG, pos) = g;
                                at<uint32_t>(wb, kOffRqE, pos) = e;
                                at<uint32_t>(wb, kOffRqRc, pos) = rcu;
                                at<uint32_t>(wb, kOffRqNa, pos) = nau;
                                at<uint32_t>(wb, kOffRqFirst, pos) = 1;
                                at<uint32_t>(wb, kOffRqM, pos) = meta;
                            }
                            rq_count = uni(rq_count + (uint32_t)__popcll(br));
                            reg_done = uni(reg_done + m);
                        }
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
                if (single) break;
                if (BK) {
                    // done once the darts of rank <= tau hold k distinct ones
                    if (bk_count >= (uint32_t)k) {
                        bk_compact();
                        if (bk_count >= (uint32_t)k) break;
                    }
                    tau_prev = tau;
                    phi *= 2.0;
                    continue;
                }
                bool filled = true;
                if (RT) {
                    filled = lane >= k || tr[7] != kNoRank;
                } else if (LSH) {
                    for (int j = lane; j < k; j += kWave) filled &= T.cnt[j] >= K;
                } else {
                    for (int j = lane; j < (int)tile_n; j += kWave) filled &= bin_rank[j] != kRankEmpty;
                }
                if (wave_all(filled)) break;
                tau_prev = tau;
                phi *= 2.0;
            }
        return status;
    };

    auto clear_buckets = [&]() {
        if (BK) {
            bk_count = 0;
            cut_r = ~0ull;
            cut_s = ~0ull;
        } else if (RT) {
#pragma unroll
            for (int m = 0; m < 8; ++m) tr[m] = kNoRank;
        } else if (LSH) {
            for (int j = lane; j < k; j += kWave) T.cnt[j] = 0;
        } else {
            for (int j = lane; j < (int)tile_n; j += kWave) {
                bin_rank[j] = kRankEmpty;
                bin_s[j] = ~0ull;
            }
        }
    };

    // Minhash outputs of buckets [tile_lo, tile_lo + tile_n) of a set (tile_lo
    // is a multiple of 64, so the tile owns whole words of the 1-bit sketch).
    auto write_tile = [&](int64_t set, bool ok) {
        for (int j = lane; j < (int)tile_n; j += kWave) {
            const uint64_t s = ok ? bin_s[j] : ~0ull;
            const uint64_t rb = ok ? bin_rank[j] : kRankEmpty;
            const int64_t o = set * k + tile_lo + j;
            if (out_u32) out_u32[o] = ok ? (uint32_t)s : 0xFFFFFFFFu;
            if (out_s) out_s[o] = s;
            if (out_rank) out_rank[o] = __longlong_as_double((long long)rb);
        }
        if (out_bits) {
            const int words = (k + 63) / 64;
            for (int wd = 0; wd * 64 < (int)tile_n; ++wd) {
                const int j = wd * 64 + lane;
                const bool bit = ok && j < (int)tile_n && (bin_s[j] & 1ull);
                const uint64_t word = __ballot(bit);
                if (lane == 0) out_bits[set * words + (int)(tile_lo / 64) + wd] = word;
            }
        }
    };

    // parts of a device plan: the planning kernel's cursor, at most the capacity
    const int64_t np = plan_dev ? min((int64_t)plan_dev[1], n_parts) : n_parts;
    for (;;) {
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(next_set, 1ull);
        const int64_t item = (int64_t)uni64(got);  // lane 0 is the first active lane
        if (item >= np + n_sets) break;
        int64_t set;
        int8_t status;
        bool tiles_written = false;  // a tiled minhash set wrote its outputs tile by tile
        n_reg = n_area = n_gen = n_rank = n_acc = n_pass = 0;
        phi_end = 0.0;
        if (MODE == kModeMinhash && item < np) {
            // ---- one part of a heavy set ----
            const Part pt = parts[item];
            if (pt.set < 0) continue;  // an empty slot of the device plan
            HeavySet* hs = heavy + pt.heavy;
            set = pt.set;
            const int64_t b0 = rp[set], b1 = rp[set + 1];
            const int64_t lo = b0 + (int64_t)pt.index * split;
            const int64_t hi = lo + split < b1 ? lo + split : b1;
            const double S = hs->sum;
            status = (int8_t)hs->status;
            if (DBG && status == kSetOk && repeated && repeated[set]) status = kSetInvalid;
            uint64_t* mine = partial + (size_t)(hs->base + pt.index) * 2 * k;
            if (status == kSetOk) {
                clear_buckets();
                if (run(lo, hi, S, phi0, -1.0, true) == kSetRange && lane == 0) atomicOr(&hs->range, 1);
                wave_sync();
                for (int j = lane; j < k; j += kWave) {
                    mine[j] = bin_rank[j];
                    mine[k + j] = bin_s[j];
                }
            }
            if (DBG && out_cnt && lane == 0) {
                // the part's share of the set's counts (the plan zeroed them)
                int64_t* oc = out_cnt + set * kCounterWords;
                atomicAdd((unsigned long long*)&oc[0], (unsigned long long)n_reg);
                atomicAdd((unsigned long long*)&oc[1], (unsigned long long)n_area);
                atomicAdd((unsigned long long*)&oc[2], (unsigned long long)n_gen);
                atomicAdd((unsigned long long*)&oc[3], (unsigned long long)n_rank);
                atomicAdd((unsigned long long*)&oc[4], (unsigned long long)n_acc);
            }
            n_reg = n_area = n_gen = n_rank = n_acc = 0;
            n_pass = 1;  // the parts together make the first pass
            phi_end = phi0;
            __threadfence();  // the buckets are visible before the part counts as done
            int last = 0;
            if (lane == 0) last = atomicAdd(&hs->done, 1) == hs->parts - 1;
            if (!uni(last)) continue;
            __threadfence();
            if (status == kSetOk && __hip_atomic_load(&hs->range, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                status = kSetRange;
            if (status == kSetOk) {
                // merge the parts' buckets, then finish the retry over the whole set
                const uint64_t* first = partial + (size_t)hs->base * 2 * k;
                for (int j = lane; j < k; j += kWave) {
                    uint64_t br = kRankEmpty, bs = ~0ull;
                    for (int q = 0; q < hs->parts; ++q) {
                        const uint64_t r = __builtin_nontemporal_load(first + (size_t)q * 2 * k + j);
                        const uint64_t v = __builtin_nontemporal_load(first + (size_t)q * 2 * k + k + j);
                        if (r < br || (r == br && v < bs)) {
                            br = r;
                            bs = v;
                        }
                    }
                    bin_rank[j] = br;
                    bin_s[j] = bs;
                }
                wave_sync();
                bool filled = true;
                for (int j = lane; j < k; j += kWave) filled &= bin_rank[j] != kRankEmpty;
                if (!wave_all(filled)) status = run(b0, b1, S, 2.0 * phi0, phi0 / S, false);
            }
        } else {
            set = order ? (int64_t)order[item - np] : item - np;  // largest sets first
            const int64_t b0 = rp[set], b1 = rp[set + 1];
            if (MODE == kModeMinhash && split > 0 && (planned ? planned[set] != 0 : b1 - b0 > split))
                continue;  // served by its parts
            const RowInfo ri = scan_row(wts, b0, b1, lane);
            status = ri.status;
            if (DBG && status == kSetOk && repeated && repeated[set]) status = kSetInvalid;
            if (status == kSetOk) {
                clear_buckets();
                status = run(b0, b1, ri.sum, phi0, -1.0, false);
            }
            if (MODE == kModeMinhash && K < k) {
                // tiled buckets: the first tile's minima are in LDS; every
                // further tile repeats the schedule for its own buckets (the
                // minimum of each bucket is the same under any schedule)
                wave_sync();
                write_tile(set, status == kSetOk);
                for (tile_lo = (uint32_t)K; tile_lo < (uint32_t)k && status == kSetOk; tile_lo += (uint32_t)K) {
                    tile_n = min((uint32_t)K, (uint32_t)k - tile_lo);
                    wave_sync();
                    clear_buckets();
                    status = run(b0, b1, ri.sum, phi0, -1.0, false);
                    wave_sync();
                    write_tile(set, status == kSetOk);
                }
                if (status != kSetOk) {
                    // a later tile met the range limit: the set's outputs are all non-OK
                    for (tile_lo = 0; tile_lo < (uint32_t)k; tile_lo += (uint32_t)K) {
                        tile_n = min((uint32_t)K, (uint32_t)k - tile_lo);
                        write_tile(set, false);
                    }
                }
                tile_lo = 0;
                tile_n = (uint32_t)K;
                tiles_written = true;
            }
        }
        if (DBG && out_cnt && lane == 0) {
            // counts of this wave's passes; a heavy set's parts added theirs already
            int64_t* oc = out_cnt + set * kCounterWords;
            const bool heavy_set = MODE == kModeMinhash && item < np;
            const uint64_t v[kCounterWords] = {n_reg, n_area, n_gen, n_rank, n_acc, n_pass,
                                               (uint64_t)__double_as_longlong(phi_end), 0};
            for (int q = 0; q < kCounterWords; ++q) {
                if (heavy_set && q < 5) atomicAdd((unsigned long long*)&oc[q], (unsigned long long)v[q]);
                else oc[q] = (int64_t)v[q];
            }
        }
        // outputs
        wave_sync();
        const bool ok = status == kSetOk;
        if (RT) {
            // table l's key folds its 8 ordered dart ids
            if (lane < k) {
                uint64_t h = 0;
                if (ok) {
                    h = H(sp->key_l ^ (uint64_t)lane);
#pragma unroll
                    for (int m2 = 0; m2 < 8; ++m2) h = H(h ^ ts[m2]);
                }
                out_keys[set * k + lane] = h;
            }
        } else if (LSH) {
            // table l's key folds its K ordered dart ids
            for (int l = lane; l < k; l += kWave) {
                uint64_t h = 0;
                if (ok) {
                    h = H(sp->key_l ^ (uint64_t)l);
                    for (int m2 = 0; m2 < K; ++m2) h = H(h ^ T.sval[(size_t)l * K + m2]);
                }
                out_keys[set * k + l] = h;
            }
        } else if (!tiles_written) {
            write_tile(set, ok);
        }
        if (out_status && lane == 0) out_status[set] = status;
        wave_sync();  // the next set reuses this wave's LDS
    }
}

__global__ void reset_counter_kernel(unsigned long long* c) { *c = 0ull; }

// Explicit instantiations: the host launches all three.
#define DMS_FAST_KERNEL(M, HK, D)                                                                 \
    template __global__ void fast_kernel<M, HK, D>(const SpecTables*, int64_t, const int64_t*, const int32_t*, \
                                            const double*, int, int, uint32_t*, uint64_t*, int8_t*,     \
                                            uint64_t*, double*, uint64_t*, double, double,             \
                                            unsigned long long*, const Part*, int64_t, HeavySet*,      \
                                            uint64_t*, int64_t, const uint32_t*, int64_t*, const uint8_t*, \
                                            const unsigned long long*, const uint8_t*);
#define DMS_FAST_KERNELS(M, HK) DMS_FAST_KERNEL(M, HK, false) DMS_FAST_KERNEL(M, HK, true)
DMS_FAST_KERNELS(kModeMinhash, kHashMix)
DMS_FAST_KERNELS(kModeLsh, kHashMix)
DMS_FAST_KERNELS(kModeBottomK, kHashMix)
DMS_FAST_KERNELS(kModeMinhash, kHashTab)
DMS_FAST_KERNELS(kModeLsh, kHashTab)
DMS_FAST_KERNELS(kModeBottomK, kHashTab)
DMS_FAST_KERNELS(kModeLshReg, kHashMix)
DMS_FAST_KERNELS(kModeLshReg, kHashTab)
#undef DMS_FAST_KERNELS
#undef DMS_FAST_KERNEL

// Device-side planning of the heavy sets.  plan[0] counts the heavy sets that
// got parts, plan[1] is the parts cursor; both start at 0 (plan_reset_kernel).
// A set above the split threshold reserves its parts with one atomic add on
// the cursor (no retry loop: many heavy sets would serialize on it); a set
// whose range passes the capacity gets no parts and is sketched whole by one
// wave, and the slots of its range below the capacity become empty parts
// (set -1) that the main kernel skips, so [0, min(cursor, capacity)) holds no
// unwritten slot.  planned[s] tells the main kernel which sets its parts serve.
__global__ void plan_reset_kernel(unsigned long long* plan)
{
    if (threadIdx.x < 8) plan[threadIdx.x] = 0ull;
}

__global__ void __launch_bounds__(256)
plan_kernel(int64_t n_sets, const int64_t* __restrict__ rp, int64_t split, int64_t part_cap,
            unsigned long long* plan, Part* parts, HeavySet* heavy, uint8_t* planned, int64_t* out_cnt)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sets) return;
    const int64_t nnz = rp[s + 1] - rp[s];
    uint8_t mine = 0;
    if (nnz > split) {
        const int64_t P = (nnz + split - 1) / split;
        const int64_t base = P < part_cap ? (int64_t)atomicAdd(&plan[1], (unsigned long long)P) : part_cap;
        if (base + P > part_cap) {
            for (int64_t p = base; p < part_cap; ++p) {
                Part pt;
                pt.set = -1;  // an empty slot of a range that did not fit
                pt.heavy = 0;
                pt.index = 0;
                parts[p] = pt;
            }
        } else {
            if (out_cnt) {  // the parts of the set add their counts
                for (int q = 0; q < kCounterWords; ++q) out_cnt[s * kCounterWords + q] = 0;
            }
            const int32_t h = (int32_t)atomicAdd(&plan[0], 1ull);
            HeavySet hs;
            hs.sum = 0.0;
            hs.set = s;
            hs.base = base;
            hs.parts = (int32_t)P;
            hs.done = 0;
            hs.range = 0;
            hs.status = kSetOk;
            heavy[h] = hs;
            for (int32_t p = 0; p < (int32_t)P; ++p) {
                Part pt;
                pt.set = s;
                pt.heavy = h;
                pt.index = p;
                parts[base + p] = pt;
            }
            mine = 1;
        }
    }
    planned[s] = mine;
}

// One wave per heavy set of a device plan (n_heavy read from plan[0]; the grid
// covers the capacity): validity and ||x||_1 of the whole row.
__global__ void __launch_bounds__(256)
plan_scan_kernel(const unsigned long long* plan, const int64_t* __restrict__ rp, const double* __restrict__ w,
                 HeavySet* heavy)
{
    const int lane = threadIdx.x & 63;
    const int64_t h = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (h >= (int64_t)plan[0]) return;
    const int64_t s = heavy[h].set;
    const RowInfo ri = scan_row(w, rp[s], rp[s + 1], lane);
    if (lane == 0) {
        heavy[h].sum = ri.sum;
        heavy[h].status = ri.status;
    }
}

// One wave per heavy set: validity and ||x||_1 of the whole row.
__global__ void __launch_bounds__(256)
heavy_scan_kernel(int64_t n_heavy, const int64_t* __restrict__ rp, const double* __restrict__ w,
                  HeavySet* heavy)
{
    const int lane = threadIdx.x & 63;
    const int64_t h = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (h >= n_heavy) return;
    const int64_t s = heavy[h].set;
    const RowInfo ri = scan_row(w, rp[s], rp[s + 1], lane);
    if (lane == 0) {
        heavy[h].sum = ri.sum;
        heavy[h].status = ri.status;
    }
}

hipError_t launch_heavy_scan(int64_t n_heavy, const int64_t* rp, const double* w, HeavySet* heavy,
                             hipStream_t st)
{
    if (n_heavy <= 0) return hipSuccess;
    hipLaunchKernelGGL(heavy_scan_kernel, dim3((unsigned)((n_heavy + 3) / 4)), dim3(256), 0, st, n_heavy,
                       rp, w, heavy);
    return hipGetLastError();
}

size_t plan_part_bytes() { return sizeof(Part); }
size_t plan_heavy_bytes() { return sizeof(HeavySet); }

hipError_t launch_plan(int64_t n_sets, const int64_t* rp, const double* w, int64_t split, int64_t part_cap,
                       unsigned long long* plan, void* parts, void* heavy, uint8_t* planned, int64_t* out_cnt,
                       hipStream_t st)
{
    hipLaunchKernelGGL(plan_reset_kernel, dim3(1), dim3(64), 0, st, plan);
    hipLaunchKernelGGL(plan_kernel, dim3((unsigned)((n_sets + 255) / 256)), dim3(256), 0, st, n_sets, rp, split,
                       part_cap, plan, (Part*)parts, (HeavySet*)heavy, planned, out_cnt);
    const int64_t heavy_cap = part_cap / 2;  // every heavy set has two parts or more
    if (heavy_cap > 0)
        hipLaunchKernelGGL(plan_scan_kernel, dim3((unsigned)((heavy_cap + 3) / 4)), dim3(256), 0, st, plan, rp, w,
                           (HeavySet*)heavy);
    return hipGetLastError();
}

// Waves per block: the count (1..4, at most 64 KiB of LDS per block) that
// keeps the most waves resident in a CU's 160 KiB of LDS; ties go to the
// larger block, which shares one copy of the tables.
size_t fast_lds(int mode, int k, int K, int waves)
{
    return kTablesBytes + (size_t)waves * wave_lds_bytes(mode, k, K);
}

// A CU has 160 KiB of LDS and hands it to blocks in units of 1,280 bytes (measured
// on gfx950: a block of 14,880 bytes occupies 15,360, so ten such blocks fit, not
// eleven; the runtime's occupancy query does not round and over-counts).
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr size_t kLdsGranule = 1280;

int fast_blocks_per_cu(int mode, int k, int K, int waves)
{
    const size_t block = fast_lds(mode, k, K, waves);
    const size_t held = (block + kLdsGranule - 1) / kLdsGranule * kLdsGranule;
    return block > 65536 ? 0 : (int)(kLdsPerCu / held);
}

int fast_waves(int mode, int k, int K)
{
    int best = 1, best_resident = 0;
    for (int w = 1; w <= 4; ++w) {
        const int resident = w * fast_blocks_per_cu(mode, k, K, w);
        if (resident >= best_resident) {
            best = w;
            best_resident = resident;
        }
    }
    return best;
}

// Buckets a minhash wave holds at once: all k when the minima fit next to the
// queues in a block of at most 64 KiB, else equal tiles of whole 64-bucket words.
int minhash_tile(int k)
{
    if (fast_lds(kModeMinhash, k, k, 1) <= 65536) return k;
    const int kmax = (int)((65536 - kTablesBytes - kQueueBytes) / 16) / 64 * 64;
    const int tiles = (k + kmax - 1) / kmax;
    return ((k + tiles - 1) / tiles + 63) / 64 * 64;
}
// The tile for an option value (0: minhash_tile(k); t: t buckets per tile when
// t < k, a multiple of 64), or 0 when t's minima do not fit one wave's LDS.
int minhash_tile_for(int k, int t)
{
    if (t <= 0 || t >= k) return minhash_tile(k);
    if (t % 64 || fast_lds(kModeMinhash, k, t, 1) > 65536) return 0;
    return t;
}
// Waves per block for an option value (0: the most resident waves), or 0 when
// the block does not fit 64 KiB of LDS.
int minhash_waves_for(int k, int kt, int waves)
{
    if (waves <= 0) return fast_waves(kModeMinhash, k, kt);
    if (waves > 4 || fast_lds(kModeMinhash, k, kt, waves) > 65536) return 0;
    return waves;
}
int fast_waves_per_block(int k) { return fast_waves(kModeMinhash, k, minhash_tile(k)); }
size_t fast_lds_bytes(int k, int waves) { return fast_lds(kModeMinhash, k, minhash_tile(k), waves); }

int lsh_fast_mode(int L, int K) { return L <= kWave && K == 8 ? kModeLshReg : kModeLsh; }

using FastKernel = void (*)(const SpecTables*, int64_t, const int64_t*, const int32_t*, const double*, int, int,
                            uint32_t*, uint64_t*, int8_t*, uint64_t*, double*, uint64_t*, double, double,
                            unsigned long long*, const Part*, int64_t, HeavySet*, uint64_t*, int64_t,
                            const uint32_t*, int64_t*, const uint8_t*, const unsigned long long*, const uint8_t*);

template <int MODE>
FastKernel pick_fast(int hash, bool dbg)
{
    if (hash == kHashTab) return dbg ? fast_kernel<MODE, kHashTab, true> : fast_kernel<MODE, kHashTab, false>;
    return dbg ? fast_kernel<MODE, kHashMix, true> : fast_kernel<MODE, kHashMix, false>;
}

// The fast kernel for a sink, a hash and whether counts or row validation are
// asked for (those run in a variant of their own, so that the plain kernel
// keeps its registers).
FastKernel fast_kernel_for(int mode, int hash, bool dbg)
{
    switch (mode) {
    case kModeLshReg: return pick_fast<kModeLshReg>(hash, dbg);
    case kModeLsh: return pick_fast<kModeLsh>(hash, dbg);
    case kModeBottomK: return pick_fast<kModeBottomK>(hash, dbg);
    default: return pick_fast<kModeMinhash>(hash, dbg);
    }
}

const void* fast_kernel_address(int mode, int hash)
{
    return reinterpret_cast<const void*>(fast_kernel_for(mode, hash, false));
}

hipError_t launch_sketch_fast_split(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                                    const int32_t* idx, const double* w, int k, uint32_t* out_u32,
                                    uint64_t* out_bits, int8_t* out_status, uint64_t* out_s,
                                    double* out_rank, double phi0, double phi_max,
                                    unsigned long long* counter, int blocks, const void* parts,
                                    int64_t n_parts, void* heavy, uint64_t* partial, int64_t split,
                                    const uint32_t* order, int hash, const LaunchExtras& x,
                                    const unsigned long long* plan_dev, const uint8_t* planned, int kt_opt,
                                    int waves_opt, hipStream_t st)
{
    if (n_sets <= 0) return hipSuccess;
    const int kt = minhash_tile_for(k, kt_opt);
    const int waves = minhash_waves_for(k, kt, waves_opt);
    if (kt <= 0 || waves <= 0) return hipErrorInvalidValue;
    if (kt < k && n_parts > 0) return hipErrorInvalidValue;  // tiled buckets are not split
    const size_t lds = fast_lds(kModeMinhash, k, kt, waves);
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    const int64_t need = (n_parts + n_sets + waves - 1) / waves;
    if (blocks <= 0 || blocks > need) blocks = (int)(need < 1 ? 1 : need);
    const FastKernel kern = fast_kernel_for(kModeMinhash, hash, x.counters || x.repeated);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), lds, st, sp,
                       n_sets, rp, idx, w, k, kt, out_u32, out_bits, out_status, out_s, out_rank,
                       (uint64_t*)nullptr, phi0, phi_max, counter, (const Part*)parts, n_parts,
                       (HeavySet*)heavy, partial, split, order, x.counters, x.repeated, plan_dev, planned);
    return hipGetLastError();
}

hipError_t launch_sketch_fast(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                              const int32_t* idx, const double* w, int k, uint32_t* out_u32,
                              uint64_t* out_bits, int8_t* out_status, uint64_t* out_s,
                              double* out_rank, double phi0, double phi_max,
                              unsigned long long* counter, int blocks, int hash, const LaunchExtras& x,
                              hipStream_t st)
{
    return launch_sketch_fast_split(sp, n_sets, rp, idx, w, k, out_u32, out_bits, out_status, out_s,
                                    out_rank, phi0, phi_max, counter, blocks, nullptr, 0, nullptr,
                                    nullptr, 0, nullptr, hash, x, nullptr, nullptr, 0, 0, st);
}

hipError_t launch_lsh_fast(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                           const int32_t* idx, const double* w, int L, int K, uint64_t* out_keys,
                           int8_t* out_status, double phi0, double phi_max,
                           unsigned long long* counter, int blocks, const uint32_t* order, int hash,
                           const LaunchExtras& x, hipStream_t st)
{
    if (n_sets <= 0) return hipSuccess;
    const int mode = lsh_fast_mode(L, K);
    const int waves = fast_waves(mode, L, K);
    const size_t lds = fast_lds(mode, L, K, waves);
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    const int64_t need = (n_sets + waves - 1) / waves;
    if (blocks <= 0 || blocks > need) blocks = (int)(need < 1 ? 1 : need);
    const FastKernel kern = fast_kernel_for(mode, hash, x.counters || x.repeated);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), lds, st, sp,
                       n_sets, rp, idx, w, L, K, (uint32_t*)nullptr, (uint64_t*)nullptr, out_status,
                       (uint64_t*)nullptr, (double*)nullptr, out_keys, phi0, phi_max, counter,
                       (const Part*)nullptr, (int64_t)0, (HeavySet*)nullptr, (uint64_t*)nullptr,
                       (int64_t)0, order, x.counters, x.repeated, (const unsigned long long*)nullptr,
                       (const uint8_t*)nullptr);
    return hipGetLastError();
}

hipError_t launch_bottomk_fast(const SpecTables* sp, int64_t n_sets, const int64_t* rp,
                               const int32_t* idx, const double* w, int k, uint64_t* out_s,
                               double* out_rank, int8_t* out_status, double phi0, double phi_max,
                               unsigned long long* counter, int blocks, const uint32_t* order, int hash,
                               const LaunchExtras& x, hipStream_t st)
{
    if (n_sets <= 0) return hipSuccess;
    const int waves = fast_waves(kModeBottomK, k, 1);
    const size_t lds = fast_lds(kModeBottomK, k, 1, waves);
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    const int64_t need = (n_sets + waves - 1) / waves;
    if (blocks <= 0 || blocks > need) blocks = (int)(need < 1 ? 1 : need);
    const FastKernel kern = fast_kernel_for(kModeBottomK, hash, x.counters || x.repeated);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * waves), lds, st, sp,
                       n_sets, rp, idx, w, k, 1, (uint32_t*)nullptr, (uint64_t*)nullptr, out_status,
                       out_s, out_rank, (uint64_t*)nullptr, phi0, phi_max, counter, (const Part*)nullptr,
                       (int64_t)0, (HeavySet*)nullptr, (uint64_t*)nullptr, (int64_t)0, order, x.counters,
                       x.repeated, (const unsigned long long*)nullptr, (const uint8_t*)nullptr);
    return hipGetLastError();
}

}  // namespace dms
