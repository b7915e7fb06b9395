// Internal declarations shared by the host runtime and the HIP kernels of the
// DartMinHash library.  Nothing here is part of the public C ABI.
#pragma once

#include <cstdint>

namespace dms {

constexpr int kTable = 64;      // region corners kept in tables (nu, rho < 64)
constexpr int kMaxIndex = 1024; // nu and rho stay below this in the supported domain
constexpr int kNumPoisson = 20; // Poisson(1) thresholds for n = 0..19
constexpr int kTabWords = 8 * 256;  // simple-tabulation tables, one per byte of the hashed word

// The hash of every hashing step: the SplitMix64 output function, or simple
// tabulation with Mersenne Twister tables (the paper's randomness source).
enum HashKind : int { kHashMix = 0, kHashTab = 1 };

// Everything a kernel needs to generate darts for one value of t.  Lives in
// device memory, one copy per t, owned by the context.
struct SpecTables {
    double W[kTable];       // W[nu]  = RN(RN(2^nu - 1) / t); for nu >= 54 it equals ldexp(u, nu)
    double R[kTable];       // R[rho] = RN(2^rho - 1);        for rho >= 54 it equals 2^rho
    uint64_t pois[kNumPoisson];
    uint64_t key_r, key_a, key_u, key_v, key_s, key_l;
    double u;               // RN(1/t)
    uint32_t t;
    uint32_t pad;
    uint64_t tab[kTabWords];  // MT19937-64 outputs 7.. for the seed: table b serves byte b
};

uint32_t t_of_k(int32_t k);
bool poisson_thresholds(uint64_t out[kNumPoisson]);
void hash_keys(uint64_t seed, uint64_t keys[6]);
void hash_tables(uint64_t seed, uint64_t tab[kTabWords]);
bool make_spec(uint64_t seed, uint32_t t, SpecTables* sp);

// Region corners for any index.  For nu >= 54, RN(2^nu - 1) = 2^nu and
// RN(2^nu / t) = 2^nu * RN(1/t) (scaling by a power of two is exact), so the
// corners past the tables are exact powers of two times u, resp. 1.
double corner_w(const SpecTables& sp, int nu);
double corner_r(const SpecTables& sp, int rho);

// Sinks of the fast kernel: k bucket minima, (L,K) LSH tables, bottom-k buffer.
// kModeLshReg: (L,K) LSH with L <= 64 and K = 8, lane l holding table l in
// registers; kModeLsh keeps the tables in LDS for every other shape.
enum FastMode : int { kModeMinhash = 0, kModeLsh = 1, kModeBottomK = 2, kModeLshReg = 3 };

// A set with more nonzeros than the split threshold is cut into parts of at
// most `split` consecutive nonzeros.  Every part runs one phi pass over its
// elements into buckets of its own (in HBM); the part that finishes last
// merges them by the exact (rank, id) minimum and, if a bucket is still empty,
// carries on with the doubling retry over the whole set.  Minimum is
// associative and idempotent, so the result equals the one-wave result.
struct HeavySet {
    double sum;      // ||x||_1 of the set (positive weights), set by the row scan
    int64_t set;     // row index within the launch
    int64_t base;    // index of its first part
    int32_t parts;
    int32_t done;    // parts finished (0 at launch)
    int32_t range;   // a part met an out-of-range index (0 at launch)
    int32_t status;  // status of the row scan
};
struct Part {
    int64_t set;
    int32_t heavy;   // index of its HeavySet
    int32_t index;   // part number within the set
};

// Per-set enumeration counts (DMS_FLAG_COUNTERS): regions, areas, darts
// generated, darts whose rank lies in the pass's new band (tau_prev, tau],
// those of them accepted, phi passes run, the last phi (bit pattern of the
// double), and a zero word.
constexpr int kCounterWords = 8;

// Per-set status values written to out_status.
enum SetStatus : int8_t { kSetOk = 0, kSetEmpty = 1, kSetRange = 2, kSetInvalid = 3, kQueryOverflow = 4 };

}  // namespace dms
