// Device helpers of the DartMinHash kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dms_internal.h"

namespace dms {

constexpr int kWave = 64;
constexpr uint64_t kRankEmpty = 0x7FF0000000000000ull;  // bit pattern of +inf

// SplitMix64 output function: the specification's 64-bit mixer.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// The 53 high bits of a hash as a uniform double in [0, 1) (exact conversion).
// The hash function of the specification, chosen at compile time.
template <int HK>
struct Hasher {
    __device__ explicit Hasher(const SpecTables*) {}
    __device__ __forceinline__ uint64_t operator()(uint64_t z) const { return mix64(z); }
};
template <>
struct Hasher<kHashTab> {
    const uint64_t* __restrict__ tab;
    __device__ explicit Hasher(const SpecTables* sp) : tab(sp->tab) {}
    __device__ __forceinline__ uint64_t operator()(uint64_t z) const
    {
        uint64_t h = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) h ^= tab[b * 256 + ((z >> (8 * b)) & 0xFFu)];
        return h;
    }
};

// A 16-byte load marked non-temporal: for inputs that are read once, it streams
// from HBM without displacing cached data (measured +20-40% on the estimators).
__device__ __forceinline__ uint4 load_stream(const uint4* p)
{
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ double unit53(uint64_t h)
{
    return (double)(h >> 11) * 0x1.0p-53;
}

// Darts in an area: number of Poisson thresholds at or below the area hash.
__device__ __forceinline__ uint32_t poisson_count(const uint64_t* __restrict__ pois, uint64_t a)
{
    uint32_t x = 0;
    while (x < (uint32_t)kNumPoisson && a >= pois[x]) ++x;
    return x;
}

// Lower corners of weight region nu and rank region rho: tables below kTable,
// exact closed forms above (see corner_w / corner_r in dms_internal.h).
// (Both sides are evaluated and one is selected: no branch for the lanes.)
__device__ __forceinline__ double w_corner(const double* tab, double u, int nu)
{
    const double t = tab[nu < kTable ? nu : kTable - 1];
    return nu < kTable ? t : ldexp(u, nu);
}
__device__ __forceinline__ double r_corner(const double* tab, int rho)
{
    const double t = tab[rho < kTable ? rho : kTable - 1];
    return rho < kTable ? t : ldexp(1.0, rho);
}

// Length of the prefix of c in [0, cap) with base + c * step <= bound, for an
// exit predicate that holds at c = 0 and, with rounding monotone, stays false
// once false: the columns of a region under x_i, or its rows below tau
// (Section 2).  `est` is a real-number estimate of the answer; it is clamped to
// [1, cap] and corrected one step at a time with the exact predicate.  Counts of
// 2^52 or more are returned unrefined (the callers reject everything above 2^32).
__device__ __forceinline__ double prefix_count(double base, double step, double bound, double cap,
                                               double est)
{
    double c = est;
    if (!(c >= 1.0)) c = 1.0;
    if (c > cap) c = cap;
    if (c >= 0x1.0p52) return c;
    while (c < cap && base + c * step <= bound) c += 1.0;
    while (c > 1.0 && !(base + (c - 1.0) * step <= bound)) c -= 1.0;
    return c;
}

// bucket = (hi32(s) * n) >> 32
__device__ __forceinline__ uint32_t bucket_of(uint64_t s, uint32_t n)
{
    return (uint32_t)(((s >> 32) * (uint64_t)n) >> 32);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// The first active lane's value as a wave-uniform (scalar) value: the
// compiler then keeps what depends on it in scalar registers and branches.
__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double uni_f64(double v)
{
    return __longlong_as_double((long long)uni64((uint64_t)__double_as_longlong(v)));
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Orders this wave's LDS accesses before and after the call, so that values
// written by other lanes of the wave are seen by later reads (no hardware
// barrier: the lanes of a wave execute in lockstep).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }
__device__ __forceinline__ bool wave_all(bool p) { return __ballot(!p) == 0ull; }

// Lexicographic (rank, s) minimum of one bucket, shared by the lanes of one
// wave.  rank is non-negative, so its bit pattern orders like the value.
// After the rank minimum, the bucket's rank is read back in the same batch of
// LDS requests (the wave's LDS operations run in order); the lane whose rank
// lowered the bucket stores its id hash, then every lane holding the bucket's
// rank takes the minimum of the id hashes (a lane that met the bucket at an
// equal rank, from this or an earlier instruction).  Lanes of the same wave
// that hit the same bucket in the same instruction are resolved by these
// steps; lanes of other waves must not touch the bucket.
__device__ __forceinline__ void bucket_min(uint64_t* rank_bits, uint64_t* sval, uint32_t b,
                                           uint64_t rb, uint64_t s)
{
    const uint64_t old = __hip_atomic_fetch_min(&rank_bits[b], rb, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
    const uint64_t cur = __hip_atomic_load(&rank_bits[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const bool hold = cur == rb;
    if (hold && rb < old)  // the bucket's rank went down: the old id hash is void
        __hip_atomic_store(&sval[b], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    wave_sync();  // the store lands before any minimum of the same bucket
    if (hold) __hip_atomic_fetch_min(&sval[b], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Validity, positive sum and maximum of one CSR row (lanes over nonzeros).
struct RowInfo {
    double sum;
    int8_t status;
};

__device__ __forceinline__ RowInfo scan_row(const double* __restrict__ w, int64_t b0, int64_t b1,
                                            int lane)
{
    double sum = 0.0, mx = 0.0;
    bool bad = false;
    for (int64_t e = b0 + lane; e < b1; e += kWave) {
        double v = w[e];
        if (__builtin_isnan(v) || v < 0.0 || __builtin_isinf(v)) bad = true;
        if (v > 0.0) {
            sum += v;
            mx = fmax(mx, v);
        }
    }
    RowInfo ri;
    // every lane holds the same sums and maxima (the butterflies add the same
    // pairs in every lane); the first lane's are taken as wave-uniform values
    ri.sum = uni_f64(wave_sum(sum));
    mx = uni_f64(wave_max(mx));
    if (wave_any(bad)) ri.status = kSetInvalid;
    else if (!(mx > 0.0)) ri.status = kSetEmpty;
    else if (mx > 0x1.0p768 || mx < 0x1.0p-768) ri.status = kSetRange;
    else ri.status = kSetOk;
    return ri;
}

}  // namespace dms
