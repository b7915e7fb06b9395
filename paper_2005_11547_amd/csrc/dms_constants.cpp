// Host-side constants of the DartMinHash specification: the dart budget t(k),
// the six hash keys, the region corner tables and the Poisson(1) thresholds.
//
// t = ceil(k ln k) + k is the budget of Theorem 1; the region corners
// W[nu] = (2^nu - 1)/t and R[rho] = 2^rho - 1 come from Section 2 ("Poisson
// darts"); the Poisson CDF table is the one the paper precomputes (Section 4,
// "Implementation").
#include "dms_internal.h"

#include <cmath>
#include <cstring>
#include <random>

namespace dms {

// ---------------------------------------------------------------------------
// t(k) = ceil(k ln k) + k.  For integer k >= 2, k ln k is irrational, so the
// ceiling is floor + 1; long double keeps about 19 significant digits, which is
// far more than the distance of k ln k from the nearest integer for every
// supported k (checked against 60-digit arithmetic in the tests).
uint32_t t_of_k(int32_t k)
{
    if (k <= 1) return 1;
    long double v = (long double)k * logl((long double)k);
    long double f = floorl(v);
    return (uint32_t)f + 1u + (uint32_t)k;
}

// ---------------------------------------------------------------------------
// Fixed point numbers with 8 little-endian 32-bit limbs: limbs 0..5 are the
// fraction (192 bits), limbs 6..7 the integer part.  Used only to derive the
// Poisson thresholds exactly.
namespace {
struct Fx {
    uint32_t l[8];
};

Fx fx_int(uint32_t v)
{
    Fx a;
    std::memset(&a, 0, sizeof a);
    a.l[6] = v;
    return a;
}

void fx_div_small(Fx& a, uint32_t d)  // a = floor(a / d)
{
    uint64_t rem = 0;
    for (int i = 7; i >= 0; --i) {
        uint64_t cur = (rem << 32) | a.l[i];
        a.l[i] = (uint32_t)(cur / d);
        rem = cur % d;
    }
}

void fx_add(Fx& a, const Fx& b)
{
    uint64_t c = 0;
    for (int i = 0; i < 8; ++i) {
        uint64_t s = (uint64_t)a.l[i] + b.l[i] + c;
        a.l[i] = (uint32_t)s;
        c = s >> 32;
    }
}

void fx_sub(Fx& a, const Fx& b)  // requires a >= b
{
    int64_t br = 0;
    for (int i = 0; i < 8; ++i) {
        int64_t s = (int64_t)a.l[i] - (int64_t)b.l[i] - br;
        br = s < 0;
        a.l[i] = (uint32_t)(s + (br ? (int64_t)1 << 32 : 0));
    }
}

Fx fx_mul(const Fx& a, const Fx& b)  // truncated product
{
    uint32_t p[16];
    std::memset(p, 0, sizeof p);
    for (int i = 0; i < 8; ++i) {
        uint64_t c = 0;
        for (int j = 0; j < 8; ++j) {
            uint64_t cur = (uint64_t)a.l[i] * b.l[j] + p[i + j] + c;
            p[i + j] = (uint32_t)cur;
            c = cur >> 32;
        }
        for (int m = i + 8; c && m < 16; ++m) {
            uint64_t cur = (uint64_t)p[m] + c;
            p[m] = (uint32_t)cur;
            c = cur >> 32;
        }
    }
    Fx r;
    for (int i = 0; i < 8; ++i) r.l[i] = p[i + 6];
    return r;
}

// floor(2^64 * a) when a < 1: the two fraction limbs right below the point.
// Returns false if a is within `slack` units of the last place of a multiple of
// 2^-64 (then the floor would not be certain).
bool fx_floor_2_64(const Fx& a, uint64_t slack, uint64_t* out)
{
    if (a.l[6] || a.l[7]) {
        // a >= 1 cannot happen for a CDF value below 1
        return false;
    }
    uint64_t hi = ((uint64_t)a.l[5] << 32) | a.l[4];
    // remaining 128 fraction bits, limbs 3..0, as a distance from both ends
    uint64_t lo_top = ((uint64_t)a.l[3] << 32) | a.l[2];
    uint64_t lo_bot = ((uint64_t)a.l[1] << 32) | a.l[0];
    bool near_low = lo_top == 0 && lo_bot <= slack;
    bool near_high = lo_top == ~0ULL && lo_bot >= ~0ULL - slack;
    if (near_low || near_high) return false;
    *out = hi;
    return true;
}
}  // namespace

// C[n] = floor(2^64 * e^-1 * sum_{m<=n} 1/m!) for n = 0..19.
bool poisson_thresholds(uint64_t out[kNumPoisson])
{
    // e^-1 = sum_m (-1)^m / m!, 40 terms: truncation error below 2^-150,
    // rounding error at most 40 units of 2^-192.
    Fx einv = fx_int(0), term = fx_int(1);
    fx_add(einv, term);
    for (uint32_t m = 1; m <= 40; ++m) {
        fx_div_small(term, m);
        if (m & 1) fx_sub(einv, term);
        else fx_add(einv, term);
    }
    Fx partial = fx_int(0);
    term = fx_int(1);
    for (int n = 0; n < kNumPoisson; ++n) {
        if (n > 0) fx_div_small(term, (uint32_t)n);
        fx_add(partial, term);
        Fx cdf = fx_mul(einv, partial);
        // total error far below 2^-140: refuse only if the value sits that close
        // to a multiple of 2^-64 (it does not, for any n < 20)
        if (!fx_floor_2_64(cdf, ~0ULL >> 8, &out[n])) return false;
    }
    return true;
}

double corner_w(const SpecTables& sp, int nu) { return nu < kTable ? sp.W[nu] : std::ldexp(sp.u, nu); }
double corner_r(const SpecTables& sp, int rho) { return rho < kTable ? sp.R[rho] : std::ldexp(1.0, rho); }

void hash_keys(uint64_t seed, uint64_t keys[6])
{
    std::mt19937_64 gen(seed);
    for (int i = 0; i < 6; ++i) keys[i] = gen();
}

void hash_tables(uint64_t seed, uint64_t tab[kTabWords])
{
    std::mt19937_64 gen(seed);
    for (int i = 0; i < 6; ++i) (void)gen();  // the keys come first
    for (int i = 0; i < kTabWords; ++i) tab[i] = gen();
}

bool make_spec(uint64_t seed, uint32_t t, SpecTables* sp)
{
    std::memset(sp, 0, sizeof *sp);
    uint64_t keys[6];
    hash_keys(seed, keys);
    hash_tables(seed, sp->tab);
    sp->key_r = keys[0];
    sp->key_a = keys[1];
    sp->key_u = keys[2];
    sp->key_v = keys[3];
    sp->key_s = keys[4];
    sp->key_l = keys[5];
    if (!poisson_thresholds(sp->pois)) return false;
    const double td = (double)t;
    for (int i = 0; i < kTable; ++i) {
        double p = std::ldexp(1.0, i);  // 2^i exactly
        double pm1 = p - 1.0;            // RN(2^i - 1)
        sp->W[i] = pm1 / td;
        sp->R[i] = pm1;
    }
    sp->u = 1.0 / td;
    sp->t = t;
    return true;
}

}  // namespace dms
