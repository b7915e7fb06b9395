/*
 * DartMinHash CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded, deliberately unoptimised implementation of the
 * DartHash enumeration (Algorithm 1, Section 2), DartMinHash (Theorem 1,
 * Section 3) and the (L,K) LSH values (Section 3, "Bottom-k minhash and fast
 * approximate near neighbor search").  It exists so that tests, the smoke
 * check and the CPU baseline can check the HIP library against it.  Nothing
 * in the product path may call, link or load this file.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
 * Every floating point `+` and `*` below is one IEEE binary64 operation with
 * round-to-nearest-even; no contraction into fused multiply-adds.
 *
 * All constants (hash keys, tables, Poisson thresholds, t) are supplied by the
 * caller in `dmso_params`; oracle/oracle.py derives them from their
 * mathematical definitions.
 *
 * Hash family (the paper assumes a fully random hash, Theorem 1, and uses
 * tabulation hashing in its experiments, Section 4 "Implementation"): the
 * 64-bit finaliser of SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), keyed by
 * six 64-bit keys drawn from MT19937-64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DMSO_TABLE 1024
#define DMSO_NPOIS 20

enum { DMSO_OK = 0, DMSO_EMPTY = 1, DMSO_RANGE = 2, DMSO_INVALID = 3, DMSO_NOMEM = 4 };
enum { DMSO_SCHED_PLUS_ONE = 0, DMSO_SCHED_DOUBLE = 1 };

typedef struct {
    uint64_t key_r, key_a, key_u, key_v, key_s, key_l;
    uint64_t pois[DMSO_NPOIS]; /* floor(2^64 * P[Poi(1) <= n]) */
    double W[DMSO_TABLE];      /* W[nu]  = RN(RN(2^nu - 1) / t)   */
    double R[DMSO_TABLE];      /* R[rho] = RN(2^rho - 1)          */
    double u;                  /* RN(1/t)                          */
    uint32_t t;
    double phi0;               /* first value of phi               */
    int32_t schedule;          /* DMSO_SCHED_*                     */
    double phi_max;            /* give up (status RANGE) beyond this */
    int32_t hash;              /* DMSO_HASH_*                      */
    uint64_t tab[8 * 256];     /* tabulation tables (DMSO_HASH_TAB) */
    int32_t validate;          /* 1: a row listing an id twice is INVALID */
} dmso_params;

enum { DMSO_HASH_MIX = 0, DMSO_HASH_TAB = 1 };

typedef struct {
    uint32_t i;     /* element id                        */
    uint16_t nu;    /* weight region                     */
    uint16_t rho;   /* rank region                       */
    uint32_t w;     /* weight subdivision in the region  */
    uint32_t r;     /* rank subdivision in the region    */
    uint32_t j;     /* dart number inside the area       */
    uint32_t pad;
    double rank;
    double weight;
    uint64_t s;     /* dart id hash                      */
} dmso_dart;

/* Enumeration counts of DartHash passes: regions and areas visited, darts
 * generated, darts with rank <= tau, darts accepted (rank <= tau and weight <=
 * x_i); rank_new and accepted_new count the last two restricted to ranks above
 * the previous pass's tau (every dart of the first pass is new).  A retry that
 * only inserts darts it has not met before needs exactly the new ones. */
typedef struct {
    int64_t regions, areas, generated, rank_pass, accepted, rank_new, accepted_new;
} dmso_counters;

/* SplitMix64 output function (bijective 64 -> 64 bit mixer). */
static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t dmso_mix64(uint64_t z) { return mix64(z); }

/* Simple tabulation hashing (the paper's randomness source, Section 4): the
 * XOR of one table word per byte of z, tables filled by the Mersenne Twister. */
static uint64_t tab64(const uint64_t* tab, uint64_t z)
{
    uint64_t h = 0;
    for (int b = 0; b < 8; b++) h ^= tab[b * 256 + ((z >> (8 * b)) & 0xFF)];
    return h;
}

/* The hash function of every hashing step of the specification. */
static uint64_t H(const dmso_params* P, uint64_t z)
{
    return P->hash == DMSO_HASH_TAB ? tab64(P->tab, z) : mix64(z);
}

/* 53 high bits of a hash as a uniform double in [0,1). */
static double unit53(uint64_t h)
{
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* Number of Poisson(1) darts in an area, from its 64-bit hash a:
 * X = min{ n : a < pois[n] }, or 20 when a is above every threshold. */
static uint32_t poisson_count(const dmso_params* P, uint64_t a)
{
    uint32_t n = 0;
    while (n < DMSO_NPOIS && a >= P->pois[n]) n++;
    return n;
}

/* Growable dart list. */
typedef struct {
    dmso_dart* d;
    int64_t n, cap;
} dart_list;

static int push_dart(dart_list* L, const dmso_dart* x)
{
    if (L->n == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 1024;
        dmso_dart* nd = (dmso_dart*)realloc(L->d, (size_t)nc * sizeof(dmso_dart));
        if (!nd) return -1;
        L->d = nd;
        L->cap = nc;
    }
    L->d[L->n++] = *x;
    return 0;
}

/*
 * DartHash_t(x, phi) (Algorithm 1).  Appends to `out` every dart of the hashed
 * Poisson process with rank <= tau = phi/||x||_1 and weight <= x_i.  The loop
 * order is the algorithm's: element, nu, rho, w, r, j.  The nu and rho loops
 * stop at the first region whose lower corner lies beyond x_i, respectively
 * tau; for real numbers this is the same as the algorithm's bounds
 * floor(log2(1+t x_i)) and floor(log2(1+phi/||x||_1)).
 *
 * Region (nu,rho) covers weights [(2^nu-1)/t, (2^(nu+1)-1)/t) and ranks
 * [2^rho-1, 2^(rho+1)-1) (Section 2, "Poisson darts"); it is split into 2^rho
 * weight columns of width delta_nu = 2^nu/(t 2^rho) and 2^nu rank rows of
 * height delta_rho = 2^rho/2^nu, so every area has size 1/t and holds
 * Poisson(1) darts.
 *
 * tau_prev only steers the rank_new / accepted_new counts (the previous
 * pass's tau; below every rank on a first pass).
 *
 * Returns DMSO_OK, DMSO_RANGE (a subdivision index or table index out of the
 * supported range) or DMSO_NOMEM.
 */
static int darthash(const dmso_params* P, int64_t nnz, const int32_t* idx,
                    const double* x, double tau, double tau_prev, dart_list* out,
                    dmso_counters* cnt)
{
    for (int64_t e = 0; e < nnz; e++) {
        double xi = x[e];
        if (!(xi > 0.0)) continue;               /* only i with x_i > 0 */
        uint32_t id = (uint32_t)idx[e];
        for (int nu = 0; P->W[nu] <= xi; nu++) {
            if (nu + 1 >= DMSO_TABLE) return DMSO_RANGE;
            for (int rho = 0; P->R[rho] <= tau; rho++) {
                if (rho + 1 >= DMSO_TABLE) return DMSO_RANGE;
                double Wn = P->W[nu];
                double Rr = P->R[rho];
                double dnu = ldexp(P->u, nu - rho);   /* 2^nu / (t 2^rho) */
                double drho = ldexp(1.0, rho - nu);   /* 2^rho / 2^nu     */
                uint64_t g = H(P, P->key_r ^ (((uint64_t)id << 32) |
                                               ((uint64_t)nu << 16) | (uint64_t)rho));
                cnt->regions++;
                double wmax = ldexp(1.0, rho); /* w runs over 0 .. 2^rho - 1 */
                for (double wd = 0.0; wd < wmax; wd += 1.0) {
                    if (xi < Wn + wd * dnu) break;
                    if (wd >= 4294967296.0) return DMSO_RANGE;
                    double rmax = ldexp(1.0, nu); /* r runs over 0 .. 2^nu - 1 */
                    for (double rd = 0.0; rd < rmax; rd += 1.0) {
                        if (tau < Rr + rd * drho) break;
                        if (rd >= 4294967296.0) return DMSO_RANGE;
                        uint32_t w = (uint32_t)wd, r = (uint32_t)rd;
                        uint64_t a = H(P, g ^ P->key_a ^ (((uint64_t)w << 32) | (uint64_t)r));
                        uint32_t X = poisson_count(P, a);
                        cnt->areas++;
                        for (uint32_t j = 0; j < X; j++) {
                            double U = unit53(H(P, a ^ P->key_u ^ (uint64_t)j));
                            double V = unit53(H(P, a ^ P->key_v ^ (uint64_t)j));
                            double weight = Wn + (wd + V) * dnu;
                            double rank = Rr + (rd + U) * drho;
                            cnt->generated++;
                            if (rank <= tau) cnt->rank_pass++;
                            if (rank <= tau && rank > tau_prev) cnt->rank_new++;
                            if (weight <= xi && rank <= tau) {
                                if (rank > tau_prev) cnt->accepted_new++;
                                dmso_dart D;
                                D.i = id; D.nu = (uint16_t)nu; D.rho = (uint16_t)rho;
                                D.w = w; D.r = r; D.j = j; D.pad = 0;
                                D.rank = rank; D.weight = weight;
                                D.s = H(P, a ^ P->key_s ^ (uint64_t)j);
                                cnt->accepted++;
                                if (push_dart(out, &D)) return DMSO_NOMEM;
                            }
                        }
                    }
                }
            }
        }
    }
    return DMSO_OK;
}

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : x > y;
}

/* 1 if some id occurs twice in the row (ids compared as uint32), else 0;
 * -1 when out of memory. */
static int has_repeat(int64_t nnz, const int32_t* idx)
{
    if (nnz < 2) return 0;
    uint32_t* c = (uint32_t*)malloc((size_t)nnz * sizeof(uint32_t));
    if (!c) return -1;
    for (int64_t e = 0; e < nnz; e++) c[e] = (uint32_t)idx[e];
    qsort(c, (size_t)nnz, sizeof(uint32_t), cmp_u32);
    int rep = 0;
    for (int64_t e = 1; e < nnz && !rep; e++) rep = c[e] == c[e - 1];
    free(c);
    return rep;
}

/* Validate a row: DMSO_INVALID for a negative, NaN or infinite weight (and,
 * when P->validate is set, for an id listed twice), DMSO_EMPTY when no weight
 * is positive, DMSO_RANGE when the largest weight is outside [2^-768, 2^768].
 * On success *S is the sum of the positive weights in row order. */
static int check_row(const dmso_params* P, int64_t nnz, const int32_t* idx, const double* x, double* S)
{
    if (P->validate) {
        int r = has_repeat(nnz, idx);
        if (r < 0) return DMSO_NOMEM;
        if (r) return DMSO_INVALID;
    }
    double sum = 0.0, mx = 0.0;
    int any = 0;
    for (int64_t e = 0; e < nnz; e++) {
        double v = x[e];
        if (isnan(v) || v < 0.0 || isinf(v)) return DMSO_INVALID;
        if (v > 0.0) {
            any = 1;
            sum += v;
            if (v > mx) mx = v;
        }
    }
    if (!any) return DMSO_EMPTY;
    if (mx > ldexp(1.0, 768) || mx < ldexp(1.0, -768)) return DMSO_RANGE;
    *S = sum;
    return DMSO_OK;
}

static double next_phi(const dmso_params* P, double phi)
{
    return P->schedule == DMSO_SCHED_DOUBLE ? 2.0 * phi : phi + 1.0;
}

/* Lexicographic order on (rank, s). */
static int dart_less(double ra, uint64_t sa, double rb, uint64_t sb)
{
    return ra < rb || (ra == rb && sa < sb);
}

/*
 * Public: DartHash_t(x, phi) for one set with an explicit tau.  Writes up to
 * `cap` darts, returns the status and stores the full dart count in *n_out.
 */
int dmso_darthash(const dmso_params* P, int64_t nnz, const int32_t* idx, const double* x,
                  double tau, dmso_dart* out, int64_t cap, int64_t* n_out, dmso_counters* cnt)
{
    dart_list L = {0, 0, 0};
    dmso_counters c;
    memset(&c, 0, sizeof c);
    int st = darthash(P, nnz, idx, x, tau, -1.0, &L, &c);
    int64_t n = L.n < cap ? L.n : cap;
    if (out && n > 0) memcpy(out, L.d, (size_t)n * sizeof(dmso_dart));
    *n_out = L.n;
    if (cnt) *cnt = c;
    free(L.d);
    return st;
}

/*
 * Enumeration counts of a schedule: cnt[0] sums every DartHash pass, cnt[1]
 * keeps the last pass only (the work of one pass at the final phi).  cnt may
 * be NULL.
 */
static void count_pass(dmso_counters* cnt, const dmso_counters* c)
{
    if (!cnt) return;
    cnt[0].regions += c->regions;
    cnt[0].areas += c->areas;
    cnt[0].generated += c->generated;
    cnt[0].rank_pass += c->rank_pass;
    cnt[0].accepted += c->accepted;
    cnt[0].rank_new += c->rank_new;
    cnt[0].accepted_new += c->accepted_new;
    cnt[1] = *c;
}

/*
 * DartMinHash for one set (Theorem 1): run DartHash_t(x, phi) for phi = phi0,
 * then the schedule's next values, hash every returned dart to one of k
 * buckets by b = (hi32(s) * k) >> 32, stop once no bucket is empty.  Bucket j's
 * minhash is its dart of smallest rank (ties broken by the smaller id hash s).
 * On success writes out_s[j], out_rank[j] for j < k and *phi_final.  cnt, if
 * not NULL, points at two counters: every pass summed, and the last pass.
 */
int dmso_minhash_set(const dmso_params* P, int32_t k, int64_t nnz, const int32_t* idx,
                     const double* x, uint64_t* out_s, double* out_rank, double* phi_final,
                     dmso_counters* cnt)
{
    double S;
    int st = check_row(P, nnz, idx, x, &S);
    if (st != DMSO_OK) return st;
    int filled = 0;
    double phi = P->phi0, tau_prev = -1.0;
    uint8_t* have = (uint8_t*)malloc((size_t)k);
    if (!have) return DMSO_NOMEM;
    for (;;) {
        if (phi > P->phi_max) { st = DMSO_RANGE; break; }
        double tau = phi / S;
        dart_list L = {0, 0, 0};
        dmso_counters c;
        memset(&c, 0, sizeof c);
        st = darthash(P, nnz, idx, x, tau, tau_prev, &L, &c);
        tau_prev = tau;
        count_pass(cnt, &c);
        if (st != DMSO_OK) { free(L.d); break; }
        memset(have, 0, (size_t)k);
        for (int64_t n = 0; n < L.n; n++) {
            const dmso_dart* D = &L.d[n];
            uint32_t b = (uint32_t)(((D->s >> 32) * (uint64_t)k) >> 32);
            if (!have[b] || dart_less(D->rank, D->s, out_rank[b], out_s[b])) {
                out_rank[b] = D->rank;
                out_s[b] = D->s;
                have[b] = 1;
            }
        }
        free(L.d);
        filled = 1;
        for (int32_t b = 0; b < k; b++) if (!have[b]) { filled = 0; break; }
        if (filled) { *phi_final = phi; break; }
        phi = next_phi(P, phi);
    }
    free(have);
    return st;
}

/*
 * Batched DartMinHash over a CSR matrix.  Sets with a non-OK status get
 * minhash 0xFFFFFFFF and all-zero bits.  Any output pointer may be NULL;
 * out_cnt holds two counters per set (every pass summed, the last pass).
 * out_u32[s*k + j] = low 32 bits of bucket j's dart hash; bit j of set s is
 * bit 0 of that hash, stored at bit (j mod 64) of word s*ceil(k/64) + j/64.
 */
int dmso_sketch_csr(const dmso_params* P, int64_t n_sets, const int64_t* row_ptr,
                    const int32_t* idx, const double* x, int32_t k, uint32_t* out_u32,
                    uint64_t* out_bits, int8_t* out_status, uint64_t* out_s, double* out_rank,
                    double* out_phi, dmso_counters* out_cnt)
{
    uint64_t* s = (uint64_t*)malloc((size_t)k * sizeof(uint64_t));
    double* rk = (double*)malloc((size_t)k * sizeof(double));
    if (!s || !rk) { free(s); free(rk); return DMSO_NOMEM; }
    int64_t words = (k + 63) / 64;
    for (int64_t q = 0; q < n_sets; q++) {
        int64_t b0 = row_ptr[q], b1 = row_ptr[q + 1];
        double phi = 0.0;
        dmso_counters c[2];
        memset(c, 0, sizeof c);
        int st = dmso_minhash_set(P, k, b1 - b0, idx + b0, x + b0, s, rk, &phi, c);
        if (st == DMSO_NOMEM) { free(s); free(rk); return DMSO_NOMEM; }
        if (out_status) out_status[q] = (int8_t)st;
        if (out_phi) out_phi[q] = st == DMSO_OK ? phi : 0.0;
        if (out_cnt) { out_cnt[2 * q] = c[0]; out_cnt[2 * q + 1] = c[1]; }
        for (int32_t j = 0; j < k; j++) {
            if (out_u32) out_u32[q * k + j] = st == DMSO_OK ? (uint32_t)s[j] : 0xFFFFFFFFu;
            if (out_s) out_s[q * k + j] = st == DMSO_OK ? s[j] : ~0ULL;
            if (out_rank) out_rank[q * k + j] = st == DMSO_OK ? rk[j] : INFINITY;
        }
        if (out_bits) {
            for (int64_t wd = 0; wd < words; wd++) out_bits[q * words + wd] = 0;
            if (st == DMSO_OK)
                for (int32_t j = 0; j < k; j++)
                    out_bits[q * words + j / 64] |= (s[j] & 1ULL) << (j % 64);
        }
    }
    free(s);
    free(rk);
    return DMSO_OK;
}

/*
 * (L,K) LSH values for one set (Section 3): DartHash with t = L*K, darts hashed
 * to L tables by l = (hi32(s) * L) >> 32, each table keeps its K darts of
 * smallest (rank, s) in ascending order, phi grows until every table holds at
 * least K darts.  A dart met twice (a repeated element id) counts once.
 * Table l's key folds the ordered dart ids: h = mix(key_l ^ l), then
 * h = mix(h ^ s_m) for m = 0..K-1.
 */
int dmso_lsh_set(const dmso_params* P, int32_t L, int32_t K, int64_t nnz, const int32_t* idx,
                 const double* x, uint64_t* out_keys, uint64_t* out_s, double* out_rank,
                 double* phi_final, dmso_counters* pass_cnt)
{
    double S;
    int st = check_row(P, nnz, idx, x, &S);
    if (st != DMSO_OK) return st;
    size_t slots = (size_t)L * (size_t)K;
    uint64_t* bs = (uint64_t*)malloc(slots * sizeof(uint64_t));
    double* br = (double*)malloc(slots * sizeof(double));
    int32_t* cnt = (int32_t*)malloc((size_t)L * sizeof(int32_t));
    if (!bs || !br || !cnt) { free(bs); free(br); free(cnt); return DMSO_NOMEM; }
    double phi = P->phi0, tau_prev = -1.0;
    for (;;) {
        if (phi > P->phi_max) { st = DMSO_RANGE; break; }
        double tau = phi / S;
        dart_list D = {0, 0, 0};
        dmso_counters c;
        memset(&c, 0, sizeof c);
        st = darthash(P, nnz, idx, x, tau, tau_prev, &D, &c);
        tau_prev = tau;
        count_pass(pass_cnt, &c);
        if (st != DMSO_OK) { free(D.d); break; }
        for (int32_t l = 0; l < L; l++) cnt[l] = 0;
        for (int64_t n = 0; n < D.n; n++) {
            const dmso_dart* d = &D.d[n];
            uint32_t l = (uint32_t)(((d->s >> 32) * (uint64_t)L) >> 32);
            double* r = br + (size_t)l * K;
            uint64_t* s = bs + (size_t)l * K;
            int32_t c0 = cnt[l];
            int dup = 0;
            for (int32_t m = 0; m < c0; m++)
                if (r[m] == d->rank && s[m] == d->s) { dup = 1; break; }
            if (dup) continue;
            /* insertion into the sorted list of at most K entries */
            int32_t pos = c0;
            while (pos > 0 && dart_less(d->rank, d->s, r[pos - 1], s[pos - 1])) pos--;
            if (pos >= K) continue;
            int32_t last = c0 < K ? c0 : K - 1;
            for (int32_t m = last; m > pos; m--) { r[m] = r[m - 1]; s[m] = s[m - 1]; }
            r[pos] = d->rank;
            s[pos] = d->s;
            if (c0 < K) cnt[l] = c0 + 1;
        }
        free(D.d);
        int full = 1;
        for (int32_t l = 0; l < L; l++) if (cnt[l] < K) { full = 0; break; }
        if (full) { *phi_final = phi; break; }
        phi = next_phi(P, phi);
    }
    if (st == DMSO_OK) {
        for (int32_t l = 0; l < L; l++) {
            uint64_t h = H(P, P->key_l ^ (uint64_t)l);
            for (int32_t m = 0; m < K; m++) h = H(P, h ^ bs[(size_t)l * K + m]);
            out_keys[l] = h;
        }
        if (out_s) memcpy(out_s, bs, slots * sizeof(uint64_t));
        if (out_rank) memcpy(out_rank, br, slots * sizeof(double));
    }
    free(bs);
    free(br);
    free(cnt);
    return st;
}

/* Batched LSH keys over a CSR matrix; non-OK sets get all-zero keys. */
int dmso_lsh_csr(const dmso_params* P, int64_t n_sets, const int64_t* row_ptr,
                 const int32_t* idx, const double* x, int32_t L, int32_t K,
                 uint64_t* out_keys, int8_t* out_status, dmso_counters* out_cnt)
{
    for (int64_t q = 0; q < n_sets; q++) {
        int64_t b0 = row_ptr[q], b1 = row_ptr[q + 1];
        double phi = 0.0;
        dmso_counters c[2];
        memset(c, 0, sizeof c);
        int st = dmso_lsh_set(P, L, K, b1 - b0, idx + b0, x + b0, out_keys + q * L, NULL, NULL, &phi, c);
        if (out_cnt) { out_cnt[2 * q] = c[0]; out_cnt[2 * q + 1] = c[1]; }
        if (st == DMSO_NOMEM) return DMSO_NOMEM;
        if (out_status) out_status[q] = (int8_t)st;
        if (st != DMSO_OK)
            for (int32_t l = 0; l < L; l++) out_keys[q * L + l] = 0;
    }
    return DMSO_OK;
}

/* qsort order of darts: (rank, id hash) ascending. */
static int cmp_dart(const void* pa, const void* pb)
{
    const dmso_dart* a = (const dmso_dart*)pa;
    const dmso_dart* b = (const dmso_dart*)pb;
    if (dart_less(a->rank, a->s, b->rank, b->s)) return -1;
    if (dart_less(b->rank, b->s, a->rank, a->s)) return 1;
    return 0;
}

/*
 * Bottom-k sketch for one set (Section 3, bottom-k minhash): DartHash_t with
 * t = k (the caller passes P->t = k), phi following the schedule until the
 * darts of rank <= tau hold at least k distinct ones; the sketch is the k
 * smallest by (rank, id hash), ascending.  A dart met twice (a repeated
 * element id) counts once.
 */
int dmso_bottomk_set(const dmso_params* P, int32_t k, int64_t nnz, const int32_t* idx,
                     const double* x, uint64_t* out_s, double* out_rank, double* phi_final,
                     dmso_counters* cnt)
{
    double S;
    int st = check_row(P, nnz, idx, x, &S);
    if (st != DMSO_OK) return st;
    double phi = P->phi0, tau_prev = -1.0;
    for (;;) {
        if (phi > P->phi_max) return DMSO_RANGE;
        dart_list L = {0, 0, 0};
        dmso_counters c;
        memset(&c, 0, sizeof c);
        st = darthash(P, nnz, idx, x, phi / S, tau_prev, &L, &c);
        tau_prev = phi / S;
        count_pass(cnt, &c);
        if (st != DMSO_OK) { free(L.d); return st; }
        if (L.n > 1) qsort(L.d, (size_t)L.n, sizeof(dmso_dart), cmp_dart);
        int64_t distinct = 0;
        for (int64_t n = 0; n < L.n; n++) {
            if (distinct > 0 && L.d[n].rank == L.d[distinct - 1].rank && L.d[n].s == L.d[distinct - 1].s)
                continue;
            L.d[distinct++] = L.d[n];
        }
        if (distinct >= k) {
            for (int32_t m = 0; m < k; m++) {
                out_s[m] = L.d[m].s;
                out_rank[m] = L.d[m].rank;
            }
            *phi_final = phi;
            free(L.d);
            return DMSO_OK;
        }
        free(L.d);
        phi = next_phi(P, phi);
    }
}

/* Batched bottom-k sketches; non-OK sets get s = ~0 and rank = +inf. */
int dmso_bottomk_csr(const dmso_params* P, int64_t n_sets, const int64_t* row_ptr,
                     const int32_t* idx, const double* x, int32_t k, uint64_t* out_s,
                     double* out_rank, int8_t* out_status, dmso_counters* out_cnt)
{
    for (int64_t q = 0; q < n_sets; q++) {
        int64_t b0 = row_ptr[q], b1 = row_ptr[q + 1];
        double phi = 0.0;
        dmso_counters c[2];
        memset(c, 0, sizeof c);
        int st = dmso_bottomk_set(P, k, b1 - b0, idx + b0, x + b0, out_s + q * k, out_rank + q * k, &phi, c);
        if (out_cnt) { out_cnt[2 * q] = c[0]; out_cnt[2 * q + 1] = c[1]; }
        if (st == DMSO_NOMEM) return DMSO_NOMEM;
        if (out_status) out_status[q] = (int8_t)st;
        if (st != DMSO_OK)
            for (int32_t m = 0; m < k; m++) {
                out_s[q * k + m] = ~0ULL;
                out_rank[q * k + m] = INFINITY;
            }
    }
    return DMSO_OK;
}
