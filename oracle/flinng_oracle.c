/*
 * FLINNG CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what FLINNG's batched
 * query path computes ("Practical Near Neighbor Search via Group Testing",
 * Engels, Coleman, Shrivastava, 2021). Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load this library. It shares no code,
 * header, table or constant generator with the HIP library; both sides
 * implement the same written hashing specification independently.
 *
 * Floating point is FP64 throughout; every SRP sign is the sign of the exact
 * real dot product (certified FP64 sum, else an exact expansion sum).
 *
 * Parity pins: every function here is pinned by tests/test_oracle_*.py against
 * closed forms, invariants, brute force or statistics; see the header comment
 * of each function for the passage it follows.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Counter-based generator: the output function of SplitMix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014),
 * applied to the state seed + (i+1)*golden gamma.  sm64(s, i) is the i-th
 * output of a SplitMix64 generator started at state s.                      */
static uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t or_sm64(uint64_t s, uint64_t i)
{
    return or_mix64(s + (i + 1ULL) * 0x9E3779B97F4A7C15ULL);
}

uint64_t or_mix64_public(uint64_t z) { return or_mix64(z); }

/* Stream tags: each random object the method draws has its own key. */
enum { OR_TAG_HYP = 1, OR_TAG_MINHASH = 2, OR_TAG_GROUP = 3 };

static uint64_t or_stream(uint64_t seed, uint64_t tag) { return or_sm64(seed, tag); }

/* ------------------------------------------------------------------------- */
/* Signed random projections (the dense LSH of the method's hashing layer,
 * Section 3 "Locality-Sensitive Hashing" and the concatenation trick).
 * Hyperplane h (h = t*K + j: bit j of table t) has entries
 *   w[h][i] = (popcount(sm64(key_HYP, h*d + i)) - 32) / 4,
 * a centred Binomial(64, 1/2)/4 value in {-8, -7.75, ..., 8}: exact in bf16. */
double or_hyperplane_entry(uint64_t seed, uint64_t h, uint32_t d, uint32_t i)
{
    uint64_t v = or_sm64(or_stream(seed, OR_TAG_HYP), h * (uint64_t)d + i);
    return ((double)__builtin_popcountll(v) - 32.0) / 4.0;
}

void or_hyperplanes(uint64_t seed, uint32_t H, uint32_t d, double *w)
{
    for (uint64_t h = 0; h < H; ++h)
        for (uint32_t i = 0; i < d; ++i)
            w[h * d + i] = or_hyperplane_entry(seed, h, d, i);
}

/* Exact sign of sum_i x[i]*w[i] by Shewchuk's Grow-Expansion with zero
 * elimination (J. R. Shewchuk, "Adaptive Precision Floating-Point Arithmetic
 * and Fast Robust Geometric Predicates", 1997).  Each product is exact in
 * FP64 (at most 24 x 6 significant bits), Two-Sum keeps every partial sum
 * exact, and the sign of a nonoverlapping expansion is the sign of its most
 * significant nonzero component.  Returns -1, 0 or +1.                      */
static int or_exact_sign(const double *x, const double *w, uint32_t d, double *e)
{
    int m = 0;
    for (uint32_t i = 0; i < d; ++i) {
        double q = x[i] * w[i];
        if (q == 0.0) continue;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double s = q + e[j];
            double bv = s - q;
            double av = s - bv;
            double br = e[j] - bv;
            double ar = q - av;
            double err = ar + br;
            q = s;
            if (err != 0.0) e[k++] = err;
        }
        if (q != 0.0) e[k++] = q;
        m = k;
    }
    if (m == 0) return 0;
    return e[m - 1] > 0.0 ? 1 : -1;
}

/* SRP bucket codes: bit j of table t is 1 iff the exact dot product of x with
 * hyperplane t*K+j is > 0 (an exact zero gives 0); the table's bucket is
 * sum_j bit_j 2^j (concatenation of K one-bit hashes).
 * The FP64 recursive sum v is certified when |v| > 2*d*2^-53 * sum|x_i w_i|
 * (the standard recursive-summation bound, doubled for the rounding of the
 * absolute sum itself); otherwise the exact expansion decides.
 * x: n*d row-major FP64 values (exact copies of the stored fp32/bf16 data).
 * codes: n*L row-major.  Returns the number of pairs that needed the exact
 * path (for reporting).                                                     */
uint64_t or_srp_codes(const double *x, uint64_t n, uint32_t d, const double *w,
                      uint32_t K, uint32_t L, uint32_t *codes)
{
    uint64_t n_exact = 0;
#pragma omp parallel for reduction(+ : n_exact) schedule(dynamic, 16)
    for (uint64_t r = 0; r < n; ++r) {
        double *ebuf = (double *)malloc(((size_t)d + 2) * sizeof(double));
        const double *xr = x + r * d;
        for (uint32_t t = 0; t < L; ++t) {
            uint32_t code = 0;
            for (uint32_t j = 0; j < K; ++j) {
                const double *wh = w + (uint64_t)(t * K + j) * d;
                double v = 0.0, a = 0.0;
                for (uint32_t i = 0; i < d; ++i) {
                    double p = xr[i] * wh[i];
                    v += p;
                    a += fabs(p);
                }
                int sgn;
                double bound = 2.0 * (double)d * 0x1p-53 * a;
                if (fabs(v) > bound) {
                    sgn = v > 0.0 ? 1 : -1;
                } else {
                    sgn = or_exact_sign(xr, wh, d, ebuf);
                    n_exact += 1;
                }
                if (sgn > 0) code |= (1u << j);
            }
            codes[r * L + t] = code;
        }
        free(ebuf);
    }
    return n_exact;
}

/* Exact sign of one projection (exposed for the pin tests). */
int or_exact_dot_sign(const double *x, const double *w, uint32_t d)
{
    double *e = (double *)malloc(((size_t)d + 2) * sizeof(double));
    int s = or_exact_sign(x, w, d, e);
    free(e);
    return s;
}

/* ------------------------------------------------------------------------- */
/* MinHash for item sets (the set-similarity LSH instance; the paper hashes
 * genome n-gram sets with MinHash, Section 7, Experiments, "Datasets").
 *   a[t][j]  = sm64(key_MH, t*K + j)
 *   pi_tj(e) = mix64(e XOR a[t][j]) >> 32           (top 32 bits)
 *   mh_tj(S) = min over e in S of pi_tj(e)          (empty set: 0xFFFFFFFF)
 *   fold:    h = sm64(key_MH, L*K + t); for j < K: h = mix64(h XOR mh_tj(S))
 *   bucket_t = h >> (64 - b)                        (b = bucket bits, 1..32)
 * items: CSR (offsets[n+1] into items[]), values are 64-bit (32-bit items are
 * zero-extended by the caller).                                             */
void or_minhash_codes(const uint64_t *items, const uint64_t *offsets, uint64_t n,
                      uint64_t seed, uint32_t K, uint32_t L, uint32_t b,
                      uint32_t *codes)
{
    const uint64_t key = or_stream(seed, OR_TAG_MINHASH);
#pragma omp parallel for schedule(dynamic, 64)
    for (uint64_t s = 0; s < n; ++s) {
        for (uint32_t t = 0; t < L; ++t) {
            uint64_t h = or_sm64(key, (uint64_t)L * K + t);
            for (uint32_t j = 0; j < K; ++j) {
                uint64_t a = or_sm64(key, (uint64_t)t * K + j);
                uint32_t mn = 0xFFFFFFFFu;
                for (uint64_t p = offsets[s]; p < offsets[s + 1]; ++p) {
                    uint32_t v = (uint32_t)(or_mix64(items[p] ^ a) >> 32);
                    if (v < mn) mn = v;
                }
                h = or_mix64(h ^ (uint64_t)mn);
            }
            codes[s * L + t] = (uint32_t)(h >> (64 - b));
        }
    }
}

/* ------------------------------------------------------------------------- */
/* N-gram item sets of symbol sequences (the paper hashes genome reads and URLs
 * as n-gram sets, Section 7, "Datasets").  Sequence s is the set of its
 * windows of `gram` symbols; a window's value is its base-`radix` number
 * v = sum_i s[p+i] radix^(gram-1-i), and its item is MurmurHash3's 64-bit
 * finaliser of (v XOR key) (item_bits 64) or its 32-bit finaliser of
 * (low32(v) XOR low32(key)) (item_bits 32) (Austin Appleby, MurmurHash3,
 * public domain).  Sequences shorter than gram have no items.  Items are
 * returned as uint64 (32-bit ones zero-extended), CSR by sequence.         */
static uint64_t or_murmur64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xFF51AFD7ED558CCDULL;
    k ^= k >> 33;
    k *= 0xC4CEB9FE1A85EC53ULL;
    k ^= k >> 33;
    return k;
}

static uint32_t or_murmur32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6BU;
    h ^= h >> 13;
    h *= 0xC2B2AE35U;
    h ^= h >> 16;
    return h;
}

uint64_t or_text_items(const uint8_t *sym, const uint64_t *off, uint64_t n,
                       uint32_t gram, uint32_t radix, uint64_t key,
                       uint32_t item_bits, uint64_t *items, uint64_t *item_off)
{
    uint64_t m = 0;
    for (uint64_t s = 0; s < n; ++s) {
        item_off[s] = m;
        const uint64_t len = off[s + 1] - off[s];
        for (uint64_t p = 0; p + gram <= len; ++p) {
            uint64_t v = 0;
            for (uint32_t i = 0; i < gram; ++i)
                v = v * radix + sym[off[s] + p + i];
            items[m++] = item_bits == 64 ? or_murmur64(v ^ key)
                                         : (uint64_t)or_murmur32((uint32_t)v ^ (uint32_t)key);
        }
    }
    item_off[n] = m;
    return m;
}

/* ------------------------------------------------------------------------- */
/* Group assignment (Algorithm 1, Index Construction): in repetition r the
 * points are permuted by a random permutation P_r and point x joins group
 * P_r(x) mod B, so each group holds floor(N/B) or ceil(N/B) points.
 * P_r is a 4-round balanced Feistel network on [0, 2^nb) (nb = the smallest
 * even number >= 2 with 2^nb >= N) with round keys sm64(key_GROUP, 4r + i)
 * and round function F_i(v) = mix64(v XOR key_i) mod 2^(nb/2), restricted to
 * [0, N) by cycle walking (Black and Rogaway, "Ciphers with arbitrary finite
 * domains", 2002).  g: R x N, repetition-major.                              */
static uint32_t or_feistel_bits(uint64_t N)
{
    uint32_t nb = 2;
    while (nb < 64 && (1ULL << nb) < N) nb += 2;
    return nb;
}

static uint64_t or_feistel(uint64_t v, uint32_t half, const uint64_t *keys)
{
    const uint64_t mask = (1ULL << half) - 1ULL;
    uint64_t hi = v >> half, lo = v & mask;
    for (int i = 0; i < 4; ++i) {
        uint64_t nlo = hi ^ (or_mix64(lo ^ keys[i]) & mask);
        hi = lo;
        lo = nlo;
    }
    return (hi << half) | lo;
}

uint64_t or_permute(uint64_t N, uint32_t r, uint64_t seed, uint64_t x)
{
    const uint64_t key = or_stream(seed, OR_TAG_GROUP);
    uint64_t keys[4];
    for (int i = 0; i < 4; ++i) keys[i] = or_sm64(key, (uint64_t)r * 4 + i);
    const uint32_t half = or_feistel_bits(N) / 2;
    uint64_t y = or_feistel(x, half, keys);
    while (y >= N) y = or_feistel(y, half, keys);
    return y;
}

void or_groups(uint64_t N, uint32_t R, uint32_t B, uint64_t seed, uint32_t *g)
{
    for (uint32_t r = 0; r < R; ++r) {
#pragma omp parallel for schedule(static)
        for (uint64_t x = 0; x < N; ++x)
            g[(uint64_t)r * N + x] = (uint32_t)(or_permute(N, r, seed, x) % B);
    }
}

/* Groups of points that arrive after the index was built (reading: the
 * paper builds its index in one pass over the data, and Algorithm 1 needs
 * the final N for its permutation).  The arrivals after the first N0 points
 * are cut into blocks of B in arrival order; within block j the point at
 * position u joins group pi_{r,j}(u) of repetition r, where pi_{r,j} is a
 * 4-round balanced Feistel network on [0, 2^nb) (nb the smallest even width
 * >= 2 with 2^nb >= B) restricted to [0, B) by cycle walking, round keys
 * sm64(key_STREAM, 4 (16 j + r) + i).  Every complete block adds exactly one
 * point to each group of each repetition, so the group sizes stay within
 * two of each other; the repetitions use independent permutations.
 * g: R x n, repetition-major, for the points x0 .. x0+n-1 (x0 >= N0).     */
enum { OR_TAG_STREAM = 4 };

void or_stream_groups(uint64_t N0, uint32_t R, uint32_t B, uint64_t seed,
                      uint64_t x0, uint64_t n, uint32_t *g)
{
    const uint64_t key = or_stream(seed, OR_TAG_STREAM);
    const uint32_t half = or_feistel_bits(B) / 2;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t a = x0 + i - N0;
        const uint64_t j = a / B, u = a % B;
        for (uint32_t r = 0; r < R; ++r) {
            uint64_t keys[4];
            for (int k = 0; k < 4; ++k)
                keys[k] = or_sm64(key, 4 * (16 * j + r) + (uint64_t)k);
            uint64_t y = or_feistel(u, half, keys);
            while (y >= B) y = or_feistel(y, half, keys);
            g[(uint64_t)r * n + i] = (uint32_t)y;
        }
    }
}

/* Members of every cell (r, b), ascending point id (reading: within a cell the
 * relaxation walks points in ascending id).  mem_off: R*(B+1), mem: R*N.     */
void or_members(const uint32_t *g, uint64_t N, uint32_t R, uint32_t B,
                uint64_t *mem_off, uint32_t *mem)
{
    for (uint32_t r = 0; r < R; ++r) {
        uint64_t *off = mem_off + (uint64_t)r * (B + 1);
        uint32_t *m = mem + (uint64_t)r * N;
        const uint32_t *gr = g + (uint64_t)r * N;
        memset(off, 0, sizeof(uint64_t) * (B + 1));
        for (uint64_t x = 0; x < N; ++x) off[gr[x] + 1]++;
        for (uint32_t b = 0; b < B; ++b) off[b + 1] += off[b];
        uint64_t *cur = (uint64_t *)malloc(sizeof(uint64_t) * B);
        memcpy(cur, off, sizeof(uint64_t) * B);
        for (uint64_t x = 0; x < N; ++x) m[cur[gr[x]]++] = (uint32_t)x;
        free(cur);
    }
}

/* ------------------------------------------------------------------------- */
/* Reverse index (Section 6, Implementation): for every table t, a map from a
 * bucket value to the list of cells whose distance-sensitive Bloom filter has
 * that bucket set.  A cell c = r*B + b holds bucket h of table t iff some
 * member x of group (r, b) has bucket_t(x) = h.  Lists are sets (a Bloom
 * filter bit is set once), stored ascending.
 * offsets: L*(2^nbits + 1) (absolute positions into cells[]).
 * Returns the number of list entries, or -(needed) if cap is too small.     */
static int or_cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int64_t or_build_lists(const uint32_t *codes, const uint32_t *g, uint64_t N,
                       uint32_t L, uint32_t R, uint32_t B, uint32_t nbits,
                       uint64_t *offsets, uint32_t *cells, uint64_t cap)
{
    const uint64_t nb = 1ULL << nbits;
    uint64_t *pairs = (uint64_t *)malloc(sizeof(uint64_t) * (N * R + 1));
    uint64_t total = 0;
    for (uint32_t t = 0; t < L; ++t) {
        uint64_t np = 0;
        for (uint64_t x = 0; x < N; ++x) {
            uint64_t h = codes[x * L + t];
            for (uint32_t r = 0; r < R; ++r) {
                uint64_t c = (uint64_t)r * B + g[(uint64_t)r * N + x];
                pairs[np++] = (h << 32) | c;
            }
        }
        qsort(pairs, np, sizeof(uint64_t), or_cmp_u64);
        uint64_t *off = offsets + (uint64_t)t * (nb + 1);
        for (uint64_t h = 0; h <= nb; ++h) off[h] = 0;
        /* count distinct pairs per bucket */
        for (uint64_t i = 0; i < np; ++i) {
            if (i > 0 && pairs[i] == pairs[i - 1]) continue;
            off[(pairs[i] >> 32) + 1]++;
        }
        off[0] = total;
        for (uint64_t h = 0; h < nb; ++h) off[h + 1] += off[h];
        for (uint64_t i = 0; i < np; ++i) {
            if (i > 0 && pairs[i] == pairs[i - 1]) continue;
            if (total < cap) cells[total] = (uint32_t)(pairs[i] & 0xFFFFFFFFULL);
            total++;
        }
    }
    free(pairs);
    if (total > cap) return -(int64_t)total;
    return (int64_t)total;
}

/* Cell collision counts through the reverse index (Section 6): for each table
 * the query's bucket list adds one to every listed cell.                    */
void or_counts(const uint64_t *offsets, const uint32_t *cells, uint32_t L,
               uint32_t nbits, uint32_t ncells, const uint32_t *qcodes,
               uint64_t nq, uint8_t *counts)
{
    const uint64_t nb = 1ULL << nbits;
    for (uint64_t q = 0; q < nq; ++q) {
        uint8_t *C = counts + q * ncells;
        memset(C, 0, ncells);
        for (uint32_t t = 0; t < L; ++t) {
            const uint64_t *off = offsets + (uint64_t)t * (nb + 1);
            uint64_t h = qcodes[q * L + t];
            for (uint64_t p = off[h]; p < off[h + 1]; ++p) C[cells[p]]++;
        }
    }
}

/* The same counts from the Bloom-filter definition, without any index
 * (Section 3, distance-sensitive Bloom filter; Section 4 group tests):
 * C[c] = number of tables t for which some member x of cell c has
 * bucket_t(x) = bucket_t(query).                                             */
void or_counts_brute(const uint32_t *codes, const uint32_t *g, uint64_t N,
                     uint32_t L, uint32_t R, uint32_t B,
                     const uint32_t *qcodes, uint64_t nq, uint8_t *counts)
{
    const uint32_t ncells = R * B;
    uint8_t *hit = (uint8_t *)malloc(ncells);
    for (uint64_t q = 0; q < nq; ++q) {
        uint8_t *C = counts + q * ncells;
        memset(C, 0, ncells);
        for (uint32_t t = 0; t < L; ++t) {
            memset(hit, 0, ncells);
            for (uint64_t x = 0; x < N; ++x)
                if (codes[x * L + t] == qcodes[q * L + t])
                    for (uint32_t r = 0; r < R; ++r)
                        hit[r * B + g[(uint64_t)r * N + x]] = 1;
            for (uint32_t c = 0; c < ncells; ++c) C[c] += hit[c];
        }
    }
    free(hit);
}

/* ------------------------------------------------------------------------- */
/* Threshold relaxation (Algorithm 3; Section 6 states it is Algorithm 2 run
 * with decreasing thresholds until k points are reported).
 *
 * What it reports, from the definitions: a point x is reported once the
 * relaxation has passed all R of its cells, i.e. at threshold
 * m(x) = min_r C[r*B + g_r(x)] (Algorithm 2 at t reports exactly the points
 * with m(x) >= t), and its score is that threshold (reading A10).  Cells are
 * passed in descending count, equal counts by ascending cell id (A2), and the
 * points of one cell by ascending id (A3), so among the points reported at
 * the same threshold, x comes after every point whose last cell precedes
 * x's last cell c*(x) = the largest cell id among x's cells of count m(x),
 * and after the smaller ids of that same cell.  The output is therefore the k
 * smallest keys (-m(x), c*(x), x), in increasing order; missing results
 * (k > N) are padded with id 0xFFFFFFFF and score 0.
 *
 * The key of every point is computed, and the k smallest are kept in a
 * bounded max-heap (a partial sort), then emitted in increasing order.     */
typedef struct { uint32_t negm, cstar, x; } or_key;

static int or_key_less(const or_key *p, const or_key *q)
{
    if (p->negm != q->negm) return p->negm < q->negm;
    if (p->cstar != q->cstar) return p->cstar < q->cstar;
    return p->x < q->x;
}

static void or_heap_down(or_key *h, uint32_t n, uint32_t i)
{
    for (;;) {
        uint32_t l = 2 * i + 1, r = l + 1, big = i;
        if (l < n && or_key_less(&h[big], &h[l])) big = l;
        if (r < n && or_key_less(&h[big], &h[r])) big = r;
        if (big == i) return;
        or_key t = h[i]; h[i] = h[big]; h[big] = t;
        i = big;
    }
}

static void or_heap_up(or_key *h, uint32_t i)
{
    while (i > 0) {
        uint32_t p = (i - 1) / 2;
        if (!or_key_less(&h[p], &h[i])) return;
        or_key t = h[i]; h[i] = h[p]; h[p] = t;
        i = p;
    }
}

/* heap: scratch of k keys. */
static void or_decode_keys(const uint8_t *counts, const uint32_t *g, uint64_t N,
                           uint32_t R, uint32_t B, uint32_t k, uint32_t *ids,
                           uint32_t *scores, or_key *heap)
{
    uint32_t n = 0;
    for (uint64_t x = 0; x < N; ++x) {
        uint32_t m = 0xFFFFFFFFu, cs = 0;
        for (uint32_t r = 0; r < R; ++r) {
            uint32_t c = r * B + g[(uint64_t)r * N + x];
            uint32_t v = counts[c];
            if (v < m || (v == m && c > cs)) {
                if (v < m) m = v;
                cs = c;
            }
        }
        or_key key = {1000u - m, cs, (uint32_t)x};
        if (n < k) {
            heap[n] = key;
            or_heap_up(heap, n);
            ++n;
        } else if (or_key_less(&key, &heap[0])) {
            heap[0] = key;
            or_heap_down(heap, n, 0);
        }
    }
    /* pop the largest to the back: increasing order */
    for (uint32_t i = n; i > 0; --i) {
        ids[i - 1] = heap[0].x;
        scores[i - 1] = 1000u - heap[0].negm;
        heap[0] = heap[i - 1];
        or_heap_down(heap, i - 1, 0);
    }
    for (uint32_t i = n; i < k; ++i) {
        ids[i] = 0xFFFFFFFFu;
        scores[i] = 0;
    }
}

void or_decode(const uint8_t *counts, const uint32_t *g, uint64_t N, uint32_t R,
               uint32_t B, uint32_t k, uint32_t *ids, uint32_t *scores)
{
    or_key *heap = (or_key *)malloc(sizeof(or_key) * (k ? k : 1));
    or_decode_keys(counts, g, N, R, B, k, ids, scores, heap);
    free(heap);
}

/* Whole queries from their bucket codes: counts through the reverse index
 * (or_counts) then the decode above, one query per thread.               */
void or_query_many(const uint64_t *offsets, const uint32_t *cells, uint32_t L,
                   uint32_t nbits, const uint32_t *g, uint64_t N, uint32_t R,
                   uint32_t B, const uint32_t *qcodes, uint64_t nq, uint32_t k,
                   uint32_t *ids, uint32_t *scores)
{
#pragma omp parallel
    {
        uint8_t *C = (uint8_t *)malloc((size_t)R * B);
        or_key *heap = (or_key *)malloc(sizeof(or_key) * (k ? k : 1));
#pragma omp for schedule(dynamic, 4)
        for (uint64_t q = 0; q < nq; ++q) {
            or_counts(offsets, cells, L, nbits, R * B, qcodes + q * L, 1, C);
            or_decode_keys(C, g, N, R, B, k, ids + q * k, scores + q * k, heap);
        }
        free(heap);
        free(C);
    }
}

/* Thread count of the parallel loops (a baseline timed on one core sets 1;
 * changes no result). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Fixed-threshold query (Algorithm 2): a cell is positive when its count is
 * at least t; the output marks the points that lie in a positive cell in
 * every repetition (intersection of the per-repetition unions).             */
void or_query_fixed_t(const uint8_t *counts, const uint32_t *g, uint64_t N,
                      uint32_t R, uint32_t B, uint32_t t, uint8_t *reported)
{
    for (uint64_t x = 0; x < N; ++x) reported[x] = 1;
    for (uint32_t r = 0; r < R; ++r) {
        for (uint64_t x = 0; x < N; ++x) {
            uint32_t c = r * B + g[(uint64_t)r * N + x];
            if (counts[c] < t) reported[x] = 0;
        }
    }
}
