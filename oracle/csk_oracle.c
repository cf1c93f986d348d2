/*
 * csk_oracle.c — plain, slow, obviously-correct CPU oracle for the streaming
 * Count-Sketch halo-finder hot path of Ivkin et al., "Scalable Streaming Tools
 * for Analyzing N-body Simulations" (arXiv:1711.00975).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes, step by step (each function cites its passage):
 *   grid       G = round(L / delta) cells per side               (Sec. 2.1, mesh on the box; Sec. 4.1)
 *   cell index i = floor(p * G / L) over exact rationals, wrapped  (Sec. 2.1; Sec. 3.1 stage 1)
 *   cell key   (ix * G + iy) * G + iz                              (Sec. 2.1: a particle becomes the ID of its cell)
 *   hashes     simple tabulation seeded by SplitMix64; one 32-bit word per row gives
 *              the bucket (bits 0..30, range-reduced) and the sign (bit 31)  (Sec. 2.2, 2-independent hashes)
 *   Add        M[r][bucket_r] += sign_r for every row r              (Sec. 2.2, Add; Alg. 1 stream loop)
 *   Estimate   lower median over rows of M[r][bucket_r] * sign_r     (Sec. 2.2, Estimate; Alg. 4 Estimate)
 *   Count-Min  variant: Add +1, Estimate = min over rows (no sign)   (Sec. 2.2, Count-Min paragraph)
 *   exact      histogram by sort + run-length                        (Sec. 4.2, exact algorithm)
 *   top-k      distinct stream cells with estimate >= theta ordered by (estimate desc, key asc)
 *              (Sec. 2.2 UpdateHeap / Alg. 1 query loop; Sec. 3.1 item 4 threshold array)
 *   full search the same over every key of the G^3 dictionary      (Sec. 2.2 item 1, CSFS; Alg. 1)
 *   hierarchy  super-items key / R in a second sketch; children of heavy super-items only
 *              (Sec. 2.2 item 3, CSHi; Alg. 3)
 *
 * Readings of points the paper leaves open (hash family, cell-ID formula, even-row
 * median, tie order, counter width) are the ones listed in the design notes; each
 * function states the reading it implements.
 *
 * Plain C99 + the GCC __int128 extension.  No threads, no SIMD, no blocking.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_W_INCOMPLETE 1
#define ORC_E_INVALID (-1)
#define ORC_E_DOMAIN (-5)

#define ORC_VARIANT_CS 0  /* Count Sketch: signed updates, median estimate */
#define ORC_VARIANT_CM 1  /* Count-Min: +1 updates, minimum estimate        */

#define ORC_CHARS 6       /* keys are < 2^48: six 8-bit characters            */

/* ---------------------------------------------------------------- grid (O1) */

/* Cells per side of the regular mesh: G = round(L / delta).  The mesh is valid
 * when delta and L are finite and positive, 1 <= G <= 65535 (so keys stay below
 * 2^48) and L / delta is within 1e-6 relative of the integer G.  Sec. 2.1 puts a
 * regular mesh on the box; Sec. 4.1 gives 500 / 0.1 Mpc/h per side. */
int orc_grid(double delta, double L, int64_t *G_out)
{
    if (!(delta > 0.0) || !(L > 0.0) || !isfinite(delta) || !isfinite(L))
        return ORC_E_INVALID;
    double q = L / delta;
    if (!(q >= 0.5) || !(q < 65535.5))
        return ORC_E_INVALID;
    int64_t G = (int64_t)llround(q);
    if (G < 1 || G > 65535)
        return ORC_E_INVALID;
    if (fabs(q - (double)G) > 1e-6 * (double)G)
        return ORC_E_INVALID;
    *G_out = G;
    return ORC_OK;
}

/* ------------------------------------------------------- cell index (O2) */

/* floor(a / b) for a signed 128-bit a and a positive b. */
static __int128 floordiv128(__int128 a, __int128 b)
{
    __int128 q = a / b;
    if ((a % b) != 0 && a < 0)
        q -= 1;
    return q;
}

/* Is the position inside the accepted domain: finite and |p| < 2L? */
int orc_in_domain(float p, double L)
{
    double x = (double)p;
    if (!isfinite(x))
        return 0;
    return fabs(x) < 2.0 * L;
}

/* Exact cell index along one axis: i = floor(p * G / L) evaluated on the exact
 * rational values of the float32 p and the binary64 L, then wrapped into [0, G)
 * (periodic box).  Sec. 2.1: each particle is replaced by the ID of the cell it
 * lies in; Sec. 3.1 stage 1.  Returns ORC_E_DOMAIN for non-finite p or |p| >= 2L.
 *
 * Method: p = mp * 2^ep with integer mp (|mp| < 2^24), L = mL * 2^eL with integer
 * mL (< 2^53); p*G/L = (mp*G) / mL * 2^(ep-eL), a ratio of integers evaluated with
 * 128-bit integer division. */
int orc_cell_index(float p, int64_t G, double L, int64_t *i_out)
{
    if (!orc_in_domain(p, L))
        return ORC_E_DOMAIN;
    int ep, eL;
    float fp = frexpf(p, &ep);          /* p = fp * 2^ep, |fp| in [0.5, 1) or 0 */
    double fL = frexp(L, &eL);          /* L = fL * 2^eL, fL in [0.5, 1)        */
    int64_t mp = (int64_t)ldexpf(fp, 24);   /* exact: fp has 24 significant bits */
    int64_t mL = (int64_t)ldexp(fL, 53);    /* exact: fL has 53 significant bits */
    ep -= 24;
    eL -= 53;
    __int128 num = (__int128)mp * (__int128)G;   /* |num| < 2^40 */
    int s = ep - eL;
    __int128 q;
    if (num == 0) {
        q = 0;
    } else if (s >= 0) {
        /* |p*G/L| < 2G <= 2^17 bounds num * 2^s below 2^71: no overflow. */
        q = floordiv128(num * ((__int128)1 << s), (__int128)mL);
    } else if (-s <= 70) {
        q = floordiv128(num, (__int128)mL << (-s));
    } else {
        /* |num| / (mL * 2^-s) < 2^40 / 2^122 < 1: the quotient lies in (-1, 1). */
        q = (num > 0) ? 0 : -1;
    }
    int64_t i = (int64_t)q;
    i %= G;
    if (i < 0)
        i += G;
    *i_out = i;
    return ORC_OK;
}

/* ------------------------------------------------------------- key (O3) */

/* Cell key of one particle: (ix * G + iy) * G + iz, x slowest, 0-based.
 * Sec. 2.1 (the dictionary of cells).  Returns ORC_E_DOMAIN if any coordinate is
 * outside the domain. */
int orc_cell_key(const float *xyz, int64_t G, double L, uint64_t *key_out)
{
    int64_t ix, iy, iz;
    if (orc_cell_index(xyz[0], G, L, &ix) != ORC_OK) return ORC_E_DOMAIN;
    if (orc_cell_index(xyz[1], G, L, &iy) != ORC_OK) return ORC_E_DOMAIN;
    if (orc_cell_index(xyz[2], G, L, &iz) != ORC_OK) return ORC_E_DOMAIN;
    *key_out = ((uint64_t)ix * (uint64_t)G + (uint64_t)iy) * (uint64_t)G + (uint64_t)iz;
    return ORC_OK;
}

/* Keys of all in-domain particles, in stream order.  Returns how many were written. */
int64_t orc_keys(const float *pos, uint64_t n, double delta, double L, uint64_t *keys_out)
{
    int64_t G;
    if (orc_grid(delta, L, &G) != ORC_OK)
        return ORC_E_INVALID;
    int64_t m = 0;
    for (uint64_t j = 0; j < n; ++j) {
        uint64_t key;
        if (orc_cell_key(pos + 3 * j, G, L, &key) == ORC_OK)
            keys_out[m++] = key;
    }
    return m;
}

/* ------------------------------------------------------ hash tables (O4) */

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): a Weyl sequence with increment
 * 0x9E3779B97F4A7C15 followed by the variant-13 finaliser. */
uint64_t orc_splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Simple-tabulation tables T[r][c][v] (r < d rows, c < 6 characters, v < 256),
 * filled in that nesting order from one SplitMix64 stream started at `seed`,
 * two 32-bit entries per 64-bit output, low half first.
 * Reading of Sec. 2.2 (t independent bucket and sign hashes, 2-independence):
 * simple tabulation is 3-independent, which implies the pairwise independence the
 * unbiasedness argument needs. */
void orc_hash_tables(uint64_t seed, uint32_t d, uint32_t *T)
{
    uint64_t state = seed;
    uint64_t total = (uint64_t)d * ORC_CHARS * 256;
    for (uint64_t idx = 0; idx < total; idx += 2) {
        uint64_t z = orc_splitmix64_next(&state);
        T[idx] = (uint32_t)(z & 0xFFFFFFFFu);
        if (idx + 1 < total)
            T[idx + 1] = (uint32_t)(z >> 32);
    }
}

/* ---------------------------------------------------------- row hash (O5) */

/* Tabulated 32-bit word of row r: XOR over the six key bytes of T[r][c][byte c]. */
uint32_t orc_row_hash(const uint32_t *T, uint32_t r, uint64_t key)
{
    const uint32_t *Tr = T + (uint64_t)r * ORC_CHARS * 256;
    uint32_t h = 0;
    for (int c = 0; c < ORC_CHARS; ++c)
        h ^= Tr[c * 256 + ((key >> (8 * c)) & 0xFFu)];
    return h;
}

/* Bucket hash h_{r,b}: the low 31 bits scaled onto [0, w) by a 64-bit product
 * (multiply-shift range reduction, exact for any w <= 2^30). */
uint32_t orc_bucket(uint32_t h, uint32_t w)
{
    return (uint32_t)(((uint64_t)(h & 0x7FFFFFFFu) * (uint64_t)w) >> 31);
}

/* Sign hash h_{r,s}: +1 when bit 31 is clear, -1 when set. */
int32_t orc_sign(uint32_t h)
{
    return (h >> 31) ? -1 : 1;
}

/* ----------------------------------------------------------- Add (O6) */

/* Stream every in-domain particle into the counters M (int32, [d][w] row-major,
 * wrapping modulo 2^32):
 *   Count Sketch:  M[r][bucket_r(key)] += sign_r(key)  for r < d  (Sec. 2.2 Add; Alg. 1; Alg. 4 Update)
 *   Count-Min:     M[r][bucket_r(key)] += 1                       (Sec. 2.2, Count-Min Add)
 * Particles outside the domain are skipped.  Returns the number skipped, or
 * ORC_E_INVALID for an invalid mesh. */
int64_t orc_sketch_update(int32_t *M, const uint32_t *T, uint32_t d, uint32_t w, int variant,
                          const float *pos, uint64_t n, double delta, double L)
{
    int64_t G;
    if (orc_grid(delta, L, &G) != ORC_OK || d < 1 || w < 1)
        return ORC_E_INVALID;
    int64_t skipped = 0;
    for (uint64_t j = 0; j < n; ++j) {
        uint64_t key;
        if (orc_cell_key(pos + 3 * j, G, L, &key) != ORC_OK) {
            ++skipped;
            continue;
        }
        for (uint32_t r = 0; r < d; ++r) {
            uint32_t h = orc_row_hash(T, r, key);
            uint32_t b = orc_bucket(h, w);
            int32_t s = (variant == ORC_VARIANT_CM) ? 1 : orc_sign(h);
            uint32_t *cell = (uint32_t *)&M[(uint64_t)r * w + b];
            *cell = *cell + (uint32_t)s;    /* modulo 2^32 */
        }
    }
    return skipped;
}

/* Add every given item key to the counters, as orc_sketch_update does for the cell
 * key of each particle (Sec. 2.2 Add).  Used for the super-item sketch of the
 * hierarchical variant, whose items are cell keys divided by the group size. */
void orc_sketch_update_keys(int32_t *M, const uint32_t *T, uint32_t d, uint32_t w, int variant,
                            const uint64_t *keys, uint64_t m)
{
    for (uint64_t j = 0; j < m; ++j) {
        for (uint32_t r = 0; r < d; ++r) {
            uint32_t h = orc_row_hash(T, r, keys[j]);
            uint32_t b = orc_bucket(h, w);
            int32_t s = (variant == ORC_VARIANT_CM) ? 1 : orc_sign(h);
            uint32_t *cell = (uint32_t *)&M[(uint64_t)r * w + b];
            *cell = *cell + (uint32_t)s;
        }
    }
}

/* ------------------------------------------------------- Estimate (O7) */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Frequency estimate of each key:
 *   Count Sketch: the element at index floor((d-1)/2) of the ascending sort of
 *                 { M[r][bucket_r] * sign_r : r < d }  (Sec. 2.2 Estimate; Alg. 4 Estimate;
 *                 for even d the lower of the two middle values)
 *   Count-Min:    min over r of M[r][bucket_r]         (Sec. 2.2, Count-Min Estimate, read without sign)
 * Products are taken modulo 2^32 and read as int32. */
void orc_estimate(const int32_t *M, const uint32_t *T, uint32_t d, uint32_t w, int variant,
                  const uint64_t *keys, uint64_t m, int32_t *est)
{
    int32_t *e = (int32_t *)malloc(sizeof(int32_t) * d);
    for (uint64_t j = 0; j < m; ++j) {
        for (uint32_t r = 0; r < d; ++r) {
            uint32_t h = orc_row_hash(T, r, keys[j]);
            uint32_t b = orc_bucket(h, w);
            uint32_t c = (uint32_t)M[(uint64_t)r * w + b];
            if (variant == ORC_VARIANT_CM)
                e[r] = (int32_t)c;
            else
                e[r] = (int32_t)(c * (uint32_t)orc_sign(h));
        }
        qsort(e, d, sizeof(int32_t), cmp_i32);
        est[j] = (variant == ORC_VARIANT_CM) ? e[0] : e[(d - 1) / 2];
    }
    free(e);
}

/* ----------------------------------------------- exact histogram (O8) */

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Exact count of every distinct key (Sec. 4.2, the exact algorithm), computed by
 * sorting a copy of the keys and run-length encoding it.  Writes distinct keys in
 * ascending order with their counts; returns the number of distinct keys. */
int64_t orc_histogram(const uint64_t *keys, uint64_t n, uint64_t *uniq, int64_t *count)
{
    if (n == 0)
        return 0;
    uint64_t *s = (uint64_t *)malloc(sizeof(uint64_t) * n);
    memcpy(s, keys, sizeof(uint64_t) * n);
    qsort(s, n, sizeof(uint64_t), cmp_u64);
    int64_t m = 0;
    for (uint64_t j = 0; j < n; ++j) {
        if (m > 0 && uniq[m - 1] == s[j]) {
            count[m - 1] += 1;
        } else {
            uniq[m] = s[j];
            count[m] = 1;
            ++m;
        }
    }
    free(s);
    return m;
}

/* ---------------------------------------------------- top-k (O9, O10) */

typedef struct {
    uint64_t key;
    int64_t value;
} orc_item;

/* value descending, then key ascending */
static int cmp_item(const void *a, const void *b)
{
    const orc_item *x = (const orc_item *)a, *y = (const orc_item *)b;
    if (x->value != y->value)
        return (x->value < y->value) ? 1 : -1;
    return (x->key > y->key) - (x->key < y->key);
}

/* Top-k from the sketch.  Candidates are the distinct cells of the stream whose
 * estimate is >= theta; they are ordered by (estimate desc, key asc) and the first
 * min(k, |C|) are written.  Sec. 2.2 (UpdateHeap keeps the k largest estimates;
 * Alg. 1 query loop), Sec. 3.1 item 4 (keep the cells above a threshold).
 * `*status` is ORC_W_INCOMPLETE when fewer than k candidates passed a theta above
 * INT32_MIN, else ORC_OK.  Returns the number written. */
int64_t orc_topk_sketch(const int32_t *M, const uint32_t *T, uint32_t d, uint32_t w, int variant,
                        const float *pos, uint64_t n, double delta, double L,
                        int32_t theta, uint64_t k,
                        uint64_t *keys_out, int32_t *est_out, int32_t *status)
{
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    int64_t nk = orc_keys(pos, n, delta, L, keys);
    if (nk < 0) {
        free(keys);
        *status = ORC_E_INVALID;
        return 0;
    }
    uint64_t *uniq = (uint64_t *)malloc(sizeof(uint64_t) * (nk ? nk : 1));
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (nk ? nk : 1));
    int64_t m = orc_histogram(keys, (uint64_t)nk, uniq, cnt);
    int32_t *est = (int32_t *)malloc(sizeof(int32_t) * (m ? m : 1));
    orc_estimate(M, T, d, w, variant, uniq, (uint64_t)m, est);
    orc_item *items = (orc_item *)malloc(sizeof(orc_item) * (m ? m : 1));
    int64_t c = 0;
    for (int64_t j = 0; j < m; ++j) {
        if (est[j] >= theta) {
            items[c].key = uniq[j];
            items[c].value = est[j];
            ++c;
        }
    }
    qsort(items, (size_t)c, sizeof(orc_item), cmp_item);
    int64_t out = (c < (int64_t)k) ? c : (int64_t)k;
    for (int64_t j = 0; j < out; ++j) {
        keys_out[j] = items[j].key;
        est_out[j] = (int32_t)items[j].value;
    }
    *status = (out < (int64_t)k && theta != INT32_MIN) ? ORC_W_INCOMPLETE : ORC_OK;
    free(items);
    free(est);
    free(cnt);
    free(uniq);
    free(keys);
    return out;
}

/* Top-k over the whole dictionary (Count Sketch with Full Search): every cell key of
 * the G^3 mesh, whether or not a particle fell in it, is estimated; the keys with
 * estimate >= theta are ordered by (estimate desc, key asc) and the first min(k, |C|)
 * are written.  Sec. 2.2 item 1 (CSFS: estimate each possible item of the dictionary
 * and find the top k) and Alg. 1 (query loop over the dictionary).  `*status` is
 * ORC_W_INCOMPLETE when fewer than k keys passed a theta above INT32_MIN, else ORC_OK;
 * ORC_E_INVALID for G < 1 or G^3 above 2^32 keys (the oracle keeps every passing key in
 * memory).  Returns the number written. */
int64_t orc_topk_dictionary(const int32_t *M, const uint32_t *T, uint32_t d, uint32_t w, int variant,
                            int64_t G, int32_t theta, uint64_t k,
                            uint64_t *keys_out, int32_t *est_out, int32_t *status)
{
    if (G < 1 || G > 1625) {   /* 1625^3 < 2^32 */
        *status = ORC_E_INVALID;
        return 0;
    }
    const uint64_t nkeys = (uint64_t)G * (uint64_t)G * (uint64_t)G;
    uint64_t cap = 1024, c = 0;
    orc_item *items = (orc_item *)malloc(sizeof(orc_item) * cap);
    for (uint64_t key = 0; key < nkeys; ++key) {
        int32_t est;
        orc_estimate(M, T, d, w, variant, &key, 1, &est);
        if (est >= theta) {
            if (c == cap) {
                cap *= 2;
                items = (orc_item *)realloc(items, sizeof(orc_item) * cap);
            }
            items[c].key = key;
            items[c].value = est;
            ++c;
        }
    }
    qsort(items, (size_t)c, sizeof(orc_item), cmp_item);
    uint64_t out = (c < k) ? c : k;
    for (uint64_t j = 0; j < out; ++j) {
        keys_out[j] = items[j].key;
        est_out[j] = (int32_t)items[j].value;
    }
    *status = (out < k && theta != INT32_MIN) ? ORC_W_INCOMPLETE : ORC_OK;
    free(items);
    return (int64_t)out;
}

/* Top-k of the hierarchical variant (Count Sketch Hierarchical): M1 counts super-items
 * key / R, M2 counts the cell keys.  Every super-item j of [0, ceil(G^3 / R)) is
 * estimated from M1; for those with estimate >= theta1, every child key of
 * [j R, min((j + 1) R, G^3)) is estimated from M2, and the children with estimate >=
 * theta2 are the candidates, ordered by (estimate desc, key asc); the first min(k, |C|)
 * are written.  Sec. 2.2 item 3 and Alg. 3 (query: heavy super-items first, then their
 * items); the paper's strict ">" thresholds are written here as ">=" on the next integer.
 * `*status` is ORC_W_INCOMPLETE when fewer than k were found while either threshold is
 * above INT32_MIN (then the candidates may not include every key), else ORC_OK;
 * ORC_E_INVALID for G < 1, G^3 above 2^32 or R < 1. */
int64_t orc_topk_hierarchical(const int32_t *M1, const uint32_t *T1, uint32_t d1, uint32_t w1,
                              const int32_t *M2, const uint32_t *T2, uint32_t d2, uint32_t w2, int variant,
                              int64_t G, uint64_t R, int32_t theta1, int32_t theta2, uint64_t k,
                              uint64_t *keys_out, int32_t *est_out, int32_t *status)
{
    if (G < 1 || G > 1625 || R < 1) {
        *status = ORC_E_INVALID;
        return 0;
    }
    const uint64_t nkeys = (uint64_t)G * (uint64_t)G * (uint64_t)G;
    const uint64_t nsuper = (nkeys + R - 1) / R;
    uint64_t cap = 1024, c = 0;
    orc_item *items = (orc_item *)malloc(sizeof(orc_item) * cap);
    for (uint64_t j = 0; j < nsuper; ++j) {
        int32_t e1;
        orc_estimate(M1, T1, d1, w1, variant, &j, 1, &e1);
        if (e1 < theta1)
            continue;
        const uint64_t hi = (j + 1) * R < nkeys ? (j + 1) * R : nkeys;
        for (uint64_t key = j * R; key < hi; ++key) {
            int32_t e2;
            orc_estimate(M2, T2, d2, w2, variant, &key, 1, &e2);
            if (e2 < theta2)
                continue;
            if (c == cap) {
                cap *= 2;
                items = (orc_item *)realloc(items, sizeof(orc_item) * cap);
            }
            items[c].key = key;
            items[c].value = e2;
            ++c;
        }
    }
    qsort(items, (size_t)c, sizeof(orc_item), cmp_item);
    uint64_t out = (c < k) ? c : k;
    for (uint64_t j = 0; j < out; ++j) {
        keys_out[j] = items[j].key;
        est_out[j] = (int32_t)items[j].value;
    }
    *status = (out < k && (theta1 != INT32_MIN || theta2 != INT32_MIN)) ? ORC_W_INCOMPLETE : ORC_OK;
    free(items);
    return (int64_t)out;
}

/* Exact top-k: the distinct keys ordered by (exact count desc, key asc), first k.
 * Sec. 4.2 (exact algorithm, step 3). */
int64_t orc_topk_exact(const uint64_t *uniq, const int64_t *count, uint64_t m, uint64_t k,
                       uint64_t *keys_out, int64_t *count_out)
{
    orc_item *items = (orc_item *)malloc(sizeof(orc_item) * (m ? m : 1));
    for (uint64_t j = 0; j < m; ++j) {
        items[j].key = uniq[j];
        items[j].value = count[j];
    }
    qsort(items, m, sizeof(orc_item), cmp_item);
    uint64_t out = (m < k) ? m : k;
    for (uint64_t j = 0; j < out; ++j) {
        keys_out[j] = items[j].key;
        count_out[j] = items[j].value;
    }
    free(items);
    return (int64_t)out;
}

/* ------------------------------------------------------ array helpers */

/* Row-r tabulated words of m keys (a loop over orc_row_hash, for the tests). */
void orc_row_hash_many(const uint32_t *T, uint32_t r, const uint64_t *keys, uint64_t m, uint32_t *out)
{
    for (uint64_t j = 0; j < m; ++j)
        out[j] = orc_row_hash(T, r, keys[j]);
}

/* Exact cell indices of m coordinates along one axis; out[j] = -1 outside the domain. */
void orc_cell_index_many(const float *p, uint64_t m, int64_t G, double L, int64_t *out)
{
    for (uint64_t j = 0; j < m; ++j) {
        int64_t i;
        out[j] = (orc_cell_index(p[j], G, L, &i) == ORC_OK) ? i : -1;
    }
}
