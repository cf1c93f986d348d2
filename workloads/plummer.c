/*
 * plummer.c — seeded synthetic particle streams standing in for the N-body
 * snapshots of the paper (Millennium, Sec. 4.1; Millennium XXL, Sec. 4.5), which
 * are not available.  Particles are drawn from Plummer-profile halos with
 * power-law masses plus a uniform background, in a periodic box [0, L)^3, and
 * written as float32 [n][3] (x, y, z).
 *
 * This module holds no arithmetic of the sketch method (no cell keys, hashes or
 * counters): it only produces positions, which both the GPU library and the CPU
 * oracle consume.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), keyed by the
 * 64-bit seed, with counter = (index low, index high, stream id, draw number).
 * Stream 0 draws the halo catalogue, stream 1 the particles, stream 2 the stream
 * order of the exact-count recipe.  Every particle depends only on (seed, index),
 * so any thread split or chunking produces identical bytes.
 *
 * Recipe (per particle):
 *   halo mass     dN/dM ~ M^-slope on [m_lo, m_hi] by inverse CDF
 *   halo centre   uniform in [0, L)^3
 *   Plummer       r = a (u^(-2/3) - 1)^(-1/2), u in (0, u_max], truncated at r = 10a
 *   direction     uniform on the sphere
 *   position      (centre + offset) wrapped into [0, L) in binary64, rounded to float32
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define WL_STREAM_HALO 0u
#define WL_STREAM_PART 1u
#define WL_STREAM_PERM 2u

/* ------------------------------------------------------------ Philox4x32-10 */

static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* Ten rounds of the Philox S-box with a Weyl key schedule. */
void wl_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(0xD2511F53u, c0, &hi0, &lo0);
        mulhilo32(0xCD9E8D57u, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static inline void draw(uint64_t seed, uint64_t index, uint32_t stream, uint32_t n, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), stream, n};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    wl_philox4x32_10(ctr, key, out);
}

/* uniform on the open interval (0, 1) from one 32-bit word */
static inline double u01(uint32_t x)
{
    return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

/* ------------------------------------------------------------ halo catalogue */

static double powerlaw_mass(double u, double m_lo, double m_hi, double slope)
{
    double e = 1.0 - slope;           /* slope 1.9 -> e = -0.9 */
    double a = pow(m_lo, e), b = pow(m_hi, e);
    return pow(a + u * (b - a), 1.0 / e);
}

/* Masses (continuous) and centres of n_halo halos. */
void wl_halo_catalogue(uint64_t seed, uint32_t n_halo, double L, double m_lo, double m_hi,
                       double slope, double *mass, double *centre /* [n_halo][3] */)
{
    for (uint32_t j = 0; j < n_halo; ++j) {
        uint32_t r[4];
        draw(seed, j, WL_STREAM_HALO, 0, r);
        mass[j] = powerlaw_mass(u01(r[0]), m_lo, m_hi, slope);
        centre[3 * j + 0] = u01(r[1]) * L;
        centre[3 * j + 1] = u01(r[2]) * L;
        centre[3 * j + 2] = u01(r[3]) * L;
    }
}

static inline float wrap_to_float(double x, double L)
{
    if (x >= L || x < 0.0) {
        x = fmod(x, L);
        if (x < 0.0)
            x += L;
    }
    return (float)x;
}

/* Enclosed mass fraction of a Plummer sphere at r = 10a: (1 + 1/100)^(-3/2). */
static double plummer_u_max(void)
{
    return pow(1.01, -1.5);
}

/* Plummer offset from three uniforms; truncated at r = 10a (u_max above). */
static inline void plummer_offset(double a, double u_max, double ur, double uc, double uphi, double off[3])
{
    double u = ur * u_max;
    double r = a / sqrt(pow(u, -2.0 / 3.0) - 1.0);
    double ct = 2.0 * uc - 1.0;
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double sp, cp;
    sincos(2.0 * M_PI * uphi, &sp, &cp);
    off[0] = r * st * cp;
    off[1] = r * st * sp;
    off[2] = r * ct;
}

/* -------------------------------------------- recipe 1: exact halo counts */

typedef struct {
    uint64_t r;
    uint64_t i;
} wl_perm_item;

static int cmp_perm(const void *a, const void *b)
{
    const wl_perm_item *x = (const wl_perm_item *)a, *y = (const wl_perm_item *)b;
    if (x->r != y->r)
        return (x->r > y->r) - (x->r < y->r);
    return (x->i > y->i) - (x->i < y->i);
}

/* n particles: halo j gets floor(M_j) particles (halos in index order until n is
 * reached), the rest are uniform in the box, then the stream order is shuffled by
 * sorting on a per-index random 64-bit word (ties by index).  threads > 0 caps the
 * OpenMP threads (1 when the caller runs several generators at once).  Returns the
 * number of halo particles. */
int64_t wl_gen_exact(uint64_t n, double L, uint32_t n_halo, double m_lo, double m_hi,
                     double slope, double a, uint64_t seed, float *pos, int threads)
{
    double *mass = (double *)malloc(sizeof(double) * (n_halo ? n_halo : 1));
    double *cen = (double *)malloc(sizeof(double) * 3 * (n_halo ? n_halo : 1));
    uint64_t *first = (uint64_t *)malloc(sizeof(uint64_t) * ((uint64_t)n_halo + 1));
    wl_halo_catalogue(seed, n_halo, L, m_lo, m_hi, slope, mass, cen);
    first[0] = 0;
    for (uint32_t j = 0; j < n_halo; ++j) {
        uint64_t c = (uint64_t)floor(mass[j]);
        uint64_t next = first[j] + c;
        first[j + 1] = next < n ? next : n;
    }
    uint64_t H = first[n_halo];
    const double u_max = plummer_u_max();
    float *nat = (float *)malloc(sizeof(float) * 3 * (n ? n : 1));
    #pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : omp_get_max_threads())
    for (int64_t ii = 0; ii < (int64_t)n; ++ii) {
        uint64_t i = (uint64_t)ii;
        uint32_t r[4];
        draw(seed, i, WL_STREAM_PART, 0, r);
        if (i < H) {
            uint32_t lo = 0, hi = n_halo;       /* find j with first[j] <= i < first[j+1] */
            while (hi - lo > 1) {
                uint32_t mid = lo + (hi - lo) / 2;
                if (first[mid] <= i) lo = mid; else hi = mid;
            }
            double off[3];
            plummer_offset(a, u_max, u01(r[0]), u01(r[1]), u01(r[2]), off);
            for (int c = 0; c < 3; ++c)
                nat[3 * i + c] = wrap_to_float(cen[3 * lo + c] + off[c], L);
        } else {
            for (int c = 0; c < 3; ++c)
                nat[3 * i + c] = wrap_to_float(u01(r[c]) * L, L);
        }
    }
    wl_perm_item *perm = (wl_perm_item *)malloc(sizeof(wl_perm_item) * (n ? n : 1));
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t r[4];
        draw(seed, i, WL_STREAM_PERM, 0, r);
        perm[i].r = (uint64_t)r[0] | ((uint64_t)r[1] << 32);
        perm[i].i = i;
    }
    qsort(perm, n, sizeof(wl_perm_item), cmp_perm);
    for (uint64_t j = 0; j < n; ++j)
        memcpy(pos + 3 * j, nat + 3 * perm[j].i, 3 * sizeof(float));
    free(perm);
    free(nat);
    free(first);
    free(cen);
    free(mass);
    return (int64_t)H;
}

/* ------------------------------------------ recipe 2: independent mixture */

typedef struct {
    double own[3];
    double alt[3];
    double prob;
    double pad;
} wl_alias_rec;

/* Vose alias table over weights w[0..m). prob in [0,1], alias in [0,m). */
static void alias_build(const double *w, uint32_t m, double *prob, uint32_t *alias)
{
    double total = 0.0;
    for (uint32_t j = 0; j < m; ++j)
        total += w[j];
    double *s = (double *)malloc(sizeof(double) * m);
    uint32_t *small = (uint32_t *)malloc(sizeof(uint32_t) * m);
    uint32_t *large = (uint32_t *)malloc(sizeof(uint32_t) * m);
    uint32_t ns = 0, nl = 0;
    for (uint32_t j = 0; j < m; ++j) {
        s[j] = w[j] * (double)m / total;
        if (s[j] < 1.0) small[ns++] = j; else large[nl++] = j;
    }
    while (ns > 0 && nl > 0) {
        uint32_t l = small[--ns], g = large[--nl];
        prob[l] = s[l];
        alias[l] = g;
        s[g] = (s[g] + s[l]) - 1.0;
        if (s[g] < 1.0) small[ns++] = g; else large[nl++] = g;
    }
    while (nl > 0) { uint32_t g = large[--nl]; prob[g] = 1.0; alias[g] = g; }
    while (ns > 0) { uint32_t l = small[--ns]; prob[l] = 1.0; alias[l] = l; }
    free(large);
    free(small);
    free(s);
}

/* Particles with global indices [start, start + n): each is background (uniform)
 * with probability f_bg, otherwise it belongs to a halo drawn with probability
 * proportional to the halo mass.  threads as for wl_gen_exact.  Returns 0. */
int64_t wl_gen_mixture(uint64_t start, uint64_t n, double L, uint32_t n_halo, double m_lo,
                       double m_hi, double slope, double a, double f_bg, uint64_t seed, float *pos,
                       int threads)
{
    double *mass = (double *)malloc(sizeof(double) * (n_halo ? n_halo : 1));
    double *cen = (double *)malloc(sizeof(double) * 3 * (n_halo ? n_halo : 1));
    double *prob = (double *)malloc(sizeof(double) * (n_halo ? n_halo : 1));
    uint32_t *alias = (uint32_t *)malloc(sizeof(uint32_t) * (n_halo ? n_halo : 1));
    wl_halo_catalogue(seed, n_halo, L, m_lo, m_hi, slope, mass, cen);
    if (n_halo > 0)
        alias_build(mass, n_halo, prob, alias);
    /* one 64-byte record per alias column: both candidate halos' centres + the cut */
    wl_alias_rec *rec = (wl_alias_rec *)malloc(sizeof(wl_alias_rec) * (n_halo ? n_halo : 1));
    for (uint32_t j = 0; j < n_halo; ++j) {
        rec[j].prob = prob[j];
        for (int c = 0; c < 3; ++c) {
            rec[j].own[c] = cen[3 * j + c];
            rec[j].alt[c] = cen[3 * (uint64_t)alias[j] + c];
        }
    }
    const double u_max = plummer_u_max();
    #pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : omp_get_max_threads())
    for (int64_t jj = 0; jj < (int64_t)n; ++jj) {
        uint64_t i = start + (uint64_t)jj;
        uint32_t r[4], q[4];
        draw(seed, i, WL_STREAM_PART, 0, r);
        float *out = pos + 3 * (uint64_t)jj;
        if (n_halo == 0 || u01(r[0]) < f_bg) {
            for (int c = 0; c < 3; ++c)
                out[c] = wrap_to_float(u01(r[1 + c]) * L, L);
        } else {
            draw(seed, i, WL_STREAM_PART, 1, q);
            uint32_t col = (uint32_t)(((uint64_t)r[1] * n_halo) >> 32);
            const double *cc = (u01(r[2]) < rec[col].prob) ? rec[col].own : rec[col].alt;
            double off[3];
            plummer_offset(a, u_max, u01(r[3]), u01(q[0]), u01(q[1]), off);
            for (int c = 0; c < 3; ++c)
                out[c] = wrap_to_float(cc[c] + off[c], L);
        }
    }
    free(rec);
    free(alias);
    free(prob);
    free(cen);
    free(mass);
    return 0;
}

/* The mixture recipe's per-column records for a device generator: rec[j] = {own centre
 * x, y, z, alias centre x, y, z, cut, 0} (8 doubles), built exactly as wl_gen_mixture
 * builds them.  Returns 0. */
int64_t wl_alias_records(uint64_t seed, uint32_t n_halo, double L, double m_lo, double m_hi, double slope,
                         double *rec_out)
{
    if (n_halo == 0)
        return 0;
    double *mass = (double *)malloc(sizeof(double) * n_halo);
    double *cen = (double *)malloc(sizeof(double) * 3 * n_halo);
    double *prob = (double *)malloc(sizeof(double) * n_halo);
    uint32_t *alias = (uint32_t *)malloc(sizeof(uint32_t) * n_halo);
    wl_halo_catalogue(seed, n_halo, L, m_lo, m_hi, slope, mass, cen);
    alias_build(mass, n_halo, prob, alias);
    wl_alias_rec *rec = (wl_alias_rec *)rec_out;
    for (uint32_t j = 0; j < n_halo; ++j) {
        rec[j].prob = prob[j];
        rec[j].pad = 0.0;
        for (int c = 0; c < 3; ++c) {
            rec[j].own[c] = cen[3 * j + c];
            rec[j].alt[c] = cen[3 * (uint64_t)alias[j] + c];
        }
    }
    free(alias);
    free(prob);
    free(cen);
    free(mass);
    return 0;
}

/* out[i] = word g mod 4 of Philox4x32-10 at counter ((g / 4) mod 2^32, (g / 4) / 2^32, stream, 0)
 * under key (seed mod 2^32, seed / 2^32), g = index0 + i, for i < n: the g-th 32-bit word of the
 * generator's output stream, four words per counter. */
void wl_philox_words(uint64_t index0, uint64_t n, uint32_t stream, uint64_t seed, uint32_t *out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    #pragma omp parallel for schedule(static)
    for (int64_t ii = 0; ii < (int64_t)n; ++ii) {
        const uint64_t g = index0 + (uint64_t)ii, c = g >> 2;
        const uint32_t ctr[4] = {(uint32_t)c, (uint32_t)(c >> 32), stream, 0u};
        uint32_t r[4];
        wl_philox4x32_10(ctr, key, r);
        out[ii] = r[g & 3u];
    }
}
