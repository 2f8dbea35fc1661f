/*
 * saoracle.c -- CPU oracle for the suffix-array / LCP / read-overlap path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline call this code.  The GPU library never links, loads or includes it, and the two
 * share no source: this file is written from the definitions in the paper, not from the
 * kernels.
 *
 * What is computed (the plain definitions; nothing here is blocked, fused or reordered):
 *
 *  Text.  T = r_0 $ r_1 $ ... r_{m-1} $, the fragments of Sec. III laid end to end, each closed
 *  by its own separator.  Separators are distinct symbols: the one closing read i sorts below
 *  the one closing read j exactly when i < j, and every separator sorts below every other byte.
 *  Other bytes compare by value (A < C < G < T for DNA).  The code is byte-generic so that the
 *  paper's worked example over {a,b,h,p,t} (Sec. III) runs unchanged.
 *
 *  SA.  The array of all suffix start positions sorted lexicographically (Sec. IV: the suffix
 *  array is the sorted array of all suffixes).  Because every suffix contains a separator that
 *  no other suffix has at the same offset, the order is total and the SA is unique.
 *
 *  LCP.  lcp[0] = 0; lcp[i] = length of the longest common prefix of the suffixes at sa[i-1]
 *  and sa[i].  Two separators never match each other (they are different symbols).
 *
 *  Lookup.  For a pattern P (bytes other than the separator), the suffixes that start with P
 *  are one interval [lo, hi) of the SA (Sec. IV: the array is searched to decide whether one
 *  string is a prefix of another).  By definition lo is the number of suffixes that sort
 *  below P without starting with it, and hi - lo is the number of text positions where P
 *  occurs; both are counted over text positions, without any suffix array.
 *
 *  Overlaps.  For every ordered pair of distinct reads (a, b), the largest l with
 *  min_len <= l <= min(|a|, |b|) such that the last l bytes of a equal the first l bytes of b;
 *  reported as (a, b, l) when such l exists, sorted by (a, b).  l = |a| is the paper's 'fir'
 *  relation (Sec. III: a fragment that is a prefix of another).
 *
 * Two overlap routines: the literal all-pairs definition (overlaps_brute) and an exact
 * seed-and-verify search (overlaps_indexed) for inputs too large for all pairs.  The second
 * only uses a hash of each read's first min_len bytes as a filter; every reported triple is
 * confirmed by direct byte comparison, so a hash collision can cost time but never change a
 * result.  The test suite pins the second against the first.
 *
 * Parity pins: brute force on tiny inputs (an independent Python literal definition), the
 * paper's worked example, closed forms and invariants; see the test suite.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SEPB ((uint8_t)'$')

/* ---------------------------------------------------------------------------------------- */
/* Suffix comparison: the ordered alphabet of the text (see header).                         */
/* ---------------------------------------------------------------------------------------- */
static int suffix_cmp(const uint8_t *t, int64_t p, int64_t q)
{
    if (p == q) return 0;
    for (int64_t k = 0;; ++k) {
        uint8_t x = t[p + k], y = t[q + k];
        if (x == SEPB && y == SEPB) return (p < q) ? -1 : 1; /* separator of the earlier read */
        if (x == SEPB) return -1;
        if (y == SEPB) return 1;
        if (x != y) return (x < y) ? -1 : 1;
    }
}

static int cmp_ctx(const void *a, const void *b, void *ctx)
{
    const uint8_t *t = (const uint8_t *)ctx;
    int32_t p = *(const int32_t *)a, q = *(const int32_t *)b;
    return suffix_cmp(t, p, q);
}

/* Exported: compare two suffixes (used by sampled checks at sizes the full sort cannot
 * afford). */
int oracle_suffix_cmp(const uint8_t *t, int64_t n, int64_t p, int64_t q)
{
    (void)n;
    return suffix_cmp(t, p, q);
}

/* Exported: longest common prefix of the suffixes at p and q (separators never match). */
int64_t oracle_lcp_pair(const uint8_t *t, int64_t n, int64_t p, int64_t q)
{
    (void)n;
    if (p == q) {
        int64_t k = 0;
        while (t[p + k] != SEPB) ++k;
        return k;
    }
    int64_t k = 0;
    while (t[p + k] == t[q + k] && t[p + k] != SEPB) ++k;
    return k;
}

/* Returns 0 when the text is well formed for the definitions above: n >= 1 and t[n-1] == '$'. */
static int text_ok(const uint8_t *t, int64_t n)
{
    return (n >= 1 && t[n - 1] == SEPB) ? 0 : -1;
}

/* ---------------------------------------------------------------------------------------- */
/* SA: sort all positions with suffix_cmp.  Parallelism is only over independent chunks that  */
/* are then merged; the order produced is the one the comparator defines.                   */
/* ---------------------------------------------------------------------------------------- */
static void merge_runs(const uint8_t *t, const int32_t *src, int32_t *dst,
                       int64_t lo, int64_t mid, int64_t hi)
{
    int64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) dst[k++] = (suffix_cmp(t, src[i], src[j]) <= 0) ? src[i++] : src[j++];
    while (i < mid) dst[k++] = src[i++];
    while (j < hi) dst[k++] = src[j++];
}

int oracle_sa(const uint8_t *t, int64_t n, int32_t *sa, int nthreads)
{
    if (text_ok(t, n)) return -1;
    if (nthreads < 1) nthreads = 1;
    for (int64_t i = 0; i < n; ++i) sa[i] = (int32_t)i;
    int64_t chunks = 1;
    while (chunks < nthreads) chunks <<= 1;
    if (n < 4096) chunks = 1;
    int64_t per = (n + chunks - 1) / chunks;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t c = 0; c < chunks; ++c) {
        int64_t lo = c * per, hi = lo + per < n ? lo + per : n;
        if (lo < hi) qsort_r(sa + lo, (size_t)(hi - lo), sizeof(int32_t), cmp_ctx, (void *)t);
    }
    if (chunks > 1) {
        int32_t *tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        if (!tmp) return -2;
        int32_t *src = sa, *dst = tmp;
        for (int64_t w = per; w < n; w *= 2) {
            int64_t npairs = (n + 2 * w - 1) / (2 * w);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
            for (int64_t pr = 0; pr < npairs; ++pr) {
                int64_t lo = pr * 2 * w;
                int64_t mid = lo + w < n ? lo + w : n;
                int64_t hi = lo + 2 * w < n ? lo + 2 * w : n;
                merge_runs(t, src, dst, lo, mid, hi);
            }
            int32_t *x = src; src = dst; dst = x;
        }
        if (src != sa) memcpy(sa, src, (size_t)n * sizeof(int32_t));
        free(tmp);
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* LCP: direct common-prefix length of each adjacent pair.                                   */
/* ---------------------------------------------------------------------------------------- */
int oracle_lcp(const uint8_t *t, int64_t n, const int32_t *sa, int32_t *lcp, int nthreads)
{
    if (text_ok(t, n)) return -1;
    if (nthreads < 1) nthreads = 1;
    lcp[0] = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t i = 1; i < n; ++i) {
        int64_t p = sa[i - 1], q = sa[i], k = 0;
        while (t[p + k] == t[q + k] && t[p + k] != SEPB) ++k;
        lcp[i] = (int32_t)k;
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* Reads: start offset and length of each read (read id = order of its separator).           */
/* ---------------------------------------------------------------------------------------- */
static int64_t read_bounds(const uint8_t *t, int64_t n, int64_t **start_out, int64_t **len_out)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) m += (t[i] == SEPB);
    int64_t *st = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    int64_t *ln = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
    int64_t r = 0, s = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (t[i] == SEPB) { st[r] = s; ln[r] = i - s; ++r; s = i + 1; }
    }
    *start_out = st;
    *len_out = ln;
    return m;
}

int64_t oracle_num_reads(const uint8_t *t, int64_t n)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) m += (t[i] == SEPB);
    return m;
}

/* Largest l in [min_len, min(|a|,|b|)] with suffix_l(a) == prefix_l(b), or 0 if none. */
static int64_t pair_overlap(const uint8_t *a, int64_t la, const uint8_t *b, int64_t lb, int64_t min_len)
{
    int64_t top = la < lb ? la : lb;
    for (int64_t l = top; l >= min_len; --l)
        if (memcmp(a + la - l, b, (size_t)l) == 0) return l;
    return 0;
}

/* Literal definition, all ordered pairs.  out may be NULL (count only).  Returns the number
 * of triples, or -1 on a malformed text.  Triples beyond cap are counted but not written. */
int64_t oracle_overlaps_brute(const uint8_t *t, int64_t n, int32_t min_len,
                              int32_t *out, int64_t cap, int nthreads)
{
    if (text_ok(t, n) || min_len < 1) return -1;
    if (nthreads < 1) nthreads = 1;
    int64_t *st, *ln;
    int64_t m = read_bounds(t, n, &st, &ln);
    int64_t *cnt = (int64_t *)calloc((size_t)(m + 1), sizeof(int64_t));
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16)
    for (int64_t a = 0; a < m; ++a) {
        int64_t c = 0;
        for (int64_t b = 0; b < m; ++b)
            if (a != b && pair_overlap(t + st[a], ln[a], t + st[b], ln[b], min_len)) ++c;
        cnt[a + 1] = c;
    }
    for (int64_t a = 0; a < m; ++a) cnt[a + 1] += cnt[a];
    int64_t total = cnt[m];
    if (out) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16)
        for (int64_t a = 0; a < m; ++a) {
            int64_t k = cnt[a];
            for (int64_t b = 0; b < m; ++b) {
                if (a == b) continue;
                int64_t l = pair_overlap(t + st[a], ln[a], t + st[b], ln[b], min_len);
                if (l) {
                    if (k < cap) { out[3 * k] = (int32_t)a; out[3 * k + 1] = (int32_t)b; out[3 * k + 2] = (int32_t)l; }
                    ++k;
                }
            }
        }
    }
    free(cnt); free(st); free(ln);
    return total;
}

/* ---------------------------------------------------------------------------------------- */
/* Exact seed-and-verify overlaps.  Every read b with |b| >= min_len is filed under a hash of  */
/* b[0..min_len).  For each read a and each start offset o with |a| - o >= min_len, the reads */
/* filed under the hash of a[o..o+min_len) are candidates; a candidate b is reported when      */
/* |b| >= |a| - o and a[o..] == b[0..|a|-o) byte for byte.  Offsets are tried in increasing     */
/* order, so the first confirmed offset for a given b is its largest overlap.                 */
/* ---------------------------------------------------------------------------------------- */
typedef struct { uint64_t h; int64_t b; } seed_t;

static uint64_t hash_bytes(const uint8_t *s, int64_t len)
{
    uint64_t h = 1469598103934665603ull; /* FNV-1a, used only as a bucket filter */
    for (int64_t i = 0; i < len; ++i) { h ^= s[i]; h *= 1099511628211ull; }
    return h;
}

static int seed_cmp(const void *x, const void *y)
{
    const seed_t *a = (const seed_t *)x, *b = (const seed_t *)y;
    if (a->h != b->h) return a->h < b->h ? -1 : 1;
    return (a->b < b->b) ? -1 : (a->b > b->b);
}

typedef struct { int32_t b, l; } hit_t;

static int hit_cmp(const void *x, const void *y)
{
    const hit_t *a = (const hit_t *)x, *b = (const hit_t *)y;
    return (a->b > b->b) - (a->b < b->b);
}

int64_t oracle_overlaps_indexed(const uint8_t *t, int64_t n, int32_t min_len,
                                int32_t *out, int64_t cap, int nthreads)
{
    if (text_ok(t, n) || min_len < 1) return -1;
    if (nthreads < 1) nthreads = 1;
    int64_t *st, *ln;
    int64_t m = read_bounds(t, n, &st, &ln);
    seed_t *seeds = (seed_t *)malloc((size_t)(m ? m : 1) * sizeof(seed_t));
    int64_t ns = 0;
    for (int64_t b = 0; b < m; ++b)
        if (ln[b] >= min_len) { seeds[ns].h = hash_bytes(t + st[b], min_len); seeds[ns].b = b; ++ns; }
    qsort(seeds, (size_t)ns, sizeof(seed_t), seed_cmp);

    hit_t **res = (hit_t **)calloc((size_t)(m ? m : 1), sizeof(hit_t *));
    int64_t *cnt = (int64_t *)calloc((size_t)(m + 1), sizeof(int64_t));
    int failed = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int64_t *stamp = (int64_t *)malloc((size_t)(m ? m : 1) * sizeof(int64_t));
        for (int64_t i = 0; i < m; ++i) stamp[i] = -1;
#pragma omp for schedule(dynamic, 64)
        for (int64_t a = 0; a < m; ++a) {
            int64_t la = ln[a];
            if (la < min_len) continue;
            const uint8_t *pa = t + st[a];
            int64_t capa = 16, k = 0;
            hit_t *h = (hit_t *)malloc((size_t)capa * sizeof(hit_t));
            for (int64_t o = 0; o + min_len <= la; ++o) {
                int64_t l = la - o;
                uint64_t key = hash_bytes(pa + o, min_len);
                /* first seed with this hash */
                int64_t lo = 0, hi = ns;
                while (lo < hi) { int64_t md = (lo + hi) / 2; if (seeds[md].h < key) lo = md + 1; else hi = md; }
                for (int64_t s = lo; s < ns && seeds[s].h == key; ++s) {
                    int64_t b = seeds[s].b;
                    if (b == a || stamp[b] == a || ln[b] < l) continue;
                    if (memcmp(pa + o, t + st[b], (size_t)l) != 0) continue;
                    stamp[b] = a;
                    if (k == capa) { capa *= 2; h = (hit_t *)realloc(h, (size_t)capa * sizeof(hit_t)); }
                    h[k].b = (int32_t)b; h[k].l = (int32_t)l; ++k;
                }
            }
            qsort(h, (size_t)k, sizeof(hit_t), hit_cmp);
            res[a] = h;
            cnt[a + 1] = k;
        }
        free(stamp);
    }
    for (int64_t a = 0; a < m; ++a) cnt[a + 1] += cnt[a];
    int64_t total = cnt[m];
    if (out) {
        for (int64_t a = 0; a < m; ++a) {
            for (int64_t j = 0; j < cnt[a + 1] - cnt[a]; ++j) {
                int64_t k = cnt[a] + j;
                if (k < cap) {
                    out[3 * k] = (int32_t)a;
                    out[3 * k + 1] = res[a][j].b;
                    out[3 * k + 2] = res[a][j].l;
                }
            }
        }
    }
    for (int64_t a = 0; a < m; ++a) free(res[a]);
    free(res); free(cnt); free(seeds); free(st); free(ln);
    (void)failed;
    return total;
}

/* ---------------------------------------------------------------------------------------- */
/* Sampled checks for sizes where the full sort is too slow.                                 */
/* ---------------------------------------------------------------------------------------- */

/* For each index i in idx[0..k): 1 if sa[i-1] < sa[i] in suffix order (i >= 1), and
 * lcp[i] (if lcp != NULL) equals the direct common prefix.  Returns the number of failures
 * and writes the first failing index to *first_bad (or -1). */
int64_t oracle_check_adjacent(const uint8_t *t, int64_t n, const int32_t *sa, const int32_t *lcp,
                              const int64_t *idx, int64_t k, int64_t *first_bad, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    int64_t bad = 0, first = -1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1024) reduction(+:bad)
    for (int64_t j = 0; j < k; ++j) {
        int64_t i = idx[j];
        int ok = 1;
        if (i < 1 || i >= n) ok = (i == 0 && (!lcp || lcp[0] == 0));
        else {
            if (suffix_cmp(t, sa[i - 1], sa[i]) >= 0) ok = 0;
            if (lcp && oracle_lcp_pair(t, n, sa[i - 1], sa[i]) != lcp[i]) ok = 0;
        }
        if (!ok) {
            ++bad;
#pragma omp critical
            { if (first < 0 || i < first) first = i; }
        }
    }
    if (first_bad) *first_bad = first;
    return bad;
}

/* Every index i in [lo, hi) (1 <= lo): 1 if sa[i-1] < sa[i] in suffix order and lcp[i] (if
 * lcp != NULL) equals the direct common prefix.  Together with a check that sa is a
 * permutation this is the whole suffix-array definition: a permutation whose adjacent suffixes
 * all ascend is the sorted order.  Returns the number of failures; the first failing index
 * goes to *first_bad (or -1).
 *
 * The same comparison as suffix_cmp / oracle_lcp_pair, organised for full-size texts: whole
 * 8-byte words are skipped while they agree and hold no separator (a word holds the byte '$'
 * exactly when some byte of w ^ 0x24..24 is zero, and a word v has a zero byte exactly when
 * (v - 0x01..01) & ~v & 0x80..80 is non-zero); the bytes from there on are compared one by one
 * as oracle_lcp_pair does, and the bytes where that stops decide the order as suffix_cmp does.
 * The test suite pins it against the byte-by-byte check above. */
static int has_sep_byte(uint64_t w)
{
    const uint64_t v = w ^ 0x2424242424242424ull;
    return ((v - 0x0101010101010101ull) & ~v & 0x8080808080808080ull) != 0;
}

int64_t oracle_check_range(const uint8_t *t, int64_t n, const int32_t *sa, const int32_t *lcp,
                           int64_t lo, int64_t hi, int64_t *first_bad, int nthreads)
{
    if (text_ok(t, n)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (lo < 1) lo = 1;
    if (hi > n) hi = n;
    int64_t bad = 0, first = -1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 65536) reduction(+:bad)
    for (int64_t i = lo; i < hi; ++i) {
        int ok = 1;
        const int64_t p = sa[i - 1], q = sa[i];
        if (p < 0 || p >= n || q < 0 || q >= n || p == q) ok = 0;
        else {
            int64_t k = 0;
            /* both suffixes end with a separator, so neither word read passes t[n-1] while no
             * separator has been met: p + k + 8 <= n holds whenever the word holds none */
            while (p + k + 8 <= n && q + k + 8 <= n) {
                uint64_t a, b;
                memcpy(&a, t + p + k, 8);
                memcpy(&b, t + q + k, 8);
                if (a != b || has_sep_byte(a)) break;
                k += 8;
            }
            while (t[p + k] == t[q + k] && t[p + k] != SEPB) ++k;
            const uint8_t x = t[p + k], y = t[q + k];
            int less;
            if (x == SEPB && y == SEPB) less = p < q;
            else if (x == SEPB) less = 1;
            else if (y == SEPB) less = 0;
            else less = x < y;
            if (!less) ok = 0;
            if (lcp && lcp[i] != k) ok = 0;
        }
        if (!ok) {
            ++bad;
#pragma omp critical
            { if (first < 0 || i < first) first = i; }
        }
    }
    if (first_bad) *first_bad = first;
    return bad;
}

/* ---------------------------------------------------------------------------------------- */
/* Pattern lookup: the SA interval of the suffixes that start with a pattern (see header).   */
/* ---------------------------------------------------------------------------------------- */

/* -1: suffix p sorts below P and does not start with it; 0: it starts with P; +1: above. */
static int suffix_vs_pattern(const uint8_t *t, int64_t p, const uint8_t *pat, int64_t m)
{
    for (int64_t k = 0; k < m; ++k) {
        uint8_t x = t[p + k];
        if (x == SEPB) return -1;  /* the suffix ends first: a separator is below every byte */
        if (x != pat[k]) return (x < pat[k]) ? -1 : 1;
    }
    return 0;
}

/* Patterns are pats[off[i] .. off[i+1]) for i < npat; lohi[2i], lohi[2i+1] receive [lo, hi).
 * Returns 0, or -1 for a pattern holding a separator or a bad text. */
int oracle_lookup(const uint8_t *t, int64_t n, const uint8_t *pats, const int64_t *off,
                  int64_t npat, int64_t *lohi, int nthreads)
{
    if (text_ok(t, n) != 0) return -1;
    for (int64_t i = 0; i < npat; ++i)
        for (int64_t k = off[i]; k < off[i + 1]; ++k)
            if (pats[k] == SEPB) return -1;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t i = 0; i < npat; ++i) {
        const uint8_t *pat = pats + off[i];
        const int64_t m = off[i + 1] - off[i];
        int64_t below = 0, occ = 0;
        for (int64_t p = 0; p < n; ++p) {
            const int c = suffix_vs_pattern(t, p, pat, m);
            if (c < 0) ++below;
            else if (c == 0) ++occ;
        }
        lohi[2 * i] = below;
        lohi[2 * i + 1] = below + occ;
    }
    return 0;
}
