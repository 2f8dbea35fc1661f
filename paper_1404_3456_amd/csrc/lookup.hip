// lookup.hip -- the suffix-array interval of the suffixes that start with a pattern.
//
// Sec. IV: the paper builds the suffix array in order to search it, deciding whether one
// string (a fragment, the paper's "ID matching") is a prefix of a suffix.  For a pattern P over
// A, C, G, T the suffixes that start with P form one interval [lo, hi) of the array: lo is the
// first index whose suffix does not sort below P, hi the first whose suffix sorts above it.
// One thread per pattern searches for both ends of the interval together until it meets a
// suffix that starts with P, then for each end in its half.  Every suffix between two suffixes that
// share x bases with P shares them too, so each comparison resumes at the smaller of the
// prefix lengths P shares with the current interval's two ends (Manber and Myers) and then
// compares 32 bases per step from 2-bit windows; a separator ends a suffix below any base.
#include "device.hpp"
#include "internal.hpp"
#include "text.hpp"

namespace saasm {

// Pattern bytes to 2-bit codes, 16 per word (word w: bytes 16w .. 16w+15 of the concatenated
// patterns, byte 16w in the top bits); bytes other than A, C, G, T raise kErrAlphabet.
__global__ __launch_bounds__(256) void k_pack_pat(const uint8_t *__restrict__ pat, int64_t total,
                                                  uint32_t *__restrict__ packed, int64_t nwords,
                                                  uint32_t *err) {
    const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    uint32_t x = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int64_t q = w * 16 + j;
        if (q < total) {
            const uint32_t c = pat[q];
            bad |= !((c == 'A') | (c == 'C') | (c == 'G') | (c == 'T'));
            x |= (((c >> 1) ^ (c >> 2)) & 3u) << (30 - 2 * j);  // A0 C1 G2 T3
        }
    }
    packed[w] = x;
    if (bad) raise_err(err, kErrAlphabet);
}

// Compares P (m bases from base `ps` of the packed patterns) with the suffix at p, whose first
// k bases are known to equal P's.  Returns < 0 when the suffix sorts below P without starting
// with it, 0 when it starts with P, > 0 when it sorts above P; *l = their common prefix (<= m).
// The text ends with a separator, so a window never starts past it.
__device__ int cmp_suffix(const uint4 *__restrict__ blk, const uint32_t *__restrict__ ppk,
                          uint64_t ps, uint32_t m, uint32_t p, uint32_t k, uint32_t *l) {
    while (true) {
        const uint32_t rem = m - k;
        if (rem == 0) { *l = m; return 0; }
        const Window t = window_at(blk, p + k);
        const uint64_t pw = codes_at(ppk, ps + k);
        const uint64_t d = pw ^ t.code;
        const uint32_t md = d ? uint32_t(__clzll((long long)d)) >> 1 : 32u;
        const uint32_t ms = t.sep ? uint32_t(__clz(t.sep)) : 32u;
        const uint32_t c = md < ms ? md : ms;
        if (rem <= c) { *l = m; return 0; }  // P ends before any difference
        if (c == 32) { k += 32; continue; }
        *l = k + c;
        if (ms <= md) return -1;  // the suffix reaches its separator first
        const uint32_t tb = uint32_t(t.code >> (62 - 2 * c)) & 3u;
        const uint32_t pb = uint32_t(pw >> (62 - 2 * c)) & 3u;
        return tb < pb ? -1 : 1;
    }
}

__global__ __launch_bounds__(256) void k_lookup(const uint4 *__restrict__ blk,
                                                const int32_t *__restrict__ sa, uint32_t n,
                                                const uint32_t *__restrict__ ppk,
                                                const int64_t *__restrict__ off, int64_t total,
                                                uint32_t npat, int32_t *__restrict__ lohi,
                                                uint32_t *err) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npat) return;
    const int64_t a = off[i], b = off[i + 1];
    if (a < 0 || b < a || b > total || b - a > int64_t(0x7fffffff)) {
        raise_err(err, kErrRange);
        lohi[2 * i] = lohi[2 * i + 1] = 0;
        return;
    }
    const uint32_t m = uint32_t(b - a);
    // Both bounds are searched together while no suffix starting with P has been met: a
    // suffix below P moves both right, one above P moves both left.  The first suffix that
    // starts with P (index mid) splits them: lo lies in [L, mid], hi in [mid + 1, R].  An
    // absent pattern thus costs one search, a present one shares most of its path.  lL and
    // lR are P's common prefixes with the suffixes just outside the current interval.
    uint32_t L = 0, R = n, lL = 0, lR = 0, mid = 0;
    bool met = false;
    while (L < R) {
        mid = L + (R - L) / 2;
        const uint32_t p = uint32_t(sa[mid]);
        if (p >= n) { raise_err(err, kErrRange); break; }
        uint32_t l;
        const int c = cmp_suffix(blk, ppk, uint64_t(a), m, p, lL < lR ? lL : lR, &l);
        if (c < 0) { L = mid + 1; lL = l; }
        else if (c > 0) { R = mid; lR = l; }
        else { met = true; break; }
    }
    uint32_t lo = L;
    if (met) {
        // lo: first index in [L, mid] whose suffix does not sort below P (mid qualifies)
        uint32_t aL = L, aR = mid, alL = lL, alR = m;
        while (aL < aR) {
            const uint32_t am = aL + (aR - aL) / 2;
            const uint32_t p = uint32_t(sa[am]);
            if (p >= n) { raise_err(err, kErrRange); break; }
            uint32_t l;
            const int c = cmp_suffix(blk, ppk, uint64_t(a), m, p, alL < alR ? alL : alR, &l);
            if (c < 0) { aL = am + 1; alL = l; }
            else { aR = am; alR = l; }
        }
        lo = aL;
        // hi: first index in [mid + 1, R] whose suffix sorts above P
        L = mid + 1;
        lL = m;
        while (L < R) {
            const uint32_t hm = L + (R - L) / 2;
            const uint32_t p = uint32_t(sa[hm]);
            if (p >= n) { raise_err(err, kErrRange); break; }
            uint32_t l;
            const int c = cmp_suffix(blk, ppk, uint64_t(a), m, p, lL < lR ? lL : lR, &l);
            if (c <= 0) { L = hm + 1; lL = l; }
            else { R = hm; lR = l; }
        }
    }
    lohi[2 * i] = int32_t(lo);
    lohi[2 * i + 1] = int32_t(L);
}

static int64_t pat_words(int64_t total) { return (total + 15) / 16 + 4; }

}  // namespace saasm

using namespace saasm;

extern "C" int64_t sa_lookup_ws_bytes(int64_t n, int64_t pat_total) {
    if (n < 1 || pat_total < 0) return -1;
    Carver c(nullptr, INT64_MAX);
    c.take<uint32_t>(packed_words(n));
    c.take<uint32_t>(sepmask_words(n));
    c.take<uint32_t>(sepmask_words(n));
    c.take<uint4>(sepmask_words(n));
    c.take<uint32_t>(pat_words(pat_total));
    c.take<uint32_t>(64);
    return c.off + 256;
}

extern "C" int sa_lookup(const uint8_t *text, int64_t n, const int32_t *sa, const uint8_t *pat,
                         const int64_t *pat_off, int64_t pat_total, int32_t n_pat, int32_t *lohi,
                         void *ws, int64_t ws_bytes, hipStream_t stream) {
    if (!text || !sa || !pat_off || !ws || (n_pat > 0 && !lohi) || (pat_total > 0 && !pat))
        return fail(SA_ERR_INVALID, "sa_lookup: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_lookup: n must be >= 1");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_lookup: n >= 2^31-2");
    if (n_pat < 0 || pat_total < 0) return fail(SA_ERR_INVALID, "sa_lookup: negative count");
    if (ws_bytes < sa_lookup_ws_bytes(n, pat_total))
        return fail(SA_ERR_NOMEM, "sa_lookup: workspace too small");
    if (n_pat == 0) return SA_OK;
    Carver c(ws, ws_bytes);
    uint32_t *packed = c.take<uint32_t>(packed_words(n));
    uint32_t *sepmask = c.take<uint32_t>(sepmask_words(n));
    uint32_t *wordcnt = c.take<uint32_t>(sepmask_words(n));
    uint4 *blk = c.take<uint4>(sepmask_words(n));
    uint32_t *ppk = c.take<uint32_t>(pat_words(pat_total));
    uint32_t *err = c.take<uint32_t>(64);
    SA_TRY(launch_fill_u32(err, 1, 0, stream));
    SA_TRY(launch_pack(text, n, packed, sepmask, wordcnt, err, stream));
    SA_TRY(launch_blocks(packed, sepmask, blk, sepmask_words(n), stream));
    const int64_t pw = pat_words(pat_total);
    hipLaunchKernelGGL(k_pack_pat, dim3(unsigned((pw + 255) / 256)), dim3(256), 0, stream, pat,
                       pat_total, ppk, pw, err);
    SA_HIP(hipGetLastError());
    {
        // algorithmic bytes: the pattern and its two result words
        TimedScope ts("lookup", double(pat_total) + 8.0 * double(n_pat), stream, double(n_pat));
        hipLaunchKernelGGL(k_lookup, dim3(unsigned((int64_t(n_pat) + 255) / 256)), dim3(256), 0,
                           stream, blk, sa, uint32_t(n), ppk, pat_off, pat_total,
                           uint32_t(n_pat), lohi, err);
        ts.finish();
    }
    SA_HIP(hipGetLastError());
    uint32_t e = 0;
    SA_HIP(hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, stream));
    SA_HIP(hipStreamSynchronize(stream));
    if (e & kErrAlphabet)
        return fail(SA_ERR_ALPHABET, "sa_lookup: text or pattern holds a byte other than A, C, G, T (or $ in the text)");
    if (e & kErrNoSepEnd) return fail(SA_ERR_INVALID, "sa_lookup: the text must end with '$'");
    if (e & kErrRange) return fail(SA_ERR_INVALID, "sa_lookup: pattern offsets or suffix array out of range");
    if (e) return fail(SA_ERR_HIP, "sa_lookup: device check failed (code " + std::to_string(e) + ")");
    return SA_OK;
}
