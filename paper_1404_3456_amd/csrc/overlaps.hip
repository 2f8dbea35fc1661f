// overlaps.hip -- longest suffix-prefix overlap of every ordered pair of reads, by walks over
// LCP intervals of the suffix array.
//
// Sec. III: a fragment is 'fir' when it is a prefix of another (or another is a prefix of it),
// and the weighted overlap graph's edges carry overlap lengths; Sec. IV: the suffix array is
// built to answer such prefix tests.  In suffix-array order, the suffixes that share at least l
// symbols with read b's first suffix form one interval around it.  A suffix s of read a whose
// whole remainder (up to a's separator) equals the first l symbols of b ends with a separator
// that sorts below every base, so it lies just before b's suffix in that interval with
// LCP(s, b) == l == length of s; when l == |b| (b is all of s) it lies before b when a < b and
// after b when a > b (separator order).  Hence, per read b with |b| >= min_len:
//   left walk:  k = j-1, j-2, ...  (j = isa[start of b]) with run = min lcp over (k, j];
//               stop when run < min_len; report (a, b, run) when suffix sa[k] has exactly
//               run symbols before its separator and a != b;
//   right walk: k = j+1, ...  while lcp[k] >= |b|; report (a, b, |b|) when suffix sa[k] has
//               exactly |b| symbols before its separator and a != b.
// A pair can be reported more than once (a read with periodic structure); the longest wins.
// Candidates are counted, scanned, written as (a << 32 | b, l), sorted by a with the stable
// radix sort (keeping b order within a), and reduced to one row per (a, b) with the largest l.
#include "device.hpp"
#include "internal.hpp"

namespace saasm {

__device__ __forceinline__ uint32_t read_of(const uint32_t *__restrict__ sepmask,
                                            const int32_t *__restrict__ sepcnt, uint32_t s) {
    const uint32_t w = s >> 5, o = s & 31;
    const uint32_t before = o ? (sepmask[w] >> (32 - o)) : 0u;  // separators at 32w .. s-1
    return uint32_t(sepcnt[w]) + __popc(before);
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_ovl_walk(
    const int32_t *__restrict__ sa, const int32_t *__restrict__ isa,
    const int32_t *__restrict__ lcp, const int32_t *__restrict__ read_end,
    const uint32_t *__restrict__ sepmask, const int32_t *__restrict__ sepcnt, uint32_t n,
    uint32_t m, int32_t min_len, uint32_t *__restrict__ counts, const int64_t *__restrict__ offs,
    uint64_t *__restrict__ hkeys, uint32_t *__restrict__ hvals, uint32_t *err) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m) return;
    const int32_t start = b == 0 ? 0 : read_end[b - 1] + 1;
    const int32_t len = read_end[b] - start;
    uint32_t c = 0;
    int64_t o = FILL ? offs[b] : 0;
    if (len >= min_len) {
        const int32_t j = isa[start];
        if (j < 0 || uint32_t(j) >= n) {
            raise_err(err, kErrRange);
        } else {
            int32_t run = len;
            for (int32_t k = j; k > 0; --k) {
                const int32_t l = lcp[k];
                run = l < run ? l : run;
                if (run < min_len) break;
                const uint32_t s = uint32_t(sa[k - 1]);
                const uint32_t a = read_of(sepmask, sepcnt, s);
                if (a >= m) { raise_err(err, kErrRange); break; }
                if (read_end[a] - int32_t(s) == run && a != b) {
                    if (FILL) {
                        hkeys[o] = (uint64_t(a) << 32) | b;
                        hvals[o] = uint32_t(run);
                        ++o;
                    }
                    ++c;
                }
            }
            for (uint32_t k = uint32_t(j) + 1; k < n && lcp[k] >= len; ++k) {
                const uint32_t s = uint32_t(sa[k]);
                const uint32_t a = read_of(sepmask, sepcnt, s);
                if (a >= m) { raise_err(err, kErrRange); break; }
                if (read_end[a] - int32_t(s) == len && a != b) {
                    if (FILL) {
                        hkeys[o] = (uint64_t(a) << 32) | b;
                        hvals[o] = uint32_t(len);
                        ++o;
                    }
                    ++c;
                }
            }
        }
    }
    if (!FILL) counts[b] = c;
}

// first[i] = 1 when row i starts a run of equal (a, b) keys
__global__ __launch_bounds__(256) void k_run_heads(const uint64_t *__restrict__ keys, uint32_t r,
                                                   uint32_t *__restrict__ first) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r) return;
    first[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_run_write(const uint64_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ vals, uint32_t r,
                                                   const uint32_t *__restrict__ first,
                                                   const int64_t *__restrict__ pos,
                                                   int32_t *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r || !first[i]) return;
    const uint64_t k = keys[i];
    uint32_t best = vals[i];
    for (uint32_t j = i + 1; j < r && keys[j] == k; ++j) best = vals[j] > best ? vals[j] : best;
    const int64_t o = pos[i];
    out[3 * o] = int32_t(k >> 32);
    out[3 * o + 1] = int32_t(k & 0xffffffffu);
    out[3 * o + 2] = int32_t(best);
}

struct OvlFixed {
    uint32_t *packed, *sepmask, *wordcnt;
    int32_t *sepcnt, *read_end;
    uint32_t *counts;
    int64_t *offs;
    uint64_t *lbflags;
    uint32_t *tick;
    uint32_t *ctr;  // [0] err; [2..3] m (int32 at ctr+2); int64 totals at ctr+8, ctr+10
};

// Text-sized part (packed text, separator rank structure) then read-sized part (m reads).
static void carve_fixed(Carver &c, int64_t n, int64_t m, OvlFixed *F) {
    F->packed = c.take<uint32_t>(packed_words(n));
    F->sepmask = c.take<uint32_t>(sepmask_words(n));
    F->wordcnt = c.take<uint32_t>(sepmask_words(n));
    F->sepcnt = c.take<int32_t>(sepmask_words(n));
    F->tick = c.take<uint32_t>(64);
    F->ctr = c.take<uint32_t>(64);
    const int64_t scan_n = sepmask_words(n) > m + 1 ? sepmask_words(n) : m + 1;
    F->lbflags = c.take<uint64_t>(scan_flags_words(scan_n) + 16);
    F->read_end = c.take<int32_t>(m);
    F->counts = c.take<uint32_t>(m + 1);
    F->offs = c.take<int64_t>(m + 1);
}

struct OvlHits {
    SortBufs sb;
    uint32_t *first;
    int64_t *pos;
    uint64_t *lbflags;
};

static void carve_hits(Carver &c, int64_t r, const Tune &t, OvlHits *H) {
    carve_sort(c, r, 32, t, &H->sb, true);
    H->first = c.take<uint32_t>(r + 1);
    H->pos = c.take<int64_t>(r + 1);
    H->lbflags = c.take<uint64_t>(scan_flags_words(r + 1) + 16);
}

static int bits_for_u(int64_t v) {
    int b = 0;
    while ((int64_t(1) << b) <= v) ++b;
    return b;
}

}  // namespace saasm

using namespace saasm;

extern "C" int64_t sa_overlaps_ws_bytes(int64_t n, int64_t m, int64_t candidates) {
    if (n < 1 || candidates < 0) return -1;
    if (m <= 0 || m > n) m = n;
    Tune t;
    resolve_tuning(nullptr, &t);
    Carver c(nullptr, INT64_MAX);
    OvlFixed F;
    carve_fixed(c, n, m, &F);
    if (candidates > 0) {
        OvlHits H;
        carve_hits(c, candidates, t, &H);
    }
    return c.off + 256;
}

extern "C" int sa_overlaps(const uint8_t *text, int64_t n, const int32_t *sa, const int32_t *isa,
                           const int32_t *lcp, int32_t min_len, int32_t *out, int64_t cap,
                           int64_t *n_out_h, void *ws, int64_t ws_bytes, int64_t *ws_needed_h,
                           hipStream_t stream) {
    if (!text || !sa || !isa || !lcp || !ws || !n_out_h || (cap > 0 && !out))
        return fail(SA_ERR_INVALID, "sa_overlaps: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_overlaps: n must be >= 1");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_overlaps: n >= 2^31-2");
    if (min_len < 1) return fail(SA_ERR_INVALID, "sa_overlaps: min_len must be >= 1");
    if (cap < 0) return fail(SA_ERR_INVALID, "sa_overlaps: cap < 0");
    // the text-sized part must fit before the read count is known
    const int64_t fixed = sa_overlaps_ws_bytes(n, 1, 0);
    if (ws_needed_h) *ws_needed_h = fixed;
    if (ws_bytes < fixed) return fail(SA_ERR_NOMEM, "sa_overlaps: workspace too small");
    Tune t;
    resolve_tuning(nullptr, &t);
    hipStream_t s = stream;
    OvlFixed F;
    {
        Carver c0(ws, ws_bytes);
        carve_fixed(c0, n, 1, &F);  // pack area and counters only; read arrays carved below
    }
    SA_TRY(launch_fill_u32(F.ctr, 64, 0, s));
    SA_TRY(launch_pack(text, n, F.packed, F.sepmask, F.wordcnt, F.ctr, s));
    const int64_t nw = (n + 31) / 32;
    SA_TRY(launch_scan_u32_i32(F.wordcnt, F.sepcnt, nw, reinterpret_cast<int32_t *>(F.ctr + 2),
                               F.lbflags, F.tick, F.ctr, s));
    uint32_t host[4];
    int32_t lcp0 = 0;
    SA_HIP(hipMemcpyAsync(host, F.ctr, 16, hipMemcpyDeviceToHost, s));
    SA_HIP(hipMemcpyAsync(&lcp0, lcp, 4, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    timing_flush();
    // sa_lcp leaves a failure it found on the device in lcp[0] (0 in every valid array)
    if (lcp0 < 0) return fail(lcp0 == SA_ERR_ALPHABET || lcp0 == SA_ERR_INVALID ? lcp0 : SA_ERR_HIP,
                              "sa_overlaps: the LCP array carries a failure from sa_lcp");
    if (lcp0 != 0) return fail(SA_ERR_INVALID, "sa_overlaps: lcp[0] must be 0");
    if (host[0] & kErrAlphabet) return fail(SA_ERR_ALPHABET, "text holds a byte other than A, C, G, T, $");
    if (host[0] & kErrNoSepEnd) return fail(SA_ERR_INVALID, "text must end with '$'");
    if (host[0]) return fail(SA_ERR_HIP, "device consistency check failed");
    const int64_t m = int32_t(host[2]);
    if (m < 1 || m > n) return fail(SA_ERR_HIP, "sa_overlaps: bad read count");
    {
        const int64_t need_m = sa_overlaps_ws_bytes(n, m, 0);
        if (ws_needed_h) *ws_needed_h = need_m;
        if (ws_bytes < need_m) return fail(SA_ERR_NOMEM, "sa_overlaps: workspace too small for the reads");
    }
    Carver c(ws, ws_bytes);
    carve_fixed(c, n, m, &F);  // same text-sized part; read arrays now sized by m
    SA_TRY(launch_read_ends(F.sepmask, F.sepcnt, n, F.read_end, s));

    // count candidates per read, then scan to offsets
    const unsigned rgrid = unsigned((m + 255) / 256);
    {
        TimedScope ts("overlap_walk", double(m) * 12.0, s, double(m));
        hipLaunchKernelGGL(k_ovl_walk<false>, dim3(rgrid), dim3(256), 0, s, sa, isa, lcp,
                           F.read_end, F.sepmask, F.sepcnt, uint32_t(n), uint32_t(m), min_len,
                           F.counts, nullptr, nullptr, nullptr, F.ctr);
        ts.finish();
        SA_HIP(hipGetLastError());
    }
    int64_t *tot = reinterpret_cast<int64_t *>(F.ctr + 8);
    SA_TRY(launch_scan_u32_i64(F.counts, F.offs, m, tot, F.lbflags, F.tick, F.ctr, s));
    int64_t r = 0;
    uint32_t e = 0;
    SA_HIP(hipMemcpyAsync(&r, tot, 8, hipMemcpyDeviceToHost, s));
    SA_HIP(hipMemcpyAsync(&e, F.ctr, 4, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    timing_flush();
    if (e) return fail(SA_ERR_HIP, "sa_overlaps: device consistency check failed (code " + std::to_string(e) + ")");
    if (r >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_overlaps: more than 2^31-2 candidate matches");
    const int64_t need = sa_overlaps_ws_bytes(n, m, r);
    if (ws_needed_h) *ws_needed_h = need;
    if (ws_bytes < need) return fail(SA_ERR_NOMEM, "sa_overlaps: workspace too small for " + std::to_string(r) + " candidates");
    if (r == 0) {
        *n_out_h = 0;
        return SA_OK;
    }
    OvlHits H;
    carve_hits(c, r, t, &H);
    H.sb.err = F.ctr;
    SA_TRY(launch_fill_u32(F.tick, 64, 0, s));
    {
        TimedScope ts("overlap_walk", double(m) * 12.0 + double(r) * 12.0, s, double(m));
        hipLaunchKernelGGL(k_ovl_walk<true>, dim3(rgrid), dim3(256), 0, s, sa, isa, lcp,
                           F.read_end, F.sepmask, F.sepcnt, uint32_t(n), uint32_t(m), min_len,
                           nullptr, F.offs, H.sb.keys[0], H.sb.vals[0], F.ctr);
        ts.finish();
        SA_HIP(hipGetLastError());
    }
    int cur = 0;
    const int abits = bits_for_u(m - 1);
    if (abits > 0) {
        SA_TRY(sort_prepare(H.sb, r, abits, t, s));
        int nparts = 0;
        SA_TRY(launch_hist(H.sb, 0, r, 32, abits, t, s, &nparts));
        SA_TRY(sort_run(H.sb, 0, nullptr, r, 32, abits, t, nparts, s, &cur));
    }
    const unsigned hgrid = unsigned((r + 255) / 256);
    hipLaunchKernelGGL(k_run_heads, dim3(hgrid), dim3(256), 0, s, H.sb.keys[cur], uint32_t(r), H.first);
    SA_HIP(hipGetLastError());
    int64_t *utot = reinterpret_cast<int64_t *>(F.ctr + 10);
    SA_TRY(launch_scan_u32_i64(H.first, H.pos, r, utot, H.lbflags, F.tick, F.ctr, s));
    int64_t u = 0;
    SA_HIP(hipMemcpyAsync(&u, utot, 8, hipMemcpyDeviceToHost, s));
    SA_HIP(hipMemcpyAsync(&e, F.ctr, 4, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    timing_flush();
    if (e) return fail(SA_ERR_HIP, "sa_overlaps: device consistency check failed (code " + std::to_string(e) + ")");
    *n_out_h = u;
    if (u > cap) return fail(SA_ERR_CAPACITY, "sa_overlaps: output holds " + std::to_string(cap) + " rows, need " + std::to_string(u));
    hipLaunchKernelGGL(k_run_write, dim3(hgrid), dim3(256), 0, s, H.sb.keys[cur], H.sb.vals[cur],
                       uint32_t(r), H.first, H.pos, out);
    SA_HIP(hipGetLastError());
    SA_HIP(hipStreamSynchronize(s));
    return SA_OK;
}
