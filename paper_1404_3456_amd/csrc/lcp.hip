// lcp.hip -- LCP array by Kasai's scan over text positions.
//
// The paper builds the suffix array to answer prefix tests between fragments by searching it
// (Sec. IV); the LCP array beside it turns those tests into interval walks.  For positions p in
// text order, the common prefix of suffix p with its predecessor in the suffix array is at
// least the previous one minus one (Kasai et al.), so a scan that carries that bound compares
// each position only past the carried length.  Here each thread scans one chunk of `chunk`
// consecutive positions and starts its carry at 0, which keeps the result exact while letting
// all chunks run in parallel.  Symbols are compared 32 at a time from the 2-bit packed text;
// a separator in either suffix ends the match (two separators are different symbols).
//
// Large texts store the scan's lengths by text position (the permuted LCP, written in order)
// and then gather LCP[i] = PLCP[SA[i]]: once the arrays exceed the last-level cache a random
// 4-byte gather costs about half of a random 4-byte scatter (measured 46 vs 25 G/s over 1.6 GB),
// while below it the scatter is the cheaper of the two.
#include <mutex>
#include <string>

#include "device.hpp"
#include "internal.hpp"
#include "text.hpp"

namespace saasm {

// PLCP: lcp is indexed by text position (plcp[p] = LCP[ISA[p]]) instead of by rank.
template <int CH, bool PLCP>
__global__ __launch_bounds__(256) void k_kasai(const uint4 *__restrict__ blk,
                                               const int32_t *__restrict__ sa,
                                               const int32_t *__restrict__ isa,
                                               int32_t *__restrict__ lcp, uint32_t n,
                                               uint32_t *err) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t p0 = uint64_t(c) * CH;
    if (p0 >= n) return;
    // all index loads of the chunk first (they do not depend on the carried length)
    int32_t iv[CH];
    uint32_t qv[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) iv[k] = (p0 + k < n) ? isa[p0 + k] : -1;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int32_t i = iv[k];
        // read once and never again: a non-temporal load (1.98 -> 1.88 ms on 50.1 M positions)
        qv[k] = (i > 0 && uint32_t(i) < n) ? uint32_t(__builtin_nontemporal_load(sa + i - 1)) : 0xffffffffu;
    }
    uint32_t h = 0;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const uint32_t p = uint32_t(p0) + k;
        if (p >= n) break;
        const int32_t i = iv[k];
        if (i <= 0 || uint32_t(i) >= n) {
            if (i == 0) lcp[PLCP ? p : 0] = 0;
            else raise_err(err, kErrRange);
            h = 0;
            continue;
        }
        const uint32_t q = qv[k];
        if (q >= n) {
            raise_err(err, kErrRange);
            if (PLCP) lcp[p] = 0;
            h = 0;
            continue;
        }
        // Kasai's bound leaves most positions a few symbols of new match: first compare what
        // the one 16-byte record holding each side's next symbol covers (32 - offset symbols);
        // only a match that runs past it takes the two-record windows below.
        bool done = false;
        if (p + h < n && q + h < n) {
            const uint32_t ia = p + h, ib = q + h, oa = ia & 31, ob = ib & 31;
            const uint4 x = blk[ia >> 5], y = blk[ib >> 5];
            const uint64_t ca = ((uint64_t(x.x) << 32) | x.y) << (2 * oa);
            const uint64_t cb = ((uint64_t(y.x) << 32) | y.y) << (2 * ob);
            const uint32_t sp = (x.z << oa) | (y.z << ob);
            const uint64_t d = ca ^ cb;
            const uint32_t md = d ? uint32_t(__clzll((long long)d)) >> 1 : 32u;
            const uint32_t ms = sp ? uint32_t(__clz(sp)) : 32u;
            const uint32_t kk = md < ms ? md : ms;
            const uint32_t valid = 32u - (oa > ob ? oa : ob);
            if (kk < valid) {
                h += kk;
                done = true;
            }
        }
        while (!done) {
            if (p + h >= n || q + h >= n) {  // only reachable for a text without final '$'
                raise_err(err, kErrRange);
                break;
            }
            const Window a = window_at(blk, p + h), b = window_at(blk, q + h);
            const uint64_t d = a.code ^ b.code;
            const uint32_t sp = a.sep | b.sep;
            const uint32_t md = d ? uint32_t(__clzll((long long)d)) >> 1 : 32u;
            const uint32_t ms = sp ? uint32_t(__clz(sp)) : 32u;
            const uint32_t kk = md < ms ? md : ms;
            h += kk;
            if (kk < 32) break;
        }
        lcp[PLCP ? p : uint32_t(i)] = int32_t(h);
        if (h > 0) --h;
    }
}

// LCP[i] = PLCP[SA[i]]
__global__ __launch_bounds__(256) void k_lcp_gather(const int32_t *__restrict__ sa,
                                                    const int32_t *__restrict__ plcp,
                                                    int32_t *__restrict__ lcp, uint32_t n,
                                                    uint32_t *err) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const uint32_t p = uint32_t(sa[i]);
        if (p < n) {
            lcp[i] = plcp[p];
        } else {
            lcp[i] = 0;
            raise_err(err, kErrRange);
        }
    }
}

static uint32_t g_lcp_chunk = 4;
// Texts of at least this many positions take the permuted-LCP form (4 bytes of LCP per
// position exceed the 256 MB last-level cache from about 64 M on).
static int64_t g_plcp_min_n = int64_t(1) << 26;

template <int CH>
static void launch_kasai(bool plcp, dim3 grid, hipStream_t s, const uint4 *blk, const int32_t *sa,
                         const int32_t *isa, int32_t *out, uint32_t n, uint32_t *err) {
    if (plcp) hipLaunchKernelGGL((k_kasai<CH, true>), grid, dim3(256), 0, s, blk, sa, isa, out, n, err);
    else hipLaunchKernelGGL((k_kasai<CH, false>), grid, dim3(256), 0, s, blk, sa, isa, out, n, err);
}

}  // namespace saasm

using namespace saasm;

namespace saasm {

// A failure the device found while computing the array (a byte other than A, C, G, T, '$'; a
// text without its final separator; an index out of range) replaces lcp[0], which is 0 in
// every valid array, by the negative status -- so an asynchronous call can still report it.
__global__ void k_lcp_flag(const uint32_t *err, int32_t *lcp) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t e = *err;
    if (e == 0) return;
    lcp[0] = (e & kErrAlphabet) ? SA_ERR_ALPHABET : (e & kErrNoSepEnd) ? SA_ERR_INVALID : SA_ERR_HIP;
}

int64_t lcp_ws_bytes(int64_t n) {
    if (n < 1) return -1;
    Carver c(nullptr, INT64_MAX);
    c.take<uint32_t>(packed_words(n));
    c.take<uint32_t>(sepmask_words(n));
    c.take<uint32_t>(sepmask_words(n));
    c.take<uint4>(sepmask_words(n));
    c.take<uint32_t>(64);
    if (n >= g_plcp_min_n) c.take<int32_t>(n);
    return c.off + 256;
}

int lcp_run(const uint8_t *text, int64_t n, const int32_t *sa, const int32_t *isa, int32_t *lcp,
            void *ws, int64_t ws_bytes, hipStream_t stream, int32_t *flag, int64_t span) {
    if (ws_bytes < lcp_ws_bytes(n)) return fail(SA_ERR_NOMEM, "sa_lcp: workspace too small");
    Carver c(ws, ws_bytes);
    uint32_t *packed = c.take<uint32_t>(packed_words(n));
    uint32_t *sepmask = c.take<uint32_t>(sepmask_words(n));
    uint32_t *wordcnt = c.take<uint32_t>(sepmask_words(n));
    uint4 *blk = c.take<uint4>(sepmask_words(n));
    uint32_t *err = c.take<uint32_t>(64);
    // the scattered writes of one text stay inside its own block of the array: with texts of
    // a batch below the threshold the direct form keeps its locality however large the batch
    const bool plcp = (span > 0 && span < n ? span : n) >= g_plcp_min_n;
    int32_t *pl = plcp ? c.take<int32_t>(n) : nullptr;
    SA_TRY(launch_fill_u32(err, 1, 0, stream));
    SA_TRY(launch_pack(text, n, packed, sepmask, wordcnt, err, stream));
    SA_TRY(launch_blocks(packed, sepmask, blk, sepmask_words(n), stream));
    const uint32_t chunk = g_lcp_chunk;
    const int64_t threads = (n + chunk - 1) / chunk;
    const dim3 grid(unsigned((threads + 255) / 256));
    int32_t *out = plcp ? pl : lcp;
    {
        // algorithmic bytes: isa[p] (4) + sa[isa[p]-1] (4) + lcp write (4) per position
        TimedScope ts("kasai", double(n) * 12.0, stream, double(n));
        switch (chunk) {
            case 1: launch_kasai<1>(plcp, grid, stream, blk, sa, isa, out, uint32_t(n), err); break;
            case 2: launch_kasai<2>(plcp, grid, stream, blk, sa, isa, out, uint32_t(n), err); break;
            case 4: launch_kasai<4>(plcp, grid, stream, blk, sa, isa, out, uint32_t(n), err); break;
            case 8: launch_kasai<8>(plcp, grid, stream, blk, sa, isa, out, uint32_t(n), err); break;
            default: launch_kasai<16>(plcp, grid, stream, blk, sa, isa, out, uint32_t(n), err); break;
        }
        ts.finish();
        SA_HIP(hipGetLastError());
    }
    if (plcp) {
        // sa[i] (4) + plcp[sa[i]] (4) + lcp[i] (4)
        TimedScope ts("lcp_gather", double(n) * 12.0, stream, double(n));
        int64_t g = (n + 255) / 256;
        if (g > 8192) g = 8192;
        hipLaunchKernelGGL(k_lcp_gather, dim3(unsigned(g)), dim3(256), 0, stream, sa, pl, lcp,
                           uint32_t(n), err);
        ts.finish();
        SA_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_lcp_flag, dim3(1), dim3(64), 0, stream, err, flag ? flag : lcp);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

}  // namespace saasm

extern "C" int64_t sa_lcp_ws_bytes(int64_t n) { return lcp_ws_bytes(n); }

extern "C" int sa_lcp(const uint8_t *text, int64_t n, const int32_t *sa, const int32_t *isa,
                      int32_t *lcp, void *ws, int64_t ws_bytes, hipStream_t stream) {
    if (!text || !sa || !isa || !lcp || !ws) return fail(SA_ERR_INVALID, "sa_lcp: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_lcp: n must be >= 1");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_lcp: n >= 2^31-2");
    return lcp_run(text, n, sa, isa, lcp, ws, ws_bytes, stream);
}

// ---- the LCP array without allocation ----------------------------------------------------
// For callers that cannot allocate (code under stream capture, tight serving loops): the
// workspace is one file-scope device array, which every GPU the library runs on holds until
// the process ends.  Host code never passes the array's name to a kernel (that is a host-side
// stand-in); the device address comes from hipGetSymbolAddress, once per device, with that
// device current.
namespace saasm {
constexpr int64_t kNoAllocMaxN = int64_t(1) << 24;  // characters
constexpr int64_t kNoAllocBytes = int64_t(18) << 20;
constexpr int kMaxDevices = 64;
}  // namespace saasm

static __device__ __align__(256) uint8_t scratch[saasm::kNoAllocBytes];

namespace saasm {
static std::once_flag g_scratch_once[kMaxDevices];
static void *g_scratch_ptr[kMaxDevices];
static hipError_t g_scratch_rc[kMaxDevices];
}  // namespace saasm

extern "C" int64_t sa_lcp_noalloc_max_n(void) { return kNoAllocMaxN; }

extern "C" int sa_lcp_noalloc(const uint8_t *text, int64_t n, const int32_t *sa,
                              const int32_t *isa, int32_t *lcp, hipStream_t stream) {
    if (!text || !sa || !isa || !lcp) return fail(SA_ERR_INVALID, "sa_lcp_noalloc: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_lcp_noalloc: n must be >= 1");
    if (n > kNoAllocMaxN)
        return fail(SA_ERR_TOO_LARGE, "sa_lcp_noalloc: n above its scratch limit of 2^24 characters");
    const int64_t need = lcp_ws_bytes(n);
    if (need > kNoAllocBytes) return fail(SA_ERR_NOMEM, "sa_lcp_noalloc: scratch too small");
    int dev = 0;
    SA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SA_ERR_INVALID, "sa_lcp_noalloc: device index");
    std::call_once(g_scratch_once[dev], [dev] {
        g_scratch_rc[dev] = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
    });
    if (g_scratch_rc[dev] != hipSuccess || !g_scratch_ptr[dev])
        return fail(SA_ERR_HIP, std::string("sa_lcp_noalloc: hipGetSymbolAddress: ") +
                                    hipGetErrorString(g_scratch_rc[dev]));
    // no timing events either: creating them may allocate
    timing_pause(true);
    const int rc = lcp_run(text, n, sa, isa, lcp, g_scratch_ptr[dev], need, stream);
    timing_pause(false);
    return rc;
}

// Waits for the stream and reports the status sa_lcp left in lcp[0].
extern "C" int sa_lcp_status(const int32_t *lcp, hipStream_t stream) {
    if (!lcp) return fail(SA_ERR_INVALID, "sa_lcp_status: NULL pointer");
    int32_t v = 0;
    SA_HIP(hipMemcpyAsync(&v, lcp, 4, hipMemcpyDeviceToHost, stream));
    SA_HIP(hipStreamSynchronize(stream));
    if (v == 0) return SA_OK;
    if (v == SA_ERR_ALPHABET) return fail(v, "sa_lcp: text holds a byte other than A, C, G, T, $");
    if (v == SA_ERR_INVALID) return fail(v, "sa_lcp: text must end with '$'");
    return fail(SA_ERR_HIP, "sa_lcp: device consistency check failed (sa/isa out of range)");
}

// Size from which sa_lcp takes the permuted-LCP form; returns the previous setting (min_n < 0:
// only reads it).
extern "C" int64_t sa_lcp_plcp_min(int64_t min_n) {
    const int64_t prev = g_plcp_min_n;
    if (min_n >= 0) g_plcp_min_n = min_n;
    return prev;
}

// Chunk length of the Kasai scan (positions per thread); exposed for tuning sweeps.
extern "C" int sa_lcp_set_chunk(int32_t chunk) {
    if (chunk != 1 && chunk != 2 && chunk != 4 && chunk != 8 && chunk != 16)
        return fail(SA_ERR_INVALID, "sa_lcp_set_chunk: 1, 2, 4, 8 or 16");
    g_lcp_chunk = uint32_t(chunk);
    return SA_OK;
}
