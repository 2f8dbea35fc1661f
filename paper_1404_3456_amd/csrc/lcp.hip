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
#include "device.hpp"
#include "internal.hpp"
#include "text.hpp"

namespace saasm {

template <int CH>
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
        qv[k] = (i > 0 && uint32_t(i) < n) ? uint32_t(sa[i - 1]) : 0xffffffffu;
    }
    uint32_t h = 0;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const uint32_t p = uint32_t(p0) + k;
        if (p >= n) break;
        const int32_t i = iv[k];
        if (i <= 0 || uint32_t(i) >= n) {
            if (i == 0) lcp[0] = 0;
            else raise_err(err, kErrRange);
            h = 0;
            continue;
        }
        const uint32_t q = qv[k];
        if (q >= n) {
            raise_err(err, kErrRange);
            h = 0;
            continue;
        }
        while (true) {
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
        lcp[i] = int32_t(h);
        if (h > 0) --h;
    }
}

static uint32_t g_lcp_chunk = 4;

}  // namespace saasm

using namespace saasm;

extern "C" int64_t sa_lcp_ws_bytes(int64_t n) {
    if (n < 1) return -1;
    Carver c(nullptr, INT64_MAX);
    c.take<uint32_t>(packed_words(n));
    c.take<uint32_t>(sepmask_words(n));
    c.take<uint32_t>(sepmask_words(n));
    c.take<uint4>(sepmask_words(n));
    c.take<uint32_t>(64);
    return c.off + 256;
}

extern "C" int sa_lcp(const uint8_t *text, int64_t n, const int32_t *sa, const int32_t *isa,
                      int32_t *lcp, void *ws, int64_t ws_bytes, hipStream_t stream) {
    if (!text || !sa || !isa || !lcp || !ws) return fail(SA_ERR_INVALID, "sa_lcp: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_lcp: n must be >= 1");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_lcp: n >= 2^31-2");
    if (ws_bytes < sa_lcp_ws_bytes(n)) return fail(SA_ERR_NOMEM, "sa_lcp: workspace too small");
    Carver c(ws, ws_bytes);
    uint32_t *packed = c.take<uint32_t>(packed_words(n));
    uint32_t *sepmask = c.take<uint32_t>(sepmask_words(n));
    uint32_t *wordcnt = c.take<uint32_t>(sepmask_words(n));
    uint4 *blk = c.take<uint4>(sepmask_words(n));
    uint32_t *err = c.take<uint32_t>(64);
    SA_TRY(launch_fill_u32(err, 1, 0, stream));
    SA_TRY(launch_pack(text, n, packed, sepmask, wordcnt, err, stream));
    SA_TRY(launch_blocks(packed, sepmask, blk, sepmask_words(n), stream));
    const uint32_t chunk = g_lcp_chunk;
    const int64_t threads = (n + chunk - 1) / chunk;
    const dim3 grid(unsigned((threads + 255) / 256)), block(256);
    // algorithmic bytes: isa[p] (4) + sa[isa[p]-1] (4) + lcp write (4) per position
    TimedScope ts("kasai", double(n) * 12.0, stream);
    switch (chunk) {
        case 1: hipLaunchKernelGGL(k_kasai<1>, grid, block, 0, stream, blk, sa, isa, lcp, uint32_t(n), err); break;
        case 2: hipLaunchKernelGGL(k_kasai<2>, grid, block, 0, stream, blk, sa, isa, lcp, uint32_t(n), err); break;
        case 4: hipLaunchKernelGGL(k_kasai<4>, grid, block, 0, stream, blk, sa, isa, lcp, uint32_t(n), err); break;
        case 8: hipLaunchKernelGGL(k_kasai<8>, grid, block, 0, stream, blk, sa, isa, lcp, uint32_t(n), err); break;
        default: hipLaunchKernelGGL(k_kasai<16>, grid, block, 0, stream, blk, sa, isa, lcp, uint32_t(n), err); break;
    }
    ts.finish();
    SA_HIP(hipGetLastError());
    return SA_OK;
}

// Chunk length of the Kasai scan (positions per thread); exposed for tuning sweeps.
extern "C" int sa_lcp_set_chunk(int32_t chunk) {
    if (chunk != 1 && chunk != 2 && chunk != 4 && chunk != 8 && chunk != 16)
        return fail(SA_ERR_INVALID, "sa_lcp_set_chunk: 1, 2, 4, 8 or 16");
    g_lcp_chunk = uint32_t(chunk);
    return SA_OK;
}
