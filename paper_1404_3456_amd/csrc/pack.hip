// pack.hip -- validation + 2-bit packing of the text, scans, read ends, fills, copy.
//
// Sec. III: DNA is a string over A, C, G, T and a fragment is a substring; the fragments are
// laid end to end, each closed by its own separator.  Packing keeps two bits per base (A=0,
// C=1, G=2, T=3) with base 0 of a word in its top bits, so that comparing two 64-bit windows
// as integers compares 32 bases lexicographically, and one separator bit per position.
#include "device.hpp"
#include "internal.hpp"

namespace saasm {

int64_t sepmask_words(int64_t n) { return (n + 31) / 32 + 4; }
int64_t packed_words(int64_t n) { return 2 * sepmask_words(n); }

// One thread per 32 text positions: one separator-mask word and two packed words.  Words past
// the end of the text are written as zeros (padding that window reads may touch).
__global__ __launch_bounds__(256) void k_pack(const uint8_t *__restrict__ text, int64_t n,
                                              uint32_t *__restrict__ packed,
                                              uint32_t *__restrict__ sepmask,
                                              uint32_t *__restrict__ wordcnt, int64_t nwords,
                                              uint32_t *err) {
    int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    int64_t p0 = w * 32;
    uint32_t hiw = 0, low = 0, sep = 0;
    bool bad = false;
    if (p0 < n) {
        uint8_t b[32];
        const bool full = (p0 + 32 <= n) && ((reinterpret_cast<uintptr_t>(text) & 15) == 0);
        if (full) {
            uint4 a = *reinterpret_cast<const uint4 *>(text + p0);
            uint4 c = *reinterpret_cast<const uint4 *>(text + p0 + 16);
            uint32_t wv[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
#pragma unroll
            for (int j = 0; j < 32; ++j) b[j] = uint8_t(wv[j >> 2] >> (8 * (j & 3)));
        } else {
#pragma unroll
            for (int j = 0; j < 32; ++j) b[j] = (p0 + j < n) ? text[p0 + j] : uint8_t('A');
        }
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            uint32_t c = b[j];
            bool in = p0 + j < n;
            bool is_sep = (c == '$') && in;
            bool ok = (c == 'A') | (c == 'C') | (c == 'G') | (c == 'T') | (c == '$');
            bad |= !ok;
            uint32_t code = is_sep ? 0u : (((c >> 1) ^ (c >> 2)) & 3u);  // A0 C1 G2 T3
            if (!in) code = 0;
            if (j < 16) hiw |= code << (30 - 2 * j);
            else low |= code << (30 - 2 * (j - 16));
            sep |= uint32_t(is_sep) << (31 - j);
        }
        if (p0 <= n - 1 && n - 1 < p0 + 32) {
            if (b[(n - 1) - p0] != '$') raise_err(err, kErrNoSepEnd);
        }
    }
    packed[2 * w] = hiw;
    packed[2 * w + 1] = low;
    sepmask[w] = sep;
    wordcnt[w] = __popc(sep);
    if (bad) raise_err(err, kErrAlphabet);
}

int launch_pack(const uint8_t *text, int64_t n, uint32_t *packed, uint32_t *sepmask,
                uint32_t *wordcnt, uint32_t *err, hipStream_t s) {
    int64_t nw = sepmask_words(n);
    TimedScope ts("pack", double(n) + double(nw) * 16.0, s, double(n));
    hipLaunchKernelGGL(k_pack, dim3(unsigned((nw + 255) / 256)), dim3(256), 0, s, text, n, packed,
                       sepmask, wordcnt, nw, err);
    ts.finish();
    SA_HIP(hipGetLastError());
    return SA_OK;
}

// Block layout of the text for random-access windows (see text.hpp): record b = {codes of
// positions 32b..32b+15, codes of 32b+16..32b+31, separator bits of 32b..32b+31, 0}.
__global__ __launch_bounds__(256) void k_blocks(const uint32_t *__restrict__ packed,
                                                const uint32_t *__restrict__ sepmask,
                                                uint4 *__restrict__ blk, int64_t nrec) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nrec) return;
    blk[b] = make_uint4(packed[2 * b], packed[2 * b + 1], sepmask[b], 0u);
}

int launch_blocks(const uint32_t *packed, const uint32_t *sepmask, uint4 *blk, int64_t nrec,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_blocks, dim3(unsigned((nrec + 255) / 256)), dim3(256), 0, s, packed,
                       sepmask, blk, nrec);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

// ---- exclusive scan with decoupled look-back ------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

int64_t scan_flags_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

template <class OutT>
__global__ __launch_bounds__(kScanBlock) void k_scan_excl(const uint32_t *__restrict__ in,
                                                          OutT *__restrict__ out, int64_t n,
                                                          OutT *total_out, uint64_t *lbflags,
                                                          uint32_t *tick, uint32_t *err) {
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    __shared__ uint64_t s_wsum[kScanBlock / kWave];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    if (tid == 0) s_tile = ticket(tick);
    __syncthreads();
    const int tile = int(s_tile);
    const int64_t base = int64_t(tile) * kScanTile + int64_t(tid) * kScanItems;
    uint32_t v[kScanItems];
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < n) ? in[base + j] : 0u;
        sum += v[j];
    }
    uint64_t inc = wave_incl_scan<SumOp>(sum);
    if (lane == kWave - 1) s_wsum[wave] = inc;
    __syncthreads();
    uint64_t before = 0, tile_total = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / kWave; ++w) {
        if (uint32_t(w) < wave) before += s_wsum[w];
        tile_total += s_wsum[w];
    }
    if (wave == 0) {
        uint64_t ex = lookback_tile<SumOp>(lbflags, tile, tile_total, err);
        if (lane == 0) s_excl = ex;
    }
    __syncthreads();
    uint64_t run = s_excl + before + inc - sum;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = OutT(run);
        run += v[j];
    }
    if (tid == 0 && int64_t(tile + 1) * kScanTile >= n) *total_out = OutT(s_excl + tile_total);
}

template <class OutT>
static int launch_scan(const uint32_t *in, OutT *out, int64_t n, OutT *total_out,
                       uint64_t *lbflags, uint32_t *tick, uint32_t *err, hipStream_t s) {
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 0) tiles = 1;
    SA_TRY(launch_fill_u64(lbflags, tiles, 0, s));
    SA_TRY(launch_fill_u32(tick, 1, 0, s));
    hipLaunchKernelGGL(k_scan_excl<OutT>, dim3(unsigned(tiles)), dim3(kScanBlock), 0, s, in, out,
                       n, total_out, lbflags, tick, err);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

int launch_scan_u32_i32(const uint32_t *in, int32_t *out, int64_t n, int32_t *total_out,
                        uint64_t *lbflags, uint32_t *tick, uint32_t *err, hipStream_t s) {
    return launch_scan<int32_t>(in, out, n, total_out, lbflags, tick, err, s);
}
int launch_scan_u32_i64(const uint32_t *in, int64_t *out, int64_t n, int64_t *total_out,
                        uint64_t *lbflags, uint32_t *tick, uint32_t *err, hipStream_t s) {
    return launch_scan<int64_t>(in, out, n, total_out, lbflags, tick, err, s);
}

// ---- separator positions (read ends) ------------------------------------------------------
__global__ __launch_bounds__(256) void k_read_ends(const uint32_t *__restrict__ sepmask,
                                                   const int32_t *__restrict__ sepcnt,
                                                   int64_t nw, int32_t *__restrict__ read_end) {
    int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    uint32_t bits = sepmask[w];
    int32_t k = sepcnt[w];
    while (bits) {
        int j = __clz(bits);  // bit 31-j <-> position 32w+j
        read_end[k++] = int32_t(w * 32 + j);
        bits &= ~(0x80000000u >> j);
    }
}

int launch_read_ends(const uint32_t *sepmask, const int32_t *sepcnt, int64_t n, int32_t *read_end,
                     hipStream_t s) {
    int64_t nw = (n + 31) / 32;
    hipLaunchKernelGGL(k_read_ends, dim3(unsigned((nw + 255) / 256)), dim3(256), 0, s, sepmask,
                       sepcnt, nw, read_end);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

// ---- fills and copy ------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_fill(T *p, int64_t n, T v) {
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

static unsigned fill_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return unsigned(b);
}

int launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return SA_OK;
    // 16-byte aligned bulk as uint4 when possible
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && n >= 4) {
        int64_t q = n / 4;
        hipLaunchKernelGGL(k_fill<uint4>, dim3(fill_grid(q)), dim3(256), 0, s,
                           reinterpret_cast<uint4 *>(p), q, make_uint4(v, v, v, v));
        SA_HIP(hipGetLastError());
        if (n % 4) {
            hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(256), 0, s, p + 4 * q, n % 4, v);
            SA_HIP(hipGetLastError());
        }
        return SA_OK;
    }
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

int launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0) return SA_OK;
    hipLaunchKernelGGL(k_fill<uint64_t>, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

__global__ __launch_bounds__(256) void k_copy_u32(uint32_t *__restrict__ dst,
                                                  const uint32_t *__restrict__ src, int64_t n) {
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace saasm

using namespace saasm;

extern "C" int64_t sa_packed_words(int64_t n) { return n < 0 ? 0 : packed_words(n); }
extern "C" int64_t sa_sepmask_words(int64_t n) { return n < 0 ? 0 : sepmask_words(n); }

extern "C" int sa_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t stream) {
    if (n < 0 || (n > 0 && (!dst || !src))) return fail(SA_ERR_INVALID, "sa_copy_u32: bad arguments");
    if (n == 0) return SA_OK;
    unsigned grid = unsigned((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    hipLaunchKernelGGL(k_copy_u32, dim3(grid), dim3(256), 0, stream, dst, src, n);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

extern "C" int64_t sa_pack_ws_bytes(int64_t n) {
    if (n < 1) return -1;
    Carver c(nullptr, INT64_MAX);
    c.take<uint32_t>(sepmask_words(n));  // per-word separator counts
    c.take<int32_t>(sepmask_words(n));   // their exclusive scan
    c.take<uint64_t>(scan_flags_words(sepmask_words(n)) + 16);
    c.take<uint32_t>(64);
    c.take<uint32_t>(64);
    return c.off + 256;
}

extern "C" int sa_pack(const uint8_t *text, int64_t n, uint32_t *packed, uint32_t *sepmask,
                       int32_t *read_end, int64_t cap_reads, int64_t *m_h, void *ws,
                       int64_t ws_bytes, hipStream_t stream) {
    if (!text || !packed || !sepmask || !m_h || !ws) return fail(SA_ERR_INVALID, "sa_pack: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_pack: n must be >= 1");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_pack: n >= 2^31-2");
    if (ws_bytes < sa_pack_ws_bytes(n)) return fail(SA_ERR_NOMEM, "sa_pack: workspace too small");
    Carver c(ws, ws_bytes);
    uint32_t *wordcnt = c.take<uint32_t>(sepmask_words(n));
    int32_t *sepcnt = c.take<int32_t>(sepmask_words(n));
    uint64_t *lbflags = c.take<uint64_t>(scan_flags_words(sepmask_words(n)) + 16);
    uint32_t *tick = c.take<uint32_t>(64);
    uint32_t *ctr = c.take<uint32_t>(64);
    SA_TRY(launch_fill_u32(ctr, 64, 0, stream));
    SA_TRY(launch_pack(text, n, packed, sepmask, wordcnt, ctr, stream));
    const int64_t nw = (n + 31) / 32;
    SA_TRY(launch_scan_u32_i32(wordcnt, sepcnt, nw, reinterpret_cast<int32_t *>(ctr + 2), lbflags,
                               tick, ctr, stream));
    uint32_t host[4];
    SA_HIP(hipMemcpyAsync(host, ctr, 16, hipMemcpyDeviceToHost, stream));
    SA_HIP(hipStreamSynchronize(stream));
    timing_flush();
    if (host[0] & kErrAlphabet) return fail(SA_ERR_ALPHABET, "text holds a byte other than A, C, G, T, $");
    if (host[0] & kErrNoSepEnd) return fail(SA_ERR_INVALID, "text must end with '$'");
    if (host[0]) return fail(SA_ERR_HIP, "sa_pack: device consistency check failed");
    const int64_t m = int32_t(host[2]);
    *m_h = m;
    if (read_end) {
        if (cap_reads < m) return fail(SA_ERR_CAPACITY, "sa_pack: read_end holds fewer than m entries");
        SA_TRY(launch_read_ends(sepmask, sepcnt, n, read_end, stream));
        SA_HIP(hipStreamSynchronize(stream));
    }
    return SA_OK;
}
