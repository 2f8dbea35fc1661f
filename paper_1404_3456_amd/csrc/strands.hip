// strands.hip -- overlaps on both strands: every read indexed with its reverse complement.
//
// The paper's overlap definition (Sec. III) lets the second fragment appear reversed and
// complemented (A <-> T, C <-> G), since a shotgun read can come from either strand.  Appending
// the reverse complement of the whole text turns those overlaps into ordinary suffix-prefix
// overlaps: the doubled text T + rc(T without its last '$') + '$' holds reads 0..m-1 as given
// and, as read m+k, the reverse complement of read m-1-k.  Its suffix array, LCP array and
// overlaps come from the usual entry points; sa_strand_rows then names each row by the two
// original reads and how they meet (strand 0: a then b; 1: a then rc(b); 2: rc(a) then b),
// drops rows that pair a read with itself and rows that repeat another in mirror image, and
// sorts them by (a, b, strand).
#include "device.hpp"
#include "internal.hpp"

namespace saasm {

__device__ __forceinline__ uint8_t complement(uint8_t c) {
    switch (c) {
        case 'A': return 'T';
        case 'C': return 'G';
        case 'G': return 'C';
        case 'T': return 'A';
        default: return c;  // '$' (and bytes the next pack step rejects) unchanged
    }
}

// Thread i: out[i] = text[i]; out[n + i] = complement(text[n - 2 - i]) for i < n - 1, and
// out[2n - 1] = '$'.  Adds the separators of text to *m_dev.
__global__ __launch_bounds__(256) void k_revcomp(const uint8_t *__restrict__ text, int64_t n,
                                                 uint8_t *__restrict__ out,
                                                 unsigned long long *m_dev) {
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    bool sep = false;
    if (i < n) {
        const uint8_t c = text[i];
        out[i] = c;
        sep = c == '$';
        out[n + i] = i < n - 1 ? complement(text[n - 2 - i]) : uint8_t('$');
    }
    const uint64_t b = ballot(sep);
    if (lane_id() == 0 && b) atomicAdd(&s_cnt, uint32_t(popc64(b)));
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(m_dev, (unsigned long long)s_cnt);
}

// Row i = (x, y, l) of the doubled text's overlaps (2m reads; read m+k is the reverse
// complement of read m-1-k).  Named (a, b, strand):
//   x <  m, y <  m : a = x, b = y,        strand 0 (the end of a meets the start of b)
//   x <  m, y >= m : a = x, b = 2m-1-y,   strand 1 (the end of a meets the start of rc(b))
//   x >= m, y <  m : a = 2m-1-x, b = y,   strand 2 (the end of rc(a) meets the start of b)
//   x >= m, y >= m : dropped -- rc(a) before rc(b) is b before a, already a strand-0 row.
// Rows pairing a read with itself (a == b) are dropped.  key = (a, b, strand).
__global__ __launch_bounds__(256) void k_strand_keys(const int32_t *__restrict__ rows, int64_t r,
                                                     uint32_t m, uint32_t *__restrict__ keep,
                                                     uint64_t *__restrict__ key,
                                                     uint32_t *err) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= r) return;
    const uint32_t x = uint32_t(rows[3 * i]), y = uint32_t(rows[3 * i + 1]);
    if (x >= 2 * m || y >= 2 * m) {
        raise_err(err, kErrRange);
        keep[i] = 0;
        return;
    }
    const bool xf = x < m, yf = y < m;
    const uint32_t a = xf ? x : 2 * m - 1 - x, b = yf ? y : 2 * m - 1 - y;
    const uint32_t strand = xf ? (yf ? 0u : 1u) : 2u;
    keep[i] = ((xf || yf) && a != b) ? 1u : 0u;
    key[i] = (uint64_t(a) << 34) | (uint64_t(b) << 2) | strand;
}

__global__ __launch_bounds__(256) void k_strand_compact(const uint32_t *__restrict__ keep,
                                                        const int64_t *__restrict__ pos,
                                                        const uint64_t *__restrict__ key,
                                                        int64_t r, uint64_t *__restrict__ kout,
                                                        uint32_t *__restrict__ vout) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= r || !keep[i]) return;
    kout[pos[i]] = key[i];
    vout[pos[i]] = uint32_t(i);
}

__global__ __launch_bounds__(256) void k_strand_write(const uint64_t *__restrict__ key,
                                                      const uint32_t *__restrict__ src,
                                                      const int32_t *__restrict__ rows, int64_t u,
                                                      int32_t *__restrict__ out) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= u) return;
    const uint64_t k = key[j];
    out[4 * j] = int32_t(k >> 34);
    out[4 * j + 1] = int32_t((k >> 2) & 0xffffffffu);
    out[4 * j + 2] = int32_t(k & 3u);
    out[4 * j + 3] = rows[3 * size_t(src[j]) + 2];
}

static int key_bits(int64_t m) {
    int b = 0;
    while ((int64_t(1) << b) < m) ++b;
    return 34 + (b > 0 ? b : 1);
}

struct StrandWs {
    uint32_t *keep;
    int64_t *pos;
    uint64_t *key;
    uint64_t *lbflags;
    uint32_t *ctr;
    SortBufs sb;
};

static void carve_strands(Carver &c, int64_t r, int64_t m, const Tune &t, StrandWs *W) {
    W->keep = c.take<uint32_t>(r + 1);
    W->pos = c.take<int64_t>(r + 1);
    W->key = c.take<uint64_t>(r + 1);
    W->lbflags = c.take<uint64_t>(scan_flags_words(r + 1) + 16);
    W->ctr = c.take<uint32_t>(64);
    carve_sort(c, r, key_bits(m), t, &W->sb, true);
}

}  // namespace saasm

using namespace saasm;

extern "C" int sa_revcomp_text(const uint8_t *text, int64_t n, uint8_t *out, int64_t *m_h,
                               void *ws, int64_t ws_bytes, hipStream_t stream) {
    if (!text || !out || !m_h || !ws) return fail(SA_ERR_INVALID, "sa_revcomp_text: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_revcomp_text: n must be >= 1");
    if (2 * n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_revcomp_text: 2n >= 2^31-2");
    if (ws_bytes < 256) return fail(SA_ERR_NOMEM, "sa_revcomp_text: workspace too small");
    Carver c(ws, ws_bytes);
    unsigned long long *m_dev = c.take<unsigned long long>(1);
    SA_TRY(launch_fill_u64(reinterpret_cast<uint64_t *>(m_dev), 1, 0, stream));
    hipLaunchKernelGGL(k_revcomp, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, text, n,
                       out, m_dev);
    SA_HIP(hipGetLastError());
    unsigned long long m = 0;
    SA_HIP(hipMemcpyAsync(&m, m_dev, 8, hipMemcpyDeviceToHost, stream));
    SA_HIP(hipStreamSynchronize(stream));
    *m_h = int64_t(m);
    return SA_OK;
}

extern "C" int64_t sa_strand_rows_ws_bytes(int64_t r, int64_t m) {
    if (r < 0 || m < 1) return -1;
    Tune t;
    resolve_tuning(nullptr, &t);
    Carver c(nullptr, INT64_MAX);
    StrandWs W;
    carve_strands(c, r > 0 ? r : 1, m, t, &W);
    return c.off + 256;
}

extern "C" int sa_strand_rows(const int32_t *rows, int64_t r, int64_t m, int32_t *out, int64_t cap,
                              int64_t *n_out_h, void *ws, int64_t ws_bytes, hipStream_t stream) {
    if (!n_out_h || !ws || (r > 0 && !rows) || (cap > 0 && !out))
        return fail(SA_ERR_INVALID, "sa_strand_rows: NULL pointer");
    if (r < 0 || cap < 0 || m < 1 || 2 * m >= kMaxN) return fail(SA_ERR_INVALID, "sa_strand_rows: bad sizes");
    if (ws_bytes < sa_strand_rows_ws_bytes(r, m)) return fail(SA_ERR_NOMEM, "sa_strand_rows: workspace too small");
    *n_out_h = 0;
    if (r == 0) return SA_OK;
    Tune t;
    resolve_tuning(nullptr, &t);
    Carver c(ws, ws_bytes);
    StrandWs W;
    carve_strands(c, r, m, t, &W);
    hipStream_t s = stream;
    SA_TRY(launch_fill_u32(W.ctr, 64, 0, s));
    const unsigned g = unsigned((r + 255) / 256);
    hipLaunchKernelGGL(k_strand_keys, dim3(g), dim3(256), 0, s, rows, r, uint32_t(m), W.keep,
                       W.key, W.ctr);
    SA_HIP(hipGetLastError());
    int64_t *utot = reinterpret_cast<int64_t *>(W.ctr + 8);
    SA_TRY(launch_scan_u32_i64(W.keep, W.pos, r, utot, W.lbflags, W.ctr + 4, W.ctr, s));
    int64_t u = 0;
    uint32_t e = 0;
    SA_HIP(hipMemcpyAsync(&u, utot, 8, hipMemcpyDeviceToHost, s));
    SA_HIP(hipMemcpyAsync(&e, W.ctr, 4, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    if (e) return fail(SA_ERR_INVALID, "sa_strand_rows: read id out of range for m reads");
    *n_out_h = u;
    if (u > cap) return fail(SA_ERR_CAPACITY, "sa_strand_rows: output holds " + std::to_string(cap) + " rows, need " + std::to_string(u));
    if (u == 0) return SA_OK;
    W.sb.err = W.ctr;
    hipLaunchKernelGGL(k_strand_compact, dim3(g), dim3(256), 0, s, W.keep, W.pos, W.key, r,
                       W.sb.keys[0], W.sb.vals[0]);
    SA_HIP(hipGetLastError());
    const int bits = key_bits(m);
    SA_TRY(sort_prepare(W.sb, u, bits, t, s));
    int nparts = 0, cur = 0;
    SA_TRY(launch_hist(W.sb, 0, u, 0, bits, t, s, &nparts));
    SA_TRY(sort_run(W.sb, 0, nullptr, u, 0, bits, t, nparts, s, &cur));
    hipLaunchKernelGGL(k_strand_write, dim3(unsigned((u + 255) / 256)), dim3(256), 0, s,
                       W.sb.keys[cur], W.sb.vals[cur], rows, u, out);
    SA_HIP(hipGetLastError());
    SA_HIP(hipMemcpyAsync(&e, W.ctr, 4, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    if (e) return fail(SA_ERR_HIP, "sa_strand_rows: device consistency check failed");
    return SA_OK;
}
