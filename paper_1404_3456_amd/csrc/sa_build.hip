// sa_build.hip -- suffix array by prefix doubling over LSD radix sorts (Sec. IV: the suffix
// array is the sorted array of all suffixes, built with a radix sort).
//
// Round 0 sorts every suffix by its first kH0 symbols (radix.hip, key0_of).  Each later round
// with prefix length h re-sorts only the suffixes whose group (set of suffixes equal on the
// first h symbols) is not yet a singleton, by the rank pair (group of p, group of p+h), which
// orders them by their first 2h symbols.  A round ends with the rank update below; the build
// stops when no group has two members.  The early stop plays the role of the paper's "check
// whether the output is sorted, and if not, continue with the next digit" (Sec. IV); because
// the suffix array is unique it never changes the result.
//
// Group labels are suffix-array indices: the label of a group is the index of its first
// member, so labels of groups that are already final never change and a round only touches
// active suffixes.  When the build ends every group is a singleton and the label array is the
// inverse suffix array.
#include "device.hpp"
#include "internal.hpp"

namespace saasm {

constexpr int kRuBlock = 256;
constexpr int kRuItems = 8;
constexpr int kRuTile = kRuBlock * kRuItems;

// Rank update over the sorted active items (K, V) of a round, whose suffix-array slots are
// S[0..A) (S == nullptr: identity, round 0).  For item i:
//   head(i)   = i == 0, or K[i] != K[i-1], or (round 0 and K[i] encodes fewer than kH0 symbols:
//               the suffix ended at its separator, which no other suffix shares);
//   single(i) = head(i) and head(i+1) (i+1 == A counts as a head);
//   label(i)  = S[g] where g is the last head at or before i.
// Writes sa[S[i]] = V[i], rank[V[i]] = label | (single ? kDone : 0), and the slots of items
// that are not singletons, compacted in order, to S_new; their count to *count_out.
__global__ __launch_bounds__(kRuBlock) void k_rank_update(
    const uint64_t *__restrict__ K, const uint32_t *__restrict__ V, const uint32_t *__restrict__ S,
    uint32_t A, uint32_t n, int round0, int32_t *__restrict__ sa, uint32_t *__restrict__ rank,
    uint32_t *__restrict__ S_new, uint64_t *lbflags, uint32_t *tick, uint32_t *count_out,
    uint32_t *err) {
    __shared__ uint64_t s_k[kRuTile + 2];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_w[kRuBlock / kWave];
    __shared__ uint64_t s_excl;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    if (tid == 0) s_tile = ticket(tick);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t tbase = tile * kRuTile;
    // keys of the tile plus one neighbour on each side (s_k[1 + i] = K[tbase + i])
    for (uint32_t i = tid; i < uint32_t(kRuTile); i += kRuBlock)
        s_k[1 + i] = (tbase + i < A) ? K[tbase + i] : 0;
    if (tid == 0) s_k[0] = tbase > 0 ? K[tbase - 1] : 0;
    if (tid == 1) s_k[kRuTile + 1] = (tbase + kRuTile < A) ? K[tbase + kRuTile] : 0;
    __syncthreads();

    const uint32_t first = tid * kRuItems;  // blocked: items first .. first+kRuItems-1
    bool head[kRuItems + 1];
#pragma unroll
    for (int j = 0; j <= kRuItems; ++j) {
        const uint32_t li = first + j;
        const uint32_t i = tbase + li;
        bool h = true;
        if (i < A && i > 0) {
            const uint64_t k = s_k[1 + li];
            h = (k != s_k[li]) || (round0 && (k & 31u) < uint64_t(kH0));
        }
        head[j] = h;  // i >= A: counts as a head for the single() test of i-1
    }
    uint32_t cnt = 0, last = 0;
#pragma unroll
    for (int j = 0; j < kRuItems; ++j) {
        const uint32_t i = tbase + first + j;
        if (i < A) {
            if (head[j]) last = i + 1;
            if (!(head[j] && head[j + 1])) ++cnt;
        }
    }
    // exclusive (count, last-head) scan over the workgroup, then over tiles
    const uint64_t mine = (uint64_t(cnt) << 31) | last;
    uint64_t inc = wave_incl_scan<CountLastOp>(mine);
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    uint64_t before = 0, tile_agg = 0;
#pragma unroll
    for (int w = 0; w < kRuBlock / kWave; ++w) {
        if (uint32_t(w) < wave) before = CountLastOp::combine(before, s_w[w]);
        tile_agg = CountLastOp::combine(tile_agg, s_w[w]);
    }
    uint64_t lane_excl = __shfl_up(inc, 1);
    if (lane == 0) lane_excl = 0;
    if (wave == 0) {
        uint64_t ex = lookback_tile<CountLastOp>(lbflags, int(tile), tile_agg, err);
        if (lane == 0) s_excl = ex;
        if (lane == 0 && tbase + kRuTile >= A)
            *count_out = uint32_t(CountLastOp::combine(ex, tile_agg) >> 31);
    }
    __syncthreads();
    const uint64_t state = CountLastOp::combine(CountLastOp::combine(s_excl, before), lane_excl);
    uint32_t out = uint32_t(state >> 31);
    uint32_t g1 = uint32_t(state & CountLastOp::kLastMask);  // last head index + 1 (0: none)
#pragma unroll
    for (int j = 0; j < kRuItems; ++j) {
        const uint32_t i = tbase + first + j;
        if (i < A) {
            if (head[j]) g1 = i + 1;
            const bool single = head[j] && head[j + 1];
            const uint32_t g = g1 - 1;  // i == 0 is always a head, so g1 >= 1
            const uint32_t slot = S ? S[i] : i;
            const uint32_t label = S ? S[g] : g;
            const uint32_t v = V[i];
            if (slot >= n || v >= n || label >= n) {  // inconsistent input: report, never write
                raise_err(err, kErrRange);
                continue;
            }
            sa[slot] = int32_t(v);
            rank[v] = label | (single ? kDone : 0u);
            if (!single) S_new[out++] = slot;
        }
    }
}

__global__ __launch_bounds__(256) void k_strip(uint32_t *__restrict__ rank, uint32_t n) {
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) rank[i] &= kRankMask;
}

static int bits_for(int64_t v) {  // bits needed to hold 0..v
    int b = 0;
    while ((int64_t(1) << b) <= v) ++b;
    return b < 1 ? 1 : b;
}

struct BuildLayout {
    uint32_t *packed, *sepmask, *wordcnt;
    uint32_t *rank;        // used when the caller gives no isa buffer
    uint32_t *slots[2];
    SortBufs sb;
    uint64_t *lbflags;
    uint32_t *tickets;
    uint32_t *ctr;         // [0] err, [1] count (rank update), [2] count (key build)
};

static void carve_build(Carver &c, int64_t n, const Tune &t, BuildLayout *L) {
    const int bits = 2 * kH0 + 5 > 2 * bits_for(n) ? 2 * kH0 + 5 : 2 * bits_for(n);
    L->packed = c.take<uint32_t>(packed_words(n));
    L->sepmask = c.take<uint32_t>(sepmask_words(n));
    L->wordcnt = c.take<uint32_t>(sepmask_words(n));
    L->rank = c.take<uint32_t>(n);
    L->slots[0] = c.take<uint32_t>(n);
    L->slots[1] = c.take<uint32_t>(n);
    carve_sort(c, n, bits, t, &L->sb, true);
    const int64_t lbw = (n + kRuTile - 1) / kRuTile + (n + 2047) / 2048 + 16;
    L->lbflags = c.take<uint64_t>(lbw);
    L->tickets = c.take<uint32_t>(64);
    L->ctr = c.take<uint32_t>(64);
}

static int launch_rank_update(const uint64_t *K, const uint32_t *V, const uint32_t *S, int64_t A,
                              int64_t n, bool round0, int32_t *sa, uint32_t *rank, uint32_t *S_new,
                              uint64_t *lbflags, uint32_t *tick, uint32_t *count_out,
                              uint32_t *err, hipStream_t s) {
    const int64_t tiles = (A + kRuTile - 1) / kRuTile;
    SA_TRY(launch_fill_u64(lbflags, tiles, 0, s));
    SA_TRY(launch_fill_u32(tick, 1, 0, s));
    // algorithmic bytes: read K (8) + V (4) + S (4 when present); write sa (4) + rank (4) +
    // S_new (4, upper bound)
    TimedScope ts("rank_update", double(A) * (S ? 28.0 : 24.0), s);
    hipLaunchKernelGGL(k_rank_update, dim3(unsigned(tiles)), dim3(kRuBlock), 0, s, K, V, S,
                       uint32_t(A), uint32_t(n), int(round0), sa, rank, S_new, lbflags, tick, count_out, err);
    ts.finish();
    SA_HIP(hipGetLastError());
    return SA_OK;
}

static int read_ctr(const uint32_t *ctr, uint32_t host[4], hipStream_t s) {
    SA_HIP(hipMemcpyAsync(host, ctr, 16, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    timing_flush();
    return SA_OK;
}

static int check_err(uint32_t e) {
    if (e & kErrAlphabet) return fail(SA_ERR_ALPHABET, "text holds a byte other than A, C, G, T, $");
    if (e & kErrNoSepEnd) return fail(SA_ERR_INVALID, "text must end with '$'");
    if (e) return fail(SA_ERR_HIP, "device consistency check failed (code " + std::to_string(e) + ")");
    return SA_OK;
}

}  // namespace saasm

using namespace saasm;

extern "C" int64_t sa_build_ws_bytes(int64_t n, const sa_tuning *tune) {
    Tune t;
    if (n < 1 || resolve_tuning(tune, &t) != SA_OK) return -1;
    Carver c(nullptr, INT64_MAX);
    BuildLayout L;
    carve_build(c, n, t, &L);
    return c.off + 256;
}

extern "C" int sa_build(const uint8_t *text, int64_t n, int32_t *sa, int32_t *isa_or_null,
                        void *ws, int64_t ws_bytes, const sa_tuning *tune, int32_t *rounds_h,
                        hipStream_t stream) {
    if (!text || !sa || !ws) return fail(SA_ERR_INVALID, "sa_build: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_build: n must be >= 1");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_build: n >= 2^30");
    Tune t;
    SA_TRY(resolve_tuning(tune, &t));
    const int64_t need = sa_build_ws_bytes(n, tune);
    if (ws_bytes < need)
        return fail(SA_ERR_NOMEM, "sa_build: workspace too small (need " + std::to_string(need) + " bytes)");
    Carver c(ws, ws_bytes);
    BuildLayout L;
    carve_build(c, n, t, &L);
    L.sb.err = L.ctr;
    uint32_t *rank = isa_or_null ? reinterpret_cast<uint32_t *>(isa_or_null) : L.rank;
    hipStream_t s = stream;

    SA_TRY(launch_fill_u32(L.ctr, 64, 0, s));
    SA_TRY(launch_pack(text, n, L.packed, L.sepmask, L.wordcnt, L.ctr, s));

    // round 0: first kH0 symbols
    const int bits0 = 2 * kH0 + 5;
    SA_TRY(sort_prepare(L.sb, n, bits0, t, s));
    SA_TRY(launch_key0(L.packed, L.sepmask, n, L.sb, 0, t, s));
    int cur = 0;
    SA_TRY(sort_run(L.sb, 0, n, 0, bits0, t, s, &cur));
    SA_TRY(launch_rank_update(L.sb.keys[cur], L.sb.vals[cur], nullptr, n, n, true, sa, rank,
                              L.slots[0], L.lbflags, L.tickets, L.ctr + 1, L.ctr, s));
    uint32_t host[4];
    SA_TRY(read_ctr(L.ctr, host, s));
    SA_TRY(check_err(host[0]));
    int64_t A = host[1];
    int rounds = 1;
    int sl = 0;
    const int rbits = bits_for(n - 1);
    int64_t h = kH0;
    while (A > 0) {
        if (h > 2 * n) return fail(SA_ERR_HIP, "sa_build: doubling did not converge");
        const int bits = 2 * rbits;
        SA_TRY(sort_prepare(L.sb, A, bits, t, s));
        SA_TRY(launch_keys_doubling(rank, n, h, rbits, L.sb, 0, L.lbflags, L.tickets, L.ctr + 2, t, s));
        SA_TRY(sort_run(L.sb, 0, A, 0, bits, t, s, &cur));
        SA_TRY(launch_rank_update(L.sb.keys[cur], L.sb.vals[cur], L.slots[sl], A, n, false, sa, rank,
                                  L.slots[sl ^ 1], L.lbflags, L.tickets, L.ctr + 1, L.ctr, s));
        SA_TRY(read_ctr(L.ctr, host, s));
        SA_TRY(check_err(host[0]));
        if (int64_t(host[2]) != A)
            return fail(SA_ERR_HIP, "sa_build: active-suffix count mismatch");
        A = host[1];
        sl ^= 1;
        h *= 2;
        ++rounds;
    }
    if (isa_or_null) {
        unsigned grid = unsigned((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
        hipLaunchKernelGGL(k_strip, dim3(grid), dim3(256), 0, s, rank, uint32_t(n));
        SA_HIP(hipGetLastError());
    }
    if (rounds_h) *rounds_h = rounds;
    return SA_OK;
}
