// dc3.hip -- suffix array by the skew recursion over the difference cover {1, 2} modulo 3.
//
// Sec. IV names its radix-sort kernel after DC3 and cites the linear-work construction of
// Kärkkäinen, Sanders and Burkhardt.  This file builds the same array as the doubling build
// (the suffix array of the text is unique) by that recursion, every sort being the LSD radix
// passes of radix.hip:
//   1. the sample suffixes (positions i with i mod 3 != 0) are sorted by their first three
//      symbols and each gets the rank of its triple as its name;
//   2. if two samples share a name, the string of names (all samples i = 1 mod 3 in position
//      order, then all i = 2 mod 3) is sorted by the same recursion; its suffix order is the
//      order of the sample suffixes;
//   3. the other suffixes (i = 0 mod 3) are sorted by (symbol at i, rank of suffix i+1), both
//      known once the samples are ranked;
//   4. the two sorted lists are merged.  Suffix i = 0 mod 3 and sample j compare by (symbol,
//      rank one further) when j = 1 mod 3, and by (two symbols, rank two further) when
//      j = 2 mod 3: in both cases the ranked suffixes are samples.
//
// Symbols.  At the top level the symbols are the text's: 0 for a separator and 1..4 for
// A, C, G, T.  The separators are distinct symbols ordered by position (read r's below read
// r+1's, all below A), so two symbols 0 compare by position, every suffix is distinct and
// the last symbol (the text ends with a separator) is unique.  A triple that holds a
// separator is the only one of its kind: its symbols after the separator are set to 0 and it
// gets a name of its own, in position order.  Deeper levels work on integer names 1..K with
// 0 past the end.  Their last symbol names a triple that holds the previous level's last,
// unique symbol, so it is unique as well; every comparison of two suffixes of a name string
// therefore ends at or before that symbol, and the recursion needs no extra dummy sample when
// the length is 1 mod 3.
//
// Each level keeps its ranks in an array over positions padded with three zeros (rank 0 is
// below every suffix: it stands for the empty suffix past the end, which no decided
// comparison reaches).  Names are ranks of triples counted from 1.  The host drives the
// levels: it reads each level's name count to decide whether to descend.
#include <algorithm>
#include <string>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace saasm {

namespace {

constexpr int kD3Block = 256;
constexpr int kMgItems = 8;                      // outputs per merge thread
constexpr int kMgTile = kD3Block * kMgItems;     // outputs per merge workgroup

unsigned grid_for(int64_t n, int per_block = kD3Block) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return unsigned(g);
}

// Symbol of a text byte: separator 0, A 1, C 2, G 3, T 4 (bytes are validated by the pack step).
__device__ __forceinline__ uint32_t text_sym(uint8_t b) {
    return b == 'A' ? 1u : b == 'C' ? 2u : b == 'G' ? 3u : b == 'T' ? 4u : 0u;
}

// Symbol at position p of a level's string: the text at the top (0 at and past the end), the
// padded name string below.
template <bool TOP>
__device__ __forceinline__ uint32_t sym(const uint8_t *__restrict__ text,
                                        const uint32_t *__restrict__ s, uint32_t n, uint32_t p) {
    if constexpr (TOP) return p < n ? text_sym(text[p]) : 0u;
    else return s[p];
}

// j-th sample position (samples in position order: 1, 2, 4, 5, 7, 8, ...)
__device__ __forceinline__ uint32_t sample_pos(uint32_t j) { return 3u * (j >> 1) + 1u + (j & 1u); }

// Position of a sample in the name string: mod-1 samples first, then mod-2 samples.
__device__ __forceinline__ uint32_t name_index(uint32_t pos, uint32_t n1) {
    return pos % 3u == 1u ? pos / 3u : n1 + pos / 3u;
}

// ---- step 1: sample keys --------------------------------------------------------------------
// Top level: three 3-bit symbols, those after a separator set to 0; a key whose last symbol
// is 0 holds a separator.
__global__ __launch_bounds__(kD3Block) void k_d3_keys_top(const uint8_t *__restrict__ text,
                                                          uint32_t n, uint32_t n12,
                                                          uint64_t *__restrict__ keys,
                                                          uint32_t *__restrict__ vals) {
    for (uint32_t j = blockIdx.x * kD3Block + threadIdx.x; j < n12; j += gridDim.x * kD3Block) {
        const uint32_t p = sample_pos(j);
        uint32_t c0 = text_sym(text[p]);
        uint32_t c1 = (c0 && p + 1 < n) ? text_sym(text[p + 1]) : 0u;
        uint32_t c2 = (c1 && p + 2 < n) ? text_sym(text[p + 2]) : 0u;
        keys[j] = (c0 << 6) | (c1 << 3) | c2;
        vals[j] = p;
    }
}

// Deeper levels: the triple of names in 3b bits (mode 0), or only its last name (mode 1, the
// first of two sorts when 3b > 64).
__global__ __launch_bounds__(kD3Block) void k_d3_keys(const uint32_t *__restrict__ s,
                                                      uint32_t n12, int b, int mode,
                                                      uint64_t *__restrict__ keys,
                                                      uint32_t *__restrict__ vals) {
    for (uint32_t j = blockIdx.x * kD3Block + threadIdx.x; j < n12; j += gridDim.x * kD3Block) {
        const uint32_t p = sample_pos(j);
        uint64_t k;
        if (mode == 0)
            k = (uint64_t(s[p]) << (2 * b)) | (uint64_t(s[p + 1]) << b) | uint64_t(s[p + 2]);
        else
            k = s[p + 2];
        keys[j] = k;
        vals[j] = p;
    }
}

// Second key of a two-sort triple: the first two names of the sample in the current order.
__global__ __launch_bounds__(kD3Block) void k_d3_rekey(const uint32_t *__restrict__ s,
                                                       uint32_t n12, int b,
                                                       uint64_t *__restrict__ keys,
                                                       const uint32_t *__restrict__ vals) {
    for (uint32_t j = blockIdx.x * kD3Block + threadIdx.x; j < n12; j += gridDim.x * kD3Block) {
        const uint32_t p = vals[j];
        keys[j] = (uint64_t(s[p]) << b) | uint64_t(s[p + 1]);
    }
}

// ---- step 1: names ------------------------------------------------------------------------
constexpr int kNsItems = 16;                      // sorted samples per thread of the name scan
constexpr int kNsTile = kD3Block * kNsItems;

// Names in sorted order: nm[j] = number of distinct triples among sorted samples 0..j.  A
// sample starts a new name when its key differs from its predecessor's (at the top level also
// when its triple holds a separator; with two sorts also when the last names differ).  One
// pass: head flags, a workgroup scan and a decoupled look-back over tiles; the last tile
// writes the name count to *total.  A tile is kNsItems rows of kD3Block consecutive samples,
// each row read and written by the whole workgroup (coalesced); a row's heads are counted
// with one ballot per wave.
template <bool TOP>
__global__ __launch_bounds__(kD3Block) void k_d3_name_scan(const uint64_t *__restrict__ keys,
                                                           const uint32_t *__restrict__ vals,
                                                           const uint32_t *__restrict__ s,
                                                           uint32_t n12, int two_sort,
                                                           uint32_t *__restrict__ nm,
                                                           uint32_t *total, uint64_t *lbflags,
                                                           uint32_t *tick, uint32_t *err) {
    constexpr int W = kD3Block / kWave;
    __shared__ uint32_t s_tile, s_excl;
    __shared__ uint32_t s_cnt[kNsItems][W];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    if (tid == 0) s_tile = ticket(tick);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t base = tile * uint32_t(kNsTile) + tid;
    uint32_t heads = 0;
    uint32_t below[kNsItems];  // heads of lower lanes of this wave in the same row
#pragma unroll
    for (int r = 0; r < kNsItems; ++r) {
        const uint32_t i = base + uint32_t(r) * kD3Block;
        bool head = false;
        if (i < n12) {
            const uint64_t k = keys[i];
            head = i == 0 || k != keys[i - 1];
            if constexpr (TOP) head = head || (k & 7u) == 0;  // holds a separator
            else if (two_sort && !head) head = s[vals[i] + 2] != s[vals[i - 1] + 2];
        }
        const uint64_t m = ballot(head);
        below[r] = uint32_t(popc64(m & lanemask_lt()));
        if (lane == 0) s_cnt[r][wave] = uint32_t(popc64(m));
        heads |= uint32_t(head) << r;
    }
    __syncthreads();
    // tile total and this thread's offset: all of rows before r, then the waves before in row r
    uint32_t tile_total = 0;
#pragma unroll
    for (int r = 0; r < kNsItems; ++r)
#pragma unroll
        for (int w = 0; w < W; ++w) tile_total += s_cnt[r][w];
    if (wave == 0) {
        const uint64_t ex = lookback_tile<SumOp>(lbflags, int(tile), tile_total, err);
        if (lane == 0) s_excl = uint32_t(ex);
    }
    __syncthreads();
    uint32_t row_base = s_excl;
#pragma unroll
    for (int r = 0; r < kNsItems; ++r) {
        uint32_t before = 0, row = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t c = s_cnt[r][w];
            if (uint32_t(w) < wave) before += c;
            row += c;
        }
        const uint32_t i = base + uint32_t(r) * kD3Block;
        if (i < n12) nm[i] = row_base + before + below[r] + ((heads >> r) & 1u);
        row_base += row;
    }
    if (tid == 0 && (tile + 1) * uint64_t(kNsTile) >= n12) *total = s_excl + tile_total;
}

// Names of the sorted samples to where the next step reads them: into the name string when
// names repeat (the recursion ranks the samples), else the ranks themselves (name = j + 1)
// and the sample order.
__global__ __launch_bounds__(kD3Block) void k_d3_scatter(const uint32_t *__restrict__ vals,
                                                         const uint32_t *__restrict__ nm,
                                                         uint32_t n12, uint32_t n1, int unique,
                                                         uint32_t *__restrict__ R,
                                                         uint32_t *__restrict__ sa12,
                                                         uint32_t *__restrict__ rank) {
    for (uint32_t j = blockIdx.x * kD3Block + threadIdx.x; j < n12; j += gridDim.x * kD3Block) {
        const uint32_t p = vals[j];
        if (unique) {
            rank[p] = j + 1u;
            sa12[j] = p;
        } else {
            R[name_index(p, n1)] = nm[j];
        }
    }
}

// ---- step 2: sample order from the suffix array of the name string ------------------------
__global__ __launch_bounds__(kD3Block) void k_d3_lift(const uint32_t *__restrict__ saR,
                                                      uint32_t n12, uint32_t n1,
                                                      uint32_t *__restrict__ sa12,
                                                      uint32_t *__restrict__ rank) {
    for (uint32_t k = blockIdx.x * kD3Block + threadIdx.x; k < n12; k += gridDim.x * kD3Block) {
        const uint32_t r = saR[k];
        const uint32_t p = r < n1 ? 3u * r + 1u : 3u * (r - n1) + 2u;
        sa12[k] = p;
        rank[p] = k + 1u;
    }
}

// ---- step 3: keys of the suffixes at positions 0 mod 3 --------------------------------------
// (symbol, rank of the next suffix); a separator at the top level orders by its position.
template <bool TOP>
__global__ __launch_bounds__(kD3Block) void k_d3_keys0(const uint8_t *__restrict__ text,
                                                       const uint32_t *__restrict__ s,
                                                       const uint32_t *__restrict__ rank,
                                                       uint32_t n, uint32_t n0, int rb,
                                                       uint64_t *__restrict__ keys,
                                                       uint32_t *__restrict__ vals) {
    for (uint32_t k = blockIdx.x * kD3Block + threadIdx.x; k < n0; k += gridDim.x * kD3Block) {
        const uint32_t i = 3u * k;
        const uint32_t c = sym<TOP>(text, s, n, i);
        keys[k] = (uint64_t(c) << rb) | uint64_t(c == 0 ? i : rank[i + 1]);
        vals[k] = i;
    }
}

// ---- step 4: merge --------------------------------------------------------------------------
struct Rec {
    uint32_t c0, c1, r1, r2;
};

// Comparison record of every position of a level, in position order: its symbol, the next
// symbol and the ranks one and two further.  A merge element then costs one random 16-byte
// read instead of one for the symbols and one for the ranks.
template <bool TOP>
__global__ __launch_bounds__(kD3Block) void k_d3_recs(const uint8_t *__restrict__ text,
                                                      const uint32_t *__restrict__ s,
                                                      const uint32_t *__restrict__ rank,
                                                      uint32_t n, uint4 *__restrict__ rec) {
    for (uint32_t x = blockIdx.x * kD3Block + threadIdx.x; x < n; x += gridDim.x * kD3Block)
        rec[x] = make_uint4(sym<TOP>(text, s, n, x), sym<TOP>(text, s, n, x + 1), rank[x + 1],
                            rank[x + 2]);
}

__device__ __forceinline__ Rec load_rec(const uint4 *__restrict__ rec, uint32_t x) {
    const uint4 v = rec[x];
    return Rec{v.x, v.y, v.z, v.w};
}

// Suffix a (a = 0 mod 3) before sample b?  Equal symbols 0 are separators (top level only:
// below it 0 appears only past the end) and compare by position.
__device__ __forceinline__ bool d3_less(const Rec &a, uint32_t ap, const Rec &b, uint32_t bp) {
    if (a.c0 != b.c0) return a.c0 < b.c0;
    if (a.c0 == 0) return ap < bp;
    if (bp % 3u == 1u) return a.r1 < b.r1;
    if (a.c1 != b.c1) return a.c1 < b.c1;
    if (a.c1 == 0) return ap < bp;
    return a.r2 < b.r2;
}

// Merge-path split of every tile boundary: split[t] = how many of the first t * kMgTile
// outputs come from A (the 0 mod 3 list).
__global__ __launch_bounds__(kD3Block) void k_d3_split(const uint4 *__restrict__ rec, uint32_t n,
                                                       const uint32_t *__restrict__ A, uint32_t na,
                                                       const uint32_t *__restrict__ B, uint32_t nb,
                                                       uint32_t ntiles,
                                                       uint32_t *__restrict__ split) {
    for (uint32_t t = blockIdx.x * kD3Block + threadIdx.x; t <= ntiles; t += gridDim.x * kD3Block) {
        const uint64_t dd = uint64_t(t) * kMgTile;
        const uint32_t d = dd < n ? uint32_t(dd) : n;
        uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            const uint32_t ap = A[mid], bp = B[d - 1 - mid];
            if (d3_less(load_rec(rec, ap), ap, load_rec(rec, bp), bp)) lo = mid + 1;
            else hi = mid;
        }
        split[t] = lo;
    }
}

// One tile of kMgTile outputs: the tile's runs of A and B with their comparison records go to
// LDS, each thread finds its own split by merge path and merges kMgItems outputs, and the
// tile is written out contiguously.
__global__ __launch_bounds__(kD3Block) void k_d3_merge(const uint4 *__restrict__ rec, uint32_t n,
                                                       const uint32_t *__restrict__ A,
                                                       uint32_t na_all,
                                                       const uint32_t *__restrict__ B,
                                                       uint32_t nb_all,
                                                       const uint32_t *__restrict__ split,
                                                       uint32_t *__restrict__ out,
                                                       uint32_t *err) {
    __shared__ uint32_t s_pos[kMgTile];
    __shared__ Rec s_rec[kMgTile];
    __shared__ uint32_t s_out[kMgTile];
    const uint32_t t = blockIdx.x, tid = threadIdx.x;
    const uint32_t d0 = t * uint32_t(kMgTile);
    const uint32_t d1 = (n - d0) < uint32_t(kMgTile) ? n : d0 + kMgTile;
    const uint32_t a0 = split[t], a1 = split[t + 1];
    const uint32_t cnt = d1 - d0;
    // The splits of a consistent order are monotone and within both lists; anything else
    // would index outside them, so the tile stops with an error instead.
    if (a1 < a0 || a1 - a0 > cnt || a1 > na_all || a0 > d0 || (d1 - a1) > nb_all) {
        if (tid == 0) raise_err(err, kErrRange);
        return;
    }
    const uint32_t b0 = d0 - a0;
    const uint32_t na = a1 - a0, nb = cnt - na;
    for (uint32_t i = tid; i < cnt; i += kD3Block) {
        const uint32_t x = i < na ? A[a0 + i] : B[b0 + (i - na)];
        s_pos[i] = x;
        s_rec[i] = load_rec(rec, x);
    }
    __syncthreads();
    const uint32_t k = tid * kMgItems;
    if (k < cnt) {
        uint32_t lo = k > nb ? k - nb : 0u, hi = k < na ? k : na;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            const uint32_t bi = na + (k - 1 - mid);
            if (d3_less(s_rec[mid], s_pos[mid], s_rec[bi], s_pos[bi])) lo = mid + 1;
            else hi = mid;
        }
        uint32_t ai = lo, bi = k - lo;
        const uint32_t kend = (k + kMgItems) < cnt ? k + kMgItems : cnt;
        for (uint32_t o = k; o < kend; ++o) {
            bool takeA;
            if (bi >= nb) takeA = true;
            else if (ai >= na) takeA = false;
            else takeA = d3_less(s_rec[ai], s_pos[ai], s_rec[na + bi], s_pos[na + bi]);
            s_out[o] = takeA ? s_pos[ai++] : s_pos[na + bi++];
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < cnt; i += kD3Block) out[d0 + i] = s_out[i];
}

__global__ __launch_bounds__(kD3Block) void k_d3_inverse(const uint32_t *__restrict__ sa,
                                                         uint32_t n, int32_t *__restrict__ isa) {
    for (uint32_t k = blockIdx.x * kD3Block + threadIdx.x; k < n; k += gridDim.x * kD3Block)
        isa[sa[k]] = int32_t(k);
}

int bits_for(int64_t v) {  // bits needed to hold 0..v
    int b = 0;
    while ((int64_t(1) << b) <= v) ++b;
    return b < 1 ? 1 : b;
}

// One level of the recursion.
struct Level {
    int64_t n = 0, n0 = 0, n1 = 0, n12 = 0;
    uint32_t *s = nullptr;     // [n + 3] symbols (levels below the top)
    uint32_t *out = nullptr;   // [n] this level's suffix array
    uint32_t *rank = nullptr;  // [n + 3]
    uint32_t *sa12 = nullptr;  // [n12] sorted samples
    uint32_t *R = nullptr;     // [n12 + 3] name string = next level's s
    uint32_t K = 0;            // largest symbol of s (the top: 4)
    bool recursed = false;
};

struct Layout {
    std::vector<Level> lev;
    uint32_t *nm = nullptr;     // [n12 of the top] names in sorted order
    uint4 *rec = nullptr;       // [n of the top] comparison records
    uint64_t *lbflags = nullptr;
    uint32_t *tick = nullptr;
    uint32_t *state = nullptr;  // [0] error bits, [1] name count
    uint32_t *split = nullptr;
    uint32_t *packed = nullptr, *sepmask = nullptr, *wordcnt = nullptr;
    SortBufs sb{};
};

void carve_dc3(Carver &c, int64_t n, const Tune &t, uint32_t *top_out, Layout *L) {
    L->lev.clear();
    int64_t m = n;
    for (int depth = 0; m > 0; ++depth) {
        Level v;
        v.n = m;
        v.n0 = (m + 2) / 3;
        v.n1 = (m + 1) / 3;
        v.n12 = m - v.n0;
        if (depth > 0) {
            v.s = L->lev.back().R;
            v.out = c.take<uint32_t>(m);
        } else {
            v.out = top_out;
        }
        v.rank = c.take<uint32_t>(m + 3);
        if (v.n12 > 0) {
            v.sa12 = c.take<uint32_t>(v.n12);
            v.R = c.take<uint32_t>(v.n12 + 3);
        }
        L->lev.push_back(v);
        m = v.n12;
    }
    const int64_t n12 = L->lev[0].n12 > 0 ? L->lev[0].n12 : 1;
    const int64_t items = std::max<int64_t>(n12, L->lev[0].n0);
    L->nm = c.take<uint32_t>(n12);
    L->rec = c.take<uint4>(n);
    L->lbflags = c.take<uint64_t>(n12 / kNsTile + 16);
    L->tick = c.take<uint32_t>(64);
    L->state = c.take<uint32_t>(64);
    L->split = c.take<uint32_t>((n + kMgTile - 1) / kMgTile + 2);
    L->packed = c.take<uint32_t>(packed_words(n));
    L->sepmask = c.take<uint32_t>(sepmask_words(n));
    L->wordcnt = c.take<uint32_t>(sepmask_words(n));
    carve_sort(c, items, 64, t, &L->sb, true);
}

struct Dc3 {
    const uint8_t *text;
    Tune t;
    Layout L;
    hipStream_t st;

    // Sorts items [0, count) already in sb.keys[cur]/vals[cur] over `bits` bits.
    int sort(int64_t count, int bits, int cur, int *cur_out) {
        SA_TRY(sort_prepare(L.sb, count, bits, t, st));
        int nparts = 0;
        SA_TRY(launch_hist(L.sb, cur, count, 0, bits, t, st, &nparts));
        return sort_run(L.sb, cur, nullptr, count, 0, bits, t, nparts, st, cur_out);
    }

    int read_words(uint32_t host[2]) {
        SA_HIP(hipMemcpyAsync(host, L.state, 8, hipMemcpyDeviceToHost, st));
        SA_HIP(hipStreamSynchronize(st));
        timing_poll();
        return SA_OK;
    }

    // Step 1 at level d: sort and name the samples; sets K of level d+1 and whether to descend.
    int name_samples(int d, bool *descend) {
        Level &v = L.lev[d];
        const bool top = d == 0;
        const uint32_t n12 = uint32_t(v.n12);
        const unsigned g = grid_for(v.n12);
        int cur = 0, bits = 0;
        bool two = false;
        {
            TimedScope ts("dc3_keys", double(v.n12) * (top ? 15.0 : 24.0), st);
            if (top) {
                hipLaunchKernelGGL(k_d3_keys_top, dim3(g), dim3(kD3Block), 0, st, text,
                                   uint32_t(v.n), n12, L.sb.keys[0], L.sb.vals[0]);
                bits = 9;
            } else {
                const int b = bits_for(v.K);
                two = 3 * b > 64;
                hipLaunchKernelGGL(k_d3_keys, dim3(g), dim3(kD3Block), 0, st, v.s, n12, b,
                                   two ? 1 : 0, L.sb.keys[0], L.sb.vals[0]);
                bits = two ? b : 3 * b;
            }
            ts.finish();
            SA_HIP(hipGetLastError());
        }
        SA_TRY(sort(v.n12, bits, 0, &cur));
        if (two) {
            const int b = bits_for(v.K);
            TimedScope ts("dc3_keys", double(v.n12) * 20.0, st);
            hipLaunchKernelGGL(k_d3_rekey, dim3(g), dim3(kD3Block), 0, st, v.s, n12, b,
                               L.sb.keys[cur], L.sb.vals[cur]);
            ts.finish();
            SA_HIP(hipGetLastError());
            SA_TRY(sort(v.n12, 2 * b, cur, &cur));
        }
        const int64_t ntiles = (v.n12 + kNsTile - 1) / kNsTile;
        SA_TRY(launch_fill_u64(L.lbflags, ntiles, 0, st));
        SA_TRY(launch_fill_u32(L.tick, 1, 0, st));
        {
            // keys 8 (+ 8 for the first two names' comparison with two sorts) + names 4
            TimedScope ts("dc3_names", double(v.n12) * (two ? 20.0 : 12.0), st);
            if (top)
                hipLaunchKernelGGL(k_d3_name_scan<true>, dim3(unsigned(ntiles)), dim3(kD3Block), 0,
                                   st, L.sb.keys[cur], L.sb.vals[cur], v.s, n12, 0, L.nm,
                                   L.state + 1, L.lbflags, L.tick, L.state);
            else
                hipLaunchKernelGGL(k_d3_name_scan<false>, dim3(unsigned(ntiles)), dim3(kD3Block), 0,
                                   st, L.sb.keys[cur], L.sb.vals[cur], v.s, n12, two ? 1 : 0, L.nm,
                                   L.state + 1, L.lbflags, L.tick, L.state);
            ts.finish();
            SA_HIP(hipGetLastError());
        }
        uint32_t host[2];
        SA_TRY(read_words(host));
        if (host[0]) return fail(host[0] & kErrAlphabet ? SA_ERR_ALPHABET : SA_ERR_HIP,
                                 "sa_build_dc3: device check failed (code " + std::to_string(host[0]) + ")");
        if (host[1] < 1 || host[1] > n12) return fail(SA_ERR_HIP, "sa_build_dc3: bad name count");
        *descend = host[1] < n12;
        if (*descend) {
            L.lev[d + 1].K = host[1];
            SA_TRY(launch_fill_u32(v.R + v.n12, 3, 0, st));
        }
        {
            // positions 4 + names 4 (descending) or sample order 4; one scattered word
            TimedScope ts("dc3_names", double(v.n12) * 12.0, st);
            hipLaunchKernelGGL(k_d3_scatter, dim3(g), dim3(kD3Block), 0, st, L.sb.vals[cur], L.nm,
                               n12, uint32_t(v.n1), *descend ? 0 : 1, v.R, v.sa12, v.rank);
            ts.finish();
            SA_HIP(hipGetLastError());
        }
        return SA_OK;
    }

    // Steps 3 and 4 at level d (its samples ranked).
    int finish(int d) {
        Level &v = L.lev[d];
        const bool top = d == 0;
        if (v.recursed) {
            TimedScope ts("dc3_lift", double(v.n12) * 16.0, st);
            hipLaunchKernelGGL(k_d3_lift, dim3(grid_for(v.n12)), dim3(kD3Block), 0, st,
                               L.lev[d + 1].out, uint32_t(v.n12), uint32_t(v.n1), v.sa12, v.rank);
            ts.finish();
            SA_HIP(hipGetLastError());
        }
        const int cb = top ? 3 : bits_for(v.K);
        const int rb = bits_for(std::max<int64_t>(v.n - 1, v.n12));
        {
            TimedScope ts("dc3_keys", double(v.n0) * (top ? 17.0 : 20.0), st);
            if (top)
                hipLaunchKernelGGL(k_d3_keys0<true>, dim3(grid_for(v.n0)), dim3(kD3Block), 0, st,
                                   text, v.s, v.rank, uint32_t(v.n), uint32_t(v.n0), rb,
                                   L.sb.keys[0], L.sb.vals[0]);
            else
                hipLaunchKernelGGL(k_d3_keys0<false>, dim3(grid_for(v.n0)), dim3(kD3Block), 0, st,
                                   text, v.s, v.rank, uint32_t(v.n), uint32_t(v.n0), rb,
                                   L.sb.keys[0], L.sb.vals[0]);
            ts.finish();
            SA_HIP(hipGetLastError());
        }
        int cur = 0;
        SA_TRY(sort(v.n0, cb + rb, 0, &cur));
        const uint32_t *A = L.sb.vals[cur];
        const uint32_t ntiles = uint32_t((v.n + kMgTile - 1) / kMgTile);
        {
            // symbols (top: 1 byte each, below: 4) + ranks 8 read; a 16-byte record written
            TimedScope ts("dc3_recs", double(v.n) * (top ? 26.0 : 32.0), st);
            if (top)
                hipLaunchKernelGGL(k_d3_recs<true>, dim3(grid_for(v.n)), dim3(kD3Block), 0, st,
                                   text, v.s, v.rank, uint32_t(v.n), L.rec);
            else
                hipLaunchKernelGGL(k_d3_recs<false>, dim3(grid_for(v.n)), dim3(kD3Block), 0, st,
                                   text, v.s, v.rank, uint32_t(v.n), L.rec);
            ts.finish();
            SA_HIP(hipGetLastError());
        }
        {
            TimedScope ts("dc3_merge", double(ntiles + 1) * 4.0, st);
            hipLaunchKernelGGL(k_d3_split, dim3(grid_for(ntiles + 1)), dim3(kD3Block), 0, st, L.rec,
                               uint32_t(v.n), A, uint32_t(v.n0), v.sa12, uint32_t(v.n12), ntiles,
                               L.split);
            ts.finish();
            SA_HIP(hipGetLastError());
        }
        {
            // list entry 4 + its 16-byte record + output 4
            TimedScope ts("dc3_merge", double(v.n) * 24.0, st);
            hipLaunchKernelGGL(k_d3_merge, dim3(ntiles), dim3(kD3Block), 0, st, L.rec, uint32_t(v.n),
                               A, uint32_t(v.n0), v.sa12, uint32_t(v.n12), L.split, v.out, L.state);
            ts.finish();
            SA_HIP(hipGetLastError());
        }
        return SA_OK;
    }

    int run(int64_t n, int32_t *levels_out) {
        SA_TRY(launch_fill_u32(L.state, 64, 0, st));
        SA_TRY(launch_pack(text, n, L.packed, L.sepmask, L.wordcnt, L.state, st));
        int depth = 0;
        for (;; ++depth) {
            Level &v = L.lev[depth];
            SA_TRY(launch_fill_u32(v.rank + v.n, 3, 0, st));
            if (v.n12 == 0) break;
            bool descend = false;
            SA_TRY(name_samples(depth, &descend));
            if (!descend) break;
            if (depth + 1 >= int(L.lev.size()))
                return fail(SA_ERR_HIP, "sa_build_dc3: recursion deeper than its levels");
            v.recursed = true;
        }
        for (int d = depth; d >= 0; --d) SA_TRY(finish(d));
        uint32_t host[2];
        SA_TRY(read_words(host));
        if (host[0] & kErrAlphabet)
            return fail(SA_ERR_ALPHABET, "text holds a byte other than A, C, G, T, $");
        if (host[0] & kErrNoSepEnd) return fail(SA_ERR_INVALID, "the text must end with '$'");
        if (host[0]) return fail(SA_ERR_HIP, "sa_build_dc3: device check failed (code " + std::to_string(host[0]) + ")");
        timing_flush();
        if (levels_out) *levels_out = depth + 1;
        return SA_OK;
    }
};

}  // namespace

}  // namespace saasm

using namespace saasm;

extern "C" int64_t sa_build_dc3_ws_bytes(int64_t n, const sa_tuning *tune) {
    Tune t;
    if (n < 1 || n >= kMaxN || resolve_tuning(tune, &t) != SA_OK) return -1;
    Carver c(nullptr, INT64_MAX);
    Layout L;
    carve_dc3(c, n, t, nullptr, &L);
    return c.off + 256;
}

static int sa_build_dc3_impl(const uint8_t *text, int64_t n, int32_t *sa, int32_t *isa_or_null,
                            void *ws, int64_t ws_bytes, const sa_tuning *tune, int32_t *levels_h,
                            hipStream_t stream) {
    if (!text || !sa || !ws) return fail(SA_ERR_INVALID, "sa_build_dc3: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_build_dc3: n must be >= 1");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_build_dc3: n >= 2^31-2");
    Dc3 D;
    SA_TRY(resolve_tuning(tune, &D.t));
    const int64_t need = sa_build_dc3_ws_bytes(n, tune);
    if (ws_bytes < need)
        return fail(SA_ERR_NOMEM, "sa_build_dc3: workspace too small (need " + std::to_string(need) + " bytes)");
    D.text = text;
    D.st = stream;
    Carver c(ws, ws_bytes);
    carve_dc3(c, n, D.t, reinterpret_cast<uint32_t *>(sa), &D.L);
    D.L.sb.err = D.L.state;
    SA_TRY(D.run(n, levels_h));
    if (isa_or_null) {
        hipLaunchKernelGGL(k_d3_inverse, dim3(grid_for(n)), dim3(kD3Block), 0, stream,
                           reinterpret_cast<const uint32_t *>(sa), uint32_t(n), isa_or_null);
        SA_HIP(hipGetLastError());
    }
    return SA_OK;
}

// ---- C entry points: bodies above, host exceptions turned into statuses ------------------
extern "C" int sa_build_dc3(const uint8_t *text, int64_t n, int32_t *sa, int32_t *isa_or_null,
                            void *ws, int64_t ws_bytes, const sa_tuning *tune, int32_t *levels_h,
                            hipStream_t stream) {
    return guard<int>([&] { return sa_build_dc3_impl(text, n, sa, isa_or_null, ws, ws_bytes, tune, levels_h, stream); });
}
