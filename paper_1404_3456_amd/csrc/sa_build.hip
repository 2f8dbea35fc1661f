// sa_build.hip -- suffix array by prefix doubling over LSD radix sorts (Sec. IV: the suffix
// array is the sorted array of all suffixes, built with a radix sort).
//
// Round 0 sorts every suffix by its first h0 symbols (radix.hip, key0_of).  Each later round
// with prefix length h re-sorts only the suffixes whose group (set of suffixes equal on the
// first h symbols) is not yet a singleton, by the rank pair (group of p, group of p+h), which
// orders them by their first 2h symbols.  A round ends with the rank update below; the build
// stops when no group has two members.  The early stop plays the role of the paper's check
// whether the output is already sorted before the next digit is processed (Sec. IV); because
// the suffix array is unique it never changes the result.
//
// Group labels are suffix-array indices: the label of a group is the index of its first
// member, so labels of groups that are already final never change and a round only touches
// active suffixes.  When the build ends every group is a singleton and the label array is the
// inverse suffix array.
//
// All round kernels read the active count and h from a small device-side state array, so a
// doubling round can be recorded once as a hipGraph and replayed; once the active count is 0
// every kernel of a replayed round returns at once.
//
// A batch of independent texts (sa_build_batched) is the same build over their
// concatenation, with each text's index placed above the first-round key: every text's
// suffixes then form one block of the order, labels of different texts never mix, and the
// block of text s is exactly the suffix array of text s (in concatenated coordinates).
#include <cstring>
#include <vector>

#include "device.hpp"
#include "internal.hpp"

namespace saasm {

constexpr int kRuBlock = 1024;
constexpr int kRuItems = 8;
constexpr int kRuTile = kRuBlock * kRuItems;
// Smallest tile of a kernel that takes the build's tile look-back words (the rank update; the
// large-group extraction's tiles are larger): the array holds one word per tile of this size,
// and every launcher checks its tile count against that on the host.
constexpr int kLbMinTile = kRuTile;

// Rank update over the sorted active items (K, V) of a round, whose suffix-array slots are
// S[0..A) (S == nullptr: identity, round 0).  For item i:
//   head(i)   = i == 0, or K[i] != K[i-1], or (round 0 and K[i] encodes fewer than h0 symbols:
//               the suffix ended at its separator, which no other suffix shares);
//   single(i) = head(i) and head(i+1) (i+1 == A counts as a head);
//   label(i)  = S[g] where g is the last head at or before i.
// Writes rank[V[i]] = label, sa[S[i]] = V[i] once item i is a singleton
// (its slot is then final; nothing reads the slots of suffixes still in a group), and the slots
// of items that are not singletons, compacted in order, to S_new; their count to
// state[kStNext].
// In a doubling round the key's upper half is the item's previous label, so rank[V[i]] is
// only rewritten when the label changes or the item becomes a singleton.
// Beside each compacted slot it writes the item's text position to P_new, with bit 31 set on
// the first member of each group, so the next round can find its groups as runs in this
// order; and it sets state[kStBigNext] when some group has more than kRunMax members.
// One tile per workgroup (tiles by ticket); the grid covers an upper bound on A and surplus
// workgroups return at once.
__global__ __launch_bounds__(kRuBlock) void k_rank_update(
    const uint64_t *__restrict__ K, const uint32_t *__restrict__ V, const uint32_t *__restrict__ S,
    uint32_t n, int round0, uint32_t h0, int rbits, int32_t *__restrict__ sa,
    uint32_t *__restrict__ rank, uint32_t *__restrict__ S_new, uint32_t *__restrict__ P_new,
    uint64_t *lbflags, uint32_t *tick, uint32_t *state, uint32_t *err) {
    // Global memory is only touched in wave-contiguous (striped) order; the per-item logic
    // works on blocked runs of kRuItems consecutive items held in LDS.
    __shared__ uint64_t s_k[kRuTile + 2];  // keys, one neighbour each side; then the outputs
    __shared__ uint32_t s_s[kRuTile];      // suffix-array slots
    __shared__ uint32_t s_v[kRuTile];      // text positions
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_w[kRuBlock / kWave];
    __shared__ uint64_t s_excl;
    constexpr uint32_t kNone = 0xffffffffu;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t A = state[kStActive];
    const uint32_t ntiles = (A + kRuTile - 1) / kRuTile;
    if (tid == 0) s_tile = ticket(tick);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) return;
    const uint32_t tbase = tile * kRuTile;
    {
        // Every load of the thread is issued before the first LDS store (indices past the
        // active count read the last item and are then dropped), so the tile costs one memory
        // latency rather than one per item and array.
        uint64_t kr[kRuItems];
        uint32_t sr[kRuItems], vr[kRuItems];
#pragma unroll
        for (int j = 0; j < kRuItems; ++j) {
            const uint32_t i = tbase + tid + uint32_t(j) * kRuBlock;
            const uint32_t c = i < A ? i : A - 1;  // A >= 1: this tile holds an item
            kr[j] = K[c];
            vr[j] = V[c];
        }
        if (S) {
#pragma unroll
            for (int j = 0; j < kRuItems; ++j) {
                const uint32_t i = tbase + tid + uint32_t(j) * kRuBlock;
                sr[j] = S[i < A ? i : A - 1];
            }
        } else {
#pragma unroll
            for (int j = 0; j < kRuItems; ++j) sr[j] = tbase + tid + uint32_t(j) * kRuBlock;
        }
        const uint64_t kprev = (tid == 0 && tbase > 0) ? K[tbase - 1] : 0;
        const uint64_t knext = (tid == 1 && tbase + kRuTile < A) ? K[tbase + kRuTile] : 0;
#pragma unroll
        for (int j = 0; j < kRuItems; ++j) {
            const uint32_t li = tid + uint32_t(j) * kRuBlock;
            const bool in = tbase + li < A;
            s_k[1 + li] = in ? kr[j] : 0;
            s_s[li] = in ? sr[j] : 0;
            s_v[li] = in ? vr[j] : 0;
        }
        if (tid == 0) s_k[0] = kprev;
        if (tid == 1) s_k[kRuTile + 1] = knext;
    }
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
            h = (k != s_k[li]) || (round0 && (k & 31u) < uint64_t(h0));
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
        if (lane == 0 && tile == ntiles - 1)
            state[kStNext] = uint32_t(CountLastOp::combine(ex, tile_agg) >> 31);
    }
    __syncthreads();
    const uint64_t state_in = CountLastOp::combine(CountLastOp::combine(s_excl, before), lane_excl);
    uint32_t out = uint32_t(state_in >> 31);
    uint32_t g1 = uint32_t(state_in & CountLastOp::kLastMask);  // last head index + 1
    const uint64_t lmask = (uint64_t(1) << rbits) - 1;
    uint32_t lab_w[kRuItems], out_w[kRuItems];  // rank word and next-round index, or kNone
#pragma unroll
    for (int j = 0; j < kRuItems; ++j) {
        const uint32_t li = first + j;
        const uint32_t i = tbase + li;
        lab_w[j] = kNone;
        out_w[j] = kNone;
        if (i < A) {
            if (head[j]) g1 = i + 1;
            const bool single = head[j] && head[j + 1];
            const uint32_t g = g1 - 1;  // i == 0 is always a head, so g1 >= 1
            const uint32_t label = g >= tbase ? s_s[g - tbase] : (S ? S[g] : g);
            if (s_s[li] >= n || s_v[li] >= n || label >= n) {  // inconsistent input: report only
                raise_err(err, kErrRange);
                continue;
            }
            const bool same = !round0 && uint32_t((s_k[1 + li] >> rbits) & lmask) == label;
            if (single || !same) lab_w[j] = label | (single ? kDone : 0u);
            if (!single) {
                out_w[j] = out++ | (head[j] ? kDone : 0u);  // bit 31: first of its group
                if (i - g == uint32_t(kRunMax)) state[kStBigNext] = 1u;
            }
        }
    }
    __syncthreads();  // every read of the keys is done: their storage now holds the outputs
    uint32_t *s_lab = reinterpret_cast<uint32_t *>(s_k);
    uint32_t *s_out = s_lab + kRuTile;
#pragma unroll
    for (int j = 0; j < kRuItems; ++j) {
        s_lab[first + j] = lab_w[j];
        s_out[first + j] = out_w[j];
    }
    __syncthreads();
    for (uint32_t i = tid; i < uint32_t(kRuTile); i += kRuBlock) {
        if (tbase + i >= A) break;
        const uint32_t slot = s_s[i], v = s_v[i];
        if (slot >= n || v >= n) continue;  // reported above
        const uint32_t lw = s_lab[i];
        if (lw != kNone) {
            rank[v] = lw & kRankMask;  // bit 31 only marks a singleton here
            if (lw & kDone) sa[slot] = int32_t(v);  // final; slots still in a group are rewritten later
        }
        const uint32_t o = s_out[i];
        if (o != kNone) {
            S_new[o & kRankMask] = slot;
            P_new[o & kRankMask] = v | (o & kDone);
        }
    }
}

// Advances the round state after a rank update (one thread).
__global__ void k_round_end(uint32_t *state, uint32_t h_first) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    state[kStBigLast] = state[kStRadixN];  // the round's large-group items (0 when none)
    state[kStRadixN] = 0;
    if (state[kStActive] == 0) return;  // the round had nothing to do
    const uint32_t rounds = state[kStRounds];
    state[kStH] = rounds == 0 ? h_first : state[kStH] * 2u;
    state[kStRounds] = rounds + 1;
    state[kStActive] = state[kStNext];
    // the next round sorts the items of groups too large for the run sort by radix passes
    state[kStBig] = state[kStBigNext];
    state[kStBigNext] = 0;
}

// Adds a block's offset to suffix-array and inverse entries built for that block alone.
__global__ __launch_bounds__(256) void k_add_offset(int32_t *__restrict__ sa, int32_t *__restrict__ isa,
                                                    int64_t n, int32_t base) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    sa[i] += base;
    if (isa) isa[i] += base;
}

// Every text of a batch must be non-empty and end with a separator.
__global__ void k_check_sets(const uint8_t *__restrict__ text, const int64_t *__restrict__ off,
                             uint32_t n_sets, uint32_t *err) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sets) return;
    if (off[s + 1] <= off[s] || text[off[s + 1] - 1] != '$') raise_err(err, kErrNoSepEnd);
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
    uint32_t *pos;         // active text positions in the last round's order (bit 31: run start)
    uint32_t *bigidx;      // list index of each large-group item of a round (radix-sorted ones)
    SortBufs sb;
    uint64_t *lbflags;
    int64_t lb_words;      // look-back words in lbflags
    uint32_t *tickets;
    uint32_t *state;       // kSt* words
    int64_t *set_off;      // batched builds: [n_sets + 1]
    void *lcp_ws;          // batched builds: workspace of the LCP computed after the build
    int64_t lcp_ws_bytes;
};

static void carve_build(Carver &c, int64_t n, int n_sets, const Tune &t, BuildLayout *L) {
    const int bits = 63 > 2 * bits_for(n) ? 63 : 2 * bits_for(n);
    L->packed = c.take<uint32_t>(packed_words(n));
    L->sepmask = c.take<uint32_t>(sepmask_words(n));
    L->wordcnt = c.take<uint32_t>(sepmask_words(n));
    L->rank = c.take<uint32_t>(n);
    L->slots[0] = c.take<uint32_t>(n);
    L->slots[1] = c.take<uint32_t>(n);
    L->pos = c.take<uint32_t>(n);
    L->bigidx = c.take<uint32_t>(n);
    carve_sort(c, n, bits, t, &L->sb, true);
    L->lb_words = (n + kLbMinTile - 1) / kLbMinTile + 16;
    L->lbflags = c.take<uint64_t>(L->lb_words);
    L->tickets = c.take<uint32_t>(64);
    L->state = c.take<uint32_t>(64);
    L->set_off = c.take<int64_t>(n_sets + 1);
    L->lcp_ws_bytes = n_sets > 0 ? lcp_ws_bytes(n) : 0;
    L->lcp_ws = n_sets > 0 ? c.take<char>(L->lcp_ws_bytes) : nullptr;
}

// Keys of a doubling round built in the previous round's sorted order and sorted group by
// group without radix passes.  The previous rank update left the active items in that order:
// slots S[0..A) and text positions P[0..A) with bit 31 on the first member of each group, so
// each group is a run whose label is the slot of its first member.  Item o of a run of at most
// kRunMax items gets
//   key = (label << rbits) | rank[p + h],
// and goes to the run's first index plus the number of run members with a smaller key (equal
// keys keep their order), which is where a stable sort of the whole array puts it.  Items of
// longer runs are left to the radix passes (k_big_extract, k_big_place) when state[kStBig] is
// set, and raise kErrRange otherwise.  Tiles of kKrTile items, loaded with kRunMax items of
// context on either side, so every run of at most kRunMax items that meets the tile lies inside
// the loaded range.  The active count and h come from state[kStActive] and state[kStH]; a count
// of 0 makes the launch a no-op.
constexpr int kKrBlock = 256;
constexpr int kKrTile = 2048;
constexpr int kKrSpan = kKrTile + 2 * kRunMax;

__global__ __launch_bounds__(kKrBlock) void k_keys_runs(
    const uint32_t *__restrict__ P, const uint32_t *__restrict__ S,
    const uint32_t *__restrict__ rank, uint32_t n, int rbits, const uint32_t *state,
    uint64_t *__restrict__ K, uint32_t *__restrict__ V, uint32_t *err) {
    __shared__ uint32_t s_p[kKrSpan];   // position | first-of-run bit; outside [0, A): the bit alone
    __shared__ uint32_t s_r2[kKrSpan];  // rank[p + h]
    __shared__ uint32_t s_lab[kKrSpan]; // slot (the label, on a run's first member)
    const uint32_t A = state[kStActive];
    const uint32_t h = state[kStH];
    const bool mixed = state[kStBig] != 0;  // longer runs exist and are sorted elsewhere
    const int64_t tbase = int64_t(blockIdx.x) * kKrTile;
    if (tbase >= int64_t(A)) return;
    const int64_t lo = tbase - kRunMax;
    for (int x = threadIdx.x; x < kKrSpan; x += kKrBlock) {
        const int64_t gi = lo + x;
        uint32_t pv = kDone, r2 = 0, lab = 0;
        if (gi >= 0 && gi < int64_t(A)) {
            pv = P[gi];
            lab = S[gi];
            const uint32_t p = pv & kRankMask;
            if (p < n && h < n - p) r2 = rank[p + h] & kRankMask;
            else raise_err(err, kErrRange);
        }
        s_p[x] = pv;
        s_r2[x] = r2;
        s_lab[x] = lab;
    }
    __syncthreads();
    const uint64_t rmask = (uint64_t(1) << rbits) - 1;
    for (int li = kRunMax + threadIdx.x; li < kRunMax + kKrTile; li += kKrBlock) {
        if (lo + li >= int64_t(A)) break;
        // run start: the nearest first-of-run bit at or before li (at most kRunMax - 1 back)
        int st = li;
        while (!(s_p[st] & kDone) && li - st < kRunMax - 1) --st;
        // run end: the next first-of-run bit after li (slots past A carry the bit)
        int en = li + 1;
        while (!(s_p[en] & kDone) && en - st < kRunMax) ++en;
        if (!(s_p[st] & kDone) || !(s_p[en] & kDone)) {
            if (!mixed) raise_err(err, kErrRange);  // a run longer than kRunMax
            continue;
        }
        const uint32_t r2 = s_r2[li];
        uint32_t before = 0;
        for (int y = st; y < en; ++y) {
            const uint32_t q = s_r2[y];
            before += (q < r2 || (q == r2 && y < li)) ? 1u : 0u;
        }
        const int64_t out = lo + st + before;
        if (out >= int64_t(A)) {
            raise_err(err, kErrRange);
            continue;
        }
        K[out] = ((uint64_t(s_lab[st]) & rmask) << rbits) | (uint64_t(r2) & rmask);
        V[out] = s_p[li] & kRankMask;
    }
}

static int launch_keys_runs(const uint32_t *P, const uint32_t *S, const uint32_t *rank,
                            int64_t a_bound, int64_t n, int rbits, const uint32_t *state,
                            uint64_t *K, uint32_t *V, uint32_t *err, hipStream_t s) {
    int64_t tiles = (a_bound + kKrTile - 1) / kKrTile;
    if (tiles < 1) tiles = 1;
    // algorithmic bytes per item: read P, S and rank[p + h] (4 each); write K (8) and V (4)
    TimedScope ts("keyruns", 0.0, 24.0, s);
    hipLaunchKernelGGL(k_keys_runs, dim3(unsigned(tiles)), dim3(kKrBlock), 0, s, P, S, rank,
                       uint32_t(n), rbits, state, K, V, err);
    ts.finish();
    SA_HIP(hipGetLastError());
    return SA_OK;
}

static int launch_rank_update(const uint64_t *K, const uint32_t *V, const uint32_t *S,
                              int64_t a_bound, int64_t n, bool round0, int h0, int rbits,
                              int32_t *sa, uint32_t *rank, uint32_t *S_new, uint32_t *P_new,
                              uint64_t *lbflags, int64_t lb_words, uint32_t *tick,
                              uint32_t *state, hipStream_t s) {
    int64_t tiles = (a_bound + kRuTile - 1) / kRuTile;
    if (tiles < 1) tiles = 1;
    if (tiles > lb_words) return fail(SA_ERR_HIP, "rank update: look-back array too small");
    SA_TRY(launch_fill_u64(lbflags, tiles, 0, s));
    SA_TRY(launch_fill_u32(tick, 1, 0, s));
    // algorithmic bytes: read K (8) + V (4) + S (4 when present); write sa (4) + rank (4) +
    // S_new (4) + P_new (4) (upper bounds)
    TimedScope ts = S ? TimedScope("rank_update", 0.0, 32.0, s)
                      : TimedScope("rank_update", double(a_bound) * 28.0, s, double(a_bound));
    hipLaunchKernelGGL(k_rank_update, dim3(unsigned(tiles)), dim3(kRuBlock), 0, s, K, V, S,
                       uint32_t(n), int(round0), uint32_t(h0), rbits, sa, rank, S_new, P_new,
                       lbflags, tick, state, state + kStErr);
    ts.finish();
    SA_HIP(hipGetLastError());
    return SA_OK;
}

static int check_err(uint32_t e) {
    if (e & kErrAlphabet) return fail(SA_ERR_ALPHABET, "text holds a byte other than A, C, G, T, $");
    if (e & kErrNoSepEnd) return fail(SA_ERR_INVALID, "every text must end with '$'");
    if (e) return fail(SA_ERR_HIP, "device consistency check failed (code " + std::to_string(e) + ")");
    return SA_OK;
}

// Pinned host words and events for reading round state without a full stream sync (one set
// per host thread; two slots so one round's state can be in flight while the other is read).
struct PinnedState {
    uint32_t *h = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ok = false;
    PinnedState() {
        ok = hipHostMalloc(reinterpret_cast<void **>(&h), 2 * kStWords * 4, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) == hipSuccess;
    }
};
static PinnedState &pinned_state() {
    static thread_local PinnedState ps;
    return ps;
}

// One suffix-array build (plain: one text; batched: n_sets texts, set_off_h on the host).
struct Build {
    const uint8_t *text;
    int64_t n;
    int n_sets;          // 0: plain text
    const int64_t *set_off_h;
    int32_t *sa;
    uint32_t *rank;
    Tune t;
    BuildLayout L;
    hipStream_t s;
    int h0 = kH0;
    int key0_bits = 2 * kH0 + 5;
    int rbits = 1;

    // copies the state words to pinned slot k and records its event (stream order)
    int snapshot(PinnedState &ps, int k) {
        SA_HIP(hipMemcpyAsync(ps.h + kStWords * k, L.state, kStWords * 4, hipMemcpyDeviceToHost, s));
        SA_HIP(hipEventRecord(ps.ev[k], s));
        return SA_OK;
    }

    int read_state(uint32_t host[kStWords]) {
        SA_HIP(hipMemcpyAsync(host, L.state, kStWords * 4, hipMemcpyDeviceToHost, s));
        SA_HIP(hipStreamSynchronize(s));
        timing_flush();
        return SA_OK;
    }

    int round0() {
        SA_TRY(launch_fill_u32(L.state, 64, 0, s));
        SA_TRY(launch_fill_u32(L.state + kStActive, 1, uint32_t(n), s));
        SA_TRY(launch_pack(text, n, L.packed, L.sepmask, L.wordcnt, L.state + kStErr, s));
        const int64_t *set_off_dev = nullptr;
        if (n_sets > 0) {
            SA_HIP(hipMemcpyAsync(L.set_off, set_off_h, size_t(n_sets + 1) * 8, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_check_sets, dim3(unsigned((n_sets + 255) / 256)), dim3(256), 0, s,
                               text, L.set_off, uint32_t(n_sets), L.state + kStErr);
            SA_HIP(hipGetLastError());
            set_off_dev = L.set_off;
        }
        SA_TRY(sort_prepare(L.sb, n, key0_bits, t, s));
        int nparts = 0;
        SA_TRY(launch_key0(L.packed, L.sepmask, n, h0, set_off_dev, n_sets, key0_bits, L.sb, 0, t, s, &nparts));
        int cur = 0;
        SA_TRY(sort_run(L.sb, 0, nullptr, n, 0, key0_bits, t, nparts, s, &cur));
        SA_TRY(launch_rank_update(L.sb.keys[cur], L.sb.vals[cur], nullptr, n, n, true, h0, rbits,
                                  sa, rank, L.slots[0], L.pos, L.lbflags, L.lb_words, L.tickets,
                                  L.state, s));
        hipLaunchKernelGGL(k_round_end, dim3(1), dim3(64), 0, s, L.state, uint32_t(h0));
        SA_HIP(hipGetLastError());
        return SA_OK;
    }

    // One doubling round reading its slots from slots[sl] and writing slots[sl ^ 1]; a_bound
    // bounds the active count (grid and fill sizes).  Groups of at most kRunMax members are
    // sorted run by run in LDS (k_keys_runs).  Unless runs_only, the items of larger groups,
    // if the device state says there are any (state[kStBig]), are taken out with their keys,
    // sorted by radix passes and put back in their groups' places; every kernel of that part
    // reads its count from device memory and does nothing when it is 0.  runs_only leaves
    // that part out, for rounds after one whose groups all had at most kRunMax members: groups
    // only split, so that stays true (a longer run would raise kErrRange).
    int doubling_round(int sl, int64_t a_bound, bool runs_only = false) {
        int cur = 0;
        if (!runs_only) {
            const int bits = 2 * rbits;
            SA_TRY(sort_prepare(L.sb, a_bound, bits, t, s));
            int nparts = 0;
            timing_scope_mode(kModeRadix);
            SA_TRY(launch_big_extract(L.pos, L.slots[sl], rank, n, rbits, a_bound, L.sb, L.bigidx,
                                      L.lbflags, L.lb_words, L.tickets, L.state, t, s, &nparts));
            SA_TRY(sort_run(L.sb, 0, L.state + kStRadixN, a_bound, 0, bits, t, nparts, s, &cur));
        }
        // the round's full list goes to the buffer the passes did not end in
        uint64_t *K = L.sb.keys[cur ^ 1];
        uint32_t *V = L.sb.vals[cur ^ 1];
        timing_scope_mode(kModeRuns);
        SA_TRY(launch_keys_runs(L.pos, L.slots[sl], rank, a_bound, n, rbits, L.state, K, V,
                                L.state + kStErr, s));
        if (!runs_only) {
            timing_scope_mode(kModeRadix);
            SA_TRY(launch_big_place(L.sb.keys[cur], L.sb.vals[cur], L.bigidx, a_bound, L.state, K, V,
                                    L.state + kStErr, s));
        }
        timing_scope_mode(kModeAny);
        SA_TRY(launch_rank_update(K, V, L.slots[sl], a_bound, n, false, h0, rbits, sa, rank,
                                  L.slots[sl ^ 1], L.pos, L.lbflags, L.lb_words, L.tickets,
                                  L.state, s));
        hipLaunchKernelGGL(k_round_end, dim3(1), dim3(64), 0, s, L.state, uint32_t(h0));
        SA_HIP(hipGetLastError());
        return SA_OK;
    }

    int run(bool use_graph, int *rounds_out) {
        rbits = bits_for(n - 1);
        SA_TRY(round0());
        uint32_t host[kStWords];
        if (use_graph) {
            SA_TRY(read_state(host));
            SA_TRY(check_err(host[kStErr]));
            int64_t A = host[kStActive];
            if (A > 0) {
                // Record two rounds (the slot buffers alternate) once and replay until done.
                // Capture on a private stream (the caller's may be the legacy default stream,
                // which cannot be captured); the graph is then launched on the caller's stream.
                const int64_t bound = A;
                hipGraph_t graph = nullptr;
                hipGraphExec_t exec = nullptr;
                hipStream_t cap = nullptr;
                SA_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
                const hipStream_t caller = s;
                s = cap;
                timing_pause(true);
                hipError_t be = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
                int rc = be == hipSuccess ? SA_OK : fail(SA_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(be));
                if (rc == SA_OK) rc = doubling_round(0, bound);
                if (rc == SA_OK) rc = doubling_round(1, bound);
                hipError_t ce = be == hipSuccess ? hipStreamEndCapture(cap, &graph) : hipSuccess;
                timing_pause(false);
                s = caller;
                hipStreamDestroy(cap);
                if (rc != SA_OK) {
                    if (graph) hipGraphDestroy(graph);
                    return rc;
                }
                SA_HIP(ce);
                hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                hipGraphDestroy(graph);
                SA_HIP(ie);
                int guard = 0;
                while (A > 0) {
                    if (++guard > 40) {
                        hipGraphExecDestroy(exec);
                        return fail(SA_ERR_HIP, "sa_build: doubling did not converge");
                    }
                    hipError_t le = hipGraphLaunch(exec, s);
                    if (le != hipSuccess) {
                        hipGraphExecDestroy(exec);
                        SA_HIP(le);
                    }
                    int rr = read_state(host);
                    if (rr != SA_OK) { hipGraphExecDestroy(exec); return rr; }
                    if (host[kStErr]) { hipGraphExecDestroy(exec); return check_err(host[kStErr]); }
                    A = host[kStActive];
                }
                SA_HIP(hipGraphExecDestroy(exec));
            }
        } else {
            // One round ahead: round r+1 is enqueued before the host looks at the state round r
            // left (copied to pinned memory behind an event), so the readback overlaps device
            // work.  A round enqueued after the last useful one finds no active suffix and every
            // kernel of it returns at once.  A round's bounds (grid and fill sizes) use the last
            // count the host has seen, which can only be larger than the true one.
            PinnedState &ps = pinned_state();
            if (!ps.ok) return fail(SA_ERR_HIP, "sa_build: no pinned host memory for round state");
            int cur = 0, sl = 0;
            int64_t bound = n;
            SA_TRY(snapshot(ps, cur));  // state after round 0
            // Round 1 waits for round 0's state: if its groups are all small, no round needs
            // the radix passes again.
            SA_HIP(hipEventSynchronize(ps.ev[cur]));
            bool runs_only = ps.h[kStWords * cur + kStBig] == 0;
            // A round's units of work are known one round late: its active count from the
            // state before it, its large-group item count from the state after it.
            int64_t prev_tag = -1, prev_active = 0;
            for (int guard = 0;; ++guard) {
                if (guard > 40) return fail(SA_ERR_HIP, "sa_build: doubling did not converge");
                const int64_t tag = timing_round_begin();
                SA_TRY(doubling_round(sl, bound, runs_only));
                SA_TRY(snapshot(ps, cur ^ 1));
                sl ^= 1;
                SA_HIP(hipEventSynchronize(ps.ev[cur]));
                memcpy(host, ps.h + kStWords * cur, sizeof(uint32_t) * kStWords);
                if (prev_tag >= 0) timing_round_items(prev_tag, prev_active, host[kStBigLast]);
                prev_tag = tag;
                prev_active = host[kStActive];  // the state before the round just enqueued
                timing_poll();
                SA_TRY(check_err(host[kStErr]));
                if (host[kStBig] == 0) runs_only = true;
                cur ^= 1;
                if (host[kStActive] == 0) {
                    // the round just enqueued is a no-op; wait for it so the stream is clean
                    SA_HIP(hipEventSynchronize(ps.ev[cur]));
                    memcpy(host, ps.h + kStWords * cur, sizeof(uint32_t) * kStWords);
                    timing_round_items(prev_tag, 0, 0);
                    timing_flush();
                    SA_TRY(check_err(host[kStErr]));
                    break;
                }
                bound = host[kStActive];
            }
        }
        if (rounds_out) *rounds_out = int(host[kStRounds]);
        return SA_OK;
    }
};

// lcp_or_null (batched builds only): the LCP array of this build's texts is computed after it
// from the final labels; a failure found on the device goes to lcp_flag[0].
static int build_common(const uint8_t *text, int64_t n, const int64_t *set_off_h, int32_t n_sets,
                        int32_t *sa, int32_t *isa_or_null, void *ws, int64_t ws_bytes,
                        const sa_tuning *tune, bool use_graph, int32_t *rounds_h,
                        hipStream_t stream, int64_t need, int32_t *lcp_or_null = nullptr,
                        int32_t *lcp_flag = nullptr) {
    Tune t;
    SA_TRY(resolve_tuning(tune, &t));
    if (ws_bytes < need)
        return fail(SA_ERR_NOMEM, "workspace too small (need " + std::to_string(need) + " bytes)");
    Build B;
    B.text = text;
    B.n = n;
    B.n_sets = n_sets;
    B.set_off_h = set_off_h;
    B.sa = sa;
    B.t = t;
    B.s = stream;
    Carver c(ws, ws_bytes);
    carve_build(c, n, n_sets, t, &B.L);
    B.L.sb.err = B.L.state + kStErr;
    B.rank = isa_or_null ? reinterpret_cast<uint32_t *>(isa_or_null) : B.L.rank;
    if (n_sets > 0) {
        int sb = 0;
        while ((int64_t(1) << sb) < n_sets) ++sb;
        B.h0 = (63 - 5 - sb) / 2 < kH0 ? (63 - 5 - sb) / 2 : kH0;
        if (B.h0 < 1) return fail(SA_ERR_INVALID, "too many texts in one batch");
        B.key0_bits = 2 * B.h0 + 5 + sb;
    }
    int rounds = 0;
    SA_TRY(B.run(use_graph, &rounds));
    if (lcp_or_null) {
        if (n_sets < 1 || !B.L.lcp_ws) return fail(SA_ERR_INVALID, "LCP output needs a batched build");
        int64_t span = 0;  // the largest text of the batch
        for (int32_t k = 0; k < n_sets; ++k)
            span = set_off_h[k + 1] - set_off_h[k] > span ? set_off_h[k + 1] - set_off_h[k] : span;
        SA_TRY(lcp_run(text, n, sa, reinterpret_cast<const int32_t *>(B.rank), lcp_or_null,
                       B.L.lcp_ws, B.L.lcp_ws_bytes, stream, lcp_flag, span));
    }
    if (rounds_h) *rounds_h = rounds;
    return SA_OK;
}

}  // namespace saasm

using namespace saasm;

extern "C" int64_t sa_build_ws_bytes(int64_t n, const sa_tuning *tune) {
    Tune t;
    if (n < 1 || resolve_tuning(tune, &t) != SA_OK) return -1;
    Carver c(nullptr, INT64_MAX);
    BuildLayout L;
    carve_build(c, n, 0, t, &L);
    return c.off + 256;
}

static int sa_build_impl(const uint8_t *text, int64_t n, int32_t *sa, int32_t *isa_or_null,
                        void *ws, int64_t ws_bytes, const sa_tuning *tune, int32_t *rounds_h,
                        hipStream_t stream) {
    if (!text || !sa || !ws) return fail(SA_ERR_INVALID, "sa_build: NULL pointer");
    if (n < 1) return fail(SA_ERR_INVALID, "sa_build: n must be >= 1");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_build: n >= 2^31-2");
    const int64_t need = sa_build_ws_bytes(n, tune);
    if (need < 0) return fail(SA_ERR_INVALID, "sa_build: bad tuning");
    return build_common(text, n, nullptr, 0, sa, isa_or_null, ws, ws_bytes, tune, false, rounds_h,
                        stream, need);
}

// Groups of consecutive texts with at most `pack` characters each (a text longer than `pack`
// forms a group of its own); pack <= 0 puts every text in one group.  Returns group bounds.
static std::vector<int32_t> pack_groups(const int64_t *off, int32_t n_sets, int64_t pack) {
    std::vector<int32_t> g{0};
    if (pack <= 0) {
        g.push_back(n_sets);
        return g;
    }
    int32_t start = 0;
    for (int32_t s = 0; s < n_sets; ++s) {
        if (s > start && off[s + 1] - off[start] > pack) {
            g.push_back(s);
            start = s;
        }
    }
    g.push_back(n_sets);
    return g;
}

static int resolve_batched(const sa_tuning *tune, Tune *t, int64_t *pack) {
    sa_tuning copy{};
    if (tune) copy = *tune;
    *pack = copy.seg_pack;
    copy.seg_pack = 0;
    if (*pack < 0) return fail(SA_ERR_INVALID, "seg_pack must be >= 0");
    return resolve_tuning(&copy, t);
}

extern "C" int64_t sa_build_batched_ws_bytes(int64_t n, int32_t n_sets, const int64_t *set_off_h,
                                             const sa_tuning *tune) {
    Tune t;
    int64_t pack = 0;
    if (n < 1 || n_sets < 1 || resolve_batched(tune, &t, &pack) != SA_OK) return -1;
    int64_t need = 0;
    if (pack > 0 && set_off_h) {
        std::vector<int32_t> g = pack_groups(set_off_h, n_sets, pack);
        for (size_t k = 0; k + 1 < g.size(); ++k) {
            Carver c(nullptr, INT64_MAX);
            BuildLayout L;
            carve_build(c, set_off_h[g[k + 1]] - set_off_h[g[k]], g[k + 1] - g[k], t, &L);
            need = c.off > need ? c.off : need;
        }
    } else {
        Carver c(nullptr, INT64_MAX);
        BuildLayout L;
        carve_build(c, n, n_sets, t, &L);
        need = c.off;
    }
    return need + 256;
}

static int sa_build_batched_impl(const uint8_t *text, int64_t n, const int64_t *set_off_h,
                                int32_t n_sets, int32_t *sa, int32_t *isa_or_null,
                                int32_t *lcp_or_null, void *ws, int64_t ws_bytes,
                                const sa_tuning *tune, int32_t use_graph, int32_t *rounds_h,
                                hipStream_t stream) {
    if (!text || !sa || !ws || !set_off_h) return fail(SA_ERR_INVALID, "sa_build_batched: NULL pointer");
    if (n < 1 || n_sets < 1) return fail(SA_ERR_INVALID, "sa_build_batched: need n >= 1 and n_sets >= 1");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_build_batched: n >= 2^31-2");
    if (set_off_h[0] != 0 || set_off_h[n_sets] != n)
        return fail(SA_ERR_INVALID, "sa_build_batched: offsets must start at 0 and end at n");
    for (int32_t i = 0; i < n_sets; ++i)
        if (set_off_h[i + 1] <= set_off_h[i])
            return fail(SA_ERR_INVALID, "sa_build_batched: every text must be non-empty");
    Tune t;
    int64_t pack = 0;
    SA_TRY(resolve_batched(tune, &t, &pack));
    const int64_t need = sa_build_batched_ws_bytes(n, n_sets, set_off_h, tune);
    if (need < 0) return fail(SA_ERR_INVALID, "sa_build_batched: bad tuning");
    sa_tuning inner{t.dbits, t.block, t.items, 0};
    std::vector<int32_t> g = pack_groups(set_off_h, n_sets, pack);
    int32_t rounds_max = 0;
    for (size_t k = 0; k + 1 < g.size(); ++k) {
        const int32_t s0 = g[k], s1 = g[k + 1];
        const int64_t base = set_off_h[s0], len = set_off_h[s1] - base;
        std::vector<int64_t> local(size_t(s1 - s0) + 1);
        for (int32_t s = s0; s <= s1; ++s) local[size_t(s - s0)] = set_off_h[s] - base;
        int32_t r = 0;
        SA_TRY(build_common(text + base, len, local.data(), s1 - s0, sa + base,
                            isa_or_null ? isa_or_null + base : nullptr, ws, ws_bytes, &inner,
                            use_graph != 0, &r, stream, need,
                            lcp_or_null ? lcp_or_null + base : nullptr, lcp_or_null));
        if (base > 0) {
            hipLaunchKernelGGL(k_add_offset, dim3(unsigned((len + 255) / 256)), dim3(256), 0, stream,
                               sa + base, isa_or_null ? isa_or_null + base : nullptr, len,
                               int32_t(base));
            SA_HIP(hipGetLastError());
        }
        rounds_max = r > rounds_max ? r : rounds_max;
    }
    if (rounds_h) *rounds_h = rounds_max;
    return SA_OK;
}

// ---- C entry points: bodies above, host exceptions turned into statuses ------------------
extern "C" int sa_build(const uint8_t *text, int64_t n, int32_t *sa, int32_t *isa_or_null,
                        void *ws, int64_t ws_bytes, const sa_tuning *tune, int32_t *rounds_h,
                        hipStream_t stream) {
    return guard<int>([&] { return sa_build_impl(text, n, sa, isa_or_null, ws, ws_bytes, tune, rounds_h, stream); });
}

extern "C" int sa_build_batched(const uint8_t *text, int64_t n, const int64_t *set_off_h,
                                int32_t n_sets, int32_t *sa, int32_t *isa_or_null,
                                int32_t *lcp_or_null, void *ws, int64_t ws_bytes,
                                const sa_tuning *tune, int32_t use_graph, int32_t *rounds_h,
                                hipStream_t stream) {
    return guard<int>([&] { return sa_build_batched_impl(text, n, set_off_h, n_sets, sa, isa_or_null, lcp_or_null, ws, ws_bytes, tune, use_graph, rounds_h, stream); });
}

// One workspace for sa_build, sa_lcp and sa_overlaps (up to n candidate matches).
extern "C" int64_t sa_workspace_bytes(int64_t n, int64_t n_reads_upper) {
    if (n < 1) return -1;
    const int64_t m = n_reads_upper <= 0 || n_reads_upper > n ? n : n_reads_upper;
    const int64_t b = sa_build_ws_bytes(n, nullptr);
    const int64_t l = sa_lcp_ws_bytes(n);
    const int64_t o = sa_overlaps_ws_bytes(n, m, n);
    int64_t need = b > l ? b : l;
    return need > o ? need : o;
}
