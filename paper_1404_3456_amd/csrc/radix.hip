// radix.hip -- LSD radix sort of (uint64 key, uint32 value) pairs for gfx950, plus the two key
// builders of the suffix-array rounds (fused with the sort's digit histograms).
//
// Sec. IV describes the radix sort the paper builds the suffix array with: each pass is a
// counting sort in which an element's output index is the number of elements in lower
// buckets plus the number already placed in its own bucket, and a pass is (1) a split of each
// on-chip chunk by the current digit, (2) per-chunk bucket counts stored digit-major, (3) a
// prefix sum over that table and (4) a scatter.  Alg. 1 is one such split for one bit.
//
// Here one pass is one kernel per tile of keys ("onesweep"):
//   * the digit counts of every pass are taken once, up front (k_hist or the key builders),
//     and summed and scanned per pass into global digit bases (k_hist_sum, k_hist_bases);
//   * each workgroup ranks its tile by digit with wave64 ballots (a d-bit multisplit instead
//     of d one-bit splits), publishes its per-digit counts in a (tile x digit) table and
//     reads the prefix of earlier tiles from that table by decoupled look-back -- the prefix
//     sum of the paper's step (3) done in the same launch;
//   * it then stages the tile in LDS in digit order and writes each digit's run contiguously,
//     so the scatter of step (4) is coalesced.
// Tiles take their index from an atomic ticket, so every tile a look-back waits on is already
// resident; every wait is bounded (kSpinLimit) so that all waves exit even on a fault.
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"

namespace saasm {

int sort_passes(int bits, const Tune &t) { return bits <= 0 ? 0 : (bits + t.dbits - 1) / t.dbits; }

static int64_t sort_tiles(int64_t n, const Tune &t) {
    int64_t tl = (n + t.tile() - 1) / t.tile();
    return tl < 1 ? 1 : tl;
}

int64_t sort_flag_words(int64_t n, int bits, const Tune &t) {
    return int64_t(sort_passes(bits, t)) * sort_tiles(n, t) * t.radix();
}

void carve_sort(Carver &c, int64_t n, int bits, const Tune &t, SortBufs *b, bool with_items) {
    const int P = sort_passes(bits, t) > 0 ? sort_passes(bits, t) : 1;
    if (with_items) {
        b->keys[0] = c.take<uint64_t>(n);
        b->keys[1] = c.take<uint64_t>(n);
        b->vals[0] = c.take<uint32_t>(n);
        b->vals[1] = c.take<uint32_t>(n);
    }
    b->hist = c.take<uint32_t>(int64_t(kHistParts) * P * t.radix());
    b->gbase = c.take<uint32_t>(int64_t(P) * t.radix());
    b->flags = c.take<uint32_t>(sort_flag_words(n, bits, t) > 0 ? sort_flag_words(n, bits, t) : 1);
    b->tickets = c.take<uint32_t>(64);
}

int sort_prepare(const SortBufs &b, int64_t n, int bits, const Tune &t, hipStream_t s) {
    const int P = sort_passes(bits, t);
    if (P == 0) return SA_OK;
    SA_TRY(launch_fill_u32(b.flags, sort_flag_words(n, bits, t), 0, s));
    SA_TRY(launch_fill_u32(b.tickets, 64, 0, s));
    return SA_OK;
}

// ---- digit histograms ---------------------------------------------------------------------
__device__ __forceinline__ uint64_t field(uint64_t k, int bit_lo, int bits) {
    k >>= bit_lo;
    return bits >= 64 ? k : (k & ((uint64_t(1) << bits) - 1));
}

template <int D>
__device__ __forceinline__ void hist_add(uint32_t *s_h, uint64_t f, int passes) {
    constexpr int R = 1 << D;
    for (int p = 0; p < passes; ++p)
        atomicAdd(&s_h[p * R + uint32_t((f >> (p * D)) & (R - 1))], 1u);
}

// Each workgroup stores its whole LDS histogram as one partial (plain stores, no atomics).
template <int D>
__device__ __forceinline__ void hist_flush(const uint32_t *s_h, uint32_t *part, int passes) {
    constexpr int R = 1 << D;
    uint32_t *dst = part + size_t(blockIdx.x) * passes * R;
    for (int i = threadIdx.x; i < passes * R; i += blockDim.x) dst[i] = s_h[i];
}

template <int D>
__global__ __launch_bounds__(256) void k_hist(const uint64_t *__restrict__ keys, uint32_t n,
                                              int bit_lo, int bits, int passes,
                                              uint32_t *__restrict__ hist) {
    constexpr int R = 1 << D;
    extern __shared__ uint32_t s_h[];
    for (int i = threadIdx.x; i < passes * R; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        hist_add<D>(s_h, field(keys[i], bit_lo, bits), passes);
    __syncthreads();
    hist_flush<D>(s_h, hist, passes);
}

// Digit totals of every pass from the per-workgroup partial histograms: workgroup (pass,
// g) sums digits 64g .. 64g+63 with 16 threads per digit, each over every 16th partial.
constexpr int kHsBlock = 1024;
constexpr int kHsDigits = 64;
constexpr int kHsSlices = kHsBlock / kHsDigits;
template <int D>
__global__ __launch_bounds__(kHsBlock) void k_hist_sum(const uint32_t *__restrict__ part,
                                                       int nparts, int passes,
                                                       uint32_t *__restrict__ tot) {
    constexpr int R = 1 << D;
    __shared__ uint32_t s_part[kHsSlices][kHsDigits];
    const int pass = blockIdx.x, dl = threadIdx.x % kHsDigits, sl = threadIdx.x / kHsDigits;
    const int d = blockIdx.y * kHsDigits + dl;
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    if (d < R) {
        const uint32_t *src = part + size_t(pass) * R + d;
        const size_t stride = size_t(passes) * R;
        int w = sl;
        for (; w + 3 * kHsSlices < nparts; w += 4 * kHsSlices) {
            a0 += src[size_t(w) * stride];
            a1 += src[size_t(w + kHsSlices) * stride];
            a2 += src[size_t(w + 2 * kHsSlices) * stride];
            a3 += src[size_t(w + 3 * kHsSlices) * stride];
        }
        for (; w < nparts; w += kHsSlices) a0 += src[size_t(w) * stride];
    }
    s_part[sl][dl] = a0 + a1 + a2 + a3;
    __syncthreads();
    if (sl == 0 && d < R) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < kHsSlices; ++k) c += s_part[k][dl];
        tot[size_t(pass) * R + d] = c;
    }
}

// Exclusive scan of one pass's digit totals into digit bases, in place (one workgroup per pass).
template <int D>
__global__ __launch_bounds__(kHsBlock) void k_hist_bases(uint32_t *__restrict__ gbase) {
    constexpr int R = 1 << D;
    constexpr int PER = (R + kHsBlock - 1) / kHsBlock;  // digits per thread
    __shared__ uint32_t s_w[kHsBlock / kWave];
    uint32_t *g = gbase + size_t(blockIdx.x) * R;
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int d = threadIdx.x * PER + j;
        v[j] = d < R ? g[d] : 0u;
        sum += v[j];
    }
    uint32_t total;
    uint32_t run = block_excl_sum<kHsBlock>(sum, s_w, &total);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int d = threadIdx.x * PER + j;
        if (d < R) g[d] = run;
        run += v[j];
    }
}

template <int D>
static void launch_hist_scan(const uint32_t *hist, int nparts, int P, uint32_t *gbase,
                             hipStream_t s) {
    constexpr int R = 1 << D;
    hipLaunchKernelGGL(k_hist_sum<D>, dim3(unsigned(P), unsigned((R + kHsDigits - 1) / kHsDigits)),
                       dim3(kHsBlock), 0, s, hist, nparts, P, gbase);
    hipLaunchKernelGGL(k_hist_bases<D>, dim3(unsigned(P)), dim3(kHsBlock), 0, s, gbase);
}

static unsigned hist_grid(int64_t n) {
    int64_t b = (n + 4095) / 4096;
    if (b > kHistParts) b = kHistParts;
    if (b < 1) b = 1;
    return unsigned(b);
}

int launch_hist(const SortBufs &b, int cur, int64_t n, int bit_lo, int bits, const Tune &t,
                hipStream_t s, int *nparts) {
    const int P = sort_passes(bits, t);
    *nparts = int(hist_grid(n));
    if (P == 0 || n == 0) return SA_OK;
    size_t lds = size_t(P) * t.radix() * 4;
    switch (t.dbits) {
        case 4: hipLaunchKernelGGL(k_hist<4>, dim3(hist_grid(n)), dim3(256), lds, s, b.keys[cur], uint32_t(n), bit_lo, bits, P, b.hist); break;
        case 8: hipLaunchKernelGGL(k_hist<8>, dim3(hist_grid(n)), dim3(256), lds, s, b.keys[cur], uint32_t(n), bit_lo, bits, P, b.hist); break;
        case 9: hipLaunchKernelGGL(k_hist<9>, dim3(hist_grid(n)), dim3(256), lds, s, b.keys[cur], uint32_t(n), bit_lo, bits, P, b.hist); break;
        case 11: hipLaunchKernelGGL(k_hist<11>, dim3(hist_grid(n)), dim3(256), lds, s, b.keys[cur], uint32_t(n), bit_lo, bits, P, b.hist); break;
        default: return fail(SA_ERR_INVALID, "unsupported digit width");
    }
    SA_HIP(hipGetLastError());
    return SA_OK;
}

// Ranks one wave's ITEMS x 64 items by digit, stably: pos[k] = the wave's running count of the
// item's digit before it (items in index order, k-major, lane-minor).  Each item's peers (the
// lanes holding the same digit) come from ballots over the digit bits; the lowest peer advances
// the count in LDS.  FULL: every item is valid (a full tile), so no validity test is made.
template <int D, int ITEMS, bool FULL, class Cnt>
__device__ __forceinline__ void rank_wave(const uint64_t (&key)[ITEMS], uint32_t (&pos)[ITEMS],
                                          uint32_t wbase, uint32_t n, uint32_t lane,
                                          uint32_t shift, uint32_t dmask, Cnt *wcnt) {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const bool valid = FULL || wbase + k * kWave + lane < n;
        const uint32_t dg = valid ? (uint32_t(key[k] >> shift) & dmask) : 0u;
        uint32_t mlo = ~0u, mhi = ~0u;
        if (!FULL) {
            const uint64_t vm = ballot(valid);
            mlo = uint32_t(vm);
            mhi = uint32_t(vm >> 32);
        }
#pragma unroll
        for (int b = 0; b < D; ++b) {
            uint32_t sb = uint32_t(int32_t(dg << (31 - b)) >> 31);  // all ones iff bit b set
            asm("" : "+v"(sb));  // keep sb in a register so the ballot compares it directly
            const uint64_t bb = ballot(sb != 0);
            // keep the lanes whose bit b equals this lane's: m & ~(ballot ^ sb), one v_bitop3
            // per half (truth table indexed by (m, ballot, sb) bits: 1 at 100b and 111b)
            mlo = __builtin_amdgcn_bitop3_b32(mlo, uint32_t(bb), sb, 0x90);
            mhi = __builtin_amdgcn_bitop3_b32(mhi, uint32_t(bb >> 32), sb, 0x90);
        }
        // peers in lower lanes: popcount(m & lanes below), by mbcnt
        const uint32_t r = __builtin_amdgcn_mbcnt_hi(mhi, __builtin_amdgcn_mbcnt_lo(mlo, 0u));
        if (valid) {
            const uint32_t c0 = wcnt[dg];
            pos[k] = c0 + r;
            if (r == 0) wcnt[dg] = Cnt(c0 + uint32_t(__popc(mlo) + __popc(mhi)));
        }
        wave_sync();
    }
}

// ---- one LSD pass ---------------------------------------------------------------------------
// One tile per workgroup, tiles numbered by ticket.  The grid covers an upper bound on the
// item count; the count itself is read from device memory when `count_dev` is given (so the
// same launch can be recorded in a graph and replayed with whatever count an earlier kernel
// produced; surplus workgroups exit at once), otherwise it is `n_host`.
template <int D, int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_onesweep(const uint64_t *__restrict__ kin,
                                                    const uint32_t *__restrict__ vin,
                                                    uint64_t *__restrict__ kout,
                                                    uint32_t *__restrict__ vout,
                                                    const uint32_t *count_dev, uint32_t n_host,
                                                    uint32_t shift, uint32_t dmask,
                                                    const uint32_t *__restrict__ gbase,
                                                    uint32_t *flags, uint32_t *tick,
                                                    uint32_t *err) {
    constexpr int R = 1 << D;
    constexpr int W = BLOCK / kWave;
    constexpr int TILE = BLOCK * ITEMS;
    constexpr int DPT = (R + BLOCK - 1) / BLOCK;  // digits owned per thread (blocked)
    using Cnt = typename std::conditional<(R > 256), uint16_t, uint32_t>::type;

    __shared__ uint32_t s_tile;
    __shared__ Cnt s_wcnt[W * R];      // per-wave running counts, then per-wave prefixes
    __shared__ uint32_t s_lstart[R];   // first local slot of each digit
    __shared__ uint32_t s_gofs[R];     // global output index minus local slot, per digit
    __shared__ uint32_t s_scan[W];
    __shared__ uint64_t s_stage[TILE]; // tile in digit order (keys, then values)

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t n = count_dev ? *count_dev : n_host;
    const uint32_t ntiles = (n + TILE - 1) / TILE;

    {
        if (tid == 0) s_tile = ticket(tick);
        for (int i = tid; i < W * R; i += BLOCK) s_wcnt[i] = 0;
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) return;
        const uint32_t tbase = tile * TILE;
        const uint32_t wbase = tbase + wave * (ITEMS * kWave);

        uint64_t key[ITEMS];
        uint32_t val[ITEMS];
        uint32_t pos[ITEMS];
        const bool full = tbase + uint32_t(TILE) <= n;
        if (full) {  // one base address per wave and immediate offsets per item
            const uint64_t *kp = kin + (wbase + lane);
            const uint32_t *vp = vin + (wbase + lane);
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                key[k] = kp[k * kWave];
                val[k] = vp[k * kWave];
            }
        } else {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const uint32_t idx = wbase + k * kWave + lane;
                key[k] = idx < n ? kin[idx] : 0;
                val[k] = idx < n ? vin[idx] : 0;
            }
        }

        // Stable rank of every item among the items of its wave with the same digit: items
        // are taken in index order (k-major, lane-minor), the running count per digit in LDS.
        if (full) rank_wave<D, ITEMS, true>(key, pos, wbase, n, lane, shift, dmask, s_wcnt + wave * R);
        else rank_wave<D, ITEMS, false>(key, pos, wbase, n, lane, shift, dmask, s_wcnt + wave * R);
        __syncthreads();

        // Per digit: exclusive prefix over waves, and the tile total.
        uint32_t tot[DPT];
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            uint32_t run = 0;
            if (d < R) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    uint32_t c = s_wcnt[w * R + d];
                    s_wcnt[w * R + d] = Cnt(run);
                    run += c;
                }
            }
            tot[j] = run;
        }
        // Publish this tile's counts before looking back, so later tiles can proceed.
        uint32_t *myflags = flags + size_t(tile) * R;
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            if (d < R) st_agent(myflags + d, lb32_word(tile == 0, tot[j]));
        }
        uint32_t tsum = 0;
#pragma unroll
        for (int j = 0; j < DPT; ++j) tsum += tot[j];
        uint32_t tile_total;
        uint32_t run = block_excl_sum<BLOCK>(tsum, s_scan, &tile_total);
        // Local digit starts first: the tile is staged in digit order while the digit owners
        // look back for the global offsets (only the final scatter needs those).
        uint32_t lstart[DPT];
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            lstart[j] = run;
            if (d < R) s_lstart[d] = run;
            run += tot[j];
        }
        __syncthreads();

        // Stage keys in digit order.
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = wbase + k * kWave + lane;
            if (idx < n) {
                const uint32_t dg = uint32_t(key[k] >> shift) & dmask;
                const uint32_t lp = s_lstart[dg] + uint32_t(s_wcnt[wave * R + dg]) + pos[k];
                s_stage[lp] = key[k];
                pos[k] = lp;
            }
        }
#pragma unroll
        for (int j = 0; j < DPT; ++j) {
            const int d = tid * DPT + j;
            if (d < R) {
                uint32_t ex = 0;
                if (tile > 0) {
                    ex = lookback_digit(flags, int(tile), R, d, err);
                    st_agent(myflags + d, lb32_word(true, ex + tot[j]));
                }
                s_gofs[d] = gbase[d] + ex - lstart[j];
            }
        }
        __syncthreads();
        const uint32_t tcount = (n - tbase) < uint32_t(TILE) ? (n - tbase) : uint32_t(TILE);
        uint32_t opos[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t lp = j * BLOCK + tid;
            opos[j] = 0xffffffffu;
            if (lp < tcount) {
                const uint64_t kk = s_stage[lp];
                const uint32_t dg = uint32_t(kk >> shift) & dmask;
                const uint32_t o = lp + s_gofs[dg];
                if (o >= n) {
                    raise_err(err, kErrRange);  // only an inconsistent histogram gets here
                } else {
                    kout[o] = kk;
                    opos[j] = o;
                }
            }
        }
        __syncthreads();
        uint32_t *s_stage32 = reinterpret_cast<uint32_t *>(s_stage);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = wbase + k * kWave + lane;
            if (idx < n) s_stage32[pos[k]] = val[k];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t lp = j * BLOCK + tid;
            if (lp < tcount && opos[j] != 0xffffffffu) vout[opos[j]] = s_stage32[lp];
        }
    }
}

static int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    return cus;
}

template <int D, int BLOCK, int ITEMS>
static int launch_pass_t(int64_t n_max, hipStream_t s, const uint64_t *kin, const uint32_t *vin,
                         uint64_t *kout, uint32_t *vout, const uint32_t *count_dev,
                         uint32_t n_host, uint32_t shift, uint32_t dmask, const uint32_t *gbase,
                         uint32_t *flags, uint32_t *tick, uint32_t *err) {
    constexpr int TILE = BLOCK * ITEMS;
    int64_t grid = (n_max + TILE - 1) / TILE;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((k_onesweep<D, BLOCK, ITEMS>), dim3(unsigned(grid)), dim3(BLOCK), 0, s, kin,
                       vin, kout, vout, count_dev, n_host, shift, dmask, gbase, flags, tick, err);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

template <int D>
static int launch_pass_d(const Tune &t, int64_t n_max, hipStream_t s, const uint64_t *kin,
                         const uint32_t *vin, uint64_t *kout, uint32_t *vout,
                         const uint32_t *count_dev, uint32_t n_host, uint32_t shift,
                         uint32_t dmask, const uint32_t *gbase, uint32_t *flags, uint32_t *tick,
                         uint32_t *err) {
    if (t.block == 256 && t.items == 8)
        return launch_pass_t<D, 256, 8>(n_max, s, kin, vin, kout, vout, count_dev, n_host, shift, dmask, gbase, flags, tick, err);
    if (t.block == 256 && t.items == 16)
        return launch_pass_t<D, 256, 16>(n_max, s, kin, vin, kout, vout, count_dev, n_host, shift, dmask, gbase, flags, tick, err);
    if (t.block == 512 && t.items == 8)
        return launch_pass_t<D, 512, 8>(n_max, s, kin, vin, kout, vout, count_dev, n_host, shift, dmask, gbase, flags, tick, err);
    if (t.block == 512 && t.items == 16)
        return launch_pass_t<D, 512, 16>(n_max, s, kin, vin, kout, vout, count_dev, n_host, shift, dmask, gbase, flags, tick, err);
    if constexpr (D <= 9) {  // 1024 x 16: a 128 KB stage; with 11-bit digits the counters no longer fit
        if (t.block == 1024 && t.items == 16)
            return launch_pass_t<D, 1024, 16>(n_max, s, kin, vin, kout, vout, count_dev, n_host, shift, dmask, gbase, flags, tick, err);
    }
    return fail(SA_ERR_INVALID, "unsupported tile shape");
}

int sort_run(const SortBufs &b, int cur, const uint32_t *count_dev, int64_t n, int bit_lo,
             int bits, const Tune &t, int nparts, hipStream_t s, int *cur_out) {
    const int P = sort_passes(bits, t);
    *cur_out = cur;
    if (P == 0 || n <= 1) return SA_OK;
    const int R = t.radix();
    switch (t.dbits) {
        case 4: launch_hist_scan<4>(b.hist, nparts, P, b.gbase, s); break;
        case 8: launch_hist_scan<8>(b.hist, nparts, P, b.gbase, s); break;
        case 9: launch_hist_scan<9>(b.hist, nparts, P, b.gbase, s); break;
        case 11: launch_hist_scan<11>(b.hist, nparts, P, b.gbase, s); break;
        default: return fail(SA_ERR_INVALID, "unsupported digit width");
    }
    SA_HIP(hipGetLastError());
    const int64_t tiles = sort_tiles(n, t);
    for (int p = 0; p < P; ++p) {
        const int lo = p * t.dbits;
        const int width = (bits - lo) < t.dbits ? (bits - lo) : t.dbits;
        const uint32_t shift = uint32_t(bit_lo + lo);
        const uint32_t dmask = (1u << width) - 1u;
        TimedScope ts = count_dev ? TimedScope("radix_pass", 0.0, 24.0, s)
                                  : TimedScope("radix_pass", double(n) * 24.0, s, double(n));
        int rc = SA_OK;
        uint32_t *fl = b.flags + size_t(p) * tiles * R;
        switch (t.dbits) {
            case 4: rc = launch_pass_d<4>(t, n, s, b.keys[cur], b.vals[cur], b.keys[cur ^ 1], b.vals[cur ^ 1], count_dev, uint32_t(n), shift, dmask, b.gbase + p * R, fl, b.tickets + p, b.err); break;
            case 8: rc = launch_pass_d<8>(t, n, s, b.keys[cur], b.vals[cur], b.keys[cur ^ 1], b.vals[cur ^ 1], count_dev, uint32_t(n), shift, dmask, b.gbase + p * R, fl, b.tickets + p, b.err); break;
            case 9: rc = launch_pass_d<9>(t, n, s, b.keys[cur], b.vals[cur], b.keys[cur ^ 1], b.vals[cur ^ 1], count_dev, uint32_t(n), shift, dmask, b.gbase + p * R, fl, b.tickets + p, b.err); break;
            case 11: rc = launch_pass_d<11>(t, n, s, b.keys[cur], b.vals[cur], b.keys[cur ^ 1], b.vals[cur ^ 1], count_dev, uint32_t(n), shift, dmask, b.gbase + p * R, fl, b.tickets + p, b.err); break;
            default: rc = fail(SA_ERR_INVALID, "unsupported digit width");
        }
        ts.finish();
        if (rc != SA_OK) return rc;
        cur ^= 1;
    }
    *cur_out = cur;
    return SA_OK;
}

// ---- key builders ---------------------------------------------------------------------------
// First-round key of suffix p (prefix length h0 <= 29): the 2-bit codes of T[p .. p+min(L_p, h0)),
// zero-padded to h0 bases, followed by min(L_p, h0) in 5 bits, where L_p is the distance from p
// to the next separator.  Comparing two such keys as integers orders the suffixes by their
// first h0 symbols with the separator below every base; keys equal with a length below h0
// belong to suffixes that end at different separators at the same offset, whose order is
// their position order (kept by the stable sort, since values are positions).  For a batch of
// independent texts the text's index is placed above these bits, so every text's suffixes
// form one contiguous block of the order.
__device__ __forceinline__ uint64_t key0_of(const uint32_t *__restrict__ packed,
                                            const uint32_t *__restrict__ sepmask, uint32_t p,
                                            uint32_t h0) {
    const uint32_t w = p >> 4, o = p & 15;
    uint64_t x = (uint64_t(packed[w]) << 32) | packed[w + 1];
    x <<= 2 * o;
    if (o) x |= uint64_t(packed[w + 2]) >> (32 - 2 * o);
    const uint32_t sw = p >> 5, so = p & 31;
    const uint64_t sm = ((uint64_t(sepmask[sw]) << 32) | sepmask[sw + 1]) << so;
    uint32_t L = sm ? uint32_t(__clzll((long long)sm)) : 64u;
    if (L > h0) L = h0;
    uint64_t code = x >> (64 - 2 * h0);
    if (L < h0) code &= ~((uint64_t(1) << (2 * (h0 - L))) - 1);
    return (code << 5) | L;
}

// Index of the text of a batch that holds position p: largest s with set_off[s] <= p.
__device__ __forceinline__ uint32_t set_of(const int64_t *__restrict__ set_off, uint32_t n_sets,
                                           uint32_t p) {
    uint32_t lo = 0, hi = n_sets;  // invariant: set_off[lo] <= p < set_off[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (set_off[mid] <= int64_t(p)) lo = mid;
        else hi = mid;
    }
    return lo;
}

constexpr int kK0Block = 1024;  // threads per key0 workgroup (grid-stride, one partial each)

template <int D>
__global__ __launch_bounds__(kK0Block) void k_key0(const uint32_t *__restrict__ packed,
                                              const uint32_t *__restrict__ sepmask, uint32_t n,
                                              uint32_t h0, const int64_t *__restrict__ set_off,
                                              uint32_t n_sets, uint64_t *__restrict__ keys,
                                              uint32_t *__restrict__ vals, int passes,
                                              uint32_t *__restrict__ hist) {
    constexpr int R = 1 << D;
    extern __shared__ uint32_t s_h[];
    for (int i = threadIdx.x; i < passes * R; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    const uint32_t stride = gridDim.x * blockDim.x;
    const int set_shift = int(2 * h0 + 5);
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        uint64_t k = key0_of(packed, sepmask, p, h0);
        if (set_off) k |= uint64_t(set_of(set_off, n_sets, p)) << set_shift;
        keys[p] = k;
        vals[p] = p;
        hist_add<D>(s_h, k, passes);
    }
    __syncthreads();
    hist_flush<D>(s_h, hist, passes);
}

int launch_key0(const uint32_t *packed, const uint32_t *sepmask, int64_t n, int h0,
                const int64_t *set_off_dev, int n_sets, int key_bits, const SortBufs &b, int cur,
                const Tune &t, hipStream_t s, int *nparts) {
    const int P = sort_passes(key_bits, t);
    *nparts = int(hist_grid(n));
    size_t lds = size_t(P) * t.radix() * 4;
    TimedScope ts("key0", double(n) * (12.0 + 0.375), s, double(n));
    const unsigned g = hist_grid(n);
    switch (t.dbits) {
        case 4: hipLaunchKernelGGL(k_key0<4>, dim3(g), dim3(kK0Block), lds, s, packed, sepmask, uint32_t(n), uint32_t(h0), set_off_dev, uint32_t(n_sets), b.keys[cur], b.vals[cur], P, b.hist); break;
        case 8: hipLaunchKernelGGL(k_key0<8>, dim3(g), dim3(kK0Block), lds, s, packed, sepmask, uint32_t(n), uint32_t(h0), set_off_dev, uint32_t(n_sets), b.keys[cur], b.vals[cur], P, b.hist); break;
        case 9: hipLaunchKernelGGL(k_key0<9>, dim3(g), dim3(kK0Block), lds, s, packed, sepmask, uint32_t(n), uint32_t(h0), set_off_dev, uint32_t(n_sets), b.keys[cur], b.vals[cur], P, b.hist); break;
        case 11: hipLaunchKernelGGL(k_key0<11>, dim3(g), dim3(kK0Block), lds, s, packed, sepmask, uint32_t(n), uint32_t(h0), set_off_dev, uint32_t(n_sets), b.keys[cur], b.vals[cur], P, b.hist); break;
        default: return fail(SA_ERR_INVALID, "unsupported digit width");
    }
    ts.finish();
    SA_HIP(hipGetLastError());
    return SA_OK;
}

// Doubling-round keys of the items in large groups (more than kRunMax members), for the radix
// passes of a round that also has small groups.  The previous rank update left the active items
// in its sorted order: slots S[0..A) and positions P[0..A) with bit 31 on the first member of
// each group, so a group is a run of consecutive items whose label is the slot of its first
// member (a run's slots are consecutive).  An item belongs to a large group when its run is
// longer than kRunMax: that is decided from the first-of-group bits of its own 64-item row and
// the rows on either side.  For the j-th such item in order (tiles by ticket; the count of
// large items and the last run start before each tile come from a look-back):
//   keys[j] = (label << rbits) | rank[p + h],  vals[j] = p,  bigidx[j] = its index in the list,
// with the label S[i] - (i - run start), and its digits added to the passes' histograms.  The
// count goes to state[kStRadixN].  state[kStBig] == 0 (no large group) makes the launch write
// zero histograms and a count of 0.  Persistent workgroups, one partial histogram each.
constexpr int kBxBlock = 512;
constexpr int kBxWaves = kBxBlock / kWave;
constexpr int kBxRows = 256;                   // rows of 64 items per tile
constexpr int kBxK = kBxRows / kBxWaves;       // rows per wave
constexpr int kBxLoad = 8;                     // rows whose loads a wave keeps in flight
constexpr int kBxTile = kBxRows * kWave;
constexpr int kBxPer = kBxRows / kWave;        // rows per lane in the row scan

template <int D>
__global__ __launch_bounds__(kBxBlock) void k_big_extract(
    const uint32_t *__restrict__ P, const uint32_t *__restrict__ S,
    const uint32_t *__restrict__ rank, uint32_t n, int rbits, uint64_t *__restrict__ keys,
    uint32_t *__restrict__ vals, uint32_t *__restrict__ bigidx, int passes,
    uint32_t *__restrict__ hist, uint64_t *lbflags, uint32_t *tick, uint32_t *state,
    uint32_t *err) {
    constexpr int R = 1 << D;
    extern __shared__ uint32_t s_h[];
    __shared__ uint64_t s_mask[kBxRows + 2];  // first-of-group bits per row; [0] and [kBxRows+1]: context
    __shared__ uint64_t s_bigm[kBxRows];      // large-group items per row
    __shared__ uint32_t s_cnt[kBxRows];       // their count, then the exclusive count
    __shared__ uint32_t s_last[kBxRows];      // last run start + 1 in the row, then before the row
    __shared__ uint32_t s_tile;
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const uint32_t A = state[kStBig] ? state[kStActive] : 0u;
    const uint32_t h = state[kStH];
    const uint32_t ntiles = (A + kBxTile - 1) / kBxTile;
    const uint64_t rmask = (uint64_t(1) << rbits) - 1;
    const uint64_t le = lane == 63 ? ~uint64_t(0) : ((uint64_t(2) << lane) - 1);  // lanes <= lane
    for (int i = tid; i < passes * R; i += kBxBlock) s_h[i] = 0;
    if (A == 0 && blockIdx.x == 0 && tid == 0) state[kStRadixN] = 0;
    while (true) {
        __syncthreads();
        if (tid == 0) s_tile = ticket(tick);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) break;
        const uint32_t tbase = tile * kBxTile;
        // 1. first-of-group masks of the tile's rows (a streaming read of the positions)
        for (int k0 = 0; k0 < kBxK; k0 += kBxLoad) {
            uint32_t pv[kBxLoad];
#pragma unroll
            for (int k = 0; k < kBxLoad; ++k) {
                const uint32_t i = tbase + ((k0 + k) * kBxWaves + wave) * kWave + lane;
                pv[k] = i < A ? P[i] : kDone;  // past the list: a group start
            }
#pragma unroll
            for (int k = 0; k < kBxLoad; ++k) {
                const uint64_t m = ballot((pv[k] & kDone) != 0);
                if (lane == 0) s_mask[1 + (k0 + k) * kBxWaves + wave] = m;
            }
        }
        if (wave < 2) {  // the rows before and after the tile
            const int64_t i = wave == 0 ? int64_t(tbase) - kWave + lane : int64_t(tbase) + kBxTile + lane;
            const uint32_t v = (i >= 0 && i < int64_t(A)) ? P[i] : kDone;
            const uint64_t m = ballot((v & kDone) != 0);
            if (lane == 0) s_mask[wave == 0 ? 0 : kBxRows + 1] = m;
        }
        __syncthreads();
        // 2. which items lie in runs longer than kRunMax: the distance back to the run start
        //    and forward to the next one (capped), from the row and its neighbours
        for (int k = 0; k < kBxK; ++k) {
            const uint32_t row = k * kBxWaves + wave;
            const uint32_t i = tbase + row * kWave + lane;
            const uint64_t prev = s_mask[row], cur = s_mask[1 + row], next = s_mask[2 + row];
            uint32_t back = 2 * kWave, fwd = 2 * kWave;
            const uint64_t mb = cur & le;
            if (mb) back = lane - (63u - uint32_t(__clzll((long long)mb)));
            else if (prev) back = lane + 1u + uint32_t(__clzll((long long)prev));
            const uint64_t mf = cur & ~le;
            if (mf) fwd = uint32_t(__ffsll((long long)mf)) - 1u - lane;
            else if (next) fwd = kWave - lane + uint32_t(__ffsll((long long)next)) - 1u;
            const uint64_t bb = ballot(i < A && back + fwd > uint32_t(kRunMax));
            if (lane == 0) {
                s_bigm[row] = bb;
                s_cnt[row] = uint32_t(popc64(bb));
                s_last[row] = cur ? tbase + row * kWave + (63u - uint32_t(__clzll((long long)cur))) + 1u : 0u;
            }
        }
        __syncthreads();
        if (wave == 0) {  // rows in order, kBxPer per lane: (count, last start) scan, then the tiles
            uint64_t v[kBxPer];
            uint64_t run = 0;
#pragma unroll
            for (int q = 0; q < kBxPer; ++q) {
                const uint32_t row = lane * kBxPer + q;
                v[q] = run;  // exclusive within the lane's rows
                run = CountLastOp::combine(run, (uint64_t(s_cnt[row]) << 31) | s_last[row]);
            }
            const uint64_t inc = wave_incl_scan<CountLastOp>(run);
            uint64_t ex = __shfl_up(inc, 1);
            if (lane == 0) ex = 0;
            const uint64_t agg = __shfl(inc, kWave - 1);
            const uint64_t before = CountLastOp::combine(
                lookback_tile<CountLastOp>(lbflags, int(tile), agg, err), ex);
#pragma unroll
            for (int q = 0; q < kBxPer; ++q) {
                const uint32_t row = lane * kBxPer + q;
                const uint64_t tot = CountLastOp::combine(before, v[q]);
                s_cnt[row] = uint32_t(tot >> 31);
                s_last[row] = uint32_t(tot & CountLastOp::kLastMask);
            }
            if (lane == 0 && tile == ntiles - 1)
                state[kStRadixN] = uint32_t(CountLastOp::combine(before, agg) >> 31);  // lane 0: ex = 0
        }
        __syncthreads();
        // 3. keys of the large-group items (rows without any are skipped)
        for (int k = 0; k < kBxK; ++k) {
            const uint32_t row = k * kBxWaves + wave;
            const uint64_t bb = s_bigm[row];
            if (!bb || !((bb >> lane) & 1u)) continue;
            const uint32_t i = tbase + row * kWave + lane;
            const uint64_t mb = s_mask[1 + row] & le;
            const uint32_t start = mb ? tbase + row * kWave + (63u - uint32_t(__clzll((long long)mb)))
                                      : s_last[row] - 1u;  // item 0 starts a run, so s_last >= 1
            const uint32_t j = s_cnt[row] + uint32_t(popc64(bb & lanemask_lt()));
            const uint32_t p = P[i] & kRankMask;
            const uint32_t sl = S[i];
            if (start > i || sl < i - start || p >= n || h >= n - p || j >= A) {
                raise_err(err, kErrRange);
                continue;
            }
            const uint32_t label = sl - (i - start);
            const uint32_t r2 = rank[p + h] & kRankMask;
            const uint64_t key = ((uint64_t(label) & rmask) << rbits) | (uint64_t(r2) & rmask);
            keys[j] = key;
            vals[j] = p;
            bigidx[j] = i;
            hist_add<D>(s_h, key, passes);
        }
    }
    __syncthreads();
    hist_flush<D>(s_h, hist, passes);
}

// The large groups' items, sorted, to their places in the full list of the round: the j-th
// sorted item goes to the j-th large item's index (both orders list the large groups in the
// same order, each group's items contiguous).
__global__ __launch_bounds__(256) void k_big_place(const uint64_t *__restrict__ ks,
                                                   const uint32_t *__restrict__ vs,
                                                   const uint32_t *__restrict__ bigidx,
                                                   const uint32_t *state, uint64_t *__restrict__ K,
                                                   uint32_t *__restrict__ V, uint32_t *err) {
    const uint32_t B = state[kStRadixN], A = state[kStActive];
    const uint32_t stride = gridDim.x * 256u;
    for (uint32_t j = blockIdx.x * 256u + threadIdx.x; j < B; j += stride) {
        const uint32_t t = bigidx[j];
        if (t >= A) {
            raise_err(err, kErrRange);
            continue;
        }
        K[t] = ks[j];
        V[t] = vs[j];
    }
}

int launch_big_extract(const uint32_t *P, const uint32_t *S, const uint32_t *rank, int64_t n,
                       int rbits, int64_t a_bound, const SortBufs &b, uint32_t *bigidx,
                       uint64_t *lbflags, int64_t lb_words, uint32_t *tick, uint32_t *state,
                       const Tune &t, hipStream_t s, int *nparts) {
    const int bits = 2 * rbits;
    const int P_ = sort_passes(bits, t);
    const int64_t tiles = (a_bound + kBxTile - 1) / kBxTile;
    if (tiles > lb_words) return fail(SA_ERR_HIP, "large-group extraction: look-back array too small");
    static int per_cu = 0;
    if (!per_cu) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_big_extract<9>, kBxBlock, size_t(P_) * t.radix() * 4) != hipSuccess || per_cu < 1)
            per_cu = 1;
    }
    int64_t grid = int64_t(device_cus()) * per_cu;
    if (grid > kHistParts) grid = kHistParts;
    if (grid > tiles) grid = tiles;
    if (grid < 1) grid = 1;
    *nparts = int(grid);
    SA_TRY(launch_fill_u64(lbflags, tiles > 0 ? tiles : 1, 0, s));
    SA_TRY(launch_fill_u32(tick, 1, 0, s));
    size_t lds = size_t(P_) * t.radix() * 4;
    // per large item: position, slot and rank[p + h] read (12), key, value and index written (16)
    TimedScope ts("keybuild", 0.0, 28.0, s);
    switch (t.dbits) {
        case 4: hipLaunchKernelGGL(k_big_extract<4>, dim3(unsigned(grid)), dim3(kBxBlock), lds, s, P, S, rank, uint32_t(n), rbits, b.keys[0], b.vals[0], bigidx, P_, b.hist, lbflags, tick, state, b.err); break;
        case 8: hipLaunchKernelGGL(k_big_extract<8>, dim3(unsigned(grid)), dim3(kBxBlock), lds, s, P, S, rank, uint32_t(n), rbits, b.keys[0], b.vals[0], bigidx, P_, b.hist, lbflags, tick, state, b.err); break;
        case 9: hipLaunchKernelGGL(k_big_extract<9>, dim3(unsigned(grid)), dim3(kBxBlock), lds, s, P, S, rank, uint32_t(n), rbits, b.keys[0], b.vals[0], bigidx, P_, b.hist, lbflags, tick, state, b.err); break;
        case 11: hipLaunchKernelGGL(k_big_extract<11>, dim3(unsigned(grid)), dim3(kBxBlock), lds, s, P, S, rank, uint32_t(n), rbits, b.keys[0], b.vals[0], bigidx, P_, b.hist, lbflags, tick, state, b.err); break;
        default: return fail(SA_ERR_INVALID, "unsupported digit width");
    }
    ts.finish();
    SA_HIP(hipGetLastError());
    return SA_OK;
}

int launch_big_place(const uint64_t *ks, const uint32_t *vs, const uint32_t *bigidx,
                     int64_t a_bound, const uint32_t *state, uint64_t *K, uint32_t *V,
                     uint32_t *err, hipStream_t s) {
    int64_t g = (a_bound + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    // per large item: key, value and index read (16), key and value written (12)
    TimedScope ts("big_place", 0.0, 28.0, s);
    hipLaunchKernelGGL(k_big_place, dim3(unsigned(g)), dim3(256), 0, s, ks, vs, bigidx, state, K, V, err);
    ts.finish();
    SA_HIP(hipGetLastError());
    return SA_OK;
}

}  // namespace saasm

// ---- public sort entry point ---------------------------------------------------------------
using namespace saasm;

extern "C" int64_t sa_sort_ws_bytes(int64_t n, const sa_tuning *tune) {
    Tune t;
    if (n < 0 || resolve_tuning(tune, &t) != SA_OK) return -1;
    Carver c(nullptr, INT64_MAX);
    SortBufs b;
    carve_sort(c, n, 64, t, &b, false);
    c.take<uint64_t>(n);  // second key buffer
    c.take<uint32_t>(n);  // second value buffer
    c.take<uint32_t>(64); // error word
    return c.off + 256;
}

extern "C" int sa_sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int32_t bit_lo,
                             int32_t bit_hi, void *ws, int64_t ws_bytes, const sa_tuning *tune,
                             hipStream_t stream) {
    if (n < 0 || (n > 0 && (!keys || !vals || !ws)))
        return fail(SA_ERR_INVALID, "sa_sort_pairs: NULL pointer or negative n");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_sort_pairs: n >= 2^31-2");
    if (bit_lo < 0 || bit_hi > 64 || bit_lo >= bit_hi)
        return fail(SA_ERR_INVALID, "sa_sort_pairs: need 0 <= bit_lo < bit_hi <= 64");
    Tune t;
    SA_TRY(resolve_tuning(tune, &t));
    if (ws_bytes < sa_sort_ws_bytes(n, tune)) return fail(SA_ERR_NOMEM, "sa_sort_pairs: workspace too small");
    if (n <= 1) return SA_OK;
    const int bits = bit_hi - bit_lo;
    Carver c(ws, ws_bytes);
    SortBufs b;
    carve_sort(c, n, bits, t, &b, false);
    b.keys[0] = keys;
    b.vals[0] = vals;
    b.keys[1] = c.take<uint64_t>(n);
    b.vals[1] = c.take<uint32_t>(n);
    b.err = c.take<uint32_t>(64);
    if (!c.ok()) return fail(SA_ERR_NOMEM, "sa_sort_pairs: workspace too small");
    SA_TRY(launch_fill_u32(b.err, 1, 0, stream));
    SA_TRY(sort_prepare(b, n, bits, t, stream));
    int nparts = 0;
    SA_TRY(launch_hist(b, 0, n, bit_lo, bits, t, stream, &nparts));
    int cur = 0;
    SA_TRY(sort_run(b, 0, nullptr, n, bit_lo, bits, t, nparts, stream, &cur));
    if (cur == 1) {
        SA_HIP(hipMemcpyAsync(keys, b.keys[1], size_t(n) * 8, hipMemcpyDeviceToDevice, stream));
        SA_HIP(hipMemcpyAsync(vals, b.vals[1], size_t(n) * 4, hipMemcpyDeviceToDevice, stream));
    }
    uint32_t err = 0;
    SA_HIP(hipMemcpyAsync(&err, b.err, 4, hipMemcpyDeviceToHost, stream));
    SA_HIP(hipStreamSynchronize(stream));
    timing_flush();
    if (err) return fail(SA_ERR_HIP, "sa_sort_pairs: device consistency check failed (code " + std::to_string(err) + ")");
    return SA_OK;
}
