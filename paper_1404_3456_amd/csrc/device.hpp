// device.hpp -- wave64 / workgroup helpers shared by the gfx950 kernels of this library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace saasm {

constexpr int kWave = 64;

// Device-side error bits, OR-ed into a word of the workspace and reported by the host.
constexpr uint32_t kErrAlphabet = 1u;   // byte outside A,C,G,T,$
constexpr uint32_t kErrNoSepEnd = 2u;   // text[n-1] != '$'
constexpr uint32_t kErrSpin = 4u;       // a look-back wait exceeded its bound
constexpr uint32_t kErrRange = 8u;      // an index a kernel derived fell outside its array

// Upper bound on look-back polls before a wait gives up (sets kErrSpin and continues).  A
// predecessor tile always publishes without waiting on anything, so the bound is never
// reached by a correct launch; it only guarantees that every wave exits.
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << lane_id()) - 1;  // lane 0 -> 0
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// Orders LDS traffic of one wavefront between iterations without a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Agent-scope atomic accesses for cross-workgroup publication (coherent across XCDs).
__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_agent(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ticket(uint32_t *ctr) {
    return __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void raise_err(uint32_t *err, uint32_t bit) {
    __hip_atomic_fetch_or(err, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- 32-bit per-digit look-back words: 0 = not yet published; otherwise bit 31 marks an
// inclusive prefix (else a tile aggregate) and bits [30:0] hold the count plus one, so counts up
// to 2^31 - 2 fit.
constexpr uint32_t kLb32Inc = 1u << 31;
__device__ __forceinline__ uint32_t lb32_word(bool inclusive, uint32_t count) {
    return (inclusive ? kLb32Inc : 0u) | (count + 1u);
}

// Exclusive prefix of this tile's count for one digit, summed over all earlier tiles.  The
// flags of tile p for digit d live at flags[p * stride + d].  The words of kLbWin earlier tiles
// are requested together, so one walk step costs one memory latency, not kLbWin of them.
constexpr int kLbWin = 4;
__device__ __forceinline__ uint32_t lookback_digit(const uint32_t *flags, int tile, uint32_t stride,
                                                   uint32_t d, uint32_t *err) {
    uint32_t excl = 0, spins = 0;
    for (int p = tile - 1; p >= 0; p -= kLbWin) {
        uint32_t v[kLbWin];
#pragma unroll
        for (int i = 0; i < kLbWin; ++i)  // tile -1 and before: an inclusive zero, never reached
            v[i] = p - i >= 0 ? ld_agent(flags + size_t(p - i) * stride + d) : (kLb32Inc | 1u);
#pragma unroll
        for (int i = 0; i < kLbWin; ++i) {
            while (v[i] == 0) {  // tile p - i has not published yet
                if (++spins > kSpinLimit) { raise_err(err, kErrSpin); v[i] = kLb32Inc | 1u; break; }
                __builtin_amdgcn_s_sleep(1);
                v[i] = ld_agent(flags + size_t(p - i) * stride + d);
            }
            excl += (v[i] & ~kLb32Inc) - 1u;
            if (v[i] & kLb32Inc) return excl;
        }
    }
    return excl;
}

// ---- 64-bit tile look-back words: [63:62] status, [61:0] payload --------------------------
constexpr uint64_t kLb64Agg = uint64_t(1) << 62;
constexpr uint64_t kLb64Inc = uint64_t(2) << 62;
constexpr uint64_t kLb64Val = (uint64_t(1) << 62) - 1;

// Payload combine operators for the 64-bit look-back.
struct SumOp {  // plain sum
    __device__ static uint64_t combine(uint64_t earlier, uint64_t later) { return earlier + later; }
};
// (count, last) pair: count in bits [61:31] (sum), last in bits [30:0] (max; 0 = none).
struct CountLastOp {
    static constexpr uint64_t kLastMask = (uint64_t(1) << 31) - 1;
    __device__ static uint64_t combine(uint64_t earlier, uint64_t later) {
        uint64_t c = (earlier >> 31) + (later >> 31);
        uint64_t l = (later & kLastMask) ? (later & kLastMask) : (earlier & kLastMask);
        return (c << 31) | l;
    }
};

// Wave-parallel look-back run by ONE wavefront of the tile (all 64 lanes active).  Publishes
// `agg` as this tile's aggregate, gathers the exclusive prefix from earlier tiles, publishes
// the inclusive value and returns the exclusive prefix (identity 0 for the first tile).
template <class Op>
__device__ uint64_t lookback_tile(uint64_t *flags, int tile, uint64_t agg, uint32_t *err) {
    const uint32_t lane = lane_id();
    if (tile == 0) {
        if (lane == 0) st_agent(flags, kLb64Inc | agg);
        return 0;
    }
    if (lane == 0) st_agent(flags + tile, kLb64Agg | agg);
    uint64_t excl = 0;
    bool have = false;
    int win = tile - 1;  // lane l inspects tile win - l
    uint32_t spins = 0;
    while (true) {
        int p = win - int(lane);
        uint64_t v = (p >= 0) ? ld_agent(flags + p) : kLb64Inc;  // virtual tile -1: inclusive 0
        uint64_t ready = ballot((v >> 62) != 0);
        uint64_t inc = ballot((v >> 62) == 2);
        int first_inc = inc ? __ffsll((long long)inc) - 1 : 64;
        uint64_t need = (first_inc >= 63) ? ~uint64_t(0) : ((uint64_t(2) << first_inc) - 1);
        if ((ready & need) != need) {
            if (++spins > kSpinLimit) { if (lane == 0) raise_err(err, kErrSpin); return excl; }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        // Combine lanes 0..first_inc (or all 64): the payload of lane l is later in text order
        // than that of lane l+1.  Lanes past first_inc contribute the identity (0 for both
        // operators), so a tree over all 64 lanes leaves the ordered combination in lane 0.
        uint64_t x = (int(lane) <= first_inc) ? (v & kLb64Val) : 0;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint64_t y = __shfl_down(x, o);  // lanes l+o.. : earlier tiles
            x = (int(lane) + o < kWave) ? Op::combine(y, x) : x;
        }
        const uint64_t acc = __shfl(x, 0);
        excl = have ? Op::combine(acc, excl) : acc;
        have = true;
        if (first_inc < 64) break;
        win -= 64;
    }
    if (lane == 0) st_agent(flags + tile, kLb64Inc | Op::combine(excl, agg));
    return excl;
}

// ---- workgroup scans -----------------------------------------------------------------------
// Inclusive wave scan with a generic operator (Op::combine(earlier, later)).
template <class Op, class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o);
        if (lane >= uint32_t(o)) x = Op::combine(y, x);
    }
    return x;
}

struct Sum32 {
    __device__ static uint32_t combine(uint32_t a, uint32_t b) { return a + b; }
};

// Exclusive workgroup scan of one uint32 per thread; writes the total to *total.
// `lds` must hold BLOCK/64 words.  Contains two __syncthreads().
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *lds, uint32_t *total) {
    constexpr int W = BLOCK / kWave;
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave;
    uint32_t inc = wave_incl_scan<Sum32>(v);
    if (lane == kWave - 1) lds[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint32_t t = lds[w];
        if (uint32_t(w) < wave) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

}  // namespace saasm
