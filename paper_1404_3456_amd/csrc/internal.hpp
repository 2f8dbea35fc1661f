// internal.hpp -- host-side plumbing shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <string>

#include "../../include/saasm.h"

namespace saasm {

// ---- errors --------------------------------------------------------------------------------
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define SA_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::saasm::fail(SA_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Runs an entry point's body; a host exception (an allocation that fails, a thread that cannot
// start) becomes an error status instead of crossing the C interface.  The messages are short
// enough to need no allocation themselves.
template <class R, class F>
R guard(F &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        set_error("host alloc fail");
        return R(SA_ERR_NOMEM);
    } catch (...) {
        set_error("host failure");
        return R(SA_ERR_HIP);
    }
}

#define SA_TRY(expr)                 \
    do {                             \
        int r_ = (expr);             \
        if (r_ != SA_OK) return r_;  \
    } while (0)

constexpr int64_t kMaxN = (int64_t(1) << 31) - 2;  // n <= kMaxN - 1: labels fit in 31 bits
constexpr uint32_t kDone = 1u << 31;      // bit 31 flag: first member of a group (positions), singleton (rank update)
constexpr uint32_t kRankMask = kDone - 1;
constexpr int kH0 = 29;                   // bases in the first-round key (58 code bits + 5)

// ---- workspace carving -----------------------------------------------------------------------
struct Carver {
    char *base;
    int64_t off = 0;
    int64_t cap;
    Carver(void *p, int64_t c) : base(static_cast<char *>(p)), cap(c) {}
    template <class T>
    T *take(int64_t count) {
        off = (off + 255) & ~int64_t(255);
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += count * int64_t(sizeof(T));
        return p;
    }
    bool ok() const { return off <= cap; }
};

// ---- tuning --------------------------------------------------------------------------------
struct Tune {
    int dbits = 9;
    int block = 1024;  // 512 when digits are wider than 9 bits (resolve_tuning)
    int items = 16;
    int tile() const { return block * items; }
    int radix() const { return 1 << dbits; }
};
int resolve_tuning(const sa_tuning *t, Tune *out);

// ---- timing --------------------------------------------------------------------------------
bool timing_on();
struct TimedScope {
    // Records a start event on `stream` when timing is on; finish() records the end event and
    // files the launch under `key` with `bytes` algorithmic bytes.  The second form is for
    // launches whose item count is only known on the device: the record waits until
    // timing_round_items() gives the count for the calling thread's current round tag.
    // `items` counts the launch's units of work (suffixes, reads, pass items); the per-item
    // form takes it from its round's count.
    const char *key;
    double bytes;
    double per_item = 0.0;
    double items = 0.0;
    int64_t tag = -1;
    int mode = 0;
    hipStream_t stream;
    hipEvent_t start = nullptr;
    TimedScope(const char *k, double b, hipStream_t s, double n_items = 0.0);
    TimedScope(const char *k, double fixed_bytes, double per_item_bytes, hipStream_t s);
    void finish();
};
int64_t timing_round_begin();                       // new tag for the calling thread's round
// Units of work of that round: scopes opened in kModeRadix count the items of its large
// groups (sorted by radix passes), the others every active item (0: no bytes).
void timing_round_items(int64_t tag, int64_t items, int64_t big_items);
constexpr int kModeAny = 0, kModeRadix = 1, kModeRuns = 2;
// The unit count that scopes opened by the calling thread from now on take from their round
// (kModeRadix: the large groups' items; otherwise all active items).
void timing_scope_mode(int mode);
void timing_flush();  // resolve pending events (waits for them)
void timing_poll();   // resolve only the pending events that have already completed
void timing_pause(bool on);  // calling thread: no events while a stream is being captured

// ---- kernels exposed across translation units ----------------------------------------------
int64_t packed_words(int64_t n);
int64_t sepmask_words(int64_t n);

// pack: packed/sepmask/per-word separator counts; err bits OR-ed into *err.
int launch_pack(const uint8_t *text, int64_t n, uint32_t *packed, uint32_t *sepmask,
                uint32_t *wordcnt, uint32_t *err, hipStream_t s);
// block layout for random-access windows (text.hpp): nrec = sepmask_words(n) records
int launch_blocks(const uint32_t *packed, const uint32_t *sepmask, uint4 *blk, int64_t nrec,
                  hipStream_t s);
// exclusive scan of uint32 values into int32 (out[i] = sum of in[0..i)); total -> *total_out
int64_t scan_flags_words(int64_t n);
int launch_scan_u32_i32(const uint32_t *in, int32_t *out, int64_t n, int32_t *total_out,
                        uint64_t *lbflags, uint32_t *ticket, uint32_t *err, hipStream_t s);
int launch_scan_u32_i64(const uint32_t *in, int64_t *out, int64_t n, int64_t *total_out,
                        uint64_t *lbflags, uint32_t *ticket, uint32_t *err, hipStream_t s);
int launch_read_ends(const uint32_t *sepmask, const int32_t *sepcnt, int64_t n, int32_t *read_end,
                     hipStream_t s);
int launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
int launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);

// LCP array (Kasai's scan; lcp.hip): workspace bytes and the body of sa_lcp.  A failure found
// on the device is written to flag[0] (default: lcp[0]) as the negative status.  `span` bounds
// the range of suffix-array indices and text positions one text's accesses fall in (a batch of
// texts: its largest text; 0: n); it chooses between the two forms of the scan.
int64_t lcp_ws_bytes(int64_t n);
int lcp_run(const uint8_t *text, int64_t n, const int32_t *sa, const int32_t *isa, int32_t *lcp,
            void *ws, int64_t ws_bytes, hipStream_t stream, int32_t *flag = nullptr,
            int64_t span = 0);

// radix sort plumbing
struct SortBufs {
    uint64_t *keys[2];
    uint32_t *vals[2];
    uint32_t *hist;     // [kHistParts][passes][radix] per-workgroup partial counts
    uint32_t *gbase;    // [passes][radix] exclusive bases
    uint32_t *flags;    // [passes][tiles][radix] look-back words
    uint32_t *tickets;  // [passes]
    uint32_t *err;
};
int sort_passes(int bits, const Tune &t);
int64_t sort_flag_words(int64_t n, int bits, const Tune &t);
void carve_sort(Carver &c, int64_t n, int bits, const Tune &t, SortBufs *b, bool with_items);
// Clears histogram, flags and tickets for a sort of n items over `bits` bits.
int sort_prepare(const SortBufs &b, int64_t n, int bits, const Tune &t, hipStream_t s);
// Upper bound on the workgroups of a histogram-producing launch; each writes one partial
// histogram (no global atomics) that the per-pass scan kernel reduces.
constexpr int kHistParts = 1024;
// Histogram of keys[cur] for all passes (when the producer did not build it); the number of
// partial histograms written goes to *nparts.
int launch_hist(const SortBufs &b, int cur, int64_t n, int bit_lo, int bits, const Tune &t,
                hipStream_t s, int *nparts);
// Runs the passes over n items (or, when count_dev is given, over the count read from device
// memory, at most n); returns the buffer index holding the sorted data in *cur_out.
int sort_run(const SortBufs &b, int cur, const uint32_t *count_dev, int64_t n, int bit_lo,
             int bits, const Tune &t, int nparts, hipStream_t s, int *cur_out);

// Device-side round state of a suffix-array build (words of a uint32 array).
constexpr int kStErr = 0;      // error bits
constexpr int kStActive = 1;   // suffixes in non-singleton groups entering the next round
constexpr int kStKeys = 2;     // keys written by the round's key build (== kStActive)
constexpr int kStH = 3;        // prefix length the groups are sorted by
constexpr int kStRounds = 4;   // rounds completed
constexpr int kStNext = 5;     // active count produced by the round's rank update
constexpr int kStBig = 6;      // 1: some group entering the round has more than kRunMax members
constexpr int kStRadixN = 7;   // items of large groups the round sorts by radix passes
constexpr int kStBigNext = 8;  // set by the rank update for the next round
constexpr int kStBigLast = 9;  // kStRadixN of the round that ended (read back for timing)
constexpr int kStWords = 16;   // state words the host reads back
constexpr int kRunMax = 32;    // largest group the run sort handles

// key builders (fused with the histogram of the sort that follows)
int launch_key0(const uint32_t *packed, const uint32_t *sepmask, int64_t n, int h0,
                const int64_t *set_off_dev, int n_sets, int key_bits, const SortBufs &b, int cur,
                const Tune &t, hipStream_t s, int *nparts);
// Keys of the items in groups of more than kRunMax members (sa_build.hip's doubling rounds),
// into b.keys[0]/b.vals[0] with their list indices in bigidx, fused with the histograms.
int launch_big_extract(const uint32_t *P, const uint32_t *S, const uint32_t *rank, int64_t n,
                       int rbits, int64_t a_bound, const SortBufs &b, uint32_t *bigidx,
                       uint64_t *lbflags, int64_t lb_words, uint32_t *tick, uint32_t *state,
                       const Tune &t, hipStream_t s, int *nparts);
// The sorted large items to their indices in the round's full key/value list.
int launch_big_place(const uint64_t *ks, const uint32_t *vs, const uint32_t *bigidx,
                     int64_t a_bound, const uint32_t *state, uint64_t *K, uint32_t *V,
                     uint32_t *err, hipStream_t s);

}  // namespace saasm
