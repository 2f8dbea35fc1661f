// api.hip -- error reporting, version, tuning resolution and per-kernel event timing.
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace saasm {

static thread_local std::string t_last_error;

void set_error(const std::string &msg) { t_last_error = msg; }

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

int resolve_tuning(const sa_tuning *tu, Tune *out) {
    Tune t;
    if (tu) {
        if (tu->digit_bits) t.dbits = tu->digit_bits;
        if (tu->block_threads) t.block = tu->block_threads;
        if (tu->items_per_thread) t.items = tu->items_per_thread;
        if (tu->seg_pack != 0) return fail(SA_ERR_INVALID, "seg_pack must be 0 for this call");
        if (!tu->block_threads && t.dbits > 9) t.block = 512;  // the widest tile needs <= 9 bits
    }
    if (t.dbits != 4 && t.dbits != 8 && t.dbits != 9 && t.dbits != 11)
        return fail(SA_ERR_INVALID, "digit_bits must be 4, 8, 9 or 11");
    if (t.block != 256 && t.block != 512 && t.block != 1024)
        return fail(SA_ERR_INVALID, "block_threads must be 256, 512 or 1024");
    if (t.items != 8 && t.items != 16) return fail(SA_ERR_INVALID, "items_per_thread must be 8 or 16");
    if (t.block == 1024 && (t.items != 16 || t.dbits > 9))
        return fail(SA_ERR_INVALID, "block_threads 1024 needs items_per_thread 16 and digit_bits <= 9");
    *out = t;
    return SA_OK;
}

// ---- timing ---------------------------------------------------------------------------------
namespace {
struct Acc {
    int64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
    double items = 0.0;
};
struct Pending {
    hipEvent_t a, b;
    std::string key;
    double bytes;
    double per_item;
    int64_t tag;  // -1: bytes final; else waiting for timing_round_items
    int mode;     // kModeAny, or the round sort mode these bytes belong to
    double items; // units of work the launch processed
};
std::atomic<int64_t> g_next_tag{1};
thread_local int64_t t_tag = -1;
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, Acc> g_acc;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

static thread_local bool t_pause = false;
static thread_local int t_mode = kModeAny;

void timing_scope_mode(int mode) { t_mode = mode; }

bool timing_on() { return g_on && !t_pause; }

void timing_pause(bool on) { t_pause = on; }

TimedScope::TimedScope(const char *k, double b, hipStream_t s, double n_items)
    : key(k), bytes(b), items(n_items), stream(s) {
    if (!g_on || t_pause) return;
    std::lock_guard<std::mutex> lk(g_mu);
    start = get_event();
    if (start && hipEventRecord(start, stream) != hipSuccess) {
        g_pool.push_back(start);
        start = nullptr;
    }
}

TimedScope::TimedScope(const char *k, double fixed_bytes, double per_item_bytes, hipStream_t s)
    : TimedScope(k, fixed_bytes, s) {
    per_item = per_item_bytes;
    tag = t_tag;
    mode = t_mode;
}

void TimedScope::finish() {
    if (!start) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t end = get_event();
    if (!end || hipEventRecord(end, stream) != hipSuccess) {
        g_pool.push_back(start);
        if (end) g_pool.push_back(end);
        start = nullptr;
        return;
    }
    g_pending.push_back(Pending{start, end, key, bytes, per_item, tag, mode, items});
    start = nullptr;
}

int64_t timing_round_begin() {
    t_tag = g_next_tag++;
    return t_tag;
}

void timing_round_items(int64_t tag, int64_t items, int64_t big_items) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &p : g_pending) {
        if (p.tag != tag) continue;
        // an empty round still launched its kernels (they exit at once): timed, no bytes; so
        // are the radix-pass kernels of a round without large groups
        const int64_t k = p.mode == kModeRadix ? big_items : items;
        p.bytes = k <= 0 ? 0.0 : p.bytes + p.per_item * double(k);
        p.items = k <= 0 ? 0.0 : double(k);
        p.tag = -1;
    }
}

// Resolves pending launch timings; when `block` is false only those whose end event has
// already completed (so it never waits on device work).
static void timing_resolve(bool block) {
    std::lock_guard<std::mutex> lk(g_mu);
    size_t keep = 0;
    for (size_t i = 0; i < g_pending.size(); ++i) {
        Pending &p = g_pending[i];
        if (p.tag >= 0 && !block) {  // item count not known yet
            g_pending[keep++] = p;
            continue;
        }
        if (!block && hipEventQuery(p.b) != hipSuccess) {
            g_pending[keep++] = p;
            continue;
        }
        // a launch whose round count never arrived belongs to a round the build did not need
        // (it found nothing active): timed, no bytes
        if (p.tag >= 0) p.bytes = p.items = 0.0;
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess &&
            hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            Acc &a = g_acc[p.key];
            a.launches += 1;
            a.ms += ms;
            a.bytes += p.bytes;
            a.items += p.items;
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.resize(keep);
}

void timing_flush() { timing_resolve(true); }
void timing_poll() { timing_resolve(false); }

}  // namespace saasm

using namespace saasm;

extern "C" const char *sa_version(void) { return "saasm 0.1 (gfx950)"; }

extern "C" const char *sa_last_error(void) { return t_last_error.c_str(); }

extern "C" int sa_timing_enable(int32_t on) {
    if (!on) timing_flush();
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return SA_OK;
}

extern "C" int sa_timing_reset(void) {
    timing_flush();
    std::lock_guard<std::mutex> lk(g_mu);
    g_acc.clear();
    return SA_OK;
}

static int sa_timing_get_impl(const char *key, int64_t *launches_h, double *total_ms_h,
                             double *bytes_h) {
    if (!key) return fail(SA_ERR_INVALID, "sa_timing_get: NULL key");
    timing_flush();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_acc.find(key);
    if (it == g_acc.end()) {
        if (launches_h) *launches_h = 0;
        if (total_ms_h) *total_ms_h = 0;
        if (bytes_h) *bytes_h = 0;
        return SA_ERR_NOTFOUND;
    }
    if (launches_h) *launches_h = it->second.launches;
    if (total_ms_h) *total_ms_h = it->second.ms;
    if (bytes_h) *bytes_h = it->second.bytes;
    return SA_OK;
}

static int sa_timing_items_impl(const char *key, double *items_h) {
    if (!key || !items_h) return fail(SA_ERR_INVALID, "sa_timing_items: NULL pointer");
    timing_flush();
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_acc.find(key);
    *items_h = it == g_acc.end() ? 0.0 : it->second.items;
    return it == g_acc.end() ? SA_ERR_NOTFOUND : SA_OK;
}

// ---- C entry points: bodies above, host exceptions turned into statuses ------------------
extern "C" int sa_timing_get(const char *key, int64_t *launches_h, double *total_ms_h,
                             double *bytes_h) {
    return guard<int>([&] { return sa_timing_get_impl(key, launches_h, total_ms_h, bytes_h); });
}

extern "C" int sa_timing_items(const char *key, double *items_h) {
    return guard<int>([&] { return sa_timing_items_impl(key, items_h); });
}
