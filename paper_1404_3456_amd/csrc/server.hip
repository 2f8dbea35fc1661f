// server.hip -- assembly-job server: continuous batching of suffix-array / LCP / overlap jobs
// under an HBM budget.
//
// The paper's setting is one fragment set per reconstruction (Sec. III); a service receives
// many such sets.  Jobs are submitted from any thread and queued.  Worker threads, each with its
// own HIP stream, repeatedly take the queued jobs that fit (FIFO with bounded look-ahead, so a
// large job at the head does not block small ones behind it for ever), lay their texts end to
// end inside the arena, and run them as one batch: sa_build_batched (its doubling rounds driven
// from the host one round ahead of the state it reads, so each batch costs no graph capture),
// sa_lcp and sa_overlaps over the concatenation.  Results are localised per
// job (positions, ranks and read ids relative to the job) and stay in the arena until the job
// is released.  With several workers, a batch admitted while another is on the GPU runs
// concurrently with it on another stream.
//
// Plain mode (one job per batch, one worker, the single-text entry points) serves as the
// per-job baseline under the same harness.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace saasm {

// ---- arena: first-fit allocator over a caller-provided device buffer ------------------------
class Arena {
  public:
    void init(char *base, int64_t bytes) {
        base_ = base;
        free_.clear();
        free_[0] = bytes;
        used_ = 0;
        cap_ = bytes;
    }
    // Returns an offset or -1.  256-byte granularity.  Scratch that lives for one batch is
    // taken first-fit from the bottom (high = false); what outlives the batch (results, overlap
    // rows) last-fit from the top, so blocks held until the client releases them do not split
    // the free space the next batch's scratch needs.
    int64_t alloc(int64_t bytes, bool high = false) {
        bytes = (bytes + 255) & ~int64_t(255);
        if (fail_after_ > 0 && --fail_after_ == 0) return -1;  // injected failure (tests)
        if (high) {
            for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
                if (it->second >= bytes) {
                    const int64_t start = it->first, off = start + it->second - bytes;
                    it->second -= bytes;
                    if (it->second == 0) free_.erase(start);
                    sizes_[off] = bytes;
                    used_ += bytes;
                    return off;
                }
            }
            return -1;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                int64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                sizes_[off] = bytes;
                used_ += bytes;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off) {
        auto sz = sizes_.find(off);
        if (sz == sizes_.end()) return;
        int64_t len = sz->second;
        sizes_.erase(sz);
        used_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return;
            }
        }
        free_[off] = len;
    }
    char *ptr(int64_t off) const { return base_ + off; }
    int64_t used() const { return used_; }
    int64_t capacity() const { return cap_; }
    void fail_after(int k) { fail_after_ = k; }

  private:
    char *base_ = nullptr;
    std::map<int64_t, int64_t> free_;   // offset -> length
    std::map<int64_t, int64_t> sizes_;  // live allocation offset -> length
    int64_t used_ = 0, cap_ = 0;
    int fail_after_ = 0;
};

struct Batch;

struct Job {
    uint64_t id = 0;
    std::vector<uint8_t> text;       // owned copy (default)
    const uint8_t *borrowed = nullptr;  // caller's text (ASM_BORROW), valid until done
    bool checked = false;            // alphabet validated and reads counted
    const uint8_t *data() const { return borrowed ? borrowed : text.data(); }
    int32_t min_len = 1;
    int64_t n = 0, m = 0;
    int status = SA_PENDING;
    double t_submit = 0, t_admit = 0, t_done = 0;
    Batch *batch = nullptr;
    int64_t off = 0;       // first character in the batch text
    int64_t read_lo = 0;   // first read id in the batch
    int64_t row_lo = 0, row_hi = 0;
    bool released = false;
};

struct Batch {
    int64_t mem_off = -1;   // persistent part: text, sa, isa, lcp
    int64_t rows_off = -1;  // persistent overlap rows
    int refs = 0;
    int32_t *sa = nullptr, *isa = nullptr, *lcp = nullptr, *rows = nullptr;
};

}  // namespace saasm

struct asm_server {
    saasm::Arena arena;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<saasm::Job *> queue;
    std::unordered_map<uint64_t, saasm::Job *> jobs;
    std::vector<std::thread> workers;
    bool stop = false;
    int mode = 0;  // 0 continuous batching, 1 plain per job
    int max_jobs = 64;
    int64_t max_chars = int64_t(1) << 30;
    int lookahead = 16;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    uint64_t next_id = 1;
    int64_t batches = 0;
    int64_t jobs_done = 0;
    int concurrent_now = 0;
    int concurrent_max = 0;
};

namespace saasm {

static double now_s(asm_server *S) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - S->t0).count();
}

// bytes each job keeps until it is released (text, sa, isa, lcp)
static int64_t job_keep_bytes(int64_t n) { return 13 * n + 4 * 256; }

// scratch a batch needs while it runs (the build workspace dominates)
static int64_t batch_scratch_bytes(int64_t n, int n_jobs) {
    int64_t b = sa_build_batched_ws_bytes(n, n_jobs, nullptr, nullptr);
    int64_t l = sa_lcp_ws_bytes(n);
    return (b > l ? b : l) + 4096;
}

// Subtracts each job's first position from its block of sa and isa (both index the same
// block: a job's suffixes occupy exactly its own range of the batch order).
__global__ void k_localize(int32_t *__restrict__ sa, int32_t *__restrict__ isa,
                           const int64_t *__restrict__ job_off, int32_t n_jobs, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t lo = 0, hi = n_jobs;  // job_off[lo] <= i < job_off[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (job_off[mid] <= i) lo = mid;
        else hi = mid;
    }
    const int32_t base = int32_t(job_off[lo]);
    sa[i] -= base;
    isa[i] -= base;
}

// rows are sorted by read a; job j owns read ids [read_lo[j], read_lo[j+1]).  bounds[j] = first
// row of job j (lower bound of read_lo[j]), bounds[n_jobs] = nrows.
__global__ void k_row_bounds(const int32_t *__restrict__ rows, int64_t nrows,
                             const int64_t *__restrict__ read_lo, int32_t n_jobs,
                             int64_t *__restrict__ bounds) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > n_jobs) return;
    if (j == n_jobs) {
        bounds[j] = nrows;
        return;
    }
    int64_t lo = 0, hi = nrows;
    const int64_t key = read_lo[j];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (rows[3 * mid] < key) lo = mid + 1;
        else hi = mid;
    }
    bounds[j] = lo;
}

__global__ void k_rows_shift(int32_t *__restrict__ rows, int64_t nrows,
                             const int64_t *__restrict__ read_lo, int32_t n_jobs) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    const int64_t a = rows[3 * i];
    int32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (read_lo[mid] <= a) lo = mid;
        else hi = mid;
    }
    rows[3 * i] -= int32_t(read_lo[lo]);
    rows[3 * i + 1] -= int32_t(read_lo[lo]);
}

// One branch-free pass (vectorisable): count separators, flag any byte outside A,C,G,T,$.
static bool scan_text(const uint8_t *t, int64_t n, int64_t *m_out) {
    int64_t m = 0;
    uint32_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        const uint8_t c = t[i];
        const uint32_t sep = c == '$';
        const uint32_t base = (c == 'A') | (c == 'C') | (c == 'G') | (c == 'T');
        m += sep;
        bad |= (sep | base) ^ 1u;
    }
    *m_out = m;
    return bad == 0;
}

static int64_t arena_alloc(asm_server *S, int64_t bytes, bool high = false) {
    std::lock_guard<std::mutex> lk(S->mu);
    return S->arena.alloc(bytes, high);
}

// Runs one batch on stream s, without the server lock.  scratch: arena offsets to release
// when the batch ends (the first is the build workspace).
static int run_batch(asm_server *S, std::vector<Job *> &js, Batch *B, hipStream_t s,
                     std::vector<int64_t> &scratch) {
    const int nj = int(js.size());
    std::vector<int64_t> off(nj + 1, 0), rlo(nj + 1, 0);
    for (int j = 0; j < nj; ++j) {
        off[j + 1] = off[j] + js[j]->n;
        rlo[j + 1] = rlo[j] + js[j]->m;
    }
    const int64_t n = off[nj];
    char *mem = S->arena.ptr(B->mem_off);
    uint8_t *text = reinterpret_cast<uint8_t *>(mem);
    int64_t o = (n + 255) & ~int64_t(255);
    B->sa = reinterpret_cast<int32_t *>(mem + o);
    o += (4 * n + 255) & ~int64_t(255);
    B->isa = reinterpret_cast<int32_t *>(mem + o);
    o += (4 * n + 255) & ~int64_t(255);
    B->lcp = reinterpret_cast<int32_t *>(mem + o);
    for (int j = 0; j < nj; ++j)
        SA_HIP(hipMemcpyAsync(text + off[j], js[j]->data(), size_t(js[j]->n), hipMemcpyHostToDevice, s));
    int64_t scr_bytes = batch_scratch_bytes(n, nj);
    char *scr = S->arena.ptr(scratch[0]);
    int32_t rounds = 0;
    if (S->mode == 1 && nj == 1) {
        SA_TRY(sa_build(text, n, B->sa, B->isa, scr, scr_bytes, nullptr, &rounds, s));
        SA_TRY(sa_lcp(text, n, B->sa, B->isa, B->lcp, scr, scr_bytes, s));
    } else {
        SA_TRY(sa_build_batched(text, n, off.data(), nj, B->sa, B->isa, B->lcp, scr, scr_bytes,
                                nullptr, 0, &rounds, s));
    }
    // overlaps (one min_len per batch; admission keeps it uniform), into scratch rows first
    int64_t cap = n / 32 + 4096;
    int64_t n_out = 0, need = 0;
    int32_t *rows_tmp = nullptr;
    int rc = SA_ERR_HIP;
    for (int attempt = 0; attempt < 8; ++attempt) {
        const int64_t r_off = arena_alloc(S, cap * 12);
        if (r_off < 0) return fail(SA_ERR_NOMEM, "server: arena full (overlap rows)");
        scratch.push_back(r_off);
        rows_tmp = reinterpret_cast<int32_t *>(S->arena.ptr(r_off));
        rc = sa_overlaps(text, n, B->sa, B->isa, B->lcp, js[0]->min_len, rows_tmp, cap, &n_out,
                         scr, scr_bytes, &need, s);
        if (rc == SA_ERR_CAPACITY) {
            cap = n_out + 1024;
            continue;
        }
        if (rc == SA_ERR_NOMEM && need > scr_bytes) {
            const int64_t more = arena_alloc(S, need);
            if (more < 0) return fail(SA_ERR_NOMEM, "server: arena full (overlap workspace)");
            scratch.push_back(more);
            scr = S->arena.ptr(more);
            scr_bytes = need;
            continue;
        }
        break;
    }
    if (rc != SA_OK) return rc;
    B->rows_off = arena_alloc(S, (n_out > 0 ? n_out : 1) * 12, true);
    if (B->rows_off < 0) return fail(SA_ERR_NOMEM, "server: arena full (rows)");
    B->rows = reinterpret_cast<int32_t *>(S->arena.ptr(B->rows_off));
    if (n_out > 0)
        SA_HIP(hipMemcpyAsync(B->rows, rows_tmp, size_t(n_out) * 12, hipMemcpyDeviceToDevice, s));
    // job offsets, read offsets and row bounds in the (now free) build workspace
    int64_t *meta = reinterpret_cast<int64_t *>(scr);
    SA_HIP(hipMemcpyAsync(meta, off.data(), size_t(nj + 1) * 8, hipMemcpyHostToDevice, s));
    SA_HIP(hipMemcpyAsync(meta + (nj + 1), rlo.data(), size_t(nj + 1) * 8, hipMemcpyHostToDevice, s));
    int64_t *bounds = meta + 2 * (nj + 1);
    hipLaunchKernelGGL(k_localize, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, B->sa, B->isa,
                       meta, nj, n);
    SA_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_row_bounds, dim3(unsigned((nj + 1 + 255) / 256)), dim3(256), 0, s, B->rows,
                       n_out, meta + (nj + 1), nj, bounds);
    SA_HIP(hipGetLastError());
    if (n_out > 0) {
        hipLaunchKernelGGL(k_rows_shift, dim3(unsigned((n_out + 255) / 256)), dim3(256), 0, s, B->rows,
                           n_out, meta + (nj + 1), nj);
        SA_HIP(hipGetLastError());
    }
    std::vector<int64_t> hb(nj + 1, 0);
    SA_HIP(hipMemcpyAsync(hb.data(), bounds, size_t(nj + 1) * 8, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < nj; ++j) {
        js[j]->off = off[j];
        js[j]->read_lo = rlo[j];
        js[j]->row_lo = hb[j];
        js[j]->row_hi = hb[j + 1];
    }
    return SA_OK;
}

// A job that ends without running (no room for it even in an empty arena): its status, time
// and count are final and its host text is dropped.  Caller holds the lock.
static void finish_unrun_locked(asm_server *S, Job *j, int status) {
    j->status = status;
    j->t_done = now_s(S);
    j->batch = nullptr;
    std::vector<uint8_t>().swap(j->text);
    j->borrowed = nullptr;
    ++S->jobs_done;
}

static void worker_main(asm_server *S) {
    hipSetDevice(S->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    const int full_limit = S->mode == 1 ? 1 : S->max_jobs;
    int limit = full_limit;  // jobs this worker lays into its next batch
    while (true) {
        std::vector<Job *> js;
        Batch *B = nullptr;
        std::vector<int64_t> scratch;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->stop && S->queue.empty()) break;
            // admission: FIFO, one min_len per batch; at most `lookahead` queued jobs that do
            // not fit this batch (another min_len, or past the character limit) are passed over
            int64_t chars = 0;
            int skipped = 0;
            for (auto it = S->queue.begin(); it != S->queue.end() && skipped < S->lookahead;) {
                Job *j = *it;
                if (!js.empty() && (j->min_len != js[0]->min_len || chars + j->n > S->max_chars)) {
                    ++skipped;
                    ++it;
                    continue;
                }
                js.push_back(j);
                chars += j->n;
                it = S->queue.erase(it);
                if (int(js.size()) >= limit) break;
            }
            if (js.empty()) continue;
            int64_t keep = 0;
            for (Job *j : js) keep += job_keep_bytes(j->n);
            const int64_t mem = S->arena.alloc(keep, true);
            const int64_t scr = mem >= 0 ? S->arena.alloc(batch_scratch_bytes(chars, int(js.size()))) : -1;
            if (mem < 0 || scr < 0) {
                if (mem >= 0) S->arena.release(mem);
                // put back, keeping FIFO order
                for (auto r = js.rbegin(); r != js.rend(); ++r) S->queue.push_front(*r);
                if (js.size() > 1) {
                    // try again at once with half the jobs; the full batch size comes back with
                    // the next admission that fits
                    limit = int(js.size()) / 2;
                    continue;
                }
                if (S->arena.used() == 0 || (S->stop && S->concurrent_now == 0)) {
                    // one job that finds no room even in an empty arena (or, while the server
                    // shuts down, no room that any batch still running will free)
                    Job *j = S->queue.front();
                    S->queue.pop_front();
                    finish_unrun_locked(S, j, SA_ERR_NOMEM);
                    S->cv.notify_all();
                    continue;
                }
                // the memory is held by batches in flight or by finished jobs the caller has not
                // released yet: wait for a batch to end or a release (both notify)
                S->cv.wait_for(lk, std::chrono::milliseconds(5));
                continue;
            }
            limit = full_limit;
            B = new Batch;
            B->mem_off = mem;
            B->refs = int(js.size());
            scratch.push_back(scr);
            const double t = now_s(S);
            for (Job *j : js) {
                j->t_admit = t;
                j->batch = B;
            }
            ++S->concurrent_now;
            if (S->concurrent_now > S->concurrent_max) S->concurrent_max = S->concurrent_now;
        }
        // borrowed texts are validated here, off the submitting thread
        std::vector<Job *> rejected;
        for (size_t k = 0; k < js.size();) {
            Job *j = js[k];
            if (!j->checked) {
                int64_t m = 0;
                const bool ok = scan_text(j->data(), j->n, &m);
                j->m = m;
                j->checked = true;
                if (!ok) {
                    rejected.push_back(j);
                    js.erase(js.begin() + long(k));
                    continue;
                }
            }
            ++k;
        }
        int rc = js.empty() ? SA_OK : run_batch(S, js, B, s, scratch);
        // A batch that failed part-way may still have kernels in flight on this stream (sa_lcp
        // does not synchronise): they must finish before its arena regions go to anyone else.
        if (rc != SA_OK) (void)hipStreamSynchronize(s);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            --S->concurrent_now;
            ++S->batches;
            for (int64_t a : scratch) S->arena.release(a);
            const double t = now_s(S);
            for (Job *j : rejected) {
                j->status = SA_ERR_ALPHABET;
                j->t_done = t;
                j->batch = nullptr;
                --B->refs;
                ++S->jobs_done;
            }
            if (rc != SA_OK || js.empty()) {
                S->arena.release(B->mem_off);
                if (B->rows_off >= 0) S->arena.release(B->rows_off);
                delete B;
            }
            for (Job *j : js) {
                j->status = rc;
                j->t_done = t;
                if (rc != SA_OK) j->batch = nullptr;
                std::vector<uint8_t>().swap(j->text);
                j->borrowed = nullptr;
                ++S->jobs_done;
            }
        }
        S->cv.notify_all();
    }
    hipStreamDestroy(s);
}

static void release_job_locked(asm_server *S, Job *j) {
    Batch *B = j->batch;
    j->batch = nullptr;
    if (B && --B->refs == 0) {
        S->arena.release(B->mem_off);
        if (B->rows_off >= 0) S->arena.release(B->rows_off);
        delete B;
    }
}

}  // namespace saasm

using namespace saasm;

static int asm_server_create_impl(void *arena, int64_t arena_bytes, int32_t max_jobs_per_batch,
                                 int32_t workers, int32_t mode, asm_server **out) {
    if (!arena || !out || arena_bytes < (int64_t(1) << 20) || workers < 1 || workers > 16 ||
        max_jobs_per_batch < 1 || (mode != 0 && mode != 1))
        return fail(SA_ERR_INVALID, "asm_server_create: bad arguments");
    asm_server *S = new asm_server;
    S->arena.init(static_cast<char *>(arena), arena_bytes);
    S->mode = mode;
    S->max_jobs = mode == 1 ? 1 : max_jobs_per_batch;
    S->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&S->device) != hipSuccess) S->device = 0;
    const int nw = mode == 1 ? 1 : workers;
    for (int i = 0; i < nw; ++i) S->workers.emplace_back(worker_main, S);
    *out = S;
    return SA_OK;
}

static int asm_submit_impl(asm_server *S, const uint8_t *text_h, int64_t n, int32_t min_len,
                          int32_t flags, uint64_t *job_id_h) {
    if (!S || !text_h || !job_id_h) return fail(SA_ERR_INVALID, "asm_submit: NULL pointer");
    if (n < 1 || min_len < 1) return fail(SA_ERR_INVALID, "asm_submit: need n >= 1, min_len >= 1");
    if (flags & ~ASM_BORROW) return fail(SA_ERR_INVALID, "asm_submit: unknown flags");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "asm_submit: n >= 2^31-2");
    if (text_h[n - 1] != '$') return fail(SA_ERR_INVALID, "asm_submit: text must end with '$'");
    if (job_keep_bytes(n) + batch_scratch_bytes(n, 1) > S->arena.capacity())
        return fail(SA_ERR_NOMEM, "asm_submit: job larger than the server's memory budget");
    Job *j = new Job;
    if (flags & ASM_BORROW) {
        j->borrowed = text_h;  // validated by the worker that runs it
    } else {
        int64_t m = 0;
        if (!scan_text(text_h, n, &m)) {
            delete j;
            return fail(SA_ERR_ALPHABET, "asm_submit: text holds a byte other than A, C, G, T, $");
        }
        j->text.assign(text_h, text_h + n);
        j->m = m;
        j->checked = true;
    }
    j->n = n;
    j->min_len = min_len;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        j->id = S->next_id++;
        j->t_submit = now_s(S);
        S->jobs[j->id] = j;
        S->queue.push_back(j);
    }
    S->cv.notify_all();
    *job_id_h = j->id;
    return SA_OK;
}

static int asm_poll_impl(asm_server *S, uint64_t job_id, asm_result *res) {
    if (!S || !res) return fail(SA_ERR_INVALID, "asm_poll: NULL pointer");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(job_id);
    if (it == S->jobs.end()) return fail(SA_ERR_NOTFOUND, "asm_poll: unknown job");
    Job *j = it->second;
    res->status = j->status;
    res->n = j->n;
    res->m = j->m;
    res->t_submit = j->t_submit;
    res->t_admit = j->t_admit;
    res->t_done = j->t_done;
    res->sa = res->isa = res->lcp = res->ovl = nullptr;
    res->n_overlaps = 0;
    if (j->status == SA_OK && j->batch) {
        Batch *B = j->batch;
        res->sa = B->sa + j->off;
        res->isa = B->isa + j->off;
        res->lcp = B->lcp + j->off;
        res->ovl = B->rows + 3 * j->row_lo;
        res->n_overlaps = j->row_hi - j->row_lo;
    }
    return j->status == SA_PENDING ? SA_PENDING : SA_OK;
}

static int asm_release_impl(asm_server *S, uint64_t job_id) {
    if (!S) return fail(SA_ERR_INVALID, "asm_release: NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(job_id);
    if (it == S->jobs.end()) return fail(SA_ERR_NOTFOUND, "asm_release: unknown job");
    Job *j = it->second;
    if (j->status == SA_PENDING) return fail(SA_ERR_INVALID, "asm_release: job still running");
    release_job_locked(S, j);
    S->jobs.erase(it);
    delete j;
    S->cv.notify_all();
    return SA_OK;
}

static int asm_server_stats_impl(asm_server *S, int64_t *out_h /* [6] */) {
    if (!S || !out_h) return fail(SA_ERR_INVALID, "asm_server_stats: NULL pointer");
    std::lock_guard<std::mutex> lk(S->mu);
    out_h[0] = S->batches;
    out_h[1] = S->jobs_done;
    out_h[2] = S->concurrent_max;
    out_h[3] = S->arena.used();
    out_h[4] = S->arena.capacity();
    out_h[5] = int64_t(S->queue.size());
    return SA_OK;
}

static int asm_server_fail_alloc_after_impl(asm_server *S, int32_t k) {
    if (!S || k < 0) return fail(SA_ERR_INVALID, "asm_server_fail_alloc_after: bad arguments");
    std::lock_guard<std::mutex> lk(S->mu);
    S->arena.fail_after(k);
    return SA_OK;
}

static int asm_server_destroy_impl(asm_server *S) {
    if (!S) return fail(SA_ERR_INVALID, "asm_server_destroy: NULL server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto &t : S->workers) t.join();
    for (auto &kv : S->jobs) delete kv.second;
    delete S;
    return SA_OK;
}

// ---- C entry points: bodies above, host exceptions turned into statuses ------------------
extern "C" int asm_server_create(void *arena, int64_t arena_bytes, int32_t max_jobs_per_batch,
                                 int32_t workers, int32_t mode, asm_server **out) {
    return guard<int>([&] { return asm_server_create_impl(arena, arena_bytes, max_jobs_per_batch, workers, mode, out); });
}

extern "C" int asm_submit(asm_server *S, const uint8_t *text_h, int64_t n, int32_t min_len,
                          int32_t flags, uint64_t *job_id_h) {
    return guard<int>([&] { return asm_submit_impl(S, text_h, n, min_len, flags, job_id_h); });
}

extern "C" int asm_poll(asm_server *S, uint64_t job_id, asm_result *res) {
    return guard<int>([&] { return asm_poll_impl(S, job_id, res); });
}

extern "C" int asm_release(asm_server *S, uint64_t job_id) {
    return guard<int>([&] { return asm_release_impl(S, job_id); });
}

extern "C" int asm_server_stats(asm_server *S, int64_t *out_h /* [6] */) {
    return guard<int>([&] { return asm_server_stats_impl(S, out_h); });
}

extern "C" int asm_server_fail_alloc_after(asm_server *S, int32_t k) {
    return guard<int>([&] { return asm_server_fail_alloc_after_impl(S, k); });
}

extern "C" int asm_server_destroy(asm_server *S) {
    return guard<int>([&] { return asm_server_destroy_impl(S); });
}
