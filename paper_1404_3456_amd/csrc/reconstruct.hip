// reconstruct.hip -- "cut and continue" reconstruction of a sequence from the fragments of two
// shotgun cuttings, searched through the suffix array (host code over the device-built index).
//
// Sec. III: a sequence is cut twice at different positions and the fragments of both cuttings
// are mixed.  A fragment is 'fir' when it is a prefix of another fragment (or another is a
// prefix of it): such a pair holds the first fragment of each cutting.  Cutting the shorter from
// the longer leaves a remainder, which must in turn be a prefix of the next fragment of the
// cutting that is behind (or that fragment a prefix of the remainder); repeating this rebuilds
// the sequence, and a dead end -- no candidate, or fragments left over -- sends the search back
// to its last choice (the paper's back-tracking).  Sec. IV replaces the prefix tests by searches
// in the suffix array of all fragments: the fragments that start with the remainder, or that are
// prefixes of it, are the fragment starts whose suffixes share enough with the remainder's
// suffix, found by walking the array outward from the remainder's rank under the running LCP
// minimum.
//
// State of the search: RS (the sequence so far) and the two cuttings' covered lengths; the
// cutting that is behind (shorter cover) takes the next fragment.  Candidates are tried in
// increasing fragment id; the first complete reconstruction is returned.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace saasm {
namespace {

// Runs f(lo, hi, chunk) over [0, n) split into contiguous chunks, one host thread each (at
// most 16); chunk c covers the c-th part, so per-chunk results concatenate in index order.
// A chunk whose thread cannot be started runs on the calling thread.  Returns false when a
// chunk failed (an allocation inside it threw); nothing escapes a thread.
template <class F>
bool parallel_chunks(int64_t n, F f) {
    unsigned t = std::thread::hardware_concurrency();
    if (t < 1) t = 1;
    if (t > 16) t = 16;
    if (n < 65536) t = 1;
    std::atomic<bool> failed{false};
    auto run = [&](int64_t lo, int64_t hi, int c) {
        try {
            f(lo, hi, c);
        } catch (...) {
            failed.store(true);
        }
    };
    std::vector<std::thread> pool;
    try {
        pool.reserve(t);
    } catch (...) {
        t = 1;
    }
    for (unsigned c = 1; c < t; ++c) {
        try {
            pool.emplace_back(run, n * c / t, n * (c + 1) / t, int(c));
        } catch (...) {
            run(n * c / t, n * (c + 1) / t, int(c));
        }
    }
    run(int64_t(0), n / t, 0);
    for (auto &th : pool) th.join();
    return !failed.load();
}

struct Recon {
    const uint8_t *t;
    int64_t n;
    const int32_t *sa, *isa, *lcp;
    std::vector<int64_t> start, len;  // per fragment
    std::vector<int32_t> frag_at;     // fragment id whose first base is position p, else -1
    std::vector<char> used;
    int64_t min_len = 0;

    // Fragments f (unused) whose text agrees with the suffix at q for min(|f|, rlen) bases,
    // |f| != rlen unless `final_ok`; in increasing id.
    void candidates(int64_t q, int64_t rlen, bool final_ok, std::vector<int32_t> &out) const {
        out.clear();
        const int64_t i = isa[q];
        auto consider = [&](int64_t k, int64_t run) {
            const int32_t f = frag_at[sa[k]];
            if (f < 0 || used[f]) return;
            const int64_t lf = len[f];
            if (lf == rlen && !final_ok) return;
            if (run >= std::min(lf, rlen)) out.push_back(f);
        };
        consider(i, rlen);  // the remainder's own suffix (never an unused fragment start here)
        const int64_t floor = std::max<int64_t>(1, std::min(min_len, rlen));
        int64_t run = INT64_MAX;
        for (int64_t k = i - 1; k >= 0; --k) {
            run = std::min<int64_t>(run, lcp[k + 1]);
            if (run < floor) break;
            consider(k, run);
        }
        run = INT64_MAX;
        for (int64_t k = i + 1; k < n; ++k) {
            run = std::min<int64_t>(run, lcp[k]);
            if (run < floor) break;
            consider(k, run);
        }
        std::sort(out.begin(), out.end());
    }
};

struct State {
    int64_t rs_len = 0, e_lo = 0, e_hi = 0;
    int32_t hi_frag = -1;  // the fragment that ends at e_hi
    size_t placed = 0;     // fragments in the placement order
};

struct Frame {
    State saved;  // state before this frame's choice
    std::vector<int32_t> cand;
    size_t next = 0;
};

}  // namespace
}  // namespace saasm

using namespace saasm;

static int reconstruct_impl(const uint8_t *text_h, int64_t n, const int32_t *sa_h,
                            const int32_t *isa_h, const int32_t *lcp_h, int32_t *order_h,
                            uint8_t *rs_h, int64_t rs_cap, int64_t *rs_len_h, int64_t max_steps) {
    if (!text_h || !sa_h || !isa_h || !lcp_h || !order_h || !rs_len_h)
        return fail(SA_ERR_INVALID, "sa_reconstruct: NULL pointer");
    if (n < 1 || text_h[n - 1] != '$') return fail(SA_ERR_INVALID, "sa_reconstruct: text must end with '$'");
    if (n >= kMaxN) return fail(SA_ERR_TOO_LARGE, "sa_reconstruct: n >= 2^31-2");
    Recon R;
    R.t = text_h;
    R.n = n;
    R.sa = sa_h;
    R.isa = isa_h;
    R.lcp = lcp_h;
    R.frag_at.resize(size_t(n));
    if (!parallel_chunks(n, [&](int64_t lo, int64_t hi, int) {
            std::fill(R.frag_at.begin() + lo, R.frag_at.begin() + hi, -1);
        }))
        return fail(SA_ERR_NOMEM, "sa_reconstruct: host thread failed");
    for (int64_t s0 = 0; s0 < n;) {  // fragment by fragment: the next separator after s0
        const void *q = memchr(text_h + s0, '$', size_t(n - s0));
        const int64_t p = static_cast<const uint8_t *>(q) - text_h;  // text_h[n-1] is '$'
        if (p == s0) return fail(SA_ERR_INVALID, "sa_reconstruct: empty fragment");
        R.frag_at[size_t(s0)] = int32_t(R.start.size());
        R.start.push_back(s0);
        R.len.push_back(p - s0);
        s0 = p + 1;
    }
    const int64_t m = int64_t(R.start.size());
    if (m < 2) return fail(SA_ERR_INVALID, "sa_reconstruct: need at least two fragments");
    R.min_len = *std::min_element(R.len.begin(), R.len.end());
    R.used.assign(size_t(m), 0);
    std::atomic<bool> bad{false};
    if (!parallel_chunks(n, [&](int64_t lo, int64_t hi, int) {
            for (int64_t i = lo; i < hi; ++i)
                if (sa_h[i] < 0 || sa_h[i] >= n || isa_h[sa_h[i]] != i) {
                    bad.store(true, std::memory_order_relaxed);
                    return;
                }
        }))
        return fail(SA_ERR_NOMEM, "sa_reconstruct: host thread failed");
    if (bad.load()) return fail(SA_ERR_INVALID, "sa_reconstruct: sa/isa are not inverse permutations");

    std::vector<uint8_t> rs;      // the sequence so far
    std::vector<int32_t> order;   // fragments in placement order
    State st;
    std::vector<Frame> stack;
    int64_t steps = 0;
    auto restore = [&](const State &x) {
        for (size_t i = x.placed; i < order.size(); ++i) R.used[size_t(order[i])] = 0;
        order.resize(x.placed);
        rs.resize(size_t(x.rs_len));
        st = x;
    };
    auto done = [&]() { return int64_t(st.placed) == m && st.e_lo == st.e_hi; };
    auto finish = [&]() -> int {
        if (rs_h && int64_t(rs.size()) > rs_cap)
            return fail(SA_ERR_CAPACITY, "sa_reconstruct: rs buffer too small");
        if (rs_h) memcpy(rs_h, rs.data(), rs.size());
        *rs_len_h = int64_t(rs.size());
        memcpy(order_h, order.data(), sizeof(int32_t) * size_t(m));
        return SA_OK;
    };
    // candidates for the current state: the remainder RS[e_lo, e_hi) is the suffix of hi_frag
    // of length e_hi - e_lo; an empty remainder before the end is a dead end
    auto push_frame = [&]() {
        Frame F;
        F.saved = st;
        if (st.e_lo < st.e_hi) {
            const int64_t rlen = st.e_hi - st.e_lo;
            const int64_t q = R.start[size_t(st.hi_frag)] + R.len[size_t(st.hi_frag)] - rlen;
            R.candidates(q, rlen, int64_t(st.placed) == m - 1, F.cand);
        }
        stack.push_back(std::move(F));
    };

    // First choice: every 'fir' pair (a a proper prefix of b; with two fragments also an equal
    // pair), by b then a in increasing id.
    std::vector<std::pair<int32_t, int32_t>> firs;
    {
        // independent read-only walks, one chunk of fragments per host thread
        std::vector<std::vector<std::pair<int32_t, int32_t>>> part(16);
        const bool ok = parallel_chunks(m, [&](int64_t lo, int64_t hi, int chunk) {
            std::vector<int32_t> c;
            for (int64_t bb = lo; bb < hi; ++bb) {
                const int32_t b = int32_t(bb);
                R.candidates(R.start[size_t(b)], R.len[size_t(b)], m == 2, c);
                for (int32_t a : c)
                    if (a != b && (R.len[size_t(a)] < R.len[size_t(b)] || m == 2))
                        part[size_t(chunk)].push_back({b, a});
            }
        });
        if (!ok) return fail(SA_ERR_NOMEM, "sa_reconstruct: out of host memory");
        for (auto &pv : part) firs.insert(firs.end(), pv.begin(), pv.end());
    }
    for (const auto &fa : firs) {
        const int32_t b = fa.first, a = fa.second;
        std::fill(R.used.begin(), R.used.end(), 0);
        order.assign({a, b});
        R.used[size_t(a)] = R.used[size_t(b)] = 1;
        rs.assign(text_h + R.start[size_t(b)], text_h + R.start[size_t(b)] + R.len[size_t(b)]);
        st.rs_len = R.len[size_t(b)];
        st.e_lo = R.len[size_t(a)];
        st.e_hi = R.len[size_t(b)];
        st.hi_frag = b;
        st.placed = 2;
        if (done()) return finish();
        stack.clear();
        push_frame();
        while (!stack.empty()) {
            if (++steps > max_steps) return fail(SA_ERR_NOTFOUND, "sa_reconstruct: step limit reached");
            Frame &F = stack.back();
            restore(F.saved);  // undo whatever the last choice under this frame placed
            if (F.next >= F.cand.size()) {  // exhausted: back-track to the parent's next choice
                stack.pop_back();
                continue;
            }
            const int32_t f = F.cand[F.next++];
            const int64_t rlen = st.e_hi - st.e_lo, lf = R.len[size_t(f)];
            R.used[size_t(f)] = 1;
            order.push_back(f);
            st.placed = order.size();
            if (lf > rlen) {  // f reaches past the other cutting and becomes the one ahead
                rs.insert(rs.end(), text_h + R.start[size_t(f)] + rlen, text_h + R.start[size_t(f)] + lf);
                st.rs_len = int64_t(rs.size());
                const int64_t lo = st.e_lo;
                st.e_lo = st.e_hi;
                st.e_hi = lo + lf;
                st.hi_frag = f;
            } else {          // f ends inside the remainder (or with it, at the very end)
                st.e_lo += lf;
            }
            if (done()) return finish();
            push_frame();
        }
    }
    return fail(SA_ERR_NOTFOUND, "sa_reconstruct: no reconstruction from two cuttings");
}

extern "C" int sa_reconstruct(const uint8_t *text_h, int64_t n, const int32_t *sa_h,
                              const int32_t *isa_h, const int32_t *lcp_h, int32_t *order_h,
                              uint8_t *rs_h, int64_t rs_cap, int64_t *rs_len_h,
                              int64_t max_steps) {
    try {  // host allocations may throw; nothing crosses the C interface
        return reconstruct_impl(text_h, n, sa_h, isa_h, lcp_h, order_h, rs_h, rs_cap, rs_len_h,
                                max_steps);
    } catch (...) {
        return fail(SA_ERR_NOMEM, "sa_reconstruct: out of host memory");
    }
}
