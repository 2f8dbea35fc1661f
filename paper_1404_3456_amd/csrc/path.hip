// path.hip -- the reconstruction read off the weighted overlap graph (Sec. III).
//
// The paper draws the fragments as the vertices of a weighted directed graph (its Fig. 3): an
// edge a -> b carries the overlap length l(a, b), and the superstring comes from a Hamiltonian
// path of maximal total weight, merging each next fragment past its overlap with the one
// before.  The edge weights are the rows sa_overlaps produces on the GPU; what is left is a
// search over a graph with one vertex per fragment, which runs on the host.
//
// Exact search (up to kExactMax fragments): dynamic programming over subsets -- best[S][v] is
// the largest weight of a path through exactly the fragments of S that ends at v, extended one
// fragment at a time -- in 2^m * m^2 steps.  Larger sets take the greedy rule: edges by weight
// (heaviest first, then by a, then by b), an edge kept when a has no successor yet, b no
// predecessor and the two are not already in one chain, and the chains that remain laid end to
// end in order of their first fragment.  Finding a maximal Hamiltonian path is NP-hard, which
// is why the paper turns to the suffix-array based "cut and continue" search for large inputs
// (sa_reconstruct); this call covers the graph formulation it starts from.
#include <algorithm>
#include <array>
#include <cstring>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace saasm {

constexpr int kExactMax = 20;

struct Frag {
    int64_t start, len;
};

static int read_frags(const uint8_t *t, int64_t n, std::vector<Frag> *out) {
    out->clear();
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (t[i] == '$') {
            out->push_back(Frag{s, i - s});
            s = i + 1;
        }
    }
    return SA_OK;
}

static inline uint64_t edge_key(int64_t a, int64_t b) { return (uint64_t(a) << 32) | uint64_t(b); }

// Order of the fragments along a Hamiltonian path of maximal total weight (exact).  Ties: the
// first extension found wins (subsets in increasing order, end fragments and extensions in
// increasing id), and the path that ends at the smallest id among the best.
static void exact_path(int m, const std::vector<int64_t> &W, std::vector<int32_t> *order) {
    const size_t full = (size_t(1) << m) - 1;
    std::vector<int64_t> best((full + 1) * size_t(m), -1);
    std::vector<int8_t> from((full + 1) * size_t(m), -1);
    for (int v = 0; v < m; ++v) best[(size_t(1) << v) * m + v] = 0;
    for (size_t S = 1; S <= full; ++S) {
        for (int v = 0; v < m; ++v) {
            const int64_t bv = best[S * m + v];
            if (bv < 0) continue;
            for (int u = 0; u < m; ++u) {
                if (S & (size_t(1) << u)) continue;
                const size_t T = S | (size_t(1) << u);
                const int64_t c = bv + W[size_t(v) * m + u];
                if (c > best[T * m + u]) {
                    best[T * m + u] = c;
                    from[T * m + u] = int8_t(v);
                }
            }
        }
    }
    int end = 0;
    for (int v = 1; v < m; ++v)
        if (best[full * m + v] > best[full * m + end]) end = v;
    order->assign(size_t(m), 0);
    size_t S = full;
    int v = end;
    for (int k = m - 1; k >= 0; --k) {
        (*order)[size_t(k)] = v;
        const int p = from[S * m + v];
        S &= ~(size_t(1) << v);
        v = p;
    }
}

static void greedy_path(int64_t m, std::vector<std::array<int32_t, 3>> &edges,
                        std::vector<int32_t> *order) {
    std::sort(edges.begin(), edges.end(), [](const std::array<int32_t, 3> &x,
                                             const std::array<int32_t, 3> &y) {
        if (x[2] != y[2]) return x[2] > y[2];
        if (x[0] != y[0]) return x[0] < y[0];
        return x[1] < y[1];
    });
    std::vector<int32_t> succ(static_cast<size_t>(m), -1), pred(static_cast<size_t>(m), -1);
    std::vector<int32_t> up(static_cast<size_t>(m), 0);
    std::iota(up.begin(), up.end(), 0);
    auto root = [&](int32_t x) {  // chains as disjoint sets (path halving)
        while (up[size_t(x)] != x) {
            up[size_t(x)] = up[size_t(up[size_t(x)])];
            x = up[size_t(x)];
        }
        return x;
    };
    for (const auto &e : edges) {
        const int32_t a = e[0], b = e[1];
        if (succ[size_t(a)] >= 0 || pred[size_t(b)] >= 0) continue;
        const int32_t ra = root(a), rb = root(b);
        if (ra == rb) continue;
        succ[size_t(a)] = b;
        pred[size_t(b)] = a;
        up[size_t(rb)] = ra;
    }
    order->clear();
    for (int64_t h = 0; h < m; ++h) {
        if (pred[size_t(h)] >= 0) continue;
        for (int32_t x = int32_t(h); x >= 0; x = succ[size_t(x)]) order->push_back(x);
    }
}

static int overlap_path_impl(const uint8_t *text_h, int64_t n, const int32_t *rows_h, int64_t r,
                             int32_t exact_max_m, int32_t *order_h, int64_t *weight_h,
                             uint8_t *rs_h, int64_t rs_cap, int64_t *rs_len_h) {
    if (!text_h || !order_h || !weight_h || !rs_len_h || (r > 0 && !rows_h) || (rs_cap > 0 && !rs_h))
        return fail(SA_ERR_INVALID, "sa_overlap_path: NULL pointer");
    if (n < 1 || text_h[n - 1] != '$') return fail(SA_ERR_INVALID, "sa_overlap_path: text must end with '$'");
    if (r < 0) return fail(SA_ERR_INVALID, "sa_overlap_path: negative row count");
    if (exact_max_m < 0 || exact_max_m > kExactMax)
        return fail(SA_ERR_INVALID, "sa_overlap_path: exact_max_m must be 0.." + std::to_string(kExactMax));
    std::vector<Frag> fr;
    read_frags(text_h, n, &fr);
    const int64_t m = int64_t(fr.size());
    // edge weights; a pair listed twice keeps its largest weight
    std::unordered_map<uint64_t, int32_t> w;
    w.reserve(size_t(r) * 2 + 1);
    for (int64_t k = 0; k < r; ++k) {
        const int32_t a = rows_h[3 * k], b = rows_h[3 * k + 1], l = rows_h[3 * k + 2];
        if (a < 0 || b < 0 || a >= m || b >= m || a == b)
            return fail(SA_ERR_INVALID, "sa_overlap_path: a row names a fragment out of range");
        if (l < 0 || l > fr[size_t(a)].len || l > fr[size_t(b)].len)
            return fail(SA_ERR_INVALID, "sa_overlap_path: a row's length exceeds its fragments");
        int32_t &slot = w[edge_key(a, b)];
        slot = std::max(slot, l);
    }
    std::vector<int32_t> order;
    if (m <= exact_max_m) {
        std::vector<int64_t> W(size_t(m * m), 0);
        for (const auto &kv : w) W[size_t(kv.first >> 32) * size_t(m) + size_t(kv.first & 0xffffffffu)] = kv.second;
        if (m > 0) exact_path(int(m), W, &order);
    } else {
        std::vector<std::array<int32_t, 3>> edges;
        edges.reserve(w.size());
        for (const auto &kv : w)
            edges.push_back({int32_t(kv.first >> 32), int32_t(kv.first & 0xffffffffu), kv.second});
        greedy_path(m, edges, &order);
    }
    int64_t weight = 0, len = m > 0 ? fr[size_t(order[0])].len : 0;
    for (size_t k = 0; k + 1 < order.size(); ++k) {
        auto it = w.find(edge_key(order[k], order[k + 1]));
        const int64_t l = it == w.end() ? 0 : it->second;
        weight += l;
        len += fr[size_t(order[k + 1])].len - l;
    }
    std::copy(order.begin(), order.end(), order_h);
    *weight_h = weight;
    *rs_len_h = len;
    if (len > rs_cap) return fail(SA_ERR_CAPACITY, "sa_overlap_path: superstring longer than rs_cap");
    int64_t o = 0;
    for (size_t k = 0; k < order.size(); ++k) {
        int64_t skip = 0;
        if (k > 0) {
            auto it = w.find(edge_key(order[k - 1], order[k]));
            skip = it == w.end() ? 0 : it->second;
        }
        const Frag &f = fr[size_t(order[k])];
        std::memcpy(rs_h + o, text_h + f.start + skip, size_t(f.len - skip));
        o += f.len - skip;
    }
    return SA_OK;
}

}  // namespace saasm

using namespace saasm;

extern "C" int sa_overlap_path(const uint8_t *text_h, int64_t n, const int32_t *rows_h, int64_t r,
                               int32_t exact_max_m, int32_t *order_h, int64_t *weight_h,
                               uint8_t *rs_h, int64_t rs_cap, int64_t *rs_len_h) {
    return guard<int>([&] {
        return overlap_path_impl(text_h, n, rows_h, r, exact_max_m, order_h, weight_h, rs_h,
                                 rs_cap, rs_len_h);
    });
}
