// Host-side graph steps that are sequential by definition: greedy
// first-fit colouring of items (elements, or element tiles) over the
// node-sharing graph, the neighbour count of every item, and the
// (family, colour) buckets the colour-by-colour launches walk. Plain C++
// (no HIP), so that it also builds and runs under the host sanitizers.
//
// An item is a list of node ids: item i holds nodes[ptr[i] .. ptr[i+1]).
// Two items are neighbours when they share a node.
#pragma once

#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

namespace fea {
namespace host {

constexpr int kMaxColours = 256;

// Greedy first fit over per-node masks of W 64-bit words (64 W colours):
// returns the number of colours, or -(1 + i) when item i would need more.
template <int W>
inline int64_t greedy_first_fit_words(int64_t n_nodes, int64_t n_items, const int64_t *ptr, const int32_t *nodes,
                                      const int64_t *order, int16_t *colour)
{
    std::vector<uint64_t> used((size_t)std::max<int64_t>(n_nodes, 1) * W, 0);
    int ncol = 0;
    for (int64_t k = 0; k < n_items; ++k) {
        const int64_t i = order ? order[k] : k;
        uint64_t m[W];
        for (int w = 0; w < W; ++w) m[w] = 0;
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p)
            for (int w = 0; w < W; ++w) m[w] |= used[(size_t)nodes[p] * W + w];
        int c = -1;
        for (int w = 0; w < W && c < 0; ++w)
            if (~m[w]) c = w * 64 + __builtin_ctzll(~m[w]);
        if (c < 0) return -(1 + i);
        colour[i] = (int16_t)c;
        ncol = std::max(ncol, c + 1);
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) used[(size_t)nodes[p] * W + c / 64] |= 1ull << (c % 64);
    }
    return ncol;
}

// Greedy first fit (Algorithm 5's colouring): items are visited in `order`
// (all n_items of them; nullptr = ascending), and each takes the smallest
// colour that no neighbour visited before it holds. Returns the number of
// colours, or -(1 + i) when item i would need more than kMaxColours. First
// with one mask word per node (a quarter of the memory traffic); only if an
// item needs a 65th colour again with the full masks, which visits the items
// in the same order and so gives the same colours.
inline int64_t greedy_first_fit(int64_t n_nodes, int64_t n_items, const int64_t *ptr, const int32_t *nodes,
                                const int64_t *order, int16_t *colour)
{
    const int64_t r = greedy_first_fit_words<1>(n_nodes, n_items, ptr, nodes, order, colour);
    if (r >= 0) return r;
    return greedy_first_fit_words<kMaxColours / 64>(n_nodes, n_items, ptr, nodes, order, colour);
}

// nneig[i] = number of other items sharing at least one node with item i
// (the neighbour count that sets a chunk's priority in Algorithm 7).
inline void neighbour_counts(int64_t n_nodes, int64_t n_items, const int64_t *ptr, const int32_t *nodes,
                             int32_t *nneig)
{
    // node -> items incidence
    std::vector<int64_t> nptr((size_t)n_nodes + 1, 0);
    for (int64_t i = 0; i < n_items; ++i)
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) ++nptr[(size_t)nodes[p] + 1];
    for (int64_t v = 0; v < n_nodes; ++v) nptr[(size_t)v + 1] += nptr[(size_t)v];
    std::vector<int64_t> fill(nptr.begin(), nptr.end() - 1);
    std::vector<int64_t> inc((size_t)std::max<int64_t>(nptr[(size_t)n_nodes], 1));
    for (int64_t i = 0; i < n_items; ++i)
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) inc[(size_t)fill[(size_t)nodes[p]]++] = i;
    std::vector<int64_t> stamp((size_t)std::max<int64_t>(n_items, 1), -1);
    for (int64_t i = 0; i < n_items; ++i) {
        int32_t cnt = 0;
        stamp[(size_t)i] = i;
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) {
            const int32_t v = nodes[p];
            for (int64_t q = nptr[(size_t)v]; q < nptr[(size_t)v + 1]; ++q) {
                const int64_t j = inc[(size_t)q];
                if (stamp[(size_t)j] != i) {
                    stamp[(size_t)j] = i;
                    ++cnt;
                }
            }
        }
        nneig[i] = cnt;
    }
}

// Visit order by descending neighbour count, ties by ascending index.
inline std::vector<int64_t> priority_order(int64_t n_items, const int32_t *nneig)
{
    std::vector<int64_t> order((size_t)n_items);
    for (int64_t i = 0; i < n_items; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return nneig[a] > nneig[b]; });
    return order;
}

// Buckets by (group, colour): group[i] in [0, n_groups), colour[i] in
// [0, ncol). seg (n_groups * (ncol + 1) entries) receives, for group g, the
// start of bucket (g, c) at seg[g * (ncol + 1) + c] and the end of its last
// bucket at seg[g * (ncol + 1) + ncol] (= the start of group g + 1's first);
// list receives the items bucket by bucket, each bucket in `order`
// (nullptr = ascending), as item - first[group] (group-local indices).
// A stable counting sort over consecutive chunks of the visit order, one
// thread each: per-chunk bucket counts, then each chunk places its items
// from its own offsets, so the result is the one-thread result. threads: 0
// = one per 2^20 items, at most 8; failing to start a thread runs its chunk
// on the calling thread.
inline void buckets(int64_t n_items, int n_groups, const uint8_t *group, const int16_t *colour, int ncol,
                    const int64_t *order, const int64_t *first, std::vector<int64_t> &seg,
                    std::vector<int32_t> &list, int threads = 0)
{
    const int64_t nb = (int64_t)n_groups * ncol;
    if (threads <= 0) threads = (int)std::min<int64_t>(8, n_items >> 20);
    threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n_items));
    std::vector<int64_t> cnt((size_t)threads * std::max<int64_t>(nb, 1), 0);
    auto item = [&](int64_t k) { return order ? order[k] : k; };
    auto in_chunks = [&](auto &&body) {
        std::vector<std::thread> pool;
        for (int p = 1; p < threads; ++p) {
            try {
                pool.emplace_back(body, p);
            } catch (...) {
                body(p);
            }
        }
        body(0);
        for (std::thread &t : pool) t.join();
    };
    in_chunks([&](int p) {
        int64_t *h = cnt.data() + (size_t)p * nb;
        for (int64_t k = n_items * p / threads, k1 = n_items * (p + 1) / threads; k < k1; ++k) {
            const int64_t i = item(k);
            ++h[group[i] * ncol + colour[i]];
        }
    });
    // bucket starts (the one-thread layout), then each chunk's start within
    // every bucket
    seg.assign((size_t)n_groups * (ncol + 1), 0);
    int64_t run = 0;
    for (int g = 0; g < n_groups; ++g) {
        for (int c = 0; c < ncol; ++c) {
            seg[(size_t)g * (ncol + 1) + c] = run;
            for (int p = 0; p < threads; ++p) {
                int64_t &h = cnt[(size_t)p * nb + g * ncol + c];
                const int64_t n = h;
                h = run;
                run += n;
            }
        }
        seg[(size_t)g * (ncol + 1) + ncol] = run;
    }
    list.assign((size_t)std::max<int64_t>(n_items, 1), 0);
    in_chunks([&](int p) {
        int64_t *off = cnt.data() + (size_t)p * nb;
        for (int64_t k = n_items * p / threads, k1 = n_items * (p + 1) / threads; k < k1; ++k) {
            const int64_t i = item(k);
            const int g = group[i];
            list[(size_t)off[g * ncol + colour[i]]++] = (int32_t)(i - (first ? first[g] : 0));
        }
    });
}

}  // namespace host
}  // namespace fea
