// Sanitizer driver of the library's host graph steps (host_graph.h), built
// by the CPU tests with -fsanitize=address,undefined: on seeded random item
// lists (and one item of size zero), greedy first fit in index and in
// priority order, neighbour counts and (family, colour) buckets are
// checked against brute force (the buckets with one and with three
// threads); items sharing one node check the colour
// count on both sides of one mask word and of kMaxColours. Exit status 0
// on success.
#include <cstdio>
#include <set>
#include <vector>

#include "../../paper_1805_03949_amd/csrc/host_graph.h"

using namespace fea::host;

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static uint64_t next_rand()
{
    // SplitMix64
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static bool share(const std::vector<int64_t> &ptr, const std::vector<int32_t> &nodes, int64_t i, int64_t j)
{
    for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p)
        for (int64_t q = ptr[j]; q < ptr[j + 1]; ++q)
            if (nodes[p] == nodes[q]) return true;
    return false;
}

static void run_case(int64_t n_nodes, int64_t n_items, int max_len)
{
    std::vector<int64_t> ptr(n_items + 1, 0);
    std::vector<int32_t> nodes;
    for (int64_t i = 0; i < n_items; ++i) {
        const int len = (int)(next_rand() % (uint64_t)(max_len + 1));  // may be 0
        std::set<int32_t> s;
        while ((int)s.size() < len) s.insert((int32_t)(next_rand() % (uint64_t)n_nodes));
        nodes.insert(nodes.end(), s.begin(), s.end());
        ptr[i + 1] = (int64_t)nodes.size();
    }
    std::vector<int32_t> nneig(n_items);
    neighbour_counts(n_nodes, n_items, ptr.data(), nodes.data(), nneig.data());
    for (int64_t i = 0; i < n_items; ++i) {
        int32_t c = 0;
        for (int64_t j = 0; j < n_items; ++j)
            if (j != i && share(ptr, nodes, i, j)) ++c;
        CHECK(nneig[i] == c);
    }
    const std::vector<int64_t> order = priority_order(n_items, nneig.data());
    for (int64_t k = 1; k < n_items; ++k) {
        CHECK(nneig[order[k - 1]] >= nneig[order[k]]);
        if (nneig[order[k - 1]] == nneig[order[k]]) CHECK(order[k - 1] < order[k]);
    }
    for (int pass = 0; pass < 2; ++pass) {
        const int64_t *ord = pass ? order.data() : nullptr;
        std::vector<int16_t> colour(n_items, -1);
        const int64_t nc = greedy_first_fit(n_nodes, n_items, ptr.data(), nodes.data(), ord, colour.data());
        CHECK(nc >= 1 || n_items == 0);
        // valid, and first fit: every smaller colour is held by a neighbour visited earlier
        std::vector<int64_t> rank(n_items);
        for (int64_t k = 0; k < n_items; ++k) rank[ord ? ord[k] : k] = k;
        for (int64_t i = 0; i < n_items; ++i) {
            CHECK(colour[i] >= 0 && colour[i] < nc);
            std::set<int> before;
            for (int64_t j = 0; j < n_items; ++j) {
                if (j == i || !share(ptr, nodes, i, j)) continue;
                CHECK(colour[i] != colour[j]);
                if (rank[j] < rank[i]) before.insert(colour[j]);
            }
            for (int c = 0; c < colour[i]; ++c) CHECK(before.count(c) == 1);
        }
        // buckets by (family, colour): every item once, in visit order
        std::vector<uint8_t> fam(n_items);
        std::vector<int64_t> first(4, 0);
        for (int64_t i = 0; i < n_items; ++i) fam[i] = (uint8_t)(4 * i / std::max<int64_t>(n_items, 1));
        for (int t = 1; t < 4; ++t) {
            first[t] = first[t - 1];
            while (first[t] < n_items && fam[first[t]] < t) ++first[t];
        }
        std::vector<int64_t> seg, seg3;
        std::vector<int32_t> list, list3;
        buckets(n_items, 4, fam.data(), colour.data(), (int)nc, ord, first.data(), seg, list, 1);
        // the chunked form (three threads) gives the one-thread result
        buckets(n_items, 4, fam.data(), colour.data(), (int)nc, ord, first.data(), seg3, list3, 3);
        CHECK(seg3 == seg && list3 == list);
        std::vector<int> seen(n_items, 0);
        for (int t = 0; t < 4; ++t)
            for (int c = 0; c < nc; ++c) {
                const int64_t b = seg[t * (nc + 1) + c], e = seg[t * (nc + 1) + c + 1];
                CHECK(b <= e);
                for (int64_t k = b; k < e; ++k) {
                    const int64_t i = first[t] + list[k];
                    CHECK(i >= 0 && i < n_items);
                    if (i < 0 || i >= n_items) continue;
                    CHECK(fam[i] == t && colour[i] == c);
                    ++seen[i];
                    if (k > b) CHECK(rank[first[t] + list[k - 1]] < rank[i]);
                }
            }
        for (int64_t i = 0; i < n_items; ++i) CHECK(seen[i] == 1);
    }
}

// k items that all hold node 0 need k colours: first fit gives item i
// colour i, through one mask word up to 64 and the full masks beyond; past
// kMaxColours the call reports the first item it cannot colour.
static void run_shared_node(int k)
{
    std::vector<int64_t> ptr(k + 1, 0);
    std::vector<int32_t> nodes;
    for (int i = 0; i < k; ++i) {
        nodes.push_back(0);
        nodes.push_back(1 + i % 3);
        ptr[i + 1] = (int64_t)nodes.size();
    }
    std::vector<int16_t> colour(k, -1), wide(k, -1);
    const int64_t nc = greedy_first_fit(4, k, ptr.data(), nodes.data(), nullptr, colour.data());
    if (k > kMaxColours) {
        CHECK(nc == -(1 + (int64_t)kMaxColours));
        return;
    }
    CHECK(nc == k);
    for (int i = 0; i < k; ++i) CHECK(colour[i] == i);
    const int64_t nw = greedy_first_fit_words<kMaxColours / 64>(4, k, ptr.data(), nodes.data(), nullptr, wide.data());
    CHECK(nw == nc && wide == colour);
}

int main()
{
    run_shared_node(1);
    run_shared_node(64);
    run_shared_node(65);
    run_shared_node(200);
    run_shared_node(kMaxColours + 1);
    run_case(1, 1, 1);
    run_case(5, 0, 3);
    run_case(40, 30, 4);
    run_case(200, 150, 8);
    run_case(60, 120, 12);
    if (failures) std::fprintf(stderr, "%d failures\n", failures);
    return failures ? 1 : 0;
}
