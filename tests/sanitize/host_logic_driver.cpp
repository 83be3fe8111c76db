// Checks the host-side planning of the general-mesh index (bucket counts,
// quantile edges, work items) on random and degenerate histograms; built
// with the address and undefined-behaviour sanitizers.  Exits non-zero on
// a violated property.
#include <cstdio>
#include <random>

#include "host_logic.hpp"

using namespace flp::host;

static int fails = 0;
#define EXPECT(c)                                                          \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::printf("%s:%d: expected %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                                       \
        }                                                                  \
    } while (0)

int main()
{
    std::mt19937_64 g(7);
    // bucket counts: within [1, max], product near the total for a cube
    for (int dim = 2; dim <= 3; ++dim) {
        const double L[3] = {1.0, 1.0, 1.0};
        for (double total : {0.5, 1.0, 7.0, 1000.0, 1e9}) {
            auto nb = bucket_counts(dim, L, total, 1024);
            double prod = 1.0;
            for (int a = 0; a < dim; ++a) {
                EXPECT(nb[a] >= 1 && nb[a] <= 1024);
                prod *= nb[a];
            }
            if (total >= 1.0 && total <= 1e6) EXPECT(prod <= 2.0 * total && prod >= 0.4 * total);
        }
        const double La[3] = {4.0, 1.0, 0.25};
        auto nb = bucket_counts(dim, La, 4096.0, 1024);
        EXPECT(nb[0] >= nb[1]);
    }
    // quantile edges: strictly increasing from lo to hi, at most nb + 1,
    // buckets of a smooth histogram hold similar counts
    for (int trial = 0; trial < 200; ++trial) {
        const int bins = 1 + (int)(g() % 4096);
        std::vector<uint32_t> h(bins);
        int64_t M = 0;
        const int kind = trial % 4;
        for (int b = 0; b < bins; ++b) {
            uint32_t v = kind == 0 ? 3u : kind == 1 ? (uint32_t)(g() % 50) : kind == 2 ? (b == bins / 2 ? 100000u : 0u)
                                                                                        : (uint32_t)(b * b % 97);
            h[b] = v;
            M += v;
        }
        if (M == 0) continue;
        const int nb = 1 + (int)(g() % 300);
        const double lo = -1.0 + (double)(g() % 100) * 0.01, hi = lo + 0.5 + (double)(g() % 100) * 0.1;
        auto e = quantile_edges(h.data(), bins, M, nb, lo, hi);
        EXPECT(e.size() >= 2 && (int)e.size() <= nb + 1);
        EXPECT(e.front() == lo && e.back() == hi);
        for (size_t k = 1; k < e.size(); ++k) EXPECT(e[k] > e[k - 1]);
        if (kind == 0 && bins >= 4 * nb) {
            // uniform histogram: every bucket within one bin count of M / nb
            const double per = (double)M / (double)(e.size() - 1);
            for (size_t k = 1; k < e.size(); ++k) {
                const double c = (e[k] - e[k - 1]) / ((hi - lo) / bins) * 3.0;
                EXPECT(c <= per + 3.0 * (double)bins / nb + 6.0);
            }
        }
    }
    // work items: cover every cell once, in order, with at most per_item cells,
    // and a bucket's items differ by at most one cell
    for (int trial = 0; trial < 200; ++trial) {
        const int64_t nbk = 1 + (int64_t)(g() % 500);
        std::vector<uint32_t> cs(nbk + 1, 0);
        for (int64_t b = 0; b < nbk; ++b) cs[b + 1] = cs[b] + (uint32_t)(trial % 3 == 0 ? g() % 3 : g() % 700);
        const int per = 1 + (int)(g() % 256);
        auto w = work_items(cs.data(), nbk, per);
        uint32_t next = 0;
        for (size_t k = 0; k < w.size(); ++k) {
            EXPECT(w[k].first == (int)next && w[k].count >= 1 && w[k].count <= per);
            EXPECT((uint32_t)w[k].first >= cs[w[k].bucket] &&
                   (uint32_t)(w[k].first + w[k].count) <= cs[w[k].bucket + 1]);
            if (k > 0 && w[k].bucket == w[k - 1].bucket) EXPECT(std::abs(w[k].count - w[k - 1].count) <= 1);
            next += (uint32_t)w[k].count;
        }
        EXPECT(next == cs[nbk]);
    }
    std::printf(fails ? "host logic driver: %d FAILED\n" : "host logic driver: ok\n", fails);
    return fails != 0;
}
