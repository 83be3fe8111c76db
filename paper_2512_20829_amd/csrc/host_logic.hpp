// Host-side planning of the general-mesh index, free of HIP so that it can be
// built and checked on the CPU (also under the address and undefined-
// behaviour sanitizers): per-axis bucket counts, bucket edges at quantiles
// of a coordinate histogram, and the gather's work items.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace flp {
namespace host {

// Buckets per axis: about `total` in all, shared out in proportion to the box
// edges L[a] (their geometric mean gets total^(1/dim)), each in [1, max_nb].
inline std::vector<int> bucket_counts(int dim, const double* L, double total, int max_nb)
{
    double gm = 1.0;
    for (int a = 0; a < dim; ++a) gm *= L[a];
    gm = std::pow(gm, 1.0 / dim);
    std::vector<int> nb(dim);
    for (int a = 0; a < dim; ++a) {
        const double want = std::pow(std::max(total, 1.0), 1.0 / dim) * L[a] / gm;
        nb[a] = (int)std::lround(std::min(std::max(want, 1.0), (double)max_nb));
    }
    return nb;
}

// Bucket edges of one axis from a histogram of `bins` equal bins over
// [lo, hi] holding M coordinates: lo, then for i = 1..nb-1 the right
// boundary of the first bin at which the cumulative count reaches i M / nb
// (skipped when it does not advance past the previous edge or reaches hi),
// then hi.  The result is strictly increasing, with at most nb + 1 entries.
inline std::vector<double> quantile_edges(const uint32_t* hist, int bins, int64_t M, int nb, double lo, double hi)
{
    std::vector<double> e{lo};
    const double w = (hi - lo) / (double)bins;
    int64_t cum = 0;
    int bin = 0;
    for (int i = 1; i < nb; ++i) {
        const double target = (double)i * (double)M / (double)nb;
        while (bin < bins && (double)(cum + hist[bin]) < target) cum += hist[bin++];
        if (bin >= bins - 1) break;
        const double edge = lo + (double)(bin + 1) * w;
        if (edge > e.back() && edge < hi) e.push_back(edge);
    }
    e.push_back(hi);
    return e;
}

// Work items of the gather: {bucket, first cell, cells} with at most
// per_item cells each; a bucket's cells (cstart[b] .. cstart[b+1]) are
// shared evenly between ceil(n / per_item) items, and empty buckets get none.
struct WorkItem {
    int bucket, first, count;
};
inline std::vector<WorkItem> work_items(const uint32_t* cstart, int64_t nbuckets, int per_item)
{
    std::vector<WorkItem> w;
    for (int64_t b = 0; b < nbuckets; ++b) {
        const int n = (int)(cstart[b + 1] - cstart[b]);
        if (n == 0) continue;
        const int items = (n + per_item - 1) / per_item;
        const int base = n / items, rem = n % items;
        int first = (int)cstart[b];
        for (int k = 0; k < items; ++k) {
            const int cnt = base + (k < rem ? 1 : 0);
            w.push_back({(int)b, first, cnt});
            first += cnt;
        }
    }
    return w;
}

}  // namespace host
}  // namespace flp
