// Host-side set-up of the windowed tally mode (see window.cpp).
#pragma once

#include <cstdint>
#include <vector>

namespace wos {

constexpr int kPage = 64;  // cells per page of the windowed tally mode

// Order of `count` points (dim 2 or 3, row-major) along a Morton curve over
// the box [lo, hi]: order[r] = index of the point of rank r (ties by index).
std::vector<int> morton_order(const double* pts, int count, int dim, const double* lo, const double* hi);

// For each of the n sites, the `want` pages (of kPage consecutive ranks of
// the ordered centres `sorted`, count of them) nearest to the site, by the
// distance from the site to the page's bounding box, nearest first (ties by
// page index).  Result: n x want page indices.
std::vector<uint16_t> nearest_pages(const double* sites, int n, const double* sorted, int count, int dim,
                                    int want);

}  // namespace wos
