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

// For each of the n sites, the `want` pages of V cells with the largest
// expected share of the site's step tallies, largest first (ties by page
// index).  A page's score is sum_c 1 / (dist(c) + h) over its cells c (dist
// the distance to the domain's boundary, `bdist`, in rank order) divided by
// (rho + h)^2, rho the mean of the distances from the site to the page's
// bounding box and to its centroid, h the mean spacing of the centres.  A
// walk takes one step per unit of r^2 of exit time, and steps pile up
// where r is small, near the boundary; the share falls off with the
// distance from the site (measured on the oracle's walks in the cube minus
// ball: 95.4 % of the tallies fall in the 68 best-scored pages, 94.7 % in
// the 68 nearest).  Result: n x want page indices.
std::vector<uint16_t> tally_pages(const double* sites, int n, const double* sorted, const double* bdist, int count,
                                  int dim, int want, double h);

}  // namespace wos
