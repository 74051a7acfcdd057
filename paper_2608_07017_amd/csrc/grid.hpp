// Host-side nearest-centre grid (see grid.cpp).
#pragma once

#include <cstdint>
#include <vector>

namespace wos {

struct GridHost {
  int dim = 2;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0};
  double h[3] = {1, 1, 1};
  // One 16-byte record per cell: up to four candidates inline, ascending,
  // unused slots repeating the first; a cell with more candidates stores
  // x = -(offset + 1) into `list` ([count, j_1 < j_2 < ...]), y = count and
  // z = the offset of its first entry in `ovf`.
  std::vector<int> rec;   // 4 ints per cell
  std::vector<int> list;
  // The overflow candidates again, in list order, as self-contained entries
  // of 4 values (the centre padded to three coordinates, then its index), so
  // that a lookup reads them without first reading the index list.
  std::vector<double> ovf;
  double frac_single = 1.0;
  double mean_multi = 1.0;
  int max_cand = 1;
};

// pts: npts x dim (double, host).  [lo, hi]: the box covered.  h_target:
// requested cell side (enlarged until the cell count is <= max_cells).
GridHost build_grid(const double* pts, int npts, int dim, const double* lo, const double* hi,
                    double h_target, int max_cells);

}  // namespace wos
