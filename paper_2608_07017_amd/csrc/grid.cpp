// Construction of the nearest-centre grids (host, FP64).  Records with fewer
// than four candidates repeat the first one in their unused slots.
//
// The toolbox bins points by their nearest centre (Voronoi membership,
// Sec. "Matrix estimators", and Rem. "implementation_tips" (iii)).  A
// uniform grid over the bounding box stores, per cell, every centre that can
// be the nearest one for some point of the cell: with c the cell centre,
// hd its half-diagonal and d* = min_j |c - y_j|, any point q of the cell has
// its nearest centre within d* + hd of q, hence within d* + 2 hd of c, so
// {j : |c - y_j| <= d* + 2 hd + margin} is a superset of the answers.  Up to
// four candidates are stored inline in the cell's 16-byte record, so one
// load resolves almost every lookup; most cells have a single candidate.  The small relative
// margin absorbs the rounding of a lookup done in FP32 and of cell indices
// computed in FP32 near cell faces.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "grid.hpp"

namespace wos {

namespace {

struct Buckets {
  std::vector<int> start;  // ncell + 1
  std::vector<int> items;
};

}  // namespace

GridHost build_grid(const double* pts, int npts, int dim, const double* lo, const double* hi,
                    double h_target, int max_cells) {
  GridHost g;
  g.dim = dim;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = 1;
    g.lo[a] = 0.0;
    g.h[a] = 1.0;
  }
  double h = h_target;
  for (;;) {
    long long tot = 1;
    for (int a = 0; a < dim; ++a) {
      const double ext = hi[a] - lo[a];
      g.n[a] = std::max(1, (int)std::ceil(ext / h));
      tot *= g.n[a];
    }
    if (tot <= max_cells) break;
    h *= 1.1;
  }
  for (int a = 0; a < dim; ++a) {
    g.lo[a] = lo[a];
    g.h[a] = (hi[a] - lo[a]) / g.n[a];
  }
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const long long ncell = (long long)n0 * n1 * n2;

  // Centres are bucketed on a coarser grid (side about the mean spacing of
  // the centres, never finer than a cell), so that searches from cells far
  // from every centre visit few buckets.
  double vol = 1.0;
  for (int a = 0; a < dim; ++a) vol *= std::max(hi[a] - lo[a], 1e-300);
  const double spacing = std::pow(vol / std::max(npts, 1), 1.0 / dim);
  int bn[3] = {1, 1, 1};
  double bh[3] = {1, 1, 1};
  for (int a = 0; a < dim; ++a) {
    const double ext = hi[a] - lo[a];
    bn[a] = std::max(1, std::min(g.n[a], (int)std::ceil(ext / std::max(spacing, g.h[a]))));
    bh[a] = ext / bn[a];
  }
  const int b0 = bn[0], b1 = bn[1], b2 = bn[2];
  auto blin = [&](int c0, int c1, int c2) -> long long { return ((long long)c0 * b1 + c1) * b2 + c2; };
  auto bucket_of = [&](const double* q, int* c) {
    for (int a = 0; a < 3; ++a) {
      if (a < dim) {
        int v = (int)std::floor((q[a] - g.lo[a]) / bh[a]);
        c[a] = std::min(std::max(v, 0), bn[a] - 1);
      } else {
        c[a] = 0;
      }
    }
  };
  const long long nbucket = (long long)b0 * b1 * b2;
  Buckets bk;
  bk.start.assign(nbucket + 1, 0);
  std::vector<long long> where(npts);
  for (int j = 0; j < npts; ++j) {
    int c[3];
    bucket_of(pts + (size_t)j * dim, c);
    where[j] = blin(c[0], c[1], c[2]);
    bk.start[where[j] + 1]++;
  }
  for (long long i = 0; i < nbucket; ++i) bk.start[i + 1] += bk.start[i];
  bk.items.resize(npts);
  {
    std::vector<int> fill(bk.start.begin(), bk.start.end() - 1);
    for (int j = 0; j < npts; ++j) bk.items[fill[where[j]]++] = j;  // ascending j per bucket
  }
  double bhmin = 1e300;
  for (int a = 0; a < dim; ++a) bhmin = std::min(bhmin, bh[a]);
  const int maxb = std::max(b0, std::max(b1, b2));

  double hd2 = 0.0, hmin = 1e300, extent = 0.0;
  for (int a = 0; a < dim; ++a) {
    hd2 += 0.25 * g.h[a] * g.h[a];
    hmin = std::min(hmin, g.h[a]);
    extent = std::max(extent, hi[a] - lo[a]);
  }
  const double hd = std::sqrt(hd2);
  const double margin = 1e-2 * hd + 1e-9 * extent;

  g.rec.assign(4 * ncell, -1);
  const unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::vector<int>> lists(nthreads);
  std::vector<std::vector<std::pair<long long, int>>> offs(nthreads);  // (cell, offset in lists[t])
  std::vector<std::pair<long long, long long>> counts(nthreads, {0, 0});  // multi cells, candidates

  auto work = [&](unsigned t) {
    std::vector<int> cand;
    for (long long cid = t; cid < ncell; cid += nthreads) {
      const int c0 = (int)(cid / ((long long)n1 * n2));
      const int c1 = (int)((cid / n2) % n1);
      const int c2 = (int)(cid % n2);
      const int cc[3] = {c0, c1, c2};
      double ctr[3] = {0, 0, 0};
      for (int a = 0; a < dim; ++a) ctr[a] = g.lo[a] + (cc[a] + 0.5) * g.h[a];
      // nearest distance by rings of buckets (Chebyshev radius s)
      int bc[3];
      bucket_of(ctr, bc);
      double best2 = 1e300;
      for (int s = 0; s <= maxb; ++s) {
        const int lo0 = bc[0] - s, hi0 = bc[0] + s;
        const int lo1 = (dim > 1) ? bc[1] - s : 0, hi1 = (dim > 1) ? bc[1] + s : 0;
        const int lo2 = (dim > 2) ? bc[2] - s : 0, hi2 = (dim > 2) ? bc[2] + s : 0;
        for (int i0 = std::max(lo0, 0); i0 <= std::min(hi0, b0 - 1); ++i0)
          for (int i1 = std::max(lo1, 0); i1 <= std::min(hi1, b1 - 1); ++i1)
            for (int i2 = std::max(lo2, 0); i2 <= std::min(hi2, b2 - 1); ++i2) {
              const int cheb = std::max(std::abs(i0 - bc[0]), std::max(std::abs(i1 - bc[1]), std::abs(i2 - bc[2])));
              if (cheb != s) continue;
              const long long b = blin(i0, i1, i2);
              for (int it = bk.start[b]; it < bk.start[b + 1]; ++it) {
                const double* y = pts + (size_t)bk.items[it] * dim;
                double d2 = 0.0;
                for (int a = 0; a < dim; ++a) d2 += (y[a] - ctr[a]) * (y[a] - ctr[a]);
                best2 = std::min(best2, d2);
              }
            }
        // every centre not yet seen is at least s bucket sides (less the
        // offset of the cell centre inside its bucket) away
        if (best2 < 1e300 && std::sqrt(best2) <= s * bhmin) break;
      }
      const double R = std::sqrt(best2) + 2.0 * hd + margin;
      const double R2 = R * R;
      int r0[3] = {0, 0, 0}, r1[3] = {0, 0, 0};
      for (int a = 0; a < dim; ++a) {
        r0[a] = std::max(0, (int)std::floor((ctr[a] - R - g.lo[a]) / bh[a]));
        r1[a] = std::min(bn[a] - 1, (int)std::floor((ctr[a] + R - g.lo[a]) / bh[a]));
      }
      cand.clear();
      for (int i0 = r0[0]; i0 <= r1[0]; ++i0)
        for (int i1 = r0[1]; i1 <= r1[1]; ++i1)
          for (int i2 = r0[2]; i2 <= r1[2]; ++i2) {
            const long long b = blin(i0, i1, i2);
            for (int it = bk.start[b]; it < bk.start[b + 1]; ++it) {
              const int j = bk.items[it];
              const double* y = pts + (size_t)j * dim;
              double d2 = 0.0;
              for (int a = 0; a < dim; ++a) d2 += (y[a] - ctr[a]) * (y[a] - ctr[a]);
              if (d2 <= R2) cand.push_back(j);
            }
          }
      // Pairwise pruning: candidate j cannot be nearest anywhere in the
      // (slightly enlarged) cell if some other candidate k is closer on the
      // whole cell.  With u = q - c and a_j = y_j - c, the difference
      // |u - a_j|^2 - |u - a_k|^2 = |a_j|^2 - |a_k|^2 + 2 u.(a_k - a_j) is
      // linear in u, so its minimum over the box is taken at a corner.  The
      // box is enlarged to cover points that an FP32 cell index assigns to
      // this cell, and the tolerance keeps near-ties.
      if (cand.size() > 1) {
        double hb[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) hb[a] = 0.5 * g.h[a] * (1.0 + 1e-3) + 1e-6 * extent;
        double hb2 = 0.0;
        for (int a = 0; a < dim; ++a) hb2 += hb[a] * hb[a];
        const size_t nc = cand.size();
        std::vector<double> av(nc * 3, 0.0), aa(nc, 0.0);
        for (size_t i = 0; i < nc; ++i) {
          const double* y = pts + (size_t)cand[i] * dim;
          for (int a = 0; a < dim; ++a) {
            av[3 * i + a] = y[a] - ctr[a];
            aa[i] += av[3 * i + a] * av[3 * i + a];
          }
        }
        auto dominated_by = [&](size_t i, size_t k) {
          double minf = aa[i] - aa[k];
          for (int a = 0; a < dim; ++a) minf -= 2.0 * std::fabs(av[3 * k + a] - av[3 * i + a]) * hb[a];
          return minf > 1e-5 * (aa[i] + hb2);
        };
        // first against the centre nearest to the cell's centre (removes
        // almost all of a long list at once), then pairwise among the rest
        size_t kn = 0;
        for (size_t i = 1; i < nc; ++i)
          if (aa[i] < aa[kn]) kn = i;
        std::vector<size_t> alive;
        for (size_t i = 0; i < nc; ++i)
          if (i == kn || !dominated_by(i, kn)) alive.push_back(i);
        std::vector<int> kept;
        for (size_t i : alive) {
          bool dominated = false;
          for (size_t k : alive)
            if (k != i && dominated_by(i, k)) {
              dominated = true;
              break;
            }
          if (!dominated) kept.push_back(cand[i]);
        }
        cand.swap(kept);
      }
      std::sort(cand.begin(), cand.end());
      if (cand.size() <= 4) {
        for (size_t c = 0; c < 4; ++c) g.rec[4 * cid + c] = cand[c < cand.size() ? c : 0];
        if (cand.size() > 1) {
          counts[t].first++;
          counts[t].second += (long long)cand.size();
        }
      } else {
        offs[t].push_back({cid, (int)lists[t].size()});
        lists[t].push_back((int)cand.size());
        lists[t].insert(lists[t].end(), cand.begin(), cand.end());
      }
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nthreads; ++t) th.emplace_back(work, t);
  for (auto& x : th) x.join();

  size_t total = 0;
  for (unsigned t = 0; t < nthreads; ++t) total += lists[t].size();
  g.list.reserve(total + 1);
  long long nmulti = 0, sumc = 0;
  int maxc = 1;
  for (unsigned t = 0; t < nthreads; ++t) {
    nmulti += counts[t].first;
    sumc += counts[t].second;
    if (counts[t].first) maxc = std::max(maxc, 2);
  }
  for (unsigned t = 0; t < nthreads; ++t) {
    const int base = (int)g.list.size();
    g.list.insert(g.list.end(), lists[t].begin(), lists[t].end());
    for (auto& pr : offs[t]) {
      g.rec[4 * pr.first] = -(base + pr.second) - 1;
      const int cnt = lists[t][pr.second];
      nmulti++;
      sumc += cnt;
      maxc = std::max(maxc, cnt);
    }
  }
  for (long long cid = 0; cid < ncell; ++cid) {
    if (g.rec[4 * cid] < 0) continue;
    int c = 1;
    while (c < 4 && g.rec[4 * cid + c] != g.rec[4 * cid]) ++c;
    maxc = std::max(maxc, c);
  }
  // overflow entries: centre coordinates and index, in list order
  for (long long cid = 0; cid < ncell; ++cid) {
    if (g.rec[4 * cid] >= 0) continue;
    const int off = -g.rec[4 * cid] - 1;
    const int cnt = g.list[off];
    g.rec[4 * cid + 1] = cnt;
    g.rec[4 * cid + 2] = (int)(g.ovf.size() / 4);
    for (int c = 0; c < cnt; ++c) {
      const int j = g.list[off + 1 + c];
      for (int a = 0; a < 3; ++a) g.ovf.push_back(a < dim ? pts[(size_t)j * dim + a] : 0.0);
      g.ovf.push_back((double)j);
    }
  }
  if (g.list.empty()) g.list.push_back(0);
  if (g.ovf.empty()) g.ovf.assign(4, 0.0);
  g.frac_single = 1.0 - (double)nmulti / (double)ncell;
  g.mean_multi = nmulti ? (double)sumc / nmulti : 1.0;
  g.max_cand = maxc;
  return g;
}

}  // namespace wos
