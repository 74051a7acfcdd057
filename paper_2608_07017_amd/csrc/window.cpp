// Host-side set-up of the windowed tally mode: the V centres and the
// boundary nodes are ranked along a Morton curve, so that a page of 64
// consecutive ranks is a compact patch of the domain, and every site gets
// the list of pages nearest to it.  The walker keeps those pages of the
// site's rows in LDS; the tallies of a walk fall in them with a probability
// that grows with the window (the walks of a site spend most of their
// occupation time near it).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

#include "window.hpp"

namespace wos {

namespace {

// spread the low 21 bits of v so that bit b lands on bit 3b (3-D) or the low
// 31 bits onto 2b (2-D)
uint64_t spread3(uint64_t v) {
  v &= 0x1FFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
uint64_t spread2(uint64_t v) {
  v &= 0xFFFFFFFFull;
  v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
  v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
  v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
  v = (v | (v << 2)) & 0x3333333333333333ull;
  v = (v | (v << 1)) & 0x5555555555555555ull;
  return v;
}

template <typename F>
void parallel_for(int n, F f) {
  const int nt = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), 16));
  if (n < 256 || nt == 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int a = t * chunk, b = std::min(n, a + chunk);
    if (a < b) th.emplace_back(f, a, b);
  }
  for (auto& t : th) t.join();
}

}  // namespace

std::vector<int> morton_order(const double* pts, int count, int dim, const double* lo, const double* hi) {
  const int bits = dim == 3 ? 21 : 31;
  const double top = (double)((1ull << bits) - 1);
  std::vector<uint64_t> code(count);
  for (int j = 0; j < count; ++j) {
    uint64_t c = 0;
    for (int a = 0; a < dim; ++a) {
      const double ext = hi[a] - lo[a];
      double t = ext > 0 ? (pts[(size_t)j * dim + a] - lo[a]) / ext : 0.0;
      t = std::min(1.0, std::max(0.0, t));
      const uint64_t q = (uint64_t)(t * top);
      c |= (dim == 3 ? spread3(q) : spread2(q)) << a;
    }
    code[j] = c;
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return code[a] < code[b]; });
  return order;
}

std::vector<uint16_t> nearest_pages(const double* sites, int n, const double* sorted, int count, int dim,
                                    int want) {
  const int npages = (count + kPage - 1) / kPage;
  want = std::min(want, npages);
  std::vector<double> plo((size_t)npages * dim), phi((size_t)npages * dim);
  for (int g = 0; g < npages; ++g)
    for (int a = 0; a < dim; ++a) {
      double l = 1e300, h = -1e300;
      for (int r = g * kPage; r < std::min(count, (g + 1) * kPage); ++r) {
        l = std::min(l, sorted[(size_t)r * dim + a]);
        h = std::max(h, sorted[(size_t)r * dim + a]);
      }
      plo[(size_t)g * dim + a] = l;
      phi[(size_t)g * dim + a] = h;
    }
  std::vector<uint16_t> out((size_t)n * want);
  parallel_for(n, [&](int i0, int i1) {
    std::vector<std::pair<double, int>> dist(npages);
    for (int i = i0; i < i1; ++i) {
      const double* x = sites + (size_t)i * dim;
      for (int g = 0; g < npages; ++g) {
        double s = 0;
        for (int a = 0; a < dim; ++a) {
          const double e = std::max(std::max(plo[(size_t)g * dim + a] - x[a], x[a] - phi[(size_t)g * dim + a]), 0.0);
          s += e * e;
        }
        dist[g] = {s, g};
      }
      std::partial_sort(dist.begin(), dist.begin() + want, dist.end());
      for (int k = 0; k < want; ++k) out[(size_t)i * want + k] = (uint16_t)dist[k].second;
    }
  });
  return out;
}

std::vector<uint16_t> tally_pages(const double* sites, int n, const double* sorted, const double* bdist, int count,
                                  int dim, int want, double h) {
  const int npages = (count + kPage - 1) / kPage;
  want = std::min(want, npages);
  std::vector<double> plo((size_t)npages * dim), phi((size_t)npages * dim), cen((size_t)npages * dim, 0.0),
      mass(npages, 0.0);
  for (int g = 0; g < npages; ++g) {
    const int r0 = g * kPage, r1 = std::min(count, (g + 1) * kPage);
    for (int a = 0; a < dim; ++a) {
      double l = 1e300, u = -1e300, c = 0;
      for (int r = r0; r < r1; ++r) {
        const double v = sorted[(size_t)r * dim + a];
        l = std::min(l, v);
        u = std::max(u, v);
        c += v;
      }
      plo[(size_t)g * dim + a] = l;
      phi[(size_t)g * dim + a] = u;
      cen[(size_t)g * dim + a] = c / (r1 - r0);
    }
    for (int r = r0; r < r1; ++r) mass[g] += 1.0 / (std::max(bdist[r], 0.0) + h);
  }
  std::vector<uint16_t> out((size_t)n * want);
  parallel_for(n, [&](int i0, int i1) {
    std::vector<std::pair<double, int>> key(npages);
    for (int i = i0; i < i1; ++i) {
      const double* x = sites + (size_t)i * dim;
      for (int g = 0; g < npages; ++g) {
        double sb = 0, sc = 0;
        for (int a = 0; a < dim; ++a) {
          const double e = std::max(std::max(plo[(size_t)g * dim + a] - x[a], x[a] - phi[(size_t)g * dim + a]), 0.0);
          const double c = cen[(size_t)g * dim + a] - x[a];
          sb += e * e;
          sc += c * c;
        }
        const double rho = 0.5 * (std::sqrt(sb) + std::sqrt(sc)) + h;
        key[g] = {-mass[g] / (rho * rho), g};  // ascending order = largest score first
      }
      std::partial_sort(key.begin(), key.begin() + want, key.end());
      for (int k = 0; k < want; ++k) out[(size_t)i * want + k] = (uint16_t)key[k].second;
    }
  });
  return out;
}

}  // namespace wos
