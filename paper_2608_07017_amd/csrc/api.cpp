// C ABI of libwos (declared in include/wos.h): validation, device storage of
// a toolbox, and the order of the kernels of one build.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "grid.hpp"
#include "window.hpp"
#include "toolbox.hpp"
#include "wos_kernels.hpp"
#include "wos_solve_kernels.hpp"

using namespace wos;

namespace {
thread_local std::string g_err;
}

namespace wos {
void set_last_error(const char* msg) { g_err = msg; }
}  // namespace wos

namespace {



wos_status fail(wos_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define WOS_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? WOS_ENOMEM : WOS_EDEVICE, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

// ------------------------------------------------------------ host geometry
double seg_dist(const double* x, const double* a, const double* b) {
  const double ex = b[0] - a[0], ey = b[1] - a[1];
  double t = ((x[0] - a[0]) * ex + (x[1] - a[1]) * ey) / (ex * ex + ey * ey);
  t = std::min(1.0, std::max(0.0, t));
  const double qx = x[0] - a[0] - t * ex, qy = x[1] - a[1] - t * ey;
  return std::sqrt(qx * qx + qy * qy);
}

double host_distance(const HostDomain& d, const double* x) {
  switch (d.kind) {
    case WOS_BALL: {
      double s = 0;
      for (int a = 0; a < d.dim; ++a) s += (x[a] - d.c[a]) * (x[a] - d.c[a]);
      return d.rad - std::sqrt(s);
    }
    case WOS_BOX: {
      double r = 1e300;
      for (int a = 0; a < d.dim; ++a) r = std::min(r, std::min(x[a] - d.lo[a], d.hi[a] - x[a]));
      return r;
    }
    case WOS_POLYGON: {
      const int nv = (int)d.verts.size() / 2;
      double r = 1e300;
      for (int e = 0; e < nv; ++e) r = std::min(r, seg_dist(x, &d.verts[2 * e], &d.verts[2 * ((e + 1) % nv)]));
      return r;
    }
    default: {
      double r = 1e300, s = 0;
      for (int a = 0; a < d.dim; ++a) {
        r = std::min(r, std::min(x[a] - d.lo[a], d.hi[a] - x[a]));
        s += (x[a] - d.c[a]) * (x[a] - d.c[a]);
      }
      return std::min(r, std::sqrt(s) - d.rad);
    }
  }
}

bool host_inside(const HostDomain& d, const double* x) {
  switch (d.kind) {
    case WOS_BALL: {
      double s = 0;
      for (int a = 0; a < d.dim; ++a) s += (x[a] - d.c[a]) * (x[a] - d.c[a]);
      return s < d.rad * d.rad;
    }
    case WOS_BOX: {
      for (int a = 0; a < d.dim; ++a)
        if (!(x[a] > d.lo[a] && x[a] < d.hi[a])) return false;
      return true;
    }
    case WOS_POLYGON: {
      const int nv = (int)d.verts.size() / 2;
      bool odd = false;
      for (int e = 0; e < nv; ++e) {
        const double* a = &d.verts[2 * e];
        const double* b = &d.verts[2 * ((e + 1) % nv)];
        if ((a[1] > x[1]) != (b[1] > x[1])) {
          const double xint = a[0] + (x[1] - a[1]) * (b[0] - a[0]) / (b[1] - a[1]);
          if (x[0] < xint) odd = !odd;
        }
      }
      return odd;
    }
    default: {
      double s = 0;
      for (int a = 0; a < d.dim; ++a) {
        if (!(x[a] > d.lo[a] && x[a] < d.hi[a])) return false;
        s += (x[a] - d.c[a]) * (x[a] - d.c[a]);
      }
      return s > d.rad * d.rad;
    }
  }
}

void host_bbox(const HostDomain& d, double* lo, double* hi) {
  for (int a = 0; a < 3; ++a) lo[a] = hi[a] = 0;
  switch (d.kind) {
    case WOS_BALL:
      for (int a = 0; a < d.dim; ++a) {
        lo[a] = d.c[a] - d.rad;
        hi[a] = d.c[a] + d.rad;
      }
      break;
    case WOS_POLYGON: {
      lo[0] = lo[1] = 1e300;
      hi[0] = hi[1] = -1e300;
      for (size_t v = 0; v < d.verts.size(); v += 2)
        for (int a = 0; a < 2; ++a) {
          lo[a] = std::min(lo[a], d.verts[v + a]);
          hi[a] = std::max(hi[a], d.verts[v + a]);
        }
      break;
    }
    default:
      for (int a = 0; a < d.dim; ++a) {
        lo[a] = d.lo[a];
        hi[a] = d.hi[a];
      }
  }
}

// boundary measure: length (d = 2) or area (d = 3)
double host_boundary_measure(const HostDomain& d) {
  const double pi = 3.14159265358979323846;
  switch (d.kind) {
    case WOS_BALL: return d.dim == 2 ? 2 * pi * d.rad : 4 * pi * d.rad * d.rad;
    case WOS_BOX: {
      if (d.dim == 2) return 2 * ((d.hi[0] - d.lo[0]) + (d.hi[1] - d.lo[1]));
      const double e0 = d.hi[0] - d.lo[0], e1 = d.hi[1] - d.lo[1], e2 = d.hi[2] - d.lo[2];
      return 2 * (e0 * e1 + e1 * e2 + e0 * e2);
    }
    case WOS_POLYGON: {
      const int nv = (int)d.verts.size() / 2;
      double L = 0;
      for (int e = 0; e < nv; ++e) {
        const double* a = &d.verts[2 * e];
        const double* b = &d.verts[2 * ((e + 1) % nv)];
        L += std::hypot(b[0] - a[0], b[1] - a[1]);
      }
      return L;
    }
    default: {
      const double e0 = d.hi[0] - d.lo[0], e1 = d.hi[1] - d.lo[1], e2 = d.hi[2] - d.lo[2];
      return 2 * (e0 * e1 + e1 * e2 + e0 * e2) + 4 * pi * d.rad * d.rad;
    }
  }
}

template <typename T>
DomainDev<T> to_dev(const HostDomain& d) {
  DomainDev<T> o{};
  o.kind = d.kind;
  o.dim = d.dim;
  for (int a = 0; a < 3; ++a) {
    o.c[a] = (T)d.c[a];
    o.lo[a] = (T)d.lo[a];
    o.hi[a] = (T)d.hi[a];
  }
  o.rad = (T)d.rad;
  return o;
}

template <typename T>
GridDev<T> view(const DevGrid& g, const void* pts) {
  GridDev<T> v{};
  for (int a = 0; a < 3; ++a) {
    v.n[a] = g.n[a];
    v.lo[a] = (T)g.lo[a];
    v.inv_h[a] = (T)(1.0 / g.h[a]);
    v.top[a] = (T)(g.n[a] - 1);
  }
  v.rec = g.rec;
  v.list = g.list;
  if constexpr (sizeof(T) == 4)
    v.ovf = g.ovf32;
  else
    v.ovf = g.ovf64;
  v.pts = static_cast<const T*>(pts);
  return v;
}

}  // namespace

namespace {

size_t tsize(const wos_toolbox* tb) { return tb->f64 ? 8 : 4; }

wos_status dev_alloc(wos_toolbox* tb, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(WOS_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  tb->bytes += bytes;
  return WOS_OK;
}

template <typename T>
std::vector<T> padded(const std::vector<double>& pts, int count, int dim) {
  const int st = dim == 2 ? 2 : 4;
  std::vector<T> o((size_t)count * st, T(0));
  for (int j = 0; j < count; ++j)
    for (int a = 0; a < dim; ++a) o[(size_t)j * st + a] = (T)pts[(size_t)j * dim + a];
  return o;
}

wos_status upload(wos_toolbox* tb, void** dst, const void* src, size_t bytes) {
  wos_status s = dev_alloc(tb, dst, bytes);
  if (s != WOS_OK) return s;
  WOS_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return WOS_OK;
}

wos_status upload_grid(wos_toolbox* tb, const GridHost& h, DevGrid* g) {
  for (int a = 0; a < 3; ++a) {
    g->n[a] = h.n[a];
    g->lo[a] = h.lo[a];
    g->h[a] = h.h[a];
  }
  g->ncell = h.rec.size() / 4;
  g->nlist = h.list.size();
  g->frac_single = h.frac_single;
  g->mean_multi = h.mean_multi;
  g->max_cand = h.max_cand;
  wos_status s = upload(tb, (void**)&g->rec, h.rec.data(), h.rec.size() * sizeof(int));
  if (s != WOS_OK) return s;
  if ((s = upload(tb, (void**)&g->list, h.list.data(), h.list.size() * sizeof(int))) != WOS_OK) return s;
  std::vector<float> o32(h.ovf.size());
  for (size_t e = 0; e < h.ovf.size(); e += 4) {
    for (int a = 0; a < 3; ++a) o32[e + a] = (float)h.ovf[e + a];
    const int j = (int)h.ovf[e + 3];
    std::memcpy(&o32[e + 3], &j, 4);
  }
  if ((s = upload(tb, (void**)&g->ovf32, o32.data(), o32.size() * sizeof(float))) != WOS_OK) return s;
  return upload(tb, (void**)&g->ovf64, h.ovf.data(), h.ovf.size() * sizeof(double));
}

void release(wos_toolbox* tb) {
  free_work(tb->sw);
  for (auto& e : tb->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  void* ptrs[] = {tb->gv.rec, tb->gv.list, tb->gv.ovf32, tb->gv.ovf64, tb->gg.rec, tb->gg.list, tb->gg.ovf32,
                  tb->gg.ovf64, tb->gv_r.ovf32, tb->gv_r.ovf64, tb->gg_r.ovf32, tb->gg_r.ovf64, tb->d_sites_f32,
                  tb->d_sites_f64, tb->d_bnodes, tb->d_segs, tb->d_verts, tb->d_A, tb->d_B,
                  tb->d_K, tb->d_H, tb->d_Hc, tb->d_vcount, tb->d_stats, tb->d_lambda,
                  tb->d_item_order, tb->gv_r.rec, tb->gv_r.list, tb->gg_r.rec, tb->gg_r.list,
                  tb->d_vsites_r, tb->d_bnodes_r, tb->d_vrank, tb->d_brank, tb->d_win, tb->d_items, tb->d_site_steps,
                  tb->d_mom_phi, tb->d_mom_psi, tb->d_mom, tb->d_SV, tb->d_SG, tb->d_bfy, tb->d_bfpart};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (tb->wv) {  // the V-side arrays are separate allocations only with a V partition of their own
    void* vptrs[] = {tb->gw.rec, tb->gw.list, tb->gw.ovf32, tb->gw.ovf64, tb->d_vsites_f32, tb->d_vsites_f64, tb->d_lambda_v, tb->d_vcount_v};
    for (void* q : vptrs)
      if (q) (void)hipFree(q);
  }
}

bool finite3(const double* v, int k) {
  for (int i = 0; i < k; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

#define WOS_TRY(x)                    \
  do {                                \
    const wos_status s_ = (x);        \
    if (s_ != WOS_OK) return s_;      \
  } while (0)

namespace {

std::atomic<uint64_t> g_next_uid{1};

// Validation shared by wos_toolbox_create_wv and wos_toolbox_plan: fills the
// host domain and the column count (*m = n without a V partition).
wos_status validate_inputs(const wos_domain* dom, const double* sites, int32_t n, const double* vcentres,
                           int32_t* m, const double* bnodes, int32_t p, const wos_build_opts* opts, HostDomain* out) {
  if (!dom || !sites || !bnodes || !opts) return fail(WOS_EINVAL, "NULL argument");
  if (dom->dim != 2 && dom->dim != 3) return fail(WOS_EINVAL, "dim must be 2 or 3");
  if (n < 1 || p < 1) return fail(WOS_EINVAL, "need n >= 1 and p >= 1 (n=%d, p=%d)", n, p);
  const bool wv = vcentres != nullptr;
  if (!wv) *m = n;
  if (*m < 1) return fail(WOS_EINVAL, "need m >= 1 V centres (m=%d)", *m);
  if (opts->walks_per_site < 1 || opts->walks_per_site > (int64_t)INT32_MAX)
    return fail(WOS_EINVAL, "walks_per_site must be in [1, 2^31)");
  if (opts->fixed_M < 0) return fail(WOS_EINVAL, "fixed_M must be >= 0");
  if (opts->fixed_M == 0 && !(opts->eps > 0.0 && std::isfinite(opts->eps)))
    return fail(WOS_EINVAL, "eps must be finite and > 0");
  if (opts->max_steps < 0) return fail(WOS_EINVAL, "max_steps must be >= 0");
  if (opts->precision != WOS_F32 && opts->precision != WOS_F64)
    return fail(WOS_EINVAL, "precision must be WOS_F32 or WOS_F64");
  if (opts->volume_samples < 0) return fail(WOS_EINVAL, "volume_samples must be >= 0");
  if (opts->regen_threshold < 0 || opts->regen_threshold > 64)
    return fail(WOS_EINVAL, "regen_threshold must be in [0, 64]");
  if (opts->walks_per_item < 0) return fail(WOS_EINVAL, "walks_per_item must be >= 0");
  if (opts->sampler != WOS_SAMPLER_MEDIAN3 && opts->sampler != WOS_SAMPLER_LAMBERT)
    return fail(WOS_EINVAL, "unknown sampler %d", opts->sampler);
  if (opts->sampler == WOS_SAMPLER_LAMBERT && dom->dim != 2)
    return fail(WOS_EINVAL, "the Lambert W sampler is for d = 2");
  if (opts->tally_mode < WOS_TALLY_AUTO || opts->tally_mode > WOS_TALLY_HBM)
    return fail(WOS_EINVAL, "unknown tally_mode %d", opts->tally_mode);
  if (opts->tally_acc < WOS_ACC_AUTO || opts->tally_acc > WOS_ACC_F64)
    return fail(WOS_EINVAL, "unknown tally_acc %d", opts->tally_acc);
  if (opts->walker_block != 0 && opts->walker_block != 256 && opts->walker_block != 448 &&
      opts->walker_block != 512 && opts->walker_block != 1024)
    return fail(WOS_EINVAL, "walker_block must be 0, 256, 448, 512 or 1024");
  if (opts->window_pages < 0 || opts->window_pages > 255 || opts->window_bpages < 0 || opts->window_bpages > 255)
    return fail(WOS_EINVAL, "window_pages and window_bpages must be in [0, 255]");
  if ((opts->test_phi || opts->test_psi) && opts->sampler != WOS_SAMPLER_MEDIAN3)
    return fail(WOS_EINVAL, "the moments of the test functionals need the median-of-three sampler");

  HostDomain& hd = *out;
  hd.kind = dom->kind;
  hd.dim = dom->dim;
  for (int a = 0; a < 3; ++a) {
    hd.c[a] = dom->center[a];
    hd.lo[a] = dom->lo[a];
    hd.hi[a] = dom->hi[a];
  }
  hd.rad = dom->radius;
  switch (dom->kind) {
    case WOS_BALL:
      if (!(dom->radius > 0) || !finite3(dom->center, dom->dim)) return fail(WOS_EINVAL, "bad ball");
      break;
    case WOS_BOX:
      for (int a = 0; a < dom->dim; ++a)
        if (!(dom->hi[a] > dom->lo[a])) return fail(WOS_EINVAL, "bad box");
      break;
    case WOS_POLYGON:
      if (dom->dim != 2) return fail(WOS_EINVAL, "polygon needs dim 2");
      if (!dom->verts || dom->nvert < 3 || dom->nvert > kMaxPolyVerts)
        return fail(WOS_EINVAL, "polygon needs 3..%d vertices", kMaxPolyVerts);
      hd.verts.assign(dom->verts, dom->verts + 2 * dom->nvert);
      if (!finite3(hd.verts.data(), 2 * dom->nvert)) return fail(WOS_EINVAL, "non-finite vertex");
      {
        double area2 = 0;
        for (int e = 0; e < dom->nvert; ++e) {
          const double* a = &hd.verts[2 * e];
          const double* b = &hd.verts[2 * ((e + 1) % dom->nvert)];
          area2 += a[0] * b[1] - a[1] * b[0];
        }
        if (!(area2 > 0)) return fail(WOS_EINVAL, "polygon vertices must be counter-clockwise");
      }
      break;
    case WOS_BOX_MINUS_BALL:
      if (dom->dim != 3) return fail(WOS_EINVAL, "box-minus-ball needs dim 3");
      for (int a = 0; a < 3; ++a)
        if (!(dom->hi[a] > dom->lo[a])) return fail(WOS_EINVAL, "bad box");
      if (!(dom->radius > 0)) return fail(WOS_EINVAL, "bad radius");
      break;
    default:
      return fail(WOS_EINVAL, "unknown domain kind %d", dom->kind);
  }
  const int d = dom->dim;
  for (int i = 0; i < n; ++i) {
    const double* x = sites + (size_t)i * d;
    if (!finite3(x, d)) return fail(WOS_EINVAL, "site %d is not finite", i);
    if (!host_inside(hd, x) || !(host_distance(hd, x) > 0))
      return fail(WOS_EDOMAIN, "site %d is not inside the domain (r = %g)", i, host_distance(hd, x));
  }
  for (int j = 0; j < p; ++j)
    if (!finite3(bnodes + (size_t)j * d, d)) return fail(WOS_EINVAL, "boundary node %d is not finite", j);
  if (wv)
    for (int j = 0; j < *m; ++j) {
      const double* y = vcentres + (size_t)j * d;
      if (!finite3(y, d)) return fail(WOS_EINVAL, "V centre %d is not finite", j);
      if (!host_inside(hd, y)) return fail(WOS_EDOMAIN, "V centre %d is not inside the domain", j);
    }
  return WOS_OK;
}

// The host decisions of a build: tally mode, accumulators, work split and
// window size.
struct Plan {
  int mode = WOS_TALLY_LDS_ROWS, acc = WOS_ACC_FIXED;
  int wpi = 1, ips = 1, pc = 0, pb = 0;
  size_t lds = 0;
  double fixed_bound = 0;
  // windowed mode: walks per item of each site (its own fixed-point bound),
  // and the number of items over all sites; wpi is then the smallest and
  // ips the most items of a site
  std::vector<int> site_wpi;
  int64_t items = 0;
};

constexpr size_t kLdsBytes = 160 * 1024;
// one walker workgroup of 1024 lanes per compute unit, using all of its LDS
// but 1 KiB (the kernel's static variables)
constexpr size_t kWindowBudget = 159 * 1024;
constexpr int64_t kWindowMinItem = 256;        // smallest item that the fixed-point guard may ask for

wos_status make_plan(const HostDomain& hd, const double* sites, int n, int m, int p, const wos_build_opts* o,
                     Plan* pl) {
  const int d = hd.dim;
  const bool f64 = o->precision == WOS_F64;
  const int nseg = hd.kind == WOS_POLYGON ? (int)hd.verts.size() / 2 : 0;
  const size_t lds_rows = walker_lds_bytes(d, m, p, nseg, f64);
  const bool rows_fit = lds_rows <= kLdsBytes;
  const bool win_ok = !f64 && (size_t)m <= permute_max_cols() && (size_t)p <= permute_max_cols();

  // bound on the sums a fixed-point word receives, per walk of an item (see
  // wos.h): |K| <= d / r0, |B| <= 4 (d / r0) R^2 / d, |A| <= 4 omega_max R^2 / d
  // over the walk's tallies, R the half-diagonal of the bounding box
  double lo[3], hi[3];
  host_bbox(hd, lo, hi);
  double R2 = 0;
  for (int a = 0; a < d; ++a) R2 += 0.25 * (hi[a] - lo[a]) * (hi[a] - lo[a]);
  std::vector<double> r0s(n);
  double r0min = 1e300;
  for (int i = 0; i < n; ++i) {
    r0s[i] = host_distance(hd, sites + (size_t)i * d);
    r0min = std::min(r0min, r0s[i]);
  }
  const double om_max = (d == 2 && o->sampler == WOS_SAMPLER_MEDIAN3) ? 12.0 : 1.0;
  auto per_walk_at = [&](double r0) {
    return std::max(d / r0, std::max(4.0 * (d / r0) * R2 / d, 4.0 * om_max * R2 / d));
  };
  const double per_walk = per_walk_at(r0min);
  // the most walks per item that keep the bound below 1/2
  const double wpi_fixed = 0.49 * 2147483648.0 / per_walk;

  int mode = o->tally_mode;
  if (mode == WOS_TALLY_AUTO)
    mode = rows_fit ? WOS_TALLY_LDS_ROWS
                    : (win_ok && wpi_fixed >= (double)std::min<int64_t>(kWindowMinItem, o->walks_per_site))
                          ? WOS_TALLY_WINDOW
                          : WOS_TALLY_HBM;
  if (mode == WOS_TALLY_LDS_ROWS && !rows_fit)
    return fail(WOS_EINVAL, "tally_mode LDS_ROWS: a site's rows take %zu bytes of LDS (at most %zu)", lds_rows,
                kLdsBytes);
  if (mode == WOS_TALLY_WINDOW && !win_ok)
    return fail(WOS_EINVAL, "tally_mode WINDOW needs an FP32 toolbox with m, p <= %zu", permute_max_cols());
  if (mode == WOS_TALLY_WINDOW && o->tally_acc == WOS_ACC_F64)
    return fail(WOS_EINVAL, "tally_mode WINDOW sums in fixed point (tally_acc FP64 is for LDS_ROWS)");
  if (mode == WOS_TALLY_WINDOW && wpi_fixed < 1.0)
    return fail(WOS_EINVAL, "tally_mode WINDOW: a site is too close to the boundary for fixed-point sums");
  pl->mode = mode;

  const int npv = (m + kPage - 1) / kPage, npb = (p + kPage - 1) / kPage;
  size_t lds = 0;
  if (mode == WOS_TALLY_WINDOW) {
    // boundary cells take one tally per walk, V cells one per step: a few
    // boundary pages and the rest of LDS for V pages (8 measured best at
    // 32768 sites, 5 % faster than 16)
    int pb = o->window_bpages > 0 ? o->window_bpages : 8;
    pb = std::max(1, std::min(pb, npb));
    int pc = o->window_pages;
    if (pc <= 0) {
      const size_t per_page = 8 * (size_t)(1 + d) * kPage;
      const size_t fixed = walker_window_lds_bytes(d, 0, pb, npv, npb, nseg) + 2 * 255;
      pc = fixed < kWindowBudget ? (int)((kWindowBudget - fixed) / per_page) : 1;
    }
    pc = std::max(1, std::min(pc, std::min(npv, 255)));
    pl->pc = pc;
    pl->pb = pb;
    lds = walker_window_lds_bytes(d, pc, pb, npv, npb, nseg);
    if (lds > kLdsBytes)
      return fail(WOS_EINVAL, "window of %d + %d pages takes %zu bytes of LDS (at most %zu)", pc, pb, lds, kLdsBytes);
  } else if (mode == WOS_TALLY_HBM) {
    lds = (f64 ? 8 : 4) * (5 * (size_t)nseg);
  } else {
    lds = lds_rows;
  }
  pl->lds = lds;

  // work split: about one (site, chunk) item per workgroup slot of the chip
  const int64_t N = o->walks_per_site;
  int64_t wpi;
  if (o->walks_per_item > 0) {
    wpi = std::min<int64_t>(o->walks_per_item, N);
  } else if (mode == WOS_TALLY_HBM) {
    // every tally goes to the toolbox in memory: split every site into items
    // of a few walks per lane, dispatched site after site, so that the rows
    // being written at any time are few and stay in the caches
    wpi = std::min<int64_t>(N, 4096);
  } else {
    const int bs = walker_block_size(lds);
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(kLdsBytes / std::max<size_t>(lds, 1), 2048 / bs));
    const int64_t slots = 256 * per_cu;
    // one round of items over the workgroup slots (two rounds, for balance,
    // cost more in per-item overhead: the 1024-site square 0.743 -> 0.699 ms)
    const int64_t ips = std::max<int64_t>(1, slots / n);
    const int64_t floor_w = std::min<int64_t>(N, 4 * (int64_t)bs);  // >= 4 walks per lane
    wpi = std::max<int64_t>((N + ips - 1) / ips, floor_w);
  }
  if (mode == WOS_TALLY_WINDOW) {
    // the windowed mode always sums in fixed point: each site's items small
    // enough for its own bound (a site far from the boundary keeps whole
    // items; fewer items, fewer flushes)
    if (N > (int64_t)INT32_MAX) return fail(WOS_EINVAL, "tally_mode WINDOW: at most 2^31 - 1 walks per site");
    pl->site_wpi.resize(n);
    int64_t wmin = wpi, imax = 1, total = 0;
    double fb = 0;
    for (int i = 0; i < n; ++i) {
      const double pw = per_walk_at(r0s[i]);
      const int64_t wi = std::max<int64_t>(1, std::min<int64_t>(wpi, (int64_t)(0.49 * 2147483648.0 / pw)));
      const int64_t k = (N + wi - 1) / wi;
      pl->site_wpi[i] = (int)wi;
      wmin = std::min(wmin, wi);
      imax = std::max(imax, k);
      total += k;
      fb = std::max(fb, (double)wi * pw / 2147483648.0);
    }
    if (total > (int64_t)INT32_MAX) return fail(WOS_EINVAL, "too many work items");
    pl->wpi = (int)wmin;
    pl->ips = (int)imax;
    pl->items = total;
    pl->fixed_bound = fb;
  } else {
    pl->wpi = (int)wpi;
    pl->ips = (int)((N + wpi - 1) / wpi);
    if ((int64_t)pl->ips * n > (int64_t)INT32_MAX) return fail(WOS_EINVAL, "too many work items");
    pl->items = (int64_t)pl->ips * n;
    pl->fixed_bound = (double)wpi * per_walk / 2147483648.0;
  }
  if (mode == WOS_TALLY_WINDOW) {
    pl->acc = WOS_ACC_FIXED;
  } else if (f64 || mode != WOS_TALLY_LDS_ROWS) {
    pl->acc = f64 ? WOS_ACC_F64 : WOS_ACC_AUTO;
  } else if (o->tally_acc == WOS_ACC_F64) {
    pl->acc = WOS_ACC_F64;
  } else if (pl->fixed_bound >= 0.5) {
    if (o->tally_acc == WOS_ACC_FIXED)
      return fail(WOS_EINVAL, "fixed-point tallies could overflow (bound %.3g of the range)", pl->fixed_bound);
    pl->acc = WOS_ACC_F64;
  } else {
    pl->acc = WOS_ACC_FIXED;
  }
  return WOS_OK;
}

}  // namespace

// Zero what a walker launch accumulates into: its statistics and, when
// sites are split over several items (atomic flushes), the tallies.
static wos_status zero_walker_outputs(wos_toolbox* tb, hipStream_t stream) {
  const size_t ts = tsize(tb);
  const size_t n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  WOS_HIP(hipMemsetAsync(tb->d_stats, 0, 4 * 8, stream));
  WOS_HIP(hipMemsetAsync(tb->d_site_steps, 0, 8 * n, stream));
  if (tb->moments) WOS_HIP(hipMemsetAsync(tb->d_mom, 0, 8 * n * (4 + 4 * d), stream));
  if (tb->items_per_site != 1 || tb->global_tally) {
    WOS_HIP(hipMemsetAsync(tb->d_A, 0, ts * n * m, stream));
    WOS_HIP(hipMemsetAsync(tb->d_B, 0, ts * d * n * m, stream));
    WOS_HIP(hipMemsetAsync(tb->d_K, 0, ts * d * n * p, stream));
    WOS_HIP(hipMemsetAsync(tb->d_Hc, 0, 4 * n * p, stream));
  }
  return WOS_OK;
}

template <typename T>
static void fill_walker_params(const wos_toolbox* tb, uint32_t k0, uint32_t k1, int block, WalkerParams<T>& P) {
  const bool f64 = std::is_same<T, double>::value;
  P.dom = to_dev<T>(tb->dom);
  P.segs = static_cast<const T*>(tb->d_segs);
  P.nseg = (int)tb->dom.verts.size() / 2;
  P.sites = static_cast<const T*>(f64 ? tb->d_sites_f64 : tb->d_sites_f32);
  P.gv = view<T>(tb->gv, f64 ? tb->d_vsites_f64 : tb->d_vsites_f32);
  P.gg = view<T>(tb->gg, tb->d_bnodes);
  P.n = tb->n;
  P.m = tb->m;
  P.p = tb->p;
  P.walks = tb->opts.walks_per_site;
  P.walks_per_item = tb->walks_per_item;
  P.items_per_site = tb->items_per_site;
  P.eps = (T)tb->opts.eps;
  P.max_steps = tb->opts.max_steps;
  P.fixed_M = tb->opts.fixed_M;
  P.k0 = k0;
  P.k1 = k1;
  P.inv_N = (T)(1.0 / (double)tb->opts.walks_per_site);
  P.regen_T = tb->regen_T;
  P.block_override = block;
  P.item_order = tb->d_item_order;
  P.items = tb->d_items;  // windowed mode (NULL otherwise)
  P.direct_store = tb->items_per_site == 1 ? 1 : 0;
  P.global_tally = tb->global_tally ? 1 : 0;
  P.window = tb->tally_mode == WOS_TALLY_WINDOW ? 1 : 0;
  if (P.window) {
    // the walker's columns are Morton ranks: grids over the ranked centres
    P.gv = view<T>(tb->gv_r, tb->d_vsites_r);
    P.gg = view<T>(tb->gg_r, tb->d_bnodes_r);
    P.win = tb->d_win;
    P.win_pc = tb->win_pc;
    P.win_pb = tb->win_pb;
    P.npv = (tb->m + kPage - 1) / kPage;
    P.npb = (tb->p + kPage - 1) / kPage;
  }
  P.exact_radius = tb->opts.sampler == WOS_SAMPLER_LAMBERT ? 1 : 0;
  P.acc_fixed = f64 ? 0 : tb->acc_fixed;  // FP64 toolboxes accumulate in FP64
  P.A = static_cast<T*>(tb->d_A);
  P.B = static_cast<T*>(tb->d_B);
  P.Hc = tb->d_Hc;
  P.K = static_cast<T*>(tb->d_K);
  P.stats = tb->d_stats;
  P.site_steps = tb->d_site_steps;
  P.mom_phi = static_cast<const T*>(tb->d_mom_phi);
  P.mom_psi = static_cast<const T*>(tb->d_mom_psi);
  P.mom = tb->moments ? tb->d_mom : nullptr;
}

// max_items > 0 launches only the first max_items items of the order (the
// autotuner's timing runs)
static wos_status launch_walker(const wos_toolbox* tb, uint32_t k0, uint32_t k1, int block, hipStream_t stream,
                                int max_items = 0) {
  int items = tb->n_items;
  if (max_items > 0) items = std::min(items, max_items);
  if (tb->f64) {
    WalkerParams<double> P{};
    fill_walker_params<double>(tb, k0, k1, block, P);
    WOS_HIP(launch_walker_f64(P, tb->dim, tb->dom.kind, items, stream));
  } else {
    WalkerParams<float> P{};
    fill_walker_params<float>(tb, k0, k1, block, P);
    WOS_HIP(launch_walker_f32(P, tb->dim, tb->dom.kind, items, stream));
  }
  return WOS_OK;
}

extern "C" {

const char* wos_last_error(void) { return g_err.c_str(); }

const char* wos_version(void) { return "libwos 0.1 (gfx950)"; }

wos_status wos_toolbox_create(const wos_domain* dom, const double* sites, int32_t n,
                              const double* bnodes, int32_t p, const wos_build_opts* opts,
                              wos_toolbox** out) {
  return wos_toolbox_create_wv(dom, sites, n, nullptr, 0, bnodes, p, opts, out);
}

wos_status wos_toolbox_plan(const wos_domain* dom, const double* sites, int32_t n, const double* vcentres,
                            int32_t m, const double* bnodes, int32_t p, const wos_build_opts* opts,
                            wos_build_plan* out) {
  g_err.clear();
  if (!out) return fail(WOS_EINVAL, "out is NULL");
  std::memset(out, 0, sizeof *out);
  HostDomain hd;
  WOS_TRY(validate_inputs(dom, sites, n, vcentres, &m, bnodes, p, opts, &hd));
  Plan pl;
  WOS_TRY(make_plan(hd, sites, n, m, p, opts, &pl));
  out->tally_mode = pl.mode;
  out->tally_acc = pl.acc;
  out->walks_per_item = pl.wpi;
  out->items_per_site = pl.ips;
  out->window_pages = pl.pc;
  out->window_bpages = pl.pb;
  out->lds_bytes = (int64_t)pl.lds;
  out->fixed_bound = pl.fixed_bound;
  return WOS_OK;
}

wos_status wos_toolbox_create_wv(const wos_domain* dom, const double* sites, int32_t n, const double* vcentres,
                                 int32_t m, const double* bnodes, int32_t p, const wos_build_opts* opts,
                                 wos_toolbox** out) {
  g_err.clear();
  if (!out) return fail(WOS_EINVAL, "out is NULL");
  *out = nullptr;
  HostDomain hd;
  WOS_TRY(validate_inputs(dom, sites, n, vcentres, &m, bnodes, p, opts, &hd));
  Plan pl;
  WOS_TRY(make_plan(hd, sites, n, m, p, opts, &pl));
  const bool wv = vcentres != nullptr;
  const int d = dom->dim;

  wos_toolbox* tb = new (std::nothrow) wos_toolbox();
  if (!tb) return fail(WOS_ENOMEM, "host allocation failed");
  tb->uid = g_next_uid.fetch_add(1);
  tb->dom = hd;
  tb->opts = *opts;
  tb->dim = d;
  tb->n = n;
  tb->m = m;
  tb->p = p;
  tb->wv = wv;
  tb->f64 = opts->precision == WOS_F64;
  tb->sites.assign(sites, sites + (size_t)n * d);
  tb->vsites.assign(wv ? vcentres : sites, (wv ? vcentres : sites) + (size_t)m * d);
  tb->bnodes.assign(bnodes, bnodes + (size_t)p * d);
  if (tb->opts.max_steps == 0) tb->opts.max_steps = kDefaultMaxSteps;
  if (tb->opts.volume_samples == 0) tb->opts.volume_samples = (int64_t)1 << 24;
  tb->regen_T = tb->opts.regen_threshold ? tb->opts.regen_threshold : 48;
  tb->tally_mode = pl.mode;
  tb->global_tally = pl.mode == WOS_TALLY_HBM || pl.mode == WOS_TALLY_WINDOW;
  tb->acc_fixed = pl.acc == WOS_ACC_FIXED ? 1 : 0;
  tb->walks_per_item = pl.wpi;
  tb->items_per_site = pl.ips;
  tb->n_items = (int)pl.items;
  tb->win_pc = pl.pc;
  tb->win_pb = pl.pb;
  tb->autotune = opts->autotune != 0;
  tb->walker_block = opts->walker_block;
  const int nseg = hd.kind == WOS_POLYGON ? dom->nvert : 0;

  // nearest-centre grids
  double lo[3], hi[3];
  host_bbox(hd, lo, hi);
  double vol = 1;
  for (int a = 0; a < d; ++a) vol *= (hi[a] - lo[a]);
  // cell side: a fraction 1/h_div of the mean centre spacing, so that most
  // cells hold at most four candidates.  2-D: 1/8.  3-D: the finest cells
  // whose records (16 bytes a cell, h_div^3 cells per centre) stay within
  // 150 MiB, with h_div between 6 and 10: finer cells list fewer
  // candidates, so fewer centre loads per lookup, until the records
  // outgrow the caches.  Measured on the walker: the 4096-site ball 13.0 ms
  // at 1/6, 11.7 at 1/9 and 1/10, 12.2 at 1/12; the 32768-site cube minus
  // ball (1e5 walks) 1374 ms at 1/6, 1348 at 1/6.75, 1368 at 1/7 (this
  // rule gives 1/6.7 there and 1/10 for the ball).  At 1/6 about 2 % of the
  // cells of uniformly scattered centres go to the overflow entries.
  auto h_div_for = [&](int count) {
    if (d == 2) return 8.0;
    const double h = std::cbrt(150.0 * 1024.0 * 1024.0 / (16.0 * count));
    return std::min(10.0, std::max(6.0, h));
  };
  const double h_v = std::pow(vol / m, 1.0 / d) / h_div_for(m);
  GridHost gvh = build_grid(tb->vsites.data(), m, d, lo, hi, h_v, 1 << 24);
  GridHost gwh;
  if (wv) gwh = build_grid(sites, n, d, lo, hi, std::pow(vol / n, 1.0 / d) / h_div_for(n), 1 << 24);
  const double bm = host_boundary_measure(hd);
  const double sp_b = d == 2 ? bm / p : std::sqrt(bm / p);
  // boundary-node grids: cells of 1/4 (2-D) or 1/6 (3-D) of the node
  // spacing (3-D at 1/6 against 1/4: the 32768-site build 1.2 % faster)
  const double b_div = d == 2 ? 4.0 : 6.0;
  GridHost ggh = build_grid(bnodes, p, d, lo, hi, sp_b / b_div, 1 << 23);

  wos_status s = WOS_OK;
#define TRY(x)          \
  do {                  \
    s = (x);            \
    if (s != WOS_OK) {  \
      release(tb);      \
      delete tb;        \
      return s;         \
    }                   \
  } while (0)
  {
    std::vector<int> order;
    order.reserve((size_t)n * tb->items_per_site);
    if (pl.mode == WOS_TALLY_WINDOW) {
      // items of sites in Morton order, each site split by its own item
      // size, in eight contiguous runs dealt to the workgroup slots
      // round-robin (workgroup b runs on accelerator die b mod 8, so each
      // die walks one compact part of the domain and its L2 holds that
      // part's grid records and toolbox rows)
      std::vector<int> so = morton_order(sites, n, d, lo, hi);
      const int64_t N = tb->opts.walks_per_site;
      std::vector<int4> items;
      items.reserve((size_t)pl.items);
      for (int i : so) {
        const int64_t wi = pl.site_wpi[i], k = (N + wi - 1) / wi;
        for (int64_t c = 0; c < k; ++c)
          items.push_back(make_int4(i, (int)(c * wi), (int)std::min<int64_t>(N, (c + 1) * wi), k == 1 ? 1 : 0));
      }
      std::vector<int4> dealt;
      dealt.reserve(items.size());
      const size_t T = items.size(), run = (T + 7) / 8;
      for (size_t k = 0; k < run; ++k)
        for (size_t x = 0; x < 8; ++x)
          if (x * run + k < T) dealt.push_back(items[x * run + k]);
      TRY(upload(tb, (void**)&tb->d_items, dealt.data(), dealt.size() * sizeof(int4)));
    } else {
      // items in order of decreasing expected work: walks from sites far
      // from the boundary take more steps
      std::vector<int> site_rank(n);
      std::vector<double> r0(n);
      for (int i = 0; i < n; ++i) {
        site_rank[i] = i;
        r0[i] = host_distance(hd, sites + (size_t)i * d);
      }
      std::stable_sort(site_rank.begin(), site_rank.end(), [&](int a, int b) { return r0[a] > r0[b]; });
      for (int i : site_rank)
        for (int c = 0; c < tb->items_per_site; ++c) order.push_back(i * tb->items_per_site + c);
    }
    if (!order.empty()) TRY(upload(tb, (void**)&tb->d_item_order, order.data(), order.size() * sizeof(int)));
  }
  TRY(upload_grid(tb, gvh, &tb->gv));
  TRY(upload_grid(tb, ggh, &tb->gg));
  if (wv)
    TRY(upload_grid(tb, gwh, &tb->gw));
  else
    tb->gw = tb->gv;
  {
    auto s32 = padded<float>(tb->sites, n, d);
    auto s64 = padded<double>(tb->sites, n, d);
    TRY(upload(tb, &tb->d_sites_f32, s32.data(), s32.size() * 4));
    TRY(upload(tb, &tb->d_sites_f64, s64.data(), s64.size() * 8));
    if (wv) {
      auto v32 = padded<float>(tb->vsites, m, d);
      auto v64 = padded<double>(tb->vsites, m, d);
      TRY(upload(tb, &tb->d_vsites_f32, v32.data(), v32.size() * 4));
      TRY(upload(tb, &tb->d_vsites_f64, v64.data(), v64.size() * 8));
    } else {
      tb->d_vsites_f32 = tb->d_sites_f32;
      tb->d_vsites_f64 = tb->d_sites_f64;
    }
    if (tb->f64) {
      auto b = padded<double>(tb->bnodes, p, d);
      TRY(upload(tb, &tb->d_bnodes, b.data(), b.size() * 8));
    } else {
      auto b = padded<float>(tb->bnodes, p, d);
      TRY(upload(tb, &tb->d_bnodes, b.data(), b.size() * 4));
    }
  }
  if (pl.mode == WOS_TALLY_WINDOW) {
    // V centres and boundary nodes ranked along a Morton curve, their grids
    // (records hold ranks), the caller index -> rank maps for the final
    // permutation, and each site's nearest pages
    const std::vector<int> vo = morton_order(tb->vsites.data(), m, d, lo, hi);
    const std::vector<int> bo = morton_order(bnodes, p, d, lo, hi);
    std::vector<double> vs((size_t)m * d), bs((size_t)p * d);
    std::vector<int> vr(m), br(p);
    for (int r = 0; r < m; ++r) {
      vr[vo[r]] = r;
      for (int a = 0; a < d; ++a) vs[(size_t)r * d + a] = tb->vsites[(size_t)vo[r] * d + a];
    }
    for (int r = 0; r < p; ++r) {
      br[bo[r]] = r;
      for (int a = 0; a < d; ++a) bs[(size_t)r * d + a] = bnodes[(size_t)bo[r] * d + a];
    }
    GridHost gvr = build_grid(vs.data(), m, d, lo, hi, h_v, 1 << 24);
    GridHost ggr = build_grid(bs.data(), p, d, lo, hi, sp_b / b_div, 1 << 23);
    TRY(upload_grid(tb, gvr, &tb->gv_r));
    TRY(upload_grid(tb, ggr, &tb->gg_r));
    auto v32 = padded<float>(vs, m, d);
    auto b32 = padded<float>(bs, p, d);
    TRY(upload(tb, &tb->d_vsites_r, v32.data(), v32.size() * 4));
    TRY(upload(tb, &tb->d_bnodes_r, b32.data(), b32.size() * 4));
    TRY(upload(tb, (void**)&tb->d_vrank, vr.data(), vr.size() * sizeof(int)));
    TRY(upload(tb, (void**)&tb->d_brank, br.data(), br.size() * sizeof(int)));
    // V pages by their expected share of the step tallies, boundary pages
    // (one exit per walk) by distance
    std::vector<double> vbd(m);
    for (int r = 0; r < m; ++r) vbd[r] = host_distance(hd, vs.data() + (size_t)r * d);
    double bvol = 1;
    for (int a = 0; a < d; ++a) bvol *= hi[a] - lo[a];
    const double hsp = std::pow(bvol / m, 1.0 / d);
    const std::vector<uint16_t> pv = tally_pages(sites, n, vs.data(), vbd.data(), m, d, pl.pc, hsp);
    const std::vector<uint16_t> pg = nearest_pages(sites, n, bs.data(), p, d, pl.pb);
    std::vector<uint16_t> win((size_t)n * (pl.pc + pl.pb));
    for (int i = 0; i < n; ++i) {
      std::copy(pv.begin() + (size_t)i * pl.pc, pv.begin() + (size_t)(i + 1) * pl.pc,
                win.begin() + (size_t)i * (pl.pc + pl.pb));
      std::copy(pg.begin() + (size_t)i * pl.pb, pg.begin() + (size_t)(i + 1) * pl.pb,
                win.begin() + (size_t)i * (pl.pc + pl.pb) + pl.pc);
    }
    TRY(upload(tb, (void**)&tb->d_win, win.data(), win.size() * sizeof(uint16_t)));
  }
  if (opts->test_phi || opts->test_psi) {
    // the test functions in the walker's numbering of the cells (Morton
    // ranks in the windowed mode), in the toolbox precision
    tb->moments = true;
    tb->test_phi.assign(m, 0.0);
    tb->test_psi.assign(p, 0.0);
    if (opts->test_phi) tb->test_phi.assign(opts->test_phi, opts->test_phi + m);
    if (opts->test_psi) tb->test_psi.assign(opts->test_psi, opts->test_psi + p);
    tb->opts.test_phi = nullptr;  // the host copies above are the toolbox's
    tb->opts.test_psi = nullptr;
    std::vector<double> ph(tb->test_phi), ps(tb->test_psi);
    if (pl.mode == WOS_TALLY_WINDOW) {
      const std::vector<int> vo = morton_order(tb->vsites.data(), m, d, lo, hi);
      const std::vector<int> bo = morton_order(bnodes, p, d, lo, hi);
      for (int r = 0; r < m; ++r) ph[r] = tb->test_phi[vo[r]];
      for (int r = 0; r < p; ++r) ps[r] = tb->test_psi[bo[r]];
    }
    if (tb->f64) {
      TRY(upload(tb, &tb->d_mom_phi, ph.data(), 8 * (size_t)m));
      TRY(upload(tb, &tb->d_mom_psi, ps.data(), 8 * (size_t)p));
    } else {
      std::vector<float> f1(ph.begin(), ph.end()), f2(ps.begin(), ps.end());
      TRY(upload(tb, &tb->d_mom_phi, f1.data(), 4 * (size_t)m));
      TRY(upload(tb, &tb->d_mom_psi, f2.data(), 4 * (size_t)p));
    }
    TRY(dev_alloc(tb, (void**)&tb->d_mom, 8 * (size_t)n * (4 + 4 * d)));
  }
  {
    std::vector<double> seg(5 * std::max(nseg, 1), 0.0);
    for (int e = 0; e < nseg; ++e) {
      const double* a = &hd.verts[2 * e];
      const double* b = &hd.verts[2 * ((e + 1) % nseg)];
      const double ex = b[0] - a[0], ey = b[1] - a[1];
      seg[5 * e + 0] = a[0];
      seg[5 * e + 1] = a[1];
      seg[5 * e + 2] = ex;
      seg[5 * e + 3] = ey;
      seg[5 * e + 4] = 1.0 / (ex * ex + ey * ey);
    }
    if (tb->f64) {
      TRY(upload(tb, &tb->d_segs, seg.data(), seg.size() * 8));
    } else {
      std::vector<float> sf(seg.begin(), seg.end());
      TRY(upload(tb, &tb->d_segs, sf.data(), sf.size() * 4));
    }
    std::vector<double> v = hd.verts;
    if (v.empty()) v.assign(2, 0.0);
    TRY(upload(tb, (void**)&tb->d_verts, v.data(), v.size() * 8));
  }
  const size_t ts = tsize(tb);
  TRY(dev_alloc(tb, &tb->d_A, ts * (size_t)n * m));
  TRY(dev_alloc(tb, &tb->d_B, ts * (size_t)d * n * m));
  TRY(dev_alloc(tb, &tb->d_K, ts * (size_t)d * n * p));
  TRY(dev_alloc(tb, &tb->d_H, ts * (size_t)n * p));
  TRY(dev_alloc(tb, (void**)&tb->d_Hc, 4 * (size_t)n * p));
  TRY(dev_alloc(tb, (void**)&tb->d_vcount, 8 * (size_t)n));
  TRY(dev_alloc(tb, (void**)&tb->d_stats, 8 * 8));
  TRY(dev_alloc(tb, (void**)&tb->d_site_steps, 8 * (size_t)n));
  TRY(dev_alloc(tb, (void**)&tb->d_lambda, 8 * (size_t)n));
  if (wv) {
    TRY(dev_alloc(tb, (void**)&tb->d_vcount_v, 8 * (size_t)m));
    TRY(dev_alloc(tb, (void**)&tb->d_lambda_v, 8 * (size_t)m));
  } else {
    tb->d_vcount_v = tb->d_vcount;
    tb->d_lambda_v = tb->d_lambda;
  }
#undef TRY
  *out = tb;
  return WOS_OK;
}

wos_status wos_toolbox_build(wos_toolbox* tb, uint64_t seed, void* stream_) {
  g_err.clear();
  if (!tb) return fail(WOS_EINVAL, "toolbox is NULL");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  const int d = tb->dim, n = tb->n, m = tb->m, p = tb->p;
  const size_t ts = tsize(tb);
  // the walker adds into the toolbox (rather than storing its rows) when a
  // site is split over several items or its tallies reach the toolbox by
  // device atomics
  const bool accumulate = tb->items_per_site != 1 || tb->global_tally;
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFull), k1 = (uint32_t)(seed >> 32);

  WOS_HIP(hipMemsetAsync(tb->d_stats, 0, 8 * 8, stream));
  WOS_HIP(hipMemsetAsync(tb->d_site_steps, 0, 8 * (size_t)n, stream));
  if (tb->moments) WOS_HIP(hipMemsetAsync(tb->d_mom, 0, 8 * (size_t)n * (4 + 4 * d), stream));
  WOS_HIP(hipMemsetAsync(tb->d_vcount, 0, 8 * (size_t)n, stream));
  if (accumulate) {
    WOS_HIP(hipMemsetAsync(tb->d_A, 0, ts * (size_t)n * m, stream));
    WOS_HIP(hipMemsetAsync(tb->d_B, 0, ts * (size_t)d * n * m, stream));
    WOS_HIP(hipMemsetAsync(tb->d_K, 0, ts * (size_t)d * n * p, stream));
    WOS_HIP(hipMemsetAsync(tb->d_Hc, 0, 4 * (size_t)n * p, stream));
  }

  if (tb->timing) WOS_HIP(hipEventRecord(tb->ev[0], stream));
  // cell weights lambda_i
  {
    VolumeParams V{};
    V.dom = to_dev<double>(tb->dom);
    host_bbox(tb->dom, V.dom.lo, V.dom.hi);  // points are drawn in the bounding box
    V.verts = tb->d_verts;
    V.nvert = (int)tb->dom.verts.size() / 2;
    V.gv = view<double>(tb->gw, tb->d_sites_f64);
    V.n = n;
    V.dim = d;
    // stratified points: tiles^d equal tiles of the bounding box, tiles the
    // largest power of two with at least 64 points per tile, and per tile
    // the largest power of two of points that fits the requested number
    const int64_t want = tb->opts.volume_samples;
    int ts = 0, ps = 0;
    while (((int64_t)1 << (d * (ts + 1))) * 64 <= want) ++ts;
    while (((int64_t)1 << (ps + 1 + d * ts)) <= want) ++ps;
    V.tile_shift = ts;
    V.point_shift = ps;
    V.inv_tiles = 1.0 / (double)((int64_t)1 << ts);
    V.npoints = (int64_t)1 << (ps + d * ts);
    V.nblocks = d == 2 ? (V.npoints + 1) / 2 : V.npoints;
    V.k0 = k0;
    V.k1 = k1;
    V.counts = tb->d_vcount;
    V.inside = tb->d_stats + 4;
    WOS_HIP(launch_volume(V, stream));
    WOS_HIP(launch_lambda(tb->d_vcount, n, tb->d_lambda, stream));
    if (tb->wv) {
      // the same points binned to the V centres: |V_j| / |D|
      WOS_HIP(hipMemsetAsync(tb->d_vcount_v, 0, 8 * (size_t)m, stream));
      V.gv = view<double>(tb->gv, tb->d_vsites_f64);
      V.n = m;
      V.counts = tb->d_vcount_v;
      V.inside = tb->d_stats + 5;
      WOS_HIP(launch_volume(V, stream));
      WOS_HIP(launch_lambda(tb->d_vcount_v, m, tb->d_lambda_v, stream));
    }
  }
  if (tb->timing) WOS_HIP(hipEventRecord(tb->ev[1], stream));

  // walker; on the first build with autotuning, every supported workgroup
  // size is timed on the toolbox's own inputs first (on the first 4096 items
  // of the launch order: several waves of workgroups over the whole chip)
  // and the fastest is kept; the timing runs' tallies are cleared before
  // the real launch
  if (tb->autotune && tb->walker_block == 0) {
    static const int kCandidates[] = {256, 448, 512, 1024};
    hipEvent_t t0 = nullptr, t1 = nullptr;
    WOS_HIP(hipEventCreate(&t0));
    WOS_HIP(hipEventCreate(&t1));
    float best_ms = 0.0f;
    int best = 0;
    for (int bs : kCandidates) {
      WOS_TRY(zero_walker_outputs(tb, stream));
      WOS_HIP(hipEventRecord(t0, stream));
      WOS_TRY(launch_walker(tb, k0, k1, bs, stream, 4096));
      WOS_HIP(hipEventRecord(t1, stream));
      WOS_HIP(hipEventSynchronize(t1));
      float ms = 0.0f;
      WOS_HIP(hipEventElapsedTime(&ms, t0, t1));
      if (best == 0 || ms < best_ms) best_ms = ms, best = bs;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    tb->walker_block = best;
    WOS_TRY(zero_walker_outputs(tb, stream));
  }
  WOS_TRY(launch_walker(tb, k0, k1, tb->walker_block, stream));
  if (tb->timing) WOS_HIP(hipEventRecord(tb->ev[2], stream));
  if (tb->tally_mode == WOS_TALLY_WINDOW) {
    // columns from Morton ranks back to the caller's order
    WOS_HIP(launch_permute_cols(tb->d_A, n, m, tb->d_vrank, stream));
    WOS_HIP(launch_permute_cols(tb->d_B, d * n, m, tb->d_vrank, stream));
    WOS_HIP(launch_permute_cols(tb->d_K, d * n, p, tb->d_brank, stream));
    WOS_HIP(launch_permute_cols(tb->d_Hc, n, p, tb->d_brank, stream));
  }
  if (tb->f64)
    WOS_HIP(launch_h_from_counts_f64(tb->d_Hc, (size_t)n * p, 1.0 / (double)tb->opts.walks_per_site,
                                     static_cast<double*>(tb->d_H), stream));
  else
    WOS_HIP(launch_h_from_counts_f32(tb->d_Hc, (size_t)n * p, (float)(1.0 / (double)tb->opts.walks_per_site),
                                     static_cast<float*>(tb->d_H), stream));
  if (tb->timing) WOS_HIP(hipEventRecord(tb->ev[3], stream));
  tb->last_stream = stream;
  tb->built = true;
  tb->gen++;
  return WOS_OK;
}

wos_status wos_toolbox_set_timing(wos_toolbox* tb, int32_t enable) {
  g_err.clear();
  if (!tb) return fail(WOS_EINVAL, "toolbox is NULL");
  if (enable && !tb->ev[0])
    for (auto& e : tb->ev) WOS_HIP(hipEventCreate(&e));
  tb->timing = enable != 0;
  return WOS_OK;
}

wos_status wos_toolbox_get_timings(const wos_toolbox* tb, double* ms_walker, double* ms_volume,
                                   double* ms_finalize) {
  g_err.clear();
  if (!tb || !ms_walker || !ms_volume || !ms_finalize) return fail(WOS_EINVAL, "NULL argument");
  if (!tb->timing || !tb->built) return fail(WOS_EINVAL, "timing not enabled before the last build");
  WOS_HIP(hipEventSynchronize(tb->ev[3]));
  float a = 0, b = 0, c = 0;
  WOS_HIP(hipEventElapsedTime(&a, tb->ev[0], tb->ev[1]));
  WOS_HIP(hipEventElapsedTime(&b, tb->ev[1], tb->ev[2]));
  WOS_HIP(hipEventElapsedTime(&c, tb->ev[2], tb->ev[3]));
  *ms_volume = a;
  *ms_walker = b;
  *ms_finalize = c;
  return WOS_OK;
}

wos_status wos_build_toolbox(const wos_domain* dom, const double* sites, int32_t n,
                             const double* bnodes, int32_t p, const wos_build_opts* opts,
                             void* stream, wos_toolbox** out) {
  wos_status s = wos_toolbox_create(dom, sites, n, bnodes, p, opts, out);
  if (s != WOS_OK) return s;
  s = wos_toolbox_build(*out, opts->seed, stream);
  if (s == WOS_OK) {
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) s = fail(WOS_EDEVICE, "build failed: %s", hipGetErrorString(e));
  }
  if (s != WOS_OK) {
    wos_toolbox_free(*out);
    *out = nullptr;
  }
  return s;
}

wos_status wos_toolbox_get_info(const wos_toolbox* tb, wos_toolbox_info* info) {
  g_err.clear();
  if (!tb || !info) return fail(WOS_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof *info);
  info->dim = tb->dim;
  info->n = tb->n;
  info->m = tb->m;
  info->p = tb->p;
  info->precision = tb->f64 ? WOS_F64 : WOS_F32;
  info->walks_per_site = tb->opts.walks_per_site;
  info->device_bytes = tb->bytes + tb->sw.bytes;
  if (tb->built) {
    WOS_HIP(hipStreamSynchronize(tb->last_stream));
    unsigned long long st[8];
    WOS_HIP(hipMemcpy(st, tb->d_stats, sizeof st, hipMemcpyDeviceToHost));
    info->walk_steps = st[0];
    info->walks = st[1];
    info->capped_walks = st[2];
    info->max_walk_steps = st[3];
    info->volume_inside = st[4];
  }
  return WOS_OK;
}

wos_status wos_toolbox_export(const wos_toolbox* tb, int32_t what, void* dst, size_t bytes,
                              int32_t dst_is_device, void* stream_) {
  g_err.clear();
  if (!tb || !dst) return fail(WOS_EINVAL, "NULL argument");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  const size_t ts = tsize(tb), n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  const void* src = nullptr;
  size_t want = 0;
  switch (what) {
    case WOS_EXPORT_A: src = tb->d_A; want = ts * n * m; break;
    case WOS_EXPORT_B: src = tb->d_B; want = ts * d * n * m; break;
    case WOS_EXPORT_H: src = tb->d_H; want = ts * n * p; break;
    case WOS_EXPORT_K: src = tb->d_K; want = ts * d * n * p; break;
    case WOS_EXPORT_HCOUNT: src = tb->d_Hc; want = 4 * n * p; break;
    case WOS_EXPORT_LAMBDA: src = tb->d_lambda; want = 8 * n; break;
    case WOS_EXPORT_VCOUNT: src = tb->d_vcount; want = 8 * n; break;
    case WOS_EXPORT_LAMBDA_V: src = tb->d_lambda_v; want = 8 * m; break;
    case WOS_EXPORT_SITE_STEPS: src = tb->d_site_steps; want = 8 * n; break;
    case WOS_EXPORT_MOMENTS:
      if (!tb->moments) return fail(WOS_EINVAL, "the toolbox was built without test functions");
      src = tb->d_mom;
      want = 8 * n * (4 + 4 * d);
      break;
    case WOS_EXPORT_SHADOW_V:
    case WOS_EXPORT_SHADOW_G:
      if (!tb->d_SV || tb->bf16_gen != tb->gen)
        return fail(WOS_EINVAL, "no BF16 shadows of the last build (wos_toolbox_make_bf16)");
      src = what == WOS_EXPORT_SHADOW_V ? (const void*)tb->d_SV : (const void*)tb->d_SG;
      want = 2 * (what == WOS_EXPORT_SHADOW_V ? m : p) * (d + 1) * n;
      break;
    default: return fail(WOS_EINVAL, "unknown export %d", what);
  }
  if (bytes != want) return fail(WOS_EINVAL, "export %d needs %zu bytes, got %zu", what, want, bytes);
  if (dst_is_device) {
    WOS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream));
  } else {
    WOS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream));
    WOS_HIP(hipStreamSynchronize(stream));
  }
  return WOS_OK;
}

wos_status wos_apply(const wos_toolbox* tb, const double* fbar, const double* g, double* u,
                     double* grad_u, void* stream_) {
  g_err.clear();
  if (!tb || !fbar || !g || !u) return fail(WOS_EINVAL, "NULL argument");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  if (tb->f64) {
    WOS_HIP(launch_apply_f64(static_cast<const double*>(tb->d_A), tb->n, tb->m, fbar,
                             static_cast<const double*>(tb->d_H), tb->p, g, u, 1, stream));
    if (grad_u)
      WOS_HIP(launch_apply_f64(static_cast<const double*>(tb->d_B), tb->n, tb->m, fbar,
                               static_cast<const double*>(tb->d_K), tb->p, g, grad_u, tb->dim, stream));
  } else {
    WOS_HIP(launch_apply_f32(static_cast<const float*>(tb->d_A), tb->n, tb->m, fbar,
                             static_cast<const float*>(tb->d_H), tb->p, g, u, 1, stream));
    if (grad_u)
      WOS_HIP(launch_apply_f32(static_cast<const float*>(tb->d_B), tb->n, tb->m, fbar,
                               static_cast<const float*>(tb->d_K), tb->p, g, grad_u, tb->dim, stream));
  }
  return WOS_OK;
}

wos_status wos_toolbox_take(wos_toolbox* dst, const wos_toolbox* src, uint32_t mask, void* stream_) {
  g_err.clear();
  if (!dst || !src) return fail(WOS_EINVAL, "NULL argument");
  if (mask < 1 || mask > 15) return fail(WOS_EINVAL, "mask must be in 1..15");
  if (!dst->built || !src->built) return fail(WOS_EINVAL, "both toolboxes must be built");
  const HostDomain &a = dst->dom, &b = src->dom;
  bool same = dst->f64 == src->f64 && dst->dim == src->dim && dst->n == src->n && dst->m == src->m &&
              dst->p == src->p && a.kind == b.kind && a.dim == b.dim && a.rad == b.rad && a.verts == b.verts &&
              dst->sites == src->sites && dst->vsites == src->vsites && dst->bnodes == src->bnodes;
  for (int k = 0; k < 3; ++k) same = same && a.c[k] == b.c[k] && a.lo[k] == b.lo[k] && a.hi[k] == b.hi[k];
  if (!same) return fail(WOS_EINVAL, "toolboxes differ in precision, domain, sites or boundary nodes");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  const size_t ts = tsize(dst), n = dst->n, m = dst->m, p = dst->p, d = dst->dim;
  if (mask & WOS_TAKE_A) WOS_HIP(hipMemcpyAsync(dst->d_A, src->d_A, ts * n * m, hipMemcpyDeviceToDevice, stream));
  if (mask & WOS_TAKE_B)
    WOS_HIP(hipMemcpyAsync(dst->d_B, src->d_B, ts * d * n * m, hipMemcpyDeviceToDevice, stream));
  if (mask & WOS_TAKE_H) {
    WOS_HIP(hipMemcpyAsync(dst->d_H, src->d_H, ts * n * p, hipMemcpyDeviceToDevice, stream));
    WOS_HIP(hipMemcpyAsync(dst->d_Hc, src->d_Hc, 4 * n * p, hipMemcpyDeviceToDevice, stream));
  }
  if (mask & WOS_TAKE_K)
    WOS_HIP(hipMemcpyAsync(dst->d_K, src->d_K, ts * d * n * p, hipMemcpyDeviceToDevice, stream));
  dst->gen++;
  return WOS_OK;
}

extern "C++" {
namespace wos {

wos_status toolbox_bf16_current(wos_toolbox* tb, hipStream_t stream) {
  if (!tb->built) return fail(WOS_EINVAL, "toolbox has not been built");
  if (tb->d_SV && tb->bf16_gen == tb->gen) return WOS_OK;
  const size_t n = tb->n, m = tb->m, p = tb->p, d = tb->dim, KB = (d + 1) * n;
  wos_status s;
  if (!tb->d_SV) {
    if ((s = dev_alloc(tb, (void**)&tb->d_SV, 2 * m * KB)) != WOS_OK) return s;
    if ((s = dev_alloc(tb, (void**)&tb->d_SG, 2 * p * KB)) != WOS_OK) return s;
    if ((s = dev_alloc(tb, (void**)&tb->d_bfy, 8 * KB)) != WOS_OK) return s;
    if ((s = dev_alloc(tb, (void**)&tb->d_bfpart, 8 * gemv_t_bf16_part_elems((int)KB))) != WOS_OK) return s;
  }
  WOS_HIP(launch_shadow_t(tb->f64, tb->d_B, (int)(d * n), (int)m, tb->d_SV, KB, 0, stream));
  WOS_HIP(launch_shadow_t(tb->f64, tb->d_A, (int)n, (int)m, tb->d_SV, KB, (int)(d * n), stream));
  WOS_HIP(launch_shadow_t(tb->f64, tb->d_K, (int)(d * n), (int)p, tb->d_SG, KB, 0, stream));
  WOS_HIP(launch_shadow_t(tb->f64, tb->d_H, (int)n, (int)p, tb->d_SG, KB, (int)(d * n), stream));
  tb->bf16_gen = tb->gen;
  return WOS_OK;
}

}  // namespace wos
}

wos_status wos_gemm_bf16_nt(int32_t M, int32_t N, int32_t K, float alpha, const uint16_t* X, int64_t ldx,
                            const uint16_t* Y, int64_t ldy, float beta, float* C, int64_t ldc, void* stream) {
  g_err.clear();
  if (M < 0 || N < 0 || K < 0) return fail(WOS_EINVAL, "negative size");
  if (M == 0 || N == 0) return WOS_OK;
  if (!C || (K > 0 && (!X || !Y))) return fail(WOS_EINVAL, "NULL argument");
  if (ldx < K || ldy < K || ldc < N) return fail(WOS_EINVAL, "leading dimension below the row length");
  WOS_HIP(gemm_nt_bf16(M, N, K, alpha, X, (size_t)ldx, Y, (size_t)ldy, beta, C, (size_t)ldc,
                       static_cast<hipStream_t>(stream)));
  return WOS_OK;
}

wos_status wos_toolbox_make_bf16(wos_toolbox* tb, void* stream) {
  g_err.clear();
  if (!tb) return fail(WOS_EINVAL, "toolbox is NULL");
  return toolbox_bf16_current(tb, static_cast<hipStream_t>(stream));
}

wos_status wos_apply_bf16(wos_toolbox* tb, const double* fbar, const double* g, double* u, double* grad_u,
                          void* stream_) {
  g_err.clear();
  if (!tb || !fbar || !g || !u) return fail(WOS_EINVAL, "NULL argument");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  wos_status s = toolbox_bf16_current(tb, stream);
  if (s != WOS_OK) return s;
  const int n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  const size_t KB = (size_t)(d + 1) * n;
  WOS_HIP(launch_gemv_t_bf16(tb->d_SV, m, (int)KB, KB, fbar, 1.0, 0.0, tb->d_bfy, tb->d_bfpart, stream));
  WOS_HIP(launch_gemv_t_bf16(tb->d_SG, p, (int)KB, KB, g, 1.0, 1.0, tb->d_bfy, tb->d_bfpart, stream));
  WOS_HIP(launch_split_apply(n, d, tb->d_bfy, u, grad_u, stream));
  return WOS_OK;
}

wos_status wos_interpolate(const wos_toolbox* tb, const double* u, const double* grad_u, const double* x,
                           int64_t npts, double* out, int32_t* site, void* stream_) {
  g_err.clear();
  if (!tb || !u || (npts > 0 && (!x || !out))) return fail(WOS_EINVAL, "NULL argument");
  if (npts < 0) return fail(WOS_EINVAL, "npts must be >= 0");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  if (tb->f64)
    WOS_HIP(launch_interpolate<double>(tb->dim, view<double>(tb->gw, tb->d_sites_f64),
                                       static_cast<const double*>(tb->d_sites_f64), u, grad_u, tb->n, x, npts, out,
                                       site, stream));
  else
    WOS_HIP(launch_interpolate<float>(tb->dim, view<float>(tb->gw, tb->d_sites_f32),
                                      static_cast<const double*>(tb->d_sites_f64), u, grad_u, tb->n, x, npts, out,
                                      site, stream));
  return WOS_OK;
}

void wos_toolbox_free(wos_toolbox* tb) {
  if (!tb) return;
  if (tb->built && tb->last_stream) (void)hipStreamSynchronize(tb->last_stream);
  release(tb);
  delete tb;
}

}  // extern "C"
