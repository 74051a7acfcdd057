// Saving and loading a built toolbox (C ABI wos_toolbox_save / _load): the
// operator toolbox is computed once and stored for reuse with any
// coefficients and data (the precomputation of eq. LOT).
//
// File layout (little endian): the magic "WOSTBOX1", a u32 format version,
// then tagged sections, each u32 tag, u64 byte count, payload:
//   1 header  (i32 dim, n, m, p, precision, wv; the domain: i32 kind,
//             f64 center[3], radius, lo[3], hi[3], i32 nvert; the build
//             options field by field; u64 statistics[8])
//   2 polygon vertices (f64, 2 nvert)    3 W centres (f64, n d)
//   4 V centres (f64, m d; only with a V partition of its own)
//   5 boundary nodes (f64, p d)
//   10 A  11 B  12 H  13 K (toolbox precision)  14 exit counts (u32)
//   15 lambda (f64, n)  16 volume counts (u64, n)
//   17 |V_j| / |D| (f64, m)  18 V volume counts (u64, m)   (V partition only)
//   19 walk-steps per site (u64, n)
//   20 test function phi (f64, m)  21 psi (f64, p)  (after section 5)
//   22 moments (f64, n (4 + 4 d))  (before the end; sections 20-22 only for a
//      toolbox built with test functions)
//   0 end
// Loading creates the toolbox from the stored inputs (grids and layouts are
// rebuilt on the host) and copies the stored arrays into its device memory.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "toolbox.hpp"

namespace wos {
void set_last_error(const char* msg);  // api.cpp
}

using namespace wos;

namespace {

constexpr char kMagic[8] = {'W', 'O', 'S', 'T', 'B', 'O', 'X', '1'};
constexpr uint32_t kVersion = 1;
constexpr size_t kChunk = (size_t)64 << 20;  // host staging per copy

enum : uint32_t {
  kEnd = 0, kHeader = 1, kVerts = 2, kSites = 3, kVSites = 4, kBnodes = 5,
  kA = 10, kB = 11, kH = 12, kK = 13, kHc = 14, kLambda = 15, kVcount = 16, kLambdaV = 17, kVcountV = 18,
  kSiteSteps = 19, kTestPhi = 20, kTestPsi = 21, kMoments = 22
};

wos_status pfail(wos_status s, const char* fmt, ...) {
  char buf[768];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  wos::set_last_error(buf);
  return s;
}

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) std::fclose(f);
  }
};

// header payload: plain fields in a fixed order
struct Header {
  int32_t dim, n, m, p, precision, wv;
  int32_t kind;
  double center[3], radius, lo[3], hi[3];
  int32_t nvert;
  int64_t walks_per_site;
  double eps;
  int32_t max_steps, fixed_M;
  uint64_t seed;
  int64_t volume_samples;
  int32_t walks_per_item, regen_threshold, autotune, tally_mode, sampler, walker_block, tally_acc, window_pages,
      window_bpages;
  uint64_t stats[8];
};

template <typename T>
void put(std::vector<unsigned char>& b, const T& v) {
  const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
  b.insert(b.end(), p, p + sizeof(T));
}
template <typename T>
bool get(const std::vector<unsigned char>& b, size_t& at, T* v) {
  if (at + sizeof(T) > b.size()) return false;
  std::memcpy(v, b.data() + at, sizeof(T));
  at += sizeof(T);
  return true;
}

std::vector<unsigned char> pack(const Header& h) {
  std::vector<unsigned char> b;
  put(b, h.dim); put(b, h.n); put(b, h.m); put(b, h.p); put(b, h.precision); put(b, h.wv);
  put(b, h.kind);
  for (double v : h.center) put(b, v);
  put(b, h.radius);
  for (double v : h.lo) put(b, v);
  for (double v : h.hi) put(b, v);
  put(b, h.nvert);
  put(b, h.walks_per_site); put(b, h.eps); put(b, h.max_steps); put(b, h.fixed_M); put(b, h.seed);
  put(b, h.volume_samples); put(b, h.walks_per_item); put(b, h.regen_threshold); put(b, h.autotune);
  put(b, h.tally_mode); put(b, h.sampler); put(b, h.walker_block); put(b, h.tally_acc); put(b, h.window_pages);
  put(b, h.window_bpages);
  for (uint64_t v : h.stats) put(b, v);
  return b;
}

bool unpack(const std::vector<unsigned char>& b, Header* h) {
  size_t at = 0;
  bool ok = get(b, at, &h->dim) && get(b, at, &h->n) && get(b, at, &h->m) && get(b, at, &h->p) &&
            get(b, at, &h->precision) && get(b, at, &h->wv) && get(b, at, &h->kind);
  for (double& v : h->center) ok = ok && get(b, at, &v);
  ok = ok && get(b, at, &h->radius);
  for (double& v : h->lo) ok = ok && get(b, at, &v);
  for (double& v : h->hi) ok = ok && get(b, at, &v);
  ok = ok && get(b, at, &h->nvert) && get(b, at, &h->walks_per_site) && get(b, at, &h->eps) &&
       get(b, at, &h->max_steps) && get(b, at, &h->fixed_M) && get(b, at, &h->seed) &&
       get(b, at, &h->volume_samples) && get(b, at, &h->walks_per_item) && get(b, at, &h->regen_threshold) &&
       get(b, at, &h->autotune) && get(b, at, &h->tally_mode) && get(b, at, &h->sampler) &&
       get(b, at, &h->walker_block) && get(b, at, &h->tally_acc) && get(b, at, &h->window_pages) &&
       get(b, at, &h->window_bpages);
  for (uint64_t& v : h->stats) ok = ok && get(b, at, &v);
  return ok && at == b.size();
}

bool write_section(FILE* f, uint32_t tag, const void* data, uint64_t bytes) {
  return std::fwrite(&tag, 4, 1, f) == 1 && std::fwrite(&bytes, 8, 1, f) == 1 &&
         (bytes == 0 || std::fwrite(data, 1, bytes, f) == bytes);
}

// a device array, staged through host memory in chunks
wos_status write_device(FILE* f, uint32_t tag, const void* dev, uint64_t bytes) {
  if (std::fwrite(&tag, 4, 1, f) != 1 || std::fwrite(&bytes, 8, 1, f) != 1)
    return pfail(WOS_EINVAL, "write failed (section %u)", tag);
  std::vector<unsigned char> buf(std::min<uint64_t>(bytes, kChunk));
  for (uint64_t at = 0; at < bytes; at += kChunk) {
    const size_t len = (size_t)std::min<uint64_t>(kChunk, bytes - at);
    const hipError_t e = hipMemcpy(buf.data(), static_cast<const unsigned char*>(dev) + at, len, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return pfail(WOS_EDEVICE, "device copy failed: %s", hipGetErrorString(e));
    if (std::fwrite(buf.data(), 1, len, f) != len) return pfail(WOS_EINVAL, "write failed (section %u)", tag);
  }
  return WOS_OK;
}

bool read_head(FILE* f, uint32_t* tag, uint64_t* bytes) {
  return std::fread(tag, 4, 1, f) == 1 && std::fread(bytes, 8, 1, f) == 1;
}

bool read_host(FILE* f, uint64_t bytes, std::vector<unsigned char>* out) {
  out->resize((size_t)bytes);
  return bytes == 0 || std::fread(out->data(), 1, (size_t)bytes, f) == bytes;
}

wos_status read_device(FILE* f, void* dev, uint64_t bytes) {
  std::vector<unsigned char> buf(std::min<uint64_t>(bytes, kChunk));
  for (uint64_t at = 0; at < bytes; at += kChunk) {
    const size_t len = (size_t)std::min<uint64_t>(kChunk, bytes - at);
    if (std::fread(buf.data(), 1, len, f) != len) return pfail(WOS_EINVAL, "file ends inside a section");
    const hipError_t e = hipMemcpy(static_cast<unsigned char*>(dev) + at, buf.data(), len, hipMemcpyHostToDevice);
    if (e != hipSuccess) return pfail(WOS_EDEVICE, "device copy failed: %s", hipGetErrorString(e));
  }
  return WOS_OK;
}

}  // namespace

extern "C" {

wos_status wos_toolbox_save(const wos_toolbox* tb, const char* path) {
  if (!tb || !path) return pfail(WOS_EINVAL, "NULL argument");
  if (!tb->built) return pfail(WOS_EINVAL, "toolbox has not been built");
  if (tb->last_stream) {
    const hipError_t e = hipStreamSynchronize(tb->last_stream);
    if (e != hipSuccess) return pfail(WOS_EDEVICE, "build failed: %s", hipGetErrorString(e));
  }
  Header h{};
  h.dim = tb->dim;
  h.n = tb->n;
  h.m = tb->m;
  h.p = tb->p;
  h.precision = tb->f64 ? WOS_F64 : WOS_F32;
  h.wv = tb->wv ? 1 : 0;
  h.kind = tb->dom.kind;
  for (int a = 0; a < 3; ++a) {
    h.center[a] = tb->dom.c[a];
    h.lo[a] = tb->dom.lo[a];
    h.hi[a] = tb->dom.hi[a];
  }
  h.radius = tb->dom.rad;
  h.nvert = (int32_t)(tb->dom.verts.size() / 2);
  const wos_build_opts& o = tb->opts;
  h.walks_per_site = o.walks_per_site;
  h.eps = o.eps;
  h.max_steps = o.max_steps;
  h.fixed_M = o.fixed_M;
  h.seed = o.seed;
  h.volume_samples = o.volume_samples;
  h.walks_per_item = o.walks_per_item;
  h.regen_threshold = o.regen_threshold;
  h.autotune = o.autotune;
  h.tally_mode = o.tally_mode;
  h.sampler = o.sampler;
  h.walker_block = o.walker_block;
  h.tally_acc = o.tally_acc;
  h.window_pages = o.window_pages;
  h.window_bpages = o.window_bpages;
  {
    const hipError_t e = hipMemcpy(h.stats, tb->d_stats, sizeof h.stats, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return pfail(WOS_EDEVICE, "device copy failed: %s", hipGetErrorString(e));
  }
  File file;
  file.f = std::fopen(path, "wb");
  if (!file.f) return pfail(WOS_EINVAL, "cannot open %s for writing", path);
  FILE* f = file.f;
  const std::vector<unsigned char> hb = pack(h);
  const size_t ts = tb->f64 ? 8 : 4, n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&kVersion, 4, 1, f) == 1 &&
            write_section(f, kHeader, hb.data(), hb.size()) &&
            write_section(f, kVerts, tb->dom.verts.data(), 8 * tb->dom.verts.size()) &&
            write_section(f, kSites, tb->sites.data(), 8 * n * d) &&
            (!tb->wv || write_section(f, kVSites, tb->vsites.data(), 8 * m * d)) &&
            write_section(f, kBnodes, tb->bnodes.data(), 8 * p * d) &&
            (!tb->moments || (write_section(f, kTestPhi, tb->test_phi.data(), 8 * m) &&
                              write_section(f, kTestPsi, tb->test_psi.data(), 8 * p)));
  if (!ok) return pfail(WOS_EINVAL, "write to %s failed", path);
  wos_status s;
  if ((s = write_device(f, kA, tb->d_A, ts * n * m)) != WOS_OK) return s;
  if ((s = write_device(f, kB, tb->d_B, ts * d * n * m)) != WOS_OK) return s;
  if ((s = write_device(f, kH, tb->d_H, ts * n * p)) != WOS_OK) return s;
  if ((s = write_device(f, kK, tb->d_K, ts * d * n * p)) != WOS_OK) return s;
  if ((s = write_device(f, kHc, tb->d_Hc, 4 * n * p)) != WOS_OK) return s;
  if ((s = write_device(f, kLambda, tb->d_lambda, 8 * n)) != WOS_OK) return s;
  if ((s = write_device(f, kVcount, tb->d_vcount, 8 * n)) != WOS_OK) return s;
  if (tb->wv) {
    if ((s = write_device(f, kLambdaV, tb->d_lambda_v, 8 * m)) != WOS_OK) return s;
    if ((s = write_device(f, kVcountV, tb->d_vcount_v, 8 * m)) != WOS_OK) return s;
  }
  if ((s = write_device(f, kSiteSteps, tb->d_site_steps, 8 * n)) != WOS_OK) return s;
  if (tb->moments && (s = write_device(f, kMoments, tb->d_mom, 8 * n * (4 + 4 * d))) != WOS_OK) return s;
  if (!write_section(f, kEnd, nullptr, 0) || std::fflush(f) != 0) return pfail(WOS_EINVAL, "write to %s failed", path);
  return WOS_OK;
}

wos_status wos_toolbox_load(const char* path, void* stream, wos_toolbox** out) {
  if (!path || !out) return pfail(WOS_EINVAL, "NULL argument");
  *out = nullptr;
  File file;
  file.f = std::fopen(path, "rb");
  if (!file.f) return pfail(WOS_EINVAL, "cannot open %s", path);
  FILE* f = file.f;
  char magic[8];
  uint32_t version = 0;
  if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, kMagic, 8) != 0)
    return pfail(WOS_EINVAL, "%s is not a saved toolbox", path);
  if (std::fread(&version, 4, 1, f) != 1 || version != kVersion)
    return pfail(WOS_EINVAL, "%s: format version %u, this library reads %u", path, version, kVersion);
  uint32_t tag;
  uint64_t bytes;
  std::vector<unsigned char> hb, verts, sites, vsites, bnodes;
  Header h{};
  if (!read_head(f, &tag, &bytes) || tag != kHeader || bytes > 4096 || !read_host(f, bytes, &hb) || !unpack(hb, &h))
    return pfail(WOS_EINVAL, "%s: bad header", path);
  if ((h.dim != 2 && h.dim != 3) || h.n < 1 || h.m < 1 || h.p < 1 || h.nvert < 0 || h.nvert > 64 ||
      (h.precision != WOS_F32 && h.precision != WOS_F64))
    return pfail(WOS_EINVAL, "%s: bad header values", path);
  const size_t n = h.n, m = h.m, p = h.p, d = h.dim;
  auto expect = [&](uint32_t want, uint64_t want_bytes, std::vector<unsigned char>* dst) -> bool {
    return read_head(f, &tag, &bytes) && tag == want && bytes == want_bytes && read_host(f, bytes, dst);
  };
  if (!expect(kVerts, 16 * (uint64_t)h.nvert, &verts) || !expect(kSites, 8 * n * d, &sites) ||
      (h.wv && !expect(kVSites, 8 * m * d, &vsites)) || !expect(kBnodes, 8 * p * d, &bnodes))
    return pfail(WOS_EINVAL, "%s: bad input sections", path);
  // optional test functions, then the first array section's head
  std::vector<unsigned char> phi, psi;
  if (!read_head(f, &tag, &bytes)) return pfail(WOS_EINVAL, "%s: file ends after the inputs", path);
  if (tag == kTestPhi) {
    if (bytes != 8 * m || !read_host(f, bytes, &phi) || !expect(kTestPsi, 8 * p, &psi) ||
        !read_head(f, &tag, &bytes))
      return pfail(WOS_EINVAL, "%s: bad test-function sections", path);
  }
  wos_domain dom{};
  dom.kind = h.kind;
  dom.dim = h.dim;
  for (int a = 0; a < 3; ++a) {
    dom.center[a] = h.center[a];
    dom.lo[a] = h.lo[a];
    dom.hi[a] = h.hi[a];
  }
  dom.radius = h.radius;
  dom.nvert = h.nvert;
  dom.verts = h.nvert ? reinterpret_cast<const double*>(verts.data()) : nullptr;
  wos_build_opts o{};
  o.walks_per_site = h.walks_per_site;
  o.eps = h.eps;
  o.max_steps = h.max_steps;
  o.fixed_M = h.fixed_M;
  o.seed = h.seed;
  o.precision = h.precision;
  o.volume_samples = h.volume_samples;
  o.walks_per_item = h.walks_per_item;
  o.regen_threshold = h.regen_threshold;
  o.autotune = h.autotune;
  o.tally_mode = h.tally_mode;
  o.sampler = h.sampler;
  o.walker_block = h.walker_block;
  o.tally_acc = h.tally_acc;
  o.window_pages = h.window_pages;
  o.window_bpages = h.window_bpages;
  if (!phi.empty()) {
    o.test_phi = reinterpret_cast<const double*>(phi.data());
    o.test_psi = reinterpret_cast<const double*>(psi.data());
  }
  wos_toolbox* tb = nullptr;
  wos_status s = wos_toolbox_create_wv(&dom, reinterpret_cast<const double*>(sites.data()), h.n,
                                       h.wv ? reinterpret_cast<const double*>(vsites.data()) : nullptr, h.m,
                                       reinterpret_cast<const double*>(bnodes.data()), h.p, &o, &tb);
  if (s != WOS_OK) return s;
  std::unique_ptr<wos_toolbox, void (*)(wos_toolbox*)> guard(tb, wos_toolbox_free);
  const size_t ts = tb->f64 ? 8 : 4;
  struct Sec {
    uint32_t tag;
    void* dev;
    uint64_t bytes;
  };
  std::vector<Sec> secs = {{kA, tb->d_A, ts * n * m},     {kB, tb->d_B, ts * d * n * m}, {kH, tb->d_H, ts * n * p},
                           {kK, tb->d_K, ts * d * n * p}, {kHc, tb->d_Hc, 4 * n * p},    {kLambda, tb->d_lambda, 8 * n},
                           {kVcount, tb->d_vcount, 8 * n}};
  if (h.wv) {
    secs.push_back({kLambdaV, tb->d_lambda_v, 8 * m});
    secs.push_back({kVcountV, tb->d_vcount_v, 8 * m});
  }
  secs.push_back({kSiteSteps, tb->d_site_steps, 8 * n});
  bool first = true;  // the first array section's head was read above
  for (const Sec& sc : secs) {
    if ((!first && !read_head(f, &tag, &bytes)) || tag != sc.tag || bytes != sc.bytes)
      return pfail(WOS_EINVAL, "%s: section %u missing or of the wrong size", path, sc.tag);
    first = false;
    if ((s = read_device(f, sc.dev, bytes)) != WOS_OK) return s;
  }
  if (!read_head(f, &tag, &bytes)) return pfail(WOS_EINVAL, "%s: no end marker", path);
  if (tb->moments) {
    if (tag != kMoments || bytes != 8 * n * (4 + 4 * d))
      return pfail(WOS_EINVAL, "%s: moments section missing or of the wrong size", path);
    if ((s = read_device(f, tb->d_mom, bytes)) != WOS_OK) return s;
    if (!read_head(f, &tag, &bytes)) return pfail(WOS_EINVAL, "%s: no end marker", path);
  }
  if (tag != kEnd) return pfail(WOS_EINVAL, "%s: no end marker", path);
  {
    const hipError_t e = hipMemcpy(tb->d_stats, h.stats, sizeof h.stats, hipMemcpyHostToDevice);
    if (e != hipSuccess) return pfail(WOS_EDEVICE, "device copy failed: %s", hipGetErrorString(e));
  }
  tb->built = true;
  tb->gen++;
  tb->last_stream = static_cast<hipStream_t>(stream);
  *out = guard.release();
  return WOS_OK;
}

}  // extern "C"
