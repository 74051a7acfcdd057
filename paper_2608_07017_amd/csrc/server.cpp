// Request server over resident toolboxes (C ABI wos_server_*).
//
// Solves arrive with wos_server_submit and are queued in arrival order.
// `slots` worker threads each own a HIP stream and solve workspaces; a worker
// takes the next queued request as soon as it is free (continuous admission:
// a request that arrives while others are on the GPU starts as soon as a
// slot is free and its workspace fits the memory budget), so the solves of
// up to `slots` requests overlap on the device.  A worker keeps the
// workspaces of the toolboxes it served; when a new one would exceed the
// budget it first frees its own, and waits while other workers hold the
// memory.  Requests on a prepared operator need no workspace; a worker that
// takes one also takes the other queued requests on the same operator (up
// to max_batch) and solves them with one batched application.  Each request
// records its submit, start and end times.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "toolbox.hpp"
#include "wos_solve_kernels.hpp"

namespace wos {
void set_last_error(const char* msg);  // api.cpp
}

using namespace wos;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

wos_status sv_fail(wos_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  wos::set_last_error(buf);
  return s;
}

struct Request {
  uint64_t id = 0;
  wos_toolbox* tb = nullptr;
  uint64_t tb_uid = 0;               // the toolbox's unique id (workspace caches key on it)
  const wos_operator* op = nullptr;  // operator request (tb unused)
  wos_coeffs co{};
  const double* f = nullptr;
  const double* g = nullptr;
  double* u = nullptr;
  double* grad_u = nullptr;
  double t_submit = 0, t_start = 0, t_end = 0;
  bool done = false;
  wos_status status = WOS_OK;
  std::string error;
  wos_solve_info info{};
};

// Device bytes a solve workspace of `tb` takes (ensure_work plus the
// regularised-solve buffers), used for admission before allocating.
size_t workspace_bytes(const wos_toolbox* tb) {
  const size_t n = tb->n, m = tb->m, p = tb->p, d = tb->dim;
  const size_t M = m + (m & 1);
  const size_t vlen = std::max(std::max(n, M), std::max(p, d * n));
  size_t b = 8 * ((d + 1) * n * (m + p) + 3 * m * m + 2 * m * p + 2 * M * M + 3 * M + 10 * vlen + n * d * d + 2);
  b += 8 * (2 * (d + 1) * n + 2) + 8;
  b += 4 * ((d + 1) * n * m + 3 * m * m + m);
  b += 12 * chol_work_elems((int)m);
  b += 8 * ((size_t)kColsqChunks + 2) * m;  // exact column norms of the mixed route
  b += 8 * gemv_part_elems((int)std::max(m, p), 1);  // partial sums of the transposed products
  b += 2 * (d + 1) * n * m + 24 * m;                 // BF16 route: weighted rows, CG vectors
  return b;
}

}  // namespace

struct wos_server {
  int device = 0;
  size_t budget = 0;  // 0: unlimited
  int max_batch = 64;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_id = 1;
  size_t reserved = 0;  // bytes of workspaces held by all workers
  int waiting = 0;      // workers waiting for memory
  bool stop = false;
  std::vector<std::thread> workers;

  void worker_loop(int slot);
};

void wos_server::worker_loop(int slot) {
  (void)slot;
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
  // workspace and its reserved bytes, by toolbox id (not by address: a freed
  // toolbox's address can be reused by a new one of another shape)
  std::map<uint64_t, std::pair<SolveWork, size_t>> ws;
  auto evict_all = [&](std::unique_lock<std::mutex>& lk) {
    (void)lk;
    for (auto& kv : ws) {
      free_work(kv.second.first);
      reserved -= kv.second.second;
    }
    ws.clear();
    cv_work.notify_all();
  };
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    if (stop && queue.empty()) break;
    Request* r = queue.front();
    if (r->op) {
      // operator requests: take every queued one on this operator, up to max_batch
      std::vector<Request*> batch;
      for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < max_batch;) {
        if ((*it)->op == r->op) {
          batch.push_back(*it);
          it = queue.erase(it);
        } else {
          ++it;
        }
      }
      if (!queue.empty()) cv_work.notify_one();
      const double t_start = now_s();
      for (Request* b : batch) b->t_start = t_start;
      lk.unlock();
      std::vector<const double*> fs, gs;
      std::vector<double*> us, gus;
      for (Request* b : batch) {
        fs.push_back(b->f);
        gs.push_back(b->g);
        us.push_back(b->u);
        gus.push_back(b->grad_u);
      }
      wos_status s = wos_operator_apply(r->op, (int32_t)batch.size(), fs.data(), gs.data(), us.data(), gus.data(), st);
      std::string err = s == WOS_OK ? std::string() : std::string(wos_last_error());
      if (s == WOS_OK && hipStreamSynchronize(st) != hipSuccess) {
        s = WOS_EDEVICE;
        err = "device error while applying an operator";
      }
      const double t_end = now_s();
      lk.lock();
      for (Request* b : batch) {
        b->status = s;
        b->error = err;
        b->t_end = t_end;
        b->info.iters = 1;
        b->done = true;
      }
      cv_done.notify_all();
      continue;
    }
    // admission by memory
    if (ws.find(r->tb_uid) == ws.end()) {
      const size_t need = workspace_bytes(r->tb);
      if (budget && reserved + need > budget) evict_all(lk);
      bool gave_up = false;
      while (budget && reserved + need > budget) {
        if (reserved == 0) {  // larger than the whole budget: refuse this request
          gave_up = true;
          break;
        }
        ++waiting;
        cv_work.wait(lk);
        --waiting;
        if (stop) break;
      }
      if (stop && queue.empty()) break;
      if (queue.empty() || queue.front() != r) continue;  // another worker took it meanwhile
      queue.pop_front();
      if (gave_up) {
        r->status = WOS_ENOMEM;
        r->error = "request workspace exceeds the server's memory budget";
        r->t_start = r->t_end = now_s();
        r->done = true;
        cv_done.notify_all();
        continue;
      }
      reserved += need;
      ws[r->tb_uid] = std::make_pair(SolveWork(), need);
    } else {
      queue.pop_front();
    }
    if (!queue.empty()) cv_work.notify_one();
    SolveWork& w = ws[r->tb_uid].first;
    r->t_start = now_s();
    lk.unlock();
    wos_status s = solve_request(r->tb, w, &r->co, r->f, r->g, r->u, r->grad_u, nullptr, &r->info, st);
    std::string err = s == WOS_OK ? std::string() : std::string(wos_last_error());
    if (s == WOS_OK && hipStreamSynchronize(st) != hipSuccess) {
      s = WOS_EDEVICE;
      err = "device error while solving";
    }
    const double t_end = now_s();
    lk.lock();
    r->status = s;
    r->error = err;
    r->t_end = t_end;
    r->done = true;
    cv_done.notify_all();
    if (waiting > 0) evict_all(lk);  // let a worker that waits for memory proceed
  }
  for (auto& kv : ws) {
    free_work(kv.second.first);
    reserved -= kv.second.second;
  }
  ws.clear();
  lk.unlock();
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
}

extern "C" {

wos_status wos_server_create(const wos_server_opts* opts, wos_server** out) {
  if (!out) return sv_fail(WOS_EINVAL, "out is NULL");
  *out = nullptr;
  const int slots = (opts && opts->slots > 0) ? opts->slots : 4;
  if (slots > 16) return sv_fail(WOS_EINVAL, "slots must be in [1, 16]");
  wos_server* sv = new (std::nothrow) wos_server();
  if (!sv) return sv_fail(WOS_ENOMEM, "out of host memory");
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return sv_fail(WOS_EDEVICE, "no current HIP device");
  }
  sv->budget = opts ? opts->mem_budget : 0;
  if (opts && opts->max_batch != 0) {
    if (opts->max_batch < 1 || opts->max_batch > 1024) {
      delete sv;
      return sv_fail(WOS_EINVAL, "max_batch must be in [1, 1024]");
    }
    sv->max_batch = opts->max_batch;
  }
  for (int i = 0; i < slots; ++i) sv->workers.emplace_back([sv, i] { sv->worker_loop(i); });
  *out = sv;
  return WOS_OK;
}

wos_status wos_server_submit(wos_server* sv, wos_toolbox* tb, const wos_coeffs* co, const double* f,
                             const double* g, double* u, double* grad_u, uint64_t* ticket) {
  if (!sv || !tb || !co || !f || !g || !u || !ticket) return sv_fail(WOS_EINVAL, "NULL argument");
  if (!tb->built) return sv_fail(WOS_EINVAL, "toolbox has not been built");
  // the shadows are shared by every slot: made beforehand, never by a worker
  if (co->precision == WOS_SOLVE_MIXED_BF16 && (!tb->d_SV || tb->bf16_gen != tb->gen))
    return sv_fail(WOS_EINVAL, "BF16 requests need the toolbox's BF16 shadows of its last build "
                               "(wos_toolbox_make_bf16, its stream synchronised) before submission");
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return sv_fail(WOS_ENOMEM, "out of host memory");
  r->tb = tb;
  r->tb_uid = tb->uid;
  r->co = *co;
  r->f = f;
  r->g = g;
  r->u = u;
  r->grad_u = grad_u;
  r->t_submit = now_s();
  std::lock_guard<std::mutex> g_(sv->mu);
  r->id = sv->next_id++;
  *ticket = r->id;
  sv->queue.push_back(r.get());
  sv->reqs.emplace(r->id, std::move(r));
  sv->cv_work.notify_one();
  return WOS_OK;
}

wos_status wos_server_submit_op(wos_server* sv, const wos_operator* op, const double* f, const double* g, double* u,
                                double* grad_u, uint64_t* ticket) {
  if (!sv || !op || !f || !g || !u || !ticket) return sv_fail(WOS_EINVAL, "NULL argument");
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return sv_fail(WOS_ENOMEM, "out of host memory");
  r->op = op;
  r->f = f;
  r->g = g;
  r->u = u;
  r->grad_u = grad_u;
  r->t_submit = now_s();
  std::lock_guard<std::mutex> g_(sv->mu);
  r->id = sv->next_id++;
  *ticket = r->id;
  sv->queue.push_back(r.get());
  sv->reqs.emplace(r->id, std::move(r));
  sv->cv_work.notify_one();
  return WOS_OK;
}

wos_status wos_server_poll(wos_server* sv, uint64_t ticket, int32_t block, wos_solve_info* info, double* times) {
  if (!sv) return sv_fail(WOS_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return sv_fail(WOS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second.get();
  if (!r->done) {
    if (!block) return WOS_EBUSY;
    sv->cv_done.wait(lk, [&] { return r->done; });
  }
  if (info) *info = r->info;
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_start;
    times[2] = r->t_end;
  }
  const wos_status s = r->status;
  const std::string err = r->error;
  sv->reqs.erase(it);
  if (s != WOS_OK) return sv_fail(s, "%s", err.c_str());
  return WOS_OK;
}

wos_status wos_server_pending(wos_server* sv, int64_t* queued, int64_t* unfinished) {
  if (!sv) return sv_fail(WOS_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (queued) *queued = (int64_t)sv->queue.size();
  if (unfinished) {
    int64_t c = 0;
    for (auto& kv : sv->reqs)
      if (!kv.second->done) ++c;
    *unfinished = c;
  }
  return WOS_OK;
}

void wos_server_destroy(wos_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (auto& t : sv->workers) t.join();
  delete sv;
}

}  // extern "C"
