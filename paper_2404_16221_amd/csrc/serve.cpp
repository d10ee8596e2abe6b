// Render server: continuous batching of novel-view requests on one GPU.
//
// Rendering a view is the inference path of the method (App. A.2: at render
// time one device gathers the per-region tuples and composites them): for every
// ray of the view, each region composites its own samples into a segment tuple
// (xl_render_segments_fwd) and the tuples are merged in ray order
// (xl_merge_fwd).  The per-region NeRF evaluation is stood in for by the
// device sample generator.
//
// Structure:
//   * xl_serve_submit puts a request on a bounded FIFO queue (XL_EAGAIN when
//     full) and stamps its arrival time.
//   * Device memory is one arena of hbm_budget_bytes, allocated when the
//     server starts and carved per request (arena.hpp): no driver allocation
//     or free happens per request, so the workers never serialise on the
//     allocator.
//   * max_slots worker threads, each owning one HIP stream (default priority)
//     and a generator workspace, take requests in arrival order.  A worker
//     runs the generator's plan phase on its own stream, with no lock held,
//     which fixes the exact footprint (result, ray offsets, samples, segment
//     arrays, tuples, tile records).  Admission is then one request at a
//     time: the admitting worker reserves that footprint in one piece,
//     waiting for memory that running requests or released results give
//     back; it holds no other reservation while it waits, so workers never
//     wait on each other's partial reservations.  A request whose footprint
//     exceeds the whole budget fails at once with XL_ENOMEM.  The worker then
//     launches generation, segment composite and merge.  Requests therefore
//     join while others are on the GPU as soon as a slot frees up, the plans
//     of different slots run side by side (a plan waits for its own counts
//     to come back to the host), and the kernels of different requests
//     overlap on the device.  The generator workspace lives outside the
//     budget: it is allocated when a slot first takes a request larger than
//     any before (about 470 bytes per ray at 8 segments per ray).
//   * Each request has its own buffers and runs the same kernels, so its result
//     does not depend on what else is in flight (bit for bit).
//   * xl_serve_poll waits for a ticket (bounded by a timeout) and reports the
//     result, its latency (completion minus arrival, host monotonic clock) and
//     its device time; xl_serve_release returns the result buffer to the arena
//     (after any copy of it made by xl_serve_copy_result has completed).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.hpp"
#include "internal.h"

namespace xl {

static int64_t now_us() {
  return std::chrono::duration_cast<std::chrono::microseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Job {
  uint64_t ticket = 0;
  xl_request req{};
  int64_t t_arrival = 0, t_admit = 0, t_done = 0;
  int32_t status = XL_PENDING;
  bool done = false;
  float* ray_out = nullptr;
  size_t arena_off = 0;         // the result block [arena_off, arena_off + result_bytes)
  hipEvent_t copied = nullptr;  // after the last xl_serve_copy_result copy
  int64_t n_rays = 0, n_samples = 0, n_seg = 0;
  uint64_t footprint = 0, result_bytes = 0;
  float device_ms = 0.f;
  float device_start_ms = -1.f, device_end_ms = -1.f;  // since the server's origin event
  char msg[160] = "";
};

struct Server {
  xl_serve_config cfg{};
  std::mutex mu;
  std::mutex admit_mu;          // one request in admission at a time
  hipEvent_t origin = nullptr;  // device-time origin of the per-request intervals
  std::condition_variable cv_queue, cv_done, cv_budget;
  std::deque<std::shared_ptr<Job>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
  std::vector<std::thread> workers;
  char* base = nullptr;  // device arena
  Arena arena;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<int64_t> latencies;  // of completed requests
  int64_t completed = 0, failed = 0, samples_done = 0;
  int64_t t_first_arrival = -1, t_last_done = 0;
};

static size_t round256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

static void finish(Server* s, const std::shared_ptr<Job>& j, int32_t status, const char* msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  j->status = status;
  j->t_done = now_us();
  j->done = true;
  if (msg) std::snprintf(j->msg, sizeof(j->msg), "%s", msg);
  if (status == XL_OK) {
    ++s->completed;
    s->samples_done += j->n_samples;
    s->latencies.push_back(j->t_done - j->t_arrival);
    s->t_last_done = std::max(s->t_last_done, j->t_done);
  } else {
    ++s->failed;
  }
  s->cv_done.notify_all();
}

static void release_block(Server* s, size_t off, size_t bytes) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->arena.release(off, bytes);
  s->cv_budget.notify_all();
}

static void run_job(Server* s, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int64_t* pinned,
                    void** ws, size_t* ws_cap, const std::shared_ptr<Job>& j) {
  const xl_request& q = j->req;
  if (q.inject_fault) {
    finish(s, j, XL_EFAULT, "fault injected by the request");
    return;
  }
  xl_gen_params p{};
  p.n_rays = static_cast<int64_t>(q.width) * q.height;
  p.ray0 = 0;
  p.n_min = q.n_min;
  p.n_max = q.n_max;
  for (int c = 0; c < 3; ++c) p.grid[c] = q.grid[c];
  p.sigma_mu = q.sigma_mu;
  p.sigma_s = q.sigma_s;
  p.zero_frac = q.zero_frac;
  p.width_mean = q.width_mean > 0 ? q.width_mean : 0.02;
  p.t_far = q.t_far > 0 ? q.t_far : 3.0;
  p.seed = q.seed;
  j->n_rays = p.n_rays;
  const int dtype = s->cfg.dtype;
  const size_t es = dtype == XL_F32 ? 4 : 2;

  // Block layout: [result | ray offsets | samples, segment arrays, region
  // offsets, tuples, tile records].  The generator's workspace (its plan,
  // read again by the fill) belongs to the slot, outside the budget.
  const int n_regions = p.grid[0] * p.grid[1] * p.grid[2];
  const size_t b_out = round256(4 * 7 * p.n_rays), b_ro = round256(8 * (p.n_rays + 1));
  const size_t head = b_out + b_ro;
  auto body = [&](int64_t n, int64_t n_seg) -> size_t {
    return round256(n * es) + round256(3 * n * es) + 2 * round256(4 * n) + round256(8 * (n_seg + 1)) +
           round256(8 * n_seg) + round256(8 * (n_regions + 1)) + round256(4 * XL_TUPLE_STRIDE * n_seg) +
           round256(xl_segments_workspace_bytes(n));
  };
  char m[200];
  auto over_budget = [&](size_t need) {
    std::snprintf(m, sizeof(m), "request needs %s%llu bytes, budget is %llu",
                  need == head ? "more than " : "", static_cast<unsigned long long>(need),
                  static_cast<unsigned long long>(s->arena.size()));
    finish(s, j, XL_ENOMEM, m);
  };
  // At least n_min samples and one segment per ray: fail before planning a
  // request that cannot fit whatever its plan gives.
  if (head > s->arena.size()) {
    over_budget(head);
    return;
  }
  const int64_t n_lo = p.n_rays * static_cast<int64_t>(p.n_min > 0 ? p.n_min : 0);
  if (head + body(n_lo, p.n_min > 0 ? p.n_rays : 0) > s->arena.size()) {
    over_budget(head + body(n_lo, p.n_min > 0 ? p.n_rays : 0));
    return;
  }
  // The slot's workspace grows to the largest request it has taken (its
  // previous request has completed: run_job synchronises before it returns).
  const size_t ws_need = gen_workspace_bytes(&p);
  if (ws_need > *ws_cap) {
    if (*ws) (void)hipFree(*ws);
    *ws = nullptr;
    *ws_cap = 0;
    if (hipMalloc(ws, ws_need) != hipSuccess) {
      *ws = nullptr;
      std::snprintf(m, sizeof(m), "generator workspace of %llu bytes could not be allocated",
                    static_cast<unsigned long long>(ws_need));
      finish(s, j, XL_ENOMEM, m);
      return;
    }
    *ws_cap = ws_need;
  }

  // The plan runs before admission and without any lock, so the plans of
  // requests taken by different slots overlap each other and running work.
  int64_t n = 0, n_seg = 0;
  int overflow = 0;
  if (gen_plan(&p, *ws, st, &n, &n_seg, &overflow, pinned) != hipSuccess || overflow) {
    (void)hipStreamSynchronize(st);  // cleanup on a path that already reports failure
    finish(s, j, XL_EHIP, "generator plan failed");
    return;
  }
  j->n_samples = n;
  j->n_seg = n_seg;
  const size_t fp = head + body(n, n_seg);
  j->footprint = fp;
  j->result_bytes = b_out;
  if (fp > s->arena.size()) {
    over_budget(fp);
    return;
  }
  // Waits (under the server mutex) until `bytes` can be carved out or the
  // server stops; false if it stopped.
  auto reserve = [&](size_t bytes, size_t* at) {
    std::unique_lock<std::mutex> lk(s->mu);
    bool got = false;
    s->cv_budget.wait(lk, [&] { return s->stop || (got = s->arena.alloc(bytes, at)); });
    return got;
  };
  // One reservation per request, one admission at a time: the admitting
  // worker holds nothing while it waits, and the others wait for it.
  size_t off = 0;
  {
    std::lock_guard<std::mutex> admission(s->admit_mu);
    if (!reserve(fp, &off)) {
      finish(s, j, XL_EAGAIN, "server stopped before the request was admitted");
      return;
    }
  }
  char* blk = s->base + off;
  float* out = reinterpret_cast<float*>(blk);
  int64_t* ro = reinterpret_cast<int64_t*>(blk + b_out);
  char* c = blk + head;

  void* sigma = c; c += round256(n * es);
  void* rgb = c; c += round256(3 * n * es);
  float* t0 = reinterpret_cast<float*>(c); c += round256(4 * n);
  float* t1 = reinterpret_cast<float*>(c); c += round256(4 * n);
  int64_t* so = reinterpret_cast<int64_t*>(c); c += round256(8 * (n_seg + 1));
  int64_t* ids = reinterpret_cast<int64_t*>(c); c += round256(8 * n_seg);
  int64_t* roff = reinterpret_cast<int64_t*>(c); c += round256(8 * (n_regions + 1));
  float* seg_out = reinterpret_cast<float*>(c); c += round256(4 * XL_TUPLE_STRIDE * n_seg);
  void* recs = c;  // per-tile records of the segment composite

  hipError_t e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = gen_fill(&p, dtype, *ws, n_seg, sigma, rgb, t0, t1, so, ro, ids, roff, st);
  SamplesDev sd{dtype, sigma, rgb, t0, t1, n};
  if (e == hipSuccess) e = launch_segments_fwd(sd, so, n_seg, seg_out, recs, st);
  if (e == hipSuccess)
    e = launch_merge_fwd(seg_out, n_seg, roff, n_regions, ro, ids, p.n_rays, out,
                         s->cfg.merge_fp64 != 0, false, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  const hipError_t es2 = hipStreamSynchronize(st);
  float ms = 0.f;
  if (e == hipSuccess && es2 == hipSuccess && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 0.f;
  j->device_ms = ms;
  if (e == hipSuccess && es2 == hipSuccess && s->origin) {
    float a = 0.f, b = 0.f;
    if (hipEventElapsedTime(&a, s->origin, e0) == hipSuccess &&
        hipEventElapsedTime(&b, s->origin, e1) == hipSuccess) {
      j->device_start_ms = a;
      j->device_end_ms = b;
    }
  }
  if (e != hipSuccess || es2 != hipSuccess) {
    release_block(s, off, fp);
    finish(s, j, XL_EHIP, hipGetErrorString(e != hipSuccess ? e : es2));
    return;
  }
  release_block(s, off + b_out, fp - b_out);  // the result stays until released
  j->ray_out = out;
  j->arena_off = off;
  finish(s, j, XL_OK, nullptr);
}

static bool stopping(Server* s) {
  std::lock_guard<std::mutex> lk(s->mu);
  return s->stop;
}

static void worker(Server* s) {
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int64_t* pinned = nullptr;  // the plan phase's readback values
  void* ws = nullptr;         // the generator's workspace, grown on demand
  size_t ws_cap = 0;
  // A slot whose stream, events or buffer cannot be made fails every request it takes.
  const bool ready = hipSetDevice(s->cfg.device) == hipSuccess &&
                     hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
                     hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
                     hipHostMalloc(reinterpret_cast<void**>(&pinned), 4 * sizeof(int64_t),
                                   hipHostMallocDefault) == hipSuccess;
  for (;;) {
    std::shared_ptr<Job> j;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_queue.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->queue.empty()) break;  // stop requested and nothing left
      j = s->queue.front();
      s->queue.pop_front();
      j->t_admit = now_us();
    }
    if (stopping(s))
      finish(s, j, XL_EAGAIN, "server destroyed before the request started");
    else if (ready)
      run_job(s, st, e0, e1, pinned, &ws, &ws_cap, j);
    else
      finish(s, j, XL_EHIP, "serving slot has no stream or events");
  }
  if (pinned) (void)hipHostFree(pinned);
  if (ws) (void)hipFree(ws);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace xl

extern "C" {

int xl_serve_create(const xl_serve_config* cfg, xl_server** out) {
  if (!cfg || !out) return xl::set_error(XL_EINVAL, "NULL config or output");
  if (cfg->max_slots < 1 || cfg->max_queue < 1)
    return xl::set_error(XL_EINVAL, "max_slots and max_queue must be >= 1");
  if (cfg->dtype != XL_F32 && cfg->dtype != XL_BF16 && cfg->dtype != XL_F16 &&
      cfg->dtype != XL_BF16_F16)
    return xl::set_error(XL_EINVAL, "unknown sample dtype %d", cfg->dtype);
  if (cfg->hbm_budget_bytes < xl::Arena::kAlign)
    return xl::set_error(XL_EINVAL, "hbm_budget_bytes must be at least %zu", xl::Arena::kAlign);
  hipError_t e = hipSetDevice(cfg->device);
  if (e != hipSuccess) return xl::set_error(XL_EHIP, "device %d: %s", cfg->device, hipGetErrorString(e));
  auto* s = new xl::Server();
  s->cfg = *cfg;
  e = hipMalloc(reinterpret_cast<void**>(&s->base), cfg->hbm_budget_bytes);
  if (e != hipSuccess) {
    delete s;
    return xl::set_error(XL_ENOMEM, "arena of %llu bytes: %s",
                         static_cast<unsigned long long>(cfg->hbm_budget_bytes), hipGetErrorString(e));
  }
  s->arena.reset(cfg->hbm_budget_bytes);
  // Device-time origin of the per-request intervals (best effort: without it
  // the intervals are reported as -1).
  if (hipEventCreate(&s->origin) != hipSuccess || hipEventRecord(s->origin, nullptr) != hipSuccess ||
      hipEventSynchronize(s->origin) != hipSuccess) {
    if (s->origin) (void)hipEventDestroy(s->origin);
    s->origin = nullptr;
  }
  for (int i = 0; i < cfg->max_slots; ++i) s->workers.emplace_back(xl::worker, s);
  *out = reinterpret_cast<xl_server*>(s);
  return xl::clear_error();
}

int xl_serve_submit(xl_server* srv, const xl_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket) return xl::set_error(XL_EINVAL, "NULL argument");
  if (req->width < 0 || req->height < 0 || req->n_min < 0 || req->n_max < req->n_min)
    return xl::set_error(XL_EINVAL, "bad image size or samples-per-ray range");
  for (int c = 0; c < 3; ++c)
    if (req->grid[c] < 1) return xl::set_error(XL_EINVAL, "grid dimensions must be >= 1");
  if (static_cast<int64_t>(req->grid[0]) * req->grid[1] * req->grid[2] > 256 ||
      req->grid[0] + req->grid[1] + req->grid[2] > 18)
    return xl::set_error(XL_EINVAL, "grid too large");
  auto* s = reinterpret_cast<xl::Server*>(srv);
  auto j = std::make_shared<xl::Job>();
  j->req = *req;
  j->t_arrival = xl::now_us();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return xl::set_error(XL_EINVAL, "server is shutting down");
  if (static_cast<int64_t>(s->queue.size()) >= s->cfg.max_queue)
    return xl::set_error(XL_EAGAIN, "queue full (%d requests waiting)", s->cfg.max_queue);
  j->ticket = s->next_ticket++;
  if (s->t_first_arrival < 0) s->t_first_arrival = j->t_arrival;
  s->jobs[j->ticket] = j;
  s->queue.push_back(j);
  *ticket = j->ticket;
  s->cv_queue.notify_one();
  return XL_OK;
}

int xl_serve_poll(xl_server* srv, uint64_t ticket, xl_result* out, int64_t timeout_us) {
  if (!srv || !out) return xl::set_error(XL_EINVAL, "NULL argument");
  auto* s = reinterpret_cast<xl::Server*>(srv);
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return xl::set_error(XL_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  std::shared_ptr<xl::Job> j = it->second;
  if (!j->done && timeout_us != 0) {
    if (timeout_us < 0)
      s->cv_done.wait(lk, [&] { return j->done; });
    else
      s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return j->done; });
  }
  std::memset(out, 0, sizeof(*out));
  out->status = j->status;
  out->n_rays = j->n_rays;
  out->n_samples = j->n_samples;
  out->n_segments = j->n_seg;
  out->footprint_bytes = j->footprint;
  if (!j->done) return XL_PENDING;
  out->ray_out = j->ray_out;
  out->latency_us = j->t_done - j->t_arrival;
  out->queue_us = j->t_admit - j->t_arrival;
  out->device_us = static_cast<int64_t>(j->device_ms * 1000.0f);
  out->device_start_us =
      j->device_start_ms < 0 ? -1 : static_cast<int64_t>(j->device_start_ms * 1000.0);
  out->device_end_us = j->device_end_ms < 0 ? -1 : static_cast<int64_t>(j->device_end_ms * 1000.0);
  if (j->status != XL_OK) return xl::set_error(j->status, "request %llu failed: %s",
                                               (unsigned long long)ticket, j->msg);
  return xl::clear_error();
}

int xl_serve_copy_result(xl_server* srv, uint64_t ticket, float* dst, void* stream) {
  if (!srv || !dst) return xl::set_error(XL_EINVAL, "NULL argument");
  auto* s = reinterpret_cast<xl::Server*>(srv);
  std::shared_ptr<xl::Job> j;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end() || !it->second->done || it->second->status != XL_OK)
      return xl::set_error(XL_EINVAL, "ticket %llu has no result", (unsigned long long)ticket);
    j = it->second;
  }
  hipError_t e = hipMemcpyAsync(dst, j->ray_out, sizeof(float) * 7 * j->n_rays,
                                hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
  // The result block may not be reused before this copy has read it.
  std::lock_guard<std::mutex> lk(s->mu);
  if (e == hipSuccess && !j->copied) e = hipEventCreateWithFlags(&j->copied, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(j->copied, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return xl::set_error(XL_EHIP, "copy: %s", hipGetErrorString(e));
  return xl::clear_error();
}

int xl_serve_release(xl_server* srv, uint64_t ticket) {
  if (!srv) return xl::set_error(XL_EINVAL, "NULL server");
  auto* s = reinterpret_cast<xl::Server*>(srv);
  std::shared_ptr<xl::Job> j;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end() || !it->second->done)
      return xl::set_error(XL_EINVAL, "ticket %llu is unknown or not finished", (unsigned long long)ticket);
    j = it->second;
    s->jobs.erase(it);
  }
  hipError_t e = hipSuccess;
  if (j->copied) {
    e = hipEventSynchronize(j->copied);
    (void)hipEventDestroy(j->copied);
    j->copied = nullptr;
  }
  if (j->ray_out) xl::release_block(s, j->arena_off, j->result_bytes);
  if (e != hipSuccess) return xl::set_error(XL_EHIP, "release: %s", hipGetErrorString(e));
  return xl::clear_error();
}

int xl_serve_stats_get(xl_server* srv, xl_serve_stats* out) {
  if (!srv || !out) return xl::set_error(XL_EINVAL, "NULL argument");
  auto* s = reinterpret_cast<xl::Server*>(srv);
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = static_cast<int64_t>(s->queue.size());
  out->samples = s->samples_done;
  out->budget_used_bytes = s->arena.used();
  std::vector<int64_t> v = s->latencies;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto q = [&](double f) {
      const size_t i = std::min(v.size() - 1, static_cast<size_t>(f * (v.size() - 1) + 0.5));
      return v[i];
    };
    out->p50_latency_us = q(0.50);
    out->p99_latency_us = q(0.99);
    out->max_latency_us = v.back();
  }
  if (s->t_first_arrival >= 0) out->span_us = s->t_last_done - s->t_first_arrival;
  return XL_OK;
}

int xl_serve_destroy(xl_server* srv) {
  if (!srv) return xl::set_error(XL_EINVAL, "NULL server");
  auto* s = reinterpret_cast<xl::Server*>(srv);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_queue.notify_all();
    s->cv_budget.notify_all();
  }
  for (auto& t : s->workers) t.join();
  hipError_t e = hipSuccess;
  for (auto& kv : s->jobs) {
    if (kv.second->copied) {
      const hipError_t ec = hipEventSynchronize(kv.second->copied);
      if (e == hipSuccess) e = ec;
      (void)hipEventDestroy(kv.second->copied);
    }
  }
  if (s->origin) (void)hipEventDestroy(s->origin);
  const hipError_t ef = hipFree(s->base);
  if (e == hipSuccess) e = ef;
  delete s;
  if (e != hipSuccess) return xl::set_error(XL_EHIP, "destroy: %s", hipGetErrorString(e));
  return xl::clear_error();
}

}  // extern "C"
