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
//   * max_slots worker threads, each owning one HIP stream (default priority),
//     take requests in arrival order.  A worker first runs the generator's plan
//     phase, which fixes the request's exact HBM footprint (samples, segment
//     arrays, tuples, workspaces, result), then waits until the footprint fits
//     into the byte budget next to the requests already in flight, allocates
//     stream-ordered memory and launches generation, segment composite and
//     merge.  Requests therefore join while others are on the GPU as soon as a
//     slot and memory free up, and the kernels of different requests overlap
//     on the device.
//   * Each request has its own buffers and runs the same kernels, so its result
//     does not depend on what else is in flight (bit for bit).
//   * xl_serve_poll waits for a ticket (bounded by a timeout) and reports the
//     result, its latency (completion minus arrival, host monotonic clock) and
//     its device time; xl_serve_release frees the result buffer.
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
  int64_t n_rays = 0, n_samples = 0, n_seg = 0;
  uint64_t footprint = 0, result_bytes = 0;
  float device_ms = 0.f;
  char msg[160] = "";
};

struct Server {
  xl_serve_config cfg{};
  std::mutex mu;
  std::condition_variable cv_queue, cv_done, cv_budget;
  std::deque<std::shared_ptr<Job>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
  std::vector<std::thread> workers;
  hipStream_t release_stream = nullptr;
  uint64_t budget_used = 0;
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

static void run_job(Server* s, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                    const std::shared_ptr<Job>& j) {
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

  const size_t ws_b = round256(gen_workspace_bytes(&p));
  void* ws = nullptr;
  if (hipMallocAsync(&ws, ws_b, st) != hipSuccess) {
    finish(s, j, XL_ENOMEM, "generator workspace allocation failed");
    return;
  }
  int64_t n = 0, n_seg = 0;
  int overflow = 0;
  if (gen_plan(&p, ws, st, &n, &n_seg, &overflow) != hipSuccess || overflow) {
    (void)hipFreeAsync(ws, st);  // cleanup on a path that already reports failure
    (void)hipStreamSynchronize(st);
    finish(s, j, XL_EHIP, "generator plan failed");
    return;
  }
  j->n_samples = n;
  j->n_seg = n_seg;
  const size_t b_sigma = round256(n * es), b_rgb = round256(3 * n * es), b_t = round256(4 * n);
  const size_t b_off = round256(8 * (n_seg + 1)), b_ro = round256(8 * (p.n_rays + 1));
  const size_t b_ids = round256(8 * n_seg), b_seg = round256(4 * 7 * n_seg);
  const size_t b_rec = round256(xl_segments_workspace_bytes(n));
  const size_t b_out = round256(4 * 7 * p.n_rays);
  const uint64_t fp = ws_b + b_sigma + b_rgb + 2 * b_t + b_off + b_ro + b_ids + b_seg + b_rec + b_out;
  j->footprint = fp;
  j->result_bytes = b_out;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (fp > s->cfg.hbm_budget_bytes) {
      lk.unlock();
      (void)hipFreeAsync(ws, st);
      (void)hipStreamSynchronize(st);
      char m[160];
      std::snprintf(m, sizeof(m), "request needs %llu bytes, budget is %llu",
                    static_cast<unsigned long long>(fp),
                    static_cast<unsigned long long>(s->cfg.hbm_budget_bytes));
      finish(s, j, XL_ENOMEM, m);
      return;
    }
    s->cv_budget.wait(lk, [&] { return s->stop || s->budget_used + fp <= s->cfg.hbm_budget_bytes; });
    s->budget_used += fp;
  }
  char* big = nullptr;
  const size_t b_tmp = b_sigma + b_rgb + 2 * b_t + b_off + b_ids + b_seg + b_rec;
  void* out = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&big), b_tmp, st);
  if (e == hipSuccess) e = hipMallocAsync(&out, b_out, st);
  int64_t* ro = nullptr;
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&ro), b_ro, st);
  if (e != hipSuccess) {
    if (big) (void)hipFreeAsync(big, st);
    if (out) (void)hipFreeAsync(out, st);
    (void)hipFreeAsync(ws, st);
    (void)hipStreamSynchronize(st);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->budget_used -= fp;
      s->cv_budget.notify_all();
    }
    finish(s, j, XL_ENOMEM, "request buffer allocation failed");
    return;
  }
  char* c = big;
  void* sigma = c; c += b_sigma;
  void* rgb = c; c += b_rgb;
  float* t0 = reinterpret_cast<float*>(c); c += b_t;
  float* t1 = reinterpret_cast<float*>(c); c += b_t;
  int64_t* off = reinterpret_cast<int64_t*>(c); c += b_off;
  int64_t* ids = reinterpret_cast<int64_t*>(c); c += b_ids;
  float* seg_out = reinterpret_cast<float*>(c); c += b_seg;
  TileRec* recs = reinterpret_cast<TileRec*>(c);

  e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = gen_fill(&p, dtype, ws, n_seg, sigma, rgb, t0, t1, off, ro, ids, st);
  SamplesDev sd{dtype, sigma, rgb, t0, t1, n};
  if (e == hipSuccess) e = launch_segments_fwd(sd, off, n_seg, seg_out, recs, st);
  if (e == hipSuccess)
    e = launch_merge_fwd(seg_out, n_seg, ro, ids, p.n_rays, static_cast<float*>(out),
                         s->cfg.merge_fp64 != 0, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  hipError_t ef = hipFreeAsync(big, st);
  if (ef == hipSuccess) ef = hipFreeAsync(ro, st);
  if (ef == hipSuccess) ef = hipFreeAsync(ws, st);
  if (e == hipSuccess) e = ef;
  const hipError_t es2 = hipStreamSynchronize(st);
  float ms = 0.f;
  if (e == hipSuccess && es2 == hipSuccess && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 0.f;
  j->device_ms = ms;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->budget_used -= fp - b_out;  // the result stays charged until released
    s->cv_budget.notify_all();
  }
  if (e != hipSuccess || es2 != hipSuccess) {
    (void)hipFreeAsync(out, st);
    (void)hipStreamSynchronize(st);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->budget_used -= b_out;
      s->cv_budget.notify_all();
    }
    finish(s, j, XL_EHIP, hipGetErrorString(e != hipSuccess ? e : es2));
    return;
  }
  j->ray_out = static_cast<float*>(out);
  finish(s, j, XL_OK, nullptr);
}

static void worker(Server* s) {
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // A slot whose stream or events cannot be made fails every request it takes.
  const bool ready = hipSetDevice(s->cfg.device) == hipSuccess &&
                     hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
                     hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
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
    if (ready)
      run_job(s, st, e0, e1, j);
    else
      finish(s, j, XL_EHIP, "serving slot has no stream or events");
  }
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
  if (cfg->dtype != XL_F32 && cfg->dtype != XL_BF16 && cfg->dtype != XL_F16)
    return xl::set_error(XL_EINVAL, "unknown sample dtype %d", cfg->dtype);
  hipError_t e = hipSetDevice(cfg->device);
  if (e != hipSuccess) return xl::set_error(XL_EHIP, "device %d: %s", cfg->device, hipGetErrorString(e));
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, cfg->device) == hipSuccess) {
    // Keep freed request buffers in the pool (a performance hint only).
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  auto* s = new xl::Server();
  s->cfg = *cfg;
  e = hipStreamCreateWithFlags(&s->release_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    return xl::set_error(XL_EHIP, "release stream: %s", hipGetErrorString(e));
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
  const hipError_t e = hipMemcpyAsync(dst, j->ray_out, sizeof(float) * 7 * j->n_rays,
                                      hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
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
  if (j->ray_out) {
    hipError_t e = hipFreeAsync(j->ray_out, s->release_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->release_stream);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->budget_used -= j->result_bytes;
      s->cv_budget.notify_all();
    }
    if (e != hipSuccess) return xl::set_error(XL_EHIP, "release: %s", hipGetErrorString(e));
  }
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
  out->budget_used_bytes = s->budget_used;
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
  for (auto& kv : s->jobs)
    if (kv.second->ray_out && e == hipSuccess) e = hipFreeAsync(kv.second->ray_out, s->release_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->release_stream);
  (void)hipStreamDestroy(s->release_stream);
  delete s;
  if (e != hipSuccess) return xl::set_error(XL_EHIP, "destroy: %s", hipGetErrorString(e));
  return xl::clear_error();
}

}  // extern "C"
