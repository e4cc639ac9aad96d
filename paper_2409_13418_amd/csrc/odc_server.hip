// Serving loop of libodc.so (include/odc.h, odc_server_*): continuous
// batching of meshing jobs on one GPU.
//
// Requests are queued by odc_server_submit.  A scheduler thread owns a few
// lanes, each an extraction context with its own stream.  Whenever a lane is
// idle it takes queued jobs (in the configured order) as long as their
// device scratch fits in what is free of one arena of hbm_budget_bytes
// (admission by footprint) and the batch stays within its size limits, and
// launches them as one job-major batch; the launch itself runs outside the
// server lock.  Jobs that arrive while other
// batches run are admitted as soon as a lane and arena memory free up, so
// their work overlaps on the device.  Every job's bit sets and active sets
// live in its arena block for the job's lifetime; only the 64-byte counts
// record of each job travels to the host.  A job whose active sets outgrow
// the capacity it was planned with goes back to the head of the queue with
// the capacity it needed.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "odc_context.h"

using namespace odc;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one device allocation; blocks are 256-byte
// aligned and coalesce on release.
class Arena {
 public:
  void reset(size_t cap) {
    cap_ = cap;
    used_ = peak_ = 0;
    free_.clear();
    if (cap) free_[0] = cap;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  void clear_peak() { peak_ = used_; }

 private:
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  double cost = 0.0;  // estimated work, for the SHORTEST policy
  odc_field field;
  odc_params params;
  odc_mesh_buffers out;
  int cap_edges = 0;
  bool guard_full = false;
  size_t bytes = 0;  // planned scratch
  size_t off = 0;    // arena block while admitted
  bool done = false;
  odc_request_result res;
};

struct Lane {
  odc_context* ctx = nullptr;
  hipEvent_t done = nullptr;
  std::vector<Request*> batch;
};

double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

}  // namespace

struct odc_server {
  int device = 0;
  std::string err;
  LaunchCfg cfg;
  odc_server_config conf;
  Clock::time_point t0;
  void* arena_base = nullptr;
  Arena arena;
  double cap_scale = 1.0;
  std::vector<Lane> lanes;

  std::mutex mu;
  std::condition_variable cv_work;  // submissions, stop
  std::condition_variable cv_done;  // completions
  std::thread thread;
  bool stop = false;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, Request*> reqs;  // until odc_server_wait releases them
  uint64_t next_ticket = 1;

  // statistics since the last reset
  double stats_t0 = 0.0, last_done = 0.0;
  std::vector<double> lat;
  int64_t submitted = 0, completed = 0, failed = 0, batches = 0, cells = 0;
};

static int32_t sfail(odc_server* s, int32_t code, const char* fmt, ...) {
  if (s) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    s->err = buf;
  }
  return code;
}

// Completion of one request (lock held).
static void finish_request(odc_server* s, Request* r, int32_t status) {
  r->res.status = status;
  r->res.done_ms = ms_since(s->t0);
  r->done = true;
  if (r->res.submit_ms < s->stats_t0) return;  // submitted before the statistics window
  if (status == ODC_OK) {
    ++s->completed;
    s->cells += r->res.counts.n_active_cells;
    s->lat.push_back(r->res.done_ms - r->res.submit_ms);
    s->last_done = r->res.done_ms;
  } else {
    ++s->failed;
  }
}

// Collects a finished lane (lock held).
static void collect(odc_server* s, Lane& L, hipError_t ev) {
  std::vector<Request*> requeue;
  for (size_t k = 0; k < L.batch.size(); ++k) {
    Request* r = L.batch[k];
    s->arena.release(r->off, r->bytes);
    if (ev != hipSuccess) {
      s->err = std::string("batch failed: ") + hipGetErrorString(ev);
      finish_request(s, r, ODC_ERR_HIP);
      continue;
    }
    fill_counts(L.ctx, (int)k, &r->res.counts);
    if (job_overflowed(L.ctx, (int)k)) {
      bool gover = false;
      const int need = needed_edges(L.ctx, (int)k, &gover);
      const int N = r->params.res;
      const double est = 12.0 * N * N + 4096.0;
      if (need > est * s->cap_scale) s->cap_scale = need / est;
      r->cap_edges = std::max(r->cap_edges, need);
      r->guard_full = r->guard_full || gover;
      r->bytes = job_scratch_bytes(&r->field, &r->params, r->cap_edges, r->guard_full);
      if (r->res.attempts >= 3 || r->bytes > s->arena.capacity()) {
        s->err = "job scratch outgrew the arena";
        finish_request(s, r, ODC_ERR_OUT_OF_MEMORY);
      } else {
        requeue.push_back(r);
      }
      continue;
    }
    const bool fits = r->res.counts.n_vertices <= r->out.cap_vertices &&
                      r->res.counts.n_triangles <= r->out.cap_triangles;
    finish_request(s, r, fits ? ODC_OK : ODC_ERR_CAPACITY);
  }
  for (auto it = requeue.rbegin(); it != requeue.rend(); ++it) s->queue.push_front(*it);
  L.batch.clear();
  s->cv_done.notify_all();
}

// Estimated work of a job in arbitrary units: grid corners plus the queries
// of the searches on the ~6 N^2 crossing edges of a typical surface (61 per
// edge), an MLP query costing ~100 analytic ones.
static double job_cost(const odc_field& f, const odc_params& p) {
  const double n = p.res, n1 = n + 1.0;
  const double queries = n1 * n1 * n1 + 61.0 * 6.0 * n * n;
  return f.kind == ODC_FIELD_MLP ? 100.0 * queries : queries;
}

// Picks queued jobs for an idle lane and reserves their arena blocks (lock
// held): in arrival order (FIFO), or cheapest first with aged jobs ahead of
// all (SHORTEST, BANDED; BANDED also leaves out jobs estimated at more than
// `band` times the batch's first job).  The picked jobs leave the queue.
static std::vector<Request*> pick(odc_server* s) {
  std::vector<Request*> batch;
  int64_t corners = 0;
  std::vector<size_t> order(s->queue.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  const double now = ms_since(s->t0);
  if (s->conf.policy != ODC_SERVE_FIFO) {
    auto aged = [&](const Request* r) { return now - r->res.submit_ms > s->conf.age_ms; };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
      const Request* ra = s->queue[a];
      const Request* rb = s->queue[b];
      const bool ga = aged(ra), gb = aged(rb);
      if (ga != gb) return ga;       // aged jobs first, in arrival order
      if (ga) return a < b;
      return ra->cost < rb->cost;    // then the cheapest
    });
  }
  std::vector<size_t> taken;
  for (size_t i : order) {
    if ((int)batch.size() >= s->conf.max_batch) break;
    Request* r = s->queue[i];
    const int64_t n1 = r->params.res + 1;
    const int64_t c = n1 * n1 * n1;
    const bool fifo = s->conf.policy == ODC_SERVE_FIFO;
    const bool must = fifo || now - r->res.submit_ms > s->conf.age_ms;
    if (!batch.empty() && corners + c > s->conf.max_batch_corners) {
      if (must) break;
      continue;
    }
    if (s->conf.policy == ODC_SERVE_BANDED && !must && !batch.empty() &&
        r->cost > (double)s->conf.band * batch.front()->cost)
      continue;
    if (!s->arena.alloc(r->bytes, &r->off)) {
      if (must) break;  // wait for memory rather than pass this job
      continue;
    }
    corners += c;
    batch.push_back(r);
    taken.push_back(i);
  }
  std::sort(taken.begin(), taken.end());
  for (auto it = taken.rbegin(); it != taken.rend(); ++it) s->queue.erase(s->queue.begin() + *it);
  for (Request* r : batch) {
    r->res.admit_ms = now;
    ++r->res.attempts;
  }
  return batch;
}

// Sets up and launches the lane's picked batch (odc_mesh_extract_batch
// semantics) without the server lock: host job records, uploads and kernel
// launches touch only the lane's own context and the jobs' arena blocks,
// which no other thread uses while the batch is in flight, so submit, poll
// and wait are never held up by them.
static int32_t launch_lane(odc_server* s, Lane& L, std::string* why) {
  const int n = (int)L.batch.size();
  if ((int)L.ctx->slots.size() < n) L.ctx->slots.resize(n);
  std::vector<odc_field> f(n);
  std::vector<odc_params> p(n);
  std::vector<odc_mesh_buffers> o(n);
  for (int k = 0; k < n; ++k) {
    const Request* r = L.batch[k];
    Slot& S = L.ctx->slots[k];
    S.ext = (char*)s->arena_base + r->off;
    S.ext_bytes = r->bytes;
    S.ext_cap_edges = r->cap_edges;
    S.guard_full = r->guard_full;
    f[k] = r->field;
    p[k] = r->params;
    o[k] = r->out;
  }
  int32_t rc = enqueue_batch(L.ctx, n, f.data(), p.data(), o.data());
  if (rc != ODC_OK) {
    *why = L.ctx->err;
    return rc;
  }
  const hipError_t he = hipEventRecord(L.done, L.ctx->stream);
  if (he != hipSuccess) {
    *why = hipGetErrorString(he);
    return ODC_ERR_HIP;
  }
  return ODC_OK;
}

static void scheduler(odc_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    bool busy = false, progressed = false;
    for (Lane& L : s->lanes) {
      if (L.batch.empty()) continue;
      const hipError_t e = hipEventQuery(L.done);
      if (e == hipErrorNotReady) {
        busy = true;
        continue;
      }
      collect(s, L, e);
      progressed = true;
    }
    for (Lane& L : s->lanes) {
      if (!L.batch.empty() || s->queue.empty()) continue;
      L.batch = pick(s);
      if (L.batch.empty()) continue;
      std::string why;
      lk.unlock();
      const int32_t rc = launch_lane(s, L, &why);
      lk.lock();
      if (rc != ODC_OK) {
        s->err = why;
        for (Request* r : L.batch) {
          s->arena.release(r->off, r->bytes);
          finish_request(s, r, rc);
        }
        L.batch.clear();
        s->cv_done.notify_all();
        continue;
      }
      ++s->batches;
      busy = progressed = true;
    }
    if (progressed) continue;
    if (busy)
      s->cv_work.wait_for(lk, std::chrono::microseconds(50));
    else
      s->cv_work.wait(lk);
  }
  // drain: wait for the batches in flight so no kernel outlives the arena
  for (Lane& L : s->lanes)
    if (!L.batch.empty()) collect(s, L, hipEventSynchronize(L.done));
}

extern "C" const char* odc_server_last_error(const odc_server* s) {
  return s ? s->err.c_str() : "no server";
}

extern "C" void odc_server_destroy(odc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  if (s->thread.joinable()) s->thread.join();
  (void)hipSetDevice(s->device);
  for (Lane& L : s->lanes) {
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.ctx) odc_context_destroy(L.ctx);
  }
  if (s->arena_base) (void)hipFree(s->arena_base);
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
}

extern "C" int32_t odc_server_create(odc_context* ctx, const odc_server_config* cfg,
                                     odc_server** out) {
  if (!out) return ODC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!ctx || !cfg) return ODC_ERR_INVALID_ARG;
  odc_server_config c = *cfg;
  if (c.n_lanes == 0) c.n_lanes = 2;
  if (c.max_batch == 0) c.max_batch = 16;
  if (c.max_batch_corners == 0) c.max_batch_corners = (int64_t)1 << 25;
  if (c.age_ms == 0.0f) c.age_ms = 1000.0f;
  if (c.band == 0.0f) c.band = 8.0f;
  if (c.hbm_budget_bytes < (1 << 20) || c.n_lanes < 1 || c.n_lanes > 8 || c.max_batch < 1 ||
      c.max_batch > kMaxJobs || c.max_batch_corners < 1 ||
      (c.policy != ODC_SERVE_FIFO && c.policy != ODC_SERVE_SHORTEST &&
       c.policy != ODC_SERVE_BANDED) ||
      !(c.age_ms > 0.0f) || !(c.band > 1.0f))
    return ctx_fail(ctx, ODC_ERR_INVALID_ARG,
                    "server needs a budget >= 1 MiB, 1..8 lanes, 1..%d jobs per batch, "
                    "a known policy and age_ms > 0",
                    kMaxJobs);
  odc_server* s = new odc_server();
  s->device = ctx->device;
  s->cfg = ctx->cfg;
  s->conf = c;
  s->t0 = Clock::now();
  int32_t rc = ODC_OK;
  if (hipSetDevice(s->device) != hipSuccess ||
      device_alloc(&s->arena_base, (size_t)c.hbm_budget_bytes) != hipSuccess) {
    (void)hipGetLastError();
    s->arena_base = nullptr;
    rc = ctx_fail(ctx, ODC_ERR_OUT_OF_MEMORY, "arena of %lld bytes could not be allocated",
                  (long long)c.hbm_budget_bytes);
  }
  if (rc == ODC_OK) {
    s->arena.reset((size_t)c.hbm_budget_bytes);
    s->lanes.resize(c.n_lanes);
    for (Lane& L : s->lanes) {
      rc = odc_context_create(s->device, nullptr, &L.ctx);
      if (rc != ODC_OK) {
        ctx_fail(ctx, rc, "lane context: %s", odc_status_string(rc));
        break;
      }
      L.ctx->cfg = s->cfg;
      if (hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
        rc = ctx_fail(ctx, ODC_ERR_HIP, "event creation failed");
        break;
      }
    }
  }
  if (rc != ODC_OK) {
    odc_server_destroy(s);
    return rc;
  }
  s->thread = std::thread(scheduler, s);
  *out = s;
  return ODC_OK;
}

extern "C" int32_t odc_server_footprint(odc_server* s, const odc_field* f, const odc_params* p,
                                        int64_t* bytes) {
  if (!s || !bytes) return ODC_ERR_INVALID_ARG;
  odc_mesh_buffers o;
  memset(&o, 0, sizeof(o));
  odc_context tmp;  // receives the validation message only
  const int32_t rc = validate_job(&tmp, f, p, &o);
  if (rc != ODC_OK) return sfail(s, rc, "%s", tmp.err.c_str());
  std::lock_guard<std::mutex> lk(s->mu);
  *bytes = (int64_t)job_scratch_bytes(f, p, estimate_edges(s->cap_scale, p->res), false);
  return ODC_OK;
}

extern "C" int32_t odc_server_submit(odc_server* s, const odc_field* f, const odc_params* p,
                                     const odc_mesh_buffers* o, uint64_t* ticket) {
  if (!s || !ticket) return ODC_ERR_INVALID_ARG;
  odc_context tmp;
  int32_t rc = validate_job(&tmp, f, p, o);
  if (rc != ODC_OK) return sfail(s, rc, "%s", tmp.err.c_str());
  Request* r = new Request();
  r->field = *f;
  r->params = *p;
  r->out = *o;
  memset(&r->res, 0, sizeof(r->res));
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->cap_edges = estimate_edges(s->cap_scale, p->res);
    r->bytes = job_scratch_bytes(f, p, r->cap_edges, false);
    r->cost = job_cost(*f, *p);
    if (r->bytes > s->arena.capacity()) {
      const size_t need = r->bytes;
      delete r;
      return sfail(s, ODC_ERR_OUT_OF_MEMORY, "job needs %zu bytes of scratch, the arena has %zu",
                   need, s->arena.capacity());
    }
    r->ticket = s->next_ticket++;
    r->res.submit_ms = ms_since(s->t0);
    s->reqs[r->ticket] = r;
    s->queue.push_back(r);
    ++s->submitted;
    *ticket = r->ticket;
  }
  s->cv_work.notify_one();
  return ODC_OK;
}

extern "C" int32_t odc_server_poll(odc_server* s, uint64_t ticket, int32_t* done) {
  if (!s || !done) return ODC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return sfail(s, ODC_ERR_INVALID_ARG, "unknown ticket %llu",
                                        (unsigned long long)ticket);
  *done = it->second->done ? 1 : 0;
  return ODC_OK;
}

extern "C" int32_t odc_server_wait(odc_server* s, uint64_t ticket, odc_request_result* res) {
  if (!s || !res) return ODC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return sfail(s, ODC_ERR_INVALID_ARG, "unknown ticket %llu",
                                        (unsigned long long)ticket);
  Request* r = it->second;
  s->cv_done.wait(lk, [&] { return r->done || s->stop; });
  if (!r->done) return sfail(s, ODC_ERR_INVALID_ARG, "server stopped");
  *res = r->res;
  s->reqs.erase(it);
  delete r;
  return ODC_OK;
}

extern "C" int32_t odc_server_get_stats(odc_server* s, odc_server_stats* st) {
  if (!s || !st) return ODC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  memset(st, 0, sizeof(*st));
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->failed = s->failed;
  st->queued = (int64_t)s->queue.size();
  for (const Lane& L : s->lanes) st->in_flight += (int64_t)L.batch.size();
  st->batches = s->batches;
  st->active_cells = s->cells;
  if (!s->lat.empty()) {
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    // nearest-rank percentiles
    auto rank = [&](double q) {
      size_t i = (size_t)std::ceil(q * (double)v.size());
      return v[i == 0 ? 0 : i - 1];
    };
    st->p50_ms = rank(0.50);
    st->p99_ms = rank(0.99);
    double sum = 0.0;
    for (double x : v) sum += x;
    st->mean_ms = sum / (double)v.size();
    st->max_ms = v.back();
    st->window_s = (s->last_done - s->stats_t0) / 1000.0;
    if (st->window_s > 0.0) st->cells_per_s = (double)s->cells / st->window_s;
  }
  st->arena_bytes = (int64_t)s->arena.capacity();
  st->arena_peak_bytes = (int64_t)s->arena.peak();
  return ODC_OK;
}

extern "C" int32_t odc_server_reset_stats(odc_server* s) {
  if (!s) return ODC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->stats_t0 = ms_since(s->t0);
  s->last_done = s->stats_t0;
  s->lat.clear();
  s->submitted = s->completed = s->failed = s->batches = s->cells = 0;
  // requests already queued or running count from here on only as load
  s->arena.clear_peak();
  return ODC_OK;
}
