// Serving: continuous batching of independent implicit-step solves behind
// the jfnk_batch_* calls of include/jfnk.h.
//
// Each of the batch's `max_slots` worker threads owns one non-blocking HIP
// stream.  A worker takes the request at the head of the FIFO queue as soon as
// (a) a cached workspace of the same shape is idle, or (b) a new workspace
// fits the device-memory budget after releasing idle workspaces in least
// recently used order.  It then runs the whole Newton solve on its own
// stream, so requests admitted while others are on the device overlap with
// them; when the solve ends the workspace goes back to the cache (or is
// released) and waiting workers re-check the queue head.  Admission is
// strictly first come, first served: a head request that does not fit yet is
// not overtaken, which bounds every request's wait by the work queued before
// it.
//
// Device memory goes back only while nothing runs: a device free waits for
// every stream of the device, so one issued while other slots compute would
// stall them.  Workspaces to be released wait in `doomed` (their bytes still
// counted against the budget); the worker that sees the device idle frees
// them, with admission closed meanwhile.  A head request that needs the room
// of idle cached workspaces waits for the device to go idle first.
//
// A workspace is one jfnk_solver (its GMRES/Newton arrays) plus FP64 device
// arrays for the iterate, the previous state and the optional source; its
// bytes count against the budget from admission until it is released.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "jfnk.h"

namespace {

bool same_shape(const jfnk_problem& a, const jfnk_problem& b) {
  if (a.id != b.id || a.nx != b.nx || a.ny != b.ny) return false;
  if (a.hx != b.hx || a.hy != b.hy || a.dt != b.dt || a.theta != b.theta) return false;
  for (int i = 0; i < 8; ++i)
    if (a.p[i] != b.p[i]) return false;
  return true;
}

struct Workspace {
  jfnk_problem prob{};
  jfnk_solver* s = nullptr;
  double* d_x = nullptr;     // Newton iterate
  double* d_prev = nullptr;  // previous time level
  double* d_src = nullptr;   // source (Kerr)
  size_t n = 0;
  size_t bytes = 0;
};

struct Request {
  long long ticket = 0;
  jfnk_problem prob{};
  jfnk_options opts{};
  std::vector<double> x_prev, source, x_out;
  size_t n = 0;
  size_t footprint = 0;
  int state = 0;  // 0 queued, 1 running, 2 finished
  jfnk_status status = JFNK_OK;
  jfnk_info info{};
  double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
};

size_t workspace_bytes(const jfnk_problem* p, int prec, int m, bool source) {
  const size_t n = jfnk_problem_size(p);
  return jfnk_footprint_bytes(p, prec, m) + (source ? 3 : 2) * n * sizeof(double);
}

}  // namespace

struct jfnk_batch {
  jfnk_batch_config cfg{};
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work;  // queue grew, memory or a workspace was freed, or stop
  std::condition_variable cv_done;  // a request finished
  std::deque<std::shared_ptr<Request>> queue;
  std::map<long long, std::shared_ptr<Request>> reqs;
  std::list<Workspace*> idle;  // front = most recently used
  std::vector<Workspace*> doomed;  // released, freed once no request runs
  bool freeing = false;        // a worker is freeing `doomed`: admission closed
  size_t in_use = 0;           // bytes of every live workspace plus reservations
  long long next_ticket = 1;
  bool stop = false;
  int running = 0;
  jfnk_batch_stats stats{};
  std::vector<std::thread> workers;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

void free_workspace(Workspace* w, hipStream_t st) {
  if (!w) return;
  if (w->s) {
    (void)jfnk_set_stream(w->s, st);
    (void)jfnk_destroy(w->s);
  }
  if (w->d_x) (void)hipFree(w->d_x);
  if (w->d_prev) (void)hipFree(w->d_prev);
  if (w->d_src) (void)hipFree(w->d_src);
  delete w;
}

jfnk_status create_workspace(const jfnk_batch* b, const Request& r, hipStream_t st, Workspace** out) {
  Workspace* w = new Workspace();
  w->prob = r.prob;
  w->n = r.n;
  w->bytes = r.footprint;
  jfnk_status rc = jfnk_create(&r.prob, b->cfg.precision, b->cfg.m, st, &w->s);
  const size_t vb = r.n * sizeof(double);
  if (rc == JFNK_OK && hipMalloc(&w->d_x, vb) != hipSuccess) rc = JFNK_ERR_OOM;
  if (rc == JFNK_OK && hipMalloc(&w->d_prev, vb) != hipSuccess) rc = JFNK_ERR_OOM;
  if (rc == JFNK_OK && !r.source.empty() && hipMalloc(&w->d_src, vb) != hipSuccess) rc = JFNK_ERR_OOM;
  if (rc != JFNK_OK) {
    free_workspace(w, st);
    return rc;
  }
  *out = w;
  return JFNK_OK;
}

// Pinned staging buffer of a worker (grown on demand).
struct Staging {
  double* p = nullptr;
  size_t cap = 0;
  bool reserve(size_t n) {
    if (n <= cap) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    void* q = nullptr;
    if (hipHostMalloc(&q, n * sizeof(double), hipHostMallocDefault) != hipSuccess) return false;
    p = static_cast<double*>(q);
    cap = n;
    return true;
  }
  ~Staging() {
    if (p) (void)hipHostFree(p);
  }
};

jfnk_status run_request(Request& r, Workspace* w, hipStream_t st, Staging& stage) {
  const size_t n = r.n;
  const bool src = !r.source.empty();
  if (!stage.reserve(src ? 2 * n : n)) return JFNK_ERR_OOM;
  if (jfnk_set_stream(w->s, st) != JFNK_OK) return JFNK_ERR_ARG;
  std::memcpy(stage.p, r.x_prev.data(), n * sizeof(double));
  if (src) std::memcpy(stage.p + n, r.source.data(), n * sizeof(double));
  if (hipMemcpyAsync(w->d_prev, stage.p, n * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
    return JFNK_ERR_HIP;
  if (src && hipMemcpyAsync(w->d_src, stage.p + n, n * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
    return JFNK_ERR_HIP;
  if (hipMemcpyAsync(w->d_x, w->d_prev, n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return JFNK_ERR_HIP;
  jfnk_status rc = jfnk_set_previous(w->s, w->d_prev, src ? w->d_src : nullptr);
  if (rc != JFNK_OK) return rc;
  rc = jfnk_newton_solve(w->s, w->d_x, &r.opts, &r.info);
  if (hipMemcpyAsync(stage.p, w->d_x, n * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return JFNK_ERR_HIP;
  r.x_out.assign(stage.p, stage.p + n);
  return rc;
}

void worker_main(jfnk_batch* b) {
  (void)hipSetDevice(b->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  Staging stage;
  for (;;) {
    std::shared_ptr<Request> r;
    Workspace* ws = nullptr;
    bool create = false;
    std::vector<Workspace*> evicted;
    {
      std::unique_lock<std::mutex> lk(b->mu);
      for (;;) {
        if (b->stop) break;
        if (b->running == 0 && !b->freeing && !b->doomed.empty()) {
          // the device is idle: free what was released while others ran
          evicted.swap(b->doomed);
          b->freeing = true;
          break;
        }
        if (!b->queue.empty() && !b->freeing) {
          const std::shared_ptr<Request>& head = b->queue.front();
          auto it = std::find_if(b->idle.begin(), b->idle.end(),
                                 [&](const Workspace* w) { return same_shape(w->prob, head->prob) && w->n == head->n &&
                                                                  (head->source.empty() || w->d_src != nullptr); });
          if (it != b->idle.end()) {
            ws = *it;
            b->idle.erase(it);
          } else if (b->in_use + head->footprint <= b->cfg.budget_bytes) {
            b->in_use += head->footprint;
            create = true;
          } else if (b->running == 0 && !b->idle.empty()) {
            // release least recently used idle workspaces (the device is idle)
            while (b->in_use + head->footprint > b->cfg.budget_bytes && !b->idle.empty()) {
              Workspace* v = b->idle.back();
              b->idle.pop_back();
              b->stats.workspaces_released += 1;
              b->doomed.push_back(v);
            }
            evicted.swap(b->doomed);
            b->freeing = true;
            break;
          }
          if (ws || create) {
            r = head;
            b->queue.pop_front();
            r->state = 1;
            r->t_start = b->now();
            b->running += 1;
            b->stats.max_running = std::max(b->stats.max_running, b->running);
            b->stats.peak_bytes = std::max(b->stats.peak_bytes, b->in_use);
            if (create) b->stats.workspaces_created += 1;
            break;
          }
        }
        b->cv_work.wait(lk);
      }
      if (!r && b->stop && evicted.empty()) break;
    }
    if (!evicted.empty()) {
      // admission is closed and nothing runs: these frees stall no one
      size_t freed = 0;
      for (Workspace* v : evicted) {
        freed += v->bytes;
        free_workspace(v, st);
      }
      {
        std::lock_guard<std::mutex> lk(b->mu);
        if (b->running > 0) b->stats.frees_while_running += 1;
        b->in_use -= freed;
        b->freeing = false;
      }
      b->cv_work.notify_all();
      continue;
    }
    if (!r) continue;

    jfnk_status rc = JFNK_OK;
    if (create) rc = create_workspace(b, *r, st, &ws);
    if (rc == JFNK_OK) rc = run_request(*r, ws, st, stage);
    {
      std::lock_guard<std::mutex> lk(b->mu);
      r->status = rc;
      r->info.status = rc;
      r->state = 2;
      r->t_done = b->now();
      b->running -= 1;
      b->stats.completed += 1;
      if (rc != JFNK_OK && rc != JFNK_ERR_NOT_CONVERGED) b->stats.failed += 1;
      if (ws == nullptr) {
        b->in_use -= r->footprint;  // creation failed: drop the reservation
      } else if (b->cfg.keep_workspaces && rc != JFNK_ERR_HIP) {
        b->idle.push_front(ws);
      } else {
        b->stats.workspaces_released += 1;
        b->doomed.push_back(ws);  // freed once no request runs
      }
    }
    b->cv_done.notify_all();
    b->cv_work.notify_all();
  }
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

jfnk_status jfnk_batch_create(const jfnk_batch_config* cfg, jfnk_batch** out) {
  if (!cfg || !out) return JFNK_ERR_ARG;
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->m < 1 || cfg->m > 32 || cfg->budget_bytes == 0) return JFNK_ERR_ARG;
  if (cfg->precision != JFNK_F64 && cfg->precision != JFNK_F32 && cfg->precision != JFNK_F16S) return JFNK_ERR_ARG;
  jfnk_batch* b = new jfnk_batch();
  b->cfg = *cfg;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return JFNK_ERR_HIP;
  }
  b->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < cfg->max_slots; ++i) b->workers.emplace_back(worker_main, b);
  *out = b;
  return JFNK_OK;
}

jfnk_status jfnk_batch_destroy(jfnk_batch* b) {
  if (!b) return JFNK_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->stop = true;
    for (auto& r : b->queue) {
      r->state = 2;
      r->status = JFNK_ERR_ARG;
      r->t_done = b->now();
    }
    b->queue.clear();
  }
  b->cv_work.notify_all();
  b->cv_done.notify_all();
  for (auto& t : b->workers) t.join();
  hipStream_t st = nullptr;
  for (Workspace* w : b->idle) free_workspace(w, st);
  for (Workspace* w : b->doomed) free_workspace(w, st);
  b->idle.clear();
  b->doomed.clear();
  delete b;
  return JFNK_OK;
}

jfnk_status jfnk_batch_submit(jfnk_batch* b, const jfnk_problem* problem, const double* x_prev,
                              const double* source, const jfnk_options* opts, long long* ticket) {
  if (!b || !problem || !x_prev || !ticket) return JFNK_ERR_ARG;
  const size_t n = jfnk_problem_size(problem);
  if (n == 0) return JFNK_ERR_ARG;
  auto r = std::make_shared<Request>();
  r->prob = *problem;
  r->n = n;
  r->x_prev.assign(x_prev, x_prev + n);
  if (source) r->source.assign(source, source + n);
  if (opts)
    r->opts = *opts;
  else
    jfnk_default_options(b->cfg.precision, &r->opts);
  r->footprint = workspace_bytes(problem, b->cfg.precision, b->cfg.m, source != nullptr);
  if (r->footprint > b->cfg.budget_bytes) return JFNK_ERR_OOM;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->stop) return JFNK_ERR_ARG;
    r->ticket = b->next_ticket++;
    r->t_submit = b->now();
    b->reqs[r->ticket] = r;
    b->queue.push_back(r);
    b->stats.submitted += 1;
    *ticket = r->ticket;
  }
  b->cv_work.notify_all();
  return JFNK_OK;
}

int jfnk_batch_poll(jfnk_batch* b, long long ticket) {
  if (!b) return -1;
  std::lock_guard<std::mutex> lk(b->mu);
  auto it = b->reqs.find(ticket);
  if (it == b->reqs.end()) return -1;
  return it->second->state == 2 ? 1 : 0;
}

jfnk_status jfnk_batch_wait(jfnk_batch* b, long long ticket, double* x_out, jfnk_info* info, double* times) {
  if (!b) return JFNK_ERR_ARG;
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(b->mu);
    auto it = b->reqs.find(ticket);
    if (it == b->reqs.end()) return JFNK_ERR_ARG;
    r = it->second;
    b->cv_done.wait(lk, [&] { return r->state == 2; });
    b->reqs.erase(ticket);
  }
  if (x_out && r->x_out.size() == r->n) std::memcpy(x_out, r->x_out.data(), r->n * sizeof(double));
  if (info) *info = r->info;
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_start;
    times[2] = r->t_done;
  }
  return r->status;
}

double jfnk_batch_clock(const jfnk_batch* b) { return b ? b->now() : 0.0; }

jfnk_status jfnk_batch_get_stats(jfnk_batch* b, jfnk_batch_stats* out) {
  if (!b || !out) return JFNK_ERR_ARG;
  std::lock_guard<std::mutex> lk(b->mu);
  *out = b->stats;
  out->bytes_in_use = b->in_use;
  return JFNK_OK;
}

}  // extern "C"
