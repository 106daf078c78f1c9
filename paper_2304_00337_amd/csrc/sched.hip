// Batched solves and the serving loop of bloch.h (bl_batch_solve, bl_server_*).
//
// Problems are grouped by shape (grid, block width p); each group runs on engines whose
// slots share every kernel launch of a round.  Engines live on streams of their own and
// advance independently (an engine's next round is queued as soon as its previous one has
// drained), so the rounds of different engines overlap on the device: while one engine
// runs its latency-bound steps (the small Ritz problem, reductions, host decisions) the
// others fill the compute units.  A shape whose single problem already fills the device
// with its finest-level launches is therefore spread over up to engine_streams engines rather
// than packed into one; small shapes are packed (their launches need the slots to fill the
// device).  Engines are created under an HBM budget: admission takes a queued problem when
// an engine of its shape has a free slot, or when a new engine fits the budget (idle
// engines of other shapes are released for it).  Later problems may pass a queued one that
// does not fit yet, but at most kPassLimit of them: then nothing else is admitted until it
// is, so the engines drain and the idle ones are released for it (no unbounded wait).
// Slots that finish a problem take the next queued one of their shape at the next round
// (continuous batching); a problem's eigenvector history stays on the device across its
// Bloch parameters.
#include "engine.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

namespace bl {
const char* last_error_message();

namespace {

struct Key {
  int n, m, p;
  double a, b;
  bool operator==(const Key& o) const { return n == o.n && m == o.m && p == o.p && a == o.a && b == o.b; }
};

struct Job {
  Task task;
  Key key{};
  bool published = false;   // serving: results handed to the caller's thread
  int passed = 0;           // later jobs admitted while this one waited for memory
  bool mem_wait = false;    // the last admission attempt failed on the memory budget
};

// Later jobs that may be admitted ahead of a waiting one before admission stops for it.
constexpr int kPassLimit = 4;

struct Eng {
  bl_solver* e = nullptr;
  Key key{};
  hipStream_t st = nullptr;
  size_t bytes = 0;
  bool pending = false;   // a round has been issued and not yet finished
};

// Finest-level unknowns x block width above which one problem fills the device (the
// finest smoother pass then has >= 1000 workgroups for that problem alone).
constexpr int64_t kFillWork = (int64_t)1 << 20;

class Scheduler {
 public:
  Scheduler(const bl_opts& o, size_t budget, int max_slots) : opts_(o), budget_(budget), max_slots_(max_slots) {}
  ~Scheduler() {
    for (auto& g : engines_) release(g);
  }

  void enqueue(Job* j) { queue_.push_back(j); }
  bool idle() const { return queue_.empty() && busy_engines() == 0 && pending_retired() == 0 && !in_flight(); }
  size_t queued() const { return queue_.size(); }
  size_t engines() const { return engines_.size(); }
  size_t bytes_used() const { return used_; }
  int64_t rounds() const { return rounds_; }
  int64_t launches() const {
    int64_t l = launches_done_;
    for (auto& g : engines_) l += g.e->launches;
    return l;
  }

  // Admit queued jobs (FIFO; later jobs may pass one that does not fit the memory budget, at
  // most kPassLimit of them, after which nothing behind it is tried; a job waiting for a slot
  // of its shape's engines gets one as their tasks end and is not counted).  Returns a device error or
  // BL_OK; a job that can never fit ends with BL_ENOMEM.
  int admit() {
    for (auto it = queue_.begin(); it != queue_.end();) {
      Job* j = *it;
      bool blocked = false;   // an older job has been passed over often enough
      for (auto jt = queue_.begin(); jt != it; ++jt)
        if ((*jt)->passed >= kPassLimit) blocked = true;
      if (blocked) break;
      int rc = place(j);
      if (rc == BL_OK) {
        for (auto jt = queue_.begin(); jt != it; ++jt)
          if ((*jt)->mem_wait) (*jt)->passed += 1;
        it = queue_.erase(it);
        continue;
      }
      if (rc == BL_EAGAIN) {
        ++it;
        continue;
      }
      if (rc == BL_EHIP) return rc;
      // task-level failure (invalid input, or larger than the whole budget)
      j->task.status = rc;
      j->task.message = last_error_message();
      j->task.finished = j->task.done = true;
      j->task.t_done = now_seconds();
      it = queue_.erase(it);
    }
    return BL_OK;
  }

  // Smoother timing of every engine (present and future); totals survive engine release.
  int set_timing(bool on) {
    timing_ = on;
    t_ms_ = 0.0;
    t_launches_ = t_cols_ = 0;
    t_bytes_ = 0.0;
    for (auto& g : engines_) {
      int rc = engine_set_timing(g.e, on);
      if (rc) return rc;
    }
    return BL_OK;
  }
  void timing(double* ms, int64_t* launches, int64_t* cols, double* bytes) const {
    *ms = t_ms_;
    *launches = t_launches_;
    *cols = t_cols_;
    *bytes = t_bytes_;
    for (auto& g : engines_) {
      *ms += g.e->timed_ms;
      *launches += g.e->timed_count;
      *cols += g.e->timed_cols;
      *bytes += g.e->timed_bytes;
    }
  }

  int engine_count() const { return (int)engines_.size(); }
  const bl_solver* engine_at(int i) const { return engines_[i].e; }

  // Advance the engines: every busy engine without a round in flight issues one; then wait
  // until at least one engine's stream has drained and finish the rounds of all that have
  // (finishing queues that engine's preconditioner and Ritz step, and the next call issues
  // its next round right behind them).  Engines therefore run out of step with each other.
  int step() {
    int rc;
    bool any = false;
    for (auto& g : engines_) {
      if (g.pending || !engine_busy(g.e)) continue;
      if ((rc = engine_issue(g.e))) return rc;
      g.pending = any = true;
    }
    bool waiting = false;
    for (auto& g : engines_) waiting = waiting || g.pending;
    while (waiting) {
      bool done = false;
      for (auto& g : engines_) {
        if (!g.pending) continue;
        const hipError_t q = hipStreamQuery(g.st);
        if (q == hipErrorNotReady) continue;
        g.pending = false;
        done = true;
        if ((rc = engine_finish(g.e))) return rc;   // reports a failed stream as a device error
      }
      if (done) break;
      std::this_thread::yield();
    }
    for (auto& g : engines_)
      if (!g.pending && !engine_busy(g.e) && !g.e->retired.empty())
        if ((rc = engine_sync_retired(g.e))) return rc;
    if (any) ++rounds_;
    return BL_OK;
  }

 private:
  int busy_engines() const {
    int b = 0;
    for (auto& g : engines_) b += engine_busy(g.e) > 0;
    return b;
  }
  bool in_flight() const {
    for (auto& g : engines_)
      if (g.pending) return true;
    return false;
  }
  int pending_retired() const {
    int r = 0;
    for (auto& g : engines_) r += (int)g.e->retired.size();
    return r;
  }

  void release(Eng& g) {
    launches_done_ += g.e->launches;
    t_ms_ += g.e->timed_ms;
    t_launches_ += g.e->timed_count;
    t_cols_ += g.e->timed_cols;
    t_bytes_ += g.e->timed_bytes;
    engine_destroy(g.e);
    if (g.st) (void)hipStreamDestroy(g.st);
    used_ -= std::min(used_, g.bytes);
    g.e = nullptr;
  }

  bl_opts engine_opts(const Key& k) const {
    bl_opts o = opts_;
    o.nev = k.p;   // each task brings its own nev; the engine only needs the block width
    o.nthrow = 0;
    return o;
  }

  int place(Job* j) {
    j->mem_wait = false;
    for (auto& g : engines_) {
      if (!(g.key == j->key)) continue;
      const int sl = engine_free_slot(g.e);
      if (sl < 0) continue;
      return engine_assign(g.e, sl, &j->task);
    }
    // a new engine: as many slots as the queue holds for this shape, within max_slots and
    // the budget.  At most opts.engine_streams engines per shape (the default of 3 leaves one
    // of the device's four hardware queues per process to the caller); beyond that the job
    // waits for a slot.  A shape that fills the device with one problem shares the queue out
    // over the engines still to be created for it.
    int want = 0, have = 0;
    for (Job* q : queue_) want += q->key == j->key;
    for (auto& g : engines_) have += g.key == j->key;
    if (have >= opts_.engine_streams) return BL_EAGAIN;
    if ((int64_t)j->key.n * j->key.m * j->key.p >= kFillWork) {
      const int spread = std::max(1, opts_.engine_streams - have);
      want = (want + spread - 1) / spread;
    }
    want = std::max(1, std::min(want, max_slots_ > 0 ? max_slots_ : kMaxSlots));
    bl_grid gr{j->key.n, j->key.m, j->key.a, j->key.b};
    bl_opts o = engine_opts(j->key);
    fill_defaults(&o);
    const size_t one = engine_footprint(&gr, &o, 1);
    const size_t per = engine_footprint(&gr, &o, 2) - one;
    if (one > budget_) return set_error(BL_ENOMEM, "problem larger than the memory budget%s");
    // with no engine left to release, a problem that does not fit never will
    auto fits = [&](int k) { return used_ + one + per * (size_t)(k - 1) <= budget_; };
    if (!fits(1)) {
      // release idle engines, least recently created first
      for (auto it = engines_.begin(); it != engines_.end() && !fits(1);) {
        if (!it->pending && engine_busy(it->e) == 0 && it->e->retired.empty()) {
          release(*it);
          it = engines_.erase(it);
        } else {
          ++it;
        }
      }
      if (!fits(1)) {
        if (engines_.empty()) return set_error(BL_ENOMEM, "problem larger than the memory budget%s");
        j->mem_wait = true;
        return BL_EAGAIN;
      }
    }
    while (want > 1 && !fits(want)) --want;
    Eng g;
    g.key = j->key;
    if (hipStreamCreateWithFlags(&g.st, hipStreamNonBlocking) != hipSuccess)
      return set_error(BL_EHIP, "stream creation failed%s");
    int rc = engine_create(&gr, &o, want, g.st, nullptr, &g.e);
    if (rc) {
      (void)hipStreamDestroy(g.st);
      if (rc == BL_ENOMEM && !engines_.empty()) {
        j->mem_wait = true;
        return BL_EAGAIN;
      }
      return rc;
    }
    if (timing_ && (rc = engine_set_timing(g.e, true))) {
      engine_destroy(g.e);
      (void)hipStreamDestroy(g.st);
      return rc;
    }
    g.bytes = g.e->dev_bytes;
    used_ += g.bytes;
    engines_.push_back(g);
    return engine_assign(engines_.back().e, 0, &j->task);
  }

  bl_opts opts_;
  size_t budget_;
  int max_slots_;
  size_t used_ = 0;
  int64_t rounds_ = 0;
  int64_t launches_done_ = 0;
  std::deque<Job*> queue_;
  std::deque<Eng> engines_;
  bool timing_ = false;
  double t_ms_ = 0.0;
  int64_t t_launches_ = 0, t_cols_ = 0;
  double t_bytes_ = 0.0;
};

int make_job(const bl_opts& common, const bl_grid* grid, const double* eps, int nev, int nthrow,
             int nk, const double* ks, const void* start_dev, Job* j) {
  if (!grid || !eps || !ks || nk < 1 || (!start_dev && !common.nested_start))
    return set_error(BL_EINVAL, "invalid problem (grid, eps, ks and a start block, unless nested_start is set, are required)%s");
  bl_opts o = common;
  o.nev = nev;
  o.nthrow = nthrow;
  fill_defaults(&o);
  int rc = validate_opts(&o);
  if (rc) return rc;
  if ((rc = validate_grid(grid, nev + nthrow))) return rc;
  const int64_t nm = (int64_t)grid->n * grid->m;
  if ((rc = validate_eps(eps, nm))) return rc;
  auto lv = hierarchy(grid->n, grid->m, o.levels, o.coarsest_min);
  const Geo gc = make_geo(lv.back().first, lv.back().second, grid->a, grid->b);
  if (gc.ne > kMaxCoarse) return set_error(BL_EINVAL, "grid cannot be coarsened to a small enough level%s");
  for (int t = 0; t < 2 * nk; ++t)
    if (!std::isfinite(ks[t])) return set_error(BL_EINVAL, "non-finite Bloch parameter%s");
  j->key = Key{grid->n, grid->m, nev + nthrow, grid->a, grid->b};
  j->task.kappa.resize(nm);
  double emin = eps[0];
  for (int64_t i = 0; i < nm; ++i) {
    j->task.kappa[i] = 1.0 / eps[i];
    emin = std::min(emin, eps[i]);
  }
  j->task.eps_min = emin;
  j->task.ks.assign(ks, ks + 2 * (size_t)nk);
  j->task.start_dev = start_dev;
  j->task.nev = nev;
  j->task.t_submit = now_seconds();
  return BL_OK;
}

size_t default_budget() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return (size_t)8 << 30;
  return fr / 10 * 9;
}

}  // namespace
}  // namespace bl

using namespace bl;

struct bl_server {
  std::unique_ptr<Scheduler> sched;
  bl_opts opts{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job*> inbox;
  std::vector<Job*> active;   // worker thread only
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  uint64_t next_ticket = 1;
  std::atomic<bool> stop{false};
  int worker_error = BL_OK;
  std::string worker_message;
  std::thread worker;
  // statistics (worker thread writes, read under mu)
  int64_t rounds = 0, launches = 0;
  size_t engines = 0, bytes = 0, queued = 0;
};

namespace {

void server_loop(bl_server* s) {
  (void)hipSetDevice(s->device);
  while (!s->stop.load()) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->sched->idle() && s->inbox.empty())
        s->cv.wait_for(lk, std::chrono::milliseconds(50), [&] { return s->stop.load() || !s->inbox.empty(); });
      while (!s->inbox.empty()) {
        s->sched->enqueue(s->inbox.front());
        s->active.push_back(s->inbox.front());
        s->inbox.pop_front();
      }
    }
    int rc = s->sched->admit();
    if (rc == BL_OK) rc = s->sched->step();
    std::lock_guard<std::mutex> lk(s->mu);
    // hand finished jobs over; the engines hold no reference to them any more
    for (auto it = s->active.begin(); it != s->active.end();) {
      if ((*it)->task.done) {
        (*it)->published = true;
        it = s->active.erase(it);
      } else {
        ++it;
      }
    }
    s->rounds = s->sched->rounds();
    s->launches = s->sched->launches();
    s->engines = s->sched->engines();
    s->bytes = s->sched->bytes_used();
    s->queued = s->sched->queued();
    if (rc != BL_OK) {
      s->worker_error = rc;
      s->worker_message = last_error_message();
      s->stop.store(true);
    }
    s->cv.notify_all();
  }
}

}  // namespace

struct bl_batch {
  bl_opts opts{};
  std::unique_ptr<Scheduler> sched;
};

namespace {

int run_batch(Scheduler& sched, const bl_opts& o, bl_problem* probs, int count, void* stream) {
  if (!probs || count < 1) return set_error(BL_EINVAL, "no problems%s");
  if (stream && hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
    return set_error(BL_EHIP, "caller stream failed%s");
  std::vector<std::unique_ptr<Job>> jobs(count);
  for (int i = 0; i < count; ++i) {
    bl_problem& pb = probs[i];
    jobs[i] = std::make_unique<Job>();
    int rc = make_job(o, &pb.grid, pb.eps, pb.nev, pb.nthrow, pb.nk, pb.ks, pb.start_dev, jobs[i].get());
    if (rc) {
      pb.status = rc;
      jobs[i]->task.finished = jobs[i]->task.done = true;
      jobs[i]->task.status = rc;
      continue;
    }
    jobs[i]->task.evecs_dev = pb.evecs_dev;
    sched.enqueue(jobs[i].get());
  }
  int rc = BL_OK;
  while (!sched.idle()) {
    if ((rc = sched.admit())) break;
    if ((rc = sched.step())) break;
  }
  if (rc) return rc;
  int status = BL_OK;
  for (int i = 0; i < count; ++i) {
    bl_problem& pb = probs[i];
    Task& t = jobs[i]->task;
    if (!t.evals.empty()) {
      const size_t cnt = (size_t)pb.nk * pb.nev;
      if (pb.evals) std::memcpy(pb.evals, t.evals.data(), cnt * 8);
      if (pb.relres) std::memcpy(pb.relres, t.relres.data(), cnt * 8);
      if (pb.iters) std::memcpy(pb.iters, t.iters.data(), (size_t)pb.nk * 4);
      if (pb.point_ms)
        for (int k = 0; k < pb.nk; ++k)
          pb.point_ms[k] = k < (int)t.t_points.size()
                               ? (t.t_points[k] - (k ? t.t_points[k - 1] : t.t_start)) * 1e3 : 0.0;
    }
    pb.status = t.status;
    if (t.status != BL_OK && status == BL_OK) status = t.status;
  }
  if (status != BL_OK) return set_error(status, "at least one problem failed (see bl_problem.status)%s");
  return BL_OK;
}

}  // namespace

extern "C" {

int bl_batch_solve(const bl_opts* opts, bl_problem* probs, int32_t count, int32_t max_slots,
                   void* stream) {
  bl_opts o;
  if (opts) o = *opts; else bl_default_opts(&o, 8);
  fill_defaults(&o);
  Scheduler sched(o, default_budget(), max_slots);
  return run_batch(sched, o, probs, count, stream);
}

int bl_batch_create(const bl_opts* opts, int32_t max_slots, size_t hbm_budget, bl_batch** out) {
  if (!out) return set_error(BL_EINVAL, "out is NULL%s");
  *out = nullptr;
  bl_batch* b = new (std::nothrow) bl_batch();
  if (!b) return set_error(BL_ENOMEM, "host allocation failed%s");
  if (opts) b->opts = *opts; else bl_default_opts(&b->opts, 8);
  fill_defaults(&b->opts);
  b->sched = std::make_unique<Scheduler>(b->opts, hbm_budget ? hbm_budget : default_budget(), max_slots);
  *out = b;
  return BL_OK;
}

int bl_batch_run(bl_batch* b, bl_problem* probs, int32_t count, void* stream) {
  if (!b) return set_error(BL_EINVAL, "batch is NULL%s");
  return run_batch(*b->sched, b->opts, probs, count, stream);
}

void bl_batch_destroy(bl_batch* b) { delete b; }

int bl_batch_engine_info(const bl_batch* b, int32_t index, bl_info* out) {
  if (!b || !out) return set_error(BL_EINVAL, "NULL argument%s");
  if (index < 0) return set_error(BL_EINVAL, "negative index%s");
  if (index >= b->sched->engine_count()) return b->sched->engine_count();
  fill_info(b->sched->engine_at(index), out);
  return b->sched->engine_count();
}

int bl_batch_set_timing(bl_batch* b, int32_t enable) {
  if (!b) return set_error(BL_EINVAL, "batch is NULL%s");
  return b->sched->set_timing(enable != 0);
}

int bl_batch_get_timing(const bl_batch* b, double* total_ms, int64_t* launches, int64_t* columns,
                        double* alg_bytes) {
  if (!b || !total_ms || !launches || !columns || !alg_bytes) return set_error(BL_EINVAL, "NULL argument%s");
  b->sched->timing(total_ms, launches, columns, alg_bytes);
  return BL_OK;
}

int bl_server_create(const bl_opts* opts, size_t hbm_budget, int32_t max_slots, bl_server** out) {
  if (!out) return set_error(BL_EINVAL, "out is NULL%s");
  *out = nullptr;
  bl_opts o;
  if (opts) o = *opts; else bl_default_opts(&o, 8);
  fill_defaults(&o);
  bl_server* s = new (std::nothrow) bl_server();
  if (!s) return set_error(BL_ENOMEM, "host allocation failed%s");
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return set_error(BL_EHIP, "no HIP device%s");
  }
  s->opts = o;
  s->sched = std::make_unique<Scheduler>(o, hbm_budget ? hbm_budget : default_budget(), max_slots);
  s->worker = std::thread(server_loop, s);
  *out = s;
  return BL_OK;
}

int bl_server_submit(bl_server* s, const bl_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return set_error(BL_EINVAL, "NULL argument%s");
  auto j = std::make_unique<Job>();
  int rc = make_job(s->opts, &r->grid, r->eps, r->nev, r->nthrow, r->nk, r->ks, r->start_dev, j.get());
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop.load()) return set_error(s->worker_error ? s->worker_error : BL_ESTATE, "server stopped: %s", s->worker_message.c_str());
  *ticket = s->next_ticket++;
  j->task.id = (int64_t)*ticket;
  s->inbox.push_back(j.get());
  s->jobs[*ticket] = std::move(j);
  s->cv.notify_all();
  return BL_OK;
}

int bl_server_poll(bl_server* s, uint64_t ticket, double* evals, double* relres, int32_t* iters,
                   bl_request_info* info) {
  if (!s) return set_error(BL_EINVAL, "server is NULL%s");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return set_error(BL_EINVAL, "unknown ticket%s");
  Task& t = it->second->task;
  if (!it->second->published) {
    if (s->stop.load()) return set_error(s->worker_error ? s->worker_error : BL_ESTATE, "server stopped: %s", s->worker_message.c_str());
    return BL_EAGAIN;
  }
  const int nk = (int)(t.ks.size() / 2);
  if (!t.evals.empty()) {
    if (evals) std::memcpy(evals, t.evals.data(), (size_t)nk * t.nev * 8);
    if (relres) std::memcpy(relres, t.relres.data(), (size_t)nk * t.nev * 8);
    if (iters) std::memcpy(iters, t.iters.data(), (size_t)nk * 4);
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = t.status;
    int tot = 0;
    for (int v : t.iters) tot += v;
    info->total_iters = tot;
    info->queue_s = t.t_start > 0 ? t.t_start - t.t_submit : 0.0;
    info->run_s = t.t_start > 0 ? t.t_done - t.t_start : 0.0;
    info->latency_s = t.t_done - t.t_submit;
  }
  const int st = t.status;
  s->jobs.erase(it);
  return st;
}

int bl_server_stats(bl_server* s, bl_server_counters* out) {
  if (!s || !out) return set_error(BL_EINVAL, "NULL argument%s");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->rounds = s->rounds;
  out->kernel_launches = s->launches;
  out->engines = (int32_t)s->engines;
  out->queued = (int32_t)(s->queued + s->inbox.size());
  out->device_bytes = s->bytes;
  out->pending = (int32_t)s->jobs.size();
  return s->worker_error;
}

void bl_server_destroy(bl_server* s) {
  if (!s) return;
  s->stop.store(true);
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->sched.reset();
  delete s;
}

}  // extern "C"
