// Continuous-batching job server for evolution jobs (the served form).
//
// Jobs (grid, physics, precision, end time) are submitted as they arrive and
// wait in a FIFO queue; a job whose parameters admit no initial data is
// refused at submission.  Jobs of one grid class (grid sizes, precision,
// kernel parameters: grmhd::same_step_class) advance together, one launch per
// kernel for the whole class (grmhd_step_batch), each class on a stream of
// its own.  Classes do not wait for one another: every tick
//   1. completion: each class's launched RK4 steps are checked with their
//      events (hipEventQuery); a completed step counts for the jobs it
//      carried, and jobs at their end time retire (latency = completion
//      minus arrival on the server clock; optionally the final state is kept
//      on the host) and free their block;
//   2. admission: queued jobs are placed, in arrival order, into the caller's
//      device arena (first fit, 256-byte aligned blocks holding the job's
//      resident and scratch buffers) as long as they fit the budget, at most
//      four per tick (a burst is admitted while the device works); an
//      admitted job gets its context and initial data on the server's
//      admission stream, a time step dt = T / ceil(T / dt_CFL) so that it
//      ends exactly at T, and then joins its class's stream; a job whose
//      admission fails is marked rejected and the tick goes on;
//   3. launch: a class with fewer than two steps in flight launches the next
//      RK4 step of its jobs that still have steps to go (so the device always
//      holds the following step of a class while the host handles the
//      completion of the current one), and records an event after it.
// A tick that completes, admits and launches nothing while work is in flight
// waits until some class's step completes.  Small-grid classes therefore run
// at their own step rate, not at the rate of the largest class.  The server
// uses the public C-ABI of the library plus two internal calls (context
// creation with shared operators, release of an idle context).  With a null
// arena it runs "dry": no device work, each step completes at once; this
// exercises admission, budget and latency bookkeeping without a GPU.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "grmhd.h"
#include "grmhd_internal.h"

namespace {

thread_local std::string g_serr;

int sfail(int code, const std::string& msg) {
  g_serr = msg;
  return code;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct Job {
  int64_t id;
  grmhd_grid grid;
  grmhd_phys phys;
  grmhd_prec prec;
  double t_end;
  int keep;
  int state;  // 0 queued, 1 running, 2 done, 3 rejected, 4 cancelled
  bool cancel = false;  // running, cancelled: released once no step is in flight
  size_t off = 0, bytes = 0, res_bytes = 0;
  grmhd_ctx* ctx = nullptr;
  int64_t steps_total = 0, steps_done = 0;
  int64_t steps_launched = 0;  // steps done + steps in flight
  double dt = 0.0;
  double t_arrival = 0.0, t_admit = -1.0, t_done = -1.0;
  std::vector<double> result;
  int cls = -1;
};

// One launched RK4 step of a class: the event recorded after it and the jobs
// it carries.
struct Launch {
  hipEvent_t ev = nullptr;
  std::vector<size_t> jobs;
};

// Steps a class may have in flight at once.
constexpr int DEPTH = 2;
// Jobs admitted per tick: admission builds each job's context and initial
// data on the host (milliseconds per job), so a burst of arrivals is admitted
// a few at a time while the classes already admitted keep the device busy.
constexpr int ADMIT_PER_TICK = 4;

// First-fit allocator over [0, size) with coalescing frees.
struct Arena {
  size_t size = 0, in_use = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t n) {
    size = n;
    free_.clear();
    if (n) free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t noff = it->first + n;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        in_use += n;
        peak = std::max(peak, in_use);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    in_use -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// jobs of one class are stepped by one batched launch sequence
bool same_class(const Job& a, const Job& b) {
  return grmhd::same_step_class(a.grid, a.phys, a.prec, b.grid, b.phys, b.prec);
}

}  // namespace

struct grmhd_server {
  char* arena_base;
  bool dry;
  int max_batch;
  hipStream_t user_stream;
  hipStream_t admit_stream = nullptr;  // initial data of admitted jobs
  bool own_admit = false;
  Arena arena;
  std::vector<Job> jobs;
  std::deque<size_t> queue;  // indices into jobs
  struct Class {
    Job rep;                   // representative job (the class predicate)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::deque<Launch> inflight;
    std::vector<hipEvent_t> spare;  // events of completed launches, reused
  };
  std::vector<Class> classes;
  // operators per (grid, cfl), built at the first submission of that grid and
  // shared by the time step and every context created for it
  struct OpsEntry {
    grmhd_grid grid;
    double cfl;
    std::unique_ptr<grmhd::Operators> ops;
  };
  std::vector<OpsEntry> ops_cache;
  std::chrono::steady_clock::time_point t0;
  double busy = 0.0;          // seconds with device work in flight
  double busy_since = -1.0;   // start of the current in-flight period
  double first_submit = -1.0;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  int inflight_total() const {
    int n = 0;
    for (const auto& c : classes) n += (int)c.inflight.size();
    return n;
  }
};

static const grmhd::Operators* operators_for(grmhd_server* s, const grmhd_grid& g, double cfl);

extern "C" {

const char* grmhd_server_last_error(void) { return g_serr.c_str(); }

int grmhd_server_create(void* dev_arena, size_t arena_bytes, int32_t max_batch, void* hip_stream,
                        grmhd_server** out) {
  if (!out) return sfail(GRMHD_E_ARG, "null output");
  if (max_batch < 1) return sfail(GRMHD_E_ARG, "max_batch >= 1");
  if (dev_arena && ((uintptr_t)dev_arena & 255)) return sfail(GRMHD_E_ARG, "arena must be 256-byte aligned");
  grmhd_server* s = new grmhd_server();
  s->arena_base = (char*)dev_arena;
  s->dry = dev_arena == nullptr;
  s->max_batch = max_batch;
  s->user_stream = (hipStream_t)hip_stream;
  s->arena.init(arena_bytes);
  if (!s->dry) {
    hipStream_t st = nullptr;
    s->own_admit = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    s->admit_stream = s->own_admit ? st : s->user_stream;
  }
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return GRMHD_OK;
}

int grmhd_server_destroy(grmhd_server* s) {
  if (!s) return GRMHD_OK;
  for (auto& c : s->classes)
    if (c.stream) (void)hipStreamSynchronize(c.stream);
  for (auto& j : s->jobs)
    if (j.ctx) grmhd::destroy_idle_context(j.ctx);
  for (auto& c : s->classes) {
    for (auto& l : c.inflight)
      if (l.ev) (void)hipEventDestroy(l.ev);
    for (auto ev : c.spare) (void)hipEventDestroy(ev);
    if (c.own_stream) (void)hipStreamDestroy(c.stream);
  }
  if (s->own_admit) (void)hipStreamDestroy(s->admit_stream);
  delete s;
  return GRMHD_OK;
}

double grmhd_server_clock(const grmhd_server* s) { return s ? s->now() : NAN; }

int grmhd_server_submit(grmhd_server* s, const grmhd_grid* grid, const grmhd_phys* phys, grmhd_prec prec,
                        double t_end, int32_t keep_state, int64_t* job_id) {
  if (!s || !grid || !phys || !job_id) return sfail(GRMHD_E_ARG, "null argument");
  if (!(t_end > 0.0) || !std::isfinite(t_end)) return sfail(GRMHD_E_ARG, "job rejected: need a finite t_end > 0");
  size_t res = 0, scr = 0;
  int rc = grmhd_query_bytes(grid, prec, &res, &scr);
  if (rc) return sfail(rc, std::string("job rejected: ") + grmhd_last_error());
  {
    std::string why;
    if (grmhd::validate_phys(*phys, true, &why)) return sfail(GRMHD_E_ARG, "job rejected: " + why);
  }
  const double dt = operators_for(s, *grid, phys->cfl)->dt;  // grid validated by the size query
  Job j;
  j.id = (int64_t)s->jobs.size();
  j.grid = *grid;
  j.phys = *phys;
  j.prec = prec;
  j.t_end = t_end;
  j.keep = keep_state;
  j.res_bytes = align256(res);
  j.bytes = align256(res) + align256(scr);
  j.steps_total = (int64_t)ceil(t_end / dt);
  j.dt = t_end / (double)j.steps_total;
  j.t_arrival = s->now();
  if (s->first_submit < 0) s->first_submit = j.t_arrival;
  *job_id = j.id;
  if (j.bytes > s->arena.size) {
    j.state = 3;
    s->jobs.push_back(j);
    return sfail(GRMHD_E_BUDGET, "job footprint exceeds the memory budget");
  }
  j.state = 0;
  s->jobs.push_back(j);
  s->queue.push_back(s->jobs.size() - 1);
  return GRMHD_OK;
}

static bool same_grid(const grmhd_grid& a, const grmhd_grid& b) {
  return a.nr == b.nr && a.nth == b.nth && a.nph == b.nph && a.r_in == b.r_in && a.r_out == b.r_out &&
         a.th_min == b.th_min && a.th_max == b.th_max && a.filt_alpha == b.filt_alpha &&
         a.filt_order == b.filt_order && a.filter_on == b.filter_on && a.dealias == b.dealias;
}

// The operators of a (validated) grid and cfl, built once per server.
static const grmhd::Operators* operators_for(grmhd_server* s, const grmhd_grid& g, double cfl) {
  for (auto& e : s->ops_cache)
    if (e.cfl == cfl && same_grid(e.grid, g)) return e.ops.get();
  grmhd_server::OpsEntry e;
  e.grid = g;
  e.cfl = cfl;
  e.ops.reset(new grmhd::Operators());
  grmhd::build_operators(g, cfl, e.ops.get());
  s->ops_cache.push_back(std::move(e));
  return s->ops_cache.back().ops.get();
}

static int class_of(grmhd_server* s, const Job& j) {
  for (size_t c = 0; c < s->classes.size(); ++c)
    if (same_class(s->classes[c].rep, j)) return (int)c;
  grmhd_server::Class c;
  c.rep = j;
  if (!s->dry) {
    hipStream_t st = nullptr;
    c.own_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    c.stream = c.own_stream ? st : s->user_stream;
  }
  s->classes.push_back(std::move(c));
  return (int)s->classes.size() - 1;
}

// A job at its end time: keep its state if asked, release its context and
// block.  Its class has no step of it in flight.
static int retire(grmhd_server* s, Job& j, double t) {
  if (!s->dry) {
    if (j.keep) {
      const size_t P = (size_t)j.grid.nr * j.grid.nth * j.grid.nph;
      j.result.resize((size_t)(j.phys.glm ? GRMHD_NFIELDS_GLM : GRMHD_NFIELDS) * P);  // psi last with GLM
      double* dU = nullptr;
      int rc = grmhd_state_ptr(j.ctx, &dU, nullptr);
      if (rc) return sfail(rc, grmhd_last_error());
      // the class stream may already hold the next step of other jobs: copy
      // on the admission stream (the job's last step has completed)
      hipError_t e = hipMemcpyAsync(j.result.data(), dU, j.result.size() * sizeof(double),
                                    hipMemcpyDeviceToHost, s->admit_stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->admit_stream);
      if (e != hipSuccess) return sfail(GRMHD_E_DEVICE, std::string("result copy: ") + hipGetErrorString(e));
    }
    grmhd::destroy_idle_context(j.ctx);
    j.ctx = nullptr;
  }
  s->arena.release(j.off, j.bytes);
  j.state = 2;
  j.t_done = t;
  return GRMHD_OK;
}

// Release the cancelled running jobs that have no step in flight (their
// class's events have passed every step launched for them).
static void release_cancelled(grmhd_server* s) {
  for (auto& j : s->jobs) {
    if (j.state != 1 || !j.cancel || j.steps_done < j.steps_launched) continue;
    if (!s->dry) {
      grmhd::destroy_idle_context(j.ctx);
      j.ctx = nullptr;
    }
    s->arena.release(j.off, j.bytes);
    j.state = 4;
    j.t_done = s->now();
  }
}

// Count the completed launches of every class (the oldest first, in stream
// order) and retire jobs that reached their end time.
static int complete(grmhd_server* s, bool* progress) {
  for (auto& c : s->classes) {
    while (!c.inflight.empty()) {
      Launch& l = c.inflight.front();
      if (!s->dry) {
        const hipError_t q = hipEventQuery(l.ev);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return sfail(GRMHD_E_DEVICE, std::string("class step: ") + hipGetErrorString(q));
      }
      const double t = s->now();
      for (size_t i : l.jobs) {
        Job& j = s->jobs[i];
        j.steps_done += 1;
        if (!j.cancel && j.steps_done >= j.steps_total) {
          int rc = retire(s, j, t);
          if (rc) return rc;
        }
      }
      if (l.ev) c.spare.push_back(l.ev);
      c.inflight.pop_front();
      *progress = true;
    }
  }
  release_cancelled(s);
  if (s->busy_since >= 0.0 && s->inflight_total() == 0) {
    s->busy += s->now() - s->busy_since;
    s->busy_since = -1.0;
  }
  return GRMHD_OK;
}

// Admission in arrival order while the head job fits.  A job whose context
// or initial data cannot be built is rejected (its message is the server's
// last error); the others go on.
static void admit(grmhd_server* s, bool* progress) {
  for (int admitted = 0; !s->queue.empty() && (s->dry || admitted < ADMIT_PER_TICK); ++admitted) {
    Job& j = s->jobs[s->queue.front()];
    size_t off = 0;
    if (!s->arena.alloc(j.bytes, &off)) break;
    s->queue.pop_front();
    *progress = true;
    j.off = off;
    j.cls = class_of(s, j);
    if (!s->dry) {
      char* res = s->arena_base + off;
      char* scr = res + j.res_bytes;
      int rc = grmhd::create_context(&j.grid, &j.phys, j.prec, res, scr, s->admit_stream,
                                     operators_for(s, j.grid, j.phys.cfl), &j.ctx);
      if (!rc) rc = grmhd_init_state(j.ctx);  // syncs the admission stream
      if (!rc) rc = grmhd_set_dt(j.ctx, j.dt);
      if (!rc) rc = grmhd_set_stream(j.ctx, s->classes[j.cls].stream);
      if (rc) {
        g_serr = "job " + std::to_string(j.id) + " rejected at admission: " + grmhd_last_error();
        if (j.ctx) grmhd::destroy_idle_context(j.ctx);
        j.ctx = nullptr;
        s->arena.release(off, j.bytes);
        j.state = 3;
        continue;
      }
    }
    j.state = 1;
    j.t_admit = s->now();
  }
}

// Launch the next step of every class with room in its pipeline.
static int launch(grmhd_server* s, bool* progress) {
  for (size_t ci = 0; ci < s->classes.size(); ++ci) {
    auto& c = s->classes[ci];
    const int depth = s->dry ? 1 : DEPTH;  // a dry step completes within its tick
    while ((int)c.inflight.size() < depth) {
      std::vector<size_t> ids;
      for (size_t i = 0; i < s->jobs.size(); ++i) {
        const Job& j = s->jobs[i];
        if (j.state == 1 && !j.cancel && j.cls == (int)ci && j.steps_launched < j.steps_total) ids.push_back(i);
      }
      if (ids.empty()) break;
      Launch l;
      l.jobs = ids;
      if (!s->dry) {
        for (size_t b = 0; b < ids.size(); b += (size_t)s->max_batch) {
          const size_t m = std::min(ids.size() - b, (size_t)s->max_batch);
          std::vector<grmhd_ctx*> ctxs(m);
          for (size_t q = 0; q < m; ++q) ctxs[q] = s->jobs[ids[b + q]].ctx;
          int rc = grmhd_step_batch(ctxs.data(), (int32_t)m, 1);
          if (rc) return sfail(rc, std::string("batched step failed: ") + grmhd_last_error());
        }
        if (!c.spare.empty()) {
          l.ev = c.spare.back();
          c.spare.pop_back();
        } else if (hipEventCreateWithFlags(&l.ev, hipEventDisableTiming) != hipSuccess) {
          return sfail(GRMHD_E_DEVICE, "event create failed");
        }
        if (hipEventRecord(l.ev, c.stream) != hipSuccess) return sfail(GRMHD_E_DEVICE, "event record failed");
      }
      for (size_t i : ids) s->jobs[i].steps_launched += 1;
      if (s->busy_since < 0.0) s->busy_since = s->now();
      c.inflight.push_back(std::move(l));
      *progress = true;
    }
  }
  return GRMHD_OK;
}

int grmhd_server_tick(grmhd_server* s, int32_t* n_pending) {
  if (!s) return sfail(GRMHD_E_ARG, "null server");
  for (int pass = 0; pass < 2; ++pass) {
    bool progress = false;
    int rc = complete(s, &progress);
    if (rc) return rc;
    admit(s, &progress);
    if ((rc = launch(s, &progress))) return rc;
    if (s->dry) {  // a dry step completes at once
      if ((rc = complete(s, &progress))) return rc;
      break;
    }
    if (progress || s->inflight_total() == 0) break;
    // nothing to do until some class's step completes: wait for that
    for (;;) {
      bool any = false;
      for (auto& c : s->classes)
        if (!c.inflight.empty()) {
          const hipError_t q = hipEventQuery(c.inflight.front().ev);
          if (q != hipErrorNotReady) any = true;
        }
      if (any) break;
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
  if (n_pending) {
    int32_t n = 0;
    for (auto& j : s->jobs) n += (j.state == 0 || j.state == 1);
    *n_pending = n;
  }
  return GRMHD_OK;
}
int grmhd_server_poll(grmhd_server* s, int64_t id, grmhd_job_info* out) {
  if (!s || !out || id < 0 || id >= (int64_t)s->jobs.size()) return sfail(GRMHD_E_ARG, "unknown job");
  const Job& j = s->jobs[id];
  out->id = j.id;
  out->state = j.state;
  out->nr = j.grid.nr;
  out->nth = j.grid.nth;
  out->nph = j.grid.nph;
  out->prec = (int32_t)j.prec;
  out->steps_done = j.steps_done;
  out->steps_total = j.steps_total;
  out->dt = j.dt;
  out->t_arrival = j.t_arrival;
  out->t_admit = j.t_admit;
  out->t_done = j.t_done;
  out->latency = j.state == 2 ? j.t_done - j.t_arrival : -1.0;
  out->bytes = j.bytes;
  return GRMHD_OK;
}

int grmhd_server_cancel(grmhd_server* s, int64_t id) {
  if (!s || id < 0 || id >= (int64_t)s->jobs.size()) return sfail(GRMHD_E_ARG, "unknown job");
  Job& j = s->jobs[id];
  if (j.state == 0) {
    const auto q = std::find(s->queue.begin(), s->queue.end(), (size_t)id);
    if (q == s->queue.end()) return sfail(GRMHD_E_STATE, "queued job missing from the queue");
    s->queue.erase(q);
    j.state = 4;
    j.t_done = s->now();
    return GRMHD_OK;
  }
  if (j.state != 1 || j.cancel) return sfail(GRMHD_E_STATE, "job already done, rejected or cancelled");
  j.cancel = true;
  release_cancelled(s);  // at once if none of its steps is in flight
  return GRMHD_OK;
}

int grmhd_server_result(grmhd_server* s, int64_t id, double* host_U, size_t n) {
  if (!s || !host_U || id < 0 || id >= (int64_t)s->jobs.size()) return sfail(GRMHD_E_ARG, "unknown job");
  const Job& j = s->jobs[id];
  if (j.state != 2 || j.result.empty()) return sfail(GRMHD_E_STATE, "job not finished or state not kept");
  if (n != j.result.size()) return sfail(GRMHD_E_SIZE, "state size must be 32 * P (33 * P for a GLM job)");
  std::copy(j.result.begin(), j.result.end(), host_U);
  return GRMHD_OK;
}

int grmhd_server_stats(grmhd_server* s, grmhd_server_summary* out) {
  if (!s || !out) return sfail(GRMHD_E_ARG, "null argument");
  grmhd_server_summary st = {};
  std::vector<double> lat;
  double last_done = s->first_submit;
  for (auto& j : s->jobs) {
    st.submitted += 1;
    if (j.state == 0) st.queued += 1;
    if (j.state == 1) st.running += 1;
    if (j.state == 3) st.rejected += 1;
    if (j.state == 4) st.cancelled += 1;
    if (j.state == 2) {
      st.completed += 1;
      lat.push_back(j.t_done - j.t_arrival);
      st.point_stage_updates += 4.0 * (double)j.steps_total * j.grid.nr * j.grid.nth * j.grid.nph;
      last_done = std::max(last_done, j.t_done);
    }
  }
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double q) {  // nearest-rank percentile
    if (lat.empty()) return 0.0;
    size_t k = (size_t)ceil(q * lat.size());
    return lat[std::min(std::max<size_t>(k, 1), lat.size()) - 1];
  };
  st.p50_latency = pct(0.50);
  st.p99_latency = pct(0.99);
  double sum = 0.0;
  for (double x : lat) sum += x;
  st.mean_latency = lat.empty() ? 0.0 : sum / lat.size();
  st.wall = s->first_submit < 0 ? 0.0 : last_done - s->first_submit;
  st.busy = s->busy;
  st.bytes_in_use = s->arena.in_use;
  st.bytes_peak = s->arena.peak;
  *out = st;
  return GRMHD_OK;
}

}  // extern "C"
