// Continuous-batching job server for evolution jobs (the served form).
//
// Jobs (grid, physics, precision, end time) are submitted as they arrive and
// wait in a FIFO queue.  Every tick:
//   1. admission: queued jobs are placed, in arrival order, into the caller's
//      device arena (first fit, 256-byte aligned blocks holding the job's
//      resident and scratch buffers) as long as they fit the budget; an
//      admitted job gets its context, initial data and a time step
//      dt = T / ceil(T / dt_CFL) so that it ends exactly at T;
//   2. one RK4 step for every running job: jobs of one grid class
//      (grid sizes, precision, kernel parameters) advance together, one
//      launch per kernel for the whole class (grmhd_step_batch), each class
//      on its own stream so that classes overlap on the device;
//   3. retirement: finished jobs record their latency (completion minus
//      arrival on the server clock), optionally keep their final state on
//      the host, and free their block, so queued jobs can enter next tick.
// The server uses only the public C-ABI of the library.  With a null arena it
// runs "dry": no device work, each step completes at once; this exercises
// admission, budget and latency bookkeeping on a machine without a GPU.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <string>
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
  int state;  // 0 queued, 1 running, 2 done, 3 rejected
  size_t off = 0, bytes = 0, res_bytes = 0;
  grmhd_ctx* ctx = nullptr;
  int64_t steps_total = 0, steps_done = 0;
  double dt = 0.0;
  double t_arrival = 0.0, t_admit = -1.0, t_done = -1.0;
  std::vector<double> result;
  int cls = -1;
};

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
  Arena arena;
  std::vector<Job> jobs;
  std::deque<size_t> queue;  // indices into jobs
  std::vector<Job> classes;  // one representative per grid class
  std::vector<hipStream_t> streams;
  std::vector<bool> own_stream;
  // operators per (grid, cfl), built at the first submission of that grid and
  // shared by the time step and every context created for it
  struct OpsEntry {
    grmhd_grid grid;
    double cfl;
    std::unique_ptr<grmhd::Operators> ops;
  };
  std::vector<OpsEntry> ops_cache;
  std::chrono::steady_clock::time_point t0;
  double busy = 0.0;
  double first_submit = -1.0;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
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
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return GRMHD_OK;
}

int grmhd_server_destroy(grmhd_server* s) {
  if (!s) return GRMHD_OK;
  for (auto& j : s->jobs)
    if (j.ctx) grmhd_destroy(j.ctx);
  for (size_t i = 0; i < s->streams.size(); ++i)
    if (s->own_stream[i]) (void)hipStreamDestroy(s->streams[i]);
  delete s;
  return GRMHD_OK;
}

double grmhd_server_clock(const grmhd_server* s) { return s ? s->now() : NAN; }

int grmhd_server_submit(grmhd_server* s, const grmhd_grid* grid, const grmhd_phys* phys, grmhd_prec prec,
                        double t_end, int32_t keep_state, int64_t* job_id) {
  if (!s || !grid || !phys || !job_id) return sfail(GRMHD_E_ARG, "null argument");
  if (!(t_end > 0.0)) return sfail(GRMHD_E_ARG, "t_end > 0");
  size_t res = 0, scr = 0;
  int rc = grmhd_query_bytes(grid, prec, &res, &scr);
  if (rc) return sfail(rc, std::string("job rejected: ") + grmhd_last_error());
  if (!(phys->cfl > 0.0)) return sfail(GRMHD_E_ARG, "job rejected: cfl > 0");
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
    if (same_class(s->classes[c], j)) return (int)c;
  s->classes.push_back(j);
  if (!s->dry) {
    hipStream_t st = nullptr;
    const bool own = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    s->streams.push_back(own ? st : s->user_stream);
    s->own_stream.push_back(own);
  }
  return (int)s->classes.size() - 1;
}

int grmhd_server_tick(grmhd_server* s, int32_t* n_pending) {
  if (!s) return sfail(GRMHD_E_ARG, "null server");
  const double tin = s->now();
  // 1. admission in arrival order while the head job fits
  while (!s->queue.empty()) {
    Job& j = s->jobs[s->queue.front()];
    size_t off = 0;
    if (!s->arena.alloc(j.bytes, &off)) break;
    j.off = off;
    j.cls = class_of(s, j);
    if (!s->dry) {
      char* res = s->arena_base + off;
      char* scr = res + j.res_bytes;
      int rc = grmhd::create_context(&j.grid, &j.phys, j.prec, res, scr, s->streams[j.cls],
                                     operators_for(s, j.grid, j.phys.cfl), &j.ctx);
      if (!rc) rc = grmhd_init_state(j.ctx);
      if (!rc) rc = grmhd_set_dt(j.ctx, j.dt);
      if (rc) {
        const std::string msg = grmhd_last_error();
        if (j.ctx) grmhd_destroy(j.ctx);
        j.ctx = nullptr;
        s->arena.release(off, j.bytes);
        j.state = 3;
        s->queue.pop_front();
        return sfail(rc, "admission failed: " + msg);
      }
    }
    j.state = 1;
    j.t_admit = s->now();
    s->queue.pop_front();
  }
  // 2. one RK4 step per running job, batched per grid class
  std::vector<std::vector<size_t>> by_class(s->classes.size());
  for (size_t i = 0; i < s->jobs.size(); ++i)
    if (s->jobs[i].state == 1) by_class[s->jobs[i].cls].push_back(i);
  for (size_t c = 0; c < by_class.size(); ++c) {
    const auto& ids = by_class[c];
    for (size_t b = 0; b < ids.size(); b += (size_t)s->max_batch) {
      const size_t m = std::min(ids.size() - b, (size_t)s->max_batch);
      if (!s->dry) {
        std::vector<grmhd_ctx*> ctxs(m);
        for (size_t q = 0; q < m; ++q) ctxs[q] = s->jobs[ids[b + q]].ctx;
        int rc = grmhd_step_batch(ctxs.data(), (int32_t)m, 1);
        if (rc) return sfail(rc, std::string("batched step failed: ") + grmhd_last_error());
      }
      for (size_t q = 0; q < m; ++q) s->jobs[ids[b + q]].steps_done += 1;
    }
  }
  if (!s->dry)
    for (auto st : s->streams)
      if (hipStreamSynchronize(st) != hipSuccess) return sfail(GRMHD_E_DEVICE, "stream synchronize failed");
  // 3. retirement
  const double tdone = s->now();
  for (auto& j : s->jobs) {
    if (j.state != 1 || j.steps_done < j.steps_total) continue;
    if (!s->dry) {
      if (j.keep) {
        const size_t P = (size_t)j.grid.nr * j.grid.nth * j.grid.nph;
        j.result.resize((size_t)(j.phys.glm ? GRMHD_NFIELDS_GLM : GRMHD_NFIELDS) * P);  // psi last with GLM
        int rc = grmhd_get_state(j.ctx, j.result.data(), j.result.size(), nullptr);
        if (rc) return sfail(rc, grmhd_last_error());
      }
      grmhd_destroy(j.ctx);
      j.ctx = nullptr;
    }
    s->arena.release(j.off, j.bytes);
    j.state = 2;
    j.t_done = tdone;
  }
  s->busy += s->now() - tin;
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
