// hg_server.hip -- the request server (hg_server_* in hgref.h): admission by
// device footprint into a caller arena, a loader thread, and an executor
// thread that advances every admitted job one label-propagation round per
// step in batched launches (continuous batching).
//
// Threads and streams
//   loader    copies a job's arrays in and runs hg_load_csr on the load
//             stream (which synchronizes that stream only)
//   executor  owns the compute stream: per step it rebuilds the work tables
//             when members joined or left, runs the pin-count pass of the
//             joiners, one round for every member, and queues the result
//             copies of members that ran their last round
// Both streams have the default priority.  A job's memory is released only
// after the event recorded behind its result copies has completed, so no
// kernel can still read it.
//
// Work tables: two halves of the table region, used alternately; a half is
// rebuilt only after the last step that read it has completed (its event).
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "hg_batch.h"

namespace hg {
namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxRounds = 1024;
constexpr int kInFlightSteps = 2;   // steps queued ahead of the GPU

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Byte offsets of a job's arrays inside its arena slice.
struct JobLayout {
  size_t eptr, pins, vwgt, ewgt, vptr, vnets, ws, ws_bytes, part, phi, netstate, block_w, km1,
      eligible, stats, total;
};

bool job_layout(int n, int m, long long P, int k, int rounds, bool wv, bool we, JobLayout& L) {
  const size_t ws = hg_workspace_size(n, m, P, k);
  const long long nsw = hg_netstate_words(m, k);
  if (ws == 0 || nsw == 0) return false;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.eptr = take(sizeof(long long) * ((size_t)m + 1));
  L.pins = take(sizeof(int) * (size_t)P);
  L.vwgt = wv ? take(sizeof(int) * (size_t)n) : (size_t)-1;
  L.ewgt = we ? take(sizeof(int) * (size_t)m) : (size_t)-1;
  L.vptr = take(sizeof(long long) * ((size_t)n + 1));
  L.vnets = take(sizeof(int) * (size_t)P);
  L.ws = take(ws);
  L.ws_bytes = ws;
  L.part = take(sizeof(int) * (size_t)n);
  L.phi = take(sizeof(int) * (size_t)m * k);
  L.netstate = take(sizeof(unsigned) * (size_t)nsw);
  L.block_w = take(sizeof(long long) * (size_t)k);
  L.km1 = take(sizeof(long long));
  L.eligible = take((size_t)n);
  L.stats = take(sizeof(hg_round_stats) * (size_t)rounds);
  L.total = off;
  return true;
}

// First-fit allocator over [0, cap) with coalescing free ranges.
class RangeAlloc {
 public:
  explicit RangeAlloc(size_t cap) : cap_(cap) {
    if (cap) free_[0] = cap;
  }
  bool take(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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
  size_t cap() const { return cap_; }
  size_t used() const { return used_; }

 private:
  size_t cap_, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Job {
  int64_t id = 0;
  hg_request r{};
  int state = HG_REQ_PENDING;
  hg_status status = HG_OK;
  char msg[160] = "";
  JobLayout lay{};
  size_t off = 0;
  char* base = nullptr;          // device address of the slice
  hg_graph_s* g = nullptr;
  long long lmax = 0;
  int64_t join_step = -1;
  int rounds_done = 0;
  bool finishing = false;
  hipEvent_t done_ev = nullptr;
  double admit_ms = 0, loaded_ms = 0, done_ms = 0;
};

using Clock = std::chrono::steady_clock;

}  // namespace
}  // namespace hg

struct hg_server_s {
  // fixed at creation
  char* arena = nullptr;
  size_t table_half = 0;
  char* host_half[2] = {nullptr, nullptr};
  hipEvent_t half_ev[2] = {nullptr, nullptr};
  bool half_used[2] = {false, false};
  int device = 0;
  int max_active = 1;
  hg_schedule sched[HG_SIZE_CLASSES];
  hipStream_t compute = nullptr, load = nullptr;
  hipEvent_t epoch_ev = nullptr;
  double epoch_ms = 0;
  hg::Clock::time_point t0;
  std::unique_ptr<hg::RangeAlloc> mem;   // job memory (offsets after the table region)
  char* job_base = nullptr;

  std::mutex mu;
  std::condition_variable cv_exec, cv_load, cv_done;
  bool stop = false;
  std::vector<std::unique_ptr<hg::Job>> jobs;
  std::deque<hg::Job*> pending, to_load, ready;
  int resident = 0;                     // admitted and not done
  hg_server_stats st{};
  hg_status fatal = HG_OK;
  char fatal_msg[160] = "";

  // executor-owned
  std::vector<hg::Job*> active;
  std::vector<hipEvent_t> step_ev_pool;
  std::deque<hipEvent_t> in_flight;
  int half = 1;
  hg::RoundPlan rp;
  hg::CountPlan cp;
  int64_t step = 0;

  std::thread exec_thread, load_thread;
};

namespace hg {
namespace {

double now_ms(const hg_server_s* s) {
  return std::chrono::duration<double, std::milli>(Clock::now() - s->t0).count();
}

// Milliseconds on the server clock at which event `e` completed.
double event_ms(const hg_server_s* s, hipEvent_t e) {
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, s->epoch_ev, e) != hipSuccess) return now_ms(s);
  return s->epoch_ms + ms;
}

void finish_failed(hg_server_s* s, Job* j, hg_status st, const char* msg) {
  j->status = st;
  snprintf(j->msg, sizeof(j->msg), "%s", msg);
  j->state = HG_REQ_DONE;
  j->done_ms = now_ms(s);
  s->st.failed += 1;
  s->cv_done.notify_all();
}

// ---- loader thread ----
hg_status load_job(hg_server_s* s, Job* j) {
  const hg_request& r = j->r;
  const JobLayout& L = j->lay;
  char* b = j->base;
  hipStream_t ls = s->load;
  HG_TRY(hipMemcpyAsync(b + L.eptr, r.eptr, sizeof(long long) * ((size_t)r.m + 1),
                        hipMemcpyHostToDevice, ls), "copy eptr");
  HG_TRY(hipMemcpyAsync(b + L.pins, r.pins, sizeof(int) * (size_t)r.P, hipMemcpyHostToDevice, ls),
         "copy pins");
  if (r.vwgt)
    HG_TRY(hipMemcpyAsync(b + L.vwgt, r.vwgt, sizeof(int) * (size_t)r.n, hipMemcpyHostToDevice,
                          ls), "copy vwgt");
  if (r.ewgt)
    HG_TRY(hipMemcpyAsync(b + L.ewgt, r.ewgt, sizeof(int) * (size_t)r.m, hipMemcpyHostToDevice,
                          ls), "copy ewgt");
  HG_TRY(hipMemcpyAsync(b + L.part, r.part, sizeof(int) * (size_t)r.n, hipMemcpyHostToDevice, ls),
         "copy part");
  hg_graph g = nullptr;
  hg_status st = hg_load_csr(r.n, r.m, r.P, (const int64_t*)(b + L.eptr),
                             (const int32_t*)(b + L.pins),
                             r.vwgt ? (const int32_t*)(b + L.vwgt) : nullptr,
                             r.ewgt ? (const int32_t*)(b + L.ewgt) : nullptr,
                             (int64_t*)(b + L.vptr), (int32_t*)(b + L.vnets), b + L.ws,
                             L.ws_bytes, r.k, ls, &g);
  if (st != HG_OK) return st;
  j->g = g;
  j->lmax = hg_max_block_weight(g, r.k, r.eps);
  return HG_OK;
}

void load_loop(hg_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_load.wait(lk, [&] { return s->stop || !s->to_load.empty(); });
    if (s->to_load.empty()) {
      if (s->stop) break;
      continue;
    }
    Job* j = s->to_load.front();
    s->to_load.pop_front();
    lk.unlock();
    const hg_status st = load_job(s, j);
    char msg[160];
    snprintf(msg, sizeof(msg), "%s", st == HG_OK ? "" : hg_last_error());
    lk.lock();
    if (st == HG_OK) {
      j->loaded_ms = now_ms(s);
      s->ready.push_back(j);
    } else {
      s->mem->give(j->off, j->lay.total);
      s->resident -= 1;
      finish_failed(s, j, st, msg);
    }
    s->cv_exec.notify_one();
  }
}

// ---- executor thread ----

// Jobs whose result copies completed: release memory, record the time.
void retire(hg_server_s* s) {
  std::vector<Job*> keep;
  for (Job* j : s->active) {
    if (!j->finishing) {
      keep.push_back(j);
      continue;
    }
    const hipError_t q = hipEventQuery(j->done_ev);
    if (q == hipErrorNotReady) {
      keep.push_back(j);
      continue;
    }
    j->done_ms = event_ms(s, j->done_ev);
    (void)hipEventDestroy(j->done_ev);
    j->done_ev = nullptr;
    hg_free(j->g);
    j->g = nullptr;
    s->mem->give(j->off, j->lay.total);
    s->resident -= 1;
    j->state = HG_REQ_DONE;
    if (q == hipSuccess) {
      s->st.completed += 1;
    } else {
      j->status = HG_ERR_DEVICE;
      snprintf(j->msg, sizeof(j->msg), "%s", hipGetErrorString(q));
      s->st.failed += 1;
    }
    s->cv_done.notify_all();
  }
  s->active.swap(keep);
}

// Admit pending jobs in arrival order while memory and slots allow.
void admit(hg_server_s* s) {
  while (!s->pending.empty() && s->resident < s->max_active) {
    Job* j = s->pending.front();
    if (j->lay.total > s->mem->cap()) {
      s->pending.pop_front();
      finish_failed(s, j, HG_ERR_WORKSPACE, "job larger than the server's job memory");
      continue;
    }
    size_t off = 0;
    if (!s->mem->take(j->lay.total, &off)) break;
    s->pending.pop_front();
    j->off = off;
    j->base = s->job_base + off;
    j->state = HG_REQ_ADMITTED;
    j->admit_ms = now_ms(s);
    s->resident += 1;
    s->st.peak_bytes = std::max<int64_t>(s->st.peak_bytes, (int64_t)s->mem->used());
    s->to_load.push_back(j);
    s->cv_load.notify_one();
  }
}

BatchMember member_of(const hg_server_s* s, const Job* j) {
  BatchMember M;
  const JobLayout& L = j->lay;
  char* b = j->base;
  M.g = j->g;
  M.k = j->r.k;
  M.cls = size_class(j->r.n);
  M.round_base = (int)j->join_step;
  M.lmax = j->lmax;
  M.part = (int*)(b + L.part);
  M.phi = (int*)(b + L.phi);
  M.netstate = (unsigned*)(b + L.netstate);
  M.block_w = (long long*)(b + L.block_w);
  M.eligible = (unsigned char*)(b + L.eligible);
  M.stats = (hg_round_stats*)(b + L.stats);
  M.km1 = (long long*)(b + L.km1);
  (void)s;
  return M;
}

// Enqueue one step for the members in `run` (joiners last, `nj` of them);
// rebuild the tables when `rebuild`.  Returns a HIP error.
hipError_t enqueue_step(hg_server_s* s, const std::vector<Job*>& run, size_t nj, bool rebuild) {
  hipStream_t cs = s->compute;
  hipError_t e = hipSuccess;
  if (rebuild) {
    const int h = s->half ^ 1;
    if (s->half_used[h]) {
      e = hipEventSynchronize(s->half_ev[h]);
      if (e != hipSuccess) return e;
    }
    std::vector<BatchMember> mem;
    std::vector<int> all, join;
    for (size_t i = 0; i < run.size(); ++i) {
      mem.push_back(member_of(s, run[i]));
      all.push_back((int)i);
      if (i + nj >= run.size()) join.push_back((int)i);
    }
    char* dev = s->arena + (size_t)h * s->table_half;
    size_t end = build_plans(mem, all, s->sched, dev, s->host_half[h], 0, s->table_half, &s->rp,
                             nullptr);
    if (end && !join.empty())
      end = build_plans(mem, join, s->sched, dev, s->host_half[h], end, s->table_half, nullptr,
                        &s->cp);
    if (end == 0) return hipErrorOutOfMemory;   // checked by the caller beforehand
    e = hipMemcpyAsync(dev, s->host_half[h], end, hipMemcpyHostToDevice, cs);
    if (e != hipSuccess) return e;
    s->half = h;
    s->st.rebuilds += 1;
  }
  if (nj > 0) {
    e = launch_counts(s->cp, true, true, cs);
    if (e != hipSuccess) return e;
  }
  e = launch_round(s->rp, (int)s->step, cs, nullptr);
  if (e != hipSuccess) return e;
  e = hipEventRecord(s->half_ev[s->half], cs);
  s->half_used[s->half] = true;
  return e;
}

// Queue the result copies of a job that ran its last round.
hipError_t enqueue_results(hg_server_s* s, Job* j) {
  const hg_request& r = j->r;
  const JobLayout& L = j->lay;
  hipStream_t cs = s->compute;
  hipError_t e = hipSuccess;
  if (r.part_out)
    e = hipMemcpyAsync(r.part_out, j->base + L.part, sizeof(int) * (size_t)r.n,
                       hipMemcpyDeviceToHost, cs);
  if (e == hipSuccess && r.stats_out)
    e = hipMemcpyAsync(r.stats_out, j->base + L.stats, sizeof(hg_round_stats) * (size_t)r.rounds,
                       hipMemcpyDeviceToHost, cs);
  if (e == hipSuccess && r.km1_out)
    e = hipMemcpyAsync(r.km1_out, j->base + L.km1, sizeof(long long), hipMemcpyDeviceToHost, cs);
  if (e == hipSuccess) e = hipEventCreate(&j->done_ev);
  if (e == hipSuccess) e = hipEventRecord(j->done_ev, cs);
  j->finishing = true;
  return e;
}

hipEvent_t step_event(hg_server_s* s) {
  if (s->step_ev_pool.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = s->step_ev_pool.back();
  s->step_ev_pool.pop_back();
  return e;
}

void exec_loop(hg_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  bool changed = true;     // membership differs from the current tables
  for (;;) {
    retire(s);
    admit(s);
    if (s->fatal != HG_OK) {
      // after a device error nothing new starts: fail what waits
      while (!s->pending.empty()) {
        finish_failed(s, s->pending.front(), s->fatal, s->fatal_msg);
        s->pending.pop_front();
      }
      while (!s->ready.empty()) {
        Job* j = s->ready.front();
        s->ready.pop_front();
        hg_free(j->g);
        j->g = nullptr;
        s->mem->give(j->off, j->lay.total);
        s->resident -= 1;
        finish_failed(s, j, s->fatal, s->fatal_msg);
      }
      // members without queued results never finish; nothing new is admitted
      // after a device error, so their memory is simply abandoned
      std::vector<Job*> keep;
      for (Job* j : s->active) {
        if (j->finishing) {
          keep.push_back(j);
          continue;
        }
        s->resident -= 1;
        finish_failed(s, j, s->fatal, s->fatal_msg);
      }
      s->active.swap(keep);
    }
    if (s->stop && s->resident == 0 && s->pending.empty()) break;
    // joiners: loaded jobs, as many as the table half can describe
    std::vector<Job*> run;
    for (Job* j : s->active)
      if (!j->finishing) run.push_back(j);
    size_t nj = 0;
    while (!s->ready.empty()) {
      Job* j = s->ready.front();
      std::vector<BatchMember> mem;
      std::vector<int> all;
      for (size_t i = 0; i < run.size(); ++i) {
        mem.push_back(member_of(s, run[i]));
        all.push_back((int)i);
      }
      j->join_step = s->step;
      mem.push_back(member_of(s, j));
      all.push_back((int)run.size());
      // round tables of everyone plus count tables of the joiners
      if (table_bound(mem, all) * 2 > s->table_half) {
        if (run.empty()) {
          s->ready.pop_front();
          hg_free(j->g);
          j->g = nullptr;
          s->mem->give(j->off, j->lay.total);
          s->resident -= 1;
          finish_failed(s, j, HG_ERR_WORKSPACE, "job too large for the server's table region");
          continue;
        }
        break;
      }
      s->ready.pop_front();
      run.push_back(j);
      ++nj;
    }
    if (run.empty()) {
      // Nothing to run.  Submits and finished loads notify; completions on
      // the GPU are polled (every 50 us while results are outstanding).
      if (!s->active.empty())
        s->cv_exec.wait_for(lk, std::chrono::microseconds(50));
      else
        s->cv_exec.wait_for(lk, std::chrono::milliseconds(1));
      continue;
    }
    if (nj > 0) changed = true;
    lk.unlock();
    // keep at most kInFlightSteps steps queued ahead of the GPU
    while ((int)s->in_flight.size() >= kInFlightSteps) {
      hipEvent_t e = s->in_flight.front();
      s->in_flight.pop_front();
      (void)hipEventSynchronize(e);
      s->step_ev_pool.push_back(e);
    }
    hipError_t e = enqueue_step(s, run, nj, changed);
    long long pins = 0;
    for (Job* j : run) pins += j->r.P;
    std::vector<Job*> leaving;
    for (Job* j : run) {
      j->rounds_done += 1;
      if (j->rounds_done >= j->r.rounds) leaving.push_back(j);
    }
    for (Job* j : leaving)
      if (e == hipSuccess) e = enqueue_results(s, j);
    hipEvent_t se = step_event(s);
    if (se && e == hipSuccess) {
      e = hipEventRecord(se, s->compute);
      s->in_flight.push_back(se);
    }
    lk.lock();
    if (e != hipSuccess && s->fatal == HG_OK) {
      s->fatal = HG_ERR_DEVICE;
      snprintf(s->fatal_msg, sizeof(s->fatal_msg), "server step: %s", hipGetErrorString(e));
    }
    for (size_t i = run.size() - nj; i < run.size(); ++i) {
      run[i]->state = HG_REQ_ACTIVE;
      s->active.push_back(run[i]);
    }
    s->st.steps += 1;
    s->st.member_rounds += (int64_t)run.size();
    s->st.pin_rounds += pins;
    s->st.max_members = std::max<int64_t>(s->st.max_members, (int64_t)run.size());
    s->step += 1;
    changed = !leaving.empty();
  }
  lk.unlock();
  while (!s->in_flight.empty()) {
    (void)hipEventSynchronize(s->in_flight.front());
    s->step_ev_pool.push_back(s->in_flight.front());
    s->in_flight.pop_front();
  }
}

}  // namespace
}  // namespace hg

using hg::fail;

extern "C" {

size_t hg_request_bytes(int32_t n, int32_t m, int64_t P, int32_t k, int32_t rounds,
                        int32_t weighted_vertices, int32_t weighted_nets) {
  if (n < 1 || m < 1 || P < m || k < 2 || k > HG_MAX_K || rounds < 1 || rounds > hg::kMaxRounds)
    return 0;
  hg::JobLayout L;
  if (!hg::job_layout(n, m, P, k, rounds, weighted_vertices != 0, weighted_nets != 0, L)) return 0;
  return L.total;
}

hg_status hg_server_create(void* arena, size_t arena_bytes, size_t table_bytes,
                           int32_t max_active, const hg_schedule* sched, hg_server* out) {
  if (!out) return fail(HG_ERR_INVALID, "out must be non-NULL");
  *out = nullptr;
  if (!arena) return fail(HG_ERR_INVALID, "arena must be non-NULL");
  if (max_active < 1) return fail(HG_ERR_INVALID, "max_active must be >= 1");
  table_bytes = table_bytes / 512 * 512;
  if (table_bytes < 2 * 65536 || table_bytes >= arena_bytes)
    return fail(HG_ERR_WORKSPACE, "table_bytes must be at least 128 KiB and below arena_bytes");
  if (sched)
    for (int c = 0; c < HG_SIZE_CLASSES; ++c)
      if (!hg::valid_schedule(sched[c]))
        return fail(HG_ERR_INVALID, "schedule of size class %d is out of range", c);
  hg_server_s* s = new (std::nothrow) hg_server_s();
  if (!s) return fail(HG_ERR_INVALID, "out of host memory");
  s->arena = (char*)arena;
  s->table_half = table_bytes / 2;
  s->job_base = s->arena + table_bytes;
  s->mem.reset(new hg::RangeAlloc(arena_bytes - table_bytes));
  s->max_active = max_active;
  memcpy(s->sched, sched ? sched : hg::kDefaultSchedule, sizeof(s->sched));
  s->t0 = hg::Clock::now();
  hipError_t e = hipGetDevice(&s->device);
  for (int h = 0; h < 2 && e == hipSuccess; ++h) {
    e = hipHostMalloc((void**)&s->host_half[h], s->table_half, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->half_ev[h], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->load, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&s->epoch_ev);
  if (e == hipSuccess) e = hipEventRecord(s->epoch_ev, s->compute);
  if (e == hipSuccess) e = hipEventSynchronize(s->epoch_ev);
  if (e != hipSuccess) {
    hg_server_free(s);
    return hg::hip_fail(e, "server set-up");
  }
  s->epoch_ms = hg::now_ms(s);
  s->exec_thread = std::thread(hg::exec_loop, s);
  s->load_thread = std::thread(hg::load_loop, s);
  *out = s;
  return HG_OK;
}

hg_status hg_server_submit(hg_server s, const hg_request* r, int64_t* id) {
  if (!s || !r) return fail(HG_ERR_INVALID, "server and request must be non-NULL");
  if (r->n < 1 || r->m < 1 || r->P < r->m || r->P > 0x7fffffffLL)
    return fail(HG_ERR_UNSUPPORTED, "need n, m >= 1 and m <= P < 2^31");
  if (r->k < 2 || r->k > HG_MAX_K) return fail(HG_ERR_UNSUPPORTED, "k must lie in [2, %d]", HG_MAX_K);
  if (r->rounds < 1 || r->rounds > hg::kMaxRounds)
    return fail(HG_ERR_INVALID, "rounds must lie in [1, %d]", hg::kMaxRounds);
  if (!(r->eps > 0.0 && r->eps < 1.0)) return fail(HG_ERR_INVALID, "eps must lie in (0, 1)");
  if (!r->eptr || !r->pins || !r->part)
    return fail(HG_ERR_INVALID, "eptr, pins and part must be non-NULL");
  std::unique_ptr<hg::Job> j(new (std::nothrow) hg::Job());
  if (!j) return fail(HG_ERR_INVALID, "out of host memory");
  if (!hg::job_layout(r->n, r->m, r->P, r->k, r->rounds, r->vwgt != nullptr,
                      r->ewgt != nullptr, j->lay))
    return fail(HG_ERR_UNSUPPORTED, "unsupported job sizes");
  j->r = *r;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fatal != HG_OK) return fail(s->fatal, "%s", s->fatal_msg);
  j->id = (int64_t)s->jobs.size();
  if (id) *id = j->id;
  s->pending.push_back(j.get());
  s->jobs.push_back(std::move(j));
  s->st.submitted += 1;
  s->cv_exec.notify_one();
  return HG_OK;
}

double hg_server_now_ms(hg_server s) { return s ? hg::now_ms(s) : 0.0; }

hg_status hg_server_info(hg_server s, int64_t id, hg_request_info* out) {
  if (!s || !out) return fail(HG_ERR_INVALID, "server and out must be non-NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (id < 0 || id >= (int64_t)s->jobs.size()) return fail(HG_ERR_INVALID, "no job %lld", (long long)id);
  const hg::Job* j = s->jobs[id].get();
  out->state = j->state;
  out->status = j->status;
  out->arrival_ms = j->r.arrival_ms;
  out->admit_ms = j->admit_ms;
  out->loaded_ms = j->loaded_ms;
  out->done_ms = j->done_ms;
  out->footprint = (int64_t)j->lay.total;
  out->first_step = j->join_step;
  if (j->status != HG_OK) fail(j->status, "%s", j->msg);
  return HG_OK;
}

hg_status hg_server_drain(hg_server s, double timeout_ms, int64_t* outstanding) {
  if (!s) return fail(HG_ERR_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] { return s->st.completed + s->st.failed >= s->st.submitted; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, done);
  } else {
    s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), done);
  }
  if (outstanding) *outstanding = s->st.submitted - s->st.completed - s->st.failed;
  if (s->fatal != HG_OK) return fail(s->fatal, "%s", s->fatal_msg);
  return HG_OK;
}

hg_status hg_server_get_stats(hg_server s, hg_server_stats* out) {
  if (!s || !out) return fail(HG_ERR_INVALID, "server and out must be non-NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return HG_OK;
}

void hg_server_free(hg_server s) {
  if (!s) return;
  if (s->exec_thread.joinable() || s->load_thread.joinable()) {
    (void)hg_server_drain(s, -1.0, nullptr);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_exec.notify_all();
    s->cv_load.notify_all();
    if (s->exec_thread.joinable()) s->exec_thread.join();
    if (s->load_thread.joinable()) s->load_thread.join();
  }
  for (auto& j : s->jobs) {
    if (j->done_ev) (void)hipEventDestroy(j->done_ev);
    if (j->g) hg_free(j->g);
  }
  for (hipEvent_t e : s->step_ev_pool) (void)hipEventDestroy(e);
  if (s->compute) (void)hipStreamSynchronize(s->compute);
  if (s->load) (void)hipStreamSynchronize(s->load);
  for (int h = 0; h < 2; ++h) {
    if (s->half_ev[h]) (void)hipEventDestroy(s->half_ev[h]);
    if (s->host_half[h]) (void)hipHostFree(s->host_half[h]);
  }
  if (s->epoch_ev) (void)hipEventDestroy(s->epoch_ev);
  if (s->compute) (void)hipStreamDestroy(s->compute);
  if (s->load) (void)hipStreamDestroy(s->load);
  delete s;
}

}  // extern "C"
