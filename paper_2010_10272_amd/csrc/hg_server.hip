// hg_server.hip -- the request server (hg_server_* in hgref.h): admission by
// device footprint into a caller arena, a loader thread, and an executor
// thread that advances every admitted job one label-propagation round per
// step in batched launches (continuous batching).
//
// Threads and streams
//   loader    copies a job's arrays in and runs hg_load_csr on the load
//             stream (which synchronizes that stream only)
//   executor  drives one or two lanes.  A lane is a set of jobs with its own
//             stream, work tables and step counter: per step it rebuilds the
//             tables when members joined or left, runs the pin-count pass of
//             the joiners, one round for every member, and queues the result
//             copies of members that ran their last round.  With two lanes,
//             jobs of at least `big_pins` pins take the second one, so small
//             jobs never wait for the round of a large one: both lanes' kernels
//             share the GPU.  The executor never blocks on the GPU; it polls
//             events and moves on to the other lane.
// Every stream has the default priority.  A job's memory is released only
// after the event recorded behind its result copies has completed, so no
// kernel can still read it.
//
// Work tables: each lane owns two halves of the table region, used
// alternately; a half is rebuilt only after the last step that read it has
// completed (its event).
#include <string.h>
#include <sys/prctl.h>

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
// Steps of a lane queued ahead of the GPU: two while a job for the lane is
// being loaded or waits to join (it joins at the next step the executor
// enqueues), more when none is coming, so that the rounds of the running
// jobs never wait for the executor thread to notice the previous one.
constexpr int kInFlightSteps = 2;
constexpr int kInFlightIdle = 8;

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
  int lane = 0;
  int64_t join_step = -1;
  int rounds_done = 0;
  bool finishing = false;
  hipEvent_t done_ev = nullptr;
  double admit_ms = 0, loaded_ms = 0, done_ms = 0;
};

using Clock = std::chrono::steady_clock;

constexpr int kMaxLanes = 2;

// Jobs advanced together on one stream (see the file comment).
struct Lane {
  hipStream_t stream = nullptr;
  char* table[2] = {nullptr, nullptr};   // device halves
  char* host[2] = {nullptr, nullptr};    // page-locked staging of each half
  size_t half_bytes = 0;
  hipEvent_t half_ev[2] = {nullptr, nullptr};
  bool half_used[2] = {false, false};
  int half = 1;
  RoundPlan rp;
  CountPlan cp;
  int64_t step = 0;
  bool changed = true;                   // membership differs from the current tables
  std::vector<Job*> active;              // executor-owned
  std::deque<Job*> ready;                // loaded, waiting to join (under the lock)
  std::deque<hipEvent_t> in_flight;      // events behind queued steps
};

}  // namespace
}  // namespace hg

struct hg_server_s {
  // fixed at creation
  char* arena = nullptr;
  int device = 0;
  int max_active = 1;
  int nlanes = 1;
  long long big_pins = 0;
  hg_schedule sched[HG_SIZE_CLASSES];
  hipStream_t load = nullptr;
  hipEvent_t epoch_ev = nullptr;
  double epoch_ms = 0;
  hg::Clock::time_point t0;
  std::unique_ptr<hg::RangeAlloc> mem;   // job memory (offsets after the table region)
  char* job_base = nullptr;
  hg::Lane lanes[hg::kMaxLanes];

  std::mutex mu;
  std::condition_variable cv_exec, cv_load, cv_done;
  bool stop = false;
  std::vector<std::unique_ptr<hg::Job>> jobs;
  std::deque<hg::Job*> pending, to_load;
  int loading_lane = -1;                // lane of the job the loader is loading
  int resident = 0;                     // admitted and not done
  hg_server_stats st{};
  hg_status fatal = HG_OK;
  char fatal_msg[160] = "";

  // executor-owned
  std::vector<hipEvent_t> step_ev_pool;

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

// Short waits of the server threads: the kernel's default timer slack
// (50 us) would stretch every 20 us poll several times over.
void precise_waits() { (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL); }

void load_loop(hg_server_s* s) {
  (void)hipSetDevice(s->device);
  precise_waits();
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_load.wait(lk, [&] { return s->stop || !s->to_load.empty(); });
    if (s->to_load.empty()) {
      if (s->stop) break;
      continue;
    }
    // small jobs first (in arrival order): a queued large load never delays them
    auto it = s->to_load.begin();
    while (it != s->to_load.end() && (*it)->lane != 0) ++it;
    if (it == s->to_load.end()) it = s->to_load.begin();
    Job* j = *it;
    s->to_load.erase(it);
    s->loading_lane = j->lane;
    lk.unlock();
    const hg_status st = load_job(s, j);
    char msg[160];
    snprintf(msg, sizeof(msg), "%s", st == HG_OK ? "" : hg_last_error());
    lk.lock();
    s->loading_lane = -1;
    if (st == HG_OK) {
      j->loaded_ms = now_ms(s);
      s->lanes[j->lane].ready.push_back(j);
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
  for (int li = 0; li < s->nlanes; ++li) {
    Lane& ln = s->lanes[li];
    std::vector<Job*> keep;
    for (Job* j : ln.active) {
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
    ln.active.swap(keep);
  }
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
    j->lane = s->nlanes > 1 && j->r.P >= s->big_pins ? 1 : 0;
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

// True when lane `ln` may rebuild its tables now (the half it would write is
// no longer read by a queued step).
bool half_free(const Lane& ln) {
  const int h = ln.half ^ 1;
  return !ln.half_used[h] || hipEventQuery(ln.half_ev[h]) != hipErrorNotReady;
}

// Enqueue one step of lane `ln` for the members in `run` (joiners last, `nj`
// of them); rebuild the tables when the lane's membership changed.  A step
// of one member launches the single-instance plans instead (the kernels of
// hg_refine, no table), which spares a lone job the table rebuilds.
hipError_t enqueue_step(hg_server_s* s, Lane& ln, const std::vector<Job*>& run, size_t nj) {
  hipStream_t cs = ln.stream;
  hipError_t e = hipSuccess;
  if (run.size() == 1) {
    const BatchMember M = member_of(s, run[0]);
    InstDesc d = make_desc(M.g, M.k, M.lmax, M.part, M.phi, M.netstate, M.block_w, M.eligible,
                           nullptr, M.km1, M.stats);
    d.round_base = M.round_base;
    if (nj > 0) {
      CountPlan cp;
      single_count_plan(d, cp);
      e = launch_counts(cp, true, true, cs);
      if (e != hipSuccess) return e;
    }
    RoundPlan rp;
    single_round_plan(d, rp);
    ln.changed = true;   // the tables (if any) describe another membership
    return launch_round(rp, (int)ln.step, cs, nullptr);
  }
  if (ln.changed) {
    const int h = ln.half ^ 1;   // free: checked by the caller (half_free)
    std::vector<BatchMember> mem;
    std::vector<int> all, join;
    for (size_t i = 0; i < run.size(); ++i) {
      mem.push_back(member_of(s, run[i]));
      all.push_back((int)i);
      if (i + nj >= run.size()) join.push_back((int)i);
    }
    size_t end = build_plans(mem, all, s->sched, ln.table[h], ln.host[h], 0, ln.half_bytes, &ln.rp,
                             nullptr);
    if (end && !join.empty())
      end = build_plans(mem, join, s->sched, ln.table[h], ln.host[h], end, ln.half_bytes, nullptr,
                        &ln.cp);
    if (end == 0) return hipErrorOutOfMemory;   // checked by the caller beforehand
    e = hipMemcpyAsync(ln.table[h], ln.host[h], end, hipMemcpyHostToDevice, cs);
    if (e != hipSuccess) return e;
    ln.half = h;
    ln.changed = false;
    s->st.rebuilds += 1;
  }
  if (nj > 0) {
    e = launch_counts(ln.cp, true, true, cs);
    if (e != hipSuccess) return e;
  }
  e = launch_round(ln.rp, (int)ln.step, cs, nullptr);
  if (e != hipSuccess) return e;
  e = hipEventRecord(ln.half_ev[ln.half], cs);
  ln.half_used[ln.half] = true;
  return e;
}

// Queue the result copies of a job that ran its last round.
hipError_t enqueue_results(hg_server_s* s, Job* j) {
  const hg_request& r = j->r;
  const JobLayout& L = j->lay;
  hipStream_t cs = s->lanes[j->lane].stream;
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

// Fail every job that cannot finish after a device error (nothing new is
// admitted then, so the memory of stuck members is simply abandoned).
void fail_all(hg_server_s* s) {
  while (!s->pending.empty()) {
    finish_failed(s, s->pending.front(), s->fatal, s->fatal_msg);
    s->pending.pop_front();
  }
  for (int li = 0; li < s->nlanes; ++li) {
    Lane& ln = s->lanes[li];
    while (!ln.ready.empty()) {
      Job* j = ln.ready.front();
      ln.ready.pop_front();
      hg_free(j->g);
      j->g = nullptr;
      s->mem->give(j->off, j->lay.total);
      s->resident -= 1;
      finish_failed(s, j, s->fatal, s->fatal_msg);
    }
    std::vector<Job*> keep;
    for (Job* j : ln.active) {
      if (j->finishing) {
        keep.push_back(j);
        continue;
      }
      s->resident -= 1;
      finish_failed(s, j, s->fatal, s->fatal_msg);
    }
    ln.active.swap(keep);
  }
}

// The members of lane `ln`'s next step: its running jobs plus as many
// loaded jobs as its table half can describe (those get join_step set).
// Returns the number of joiners (appended last to `run`).
size_t gather_step(hg_server_s* s, Lane& ln, std::vector<Job*>& run) {
  run.clear();
  for (Job* j : ln.active)
    if (!j->finishing) run.push_back(j);
  size_t nj = 0;
  while (!ln.ready.empty()) {
    Job* j = ln.ready.front();
    std::vector<BatchMember> mem;
    std::vector<int> all;
    for (size_t i = 0; i < run.size(); ++i) {
      mem.push_back(member_of(s, run[i]));
      all.push_back((int)i);
    }
    j->join_step = ln.step;
    mem.push_back(member_of(s, j));
    all.push_back((int)run.size());
    // round tables of everyone plus count tables of the joiners
    if (table_bound(mem, all) * 2 > ln.half_bytes) {
      if (run.empty()) {
        ln.ready.pop_front();
        hg_free(j->g);
        j->g = nullptr;
        s->mem->give(j->off, j->lay.total);
        s->resident -= 1;
        finish_failed(s, j, HG_ERR_WORKSPACE, "job too large for the server's table region");
        continue;
      }
      break;
    }
    ln.ready.pop_front();
    run.push_back(j);
    ++nj;
  }
  return nj;
}

void exec_loop(hg_server_s* s) {
  (void)hipSetDevice(s->device);
  precise_waits();
  std::unique_lock<std::mutex> lk(s->mu);
  std::vector<Job*> run;
  for (;;) {
    retire(s);
    admit(s);
    if (s->fatal != HG_OK) fail_all(s);
    if (s->stop && s->resident == 0 && s->pending.empty()) break;
    bool stepped = false;
    for (int li = 0; li < s->nlanes; ++li) {
      Lane& ln = s->lanes[li];
      // steps of this lane queued ahead of the GPU: few while a job for it
      // is on its way (it joins at the next enqueued step)
      while (!ln.in_flight.empty() && hipEventQuery(ln.in_flight.front()) != hipErrorNotReady) {
        s->step_ev_pool.push_back(ln.in_flight.front());
        ln.in_flight.pop_front();
      }
      bool incoming = !ln.ready.empty() || s->loading_lane == li;
      for (const Job* j : s->to_load) incoming = incoming || j->lane == li;
      if ((int)ln.in_flight.size() >= (incoming ? kInFlightSteps : kInFlightIdle)) continue;
      const bool wants_rebuild = ln.changed || !ln.ready.empty();
      if (wants_rebuild && !half_free(ln)) continue;
      const size_t nj = gather_step(s, ln, run);
      if (run.empty()) continue;
      if (nj > 0) ln.changed = true;
      lk.unlock();
      hipError_t e = enqueue_step(s, ln, run, nj);
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
        e = hipEventRecord(se, ln.stream);
        ln.in_flight.push_back(se);
      }
      lk.lock();
      if (e != hipSuccess && s->fatal == HG_OK) {
        s->fatal = HG_ERR_DEVICE;
        snprintf(s->fatal_msg, sizeof(s->fatal_msg), "server step: %s", hipGetErrorString(e));
      }
      for (size_t i = run.size() - nj; i < run.size(); ++i) {
        run[i]->state = HG_REQ_ACTIVE;
        ln.active.push_back(run[i]);
      }
      s->st.steps += 1;
      s->st.member_rounds += (int64_t)run.size();
      s->st.pin_rounds += pins;
      s->st.max_members = std::max<int64_t>(s->st.max_members, (int64_t)run.size());
      ln.step += 1;
      if (!leaving.empty()) ln.changed = true;
      stepped = true;
    }
    if (!stepped) {
      // Nothing could start.  Submits and finished loads notify; the GPU is
      // polled (every 20 us while steps or results are outstanding).
      bool busy = false;
      for (int li = 0; li < s->nlanes; ++li)
        busy = busy || !s->lanes[li].active.empty() || !s->lanes[li].in_flight.empty();
      if (busy)
        s->cv_exec.wait_for(lk, std::chrono::microseconds(20));
      else
        s->cv_exec.wait_for(lk, std::chrono::milliseconds(1));
    }
  }
  lk.unlock();
  for (int li = 0; li < s->nlanes; ++li) {
    Lane& ln = s->lanes[li];
    while (!ln.in_flight.empty()) {
      (void)hipEventSynchronize(ln.in_flight.front());
      s->step_ev_pool.push_back(ln.in_flight.front());
      ln.in_flight.pop_front();
    }
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
                           int32_t max_active, int64_t big_pins, const hg_schedule* sched,
                           hg_server* out) {
  if (!out) return fail(HG_ERR_INVALID, "out must be non-NULL");
  *out = nullptr;
  if (!arena) return fail(HG_ERR_INVALID, "arena must be non-NULL");
  if (max_active < 1) return fail(HG_ERR_INVALID, "max_active must be >= 1");
  if (big_pins < 0) return fail(HG_ERR_INVALID, "big_pins must be >= 0");
  const int nlanes = big_pins > 0 ? 2 : 1;
  const size_t quarter = table_bytes / (2 * nlanes) / 256 * 256;
  if (quarter < 65536 || table_bytes >= arena_bytes)
    return fail(HG_ERR_WORKSPACE, "table_bytes must be at least %d KiB and below arena_bytes",
                nlanes * 128);
  if (sched)
    for (int c = 0; c < HG_SIZE_CLASSES; ++c)
      if (!hg::valid_schedule(sched[c]))
        return fail(HG_ERR_INVALID, "schedule of size class %d is out of range", c);
  hg_server_s* s = new (std::nothrow) hg_server_s();
  if (!s) return fail(HG_ERR_INVALID, "out of host memory");
  s->arena = (char*)arena;
  s->nlanes = nlanes;
  s->big_pins = big_pins;
  s->job_base = s->arena + table_bytes;
  s->mem.reset(new hg::RangeAlloc(arena_bytes - table_bytes));
  s->max_active = max_active;
  // without a schedule: one unit per work item (a step usually holds a few
  // jobs, which then get the most workgroups; the batch defaults group units
  // for batches of hundreds)
  static const hg_schedule kServerSchedule[HG_SIZE_CLASSES] = {
      {1, 1, 1, 0}, {1, 1, 1, 0}, {1, 1, 1, 0}, {1, 1, 1, 0}};
  memcpy(s->sched, sched ? sched : kServerSchedule, sizeof(s->sched));
  s->t0 = hg::Clock::now();
  hipError_t e = hipGetDevice(&s->device);
  for (int li = 0; li < nlanes && e == hipSuccess; ++li) {
    hg::Lane& ln = s->lanes[li];
    ln.half_bytes = quarter;
    for (int h = 0; h < 2 && e == hipSuccess; ++h) {
      ln.table[h] = s->arena + (size_t)(2 * li + h) * quarter;
      e = hipHostMalloc((void**)&ln.host[h], quarter, hipHostMallocDefault);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ln.half_ev[h], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->load, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&s->epoch_ev);
  if (e == hipSuccess) e = hipEventRecord(s->epoch_ev, s->lanes[0].stream);
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
  if (s->load) (void)hipStreamSynchronize(s->load);
  for (int li = 0; li < hg::kMaxLanes; ++li) {
    hg::Lane& ln = s->lanes[li];
    if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    for (int h = 0; h < 2; ++h) {
      if (ln.half_ev[h]) (void)hipEventDestroy(ln.half_ev[h]);
      if (ln.host[h]) (void)hipHostFree(ln.host[h]);
    }
    if (ln.stream) (void)hipStreamDestroy(ln.stream);
  }
  if (s->epoch_ev) (void)hipEventDestroy(s->epoch_ev);
  if (s->load) (void)hipStreamDestroy(s->load);
  delete s;
}

}  // extern "C"
