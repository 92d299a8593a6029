// hg_batch.hip -- batches of independent refinements (hg_batch_* in hgref.h)
// and the work-table builder they share with the request server.
//
// A batch is a set of members (loaded hypergraph + partition state).  The
// host builds one work table per kernel launch of a round (and of the
// pin-count pass that starts a refinement), copies the tables and the
// members' descriptors into a device table buffer, and then every round is
// the same dozen launches whatever the number of members.
//
// Placement: the sweeps (select, finalize, pin counts, block weights) keep a
// member on one XCD -- members are assigned to the eight XCDs by longest
// processing time first on their pin + vertex count, and a member larger
// than 1/16 of the whole batch is spread over all eight.  Their work items
// are queued per XCD (see Launch in hg_internal.h).  The per-block and
// per-tile kernels (thresholds, tile sums and scans, approve) take one item
// per workgroup in member order.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "hg_batch.h"

namespace hg {

const hg_schedule kDefaultSchedule[HG_SIZE_CLASSES] = {
    {1, 1, 1, 0}, {2, 2, 2, 0}, {4, 4, 4, 0}, {8, 8, 8, 0}};

namespace {

constexpr int kMaxScheduleChunks = 64;
constexpr int kHeavyPerGroup = kBlock / kWave;   // heavy vertices per select workgroup
constexpr size_t kLaunchSlack = 32 * 256;       // 256-byte alignment of every launch's table

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

int net_lanes(int k, int want) { return want > group_lanes(k) ? want : group_lanes(k); }

// Work items of one launch, queued per XCD (split) or in one list.
struct KindItems {
  void* kernel = nullptr;
  size_t lds = 0;
  std::vector<WorkItem> q[kNumXcd];
  std::vector<WorkItem> flat;
};

KindItems* variant(std::vector<KindItems>& v, void* kernel) {
  for (KindItems& x : v)
    if (x.kernel == kernel) return &x;
  v.push_back(KindItems());
  v.back().kernel = kernel;
  return &v.back();
}

// Items of `units` units in pieces of `per` for member `inst`, to its XCD (or
// spread over all XCDs in eight contiguous parts when xcd < 0).
void add_split(KindItems& kind, int inst, long long units, int per, int xcd) {
  std::vector<WorkItem> items;
  for (long long f = 0; f < units; f += per) {
    WorkItem w;
    w.inst = inst;
    w.first = (int)f;
    w.count = (int)std::min<long long>(per, units - f);
    w.stride = 1;
    items.push_back(w);
  }
  if (xcd >= 0) {
    kind.q[xcd].insert(kind.q[xcd].end(), items.begin(), items.end());
    return;
  }
  const size_t len = items.size();
  for (int x = 0; x < kNumXcd; ++x) {
    const size_t lo = len * x / kNumXcd, hi = len * (x + 1) / kNumXcd;
    kind.q[x].insert(kind.q[x].end(), items.begin() + lo, items.begin() + hi);
  }
}

}  // namespace

int size_class(int n) {
  if (n < (1 << 13)) return 0;
  if (n < (1 << 16)) return 1;
  if (n < (1 << 19)) return 2;
  return 3;
}

bool valid_schedule(const hg_schedule& s) {
  auto chunks_ok = [](int c) { return c >= 1 && c <= kMaxScheduleChunks; };
  const int l = s.net_lanes;
  return chunks_ok(s.select_chunks) && chunks_ok(s.finalize_chunks) &&
         chunks_ok(s.count_chunks) && (l == 0 || l == 4 || l == 8 || l == 16 || l == 32);
}

size_t table_bound(const std::vector<BatchMember>& mem, const std::vector<int>& which) {
  long long items = 0;
  for (int i : which) {
    const BatchMember& x = mem[i];
    const hg_graph_s* g = x.g;
    const long long tiles = ceil_div(g->n, kTile);
    items += ceil_div(g->n, kBlock);                                 // select
    items += ceil_div(g->info.heavy_count, kHeavyPerGroup);          // heavy select
    items += x.k;                                                    // per block
    items += tiles;                                                  // tile sums
    items += tiles + x.k;                                            // approve
    items += ceil_div(g->m, kFinalChunk);                            // finalize
    items += ceil_div(g->m, kBlock);                                 // pin counts
    items += ceil_div(g->n, kBwChunk);                               // block weights
    items += 2;                                                      // per member
  }
  return align256(sizeof(InstDesc) * which.size()) + sizeof(WorkItem) * (size_t)items +
         kLaunchSlack;
}

size_t build_plans(const std::vector<BatchMember>& mem, const std::vector<int>& which,
                   const hg_schedule* sched, char* dev, char* host, size_t at, size_t cap,
                   RoundPlan* rp, CountPlan* cp) {
  const int cnt = (int)which.size();
  // XCD placement: longest processing time first on P + n
  std::vector<long long> cost(cnt);
  long long total = 0;
  for (int i = 0; i < cnt; ++i) {
    const hg_graph_s* g = mem[which[i]].g;
    cost[i] = g->P + g->n;
    total += cost[i];
  }
  std::vector<int> order(cnt), home(cnt, -1);
  for (int i = 0; i < cnt; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
  long long load[kNumXcd] = {0};
  for (int i : order) {
    if (cost[i] * 16 > total) continue;   // spread over every XCD
    int best = 0;
    for (int x = 1; x < kNumXcd; ++x)
      if (load[x] < load[best]) best = x;
    home[i] = best;
    load[best] += cost[i];
  }

  std::vector<InstDesc> descs(cnt);
  std::vector<KindItems> sel, fin, pc;
  KindItems heavy, blocks, tiles, approve, inst, verts;
  bool any_heavy = false;
  for (int i = 0; i < cnt; ++i) {
    const BatchMember& M = mem[which[i]];
    hg_graph_s* g = M.g;
    const hg_schedule& S = sched[M.cls];
    InstDesc d = make_desc(g, M.k, M.lmax, M.part, M.phi, M.netstate, M.block_w, M.eligible,
                           nullptr, M.km1, M.stats);
    d.hist_reps = home[i] < 0 ? kHistReplicas : 1;
    d.round_base = M.round_base;
    descs[i] = d;
    const int k = M.k;
    const int G = net_lanes(k, S.net_lanes);
    if (rp) {
      add_split(*variant(sel, (void*)select_kernel(k, d.view, d.P, d.n)), i, ceil_div(g->n, kBlock),
                S.select_chunks, home[i]);
      add_split(*variant(fin, (void*)finalize_kernel_g(G, false)), i, ceil_div(g->m, kFinalChunk),
                S.finalize_chunks, home[i]);
      for (long long h = 0; h < ceil_div(g->info.heavy_count, kHeavyPerGroup); ++h)
        heavy.flat.push_back(WorkItem{i, (int)h, 1, 1});
      if (g->info.heavy_count > 0) any_heavy = true;
      for (int t = 0; t < k; ++t) blocks.flat.push_back(WorkItem{i, t, 1, 1});
      for (int t = 0; t < d.num_tiles; ++t) tiles.flat.push_back(WorkItem{i, t, 1, 1});
      for (int t = 0; t < d.num_tiles; ++t) approve.flat.push_back(WorkItem{i, t, 1, 1});
      for (int t = 0; t < k; ++t) approve.flat.push_back(WorkItem{i, t, -1, 1});
    }
    if (cp) {
      KindItems* p = variant(pc, (void*)pincount_kernel_g(G));
      add_split(*p, i, ceil_div(g->m, kBlock / G), S.count_chunks * G, home[i]);
      p->lds = std::max(p->lds, pincount_lds(G, k));
      add_split(verts, i, ceil_div(g->n, kBwChunk), 1, home[i]);
    }
    inst.flat.push_back(WorkItem{i, 0, 1, 1});
  }

  // serialize: descriptors, then every launch's items (256-byte aligned)
  size_t off = align256(at);
  const size_t desc_at = off;
  if (off + sizeof(InstDesc) * cnt > cap) return 0;
  memcpy(host + off, descs.data(), sizeof(InstDesc) * cnt);
  off += sizeof(InstDesc) * cnt;
  Launch base;
  memset(&base, 0, sizeof(base));
  base.descs = (const InstDesc*)(dev + desc_at);
  bool ok = true;
  auto put = [&](const WorkItem* src, size_t n) {
    if (!ok || off + sizeof(WorkItem) * n > cap) {
      ok = false;
      return;
    }
    memcpy(host + off, src, sizeof(WorkItem) * n);
    off += sizeof(WorkItem) * n;
  };
  auto emit_split = [&](const KindItems& kind, PlanLaunch& pl) {
    off = align256(off);
    Launch L = base;
    L.items = (const WorkItem*)(dev + off);
    L.split = 1;
    size_t run = 0, longest = 0;
    for (int x = 0; x < kNumXcd; ++x) {
      L.xoff[x] = (int)run;
      put(kind.q[x].data(), kind.q[x].size());
      run += kind.q[x].size();
      longest = std::max(longest, kind.q[x].size());
    }
    L.xoff[kNumXcd] = (int)run;
    pl.kernel = kind.kernel;
    pl.lds = kind.lds;
    pl.grid = (unsigned)(longest * kNumXcd);
    pl.L = L;
  };
  auto emit_flat = [&](const KindItems& kind, PlanLaunch& pl) {
    off = align256(off);
    Launch L = base;
    L.items = (const WorkItem*)(dev + off);
    L.split = 0;
    put(kind.flat.data(), kind.flat.size());
    pl.kernel = kind.kernel;
    pl.grid = (unsigned)kind.flat.size();
    pl.L = L;
  };
  if (rp) {
    *rp = RoundPlan();
    for (const KindItems& k : sel) {
      rp->select.push_back(PlanLaunch());
      emit_split(k, rp->select.back());
    }
    if (any_heavy) {
      rp->heavy.push_back(PlanLaunch());
      emit_flat(heavy, rp->heavy.back());
      rp->any_heavy = true;
    }
    emit_flat(blocks, rp->blocks);
    emit_flat(tiles, rp->tiles);
    emit_flat(approve, rp->approve);
    for (const KindItems& k : fin) {
      rp->finalize.push_back(PlanLaunch());
      emit_split(k, rp->finalize.back());
    }
    emit_flat(inst, rp->stats);
  }
  if (cp) {
    *cp = CountPlan();
    for (const KindItems& k : pc) {
      cp->pincounts.push_back(PlanLaunch());
      emit_split(k, cp->pincounts.back());
    }
    emit_flat(inst, cp->instances);
    emit_split(verts, cp->vertices);
  }
  return ok ? off : 0;
}

}  // namespace hg

struct hg_batch_s {
  std::vector<hg::BatchMember> members;
  hg_schedule sched[HG_SIZE_CLASSES];
  char* table = nullptr;        // device
  size_t table_bytes = 0;
  char* host = nullptr;         // pinned staging copy of the table
  size_t host_bytes = 0;
  hipEvent_t copied = nullptr;  // the last table copy
  bool copy_pending = false;
  hg::RoundPlan round;
  hg::CountPlan counts;
  unsigned long long table_gen = 0;
  void* graph_exec = nullptr;
  void* cap_stream = nullptr;
  int graph_rounds = -1;
  unsigned long long graph_gen = 0;
};

namespace hg {
namespace {

std::vector<int> iota_vec(size_t n) {
  std::vector<int> v(n);
  for (size_t i = 0; i < n; ++i) v[i] = (int)i;
  return v;
}

// Build the tables of members `which` with `sched` and copy them to the
// batch's device table on `s` (after the previous copy has left the staging
// buffer).
hg_status build_tables(hg_batch_s* b, const std::vector<int>& which, const hg_schedule* sched,
                       hipStream_t s, RoundPlan& rp, CountPlan& cp) {
  if (b->copy_pending) {
    HG_TRY(hipEventSynchronize(b->copied), "hipEventSynchronize");
    b->copy_pending = false;
  }
  const size_t end = build_plans(b->members, which, sched, b->table, b->host, 0,
                                 std::min(b->host_bytes, b->table_bytes), &rp, &cp);
  if (end == 0) return fail(HG_ERR_WORKSPACE, "batch table too small");
  HG_TRY(hipMemcpyAsync(b->table, b->host, end, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
  HG_TRY(hipEventRecord(b->copied, s), "hipEventRecord");
  b->copy_pending = true;
  b->table_gen += 1;
  return HG_OK;
}

hg_status build_all(hg_batch_s* b, hipStream_t s) {
  return build_tables(b, iota_vec(b->members.size()), b->sched, s, b->round, b->counts);
}

void drop_graph(hg_batch_s* b) {
  if (b->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)b->graph_exec);
  b->graph_exec = nullptr;
  b->graph_rounds = -1;
}

hipError_t enqueue_batch(const RoundPlan& rp, const CountPlan& cp, int rounds, hipStream_t s) {
  hipError_t e = launch_counts(cp, true, true, s);
  for (int r = 0; r < rounds && e == hipSuccess; ++r) e = launch_round(rp, r, s, nullptr);
  return e;
}

hg_status check_members(const hg_instance* mem, int count, std::vector<BatchMember>& out) {
  if (!mem || count < 1) return fail(HG_ERR_INVALID, "a batch needs at least one member");
  out.resize(count);
  std::vector<const void*> graphs(count);
  for (int i = 0; i < count; ++i) {
    const hg_instance& x = mem[i];
    hg_status st = check_k(x.g, x.k);
    if (st != HG_OK) return fail(st, "member %d: %s", i, hg_last_error());
    if (!(x.eps > 0.0 && x.eps < 1.0))
      return fail(HG_ERR_INVALID, "member %d: eps must lie in (0, 1)", i);
    if (!x.part || !x.phi || !x.netstate || !x.block_w || !x.eligible || !x.stats || !x.km1)
      return fail(HG_ERR_INVALID,
                  "member %d: part, phi, netstate, block_w, eligible, stats and km1 must be "
                  "non-NULL", i);
    BatchMember& M = out[i];
    M.g = x.g;
    M.k = x.k;
    M.cls = size_class(x.g->n);
    M.round_base = 0;
    M.lmax = hg_max_block_weight(x.g, x.k, x.eps);
    M.part = x.part;
    M.phi = x.phi;
    M.netstate = x.netstate;
    M.block_w = (long long*)x.block_w;
    M.eligible = x.eligible;
    M.stats = x.stats;
    M.km1 = (long long*)x.km1;
    graphs[i] = x.g;
  }
  std::sort(graphs.begin(), graphs.end());
  if (std::adjacent_find(graphs.begin(), graphs.end()) != graphs.end())
    return fail(HG_ERR_INVALID, "a graph handle appears in two members of the batch");
  return HG_OK;
}

}  // namespace
}  // namespace hg

using hg::fail;

extern "C" {

size_t hg_batch_table_bytes(const hg_instance* members, int32_t count) {
  std::vector<hg::BatchMember> mem;
  if (hg::check_members(members, count, mem) != HG_OK) return 0;
  return hg::table_bound(mem, hg::iota_vec(mem.size()));
}

hg_status hg_batch_get_schedule(hg_batch b, hg_schedule* sched) {
  if (!sched) return fail(HG_ERR_INVALID, "sched must be non-NULL");
  memcpy(sched, b ? b->sched : hg::kDefaultSchedule, sizeof(hg_schedule) * HG_SIZE_CLASSES);
  return HG_OK;
}

hg_status hg_batch_create(const hg_instance* members, int32_t count, const hg_schedule* sched,
                          void* table, size_t table_bytes, void* stream, hg_batch* out) {
  if (!out) return fail(HG_ERR_INVALID, "out must be non-NULL");
  *out = nullptr;
  std::vector<hg::BatchMember> mem;
  hg_status st = hg::check_members(members, count, mem);
  if (st != HG_OK) return st;
  if (sched)
    for (int c = 0; c < HG_SIZE_CLASSES; ++c)
      if (!hg::valid_schedule(sched[c]))
        return fail(HG_ERR_INVALID, "schedule of size class %d is out of range", c);
  const size_t need = hg::table_bound(mem, hg::iota_vec(mem.size()));
  if (!table || table_bytes < need)
    return fail(HG_ERR_WORKSPACE, "batch table needs %zu bytes (got %zu)", need, table_bytes);
  hg_batch_s* b = new (std::nothrow) hg_batch_s();
  if (!b) return fail(HG_ERR_INVALID, "out of host memory");
  b->members.swap(mem);
  memcpy(b->sched, sched ? sched : hg::kDefaultSchedule, sizeof(b->sched));
  b->table = (char*)table;
  b->table_bytes = table_bytes;
  b->host_bytes = need;
  hipError_t e = hipHostMalloc((void**)&b->host, need, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied, hipEventDisableTiming);
  if (e != hipSuccess) {
    hg_batch_free(b);
    return hg::hip_fail(e, "batch set-up");
  }
  st = hg::build_all(b, (hipStream_t)stream);
  if (st != HG_OK) {
    hg_batch_free(b);
    return st;
  }
  *out = b;
  return HG_OK;
}

void hg_batch_free(hg_batch b) {
  if (!b) return;
  if (b->copy_pending) (void)hipEventSynchronize(b->copied);
  hg::drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy((hipStream_t)b->cap_stream);
  if (b->copied) (void)hipEventDestroy(b->copied);
  if (b->host) (void)hipHostFree(b->host);
  delete b;
}

hg_status hg_batch_start(hg_batch b, void* stream) {
  if (!b) return fail(HG_ERR_INVALID, "batch handle is NULL");
  HG_TRY(hg::launch_counts(b->counts, true, true, (hipStream_t)stream), "batch start");
  return HG_OK;
}

hg_status hg_batch_round(hg_batch b, int32_t round, void* stream) {
  if (!b) return fail(HG_ERR_INVALID, "batch handle is NULL");
  if (round < 0) return fail(HG_ERR_INVALID, "round must be >= 0");
  HG_TRY(hg::launch_round(b->round, round, (hipStream_t)stream, nullptr), "batch round");
  return HG_OK;
}

hg_status hg_batch_refine(hg_batch b, int32_t rounds, int32_t use_graph, void* stream) {
  if (!b) return fail(HG_ERR_INVALID, "batch handle is NULL");
  if (rounds < 0) return fail(HG_ERR_INVALID, "rounds must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  if (!use_graph) {
    HG_TRY(hg::enqueue_batch(b->round, b->counts, rounds, s), "batch refine");
    return HG_OK;
  }
  if (!b->graph_exec || b->graph_rounds != rounds || b->graph_gen != b->table_gen) {
    hg::drop_graph(b);
    if (!b->cap_stream) {
      hipStream_t cs;
      HG_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
      b->cap_stream = cs;
    }
    hipStream_t cs = (hipStream_t)b->cap_stream;
    HG_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e = hg::enqueue_batch(b->round, b->counts, rounds, cs);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hg::hip_fail(e, "batch capture");
    }
    if (e2 != hipSuccess) return hg::hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hg::hip_fail(e, "hipGraphInstantiate");
    b->graph_exec = exec;
    b->graph_rounds = rounds;
    b->graph_gen = b->table_gen;
  }
  HG_TRY(hipGraphLaunch((hipGraphExec_t)b->graph_exec, s), "hipGraphLaunch");
  return HG_OK;
}

hg_status hg_batch_autotune(hg_batch b, int32_t* part_save, int64_t save_elems, int32_t repeats,
                            void* stream, hg_schedule* best) {
  if (!b) return fail(HG_ERR_INVALID, "batch handle is NULL");
  if (repeats < 1 || repeats > 100) return fail(HG_ERR_INVALID, "repeats must lie in [1, 100]");
  hipStream_t s = (hipStream_t)stream;
  const int cnt = (int)b->members.size();
  std::vector<long long> save_off(cnt);
  long long need = 0;
  for (int i = 0; i < cnt; ++i) {
    save_off[i] = need;
    need += b->members[i].g->n;
  }
  if (!part_save || save_elems < need)
    return fail(HG_ERR_WORKSPACE, "part_save needs %lld elements", need);
  for (int i = 0; i < cnt; ++i)
    HG_TRY(hipMemcpyAsync(part_save + save_off[i], b->members[i].part,
                          sizeof(int32_t) * b->members[i].g->n, hipMemcpyDeviceToDevice, s),
           "hipMemcpyAsync");
  auto restore = [&](const std::vector<int>& which) -> hg_status {
    for (int i : which)
      HG_TRY(hipMemcpyAsync(b->members[i].part, part_save + save_off[i],
                            sizeof(int32_t) * b->members[i].g->n, hipMemcpyDeviceToDevice, s),
             "hipMemcpyAsync");
    return HG_OK;
  };
  hipEvent_t ev[2];
  HG_TRY(hipEventCreate(&ev[0]), "hipEventCreate");
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(HG_ERR_DEVICE, "hipEventCreate failed");
  }
  hg_schedule cur[HG_SIZE_CLASSES];
  memcpy(cur, b->sched, sizeof(cur));
  hg_status st = HG_OK;
  hg::RoundPlan rp;
  hg::CountPlan cp;
  // time of start + one round for members `which` under schedule `trial`
  auto trial_ms = [&](const std::vector<int>& which, const hg_schedule* trial, float* best_ms) {
    hg_status r = hg::build_tables(b, which, trial, s, rp, cp);
    if (r != HG_OK) return r;
    *best_ms = 1e30f;
    for (int rep = 0; rep < repeats; ++rep) {
      if ((r = restore(which)) != HG_OK) return r;
      HG_TRY(hipEventRecord(ev[0], s), "hipEventRecord");
      HG_TRY(hg::enqueue_batch(rp, cp, 1, s), "tuning trial");
      HG_TRY(hipEventRecord(ev[1], s), "hipEventRecord");
      HG_TRY(hipEventSynchronize(ev[1]), "hipEventSynchronize");
      float ms = 0.0f;
      HG_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]), "hipEventElapsedTime");
      *best_ms = std::min(*best_ms, ms);
    }
    return (hg_status)HG_OK;
  };
  static const int kChunkCands[] = {1, 2, 4, 8, 16};
  static const int kLaneCands[] = {0, 8, 16, 32};
  for (int c = 0; c < HG_SIZE_CLASSES && st == HG_OK; ++c) {
    std::vector<int> which;
    for (int i = 0; i < cnt; ++i)
      if (b->members[i].cls == c) which.push_back(i);
    if (which.empty()) continue;
    for (int field = 0; field < 4 && st == HG_OK; ++field) {
      const int* cands = field == 3 ? kLaneCands : kChunkCands;
      const int ncand = field == 3 ? 4 : 5;
      int32_t* slot = field == 0   ? &cur[c].select_chunks
                      : field == 1 ? &cur[c].finalize_chunks
                      : field == 2 ? &cur[c].count_chunks
                                   : &cur[c].net_lanes;
      float best_t = 1e30f;
      int best_v = *slot;
      for (int j = 0; j < ncand && st == HG_OK; ++j) {
        *slot = cands[j];
        float t = 0.0f;
        st = trial_ms(which, cur, &t);
        if (st == HG_OK && t < best_t) {
          best_t = t;
          best_v = cands[j];
        }
      }
      *slot = best_v;
    }
  }
  if (st == HG_OK) st = restore(hg::iota_vec(cnt));
  if (st == HG_OK) {
    memcpy(b->sched, cur, sizeof(cur));
    st = hg::build_all(b, s);
  } else {
    (void)hg::build_all(b, s);
  }
  if (st == HG_OK && hipStreamSynchronize(s) != hipSuccess)
    st = fail(HG_ERR_DEVICE, "hipStreamSynchronize failed");
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (st == HG_OK && best) memcpy(best, b->sched, sizeof(b->sched));
  return st;
}

}  // extern "C"
