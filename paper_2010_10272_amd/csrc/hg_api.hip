// hg_api.hip -- the C ABI declared in include/hgref.h: argument checks,
// workspace carving, launch sequencing and the recorded refinement graph.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <array>
#include <vector>

#include "hg_internal.h"
#include "hg_sort.h"
#include "hg_lp.h"

namespace hg {
}

namespace {
thread_local char g_msg[512] = "";
}  // namespace

namespace hg {

hg_status fail(hg_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
  return code;
}

hg_status hip_fail(hipError_t e, const char* what) {
  return fail(HG_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

hg_status check_k(hg_graph g, int k) {
  if (!g) return fail(HG_ERR_INVALID, "graph handle is NULL");
  if (k < 2) return fail(HG_ERR_INVALID, "k must be at least 2 (got %d)", k);
  if (k > HG_MAX_K) return fail(HG_ERR_UNSUPPORTED, "k must be at most %d (got %d)", HG_MAX_K, k);
  if (k > g->k_max)
    return fail(HG_ERR_WORKSPACE, "k = %d exceeds the k_max = %d the workspace was sized for", k,
                g->k_max);
  return HG_OK;
}

}  // namespace hg

namespace {

using hg::check_k;
using hg::fail;
using hg::hip_fail;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr long long kMaxPins = 0x7fffffffLL;

const char* describe_err(int err) {
  if (err & hg::kErrCsr) return "net offsets must increase strictly from 0 to P (no empty net)";
  if (err & hg::kErrPin) return "a pin lies outside [0, n)";
  if (err & hg::kErrWeight) return "vertex and net weights must be positive";
  if (err & hg::kErrDuplicate) return "a vertex appears twice in one net (nets are sets)";
  if (err & hg::kErrPart) return "a partition id lies outside [0, k)";
  if (err & hg::kErrCluster) return "a cluster id lies outside [0, n)";
  if (err & hg::kErrClusterWeight) return "a cluster weighs 2^31 or more";
  if (err & hg::kErrMoves)
    return "a move sequence moves a vertex twice, to a block outside [0, k) or to its own block";
  return "invalid input";
}

hg_status read_info(hg_graph_s* g, hipStream_t s) {
  HG_TRY(hipMemcpyAsync(&g->info, g->ws + g->lay.info, sizeof(hg::LoadInfo),
                        hipMemcpyDeviceToHost, s),
         "hipMemcpyAsync");
  HG_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return HG_OK;
}

// Events of timed rounds.  Each round has four marks (round start, after
// select, after approve/apply, round end); `spans` keeps them for the
// elapsed times, `marks` the handles the launch records (the start left null
// when it is the previous round's end, which the launch then need not
// record again: each recorded mark costs a few microseconds of idle GPU).
// `pool` holds the events, reused after every collect.
struct TimingState {
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<std::array<hipEvent_t, 4>> marks, spans;
};

void release_timing(hg_graph_s* g) {
  TimingState* t = (TimingState*)g->timing_state;
  if (!t) return;
  for (hipEvent_t e : t->pool) (void)hipEventDestroy(e);
  delete t;
  g->timing_state = nullptr;
}

// The marks of the next round, or *marks = nullptr when timing is off or the
// stream is being captured.  With chain, the caller has enqueued nothing on
// the stream since the previous round's end mark, which then also starts
// this round.
hg_status timing_marks(hg_graph_s* g, hipStream_t s, hipEvent_t** marks, bool chain = false) {
  *marks = nullptr;
  if (!g->timing) return HG_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HG_TRY(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone) return HG_OK;
  TimingState* t = (TimingState*)g->timing_state;
  if (!t) {
    t = new (std::nothrow) TimingState();
    if (!t) return fail(HG_ERR_INVALID, "out of host memory");
    g->timing_state = t;
  }
  const bool shared = chain && !t->spans.empty();
  const size_t take = shared ? 3 : 4;
  while (t->pool.size() < t->next + take) {
    // timing only: without the system-scope fence, recording a mark costs no
    // cache writeback and invalidation between the phases it separates
    hipEvent_t e;
    HG_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreateWithFlags");
    t->pool.push_back(e);
  }
  std::array<hipEvent_t, 4> rec, span;
  for (int i = 0; i < 4; ++i) rec[i] = nullptr;
  for (size_t i = 0; i < take; ++i) rec[4 - take + i] = t->pool[t->next + i];
  span = rec;
  if (shared) span[0] = t->spans.back()[3];
  t->next += take;
  t->marks.push_back(rec);
  t->spans.push_back(span);
  *marks = t->marks.back().data();
  return HG_OK;
}

}  // namespace

namespace hg {

WsLayout ws_layout(int n, int m, long long P, int k_max) {
  WsLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  L.num_tiles = (int)(((long long)n + kTile - 1) / kTile);
  L.scan_blocks = (int)(((long long)n + kBlock * 8 - 1) / (kBlock * 8));
  L.cand = take(sizeof(long long) * (size_t)n);
  L.touched = take(touched_bytes(m));   // one flag byte per net, zero past m
  L.heavy = take(sizeof(int) * (size_t)n);
  L.big = take(sizeof(int) * (size_t)n);
  L.hist = take(sizeof(unsigned long long) * (size_t)kHistReplicas * k_max * kBuckets);
  L.overflow = take(sizeof(int) * (size_t)k_max);
  L.thr = take(sizeof(Threshold) * (size_t)k_max);
  L.tilesum = take(sizeof(long long) * (size_t)k_max * (size_t)L.num_tiles);
  L.ctr = take(sizeof(RoundCounters));
  L.info = take(sizeof(LoadInfo));
  L.scan = take(sizeof(long long) * (size_t)L.scan_blocks);
  L.flags = take(256);
  L.red = take(sizeof(unsigned long long) * kSlots);
  L.bw_slots = take(sizeof(long long) * kSlots * (size_t)k_max);
  L.part8 = take((size_t)n);
  L.lkey[0] = take(sizeof(unsigned) * (size_t)P);
  L.lkey[1] = take(sizeof(unsigned) * (size_t)P);
  L.lval = take(sizeof(int) * (size_t)P);
  L.lhist = take(sizeof(unsigned) * (size_t)kDigits * (size_t)sort_tiles(P));
  L.ldtot = take(sizeof(unsigned) * kDigits);
  L.lpart = take(sizeof(LoadPart) * kLoadGrid);
  L.total = off;
  return L;
}

InstDesc make_desc(hg_graph_s* g, int k, long long lmax, int* part, int* phi,
                   unsigned* netstate, long long* block_w, unsigned char* eligible,
                   unsigned char* moved, long long* km1, hg_round_stats* stats) {
  InstDesc d;
  memset(&d, 0, sizeof(d));
  char* ws = g->ws;
  d.n = g->n;
  d.m = g->m;
  d.P = g->P;
  d.k = k;
  d.rw = net_words(k);
  d.view = net_view(k, g->unit_nets);
  d.unit_nets = g->unit_nets ? 1 : 0;
  d.cmax = g->info.max_vertex_weight;
  d.lds_buckets = lds_buckets(k);
  d.heavy_count = g->info.heavy_count;
  d.num_tiles = g->lay.num_tiles;
  d.hist_stride = g->k_max * kBuckets;
  d.hist_reps = kHistReplicas;
  d.lmax = lmax;
  d.eptr = g->eptr;
  d.pins = g->pins;
  d.vwgt = g->vwgt;
  d.ewgt = g->ewgt;
  d.vptr = g->vptr;
  d.vnets = g->vnets;
  d.heavy_list = (const int*)(ws + g->lay.heavy);
  d.part = part;
  d.phi = phi;
  d.netstate = netstate;
  d.view_ptr = netstate ? netstate + (size_t)g->m * d.rw : nullptr;
  d.block_w = block_w;
  d.eligible = eligible;
  d.moved = moved;
  d.km1 = km1;
  d.stats = stats;
  d.cand = (long long*)(ws + g->lay.cand);
  d.touched = (unsigned char*)(ws + g->lay.touched);
  d.hist = (unsigned long long*)(ws + g->lay.hist);
  d.overflow = (int*)(ws + g->lay.overflow);
  d.thr = (Threshold*)(ws + g->lay.thr);
  d.tilesum = (long long*)(ws + g->lay.tilesum);
  d.ctr = (RoundCounters*)(ws + g->lay.ctr);
  d.err_flags = (int*)(ws + g->lay.flags);
  d.red = (unsigned long long*)(ws + g->lay.red);
  d.bw_slots = (long long*)(ws + g->lay.bw_slots);
  d.part8 = (unsigned char*)(ws + g->lay.part8);
  return d;
}

}  // namespace hg

extern "C" {

int32_t hg_net_words(int32_t k) { return hg::net_words(k); }

int64_t hg_netstate_words(int32_t m, int32_t k) {
  if (m < 1 || hg::net_words(k) == 0) return 0;
  return (int64_t)m * (hg::net_words(k) + hg::view_words(k));
}

size_t hg_workspace_size(int32_t n, int32_t m, int64_t P, int32_t k_max) {
  if (n < 1 || m < 1 || P < m || P > kMaxPins || k_max < 2 || k_max > HG_MAX_K) return 0;
  return hg::ws_layout(n, m, P, k_max).total;
}

const char* hg_last_error(void) { return g_msg; }

hg_status hg_load_csr(int32_t n, int32_t m, int64_t P, const int64_t* eptr, const int32_t* pins,
                      const int32_t* vwgt, const int32_t* ewgt, int64_t* vptr, int32_t* vnets,
                      void* workspace, size_t ws_bytes, int32_t k_max, void* stream,
                      hg_graph* out) {
  if (!out) return fail(HG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1 || m < 1) return fail(HG_ERR_INVALID, "need n >= 1 and m >= 1 (got %d, %d)", n, m);
  if (P < m) return fail(HG_ERR_INVALID, "P = %lld pins cannot fill m = %d non-empty nets",
                         (long long)P, m);
  if (P > kMaxPins) return fail(HG_ERR_UNSUPPORTED, "P = %lld exceeds 2^31 - 1", (long long)P);
  if (k_max < 2 || k_max > HG_MAX_K)
    return fail(HG_ERR_UNSUPPORTED, "k_max must lie in [2, %d] (got %d)", HG_MAX_K, k_max);
  if (!eptr || !pins || !vptr || !vnets || !workspace)
    return fail(HG_ERR_INVALID, "eptr, pins, vptr, vnets and workspace must be non-NULL");
  hg::WsLayout lay = hg::ws_layout(n, m, P, k_max);
  if (ws_bytes < lay.total)
    return fail(HG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed",
                ws_bytes, lay.total);
  hipStream_t s = (hipStream_t)stream;
  hg_graph_s* g = new (std::nothrow) hg_graph_s();
  if (!g) return fail(HG_ERR_INVALID, "out of host memory");
  g->n = n;
  g->m = m;
  g->P = P;
  g->eptr = (const long long*)eptr;
  g->pins = pins;
  g->vwgt = vwgt;
  g->ewgt = ewgt;
  g->vptr = (long long*)vptr;
  g->vnets = vnets;
  g->ws = (char*)workspace;
  g->ws_bytes = ws_bytes;
  g->k_max = k_max;
  g->lay = lay;
  g->graph_exec = nullptr;
  g->cap_stream = nullptr;
  g->timing = 0;
  g->timing_state = nullptr;
  auto bail = [&](hg_status st) {
    delete g;
    return st;
  };
  hipError_t e = hg::load_check(g, s);
  if (e != hipSuccess) return bail(hip_fail(e, "load checks"));
  hg_status st = read_info(g, s);
  if (st != HG_OK) return bail(st);
  if (g->info.err) return bail(fail(HG_ERR_INVALID, "%s", describe_err(g->info.err)));
  if (g->info.total_net_weight > 0x7fffffffULL)
    return bail(fail(HG_ERR_UNSUPPORTED, "total net weight %llu exceeds 2^31 - 1",
                     g->info.total_net_weight));
  if (g->info.total_vertex_weight > (1ULL << 62))
    return bail(fail(HG_ERR_UNSUPPORTED, "total vertex weight exceeds 2^62"));
  e = hg::load_build(g, s);
  if (e != hipSuccess) return bail(hip_fail(e, "incidence build"));
  // zero the round state kept in the workspace
  char* ws = g->ws;
  hg::ZeroRanges Z;
  Z.add(ws + lay.touched, (long long)hg::touched_bytes(m));
  Z.add(ws + lay.hist, (long long)sizeof(long long) * hg::kHistReplicas * k_max * hg::kBuckets);
  Z.add(ws + lay.overflow, (long long)sizeof(int) * k_max);
  Z.add(ws + lay.ctr, (long long)sizeof(hg::RoundCounters));
  Z.add(ws + lay.flags, (long long)sizeof(int) * 64);
  Z.add(ws + lay.red, (long long)sizeof(long long) * hg::kSlots);
  Z.add(ws + lay.bw_slots, (long long)sizeof(long long) * hg::kSlots * k_max);
  e = hg::zero_ranges(Z, s);
  if (e != hipSuccess) return bail(hip_fail(e, "workspace init"));
  st = read_info(g, s);
  if (st != HG_OK) return bail(st);
  if (g->info.err) return bail(fail(HG_ERR_INVALID, "%s", describe_err(g->info.err)));
  g->unit_nets = g->info.total_net_weight == (unsigned long long)m;
  *out = g;
  return HG_OK;
}

void hg_free(hg_graph g) {
  if (!g) return;
  if (g->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)g->graph_exec);
  if (g->cap_stream) (void)hipStreamDestroy((hipStream_t)g->cap_stream);
  release_timing(g);
  delete g;
}

hg_status hg_get_info(hg_graph g, hg_graph_info* info) {
  if (!g || !info) return fail(HG_ERR_INVALID, "graph handle or info is NULL");
  info->n = g->n;
  info->m = g->m;
  info->P = g->P;
  info->total_vertex_weight = (int64_t)g->info.total_vertex_weight;
  info->total_net_weight = (int64_t)g->info.total_net_weight;
  info->max_degree = g->info.max_degree;
  info->max_net_size = g->info.max_net_size;
  info->max_incident_weight = g->info.max_incident_weight;
  info->heavy_vertices = g->info.heavy_count;
  return HG_OK;
}

int64_t hg_max_block_weight(hg_graph g, int32_t k, double eps) {
  if (!g || k < 2 || !(eps > 0.0 && eps < 1.0)) return -1;
  const long long W = (long long)g->info.total_vertex_weight;
  const long long avg = (W + k - 1) / k;
  return (int64_t)floor((1.0 + eps) * (double)avg);
}

hg_status hg_compute_pincounts(hg_graph g, int32_t k, const int32_t* part, int32_t* phi,
                               uint32_t* netstate, int64_t* block_w, int64_t* km1_out,
                               void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!part || !phi || !netstate || !block_w)
    return fail(HG_ERR_INVALID, "part, phi, netstate and block_w must be non-NULL");
  hg::InstDesc d = hg::make_desc(g, k, 0, (int*)part, phi, netstate, (long long*)block_w, nullptr,
                                 nullptr, (long long*)km1_out, nullptr);
  hg::CountPlan plan;
  hg::single_count_plan(d, plan);
  HG_TRY(hg::launch_counts(plan, km1_out != nullptr, false, (hipStream_t)stream), "pin counts");
  return HG_OK;
}

hg_status hg_km1(hg_graph g, int32_t k, const uint32_t* netstate, int64_t* km1_out,
                 void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!netstate || !km1_out) return fail(HG_ERR_INVALID, "netstate and km1_out must be non-NULL");
  HG_TRY(hg::launch_km1(g, k, netstate, (long long*)km1_out, (hipStream_t)stream), "km1");
  return HG_OK;
}

hg_status hg_gains(hg_graph g, int32_t k, const int32_t* part, const uint32_t* netstate,
                   int64_t* gains, int64_t* benefit, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!part || !netstate || !gains)
    return fail(HG_ERR_INVALID, "part, netstate and gains must be non-NULL");
  if (((uintptr_t)gains & 15) != 0) return fail(HG_ERR_INVALID, "gains must be 16-byte aligned");
  hg::InstDesc d = hg::make_desc(g, k, 0, (int*)part, nullptr, (unsigned*)netstate, nullptr,
                                 nullptr, nullptr, nullptr, nullptr);
  HG_TRY(hg::launch_gains(g, d, (long long*)gains, (long long*)benefit, (hipStream_t)stream),
         "gains");
  return HG_OK;
}

hg_status hg_lp_round(hg_graph g, int32_t k, int64_t max_block_w, int32_t* part, int32_t* phi,
                      uint32_t* netstate, int64_t* block_w, uint8_t* eligible, uint8_t* moved,
                      int64_t* km1, hg_round_stats* stats, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!part || !phi || !netstate || !block_w || !eligible || !km1 || !stats)
    return fail(HG_ERR_INVALID,
                "part, phi, netstate, block_w, eligible, km1 and stats must be non-NULL");
  if (max_block_w < 0) return fail(HG_ERR_INVALID, "max_block_w must be >= 0");
  hipEvent_t* marks = nullptr;
  st = timing_marks(g, (hipStream_t)stream, &marks);
  if (st != HG_OK) return st;
  hg::InstDesc d = hg::make_desc(g, k, max_block_w, part, phi, netstate, (long long*)block_w,
                                 eligible, moved, (long long*)km1, stats);
  hg::RoundPlan plan;
  hg::single_round_plan(d, plan);
  HG_TRY(hg::launch_round(plan, 0, (hipStream_t)stream, marks), "label-propagation round");
  return HG_OK;
}

static hipError_t enqueue_refine(hg_graph g, int k, long long lmax, int rounds, int32_t* part,
                                 int32_t* phi, uint32_t* netstate, int64_t* block_w,
                                 uint8_t* eligible, hg_round_stats* stats, int64_t* km1,
                                 hipStream_t s) {
  hg::InstDesc d = hg::make_desc(g, k, lmax, part, phi, netstate, (long long*)block_w, eligible,
                                 nullptr, (long long*)km1, stats);
  hg::CountPlan cplan;
  hg::single_count_plan(d, cplan);
  hipError_t e = hg::launch_counts(cplan, true, true, s);
  hg::RoundPlan plan;
  for (int r = 0; r < rounds && e == hipSuccess; ++r) {
    hipEvent_t* marks = nullptr;
    if (timing_marks(g, s, &marks, r > 0) != HG_OK) return hipErrorUnknown;
    d.stats = stats + r;
    hg::single_round_plan(d, plan);
    e = hg::launch_round(plan, 0, s, marks);
  }
  return e;
}

hg_status hg_refine(hg_graph g, int32_t k, double eps, int32_t rounds, int32_t* part,
                    int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                    hg_round_stats* stats, int64_t* km1_out, int32_t use_graph, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!(eps > 0.0 && eps < 1.0)) return fail(HG_ERR_INVALID, "eps must lie in (0, 1)");
  if (rounds < 0) return fail(HG_ERR_INVALID, "rounds must be >= 0");
  if (!part || !phi || !netstate || !block_w || !eligible || !km1_out || (rounds > 0 && !stats))
    return fail(HG_ERR_INVALID, "part, phi, netstate, block_w, eligible, stats and km1_out must "
                                "be non-NULL");
  const long long lmax = hg_max_block_weight(g, k, eps);
  hipStream_t s = (hipStream_t)stream;
  if (!use_graph) {
    HG_TRY(enqueue_refine(g, k, lmax, rounds, part, phi, netstate, block_w, eligible, stats,
                          km1_out, s),
           "refine");
    return HG_OK;
  }
  unsigned long long key[12] = {(unsigned long long)k,        (unsigned long long)rounds,
                                (unsigned long long)lmax,     (unsigned long long)part,
                                (unsigned long long)phi,      (unsigned long long)netstate,
                                (unsigned long long)block_w,  (unsigned long long)eligible,
                                (unsigned long long)stats,    (unsigned long long)km1_out,
                                1ull,                         0ull};
  if (!g->graph_exec || memcmp(key, g->graph_key, sizeof(key)) != 0) {
    if (g->graph_exec) {
      (void)hipGraphExecDestroy((hipGraphExec_t)g->graph_exec);
      g->graph_exec = nullptr;
    }
    if (!g->cap_stream) {
      hipStream_t cs;
      HG_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
      g->cap_stream = cs;
    }
    hipStream_t cs = (hipStream_t)g->cap_stream;
    HG_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e = enqueue_refine(g, k, lmax, rounds, part, phi, netstate, block_w, eligible,
                                  stats, km1_out, cs);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(e, "refine capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    g->graph_exec = exec;
    memcpy(g->graph_key, key, sizeof(key));
  }
  HG_TRY(hipGraphLaunch((hipGraphExec_t)g->graph_exec, s), "hipGraphLaunch");
  return HG_OK;
}

// ------------------------------------------------------------ gain cache

int64_t hg_gain_cache_bytes(int32_t n, int32_t k) {
  if (n < 1 || k < 2 || k > HG_MAX_K) return -1;
  return 4 * (hg::cache_pbase(n) + (int64_t)n * hg::cache_stride(k));
}

hg_status hg_gain_cache_init(hg_graph g, int32_t k, const int32_t* part, const uint32_t* netstate,
                             int32_t* cache, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!part || !netstate || !cache)
    return fail(HG_ERR_INVALID, "part, netstate and cache must be non-NULL");
  if (((uintptr_t)cache & 15) != 0) return fail(HG_ERR_INVALID, "cache must be 16-byte aligned");
  hg::InstDesc d = hg::make_desc(g, k, 0, (int*)part, nullptr, (unsigned*)netstate, nullptr,
                                 nullptr, nullptr, nullptr, nullptr);
  HG_TRY(hg::launch_gains(g, d, nullptr, nullptr, (hipStream_t)stream, cache), "gain cache");
  return HG_OK;
}

hg_status hg_lp_round_cached(hg_graph g, int32_t k, int64_t max_block_w, int32_t* part,
                             int32_t* phi, uint32_t* netstate, int64_t* block_w,
                             uint8_t* eligible, uint8_t* moved, int64_t* km1,
                             hg_round_stats* stats, int32_t* cache, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!part || !phi || !netstate || !block_w || !eligible || !moved || !km1 || !stats || !cache)
    return fail(HG_ERR_INVALID, "part, phi, netstate, block_w, eligible, moved, km1, stats and "
                                "cache must be non-NULL");
  if (((uintptr_t)cache & 15) != 0) return fail(HG_ERR_INVALID, "cache must be 16-byte aligned");
  if (max_block_w < 0) return fail(HG_ERR_INVALID, "max_block_w must be >= 0");
  hipEvent_t* marks = nullptr;
  st = timing_marks(g, (hipStream_t)stream, &marks);
  if (st != HG_OK) return st;
  hg::InstDesc d = hg::make_desc(g, k, max_block_w, part, phi, netstate, (long long*)block_w,
                                 eligible, moved, (long long*)km1, stats);
  d.cache = cache;
  hg::RoundPlan plan;
  hg::cached_round_plan(d, plan);
  HG_TRY(hg::launch_cached_round(plan, 0, (hipStream_t)stream, marks), "cached round");
  return HG_OK;
}

hg_status hg_refine_cached(hg_graph g, int32_t k, double eps, int32_t rounds, int32_t* part,
                           int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                           uint8_t* moved, hg_round_stats* stats, int64_t* km1_out,
                           int32_t* cache, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!(eps > 0.0 && eps < 1.0)) return fail(HG_ERR_INVALID, "eps must lie in (0, 1)");
  if (rounds < 0) return fail(HG_ERR_INVALID, "rounds must be >= 0");
  if (!part || !phi || !netstate || !block_w || !eligible || !moved || !km1_out || !cache ||
      (rounds > 0 && !stats))
    return fail(HG_ERR_INVALID, "part, phi, netstate, block_w, eligible, moved, stats, km1_out "
                                "and cache must be non-NULL");
  if (((uintptr_t)cache & 15) != 0) return fail(HG_ERR_INVALID, "cache must be 16-byte aligned");
  const long long lmax = hg_max_block_weight(g, k, eps);
  hipStream_t s = (hipStream_t)stream;
  hg::InstDesc d = hg::make_desc(g, k, lmax, part, phi, netstate, (long long*)block_w, eligible,
                                 moved, (long long*)km1_out, stats);
  hg::CountPlan cplan;
  hg::single_count_plan(d, cplan);
  HG_TRY(hg::launch_counts(cplan, true, true, s), "pin counts");
  HG_TRY(hg::launch_gains(g, d, nullptr, nullptr, s, cache), "gain cache");
  d.cache = cache;
  hg::RoundPlan plan;
  for (int r = 0; r < rounds; ++r) {
    hipEvent_t* marks = nullptr;
    st = timing_marks(g, s, &marks, r > 0);
    if (st != HG_OK) return st;
    d.stats = stats + r;
    hg::cached_round_plan(d, plan);
    HG_TRY(hg::launch_cached_round(plan, 0, s, marks), "cached round");
  }
  return HG_OK;
}

hg_status hg_timing_enable(hg_graph g, int32_t enable) {
  if (!g) return fail(HG_ERR_INVALID, "graph handle is NULL");
  g->timing = enable ? 1 : 0;
  return HG_OK;
}

hg_status hg_timing_collect(hg_graph g, double* ms, int64_t* rounds) {
  if (!g || !ms || !rounds) return fail(HG_ERR_INVALID, "graph handle, ms and rounds must be non-NULL");
  TimingState* t = (TimingState*)g->timing_state;
  if (!t || t->spans.empty()) return HG_OK;
  for (const auto& span : t->spans) {
    HG_TRY(hipEventSynchronize(span[3]), "hipEventSynchronize");
    for (int p = 0; p < HG_NUM_PHASES; ++p) {
      float x = 0.0f;
      HG_TRY(hipEventElapsedTime(&x, span[p], span[p + 1]), "hipEventElapsedTime");
      ms[p] += x;
    }
    *rounds += 1;
  }
  t->marks.clear();
  t->spans.clear();
  t->next = 0;
  return HG_OK;
}

hg_status hg_sync_status(hg_graph g, void* stream) {
  if (!g) return fail(HG_ERR_INVALID, "graph handle is NULL");
  hipStream_t s = (hipStream_t)stream;
  HG_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  int flags = 0;
  HG_TRY(hipMemcpyAsync(&flags, g->ws + g->lay.flags, sizeof(int), hipMemcpyDeviceToHost, s),
         "hipMemcpyAsync");
  HG_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (flags) {
    HG_TRY(hg::fill_i32((int*)(g->ws + g->lay.flags), 0, 1, s), "flag reset");
    HG_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    return fail(HG_ERR_INVALID, "%s", describe_err(flags));
  }
  return HG_OK;
}

}  // extern "C"
