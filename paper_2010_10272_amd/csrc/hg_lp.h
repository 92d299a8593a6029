// hg_lp.h -- launch plans: which kernels a round (or a pin-count pass) runs,
// with which grid and arguments, for one instance or a batch.
#pragma once

#include <vector>

#include "hg_internal.h"

namespace hg {

constexpr int kFinalChunk = 4 * kBlock;   // nets per unit of the finalize sweep (4 flags per thread)

typedef void (*SelectKernel)(Launch);
typedef void (*FinalizeKernel)(Launch);
typedef void (*GroupKernel)(Launch);
typedef void (*GainsKernel)(Launch);

struct PlanLaunch {
  void* kernel = nullptr;   // for templated kernels: which instantiation
  unsigned grid = 0;
  size_t lds = 0;           // dynamic LDS bytes (pin counts)
  Launch L{};
};

// One LP round: select launches (one per kernel variant in a batch), heavy
// select, per-block kernels (threshold, overflow, tilescan), tiles, approve,
// finalize launches (one per group width), stats.
struct RoundPlan {
  std::vector<PlanLaunch> select, heavy, finalize;
  PlanLaunch blocks, tiles, approve, stats;
  bool any_heavy = false;
};

// Pin counts (one launch per group width), then the per-instance km1 slot
// sums, the block-weight reset and sweep.
struct CountPlan {
  std::vector<PlanLaunch> pincounts;
  PlanLaunch instances;     // one workgroup per instance
  PlanLaunch vertices;      // block weights: units of kBwChunk vertices
};

constexpr int kBwChunk = kBlock * 16;   // vertices per unit of the block-weight sweep

SelectKernel select_kernel(int k, int view, long long P, int n);
// lanes per net: group_lanes(k); cache: the variant that also applies the
// gain-cache deltas (it must be used exactly when the descriptor has a cache)
FinalizeKernel finalize_kernel(int k, bool cache);
FinalizeKernel finalize_kernel_g(int G, bool cache);   // G lanes per net (4, 8, 16 or 32)
GroupKernel pincount_kernel(int k);          // lanes per net: group_lanes(k)
GroupKernel pincount_kernel_g(int G);        // G lanes per net (4, 8, 16 or 32)
size_t pincount_lds(int G, int k);           // its dynamic LDS bytes
GainsKernel gains_kernel(int k, int view);
int group_lanes(int k);

// Enqueue one round; the round record goes to stats[round] of every instance.
hipError_t launch_round(const RoundPlan& plan, int round, hipStream_t s, hipEvent_t* marks);
// Its two halves: select .. approve (+ apply), then finalize and the record.
hipError_t launch_round_front(const RoundPlan& plan, hipStream_t s, hipEvent_t* marks);
hipError_t launch_round_back(const RoundPlan& plan, int round, hipStream_t s, hipEvent_t* marks);
// launch_round_back in two steps: finalize, then the round record.
hipError_t launch_round_finalize(const RoundPlan& plan, hipStream_t s, hipEvent_t* marks);
hipError_t launch_round_stats(const RoundPlan& plan, int round, hipStream_t s, hipEvent_t* marks);
void single_round_plan(const InstDesc& d, RoundPlan& plan);
// Gain-cache rounds (single instance, d.cache and d.moved set): the plan and
// its launch (front, finalize with cache deltas, movers' b, record).
SelectKernel select_cached_kernel(int k);
void cached_round_plan(const InstDesc& d, RoundPlan& plan);
hipError_t launch_cached_round(const RoundPlan& plan, int round, hipStream_t s,
                               hipEvent_t* marks);

// Pin counts, block weights and (want_km1) km1 of every instance; with
// mark_eligible every vertex is made eligible as well.
hipError_t launch_counts(const CountPlan& plan, bool want_km1, bool mark_eligible, hipStream_t s);
void single_count_plan(const InstDesc& d, CountPlan& plan);

// All gains (or, with `cache`, a gain cache: b, w(I), p rows; see hgref.h;
// with only_over, only the rows of vertices in blocks heavier than d.lmax).
hipError_t launch_gains(hg_graph_s* g, const InstDesc& d, long long* gains, long long* benefit,
                        hipStream_t s, int* cache = nullptr, int only_over = 0);
hipError_t launch_km1(hg_graph_s* g, int k, const unsigned* netstate, long long* km1,
                      hipStream_t s);

}  // namespace hg
