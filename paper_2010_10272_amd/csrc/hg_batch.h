// hg_batch.h -- work tables of batched launches, shared by the batch API
// (hg_batch_*) and the request server (hg_server_*).
#pragma once

#include <vector>

#include "hg_internal.h"
#include "hg_lp.h"

namespace hg {

// One member of a batched launch: a loaded graph, the state of one k-way
// partition, its L_max, its size class (which schedule applies) and the
// round index it started at (round r's record goes to stats[r - round_base]).
struct BatchMember {
  hg_graph_s* g;
  int k;
  int cls;
  int round_base;
  long long lmax;
  int* part;
  int* phi;
  unsigned* netstate;
  long long* block_w;
  unsigned char* eligible;
  hg_round_stats* stats;
  long long* km1;
};

extern const hg_schedule kDefaultSchedule[HG_SIZE_CLASSES];

int size_class(int n);
bool valid_schedule(const hg_schedule& s);

// Table bytes members `which` of `mem` can need, for any schedule.
size_t table_bound(const std::vector<BatchMember>& mem, const std::vector<int>& which);

// Build the descriptors and work tables of members `which` under `sched`
// into the host staging buffer `host` at byte offset `at` (capacity `cap`),
// addressed on the device as `dev` (the same offsets), and fill the round
// plan (rp) and/or the pin-count plan (cp) that read them.  Returns the end
// offset, or 0 when `cap` is too small.  Placement on XCDs is computed here
// from the members' sizes.
size_t build_plans(const std::vector<BatchMember>& mem, const std::vector<int>& which,
                   const hg_schedule* sched, char* dev, char* host, size_t at, size_t cap,
                   RoundPlan* rp, CountPlan* cp);

}  // namespace hg
