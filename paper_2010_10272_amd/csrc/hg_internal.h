// hg_internal.h -- shared definitions of the HIP implementation behind hgref.h.
//
// Data layout in device memory (all caller-owned):
//   net CSR          eptr int64[m+1], pins int32[P]
//   incidence CSR    vptr int64[n+1], vnets int32[P] (rows sorted by net id)
//   partition state  part int32[n], phi int32[m*k] (row-major by net),
//                    netstate uint32[m*RW] (RW = hg_net_words(k)), block_w int64[k]
//   workspace        carved by WsLayout below
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hgref.h"

namespace hg {

constexpr int kWave = 64;
constexpr int kBlock = 256;            // threads per workgroup in every kernel
constexpr int kTile = 512;             // vertices per approval tile (256 threads x 2)
constexpr int kPerThreadTile = kTile / kBlock;
constexpr int kBuckets = 256;          // gain buckets per target block (0..254 exact, 255 = ">=255")
constexpr int kLightLimit = 255;       // w(I(v)) <= 255: bit-sliced register path
constexpr int kPlanes = 8;             // bit planes for counters <= 255
constexpr int kSmallRow = 64;          // incidence rows up to this length sort in-thread
constexpr int kNumXcd = 8;             // MI355X: 8 XCDs, each with its own L2
constexpr int kLdsHistEntries = 2048;  // per-workgroup LDS gain histogram (k * buckets)
constexpr int kSelectGrid = 2048;      // persistent workgroups of the select sweep
constexpr int kUnroll = 4;             // record gathers in flight per thread in the gains sweep
constexpr int kFinalizeGrid = 2048;    // persistent workgroups of the finalize sweep

// Validation bits raised on the device.
enum : int {
  kErrCsr = 1,         // eptr not increasing / wrong ends
  kErrPin = 2,         // pin outside [0,n)
  kErrWeight = 4,      // non-positive weight
  kErrDuplicate = 8,   // a vertex twice in one net
  kErrPart = 16,       // partition id outside [0,k)
  kErrNetWeight = 32,  // total net weight >= 2^31
  kErrMoves = 64,      // a move sequence names a vertex twice, a bad target or its own block
  kErrCluster = 128,   // cluster id outside [0,n)
  kErrClusterWeight = 256,  // a cluster weighs 2^31 or more
};

// Same-address global atomics serialize (tens of ns each), so every
// accumulator that many workgroups add to is split into kSlots partial sums
// (workgroup b adds to slot b % kSlots) and the partials are summed once by a
// single small kernel.  Histograms get one replica per XCD.
constexpr int kSlots = 64;
constexpr int kHistReplicas = kNumXcd;

enum CounterId : int {
  kCtrEligible = 0,
  kCtrBoundary,
  kCtrCandidates,
  kCtrApproved,
  kCtrMovedPins,
  kCtrDeltaAttr,    // two's complement int64 sums
  kCtrDeltaCheck,
  kCtrActivePins,
  kCtrTouched,
  kCtrMarked,       // approved moves marked for a monotone round (before the prefix cut)
  kCtrTouchedPins,  // sum of |e| over touched nets
  kNumCounters
};

// Per-round counters kept in the workspace.  Zero between rounds.
struct RoundCounters {
  unsigned long long slot[kNumCounters][kSlots];
  unsigned int any_overflow;       // some block's threshold fell into the ">=255" bucket
  unsigned int pad[63];
};

// Approval threshold of one target block.
struct Threshold {
  int gstar;          // gains > gstar approved; == gstar decided by vertex order; -1: all approved
  int tau;            // tile holding the last approved vertex of gain gstar (numTiles: none)
  long long rem;      // budget left for gain-gstar candidates after all higher gains
  long long rem_tile; // budget left inside tile tau
};

// Facts gathered at load time (device side, copied to the host once).
struct LoadInfo {
  int err;
  int max_degree;
  int max_net_size;
  int max_incident_weight;
  int max_vertex_weight;
  int heavy_count;
  unsigned long long total_vertex_weight;
  unsigned long long total_net_weight;
  int big_rows;       // incidence rows longer than kSmallRow
  int pad[5];
};

// One load workgroup's share of the LoadInfo maxima and sums; the load folds
// them into LoadInfo with one small kernel instead of one atomic per
// workgroup on the same words.
constexpr int kLoadGrid = 1024;   // workgroups of the load's sweeps
struct LoadPart {
  unsigned long long total_net_weight, total_vertex_weight;
  int max_net_size, max_vertex_weight, max_degree, max_incident_weight;
};

// Everything a kernel needs about one instance: a loaded hypergraph, its
// workspace, and one k-way partition state.  Single-instance entry points pass
// one by value inside the kernel arguments; batched launches pass a device
// array and a per-workgroup work table.
struct InstDesc {
  int n, m;
  int k, rw, view, unit_nets;
  int cmax, lds_buckets, heavy_count, num_tiles;
  int hist_stride;               // k_max * kBuckets: distance between histogram replicas
  int hist_reps;                 // histogram replicas in use (workgroup b adds to b % hist_reps)
  int round_base;                // round r's record goes to stats[r - round_base]
  int pad1;
  long long P, lmax;
  const long long* eptr;
  const int* pins;
  const int* vwgt;
  const int* ewgt;
  const long long* vptr;
  const int* vnets;
  const int* heavy_list;
  int* part;
  int* phi;
  unsigned* netstate;
  unsigned* view_ptr;            // compact Lambda/S copy (behind the records)
  long long* block_w;
  unsigned char* eligible;
  unsigned char* moved;          // may be null
  long long* km1;
  hg_round_stats* stats;
  long long* cand;
  unsigned char* touched;
  unsigned long long* hist;
  int* overflow;
  Threshold* thr;
  long long* tilesum;
  RoundCounters* ctr;
  int* err_flags;
  unsigned long long* red;
  long long* bw_slots;           // kSlots x k block-weight deltas of a round's moves
  unsigned char* part8;          // byte copy of part written by the block-weight sweep
  unsigned char* appr;           // monotone rounds: approve marks moves here instead of applying
  int4* seq_cell;                // monotone rounds: per (net, block) cells the marking sets empty
  int* cache;                    // gain cache (b[n], w(I)[n], p[n*k]); null: none
};

// One workgroup's share of a batched launch: instance, and the units it
// handles: first, first + stride, ... (count of them).  What a unit is
// depends on the kernel (a 256-vertex chunk, a target block, a tile, ...).
struct WorkItem {
  int inst, first, count, stride;
};

// Kernel argument: a batch (descs + items, both device arrays) or one
// instance by value (descs == nullptr; each kernel then derives its units
// from blockIdx as documented with it).
//
// In a batch the items are either one per workgroup (split == 0) or grouped
// by XCD (split == 1): workgroup b runs on XCD b % 8 and takes item
// b / 8 of that XCD's queue items[xoff[x] .. xoff[x+1]), or nothing once the
// queue is used up.  Grouping keeps an instance's sweep on the XCD (and L2)
// it was placed on.
struct Launch {
  const InstDesc* descs;
  const WorkItem* items;
  int round;                     // round record index: stats + round (k_round_stats)
  int split;
  int xoff[kNumXcd + 1];
  int pad;
  InstDesc one;
};

// This workgroup's work item; `fallback` in single-instance mode.  An empty
// item (count == 0) means: nothing to do.
__device__ __forceinline__ WorkItem work_item(const Launch& L, WorkItem fallback) {
  if (!L.items) return fallback;
  if (!L.split) return L.items[blockIdx.x];
  const int x = (int)(blockIdx.x % kNumXcd);
  const int o = L.xoff[x] + (int)(blockIdx.x / kNumXcd);
  if (o >= L.xoff[x + 1]) {
    WorkItem w;
    w.inst = 0;
    w.first = 0;
    w.count = 0;
    w.stride = 1;
    return w;
  }
  return L.items[o];
}

__device__ __forceinline__ InstDesc inst_desc(const Launch& L, int inst) {
  return L.descs ? L.descs[inst] : L.one;
}

// Launch argument for one instance (kernels take their units from blockIdx).
inline Launch single_launch(const InstDesc& d) {
  Launch L;
  L.descs = nullptr;
  L.items = nullptr;
  L.round = 0;
  L.split = 0;
  for (int x = 0; x <= kNumXcd; ++x) L.xoff[x] = 0;
  L.pad = 0;
  L.one = d;
  return L;
}

struct WsLayout {
  size_t cand, touched, heavy, big, hist, overflow, thr, tilesum, ctr, info, scan, flags;
  size_t red;   // kSlots partial sums for whole-array reductions (km1)
  size_t bw_slots;   // kSlots x k_max block-weight deltas (apply), folded in by the round record
  size_t part8;      // n bytes: the partition as block ids of one byte (pin-count gathers)
  size_t lkey[2], lval, lhist, ldtot;   // load only: radix-sort buffers of the transpose
  size_t lpart;      // load only: per-workgroup partial facts (LoadPart[kLoadGrid])
  size_t total;
  int num_tiles;
  int scan_blocks;
};

WsLayout ws_layout(int n, int m, long long P, int k_max);

// Touched-net flags: one byte per net, padded to whole finalize chunks of
// 1024 nets so that the sweep reads them four at a time without bounds tests.
inline size_t touched_bytes(int m) { return (((size_t)m + 1023) / 1024) * 1024; }

// 32-bit words per block bitset in a net record: ceil(k/32) rounded up to a
// power of two (1, 2, 4 or 8), so that word offsets are compile-time friendly.
__host__ __device__ inline int bit_words(int k) {
  int w = 1;
  while (w * 32 < k) w *= 2;
  return w;
}

// Compact per-net view read by the select and gain sweeps when every net
// weight is 1 and k <= 64: only the Lambda and S bitsets, packed into 4, 8 or
// 16 bytes (w(e) = 1 is implied and lambda(e) = popcount(Lambda)).  With k <=
// 16 a million nets take 4 MB, one XCD's L2.  kViewFull means the sweeps read
// the full net record instead.
enum NetView : int { kViewFull = 0, kView16 = 1, kView32 = 2, kView64 = 3 };

__host__ __device__ inline int net_view(int k, bool unit_nets) {
  if (!unit_nets) return kViewFull;
  if (k <= 16) return kView16;
  if (k <= 32) return kView32;
  if (k <= 64) return kView64;
  return kViewFull;
}

__host__ __device__ inline int view_bytes(int view) {
  return view == kView16 ? 4 : view == kView32 ? 8 : view == kView64 ? 16 : 0;
}

// 32-bit words per net reserved for the compact view in a net-state array
// (present for every k <= 64; maintained only for unit net weights).
__host__ __device__ inline int view_words(int k) {
  return k <= 16 ? 1 : k <= 32 ? 2 : k <= 64 ? 4 : 0;
}

// Words per net record: 2 + 2 * bit_words(k) rounded up to a power of two.
__host__ __device__ inline int net_words(int k) {
  if (k < 2 || k > HG_MAX_K) return 0;
  int need = 2 + 2 * bit_words(k);
  int rw = 4;
  while (rw < need) rw *= 2;
  return rw;
}

}  // namespace hg

struct hg_graph_s {
  int n, m;
  long long P;
  const long long* eptr;
  const int* pins;
  const int* vwgt;   // may be null (unit)
  const int* ewgt;   // may be null (unit)
  long long* vptr;
  int* vnets;
  char* ws;
  size_t ws_bytes;
  int k_max;
  bool unit_nets;    // every net weight is 1 (the compact net view is maintained)
  hg::WsLayout lay;
  hg::LoadInfo info;
  // recorded refinement graph (hipGraphExec_t) and the private stream it is
  // captured on (the caller's stream may be the legacy null stream)
  void* graph_exec;
  void* cap_stream;
  unsigned long long graph_key[12];
  // optional per-phase timing of label-propagation rounds (see hg_timing_*)
  int timing;
  void* timing_state;
};

namespace hg {

// ---- error reporting (hg_last_error) ----
hg_status fail(hg_status code, const char* fmt, ...);
size_t moves_workspace_size(long long n, long long m, int k);
size_t rebalance_workspace_size(long long n, int k);
size_t contract_workspace_size(long long n, long long m, long long P);
hg_status hip_fail(hipError_t e, const char* what);
hg_status check_k(hg_graph_s* g, int k);

#define HG_TRY(expr, what)                               \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return hg::hip_fail(_e, what); \
  } while (0)

// ---- launch helpers implemented in the .hip files (return hipError_t) ----
// Up to kZeroRanges byte ranges of device memory, cleared by one launch of
// zero_ranges (add() ignores empty ranges; more than kZeroRanges is a bug).
constexpr int kZeroRanges = 8;
struct ZeroRanges {
  unsigned char* p[kZeroRanges];
  long long bytes[kZeroRanges];
  int count = 0;
  void add(void* ptr, long long nbytes);
};
hipError_t zero_ranges(const ZeroRanges& R, hipStream_t s);

hipError_t fill_i64(long long* p, long long v, long long count, hipStream_t s);
hipError_t fill_u8(unsigned char* p, unsigned char v, long long count, hipStream_t s);
hipError_t fill_i32(int* p, int v, long long count, hipStream_t s);

hipError_t load_check(hg_graph_s* g, hipStream_t s);
hipError_t load_build(hg_graph_s* g, hipStream_t s);

// Gain cache (int32): b(u) at [u], w(I(u)) at [n + u], and the penalty row
// p_0(u) .. p_{k-1}(u) at [cache_pbase(n) + u * cache_stride(k)], rows padded
// to whole 16-byte quads.
__host__ __device__ inline long long cache_pbase(long long n) { return (2 * n + 3) & ~3LL; }
__host__ __device__ inline int cache_stride(int k) { return (k + 3) & ~3; }

// Gain-histogram buckets kept in LDS per target block by the select sweep.
inline int lds_buckets(int k) {
  int b = kBuckets;
  while (b > 1 && b * k > kLdsHistEntries) b >>= 1;
  return b;
}

// Descriptor of one instance: graph g, its workspace, and the caller's state.
InstDesc make_desc(hg_graph_s* g, int k, long long lmax, int* part, int* phi,
                   unsigned* netstate, long long* block_w, unsigned char* eligible,
                   unsigned char* moved, long long* km1, hg_round_stats* stats);

}  // namespace hg
