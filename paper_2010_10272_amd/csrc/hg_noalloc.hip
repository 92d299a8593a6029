// hg_noalloc.hip -- hg_lp_round_noalloc: one label-propagation round whose
// round scratch (candidate words, touched-net flags, gain histograms,
// thresholds, tile sums, counter and block-weight slots) lives in a
// file-scope device array instead of the graph's workspace.  It runs the same
// kernels as hg_lp_round; only the scratch pointers in the descriptor differ.
//
// The array is sized for n, m <= 2^20 and every k <= HG_MAX_K.  Each GPU the
// library runs on holds its own copy for the life of the process.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in,
// not a device address): the device address of each GPU's copy is looked up
// once, on that GPU's first call, with hipGetSymbolAddress and kept per
// device.
#include <mutex>

#include "hg_internal.h"
#include "hg_lp.h"

namespace {

constexpr long long kNoallocMaxN = 1LL << 20;
constexpr long long kNoallocMaxM = 1LL << 20;
constexpr int kMaxDevices = 64;

constexpr size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the round scratch for n vertices, m nets and k blocks.
struct NoallocLayout {
  size_t cand, touched, hist, overflow, thr, tilesum, ctr, bw_slots, total;
};

constexpr NoallocLayout noalloc_layout(long long n, long long m, int k) {
  NoallocLayout L{};
  const long long tiles = (n + hg::kTile - 1) / hg::kTile;
  size_t off = 0;
  L.cand = off;
  off = up256(off + sizeof(long long) * (size_t)n);
  L.touched = off;
  off = up256(off + (size_t)((m + 1023) / 1024) * 1024);
  L.hist = off;
  off = up256(off + sizeof(unsigned long long) * (size_t)hg::kHistReplicas * k * hg::kBuckets);
  L.overflow = off;
  off = up256(off + sizeof(int) * (size_t)k);
  L.thr = off;
  off = up256(off + sizeof(hg::Threshold) * (size_t)k);
  L.tilesum = off;
  off = up256(off + sizeof(long long) * (size_t)k * (size_t)tiles);
  L.ctr = off;
  off = up256(off + sizeof(hg::RoundCounters));
  L.bw_slots = off;
  off = up256(off + sizeof(long long) * hg::kSlots * (size_t)k);
  L.total = off;
  return L;
}

constexpr size_t kScratchBytes = noalloc_layout(kNoallocMaxN, kNoallocMaxM, HG_MAX_K).total;

// About 15 MB: candidate words 8 MB, touched flags 1 MB, histograms 4 MB,
// tile sums 2 MB, the rest small.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch` (looked up once per
// device, with that device current).
hg_status scratch_ptr(unsigned char** out) {
  int dev = -1;
  HG_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return hg::fail(HG_ERR_UNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HG_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) return hg::fail(HG_ERR_DEVICE, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return HG_OK;
}

}  // namespace

extern "C" {

hg_status hg_lp_round_noalloc(hg_graph g, int32_t k, int64_t max_block_w, int32_t* part,
                              int32_t* phi, uint32_t* netstate, int64_t* block_w,
                              uint8_t* eligible, uint8_t* moved, int64_t* km1,
                              hg_round_stats* stats, void* stream) {
  hg_status st = hg::check_k(g, k);
  if (st != HG_OK) return st;
  if (!part || !phi || !netstate || !block_w || !eligible || !km1 || !stats)
    return hg::fail(HG_ERR_INVALID,
                    "part, phi, netstate, block_w, eligible, km1 and stats must be non-NULL");
  if (max_block_w < 0) return hg::fail(HG_ERR_INVALID, "max_block_w must be >= 0");
  if (g->n > kNoallocMaxN || g->m > kNoallocMaxM)
    return hg::fail(HG_ERR_UNSUPPORTED,
                    "hg_lp_round_noalloc supports n, m <= %lld (got n = %d, m = %d); "
                    "use hg_lp_round",
                    kNoallocMaxN, g->n, g->m);
  unsigned char* base = nullptr;
  st = scratch_ptr(&base);
  if (st != HG_OK) return st;
  const NoallocLayout lay = noalloc_layout(g->n, g->m, k);
  hg::InstDesc d = hg::make_desc(g, k, max_block_w, part, phi, netstate, (long long*)block_w,
                                 eligible, moved, (long long*)km1, stats);
  d.cand = (long long*)(base + lay.cand);
  d.touched = base + lay.touched;
  d.hist = (unsigned long long*)(base + lay.hist);
  d.hist_stride = k * hg::kBuckets;
  d.hist_reps = hg::kHistReplicas;
  d.overflow = (int*)(base + lay.overflow);
  d.thr = (hg::Threshold*)(base + lay.thr);
  d.tilesum = (long long*)(base + lay.tilesum);
  d.ctr = (hg::RoundCounters*)(base + lay.ctr);
  d.bw_slots = (long long*)(base + lay.bw_slots);
  hipStream_t s = (hipStream_t)stream;
  // The round kernels expect these zero on entry (and leave them zero); the
  // array keeps whatever the previous call on this GPU left, so clear them.
  // One fill kernel rather than hipMemsetAsync, so a captured graph holds no
  // memset nodes.
  hg::ZeroRanges Z;
  Z.add(d.touched, (long long)hg::touched_bytes(g->m));
  Z.add((void*)d.hist, (long long)sizeof(long long) * hg::kHistReplicas * k * hg::kBuckets);
  Z.add(d.overflow, (long long)sizeof(int) * k);
  Z.add(d.ctr, (long long)sizeof(hg::RoundCounters));
  Z.add(d.bw_slots, (long long)sizeof(long long) * hg::kSlots * k);
  hipError_t e = hg::zero_ranges(Z, s);
  if (e != hipSuccess) return hg::hip_fail(e, "scratch clear");
  hg::RoundPlan plan;
  hg::single_round_plan(d, plan);
  HG_TRY(hg::launch_round(plan, 0, s, nullptr), "label-propagation round (no allocation)");
  return HG_OK;
}

}  // extern "C"
