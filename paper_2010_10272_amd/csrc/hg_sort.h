// hg_sort.h -- stable LSD radix sort of (uint32 key, int32 value) pairs,
// 8 bits per pass, for the loader, the move-sequence, rebalancing and
// contraction kernels.  A pass is three launches (sort_pass): per-tile digit
// counts, a scan of each digit's counts over the tiles, and a stable
// scatter.
// Included by each source file that sorts (the kernels have internal
// linkage there).
#pragma once

#include "hg_device.h"
#include "hg_internal.h"

namespace hg {
namespace {

// Items per thread of a radix-sort tile: 16 (4096-item tiles) by default,
// 32 for long sorts (fewer, fuller digit runs per tile; half the occupancy).
constexpr int kSortPer = 16;
constexpr int kSortPerLong = 32;
constexpr int kSortTile = kSortPer * kBlock;
constexpr int kSortWaves = kBlock / kWave;
constexpr int kDigits = 256;                // 8-bit digits
static_assert(kDigits == kBlock, "one thread per digit");

// Item r of this thread in the tile at `base`: wave w holds the tile's items
// [w * PER * 64, (w + 1) * PER * 64), 64 consecutive per round, so every
// load is coalesced and a wave's items are contiguous (the scatter ranks them
// without workgroup barriers).
template <int PER>
__device__ __forceinline__ long long sort_item(long long base, int r) {
  return base + (long long)(threadIdx.x / kWave) * (PER * kWave) + r * kWave + lane_id();
}

struct SortPass {
  const unsigned* key_in;
  const int* val_in;
  unsigned* key_out;
  int* val_out;
  unsigned* hist;   // [kDigits][tiles], digit-major
  unsigned* dtot;   // [kDigits]
  int n, tiles, shift;
  // when set, the item count is *n_dev (known only on the device, at most n;
  // tiles past it are empty)
  const int* n_dev = nullptr;
  // Marks mode (the first pass of a monotone round's move order): item i is
  // vertex i, present only where marks[i] != 0, with key top - gain(cand[i])
  // and value i; the scatter clears the marks it reads and workgroup 0
  // stores the number of present items in *count_out.  key_in / val_in are
  // not read.
  unsigned char* marks = nullptr;
  const long long* cand = nullptr;
  unsigned top = 0;
  int* count_out = nullptr;
  // Range check (the loader's first pass, whose keys are the caller's pins):
  // when err is set, the digit-count kernel also ORs err_bit into *err if a
  // present key is >= key_limit.  The counts stay in range either way.
  int* err = nullptr;
  int err_bit = 0;
  unsigned key_limit = 0;
};

__device__ __forceinline__ int sort_items(const SortPass& P) { return P.n_dev ? *P.n_dev : P.n; }

// The PER items of this thread in tile `base`: keys, values (when want_val)
// and presence.  Every load of the tile is issued before the first wait; in
// marks mode the candidate words are read for marked vertices only.
template <int PER>
__device__ __forceinline__ void sort_load(const SortPass& P, int n, long long base, bool want_val,
                                          unsigned* key, int* val, bool* live) {
  if (P.marks) {
    unsigned char mk[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const long long i = sort_item<PER>(base, r);
      mk[r] = i < n ? P.marks[i] : 0;
    }
    long long x[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const long long i = sort_item<PER>(base, r);
      x[r] = mk[r] ? P.cand[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      live[r] = mk[r] != 0;
      key[r] = P.top - (unsigned)(int)(x[r] >> 32);   // select gain, 0 <= gain <= top
      if (want_val) val[r] = (int)sort_item<PER>(base, r);
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const long long i = sort_item<PER>(base, r);
    live[r] = i < n;
    key[r] = i < n ? P.key_in[i] : 0u;
    if (want_val) val[r] = i < n ? P.val_in[i] : 0;
  }
}

__device__ __forceinline__ unsigned digit_of(unsigned key, int shift) {
  return (key >> shift) & (kDigits - 1);
}

template <int PER>
__global__ __launch_bounds__(kBlock) void k_sort_hist(SortPass P) {
  __shared__ unsigned s_h[kDigits];
  const int n = sort_items(P);
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * (PER * kBlock);
  unsigned key[PER];
  bool live[PER];
  sort_load<PER>(P, n, base, false, key, nullptr, live);
#pragma unroll
  for (int r = 0; r < PER; ++r)
    if (live[r]) atomicAdd(&s_h[digit_of(key[r], P.shift)], 1u);
  if (P.err) {
    bool bad = false;
#pragma unroll
    for (int r = 0; r < PER; ++r) bad |= live[r] && key[r] >= P.key_limit;
    if (bad) atomicOr(P.err, P.err_bit);
  }
  __syncthreads();
  P.hist[(size_t)threadIdx.x * P.tiles + blockIdx.x] = s_h[threadIdx.x];
}

// One workgroup per digit: exclusive scan of its per-tile counts; total.
// Each thread takes kSortScanPer consecutive counts per step (all loaded before
// the first wait), so a 7,000-tile row is four workgroup scans, not 28.
constexpr int kSortScanPer = 8;

__global__ __launch_bounds__(kBlock) __attribute__((unused)) void k_sort_scan(SortPass P) {
  __shared__ long long s_tmp[kBlock / kWave];
  unsigned* row = P.hist + (size_t)blockIdx.x * P.tiles;
  long long carry = 0;
  for (int b = 0; b < P.tiles; b += kBlock * kSortScanPer) {
    const int i0 = b + threadIdx.x * kSortScanPer;
    unsigned c[kSortScanPer];
#pragma unroll
    for (int q = 0; q < kSortScanPer; ++q) c[q] = i0 + q < P.tiles ? row[i0 + q] : 0u;
    long long sum = 0;
#pragma unroll
    for (int q = 0; q < kSortScanPer; ++q) sum += c[q];
    long long tot;
    long long run = carry + block_excl_scan64(sum, s_tmp, &tot);
#pragma unroll
    for (int q = 0; q < kSortScanPer; ++q) {
      if (i0 + q < P.tiles) row[i0 + q] = (unsigned)run;
      run += c[q];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) P.dtot[blockIdx.x] = (unsigned)carry;
}

// Stable scatter of one tile.  The tile is first ranked into LDS in digit
// order, then written out slot by slot, so that each digit's run of the
// tile leaves as consecutive addresses instead of every store touching many
// runs.  Ranking: each wave walks its contiguous items 64 at a time; lanes
// with equal digits find each other by ballots, and a wave-private LDS
// counter per digit gives each item its offset among the wave's items of
// that digit (no workgroup barrier inside the walk).  Offsets of the waves
// before it and of the smaller digits complete the LDS slot, which keeps
// item order within each digit.
template <int PER>
__global__ __launch_bounds__(kBlock) void k_sort_scatter(SortPass P) {
  constexpr int kTile = PER * kBlock;
  __shared__ unsigned s_key[kTile];
  __shared__ int s_val[kTile];
  __shared__ unsigned s_run[kDigits];     // first LDS slot of each digit
  __shared__ unsigned s_gofs[kDigits];    // output index of LDS slot 0 for each digit
  __shared__ unsigned s_wcnt[kSortWaves][kDigits];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ unsigned s_count;            // items present in this tile
  const long long base = (long long)blockIdx.x * kTile;
  const int n = sort_items(P);
  if (base >= n) return;                  // an empty tile (device-side count)
  unsigned key[PER];
  int val[PER];
  bool item[PER];
  sort_load<PER>(P, n, base, true, key, val, item);
  {
    // digit d = threadIdx.x: its count in this tile is the difference of the
    // scanned per-tile offsets; its LDS run starts after the smaller digits'
    const int d = threadIdx.x;
    const unsigned here = P.hist[(size_t)d * P.tiles + blockIdx.x];
    const unsigned next =
        (int)blockIdx.x + 1 < P.tiles ? P.hist[(size_t)d * P.tiles + blockIdx.x + 1] : P.dtot[d];
    long long tot;
    const long long below = block_excl_scan64(P.dtot[d], s_tmp, &tot);
    if (P.count_out && blockIdx.x == 0 && d == 0) *P.count_out = (int)tot;
    const long long loff = block_excl_scan64(next - here, s_tmp, &tot);
    if (d == 0) s_count = (unsigned)tot;
    s_run[d] = (unsigned)loff;
    s_gofs[d] = (unsigned)(below + here - loff);   // modulo 2^32; slot + this is in range
    for (int w = 0; w < kSortWaves; ++w) s_wcnt[w][d] = 0;
  }
  __syncthreads();
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  const unsigned long long lt = (1ull << lane) - 1ull;
  unsigned off[PER];   // offset among this wave's items of the same digit
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const bool live = item[r];
    if (live && P.marks) P.marks[sort_item<PER>(base, r)] = 0;
    const unsigned d = digit_of(key[r], P.shift);
    // lanes of this wave with the same digit
    unsigned long long peers = __ballot(live);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const unsigned long long ones = __ballot(live && ((d >> bit) & 1u));
      peers &= ((d >> bit) & 1u) ? ones : ~ones;
    }
    const unsigned rank = (unsigned)__popcll(peers & lt);
    const unsigned before = live ? s_wcnt[wv][d] : 0u;
    wave_lds_sync();   // every lane has read its counter before the leaders add
    off[r] = before + rank;
    if (live && rank == 0) s_wcnt[wv][d] = before + (unsigned)__popcll(peers);
    wave_lds_sync();
  }
  __syncthreads();
  {
    // per digit: counts of the waves before each wave
    const int d = threadIdx.x;
    unsigned acc = 0;
    for (int w = 0; w < kSortWaves; ++w) {
      const unsigned c = s_wcnt[w][d];
      s_wcnt[w][d] = acc;
      acc += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    if (item[r]) {
      const unsigned d = digit_of(key[r], P.shift);
      const unsigned slot = s_run[d] + s_wcnt[wv][d] + off[r];
      s_key[slot] = key[r];
      s_val[slot] = val[r];
    }
  }
  __syncthreads();
  const int count = (int)s_count;
  for (int j = threadIdx.x; j < count; j += kBlock) {
    const unsigned k = s_key[j];
    const unsigned pos = s_gofs[digit_of(k, P.shift)] + (unsigned)j;
    P.key_out[pos] = k;
    P.val_out[pos] = s_val[j];
  }
}

// One pass on stream s: items [0, P.n), digit (key >> P.shift) & 255.
// P.tiles must be sort_tiles<PER>(P.n).
template <int PER = kSortPer>
inline void sort_pass(const SortPass& P, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_hist<PER>, dim3(P.tiles), dim3(kBlock), 0, s, P);
  hipLaunchKernelGGL(k_sort_scan, dim3(kDigits), dim3(kBlock), 0, s, P);
  hipLaunchKernelGGL(k_sort_scatter<PER>, dim3(P.tiles), dim3(kBlock), 0, s, P);
}

// The rest of a pass whose digit counts are already in P.hist (k_sort_hist
// ran earlier on the same stream with the same P): scan and scatter.
template <int PER = kSortPer>
inline void sort_pass_counted(const SortPass& P, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_scan, dim3(kDigits), dim3(kBlock), 0, s, P);
  hipLaunchKernelGGL(k_sort_scatter<PER>, dim3(P.tiles), dim3(kBlock), 0, s, P);
}

template <int PER = kSortPer>
inline int sort_tiles(long long n) { return (int)((n + PER * kBlock - 1) / (PER * kBlock)); }

// Ascending bitonic sort of len int32 items by one workgroup (indices past
// the end act as +infinity and never move); get/put address LDS or global
// memory.  Every comparator stage ends with a barrier.
template <typename Get, typename Put>
__device__ void bitonic_sort_block(int len, int pow2, Get get, Put put) {
  for (int size = 2; size <= pow2; size <<= 1) {
    // first step of each merge: compare i with its mirror in the size-block
    for (int i = threadIdx.x; i < pow2 / 2; i += blockDim.x) {
      int blk = i / (size / 2), off = i % (size / 2);
      int a = blk * size + off, b = blk * size + size - 1 - off;
      if (b < len) {
        int x = get(a), y = get(b);
        if (x > y) { put(a, y); put(b, x); }
      }
    }
    __syncthreads();
    for (int stride = size / 4; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < pow2 / 2; i += blockDim.x) {
        int blk = i / stride, off = i % stride;
        int a = blk * 2 * stride + off, b = a + stride;
        if (b < len) {
          int x = get(a), y = get(b);
          if (x > y) { put(a, y); put(b, x); }
        }
      }
      __syncthreads();
    }
  }
}

}  // namespace
}  // namespace hg
