// hg_sort.h -- stable LSD radix sort of (uint32 key, int32 value) pairs,
// 8 bits per pass, for the move-sequence, rebalancing and contraction
// kernels.  A pass is three launches: per-tile digit counts, a scan of each
// digit's counts over the tiles, and a stable scatter.  Included by each
// source file that sorts (the kernels have internal linkage there).
#pragma once

#include "hg_device.h"
#include "hg_internal.h"

namespace hg {
namespace {

constexpr int kSortTile = kTile;            // items per radix-sort workgroup (4 per thread)
constexpr int kDigits = 256;                // 8-bit digits

struct SortPass {
  const unsigned* key_in;
  const int* val_in;
  unsigned* key_out;
  int* val_out;
  unsigned* hist;   // [kDigits][tiles], digit-major
  unsigned* dtot;   // [kDigits]
  int n, tiles, shift;
};

__device__ __forceinline__ unsigned digit_of(unsigned key, int shift) {
  return (key >> shift) & (kDigits - 1);
}

__global__ __launch_bounds__(kBlock) void k_sort_hist(SortPass P) {
  __shared__ unsigned s_h[kDigits];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortTile / kBlock; ++r) {
    const long long i = base + r * kBlock + threadIdx.x;
    if (i < P.n) atomicAdd(&s_h[digit_of(P.key_in[i], P.shift)], 1u);
  }
  __syncthreads();
  P.hist[(size_t)threadIdx.x * P.tiles + blockIdx.x] = s_h[threadIdx.x];
}

// One workgroup per digit: exclusive scan of its per-tile counts; total.
__global__ __launch_bounds__(kBlock) void k_sort_scan(SortPass P) {
  __shared__ long long s_tmp[kBlock / kWave];
  unsigned* row = P.hist + (size_t)blockIdx.x * P.tiles;
  long long carry = 0;
  for (int b = 0; b < P.tiles; b += kBlock) {
    const int i = b + threadIdx.x;
    const long long v = i < P.tiles ? row[i] : 0;
    long long tot;
    const long long ex = block_excl_scan64(v, s_tmp, &tot);
    if (i < P.tiles) row[i] = (unsigned)(carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0) P.dtot[blockIdx.x] = (unsigned)carry;
}

// Stable scatter of one tile: items r*kBlock + threadIdx.x for r = 0..3 in
// order; ranks among equal digits by wave ballots, waves and rounds in order.
__global__ __launch_bounds__(kBlock) void k_sort_scatter(SortPass P) {
  __shared__ unsigned s_base[kDigits];
  __shared__ unsigned s_wcnt[kBlock / kWave][kDigits];
  __shared__ long long s_tmp[kBlock / kWave];
  // digit bases: digits below d in full, plus this digit in earlier tiles
  long long tot;
  const long long below = block_excl_scan64(P.dtot[threadIdx.x], s_tmp, &tot);
  s_base[threadIdx.x] = (unsigned)below + P.hist[(size_t)threadIdx.x * P.tiles + blockIdx.x];
  for (int w = 0; w < kBlock / kWave; ++w) s_wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const long long base = (long long)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortTile / kBlock; ++r) {
    const long long i = base + r * kBlock + threadIdx.x;
    const bool live = i < P.n;
    unsigned key = 0;
    int val = 0;
    unsigned d = 0;
    if (live) {
      key = P.key_in[i];
      val = P.val_in[i];
      d = digit_of(key, P.shift);
    }
    // lanes of this wave with the same digit
    unsigned long long peers = __ballot(live);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const unsigned long long ones = __ballot(live && ((d >> bit) & 1u));
      peers &= ((d >> bit) & 1u) ? ones : ~ones;
    }
    const unsigned rank = (unsigned)__popcll(peers & lt);
    if (live && rank == 0) s_wcnt[wv][d] = (unsigned)__popcll(peers);
    __syncthreads();
    if (live) {
      unsigned pos = s_base[d] + rank;
      for (int w = 0; w < wv; ++w) pos += s_wcnt[w][d];
      P.key_out[pos] = key;
      P.val_out[pos] = val;
    }
    __syncthreads();
    unsigned add = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      add += s_wcnt[w][threadIdx.x];
      s_wcnt[w][threadIdx.x] = 0;
    }
    s_base[threadIdx.x] += add;
    __syncthreads();
  }
}

// One pass on stream s: items [0, P.n), digit (key >> P.shift) & 255.
inline void sort_pass(const SortPass& P, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_hist, dim3(P.tiles), dim3(kBlock), 0, s, P);
  hipLaunchKernelGGL(k_sort_scan, dim3(kDigits), dim3(kBlock), 0, s, P);
  hipLaunchKernelGGL(k_sort_scatter, dim3(P.tiles), dim3(kBlock), 0, s, P);
}

inline int sort_tiles(long long n) { return (int)((n + kSortTile - 1) / kSortTile); }

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
