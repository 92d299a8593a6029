// hg_device.h -- wavefront-level building blocks for gfx950 (64-wide waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hg_internal.h"

namespace hg {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Make LDS writes of this wave visible to the other lanes of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap the hardware
// workgroup id so that each XCD works on one contiguous range of logical
// workgroups: neighbouring vertices (which share nets) then hit the same L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned bid, unsigned nblocks) {
  unsigned xcd = bid % kNumXcd, local = bid / kNumXcd;
  unsigned per = nblocks / kNumXcd, rem = nblocks % kNumXcd;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// ---- convergent wave reductions (every lane of the wave must call) ----
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int w = __shfl_up(v, o);
    if (lane >= o) v += w;
  }
  return v;
}

__device__ __forceinline__ long long wave_incl_scan64(long long v) {
  int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    long long w = __shfl_up(v, o);
    if (lane >= o) v += w;
  }
  return v;
}

// Workgroup-wide sum of a 64-bit value (all threads call; kBlock threads).
__device__ __forceinline__ long long block_sum64(long long v, long long* s_tmp /*[kBlock/kWave]*/) {
  v = wave_sum(v);
  int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) s_tmp[w] = v;
  __syncthreads();
  long long r = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kWave; ++i) r += s_tmp[i];
  return r;
}

// Workgroup-wide exclusive scan of a 64-bit value; returns the exclusive
// prefix and writes the total to *total.
__device__ __forceinline__ long long block_excl_scan64(long long v, long long* s_tmp,
                                                       long long* total) {
  long long incl = wave_incl_scan64(v);
  int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == kWave - 1) s_tmp[w] = incl;
  __syncthreads();
  long long off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kWave; ++i) {
    long long x = s_tmp[i];
    if (i < w) off += x;
    tot += x;
  }
  *total = tot;
  return off + incl - v;
}

// Wave-aggregated append: one atomic per wave.  Convergent.  Returns the slot
// index for lanes with pred, -1 otherwise.
__device__ __forceinline__ int wave_append(unsigned int* counter, bool pred) {
  unsigned long long mask = __ballot(pred);
  int base = 0;
  if (mask) {
    int leader = __ffsll((long long)mask) - 1;
    if (lane_id() == leader) base = (int)atomicAdd(counter, (unsigned int)__popcll(mask));
    base = __shfl(base, leader);
  }
  return pred ? base + __popcll(mask & (((unsigned long long)1 << lane_id()) - 1)) : -1;
}

// A select candidate: gain in the high word, target block in the low word.
__device__ __forceinline__ long long pack_cand(int gain, int target) {
  return ((long long)gain << 32) | (unsigned)target;
}
__device__ __forceinline__ int cand_target(long long x) { return (int)(x & 0xffffffffLL); }
__device__ __forceinline__ int cand_gain(long long x) { return (int)(x >> 32); }

// The same pointer in the global address space.  Pointers that reach a
// kernel inside a descriptor (rather than as a plain kernel argument) are
// generic to the compiler, which then issues flat loads; global loads are the
// plain vector-memory path.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global_ptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// Plain vector types for 8- and 16-byte global loads and nontemporal stores
// (the HIP vector structs cannot be copied out of another address space, nor
// passed to the nontemporal builtins).
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef long long i64x2 __attribute__((ext_vector_type(2)));

}  // namespace hg
