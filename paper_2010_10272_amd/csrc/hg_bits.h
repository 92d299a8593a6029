// hg_bits.h -- bit-sliced per-block counters held in registers.
//
// For a vertex u, conn_i = w({e in I(u) : i in Lambda(e)}) is needed for every
// block i; then p_i(u) = w(I(u)) - conn_i (section "Parallel Gain
// Calculation").  When w(I(u)) <= 255 every conn_i fits in 8 bits, so the k
// counters are stored transposed: plane p holds bit p of all counters, one
// 32-bit word per 32 blocks.  Adding w(e) to every block of Lambda(e) is a
// ripple-carry add of the bitset into the planes, and the arg-max over a set
// of blocks is a walk from the top plane down.  Everything stays in VGPRs:
// one thread per vertex, no LDS, full occupancy for the random net gathers.
#pragma once

#include "hg_internal.h"

namespace hg {

template <int WK>
struct BitCounters {
  unsigned c[kPlanes][WK];

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int p = 0; p < kPlanes; ++p)
#pragma unroll
      for (int w = 0; w < WK; ++w) c[p][w] = 0u;
  }

  // counter_i += wgt for every i in mask (wgt in [1, 255]).
  __device__ __forceinline__ void add(const unsigned (&mask)[WK], unsigned wgt) {
#pragma unroll
    for (int j = 0; j < kPlanes; ++j) {
      if ((wgt >> j) & 1u) {
#pragma unroll
        for (int w = 0; w < WK; ++w) {
          unsigned carry = mask[w];
#pragma unroll
          for (int p = 0; p < kPlanes; ++p) {
            if (p >= j) {
              unsigned t = c[p][w] & carry;
              c[p][w] ^= carry;
              carry = t;
            }
          }
        }
      }
    }
  }

  // counter_i += 1 for every i in mask: one ripple-carry pass, no weight
  // bits to test (unit net weights).
  __device__ __forceinline__ void add_one(const unsigned (&mask)[WK]) {
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      unsigned carry = mask[w];
#pragma unroll
      for (int p = 0; p < kPlanes; ++p) {
        const unsigned t = c[p][w] & carry;
        c[p][w] ^= carry;
        carry = t;
      }
    }
  }

  // Blocks with a non-zero counter.
  __device__ __forceinline__ void nonzero(unsigned (&out)[WK]) const {
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      unsigned x = 0;
#pragma unroll
      for (int p = 0; p < kPlanes; ++p) x |= c[p][w];
      out[w] = x;
    }
  }

  // Narrow `set` to the blocks whose counter is maximal within it; returns
  // that maximum.  `set` must be non-empty.
  __device__ __forceinline__ unsigned narrow_to_max(unsigned (&set)[WK]) const {
    unsigned best = 0;
#pragma unroll
    for (int p = kPlanes - 1; p >= 0; --p) {
      unsigned t[WK];
      unsigned any = 0;
#pragma unroll
      for (int w = 0; w < WK; ++w) {
        t[w] = set[w] & c[p][w];
        any |= t[w];
      }
      if (any) {
#pragma unroll
        for (int w = 0; w < WK; ++w) set[w] = t[w];
        best |= 1u << p;
      }
    }
    return best;
  }

  // Counter of block 32*w + b (w a compile-time word index).
  __device__ __forceinline__ unsigned value(int w, int b) const {
    unsigned v = 0;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) v |= ((c[p][w] >> b) & 1u) << p;
    return v;
  }
};

}  // namespace hg
