// hg_sweep.h -- what the vertex sweeps (LP select, gains) read per incident
// net, from either the full net record or the compact Lambda/S view.
#pragma once

#include "hg_device.h"
#include "hg_internal.h"

namespace hg {

// Per incident net e of a vertex in block a (aw = a / 32):
//   w    w(e)
//   cut  lambda(e) > 1
//   L    Lambda(e) bitset words
//   S    the S(e) word that holds a's bit
template <int WK, int VIEW>
__device__ __forceinline__ void read_net(const unsigned* __restrict__ netstate, int rw,
                                         const unsigned* __restrict__ view, int e, int aw,
                                         unsigned& w, bool& cut, unsigned (&L)[WK], unsigned& S) {
  if constexpr (VIEW == kView16) {
    const unsigned x = global_ptr(view)[e];
    L[0] = x & 0xffffu;
    S = x >> 16;
    w = 1;
    cut = __popc(L[0]) > 1;
  } else if constexpr (VIEW == kView32) {
    const u32x2 x = global_ptr(reinterpret_cast<const u32x2*>(view))[e];
    L[0] = x.x;
    S = x.y;
    w = 1;
    cut = __popc(L[0]) > 1;
  } else if constexpr (VIEW == kView64) {
    const u32x4 x = global_ptr(reinterpret_cast<const u32x4*>(view))[e];
    L[0] = x.x;
    L[1] = x.y;
    S = aw ? x.w : x.z;
    w = 1;
    cut = __popc(x.x) + __popc(x.y) > 1;
  } else {
    const auto r = global_ptr(netstate + (long long)e * rw);
    const u32x4 q = *global_ptr(reinterpret_cast<const u32x4*>(netstate + (long long)e * rw));
    w = q.x;
    cut = q.y > 1u;
    L[0] = q.z;
    if (WK == 1) {
      S = q.w;
    } else {
      L[1] = q.w;
#pragma unroll
      for (int j = 2; j < WK; ++j) L[j] = r[2 + j];
      S = r[2 + WK + aw];
    }
  }
}

}  // namespace hg
