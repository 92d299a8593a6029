// hg_state.hip -- pin counts Phi(e,i), connectivity sets Lambda(e), the
// singleton sets S(e) = {i : Phi(e,i) = 1}, block weights c(V_i) and km1.
//
// Section "Preliminaries" defines Phi, Lambda, lambda and km1; subsection
// "Data Structures for Gain Calculation" keeps Phi and a bitset Lambda per
// net.  Here one group of G lanes owns one net at a time: it counts the net's
// pins per block in LDS, writes the Phi row with coalesced stores and builds
// the bitsets with wave ballots.  No global atomics touch Phi, so the result
// is deterministic by construction.
#include "hg_device.h"
#include "hg_internal.h"
#include "hg_netrec.h"

namespace hg {

constexpr int kStateGrid = 8192;   // persistent workgroups of the net sweep

// G lanes per net (G divides 64); LDS counters: (kBlock/G) groups x k ints.
// Workgroup lb owns a contiguous run of nets (XCD-aware order).
template <int G>
__global__ __launch_bounds__(kBlock) void k_pincounts(int m, int k, int rw,
                                                      const long long* __restrict__ eptr,
                                                      const int* __restrict__ pins,
                                                      const int* __restrict__ ewgt,
                                                      const int* __restrict__ part,
                                                      int* __restrict__ phi,
                                                      unsigned* __restrict__ netstate,
                                                      unsigned long long* __restrict__ km1_slots,
                                                      int* __restrict__ err_flags,
                                                      unsigned* __restrict__ view, int view_kind) {
  extern __shared__ int s_cnt[];   // [kBlock/G][k]
  __shared__ long long s_tmp[kBlock / kWave];
  constexpr int kGroups = kBlock / G;
  const int grp = threadIdx.x / G;
  const int gl = threadIdx.x % G;
  int* cnt = s_cnt + grp * k;
  const long long lb = xcd_remap(blockIdx.x, gridDim.x);
  const long long per = (((long long)m + kGroups - 1) / kGroups + gridDim.x - 1) / gridDim.x;
  const long long e_begin = lb * per * kGroups;
  long long e_end = e_begin + per * kGroups;
  if (e_end > m) e_end = m;
  long long km1_local = 0;
  int err = 0;
  for (long long e = e_begin + grp; e < e_end; e += kGroups) {
    for (int i = gl; i < k; i += G) cnt[i] = 0;
    wave_lds_sync();
    const long long b = eptr[e], t = eptr[e + 1];
    for (long long p = b + gl; p < t; p += G) {
      const int blk = part[pins[p]];
      if ((unsigned)blk < (unsigned)k) atomicAdd(&cnt[blk], 1);
      else err = kErrPart;
    }
    wave_lds_sync();
    NetBits bits;
    netbits_from_counts<G>(cnt, k, gl, bits, phi + e * (long long)k);
    const int w = ewgt ? ewgt[e] : 1;
    write_netrec(netstate + e * (long long)rw, gl, w, bits, k);
    if (view_kind != kViewFull) write_view(view, e, view_kind, gl, bits);
    if (gl == 0) km1_local += (long long)(bits.lambda - 1) * w;
    wave_lds_sync();
  }
  if (err) atomicOr(err_flags, err);
  const long long tot = block_sum64(km1_local, s_tmp);
  if (threadIdx.x == 0 && tot)
    atomicAdd(&km1_slots[blockIdx.x % kSlots], (unsigned long long)tot);
}

// Block weights: LDS partial sums per workgroup, then one atomic per block.
__global__ __launch_bounds__(kBlock) void k_block_weights(int n, int k, const int* part,
                                                          const int* vwgt,
                                                          unsigned long long* block_w,
                                                          int* err_flags) {
  __shared__ unsigned long long s_w[HG_MAX_K];
  for (int i = threadIdx.x; i < k; i += kBlock) s_w[i] = 0;
  __syncthreads();
  long long stride = (long long)gridDim.x * kBlock;
  int err = 0;
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
    int blk = part[v];
    if ((unsigned)blk < (unsigned)k)
      atomicAdd(&s_w[blk], (unsigned long long)(vwgt ? vwgt[v] : 1));
    else
      err = kErrPart;
  }
  if (err) atomicOr(err_flags, err);
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock)
    if (s_w[i]) atomicAdd(&block_w[i], s_w[i]);
}

// km1 partial sums from the net-state records.
__global__ __launch_bounds__(kBlock) void k_km1(int m, int rw, const unsigned* netstate,
                                                unsigned long long* km1_slots) {
  __shared__ long long s_tmp[kBlock / kWave];
  long long stride = (long long)gridDim.x * kBlock;
  long long acc = 0;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < m; e += stride) {
    const unsigned* r = netstate + e * rw;
    acc += (long long)((int)r[1] - 1) * (int)r[0];
  }
  acc = block_sum64(acc, s_tmp);
  if (threadIdx.x == 0 && acc) atomicAdd(&km1_slots[blockIdx.x % kSlots], (unsigned long long)acc);
}

// Sum the kSlots partials into *out and clear them (one wavefront).
__global__ void k_sum_slots(unsigned long long* slots, long long* out) {
  const int lane = lane_id();
  long long v = (long long)slots[lane];
  slots[lane] = 0;
  v = wave_sum(v);
  if (lane == 0) *out = v;
}

static unsigned grid_cap(long long items, int per_block, int cap) {
  long long b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

template <int G>
static void launch_pincounts_g(hg_graph_s* g, int k, const int* part, int* phi,
                               unsigned* netstate, unsigned long long* slots, int* err,
                               hipStream_t s) {
  unsigned grid = grid_cap(g->m, kBlock / G, kStateGrid);
  size_t lds = sizeof(int) * (size_t)(kBlock / G) * k;
  hipLaunchKernelGGL(k_pincounts<G>, dim3(grid), dim3(kBlock), lds, s, g->m, k, net_words(k),
                     g->eptr, g->pins, g->ewgt, part, phi, netstate, slots, err,
                     netstate + (size_t)g->m * net_words(k), net_view(k, g->unit_nets));
}

// Lanes per net for the net-centric sweeps: enough lanes to hold every word
// of the net record (2 + 2 * bit_words(k), padded), few enough that a wave
// works on several nets at once (most nets have only a handful of pins).
int group_lanes(int k) {
  if (k <= 4) return 4;
  if (k <= 8) return 8;
  if (k <= 128) return 16;
  return 32;
}

hipError_t launch_pincounts(hg_graph_s* g, int k, const int* part, int* phi,
                            unsigned* netstate, long long* block_w, long long* km1,
                            hipStream_t s) {
  int* err = (int*)(g->ws + g->lay.flags);
  unsigned long long* slots = (unsigned long long*)(g->ws + g->lay.red);
  switch (group_lanes(k)) {
    case 4: launch_pincounts_g<4>(g, k, part, phi, netstate, slots, err, s); break;
    case 8: launch_pincounts_g<8>(g, k, part, phi, netstate, slots, err, s); break;
    case 16: launch_pincounts_g<16>(g, k, part, phi, netstate, slots, err, s); break;
    case 32: launch_pincounts_g<32>(g, k, part, phi, netstate, slots, err, s); break;
    default: launch_pincounts_g<64>(g, k, part, phi, netstate, slots, err, s); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (net_view(k, g->unit_nets) == kViewFull && view_words(k) > 0) {
    // the compact copy is not used for weighted nets: keep it defined (zero)
    e = fill_i32((int*)netstate + (size_t)g->m * net_words(k), 0,
                 (long long)g->m * view_words(k), s);
    if (e != hipSuccess) return e;
  }
  if (km1) {
    hipLaunchKernelGGL(k_sum_slots, dim3(1), dim3(kWave), 0, s, slots, km1);
  } else {
    e = fill_i64((long long*)slots, 0, kSlots, s);
    if (e != hipSuccess) return e;
  }
  e = fill_i64(block_w, 0, k, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_block_weights, dim3(grid_cap(g->n, kBlock * 16, 4096)), dim3(kBlock), 0,
                     s, g->n, k, part, g->vwgt, (unsigned long long*)block_w, err);
  return hipGetLastError();
}

hipError_t launch_km1(hg_graph_s* g, int k, const unsigned* netstate, long long* km1,
                      hipStream_t s) {
  unsigned long long* slots = (unsigned long long*)(g->ws + g->lay.red);
  hipLaunchKernelGGL(k_km1, dim3(grid_cap(g->m, kBlock * 8, kStateGrid)), dim3(kBlock), 0, s,
                     g->m, net_words(k), netstate, slots);
  hipLaunchKernelGGL(k_sum_slots, dim3(1), dim3(kWave), 0, s, slots, km1);
  return hipGetLastError();
}

}  // namespace hg
