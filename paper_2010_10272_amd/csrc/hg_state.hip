// hg_state.hip -- pin counts Phi(e,i), connectivity sets Lambda(e), the
// singleton sets S(e) = {i : Phi(e,i) = 1}, block weights c(V_i) and km1.
//
// Section "Preliminaries" defines Phi, Lambda, lambda and km1; subsection
// "Data Structures for Gain Calculation" keeps Phi and a bitset Lambda per
// net.  Here one group of G lanes owns one net at a time: it counts the net's
// pins per block in LDS, writes the Phi row (16-byte streaming stores when
// rows are aligned, coalesced 4-byte stores otherwise) and builds the bitsets
// with wave ballots.  No global atomics touch Phi, so the result is
// deterministic by construction.
#include "hg_device.h"
#include "hg_internal.h"
#include "hg_lp.h"
#include "hg_netrec.h"

namespace hg {

constexpr int kStateGrid = 8192;   // persistent workgroups of the single-instance net sweep
constexpr int kKm1Chunk = kBlock * 8;

__device__ __forceinline__ WorkItem contiguous_units(long long units) {
  const long long lb = xcd_remap(blockIdx.x, gridDim.x);
  const long long per = (units + gridDim.x - 1) / gridDim.x;
  long long end = (lb + 1) * per;
  if (end > units) end = units;
  WorkItem w;
  w.inst = 0;
  w.first = (int)(lb * per);
  w.stride = 1;
  w.count = lb * per < end ? (int)(end - lb * per) : 0;
  return w;
}

// Pin slots per lane and pass: the pin loads of kCountSlots * G pins, then
// their block-id loads, are in flight together (the sweep is bound by their
// latency); slots past the net's end repeat its first pin and are masked.
// Block ids are gathered from the byte copy part8 that the block-weight
// sweep writes just before (a quarter of the bytes of part: on a 4M-vertex
// netlist 4 MB, which an XCD's L2 mostly holds, instead of 16 MB).
constexpr int kCountSlots = 4;

// Unit: kBlock/G consecutive nets (one per group).  G lanes per net (G
// divides 64, G >= the record words); LDS counters: (kBlock/G) groups x k
// ints.
template <int G>
__global__ __launch_bounds__(kBlock) void k_pincounts(Launch L) {
  extern __shared__ int s_cnt[];   // [kBlock/G][k]
  __shared__ long long s_tmp[kBlock / kWave];
  constexpr int kGroups = kBlock / G;
  const WorkItem wi = work_item(L, contiguous_units((L.one.m + kGroups - 1) / kGroups));
  if (wi.count == 0) return;
  const InstDesc D = inst_desc(L, wi.inst);
  const int grp = threadIdx.x / G;
  const int gl = threadIdx.x % G;
  const int k = D.k, m = D.m, rw = D.rw;
  int* cnt = s_cnt + grp * k;
  // Phi rows leave as 16-byte streaming stores when rows are 16-byte aligned
  const bool vec_phi = (k & 3) == 0 && ((uintptr_t)D.phi & 15) == 0;
  long long km1_local = 0;
  // the next net's pin range is loaded while this net's pins are counted
  // (one dependent load fewer per net)
  long long nb = 0, nt = 0;
  {
    const long long e0 = (long long)wi.first * kGroups + grp;
    if (e0 < m) {
      nb = D.eptr[e0];
      nt = D.eptr[e0 + 1];
    }
  }
  for (int it = 0; it < wi.count; ++it) {
    const long long e = ((long long)wi.first + (long long)it * wi.stride) * kGroups + grp;
    const long long b = nb, t = nt;
    if (e < m)
      for (int i = gl; i < k; i += G) cnt[i] = 0;
    wave_lds_sync();
    if (it + 1 < wi.count) {
      const long long en = e + (long long)wi.stride * kGroups;
      nb = nt = 0;
      if (en < m) {
        nb = D.eptr[en];
        nt = D.eptr[en + 1];
      }
    }
    for (long long p0 = b + gl; p0 < t; p0 += kCountSlots * G) {
      int v[kCountSlots];
#pragma unroll
      for (int q = 0; q < kCountSlots; ++q) v[q] = D.pins[p0 + q * G < t ? p0 + q * G : p0];
#pragma unroll
      for (int q = 0; q < kCountSlots; ++q) v[q] = D.part8[v[q]];
#pragma unroll
      for (int q = 0; q < kCountSlots; ++q) {
        // part itself was checked by the block-weight sweep
        if (p0 + q * G < t && (unsigned)v[q] < (unsigned)k) atomicAdd(&cnt[v[q]], 1);
      }
    }
    wave_lds_sync();
    if (e < m) {
      const NetBits bits = net_bits<G>(k, gl, [&](int i) { return cnt[i]; });
      int* phi_row = D.phi + e * (long long)k;
      if (vec_phi) {
        for (int i = gl; i < (k >> 2); i += G)
          __builtin_nontemporal_store(reinterpret_cast<const i32x4*>(cnt)[i],
                                      reinterpret_cast<i32x4*>(phi_row) + i);
      } else {
        for (int i = gl; i < k; i += G) phi_row[i] = cnt[i];
      }
      const int w = D.ewgt ? D.ewgt[e] : 1;
      write_netrec(D.netstate + e * (long long)rw, gl, w, bits, k);
      if (D.view != kViewFull) {
        write_view(D.view_ptr, e, D.view, gl, bits);
      } else if (gl < view_words(k)) {
        // the compact copy is not used for weighted nets: keep it defined (zero)
        D.view_ptr[e * view_words(k) + gl] = 0u;
      }
      if (gl == 0) km1_local += (long long)(bits.lambda - 1) * w;
    }
    wave_lds_sync();
  }
  const long long tot = block_sum64(km1_local, s_tmp);
  if (threadIdx.x == 0 && tot)
    atomicAdd(&D.red[blockIdx.x % kSlots], (unsigned long long)tot);
}

// Unit: one instance.  Sum its km1 slots into *km1 (or just clear them) and
// fold the block-weight slot rows of the sweep before into block_w (clearing
// them for the rounds).
__global__ __launch_bounds__(kBlock) void k_count_epilogue(Launch L, int want_km1) {
  const WorkItem wi = work_item(L, WorkItem{0, 0, 1, 1});
  const InstDesc D = inst_desc(L, wi.inst);
  if (threadIdx.x < kWave) {
    const int lane = lane_id();
    long long v = (long long)D.red[lane];
    D.red[lane] = 0;
    v = wave_sum(v);
    if (lane == 0 && want_km1) *D.km1 = v;
  }
  const size_t ks = (size_t)D.k;
  for (int i = threadIdx.x; i < D.k; i += kBlock) {
    long long* col = D.bw_slots + i;
    long long w = 0;
    for (int s0 = 0; s0 < kSlots; s0 += 16) {      // 16 loads in flight, then the clears
      long long cells[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) cells[q] = col[(s0 + q) * ks];
#pragma unroll
      for (int q = 0; q < 16; ++q) w += cells[q];
#pragma unroll
      for (int q = 0; q < 16; ++q) col[(s0 + q) * ks] = 0;
    }
    D.block_w[i] = w;
  }
}

// Unit: kBwChunk consecutive vertices.  LDS partial sums per workgroup, then
// one atomic per block into the workgroup's slot row (the epilogue folds the
// rows into block_w).  Every vertex's block also goes to part8 (one byte).
// With mark_eligible every vertex is also made eligible (the start of a
// refinement).
__global__ __launch_bounds__(kBlock) void k_block_weights(Launch L, int mark_eligible) {
  __shared__ unsigned long long s_w[HG_MAX_K];
  const WorkItem wi = work_item(L, contiguous_units((L.one.n + kBwChunk - 1) / kBwChunk));
  if (wi.count == 0) return;
  const InstDesc D = inst_desc(L, wi.inst);
  const int k = D.k, n = D.n;
  for (int i = threadIdx.x; i < k; i += kBlock) s_w[i] = 0;
  __syncthreads();
  int err = 0;
  constexpr int kPer = kBwChunk / kBlock;
  for (int it = 0; it < wi.count; ++it) {
    const long long base = ((long long)wi.first + (long long)it * wi.stride) * kBwChunk;
    // every vertex's block and weight requested before the first wait
    int blk[kPer], cw[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const long long v = base + (long long)j * kBlock + threadIdx.x;
      blk[j] = v < n ? D.part[v] : 0;
      cw[j] = v < n && D.vwgt ? D.vwgt[v] : 1;
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const long long v = base + (long long)j * kBlock + threadIdx.x;
      if (v < n) {
        if (mark_eligible) D.eligible[v] = 1;
        D.part8[v] = (unsigned char)blk[j];
        if ((unsigned)blk[j] < (unsigned)k)
          atomicAdd(&s_w[blk[j]], (unsigned long long)cw[j]);
        else
          err = kErrPart;
      }
    }
  }
  if (err) atomicOr(D.err_flags, err);
  __syncthreads();
  long long* my_w = D.bw_slots + (size_t)(blockIdx.x % kSlots) * k;
  for (int i = threadIdx.x; i < k; i += kBlock)
    if (s_w[i]) atomicAdd((unsigned long long*)&my_w[i], s_w[i]);
}

// km1 partial sums from the net-state records (single instance only).
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

// Lanes per net for the net-centric sweeps (pin counts, finalize): enough
// lanes to hold every word of the net record (2 + 2 * bit_words(k), padded),
// and no more than that (but 8 for 4 < k <= 64): most nets have only a
// handful of pins, so narrower groups put more nets' loads in flight per
// wavefront.
int group_lanes(int k) {
  if (k <= 4) return 4;
  return net_words(k) > 8 ? net_words(k) : 8;
}

size_t pincount_lds(int G, int k) { return sizeof(int) * (size_t)(kBlock / G) * k; }

GroupKernel pincount_kernel(int k) { return pincount_kernel_g(group_lanes(k)); }

GroupKernel pincount_kernel_g(int G) {
  switch (G) {
    case 4: return k_pincounts<4>;
    case 8: return k_pincounts<8>;
    case 16: return k_pincounts<16>;
    default: return k_pincounts<32>;
  }
}

void single_count_plan(const InstDesc& d, CountPlan& plan) {
  plan = CountPlan();
  const Launch L = single_launch(d);
  PlanLaunch pc;
  pc.kernel = (void*)pincount_kernel(d.k);
  pc.grid = grid_cap(d.m, kBlock / group_lanes(d.k), kStateGrid);
  pc.lds = pincount_lds(group_lanes(d.k), d.k);
  pc.L = L;
  plan.pincounts.push_back(pc);
  plan.instances.grid = 1;
  plan.instances.L = L;
  plan.vertices.grid = grid_cap(d.n, kBwChunk, 4096);
  plan.vertices.L = L;
}

// Block weights (and the byte partition), then pin counts, then km1 and the
// block-weight fold.
hipError_t launch_counts(const CountPlan& plan, bool want_km1, bool mark_eligible, hipStream_t s) {
  hipLaunchKernelGGL(k_block_weights, dim3(plan.vertices.grid), dim3(kBlock), 0, s,
                     plan.vertices.L, mark_eligible ? 1 : 0);
  for (const PlanLaunch& pl : plan.pincounts)
    hipLaunchKernelGGL((GroupKernel)pl.kernel, dim3(pl.grid), dim3(kBlock), pl.lds, s, pl.L);
  hipLaunchKernelGGL(k_count_epilogue, dim3(plan.instances.grid), dim3(kBlock), 0, s,
                     plan.instances.L, want_km1 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_km1(hg_graph_s* g, int k, const unsigned* netstate, long long* km1,
                      hipStream_t s) {
  unsigned long long* slots = (unsigned long long*)(g->ws + g->lay.red);
  hipLaunchKernelGGL(k_km1, dim3(grid_cap(g->m, kKm1Chunk, kStateGrid)), dim3(kBlock), 0, s,
                     g->m, net_words(k), netstate, slots);
  hipLaunchKernelGGL(k_sum_slots, dim3(1), dim3(kWave), 0, s, slots, km1);
  return hipGetLastError();
}

}  // namespace hg
