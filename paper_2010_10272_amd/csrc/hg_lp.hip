// hg_lp.hip -- one synchronous label-propagation round (section "Label
// Propagation"), split into select / approve / apply / finalize kernels that
// all read the round-start state.
//
//   select     per eligible vertex: boundary test, best feasible target by
//              (gain desc, block weight asc, block id asc), move rule; writes
//              a candidate word per vertex and adds c(u) to a per-(target,
//              gain) weight histogram.
//   threshold  per target block: the highest gain g* at which the cumulative
//              candidate weight (from the top gain down) overflows
//              L_max - c(V_t); gains above g* are approved whole.
//   tilesum    per tile of 512 vertices: weight of gain-g* candidates per
//              target block (vertex id order is tile order).
//   tilescan   per target block: the tile where the budget runs out.
//   approve    per tile: decide every candidate; the one boundary tile per
//              block is resolved by a workgroup-wide prefix sum in vertex
//              order.  Approved moves are applied right away: Phi updated
//              with integer atomics (order-independent), the attributed km1
//              change summed from the atomics' old values (subsection
//              "Attributed Gains"), touched nets flagged.
//   finalize   per touched net: Lambda, S and lambda recomputed from the
//              final Phi row, its pins made eligible for the next round.
//   stats      one workgroup per instance sums the counter slots into the
//              round record.
//
// Every kernel takes a Launch: one instance by value, or a batch of
// instances with a per-workgroup work table (see hg_internal.h).
//
// Candidate word: (gain << 32) | target, or -1 for "no candidate".
#include <limits.h>

#include "hg_bits.h"
#include "hg_device.h"
#include "hg_internal.h"
#include "hg_lp.h"
#include "hg_netrec.h"
#include "hg_sweep.h"

namespace hg {


// XCD-aware strided split of `units` over `grid` workgroups: XCD x owns the
// contiguous range [x*per_xcd, (x+1)*per_xcd) and its workgroups take
// neighbouring units side by side.
__device__ __forceinline__ WorkItem xcd_sweep(long long units) {
  const int xcd = blockIdx.x % kNumXcd;
  const int wg_on_xcd = (gridDim.x - xcd + kNumXcd - 1) / kNumXcd;
  const int li = blockIdx.x / kNumXcd;
  const long long per_xcd = (units + kNumXcd - 1) / kNumXcd;
  const long long c_begin = xcd * per_xcd;
  long long c_end = c_begin + per_xcd;
  if (c_end > units) c_end = units;
  WorkItem w;
  w.inst = 0;
  w.first = (int)(c_begin + li);
  w.stride = wg_on_xcd;
  w.count = c_begin + li < c_end ? (int)((c_end - (c_begin + li) + wg_on_xcd - 1) / wg_on_xcd) : 0;
  return w;
}

// Contiguous XCD-aware split: workgroup blockIdx gets units [lb*per, (lb+1)*per).
__device__ __forceinline__ WorkItem xcd_block(long long units) {
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

__device__ __forceinline__ WorkItem single_unit(int unit) {
  WorkItem w;
  w.inst = 0;
  w.first = unit;
  w.count = 1;
  w.stride = 1;
  return w;
}

// --------------------------------------------------------------- select

// Light vertices, one thread each.  Unit: a chunk of 256 vertices.  Single
// instance: persistent grid, XCD-aware sweep (each XCD walks one vertex
// range with its workgroups side by side, so neighbouring vertices' net
// records stay in that XCD's L2).  Candidate weights go to an LDS histogram
// (buckets [0, B) per target block, B = min(256, 2048/k)); higher gains and
// the final flush go to the histogram replica of this workgroup's XCD.
constexpr int kDenseWave = 3 * kWave / 4;   // eligible lanes that make a wave's slice dense

template <int WK, int VIEW, int U>
__global__ __launch_bounds__(kBlock) void k_select_light(Launch L) {
  __shared__ long long s_W[HG_MAX_K];
  __shared__ unsigned s_open[WK];
  __shared__ unsigned long long s_hist[kLdsHistEntries];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_q[kBlock / kWave][2 * kWave];   // per-wave queues of eligible vertices
  const InstDesc D0 = L.one;
  const WorkItem wi = work_item(L, xcd_sweep((D0.n + kBlock - 1) / kBlock));
  if (wi.count == 0) return;
  const InstDesc D = inst_desc(L, wi.inst);
  const int k = D.k, B = D.lds_buckets, n = D.n;
  const long long lmax = D.lmax;
  for (int i = threadIdx.x; i < WK; i += kBlock) s_open[i] = 0;
  for (int i = threadIdx.x; i < k * B; i += kBlock) s_hist[i] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock) {
    long long W = D.block_w[i];
    s_W[i] = W;
    if (W + D.cmax <= lmax) atomicOr(&s_open[i >> 5], 1u << (i & 31));
  }
  __syncthreads();
  unsigned long long* my_hist = D.hist + (size_t)(blockIdx.x % D.hist_reps) * D.hist_stride;
  long long n_elig = 0, n_bnd = 0, n_cand = 0, n_apins = 0;
  // valid-block masks (only blocks < k; guards against stale caller state)
  unsigned valid[WK];
#pragma unroll
  for (int w = 0; w < WK; ++w) {
    const int lo = w * 32;
    valid[w] = k >= lo + 32 ? ~0u : (k > lo ? (1u << (k - lo)) - 1u : 0u);
  }
  const long long* __restrict__ vptr = D.vptr;
  const int* __restrict__ vnets = D.vnets;
  const unsigned* __restrict__ netstate = D.netstate;
  const unsigned* __restrict__ view = D.view_ptr;
  const int rw = D.rw;
  // Each wave queues the eligible vertices of its 64-vertex slices in LDS
  // and processes them 64 at a time, so that later rounds (few eligible
  // vertices) run full waves instead of mostly idle ones; slices that are
  // mostly eligible (every vertex in round 1) are processed in place.  No
  // workgroup barrier is involved, so waves keep sweeping independently.
  // Every vertex gets its moved flag cleared, and the non-eligible ones
  // their "no candidate" word, when its slice is read.
  auto one_vertex = [&](const long long u) {
    const int a = D.part[u];
    if ((unsigned)a >= (unsigned)k) {
      atomicOr(D.err_flags, kErrPart);
      D.cand[u] = -1;
      D.eligible[u] = 0;
      return;
    }
    const long long b0 = vptr[u], b1 = vptr[u + 1];
    if (b1 - b0 > kLightLimit) return;        // heavy vertex: the wavefront kernel owns it
    BitCounters<WK> C;
    C.clear();
    int tot = 0, ben = 0;
    bool bnd = false, heavy = false;
    const int aw = a >> 5;
    const unsigned abit = 1u << (a & 31);
    // Software-pipelined sweep: issue U independent record gathers before
    // consuming any of them (U = 8 for average degrees of 12 and more, else
    // 4).  Slots past the row end load the row's
    // first entry again (always valid) and are masked afterwards, so no load
    // sits in a branch of its own.  With unit nets w(I(u)) is the degree,
    // which the row length already bounds, so only weighted nets are
    // watched for the heavy limit.
    const int deg = (int)(b1 - b0);
    const auto row = global_ptr(vnets + b0);
    for (int jj = 0; jj < deg; jj += U) {
      unsigned w[U], S[U], Lb[U][WK];
      bool cut[U];
      int e[U];
#pragma unroll
      for (int q = 0; q < U; ++q) e[q] = row[jj + q < deg ? jj + q : jj];
#pragma unroll
      for (int q = 0; q < U; ++q)
        read_net<WK, VIEW>(netstate, rw, view, e[q], aw, w[q], cut[q], Lb[q], S[q]);
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (jj + q >= deg) {
          w[q] = 0;
          cut[q] = false;
          S[q] = 0;
#pragma unroll
          for (int x = 0; x < WK; ++x) Lb[q][x] = 0;
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        bnd |= cut[q];
        if (S[q] & abit) ben += (int)w[q];
      }
      if constexpr (VIEW == kViewFull) {
#pragma unroll
        for (int q = 0; q < U; ++q) tot += (int)w[q];
        if (tot > kLightLimit) {
          heavy = true;
          break;
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if constexpr (VIEW != kViewFull) {
          C.add_one(Lb[q]);               // unit nets (masked slots add nothing)
        } else if (w[q]) {
          C.add(Lb[q], w[q]);
        }
      }
    }
    if constexpr (VIEW != kViewFull) tot = deg;
    if (heavy) return;
    D.eligible[u] = 0;
    n_elig += 1;
    long long out = -1;
    if (bnd) {
      n_bnd += 1;
      n_apins += b1 - b0;
      const long long cu = D.vwgt ? D.vwgt[u] : 1;
      unsigned T[WK], F[WK];
      C.nonzero(T);
      unsigned anyF = 0;
#pragma unroll
      for (int w = 0; w < WK; ++w) {
        T[w] &= valid[w];
        if (w == aw) T[w] &= ~abit;
        F[w] = T[w] & s_open[w];
        unsigned rest = T[w] & ~s_open[w];
        while (rest) {
          int b = __ffs(rest) - 1;
          rest &= rest - 1;
          if (s_W[w * 32 + b] + cu <= lmax) F[w] |= 1u << b;
        }
        anyF |= F[w];
      }
      if (anyF) {
        const int conn = (int)C.narrow_to_max(F);
        int t = -1;
        long long tw = 0;
#pragma unroll
        for (int w = 0; w < WK; ++w) {
          unsigned x = F[w];
          while (x) {
            int b = __ffs(x) - 1;
            x &= x - 1;
            int i = w * 32 + b;
            long long Wi = s_W[i];
            if (t < 0 || Wi < tw) {
              t = i;
              tw = Wi;
            }
          }
        }
        const int g = ben - tot + conn;
        if (g > 0 || (g == 0 && tw + cu < s_W[a])) {
          out = pack_cand(g, t);
          n_cand += 1;
          if (g < B)
            atomicAdd(&s_hist[t * B + g], (unsigned long long)cu);
          else
            atomicAdd(&my_hist[t * kBuckets + (g < kBuckets ? g : kBuckets - 1)],
                      (unsigned long long)cu);
        }
      }
    }
    D.cand[u] = out;
  };
  const int lane = lane_id();
  int* my_q = s_q[threadIdx.x / kWave];
  int qn = 0;                                  // this wave's queue length (wave-uniform)
  // one call site of one_vertex (the select body is large): the extra last
  // iteration flushes the queue
  for (int it = 0; it <= wi.count; ++it) {
    long long todo = -1;
    if (it < wi.count) {
      const long long c = (long long)wi.first + (long long)it * wi.stride;
      const long long u = c * kBlock + threadIdx.x;
      bool el = false;
      if (u < n) {
        if (D.moved) D.moved[u] = 0;
        el = D.eligible[u] != 0;
        if (!el) D.cand[u] = -1;
      }
      const unsigned long long mask = __ballot(el);
      const int cnt = __popcll(mask);
      if (cnt >= kDenseWave) {                 // mostly eligible: in place
        todo = el ? u : -1;
      } else {
        if (el) my_q[qn + __popcll(mask & ((1ull << lane) - 1))] = (int)u;
        qn += cnt;                             // < 2 * kWave
        wave_lds_sync();
        if (qn >= kWave) {
          todo = my_q[lane];
          const int rest = qn - kWave;
          const int keep = lane < rest ? my_q[kWave + lane] : 0;
          wave_lds_sync();
          if (lane < rest) my_q[lane] = keep;
          qn = rest;
          wave_lds_sync();
        }
      }
    } else if (lane < qn) {
      todo = my_q[lane];
    }
    if (todo >= 0) one_vertex(todo);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k * B; i += kBlock) {
    const unsigned long long v = s_hist[i];
    if (v) atomicAdd(&my_hist[(i / B) * kBuckets + (i % B)], v);
  }
  n_elig = block_sum64(n_elig, s_tmp);
  n_bnd = block_sum64(n_bnd, s_tmp);
  n_cand = block_sum64(n_cand, s_tmp);
  n_apins = block_sum64(n_apins, s_tmp);
  if (threadIdx.x == 0) {
    const int sl = blockIdx.x % kSlots;
    RoundCounters* ctr = D.ctr;
    if (n_apins) atomicAdd(&ctr->slot[kCtrActivePins][sl], (unsigned long long)n_apins);
    if (n_elig) atomicAdd(&ctr->slot[kCtrEligible][sl], (unsigned long long)n_elig);
    if (n_bnd) atomicAdd(&ctr->slot[kCtrBoundary][sl], (unsigned long long)n_bnd);
    if (n_cand) atomicAdd(&ctr->slot[kCtrCandidates][sl], (unsigned long long)n_cand);
  }
}

// One wavefront per heavy vertex (w(I(u)) > 255): per-block connection
// weights in LDS (int32, enough because w(E) < 2^31), lanes stride over I(u).
// Unit: 4 consecutive entries of the heavy list (one per wavefront).
__global__ __launch_bounds__(kBlock) void k_select_heavy(Launch L) {
  __shared__ long long s_W[HG_MAX_K];
  __shared__ int s_conn[kBlock / kWave][HG_MAX_K];
  const WorkItem wi = work_item(L, single_unit(blockIdx.x));
  const InstDesc D = inst_desc(L, wi.inst);
  const int k = D.k;
  for (int i = threadIdx.x; i < k; i += kBlock) s_W[i] = D.block_w[i];
  __syncthreads();
  const int wv = threadIdx.x / kWave, lane = lane_id();
  const long long idx = (long long)wi.first * (kBlock / kWave) + wv;
  if (idx >= D.heavy_count) return;
  const int sl = (int)(idx % kSlots);
  unsigned long long* my_hist = D.hist + (size_t)(blockIdx.x % D.hist_reps) * D.hist_stride;
  RoundCounters* ctr = D.ctr;
  const int u = D.heavy_list[idx];
  const int a = D.part[u];
  const unsigned char el = D.eligible[u];
  if (!el || (unsigned)a >= (unsigned)k) {
    if (lane == 0) {
      D.cand[u] = -1;
      if (el) {
        atomicOr(D.err_flags, kErrPart);
        D.eligible[u] = 0;
      }
    }
    return;
  }
  int* conn = s_conn[wv];
  for (int i = lane; i < k; i += kWave) conn[i] = 0;
  wave_lds_sync();
  const long long b0 = D.vptr[u], b1 = D.vptr[u + 1];
  const int wk = bit_words(k);
  int tot = 0, ben = 0;
  bool bnd = false;
  for (long long j = b0 + lane; j < b1; j += kWave) {
    const int e = D.vnets[j];
    const unsigned* r = D.netstate + (long long)e * D.rw;
    const int w = (int)r[0];
    tot += w;
    bnd |= r[1] > 1u;
    if ((r[2 + wk + (a >> 5)] >> (a & 31)) & 1u) ben += w;
    for (int q = 0; q < wk; ++q) {
      unsigned x = r[2 + q];
      while (x) {
        int b = __ffs(x) - 1;
        x &= x - 1;
        atomicAdd(&conn[q * 32 + b], w);
      }
    }
  }
  wave_lds_sync();
  tot = wave_sum(tot);
  ben = wave_sum(ben);
  bnd = __any(bnd);
  const long long cu = D.vwgt ? D.vwgt[u] : 1;
  // best feasible neighbouring block on this lane's share of the blocks
  int bc = -1, bi = -1;
  long long bw = 0;
  for (int i = lane; i < k; i += kWave) {
    int ci = conn[i];
    if (i == a || ci <= 0 || s_W[i] + cu > D.lmax) continue;
    long long Wi = s_W[i];
    if (bi < 0 || ci > bc || (ci == bc && (Wi < bw || (Wi == bw && i < bi)))) {
      bc = ci;
      bi = i;
      bw = Wi;
    }
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    int oc = __shfl_xor(bc, o), oi = __shfl_xor(bi, o);
    long long ow = __shfl_xor(bw, o);
    bool take = oi >= 0 && (bi < 0 || oc > bc || (oc == bc && (ow < bw || (ow == bw && oi < bi))));
    if (take) {
      bc = oc;
      bi = oi;
      bw = ow;
    }
  }
  if (lane == 0) {
    D.eligible[u] = 0;
    atomicAdd(&ctr->slot[kCtrEligible][sl], 1ull);
    long long out = -1;
    if (bnd) {
      atomicAdd(&ctr->slot[kCtrBoundary][sl], 1ull);
      atomicAdd(&ctr->slot[kCtrActivePins][sl], (unsigned long long)(b1 - b0));
      if (bi >= 0) {
        const int g = ben - tot + bc;
        if (g > 0 || (g == 0 && bw + cu < s_W[a])) {
          out = pack_cand(g, bi);
          atomicAdd(&ctr->slot[kCtrCandidates][sl], 1ull);
          atomicAdd(&my_hist[bi * kBuckets + (g < kBuckets ? g : kBuckets - 1)],
                    (unsigned long long)cu);
          if (g > kBuckets - 1) atomicOr(&D.overflow[bi], 1);
        }
      }
    }
    D.cand[u] = out;
  }
}

// Select from a gain cache (subsection "Gain Caching"): the same decisions
// as k_select_light / k_select_heavy, read from b(u), w(I(u)) and the
// penalty row instead of the incident nets.  Block i neighbours u iff
// conn_i = w(I(u)) - p_i(u) > 0, and then g_i(u) = b(u) - w(I(u)) + conn_i.
// G lanes share a vertex, each reading 16-byte quads of its row, so one
// wavefront reads 64 / G consecutive rows.  Unit: a chunk of 256 vertices;
// every vertex, light or heavy, is handled here.
template <int G>
__global__ __launch_bounds__(kBlock) void k_select_cached(Launch L) {
  __shared__ long long s_W[HG_MAX_K];
  __shared__ unsigned long long s_hist[kLdsHistEntries];
  __shared__ long long s_tmp[kBlock / kWave];
  const InstDesc D0 = L.one;
  const WorkItem wi = work_item(L, xcd_sweep((D0.n + kBlock - 1) / kBlock));
  if (wi.count == 0) return;
  const InstDesc D = inst_desc(L, wi.inst);
  const int k = D.k, B = D.lds_buckets, n = D.n;
  const long long lmax = D.lmax;
  for (int i = threadIdx.x; i < k * B; i += kBlock) s_hist[i] = 0;
  for (int i = threadIdx.x; i < k; i += kBlock) s_W[i] = D.block_w[i];
  __syncthreads();
  unsigned long long* my_hist = D.hist + (size_t)(blockIdx.x % D.hist_reps) * D.hist_stride;
  long long n_elig = 0, n_bnd = 0, n_cand = 0, n_apins = 0;
  const int gl = threadIdx.x % G;
  constexpr int kPer = kBlock / G;
  const int Q = cache_stride(k) / 4;
  const int* __restrict__ cb = D.cache;
  const int4* __restrict__ rows = (const int4*)(D.cache + cache_pbase(n));
  for (int it = 0; it < wi.count; ++it) {
    const long long c = (long long)wi.first + (long long)it * wi.stride;
    for (int sub = 0; sub < G; ++sub) {
      // every lane of a group has the same u, so control flow below is
      // uniform within the group
      const long long u = c * kBlock + sub * kPer + threadIdx.x / G;
      if (u >= n) continue;
      if (gl == 0 && D.moved) D.moved[u] = 0;
      const unsigned char el = D.eligible[u];
      if (!el) {
        if (gl == 0) D.cand[u] = -1;
        continue;
      }
      const int a = D.part[u];
      if ((unsigned)a >= (unsigned)k) {
        if (gl == 0) {
          atomicOr(D.err_flags, kErrPart);
          D.cand[u] = -1;
          D.eligible[u] = 0;
        }
        continue;
      }
      const int ben = cb[u], tot = cb[n + u];
      const long long cu = D.vwgt ? D.vwgt[u] : 1;
      bool bnd = false;
      int bc = -1, bi = -1;
      long long bw = 0;
      for (int q = gl; q < Q; q += G) {
        const int4 p4 = rows[u * Q + q];
        const int pv[4] = {p4.x, p4.y, p4.z, p4.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = q * 4 + j;
          const int ci = tot - pv[j];
          if (i >= k || i == a || ci <= 0) continue;
          bnd = true;
          const long long Wi = s_W[i];
          if (Wi + cu > lmax) continue;
          if (bi < 0 || ci > bc || (ci == bc && Wi < bw)) {
            bc = ci;
            bi = i;
            bw = Wi;
          }
        }
      }
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) {
        const int oc = __shfl_xor(bc, o, G), oi = __shfl_xor(bi, o, G);
        const long long ow = __shfl_xor(bw, o, G);
        bnd |= __shfl_xor((int)bnd, o, G) != 0;
        const bool take =
            oi >= 0 && (bi < 0 || oc > bc || (oc == bc && (ow < bw || (ow == bw && oi < bi))));
        if (take) {
          bc = oc;
          bi = oi;
          bw = ow;
        }
      }
      if (gl != 0) continue;
      D.eligible[u] = 0;
      n_elig += 1;
      long long out = -1;
      if (bnd) {
        n_bnd += 1;
        n_apins += D.vptr[u + 1] - D.vptr[u];
        if (bi >= 0) {
          const int g = ben - tot + bc;
          if (g > 0 || (g == 0 && bw + cu < s_W[a])) {
            out = pack_cand(g, bi);
            n_cand += 1;
            if (g < B) {
              atomicAdd(&s_hist[bi * B + g], (unsigned long long)cu);
            } else {
              atomicAdd(&my_hist[bi * kBuckets + (g < kBuckets ? g : kBuckets - 1)],
                        (unsigned long long)cu);
              if (g > kBuckets - 1) atomicOr(&D.overflow[bi], 1);
            }
          }
        }
      }
      D.cand[u] = out;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k * B; i += kBlock) {
    const unsigned long long v = s_hist[i];
    if (v) atomicAdd(&my_hist[(i / B) * kBuckets + (i % B)], v);
  }
  n_elig = block_sum64(n_elig, s_tmp);
  n_bnd = block_sum64(n_bnd, s_tmp);
  n_cand = block_sum64(n_cand, s_tmp);
  n_apins = block_sum64(n_apins, s_tmp);
  if (threadIdx.x == 0) {
    const int sl = blockIdx.x % kSlots;
    RoundCounters* ctr = D.ctr;
    if (n_apins) atomicAdd(&ctr->slot[kCtrActivePins][sl], (unsigned long long)n_apins);
    if (n_elig) atomicAdd(&ctr->slot[kCtrEligible][sl], (unsigned long long)n_elig);
    if (n_bnd) atomicAdd(&ctr->slot[kCtrBoundary][sl], (unsigned long long)n_bnd);
    if (n_cand) atomicAdd(&ctr->slot[kCtrCandidates][sl], (unsigned long long)n_cand);
  }
}

// b(u) of every vertex that moved this round, from the finalized net records
// (the nets where u is the only pin of its new block).  Unit: one vertex.
__global__ __launch_bounds__(kBlock) void k_cache_movers(Launch L) {
  const InstDesc D = L.one;
  const long long u = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (u >= D.n || !D.moved[u]) return;
  const int a = D.part[u];
  const int wk = bit_words(D.k);
  const int sw = 2 + wk + (a >> 5);
  const unsigned bit = 1u << (a & 31);
  int ben = 0;
  for (long long j = D.vptr[u]; j < D.vptr[u + 1]; ++j) {
    const unsigned* r = D.netstate + (long long)D.vnets[j] * D.rw;
    if (r[sw] & bit) ben += (int)r[0];
  }
  D.cache[u] = ben;
}

int cached_group(int k) {
  const int q = cache_stride(k) / 4;
  int G = 1;
  while (G < q && G < kWave) G <<= 1;
  return G;
}

SelectKernel select_cached_kernel(int k) {
  switch (cached_group(k)) {
    case 1: return k_select_cached<1>;
    case 2: return k_select_cached<2>;
    case 4: return k_select_cached<4>;
    case 8: return k_select_cached<8>;
    case 16: return k_select_cached<16>;
    case 32: return k_select_cached<32>;
    default: return k_select_cached<64>;
  }
}

// A single-instance round that reads and updates the gain cache d.cache:
// cached select in place of the light and heavy sweeps, the finalize that
// applies the net deltas, and the movers' b before the round record.
void cached_round_plan(const InstDesc& d, RoundPlan& plan) {
  single_round_plan(d, plan);
  plan.select[0].kernel = (void*)select_cached_kernel(d.k);
  plan.heavy.clear();   // any_heavy stays: heavy vertices can still overflow the buckets
}

hipError_t launch_cached_round(const RoundPlan& plan, int round, hipStream_t s,
                               hipEvent_t* marks) {
  hipError_t e = launch_round_front(plan, s, marks);
  if (e == hipSuccess) e = launch_round_finalize(plan, s, marks);
  if (e != hipSuccess) return e;
  const InstDesc& d = plan.stats.L.one;
  hipLaunchKernelGGL(k_cache_movers, dim3((unsigned)((d.n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, plan.stats.L);
  return launch_round_stats(plan, round, s, marks);
}

// --------------------------------------------------------------- threshold

// Unit: one target block t.  Thread j looks at gain bucket 255 - j (summed
// over the XCD replicas, which it also clears for the next round).
__global__ __launch_bounds__(kBlock) void k_threshold(Launch L) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_first;
  const WorkItem wi = work_item(L, single_unit(blockIdx.x));
  const InstDesc D = inst_desc(L, wi.inst);
  const int t = wi.first;
  const int bucket = kBuckets - 1 - threadIdx.x;
  long long h = 0;
  unsigned long long* col = D.hist + (size_t)t * kBuckets + bucket;
  unsigned long long rv[kHistReplicas];
  // all replicas' cells requested before the stores that clear them
#pragma unroll
  for (int rep = 0; rep < kHistReplicas; ++rep)
    rv[rep] = rep < D.hist_reps ? col[(size_t)rep * D.hist_stride] : 0ull;
#pragma unroll
  for (int rep = 0; rep < kHistReplicas; ++rep) {
    h += (long long)rv[rep];
    if (rep < D.hist_reps) col[(size_t)rep * D.hist_stride] = 0;
  }
  const long long budget = D.lmax - D.block_w[t];
  if (threadIdx.x == 0) s_first = kBlock;
  long long total;
  const long long above = block_excl_scan64(h, s_tmp, &total);   // weight of higher gains
  if (h > 0 && above + h > budget) atomicMin(&s_first, (int)threadIdx.x);
  __syncthreads();
  const int f = s_first;
  if ((int)threadIdx.x == (f < kBlock ? f : 0)) {
    Threshold r;
    r.tau = 0;
    r.rem_tile = 0;
    if (f < kBlock) {
      r.gstar = bucket;
      r.rem = budget - above;
    } else {
      r.gstar = -1;
      r.rem = 0;
    }
    D.thr[t] = r;
    if (f < kBlock && bucket == kBuckets - 1 && D.overflow[t]) {
      atomicOr(&D.ctr->any_overflow, 1u);
    } else {
      D.overflow[t] = 0;
    }
  }
}

// Only for graphs with heavy vertices: the ">= 255" bucket of block t holds
// several gain values and its budget ran out inside it.  Find the exact
// threshold gain by bisection over all candidates (a slow but rare path).
// Unit: one target block.
__global__ __launch_bounds__(kBlock) void k_overflow_resolve(Launch L) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ long long s_max[kBlock / kWave];
  const WorkItem wi = work_item(L, single_unit(blockIdx.x));
  const InstDesc D = inst_desc(L, wi.inst);
  const int t = wi.first;
  if (!D.ctr->any_overflow) return;
  if (!D.overflow[t]) return;
  const long long rem = D.thr[t].rem;
  const int n = D.n;
  const long long* cand = D.cand;
  long long gmax = 0;
  for (long long u = threadIdx.x; u < n; u += kBlock) {
    long long x = cand[u];
    if (x >= 0 && cand_target(x) == t && cand_gain(x) > gmax) gmax = cand_gain(x);
  }
  {
    long long v = wave_max(gmax);
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = v;
    __syncthreads();
    gmax = 0;
    for (int i = 0; i < kBlock / kWave; ++i) gmax = s_max[i] > gmax ? s_max[i] : gmax;
    __syncthreads();
  }
  long long lo = kBuckets - 1, hi = gmax + 1, w_hi = 0;   // weight(>= lo) > rem >= weight(>= hi)
  while (hi - lo > 1) {
    long long mid = (lo + hi) / 2;
    long long s = 0;
    for (long long u = threadIdx.x; u < n; u += kBlock) {
      long long x = cand[u];
      if (x >= 0 && cand_target(x) == t && cand_gain(x) >= mid) s += D.vwgt ? D.vwgt[u] : 1;
    }
    s = block_sum64(s, s_tmp);
    if (s > rem) {
      lo = mid;
    } else {
      hi = mid;
      w_hi = s;
    }
  }
  if (threadIdx.x == 0) {
    D.thr[t].gstar = (int)lo;
    D.thr[t].rem = rem - w_hi;
    D.overflow[t] = 0;
  }
}

// --------------------------------------------------------------- tiles

// Unit: one tile of kTile vertices.
__global__ __launch_bounds__(kBlock) void k_tilesum(Launch L) {
  __shared__ unsigned long long s_sum[HG_MAX_K];
  __shared__ int s_g[HG_MAX_K];
  const WorkItem wi = work_item(L, single_unit(blockIdx.x));
  const InstDesc D = inst_desc(L, wi.inst);
  const int k = D.k;
  for (int i = threadIdx.x; i < k; i += kBlock) {
    s_sum[i] = 0;
    s_g[i] = D.thr[i].gstar;
  }
  __syncthreads();
  const int tile = wi.first;
  const long long base = (long long)tile * kTile;
  // every candidate word and weight of this thread requested before the first wait
  long long x[kPerThreadTile];
  int cw[kPerThreadTile];
#pragma unroll
  for (int j = 0; j < kPerThreadTile; ++j) {
    const long long u = base + (long long)j * kBlock + threadIdx.x;
    x[j] = u < D.n ? D.cand[u] : -1;
    cw[j] = u < D.n && D.vwgt ? D.vwgt[u] : 1;
  }
#pragma unroll
  for (int j = 0; j < kPerThreadTile; ++j) {
    if (x[j] >= 0) {
      const int t = cand_target(x[j]);
      if (cand_gain(x[j]) == s_g[t]) atomicAdd(&s_sum[t], (unsigned long long)cw[j]);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock)
    D.tilesum[(long long)i * D.num_tiles + tile] = (long long)s_sum[i];
}

// Unit: one target block.  Thread i takes kScanPerThread consecutive tiles
// of each span of kBlock * kScanPerThread tiles (one span covers 2048 tiles,
// about a million vertices): one workgroup scan per span.
constexpr int kScanPerThread = 8;

__global__ __launch_bounds__(kBlock) void k_tilescan(Launch L) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_tau;
  __shared__ long long s_remt;
  const WorkItem wi = work_item(L, single_unit(blockIdx.x));
  const InstDesc D = inst_desc(L, wi.inst);
  const int t = wi.first;
  const int num_tiles = D.num_tiles;
  const Threshold r = D.thr[t];
  if (r.gstar < 0) {
    if (threadIdx.x == 0) D.thr[t].tau = num_tiles;
    return;
  }
  if (threadIdx.x == 0) {
    s_tau = num_tiles;
    s_remt = 0;
  }
  const long long* row = D.tilesum + (long long)t * num_tiles;
  long long carry = 0;
  for (int base = 0; base < num_tiles; base += kBlock * kScanPerThread) {
    const int first = base + threadIdx.x * kScanPerThread;
    long long v[kScanPerThread];
    long long mine = 0;
#pragma unroll
    for (int q = 0; q < kScanPerThread; ++q) {
      v[q] = first + q < num_tiles ? row[first + q] : 0;
      mine += v[q];
    }
    long long tot;
    long long run = carry + block_excl_scan64(mine, s_tmp, &tot);
    // this thread's first tile whose gain-g* weight overflows the budget,
    // and the weight before it
    int hit = -1;
    long long hit_before = 0;
#pragma unroll
    for (int q = 0; q < kScanPerThread; ++q) {
      if (hit < 0 && v[q] > 0 && run + v[q] > r.rem) {
        hit = first + q;
        hit_before = run;
      }
      run += v[q];
    }
    if (hit >= 0) atomicMin(&s_tau, hit);
    __syncthreads();
    const int f = s_tau;
    if (f < num_tiles) {
      if (hit == f) s_remt = r.rem - hit_before;   // budget left at tile f's start
      break;
    }
    carry += tot;
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    D.thr[t].tau = s_tau;
    D.thr[t].rem_tile = s_remt;
  }
}

// --------------------------------------------------------------- approve + apply

// Apply the moves held in s_list[0..count) (vertex ids; targets in s_tgt):
// part, moved flags and block-weight deltas per mover, then the movers'
// incident nets as one flattened range split over all 256 threads (so a tile
// with few movers still keeps four wavefronts busy, and a high-degree mover is
// spread over the workgroup).  Phi is updated with integer atomics whose old
// values give the attributed km1 change; every incident net gets its touched
// flag (a plain byte store: all writers store the same value).
// The mover owning flattened incidence j: the largest i < count with
// s_off[i] <= j.
__device__ __forceinline__ int list_owner(const int* s_off, int count, long long j) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_off[mid] <= j) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ void apply_list(const InstDesc& D, const int* s_list, const int* s_tgt, int count,
                           int* s_from, long long* s_beg, int* s_off, long long* s_tmp,
                           unsigned long long* s_dW, long long& delta, long long& moved_pins,
                           long long& approved) {
  // per mover: move it, record where its incident nets start
  long long my_len = 0;
  int lens[kPerThreadTile];
  const int first = threadIdx.x * kPerThreadTile;   // entries [first, first + kPerThreadTile)
#pragma unroll
  for (int q = 0; q < kPerThreadTile; ++q) {
    const int i = first + q;
    lens[q] = 0;
    if (i < count) {
      const int u = s_list[i], t = s_tgt[i];
      const int a = D.part[u];
      const long long b = D.vptr[u];
      const int len = (int)(D.vptr[u + 1] - b);
      const long long cu = D.vwgt ? D.vwgt[u] : 1;
      D.part[u] = t;
      if (D.moved) D.moved[u] = 1;
      atomicAdd(&s_dW[t], (unsigned long long)cu);
      atomicAdd(&s_dW[a], (unsigned long long)(-cu));
      s_from[i] = a;
      s_beg[i] = b;
      lens[q] = len;
      my_len += len;
      moved_pins += len;
      approved += 1;
    }
  }
  long long total;
  long long off = block_excl_scan64(my_len, s_tmp, &total);
#pragma unroll
  for (int q = 0; q < kPerThreadTile; ++q) {
    if (first + q < count) s_off[first + q] = (int)off;
    off += lens[q];
  }
  __syncthreads();
  const int k = D.k;
  for (long long j = threadIdx.x; j < total; j += kBlock) {
    const int lo = list_owner(s_off, count, j);
    const int e = D.vnets[s_beg[lo] + (j - s_off[lo])];
    const int ao = s_from[lo], to = s_tgt[lo];
    const int oa = atomicSub(&D.phi[(long long)e * k + ao], 1);
    const int ot = atomicAdd(&D.phi[(long long)e * k + to], 1);
    if (oa == 1 || ot == 0) {
      const int w = D.unit_nets ? 1 : (int)D.netstate[(long long)e * D.rw];
      if (oa == 1) delta += w;    // Phi(e, a) drops to zero
      if (ot == 0) delta -= w;    // Phi(e, t) rises from zero
    }
    D.touched[e] = 1;
  }
}

// Monotone rounds: mark the approved moves, and set the cells (e, source) and
// (e, target) of their incident nets empty for the exact-gain kernels that
// follow (out_max 0, in_min "none", out_cnt 0); the incidences are spread
// over the workgroup as in apply_list.
__device__ void mark_list(const InstDesc& D, const int* s_list, const int* s_tgt, int count,
                          int* s_from, long long* s_beg, int* s_off, long long* s_tmp) {
  long long my_len = 0;
  int lens[kPerThreadTile];
  const int first = threadIdx.x * kPerThreadTile;
#pragma unroll
  for (int q = 0; q < kPerThreadTile; ++q) {
    const int i = first + q;
    lens[q] = 0;
    if (i < count) {
      const int u = s_list[i];
      const long long b = D.vptr[u];
      D.appr[u] = 1;
      s_from[i] = D.part[u];
      s_beg[i] = b;
      lens[q] = (int)(D.vptr[u + 1] - b);
      my_len += lens[q];
    }
  }
  long long total;
  long long off = block_excl_scan64(my_len, s_tmp, &total);
#pragma unroll
  for (int q = 0; q < kPerThreadTile; ++q) {
    if (first + q < count) s_off[first + q] = (int)off;
    off += lens[q];
  }
  __syncthreads();
  const int k = D.k;
  const int4 empty = make_int4(0, 0x7fffffff, 0, 0);
  for (long long j = threadIdx.x; j < total; j += kBlock) {
    const int lo = list_owner(s_off, count, j);
    const long long e = D.vnets[s_beg[lo] + (j - s_off[lo])];
    D.seq_cell[e * k + s_from[lo]] = empty;
    D.seq_cell[e * k + s_tgt[lo]] = empty;
  }
}

// Unit: a tile of kTile vertices (count = 1), or -- boundary workgroups --
// the tile of target block `first` where its budget runs out (count = -1).
// Single instance: workgroups [0, num_tiles) are tiles (XCD-remapped), the
// k after them the boundary workgroups.
__global__ __launch_bounds__(kBlock) void k_approve_apply(Launch L) {
  __shared__ int s_list[kTile];
  __shared__ int s_tgt[kTile];
  __shared__ int s_from[kTile];
  __shared__ int s_off[kTile];
  __shared__ long long s_beg[kTile];
  __shared__ int s_g[HG_MAX_K];
  __shared__ int s_tau[HG_MAX_K];
  __shared__ unsigned long long s_dW[HG_MAX_K];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ unsigned s_count;
  WorkItem fb;
  {
    const int nt = L.one.num_tiles;
    fb = (int)blockIdx.x < nt ? single_unit((int)xcd_remap(blockIdx.x, nt))
                              : single_unit((int)blockIdx.x - nt);
    if ((int)blockIdx.x >= nt) fb.count = -1;
  }
  const WorkItem wi = work_item(L, fb);
  const InstDesc D = inst_desc(L, wi.inst);
  const int k = D.k, n = D.n, num_tiles = D.num_tiles;
  for (int i = threadIdx.x; i < k; i += kBlock) {
    s_g[i] = D.thr[i].gstar;
    s_tau[i] = D.thr[i].tau;
    s_dW[i] = 0;
  }
  if (threadIdx.x == 0) s_count = 0;
  __syncthreads();
  const long long* __restrict__ cand = D.cand;
  if (wi.count >= 0) {
    const int tile = wi.first;
    const long long base = (long long)tile * kTile;
    long long xs[kPerThreadTile];   // requested before the first wait
#pragma unroll
    for (int j = 0; j < kPerThreadTile; ++j) {
      const long long u = base + (long long)j * kBlock + threadIdx.x;
      xs[j] = u < n ? cand[u] : -1;
    }
#pragma unroll
    for (int j = 0; j < kPerThreadTile; ++j) {
      const long long u = base + (long long)j * kBlock + threadIdx.x;
      bool ok = false;
      int t = 0;
      const long long x = xs[j];
      if (x >= 0) {
        t = cand_target(x);
        const int g = cand_gain(x), gs = s_g[t];
        ok = g > gs || (g == gs && tile < s_tau[t]);
      }
      const int slot = wave_append(&s_count, ok);   // LDS counter, one atomic per wave
      if (ok) {
        s_list[slot] = (int)u;
        s_tgt[slot] = t;
      }
    }
  } else {
    // the tile where block t's budget runs out: prefix sums in vertex order
    const int t = wi.first;
    const Threshold r = D.thr[t];
    if (r.gstar < 0 || r.tau >= num_tiles) return;   // whole workgroup leaves together
    const long long base = (long long)r.tau * kTile + (long long)threadIdx.x * kPerThreadTile;
    long long mine = 0;
    for (int j = 0; j < kPerThreadTile; ++j) {
      const long long u = base + j;
      if (u < n) {
        const long long x = cand[u];
        if (x >= 0 && cand_target(x) == t && cand_gain(x) == r.gstar)
          mine += D.vwgt ? D.vwgt[u] : 1;
      }
    }
    long long tot;
    long long run = block_excl_scan64(mine, s_tmp, &tot);
    for (int j = 0; j < kPerThreadTile; ++j) {
      const long long u = base + j;
      bool ok = false;
      if (u < n) {
        const long long x = cand[u];
        if (x >= 0 && cand_target(x) == t && cand_gain(x) == r.gstar) {
          const long long cu = D.vwgt ? D.vwgt[u] : 1;
          ok = run + cu <= r.rem_tile;
          run += cu;
        }
      }
      const int slot = wave_append(&s_count, ok);
      if (ok) {
        s_list[slot] = (int)u;
        s_tgt[slot] = t;
      }
    }
  }
  __syncthreads();
  const int count = (int)s_count;
  long long delta = 0, moved_pins = 0, approved = 0;
  if (count > 0 && D.appr) {
    // monotone round: only mark; the moves are ordered, re-gained and cut later
    mark_list(D, s_list, s_tgt, count, s_from, s_beg, s_off, s_tmp);
    if (threadIdx.x == 0)
      atomicAdd(&D.ctr->slot[kCtrMarked][blockIdx.x % kSlots], (unsigned long long)count);
  } else if (count > 0) {
    apply_list(D, s_list, s_tgt, count, s_from, s_beg, s_off, s_tmp, s_dW, delta, moved_pins,
               approved);
  }
  __syncthreads();
  // block-weight deltas go to one of kSlots partial rows (a single row
  // would serialize one atomic per tile on each of the k addresses); the
  // round record folds them into block_w
  long long* my_dw = D.bw_slots + (size_t)(blockIdx.x % kSlots) * k;
  for (int i = threadIdx.x; i < k; i += kBlock)
    if (s_dW[i]) atomicAdd((unsigned long long*)&my_dw[i], s_dW[i]);
  delta = block_sum64(delta, s_tmp);
  moved_pins = block_sum64(moved_pins, s_tmp);
  approved = block_sum64(approved, s_tmp);
  if (threadIdx.x == 0) {
    const int sl = blockIdx.x % kSlots;
    RoundCounters* ctr = D.ctr;
    if (delta) atomicAdd(&ctr->slot[kCtrDeltaAttr][sl], (unsigned long long)delta);
    if (moved_pins) atomicAdd(&ctr->slot[kCtrMovedPins][sl], (unsigned long long)moved_pins);
    if (approved) atomicAdd(&ctr->slot[kCtrApproved][sl], (unsigned long long)approved);
  }
}

// --------------------------------------------------------------- finalize

// Unit: a chunk of kFinalChunk nets.  The workgroup reads their touched
// flags (coalesced), lists the touched ones in LDS and hands them to groups
// of G lanes: Lambda, S and lambda are rebuilt from the final Phi row, the
// flag is cleared and every pin becomes eligible.  The lane that rewrites
// lambda(e) reads the old value first, so the drop (lambda_old - lambda_new)
// * w(e) summed over touched nets checks the attributed total.  Single
// instance: contiguous XCD-aware runs of chunks.
// Gain cache update of one touched net e (subsection "Gain Caching"): the
// four update rules, summed over all moves of the round, change p_i(v) for
// every pin v by +w(e) when block i lost its last pin of e and by -w(e)
// when it gained its first, and b(v) of a pin that did not move (block c)
// by +w(e) when c now holds exactly one pin of e and by -w(e) when it no
// longer does.  Moved vertices get b recomputed after the round.  Every lane
// of the group calls this with its record word before (old_w) and after
// (new_w) the round; the pins are also made eligible.
template <int G>
__device__ void cache_net_delta(const InstDesc& D, long long e, int wk, int gl, unsigned old_w,
                                unsigned new_w, long long b, long long t) {
  const int base = lane_id() - gl;
  unsigned lo[8], ln[8], so[8], sn[8];
#pragma unroll
  for (int x = 0; x < 8; ++x) {
    const int lam = 2 + (x < wk ? x : 0), sgl = 2 + wk + (x < wk ? x : 0);
    lo[x] = __shfl(old_w, base + lam);
    ln[x] = __shfl(new_w, base + lam);
    so[x] = __shfl(old_w, base + sgl);
    sn[x] = __shfl(new_w, base + sgl);
  }
  const int w = D.ewgt ? D.ewgt[e] : 1;
  const int ks = cache_stride(D.k);
  int* cb = D.cache;
  int* cp = D.cache + cache_pbase(D.n);
  unsigned dl = 0, ds = 0;
#pragma unroll
  for (int x = 0; x < 8; ++x) {
    dl |= lo[x] ^ ln[x];
    ds |= so[x] ^ sn[x];
  }
  for (long long p = b + gl; p < t; p += G) {
    const int v = D.pins[p];
    D.eligible[v] = 1;
    if (dl) {
#pragma unroll
      for (int x = 0; x < 8; ++x) {
        if (x >= wk) break;
        unsigned d = lo[x] ^ ln[x];
        while (d) {
          const int bit = __ffs(d) - 1;
          d &= d - 1;
          atomicAdd(&cp[(long long)v * ks + x * 32 + bit], ((lo[x] >> bit) & 1u) ? w : -w);
        }
      }
    }
    if (ds && !D.moved[v]) {
      const int c = D.part[v];
      unsigned dso = 0, dsn = 0;
#pragma unroll
      for (int x = 0; x < 8; ++x)
        if (x == (c >> 5)) {
          dso = so[x];
          dsn = sn[x];
        }
      const int bit = c & 31;
      if (((dso ^ dsn) >> bit) & 1u) atomicAdd(&cb[v], ((dsn >> bit) & 1u) ? w : -w);
    }
  }
}

// Gain-cache rounds: the same record rebuild, with the cache deltas of each
// touched net applied by its group while it walks the net's pins (and marks
// them eligible).  Unit: a chunk of kCachedChunk nets, one touched flag per
// thread; many small units keep the atomics-heavy pin walks spread over
// the whole GPU.
constexpr int kCachedChunk = kBlock;
constexpr int kCachedGrid = 16384;   // persistent workgroups of the cached finalize

template <int G>
__global__ __launch_bounds__(kBlock) void k_finalize_cached(Launch L) {
  __shared__ int s_list[kCachedChunk];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ unsigned s_cnt;
  constexpr int kGroups = kBlock / G;
  const WorkItem wi = work_item(L, xcd_block((L.one.m + kCachedChunk - 1) / kCachedChunk));
  if (wi.count == 0) return;
  const InstDesc D = inst_desc(L, wi.inst);
  const int grp = threadIdx.x / G, gl = threadIdx.x % G;
  const int k = D.k, wk = bit_words(k), rw = D.rw;
  long long dcheck = 0, ntouched = 0, tpins = 0;
  for (int it = 0; it < wi.count; ++it) {
    const long long c = (long long)wi.first + (long long)it * wi.stride;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    // one flag per thread (the flag array is padded to whole chunks, zero past m)
    const long long e0 = c * kCachedChunk + threadIdx.x;
    const bool t0 = D.touched[e0] != 0;
    const int slot = wave_append(&s_cnt, t0);
    if (t0) s_list[slot] = (int)e0;
    __syncthreads();
    const int cnt = (int)s_cnt;
    ntouched += cnt;
    for (int i = grp; i < cnt; i += kGroups) {
      const int e = s_list[i];
      const int* row = D.phi + (long long)e * k;
      unsigned* rec = D.netstate + (long long)e * rw;
      int lam_old = 0, w = 0;
      if (gl == 1) {
        lam_old = (int)rec[1];
        w = (int)rec[0];
      }
      // the record's Lambda / S words before this round
      const unsigned old_word = gl >= 2 && gl < 2 + 2 * wk ? rec[gl] : 0u;
      NetBits nb = net_bits<G>(k, gl, [&](int i2) { return row[i2]; });
      if (gl >= 1 && gl < 2 + 2 * wk) rec[gl] = nb.word;
      if (D.view != kViewFull) write_view(D.view_ptr, e, D.view, gl, nb);
      if (gl == 1) dcheck += (long long)(lam_old - nb.lambda) * w;
      const long long b = D.eptr[e], t = D.eptr[e + 1];
      if (gl == 0) {
        D.touched[e] = 0;
        tpins += t - b;
      }
      cache_net_delta<G>(D, e, wk, gl, old_word, nb.word, b, t);
    }
    __syncthreads();
  }
  dcheck = block_sum64(dcheck, s_tmp);
  tpins = block_sum64(tpins, s_tmp);
  if (threadIdx.x == 0) {
    const int sl = blockIdx.x % kSlots;
    if (dcheck) atomicAdd(&D.ctr->slot[kCtrDeltaCheck][sl], (unsigned long long)dcheck);
    if (ntouched) atomicAdd(&D.ctr->slot[kCtrTouched][sl], (unsigned long long)ntouched);
    if (tpins) atomicAdd(&D.ctr->slot[kCtrTouchedPins][sl], (unsigned long long)tpins);
  }
}

// Unit: a block of kFinalChunk (1024) nets.  Every thread reads four touched
// flags with one load; the touched nets of the block are listed in LDS.
// Groups of G lanes then rebuild each listed net's Lambda, S and lambda from
// its final Phi row and clear its flag; the lane that rewrites lambda(e)
// reads the old value first, so the drop (lambda_old - lambda_new) * w(e)
// summed over touched nets checks the attributed total.  Last, the pins of
// all listed nets are made eligible as one flattened list spread over the
// whole workgroup (offsets by a prefix sum, owner by binary search), so a
// long net does not serialize on one group.  With the gain cache the group
// walks its net's pins itself (cache_net_delta marks them too).  Single
// instance: contiguous XCD-aware runs of blocks.
constexpr int kMarkSlots = 4;   // pin positions per thread in flight in the marks

template <int G>
__global__ __launch_bounds__(kBlock) void k_finalize(Launch L) {
  __shared__ int s_list[kFinalChunk];
  __shared__ int s_off[kFinalChunk];        // first flattened pin position of each listed net
  __shared__ int s_beg[kFinalChunk];        // eptr of each listed net (P < 2^31)
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ unsigned s_cnt;
  constexpr int kGroups = kBlock / G;
  constexpr int kFlags = kFinalChunk / kBlock;   // 4
  const WorkItem wi = work_item(L, xcd_block((L.one.m + kFinalChunk - 1) / kFinalChunk));
  if (wi.count == 0) return;
  const InstDesc D = inst_desc(L, wi.inst);
  const int grp = threadIdx.x / G, gl = threadIdx.x % G;
  const int k = D.k, wk = bit_words(k), rw = D.rw;
  long long dcheck = 0, ntouched = 0, tpins = 0;
  // four flags per thread in one load (the flag array is padded to whole
  // blocks and zero past m; the workspace keeps it 4-byte aligned); the next
  // block's flags are loaded while this block is finalized
  unsigned next_f4 = *reinterpret_cast<const unsigned*>(
      D.touched + (long long)wi.first * kFinalChunk + (long long)threadIdx.x * kFlags);
  for (int it = 0; it < wi.count; ++it) {
    const long long c = (long long)wi.first + (long long)it * wi.stride;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const long long e0 = c * kFinalChunk + (long long)threadIdx.x * kFlags;
    const unsigned f4 = next_f4;
    if (it + 1 < wi.count)
      next_f4 = *reinterpret_cast<const unsigned*>(D.touched + e0 + (long long)wi.stride * kFinalChunk);
    int mine = 0;
#pragma unroll
    for (int q = 0; q < kFlags; ++q) mine += ((f4 >> (8 * q)) & 0xffu) != 0;
    const int incl = wave_incl_scan(mine);
    int base = 0;
    if (lane_id() == kWave - 1 && incl) base = (int)atomicAdd(&s_cnt, (unsigned)incl);
    base = __shfl(base, kWave - 1) + incl - mine;
#pragma unroll
    for (int q = 0; q < kFlags; ++q)
      if ((f4 >> (8 * q)) & 0xffu) s_list[base++] = (int)(e0 + q);
    __syncthreads();
    const int cnt = (int)s_cnt;
    ntouched += cnt;
    for (int i = grp; i < cnt; i += kGroups) {
      const int e = s_list[i];
      const int* row = D.phi + (long long)e * k;
      unsigned* rec = D.netstate + (long long)e * rw;
      int lam_old = 0, w = 0;
      if (gl == 1) {
        lam_old = (int)rec[1];
        w = (int)rec[0];
      }
      const long long b = D.eptr[e], t = D.eptr[e + 1];
      NetBits nb = net_bits<G>(k, gl, [&](int i2) { return row[i2]; });
      if (gl >= 1 && gl < 2 + 2 * wk) rec[gl] = nb.word;
      if (D.view != kViewFull) write_view(D.view_ptr, e, D.view, gl, nb);
      if (gl == 1) dcheck += (long long)(lam_old - nb.lambda) * w;
      if (gl == 0) {
        D.touched[e] = 0;
        tpins += t - b;
        s_beg[i] = (int)b;
        s_off[i] = (int)(t - b);          // the length, until the scan below
      }
    }
    {
      __syncthreads();
      // flattened pin positions: exclusive prefix of the lengths (four list
      // entries per thread)
      int len[kFlags];
      long long sum = 0;
#pragma unroll
      for (int q = 0; q < kFlags; ++q) {
        const int i = threadIdx.x * kFlags + q;
        len[q] = i < cnt ? s_off[i] : 0;
        sum += len[q];
      }
      long long total64;
      long long off = block_excl_scan64(sum, s_tmp, &total64);
#pragma unroll
      for (int q = 0; q < kFlags; ++q) {
        const int i = threadIdx.x * kFlags + q;
        if (i < cnt) s_off[i] = (int)off;
        off += len[q];
      }
      __syncthreads();
      const int total = (int)total64;     // at most P < 2^31
      for (int j0 = threadIdx.x; j0 < total; j0 += kBlock * kMarkSlots) {
        int at[kMarkSlots];
#pragma unroll
        for (int q = 0; q < kMarkSlots; ++q) {
          const int j = j0 + q * kBlock < total ? j0 + q * kBlock : j0;
          // owner: the last listed net whose first position is <= j
          int lo = 0, hi = cnt - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= j) lo = mid; else hi = mid - 1;
          }
          at[q] = s_beg[lo] + (j - s_off[lo]);
        }
        int v[kMarkSlots];
#pragma unroll
        for (int q = 0; q < kMarkSlots; ++q) v[q] = D.pins[at[q]];
#pragma unroll
        for (int q = 0; q < kMarkSlots; ++q)
          if (j0 + q * kBlock < total) D.eligible[v[q]] = 1;
      }
    }
    __syncthreads();
  }
  dcheck = block_sum64(dcheck, s_tmp);
  tpins = block_sum64(tpins, s_tmp);
  if (threadIdx.x == 0) {
    const int sl = blockIdx.x % kSlots;
    if (dcheck) atomicAdd(&D.ctr->slot[kCtrDeltaCheck][sl], (unsigned long long)dcheck);
    if (ntouched) atomicAdd(&D.ctr->slot[kCtrTouched][sl], (unsigned long long)ntouched);
    if (tpins) atomicAdd(&D.ctr->slot[kCtrTouchedPins][sl], (unsigned long long)tpins);
  }
}

// Unit: one instance.  Fold the apply's block-weight slots into block_w, sum
// the counter slots, write the round record, move km1 by the attributed drop,
// reset the slots and counters for the next round.
__global__ __launch_bounds__(kBlock) void k_round_stats(Launch L) {
  __shared__ long long s_sum[kNumCounters];
  __shared__ long long s_max[kBlock / kWave];
  const WorkItem wi = work_item(L, single_unit(0));
  const InstDesc D = inst_desc(L, wi.inst);
  RoundCounters* ctr = D.ctr;
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  // loads of the counter rows, and of the slot cells 16 at a time, are
  // issued before the stores that clear them (not one round trip per cell)
  constexpr int kRows = (kNumCounters + kBlock / kWave - 1) / (kBlock / kWave);
  unsigned long long v[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int c = wv + r * (kBlock / kWave);
    v[r] = c < kNumCounters ? ctr->slot[c][lane] : 0ull;
  }
  long long mx = LLONG_MIN;
  for (int i = threadIdx.x; i < D.k; i += kBlock) {
    long long* col = D.bw_slots + i;
    const size_t ks = (size_t)D.k;
    long long d = D.block_w[i];
    for (int s0 = 0; s0 < kSlots; s0 += 16) {      // 16 loads in flight, then the clears
      long long cells[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) cells[q] = col[(s0 + q) * ks];
#pragma unroll
      for (int q = 0; q < 16; ++q) d += cells[q];
#pragma unroll
      for (int q = 0; q < 16; ++q) col[(s0 + q) * ks] = 0;
    }
    D.block_w[i] = d;
    mx = d > mx ? d : mx;
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int c = wv + r * (kBlock / kWave);
    if (c < kNumCounters) {
      const long long sum = wave_sum((long long)v[r]);
      if (lane == 0) s_sum[c] = sum;
      ctr->slot[c][lane] = 0;
    }
  }
  mx = wave_max(mx);
  if (lane == 0) s_max[wv] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long m = s_max[0];
    for (int i = 1; i < kBlock / kWave; ++i) m = s_max[i] > m ? s_max[i] : m;
    hg_round_stats st;
    st.eligible = s_sum[kCtrEligible];
    st.boundary = s_sum[kCtrBoundary];
    st.candidates = s_sum[kCtrCandidates];
    st.approved = s_sum[kCtrApproved];
    st.moved_pins = s_sum[kCtrMovedPins];
    st.touched_nets = s_sum[kCtrTouched];
    st.km1_delta = s_sum[kCtrDeltaAttr];
    st.km1_delta_recomputed = s_sum[kCtrDeltaCheck];
    st.active_pins = s_sum[kCtrActivePins];
    st.touched_pins = s_sum[kCtrTouchedPins];
    st.km1_after = *D.km1 - st.km1_delta;
    st.max_block_weight = m;
    *D.km1 = st.km1_after;
    D.stats[L.round - D.round_base] = st;
    ctr->any_overflow = 0;
  }
}

// --------------------------------------------------------------- launch

int group_lanes(int k);

// Kernel selection per instance shape (shared with the batch planner).
// Record gathers in flight per vertex: eight where the average degree is
// 12 or more (half the dependent load steps for the typical vertex), four
// below (eight would mostly load padding slots).
template <int U>
SelectKernel select_kernel_u(int k, int view) {
  switch (view) {
    case kView16: return k_select_light<1, kView16, U>;
    case kView32: return k_select_light<1, kView32, U>;
    case kView64: return k_select_light<2, kView64, U>;
    default: break;
  }
  switch (bit_words(k)) {
    case 1: return k_select_light<1, kViewFull, U>;
    case 2: return k_select_light<2, kViewFull, U>;
    case 4: return k_select_light<4, kViewFull, U>;
    default: return k_select_light<8, kViewFull, U>;
  }
}

SelectKernel select_kernel(int k, int view, long long P, int n) {
  return P >= 12LL * n ? select_kernel_u<8>(k, view) : select_kernel_u<4>(k, view);
}

// The plain finalize reads one Phi row and writes one record per net: for
// k <= 16 four lanes hold the record and the row's counts, and narrower
// groups put twice as many nets in flight per wave (its pins are marked by
// the whole workgroup).  The cache variant walks the pins in the group.
FinalizeKernel finalize_kernel(int k, bool cache) {
  return finalize_kernel_g(!cache && k <= 16 ? 4 : group_lanes(k), cache);
}

// The gain-cache update lives in its own instantiation: the plain one then
// needs far fewer registers (more workgroups per compute unit).
FinalizeKernel finalize_kernel_g(int G, bool cache) {
  switch (G) {
    case 4: return cache ? k_finalize_cached<4> : k_finalize<4>;
    case 8: return cache ? k_finalize_cached<8> : k_finalize<8>;
    case 16: return cache ? k_finalize_cached<16> : k_finalize<16>;
    default: return cache ? k_finalize_cached<32> : k_finalize<32>;
  }
}

// Launch one round of every kernel for a batch (items per kernel kind) or a
// single instance (L.descs == nullptr).
hipError_t launch_round(const RoundPlan& plan, int round, hipStream_t s, hipEvent_t* marks) {
  hipError_t e = launch_round_front(plan, s, marks);
  if (e != hipSuccess) return e;
  return launch_round_back(plan, round, s, marks);
}

// Select, thresholds, tiles and approve (+ apply unless the descriptor asks
// for marks only).
hipError_t launch_round_front(const RoundPlan& plan, hipStream_t s, hipEvent_t* marks) {
  // a null start mark: the previous round's end mark starts this round
  if (marks && marks[0]) (void)hipEventRecord(marks[0], s);
  for (const PlanLaunch& pl : plan.select)
    hipLaunchKernelGGL((SelectKernel)pl.kernel, dim3(pl.grid), dim3(kBlock), 0, s, pl.L);
  for (const PlanLaunch& pl : plan.heavy)
    hipLaunchKernelGGL(k_select_heavy, dim3(pl.grid), dim3(kBlock), 0, s, pl.L);
  if (marks) (void)hipEventRecord(marks[1], s);
  hipLaunchKernelGGL(k_threshold, dim3(plan.blocks.grid), dim3(kBlock), 0, s, plan.blocks.L);
  if (plan.any_heavy)
    hipLaunchKernelGGL(k_overflow_resolve, dim3(plan.blocks.grid), dim3(kBlock), 0, s,
                       plan.blocks.L);
  hipLaunchKernelGGL(k_tilesum, dim3(plan.tiles.grid), dim3(kBlock), 0, s, plan.tiles.L);
  hipLaunchKernelGGL(k_tilescan, dim3(plan.blocks.grid), dim3(kBlock), 0, s, plan.blocks.L);
  hipLaunchKernelGGL(k_approve_apply, dim3(plan.approve.grid), dim3(kBlock), 0, s,
                     plan.approve.L);
  return hipGetLastError();
}

// Finalize (touched nets, next eligible set) and the round record.
hipError_t launch_round_back(const RoundPlan& plan, int round, hipStream_t s, hipEvent_t* marks) {
  hipError_t e = launch_round_finalize(plan, s, marks);
  if (e != hipSuccess) return e;
  return launch_round_stats(plan, round, s, marks);
}

hipError_t launch_round_finalize(const RoundPlan& plan, hipStream_t s, hipEvent_t* marks) {
  if (marks) (void)hipEventRecord(marks[2], s);
  for (const PlanLaunch& pl : plan.finalize)
    hipLaunchKernelGGL((FinalizeKernel)pl.kernel, dim3(pl.grid), dim3(kBlock), 0, s, pl.L);
  return hipGetLastError();
}

hipError_t launch_round_stats(const RoundPlan& plan, int round, hipStream_t s, hipEvent_t* marks) {
  Launch ls = plan.stats.L;
  ls.round = round;
  hipLaunchKernelGGL(k_round_stats, dim3(plan.stats.grid), dim3(kBlock), 0, s, ls);
  if (marks) (void)hipEventRecord(marks[3], s);
  return hipGetLastError();
}

// Plan for one instance (no work tables; kernels derive units from blockIdx).
void single_round_plan(const InstDesc& d, RoundPlan& plan) {
  plan = RoundPlan();
  const Launch L = single_launch(d);
  const long long chunks = ((long long)d.n + kBlock - 1) / kBlock;
  PlanLaunch sel;
  sel.kernel = (void*)select_kernel(d.k, d.view, d.P, d.n);
  sel.grid = (unsigned)(chunks < kSelectGrid ? chunks : kSelectGrid);
  sel.L = L;
  plan.select.push_back(sel);
  if (d.heavy_count > 0) {
    PlanLaunch hv;
    hv.grid = (unsigned)((d.heavy_count + (kBlock / kWave) - 1) / (kBlock / kWave));
    hv.L = L;
    plan.heavy.push_back(hv);
    plan.any_heavy = true;
  }
  plan.blocks.grid = (unsigned)d.k;
  plan.blocks.L = L;
  plan.tiles.grid = (unsigned)d.num_tiles;
  plan.tiles.L = L;
  plan.approve.grid = (unsigned)(d.num_tiles + d.k);
  plan.approve.L = L;
  PlanLaunch fin;
  fin.kernel = (void*)finalize_kernel(d.k, d.cache != nullptr);
  const long long unit = d.cache ? kCachedChunk : kFinalChunk;
  const long long cap = d.cache ? kCachedGrid : kFinalizeGrid;
  long long fchunks = ((long long)d.m + unit - 1) / unit;
  fin.grid = (unsigned)(fchunks < cap ? fchunks : cap);
  fin.L = L;
  plan.finalize.push_back(fin);
  plan.stats.grid = 1;
  plan.stats.L = L;
}

}  // namespace hg
