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
//   tilesum    per tile of 4096 vertices: weight of gain-g* candidates per
//              target block (vertex id order is tile order).
//   tilescan   per target block: the tile where the budget runs out.
//   approve    per tile: decide every candidate; the one boundary tile per
//              block is resolved by a workgroup-wide prefix sum in vertex
//              order.  Approved moves are applied right away: Phi updated
//              with integer atomics (order-independent), the attributed km1
//              change summed from the atomics' old values (subsection
//              "Attributed Gains"), touched nets listed.
//   finalize   per touched net: Lambda, S and lambda recomputed from the
//              final Phi row, its pins made eligible for the next round.
//   stats      one workgroup sums the counter slots into the round record.
//
// Candidate word: (gain << 32) | target, or -1 for "no candidate".
#include <limits.h>

#include "hg_bits.h"
#include "hg_device.h"
#include "hg_internal.h"
#include "hg_netrec.h"

namespace hg {

__device__ __forceinline__ long long pack_cand(int gain, int target) {
  return ((long long)gain << 32) | (unsigned)target;
}
__device__ __forceinline__ int cand_target(long long x) { return (int)(x & 0xffffffffLL); }
__device__ __forceinline__ int cand_gain(long long x) { return (int)(x >> 32); }

struct TouchedNet {
  int net;
  int lambda_old;
};

// --------------------------------------------------------------- select

// Record words 0 .. 1+WK (w, lambda, Lambda) plus the S word of block a.
template <int WK>
__device__ __forceinline__ void load_rec(const unsigned* __restrict__ r, int aw, unsigned& w,
                                         unsigned& lam, unsigned (&L)[WK], unsigned& S) {
  const uint4 q = *reinterpret_cast<const uint4*>(r);
  w = q.x;
  lam = q.y;
  if (WK == 1) {
    L[0] = q.z;
    S = q.w;
  } else {
    L[0] = q.z;
    L[1] = q.w;
#pragma unroll
    for (int j = 2; j < WK; ++j) L[j] = r[2 + j];
    S = r[2 + WK + aw];
  }
}

// Light vertices, one thread each, on a persistent grid: workgroup lb owns
// a contiguous run of 256-vertex chunks (so each XCD sweeps one vertex range
// and reuses the net records its neighbours pulled into its L2).  Candidate
// weights go to an LDS histogram (buckets [0, B) per target block, B =
// min(256, 2048/k)); higher gains and the final flush go to the histogram
// replica of this workgroup's XCD.
template <int WK>
__global__ __launch_bounds__(kBlock) void k_select_light(
    int n, int k, int rw, int lds_buckets, long long lmax, int cmax,
    const long long* __restrict__ vptr, const int* __restrict__ vnets,
    const int* __restrict__ vwgt, const int* __restrict__ part,
    const unsigned* __restrict__ netstate, const long long* __restrict__ block_w,
    unsigned char* __restrict__ eligible, unsigned char* __restrict__ moved,
    long long* __restrict__ cand, unsigned long long* __restrict__ hist,
    RoundCounters* __restrict__ ctr, int* __restrict__ err_flags) {
  __shared__ long long s_W[HG_MAX_K];
  __shared__ unsigned s_open[WK];
  __shared__ unsigned long long s_hist[kLdsHistEntries];
  __shared__ long long s_tmp[kBlock / kWave];
  const int B = lds_buckets;
  for (int i = threadIdx.x; i < WK; i += kBlock) s_open[i] = 0;
  for (int i = threadIdx.x; i < k * B; i += kBlock) s_hist[i] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock) {
    long long W = block_w[i];
    s_W[i] = W;
    if (W + cmax <= lmax) atomicOr(&s_open[i >> 5], 1u << (i & 31));
  }
  __syncthreads();
  unsigned long long* my_hist =
      hist + (size_t)(blockIdx.x % kHistReplicas) * HG_MAX_K * kBuckets;
  const long long chunks = ((long long)n + kBlock - 1) / kBlock;
  const long long per = (chunks + gridDim.x - 1) / gridDim.x;
  const long long lb = xcd_remap(blockIdx.x, gridDim.x);
  const long long c_end = (lb + 1) * per < chunks ? (lb + 1) * per : chunks;
  long long n_elig = 0, n_bnd = 0, n_cand = 0, n_apins = 0;
  // valid-block masks (only blocks < k; guards against stale caller state)
  unsigned valid[WK];
#pragma unroll
  for (int w = 0; w < WK; ++w) {
    const int lo = w * 32;
    valid[w] = k >= lo + 32 ? ~0u : (k > lo ? (1u << (k - lo)) - 1u : 0u);
  }
  for (long long c = lb * per; c < c_end; ++c) {
    const long long u = c * kBlock + threadIdx.x;
    if (u >= n) continue;
    if (moved) moved[u] = 0;
    const unsigned char el = eligible[u];
    if (!el) {
      cand[u] = -1;
      continue;
    }
    const int a = part[u];
    if ((unsigned)a >= (unsigned)k) {
      atomicOr(err_flags, kErrPart);
      cand[u] = -1;
      eligible[u] = 0;
      continue;
    }
    const long long b0 = vptr[u], b1 = vptr[u + 1];
    if (b1 - b0 > kLightLimit) continue;        // heavy vertex: the wavefront kernel owns it
    BitCounters<WK> C;
    C.clear();
    int tot = 0, ben = 0;
    bool bnd = false, heavy = false;
    const int aw = a >> 5;
    const unsigned abit = 1u << (a & 31);
    for (long long j = b0; j < b1; ++j) {
      const int e = vnets[j];
      unsigned w, lam, S, L[WK];
      load_rec<WK>(netstate + (long long)e * rw, aw, w, lam, L, S);
      tot += (int)w;
      if (tot > kLightLimit) {
        heavy = true;
        break;
      }
      bnd |= lam > 1u;
      if (S & abit) ben += (int)w;
      C.add(L, w);
    }
    if (heavy) continue;
    eligible[u] = 0;
    n_elig += 1;
    long long out = -1;
    if (bnd) {
      n_bnd += 1;
      n_apins += b1 - b0;
      const long long cu = vwgt ? vwgt[u] : 1;
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
    cand[u] = out;
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
    if (n_apins) atomicAdd(&ctr->slot[kCtrActivePins][sl], (unsigned long long)n_apins);
    if (n_elig) atomicAdd(&ctr->slot[kCtrEligible][sl], (unsigned long long)n_elig);
    if (n_bnd) atomicAdd(&ctr->slot[kCtrBoundary][sl], (unsigned long long)n_bnd);
    if (n_cand) atomicAdd(&ctr->slot[kCtrCandidates][sl], (unsigned long long)n_cand);
  }
}

// One wavefront per heavy vertex (w(I(u)) > 255): per-block connection
// weights in LDS (int32, enough because w(E) < 2^31), lanes stride over I(u).
__global__ __launch_bounds__(kBlock) void k_select_heavy(
    int heavy_count, int k, int rw, long long lmax, const int* __restrict__ heavy_list,
    const long long* __restrict__ vptr, const int* __restrict__ vnets,
    const int* __restrict__ vwgt, const int* __restrict__ part,
    const unsigned* __restrict__ netstate, const long long* __restrict__ block_w,
    unsigned char* __restrict__ eligible, long long* __restrict__ cand,
    unsigned long long* __restrict__ hist, int* __restrict__ overflow,
    RoundCounters* __restrict__ ctr, int* __restrict__ err_flags) {
  __shared__ long long s_W[HG_MAX_K];
  __shared__ int s_conn[kBlock / kWave][HG_MAX_K];
  for (int i = threadIdx.x; i < k; i += kBlock) s_W[i] = block_w[i];
  __syncthreads();
  const int wv = threadIdx.x / kWave, lane = lane_id();
  const long long idx = (long long)blockIdx.x * (kBlock / kWave) + wv;
  if (idx >= heavy_count) return;
  const int sl = (int)(idx % kSlots);
  unsigned long long* my_hist = hist + (size_t)(blockIdx.x % kHistReplicas) * HG_MAX_K * kBuckets;
  const int u = heavy_list[idx];
  const int a = part[u];
  const unsigned char el = eligible[u];
  if (!el || (unsigned)a >= (unsigned)k) {
    if (lane == 0) {
      cand[u] = -1;
      if (el) {
        atomicOr(err_flags, kErrPart);
        eligible[u] = 0;
      }
    }
    return;
  }
  int* conn = s_conn[wv];
  for (int i = lane; i < k; i += kWave) conn[i] = 0;
  wave_lds_sync();
  const long long b0 = vptr[u], b1 = vptr[u + 1];
  const int wk = bit_words(k);
  int tot = 0, ben = 0;
  bool bnd = false;
  for (long long j = b0 + lane; j < b1; j += kWave) {
    const int e = vnets[j];
    const unsigned* r = netstate + (long long)e * rw;
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
  const long long cu = vwgt ? vwgt[u] : 1;
  // best feasible neighbouring block on this lane's share of the blocks
  int bc = -1, bi = -1;
  long long bw = 0;
  for (int i = lane; i < k; i += kWave) {
    int ci = conn[i];
    if (i == a || ci <= 0 || s_W[i] + cu > lmax) continue;
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
    eligible[u] = 0;
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
          if (g > kBuckets - 1) atomicOr(&overflow[bi], 1);
        }
      }
    }
    cand[u] = out;
  }
}

// --------------------------------------------------------------- threshold

// One workgroup per target block t; thread j looks at gain bucket 255 - j
// (summed over the XCD replicas, which it also clears for the next round).
__global__ __launch_bounds__(kBlock) void k_threshold(int k, long long lmax,
                                                      const long long* __restrict__ block_w,
                                                      unsigned long long* __restrict__ hist,
                                                      int* __restrict__ overflow,
                                                      Threshold* __restrict__ thr,
                                                      RoundCounters* __restrict__ ctr) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_first;
  const int t = blockIdx.x;
  const int bucket = kBuckets - 1 - threadIdx.x;
  long long h = 0;
#pragma unroll
  for (int rep = 0; rep < kHistReplicas; ++rep) {
    unsigned long long* cell = hist + ((size_t)rep * HG_MAX_K + t) * kBuckets + bucket;
    h += (long long)*cell;
    *cell = 0;
  }
  const long long budget = lmax - block_w[t];
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
    thr[t] = r;
    if (f < kBlock && bucket == kBuckets - 1 && overflow[t]) {
      atomicOr(&ctr->any_overflow, 1u);
    } else {
      overflow[t] = 0;
    }
  }
}

// Only for graphs with heavy vertices: the ">= 255" bucket of block t holds
// several gain values and its budget ran out inside it.  Find the exact
// threshold gain by bisection over all candidates (a slow but rare path).
__global__ __launch_bounds__(kBlock) void k_overflow_resolve(
    int n, int k, const long long* __restrict__ cand, const int* __restrict__ vwgt,
    int* __restrict__ overflow, Threshold* __restrict__ thr, RoundCounters* __restrict__ ctr) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ long long s_max[kBlock / kWave];
  const int t = blockIdx.x;
  if (!ctr->any_overflow) return;
  if (!overflow[t]) return;
  const long long rem = thr[t].rem;
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
      if (x >= 0 && cand_target(x) == t && cand_gain(x) >= mid) s += vwgt ? vwgt[u] : 1;
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
    thr[t].gstar = (int)lo;
    thr[t].rem = rem - w_hi;
    overflow[t] = 0;
  }
}

// --------------------------------------------------------------- tiles

__global__ __launch_bounds__(kBlock) void k_tilesum(int n, int k, int num_tiles,
                                                    const long long* __restrict__ cand,
                                                    const int* __restrict__ vwgt,
                                                    const Threshold* __restrict__ thr,
                                                    long long* __restrict__ tilesum) {
  __shared__ unsigned long long s_sum[HG_MAX_K];
  __shared__ int s_g[HG_MAX_K];
  for (int i = threadIdx.x; i < k; i += kBlock) {
    s_sum[i] = 0;
    s_g[i] = thr[i].gstar;
  }
  __syncthreads();
  const int tile = blockIdx.x;
  const long long base = (long long)tile * kTile;
  for (int j = 0; j < kPerThreadTile; ++j) {
    long long u = base + (long long)j * kBlock + threadIdx.x;
    if (u < n) {
      long long x = cand[u];
      if (x >= 0) {
        int t = cand_target(x);
        if (cand_gain(x) == s_g[t]) atomicAdd(&s_sum[t], (unsigned long long)(vwgt ? vwgt[u] : 1));
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock)
    tilesum[(long long)i * num_tiles + tile] = (long long)s_sum[i];
}

__global__ __launch_bounds__(kBlock) void k_tilescan(int num_tiles,
                                                     const long long* __restrict__ tilesum,
                                                     Threshold* __restrict__ thr) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_tau;
  __shared__ long long s_remt;
  const int t = blockIdx.x;
  const Threshold r = thr[t];
  if (r.gstar < 0) {
    if (threadIdx.x == 0) thr[t].tau = num_tiles;
    return;
  }
  if (threadIdx.x == 0) {
    s_tau = num_tiles;
    s_remt = 0;
  }
  long long carry = 0;
  for (int base = 0; base < num_tiles; base += kBlock) {
    int i = base + threadIdx.x;
    long long v = i < num_tiles ? tilesum[(long long)t * num_tiles + i] : 0;
    long long tot;
    long long ex = block_excl_scan64(v, s_tmp, &tot);
    if (i < num_tiles && v > 0 && carry + ex + v > r.rem) atomicMin(&s_tau, i);
    __syncthreads();
    const int f = s_tau;
    if (f < num_tiles) {
      if (i == f) s_remt = r.rem - (carry + ex);
      break;
    }
    carry += tot;
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    thr[t].tau = s_tau;
    thr[t].rem_tile = s_remt;
  }
}

// --------------------------------------------------------------- approve + apply

struct ApplyArgs {
  int k, rw;
  const long long* vptr;
  const int* vnets;
  const int* vwgt;
  int* part;
  int* phi;
  const unsigned* netstate;
  unsigned char* moved;
  unsigned* touched;
  TouchedNet* tlist;
  RoundCounters* ctr;
};

constexpr int kStage = 512;          // touched nets staged per wavefront before a flush

// Copy a wavefront's staged touched nets to the global list with one atomic.
__device__ __forceinline__ void flush_stage(const ApplyArgs& A, const TouchedNet* stage, int cnt) {
  int base = 0;
  if (lane_id() == 0) base = (int)atomicAdd(&A.ctr->touched, (unsigned)cnt);
  base = __shfl(base, 0);
  for (int j = lane_id(); j < cnt; j += kWave) A.tlist[base + j] = stage[j];
}

// Apply the moves held in s_list[0..count) (vertex ids; targets in s_tgt).
// Each wave takes 64 movers at a time and walks their incident nets
// load-balanced.  Block-weight changes go to s_dW; newly touched nets are
// staged per wavefront in LDS and appended to the global list in bulk.
__device__ void apply_list(const ApplyArgs& A, const int* s_list, const int* s_tgt, int count,
                           unsigned long long* s_dW, int* s_excl, long long* s_beg,
                           TouchedNet* stage, long long& delta, long long& moved_pins,
                           long long& approved) {
  const int wv = threadIdx.x / kWave, lane = lane_id();
  int staged = 0;   // wave-uniform
  for (int base = wv * kWave; base < count; base += kBlock) {
    const int i = base + lane;
    int u = -1, a = 0, t = 0, len = 0;
    long long b = 0;
    if (i < count) {
      u = s_list[i];
      t = s_tgt[i];
      a = A.part[u];
      b = A.vptr[u];
      len = (int)(A.vptr[u + 1] - b);
      const long long cu = A.vwgt ? A.vwgt[u] : 1;
      A.part[u] = t;
      if (A.moved) A.moved[u] = 1;
      atomicAdd(&s_dW[t], (unsigned long long)cu);
      atomicAdd(&s_dW[a], (unsigned long long)(-cu));
      moved_pins += len;
      approved += 1;
    }
    wave_expand(b, len, s_excl + wv * kWave, s_beg + wv * kWave,
                [&](bool act, int owner, long long j) {
                  const int ao = __shfl(a, owner);
                  const int to = __shfl(t, owner);
                  bool fresh = false;
                  int e = 0, lam = 0;
                  if (act) {
                    e = A.vnets[j];
                    const unsigned* r = A.netstate + (long long)e * A.rw;
                    const int w = (int)r[0];
                    const int oa = atomicSub(&A.phi[(long long)e * A.k + ao], 1);
                    const int ot = atomicAdd(&A.phi[(long long)e * A.k + to], 1);
                    if (oa == 1) delta += w;    // Phi(e, a) drops to zero
                    if (ot == 0) delta -= w;    // Phi(e, t) rises from zero
                    const unsigned bit = 1u << (e & 31);
                    const unsigned old = atomicOr(&A.touched[e >> 5], bit);
                    fresh = !(old & bit);
                    if (fresh) lam = (int)r[1];
                  }
                  const unsigned long long mask = __ballot(fresh);
                  if (fresh) {
                    TouchedNet tn;
                    tn.net = e;
                    tn.lambda_old = lam;
                    stage[staged + __popcll(mask & (((unsigned long long)1 << lane) - 1))] = tn;
                  }
                  staged += __popcll(mask);
                  if (staged > kStage - kWave) {
                    wave_lds_sync();
                    flush_stage(A, stage, staged);
                    wave_lds_sync();
                    staged = 0;
                  }
                });
  }
  if (staged) {
    wave_lds_sync();
    flush_stage(A, stage, staged);
    wave_lds_sync();
  }
}

__global__ __launch_bounds__(kBlock) void k_approve_apply(
    int n, int num_tiles, ApplyArgs A, const long long* __restrict__ cand,
    const Threshold* __restrict__ thr, long long* __restrict__ block_w) {
  __shared__ int s_list[kTile];
  __shared__ int s_tgt[kTile];
  __shared__ TouchedNet s_stage[kBlock / kWave][kStage];
  __shared__ int s_g[HG_MAX_K];
  __shared__ int s_tau[HG_MAX_K];
  __shared__ unsigned long long s_dW[HG_MAX_K];
  __shared__ int s_excl[kBlock];
  __shared__ long long s_beg[kBlock];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ unsigned s_count;
  const int k = A.k;
  for (int i = threadIdx.x; i < k; i += kBlock) {
    s_g[i] = thr[i].gstar;
    s_tau[i] = thr[i].tau;
    s_dW[i] = 0;
  }
  if (threadIdx.x == 0) s_count = 0;
  __syncthreads();
  const bool boundary_wg = (int)blockIdx.x >= num_tiles;
  if (!boundary_wg) {
    const int tile = (int)xcd_remap(blockIdx.x, num_tiles);
    const long long base = (long long)tile * kTile;
    for (int j = 0; j < kPerThreadTile; ++j) {
      const long long u = base + (long long)j * kBlock + threadIdx.x;
      bool ok = false;
      int t = 0;
      if (u < n) {
        const long long x = cand[u];
        if (x >= 0) {
          t = cand_target(x);
          const int g = cand_gain(x), gs = s_g[t];
          ok = g > gs || (g == gs && tile < s_tau[t]);
        }
      }
      const int slot = wave_append(&s_count, ok);   // LDS counter, one atomic per wave
      if (ok) {
        s_list[slot] = (int)u;
        s_tgt[slot] = t;
      }
    }
  } else {
    // the tile where block t's budget runs out: prefix sums in vertex order
    const int t = (int)blockIdx.x - num_tiles;
    const Threshold r = thr[t];
    if (r.gstar < 0 || r.tau >= num_tiles) return;   // whole workgroup leaves together
    const long long base = (long long)r.tau * kTile + (long long)threadIdx.x * kPerThreadTile;
    long long mine = 0;
    for (int j = 0; j < kPerThreadTile; ++j) {
      const long long u = base + j;
      if (u < n) {
        const long long x = cand[u];
        if (x >= 0 && cand_target(x) == t && cand_gain(x) == r.gstar)
          mine += A.vwgt ? A.vwgt[u] : 1;
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
          const long long cu = A.vwgt ? A.vwgt[u] : 1;
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
  apply_list(A, s_list, s_tgt, count, s_dW, s_excl, s_beg, s_stage[threadIdx.x / kWave], delta,
             moved_pins, approved);
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock)
    if (s_dW[i]) atomicAdd((unsigned long long*)&block_w[i], s_dW[i]);
  delta = block_sum64(delta, s_tmp);
  moved_pins = block_sum64(moved_pins, s_tmp);
  approved = block_sum64(approved, s_tmp);
  if (threadIdx.x == 0) {
    const int sl = blockIdx.x % kSlots;
    if (delta) atomicAdd(&A.ctr->slot[kCtrDeltaAttr][sl], (unsigned long long)delta);
    if (moved_pins) atomicAdd(&A.ctr->slot[kCtrMovedPins][sl], (unsigned long long)moved_pins);
    if (approved) atomicAdd(&A.ctr->slot[kCtrApproved][sl], (unsigned long long)approved);
  }
}

// --------------------------------------------------------------- finalize

template <int G>
__global__ __launch_bounds__(kBlock) void k_finalize(
    int k, int rw, const long long* __restrict__ eptr, const int* __restrict__ pins,
    const int* __restrict__ phi, unsigned* __restrict__ netstate,
    unsigned* __restrict__ touched, const TouchedNet* __restrict__ tlist,
    unsigned char* __restrict__ eligible, RoundCounters* __restrict__ ctr) {
  __shared__ long long s_tmp[kBlock / kWave];
  const int grp = threadIdx.x / G, gl = threadIdx.x % G;
  const long long ngroups = (long long)gridDim.x * (kBlock / G);
  const long long count = (long long)ctr->touched;
  const int wk = bit_words(k);
  long long dcheck = 0;
  for (long long idx = (long long)blockIdx.x * (kBlock / G) + grp; idx < count; idx += ngroups) {
    const TouchedNet tn = tlist[idx];
    const int e = tn.net;
    const int* row = phi + (long long)e * k;
    unsigned* rec = netstate + (long long)e * rw;
    NetBits nb = net_bits<G>(k, gl, [&](int i) { return row[i]; }, [&](int, int) {});
    if (gl >= 1 && gl < 2 + 2 * wk) rec[gl] = nb.word;
    if (gl == 0) {
      const int w = (int)rec[0];
      dcheck += (long long)(tn.lambda_old - nb.lambda) * w;
      atomicAnd(&touched[e >> 5], ~(1u << (e & 31)));
    }
    const long long b = eptr[e], t = eptr[e + 1];
    for (long long p = b + gl; p < t; p += G) eligible[pins[p]] = 1;
  }
  dcheck = block_sum64(dcheck, s_tmp);
  if (threadIdx.x == 0 && dcheck)
    atomicAdd(&ctr->slot[kCtrDeltaCheck][blockIdx.x % kSlots], (unsigned long long)dcheck);
}

// One workgroup: sum the counter slots, write the round record, move km1 by
// the attributed drop, reset the counters for the next round.
__global__ __launch_bounds__(kBlock) void k_round_stats(int k, RoundCounters* __restrict__ ctr,
                                                        const long long* __restrict__ block_w,
                                                        long long* __restrict__ km1,
                                                        hg_round_stats* __restrict__ stats) {
  __shared__ long long s_sum[kNumCounters];
  __shared__ long long s_max[kBlock / kWave];
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  for (int c = wv; c < kNumCounters; c += kBlock / kWave) {
    long long v = (long long)ctr->slot[c][lane];
    v = wave_sum(v);
    if (lane == 0) s_sum[c] = v;
    ctr->slot[c][lane] = 0;
  }
  long long mx = LLONG_MIN;
  for (int i = threadIdx.x; i < k; i += kBlock) mx = block_w[i] > mx ? block_w[i] : mx;
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
    st.touched_nets = (long long)ctr->touched;
    st.km1_delta = s_sum[kCtrDeltaAttr];
    st.km1_delta_recomputed = s_sum[kCtrDeltaCheck];
    st.active_pins = s_sum[kCtrActivePins];
    st.km1_after = *km1 - st.km1_delta;
    st.max_block_weight = m;
    *km1 = st.km1_after;
    *stats = st;
    ctr->touched = 0;
    ctr->any_overflow = 0;
  }
}

// --------------------------------------------------------------- launch

int group_lanes(int k);

static int lds_buckets(int k) {
  int b = kBuckets;
  while (b > 1 && b * k > kLdsHistEntries) b >>= 1;
  return b;
}

template <int WK>
static void launch_select_light(hg_graph_s* g, int k, long long lmax, const int* part,
                                const unsigned* netstate, const long long* block_w,
                                unsigned char* eligible, unsigned char* moved, hipStream_t s) {
  char* ws = g->ws;
  long long chunks = ((long long)g->n + kBlock - 1) / kBlock;
  unsigned grid = (unsigned)(chunks < kSelectGrid ? chunks : kSelectGrid);
  hipLaunchKernelGGL(k_select_light<WK>, dim3(grid), dim3(kBlock), 0, s, g->n, k, net_words(k),
                     lds_buckets(k), lmax, g->info.max_vertex_weight, g->vptr, g->vnets, g->vwgt,
                     part, netstate, block_w, eligible, moved, (long long*)(ws + g->lay.cand),
                     (unsigned long long*)(ws + g->lay.hist), (RoundCounters*)(ws + g->lay.ctr),
                     (int*)(ws + g->lay.flags));
}

template <int G>
static void launch_finalize(hg_graph_s* g, int k, const int* phi, unsigned* netstate,
                            unsigned char* eligible, hipStream_t s) {
  char* ws = g->ws;
  long long blocks = ((long long)g->m + (kBlock / G) - 1) / (kBlock / G);
  if (blocks > kFinalizeGrid) blocks = kFinalizeGrid;
  hipLaunchKernelGGL(k_finalize<G>, dim3((unsigned)blocks), dim3(kBlock), 0, s, k, net_words(k),
                     g->eptr, g->pins, phi, netstate, (unsigned*)(ws + g->lay.touched),
                     (const TouchedNet*)(ws + g->lay.tlist), eligible,
                     (RoundCounters*)(ws + g->lay.ctr));
}

hipError_t launch_lp_round(hg_graph_s* g, int k, long long lmax, int* part, int* phi,
                           unsigned* netstate, long long* block_w, unsigned char* eligible,
                           unsigned char* moved, long long* km1, hg_round_stats* stats,
                           hipStream_t s, hipEvent_t* marks) {
  char* ws = g->ws;
  if (marks) (void)hipEventRecord(marks[0], s);
  switch (bit_words(k)) {
    case 1: launch_select_light<1>(g, k, lmax, part, netstate, block_w, eligible, moved, s); break;
    case 2: launch_select_light<2>(g, k, lmax, part, netstate, block_w, eligible, moved, s); break;
    case 4: launch_select_light<4>(g, k, lmax, part, netstate, block_w, eligible, moved, s); break;
    default: launch_select_light<8>(g, k, lmax, part, netstate, block_w, eligible, moved, s); break;
  }
  RoundCounters* ctr = (RoundCounters*)(ws + g->lay.ctr);
  unsigned long long* hist = (unsigned long long*)(ws + g->lay.hist);
  int* overflow = (int*)(ws + g->lay.overflow);
  Threshold* thr = (Threshold*)(ws + g->lay.thr);
  long long* cand = (long long*)(ws + g->lay.cand);
  const int heavy = g->info.heavy_count;
  if (heavy > 0) {
    unsigned grid = (unsigned)((heavy + (kBlock / kWave) - 1) / (kBlock / kWave));
    hipLaunchKernelGGL(k_select_heavy, dim3(grid), dim3(kBlock), 0, s, heavy, k, net_words(k),
                       lmax, (const int*)(ws + g->lay.heavy), g->vptr, g->vnets, g->vwgt, part,
                       netstate, block_w, eligible, cand, hist, overflow, ctr,
                       (int*)(ws + g->lay.flags));
  }
  if (marks) (void)hipEventRecord(marks[1], s);
  hipLaunchKernelGGL(k_threshold, dim3(k), dim3(kBlock), 0, s, k, lmax, block_w, hist, overflow,
                     thr, ctr);
  if (heavy > 0)
    hipLaunchKernelGGL(k_overflow_resolve, dim3(k), dim3(kBlock), 0, s, g->n, k, cand, g->vwgt,
                       overflow, thr, ctr);
  const int nt = g->lay.num_tiles;
  long long* tilesum = (long long*)(ws + g->lay.tilesum);
  hipLaunchKernelGGL(k_tilesum, dim3(nt), dim3(kBlock), 0, s, g->n, k, nt, cand, g->vwgt, thr,
                     tilesum);
  hipLaunchKernelGGL(k_tilescan, dim3(k), dim3(kBlock), 0, s, nt, tilesum, thr);
  ApplyArgs A;
  A.k = k;
  A.rw = net_words(k);
  A.vptr = g->vptr;
  A.vnets = g->vnets;
  A.vwgt = g->vwgt;
  A.part = part;
  A.phi = phi;
  A.netstate = netstate;
  A.moved = moved;
  A.touched = (unsigned*)(ws + g->lay.touched);
  A.tlist = (TouchedNet*)(ws + g->lay.tlist);
  A.ctr = ctr;
  hipLaunchKernelGGL(k_approve_apply, dim3(nt + k), dim3(kBlock), 0, s, g->n, nt, A, cand, thr,
                     block_w);
  if (marks) (void)hipEventRecord(marks[2], s);
  switch (group_lanes(k)) {
    case 4: launch_finalize<4>(g, k, phi, netstate, eligible, s); break;
    case 8: launch_finalize<8>(g, k, phi, netstate, eligible, s); break;
    case 16: launch_finalize<16>(g, k, phi, netstate, eligible, s); break;
    case 32: launch_finalize<32>(g, k, phi, netstate, eligible, s); break;
    default: launch_finalize<64>(g, k, phi, netstate, eligible, s); break;
  }
  hipLaunchKernelGGL(k_round_stats, dim3(1), dim3(kBlock), 0, s, k, ctr, block_w, km1, stats);
  if (marks) (void)hipEventRecord(marks[3], s);
  return hipGetLastError();
}

}  // namespace hg
