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
#include "hg_sweep.h"

namespace hg {

__device__ __forceinline__ long long pack_cand(int gain, int target) {
  return ((long long)gain << 32) | (unsigned)target;
}
__device__ __forceinline__ int cand_target(long long x) { return (int)(x & 0xffffffffLL); }
__device__ __forceinline__ int cand_gain(long long x) { return (int)(x >> 32); }

// --------------------------------------------------------------- select

// Light vertices, one thread each, on a persistent grid: workgroup lb owns
// a contiguous run of 256-vertex chunks (so each XCD sweeps one vertex range
// and reuses the net records its neighbours pulled into its L2).  Candidate
// weights go to an LDS histogram (buckets [0, B) per target block, B =
// min(256, 2048/k)); higher gains and the final flush go to the histogram
// replica of this workgroup's XCD.
template <int WK, int VIEW>
__global__ __launch_bounds__(kBlock) void k_select_light(
    int n, int k, int rw, int lds_buckets, long long lmax, int cmax,
    const long long* __restrict__ vptr, const int* __restrict__ vnets,
    const int* __restrict__ vwgt, const int* __restrict__ part,
    const unsigned* __restrict__ netstate, const unsigned* __restrict__ view,
    const long long* __restrict__ block_w,
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
  // XCD x sweeps vertex chunks [x*per_xcd, (x+1)*per_xcd); its workgroups
  // take consecutive chunks side by side, so at any time one XCD works on a
  // narrow window of vertices whose net records stay in its L2.
  const long long chunks = ((long long)n + kBlock - 1) / kBlock;
  const int xcd = blockIdx.x % kNumXcd;
  const long long wg_on_xcd = (gridDim.x - xcd + kNumXcd - 1) / kNumXcd;
  const long long li = blockIdx.x / kNumXcd;
  const long long per_xcd = (chunks + kNumXcd - 1) / kNumXcd;
  const long long c_begin = xcd * per_xcd;
  const long long c_end = c_begin + per_xcd < chunks ? c_begin + per_xcd : chunks;
  long long n_elig = 0, n_bnd = 0, n_cand = 0, n_apins = 0;
  // valid-block masks (only blocks < k; guards against stale caller state)
  unsigned valid[WK];
#pragma unroll
  for (int w = 0; w < WK; ++w) {
    const int lo = w * 32;
    valid[w] = k >= lo + 32 ? ~0u : (k > lo ? (1u << (k - lo)) - 1u : 0u);
  }
  for (long long c = c_begin + li; c < c_end; c += wg_on_xcd) {
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
    // Software-pipelined sweep: issue kUnroll independent record gathers
    // before consuming any of them.
    for (long long j = b0; j < b1 && !heavy; j += kUnroll) {
      unsigned w[kUnroll], S[kUnroll], L[kUnroll][WK];
      bool cut[kUnroll];
      int e[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) e[q] = j + q < b1 ? vnets[j + q] : -1;
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        if (e[q] >= 0) {
          read_net<WK, VIEW>(netstate, rw, view, e[q], aw, w[q], cut[q], L[q], S[q]);
        } else {
          w[q] = 0;
          cut[q] = false;
          S[q] = 0;
#pragma unroll
          for (int x = 0; x < WK; ++x) L[q][x] = 0;
        }
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        tot += (int)w[q];
        bnd |= cut[q];
        if (S[q] & abit) ben += (int)w[q];
      }
      if (tot > kLightLimit) {
        heavy = true;
        break;
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q)
        if (w[q]) C.add(L[q], w[q]);
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
  bool unit_nets;
  const long long* vptr;
  const int* vnets;
  const int* vwgt;
  int* part;
  int* phi;
  const unsigned* netstate;
  unsigned char* moved;
  unsigned char* touched;
  RoundCounters* ctr;
};

// Apply the moves held in s_list[0..count) (vertex ids; targets in s_tgt):
// part, moved flags and block-weight deltas per mover, then the movers'
// incident nets as one flattened range split over all 256 threads (so a tile
// with few movers still keeps four wavefronts busy, and a high-degree mover is
// spread over the workgroup).  Phi is updated with integer atomics whose old
// values give the attributed km1 change; every incident net gets its touched
// flag (a plain byte store: all writers store the same value).
__device__ void apply_list(const ApplyArgs& A, const int* s_list, const int* s_tgt, int count,
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
      const int a = A.part[u];
      const long long b = A.vptr[u];
      const int len = (int)(A.vptr[u + 1] - b);
      const long long cu = A.vwgt ? A.vwgt[u] : 1;
      A.part[u] = t;
      if (A.moved) A.moved[u] = 1;
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
  for (long long j = threadIdx.x; j < total; j += kBlock) {
    // owner: largest i < count with s_off[i] <= j
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= j) lo = mid; else hi = mid - 1;
    }
    const int e = A.vnets[s_beg[lo] + (j - s_off[lo])];
    const int ao = s_from[lo], to = s_tgt[lo];
    const int oa = atomicSub(&A.phi[(long long)e * A.k + ao], 1);
    const int ot = atomicAdd(&A.phi[(long long)e * A.k + to], 1);
    if (oa == 1 || ot == 0) {
      const int w = A.unit_nets ? 1 : (int)A.netstate[(long long)e * A.rw];
      if (oa == 1) delta += w;    // Phi(e, a) drops to zero
      if (ot == 0) delta -= w;    // Phi(e, t) rises from zero
    }
    A.touched[e] = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_approve_apply(
    int n, int num_tiles, ApplyArgs A, const long long* __restrict__ cand,
    const Threshold* __restrict__ thr, long long* __restrict__ block_w) {
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
  if (count > 0)
    apply_list(A, s_list, s_tgt, count, s_from, s_beg, s_off, s_tmp, s_dW, delta, moved_pins,
               approved);
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

// Workgroup lb owns a contiguous run of nets (XCD-aware).  It reads their
// touched flags 1024 at a time (coalesced), lists the touched ones in LDS and
// hands them to groups of G lanes: Lambda, S and lambda are rebuilt from the
// final Phi row, the flag is cleared and every pin becomes eligible.  The
// lane that rewrites lambda(e) reads the old value first, so the drop
// (lambda_old - lambda_new) * w(e) summed over touched nets checks the
// attributed total.
constexpr int kFinalChunk = kBlock;

template <int G>
__global__ __launch_bounds__(kBlock) void k_finalize(
    int m, int k, int rw, const long long* __restrict__ eptr, const int* __restrict__ pins,
    const int* __restrict__ phi, unsigned* __restrict__ netstate,
    unsigned char* __restrict__ touched, unsigned char* __restrict__ eligible,
    RoundCounters* __restrict__ ctr, unsigned* __restrict__ view, int view_kind) {
  __shared__ int s_list[kFinalChunk];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ unsigned s_cnt;
  constexpr int kGroups = kBlock / G;
  const int grp = threadIdx.x / G, gl = threadIdx.x % G;
  const int wk = bit_words(k);
  const long long chunks = ((long long)m + kFinalChunk - 1) / kFinalChunk;
  const long long per = (chunks + gridDim.x - 1) / gridDim.x;
  const long long lb = xcd_remap(blockIdx.x, gridDim.x);
  const long long c_end = (lb + 1) * per < chunks ? (lb + 1) * per : chunks;
  long long dcheck = 0, ntouched = 0;
  for (long long c = lb * per; c < c_end; ++c) {
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    // one flag per thread (the flag array is padded to whole chunks, zero past m)
    const long long e0 = c * kFinalChunk + threadIdx.x;
    const bool t0 = touched[e0] != 0;
    const int slot = wave_append(&s_cnt, t0);
    if (t0) s_list[slot] = (int)e0;
    __syncthreads();
    const int cnt = (int)s_cnt;
    ntouched += cnt;
    for (int i = grp; i < cnt; i += kGroups) {
      const int e = s_list[i];
      const int* row = phi + (long long)e * k;
      unsigned* rec = netstate + (long long)e * rw;
      int lam_old = 0, w = 0;
      if (gl == 1) {
        lam_old = (int)rec[1];
        w = (int)rec[0];
      }
      NetBits nb = net_bits<G>(k, gl, [&](int i2) { return row[i2]; }, [&](int, int) {});
      if (gl >= 1 && gl < 2 + 2 * wk) rec[gl] = nb.word;
      if (view_kind != kViewFull) write_view(view, e, view_kind, gl, nb);
      if (gl == 1) dcheck += (long long)(lam_old - nb.lambda) * w;
      if (gl == 0) touched[e] = 0;
      const long long b = eptr[e], t = eptr[e + 1];
      for (long long p = b + gl; p < t; p += G) eligible[pins[p]] = 1;
    }
    __syncthreads();
  }
  dcheck = block_sum64(dcheck, s_tmp);
  if (threadIdx.x == 0) {
    const int sl = blockIdx.x % kSlots;
    if (dcheck) atomicAdd(&ctr->slot[kCtrDeltaCheck][sl], (unsigned long long)dcheck);
    if (ntouched) atomicAdd(&ctr->slot[kCtrTouched][sl], (unsigned long long)ntouched);
  }
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
    st.touched_nets = s_sum[kCtrTouched];
    st.km1_delta = s_sum[kCtrDeltaAttr];
    st.km1_delta_recomputed = s_sum[kCtrDeltaCheck];
    st.active_pins = s_sum[kCtrActivePins];
    st.km1_after = *km1 - st.km1_delta;
    st.max_block_weight = m;
    *km1 = st.km1_after;
    *stats = st;
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
  const unsigned* view = netstate + (size_t)g->m * net_words(k);
  auto kern = k_select_light<WK, kViewFull>;
  switch (net_view(k, g->unit_nets)) {
    case kView16: kern = k_select_light<1, kView16>; break;
    case kView32: kern = k_select_light<1, kView32>; break;
    case kView64: kern = k_select_light<2, kView64>; break;
    default: break;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, g->n, k, net_words(k),
                     lds_buckets(k), lmax, g->info.max_vertex_weight, g->vptr, g->vnets, g->vwgt,
                     part, netstate, view, block_w, eligible, moved, (long long*)(ws + g->lay.cand),
                     (unsigned long long*)(ws + g->lay.hist), (RoundCounters*)(ws + g->lay.ctr),
                     (int*)(ws + g->lay.flags));
}

template <int G>
static void launch_finalize(hg_graph_s* g, int k, const int* phi, unsigned* netstate,
                            unsigned char* eligible, hipStream_t s) {
  char* ws = g->ws;
  long long blocks = ((long long)g->m + kFinalChunk - 1) / kFinalChunk;
  if (blocks > kFinalizeGrid) blocks = kFinalizeGrid;
  hipLaunchKernelGGL(k_finalize<G>, dim3((unsigned)blocks), dim3(kBlock), 0, s, g->m, k,
                     net_words(k), g->eptr, g->pins, phi, netstate,
                     (unsigned char*)(ws + g->lay.touched), eligible,
                     (RoundCounters*)(ws + g->lay.ctr),
                     netstate + (size_t)g->m * net_words(k), net_view(k, g->unit_nets));
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
  A.touched = (unsigned char*)(ws + g->lay.touched);
  A.unit_nets = g->unit_nets;
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
