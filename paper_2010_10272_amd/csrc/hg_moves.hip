// hg_moves.hip -- move sequences: exact gains of an ordered sequence of moves
// (section "Parallel Gain Calculation", subsection "Parallel Gain
// Recalculation" and its Lemma), the best prefix of such a sequence (section
// "Direct k-way FM", second phase), and the monotone label-propagation round
// built from them.
//
// Exact gains.  Move j (1-based index J) takes u_j from block a to block b.
// For every (net, block) cell touched by the sequence the kernels gather
//   out_max(e, i)  the largest J moving a pin of e out of i   (0 if none)
//   in_min(e, i)   the smallest J moving a pin of e into i     (INT_MAX if none)
//   out_cnt(e, i)  how many moves take a pin of e out of i
// with integer atomics (max, min, add: order-independent) on one 16-byte cell
// per (net, block), so a move touches one cache line per cell.  A cell with
// Phi(e, i) = 1 has at most one mover out of i, which stores out_max with a
// plain store; its out_cnt is then (out_max > 0) and is never counted.  Then,
// per move and incident net e, Psi(e, i) = Phi(e, i) - out_cnt(e, i) and the
// Lemma:
//   Phi(e, a) = 1 just before move J  iff  Psi(e,a) = 0, out_max(e,a) = J,
//                                          in_min(e,a) > J
//   Phi(e, b) = 0 just before move J  iff  Psi(e,b) = 0, in_min(e,b) = J,
//                                          out_max(e,b) < J
// so gain_J = w({e : first}) - w({e : second}).  Only cells of nets incident
// to a mover are written (an init pass sets them first), so the m x k arrays
// never need a full clear.
//
// Monotone round.  Select and approval run as in a plain round, but approve
// only marks the approved moves (and sets their cells empty).  A stable radix
// sort of the marked vertices orders them by (select gain desc, vertex id
// asc): its first pass reads the marks and candidate words directly, so the
// moves are compacted and ordered in one pass when gains fit 8 bits.  Their
// exact gains in that order come from the kernels above, each 64-move tile
// leaves its sum and its best prefix, one workgroup scans those for the
// prefix with the largest total (ties: the longer), and only that prefix is
// applied; finalize and the round record follow as usual.
// Every prefix of approved moves respects L_max (the approval budgets each
// target for all of its moves; moves out of a block only lower it), so the
// cut needs no balance test, and km1 never increases.
#include <limits.h>
#include <string.h>

#include <algorithm>

#include "hg_device.h"
#include "hg_internal.h"
#include "hg_lp.h"
#include "hg_sort.h"

namespace hg {
namespace {

// Moves per tile of the sequence kernels (one wavefront's worth: a tile's
// gains are scanned by one wave), and their persistent grid.
constexpr int kSeqTile = kWave;
constexpr int kSeqGrid = 1024;

// Layout of the caller's move-sequence workspace.
struct MovesLayout {
  size_t cell, seen, appr, key[2], val[2], hist, dtot, gains, tsum, tbest_v, tbest_i, best, tdev,
      total;
  int sort_tiles, seq_tiles;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

MovesLayout moves_layout(long long n, long long m, int k) {
  MovesLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  const size_t cells = (size_t)m * (size_t)k;
  L.sort_tiles = (int)((n + kSortTile - 1) / kSortTile);
  L.seq_tiles = (int)((n + kSeqTile - 1) / kSeqTile);
  L.cell = take(sizeof(int4) * cells);
  L.seen = take(sizeof(int) * (size_t)n);
  L.appr = take((size_t)n);
  for (int i = 0; i < 2; ++i) {
    L.key[i] = take(sizeof(unsigned) * (size_t)n);
    L.val[i] = take(sizeof(int) * (size_t)n);
  }
  L.hist = take(sizeof(unsigned) * (size_t)kDigits * L.sort_tiles);
  L.dtot = take(sizeof(unsigned) * kDigits);
  L.gains = take(sizeof(long long) * (size_t)n);
  L.tsum = take(sizeof(long long) * (size_t)L.seq_tiles);
  L.tbest_v = take(sizeof(long long) * (size_t)L.seq_tiles);
  L.tbest_i = take(sizeof(int) * (size_t)L.seq_tiles);
  L.best = take(sizeof(long long) * 2);
  L.tdev = take(sizeof(int));
  L.total = off;
  return L;
}

// A move sequence as the kernels read it.  Move j (0-based) moves u = mu[j]
// from part[u] to mt[j], or -- sorted monotone rounds -- to the target in
// cand[u].  The length is t, or *t_dev when that is set (known only on the
// device).
struct Seq {
  const int* mu;
  const int* mt;                 // null: target from cand
  const long long* cand;
  int t;
  const int* t_dev;              // length known only on the device (monotone rounds)
  const int* part;
  const int* phi;
  const long long* vptr;
  const int* vnets;
  const int* ewgt;
  const int* vwgt;
  int n, k;
  int4* cell;                    // per (net, block): out_max, in_min, out_cnt, unused
  int* seen;
  int* err_flags;
};

__device__ __forceinline__ int seq_len(const Seq& S) { return S.t_dev ? *S.t_dev : S.t; }

// Source and target of move j, or false for a move the checks reject.
__device__ __forceinline__ bool seq_move(const Seq& S, int j, int& u, int& a, int& b) {
  u = S.mu[j];
  if ((unsigned)u >= (unsigned)S.n) return false;
  b = S.mt ? S.mt[j] : (int)(S.cand[u] & 0xffffffffLL);
  a = S.part[u];
  return (unsigned)b < (unsigned)S.k && (unsigned)a < (unsigned)S.k && a != b;
}

// Every incidence (move j, net e) of the kSeqTile moves of tile `tile`,
// spread over all threads of the workgroup (prefix sum of the movers'
// degrees, owner by binary search in LDS).  f(j, u, a, b, e) is called once
// per incidence.  Tiles are short, so a short sequence still spreads over
// many workgroups; the kernels below loop over tiles with a grid stride.

template <typename F>
__device__ void for_incidences(const Seq& S, int t, int tile, F f) {
  __shared__ long long s_beg[kBlock];
  __shared__ int s_off[kBlock + 1];
  __shared__ int s_u[kBlock], s_a[kBlock], s_b[kBlock];
  __shared__ long long s_tmp[kBlock / kWave];
  const int j = tile * kSeqTile + threadIdx.x;
  int u = -1, a = 0, b = 0;
  long long len = 0, beg = 0;
  if (threadIdx.x < kSeqTile && j < t && seq_move(S, j, u, a, b)) {
    beg = S.vptr[u];
    len = S.vptr[u + 1] - beg;
  } else {
    u = -1;
  }
  long long total;
  const long long off = block_excl_scan64(len, s_tmp, &total);
  s_off[threadIdx.x] = (int)off;
  s_beg[threadIdx.x] = beg;
  s_u[threadIdx.x] = u;
  s_a[threadIdx.x] = a;
  s_b[threadIdx.x] = b;
  __syncthreads();
  for (long long x = threadIdx.x; x < total; x += kBlock) {
    int lo = 0, hi = kSeqTile - 1;   // owner: last slot with s_off <= x
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    // slots without a move have length 0, so the owner always holds one
    const int e = S.vnets[s_beg[lo] + (x - s_off[lo])];
    f(tile * kSeqTile + lo, s_u[lo], s_a[lo], s_b[lo], e);
  }
  __syncthreads();   // the LDS lists are reused by the workgroup's next tile
}

// Checks of an explicit sequence: vertex and target in range, target !=
// source, no vertex twice (seen[u] claims u for its first move).
__global__ __launch_bounds__(kBlock) void k_seq_check(Seq S) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= S.t) return;
  int u, a, b;
  if (!seq_move(S, j, u, a, b)) {
    atomicOr(S.err_flags, kErrMoves);
    return;
  }
  if (atomicCAS(&S.seen[u], 0, j + 1) != 0) atomicOr(S.err_flags, kErrMoves);
}

__global__ __launch_bounds__(kBlock) void k_seq_clear(Seq S) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= S.t) return;
  const int u = S.mu[j];
  if ((unsigned)u < (unsigned)S.n) S.seen[u] = 0;
}

// Cells (e, a) and (e, b) of every incidence start empty.
__global__ __launch_bounds__(kBlock) void k_seq_init(Seq S) {
  const int t = seq_len(S);
  for (int tile = blockIdx.x; tile * kSeqTile < t; tile += gridDim.x)
    for_incidences(S, t, tile, [&](int, int, int a, int b, int e) {
      const size_t ca = (size_t)e * S.k + a, cb = (size_t)e * S.k + b;
      S.cell[ca] = make_int4(0, INT_MAX, 0, 0);
      S.cell[cb] = make_int4(0, INT_MAX, 0, 0);
    });
}

__global__ __launch_bounds__(kBlock) void k_seq_collect(Seq S) {
  const int t = seq_len(S);
  for (int tile = blockIdx.x; tile * kSeqTile < t; tile += gridDim.x)
    for_incidences(S, t, tile, [&](int j, int, int a, int b, int e) {
      const size_t ca = (size_t)e * S.k + a, cb = (size_t)e * S.k + b;
      atomicMin(&S.cell[cb].y, j + 1);
      if (S.phi[ca] == 1) {
        S.cell[ca].x = j + 1;   // the only pin of e in a: the cell's only mover out
      } else {
        atomicMax(&S.cell[ca].x, j + 1);
        atomicAdd(&S.cell[ca].z, 1);
      }
    });
}

// Best (total, length) of two prefixes; ties to the longer.
__device__ __forceinline__ bool better(long long v, int p, long long bv, int bp) {
  return v > bv || (v == bv && p > bp);
}

// gains[j] = exact gain of move j (the Lemma).  With tsum set, each tile also
// leaves its gain total and the best prefix ending inside it (value relative
// to the tile's start, length counted from the sequence start).
__global__ __launch_bounds__(kBlock) void k_seq_gains(Seq S, long long* gains, long long* tsum,
                                                      long long* tbest_v, int* tbest_i) {
  __shared__ long long s_gain[kSeqTile];
  const int t = seq_len(S);
  for (int tile = blockIdx.x; tile * kSeqTile < t; tile += gridDim.x) {
    if (threadIdx.x < kSeqTile) s_gain[threadIdx.x] = 0;
    __syncthreads();
    for_incidences(S, t, tile, [&](int j, int, int a, int b, int e) {
      const int J = j + 1;
      const size_t ca = (size_t)e * S.k + a, cb = (size_t)e * S.k + b;
      // all four reads first (no short-circuit: loads in branches would not overlap)
      const int4 A = S.cell[ca], B = S.cell[cb];
      const int pa = S.phi[ca], pb = S.phi[cb];
      // out counts; a cell with one pin records only whether it moved
      const int za = pa == 1 ? (A.x > 0) : A.z;
      const int zb = pb == 1 ? (B.x > 0) : B.z;
      const bool last_out = (pa - za == 0) & (A.x == J) & (A.y > J);
      const bool first_in = (pb - zb == 0) & (B.y == J) & (B.x < J);
      if (last_out != first_in) {
        const long long w = S.ewgt ? S.ewgt[e] : 1;
        atomicAdd((unsigned long long*)&s_gain[j - tile * kSeqTile],
                  (unsigned long long)(last_out ? w : -w));
      }
    });
    const int j = tile * kSeqTile + threadIdx.x;
    if (threadIdx.x < kSeqTile) {
      const bool in = j < t;
      const long long g = in ? s_gain[threadIdx.x] : 0;
      if (in) gains[j] = g;
      if (tsum) {
        // one wavefront: scan of the tile's gains, argmax of the prefixes
        const long long incl = wave_incl_scan64(g);
        long long bv = in ? incl : LLONG_MIN;
        int bp = in ? j + 1 : -1;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
          const long long ov = __shfl_xor(bv, o);
          const int op = __shfl_xor(bp, o);
          if (better(ov, op, bv, bp)) {
            bv = ov;
            bp = op;
          }
        }
        if (threadIdx.x == kSeqTile - 1) tsum[tile] = incl;
        if (threadIdx.x == 0) {
          tbest_v[tile] = bv;
          tbest_i[tile] = bp;
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ best prefix

// One workgroup: exclusive scan of the chunk sums.
__global__ __launch_bounds__(kBlock) void k_prefix_top(const long long* csum, long long* coff,
                                                       int chunks) {
  __shared__ long long s_tmp[kBlock / kWave];
  long long carry = 0;
  for (int b = 0; b < chunks; b += kBlock) {
    const int i = b + threadIdx.x;
    const long long v = i < chunks ? csum[i] : 0;
    long long tot;
    const long long ex = block_excl_scan64(v, s_tmp, &tot);
    if (i < chunks) coff[i] = carry + ex;
    carry += tot;
  }
}

// One workgroup: the best prefix of the whole sequence from the tiles'
// summaries (exclusive scan of the tile totals plus each tile's best), and
// the empty prefix -> best[0] (total), best[1] (length); ties to the longer.
__global__ __launch_bounds__(kBlock) void k_prefix_pick(const int* t_dev, const long long* tsum,
                                                        const long long* tbest_v,
                                                        const int* tbest_i, long long* best) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ long long s_bv[kBlock / kWave];
  __shared__ int s_bp[kBlock / kWave];
  const int tiles = (*t_dev + kSeqTile - 1) / kSeqTile;
  long long bv = 0, carry = 0;
  int bp = 0;   // the empty prefix
  for (int b = 0; b < tiles; b += kBlock) {
    const int i = b + threadIdx.x;
    const long long v = i < tiles ? tsum[i] : 0;
    long long tot;
    const long long ex = block_excl_scan64(v, s_tmp, &tot);
    if (i < tiles && better(carry + ex + tbest_v[i], tbest_i[i], bv, bp)) {
      bv = carry + ex + tbest_v[i];
      bp = tbest_i[i];
    }
    carry += tot;
  }
  const int lane = lane_id(), wv = threadIdx.x / kWave;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const long long ov = __shfl_xor(bv, o);
    const int op = __shfl_xor(bp, o);
    if (better(ov, op, bv, bp)) {
      bv = ov;
      bp = op;
    }
  }
  if (lane == 0) {
    s_bv[wv] = bv;
    s_bp[wv] = bp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w)
      if (better(s_bv[w], s_bp[w], bv, bp)) {
        bv = s_bv[w];
        bp = s_bp[w];
      }
    best[0] = bv;
    best[1] = bp;
  }
}

// Apply moves [0, best[1]) of a sorted monotone-round sequence: part, moved,
// Phi (integer atomics; their old values give the attributed km1 change),
// touched nets, block-weight deltas (slots), counters.
__global__ __launch_bounds__(kBlock) void k_apply_prefix(Seq S, const long long* best,
                                                         InstDesc D) {
  __shared__ unsigned long long s_dW[HG_MAX_K];
  __shared__ long long s_tmp2[kBlock / kWave];
  const int p = (int)best[1];
  if ((int)(blockIdx.x * kSeqTile) >= p) return;
  const int k = D.k;
  for (int i = threadIdx.x; i < k; i += kBlock) s_dW[i] = 0;
  __syncthreads();
  long long delta = 0, moved_pins = 0, approved = 0;
  for (int tile = blockIdx.x; tile * kSeqTile < p; tile += gridDim.x) {
    {
      const int j = tile * kSeqTile + threadIdx.x;
      int u, a, b;
      if (threadIdx.x < kSeqTile && j < p && seq_move(S, j, u, a, b)) {
        const long long cu = D.vwgt ? D.vwgt[u] : 1;
        atomicAdd(&s_dW[b], (unsigned long long)cu);
        atomicAdd(&s_dW[a], (unsigned long long)(-cu));
        approved += 1;
        moved_pins += D.vptr[u + 1] - D.vptr[u];
        if (D.moved) D.moved[u] = 1;
      }
    }
    // part is read by for_incidences (source blocks): update it only after
    for_incidences(S, p, tile, [&](int, int, int a, int b, int e) {
      const int oa = atomicSub(&D.phi[(long long)e * k + a], 1);
      const int ot = atomicAdd(&D.phi[(long long)e * k + b], 1);
      if (oa == 1 || ot == 0) {
        const int w = D.ewgt ? D.ewgt[e] : 1;
        if (oa == 1) delta += w;
        if (ot == 0) delta -= w;
      }
      D.touched[e] = 1;
    });
    {
      const int j = tile * kSeqTile + threadIdx.x;
      int u, a, b;
      if (threadIdx.x < kSeqTile && j < p && seq_move(S, j, u, a, b)) D.part[u] = b;
    }
  }
  __syncthreads();
  long long* my_dw = D.bw_slots + (size_t)(blockIdx.x % kSlots) * k;
  for (int i = threadIdx.x; i < k; i += kBlock)
    if (s_dW[i]) atomicAdd((unsigned long long*)&my_dw[i], s_dW[i]);
  delta = block_sum64(delta, s_tmp2);
  moved_pins = block_sum64(moved_pins, s_tmp2);
  approved = block_sum64(approved, s_tmp2);
  if (threadIdx.x == 0) {
    const int sl = blockIdx.x % kSlots;
    if (delta) atomicAdd(&D.ctr->slot[kCtrDeltaAttr][sl], (unsigned long long)delta);
    if (moved_pins) atomicAdd(&D.ctr->slot[kCtrMovedPins][sl], (unsigned long long)moved_pins);
    if (approved) atomicAdd(&D.ctr->slot[kCtrApproved][sl], (unsigned long long)approved);
  }
}

// Best balanced prefix of an explicit sequence (one workgroup, k <= 256):
// tiles of kBlock moves; thread i follows the weight of block i through the
// tile's moves in order and records when it crosses L_max; scans of those
// crossings and of the gains give, per prefix, the number of overloaded
// blocks and the total gain.  out[0] = total, out[1] = length.
__global__ __launch_bounds__(kBlock) void k_best_prefix_balanced(Seq S, long long lmax,
                                                                 const long long* block_w,
                                                                 const long long* gains,
                                                                 long long* out) {
  __shared__ int s_a[kBlock], s_b[kBlock], s_tr[kBlock];
  __shared__ long long s_c[kBlock];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ long long s_bv[kBlock / kWave];
  __shared__ int s_bp[kBlock / kWave];
  const int k = S.k, t = S.t, i = threadIdx.x;
  long long W = i < k ? block_w[i] : 0;
  long long over0, tmp;
  over0 = block_excl_scan64(i < k && W > lmax ? 1 : 0, s_tmp, &tmp);
  over0 = tmp;
  long long over = over0, total = 0, bv = 0;
  int bp = 0;
  for (int base = 0; base < t; base += kBlock) {
    const int j = base + i;
    int u = 0, a = -1, b = -1;
    long long c = 0;
    if (j < t && seq_move(S, j, u, a, b)) c = S.vwgt ? S.vwgt[u] : 1;
    s_a[i] = a;
    s_b[i] = b;
    s_c[i] = c;
    s_tr[i] = 0;
    __syncthreads();
    const int cnt = t - base < kBlock ? t - base : kBlock;
    if (i < k) {
      for (int q = 0; q < cnt; ++q) {
        if (s_a[q] == i) {
          const bool was = W > lmax;
          W -= s_c[q];
          if (was != (W > lmax)) atomicAdd(&s_tr[q], was ? -1 : 1);
        }
        if (s_b[q] == i) {
          const bool was = W > lmax;
          W += s_c[q];
          if (was != (W > lmax)) atomicAdd(&s_tr[q], was ? -1 : 1);
        }
      }
    }
    __syncthreads();
    const long long g = j < t ? gains[j] : 0;
    long long tg, tt;
    const long long gi = block_excl_scan64(g, s_tmp, &tg) + g;
    const long long oi = block_excl_scan64(s_tr[i], s_tmp, &tt) + s_tr[i];
    long long mv = LLONG_MIN;
    int mp = -1;
    if (j < t && over + oi == 0) {
      mv = total + gi;
      mp = j + 1;
    }
    // workgroup argmax of this tile
    const int lane = lane_id(), wv = i / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      const long long ov = __shfl_xor(mv, o);
      const int op = __shfl_xor(mp, o);
      if (better(ov, op, mv, mp)) {
        mv = ov;
        mp = op;
      }
    }
    if (lane == 0) {
      s_bv[wv] = mv;
      s_bp[wv] = mp;
    }
    __syncthreads();
    for (int w = 0; w < kBlock / kWave; ++w)
      if (s_bp[w] > 0 && better(s_bv[w], s_bp[w], bv, bp)) {
        bv = s_bv[w];
        bp = s_bp[w];
      }
    total += tg;
    over += tt;
    __syncthreads();
  }
  if (i == 0) {
    out[0] = bv;
    out[1] = bp;
  }
}

__global__ void k_copy_best(const long long* best, int* best_len, long long* best_gain) {
  if (threadIdx.x == 0) {
    if (best_len) *best_len = (int)best[1];
    if (best_gain) *best_gain = best[0];
  }
}

// ------------------------------------------------------------ rebalancing
// One synchronous rebalancing round (section "Rebalancing"): vertices of
// overloaded blocks pick their best feasible target from a gain cache; a
// stable sort orders the candidates by (gain desc, id asc), a second stable
// pass groups them by source block, and a segmented scan proposes, per
// source, the shortest prefix whose weight reaches the block's excess; the
// proposals, regrouped by target the same way, are approved as the longest
// prefix per target that fits under L_max, and applied.

struct Rb {
  const int* cache;            // gain cache of the round-start partition
  long long* excess;           // [k]: c(V_i) - L_max
  int* cnt_src;                // [k + 1]: candidates per source (sentinel k last)
  int* cnt_tgt;                // [k + 1]: proposals per target
  int* cnt_slots;              // [kSlots][k + 1]: per-workgroup-slot counts, summed into cnt
  unsigned char* prop;         // [n]: proposed this round
  int* mt;                     // [n]: target of sorted item i (own block: rejected)
  int* gord;                   // [n]: candidates in (gain desc, id asc) order
  long long* scan;             // [n]: exclusive prefix of item weights
  long long* csum;             // [chunks]
  long long* coff;             // [chunks]
  long long* best;             // [2]: {0, number of proposals}, the apply's sequence length
  unsigned bias;               // max incident weight: key = bias - gain >= 0
};

__global__ __launch_bounds__(kBlock) void k_rb_begin(InstDesc D, Rb R) {
  const int k = D.k;
  for (int i = threadIdx.x; i <= k; i += kBlock) {
    if (i < k) R.excess[i] = D.block_w[i] - D.lmax;
    R.cnt_src[i] = 0;
    R.cnt_tgt[i] = 0;
  }
  for (int i = threadIdx.x; i < kSlots * (k + 1); i += kBlock) R.cnt_slots[i] = 0;
  if (threadIdx.x == 0) {
    R.best[0] = 0;
    R.best[1] = D.n;
  }
}

// G lanes per vertex read its penalty row in 16-byte quads.  Every vertex
// gets defaults (not moved, not proposed, no candidate, key 0, value u);
// those of overloaded blocks look for the best block i != Pi(u) with
// c(V_i) + c(u) <= L_max by (p_i(u) asc = gain desc, c(V_i) asc, i asc).
template <int G>
__global__ __launch_bounds__(kBlock) void k_rb_select(InstDesc D, Rb R, unsigned* key, int* val) {
  __shared__ long long s_W[HG_MAX_K];
  __shared__ long long s_tmp[kBlock / kWave];
  const int k = D.k, n = D.n;
  const long long lmax = D.lmax;
  for (int i = threadIdx.x; i < k; i += kBlock) s_W[i] = D.block_w[i];
  __syncthreads();
  const int gl = threadIdx.x % G;
  constexpr int kPer = kBlock / G;
  const int Q = cache_stride(k) / 4;
  const int4* __restrict__ rows = (const int4*)(R.cache + cache_pbase(n));
  long long n_cons = 0, n_pins = 0, n_cand = 0;
  for (long long base = (long long)blockIdx.x * kPer; base < n; base += (long long)gridDim.x * kPer) {
    const long long u = base + threadIdx.x / G;
    if (u >= n) continue;
    if (gl == 0) {
      D.moved[u] = 0;
      R.prop[u] = 0;
      D.cand[u] = -1;
      key[u] = 0;
      val[u] = (int)u;
    }
    const int a = D.part[u];
    if ((unsigned)a >= (unsigned)k) {
      if (gl == 0) atomicOr(D.err_flags, kErrPart);
      continue;
    }
    if (s_W[a] <= lmax) continue;
    const long long cu = D.vwgt ? D.vwgt[u] : 1;
    int bp = 0, bi = -1;
    long long bw = 0;
    for (int q = gl; q < Q; q += G) {
      const int4 p4 = rows[u * Q + q];
      const int pv[4] = {p4.x, p4.y, p4.z, p4.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = q * 4 + j;
        if (i >= k || i == a) continue;
        const long long Wi = s_W[i];
        if (Wi + cu > lmax) continue;
        if (bi < 0 || pv[j] < bp || (pv[j] == bp && Wi < bw)) {
          bp = pv[j];
          bi = i;
          bw = Wi;
        }
      }
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
      const int op = __shfl_xor(bp, o, G), oi = __shfl_xor(bi, o, G);
      const long long ow = __shfl_xor(bw, o, G);
      if (oi >= 0 && (bi < 0 || op < bp || (op == bp && (ow < bw || (ow == bw && oi < bi))))) {
        bp = op;
        bi = oi;
        bw = ow;
      }
    }
    if (gl != 0) continue;
    n_cons += 1;
    n_pins += D.vptr[u + 1] - D.vptr[u];
    if (bi >= 0) {
      const int g = R.cache[u] - bp;
      D.cand[u] = pack_cand(g, bi);
      key[u] = R.bias - (unsigned)g;
      n_cand += 1;
    }
  }
  n_cons = block_sum64(n_cons, s_tmp);
  n_pins = block_sum64(n_pins, s_tmp);
  n_cand = block_sum64(n_cand, s_tmp);
  if (threadIdx.x == 0) {
    const int sl = blockIdx.x % kSlots;
    RoundCounters* ctr = D.ctr;
    if (n_cons) atomicAdd(&ctr->slot[kCtrEligible][sl], (unsigned long long)n_cons);
    if (n_pins) atomicAdd(&ctr->slot[kCtrActivePins][sl], (unsigned long long)n_pins);
    if (n_cand) atomicAdd(&ctr->slot[kCtrCandidates][sl], (unsigned long long)n_cand);
  }
}

// Regroup keys: item i of `order` gets key = source block (by_target = 0)
// or, for proposals, target block (by_target = 1); everything else the
// sentinel k.  Counts per key go to the count slots (k_rb_sum_counts).
__global__ __launch_bounds__(kBlock) void k_rb_keys(InstDesc D, Rb R, const int* order,
                                                    int by_target, unsigned* key_out,
                                                    int* val_out) {
  __shared__ int s_cnt[HG_MAX_K + 1];
  const int k = D.k;
  for (int i = threadIdx.x; i <= k; i += kBlock) s_cnt[i] = 0;
  __syncthreads();
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const bool live = i < D.n;
  int key = k;
  if (live) {
    const int u = order[i];
    const long long c = D.cand[u];
    if (!by_target) {
      R.gord[i] = u;
      if (c != -1) key = D.part[u];
    } else if (R.prop[u]) {
      key = (int)(c & 0xffffffffLL);
    }
    key_out[i] = (unsigned)key;
    val_out[i] = u;
  }
  // most lanes share a key (the sentinel above all): one LDS add per
  // distinct key and wavefront
  unsigned long long left = __ballot(live);
  while (left) {
    const int leader = __ffsll((long long)left) - 1;
    const int lk = __shfl(key, leader);
    const unsigned long long same = __ballot(live && key == lk);
    if (lane_id() == leader) atomicAdd(&s_cnt[lk], (int)__popcll(same));
    left &= ~same;
  }
  __syncthreads();
  // one of kSlots partial counts per workgroup (a single shared counter
  // would take every workgroup's atomic in turn)
  int* slot = R.cnt_slots + (blockIdx.x % kSlots) * (k + 1);
  for (int j = threadIdx.x; j <= k; j += kBlock)
    if (s_cnt[j]) atomicAdd(&slot[j], s_cnt[j]);
}

// cnt[j] = the sum of the slots' counts of key j; the slots are cleared for
// the next regrouping.  For the regrouping by target (set_len), the number
// of proposals (keys below the sentinel, sorted first) becomes the length of
// the sequence the apply walks.
__global__ __launch_bounds__(kBlock) void k_rb_sum_counts(InstDesc D, Rb R, int* cnt,
                                                          int set_len) {
  __shared__ long long s_tmp[kBlock / kWave];
  const int k = D.k;
  long long below = 0;
  for (int j = threadIdx.x; j <= k; j += kBlock) {
    int sum = 0;
    for (int q = 0; q < kSlots; ++q) {
      sum += R.cnt_slots[q * (k + 1) + j];
      R.cnt_slots[q * (k + 1) + j] = 0;
    }
    cnt[j] = sum;
    if (j < k) below += sum;
  }
  below = block_sum64(below, s_tmp);
  if (set_len && threadIdx.x == 0) R.best[1] = below;
}

// Items in sorted order with their weights: c(u) for items not keyed by
// the sentinel, else 0.
struct RbItems {
  const unsigned* key;
  const int* val;
  const int* vwgt;
  unsigned sentinel;
  int n;
};

__device__ __forceinline__ long long rb_weight(const RbItems& I, long long i) {
  if (i >= I.n || I.key[i] == I.sentinel) return 0;
  return I.vwgt ? I.vwgt[I.val[i]] : 1;
}

__global__ __launch_bounds__(kBlock) void k_rb_chunk_sums(RbItems I, long long* csum) {
  __shared__ long long s_tmp[kBlock / kWave];
  const long long v = rb_weight(I, (long long)blockIdx.x * kBlock + threadIdx.x);
  const long long tot = block_sum64(v, s_tmp);
  if (threadIdx.x == 0) csum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_rb_scan(RbItems I, const long long* coff,
                                                    long long* scan) {
  __shared__ long long s_tmp[kBlock / kWave];
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  long long tot;
  const long long ex = block_excl_scan64(rb_weight(I, i), s_tmp, &tot);
  if (i < I.n) scan[i] = coff[blockIdx.x] + ex;
}

// Start of every key's segment: exclusive scan of the counts (k + 1 <= 257
// entries, one workgroup).
__device__ void rb_segment_starts(const int* cnt, int k, long long* s_start, long long* s_tmp) {
  for (int b = 0; b <= k; b += kBlock) {
    const int i = b + threadIdx.x;
    long long tot;
    const long long ex = block_excl_scan64(i <= k ? cnt[i] : 0, s_tmp, &tot);
    if (i <= k) s_start[i] = ex + (b ? s_start[b - 1] + cnt[b - 1] : 0);
    __syncthreads();
  }
}

// Per source: propose the items whose weight before them (same source) is
// still below the excess.
__global__ __launch_bounds__(kBlock) void k_rb_propose(InstDesc D, Rb R, RbItems I) {
  __shared__ long long s_start[HG_MAX_K + 1];
  __shared__ long long s_tmp[kBlock / kWave];
  rb_segment_starts(R.cnt_src, D.k, s_start, s_tmp);
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  long long np = 0;
  if (i < I.n && I.key[i] != I.sentinel) {
    const int a = (int)I.key[i];
    const long long pre = R.scan[i] - R.scan[s_start[a]];
    if (pre < R.excess[a]) {
      R.prop[I.val[i]] = 1;
      np = 1;
    }
  }
  np = block_sum64(np, s_tmp);
  if (threadIdx.x == 0 && np)
    atomicAdd(&D.ctr->slot[kCtrBoundary][blockIdx.x % kSlots], (unsigned long long)np);
}

// Per target: approve the items that still fit; mt[i] = target, or the
// vertex's own block (a move the apply skips).
__global__ __launch_bounds__(kBlock) void k_rb_approve(InstDesc D, Rb R, RbItems I) {
  __shared__ long long s_start[HG_MAX_K + 1];
  __shared__ long long s_tmp[kBlock / kWave];
  rb_segment_starts(R.cnt_tgt, D.k, s_start, s_tmp);
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= I.n) return;
  const int u = I.val[i];
  int to = D.part[u];
  if (I.key[i] != I.sentinel) {
    const int t = (int)I.key[i];
    const long long cu = I.vwgt ? I.vwgt[u] : 1;
    const long long pre = R.scan[i] - R.scan[s_start[t]];
    if (D.block_w[t] + pre + cu <= D.lmax) to = t;
  }
  R.mt[i] = to;
}

}  // namespace

struct MovesLayoutBest {
  size_t best;
};

// ------------------------------------------------------------ host side

size_t moves_workspace_size(long long n, long long m, int k) { return moves_layout(n, m, k).total; }

MovesLayoutBest moves_best_slot(long long n, long long m, int k) {
  MovesLayoutBest b;
  b.best = moves_layout(n, m, k).best;
  return b;
}

static Seq make_seq(hg_graph_s* g, int k, char* ws, const MovesLayout& L, const int* part,
                    const int* phi, const int* mu, const int* mt, int t) {
  Seq S;
  memset(&S, 0, sizeof(S));
  S.mu = mu;
  S.mt = mt;
  S.t = t;
  S.part = part;
  S.phi = phi;
  S.vptr = g->vptr;
  S.vnets = g->vnets;
  S.ewgt = g->ewgt;
  S.vwgt = g->vwgt;
  S.n = g->n;
  S.k = k;
  S.cell = (int4*)(ws + L.cell);
  S.seen = (int*)(ws + L.seen);
  S.err_flags = (int*)(g->ws + g->lay.flags);
  return S;
}

static unsigned grid_of(long long items, int per) {
  long long b = (items + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_move_gains(hg_graph_s* g, int k, const int* part, const int* phi, int t,
                             const int* mu, const int* mt, long long* gains, char* ws,
                             hipStream_t s) {
  const MovesLayout L = moves_layout(g->n, g->m, k);
  Seq S = make_seq(g, k, ws, L, part, phi, mu, mt, t);
  const unsigned grid = grid_of(t, kBlock);
  // seen[] of the sequence's vertices starts at zero (the workspace may hold
  // anything), then the checks claim each vertex once
  hipLaunchKernelGGL(k_seq_clear, dim3(grid), dim3(kBlock), 0, s, S);
  hipLaunchKernelGGL(k_seq_check, dim3(grid), dim3(kBlock), 0, s, S);
  const unsigned tiles = grid_of(t, kSeqTile);
  hipLaunchKernelGGL(k_seq_init, dim3(tiles), dim3(kBlock), 0, s, S);
  hipLaunchKernelGGL(k_seq_collect, dim3(tiles), dim3(kBlock), 0, s, S);
  hipLaunchKernelGGL(k_seq_gains, dim3(tiles), dim3(kBlock), 0, s, S, gains, nullptr, nullptr,
                     nullptr);
  hipLaunchKernelGGL(k_seq_clear, dim3(grid), dim3(kBlock), 0, s, S);
  return hipGetLastError();
}

hipError_t launch_best_prefix(hg_graph_s* g, int k, long long lmax, const int* part,
                              const long long* block_w, int t, const int* mu, const int* mt,
                              const long long* gains, long long* out2, int* best_len,
                              long long* best_gain, hipStream_t s) {
  MovesLayout L;
  memset(&L, 0, sizeof(L));
  Seq S = make_seq(g, k, nullptr, L, part, nullptr, mu, mt, t);
  S.cell = nullptr;
  S.seen = nullptr;
  hipLaunchKernelGGL(k_best_prefix_balanced, dim3(1), dim3(kBlock), 0, s, S, lmax, block_w, gains,
                     out2);
  hipLaunchKernelGGL(k_copy_best, dim3(1), dim3(kWave), 0, s, out2, best_len, best_gain);
  return hipGetLastError();
}

// One monotone round of a single instance (see the file comment).  With
// marks_clear the caller knows the approval marks are all zero (a previous
// round of the same workspace cleared them).
hipError_t launch_round_exact(hg_graph_s* g, InstDesc d, int round, char* ws, bool marks_clear,
                              hipStream_t s) {
  const MovesLayout L = moves_layout(g->n, g->m, d.k);
  d.appr = (unsigned char*)(ws + L.appr);
  d.seq_cell = (int4*)(ws + L.cell);
  RoundPlan plan;
  single_round_plan(d, plan);
  hipError_t e = hipSuccess;
  if (!marks_clear) e = fill_u8(d.appr, 0, g->n, s);
  if (e == hipSuccess) e = launch_round_front(plan, s, nullptr);
  if (e != hipSuccess) return e;
  // the marked moves ordered by a stable radix sort of keys top - gain (gains
  // are at most the largest incident weight): 8-bit passes over the bits a
  // gain can occupy, the first one reading the marks and clearing them (the
  // count t lives on the device)
  const int n = g->n;
  const long long maxw = g->info.max_incident_weight;   // bounds every gain
  const bool one_pass = maxw < 255;
  int* tdev = (int*)(ws + L.tdev);
  int bits = 1;
  while (bits < 31 && (1ll << bits) <= maxw) ++bits;
  int cur = 0;
  for (int shift = 0; shift < (one_pass ? 8 : bits); shift += 8) {
    SortPass P;
    P.key_in = (const unsigned*)(ws + L.key[cur]);
    P.val_in = (const int*)(ws + L.val[cur]);
    P.key_out = (unsigned*)(ws + L.key[cur ^ 1]);
    P.val_out = (int*)(ws + L.val[cur ^ 1]);
    P.hist = (unsigned*)(ws + L.hist);
    P.dtot = (unsigned*)(ws + L.dtot);
    P.n = n;
    P.tiles = L.sort_tiles;
    P.shift = shift;
    if (shift == 0) {
      P.marks = d.appr;
      P.cand = d.cand;
      // keys 0x7fffffff - g differ from 0x7fffffff only in the low `bits` bits
      P.top = one_pass ? 254u : 0x7fffffffu;
      P.count_out = tdev;
    } else {
      P.n_dev = tdev;
    }
    sort_pass(P, s);
    cur ^= 1;
  }
  // exact gains of the sorted sequence (its cells were set empty by the
  // approval), best prefix, apply it
  Seq S = make_seq(g, d.k, ws, L, d.part, d.phi, (const int*)(ws + L.val[cur]), nullptr, 0);
  S.cand = d.cand;
  S.t_dev = tdev;
  long long* gains = (long long*)(ws + L.gains);
  long long* tsum = (long long*)(ws + L.tsum);
  long long* tbv = (long long*)(ws + L.tbest_v);
  int* tbi = (int*)(ws + L.tbest_i);
  long long* best = (long long*)(ws + L.best);
  // persistent grids: the kernels stride over the sequence's tiles, whose
  // count is known only on the device
  const unsigned tiles = std::min(grid_of(n, kSeqTile), (unsigned)kSeqGrid);
  hipLaunchKernelGGL(k_seq_collect, dim3(tiles), dim3(kBlock), 0, s, S);
  hipLaunchKernelGGL(k_seq_gains, dim3(tiles), dim3(kBlock), 0, s, S, gains, tsum, tbv, tbi);
  hipLaunchKernelGGL(k_prefix_pick, dim3(1), dim3(kBlock), 0, s, tdev, tsum, tbv, tbi, best);
  hipLaunchKernelGGL(k_apply_prefix, dim3(tiles), dim3(kBlock), 0, s, S, best, d);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_round_back(plan, round, s, nullptr);
}

// ------------------------------------------------------------ rebalancing

struct RebalLayout {
  size_t cache, key[2], val[2], gord, prop, mt, scan, csum, coff, excess, cnt_src, cnt_tgt,
      cnt_slots, best,
      hist, dtot, total;
  int sort_tiles, chunks;
};

static RebalLayout rebal_layout(long long n, int k) {
  RebalLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  L.sort_tiles = (int)((n + kSortTile - 1) / kSortTile);
  L.chunks = (int)((n + kBlock - 1) / kBlock);
  L.cache = take(4 * (size_t)(cache_pbase(n) + n * (long long)cache_stride(k)));
  for (int i = 0; i < 2; ++i) {
    L.key[i] = take(sizeof(unsigned) * (size_t)n);
    L.val[i] = take(sizeof(int) * (size_t)n);
  }
  L.gord = take(sizeof(int) * (size_t)n);
  L.prop = take((size_t)n);
  L.mt = take(sizeof(int) * (size_t)n);
  L.scan = take(sizeof(long long) * (size_t)n);
  L.csum = take(sizeof(long long) * (size_t)L.chunks);
  L.coff = take(sizeof(long long) * (size_t)L.chunks);
  L.excess = take(sizeof(long long) * HG_MAX_K);
  L.cnt_src = take(sizeof(int) * (HG_MAX_K + 1));
  L.cnt_tgt = take(sizeof(int) * (HG_MAX_K + 1));
  L.cnt_slots = take(sizeof(int) * kSlots * (HG_MAX_K + 1));
  L.best = take(sizeof(long long) * 2);
  L.hist = take(sizeof(unsigned) * (size_t)kDigits * L.sort_tiles);
  L.dtot = take(sizeof(unsigned) * kDigits);
  L.total = off;
  return L;
}

size_t rebalance_workspace_size(long long n, int k) { return rebal_layout(n, k).total; }

// One rebalancing round of a single instance (see the kernels' comment).
static hipError_t launch_rebalance_round(hg_graph_s* g, InstDesc d, char* ws, hipStream_t s) {
  const RebalLayout L = rebal_layout(g->n, d.k);
  const int n = g->n, k = d.k;
  Rb R;
  R.cache = (const int*)(ws + L.cache);
  R.excess = (long long*)(ws + L.excess);
  R.cnt_src = (int*)(ws + L.cnt_src);
  R.cnt_tgt = (int*)(ws + L.cnt_tgt);
  R.cnt_slots = (int*)(ws + L.cnt_slots);
  R.prop = (unsigned char*)(ws + L.prop);
  R.mt = (int*)(ws + L.mt);
  R.gord = (int*)(ws + L.gord);
  R.scan = (long long*)(ws + L.scan);
  R.csum = (long long*)(ws + L.csum);
  R.coff = (long long*)(ws + L.coff);
  R.best = (long long*)(ws + L.best);
  const long long maxw = g->info.max_incident_weight;   // |gain| <= maxw
  R.bias = (unsigned)maxw;
  unsigned* key[2] = {(unsigned*)(ws + L.key[0]), (unsigned*)(ws + L.key[1])};
  int* val[2] = {(int*)(ws + L.val[0]), (int*)(ws + L.val[1])};
  hipLaunchKernelGGL(k_rb_begin, dim3(1), dim3(kBlock), 0, s, d, R);
  hipError_t e = launch_gains(g, d, nullptr, nullptr, s, (int*)(ws + L.cache), 1);
  if (e != hipSuccess) return e;
  // candidates: lanes per vertex as the penalty row needs
  const int q = cache_stride(k) / 4;
  int G = 1;
  while (G < q && G < kWave) G <<= 1;
  typedef void (*SelK)(InstDesc, Rb, unsigned*, int*);
  SelK sel = G == 1    ? (SelK)k_rb_select<1>
             : G == 2  ? (SelK)k_rb_select<2>
             : G == 4  ? (SelK)k_rb_select<4>
             : G == 8  ? (SelK)k_rb_select<8>
             : G == 16 ? (SelK)k_rb_select<16>
             : G == 32 ? (SelK)k_rb_select<32>
                       : (SelK)k_rb_select<64>;
  long long sg = ((long long)n + kBlock / G - 1) / (kBlock / G);
  if (sg > 4096) sg = 4096;
  hipLaunchKernelGGL(sel, dim3((unsigned)sg), dim3(kBlock), 0, s, d, R, key[0], val[0]);
  int cur = 0;
  auto pass = [&](int shift) {
    SortPass P;
    P.key_in = key[cur];
    P.val_in = val[cur];
    P.key_out = key[cur ^ 1];
    P.val_out = val[cur ^ 1];
    P.hist = (unsigned*)(ws + L.hist);
    P.dtot = (unsigned*)(ws + L.dtot);
    P.n = n;
    P.tiles = L.sort_tiles;
    P.shift = shift;
    sort_pass(P, s);
    cur ^= 1;
  };
  // (gain desc, id asc): keys bias - gain lie in [0, 2 * bias]
  int bits = 1;
  while (bits < 32 && (1ull << bits) <= 2ull * (unsigned long long)maxw) ++bits;
  for (int shift = 0; shift < bits; shift += 8) pass(shift);
  const int kbits = k < 256 ? 8 : 16;   // block keys 0..k, the sentinel k included
  const unsigned grid = grid_of(n, kBlock);
  auto scan = [&](const RbItems& I) {
    hipLaunchKernelGGL(k_rb_chunk_sums, dim3(L.chunks), dim3(kBlock), 0, s, I, R.csum);
    hipLaunchKernelGGL(k_prefix_top, dim3(1), dim3(kBlock), 0, s, R.csum, R.coff, L.chunks);
    hipLaunchKernelGGL(k_rb_scan, dim3(L.chunks), dim3(kBlock), 0, s, I, R.coff, R.scan);
  };
  // by source block, proposals per source
  hipLaunchKernelGGL(k_rb_keys, dim3(grid), dim3(kBlock), 0, s, d, R, val[cur], 0, key[cur ^ 1],
                     val[cur ^ 1]);
  hipLaunchKernelGGL(k_rb_sum_counts, dim3(1), dim3(kBlock), 0, s, d, R, R.cnt_src, 0);
  cur ^= 1;
  for (int shift = 0; shift < kbits; shift += 8) pass(shift);
  RbItems I;
  I.vwgt = g->vwgt;
  I.sentinel = (unsigned)k;
  I.n = n;
  I.key = key[cur];
  I.val = val[cur];
  scan(I);
  hipLaunchKernelGGL(k_rb_propose, dim3(grid), dim3(kBlock), 0, s, d, R, I);
  // proposals by target block, approvals per target
  hipLaunchKernelGGL(k_rb_keys, dim3(grid), dim3(kBlock), 0, s, d, R, R.gord, 1, key[cur ^ 1],
                     val[cur ^ 1]);
  hipLaunchKernelGGL(k_rb_sum_counts, dim3(1), dim3(kBlock), 0, s, d, R, R.cnt_tgt, 1);
  cur ^= 1;
  for (int shift = 0; shift < kbits; shift += 8) pass(shift);
  I.key = key[cur];
  I.val = val[cur];
  scan(I);
  hipLaunchKernelGGL(k_rb_approve, dim3(grid), dim3(kBlock), 0, s, d, R, I);
  // apply the approved moves (the others carry their own block as target)
  Seq S;
  memset(&S, 0, sizeof(S));
  S.mu = val[cur];
  S.mt = R.mt;
  S.t = n;
  S.part = d.part;
  S.phi = d.phi;
  S.vptr = g->vptr;
  S.vnets = g->vnets;
  S.ewgt = g->ewgt;
  S.vwgt = g->vwgt;
  S.n = n;
  S.k = k;
  S.err_flags = d.err_flags;
  hipLaunchKernelGGL(k_apply_prefix, dim3(grid_of(n, kSeqTile)), dim3(kBlock), 0, s, S,
                     (const long long*)R.best, d);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  RoundPlan plan;
  single_round_plan(d, plan);
  e = launch_round_finalize(plan, s, nullptr);
  if (e != hipSuccess) return e;
  return launch_round_stats(plan, 0, s, nullptr);
}

}  // namespace hg

using hg::check_k;
using hg::fail;

extern "C" {

size_t hg_moves_workspace_size(int32_t n, int32_t m, int32_t k) {
  if (n < 1 || m < 1 || k < 2 || k > HG_MAX_K) return 0;
  return hg::moves_workspace_size(n, m, k);
}

static hg_status check_moves_ws(hg_graph g, int k, void* ws, size_t ws_bytes) {
  const size_t need = hg::moves_workspace_size(g->n, g->m, k);
  if (!ws || ws_bytes < need)
    return fail(HG_ERR_WORKSPACE, "move workspace needs %zu bytes (got %zu)", need, ws_bytes);
  return HG_OK;
}

hg_status hg_move_gains(hg_graph g, int32_t k, const int32_t* part, const int32_t* phi,
                        int32_t t, const int32_t* move_u, const int32_t* move_to,
                        int64_t* gains, void* workspace, size_t ws_bytes, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (t < 0 || t > g->n) return fail(HG_ERR_INVALID, "t must lie in [0, n]");
  if (t == 0) return HG_OK;
  if (!part || !phi || !move_u || !move_to || !gains)
    return fail(HG_ERR_INVALID, "part, phi, move_u, move_to and gains must be non-NULL");
  st = check_moves_ws(g, k, workspace, ws_bytes);
  if (st != HG_OK) return st;
  HG_TRY(hg::launch_move_gains(g, k, part, phi, t, move_u, move_to, (long long*)gains,
                               (char*)workspace, (hipStream_t)stream),
         "move gains");
  return HG_OK;
}

hg_status hg_best_prefix(hg_graph g, int32_t k, int64_t max_block_w, const int32_t* part,
                         const int64_t* block_w, int32_t t, const int32_t* move_u,
                         const int32_t* move_to, const int64_t* gains, int32_t* best_len,
                         int64_t* best_gain, void* workspace, size_t ws_bytes, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (t < 0 || t > g->n) return fail(HG_ERR_INVALID, "t must lie in [0, n]");
  if (!part || !block_w || (t > 0 && (!move_u || !move_to || !gains)) || !best_len || !best_gain)
    return fail(HG_ERR_INVALID, "part, block_w, the moves, gains, best_len and best_gain must be "
                                "non-NULL");
  st = check_moves_ws(g, k, workspace, ws_bytes);
  if (st != HG_OK) return st;
  const hg::MovesLayoutBest lb = hg::moves_best_slot(g->n, g->m, k);
  HG_TRY(hg::launch_best_prefix(g, k, max_block_w, part, (const long long*)block_w, t, move_u,
                                move_to, (const long long*)gains,
                                (long long*)((char*)workspace + lb.best), best_len,
                                (long long*)best_gain, (hipStream_t)stream),
         "best prefix");
  return HG_OK;
}

hg_status hg_lp_round_exact(hg_graph g, int32_t k, int64_t max_block_w, int32_t* part,
                            int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                            uint8_t* moved, int64_t* km1, hg_round_stats* stats, void* workspace,
                            size_t ws_bytes, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!part || !phi || !netstate || !block_w || !eligible || !km1 || !stats)
    return fail(HG_ERR_INVALID,
                "part, phi, netstate, block_w, eligible, km1 and stats must be non-NULL");
  if (max_block_w < 0) return fail(HG_ERR_INVALID, "max_block_w must be >= 0");
  st = check_moves_ws(g, k, workspace, ws_bytes);
  if (st != HG_OK) return st;
  hg::InstDesc d = hg::make_desc(g, k, max_block_w, part, phi, netstate, (long long*)block_w,
                                 eligible, moved, (long long*)km1, stats);
  HG_TRY(hg::launch_round_exact(g, d, 0, (char*)workspace, false, (hipStream_t)stream),
         "monotone round");
  return HG_OK;
}

hg_status hg_refine_exact(hg_graph g, int32_t k, double eps, int32_t rounds, int32_t* part,
                          int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                          hg_round_stats* stats, int64_t* km1_out, void* workspace,
                          size_t ws_bytes, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (!(eps > 0.0 && eps < 1.0)) return fail(HG_ERR_INVALID, "eps must lie in (0, 1)");
  if (rounds < 0) return fail(HG_ERR_INVALID, "rounds must be >= 0");
  if (!part || !phi || !netstate || !block_w || !eligible || !km1_out || (rounds > 0 && !stats))
    return fail(HG_ERR_INVALID, "part, phi, netstate, block_w, eligible, stats and km1_out must "
                                "be non-NULL");
  st = check_moves_ws(g, k, workspace, ws_bytes);
  if (st != HG_OK) return st;
  const long long lmax = hg_max_block_weight(g, k, eps);
  hipStream_t s = (hipStream_t)stream;
  hg::InstDesc d = hg::make_desc(g, k, lmax, part, phi, netstate, (long long*)block_w, eligible,
                                 nullptr, (long long*)km1_out, stats);
  hg::CountPlan cplan;
  hg::single_count_plan(d, cplan);
  HG_TRY(hg::launch_counts(cplan, true, true, s), "pin counts");
  for (int r = 0; r < rounds; ++r) {
    d.stats = stats + r;
    // every round after the first finds the marks cleared by its predecessor
    HG_TRY(hg::launch_round_exact(g, d, 0, (char*)workspace, r > 0, s), "monotone round");
  }
  return HG_OK;
}


size_t hg_rebalance_workspace_size(int32_t n, int32_t k) {
  if (n < 1 || k < 2 || k > HG_MAX_K) return 0;
  return hg::rebalance_workspace_size(n, k);
}

hg_status hg_rebalance(hg_graph g, int32_t k, int64_t max_block_w, int32_t rounds, int32_t* part,
                       int32_t* phi, uint32_t* netstate, int64_t* block_w, uint8_t* eligible,
                       uint8_t* moved, int64_t* km1, hg_round_stats* stats, void* workspace,
                       size_t ws_bytes, void* stream) {
  hg_status st = check_k(g, k);
  if (st != HG_OK) return st;
  if (rounds < 0) return fail(HG_ERR_INVALID, "rounds must be >= 0");
  if (max_block_w < 0) return fail(HG_ERR_INVALID, "max_block_w must be >= 0");
  if (!part || !phi || !netstate || !block_w || !eligible || !moved || !km1 ||
      (rounds > 0 && !stats))
    return fail(HG_ERR_INVALID, "part, phi, netstate, block_w, eligible, moved, km1 and stats "
                                "must be non-NULL");
  const size_t need = hg::rebalance_workspace_size(g->n, k);
  if (!workspace || ws_bytes < need)
    return fail(HG_ERR_WORKSPACE, "rebalance workspace needs %zu bytes (got %zu)", need, ws_bytes);
  if (((uintptr_t)workspace & 255) != 0)
    return fail(HG_ERR_INVALID, "the rebalance workspace must be 256-byte aligned");
  hg::InstDesc d = hg::make_desc(g, k, max_block_w, part, phi, netstate, (long long*)block_w,
                                 eligible, moved, (long long*)km1, stats);
  for (int r = 0; r < rounds; ++r) {
    d.stats = stats + r;
    HG_TRY(hg::launch_rebalance_round(g, d, (char*)workspace, (hipStream_t)stream),
           "rebalance round");
  }
  return HG_OK;
}

}  // extern "C"
