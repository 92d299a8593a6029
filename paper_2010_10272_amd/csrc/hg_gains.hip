// hg_gains.hip -- all k-way move gains g_i(u) = b(u) - p_i(u) (section
// "Parallel Gain Calculation"), for every vertex and block.
//
// With conn_i = w({e in I(u) : i in Lambda(e)}) one has p_i(u) = w(I(u)) -
// conn_i, so a sweep over I(u) that reads each net once (w, Lambda, and the
// S bit of Pi(u) for b(u)) gives the whole row.  Light vertices (w(I(u)) <=
// 255) keep the k counters bit-sliced in registers, one thread per vertex;
// heavy vertices use one wavefront each with LDS counters.
#include "hg_bits.h"
#include "hg_device.h"
#include "hg_internal.h"
#include "hg_lp.h"
#include "hg_sweep.h"

namespace hg {

// Unit: a chunk of 256 vertices (single instance: blockIdx, XCD-remapped).
// Row u of `gains` (k int64) and benefit[u] are written.
// With `cache` set, the sweeps fill a gain cache instead (subsection "Gain
// Caching"): b(u), w(I(u)) and the row p_i(u) = w(I(u)) - conn_i (0 for the
// own block), laid out as cache_pbase / cache_stride say.  With only_over
// set, only vertices of blocks heavier than L_max are filled (the rows the
// rebalancer reads).
// Staged output of a wavefront's gain rows (k a multiple of S): the lanes
// put S gains of their own rows into LDS, then write them out as 64 rows of
// S * 8 contiguous bytes, S / 2 lanes per row, so that every store covers
// whole cache lines (S = 16: one line) instead of touching 64 rows at once.
// The stores are nontemporal: the rows are not read again by this pass.
constexpr int kStageMax = 16;

template <int S, int WK>
__device__ __forceinline__ void write_rows_staged(long long (*stage)[kStageMax + 1],
                                                  long long* __restrict__ gains, int k,
                                                  long long row0, unsigned long long mine,
                                                  bool have, int a, long long base,
                                                  const BitCounters<WK>& C) {
  const int lane = lane_id();
#pragma unroll
  for (int w = 0; w < WK; ++w) {
#pragma unroll
    for (int h = 0; h < 32; h += S) {
      const int c0 = w * 32 + h;
      if (c0 >= k) break;                              // k is a multiple of S
      if (have) {
#pragma unroll
        for (int x = 0; x < S; ++x) stage[lane][x] = c0 + x == a ? 0 : base + C.value(w, h + x);
      }
      wave_lds_sync();
#pragma unroll
      for (int p0 = 0; p0 < S / 2; ++p0) {
        const int p = p0 * kWave + lane;
        const int r = p / (S / 2), piece = p % (S / 2);
        if ((mine >> r) & 1ull) {
          const i64x2 v = {stage[r][2 * piece], stage[r][2 * piece + 1]};
          __builtin_nontemporal_store(
              v, reinterpret_cast<i64x2*>(gains + (row0 + r) * k + c0 + 2 * piece));
        }
      }
      wave_lds_sync();
    }
  }
}

template <int WK, int VIEW>
__global__ __launch_bounds__(kBlock) void k_gains_light(Launch L, long long* __restrict__ gains,
                                                        long long* __restrict__ benefit,
                                                        int* __restrict__ cache, int only_over) {
  // rows of a multiple of 8 blocks leave through LDS (write_rows_staged)
  __shared__ long long s_stage[kBlock / kWave][kWave][kStageMax + 1];
  WorkItem fb;
  fb.inst = 0;
  fb.first = (int)xcd_remap(blockIdx.x, gridDim.x);
  fb.count = 1;
  fb.stride = 1;
  const WorkItem wi = work_item(L, fb);
  const InstDesc D = inst_desc(L, wi.inst);
  const int k = D.k;
  const long long u = (long long)wi.first * kBlock + threadIdx.x;
  const bool staged = !cache && gains && k % 8 == 0;
  // done: nothing to compute for this lane (out of range, invalid block, or
  // a block within L_max when only overloaded blocks are asked for);
  // have: this lane's row was computed here (a light vertex)
  bool done = false, have = false;
  int a = 0, tot = 0, ben = 0;
  BitCounters<WK> C;
  C.clear();
  if (u < D.n) {
    a = D.part[u];
    if ((unsigned)a >= (unsigned)k) {
      atomicOr(D.err_flags, kErrPart);
      if (!cache) {
        long long* row = gains + u * k;
        for (int i = 0; i < k; ++i) row[i] = 0;
        if (benefit) benefit[u] = 0;
      }
      done = true;
    } else if (only_over && D.block_w[a] <= D.lmax) {
      done = true;
    }
  } else {
    done = true;
  }
  if (!done) {
    const long long b0 = D.vptr[u], b1 = D.vptr[u + 1];
    if (b1 - b0 <= kLightLimit) {                    // longer rows: the heavy kernel
      const int aw = a >> 5;
      const unsigned abit = 1u << (a & 31);
      bool heavy = false;
      for (long long j = b0; j < b1 && !heavy; j += kUnroll) {
        unsigned w[kUnroll], S[kUnroll], Lb[kUnroll][WK];
        bool cut[kUnroll];
        int e[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) e[q] = global_ptr(D.vnets)[j + q < b1 ? j + q : j];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q)
          read_net<WK, VIEW>(D.netstate, D.rw, D.view_ptr, e[q], aw, w[q], cut[q], Lb[q], S[q]);
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
          if (j + q >= b1) {             // past the row end: a repeated slot, masked
            w[q] = 0;
            S[q] = 0;
#pragma unroll
            for (int x = 0; x < WK; ++x) Lb[q][x] = 0;
          }
        }
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
          tot += (int)w[q];
          if (S[q] & abit) ben += (int)w[q];
        }
        if (tot > kLightLimit) {
          heavy = true;                   // heavier rows: the heavy kernel
          break;
        }
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
          if constexpr (VIEW != kViewFull) {
            C.add_one(Lb[q]);             // unit nets (masked slots add nothing)
          } else if (w[q]) {
            C.add(Lb[q], w[q]);
          }
        }
      }
      have = !heavy;
    }
  }
  if (have && cache) {
    const long long n = D.n;
    cache[u] = ben;
    cache[n + u] = tot;
    int* prow = cache + cache_pbase(n) + (long long)u * cache_stride(k);
#pragma unroll
    for (int w = 0; w < WK; ++w)
      for (int b = 0; b < 32; ++b) {
        const int i = w * 32 + b;
        if (i >= k) break;
        prow[i] = tot - (int)C.value(w, b);
      }
  }
  if (cache) return;
  const long long base = (long long)ben - tot;
  if (have && benefit) benefit[u] = ben;
  if (!staged) {
    if (!have) return;
    long long* row = gains + u * k;
#pragma unroll
    for (int w = 0; w < WK; ++w) {
      for (int b = 0; b < 32; b += 2) {
        const int i = w * 32 + b;
        if (i >= k) break;
        long long g0 = i == a ? 0 : base + C.value(w, b);
        if (i + 1 < k) {
          long long g1 = i + 1 == a ? 0 : base + C.value(w, b + 1);
          if ((k & 1) == 0) {
            *reinterpret_cast<longlong2*>(row + i) = make_longlong2(g0, g1);
          } else {
            row[i] = g0;
            row[i + 1] = g1;
          }
        } else {
          row[i] = g0;
        }
      }
    }
    return;
  }
  // staged rows: every lane of the wavefront takes part, writing only the
  // rows whose lane computed them
  const unsigned long long mine = __ballot(have);
  const long long row0 = u - lane_id();             // the wavefront's first vertex
  long long(*stage)[kStageMax + 1] = s_stage[threadIdx.x / kWave];
  if (k % 16 == 0)
    write_rows_staged<16, WK>(stage, gains, k, row0, mine, have, a, base, C);
  else
    write_rows_staged<8, WK>(stage, gains, k, row0, mine, have, a, base, C);
}

// Unit: 4 consecutive heavy-list entries (one per wavefront).
__global__ __launch_bounds__(kBlock) void k_gains_heavy(Launch L, long long* __restrict__ gains,
                                                        long long* __restrict__ benefit,
                                                        int* __restrict__ cache, int only_over) {
  __shared__ int s_conn[kBlock / kWave][HG_MAX_K];
  WorkItem fb;
  fb.inst = 0;
  fb.first = blockIdx.x;
  fb.count = 1;
  fb.stride = 1;
  const WorkItem wi = work_item(L, fb);
  const InstDesc D = inst_desc(L, wi.inst);
  const int k = D.k;
  const int wv = threadIdx.x / kWave, lane = lane_id();
  const long long idx = (long long)wi.first * (kBlock / kWave) + wv;
  if (idx >= D.heavy_count) return;
  const int u = D.heavy_list[idx];
  const int a = D.part[u];
  if ((unsigned)a >= (unsigned)k) return;           // flagged and zeroed by the light kernel
  if (only_over && D.block_w[a] <= D.lmax) return;
  int* conn = s_conn[wv];
  for (int i = lane; i < k; i += kWave) conn[i] = 0;
  wave_lds_sync();
  const int wk = bit_words(k);
  const long long b0 = D.vptr[u], b1 = D.vptr[u + 1];
  int tot = 0, ben = 0;
  for (long long j = b0 + lane; j < b1; j += kWave) {
    const unsigned* r = D.netstate + (long long)D.vnets[j] * D.rw;
    const int w = (int)r[0];
    tot += w;
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
  if (cache) {
    const long long n = D.n;
    int* prow = cache + cache_pbase(n) + (long long)u * cache_stride(k);
    for (int i = lane; i < k; i += kWave) prow[i] = tot - conn[i];
    if (lane == 0) {
      cache[u] = ben;
      cache[n + u] = tot;
    }
    return;
  }
  long long* row = gains + (long long)u * k;
  for (int i = lane; i < k; i += kWave)
    row[i] = i == a ? 0 : (long long)ben - tot + conn[i];
  if (lane == 0 && benefit) benefit[u] = ben;
}

GainsKernel gains_kernel(int k, int view) {
  typedef void (*K)(Launch, long long*, long long*, int*, int);
  K kern;
  switch (view) {
    case kView16: kern = k_gains_light<1, kView16>; break;
    case kView32: kern = k_gains_light<1, kView32>; break;
    case kView64: kern = k_gains_light<2, kView64>; break;
    default:
      switch (bit_words(k)) {
        case 1: kern = k_gains_light<1, kViewFull>; break;
        case 2: kern = k_gains_light<2, kViewFull>; break;
        case 4: kern = k_gains_light<4, kViewFull>; break;
        default: kern = k_gains_light<8, kViewFull>; break;
      }
  }
  return (GainsKernel)(void*)kern;
}

hipError_t launch_gains(hg_graph_s* g, const InstDesc& d, long long* gains, long long* benefit,
                        hipStream_t s, int* cache, int only_over) {
  typedef void (*K)(Launch, long long*, long long*, int*, int);
  const Launch L = single_launch(d);
  unsigned grid = (unsigned)(((long long)d.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((K)(void*)gains_kernel(d.k, d.view), dim3(grid), dim3(kBlock), 0, s, L,
                     gains, benefit, cache, only_over);
  if (d.heavy_count > 0) {
    unsigned hg = (unsigned)((d.heavy_count + (kBlock / kWave) - 1) / (kBlock / kWave));
    hipLaunchKernelGGL(k_gains_heavy, dim3(hg), dim3(kBlock), 0, s, L, gains, benefit, cache,
                       only_over);
  }
  (void)g;
  return hipGetLastError();
}

}  // namespace hg
