// hg_gains.hip -- all k-way move gains g_i(u) = b(u) - p_i(u) (section
// "Parallel Gain Calculation"), for every vertex and block.
//
// With conn_i = w({e in I(u) : i in Lambda(e)}) one has p_i(u) = w(I(u)) -
// conn_i, so a sweep over I(u) that reads each net record once (w, Lambda,
// and the S bit of Pi(u) for b(u)) gives the whole row.  Light vertices
// (w(I(u)) <= 255) keep the k counters bit-sliced in registers, one thread
// per vertex; heavy vertices use one wavefront each with LDS counters.
#include "hg_bits.h"
#include "hg_device.h"
#include "hg_internal.h"
#include "hg_sweep.h"

namespace hg {

template <int WK, int VIEW>
__global__ __launch_bounds__(kBlock) void k_gains_light(
    int n, int k, int rw, const long long* __restrict__ vptr, const int* __restrict__ vnets,
    const int* __restrict__ part, const unsigned* __restrict__ netstate,
    const unsigned* __restrict__ view,
    long long* __restrict__ gains, long long* __restrict__ benefit, int* __restrict__ err_flags) {
  const unsigned lb = xcd_remap(blockIdx.x, gridDim.x);
  const long long u = (long long)lb * kBlock + threadIdx.x;
  if (u >= n) return;
  const int a = part[u];
  long long* row = gains + u * k;
  if ((unsigned)a >= (unsigned)k) {
    atomicOr(err_flags, kErrPart);
    for (int i = 0; i < k; ++i) row[i] = 0;
    if (benefit) benefit[u] = 0;
    return;
  }
  const long long b0 = vptr[u], b1 = vptr[u + 1];
  if (b1 - b0 > kLightLimit) return;                 // heavy: other kernel
  BitCounters<WK> C;
  C.clear();
  int tot = 0, ben = 0;
  const int aw = a >> 5;
  const unsigned abit = 1u << (a & 31);
  for (long long j = b0; j < b1; j += kUnroll) {
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
        S[q] = 0;
#pragma unroll
        for (int x = 0; x < WK; ++x) L[q][x] = 0;
      }
    }
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      tot += (int)w[q];
      if (S[q] & abit) ben += (int)w[q];
    }
    if (tot > kLightLimit) return;                  // heavy: other kernel
#pragma unroll
    for (int q = 0; q < kUnroll; ++q)
      if (w[q]) C.add(L[q], w[q]);
  }
  const long long base = (long long)ben - tot;
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
  if (benefit) benefit[u] = ben;
}

__global__ __launch_bounds__(kBlock) void k_gains_heavy(
    int heavy_count, int k, int rw, const int* __restrict__ heavy_list,
    const long long* __restrict__ vptr, const int* __restrict__ vnets,
    const int* __restrict__ part, const unsigned* __restrict__ netstate,
    long long* __restrict__ gains, long long* __restrict__ benefit) {
  __shared__ int s_conn[kBlock / kWave][HG_MAX_K];
  const int wv = threadIdx.x / kWave, lane = lane_id();
  const long long idx = (long long)blockIdx.x * (kBlock / kWave) + wv;
  if (idx >= heavy_count) return;
  const int u = heavy_list[idx];
  const int a = part[u];
  if ((unsigned)a >= (unsigned)k) return;           // flagged and zeroed by the light kernel
  int* conn = s_conn[wv];
  for (int i = lane; i < k; i += kWave) conn[i] = 0;
  wave_lds_sync();
  const int wk = bit_words(k);
  const long long b0 = vptr[u], b1 = vptr[u + 1];
  int tot = 0, ben = 0;
  for (long long j = b0 + lane; j < b1; j += kWave) {
    const unsigned* r = netstate + (long long)vnets[j] * rw;
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
  long long* row = gains + (long long)u * k;
  for (int i = lane; i < k; i += kWave)
    row[i] = i == a ? 0 : (long long)ben - tot + conn[i];
  if (lane == 0 && benefit) benefit[u] = ben;
}

template <int WK>
static void launch_light(hg_graph_s* g, int k, const int* part, const unsigned* netstate,
                         long long* gains, long long* benefit, hipStream_t s) {
  unsigned grid = (unsigned)(((long long)g->n + kBlock - 1) / kBlock);
  const unsigned* view = netstate + (size_t)g->m * net_words(k);
  auto kern = k_gains_light<WK, kViewFull>;
  switch (net_view(k, g->unit_nets)) {
    case kView16: kern = k_gains_light<1, kView16>; break;
    case kView32: kern = k_gains_light<1, kView32>; break;
    case kView64: kern = k_gains_light<2, kView64>; break;
    default: break;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, g->n, k, net_words(k), g->vptr,
                     g->vnets, part, netstate, view, gains, benefit,
                     (int*)(g->ws + g->lay.flags));
}

hipError_t launch_gains(hg_graph_s* g, int k, const int* part, const unsigned* netstate,
                        long long* gains, long long* benefit, hipStream_t s) {
  switch (bit_words(k)) {
    case 1: launch_light<1>(g, k, part, netstate, gains, benefit, s); break;
    case 2: launch_light<2>(g, k, part, netstate, gains, benefit, s); break;
    case 4: launch_light<4>(g, k, part, netstate, gains, benefit, s); break;
    default: launch_light<8>(g, k, part, netstate, gains, benefit, s); break;
  }
  const int heavy = g->info.heavy_count;
  if (heavy > 0) {
    unsigned grid = (unsigned)((heavy + (kBlock / kWave) - 1) / (kBlock / kWave));
    hipLaunchKernelGGL(k_gains_heavy, dim3(grid), dim3(kBlock), 0, s, heavy, k, net_words(k),
                       (const int*)(g->ws + g->lay.heavy), g->vptr, g->vnets, part, netstate,
                       gains, benefit);
  }
  return hipGetLastError();
}

}  // namespace hg
