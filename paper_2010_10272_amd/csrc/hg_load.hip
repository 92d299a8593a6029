// hg_load.hip -- input checks, incidence CSR (transpose of the net CSR) and
// static per-vertex facts.  Runs once per loaded hypergraph.
//
// The paper stores a hypergraph as two adjacency arrays, the pins of each net
// and the incident nets of each vertex (section "Coarsening", subsection
// "Contraction").  Here the second array is built on the device: degree count
// (integer atomics), exclusive scan, scatter, then every row is sorted so that
// I(v) lists nets in increasing id and the result does not depend on the
// order in which the scatter's atomics happened.
#include "hg_device.h"
#include "hg_internal.h"
#include "hg_sort.h"

namespace hg {

// ------------------------------------------------------------------ fills
__global__ void k_fill_i64(long long* p, long long v, long long count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}
__global__ void k_fill_i32(int* p, int v, long long count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}
__global__ void k_fill_u8(unsigned char* p, unsigned char v, long long count) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

static unsigned grid_for(long long count, int per_thread = 1) {
  long long blocks = (count + (long long)kBlock * per_thread - 1) / ((long long)kBlock * per_thread);
  if (blocks < 1) blocks = 1;
  if (blocks > 65536) blocks = 65536;
  return (unsigned)blocks;
}

hipError_t fill_i64(long long* p, long long v, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(count)), dim3(kBlock), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t fill_i32(int* p, int v, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count)), dim3(kBlock), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t fill_u8(unsigned char* p, unsigned char v, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(count)), dim3(kBlock), 0, s, p, v, count);
  return hipGetLastError();
}

// ------------------------------------------------------------------ checks
// Load-time checks run on a capped grid and reduce per workgroup, so that
// each shared LoadInfo field takes at most one atomic per workgroup.
constexpr int kLoadGrid = 1024;

__device__ __forceinline__ int block_max_int(int v, int* s_tmp) {
  v = wave_max(v);
  __syncthreads();
  if (lane_id() == 0) s_tmp[threadIdx.x / kWave] = v;
  __syncthreads();
  int r = s_tmp[0];
  for (int i = 1; i < kBlock / kWave; ++i) r = s_tmp[i] > r ? s_tmp[i] : r;
  return r;
}

// Nets: increasing offsets with fixed ends (no empty net), positive weights.
__global__ __launch_bounds__(kBlock) void k_check_nets(int m, long long P,
                                                       const long long* eptr, const int* ewgt,
                                                       LoadInfo* info) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_imax[kBlock / kWave];
  int err = 0, size = 0;
  long long wsum = 0;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < m; e += stride) {
    const long long s = eptr[e], t = eptr[e + 1];
    if (e == 0 && s != 0) err |= kErrCsr;
    if (e == m - 1 && t != P) err |= kErrCsr;
    if (t <= s || s < 0 || t > P) err |= kErrCsr;
    else if (t - s > size) size = (int)((t - s) > 0x7fffffffLL ? 0x7fffffff : (t - s));
    const long long w = ewgt ? ewgt[e] : 1;
    if (w <= 0) err |= kErrWeight;
    else wsum += w;
  }
  if (err) atomicOr(&info->err, err);
  const int mx = block_max_int(size, s_imax);
  const long long ws = block_sum64(wsum, s_tmp);
  if (threadIdx.x == 0) {
    atomicMax(&info->max_net_size, mx);
    atomicAdd(&info->total_net_weight, (unsigned long long)ws);
  }
}

__global__ __launch_bounds__(kBlock) void k_check_pins(int n, long long P, const int* pins,
                                                       LoadInfo* info) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  int err = 0;
  for (; i < P; i += stride) {
    int v = pins[i];
    if (v < 0 || v >= n) err = kErrPin;
  }
  if (err) atomicOr(&info->err, err);
}

__global__ __launch_bounds__(kBlock) void k_check_vertices(int n, const int* vwgt,
                                                           LoadInfo* info) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_imax[kBlock / kWave];
  int err = 0, cmax = 0;
  long long csum = 0;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
    const long long c = vwgt ? vwgt[v] : 1;
    if (c <= 0) {
      err = kErrWeight;
    } else {
      csum += c;
      if (c > cmax) cmax = (int)c;
    }
  }
  if (err) atomicOr(&info->err, err);
  const int mx = block_max_int(cmax, s_imax);
  const long long cs = block_sum64(csum, s_tmp);
  if (threadIdx.x == 0) {
    atomicAdd(&info->total_vertex_weight, (unsigned long long)cs);
    atomicMax(&info->max_vertex_weight, mx);
  }
}

static unsigned grid_cap_load(long long items) {
  long long b = (items + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > kLoadGrid) b = kLoadGrid;
  return (unsigned)b;
}

hipError_t load_check(hg_graph_s* g, hipStream_t s) {
  LoadInfo* info = (LoadInfo*)(g->ws + g->lay.info);
  hipError_t e = fill_i32((int*)info, 0, sizeof(LoadInfo) / sizeof(int), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_nets, dim3(grid_cap_load(g->m)), dim3(kBlock), 0, s, g->m, g->P,
                     g->eptr, g->ewgt, info);
  hipLaunchKernelGGL(k_check_pins, dim3(grid_for(g->P, 4)), dim3(kBlock), 0, s, g->n, g->P,
                     g->pins, info);
  hipLaunchKernelGGL(k_check_vertices, dim3(grid_cap_load(g->n)), dim3(kBlock), 0, s, g->n,
                     g->vwgt, info);
  return hipGetLastError();
}

// ------------------------------------------------------------------ transpose
// Degree count: one integer atomic per pin (order-independent result).
__global__ void k_count_degrees(long long P, const int* pins, int* deg) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < P; i += stride) atomicAdd(&deg[pins[i]], 1);
}

// Exclusive scan of deg[0..n) into vptr[0..n], three passes.
constexpr int kScanPerBlock = kBlock * 8;

__global__ void k_scan_partials(int n, const int* deg, long long* partial) {
  __shared__ long long s_tmp[kBlock / kWave];
  long long base = (long long)blockIdx.x * kScanPerBlock;
  long long sum = 0;
  for (int j = 0; j < 8; ++j) {
    long long i = base + (long long)j * kBlock + threadIdx.x;
    if (i < n) sum += deg[i];
  }
  long long tot = block_sum64(sum, s_tmp);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One workgroup scans the per-block partial sums in place (exclusive).
__global__ void k_scan_top(int nblocks, long long* partial) {
  __shared__ long long s_tmp[kBlock / kWave];
  long long carry = 0;
  for (int base = 0; base < nblocks; base += kBlock) {
    int i = base + threadIdx.x;
    long long v = i < nblocks ? partial[i] : 0;
    long long tot;
    long long ex = block_excl_scan64(v, s_tmp, &tot);
    if (i < nblocks) partial[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
}

__global__ void k_scan_final(int n, const int* deg, const long long* partial, long long* vptr,
                             long long P) {
  __shared__ long long s_tmp[kBlock / kWave];
  long long base = (long long)blockIdx.x * kScanPerBlock;
  // each thread owns 8 consecutive entries
  long long first = base + (long long)threadIdx.x * 8;
  int d[8];
  long long local = 0;
  for (int j = 0; j < 8; ++j) {
    long long i = first + j;
    d[j] = i < n ? deg[i] : 0;
    local += d[j];
  }
  long long tot;
  long long ex = block_excl_scan64(local, s_tmp, &tot);
  long long run = partial[blockIdx.x] + ex;
  for (int j = 0; j < 8; ++j) {
    long long i = first + j;
    if (i < n) vptr[i] = run;
    run += d[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) vptr[n] = P;
}

// Scatter: each wave walks the pins of 64 consecutive nets, load-balanced.
__global__ void k_scatter(int m, const long long* eptr, const int* pins, const long long* vptr,
                          int* cursor, int* vnets) {
  __shared__ int s_excl[kBlock / kWave][kWave];
  __shared__ long long s_begin[kBlock / kWave][kWave];
  int w = threadIdx.x / kWave, lane = lane_id();
  long long wave_global = (long long)blockIdx.x * (kBlock / kWave) + w;
  long long e = wave_global * kWave + lane;
  long long b = 0;
  int len = 0;
  if (e < m) {
    b = eptr[e];
    len = (int)(eptr[e + 1] - b);
  }
  int first_net = (int)(wave_global * kWave);
  wave_expand(b, len, s_excl[w], s_begin[w], [&](bool act, int owner, long long p) {
    if (act) {
      int v = pins[p];
      int pos = atomicAdd(&cursor[v], 1);
      vnets[vptr[v] + pos] = first_net + owner;
    }
  });
}

// Sort incidence rows of length <= kSmallRow in place (one thread per
// vertex, insertion sort), then gather per-vertex facts.  Longer rows are
// listed for k_sort_big_rows.
__global__ __launch_bounds__(kBlock) void k_sort_small_rows(int n, const long long* vptr,
                                                            int* vnets, const int* ewgt,
                                                            int* big_list, int* heavy_list,
                                                            LoadInfo* info) {
  __shared__ int s_imax[kBlock / kWave];
  __shared__ unsigned s_big, s_heavy, s_big_base, s_heavy_base;
  __shared__ int s_bigv[kBlock], s_heavyv[kBlock];
  int err = 0, maxdeg = 0, maxincw = 0;
  const long long stride = (long long)gridDim.x * kBlock;
  const long long rounds = ((long long)n + stride - 1) / stride;
  for (long long r = 0; r < rounds; ++r) {
    const long long v = r * stride + (long long)blockIdx.x * kBlock + threadIdx.x;
    if (threadIdx.x == 0) s_big = s_heavy = 0;
    __syncthreads();
    bool big = false, heavy = false;
    if (v < n) {
      const long long b = vptr[v];
      const int deg = (int)(vptr[v + 1] - b);
      maxdeg = deg > maxdeg ? deg : maxdeg;
      if (deg > kSmallRow) {
        big = true;
      } else {
        int* row = vnets + b;
        for (int i = 1; i < deg; ++i) {
          const int x = row[i];
          int j = i - 1;
          while (j >= 0 && row[j] > x) {
            row[j + 1] = row[j];
            --j;
          }
          row[j + 1] = x;
        }
        long long tot = 0;
        for (int i = 0; i < deg; ++i) {
          if (i > 0 && row[i] == row[i - 1]) err = kErrDuplicate;
          tot += ewgt ? ewgt[row[i]] : 1;
        }
        const int incw = tot > 0x7fffffffLL ? 0x7fffffff : (int)tot;
        maxincw = incw > maxincw ? incw : maxincw;
        heavy = tot > kLightLimit;
      }
    }
    if (big) s_bigv[atomicAdd(&s_big, 1u)] = (int)v;
    if (heavy) s_heavyv[atomicAdd(&s_heavy, 1u)] = (int)v;
    __syncthreads();
    if (threadIdx.x == 0) {
      s_big_base = s_big ? atomicAdd((unsigned*)&info->big_rows, s_big) : 0;
      s_heavy_base = s_heavy ? atomicAdd((unsigned*)&info->heavy_count, s_heavy) : 0;
    }
    __syncthreads();
    if (threadIdx.x < s_big) big_list[s_big_base + threadIdx.x] = s_bigv[threadIdx.x];
    if (threadIdx.x < s_heavy) heavy_list[s_heavy_base + threadIdx.x] = s_heavyv[threadIdx.x];
    __syncthreads();
  }
  if (err) atomicOr(&info->err, err);
  const int md = block_max_int(maxdeg, s_imax);
  const int mi = block_max_int(maxincw, s_imax);
  if (threadIdx.x == 0) {
    atomicMax(&info->max_degree, md);
    atomicMax(&info->max_incident_weight, mi);
  }
}

// One workgroup per long row: bitonic sort with all comparators ascending
// (indices past the row end act as +infinity and never move), in LDS when the
// padded row fits, else in place in global memory.
constexpr int kLdsSortCap = 8192;

__global__ void k_sort_big_rows(const long long* vptr, int* vnets, const int* ewgt,
                                const int* big_list, int* heavy_list, LoadInfo* info) {
  __shared__ int s_row[kLdsSortCap];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_err;
  int v = big_list[blockIdx.x];
  long long b = vptr[v];
  int len = (int)(vptr[v + 1] - b);
  int pow2 = 1;
  while (pow2 < len) pow2 <<= 1;
  int* row = vnets + b;
  if (threadIdx.x == 0) s_err = 0;
  if (pow2 <= kLdsSortCap) {
    for (int i = threadIdx.x; i < len; i += blockDim.x) s_row[i] = row[i];
    __syncthreads();
    bitonic_sort_block(len, pow2, [&](int i) { return s_row[i]; },
                       [&](int i, int x) { s_row[i] = x; });
    for (int i = threadIdx.x; i < len; i += blockDim.x) row[i] = s_row[i];
    __syncthreads();
  } else {
    __syncthreads();
    bitonic_sort_block(len, pow2, [&](int i) { return row[i]; },
                       [&](int i, int x) { row[i] = x; });
  }
  long long tot = 0;
  int err = 0;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    if (i > 0 && row[i] == row[i - 1]) err = kErrDuplicate;
    tot += ewgt ? ewgt[row[i]] : 1;
  }
  if (err) atomicOr(&s_err, err);
  tot = block_sum64(tot, s_tmp);
  if (threadIdx.x == 0) {
    if (s_err) atomicOr(&info->err, s_err);
    int incw = tot > 0x7fffffffLL ? 0x7fffffff : (int)tot;
    atomicMax(&info->max_degree, len);
    atomicMax(&info->max_incident_weight, incw);
    if (tot > kLightLimit) {
      int hi = atomicAdd(&info->heavy_count, 1);
      heavy_list[hi] = v;
    }
  }
}

// Builds vptr/vnets.  Needs LoadInfo.big_rows from a synchronized read to
// launch the long-row pass, so it is split: this part runs the small-row pass
// and leaves big_rows for load_sort_big.
hipError_t load_build(hg_graph_s* g, hipStream_t s) {
  LoadInfo* info = (LoadInfo*)(g->ws + g->lay.info);
  int* deg = (int*)(g->ws + g->lay.cand);     // the candidate array is free at load time
  int* cursor = deg + g->n;
  long long* partial = (long long*)(g->ws + g->lay.scan);
  int* big = (int*)(g->ws + g->lay.big);
  int* heavy = (int*)(g->ws + g->lay.heavy);
  hipError_t e = fill_i32(deg, 0, 2LL * g->n, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_count_degrees, dim3(grid_for(g->P, 4)), dim3(kBlock), 0, s, g->P,
                     g->pins, deg);
  int nb = g->lay.scan_blocks;
  hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kBlock), 0, s, g->n, deg, partial);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, nb, partial);
  hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kBlock), 0, s, g->n, deg, partial, g->vptr,
                     g->P);
  long long waves = ((long long)g->m + kWave - 1) / kWave;
  unsigned blocks = (unsigned)((waves + kBlock / kWave - 1) / (kBlock / kWave));
  hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(kBlock), 0, s, g->m, g->eptr, g->pins,
                     g->vptr, cursor, g->vnets);
  hipLaunchKernelGGL(k_sort_small_rows, dim3(grid_cap_load(g->n)), dim3(kBlock), 0, s, g->n,
                     g->vptr, g->vnets, g->ewgt, big, heavy, info);
  return hipGetLastError();
}

hipError_t load_sort_big(hg_graph_s* g, int big_rows, hipStream_t s) {
  if (big_rows <= 0) return hipSuccess;
  LoadInfo* info = (LoadInfo*)(g->ws + g->lay.info);
  int* big = (int*)(g->ws + g->lay.big);
  int* heavy = (int*)(g->ws + g->lay.heavy);
  hipLaunchKernelGGL(k_sort_big_rows, dim3(big_rows), dim3(kBlock), 0, s, g->vptr, g->vnets,
                     g->ewgt, big, heavy, info);
  return hipGetLastError();
}

}  // namespace hg
