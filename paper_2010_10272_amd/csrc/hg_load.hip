// hg_load.hip -- input checks, incidence CSR (transpose of the net CSR) and
// static per-vertex facts.  Runs once per loaded hypergraph.
//
// The paper stores a hypergraph as two adjacency arrays, the pins of each net
// and the incident nets of each vertex (section "Coarsening", subsection
// "Contraction").  Here the second array is built on the device by a stable
// radix sort of the (pin, net) pairs by pin, so that I(v) lists nets in
// increasing id.
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

// Byte ranges cleared by one launch: each range's unaligned head and tail
// byte by byte, its middle in 16-byte stores.  One launch instead of one per
// range matters where a call clears many small arrays (a few microseconds
// of launch each).
__global__ void k_zero_ranges(ZeroRanges R) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (int r = 0; r < R.count; ++r) {
    unsigned char* p = R.p[r];
    const long long bytes = R.bytes[r];
    long long head = (long long)((16 - ((uintptr_t)p & 15)) & 15);
    if (head > bytes) head = bytes;
    const long long words = (bytes - head) / 16;
    const long long tail = head + words * 16;
    for (long long i = tid; i < head; i += stride) p[i] = 0;
    int4* w = reinterpret_cast<int4*>(p + head);
    for (long long i = tid; i < words; i += stride) w[i] = make_int4(0, 0, 0, 0);
    for (long long i = tail + tid; i < bytes; i += stride) p[i] = 0;
  }
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
void ZeroRanges::add(void* ptr, long long nbytes) {
  if (nbytes <= 0) return;
  if (count == kZeroRanges) __builtin_trap();   // a caller listed too many ranges
  p[count] = (unsigned char*)ptr;
  bytes[count] = nbytes;
  ++count;
}

hipError_t zero_ranges(const ZeroRanges& R, hipStream_t s) {
  long long most = 0;
  for (int r = 0; r < R.count; ++r) most = R.bytes[r] > most ? R.bytes[r] : most;
  if (most == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ranges, dim3(grid_for(most, 16)), dim3(kBlock), 0, s, R);
  return hipGetLastError();
}

hipError_t fill_u8(unsigned char* p, unsigned char v, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(count)), dim3(kBlock), 0, s, p, v, count);
  return hipGetLastError();
}

// ------------------------------------------------------------------ checks
// Load-time checks run on a capped grid (kLoadGrid) and reduce per
// workgroup into that workgroup's LoadPart; k_fold_load folds the parts.

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
                                                       LoadInfo* info, LoadPart* part) {
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
    part[blockIdx.x].max_net_size = mx;
    part[blockIdx.x].total_net_weight = (unsigned long long)ws;
  }
}

__global__ __launch_bounds__(kBlock) void k_check_vertices(int n, const int* vwgt,
                                                           LoadInfo* info, LoadPart* part) {
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
    part[blockIdx.x].total_vertex_weight = (unsigned long long)cs;
    part[blockIdx.x].max_vertex_weight = mx;
  }
}

// LoadInfo's maxima and sums from the workgroups' parts (one workgroup).
__global__ __launch_bounds__(kBlock) void k_fold_load(const LoadPart* part, LoadInfo* info) {
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_imax[kBlock / kWave];
  unsigned long long tnw = 0, tvw = 0;
  int mns = 0, mvw = 0, md = 0, miw = 0;
  for (int b = threadIdx.x; b < kLoadGrid; b += kBlock) {
    const LoadPart p = part[b];
    tnw += p.total_net_weight;
    tvw += p.total_vertex_weight;
    mns = p.max_net_size > mns ? p.max_net_size : mns;
    mvw = p.max_vertex_weight > mvw ? p.max_vertex_weight : mvw;
    md = p.max_degree > md ? p.max_degree : md;
    miw = p.max_incident_weight > miw ? p.max_incident_weight : miw;
  }
  tnw = (unsigned long long)block_sum64((long long)tnw, s_tmp);
  tvw = (unsigned long long)block_sum64((long long)tvw, s_tmp);
  mns = block_max_int(mns, s_imax);
  mvw = block_max_int(mvw, s_imax);
  md = block_max_int(md, s_imax);
  miw = block_max_int(miw, s_imax);
  if (threadIdx.x == 0) {
    info->total_net_weight = tnw;
    info->total_vertex_weight = tvw;
    info->max_net_size = mns;
    info->max_vertex_weight = mvw;
    info->max_degree = md;
    info->max_incident_weight = miw;
  }
}

static unsigned grid_cap_load(long long items) {
  long long b = (items + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > kLoadGrid) b = kLoadGrid;
  return (unsigned)b;
}

// The transpose's radix sort: long sorts in 8192-item tiles (fuller digit
// runs per tile; the netlist's 56.5M pairs sort 11% faster), shorter ones in
// 4096-item tiles (more workgroups: 7% faster on 10M pairs).
static bool long_load_sort(long long P) { return P >= (1LL << 24); }

// The sort's first pass: the keys are the caller's pins, read in place.
static SortPass first_load_pass(hg_graph_s* g) {
  SortPass SP;
  SP.hist = (unsigned*)(g->ws + g->lay.lhist);
  SP.dtot = (unsigned*)(g->ws + g->lay.ldtot);
  SP.n = (int)g->P;
  SP.tiles = long_load_sort(g->P) ? sort_tiles<kSortPerLong>(g->P) : sort_tiles(g->P);
  SP.key_in = (const unsigned*)g->pins;
  SP.shift = 0;
  return SP;
}

hipError_t load_check(hg_graph_s* g, hipStream_t s) {
  LoadInfo* info = (LoadInfo*)(g->ws + g->lay.info);
  LoadPart* part = (LoadPart*)(g->ws + g->lay.lpart);
  ZeroRanges Z;
  Z.add(info, sizeof(LoadInfo));
  Z.add(part, (long long)sizeof(LoadPart) * kLoadGrid);
  hipError_t e = zero_ranges(Z, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_nets, dim3(grid_cap_load(g->m)), dim3(kBlock), 0, s, g->m, g->P,
                     g->eptr, g->ewgt, info, part);
  // the pins' range check is the sort's first digit count, which reads every
  // pin anyway (a pin outside [0, n) only lands in some digit's count; the
  // build does not start unless the checks pass)
  SortPass SP = first_load_pass(g);
  SP.err = &info->err;
  SP.err_bit = kErrPin;
  SP.key_limit = (unsigned)g->n;
  if (long_load_sort(g->P))
    hipLaunchKernelGGL(k_sort_hist<kSortPerLong>, dim3(SP.tiles), dim3(kBlock), 0, s, SP);
  else
    hipLaunchKernelGGL(k_sort_hist<kSortPer>, dim3(SP.tiles), dim3(kBlock), 0, s, SP);
  hipLaunchKernelGGL(k_check_vertices, dim3(grid_cap_load(g->n)), dim3(kBlock), 0, s, g->n,
                     g->vwgt, info, part);
  hipLaunchKernelGGL(k_fold_load, dim3(1), dim3(kBlock), 0, s, (const LoadPart*)part, info);
  return hipGetLastError();
}

constexpr int kBigRowGrid = 256;   // workgroups striding over the long rows

// ------------------------------------------------------------------ transpose
// (pin, net) pairs in net order, stably radix-sorted by pin: the values are
// then the incidence rows, each listing its nets in increasing id, with no
// atomics anywhere (so nothing depends on timing).  Row starts come from
// where the sorted keys change.

// Each wave expands the pins of 64 consecutive nets into the net id of every
// pin position: the pairs' values (their keys are the pins themselves, which
// the first sort pass reads in place).  The nets' pins form one contiguous
// run; it is written 64 positions per step, and a position's net is the
// count of nets starting at or before it: each net flags its first position
// of the step in LDS and one ballot gives every lane the count (nets are
// non-empty, so their starts are distinct).
__global__ void k_pin_pairs(int m, const long long* eptr, int* val) {
  __shared__ unsigned char s_start[kBlock / kWave][kWave];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const long long wave_global = (long long)blockIdx.x * (kBlock / kWave) + w;
  const long long e = wave_global * kWave + lane;
  long long b = 0;
  int len = 0;
  if (e < m) {
    b = eptr[e];
    len = (int)(eptr[e + 1] - b);
  }
  const int incl = wave_incl_scan(len);
  const int total = __shfl(incl, kWave - 1);
  const int first = incl - len;                  // this net's offset in the run
  const long long run = __shfl(b, 0);            // the run starts at the wave's first net
  const int first_net = (int)(wave_global * kWave);
  const unsigned long long upto = ~0ull >> (kWave - 1 - lane);   // lanes 0 .. this one
  s_start[w][lane] = 0;
  wave_lds_sync();
  int before = 0;                                // nets starting before this step
  for (int base = 0; base < total; base += kWave) {
    if (len > 0 && first >= base && first < base + kWave) s_start[w][first - base] = 1;
    wave_lds_sync();
    const unsigned long long starts = __ballot(s_start[w][lane] != 0);
    s_start[w][lane] = 0;
    wave_lds_sync();
    if (base + lane < total)
      val[run + base + lane] = first_net + before + __popcll(starts & upto) - 1;
    before += __popcll(starts);
  }
}

// vptr[v] = the first sorted position with key >= v; vptr[n] = P.  A pair
// equal to its predecessor (same pin, same net) is a vertex listed twice in
// one net: the stable sort puts such pairs side by side.  Four positions per
// thread (16-byte loads of keys and values when both arrays are 16-byte
// aligned, `vec`), each compared with the one before it.
constexpr int kRowStartsPer = 4;

__global__ void k_row_starts(long long P, int n, const unsigned* key, const int* val, int vec,
                             long long* vptr, LoadInfo* info) {
  const long long i0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * kRowStartsPer;
  if (i0 >= P) return;
  long long k[kRowStartsPer + 1];
  int v[kRowStartsPer + 1];
  k[0] = i0 == 0 ? -1 : (long long)key[i0 - 1];
  v[0] = i0 == 0 ? -1 : val[i0 - 1];
  if (vec && i0 + kRowStartsPer <= P) {
    const uint4 kq = *reinterpret_cast<const uint4*>(key + i0);
    const int4 vq = *reinterpret_cast<const int4*>(val + i0);
    k[1] = kq.x; k[2] = kq.y; k[3] = kq.z; k[4] = kq.w;
    v[1] = vq.x; v[2] = vq.y; v[3] = vq.z; v[4] = vq.w;
  } else {
    for (int q = 0; q < kRowStartsPer; ++q) {
      k[q + 1] = i0 + q < P ? (long long)key[i0 + q] : -1;
      v[q + 1] = i0 + q < P ? val[i0 + q] : 0;
    }
  }
  int err = 0;
  for (int q = 0; q < kRowStartsPer && i0 + q < P; ++q) {
    const long long i = i0 + q, cur = k[q + 1], prev = k[q];
    if (cur == prev && v[q + 1] == v[q]) err = kErrDuplicate;
    for (long long x = prev + 1; x <= cur; ++x) vptr[x] = i;
    if (i == P - 1)
      for (long long x = cur + 1; x <= n; ++x) vptr[x] = P;
  }
  if (err) atomicOr(&info->err, err);
}

// Per-vertex facts of the sorted rows: degree, w(I(v)), the heavy list.
// With unit net weights (ewgt == NULL) w(I(v)) is the degree and only the
// offsets are read.  Otherwise one thread sums a row of up to kSmallRow
// incidences; longer rows are listed for k_big_row_facts.
__global__ __launch_bounds__(kBlock) void k_row_facts(int n, const long long* vptr,
                                                      const int* vnets, const int* ewgt,
                                                      int* big_list, int* heavy_list,
                                                      LoadInfo* info, LoadPart* part) {
  __shared__ int s_imax[kBlock / kWave];
  __shared__ unsigned s_big, s_heavy, s_big_base, s_heavy_base;
  __shared__ int s_bigv[kBlock], s_heavyv[kBlock];
  int maxdeg = 0, maxincw = 0;
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
      if (!ewgt) {
        maxincw = deg > maxincw ? deg : maxincw;
        heavy = deg > kLightLimit;
      } else if (deg > kSmallRow) {
        big = true;
      } else {
        // the row's entries in groups of four, loaded before their weights
        const int* row = vnets + b;
        long long tot = 0;
        for (int i0 = 0; i0 < deg; i0 += 4) {
          int x[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) x[q] = row[i0 + q < deg ? i0 + q : i0];
          int wq[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) wq[q] = ewgt[x[q]];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (i0 + q < deg) tot += wq[q];
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
  const int md = block_max_int(maxdeg, s_imax);
  const int mi = block_max_int(maxincw, s_imax);
  if (threadIdx.x == 0) {
    part[blockIdx.x].max_degree = md;
    part[blockIdx.x].max_incident_weight = mi;
  }
}

// One workgroup per long row: the same facts with the row's entries spread
// over the workgroup.
__global__ void k_big_row_facts(const long long* vptr, const int* vnets, const int* ewgt,
                                const int* big_list, int* heavy_list, LoadInfo* info) {
  __shared__ long long s_tmp[kBlock / kWave];
  // the count comes from the short-row pass (an earlier launch), so the host
  // need not read it first; a fixed grid strides over the list
  const int nbig = info->big_rows;
  for (int bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const int v = big_list[bi];
    const long long b = vptr[v];
    const int len = (int)(vptr[v + 1] - b);
    const int* row = vnets + b;
    long long tot = 0;
    for (int i = threadIdx.x; i < len; i += blockDim.x) tot += ewgt[row[i]];
    tot = block_sum64(tot, s_tmp);
    if (threadIdx.x == 0) {
      const int incw = tot > 0x7fffffffLL ? 0x7fffffff : (int)tot;
      atomicMax(&info->max_degree, len);
      atomicMax(&info->max_incident_weight, incw);
      if (tot > kLightLimit) {
        const int hi = atomicAdd(&info->heavy_count, 1);
        heavy_list[hi] = v;
      }
    }
    __syncthreads();
  }
}

// Builds vptr/vnets and the rows' facts (short rows one per thread, long
// rows one per workgroup).
hipError_t load_build(hg_graph_s* g, hipStream_t s) {
  LoadInfo* info = (LoadInfo*)(g->ws + g->lay.info);
  int* big = (int*)(g->ws + g->lay.big);
  int* heavy = (int*)(g->ws + g->lay.heavy);
  const long long P = g->P;
  int passes = 0;
  for (int bits = 0; bits < 32 && (1ll << bits) < (long long)g->n; bits += 8) ++passes;
  if (passes == 0) passes = 1;
  // the last pass must leave its values in vnets
  unsigned* key[2] = {(unsigned*)(g->ws + g->lay.lkey[0]), (unsigned*)(g->ws + g->lay.lkey[1])};
  int* scratch = (int*)(g->ws + g->lay.lval);
  int* val[2];
  val[passes & 1] = g->vnets;
  val[(passes & 1) ^ 1] = scratch;
  const long long waves = ((long long)g->m + kWave - 1) / kWave;
  const unsigned blocks = (unsigned)((waves + kBlock / kWave - 1) / (kBlock / kWave));
  hipLaunchKernelGGL(k_pin_pairs, dim3(blocks), dim3(kBlock), 0, s, g->m, g->eptr, val[0]);
  // the first pass reads the (validated, non-negative) pins as its keys; its
  // digit counts were taken by the checks
  SortPass SP = first_load_pass(g);
  const bool long_sort = long_load_sort(P);
  for (int q = 0; q < passes; ++q) {
    SP.val_in = val[q & 1];
    SP.key_out = key[(q & 1) ^ 1];
    SP.val_out = val[(q & 1) ^ 1];
    SP.shift = 8 * q;
    if (q == 0 && long_sort)
      sort_pass_counted<kSortPerLong>(SP, s);
    else if (q == 0)
      sort_pass_counted(SP, s);
    else if (long_sort)
      sort_pass<kSortPerLong>(SP, s);
    else
      sort_pass(SP, s);
    SP.key_in = SP.key_out;
  }
  const long long rs_threads = (P + kRowStartsPer - 1) / kRowStartsPer;
  const unsigned* skey = key[passes & 1];
  const int vec = (((uintptr_t)skey | (uintptr_t)g->vnets) & 15) == 0;
  hipLaunchKernelGGL(k_row_starts, dim3((unsigned)((rs_threads + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, P, g->n, skey, (const int*)g->vnets, vec, g->vptr, info);
  // all net weights 1 (the checks summed them to m): rows need no weights
  const int* ew = g->info.total_net_weight == (unsigned long long)g->m ? nullptr : g->ewgt;
  LoadPart* part = (LoadPart*)(g->ws + g->lay.lpart);
  hipLaunchKernelGGL(k_row_facts, dim3(grid_cap_load(g->n)), dim3(kBlock), 0, s, g->n, g->vptr,
                     g->vnets, ew, big, heavy, info, part);
  hipLaunchKernelGGL(k_fold_load, dim3(1), dim3(kBlock), 0, s, (const LoadPart*)part, info);
  if (ew)
    hipLaunchKernelGGL(k_big_row_facts, dim3(kBigRowGrid), dim3(kBlock), 0, s, g->vptr, g->vnets,
                       ew, big, heavy, info);
  return hipGetLastError();
}

}  // namespace hg
