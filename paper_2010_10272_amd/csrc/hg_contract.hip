// hg_contract.hip -- contraction of a vertex clustering into a coarse
// hypergraph (section "Coarsening", subsection "Contraction"), as a second
// HBM-bound workload beside refinement.
//
//   1. used cluster ids are flagged and renumbered by a prefix sum (the
//      rank of the id among the used ones): map[v];
//   2. coarse vertex weights by integer atomics;
//   3. every net's pins are mapped, sorted and deduplicated in the net's own
//      slots of a scratch copy (tmp[eptr[e] ..]): nets of up to kSmallNet
//      pins a tile of consecutive nets per workgroup in LDS (stable rank
//      inside the net, first occurrences numbered by a block scan), longer
//      nets one workgroup each (bitonic sort in LDS, or in place beyond the
//      LDS capacity, then a compaction by block scans); the same pass gives
//      the surviving size and the fingerprint;
//   4. nets left with fewer than two pins are dropped;
//   5. identical nets (parallel INRSRT): the fingerprint sum of v^2 and the
//      size of every net are hashed to a 32-bit key; a stable sort by key
//      puts candidates for identity next to each other in net-id order, and
//      each net compares its pins with the nets before it in its run, from
//      the run's head, until the first identical one -- whose id is then the
//      lowest among them and becomes the representative; weights are summed
//      at the representative;
//   6. representatives are numbered in net-id order and written out as net
//      CSR with their sorted pins (prefix sums over kept nets and sizes).
// The order of every output is fixed by the definition (ranks, net ids,
// sorted pins), so the result is deterministic and equals the plain
// sequential contraction.
#include <string.h>

#include "hg_device.h"
#include "hg_internal.h"
#include "hg_scan.h"
#include "hg_sort.h"

namespace hg {
namespace {

struct Ct {
  // input
  int n, m;
  long long P;
  const long long* eptr;
  const int* pins;
  const int* vwgt;
  const int* ewgt;
  const int* cluster;
  // output
  int* map;
  int* cvwgt;
  long long* ceptr;
  int* cpins;
  int* cewgt;
  long long* sizes;      // n', m', P'
  // workspace
  unsigned char* used;   // [n]
  long long* rank;       // [n]
  unsigned long long* cw;// [n]
  int* tmp;              // [P]: net e's sorted distinct coarse pins at eptr[e] ..
  int* big;              // [m]: nets longer than kSmallNet
  int* big_count;        // [1]
  int* tile_first;       // [tiles + 1]: first net starting in each small-net tile
  int* nsize;            // [m]: pins after deduplication
  unsigned long long* fp;// [m]
  unsigned* nkey[2];     // [m]
  int* nval[2];          // [m]
  long long* hscan;      // [m]: run heads before a sorted position
  int* heads;            // [m]: sorted position of every run head
  int* rep;              // [m]: representative, -1 for dropped nets
  unsigned* wsum;        // [m]
  long long* nid;        // [m]: coarse id of a kept net
  long long* npos;       // [m]: first coarse pin of a kept net
  int* err;
};

__global__ __launch_bounds__(kBlock) void k_ct_mark(Ct C) {
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= C.n) return;
  const int c = C.cluster[v];
  if ((unsigned)c >= (unsigned)C.n) {
    atomicOr(C.err, kErrCluster);
    return;
  }
  C.used[c] = 1;
}

struct UsedF {
  const unsigned char* used;
  __device__ long long operator()(long long i) const { return used[i]; }
};

__global__ __launch_bounds__(kBlock) void k_ct_map(Ct C) {
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= C.n) return;
  const int c = C.cluster[v];
  if ((unsigned)c >= (unsigned)C.n) return;
  const int x = (int)C.rank[c];
  C.map[v] = x;
  atomicAdd(&C.cw[x], (unsigned long long)(C.vwgt ? C.vwgt[v] : 1));
}

__global__ __launch_bounds__(kBlock) void k_ct_vweights(Ct C) {
  const long long x = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (x >= C.sizes[0]) return;
  const unsigned long long w = C.cw[x];
  if (w > 0x7fffffffULL) atomicOr(C.err, kErrClusterWeight);
  C.cvwgt[x] = (int)w;
}

__device__ __forceinline__ unsigned ct_hash(unsigned long long fp, int size) {
  unsigned long long h = fp * 0x9E3779B97F4A7C15ULL + (unsigned long long)size * 0xC2B2AE3D27D4EB4FULL;
  h ^= h >> 29;
  h *= 0xBF58476D1CE4E5B9ULL;
  h ^= h >> 32;
  return (unsigned)h;
}

constexpr int kSmallNet = 128;      // nets up to this many pins go through the tiles
constexpr int kNetLdsCap = 8192;    // longer nets sort in LDS up to this many pins

__device__ __forceinline__ void ct_net_done(const Ct& C, long long e, int size,
                                            unsigned long long fp) {
  C.nsize[e] = size;
  C.fp[e] = fp;
  C.nkey[0][e] = size >= 2 ? ct_hash(fp, size) : 0xffffffffu;
  C.nval[0][e] = (int)e;
  C.rep[e] = -1;
  C.wsum[e] = 0;
}

constexpr int kNetTile = 1024;      // pins per small-net tile (by net start)

// tile_first[t] = the first net whose first pin is at or after kNetTile * t
// (m when there is none); every net writes the entries of the tiles between
// its predecessor's start and its own.
__global__ __launch_bounds__(kBlock) void k_ct_tiles(Ct C, long long tiles) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e > C.m) return;
  const long long from = e == 0 ? 0 : (C.eptr[e - 1] / kNetTile) + 1;
  const long long to = e == C.m ? tiles : C.eptr[e] / kNetTile;
  for (long long t = from; t <= to; ++t) C.tile_first[t] = (int)e;
}

// Small nets, a tile at a time: the nets whose first pin lies in pins
// [kNetTile * t, kNetTile * (t + 1)) -- at most kNetTile + kSmallNet - 1 pins
// when every one of them is small, because a long net ends the tile.  Their
// mapped pins go to LDS; every pin learns whether it is the first of its
// value in its net and, if so, how many distinct values of the net are
// smaller (its place in the sorted distinct list); sizes and fingerprints
// are LDS sums per net.  Long nets are listed for k_ct_big_nets.
__global__ __launch_bounds__(kBlock) void k_ct_small_nets(Ct C) {
  constexpr int kCap = kNetTile + kSmallNet;
  __shared__ int s_val[kCap];
  __shared__ short s_net[kCap];
  __shared__ int s_sorted[kCap];
  __shared__ int s_rank[kCap + 1];
  __shared__ int s_start[kNetTile + 1];
  __shared__ unsigned long long s_fp[kNetTile];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_e0, s_e1;
  __shared__ unsigned s_big, s_big_base;
  __shared__ int s_bigv[kNetTile / (kSmallNet + 1) + 2];   // long nets starting in a tile
  const long long tiles = (C.P + kNetTile - 1) / kNetTile;
  for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
    if (threadIdx.x < 2) {
      const int f = C.tile_first[t + threadIdx.x];
      if (threadIdx.x == 0) s_e0 = f; else s_e1 = f;
    }
    if (threadIdx.x == 0) s_big = 0;
    __syncthreads();
    const int e0 = s_e0, nets = s_e1 - s_e0;
    // local offsets of the small nets (long nets take no room)
    long long carry = 0;
    for (int j0 = 0; j0 < nets; j0 += kBlock) {
      const int j = j0 + threadIdx.x;
      int size = 0;
      if (j < nets) {
        const long long e = e0 + j;
        size = (int)(C.eptr[e + 1] - C.eptr[e]);
        if (size > kSmallNet) {
          s_bigv[atomicAdd(&s_big, 1u)] = (int)e;
          size = 0;
        }
      }
      long long tot;
      const long long ex = block_excl_scan64(size, s_tmp, &tot);
      if (j < nets) {
        s_start[j] = (int)(carry + ex);
        s_fp[j] = 0;
      }
      carry += tot;
    }
    const int total = (int)carry;
    if (threadIdx.x == 0) s_start[nets] = total;
    __syncthreads();
    // mapped pins into LDS: every thread's positions first, then all their
    // pin loads, then all their map loads (independent loads in flight)
    constexpr int kPer = (kCap + kBlock - 1) / kBlock;
    long long src[kPer];
    int pin[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int q = threadIdx.x + r * kBlock;
      src[r] = -1;
      if (q < total) {
        int lo = 0, hi = nets - 1;     // net: the last j with s_start[j] <= q
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_start[mid] <= q) lo = mid; else hi = mid - 1;
        }
        src[r] = C.eptr[e0 + lo] + (q - s_start[lo]);
        s_net[q] = (short)lo;
      }
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) pin[r] = src[r] >= 0 ? C.pins[src[r]] : 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r)
      if (src[r] >= 0) s_val[threadIdx.x + r * kBlock] = C.map[pin[r]];
    __syncthreads();
    // stable rank inside the net -> sorted copy (a permutation of the net)
    for (int q = threadIdx.x; q < total; q += kBlock) {
      const int j = s_net[q], x = s_val[q];
      const int b = s_start[j], t2 = s_start[j + 1];
      int rank = 0;
#pragma unroll 4
      for (int r = b; r < t2; ++r) {
        const int v = s_val[r];
        rank += v < x || (v == x && r < q);
      }
      s_sorted[b + rank] = x;
    }
    __syncthreads();
    // first occurrences in sorted order, numbered by a scan over the tile
    long long run = 0;
    int firsts[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int q = threadIdx.x + r * kBlock;
      int f = 0;
      if (q < total) {
        const int j = s_net[q];
        f = q == s_start[j] || s_sorted[q - 1] != s_sorted[q];
      }
      firsts[r] = f;
      long long tot;
      const long long ex = block_excl_scan64(f, s_tmp, &tot);
      if (q < total) s_rank[q] = (int)(run + ex);
      run += tot;
    }
    if (threadIdx.x == 0) s_rank[total] = (int)run;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int q = threadIdx.x + r * kBlock;
      if (q >= total || !firsts[r]) continue;
      const int j = s_net[q], x = s_sorted[q];
      C.tmp[C.eptr[e0 + j] + (s_rank[q] - s_rank[s_start[j]])] = x;
      atomicAdd(&s_fp[j], (unsigned long long)(unsigned)x * (unsigned)x);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nets; j += kBlock)
      if (s_start[j + 1] > s_start[j])
        ct_net_done(C, e0 + j, s_rank[s_start[j + 1]] - s_rank[s_start[j]], s_fp[j]);
    if (threadIdx.x == 0 && s_big) s_big_base = atomicAdd((unsigned*)C.big_count, s_big);
    __syncthreads();
    for (int j = threadIdx.x; j < (int)s_big; j += kBlock) C.big[s_big_base + j] = s_bigv[j];
    __syncthreads();
  }
}

// One workgroup per listed net (workgroups stride over the list): map,
// bitonic sort (LDS when it fits), then keep first occurrences in order by
// block scans over chunks of the sorted row.
__global__ __launch_bounds__(kBlock) void k_ct_big_nets(Ct C) {
  __shared__ int s_row[kNetLdsCap];
  __shared__ long long s_tmp[kBlock / kWave];
  __shared__ int s_prev;
  const int count = *C.big_count;
  for (int idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int e = C.big[idx];
    const long long b = C.eptr[e];
    const int len = (int)(C.eptr[e + 1] - b);
    int pow2 = 1;
    while (pow2 < len) pow2 <<= 1;
    int* row = C.tmp + b;
    if (pow2 <= kNetLdsCap) {
      for (int i = threadIdx.x; i < len; i += kBlock) s_row[i] = C.map[C.pins[b + i]];
      __syncthreads();
      bitonic_sort_block(len, pow2, [&](int i) { return s_row[i]; },
                         [&](int i, int x) { s_row[i] = x; });
      for (int i = threadIdx.x; i < len; i += kBlock) row[i] = s_row[i];
    } else {
      for (int i = threadIdx.x; i < len; i += kBlock) row[i] = C.map[C.pins[b + i]];
      __syncthreads();
      bitonic_sort_block(len, pow2, [&](int i) { return row[i]; },
                         [&](int i, int x) { row[i] = x; });
    }
    __syncthreads();
    // compaction in place: writes never pass the chunk being read
    long long kept = 0;
    unsigned long long fp = 0;
    if (threadIdx.x == 0) s_prev = -1;
    __syncthreads();
    for (int c0 = 0; c0 < len; c0 += kBlock) {
      const int i = c0 + threadIdx.x;
      const int x = i < len ? row[i] : 0;
      const int before = i == 0 ? -1 : (threadIdx.x == 0 ? s_prev : row[i - 1]);
      const bool first = i < len && (i == 0 || x != before);
      long long tot;
      const long long at = kept + block_excl_scan64(first ? 1 : 0, s_tmp, &tot);
      if (threadIdx.x == kBlock - 1 || i == len - 1) s_prev = x;
      __syncthreads();
      if (first) {
        row[at] = x;
        fp += (unsigned long long)(unsigned)x * (unsigned)x;
      }
      kept += tot;
      __syncthreads();
    }
    const unsigned long long f = (unsigned long long)block_sum64((long long)fp, s_tmp);
    if (threadIdx.x == 0) ct_net_done(C, e, (int)kept, f);
    __syncthreads();
  }
}

struct HeadF {
  const unsigned* key;
  __device__ long long operator()(long long j) const { return j == 0 || key[j] != key[j - 1]; }
};

__global__ __launch_bounds__(kBlock) void k_ct_heads(Ct C, const unsigned* key) {
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= C.m) return;
  if (j == 0 || key[j] != key[j - 1]) C.heads[C.hscan[j]] = (int)j;
}

__device__ bool ct_same(const Ct& C, long long be, long long bf, int size) {
  for (int x = 0; x < size; ++x)
    if (C.tmp[be + x] != C.tmp[bf + x]) return false;
  return true;
}

// Sorted position j: the first net of j's run (from the head, in net-id
// order) with the same pins is the representative of j's net.
__global__ __launch_bounds__(kBlock) void k_ct_reps(Ct C, const unsigned* key, const int* val) {
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= C.m) return;
  const int e = val[j];
  const int size = C.nsize[e];
  if (size < 2) return;
  const bool head = j == 0 || key[j] != key[j - 1];
  const long long h = C.heads[C.hscan[j] + (head ? 1 : 0) - 1];
  const unsigned long long fe = C.fp[e];
  const long long be = C.eptr[e];
  int r = e;
  for (long long i = h; i < j; ++i) {
    const int f = val[i];
    if (C.nsize[f] != size || C.fp[f] != fe) continue;
    if (ct_same(C, be, C.eptr[f], size)) {
      r = f;
      break;
    }
  }
  C.rep[e] = r;
  atomicAdd(&C.wsum[r], (unsigned)(C.ewgt ? C.ewgt[e] : 1));
}

struct KeptF {
  const int* rep;
  __device__ long long operator()(long long e) const { return rep[e] == e; }
};

struct KeptSizeF {
  const int* rep;
  const int* nsize;
  __device__ long long operator()(long long e) const { return rep[e] == e ? nsize[e] : 0; }
};

// kEmitLanes lanes per net copy a kept net's pins side by side.
constexpr int kEmitLanes = 8;

__global__ __launch_bounds__(kBlock) void k_ct_emit(Ct C) {
  const long long e = ((long long)blockIdx.x * kBlock + threadIdx.x) / kEmitLanes;
  const int gl = threadIdx.x % kEmitLanes;
  if (e >= C.m || C.rep[e] != e) return;
  const long long id = C.nid[e], pos = C.npos[e];
  const long long b = C.eptr[e];
  const int size = C.nsize[e];
  if (gl == 0) {
    C.ceptr[id] = pos;
    C.cewgt[id] = (int)C.wsum[e];
  }
  for (int x = gl; x < size; x += kEmitLanes) C.cpins[pos + x] = C.tmp[b + x];
}

__global__ void k_ct_close(Ct C) {
  if (threadIdx.x == 0) C.ceptr[C.sizes[1]] = C.sizes[2];
}

}  // namespace

struct ContractLayout {
  size_t used, rank, cw, tmp, big, big_count, tile_first, nsize, fp, nkey[2], nval[2], hscan, heads, rep, wsum,
      nid, npos, csum, coff, nhist, ndtot, total;
};

static ContractLayout contract_layout(long long n, long long m, long long P) {
  ContractLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return at;
  };
  L.used = take((size_t)n);
  L.rank = take(8 * (size_t)n);
  L.cw = take(8 * (size_t)n);
  L.tmp = take(4 * (size_t)P);
  L.big = take(4 * (size_t)m);
  L.big_count = take(4);
  L.tile_first = take(4 * (size_t)((P + kNetTile - 1) / kNetTile + 1));
  for (int i = 0; i < 2; ++i) {
    L.nkey[i] = take(4 * (size_t)m);
    L.nval[i] = take(4 * (size_t)m);
  }
  L.nsize = take(4 * (size_t)m);
  L.fp = take(8 * (size_t)m);
  L.hscan = take(8 * (size_t)m);
  L.heads = take(4 * (size_t)m);
  L.rep = take(4 * (size_t)m);
  L.wsum = take(4 * (size_t)m);
  L.nid = take(8 * (size_t)m);
  L.npos = take(8 * (size_t)m);
  const long long most = n > m ? n : m;
  L.csum = take(8 * (size_t)scan_chunks(most));
  L.coff = take(8 * (size_t)scan_chunks(most));
  L.nhist = take(4 * (size_t)kDigits * sort_tiles(m));
  L.ndtot = take(4 * (size_t)kDigits);
  L.total = off;
  return L;
}

size_t contract_workspace_size(long long n, long long m, long long P) {
  return contract_layout(n, m, P).total;
}

static unsigned blocks_of(long long items) {
  long long b = (items + kBlock - 1) / kBlock;
  return (unsigned)(b < 1 ? 1 : b);
}

static hipError_t launch_contract(hg_graph_s* g, const int* cluster, int* map, int* cvwgt,
                                  long long* ceptr, int* cpins, int* cewgt, long long* sizes,
                                  char* ws, hipStream_t s) {
  const ContractLayout L = contract_layout(g->n, g->m, g->P);
  Ct C;
  memset(&C, 0, sizeof(C));
  C.n = g->n;
  C.m = g->m;
  C.P = g->P;
  C.eptr = g->eptr;
  C.pins = g->pins;
  C.vwgt = g->vwgt;
  C.ewgt = g->ewgt;
  C.cluster = cluster;
  C.map = map;
  C.cvwgt = cvwgt;
  C.ceptr = ceptr;
  C.cpins = cpins;
  C.cewgt = cewgt;
  C.sizes = sizes;
  C.used = (unsigned char*)(ws + L.used);
  C.rank = (long long*)(ws + L.rank);
  C.cw = (unsigned long long*)(ws + L.cw);
  for (int i = 0; i < 2; ++i) {
    C.nkey[i] = (unsigned*)(ws + L.nkey[i]);
    C.nval[i] = (int*)(ws + L.nval[i]);
  }
  C.tmp = (int*)(ws + L.tmp);
  C.big = (int*)(ws + L.big);
  C.big_count = (int*)(ws + L.big_count);
  C.tile_first = (int*)(ws + L.tile_first);
  C.nsize = (int*)(ws + L.nsize);
  C.fp = (unsigned long long*)(ws + L.fp);
  C.hscan = (long long*)(ws + L.hscan);
  C.heads = (int*)(ws + L.heads);
  C.rep = (int*)(ws + L.rep);
  C.wsum = (unsigned*)(ws + L.wsum);
  C.nid = (long long*)(ws + L.nid);
  C.npos = (long long*)(ws + L.npos);
  C.err = (int*)(g->ws + g->lay.flags);
  ScanBufs B;
  B.csum = (long long*)(ws + L.csum);
  B.coff = (long long*)(ws + L.coff);
  const long long n = g->n, m = g->m;

  // 1-2. renumbering, map, coarse weights
  ZeroRanges Z;
  Z.add(C.used, n);
  Z.add((void*)C.cw, (long long)sizeof(long long) * n);
  Z.add(C.big_count, (long long)sizeof(int));
  hipError_t e = zero_ranges(Z, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ct_mark, dim3(blocks_of(n)), dim3(kBlock), 0, s, C);
  exclusive_scan(UsedF{C.used}, n, C.rank, &sizes[0], B, s);
  hipLaunchKernelGGL(k_ct_map, dim3(blocks_of(n)), dim3(kBlock), 0, s, C);
  hipLaunchKernelGGL(k_ct_vweights, dim3(blocks_of(n)), dim3(kBlock), 0, s, C);

  // 3-4. per net: mapped, sorted, deduplicated pins, size, fingerprint
  const long long tiles = (g->P + kNetTile - 1) / kNetTile;
  hipLaunchKernelGGL(k_ct_tiles, dim3(blocks_of(m + 1)), dim3(kBlock), 0, s, C, tiles);
  long long sg = tiles < 8192 ? tiles : 8192;
  hipLaunchKernelGGL(k_ct_small_nets, dim3((unsigned)sg), dim3(kBlock), 0, s, C);
  hipLaunchKernelGGL(k_ct_big_nets, dim3(1024), dim3(kBlock), 0, s, C);

  // 5. identical nets
  int ncur = 0;
  SortPass SN;
  SN.hist = (unsigned*)(ws + L.nhist);
  SN.dtot = (unsigned*)(ws + L.ndtot);
  SN.n = (int)m;
  SN.tiles = sort_tiles(m);
  for (int shift = 0; shift < 32; shift += 8) {
    SN.key_in = C.nkey[ncur];
    SN.val_in = C.nval[ncur];
    SN.key_out = C.nkey[ncur ^ 1];
    SN.val_out = C.nval[ncur ^ 1];
    SN.shift = shift;
    sort_pass(SN, s);
    ncur ^= 1;
  }
  exclusive_scan(HeadF{C.nkey[ncur]}, m, C.hscan, nullptr, B, s);
  hipLaunchKernelGGL(k_ct_heads, dim3(blocks_of(m)), dim3(kBlock), 0, s, C, C.nkey[ncur]);
  hipLaunchKernelGGL(k_ct_reps, dim3(blocks_of(m)), dim3(kBlock), 0, s, C, C.nkey[ncur],
                     C.nval[ncur]);

  // 6. coarse net CSR in representative order
  exclusive_scan(KeptF{C.rep}, m, C.nid, &sizes[1], B, s);
  exclusive_scan(KeptSizeF{C.rep, C.nsize}, m, C.npos, &sizes[2], B, s);
  hipLaunchKernelGGL(k_ct_emit, dim3(blocks_of(m * kEmitLanes)), dim3(kBlock), 0, s, C);
  hipLaunchKernelGGL(k_ct_close, dim3(1), dim3(kWave), 0, s, C);
  return hipGetLastError();
}

}  // namespace hg

using hg::fail;

extern "C" {

size_t hg_contract_workspace_size(int32_t n, int32_t m, int64_t P) {
  if (n < 1 || m < 1 || P < 1 || P > 0x7fffffffLL) return 0;
  return hg::contract_workspace_size(n, m, P);
}

hg_status hg_contract(hg_graph g, const int32_t* cluster, int32_t* map, int32_t* cvwgt,
                      int64_t* ceptr, int32_t* cpins, int32_t* cewgt, int64_t* sizes,
                      void* workspace, size_t ws_bytes, void* stream) {
  if (!g) return fail(HG_ERR_INVALID, "graph handle is NULL");
  if (!cluster || !map || !cvwgt || !ceptr || !cpins || !cewgt || !sizes)
    return fail(HG_ERR_INVALID, "cluster, map, cvwgt, ceptr, cpins, cewgt and sizes must be "
                                "non-NULL");
  if (g->P > 0x7fffffffLL)
    return fail(HG_ERR_UNSUPPORTED, "contraction needs fewer than 2^31 pins");
  const size_t need = hg::contract_workspace_size(g->n, g->m, g->P);
  if (!workspace || ws_bytes < need)
    return fail(HG_ERR_WORKSPACE, "contraction workspace needs %zu bytes (got %zu)", need,
                ws_bytes);
  if (((uintptr_t)workspace & 255) != 0)
    return fail(HG_ERR_INVALID, "the contraction workspace must be 256-byte aligned");
  HG_TRY(hg::launch_contract(g, cluster, map, cvwgt, (long long*)ceptr, cpins, cewgt,
                             (long long*)sizes, (char*)workspace, (hipStream_t)stream),
         "contraction");
  return HG_OK;
}

}  // extern "C"
