// hg_contract.hip -- contraction of a vertex clustering into a coarse
// hypergraph (section "Coarsening", subsection "Contraction"), as a second
// HBM-bound workload beside refinement.
//
//   1. used cluster ids are flagged and renumbered by a prefix sum (the
//      rank of the id among the used ones): map[v];
//   2. coarse vertex weights by integer atomics;
//   3. every pin is mapped; a stable radix sort by the mapped pin and then
//      by the net id sorts the pins inside every net while keeping the nets
//      where they were (net e still owns positions eptr[e] .. eptr[e+1]);
//      the first occurrence of each pin survives (a prefix sum compacts
//      them);
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
  unsigned* pkey[2];     // [P]
  int* pval[2];          // [P]
  long long* dpos;       // [P]: compacted position of a surviving pin
  int* dp;               // [P]: surviving pins, net by net
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

// Sort input: key = mapped pin, value = its net (binary search in eptr).
__global__ __launch_bounds__(kBlock) void k_ct_pin_keys(Ct C) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= C.P) return;
  int lo = 0, hi = C.m - 1;     // net: last e with eptr[e] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (C.eptr[mid] <= i) lo = mid; else hi = mid - 1;
  }
  const int v = C.pins[i];
  C.pkey[0][i] = (unsigned)((unsigned)v < (unsigned)C.n ? C.map[v] : 0);
  C.pval[0][i] = lo;
}

// After both sorts: pins (sorted in their net) in `pin`, nets in `net`.
struct FirstF {
  const int* pin;
  const unsigned* net;
  __device__ long long operator()(long long i) const {
    return i == 0 || net[i] != net[i - 1] || pin[i] != pin[i - 1];
  }
};

__global__ __launch_bounds__(kBlock) void k_ct_compact(Ct C, const int* pin, const unsigned* net) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= C.P) return;
  if (i == 0 || net[i] != net[i - 1] || pin[i] != pin[i - 1]) C.dp[C.dpos[i]] = pin[i];
}

__device__ __forceinline__ unsigned ct_hash(unsigned long long fp, int size) {
  unsigned long long h = fp * 0x9E3779B97F4A7C15ULL + (unsigned long long)size * 0xC2B2AE3D27D4EB4FULL;
  h ^= h >> 29;
  h *= 0xBF58476D1CE4E5B9ULL;
  h ^= h >> 32;
  return (unsigned)h;
}

// Per net: identity order for the net sort, no representative yet.
__global__ __launch_bounds__(kBlock) void k_ct_nets(Ct C) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= C.m) return;
  C.nval[0][e] = (int)e;
  C.rep[e] = -1;
  C.wsum[e] = 0;
}

// Per net: surviving size, fingerprint, sort key (dropped nets: all ones).
// The last net ends at the total of the first-occurrence scan.
__global__ __launch_bounds__(kBlock) void k_ct_fingerprints(Ct C, const long long* dtotal) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= C.m) return;
  const long long b = C.dpos[C.eptr[e]];
  const long long t = e + 1 < C.m ? C.dpos[C.eptr[e + 1]] : *dtotal;
  const int size = (int)(t - b);
  unsigned long long fp = 0;
  for (long long j = b; j < t; ++j) {
    const unsigned long long v = (unsigned)C.dp[j];
    fp += v * v;
  }
  C.nsize[e] = size;
  C.fp[e] = fp;
  C.nkey[0][e] = size >= 2 ? ct_hash(fp, size) : 0xffffffffu;
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
    if (C.dp[be + x] != C.dp[bf + x]) return false;
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
  const long long be = C.dpos[C.eptr[e]];
  int r = e;
  for (long long i = h; i < j; ++i) {
    const int f = val[i];
    if (C.nsize[f] != size || C.fp[f] != fe) continue;
    if (ct_same(C, be, C.dpos[C.eptr[f]], size)) {
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

__global__ __launch_bounds__(kBlock) void k_ct_emit(Ct C) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= C.m || C.rep[e] != e) return;
  const long long id = C.nid[e], pos = C.npos[e];
  const long long b = C.dpos[C.eptr[e]];
  const int size = C.nsize[e];
  C.ceptr[id] = pos;
  C.cewgt[id] = (int)C.wsum[e];
  for (int x = 0; x < size; ++x) C.cpins[pos + x] = C.dp[b + x];
}

__global__ void k_ct_close(Ct C) {
  if (threadIdx.x == 0) C.ceptr[C.sizes[1]] = C.sizes[2];
}

}  // namespace

struct ContractLayout {
  size_t used, rank, cw, pkey[2], pval[2], dpos, dp, nsize, fp, nkey[2], nval[2], hscan, heads,
      rep, wsum, nid, npos, csum, coff, phist, pdtot, nhist, ndtot, dtotal, total;
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
  for (int i = 0; i < 2; ++i) {
    L.pkey[i] = take(4 * (size_t)P);
    L.pval[i] = take(4 * (size_t)P);
    L.nkey[i] = take(4 * (size_t)m);
    L.nval[i] = take(4 * (size_t)m);
  }
  L.dpos = take(8 * (size_t)P);
  L.dp = take(4 * (size_t)P);
  L.nsize = take(4 * (size_t)m);
  L.fp = take(8 * (size_t)m);
  L.hscan = take(8 * (size_t)m);
  L.heads = take(4 * (size_t)m);
  L.rep = take(4 * (size_t)m);
  L.wsum = take(4 * (size_t)m);
  L.nid = take(8 * (size_t)m);
  L.npos = take(8 * (size_t)m);
  long long most = n > m ? n : m;
  if (P > most) most = P;
  L.csum = take(8 * (size_t)scan_chunks(most));
  L.coff = take(8 * (size_t)scan_chunks(most));
  L.phist = take(4 * (size_t)kDigits * sort_tiles(P));
  L.pdtot = take(4 * (size_t)kDigits);
  L.nhist = take(4 * (size_t)kDigits * sort_tiles(m));
  L.ndtot = take(4 * (size_t)kDigits);
  L.dtotal = take(8);
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

static int bits_for(long long max_value) {
  int b = 1;
  while (b < 32 && (1ll << b) <= max_value) ++b;
  return b;
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
    C.pkey[i] = (unsigned*)(ws + L.pkey[i]);
    C.pval[i] = (int*)(ws + L.pval[i]);
    C.nkey[i] = (unsigned*)(ws + L.nkey[i]);
    C.nval[i] = (int*)(ws + L.nval[i]);
  }
  C.dpos = (long long*)(ws + L.dpos);
  C.dp = (int*)(ws + L.dp);
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
  long long* dtotal = (long long*)(ws + L.dtotal);
  const long long n = g->n, m = g->m, P = g->P;

  // 1-2. renumbering, map, coarse weights
  hipError_t e = fill_u8(C.used, 0, n, s);
  if (e == hipSuccess) e = fill_i64((long long*)C.cw, 0, n, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ct_mark, dim3(blocks_of(n)), dim3(kBlock), 0, s, C);
  exclusive_scan(UsedF{C.used}, n, C.rank, &sizes[0], B, s);
  hipLaunchKernelGGL(k_ct_map, dim3(blocks_of(n)), dim3(kBlock), 0, s, C);
  hipLaunchKernelGGL(k_ct_vweights, dim3(blocks_of(n)), dim3(kBlock), 0, s, C);

  // 3. mapped pins sorted inside their nets: by pin, then (stably) by net
  hipLaunchKernelGGL(k_ct_pin_keys, dim3(blocks_of(P)), dim3(kBlock), 0, s, C);
  int cur = 0;
  SortPass SP;
  SP.hist = (unsigned*)(ws + L.phist);
  SP.dtot = (unsigned*)(ws + L.pdtot);
  SP.n = (int)P;
  SP.tiles = sort_tiles(P);
  const int pin_bits = bits_for(n - 1), net_bits = bits_for(m - 1);
  for (int shift = 0; shift < pin_bits; shift += 8) {
    SP.key_in = C.pkey[cur];
    SP.val_in = C.pval[cur];
    SP.key_out = C.pkey[cur ^ 1];
    SP.val_out = C.pval[cur ^ 1];
    SP.shift = shift;
    sort_pass(SP, s);
    cur ^= 1;
  }
  // the same buffers with the roles swapped: key = net, value = pin
  for (int shift = 0; shift < net_bits; shift += 8) {
    SP.key_in = (const unsigned*)C.pval[cur];
    SP.val_in = (const int*)C.pkey[cur];
    SP.key_out = (unsigned*)C.pval[cur ^ 1];
    SP.val_out = (int*)C.pkey[cur ^ 1];
    SP.shift = shift;
    sort_pass(SP, s);
    cur ^= 1;
  }
  const unsigned* pnet = (const unsigned*)C.pval[cur];
  const int* ppin = (const int*)C.pkey[cur];
  exclusive_scan(FirstF{ppin, pnet}, P, C.dpos, dtotal, B, s);
  hipLaunchKernelGGL(k_ct_compact, dim3(blocks_of(P)), dim3(kBlock), 0, s, C, ppin, pnet);

  // 4-5. sizes, fingerprints, identical nets
  hipLaunchKernelGGL(k_ct_nets, dim3(blocks_of(m)), dim3(kBlock), 0, s, C);
  hipLaunchKernelGGL(k_ct_fingerprints, dim3(blocks_of(m)), dim3(kBlock), 0, s, C,
                     (const long long*)dtotal);
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
  hipLaunchKernelGGL(k_ct_emit, dim3(blocks_of(m)), dim3(kBlock), 0, s, C);
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
