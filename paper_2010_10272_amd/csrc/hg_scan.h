// hg_scan.h -- exclusive prefix sums (int64) of n values f(0) .. f(n-1)
// given by a device functor, in three launches: per-chunk sums, one
// workgroup scanning the chunk sums (and writing the grand total), and the
// chunk scans plus their offsets.  A chunk is 1024 values, four consecutive
// ones per thread.  Included by each source file that scans (the kernels
// have internal linkage there).
#pragma once

#include "hg_device.h"
#include "hg_internal.h"

namespace hg {
namespace {

constexpr int kScanChunk = 4 * kBlock;
constexpr int kScanPer = kScanChunk / kBlock;

template <class F>
__global__ __launch_bounds__(kBlock) void k_scan_sums(F f, long long n, long long* csum) {
  __shared__ long long s_tmp[kBlock / kWave];
  const long long base = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanPer;
  long long v = 0;
#pragma unroll
  for (int r = 0; r < kScanPer; ++r)
    if (base + r < n) v += f(base + r);
  v = block_sum64(v, s_tmp);
  if (threadIdx.x == 0) csum[blockIdx.x] = v;
}

__global__ __launch_bounds__(kBlock) void k_scan_top(const long long* csum, long long* coff,
                                                     long long chunks, long long* total) {
  __shared__ long long s_tmp[kBlock / kWave];
  long long carry = 0;
  for (long long b = 0; b < chunks; b += kBlock) {
    const long long i = b + threadIdx.x;
    const long long v = i < chunks ? csum[i] : 0;
    long long tot;
    const long long ex = block_excl_scan64(v, s_tmp, &tot);
    if (i < chunks) coff[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <class F>
__global__ __launch_bounds__(kBlock) void k_scan_out(F f, long long n, const long long* coff,
                                                     long long* out) {
  __shared__ long long s_tmp[kBlock / kWave];
  const long long base = (long long)blockIdx.x * kScanChunk + (long long)threadIdx.x * kScanPer;
  long long v[kScanPer];
  long long sum = 0;
#pragma unroll
  for (int r = 0; r < kScanPer; ++r) {
    v[r] = base + r < n ? f(base + r) : 0;
    sum += v[r];
  }
  long long tot;
  long long run = coff[blockIdx.x] + block_excl_scan64(sum, s_tmp, &tot);
#pragma unroll
  for (int r = 0; r < kScanPer; ++r) {
    if (base + r < n) out[base + r] = run;
    run += v[r];
  }
}

struct ScanBufs {
  long long* csum;   // [scan_chunks(n)]
  long long* coff;   // [scan_chunks(n)]
};

inline long long scan_chunks(long long n) { return n < 1 ? 1 : (n + kScanChunk - 1) / kScanChunk; }

// out[i] = f(0) + .. + f(i-1); *total (device, may be null) = the sum of all.
template <class F>
inline void exclusive_scan(F f, long long n, long long* out, long long* total, ScanBufs B,
                           hipStream_t s) {
  const long long chunks = scan_chunks(n);
  hipLaunchKernelGGL(k_scan_sums<F>, dim3((unsigned)chunks), dim3(kBlock), 0, s, f, n, B.csum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, B.csum, B.coff, chunks, total);
  hipLaunchKernelGGL(k_scan_out<F>, dim3((unsigned)chunks), dim3(kBlock), 0, s, f, n, B.coff,
                     out);
}

}  // namespace
}  // namespace hg
