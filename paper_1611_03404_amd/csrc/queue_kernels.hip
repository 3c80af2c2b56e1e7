// Device work queue of a fit iteration (the batching of section III-C's many uneven sources on
// one device): the work items of the sources still being fitted are compacted into one list,
// so that persistent pixel kernels draw only their work.
#include "celeste_internal.h"

namespace celeste {

namespace {

constexpr int QB = 1024;   // threads of the builder (one block)

// Exclusive block scan of one int per thread (Hillis-Steele in LDS); returns the thread's
// prefix and writes the block total to *total.
__device__ int block_scan(int v, int* sh, int* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < QB; o <<= 1) {
    const int a = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const int incl = sh[t];
  *total = sh[QB - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(QB) void k_build_queue(WorkQueue q, int n_src, const int* __restrict__ flag) {
  __shared__ int sh[QB];
  const int t = threadIdx.x;
  const int per = (n_src + QB - 1) / QB;
  const int s0 = min(n_src, t * per), s1 = min(n_src, s0 + per);
  int ni = 0;
  for (int s = s0; s < s1; ++s)
    if (flag[s]) ni += q.srcs[s].item_end - q.srcs[s].item_begin;
  int total;
  int o = block_scan(ni, sh, &total);
  for (int s = s0; s < s1; ++s)
    if (flag[s]) {
      const SrcDev sd = q.srcs[s];
      for (int it = sd.item_begin; it < sd.item_end; ++it) q.items[o++] = it;
    }
  if (t == 0) {
    q.hdr[0] = total;
    q.hdr[1] = 0;
  }
}

}  // namespace

hipError_t launch_build_queue(WorkQueue q, int n_src, const int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_build_queue, dim3(1), dim3(QB), 0, st, q, n_src, flag);
  return hipGetLastError();
}

}  // namespace celeste
