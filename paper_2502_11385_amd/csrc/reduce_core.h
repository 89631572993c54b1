// Fixed-order FP64 summation helpers shared by the reduction kernels.
#pragma once
#include "device_common.h"

namespace qsv {

// -------------------------------------------------- compensated summation

__device__ __forceinline__ void nadd(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

// Fixed-order tree reduction of (s, c) pairs over a 256-thread block.
__device__ __forceinline__ void block_reduce_pair(double& s, double& c, double* sh) {
  const int t = threadIdx.x;
  sh[t] = s;
  sh[256 + t] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      double s2 = sh[t], c2 = sh[256 + t];
      nadd(s2, c2, sh[t + w]);
      c2 += sh[256 + t + w];
      sh[t] = s2;
      sh[256 + t] = c2;
    }
    __syncthreads();
  }
  s = sh[0];
  c = sh[256];
}

template <typename C>
__device__ __forceinline__ double prob_of(C v) {
  // one rounding order in every kernel that computes it (the fused
  // multiply-add written out, not left to contraction)
  const double x = double(v.x), y = double(v.y);
  return __builtin_fma(x, x, y * y);
}

}  // namespace qsv
