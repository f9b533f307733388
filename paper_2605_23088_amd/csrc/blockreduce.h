// Fixed-order workgroup reductions (bitwise reproducible run to run).
#pragma once

#include "common.h"

namespace yasps {

// Sum of one double per thread over a workgroup of BLOCK threads, combined in a
// fixed binary tree in LDS.  Every thread must call it; thread 0 gets the sum.
template <int BLOCK>
YDEV double block_sum(double v, double* lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (t < s) lds[t] = lds[t] + lds[t + s];
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

template <int BLOCK>
YDEV double block_min(double v, double* lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (t < s) lds[t] = fmin(lds[t], lds[t + s]);
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

template <int BLOCK>
YDEV double block_max(double v, double* lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (t < s) lds[t] = fmax(lds[t], lds[t + s]);
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

}  // namespace yasps
