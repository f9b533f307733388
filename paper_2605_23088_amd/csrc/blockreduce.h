// Fixed-order workgroup reductions (bitwise reproducible run to run).
//
// Each 64-lane wavefront first combines its values with a butterfly of
// cross-lane exchanges (no LDS, no barrier); lane 0's result of each wavefront
// then goes through LDS and the wavefronts' values are added in index order.
// The association order is fixed, so the results are reproducible.
#pragma once

#include "common.h"

namespace yasps {

constexpr int WAVE = 64;

template <class OP>
YDEV double wave_reduce(double v, OP op) {
#pragma unroll
  for (int m = WAVE / 2; m > 0; m >>= 1) v = op(v, __shfl_xor(v, m, WAVE));
  return v;
}

template <int BLOCK, class OP>
YDEV double block_reduce(double v, double* lds, OP op) {
  static_assert(BLOCK % WAVE == 0, "workgroups are whole wavefronts");
  v = wave_reduce(v, op);
  if ((threadIdx.x & (WAVE - 1)) == 0) lds[threadIdx.x / WAVE] = v;
  __syncthreads();
  double r = lds[0];
#pragma unroll
  for (int k = 1; k < BLOCK / WAVE; ++k) r = op(r, lds[k]);
  __syncthreads();  // lds may be reused right away
  return r;
}

// Every thread must call these; every thread gets the result.
template <int BLOCK>
YDEV double block_sum(double v, double* lds) {
  return block_reduce<BLOCK>(v, lds, [](double a, double b) { return a + b; });
}

template <int BLOCK>
YDEV double block_min(double v, double* lds) {
  return block_reduce<BLOCK>(v, lds, [](double a, double b) { return fmin(a, b); });
}

template <int BLOCK>
YDEV double block_max(double v, double* lds) {
  return block_reduce<BLOCK>(v, lds, [](double a, double b) { return fmax(a, b); });
}

}  // namespace yasps
