// Atomic-free assembly, block-Jacobi inverse, reductions and vector helpers.
//
// The paper accumulates every local block into its global slot with atomic
// additions (appendix "Global Hessian Compression", "Assembly").  Here the
// stencil kernels write each contribution to a staging array at a position
// precomputed from the slot map, grouped by destination slot, so assembly is a
// streaming segmented sum in a fixed order: no atomics, bitwise reproducible,
// and the only scattered accesses are the writes of the compute-bound stencil
// kernels.  The diagonal blocks are inverted independently for the block-Jacobi
// preconditioner (appendix "Preconditioner").
#include "blockreduce.h"
#include "kernels.h"

namespace yasps {

namespace {

// One thread per (slot, component): out[9 k + c] = sum_j staged[9 j + c],
// j over the slot's contiguous contribution range.
template <class T, class ACC>
__global__ __launch_bounds__(RED_BLOCK) void segsum_blocks_kernel(int nslots, const int32_t* __restrict__ cptr,
                                                                  const T* __restrict__ stg, T* __restrict__ out) {
  const size_t t = (size_t)blockIdx.x * RED_BLOCK + threadIdx.x;
  if (t >= (size_t)nslots * 9) return;
  const int k = (int)(t / 9), c = (int)(t % 9);
  const int b = cptr[k], e = cptr[k + 1];
  ACC acc = ACC(0);
  for (int j = b; j < e; ++j) acc += ACC(stg[9 * (size_t)j + c]);
  out[t] = T(acc);
}

__global__ __launch_bounds__(RED_BLOCK) void segsum_grad_kernel(int n, const int32_t* __restrict__ gs,
                                                                const double* __restrict__ ss,
                                                                const int32_t* __restrict__ gd,
                                                                const double* __restrict__ sd,
                                                                double* __restrict__ grad) {
  const size_t t = (size_t)blockIdx.x * RED_BLOCK + threadIdx.x;
  if (t >= (size_t)n * 3) return;
  const int v = (int)(t / 3), c = (int)(t % 3);
  double acc = 0.0;
  for (int j = gs[v], e = gs[v + 1]; j < e; ++j) acc += ss[3 * (size_t)j + c];
  if (gd)
    for (int j = gd[v], e = gd[v + 1]; j < e; ++j) acc += sd[3 * (size_t)j + c];
  grad[t] = acc;
}

template <class T>
__global__ __launch_bounds__(RED_BLOCK) void block_inverse_kernel(int n, const int32_t* __restrict__ rp_s,
                                                                  const T* __restrict__ vs,
                                                                  const int32_t* __restrict__ ddiag,
                                                                  const T* __restrict__ vd, double* __restrict__ inv,
                                                                  uint32_t* flags) {
  const int v = blockIdx.x * RED_BLOCK + threadIdx.x;
  if (v >= n) return;
  double D[9];
  const T* s = vs + 9 * (size_t)rp_s[v];
#pragma unroll
  for (int k = 0; k < 9; ++k) D[k] = double(s[k]);
  if (ddiag) {
    const int dd = ddiag[v];
    if (dd >= 0) {
#pragma unroll
      for (int k = 0; k < 9; ++k) D[k] += double(vd[9 * (size_t)dd + k]);
    }
  }
  // adjugate / determinant; the block is symmetric, so compute the upper
  // cofactors and mirror them
  const double c00 = D[4] * D[8] - D[5] * D[7];
  const double c01 = D[2] * D[7] - D[1] * D[8];
  const double c02 = D[1] * D[5] - D[2] * D[4];
  const double c11 = D[0] * D[8] - D[2] * D[6];
  const double c12 = D[2] * D[3] - D[0] * D[5];
  const double c22 = D[0] * D[4] - D[1] * D[3];
  const double det = D[0] * c00 + D[1] * (D[5] * D[6] - D[3] * D[8]) + D[2] * (D[3] * D[7] - D[4] * D[6]);
  const double id = 1.0 / det;
  double* o = inv + 9 * (size_t)v;
  o[0] = c00 * id;
  o[1] = c01 * id;
  o[2] = c02 * id;
  o[3] = c01 * id;
  o[4] = c11 * id;
  o[5] = c12 * id;
  o[6] = c02 * id;
  o[7] = c12 * id;
  o[8] = c22 * id;
  if (!finite(id)) atomicOr(flags, FLAG_NONFINITE);
}

constexpr int MAX_SEG = 8;
struct FinalizeArgs {
  int nseg;
  int off[MAX_SEG + 1];
  int kind[MAX_SEG];  // 0 sum, 1 min, 2 max
};

__global__ __launch_bounds__(RED_BLOCK) void finalize_kernel(FinalizeArgs f, const double* __restrict__ parts,
                                                             double* __restrict__ out) {
  __shared__ double lds[RED_BLOCK];
  for (int k = 0; k < f.nseg; ++k) {
    const int kind = f.kind[k];
    double acc = kind == 0 ? 0.0 : (kind == 1 ? __builtin_inf() : -__builtin_inf());
    for (int j = f.off[k] + threadIdx.x; j < f.off[k + 1]; j += RED_BLOCK) {
      const double p = parts[j];
      acc = kind == 0 ? acc + p : (kind == 1 ? fmin(acc, p) : fmax(acc, p));
    }
    double r;
    if (kind == 0)
      r = block_sum<RED_BLOCK>(acc, lds);
    else if (kind == 1)
      r = block_min<RED_BLOCK>(acc, lds);
    else
      r = block_max<RED_BLOCK>(acc, lds);
    if (threadIdx.x == 0) out[k] = r;
  }
}

__global__ __launch_bounds__(RED_BLOCK) void axpy_to_kernel(int n3, const double* __restrict__ x, double a,
                                                            const double* __restrict__ p, double* __restrict__ y) {
  const int i = blockIdx.x * RED_BLOCK + threadIdx.x;
  if (i < n3) y[i] = fma(a, p[i], x[i]);
}

__global__ __launch_bounds__(RED_BLOCK) void scale_kernel(int n3, const double* __restrict__ x, double a,
                                                          double* __restrict__ y) {
  const int i = blockIdx.x * RED_BLOCK + threadIdx.x;
  if (i < n3) y[i] = a * x[i];
}

// per-workgroup max |p_v| (slot 0) and partial g.p is done elsewhere
__global__ __launch_bounds__(RED_BLOCK) void max_norm3_kernel(int n, const double* __restrict__ p,
                                                              double* __restrict__ part) {
  __shared__ double lds[RED_BLOCK];
  const int v = blockIdx.x * RED_BLOCK + threadIdx.x;
  double m = 0.0;
  if (v < n) {
    const double a = p[3 * (size_t)v], b = p[3 * (size_t)v + 1], c = p[3 * (size_t)v + 2];
    m = sqrt(a * a + b * b + c * c);
  }
  const double r = block_max<RED_BLOCK>(m, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(RED_BLOCK) void dot_kernel(int n3, const double* __restrict__ a,
                                                        const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double lds[RED_BLOCK];
  double acc = 0.0;
  for (int i = blockIdx.x * RED_BLOCK + threadIdx.x; i < n3; i += gridDim.x * RED_BLOCK) acc = fma(a[i], b[i], acc);
  const double r = block_sum<RED_BLOCK>(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

}  // namespace

void launch_dot(int n3, const double* a, const double* b, double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(nblk), dim3(RED_BLOCK), 0, s, n3, a, b, part);
}

void launch_segsum_blocks(int nslots, const int32_t* cptr, const double* staged, double* out, hipStream_t s) {
  if (nslots == 0) return;
  const size_t nt = (size_t)nslots * 9;
  hipLaunchKernelGGL((segsum_blocks_kernel<double, double>), dim3((nt + RED_BLOCK - 1) / RED_BLOCK),
                     dim3(RED_BLOCK), 0, s, nslots, cptr, staged, out);
}

void launch_segsum_blocks_f32(int nslots, const int32_t* cptr, const float* staged, float* out, hipStream_t s) {
  if (nslots == 0) return;
  const size_t nt = (size_t)nslots * 9;
  hipLaunchKernelGGL((segsum_blocks_kernel<float, float>), dim3((nt + RED_BLOCK - 1) / RED_BLOCK),
                     dim3(RED_BLOCK), 0, s, nslots, cptr, staged, out);
}

void launch_segsum_grad(int n, const int32_t* gptr_s, const double* stg_s, const int32_t* gptr_d,
                        const double* stg_d, double* grad, hipStream_t s) {
  if (n == 0) return;
  const size_t nt = (size_t)n * 3;
  hipLaunchKernelGGL(segsum_grad_kernel, dim3((nt + RED_BLOCK - 1) / RED_BLOCK), dim3(RED_BLOCK), 0, s, n,
                     gptr_s, stg_s, gptr_d, stg_d, grad);
}

void launch_block_inverse(int n, const int32_t* row_ptr_s, const double* vals_s, const int32_t* ddiag,
                          const double* vals_d, double* inv, uint32_t* flags, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((block_inverse_kernel<double>), dim3((n + RED_BLOCK - 1) / RED_BLOCK), dim3(RED_BLOCK), 0, s,
                     n, row_ptr_s, vals_s, ddiag, vals_d, inv, flags);
}

void launch_block_inverse_f32(int n, const int32_t* row_ptr_s, const float* vals_s, const int32_t* ddiag,
                              const float* vals_d, double* inv, uint32_t* flags, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((block_inverse_kernel<float>), dim3((n + RED_BLOCK - 1) / RED_BLOCK), dim3(RED_BLOCK), 0, s,
                     n, row_ptr_s, vals_s, ddiag, vals_d, inv, flags);
}

void launch_finalize(int nseg, const int* off_host, const double* parts, const int* kind_host, double* out,
                     hipStream_t s) {
  FinalizeArgs f{};
  f.nseg = nseg;
  for (int k = 0; k <= nseg; ++k) f.off[k] = off_host[k];
  for (int k = 0; k < nseg; ++k) f.kind[k] = kind_host[k];
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(RED_BLOCK), 0, s, f, parts, out);
}

void launch_axpy_to(int n3, const double* x, double alpha, const double* p, double* y, hipStream_t s) {
  if (n3 == 0) return;
  hipLaunchKernelGGL(axpy_to_kernel, dim3((n3 + RED_BLOCK - 1) / RED_BLOCK), dim3(RED_BLOCK), 0, s, n3, x,
                     alpha, p, y);
}

void launch_scale(int n3, const double* x, double a, double* y, hipStream_t s) {
  if (n3 == 0) return;
  hipLaunchKernelGGL(scale_kernel, dim3((n3 + RED_BLOCK - 1) / RED_BLOCK), dim3(RED_BLOCK), 0, s, n3, x, a, y);
}

void launch_max_norm3(int n, const double* p, double* part, int nblk, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(max_norm3_kernel, dim3(nblk), dim3(RED_BLOCK), 0, s, n, p, part);
}

}  // namespace yasps
