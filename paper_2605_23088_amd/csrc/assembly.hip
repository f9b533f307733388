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

// Short segments (the static blocks: bounded valence): a workgroup takes SPW
// consecutive segments, whose contributions are contiguous in the staging
// array.  It copies them to LDS in rounds of CAP contributions with plain
// coalesced loads (every thread issues its share of a round before any is
// stored), and thread (segment, component) then adds its segment's values in
// contribution order.  Every output is a sequential sum over its segment, so
// the result does not depend on SPW or CAP.
template <class T, int W, int SPW, int CAP>
__global__ __launch_bounds__(RED_BLOCK) void segsum_lds_kernel(int nseg, const int32_t* __restrict__ ptr,
                                                               const T* __restrict__ stg, T* __restrict__ out) {
  static_assert(SPW * W <= RED_BLOCK, "one output per thread");
  constexpr int PER = (CAP * W + RED_BLOCK - 1) / RED_BLOCK;
  __shared__ T buf[CAP * W];
  const int t = threadIdx.x;
  const int s_lo = blockIdx.x * SPW;
  const int s_hi = min(s_lo + SPW, nseg);
  const int seg = s_lo + t / W, comp = t - W * (t / W);
  const bool mine = t < SPW * W && seg < s_hi;
  const int c0 = ptr[s_lo], c1 = ptr[s_hi];
  int j = mine ? ptr[seg] : 0;
  const int je = mine ? ptr[seg + 1] : 0;
  double acc = 0.0;
  for (int base = c0; base < c1; base += CAP) {
    const int m = W * min(CAP, c1 - base);
    const T* src = stg + (size_t)W * base;
    T v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = t + i * RED_BLOCK;
      v[i] = q < m ? src[q] : T(0);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int q = t + i * RED_BLOCK;
      if (q < m) buf[q] = v[i];
    }
    __syncthreads();
    const int lim = min(je, base + CAP);
    for (; j < lim; ++j) acc += double(buf[W * (j - base) + comp]);
    __syncthreads();  // buf is refilled by the next round
  }
  if (mine) out[(size_t)W * seg + comp] = T(acc);
}

// acc += contributions j, j + G, ... below e, in that order; four are loaded
// before any is added (more loads in flight on long segments).
template <class T, int W, int G>
YDEV void lane_sum(int j, int e, const T* __restrict__ stg, double acc[W]) {
  for (; j + 3 * G < e; j += 4 * G) {
    T v[4][W];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < W; ++c) v[u][c] = stg[(size_t)W * (j + u * G) + c];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < W; ++c) acc[c] += double(v[u][c]);
  }
  for (; j < e; j += G) {
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] += double(stg[(size_t)W * j + c]);
  }
}

// Long or skewed segments (contacts, gradient rows): a group of G lanes per
// segment: lane l sums contributions l, l + G, ... of its segment (W values
// each, contiguous, so a group reads G consecutive contributions per step),
// then the group combines its partial sums with a fixed butterfly and lane 0
// writes the W results.  Up to three ranges (static, dynamic and body-contact
// parts of the gradient) may be chained per segment.
template <class T, int W, int G>
__global__ __launch_bounds__(RED_BLOCK) void segsum_kernel(int nseg, const int32_t* __restrict__ p1,
                                                           const T* __restrict__ s1, const int32_t* __restrict__ p2,
                                                           const T* __restrict__ s2, const int32_t* __restrict__ p3,
                                                           const T* __restrict__ s3, T* __restrict__ out) {
  const int seg = (blockIdx.x * RED_BLOCK + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  double acc[W];
#pragma unroll
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
  if (seg < nseg) {
    lane_sum<T, W, G>(p1[seg] + lane, p1[seg + 1], s1, acc);
    if (p2) lane_sum<T, W, G>(p2[seg] + lane, p2[seg + 1], s2, acc);
    if (p3) lane_sum<T, W, G>(p3[seg] + lane, p3[seg + 1], s3, acc);
  }
#pragma unroll
  for (int m = G / 2; m > 0; m >>= 1) {
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] += __shfl_xor(acc[c], m, G);
  }
  if (seg < nseg && lane == 0) {
#pragma unroll
    for (int c = 0; c < W; ++c) out[(size_t)W * seg + c] = T(acc[c]);
  }
}

// group size from the mean segment length (power of two in [4, 64])
int group_for(long long items, int nseg) {
  const double mean = nseg > 0 ? double(items) / nseg : 1.0;
  int g = 4;
  while (g < 64 && g < mean) g *= 2;
  return g;
}

template <class T, int W>
void launch_segsum(int nseg, const int32_t* p1, const T* s1, const int32_t* p2, const T* s2, T* out, int G,
                   hipStream_t s, const int32_t* p3 = nullptr, const T* s3 = nullptr) {
  if (nseg == 0) return;
  const size_t threads = (size_t)nseg * G;
  const dim3 grid((unsigned)((threads + RED_BLOCK - 1) / RED_BLOCK)), b(RED_BLOCK);
  switch (G) {
    case 4: hipLaunchKernelGGL((segsum_kernel<T, W, 4>), grid, b, 0, s, nseg, p1, s1, p2, s2, p3, s3, out); break;
    case 8: hipLaunchKernelGGL((segsum_kernel<T, W, 8>), grid, b, 0, s, nseg, p1, s1, p2, s2, p3, s3, out); break;
    case 16: hipLaunchKernelGGL((segsum_kernel<T, W, 16>), grid, b, 0, s, nseg, p1, s1, p2, s2, p3, s3, out); break;
    case 32: hipLaunchKernelGGL((segsum_kernel<T, W, 32>), grid, b, 0, s, nseg, p1, s1, p2, s2, p3, s3, out); break;
    default: hipLaunchKernelGGL((segsum_kernel<T, W, 64>), grid, b, 0, s, nseg, p1, s1, p2, s2, p3, s3, out); break;
  }
}

// Slots of at most this mean number of contributions go to the LDS kernel.
constexpr double LDS_MEAN_MAX = 24.0;
constexpr int BLK_SPW = RED_BLOCK / 9, BLK_CAP = 256;  // 28 slots, 18 KiB (float64) per round

template <class T>
void launch_block_sums(int nslots, long long ncontrib, const int32_t* cptr, const T* staged, T* out,
                       hipStream_t s) {
  if (nslots == 0) return;
  if (ncontrib <= LDS_MEAN_MAX * nslots) {
    hipLaunchKernelGGL((segsum_lds_kernel<T, 9, BLK_SPW, BLK_CAP>), dim3((nslots + BLK_SPW - 1) / BLK_SPW),
                       dim3(RED_BLOCK), 0, s, nslots, cptr, staged, out);
  } else {
    launch_segsum<T, 9>(nslots, cptr, staged, nullptr, nullptr, out, group_for(ncontrib, nslots), s);
  }
}

template <class T>
__global__ __launch_bounds__(RED_BLOCK) void mass_shift_kernel(int n, const int32_t* __restrict__ rp,
                                                               const double* __restrict__ mass, double shift,
                                                               T* __restrict__ vals) {
  const int v = blockIdx.x * RED_BLOCK + threadIdx.x;
  if (v >= n) return;
  T* B = vals + 9 * (size_t)rp[v];
  const T d = T(shift * mass[v]);
  B[0] += d;
  B[4] += d;
  B[8] += d;
}

template <class T>
__global__ __launch_bounds__(RED_BLOCK) void block_inverse_kernel(int n, const int32_t* __restrict__ rp_s,
                                                                  const T* __restrict__ vs,
                                                                  const int32_t* __restrict__ ddiag,
                                                                  const T* __restrict__ vd, double* __restrict__ inv,
                                                                  uint32_t* flags, const int32_t* __restrict__ bdiag,
                                                                  const T* __restrict__ vb) {
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
  if (bdiag) {
    const int bd = bdiag[v];
    if (bd >= 0) {
#pragma unroll
      for (int k = 0; k < 9; ++k) D[k] += double(vb[9 * (size_t)bd + k]);
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
  for (int k = blockIdx.x; k < f.nseg; k += gridDim.x) {  // one workgroup per segment
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

__global__ __launch_bounds__(RED_BLOCK) void axpy_to_dev_kernel(int n3, const double* __restrict__ x,
                                                                const double* __restrict__ a,
                                                                const double* __restrict__ p,
                                                                double* __restrict__ y) {
  const int i = blockIdx.x * RED_BLOCK + threadIdx.x;
  if (i < n3) y[i] = fma(*a, p[i], x[i]);
}

__global__ void step_bound_kernel(const double* __restrict__ min_d, const double* __restrict__ pmax, int contacts,
                                  double* __restrict__ out) {
  const double pm = *pmax;
  double a = 1.0;
  if (contacts && pm > 0.0) a = fmin(1.0, 0.4 * sqrt(*min_d) / pm);
  *out = a;
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

void launch_segsum_blocks(int nslots, long long ncontrib, const int32_t* cptr, const double* staged, double* out,
                          hipStream_t s) {
  launch_block_sums<double>(nslots, ncontrib, cptr, staged, out, s);
}

void launch_segsum_blocks_f32(int nslots, long long ncontrib, const int32_t* cptr, const float* staged, float* out,
                              hipStream_t s) {
  launch_block_sums<float>(nslots, ncontrib, cptr, staged, out, s);
}

void launch_segsum_grad(int n, long long ncontrib, const int32_t* gptr_s, const double* stg_s,
                        const int32_t* gptr_d, const double* stg_d, double* grad, hipStream_t s,
                        const int32_t* gptr_b, const double* stg_b) {
  launch_segsum<double, 3>(n, gptr_s, stg_s, gptr_d, stg_d, grad, group_for(ncontrib, n), s, gptr_b, stg_b);
}

void launch_add_mass_shift(int n, const int32_t* row_ptr_s, const double* mass, double shift, double* vals_s,
                           float* vals_s32, hipStream_t s) {
  if (n == 0 || shift == 0.0) return;
  const dim3 grid((n + RED_BLOCK - 1) / RED_BLOCK);
  if (vals_s32)
    hipLaunchKernelGGL((mass_shift_kernel<float>), grid, dim3(RED_BLOCK), 0, s, n, row_ptr_s, mass, shift, vals_s32);
  else
    hipLaunchKernelGGL((mass_shift_kernel<double>), grid, dim3(RED_BLOCK), 0, s, n, row_ptr_s, mass, shift, vals_s);
}

namespace {

// ratio[v] = |tr(D_v)| / (3 m_v), D_v the assembled diagonal block (static + dynamic)
template <class T>
__global__ __launch_bounds__(RED_BLOCK) void diag_ratio_kernel(int n, const int32_t* __restrict__ rp_s,
                                                               const T* __restrict__ vs,
                                                               const int32_t* __restrict__ ddiag,
                                                               const T* __restrict__ vd,
                                                               const int32_t* __restrict__ bdiag,
                                                               const T* __restrict__ vb,
                                                               const double* __restrict__ mass,
                                                               double* __restrict__ ratio) {
  const int v = blockIdx.x * RED_BLOCK + threadIdx.x;
  if (v >= n) return;
  const T* d = vs + 9 * (size_t)rp_s[v];
  double tr = double(d[0]) + double(d[4]) + double(d[8]);
  if (ddiag && ddiag[v] >= 0) {
    const T* e = vd + 9 * (size_t)ddiag[v];
    tr += double(e[0]) + double(e[4]) + double(e[8]);
  }
  if (bdiag && bdiag[v] >= 0) {
    const T* e = vb + 9 * (size_t)bdiag[v];
    tr += double(e[0]) + double(e[4]) + double(e[8]);
  }
  ratio[v] = fabs(tr) / (3.0 * mass[v]);
}

}  // namespace

void launch_diag_ratio(int n, const int32_t* row_ptr_s, const void* vals_s, const int32_t* ddiag, const void* vals_d,
                       const int32_t* bdiag, const void* vals_b, bool f32, const double* mass, double* ratio,
                       hipStream_t s) {
  if (n == 0) return;
  const dim3 g((n + RED_BLOCK - 1) / RED_BLOCK), b(RED_BLOCK);
  if (f32)
    hipLaunchKernelGGL((diag_ratio_kernel<float>), g, b, 0, s, n, row_ptr_s, static_cast<const float*>(vals_s), ddiag,
                       static_cast<const float*>(vals_d), bdiag, static_cast<const float*>(vals_b), mass, ratio);
  else
    hipLaunchKernelGGL((diag_ratio_kernel<double>), g, b, 0, s, n, row_ptr_s, static_cast<const double*>(vals_s),
                       ddiag, static_cast<const double*>(vals_d), bdiag, static_cast<const double*>(vals_b), mass,
                       ratio);
}

void launch_block_inverse(int n, const int32_t* row_ptr_s, const double* vals_s, const int32_t* ddiag,
                          const double* vals_d, double* inv, uint32_t* flags, hipStream_t s, const int32_t* bdiag,
                          const double* vals_b) {
  if (n == 0) return;
  hipLaunchKernelGGL((block_inverse_kernel<double>), dim3((n + RED_BLOCK - 1) / RED_BLOCK), dim3(RED_BLOCK), 0, s,
                     n, row_ptr_s, vals_s, ddiag, vals_d, inv, flags, bdiag, vals_b);
}

void launch_block_inverse_f32(int n, const int32_t* row_ptr_s, const float* vals_s, const int32_t* ddiag,
                              const float* vals_d, double* inv, uint32_t* flags, hipStream_t s,
                              const int32_t* bdiag, const float* vals_b) {
  if (n == 0) return;
  hipLaunchKernelGGL((block_inverse_kernel<float>), dim3((n + RED_BLOCK - 1) / RED_BLOCK), dim3(RED_BLOCK), 0, s,
                     n, row_ptr_s, vals_s, ddiag, vals_d, inv, flags, bdiag, vals_b);
}

void launch_finalize(int nseg, const int* off_host, const double* parts, const int* kind_host, double* out,
                     hipStream_t s) {
  FinalizeArgs f{};
  f.nseg = nseg;
  for (int k = 0; k <= nseg; ++k) f.off[k] = off_host[k];
  for (int k = 0; k < nseg; ++k) f.kind[k] = kind_host[k];
  hipLaunchKernelGGL(finalize_kernel, dim3(std::max(nseg, 1)), dim3(RED_BLOCK), 0, s, f, parts, out);
}

void launch_axpy_to(int n3, const double* x, double alpha, const double* p, double* y, hipStream_t s) {
  if (n3 == 0) return;
  hipLaunchKernelGGL(axpy_to_kernel, dim3((n3 + RED_BLOCK - 1) / RED_BLOCK), dim3(RED_BLOCK), 0, s, n3, x,
                     alpha, p, y);
}

void launch_axpy_to_dev(int n3, const double* x, const double* alpha, const double* p, double* y, hipStream_t s) {
  if (n3 == 0) return;
  hipLaunchKernelGGL(axpy_to_dev_kernel, dim3((n3 + RED_BLOCK - 1) / RED_BLOCK), dim3(RED_BLOCK), 0, s, n3, x,
                     alpha, p, y);
}

void launch_step_bound(const double* min_d, const double* pmax, int contacts, double* out, hipStream_t s) {
  hipLaunchKernelGGL(step_bound_kernel, dim3(1), dim3(1), 0, s, min_d, pmax, contacts, out);
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
