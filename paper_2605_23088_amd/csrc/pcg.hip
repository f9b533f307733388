// Block-Jacobi preconditioned conjugate gradient on the symmetric 3x3 BSR
// Hessian (section "Solver", appendices "SpMV" and "Preconditioner").
//
// SpMV.  The Hessian is stored once, as its upper triangle (appendix "Global
// Hessian Compression"); the paper's SpMV adds, for every off-diagonal block,
// the transposed product with atomics (Algorithm "CUDA Block Level SpMV").
// Here a group of G lanes owns one block row and gathers both its row blocks
// (B x_col) and, through a precomputed transpose index, the blocks whose
// column is this row (B^T x_row); the lanes' partial 3-vectors are combined by
// a fixed butterfly.  No atomics, deterministic, and every block is read twice
// (once per side), the same traffic as full symmetric storage without storing it.
//
// Iteration.  PCG with one global reduction phase per iteration (the
// Chronopoulos-Gear arrangement, equal to standard PCG in exact arithmetic):
//   u = M^-1 r, w = H u, gamma = r.u, delta = u.w
//   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev)
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s
// Two kernels per iteration: (B) w = H u with the delta partials, and (C) the
// scalar recurrences, vector updates, preconditioning and the next gamma and
// |r|^2 partials.  The last workgroup of each kernel (detected with a counter)
// sums the partials in a fixed order, so results are bitwise reproducible.
// Convergence is tested on the device; the host only polls a flag every few
// iterations.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "blockreduce.h"
#include "kernels.h"

namespace yasps {

constexpr int SPMV_G = 8;                       // lanes per block row
constexpr int SPMV_ROWS = RED_BLOCK / SPMV_G;  // block rows per workgroup

struct PcgState {
  double gamma, gamma_prev, delta, rr, bb, alpha, tol2;
  int iter, done, status, max_iter;
  unsigned int counter_b, counter_c;
};

namespace {

YDEV double load_relaxed(const double* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Sum of the partials by the last workgroup to finish (fixed order).
YDEV bool last_block(unsigned int* counter) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  return last;
}

YDEV double sum_partials(const double* part, int n, double* lds) {
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += RED_BLOCK) acc += load_relaxed(part + j);
  return block_sum<RED_BLOCK>(acc, lds);
}

template <class T>
YDEV void block_mv(const T* B, const double* x, double acc[3]) {
  const double x0 = x[0], x1 = x[1], x2 = x[2];
  acc[0] = fma(double(B[0]), x0, fma(double(B[1]), x1, fma(double(B[2]), x2, acc[0])));
  acc[1] = fma(double(B[3]), x0, fma(double(B[4]), x1, fma(double(B[5]), x2, acc[1])));
  acc[2] = fma(double(B[6]), x0, fma(double(B[7]), x1, fma(double(B[8]), x2, acc[2])));
}
template <class T>
YDEV void block_mtv(const T* B, const double* x, double acc[3]) {
  const double x0 = x[0], x1 = x[1], x2 = x[2];
  acc[0] = fma(double(B[0]), x0, fma(double(B[3]), x1, fma(double(B[6]), x2, acc[0])));
  acc[1] = fma(double(B[1]), x0, fma(double(B[4]), x1, fma(double(B[7]), x2, acc[1])));
  acc[2] = fma(double(B[2]), x0, fma(double(B[5]), x1, fma(double(B[8]), x2, acc[2])));
}

template <class T>
YDEV void row_part(const int32_t* rp, const int32_t* ci, const T* v, const int32_t* tp, const int32_t* ts,
                   const int32_t* tr, int row, int lane, const double* x, double acc[3]) {
  for (int k = rp[row] + lane, e = rp[row + 1]; k < e; k += SPMV_G) block_mv(v + 9 * (size_t)k, x + 3 * (size_t)ci[k], acc);
  for (int k = tp[row] + lane, e = tp[row + 1]; k < e; k += SPMV_G)
    block_mtv(v + 9 * (size_t)ts[k], x + 3 * (size_t)tr[k], acc);
}

// y_row = (H x)_row for the row owned by this lane group; valid in lane 0 of the group.
YDEV void spmv_row(const PcgMatrix& A, int row, int lane, const double* x, double acc[3]) {
  acc[0] = acc[1] = acc[2] = 0.0;
  if (row < A.n) {
    if (A.v_s32)
      row_part(A.rp_s, A.ci_s, A.v_s32, A.tp_s, A.tslot_s, A.trow_s, row, lane, x, acc);
    else
      row_part(A.rp_s, A.ci_s, A.v_s, A.tp_s, A.tslot_s, A.trow_s, row, lane, x, acc);
    if (A.rp_d) {
      if (A.v_d32)
        row_part(A.rp_d, A.ci_d, A.v_d32, A.tp_d, A.tslot_d, A.trow_d, row, lane, x, acc);
      else
        row_part(A.rp_d, A.ci_d, A.v_d, A.tp_d, A.tslot_d, A.trow_d, row, lane, x, acc);
    }
  }
#pragma unroll
  for (int m = SPMV_G / 2; m > 0; m >>= 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += __shfl_xor(acc[c], m, SPMV_G);
  }
}

struct Vecs {
  double *r, *u, *w, *p, *s, *part_b, *part_c;  // part_c holds 2 * nblocks_c partials
};

YDEV void precondition(const double* minv, int v, const double r[3], double u[3]) {
  const double* M = minv + 9 * (size_t)v;
  u[0] = M[0] * r[0] + M[1] * r[1] + M[2] * r[2];
  u[1] = M[3] * r[0] + M[4] * r[1] + M[5] * r[2];
  u[2] = M[6] * r[0] + M[7] * r[1] + M[8] * r[2];
}

// r = b, x = 0, p = s = 0, u = M^-1 r; gamma, |r|^2 partials.
__global__ __launch_bounds__(RED_BLOCK) void pcg_init_kernel(PcgMatrix A, const double* __restrict__ b,
                                                             double* __restrict__ x, Vecs V, PcgState* st) {
  __shared__ double lds[RED_BLOCK];
  const int v = blockIdx.x * RED_BLOCK + threadIdx.x;
  double g = 0.0, rr = 0.0;
  if (v < A.n) {
    double r[3], u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = b[3 * (size_t)v + c];
      V.r[3 * (size_t)v + c] = r[c];
      x[3 * (size_t)v + c] = 0.0;
      V.p[3 * (size_t)v + c] = 0.0;
      V.s[3 * (size_t)v + c] = 0.0;
    }
    precondition(A.minv, v, r, u);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      V.u[3 * (size_t)v + c] = u[c];
      g = fma(r[c], u[c], g);
      rr = fma(r[c], r[c], rr);
    }
  }
  const double gs = block_sum<RED_BLOCK>(g, lds);
  const double rs = block_sum<RED_BLOCK>(rr, lds);
  if (threadIdx.x == 0) {
    V.part_c[blockIdx.x] = gs;
    V.part_c[gridDim.x + blockIdx.x] = rs;
  }
  if (last_block(&st->counter_c)) {
    const double G = sum_partials(V.part_c, gridDim.x, lds);
    const double R = sum_partials(V.part_c + gridDim.x, gridDim.x, lds);
    if (threadIdx.x == 0) {
      st->gamma = G;
      st->gamma_prev = 1.0;
      st->rr = R;
      st->bb = R;
      st->alpha = 1.0;
      st->iter = 0;
      st->status = 0;
      st->done = (R <= st->tol2 * R) ? 1 : 0;
      if (!st->done && st->max_iter <= 0) {
        st->done = 1;
        st->status = -5;
      }
      st->counter_c = 0;
    }
  }
}

// w = H u, delta partials.
__global__ __launch_bounds__(RED_BLOCK) void pcg_spmv_kernel(PcgMatrix A, Vecs V, PcgState* st) {
  if (st->done) return;
  __shared__ double lds[RED_BLOCK];
  const int row = blockIdx.x * SPMV_ROWS + threadIdx.x / SPMV_G;
  const int lane = threadIdx.x % SPMV_G;
  double acc[3];
  spmv_row(A, row, lane, V.u, acc);
  double d = 0.0;
  if (lane == 0 && row < A.n) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      V.w[3 * (size_t)row + c] = acc[c];
      d = fma(V.u[3 * (size_t)row + c], acc[c], d);
    }
  }
  const double ds = block_sum<RED_BLOCK>(d, lds);
  if (threadIdx.x == 0) V.part_b[blockIdx.x] = ds;
  if (last_block(&st->counter_b)) {
    const double D = sum_partials(V.part_b, gridDim.x, lds);
    if (threadIdx.x == 0) {
      st->delta = D;
      st->counter_b = 0;
    }
  }
}

__global__ __launch_bounds__(RED_BLOCK) void pcg_update_kernel(PcgMatrix A, double* __restrict__ x, Vecs V,
                                                               PcgState* st) {
  if (st->done) return;
  __shared__ double lds[RED_BLOCK];
  const double gamma = st->gamma, delta = st->delta;
  const int iter = st->iter;
  const double beta = iter == 0 ? 0.0 : gamma / st->gamma_prev;
  const double pAp = iter == 0 ? delta : delta - beta * gamma / st->alpha;
  const bool breakdown = !(pAp > 0.0);
  const double alpha = gamma / pAp;
  const int v = blockIdx.x * RED_BLOCK + threadIdx.x;
  double g = 0.0, rr = 0.0;
  if (v < A.n && !breakdown) {
    double r[3], u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t i = 3 * (size_t)v + c;
      const double p = fma(beta, V.p[i], V.u[i]);
      const double s = fma(beta, V.s[i], V.w[i]);
      V.p[i] = p;
      V.s[i] = s;
      x[i] = fma(alpha, p, x[i]);
      r[c] = fma(-alpha, s, V.r[i]);
      V.r[i] = r[c];
    }
    precondition(A.minv, v, r, u);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      V.u[3 * (size_t)v + c] = u[c];
      g = fma(r[c], u[c], g);
      rr = fma(r[c], r[c], rr);
    }
  }
  const double gs = block_sum<RED_BLOCK>(g, lds);
  const double rs = block_sum<RED_BLOCK>(rr, lds);
  if (threadIdx.x == 0) {
    V.part_c[blockIdx.x] = gs;
    V.part_c[gridDim.x + blockIdx.x] = rs;
  }
  if (last_block(&st->counter_c)) {
    const double G = sum_partials(V.part_c, gridDim.x, lds);
    const double R = sum_partials(V.part_c + gridDim.x, gridDim.x, lds);
    if (threadIdx.x == 0) {
      if (breakdown) {
        st->done = 1;
        st->status = -6;
      } else {
        st->gamma_prev = gamma;
        st->gamma = G;
        st->rr = R;
        st->alpha = alpha;
        st->iter = iter + 1;
        if (R <= st->tol2 * st->bb) {
          st->done = 1;
        } else if (iter + 1 >= st->max_iter) {
          st->done = 1;
          st->status = -5;
        }
      }
      st->counter_c = 0;
    }
  }
}

}  // namespace

size_t pcg_workspace_bytes(int n) {
  const size_t n3 = 3 * (size_t)std::max(n, 1);
  const size_t nb_b = ((size_t)n + SPMV_ROWS - 1) / SPMV_ROWS + 1;
  const size_t nb_c = ((size_t)n + RED_BLOCK - 1) / RED_BLOCK + 1;
  return sizeof(PcgState) + 256 + sizeof(double) * (5 * n3 + nb_b + 2 * nb_c) + 256;
}

namespace {

void carve(void* work, int n, PcgState*& st, Vecs& V) {
  const size_t n3 = 3 * (size_t)n;
  char* w = static_cast<char*>(work);
  st = reinterpret_cast<PcgState*>(w);
  double* base = reinterpret_cast<double*>(w + ((sizeof(PcgState) + 255) / 256) * 256);
  const int nb_b = (n + SPMV_ROWS - 1) / SPMV_ROWS;
  V.r = base;
  V.u = V.r + n3;
  V.w = V.u + n3;
  V.p = V.w + n3;
  V.s = V.p + n3;
  V.part_b = V.s + n3;
  V.part_c = V.part_b + nb_b + 1;
}

}  // namespace

void launch_spmv(const PcgMatrix& A, const double* x, double* y, void* work, hipStream_t s) {
  if (A.n == 0) return;
  PcgState* st;
  Vecs V;
  carve(work, A.n, st, V);
  V.u = const_cast<double*>(x);
  V.w = y;
  (void)hipMemsetAsync(st, 0, sizeof(PcgState), s);
  hipLaunchKernelGGL(pcg_spmv_kernel, dim3((A.n + SPMV_ROWS - 1) / SPMV_ROWS), dim3(RED_BLOCK), 0, s, A, V, st);
}

int pcg_solve(const PcgMatrix& A, const double* b, double* x, double rtol, int max_iter, bool mixed, void* work,
              double* rel_out, int* status_out, hipStream_t s, LaunchTimer* tm) {
  (void)mixed;
  const int n = A.n;
  PcgState* st;
  Vecs V;
  carve(work, n, st, V);
  const int nb_b = (n + SPMV_ROWS - 1) / SPMV_ROWS;
  const int nb_c = (n + RED_BLOCK - 1) / RED_BLOCK;
  PcgState h{};
  h.tol2 = rtol * rtol;
  h.max_iter = max_iter;
  if (hipMemcpyAsync(st, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess) return -2;
  if (n == 0) {
    *rel_out = 0.0;
    *status_out = 0;
    return 0;
  }
  if (tm) tm->begin(6);
  hipLaunchKernelGGL(pcg_init_kernel, dim3(nb_c), dim3(RED_BLOCK), 0, s, A, b, x, V, st);
  if (tm) tm->end();
  int batch = 8;
  PcgState hs{};
  for (;;) {
    for (int k = 0; k < batch; ++k) {
      if (tm) tm->begin(5);
      hipLaunchKernelGGL(pcg_spmv_kernel, dim3(nb_b), dim3(RED_BLOCK), 0, s, A, V, st);
      if (tm) tm->end();
      if (tm) tm->begin(6);
      hipLaunchKernelGGL(pcg_update_kernel, dim3(nb_c), dim3(RED_BLOCK), 0, s, A, x, V, st);
      if (tm) tm->end();
    }
    if (hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s) != hipSuccess) return -2;
    if (hipStreamSynchronize(s) != hipSuccess) return -2;
    if (hs.done) break;
    batch = std::min(batch * 2, 64);
  }
  *rel_out = hs.bb > 0.0 ? sqrt(hs.rr / hs.bb) : 0.0;
  *status_out = hs.status;
  return hs.iter;
}

}  // namespace yasps
