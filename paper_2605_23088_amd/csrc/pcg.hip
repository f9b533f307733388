// Block-Jacobi preconditioned conjugate gradient on the symmetric 3x3 BSR
// Hessian (section "Solver", appendices "SpMV" and "Preconditioner").
//
// SpMV.  The Hessian is assembled once, as its upper triangle (appendix
// "Global Hessian Compression"); the paper's SpMV adds, for every off-diagonal
// block, the transposed product with atomics (Algorithm "CUDA Block Level
// SpMV").  Here, after each assembly, a gather pass writes both triangles of
// H_static + H_dynamic row by row in structure-of-arrays form; a group of G
// lanes owns one block row, the lanes read consecutive blocks (coalesced), and
// their partial 3-vectors are combined by a fixed butterfly.  No atomics,
// deterministic; every off-diagonal block is read twice per product (once per
// side), as with full symmetric storage.
//
// Iteration.  PCG with one global reduction phase per iteration (the
// Chronopoulos-Gear arrangement, equal to standard PCG in exact arithmetic):
//   u = M^-1 r, w = H u, gamma = r.u, delta = u.w
//   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev)
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s
// Two kernels per iteration: (B) w = H u and delta, and (C) the scalar
// recurrences, vector updates, preconditioning, the next gamma and |r|^2 and
// the convergence test.  Each kernel's workgroups publish partial sums; the
// workgroup that arrives last (one ticket per workgroup) adds them in index
// order and writes the scalars, so the next kernel reads a few scalars instead
// of re-summing partials in every workgroup.  The sums have a fixed order, so
// the results are bitwise reproducible.  The host only polls a flag every few
// iterations.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "blockreduce.h"
#include "kernels.h"

namespace yasps {

constexpr int SPMV_G = 8;                       // lanes per block row
constexpr int SPMV_ROWS = RED_BLOCK / SPMV_G;  // block rows per workgroup and pass
constexpr int MAX_WG_B = 2048;                  // workgroups of the SpMV kernel
constexpr int MAX_WG_C = 2048;                  // workgroups of the update kernel
constexpr int UPD_VERTS = 64;                   // vertices per update-kernel workgroup pass
constexpr int UPD_BLOCK = 3 * UPD_VERTS;        // update kernel: one thread per vertex component

// Device scalars.  gamma / alpha are double-buffered by iteration parity so a
// kernel never reads a slot that its own last workgroup writes; `iter` counts
// completed iterations (matrix-vector products).  The tickets count arrivals
// of the SpMV (b) and update / init / replacement (c) workgroups and are reset
// by the last arrival.
struct PcgState {
  double gamma[2], alpha[2];
  double delta, bb, rr, tol2;
  int iter, done, status, max_iter;
  int restart_at;  // iteration whose search direction restarts from u (beta = 0)
  unsigned int ticket_b, ticket_c;
};

namespace {

// Called by every thread after thread 0 stored this workgroup's partials:
// true in the workgroup that arrives last, which then sees every partial.
YDEV bool last_arrival(unsigned int* ticket, int* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();  // release: this workgroup's partials before its ticket
    *flag = atomicAdd(ticket, 1u) == gridDim.x - 1 ? 1 : 0;
  }
  __syncthreads();
  const bool last = *flag != 0;
  if (last) __threadfence();  // acquire: the other workgroups' partials
  return last;
}

// Sum of the n partials in a fixed order (strided per thread, then a fixed
// tree), read through the device-coherent path.
template <int BLOCK>
YDEV double sum_partials(const double* part, int n, double* lds) {
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += BLOCK) acc += __hip_atomic_load(part + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return block_sum<BLOCK>(acc, lds);
}

// The last workgroup's bookkeeping of a gamma / |r|^2 reduction for iteration i:
// store both, test convergence (and the iteration cap), reset the ticket.
template <int BLOCK>
YDEV void finish_gamma(PcgState* st, const double* part_c, int i, bool first_iteration, double* lds) {
  const int nb = gridDim.x;
  const double G = sum_partials<BLOCK>(part_c, nb, lds);
  const double R = sum_partials<BLOCK>(part_c + nb, nb, lds);
  if (threadIdx.x == 0) {
    if (first_iteration) st->bb = R;
    const double bb = first_iteration ? R : st->bb;
    st->gamma[i & 1] = G;
    st->rr = R;
    st->iter = i;
    if (R <= st->tol2 * bb) {
      st->status = 0;
      st->done = 1;
    } else if (i >= st->max_iter) {
      st->status = -5;
      st->done = 1;
    }
    st->ticket_c = 0;
  }
}

// (H x)_row for the row owned by this lane group: each lane takes every
// SPMV_G-th block of the row (structure-of-arrays values, so the lanes of a
// group read consecutive addresses); the sum is valid in every lane of the
// group after the butterfly.
template <class T, class X>
YDEV void row_blocks(const PcgMatrix& A, const T* __restrict__ v, int row, int lane, const X* x, double acc[3]) {
  const size_t nnz = (size_t)A.nnz;
  for (int k = A.rp[row] + lane, e = A.rp[row + 1]; k < e; k += SPMV_G) {
    const X* xc = x + 3 * (size_t)A.col[k];
    const double x0 = double(xc[0]), x1 = double(xc[1]), x2 = double(xc[2]);
    const T* b = v + k;
    acc[0] = fma(double(b[0]), x0, fma(double(b[nnz]), x1, fma(double(b[2 * nnz]), x2, acc[0])));
    acc[1] = fma(double(b[3 * nnz]), x0, fma(double(b[4 * nnz]), x1, fma(double(b[5 * nnz]), x2, acc[1])));
    acc[2] = fma(double(b[6 * nnz]), x0, fma(double(b[7 * nnz]), x1, fma(double(b[8 * nnz]), x2, acc[2])));
  }
}

template <class X>
YDEV void spmv_row(const PcgMatrix& A, int row, int lane, const X* x, double acc[3]) {
  acc[0] = acc[1] = acc[2] = 0.0;
  if (row < A.n) {
    if (A.v32)
      row_blocks(A, A.v32, row, lane, x, acc);
    else
      row_blocks(A, A.v, row, lane, x, acc);
  }
#pragma unroll
  for (int m = SPMV_G / 2; m > 0; m >>= 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += __shfl_xor(acc[c], m, SPMV_G);
  }
}

// Krylov vectors in VT (float64, or float32 in the precision form); the
// solution x is always float64.
template <class VT>
struct Vecs {
  VT *r, *u, *w, *p, *s;
  double *part_b, *part_c;  // part_c holds 2 * MAX_WG_C partials
};

YDEV void precondition(const double* minv, int v, const double r[3], double u[3]) {  // u = M^-1 r
  const double* M = minv + 9 * (size_t)v;
  u[0] = M[0] * r[0] + M[1] * r[1] + M[2] * r[2];
  u[1] = M[3] * r[0] + M[4] * r[1] + M[5] * r[2];
  u[2] = M[6] * r[0] + M[7] * r[1] + M[8] * r[2];
}

// r = b, x = 0, p = s = 0, u = M^-1 r; gamma and |r|^2 partials.
template <class VT>
__global__ __launch_bounds__(RED_BLOCK) void pcg_init_kernel(PcgMatrix A, const double* __restrict__ b,
                                                             double* __restrict__ x, Vecs<VT> V, PcgState* st) {
  __shared__ double lds[RED_BLOCK];
  double g = 0.0, rr = 0.0;
  for (int v = blockIdx.x * RED_BLOCK + threadIdx.x; v < A.n; v += gridDim.x * RED_BLOCK) {
    double r[3], u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[c] = double(VT(b[3 * (size_t)v + c]));
      V.r[3 * (size_t)v + c] = VT(r[c]);
      x[3 * (size_t)v + c] = 0.0;
      V.p[3 * (size_t)v + c] = VT(0);
      V.s[3 * (size_t)v + c] = VT(0);
    }
    precondition(A.minv, v, r, u);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const VT uc = VT(u[c]);
      V.u[3 * (size_t)v + c] = uc;
      g = fma(r[c], double(uc), g);
      rr = fma(r[c], r[c], rr);
    }
  }
  const double gs = block_sum<RED_BLOCK>(g, lds);
  const double rs = block_sum<RED_BLOCK>(rr, lds);
  __shared__ int flag;
  if (threadIdx.x == 0) {
    V.part_c[blockIdx.x] = gs;
    V.part_c[gridDim.x + blockIdx.x] = rs;
  }
  if (last_arrival(&st->ticket_c, &flag)) finish_gamma<RED_BLOCK>(st, V.part_c, 0, true, lds);
}

// Residual replacement (precision form): r = b - H x evaluated with float64
// vectors and accumulation, then u = M^-1 r, gamma and |r|^2 of the current
// iteration (replacing what the float32 recurrence carried) and the
// convergence test on this true residual.
template <class VT>
__global__ __launch_bounds__(RED_BLOCK) void pcg_replace_kernel(PcgMatrix A, const double* __restrict__ b,
                                                                const double* __restrict__ x, Vecs<VT> V,
                                                                PcgState* st) {
  if (st->done) return;
  __shared__ double lds[RED_BLOCK];
  const int lane = threadIdx.x % SPMV_G;
  double g = 0.0, rr = 0.0;
  for (int base = blockIdx.x * SPMV_ROWS; base < A.n; base += gridDim.x * SPMV_ROWS) {
    const int row = base + threadIdx.x / SPMV_G;
    double acc[3];
    spmv_row(A, row, lane, x, acc);
    if (lane == 0 && row < A.n) {
      double r[3], u[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = b[3 * (size_t)row + c] - acc[c];
      precondition(A.minv, row, r, u);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const VT rc = VT(r[c]), uc = VT(u[c]);
        V.r[3 * (size_t)row + c] = rc;
        V.u[3 * (size_t)row + c] = uc;
        g = fma(double(rc), double(uc), g);
        rr = fma(r[c], r[c], rr);
      }
    }
  }
  const double gs = block_sum<RED_BLOCK>(g, lds);
  const double rs = block_sum<RED_BLOCK>(rr, lds);
  __shared__ int flag;
  if (threadIdx.x == 0) {
    V.part_c[blockIdx.x] = gs;
    V.part_c[gridDim.x + blockIdx.x] = rs;
  }
  if (last_arrival(&st->ticket_c, &flag)) finish_gamma<RED_BLOCK>(st, V.part_c, st->iter, false, lds);
}

// Iteration i: w = H u and delta = u.w.  standalone: plain y = H x (no
// solver bookkeeping).
template <class VT>
__global__ __launch_bounds__(RED_BLOCK) void pcg_spmv_kernel(PcgMatrix A, Vecs<VT> V, PcgState* st, int standalone) {
  __shared__ double lds[RED_BLOCK];
  __shared__ int flag;
  if (!standalone && st->done) return;
  const int lane = threadIdx.x % SPMV_G;
  double d = 0.0;
  for (int base = blockIdx.x * SPMV_ROWS; base < A.n; base += gridDim.x * SPMV_ROWS) {
    const int row = base + threadIdx.x / SPMV_G;
    double acc[3];
    spmv_row(A, row, lane, V.u, acc);
    if (lane == 0 && row < A.n) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const VT wc = VT(acc[c]);
        V.w[3 * (size_t)row + c] = wc;
        d = fma(double(V.u[3 * (size_t)row + c]), double(wc), d);
      }
    }
  }
  if (standalone) return;
  const double ds = block_sum<RED_BLOCK>(d, lds);
  if (threadIdx.x == 0) V.part_b[blockIdx.x] = ds;
  if (last_arrival(&st->ticket_b, &flag)) {
    const double delta = sum_partials<RED_BLOCK>(V.part_b, gridDim.x, lds);
    if (threadIdx.x == 0) {
      st->delta = delta;
      st->ticket_b = 0;
    }
  }
}

// Iteration i: scalar recurrences, vector updates, preconditioning, then
// gamma / |r|^2 of iteration i + 1 and the convergence test (last workgroup).
// One thread per vertex component (coalesced vector traffic, 3x the threads
// of a per-vertex mapping); the three residual components of a vertex meet in
// LDS for the 3x3 block-Jacobi product.
template <class VT>
__global__ __launch_bounds__(UPD_BLOCK) void pcg_update_kernel(PcgMatrix A, double* __restrict__ x, Vecs<VT> V,
                                                               PcgState* st) {
  if (st->done) return;
  __shared__ double lds[UPD_BLOCK];
  __shared__ double rsh[UPD_BLOCK];
  __shared__ int flag;
  const int i = st->iter;
  const double gamma = st->gamma[i & 1];
  const double delta = st->delta;
  const bool restart = i == st->restart_at;
  const double beta = restart ? 0.0 : gamma / st->gamma[(i - 1) & 1];
  const double pAp = restart ? delta : delta - beta * gamma / st->alpha[(i - 1) & 1];
  const bool broken = !(pAp > 0.0);  // identical in every workgroup
  const double alpha = broken ? 0.0 : gamma / pAp;
  const int t = threadIdx.x;
  const int vl = t / 3, c = t - 3 * (t / 3);
  double g = 0.0, rr = 0.0;
  if (!broken) {
    for (int base = blockIdx.x * UPD_VERTS; base < A.n; base += gridDim.x * UPD_VERTS) {
      const int v = base + vl;
      const bool live = v < A.n;
      const size_t k = 3 * (size_t)base + t;  // = 3 v + c
      double r = 0.0;
      if (live) {
        const VT p = VT(fma(beta, double(V.p[k]), double(V.u[k])));
        const VT sv = VT(fma(beta, double(V.s[k]), double(V.w[k])));
        V.p[k] = p;
        V.s[k] = sv;
        x[k] = fma(alpha, double(p), x[k]);
        const VT rc = VT(fma(-alpha, double(sv), double(V.r[k])));
        V.r[k] = rc;
        r = double(rc);
      }
      rsh[t] = r;
      __syncthreads();
      if (live) {
        const double* M = A.minv + 9 * (size_t)v + 3 * c;  // row c of the vertex's M^-1
        const VT uc = VT(M[0] * rsh[3 * vl] + M[1] * rsh[3 * vl + 1] + M[2] * rsh[3 * vl + 2]);
        V.u[k] = uc;
        g = fma(r, double(uc), g);
        rr = fma(r, r, rr);
      }
      __syncthreads();  // rsh is rewritten by the next pass
    }
  }
  const double gs = block_sum<UPD_BLOCK>(g, lds);
  const double rs = block_sum<UPD_BLOCK>(rr, lds);
  if (threadIdx.x == 0) {
    V.part_c[blockIdx.x] = gs;
    V.part_c[gridDim.x + blockIdx.x] = rs;
  }
  if (last_arrival(&st->ticket_c, &flag)) {
    if (broken) {
      if (threadIdx.x == 0) {
        st->status = -6;
        st->done = 1;
        st->ticket_c = 0;
      }
    } else {
      if (threadIdx.x == 0) st->alpha[i & 1] = alpha;
      finish_gamma<UPD_BLOCK>(st, V.part_c, i + 1, false, lds);
    }
  }
}

int grid_b(int n) { return std::max(1, std::min((n + SPMV_ROWS - 1) / SPMV_ROWS, MAX_WG_B)); }
int grid_c(int n) { return std::max(1, std::min((n + UPD_VERTS - 1) / UPD_VERTS, MAX_WG_C)); }

template <class VT>
void carve(void* work, int n, PcgState*& st, Vecs<VT>& V) {
  const size_t n3 = 3 * (size_t)n;
  char* w = static_cast<char*>(work);
  st = reinterpret_cast<PcgState*>(w);
  double* parts = reinterpret_cast<double*>(w + ((sizeof(PcgState) + 255) / 256) * 256);
  V.part_b = parts;
  V.part_c = parts + MAX_WG_B;
  VT* base = reinterpret_cast<VT*>(parts + MAX_WG_B + 2 * MAX_WG_C);
  V.r = base;
  V.u = V.r + n3;
  V.w = V.u + n3;
  V.p = V.w + n3;
  V.s = V.p + n3;
}

}  // namespace

size_t pcg_workspace_bytes(int n) {
  const size_t n3 = 3 * (size_t)std::max(n, 1);
  return 256 + ((sizeof(PcgState) + 255) / 256) * 256 + sizeof(double) * (5 * n3 + MAX_WG_B + 2 * MAX_WG_C);
}  // float64 vectors; the float32 form uses half of the vector part

void launch_spmv(const PcgMatrix& A, const double* x, double* y, void* work, hipStream_t s) {
  if (A.n == 0) return;
  PcgState* st;
  Vecs<double> V;
  carve(work, A.n, st, V);
  V.u = const_cast<double*>(x);
  V.w = y;
  hipLaunchKernelGGL(pcg_spmv_kernel<double>, dim3(grid_b(A.n)), dim3(RED_BLOCK), 0, s, A, V, st, 1);
}

namespace {

template <class VT>
int pcg_run(const PcgMatrix& A, const double* b, double* x, double rtol, int max_iter, void* work, double* rel_out,
            int* status_out, hipStream_t s, LaunchTimer* tm) {
  constexpr bool MIXED = sizeof(VT) == 4;
  constexpr int REPLACE_EVERY = 50;  // float64 residual replacement period (precision form)
  const int n = A.n;
  PcgState* st;
  Vecs<VT> V;
  carve(work, n, st, V);
  const int nb_b = grid_b(n), nb_c = grid_c(n);
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
  hipLaunchKernelGGL(pcg_init_kernel<VT>, dim3(nb_c), dim3(RED_BLOCK), 0, s, A, b, x, V, st);
  if (tm) tm->end();
  int batch = 8;
  long long launched = 0;  // (SpMV, update) pairs issued (the replacement period counts these)
  PcgState hs{};
  int verified_at = -1;
  int restarts = 0;
  constexpr int MAX_RESTARTS = 32;
  for (;;) {
    for (int k = 0; k < batch; ++k) {
      if (tm) tm->begin(5);
      hipLaunchKernelGGL(pcg_spmv_kernel<VT>, dim3(nb_b), dim3(RED_BLOCK), 0, s, A, V, st, 0);
      if (tm) tm->end();
      if (tm) tm->begin(6);
      hipLaunchKernelGGL(pcg_update_kernel<VT>, dim3(nb_c), dim3(UPD_BLOCK), 0, s, A, x, V, st);
      if (tm) tm->end();
      ++launched;
      if (MIXED && launched % REPLACE_EVERY == 0) {
        if (tm) tm->begin(5);
        hipLaunchKernelGGL(pcg_replace_kernel<VT>, dim3(nb_c), dim3(RED_BLOCK), 0, s, A, b, x, V, st);
        if (tm) tm->end();
      }
    }
    if (hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s) != hipSuccess) return -2;
    if (hipStreamSynchronize(s) != hipSuccess) return -2;
    if (hs.done && MIXED && hs.status == -6 && restarts < MAX_RESTARTS) {
      // float32 recurrence lost positivity of p^T H p: restart the search
      // direction from a float64 true residual at the same iterate
      ++restarts;
      PcgState fix = hs;
      fix.done = 0;
      fix.status = 0;
      fix.restart_at = hs.iter;
      fix.iter = hs.iter;
      if (hipMemcpyAsync(st, &fix, sizeof(fix), hipMemcpyHostToDevice, s) != hipSuccess) return -2;
      hipLaunchKernelGGL(pcg_replace_kernel<VT>, dim3(nb_c), dim3(RED_BLOCK), 0, s, A, b, x, V, st);
      launched = hs.iter;
      batch = 8;
      continue;
    }
    if (hs.done) {
      if (!MIXED || hs.status != 0 || verified_at == hs.iter) break;
      // converged on the recurrence residual: confirm with a float64 true residual
      verified_at = hs.iter;
      const int zero = 0;
      if (hipMemcpyAsync(&st->done, &zero, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess) return -2;
      hipLaunchKernelGGL(pcg_replace_kernel<VT>, dim3(nb_c), dim3(RED_BLOCK), 0, s, A, b, x, V, st);
      launched = hs.iter;
      batch = 8;
      continue;
    }
    batch = std::min(batch * 2, 64);
  }
  *rel_out = hs.bb > 0.0 ? sqrt(hs.rr / hs.bb) : 0.0;
  *status_out = hs.status;
  return hs.iter;
}

}  // namespace

int pcg_solve(const PcgMatrix& A, const double* b, double* x, double rtol, int max_iter, bool mixed, void* work,
              double* rel_out, int* status_out, hipStream_t s, LaunchTimer* tm) {
  return mixed ? pcg_run<float>(A, b, x, rtol, max_iter, work, rel_out, status_out, s, tm)
               : pcg_run<double>(A, b, x, rtol, max_iter, work, rel_out, status_out, s, tm);
}

}  // namespace yasps
