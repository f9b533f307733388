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
// Two kernels per iteration: (B) the convergence test and w = H u with the
// delta partials, and (C) the scalar recurrences, vector updates,
// preconditioning and the next gamma and |r|^2 partials.  Each kernel runs a
// bounded grid (grid-stride loops) and every workgroup re-sums the previous
// kernel's partials in the same fixed order, so there are no atomics and the
// results are bitwise reproducible.  Convergence is tested on the device; the
// host only polls a flag every few iterations.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "blockreduce.h"
#include "kernels.h"

namespace yasps {

// Launch shapes (compile-time; the defaults come from sweeps on the 40^3 and
// 80x80x52 workloads).
#ifndef YASPS_SPMV_NARROW_MEAN
#define YASPS_SPMV_NARROW_MEAN 20
#endif
#ifndef YASPS_MAX_WG_B
#define YASPS_MAX_WG_B 4096
#endif
#ifndef YASPS_MAX_WG_C
#define YASPS_MAX_WG_C 512
#endif
#ifndef YASPS_UPD_VERTS
#define YASPS_UPD_VERTS 128
#endif
// Lanes per block row of the SpMV-shaped kernels: 8 when the full rows hold at
// most SPMV_NARROW_MEAN blocks on average (tet meshes: about 15), else 16
// (cloth with contacts: about 29); block rows per workgroup and pass =
// RED_BLOCK / lanes.
constexpr int SPMV_NARROW_MEAN = YASPS_SPMV_NARROW_MEAN;
constexpr int MAX_WG_B = YASPS_MAX_WG_B;        // workgroups of the SpMV kernel
constexpr int MAX_WG_C = YASPS_MAX_WG_C;        // workgroups of the update kernel
constexpr int UPD_VERTS = YASPS_UPD_VERTS;      // vertices per update-kernel workgroup pass
constexpr int UPD_BLOCK = 3 * UPD_VERTS;        // update kernel: one thread per vertex component

// Device scalars.  gamma / alpha are double-buffered by iteration parity;
// `iter` is written only by the update kernel and `iter_b` only by the SpMV
// kernel, so no kernel reads a scalar that it also writes.
struct PcgState {
  double gamma[2], alpha[2];
  double bb, rr, tol2;
  int iter, iter_b, done, status, max_iter;
  int restart_at;  // iteration whose search direction restarts from u (beta = 0)
};

namespace {

// The block rows of the SpMV-shaped kernels are split into NXCD contiguous
// ranges of equal work (A.xsplit), one per XCD: workgroups are dispatched to
// the XCDs round robin by index, so workgroup b runs on XCD b % NXCD and makes
// passes over that XCD's range.  The column gathers of one XCD then stay near
// its own rows (mesh locality) and in its own L2.  These kernels' grids are
// multiples of NXCD.
constexpr int NXCD = PCG_XCDS;
static_assert(MAX_WG_B % NXCD == 0 && MAX_WG_C % NXCD == 0, "partial-sum arrays hold the rounded grids");
struct RowRange {
  int end, first, stride;
};
template <int G>
YDEV RowRange xcd_rows(const PcgMatrix& A) {
  constexpr int ROWS = RED_BLOCK / G;
  const int xcd = blockIdx.x % NXCD, j = blockIdx.x / NXCD, per = gridDim.x / NXCD;
  RowRange r;
  r.end = A.xsplit[xcd + 1];
  r.first = A.xsplit[xcd] + j * ROWS;
  r.stride = per * ROWS;
  return r;
}

// (H x)_row for the row owned by this lane group: each lane takes every
// G-th entry of the full row, reads the stored upper block that the entry
// names (9 contiguous values; transposed for an entry below the diagonal, so
// every stored block is read by its own row and by its column's row, the
// second time from L2 when the rows are near each other; a far entry names
// its transposed copy instead) and the gathered x; the sum is valid in every
// lane of the group after the butterfly.
template <int G, class X>
YDEV void row_blocks(const PcgMatrix& A, int row, int lane, const X* x, double acc[3]) {
  const double* __restrict__ vals = A.vals;
  for (int k = A.rp[row] + lane, e = A.rp[row + 1]; k < e; k += G) {
    const int32_t sk = A.src[k];
    const bool tr = sk < 0;
    const double* p = vals + 9 * (size_t)(tr ? -sk - 1 : sk);
    const X* xc = x + 3 * (size_t)A.col[k];
    double B[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) B[q] = p[q];
    const double b01 = tr ? B[3] : B[1], b02 = tr ? B[6] : B[2], b10 = tr ? B[1] : B[3];
    const double b12 = tr ? B[7] : B[5], b20 = tr ? B[2] : B[6], b21 = tr ? B[5] : B[7];
    const double x0 = double(xc[0]), x1 = double(xc[1]), x2 = double(xc[2]);
    acc[0] = fma(B[0], x0, fma(b01, x1, fma(b02, x2, acc[0])));
    acc[1] = fma(b10, x0, fma(B[4], x1, fma(b12, x2, acc[1])));
    acc[2] = fma(b20, x0, fma(b21, x1, fma(B[8], x2, acc[2])));
  }
}

// Precision form: each lane takes every G-th entry of the row from the
// float32 structure-of-arrays copy (the lanes of a group read consecutive
// addresses).
template <int G, class X>
YDEV void row_blocks_f32(const PcgMatrix& A, int row, int lane, const X* x, double acc[3]) {
  const size_t nnz = (size_t)A.nnz;
  for (int k = A.rp[row] + lane, e = A.rp[row + 1]; k < e; k += G) {
    const X* xc = x + 3 * (size_t)A.col[k];
    const double x0 = double(xc[0]), x1 = double(xc[1]), x2 = double(xc[2]);
    const float* b = A.v32 + k;
    acc[0] = fma(double(b[0]), x0, fma(double(b[nnz]), x1, fma(double(b[2 * nnz]), x2, acc[0])));
    acc[1] = fma(double(b[3 * nnz]), x0, fma(double(b[4 * nnz]), x1, fma(double(b[5 * nnz]), x2, acc[1])));
    acc[2] = fma(double(b[6 * nnz]), x0, fma(double(b[7 * nnz]), x1, fma(double(b[8 * nnz]), x2, acc[2])));
  }
}

// MF32: the precision form's float32 copy (a compile-time choice, so that
// each kernel carries the registers of one layout only).
template <bool MF32, int G, class X>
YDEV void spmv_row(const PcgMatrix& A, int row, int lane, const X* x, double acc[3]) {
  acc[0] = acc[1] = acc[2] = 0.0;
  if (row < A.n) {
    if constexpr (MF32)
      row_blocks_f32<G>(A, row, lane, x, acc);
    else
      row_blocks<G>(A, row, lane, x, acc);
  }
#pragma unroll
  for (int m = G / 2; m > 0; m >>= 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += __shfl_xor(acc[c], m, G);
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
  if (threadIdx.x == 0) {
    V.part_c[blockIdx.x] = gs;
    V.part_c[gridDim.x + blockIdx.x] = rs;
  }
}

// Residual replacement (precision form): r = b - H x evaluated with float64
// vectors and accumulation, then u = M^-1 r and the gamma / |r|^2 partials,
// replacing what the float32 recurrence carried.  Launched on the update
// kernel's grid: its partials take the same [gamma | |r|^2] layout of gridDim.x
// entries each that the next SpMV kernel sums.
template <class VT, int G, bool MF32 = sizeof(VT) == 4>
__global__ __launch_bounds__(RED_BLOCK) void pcg_replace_kernel(PcgMatrix A, const double* __restrict__ b,
                                                                const double* __restrict__ x, Vecs<VT> V,
                                                                PcgState* st) {
  if (st->done) return;
  __shared__ double lds[RED_BLOCK];
  const int lane = threadIdx.x % G;
  double g = 0.0, rr = 0.0;
  const RowRange R = xcd_rows<G>(A);
  for (int base = R.first; base < R.end; base += R.stride) {
    const int row = base + threadIdx.x / G;
    const bool live = row < R.end;
    double acc[3];
    spmv_row<MF32, G>(A, live ? row : A.n, lane, x, acc);
    if (lane == 0 && live) {
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
  if (threadIdx.x == 0) {
    V.part_c[blockIdx.x] = gs;
    V.part_c[gridDim.x + blockIdx.x] = rs;
  }
}

// Iteration i: w = H u with the u.w partials, then (workgroup 0) the
// convergence test on |r_i| from the update kernel's partials.  Only workgroup
// 0 needs gamma_i and |r_i|^2, so no other workgroup reduces them; their
// partials are loaded before the product and summed after it, so the loads
// overlap the matrix stream.  When the test finds convergence (or max_iter),
// this launch's w is not used: `done` stops the update kernel and every later
// launch.  `nb_c` is the update kernel's grid (number of gamma / |r|^2
// partials).  standalone: plain y = H x (no solver bookkeeping).
template <class VT, int G, bool MF32 = sizeof(VT) == 4>
__global__ __launch_bounds__(RED_BLOCK) void pcg_spmv_kernel(PcgMatrix A, Vecs<VT> V, PcgState* st, int nb_c,
                                                             int standalone) {
  __shared__ double lds[RED_BLOCK];
  if (!standalone && st->done) return;
  const bool book = !standalone && blockIdx.x == 0;  // uniform per workgroup
  constexpr int PC = (MAX_WG_C + RED_BLOCK - 1) / RED_BLOCK;
  double gp[PC], rp[PC];
#pragma unroll
  for (int q = 0; q < PC; ++q) {
    const int j = threadIdx.x + q * RED_BLOCK;
    const bool in = book && j < nb_c;
    gp[q] = in ? V.part_c[j] : 0.0;
    rp[q] = in ? V.part_c[nb_c + j] : 0.0;
  }
  const int lane = threadIdx.x % G;
  double d = 0.0;
  const RowRange R = xcd_rows<G>(A);
  for (int base = R.first; base < R.end; base += R.stride) {
    const int row = base + threadIdx.x / G;
    const bool live = row < R.end;
    double acc[3];
    spmv_row<MF32, G>(A, live ? row : A.n, lane, V.u, acc);
    if (lane == 0 && live) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const VT wc = VT(acc[c]);
        V.w[3 * (size_t)row + c] = wc;
        d = fma(double(V.u[3 * (size_t)row + c]), double(wc), d);
      }
    }
  }
  const double ds = block_sum<RED_BLOCK>(d, lds);
  if (threadIdx.x == 0) V.part_b[blockIdx.x] = ds;
  if (!book) return;
  // the same association as a strided per-thread sum followed by block_sum
  double ga = 0.0, ra = 0.0;
#pragma unroll
  for (int q = 0; q < PC; ++q) {
    ga += gp[q];
    ra += rp[q];
  }
  const double gamma = block_sum<RED_BLOCK>(ga, lds);
  const double Rr = block_sum<RED_BLOCK>(ra, lds);
  if (threadIdx.x == 0) {
    const int i = st->iter;
    const double bb = i == 0 ? Rr : st->bb;
    const bool conv = Rr <= st->tol2 * bb;
    st->gamma[i & 1] = gamma;
    st->rr = Rr;
    st->iter_b = i;
    if (i == 0) st->bb = bb;
    if (conv || i >= st->max_iter) {
      st->status = conv ? 0 : -5;
      st->done = 1;
    }
  }
}

// One pass of the update kernel: the values a thread reads, loaded before the
// scalars that combine them are known.
template <class VT>
struct UpdLoads {
  double p, s, u, w, x, r, m0, m1, m2;
};

template <class VT>
YDEV UpdLoads<VT> upd_load(const PcgMatrix& A, const double* x, const Vecs<VT>& V, int base, int t, int vl, int c) {
  UpdLoads<VT> L{};
  const int v = base + vl;
  if (v < A.n) {
    const size_t k = 3 * (size_t)base + t;  // = 3 v + c
    L.p = double(V.p[k]);
    L.s = double(V.s[k]);
    L.u = double(V.u[k]);
    L.w = double(V.w[k]);
    L.x = x[k];
    L.r = double(V.r[k]);
    const double* M = A.minv + 9 * (size_t)v + 3 * c;  // row c of the vertex's M^-1
    L.m0 = M[0];
    L.m1 = M[1];
    L.m2 = M[2];
  }
  return L;
}

// Iteration i: scalar recurrences, vector updates, preconditioning, and the
// gamma / |r|^2 partials of iteration i + 1.  `nb_b` = SpMV grid.  One thread
// per vertex component (coalesced vector traffic, 3x the threads of a
// per-vertex mapping); the three residual components of a vertex meet in LDS
// for the 3x3 block-Jacobi product.  Each pass's vectors are loaded before
// alpha and beta are known (the first pass before the reduction of the SpMV
// partials, the next one while the current one computes).
template <class VT>
__global__ __launch_bounds__(UPD_BLOCK) void pcg_update_kernel(PcgMatrix A, double* __restrict__ x, Vecs<VT> V,
                                                               PcgState* st, int nb_b) {
  if (st->done) return;
  __shared__ double lds[UPD_BLOCK];
  __shared__ double rsh[UPD_BLOCK];
  const int t = threadIdx.x;
  const int vl = t / 3, c = t - 3 * (t / 3);
  const int stride = gridDim.x * UPD_VERTS;
  int base = blockIdx.x * UPD_VERTS;
  // the SpMV partials first (their sum is needed first), then the first pass
  constexpr int PB = (MAX_WG_B + UPD_BLOCK - 1) / UPD_BLOCK;
  double bp[PB];
#pragma unroll
  for (int q = 0; q < PB; ++q) {
    const int j = t + q * UPD_BLOCK;
    bp[q] = j < nb_b ? V.part_b[j] : 0.0;
  }
  UpdLoads<VT> cur = upd_load(A, x, V, base, t, vl, c);
  const int i = st->iter_b;
  const double gamma = st->gamma[i & 1];
  double dacc = 0.0;  // the association of a strided per-thread sum
#pragma unroll
  for (int q = 0; q < PB; ++q) dacc += bp[q];
  const double delta = block_sum<UPD_BLOCK>(dacc, lds);
  const bool restart = i == st->restart_at;
  const double beta = restart ? 0.0 : gamma / st->gamma[(i - 1) & 1];
  const double pAp = restart ? delta : delta - beta * gamma / st->alpha[(i - 1) & 1];
  const bool first = blockIdx.x == 0 && threadIdx.x == 0;
  if (!(pAp > 0.0)) {
    if (first) {
      st->status = -6;
      st->done = 1;
    }
    return;
  }
  const double alpha = gamma / pAp;
  double g = 0.0, rr = 0.0;
  for (; base < A.n; base += stride) {
    const UpdLoads<VT> nxt = upd_load(A, x, V, base + stride, t, vl, c);
    const int v = base + vl;
    const bool live = v < A.n;
    const size_t k = 3 * (size_t)base + t;  // = 3 v + c
    double r = 0.0;
    if (live) {
      const VT p = VT(fma(beta, cur.p, cur.u));
      const VT sv = VT(fma(beta, cur.s, cur.w));
      V.p[k] = p;
      V.s[k] = sv;
      x[k] = fma(alpha, double(p), cur.x);
      const VT rc = VT(fma(-alpha, double(sv), cur.r));
      V.r[k] = rc;
      r = double(rc);
    }
    rsh[t] = r;
    __syncthreads();
    if (live) {
      const VT uc = VT(cur.m0 * rsh[3 * vl] + cur.m1 * rsh[3 * vl + 1] + cur.m2 * rsh[3 * vl + 2]);
      V.u[k] = uc;
      g = fma(r, double(uc), g);
      rr = fma(r, r, rr);
    }
    __syncthreads();  // rsh is rewritten by the next pass
    cur = nxt;
  }
  const double gs = block_sum<UPD_BLOCK>(g, lds);
  const double rs = block_sum<UPD_BLOCK>(rr, lds);
  if (threadIdx.x == 0) {
    V.part_c[blockIdx.x] = gs;
    V.part_c[gridDim.x + blockIdx.x] = rs;
  }
  if (first) {
    st->alpha[i & 1] = alpha;
    st->iter = i + 1;
  }
}

// Grids are multiples of NXCD (the SpMV-shaped kernels split rows per XCD; the
// replacement kernel runs on the update kernel's grid).
int round_xcd(int g) { return (g + NXCD - 1) / NXCD * NXCD; }
bool narrow_rows(const PcgMatrix& A) { return A.nnz <= (long long)SPMV_NARROW_MEAN * A.n; }
int grid_b(int n, int g) {
  const int rows = RED_BLOCK / g;
  return round_xcd(std::max(1, std::min((n + rows - 1) / rows, MAX_WG_B)));
}
int grid_c(int n) { return round_xcd(std::max(1, std::min((n + UPD_VERTS - 1) / UPD_VERTS, MAX_WG_C))); }

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

// Fixed solver workspace for callers that cannot allocate (yasps_pcg_noalloc):
// one array per GPU, held from the module's load until the process ends.  Its
// name is a host-side stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

void launch_spmv(const PcgMatrix& A, const double* x, double* y, void* work, hipStream_t s) {
  if (A.n == 0) return;
  PcgState* st;
  Vecs<double> V;
  carve(work, A.n, st, V);
  V.u = const_cast<double*>(x);
  V.w = y;
  // the precision form's float32 copy with float64 vectors, or the stored blocks
  const dim3 b(RED_BLOCK);
  if (narrow_rows(A)) {
    if (A.v32)
      hipLaunchKernelGGL((pcg_spmv_kernel<double, 8, true>), dim3(grid_b(A.n, 8)), b, 0, s, A, V, st, 1, 1);
    else
      hipLaunchKernelGGL((pcg_spmv_kernel<double, 8, false>), dim3(grid_b(A.n, 8)), b, 0, s, A, V, st, 1, 1);
  } else {
    if (A.v32)
      hipLaunchKernelGGL((pcg_spmv_kernel<double, 16, true>), dim3(grid_b(A.n, 16)), b, 0, s, A, V, st, 1, 1);
    else
      hipLaunchKernelGGL((pcg_spmv_kernel<double, 16, false>), dim3(grid_b(A.n, 16)), b, 0, s, A, V, st, 1, 1);
  }
}

namespace {

// Launch, timed by events that the launch itself carries when a profiler asks.
template <class KERNEL, class... ARGS>
void timed_launch(LaunchTimer* tm, int cls, KERNEL kernel, int grid, int block, hipStream_t s, ARGS... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (tm && tm->kernel_events(cls, &a, &b))
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, a, b, 0, args...);
  else
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, args...);
}

template <class VT, int G>
int pcg_run(const PcgMatrix& A, const double* b, double* x, double rtol, int max_iter, void* work, double* rel_out,
            int* status_out, hipStream_t s, LaunchTimer* tm, PcgState& hs, int* hint) {
  static_assert(sizeof(PcgState) <= 128, "the pinned polling buffer holds 128 bytes");
  constexpr bool MIXED = sizeof(VT) == 4;
  constexpr int REPLACE_EVERY = 50;  // float64 residual replacement period (precision form)
  const int n = A.n;
  PcgState* st;
  Vecs<VT> V;
  carve(work, n, st, V);
  const int nb_b = grid_b(n, G), nb_c = grid_c(n);
  PcgState h{};
  h.tol2 = rtol * rtol;
  h.max_iter = max_iter;
  if (hipMemcpyAsync(st, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess) return -2;
  if (n == 0) {
    *rel_out = 0.0;
    *status_out = 0;
    return 0;
  }
  timed_launch(tm, 6, pcg_init_kernel<VT>, nb_c, RED_BLOCK, s, A, b, x, V, st);
  // Launches between polls.  The launch that finds convergence after k
  // iterations is the (k + 1)-th: with a hint k the first batch is k + 2
  // launches (one poll when the count repeats or drops a little; launches past
  // convergence exit at once, a few microseconds each, against tens for a
  // poll), then batches of 8; without a hint 8, 16, 32, 64, 64, ...
  const bool hinted = hint && *hint > 16;
  int batch = hinted ? *hint + 2 : 8;
  long long launched = 0;  // (SpMV, update) pairs issued = iteration index while not done
  int verified_at = -1;
  int restarts = 0;
  constexpr int MAX_RESTARTS = 32;
  for (;;) {
    for (int k = 0; k < batch; ++k) {
      timed_launch(tm, 5, pcg_spmv_kernel<VT, G>, nb_b, RED_BLOCK, s, A, V, st, nb_c, 0);
      timed_launch(tm, 6, pcg_update_kernel<VT>, nb_c, UPD_BLOCK, s, A, x, V, st, nb_b);
      ++launched;
      if (MIXED && launched % REPLACE_EVERY == 0)
        timed_launch(tm, 5, pcg_replace_kernel<VT, G>, nb_c, RED_BLOCK, s, A, b, x, V, st);
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
      fix.restart_at = hs.iter_b;
      fix.iter = hs.iter_b;
      if (hipMemcpyAsync(st, &fix, sizeof(fix), hipMemcpyHostToDevice, s) != hipSuccess) return -2;
      hipLaunchKernelGGL((pcg_replace_kernel<VT, G>), dim3(nb_c), dim3(RED_BLOCK), 0, s, A, b, x, V, st);
      launched = hs.iter_b;
      batch = 8;
      continue;
    }
    if (hs.done) {
      if (!MIXED || hs.status != 0 || verified_at == hs.iter_b) break;
      // converged on the recurrence residual: confirm with a float64 true residual
      verified_at = hs.iter_b;
      const int zero = 0;
      if (hipMemcpyAsync(&st->done, &zero, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess) return -2;
      hipLaunchKernelGGL((pcg_replace_kernel<VT, G>), dim3(nb_c), dim3(RED_BLOCK), 0, s, A, b, x, V, st);
      launched = hs.iter_b;
      batch = 8;
      continue;
    }
    batch = hinted ? 8 : std::min(batch * 2, 64);
  }
  *rel_out = hs.bb > 0.0 ? sqrt(hs.rr / hs.bb) : 0.0;
  *status_out = hs.status;
  if (hint) *hint = hs.iter_b;
  return hs.iter_b;
}

}  // namespace

int pcg_solve(const PcgMatrix& A, const double* b, double* x, double rtol, int max_iter, bool mixed, void* work,
              double* rel_out, int* status_out, hipStream_t s, LaunchTimer* tm, void* host_state, int* hint) {
  PcgState& hs = *static_cast<PcgState*>(host_state);
  if (narrow_rows(A))
    return mixed ? pcg_run<float, 8>(A, b, x, rtol, max_iter, work, rel_out, status_out, s, tm, hs, hint)
                 : pcg_run<double, 8>(A, b, x, rtol, max_iter, work, rel_out, status_out, s, tm, hs, hint);
  return mixed ? pcg_run<float, 16>(A, b, x, rtol, max_iter, work, rel_out, status_out, s, tm, hs, hint)
               : pcg_run<double, 16>(A, b, x, rtol, max_iter, work, rel_out, status_out, s, tm, hs, hint);
}

}  // namespace yasps
