// Block-Jacobi preconditioned conjugate gradient on the symmetric 3x3 BSR
// Hessian (section "Solver", appendices "SpMV" and "Preconditioner").
//
// SpMV.  The Hessian is assembled once, as its upper triangle (appendix
// "Global Hessian Compression"), in two parts (static and dynamic).  The
// paper's SpMV adds, for every off-diagonal block, the transposed product with
// atomics (Algorithm "CUDA Block Level SpMV").  Here every stored block is
// read once: the blocks of each part are cut into chunks of consecutive blocks
// (spmvplan.hip); the workgroup of a chunk forms B x_j for the block's row i
// and, off the diagonal, B^T x_i for row j, and sums the products of each
// target row in LDS in a fixed order (the LDS entries come from the plan);
// the sum of every (chunk, target row) is written to its slot of W.  A row's
// slots are contiguous and few (its own chunk, plus the chunks of earlier rows
// that reach it), and the next kernel adds them in order.  No atomics; the
// results are bitwise reproducible.  The values are read from the assembled
// blocks themselves, float64 or (precision form) float32.
//
// Iteration.  PCG with one global reduction phase per iteration (the
// Chronopoulos-Gear arrangement, equal to standard PCG in exact arithmetic):
//   u = M^-1 r, w = H u, gamma = r.u, delta = u.w
//   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev)
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s
// Two kernels per iteration: (B) the chunked product into W with the delta
// partials (delta = u^T H u summed block by block: u_i . B u_j, twice off the
// diagonal) and, in workgroup 0, the convergence test; (C) w from the W slots,
// the scalar recurrences, vector updates, preconditioning and the next gamma
// and |r|^2 partials.  Each kernel re-sums the previous kernel's partials in a
// fixed order (workgroup 0 of B only, every workgroup of C); convergence is
// tested on the device and the host polls a flag between batches of launches.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>

#include "blockreduce.h"
#include "kernels.h"

namespace yasps {

// Launch shapes (compile-time; the defaults come from sweeps on the 40^3 and
// 80x80x52 workloads).
#ifndef YASPS_MAX_WG_B
#define YASPS_MAX_WG_B 2048
#endif
#ifndef YASPS_MAX_WG_C
#define YASPS_MAX_WG_C 512
#endif
#ifndef YASPS_UPD_VERTS
#define YASPS_UPD_VERTS 128
#endif
constexpr int MAX_WG_B = YASPS_MAX_WG_B;        // workgroups of the SpMV kernel (chunks are shared out)
constexpr int MAX_WG_C = YASPS_MAX_WG_C;        // workgroups of the update kernel
constexpr int UPD_VERTS = YASPS_UPD_VERTS;      // vertices per update-kernel workgroup pass
constexpr int UPD_BLOCK = 3 * UPD_VERTS;        // update kernel: one thread per vertex component
// kernel classes of the profiler (yasps.h): the SpMV and the PCG update
constexpr int SPMV_CLASS = 5, UPDATE_CLASS = 6;

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

// The chunks (static part first, then dynamic) are split into NXCD contiguous
// ranges, one per XCD: workgroups are dispatched to the XCDs round robin by
// index, so workgroup b runs on XCD b % NXCD and takes chunks of that XCD's
// range; the vector gathers of one XCD stay near its own rows (mesh locality)
// and in its own L2.  The SpMV grid is a multiple of NXCD.
constexpr int NXCD = PCG_XCDS;
static_assert(MAX_WG_B % NXCD == 0 && MAX_WG_C % NXCD == 0, "partial-sum arrays hold the rounded grids");

enum SpmvMode { SPMV_PCG = 0, SPMV_PLAIN = 1, SPMV_REPLACE = 2 };

// Krylov vectors in VT (float64, or float32 in the precision form); the
// solution x is always float64.  W[p]: the SpMV slots of part p (float64, 3
// per slot).
template <class VT>
struct Vecs {
  VT *r, *u, *p, *s;
  double *part_b, *part_c;  // part_c holds 2 * MAX_WG_C partials
  double* W[PCG_PARTS];     // SpMV slots of each part
};

// Adds the slots [e, f) of one part to w in slot order; four loads are issued
// before they are added (a missing slot adds +0, which leaves w unchanged).
YDEV double add_slots(double w, const double* __restrict__ W, int e, int f, int c) {
  for (; e < f; e += 4) {
    const double a0 = W[3 * (size_t)e + c];
    const double a1 = e + 1 < f ? W[3 * (size_t)(e + 1) + c] : 0.0;
    const double a2 = e + 2 < f ? W[3 * (size_t)(e + 2) + c] : 0.0;
    const double a3 = e + 3 < f ? W[3 * (size_t)(e + 3) + c] : 0.0;
    w += a0;
    w += a1;
    w += a2;
    w += a3;
  }
  return w;
}

// w_v[c] = sum of the SpMV slots of row v, part by part, in slot order
struct Slots {
  double* W[PCG_PARTS];
};
YDEV double w_sum(const PcgMatrix& A, const Slots& S, int v, int c) {
  double w = 0.0;
#pragma unroll
  for (int p = 0; p < PCG_PARTS; ++p)
    if (const int32_t* h = A.part[p].hptr) w = add_slots(w, S.W[p], h[v], h[v + 1], c);
  return w;
}

template <class VT>
YHD Slots slots_of(const Vecs<VT>& V) {
  Slots S;
#pragma unroll
  for (int p = 0; p < PCG_PARTS; ++p) S.W[p] = V.W[p];
  return S;
}

// Chunked product W = slots of H u (see the file comment).  BT: stored block
// type, XT: vector type.  The threads of a workgroup take the blocks of its
// chunk in turn (coalesced value and index loads, independent of each other),
// write both products of every block to their LDS entries, and after a
// barrier sum each target row's entries into its W slot.  Modes: SPMV_PCG
// (delta partials into part_b; workgroup 0 also runs the convergence test on
// the update kernel's gamma / |r|^2 partials, loaded before the product and
// summed after it), SPMV_PLAIN (product only), SPMV_REPLACE (product only,
// skipped once the solver is done).
// One stored block of the chunked product: its target rows, entries, values
// and the two gathered vector rows.
template <class BT, class XT>
struct BlockIn {
  int j, r, ey, et;
  BT B[9];
  XT x[3], u[3];
};

template <class BT, class XT>
YDEV BlockIn<BT, XT> block_load(const SpmvPart& P, const BT* __restrict__ vals, const XT* __restrict__ u,
                                const int32_t* __restrict__ rl, int m0, int k) {
  BlockIn<BT, XT> L;
  const uint32_t meta = P.meta[k];
  L.j = P.col[k];
  const int m = m0 + (int)(meta & 1023u);
  L.r = rl ? rl[m] : m;
  L.ey = (int)((meta >> 10) & 2047u);
  L.et = (int)(meta >> 21);
  const BT* bp = vals + 9 * (size_t)k;
#pragma unroll
  for (int q = 0; q < 9; ++q) L.B[q] = bp[q];
  const XT* xj = u + 3 * (size_t)L.j;
  const XT* xr = u + 3 * (size_t)L.r;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    L.x[q] = xj[q];
    L.u[q] = xr[q];
  }
  return L;
}

// B x_j to the row's entry; off the diagonal B^T u_r to the column's entry;
// the block's share of delta = u^T H u.
template <class BT, class XT>
YDEV void block_products(const BlockIn<BT, XT>& L, double* E, double& dlt) {
  double B[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) B[q] = double(L.B[q]);
  const double x0 = double(L.x[0]), x1 = double(L.x[1]), x2 = double(L.x[2]);
  const double u0 = double(L.u[0]), u1 = double(L.u[1]), u2 = double(L.u[2]);
  const double y0 = fma(B[0], x0, fma(B[1], x1, B[2] * x2));
  const double y1 = fma(B[3], x0, fma(B[4], x1, B[5] * x2));
  const double y2 = fma(B[6], x0, fma(B[7], x1, B[8] * x2));
  E[3 * L.ey] = y0;
  E[3 * L.ey + 1] = y1;
  E[3 * L.ey + 2] = y2;
  const double uy = fma(u0, y0, fma(u1, y1, u2 * y2));
  if (L.j != L.r) {
    E[3 * L.et] = fma(B[0], u0, fma(B[3], u1, B[6] * u2));
    E[3 * L.et + 1] = fma(B[1], u0, fma(B[4], u1, B[7] * u2));
    E[3 * L.et + 2] = fma(B[2], u0, fma(B[5], u1, B[8] * u2));
    dlt = fma(2.0, uy, dlt);
  } else {
    dlt += uy;
  }
}

template <class BT, class XT>
__global__ __launch_bounds__(RED_BLOCK) void spmv_chunk_kernel(PcgMatrix A, const XT* __restrict__ u, Slots S,
                                                               double* __restrict__ part_b,
                                                               const double* __restrict__ part_c, PcgState* st,
                                                               int nb_c, int mode) {
  extern __shared__ double E[];  // [entries][3] products of one chunk, grouped by target row
  __shared__ double lds[RED_BLOCK];
  // The solver's done flag is loaded with the first chunk's data and tested
  // before the first barrier (a finished solve leaves before any store).
  const int dn = mode != SPMV_PLAIN ? st->done : 0;
  const bool book = mode == SPMV_PCG && blockIdx.x == 0;  // uniform per workgroup
  constexpr int PC = (MAX_WG_C + RED_BLOCK - 1) / RED_BLOCK;
  double gp[PC], rp[PC];
#pragma unroll
  for (int q = 0; q < PC; ++q) {
    const int j = threadIdx.x + q * RED_BLOCK;
    const bool in = book && j < nb_c;
    gp[q] = in ? part_c[j] : 0.0;
    rp[q] = in ? part_c[nb_c + j] : 0.0;
  }
  const int C0 = A.part[0].nchunk, C1 = C0 + A.part[1].nchunk, C = C1 + A.part[2].nchunk;
  const int xcd = blockIdx.x % NXCD, per = gridDim.x / NXCD;
  const int cend = (int)((long long)C * (xcd + 1) / NXCD);
  double dlt = 0.0;
  for (int c = (int)((long long)C * xcd / NXCD) + (int)blockIdx.x / NXCD; c < cend; c += per) {
    const int pi = c < C0 ? 0 : (c < C1 ? 1 : 2);
    const SpmvPart& P = A.part[pi];
    const int cc = c - (pi == 0 ? 0 : (pi == 1 ? C0 : C1));
    const int b0 = cc * P.chunk, b1 = min(b0 + P.chunk, P.nblk);
    const int m0 = P.m0[cc];
    const int32_t* __restrict__ rl = P.rl;  // null when every row holds blocks (row = compressed row)
    const BT* __restrict__ vals = static_cast<const BT*>(P.vals);
    // the first target row of this thread: its entry range and slot are
    // loaded with the blocks, ahead of the barrier
    const int t0 = P.tb[cc], nt = P.tb[cc + 1] - t0;
    const int q0 = threadIdx.x;
    const int pe1 = q0 < nt ? P.tend[t0 + q0] : 0;
    const int pe0 = q0 < nt && q0 ? P.tend[t0 + q0 - 1] : 0;
    const int pws = q0 < nt ? P.wslot[t0 + q0] : 0;
    // two blocks per thread and trip, all loads of both issued before either
    // product (a chunk of RED_BLOCK blocks or fewer takes one)
    for (int k = b0 + (int)threadIdx.x; k < b1; k += 2 * RED_BLOCK) {
      const int k2 = k + RED_BLOCK;
      const bool two = b1 - b0 > RED_BLOCK && k2 < b1;
      BlockIn<BT, XT> L0 = block_load<BT, XT>(P, vals, u, rl, m0, k);
      BlockIn<BT, XT> L1;
      if (two) L1 = block_load<BT, XT>(P, vals, u, rl, m0, k2);
      block_products(L0, E, dlt);
      if (two) block_products(L1, E, dlt);
    }
    if (dn) return;  // uniform: every thread of the workgroup leaves here
    __syncthreads();
    double* __restrict__ W = S.W[pi];
    for (int q = threadIdx.x; q < nt; q += RED_BLOCK) {
      const bool f = q == q0;
      const int e1 = f ? pe1 : P.tend[t0 + q], e0 = f ? pe0 : (q ? P.tend[t0 + q - 1] : 0);
      const int ws = f ? pws : P.wslot[t0 + q];
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int e = e0; e < e1; ++e) {
        s0 += E[3 * e];
        s1 += E[3 * e + 1];
        s2 += E[3 * e + 2];
      }
      double* w = W + 3 * (size_t)ws;
      w[0] = s0;
      w[1] = s1;
      w[2] = s2;
    }
    __syncthreads();  // E is refilled by the next chunk
  }
  if (mode != SPMV_PCG || dn) return;
  const double ds = block_sum<RED_BLOCK>(dlt, lds);
  if (threadIdx.x == 0) part_b[blockIdx.x] = ds;
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

// Residual replacement (precision form), after a SPMV_REPLACE product of the
// float64 x: r = b - H x in float64, then u = M^-1 r and the gamma / |r|^2
// partials, replacing what the float32 recurrence carried.  Launched on the
// update kernel's grid: its partials take the same [gamma | |r|^2] layout of
// gridDim.x entries each that the next SpMV kernel sums.
template <class VT>
__global__ __launch_bounds__(RED_BLOCK) void pcg_replace_kernel(PcgMatrix A, const double* __restrict__ b,
                                                                Vecs<VT> V, PcgState* st) {
  if (st->done) return;
  __shared__ double lds[RED_BLOCK];
  double g = 0.0, rr = 0.0;
  for (int v = blockIdx.x * RED_BLOCK + threadIdx.x; v < A.n; v += gridDim.x * RED_BLOCK) {
    double r[3], u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = b[3 * (size_t)v + c] - w_sum(A, slots_of(V), v, c);
    precondition(A.minv, v, r, u);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const VT rc = VT(r[c]), uc = VT(u[c]);
      V.r[3 * (size_t)v + c] = rc;
      V.u[3 * (size_t)v + c] = uc;
      g = fma(double(rc), double(uc), g);
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

// y = H x from the slots of a SPMV_PLAIN product
__global__ __launch_bounds__(RED_BLOCK) void spmv_finish_kernel(PcgMatrix A, Slots S, double* __restrict__ y) {
  const long long i = (long long)blockIdx.x * RED_BLOCK + threadIdx.x;
  if (i >= 3ll * A.n) return;
  const int v = (int)(i / 3), c = (int)(i - 3ll * v);
  y[i] = w_sum(A, S, v, c);
}

// One pass of the update kernel: the values a thread reads, loaded before the
// scalars that combine them are known (w summed from the SpMV slots).
struct UpdLoads {
  double p, s, u, w, x, r, m0, m1, m2;
};

template <class VT>
YDEV UpdLoads upd_load(const PcgMatrix& A, const double* x, const Vecs<VT>& V, int base, int t, int vl, int c) {
  UpdLoads L{};
  const int v = base + vl;
  if (v < A.n) {
    const size_t k = 3 * (size_t)base + t;  // = 3 v + c
    L.p = double(V.p[k]);
    L.s = double(V.s[k]);
    L.u = double(V.u[k]);
    L.x = x[k];
    L.r = double(V.r[k]);
    const double* M = A.minv + 9 * (size_t)v + 3 * c;  // row c of the vertex's M^-1
    L.m0 = M[0];
    L.m1 = M[1];
    L.m2 = M[2];
    L.w = double(VT(w_sum(A, slots_of(V), v, c)));
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
  // every scalar of the state in one batch of loads, tested after the first
  // pass's vector loads are issued
  const int dn = st->done, i = st->iter_b, ra = st->restart_at;
  const double g0 = st->gamma[0], g1 = st->gamma[1], a0 = st->alpha[0], a1 = st->alpha[1];
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
  UpdLoads cur = upd_load(A, x, V, base, t, vl, c);
  if (dn) return;
  const double gamma = (i & 1) ? g1 : g0;
  double dacc = 0.0;  // the association of a strided per-thread sum
#pragma unroll
  for (int q = 0; q < PB; ++q) dacc += bp[q];
  const double delta = block_sum<UPD_BLOCK>(dacc, lds);
  const bool restart = i == ra;
  const double beta = restart ? 0.0 : gamma / ((i & 1) ? g0 : g1);
  const double pAp = restart ? delta : delta - beta * gamma / ((i & 1) ? a0 : a1);
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
    const UpdLoads nxt = upd_load(A, x, V, base + stride, t, vl, c);
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

int round_xcd(int g) { return (g + NXCD - 1) / NXCD * NXCD; }
// SpMV workgroups at most (YASPS_SPMV_WG: a tuning override, NXCD .. MAX_WG_B)
int wg_cap_b() {
  static const int cap = [] {
    const char* e = std::getenv("YASPS_SPMV_WG");
    const int v = e ? std::atoi(e) : 0;
    return (v >= NXCD && v <= MAX_WG_B) ? v / NXCD * NXCD : MAX_WG_B;
  }();
  return cap;
}
int grid_b(const PcgMatrix& A) {
  return round_xcd(std::max(1, std::min(A.part[0].nchunk + A.part[1].nchunk + A.part[2].nchunk, wg_cap_b())));
}
int grid_c(int n) { return round_xcd(std::max(1, std::min((n + UPD_VERTS - 1) / UPD_VERTS, MAX_WG_C))); }
// LDS of the chunk kernel: the larger chunk's products
size_t spmv_lds_bytes(const PcgMatrix& A) {
  int m = 1;
  for (const SpmvPart& P : A.part) m = std::max(m, P.max_entries);
  return 3 * sizeof(double) * (size_t)m;
}

template <class VT>
void carve(void* work, const PcgMatrix& A, PcgState*& st, Vecs<VT>& V) {
  const size_t n3 = 3 * (size_t)A.n;
  char* w = static_cast<char*>(work);
  st = reinterpret_cast<PcgState*>(w);
  double* parts = reinterpret_cast<double*>(w + ((sizeof(PcgState) + 255) / 256) * 256);
  V.part_b = parts;
  V.part_c = parts + MAX_WG_B;
  double* q = parts + MAX_WG_B + 2 * MAX_WG_C;
  for (int p = 0; p < PCG_PARTS; ++p) {
    V.W[p] = q;
    q += 3 * (size_t)A.part[p].ntarget;
  }
  VT* base = reinterpret_cast<VT*>(q);
  V.r = base;
  V.u = V.r + n3;
  V.p = V.u + n3;
  V.s = V.p + n3;
}

// Launch, timed by events that the launch itself carries when a profiler asks.
template <class KERNEL, class... ARGS>
void timed_launch(LaunchTimer* tm, int cls, KERNEL kernel, int grid, int block, size_t shmem, hipStream_t s,
                  ARGS... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (tm && tm->kernel_events(cls, &a, &b))
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, s, a, b, 0, args...);
  else
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, s, args...);
}

// The chunked product.
template <class BT, class XT, class VT>
void launch_chunks(LaunchTimer* tm, const PcgMatrix& A, const XT* u, const Vecs<VT>& V, double* part_b,
                   const double* part_c, PcgState* st, int nb_c, int mode, hipStream_t s) {
  timed_launch(tm, SPMV_CLASS, spmv_chunk_kernel<BT, XT>, grid_b(A), RED_BLOCK, spmv_lds_bytes(A), s, A, u,
               slots_of(V), part_b, part_c, st, nb_c, mode);
}

}  // namespace

size_t pcg_workspace_bytes(int n, long long nslots) {
  const size_t n3 = 3 * (size_t)std::max(n, 1);
  return 256 + ((sizeof(PcgState) + 255) / 256) * 256 +
         sizeof(double) * (4 * n3 + MAX_WG_B + 2 * MAX_WG_C + 3 * (size_t)std::max(nslots, 0ll));
}  // float64 vectors; the float32 form uses half of the vector part

size_t spmv_max_lds_bytes() { return 3 * sizeof(double) * 2 * SPMV_MAX_CHUNK; }

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

void launch_spmv(const PcgMatrix& A, const double* x, double* y, void* work, hipStream_t s, LaunchTimer* tm) {
  if (A.n == 0) return;
  PcgState* st;
  Vecs<double> V;
  carve(work, A, st, V);
  if (A.f32)
    launch_chunks<float, double>(tm, A, x, V, nullptr, nullptr, nullptr, 0, SPMV_PLAIN, s);
  else
    launch_chunks<double, double>(tm, A, x, V, nullptr, nullptr, nullptr, 0, SPMV_PLAIN, s);
  const long long n3 = 3ll * A.n;
  timed_launch(tm, SPMV_CLASS, spmv_finish_kernel, (int)((n3 + RED_BLOCK - 1) / RED_BLOCK), RED_BLOCK, 0, s, A,
               slots_of(V), y);
}

namespace {

template <class VT>
int pcg_run(const PcgMatrix& A, const double* b, double* x, double rtol, int max_iter, void* work, double* rel_out,
            int* status_out, hipStream_t s, LaunchTimer* tm, PcgState& hs, int* hint) {
  static_assert(sizeof(PcgState) <= 128, "the pinned polling buffer holds 128 bytes");
  constexpr bool MIXED = sizeof(VT) == 4;
  using BT = VT;  // stored blocks: float32 in the precision form
  constexpr int REPLACE_EVERY = 50;  // float64 residual replacement period (precision form)
  const int n = A.n;
  PcgState* st;
  Vecs<VT> V;
  carve(work, A, st, V);
  const int nb_b = grid_b(A), nb_c = grid_c(n);
  PcgState h{};
  h.tol2 = rtol * rtol;
  h.max_iter = max_iter;
  if (hipMemcpyAsync(st, &h, sizeof(h), hipMemcpyHostToDevice, s) != hipSuccess) return -2;
  if (n == 0) {
    *rel_out = 0.0;
    *status_out = 0;
    return 0;
  }
  auto replace = [&]() {  // r = b - H x in float64 (precision form)
    launch_chunks<BT, double>(nullptr, A, x, V, nullptr, nullptr, st, 0, SPMV_REPLACE, s);
    hipLaunchKernelGGL((pcg_replace_kernel<VT>), dim3(nb_c), dim3(RED_BLOCK), 0, s, A, b, V, st);
  };
  timed_launch(tm, UPDATE_CLASS, pcg_init_kernel<VT>, nb_c, RED_BLOCK, 0, s, A, b, x, V, st);
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
      launch_chunks<BT, VT>(tm, A, V.u, V, V.part_b, V.part_c, st, nb_c, SPMV_PCG, s);
      timed_launch(tm, UPDATE_CLASS, pcg_update_kernel<VT>, nb_c, UPD_BLOCK, 0, s, A, x, V, st, nb_b);
      ++launched;
      if (MIXED && launched % REPLACE_EVERY == 0) replace();
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
      replace();
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
      replace();
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
  if (mixed != A.f32) return -2;
  return mixed ? pcg_run<float>(A, b, x, rtol, max_iter, work, rel_out, status_out, s, tm, hs, hint)
               : pcg_run<double>(A, b, x, rtol, max_iter, work, rel_out, status_out, s, tm, hs, hint);
}

}  // namespace yasps
