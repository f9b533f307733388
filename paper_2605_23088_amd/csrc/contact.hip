// Log-barrier contact kernels: one thread per stencil, stencils grouped by
// (type, number of free vertices) so every group runs one specialised kernel.
// The per-stencil arithmetic is in contact_math.h.
#include "blockreduce.h"
#include "contact_math.h"
#include "kernels.h"

namespace yasps {

namespace {

using namespace cmath;

YDEV const double* vptr(const ContactArgs& a, int v) {
  return v < a.n_free ? a.x + 3 * (size_t)v : a.x_fixed + 3 * (size_t)(v - a.n_free);
}

template <int TYPE, int K, bool EXACT, bool TRI_FREE>
__global__ __launch_bounds__(EVAL_BLOCK) void contact_kernel(ContactArgs a) {
  constexpr int NV = Topo<TYPE>::NV;
  __shared__ double lds[EVAL_BLOCK];
  const int s = a.begin + blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0, dmin = __builtin_inf(), nact = 0.0;
  if (s < a.end) {
    const int nc = a.nc;
    int v[4] = {0, 0, 0, 0};
    double xv[4][3] = {};
    int fl[4] = {0, 0, 0, 0};  // local index of the j-th free vertex (static indexing only)
    int nf = 0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      v[k] = a.idx[k * nc + s];
      const double* p = vptr(a, v[k]);
      xv[k][0] = p[0];
      xv[k][1] = p[1];
      xv[k][2] = p[2];
      const bool f = v[k] < a.n_free;
#pragma unroll
      for (int j = 0; j < 4; ++j) fl[j] = (f && nf == j) ? k : fl[j];
      nf += f ? 1 : 0;
    }
    double d, side;
    auto gsink = [&](int k, const double (&g)[3]) {
      const int pos = a.gpos[fl[k] * nc + s];
      double* dst = a.grd + 3 * (size_t)pos;
      dst[0] = g[0];
      dst[1] = g[1];
      dst[2] = g[2];
    };
    auto bsink = [&](int I, int J, const double (&B)[3][3]) {
      const int pos = a.spos[pair_index(fl[I], fl[J], NV) * nc + s];
      const bool tr = v[fl[I]] > v[fl[J]];
      if (a.blk32) {
        float* dst = a.blk32 + 9 * (size_t)pos;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int l = 0; l < 3; ++l) dst[3 * i + l] = float(tr ? B[l][i] : B[i][l]);
      } else {
        double* dst = a.blk + 9 * (size_t)pos;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int l = 0; l < 3; ++l) dst[3 * i + l] = tr ? B[l][i] : B[i][l];
      }
    };
    const double eps = (TYPE == 1 && a.eps) ? a.eps[s] : 0.0;
    const bool ok = contact_stencil<TYPE, K, EXACT, TRI_FREE>(xv, fl, a.kappa, a.dhat, a.barrier, e, d, side, gsink, bsink, eps);
    a.d_out[s] = d;
    dmin = d;
    if (!ok || !finite(d) || !finite(e)) atomicOr(a.flags, FLAG_NONFINITE);
    if (finite(d) && !(d > 0.0)) atomicOr(a.flags, FLAG_DOMAIN);
    nact = (d > 0.0 && d < a.dhat) ? 1.0 : 0.0;
  }
  const double es = block_sum<EVAL_BLOCK>(e, lds);
  const double dm = block_min<EVAL_BLOCK>(dmin, lds);
  const double na = block_sum<EVAL_BLOCK>(nact, lds);
  if (threadIdx.x == 0) {
    a.e_part[blockIdx.x] = es;
    a.dmin_part[blockIdx.x] = dm;
    a.nact_part[blockIdx.x] = na;
  }
}

// Line search trial at y = x + alpha p (already formed in a.x); x0 holds the
// positions of the start of the step for the side test.
template <int TYPE>
__global__ __launch_bounds__(EVAL_BLOCK) void contact_energy_kernel(ContactArgs a, const double* x0,
                                                                    double* bad_part) {
  constexpr int NV = Topo<TYPE>::NV, NU = Topo<TYPE>::NU;
  __shared__ double lds[EVAL_BLOCK];
  const int s = a.begin + blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0, bad = 0.0;
  if (s < a.end) {
    const int nc = a.nc;
    double xv[4][3], xo[4][3];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int v = a.idx[k * nc + s];
      const double* p = vptr(a, v);
      const double* q = v < a.n_free ? x0 + 3 * (size_t)v : p;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        xv[k][i] = p[i];
        xo[k][i] = q[i];
      }
    }
    double u[NU][3], uo[NU][3];
    const bool ok = diff_vars<TYPE>(xv, u) && diff_vars<TYPE>(xo, uo);
    Dist<TYPE> D, Do;
    double side, side0;
    distance<TYPE>(u, D, side);
    distance<TYPE>(uo, Do, side0);
    if (!ok || !(D.d > 0.0) || !finite(D.d)) bad = 1.0;
    if ((TYPE == 0 || TYPE == 1) && ((side > 0.0) != (side0 > 0.0) || side == 0.0)) bad = 1.0;
    if (bad == 0.0 && D.d < a.dhat) {
      double b0, b1, b2;
      barrier(D.d, a.dhat, a.barrier, b0, b1, b2);
      double m = 1.0;
      if constexpr (TYPE == 1) m = a.eps ? ee_mollifier(u, a.eps[s]) : 1.0;
      e = m < 1.0 ? a.kappa * m * b0 : a.kappa * b0;
    }
  }
  const double es = block_sum<EVAL_BLOCK>(e, lds);
  const double bs = block_sum<EVAL_BLOCK>(bad, lds);
  if (threadIdx.x == 0) {
    a.e_part[blockIdx.x] = es;
    bad_part[blockIdx.x] = bs;
  }
}

template <int TYPE, int K, bool TRI_FREE = false>
void launch_tk(const ContactArgs& a, bool exact, hipStream_t s) {
  const int grid = (a.end - a.begin + EVAL_BLOCK - 1) / EVAL_BLOCK;
  if (exact)
    hipLaunchKernelGGL((contact_kernel<TYPE, K, true, TRI_FREE>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL((contact_kernel<TYPE, K, false, TRI_FREE>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
}

}  // namespace

void launch_contact_eval(int type, int nfree, const ContactArgs& a, bool exact, hipStream_t s) {
  if (a.end <= a.begin) return;
  switch (type * 8 + nfree) {
    case 0 * 8 + 1: launch_tk<0, 1>(a, exact, s); break;
    case 0 * 8 + 2: launch_tk<0, 2>(a, exact, s); break;
    case 0 * 8 + 3: launch_tk<0, 3>(a, exact, s); break;
    case 0 * 8 + 4: launch_tk<0, 4>(a, exact, s); break;
    case 0 * 8 + PT_TRIANGLE_FREE: launch_tk<0, 3, true>(a, exact, s); break;
    case 1 * 8 + 1: launch_tk<1, 1>(a, exact, s); break;
    case 1 * 8 + 2: launch_tk<1, 2>(a, exact, s); break;
    case 1 * 8 + 3: launch_tk<1, 3>(a, exact, s); break;
    case 1 * 8 + 4: launch_tk<1, 4>(a, exact, s); break;
    case 2 * 8 + 1: launch_tk<2, 1>(a, exact, s); break;
    case 2 * 8 + 2: launch_tk<2, 2>(a, exact, s); break;
    case 2 * 8 + 3: launch_tk<2, 3>(a, exact, s); break;
    case 3 * 8 + 1: launch_tk<3, 1>(a, exact, s); break;
    case 3 * 8 + 2: launch_tk<3, 2>(a, exact, s); break;
    default: break;
  }
}

void launch_contact_energy(int type, const ContactArgs& a, const double* x0, double* bad_part,
                           hipStream_t s) {
  if (a.end <= a.begin) return;
  const int grid = (a.end - a.begin + EVAL_BLOCK - 1) / EVAL_BLOCK;
  switch (type) {
    case 0: hipLaunchKernelGGL((contact_energy_kernel<0>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a, x0, bad_part); break;
    case 1: hipLaunchKernelGGL((contact_energy_kernel<1>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a, x0, bad_part); break;
    case 2: hipLaunchKernelGGL((contact_energy_kernel<2>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a, x0, bad_part); break;
    default: hipLaunchKernelGGL((contact_energy_kernel<3>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a, x0, bad_part); break;
  }
}

}  // namespace yasps
