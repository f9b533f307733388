// Cloth kernels: StVK membrane triangles and dihedral bending hinges, one
// thread per stencil.  Hinges are stored grouped by their number of free
// vertices so each group runs one specialised kernel (as the contact
// stencils).  Per-stencil arithmetic is in cloth_math.h; outputs go to the
// static part's staging arrays like the tets'.
#include "blockreduce.h"
#include "cloth_math.h"
#include "kernels.h"

namespace yasps {

namespace {

YDEV const double* vtx(const double* x, const double* x_fixed, int n_free, int v) {
  return v < n_free ? x + 3 * (size_t)v : x_fixed + 3 * (size_t)(v - n_free);
}

YDEV void put_block(double* blk, float* blk32, int pos, const double (&B)[3][3], bool tr) {
  if (blk32) {
    float* dst = blk32 + 9 * (size_t)pos;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int l = 0; l < 3; ++l) dst[3 * i + l] = float(tr ? B[l][i] : B[i][l]);
  } else {
    double* dst = blk + 9 * (size_t)pos;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int l = 0; l < 3; ++l) dst[3 * i + l] = tr ? B[l][i] : B[i][l];
  }
}

YDEV void load_membrane(const MembraneArgs& a, int f, int (&v)[3], double (&xv)[3][3], double (&D)[2][2]) {
  const int nf = a.nf;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[k] = a.idx[k * nf + f];
    const double* p = vtx(a.x, a.x_fixed, a.n_free, v[k]);
    xv[k][0] = p[0];
    xv[k][1] = p[1];
    xv[k][2] = p[2];
  }
  D[0][0] = a.dm_inv[0 * nf + f];
  D[0][1] = a.dm_inv[1 * nf + f];
  D[1][0] = a.dm_inv[2 * nf + f];
  D[1][1] = a.dm_inv[3 * nf + f];
}

template <bool EXACT>
__global__ __launch_bounds__(EVAL_BLOCK) void membrane_kernel(MembraneArgs a) {
  __shared__ double lds[EVAL_BLOCK];
  const int f = blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0;
  if (f < a.nf) {
    const int nf = a.nf;
    int v[3];
    double xv[3][3], D[2][2];
    load_membrane(a, f, v, xv, D);
    const bool fr[3] = {v[0] < a.n_free, v[1] < a.n_free, v[2] < a.n_free};
    auto gsink = [&](int k, const double (&g)[3]) {
      double* dst = a.grd + 3 * (size_t)a.gpos[k * nf + f];
      dst[0] = g[0];
      dst[1] = g[1];
      dst[2] = g[2];
    };
    auto bsink = [&](int p, int q, const double (&B)[3][3]) {
      put_block(a.blk, a.blk32, a.spos[cmath::pair_index(p, q, 3) * nf + f], B, v[p] > v[q]);
    };
    const bool ok = cloth::membrane_stencil<EXACT>(xv, D, a.area[f], a.thick, a.mu, a.lam, a.h2, fr, e, gsink, bsink);
    if (!ok) atomicOr(a.flags, FLAG_NONFINITE);
  }
  const double es = block_sum<EVAL_BLOCK>(e, lds);
  if (threadIdx.x == 0) a.e_part[blockIdx.x] = es;
}

__global__ __launch_bounds__(EVAL_BLOCK) void membrane_energy_kernel(MembraneArgs a) {
  __shared__ double lds[EVAL_BLOCK];
  const int f = blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0;
  if (f < a.nf) {
    int v[3];
    double xv[3][3], D[2][2];
    load_membrane(a, f, v, xv, D);
    // F = [x1 - x0, x2 - x0] Dm^-1 and the StVK energy only
    double F[3][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        F[i][j] = (xv[1][i] - xv[0][i]) * D[0][j] + (xv[2][i] - xv[0][i]) * D[1][j];
    double G[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int l = 0; l < 2; ++l)
        G[j][l] = 0.5 * (F[0][j] * F[0][l] + F[1][j] * F[1][l] + F[2][j] * F[2][l] - (j == l ? 1.0 : 0.0));
    const double trG = G[0][0] + G[1][1];
    e = a.h2 * a.area[f] * a.thick *
        (a.mu * (G[0][0] * G[0][0] + 2.0 * G[0][1] * G[0][1] + G[1][1] * G[1][1]) + 0.5 * a.lam * trG * trG);
  }
  const double es = block_sum<EVAL_BLOCK>(e, lds);
  if (threadIdx.x == 0) a.e_part[blockIdx.x] = es;
}

template <int K, bool EXACT>
__global__ __launch_bounds__(EVAL_BLOCK) void hinge_kernel(HingeArgs a) {
  __shared__ double lds[EVAL_BLOCK];
  const int h = a.begin + blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0;
  if (h < a.end) {
    const int nh = a.nh;
    int v[4];
    double xv[4][3];
    int fl[4] = {0, 0, 0, 0};
    int nf = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = a.idx[k * nh + h];
      const double* p = vtx(a.x, a.x_fixed, a.n_free, v[k]);
      xv[k][0] = p[0];
      xv[k][1] = p[1];
      xv[k][2] = p[2];
      const bool f = v[k] < a.n_free;
#pragma unroll
      for (int j = 0; j < 4; ++j) fl[j] = (f && nf == j) ? k : fl[j];
      nf += f ? 1 : 0;
    }
    auto gsink = [&](int k, const double (&g)[3]) {
      double* dst = a.grd + 3 * (size_t)a.gpos[fl[k] * nh + h];
      dst[0] = g[0];
      dst[1] = g[1];
      dst[2] = g[2];
    };
    auto bsink = [&](int I, int J, const double (&B)[3][3]) {
      put_block(a.blk, a.blk32, a.spos[cmath::pair_index(fl[I], fl[J], 4) * nh + h], B, v[fl[I]] > v[fl[J]]);
    };
    double theta;
    const bool ok = cloth::hinge_stencil<K, EXACT>(xv, fl, a.rest[h], a.rest[nh + h], a.h2, e, theta, gsink, bsink);
    if (!ok) atomicOr(a.flags, FLAG_NONFINITE);
  }
  const double es = block_sum<EVAL_BLOCK>(e, lds);
  if (threadIdx.x == 0) a.e_part[blockIdx.x] = es;
}

__global__ __launch_bounds__(EVAL_BLOCK) void hinge_energy_kernel(HingeArgs a) {
  __shared__ double lds[EVAL_BLOCK];
  const int h = a.begin + blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0;
  if (h < a.end) {
    const int nh = a.nh;
    double x0[3], u[3][3];
    const double* p0 = vtx(a.x, a.x_fixed, a.n_free, a.idx[h]);
    x0[0] = p0[0];
    x0[1] = p0[1];
    x0[2] = p0[2];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      const double* p = vtx(a.x, a.x_fixed, a.n_free, a.idx[k * nh + h]);
#pragma unroll
      for (int i = 0; i < 3; ++i) u[k - 1][i] = p[i] - x0[i];
    }
    double axb[3];
    cmath::cross(u[1], u[2], axb);
    const double gam = cmath::dot(u[0], u[0]);
    const double P = -sqrt(gam) * cmath::dot(u[0], axb);
    const double Q = cmath::dot(u[0], u[1]) * cmath::dot(u[0], u[2]) - gam * cmath::dot(u[1], u[2]);
    const double d = atan2(P, Q) - a.rest[h];
    e = a.h2 * a.rest[nh + h] * d * d;
  }
  const double es = block_sum<EVAL_BLOCK>(e, lds);
  if (threadIdx.x == 0) a.e_part[blockIdx.x] = es;
}

template <int K>
void launch_hk(const HingeArgs& a, bool exact, hipStream_t s) {
  const int grid = (a.end - a.begin + EVAL_BLOCK - 1) / EVAL_BLOCK;
  if (exact)
    hipLaunchKernelGGL((hinge_kernel<K, true>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL((hinge_kernel<K, false>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
}

}  // namespace

void launch_membrane_eval(const MembraneArgs& a, bool exact, hipStream_t s) {
  if (a.nf <= 0) return;
  const int grid = (a.nf + EVAL_BLOCK - 1) / EVAL_BLOCK;
  if (exact)
    hipLaunchKernelGGL((membrane_kernel<true>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL((membrane_kernel<false>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
}

void launch_membrane_energy(const MembraneArgs& a, hipStream_t s) {
  if (a.nf <= 0) return;
  const int grid = (a.nf + EVAL_BLOCK - 1) / EVAL_BLOCK;
  hipLaunchKernelGGL(membrane_energy_kernel, dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
}

void launch_hinge_eval(int nfree, const HingeArgs& a, bool exact, hipStream_t s) {
  if (a.end <= a.begin) return;
  switch (nfree) {
    case 1: launch_hk<1>(a, exact, s); break;
    case 2: launch_hk<2>(a, exact, s); break;
    case 3: launch_hk<3>(a, exact, s); break;
    case 4: launch_hk<4>(a, exact, s); break;
    default: break;
  }
}

void launch_hinge_energy(const HingeArgs& a, hipStream_t s) {
  if (a.end <= a.begin) return;
  const int grid = (a.end - a.begin + EVAL_BLOCK - 1) / EVAL_BLOCK;
  hipLaunchKernelGGL(hinge_energy_kernel, dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
}

}  // namespace yasps
