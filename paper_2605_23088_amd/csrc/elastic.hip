// Stable Neo-Hookean tetrahedra: energy, gradient and F-space projected Hessian.
//
// Energy (Eq. snh, section "Eigendecomposition: Manual Optimization"):
//   Psi = V [mu/2 (I_C - 3) - mu/2 log(I_C + 1) + lam/2 (J - alpha)^2] - Psi(I),
//   F = Ds Dm^-1, I_C = |F|_F^2, J = det F, alpha = 1 + 3 mu / (4 lam).
// Derivatives, written by hand with F's columns f_j and vec F column-major
// (entry F_ij at i + 3j):
//   dPsi/dF   = V [mu (1 - 1/(I_C+1)) F + lam (J - alpha) cof F],
//               cof F = [f1 x f2, f2 x f0, f0 x f1] (= dJ/dF)
//   d2Psi/dF2 = V [mu (1 - 1/(I_C+1)) I9 + 2 mu/(I_C+1)^2 vec F vec F^T
//                  + lam vec cofF vec cofF^T + lam (J - alpha) H_J],
//   H_J block (j, k), j != k, m the third column index: eps_jkm [f_m]x^T.
// The x-space Hessian is h^2 J_F^T Proj(d2Psi/dF2) J_F: because F is linear
// in x the reduced 9x9 matrix is projected instead of the 12x12 one (section
// "Eigendecomposition (EVD) and PSD Projection", "Projecting in reduced
// coordinates").  With D' = [-(1^T Dm^-1); Dm^-1] (4x3), dF_{:,j}/dx_a = D'_aj I3,
// so block (a, b) = sum_jk D'_aj D'_bk [P]_(jk) with [P]_(jk) the 3x3 block of
// the projected matrix at column blocks (j, k).
#include "blockreduce.h"
#include "contact_math.h"
#include "eigen.h"
#include "kernels.h"
#include "snh_math.h"

namespace yasps {

namespace {

template <class R>
struct Tet {
  int v[4];
  R Dp[4][3];
  R F[3][3];
  R vol, mu, lam;
};

YDEV const double* vertex_ptr(const double* x, const double* xf, int n_free, int v) {
  return v < n_free ? x + 3 * (size_t)v : xf + 3 * (size_t)(v - n_free);
}

template <class R>
YDEV bool load_tet(const SnhArgs& a, int t, Tet<R>& T) {
  const int nt = a.nt;
  double xa[4][3];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T.v[k] = a.idx[k * nt + t];
    const double* p = vertex_ptr(a.x, a.x_fixed, a.n_free, T.v[k]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      xa[k][i] = p[i];
      ok = ok && finite(xa[k][i]);
    }
  }
  double D[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) D[r][c] = a.dm_inv[(3 * r + c) * nt + t];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    T.Dp[0][j] = R(-(D[0][j] + D[1][j] + D[2][j]));
#pragma unroll
    for (int k = 0; k < 3; ++k) T.Dp[k + 1][j] = R(D[k][j]);
  }
  // F = Ds Dm^-1 from edge differences (no cancellation against the absolute position)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) acc = fma(xa[k + 1][i] - xa[0][i], D[k][j], acc);
      T.F[i][j] = R(acc);
    }
  T.vol = R(a.vol[t]);
  if (a.mu_lam) {
    T.mu = R(a.mu_lam[t]);
    T.lam = R(a.mu_lam[nt + t]);
  } else {
    T.mu = R(a.mu);
    T.lam = R(a.lam);
  }
  return ok;
}

template <class R>
YDEV void cross3(const R a[3], const R b[3], R c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Element (i, l) of the cross-product matrix [a]x.
template <class R>
YDEV R crossmat(const R a[3], int i, int l) {
  if (i == l) return R(0);
  if (i == 0 && l == 1) return -a[2];
  if (i == 0 && l == 2) return a[1];
  if (i == 1 && l == 0) return a[2];
  if (i == 1 && l == 2) return -a[0];
  if (i == 2 && l == 0) return -a[1];
  return a[0];  // (2, 1)
}

// Levi-Civita symbol of three distinct indices in {0,1,2}.
YDEV constexpr int eps3(int j, int k, int m) {
  return ((j == 0 && k == 1 && m == 2) || (j == 1 && k == 2 && m == 0) || (j == 2 && k == 0 && m == 1)) ? 1 : -1;
}

template <class R>
struct Invariants {
  R f[3][3];    // columns of F
  R cof[3][3];  // columns of cof F
  R Ic, J, alpha, Jm, ic1, k1;
};

template <class R>
YDEV void invariants(const Tet<R>& T, Invariants<R>& I) {
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 3; ++i) I.f[j][i] = T.F[i][j];
  cross3(I.f[1], I.f[2], I.cof[0]);
  cross3(I.f[2], I.f[0], I.cof[1]);
  cross3(I.f[0], I.f[1], I.cof[2]);
  R Ic = R(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Ic = fmaR(T.F[i][j], T.F[i][j], Ic);
  I.Ic = Ic;
  I.J = I.f[0][0] * I.cof[0][0] + I.f[0][1] * I.cof[0][1] + I.f[0][2] * I.cof[0][2];
  I.alpha = R(1) + R(3) * T.mu / (R(4) * T.lam);
  I.Jm = I.J - I.alpha;
  I.ic1 = R(1) / (Ic + R(1));
  I.k1 = T.mu * (R(1) - I.ic1);
}

// Psi (without h^2) and P = dPsi/dF.
template <class R>
YDEV R snh_energy_grad(const Tet<R>& T, R P[3][3]) {
  Invariants<R> I;
  invariants(T, I);
  const R mu = T.mu, lam = T.lam, V = T.vol;
  const R psi_rest = -R(0.5) * mu * logR(R(4)) + R(0.5) * lam * (R(1) - I.alpha) * (R(1) - I.alpha);
  const R psi = V * (R(0.5) * mu * (I.Ic - R(3)) - R(0.5) * mu * logR(I.Ic + R(1)) + R(0.5) * lam * I.Jm * I.Jm -
                     psi_rest);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) P[i][j] = V * (I.k1 * T.F[i][j] + lam * I.Jm * I.cof[j][i]);
  return psi;
}

// H = d2Psi/dF2 (9x9, vec column-major).
template <class R>
YDEV void snh_hessian(const Tet<R>& T, Sym<9, R>& H) {
  Invariants<R> I;
  invariants(T, I);
  const R lam = T.lam, V = T.vol;
  const R k2 = R(2) * T.mu * I.ic1 * I.ic1;
  const R kJ = lam * I.Jm;
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = r; c < 9; ++c) {
      const int i = r % 3, j = r / 3, l = c % 3, k = c / 3;
      R h = k2 * I.f[j][i] * I.f[k][l] + lam * I.cof[j][i] * I.cof[k][l];
      if (r == c) h += I.k1;
      if (j != k) {
        const int m = 3 - j - k;
        // eps_jkm [f_m]x^T (i, l) = -eps_jkm [f_m]x (i, l)
        h += kJ * R(-eps3(j, k, m)) * crossmat(I.f[m], i, l);
      }
      H(r, c) = V * h;
    }
}

template <class R>
YDEV void convert_tet(const Tet<double>& T, Tet<R>& O) {
#pragma unroll
  for (int k = 0; k < 4; ++k) O.v[k] = T.v[k];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) O.Dp[a][j] = R(T.Dp[a][j]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) O.F[i][j] = R(T.F[i][j]);
  O.vol = R(T.vol);
  O.mu = R(T.mu);
  O.lam = R(T.lam);
}

template <class R, class OUT>
YDEV void store_block(OUT* dst, const R B[3][3], bool transpose) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int l = 0; l < 3; ++l) dst[3 * i + l] = OUT(transpose ? B[l][i] : B[i][l]);
}

// The 4 gradient rows h^2 J_F^T vec P (float64) to their staged slots.
YDEV void scatter_grad(const SnhArgs& a, int t, const Tet<double>& T, const double P[3][3]) {
  const int nt = a.nt;
#pragma unroll
  for (int aa = 0; aa < 4; ++aa) {
    const int pos = a.gpos[aa * nt + t];
    if (pos < 0) continue;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) acc = fma(T.Dp[aa][j], P[i][j], acc);
      a.grd[3 * (size_t)pos + i] = a.h2 * acc;
    }
  }
}

// Writes the 10 upper 3x3 blocks h^2 J_F^T A J_F (A = projected or exact
// d2Psi/dF2) to their staged slots.
template <class R, class OUT>
YDEV void scatter_tet(const SnhArgs& a, int t, const Tet<R>& T, const Sym<9, R>& A, OUT* blk) {
  const int nt = a.nt;
  const R h2 = R(a.h2);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    // Tb[j][i][l] = sum_k D'_bk A(i + 3j, l + 3k)
    R Tb[3][3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          R acc = R(0);
#pragma unroll
          for (int k = 0; k < 3; ++k) acc = fmaR(T.Dp[b][k], A(i + 3 * j, l + 3 * k), acc);
          Tb[j][i][l] = acc;
        }
#pragma unroll
    for (int aa = 0; aa <= b; ++aa) {
      const int q = aa * 4 - (aa * (aa - 1)) / 2 + (b - aa);
      const int pos = a.spos[q * nt + t];
      if (pos < 0) continue;
      R B[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          R acc = R(0);
#pragma unroll
          for (int j = 0; j < 3; ++j) acc = fmaR(T.Dp[aa][j], Tb[j][i][l], acc);
          B[i][l] = h2 * acc;
        }
      if (aa == b) {  // exactly symmetric diagonal block
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int l = i + 1; l < 3; ++l) {
            const R s = R(0.5) * (B[i][l] + B[l][i]);
            B[i][l] = s;
            B[l][i] = s;
          }
      }
      store_block(blk + 9 * (size_t)pos, B, T.v[aa] > T.v[b]);
    }
  }
}

// X-space projection (the paper's plain "YASPS" rows of Table 1): Proj of
// the x-space Hessian J_F^T A J_F (A = d2Psi/dF2, exact) over the tet's free
// vertices.  With a 4 x 3 matrix S whose columns span the free directions,
// C = D'^T S and Y = (C (x) I3)^T A (C (x) I3) is that Hessian in the basis
// S (x) I3, so the x-space blocks are sum_pq S_ap S_bq Proj(Y)_(pq): the
// same map as the F-space scatter with D' replaced by S.
//  * all four vertices free: S = the Helmert basis (the energy is translation
//    invariant, so the 12 x 12 Hessian annihilates the translations and the
//    projection reduces exactly to this 9 x 9 one);
//  * otherwise S selects the free vertices (columns of the fixed ones stay
//    zero, and Proj of a matrix padded with zero rows and columns is the
//    padded projection), which is the projection of the free principal
//    submatrix.
template <class R>
YDEV void xspace_projection(Tet<R>& T, const Sym<9, R>& A, int n_free, Sym<9, R>& Y) {
  R S[4][3];
  const bool all_free = T.v[0] < n_free && T.v[1] < n_free && T.v[2] < n_free && T.v[3] < n_free;
  int nf = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const bool fr = T.v[a] < n_free;
#pragma unroll
    for (int p = 0; p < 3; ++p)
      S[a][p] = all_free ? R(cmath::helmert(a, p)) : ((fr && nf == p) ? R(1) : R(0));
    nf += fr ? 1 : 0;
  }
  R C[3][3];  // C[j][p] = sum_a D'_aj S_ap
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      R acc = R(0);
#pragma unroll
      for (int a = 0; a < 4; ++a) acc = fmaR(T.Dp[a][j], S[a][p], acc);
      C[j][p] = acc;
    }
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = r; c < 9; ++c) {
      const int i = r % 3, p = r / 3, l = c % 3, q = c / 3;
      R acc = R(0);
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k) acc = fmaR(C[j][p] * C[k][q], A(i + 3 * j, l + 3 * k), acc);
      Y(r, c) = acc;
    }
  psd_project<9, R>(Y);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int p = 0; p < 3; ++p) T.Dp[a][p] = S[a][p];
}

template <class R, bool EXACT, bool XSPACE>
__global__ __launch_bounds__(EVAL_BLOCK) void snh_eval_kernel(SnhArgs a) {
  __shared__ double lds[EVAL_BLOCK];
  const int t = blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0;
  if (t < a.nt) {
    // energy and gradient in float64; Hessian and its projection in R
    Tet<double> T;
    const bool ok = load_tet<double>(a, t, T);
    {
      double P[3][3];
      e = a.h2 * snh_energy_grad<double>(T, P);
      scatter_grad(a, t, T, P);
    }
    if (!ok || !finite(e)) atomicOr(a.flags, FLAG_NONFINITE);
    // projected: closed-form eigensystem of d2Psi/dF2 (snh_math.h); exact: the Hessian itself
    // x-space: Proj of the free-vertex x-space Hessian (xspace_projection)
    Sym<9, R> H;
    if constexpr (sizeof(R) == 8) {
      if (EXACT || XSPACE)
        snh_hessian<double>(T, H);
      else
        snh::projected_hessian<double>(T.F, T.mu, T.lam, T.vol, H);
      if (XSPACE && !EXACT) {
        Sym<9, double> Y;
        xspace_projection<double>(T, H, a.n_free, Y);
        scatter_tet<double, double>(a, t, T, Y, a.blk);
      } else {
        scatter_tet<double, double>(a, t, T, H, a.blk);
      }
    } else {
      Tet<R> TR;
      convert_tet<R>(T, TR);
      if (EXACT || XSPACE)
        snh_hessian<R>(TR, H);
      else
        snh::projected_hessian<R>(TR.F, TR.mu, TR.lam, TR.vol, H);
      if (XSPACE && !EXACT) {
        Sym<9, R> Y;
        xspace_projection<R>(TR, H, a.n_free, Y);
        scatter_tet<R, float>(a, t, TR, Y, a.blk32);
      } else {
        scatter_tet<R, float>(a, t, TR, H, a.blk32);
      }
    }
  }
  const double s = block_sum<EVAL_BLOCK>(e, lds);
  if (threadIdx.x == 0) a.e_part[blockIdx.x] = s;
}

__global__ __launch_bounds__(EVAL_BLOCK) void snh_energy_kernel(SnhArgs a) {
  __shared__ double lds[EVAL_BLOCK];
  const int t = blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0;
  if (t < a.nt) {
    Tet<double> T;
    const bool ok = load_tet<double>(a, t, T);
    double P[3][3];
    e = a.h2 * snh_energy_grad<double>(T, P);
    if (!ok || !finite(e)) e = __builtin_nan("");
  }
  const double s = block_sum<EVAL_BLOCK>(e, lds);
  if (threadIdx.x == 0) a.e_part[blockIdx.x] = s;
}

__global__ __launch_bounds__(EVAL_BLOCK) void snh_theta_kernel(SnhArgs a, const double* lambda,
                                                               const double* theta, double* out) {
  const int t = blockIdx.x * EVAL_BLOCK + threadIdx.x;
  if (t >= a.nt) return;
  Tet<double> T;
  load_tet<double>(a, t, T);
  double P[3][3];
  snh_energy_grad<double>(T, P);
  double acc = 0.0;
#pragma unroll
  for (int aa = 0; aa < 4; ++aa) {
    const int v = T.v[aa];
    if (v >= a.n_free) continue;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double gi = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) gi = fma(T.Dp[aa][j], P[i][j], gi);
      acc = fma(lambda[3 * (size_t)v + i], gi, acc);
    }
  }
  out[t] = -a.h2 * acc / theta[t];
}

}  // namespace

void launch_snh_eval(const SnhArgs& a, bool exact, bool mixed, bool xspace, hipStream_t s) {
  if (a.nt == 0) return;
  const int grid = (a.nt + EVAL_BLOCK - 1) / EVAL_BLOCK;
  const dim3 g(grid), b(EVAL_BLOCK);
  if (mixed) {
    if (exact)
      hipLaunchKernelGGL((snh_eval_kernel<float, true, false>), g, b, 0, s, a);
    else if (xspace)
      hipLaunchKernelGGL((snh_eval_kernel<float, false, true>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((snh_eval_kernel<float, false, false>), g, b, 0, s, a);
  } else {
    if (exact)
      hipLaunchKernelGGL((snh_eval_kernel<double, true, false>), g, b, 0, s, a);
    else if (xspace)
      hipLaunchKernelGGL((snh_eval_kernel<double, false, true>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((snh_eval_kernel<double, false, false>), g, b, 0, s, a);
  }
}

void launch_snh_energy(const SnhArgs& a, hipStream_t s) {
  if (a.nt == 0) return;
  const int grid = (a.nt + EVAL_BLOCK - 1) / EVAL_BLOCK;
  hipLaunchKernelGGL(snh_energy_kernel, dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
}

void launch_snh_theta_adjoint(const SnhArgs& a, const double* lambda, const double* theta,
                              double* out, hipStream_t s) {
  if (a.nt == 0) return;
  const int grid = (a.nt + EVAL_BLOCK - 1) / EVAL_BLOCK;
  hipLaunchKernelGGL(snh_theta_kernel, dim3(grid), dim3(EVAL_BLOCK), 0, s, a, lambda, theta, out);
}

// ---------------------------------------------------------------- inertia

namespace {

__global__ __launch_bounds__(EVAL_BLOCK) void inertia_kernel(InertiaArgs a, int with_blocks) {
  __shared__ double lds[EVAL_BLOCK];
  const int v = blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0;
  if (v < a.n) {
    const double m = a.mass[v];
    double g[3];
    bool ok = true;
    if (a.is_static) {
      // gravity potential -m g . x
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double xi = a.x[3 * (size_t)v + i];
        ok = ok && finite(xi);
        e = fma(-m * a.g[i], xi, e);
        g[i] = -m * a.g[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double dx = a.x[3 * (size_t)v + i] - a.x_tilde[3 * (size_t)v + i];
        ok = ok && finite(dx);
        e = fma(0.5 * m * dx, dx, e);
        g[i] = m * dx;
      }
    }
    if (!ok) atomicOr(a.flags, FLAG_NONFINITE);
    if (with_blocks) {
      const int gp = a.gpos[v];
#pragma unroll
      for (int i = 0; i < 3; ++i) a.grd[3 * (size_t)gp + i] = g[i];
      const int sp = a.spos[v];
      if (sp >= 0) {
        if (a.blk32) {
#pragma unroll
          for (int k = 0; k < 9; ++k) a.blk32[9 * (size_t)sp + k] = (k % 4 == 0) ? float(m) : 0.0f;
        } else {
#pragma unroll
          for (int k = 0; k < 9; ++k) a.blk[9 * (size_t)sp + k] = (k % 4 == 0) ? m : 0.0;
        }
      }
    } else if (!ok) {
      e = __builtin_nan("");
    }
  }
  const double s = block_sum<EVAL_BLOCK>(e, lds);
  if (threadIdx.x == 0) a.e_part[blockIdx.x] = s;
}

}  // namespace

void launch_inertia(const InertiaArgs& a, hipStream_t s) {
  if (a.n == 0) return;
  hipLaunchKernelGGL(inertia_kernel, dim3((a.n + EVAL_BLOCK - 1) / EVAL_BLOCK), dim3(EVAL_BLOCK), 0, s,
                     a, 1);
}

void launch_inertia_energy(const InertiaArgs& a, hipStream_t s) {
  if (a.n == 0) return;
  hipLaunchKernelGGL(inertia_kernel, dim3((a.n + EVAL_BLOCK - 1) / EVAL_BLOCK), dim3(EVAL_BLOCK), 0, s,
                     a, 0);
}

}  // namespace yasps
