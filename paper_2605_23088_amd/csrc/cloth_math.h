// Cloth stencils: StVK membrane triangles and dihedral bending hinges (host /
// device arithmetic shared by the kernels and the host checks).
//
// Membrane.  F = [x1 - x0, x2 - x0] Dm^-1 (3x2), G = (F^T F - I) / 2,
//   Psi = A t [mu tr(G^2) + lam/2 (tr G)^2],  dPsi/dF = A t F S with
//   S = 2 mu G + lam tr(G) I, and
//   d2Psi/dF_ij dF_kl = A t [d_ik S_lj + mu F_il F_kj + mu (F F^T)_ik d_jl
//                            + lam F_ij F_kl].
// F is linear in x: dF_ij/dx_{v,c} = d_ic a_vj with a_1j = Dm^-1_0j,
// a_2j = Dm^-1_1j, a_0j = -(a_1j + a_2j).  The 6x6 d2Psi/dF2 is projected in F
// space (the paper's choice for elastic energies, section "Eigendecomposition
// (EVD) and PSD Projection"), then mapped to x and restricted to free vertices.
//
// Hinge.  With e = x1 - x0, a = x2 - x0, b = x3 - x0, the normals
// n1 = e x a, n2 = b x e give n1 . n2 = (e.a)(e.b) - |e|^2 (a.b) =: Q and
// (n1 x n2) . e/|e| = -|e| det[e, a, b] =: P, so theta = atan2(P, Q) and
// E = k (theta - theta_bar)^2 (discrete-shells bending, k = k_b 3|e_bar|^2 /
// (A1 + A2) precomputed).  Derivatives in u = (e, a, b):
//   theta_P = Q / r^2, theta_Q = -P / r^2, r^2 = P^2 + Q^2,
//   theta_PP = -2PQ / r^4 = -theta_QQ, theta_PQ = (P^2 - Q^2) / r^4;
//   P = -L V with L = |e|, V = e . (a x b):
//     grad V = (a x b, b x e, e x a), hess V blocks (e,a) = -[b]x,
//     (e,b) = [a]x, (a,b) = -[e]x; grad L = (e/L, 0, 0),
//     hess L (e,e) = (I - e e^T / L^2) / L;
//   Q = alpha beta - gamma delta, alpha = e.a, beta = e.b, gamma = e.e,
//     delta = a.b, whose gradients / constant Hessians are read off directly.
// The 12x12 Hessian is projected through the same reduction as the contact
// stencils (Helmert basis when all four vertices are free).
#pragma once

#include "contact_math.h"

namespace yasps {
namespace cloth {

using cmath::cm;
using cmath::cross;
using cmath::dot;

// Energy, gradient rows and upper blocks of one membrane triangle.  free[v]
// selects the vertices that receive gradient rows and blocks (fixed vertices
// are dropped after the F-space projection).  Sinks: grad_sink(v, g[3]),
// block_sink(v, w, B[3][3]) for v <= w local vertex indices.  Everything is
// scaled by h2 (the elastic term of the incremental potential).
template <bool EXACT, class GS, class BS>
YHD bool membrane_stencil(const double (&xv)[3][3], const double (&Dinv)[2][2], double area, double thick, double mu,
                          double lam, double h2, const bool (&free)[3], double& e, GS&& grad_sink, BS&& block_sink) {
  double a[3][2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    a[1][j] = Dinv[0][j];
    a[2][j] = Dinv[1][j];
    a[0][j] = -(Dinv[0][j] + Dinv[1][j]);
  }
  double F[3][2];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int v = 0; v < 3; ++v) acc = fma(a[v][j], xv[v][i], acc);
      F[i][j] = acc;
      ok = ok && finite(acc);
    }
  double G[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int l = 0; l < 2; ++l)
      G[j][l] = 0.5 * (F[0][j] * F[0][l] + F[1][j] * F[1][l] + F[2][j] * F[2][l] - (j == l ? 1.0 : 0.0));
  const double trG = G[0][0] + G[1][1];
  const double At = area * thick;
  e = h2 * At * (mu * (G[0][0] * G[0][0] + 2.0 * G[0][1] * G[0][1] + G[1][1] * G[1][1]) + 0.5 * lam * trG * trG);
  double S[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int l = 0; l < 2; ++l) S[j][l] = 2.0 * mu * G[j][l] + (j == l ? lam * trG : 0.0);
  double P[3][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) P[i][j] = At * (F[i][0] * S[0][j] + F[i][1] * S[1][j]);
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    if (!free[v]) continue;
    double g[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = h2 * (a[v][0] * P[i][0] + a[v][1] * P[i][1]);
    grad_sink(v, g);
  }
  // d2Psi/dF2, F-space index f(i, j) = i + 3 j
  double FFt[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) FFt[i][k] = F[i][0] * F[k][0] + F[i][1] * F[k][1];
  Sym<6, double> K;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r; c < 6; ++c) {
      const int i = r % 3, j = r / 3, k = c % 3, l = c / 3;
      double h = mu * F[i][l] * F[k][j] + lam * F[i][j] * F[k][l];
      if (i == k) h += S[l][j];
      if (j == l) h += mu * FFt[i][k];
      K(r, c) = At * h;
    }
  if (!EXACT) psd_project<6, double>(K);
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int w = v; w < 3; ++w) {
      if (!free[v] || !free[w]) continue;
      double B[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int l = 0; l < 2; ++l) acc = fma(a[v][j] * a[w][l], K(i + 3 * j, k + 3 * l), acc);
          B[i][k] = h2 * acc;
        }
      if (v == w) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int k = i + 1; k < 3; ++k) {
            const double m = 0.5 * (B[i][k] + B[k][i]);
            B[i][k] = m;
            B[k][i] = m;
          }
      }
      block_sink(v, w, B);
    }
  return ok && finite(e);
}

// Hinge difference variables u = (e, a, b) = (x1 - x0, x2 - x0, x3 - x0).
struct HingeTopo {
  static constexpr int NV = 4, NU = 3;
  static YHD constexpr int M(int U, int a) { return a == U + 1 ? 1 : (a == 0 ? -1 : 0); }
};

// Hessian block (U, W) entry (i, l) of V = e . (a x b) in u = (e, a, b).
YHD double hessV(const double e[3], const double a[3], const double b[3], int U, int W, int i, int l) {
  if (U == W) return 0.0;
  if (U == 0 && W == 1) return -cm(b, i, l);
  if (U == 0 && W == 2) return cm(a, i, l);
  if (U == 1 && W == 2) return -cm(e, i, l);
  if (U == 1 && W == 0) return -cm(b, l, i);
  if (U == 2 && W == 0) return cm(a, l, i);
  return -cm(e, l, i);  // (2, 1)
}

// Energy, free-vertex gradient rows and projected upper blocks of one hinge
// with K free vertices (fl as in cmath::emit_reduced), scaled by h2.
template <int K, bool EXACT, class GS, class BS>
YHD bool hinge_stencil(const double (&xv)[4][3], const int (&fl)[4], double theta_bar, double stiff, double h2,
                       double& e_out, double& theta_out, GS&& grad_sink, BS&& block_sink) {
  double u[3][3];
  bool ok = true;
#pragma unroll
  for (int U = 0; U < 3; ++U)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u[U][i] = xv[U + 1][i] - xv[0][i];
      ok = ok && finite(u[U][i]);
    }
  const double *e = u[0], *a = u[1], *b = u[2];
  double axb[3], bxe[3], exa[3];
  cross(a, b, axb);
  cross(b, e, bxe);
  cross(e, a, exa);
  const double V = dot(e, axb);
  const double gam = dot(e, e), L = sqrt(gam), iL = 1.0 / L;
  const double al = dot(e, a), be = dot(e, b), de = dot(a, b);
  const double P = -L * V;
  const double Q = al * be - gam * de;
  const double theta = atan2(P, Q);
  const double r2 = P * P + Q * Q, ir2 = 1.0 / r2, ir4 = ir2 * ir2;
  ok = ok && finite(ir4) && L > 0.0;  // degenerate hinge: zero-area wing or edge
  const double tP = Q * ir2, tQ = -P * ir2;
  const double tPP = -2.0 * P * Q * ir4, tQQ = -tPP, tPQ = (P * P - Q * Q) * ir4;
  // first derivatives in u
  double gV[9], gL[9], gP[9], gQ[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gV[i] = axb[i];
    gV[3 + i] = bxe[i];
    gV[6 + i] = exa[i];
    gL[i] = e[i] * iL;
    gL[3 + i] = 0.0;
    gL[6 + i] = 0.0;
  }
#pragma unroll
  for (int r = 0; r < 9; ++r) gP[r] = -(V * gL[r] + L * gV[r]);
  // grad Q = beta grad alpha + alpha grad beta - delta grad gamma - gamma grad delta
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gQ[i] = be * a[i] + al * b[i] - 2.0 * de * e[i];
    gQ[3 + i] = be * e[i] - gam * b[i];
    gQ[6 + i] = al * e[i] - gam * a[i];
  }
  double gth[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) gth[r] = tP * gP[r] + tQ * gQ[r];
  const double dth = theta - theta_bar;
  const double c1 = 2.0 * stiff * h2;
  e_out = stiff * h2 * dth * dth;
  theta_out = theta;
  double gu[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) gu[r] = c1 * dth * gth[r];
  // gradients of alpha, beta, gamma, delta (for the Q Hessian)
  double ga[9], gb[9], gg[9], gd[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ga[i] = a[i], ga[3 + i] = e[i], ga[6 + i] = 0.0;
    gb[i] = b[i], gb[3 + i] = 0.0, gb[6 + i] = e[i];
    gg[i] = 2.0 * e[i], gg[3 + i] = 0.0, gg[6 + i] = 0.0;
    gd[i] = 0.0, gd[3 + i] = b[i], gd[6 + i] = a[i];
  }
  Sym<9, double> H;
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = r; c < 9; ++c) {
      const int U = r / 3, W = c / 3, i = r % 3, l = c % 3;
      const double dil = i == l ? 1.0 : 0.0;
      // hess L, hess V, hess P
      const double hL = (U == 0 && W == 0) ? (dil - e[i] * e[l] * iL * iL) * iL : 0.0;
      const double hV = hessV(e, a, b, U, W, i, l);
      const double hP = -(V * hL + gL[r] * gV[c] + gV[r] * gL[c] + L * hV);
      // constant Hessians of alpha (e,a), beta (e,b), gamma (e,e), delta (a,b)
      const double ha = ((U == 0 && W == 1) || (U == 1 && W == 0)) ? dil : 0.0;
      const double hb = ((U == 0 && W == 2) || (U == 2 && W == 0)) ? dil : 0.0;
      const double hg = (U == 0 && W == 0) ? 2.0 * dil : 0.0;
      const double hd = ((U == 1 && W == 2) || (U == 2 && W == 1)) ? dil : 0.0;
      const double hQ = ga[r] * gb[c] + gb[r] * ga[c] + be * ha + al * hb - (gg[r] * gd[c] + gd[r] * gg[c]) -
                        de * hg - gam * hd;
      const double hth = tP * hP + tQ * hQ + tPP * gP[r] * gP[c] + tQQ * gQ[r] * gQ[c] +
                         tPQ * (gP[r] * gQ[c] + gQ[r] * gP[c]);
      H(r, c) = c1 * (gth[r] * gth[c] + dth * hth);
    }
  cmath::emit_reduced<HingeTopo, K, EXACT>(gu, H, fl, grad_sink, block_sink);
  return ok && finite(e_out);
}

}  // namespace cloth
}  // namespace yasps
