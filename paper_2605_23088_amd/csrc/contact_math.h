// Log-barrier contact stencils: energy, gradient and projected local Hessian
// of one stencil (host/device arithmetic shared by the kernels and the host
// checks of the device math).
//
// Barrier (section "Eigendecomposition: Automatic Optimization" and the
// point-point code listing of section "Energies"), d a SQUARED distance:
//   b(d) = (d - dhat)^2 log(d/dhat)^2,  E = kappa b(d) for 0 < d < dhat, else 0.
// With u = d - dhat, L = log(d/dhat):
//   b' = 2uL^2 + 2u^2 L/d,   b'' = 2L^2 + 8uL/d + 2u^2 (1 - L)/d^2.
// (classic IPC form -u^2 L: b' = -2uL - u^2/d, b'' = -2L - 4u/d + u^2/d^2.)
//
// Distances are type-fixed (the stencil's type names the closest-feature pair):
//   PT, EE: d = s^2/N,  s = w . (e1 x e2),  N = |e1 x e2|^2 with
//           PT: w = p - t0, e1 = t1 - t0, e2 = t2 - t0
//           EE: w = a0 - b0, e1 = a1 - a0, e2 = b1 - b0
//   PE:     d = S/N,  S = |a x b|^2,  N = |b - a|^2,  a = e0 - p, b = e1 - p
//   PP:     d = |q - p|^2
// Derivatives are taken in these difference variables u (hand-derived closed
// forms below) and mapped to the stencil's vertices by the constant incidence
// matrix M (u_U = sum_a M[U][a] x_a):  H_x = (M (x) I3)^T H_u (M (x) I3).
//
// Projection (section "Eigendecomposition (EVD) and PSD Projection") acts on
// the Hessian restricted to the stencil's free vertices (fixed vertices are
// excluded from differentiation).  When every vertex is free the energy is
// translation invariant, H_x annihilates the 3 translations, and
// Proj(H_x) = Q Proj(Q^T H_x Q) Q^T with Q = Hm (x) I3 (Hm the Helmert basis
// of the vectors orthogonal to (1,...,1)): an exact reduction from 12 to 9
// (PT, EE), 9 to 6 (PE) and 6 to 3 (PP) dimensions.
#pragma once

#include "eigen.h"

namespace yasps {
namespace cmath {

template <int TYPE>
struct Topo;
// PT: x = (p, t0, t1, t2); u = (w, e1, e2)
template <>
struct Topo<0> {
  static constexpr int NV = 4, NU = 3;
  static YHD constexpr int M(int U, int a) {
    return U == 0 ? (a == 0 ? 1 : a == 1 ? -1 : 0) : U == 1 ? (a == 2 ? 1 : a == 1 ? -1 : 0)
                                                            : (a == 3 ? 1 : a == 1 ? -1 : 0);
  }
};
// EE: x = (a0, a1, b0, b1); u = (w = a0 - b0, e1 = a1 - a0, e2 = b1 - b0)
template <>
struct Topo<1> {
  static constexpr int NV = 4, NU = 3;
  static YHD constexpr int M(int U, int a) {
    return U == 0 ? (a == 0 ? 1 : a == 2 ? -1 : 0) : U == 1 ? (a == 1 ? 1 : a == 0 ? -1 : 0)
                                                            : (a == 3 ? 1 : a == 2 ? -1 : 0);
  }
};
// PE: x = (p, e0, e1); u = (a = e0 - p, b = e1 - p)
template <>
struct Topo<2> {
  static constexpr int NV = 3, NU = 2;
  static YHD constexpr int M(int U, int a) {
    return U == 0 ? (a == 1 ? 1 : a == 0 ? -1 : 0) : (a == 2 ? 1 : a == 0 ? -1 : 0);
  }
};
// PP: x = (p, q); u = q - p
template <>
struct Topo<3> {
  static constexpr int NV = 2, NU = 1;
  static YHD constexpr int M(int, int a) { return a == 1 ? 1 : -1; }
};

// Helmert basis: column j (j = 0..k-2) of the k x (k-1) orthonormal basis of
// vectors orthogonal to (1, ..., 1).
YHD double helmert(int a, int j) {
  const double s = 1.0 / sqrt(double((j + 1) * (j + 2)));
  return a <= j ? s : (a == j + 1 ? -double(j + 1) * s : 0.0);
}

YHD void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
YHD double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
// [a]x (i, l)
YHD double cm(const double a[3], int i, int l) {
  if (i == l) return 0.0;
  if (i == 0) return l == 1 ? -a[2] : a[1];
  if (i == 1) return l == 0 ? a[2] : -a[0];
  return l == 0 ? -a[1] : a[0];
}

// Squared distance, its gradient and Hessian in the difference variables.
template <int TYPE>
struct Dist {
  static constexpr int NU = Topo<TYPE>::NU;
  double d;
  double g[3 * NU];
  Sym<3 * NU, double> H;
};

// Q(x) = |x1 x x2|^2 type quantity: gradient and Hessian blocks for
// n = e1 x e2:  dN/de1 = 2 e2 x n, dN/de2 = 2 n x e1,
//   (e1,e1) = 2(|e2|^2 I - e2 e2^T), (e2,e2) = 2(|e1|^2 I - e1 e1^T),
//   (e1,e2) = 2(e1 e2^T - (e1.e2) I - [n]x).
YHD double crossnorm_hess(const double e1[3], const double e2[3], const double n[3], int B1, int B2,
                           int i, int l) {
  if (B1 == 0 && B2 == 0) return 2.0 * ((i == l ? dot(e2, e2) : 0.0) - e2[i] * e2[l]);
  if (B1 == 1 && B2 == 1) return 2.0 * ((i == l ? dot(e1, e1) : 0.0) - e1[i] * e1[l]);
  if (B1 == 0 && B2 == 1) return 2.0 * (e1[i] * e2[l] - (i == l ? dot(e1, e2) : 0.0) - cm(n, i, l));
  // (e2, e1) = transpose of (e1, e2)
  return 2.0 * (e1[l] * e2[i] - (i == l ? dot(e1, e2) : 0.0) - cm(n, l, i));
}

// PT / EE: u = (w, e1, e2), d = s^2 / N.
//   ds = (n, e2 x w, w x e1);  d2s: (w,e1) = -[e2]x, (w,e2) = [e1]x, (e1,e2) = -[w]x
//   dN = (0, 2 e2 x n, 2 n x e1);  d2N as crossnorm_hess on (e1, e2)
//   grad d = (2s/N) ds - (s^2/N^2) dN
//   hess d = (2/N) ds ds^T + (2s/N) d2s - (2s/N^2)(ds dN^T + dN ds^T)
//            - (s^2/N^2) d2N + (2 s^2/N^3) dN dN^T
YHD double d2s_block(const double w[3], const double e1[3], const double e2[3], int B1, int B2, int i,
                      int l) {
  if (B1 == B2) return 0.0;
  if (B1 == 0 && B2 == 1) return -cm(e2, i, l);
  if (B1 == 0 && B2 == 2) return cm(e1, i, l);
  if (B1 == 1 && B2 == 2) return -cm(w, i, l);
  if (B1 == 1 && B2 == 0) return -cm(e2, l, i);
  if (B1 == 2 && B2 == 0) return cm(e1, l, i);
  return -cm(w, l, i);  // (2, 1)
}

template <int TYPE>
YHD void distance(const double (&u)[Topo<TYPE>::NU][3], Dist<TYPE>& D, double& side) {
  if constexpr (TYPE == 0 || TYPE == 1) {
    const double *w = u[0], *e1 = u[1], *e2 = u[2];
    double n[3], e2w[3], we1[3], e2n[3], ne1[3];
    cross(e1, e2, n);
    cross(e2, w, e2w);
    cross(w, e1, we1);
    cross(e2, n, e2n);
    cross(n, e1, ne1);
    const double s = dot(w, n), N = dot(n, n);
    side = s;
    const double iN = 1.0 / N;
    const double d = s * s * iN;
    D.d = d;
    double ds[9], dN[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ds[i] = n[i];
      ds[3 + i] = e2w[i];
      ds[6 + i] = we1[i];
      dN[i] = 0.0;
      dN[3 + i] = 2.0 * e2n[i];
      dN[6 + i] = 2.0 * ne1[i];
    }
    const double c1 = 2.0 * s * iN, c2 = s * s * iN * iN;
#pragma unroll
    for (int r = 0; r < 9; ++r) D.g[r] = c1 * ds[r] - c2 * dN[r];
    const double k_ss = 2.0 * iN, k_s = 2.0 * s * iN, k_sN = 2.0 * s * iN * iN, k_N = c2,
                 k_NN = 2.0 * s * s * iN * iN * iN;
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int c = r; c < 9; ++c) {
        const int B1 = r / 3, B2 = c / 3, i = r % 3, l = c % 3;
        const double hN = (B1 == 0 || B2 == 0) ? 0.0 : crossnorm_hess(e1, e2, n, B1 - 1, B2 - 1, i, l);
        D.H(r, c) = k_ss * ds[r] * ds[c] + k_s * d2s_block(w, e1, e2, B1, B2, i, l) -
                    k_sN * (ds[r] * dN[c] + dN[r] * ds[c]) - k_N * hN + k_NN * dN[r] * dN[c];
      }
  } else if constexpr (TYPE == 2) {
    // PE: u = (a, b), d = S/N, S = |a x b|^2, N = |b - a|^2
    const double *a = u[0], *b = u[1];
    double c[3], bc[3], ca[3], ba[3];
    cross(a, b, c);
    cross(b, c, bc);
    cross(c, a, ca);
#pragma unroll
    for (int i = 0; i < 3; ++i) ba[i] = b[i] - a[i];
    const double S = dot(c, c), N = dot(ba, ba);
    side = 1.0;
    const double iN = 1.0 / N;
    D.d = S * iN;
    double dS[6], dN[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dS[i] = 2.0 * bc[i];
      dS[3 + i] = 2.0 * ca[i];
      dN[i] = -2.0 * ba[i];
      dN[3 + i] = 2.0 * ba[i];
    }
    const double k_S = iN, k_N = S * iN * iN;
#pragma unroll
    for (int r = 0; r < 6; ++r) D.g[r] = k_S * dS[r] - k_N * dN[r];
    const double k_SN = iN * iN, k_NN = 2.0 * S * iN * iN * iN;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int cc = r; cc < 6; ++cc) {
        const int B1 = r / 3, B2 = cc / 3, i = r % 3, l = cc % 3;
        const double hS = crossnorm_hess(a, b, c, B1, B2, i, l);
        const double hN = (i == l) ? (B1 == B2 ? 2.0 : -2.0) : 0.0;
        D.H(r, cc) = k_S * hS - k_SN * (dS[r] * dN[cc] + dN[r] * dS[cc]) - k_N * hN + k_NN * dN[r] * dN[cc];
      }
  } else {
    const double* v = u[0];
    side = 1.0;
    D.d = dot(v, v);
#pragma unroll
    for (int i = 0; i < 3; ++i) D.g[i] = 2.0 * v[i];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = r; cc < 3; ++cc) D.H(r, cc) = (r == cc) ? 2.0 : 0.0;
  }
}

// b, b', b'' of the barrier.
YHD void barrier(double d, double dhat, int classic, double& b0, double& b1, double& b2) {
  const double u = d - dhat, L = log(d / dhat), id = 1.0 / d;
  if (classic) {
    b0 = -u * u * L;
    b1 = -2.0 * u * L - u * u * id;
    b2 = -2.0 * L - 4.0 * u * id + u * u * id * id;
  } else {
    b0 = u * u * L * L;
    b1 = 2.0 * u * L * L + 2.0 * u * u * L * id;
    b2 = 2.0 * L * L + 8.0 * u * L * id + 2.0 * u * u * (1.0 - L) * id * id;
  }
}

YHD int pair_index(int a, int b, int k) { return a * k - (a * (a - 1)) / 2 + (b - a); }

// Difference variables u_U = sum_a M[U][a] x_a of a stencil; false on non-finite input.
template <int TYPE>
YHD bool diff_vars(const double (&xv)[4][3], double (&u)[Topo<TYPE>::NU][3]) {
  constexpr int NV = Topo<TYPE>::NV, NU = Topo<TYPE>::NU;
  bool ok = true;
#pragma unroll
  for (int U = 0; U < NU; ++U)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int m = Topo<TYPE>::M(U, k);
        if (m == 1) acc += xv[k][i];
        if (m == -1) acc -= xv[k][i];
      }
      u[U][i] = acc;
      ok = ok && finite(acc);
    }
  return ok;
}

// Rows (t/|t|, n/|n| x t/|t|, n/|n|) for t orthogonal to n; the identity
// when either vanishes (the stencils below then have a distance that is zero
// or not finite, hence a zero Hessian, which every frame projects to zero).
YHD void orthonormal_frame(const double (&t)[3], const double (&n)[3], double (&Fr)[3][3]) {
  const double lt = sqrt(dot(t, t)), ln = sqrt(dot(n, n));
  const bool ok = lt > 0.0 && ln > 0.0 && finite(lt) && finite(ln);
  const double it = ok ? 1.0 / lt : 0.0, in = ok ? 1.0 / ln : 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Fr[0][i] = ok ? t[i] * it : (i == 0 ? 1.0 : 0.0);
    Fr[2][i] = ok ? n[i] * in : (i == 2 ? 1.0 : 0.0);
  }
  double c[3];
  cross(Fr[2], Fr[0], c);
#pragma unroll
  for (int i = 0; i < 3; ++i) Fr[1][i] = c[i];
}

// Closed-form PSD projection of a symmetric 2 x 2 matrix.  Its eigenvalues are
// mid +- r (mid = (a + c)/2, r = sqrt(((a - c)/2)^2 + b^2)); with one of each
// sign, A - l_- I is (l_+ - l_-) times the projector onto the positive
// eigenvector, so Proj(A) = l_+ (A - l_- I) / (l_+ - l_-).
YHD void psd_project2(Sym<2, double>& A) {
  const double a = A(0, 0), b = A(0, 1), c = A(1, 1);
  const double h = 0.5 * (a - c), mid = 0.5 * (a + c);
  const double r = sqrt(fma(h, h, b * b));
  const double lp = mid + r, lm = mid - r;
  const bool keep = lm >= 0.0;  // both eigenvalues non-negative
  const double f = lp > 0.0 ? lp / (r > 0.0 ? 2.0 * r : 1.0) : 0.0;
  const double sc = keep ? 1.0 : f, sh = keep ? 0.0 : lm;
  A(0, 0) = sc * (a - sh);
  A(0, 1) = sc * b;
  A(1, 1) = sc * (c - sh);
}

template <int N>
YHD void psd_small(Sym<N, double>& A) {
  if constexpr (N == 2)
    psd_project2(A);
  else
    psd_project<N, double>(A);
}

// Frame coordinates of one vertex-slot block of a reduced Hessian A (3 m x 3 m,
// blocks (I, J) of 3 x 3): P'(a, b) = sum_ij Fr[a][i] A(3I + i, 3J + j) Fr[b][j].
template <int NN>
YHD void block_to_frame(const Sym<NN, double>& A, int I, int J, const double (&Fr)[3][3], double (&P)[3][3]) {
  double T[3][3];  // Fr A_IJ
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i) acc = fma(Fr[a][i], A(3 * I + i, 3 * J + j), acc);
      T[a][j] = acc;
    }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) acc = fma(T[a][j], Fr[b][j], acc);
      P[a][b] = acc;
    }
}

// The inverse map: A_IJ = Fr^T P' Fr (the upper entries of a diagonal block).
template <int NN>
YHD void block_from_frame(Sym<NN, double>& A, int I, int J, const double (&Fr)[3][3], const double (&P)[3][3]) {
  double T[3][3];  // P' Fr
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b) acc = fma(P[a][b], Fr[b][j], acc);
      T[a][j] = acc;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (I == J && j < i) continue;
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) acc = fma(Fr[a][i], T[a][j], acc);
      A(3 * I + i, 3 * J + j) = acc;
    }
}

// PSD projection of the reduced Hessian A of a point-triangle or edge-edge
// barrier (m vertex slots: the free vertices, or the Helmert combinations of
// all four).  Fr holds the orthonormal frame (t1, t2, n) of the stencil's plane
// (the triangle's plane; the plane of both edge directions).  The squared
// distance d = s^2/N does not change when the vertices move inside planes
// parallel to it (the triangle stays in its plane and the point keeps its
// height; each edge stays in its own parallel plane), so d is constant on that
// 2m-dimensional affine subspace: its gradient and Hessian vanish there, and
// so does the barrier Hessian kappa (b'' grad d grad d^T + b' hess d).  In
// frame coordinates (two in-plane and one normal component per slot) the
// Hessian is M = [[0, B^T], [B, C]] with the m x 2m normal-by-in-plane block B
// and the m x m normal block C.  With the Householder factorisation
// B^T = Q R (Q 2m x m orthonormal), M = W M' W^T, W = diag(Q, I_m),
// M' = [[0, R], [R^T, C]], and M annihilates the in-plane directions
// orthogonal to Q; so Proj(M) = W Proj(M') W^T, a 2m x 2m eigenproblem in
// place of a 3m x 3m one (closed form for m = 1).  The computed in-plane block
// is zero up to rounding and is dropped.
//
// SHIFT_NULL (the three free slots are a triangle's vertices, the point
// fixed): moving the whole triangle along its normal changes the distance but
// not where the point's foot lies in it, so B annihilates the uniform normal
// shift s = (1, 1, 1)/sqrt(3).  In the normal coordinates rotated to
// (s, the two Helmert directions orthogonal to it) B's first column vanishes
// and is dropped: Q is 2m x (m - 1) and M' is (2m - 1) x (2m - 1).
template <int m, bool SHIFT_NULL = false>
YHD void project_plane(Sym<3 * m, double>& A, const double (&Fr)[3][3]) {
  constexpr int nW = SHIFT_NULL ? m - 1 : m;  // normal directions B reaches
  constexpr int NM = nW + m;                  // size of the reduced problem
  double Bt[2 * m][m];  // Bt[2I + a][J] = P'(I a, J n), a in {t1, t2}
  double Cn[m][m];      // P'(I n, J n)
#pragma unroll
  for (int I = 0; I < m; ++I)
#pragma unroll
    for (int J = I; J < m; ++J) {
      double P[3][3];
      block_to_frame<3 * m>(A, I, J, Fr, P);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        Bt[2 * I + a][J] = P[a][2];
        if (J > I) Bt[2 * J + a][I] = P[2][a];
      }
      Cn[I][J] = P[2][2];
      Cn[J][I] = P[2][2];
    }
  // normal coordinates: Wb[j][c] = component of slot j of direction c (the
  // identity, or (s, Helmert directions))
  double Wb[m][m];
#pragma unroll
  for (int j = 0; j < m; ++j)
#pragma unroll
    for (int c = 0; c < m; ++c)
      Wb[j][c] = SHIFT_NULL ? (c == 0 ? 1.0 / sqrt(double(m)) : helmert(j, c - 1)) : (j == c ? 1.0 : 0.0);
  double Bw[2 * m][nW];  // the columns of Bt Wb that B reaches
#pragma unroll
  for (int r = 0; r < 2 * m; ++r)
#pragma unroll
    for (int c = 0; c < nW; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < m; ++j) acc = fma(Bt[r][j], Wb[j][c + (m - nW)], acc);
      Bw[r][c] = acc;
    }
  double Cw[m][m];  // Wb^T Cn Wb
#pragma unroll
  for (int c = 0; c < m; ++c)
#pragma unroll
    for (int d = 0; d < m; ++d) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < m; ++j)
#pragma unroll
        for (int l = 0; l < m; ++l) acc = fma(Wb[j][c] * Cn[j][l], Wb[l][d], acc);
      Cw[c][d] = acc;
    }
  // Householder QR of Bw (2m x nW): Bw = Q R
  double V[nW][2 * m];  // reflector vectors (v_k has zeros above row k)
  double R[nW][nW];
#pragma unroll
  for (int k = 0; k < nW; ++k) {
    double nrm2 = 0.0;
#pragma unroll
    for (int r = 0; r < 2 * m; ++r) nrm2 = r >= k ? fma(Bw[r][k], Bw[r][k], nrm2) : nrm2;
    const double nrm = sqrt(nrm2);
    const double alpha = Bw[k][k] >= 0.0 ? -nrm : nrm;  // v = x - alpha e_k, no cancellation
    double vn2 = 0.0;
#pragma unroll
    for (int r = 0; r < 2 * m; ++r) {
      const double v = r < k ? 0.0 : (r == k ? Bw[k][k] - alpha : Bw[r][k]);
      V[k][r] = v;
      vn2 = fma(v, v, vn2);
    }
    const double inv = vn2 > 0.0 ? 2.0 / vn2 : 0.0;  // H_k = I - inv v v^T (identity when x = 0)
#pragma unroll
    for (int c = 0; c < nW; ++c) {
      if (c < k) continue;
      double dotv = 0.0;
#pragma unroll
      for (int r = 0; r < 2 * m; ++r) dotv = fma(V[k][r], Bw[r][c], dotv);
      const double f = inv * dotv;
#pragma unroll
      for (int r = 0; r < 2 * m; ++r) Bw[r][c] = fma(-f, V[k][r], Bw[r][c]);
    }
#pragma unroll
    for (int c = 0; c < nW; ++c) R[k][c] = c < k ? 0.0 : Bw[k][c];
    const double sq = sqrt(inv);  // scale so that H_k = I - v v^T
#pragma unroll
    for (int r = 0; r < 2 * m; ++r) V[k][r] *= sq;
  }
  // Q = H_0 ... H_{nW-1} applied to the first nW columns of I_2m
  double Q[2 * m][nW];
#pragma unroll
  for (int r = 0; r < 2 * m; ++r)
#pragma unroll
    for (int c = 0; c < nW; ++c) Q[r][c] = r == c ? 1.0 : 0.0;
#pragma unroll
  for (int k = nW - 1; k >= 0; --k)
#pragma unroll
    for (int c = 0; c < nW; ++c) {
      double dotv = 0.0;
#pragma unroll
      for (int r = 0; r < 2 * m; ++r) dotv = fma(V[k][r], Q[r][c], dotv);
#pragma unroll
      for (int r = 0; r < 2 * m; ++r) Q[r][c] = fma(-dotv, V[k][r], Q[r][c]);
    }
  // the reduced matrix [[0, R~], [R~^T, Cw]] (R~ = R beside a zero column for s) and its projection
  Sym<NM, double> M;
#pragma unroll
  for (int i = 0; i < nW; ++i)
#pragma unroll
    for (int j = i; j < nW; ++j) M(i, j) = 0.0;
#pragma unroll
  for (int i = 0; i < nW; ++i)
#pragma unroll
    for (int c = 0; c < m; ++c) M(i, nW + c) = c < m - nW ? 0.0 : R[i][c - (m - nW)];
#pragma unroll
  for (int c = 0; c < m; ++c)
#pragma unroll
    for (int d = c; d < m; ++d) M(nW + c, nW + d) = Cw[c][d];
  psd_small<NM>(M);
  // back to frame coordinates: P'_SS = Q P11 Q^T, P'_SN = Q P12 Wb^T, P'_NN = Wb P22 Wb^T
  double QP11[2 * m][nW], PSN[2 * m][m], PNN[m][m];
#pragma unroll
  for (int r = 0; r < 2 * m; ++r) {
#pragma unroll
    for (int c = 0; c < nW; ++c) {
      double a1 = 0.0;
#pragma unroll
      for (int k = 0; k < nW; ++k) a1 = fma(Q[r][k], M(k, c), a1);
      QP11[r][c] = a1;
    }
    double qp12[m];
#pragma unroll
    for (int c = 0; c < m; ++c) {
      double a2 = 0.0;
#pragma unroll
      for (int k = 0; k < nW; ++k) a2 = fma(Q[r][k], M(k, nW + c), a2);
      qp12[c] = a2;
    }
#pragma unroll
    for (int j = 0; j < m; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < m; ++c) acc = fma(qp12[c], Wb[j][c], acc);
      PSN[r][j] = acc;
    }
  }
#pragma unroll
  for (int I = 0; I < m; ++I)
#pragma unroll
    for (int J = 0; J < m; ++J) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < m; ++c)
#pragma unroll
        for (int d = 0; d < m; ++d) acc = fma(Wb[I][c] * M(nW + c, nW + d), Wb[J][d], acc);
      PNN[I][J] = acc;
    }
#pragma unroll
  for (int I = 0; I < m; ++I)
#pragma unroll
    for (int J = I; J < m; ++J) {
      double P[3][3];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < nW; ++k) acc = fma(QP11[2 * I + a][k], Q[2 * J + b][k], acc);
          P[a][b] = acc;
        }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        P[a][2] = PSN[2 * I + a][J];
        P[2][a] = PSN[2 * J + a][I];
      }
      P[2][2] = PNN[I][J];
      block_from_frame<3 * m>(A, I, J, Fr, P);
    }
}

// PSD projection of the reduced Hessian A of a point-edge barrier (m slots as
// in project_plane).  Fr holds the orthonormal frame (e, nu, n): e along the
// edge, n normal to the plane of the point and the edge, nu = n x e.  The
// distance from the point to the edge's line does not change when any vertex
// moves along e (the point slides parallel to the line, an edge vertex along
// it), so the Hessian's (e, e) block vanishes; the reflection through the
// stencil's plane maps the stencil onto itself, so the n components decouple
// from the in-plane ones.  In frame coordinates the Hessian is therefore
// diag(M, Nn) with M = [[0, B], [B^T, C]] over the (e, nu) components and Nn
// over the n components: a 2m x 2m and an m x m eigenproblem in place of a
// 3m x 3m one (both in closed form for m = 1, the second for m = 2).  The
// computed (e, e) and cross blocks are zero up to rounding and are dropped.
template <int m>
YHD void project_line(Sym<3 * m, double>& A, const double (&Fr)[3][3]) {
  Sym<2 * m, double> M;
  Sym<m, double> Nn;
#pragma unroll
  for (int I = 0; I < m; ++I)
#pragma unroll
    for (int J = I; J < m; ++J) {
      double P[3][3];
      block_to_frame<3 * m>(A, I, J, Fr, P);
      M(I, J) = 0.0;
      M(I, m + J) = P[0][1];
      if (J > I) M(J, m + I) = P[1][0];
      M(m + I, m + J) = P[1][1];
      Nn(I, J) = P[2][2];
    }
  psd_small<2 * m>(M);
  if constexpr (m == 1)
    Nn(0, 0) = fmax(Nn(0, 0), 0.0);
  else
    psd_small<m>(Nn);
#pragma unroll
  for (int I = 0; I < m; ++I)
#pragma unroll
    for (int J = I; J < m; ++J) {
      double P[3][3];
      P[0][0] = M(I, J);
      P[0][1] = M(I, m + J);
      P[1][0] = M(J, m + I);
      P[1][1] = M(m + I, m + J);
      P[0][2] = P[1][2] = P[2][0] = P[2][1] = 0.0;
      P[2][2] = Nn(I, J);
      block_from_frame<3 * m>(A, I, J, Fr, P);
    }
}

// Maps a u-space gradient gu (3 NU) and Hessian Hu (3 NU x 3 NU, upper) of an
// energy of the difference variables u_U = sum_a TOPO::M(U, a) x_a to the
// stencil's K free vertices (fl[k] = local index of the k-th free vertex,
// increasing): grad_sink(k, g[3]) receives the gradient row of free vertex k,
// block_sink(I, J, B[3][3]) the upper block of free vertices I <= J (rows of
// vertex fl[I]).  Unless EXACT the Hessian is projected to the PSD cone: in the
// Helmert basis when every vertex is free (exact reduction, the energy is
// translation invariant), else on the free principal submatrix.
//
// SPLIT selects the structured projection of that reduced matrix in the frame
// *Fr: 1 = project_plane (point-triangle, edge-edge), 3 = project_plane with
// the triangle's uniform normal shift (free slots = the triangle's vertices),
// 2 = project_line (point-edge), 0 = a dense eigendecomposition.
template <class TOPO, int K, bool EXACT, int SPLIT = 0, class GS, class BS>
YHD void emit_reduced(const double (&gu)[3 * TOPO::NU], Sym<3 * TOPO::NU, double>& Hu, const int (&fl)[4],
                      GS&& grad_sink, BS&& block_sink, const double (*Fr)[3][3] = nullptr) {
  constexpr int NV = TOPO::NV, NU = TOPO::NU;
  // coefficients M[U][fl[k]] selected at run time from the compile-time table
  double Mf[NU][K];
#pragma unroll
  for (int U = 0; U < NU; ++U)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double m = 0.0;
#pragma unroll
      for (int q = 0; q < NV; ++q) m = (fl[k] == q) ? double(TOPO::M(U, q)) : m;
      Mf[U][k] = m;
    }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double g[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int U = 0; U < NU; ++U) acc = fma(Mf[U][k], gu[3 * U + i], acc);
      g[i] = acc;
    }
    grad_sink(k, g);
  }
  if constexpr (K == NV && !EXACT) {
    // all vertices free: project in the Helmert basis (translation-free subspace)
    constexpr int NR = NV - 1;
    double R[NU][NR];
#pragma unroll
    for (int U = 0; U < NU; ++U)
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < NV; ++q) acc += double(TOPO::M(U, q)) * helmert(q, j);
        R[U][j] = acc;
      }
    Sym<3 * NR, double> A;
#pragma unroll
    for (int I = 0; I < NR; ++I)
#pragma unroll
      for (int J = I; J < NR; ++J)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            if (I == J && l < i) continue;
            double acc = 0.0;
#pragma unroll
            for (int U = 0; U < NU; ++U)
#pragma unroll
              for (int W = 0; W < NU; ++W) acc = fma(R[U][I] * R[W][J], Hu(3 * U + i, 3 * W + l), acc);
            A(3 * I + i, 3 * J + l) = acc;
          }
    if constexpr (SPLIT == 1)
      project_plane<NR>(A, *Fr);
    else if constexpr (SPLIT == 2)
      project_line<NR>(A, *Fr);
    else
      psd_project<3 * NR, double>(A);
#pragma unroll
    for (int p = 0; p < NV; ++p)
#pragma unroll
      for (int q = p; q < NV; ++q) {
        double B[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            double acc = 0.0;
#pragma unroll
            for (int I = 0; I < NR; ++I)
#pragma unroll
              for (int J = 0; J < NR; ++J) acc = fma(helmert(p, I) * helmert(q, J), A(3 * I + i, 3 * J + l), acc);
            B[i][l] = acc;
          }
        if (p == q) {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int l = i + 1; l < 3; ++l) {
              const double m = 0.5 * (B[i][l] + B[l][i]);
              B[i][l] = m;
              B[l][i] = m;
            }
        }
        block_sink(p, q, B);
      }
  } else {
    // free principal submatrix: block (I, J) = sum_UW M[U][fl_I] M[W][fl_J] H_u(U, W)
    Sym<3 * K, double> A;
#pragma unroll
    for (int I = 0; I < K; ++I)
#pragma unroll
      for (int J = I; J < K; ++J)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            if (I == J && l < i) continue;
            double acc = 0.0;
#pragma unroll
            for (int U = 0; U < NU; ++U)
#pragma unroll
              for (int W = 0; W < NU; ++W) acc = fma(Mf[U][I] * Mf[W][J], Hu(3 * U + i, 3 * W + l), acc);
            A(3 * I + i, 3 * J + l) = acc;
          }
    if constexpr (!EXACT) {
      if constexpr (SPLIT == 1)
        project_plane<K>(A, *Fr);
      else if constexpr (SPLIT == 3)
        project_plane<K, true>(A, *Fr);
      else if constexpr (SPLIT == 2)
        project_line<K>(A, *Fr);
      else
        psd_project<3 * K, double>(A);
    }
#pragma unroll
    for (int I = 0; I < K; ++I)
#pragma unroll
      for (int J = I; J < K; ++J) {
        double B[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int l = 0; l < 3; ++l) B[i][l] = A(3 * I + i, 3 * J + l);
        block_sink(I, J, B);
      }
  }
}

// Edge-edge mollifier of near-parallel edges (IPC, Li et al. 2020): with
// c = |e1 x e2|^2 and a threshold eps (eps_x = 1e-3 |e1_rest|^2 |e2_rest|^2),
// m(c) = (c / eps)(2 - c / eps) below eps and 1 above; the barrier of the
// stencil is m(c) b(d).  m is C^1 at eps (m' = 2 (1 - c / eps) / eps vanishes
// there).  eps <= 0 means no mollifier.  u = (w, e1, e2) of an EE stencil.
YHD double ee_mollifier(const double (&u)[3][3], double eps) {
  if (!(eps > 0.0)) return 1.0;
  double n[3];
  cross(u[1], u[2], n);
  const double r = dot(n, n) / eps;
  return r < 1.0 ? r * (2.0 - r) : 1.0;
}

// Energy, free-vertex gradient rows and free-vertex upper Hessian blocks of one
// contact stencil with K free vertices (sinks as in emit_reduced).  Returns
// false when an input is not finite.  d receives the squared distance;
// e = kappa b(d) (0 when d >= dhat or d <= 0), times the mollifier m(c) for
// an edge-edge stencil with eps > 0 (ee_mollifier).  The projection is the
// structured one of the stencil's type (project_plane, project_line, the
// point-point closed form), except for a mollified edge-edge stencil: the
// mollifier varies with the edges' in-plane directions, so that Hessian takes
// the dense eigendecomposition.  TRI_FREE: a point-triangle stencil whose free
// vertices are exactly the triangle's (fl = 1, 2, 3; the point fixed), which
// takes project_plane's uniform-shift reduction.
template <int TYPE, int K, bool EXACT, bool TRI_FREE = false, class GS, class BS>
YHD bool contact_stencil(const double (&xv)[4][3], const int (&fl)[4], double kappa, double dhat, int classic,
                         double& e, double& d, double& side, GS&& grad_sink, BS&& block_sink, double eps = 0.0) {
  constexpr int NU = Topo<TYPE>::NU;
  double u[NU][3];
  const bool ok = diff_vars<TYPE>(xv, u);
  Dist<TYPE> D;
  distance<TYPE>(u, D, side);
  d = D.d;
  const bool active = D.d > 0.0 && D.d < dhat;
  double b0 = 0.0, b1 = 0.0, b2 = 0.0;
  if (active) barrier(D.d, dhat, classic, b0, b1, b2);
  e = kappa * b0;
  const double kb1 = kappa * b1, kb2 = kappa * b2;
  // u-space barrier gradient and Hessian (zero when inactive)
  double gu[3 * NU];
  bool mollified = false;
  if constexpr (TYPE == 1) {
    if (active && eps > 0.0) {
      // m(c) b(d): gradient m b' grad d + b grad m, Hessian
      // m (b'' grad d grad d^T + b' hess d) + b' (grad d grad m^T + grad m grad d^T) + b hess m,
      // grad m = m' grad c, hess m = m'' grad c grad c^T + m' hess c (c = N of the distance)
      const double *e1 = u[1], *e2 = u[2];
      double n[3], e2n[3], ne1[3];
      cross(e1, e2, n);
      const double N = dot(n, n);
      if (N < eps) {
        mollified = true;
        cross(e2, n, e2n);
        cross(n, e1, ne1);
        double dN[9];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          dN[i] = 0.0;
          dN[3 + i] = 2.0 * e2n[i];
          dN[6 + i] = 2.0 * ne1[i];
        }
        const double r = N / eps, m = r * (2.0 - r), m1 = 2.0 * (1.0 - r) / eps, m2 = -2.0 / (eps * eps);
        e = kappa * m * b0;
        const double km = kappa * m, kb0 = kappa * b0;
#pragma unroll
        for (int q = 0; q < 9; ++q) gu[q] = fma(km * b1, D.g[q], kb0 * m1 * dN[q]);
#pragma unroll
        for (int q = 0; q < 9; ++q)
#pragma unroll
          for (int c = q; c < 9; ++c) {
            const int B1 = q / 3, B2 = c / 3, i = q % 3, l = c % 3;
            const double hN = (B1 == 0 || B2 == 0) ? 0.0 : crossnorm_hess(e1, e2, n, B1 - 1, B2 - 1, i, l);
            const double hb = fma(kb2 * D.g[q], D.g[c], kb1 * D.H(q, c));
            const double cross_t = kb1 * m1 * (D.g[q] * dN[c] + dN[q] * D.g[c]);
            const double hm = kb0 * (m2 * dN[q] * dN[c] + m1 * hN);
            D.H(q, c) = m * hb + cross_t + hm;
          }
      }
    }
  }
  if (!mollified) {
#pragma unroll
    for (int r = 0; r < 3 * NU; ++r) gu[r] = kb1 * D.g[r];
#pragma unroll
    for (int r = 0; r < 3 * NU; ++r)
#pragma unroll
      for (int c = r; c < 3 * NU; ++c) D.H(r, c) = fma(kb2 * D.g[r], D.g[c], kb1 * D.H(r, c));
  }
  if constexpr ((TYPE == 0 || TYPE == 1 || TYPE == 2) && !EXACT) {
    // point-triangle / edge-edge: t along e1, n along e1 x e2;
    // point-edge (u = (a, b)): t along the edge b - a, n along a x b
    double t[3], n[3], Fr[3][3];
    if constexpr (TYPE == 2) {
#pragma unroll
      for (int i = 0; i < 3; ++i) t[i] = u[1][i] - u[0][i];
      cross(u[0], u[1], n);
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) t[i] = u[1][i];
      cross(u[1], u[2], n);
    }
    orthonormal_frame(t, n, Fr);
    if (TYPE == 1 && mollified)
      emit_reduced<Topo<TYPE>, K, EXACT>(gu, D.H, fl, grad_sink, block_sink);
    else
      emit_reduced<Topo<TYPE>, K, EXACT, TYPE == 2 ? 2 : (TRI_FREE && TYPE == 0 && K == 3 ? 3 : 1)>(
          gu, D.H, fl, grad_sink, block_sink, &Fr);
  } else if constexpr (TYPE == 3 && !EXACT) {
    // point-point in closed form: with u = q - p and d = |u|^2 the u-space
    // Hessian kappa (b'' grad d grad d^T + b' hess d) = 4 kappa b'' u u^T + 2 kappa b' I
    // has the eigenvalue 4 kappa b'' d + 2 kappa b' along u and 2 kappa b' twice
    // across it; clamping them projects it, and the x-space Hessian (u-space
    // block times [[1, -1], [-1, 1]], or the block itself with one vertex
    // free) is then already positive semi-definite
    const double la = fma(4.0 * kb2, D.d, 2.0 * kb1), lp = 2.0 * kb1;
    const double pa = la > 0.0 ? la : 0.0, pp = lp > 0.0 ? lp : 0.0;
    const double c = D.d > 0.0 ? (pa - pp) / D.d : 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = r; q < 3; ++q) D.H(r, q) = (r == q ? pp : 0.0) + c * u[0][r] * u[0][q];
    emit_reduced<Topo<TYPE>, K, true>(gu, D.H, fl, grad_sink, block_sink);
  } else {
    emit_reduced<Topo<TYPE>, K, EXACT>(gu, D.H, fl, grad_sink, block_sink);
  }
  return ok;
}

}  // namespace cmath
}  // namespace yasps
