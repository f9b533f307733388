// Closed-form eigensystem of the stable Neo-Hookean F-space Hessian.
//
// Psi(F) = V [f(I_C) + g(J)] with f(I) = mu/2 (I - 3) - mu/2 log(I + 1) and
// g(J) = lam/2 (J - alpha)^2 (Eq. snh), so
//   d2Psi/dF2 = V [2 f' I9 + 4 f'' vec F vec F^T + g'' vec cofF vec cofF^T + g' H_J].
// With the rotation-variant SVD F = U diag(s) V^T (U, V rotations, s_2 may be
// negative) the matrix is block diagonal in the basis vec(U M V^T):
//  * for each pair i < j (k the third index), the "twist" M = (E_ij - E_ji)/sqrt2
//    and "flip" M = (E_ij + E_ji)/sqrt2 have eigenvalues
//    V (2 f' + g' s_k) and V (2 f' - g' s_k)  (det(S + d) contains -s_k d_ij d_ji);
//  * the diagonal modes M = diag(e) span a 3x3 block
//    A_ij = 2 f' d_ij + 4 f'' s_i s_j + g'' c_i c_j + g' (i != j) s_k,
//    c_i = prod_{m != i} s_m, whose eigenvectors e are found numerically.
// The projection (negative eigenvalues clamped to zero, section
// "Eigendecomposition (EVD) and PSD Projection") is then the sum of the
// kept rank-one terms.  This replaces a 9x9 iterative eigensolve by a 3x3 one
// plus a 3x3 SVD (the paper lists closed-form eigensystems as the second way to
// cut projection cost).
#pragma once

#include "eigen.h"

namespace yasps {
namespace snh {

template <class R>
YHD void cross(const R a[3], const R b[3], R c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi: A = Q diag(w) Q^T.
template <class R>
YHD void eig3(Sym<3, R> A, R w[3], R (&Q)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Q[i][j] = (i == j) ? R(1) : R(0);
  R norm2 = R(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) norm2 = fmaR(A(i, j), A(i, j), norm2);
  const R tol = (sizeof(R) == 8 ? R(1e-32) : R(1e-14)) * norm2;
  for (int sweep = 0; sweep < 12; ++sweep) {
    if (!(off_diagonal2<3, R>(A) > tol)) break;
    JacobiSweep<3, 0, 1, R>::run(A, Q);
  }
  w[0] = A(0, 0);
  w[1] = A(1, 1);
  w[2] = A(2, 2);
}

// Rotation-variant SVD F = U diag(s) V^T with det U = det V = +1.
template <class R>
YHD void svd3(const R F[3][3], R (&U)[3][3], R s[3], R (&V)[3][3]) {
  Sym<3, R> S;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      R acc = R(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) acc = fmaR(F[k][i], F[k][j], acc);
      S(i, j) = acc;
    }
  R w[3];
  eig3<R>(S, w, V);
  // right-handed V
  R c01[3];
  const R v0[3] = {V[0][0], V[1][0], V[2][0]}, v1[3] = {V[0][1], V[1][1], V[2][1]};
  cross(v0, v1, c01);
  if (c01[0] * V[0][2] + c01[1] * V[1][2] + c01[2] * V[2][2] < R(0)) {
#pragma unroll
    for (int i = 0; i < 3; ++i) V[i][2] = -V[i][2];
  }
  // b_i = F v_i (= s_i u_i)
  R b[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < 3; ++i) b[c][i] = F[i][0] * V[0][c] + F[i][1] * V[1][c] + F[i][2] * V[2][c];
  // order the columns by decreasing singular value: a, m, z
  int a = 0, m = 1, z = 2;
  if (w[m] > w[a]) { int t = a; a = m; m = t; }
  if (w[z] > w[a]) { int t = a; a = z; z = t; }
  if (w[z] > w[m]) { int t = m; m = z; z = t; }
  R ua[3], um[3], uz[3];
  {
    R ba[3], bm[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ba[i] = a == 0 ? b[0][i] : (a == 1 ? b[1][i] : b[2][i]);
      bm[i] = m == 0 ? b[0][i] : (m == 1 ? b[1][i] : b[2][i]);
    }
    R na = sqrtR(ba[0] * ba[0] + ba[1] * ba[1] + ba[2] * ba[2]);
    if (!(na > R(0))) {  // F = 0: any rotation
      ba[0] = R(1); ba[1] = R(0); ba[2] = R(0);
      na = R(1);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) ua[i] = ba[i] / na;
    const R pr = ua[0] * bm[0] + ua[1] * bm[1] + ua[2] * bm[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) bm[i] -= pr * ua[i];
    R nm = sqrtR(bm[0] * bm[0] + bm[1] * bm[1] + bm[2] * bm[2]);
    if (!(nm > R(1e-30) * na)) {  // rank one: any unit vector orthogonal to ua
      const R e[3] = {fabsR(ua[0]) < R(0.6) ? R(1) : R(0), fabsR(ua[0]) < R(0.6) ? R(0) : R(1), R(0)};
      cross(ua, e, bm);
      nm = sqrtR(bm[0] * bm[0] + bm[1] * bm[1] + bm[2] * bm[2]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) um[i] = bm[i] / nm;
  }
  // third column completes a rotation: (a, m, z) cyclic -> uz = ua x um, else um x ua
  const bool cyclic = (a == 0 && m == 1) || (a == 1 && m == 2) || (a == 2 && m == 0);
  if (cyclic)
    cross(ua, um, uz);
  else
    cross(um, ua, uz);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    U[i][a] = ua[i];
    U[i][m] = um[i];
    U[i][z] = uz[i];
  }
  // s_i = u_i . F v_i (signed: negative for an inverted element)
#pragma unroll
  for (int c = 0; c < 3; ++c) s[c] = U[0][c] * b[c][0] + U[1][c] * b[c][1] + U[2][c] * b[c][2];
}

// Accumulates P += lam_plus vec(Q) vec(Q)^T, vec column-major (entry (i,j) at i + 3j).
template <class R>
YHD void add_mode(Sym<9, R>& P, R lam, const R (&Q)[3][3]) {
  if (!(lam > R(0))) return;
  R q[9];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i + 3 * j] = Q[i][j];
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int c = r; c < 9; ++c) P(r, c) = fmaR(lam * q[r], q[c], P(r, c));
}

// P = Proj(d2Psi/dF2) for Psi = vol * [f(I_C) + g(J)] (stable Neo-Hookean).
template <class R>
YHD void projected_hessian(const R F[3][3], R mu, R lam, R vol, Sym<9, R>& P) {
  R U[3][3], V[3][3], s[3];
  svd3<R>(F, U, s, V);
  const R Ic = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
  const R J = s[0] * s[1] * s[2];
  const R alpha = R(1) + R(3) * mu / (R(4) * lam);
  const R ic1 = R(1) / (Ic + R(1));
  const R f1x2 = mu * (R(1) - ic1);  // 2 f'
  const R f2x4 = R(2) * mu * ic1 * ic1;  // 4 f''
  const R g1 = lam * (J - alpha);         // g'
  const R g2 = lam;                       // g''
#pragma unroll
  for (int k = 0; k < Sym<9, R>::SIZE; ++k) P.v[k] = R(0);
  const R rs2 = R(0.70710678118654752440);
  // twist and flip modes of the pairs (i, j), k the third index
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i + 1; j < 3; ++j) {
      const int k = 3 - i - j;
      const R lt = vol * (f1x2 + g1 * s[k]);
      const R lf = vol * (f1x2 - g1 * s[k]);
      R Qt[3][3], Qf[3][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const R a = U[r][i] * V[c][j], b = U[r][j] * V[c][i];
          Qt[r][c] = rs2 * (a - b);
          Qf[r][c] = rs2 * (a + b);
        }
      add_mode<R>(P, lt, Qt);
      add_mode<R>(P, lf, Qf);
    }
  // scaling modes
  const R c[3] = {s[1] * s[2], s[0] * s[2], s[0] * s[1]};
  Sym<3, R> A;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) A(i, j) = f2x4 * s[i] * s[j] + g2 * c[i] * c[j] + (i == j ? f1x2 : g1 * s[3 - i - j]);
  R w[3], E[3][3];
  eig3<R>(A, w, E);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    R Q[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        Q[r][cc] = U[r][0] * E[0][m] * V[cc][0] + U[r][1] * E[1][m] * V[cc][1] + U[r][2] * E[2][m] * V[cc][2];
    add_mode<R>(P, vol * w[m], Q);
  }
}

}  // namespace snh
}  // namespace yasps
