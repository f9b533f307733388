// PSD projection of small symmetric matrices, one matrix per GPU thread.
//
// The paper makes every local Hessian positive semi-definite by an explicit
// eigendecomposition followed by clamping the negative eigenvalues to zero
// (section "Eigendecomposition (EVD) and PSD Projection"); it runs a library
// eigensolver per GPU thread.  Here the eigensolver is a cyclic two-sided
// Jacobi iteration (Golub & Van Loan, "Matrix Computations", the symmetric
// Schur rotation and the cyclic-by-row sweep), fully unrolled for a
// compile-time size N so the matrix and its eigenvectors stay in registers.
// Jacobi computes small and large eigenvalues to high relative accuracy, so
// the clamp decides the same eigenvalues as a dense LAPACK solver up to the
// rounding of values that are zero to working precision.
#pragma once

#include "common.h"

namespace yasps {

// One Jacobi rotation zeroing A(p, q); V accumulates the rotations (A = V L V^T).
template <int N, int P, int Q, class R>
YHD void jacobi_rotate(Sym<N, R>& A, R (&V)[N][N]) {
  const R apq = A(P, Q);
  const R app = A(P, P);
  const R aqq = A(Q, Q);
  // Branch-free: the divisions always run (with a harmless denominator when
  // apq = 0) and a select discards them, so no values stay live across
  // divergent control flow (which multiplied the register footprint).
  const bool zero = (apq == R(0));
  const R theta = (aqq - app) / (zero ? R(1) : R(2) * apq);
  const R sgn = theta >= R(0) ? R(1) : R(-1);
  // t = tan of the rotation angle, the smaller root of t^2 + 2 theta t - 1 = 0
  const R tr = sgn / (fabsR(theta) + sqrtR(fmaR(theta, theta, R(1))));
  const R t = zero ? R(0) : tr;
  const R c = R(1) / sqrtR(fmaR(t, t, R(1)));
  const R s = t * c;
  A(P, P) = fmaR(-t, apq, app);
  A(Q, Q) = fmaR(t, apq, aqq);
  A(P, Q) = R(0);
#pragma unroll
  for (int r = 0; r < N; ++r) {
    if (r == P || r == Q) continue;
    const R g = A(r, P), h = A(r, Q);
    A(r, P) = fmaR(c, g, -s * h);
    A(r, Q) = fmaR(s, g, c * h);
  }
#pragma unroll
  for (int r = 0; r < N; ++r) {
    const R g = V[r][P], h = V[r][Q];
    V[r][P] = fmaR(c, g, -s * h);
    V[r][Q] = fmaR(s, g, c * h);
  }
}

template <int N, int P, int Q, class R>
struct JacobiSweep {
  static YHD void run(Sym<N, R>& A, R (&V)[N][N]) {
    jacobi_rotate<N, P, Q, R>(A, V);
    if constexpr (Q + 1 < N) {
      JacobiSweep<N, P, Q + 1, R>::run(A, V);
    } else if constexpr (P + 2 < N) {
      JacobiSweep<N, P + 1, P + 2, R>::run(A, V);
    }
  }
};

template <int N, class R>
YHD R off_diagonal2(const Sym<N, R>& A) {
  R off = R(0);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i + 1; j < N; ++j) off = fmaR(A(i, j), A(i, j), off);
  return off;
}

// Replaces A by Proj(A) = Q max(Lambda, 0) Q^T in place.
template <int N, class R>
YHD void psd_project(Sym<N, R>& A) {
  if constexpr (N == 1) {
    A(0, 0) = fmaxR(A(0, 0), R(0));
  } else {
    R V[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) V[i][j] = (i == j) ? R(1) : R(0);
    R norm2 = R(0);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i; j < N; ++j) norm2 = fmaR(A(i, j), A(i, j), norm2);
    // stop once the off-diagonal part is below the rounding of the data
    const R tol = (sizeof(R) == 8 ? R(1e-32) : R(1e-14)) * norm2;
    for (int sweep = 0; sweep < 16; ++sweep) {
      if (!(off_diagonal2<N, R>(A) > tol)) break;
      JacobiSweep<N, 0, 1, R>::run(A, V);
    }
    R lam[N];
#pragma unroll
    for (int k = 0; k < N; ++k) lam[k] = fmaxR(A(k, k), R(0));
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i; j < N; ++j) {
        R acc = R(0);
#pragma unroll
        for (int k = 0; k < N; ++k) acc = fmaR(V[i][k] * lam[k], V[j][k], acc);
        A(i, j) = acc;
      }
  }
}

}  // namespace yasps
