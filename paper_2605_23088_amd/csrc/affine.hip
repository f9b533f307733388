// Affine bodies mixed with free vertices (the paper's alternative
// parameterisation of positions, sections "UNION" and "Differentiation of
// Unioned Attributes").
//
// A body vertex sits at p = A r + t = r_1 a_1 + r_2 a_2 + r_3 a_3 + t, linear
// in the body's four rows of degrees of freedom (a_j the columns of A).
//
// Bodies.  Per body, one thread: the inertia 1/2 sum_ab M4_ab (q_a - q~_a) .
// (q_b - q~_b) (M4 = sum_v m_v w_v w_v^T, w = (r, 1); static problems take the
// gravity potential -g . sum_v m_v p_v = -g . (sum_j M4_3j a_j + M4_33 t)
// instead), and the orthogonality energy E = h^2 k 1/2 |G|^2, G = A^T A - I:
//   dE/da_j = h^2 k 2 sum_l G_jl a_l,
//   d2E/da_j da_l = h^2 k 2 [delta_jl A A^T + a_l a_j^T + G_jl I],
// its 9x9 Hessian projected to the PSD cone unless exact.
//
// Body contacts.  Pass 1 (one thread per stencil) forms the vertex positions
// from the union of free, fixed and body vertices and evaluates the barrier
// with the contact arithmetic of contact_math.h, treating every free or body
// vertex as movable: the projection acts on the Hessian over the movable
// positions (Helmert-reduced when all are movable), which is the
// reduced-coordinate projection of section "Eigendecomposition (EVD) and PSD
// Projection" since positions are linear in the degrees of freedom.  Pass 2
// maps the position-space gradient rows and blocks to the stencil's row list
// with the weights of the union (1 for a free vertex; r_1, r_2, r_3, 1 for a
// body vertex): block (alpha, beta) = sum_IJ w_I(alpha) w_J(beta) H_IJ.
#include "blockreduce.h"
#include "contact_math.h"
#include "eigen.h"
#include "kernels.h"

namespace yasps {

namespace {

using namespace cmath;

// ---------------------------------------------------------------- bodies

template <bool EXACT, bool ENERGY_ONLY>
__global__ __launch_bounds__(EVAL_BLOCK) void body_kernel(BodyArgs a) {
  __shared__ double lds[EVAL_BLOCK];
  const int b = blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e_in = 0.0, e_or = 0.0;
  if (b < a.nb) {
    const double* q = a.x + 3 * ((size_t)a.nv + 4 * (size_t)b);
    double Q[4][3];
    bool ok = true;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        Q[r][i] = q[3 * r + i];
        ok = ok && finite(Q[r][i]);
      }
    double M[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) M[r][c] = a.M4[16 * (size_t)b + 4 * r + c];
    // inertia (or the gravity potential) and its gradient rows
    double g[4][3];
    if (a.is_static) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          g[r][i] = -M[3][r] * a.g[i];
          e_in = fma(g[r][i], Q[r][i], e_in);
        }
    } else {
      const double* qt = a.x_tilde + 3 * ((size_t)a.nv + 4 * (size_t)b);
      double D[4][3];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int i = 0; i < 3; ++i) D[r][i] = Q[r][i] - qt[3 * r + i];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          double acc = 0.0;
#pragma unroll
          for (int c = 0; c < 4; ++c) acc = fma(M[r][c], D[c][i], acc);
          g[r][i] = acc;
          e_in = fma(0.5 * D[r][i], acc, e_in);
        }
    }
    // orthogonality: G = A^T A - I with A's columns the rows a_j
    const double hk = a.h2 * a.k[b];
    double G[3][3], AAt[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        G[j][l] = Q[j][0] * Q[l][0] + Q[j][1] * Q[l][1] + Q[j][2] * Q[l][2] - (j == l ? 1.0 : 0.0);
        AAt[j][l] = Q[0][j] * Q[0][l] + Q[1][j] * Q[1][l] + Q[2][j] * Q[2][l];
      }
    double gg = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int l = 0; l < 3; ++l) gg = fma(G[j][l], G[j][l], gg);
    e_or = 0.5 * hk * gg;
    if (!ok || !finite(e_in) || !finite(e_or)) atomicOr(a.flags, FLAG_NONFINITE);
    if constexpr (!ENERGY_ONLY) {
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          double acc = 0.0;
#pragma unroll
          for (int l = 0; l < 3; ++l) acc = fma(G[j][l], Q[l][i], acc);
          g[j][i] = fma(2.0 * hk, acc, g[j][i]);
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double* dst = a.grd + 3 * (size_t)a.gpos[r * a.nb + b];
#pragma unroll
        for (int i = 0; i < 3; ++i) dst[i] = g[r][i];
      }
      // 9x9 orthogonality Hessian over (a_1, a_2, a_3): row (j, i), column (l, m)
      Sym<9, double> H;
#pragma unroll
      for (int r = 0; r < 9; ++r)
#pragma unroll
        for (int c = r; c < 9; ++c) {
          const int j = r / 3, i = r % 3, l = c / 3, m = c % 3;
          double h = Q[l][i] * Q[j][m] + (i == m ? G[j][l] : 0.0) + (j == l ? AAt[i][m] : 0.0);
          H(r, c) = 2.0 * hk * h;
        }
      if (!EXACT) psd_project<9, double>(H);
      // the 10 upper blocks over the rows (a_1, a_2, a_3, t): inertia M4 I3 plus orthogonality
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = r; c < 4; ++c) {
          const int qi = r * 4 - (r * (r - 1)) / 2 + (c - r);
          const double mi = a.is_static ? 0.0 : M[r][c];
          double B[3][3];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int m = 0; m < 3; ++m) B[i][m] = (i == m ? mi : 0.0) + (c < 3 ? H(3 * r + i, 3 * c + m) : 0.0);
          const size_t pos = 9 * (size_t)a.spos[qi * a.nb + b];
          if (a.blk32) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int m = 0; m < 3; ++m) a.blk32[pos + 3 * i + m] = float(B[i][m]);
          } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int m = 0; m < 3; ++m) a.blk[pos + 3 * i + m] = B[i][m];
          }
        }
    }
  }
  const double si = block_sum<EVAL_BLOCK>(e_in, lds);
  const double so = block_sum<EVAL_BLOCK>(e_or, lds);
  if (threadIdx.x == 0) {
    a.e_inertia[blockIdx.x] = si;
    a.e_orth[blockIdx.x] = so;
  }
}

// ---------------------------------------------------------------- body contacts

// Position of vertex v from the union; movable = free or body vertex.
YDEV void union_position(const BodyContactArgs& a, int v, double p[3], bool& movable) {
  const int base = a.nv + a.nfix;
  if (v < a.nv) {
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = a.x[3 * (size_t)v + i];
    movable = true;
  } else if (v < base) {
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = a.x_fixed[3 * (size_t)(v - a.nv) + i];
    movable = false;
  } else {
    const int k = v - base;
    const double* r = a.body_rest + 3 * (size_t)k;
    const double* q = a.x + 3 * ((size_t)a.nv + 4 * (size_t)a.body_of[k]);
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = fma(r[0], q[i], fma(r[1], q[3 + i], fma(r[2], q[6 + i], q[9 + i])));
    movable = true;
  }
}

template <int TYPE, int K, bool EXACT>
__global__ __launch_bounds__(EVAL_BLOCK) void body_contact_kernel(BodyContactArgs a) {
  constexpr int NV = Topo<TYPE>::NV;
  __shared__ double lds[EVAL_BLOCK];
  const int s = a.begin + blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0, dmin = __builtin_inf(), nact = 0.0;
  if (s < a.end) {
    const int ns = a.ns;
    double xv[4][3] = {};
    int fl[4] = {0, 0, 0, 0};  // local index of the j-th movable vertex (static indexing only)
    int nf = 0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      bool mv;
      union_position(a, a.idx[k * ns + s], xv[k], mv);
#pragma unroll
      for (int j = 0; j < 4; ++j) fl[j] = (mv && nf == j) ? k : fl[j];
      nf += mv ? 1 : 0;
    }
    double d, side;
    double* pg = a.pos_grd + 12 * (size_t)s;
    double* pb = a.pos_blk + 90 * (size_t)s;
    auto gsink = [&](int k, const double (&g)[3]) {
#pragma unroll
      for (int i = 0; i < 3; ++i) pg[3 * k + i] = g[i];
    };
    auto bsink = [&](int I, int J, const double (&B)[3][3]) {
      double* dst = pb + 9 * pair_index(I, J, 4);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int l = 0; l < 3; ++l) dst[3 * i + l] = B[i][l];
    };
    const double eps = (TYPE == 1 && a.eps) ? a.eps[s] : 0.0;
    const bool ok =
        contact_stencil<TYPE, K, EXACT>(xv, fl, a.kappa, a.dhat, a.barrier, e, d, side, gsink, bsink, eps);
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

// Pass 2 over all body contacts: the row-list gradient and blocks.
__global__ __launch_bounds__(EVAL_BLOCK) void body_map_kernel(BodyContactArgs a) {
  const int s = blockIdx.x * EVAL_BLOCK + threadIdx.x;
  if (s >= a.ns) return;
  const int ns = a.ns, base = a.nv + a.nfix;
  // movable vertices in vertex order: first list position, row count, weights
  int p0[4], cnt[4], K = 0;
  double w[4][4];
  for (int k = 0; k < 4; ++k) {
    const int v = a.idx[k * ns + s];
    const int vp = a.vpos[k * ns + s];
    if (v < 0 || vp < 0) continue;
    p0[K] = vp;
    if (v < a.nv) {
      cnt[K] = 1;
      w[K][0] = 1.0;
    } else {
      const double* r = a.body_rest + 3 * (size_t)(v - base);
      cnt[K] = 4;
      w[K][0] = r[0];
      w[K][1] = r[1];
      w[K][2] = r[2];
      w[K][3] = 1.0;
    }
    ++K;
  }
  int L = 0;
  int rows[8];
  for (int j = 0; j < 8; ++j) {
    rows[j] = a.rows[j * ns + s];
    L += rows[j] >= 0 ? 1 : 0;
  }
  const double* pg = a.pos_grd + 12 * (size_t)s;
  const double* pb = a.pos_blk + 90 * (size_t)s;
  auto weight = [&](int I, int alpha) { return alpha >= p0[I] && alpha < p0[I] + cnt[I] ? w[I][alpha - p0[I]] : 0.0; };
  for (int al = 0; al < L; ++al) {
    double g[3] = {0.0, 0.0, 0.0};
    for (int I = 0; I < K; ++I) {
      const double wi = weight(I, al);
      if (wi == 0.0) continue;
      for (int i = 0; i < 3; ++i) g[i] = fma(wi, pg[3 * I + i], g[i]);
    }
    double* dst = a.grd + 3 * (size_t)a.gpos[al * ns + s];
    for (int i = 0; i < 3; ++i) dst[i] = g[i];
  }
  int q = 0;
  for (int al = 0; al < L; ++al)
    for (int be = al; be < L; ++be, ++q) {
      double B[3][3] = {};
      for (int I = 0; I < K; ++I) {
        const double wi = weight(I, al);
        if (wi == 0.0) continue;
        for (int J = 0; J < K; ++J) {
          const double wj = weight(J, be);
          if (wj == 0.0) continue;
          const double ww = wi * wj;
          const double* H = pb + 9 * pair_index(I < J ? I : J, I < J ? J : I, 4);
          const bool tr = I > J;
          for (int i = 0; i < 3; ++i)
            for (int l = 0; l < 3; ++l) B[i][l] = fma(ww, tr ? H[3 * l + i] : H[3 * i + l], B[i][l]);
        }
      }
      const bool flip = rows[al] > rows[be];
      const size_t pos = 9 * (size_t)a.spos[q * ns + s];
      if (a.blk32) {
        for (int i = 0; i < 3; ++i)
          for (int l = 0; l < 3; ++l) a.blk32[pos + 3 * i + l] = float(flip ? B[l][i] : B[i][l]);
      } else {
        for (int i = 0; i < 3; ++i)
          for (int l = 0; l < 3; ++l) a.blk[pos + 3 * i + l] = flip ? B[l][i] : B[i][l];
      }
    }
}

// Line-search trial: energy, and feasibility (d > 0; PT / EE keep their side
// relative to the positions at x0).
template <int TYPE>
__global__ __launch_bounds__(EVAL_BLOCK) void body_contact_energy_kernel(BodyContactArgs a, const double* x0,
                                                                         double* bad_part) {
  constexpr int NV = Topo<TYPE>::NV, NU = Topo<TYPE>::NU;
  __shared__ double lds[EVAL_BLOCK];
  const int s = a.begin + blockIdx.x * EVAL_BLOCK + threadIdx.x;
  double e = 0.0, bad = 0.0;
  if (s < a.end) {
    const int ns = a.ns;
    BodyContactArgs a0 = a;
    a0.x = x0;
    double xv[4][3] = {}, xo[4][3] = {};
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int v = a.idx[k * ns + s];
      bool mv;
      union_position(a, v, xv[k], mv);
      union_position(a0, v, xo[k], mv);
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

template <int TYPE, int K>
void launch_bk(const BodyContactArgs& a, bool exact, hipStream_t s) {
  const int grid = (a.end - a.begin + EVAL_BLOCK - 1) / EVAL_BLOCK;
  if (exact)
    hipLaunchKernelGGL((body_contact_kernel<TYPE, K, true>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL((body_contact_kernel<TYPE, K, false>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
}

}  // namespace

void launch_body_eval(const BodyArgs& a, bool exact, hipStream_t s) {
  if (a.nb == 0) return;
  const int grid = (a.nb + EVAL_BLOCK - 1) / EVAL_BLOCK;
  if (exact)
    hipLaunchKernelGGL((body_kernel<true, false>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL((body_kernel<false, false>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a);
}

void launch_body_energy(const BodyArgs& a, hipStream_t s) {
  if (a.nb == 0) return;
  hipLaunchKernelGGL((body_kernel<false, true>), dim3((a.nb + EVAL_BLOCK - 1) / EVAL_BLOCK), dim3(EVAL_BLOCK), 0, s,
                     a);
}

// Pass 1 of one group; the caller launches body_map over all stencils after
// the last group (nmov = -1).
void launch_body_contact_eval(int type, int nmov, const BodyContactArgs& a, bool exact, hipStream_t s) {
  if (nmov < 0) {
    if (a.ns > 0)
      hipLaunchKernelGGL(body_map_kernel, dim3((a.ns + EVAL_BLOCK - 1) / EVAL_BLOCK), dim3(EVAL_BLOCK), 0, s, a);
    return;
  }
  if (a.end <= a.begin) return;
  switch (type * 8 + nmov) {
    case 0 * 8 + 1: launch_bk<0, 1>(a, exact, s); break;
    case 0 * 8 + 2: launch_bk<0, 2>(a, exact, s); break;
    case 0 * 8 + 3: launch_bk<0, 3>(a, exact, s); break;
    case 0 * 8 + 4: launch_bk<0, 4>(a, exact, s); break;
    case 1 * 8 + 1: launch_bk<1, 1>(a, exact, s); break;
    case 1 * 8 + 2: launch_bk<1, 2>(a, exact, s); break;
    case 1 * 8 + 3: launch_bk<1, 3>(a, exact, s); break;
    case 1 * 8 + 4: launch_bk<1, 4>(a, exact, s); break;
    case 2 * 8 + 1: launch_bk<2, 1>(a, exact, s); break;
    case 2 * 8 + 2: launch_bk<2, 2>(a, exact, s); break;
    case 2 * 8 + 3: launch_bk<2, 3>(a, exact, s); break;
    case 3 * 8 + 1: launch_bk<3, 1>(a, exact, s); break;
    case 3 * 8 + 2: launch_bk<3, 2>(a, exact, s); break;
    default: break;
  }
}

void launch_body_contact_energy(int type, const BodyContactArgs& a, const double* x0, double* bad_part,
                                hipStream_t s) {
  if (a.end <= a.begin) return;
  const int grid = (a.end - a.begin + EVAL_BLOCK - 1) / EVAL_BLOCK;
  switch (type) {
    case 0: hipLaunchKernelGGL((body_contact_energy_kernel<0>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a, x0, bad_part); break;
    case 1: hipLaunchKernelGGL((body_contact_energy_kernel<1>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a, x0, bad_part); break;
    case 2: hipLaunchKernelGGL((body_contact_energy_kernel<2>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a, x0, bad_part); break;
    default: hipLaunchKernelGGL((body_contact_energy_kernel<3>), dim3(grid), dim3(EVAL_BLOCK), 0, s, a, x0, bad_part); break;
  }
}

}  // namespace yasps
