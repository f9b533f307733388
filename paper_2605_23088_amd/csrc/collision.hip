// Proximity search, the contact energy of the pairs found, and continuous
// collision detection, for time stepping with contact.
//
// The paper leaves collision detection and CCD to an external module
// (section "Limitations"; its examples use GIPC's, timed as "CCD+CD+
// LargestStep").  The definitions here are Incremental Potential Contact's:
// every point-triangle and edge-edge pair of the collision surface (no shared
// vertex, at least one free or affine-body vertex, not all of one body)
// closer than sqrt(dhat) contributes one
// barrier stencil, typed by where its closest points lie (point-triangle: face
// / edge / vertex -> PT / PE / PP; edge-edge: interiors / one endpoint / two
// endpoints -> EE / PE / PP), found with the textbook closest-feature
// constructions (Ericson, Real-Time Collision Detection, sections 5.1.5 and
// 5.1.9).  The step bound is additive CCD (Li, Kaufman, Jiang 2021,
// "Codimensional Incremental Potential Contact").
//
// Broad phase: a uniform grid.  The primitives of one side (triangles, or
// edges) are registered in every cell their box inflated by R covers, over
// the box of cells the registered boxes span: counted per cell, scanned and
// placed when that box holds at most 2^22 cells, else radix-sorted by cell
// index; every (query primitive, registered entry) of the cells a query's
// own box covers is listed (count, scan, fill), and one thread per listed
// pair runs the tests: a pair is a candidate when the
// primitives' boxes, each inflated by r, overlap (the exact test); R = 2r (1 +
// 1e-9) makes the grid a superset of that, and a pair is taken only in the
// cell that holds the low corner of the two grid boxes' intersection, so each
// pair is tested once.  Swept boxes (over x and x + t p) serve the CCD.
//
// Floating point: this file is compiled without contraction into fused
// multiply-adds (pragma below), so every quantity that decides a type, a
// candidate or a CCD step is computed by the same operations, in the same
// order, as the textbook definitions written out plainly; the results do
// not depend on the launch shape.  Output order is fixed: point-triangle
// pairs by (point, triangle), then edge-edge pairs by (edge, edge): the
// listing order, each query's candidates being sorted by primitive.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdlib>

#include "blockreduce.h"
#include "contact_math.h"
#include "devsort.h"
#include "kernels.h"

namespace yasps {

namespace {

using devsort::DI_BLOCK;
constexpr int CD_BLOCK = 256;
constexpr long long CELL_OFF = 1ll << 20;  // cell coordinates in [-2^20, 2^20)
constexpr int ACCD_MAX_STEPS = 10000;
constexpr long long MAX_BOX_CELLS = 1 << 16;  // a box over more cells (a non-finite position, or a cell size
                                              // far below the motion) is an error, so every loop is bounded
constexpr long long DENSE_MAX_CELLS = 1 << 22;  // registrations over more grid cells sort their entries instead

YHD void sub3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[0] - b[0];
  c[1] = a[1] - b[1];
  c[2] = a[2] - b[2];
}
YHD double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
YHD double dist2(const double a[3], const double b[3]) {
  double d[3];
  sub3(a, b, d);
  return dot3(d, d);
}
YHD double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

// Closest feature of triangle (a, b, c) to p: kind 0 face, 1 edge (l0, l1),
// 2 vertex (l0); squared distance.
YHD double point_triangle(const double p[3], const double a[3], const double b[3], const double c[3], int& kind,
                          int& l0, int& l1) {
  double ab[3], ac[3], ap[3], bp[3], cp[3], q[3];
  sub3(b, a, ab);
  sub3(c, a, ac);
  sub3(p, a, ap);
  const double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  l1 = -1;
  if (d1 <= 0.0 && d2 <= 0.0) {
    kind = 2;
    l0 = 0;
    return dist2(p, a);
  }
  sub3(p, b, bp);
  const double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) {
    kind = 2;
    l0 = 1;
    return dist2(p, b);
  }
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
    const double v = d1 / (d1 - d3);
    for (int k = 0; k < 3; ++k) q[k] = a[k] + v * ab[k];
    kind = 1;
    l0 = 0;
    l1 = 1;
    return dist2(p, q);
  }
  sub3(p, c, cp);
  const double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) {
    kind = 2;
    l0 = 2;
    return dist2(p, c);
  }
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
    const double w = d2 / (d2 - d6);
    for (int k = 0; k < 3; ++k) q[k] = a[k] + w * ac[k];
    kind = 1;
    l0 = 0;
    l1 = 2;
    return dist2(p, q);
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    double bc[3];
    sub3(c, b, bc);
    for (int k = 0; k < 3; ++k) q[k] = b[k] + w * bc[k];
    kind = 1;
    l0 = 1;
    l1 = 2;
    return dist2(p, q);
  }
  const double den = 1.0 / (va + vb + vc);
  const double v = vb * den, w = vc * den;
  for (int k = 0; k < 3; ++k) q[k] = a[k] + ab[k] * v + ac[k] * w;
  kind = 0;
  l0 = 0;
  return dist2(p, q);
}

// Closest points of segments p1q1, p2q2: parameters s, t in [0, 1]; squared distance.
YHD double segment_segment(const double p1[3], const double q1[3], const double p2[3], const double q2[3],
                           double& s, double& t) {
  double d1[3], d2[3], r[3];
  sub3(q1, p1, d1);
  sub3(q2, p2, d2);
  sub3(p1, p2, r);
  const double a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
  const double c = dot3(d1, r), b = dot3(d1, d2);
  const double den = a * e - b * b;
  s = den != 0.0 ? clamp01((b * f - c * e) / den) : 0.0;
  t = (b * s + f) / e;
  if (t < 0.0) {
    t = 0.0;
    s = clamp01(-c / a);
  } else if (t > 1.0) {
    t = 1.0;
    s = clamp01((b - c) / a);
  }
  double c1[3], c2[3];
  for (int k = 0; k < 3; ++k) {
    c1[k] = p1[k] + d1[k] * s;
    c2[k] = p2[k] + d2[k] * t;
  }
  return dist2(c1, c2);
}

// An affine body's vertex from its body's rows q = (a_1, a_2, a_3, t):
// r_1 a_1 + r_2 a_2 + r_3 a_3 + t, summed left to right.
YDEV void body_point(const CdPositions& X, int k, const double* rows, double q[3]) {
  const double* r = X.body_rest + 3 * (size_t)k;
  const double* a = rows + 3 * ((size_t)X.nv + 4 * (size_t)X.body_of[k]);
  for (int i = 0; i < 3; ++i) q[i] = r[0] * a[i] + r[1] * a[3 + i] + r[2] * a[6 + i] + a[9 + i];
}
YDEV void vpos(const CdPositions& X, int v, double q[3]) {
  if (v >= X.nv + X.nfix) {
    body_point(X, v - X.nv - X.nfix, X.x, q);
    return;
  }
  const double* s = v < X.nv ? X.x + 3 * (size_t)v : X.xf + 3 * (size_t)(v - X.nv);
  q[0] = s[0];
  q[1] = s[1];
  q[2] = s[2];
}
YDEV bool movable(const CdPositions& X, int v) { return v < X.nv || v >= X.nv + X.nfix; }
YDEV int body_id(const CdPositions& X, int v) { return v >= X.nv + X.nfix ? X.body_of[v - X.nv - X.nfix] : -1; }
// The vertex's displacement under the row motion p (0 for fixed; for a body
// vertex the same affine map of the body's row motion, which is linear).
YDEV void vmove(const CdPositions& X, int v, double d[3]) {
  if (X.p && v >= X.nv + X.nfix) {
    body_point(X, v - X.nv - X.nfix, X.p, d);
  } else if (X.p && v < X.nv) {
    const double* s = X.p + 3 * (size_t)v;
    d[0] = s[0];
    d[1] = s[1];
    d[2] = s[2];
  } else {
    d[0] = d[1] = d[2] = 0.0;
  }
}

// Box of a primitive inflated by r (over x, and x + t p when X.p is set).
template <int K>
YDEV void pbox(const CdPositions& X, const int (&ids)[K], double r, double lo[3], double hi[3]) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = __builtin_inf();
    hi[k] = -__builtin_inf();
  }
  for (int a = 0; a < K; ++a) {
    double q[3];
    vpos(X, ids[a], q);
    for (int k = 0; k < 3; ++k) {
      lo[k] = fmin(lo[k], q[k]);
      hi[k] = fmax(hi[k], q[k]);
    }
    if (X.p) {
      double d[3];
      vmove(X, ids[a], d);
      for (int k = 0; k < 3; ++k) {
        const double e = q[k] + X.t * d[k];
        lo[k] = fmin(lo[k], e);
        hi[k] = fmax(hi[k], e);
      }
    }
  }
  for (int k = 0; k < 3; ++k) {
    lo[k] = lo[k] - r;
    hi[k] = hi[k] + r;
  }
}

YDEV long long cell_of(double v, double cell) {
  double f = floor(v / cell);
  if (!(f == f)) f = 0.0;  // NaN: any cell (the box is rejected by its cell count or its exact test)
  const long long c = f < -(double)CELL_OFF ? -CELL_OFF : (f >= (double)(CELL_OFF - 1) ? CELL_OFF - 1 : (long long)f);
  return c + CELL_OFF;
}
// Grid cells of one registration: the box of cells the registered boxes
// cover (lowest coordinate and span per axis), a cell's index within it
// x-major.
struct CellGrid {
  int base[3];
  long long span[3];
};
YDEV bool cell_in(const CellGrid& G, long long ix, long long iy, long long iz) {
  const long long d[3] = {ix - G.base[0], iy - G.base[1], iz - G.base[2]};
  bool in = true;
  for (int k = 0; k < 3; ++k) in = in && d[k] >= 0 && d[k] < G.span[k];
  return in;
}
YDEV uint64_t cell_index(const CellGrid& G, long long ix, long long iy, long long iz) {
  return ((uint64_t)(ix - G.base[0]) * (uint64_t)G.span[1] + (uint64_t)(iy - G.base[1])) * (uint64_t)G.span[2] +
         (uint64_t)(iz - G.base[2]);
}
YDEV void cell_coords(const CellGrid& G, uint64_t c, long long& ix, long long& iy, long long& iz) {
  iz = (long long)(c % (uint64_t)G.span[2]) + G.base[2];
  const uint64_t r = c / (uint64_t)G.span[2];
  iy = (long long)(r % (uint64_t)G.span[1]) + G.base[1];
  ix = (long long)(r / (uint64_t)G.span[1]) + G.base[0];
}

template <int K>
YDEV void load_ids(const int32_t* prims, int m, int j, int (&ids)[K]) {
  for (int a = 0; a < K; ++a) ids[a] = prims[(size_t)a * m + j];
}

// Cells covered by a box; 0 (and the error flag) when more than MAX_BOX_CELLS.
YDEV long long box_cells(const double lo[3], const double hi[3], double cell, int* err) {
  long long c = 1;
  for (int k = 0; k < 3; ++k) {
    const long long w = cell_of(hi[k], cell) - cell_of(lo[k], cell) + 1;
    if (w < 1 || w > MAX_BOX_CELLS) {
      atomicOr(err, 1);
      return 0;
    }
    c *= w;
  }
  if (c > MAX_BOX_CELLS) {
    atomicOr(err, 1);
    return 0;
  }
  return c;
}

// Cells per registered box, and the range of cells they cover (range[0..2]
// lowest, range[3..5] highest coordinate per axis), reduced over the
// workgroup first (one atomic per workgroup and value).
template <int K>
__global__ void reg_count_kernel(int m, const int32_t* prims, CdPositions X, double R, double cell, int32_t* cnt,
                                 int* err, int* range) {
  const int j = blockIdx.x * DI_BLOCK + threadIdx.x;
  int r[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
  if (j < m) {
    int ids[K];
    load_ids<K>(prims, m, j, ids);
    double lo[3], hi[3];
    pbox<K>(X, ids, R, lo, hi);
    const long long c = box_cells(lo, hi, cell, err);
    cnt[j] = (int32_t)c;
    if (c)
      for (int k = 0; k < 3; ++k) {
        r[k] = (int)cell_of(lo[k], cell);
        r[3 + k] = (int)cell_of(hi[k], cell);
      }
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 3; ++k) {
      r[k] = min(r[k], __shfl_xor(r[k], o));
      r[3 + k] = max(r[3 + k], __shfl_xor(r[3 + k], o));
    }
  __shared__ int wr[DI_BLOCK / 64][6];
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 6; ++k) wr[threadIdx.x >> 6][k] = r[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < DI_BLOCK / 64; ++w)
      for (int k = 0; k < 3; ++k) {
        r[k] = min(r[k], wr[w][k]);
        r[3 + k] = max(r[3 + k], wr[w][3 + k]);
      }
    if (r[0] != INT_MAX)
      for (int k = 0; k < 3; ++k) {
        atomicMin(&range[k], r[k]);
        atomicMax(&range[3 + k], r[3 + k]);
      }
  }
}

template <int K>
__global__ void reg_fill_kernel(int m, const int32_t* prims, CdPositions X, double R, double cell, CellGrid G,
                                const int32_t* off, uint64_t* keys, int32_t* vals, int* err) {
  const int j = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (j >= m) return;
  int ids[K];
  load_ids<K>(prims, m, j, ids);
  double lo[3], hi[3];
  pbox<K>(X, ids, R, lo, hi);
  if (box_cells(lo, hi, cell, err) == 0) return;  // counted as 0
  long long l[3], h[3];
  for (int k = 0; k < 3; ++k) {
    l[k] = cell_of(lo[k], cell);
    h[k] = cell_of(hi[k], cell);
  }
  int o = off[j];
  for (long long z = l[2]; z <= h[2]; ++z)
    for (long long y = l[1]; y <= h[1]; ++y)
      for (long long x = l[0]; x <= h[0]; ++x) {
        keys[o] = cell_index(G, x, y, z);
        vals[o] = j;
        ++o;
      }
}

// Dense registration (the grid's cells counted directly): pass 1 counts the
// entries of every cell, pass 2 places them (in any order inside a cell;
// cell_sort_kernel orders them).  A team of REG_TEAM lanes takes one
// primitive and shares out the cells of its box (x fastest), so the atomics
// of one box are issued side by side instead of one after another.
constexpr int REG_TEAM = 8;
template <int K, bool PLACE>
__global__ void reg_dense_kernel(int m, const int32_t* prims, CdPositions X, double R, double cell, CellGrid G,
                                 int32_t* count, int32_t* cursor, uint64_t* keys, int32_t* vals, int* err) {
  const long long g = (long long)blockIdx.x * DI_BLOCK + threadIdx.x;
  const int j = (int)(g / REG_TEAM), t = (int)(g % REG_TEAM);
  if (j >= m) return;
  int ids[K];
  load_ids<K>(prims, m, j, ids);
  double lo[3], hi[3];
  pbox<K>(X, ids, R, lo, hi);
  const long long total = box_cells(lo, hi, cell, err);
  if (total == 0) return;
  long long l[3], w[3];
  for (int k = 0; k < 3; ++k) {
    l[k] = cell_of(lo[k], cell);
    w[k] = cell_of(hi[k], cell) - l[k] + 1;
  }
  for (long long q = t; q < total; q += REG_TEAM) {
    const long long x = l[0] + q % w[0], r = q / w[0];
    const long long y = l[1] + r % w[1], z = l[2] + r / w[1];
    const uint64_t c = cell_index(G, x, y, z);
    if constexpr (PLACE) {
      const int o = atomicAdd(&cursor[c], 1);
      keys[o] = c;
      vals[o] = j;
    } else {
      atomicAdd(&count[c], 1);
    }
  }
}

// The edge-edge outputs in (edge, partner) order: out[k] = in[perm[k]].
__global__ void gather_kernel(int m, const int32_t* __restrict__ perm, const int32_t* __restrict__ ti,
                              const int32_t* __restrict__ ii, int istride, const double* __restrict__ ei,
                              int32_t* __restrict__ to, int32_t* __restrict__ io, int ostride,
                              double* __restrict__ eo) {
  const int k = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (k >= m) return;
  const int s = perm[k];
  to[k] = ti[s];
  eo[k] = ei[s];
  for (int a = 0; a < 4; ++a) io[(size_t)a * ostride + k] = ii[(size_t)a * istride + s];
}

__global__ void iota32_kernel(int m, int32_t* v) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i < m) v[i] = i;
}

// The entries of every cell in primitive order.  A cell holds the few
// primitives whose boxes reach it (each once; about 20 on the surfaces here).
// A thread loads its cell's entries into registers (all loads issued at once,
// empty slots padded with INT_MAX), sorts them with a bitonic network of N
// inputs, N the wavefront's largest cell rounded up to 8, 16, 32 or 64 (one
// network per wavefront, all compare-exchanges fixed at compile time), and
// writes them back in order.  A cell of more than 64 entries is
// insertion-sorted in place by its thread.
static_assert(DI_BLOCK % 64 == 0, "cell_sort_kernel: whole wavefronts");
template <int N>
YDEV void network_sort(int32_t* __restrict__ p, int k) {
  int v[N];
#pragma unroll
  for (int a = 0; a < N; ++a) v[a] = a < k ? p[a] : INT_MAX;
#pragma unroll
  for (int m = 2; m <= N; m <<= 1)
#pragma unroll
    for (int j = m >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const int a = v[i], b = v[l];
          const bool up = (i & m) == 0;
          v[i] = up ? min(a, b) : max(a, b);
          v[l] = up ? max(a, b) : min(a, b);
        }
      }
#pragma unroll
  for (int a = 0; a < N; ++a)
    if (a < k) p[a] = v[a];
}
__global__ __launch_bounds__(DI_BLOCK) void cell_sort_kernel(long long ncell, const int32_t* __restrict__ cstart, int32_t* __restrict__ vals) {
  const long long c = (long long)blockIdx.x * DI_BLOCK + threadIdx.x;
  const bool in = c < ncell;
  const int e0 = in ? cstart[c] : 0;
  const int k = in ? cstart[c + 1] - e0 : 0;
  int kmax = k;
  for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
  if (kmax <= 1) return;  // uniform
  int32_t* p = vals + e0;
  if (kmax <= 8) {
    network_sort<8>(p, k);
  } else if (kmax <= 16) {
    network_sort<16>(p, k);
  } else if (kmax <= 32) {
    network_sort<32>(p, k);
  } else if (k <= 64) {
    network_sort<64>(p, k);
  } else {
    for (int a = 1; a < k; ++a) {
      const int v = p[a];
      int b = a - 1;
      while (b >= 0 && p[b] > v) {
        p[b + 1] = p[b];
        --b;
      }
      p[b + 1] = v;
    }
  }
}

YDEV int lower_bound(const uint64_t* keys, int n, uint64_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Squared distance of a point-triangle (x4 = p, a, b, c) or edge-edge pair.
template <bool EEP>
YDEV double pair_d2(const double (&x4)[4][3]) {
  if constexpr (EEP) {
    double s, t;
    return segment_segment(x4[0], x4[1], x4[2], x4[3], s, t);
  } else {
    int kind, l0, l1;
    return point_triangle(x4[0], x4[1], x4[2], x4[3], kind, l0, l1);
  }
}

// Additive CCD of one pair along x + t p, t <= t_c.
template <bool EEP>
YDEV double accd(const double (&x4in)[4][3], const double (&p4)[4][3], double s, double t_c) {
  double pm[3], pr[4][3], nrm[4], x4[4][3];
  for (int k = 0; k < 3; ++k) pm[k] = (((0.0 + p4[0][k]) + p4[1][k]) + p4[2][k] + p4[3][k]) / 4.0;
  for (int a = 0; a < 4; ++a) {
    sub3(p4[a], pm, pr[a]);
    nrm[a] = sqrt(dot3(pr[a], pr[a]));
    for (int k = 0; k < 3; ++k) x4[a][k] = x4in[a][k];
  }
  const double lp = EEP ? fmax(nrm[0], nrm[1]) + fmax(nrm[2], nrm[3]) : nrm[0] + fmax(fmax(nrm[1], nrm[2]), nrm[3]);
  if (lp == 0.0) return t_c;
  double d = sqrt(pair_d2<EEP>(x4));
  if (d == 0.0) return 0.0;
  const double g = s * d;
  double t = 0.0, tl = (1.0 - s) * d / lp;
  for (int it = 0; it < ACCD_MAX_STEPS; ++it) {
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k) x4[a][k] = x4[a][k] + tl * pr[a][k];
    d = sqrt(pair_d2<EEP>(x4));
    if (t > 0.0 && d < g) return t;
    t = t + tl;
    if (t > t_c) return t_c;
    tl = 0.9 * d / lp;
  }
  return t;
}

// Type-fixed squared distance of a stencil (the closed forms of the stencil
// kernels, written plainly) and its barrier energy.
YDEV double stencil_energy(int type, const double (&x4)[4][3], double eps, double kappa, double dhat, int classic) {
  double d, m = 1.0;
  if (type == 0 || type == 1) {
    double e1[3], e2[3], n[3], w[3];
    if (type == 0) {
      sub3(x4[2], x4[1], e1);
      sub3(x4[3], x4[1], e2);
      sub3(x4[0], x4[1], w);
    } else {
      sub3(x4[1], x4[0], e1);
      sub3(x4[3], x4[2], e2);
      sub3(x4[0], x4[2], w);
    }
    cmath::cross(e1, e2, n);
    const double s = dot3(w, n), N = dot3(n, n);
    d = s * s / N;
    if (type == 1 && eps > 0.0) {
      const double r = N / eps;
      m = r < 1.0 ? r * (2.0 - r) : 1.0;
    }
  } else if (type == 2) {
    double a[3], b[3], c[3], e[3];
    sub3(x4[1], x4[0], a);
    sub3(x4[2], x4[0], b);
    cmath::cross(a, b, c);
    sub3(x4[2], x4[1], e);
    d = dot3(c, c) / dot3(e, e);
  } else {
    d = dist2(x4[0], x4[1]);
  }
  if (!(d > 0.0) || !(d < dhat)) return 0.0;
  double b0, b1, b2;
  cmath::barrier(d, dhat, classic, b0, b1, b2);
  return m < 1.0 ? kappa * m * b0 : kappa * b0;
}

struct QueryArgs {
  int ma;                // query primitives
  const int32_t* pa;     // [KA][ma]
  int mb;                // registered primitives
  const int32_t* pb;     // [KB][mb]
  bool ee;               // edge-edge: the same set on both sides, pairs i < j
  CdPositions X;
  double r, R, cell;
  int nreg;
  const uint64_t* keys;  // cell of every registered entry (entries grouped by cell, cells ascending)
  const int32_t* vals;   // their primitive ids
  CellGrid grid;         // the registration's cells
  const int32_t* cstart; // [cells + 1] first entry of every cell (dense registration), else null
  const double* len2;    // squared rest lengths of the edges (EE mollifier) or null
  double dhat, kappa;
  int classic;
  double s_ccd, t_max;
  // candidates: every (query, registered entry) of the cells a query's box covers
  int32_t* ccnt;         // [ma] candidates per query
  const int32_t* coff;   // [ma + 1] their offsets
  int ncand;
  int32_t* cq;           // [ncand] query of each candidate
  int32_t* ce;           // [ncand] registered entry (index into keys / vals)
  int32_t* hit;          // [ncand] 1 if the candidate gives a stencil (count pass)
  const int32_t* hoff;   // [ncand + 1] output position of each hit (fill pass)
  int out0;              // first output of this query set
  uint64_t* okey;        // edge-edge outputs: (edge, partner) sort key, edge << kbits | partner
  int kbits;             // bits of an edge index
  int cap;               // stride of the output idx array
  int32_t* otype;
  int32_t* oidx;         // [4][cap]
  double* oeps;
  double* part;          // per-workgroup energy sums / CCD minima
  int* err;              // set when a box spans too many cells
};

enum { Q_COUNT, Q_FILL, Q_ENERGY, Q_CCD };

// The stencil of a candidate pair at positions X (type < 0: none).
template <bool EEP>
YDEV int narrow(const QueryArgs& q, int i, int j, const int* ia, const int* ib, int (&ids)[4], double& eps) {
  double P[4][3];
  eps = 0.0;
  ids[0] = ids[1] = ids[2] = ids[3] = -1;
  if constexpr (!EEP) {
    vpos(q.X, ia[0], P[0]);
    for (int a = 0; a < 3; ++a) vpos(q.X, ib[a], P[1 + a]);
    int kind, l0, l1;
    const double d2 = point_triangle(P[0], P[1], P[2], P[3], kind, l0, l1);
    if (!(d2 < q.dhat)) return -1;
    ids[0] = ia[0];
    if (kind == 0) {
      ids[1] = ib[0];
      ids[2] = ib[1];
      ids[3] = ib[2];
      return 0;
    }
    if (kind == 1) {
      ids[1] = ib[l0];
      ids[2] = ib[l1];
      return 2;
    }
    ids[1] = ib[l0];
    return 3;
  } else {
    for (int a = 0; a < 2; ++a) {
      vpos(q.X, ia[a], P[a]);
      vpos(q.X, ib[a], P[2 + a]);
    }
    double s, t;
    const double d2 = segment_segment(P[0], P[1], P[2], P[3], s, t);
    if (!(d2 < q.dhat)) return -1;
    const int sa = s == 0.0 ? 0 : (s == 1.0 ? 1 : -1);
    const int tb = t == 0.0 ? 0 : (t == 1.0 ? 1 : -1);
    if (sa < 0 && tb < 0) {
      ids[0] = ia[0];
      ids[1] = ia[1];
      ids[2] = ib[0];
      ids[3] = ib[1];
      if (q.len2) eps = 1e-3 * q.len2[i] * q.len2[j];
      return 1;
    }
    if (sa >= 0 && tb < 0) {
      ids[0] = ia[sa];
      ids[1] = ib[0];
      ids[2] = ib[1];
      return 2;
    }
    if (sa < 0 && tb >= 0) {
      ids[0] = ib[tb];
      ids[1] = ia[0];
      ids[2] = ia[1];
      return 2;
    }
    ids[0] = ia[sa];
    ids[1] = ib[tb];
    return 3;
  }
}

// The cell range of a query primitive's own box (none when it spans too many cells).
template <int KA>
YDEV bool query_cells(const QueryArgs& q, int i, int (&ia)[KA], double (&lo0)[3], long long (&cl)[3],
                      long long (&ch)[3]) {
  load_ids<KA>(q.pa, q.ma, i, ia);
  double hi0[3];
  pbox<KA>(q.X, ia, 0.0, lo0, hi0);
  for (int k = 0; k < 3; ++k) {
    cl[k] = cell_of(lo0[k], q.cell);
    ch[k] = cell_of(hi0[k], q.cell);
  }
  return box_cells(lo0, hi0, q.cell, q.err) != 0;
}

// Pass 1 (WRITE = false): candidates per query, the registered entries of the
// cells its box covers; pass 2 (WRITE = true): the (query, entry) list, query
// by query, cells in (z, y, x) order, entries in primitive order.  In pass 2 a
// team of CAND_TEAM lanes takes one query: the lanes walk its cells together
// and share out each cell's entries, every entry going to the same position
// as in a walk by one thread.
constexpr int CAND_TEAM = 8;
template <int KA, bool WRITE>
__global__ __launch_bounds__(CD_BLOCK) void cand_kernel(QueryArgs q) {
  constexpr int T = WRITE ? CAND_TEAM : 1;
  const long long g = (long long)blockIdx.x * CD_BLOCK + threadIdx.x;
  const int i = (int)(g / T), t = (int)(g % T);
  if (i >= q.ma) return;
  int ia[KA];
  double lo0[3];
  long long cl[3], ch[3];
  int c = 0;
  if (query_cells<KA>(q, i, ia, lo0, cl, ch)) {
    int o = WRITE ? q.coff[i] : 0;
    for (long long z = cl[2]; z <= ch[2]; ++z)
      for (long long y = cl[1]; y <= ch[1]; ++y)
        for (long long x = cl[0]; x <= ch[0]; ++x) {
          if (!cell_in(q.grid, x, y, z)) continue;  // no registered entry there
          const uint64_t key = cell_index(q.grid, x, y, z);
          int e0, e1;
          if (q.cstart) {
            e0 = q.cstart[key];
            e1 = q.cstart[key + 1];
          } else {
            e0 = lower_bound(q.keys, q.nreg, key);
            e1 = e0;
            while (e1 < q.nreg && q.keys[e1] == key) ++e1;
          }
          if constexpr (WRITE) {
            for (int e = e0 + t; e < e1; e += T) {
              q.cq[o + (e - e0)] = i;
              q.ce[o + (e - e0)] = e;
            }
            o += e1 - e0;
          }
          c += e1 - e0;
        }
  }
  if constexpr (!WRITE) q.ccnt[i] = c;
}

// One candidate per thread: the exact candidate test, the owner-cell test,
// the shared-vertex and fixed-pair filters, then per MODE the narrow phase
// (hit flag, stencil output, barrier energy) or additive CCD.
template <int KA, int KB, int MODE>
__global__ __launch_bounds__(CD_BLOCK) void pair_kernel(QueryArgs q) {
  constexpr bool EEP = KA == 2;
  __shared__ double lds[CD_BLOCK];
  const int t = blockIdx.x * CD_BLOCK + threadIdx.x;
  double acc = 0.0, tmin = q.t_max;
  int hit = 0;
  if (t < q.ncand) {
    const int i = q.cq[t], e = q.ce[t];
    const int j = q.vals[e];
    long long x, y, z;
    cell_coords(q.grid, q.keys[e], x, y, z);
    bool take = !(q.ee && j <= i);
    int ia[KA], ib[KB];
    load_ids<KA>(q.pa, q.ma, i, ia);
    load_ids<KB>(q.pb, q.mb, j, ib);
    if (take) {
      // the exact candidate test: boxes inflated by r overlap
      double lor[3], hir[3], lob[3], hib[3];
      pbox<KA>(q.X, ia, q.r, lor, hir);
      pbox<KB>(q.X, ib, q.r, lob, hib);
      for (int k = 0; k < 3; ++k) take = take && lor[k] <= hib[k] && lob[k] <= hir[k];
    }
    if (take) {
      // taken only in the cell of the low corner of the grid boxes' intersection
      double lo0[3], hi0[3], loR[3], hiR[3];
      pbox<KA>(q.X, ia, 0.0, lo0, hi0);
      pbox<KB>(q.X, ib, q.R, loR, hiR);
      take = cell_of(fmax(lo0[0], loR[0]), q.cell) == x && cell_of(fmax(lo0[1], loR[1]), q.cell) == y &&
             cell_of(fmax(lo0[2], loR[2]), q.cell) == z;
    }
    if (take) {
      // no shared vertex, something movable (free or body vertices), and not
      // all the vertices of one affine body (its surface keeps its shape)
      bool shared = false, mov = false, one_body = true;
      const int b0 = body_id(q.X, ia[0]);
      for (int a = 0; a < KA; ++a) {
        mov |= movable(q.X, ia[a]);
        one_body &= b0 >= 0 && body_id(q.X, ia[a]) == b0;
        for (int b = 0; b < KB; ++b) shared |= ia[a] == ib[b];
      }
      for (int b = 0; b < KB; ++b) {
        mov |= movable(q.X, ib[b]);
        one_body &= b0 >= 0 && body_id(q.X, ib[b]) == b0;
      }
      take = !shared && mov && !one_body;
    }
    if (take) {
      if constexpr (MODE == Q_CCD) {
        double P4[4][3], D4[4][3];
        int v4[4];
        if constexpr (EEP) {
          v4[0] = ia[0], v4[1] = ia[1], v4[2] = ib[0], v4[3] = ib[1];
        } else {
          v4[0] = ia[0], v4[1] = ib[0], v4[2] = ib[1], v4[3] = ib[2];
        }
        for (int a = 0; a < 4; ++a) {
          vpos(q.X, v4[a], P4[a]);
          vmove(q.X, v4[a], D4[a]);
        }
        tmin = accd<EEP>(P4, D4, q.s_ccd, q.t_max);
      } else {
        int ids[4];
        double eps;
        const int type = narrow<EEP>(q, i, j, ia, ib, ids, eps);
        if (type >= 0) {
          hit = 1;
          if constexpr (MODE == Q_FILL) {
            const int o = q.out0 + q.hoff[t];
            q.otype[o] = type;
            for (int a = 0; a < 4; ++a) q.oidx[(size_t)a * q.cap + o] = ids[a];
            q.oeps[o] = eps;
            if (EEP) q.okey[q.hoff[t]] = ((uint64_t)i << q.kbits) | (uint64_t)j;
          } else if constexpr (MODE == Q_ENERGY) {
            double P4[4][3] = {};
            for (int a = 0; a < 4; ++a)
              if (ids[a] >= 0) vpos(q.X, ids[a], P4[a]);
            acc = stencil_energy(type, P4, eps, q.kappa, q.dhat, q.classic);
          }
        }
      }
    }
  }
  if constexpr (MODE == Q_COUNT) {
    if (t < q.ncand) q.hit[t] = hit;
  }
  if constexpr (MODE == Q_ENERGY) {
    const double es = block_sum<CD_BLOCK>(acc, lds);
    if (threadIdx.x == 0) q.part[blockIdx.x] = es;
  }
  if constexpr (MODE == Q_CCD) {
    const double tm = block_min<CD_BLOCK>(tmin, lds);
    if (threadIdx.x == 0) q.part[blockIdx.x] = tm;
  }
}

// part[0] = sum (kind 0) or min (kind 1) of part[0 .. m)
__global__ __launch_bounds__(CD_BLOCK) void fold_kernel(double* part, int m, int kind) {
  __shared__ double lds[CD_BLOCK];
  double v = kind ? __builtin_inf() : 0.0;
  for (int k = threadIdx.x; k < m; k += CD_BLOCK) v = kind ? fmin(v, part[k]) : v + part[k];
  const double r = kind ? block_min<CD_BLOCK>(v, lds) : block_sum<CD_BLOCK>(v, lds);
  if (threadIdx.x == 0) part[0] = r;
}

// x_tilde = x + h v + h^2 g over the rows: the free rows and each body's t
// row take gravity, the bodies' a rows none (the generalised gravity force of
// a body is M4 e_4 (x) g, so M4^-1 of it moves t only); and v = (x - x_start) / h.
__global__ void frame_tilde_kernel(int nv, int n3, const double* __restrict__ x, const double* __restrict__ v,
                                   double h, double g0, double g1, double g2, double* __restrict__ xt) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i >= n3) return;
  const int row = i / 3, c = i % 3;
  const bool grav = row < nv || (row - nv) % 4 == 3;
  const double g = grav ? (c == 0 ? g0 : (c == 1 ? g1 : g2)) : 0.0;
  xt[i] = x[i] + h * v[i] + h * h * g;
}
__global__ void frame_velocity_kernel(int n3, const double* __restrict__ x, const double* __restrict__ xs, double h,
                                      double* __restrict__ v) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i >= n3) return;
  v[i] = (x[i] - xs[i]) / h;
}

int grid_q(long long m) { return (int)((m + CD_BLOCK - 1) / CD_BLOCK); }

#define CD_CHECK(call)                  \
  do {                                  \
    if ((call) != hipSuccess) return -1; \
  } while (0)

// Registration of one side (triangles: K = 3, edges: K = 2): sorted cell keys.
struct Reg {
  int n = 0;
  uint64_t* keys = nullptr;
  int32_t* vals = nullptr;
  CellGrid grid{};
  int32_t* cstart = nullptr;
};

// Slots of the pinned read-back scratch: counts first, the error flag at
// PIN_ERR, a folded double at PIN_VAL, the two registrations' counts and
// ranges at PIN_REG_T and PIN_REG_E (8 each).
constexpr int PIN_ERR = 15, PIN_VAL = 16, PIN_REG_T = 24, PIN_REG_E = 32;

// Registration of one side in two phases, so that both sides share one host
// round trip: count_side queues the per-box cell counts, their scan and the
// cell range, read back into pin[0..7] (total, error flag, range); after the
// synchronisation place_side builds the grid registration.
struct RegCount {
  int m = 0;
  const int32_t* prims = nullptr;
  int32_t* off = nullptr;
  int* pin = nullptr;
};

template <int K>
int count_side(int m, const int32_t* prims, const CdPositions& X, double R, double cell, devsort::Temp& tmp,
               hipStream_t s, int* err, int* pin, RegCount& rc) {
  rc = RegCount{m, prims, nullptr, pin};
  if (m == 0) return 0;
  int32_t* cnt = tmp.get<int32_t>(m);
  rc.off = tmp.get<int32_t>(m + 1);
  int* range = tmp.get<int>(6);
  CD_CHECK(tmp.err);
  CD_CHECK(hipMemsetD32Async(range, INT_MAX, 3, s));
  CD_CHECK(hipMemsetD32Async(range + 3, INT_MIN, 3, s));
  hipLaunchKernelGGL(reg_count_kernel<K>, dim3(devsort::grid_of(m)), dim3(DI_BLOCK), 0, s, m, prims, X, R, cell,
                     cnt, err, range);
  CD_CHECK(devsort::prefix(tmp, cnt, rc.off, m, s));
  CD_CHECK(hipMemcpyAsync(&pin[0], rc.off + m, sizeof(int), hipMemcpyDeviceToHost, s));
  CD_CHECK(hipMemcpyAsync(&pin[1], err, sizeof(int), hipMemcpyDeviceToHost, s));
  CD_CHECK(hipMemcpyAsync(&pin[2], range, 6 * sizeof(int), hipMemcpyDeviceToHost, s));
  return 0;
}

template <int K>
int place_side(const RegCount& rc, const CdPositions& X, double R, double cell, const CdAlloc& alloc, int which,
               devsort::Temp& tmp, hipStream_t s, int* err, Reg& out) {
  out = Reg{};
  const int m = rc.m;
  if (m == 0) return 0;
  const int32_t* prims = rc.prims;
  const int* h = rc.pin;  // total, error flag, cell range
  const int* rg = rc.pin + 2;
  if (h[1]) return -2;
  const int total = h[0];
  if (total <= 0) return -2;
  CellGrid G{};
  double ncell = 1.0;
  for (int k = 0; k < 3; ++k) {
    G.base[k] = rg[k];
    G.span[k] = (long long)rg[3 + k] - rg[k] + 1;
    ncell *= (double)G.span[k];
  }
  uint64_t* ks = static_cast<uint64_t*>(alloc(which, sizeof(uint64_t) * (size_t)total));
  int32_t* vs = static_cast<int32_t*>(alloc(which + 1, sizeof(int32_t) * (size_t)total));
  if (!ks || !vs) return -1;
  long long dense_max = DENSE_MAX_CELLS;
  if (const char* ev = std::getenv("YASPS_GRID_DENSE_MAX")) dense_max = std::atoll(ev);  // test override
  if (ncell <= (double)dense_max) {
    // dense: count per cell, scan, place
    const long long nc = (long long)ncell;
    int32_t* count = tmp.get<int32_t>(nc);
    int32_t* cursor = tmp.get<int32_t>(nc + 1);
    CD_CHECK(tmp.err);
    int32_t* cs = static_cast<int32_t*>(alloc(which + 2, sizeof(int32_t) * (size_t)(nc + 1)));
    if (!cs) return -1;
    CD_CHECK(hipMemsetAsync(count, 0, sizeof(int32_t) * (size_t)nc, s));
    const dim3 teams(devsort::grid_of((long long)REG_TEAM * m));
    hipLaunchKernelGGL((reg_dense_kernel<K, false>), teams, dim3(DI_BLOCK), 0, s, m, prims, X, R, cell, G, count,
                       nullptr, nullptr, nullptr, err);
    CD_CHECK(devsort::prefix(tmp, count, cs, nc, s));
    CD_CHECK(hipMemcpyAsync(cursor, cs, sizeof(int32_t) * (size_t)(nc + 1), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL((reg_dense_kernel<K, true>), teams, dim3(DI_BLOCK), 0, s, m, prims, X, R, cell, G, nullptr,
                       cursor, ks, vs, err);
    hipLaunchKernelGGL(cell_sort_kernel, dim3(devsort::grid_of(nc)), dim3(DI_BLOCK), 0, s, nc, cs, vs);
    out.cstart = cs;
  } else {
    // sparse: keys per (primitive, cell), stably sorted by cell
    uint64_t* keys = tmp.get<uint64_t>(total);
    int32_t* vals = tmp.get<int32_t>(total);
    CD_CHECK(tmp.err);
    hipLaunchKernelGGL(reg_fill_kernel<K>, dim3(devsort::grid_of(m)), dim3(DI_BLOCK), 0, s, m, prims, X, R, cell, G,
                       rc.off, keys, vals, err);
    CD_CHECK(devsort::sort_pairs(tmp, keys, ks, vals, vs, total, devsort::bits_for((long long)(ncell - 1.0)), s));
  }
  out.grid = G;
  out.n = total;
  out.keys = ks;
  out.vals = vs;
  return 0;
}

QueryArgs query_args(const CdSurface& S, const CdPositions& X, bool ee, const Reg& reg, double r, double dhat,
                     int* err) {
  QueryArgs q{};
  q.err = err;
  q.ee = ee;
  q.ma = ee ? S.ne : S.np;
  q.pa = ee ? S.edges : S.points;
  q.mb = ee ? S.ne : S.nt;
  q.pb = ee ? S.edges : S.tris;
  q.X = X;
  q.r = r;
  q.R = 2.0 * r * (1.0 + 1e-9);
  q.cell = S.cell;
  q.nreg = reg.n;
  q.keys = reg.keys;
  q.vals = reg.vals;
  q.grid = reg.grid;
  q.cstart = reg.cstart;
  q.kbits = devsort::bits_for(std::max(S.ne, 1));
  q.len2 = S.len2;
  q.dhat = dhat;
  return q;
}

}  // namespace

void launch_frame_tilde(int nv, int n, const double* x, const double* v, double h, const double g[3], double* xt,
                        hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(frame_tilde_kernel, dim3(devsort::grid_of(3ll * n)), dim3(DI_BLOCK), 0, s, nv, 3 * n, x, v, h,
                     g[0], g[1], g[2], xt);
}

void launch_frame_velocity(int nv, const double* x, const double* xs, double h, double* v, hipStream_t s) {
  if (nv == 0) return;
  hipLaunchKernelGGL(frame_velocity_kernel, dim3(devsort::grid_of(3ll * nv)), dim3(DI_BLOCK), 0, s, 3 * nv, x, xs,
                     h, v);
}

namespace {

// Registrations of both sides and the two query argument sets; 0, -1 (HIP) or
// -2 (a box over too many cells).
int prepare(const CdSurface& S, const CdPositions& X, double dhat, const CdAlloc& alloc, devsort::Temp& tmp,
            hipStream_t s, int*& err, QueryArgs& qp, QueryArgs& qe) {
  const double r = 0.5 * std::sqrt(dhat), R = 2.0 * r * (1.0 + 1e-9);
  err = tmp.get<int>(1);
  CD_CHECK(tmp.err);
  CD_CHECK(hipMemsetAsync(err, 0, sizeof(int), s));
  Reg rt, re;
  RegCount ct, ce;
  int e = count_side<3>(S.nt, S.tris, X, R, S.cell, tmp, s, err, tmp.pin + PIN_REG_T, ct);
  if (e) return e;
  e = count_side<2>(S.ne, S.edges, X, R, S.cell, tmp, s, err, tmp.pin + PIN_REG_E, ce);
  if (e) return e;
  CD_CHECK(hipStreamSynchronize(s));
  e = place_side<3>(ct, X, R, S.cell, alloc, CD_REG_T, tmp, s, err, rt);
  if (e) return e;
  e = place_side<2>(ce, X, R, S.cell, alloc, CD_REG_E, tmp, s, err, re);
  if (e) return e;
  qp = query_args(S, X, false, rt, r, dhat, err);
  qe = query_args(S, X, true, re, r, dhat, err);
  return 0;
}

// The error flag (synchronises the stream; read-backs queued before it are
// then complete too).
int finish(devsort::Temp& tmp, int* err, hipStream_t s) {
  CD_CHECK(hipMemcpyAsync(tmp.pin + PIN_ERR, err, sizeof(int), hipMemcpyDeviceToHost, s));
  CD_CHECK(hipStreamSynchronize(s));
  return tmp.pin[PIN_ERR] ? -2 : 0;
}

// Candidate lists of both query sets (one count read-back for the two).
int candidates(QueryArgs& qp, QueryArgs& qe, devsort::Temp& tmp, hipStream_t s, int* err) {
  QueryArgs* qs[2] = {&qp, &qe};
  int32_t* off[2] = {nullptr, nullptr};
  for (int k = 0; k < 2; ++k) {
    QueryArgs& q = *qs[k];
    if (q.ma == 0 || q.nreg == 0) continue;
    q.ccnt = tmp.get<int32_t>(q.ma);
    off[k] = tmp.get<int32_t>((size_t)q.ma + 1);
    CD_CHECK(tmp.err);
    if (q.ee)
      hipLaunchKernelGGL((cand_kernel<2, false>), dim3(grid_q(q.ma)), dim3(CD_BLOCK), 0, s, q);
    else
      hipLaunchKernelGGL((cand_kernel<1, false>), dim3(grid_q(q.ma)), dim3(CD_BLOCK), 0, s, q);
    CD_CHECK(devsort::prefix(tmp, q.ccnt, off[k], q.ma, s));
  }
  int* h = tmp.pin;
  for (int k = 0; k < 2; ++k) {
    h[k] = 0;
    if (off[k]) CD_CHECK(hipMemcpyAsync(&h[k], off[k] + qs[k]->ma, sizeof(int), hipMemcpyDeviceToHost, s));
  }
  CD_CHECK(hipMemcpyAsync(&h[2], err, sizeof(int), hipMemcpyDeviceToHost, s));
  CD_CHECK(hipStreamSynchronize(s));
  if (h[2]) return -2;
  for (int k = 0; k < 2; ++k) {
    QueryArgs& q = *qs[k];
    q.ncand = 0;
    if (!off[k]) continue;
    if (h[k] < 0) return -2;  // more candidates than an int counts
    q.ncand = h[k];
    q.coff = off[k];
    q.cq = tmp.get<int32_t>(std::max(h[k], 1));
    q.ce = tmp.get<int32_t>(std::max(h[k], 1));
    CD_CHECK(tmp.err);
    if (q.ee)
      hipLaunchKernelGGL((cand_kernel<2, true>), dim3(grid_q((long long)CAND_TEAM * q.ma)), dim3(CD_BLOCK), 0, s, q);
    else
      hipLaunchKernelGGL((cand_kernel<1, true>), dim3(grid_q((long long)CAND_TEAM * q.ma)), dim3(CD_BLOCK), 0, s, q);
  }
  return 0;
}

template <int MODE>
void launch_pairs(const QueryArgs& q, hipStream_t s) {
  if (q.ncand == 0) return;
  if (q.ee)
    hipLaunchKernelGGL((pair_kernel<2, 2, MODE>), dim3(grid_q(q.ncand)), dim3(CD_BLOCK), 0, s, q);
  else
    hipLaunchKernelGGL((pair_kernel<1, 3, MODE>), dim3(grid_q(q.ncand)), dim3(CD_BLOCK), 0, s, q);
}

// Per-workgroup partials of both query sets folded into one value (kind 0
// sum, 1 min), read back into the pinned scratch at PIN_VAL (valid after
// finish), which starts at init.
int fold_both(QueryArgs& qp, QueryArgs& qe, int mode, devsort::Temp& tmp, hipStream_t s, double init) {
  double* out = reinterpret_cast<double*>(tmp.pin + PIN_VAL);
  const int gp = qp.ncand ? grid_q(qp.ncand) : 0, ge = qe.ncand ? grid_q(qe.ncand) : 0;
  double* part = tmp.get<double>((size_t)gp + ge + 1);
  CD_CHECK(tmp.err);
  qp.part = part;
  qe.part = part + gp;
  if (mode == Q_ENERGY) {
    launch_pairs<Q_ENERGY>(qp, s);
    launch_pairs<Q_ENERGY>(qe, s);
  } else {
    launch_pairs<Q_CCD>(qp, s);
    launch_pairs<Q_CCD>(qe, s);
  }
  *out = init;
  if (gp + ge) {
    hipLaunchKernelGGL(fold_kernel, dim3(1), dim3(CD_BLOCK), 0, s, part, gp + ge, mode == Q_CCD ? 1 : 0);
    CD_CHECK(hipMemcpyAsync(out, part, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  CD_CHECK(hipGetLastError());
  return 0;
}

}  // namespace

int cd_detect(const CdSurface& S, const CdPositions& X, double dhat, const CdAlloc& alloc, void* arena,
              size_t arena_bytes, size_t* arena_needed, int* pin, hipStream_t s, CdOutput& out) {
  devsort::Temp tmp;
  tmp.arena = static_cast<char*>(arena);
  tmp.cap = arena_bytes;
  tmp.pin = pin;
  out = CdOutput{};
  int* err = nullptr;
  QueryArgs qp{}, qe{};
  int e = prepare(S, X, dhat, alloc, tmp, s, err, qp, qe);
  if (e) return e;
  e = candidates(qp, qe, tmp, s, err);
  if (e) return e;
  // hits per candidate, scanned into output positions
  int32_t* hoff[2] = {nullptr, nullptr};
  QueryArgs* qs[2] = {&qp, &qe};
  for (int k = 0; k < 2; ++k) {
    QueryArgs& q = *qs[k];
    if (q.ncand == 0) continue;
    q.hit = tmp.get<int32_t>(q.ncand);
    hoff[k] = tmp.get<int32_t>((size_t)q.ncand + 1);
    CD_CHECK(tmp.err);
    launch_pairs<Q_COUNT>(q, s);
    CD_CHECK(devsort::prefix(tmp, q.hit, hoff[k], q.ncand, s));
  }
  int* m = tmp.pin;
  for (int k = 0; k < 2; ++k) {
    m[k] = 0;
    if (hoff[k]) CD_CHECK(hipMemcpyAsync(&m[k], hoff[k] + qs[k]->ncand, sizeof(int), hipMemcpyDeviceToHost, s));
  }
  e = finish(tmp, err, s);
  if (e) return e;
  const int total = m[0] + m[1], cap = std::max(total, 1);
  out.type = static_cast<int32_t*>(alloc(CD_TYPE, sizeof(int32_t) * (size_t)cap));
  out.idx = static_cast<int32_t*>(alloc(CD_IDX, 4 * sizeof(int32_t) * (size_t)cap));
  out.eps = static_cast<double*>(alloc(CD_EPS, sizeof(double) * (size_t)cap));
  if (!out.type || !out.idx || !out.eps) return -1;
  // point-triangle outputs first (a point's box is one cell, whose entries are
  // in triangle order: the listing is in (point, triangle) order), then the
  // edge-edge ones, written to a side buffer and put in (edge, partner) order
  const int me = std::max(m[1], 1);
  int32_t* te = tmp.get<int32_t>(me);
  int32_t* ie = tmp.get<int32_t>(4 * (size_t)me);
  double* ee = tmp.get<double>(me);
  uint64_t* key = tmp.get<uint64_t>(me);
  uint64_t* key_s = tmp.get<uint64_t>(me);
  int32_t* perm = tmp.get<int32_t>(me);
  int32_t* perm_s = tmp.get<int32_t>(me);
  CD_CHECK(tmp.err);
  if (m[0]) {
    qp.hoff = hoff[0];
    qp.out0 = 0;
    qp.cap = total;
    qp.otype = out.type;
    qp.oidx = out.idx;
    qp.oeps = out.eps;
    launch_pairs<Q_FILL>(qp, s);
  }
  if (m[1]) {
    qe.hoff = hoff[1];
    qe.out0 = 0;
    qe.cap = m[1];
    qe.otype = te;
    qe.oidx = ie;
    qe.oeps = ee;
    qe.okey = key;
    launch_pairs<Q_FILL>(qe, s);
    hipLaunchKernelGGL(iota32_kernel, dim3(devsort::grid_of(m[1])), dim3(DI_BLOCK), 0, s, m[1], perm);
    CD_CHECK(devsort::sort_pairs(tmp, key, key_s, perm, perm_s, m[1], 2 * qe.kbits, s));
    hipLaunchKernelGGL(gather_kernel, dim3(devsort::grid_of(m[1])), dim3(DI_BLOCK), 0, s, m[1], perm_s, te, ie, m[1],
                       ee, out.type + m[0], out.idx + m[0], total, out.eps + m[0]);
  }
  CD_CHECK(hipGetLastError());
  e = finish(tmp, err, s);  // also keeps the temporaries alive until the kernels are done
  if (e) return e;
  out.n = total;
  *arena_needed = tmp.used;
  return 0;
}

int cd_energy(const CdSurface& S, const CdPositions& X, double dhat, double kappa, int classic, const CdAlloc& alloc,
              void* arena, size_t arena_bytes, size_t* arena_needed, int* pin, hipStream_t s, double* e_out) {
  devsort::Temp tmp;
  tmp.arena = static_cast<char*>(arena);
  tmp.cap = arena_bytes;
  tmp.pin = pin;
  int* err = nullptr;
  QueryArgs qp{}, qe{};
  int e = prepare(S, X, dhat, alloc, tmp, s, err, qp, qe);
  if (e) return e;
  e = candidates(qp, qe, tmp, s, err);
  if (e) return e;
  for (QueryArgs* q : {&qp, &qe}) {
    q->kappa = kappa;
    q->classic = classic;
  }
  e = fold_both(qp, qe, Q_ENERGY, tmp, s, 0.0);
  if (e) return e;
  e = finish(tmp, err, s);
  if (e) return e;
  *e_out = *reinterpret_cast<const double*>(tmp.pin + PIN_VAL);
  *arena_needed = tmp.used;
  return 0;
}

int cd_ccd(const CdSurface& S, const CdPositions& X, double dhat, double t_max, double s_ccd, const CdAlloc& alloc,
           void* arena, size_t arena_bytes, size_t* arena_needed, int* pin, hipStream_t s, double* t_out) {
  devsort::Temp tmp;
  tmp.arena = static_cast<char*>(arena);
  tmp.cap = arena_bytes;
  tmp.pin = pin;
  int* err = nullptr;
  QueryArgs qp{}, qe{};
  int e = prepare(S, X, dhat, alloc, tmp, s, err, qp, qe);
  if (e) return e;
  e = candidates(qp, qe, tmp, s, err);
  if (e) return e;
  for (QueryArgs* q : {&qp, &qe}) {
    q->s_ccd = s_ccd;
    q->t_max = t_max;
  }
  e = fold_both(qp, qe, Q_CCD, tmp, s, t_max);
  if (e) return e;
  e = finish(tmp, err, s);
  if (e) return e;
  *t_out = std::fmin(*reinterpret_cast<const double*>(tmp.pin + PIN_VAL), t_max);
  *arena_needed = tmp.used;
  return 0;
}

}  // namespace yasps
