// Host-side entry to the per-stencil cloth arithmetic of the GPU kernels
// (cloth_math.h is __host__ __device__), so CPU tests can compare it with the
// oracle without a GPU.  Test infrastructure only.
#include "../../paper_2605_23088_amd/csrc/cloth_math.h"

using namespace yasps;

namespace {

template <int K, bool EX>
int hinge_run(const double* x12, const int* fl4, double tb, double k, double h2, double* e, double* th, double* g12,
              double* H144) {
  double xv[4][3];
  int fl[4];
  for (int a = 0; a < 4; ++a) {
    fl[a] = fl4[a];
    for (int i = 0; i < 3; ++i) xv[a][i] = x12[3 * a + i];
  }
  for (int i = 0; i < 12; ++i) g12[i] = 0.0;
  for (int i = 0; i < 144; ++i) H144[i] = 0.0;
  auto gs = [&](int q, const double (&gg)[3]) {
    for (int i = 0; i < 3; ++i) g12[3 * fl[q] + i] = gg[i];
  };
  auto bs = [&](int I, int J, const double (&B)[3][3]) {
    for (int i = 0; i < 3; ++i)
      for (int l = 0; l < 3; ++l) {
        H144[(3 * fl[I] + i) * 12 + 3 * fl[J] + l] = B[i][l];
        H144[(3 * fl[J] + l) * 12 + 3 * fl[I] + i] = B[i][l];
      }
  };
  return cloth::hinge_stencil<K, EX>(xv, fl, tb, k, h2, *e, *th, gs, bs) ? 0 : 1;
}

template <bool EX>
int hinge_dispatch(int nfree, const double* x12, const int* fl4, double tb, double k, double h2, double* e, double* th,
                   double* g, double* H) {
  switch (nfree) {
    case 1: return hinge_run<1, EX>(x12, fl4, tb, k, h2, e, th, g, H);
    case 2: return hinge_run<2, EX>(x12, fl4, tb, k, h2, e, th, g, H);
    case 3: return hinge_run<3, EX>(x12, fl4, tb, k, h2, e, th, g, H);
    case 4: return hinge_run<4, EX>(x12, fl4, tb, k, h2, e, th, g, H);
    default: return 2;
  }
}

template <bool EX>
int membrane_run(const double* x9, const double* dinv4, double area, double thick, double mu, double lam, double h2,
                 const int* free3, double* e, double* g9, double* H81) {
  double xv[3][3], D[2][2];
  bool fr[3];
  for (int a = 0; a < 3; ++a) {
    fr[a] = free3[a] != 0;
    for (int i = 0; i < 3; ++i) xv[a][i] = x9[3 * a + i];
  }
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) D[r][c] = dinv4[2 * r + c];
  for (int i = 0; i < 9; ++i) g9[i] = 0.0;
  for (int i = 0; i < 81; ++i) H81[i] = 0.0;
  auto gs = [&](int v, const double (&gg)[3]) {
    for (int i = 0; i < 3; ++i) g9[3 * v + i] = gg[i];
  };
  auto bs = [&](int v, int w, const double (&B)[3][3]) {
    for (int i = 0; i < 3; ++i)
      for (int l = 0; l < 3; ++l) {
        H81[(3 * v + i) * 9 + 3 * w + l] = B[i][l];
        H81[(3 * w + l) * 9 + 3 * v + i] = B[i][l];
      }
  };
  return cloth::membrane_stencil<EX>(xv, D, area, thick, mu, lam, h2, fr, *e, gs, bs) ? 0 : 1;
}

}  // namespace

extern "C" int hinge_host(int nfree, int exact, const double* x12, const int* fl4, double theta_bar, double stiff,
                          double h2, double* e, double* theta, double* g12, double* H144) {
  return exact ? hinge_dispatch<true>(nfree, x12, fl4, theta_bar, stiff, h2, e, theta, g12, H144)
               : hinge_dispatch<false>(nfree, x12, fl4, theta_bar, stiff, h2, e, theta, g12, H144);
}

extern "C" int membrane_host(int exact, const double* x9, const double* dinv4, double area, double thick, double mu,
                             double lam, double h2, const int* free3, double* e, double* g9, double* H81) {
  return exact ? membrane_run<true>(x9, dinv4, area, thick, mu, lam, h2, free3, e, g9, H81)
               : membrane_run<false>(x9, dinv4, area, thick, mu, lam, h2, free3, e, g9, H81);
}
