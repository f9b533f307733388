// Host-side entry to the per-stencil contact arithmetic of the GPU kernels
// (contact_math.h is __host__ __device__), so CPU tests can compare it with
// the oracle without a GPU.  Test infrastructure only.
#include "../../paper_2605_23088_amd/csrc/contact_math.h"

using namespace yasps;
using namespace yasps::cmath;

namespace {

template <int T, int K, bool EX, bool TRI = false>
int run(const double* x12, const int* fl4, double kappa, double dhat, int classic, double eps, double* e, double* d,
        double* g12, double* H144) {
  double xv[4][3];
  int fl[4];
  for (int a = 0; a < 4; ++a) {
    fl[a] = fl4[a];
    for (int i = 0; i < 3; ++i) xv[a][i] = x12[3 * a + i];
  }
  for (int i = 0; i < 12; ++i) g12[i] = 0.0;
  for (int i = 0; i < 144; ++i) H144[i] = 0.0;
  auto gs = [&](int k, const double (&gg)[3]) {
    for (int i = 0; i < 3; ++i) g12[3 * fl[k] + i] = gg[i];
  };
  auto bs = [&](int I, int J, const double (&B)[3][3]) {
    for (int i = 0; i < 3; ++i)
      for (int l = 0; l < 3; ++l) {
        H144[(3 * fl[I] + i) * 12 + 3 * fl[J] + l] = B[i][l];
        H144[(3 * fl[J] + l) * 12 + 3 * fl[I] + i] = B[i][l];
      }
  };
  double side;
  return contact_stencil<T, K, EX, TRI>(xv, fl, kappa, dhat, classic, *e, *d, side, gs, bs, eps) ? 0 : 1;
}

template <bool EX>
int dispatch(int type, int nfree, const double* x12, const int* fl4, double kappa, double dhat, int classic,
             double eps, double* e, double* d, double* g, double* H) {
  switch (type * 8 + nfree) {
    case 0 * 8 + 1: return run<0, 1, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 0 * 8 + 2: return run<0, 2, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 0 * 8 + 3:  // the library runs a triangle-free stencil through its own kernel
      if (fl4[0] == 1 && fl4[1] == 2 && fl4[2] == 3) return run<0, 3, EX, true>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
      return run<0, 3, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 0 * 8 + 4: return run<0, 4, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 1 * 8 + 1: return run<1, 1, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 1 * 8 + 2: return run<1, 2, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 1 * 8 + 3: return run<1, 3, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 1 * 8 + 4: return run<1, 4, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 2 * 8 + 1: return run<2, 1, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 2 * 8 + 2: return run<2, 2, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 2 * 8 + 3: return run<2, 3, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 3 * 8 + 1: return run<3, 1, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    case 3 * 8 + 2: return run<3, 2, EX>(x12, fl4, kappa, dhat, classic, eps, e, d, g, H);
    default: return 2;
  }
}

}  // namespace

extern "C" int contact_host(int type, int nfree, int exact, const double* x12, const int* fl4, double kappa,
                            double dhat, int classic, double eps, double* e, double* d, double* g12, double* H144) {
  return exact ? dispatch<true>(type, nfree, x12, fl4, kappa, dhat, classic, eps, e, d, g12, H144)
               : dispatch<false>(type, nfree, x12, fl4, kappa, dhat, classic, eps, e, d, g12, H144);
}
