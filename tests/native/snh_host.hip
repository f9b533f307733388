// Host-side entry to the closed-form Neo-Hookean projection of the GPU kernels
// (snh_math.h is __host__ __device__).  Test infrastructure only.
#include "../../paper_2605_23088_amd/csrc/snh_math.h"

using namespace yasps;

extern "C" void snh_proj_host(const double* F9, double mu, double lam, double vol, double* P81, double* U9,
                              double* s3, double* V9) {
  double F[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F[i][j] = F9[3 * i + j];
  Sym<9, double> P;
  snh::projected_hessian<double>(F, mu, lam, vol, P);
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) P81[9 * r + c] = P(r, c);
  double U[3][3], V[3][3], s[3];
  snh::svd3<double>(F, U, s, V);
  for (int i = 0; i < 3; ++i) {
    s3[i] = s[i];
    for (int j = 0; j < 3; ++j) {
      U9[3 * i + j] = U[i][j];
      V9[3 * i + j] = V[i][j];
    }
  }
}

extern "C" void snh_proj_host_f32(const double* F9, double mu, double lam, double vol, double* P81) {
  float F[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F[i][j] = float(F9[3 * i + j]);
  Sym<9, float> P;
  snh::projected_hessian<float>(F, float(mu), float(lam), float(vol), P);
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) P81[9 * r + c] = double(P(r, c));
}
