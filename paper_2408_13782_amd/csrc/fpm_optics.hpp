// fpm_optics.hpp - pupil-plane functions shared by the kernels: OSA/ANSI
// Zernike terms (Eq. 3's aberrated pupil) and the defocus phase of H(k, z).
#pragma once
#include <hip/hip_runtime.h>

namespace fpm {

constexpr int kZern = 15;
constexpr int kPar = 16;   // 15 Zernike coefficients + defocus

// OSA/ANSI Zernike terms j = 0..14, unit RMS on the unit disk, as Cartesian
// polynomials of the normalised pupil coordinates (x along k_x, y along k_y).
template <class R>
__device__ __forceinline__ void zernike15(R x, R y, R* z) {
  const R s3 = R(1.7320508075688772), s5 = R(2.2360679774997897), s6 = R(2.4494897427831781);
  const R s8 = R(2.8284271247461901), s10 = R(3.1622776601683795);
  const R x2 = x * x, y2 = y * y, r2 = x2 + y2, xy = x * y;
  z[0] = R(1);
  z[1] = R(2) * y;
  z[2] = R(2) * x;
  z[3] = s6 * R(2) * xy;
  z[4] = s3 * (R(2) * r2 - R(1));
  z[5] = s6 * (x2 - y2);
  z[6] = s8 * (R(3) * x2 - y2) * y;
  z[7] = s8 * (R(3) * r2 - R(2)) * y;
  z[8] = s8 * (R(3) * r2 - R(2)) * x;
  z[9] = s8 * (x2 - R(3) * y2) * x;
  z[10] = s10 * R(4) * xy * (x2 - y2);
  z[11] = s10 * (R(4) * r2 - R(3)) * R(2) * xy;
  z[12] = s5 * (R(6) * r2 * r2 - R(6) * r2 + R(1));
  z[13] = s10 * (R(4) * r2 - R(3)) * (x2 - y2);
  z[14] = s10 * (x2 * x2 - R(6) * x2 * y2 + y2 * y2);
}

// The same terms as linear combinations of the 15 monomials x^a y^b, a + b <= 4,
// in the order (0,0) (1,0) (0,1) (2,0) (1,1) (0,2) (3,0) (2,1) (1,2) (0,3)
// (4,0) (3,1) (2,2) (1,3) (0,4): Z_j = sum_k kZernMono[j][k] m_k. A sum of
// g(u) Z_j(u) over the pupil is then kZernMono applied to the 15 moments
// sum_u g(u) x^a y^b.
constexpr int kMono = 15;
constexpr double kZernMono[kZern][kMono] = {
    {1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 2, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 2, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 4.8989794855663558, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {-1.7320508075688772, 0, 0, 3.4641016151377544, 0, 3.4641016151377544, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 2.4494897427831779, 0, -2.4494897427831779, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 8.4852813742385713, 0, -2.8284271247461903, 0, 0, 0, 0, 0},
    {0, 0, -5.6568542494923806, 0, 0, 0, 0, 8.4852813742385713, 0, 8.4852813742385713, 0, 0, 0, 0, 0},
    {0, -5.6568542494923806, 0, 0, 0, 0, 8.4852813742385713, 0, 8.4852813742385713, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 2.8284271247461903, 0, -8.4852813742385713, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 12.649110640673518, 0, -12.649110640673518, 0},
    {0, 0, 0, 0, -18.973665961010276, 0, 0, 0, 0, 0, 0, 25.298221281347036, 0, 25.298221281347036, 0},
    {2.2360679774997898, 0, 0, -13.416407864998739, 0, -13.416407864998739, 0, 0, 0, 0, 13.416407864998739, 0, 26.832815729997478, 0, 13.416407864998739},
    {0, 0, 0, -9.4868329805051381, 0, 9.4868329805051381, 0, 0, 0, 0, 12.649110640673518, 0, 0, 0, -12.649110640673518},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 3.1622776601683795, 0, -18.973665961010276, 0, 3.1622776601683795},
};

// Defocus phase per um, kappa = 2 pi (sqrt(1/l^2 - k^2) - 1/l), written in the
// cancellation-free form -2 pi k^2 / (sqrt(1/l^2 - k^2) + 1/l); 0 if evanescent.
template <class R>
__device__ __forceinline__ R defocus_kappa(R k2, R inv_l) {
  const R a = inv_l * inv_l - k2;
  if (a < R(0)) return R(0);
  return R(-6.283185307179586) * k2 / (sqrt(a) + inv_l);
}

// Pupil-plane constants (N, 1/radius in pixels, dk^2, 1/lambda).
struct PupilGeom {
  int n;
  double inv_r;
  double dk2;
  double inv_l;
};

}  // namespace fpm
