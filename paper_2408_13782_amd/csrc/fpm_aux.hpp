// fpm_aux.hpp - pupil model, parameter-gradient projection, Adam and the
// high-resolution transforms (spectrum <-> object, initial value, refocus).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_line.hpp"
#include "fpm_kernels.hpp"

namespace fpm {

constexpr int kZern = 15;
constexpr int kPar = 16;   // 15 Zernike coefficients + defocus

// Optics constants handed to the pupil kernels.
struct PupilGeom {
  int n;            // N
  double inv_r;     // 1 / pupil radius in spectral pixels
  double dk2;       // dk^2
  double inv_l;     // 1 / lambda
};

// OSA/ANSI Zernike terms j = 0..14, unit RMS on the unit disk, as Cartesian
// polynomials of the normalised pupil coordinates (x along k_x, y along k_y).
__device__ __forceinline__ void zernike15(double x, double y, double* z) {
  const double s3 = 1.7320508075688772, s5 = 2.2360679774997897, s6 = 2.4494897427831781;
  const double s8 = 2.8284271247461901, s10 = 3.1622776601683795;
  const double x2 = x * x, y2 = y * y, r2 = x2 + y2, xy = x * y;
  z[0] = 1.0;
  z[1] = 2.0 * y;
  z[2] = 2.0 * x;
  z[3] = s6 * 2.0 * xy;
  z[4] = s3 * (2.0 * r2 - 1.0);
  z[5] = s6 * (x2 - y2);
  z[6] = s8 * (3.0 * x2 - y2) * y;
  z[7] = s8 * (3.0 * r2 - 2.0) * y;
  z[8] = s8 * (3.0 * r2 - 2.0) * x;
  z[9] = s8 * (x2 - 3.0 * y2) * x;
  z[10] = s10 * 4.0 * xy * (x2 - y2);
  z[11] = s10 * (4.0 * r2 - 3.0) * 2.0 * xy;
  z[12] = s5 * (6.0 * r2 * r2 - 6.0 * r2 + 1.0);
  z[13] = s10 * (4.0 * r2 - 3.0) * (x2 - y2);
  z[14] = s10 * (x2 * x2 - 6.0 * x2 * y2 + y2 * y2);
}

// Defocus phase per um, kappa = 2 pi (sqrt(1/l^2 - k^2) - 1/l), written in the
// cancellation-free form -2 pi k^2 / (sqrt(1/l^2 - k^2) + 1/l); 0 if evanescent.
__device__ __forceinline__ double defocus_kappa(double k2, double inv_l) {
  const double a = inv_l * inv_l - k2;
  if (a < 0.0) return 0.0;
  return -2.0 * 3.141592653589793 * k2 / (sqrt(a) + inv_l);
}

__global__ void __launch_bounds__(256)
pupil_build(PupilGeom g, const int2* __restrict__ rowext, const float* __restrict__ coeffs,
            int n_zern, const float* __restrict__ z_um, float2* __restrict__ P) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = g.n;
  if (idx >= n * n) return;
  const int ky = idx / n, kx = idx - ky * n;
  const int2 e = rowext[ky];
  if (kx < e.x || kx > e.y) {
    P[idx] = make_float2(0.f, 0.f);
    return;
  }
  const double ux = kx - n / 2, uy = ky - n / 2;
  double th = 0.0;
  if (coeffs && n_zern > 0) {
    double z[kZern];
    zernike15(ux * g.inv_r, uy * g.inv_r, z);
    for (int j = 0; j < n_zern; ++j) th += (double)coeffs[j] * z[j];
  }
  if (z_um) th += (double)z_um[0] * defocus_kappa((ux * ux + uy * uy) * g.dk2, g.inv_l);
  double sn, cs;
  sincos(th, &sn, &cs);
  P[idx] = make_float2((float)cs, (float)sn);
}

// g_par[j] += sum_u Im(gP conj P) Z_j, g_par[15] += sum_u Im(gP conj P) kappa.
// With `clear`, gP is zeroed on the disk after it is read.
__global__ void __launch_bounds__(256)
pupil_grad(PupilGeom g, const int2* __restrict__ rowext, float2* __restrict__ gP,
           const float2* __restrict__ P, double* __restrict__ g_par, int clear) {
  __shared__ double part[4][kPar];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = g.n;
  double acc[kPar];
#pragma unroll
  for (int j = 0; j < kPar; ++j) acc[j] = 0.0;
  if (idx < n * n) {
    const int ky = idx / n, kx = idx - ky * n;
    const int2 e = rowext[ky];
    if (kx >= e.x && kx <= e.y) {
      const float2 gp = gP[idx];
      const float2 p = P[idx];
      const double gth = (double)gp.y * p.x - (double)gp.x * p.y;
      const double ux = kx - n / 2, uy = ky - n / 2;
      double z[kZern];
      zernike15(ux * g.inv_r, uy * g.inv_r, z);
#pragma unroll
      for (int j = 0; j < kZern; ++j) acc[j] = gth * z[j];
      acc[kZern] = gth * defocus_kappa((ux * ux + uy * uy) * g.dk2, g.inv_l);
      if (clear) gP[idx] = make_float2(0.f, 0.f);
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < kPar; ++j) {
    double v = acc[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) part[wave][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < kPar) {
    const double s = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                     part[3][threadIdx.x];
    unsafeAtomicAdd(g_par + threadIdx.x, s);
  }
}

// Adam over 32 x 32 tiles of the HR spectrum (each thread: 8 consecutive floats);
// the gradient is read and cleared.
struct AdamCoef {
  float b1, b2, eps, step_size, sqrt_bc2;
};

__device__ __forceinline__ void adam1(float& p, float& m, float& v, float g, const AdamCoef& c) {
  m = c.b1 * m + (1.0f - c.b1) * g;
  v = c.b2 * v + (1.0f - c.b2) * g * g;
  const float den = sqrtf(v) / c.sqrt_bc2 + c.eps;
  p -= c.step_size * (m / den);
}

__global__ void __launch_bounds__(256)
adam_object(const int2* __restrict__ tiles, int M, float* __restrict__ O, float* __restrict__ mO,
            float* __restrict__ vO, float* __restrict__ gO, AdamCoef c) {
  const int2 tl = tiles[blockIdx.x];
  const int r = tl.x * 32 + (threadIdx.x >> 3);
  const int col = tl.y * 32 + (threadIdx.x & 7) * 4;         // complex column
  const size_t f = ((size_t)r * M + col) * 2;                  // float offset
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float4* po = reinterpret_cast<float4*>(O + f) + h;
    float4* pm = reinterpret_cast<float4*>(mO + f) + h;
    float4* pv = reinterpret_cast<float4*>(vO + f) + h;
    float4* pg = reinterpret_cast<float4*>(gO + f) + h;
    float4 o = *po, m = *pm, v = *pv, g = *pg;
    adam1(o.x, m.x, v.x, g.x, c);
    adam1(o.y, m.y, v.y, g.y, c);
    adam1(o.z, m.z, v.z, g.z, c);
    adam1(o.w, m.w, v.w, g.w, c);
    *po = o;
    *pm = m;
    *pv = v;
    *pg = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// Adam on the pupil parameters (15 Zernike coefficients, defocus), FP64 inside;
// clears the accumulated gradients.
struct AdamScalarArgs {
  float* coeffs; float* m_c; float* v_c; int learn_c;
  float* z; float* m_z; float* v_z; int learn_z;
  double lr_c, lr_z, b1, b2, eps, bc1, sqrt_bc2;
};

__global__ void adam_scalars(AdamScalarArgs a, double* __restrict__ g_par) {
  const int j = threadIdx.x;
  if (j >= kPar) return;
  const double g = g_par[j];
  g_par[j] = 0.0;
  float *p, *m, *v;
  double lr;
  if (j < kZern) {
    // piston (j = 0): a global phase with an identically zero gradient, held fixed
    if (!a.learn_c || j == 0) return;
    p = a.coeffs + j; m = a.m_c + j; v = a.v_c + j; lr = a.lr_c;
  } else {
    if (!a.learn_z) return;
    p = a.z; m = a.m_z; v = a.v_z; lr = a.lr_z;
  }
  const double mm = a.b1 * (double)*m + (1.0 - a.b1) * g;
  const double vv = a.b2 * (double)*v + (1.0 - a.b2) * g * g;
  const double den = sqrt(vv) / a.sqrt_bc2 + a.eps;
  *p = (float)((double)*p - (lr / a.bc1) * mm / den);
  *m = (float)mm;
  *v = (float)vv;
}

// ---------------------------------------------------------------------------
// High-resolution 2-D transforms, split into a row pass and a column pass.

template <int M> struct HrRowLines { static constexpr int value = (128 / Plan1D<M>::T) > 0 ? 128 / Plan1D<M>::T : 1; };
template <int M> struct HrColLines { static constexpr int value = M >= 2048 ? 8 : 16; };

enum HrRowMode { kRowFwd = 0, kRowInv = 1, kRowInit = 2, kRowRefocus = 3 };

struct HrArgs {
  const float2* in;     // row-pass source (object, spectrum)
  const float* img;     // kRowInit: centre amplitude image [n][n]
  int n, s;             // kRowInit: LR size and upsampling
  const float* z_um;    // kRowRefocus: device pointer to the distance
  double dk2, inv_l;    // kRowRefocus
  float2* out;          // destination of both passes
};

// Forward (DIR -1): rows of o, DFT, fftshift along k_x.
// Inverse (DIR +1): ifftshift along k_x (times H(z) when refocusing), inverse DFT.
template <int M, int MODE>
__global__ void __launch_bounds__(HrRowLines<M>::value * Plan1D<M>::T)
hr_rows(HrArgs a, const float2* __restrict__ tw) {
  constexpr int T = Plan1D<M>::T;
  constexpr int E = M / T;
  constexpr int L = HrRowLines<M>::value;
  constexpr int DIR = (MODE == kRowFwd || MODE == kRowInit) ? -1 : +1;
  __shared__ float2 lds[L * (M + 1)];
  const int line = threadIdx.x / T, t = threadIdx.x % T;
  const int row = blockIdx.x * L + line;   // grid covers M rows exactly
  float2 v[E];
  if constexpr (MODE == kRowFwd) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = a.in[(size_t)row * M + t + m * T];
  } else if constexpr (MODE == kRowInit) {
    // bilinear upsampling by s, pixel-centre aligned, borders clamped
    const float sy = fmaxf((row + 0.5f) / a.s - 0.5f, 0.f);
    int y0 = min((int)floorf(sy), a.n - 1);
    const int y1 = min(y0 + 1, a.n - 1);
    const float wy = sy - (float)y0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int X = t + m * T;
      const float sx = fmaxf((X + 0.5f) / a.s - 0.5f, 0.f);
      const int x0 = min((int)floorf(sx), a.n - 1);
      const int x1 = min(x0 + 1, a.n - 1);
      const float wx = sx - (float)x0;
      const float top = a.img[y0 * a.n + x0] * (1.f - wx) + a.img[y0 * a.n + x1] * wx;
      const float bot = a.img[y1 * a.n + x0] * (1.f - wx) + a.img[y1 * a.n + x1] * wx;
      v[m] = make_float2(top * (1.f - wy) + bot * wy, 0.f);
    }
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kx = half_shift<M>(t + m * T);
      float2 val = a.in[(size_t)row * M + kx];
      if constexpr (MODE == kRowRefocus) {
        const double uy = row - M / 2, ux = kx - M / 2;
        const double k2 = (ux * ux + uy * uy) * a.dk2;
        if (k2 > a.inv_l * a.inv_l) {
          val = make_float2(0.f, 0.f);
        } else {
          double sn, cs;
          sincos((double)*a.z_um * defocus_kappa(k2, a.inv_l), &sn, &cs);
          val = cmul(val, make_float2((float)cs, (float)sn));
        }
      }
      v[m] = val;
    }
  }
  Plan1D<M>::template run<DIR>(v, t, lds + line * (M + 1), [](int n) { return n; }, tw);
  float2* orow = a.out + (size_t)row * M;
  if constexpr (DIR < 0) {
#pragma unroll
    for (int m = 0; m < E; ++m) orow[half_shift<M>(t + m * T)] = v[m];
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) orow[t + m * T] = v[m];
  }
}

// Column pass in place on a.out, scaled by 1/M. Forward: DFT, fftshift along
// k_y. Inverse: ifftshift along k_y, inverse DFT.
template <int M, int DIR>
__global__ void __launch_bounds__(HrColLines<M>::value * Plan1D<M>::T)
hr_cols(float2* __restrict__ data, const float2* __restrict__ tw) {
  constexpr int T = Plan1D<M>::T;
  constexpr int E = M / T;
  constexpr int L = HrColLines<M>::value;
  __shared__ float2 lds[M * (L + 1)];
  const int line = threadIdx.x % L, t = threadIdx.x / L;
  const int x = blockIdx.x * L + line;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int n = t + m * T;
    v[m] = data[(size_t)(DIR > 0 ? half_shift<M>(n) : n) * M + x];
  }
  auto lay = [line](int n) { return n * (L + 1) + line; };
  Plan1D<M>::template run<DIR>(v, t, lds, lay, tw);
  constexpr float inv = 1.0f / M;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int n = t + m * T;
    data[(size_t)(DIR < 0 ? half_shift<M>(n) : n) * M + x] = cscale(v[m], inv);
  }
}

}  // namespace fpm
