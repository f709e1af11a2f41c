// fpm_kernels.hpp - device kernels of the Batch-FPM hot path (gfx950).
//
// Per random batch of B LEDs, a loss-and-gradient pass is three launches
// (the 2-D transforms of N x N images do not fit one CU's LDS for N >= 256,
// so they are split into row and column passes that meet in an L2/MALL
// resident scratch X[B][N][N]):
//
//   rows_forward   crop C_b = O[w_b + u] on the pupil disk, Phi = C_b P,
//                  ifftshift along k_x, inverse DFT of each disk row -> X
//   cols           inverse DFT of each column (ifftshift along k_y) -> psi,
//                  amplitude residual e = sqrt(gamma)|psi| - A, loss,
//                  g_psi = 2 sqrt(gamma) e psi / |psi|, forward DFT of each
//                  column, keep disk rows (fftshift) -> X (in place)
//   rows_backward  forward DFT of each disk row, keep disk columns, scatter-add
//                  conj(P) g_Phi into g_O and conj(C_b) g_Phi into g_P
//
// Workgroups of one LED are placed on one XCD (workgroup id mod 8 selects
// the XCD) so that the scratch written by one pass is read from the same
// XCD's L2 by the next.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_line.hpp"

namespace fpm {

constexpr int kRowThreads = 128;   // threads per workgroup in the row passes
constexpr int kXcds = 8;

template <int N> struct ColLines { static constexpr int value = 16; };
template <> struct ColLines<512> { static constexpr int value = 8; };

// (n + N/2) mod N: the index shift between centred and DFT order.
template <int N>
__device__ __forceinline__ int half_shift(int n) {
  if constexpr ((N & (N - 1)) == 0) {
    return n ^ (N / 2);
  } else {
    return n < N / 2 ? n + N / 2 : n - N / 2;
  }
}

// Workgroup -> (batch slot b, chunk c) with all chunks of slot b on XCD b mod 8.
__device__ __forceinline__ bool xcd_map(int wg, int chunks, int B, int& b, int& c) {
  const int xcd = wg % kXcds;
  const int q = wg / kXcds;
  const int r = q / chunks;
  c = q - r * chunks;
  b = xcd + kXcds * r;
  return b < B;
}

__device__ __forceinline__ void atomic_add_c(float2* p, float2 v) {
  float* f = reinterpret_cast<float*>(p);
  unsafeAtomicAdd(f, v.x);
  unsafeAtomicAdd(f + 1, v.y);
}

// Sum a per-thread double over the workgroup and add it to *dst (one atomic per wave).
__device__ __forceinline__ void wave_atomic_add(double v, double* dst) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) unsafeAtomicAdd(dst, v);
}

// ---------------------------------------------------------------------------
// Row pass 1: crop, pupil, inverse DFT along k_x.
template <int N>
__global__ void __launch_bounds__(kRowThreads)
rows_forward(const float2* __restrict__ O, int M, const float2* __restrict__ P,
             const int2* __restrict__ rowext, int ky0, int nrows,
             const int2* __restrict__ shifts, const int* __restrict__ leds, int B, int n_led,
             int chunks, float2* __restrict__ X, const float2* __restrict__ tw) {
  constexpr int T = Plan1D<N>::T;
  constexpr int E = N / T;
  constexpr int L = kRowThreads / T;
  __shared__ float2 lds[L * (N + 1)];
  int b, c;
  if (!xcd_map(blockIdx.x, chunks, B, b, c)) return;
  const int led = leds[b];
  if ((unsigned)led >= (unsigned)n_led) return;   // invalid id: the image contributes nothing
  const int line = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const int rr = c * L + line;
  const bool active = rr < nrows;
  const int ky = ky0 + (active ? rr : 0);
  const int2 s = shifts[led];
  const int base = M / 2 - N / 2;
  const int2 ext = rowext[ky];
  const float2* orow = O + (size_t)(base + s.x + ky) * M + (base + s.y);
  const float2* prow = P + (size_t)ky * N;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kx = half_shift<N>(t + m * T);
    v[m] = (active && kx >= ext.x && kx <= ext.y) ? cmul(orow[kx], prow[kx]) : make_float2(0.f, 0.f);
  }
  float2* my = lds + line * (N + 1);
  Plan1D<N>::template run<+1>(v, t, my, [](int n) { return n; }, tw);
  if (active) {
    float2* xr = X + ((size_t)b * N + ky) * N;
#pragma unroll
    for (int m = 0; m < E; ++m) xr[t + m * T] = v[m];
  }
}

// Column pass: inverse DFT along k_y, amplitude loss, residual, forward DFT.
// kForward: write amplitudes (and fields) instead of the residual transform.
template <int N, bool kForward>
__global__ void __launch_bounds__(ColLines<N>::value * Plan1D<N>::T)
cols(float2* __restrict__ X, const float* __restrict__ A, const float* __restrict__ gamma,
     const int* __restrict__ leds, int B, int n_led, int ky_lo, int ky_hi, int groups,
     double* __restrict__ loss, float* __restrict__ amp_out, float2* __restrict__ field_out,
     const float2* __restrict__ tw, float inv_m) {
  constexpr int T = Plan1D<N>::T;
  constexpr int E = N / T;
  constexpr int L = ColLines<N>::value;
  __shared__ float2 lds[N * (L + 1)];
  int b, g;
  if (!xcd_map(blockIdx.x, groups, B, b, g)) return;
  const int led = leds[b];
  if ((unsigned)led >= (unsigned)n_led) return;
  const int line = threadIdx.x % L;
  const int t = threadIdx.x / L;
  const int x = g * L + line;
  float2* xb = X + (size_t)b * N * N;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int ky = half_shift<N>(t + m * T);
    v[m] = (ky >= ky_lo && ky <= ky_hi) ? xb[(size_t)ky * N + x] : make_float2(0.f, 0.f);
  }
  auto lay = [line](int n) { return n * (L + 1) + line; };
  Plan1D<N>::template run<+1>(v, t, lds, lay, tw);
  const float sg = gamma ? sqrtf(gamma[led]) : 1.0f;
  if constexpr (kForward) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int y = t + m * T;
      const float2 psi = cscale(v[m], inv_m);
      const size_t o = ((size_t)b * N + y) * N + x;
      amp_out[o] = sg * sqrtf(psi.x * psi.x + psi.y * psi.y);
      if (field_out) field_out[o] = psi;
    }
  } else {
    const float* ab = A + (size_t)led * N * N;
    float acc = 0.f;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int y = t + m * T;
      const float2 psi = cscale(v[m], inv_m);
      const float a = sqrtf(psi.x * psi.x + psi.y * psi.y);
      const float e = sg * a - ab[(size_t)y * N + x];
      acc += e * e;
      const float f = a > 0.f ? 2.f * sg * e / a : 0.f;
      v[m] = cscale(psi, f);
    }
    Plan1D<N>::template run<-1>(v, t, lds, lay, tw);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int ky = half_shift<N>(t + m * T);
      if (ky >= ky_lo && ky <= ky_hi) xb[(size_t)ky * N + x] = cscale(v[m], inv_m);
    }
    if (loss) wave_atomic_add((double)acc, loss);
  }
}

// Row pass 2: forward DFT along x, conj-pupil, scatter-add into g_O and g_P.
template <int N>
__global__ void __launch_bounds__(kRowThreads)
rows_backward(const float2* __restrict__ X, const float2* __restrict__ O, int M,
              const float2* __restrict__ P, const int2* __restrict__ rowext, int ky0, int nrows,
              const int2* __restrict__ shifts, const int* __restrict__ leds, int B, int n_led,
              int chunks, float2* __restrict__ gO, float2* __restrict__ gP,
              const float2* __restrict__ tw) {
  constexpr int T = Plan1D<N>::T;
  constexpr int E = N / T;
  constexpr int L = kRowThreads / T;
  __shared__ float2 lds[L * (N + 1)];
  int b, c;
  if (!xcd_map(blockIdx.x, chunks, B, b, c)) return;
  const int led = leds[b];
  if ((unsigned)led >= (unsigned)n_led) return;
  const int line = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const int rr = c * L + line;
  const bool active = rr < nrows;
  const int ky = ky0 + (active ? rr : 0);
  const float2* xr = X + ((size_t)b * N + ky) * N;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = active ? xr[t + m * T] : make_float2(0.f, 0.f);
  float2* my = lds + line * (N + 1);
  Plan1D<N>::template run<-1>(v, t, my, [](int n) { return n; }, tw);
  if (!active) return;
  const int2 s = shifts[led];
  const int base = M / 2 - N / 2;
  const int2 ext = rowext[ky];
  const size_t orow = (size_t)(base + s.x + ky) * M + (base + s.y);
  const float2* prow = P + (size_t)ky * N;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kx = half_shift<N>(t + m * T);
    if (kx >= ext.x && kx <= ext.y) {
      const float2 g = v[m];
      atomic_add_c(gO + orow + kx, cmulc(prow[kx], g));
      if (gP) atomic_add_c(gP + (size_t)ky * N + kx, cmulc(O[orow + kx], g));
    }
  }
}

}  // namespace fpm
