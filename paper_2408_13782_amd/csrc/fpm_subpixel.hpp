// fpm_subpixel.hpp - the multi-parameter path: sub-pixel LED offsets from the
// LED-array geometry, bilinear crop and its adjoint, gradients with respect to
// the geometry and the LED intensities (paper Sec. 2.1 k_m and Eq. 3; Sec. 2.2).
//
// Launch order of one loss-and-gradient call:
//   led_subpixel       offsets s_b = k_b(geometry) / dk, their Jacobian (FP64)
//   rows_forward_sub   bilinear crop C_b (4 taps) * P, inverse DFT of disk rows
//   cols<.., kGamma>   as in the nearest path, plus sum e |psi| per workgroup
//   rows_backward_sub  forward DFT of disk rows; patch conj(P) g_Phi; pupil
//                      moments; dL/ds_b = sum Re(conj(g_C) dC/ds) partials
//   gather_dense       g_O += sum_b sum_taps w_t patch_b (each pixel one thread)
//   loss_grad_reduce   loss, Zernike/defocus, geometry (J_b^T dL/ds_b), gamma
#pragma once
#include <hip/hip_runtime.h>

#include "fft_line.hpp"
#include "fpm_kernels.hpp"
#include "fpm_optics.hpp"

namespace fpm {

// One batch slot of the sub-pixel path: window corner (integer part), the
// fractional part, and ds/d(shift_x, shift_y, rot, dh) as rows (s_row, s_col).
struct SubSlot {
  int fr, fc;
  float ay, ax;
  double J[8];
};

// LED-array geometry (nominal grid plus learned errors) and optics constants.
struct GeomArgs {
  int n_side;
  double pitch_mm, height_mm, roi_x_mm, roi_y_mm;
  double base_dx, base_dy, base_rot, base_dh;   // nominal errors of the grid description
  double inv_dk, lambda;
  int N, M;
};

// Offsets of the batch's LEDs. With geom == NULL the plan's integer offsets
// are used (zero fractional part, zero Jacobian). A window that would leave
// the HR grid (with one pixel of bilinear margin) is clamped and counted in
// *oob (the caller reports it).
__global__ void led_subpixel(GeomArgs g, const double* __restrict__ geom, Batch bt,
                             SubSlot* __restrict__ out, int* __restrict__ oob) {
  const int b = threadIdx.x;
  if (b >= bt.B) return;
  const int base = g.M / 2 - g.N / 2;
  SubSlot sl;
  for (int q = 0; q < 8; ++q) sl.J[q] = 0.0;
  double sr, sc;
  if (!geom) {
    sr = bt.win[b].x - base;
    sc = bt.win[b].y - base;
  } else {
    const double dxm = g.base_dx + geom[0], dym = g.base_dy + geom[1];
    const double rot = g.base_rot + geom[2], dh = g.base_dh + geom[3];
    const int led = bt.led[b];
    const int row = led / g.n_side, col = led - row * g.n_side;
    const double c = (g.n_side - 1) / 2.0;
    const double i = col - c, j = row - c;
    const double cr = cos(rot), snr = sin(rot);
    const double xr = g.pitch_mm * (i * cr - j * snr), yr = g.pitch_mm * (i * snr + j * cr);
    const double X = xr + dxm - g.roi_x_mm, Y = yr + dym - g.roi_y_mm, H = g.height_mm + dh;
    const double D = sqrt(X * X + Y * Y + H * H);
    sr = Y / D / g.lambda * g.inv_dk;
    sc = X / D / g.lambda * g.inv_dk;
    const double D3 = g.lambda * D * D * D;
    // d(k_x, k_y)/d(X, Y, H), then d(X, Y, H)/d(shift_x, shift_y, rot, dh)
    const double kxX = (D * D - X * X) / D3, kxY = -X * Y / D3, kxH = -X * H / D3;
    const double kyX = -X * Y / D3, kyY = (D * D - Y * Y) / D3, kyH = -Y * H / D3;
    sl.J[0] = kyX * g.inv_dk;                       // s_row / shift_x
    sl.J[1] = kyY * g.inv_dk;                       // s_row / shift_y
    sl.J[2] = (-kyX * yr + kyY * xr) * g.inv_dk;    // s_row / rot
    sl.J[3] = kyH * g.inv_dk;                       // s_row / dh
    sl.J[4] = kxX * g.inv_dk;
    sl.J[5] = kxY * g.inv_dk;
    sl.J[6] = (-kxX * yr + kxY * xr) * g.inv_dk;
    sl.J[7] = kxH * g.inv_dk;
  }
  const double wr = base + sr, wc = base + sc;
  int fr = (int)floor(wr), fc = (int)floor(wc);
  sl.ay = (float)(wr - fr);
  sl.ax = (float)(wc - fc);
  const int lo = 0, hi = g.M - g.N - 1;
  if (fr < lo || fr > hi || fc < lo || fc > hi) {
    atomicAdd(oob, 1);
    fr = min(max(fr, lo), hi);
    fc = min(max(fc, lo), hi);
  }
  sl.fr = fr;
  sl.fc = fc;
  out[b] = sl;
}

// Bilinear sample of the spectrum at window (fr, fc) + (ky, kx) + (ay, ax).
__device__ __forceinline__ void taps4(const float2* __restrict__ O, int M, int r, int c,
                                      float2& t00, float2& t01, float2& t10, float2& t11) {
  const float2* p = O + (size_t)r * M + c;
  t00 = p[0];
  t01 = p[1];
  t10 = p[M];
  t11 = p[M + 1];
}

__device__ __forceinline__ float2 blend(float2 t00, float2 t01, float2 t10, float2 t11, float ay,
                                        float ax) {
  const float w00 = (1.f - ay) * (1.f - ax), w01 = (1.f - ay) * ax;
  const float w10 = ay * (1.f - ax), w11 = ay * ax;
  return make_float2(w00 * t00.x + w01 * t01.x + w10 * t10.x + w11 * t11.x,
                     w00 * t00.y + w01 * t01.y + w10 * t10.y + w11 * t11.y);
}

template <int N>
__global__ void __launch_bounds__(kRowThreads)
rows_forward_sub(const float2* __restrict__ O, const float2* __restrict__ P, Batch bt, Disk dk,
                 const SubSlot* __restrict__ sub, int chunks, float2* __restrict__ X,
                 const float2* __restrict__ tw) {
  constexpr int T = RowPlan<N>::T;
  constexpr int E = N / T;
  constexpr int L = kRowThreads / T;
  __shared__ float2 lds[L * RowLds<N>::kStride];
  __shared__ float2 lds_tw[N];
  int b, c;
  if (!xcd_map(blockIdx.x, chunks, bt.B, b, c)) return;
  stage_twiddles<N>(lds_tw, tw);
  const int line = threadIdx.x / T, t = threadIdx.x % T;
  const int rr = c * L + line;
  const bool active = rr < dk.nrows;
  const int ky = dk.ky_lo + (active ? rr : 0);
  const int2 ext = disk_extent<N>(dk, ky);
  const SubSlot sl = sub[b];
  const float2* prow = P + (size_t)ky * N;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kx0 = half_shift<N>(t + m * T);
    const int kx = min(max(kx0, ext.x), ext.y);
    float2 t00, t01, t10, t11;
    taps4(O, bt.M, sl.fr + ky, sl.fc + kx, t00, t01, t10, t11);
    const float2 C = blend(t00, t01, t10, t11, sl.ay, sl.ax);
    const bool in = active && kx0 >= ext.x && kx0 <= ext.y;
    v[m] = in ? cmul(C, prow[kx]) : make_float2(0.f, 0.f);
  }
  RowPlan<N>::template run<+1>(v, t, lds + line * RowLds<N>::kStride,
                              [](int n) { return RowLds<N>::at(n); }, lds_tw);
  if (active) {
    float2* xr = X + ((size_t)b * N + ky) * N;
#pragma unroll
    for (int m = 0; m < E; ++m) xr[t + m * T] = v[m];
  }
}

constexpr int kSubPar = kPar + 2;   // pupil moments, then dL/ds (row, col)

template <int N>
__global__ void __launch_bounds__(kRowThreads)
rows_backward_sub(float2* __restrict__ X, const float2* __restrict__ O,
                  const float2* __restrict__ P, Batch bt, Disk dk, PupilGeom pg,
                  const SubSlot* __restrict__ sub, int chunks, double* __restrict__ part,
                  const float* __restrict__ kappa_tab, const float2* __restrict__ tw) {
  constexpr int T = RowPlan<N>::T;
  constexpr int E = N / T;
  constexpr int L = kRowThreads / T;
  __shared__ float2 lds[L * RowLds<N>::kStride];
  __shared__ float2 lds_tw[N];
  int b, c;
  const bool live = xcd_map(blockIdx.x, chunks, bt.B, b, c);
  if (live) stage_twiddles<N>(lds_tw, tw);
  const int line = threadIdx.x / T, t = threadIdx.x % T;
  const int rr = c * L + line;
  const bool active = rr < dk.nrows;
  const int ky = dk.ky_lo + (active ? rr : 0);
  float acc[kSubPar];
#pragma unroll
  for (int j = 0; j < kSubPar; ++j) acc[j] = 0.f;
  if (live) {
    float2* xr = X + ((size_t)b * N + ky) * N;
    const int2 ext = disk_extent<N>(dk, ky);
    const SubSlot sl = sub[b];
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = xr[t + m * T];
    RowPlan<N>::template run<-1>(v, t, lds + line * RowLds<N>::kStride,
                                [](int n) { return RowLds<N>::at(n); }, lds_tw);
    if (active) {
      const float2* prow = P + (size_t)ky * N;
      const int uy = ky - N / 2;
      const float ir = (float)pg.inv_r;
      float S0 = 0.f, S1 = 0.f, S2 = 0.f, S3 = 0.f, S4 = 0.f, SK = 0.f, GY = 0.f, GX = 0.f;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int kx = half_shift<N>(t + m * T);
        if (kx >= ext.x && kx <= ext.y) {
          const float2 g = v[m];
          const float2 p = prow[kx];
          const float2 gc = cmulc(p, g);                      // g_C = conj(P) g_Phi
          xr[kx] = gc;
          float2 t00, t01, t10, t11;
          taps4(O, bt.M, sl.fr + ky, sl.fc + kx, t00, t01, t10, t11);
          const float2 C = blend(t00, t01, t10, t11, sl.ay, sl.ax);
          const float2 gp = cmulc(C, g);                      // conj(C) g_Phi
          const float gth = gp.y * p.x - gp.x * p.y;          // Im(g_P conj(P))
          const int ux = kx - N / 2;
          const float xx = (float)ux * ir;
          const float gx = gth * xx, gx2 = gx * xx, gx3 = gx2 * xx;
          S0 += gth; S1 += gx; S2 += gx2; S3 += gx3; S4 += gx3 * xx;
          SK += gth * kappa_tab[ux * ux + uy * uy];
          // dC/da_y and dC/da_x of the bilinear blend
          const float2 dy = make_float2((1.f - sl.ax) * (t10.x - t00.x) + sl.ax * (t11.x - t01.x),
                                        (1.f - sl.ax) * (t10.y - t00.y) + sl.ax * (t11.y - t01.y));
          const float2 dx = make_float2((1.f - sl.ay) * (t01.x - t00.x) + sl.ay * (t11.x - t10.x),
                                        (1.f - sl.ay) * (t01.y - t00.y) + sl.ay * (t11.y - t10.y));
          GY += gc.x * dy.x + gc.y * dy.y;
          GX += gc.x * dx.x + gc.y * dx.y;
        }
      }
      const float y = (float)uy * ir, y2 = y * y, y3 = y2 * y, y4 = y3 * y;
      acc[0] = S0;  acc[1] = S1;  acc[2] = S0 * y;
      acc[3] = S2;  acc[4] = S1 * y;  acc[5] = S0 * y2;
      acc[6] = S3;  acc[7] = S2 * y;  acc[8] = S1 * y2;  acc[9] = S0 * y3;
      acc[10] = S4; acc[11] = S3 * y; acc[12] = S2 * y2; acc[13] = S1 * y3; acc[14] = S0 * y4;
      acc[15] = SK;
      acc[16] = GY;
      acc[17] = GX;
    }
  }
  block_partials<kSubPar>(acc, part);
}

// g_O += sum over slots and taps of w_t patch_b(p - f_b - t); one thread per
// 4 consecutive pixels, so every pixel is written by one thread (no atomics).
template <int N>
__global__ void __launch_bounds__(256)
gather_dense(const float2* __restrict__ X, Batch bt, Disk dk, const SubSlot* __restrict__ sub,
             float2* __restrict__ gO) {
  const int tiles_per_row = bt.M / 32;
  const int tr0 = (blockIdx.x / tiles_per_row) * 32, tc0 = (blockIdx.x % tiles_per_row) * 32;
  const int r = tr0 + (threadIdx.x >> 3);
  const int c0 = tc0 + (threadIdx.x & 7) * 4;
  float2 g[4];
  bool any = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) g[q] = make_float2(0.f, 0.f);
  for (int b = 0; b < bt.B; ++b) {
    const SubSlot sl = sub[b];
    // disk box of the window, one pixel wider for the taps
    if (tr0 + 31 < sl.fr + dk.ky_lo || tr0 > sl.fr + dk.ky_hi + 1 ||
        tc0 + 31 < sl.fc + dk.ky_lo || tc0 > sl.fc + dk.ky_hi + 1)
      continue;
    any = true;
    const float wts[4] = {(1.f - sl.ay) * (1.f - sl.ax), (1.f - sl.ay) * sl.ax,
                          sl.ay * (1.f - sl.ax), sl.ay * sl.ax};
#pragma unroll
    for (int tap = 0; tap < 4; ++tap) {
      const int dy = tap >> 1, dxx = tap & 1;
      const int ky = r - sl.fr - dy;
      const int kyc = min(max(ky, dk.ky_lo), dk.ky_hi);
      const int2 e = disk_extent<N>(dk, kyc);
      const float2* xr = X + ((size_t)b * N + kyc) * N;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kx = c0 + q - sl.fc - dxx;
        const float2 val = xr[min(max(kx, e.x), e.y)];
        if (ky == kyc && kx >= e.x && kx <= e.y) {
          g[q].x += wts[tap] * val.x;
          g[q].y += wts[tap] * val.y;
        }
      }
    }
  }
  if (!any) return;
  float2* out = gO + (size_t)r * bt.M + c0;
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = make_float2(out[q].x + g[q].x, out[q].y + g[q].y);
}

// Final sums of a loss-and-gradient call, in fixed order (one workgroup).
struct ReduceArgs {
  const double* col_part;    // [col_wgs][2]: loss, sum e |psi| (intensity loss: e |psi|^2)
  int col_wgs, col_chunks;
  const double* row_part;    // [row_wgs][kSubPar]
  int row_wgs, row_chunks;
  const SubSlot* sub;
  Batch bt;
  const float* gamma;        // [n_led] or NULL
  double* loss;              // += (nullable)
  double* g_par;             // [16] += (nullable)
  double* g_geom;            // [4] += (nullable)
  double* g_gamma;           // [n_led] += (nullable)
};

__global__ void __launch_bounds__(256) loss_grad_reduce(ReduceArgs a) {
  __shared__ double red[256];
  __shared__ double mom[kPar];
  __shared__ double gs[kMaxSlots][2];
  __shared__ double ea[kMaxSlots];
  const int tid = threadIdx.x;
  // pupil moments: thread (j, lane) sums workgroups lane, lane + 16, ...
  {
    const int j = tid & (kPar - 1), lane = tid / kPar;
    double s = 0.0;
    for (int w = lane; w < a.row_wgs; w += 256 / kPar) s += a.row_part[(size_t)w * kSubPar + j];
    red[tid] = s;
    __syncthreads();
    if (tid < kPar) {
      double m = 0.0;
      for (int k = 0; k < 256 / kPar; ++k) m += red[k * kPar + tid];
      mom[tid] = m;
    }
    __syncthreads();
  }
  // per slot: dL/ds from the row pass, sum e |psi| from the column pass
  if (tid < a.bt.B) {
    double gy = 0.0, gx = 0.0, e = 0.0;
    for (int w = 0; w < a.row_wgs; ++w) {
      int b, c;
      if (xcd_map(w, a.row_chunks, a.bt.B, b, c) && b == tid) {
        gy += a.row_part[(size_t)w * kSubPar + kPar];
        gx += a.row_part[(size_t)w * kSubPar + kPar + 1];
      }
    }
    for (int w = 0; w < a.col_wgs; ++w) {
      int b, c;
      if (xcd_map(w, a.col_chunks, a.bt.B, b, c) && b == tid) e += a.col_part[(size_t)w * 2 + 1];
    }
    gs[tid][0] = gy;
    gs[tid][1] = gx;
    ea[tid] = e;
  }
  __syncthreads();
  if (tid == 0) {
    if (a.loss) {
      double l = 0.0;
      for (int w = 0; w < a.col_wgs; ++w) l += a.col_part[(size_t)w * 2];
      *a.loss += l;
    }
    if (a.g_geom) {
      double gg[4] = {0.0, 0.0, 0.0, 0.0};
      for (int b = 0; b < a.bt.B; ++b)
        for (int p = 0; p < 4; ++p)
          gg[p] += a.sub[b].J[p] * gs[b][0] + a.sub[b].J[4 + p] * gs[b][1];
      for (int p = 0; p < 4; ++p) a.g_geom[p] += gg[p];
    }
    if (a.g_gamma) {
      for (int b = 0; b < a.bt.B; ++b) {
        const int led = a.bt.led[b];
        if (a.bt.intensity) {
          a.g_gamma[led] += 2.0 * ea[b];
        } else {
          const double sg = a.gamma ? sqrt((double)a.gamma[led]) : 1.0;
          a.g_gamma[led] += ea[b] / sg;
        }
      }
    }
  }
  if (a.g_par && tid < kPar) {
    double g = mom[kZern];
    if (tid < kZern) {
      g = 0.0;
      for (int k = 0; k < kMono; ++k) g += kZernMono[tid][k] * mom[k];
    }
    a.g_par[tid] += g;
  }
}

}  // namespace fpm
