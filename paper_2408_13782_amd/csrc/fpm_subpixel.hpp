// fpm_subpixel.hpp - the multi-parameter path: sub-pixel LED offsets from the
// LED-array geometry, bilinear crop and its adjoint, gradients with respect to
// the geometry and the LED intensities (paper Sec. 2.1 k_m and Eq. 3; Sec. 2.2).
//
// The forward row pass derives the offsets of its batch slots, in FP64, from
// the nominal grid and the current geometry errors (subslot_of), so no launch
// is spent on them, and stores them for the later kernels of the call.
// Launch order of one loss-and-gradient call:
//   pupil_build        P from the Zernike coefficients and defocus
//   rows_forward_sub   bilinear crop C_b (4 taps) * P, inverse DFT of disk rows
//   cols<.., kGamma>   as in the nearest path, plus sum e |psi| per workgroup
//   rows_backward_sub  forward DFT of disk rows; patch conj(P) g_Phi; pupil
//                      moments; dL/ds_b = sum Re(conj(g_C) dC/ds) partials
//   gather_dense       g_O += sum_b sum_taps w_t patch_b (each pixel one thread)
//   loss_grad_reduce   loss, Zernike/defocus, geometry (J_b^T dL/ds_b), gamma
// and of one fused multi-parameter step: rows_forward_sub, cols,
// rows_backward_sub, update_multi (Adam on the spectrum over the whole HR grid,
// on the Zernike coefficients, defocus and geometry, and the pupil rebuild).
#pragma once
#include <hip/hip_runtime.h>

#include "fft_line.hpp"
#include "fpm_aux.hpp"
#include "fpm_kernels.hpp"
#include "fpm_optics.hpp"

namespace fpm {

// One batch slot of the sub-pixel path: window corner (integer part), the
// fractional part, and ds/d(shift_x, shift_y, rot, dh) as rows (s_row, s_col).
struct SubSlot {
  int fr, fc;
  float ay, ax;
  double J[8];
  int clamped;   // the window was clamped into the HR grid
};

// LED-array geometry (nominal grid plus learned errors) and optics constants.
struct GeomArgs {
  int n_side;
  double pitch_mm, height_mm, roi_x_mm, roi_y_mm;
  double base_dx, base_dy, base_rot, base_dh;   // nominal errors of the grid description
  double inv_dk, lambda;
  int N, M;
};

// Offsets of batch slot b. With geom == NULL the plan's integer offsets are
// used (zero fractional part, zero Jacobian). A window that would leave the HR
// grid (with one pixel of bilinear margin) is clamped; *clamped tells.
__device__ inline SubSlot subslot_of(const GeomArgs& g, const double* __restrict__ geom,
                                     const Batch& bt, int b, bool* clamped) {
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
  *clamped = fr < lo || fr > hi || fc < lo || fc > hi;
  sl.fr = min(max(fr, lo), hi);
  sl.fc = min(max(fc, lo), hi);
  return sl;
}

// The offsets of every slot of the batch into LDS, from the copies that
// rows_forward_sub stored (threads b < B load slot b).
__device__ __forceinline__ void subslots_to_lds(const SubSlot* __restrict__ stored,
                                                const Batch& bt, SubSlot* sh) {
  if ((int)threadIdx.x < bt.B) sh[threadIdx.x] = stored[threadIdx.x];
  __syncthreads();
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

// Shape of rows_forward_sub: at N = 512, 64 threads per row (two rows per
// workgroup) take 1.8 us off the pass against 32.
template <int N> struct SubFwdRow { static constexpr int T = RowT<N>::value, threads = kRowThreads; };
template <> struct SubFwdRow<512> { static constexpr int T = 64, threads = kRowThreads; };

template <int N>
__global__ void __launch_bounds__(SubFwdRow<N>::threads)
rows_forward_sub(const float2* __restrict__ O, const float2* __restrict__ P, Batch bt, Disk dk,
                 GeomArgs ga, const double* __restrict__ geom, int* __restrict__ oob,
                 SubSlot* __restrict__ sub_out, const SubSlot* __restrict__ pre, int chunks,
                 float2* __restrict__ X, const float2* __restrict__ tw) {
  constexpr int T = SubFwdRow<N>::T;
  constexpr int E = N / T;
  constexpr int L = SubFwdRow<N>::threads / T;
  __shared__ float2 lds[L * RowLds<N>::kStride];
  __shared__ float2 lds_tw[N];
  int b, c;
  if (!xcd_map(blockIdx.x, chunks, bt.B, b, c)) return;
  const int line = threadIdx.x / T, t = threadIdx.x % T;
  const int rr = c * L + line;
  const bool active = rr < dk.nrows;
  const int ky = dk.ky_lo + (active ? rr : 0);
  const int2 ext = disk_extent<N>(dk, ky);
  // The loads that do not depend on the slot's offsets (pupil row, twiddles)
  // go out first; the first wave then derives the offsets (a chain of FP64
  // operations that the second wave would only repeat) and shares them
  // through LDS, and the taps are loaded once they are known.
  constexpr int kThreads = SubFwdRow<N>::threads;
  constexpr int K = (N + kThreads - 1) / kThreads;
  float2 twr[K];
#pragma unroll
  for (int k = 0; k < K; ++k) twr[k] = tw[min((int)threadIdx.x + k * kThreads, N - 1)];
  const float2* prow = P + (size_t)ky * N;
  float2 pv[E];
#pragma unroll
  for (int m = 0; m < E; ++m) pv[m] = prow[min(max(half_shift<N>(t + m * T), ext.x), ext.y)];
  __shared__ int4 slot;   // fr, fc and the bits of ay, ax
  if (pre) {
    // derived by the previous step's update kernel from the same geometry
    if (threadIdx.x == 0) {
      const SubSlot& s0 = pre[b];
      slot = make_int4(s0.fr, s0.fc, __float_as_int(s0.ay), __float_as_int(s0.ax));
      if (c == 0 && s0.clamped && oob) atomicAdd(oob, 1);
    }
  } else if (threadIdx.x < 64) {
    bool clamped;
    SubSlot s0 = subslot_of(ga, geom, bt, b, &clamped);
    if (threadIdx.x == 0) {
      slot = make_int4(s0.fr, s0.fc, __float_as_int(s0.ay), __float_as_int(s0.ax));
      if (c == 0) {
        if (clamped && oob) atomicAdd(oob, 1);
        s0.clamped = clamped;
        sub_out[b] = s0;   // for the later kernels of the call
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) lds_tw[min((int)threadIdx.x + k * kThreads, N - 1)] = twr[k];
  __syncthreads();
  const int4 si = slot;
  const int sfr = si.x, sfc = si.y;
  const float say = __int_as_float(si.z), sax = __int_as_float(si.w);
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kx0 = half_shift<N>(t + m * T);
    const int kx = min(max(kx0, ext.x), ext.y);
    float2 t00, t01, t10, t11;
    taps4(O, bt.M, sfr + ky, sfc + kx, t00, t01, t10, t11);
    const float2 C = blend(t00, t01, t10, t11, say, sax);
    const bool in = active && kx0 >= ext.x && kx0 <= ext.y;
    v[m] = in ? cmul(C, pv[m]) : make_float2(0.f, 0.f);
  }
  PlanT<N, T>::template run<+1>(v, t, lds + line * RowLds<N>::kStride,
                              [](int n) { return RowLds<N>::at(n); }, lds_tw);
  if (active) {
    float2* xr = X + ((size_t)b * N + ky) * N;
#pragma unroll
    for (int m = 0; m < E; ++m) xr[t + m * T] = v[m];
  }
}

constexpr int kSubPar = kPar + 2;   // pupil moments, then dL/ds (row, col)

// Threads per workgroup of rows_backward_sub: from N = 512 up, twice those of
// the other row passes (eight rows per workgroup), which halves the partials
// that every pupil workgroup of the update sums (2.9 us less in update_multi
// against 0.7 us more here at N = 512, B = 32).
template <int N> struct SubBwdThreads { static constexpr int value = N >= 512 ? 2 * kRowThreads : kRowThreads; };

template <int N, int kThreads = SubBwdThreads<N>::value>
__global__ void __launch_bounds__(kThreads)
rows_backward_sub(float2* __restrict__ X, const float2* __restrict__ O,
                  const float2* __restrict__ P, Batch bt, Disk dk, PupilGeom pg,
                  const SubSlot* __restrict__ stored, int chunks, double* __restrict__ part,
                  const float* __restrict__ kappa_tab, const float2* __restrict__ tw) {
  constexpr int T = RowPlan<N>::T;
  constexpr int E = N / T;
  constexpr int L = kThreads / T;
  __shared__ float2 lds[L * RowLds<N>::kStride];
  __shared__ float2 lds_tw[N];
  int b, c;
  const bool live = xcd_map(blockIdx.x, chunks, bt.B, b, c);
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
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = xr[t + m * T];
    // the slot's offsets as rows_forward_sub derived and stored them (the taps
    // are read only after the transform, so this load is off the critical path;
    // deriving them here again cost each workgroup a chain of FP64 operations
    // before its first load)
    const SubSlot sl = stored[b];
    stage_twiddles_after_loads<N, kThreads>(lds_tw, tw);
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
  // (a buffer for this workgroup's waves only: at N = 512 the pass then fits
  // four workgroups per CU in LDS instead of three)
  block_partials<kSubPar, (kThreads + 63) / 64>(acc, part);
}

// Window corner and fractional offsets of every batch slot, compact, in LDS,
// and the mask of the slots whose window (disk box, one pixel wider for the
// taps) meets the 32 x 32 tile at (tr0, tc0). Uniform over the workgroup.
struct Corner {
  int fr, fc;
  float ay, ax;
};

__device__ __forceinline__ unsigned long long tile_slots(const SubSlot* __restrict__ stored,
                                                          const Batch& bt, const Disk& dk,
                                                          int tr0, int tc0, Corner* cs) {
  // the B <= 64 slots are served by the first wave; its ballot is the mask
  __shared__ unsigned long long mask;
  if (threadIdx.x < 64) {
    bool meets = false;
    if ((int)threadIdx.x < bt.B) {
      const SubSlot sl = stored[threadIdx.x];
      cs[threadIdx.x] = Corner{sl.fr, sl.fc, sl.ay, sl.ax};
      meets = !(tr0 + 31 < sl.fr + dk.ky_lo || tr0 > sl.fr + dk.ky_hi + 1 ||
                tc0 + 31 < sl.fc + dk.ky_lo || tc0 > sl.fc + dk.ky_hi + 1);
    }
    const unsigned long long m = __ballot(meets);
    if (threadIdx.x == 0) mask = m;
  }
  __syncthreads();
  return mask;
}

// Bilinear adjoint at the 4 pixels of a tile thread (row r, columns
// c0 + tile_col(q)): the sum, over the slots of `hit` in batch order and their
// 4 taps, of w_t patch_b(p - f_b - t).
template <int N>
__device__ __forceinline__ void gather_bilinear(const float2* __restrict__ X, const Disk& dk,
                                                const Corner* cs, unsigned long long hit,
                                                int r, int c0, float2 (&g)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) g[q] = make_float2(0.f, 0.f);
  while (hit) {
    const int b = __ffsll((long long)hit) - 1;
    hit &= hit - 1;
    const Corner sl = cs[b];
    const float wts[4] = {(1.f - sl.ay) * (1.f - sl.ax), (1.f - sl.ay) * sl.ax,
                          sl.ay * (1.f - sl.ax), sl.ay * sl.ax};
    // tap (dy, dx) of pixel q reads patch column c0 + tile_col(q) - fc - dx:
    // the two pixels of a column pair share their middle column, so each
    // patch row needs 3 values per pair (12 loads per slot instead of 16)
    float2 val[2][2][3];
    bool ok[2][2][3];
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const int ky = r - sl.fr - dy;
      const int kyc = min(max(ky, dk.ky_lo), dk.ky_hi);
      const int2 e = disk_extent<N>(dk, kyc);
      const float2* xr = X + ((size_t)b * N + kyc) * N;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const int kx = c0 + 16 * p - sl.fc + j - 1;
          val[dy][p][j] = xr[min(max(kx, e.x), e.y)];
          ok[dy][p][j] = ky == kyc && kx >= e.x && kx <= e.y;
        }
      }
    }
    // accumulated per pixel in tap order
#pragma unroll
    for (int tap = 0; tap < 4; ++tap) {
      const int dy = tap >> 1, dxx = tap & 1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int p = q >> 1, j = (q & 1) - dxx + 1;
        if (ok[dy][p][j]) {
          g[q].x += wts[tap] * val[dy][p][j].x;
          g[q].y += wts[tap] * val[dy][p][j].y;
        }
      }
    }
  }
}

// g_O += the batch's bilinear adjoint; one thread per 4 pixels of a 32 x 32
// tile, so every pixel is written by one thread (no atomics).
template <int N>
__global__ void __launch_bounds__(256)
gather_dense(const float2* __restrict__ X, Batch bt, Disk dk,
             const SubSlot* __restrict__ stored, float2* __restrict__ gO) {
  __shared__ Corner cs[kMaxSlots];
  const int tiles_per_row = bt.M / 32;
  const int tr0 = (blockIdx.x / tiles_per_row) * 32, tc0 = (blockIdx.x % tiles_per_row) * 32;
  const unsigned long long hit = tile_slots(stored, bt, dk, tr0, tc0, cs);
  if (!hit) return;
  const int r = tr0 + (threadIdx.x >> 3);
  const int c0 = tc0 + (threadIdx.x & 7) * 2;
  float2 g[4];
  gather_bilinear<N>(X, dk, cs, hit, r, c0, g);
  float2* out = gO + (size_t)r * bt.M + c0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float2& o = out[tile_col(q)];
    o = make_float2(o.x + g[q].x, o.y + g[q].y);
  }
}

// Final sums of a loss-and-gradient call, in fixed order (one workgroup).
struct ReduceArgs {
  const double* col_part;    // [col_wgs][2]: loss, sum e |psi| (intensity loss: e |psi|^2)
  int col_wgs, col_chunks;
  const double* row_part;    // [row_wgs][kSubPar]
  int row_wgs, row_chunks;
  const SubSlot* sub;        // [B] offsets stored by rows_forward_sub
  Batch bt;
  const float* gamma;        // [n_led] or NULL
  double* loss;              // += (nullable)
  double* g_par;             // [16] += (nullable)
  double* g_geom;            // [4] += (nullable)
  double* g_gamma;           // [n_led] += (nullable)
};

__global__ void __launch_bounds__(256) loss_grad_reduce(ReduceArgs a) {
  __shared__ SubSlot sub[kMaxSlots];
  subslots_to_lds(a.sub, a.bt, sub);
  __shared__ double red[256];
  __shared__ double mom[kPar];
  __shared__ double gs[kMaxSlots][2];
  __shared__ double ea[kMaxSlots];
  const int tid = threadIdx.x;
  if (a.loss) add_batch_loss(a.col_part, a.col_wgs, a.loss, 2);   // the whole workgroup
  // pupil moments: thread (j, lane) sums workgroups lane, lane + 16, ...
  {
    const int j = tid & (kPar - 1), lane = tid / kPar;
    const int cnt = lane < a.row_wgs ? (a.row_wgs - lane + 256 / kPar - 1) / (256 / kPar) : 0;
    red[tid] = ordered_sum(a.row_part + (size_t)lane * kSubPar + j, cnt, (256 / kPar) * kSubPar);
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
    // the workgroups of slot tid are xcd_wg(tid, c) = xcd_wg(tid, 0) + 8 c
    const double* rp = a.row_part + (size_t)xcd_wg(tid, 0, a.row_chunks) * kSubPar;
    const double gy = ordered_sum<32>(rp + kPar, a.row_chunks, kXcds * kSubPar);
    const double gx = ordered_sum<32>(rp + kPar + 1, a.row_chunks, kXcds * kSubPar);
    const double e = ordered_sum(a.col_part + (size_t)xcd_wg(tid, 0, a.col_chunks) * 2 + 1,
                                 a.col_chunks, kXcds * 2);
    gs[tid][0] = gy;
    gs[tid][1] = gx;
    ea[tid] = e;
  }
  __syncthreads();
  if (tid == 0) {
    if (a.g_geom) {
      double gg[4] = {0.0, 0.0, 0.0, 0.0};
      for (int b = 0; b < a.bt.B; ++b)
        for (int p = 0; p < 4; ++p)
          gg[p] += sub[b].J[p] * gs[b][0] + sub[b].J[4 + p] * gs[b][1];
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

// ---------------------------------------------------------------------------
// Fused multi-parameter step: the learned scalars of step t live in a
// parameter block (double-buffered by step parity), so that every kernel of a
// step reads the geometry the step started with while its last kernel writes
// the next one.

struct MultiParams {
  float c[kPar], m_c[kPar], v_c[kPar];   // Zernike 0..14, defocus at index 15
  double g[4], m_g[4], v_g[4];           // LED-array geometry errors and their moments
};

// Copy the caller's scalar state into a parameter block, or back.
struct MultiState {
  float* coeffs; float* m_c; float* v_c;
  float* z; float* m_z; float* v_z;
  double* g; double* m_g; double* v_g;
};

__global__ void multi_params_io(MultiState s, MultiParams* __restrict__ blk, int to_block) {
  const int i = threadIdx.x;
  if (i < kPar) {
    float* pc = i < kZern ? s.coeffs + i : s.z;
    float* pm = i < kZern ? s.m_c + i : s.m_z;
    float* pv = i < kZern ? s.v_c + i : s.v_z;
    if (to_block) {
      blk->c[i] = *pc;
      blk->m_c[i] = *pm;
      blk->v_c[i] = *pv;
    } else {
      *pc = blk->c[i];
      *pm = blk->m_c[i];
      *pv = blk->v_c[i];
    }
  } else if (i < kPar + 4) {
    const int k = i - kPar;
    if (to_block) {
      blk->g[k] = s.g[k];
      blk->m_g[k] = s.m_g[k];
      blk->v_g[k] = s.v_g[k];
    } else {
      s.g[k] = blk->g[k];
      s.m_g[k] = blk->m_g[k];
      s.v_g[k] = blk->v_g[k];
    }
  }
}

// Mark the 32 x 32 HR tiles whose Adam moments are not all zero (the tiles a
// multi-parameter run must keep updating even when no window of the batch
// covers them). One workgroup per tile.
__global__ void __launch_bounds__(256) tiles_with_moments(const float* __restrict__ mO,
                                                          const float* __restrict__ vO, int M,
                                                          int* __restrict__ flags) {
  const int tpr = M / 32;
  const int r = (blockIdx.x / tpr) * 32 + (threadIdx.x >> 3);
  const int c0 = (blockIdx.x % tpr) * 32 + (threadIdx.x & 7) * 4;
  const size_t f = ((size_t)r * M + c0) * 2;
  const float4* pm = reinterpret_cast<const float4*>(mO + f);
  const float4* pv = reinterpret_cast<const float4*>(vO + f);
  bool nz = false;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float4 m = pm[h], v = pv[h];
    nz = nz || m.x != 0.f || m.y != 0.f || m.z != 0.f || m.w != 0.f || v.x != 0.f ||
         v.y != 0.f || v.z != 0.f || v.w != 0.f;
  }
  nz = __syncthreads_or(nz);
  if (threadIdx.x == 0) flags[blockIdx.x] = nz ? 1 : 0;
}

struct MultiUpdateArgs {
  int M;
  int* tile_flags;                    // [(M/32)^2] 1: moments may be non-zero
  float* O; float* mO; float* vO;
  AdamCoef c;
  const float2* X; Batch bt; Disk dk;
  const SubSlot* sub;                 // [B] offsets stored by rows_forward_sub
  const double* loss_part; int n_loss; double* loss;
  const double* row_part; int n_rows, row_chunks;
  const MultiParams* cur; MultiParams* next;
  ScalarAdam sa;
  int learn_geom; double lr_geom[4];
  double* g_par; double* g_geom;      // diagnostics, += (nullable)
  PupilGeom pg; float2* P;
  // the next step's batch: its slot offsets from the new geometry (nullable)
  SubSlot* next_sub; Batch bt_next; GeomArgs ga;
};

// Last launch of a fused multi-parameter step:
//  tile workgroups (after the pupil ones): Adam over every 32 x 32 tile of the
//    HR grid (the union of windows moves with the geometry), the gradient
//    gathered bilinearly from the batch's patches in batch order;
//  pupil workgroups: sum the moment and offset-gradient partials in a fixed
//    order, Adam on the Zernike coefficients, defocus and geometry (all of
//    them compute the same numbers, workgroup 0 writes the next parameter
//    block and, with next_sub, the next step's slot offsets derived from the
//    new geometry), rebuild their share of the pupil;
//  the workgroup after them: adds the batch loss to *loss.
template <int N>
__global__ void __launch_bounds__(256) update_multi(MultiUpdateArgs a) {
  const int n_pw = pupil_wg_slots(N, a.dk.nrows);
  if ((int)blockIdx.x >= n_pw) {
    __shared__ Corner cs[kMaxSlots];
    const int ti = blockIdx.x - n_pw, tpr = a.M / 32;
    const int tr0 = (ti / tpr) * 32, tc0 = (ti % tpr) * 32;
    // Adam moves a pixel only if its moments or its gradient are non-zero: a tile
    // that no window of this batch covers and whose moments are all zero stays
    // as it is (exactly), and is skipped (the flag is fetched together with the
    // batch's slot data)
    const int flagged = a.tile_flags[ti];
    const unsigned long long hit = tile_slots(a.sub, a.bt, a.dk, tr0, tc0, cs);
    if (!hit && !flagged) return;
    if (hit && !flagged && threadIdx.x == 0) a.tile_flags[ti] = 1;
    const int r = tr0 + (threadIdx.x >> 3);
    const int c0 = tc0 + (threadIdx.x & 7) * 2;
    const size_t f = ((size_t)r * a.M + c0) * 2;
    float4* po = reinterpret_cast<float4*>(a.O + f);
    float4* pm = reinterpret_cast<float4*>(a.mO + f);
    float4* pv = reinterpret_cast<float4*>(a.vO + f);
    float4 o[2], m[2], v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {   // in flight while the gradient is gathered
      o[h] = po[8 * h];
      m[h] = pm[8 * h];
      v[h] = pv[8 * h];
    }
    float2 g[4];
    gather_bilinear<N>(a.X, a.dk, cs, hit, r, c0, g);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      adam1(o[h].x, m[h].x, v[h].x, g[2 * h].x, a.c);
      adam1(o[h].y, m[h].y, v[h].y, g[2 * h].y, a.c);
      adam1(o[h].z, m[h].z, v[h].z, g[2 * h + 1].x, a.c);
      adam1(o[h].w, m[h].w, v[h].w, g[2 * h + 1].y, a.c);
      store_next4<N>(po + 8 * h, o[h]);
      store_next4<N>(pm + 8 * h, m[h]);
      store_next4<N>(pv + 8 * h, v[h]);
    }
    return;
  }
  const int pw = blockIdx.x;
  const int n_pupil = pupil_wg_count(N, a.dk.nrows);
  if (pw == n_pupil) {   // the loss workgroup
    if (a.loss) add_batch_loss(a.loss_part, a.n_loss, a.loss);
    return;
  }
  if (pw > n_pupil) return;   // padding
  __shared__ double red[256];
  __shared__ double gsum[kPar];
  __shared__ double gs[kMaxSlots][2];
  __shared__ double gg[4];
  __shared__ float nextc[3][kPar];
  __shared__ double nextg[3][4];
  // pupil moments: thread (j, lane) sums partials lane, lane + 16, ...
  {
    const int j = threadIdx.x & (kPar - 1), lane = threadIdx.x / kPar;
    const int cnt = lane < a.n_rows ? (a.n_rows - lane + 256 / kPar - 1) / (256 / kPar) : 0;
    red[threadIdx.x] = ordered_sum<24>(a.row_part + (size_t)lane * kSubPar + j, cnt,
                                   (256 / kPar) * kSubPar);
  }
  // offset gradients of each slot, from the workgroups that served it
  if ((int)threadIdx.x < a.bt.B) {
    const double* rp = a.row_part + (size_t)xcd_wg(threadIdx.x, 0, a.row_chunks) * kSubPar;
    const double gy = ordered_sum<24>(rp + kPar, a.row_chunks, kXcds * kSubPar);
    const double gx = ordered_sum<24>(rp + kPar + 1, a.row_chunks, kXcds * kSubPar);
    gs[threadIdx.x][0] = gy;
    gs[threadIdx.x][1] = gx;
  }
  __syncthreads();
  if (threadIdx.x < kPar) {
    double mom = 0.0;
    for (int k = 0; k < 256 / kPar; ++k) mom += red[k * kPar + threadIdx.x];
    gsum[threadIdx.x] = mom;
  }
  if (threadIdx.x == 0) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < a.bt.B; ++b)
      for (int q = 0; q < 4; ++q)
        t[q] += a.sub[b].J[q] * gs[b][0] + a.sub[b].J[4 + q] * gs[b][1];
    for (int q = 0; q < 4; ++q) gg[q] = t[q];
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i < kPar) {
    double g = gsum[kZern];
    if (i < kZern) {
      g = 0.0;
#pragma unroll
      for (int k = 0; k < kMono; ++k) g += kZernMono[i][k] * gsum[k];
    }
    red[i] = g;
    float p = a.cur->c[i], m = a.cur->m_c[i], v = a.cur->v_c[i];
    const bool is_z = i == kZern;
    const bool learn = is_z ? a.sa.learn_z : (a.sa.learn_c && i != 0);   // piston held
    if (learn) {
      const double lr = is_z ? a.sa.lr_z : a.sa.lr_c;
      const double mm = a.sa.b1 * (double)m + (1.0 - a.sa.b1) * g;
      const double vv = a.sa.b2 * (double)v + (1.0 - a.sa.b2) * g * g;
      const double den = sqrt(vv) / a.sa.sqrt_bc2 + a.sa.eps;
      p = (float)((double)p - lr / a.sa.bc1 * mm / den);
      m = (float)mm;
      v = (float)vv;
    }
    nextc[0][i] = p;
    nextc[1][i] = m;
    nextc[2][i] = v;
  } else if (i < kPar + 4) {
    const int k = i - kPar;
    double p = a.cur->g[k], m = a.cur->m_g[k], v = a.cur->v_g[k];
    if (a.learn_geom) {
      const double g = gg[k];
      m = a.sa.b1 * m + (1.0 - a.sa.b1) * g;
      v = a.sa.b2 * v + (1.0 - a.sa.b2) * g * g;
      p -= a.lr_geom[k] / a.sa.bc1 * m / (sqrt(v) / a.sa.sqrt_bc2 + a.sa.eps);
    }
    nextg[0][k] = p;
    nextg[1][k] = m;
    nextg[2][k] = v;
  }
  __syncthreads();
  if (pw == 0) {
    if (i < kPar) {
      a.next->c[i] = nextc[0][i];
      a.next->m_c[i] = nextc[1][i];
      a.next->v_c[i] = nextc[2][i];
      if (a.g_par) a.g_par[i] += red[i];
    } else if (i < kPar + 4) {
      const int k = i - kPar;
      a.next->g[k] = nextg[0][k];
      a.next->m_g[k] = nextg[1][k];
      a.next->v_g[k] = nextg[2][k];
      if (a.g_geom) a.g_geom[k] += gg[k];
    }
    // the next step's forward row pass reads these instead of deriving them
    if (a.next_sub && i < a.bt_next.B) {
      bool clamped;
      SubSlot sl = subslot_of(a.ga, nextg[0], a.bt_next, i, &clamped);
      sl.clamped = clamped;
      a.next_sub[i] = sl;
    }
  }
  // rebuild this workgroup's rows of the pupil from the new parameters
  rebuild_pupil_rows<N, true>(pw, a.dk, a.pg, nextc[0], true, a.P);
}

}  // namespace fpm
