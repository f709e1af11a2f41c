// fpm_fused.hpp - the loss and its adjoint for one random batch in a single
// launch, when an N x N complex64 image fits one CU's LDS (served at N = 64,
// 35 KB of image: there a step of 16 LEDs takes 19.1 us against 23.4 us for the
// three-pass path; at N = 128 one CU per LED measured slower than the split
// passes, 37.6 against 21.2 us, and the split path serves it).
//
// One workgroup per LED of the batch holds that LED's image in LDS and runs
// the three passes of the split path (fpm_kernels.hpp) back to back, with
// workgroup barriers where the split path has kernel boundaries:
//
//   rows     crop C_b = O[w_b + u] on the pupil disk, Phi = C_b P, inverse
//            DFT of each disk row (Eqs. 2-3) -> image rows
//   columns  inverse DFT of each column -> psi; loss and residual
//            (Eqs. 4-5); forward DFT of each column -> image (disk rows)
//   rows     forward DFT of each disk row; the patch conj(P) g_Phi on the
//            disk is stored for the update kernel to gather in batch order;
//            the Zernike/defocus moments of g_theta are reduced in the
//            workgroup
//
// The intermediate never leaves the CU, and a batch is one launch instead of
// three. Every line transform uses its own slots of the image as the exchange
// buffer of its Stockham stages (its values are in registers by then), so the
// image and the twiddles are all the LDS the kernel needs.
//
// Outputs match the split path's: the patch in X[b][ky][kx] on the disk, one
// loss partial and one set of 16 moment partials per workgroup (slot).
#pragma once
#include <hip/hip_runtime.h>

#include "fft_line.hpp"
#include "fpm_kernels.hpp"

namespace fpm {

template <int N> struct Fused {
  static constexpr int T = 8;                    // threads per line transform
  static constexpr int E = N / T;                // elements per thread
  static constexpr int threads = 512;            // 64 lines of 8 threads
  static constexpr int lines = threads / T;      // lines transformed at once
  static constexpr int passes = N / lines;       // row (column) passes over the N rows (columns)
  static constexpr int stride = N + N / 16;      // LDS slots per image row (one pad per 16)
};

template <int N> struct FusedSupported { static constexpr bool value = N == 64; };

// LDS slot of image element (row, col): rows of `stride` slots, one padding
// slot after every 16 columns (the row exchanges' strided writes then hit
// distinct banks; consecutive columns stay consecutive for the column phase).
template <int N>
__device__ __forceinline__ int img_slot(int row, int col) {
  return row * Fused<N>::stride + col + (col >> 4);
}

// Image row served by row-phase line l (0 <= l < N): the disk rows first (line
// l < nrows takes disk row l), then every other row once, so that the lines
// past the disk run their (unused) transforms on rows the column phase never reads.
template <int N>
__device__ __forceinline__ int line_row(const Disk& dk, int l) {
  return l < dk.nrows ? dk.ky_lo + l : (dk.ky_hi + 1 + (l - dk.nrows)) % N;
}

// MODE: kPatch (object only) or kPatchZern (also the pupil-parameter moments).
template <int N, int MODE>
__global__ void __launch_bounds__(Fused<N>::threads)
chain_fused(const float2* __restrict__ O, const float2* __restrict__ P,
            const float* __restrict__ A, const float* __restrict__ gamma, Batch bt, Disk dk,
            PupilGeom pg, float2* __restrict__ X, const float2* __restrict__ tw,
            const float* __restrict__ kappa_tab, double* __restrict__ loss_part,
            double* __restrict__ zpart, float inv_m, int commit,
            const float* __restrict__ staging, ScalarState scal) {
  using F = Fused<N>;
  constexpr int T = F::T, E = F::E, NT = F::threads, L = F::lines, NP = F::passes;
  __shared__ float2 img[N * F::stride];            // the image, rows of `stride` slots
  __shared__ float2 lds_tw[N];
  __shared__ float tot[N][6];                      // per-line moment totals
  __shared__ double msum[16][16];                  // moment partial sums
  if (commit && blockIdx.x == 0) commit_scalars(staging, scal, threadIdx.x);
  const int b = blockIdx.x;
  const int led = bt.led[b];
  const int2 w = bt.win[b];
  const int tid = threadIdx.x;
  const int t = tid % T;                           // thread of a row line
  const int x0 = tid % L, tc = tid / L;            // column (of a pass), thread of the column

  // row line of pass p: its image row, whether it is a disk row, its extent, and
  // a disk row (with extent) for loads at clamped addresses
  struct Line { int ky, kyc; bool active; int2 ext, extc; };
  auto line_of = [&](int p) {
    Line q;
    const int l = p * L + tid / T;
    q.active = l < dk.nrows;
    q.ky = line_row<N>(dk, l);
    q.ext = q.active ? disk_extent<N>(dk, q.ky) : make_int2(N, -1);
    q.kyc = q.active ? q.ky : dk.ky_lo;
    q.extc = q.active ? q.ext : disk_extent<N>(dk, q.kyc);
    return q;
  };

  // the measured amplitudes of the column phase, requested first
  float a_meas[NP][E];
  {
    const float* ab = A + (size_t)led * N * N;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int m = 0; m < E; ++m) a_meas[p][m] = ab[(size_t)(tc + m * T) * N + p * L + x0];
  }
  const float sg = gamma ? sqrtf(gamma[led]) : 1.0f;

  // ---- row phase (inverse): crop times pupil, inverse DFT of each disk row
  // (with one pass, the crop, the pupil and kappa at the thread's columns stay
  // in registers for the forward row phase, which needs them at the same places)
  float2 v[E];
  float2 ov[E], pvv[E];
  float kap0[MODE == kPatchZern && NP == 1 ? E : 1];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const Line q = line_of(p);
    const float2* orow = O + (size_t)(w.x + q.kyc) * bt.M + w.y;
    const float2* prow = P + (size_t)q.kyc * N;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kx = min(max(half_shift<N>(t + m * T), q.extc.x), q.extc.y);
      ov[m] = orow[kx];
      pvv[m] = prow[kx];
      if constexpr (MODE == kPatchZern && NP == 1) {
        const int ux = kx - N / 2, uy = q.kyc - N / 2;
        kap0[m] = kappa_tab[ux * ux + uy * uy];
      }
    }
    if (p == 0) stage_twiddles_after_loads<N, NT>(lds_tw, tw);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kx = half_shift<N>(t + m * T);
      const bool in = q.active && kx >= q.ext.x && kx <= q.ext.y;
      v[m] = in ? cmul(ov[m], pvv[m]) : make_float2(0.f, 0.f);
    }
    const int ky = q.ky;
    PlanT<N, T>::template run<+1>(v, t, img, [ky](int n) { return img_slot<N>(ky, n); }, lds_tw);
    if (q.active) {
#pragma unroll
      for (int m = 0; m < E; ++m) img[img_slot<N>(ky, t + m * T)] = v[m];
    }
  }
  __syncthreads();

  // ---- column phase: inverse DFT, loss and residual, forward DFT of each column
  float acc = 0.f, acc_ea = 0.f;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int x = p * L + x0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kyy = half_shift<N>(tc + m * T);
      v[m] = (kyy >= dk.ky_lo && kyy <= dk.ky_hi) ? img[img_slot<N>(kyy, x)]
                                                   : make_float2(0.f, 0.f);
    }
    __syncthreads();   // every column read before the transforms reuse its slots
    auto col_lay = [x](int n) { return img_slot<N>(n, x); };
    PlanT<N, T>::template run<+1>(v, tc, img, col_lay, lds_tw);
#pragma unroll
    for (int m = 0; m < E; ++m)
      v[m] = cscale(v[m], residual_factor<false>(v[m], a_meas[p][m], sg, bt.intensity, inv_m,
                                                 acc, acc_ea));
    PlanT<N, T>::template run<-1>(v, tc, img, col_lay, lds_tw);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kyy = half_shift<N>(tc + m * T);
      if (kyy >= dk.ky_lo && kyy <= dk.ky_hi) img[img_slot<N>(kyy, x)] = v[m];
    }
  }
  block_partials<1, NT / 64>(&acc, loss_part);   // (its barrier also ends the column phase)

  // ---- row phase (forward): the patch conj(P) g_Phi on the disk and the moments
  float zs[NP][6];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const Line q = line_of(p);
#pragma unroll
    for (int j = 0; j < 6; ++j) zs[p][j] = 0.f;
    float2 pv[E], cv[E];
    float kap[MODE == kPatchZern ? E : 1];
    if constexpr (NP == 1) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        pv[m] = pvv[m];
        cv[m] = ov[m];
        if constexpr (MODE == kPatchZern) kap[m] = kap0[m];
      }
    } else {
      const float2* orow = O + (size_t)(w.x + q.kyc) * bt.M + w.y;
      const float2* prow = P + (size_t)q.kyc * N;
      const int uy = q.kyc - N / 2;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int kx = min(max(half_shift<N>(t + m * T), q.extc.x), q.extc.y);
        pv[m] = prow[kx];
        if constexpr (MODE == kPatchZern) {
          cv[m] = orow[kx];
          const int ux = kx - N / 2;
          kap[m] = kappa_tab[ux * ux + uy * uy];
        }
      }
    }
    const int ky = q.ky;
#pragma unroll
    for (int m = 0; m < E; ++m)
      v[m] = q.active ? img[img_slot<N>(ky, t + m * T)] : make_float2(0.f, 0.f);
    __syncthreads();   // every row read before the transforms reuse its slots
    PlanT<N, T>::template run<-1>(v, t, img, [ky](int n) { return img_slot<N>(ky, n); }, lds_tw);
    if (q.active) {
      float2* xr = X + ((size_t)b * N + ky) * N;
      const float ir = (float)pg.inv_r;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int kx = half_shift<N>(t + m * T);
        if (kx >= q.ext.x && kx <= q.ext.y) {
          store_next<N>(xr + kx, cmulc(pv[m], v[m]));
          if constexpr (MODE == kPatchZern)
            add_row_moments(v[m], pv[m], cv[m], (float)(kx - N / 2) * ir, kap[m], zs[p]);
        }
      }
    }
  }
  if constexpr (MODE == kPatchZern) {
    // line totals (T lanes per line: in-row sums over windows of T lanes), then
    // the 16 moments sum_rows sum_x g_theta x^a y^b (a + b <= 4) and
    // sum g_theta kappa in FP64: thread (k, q) adds the lines q, q + 16, ... of
    // moment k, then thread k adds its 16 partial sums in order
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        float s = zs[p][j];
        s += dpp_move_f<0x111>(s);
        s += dpp_move_f<0x112>(s);
        s += dpp_move_f<0x114>(s);
        if constexpr (T >= 16) s += dpp_move_f<0x118>(s);
        zs[p][j] = s;
      }
      if (t == T - 1) {
#pragma unroll
        for (int j = 0; j < 6; ++j) tot[p * L + tid / T][j] = zs[p][j];
      }
    }
    __syncthreads();
    if (tid < 256) {
      const int k = tid & 15, qq = tid >> 4;
      // monomial k < 15 is x^a y^b with degree d = a + b: k = d (d + 1) / 2 + b
      int d = 0;
      while ((d + 1) * (d + 2) / 2 <= k) ++d;
      const int pb = k < 15 ? k - d * (d + 1) / 2 : 0;
      const int j = k < 15 ? d - pb : 5;
      double s = 0.0;
      for (int ll = qq; ll < dk.nrows; ll += 16) {
        double sj = (double)tot[ll][j];
        const double y = (double)(dk.ky_lo + ll - N / 2) * pg.inv_r;
        for (int e = 0; e < pb; ++e) sj *= y;
        s += sj;
      }
      msum[qq][k] = s;
    }
    __syncthreads();
    if (tid < 16) {
      double s = 0.0;
      for (int qq = 0; qq < 16; ++qq) s += msum[qq][tid];
      zpart[(size_t)blockIdx.x * 16 + tid] = s;
    }
  }
}

}  // namespace fpm
