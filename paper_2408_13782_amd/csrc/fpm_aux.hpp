// fpm_aux.hpp - pupil model, parameter-gradient projection, Adam and the
// high-resolution transforms (spectrum <-> object, initial value, refocus).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_line.hpp"
#include "fpm_kernels.hpp"
#include "fpm_optics.hpp"

namespace fpm {

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

// g_par[j] += sum_u Im(gP conj P) Z_j, g_par[15] += sum_u Im(gP conj P) kappa (FP64).
__global__ void __launch_bounds__(256)
pupil_grad(PupilGeom g, const int2* __restrict__ rowext, const float2* __restrict__ gP,
           const float2* __restrict__ P, Reduction red, double* __restrict__ g_par) {
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
    }
  }
  grid_reduce<kPar>(acc, red, [&](const double* tot, int lane) {
    if (lane < kPar) {
      double gj = 0.0;
#pragma unroll
      for (int j = 0; j < kPar; ++j)
        if (j == lane) gj = tot[j];
      g_par[lane] += gj;
    }
  });
}

// Adam (torch.optim.Adam arithmetic) on one float of the spectrum.
struct AdamCoef {
  float b1, b2, eps, step_size, sqrt_bc2;
};

__device__ __forceinline__ void adam1(float& p, float& m, float& v, float g, const AdamCoef& c) {
  m = c.b1 * m + (1.0f - c.b1) * g;
  v = c.b2 * v + (1.0f - c.b2) * g * g;
  const float den = sqrtf(v) / c.sqrt_bc2 + c.eps;
  p -= c.step_size * (m / den);
}

// Adam on the pupil parameters (Zernike 1..14, defocus), FP64 arithmetic.
struct ScalarAdam {
  int learn_c, learn_z;
  double lr_c, lr_z, b1, b2, eps, bc1, sqrt_bc2;
};

// The last launch of a step:
//  the last n_tiles workgroups: Adam over 32 x 32 tiles of the spectrum (each
//    thread 4 consecutive complex values), the gradient gathered from the
//    batch's patches in batch order (deterministic, no atomics);
//  the first workgroups: with `pupil`, each one sums the per-workgroup
//    Zernike/defocus partials of the row pass in a fixed order, applies Adam
//    to the 16 pupil parameters (all of them compute the same numbers), and
//    rebuilds its share of the pupil from the new parameters; workgroup 0 of
//    them stages the new parameter state and adds the gradients to g_par;
//  the workgroup after them (workgroup 0 without `pupil`): adds the batch
//    loss (summed from the column pass's partials) to *loss.
//  Batches of more than kMaxSlots LEDs are processed in groups: for every
//  group but the last the kernel only accumulates (acc_out: g_acc = the
//  group's gathered sum, started from g_acc when acc_in, no Adam); the last
//  group's launch starts its sums from g_acc (acc_in) and applies Adam. The
//  additions then happen in batch order, as in a single pass.
// Tiles per side of the update kernel's rectangle at most (M <= 4096).
constexpr int kMaxTileSide = 128;

struct UpdateArgs {
  int2 tile0; int tile_cols; int M;   // the rectangle of tiles: first tile, width
  float* O; float* mO; float* vO;
  float* gacc; int acc_in, acc_out;
  AdamCoef c;
  // the batch's conj(P) g_Phi patches, stored in X by the row pass
  const float2* X; Batch bt; Disk dk; int n;
  const double* loss_part; int n_loss; double* loss;
  int pupil;
  const double* zpart; int n_zpart;
  ScalarState cur; ScalarAdam sa; double* g_par; float* staging;
  PupilGeom pg; const int2* rowext; float2* P;
  // batch slots whose window's disk rows (columns) meet tile row (column) i of
  // the rectangle: a tile's slots are hit_row[row] & hit_col[column]
  unsigned long long hit_row[kMaxTileSide], hit_col[kMaxTileSide];
};

// Pupil rows rebuilt per workgroup of the update kernels (about 256 points or
// fewer each). Every pupil workgroup first sums all of the row pass's moment
// partials, so only rows that hold disk points get a workgroup.
// One disk row per workgroup up to N = 256 (at most N threads' worth of points,
// so every thread rebuilds at most one); two above, where the pupil workgroups
// (summing many more moment partials) are not on the kernel's critical path.
__host__ __device__ constexpr int pupil_rows_per_wg(int n) {
  return n <= 64 ? 8 : n <= 128 ? 4 : n <= 256 ? 1 : 2;
}
__host__ __device__ constexpr int pupil_wg_count(int n, int disk_rows) {
  return (disk_rows + pupil_rows_per_wg(n) - 1) / pupil_rows_per_wg(n);
}
// Workgroup slots given to them and to the loss workgroup that follows them: a
// multiple of the 8 XCDs, so that HR tile t (workgroup pupil_wg_slots + t) runs
// on XCD t mod 8 whatever the pupil size; the padding workgroups return at once.
__host__ __device__ constexpr int pupil_wg_slots(int n, int disk_rows) {
  return (pupil_wg_count(n, disk_rows) + 1 + 7) / 8 * 8;
}

// The batch loss of a step, by one workgroup of 256 threads (all of them call
// this): *loss += the sum of the column pass's n partials part[i * stride]
// (thread t adds partials t, t + 256, ... in increasing order, their loads
// issued kU at a time; then the four waves' totals in order). The partials and
// *loss are all requested at once: in the update kernels a workgroup of its
// own does this, so the sum does not wait behind, or delay, the pupil update.
__device__ __forceinline__ void add_batch_loss(const double* __restrict__ part, int n,
                                               double* loss, int stride = 1) {
  constexpr int kU = 8;
  __shared__ double wsum[4];
  const double prev = *loss;
  double s = 0.0;
  for (int i0 = threadIdx.x; i0 < n; i0 += 256 * kU) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = part[(size_t)min(i0 + u * 256, n - 1) * stride];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (i0 + u * 256 < n) s += v[u];
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *loss = prev + (((wsum[0] + wsum[1]) + wsum[2]) + wsum[3]);
}

// exp(i th) rounded to complex64: th reduced to [-pi, pi] in FP64 (exact to
// FP64 rounding for the phases of a pupil), then the FP32 sine and cosine of
// the reduced angle, whose error (an FP32 ulp) is that of the final rounding;
// an FP64 sincos costs several times the instructions for the same stored value.
__device__ __forceinline__ float2 unit_phasor(double th) {
  constexpr double kTwoPi = 6.283185307179586;
  const double r = th - kTwoPi * rint(th * (1.0 / kTwoPi));
  float sn, cs;
  sincosf((float)r, &sn, &cs);
  return make_float2(cs, sn);
}

// Pupil workgroup pw rebuilds P on the disk points of disk rows pw R .. pw R + R - 1
// (R = pupil_rows_per_wg(N)) from the phase coefficients coef[0..14] (Zernike)
// and, with `defocus`, coef[15] (z); the workgroup's 256 threads are spread
// over those rows' points. FP64 phase, FP32 store; off the disk P stays zero.
// kReload: re-read the coefficients for every point instead of keeping them
// live across the loop (for a host kernel that is short of registers).
template <int N, bool kReload>
__device__ __forceinline__ void rebuild_pupil_rows(int pw, const Disk& dk, const PupilGeom& pg,
                                                   const float* coef, bool defocus, float2* P) {
  constexpr int R = pupil_rows_per_wg(N);
  const int r0 = pw * R;
  int start[R], first[R];
  int total = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int2 e = r0 + r < dk.nrows ? disk_extent<N>(dk, dk.ky_lo + r0 + r) : make_int2(0, -1);
    start[r] = total;
    first[r] = e.x;
    total += max(e.y - e.x + 1, 0);
  }
  // the phase as a polynomial in the monomials x^a y^b (a + b <= 4):
  // sum_j c_j Z_j = sum_k (sum_j c_j kZernMono[j][k]) x^a y^b
  __shared__ double mono[kMono];
  if (threadIdx.x < kMono) {
    double m = 0.0;
    for (int j = 0; j < kZern; ++j) m += (double)coef[j] * kZernMono[j][threadIdx.x];
    mono[threadIdx.x] = m;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < total; i += 256) {
    if constexpr (kReload) asm volatile("" ::: "memory");
    int r = 0, s0 = 0, x0 = first[0];
#pragma unroll
    for (int q = 1; q < R; ++q)
      if (i >= start[q]) { r = q; s0 = start[q]; x0 = first[q]; }
    const int ky = dk.ky_lo + r0 + r, kx = x0 + (i - s0);
    const double ux = kx - N / 2, uy = ky - N / 2;
    const double x = ux * pg.inv_r, y = uy * pg.inv_r;
    const double x2 = x * x, y2 = y * y, xy = x * y;
    double th = mono[0] + mono[1] * x + mono[2] * y + mono[3] * x2 + mono[4] * xy + mono[5] * y2;
    th += (mono[6] * x + mono[7] * y) * x2 + (mono[8] * x + mono[9] * y) * y2;
    th += (mono[10] * x2 + mono[11] * xy + mono[12] * y2) * x2 + (mono[13] * xy + mono[14] * y2) * y2;
    if (defocus) th += (double)coef[kZern] * defocus_kappa((ux * ux + uy * uy) * pg.dk2, pg.inv_l);
    P[(size_t)ky * N + kx] = unit_phasor(th);
  }
}

// Gradient of the spectrum at the 4 pixels of a tile thread (row r, columns
// c0 + tile_col(q)): the sum, in batch order, of the patches of the LEDs whose
// disk covers them.
// g holds the running sums on entry (zero, or the earlier groups' sums).
template <int N>
__device__ __forceinline__ void gather_gradient(const UpdateArgs& a, int r, int c0, int tr, int tc,
                                                float2 (&g)[4]) {
  // slots whose disk bounding box meets this 32 x 32 tile (uniform over the
  // workgroup), from the per-row and per-column masks of the launch
  unsigned long long hit = a.hit_row[tr] & a.hit_col[tc];
  constexpr int kRound = 4;
  while (hit) {
    // kRound slots per round: their windows read together, then all loads
    // issued (at addresses clamped into the disk) before the masked, in-order
    // accumulation
    int bs[kRound];
    int2 wv[kRound];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
      bs[u] = hit ? __ffsll((long long)hit) - 1 : -1;
      if (hit) hit &= hit - 1;
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u) wv[u] = a.bt.win[bs[u] < 0 ? bs[0] : bs[u]];
    float2 val[kRound][4];
    bool ok[kRound][4];
#pragma unroll
    for (int u = 0; u < kRound; ++u) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ok[u][q] = false;
        val[u][q] = make_float2(0.f, 0.f);
      }
      if (bs[u] < 0) continue;   // uniform: no loads for an empty slot
      const int b = bs[u];
      const int wr = wv[u].x, wc = wv[u].y;
      const int ky = r - wr;
      const int kyc = min(max(ky, a.dk.ky_lo), a.dk.ky_hi);
      const int2 e = disk_extent<N>(a.dk, kyc);
      const float2* xr = a.X + ((size_t)b * N + kyc) * N;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kx = c0 + tile_col(q) - wc;
        ok[u][q] = ky == kyc && kx >= e.x && kx <= e.y;
        val[u][q] = xr[min(max(kx, e.x), e.y)];
      }
    }
#pragma unroll
    for (int u = 0; u < kRound; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (ok[u][q]) {
          g[q].x += val[u][q].x;
          g[q].y += val[u][q].y;
        }
  }
}

template <int N>
__global__ void __launch_bounds__(256) update(UpdateArgs a) {
  const int n_pw = a.pupil ? pupil_wg_slots(N, a.dk.nrows) : 1;
  if ((int)blockIdx.x >= n_pw) {
    const int i = blockIdx.x - n_pw;
    const int tr = i / a.tile_cols;
    const int2 tl = make_int2(a.tile0.x + tr, a.tile0.y + (i - tr * a.tile_cols));
    const int r = tl.x * 32 + (threadIdx.x >> 3);
    const int col = tl.y * 32 + (threadIdx.x & 7) * 2;         // complex column
    const size_t f = ((size_t)r * a.M + col) * 2;                // float offset
    float4* po = reinterpret_cast<float4*>(a.O + f);
    float4* pm = reinterpret_cast<float4*>(a.mO + f);
    float4* pv = reinterpret_cast<float4*>(a.vO + f);
    float4 o[2], m[2], v[2], gi[2];
    float4* pg = a.gacc ? reinterpret_cast<float4*>(a.gacc + f) : nullptr;
#pragma unroll
    for (int h = 0; h < 2; ++h) {   // in flight while the gradient is gathered
      if (!a.acc_out) {
        o[h] = po[8 * h];
        m[h] = pm[8 * h];
        v[h] = pv[8 * h];
      }
      gi[h] = a.acc_in ? pg[8 * h] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float2 g[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      g[2 * h] = make_float2(gi[h].x, gi[h].y);
      g[2 * h + 1] = make_float2(gi[h].z, gi[h].w);
    }
    gather_gradient<N>(a, r, col, tr, i - tr * a.tile_cols, g);
    if (a.acc_out) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
        store_next4<N>(pg + 8 * h, make_float4(g[2 * h].x, g[2 * h].y, g[2 * h + 1].x, g[2 * h + 1].y));
      return;
    }
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
  const int n_pupil = a.pupil ? pupil_wg_count(N, a.dk.nrows) : 0;
  if (pw == n_pupil) {   // the loss workgroup
    if (a.loss) add_batch_loss(a.loss_part, a.n_loss, a.loss);
    return;
  }
  if (pw > n_pupil) return;   // padding
  __shared__ double red[256];
  __shared__ double gsum[kPar];
  __shared__ float next[kScal];
  {
    // moments of the row pass: thread t sums entry t % 16 of partials t/16, t/16 + 16, ...
    // (independent loads in flight, then a fixed summation order)
    const int j = threadIdx.x & (kPar - 1);
    double sj = 0.0;
    // 40 loads per thread in flight: all 640 partials of a batch of 16 at N = 256
    constexpr int kStride = 256 / kPar, kUnroll = 40;
    for (int i0 = threadIdx.x / kPar; i0 < a.n_zpart; i0 += kStride * kUnroll) {
      double vals[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = i0 + u * kStride;
        vals[u] = a.zpart[(size_t)min(i, a.n_zpart - 1) * kPar + j];
        if (i >= a.n_zpart) vals[u] = 0.0;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) sj += vals[u];
    }
    red[threadIdx.x] = sj;
    __syncthreads();
    if (threadIdx.x < kPar) {
      double mom = 0.0;
      for (int k = 0; k < kStride; ++k) mom += red[k * kPar + threadIdx.x];
      gsum[threadIdx.x] = mom;
    }
    __syncthreads();
    if (threadIdx.x < kPar) {
      // Zernike gradients from the monomial moments; defocus gradient directly
      double g = gsum[kZern];
      if (threadIdx.x < kZern) {
        g = 0.0;
#pragma unroll
        for (int k = 0; k < kMono; ++k) g += kZernMono[threadIdx.x][k] * gsum[k];
      }
      red[threadIdx.x] = g;
      // current value, moments; unchanged unless learned
      const bool is_z = threadIdx.x == kZern;
      // (a NULL array stands for zeros: the Zernike state may be absent when
      // only the defocus is learned, and the reverse)
      const float* pc = is_z ? a.cur.z : a.cur.coeffs ? a.cur.coeffs + threadIdx.x : nullptr;
      const float* pm = is_z ? a.cur.m_z : a.cur.m_c ? a.cur.m_c + threadIdx.x : nullptr;
      const float* pv = is_z ? a.cur.v_z : a.cur.v_c ? a.cur.v_c + threadIdx.x : nullptr;
      float p = pc ? *pc : 0.f, m = pm ? *pm : 0.f, v = pv ? *pv : 0.f;
      // piston (j = 0): a global phase with an identically zero gradient, held fixed
      const bool learn = is_z ? a.sa.learn_z : (a.sa.learn_c && threadIdx.x != 0);
      if (learn) {
        const double lr = is_z ? a.sa.lr_z : a.sa.lr_c;
        const double mm = a.sa.b1 * (double)m + (1.0 - a.sa.b1) * g;
        const double vv = a.sa.b2 * (double)v + (1.0 - a.sa.b2) * g * g;
        const double den = sqrt(vv) / a.sa.sqrt_bc2 + a.sa.eps;
        p = (float)((double)p - lr / a.sa.bc1 * mm / den);
        m = (float)mm;
        v = (float)vv;
      }
      next[threadIdx.x] = p;
      next[kPar + threadIdx.x] = m;
      next[2 * kPar + threadIdx.x] = v;
    }
    __syncthreads();
    if (pw == 0 && threadIdx.x < kScal) a.staging[threadIdx.x] = next[threadIdx.x];
    if (pw == 0 && threadIdx.x < kPar && a.g_par) a.g_par[threadIdx.x] += red[threadIdx.x];
    // rebuild this workgroup's rows of the pupil from the new parameters
    rebuild_pupil_rows<N, false>(pw, a.dk, a.pg, next, a.cur.z != nullptr, a.P);
  }
}

// ---------------------------------------------------------------------------
// High-resolution 2-D transforms, split into a row pass and a column pass.

template <int M> struct HrRowLines { static constexpr int value = (128 / Plan1D<M>::T) > 0 ? 128 / Plan1D<M>::T : 1; };
// columns per workgroup of the HR column pass: M x HrColStride complex slots of LDS
template <int M> struct HrColLines { static constexpr int value = M > 1024 ? 8 : 16; };
// LDS slots between consecutive elements of one column: one padding slot,
// none at M = 2048 (8 columns of 128 threads), where by a model of 32 banks
// and 16 lanes per 8-byte access one slot of padding doubles the cycles of
// the exchanges (the bank-conflict counter read 50 % of the pass's LDS cycles)
// and none costs 1.25 times the conflict-free cycles.
template <int M> struct HrColStride { static constexpr int value = HrColLines<M>::value + (M == 2048 ? 0 : 1); };

enum HrRowMode { kRowFwd = 0, kRowInv = 1, kRowInit = 2, kRowRefocus = 3 };

struct HrArgs {
  const float2* in;     // row-pass source (object, spectrum)
  const float* img;     // kRowInit: centre amplitude image [n][n]
  int n, s;             // kRowInit: LR size and upsampling
  const float* z_um;    // kRowRefocus: device pointer to the distances, one per grid row y
  double dk2, inv_l;    // kRowRefocus
  float2* out;          // destination of both passes; transform y of a batch at out + y M^2
};

// Forward (DIR -1): rows of o, DFT, fftshift along k_x.
// Inverse (DIR +1): ifftshift along k_x (times H(z) when refocusing), inverse DFT.
// A refocusing launch serves a batch of distances: grid row y computes the
// transform at z_um[y] into out + y M^2 (one launch per pass for the sweep).
template <int M, int MODE>
__global__ void __launch_bounds__(HrRowLines<M>::value * Plan1D<M>::T)
hr_rows(HrArgs a, const float2* __restrict__ tw) {
  constexpr int T = Plan1D<M>::T;
  constexpr int E = M / T;
  constexpr int L = HrRowLines<M>::value;
  constexpr int DIR = (MODE == kRowFwd || MODE == kRowInit) ? -1 : +1;
  __shared__ float2 lds[L * RowLds<M>::kStride];
  const int line = threadIdx.x / T, t = threadIdx.x % T;
  const int row = blockIdx.x * L + line;   // grid covers M rows exactly
  float2* out = a.out + (size_t)blockIdx.y * M * M;
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
    const double z = MODE == kRowRefocus ? (double)a.z_um[blockIdx.y] : 0.0;
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
          sincos(z * defocus_kappa(k2, a.inv_l), &sn, &cs);
          val = cmul(val, make_float2((float)cs, (float)sn));
        }
      }
      v[m] = val;
    }
  }
  Plan1D<M>::template run<DIR>(v, t, lds + line * RowLds<M>::kStride, [](int n) { return RowLds<M>::at(n); }, tw);
  float2* orow = out + (size_t)row * M;
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
  constexpr int S = HrColStride<M>::value;
  __shared__ float2 lds[M * S];
  const int line = threadIdx.x % L, t = threadIdx.x / L;
  const int x = blockIdx.x * L + line;
  data += (size_t)blockIdx.y * M * M;   // transform y of a batch
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int n = t + m * T;
    v[m] = data[(size_t)(DIR > 0 ? half_shift<M>(n) : n) * M + x];
  }
  auto lay = [line](int n) { return n * S + line; };
  Plan1D<M>::template run<DIR>(v, t, lds, lay, tw);
  constexpr float inv = 1.0f / M;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int n = t + m * T;
    data[(size_t)(DIR < 0 ? half_shift<M>(n) : n) * M + x] = cscale(v[m], inv);
  }
}

}  // namespace fpm
