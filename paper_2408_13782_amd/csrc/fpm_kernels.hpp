// fpm_kernels.hpp - device kernels of the Batch-FPM hot path (gfx950).
//
// Per random batch of B LEDs, the loss and its adjoint are three launches
// (the 2-D transforms of N x N images do not fit one CU's LDS for N >= 256,
// so they are split into row and column passes that meet in an L2/MALL
// resident scratch X[B][N][N]):
//
//   rows_forward   crop C_b = O[w_b + u] on the pupil disk, Phi = C_b P
//                  (P read, or rebuilt from its Zernike/defocus parameters),
//                  ifftshift along k_x, inverse DFT of each disk row -> X
//   cols           inverse DFT of each column (ifftshift along k_y) -> psi,
//                  amplitude residual e = sqrt(gamma)|psi| - A, loss,
//                  g_psi = 2 sqrt(gamma) e psi / |psi|, forward DFT of each
//                  column, keep disk rows (fftshift) -> X (in place)
//   rows_backward  forward DFT of each disk row, keep disk columns, scatter-add
//                  conj(P) g_Phi into g_O; the pupil gradient either
//                  scatter-added into g_P or projected on the spot onto the
//                  Zernike/defocus parameters
//
// Scalar results (loss, parameter gradients) are reduced without contended
// atomics or device-scope fences (a fence writes back the XCD's L2): each
// workgroup stores a partial sum, and a later kernel of the same stream adds
// the partials in a fixed order, so the sums are deterministic.
//
// Workgroups of one LED are placed on one XCD (workgroup id mod 8 selects
// the XCD) so that the scratch written by one pass is read from the same
// XCD's L2 by the next.
#pragma once
#include <hip/hip_runtime.h>
#include <cfloat>
#include <stdint.h>

#include "fft_line.hpp"
#include "fpm_optics.hpp"

namespace fpm {

constexpr int kRowThreads = 128;   // threads per workgroup in the row passes
constexpr int kXcds = 8;

// Threads per row transform in the row passes (more threads per line than
// the default plan: more waves in flight for the few rows of a batch).
template <int N> struct RowT { static constexpr int value = DefaultT<N>::value; };
template <> struct RowT<128> { static constexpr int value = 32; };
template <> struct RowT<256> { static constexpr int value = 32; };
template <> struct RowT<512> { static constexpr int value = 32; };
template <int N> using RowPlan = PlanT<N, RowT<N>::value>;

// The nearest-pixel row passes, each with its own shape. At N = 256, 64
// threads per row take 0.26 us off the forward pass (two rows per workgroup);
// at N = 512, 64 threads per row in both passes take 2.8 us off a step
// (B = 32). The backward pass keeps the common rows per workgroup (with 64
// threads per row, in 256-thread workgroups): its workgroup count is the
// number of moment partials that every pupil workgroup of the update sums. At
// N = 256 that shape measured no better than 32 threads per row.
template <int N> struct FwdRow { static constexpr int T = RowT<N>::value, threads = kRowThreads; };
template <> struct FwdRow<256> { static constexpr int T = 64, threads = kRowThreads; };
template <> struct FwdRow<512> { static constexpr int T = 64, threads = kRowThreads; };
template <int N> struct BwdRow { static constexpr int T = RowT<N>::value, threads = kRowThreads; };
template <> struct BwdRow<512> { static constexpr int T = 64, threads = 2 * kRowThreads; };

template <int N> struct ColLines { static constexpr int value = 16; };
template <> struct ColLines<512> { static constexpr int value = 8; };

// Threads per column transform in the column pass (more threads per column
// than the row passes: with B = 16 the pass has about one wave per SIMD at 16
// elements per thread, and more waves hide the LDS and dependency latency).
template <int N> struct ColT { static constexpr int value = DefaultT<N>::value; };
template <> struct ColT<128> { static constexpr int value = 32; };
template <> struct ColT<256> { static constexpr int value = 32; };
template <> struct ColT<512> { static constexpr int value = 64; };
template <int N> using ColPlan = PlanT<N, ColT<N>::value>;
// LDS slots between consecutive elements of one column (padding by radix).
// N = 512 (8 columns of 64 threads): no padding. By a model of 32 banks and 16
// lanes per 8-byte access, two padding slots made the exchanges take twice
// the conflict-free cycles (the bank-conflict counter read 46 % of the pass's
// LDS cycles), none 1.25 times; the pass also fits four workgroups per CU in
// LDS instead of three. Measured 2.8 us less per launch (30.2-31.1 -> 27.4-27.8).
template <int N> struct ColStride {
  static constexpr int value = ColLines<N>::value + (N / ColT<N>::value >= 16 ? 1 : 2);
};
template <> struct ColStride<512> { static constexpr int value = ColLines<512>::value; };

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

// Stores of data that the next kernel reads (the intermediate rows, the
// patches, the optimiser state). Up to N = 256 (spectrum state <= 24 MB) they
// are non-temporal: they do not linger in the L2 as dirty lines to be written
// back when the kernel ends (0.4 us per step measured at N = 256). At larger
// sizes plain stores are faster (the state then stays in the memory-side cache
// for the next step: 10 us per step at N = 512).
template <int N> struct NtStores { static constexpr bool value = N <= 256; };

template <int N>
__device__ __forceinline__ void store_next(float2* p, float2 v) {
  if constexpr (NtStores<N>::value) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
  } else {
    *p = v;
  }
}

// Tile kernels (32 x 32 HR tiles, 256 threads): thread t covers row t / 8 of
// the tile and the complex columns 2 (t % 8) + tile_col(q), q = 0..3, i.e. the
// float4 t % 8 and t % 8 + 8 of the row, so that each 16-byte access of 8
// neighbouring lanes fills one whole 128-byte line.
__device__ __forceinline__ constexpr int tile_col(int q) { return (q & 1) + (q >> 1) * 16; }

template <int N>
__device__ __forceinline__ void store_next4(float4* p, float4 v) {
  if constexpr (NtStores<N>::value) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z);
    __builtin_nontemporal_store(v.w, &p->w);
  } else {
    *p = v;
  }
}

// sum_{i < n} src[i * stride] in increasing i, the loads issued kU at a time.
template <int kU = 16>
__device__ __forceinline__ double ordered_sum(const double* __restrict__ src, int n, int stride) {
  double s = 0.0;
  for (int i0 = 0; i0 < n; i0 += kU) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = src[(size_t)min(i0 + u, n - 1) * stride];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (i0 + u < n) s += v[u];
  }
  return s;
}

// Inverse of xcd_map: the workgroup that serves chunk c of batch slot b.
__device__ __forceinline__ int xcd_wg(int b, int c, int chunks) {
  return (b % kXcds) + kXcds * ((b / kXcds) * chunks + c);
}

__device__ __forceinline__ void atomic_add_c(float2* p, float2 v) {
  float* f = reinterpret_cast<float*>(p);
  unsafeAtomicAdd(f, v.x);
  unsafeAtomicAdd(f + 1, v.y);
}

// The batch, passed by value: LED ids and the top-left corner (HR row, column)
// of each LED's window, so no kernel has to look them up in memory.
constexpr int kMaxSlots = 64;

struct Batch {
  int B;
  int M;
  int intensity;   // 0: amplitude loss (Eq. 5 form), 1: intensity loss (Eq. 4)
  int led[kMaxSlots];
  int2 win[kMaxSlots];
};

// Pupil disk |u|^2 <= R^2: per-row column extents, the row range, and
// floor(R^2) (the test on integer |u|^2 is exact against it).
struct Disk {
  const int2* rowext;
  int ky_lo, ky_hi, nrows;
  int r2i;
};

// First and last disk column of pupil row ky (exact integer square root).
template <int N>
__device__ __forceinline__ int2 disk_extent(const Disk& dk, int ky) {
  const int uy = ky - N / 2;
  const int q = dk.r2i - uy * uy;
  if (q < 0) return make_int2(N, -1);
  // floor(sqrt(q)): sqrt(q + 1/2) is never an integer and lies far enough from
  // one (at least 1/(4 sqrt(q + 1))) for a float square root to truncate to the
  // exact value for q < 2^22; the two selects keep it exact without loops
  int h = (int)sqrtf((float)q + 0.5f);
  h -= h * h > q ? 1 : 0;
  h += (h + 1) * (h + 1) <= q ? 1 : 0;
  return make_int2(N / 2 - h, N / 2 + h);
}

// Per-workgroup partials and the completion counter of a last-workgroup reduction.
struct Reduction {
  double* part;
  unsigned* counter;
};

// Data-parallel-primitive (DPP) lane moves of a double, out-of-row lanes read 0.
template <int kCtrl>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum of v over the 64 lanes of the wave, the same value in every lane: an
// in-row prefix sum with row_shr 1, 2, 4, 8 (lane 15 of each row of 16 then
// holds the row's total), then the four row totals added in order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0x111>(v);
  v += dpp_move<0x112>(v);
  v += dpp_move<0x114>(v);
  v += dpp_move<0x118>(v);
  return ((read_lane(v, 15) + read_lane(v, 31)) + read_lane(v, 47)) + read_lane(v, 63);
}

template <int kCtrl>
__device__ __forceinline__ float dpp_move_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xF, 0xF, true));
}

// Zernike/defocus moment partials of one row-pass workgroup. Thread t of the
// team of T threads that owns row `line` holds the six row sums
// s = (sum g, sum g x, ..., sum g x^4, sum g kappa) over its elements; the
// teams' totals are formed with in-row prefix sums (DPP row_shr, FP32), and
// threads 0..15 expand them with the powers of the rows' y into the 16 moments
// sum g x^a y^b (a + b <= 4, the monomial order of kZernMono) and sum g kappa,
// summed over the workgroup's rows in FP64 and stored to part[blockIdx.x][16].
// Every thread of the workgroup must call this (lanes outside the disk pass 0).
template <int T, int L>
__device__ __forceinline__ void row_moment_partials(float (&sv)[6], int row0, const Disk& dk,
                                                    int half_n, float inv_r, double* part) {
  static_assert(T == 8 || T == 16 || T == 32 || T == 64, "row team of 8 to 64 threads");
  constexpr int kRows16 = L * T / 16;            // rows of 16 lanes in the workgroup
  __shared__ float tot[kRows16 > L ? kRows16 : L][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    float v = sv[j];
    v += dpp_move_f<0x111>(v);
    v += dpp_move_f<0x112>(v);
    v += dpp_move_f<0x114>(v);
    if constexpr (T >= 16) v += dpp_move_f<0x118>(v);
    sv[j] = v;
  }
  // T <= 16: the team's last lane holds its total; T > 16: each row of 16 lanes'
  // last lane holds that row's total
  constexpr int kSeg = T < 16 ? T : 16;
  if ((threadIdx.x % kSeg) == kSeg - 1) {
#pragma unroll
    for (int j = 0; j < 6; ++j) tot[threadIdx.x / kSeg][j] = sv[j];
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (k < 16) {
    // monomial k < 15 is x^a y^b with degree d = a + b: k = d (d + 1) / 2 + b
    int d = 0;
    while ((d + 1) * (d + 2) / 2 <= k) ++d;
    const int pb = k < 15 ? k - d * (d + 1) / 2 : 0;
    const int j = k < 15 ? d - pb : 5;
    double acc = 0.0;
    for (int l = 0; l < L; ++l) {
      if (row0 + l >= dk.nrows) break;
      double sj = 0.0;
#pragma unroll
      for (int q = 0; q < T / kSeg; ++q) sj += (double)tot[l * (T / kSeg) + q][j];
      const double y = (double)(dk.ky_lo + row0 + l - half_n) * (double)inv_r;
      for (int e = 0; e < pb; ++e) sj *= y;
      acc += sj;
    }
    part[(size_t)blockIdx.x * 16 + k] = acc;
  }
}

// Sum K per-thread values over the workgroup; thread k < K stores total k into
// part[blockIdx.x * K + k]. Fixed summation order. No ordering with other
// workgroups is implied.
// kWaves: the most waves a workgroup of the caller has (sizes the LDS buffer).
template <int K, int kWaves = 16, class V>
__device__ __forceinline__ void block_partials(const V* vals, double* part) {
  __shared__ double wsum[kWaves][K];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double v = wave_sum((double)vals[k]);
    if (lane == 0) wsum[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += wsum[w][threadIdx.x];
    part[(size_t)blockIdx.x * K + threadIdx.x] = s;
  }
}

// Sum K per-thread values over the workgroup into part[blockIdx.x * K + k], then
// let the last workgroup to arrive call done(sums) with the grid-wide totals
// (summed in workgroup order). Every workgroup of the grid must call this.
template <int K, class V, class Done>
__device__ __forceinline__ void grid_reduce(const V* vals, Reduction red, Done done) {
  __shared__ double wsum[16][K];
  __shared__ int is_last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double v = vals[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) wsum[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += wsum[w][threadIdx.x];
    red.part[(size_t)blockIdx.x * K + threadIdx.x] = s;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(red.counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  if (threadIdx.x < 64) {
    double tot[K];
#pragma unroll
    for (int k = 0; k < K; ++k) tot[k] = 0.0;
    const volatile double* part = red.part;
    for (unsigned i = lane; i < gridDim.x; i += 64) {
#pragma unroll
      for (int k = 0; k < K; ++k) tot[k] += part[(size_t)i * K + k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) tot[k] += __shfl_xor(tot[k], off);
    }
    if (lane == 0) {
      *red.counter = 0u;
    }
    done(tot, lane);
  }
}

// ---------------------------------------------------------------------------
// Pupil-parameter state in one block: [0,15) coeffs, 15 z, [16,31) m_c, 31 m_z,
// [32,47) v_c, 47 v_z. The update kernel writes the next state to a staging
// block, which the following step's first kernel (or a commit launch) copies
// into the caller's buffers; so no kernel reads state that it also writes.
constexpr int kScal = 3 * kPar;

struct ScalarState {
  float* coeffs; float* m_c; float* v_c;
  float* z; float* m_z; float* v_z;
};

__device__ __forceinline__ void commit_scalars(const float* __restrict__ staging, ScalarState d,
                                               int i) {
  if (i >= kScal) return;
  const int part = i / kPar, j = i - part * kPar;
  float* dst;
  if (j < kZern) {
    dst = part == 0 ? d.coeffs : part == 1 ? d.m_c : d.v_c;
    if (dst) dst[j] = staging[i];
  } else {
    dst = part == 0 ? d.z : part == 1 ? d.m_z : d.v_z;
    if (dst) dst[0] = staging[i];
  }
}

__global__ void commit_scalar_state(const float* __restrict__ staging, ScalarState d) {
  commit_scalars(staging, d, threadIdx.x);
}

// Row pass 1: crop, pupil, inverse DFT along k_x. With `commit`, workgroup 0
// also copies the staged pupil-parameter state of the previous step.
template <int N>
__global__ void __launch_bounds__(FwdRow<N>::threads)
rows_forward(const float2* __restrict__ O, const float2* __restrict__ P, Batch bt, Disk dk,
             int chunks, float2* __restrict__ X, const float2* __restrict__ tw, int commit,
             const float* __restrict__ staging, ScalarState scal) {
  constexpr int T = FwdRow<N>::T;
  constexpr int E = N / T;
  constexpr int L = FwdRow<N>::threads / T;
  __shared__ float2 lds[L * RowLds<N>::kStride];
  __shared__ float2 lds_tw[N];
  if (commit && blockIdx.x == 0) commit_scalars(staging, scal, threadIdx.x);
  int b, c;
  if (!xcd_map(blockIdx.x, chunks, bt.B, b, c)) return;
  const int line = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const int rr = c * L + line;
  const bool active = rr < dk.nrows;
  const int ky = dk.ky_lo + (active ? rr : 0);
  const int2 ext = disk_extent<N>(dk, ky);
  const int2 w = bt.win[b];
  const float2* orow = O + (size_t)(w.x + ky) * bt.M + w.y;
  const float2* prow = P + (size_t)ky * N;
  // Unconditional loads at addresses clamped into the disk (the same cache lines
  // as the neighbouring disk pixels), then masked: every load of the thread is
  // in flight at once instead of one branch-guarded load after another.
  float2 ov[E], pvv[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kx = min(max(half_shift<N>(t + m * T), ext.x), ext.y);
    ov[m] = orow[kx];
    pvv[m] = prow[kx];
  }
  stage_twiddles_after_loads<N, FwdRow<N>::threads>(lds_tw, tw);
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kx = half_shift<N>(t + m * T);
    const bool in = active && kx >= ext.x && kx <= ext.y;
    v[m] = in ? cmul(ov[m], pvv[m]) : make_float2(0.f, 0.f);
  }
  PlanT<N, T>::template run<+1>(v, t, lds + line * RowLds<N>::kStride, [](int n) { return RowLds<N>::at(n); }, lds_tw);
  if (active) {
    float2* xr = X + ((size_t)b * N + ky) * N;
#pragma unroll
    for (int m = 0; m < E; ++m) store_next<N>(xr + t + m * T, v[m]);
  }
}

// The loss term of one pixel and the factor that turns the inverse DFT's output
// v = M psi into the residual's input to the forward DFT (Eqs. 4-5). Both 1/M
// scalings (of psi and of the residual's forward transform, which is linear)
// are folded into the factor. acc += e^2; with kGamma, acc_ea += the pixel's
// term of dL/dgamma (e |psi| for the amplitude loss, e |psi|^2 for intensity).
template <bool kGamma>
__device__ __forceinline__ float residual_factor(float2 v, float a_meas, float sg, int intensity,
                                                 float inv_m, float& acc, float& acc_ea) {
  const float inv_m2 = inv_m * inv_m, m_side = 1.f / inv_m;
  const float qv = v.x * v.x + v.y * v.y;   // M^2 |psi|^2
  if (intensity) {
    // e = gamma |psi|^2 - A^2, g_psi = 4 gamma e psi; dL/dgamma = 2 sum e |psi|^2
    const float q = qv * inv_m2;
    const float e = sg * sg * q - a_meas * a_meas;
    acc += e * e;
    if constexpr (kGamma) acc_ea += e * q;
    return 4.f * sg * sg * e * inv_m2;
  }
  // e = sqrt(gamma) |psi| - A and g_psi = 2 sqrt(gamma) e psi/|psi|
  //   = 2 sqrt(gamma) (sqrt(gamma) - A/|psi|) psi, with 1/|psi| from one
  // reciprocal square root (1 ulp) instead of a square root and a division;
  // where |psi|^2 is below the normal range, 1/|psi| is taken as 0 (then
  // e = -A and g_psi vanishes with psi)
  const float rv = qv >= FLT_MIN ? __builtin_amdgcn_rsqf(qv) : 0.f;   // 1/(M |psi|)
  const float a = qv * rv * inv_m;
  const float e = sg * a - a_meas;
  acc += e * e;
  if constexpr (kGamma) acc_ea += e * a;
  return 2.f * sg * (sg - a_meas * rv * m_side) * inv_m2;
}

// Column pass: inverse DFT along k_y, amplitude loss, residual, forward DFT.
// kForward: write amplitudes (and fields) instead of the residual transform.
template <int N, bool kForward, bool kGamma = false>
__global__ void __launch_bounds__(ColLines<N>::value * ColPlan<N>::T)
cols(float2* __restrict__ X, const float* __restrict__ A, const float* __restrict__ gamma,
     Batch bt, Disk dk, int groups, double* __restrict__ loss_part,
     float* __restrict__ amp_out, float2* __restrict__ field_out, const float2* __restrict__ tw,
     float inv_m) {
  constexpr int T = ColPlan<N>::T;
  constexpr int E = N / T;
  constexpr int L = ColLines<N>::value;
  __shared__ float2 lds[N * ColStride<N>::value];
  __shared__ float2 lds_tw[N];
  int b, g;
  const bool live = xcd_map(blockIdx.x, groups, bt.B, b, g);
  const int line = threadIdx.x % L;
  const int t = threadIdx.x / L;
  const int x = g * L + line;
  float acc = 0.f, acc_ea = 0.f;   // sum e^2, sum e |psi| (the latter for dL/dgamma)
  if (live) {
    const int led = bt.led[b];
    float2* xb = X + (size_t)b * N * N;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int ky = half_shift<N>(t + m * T);
      v[m] = (ky >= dk.ky_lo && ky <= dk.ky_hi) ? xb[(size_t)ky * N + x] : make_float2(0.f, 0.f);
    }
    float a_meas[kForward ? 1 : E];
    if constexpr (!kForward) {
      const float* ab = A + (size_t)led * N * N;
#pragma unroll
      for (int m = 0; m < E; ++m) a_meas[m] = ab[(size_t)(t + m * T) * N + x];   // prefetch
    }
    stage_twiddles_after_loads<N, L * T>(lds_tw, tw);
    const float sg = gamma ? sqrtf(gamma[led]) : 1.0f;
    auto lay = [line](int n) { return n * ColStride<N>::value + line; };
    ColPlan<N>::template run<+1>(v, t, lds, lay, lds_tw);
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
#pragma unroll
      for (int m = 0; m < E; ++m)
        v[m] = cscale(v[m], residual_factor<kGamma>(v[m], a_meas[m], sg, bt.intensity, inv_m, acc,
                                                    acc_ea));
      ColPlan<N>::template run<-1>(v, t, lds, lay, lds_tw);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int ky = half_shift<N>(t + m * T);
        if (ky >= dk.ky_lo && ky <= dk.ky_hi) store_next<N>(xb + (size_t)ky * N + x, v[m]);
      }
    }
  }
  if constexpr (!kForward) {
    if constexpr (kGamma) {
      const float both[2] = {acc, acc_ea};
      block_partials<2>(both, loss_part);
    } else {
      if (loss_part) block_partials<1>(&acc, loss_part);
    }
  }
}

// One disk pixel's share of the Zernike/defocus moments: with g_P = conj(C) g_Phi
// and g_theta = Im(g_P conj(P)) (P = mask exp(i theta)), the row sums
// S = (sum g_theta x^a for a = 0..4, sum g_theta kappa), x = u_x / R.
__device__ __forceinline__ void add_row_moments(float2 g, float2 p, float2 c, float xx, float kap,
                                                float (&S)[6]) {
  const float2 gp = cmulc(c, g);                  // conj(C) g_Phi
  const float gth = gp.y * p.x - gp.x * p.y;      // Im(g_P conj(P))
  const float gx = gth * xx, gx2 = gx * xx, gx3 = gx2 * xx;
  S[0] += gth;
  S[1] += gx;
  S[2] += gx2;
  S[3] += gx3;
  S[4] += gx3 * xx;
  S[5] += gth * kap;
}

// kGradO: g_O scatter-added with atomics; kGradOP: and g_P; kPatch: conj(P) g_Phi
// is stored in place in X (disk positions of each row) for the update kernel to
// gather; kPatchZern: kPatch plus the pupil-parameter moments.
enum RowsBackwardMode { kGradO = 0, kGradOP = 1, kPatch = 2, kPatchZern = 3 };

// Row pass 2: forward DFT along x, conj-pupil, scatter-add into g_O; the pupil
// gradient is scatter-added into g_P (kGradOP) or reduced to the moments
// sum_u g_theta x^a y^b (a + b <= 4) and sum_u g_theta kappa (kGradOZern:
// per-workgroup partials in zpart; kappa_tab[|u|^2] = kappa), from which the
// Zernike gradients follow by the fixed map kZernMono.
template <int N, int MODE>
__global__ void __launch_bounds__(BwdRow<N>::threads)
rows_backward(float2* __restrict__ X, const float2* __restrict__ O,
              const float2* __restrict__ P, Batch bt, Disk dk, PupilGeom pg, int chunks,
              float2* __restrict__ gO, float2* __restrict__ gP, double* __restrict__ zpart,
              const float* __restrict__ kappa_tab, const float2* __restrict__ tw) {
  constexpr int T = BwdRow<N>::T;
  constexpr int E = N / T;
  constexpr int L = BwdRow<N>::threads / T;
  constexpr bool kNeedC = MODE == kGradOP || MODE == kPatchZern;
  __shared__ float2 lds[L * RowLds<N>::kStride];
  __shared__ float2 lds_tw[N];
  int b, c;
  const bool live = xcd_map(blockIdx.x, chunks, bt.B, b, c);
  const int line = threadIdx.x / T;
  const int t = threadIdx.x % T;
  const int rr = c * L + line;
  const bool active = rr < dk.nrows;
  const int ky = dk.ky_lo + (active ? rr : 0);
  float zs[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // row sums of g_theta x^a, g_theta kappa
  if (live) {
    float2* xr = X + ((size_t)b * N + ky) * N;
    const int2 ext = disk_extent<N>(dk, ky);
    const int2 w = bt.win[b];
    const size_t orow = (size_t)(w.x + ky) * bt.M + w.y;
    const float2* prow = P + (size_t)ky * N;
    float2 v[E], pv[E], cv[kNeedC ? E : 1];
    float kap[MODE == kPatchZern ? E : 1];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = xr[t + m * T];   // rows past the disk are never used
    // the pupil, the cropped spectrum and kappa at this thread's output columns,
    // fetched before the transform at addresses clamped into the disk
    const int uy = ky - N / 2;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kx = min(max(half_shift<N>(t + m * T), ext.x), ext.y);
      pv[m] = prow[kx];
      if constexpr (kNeedC) cv[m] = O[orow + kx];
      if constexpr (MODE == kPatchZern) {
        const int ux = kx - N / 2;
        kap[m] = kappa_tab[ux * ux + uy * uy];
      }
    }
    stage_twiddles_after_loads<N, BwdRow<N>::threads>(lds_tw, tw);
    PlanT<N, T>::template run<-1>(v, t, lds + line * RowLds<N>::kStride, [](int n) { return RowLds<N>::at(n); }, lds_tw);
    if (active) {
      const float ir = (float)pg.inv_r;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int kx = half_shift<N>(t + m * T);
        if (kx >= ext.x && kx <= ext.y) {
          const float2 g = v[m];
          const float2 p = pv[m];
          if constexpr (MODE == kGradO || MODE == kGradOP) {
            atomic_add_c(gO + orow + kx, cmulc(p, g));
          } else {
            store_next<N>(xr + kx, cmulc(p, g));   // this row was read whole into registers above
          }
          if constexpr (MODE == kGradOP) {
            atomic_add_c(gP + (size_t)ky * N + kx, cmulc(cv[m], g));
          } else if constexpr (MODE == kPatchZern) {
            add_row_moments(g, p, cv[m], (float)(kx - N / 2) * ir, kap[m], zs);
          }
        }
      }
    }
  }
  if constexpr (MODE == kPatchZern)
    row_moment_partials<T, L>(zs, c * L, dk, N / 2, (float)pg.inv_r, zpart);
}

}  // namespace fpm
