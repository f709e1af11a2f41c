// fft_line.hpp - register and LDS building blocks of the complex64 FFTs.
//
// A "line" is one 1-D transform of length N done by a team of T threads of
// one workgroup; thread t of the team holds E = N/T elements in registers,
// element m being x[t + m*T] on entry and X[t + m*T] on exit. Stages are
// Stockham auto-sort stages of radix R (E/R butterflies per thread per
// stage); between stages the team exchanges through LDS. The last stage
// writes straight back into the same register slots, so an s-stage
// transform makes s-1 LDS round trips.
//
// Direction DIR = -1 is the forward DFT X[k] = sum_n x[n] e^{-2 pi i k n / N},
// DIR = +1 the unnormalised inverse.
#pragma once
#include <hip/hip_runtime.h>

namespace fpm {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// cos and sin of 2 pi m / 48: every root of unity the radices 2,3,4,6,8,12,16 need.
__device__ constexpr double kCos48[48] = {
    1,
    0.99144486137381038,
    0.96592582628906831,
    0.92387953251128674,
    0.86602540378443871,
    0.79335334029123517,
    0.70710678118654757,
    0.60876142900872066,
    0.50000000000000011,
    0.38268343236508984,
    0.25881904510252074,
    0.13052619222005171,
    6.123233995736766e-17,
    -0.1305261922200516,
    -0.25881904510252063,
    -0.3826834323650895,
    -0.49999999999999978,
    -0.60876142900872066,
    -0.70710678118654746,
    -0.79335334029123505,
    -0.86602540378443871,
    -0.92387953251128674,
    -0.9659258262890682,
    -0.99144486137381038,
    -1,
    -0.99144486137381038,
    -0.96592582628906831,
    -0.92387953251128685,
    -0.86602540378443882,
    -0.79335334029123517,
    -0.70710678118654791,
    -0.60876142900872088,
    -0.50000000000000044,
    -0.3826834323650895,
    -0.25881904510252063,
    -0.13052619222005163,
    -1.8369701987210297e-16,
    0.13052619222005127,
    0.2588190451025203,
    0.38268343236508917,
    0.50000000000000011,
    0.60876142900871988,
    0.70710678118654735,
    0.79335334029123494,
    0.86602540378443837,
    0.92387953251128685,
    0.96592582628906809,
    0.99144486137381038
};
__device__ constexpr double kSin48[48] = {
    0,
    0.13052619222005157,
    0.25881904510252074,
    0.38268343236508978,
    0.49999999999999994,
    0.60876142900872066,
    0.70710678118654746,
    0.79335334029123517,
    0.8660254037844386,
    0.92387953251128674,
    0.96592582628906831,
    0.99144486137381038,
    1,
    0.99144486137381038,
    0.96592582628906831,
    0.92387953251128685,
    0.86602540378443871,
    0.79335334029123517,
    0.70710678118654757,
    0.60876142900872088,
    0.49999999999999994,
    0.38268343236508989,
    0.25881904510252102,
    0.13052619222005199,
    1.2246467991473532e-16,
    -0.13052619222005177,
    -0.25881904510252079,
    -0.38268343236508967,
    -0.49999999999999972,
    -0.60876142900872066,
    -0.70710678118654713,
    -0.79335334029123494,
    -0.86602540378443837,
    -0.92387953251128685,
    -0.96592582628906831,
    -0.99144486137381038,
    -1,
    -0.99144486137381049,
    -0.96592582628906842,
    -0.92387953251128696,
    -0.8660254037844386,
    -0.79335334029123572,
    -0.70710678118654768,
    -0.60876142900872088,
    -0.50000000000000044,
    -0.38268343236508956,
    -0.25881904510252157,
    -0.13052619222005168
};

// a * exp(DIR * 2 pi i * m / 48) for a compile-time m (trivial rotations folded).
template <int DIR, int M48>
__device__ __forceinline__ float2 rot48(float2 a) {
  constexpr int m = ((M48 % 48) + 48) % 48;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 12) {          // * (DIR i)
    return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
  } else if constexpr (m == 24) {          // * -1
    return make_float2(-a.x, -a.y);
  } else if constexpr (m == 36) {          // * (-DIR i)
    return DIR > 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
  } else {
    constexpr float c = (float)kCos48[m];
    constexpr float s = (float)(DIR * kSin48[m]);
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

template <int I, int N> struct For {
  template <class F> __device__ __forceinline__ static void run(F&& f) {
    if constexpr (I < N) {
      f(std::integral_constant<int, I>{});
      For<I + 1, N>::run(f);
    }
  }
};

// In-place DFT of R points held in x[0..R-1] (natural order in and out).
template <int R, int DIR> struct Dft;

template <int DIR> struct Dft<1, DIR> {
  __device__ __forceinline__ static void run(float2*) {}
};

template <int DIR> struct Dft<2, DIR> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int DIR> struct Dft<3, DIR> {
  __device__ __forceinline__ static void run(float2* x) {
    constexpr float h = 0.86602540378443865f * DIR;   // DIR sin(2 pi / 3)
    float2 t1 = cadd(x[1], x[2]);
    float2 t2 = csub(x[1], x[2]);
    float2 y0 = cadd(x[0], t1);
    float2 m = make_float2(x[0].x - 0.5f * t1.x, x[0].y - 0.5f * t1.y);
    float2 r = make_float2(-h * t2.y, h * t2.x);     // i h t2
    x[0] = y0;
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
  }
};

template <int DIR> struct Dft<4, DIR> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 a0 = cadd(x[0], x[2]);
    float2 a1 = csub(x[0], x[2]);
    float2 a2 = cadd(x[1], x[3]);
    float2 a3 = rot48<DIR, 12>(csub(x[1], x[3]));
    x[0] = cadd(a0, a2);
    x[2] = csub(a0, a2);
    x[1] = cadd(a1, a3);
    x[3] = csub(a1, a3);
  }
};

// R = R1 * R2: input index n = n1 + R1 n2, output index k = k2 + R2 k1.
template <int R1, int R2, int DIR> struct DftComposite {
  __device__ __forceinline__ static void run(float2* x) {
    constexpr int R = R1 * R2;
    float2 t[R];
    For<0, R1>::run([&](auto n1c) {
      constexpr int n1 = decltype(n1c)::value;
      float2 u[R2];
      For<0, R2>::run([&](auto n2c) { u[decltype(n2c)::value] = x[n1 + R1 * decltype(n2c)::value]; });
      Dft<R2, DIR>::run(u);
      For<0, R2>::run([&](auto k2c) {
        constexpr int k2 = decltype(k2c)::value;
        t[n1 + R1 * k2] = rot48<DIR, (48 / R) * n1 * k2>(u[k2]);
      });
    });
    For<0, R2>::run([&](auto k2c) {
      constexpr int k2 = decltype(k2c)::value;
      float2 u[R1];
      For<0, R1>::run([&](auto n1c) { u[decltype(n1c)::value] = t[decltype(n1c)::value + R1 * k2]; });
      Dft<R1, DIR>::run(u);
      For<0, R1>::run([&](auto k1c) { x[k2 + R2 * decltype(k1c)::value] = u[decltype(k1c)::value]; });
    });
  }
};

template <int DIR> struct Dft<6, DIR> : DftComposite<2, 3, DIR> {};
template <int DIR> struct Dft<8, DIR> : DftComposite<2, 4, DIR> {};
template <int DIR> struct Dft<12, DIR> : DftComposite<4, 3, DIR> {};
template <int DIR> struct Dft<16, DIR> : DftComposite<4, 4, DIR> {};

// ---------------------------------------------------------------------------
// Line transform. Lay maps an element index n in [0, N) to an LDS slot.
// tw: table of exp(-2 pi i m / N), m in [0, N), computed in FP64 on the host.

template <int N, int T, int DIR, int P, int R, int... Rest>
struct Stages {
  template <class Lay>
  __device__ __forceinline__ static void run(float2 (&v)[N / T], int t, float2* lds, Lay lay,
                                             const float2* __restrict__ tw) {
    constexpr int E = N / T;
    constexpr int Q = E / R;
    static_assert(E % R == 0, "elements per thread must be a multiple of the radix");
    constexpr bool kLast = sizeof...(Rest) == 0;
    static_assert(!kLast || P * R == N, "radices must multiply to N");
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = t + q * T;
      const int k = i % P;
      float2 x[R];
#pragma unroll
      for (int j = 0; j < R; ++j) x[j] = v[q + j * Q];
      if constexpr (P > 1) {
#pragma unroll
        for (int j = 1; j < R; ++j) {
          float2 w = tw[j * k * (N / (P * R))];
          if constexpr (DIR > 0) w.y = -w.y;
          x[j] = cmul(x[j], w);
        }
      }
      Dft<R, DIR>::run(x);
      if constexpr (kLast) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[q + r * Q] = x[r];
      } else {
        const int base = (i - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lay(base + r * P)] = x[r];
      }
    }
    if constexpr (!kLast) {
      __syncthreads();
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = lds[lay(t + m * T)];
      __syncthreads();
      Stages<N, T, DIR, P * R, Rest...>::run(v, t, lds, lay, tw);
    }
  }
};

// LDS layout of one line in the row passes: one padding slot after every 16
// elements, so the first Stockham stage's writes (stride 16) and the strided
// reads hit distinct banks.
template <int N> struct RowLds {
  static constexpr int kStride = N + N / 16;   // slots per line
  __device__ __forceinline__ static int at(int n) { return n + (n >> 4); }
};

// Copy the twiddle table into LDS, by a workgroup of exactly kThreads threads
// (call before the first transform; the first stage needs no twiddles and its
// exchange barrier orders these writes before any twiddle read). Unrolled and
// without a branch (threads past the table copy its last entry again, the same
// value to the same slot), and called after the kernel's first data loads:
// the twiddle loads then join them in flight, where a loop or a branch would
// end the scheduling region and the data loads would wait for the twiddles.
template <int N, int kThreads>
__device__ __forceinline__ void stage_twiddles_after_loads(float2* __restrict__ lds_tw,
                                                           const float2* __restrict__ tw) {
  constexpr int K = (N + kThreads - 1) / kThreads;
  float2 r[K];
#pragma unroll
  for (int k = 0; k < K; ++k) r[k] = tw[min((int)threadIdx.x + k * kThreads, N - 1)];
#pragma unroll
  for (int k = 0; k < K; ++k) lds_tw[min((int)threadIdx.x + k * kThreads, N - 1)] = r[k];
}

// Radix plans: stage radices for a transform of length N done by T threads.
template <int N, int T> struct PlanT;

#define FPM_PLAN(N_, T_, ...)                                                            \
  template <> struct PlanT<N_, T_> {                                                     \
    static constexpr int T = T_;                                                         \
    template <int DIR, class Lay>                                                        \
    __device__ __forceinline__ static void run(float2 (&v)[N_ / T_], int t, float2* lds, \
                                               Lay lay, const float2* tw) {              \
      Stages<N_, T_, DIR, 1, __VA_ARGS__>::run(v, t, lds, lay, tw);                      \
    }                                                                                    \
  };

FPM_PLAN(64, 4, 16, 4)
FPM_PLAN(64, 8, 8, 8)
FPM_PLAN(64, 16, 4, 4, 4)
FPM_PLAN(128, 8, 16, 8)
FPM_PLAN(128, 16, 8, 4, 4)
FPM_PLAN(128, 32, 4, 4, 4, 2)
FPM_PLAN(256, 16, 16, 16)
FPM_PLAN(256, 32, 8, 4, 8)
FPM_PLAN(256, 64, 4, 4, 4, 4)
FPM_PLAN(512, 32, 16, 16, 2)
FPM_PLAN(512, 64, 8, 8, 8)
FPM_PLAN(512, 128, 4, 4, 4, 4, 2)
FPM_PLAN(1024, 64, 16, 8, 8)
FPM_PLAN(2048, 128, 16, 16, 8)
// 3 * 2^k sizes: 12 elements per thread (24 for 1536), one radix-12 stage
FPM_PLAN(192, 16, 12, 4, 4)
FPM_PLAN(384, 32, 12, 4, 4, 2)
FPM_PLAN(768, 64, 12, 4, 4, 4)
FPM_PLAN(1536, 64, 12, 8, 4, 4)
#undef FPM_PLAN

// Default threads per line: 16 elements per thread where the radices allow,
// 12 (or 24) for the sizes with a factor 3.
template <int N> struct DefaultT {
  static constexpr int value = N <= 128 ? 8 : N == 256 ? 16 : N == 512 ? 64 : N / 16;
};
template <> struct DefaultT<192> { static constexpr int value = 16; };
template <> struct DefaultT<384> { static constexpr int value = 32; };
template <> struct DefaultT<768> { static constexpr int value = 64; };
template <> struct DefaultT<1536> { static constexpr int value = 64; };
template <int N> using Plan1D = PlanT<N, DefaultT<N>::value>;

}  // namespace fpm
