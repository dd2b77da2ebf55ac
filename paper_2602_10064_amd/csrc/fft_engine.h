// Stockham FFT engine for gfx950, staged in LDS.
//
// A transform of length N is done by a group of G threads.  Stage j with
// radix R and sub-transform length P (product of the earlier radices)
// computes N/R butterflies; butterfly b reads src[b + r N/R] (r < R), applies
// the twiddles W_{PR}^{r (b mod P)}, does an R-point DFT and writes
// dst[(b div P) P R + (b mod P) + r P].  After the last stage the output is in
// natural order (autosort).  Consecutive threads read consecutive addresses,
// which keeps every stage's reads conflict-free in LDS.
//
// Sign convention: forward uses exp(-2 pi i n k / N) (the same kernel as the
// structure-factor phase exp(-2 pi i k.r_j)), inverse exp(+2 pi i n k / N);
// neither is normalised.  Twiddles come from a table tw[m] = exp(-2 pi i m/N)
// computed in FP64 and rounded to FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace tacaw {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Small DFTs on registers, in place.  INV selects the sign of the exponent.
// ---------------------------------------------------------------------------
template <bool INV>
__device__ __forceinline__ void dft2(float2* x) {
  float2 a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2* x) {
  const float s = 0.86602540378443864676f;  // sin(2 pi / 3)
  float2 t1 = cadd(x[1], x[2]);
  float2 t2 = make_float2(x[0].x - 0.5f * t1.x, x[0].y - 0.5f * t1.y);
  float2 d = cscale(csub(x[1], x[2]), s);
  float2 rd = rot90<INV>(d);
  x[0] = cadd(x[0], t1);
  x[1] = cadd(t2, rd);
  x[2] = csub(t2, rd);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2* x) {
  float2 a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
  float2 c = cadd(x[1], x[3]), d = rot90<INV>(csub(x[1], x[3]));
  x[0] = cadd(a, c);
  x[2] = csub(a, c);
  x[1] = cadd(b, d);
  x[3] = csub(b, d);
}

template <bool INV>
__device__ __forceinline__ void dft5(float2* x) {
  const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
  const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
  const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
  const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
  float2 a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
  float2 a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
  float2 x0 = x[0];
  float2 r1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
  float2 r2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
  float2 i1 = rot90<INV>(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
  float2 i2 = rot90<INV>(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
  x[0] = cadd(x0, cadd(a1, a2));
  x[1] = cadd(r1, i1);
  x[4] = csub(r1, i1);
  x[2] = cadd(r2, i2);
  x[3] = csub(r2, i2);
}

// 6-point DFT: two 3-point DFTs (even and odd inputs), the odd outputs
// rotated by W6^k, then 2-point butterflies.
template <bool INV>
__device__ __forceinline__ void dft6(float2* x) {
  const float h = 0.5f, s = 0.86602540378443864676f;
  float2 e[3] = {x[0], x[2], x[4]};
  float2 o[3] = {x[1], x[3], x[5]};
  dft3<INV>(e);
  dft3<INV>(o);
  // W6^1 = (1/2, -s), W6^2 = (-1/2, -s) forward; conjugates inverse
  const float sg = INV ? s : -s;
  const float2 o1 = make_float2(h * o[1].x - sg * o[1].y, h * o[1].y + sg * o[1].x);
  const float2 o2 = make_float2(-h * o[2].x - sg * o[2].y, -h * o[2].y + sg * o[2].x);
  x[0] = cadd(e[0], o[0]);
  x[3] = csub(e[0], o[0]);
  x[1] = cadd(e[1], o1);
  x[4] = csub(e[1], o1);
  x[2] = cadd(e[2], o2);
  x[5] = csub(e[2], o2);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* x) {
  const float h = 0.70710678118654752440f;
  float2 e[4] = {x[0], x[2], x[4], x[6]};
  float2 o[4] = {x[1], x[3], x[5], x[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // W8^1, W8^2, W8^3 (forward: exp(-i pi/4 k))
  float2 o1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                  : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
  float2 o2 = rot90<INV>(o[2]);
  float2 o3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                  : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
  x[0] = cadd(e[0], o[0]);
  x[4] = csub(e[0], o[0]);
  x[1] = cadd(e[1], o1);
  x[5] = csub(e[1], o1);
  x[2] = cadd(e[2], o2);
  x[6] = csub(e[2], o2);
  x[3] = cadd(e[3], o3);
  x[7] = csub(e[3], o3);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2* x) {
  if constexpr (R == 2) dft2<INV>(x);
  else if constexpr (R == 3) dft3<INV>(x);
  else if constexpr (R == 4) dft4<INV>(x);
  else if constexpr (R == 5) dft5<INV>(x);
  else if constexpr (R == 6) dft6<INV>(x);
  else if constexpr (R == 8) dft8<INV>(x);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// One Stockham butterfly: reads R inputs, twiddles, DFT, writes R outputs.
// N, R, P are compile-time in the fixed-size engine.
// ---------------------------------------------------------------------------
template <int N, int R, int P, bool INV>
__device__ __forceinline__ void butterfly_ct(const float2* __restrict__ src, float2* __restrict__ dst,
                                             const float2* __restrict__ tw, int b) {
  constexpr int S = N / R;
  float2 x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = src[b + r * S];
  const int k = b % P;
  if constexpr (P > 1) {
    constexpr int STEP = N / (P * R);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      float2 w = tw[r * k * STEP];
      x[r] = INV ? cmulc(x[r], w) : cmul(x[r], w);
    }
  }
  dft<R, INV>(x);
  const int base = (b - k) * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[base + r * P] = x[r];
}

template <int... Rs>
struct Radices {};

// Runs the stages of Radices<R, Rest...> with ping-pong buffers; returns the
// buffer that holds the result.  Every stage ends with a workgroup barrier, so
// all thread groups of the workgroup must call it together.
template <int N, int G, bool INV, int P, typename Rad>
struct Stages;

template <int N, int G, bool INV, int P>
struct Stages<N, G, INV, P, Radices<>> {
  __device__ __forceinline__ static float2* run(float2* src, float2*, const float2*, int) { return src; }
};

template <int N, int G, bool INV, int P, int R, int... Rest>
struct Stages<N, G, INV, P, Radices<R, Rest...>> {
  __device__ __forceinline__ static float2* run(float2* src, float2* dst, const float2* tw, int t) {
    constexpr int S = N / R;
    constexpr int ITER = (S + G - 1) / G;
#pragma unroll
    for (int q = 0; q < ITER; ++q) {
      const int b = t + q * G;
      if ((S % G) == 0 || b < S) butterfly_ct<N, R, P, INV>(src, dst, tw, b);
    }
    __syncthreads();
    return Stages<N, G, INV, P * R, Radices<Rest...>>::run(dst, src, tw, t);
  }
};

// In-place variant: every thread keeps all of its butterflies of a stage in
// registers between a read phase and a write phase, so one LDS buffer of N
// values suffices.  Two workgroup barriers per stage.
template <int N, int G, bool INV, int P, typename Rad>
struct StagesIP;

template <int N, int G, bool INV, int P>
struct StagesIP<N, G, INV, P, Radices<>> {
  __device__ __forceinline__ static void run(float2*, const float2*, int) {}
};

template <int N, int G, bool INV, int P, int R, int... Rest>
struct StagesIP<N, G, INV, P, Radices<R, Rest...>> {
  __device__ __forceinline__ static void run(float2* buf, const float2* tw, int t) {
    constexpr int S = N / R;
    constexpr int NB = (S + G - 1) / G;
    float2 x[NB][R];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int b = t + q * G;
      if ((S % G) == 0 || b < S) {
#pragma unroll
        for (int r = 0; r < R; ++r) x[q][r] = buf[b + r * S];
        if constexpr (P > 1) {
          constexpr int STEP = N / (P * R);
          const int k = b % P;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = tw[r * k * STEP];
            x[q][r] = INV ? cmulc(x[q][r], w) : cmul(x[q][r], w);
          }
        }
        dft<R, INV>(x[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int b = t + q * G;
      if ((S % G) == 0 || b < S) {
        const int k = b % P;
        const int base = (b - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[base + r * P] = x[q][r];
      }
    }
    __syncthreads();
    StagesIP<N, G, INV, P * R, Radices<Rest...>>::run(buf, tw, t);
  }
};

template <int A, int... B>
struct Product {
  static constexpr int value = A * Product<B...>::value;
};
template <int A>
struct Product<A> {
  static constexpr int value = A;
};

// ---------------------------------------------------------------------------
// Fixed-size plans: radix sequence and threads per transform (G divides every
// N/R so no butterfly loop has a ragged tail).
// ---------------------------------------------------------------------------
template <int N>
struct Plan;
#define TACAW_PLAN(NN, GG, ...)                                         \
  template <>                                                           \
  struct Plan<NN> {                                                     \
    static constexpr int G = GG;                                        \
    using R = Radices<__VA_ARGS__>;                                     \
    static_assert(Product<__VA_ARGS__>::value == NN, "plan product");   \
  };
TACAW_PLAN(16, 4, 4, 4)
TACAW_PLAN(32, 4, 8, 4)
TACAW_PLAN(48, 4, 4, 4, 3)
TACAW_PLAN(64, 8, 8, 8)
TACAW_PLAN(96, 4, 8, 4, 3)
TACAW_PLAN(128, 16, 8, 4, 4)
TACAW_PLAN(160, 4, 8, 4, 5)
TACAW_PLAN(192, 8, 8, 8, 3)
TACAW_PLAN(256, 32, 8, 8, 4)
TACAW_PLAN(320, 8, 8, 8, 5)
TACAW_PLAN(384, 16, 8, 4, 4, 3)
TACAW_PLAN(512, 64, 8, 8, 8)
TACAW_PLAN(640, 16, 8, 4, 4, 5)
TACAW_PLAN(768, 32, 8, 8, 4, 3)
TACAW_PLAN(1024, 64, 8, 8, 4, 4)
TACAW_PLAN(2048, 64, 8, 8, 8, 4)
#undef TACAW_PLAN

// ---------------------------------------------------------------------------
// Runtime-radix engine (time axis: any 2*3*5-smooth length).  The plan is a
// list of radices; P and the twiddle stride are computed as the stages go.
// ---------------------------------------------------------------------------
template <int R, bool INV>
__device__ __forceinline__ void butterfly_rt(const float2* __restrict__ src, float2* __restrict__ dst,
                                             const float2* __restrict__ tw, int n, int p, int b) {
  const int s = n / R;
  float2 x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = src[b + r * s];
  const int k = b % p;
  if (p > 1) {
    const int step = n / (p * R);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      float2 w = tw[r * k * step];
      x[r] = INV ? cmulc(x[r], w) : cmul(x[r], w);
    }
  }
  dft<R, INV>(x);
  const int base = (b - k) * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[base + r * p] = x[r];
}

// Radix sequence of the runtime engine: 8s, then a 4, then a 2, then 3s,
// then 5s (n must be 2*3*5-smooth).
__host__ __device__ __forceinline__ int rt_next_radix(int rem) {
  if (rem % 8 == 0) return 8;
  if (rem % 4 == 0) return 4;
  if (rem % 2 == 0) return 2;
  if (rem % 3 == 0) return 3;
  return 5;
}

// G threads (index t) transform one sequence of length n; all groups of the
// workgroup call together (one barrier per stage).  Returns the buffer that
// holds the result.
template <bool INV>
__device__ float2* stockham_rt(int n, float2* src, float2* dst, const float2* tw, int t, int G) {
  int p = 1;
  int rem = n;
  while (rem > 1) {
    const int R = rt_next_radix(rem);
    const int s = n / R;
    for (int b = t; b < s; b += G) {
      switch (R) {
        case 2: butterfly_rt<2, INV>(src, dst, tw, n, p, b); break;
        case 3: butterfly_rt<3, INV>(src, dst, tw, n, p, b); break;
        case 4: butterfly_rt<4, INV>(src, dst, tw, n, p, b); break;
        case 5: butterfly_rt<5, INV>(src, dst, tw, n, p, b); break;
        default: butterfly_rt<8, INV>(src, dst, tw, n, p, b); break;
      }
    }
    __syncthreads();
    float2* tmp = src;
    src = dst;
    dst = tmp;
    p *= R;
    rem /= R;
  }
  return src;
}

}  // namespace tacaw
