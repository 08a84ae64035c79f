// Device-side building blocks: the counter-based generator, the integer maps
// that turn its words into indices, lengths and masks, and the fitness terms.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "de_internal.h"

namespace de {

// Pointers into device memory are carried as generic pointers in the run
// records; re-qualifying them as global lets the compiler use global (not
// flat) memory instructions, whose loads it can keep in flight together.
// (The host compilation pass only parses device code; it sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define DE_GLOBAL __attribute__((address_space(1)))
#else
#define DE_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ const DE_GLOBAL T* gconst(const void* p) {
  return (const DE_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ DE_GLOBAL T* gmut(void* p) {
  return (DE_GLOBAL T*)p;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten S-box rounds on a
// 128-bit counter; each round multiplies words 0 and 2 by the two Philox
// constants, and the two-word key advances by the Weyl constants between
// rounds.  The 64-bit products give high and low halves in one multiply.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t q = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = static_cast<uint32_t>(q >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(p >> 32) ^ c3 ^ k1;
    c1 = static_cast<uint32_t>(q);
    c3 = static_cast<uint32_t>(p);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// Block `blk` of stream `tag` for individual i in generation g of run `run`.
__device__ __forceinline__ uint4 draw(const RunDev& P, uint32_t tag, uint32_t g, uint32_t i,
                                      uint32_t blk) {
  return philox(blk, i, g, (tag << 24) | (P.run_id & 0xFFFFFFu), P.key0, P.key1);
}

__device__ __forceinline__ uint32_t word_of(const uint4& b, int k) {
  return k == 0 ? b.x : k == 1 ? b.y : k == 2 ? b.z : b.w;
}

// floor(n * w / 2^32): an index in [0, n).
__device__ __forceinline__ uint32_t scale_index(uint32_t w, uint32_t n) {
  return static_cast<uint32_t>((static_cast<uint64_t>(w) * n) >> 32);
}

// Base r0 and difference pair r1, r2 of DE/rand/1, all distinct and != i:
// draw from the shrunken range, then step over the excluded rows in
// increasing order.
__device__ __forceinline__ void pick_indices(uint4 b, uint32_t N, uint32_t i, uint32_t& r0,
                                             uint32_t& r1, uint32_t& r2) {
  r0 = scale_index(b.x, N - 1);
  r0 += (r0 >= i);
  const uint32_t a = min(i, r0), c = max(i, r0);
  r1 = scale_index(b.y, N - 2);
  r1 += (r1 >= a);
  r1 += (r1 >= c);
  uint32_t e0 = a, e1 = c, e2 = r1;  // sort three excluded rows
  if (e2 < e1) { uint32_t t = e1; e1 = e2; e2 = t; }
  if (e1 < e0) { uint32_t t = e0; e0 = e1; e1 = t; }
  r2 = scale_index(b.z, N - 3);
  r2 += (r2 >= e0);
  r2 += (r2 >= e1);
  r2 += (r2 >= e2);
}

// Keyed pseudo-random permutation of [0, N) for generation g (the shuffle of
// Alg 2 and Alg 5's base permutation): an eight-round balanced Feistel
// network on m-bit integers (m even, 2^m >= N, m >= 2) whose round r mixes
// the right half with K_r, word r%4 of Philox block r/4 (individual 0); the
// image is walked through the permutation until it lands in [0, N).  A walk
// ends at the latest when it returns to k, after at most 2^m < 4N steps.
__device__ __forceinline__ uint32_t perm_mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ uint32_t permute(const RunDev& P, uint32_t tag, uint32_t g, uint32_t N,
                                            uint32_t k) {
  uint32_t m = 2;
  while ((1u << m) < N) m += 2;
  const uint32_t h = m / 2, hmask = (1u << h) - 1u;
  const uint4 a = draw(P, tag, g, 0, 0);
  const uint4 b = draw(P, tag, g, 0, 1);
  const uint32_t K[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  uint32_t x = k;
  for (uint32_t step = 0; step < (1u << m); ++step) {
    uint32_t L = x >> h, R = x & hmask;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t t = L ^ (perm_mix(R ^ K[r]) & hmask);
      L = R;
      R = t;
    }
    x = (L << h) | R;
    if (x < N) break;
  }
  return x < N ? x : k;  // always x < N: the cycle through k returns within 2^m steps
}

// Storage row of position k in generation g (identity without the shuffle).
__device__ __forceinline__ uint32_t row_of(const RunDev& P, uint32_t g, uint32_t k) {
  return P.shuffle ? permute(P, TAG_SHUFFLE, g, static_cast<uint32_t>(P.N), k) : k;
}

// r0, r1, r2 (positions) of position k under the run's base scheme: the
// classic distinct rule, or Alg 3 / 4 / 5 for r0 with Alg 6's offsets
// o = 1 + randint(N - 1) for r1 = r0 + o1 and r2 = r1 + o2 (mod N).
__device__ __forceinline__ void pick_scheme(const RunDev& P, uint32_t g, uint32_t k, uint32_t N,
                                            uint32_t& r0, uint32_t& r1, uint32_t& r2) {
  const uint4 b = draw(P, TAG_IDX, g, k, 0);
  if (P.base == BASE_CLASSIC) {
    pick_indices(b, N, k, r0, r1, r2);
    return;
  }
  if (P.base == BASE_RANDOM) {
    r0 = scale_index(b.x, N);
  } else if (P.base == BASE_OFFSET) {
    const uint32_t rg = 1 + scale_index(draw(P, TAG_OFFSET, g, 0, 0).x, N - 1);
    r0 = k + rg >= N ? k + rg - N : k + rg;
  } else {
    r0 = permute(P, TAG_PERM, g, N, k);
  }
  const uint32_t o1 = 1 + scale_index(b.y, N - 1);
  const uint32_t o2 = 1 + scale_index(b.z, N - 1);
  r1 = r0 + o1 >= N ? r0 + o1 - N : r0 + o1;
  r2 = r1 + o2 >= N ? r1 + o2 - N : r1 + o2;
}

// NEC run length from word w: the number of k in [1, D] with w < T[k], where
// T[k] is the number of words whose uniform (w + 1/2) 2^-32 lies below
// CR^(k-1) (the power as a running FP64 product).  T decreases in k, so the k
// that pass form a prefix: each lane of the wavefront tests one k, 64 at a
// time (one coalesced load of the table), and the run length is the count.
// Must be called by the whole wavefront with the same w.
// The table words the first step of nec_length needs (lane l: T[1 + l],
// clamped to the last entry T[D + 1]), loaded on their own so that a caller
// can issue the load early and overlap it with other memory traffic.
__device__ __forceinline__ uint64_t nec_prefetch(const RunDev& P) {
  const uint32_t D = static_cast<uint32_t>(P.D);
  const uint32_t k = 1 + __lane_id();
  return gconst<uint64_t>(P.T)[k <= D ? k : D + 1];
}

__device__ __forceinline__ uint32_t nec_length(const RunDev& P, uint32_t w, uint64_t t1) {
  const uint32_t D = static_cast<uint32_t>(P.D);
  if (P.inv_ln_cr == 0.0) return P.CR >= 1.0 ? D : 1u;
  const uint32_t lane = __lane_id();
  const uint64_t ww = w;
  uint32_t L = static_cast<uint32_t>(__popcll(__ballot(1 + lane <= D && ww < t1)));
  if (L < 64) return L;
  const DE_GLOBAL uint64_t* T = gconst<uint64_t>(P.T);
  for (uint32_t k0 = 65; k0 <= D; k0 += 64) {
    const uint32_t k = k0 + lane;
    const bool in = k <= D && ww < T[k];
    const uint32_t n = static_cast<uint32_t>(__popcll(__ballot(in)));
    L += n;
    if (n < 64) break;
  }
  return L;
}

__device__ __forceinline__ uint32_t nec_length(const RunDev& P, uint32_t w) {
  return nec_length(P, w, nec_prefetch(P));
}

// Classic exponential crossover length (Alg 8), draws taken one at a time in
// order: draw e (EXP block e/4, word e%4) decides whether element e+2 joins.
// With CR = 1 every draw passes (L = D), with CR = 0 the first one fails
// (L = 1): both lengths are known without drawing.
__device__ __forceinline__ uint32_t exp_length_serial(const RunDev& P, uint32_t g, uint32_t i) {
  const uint32_t D = static_cast<uint32_t>(P.D);
  if (P.thr >= 4294967296ull) return D;
  if (P.thr == 0) return 1;
  uint32_t L = 1;
  uint4 b = make_uint4(0, 0, 0, 0);
  for (uint32_t e = 0; L < D; ++e) {
    if ((e & 3u) == 0) b = draw(P, TAG_EXP, g, i, e >> 2);
    if (static_cast<uint64_t>(word_of(b, e & 3u)) < P.thr) ++L;
    else break;
  }
  return L;
}

// The same length found 256 draws at a time by one wavefront: each lane tests
// one Philox block (4 draws) and the lowest failing draw ends the run.
__device__ __forceinline__ uint32_t exp_length_scan(const RunDev& P, uint32_t g, uint32_t i) {
  const uint32_t D = static_cast<uint32_t>(P.D);
  if (P.thr >= 4294967296ull) return D;
  if (P.thr == 0) return 1;
  const uint32_t lane = __lane_id();
  for (uint32_t base = 0; base + 1 < D; base += 256) {
    const uint32_t e0 = base + 4 * lane;
    const uint4 b = draw(P, TAG_EXP, g, i, e0 >> 2);
    uint32_t fail = 4;
#pragma unroll
    for (int k = 3; k >= 0; --k)
      if (static_cast<uint64_t>(word_of(b, k)) >= P.thr) fail = k;
    const bool hit = fail < 4 && e0 + fail + 1 < D;
    const uint64_t bal = __ballot(hit);
    if (bal) {
      const uint32_t first = __ffsll(static_cast<unsigned long long>(bal)) - 1;
      const uint32_t f = __shfl(fail, first);
      return base + 4 * first + f + 1;  // draws 0..e-1 passed, draw e failed: L = e + 1
    }
  }
  return D;
}

// ---- fitness terms --------------------------------------------------------
template <typename T> struct Math;
template <> struct Math<double> {
  static __device__ __forceinline__ double fma_(double a, double b, double c) {
    return __builtin_fma(a, b, c);
  }
  static __device__ __forceinline__ double cos_(double x) { return cos(x); }
  static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
  static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }
  static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
};
template <> struct Math<float> {
  static __device__ __forceinline__ float fma_(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
  }
  static __device__ __forceinline__ float cos_(float x) { return cosf(x); }
  static __device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
  static __device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
  static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
};

// sin^2(pi z) without a library call.  r = z - rint(z) lies in [-1/2, 1/2]
// and is exact; sin(pi r) = r * P(r^2), summed by Horner's rule.  FP64: P is
// the degree-8 minimax polynomial of sin(pi sqrt(t)) / sqrt(t) on [0, 1/4]
// for the relative error (a Remez fit, paper_2101_06599_amd/fit_sinpi.py;
// approximation error 2.6e-19), so the rounding of the evaluation decides
// the accuracy: the evaluated sin^2 stays within 2.1 ulp (20 sin^2 within
// 2.9 ulp).  FP32: the Taylor series of sine, c_k = (-1)^k pi^(2k+1) /
// (2k+1)!, through k = 6 (dropped terms below 1e-9).  sin^2(pi z) =
// sin^2(pi r) because sine changes only its sign between the two.  NaN and
// infinities give NaN.
__device__ __forceinline__ double sinpi_sq(double z) {
  const double r = z - __builtin_rint(z);
  const double t = r * r;
  double p = 0x1.9d1b869195c75p-21;
  p = __builtin_fma(p, t, -0x1.6f79770c2d50fp-16);
  p = __builtin_fma(p, t, 0x1.e8f35e9d58319p-12);
  p = __builtin_fma(p, t, -0x1.e3074ddd1d695p-8);
  p = __builtin_fma(p, t, 0x1.50783485190cap-4);
  p = __builtin_fma(p, t, -0x1.32d2cce627543p-1);
  p = __builtin_fma(p, t, 0x1.466bc6775aa6ep+1);
  p = __builtin_fma(p, t, -0x1.4abbce625be52p+2);
  p = __builtin_fma(p, t, 0x1.921fb54442d18p+1);
  const double sv = r * p;
  return sv * sv;
}

__device__ __forceinline__ float sinpi_sq(float z) {
  const float r = z - __builtin_rintf(z);
  const float t = r * r;
  float p = 0x1.e8f434p-12f;
  p = __builtin_fmaf(p, t, -0x1.e3075p-8f);
  p = __builtin_fmaf(p, t, 0x1.507834p-4f);
  p = __builtin_fmaf(p, t, -0x1.32d2ccp-1f);
  p = __builtin_fmaf(p, t, 0x1.466bc6p+1f);
  p = __builtin_fmaf(p, t, -0x1.4abbcep+2f);
  p = __builtin_fmaf(p, t, 0x1.921fb6p+1f);
  const float sv = r * p;
  return sv * sv;
}

// 20 sin^2(pi z), the Rastrigin term's periodic part: the same polynomials
// with every coefficient multiplied by sqrt(20) (saves the final multiply).
__device__ __forceinline__ double sinpi_sq20(double z) {
  const double r = z - __builtin_rint(z);
  const double t = r * r;
  double p = 0x1.cdde45ade783cp-19;
  p = __builtin_fma(p, t, -0x1.9ad954d2dd022p-14);
  p = __builtin_fma(p, t, 0x1.1154ec3d37860p-9);
  p = __builtin_fma(p, t, -0x1.0e056a9d9acf8p-5);
  p = __builtin_fma(p, t, 0x1.782f347c9992ep-2);
  p = __builtin_fma(p, t, -0x1.5709fe171b213p+1);
  p = __builtin_fma(p, t, 0x1.6cf3241671ea3p+3);
  p = __builtin_fma(p, t, -0x1.71c57c2da483cp+4);
  p = __builtin_fma(p, t, 0x1.c196908691da7p+3);
  const double sv = r * p;
  return sv * sv;
}

__device__ __forceinline__ float sinpi_sq20(float z) {
  const float r = z - __builtin_rintf(z);
  const float t = r * r;
  float p = 0x1.115564p-9f;
  p = __builtin_fmaf(p, t, -0x1.0e056cp-5f);
  p = __builtin_fmaf(p, t, 0x1.782f34p-2f);
  p = __builtin_fmaf(p, t, -0x1.5709fep+1f);
  p = __builtin_fmaf(p, t, 0x1.6cf324p+3f);
  p = __builtin_fmaf(p, t, -0x1.71c57cp+4f);
  p = __builtin_fmaf(p, t, 0x1.c19690p+3f);
  const float sv = r * p;
  return sv * sv;
}

// Separable per-element term: sphere x^2, Rastrigin z^2 + 20 sin^2(pi z)
// (= z^2 - 10 cos(2 pi z) + 10 without the cancellation near integers).
template <typename T, int FN>
__device__ __forceinline__ T point_term(T x, T o) {
  if constexpr (FN == FN_SPHERE) {
    return x * x;
  } else {
    const T z = x - o;
    return Math<T>::fma_(z, z, sinpi_sq20(z));
  }
}

// Rosenbrock pair term for z_j, z_{j+1} with z = x - o + 1.
template <typename T>
__device__ __forceinline__ T rosen_term(T z0, T z1) {
  const T a = z1 - z0 * z0;
  const T b = z0 - T(1);
  return Math<T>::fma_(T(100) * a, a, b * b);
}

// Ackley and Griewank (Sec. 4) need two row statistics: s1 = sum x_j^2 and a
// second one, s2, combined once the row is reduced.
//   Ackley:   s2 = sum sin^2(pi x_j), since mean cos(2 pi x) = 1 - 2 s2 / D; then
//             f = -20 expm1(-0.02 sqrt(s1 / D)) - e expm1(-2 s2 / D), the same
//             value as the printed form without its cancellation near x = 0.
//   Griewank: s2 = prod cos(x_j / sqrt(j)) (j from 1); f = (1 - s2) + s1 / 4000.
template <int FN> constexpr bool kTwoStat = FN == FN_ACKLEY || FN == FN_GRIEWANK;

template <typename T, int FN>
__device__ __forceinline__ T stat2_init() {
  return FN == FN_GRIEWANK ? T(1) : T(0);
}

// Element j's part of s2 (j counted from 0).
template <typename T, int FN>
__device__ __forceinline__ T stat2_term(T x, uint32_t j) {
  if constexpr (FN == FN_ACKLEY) {
    return sinpi_sq(x);
  } else {
    return Math<T>::cos_(x / Math<T>::sqrt_(static_cast<T>(j + 1)));
  }
}

template <typename T, int FN>
__device__ __forceinline__ T stat2_join(T a, T b) {
  return FN == FN_GRIEWANK ? a * b : a + b;
}

template <typename T, int FN>
__device__ __forceinline__ T stat2_finish(T s1, T s2, uint32_t D) {
  if constexpr (FN == FN_ACKLEY) {
    const T d = static_cast<T>(D);
    const T r = Math<T>::sqrt_(s1 / d);
    return T(-20) * Math<T>::expm1_(T(-0.02) * r) -
           T(2.718281828459045235360287) * Math<T>::expm1_(T(-2) * s2 / d);
  } else {
    return (T(1) - s2) + s1 / T(4000);
  }
}

template <typename T>
__device__ __forceinline__ T wave_prod(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v *= __shfl_xor(v, off);
  return v;
}

template <typename T, int FN>
__device__ __forceinline__ T wave_stat2(T v) {
  if constexpr (FN == FN_GRIEWANK) {
    return wave_prod(v);
  } else {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
  }
}

// Pieces of a value for the split-bf16 products: hi = bf16(v), then the
// rounding remainders (hi + mid + lo carries the 24 bits of an FP32 value).
__device__ __forceinline__ void split3(float v, __bf16& a, __bf16& b, __bf16& c) {
  a = static_cast<__bf16>(v);
  const float r1 = v - static_cast<float>(a);
  b = static_cast<__bf16>(r1);
  const float r2 = r1 - static_cast<float>(b);
  c = static_cast<__bf16>(r2);
}

__device__ __forceinline__ uint32_t pack_bf16(__bf16 a, __bf16 b) {
  return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, a)) |
         (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, b)) << 16);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <typename T>
__device__ __forceinline__ T canon(T f) {
  return f != f ? Math<T>::inf() : f;
}

}  // namespace de
