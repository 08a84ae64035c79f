// Row-level building blocks of the generation kernels (k_generation.hip keeps
// a row's trial in registers, k_stream.hip streams it): loads and stores of
// 4-element chunks, the per-row context, the crossover mask and trial of a
// chunk, and the fitness terms of a chunk.
#pragma once

#include "de_device.h"

namespace de {

template <typename T> struct V4 { T v[4]; };

template <typename T>
__device__ __forceinline__ V4<T> load4(const DE_GLOBAL T* p) {
  V4<T> r;
  if constexpr (sizeof(T) == 4) {
    const float4 f = *(const DE_GLOBAL float4*)p;
    r.v[0] = f.x; r.v[1] = f.y; r.v[2] = f.z; r.v[3] = f.w;
  } else {
    const double2 a = ((const DE_GLOBAL double2*)p)[0];
    const double2 b = ((const DE_GLOBAL double2*)p)[1];
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
  }
  return r;
}

// Split-bf16 rotated runs: the np bf16 pieces of one chunk of (trial - o),
// written where the product reads them, so no separate split pass over the
// trial rows is needed.  Piece p of a row lives in plane p of the piece
// buffer (planes of N rows of pitch ldk): chunk c's four values of piece p
// are at row + p * plane + 4 c.
template <typename T>
__device__ __forceinline__ void store_pieces(DE_GLOBAL __bf16* row, int64_t plane, int np,
                                             uint32_t c, const T (&u)[4], const V4<T>& o) {
  if constexpr (sizeof(T) == 4) {
    __bf16 h[4], m[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) split3(u[e] - o.v[e], h[e], m[e], l[e]);
    DE_GLOBAL __bf16* q = row + 4 * c;
    *(DE_GLOBAL uint2*)q = make_uint2(pack_bf16(h[0], h[1]), pack_bf16(h[2], h[3]));
    *(DE_GLOBAL uint2*)(q + plane) = make_uint2(pack_bf16(m[0], m[1]), pack_bf16(m[2], m[3]));
    if (np == 3)
      *(DE_GLOBAL uint2*)(q + 2 * plane) = make_uint2(pack_bf16(l[0], l[1]), pack_bf16(l[2], l[3]));
  }
}

template <typename T>
__device__ __forceinline__ void store4(DE_GLOBAL T* p, const T (&u)[4]) {
  if constexpr (sizeof(T) == 4) {
    *(DE_GLOBAL float4*)p = make_float4(u[0], u[1], u[2], u[3]);
  } else {
    ((DE_GLOBAL double2*)p)[0] = make_double2(u[0], u[1]);
    ((DE_GLOBAL double2*)p)[1] = make_double2(u[2], u[3]);
  }
}

// Everything a row needs, gathered once per row (all wave-uniform).
template <typename T>
struct RowCtx {
  const DE_GLOBAL T* xi;
  const DE_GLOBAL T* x0;
  const DE_GLOBAL T* x1;
  const DE_GLOBAL T* x2;
  const DE_GLOBAL T* o;
  DE_GLOBAL T* dst;
  T F;
  uint64_t thr;
  uint32_t D, jr, L, g, i;
  int xo;
};

// Whether chunk c holds an element of the run of L elements from j0 (mod D);
// L = 0 is the empty run, L >= D the whole row.
__device__ __forceinline__ bool run_touches(uint32_t j0, uint32_t L, uint32_t c, uint32_t D) {
  if (L >= D) return true;
  bool hit = false;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const uint32_t j = 4 * c + v;
    const uint32_t off = j >= j0 ? j - j0 : j + D - j0;
    hit |= j < D && off < L;
  }
  return hit;
}

// Chunk c of the trial row: mask bits (bit v = element 4c+v crosses) and the
// four trial values.  Elements at or beyond D keep the parent's (padding).
template <typename T>
__device__ __forceinline__ uint32_t build_chunk_from(const RunDev& P, const RowCtx<T>& R,
                                                     uint32_t c, const V4<T>& x, T (&u)[4]) {
  const uint32_t j0 = 4 * c;
  uint32_t m = 0;
  if (R.xo == XO_BIN) {
    const uint4 b = draw(P, TAG_BIN, R.g, R.i, c);
    m = (static_cast<uint64_t>(b.x) < R.thr ? 1u : 0u) | (static_cast<uint64_t>(b.y) < R.thr ? 2u : 0u) |
        (static_cast<uint64_t>(b.z) < R.thr ? 4u : 0u) | (static_cast<uint64_t>(b.w) < R.thr ? 8u : 0u);
    if (R.jr >= j0 && R.jr < j0 + 4) m |= 1u << (R.jr - j0);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t j = j0 + v;
      const uint32_t off = j >= R.jr ? j - R.jr : j + R.D - R.jr;
      m |= (off < R.L ? 1u : 0u) << v;
    }
  }
  const uint32_t valid = R.D - j0 >= 4 ? 0xFu : ((1u << (R.D - j0)) - 1u);
  m &= valid;
#pragma unroll
  for (int v = 0; v < 4; ++v) u[v] = x.v[v];
  if (m) {
    const V4<T> a = load4(R.x0 + j0);
    const V4<T> b = load4(R.x1 + j0);
    const V4<T> d = load4(R.x2 + j0);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (m & (1u << v)) u[v] = Math<T>::fma_(R.F, b.v[v] - d.v[v], a.v[v]);
  }
  return m;
}

template <typename T>
__device__ __forceinline__ uint32_t build_chunk(const RunDev& P, const RowCtx<T>& R, uint32_t c,
                                                T (&u)[4]) {
  return build_chunk_from(P, R, c, load4(R.xi + 4 * c), u);
}

// Trial value of a single element j whose parent value xj is in hand (the
// Rosenbrock neighbour of a chunk's last element); the donors are read only
// when the mask covers j.
template <typename T>
__device__ __forceinline__ T trial_from(const RunDev& P, const RowCtx<T>& R, uint32_t j, T xj) {
  bool m;
  if (R.xo == XO_BIN) {
    const uint4 b = draw(P, TAG_BIN, R.g, R.i, j >> 2);
    m = static_cast<uint64_t>(word_of(b, j & 3u)) < R.thr || j == R.jr;
  } else {
    const uint32_t off = j >= R.jr ? j - R.jr : j + R.D - R.jr;
    m = off < R.L;
  }
  return m ? Math<T>::fma_(R.F, R.x1[j] - R.x2[j], R.x0[j]) : xj;
}

template <typename T>
__device__ __forceinline__ T trial_elem(const RunDev& P, const RowCtx<T>& R, uint32_t j) {
  return trial_from(P, R, j, R.xi[j]);
}

// Fitness contribution of one chunk; for Rosenbrock only the pairs inside the
// chunk (the pair that crosses into the next chunk is added separately).
template <typename T, int FN>
__device__ __forceinline__ T chunk_terms(const RowCtx<T>& R, uint32_t c, const T (&u)[4],
                                         const V4<T>& o, T& zfirst) {
  const uint32_t j0 = 4 * c;
  T acc = T(0);
  if constexpr (FN == FN_SPHERE || kTwoStat<FN>) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (j0 + v < R.D) acc += point_term<T, FN_SPHERE>(u[v], T(0));
  } else if constexpr (FN == FN_RASTRIGIN) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (j0 + v < R.D) acc += point_term<T, FN>(u[v], o.v[v]);
  } else if constexpr (FN == FN_ROSENBROCK) {
    T z[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) z[v] = (u[v] - o.v[v]) + T(1);
#pragma unroll
    for (int v = 0; v < 3; ++v)
      if (j0 + v + 1 < R.D) acc += rosen_term(z[v], z[v + 1]);
    zfirst = z[0];
  }
  return acc;
}

// The second row statistic of Ackley and Griewank over one chunk.
template <typename T, int FN>
__device__ __forceinline__ void chunk_stat2(const RowCtx<T>& R, uint32_t c, const T (&u)[4], T& s2) {
  if constexpr (kTwoStat<FN>) {
    const uint32_t j0 = 4 * c;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (j0 + v < R.D) s2 = stat2_join<T, FN>(s2, stat2_term<T, FN>(u[v], j0 + v));
  }
}

template <typename T>
__device__ __forceinline__ T runtime_terms(int fn, const RowCtx<T>& R, uint32_t c, const T (&u)[4],
                                           const V4<T>& o, T& zf) {
  if (fn == FN_SPHERE) return chunk_terms<T, FN_SPHERE>(R, c, u, o, zf);
  if (fn == FN_RASTRIGIN) return chunk_terms<T, FN_RASTRIGIN>(R, c, u, o, zf);
  return chunk_terms<T, FN_ROSENBROCK>(R, c, u, o, zf);
}

template <int TPR> struct Shape {
  static constexpr int BS = TPR >= 256 ? TPR : 256;  // threads per block
  static constexpr int RPB = BS / TPR;               // rows per block
  static constexpr int NW = TPR / 64;                // wavefronts per row
  // chunks of 4 elements held in registers per thread: D <= 16 * TPR (20 * 512
  // for 512-wide rows, 8 * 128 for 128-wide rows) stays in registers between
  // evaluation and write-back
  static constexpr int MAXIT = TPR == 512 ? 5 : TPR == 128 ? 2 : 4;
  // 64- and 128-lane rows issue every cached chunk's parent loads before
  // using any (more loads in flight per wave); wider rows would lose
  // occupancy to it
  static constexpr bool PREFETCH = TPR <= 128;
};


// Chunks that hold elements of the run of L elements from j0 (mod D), as up
// to two increasing ranges [a0, a1) and [b0, b1) (the second when the run
// wraps past D - 1); L = 0 gives none, L >= D every chunk.
struct RunChunks {
  uint32_t a0, a1, b0, b1;
};
__device__ __forceinline__ RunChunks run_chunks(uint32_t j0, uint32_t L, uint32_t D) {
  RunChunks r{0, 0, 0, 0};
  if (L == 0) return r;
  if (L >= D) {
    r.a1 = (D + 3) >> 2;
    return r;
  }
  const uint32_t end = j0 + L;  // one past the run's last element, before the wrap
  r.a0 = j0 >> 2;
  r.a1 = ((end < D ? end : D) + 3) >> 2;
  if (end > D) r.b1 = (end - D + 3) >> 2;
  return r;
}

}  // namespace de
