// The fused generation kernel: for each individual, index choice, crossover
// mask, masked DE/rand/1 mutation, fitness and greedy selection in one pass
// over the row (Alg 2 lines 6-14 for one row).
//
// Layout: TPR threads own one row (TPR >= 64, so a row is one or more whole
// wavefronts and every per-row draw is wave-uniform).  Thread t of a row
// handles 4-element chunks c = k*TPR + t, so a wavefront reads 64 consecutive
// chunks of the parent row (1 KiB FP32 / 2 KiB FP64) per step.  The trial row
// stays in registers until the row's fitness is known; only winners write it,
// into the buffer that does not hold the parent (the population is double
// buffered per row and a flag array per generation parity says which buffer
// holds each row), so no row is read and written in the same generation.
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
// written where the product reads them (groups of 8 elements; piece p of
// chunk c at row + ((c / 2) * np + p) * 8 + (c % 2) * 4), so no separate
// split pass over the trial rows is needed.
template <typename T>
__device__ __forceinline__ void store_pieces(DE_GLOBAL __bf16* row, int np, uint32_t c,
                                             const T (&u)[4], const V4<T>& o) {
  if constexpr (sizeof(T) == 4) {
    __bf16 h[4], m[4], l[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) split3(u[e] - o.v[e], h[e], m[e], l[e]);
    DE_GLOBAL __bf16* q = row + (c >> 1) * np * 8 + (c & 1u) * 4;
    *(DE_GLOBAL uint2*)q = make_uint2(pack_bf16(h[0], h[1]), pack_bf16(h[2], h[3]));
    *(DE_GLOBAL uint2*)(q + 8) = make_uint2(pack_bf16(m[0], m[1]), pack_bf16(m[2], m[3]));
    if (np == 3) *(DE_GLOBAL uint2*)(q + 16) = make_uint2(pack_bf16(l[0], l[1]), pack_bf16(l[2], l[3]));
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

// Trial value of a single element j (used only past the register-cached part
// of very long rows, for the Rosenbrock neighbour of a chunk's last element).
template <typename T>
__device__ __forceinline__ T trial_elem(const RunDev& P, const RowCtx<T>& R, uint32_t j) {
  bool m;
  if (R.xo == XO_BIN) {
    const uint4 b = draw(P, TAG_BIN, R.g, R.i, j >> 2);
    m = static_cast<uint64_t>(word_of(b, j & 3u)) < R.thr || j == R.jr;
  } else {
    const uint32_t off = j >= R.jr ? j - R.jr : j + R.D - R.jr;
    m = off < R.L;
  }
  return m ? Math<T>::fma_(R.F, R.x1[j] - R.x2[j], R.x0[j]) : R.xi[j];
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

// FN: a fixed function, FN_ANY (taken from the run record) or FN_NONE (build
// and store the trial only; the rotated function's product evaluates it).
// XO: a fixed crossover or XO_ANY.  BATCH: rows come from a row map that
// spans several runs.
template <typename T, int FN, int XO, int TPR, int MAXIT, bool BATCH>
__global__ void __launch_bounds__(Shape<TPR>::BS)
k_generation(const RunDev* __restrict__ runs, int32_t run_single, const uint2* __restrict__ rowmap,
             int64_t rows, GenNo gn) {
  using S = Shape<TPR>;
  __shared__ T red[S::RPB * S::NW];
  __shared__ uint32_t redc[S::RPB * S::NW];
  __shared__ T red2[kTwoStat<FN> ? S::RPB * S::NW : 1];
  __shared__ T zsh[(FN == FN_ROSENBROCK || FN == FN_ANY) ? S::RPB * TPR * MAXIT + 1 : 1];

  const uint32_t t = threadIdx.x % TPR;
  const uint32_t slot = threadIdx.x / TPR;
  const uint32_t wave = t / 64, lane = threadIdx.x % 64;
  int64_t grow = static_cast<int64_t>(blockIdx.x) * S::RPB + slot;
  const bool live = grow < rows;
  if (!live) grow = rows - 1;
  uint32_t run = static_cast<uint32_t>(run_single), i = static_cast<uint32_t>(grow);
  if constexpr (BATCH) {
    const uint2 m = rowmap[grow];
    run = m.x;
    i = m.y;
  }
  run = __builtin_amdgcn_readfirstlane(run);
  i = __builtin_amdgcn_readfirstlane(i);
  const RunDev& P = runs[run];
  const int fn = FN == FN_ANY ? P.fn : FN;
  RowCtx<T> R;
  R.xo = XO == XO_ANY ? P.xo : XO;
  R.D = static_cast<uint32_t>(P.D);
  R.thr = P.thr;
  R.i = i;
  const uint32_t gnew = __builtin_amdgcn_readfirstlane(gen_value(gn));
  R.g = run_gen(P, gnew);
  R.F = sizeof(T) == 4 ? static_cast<T>(P.Ff) : static_cast<T>(P.F);
  const uint32_t N = static_cast<uint32_t>(P.N);
  const int64_t ld = P.ld;
  DE_GLOBAL T* fit = gmut<T>(P.fit);
  // i is the row's position in Alg 2 (it addresses every draw); si is the
  // storage row of the individual at that position (i itself unless the run
  // shuffles, Alg 2 line 5).
  const uint32_t si = __builtin_amdgcn_readfirstlane(row_of(P, R.g, i));
  const T fold = FN != FN_NONE ? fit[si] : T(0);  // only row si's block writes it
  // The row's dirty record (only row si's block writes it): lane l holds its
  // word l % 4.  A vector load, so its wait is counted and comes only at the
  // write-back (a scalar load would hold up every later scalar-cache wait).
  const uint32_t dword = gconst<uint32_t>(P.dirty)[4 * static_cast<int64_t>(si) + (__lane_id() & 3u)];

  // Alg 2 line 6 and the index draws of Alg 6: base r0, difference r1 - r2,
  // then the storage rows they name.
  uint32_t r0, r1, r2;
  pick_scheme(P, R.g, i, N, r0, r1, r2);
  if (P.shuffle) {
    r0 = row_of(P, R.g, r0);
    r1 = row_of(P, R.g, r1);
    r2 = row_of(P, R.g, r2);
  }
  const DE_GLOBAL uint8_t* cur = gconst<uint8_t>(P.flags) + ((R.g - 1) & 1u) * static_cast<int64_t>(N);
  DE_GLOBAL uint8_t* nxt = gmut<uint8_t>(P.flags) + (R.g & 1u) * static_cast<int64_t>(N);
  // wave-uniform by construction; keep them (and the row pointers) scalar
  r0 = __builtin_amdgcn_readfirstlane(r0);
  r1 = __builtin_amdgcn_readfirstlane(r1);
  r2 = __builtin_amdgcn_readfirstlane(r2);
  // The four buffer flags and the first NEC table words go out together; the
  // parent row is requested as soon as its flag is back, and the run length
  // is counted while that row is in flight.
  const uint32_t fi = cur[si], f0 = cur[r0], f1 = cur[r1], f2 = cur[r2];
  // Alg 2 line 7: the crossover mask comes first (j_rand, and L for exp/NEC).
  const uint4 bx = draw(P, TAG_XO, R.g, i, 0);
  R.jr = __builtin_amdgcn_readfirstlane(scale_index(bx.x, R.D));
  uint64_t t1 = 0;
  if (R.xo == XO_NEC) t1 = nec_prefetch(P);
  const uint32_t ci = __builtin_amdgcn_readfirstlane(fi);
  const uint32_t c0 = __builtin_amdgcn_readfirstlane(f0);
  const uint32_t c1 = __builtin_amdgcn_readfirstlane(f1);
  const uint32_t c2 = __builtin_amdgcn_readfirstlane(f2);
  R.xi = gconst<T>(P.X[ci]) + static_cast<int64_t>(si) * ld;
  R.x0 = gconst<T>(P.X[c0]) + static_cast<int64_t>(r0) * ld;
  R.x1 = gconst<T>(P.X[c1]) + static_cast<int64_t>(r1) * ld;
  R.x2 = gconst<T>(P.X[c2]) + static_cast<int64_t>(r2) * ld;
  R.o = gconst<T>(P.o);
  R.dst = gmut<T>(P.X[ci ^ 1u]) + static_cast<int64_t>(si) * ld;

  const uint32_t nchunk = (R.D + 3) >> 2;
  const bool tracing = P.tr_idx != nullptr || P.tr_mask != nullptr || P.tr_trial != nullptr;
  T u[MAXIT][4];
  uint32_t mb[MAXIT];
  T acc = T(0);
  T acc2 = stat2_init<T, FN>();  // Ackley / Griewank only
  uint32_t cnt = 0;
  T* zrow = zsh + slot * (TPR * MAXIT);

  // Alg 2 lines 8-10 for this row: trial = parent with the masked elements
  // replaced by x_r0 + F (x_r1 - x_r2), evaluated on the fly.
  // Phase 1 (64- and 128-lane rows of one run): every cached chunk's parent (and
  // shift) loads go out together; wide rows and batched launches, where
  // occupancy matters more, load each chunk as they reach it.
  constexpr bool kPrefetch = S::PREFETCH && !BATCH;
  constexpr bool kShift = FN == FN_RASTRIGIN || FN == FN_ROSENBROCK || FN == FN_ANY;
  // Rotated split-bf16 runs (FP32 only) also write the pieces of trial - o.
  const bool pieces = FN == FN_NONE && sizeof(T) == 4 && P.apc != nullptr;
  const int np = P.mm == MM_BF16X6 ? 3 : 2;
  DE_GLOBAL __bf16* prow = pieces ? gmut<__bf16>(P.apc) + static_cast<int64_t>(si) * np * P.ldk
                                  : nullptr;
  const bool shifted = (kShift && (FN != FN_ANY || fn != FN_SPHERE)) || pieces;
  V4<T> xs[MAXIT], os[MAXIT];
  if constexpr (kPrefetch) {
    // Unconditional (lanes past the row reload its last chunk), so that the
    // counted waits below can let these loads stay in flight.
#pragma unroll
    for (int k = 0; k < MAXIT; ++k) {
      const uint32_t c = min(k * TPR + t, nchunk - 1);
      xs[k] = load4(R.xi + 4 * c);
      if (shifted) os[k] = load4(R.o + 4 * c);
    }
  }
  R.L = 0;
  if (R.xo == XO_NEC) R.L = nec_length(P, bx.y, t1);
  else if (R.xo == XO_EXP) R.L = P.exp_impl == EXPI_SCAN ? exp_length_scan(P, R.g, i)
                                                          : exp_length_serial(P, R.g, i);
  R.L = __builtin_amdgcn_readfirstlane(R.L);
  // Phase 2: mask, donors where the mask is set, trial and fitness terms.
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    const uint32_t c = k * TPR + t;
    mb[k] = 0;
    if (c < nchunk) {
      if constexpr (!kPrefetch) {
        xs[k] = load4(R.xi + 4 * c);
        if (shifted) os[k] = load4(R.o + 4 * c);
      }
      mb[k] = build_chunk_from(P, R, c, xs[k], u[k]);
      cnt += __popc(mb[k]);
      if constexpr (FN != FN_NONE) {
        T zf = T(0);
        acc += FN == FN_ANY ? runtime_terms(fn, R, c, u[k], os[k], zf)
                            : chunk_terms<T, FN>(R, c, u[k], os[k], zf);
        chunk_stat2<T, FN>(R, c, u[k], acc2);
        if constexpr (FN == FN_ROSENBROCK || FN == FN_ANY) zrow[c] = zf;
      }
    }
  }
  // Rows longer than the register cache: evaluate the rest now, rebuild later.
  for (uint32_t c = MAXIT * TPR + t; c < nchunk; c += TPR) {
    T v[4];
    const uint32_t m = build_chunk(P, R, c, v);
    cnt += __popc(m);
    if constexpr (FN != FN_NONE) {
      T zf = T(0);
      V4<T> ov;
      if (kShift && (FN != FN_ANY || fn != FN_SPHERE)) ov = load4(R.o + 4 * c);
      acc += FN == FN_ANY ? runtime_terms(fn, R, c, v, ov, zf)
                          : chunk_terms<T, FN>(R, c, v, ov, zf);
      chunk_stat2<T, FN>(R, c, v, acc2);
      if ((FN == FN_ROSENBROCK || (FN == FN_ANY && fn == FN_ROSENBROCK)) && 4 * c + 4 < R.D) {
        const T zn = (trial_elem(P, R, 4 * c + 4) - R.o[4 * c + 4]) + T(1);
        const T zl = (v[3] - R.o[4 * c + 3]) + T(1);
        acc += rosen_term(zl, zn);
      }
    }
  }

  if constexpr (FN == FN_ROSENBROCK || FN == FN_ANY) {
    __syncthreads();  // unconditional: rows of one block may run different functions
    if (FN == FN_ROSENBROCK || fn == FN_ROSENBROCK) {
#pragma unroll
      for (int k = 0; k < MAXIT; ++k) {
        const uint32_t c = k * TPR + t;
        if (c < nchunk && 4 * c + 4 < R.D) {
          const uint32_t cn = c + 1;
          T zn;
          if (cn < MAXIT * TPR) {
            zn = zrow[cn];
          } else {
            zn = (trial_elem(P, R, 4 * cn) - R.o[4 * cn]) + T(1);
          }
          const T zl = (u[k][3] - R.o[4 * c + 3]) + T(1);
          acc += rosen_term(zl, zn);
        }
      }
    }
  }

  // Row reduction in a fixed order (wave butterfly, then waves in order).
  T tot = wave_sum(acc);
  T tot2 = T(0);
  if constexpr (kTwoStat<FN>) tot2 = wave_stat2<T, FN>(acc2);
  uint32_t ctot = tracing ? static_cast<uint32_t>(wave_sum(static_cast<int>(cnt))) : 0u;
  if constexpr (S::NW > 1) {
    if (lane == 0) {
      red[slot * S::NW + wave] = tot;
      redc[slot * S::NW + wave] = ctot;
      if constexpr (kTwoStat<FN>) red2[slot * S::NW + wave] = tot2;
    }
    __syncthreads();
    tot = T(0);
    ctot = 0;
    if constexpr (kTwoStat<FN>) tot2 = stat2_init<T, FN>();
#pragma unroll
    for (int w = 0; w < S::NW; ++w) {
      tot += red[slot * S::NW + w];
      ctot += redc[slot * S::NW + w];
      if constexpr (kTwoStat<FN>) tot2 = stat2_join<T, FN>(tot2, red2[slot * S::NW + w]);
    }
  }

  if (!live) return;
  T fraw = tot;
  if constexpr (kTwoStat<FN>) fraw = stat2_finish<T, FN>(tot, tot2, R.D);
  const T fu = canon(fraw);
  bool win = true;
  if constexpr (FN != FN_NONE) {
    // Alg 1 line 10 / Alg 2 line 11: strictly lower fitness replaces.
    win = fu < fold;
  }
  if (win) {
    // Write-back into the other buffer.  It already equals the parent outside
    // the run in the row's record, and the trial equals the parent outside its
    // mask, so in partial mode only chunks in either are written; the buffers
    // then differ exactly where the mask was set.  Binomial masks are
    // scattered, and small populations (which live in the caches and read a
    // freshly written row fastest) use whole mode: whole rows are written.
    const uint32_t pj = __builtin_amdgcn_readlane(dword, 0);
    const uint32_t pl = __builtin_amdgcn_readlane(dword, 1);
    const uint32_t pw = __builtin_amdgcn_readlane(dword, 2);
    const bool whole = R.xo == XO_BIN || pw == 0 || pl >= R.D;
    if (whole) {
#pragma unroll
      for (int k = 0; k < MAXIT; ++k) {
        const uint32_t c = k * TPR + t;
        if (c < nchunk) {
          store4(R.dst + 4 * c, u[k]);
          if (pieces) store_pieces(prow, np, c, u[k], os[k]);
        }
      }
      for (uint32_t c = MAXIT * TPR + t; c < nchunk; c += TPR) {
        T v[4];
        build_chunk(P, R, c, v);
        store4(R.dst + 4 * c, v);
        if (pieces) store_pieces(prow, np, c, v, load4(R.o + 4 * c));
      }
    } else {
#pragma unroll
      for (int k = 0; k < MAXIT; ++k) {
        const uint32_t c = k * TPR + t;
        if (c < nchunk && (mb[k] != 0 || run_touches(pj, pl, c, R.D))) store4(R.dst + 4 * c, u[k]);
        if (pieces && c < nchunk) store_pieces(prow, np, c, u[k], os[k]);
      }
      for (uint32_t c = MAXIT * TPR + t; c < nchunk; c += TPR) {
        T v[4];
        const uint32_t m = build_chunk(P, R, c, v);
        if (m != 0 || run_touches(pj, pl, c, R.D)) store4(R.dst + 4 * c, v);
        if (pieces) store_pieces(prow, np, c, v, load4(R.o + 4 * c));
      }
    }
    if (t == 0 && pw != 0)
      gmut<uint4>(P.dirty)[si] = R.xo == XO_BIN ? make_uint4(0u, kDirtyAll, pw, 0u)
                                                : make_uint4(R.jr, R.L, pw, 0u);
  }
  if constexpr (FN != FN_NONE) {
    if (t == 0) {
      nxt[si] = static_cast<uint8_t>(win ? ci ^ 1u : ci);
      if (win) fit[si] = fu;
      // deferred best-so-far: winners' new fitness, +inf for the others
      gmut<T>(P.hist)[static_cast<int64_t>(gnew % kHist) * N + si] = win ? fu : Math<T>::inf();
    }
  }

  if (tracing) {
    const int64_t D = R.D;
    if (P.tr_idx && t == 0) {
      int64_t* q = P.tr_idx + 6 * static_cast<int64_t>(si);
      q[0] = r0; q[1] = r1; q[2] = r2; q[3] = R.jr;
      q[4] = R.xo == XO_BIN ? ctot : R.L;
      q[5] = (FN == FN_NONE) ? 0 : (win ? 1 : 0);
    }
    if (P.tr_ftrial && t == 0 && FN != FN_NONE) static_cast<T*>(P.tr_ftrial)[si] = fu;
    for (uint32_t c = t; c < nchunk; c += TPR) {
      T v[4];
      const uint32_t m = build_chunk(P, R, c, v);
      for (int e = 0; e < 4; ++e) {
        const uint32_t j = 4 * c + e;
        if (j >= R.D) break;
        if (P.tr_mask) P.tr_mask[si * D + j] = static_cast<uint8_t>((m >> e) & 1u);
        if (P.tr_trial) static_cast<T*>(P.tr_trial)[si * D + j] = v[e];
      }
    }
  }
}

// ---- host-side dispatch ----------------------------------------------------

template <typename T, int FN, int XO, int TPR>
static hipError_t go(const GenLaunch& L, bool batched) {
  using S = Shape<TPR>;
  const int64_t blocks = (L.rows + S::RPB - 1) / S::RPB;
  if (blocks <= 0) return hipSuccess;
  if (batched)
    hipLaunchKernelGGL((k_generation<T, FN, XO, TPR, S::MAXIT, true>), dim3(blocks), dim3(S::BS), 0, L.s,
                       L.runs, L.run, L.rowmap, L.rows, L.gnew);
  else
    hipLaunchKernelGGL((k_generation<T, FN, XO, TPR, S::MAXIT, false>), dim3(blocks), dim3(S::BS), 0, L.s,
                       L.runs, L.run, L.rowmap, L.rows, L.gnew);
  return hipGetLastError();
}

template <typename T, int FN, int XO>
static hipError_t go_tpr(const GenLaunch& L, bool batched) {
  switch (L.tpr) {
    case 64: return go<T, FN, XO, 64>(L, batched);
    case 128: return go<T, FN, XO, 128>(L, batched);
    case 256: return go<T, FN, XO, 256>(L, batched);
    case 512: return go<T, FN, XO, 512>(L, batched);
    case 1024: return go<T, FN, XO, 1024>(L, batched);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int FN>
static hipError_t go_xo(const GenLaunch& L, int xo, bool batched) {
  switch (xo) {
    case XO_BIN: return go_tpr<T, FN, XO_BIN>(L, batched);
    case XO_EXP: return go_tpr<T, FN, XO_EXP>(L, batched);
    case XO_NEC: return go_tpr<T, FN, XO_NEC>(L, batched);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t go_fn(const GenLaunch& L, int fn, int xo, bool batched) {
  if (batched) {
    if (L.tpr != 64) return hipErrorInvalidValue;
    return go<T, FN_ANY, XO_ANY, 64>(L, true);
  }
  switch (fn) {
    case FN_SPHERE: return go_xo<T, FN_SPHERE>(L, xo, false);
    case FN_RASTRIGIN: return go_xo<T, FN_RASTRIGIN>(L, xo, false);
    case FN_ROSENBROCK: return go_xo<T, FN_ROSENBROCK>(L, xo, false);
    case FN_ACKLEY: return go_xo<T, FN_ACKLEY>(L, xo, false);
    case FN_GRIEWANK: return go_xo<T, FN_GRIEWANK>(L, xo, false);
    case FN_NONE: return go_xo<T, FN_NONE>(L, xo, false);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_generation(const GenLaunch& L, int fn, int xo, int dtype, bool batched) {
  return dtype == 0 ? go_fn<double>(L, fn, xo, batched) : go_fn<float>(L, fn, xo, batched);
}

}  // namespace de
