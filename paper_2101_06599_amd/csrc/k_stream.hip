// The generation kernel for the exponential crossovers (classic and NEC) on
// long rows: the row is streamed instead of held in registers.
#include "gen_row.h"

namespace de {

// The generation for the exponential crossovers (classic and NEC) on rows
// too long to keep in registers.  The trial equals the parent outside the run
// of L elements from j_rand, so the row is streamed once, chunk by chunk (U
// chunks per lane in flight), with donors loaded only where the run covers a
// chunk and the fitness accumulated on the way; nothing of the row is kept.
// A winner then rebuilds and writes only the chunks of its run and of the run
// in which the row's other buffer still differs (partial write-back; whole
// rows when the record says the buffers are unrelated or the run is whole),
// reading the parent and donors of those few chunks a second time.
template <typename T, int FN, int XO, int TPR, int U>
__global__ void __launch_bounds__(Shape<TPR>::BS)
k_generation_stream(const RunDev* __restrict__ runs, int32_t run, int64_t rows, GenNo gn) {
  static_assert(XO == XO_EXP || XO == XO_NEC, "streaming needs a run-shaped mask");
  static_assert(FN != FN_NONE && FN != FN_ANY, "streaming evaluates one known function");
  using S = Shape<TPR>;
  __shared__ T red[S::RPB * S::NW];
  __shared__ uint32_t redc[S::RPB * S::NW];
  __shared__ T red2[kTwoStat<FN> ? S::RPB * S::NW : 1];

  const uint32_t t = threadIdx.x % TPR;
  const uint32_t slot = threadIdx.x / TPR;
  const uint32_t wave = t / 64, lane = threadIdx.x % 64;
  int64_t grow = static_cast<int64_t>(blockIdx.x) * S::RPB + slot;
  const bool live = grow < rows;
  if (!live) grow = rows - 1;
  const uint32_t i = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(grow));
  const RunDev& P = runs[run];
  RowCtx<T> R;
  R.xo = XO;
  R.D = static_cast<uint32_t>(P.D);
  R.thr = P.thr;
  R.i = i;
  const uint32_t gnew = __builtin_amdgcn_readfirstlane(gen_value(gn));
  R.g = run_gen(P, gnew);
  R.F = sizeof(T) == 4 ? static_cast<T>(P.Ff) : static_cast<T>(P.F);
  const uint32_t N = static_cast<uint32_t>(P.N);
  const int64_t ld = P.ld;
  DE_GLOBAL T* fit = gmut<T>(P.fit);
  const uint32_t si = __builtin_amdgcn_readfirstlane(row_of(P, R.g, i));
  const T fold = fit[si];
  const uint32_t dword = gconst<uint32_t>(P.dirty)[4 * static_cast<int64_t>(si) + (__lane_id() & 3u)];

  uint32_t r0, r1, r2;
  pick_scheme(P, R.g, i, N, r0, r1, r2);
  if (P.shuffle) {
    r0 = row_of(P, R.g, r0);
    r1 = row_of(P, R.g, r1);
    r2 = row_of(P, R.g, r2);
  }
  const DE_GLOBAL uint8_t* cur = gconst<uint8_t>(P.flags) + ((R.g - 1) & 1u) * static_cast<int64_t>(N);
  DE_GLOBAL uint8_t* nxt = gmut<uint8_t>(P.flags) + (R.g & 1u) * static_cast<int64_t>(N);
  r0 = __builtin_amdgcn_readfirstlane(r0);
  r1 = __builtin_amdgcn_readfirstlane(r1);
  r2 = __builtin_amdgcn_readfirstlane(r2);
  const uint32_t fi = cur[si], f0 = cur[r0], f1 = cur[r1], f2 = cur[r2];
  const uint4 bx = draw(P, TAG_XO, R.g, i, 0);
  R.jr = __builtin_amdgcn_readfirstlane(scale_index(bx.x, R.D));
  uint64_t t1 = 0;
  if (XO == XO_NEC) t1 = nec_prefetch(P);
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
  if (XO == XO_NEC) R.L = nec_length(P, bx.y, t1);
  else R.L = P.exp_impl == EXPI_SCAN ? exp_length_scan(P, R.g, i) : exp_length_serial(P, R.g, i);
  R.L = __builtin_amdgcn_readfirstlane(R.L);

  const uint32_t nchunk = (R.D + 3) >> 2;
  constexpr bool shifted = FN == FN_RASTRIGIN || FN == FN_ROSENBROCK;
  T acc = T(0);
  T acc2 = stat2_init<T, FN>();
  uint32_t cnt = 0;
  // Alg 2's copy, masked mutation and evaluation for this row, streamed.  The
  // trip count is the same for every lane of the row (the cross-lane shuffle
  // below needs the whole wavefront).
  for (uint32_t base = 0; base < nchunk; base += U * TPR) {
    V4<T> xs[U], os[U];
    T xn[U], on[U];  // Rosenbrock: a wavefront's last lane's next element
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t c = min(base + u * TPR + t, nchunk - 1);
      xs[u] = load4(R.xi + 4 * c);
      if (shifted) os[u] = load4(R.o + 4 * c);
      xn[u] = on[u] = T(0);
      if constexpr (FN == FN_ROSENBROCK) {
        if (lane == 63) {
          const uint32_t jn = min(4 * c + 4, R.D - 1);
          xn[u] = R.xi[jn];
          on[u] = R.o[jn];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t c = base + u * TPR + t;
      const bool in = c < nchunk;
      T v[4] = {T(0), T(0), T(0), T(0)};
      T zf = T(0);
      if (in) {
        const uint32_t m = build_chunk_from(P, R, c, xs[u], v);
        cnt += __popc(m);
        acc += chunk_terms<T, FN>(R, c, v, os[u], zf);
        chunk_stat2<T, FN>(R, c, v, acc2);
      }
      if constexpr (FN == FN_ROSENBROCK) {
        // the pair that crosses into chunk c + 1: its first z is the next
        // lane's (a wavefront's chunks are consecutive), or computed here by
        // the wavefront's last lane from the element loaded with its chunk
        const T znb = __shfl_down(zf, 1);
        if (in && 4 * c + 4 < R.D) {
          const T zn = lane != 63 ? znb : (trial_from(P, R, 4 * c + 4, xn[u]) - on[u]) + T(1);
          const T zl = (v[3] - os[u].v[3]) + T(1);
          acc += rosen_term(zl, zn);
        }
      }
    }
  }

  // Row reduction in a fixed order (wave butterfly, then waves in order).
  const bool tracing = P.tr_idx != nullptr || P.tr_mask != nullptr || P.tr_trial != nullptr;
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
  // Alg 1's replacement test: strictly lower fitness replaces the parent.
  const bool win = fu < fold;
  if (win) {
    const uint32_t pj = __builtin_amdgcn_readlane(dword, 0);
    const uint32_t pl = __builtin_amdgcn_readlane(dword, 1);
    const uint32_t pw = __builtin_amdgcn_readlane(dword, 2);
    if (pw == 0 || pl >= R.D || R.L >= R.D) {
      for (uint32_t c = t; c < nchunk; c += TPR) {
        T v[4];
        build_chunk(P, R, c, v);
        store4(R.dst + 4 * c, v);
      }
    } else {
      // the other buffer equals the parent outside its recorded run and the
      // trial equals the parent outside its own run: write both runs' chunks
      const RunChunks a = run_chunks(R.jr, R.L, R.D), b = run_chunks(pj, pl, R.D);
      const uint32_t lo[4] = {a.a0, a.b0, b.a0, b.b0}, hi[4] = {a.a1, a.b1, b.a1, b.b1};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        for (uint32_t c = lo[q] + t; c < hi[q]; c += TPR) {
          T v[4];
          build_chunk(P, R, c, v);
          store4(R.dst + 4 * c, v);
        }
    }
    if (t == 0 && pw != 0) gmut<uint4>(P.dirty)[si] = make_uint4(R.jr, R.L, pw, 0u);
  }
  if (t == 0) {
    nxt[si] = static_cast<uint8_t>(win ? ci ^ 1u : ci);
    if (win) fit[si] = fu;
    gmut<T>(P.hist)[static_cast<int64_t>(gnew % kHist) * N + si] = win ? fu : Math<T>::inf();
  }

  if (tracing) {
    const int64_t D = R.D;
    if (P.tr_idx && t == 0) {
      int64_t* q = P.tr_idx + 6 * static_cast<int64_t>(si);
      q[0] = r0; q[1] = r1; q[2] = r2; q[3] = R.jr;
      q[4] = R.L;
      q[5] = win ? 1 : 0;
    }
    if (P.tr_ftrial && t == 0) static_cast<T*>(P.tr_ftrial)[si] = fu;
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

// chunks per lane in flight (C5's D = 10^4 FP32 rows at 256 lanes: 2 chunks
// 73 us per generation, 1: 77, 3: 76, 4: 81, 8: 96)
#ifndef DE_STREAM_U
#define DE_STREAM_U 2
#endif
constexpr int kStreamU = DE_STREAM_U;

template <typename T, int FN, int XO, int TPR>
static hipError_t go(const GenLaunch& L) {
  using S = Shape<TPR>;
  const int64_t blocks = (L.rows + S::RPB - 1) / S::RPB;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_generation_stream<T, FN, XO, TPR, kStreamU>), dim3(blocks), dim3(S::BS), 0,
                     L.s, L.runs, L.run, L.rows, L.gnew);
  return hipGetLastError();
}

template <typename T, int FN, int XO>
static hipError_t go_tpr(const GenLaunch& L) {
  switch (L.tpr) {
    case 64: return go<T, FN, XO, 64>(L);
    case 128: return go<T, FN, XO, 128>(L);
    case 256: return go<T, FN, XO, 256>(L);
    case 512: return go<T, FN, XO, 512>(L);
    case 1024: return go<T, FN, XO, 1024>(L);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int FN>
static hipError_t go_xo(const GenLaunch& L, int xo) {
  if (xo == XO_NEC) return go_tpr<T, FN, XO_NEC>(L);
  if (xo == XO_EXP) return go_tpr<T, FN, XO_EXP>(L);
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t go_fn(const GenLaunch& L, int fn, int xo) {
  switch (fn) {
    case FN_SPHERE: return go_xo<T, FN_SPHERE>(L, xo);
    case FN_RASTRIGIN: return go_xo<T, FN_RASTRIGIN>(L, xo);
    case FN_ROSENBROCK: return go_xo<T, FN_ROSENBROCK>(L, xo);
    case FN_ACKLEY: return go_xo<T, FN_ACKLEY>(L, xo);
    case FN_GRIEWANK: return go_xo<T, FN_GRIEWANK>(L, xo);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_generation_stream(const GenLaunch& L, int fn, int xo, int dtype) {
  return dtype == 0 ? go_fn<double>(L, fn, xo) : go_fn<float>(L, fn, xo);
}

}  // namespace de
