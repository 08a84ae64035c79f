// The fused generation kernel: for each individual, index choice, crossover
// mask, masked DE/rand/1 mutation, fitness and greedy selection in one pass
// over the row (the body of Alg 2's generation loop for one row).
//
// Layout: TPR threads own one row (TPR >= 64, so a row is one or more whole
// wavefronts and every per-row draw is wave-uniform).  Thread t of a row
// handles 4-element chunks c = k*TPR + t, so a wavefront reads 64 consecutive
// chunks of the parent row (1 KiB FP32 / 2 KiB FP64) per step.  The trial row
// stays in registers until the row's fitness is known; only winners write it,
// into the buffer that does not hold the parent (the population is double
// buffered per row and a flag array per generation parity says which buffer
// holds each row), so no row is read and written in the same generation.
#include "gen_row.h"

namespace de {

// FN: a fixed function, FN_ANY (taken from the run record) or FN_NONE (build
// and store the trial only; the rotated function's product evaluates it).
// XO: a fixed crossover or XO_ANY.  BATCH: rows come from a row map that
// spans several runs.
// FP32 rows are held to 64 registers per lane, 8 wavefronts per SIMD (the
// batched 512-run table: 148 -> 129 us per generation with the prefetch
// below; single runs unchanged).  FP64 rows, Griewank's product butterfly
// and the split-piece stores of rotated runs need more (they would spill).
template <typename T, int FN, int XO, int TPR, int MAXIT, bool BATCH>
__global__ void __launch_bounds__(Shape<TPR>::BS) __attribute__((
    amdgpu_waves_per_eu(sizeof(T) == 4 && FN != FN_GRIEWANK && FN != FN_NONE ? 8 : 1)))
k_generation(const RunDev* __restrict__ runs, int32_t run_single, const uint2* __restrict__ rowmap,
             int64_t rows, GenNo gn) {
  using S = Shape<TPR>;
  __shared__ T red[S::RPB * S::NW];
  __shared__ uint32_t redc[S::RPB * S::NW];
  __shared__ T red2[kTwoStat<FN> ? S::RPB * S::NW : 1];
  // Rosenbrock pairs that cross from one wavefront of a row into the next:
  // first and last z of each wavefront's chunks (rows of several wavefronts).
  constexpr bool kRosenEdge = (FN == FN_ROSENBROCK || FN == FN_ANY) && S::NW > 1;
  constexpr int kEdge = kRosenEdge ? S::RPB * S::NW * MAXIT : 1;
  __shared__ T zfirst[kEdge], zlast[kEdge];

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
  // shuffles, Alg 2).
  const uint32_t si = __builtin_amdgcn_readfirstlane(row_of(P, R.g, i));
  const T fold = FN != FN_NONE ? fit[si] : T(0);  // only row si's block writes it
  // The row's dirty record (only row si's block writes it): lane l holds its
  // word l % 4.  A vector load, so its wait is counted and comes only at the
  // write-back (a scalar load would hold up every later scalar-cache wait).
  const uint32_t dword = gconst<uint32_t>(P.dirty)[4 * static_cast<int64_t>(si) + (__lane_id() & 3u)];

  // Alg 2's index choice and the draws of Alg 6: base r0, difference r1 - r2,
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
  // Alg 2 builds the crossover mask first (j_rand, and L for exp/NEC).
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

  // Alg 2's copy, masked mutation and evaluation for this row: trial = parent with the masked elements
  // replaced by x_r0 + F (x_r1 - x_r2), evaluated on the fly.
  // Phase 1 (64- and 128-lane rows of one run): every cached chunk's parent (and
  // shift) loads go out together; batched launches request their first two
  // chunks so (most of their rows have no more), and wide rows, where
  // occupancy matters more, load each chunk as they reach it.
  constexpr bool kPrefetch = S::PREFETCH && !BATCH;
  constexpr int PF = kPrefetch ? MAXIT : BATCH ? (MAXIT < 2 ? MAXIT : 2) : 0;
  constexpr bool kShift = FN == FN_RASTRIGIN || FN == FN_ROSENBROCK || FN == FN_ANY;
  // Rotated split-bf16 runs (FP32 only) also write the pieces of trial - o.
  const bool pieces = FN == FN_NONE && sizeof(T) == 4 && P.apc != nullptr;
  const int np = P.mm == MM_BF16X6 ? 3 : 2;
  DE_GLOBAL __bf16* prow = pieces ? gmut<__bf16>(P.apc) + static_cast<int64_t>(si) * P.ldk : nullptr;
  const int64_t plane = P.N * P.ldk;  // pitch of the piece planes
  const bool shifted = (kShift && (FN != FN_ANY || fn != FN_SPHERE)) || pieces;
  V4<T> xs[MAXIT], os[MAXIT];
  if constexpr (PF > 0) {
    // Unconditional (lanes past the row reload its last chunk), so that the
    // counted waits below can let these loads stay in flight.
#pragma unroll
    for (int k = 0; k < PF; ++k) {
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
  // Rosenbrock's pair across chunks c and c + 1 is added right after chunk c
  // when the first z of chunk c + 1 is the next lane's (a wavefront's chunks
  // are consecutive).  A wavefront's last lane pairs with the first lane of
  // the next wavefront of the row: through LDS after the loop, or (one
  // wavefront per row) with lane 0's value one chunk group later, carried in
  // a register; only the pair that leaves the cached chunks computes the
  // neighbouring element itself.  Whether the row is Rosenbrock is
  // wave-uniform (one run per wavefront).
  const bool rosen = FN == FN_ROSENBROCK || (FN == FN_ANY && fn == FN_ROSENBROCK);
  T zcarry = T(0);
  bool carry = false;
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    const uint32_t c = k * TPR + t;
    const bool in = c < nchunk;
    mb[k] = 0;
    T zf = T(0);
    if (in) {
      if (k >= PF) {
        xs[k] = load4(R.xi + 4 * c);
        if (shifted) os[k] = load4(R.o + 4 * c);
      }
      mb[k] = build_chunk_from(P, R, c, xs[k], u[k]);
      cnt += __popc(mb[k]);
      if constexpr (FN != FN_NONE) {
        acc += FN == FN_ANY ? runtime_terms(fn, R, c, u[k], os[k], zf)
                            : chunk_terms<T, FN>(R, c, u[k], os[k], zf);
        chunk_stat2<T, FN>(R, c, u[k], acc2);
      }
    }
    if constexpr (FN == FN_ROSENBROCK || FN == FN_ANY) {
      if (rosen) {
        const T znb = __shfl_down(zf, 1);
        if constexpr (S::NW == 1) {
          const T z0 = __shfl(zf, 0);
          if (carry) acc += rosen_term(zcarry, z0);
          carry = false;
        } else if (lane == 0) {
          zfirst[(slot * S::NW + wave) * MAXIT + k] = zf;
        }
        if (in && 4 * c + 4 < R.D) {
          const T zl = (u[k][3] - os[k].v[3]) + T(1);
          if (lane != 63) {
            acc += rosen_term(zl, znb);
          } else if (k + 1 < MAXIT && S::NW == 1) {
            zcarry = zl;
            carry = true;
          } else if (k + 1 < MAXIT || wave + 1 < S::NW) {
            if constexpr (kRosenEdge) zlast[(slot * S::NW + wave) * MAXIT + k] = zl;
          } else {
            acc += rosen_term(zl, (trial_elem(P, R, 4 * c + 4) - R.o[4 * c + 4]) + T(1));
          }
        }
      }
    }
  }
  if constexpr (kRosenEdge) {
    // every row of the block reaches this barrier (batched rows of other
    // functions included)
    __syncthreads();
    if (rosen && lane == 63) {
#pragma unroll
      for (int k = 0; k < MAXIT; ++k) {
        const uint32_t c = k * TPR + t;
        if (c < nchunk && 4 * c + 4 < R.D && (k + 1 < MAXIT || wave + 1 < S::NW)) {
          const int nk = wave + 1 < S::NW ? k : k + 1;
          const uint32_t nw = wave + 1 < S::NW ? wave + 1 : 0u;
          acc += rosen_term(zlast[(slot * S::NW + wave) * MAXIT + k],
                            zfirst[(slot * S::NW + nw) * MAXIT + nk]);
        }
      }
    }
  }
  // Rows longer than the register cache: evaluate the rest now, rebuild later
  // (the same trip count for every lane of the row, for the shuffle).
  for (uint32_t cb = MAXIT * TPR; cb < nchunk; cb += TPR) {
    const uint32_t c = cb + t;
    const bool in = c < nchunk;
    T v[4] = {T(0), T(0), T(0), T(0)};
    T zf = T(0);
    V4<T> ov;
    if (in) {
      const uint32_t m = build_chunk(P, R, c, v);
      cnt += __popc(m);
      if constexpr (FN != FN_NONE) {
        if (kShift && (FN != FN_ANY || fn != FN_SPHERE)) ov = load4(R.o + 4 * c);
        acc += FN == FN_ANY ? runtime_terms(fn, R, c, v, ov, zf)
                            : chunk_terms<T, FN>(R, c, v, ov, zf);
        chunk_stat2<T, FN>(R, c, v, acc2);
      }
    }
    if constexpr (FN == FN_ROSENBROCK || FN == FN_ANY) {
      if (rosen) {
        const T znb = __shfl_down(zf, 1);
        if (in && 4 * c + 4 < R.D) {
          const T zn = lane != 63 ? znb : (trial_elem(P, R, 4 * c + 4) - R.o[4 * c + 4]) + T(1);
          const T zl = (v[3] - ov.v[3]) + T(1);
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
    // Alg 1's replacement test, as in Alg 2's selection: strictly lower fitness replaces.
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
          if (pieces) store_pieces(prow, plane, np, c, u[k], os[k]);
        }
      }
      for (uint32_t c = MAXIT * TPR + t; c < nchunk; c += TPR) {
        T v[4];
        build_chunk(P, R, c, v);
        store4(R.dst + 4 * c, v);
        if (pieces) store_pieces(prow, plane, np, c, v, load4(R.o + 4 * c));
      }
    } else {
#pragma unroll
      for (int k = 0; k < MAXIT; ++k) {
        const uint32_t c = k * TPR + t;
        if (c < nchunk && (mb[k] != 0 || run_touches(pj, pl, c, R.D))) store4(R.dst + 4 * c, u[k]);
        if (pieces && c < nchunk) store_pieces(prow, plane, np, c, u[k], os[k]);
      }
      for (uint32_t c = MAXIT * TPR + t; c < nchunk; c += TPR) {
        T v[4];
        const uint32_t m = build_chunk(P, R, c, v);
        if (m != 0 || run_touches(pj, pl, c, R.D)) store4(R.dst + 4 * c, v);
        if (pieces) store_pieces(prow, plane, np, c, v, load4(R.o + 4 * c));
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
    switch (L.tpr) {
      case 64: return go<T, FN_ANY, XO_ANY, 64>(L, true);
      case 128: return go<T, FN_ANY, XO_ANY, 128>(L, true);
      case 256: return go<T, FN_ANY, XO_ANY, 256>(L, true);
      default: return hipErrorInvalidValue;
    }
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
