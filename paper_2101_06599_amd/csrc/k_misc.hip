// Supporting kernels: initial population and shift, whole-row fitness,
// best-so-far tracking, the classic exponential crossover as one job per
// individual, and state helpers.
#include "de_device.h"

namespace de {

// ---- initialisation (Alg 2, before its generation loop) --------------------

// Uniform in [lo, hi]: FP64 takes 53 bits from two words of block j/2, FP32
// takes 24 bits from word j%4 of block j/4.
template <typename T>
__device__ __forceinline__ T init_value(const RunDev& P, uint32_t tag, uint32_t i, uint32_t j,
                                        double lo, double hi) {
  if constexpr (sizeof(T) == 8) {
    const uint4 b = draw(P, tag, 0, i, j >> 1);
    const uint32_t a = (j & 1u) ? b.z : b.x;
    const uint32_t c = (j & 1u) ? b.w : b.y;
    const uint64_t bits = (static_cast<uint64_t>(a >> 5) << 26) | (c >> 6);
    const double u = static_cast<double>(bits) * 0x1p-53;
    return __builtin_fma(hi - lo, u, lo);
  } else {
    const uint4 b = draw(P, tag, 0, i, j >> 2);
    const float u = static_cast<float>(word_of(b, j & 3u) >> 8) * 0x1p-24f;
    const float lof = static_cast<float>(lo), hif = static_cast<float>(hi);
    return __builtin_fmaf(hif - lof, u, lof);
  }
}

// One thread per element of both population buffers (padding zeroed), plus
// the shift vector in block row 0 and the flag arrays.
template <typename T>
__global__ void k_init(const RunDev* __restrict__ runs, int32_t run, double lo, double hi,
                       double olo, double ohi, const T* __restrict__ shift_src, int gen_shift) {
  const RunDev& P = runs[run];
  const int64_t ld = P.ld, N = P.N, D = P.D;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < N * ld) {
    const int64_t i = e / ld, j = e % ld;
    const T v = j < D ? init_value<T>(P, TAG_INIT, static_cast<uint32_t>(i),
                                      static_cast<uint32_t>(j), lo, hi)
                      : T(0);
    // both buffers start equal, so a row's first write-back is partial too
    static_cast<T*>(P.X[0])[e] = v;
    static_cast<T*>(P.X[1])[e] = v;
  }
  if (e < N) P.dirty[e] = make_uint4(0u, 0u, static_cast<uint32_t>(P.partial_wb), 0u);
  if (e < ld) {
    T ov = T(0);
    if (e < D) {
      if (shift_src) ov = shift_src[e];
      else if (gen_shift) ov = init_value<T>(P, TAG_SHIFT, 0, static_cast<uint32_t>(e), olo, ohi);
    }
    static_cast<T*>(const_cast<void*>(P.o))[e] = ov;
  }
  if (e < 2 * N) P.flags[e] = 0;
}

// ---- whole-row fitness ----------------------------------------------------

template <typename T, int FN>
__device__ __forceinline__ T elem_term(const T* x, const T* o, uint32_t j, uint32_t D) {
  if constexpr (FN == FN_SPHERE) {
    return point_term<T, FN_SPHERE>(x[j], T(0));
  } else if constexpr (FN == FN_RASTRIGIN) {
    return point_term<T, FN_RASTRIGIN>(x[j], o[j]);
  } else {
    if (j + 1 >= D) return T(0);
    const T z0 = (x[j] - o[j]) + T(1);
    const T z1 = (x[j + 1] - o[j + 1]) + T(1);
    return rosen_term(z0, z1);
  }
}

// f of one row with a 256-thread block (strided loop, fixed-order reduction).
template <typename T, int FN>
__device__ T block_row_fitness(const T* x, const T* o, uint32_t D) {
  __shared__ T red[4];
  T acc = T(0);
  for (uint32_t j = threadIdx.x; j < D; j += blockDim.x) acc += elem_term<T, FN>(x, o, j, D);
  acc = wave_sum(acc);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  return canon(red[0] + red[1] + red[2] + red[3]);
}

// Ackley / Griewank: both row statistics, then their combination.
template <typename T, int FN>
__device__ T block_row_fitness2(const T* x, uint32_t D) {
  __shared__ T red[8];
  T s1 = T(0), s2 = stat2_init<T, FN>();
  for (uint32_t j = threadIdx.x; j < D; j += blockDim.x) {
    s1 += x[j] * x[j];
    s2 = stat2_join<T, FN>(s2, stat2_term<T, FN>(x[j], j));
  }
  s1 = wave_sum(s1);
  s2 = wave_stat2<T, FN>(s2);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = s1;
    red[4 + (threadIdx.x >> 6)] = s2;
  }
  __syncthreads();
  T t2 = stat2_init<T, FN>();
  for (int w = 0; w < 4; ++w) t2 = stat2_join<T, FN>(t2, red[4 + w]);
  return canon(stat2_finish<T, FN>(red[0] + red[1] + red[2] + red[3], t2, D));
}

template <typename T>
__device__ T block_row_fitness_rt(int fn, const T* x, const T* o, uint32_t D) {
  if (fn == FN_SPHERE) return block_row_fitness<T, FN_SPHERE>(x, o, D);
  if (fn == FN_RASTRIGIN) return block_row_fitness<T, FN_RASTRIGIN>(x, o, D);
  if (fn == FN_ACKLEY) return block_row_fitness2<T, FN_ACKLEY>(x, D);
  if (fn == FN_GRIEWANK) return block_row_fitness2<T, FN_GRIEWANK>(x, D);
  return block_row_fitness<T, FN_ROSENBROCK>(x, o, D);
}

// Initial evaluation (Alg 2, before its generation loop): rows of buffer 0.
template <typename T>
__global__ void __launch_bounds__(256) k_eval_pop(const RunDev* __restrict__ runs, int32_t run) {
  const RunDev& P = runs[run];
  const int64_t i = blockIdx.x;
  const T* x = static_cast<const T*>(P.X[0]) + i * P.ld;
  const T f = block_row_fitness_rt<T>(P.fn, x, static_cast<const T*>(P.o),
                                      static_cast<uint32_t>(P.D));
  if (threadIdx.x == 0) static_cast<T*>(P.fit)[i] = f;
}

// Caller rows (dense, pitch ldx) -> out.
template <typename T>
__global__ void __launch_bounds__(256) k_eval_rows(int fn, const T* __restrict__ X, int64_t ldx,
                                                   const T* __restrict__ o, uint32_t D,
                                                   T* __restrict__ out) {
  const int64_t r = blockIdx.x;
  const T f = block_row_fitness_rt<T>(fn, X + r * ldx, o, D);
  if (threadIdx.x == 0) out[r] = f;
}

// Fitness of the trial each row left in its non-current buffer, then greedy
// selection (used after the job-per-individual exponential crossover).
template <typename T>
__global__ void __launch_bounds__(256) k_eval_select(const RunDev* __restrict__ runs, int32_t run,
                                                     GenNo gn) {
  const RunDev& P = runs[run];
  const uint32_t gnew = gen_value(gn);
  const uint32_t i = blockIdx.x;
  const uint32_t N = static_cast<uint32_t>(P.N), D = static_cast<uint32_t>(P.D);
  const uint32_t g = run_gen(P, gnew);
  const uint8_t* cur = P.flags + ((g - 1) & 1u) * static_cast<int64_t>(N);
  uint8_t* nxt = P.flags + (g & 1u) * static_cast<int64_t>(N);
  const uint32_t ci = cur[i];
  const T* u = static_cast<const T*>(P.X[ci ^ 1u]) + static_cast<int64_t>(i) * P.ld;
  const T fu = block_row_fitness_rt<T>(P.fn, u, static_cast<const T*>(P.o), D);
  T* fit = static_cast<T*>(P.fit);
  const bool win = fu < fit[i];
  if (threadIdx.x == 0) {
    nxt[i] = static_cast<uint8_t>(win ? ci ^ 1u : ci);
    if (win) fit[i] = fu;
    static_cast<T*>(P.hist)[static_cast<int64_t>(gnew % kHist) * N + i] = win ? fu : Math<T>::inf();
    if (P.tr_idx) P.tr_idx[6 * static_cast<int64_t>(i) + 5] = win ? 1 : 0;
    if (P.tr_ftrial) static_cast<T*>(P.tr_ftrial)[i] = fu;
  }
}

// ---- classic exponential crossover, one job per individual (Alg 8) --------
// One work-item builds individual i's whole trial: copy the parent,
// then walk from j_rand taking the mutant element and drawing the next
// uniform until a draw reaches Cr or the whole row is taken.
template <typename T>
__global__ void __launch_bounds__(64) k_pexp_trial(const RunDev* __restrict__ runs, int32_t run,
                                                   GenNo gn) {
  const RunDev& P = runs[run];
  const uint32_t gnew = gen_value(gn);
  const uint32_t N = static_cast<uint32_t>(P.N), D = static_cast<uint32_t>(P.D);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;  // position (draws)
  if (i >= N) return;
  const uint32_t g = run_gen(P, gnew);
  const uint32_t si = row_of(P, g, i);                          // storage row
  const int64_t ld = P.ld;
  uint32_t r0, r1, r2;
  pick_scheme(P, g, i, N, r0, r1, r2);
  if (P.shuffle) {
    r0 = row_of(P, g, r0);
    r1 = row_of(P, g, r1);
    r2 = row_of(P, g, r2);
  }
  const uint32_t jr = scale_index(draw(P, TAG_XO, g, i, 0).x, D);
  const uint8_t* cur = P.flags + ((g - 1) & 1u) * static_cast<int64_t>(N);
  const uint32_t ci = cur[si];
  const T* xi = static_cast<const T*>(P.X[ci]) + static_cast<int64_t>(si) * ld;
  const T* x0 = static_cast<const T*>(P.X[cur[r0]]) + static_cast<int64_t>(r0) * ld;
  const T* x1 = static_cast<const T*>(P.X[cur[r1]]) + static_cast<int64_t>(r1) * ld;
  const T* x2 = static_cast<const T*>(P.X[cur[r2]]) + static_cast<int64_t>(r2) * ld;
  T* u = static_cast<T*>(P.X[ci ^ 1u]) + static_cast<int64_t>(si) * ld;
  const T F = sizeof(T) == 4 ? static_cast<T>(P.Ff) : static_cast<T>(P.F);
  // u becomes the whole trial; whichever way selection goes, the two buffers
  // then differ only inside this run
  for (uint32_t j = 0; j < D; ++j) u[j] = xi[j];
  uint32_t j = jr, L = 0, e = 0;
  uint4 b = make_uint4(0, 0, 0, 0);
  bool more;
  do {
    u[j] = Math<T>::fma_(F, x1[j] - x2[j], x0[j]);
    j = (j + 1 == D) ? 0 : j + 1;
    ++L;
    if ((e & 3u) == 0) b = draw(P, TAG_EXP, g, i, e >> 2);
    more = static_cast<uint64_t>(word_of(b, e & 3u)) < P.thr && L < D;
    ++e;
  } while (more);
  P.dirty[si] = make_uint4(jr, L, static_cast<uint32_t>(P.partial_wb), 0u);
  if (P.tr_idx) {
    int64_t* q = P.tr_idx + 6 * static_cast<int64_t>(si);
    q[0] = r0; q[1] = r1; q[2] = r2; q[3] = jr; q[4] = L; q[5] = 0;
  }
  if (P.tr_trial)
    for (uint32_t s = 0; s < D; ++s) static_cast<T*>(P.tr_trial)[static_cast<int64_t>(si) * D + s] = u[s];
  if (P.tr_mask)
    for (uint32_t s = 0; s < D; ++s) {
      const uint32_t off = s >= jr ? s - jr : s + D - jr;
      P.tr_mask[static_cast<int64_t>(si) * D + s] = static_cast<uint8_t>(off < L);
    }
}

// ---- best so far (Tables 3-5: best value, best gen) ------------------------

// argmin over n values (lowest index on ties) with one 256-thread block.
template <typename T>
__device__ GenMin block_argmin(const T* v, int64_t n) {
  __shared__ double sf[256];
  __shared__ int64_t si[256];
  double bf = __builtin_huge_val();
  int64_t bi = n;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double f = static_cast<double>(v[i]);
    if (bi == n || f < bf) {  // strict: the lowest index keeps a tie
      bf = f;
      bi = i;
    }
  }
  sf[threadIdx.x] = bf;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double f2 = sf[threadIdx.x + s], f1 = sf[threadIdx.x];
      const int64_t i2 = si[threadIdx.x + s], i1 = si[threadIdx.x];
      if (i2 < n && (i1 >= n || f2 < f1 || (f2 == f1 && i2 < i1))) {
        sf[threadIdx.x] = f2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  GenMin r{sf[0], si[0] < n ? si[0] : 0};
  __syncthreads();
  return r;
}

// Generation 0: the best of the initial population (one block per run).
__global__ void __launch_bounds__(256) k_best_init(const RunDev* __restrict__ runs) {
  const RunDev& P = runs[blockIdx.x];
  const GenMin m = P.dtype == 0 ? block_argmin(static_cast<const double*>(P.fit), P.N)
                                : block_argmin(static_cast<const float*>(P.fit), P.N);
  if (threadIdx.x == 0) {
    BestState* B = P.best;
    B->f = m.f;
    B->idx = m.idx;
    B->gen = run_gen(P, 0);
    B->g = run_gen(P, 0);
  }
}

// Deferred update, pass 1: the minimum over the rows each generation
// replaced (block (k, run) handles generation gfirst + k of that run).
__global__ void __launch_bounds__(256) k_best_gen_min(const RunDev* __restrict__ runs,
                                                      GenNo gfirst) {
  const RunDev& P = runs[blockIdx.y];
  const uint32_t gnew = gen_value(gfirst) + blockIdx.x;
  const int64_t off = static_cast<int64_t>(gnew % kHist) * P.N;
  const GenMin m = P.dtype == 0 ? block_argmin(static_cast<const double*>(P.hist) + off, P.N)
                                : block_argmin(static_cast<const float*>(P.hist) + off, P.N);
  if (threadIdx.x == 0) P.mins[gnew % kHist] = m;
}

// Pass 2: walk the generations in order; a strictly lower minimum than the
// best so far records that generation.  Between improvements every row keeps
// f_i >= best, so the minimum over the replaced rows decides.
__global__ void k_best_scan(const RunDev* __restrict__ runs, int n_runs, GenNo gfirst_no,
                            int count) {
  const uint32_t gfirst = gen_value(gfirst_no);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_runs) return;
  const RunDev& P = runs[r];
  BestState* B = P.best;
  double bf = B->f;
  int64_t bi = B->idx, bg = B->gen;
  for (int k = 0; k < count; ++k) {
    const uint32_t gnew = gfirst + k;
    const GenMin m = P.mins[gnew % kHist];
    if (m.f < bf) {
      bf = m.f;
      bi = m.idx;
      bg = run_gen(P, gnew);
    }
  }
  B->f = bf;
  B->idx = bi;
  B->gen = bg;
  B->g = run_gen(P, gfirst + count - 1);
}

// FP64 fitness of the best row, recomputed from the stored vector.
template <typename T>
__global__ void __launch_bounds__(256) k_best_fp64(const RunDev* __restrict__ runs, int32_t run,
                                                   uint32_t gcur, double* __restrict__ out) {
  const RunDev& P = runs[run];
  const uint32_t N = static_cast<uint32_t>(P.N), D = static_cast<uint32_t>(P.D);
  const int64_t i = P.best->idx;
  const uint8_t* cur = P.flags + (run_gen(P, gcur) & 1u) * static_cast<int64_t>(N);
  const T* x = static_cast<const T*>(P.X[cur[i]]) + i * P.ld;
  const T* o = static_cast<const T*>(P.o);
  __shared__ double red[4];
  if (P.fn == FN_ACKLEY || P.fn == FN_GRIEWANK) {
    // FP64 re-evaluation of the stored-precision row
    double s1 = 0.0, s2 = P.fn == FN_GRIEWANK ? 1.0 : 0.0;
    for (uint32_t j = threadIdx.x; j < D; j += blockDim.x) {
      const double xj = static_cast<double>(x[j]);
      s1 += xj * xj;
      s2 = P.fn == FN_GRIEWANK ? s2 * stat2_term<double, FN_GRIEWANK>(xj, j)
                               : s2 + stat2_term<double, FN_ACKLEY>(xj, j);
    }
    s1 = wave_sum(s1);
    s2 = P.fn == FN_GRIEWANK ? wave_stat2<double, FN_GRIEWANK>(s2) : wave_sum(s2);
    __shared__ double red2[4];
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6] = s1;
      red2[threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double t1 = red[0] + red[1] + red[2] + red[3];
      const double f = P.fn == FN_GRIEWANK
                           ? stat2_finish<double, FN_GRIEWANK>(t1, red2[0] * red2[1] * red2[2] * red2[3], D)
                           : stat2_finish<double, FN_ACKLEY>(t1, red2[0] + red2[1] + red2[2] + red2[3], D);
      *out = canon(f);
    }
    return;
  }
  double acc = 0.0;
  {
    for (uint32_t j = threadIdx.x; j < D; j += blockDim.x) {
      const double xj = static_cast<double>(x[j]);
      const double oj = P.fn == FN_SPHERE ? 0.0 : static_cast<double>(o[j]);
      if (P.fn == FN_SPHERE) acc += point_term<double, FN_SPHERE>(xj, 0.0);
      else if (P.fn == FN_RASTRIGIN) acc += point_term<double, FN_RASTRIGIN>(xj, oj);
      else if (j + 1 < D)
        acc += rosen_term((xj - oj) + 1.0,
                          (static_cast<double>(x[j + 1]) - static_cast<double>(o[j + 1])) + 1.0);
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = canon(red[0] + red[1] + red[2] + red[3]);
}

// The rotated function's FP64 recompute: term k = w_k z_k^2 with
// z_k = sum_j M_kj (x_j - o_j), the caller's FP64 M and the weights
// 10^(6k/(D-1)) in FP64; one wavefront per k reads row k of M in coalesced
// runs and reduces its lanes in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) k_best_rot_terms(const RunDev* __restrict__ runs,
                                                        int32_t run, uint32_t gcur) {
  const RunDev& P = runs[run];
  const uint32_t N = static_cast<uint32_t>(P.N), D = static_cast<uint32_t>(P.D);
  const uint32_t k = blockIdx.x * 4 + threadIdx.x / 64;
  if (k >= D) return;  // whole wavefronts leave together
  const int64_t i = P.best->idx;
  const uint8_t* cur = P.flags + (run_gen(P, gcur) & 1u) * static_cast<int64_t>(N);
  const T* x = static_cast<const T*>(P.X[cur[i]]) + i * P.ld;
  const T* o = static_cast<const T*>(P.o);
  const double* m = P.rot + static_cast<int64_t>(k) * D;
  double z = 0.0;
  for (uint32_t j = threadIdx.x % 64; j < D; j += 64)
    z = __builtin_fma(m[j], static_cast<double>(x[j]) - static_cast<double>(o[j]), z);
  z = wave_sum(z);
  if (threadIdx.x % 64 == 0) {
    const double wk = D > 1 ? pow(10.0, 6.0 * static_cast<double>(k) / static_cast<double>(D - 1)) : 1.0;
    P.bpart[k] = wk * z * z;
  }
}

// Sum of the D terms in a fixed order (strided per thread, then a tree).
__global__ void __launch_bounds__(256) k_best_rot_sum(const RunDev* __restrict__ runs, int32_t run,
                                                      double* __restrict__ out) {
  const RunDev& P = runs[run];
  const int64_t D = P.D;
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < D; k += 256) acc += P.bpart[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = canon(red[0]);
}

// ---- state helpers ---------------------------------------------------------

// Move every row into buffer 0 (rows whose current copy is in buffer 1 are
// copied back) and clear the current flags, so buffer 0 is the population.
template <typename T>
__global__ void __launch_bounds__(256) k_normalize(const RunDev* __restrict__ runs, int32_t run,
                                                   uint32_t gcur) {
  const RunDev& P = runs[run];
  const int64_t N = P.N, ld = P.ld;
  const uint32_t g = run_gen(P, gcur);
  uint8_t* cur = P.flags + (g & 1u) * N;
  const int64_t i = blockIdx.x;
  if (cur[i] == 0) return;
  const T* src = static_cast<const T*>(P.X[1]) + i * ld;
  T* dst = static_cast<T*>(P.X[0]) + i * ld;
  for (int64_t j = threadIdx.x; j < ld; j += blockDim.x) dst[j] = src[j];
  __syncthreads();
  if (threadIdx.x == 0) cur[i] = 0;
}

__global__ void k_gen_base(uint32_t* base, uint32_t v, int add) {
  if (threadIdx.x == 0) *base = add ? *base + v : v;
}

__global__ void k_dirty_reset(const RunDev* __restrict__ runs, int32_t run, uint32_t L) {
  const RunDev& P = runs[run];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < P.N) P.dirty[i] = make_uint4(0u, L, static_cast<uint32_t>(P.partial_wb), 0u);
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

// ---- launchers ---------------------------------------------------------------

static inline unsigned nblk(int64_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

hipError_t launch_dirty_reset(const RunDev* runs, const RunDev& h, int run, uint32_t L,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_dirty_reset, dim3(nblk(h.N, 256)), dim3(256), 0, s, runs, run, L);
  return hipGetLastError();
}

hipError_t launch_init_impl(const RunDev* runs, const RunDev& h, int run, double lo, double hi,
                            double olo, double ohi, const void* shift, hipStream_t s) {
  const int64_t n = h.N * h.ld;
  const bool shifted = h.fn == FN_RASTRIGIN || h.fn == FN_ROSENBROCK || h.fn == FN_ELLIPSOID;
  const int gen_shift = shifted && shift == nullptr;
  if (h.dtype == 0)
    hipLaunchKernelGGL(k_init<double>, dim3(nblk(n, 256)), dim3(256), 0, s, runs, run, lo, hi, olo,
                       ohi, static_cast<const double*>(shift), gen_shift);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(nblk(n, 256)), dim3(256), 0, s, runs, run, lo, hi, olo,
                       ohi, static_cast<const float*>(shift), gen_shift);
  return hipGetLastError();
}

hipError_t launch_eval_pop(const RunDev* runs, const RunDev& h, int run, hipStream_t s) {
  if (h.dtype == 0) hipLaunchKernelGGL(k_eval_pop<double>, dim3(h.N), dim3(256), 0, s, runs, run);
  else hipLaunchKernelGGL(k_eval_pop<float>, dim3(h.N), dim3(256), 0, s, runs, run);
  return hipGetLastError();
}

hipError_t launch_eval_rows(const RunDev& h, const void* X, int64_t rows, int64_t ldx, void* out,
                            hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (h.dtype == 0)
    hipLaunchKernelGGL(k_eval_rows<double>, dim3(rows), dim3(256), 0, s, h.fn,
                       static_cast<const double*>(X), ldx, static_cast<const double*>(h.o),
                       static_cast<uint32_t>(h.D), static_cast<double*>(out));
  else
    hipLaunchKernelGGL(k_eval_rows<float>, dim3(rows), dim3(256), 0, s, h.fn,
                       static_cast<const float*>(X), ldx, static_cast<const float*>(h.o),
                       static_cast<uint32_t>(h.D), static_cast<float*>(out));
  return hipGetLastError();
}

hipError_t launch_eval_select(const RunDev* runs, const RunDev& h, int run, GenNo gnew,
                              hipStream_t s) {
  if (h.dtype == 0) hipLaunchKernelGGL(k_eval_select<double>, dim3(h.N), dim3(256), 0, s, runs, run, gnew);
  else hipLaunchKernelGGL(k_eval_select<float>, dim3(h.N), dim3(256), 0, s, runs, run, gnew);
  return hipGetLastError();
}

hipError_t launch_pexp_trial(const RunDev* runs, const RunDev& h, int run, GenNo gnew,
                             hipStream_t s) {
  if (h.dtype == 0) hipLaunchKernelGGL(k_pexp_trial<double>, dim3(nblk(h.N, 64)), dim3(64), 0, s, runs, run, gnew);
  else hipLaunchKernelGGL(k_pexp_trial<float>, dim3(nblk(h.N, 64)), dim3(64), 0, s, runs, run, gnew);
  return hipGetLastError();
}

hipError_t launch_best_init(const RunDev* runs, int n_runs, hipStream_t s) {
  hipLaunchKernelGGL(k_best_init, dim3(n_runs), dim3(256), 0, s, runs);
  return hipGetLastError();
}

hipError_t launch_best_flush(const RunDev* runs, int n_runs, GenNo gfirst, int count,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_best_gen_min, dim3(count, n_runs), dim3(256), 0, s, runs, gfirst);
  hipLaunchKernelGGL(k_best_scan, dim3(nblk(n_runs, 256)), dim3(256), 0, s, runs, n_runs, gfirst,
                     count);
  return hipGetLastError();
}

hipError_t launch_best_fp64(const RunDev* runs, const RunDev& h, int run, uint32_t gcur,
                            double* out, hipStream_t s) {
  if (h.fn == FN_ELLIPSOID) {
    const unsigned blocks = static_cast<unsigned>((h.D + 3) / 4);
    if (h.dtype == 0)
      hipLaunchKernelGGL(k_best_rot_terms<double>, dim3(blocks), dim3(256), 0, s, runs, run, gcur);
    else
      hipLaunchKernelGGL(k_best_rot_terms<float>, dim3(blocks), dim3(256), 0, s, runs, run, gcur);
    hipLaunchKernelGGL(k_best_rot_sum, dim3(1), dim3(256), 0, s, runs, run, out);
    return hipGetLastError();
  }
  if (h.dtype == 0) hipLaunchKernelGGL(k_best_fp64<double>, dim3(1), dim3(256), 0, s, runs, run, gcur, out);
  else hipLaunchKernelGGL(k_best_fp64<float>, dim3(1), dim3(256), 0, s, runs, run, gcur, out);
  return hipGetLastError();
}

hipError_t launch_normalize(const RunDev* runs, const RunDev& h, int run, uint32_t gcur,
                            hipStream_t s) {
  if (h.dtype == 0) hipLaunchKernelGGL(k_normalize<double>, dim3(h.N), dim3(256), 0, s, runs, run, gcur);
  else hipLaunchKernelGGL(k_normalize<float>, dim3(h.N), dim3(256), 0, s, runs, run, gcur);
  return hipGetLastError();
}

hipError_t launch_gen_base(uint32_t* base, uint32_t v, bool add, hipStream_t s) {
  hipLaunchKernelGGL(k_gen_base, dim3(1), dim3(64), 0, s, base, v, add ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u8, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace de
