/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain sequential reference of parallel DE (Pan, arXiv:2101.06599).
 * Each function names the passage of the paper it follows.  Nothing here is
 * blocked, fused or reordered beyond what the paper states; the generation is
 * synchronous (all trials of generation g are built from generation g-1's
 * population before any selection), which is what Alg 2 does.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared oracle.c -lm  (no fast-math:
 * the trial arithmetic must round exactly as written).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 S-box       */
/* with multipliers 0xD2511F53 / 0xCD9E8D57 and a Weyl key schedule          */
/* (0x9E3779B9, 0xBB67AE85) applied between rounds.                          */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint32_t oracle_word(uint64_t seed, uint32_t run, uint32_t tag, uint32_t g, uint32_t i,
                     uint32_t block, int k) {
  uint32_t ctr[4] = {block, i, g, (tag << 24) | (run & 0xFFFFFFu)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  oracle_philox4x32_10(ctr, key, out);
  return out[k];
}

/* rand(0,1) of the paper as an open-interval uniform (Sec. 3.1 needs U in (0,1)
 * so that ln U is finite). */
double oracle_uniform(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* randint(n) of Alg 7: floor(n * rand) with rand = w 2^-32 in [0,1).  The
 * product is exact in FP64 for n < 2^21. */
int64_t oracle_randint(uint32_t w, int64_t n) {
  return (int64_t)floor((double)w * 0x1p-32 * (double)n);
}

/* Maps r in [0, n - |S|) onto [0, n) \ S, keeping order: walk the excluded
 * values in ascending order and step over each one that is <= r. */
int64_t oracle_skip(int64_t r, const int64_t* excl, int n_excl) {
  int64_t s[8];
  for (int a = 0; a < n_excl; ++a) s[a] = excl[a];
  for (int a = 1; a < n_excl; ++a) /* insertion sort */
    for (int b = a; b > 0 && s[b - 1] > s[b]; --b) {
      int64_t t = s[b]; s[b] = s[b - 1]; s[b - 1] = t;
    }
  for (int a = 0; a < n_excl; ++a)
    if (r >= s[a]) ++r;
  return r;
}

/* DE/rand/1 index choice (Alg 1, Eq 1): base r0 and difference pair
 * r1, r2, all distinct and different from i.  Uses words 0..2 of the IDX block. */
void oracle_indices(uint64_t seed, uint32_t run, int64_t N, uint32_t g, int64_t i, int64_t r[3]) {
  uint32_t w0 = oracle_word(seed, run, OR_TAG_IDX, g, (uint32_t)i, 0, 0);
  uint32_t w1 = oracle_word(seed, run, OR_TAG_IDX, g, (uint32_t)i, 0, 1);
  uint32_t w2 = oracle_word(seed, run, OR_TAG_IDX, g, (uint32_t)i, 0, 2);
  int64_t e1[1] = {i};
  r[0] = oracle_skip(oracle_randint(w0, N - 1), e1, 1);
  int64_t e2[2] = {i, r[0]};
  r[1] = oracle_skip(oracle_randint(w1, N - 2), e2, 2);
  int64_t e3[3] = {i, r[0], r[1]};
  r[2] = oracle_skip(oracle_randint(w2, N - 3), e3, 3);
}

/* A keyed pseudo-random permutation of [0, N) for generation g, used where
 * the paper shuffles (Alg 2, Alg 5).  The paper names no shuffling
 * method; this reading takes a balanced eight-round Feistel network (Luby and
 * Rackoff) on m-bit integers, m even with 2^m >= N (m >= 2), and walks the
 * cycle (Black and Rogaway) until the image falls inside [0, N).  Round r
 * swaps the halves and XORs mix(R ^ K_r) into the new right half; K_r is word
 * r%4 of Philox block r/4 (individual 0, generation g, tag).  mix is the
 * 32-bit integer hash x ^= x>>16; x *= 0x7feb352d; x ^= x>>15;
 * x *= 0x846ca68b; x ^= x>>16.  Eight rounds keep even 4-bit domains close
 * to uniform. */
static uint32_t perm_mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

int64_t oracle_permute(uint64_t seed, uint32_t run, uint32_t tag, uint32_t g, int64_t N, int64_t k) {
  int m = 2;
  while (((int64_t)1 << m) < N) m += 2;
  const int h = m / 2;
  const uint32_t hmask = (1u << h) - 1u;
  uint32_t K[8];
  for (int r = 0; r < 8; ++r) K[r] = oracle_word(seed, run, tag, g, 0, (uint32_t)(r / 4), r % 4);
  uint32_t x = (uint32_t)k;
  do {
    uint32_t L = x >> h, R = x & hmask;
    for (int r = 0; r < 8; ++r) {
      uint32_t t = L ^ (perm_mix(R ^ K[r]) & hmask);
      L = R;
      R = t;
    }
    x = (L << h) | R;
  } while ((int64_t)x >= N);
  return (int64_t)x;
}

/* Base index selection for row (position) i of generation g.
 *   OR_BASE_CLASSIC: r0, r1, r2 as in oracle_indices (Alg 1, distinct, != i).
 *   OR_BASE_RANDOM:  Alg 3, r0 = floor(N U) (IDX word 0).
 *   OR_BASE_OFFSET:  Alg 4, r0 = (i + r_g) mod N with one r_g = ceil((N-1) U)
 *                    per generation, drawn as 1 + randint(N-1) from word 0 of
 *                    the OFFSET block (block 0, individual 0, generation g).
 *   OR_BASE_PERM:    Alg 5, r0 = sigma_g(i), sigma_g = oracle_permute(PERM tag).
 * The three paper schemes take r1, r2 from Alg 6: r1 = (r0 + o1) mod N and
 * r2 = (r1 + o2) mod N with o = ceil((N-1) U), drawn as 1 + randint(N-1) from
 * IDX words 1 and 2 (so r1 != r0 and r2 != r1; nothing else is excluded). */
void oracle_indices_scheme(uint64_t seed, uint32_t run, int base, int64_t N, uint32_t g, int64_t i,
                           int64_t r[3]) {
  if (base == OR_BASE_CLASSIC) {
    oracle_indices(seed, run, N, g, i, r);
    return;
  }
  if (base == OR_BASE_RANDOM) {
    r[0] = oracle_randint(oracle_word(seed, run, OR_TAG_IDX, g, (uint32_t)i, 0, 0), N);
  } else if (base == OR_BASE_OFFSET) {
    int64_t rg = 1 + oracle_randint(oracle_word(seed, run, OR_TAG_OFFSET, g, 0, 0, 0), N - 1);
    r[0] = (i + rg) % N;
  } else {
    r[0] = oracle_permute(seed, run, OR_TAG_PERM, g, N, i);
  }
  int64_t o1 = 1 + oracle_randint(oracle_word(seed, run, OR_TAG_IDX, g, (uint32_t)i, 0, 1), N - 1);
  int64_t o2 = 1 + oracle_randint(oracle_word(seed, run, OR_TAG_IDX, g, (uint32_t)i, 0, 2), N - 1);
  r[1] = (r[0] + o1) % N;
  r[2] = (r[1] + o2) % N;
}

/* Alg 7 / Eq 2: element j crosses if rand < Cr or j = j_rand.  The rand of
 * element j is word j%4 of BIN block j/4. */
void oracle_mask_bin(uint64_t seed, uint32_t run, int64_t D, double CR, uint32_t g, int64_t i,
                     int64_t jrand, uint8_t* mask) {
  for (int64_t j = 0; j < D; ++j) {
    uint32_t w = oracle_word(seed, run, OR_TAG_BIN, g, (uint32_t)i, (uint32_t)(j / 4), (int)(j % 4));
    mask[j] = (uint8_t)((oracle_uniform(w) < CR) || (j == jrand));
  }
}

/* Alg 8: do { take one more element; L++ } while (rand < Cr and L < D).  The
 * rand tested after the L-th element is EXP draw e = L-1 (block e/4, word e%4). */
int64_t oracle_exp_length(uint64_t seed, uint32_t run, int64_t D, double CR, uint32_t g, int64_t i) {
  int64_t L = 0;
  int cont;
  do {
    L += 1;
    int64_t e = L - 1;
    uint32_t w = oracle_word(seed, run, OR_TAG_EXP, g, (uint32_t)i, (uint32_t)(e / 4), (int)(e % 4));
    cont = (oracle_uniform(w) < CR) && (L < D);
  } while (cont);
  return L;
}

/* Eq 9.  For Cr in (0,1), ceil(ln U / ln Cr) >= k exactly when U < Cr^(k-1)
 * (Sec. 3.1, inversion of Eq 4), so L = min(ceil(ln U/ln Cr), D) is the number
 * of k in [1, D] with U < Cr^(k-1).  The powers are the running product
 * Cr^(k-1) = Cr^(k-2) * Cr in FP64.  Cr = 0 gives L = 1 and Cr = 1 gives L = D,
 * the two special cases Eq 9 lists. */
int64_t oracle_nec_length(double U, double CR, int64_t D) {
  int64_t L = 1;
  double t = 1.0;
  while (L < D) {
    t = t * CR;
    if (U < t) L += 1;
    else break;
  }
  return L;
}

/* Eq 9 with logarithms, as printed.  Used only to cross-check the form above. */
int64_t oracle_nec_length_log(double U, double CR, int64_t D) {
  if (CR <= 0.0) return 1;
  if (CR >= 1.0) return D;
  double x = log(U) / log(CR);
  double L = ceil(x);
  if (L > (double)D) return D;
  if (L < 1.0) return 1;
  return (int64_t)L;
}

/* Alg 9: starting at j, copy L elements with wrap-around. */
void oracle_alg9_mask(int64_t D, int64_t j, int64_t L, uint8_t* mask) {
  memset(mask, 0, (size_t)D);
  int64_t l = 0;
  do {
    mask[j] = 1;
    j = (j + 1) % D;
    l += 1;
  } while (l < L);
}

/* Alg 10 builds the run mask elementwise from (j_rand, L).  As printed its XOR
 * of two comparisons does not reproduce Alg 9 (it misses every run that wraps
 * past D-1); the elementwise statement of the same run is
 * mask_s = ((s - j_rand) mod D) < L. */
void oracle_alg10_mask(int64_t D, int64_t j, int64_t L, uint8_t* mask) {
  for (int64_t s = 0; s < D; ++s) {
    int64_t off = ((s - j) % D + D) % D;
    mask[s] = (uint8_t)(off < L);
  }
}

void oracle_lengths(int kind, uint64_t seed, uint32_t run, int64_t D, double CR, int64_t n,
                    int64_t* out) {
  for (int64_t k = 0; k < n; ++k) {
    uint32_t g = (uint32_t)(1 + k / 4096);
    int64_t i = k % 4096;
    if (kind == 0) {
      out[k] = oracle_exp_length(seed, run, D, CR, g, i);
    } else {
      uint32_t w = oracle_word(seed, run, OR_TAG_XO, g, (uint32_t)i, 0, 1);
      out[k] = oracle_nec_length(oracle_uniform(w), CR, D);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Fitness (Sec. 4 and the shifted/rotated forms used by the experiments).   */
/* Sums in long double; NaN maps to +inf so that it never wins selection.    */
/* ------------------------------------------------------------------------ */
static const long double PI_L = 3.141592653589793238462643383279502884L;

void oracle_ellipsoid_weights(int64_t D, double* w) {
  for (int64_t k = 0; k < D; ++k)
    w[k] = (D > 1) ? pow(10.0, 6.0 * (double)k / (double)(D - 1)) : 1.0;
}

static double finite_or_inf(long double v) {
  double d = (double)v;
  return isnan(d) ? INFINITY : d;
}

/* Ackley (Sec. 4): -20 exp(-0.02 sqrt(mean x^2)) - exp(mean cos 2 pi x) + 20 + e.
 * Written as the sum of two non-negative terms: with a = -0.02 sqrt(mean x^2)
 * and cos(2 pi x) = 1 - 2 sin^2(pi x), exp(mean cos 2 pi x) = e exp(b) with
 * b = -2 mean sin^2(pi x), so
 *   f = 20 (1 - e^a) + e (1 - e^b) = -20 expm1(a) - e expm1(b).
 * The printed order subtracts numbers close to 20 + e and keeps only their
 * absolute accuracy near x = 0; this order keeps f's relative accuracy.  The
 * sine is taken of pi r with r = x - nearest integer (exact in FP64), so its
 * argument carries no rounding.  oracle_ackley_printed() evaluates the
 * printed order for a cross-check. */
static const long double E_L = 2.718281828459045235360287471352662498L;

static void ackley_terms(int64_t D, const double* x, long double* t1, long double* t2) {
  long double sq = 0.0L, s2 = 0.0L;
  for (int64_t j = 0; j < D; ++j) {
    sq += (long double)x[j] * (long double)x[j];
    double r = x[j] - nearbyint(x[j]);
    long double sn = sinl(PI_L * (long double)r);
    s2 += sn * sn;
  }
  *t1 = -20.0L * expm1l(-0.02L * sqrtl(sq / (long double)D));
  *t2 = -E_L * expm1l(-2.0L * s2 / (long double)D);
}

double oracle_ackley_printed(int64_t D, const double* x) {
  long double sq = 0.0L, cs = 0.0L;
  for (int64_t j = 0; j < D; ++j) {
    sq += (long double)x[j] * (long double)x[j];
    cs += cosl(2.0L * PI_L * (long double)x[j]);
  }
  long double s = -20.0L * expl(-0.02L * sqrtl(sq / (long double)D)) - expl(cs / (long double)D) +
                  20.0L + E_L;
  return finite_or_inf(s);
}

double oracle_fitness(int fn, int64_t D, const double* x, const double* o, const double* rot,
                      const double* w) {
  long double s = 0.0L;
  switch (fn) {
    case OR_FN_SPHERE:
      for (int64_t j = 0; j < D; ++j) s += (long double)x[j] * (long double)x[j];
      break;
    case OR_FN_RASTRIGIN:
      /* z^2 - 10 cos(2 pi z) + 10 = z^2 + 20 sin^2(pi z) */
      for (int64_t j = 0; j < D; ++j) {
        long double z = (long double)x[j] - (long double)o[j];
        long double sn = sinl(PI_L * z);
        s += z * z + 20.0L * sn * sn;
      }
      break;
    case OR_FN_ROSENBROCK:
      /* z = x - o + 1; sum_{j<D-1} 100 (z_{j+1} - z_j^2)^2 + (z_j - 1)^2 */
      for (int64_t j = 0; j + 1 < D; ++j) {
        long double z0 = (long double)x[j] - (long double)o[j] + 1.0L;
        long double z1 = (long double)x[j + 1] - (long double)o[j + 1] + 1.0L;
        long double a = z1 - z0 * z0;
        long double b = z0 - 1.0L;
        s += 100.0L * a * a + b * b;
      }
      break;
    case OR_FN_ACKLEY: {
      long double t1, t2;
      ackley_terms(D, x, &t1, &t2);
      s = t1 + t2;
      break;
    }
    case OR_FN_GRIEWANK: {
      /* Sec. 4: sum x_j^2 / 4000 - prod cos(x_j / sqrt(j)) + 1, j from 1 */
      long double sq = 0.0L, pr = 1.0L;
      for (int64_t j = 0; j < D; ++j) {
        sq += (long double)x[j] * (long double)x[j];
        pr *= cosl((long double)x[j] / sqrtl((long double)(j + 1)));
      }
      s = sq / 4000.0L - pr + 1.0L;
      break;
    }
    case OR_FN_ELLIPSOID_ROT:
      /* z = M (x - o); sum_k w_k z_k^2 */
      for (int64_t k = 0; k < D; ++k) {
        long double z = 0.0L;
        for (int64_t j = 0; j < D; ++j)
          z += (long double)rot[k * D + j] * ((long double)x[j] - (long double)o[j]);
        s += (long double)w[k] * z * z;
      }
      break;
    default:
      return NAN;
  }
  return finite_or_inf(s);
}

double oracle_fitness_phi(int fn, int64_t D, const double* x, const double* o, const double* rot,
                          const double* w) {
  if (fn == OR_FN_ACKLEY) {
    /* the two terms of the cancellation-free form, each taken positive */
    long double t1, t2;
    ackley_terms(D, x, &t1, &t2);
    return finite_or_inf(fabsl(t1) + fabsl(t2));
  }
  if (fn == OR_FN_GRIEWANK) {
    /* 1 - prod cos cancels near the optimum: scale by the parts */
    long double sq = 0.0L, pr = 1.0L;
    for (int64_t j = 0; j < D; ++j) {
      sq += (long double)x[j] * (long double)x[j];
      pr *= cosl((long double)x[j] / sqrtl((long double)(j + 1)));
    }
    return finite_or_inf(sq / 4000.0L + fabsl(pr) + 1.0L);
  }
  if (fn != OR_FN_ROSENBROCK) return oracle_fitness(fn, D, x, o, rot, w);
  long double s = 0.0L;
  for (int64_t j = 0; j + 1 < D; ++j) {
    long double z0 = (long double)x[j] - (long double)o[j] + 1.0L;
    long double z1 = (long double)x[j + 1] - (long double)o[j + 1] + 1.0L;
    long double a = fabsl(z1) + z0 * z0;
    long double b = fabsl(z0) + 1.0L;
    s += 100.0L * a * a + b * b;
  }
  return finite_or_inf(s);
}

/* ------------------------------------------------------------------------ */
/* A whole run: Alg 2 with the generation made synchronous.                 */
/* ------------------------------------------------------------------------ */
struct oracle_state {
  oracle_desc d;
  double* x;      /* N x D; FP32 runs hold float values */
  double* fit;    /* N */
  double* o;      /* D */
  double* rot;    /* D x D or NULL */
  double* w;      /* D */
  double* u;      /* N x D trial scratch */
  double* fu;     /* N */
  int64_t* tr;    /* N x 6 */
  uint8_t* mask;  /* N x D */
  int64_t gen;
  double best_f;
  int64_t best_idx, best_gen;
};

static int uses_shift(int fn) {
  return fn == OR_FN_RASTRIGIN || fn == OR_FN_ROSENBROCK || fn == OR_FN_ELLIPSOID_ROT;
}

/* Uniform sample in [lo, hi] for element j: FP64 takes 53 bits from two
 * words of block j/2, FP32 takes 24 bits from word j%4 of block j/4. */
static double init_value(const oracle_desc* d, uint32_t tag, uint32_t i, int64_t j, double lo,
                         double hi) {
  if (d->dtype == OR_FP64) {
    uint32_t a = oracle_word(d->seed, (uint32_t)d->run, tag, 0, i, (uint32_t)(j / 2), (int)(2 * (j % 2)));
    uint32_t b = oracle_word(d->seed, (uint32_t)d->run, tag, 0, i, (uint32_t)(j / 2), (int)(2 * (j % 2) + 1));
    double u53 = ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * 0x1p-53;
    return fma(hi - lo, u53, lo);
  } else {
    uint32_t a = oracle_word(d->seed, (uint32_t)d->run, tag, 0, i, (uint32_t)(j / 4), (int)(j % 4));
    float u24 = (float)(a >> 8) * 0x1p-24f;
    float lof = (float)lo, hif = (float)hi;
    return (double)fmaf(hif - lof, u24, lof);
  }
}

static double eval_row(const oracle_state* s, const double* x) {
  return oracle_fitness(s->d.fn, s->d.D, x, s->o, s->rot, s->w);
}

/* best value / best gen of Tables 3-5: m = argmin fit (lowest index on ties);
 * a strict improvement on the best so far records the generation. */
static void update_best(oracle_state* s) {
  int64_t m = 0;
  for (int64_t i = 1; i < s->d.N; ++i)
    if (s->fit[i] < s->fit[m]) m = i;
  if (s->fit[m] < s->best_f) {
    s->best_f = s->fit[m];
    s->best_idx = m;
    s->best_gen = s->gen;
  }
}

oracle_state* oracle_create(const oracle_desc* d) {
  if (d->N < 4 || d->D < 1 || d->N >= (1 << 21) || d->D >= (1 << 21)) return NULL;
  if (d->base < OR_BASE_CLASSIC || d->base > OR_BASE_PERM) return NULL;
  if (d->fn == OR_FN_ELLIPSOID_ROT && (d->rot == NULL || d->D < 2)) return NULL;
  oracle_state* s = (oracle_state*)calloc(1, sizeof(oracle_state));
  s->d = *d;
  int64_t N = d->N, D = d->D;
  s->x = (double*)malloc(sizeof(double) * N * D);
  s->u = (double*)malloc(sizeof(double) * N * D);
  s->fit = (double*)malloc(sizeof(double) * N);
  s->fu = (double*)malloc(sizeof(double) * N);
  s->o = (double*)calloc((size_t)D, sizeof(double));
  s->w = (double*)malloc(sizeof(double) * D);
  s->tr = (int64_t*)malloc(sizeof(int64_t) * 6 * N);
  s->mask = (uint8_t*)malloc((size_t)(N * D));
  s->rot = NULL;
  if (d->fn == OR_FN_ELLIPSOID_ROT) {
    s->rot = (double*)malloc(sizeof(double) * D * D);
    memcpy(s->rot, d->rot, sizeof(double) * D * D);
  }
  s->d.rot = s->rot;
  oracle_ellipsoid_weights(D, s->w);
  if (uses_shift(d->fn)) {
    for (int64_t j = 0; j < D; ++j) {
      if (d->shift) s->o[j] = d->dtype == OR_FP32 ? (double)(float)d->shift[j] : d->shift[j];
      else s->o[j] = init_value(d, OR_TAG_SHIFT, 0, j, d->olo, d->ohi);
    }
  }
  s->d.shift = NULL;
  /* Alg 2, before its loop: initialise the population matrix and evaluate it. */
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = 0; j < D; ++j)
      s->x[i * D + j] = init_value(d, OR_TAG_INIT, (uint32_t)i, j, d->lo, d->hi);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) s->fit[i] = d->lazy ? NAN : eval_row(s, s->x + i * D);
  s->gen = 0;
  s->best_f = INFINITY;
  s->best_idx = 0;
  s->best_gen = 0;
  update_best(s);
  if (s->best_f == INFINITY) { s->best_idx = 0; s->best_gen = 0; }
  return s;
}

void oracle_destroy(oracle_state* s) {
  if (!s) return;
  free(s->x); free(s->u); free(s->fit); free(s->fu); free(s->o); free(s->w);
  free(s->tr); free(s->mask); free(s->rot); free(s);
}

/* Storage row of position k in generation g: with the shuffle of Alg 2 the
 * individuals are reordered by pi_g before anything else, so
 * position k holds the individual stored in row pi_g(k); without it, k. */
static int64_t row_of(const oracle_desc* d, uint32_t g, int64_t k) {
  return d->shuffle ? oracle_permute(d->seed, (uint32_t)d->run, OR_TAG_SHUFFLE, g, d->N, k) : k;
}

/* Generation g's trial for position i from population x (the body of Alg 2's
 * loop for one row): choose r0, r1, r2, build the crossover mask first,
 * copy the individual at position i and overwrite the masked elements with
 * the DE/rand/1 mutant x_r0 + F (x_r1 - x_r2) (Eq 1), then
 * evaluate.  Draws are addressed by position; t[0..2] are the
 * storage rows of r0, r1, r2. */
static void build_trial(const oracle_state* s, const double* x, uint32_t g, int64_t i,
                        int64_t* t, uint8_t* m, double* ui, double* fu) {
  const oracle_desc* d = &s->d;
  int64_t N = d->N, D = d->D;
  int64_t r[3];
  oracle_indices_scheme(d->seed, (uint32_t)d->run, d->base, N, g, i, r);
  for (int a = 0; a < 3; ++a) r[a] = row_of(d, g, r[a]);
  uint32_t xw0 = oracle_word(d->seed, (uint32_t)d->run, OR_TAG_XO, g, (uint32_t)i, 0, 0);
  uint32_t xw1 = oracle_word(d->seed, (uint32_t)d->run, OR_TAG_XO, g, (uint32_t)i, 0, 1);
  int64_t jrand = oracle_randint(xw0, D);
  int64_t L;
  if (d->xo == OR_XO_BIN) {
    oracle_mask_bin(d->seed, (uint32_t)d->run, D, d->CR, g, i, jrand, m);
    L = 0;
    for (int64_t j = 0; j < D; ++j) L += m[j];
  } else {
    if (d->xo == OR_XO_EXP) L = oracle_exp_length(d->seed, (uint32_t)d->run, D, d->CR, g, i);
    else L = oracle_nec_length(oracle_uniform(xw1), d->CR, D);
    oracle_alg9_mask(D, jrand, L, m);
  }
  const double* x0 = x + r[0] * D;
  const double* x1 = x + r[1] * D;
  const double* x2 = x + r[2] * D;
  const double* xi = x + row_of(d, g, i) * D;
  for (int64_t j = 0; j < D; ++j) {
    if (!m[j]) {
      ui[j] = xi[j];
    } else if (d->dtype == OR_FP64) {
      ui[j] = fma(d->F, x1[j] - x2[j], x0[j]);
    } else {
      float diff = (float)x1[j] - (float)x2[j];
      ui[j] = (double)fmaf((float)d->F, diff, (float)x0[j]);
    }
  }
  *fu = eval_row(s, ui);
  t[0] = r[0]; t[1] = r[1]; t[2] = r[2]; t[3] = jrand; t[4] = L; t[5] = 0;
}

/* One generation of Alg 2: every trial is built from generation
 * g-1, then u_i replaces x_i wherever f(u_i) < f_i strictly (Alg 2's
 * selection, Alg 1's replacement test).  The shuffle is a relabelling: position k works
 * on storage row pi_g(k) and its result goes back to that row, so the
 * population is never moved (see row_of).  Trace arrays are kept by row. */
static void one_generation(oracle_state* s) {
  const oracle_desc* d = &s->d;
  int64_t N = d->N, D = d->D;
  uint32_t g = (uint32_t)(s->gen + 1);
  /* the N trials are independent (each reads x and writes its own row of
   * the scratch arrays), so an OpenMP build gives the same bits */
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < N; ++k) {
    int64_t i = row_of(d, g, k);
    build_trial(s, s->x, g, k, s->tr + 6 * i, s->mask + i * D, s->u + i * D, s->fu + i);
  }
  s->gen += 1;
  for (int64_t i = 0; i < N; ++i) {
    if (s->fu[i] < s->fit[i]) {
      memcpy(s->x + i * D, s->u + i * D, sizeof(double) * D);
      s->fit[i] = s->fu[i];
      s->tr[6 * i + 5] = 1;
    }
  }
  update_best(s);
}

void oracle_individual(const oracle_state* s, const double* pop, int64_t g, int64_t i,
                       int64_t* idx6, uint8_t* mask, double* trial, double* ftrial) {
  int64_t k = i;
  if (s->d.shuffle)  /* the position whose storage row is i */
    for (k = 0; k < s->d.N && row_of(&s->d, (uint32_t)g, k) != i; ++k) {
    }
  build_trial(s, pop, (uint32_t)g, k, idx6, mask, trial, ftrial);
}

int oracle_generation(oracle_state* s, int64_t n, int64_t* trace_idx, uint8_t* trace_mask,
                      double* trace_trial, double* trace_ftrial) {
  if (!s || n < 0 || s->d.lazy) return 1;
  for (int64_t k = 0; k < n; ++k) one_generation(s);
  if (n > 0) {
    int64_t N = s->d.N, D = s->d.D;
    if (trace_idx) memcpy(trace_idx, s->tr, sizeof(int64_t) * 6 * N);
    if (trace_mask) memcpy(trace_mask, s->mask, (size_t)(N * D));
    if (trace_trial) memcpy(trace_trial, s->u, sizeof(double) * N * D);
    if (trace_ftrial) memcpy(trace_ftrial, s->fu, sizeof(double) * N);
  }
  return 0;
}

void oracle_get_state(const oracle_state* s, double* pop, double* fit, int64_t* gen) {
  if (pop) memcpy(pop, s->x, sizeof(double) * s->d.N * s->d.D);
  if (fit) memcpy(fit, s->fit, sizeof(double) * s->d.N);
  if (gen) *gen = s->gen;
}

void oracle_set_state(oracle_state* s, const double* pop, const double* fit, int64_t gen,
                      double best_f, int64_t best_idx, int64_t best_gen) {
  int64_t N = s->d.N, D = s->d.D;
  for (int64_t k = 0; k < N * D; ++k)
    s->x[k] = s->d.dtype == OR_FP32 ? (double)(float)pop[k] : pop[k];
  for (int64_t i = 0; i < N; ++i) s->fit[i] = isnan(fit[i]) ? INFINITY : fit[i];
  s->gen = gen;
  s->best_f = best_f;
  s->best_idx = best_idx;
  s->best_gen = best_gen;
}

void oracle_get_best(const oracle_state* s, double* f, int64_t* idx, int64_t* gen, double* xbest) {
  if (f) *f = s->best_f;
  if (idx) *idx = s->best_idx;
  if (gen) *gen = s->best_gen;
  if (xbest) memcpy(xbest, s->x + s->best_idx * s->d.D, sizeof(double) * s->d.D);
}

void oracle_get_shift(const oracle_state* s, double* o) {
  memcpy(o, s->o, sizeof(double) * s->d.D);
}

int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
