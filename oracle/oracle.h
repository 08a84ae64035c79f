/*
 * oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU reference of one generation of parallel
 * differential evolution (DE/rand/1 with binomial, classic exponential or the
 * paper's new exponential crossover, fitness evaluation and greedy
 * selection), written from Pan, "Performance Analysis and Improvement of
 * Parallel Differential Evolution" (arXiv:2101.06599).  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU library never links, calls or includes anything from this directory.
 *
 * Arithmetic is FP64 (fitness sums in long double) unless the run's dtype is
 * FP32, in which case the trial arithmetic is FP32 (the population is stored
 * as float) and fitness is still evaluated in extended precision on the
 * promoted values.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), one
 * 128-bit block per counter (c0 = block, c1 = individual, c2 = generation,
 * c3 = tag << 24 | run), key = (seed low 32 bits, seed high 32 bits).
 * A 32-bit word w stands for the uniform number U = (w + 1/2) 2^-32 in (0,1).
 *
 * Parity: every function here is pinned by a CPU test except where its
 * comment says "parity unpinned".
 */
#ifndef DE_ORACLE_H
#define DE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_XO_BIN = 0, OR_XO_EXP = 1, OR_XO_NEC = 2 };
enum { OR_FN_SPHERE = 0, OR_FN_RASTRIGIN = 1, OR_FN_ROSENBROCK = 2, OR_FN_ELLIPSOID_ROT = 3,
       OR_FN_ACKLEY = 4, OR_FN_GRIEWANK = 5 };
enum { OR_FP64 = 0, OR_FP32 = 1 };
enum { OR_TAG_INIT = 1, OR_TAG_SHIFT = 2, OR_TAG_IDX = 3, OR_TAG_XO = 4, OR_TAG_BIN = 5, OR_TAG_EXP = 6,
       OR_TAG_OFFSET = 7, OR_TAG_PERM = 8, OR_TAG_SHUFFLE = 9 };
/* base index selection: classic DE/rand/1 (r0, r1, r2 distinct and != i),
 * or Alg 3 / Alg 4 / Alg 5 for r0 with Alg 6's offsets for r1, r2 */
enum { OR_BASE_CLASSIC = 0, OR_BASE_RANDOM = 1, OR_BASE_OFFSET = 2, OR_BASE_PERM = 3 };

/* ---- random numbers ---------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* word `k` (0..3) of the block addressed by (block, i, g, tag, run) */
uint32_t oracle_word(uint64_t seed, uint32_t run, uint32_t tag, uint32_t g, uint32_t i,
                     uint32_t block, int k);
double oracle_uniform(uint32_t w);                        /* (w + 1/2) 2^-32 */
int64_t oracle_randint(uint32_t w, int64_t n);            /* floor(n * w 2^-32) */
int64_t oracle_skip(int64_t r, const int64_t* excl, int n_excl);

/* ---- operators (one individual) ---------------------------------------- */
/* r0 (base), r1, r2 (difference pair) for individual i, generation g */
void oracle_indices(uint64_t seed, uint32_t run, int64_t N, uint32_t g, int64_t i, int64_t r[3]);
/* r0, r1, r2 for row (position) i under a base scheme (OR_BASE_*) */
void oracle_indices_scheme(uint64_t seed, uint32_t run, int base, int64_t N, uint32_t g, int64_t i,
                           int64_t r[3]);
/* keyed pseudo-random permutation of [0, N) for generation g: image of k */
int64_t oracle_permute(uint64_t seed, uint32_t run, uint32_t tag, uint32_t g, int64_t N, int64_t k);
/* binomial mask (Alg 7, Eq 2) */
void oracle_mask_bin(uint64_t seed, uint32_t run, int64_t D, double CR, uint32_t g, int64_t i,
                     int64_t jrand, uint8_t* mask);
/* classic exponential crossover run length (Alg 8): one draw per step */
int64_t oracle_exp_length(uint64_t seed, uint32_t run, int64_t D, double CR, uint32_t g, int64_t i);
/* NEC run length, Eq 9 as the event U < Cr^(k-1) for k = 2..D (see oracle.c) */
int64_t oracle_nec_length(double U, double CR, int64_t D);
/* NEC run length, Eq 9 written with logarithms (cross-check only) */
int64_t oracle_nec_length_log(double U, double CR, int64_t D);
/* Alg 9 for one individual: copy L elements from v into u starting at j with wrap */
void oracle_alg9_mask(int64_t D, int64_t j, int64_t L, uint8_t* mask);
/* Alg 10 with the comparison fixed (see oracle.c): elementwise run mask */
void oracle_alg10_mask(int64_t D, int64_t j, int64_t L, uint8_t* mask);
/* Run lengths of n individuals for the statistical pins: individual k is
 * (generation 1 + k / 4096, position k % 4096) of the run.  kind 0: Alg 8
 * (oracle_exp_length), kind 1: NEC (oracle_nec_length of XO word 1). */
void oracle_lengths(int kind, uint64_t seed, uint32_t run, int64_t D, double CR, int64_t n,
                    int64_t* out);

/* ---- fitness ------------------------------------------------------------ */
/* f(x); o may be NULL for the sphere; rot (D x D row-major) and w only for the
 * rotated ellipsoid.  Returns +inf for NaN. */
double oracle_fitness(int fn, int64_t D, const double* x, const double* o, const double* rot,
                      const double* w);
/* Tolerance scale: the sum of the absolute values of the terms whose rounding
 * the evaluation carries.  Rosenbrock: each pair's parts |z_{j+1}| + z_j^2
 * and |z_j| + 1; Griewank: sum x^2 / 4000 + |prod cos| + 1 (the final
 * 1 - prod cancels); Ackley: the two terms of its cancellation-free form,
 * which are both >= 0, so the scale is f itself; the sphere, Rastrigin and
 * the ellipsoid are sums of non-negative terms: f. */
double oracle_fitness_phi(int fn, int64_t D, const double* x, const double* o, const double* rot,
                          const double* w);
void oracle_ellipsoid_weights(int64_t D, double* w);
/* Ackley in the order Sec. 4 prints it (cross-check only) */
double oracle_ackley_printed(int64_t D, const double* x);

/* ---- a whole run --------------------------------------------------------- */
typedef struct {
  int64_t N, D;
  double F, CR;
  int32_t xo, fn, dtype, run;
  double lo, hi;        /* initial box */
  double olo, ohi;      /* shift box, used when shift == NULL */
  uint64_t seed;
  const double* shift;  /* D values or NULL */
  const double* rot;    /* D x D row-major, rotated ellipsoid only */
  int32_t lazy;         /* 1: skip the initial evaluation (per-individual use only) */
  int32_t base;         /* OR_BASE_* */
  int32_t shuffle;      /* 1: shuffle the individuals every generation (Alg 2) */
  int32_t pad;
} oracle_desc;

typedef struct oracle_state oracle_state;

oracle_state* oracle_create(const oracle_desc* d);   /* init + evaluate; g = 0 */
void oracle_destroy(oracle_state* s);
/* n generations; if trace_idx != NULL the last generation's decisions are kept:
 * trace_idx N x 6 (r0, r1, r2, jrand, L, win), trace_mask N x D,
 * trace_trial N x D (promoted), trace_ftrial N. */
int oracle_generation(oracle_state* s, int64_t n, int64_t* trace_idx, uint8_t* trace_mask,
                      double* trace_trial, double* trace_ftrial);
void oracle_get_state(const oracle_state* s, double* pop, double* fit, int64_t* gen);
void oracle_set_state(oracle_state* s, const double* pop, const double* fit, int64_t gen,
                      double best_f, int64_t best_idx, int64_t best_gen);
void oracle_get_best(const oracle_state* s, double* f, int64_t* idx, int64_t* gen, double* xbest);
void oracle_get_shift(const oracle_state* s, double* o);
/* Threads used for the per-individual loops of a generation (OpenMP build);
 * n <= 0 leaves the count unchanged.  Returns the count now in effect (1 when
 * built without OpenMP).  Results do not depend on it. */
int oracle_set_threads(int n);
/* Generation g's trial for the individual stored in row i, built from the
 * population `pop` (N x D, the population after generation g-1): idx6 = r0,
 * r1, r2 (rows read), jrand, L, 0; mask and trial D values; *ftrial =
 * f(trial).  With the shuffle, row i is the one at position k = pi_g^-1(i). */
void oracle_individual(const oracle_state* s, const double* pop, int64_t g, int64_t i,
                       int64_t* idx6, uint8_t* mask, double* trial, double* ftrial);

#ifdef __cplusplus
}
#endif
#endif
