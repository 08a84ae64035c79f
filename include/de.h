/*
 * de.h -- C ABI of the MI355X (gfx950) differential-evolution library.
 *
 * One call of de_generation() performs whole generations of parallel DE as
 * restructured in Pan, "Performance Analysis and Improvement of Parallel
 * Differential Evolution" (arXiv:2101.06599), Sec. 2, Alg 2: for every
 * individual of an N x D population (Sec. 2, first paragraph) choose the base
 * and difference indices, build the crossover mask first (binomial, Alg 7 and
 * Eq 2; classic exponential, Alg 8; the new exponential crossover NEC, Eq 9
 * and Alg 9/10), mutate only the masked elements with DE/rand/1 (Eq 1),
 * evaluate the trial and keep it when its fitness is strictly lower (Alg 1).
 * The library also reports the best value and the generation that found it
 * (the "best value / best gen" columns of Tables 3-5).
 *
 * Conventions shared by every entry point:
 *  - Device memory belongs to the caller.  The library never allocates device
 *    memory: all of its state lives in the caller's workspace (de_init), and
 *    every device pointer passed in must stay valid for the handle's life
 *    (workspace, shift, rot) or for the call (X, fit_out, trace buffers).
 *  - Host pointers are borrowed for the duration of the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it in order; calls marked "syncs" wait for it.
 *  - Calls return a de_status and never throw.  A failed HIP call returns
 *    DE_E_HIP; errors of earlier asynchronous work surface at the next call
 *    that synchronises.  de_last_error() returns a message for the last
 *    failure on that handle.
 *  - A handle is not thread-safe; distinct handles are independent.  Work of
 *    one handle enqueued on different streams must be ordered by the caller
 *    (events or synchronisation): generations and evaluations share the
 *    handle's workspace (populations, staging rows, partial sums).
 *  - Population layout in host buffers and in caller device buffers: dense
 *    row-major N x D of the run's dtype (individual i is row i).
 *
 * Random numbers: counter-based Philox4x32-10 keyed by the run's seed; the
 * draws of individual i in generation g do not depend on any other draw, so
 * results are reproducible per (seed, run, generation, individual, element)
 * and independent of launch shape.
 */
#ifndef DE_H
#define DE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DE_OK = 0,
  DE_E_INVALID = 1,      /* argument out of range, NULL where a pointer is required */
  DE_E_UNSUPPORTED = 2,  /* valid but not implemented (e.g. dtype/matmul combination) */
  DE_E_HIP = 3,          /* a HIP runtime call failed */
  DE_E_WORKSPACE = 4,    /* workspace too small or misaligned */
  DE_E_STATE = 5         /* call not valid in the handle's state */
} de_status;

/* Crossover (Sec. 2 Alg 7 / Eq 2; Sec. 3.1 Alg 8; Sec. 3.2 Eq 9, Alg 9, Alg 10). */
typedef enum { DE_XO_BIN = 0, DE_XO_EXP = 1, DE_XO_NEC = 2 } de_crossover;

/* How the classic exponential crossover finds its run length on the GPU.  All
 * three give bit-identical results; they differ only in how the work maps
 * onto the hardware.
 *   DE_EXP_LANE: one lane per individual walks Alg 8's draws in order, the
 *                rest of the row is processed element-parallel.
 *   DE_EXP_JOB:  one work-item per individual builds the whole trial row with
 *                Alg 8's loop (the "job per individual" mapping of Sec. 3.1).
 *   DE_EXP_SCAN: the wavefront tests 256 of Alg 8's draws at a time and takes
 *                the first failing one. */
typedef enum { DE_EXP_LANE = 0, DE_EXP_JOB = 1, DE_EXP_SCAN = 2 } de_exp_impl;

/* Fitness functions.  z = x - o for the shifted functions.
 *   SPHERE:        sum x_j^2
 *   RASTRIGIN:     sum z_j^2 - 10 cos(2 pi z_j) + 10
 *   ROSENBROCK:    sum_{j<D-1} 100 (z_{j+1} - z_j^2)^2 + (z_j - 1)^2 with z = x - o + 1
 *   ELLIPSOID_ROT: sum_k 10^(6k/(D-1)) (M (x - o))_k^2, M a caller-supplied D x D matrix
 *   ACKLEY:        -20 exp(-0.02 sqrt(mean x_j^2)) - exp(mean cos(2 pi x_j)) + 20 + e
 *                  (Sec. 4, with its 0.02; not shifted)
 *   GRIEWANK:      sum x_j^2 / 4000 - prod_j cos(x_j / sqrt(j)) + 1, j counted from 1
 *                  (Sec. 4; not shifted)
 * ACKLEY and GRIEWANK run as single runs only (not in batched handles). */
typedef enum {
  DE_FN_SPHERE = 0,
  DE_FN_RASTRIGIN = 1,
  DE_FN_ROSENBROCK = 2,
  DE_FN_ELLIPSOID_ROT = 3,
  DE_FN_ACKLEY = 4,
  DE_FN_GRIEWANK = 5
} de_function;

typedef enum { DE_FP64 = 0, DE_FP32 = 1 } de_dtype;

/* Base index selection (Sec. 2).
 *   DE_BASE_CLASSIC: r0, r1, r2 uniform, mutually distinct and != i (Alg 1).
 *   DE_BASE_RANDOM:  Alg 3, r0 uniform on [0, N) (may equal i).
 *   DE_BASE_OFFSET:  Alg 4, r0 = (i + r_g) mod N, one r_g in [1, N-1] per
 *                    generation.
 *   DE_BASE_PERM:    Alg 5, r0 = sigma_g(i), a fresh pseudo-random
 *                    permutation of [0, N) every generation.
 * RANDOM, OFFSET and PERM take the difference pair from Alg 6:
 * r1 = (r0 + o1) mod N, r2 = (r1 + o2) mod N with o1, o2 uniform on [1, N-1].
 * The permutation is an eight-round keyed Feistel network on the smallest
 * even-bit power of two >= N, walked until it lands in [0, N) (the paper
 * names no shuffling method). */
typedef enum {
  DE_BASE_CLASSIC = 0,
  DE_BASE_RANDOM = 1,
  DE_BASE_OFFSET = 2,
  DE_BASE_PERM = 3
} de_base;

/* Arithmetic of the rotated function's N x D x D product (ELLIPSOID_ROT only):
 *   DE_MM_FP64:   FP64 matrix cores, FP64 accumulation (dtype FP64)
 *   DE_MM_FP32:   FP32 matrix cores, FP32 accumulation (dtype FP32)
 *   DE_MM_BF16X3: operands split into 2 bf16 pieces, 3 products, FP32 accumulation
 *   DE_MM_BF16X6: operands split into 3 bf16 pieces, 6 products, FP32 accumulation */
typedef enum { DE_MM_FP64 = 0, DE_MM_FP32 = 1, DE_MM_BF16X3 = 2, DE_MM_BF16X6 = 3 } de_matmul;

typedef struct {
  int64_t N;        /* population size, 4 <= N < 2^21 */
  int64_t D;        /* dimension, 1 <= D < 2^21 (2 <= D for ELLIPSOID_ROT) */
  double F;         /* differential weight, finite, >= 0 */
  double CR;        /* crossover rate, 0 <= CR <= 1 */
  int32_t xo;       /* de_crossover */
  int32_t fn;       /* de_function */
  int32_t dtype;    /* de_dtype of population and trial arithmetic */
  int32_t mm;       /* de_matmul, ELLIPSOID_ROT only (ignored otherwise) */
  int32_t exp_impl; /* de_exp_impl, DE_XO_EXP only */
  int32_t tpr;      /* lanes per individual in the generation kernel: 0 = chosen
                       from D, N and dtype; 64, 128, 256, 512 or 1024 forces
                       it (batched: 0, 64, 128 or 256, the same for every
                       run of the batch).  Exp and NEC rows of more than
                       4096 elements are streamed rather than held in
                       registers (256 lanes unless forced).  Indices, masks and
                       trial rows do not depend on it; fitness sums only
                       change their rounding order. */
  int32_t base;     /* de_base */
  int32_t shuffle;  /* 1: shuffle the individuals at the start of every
                       generation (the shuffle of Alg 2), 0: do not.  Applied as a
                       relabelling: position k of generation g works on the
                       individual stored in row pi_g(k) and writes its result
                       back there, so rows never move; draws are addressed by
                       position, trace rows by storage row. */
  int32_t wb;       /* winners' write-back into the row's other buffer:
                       0 = chosen from the population size (whole rows while
                       one buffer of the handle fits in 48 MiB, else only the
                       changed chunks; always the latter for ELLIPSOID_ROT),
                       1 = whole rows, 2 = only the chunks in
                       which the two buffers differ (exp and NEC; binomial
                       rows are always written whole).  Results do not depend
                       on it. */
  int32_t tile;     /* split-bf16 product block shape (ELLIPSOID_ROT with
                       DE_MM_BF16X3 / DE_MM_BF16X6): 0 = the default, 1..3 =
                       three measured shapes (3 pieces: 256x128 and 128x256
                       blocks in two alternating wave groups, 256x128 in one;
                       2 pieces: 128x256 in two groups, 128x128, 256x128 in
                       two groups), of which 0 means 1.  All use the 16x16x32
                       matrix-core form and the same k order, so results do
                       not depend on it.  Must be 0 otherwise. */
  double lo, hi;    /* initial population drawn uniformly from [lo, hi]^D, lo < hi */
  double olo, ohi;  /* shift o drawn uniformly from [olo, ohi]^D when shift == NULL */
  uint64_t seed;    /* Philox key */
  const void* shift;  /* device, D values of dtype, or NULL (not read for SPHERE,
                         ACKLEY, GRIEWANK) */
  const double* rot;  /* device, D x D row-major FP64 M (ELLIPSOID_ROT only, else NULL) */
} de_run_desc;

typedef struct de_handle de_handle;

/* Bytes of device workspace that de_init needs for these runs. */
de_status de_workspace_size(const de_run_desc* runs, int32_t n_runs, size_t* bytes);

/* Alg 2's set-up, before its generation loop: draws every initial population
 * uniformly from the run's box (and the shift), evaluates it (generation 0)
 * and records the best.  Also validates the runs and lays out the workspace
 * (256-byte aligned device memory of at least de_workspace_size bytes).
 * Runs step together: each de_generation call advances all of them.
 * Asynchronous on `stream` apart from a small host-to-device copy of the run
 * tables. */
de_status de_init(de_handle** h, const de_run_desc* runs, int32_t n_runs, void* workspace,
                  size_t ws_bytes, void* stream);

/* Runs n_gens >= 0 generations of every run: Alg 2's generation loop body
 * (index choice, crossover mask, masked mutation, evaluation and selection
 * for all N individuals, synchronously) plus the best-so-far record.
 * Asynchronous. */
de_status de_generation(de_handle* h, int32_t n_gens, void* stream);

/* Alg 2's evaluation on caller rows: fit_out[r] = f(X[r]) for r < rows, with
 * the run's function, shift and dtype (the functions of Sec. 4 and the
 * shifted benchmarks; see de_function).  X: device, rows x D dense of dtype;
 * fit_out: device, rows values of dtype.  Asynchronous. */
de_status de_evaluate(de_handle* h, int32_t run, const void* X, int64_t rows, void* fit_out,
                      void* stream);

/* Best so far of one run: the FP64 fitness of the best vector recomputed on
 * the GPU, its index in the population, the generation that found it (0 = the
 * initial population) and, if x_best_host != NULL, the vector itself (D
 * values of dtype).  Any output pointer may be NULL.  Syncs. */
de_status de_best(de_handle* h, int32_t run, double* f_best, int64_t* idx, int64_t* gen,
                  void* x_best_host, void* stream);

/* Current population (N x D of dtype), fitness (N of dtype) and generation
 * count of one run, copied to the host.  NULL outputs are skipped.  Syncs. */
de_status de_get_state(de_handle* h, int32_t run, void* pop_host, void* fit_host, int64_t* gen,
                       void* stream);

/* Replaces one run's population, fitness and generation count (checkpoint
 * resume).  The best so far becomes (best_f, best_idx, best_gen) when
 * best_idx >= 0, otherwise the argmin of fit_host at generation `gen`.
 * Syncs. */
de_status de_set_state(de_handle* h, int32_t run, const void* pop_host, const void* fit_host,
                       int64_t gen, double best_f, int64_t best_idx, int64_t best_gen,
                       void* stream);

/* The crossover masks of generation `gen` (>= 1, the run's own generation
 * number) of one run, exactly as that generation applies them: the N x D
 * 0/1 matrix that Alg 7 (binomial) and Alg 10 (NEC) return, or the run of
 * Alg 8 (classic exponential), one byte per element, row-major, written to
 * the device buffer `mask` (N * D bytes, caller-owned).  The run's exp_impl
 * picks the classic exponential mapping: DE_EXP_JOB has one work-item per
 * individual walk Alg 8 and write its row (Sec. 3.1's p-exp); LANE and SCAN
 * use a wavefront per row.  All give the same bytes.  Does not change the
 * run's state.  Asynchronous. */
de_status de_masks(de_handle* h, int32_t run, int64_t gen, uint8_t* mask, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the masks
 * de_masks returns, for a run that has no handle and no workspace.  `run`
 * describes the run (N, D, CR, seed, xo, exp_impl are read; the rest is
 * ignored) and run_index is its position in the handle whose draws it
 * reproduces (0 for a single-run handle; [0, 2^24)).  The output is the
 * bytes de_masks(h, run_index, gen, ...) writes for a handle built from the
 * same description.  Needs D <= DE_MASKS_NOALLOC_MAX_D (else DE_E_INVALID).
 * The call's run record and NEC threshold table live in a fixed 1 MiB
 * device array inside the library, one per GPU, kept until the process
 * ends; the call allocates nothing and rewrites every part of the array it
 * reads.  Calls that overlap on one GPU (on different streams, or from
 * different threads) share that array and race: order them.  Asynchronous;
 * errors are read with de_last_error(NULL). */
#define DE_MASKS_NOALLOC_MAX_D 131006
de_status de_masks_noalloc(const de_run_desc* run, int32_t run_index, int64_t gen, uint8_t* mask,
                           void* stream);

/* Debug trace of one run, written by the production kernels for every later
 * generation (each overwrites the previous one).  All device pointers, each
 * may be NULL; all NULL switches tracing off.
 *   idx:    N x 6 int64: r0, r1, r2, j_rand, L, win (L = run length for
 *           exp/NEC, number of crossed elements for bin)
 *   mask:   N x D uint8 crossover mask
 *   trial:  N x D trial vectors of dtype
 *   ftrial: N trial fitness values of dtype */
de_status de_trace(de_handle* h, int32_t run, int64_t* idx, uint8_t* mask, void* trial,
                   void* ftrial);

/* Kernel timing for measurement: while enabled, de_generation records HIP
 * events on the launch stream around the generation's main kernel: around
 * each launch when a generation takes several kernels (the rotated
 * function's product, with its bf16 split pass when the job-per-individual
 * exponential crossover builds the trials, or that crossover's trial kernel),
 * else around the whole run of back-to-back generation launches of the call.
 * de_profile_read syncs and returns the elapsed milliseconds recorded since
 * enabling and the number of main-kernel launches they cover. */
de_status de_profile(de_handle* h, int32_t enable);
de_status de_profile_read(de_handle* h, double* main_ms, int64_t* main_launches);

/* Graph replay: with enable = 1, de_generation runs whole blocks of 64
 * generations (with their best-so-far update) by launching one HIP graph
 * instead of launching each kernel; enable = B > 1 uses blocks of B
 * generations (the best-so-far is updated after every 64 of them and after
 * the last); 0 switches graphs off.  The graph is captured and uploaded to
 * the device by this call (synchronising a private stream; nothing runs on
 * the population), so the first replay costs what later ones do.
 * Generations left over from whole blocks are launched directly.  Results
 * are identical either way.  Ignored while kernel timing (de_profile) is on.
 * DE_E_INVALID for a negative enable; a failed capture returns its HIP error
 * and leaves graphs on, to be captured again on the next call. */
de_status de_graph(de_handle* h, int32_t enable);

/* Message for the last failed call on h (or on a NULL handle); valid until
 * the next call on the same handle. */
const char* de_last_error(const de_handle* h);

/* Frees the host-side handle.  The workspace stays the caller's. */
void de_destroy(de_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* DE_H */
