// Internal layout shared by the runtime (de_runtime.hip) and the kernels.
// Everything a kernel needs about a run sits in one RunDev record in the
// workspace, so one launch can serve one run or hundreds of them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace de {

enum : int { FN_SPHERE = 0, FN_RASTRIGIN = 1, FN_ROSENBROCK = 2, FN_ELLIPSOID = 3, FN_ANY = -1,
             FN_NONE = -2 };
enum : int { XO_BIN = 0, XO_EXP = 1, XO_NEC = 2, XO_ANY = -1 };
enum : int { EXPI_LANE = 0, EXPI_JOB = 1, EXPI_SCAN = 2 };
enum : uint32_t { TAG_INIT = 1, TAG_SHIFT = 2, TAG_IDX = 3, TAG_XO = 4, TAG_BIN = 5, TAG_EXP = 6 };

// Per-run mutable scalars.  `gen` counts completed generations; the kernels
// of generation g = gen + 1 read it and the last kernel of the generation
// advances it, so graph replays need no host involvement.
struct alignas(32) BestState {
  double f;       // best fitness so far (stored precision promoted to FP64)
  int64_t idx;    // row of the best individual
  int64_t gen;    // generation that found it
  uint32_t g;     // completed generations
  uint32_t pad;
};

struct alignas(64) RunDev {
  int64_t N, D, ld;       // ld: row pitch in elements (multiple of 32)
  double F, CR;
  double inv_ln_cr;       // 1 / ln(CR) for the NEC length estimate (0 if CR in {0,1})
  uint64_t thr;           // number of 32-bit words w with (w + 1/2) 2^-32 < CR
  float Ff, pad0;
  uint32_t key0, key1, run_id;
  int32_t fn, xo, exp_impl, dtype, mm;
  void* X[2];             // double-buffered populations, N x ld
  void* fit;              // N fitness values (dtype)
  uint8_t* flags;         // 2 x N: flags[(g & 1) * N + i] = buffer holding row i after gen g
  const void* o;          // shift, ld values (dtype), zero padded
  const uint64_t* T;      // NEC thresholds, T[k] for k = 0..D+1
  BestState* best;
  // rotated function
  const double* rot;      // caller's FP64 M, D x D row-major
  const void* w;          // D weights (dtype)
  const void* B[3];       // M pieces, D x ldk (FP64 / FP32 / bf16 hi, mid, lo)
  int64_t ldk;            // pitch of M pieces and of the partial-sum row
  void* part;             // N x ntile partial sums (dtype)
  int32_t ntile, pad1;
  void* stage;            // N x ld staging rows (rotated evaluate)
  // trace (tests)
  int64_t* tr_idx;
  uint8_t* tr_mask;
  void* tr_trial;
  void* tr_ftrial;
};

// ---- launch helpers implemented in the kernel translation units ---------
struct GenLaunch {
  const RunDev* runs;     // device array
  const RunDev* host;     // host mirror of the same records
  int32_t run;            // run index for single-run launches
  const uint2* rowmap;    // batched: global row -> (run, row)
  int64_t rows;           // rows in this launch
  int32_t tpr;            // threads per row
  hipStream_t s;
};

hipError_t launch_init_impl(const RunDev* runs, const RunDev& h, int run, double lo, double hi,
                            double olo, double ohi, const void* shift, hipStream_t s);
hipError_t launch_eval_pop(const RunDev* runs, const RunDev& h, int run, hipStream_t s);
hipError_t launch_best(const RunDev* runs, int n_runs, bool init, hipStream_t s);
hipError_t launch_generation(const GenLaunch& L, int fn, int xo, int dtype, bool batched);
hipError_t launch_pexp_trial(const RunDev* runs, const RunDev& h, int run, hipStream_t s);
hipError_t launch_eval_select(const RunDev* runs, const RunDev& h, int run, hipStream_t s);
hipError_t launch_eval_rows(const RunDev& h, const void* X, int64_t rows, int64_t ldx, void* out,
                            hipStream_t s);
hipError_t launch_best_fp64(const RunDev* runs, const RunDev& h, int run, double* out,
                            hipStream_t s);
hipError_t launch_normalize(const RunDev* runs, const RunDev& h, int run, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
// rotated function: M pieces and weights from the caller's FP64 M; fitness of
// N rows (the trials of the coming generation when `trials`, else the
// population) into fit_dst or, when select, straight into greedy selection.
hipError_t launch_prepare_rot(const RunDev& h, hipStream_t s);
hipError_t launch_rot_fitness(const RunDev* runs, const RunDev& h, int run, bool trials,
                              hipStream_t s);
hipError_t launch_rot_select(const RunDev* runs, const RunDev& h, int run, hipStream_t s);
hipError_t launch_rot_init_fit(const RunDev* runs, const RunDev& h, int run, hipStream_t s);
hipError_t launch_rot_eval_rows(const RunDev* runs, const RunDev& h, int run, const void* X,
                                int64_t rows, void* out, hipStream_t s);

int rot_tile_n();  // column-tile width of the rotated-function product

}  // namespace de
