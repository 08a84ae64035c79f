// Internal layout shared by the runtime (de_runtime.hip) and the kernels.
// Everything a kernel needs about a run sits in one RunDev record in the
// workspace, so one launch can serve one run or hundreds of them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace de {

enum : int { FN_SPHERE = 0, FN_RASTRIGIN = 1, FN_ROSENBROCK = 2, FN_ELLIPSOID = 3, FN_ACKLEY = 4,
             FN_GRIEWANK = 5, FN_ANY = -1, FN_NONE = -2 };
enum : int { XO_BIN = 0, XO_EXP = 1, XO_NEC = 2, XO_ANY = -1 };
enum : int { EXPI_LANE = 0, EXPI_JOB = 1, EXPI_SCAN = 2 };
enum : uint32_t { TAG_INIT = 1, TAG_SHIFT = 2, TAG_IDX = 3, TAG_XO = 4, TAG_BIN = 5, TAG_EXP = 6,
                  TAG_OFFSET = 7, TAG_PERM = 8, TAG_SHUFFLE = 9 };
enum : int { BASE_CLASSIC = 0, BASE_RANDOM = 1, BASE_OFFSET = 2, BASE_PERM = 3 };
enum : int { MM_FP64 = 0, MM_FP32 = 1, MM_BF16X3 = 2, MM_BF16X6 = 3 };  // rotated product modes

// Best so far of one run, as of generation g.  Kernels of a generation get
// the handle's generation number as an argument (the host knows it without
// asking the device); a run's own number is that plus its gen_offset.
struct alignas(32) BestState {
  double f;       // best fitness so far (stored precision promoted to FP64)
  int64_t idx;    // row of the best individual
  int64_t gen;    // generation that found it
  uint32_t g;     // generation the record is up to date with
  uint32_t pad;
};

// Generations whose best-so-far update is deferred: every row writes its
// post-selection fitness (winners) or +inf (others) into slot g % kHist of a
// ring, and one pass over up to kHist generations updates the BestState.
constexpr int kHist = 64;

constexpr uint32_t kDirtyAll = 0xFFFFFFFFu;  // dirty run length meaning "the whole row"

struct alignas(16) GenMin {
  double f;
  int64_t idx;
};

struct alignas(64) RunDev {
  int64_t N, D, ld;       // ld: row pitch in elements (multiple of 32)
  double F, CR;
  double inv_ln_cr;       // 1 / ln(CR), 0 when CR is 0 or 1 (NEC length short-cut)
  uint64_t thr;           // number of 32-bit words w with (w + 1/2) 2^-32 < CR
  float Ff, pad0;
  uint32_t key0, key1, run_id;
  int32_t fn, xo, exp_impl, dtype, mm;
  int32_t base, shuffle;  // base index scheme; per-generation shuffle on/off
  int32_t partial_wb;     // winners write only the chunks their buffers differ in
  int32_t tile;           // split-bf16 product tile shape (0 = default)
  void* X[2];             // double-buffered populations, N x ld
  void* fit;              // N fitness values (dtype)
  uint8_t* flags;         // 2 x N: flags[(g & 1) * N + i] = buffer holding row i after gen g
  uint4* dirty;           // N: (j0, L, partial, 0): row i's two buffers agree outside the
                          // run of L elements from j0 (mod D), L = 0: equal, L >= D:
                          // unknown; partial = 1 when winners write only that run and
                          // their own (a copy of partial_wb next to the data it governs)
  const void* o;          // shift, ld values (dtype), zero padded
  const uint64_t* T;      // NEC thresholds, T[k] for k = 0..D+1
  BestState* best;
  int64_t gen_offset;     // run generation = handle generation + gen_offset
  void* hist;             // kHist x N winner fitness (dtype), +inf for losers
  GenMin* mins;           // kHist per-generation minima of this run
  // rotated function
  const double* rot;      // caller's FP64 M, D x D row-major
  const void* w;          // D weights (dtype)
  const void* B[3];       // M pieces, D x ldk (FP64 / FP32 / bf16 hi, mid, lo)
  int64_t ldk;            // pitch of M pieces and of the partial-sum row
  void* part;             // N x ntile partial sums (dtype)
  int32_t ntile, pad1;
  void* stage;            // N x ld staging rows (rotated evaluate)
  void* apc;              // split-bf16 modes: pieces of U - o, P planes of N x ldk bf16
  double* bpart;          // D FP64 terms w_k z_k^2 of the best row's recomputed fitness
  // trace (tests)
  int64_t* tr_idx;
  uint8_t* tr_mask;
  void* tr_trial;
  void* tr_ftrial;
};

// Handle generation number of a launch: `g` itself, or *base + g when the
// launch belongs to a captured graph that is replayed (the graph's last
// kernel advances *base on the device).
struct GenNo {
  uint32_t g;
  uint32_t pad;
  const uint32_t* base;
};
__device__ __forceinline__ uint32_t gen_value(const GenNo& n) {
  return n.base ? *n.base + n.g : n.g;
}

// ---- launch helpers implemented in the kernel translation units ---------
struct GenLaunch {
  const RunDev* runs;     // device array
  const RunDev* host;     // host mirror of the same records
  int32_t run;            // run index for single-run launches
  const uint2* rowmap;    // batched: global row -> (run, row)
  int64_t rows;           // rows in this launch
  int32_t tpr;            // threads per row
  GenNo gnew;             // handle generation being computed
  hipStream_t s;
  bool stream;            // exp / NEC rows streamed instead of held in registers
};

__host__ __device__ inline uint32_t run_gen(const RunDev& P, uint32_t gnew) {
  return static_cast<uint32_t>(static_cast<int64_t>(gnew) + P.gen_offset);
}

hipError_t launch_init_impl(const RunDev* runs, const RunDev& h, int run, double lo, double hi,
                            double olo, double ohi, const void* shift, hipStream_t s);
hipError_t launch_eval_pop(const RunDev* runs, const RunDev& h, int run, hipStream_t s);
hipError_t launch_best_init(const RunDev* runs, int n_runs, hipStream_t s);
// best-so-far over the deferred generations [gfirst, gfirst + count)
hipError_t launch_best_flush(const RunDev* runs, int n_runs, GenNo gfirst, int count,
                             hipStream_t s);
// *base = v, or *base += v (graph bookkeeping)
hipError_t launch_gen_base(uint32_t* base, uint32_t v, bool add, hipStream_t s);
hipError_t launch_generation(const GenLaunch& L, int fn, int xo, int dtype, bool batched);
// exp / NEC rows streamed (single runs; fn separable or Ackley / Griewank)
hipError_t launch_generation_stream(const GenLaunch& L, int fn, int xo, int dtype);
hipError_t launch_pexp_trial(const RunDev* runs, const RunDev& h, int run, GenNo gnew,
                             hipStream_t s);
hipError_t launch_eval_select(const RunDev* runs, const RunDev& h, int run, GenNo gnew,
                              hipStream_t s);
hipError_t launch_eval_rows(const RunDev& h, const void* X, int64_t rows, int64_t ldx, void* out,
                            hipStream_t s);
hipError_t launch_best_fp64(const RunDev* runs, const RunDev& h, int run, uint32_t gcur,
                            double* out, hipStream_t s);
hipError_t launch_normalize(const RunDev* runs, const RunDev& h, int run, uint32_t gcur,
                            hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
// every row's dirty record := (0, L, run's write-back mode, 0)
hipError_t launch_dirty_reset(const RunDev* runs, const RunDev& h, int run, uint32_t L,
                              hipStream_t s);
// crossover masks of generation g (run generation number), N x D bytes
hipError_t launch_masks(const RunDev* runs, const RunDev& h, int run, uint32_t g, uint8_t* out,
                        hipStream_t s);
// record of a workspace-less mask call stored at dst, plus its NEC table at
// rec.T when `table`
hipError_t launch_masks_setup(RunDev* dst, const RunDev& rec, bool table, hipStream_t s);
// rotated function: M pieces and weights from the caller's FP64 M; fitness of
// N rows (the trials of the coming generation when `trials`, else the
// population) into fit_dst or, when select, straight into greedy selection.
hipError_t launch_prepare_rot(const RunDev& h, hipStream_t s);
// split: false when the trial kernel has written the bf16 pieces already
hipError_t launch_rot_fitness(const RunDev* runs, const RunDev& h, int run, GenNo gnew,
                              bool split, hipStream_t s);
hipError_t launch_rot_select(const RunDev* runs, const RunDev& h, int run, GenNo gnew,
                             hipStream_t s);
hipError_t launch_rot_init_fit(const RunDev* runs, const RunDev& h, int run, hipStream_t s);
hipError_t launch_rot_eval_rows(const RunDev* runs, const RunDev& h, int run, const void* X,
                                int64_t rows, void* out, hipStream_t s);

int rot_tile_n();  // column-tile width of the rotated-function product

}  // namespace de
