// C ABI of the library (declared in include/de.h): argument checks, the
// workspace layout, launch sequencing per generation and state transfer.
// No device memory is allocated here: every device byte comes from the
// caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "de.h"
#include "de_internal.h"

using de::RunDev;
using de::BestState;

struct de_handle {
  int n_runs = 0;
  bool batched = false;
  int dtype = 0;
  std::vector<de_run_desc> desc;
  std::vector<RunDev> host;          // mirror of the device records
  RunDev* dev_runs = nullptr;
  BestState* best = nullptr;
  double* scratch_f64 = nullptr;     // one FP64 for de_best
  uint32_t* gbase = nullptr;         // device generation base read by graph replays
  int32_t graph_block = 0;           // generations per captured graph (0: no graphs)
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;
  bool base_valid = false;           // device *gbase equals base_value
  uint32_t base_value = 0;
  uint2* rowmap = nullptr;
  int64_t total_rows = 0;
  std::vector<uint2> rowmap_host;
  std::vector<std::vector<uint64_t>> tables;  // host copies of the NEC tables
  std::vector<int> tpr;
  std::vector<char> stream;          // run uses the streaming exp / NEC kernel
  uint32_t done = 0;                 // generations completed by the handle
  int pending = 0;                   // of which the best-so-far is not yet updated
  std::string err;
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int64_t> ev_launches;  // main-kernel launches between event pairs
  bool single_kernel = false;        // every generation is one kernel launch
};

namespace {

thread_local std::string g_err;

de_status fail(de_handle* h, de_status st, const std::string& msg) {
  if (h) h->err = msg;
  g_err = msg;
  return st;
}

de_status hip_fail(de_handle* h, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(h, DE_E_HIP, m);
}

#define HIPCHECK(h, expr)                                   \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return hip_fail((h), e_, #expr);  \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t up64(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int esz(int dtype) { return dtype == DE_FP64 ? 8 : 4; }
int mm_pieces(int mm) { return mm == DE_MM_BF16X6 ? 3 : (mm == DE_MM_BF16X3 ? 2 : 1); }
int mm_elem(int mm) { return mm == DE_MM_FP64 ? 8 : (mm == DE_MM_FP32 ? 4 : 2); }
int mm_tile_n(int mm) { return mm == DE_MM_FP64 ? 64 : 128; }

// Number of words w with (w + 1/2) 2^-32 < p, i.e. ceil(p 2^32 - 1/2) clamped
// to [0, 2^32]; exact in FP64 for p in [0, 1].
uint64_t threshold(double p) {
  double v = std::ceil(std::ldexp(p, 32) - 0.5);
  if (!(v > 0.0)) return 0;
  if (v >= 4294967296.0) return 4294967296ull;
  return static_cast<uint64_t>(v);
}

struct Layout {
  size_t total = 0;
  size_t runs_off = 0, best_off = 0, scratch_off = 0, rowmap_off = 0;
  struct Run {
    size_t X0, X1, fit, flags, dirty, o, T, hist, mins, w, B[3], part, stage, apc, bp;
    int64_t ld, ldk, ntile;
  };
  std::vector<Run> r;
};

size_t bump(size_t& cur, size_t bytes) {
  size_t at = cur;
  cur = up(cur + bytes, kAlign);
  return at;
}

// Functions evaluated at z = x - o (the others never read a shift).
bool is_shifted(int fn) {
  return fn == DE_FN_RASTRIGIN || fn == DE_FN_ROSENBROCK || fn == DE_FN_ELLIPSOID_ROT;
}

de_status validate(const de_run_desc* runs, int32_t n_runs, std::string& msg) {
  if (!runs || n_runs < 1) { msg = "runs must be a non-empty array"; return DE_E_INVALID; }
  for (int r = 0; r < n_runs; ++r) {
    const de_run_desc& d = runs[r];
    char buf[160];
    auto bad = [&](const char* what) {
      std::snprintf(buf, sizeof buf, "run %d: %s", r, what);
      msg = buf;
      return DE_E_INVALID;
    };
    if (d.N < 4 || d.N >= (1 << 21)) return bad("N must satisfy 4 <= N < 2^21");
    if (d.D < 1 || d.D >= (1 << 21)) return bad("D must satisfy 1 <= D < 2^21");
    if (!(d.CR >= 0.0 && d.CR <= 1.0)) return bad("CR must lie in [0, 1]");
    if (!std::isfinite(d.F) || d.F < 0.0) return bad("F must be finite and >= 0");
    if (!(std::isfinite(d.lo) && std::isfinite(d.hi) && d.lo < d.hi)) return bad("need finite lo < hi");
    if (d.dtype != DE_FP64 && d.dtype != DE_FP32) return bad("unknown dtype");
    if (d.xo < DE_XO_BIN || d.xo > DE_XO_NEC) return bad("unknown crossover");
    if (d.fn < DE_FN_SPHERE || d.fn > DE_FN_GRIEWANK) return bad("unknown function");
    if (d.exp_impl < DE_EXP_LANE || d.exp_impl > DE_EXP_SCAN) return bad("unknown exp_impl");
    if (d.base < DE_BASE_CLASSIC || d.base > DE_BASE_PERM) return bad("unknown base scheme");
    if (d.shuffle != 0 && d.shuffle != 1) return bad("shuffle must be 0 or 1");
    if (d.wb < 0 || d.wb > 2) return bad("wb must be 0, 1 or 2");
    if (d.tile < 0 || d.tile > 3) return bad("tile must be 0, 1, 2 or 3");
    if (d.tile != 0 && !(d.fn == DE_FN_ELLIPSOID_ROT && (d.mm == DE_MM_BF16X3 || d.mm == DE_MM_BF16X6)))
      return bad("tile applies to the split-bf16 rotated product only");
    if (d.tpr != 0 && d.tpr != 64 && d.tpr != 128 && d.tpr != 256 && d.tpr != 512 && d.tpr != 1024)
      return bad("tpr must be 0, 64, 128, 256, 512 or 1024");
    if (n_runs > 1 && d.tpr != 0 && d.tpr != 64 && d.tpr != 128 && d.tpr != 256)
      return bad("batched runs use tpr 0, 64, 128 or 256");
    if (n_runs > 1 && d.tpr != runs[0].tpr) return bad("the runs of a batch share one tpr");
    if (is_shifted(d.fn) && !d.shift &&
        !(std::isfinite(d.olo) && std::isfinite(d.ohi) && d.olo <= d.ohi))
      return bad("need finite olo <= ohi when shift is NULL");
    if (d.fn == DE_FN_ELLIPSOID_ROT) {
      if (d.D < 2) return bad("the rotated function needs D >= 2");
      if (!d.rot) return bad("the rotated function needs rot");
      if (d.mm < DE_MM_FP64 || d.mm > DE_MM_BF16X6) return bad("unknown matmul mode");
      const bool ok = (d.dtype == DE_FP64 && d.mm == DE_MM_FP64) ||
                      (d.dtype == DE_FP32 && d.mm != DE_MM_FP64);
      if (!ok) {
        std::snprintf(buf, sizeof buf, "run %d: matmul mode %d does not go with dtype %d", r,
                      d.mm, d.dtype);
        msg = buf;
        return DE_E_UNSUPPORTED;
      }
    }
    if (n_runs > 1) {
      if (d.fn == DE_FN_ELLIPSOID_ROT || d.fn == DE_FN_ACKLEY || d.fn == DE_FN_GRIEWANK ||
          (d.xo == DE_XO_EXP && d.exp_impl == DE_EXP_JOB)) {
        std::snprintf(buf, sizeof buf,
                      "run %d: batched launches support sphere, Rastrigin and Rosenbrock and the "
                      "lane/scan exponential crossover only", r);
        msg = buf;
        return DE_E_UNSUPPORTED;
      }
      if (d.dtype != runs[0].dtype) {
        msg = "all runs of a batch must share one dtype";
        return DE_E_UNSUPPORTED;
      }
    }
  }
  return DE_OK;
}

Layout layout(const de_run_desc* runs, int32_t n_runs) {
  Layout L;
  size_t cur = 0;
  L.runs_off = bump(cur, sizeof(RunDev) * n_runs);
  L.best_off = bump(cur, sizeof(BestState) * n_runs);
  L.scratch_off = bump(cur, 64);
  int64_t total_rows = 0;
  for (int r = 0; r < n_runs; ++r) total_rows += runs[r].N;
  L.rowmap_off = bump(cur, n_runs > 1 ? sizeof(uint2) * total_rows : 0);
  L.r.resize(n_runs);
  for (int r = 0; r < n_runs; ++r) {
    const de_run_desc& d = runs[r];
    Layout::Run& q = L.r[r];
    const size_t s = esz(d.dtype);
    q.ld = up64(d.D, 32);
    const size_t pop = s * d.N * q.ld;
    q.X0 = bump(cur, pop);
    q.X1 = bump(cur, pop);
    q.fit = bump(cur, s * d.N);
    q.flags = bump(cur, 2 * d.N);
    q.dirty = bump(cur, sizeof(uint4) * d.N);
    q.o = bump(cur, s * q.ld);
    q.T = bump(cur, 8 * (d.D + 2));
    q.hist = bump(cur, s * d.N * de::kHist);
    q.mins = bump(cur, sizeof(de::GenMin) * de::kHist);
    q.ldk = 0;
    q.ntile = 0;
    q.w = q.part = q.stage = q.apc = q.bp = 0;
    q.B[0] = q.B[1] = q.B[2] = 0;
    if (d.fn == DE_FN_ELLIPSOID_ROT) {
      q.ldk = up64(d.D, 32);
      q.ntile = (d.D + mm_tile_n(d.mm) - 1) / mm_tile_n(d.mm);
      const int64_t rows_pad = up64(d.D, 256);  // M rows: whole tiles of the widest product
      q.w = bump(cur, s * d.D);
      for (int p = 0; p < mm_pieces(d.mm); ++p)
        q.B[p] = bump(cur, static_cast<size_t>(mm_elem(d.mm)) * rows_pad * q.ldk);
      q.part = bump(cur, s * d.N * q.ntile);
      q.stage = bump(cur, pop);
      q.bp = bump(cur, sizeof(double) * d.D);
      if (d.mm == DE_MM_BF16X3 || d.mm == DE_MM_BF16X6)
        q.apc = bump(cur, static_cast<size_t>(2) * mm_pieces(d.mm) * d.N * q.ldk);
    }
  }
  L.total = cur;
  return L;
}

int pick_tpr(const de_run_desc& d, bool batched) {
  if (batched) return d.tpr == 0 ? 64 : d.tpr;
  if (d.tpr != 0) return d.tpr;
  // Measured defaults (MI355X): a row held in registers by as few lanes as
  // fit; rows of up to 1024 elements take 128 lanes (2 chunks each) where the
  // shorter per-lane chain pays for the second wavefront: FP64 runs of the
  // ALU-heavy functions (Rastrigin NEC 8.5 vs 9.0 us at N = 2048) and
  // binomial runs (11.4 vs 12.2 us); FP32 exp/NEC (6.4 vs 6.7 us) and the
  // sphere (6.6 vs 7.1 us) stay at 64 ...
  const int64_t nchunk = (d.D + 3) / 4;
  int t = nchunk <= 64 * 4 ? 64 : nchunk <= 256 * 4 ? 256 : nchunk <= 512 * 5 ? 512 : 1024;
  const bool alu_heavy = d.dtype == DE_FP64 && d.fn != DE_FN_SPHERE;
  if (t == 64 && nchunk > 64 && (alu_heavy || d.xo == DE_XO_BIN)) t = 128;
  // ... widened while the run has fewer wavefronts than half the chip's SIMDs
  // (256 CUs x 4) and every lane still has more than one chunk: small
  // populations then finish each row in fewer dependent steps (Ackley
  // D = 1000 N = 500: 5.8 us at 128 lanes, 6.1 at 256, 8.4 at 64).
  while (t < 1024 && nchunk > t && d.N * (t / 64) < 512) t = t == 64 ? 128 : 2 * t;
  return t;
}

hipError_t upload_run(de_handle* h, int r, hipStream_t s) {
  return hipMemcpyAsync(h->dev_runs + r, &h->host[r], sizeof(RunDev), hipMemcpyHostToDevice, s);
}

hipEvent_t next_event(de_handle* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

void add_pair_count(de_handle* h, int64_t n) {
  if (h->ev_used % 2 == 0 && h->ev_used >= 2) h->ev_launches.push_back(n);
}

// Best-so-far over the generations run since the last update.
de_status flush_best(de_handle* h, hipStream_t s) {
  if (h->pending == 0) return DE_OK;
  const uint32_t gfirst = h->done - static_cast<uint32_t>(h->pending) + 1;
  HIPCHECK(h, de::launch_best_flush(h->dev_runs, h->n_runs, de::GenNo{gfirst, 0, nullptr},
                                    h->pending, s));
  h->pending = 0;
  return DE_OK;
}

// The launches of one generation of one run (single-run handles) or of all
// runs (batched); `mark` brackets the dominant kernel with events if enabled.
de_status generation_launches(de_handle* h, hipStream_t s, de::GenNo gnew) {
  // per-launch event pairs only where a generation has several kernels; a
  // one-kernel generation is timed as a span of launches in de_generation
  auto mark = [&]() {
    if (!h->prof || h->single_kernel) return;
    hipEvent_t e = next_event(h);
    if (e) (void)hipEventRecord(e, s);
    add_pair_count(h, 1);
  };
  if (h->batched) {
    de::GenLaunch L{h->dev_runs, h->host.data(), 0, h->rowmap, h->total_rows, h->tpr[0], gnew, s,
                    false};
    mark();
    HIPCHECK(h, de::launch_generation(L, de::FN_ANY, de::XO_ANY, h->dtype, true));
    mark();
  } else {
    for (int r = 0; r < h->n_runs; ++r) {
      const de_run_desc& d = h->desc[r];
      const RunDev& H = h->host[r];
      const bool job = d.xo == DE_XO_EXP && d.exp_impl == DE_EXP_JOB;
      if (d.fn == DE_FN_ELLIPSOID_ROT) {
        if (job) {
          HIPCHECK(h, de::launch_pexp_trial(h->dev_runs, H, r, gnew, s));
        } else {
          de::GenLaunch L{h->dev_runs, h->host.data(), r, nullptr, d.N, h->tpr[r], gnew, s, false};
          HIPCHECK(h, de::launch_generation(L, de::FN_NONE, d.xo, d.dtype, false));
        }
        mark();
        // the fused trial kernel writes the bf16 pieces; the p-exp one does not
        HIPCHECK(h, de::launch_rot_fitness(h->dev_runs, H, r, gnew, job, s));
        mark();
        HIPCHECK(h, de::launch_rot_select(h->dev_runs, H, r, gnew, s));
      } else if (job) {
        mark();
        HIPCHECK(h, de::launch_pexp_trial(h->dev_runs, H, r, gnew, s));
        mark();
        HIPCHECK(h, de::launch_eval_select(h->dev_runs, H, r, gnew, s));
      } else {
        de::GenLaunch L{h->dev_runs, h->host.data(), r, nullptr, d.N, h->tpr[r], gnew, s,
                        h->stream[r] != 0};
        mark();
        if (L.stream) HIPCHECK(h, de::launch_generation_stream(L, d.fn, d.xo, d.dtype));
        else HIPCHECK(h, de::launch_generation(L, d.fn, d.xo, d.dtype, false));
        mark();
      }
    }
  }
  return DE_OK;
}

de_status one_generation(de_handle* h, hipStream_t s) {
  const uint32_t gnew = h->done + 1;
  de_status st = generation_launches(h, s, de::GenNo{gnew, 0, nullptr});
  if (st != DE_OK) return st;
  h->done = gnew;
  if (++h->pending == de::kHist) return flush_best(h, s);
  return DE_OK;
}

// Captures B = graph_block generations, the best-so-far update after every
// kHist of them and after the last, and the advance of the device generation
// base into one graph (on a private stream; the graph is then launched on the
// caller's stream).  Generation numbers inside are *gbase + 1 .. *gbase + B.
de_status capture_block(de_handle* h) {
  if (!h->cap_stream) HIPCHECK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = h->cap_stream;
  const int B = h->graph_block;
  HIPCHECK(h, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  de_status st = DE_OK;
  hipError_t e = hipSuccess;
  for (int k = 1; k <= B && st == DE_OK && e == hipSuccess; ++k) {
    st = generation_launches(h, cs, de::GenNo{static_cast<uint32_t>(k), 0, h->gbase});
    if (st == DE_OK && (k % de::kHist == 0 || k == B)) {
      const int cnt = k % de::kHist == 0 ? de::kHist : k % de::kHist;
      e = de::launch_best_flush(h->dev_runs, h->n_runs,
                                de::GenNo{static_cast<uint32_t>(k - cnt + 1), 0, h->gbase}, cnt, cs);
    }
  }
  if (st == DE_OK && e == hipSuccess)
    e = de::launch_gen_base(h->gbase, static_cast<uint32_t>(B), true, cs);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(cs, &g);
  if (st != DE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(h, e, "launch during graph capture");
  }
  if (e2 != hipSuccess) return hip_fail(h, e2, "hipStreamEndCapture");
  e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->gexec = nullptr;
    return hip_fail(h, e, "hipGraphInstantiate");
  }
  return DE_OK;
}

// ---- allocation-free mask calls ------------------------------------------
// de_masks_noalloc keeps the run record and the NEC threshold table of its
// call in this array instead of a workspace.  Each GPU holds its own copy
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy: it uses the device address hipGetSymbolAddress returns
// for the current device, looked up once per device and kept.
constexpr size_t kNoAllocBytes = size_t(1) << 20;
constexpr size_t kNoAllocTableOff = 512;  // run record first, table after it
static_assert(sizeof(RunDev) <= kNoAllocTableOff, "run record fits before the table");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // per device id; null until looked up

hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (static_cast<int>(g_scratch_dev.size()) <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

de_status check_run(de_handle* h, int32_t run) {
  if (!h) return fail(nullptr, DE_E_INVALID, "NULL handle");
  if (run < 0 || run >= h->n_runs) return fail(h, DE_E_INVALID, "run index out of range");
  return DE_OK;
}

}  // namespace

extern "C" {

de_status de_workspace_size(const de_run_desc* runs, int32_t n_runs, size_t* bytes) {
  std::string msg;
  de_status st = validate(runs, n_runs, msg);
  if (st != DE_OK) return fail(nullptr, st, msg);
  if (!bytes) return fail(nullptr, DE_E_INVALID, "bytes is NULL");
  *bytes = layout(runs, n_runs).total;
  return DE_OK;
}

de_status de_init(de_handle** out, const de_run_desc* runs, int32_t n_runs, void* workspace,
                  size_t ws_bytes, void* stream) {
  if (!out) return fail(nullptr, DE_E_INVALID, "h is NULL");
  *out = nullptr;
  std::string msg;
  de_status st = validate(runs, n_runs, msg);
  if (st != DE_OK) return fail(nullptr, st, msg);
  const Layout L = layout(runs, n_runs);
  if (!workspace) return fail(nullptr, DE_E_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(nullptr, DE_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(nullptr, DE_E_WORKSPACE, "workspace too small");

  de_handle* h = new de_handle();
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  h->n_runs = n_runs;
  h->batched = n_runs > 1;
  h->dtype = runs[0].dtype;
  h->desc.assign(runs, runs + n_runs);
  h->dev_runs = reinterpret_cast<RunDev*>(ws + L.runs_off);
  h->best = reinterpret_cast<BestState*>(ws + L.best_off);
  h->scratch_f64 = reinterpret_cast<double*>(ws + L.scratch_off);
  h->gbase = reinterpret_cast<uint32_t*>(ws + L.scratch_off + 16);
  h->rowmap = h->batched ? reinterpret_cast<uint2*>(ws + L.rowmap_off) : nullptr;
  h->host.resize(n_runs);
  h->tables.resize(n_runs);
  h->tpr.resize(n_runs);
  for (int r = 0; r < n_runs; ++r) {
    const de_run_desc& d = runs[r];
    const Layout::Run& q = L.r[r];
    RunDev& R = h->host[r];
    std::memset(&R, 0, sizeof R);
    R.N = d.N; R.D = d.D; R.ld = q.ld;
    R.F = d.F; R.CR = d.CR; R.Ff = static_cast<float>(d.F);
    R.inv_ln_cr = (d.CR > 0.0 && d.CR < 1.0) ? 1.0 / std::log(d.CR) : 0.0;
    R.thr = threshold(d.CR);
    R.key0 = static_cast<uint32_t>(d.seed);
    R.key1 = static_cast<uint32_t>(d.seed >> 32);
    R.run_id = static_cast<uint32_t>(r);
    R.fn = d.fn; R.xo = d.xo; R.exp_impl = d.exp_impl; R.dtype = d.dtype; R.mm = d.mm;
    R.base = d.base; R.shuffle = d.shuffle; R.tile = d.tile;
    R.X[0] = ws + q.X0;
    R.X[1] = ws + q.X1;
    R.fit = ws + q.fit;
    R.flags = reinterpret_cast<uint8_t*>(ws + q.flags);
    R.dirty = reinterpret_cast<uint4*>(ws + q.dirty);
    R.o = ws + q.o;
    R.T = reinterpret_cast<const uint64_t*>(ws + q.T);
    R.best = h->best + r;
    R.gen_offset = 0;
    R.hist = ws + q.hist;
    R.mins = reinterpret_cast<de::GenMin*>(ws + q.mins);
    if (d.fn == DE_FN_ELLIPSOID_ROT) {
      R.rot = d.rot;
      R.w = ws + q.w;
      for (int p = 0; p < mm_pieces(d.mm); ++p) R.B[p] = ws + q.B[p];
      R.ldk = q.ldk;
      R.part = ws + q.part;
      R.ntile = static_cast<int32_t>(q.ntile);
      R.stage = ws + q.stage;
      R.apc = q.apc ? ws + q.apc : nullptr;
      R.bpart = reinterpret_cast<double*>(ws + q.bp);
    }
    // NEC thresholds: T[k] = #words below CR^(k-1), the power taken as a
    // running FP64 product; T[D+1] = 0 ends the search.
    std::vector<uint64_t>& T = h->tables[r];
    T.assign(d.D + 2, 0);
    T[0] = 4294967296ull;
    double t = 1.0;
    for (int64_t k = 1; k <= d.D; ++k) {
      if (k > 1) t = t * d.CR;
      T[k] = threshold(t);
    }
    T[d.D + 1] = 0;
    h->tpr[r] = pick_tpr(d, h->batched);
  }
  // Partial write-back pays once one population buffer of the handle outgrows
  // the caches (measured crossover on MI355X: 30-80 MB; below, whole rows).
  size_t pop_bytes = 0;
  for (int r = 0; r < n_runs; ++r)
    pop_bytes += static_cast<size_t>(esz(runs[r].dtype)) * runs[r].N * L.r[r].ld;
  // Rotated runs always: their generation is dominated by the product, and
  // the trial kernel's smaller stores measured faster at every size tried.
  for (int r = 0; r < n_runs; ++r)
    h->host[r].partial_wb = runs[r].wb == 2 ||
                            (runs[r].wb == 0 && (pop_bytes > (size_t(48) << 20) ||
                                                 runs[r].fn == DE_FN_ELLIPSOID_ROT));
  // Exp and NEC rows longer than 4096 elements (rows the register-cached
  // kernel would need 512 or more lanes for) are streamed: the trial differs
  // from the parent only in its run, so no copy of the row is kept.  The
  // choice depends on the run's shape only, never on the write-back mode.
  // 256 lanes per row unless the descriptor asks for another width (measured
  // on MI355X, D = 10^4 N = 8192 FP32 NEC, two chunks per lane in flight:
  // 64 lanes 74.7 us, 128 75.7, 256 73.3 per generation).
  h->stream.assign(n_runs, 0);
  for (int r = 0; r < n_runs; ++r) {
    const de_run_desc& d = runs[r];
    const bool runs_xo = d.xo == DE_XO_NEC || (d.xo == DE_XO_EXP && d.exp_impl != DE_EXP_JOB);
    if (!h->batched && runs_xo && d.fn != DE_FN_ELLIPSOID_ROT && d.D > 4096) {
      h->stream[r] = 1;
      h->tpr[r] = d.tpr == 0 ? 256 : d.tpr;
    }
  }
  h->single_kernel = true;
  for (int r = 0; r < n_runs; ++r)
    if (runs[r].fn == DE_FN_ELLIPSOID_ROT || (runs[r].xo == DE_XO_EXP && runs[r].exp_impl == DE_EXP_JOB))
      h->single_kernel = false;
  if (h->batched) {
    for (int r = 0; r < n_runs; ++r)
      for (int64_t i = 0; i < runs[r].N; ++i)
        h->rowmap_host.push_back(make_uint2(static_cast<unsigned>(r), static_cast<unsigned>(i)));
    h->total_rows = static_cast<int64_t>(h->rowmap_host.size());
  }

  auto bail = [&](de_status st2) {
    g_err = h->err;
    delete h;
    return st2;
  };
#define HIPINIT(expr)                                          \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return bail(hip_fail(h, e_, #expr)); \
  } while (0)

  HIPINIT(hipMemcpyAsync(h->dev_runs, h->host.data(), sizeof(RunDev) * n_runs,
                         hipMemcpyHostToDevice, s));
  if (h->batched)
    HIPINIT(hipMemcpyAsync(h->rowmap, h->rowmap_host.data(), sizeof(uint2) * h->total_rows,
                           hipMemcpyHostToDevice, s));
  for (int r = 0; r < n_runs; ++r) {
    const de_run_desc& d = runs[r];
    const RunDev& R = h->host[r];
    HIPINIT(hipMemcpyAsync(const_cast<uint64_t*>(R.T), h->tables[r].data(),
                           sizeof(uint64_t) * (d.D + 2), hipMemcpyHostToDevice, s));
    HIPINIT(de::launch_init_impl(h->dev_runs, R, r, d.lo, d.hi, d.olo, d.ohi,
                                 is_shifted(d.fn) ? d.shift : nullptr, s));
    if (d.fn == DE_FN_ELLIPSOID_ROT) {
      HIPINIT(de::launch_prepare_rot(R, s));
      HIPINIT(de::launch_rot_init_fit(h->dev_runs, R, r, s));
    } else {
      HIPINIT(de::launch_eval_pop(h->dev_runs, R, r, s));
    }
  }
  HIPINIT(de::launch_best_init(h->dev_runs, n_runs, s));
  // host tables must outlive the asynchronous copies
  HIPINIT(hipStreamSynchronize(s));
#undef HIPINIT
  *out = h;
  return DE_OK;
}

de_status de_generation(de_handle* h, int32_t n_gens, void* stream) {
  if (!h) return fail(nullptr, DE_E_INVALID, "NULL handle");
  if (n_gens < 0) return fail(h, DE_E_INVALID, "n_gens must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (static_cast<uint64_t>(h->done) + static_cast<uint64_t>(n_gens) >= 0xFFFFFFF0ull)
    return fail(h, DE_E_STATE, "generation counter would overflow");
  const bool span = h->prof && h->single_kernel && n_gens > 0;
  if (span) {
    hipEvent_t e = next_event(h);
    if (e) (void)hipEventRecord(e, s);
  }
  int32_t left = n_gens;
  const int32_t B = h->graph_block;
  if (B > 0 && !h->prof && left >= B) {
    // a captured block starts on a flushed best-so-far (every call ends with
    // one, so this runs no generation unless a caller mixes in others)
    while (left > 0 && h->pending != 0) {
      de_status st = one_generation(h, s);
      if (st != DE_OK) return st;
      --left;
    }
    while (left >= B) {
      if (!h->gexec) {
        de_status st = capture_block(h);
        if (st != DE_OK) return st;
      }
      if (!h->base_valid || h->base_value != h->done) {
        HIPCHECK(h, de::launch_gen_base(h->gbase, h->done, false, s));
        h->base_valid = true;
      }
      HIPCHECK(h, hipGraphLaunch(h->gexec, s));
      h->done += static_cast<uint32_t>(B);
      h->base_value = h->done;
      left -= B;
    }
  }
  for (int32_t k = 0; k < left; ++k) {
    de_status st = one_generation(h, s);
    if (st != DE_OK) return st;
  }
  if (span) {
    hipEvent_t e = next_event(h);
    if (e) (void)hipEventRecord(e, s);
    add_pair_count(h, n_gens);
  }
  return flush_best(h, s);
}

de_status de_evaluate(de_handle* h, int32_t run, const void* X, int64_t rows, void* fit_out,
                      void* stream) {
  de_status st = check_run(h, run);
  if (st != DE_OK) return st;
  if (rows < 0) return fail(h, DE_E_INVALID, "rows must be >= 0");
  if (rows > 0 && (!X || !fit_out)) return fail(h, DE_E_INVALID, "X and fit_out are required");
  if (rows == 0) return DE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const RunDev& R = h->host[run];
  if (R.fn == DE_FN_ELLIPSOID_ROT) {
    HIPCHECK(h, de::launch_rot_eval_rows(h->dev_runs, R, run, X, rows, fit_out, s));
  } else {
    HIPCHECK(h, de::launch_eval_rows(R, X, rows, R.D, fit_out, s));
  }
  return DE_OK;
}

de_status de_best(de_handle* h, int32_t run, double* f_best, int64_t* idx, int64_t* gen,
                  void* x_best_host, void* stream) {
  de_status st = check_run(h, run);
  if (st != DE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const RunDev& R = h->host[run];
  st = flush_best(h, s);
  if (st != DE_OK) return st;
  HIPCHECK(h, de::launch_best_fp64(h->dev_runs, R, run, h->done, h->scratch_f64, s));
  BestState B;
  double f = 0.0;
  HIPCHECK(h, hipMemcpyAsync(&B, h->best + run, sizeof B, hipMemcpyDeviceToHost, s));
  HIPCHECK(h, hipMemcpyAsync(&f, h->scratch_f64, sizeof f, hipMemcpyDeviceToHost, s));
  HIPCHECK(h, hipStreamSynchronize(s));
  if (f_best) *f_best = f;
  if (idx) *idx = B.idx;
  if (gen) *gen = B.gen;
  if (x_best_host) {
    uint8_t flag = 0;
    HIPCHECK(h, hipMemcpyAsync(&flag, R.flags + (B.g & 1u) * R.N + B.idx, 1,
                               hipMemcpyDeviceToHost, s));
    HIPCHECK(h, hipStreamSynchronize(s));
    const size_t e = esz(R.dtype);
    const char* src = static_cast<const char*>(R.X[flag ? 1 : 0]) + e * B.idx * R.ld;
    HIPCHECK(h, hipMemcpyAsync(x_best_host, src, e * R.D, hipMemcpyDeviceToHost, s));
    HIPCHECK(h, hipStreamSynchronize(s));
  }
  return DE_OK;
}

de_status de_get_state(de_handle* h, int32_t run, void* pop_host, void* fit_host, int64_t* gen,
                       void* stream) {
  de_status st = check_run(h, run);
  if (st != DE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const RunDev& R = h->host[run];
  const size_t e = esz(R.dtype);
  st = flush_best(h, s);
  if (st != DE_OK) return st;
  if (pop_host) {
    HIPCHECK(h, de::launch_normalize(h->dev_runs, R, run, h->done, s));
    HIPCHECK(h, hipMemcpy2DAsync(pop_host, e * R.D, R.X[0], e * R.ld, e * R.D, R.N,
                                 hipMemcpyDeviceToHost, s));
  }
  if (fit_host) HIPCHECK(h, hipMemcpyAsync(fit_host, R.fit, e * R.N, hipMemcpyDeviceToHost, s));
  BestState B;
  HIPCHECK(h, hipMemcpyAsync(&B, h->best + run, sizeof B, hipMemcpyDeviceToHost, s));
  HIPCHECK(h, hipStreamSynchronize(s));
  if (gen) *gen = static_cast<int64_t>(h->done) + R.gen_offset;
  return DE_OK;
}

de_status de_set_state(de_handle* h, int32_t run, const void* pop_host, const void* fit_host,
                       int64_t gen, double best_f, int64_t best_idx, int64_t best_gen,
                       void* stream) {
  de_status st = check_run(h, run);
  if (st != DE_OK) return st;
  if (!pop_host || !fit_host) return fail(h, DE_E_INVALID, "pop_host and fit_host are required");
  if (gen < 0 || gen >= 0xFFFFFFFFll) return fail(h, DE_E_INVALID, "gen out of range");
  hipStream_t s = static_cast<hipStream_t>(stream);
  RunDev& R = h->host[run];
  if (best_idx >= R.N) return fail(h, DE_E_INVALID, "best_idx out of range");
  st = flush_best(h, s);
  if (st != DE_OK) return st;
  R.gen_offset = gen - static_cast<int64_t>(h->done);
  const size_t e = esz(R.dtype);
  BestState B{};
  B.g = static_cast<uint32_t>(gen);
  if (best_idx >= 0) {
    B.f = best_f;
    B.idx = best_idx;
    B.gen = best_gen;
  } else {
    int64_t m = 0;
    double fm = 0.0;
    for (int64_t i = 0; i < R.N; ++i) {
      double v = R.dtype == DE_FP64 ? static_cast<const double*>(fit_host)[i]
                                    : static_cast<double>(static_cast<const float*>(fit_host)[i]);
      if (v != v) v = INFINITY;
      if (i == 0 || v < fm) { fm = v; m = i; }
    }
    B.f = fm;
    B.idx = m;
    B.gen = gen;
  }
  HIPCHECK(h, hipMemcpy2DAsync(R.X[0], e * R.ld, pop_host, e * R.D, e * R.D, R.N,
                               hipMemcpyHostToDevice, s));
  HIPCHECK(h, hipMemcpyAsync(R.fit, fit_host, e * R.N, hipMemcpyHostToDevice, s));
  HIPCHECK(h, de::launch_fill_u8(R.flags, 2 * R.N, 0, s));
  // buffer 1 no longer matches buffer 0 anywhere in particular
  HIPCHECK(h, de::launch_dirty_reset(h->dev_runs, R, run, de::kDirtyAll, s));
  HIPCHECK(h, hipMemcpyAsync(h->best + run, &B, sizeof B, hipMemcpyHostToDevice, s));
  HIPCHECK(h, upload_run(h, run, s));
  HIPCHECK(h, hipStreamSynchronize(s));
  return DE_OK;
}

de_status de_masks(de_handle* h, int32_t run, int64_t gen, uint8_t* mask, void* stream) {
  de_status st = check_run(h, run);
  if (st != DE_OK) return st;
  if (gen < 1 || gen >= 0xFFFFFFFFll) return fail(h, DE_E_INVALID, "gen must be in [1, 2^32 - 1)");
  if (!mask) return fail(h, DE_E_INVALID, "mask is NULL");
  HIPCHECK(h, de::launch_masks(h->dev_runs, h->host[run], run, static_cast<uint32_t>(gen), mask,
                               static_cast<hipStream_t>(stream)));
  return DE_OK;
}

de_status de_masks_noalloc(const de_run_desc* run, int32_t run_index, int64_t gen, uint8_t* mask,
                           void* stream) {
  if (!run) return fail(nullptr, DE_E_INVALID, "run is NULL");
  const de_run_desc& d = *run;
  if (d.N < 4 || d.N >= (1 << 21)) return fail(nullptr, DE_E_INVALID, "N must satisfy 4 <= N < 2^21");
  if (d.D < 1 || d.D > DE_MASKS_NOALLOC_MAX_D)
    return fail(nullptr, DE_E_INVALID,
                "D must satisfy 1 <= D <= DE_MASKS_NOALLOC_MAX_D (the threshold table of the "
                "call must fit in the library's static scratch)");
  if (!(d.CR >= 0.0 && d.CR <= 1.0)) return fail(nullptr, DE_E_INVALID, "CR must lie in [0, 1]");
  if (d.xo < DE_XO_BIN || d.xo > DE_XO_NEC) return fail(nullptr, DE_E_INVALID, "unknown crossover");
  if (d.exp_impl < DE_EXP_LANE || d.exp_impl > DE_EXP_SCAN)
    return fail(nullptr, DE_E_INVALID, "unknown exp_impl");
  if (run_index < 0 || run_index >= (1 << 24))
    return fail(nullptr, DE_E_INVALID, "run_index must lie in [0, 2^24)");
  if (gen < 1 || gen >= 0xFFFFFFFFll) return fail(nullptr, DE_E_INVALID, "gen must be in [1, 2^32 - 1)");
  if (!mask) return fail(nullptr, DE_E_INVALID, "mask is NULL");
  static_assert(kNoAllocTableOff + 8 * (DE_MASKS_NOALLOC_MAX_D + 2) <= kNoAllocBytes,
                "largest table fits in the scratch");
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
  // the run record a handle would hold for this run, reduced to what the
  // mask kernels read
  RunDev R;
  std::memset(&R, 0, sizeof R);
  R.N = d.N; R.D = d.D; R.ld = up64(d.D, 32);
  R.CR = d.CR; R.F = d.F; R.Ff = static_cast<float>(d.F);
  R.inv_ln_cr = (d.CR > 0.0 && d.CR < 1.0) ? 1.0 / std::log(d.CR) : 0.0;
  R.thr = threshold(d.CR);
  R.key0 = static_cast<uint32_t>(d.seed);
  R.key1 = static_cast<uint32_t>(d.seed >> 32);
  R.run_id = static_cast<uint32_t>(run_index);
  R.fn = d.fn; R.xo = d.xo; R.exp_impl = d.exp_impl; R.dtype = d.dtype;
  R.T = reinterpret_cast<const uint64_t*>(static_cast<char*>(base) + kNoAllocTableOff);
  RunDev* rec = static_cast<RunDev*>(base);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the table is read only by NEC with 0 < CR < 1 (the other cases need no table)
  const bool table = d.xo == DE_XO_NEC && R.inv_ln_cr != 0.0;
  e = de::launch_masks_setup(rec, R, table, s);
  if (e != hipSuccess) return hip_fail(nullptr, e, "mask set-up launch");
  e = de::launch_masks(rec, R, 0, static_cast<uint32_t>(gen), mask, s);
  if (e != hipSuccess) return hip_fail(nullptr, e, "mask launch");
  return DE_OK;
}

de_status de_trace(de_handle* h, int32_t run, int64_t* idx, uint8_t* mask, void* trial,
                   void* ftrial) {
  de_status st = check_run(h, run);
  if (st != DE_OK) return st;
  HIPCHECK(h, hipDeviceSynchronize());
  RunDev& R = h->host[run];
  R.tr_idx = idx;
  R.tr_mask = mask;
  R.tr_trial = trial;
  R.tr_ftrial = ftrial;
  HIPCHECK(h, hipMemcpy(h->dev_runs + run, &R, sizeof R, hipMemcpyHostToDevice));
  return DE_OK;
}

de_status de_profile(de_handle* h, int32_t enable) {
  if (!h) return fail(nullptr, DE_E_INVALID, "NULL handle");
  h->prof = enable != 0;
  h->ev_used = 0;
  h->ev_launches.clear();
  return DE_OK;
}

de_status de_profile_read(de_handle* h, double* main_ms, int64_t* main_launches) {
  if (!h) return fail(nullptr, DE_E_INVALID, "NULL handle");
  double total = 0.0;
  int64_t n = 0;
  for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
    HIPCHECK(h, hipEventSynchronize(h->ev_pool[k + 1]));
    float ms = 0.0f;
    HIPCHECK(h, hipEventElapsedTime(&ms, h->ev_pool[k], h->ev_pool[k + 1]));
    total += ms;
    n += k / 2 < h->ev_launches.size() ? h->ev_launches[k / 2] : 1;
  }
  if (main_ms) *main_ms = total;
  if (main_launches) *main_launches = n;
  return DE_OK;
}

const char* de_last_error(const de_handle* h) {
  if (h) return h->err.c_str();
  return g_err.c_str();
}

de_status de_graph(de_handle* h, int32_t enable) {
  if (!h) return fail(nullptr, DE_E_INVALID, "NULL handle");
  if (enable < 0) return fail(h, DE_E_INVALID, "enable must be >= 0");
  const int32_t B = enable == 1 ? de::kHist : enable;
  if (B != h->graph_block && h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);  // captured for another block length
    h->gexec = nullptr;
  }
  h->graph_block = B;
  if (B > 0 && !h->gexec) {
    // capture and upload now, so that the first block replayed costs what
    // every later one does (the captured kernels take their generation
    // numbers from the device base, so the graph depends on no state here)
    de_status st = capture_block(h);
    if (st != DE_OK) return st;
    HIPCHECK(h, hipGraphUpload(h->gexec, h->cap_stream));
    HIPCHECK(h, hipStreamSynchronize(h->cap_stream));
  }
  return DE_OK;
}

void de_destroy(de_handle* h) {
  if (!h) return;
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
}

}  // extern "C"
