// Rotated ellipsoid fitness f_i = sum_k w_k z_ik^2 with z_i = M (u_i - o):
// the one dense contraction of the path, Z = (U - 1 o^T) M^T, an N x D x D
// product with both operands contiguous along the contraction index.
//
// One kernel does the product on the matrix cores with the weighted square
// sum fused into the epilogue, so Z is never stored: each block writes one
// partial sum per row for its 128 output columns.  A second kernel adds the
// partials of a row in a fixed order and performs greedy selection.
//
// Modes: FP64 (v_mfma_f64_16x16x4) and FP32 (v_mfma_f32_16x16x4), with the
// shift subtracted in the A-tile load; and splits of both operands into 2 or
// 3 bf16 pieces whose 3 or 6 leading cross products are accumulated in FP32
// (v_mfma_f32_16x16x32_bf16 / v_mfma_f32_32x32x16_bf16).  The bf16 pieces of
// U - o are written by the trial kernel (or a split pass for rows no trial
// kernel wrote), those of M once at set-up.
//
// Lane layouts (checked on gfx950 with integer-valued operands): in the 16x16
// forms lane l supplies A[l%16][(l/16)*KPL + e] and B[(l/16)*KPL + e][l%16]
// (KPL = 8 for bf16, 1 for f32/f64); accumulator register r of lane l holds
// C[(l/16)*4 + r][l%16] for the f32/bf16 forms and C[4r + l/16][l%16] for the
// f64 form.  In the 32x32x16 form lane l supplies A[l%32][(l/32)*8 + e] and
// B[(l/32)*8 + e][l%32], and register r holds C[8(r/4) + 4(l/32) + r%4][l%32].
#include <type_traits>
#include <utility>

#include "de_device.h"

namespace de {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) double f64x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;


template <int MODE> struct MM;
template <> struct MM<MM_FP64> {
  using T = double; using L = double; static constexpr int P = 1, KT = 16, BM = 64, BN = 64, PAD = 1, NW = 8;
};
template <> struct MM<MM_FP32> {
  using T = float; using L = float; static constexpr int P = 1, KT = 32, BM = 128, BN = 128, PAD = 2, NW = 4;
};

int rot_tile_n() { return 128; }  // BN of the FP32 and bf16 modes; FP64 uses 64

// Row source for the A operand.
//   src 0: trials of the coming generation (non-current buffer of each row)
//   src 1: current population
//   src 2: staging rows (caller data for de_evaluate)
//   gh: handle generation (the one being computed for src 0, the current one
//   for src 1)
template <typename T>
__device__ __forceinline__ const T* a_row(const RunDev& P, int src, uint32_t gh, int64_t i) {
  // (gh is uniform: the handle generation, resolved once per block)
  if (src == 2) return static_cast<const T*>(P.stage) + i * P.ld;
  const uint32_t N = static_cast<uint32_t>(P.N);
  const uint32_t g = run_gen(P, gh);
  const uint8_t* cur = P.flags + ((src == 0 ? g - 1 : g) & 1u) * static_cast<int64_t>(N);
  const uint32_t b = cur[i] ^ (src == 0 ? 1u : 0u);
  return static_cast<const T*>(P.X[b]) + i * P.ld;
}

// 16-byte vector moves of N elements of type V (N * sizeof(V) a multiple of 16).
template <typename V, int N>
__device__ __forceinline__ void copy16(V* __restrict__ dst, const V* __restrict__ src) {
  static_assert((N * sizeof(V)) % 16 == 0, "whole 16-byte vectors");
#pragma unroll
  for (int q = 0; q < static_cast<int>(N * sizeof(V) / 16); ++q)
    reinterpret_cast<uint4*>(dst)[q] = reinterpret_cast<const uint4*>(src)[q];
}

// Pieces of A = U - o for the split-bf16 modes, zero past D: piece p of row i
// is row i of plane p, apc + (p N + i) ldk.  One thread per 8 values.
template <int P>
__global__ void __launch_bounds__(256) k_rot_split(const RunDev* __restrict__ runs, int32_t run,
                                                  int src, GenNo ghn, int64_t rows) {
  const RunDev& Pr = runs[run];
  const int64_t ldk = Pr.ldk;  // equals the population pitch ld
  const int64_t e = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * 8;
  if (e >= rows * ldk) return;
  const int64_t i = e / ldk, k0 = e % ldk;  // ldk is a multiple of 32
  // padding columns are zero in every row source and in the shift
  const float4* a = reinterpret_cast<const float4*>(a_row<float>(Pr, src, gen_value(ghn), i) + k0);
  const float4* o = reinterpret_cast<const float4*>(static_cast<const float*>(Pr.o) + k0);
  const float4 a0 = a[0], a1 = a[1], o0 = o[0], o1 = o[1];
  const float d[8] = {a0.x - o0.x, a0.y - o0.y, a0.z - o0.z, a0.w - o0.w,
                      a1.x - o1.x, a1.y - o1.y, a1.z - o1.z, a1.w - o1.w};
  uint32_t h[4], m[4], l[4];  // pairs of bf16 pieces
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    __bf16 h0, m0, l0, h1, m1, l1;
    split3(d[2 * v], h0, m0, l0);
    split3(d[2 * v + 1], h1, m1, l1);
    h[v] = pack_bf16(h0, h1);
    m[v] = pack_bf16(m0, m1);
    l[v] = pack_bf16(l0, l1);
  }
  __bf16* out = static_cast<__bf16*>(Pr.apc) + i * ldk + k0;
  const int64_t plane = Pr.N * ldk;
  *reinterpret_cast<uint4*>(out) = make_uint4(h[0], h[1], h[2], h[3]);
  *reinterpret_cast<uint4*>(out + plane) = make_uint4(m[0], m[1], m[2], m[3]);
  if constexpr (P == 3) *reinterpret_cast<uint4*>(out + 2 * plane) = make_uint4(l[0], l[1], l[2], l[3]);
}

// FP32 / FP64 product, one 128x128 (FP64: 64x64) tile of Z per block of NW
// waves (NW/2 along rows, 2 along columns), with the shift subtracted as the
// A slice goes into LDS.  The next K slice is fetched into registers while
// the matrix cores work on the current one from LDS, then written into the
// other LDS buffer, so one barrier per K step separates the two.  FP64 uses 8
// waves of 16x32 (57 registers, up to 8 waves per SIMD: 0.61 vs 0.70 ms with
// 4 waves of 32x32, the same results bit for bit); FP32 4 waves of 64x64 (8
// waves measured the same).
template <int MODE>
__global__ void __launch_bounds__(64 * MM<MODE>::NW) k_rot_gemm(const RunDev* __restrict__ runs, int32_t run,
                                                               int src, GenNo ghn, int64_t rows) {
  const uint32_t gh = gen_value(ghn);
  using C = MM<MODE>;
  using T = typename C::T;
  constexpr int BM = C::BM, BN = C::BN, KT = C::KT, LDK = KT + C::PAD;
  constexpr int NT = 64 * C::NW, WVM = C::NW / 2;   // threads; waves along rows
  constexpr int WM = BM / (16 * WVM), WN = BN / 32;  // 16x16 subtiles per wave
  __shared__ __attribute__((aligned(16))) T As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][BN][LDK];
  __shared__ T red[2][BM];

  const RunDev& Pr = runs[run];
  const int64_t D = Pr.D, ldk = Pr.ldk;
  const int ntm = static_cast<int>((rows + BM - 1) / BM);
  const int ntn = static_cast<int>((D + BN - 1) / BN);
  // XCD-aware order: consecutive blocks go round-robin over the 8 XCDs, so
  // hand each XCD whole rows of tiles (tiles of one row block share A) and
  // visit them column by column, so that the blocks in flight on an XCD
  // cover a squarer patch of Z and fetch fewer operand rows from beyond its
  // L2 (the FP64 product with 4 waves per block: 0.69-0.70 vs 0.71-0.72 ms
  // with row-major order); else a contiguous range of tiles per XCD.
  const int nb = ntm * ntn;
  int b = blockIdx.x;
  int tm = b / ntn, tn = b % ntn;
  if (nb % 8 == 0 && (nb / 8) % ntn == 0) {
    const int rx = nb / 8 / ntn, x = b % 8, loc = b / 8;
    tm = x * rx + loc % rx;
    tn = loc / rx;
  } else if (nb % 8 == 0) {
    b = (b % 8) * (nb / 8) + b / 8;
    tm = b / ntn;
    tn = b % ntn;
  }
  const int64_t row0 = static_cast<int64_t>(tm) * BM, col0 = static_cast<int64_t>(tn) * BN;

  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave / 2, wn = wave % 2;

  // Global -> LDS assignment: each thread moves one row segment of the A and
  // of the B slice (A_SEG, B_SEG contiguous values; 16 bytes or more).
  constexpr int A_TPR = NT / BM, A_SEG = KT / A_TPR;
  constexpr int B_TPR = NT / BN, B_SEG = KT / B_TPR;
  const int a_r = tid / A_TPR, a_k = (tid % A_TPR) * A_SEG;
  const int b_r = tid / B_TPR, b_k = (tid % B_TPR) * B_SEG;
  const int64_t ai = min(row0 + a_r, rows - 1);
  const T* arow = a_row<T>(Pr, src, gh, ai) + a_k;
  const T* orow = static_cast<const T*>(Pr.o) + a_k;
  // rows of M are padded to a multiple of 256
  const T* brow = static_cast<const T*>(Pr.B[0]) + (col0 + b_r) * ldk + b_k;

  // The next K slice, held as 16-byte vectors only (element access through
  // casts of local arrays would put them in scratch memory).
  constexpr int E = 16 / static_cast<int>(sizeof(T));  // elements per vector
  constexpr int AV = A_SEG / E, BV = B_SEG / E;
  static_assert(AV * E == A_SEG && BV * E == B_SEG, "whole 16-byte segments");
  uint4 va[AV], vo[AV], vb[BV];
  auto ld16 = [](const void* p) { return *reinterpret_cast<const uint4*>(p); };
  // LDS rows are KT + PAD elements = 136 bytes, an odd multiple of 8: the 16
  // rows one fragment read touches at a given k fall into distinct banks
  // (with 144-byte rows a third of the LDS cycles were bank conflicts).  The
  // rows are 8-byte aligned, so a 16-byte segment goes in as two stores.
  auto st16 = [](void* p, uint4 v) {
    reinterpret_cast<uint2*>(p)[0] = make_uint2(v.x, v.y);
    reinterpret_cast<uint2*>(p)[1] = make_uint2(v.z, v.w);
  };
#define DE_ROT_FETCH(K0)                                                                  \
  do {                                                                                    \
    const int64_t k0_ = (K0);                                                             \
    _Pragma("unroll") for (int q = 0; q < AV; ++q) {                                     \
      va[q] = ld16(arow + k0_ + q * E);                                                   \
      vo[q] = ld16(orow + k0_ + q * E); /* padding columns are zero on both sides */      \
    }                                                                                     \
    _Pragma("unroll") for (int q = 0; q < BV; ++q) vb[q] = ld16(brow + k0_ + q * E);     \
  } while (0)
#define DE_ROT_STASH(BUF)                                                                 \
  do {                                                                                    \
    const int b_ = (BUF);                                                                 \
    _Pragma("unroll") for (int q = 0; q < AV; ++q) {                                     \
      if constexpr (sizeof(T) == 4) {                                                     \
        const float4 x = __builtin_bit_cast(float4, va[q]);                              \
        const float4 y = __builtin_bit_cast(float4, vo[q]);                              \
        st16(&As[b_][a_r][a_k + q * E],                                                   \
             __builtin_bit_cast(uint4, make_float4(x.x - y.x, x.y - y.y, x.z - y.z, x.w - y.w))); \
      } else {                                                                            \
        const double2 x = __builtin_bit_cast(double2, va[q]);                            \
        const double2 y = __builtin_bit_cast(double2, vo[q]);                            \
        st16(&As[b_][a_r][a_k + q * E], __builtin_bit_cast(uint4, make_double2(x.x - y.x, x.y - y.y))); \
      }                                                                                   \
    }                                                                                     \
    _Pragma("unroll") for (int q = 0; q < BV; ++q) st16(&Bs[b_][b_r][b_k + q * E], vb[q]); \
  } while (0)

  using Acc = typename std::conditional<MODE == MM_FP64, f64x4, f32x4>::type;
  Acc acc[WM][WN];
#pragma unroll
  for (int m = 0; m < WM; ++m)
#pragma unroll
    for (int n = 0; n < WN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][n][r] = 0;

  const int nk = static_cast<int>((D + KT - 1) / KT);
  DE_ROT_FETCH(0);
  DE_ROT_STASH(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) DE_ROT_FETCH(static_cast<int64_t>(kt + 1) * KT);
#pragma unroll
    for (int s = 0; s < KT / 4; ++s) {
      T af[WM], bf[WN];
#pragma unroll
      for (int m = 0; m < WM; ++m) af[m] = As[buf][wm * (BM / WVM) + m * 16 + lane % 16][4 * s + lane / 16];
#pragma unroll
      for (int n = 0; n < WN; ++n) bf[n] = Bs[buf][wn * (BN / 2) + n * 16 + lane % 16][4 * s + lane / 16];
#pragma unroll
      for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int n = 0; n < WN; ++n) {
          if constexpr (MODE == MM_FP64)
            acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[m], bf[n], acc[m][n], 0, 0, 0);
          else
            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[m], bf[n], acc[m][n], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) DE_ROT_STASH(buf ^ 1);
    __syncthreads();
  }

#undef DE_ROT_FETCH
#undef DE_ROT_STASH

  // ---- epilogue: sum_k w_k z_ik^2 over this block's columns ----
  const T* w = static_cast<const T*>(Pr.w);
  T rs[WM][4];
#pragma unroll
  for (int m = 0; m < WM; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) rs[m][r] = T(0);
#pragma unroll
  for (int n = 0; n < WN; ++n) {
    const int64_t k = col0 + wn * (BN / 2) + n * 16 + lane % 16;
    const T wk = k < D ? w[k] : T(0);
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T z = static_cast<T>(acc[m][n][r]);
        rs[m][r] += wk * z * z;
      }
  }
  // reduce over the 16 lanes that share a row (fixed butterfly order)
#pragma unroll
  for (int m = 0; m < WM; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      T v = rs[m][r];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      rs[m][r] = v;
    }
  if (lane % 16 == 0) {
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = MODE == MM_FP64 ? 4 * r + lane / 16 : (lane / 16) * 4 + r;
        red[wn][wm * (BM / WVM) + m * 16 + rr] = rs[m][r];
      }
  }
  __syncthreads();
  T* part = static_cast<T*>(Pr.part);
  const int ntot = Pr.ntile;
  for (int rr = tid; rr < BM; rr += NT) {
    const int64_t i = row0 + rr;
    if (i < rows) part[i * ntot + tn] = red[0][rr] + red[1][rr];
  }
}

// ---- split-bf16 product -----------------------------------------------------

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N-1>): indices
// known at compile time, so the register arrays they index stay in registers.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Pieces multiplied by cross product Q of a P-piece split: (A piece, B
// piece), smallest products first: hi*lo terms before hi*hi.
template <int P, int Q> struct SplitProd {
  static constexpr int q = P == 3 ? Q : Q + 3;
  static constexpr int a = q == 0 ? 2 : q == 1 ? 1 : q == 2 ? 0 : q == 3 ? 1 : q == 4 ? 0 : 0;
  static constexpr int b = q == 0 ? 0 : q == 1 ? 1 : q == 2 ? 2 : q == 3 ? 0 : q == 4 ? 1 : 0;
};

// The LDS slices hold rows of KT bf16 (KT / 8 chunks of 16 bytes) with the
// chunk index XOR-ed by a function of the row, so that the 16-byte fragment
// reads of consecutive rows at one k fall into different banks without
// padding: chunk kc of row r sits at kc ^ swz(r).
template <int KT>
__device__ __forceinline__ int swz(int row) {
  constexpr int KC = KT / 8, R128 = 64 / KT > 0 ? 64 / KT : 1;  // rows per 128 bytes
  return (row / R128) % KC;
}

// The slices go from global memory to LDS by the LDS-DMA load: lane l's 16
// bytes at base + off land at LDS byte address lds + 16 l (base and lds
// wave-uniform, lds in M0, off a per-lane byte offset) without passing
// through registers; the load counts in vmcnt.  Written as asm: through the
// compiler builtin, every LDS read and every barrier after it would wait for
// all DMA loads in flight, which serialises the fetch of the next slice with
// the products of this one.  It has no output register; the kernel orders it
// with explicit vmcnt waits before the barrier that publishes a slice.  One
// wait state separates the M0 write from the load that reads it (the
// compiler keeps the same distance for the builtin).  M0 has no other user in
// the kernels that call it.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void lds_dma16(const void* base, uint32_t off, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(off), "s"(base), "s"(lds)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// s_waitcnt immediate for vmcnt(n), the other counters left alone
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// Split-bf16 product, one BM x BN tile of Z per block of (BM/64) x (BN/64)
// waves, each wave a 64x64 sub-tile as MF x MF matrix-core tiles (MF = 16:
// 16x16x32, MF = 32: 32x32x16).  The A pieces come from the piece planes of
// the rows (apc), the B pieces from the split M.  K advances KT columns per
// step through NBUF LDS buffers.
//   Without PP, every wave loads its share of the slices, NBUF - 1 slices in
// flight: at the start of step kt a wave waits for its own loads of slice kt,
// a barrier makes all of slice kt visible (and ends every read of slice
// kt - 1), and the wave then starts the loads of slice kt + NBUF - 1 into the
// buffer slice kt - 1 held before computing on slice kt.
//   With PP (8 waves, two buffers) the waves form two groups of four, one
// wave of each per SIMD, half a step apart: every wave runs "read the
// fragments of slice k | barrier | products of slice k | barrier", group 1
// one barrier behind group 0, so that on each SIMD one wave issues
// matrix-core ops while the other reads LDS; the product phase runs at raised
// wave priority.  Group 0 loads all of slice k + 1 when it starts reading
// slice k (both groups are done with slice k - 1, whose buffer it refills)
// and waits for it at the end of its products of slice k.
// What the split product reads of a run, passed by value (kernel arguments
// rather than loads from the run record keep the addresses in registers).
struct SplitArgs {
  const __bf16* apc;   // A pieces: plane p, row i at apc + (p N + i) ldk
  const __bf16* B[3];  // M pieces, rows padded to a multiple of 256, pitch ldk
  const float* w;      // D weights
  float* part;         // rows x ntile partial sums
  int64_t N, D, ldk;
  int32_t ntile;
};

template <int P, int BM, int BN, int KT, int MF, int NBUF, bool PP>
__global__ void __launch_bounds__((BM / 64) * (BN / 64) * 64)
k_rot_gemm_split(SplitArgs Pr, int64_t rows) {
  constexpr int WNV = BN / 64, NT = (BM / 64) * WNV * 64, WAVES = NT / 64;
  constexpr int KC = KT / 8;  // 16-byte chunks per slice row
  static_assert(!PP || (WAVES == 8 && NBUF == 2), "ping-pong: 8 waves, two buffers");
  // a piece's slice is BM * KC (BN * KC) chunks = ABLK (BBLK) blocks of 64
  // chunks, one DMA load of a wave each; loading wave w loads blocks w,
  // w + LW, ...
  constexpr int LW = PP ? WAVES / 2 : WAVES;
  constexpr int ABLK = BM * KC / 64, BBLK = BN * KC / 64;
  static_assert(ABLK % LW == 0 && BBLK % LW == 0, "whole blocks per loading wave");
  constexpr int NA = ABLK / LW, NB = BBLK / LW, LPS = P * (NA + NB);
  static_assert(MF == 32 ? KT % 16 == 0 : KT % 32 == 0, "k steps of the matrix-core form");
  static_assert(NBUF >= 2 && LPS * (NBUF - 2) < 64, "vmcnt range");
  __shared__ __attribute__((aligned(16))) __bf16 As[NBUF][P][BM * KT];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NBUF][P][BN * KT];
  __shared__ float red[WNV][BM];

  const int64_t D = Pr.D, ldk = Pr.ldk;
  const int ntm = static_cast<int>((rows + BM - 1) / BM);
  const int ntn = static_cast<int>((D + BN - 1) / BN);
  const int nb = ntm * ntn;
  int b = blockIdx.x;
  if (nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;  // a contiguous range of tiles per XCD
  const int tm = b / ntn, tn = b % ntn;
  const int64_t row0 = static_cast<int64_t>(tm) * BM, col0 = static_cast<int64_t>(tn) * BN;
  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int wm = wave / WNV, wn = wave % WNV;
  const bool g1 = PP && wave >= LW;
  const int lw = wave % LW;

  // lane l of block blk fills chunk u = 64 blk + l of the slice: row u / KC,
  // stored chunk u % KC, which holds logical chunk (u % KC) ^ swz(row).  Byte
  // offsets from the tile's first row (< BM ldk 2 bytes; rows past the end
  // re-read the last row).
  uint32_t oa[NA], ob[NB];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const int u = (lw + j * LW) * 64 + lane, r = u / KC, kc = (u % KC) ^ swz<KT>(r);
    const int64_t rr = min(row0 + r, rows - 1) - row0;
    oa[j] = static_cast<uint32_t>((rr * ldk + kc * 8) * 2);
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int u = (lw + j * LW) * 64 + lane, r = u / KC, kc = (u % KC) ^ swz<KT>(r);
    ob[j] = static_cast<uint32_t>((static_cast<int64_t>(r) * ldk + kc * 8) * 2);  // M rows padded to 256
  }
  const __bf16* abase = Pr.apc + row0 * ldk;
  const int64_t plane = Pr.N * ldk;
  const uint32_t lds_a = __builtin_amdgcn_readfirstlane(
      static_cast<uint32_t>(reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) void*)&As[0][0][0])));
  const uint32_t lds_b = __builtin_amdgcn_readfirstlane(
      static_cast<uint32_t>(reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) void*)&Bs[0][0][0])));
  auto fetch = [&](int slice, int buf) {
    const int64_t k0 = static_cast<int64_t>(slice) * KT;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const __bf16* pa = abase + p * plane + k0;
      const __bf16* pb = Pr.B[p] + col0 * ldk + k0;
#pragma unroll
      for (int j = 0; j < NA; ++j)
        lds_dma16(pa, oa[j], lds_a + 2u * static_cast<uint32_t>((buf * P + p) * BM * KT + (lw + j * LW) * 512));
#pragma unroll
      for (int j = 0; j < NB; ++j)
        lds_dma16(pb, ob[j], lds_b + 2u * static_cast<uint32_t>((buf * P + p) * BN * KT + (lw + j * LW) * 512));
    }
  };

  constexpr int NPR = P == 3 ? 6 : 3;
  constexpr int SM = 64 / MF;             // matrix-core tiles per wave side
  constexpr int KS = MF == 32 ? 16 : 32;  // k per matrix-core op
  using Acc = typename std::conditional<MF == 32, f32x16, f32x4>::type;
  Acc acc[SM][SM];
#pragma unroll
  for (int m = 0; m < SM; ++m)
#pragma unroll
    for (int n = 0; n < SM; ++n) acc[m][n] = Acc{};
  bf16x8 fa[P][SM], fb[P][SM];
  auto read_fragments = [&](int buf, int ks) {
    const int kc = ks * (KS / 8) + lane / MF;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int m = 0; m < SM; ++m) {
        const int ra = wm * 64 + m * MF + lane % MF;
        const int rb = wn * 64 + m * MF + lane % MF;
        fa[p][m] = *reinterpret_cast<const bf16x8*>(&As[buf][p][ra * KT + (kc ^ swz<KT>(ra)) * 8]);
        fb[p][m] = *reinterpret_cast<const bf16x8*>(&Bs[buf][p][rb * KT + (kc ^ swz<KT>(rb)) * 8]);
      }
  };
  // the product loop is outermost, so consecutive matrix-core ops use
  // different accumulators
  auto products = [&]() {
    static_for<NPR>([&](auto qc) {
      constexpr int ia = SplitProd<P, decltype(qc)::value>::a;
      constexpr int ib = SplitProd<P, decltype(qc)::value>::b;
#pragma unroll
      for (int m = 0; m < SM; ++m)
#pragma unroll
        for (int n = 0; n < SM; ++n) {
          if constexpr (MF == 32)
            acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[ia][m], fb[ib][n], acc[m][n], 0, 0, 0);
          else
            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[ia][m], fb[ib][n], acc[m][n], 0, 0, 0);
        }
    });
  };

  const int nk = static_cast<int>((D + KT - 1) / KT);
  if constexpr (PP) {
    static_assert(KT == KS, "one fragment set per step");
    if (!g1) {
      fetch(0, 0);
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    }
    __syncthreads();
    if (g1) __syncthreads();
    // sched_barrier(0) keeps the compiler from moving matrix-core ops across
    // the barriers, which would undo the phases
    for (int k = 0; k < nk; ++k) {
      if (!g1 && k + 1 < nk) fetch(k + 1, (k + 1) & 1);
      read_fragments(k & 1, 0);
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_setprio(1);
      products();
      __builtin_amdgcn_s_setprio(0);
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
    }
    if (!g1) __syncthreads();
  } else {
#pragma unroll
    for (int sl = 0; sl < NBUF - 1; ++sl)
      if (sl < nk) fetch(sl, sl);
    for (int kt = 0; kt < nk; ++kt) {
      // slice kt landed once at most the NBUF - 2 slices after it are in flight
      if (kt + NBUF - 2 < nk) __builtin_amdgcn_s_waitcnt(vmcnt_imm(LPS * (NBUF - 2)));
      else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
      __syncthreads();
      if (kt + NBUF - 1 < nk) fetch(kt + NBUF - 1, (kt + NBUF - 1) % NBUF);
#pragma unroll
      for (int ks = 0; ks < KT / KS; ++ks) {
        read_fragments(kt % NBUF, ks);
        products();
      }
    }
  }
  // the last step waited for vmcnt(0): no load is in flight past here

  // ---- epilogue: sum_n w_n z_in^2 over this block's columns ----
  constexpr int NR = MF == 32 ? 16 : 4;  // accumulator registers per tile
  const float* w = Pr.w;
  float rs[SM][NR];
#pragma unroll
  for (int m = 0; m < SM; ++m)
#pragma unroll
    for (int r = 0; r < NR; ++r) rs[m][r] = 0.f;
#pragma unroll
  for (int n = 0; n < SM; ++n) {
    const int64_t k = col0 + wn * 64 + n * MF + lane % MF;
    const float wk = k < D ? w[k] : 0.f;
#pragma unroll
    for (int m = 0; m < SM; ++m)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const float z = acc[m][n][r];
        rs[m][r] += wk * z * z;
      }
  }
  // reduce over the MF lanes that share a row (fixed butterfly order)
#pragma unroll
  for (int m = 0; m < SM; ++m)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      float v = rs[m][r];
#pragma unroll
      for (int off = 1; off < MF; off <<= 1) v += __shfl_xor(v, off);
      rs[m][r] = v;
    }
  if (lane % MF == 0) {
#pragma unroll
    for (int m = 0; m < SM; ++m)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int rr = MF == 32 ? 8 * (r / 4) + 4 * (lane / 32) + (r % 4) : (lane / 16) * 4 + r;
        red[wn][wm * 64 + m * MF + rr] = rs[m][r];
      }
  }
  __syncthreads();
  // one partial per 128 columns (two wave columns), whatever the tile width,
  // so every tile shape writes the same partial sums
  constexpr int PG = BN / 128;
  float* part = Pr.part;
  for (int e = tid; e < BM * PG; e += NT) {
    const int rr = e % BM, q = e / BM;
    const int64_t i = row0 + rr;
    const int col = tn * PG + q;
    if (i < rows && col < Pr.ntile) part[i * Pr.ntile + col] = red[2 * q][rr] + red[2 * q + 1][rr];
  }
}

// Sum of the partials of row i in tile order.
template <typename T>
__device__ __forceinline__ T row_total(const RunDev& P, int64_t i, int ntn) {
  const T* part = static_cast<const T*>(P.part) + i * P.ntile;
  T f = T(0);
  for (int t = 0; t < ntn; ++t) f += part[t];
  return canon(f);
}

// Greedy selection on the trials of generation g (Alg 2's selection).
template <typename T>
__global__ void k_rot_select(const RunDev* __restrict__ runs, int32_t run, int ntn, GenNo gn) {
  const uint32_t gnew = gen_value(gn);
  const RunDev& P = runs[run];
  const uint32_t N = static_cast<uint32_t>(P.N);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t g = run_gen(P, gnew);
  const uint8_t* cur = P.flags + ((g - 1) & 1u) * static_cast<int64_t>(N);
  uint8_t* nxt = P.flags + (g & 1u) * static_cast<int64_t>(N);
  const uint32_t ci = cur[i];
  const T fu = row_total<T>(P, i, ntn);
  T* fit = static_cast<T*>(P.fit);
  const bool win = fu < fit[i];
  nxt[i] = static_cast<uint8_t>(win ? ci ^ 1u : ci);
  if (win) fit[i] = fu;
  static_cast<T*>(P.hist)[static_cast<int64_t>(gnew % kHist) * N + i] = win ? fu : Math<T>::inf();
  if (P.tr_idx) P.tr_idx[6 * static_cast<int64_t>(i) + 5] = win ? 1 : 0;
  if (P.tr_ftrial) static_cast<T*>(P.tr_ftrial)[i] = fu;
}

template <typename T>
__global__ void k_rot_store(const RunDev* __restrict__ runs, int32_t run, int ntn, int64_t rows,
                            T* __restrict__ out) {
  const RunDev& P = runs[run];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  out[i] = row_total<T>(P, i, ntn);
}

// M pieces (rows padded to a multiple of 256, columns to ldk, zero filled)
// and the weights 10^(6k/(D-1)).
template <int MODE>
__global__ void k_rot_prepare(RunDev Pr, int64_t rows_pad) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t D = Pr.D, ldk = Pr.ldk;
  if (e < rows_pad * ldk) {
    const int64_t n = e / ldk, k = e % ldk;
    const double m = (n < D && k < D) ? Pr.rot[n * D + k] : 0.0;
    if constexpr (MODE == MM_FP64) {
      static_cast<double*>(const_cast<void*>(Pr.B[0]))[e] = m;
    } else if constexpr (MODE == MM_FP32) {
      static_cast<float*>(const_cast<void*>(Pr.B[0]))[e] = static_cast<float>(m);
    } else {
      // split the FP64 value directly: each remainder is exact in FP64
      const __bf16 h = static_cast<__bf16>(static_cast<float>(m));
      const double r1 = m - static_cast<double>(static_cast<float>(h));
      const __bf16 md = static_cast<__bf16>(static_cast<float>(r1));
      const double r2 = r1 - static_cast<double>(static_cast<float>(md));
      const __bf16 l = static_cast<__bf16>(static_cast<float>(r2));
      static_cast<__bf16*>(const_cast<void*>(Pr.B[0]))[e] = h;
      static_cast<__bf16*>(const_cast<void*>(Pr.B[1]))[e] = md;
      if (MODE == MM_BF16X6) static_cast<__bf16*>(const_cast<void*>(Pr.B[2]))[e] = l;
    }
  }
}

template <typename T>
__global__ void k_rot_weights(T* w, int64_t D) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < D) w[k] = static_cast<T>(D > 1 ? pow(10.0, 6.0 * static_cast<double>(k) / static_cast<double>(D - 1)) : 1.0);
}

// Dense caller rows -> padded staging rows (zero padding).
template <typename T>
__global__ void k_rot_stage(T* __restrict__ dst, int64_t ld, const T* __restrict__ src, int64_t D,
                            int64_t rows) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rows * ld) return;
  const int64_t i = e / ld, k = e % ld;
  dst[e] = k < D ? src[i * D + k] : T(0);
}

static inline unsigned nb(int64_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

static int tile_n_of(int mode) { return mode == MM_FP64 ? MM<MM_FP64>::BN : 128; }
static int tile_m_of(int mode) { return mode == MM_FP64 ? MM<MM_FP64>::BM : MM<MM_FP32>::BM; }

hipError_t launch_prepare_rot(const RunDev& h, hipStream_t s) {
  const int64_t rows_pad = (h.D + 255) / 256 * 256;
  const int64_t n = rows_pad * h.ldk;
  switch (h.mm) {
    case MM_FP64: hipLaunchKernelGGL(k_rot_prepare<MM_FP64>, dim3(nb(n, 256)), dim3(256), 0, s, h, rows_pad); break;
    case MM_FP32: hipLaunchKernelGGL(k_rot_prepare<MM_FP32>, dim3(nb(n, 256)), dim3(256), 0, s, h, rows_pad); break;
    case MM_BF16X3: hipLaunchKernelGGL(k_rot_prepare<MM_BF16X3>, dim3(nb(n, 256)), dim3(256), 0, s, h, rows_pad); break;
    case MM_BF16X6: hipLaunchKernelGGL(k_rot_prepare<MM_BF16X6>, dim3(nb(n, 256)), dim3(256), 0, s, h, rows_pad); break;
    default: return hipErrorInvalidValue;
  }
  if (h.dtype == 0)
    hipLaunchKernelGGL(k_rot_weights<double>, dim3(nb(h.D, 256)), dim3(256), 0, s,
                       static_cast<double*>(const_cast<void*>(h.w)), h.D);
  else
    hipLaunchKernelGGL(k_rot_weights<float>, dim3(nb(h.D, 256)), dim3(256), 0, s,
                       static_cast<float*>(const_cast<void*>(h.w)), h.D);
  return hipGetLastError();
}

// Tile shapes of the split-bf16 product (BM x BN block tile, KT, matrix-core
// form MF, NBUF LDS buffers, ping-pong wave groups PP) for P pieces: option 1 is the default, 2 and 3
// the runners-up, from sweeps on MI355X at 4096 x 2048 x 2048 (rows, D, D) in
// a harness and in place behind the trial kernel; the tuner picks among them
// per shape.
template <int P, int OPT> struct SplitShape;
template <> struct SplitShape<3, 1> { static constexpr int BM = 256, BN = 128, KT = 32, MF = 16, NBUF = 2; static constexpr bool PP = true; };
template <> struct SplitShape<3, 2> { static constexpr int BM = 128, BN = 256, KT = 32, MF = 16, NBUF = 2; static constexpr bool PP = true; };
template <> struct SplitShape<3, 3> { static constexpr int BM = 256, BN = 128, KT = 32, MF = 16, NBUF = 2; static constexpr bool PP = false; };
template <> struct SplitShape<2, 1> { static constexpr int BM = 128, BN = 256, KT = 32, MF = 16, NBUF = 2; static constexpr bool PP = true; };
template <> struct SplitShape<2, 2> { static constexpr int BM = 128, BN = 128, KT = 32, MF = 16, NBUF = 2; static constexpr bool PP = false; };
template <> struct SplitShape<2, 3> { static constexpr int BM = 256, BN = 128, KT = 32, MF = 16, NBUF = 2; static constexpr bool PP = true; };

template <int P, int OPT>
static void launch_split_gemm(const SplitArgs& a, int64_t rows, hipStream_t s) {
  using S = SplitShape<P, OPT>;
  const int64_t blocks = ((rows + S::BM - 1) / S::BM) * ((a.D + S::BN - 1) / S::BN);
  hipLaunchKernelGGL((k_rot_gemm_split<P, S::BM, S::BN, S::KT, S::MF, S::NBUF, S::PP>), dim3(blocks),
                     dim3((S::BM / 64) * (S::BN / 64) * 64), 0, s, a, rows);
}

template <int P>
static void launch_split_gemm(const RunDev& h, int64_t rows, hipStream_t s) {
  SplitArgs a;
  a.apc = static_cast<const __bf16*>(h.apc);
  for (int p = 0; p < 3; ++p) a.B[p] = static_cast<const __bf16*>(h.B[p]);
  a.w = static_cast<const float*>(h.w);
  a.part = static_cast<float*>(h.part);
  a.N = h.N;
  a.D = h.D;
  a.ldk = h.ldk;
  a.ntile = h.ntile;
  switch (h.tile) {
    case 2: launch_split_gemm<P, 2>(a, rows, s); break;
    case 3: launch_split_gemm<P, 3>(a, rows, s); break;
    default: launch_split_gemm<P, 1>(a, rows, s); break;
  }
}

// split: write the bf16 pieces of the row source first (split-bf16 modes);
// the trial kernel of a generation writes them itself.
static hipError_t gemm(const RunDev* runs, const RunDev& h, int run, int src, GenNo gh,
                       int64_t rows, hipStream_t s, bool split = true) {
  if (h.mm == MM_BF16X3 || h.mm == MM_BF16X6) {
    if (split) {
      const unsigned sb = nb(rows * h.ldk / 8, 256);
      if (h.mm == MM_BF16X3)
        hipLaunchKernelGGL(k_rot_split<2>, dim3(sb), dim3(256), 0, s, runs, run, src, gh, rows);
      else
        hipLaunchKernelGGL(k_rot_split<3>, dim3(sb), dim3(256), 0, s, runs, run, src, gh, rows);
    }
    if (h.mm == MM_BF16X3) launch_split_gemm<2>(h, rows, s);
    else launch_split_gemm<3>(h, rows, s);
    return hipGetLastError();
  }
  const int bm = tile_m_of(h.mm), bn = tile_n_of(h.mm);
  const int64_t blocks = ((rows + bm - 1) / bm) * ((h.D + bn - 1) / bn);
  switch (h.mm) {
    case MM_FP64:
      hipLaunchKernelGGL(k_rot_gemm<MM_FP64>, dim3(blocks), dim3(64 * MM<MM_FP64>::NW), 0, s, runs, run, src, gh, rows);
      break;
    case MM_FP32:
      hipLaunchKernelGGL(k_rot_gemm<MM_FP32>, dim3(blocks), dim3(64 * MM<MM_FP32>::NW), 0, s, runs, run, src, gh, rows);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rot_fitness(const RunDev* runs, const RunDev& h, int run, GenNo gnew,
                              bool split, hipStream_t s) {
  return gemm(runs, h, run, 0, gnew, h.N, s, split);
}

hipError_t launch_rot_select(const RunDev* runs, const RunDev& h, int run, GenNo gnew,
                             hipStream_t s) {
  const int ntn = static_cast<int>((h.D + tile_n_of(h.mm) - 1) / tile_n_of(h.mm));
  if (h.dtype == 0) hipLaunchKernelGGL(k_rot_select<double>, dim3(nb(h.N, 256)), dim3(256), 0, s, runs, run, ntn, gnew);
  else hipLaunchKernelGGL(k_rot_select<float>, dim3(nb(h.N, 256)), dim3(256), 0, s, runs, run, ntn, gnew);
  return hipGetLastError();
}

hipError_t launch_rot_init_fit(const RunDev* runs, const RunDev& h, int run, hipStream_t s) {
  hipError_t e = gemm(runs, h, run, 1, GenNo{0, 0, nullptr}, h.N, s);
  if (e != hipSuccess) return e;
  const int ntn = static_cast<int>((h.D + tile_n_of(h.mm) - 1) / tile_n_of(h.mm));
  if (h.dtype == 0)
    hipLaunchKernelGGL(k_rot_store<double>, dim3(nb(h.N, 256)), dim3(256), 0, s, runs, run, ntn, h.N,
                       static_cast<double*>(h.fit));
  else
    hipLaunchKernelGGL(k_rot_store<float>, dim3(nb(h.N, 256)), dim3(256), 0, s, runs, run, ntn, h.N,
                       static_cast<float*>(h.fit));
  return hipGetLastError();
}

// Caller rows in chunks of N through the staging buffer.
hipError_t launch_rot_eval_rows(const RunDev* runs, const RunDev& h, int run, const void* X,
                                int64_t rows, void* out, hipStream_t s) {
  const int ntn = static_cast<int>((h.D + tile_n_of(h.mm) - 1) / tile_n_of(h.mm));
  const int64_t esz = h.dtype == 0 ? 8 : 4;
  for (int64_t r0 = 0; r0 < rows; r0 += h.N) {
    const int64_t n = rows - r0 < h.N ? rows - r0 : h.N;
    const char* src = static_cast<const char*>(X) + r0 * h.D * esz;
    char* dst = static_cast<char*>(out) + r0 * esz;
    if (h.dtype == 0)
      hipLaunchKernelGGL(k_rot_stage<double>, dim3(nb(n * h.ld, 256)), dim3(256), 0, s,
                         static_cast<double*>(h.stage), h.ld, reinterpret_cast<const double*>(src), h.D, n);
    else
      hipLaunchKernelGGL(k_rot_stage<float>, dim3(nb(n * h.ld, 256)), dim3(256), 0, s,
                         static_cast<float*>(h.stage), h.ld, reinterpret_cast<const float*>(src), h.D, n);
    hipError_t e = gemm(runs, h, run, 2, GenNo{0, 0, nullptr}, n, s);
    if (e != hipSuccess) return e;
    if (h.dtype == 0)
      hipLaunchKernelGGL(k_rot_store<double>, dim3(nb(n, 256)), dim3(256), 0, s, runs, run, ntn, n,
                         reinterpret_cast<double*>(dst));
    else
      hipLaunchKernelGGL(k_rot_store<float>, dim3(nb(n, 256)), dim3(256), 0, s, runs, run, ntn, n,
                         reinterpret_cast<float*>(dst));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace de
