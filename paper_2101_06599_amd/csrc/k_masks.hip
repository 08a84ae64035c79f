// Crossover masks on their own: for generation g of a run, the N x D 0/1
// matrix of Alg 7 (binomial), Alg 8 (classic exponential) or Eq 9 + Alg 10
// (NEC) that the generation kernel applies, written row-major as bytes.
// One wavefront per individual; the draws are the generation kernel's.
#include "de_device.h"

namespace de {

// Mask bits of chunk c (elements 4c .. 4c+3; bit v for element 4c + v).
template <int XO>
__device__ __forceinline__ uint32_t chunk_mask(const RunDev& P, uint32_t g, uint32_t i, uint32_t c,
                                               uint32_t jr, uint32_t L, uint32_t D) {
  const uint32_t j0 = 4 * c;
  uint32_t m = 0;
  if constexpr (XO == XO_BIN) {
    const uint4 b = draw(P, TAG_BIN, g, i, c);
    m = (static_cast<uint64_t>(b.x) < P.thr ? 1u : 0u) | (static_cast<uint64_t>(b.y) < P.thr ? 2u : 0u) |
        (static_cast<uint64_t>(b.z) < P.thr ? 4u : 0u) | (static_cast<uint64_t>(b.w) < P.thr ? 8u : 0u);
    if (jr >= j0 && jr < j0 + 4) m |= 1u << (jr - j0);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t j = j0 + v;
      const uint32_t off = j >= jr ? j - jr : j + D - jr;
      m |= (off < L ? 1u : 0u) << v;
    }
  }
  return m;
}

// Four mask bits as four 0/1 bytes of a little-endian word.
__device__ __forceinline__ uint32_t mask_bytes(uint32_t m) {
  return (m & 1u) | ((m & 2u) << 7) | ((m & 4u) << 14) | ((m & 8u) << 21);
}

// One wavefront per individual.  When D is a multiple of 4, every 16-byte
// aligned unit of a row starts at a chunk boundary: a lane builds four chunks
// and writes them with one 16-byte store, and the at most three chunks before
// the row's first and after its last aligned unit take 4-byte stores.  Other
// rows are written four bytes (or, unaligned, one byte) at a time.
template <int XO>
__global__ void __launch_bounds__(256) k_masks(const RunDev* __restrict__ runs, int32_t run,
                                               uint32_t g, uint8_t* __restrict__ out) {
  const RunDev& P = runs[run];
  const uint32_t N = static_cast<uint32_t>(P.N), D = static_cast<uint32_t>(P.D);
  const uint32_t row = blockIdx.x * 4 + threadIdx.x / 64;
  if (row >= N) return;  // rows are whole wavefronts: a wavefront leaves together
  const uint32_t i = __builtin_amdgcn_readfirstlane(row);
  const uint32_t lane = threadIdx.x % 64;
  const uint4 bx = draw(P, TAG_XO, g, i, 0);
  const uint32_t jr = scale_index(bx.x, D);
  uint32_t L = 0;
  if constexpr (XO == XO_NEC) L = nec_length(P, bx.y);
  if constexpr (XO == XO_EXP)
    L = P.exp_impl == EXPI_SCAN ? exp_length_scan(P, g, i) : exp_length_serial(P, g, i);
  const int64_t base = static_cast<int64_t>(i) * D;
  DE_GLOBAL uint8_t* o = gmut<uint8_t>(out) + base;
  const uint32_t nchunk = (D + 3) >> 2;
  if ((D & 3u) == 0) {
    // chunks [0, h) before the first 16-byte boundary, [h, h + 4 nu) in
    // 16-byte units, the rest after the last one
    const uint32_t h = min(static_cast<uint32_t>((16 - (base & 15)) & 15) >> 2, nchunk);
    const uint32_t nu = (nchunk - h) >> 2;
    for (uint32_t u = lane; u < nu; u += 64) {
      const uint32_t c = h + 4 * u;
      uint4 v;
      v.x = mask_bytes(chunk_mask<XO>(P, g, i, c, jr, L, D));
      v.y = mask_bytes(chunk_mask<XO>(P, g, i, c + 1, jr, L, D));
      v.z = mask_bytes(chunk_mask<XO>(P, g, i, c + 2, jr, L, D));
      v.w = mask_bytes(chunk_mask<XO>(P, g, i, c + 3, jr, L, D));
      *(DE_GLOBAL uint4*)(o + 4 * c) = v;
    }
    const uint32_t tail = h + 4 * nu;
    if (lane < h) *(DE_GLOBAL uint32_t*)(o + 4 * lane) = mask_bytes(chunk_mask<XO>(P, g, i, lane, jr, L, D));
    if (tail + lane < nchunk)
      *(DE_GLOBAL uint32_t*)(o + 4 * (tail + lane)) = mask_bytes(chunk_mask<XO>(P, g, i, tail + lane, jr, L, D));
    return;
  }
  const bool word_aligned = (base & 3) == 0;
  for (uint32_t c = lane; c < nchunk; c += 64) {
    const uint32_t j0 = 4 * c;
    const uint32_t m = chunk_mask<XO>(P, g, i, c, jr, L, D);
    if (word_aligned && j0 + 4 <= D) {
      *(DE_GLOBAL uint32_t*)(o + j0) = mask_bytes(m);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (j0 + v < D) o[j0 + v] = static_cast<uint8_t>((m >> v) & 1u);
    }
  }
}

// Classic exponential masks with one work-item per individual (the p-exp
// mapping of Sec. 3.1): the work-item walks Alg 8 from j_rand, marking one
// element per passed draw, then writes the zeros of the rest of its row in
// the same walking order.
__global__ void __launch_bounds__(64) k_masks_job(const RunDev* __restrict__ runs, int32_t run,
                                                  uint32_t g, uint8_t* __restrict__ out) {
  const RunDev& P = runs[run];
  const uint32_t N = static_cast<uint32_t>(P.N), D = static_cast<uint32_t>(P.D);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t jr = scale_index(draw(P, TAG_XO, g, i, 0).x, D);
  DE_GLOBAL uint8_t* o = gmut<uint8_t>(out) + static_cast<int64_t>(i) * D;
  uint32_t j = jr, L = 0, e = 0;
  uint4 b = make_uint4(0, 0, 0, 0);
  bool more;
  do {
    o[j] = 1;
    j = (j + 1 == D) ? 0 : j + 1;
    ++L;
    if ((e & 3u) == 0) b = draw(P, TAG_EXP, g, i, e >> 2);
    more = static_cast<uint64_t>(word_of(b, e & 3u)) < P.thr && L < D;
    ++e;
  } while (more);
  for (; L < D; ++L) {
    o[j] = 0;
    j = (j + 1 == D) ? 0 : j + 1;
  }
}

// Number of words w with (w + 1/2) 2^-32 < p: ceil(p 2^32 - 1/2) clamped to
// [0, 2^32] (the scaling is exact, the subtraction is one rounding).
__device__ __forceinline__ uint64_t word_threshold(double p) {
  const double v = ceil(ldexp(p, 32) - 0.5);
  if (!(v > 0.0)) return 0;
  if (v >= 4294967296.0) return 4294967296ull;
  return static_cast<uint64_t>(v);
}

// Set-up of a mask call that has no workspace: stores the run record at
// `dst` and, when `table`, the NEC thresholds at rec.T: T[0] = 2^32,
// T[k] = word_threshold(CR^(k-1)) for k = 1..D with the power taken as a
// running FP64 product (the order the handle's own table is built in), and
// T[D+1] = 0.  For CR < 1 the product only decreases, so once a threshold is
// 0 every later one is: one lane walks the non-zero prefix and the block
// writes the zeros after it.
__global__ void __launch_bounds__(256) k_masks_setup(RunDev rec, RunDev* __restrict__ dst,
                                                     int table) {
  __shared__ int64_t kend;
  uint64_t* T = const_cast<uint64_t*>(rec.T);
  const int64_t D = rec.D;
  if (threadIdx.x == 0) {
    *dst = rec;
    int64_t k = 1;
    if (table) {
      T[0] = 4294967296ull;
      double t = 1.0;
      for (; k <= D; ++k) {
        if (k > 1) t = t * rec.CR;
        const uint64_t v = word_threshold(t);
        T[k] = v;
        if (v == 0) {
          ++k;
          break;
        }
      }
    }
    kend = k;
  }
  __syncthreads();
  if (table)
    for (int64_t k = kend + threadIdx.x; k <= D + 1; k += blockDim.x) T[k] = 0;
}

hipError_t launch_masks_setup(RunDev* dst, const RunDev& rec, bool table, hipStream_t s) {
  hipLaunchKernelGGL(k_masks_setup, dim3(1), dim3(256), 0, s, rec, dst, table ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_masks(const RunDev* runs, const RunDev& h, int run, uint32_t g, uint8_t* out,
                        hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((h.N + 3) / 4);
  if (h.xo == XO_EXP && h.exp_impl == EXPI_JOB) {
    hipLaunchKernelGGL(k_masks_job, dim3(static_cast<unsigned>((h.N + 63) / 64)), dim3(64), 0, s,
                       runs, run, g, out);
    return hipGetLastError();
  }
  switch (h.xo) {
    case XO_BIN: hipLaunchKernelGGL(k_masks<XO_BIN>, dim3(blocks), dim3(256), 0, s, runs, run, g, out); break;
    case XO_EXP: hipLaunchKernelGGL(k_masks<XO_EXP>, dim3(blocks), dim3(256), 0, s, runs, run, g, out); break;
    case XO_NEC: hipLaunchKernelGGL(k_masks<XO_NEC>, dim3(blocks), dim3(256), 0, s, runs, run, g, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace de
