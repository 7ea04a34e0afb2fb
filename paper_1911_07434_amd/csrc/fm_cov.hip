// fm_cov.hip -- stage 1: sample covariance R = X X^H / T (eqs. (2)-(3)).
//
// Complex Hermitian rank-T update on the FP32 matrix cores of gfx950, with
// Gauss's three-product form of the complex product.  For one snapshot of
// channels i and j, x_i = a + ib and x_j = c + id:
//   k1 = (a + b) c,   k2 = a (c + d),   k3 = b (c - d)
//   Re x_i conj(x_j) = ac + bd = k1 - k3,   Im x_i conj(x_j) = bc - ad = k1 - k2
// so a 32x32 complex block costs three v_mfma_f32_32x32x2_f32 per pair of
// snapshots instead of four (the sums a + b, c + d, c - d are rounded to
// FP32 once per snapshot: the error stays at FP32 level, a small constant
// above the four-product form's).  One wave (a one-wave workgroup) owns a
// 64x32 block of the lower triangle, two 32x32 blocks stacked, with three
// accumulators each (96 registers, so two waves share a SIMD); it stores
// R_ij and, mirrored, conj(R_ij) at (j, i), so R is exactly Hermitian and its
// diagonal exactly real.  Blocks on the diagonal skip their 32x32 block above
// it.  Operands stream from global memory straight into MFMA registers (each
// lane owns a run of 4 consecutive snapshots of one channel), three chunks of
// snapshots in flight per wave.
#include "fm_internal.h"

namespace fm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Work unit u of a frame -> wave block (bi, bj): 64-row block bi holds the
// units bi (bi + 1) .. (bi + 1)(bi + 2) - 1, bj = 0 .. 2 bi + 1.
__device__ inline void block_of(int u, int &bi, int &bj) {
  int t = (int)((sqrtf(4.0f * (float)u + 1.0f) - 1.0f) * 0.5f);
  while ((t + 1) * (t + 2) <= u) ++t;
  while (t * (t + 1) > u) --t;
  bi = t;
  bj = u - t * (t + 1);
}

// One wave: a 64x32 complex block = two 32x32 MFMA blocks (q = 0, 1 stacked
// in rows), each with the three Gauss accumulators.
struct CovAcc {
  floatx16 k1[2], k2[2], k3[2];
};

// kSkip0: the wave's block is the second of its block row that touches the
// diagonal; its upper 32x32 block (q = 0) lies above the diagonal and is
// never stored, so its products are skipped.
template <bool kSkip0>
__device__ __forceinline__ void cov_step(CovAcc &acc, const float2 (&a)[2][4],
                                         const float2 (&b)[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float p = b[s].x + b[s].y;   // c + d
    const float m = b[s].x - b[s].y;   // c - d
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (kSkip0 && q == 0) continue;
      const float sa = a[q][s].x + a[q][s].y;   // a + b
      acc.k1[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(sa, b[s].x, acc.k1[q], 0, 0, 0);
      acc.k2[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q][s].x, p, acc.k2[q], 0, 0, 0);
      acc.k3[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q][s].y, m, acc.k3[q], 0, 0, 0);
    }
  }
}

// global-address-space view of a frame pointer (FrameDev holds generic
// pointers; global loads avoid the flat path's shared counters)
typedef FM_GLOBAL const float2 gfloat2;

__device__ __forceinline__ void load8(float2 (&a)[2][4], float2 (&b)[4],
                                      const gfloat2 *const (&pa)[2], const gfloat2 *pb, int t) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
#pragma unroll
    for (int q = 0; q < 2; ++q) a[q][s] = pa[q][t + s];
    b[s] = pb[t + s];
  }
}

// The wave's (Re, Im) sums over T, value 32 q + v (Re) and 32 q + 16 + v
// (Im) of MFMA block q's accumulator element v
struct CovSum {
  float v[64];
};

// a segment's Re = k1 - k3, Im = k1 - k2 added to the sums, the
// accumulators cleared for the next segment (sums in registers, or in the
// wave's LDS array: value k of lane l at k * 64 + l)
__device__ __forceinline__ void cov_fold(CovAcc &acc, CovSum &sum) {
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      sum.v[32 * q + v] += acc.k1[q][v] - acc.k3[q][v];
      sum.v[32 * q + 16 + v] += acc.k1[q][v] - acc.k2[q][v];
      acc.k1[q][v] = 0.f;
      acc.k2[q][v] = 0.f;
      acc.k3[q][v] = 0.f;
    }
}
__device__ __forceinline__ void cov_fold(CovAcc &acc, float *lsum, int lane) {
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      lsum[(32 * q + v) * 64 + lane] += acc.k1[q][v] - acc.k3[q][v];
      lsum[(32 * q + 16 + v) * 64 + lane] += acc.k1[q][v] - acc.k2[q][v];
      acc.k1[q][v] = 0.f;
      acc.k2[q][v] = 0.f;
      acc.k3[q][v] = 0.f;
    }
}

// All full chunks of 8 snapshots, three register buffers in rotation: the
// loads of chunk c + 2 are in flight while chunk c feeds the matrix cores.
// Prefetch addresses are clamped to the last full chunk, so every load is
// valid and no register copies are needed.
template <bool kSkip0>
__device__ __forceinline__ void full_chunks(CovAcc &acc, const gfloat2 *const (&pa)[2],
                                            const gfloat2 *pb, int nfull) {
  const int tlast = (nfull - 1) * 8;
  float2 a0[2][4], b0[4], a1[2][4], b1[4], a2[2][4], b2[4];
  load8(a0, b0, pa, pb, 0);
  load8(a1, b1, pa, pb, min(8, tlast));
  for (int c = 0; c < nfull; c += 3) {
    load8(a2, b2, pa, pb, min((c + 2) * 8, tlast));
    cov_step<kSkip0>(acc, a0, b0);
    load8(a0, b0, pa, pb, min((c + 3) * 8, tlast));
    if (c + 1 < nfull) cov_step<kSkip0>(acc, a1, b1);
    load8(a1, b1, pa, pb, min((c + 4) * 8, tlast));
    if (c + 2 < nfull) cov_step<kSkip0>(acc, a2, b2);
  }
}

// All full chunks of a wave running every T segment in turn: the same
// three-buffer rotation as full_chunks, continuous across segments, with the
// accumulators folded into the sums where a segment starts.
template <bool kSkip0>
__device__ __forceinline__ void full_chunks_seq(CovAcc &acc, float *lsum, int lane,
                                                const gfloat2 *const (&pa)[2], const gfloat2 *pb,
                                                int nfull, int G) {
  const int tlast = (nfull - 1) * 8;
  float2 a0[2][4], b0[4], a1[2][4], b1[4], a2[2][4], b2[4];
  int seg = 1, next = cov_seg_chunk(1, G, nfull);
  auto step = [&](int c, const float2 (&a)[2][4], const float2 (&b)[4]) {
    if (c == next) {
      cov_fold(acc, lsum, lane);
      ++seg;
      next = cov_seg_chunk(seg, G, nfull);
    }
    cov_step<kSkip0>(acc, a, b);
  };
  load8(a0, b0, pa, pb, 0);
  load8(a1, b1, pa, pb, min(8, tlast));
  for (int c = 0; c < nfull; c += 3) {
    load8(a2, b2, pa, pb, min((c + 2) * 8, tlast));
    step(c, a0, b0);
    load8(a0, b0, pa, pb, min((c + 3) * 8, tlast));
    if (c + 1 < nfull) step(c + 1, a1, b1);
    load8(a1, b1, pa, pb, min((c + 4) * 8, tlast));
    if (c + 2 < nfull) step(c + 2, a2, b2);
  }
}

// The ragged chunk past the last full one (snapshots past T contribute
// zero); nothing when 8 divides T
__device__ __forceinline__ void cov_tail(CovAcc &acc, const gfloat2 *const (&pa0)[2],
                                         const gfloat2 *pb0, int T, int h) {
  const int Tfull = (T >> 3) * 8;
  if (Tfull >= T) return;
  float2 a[2][4], b[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const bool ok = (Tfull + 4 * h + s) < T;
#pragma unroll
    for (int q = 0; q < 2; ++q) a[q][s] = make_float2(0.f, 0.f);
    b[s] = make_float2(0.f, 0.f);
    if (ok) {
#pragma unroll
      for (int q = 0; q < 2; ++q) a[q][s] = pa0[q][Tfull + s];
      b[s] = pb0[Tfull + s];
    }
  }
  cov_step<false>(acc, a, b);  // (a skipped block is computed here, not stored)
}

// One T segment of the wave's block: chunks [c0, c1) of 8 snapshots, plus the
// ragged tail past the last full chunk when `tail`; the Gauss accumulators
// start from zero and the segment's Re = k1 - k3, Im = k1 - k2 are added to
// `sum` (0 + x = x, so a first segment is stored as computed).
__device__ __forceinline__ void cov_segment(CovSum &sum, const gfloat2 *const (&pa0)[2],
                                            const gfloat2 *pb0, int c0, int c1, bool skip0,
                                            bool tail, int T, int h) {
  CovAcc acc;
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      acc.k1[q][v] = 0.f;
      acc.k2[q][v] = 0.f;
      acc.k3[q][v] = 0.f;
    }
  if (c1 > c0) {
    const gfloat2 *const pa[2] = {pa0[0] + 8 * c0, pa0[1] + 8 * c0};
    const gfloat2 *pb = pb0 + 8 * c0;
    // (the count is passed through an empty asm so the loop is compiled
    // without the guard's knowledge that it runs at least once)
    int n = c1 - c0;
    __asm__ volatile("" : "+s"(n));
    if (skip0) full_chunks<true>(acc, pa, pb, n);
    else full_chunks<false>(acc, pa, pb, n);
  }
  if (tail) cov_tail(acc, pa0, pb0, T, h);
  cov_fold(acc, sum);
}

// Operand rows of the wave's block (rows past M are clamped to a valid row:
// they only feed outputs that are never stored)
struct CovRows {
  const gfloat2 *pa[2];
  const gfloat2 *pb;
};
__device__ __forceinline__ CovRows cov_rows(const FrameDev &f, int ib, int jb, int r, int h) {
  CovRows c;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int ia = min(ib + 32 * q + r, f.M - 1);
    c.pa[q] = (const gfloat2 *)(f.X + (size_t)ia * f.ldx + 4 * h);
  }
  c.pb = (const gfloat2 *)(f.X + (size_t)min(jb + r, f.M - 1) * f.ldx + 4 * h);
  return c;
}

// R = sum / T on the wave's block: the lower triangle and its conjugate
// mirror (the diagonal's imaginary part is exactly zero); correctly rounded
// divide
__device__ __forceinline__ void cov_store(const FrameDev &f, const CovSum &sum, int ib, int jb,
                                          bool diag, int r, int h) {
  const int M = f.M;
  const float Tf = (float)f.T;
  float2 *const R = f.R;
  const long long ldr = f.ldr;
  if (!diag && ib + kCovBlock <= M && ((uintptr_t)R & 15) == 0 && (ldr & 1) == 0) {
    // interior block strictly below the diagonal: the mirror of a lane's four
    // consecutive rows is a run of four entries of row j, stored as 32 bytes
    const int j = jb + r;
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int i0 = ib + 32 * q + 8 * g + 4 * h;
        float re[4], im[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int v = 4 * g + u;
          re[u] = sum.v[32 * q + v] / Tf;
          im[u] = sum.v[32 * q + 16 + v] / Tf;
          R[(size_t)(i0 + u) * ldr + j] = make_float2(re[u], im[u]);
        }
        float4 *mr = (float4 *)(R + (size_t)j * ldr + i0);
        mr[0] = make_float4(re[0], -im[0], re[1], -im[1]);
        mr[1] = make_float4(re[2], -im[2], re[3], -im[3]);
      }
    return;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = ib + 32 * q + (v >> 2) * 8 + h * 4 + (v & 3);
      const int j = jb + r;
      if (i >= M || j >= M || i < j) continue;
      const float re = sum.v[32 * q + v] / Tf;
      const float im = (i == j) ? 0.f : sum.v[32 * q + 16 + v] / Tf;
      R[(size_t)i * ldr + j] = make_float2(re, im);
      if (i != j) R[(size_t)j * ldr + i] = make_float2(re, -im);
    }
}

enum CovMode { kCovSeq = 0, kCovPart = 1, kCovReduce = 2 };

// one wave: the 64x32 block of R with rows 64 bi .., columns 32 bj ..
// (bj <= 2 bi + 1).  kCovSeq: every T segment in turn, then R; kCovPart:
// segment g's sums into cpart; kCovReduce: R from the segments' sums in
// segment order.
template <int kMode>
__device__ __forceinline__ void cov_block(const FrameDev &f, int bi, int bj, int g,
                                          float *lsum = nullptr) {
  const int lane = threadIdx.x & 63;
  const int M = f.M, T = f.T;
  const int r = lane & 31, h = lane >> 5;
  const int ib = bi * kCovBlock;
  const int jb = bj * kCovCols;
  if (jb >= M) return;  // (single-frame launches cover whole block rows)
  // bj == 2 bi: the block's upper 32x32 block is on the diagonal;
  // bj == 2 bi + 1: its upper block is above the diagonal (skipped), its
  // lower block on it
  const bool diag = bj >= 2 * bi;
  const bool skip0 = bj == 2 * bi + 1;
  const int G = cov_segments(M, T), nfull = T >> 3;
  FM_GLOBAL float *part =
      (FM_GLOBAL float *)f.cpart + (size_t)cov_unit_index(bi, bj) * G * kCovPartFloats + lane;
  CovSum sum;
#pragma unroll
  for (int k = 0; k < 64; ++k) sum.v[k] = 0.f;
  if constexpr (kMode == kCovReduce) {
    for (int s = 0; s < G; ++s) {
      // (all of a segment's loads issued before its adds)
      const FM_GLOBAL float *ps = part + (size_t)s * kCovPartFloats;
      float t[64];
#pragma unroll
      for (int k = 0; k < 64; ++k) t[k] = __builtin_nontemporal_load(ps + 64 * k);
#pragma unroll
      for (int k = 0; k < 64; ++k) sum.v[k] += t[k];
    }
  } else {
    const CovRows c = cov_rows(f, ib, jb, r, h);
    if constexpr (kMode == kCovSeq) {
      CovAcc acc;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          acc.k1[q][v] = 0.f;
          acc.k2[q][v] = 0.f;
          acc.k3[q][v] = 0.f;
        }
      // the sums stay in LDS while the segments run (registers hold the
      // accumulators and three chunks of operands)
#pragma unroll
      for (int k = 0; k < 64; ++k) lsum[k * 64 + lane] = 0.f;
      if (nfull > 0) {
        int n = nfull;
        __asm__ volatile("" : "+s"(n));
        if (skip0) full_chunks_seq<true>(acc, lsum, lane, c.pa, c.pb, n, G);
        else full_chunks_seq<false>(acc, lsum, lane, c.pa, c.pb, n, G);
      }
      // the last segment: the ragged tail, then its fold
      cov_tail(acc, c.pa, c.pb, T, h);
      cov_fold(acc, lsum, lane);
#pragma unroll
      for (int k = 0; k < 64; ++k) sum.v[k] = lsum[k * 64 + lane];
    } else {
      cov_segment(sum, c.pa, c.pb, cov_seg_chunk(g, G, nfull), cov_seg_chunk(g + 1, G, nfull),
                  skip0, g == G - 1, T, h);
      FM_GLOBAL float *ps = part + (size_t)g * kCovPartFloats;
#pragma unroll
      for (int k = 0; k < 64; ++k) ps[64 * k] = sum.v[k];
      return;
    }
  }
  cov_store(f, sum, ib, jb, diag, r, h);
}

template <bool kBatched>
__global__ __launch_bounds__(64, 2) void cov_fp32_kernel(FrameDev single,
                                                      const FrameDev *__restrict__ frames,
                                                      const Item *__restrict__ items) {
  __shared__ float lsum[64 * 64];
  if constexpr (kBatched) {
    const Item it = items[blockIdx.x];
    const FrameDev f = frames[it.frame];
    cov_block<kCovSeq>(f, it.a, it.b, 0, lsum);
  } else {
    int bi, bj;
    block_of(blockIdx.x, bi, bj);
    cov_block<kCovSeq>(single, bi, bj, 0, lsum);
  }
}

// T segments on separate waves (kMode kCovPart) and their in-order
// reduction (kCovReduce); a single frame's launch is units x segments, then
// units
template <int kMode, bool kBatched>
__global__ __launch_bounds__(64, 2) void cov_split_kernel(FrameDev single,
                                                       const FrameDev *__restrict__ frames,
                                                       const Item *__restrict__ items) {
  if constexpr (kBatched) {
    const Item it = items[blockIdx.x];
    const FrameDev f = frames[it.frame];
    cov_block<kMode>(f, it.a, it.b, it.c);
  } else {
    const int G = kMode == kCovPart ? cov_segments(single.M, single.T) : 1;
    int bi, bj;
    block_of(blockIdx.x / G, bi, bj);
    cov_block<kMode>(single, bi, bj, blockIdx.x % G);
  }
}

}  // namespace

hipError_t launch_covariance_split(const FrameDev &single, const FrameDev *frames,
                                   const Item *items, int n_items, int mode, hipStream_t s) {
  if (items) {
    if (n_items <= 0) return hipSuccess;
    if (mode == 0)
      hipLaunchKernelGGL((cov_split_kernel<kCovPart, true>), dim3(n_items), dim3(64), 0, s, single,
                         frames, items);
    else
      hipLaunchKernelGGL((cov_split_kernel<kCovReduce, true>), dim3(n_items), dim3(64), 0, s,
                         single, frames, items);
  } else {
    const int units = cov_units(single.M, FM_FP32);
    if (mode == 0)
      hipLaunchKernelGGL((cov_split_kernel<kCovPart, false>),
                         dim3(units * cov_segments(single.M, single.T)), dim3(64), 0, s, single, frames,
                         items);
    else
      hipLaunchKernelGGL((cov_split_kernel<kCovReduce, false>), dim3(units), dim3(64), 0, s,
                         single, frames, items);
  }
  return hipGetLastError();
}

hipError_t launch_covariance(const FrameDev &single, const FrameDev *frames, const Item *items,
                             int n_items, fm_prec prec, hipStream_t s) {
  if (prec != FM_FP32) return launch_covariance16(single, frames, items, n_items, prec, s);
  if (items) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(cov_fp32_kernel<true>, dim3(n_items), dim3(64), 0, s, single, frames,
                       items);
  } else {
    hipLaunchKernelGGL(cov_fp32_kernel<false>, dim3(cov_units(single.M, FM_FP32)), dim3(64), 0, s,
                       single, frames, items);
  }
  return hipGetLastError();
}

}  // namespace fm
