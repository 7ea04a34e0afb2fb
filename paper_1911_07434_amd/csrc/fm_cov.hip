// fm_cov.hip -- stage 1: sample covariance R = X X^H / T (eqs. (2)-(3)).
//
// Complex Hermitian rank-T update on the FP32 matrix cores of gfx950.  The
// complex product is written as real products (re/im of each snapshot are
// separate MFMA operands):
//   Re R_ij = sum_t xr_i xr_j + xi_i xi_j
//   Im R_ij = sum_t xi_i xr_j - xr_i xi_j
// so each 32x32 complex block costs four v_mfma_f32_32x32x2_f32 per pair of
// snapshots.  One wave (a one-wave workgroup) owns a 64x64 block of the lower
// triangle; it stores R_ij and, mirrored, conj(R_ij) at (j, i), so R is
// exactly Hermitian and its diagonal exactly real.  Blocks on the diagonal
// skip their 32x32 quarter above it.  Operands stream from global memory
// straight into MFMA registers (each lane owns a run of 4 consecutive
// snapshots of one channel), three chunks of snapshots in flight per wave.
#include "fm_internal.h"

namespace fm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ inline void block_of(int b, int &ti, int &tj) {
  // b enumerates the lower triangle row by row: (0,0), (1,0), (1,1), (2,0) ...
  int t = (int)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
  while ((t + 1) * (t + 2) / 2 <= b) ++t;
  while (t * (t + 1) / 2 > b) --t;
  ti = t;
  tj = b - t * (t + 1) / 2;
}

// One wave: a 64x64 complex block = 2x2 MFMA blocks of 32x32, each with an
// accumulator for the real and for the imaginary part.
struct CovAcc {
  floatx16 re[2][2];
  floatx16 im[2][2];
};

// kSkip01: the wave's 64x64 block straddles the diagonal of R, so its upper
// 32x32 block (rows 0-31, columns 32-63) lies above the diagonal and is never
// stored; its products are skipped.
template <bool kSkip01>
__device__ __forceinline__ void cov_step(CovAcc &acc, const float2 (&a)[2][4],
                                         const float2 (&b)[2][4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        if (kSkip01 && bi == 0 && bj == 1) continue;
        acc.re[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bi][s].x, b[bj][s].x,
                                                              acc.re[bi][bj], 0, 0, 0);
        acc.im[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bi][s].y, b[bj][s].x,
                                                              acc.im[bi][bj], 0, 0, 0);
      }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        if (kSkip01 && bi == 0 && bj == 1) continue;
        acc.re[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bi][s].y, b[bj][s].y,
                                                              acc.re[bi][bj], 0, 0, 0);
        acc.im[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[bi][s].x, b[bj][s].y,
                                                              acc.im[bi][bj], 0, 0, 0);
      }
  }
}

// global-address-space view of a frame pointer (FrameDev holds generic
// pointers; global loads avoid the flat path's shared counters)
typedef FM_GLOBAL const float2 gfloat2;

__device__ __forceinline__ void load8(float2 (&a)[2][4], float2 (&b)[2][4],
                                      const gfloat2 *const (&pa)[2],
                                      const gfloat2 *const (&pb)[2], int t) {
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a[q][s] = pa[q][t + s];
      b[q][s] = pb[q][t + s];
    }
}

// All full chunks of 8 snapshots, three register buffers in rotation: the
// loads of chunk c + 2 are in flight while chunk c feeds the matrix cores.
// Prefetch addresses are clamped to the last full chunk, so every load is
// valid and no register copies are needed.
template <bool kSkip01>
__device__ __forceinline__ void full_chunks(CovAcc &acc, const gfloat2 *const (&pa)[2],
                                            const gfloat2 *const (&pb)[2], int nfull) {
  const int tlast = (nfull - 1) * 8;
  float2 a0[2][4], b0[2][4], a1[2][4], b1[2][4], a2[2][4], b2[2][4];
  load8(a0, b0, pa, pb, 0);
  load8(a1, b1, pa, pb, min(8, tlast));
  for (int c = 0; c < nfull; c += 3) {
    load8(a2, b2, pa, pb, min((c + 2) * 8, tlast));
    cov_step<kSkip01>(acc, a0, b0);
    load8(a0, b0, pa, pb, min((c + 3) * 8, tlast));
    if (c + 1 < nfull) cov_step<kSkip01>(acc, a1, b1);
    load8(a1, b1, pa, pb, min((c + 4) * 8, tlast));
    if (c + 2 < nfull) cov_step<kSkip01>(acc, a2, b2);
  }
}

// one wave: the 64x64 block of R with block row bi and block column bj <= bi
__device__ __forceinline__ void cov_block(const FrameDev &f, int bi, int bj) {
  const int lane = threadIdx.x & 63;
  const bool diag = bi == bj;
  const int M = f.M, T = f.T;
  const int r = lane & 31, h = lane >> 5;
  const int ib = bi * kCovBlock;
  const int jb = bj * kCovBlock;
  // rows past M are clamped to a valid row: they only feed outputs that are
  // never stored
  const gfloat2 *pa[2], *pb[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int ia = min(ib + 32 * q + r, M - 1);
    const int ja = min(jb + 32 * q + r, M - 1);
    pa[q] = (const gfloat2 *)(f.X + (size_t)ia * f.ldx + 4 * h);
    pb[q] = (const gfloat2 *)(f.X + (size_t)ja * f.ldx + 4 * h);
  }
  CovAcc acc;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc.re[bi][bj][v] = 0.f;
        acc.im[bi][bj][v] = 0.f;
      }

  const int nfull = T >> 3;
  if (nfull > 0) {
    // (the count is passed through an empty asm so the loop is compiled
    // without the guard's knowledge that it runs at least once, which keeps
    // the kernel at two waves per SIMD)
    int n = nfull;
    __asm__ volatile("" : "+s"(n));
    if (diag) full_chunks<true>(acc, pa, pb, n);
    else full_chunks<false>(acc, pa, pb, n);
  }
  const int Tfull = nfull * 8;
  if (Tfull < T) {
    // ragged tail: snapshots past T contribute zero
    float2 a[2][4], b[2][4];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool ok = (Tfull + 4 * h + s) < T;
        a[q][s] = make_float2(0.f, 0.f);
        b[q][s] = make_float2(0.f, 0.f);
        if (ok) {
          a[q][s] = pa[q][Tfull + s];
          b[q][s] = pb[q][Tfull + s];
        }
      }
    cov_step<false>(acc, a, b);  // (a diagonal block's unused quarter is computed, not stored)
  }

  // epilogue: scale by 1/T after accumulation (correctly rounded divide),
  // store the lower triangle and its conjugate mirror
  const float Tf = (float)T;
  float2 *const R = f.R;
  const long long ldr = f.ldr;
  if (!diag && ib + kCovBlock <= M && ((uintptr_t)R & 15) == 0 && (ldr & 1) == 0) {
    // interior block strictly below the diagonal: the mirror of a lane's four
    // consecutive rows is a run of four entries of row j, stored as 32 bytes
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int i0 = ib + 32 * bi + 8 * g + 4 * h;
          const int j = jb + 32 * bj + r;
          float re[4], im[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            re[u] = acc.re[bi][bj][4 * g + u] / Tf;
            im[u] = acc.im[bi][bj][4 * g + u] / Tf;
            R[(size_t)(i0 + u) * ldr + j] = make_float2(re[u], im[u]);
          }
          float4 *m = (float4 *)(R + (size_t)j * ldr + i0);
          m[0] = make_float4(re[0], -im[0], re[1], -im[1]);
          m[1] = make_float4(re[2], -im[2], re[3], -im[3]);
        }
    return;
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = ib + 32 * bi + (v >> 2) * 8 + h * 4 + (v & 3);
        const int j = jb + 32 * bj + r;
        if (i >= M || j >= M || i < j) continue;
        const float re = acc.re[bi][bj][v] / Tf;
        const float im = (i == j) ? 0.f : acc.im[bi][bj][v] / Tf;
        R[(size_t)i * ldr + j] = make_float2(re, im);
        if (i != j) R[(size_t)j * ldr + i] = make_float2(re, -im);
      }
}

template <bool kBatched>
__global__ __launch_bounds__(64, 2) void cov_fp32_kernel(FrameDev single,
                                                      const FrameDev *__restrict__ frames,
                                                      const Item *__restrict__ items) {
  if constexpr (kBatched) {
    const Item it = items[blockIdx.x];
    const FrameDev f = frames[it.frame];
    cov_block(f, it.a, it.b);
  } else {
    int bi, bj;
    block_of(blockIdx.x, bi, bj);
    cov_block(single, bi, bj);
  }
}

}  // namespace

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
