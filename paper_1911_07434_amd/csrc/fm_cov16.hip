// fm_cov16.hip -- stage 1 with 16-bit operands: R = X X^H / T with the
// snapshots rounded to FP16 or BF16 and FP32 accumulation (eqs. (2)-(3)).
//
// v_mfma_f32_32x32x16_{f16,bf16}: K = 16 real values = 8 complex snapshots
// in the interleaved (re, im) order of X, so
//   Re R_ij = x^_i . x^_j          (x^ = the interleaved row)
//   Im R_ij = x'_i . x^_j,  x' = (im, -re) pairs of the row
// and a 32x32 complex block costs two MFMAs per 8 snapshots.  At the 16-bit
// matrix rate the operands must come from LDS: each workgroup stages its
// 128 A rows and 128 B rows, 32 snapshots at a time, converted to 16 bits
// on the way in, double buffered; rows are padded by 16 bytes so the
// 16-byte MFMA operand reads of 32 consecutive rows do not collide in a
// bank.  Diagonal tiles load their rows once.  Same lower-triangle tiling,
// mirrored store and 1/T epilogue as the FP32 kernel.
#include "fm_internal.h"

namespace fm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef FM_GLOBAL const float4 gfloat4;

constexpr int kBK = 32;                       // snapshots per stage
constexpr int kRowHalves = 2 * kBK + 8;       // 64 halves + 16 bytes of padding
constexpr int kTileHalves = kCovTile * kRowHalves;

template <class H>
struct Mma;
template <>
struct Mma<_Float16> {
  typedef f16x8 vec;
  __device__ static floatx16 run(vec a, vec b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<__bf16> {
  typedef bf16x8 vec;
  __device__ static floatx16 run(vec a, vec b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

__device__ inline void tile_of(int b, int &ti, int &tj) {
  int t = (int)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
  while ((t + 1) * (t + 2) / 2 <= b) ++t;
  while (t * (t + 1) / 2 > b) --t;
  ti = t;
  tj = b - t * (t + 1) / 2;
}

// Global -> registers for one stage: 128 rows x 32 complex snapshots of one
// operand = 2048 float4 (two snapshots each); 8 per thread.  Full stages take
// the unconditional path; only the last, ragged stage checks T.
__device__ __forceinline__ void stage_load(float4 (&v)[8], const FrameDev &f, int row0, int t0) {
  const int M = f.M, T = f.T;
  const int tsub = 2 * (threadIdx.x & 15);
  if (t0 + kBK <= T) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int row = min(row0 + ((threadIdx.x >> 4) + 16 * j), M - 1);
      v[j] = *(const gfloat4 *)(f.X + (size_t)row * f.ldx + t0 + tsub);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int row = min(row0 + ((threadIdx.x >> 4) + 16 * j), M - 1);
      const int tp = t0 + tsub;
      const float2 *p = f.X + (size_t)row * f.ldx + tp;
      v[j] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (tp + 1 < T) {
        v[j] = *(const gfloat4 *)p;
      } else if (tp < T) {
        const float2 x = *(FM_GLOBAL const float2 *)p;
        v[j].x = x.x;
        v[j].y = x.y;
      }
    }
  }
}

// registers -> LDS, converted to 16 bits (one 8-byte store per float4)
template <class H>
__device__ __forceinline__ void stage_store(const float4 (&v)[8], H *lds, int base) {
  typedef H h4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int row = (threadIdx.x >> 4) + 16 * j;
    h4 w;
    w[0] = (H)v[j].x;
    w[1] = (H)v[j].y;
    w[2] = (H)v[j].z;
    w[3] = (H)v[j].w;
    *(h4 *)(lds + base + row * kRowHalves + 4 * (threadIdx.x & 15)) = w;
  }
}

template <class H>
__device__ __forceinline__ void cov16_tile(const FrameDev &f, int ti, int tj, H *lds) {
  typedef typename Mma<H>::vec vec;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int T = f.T;
  const int r = lane & 31, h = lane >> 5;
  const bool diag = ti == tj;
  // the upper 64x64 block of a diagonal tile mirrors the lower one: that wave
  // still loads and synchronises, but skips its MFMAs and stores
  const bool active = !(diag && wi < wj);
  const int ra = ti * kCovTile, rb = tj * kCovTile;
  // LDS offsets (in halves): [buffer][A|B][128 rows][kRowHalves]; a diagonal
  // tile reads B from A's buffer
  const int offB = diag ? 0 : kTileHalves;

  floatx16 accR[2][2], accI[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        accR[bi][bj][v] = 0.f;
        accI[bi][bj][v] = 0.f;
      }

  const int nst = (T + kBK - 1) / kBK;
  float4 va[8], vb[8];
  stage_load(va, f, ra, 0);
  if (!diag) stage_load(vb, f, rb, 0);
  stage_store<H>(va, lds, 0);
  if (!diag) stage_store<H>(vb, lds, kTileHalves);
  __syncthreads();
  const int rowA = (wi * 64 + r) * kRowHalves + 8 * h;
  const int rowB = (wj * 64 + r) * kRowHalves + 8 * h;
  for (int st = 0; st < nst; ++st) {
    const bool more = st + 1 < nst;
    if (more) {
      stage_load(va, f, ra, (st + 1) * kBK);
      if (!diag) stage_load(vb, f, rb, (st + 1) * kBK);
    }
    const int cur = (st & 1) * 2 * kTileHalves;
    if (active) {
#pragma unroll
      for (int ks = 0; ks < kBK / 8; ++ks) {
        vec a[2], ap[2], b[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          a[q] = *(const vec *)(lds + cur + rowA + 32 * q * kRowHalves + 16 * ks);
          b[q] = *(const vec *)(lds + cur + offB + rowB + 32 * q * kRowHalves + 16 * ks);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            ap[q][2 * c] = a[q][2 * c + 1];
            ap[q][2 * c + 1] = -a[q][2 * c];
          }
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            accR[bi][bj] = Mma<H>::run(a[bi], b[bj], accR[bi][bj]);
            accI[bi][bj] = Mma<H>::run(ap[bi], b[bj], accI[bi][bj]);
          }
      }
    }
    if (more) {
      const int nxt = ((st + 1) & 1) * 2 * kTileHalves;
      stage_store<H>(va, lds, nxt);
      if (!diag) stage_store<H>(vb, lds, nxt + kTileHalves);
    }
    __syncthreads();
  }
  if (!active) return;
  const int M = f.M;

  const int ib = ra + wi * 64, jb = rb + wj * 64;
  const float Tf = (float)T;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = ib + 32 * bi + (v >> 2) * 8 + h * 4 + (v & 3);
        const int j = jb + 32 * bj + r;
        if (i >= M || j >= M || i < j) continue;
        const float re = accR[bi][bj][v] / Tf;
        const float im = (i == j) ? 0.f : accI[bi][bj][v] / Tf;
        f.R[(size_t)i * f.ldr + j] = make_float2(re, im);
        if (i != j) f.R[(size_t)j * f.ldr + i] = make_float2(re, -im);
      }
}

template <class H, bool kBatched>
__global__ __launch_bounds__(256) void cov16_kernel(FrameDev single,
                                                    const FrameDev *__restrict__ frames,
                                                    const Item *__restrict__ items) {
  __shared__ __attribute__((aligned(16))) H lds[4 * kTileHalves];
  if constexpr (kBatched) {
    const Item it = items[blockIdx.x];
    cov16_tile<H>(frames[it.frame], it.a, it.b, lds);
  } else {
    int ti, tj;
    tile_of(blockIdx.x, ti, tj);
    cov16_tile<H>(single, ti, tj, lds);
  }
}

}  // namespace

hipError_t launch_covariance16(const FrameDev &single, const FrameDev *frames, const Item *items,
                               int n_items, fm_prec prec, hipStream_t s) {
  const dim3 g(items ? n_items : cov_tiles(single.M)), b(256);
  if (prec == FM_FP16) {
    if (items) hipLaunchKernelGGL((cov16_kernel<_Float16, true>), g, b, 0, s, single, frames, items);
    else hipLaunchKernelGGL((cov16_kernel<_Float16, false>), g, b, 0, s, single, frames, items);
  } else {
    if (items) hipLaunchKernelGGL((cov16_kernel<__bf16, true>), g, b, 0, s, single, frames, items);
    else hipLaunchKernelGGL((cov16_kernel<__bf16, false>), g, b, 0, s, single, frames, items);
  }
  return hipGetLastError();
}

}  // namespace fm
