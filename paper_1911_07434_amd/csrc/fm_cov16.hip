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
// native vectors: a struct copy (HIP's float4) would go through a generic
// reference and turn the global loads into flat ones
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef FM_GLOBAL const f32x4 gf32x4;
typedef FM_GLOBAL const f32x2 gf32x2;
typedef FM_GLOBAL const char gbyte;

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

// The frame fields the tile needs, copied out of the descriptor once (a
// reference into the descriptor array would be re-read after every store).
struct Src {
  const float2 *X;
  long long ldx;
  int M, T;
};

// Global -> registers for one stage: 128 rows x 32 complex snapshots of one
// operand = 2048 float4 (two snapshots each), 8 per thread: rows
// row0 + (tid >> 4) + 16 j, snapshots t0 + 2 (tid & 15) + {0, 1}.  Without
// kClamp (all 128 rows exist) the thread's address is a 32-bit byte offset
// `off` fixed for the tile, added to a uniform base that advances by 16 rows
// per load: no vector address arithmetic per load.  With kClamp (the last
// row tile of a frame) rows past M are clamped to row M-1 and each address
// is computed.
template <bool kClamp>
__device__ __forceinline__ gbyte *row_addr(const Src &x, int row0, unsigned off, int j, int t0) {
  if constexpr (!kClamp) {
    return (gbyte *)(x.X + t0 + (long long)16 * j * x.ldx) + off;
  } else {
    const int row = min(row0 + (int)(threadIdx.x >> 4) + 16 * j, x.M - 1);
    return (gbyte *)(x.X + (long long)row * x.ldx + t0 + 2 * (int)(threadIdx.x & 15));
  }
}

template <bool kClamp>
__device__ __forceinline__ void stage_load(f32x4 (&v)[8], const Src &x, int row0, unsigned off,
                                           int t0) {
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = *(gf32x4 *)row_addr<kClamp>(x, row0, off, j, t0);
}

// the last, ragged stage: snapshots past T read as zero
template <bool kClamp>
__device__ __forceinline__ void stage_load_tail(f32x4 (&v)[8], const Src &x, int row0,
                                                unsigned off, int t0) {
  const int tp = t0 + 2 * (int)(threadIdx.x & 15);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    v[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (tp + 1 < x.T) {
      v[j] = *(gf32x4 *)row_addr<kClamp>(x, row0, off, j, t0);
    } else if (tp < x.T) {
      const f32x2 y = *(gf32x2 *)row_addr<kClamp>(x, row0, off, j, t0);
      v[j].x = y.x;
      v[j].y = y.y;
    }
  }
}

// registers -> LDS, converted to 16 bits (one 8-byte store per float4)
template <class H>
__device__ __forceinline__ void stage_store(const f32x4 (&v)[8], H *lds, int base) {
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

template <class H, bool kClamp>
__device__ __forceinline__ void cov16_tile(const FrameDev &f, const Src &x, int ti, int tj,
                                           H *lds) {
  typedef typename Mma<H>::vec vec;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int T = x.T;
  const int r = lane & 31, h = lane >> 5;
  const bool diag = ti == tj;
  // the upper 64x64 block of a diagonal tile mirrors the lower one: that wave
  // still loads and synchronises, but skips its MFMAs and stores
  const bool active = !(diag && wi < wj);
  const int ra = ti * kCovTile, rb = tj * kCovTile;
  // LDS offsets (in halves): [buffer][A|B][128 rows][kRowHalves]; a diagonal
  // tile reads B from A's buffer
  const int offB = diag ? 0 : kTileHalves;
  const unsigned lane_off = (unsigned)(((long long)(threadIdx.x >> 4) * x.ldx +
                                        2 * (int)(threadIdx.x & 15)) * 8);
  const unsigned oa = (unsigned)((long long)ra * x.ldx * 8) + lane_off;
  const unsigned ob = (unsigned)((long long)rb * x.ldx * 8) + lane_off;

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

  const int nfull = T / kBK;
  const bool tail = nfull * kBK < T;
  const int rowA = (wi * 64 + r) * kRowHalves + 8 * h;
  const int rowB = (wj * 64 + r) * kRowHalves + 8 * h;
  // MFMAs of one stage held in LDS buffer `buf`
  auto compute = [&](int buf) {
    if (!active) return;
    const int cur = buf * 2 * kTileHalves;
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
  };
  auto store = [&](const f32x4 (&pa)[8], const f32x4 (&pb)[8], int buf) {
    stage_store<H>(pa, lds, buf * 2 * kTileHalves);
    if (!diag) stage_store<H>(pb, lds, buf * 2 * kTileHalves + kTileHalves);
  };
  f32x4 va[8], vb[8];
  if (nfull == 0) {
    // fewer than kBK snapshots: one ragged stage
    stage_load_tail<kClamp>(va, x, ra, oa, 0);
    if (!diag) stage_load_tail<kClamp>(vb, x, rb, ob, 0);
    store(va, vb, 0);
    __syncthreads();
    compute(0);
  } else {
    stage_load<kClamp>(va, x, ra, oa, 0);
    if (!diag) stage_load<kClamp>(vb, x, rb, ob, 0);
    store(va, vb, 0);
    __syncthreads();
    // full stages: the next stage's loads are in flight during this stage's
    // MFMAs; one barrier per stage publishes the next buffer
    for (int st = 0; st + 1 < nfull; ++st) {
      stage_load<kClamp>(va, x, ra, oa, (st + 1) * kBK);
      if (!diag) stage_load<kClamp>(vb, x, rb, ob, (st + 1) * kBK);
      compute(st & 1);
      store(va, vb, (st + 1) & 1);
      __syncthreads();
    }
    if (tail) {
      stage_load_tail<kClamp>(va, x, ra, oa, nfull * kBK);
      if (!diag) stage_load_tail<kClamp>(vb, x, rb, ob, nfull * kBK);
    }
    compute((nfull - 1) & 1);
    if (tail) {
      store(va, vb, nfull & 1);
      __syncthreads();
      compute(nfull & 1);
    }
  }
  if (!active) return;
  const int M = x.M;
  float2 *R = f.R;
  const long long ldr = f.ldr;

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
        *(FM_GLOBAL f32x2 *)(R + (size_t)i * ldr + j) = f32x2{re, im};
        if (i != j) *(FM_GLOBAL f32x2 *)(R + (size_t)j * ldr + i) = f32x2{re, -im};
      }
}

// two workgroups per CU (two waves per SIMD) hide the load latency: the
// register budget is capped so the occupancy cannot fall to one
template <class H, bool kBatched>
__global__ __launch_bounds__(256, 2) void cov16_kernel(FrameDev single,
                                                       const FrameDev *__restrict__ frames,
                                                       const Item *__restrict__ items) {
  __shared__ __attribute__((aligned(16))) H lds[4 * kTileHalves];
  int ti, tj;
  const FrameDev *fp;
  if constexpr (kBatched) {
    const Item it = items[blockIdx.x];
    fp = &frames[it.frame];
    ti = it.a;
    tj = it.b;
  } else {
    fp = &single;
    tile_of(blockIdx.x, ti, tj);
  }
  const Src x{fp->X, fp->ldx, fp->M, fp->T};
  // only the last row tile of a frame has rows past M (tj <= ti)
  if ((ti + 1) * kCovTile > x.M) cov16_tile<H, true>(*fp, x, ti, tj, lds);
  else cov16_tile<H, false>(*fp, x, ti, tj, lds);
}

}  // namespace

hipError_t launch_covariance16(const FrameDev &single, const FrameDev *frames, const Item *items,
                               int n_items, fm_prec prec, hipStream_t s) {
  const dim3 g(items ? n_items : cov_units(single.M, prec)), b(256);
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
