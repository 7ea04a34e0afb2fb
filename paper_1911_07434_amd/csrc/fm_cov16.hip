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
//
// Split variant (kSplit, precisions FM_FP16X3 / FM_BF16X3): each snapshot is
// written as hi + lo with hi its 16-bit rounding and lo the 16-bit rounding
// of the remainder, and the block accumulates lo*hi + hi*lo + hi*hi (the
// lo*lo term is below FP32 rounding of the sum), six MFMAs per complex block
// per 8 snapshots.  The products are exact in FP32, so the result carries
// FP32-level error (FP16: 22 significant bits per operand, BF16: 16).  Both
// halves of a stage sit in LDS; stages hold 16 snapshots so two workgroups
// still share a CU's LDS.
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

// Stage geometry: kBK snapshots per stage, LDS rows of 2 kBK halves plus 16
// bytes of padding, a tile plane of 128 such rows; the split variant keeps
// a hi and a lo plane of each operand.
template <bool kSplit>
struct Geo {
  static constexpr int kBK = kSplit ? 16 : 32;
  static constexpr int kRowHalves = 2 * kBK + 8;
  static constexpr int kTileHalves = kCovTile * kRowHalves;
  static constexpr int kPlanes = kSplit ? 4 : 2;          // per buffer: A, B (hi, then lo)
  static constexpr int kTPR = kBK / 2;                    // threads per row (2 snapshots each)
  static constexpr int kRowsPerPass = 256 / kTPR;
  static constexpr int kLoads = kCovTile / kRowsPerPass;  // float4 loads per operand per stage
  static constexpr int kLdsHalves = 2 * kPlanes * kTileHalves;
};
static_assert(Geo<false>::kLdsHalves * 2 * 2 <= 160 * 1024, "two workgroups per CU");
static_assert(Geo<true>::kLdsHalves * 2 * 2 <= 160 * 1024, "two workgroups per CU");

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

// Global -> registers for one stage: 128 rows x kBK complex snapshots of one
// operand, as float4 (two snapshots each), kLoads per thread: rows
// row0 + tid / kTPR + kRowsPerPass j, snapshots t0 + 2 (tid % kTPR) + {0, 1}.
// Without kClamp (all 128 rows exist) the thread's address is a 32-bit byte
// offset `off` fixed for the tile, added to a uniform base that advances by
// kRowsPerPass rows per load: no vector address arithmetic per load.  With
// kClamp (the last row tile of a frame) rows past M are clamped to row M-1
// and each address is computed.
template <bool kSplit, bool kClamp>
__device__ __forceinline__ gbyte *row_addr(const Src &x, int row0, unsigned off, int j, int t0) {
  typedef Geo<kSplit> G;
  if constexpr (!kClamp) {
    return (gbyte *)(x.X + t0 + (long long)G::kRowsPerPass * j * x.ldx) + off;
  } else {
    const int row =
        min(row0 + (int)(threadIdx.x / G::kTPR) + G::kRowsPerPass * j, x.M - 1);
    return (gbyte *)(x.X + (long long)row * x.ldx + t0 + 2 * (int)(threadIdx.x % G::kTPR));
  }
}

template <bool kSplit, bool kClamp>
__device__ __forceinline__ void stage_load(f32x4 (&v)[Geo<kSplit>::kLoads], const Src &x, int row0,
                                           unsigned off, int t0) {
#pragma unroll
  for (int j = 0; j < Geo<kSplit>::kLoads; ++j)
    v[j] = *(gf32x4 *)row_addr<kSplit, kClamp>(x, row0, off, j, t0);
}

// the last, ragged stage: snapshots past T read as zero
template <bool kSplit, bool kClamp>
__device__ __forceinline__ void stage_load_tail(f32x4 (&v)[Geo<kSplit>::kLoads], const Src &x,
                                                int row0, unsigned off, int t0) {
  const int tp = t0 + 2 * (int)(threadIdx.x % Geo<kSplit>::kTPR);
#pragma unroll
  for (int j = 0; j < Geo<kSplit>::kLoads; ++j) {
    v[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (tp + 1 < x.T) {
      v[j] = *(gf32x4 *)row_addr<kSplit, kClamp>(x, row0, off, j, t0);
    } else if (tp < x.T) {
      const f32x2 y = *(gf32x2 *)row_addr<kSplit, kClamp>(x, row0, off, j, t0);
      v[j].x = y.x;
      v[j].y = y.y;
    }
  }
}

// registers -> LDS, converted to 16 bits (one 8-byte store per float4 and
// plane); the split variant also stores lo = 16-bit rounding of v - hi (the
// difference is exact in FP32) at `lo_off` halves past the hi plane
template <class H, bool kSplit>
__device__ __forceinline__ void stage_store(const f32x4 (&v)[Geo<kSplit>::kLoads], H *lds, int base,
                                            int lo_off) {
  typedef Geo<kSplit> G;
  typedef H h4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int j = 0; j < G::kLoads; ++j) {
    const int row = (int)(threadIdx.x / G::kTPR) + G::kRowsPerPass * j;
    const int at = base + row * G::kRowHalves + 4 * (int)(threadIdx.x % G::kTPR);
    h4 w;
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = (H)v[j][e];
    *(h4 *)(lds + at) = w;
    if constexpr (kSplit) {
      h4 lo;
#pragma unroll
      for (int e = 0; e < 4; ++e) lo[e] = (H)(v[j][e] - (float)w[e]);
      *(h4 *)(lds + at + lo_off) = lo;
    }
  }
}

template <class H, bool kSplit, bool kClamp>
__device__ __forceinline__ void cov16_tile(const FrameDev &f, const Src &x, int ti, int tj,
                                           H *lds) {
  typedef typename Mma<H>::vec vec;
  typedef Geo<kSplit> G;
  constexpr int kBK = G::kBK, kRowHalves = G::kRowHalves, kTileHalves = G::kTileHalves;
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
  // LDS offsets (in halves): [buffer][plane][128 rows][kRowHalves] with the
  // planes A, B (hi) and, split, A, B (lo); a diagonal tile reads B from A's
  // planes
  const int offB = diag ? 0 : kTileHalves;
  constexpr int kLo = 2 * kTileHalves;
  constexpr int kBuf = G::kPlanes * kTileHalves;
  const unsigned lane_off = (unsigned)(((long long)(threadIdx.x / G::kTPR) * x.ldx +
                                        2 * (int)(threadIdx.x % G::kTPR)) * 8);
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
  // (im, -re) pairs of an interleaved row segment
  auto swap_neg = [](vec a) {
    vec p;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      p[2 * c] = a[2 * c + 1];
      p[2 * c + 1] = -a[2 * c];
    }
    return p;
  };
  // MFMAs of one stage held in LDS buffer `buf`
  auto compute = [&](int buf) {
    if (!active) return;
    const int cur = buf * kBuf;
#pragma unroll
    for (int ks = 0; ks < kBK / 8; ++ks) {
      vec a[2], ap[2], b[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        a[q] = *(const vec *)(lds + cur + rowA + 32 * q * kRowHalves + 16 * ks);
        b[q] = *(const vec *)(lds + cur + offB + rowB + 32 * q * kRowHalves + 16 * ks);
        ap[q] = swap_neg(a[q]);
      }
      if constexpr (kSplit) {
        // lo*hi and hi*lo first (each round touches all eight accumulators,
        // so consecutive MFMAs are independent), then hi*hi
        vec al[2], apl[2], bl[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          al[q] = *(const vec *)(lds + cur + kLo + rowA + 32 * q * kRowHalves + 16 * ks);
          bl[q] = *(const vec *)(lds + cur + kLo + offB + rowB + 32 * q * kRowHalves + 16 * ks);
          apl[q] = swap_neg(al[q]);
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            accR[bi][bj] = Mma<H>::run(al[bi], b[bj], accR[bi][bj]);
            accI[bi][bj] = Mma<H>::run(apl[bi], b[bj], accI[bi][bj]);
          }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj) {
            accR[bi][bj] = Mma<H>::run(a[bi], bl[bj], accR[bi][bj]);
            accI[bi][bj] = Mma<H>::run(ap[bi], bl[bj], accI[bi][bj]);
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
  auto store = [&](const f32x4 (&pa)[G::kLoads], const f32x4 (&pb)[G::kLoads], int buf) {
    stage_store<H, kSplit>(pa, lds, buf * kBuf, kLo);
    if (!diag) stage_store<H, kSplit>(pb, lds, buf * kBuf + kTileHalves, kLo);
  };
  f32x4 va[G::kLoads], vb[G::kLoads];
  if (nfull == 0) {
    // fewer than kBK snapshots: one ragged stage
    stage_load_tail<kSplit, kClamp>(va, x, ra, oa, 0);
    if (!diag) stage_load_tail<kSplit, kClamp>(vb, x, rb, ob, 0);
    store(va, vb, 0);
    __syncthreads();
    compute(0);
  } else {
    stage_load<kSplit, kClamp>(va, x, ra, oa, 0);
    if (!diag) stage_load<kSplit, kClamp>(vb, x, rb, ob, 0);
    store(va, vb, 0);
    __syncthreads();
    // full stages: the next stage's loads are in flight during this stage's
    // MFMAs; one barrier per stage publishes the next buffer
    for (int st = 0; st + 1 < nfull; ++st) {
      stage_load<kSplit, kClamp>(va, x, ra, oa, (st + 1) * kBK);
      if (!diag) stage_load<kSplit, kClamp>(vb, x, rb, ob, (st + 1) * kBK);
      compute(st & 1);
      store(va, vb, (st + 1) & 1);
      __syncthreads();
    }
    if (tail) {
      stage_load_tail<kSplit, kClamp>(va, x, ra, oa, nfull * kBK);
      if (!diag) stage_load_tail<kSplit, kClamp>(vb, x, rb, ob, nfull * kBK);
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
template <class H, bool kSplit, bool kBatched>
__global__ __launch_bounds__(256, 2) void cov16_kernel(FrameDev single,
                                                       const FrameDev *__restrict__ frames,
                                                       const Item *__restrict__ items) {
  __shared__ __attribute__((aligned(16))) H lds[Geo<kSplit>::kLdsHalves];
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
  if ((ti + 1) * kCovTile > x.M) cov16_tile<H, kSplit, true>(*fp, x, ti, tj, lds);
  else cov16_tile<H, kSplit, false>(*fp, x, ti, tj, lds);
}

template <class H, bool kSplit>
void launch16(const FrameDev &single, const FrameDev *frames, const Item *items, int n_items,
              hipStream_t s) {
  const dim3 g(items ? n_items : cov_units(single.M, FM_FP16)), b(256);
  if (items) hipLaunchKernelGGL((cov16_kernel<H, kSplit, true>), g, b, 0, s, single, frames, items);
  else hipLaunchKernelGGL((cov16_kernel<H, kSplit, false>), g, b, 0, s, single, frames, items);
}

}  // namespace

hipError_t launch_covariance16(const FrameDev &single, const FrameDev *frames, const Item *items,
                               int n_items, fm_prec prec, hipStream_t s) {
  switch (prec) {
    case FM_FP16: launch16<_Float16, false>(single, frames, items, n_items, s); break;
    case FM_BF16: launch16<__bf16, false>(single, frames, items, n_items, s); break;
    case FM_FP16X3: launch16<_Float16, true>(single, frames, items, n_items, s); break;
    case FM_BF16X3: launch16<__bf16, true>(single, frames, items, n_items, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fm
