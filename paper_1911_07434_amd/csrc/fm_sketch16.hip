// fm_sketch16.hip -- Method 2 products Y = R V (Alg. 2, eq. (11)) on 16-bit
// matrix cores with compensated operands, for the mixed-precision path.
//
// Complex product as one real contraction with the (re, im) pairs of each
// channel m interleaved on the MFMA K index: row i of A is R[i][.] as stored
// (Rr_m, Ri_m), and column c of B is (Vr_m, -Vi_m) for Re Y[i][c] and
// (Vi_m, Vr_m) for Im Y[i][c]:
//   Re Y = sum_m Rr Vr - Ri Vi,   Im Y = sum_m Rr Vi + Ri Vr.
// Both operands are split into FP16 hi + lo halves and hi.hi + hi.lo + lo.hi
// accumulate in FP32 (~22-bit products) on v_mfma_f32_32x32x16_f16.  R is
// read straight from HBM (the kernel's bound) and split in registers; V is
// split once per workgroup and chunk into LDS.  Power-of-two scales keep
// both halves in FP16's normal range: R by 2^(8 - ceil(log2 max_i R_ii))
// (every |R_ij| <= max_i R_ii), V by 2^round(log2 sqrt(M)) when V is an
// orthonormal basis; Y is unscaled exactly before it is stored.
//
// Layout of a workgroup: four waves x 32 rows of R, 2n <= 64 real output
// columns in NB blocks of 32 (Re Y_c in column c, Im Y_c in column n + c, as
// the FP32 sketch).  Channels go in chunks of 32: per chunk a lane loads 4 x
// 4 complex values of its row (one MFMA K-slice each), prefetched a chunk
// ahead.  The epilogue forms the Gram partials of the workgroup's 128 rows,
// exactly as the FP32 sketch does.
#include "fm_internal.h"
#include "fm_gram.h"

namespace fm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef FM_GLOBAL const f32x4 gf32x4;
typedef FM_GLOBAL const f32x2 gf32x2;

constexpr int kCh = 32;              // channels per chunk
constexpr int kBRow = 2 * kCh + 8;   // halves per B column in LDS (16 bytes of padding)

// workgroup -> (frame, row block, channel segment); a single frame's split
// launch is row blocks x segments
template <int NB, bool kBatched>
__device__ __forceinline__ const FrameDev &frame16(const FrameDev &single, const FrameDev *frames,
                                                   const Item *items, int split, int &blk,
                                                   int &seg) {
  if constexpr (kBatched) {
    const Item &it = items[blockIdx.x];
    blk = it.a;
    seg = it.c;
    return frames[it.frame];
  } else {
    const int S = split == 1 ? sketch_segments(single.M, NB) : 1;
    blk = blockIdx.x / S;
    seg = blockIdx.x % S;
    return single;
  }
}

__device__ __forceinline__ void split8(const f32x4 &x0, const f32x4 &x1, float s, h8 &hi,
                                       h8 &lo) {
  const float v[8] = {x0.x * s, x0.y * s, x0.z * s, x0.w * s,
                      x1.x * s, x1.y * s, x1.z * s, x1.w * s};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    hi[j] = (_Float16)v[j];
    lo[j] = (_Float16)(v[j] - (float)hi[j]);
  }
}

template <int NB, bool kBatched>
__global__ __launch_bounds__(256) void sketch16_kernel(FrameDev single, const FrameDev *frames,
                                                       const Item *items, int round, int split) {
  constexpr int kPlane = 32 * NB * kBRow;  // halves in one plane (hi or lo) of one buffer
  __shared__ __attribute__((aligned(16))) _Float16 bsm[2 * 2 * kPlane];
  __shared__ float red[4];
  int blk, seg;
  const FrameDev &f = frame16<NB, kBatched>(single, frames, items, split, blk, seg);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int M = f.M, n = f.n;
  const long long ldr = f.ldr;
  const float2 *R = f.R;
  const float2 *V = f.V;
  const int i0 = blk * kSketchRows + wave * 32;

  // scales: R from its largest diagonal entry, V from its kind
  {
    float mx = 0.f;
    for (int i = tid; i < M; i += blockDim.x) mx = fmaxf(mx, R[(size_t)i * ldr + i].x);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0) red[wave] = mx;
  }
  __syncthreads();
  const float rmax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  const float sR = (rmax > 0.f && rmax < 3.0e38f) ? exp2f(8.f - ceilf(log2f(rmax))) : 1.f;
  const bool orth_v = round > 0 || f.q == 0;   // round 0 with q > 0 multiplies Omega
  const float sV = orth_v ? exp2f(rintf(0.5f * log2f((float)M))) : 1.f;

  // zero the B columns past 2n once (both buffers, both planes)
  for (int e = tid; e < 4 * kPlane; e += blockDim.x) {
    const int col = (e % kPlane) / kBRow;
    if (col >= 2 * n) bsm[e] = (_Float16)0.f;
  }

  // B staging in two steps, so that the chunk's MFMAs run between them and
  // the wait for V never waits for the R prefetch issued after it: load the
  // V chunk (kCh x n complex, row-major) into registers (elements past `lim`,
  // rows past M, come from a valid address and are stored as zero), then
  // split it into hi / lo columns in LDS
  constexpr int JB = (kCh * 16 * NB + 255) / 256;
  f32x2 vreg[JB];
  // (global-address-space loads: a flat load's wait would also wait for the
  // R prefetch and the LDS traffic)
  // The first product of a power iteration (round 0, q > 0) multiplies the
  // real test matrix, read as such (zero imaginary parts); that launch also
  // clears the frame's workspace status word, which the orth steps may set.
  const gf32x2 *Vg = (const gf32x2 *)V;
  const FM_GLOBAL float *Vr = orth_v ? nullptr : (const FM_GLOBAL float *)f.Omega;
  if (!orth_v && blk == 0 && seg == 0 && tid == 0 && split != 2) *wstat_of(f) = 0u;
  auto load_b = [&](int c, int lim) {
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      const int e = min(tid + 256 * j, lim - 1);
      if (Vr)
        vreg[j] = f32x2{Vr[(size_t)c * kCh * n + e], 0.f};
      else
        vreg[j] = Vg[(size_t)c * kCh * n + e];
    }
  };
  auto store_b = [&](int buf, int lim) {
    _Float16 *bh = bsm + buf * 2 * kPlane, *bl = bh + kPlane;
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      const int e = tid + 256 * j;
      if (e >= kCh * n) continue;
      const int ml = e / n, cc = e % n;
      const f32x2 v = e < lim ? vreg[j] : f32x2{0.f, 0.f};
      const float vr = v.x * sV, vi = v.y * sV;
      const float q[4] = {vr, -vi, vi, vr};   // Re column: (vr, -vi); Im column: (vi, vr)
      _Float16 qh[4], ql[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        qh[k] = (_Float16)q[k];
        ql[k] = (_Float16)(q[k] - (float)qh[k]);
      }
      const int ore = cc * kBRow + 2 * ml, oim = (n + cc) * kBRow + 2 * ml;
      bh[ore] = qh[0];
      bh[ore + 1] = qh[1];
      bh[oim] = qh[2];
      bh[oim + 1] = qh[3];
      bl[ore] = ql[0];
      bl[ore + 1] = ql[1];
      bl[oim] = ql[2];
      bl[oim + 1] = ql[3];
    }
  };

  // A prefetch: for K-slice ks (8 channels) the lane holds channels
  // 8 ks + 4 h .. + 3 of its row = two float4
  const int row = min(i0 + r, M - 1);
  const float *Rrow = reinterpret_cast<const float *>(R + (size_t)row * ldr);
  // a chunk inside M: unconditional loads
  auto load_r_full = [&](f32x4 (&a)[8], int c) {
    const int mb = c * kCh;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        a[2 * ks + q] = *(gf32x4 *)(Rrow + 2 * (mb + 8 * ks + 4 * h + 2 * q));
  };
  // the ragged last chunk: channels past M read as zero
  auto load_r_tail = [&](f32x4 (&a)[8], int c) {
    const int mb = c * kCh;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int m = mb + 8 * ks + 4 * h + 2 * q;
        f32x4 x = f32x4{0.f, 0.f, 0.f, 0.f};
        if (m < M) {
          const f32x2 y = *(gf32x2 *)(Rrow + 2 * m);
          x.x = y.x;
          x.y = y.y;
        }
        if (m + 1 < M) {
          const f32x2 y = *(gf32x2 *)(Rrow + 2 * (m + 1));
          x.z = y.x;
          x.w = y.y;
        }
        a[2 * ks + q] = x;
      }
  };

  floatx16 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;

  auto compute = [&](const f32x4 (&a)[8], int buf) {
    const _Float16 *bh = bsm + buf * 2 * kPlane, *bl = bh + kPlane;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      h8 ahi, alo;
      split8(a[2 * ks], a[2 * ks + 1], sR, ahi, alo);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int o = (32 * b + r) * kBRow + 16 * ks + 8 * h;
        const h8 bhi = *(const h8 *)(bh + o);
        const h8 blo = *(const h8 *)(bl + o);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, bhi, acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, blo, acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, bhi, acc[b], 0, 0, 0);
      }
    }
  };

  // Channel segments (sketch_segments): each segment's MFMAs accumulate
  // from zero and the segment sums are added in order.  split 0: the
  // segments in turn (fold at each segment start); 1: segment `seg` only,
  // its sums to spart; 2: no products, the sums read back in order -- the
  // same bits as 0.  Full chunks: the prefetch of chunk c + 1 is clamped to
  // the segment's last chunk (a repeat hits the cache), so every load in the
  // loop is unconditional and the compiler's waits cover only what each
  // step uses.
  const int nfull = M / kCh;
  const int vfull = kCh * n;
  const int segs = sketch_segments(M, NB);
  const int cb = split == 1 ? sketch_seg_chunk(seg, segs, nfull) : 0;
  const int ce = split == 1 ? sketch_seg_chunk(seg + 1, segs, nfull) : (split == 2 ? 0 : nfull);
  const bool last = split != 1 || seg == segs - 1;
  floatx16 sum[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) sum[b][v] = 0.f;
  int sg = 1, next = (split == 0 && segs > 1) ? sketch_seg_chunk(1, segs, nfull) : -1;
  auto fold = [&]() {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        sum[b][v] += acc[b][v];
        acc[b][v] = 0.f;
      }
  };
  auto at = [&](int c) {
    if (c == next) {
      fold();
      ++sg;
      next = sg < segs ? sketch_seg_chunk(sg, segs, nfull) : -1;
    }
  };
  f32x4 a0[8], a1[8];
  __syncthreads();  // zero columns written before any staging
  if (ce > cb) {
    load_b(cb, vfull);
    load_r_full(a0, cb);
    store_b(0, vfull);
    __syncthreads();
    for (int c = cb; c < ce; c += 2) {
      const int c1 = min(c + 1, ce - 1);
      load_b(c1, vfull);
      load_r_full(a1, c1);
      __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
      at(c);
      compute(a0, 0);
      store_b(1, vfull);
      __syncthreads();
      if (c + 1 >= ce) break;
      const int c2 = min(c + 2, ce - 1);
      load_b(c2, vfull);
      load_r_full(a0, c2);
      __builtin_amdgcn_sched_barrier(0);
      at(c + 1);
      compute(a1, 1);
      store_b(0, vfull);
      __syncthreads();
    }
  }
  if (split != 2 && last && nfull * kCh < M) {
    // ragged last chunk; buffer 0 is free (every wave passed the last barrier)
    load_b(nfull, (M - nfull * kCh) * n);
    load_r_tail(a0, nfull);
    store_b(0, (M - nfull * kCh) * n);
    __syncthreads();
    compute(a0, 0);
  }
  __syncthreads();  // the epilogue reuses the LDS buffers
  if (segs > 1) {
    // segment sums: this workgroup's slot [block][segment][NB][16][256]
    FM_GLOBAL float *sp = (FM_GLOBAL float *)f.spart + (size_t)blk * segs * NB * kSketchPartFloats + tid;
    if (split == 1) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) sp[((size_t)seg * NB * 16 + b * 16 + v) * 256] = acc[b][v];
      return;
    }
    if (split == 2) {
      for (int q = 0; q < segs; ++q) {
        float t[NB][16];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v)
            t[b][v] = __builtin_nontemporal_load(sp + ((size_t)q * NB * 16 + b * 16 + v) * 256);
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v) sum[b][v] += t[b][v];
      }
    } else {
      fold();
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = sum[b];
  }

  // store Y (unscaled), Re Y_c from column c, Im Y_c from column n + c
  const float inv = 1.f / (sR * sV);
  FM_GLOBAL float *Yf = (FM_GLOBAL float *)f.Y;   // global stores (a flat one also holds up LDS waits)
  float *yt = reinterpret_cast<float *>(bsm);   // [128][n] complex tile for the Gram step
  const int gmode = round < 0 ? -1 : (round < f.q ? kGramSelf : kGramFinal);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int nn = 32 * b + r;
    if (nn >= 2 * n) continue;
    const int part = nn < n ? 0 : 1, col = nn < n ? nn : nn - n;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int il = wave * 32 + (v >> 2) * 8 + h * 4 + (v & 3);
      const float y = acc[b][v] * inv;
      if (blk * kSketchRows + il < M) Yf[((size_t)(blk * kSketchRows + il) * n + col) * 2 + part] = y;
      if (gmode >= 0) yt[(il * n + col) * 2 + part] = y;
    }
  }
  if (gmode < 0) return;
  __syncthreads();
  const int m0 = blk * kGramRows;
  const int rows = min(M, m0 + kGramRows) - m0;
  const float2 *Yt = reinterpret_cast<const float2 *>(yt);
  const FM_LDS float2 *Yl = (const FM_LDS float2 *)Yt;
  gram_rows(Yl, Yl, f.part + (size_t)(blk * 2 + (gmode == kGramSelf ? 0 : 1)) * n * n, n, rows);
  if (gmode == kGramFinal)
    gram_rows((const FM_GLOBAL float2 *)(f.V + (size_t)m0 * n), Yl,
              f.part + (size_t)(blk * 2) * n * n, n, rows);
}

template <int NB>
hipError_t launch16(const FrameDev &single, const FrameDev *frames, const Item *items,
                    int n_items, int round, int split, hipStream_t s) {
  const int S = split == 1 ? sketch_segments(single.M, NB) : 1;
  const dim3 g(items ? n_items : S * ((single.M + kSketchRows - 1) / kSketchRows)), b(256);
  if (items)
    hipLaunchKernelGGL((sketch16_kernel<NB, true>), g, b, 0, s, single, frames, items, round, split);
  else
    hipLaunchKernelGGL((sketch16_kernel<NB, false>), g, b, 0, s, single, frames, items, round, split);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sketch16(const FrameDev &single, const FrameDev *frames, const Item *items,
                           int n_items, int nb, int round, int split, hipStream_t s) {
  return nb <= 1 ? launch16<1>(single, frames, items, n_items, round, split, s)
                 : launch16<2>(single, frames, items, n_items, round, split, s);
}

}  // namespace fm
