// fm_subspace.hip -- stage 2: randomized signal subspace (Alg. 1 and Alg. 2).
//
// Both methods reduce to: a sketch C (M x n) and a Nystrom core (n x n) with
// S~ = C core^+ C^H (eqs. (8)-(9)); the K leading eigen-directions of S~ are
// the signal subspace (rank restriction, Sec. III-A).
//   Method 1: C = R(:, I), core = R(I, I).
//   Method 2: C = R V with V = orth(R^q Omega), core = V^H C.
//
// The GPU evaluates this without forming S~:
//   core = E diag(lambda) E^H (Jacobi), P = E_r diag(lambda_r^-1/2)
//     (eigenvalues lambda <= rcond * lambda_max dropped: the pseudo-inverse)
//   H = P^H (C^H C) P = W diag(sigma) W^H (Jacobi)
//   U_s = C P W_K diag(sigma_K^-1/2)
// which gives the same eigenpairs as S~ = (C P)(C P)^H.  orth() uses the same
// eigen route on the Gram Y^H Y: V = Y E diag(lambda^-1/2).
//
// Kernels (one launch covers every frame of a plan):
//   omega   Omega (real) -> complex V or Y
//   sketch  Y = R V on FP32 MFMA (R streamed once per product)
//   gather  C = R(:, I) (read as conj of rows I of the Hermitian R), core
//   gram    partial sums of A^H B over 128-row chunks, FP64
//   small   one workgroup per frame: chunk sums, Jacobi eigen-solves, small
//           products, in FP64 (LDS-resident up to n = 64)
//   apply   V = Y T (complex64) or U_s = C T_f (complex128 + FP32 copy)
#include "fm_internal.h"
#include "fm_gram.h"

namespace fm {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr double kRcondOrth = 64.0 * 2.220446049250313e-16;  // orth(): drop exact zeros
// orth() by Cholesky of the Gram unless a pivot falls below this fraction of
// the largest diagonal entry (then the eigen route, which drops null directions)
constexpr double kCholPivot = 1e-10;
constexpr int kMaxSweeps = 40;

template <bool kBatched>
__device__ __forceinline__ const FrameDev &frame_of(const FrameDev &single,
                                                    const FrameDev *frames,
                                                    const Item *items, int &a, int &b) {
  if constexpr (kBatched) {
    const Item &it = items[blockIdx.x];
    a = it.a;
    b = it.b;
    return frames[it.frame];
  } else {
    a = blockIdx.x;
    b = 0;
    return single;
  }
}

__device__ inline double2 *slot(const FrameDev &f, int s) {
  return f.small + (size_t)s * f.npad * f.npad;
}
enum Slot { kSlotT = 0, kSlotCore = 1, kSlotGc = 2, kSlotP = 3, kSlotZ = 4, kSlotA = 5, kSlotV = 6 };

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// ---------------------------------------------------------------------------
// omega: real Gaussian test matrix -> complex operand
// ---------------------------------------------------------------------------
template <bool kBatched>
__global__ __launch_bounds__(256) void omega_kernel(FrameDev single, const FrameDev *frames,
                                                    const Item *items, int to_y) {
  int chunk, unused;
  const FrameDev &f = frame_of<kBatched>(single, frames, items, chunk, unused);
  const int n = f.n;
  const int m0 = chunk * kApplyRows;
  const int mend = min(f.M, m0 + kApplyRows);
  (void)to_y;
  // q = 0: V = orth(Omega) comes first, so Omega goes to Y; else V = Omega
  float2 *dst = f.q == 0 ? f.Y : f.V;
  for (int e = threadIdx.x; e < (mend - m0) * n; e += blockDim.x) {
    const int m = m0 + e / n, c = e % n;
    dst[(size_t)m * n + c] = make_float2(f.Omega[(size_t)m * n + c], 0.f);
  }
  if (chunk == 0 && threadIdx.x == 0) *wstat_of(f) = 0u;
}

// ---------------------------------------------------------------------------
// sketch: Y = R V on FP32 MFMA.  One wave = 32 rows of R, all 2n real output
// columns (n real parts, then n imaginary parts) in NB blocks of 32:
//   Re Y = Rr Vr - Ri Vi,  Im Y = Rr Vi + Ri Vr
// R streams in chunks of 32 columns: each lane owns 16 elements of its row
// (pairs of columns, the two half-waves interleaved: lane h holds columns
// 4j + 2h and 4j + 2h + 1), prefetched one chunk ahead in ping-pong
// registers; the chunk of V (32 x n) is staged once per workgroup in
// double-buffered LDS.  MFMA step s pairs the s-th column of each half.
// ---------------------------------------------------------------------------
constexpr int kSkChunkMax = 32;
static_assert(kSketchRows == kGramRows, "a sketch workgroup covers one Gram chunk");
static_assert(kSkChunkMax * kMaxL * 2 >= kSketchRows * 32, "Y tile of n <= 32 fits the V buffers");
typedef FM_GLOBAL const float2 gfloat2;
typedef FM_GLOBAL const double2 gdouble2;

// SK = elements of its row each lane holds per chunk (chunk = 2 SK columns);
// wide column classes use SK = 8 to stay within the register file
// Y = scale * A B with A [M][kdim] (leading dimension lda) and B [kdim][n]:
// the products with R (A = R, B = V, kdim = M, scale 1) and, without forming
// R, the second half of R V = X (X^H V) / T (A = X, B = Z, kdim = T,
// scale 1/T).
//
// Channel segments (products with R): the contraction runs over `segs` fixed
// segments of whole chunks (the ragged chunk in the last); each segment's
// MFMAs accumulate from zero and the segment sums are added in order.
// split 0: every segment in turn; 1: segment `seg` only, its sums to the
// frame's spart; 2: no contraction, the sums of every segment read back from
// spart in order -- the same bits as split 0.
template <int NB, int SK>
__device__ __forceinline__ void sketch_rows(const FrameDev &f, int i0, int chunk, int gmode,
                                            const float2 *Am, long long lda, int kdim,
                                            const float2 *Bm, float scale,
                                            float2 (*vbuf)[kSkChunkMax * kMaxL],
                                            int segs = 1, int split = 0, int seg = 0,
                                            const float *Breal = nullptr) {
  constexpr int kSkChunk = 2 * SK;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int r = lane & 31, h = lane >> 5;
  const int M = f.M, n = f.n;
  const int row = min(i0 + r, M - 1);
  // element s of a lane's chunk run is column 4 (s / 2) + 2 h + s % 2 of the
  // chunk: the two half-waves read neighbouring 16-byte pieces, so each load
  // instruction touches one cache line per row, not two
  const gfloat2 *pr = (const gfloat2 *)(Am + (size_t)row * lda + 2 * h);
  int col[NB], part[NB];
  bool okc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int nn = 32 * b + r;
    okc[b] = nn < 2 * n;
    part[b] = nn < n ? 0 : 1;
    col[b] = okc[b] ? (nn < n ? nn : nn - n) : 0;
  }
  floatx16 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;

  // Chunks whose SK-runs all lie inside kdim ("full") stream with every
  // load unconditional: the prefetch of chunk c + 1 is clamped to the last
  // full chunk (a repeat of it hits the cache), and V is read into
  // registers before the R prefetch and written to LDS only after the
  // chunk's MFMAs, so the wait for V never waits for the R prefetch behind
  // it.  A ragged last chunk runs after the loop with per-element guards.
  const int velems = kSkChunk * n;  // <= 16 * 16 NB (SK = 8) or 32 * 16 NB (SK = 16)
  constexpr int JV = (kSkChunk * 16 * NB + 255) / 256;
  const gfloat2 *V = (const gfloat2 *)Bm;
  float2 vst[JV];
  // V rows of chunk c (kSkChunk x n, row-major); elements past `lim` (rows
  // past kdim) are read from a valid address and replaced by zero on store
  // (Breal: B is real, given as its [kdim][n] values -- the Gaussian test
  // matrix of the first product -- and enters with zero imaginary parts)
  const FM_GLOBAL float *Vr = (const FM_GLOBAL float *)Breal;
  auto load_v = [&](int c, int lim) {
#pragma unroll
    for (int j = 0; j < JV; ++j) {
      const int e = min(tid + 256 * j, lim - 1);
      if (Vr)
        vst[j] = make_float2(Vr[(size_t)c * kSkChunk * n + e], 0.f);
      else
        vst[j] = V[(size_t)c * kSkChunk * n + e];
    }
  };
  auto store_v = [&](int buf, int lim) {
#pragma unroll
    for (int j = 0; j < JV; ++j) {
      const int e = tid + 256 * j;
      if (e < velems) vbuf[buf][e] = e < lim ? vst[j] : make_float2(0.f, 0.f);
    }
  };
  auto load_r_full = [&](float2 (&a)[SK], int c) {
#pragma unroll
    for (int s = 0; s < SK; ++s) a[s] = pr[c * kSkChunk + 4 * (s >> 1) + (s & 1)];
  };
  auto compute = [&](const float2 (&a)[SK], const float2 *vb) {
#pragma unroll
    for (int s = 0; s < SK; ++s) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int m = 4 * (s >> 1) + 2 * h + (s & 1);
        // unconditional read (col is 0 for an unused block), then a select:
        // a conditional read would branch around every MFMA pair and wait
        // for its own LDS read
        const float2 v0 = vb[m * n + col[b]];
        const float2 v = make_float2(okc[b] ? v0.x : 0.f, okc[b] ? v0.y : 0.f);
        const float bre = part[b] == 0 ? v.x : v.y;
        const float bim = part[b] == 0 ? -v.y : v.x;
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s].x, bre, acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s].y, bim, acc[b], 0, 0, 0);
      }
    }
  };

  const int nfull = kdim / kSkChunk;
  // this call's chunks [cb, ce); `next` is the start of the next segment
  // (a fold point) in a sequential run
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
  float2 a0[SK], a1[SK];
  if (ce > cb) {
    load_v(cb, velems);
    load_r_full(a0, cb);
    store_v(0, velems);
    __syncthreads();
    for (int c = cb; c < ce; c += 2) {
      // chunk c from (a0, vbuf[0]); chunk c+1 from (a1, vbuf[1])
      const int c1 = min(c + 1, ce - 1);
      load_v(c1, velems);
      load_r_full(a1, c1);
      at(c);
      compute(a0, vbuf[0]);
      store_v(1, velems);
      __syncthreads();
      if (c + 1 >= ce) break;
      const int c2 = min(c + 2, ce - 1);
      load_v(c2, velems);
      load_r_full(a0, c2);
      at(c + 1);
      compute(a1, vbuf[1]);
      store_v(0, velems);
      __syncthreads();
    }
  }
  if (split != 2 && last && nfull * kSkChunk < kdim) {
    // ragged last chunk: columns past kdim read as zero, V rows past kdim
    // are zero in LDS; vbuf[0] is free (every wave passed the last barrier)
    const int c = nfull;
    const int lim = (kdim - c * kSkChunk) * n;
    load_v(c, lim);
#pragma unroll
    for (int s = 0; s < SK; ++s) {
      const int mo = 4 * (s >> 1) + (s & 1);
      a0[s] = make_float2(0.f, 0.f);
      if (c * kSkChunk + mo + 2 * h < kdim) a0[s] = pr[c * kSkChunk + mo];
    }
    store_v(0, lim);
    __syncthreads();
    compute(a0, vbuf[0]);
  }
  if (segs > 1) {
    // segment sums: this workgroup's slot [chunk][segment][NB][16][256]
    FM_GLOBAL float *sp = (FM_GLOBAL float *)f.spart + (size_t)chunk * segs * NB * 4096 + tid;
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
  if (scale != 1.f) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[b][v] *= scale;
  }
  FM_GLOBAL float *Yf = (FM_GLOBAL float *)f.Y;   // global stores (a flat one also holds up LDS waits)
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (!okc[b]) continue;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = i0 + (v >> 2) * 8 + h * 4 + (v & 3);
      if (i < M) Yf[((size_t)i * n + col[b]) * 2 + part[b]] = acc[b][v];
    }
  }
  if constexpr (NB <= 2) {
    // Gram partials of this workgroup's 128 rows of Y (the chunk the Gram
    // step sums over), from the FP32 values just stored, staged in LDS
    if (gmode < 0) return;
    __syncthreads();  // every wave is done with the V buffers
    float *yt = reinterpret_cast<float *>(&vbuf[0][0]);  // [128][n] complex
    const int il0 = (tid >> 6) * 32;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (!okc[b]) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int il = il0 + (v >> 2) * 8 + h * 4 + (v & 3);
        yt[(il * n + col[b]) * 2 + part[b]] = acc[b][v];
      }
    }
    __syncthreads();
    const int m0 = chunk * kGramRows;
    const int rows = min(M, m0 + kGramRows) - m0;
    const float2 *Yt = reinterpret_cast<const float2 *>(yt);
    const FM_LDS float2 *Yl = (const FM_LDS float2 *)Yt;
    gram_rows(Yl, Yl, f.part + (size_t)(chunk * 2 + (gmode == kGramSelf ? 0 : 1)) * n * n, n,
              rows);
    if (gmode == kGramFinal)
      gram_rows((const FM_GLOBAL float2 *)(f.V + (size_t)m0 * n), Yl,
                f.part + (size_t)(chunk * 2) * n * n, n, rows);
  }
}

// one instantiation per NB = ceil(2n / 32); a launch only holds frames of one
// class (the plan groups them), so no kernel carries the registers of a
// wider class
// `round` is the index of this product among the frame's q + 1: for column
// classes NB <= 2 the Gram partials that follow it (orth of the next round,
// or the final core and Gram after the last product) are formed here.
// split: 0 every channel segment in turn, 1 one segment (Item::c, or the
// single frame's blockIdx % segments), 2 the in-order reduction
template <int NB, bool kBatched>
__global__ __launch_bounds__(256) void sketch_kernel(FrameDev single, const FrameDev *frames,
                                                     const Item *items, int round, int split) {
  __shared__ float2 vbuf[2][kSkChunkMax * kMaxL];
  int blk, seg = 0;
  const FrameDev *fp;
  if constexpr (kBatched) {
    const Item &it = items[blockIdx.x];
    fp = &frames[it.frame];
    blk = it.a;
    seg = it.c;
  } else {
    fp = &single;
    const int S = split == 1 ? sketch_segments(single.M, NB) : 1;
    blk = blockIdx.x / S;
    seg = blockIdx.x % S;
  }
  const FrameDev &f = *fp;
  // every wave takes part in the V staging and the barriers; waves whose
  // rows start past M clamp to row M-1 and store nothing
  const int i0 = blk * kSketchRows + (threadIdx.x >> 6) * 32;
  const int gmode = round < 0 ? -1 : (round < f.q ? kGramSelf : kGramFinal);
  // the first product of a power iteration multiplies the test matrix itself
  // (read here as real values) and clears the frame's workspace status word,
  // which the orth steps that follow may set
  const bool first = round == 0 && f.q > 0;
  if (first && blk == 0 && seg == 0 && threadIdx.x == 0 && split != 2) *wstat_of(f) = 0u;
  sketch_rows<NB, (NB <= 2 ? 16 : 8)>(f, i0, blk, gmode, f.R, f.ldr, f.M, f.V, 1.f, vbuf,
                                      sketch_segments(f.M, NB), split, seg,
                                      first ? f.Omega : nullptr);
}

// ---------------------------------------------------------------------------
// products with R without forming R: R V = X (X^H V) / T
// ---------------------------------------------------------------------------
// Z = X^H V, Z[t][c] = sum_m conj(X[m][t]) V[m][c].  One wave = 32 snapshots
// t (the MFMA rows), all 2n real output columns; the contraction runs over
// the channels m two at a time (one per half-wave), so the lanes of a wave
// read two rows of X at 32 consecutive snapshots -- contiguous 256 bytes.
//   Re Z = Xr Vr + Xi Vi,   Im Z = Xr Vi - Xi Vr.
// V chunks are staged in LDS as in the sketch; X is prefetched a chunk ahead.
template <int NB>
__device__ __forceinline__ void xhv_cols(const FrameDev &f, int t0w,
                                         float2 (*vbuf)[kSkChunkMax * kMaxL]) {
  constexpr int kCh = 32, kSteps = kCh / 2;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int r = lane & 31, h = lane >> 5;
  const int M = f.M, T = f.T, n = f.n;
  const int t = min(t0w + r, T - 1);
  const gfloat2 *px = (const gfloat2 *)(f.X + t);
  const long long ldx = f.ldx;
  int col[NB], part[NB];
  bool okc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int nn = 32 * b + r;
    okc[b] = nn < 2 * n;
    part[b] = nn < n ? 0 : 1;
    col[b] = okc[b] ? (nn < n ? nn : nn - n) : 0;
  }
  floatx16 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[b][v] = 0.f;
  const int nchunk = (M + kCh - 1) / kCh;
  const int velems = kCh * n;
  const gfloat2 *V = (const gfloat2 *)f.V;
  float2 vst[8];
  auto load_v = [&](int c) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      const int m = c * kCh + e / n;
      vst[j] = make_float2(0.f, 0.f);
      if (e < velems && m < M) vst[j] = V[(size_t)c * kCh * n + e];
    }
  };
  auto store_v = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      if (e < velems) vbuf[buf][e] = vst[j];
    }
  };
  // chunk c: step s holds X[m][t] for m = 32 c + 2 s + h; rows past M are zero
  auto load_x = [&](float2 (&a)[kSteps], int c) {
    const int m0 = c * kCh;
    if (m0 + kCh <= M) {
#pragma unroll
      for (int s = 0; s < kSteps; ++s) a[s] = px[(size_t)(m0 + 2 * s + h) * ldx];
    } else {
#pragma unroll
      for (int s = 0; s < kSteps; ++s) {
        const int m = m0 + 2 * s + h;
        a[s] = make_float2(0.f, 0.f);
        if (m < M) a[s] = px[(size_t)m * ldx];
      }
    }
  };
  auto compute = [&](const float2 (&a)[kSteps], const float2 *vb) {
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float2 v0 = vb[(2 * s + h) * n + col[b]];  // unconditional, as in sketch_rows
        const float2 v = make_float2(okc[b] ? v0.x : 0.f, okc[b] ? v0.y : 0.f);
        const float b1 = part[b] == 0 ? v.x : v.y;    // with Xr
        const float b2 = part[b] == 0 ? v.y : -v.x;   // with Xi
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s].x, b1, acc[b], 0, 0, 0);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s].y, b2, acc[b], 0, 0, 0);
      }
    }
  };
  float2 a0[kSteps], a1[kSteps];
  load_v(0);
  store_v(0);
  load_x(a0, 0);
  __syncthreads();
  for (int c = 0; c < nchunk; c += 2) {
    const bool has1 = c + 1 < nchunk;
    if (has1) {
      load_v(c + 1);
      load_x(a1, c + 1);
    }
    compute(a0, vbuf[0]);
    if (has1) store_v(1);
    __syncthreads();
    if (!has1) break;
    const bool has2 = c + 2 < nchunk;
    if (has2) {
      load_v(c + 2);
      load_x(a0, c + 2);
    }
    compute(a1, vbuf[1]);
    if (has2) store_v(0);
    __syncthreads();
  }
  float *Zf = reinterpret_cast<float *>(f.Z);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (!okc[b]) continue;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int tt = t0w + (v >> 2) * 8 + h * 4 + (v & 3);
      if (tt < T) Zf[((size_t)tt * n + col[b]) * 2 + part[b]] = acc[b][v];
    }
  }
}

template <int NB, bool kBatched>
__global__ __launch_bounds__(256) void xhv_kernel(FrameDev single, const FrameDev *frames,
                                                  const Item *items) {
  __shared__ float2 vbuf[2][kSkChunkMax * kMaxL];
  int blk, unused;
  const FrameDev &f = frame_of<kBatched>(single, frames, items, blk, unused);
  xhv_cols<NB>(f, blk * kXhvCols + (threadIdx.x >> 6) * 32, vbuf);
}

template <int NB, bool kBatched>
__global__ __launch_bounds__(256) void xz_kernel(FrameDev single, const FrameDev *frames,
                                                 const Item *items, int round) {
  __shared__ float2 vbuf[2][kSkChunkMax * kMaxL];
  int blk, unused;
  const FrameDev &f = frame_of<kBatched>(single, frames, items, blk, unused);
  const int i0 = blk * kSketchRows + (threadIdx.x >> 6) * 32;
  const int gmode = round < 0 ? -1 : (round < f.q ? kGramSelf : kGramFinal);
  sketch_rows<NB, (NB <= 2 ? 16 : 8)>(f, i0, blk, gmode, f.X, f.ldx, f.T, f.Z,
                                      1.f / (float)f.T, vbuf);
}

// ---------------------------------------------------------------------------
// Method 1 without forming R: C = R(:, I) = X X(I, :)^H / T, core = C(I, :)
// ---------------------------------------------------------------------------
// Z[t][j] = conj(X[idx_j][t]) (the B operand of C = X Z / T), through an LDS
// tile so that both the reads (along a row of X) and the writes (along j)
// are contiguous.  Indices are clamped here and checked by xcore_kernel.
template <bool kBatched>
__global__ __launch_bounds__(256) void zx_kernel(FrameDev single, const FrameDev *frames,
                                                 const Item *items) {
  __shared__ float2 tile[kMaxL][kZxCols + 1];
  int blk, unused;
  const FrameDev &f = frame_of<kBatched>(single, frames, items, blk, unused);
  const int p = f.n, M = f.M, T = f.T;
  const int t0 = blk * kZxCols;
  const int cols = min(T, t0 + kZxCols) - t0;
  for (int e = threadIdx.x; e < p * kZxCols; e += blockDim.x) {
    const int j = e / kZxCols, tt = e % kZxCols;
    const int ij = min(max(f.idx[j], 0), M - 1);
    float2 v = make_float2(0.f, 0.f);
    if (tt < cols) v = f.X[(size_t)ij * f.ldx + t0 + tt];
    tile[j][tt] = make_float2(v.x, -v.y);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < cols * p; e += blockDim.x) {
    const int tt = e / p, j = e % p;
    f.Z[(size_t)(t0 + tt) * p + j] = tile[j][tt];
  }
}

// core = C(I, :) in FP64 (C = R(:, I) just formed in Y), the index check, and
// the frame's status word
template <bool kBatched>
__global__ __launch_bounds__(256) void xcore_kernel(FrameDev single, const FrameDev *frames,
                                                    const Item *items) {
  __shared__ unsigned bad;
  int unused_a, unused_b;
  const FrameDev &f = frame_of<kBatched>(single, frames, items, unused_a, unused_b);
  const int n = f.n, M = f.M, np = f.npad;
  if (threadIdx.x == 0) bad = 0u;
  __syncthreads();
  double2 *core = slot(f, kSlotCore);
  for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
    const int a = e / np, b = e % np;
    double2 v = make_double2(0.0, 0.0);
    if (a < n && b < n) {
      const int ia = f.idx[a], ib = f.idx[b];
      if (ia < 0 || ia >= M || (a != b && ia == ib)) atomicOr(&bad, (unsigned)FM_ST_BAD_INDEX);
      const float2 c = f.Y[(size_t)min(max(ia, 0), M - 1) * n + b];
      v = make_double2(c.x, c.y);
    }
    core[e] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) *wstat_of(f) = bad;
}

// ---------------------------------------------------------------------------
// gather (Method 1): C[m][j] = R[m][idx_j] = conj(R[idx_j][m]); chunk 0 also
// forms core = R(I, I) in FP64 and checks the index set.
// ---------------------------------------------------------------------------
template <bool kBatched>
__global__ __launch_bounds__(256) void gather_kernel(FrameDev single, const FrameDev *frames,
                                                     const Item *items) {
  int chunk, unused;
  const FrameDev &f = frame_of<kBatched>(single, frames, items, chunk, unused);
  const int n = f.n, M = f.M;
  const int m0 = chunk * kApplyRows;
  const int rows = min(M, m0 + kApplyRows) - m0;
  for (int e = threadIdx.x; e < rows * n; e += blockDim.x) {
    const int j = e / rows, m = m0 + e % rows;  // consecutive threads read along a row of R
    const int ij = min(max(f.idx[j], 0), M - 1);
    const float2 v = f.R[(size_t)ij * f.ldr + m];
    f.Y[(size_t)m * n + j] = make_float2(v.x, -v.y);
  }
  if (chunk == 0) {
    __shared__ unsigned bad;
    if (threadIdx.x == 0) bad = 0u;
    __syncthreads();
    double2 *core = slot(f, kSlotCore);
    const int np = f.npad;
    for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
      const int a = e / np, b = e % np;
      double2 v = make_double2(0.0, 0.0);
      if (a < n && b < n) {
        const int ia = f.idx[a], ib = f.idx[b];
        if (ia < 0 || ia >= M || (a != b && ia == ib)) atomicOr(&bad, (unsigned)FM_ST_BAD_INDEX);
        const float2 r = f.R[(size_t)min(max(ia, 0), M - 1) * f.ldr + min(max(ib, 0), M - 1)];
        v = make_double2(r.x, r.y);
      }
      core[e] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) *wstat_of(f) = bad;
  }
}

// ---------------------------------------------------------------------------
// gram: partial sums over a 128-row chunk of A^H B, FP64 accumulation of the
// FP32 inputs (their products are exact in FP64).  Each thread owns a TB x TB
// block of entries.
// ---------------------------------------------------------------------------
template <int TB>
__device__ __forceinline__ void gram_block(const float2 *Ain, const float2 *Bin, double2 *outp,
                                           int n, int m0, int m1) {
  // the operands and partials live in global workspace: global-address
  // loads, so the compiler's waits count only these loads
  const gfloat2 *A = (const gfloat2 *)Ain;
  const gfloat2 *B = (const gfloat2 *)Bin;
  FM_GLOBAL double2 *out = (FM_GLOBAL double2 *)outp;
  const int nbk = (n + TB - 1) / TB;
  for (int blk = threadIdx.x; blk < nbk * nbk; blk += blockDim.x) {
    const int a0 = (blk / nbk) * TB, b0 = (blk % nbk) * TB;
    double2 acc[TB][TB];
#pragma unroll
    for (int x = 0; x < TB; ++x)
#pragma unroll
      for (int y = 0; y < TB; ++y) acc[x][y] = make_double2(0.0, 0.0);
    for (int m = m0; m < m1; ++m) {
      float2 av[TB], bv[TB];
#pragma unroll
      for (int x = 0; x < TB; ++x) {
        const float2 a = A[(size_t)m * n + min(a0 + x, n - 1)];
        const float2 b = B[(size_t)m * n + min(b0 + x, n - 1)];
        av[x] = (a0 + x < n) ? a : make_float2(0.f, 0.f);
        bv[x] = (b0 + x < n) ? b : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int x = 0; x < TB; ++x)
#pragma unroll
        for (int y = 0; y < TB; ++y) {
          const double ar = av[x].x, ai = av[x].y, br = bv[y].x, bi = bv[y].y;
          acc[x][y].x = fma(ar, br, acc[x][y].x);
          acc[x][y].x = fma(ai, bi, acc[x][y].x);
          acc[x][y].y = fma(ar, bi, acc[x][y].y);
          acc[x][y].y = fma(-ai, br, acc[x][y].y);
        }
    }
#pragma unroll
    for (int x = 0; x < TB; ++x)
#pragma unroll
      for (int y = 0; y < TB; ++y)
        if (a0 + x < n && b0 + y < n) out[(size_t)(a0 + x) * n + b0 + y] = acc[x][y];
  }
}

template <bool kBatched>
__global__ __launch_bounds__(256) void gram_kernel(FrameDev single, const FrameDev *frames,
                                                   const Item *items, int mode) {
  int chunk, unused;
  const FrameDev &f = frame_of<kBatched>(single, frames, items, chunk, unused);
  const int n = f.n;
  const int m0 = chunk * kGramRows, m1 = min(f.M, m0 + kGramRows);
  double2 *p0 = f.part + (size_t)(chunk * 2 + 0) * n * n;
  double2 *p1 = f.part + (size_t)(chunk * 2 + 1) * n * n;
  const int tb = (n <= 16) ? 1 : (n <= 32 ? 2 : 4);
  auto run = [&](const float2 *A, const float2 *B, double2 *out) {
    if (tb == 1) gram_block<1>(A, B, out, n, m0, m1);
    else if (tb == 2) gram_block<2>(A, B, out, n, m0, m1);
    else gram_block<4>(A, B, out, n, m0, m1);
  };
  if (mode == kGramSelf) {
    run(f.Y, f.Y, p0);
  } else if (f.method == FM_METHOD_PROJECT || f.method == FM_METHOD_PROJECT_X) {
    run(f.V, f.Y, p0);   // core = V^H (R V)
    run(f.Y, f.Y, p1);   // C^H C
  } else {
    run(f.Y, f.Y, p1);   // C^H C (core comes from the gather)
  }
}

// ---------------------------------------------------------------------------
// small dense: Jacobi eigen-solver for a Hermitian matrix, one workgroup
// ---------------------------------------------------------------------------
struct Rot {
  double2 jpp, jpq, jqp, jqq;
  double ap, aq;
  int p, q, mode;  // mode 0: identity, 1: rotate, 2: identity + zero A_pq
};

__device__ inline int rr_index(int pos, int round, int np) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (np - 1);
}

// Block sums of two doubles per thread in a fixed order: an xor butterfly
// inside each wave (both partners add the same two operands, so every lane
// ends with the same bits), then the wave sums in wave order.  Two barriers.
__device__ void block_sum2(double &a, double &b, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int i = 0; i < nw; ++i) {
    a += red[2 * i];
    b += red[2 * i + 1];
  }
  __syncthreads();  // red is reused by the next call
}

// Cyclic Jacobi with round-robin (parallel) ordering on an np x np Hermitian
// matrix A (np even; rows/columns >= n are zero padding).  V accumulates the
// rotations (must start as the identity).  A becomes diagonal.  Returns the
// number of sweeps or -1 at the sweep limit.
__device__ int jacobi_eigh(double2 *A, double2 *V, int np, Rot *rot, double *red) {
  const int nh = np / 2;
  for (int sweep = 0;; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
      const double2 v = A[e];
      const double a2 = v.x * v.x + v.y * v.y;
      tot += a2;
      if (e / np != e % np) off += a2;
    }
    block_sum2(off, tot, red);
    if (off == 0.0 || off <= 1e-30 * tot) return sweep;
    if (sweep == kMaxSweeps) return -1;
    for (int round = 0; round < np - 1; ++round) {
      for (int k = threadIdx.x; k < nh; k += blockDim.x) {
        int p = rr_index(k, round, np), q = rr_index(np - 1 - k, round, np);
        if (p > q) { const int t = p; p = q; q = t; }
        Rot R;
        R.p = p;
        R.q = q;
        R.jpp = make_double2(1.0, 0.0);
        R.jpq = make_double2(0.0, 0.0);
        R.jqp = make_double2(0.0, 0.0);
        R.jqq = make_double2(1.0, 0.0);
        R.ap = A[(size_t)p * np + p].x;
        R.aq = A[(size_t)q * np + q].x;
        R.mode = 0;
        const double2 b = A[(size_t)p * np + q];
        const double ab = sqrt(b.x * b.x + b.y * b.y);
        if (ab > 0.0) {
          if (ab <= 1e-18 * sqrt(fabs(R.ap) * fabs(R.aq))) {
            R.mode = 2;
          } else {
            const double z = (R.aq - R.ap) / (2.0 * ab);
            const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double s = t * c;
            const double2 e = make_double2(b.x / ab, -b.y / ab);  // e^{-i phi}
            R.jpp = make_double2(c, 0.0);
            R.jpq = make_double2(s, 0.0);
            R.jqp = make_double2(-s * e.x, -s * e.y);
            R.jqq = make_double2(c * e.x, c * e.y);
            R.ap = R.ap - t * ab;
            R.aq = R.aq + t * ab;
            R.mode = 1;
          }
        }
        rot[k] = R;
      }
      __syncthreads();
      // A <- J^H A J on 2x2 blocks (rows of pair ki, columns of pair kj)
      for (int e = threadIdx.x; e < nh * nh; e += blockDim.x) {
        const int ki = e / nh, kj = e % nh;
        const Rot &Ri = rot[ki];
        const Rot &Rj = rot[kj];
        const size_t pp = (size_t)Ri.p * np + Rj.p, pq = (size_t)Ri.p * np + Rj.q;
        const size_t qp = (size_t)Ri.q * np + Rj.p, qq = (size_t)Ri.q * np + Rj.q;
        if (ki == kj) {
          if (Ri.mode == 1) {
            A[pp] = make_double2(Ri.ap, 0.0);
            A[qq] = make_double2(Ri.aq, 0.0);
            A[pq] = make_double2(0.0, 0.0);
            A[qp] = make_double2(0.0, 0.0);
          } else if (Ri.mode == 2) {
            A[pq] = make_double2(0.0, 0.0);
            A[qp] = make_double2(0.0, 0.0);
          }
          continue;
        }
        if (Ri.mode != 1 && Rj.mode != 1) continue;
        const double2 b00 = A[pp], b01 = A[pq], b10 = A[qp], b11 = A[qq];
        // C = B J_j
        const double2 c00 = cadd(cmul(b00, Rj.jpp), cmul(b01, Rj.jqp));
        const double2 c01 = cadd(cmul(b00, Rj.jpq), cmul(b01, Rj.jqq));
        const double2 c10 = cadd(cmul(b10, Rj.jpp), cmul(b11, Rj.jqp));
        const double2 c11 = cadd(cmul(b10, Rj.jpq), cmul(b11, Rj.jqq));
        // D = J_i^H C
        A[pp] = cadd(cmulc(Ri.jpp, c00), cmulc(Ri.jqp, c10));
        A[pq] = cadd(cmulc(Ri.jpp, c01), cmulc(Ri.jqp, c11));
        A[qp] = cadd(cmulc(Ri.jpq, c00), cmulc(Ri.jqq, c10));
        A[qq] = cadd(cmulc(Ri.jpq, c01), cmulc(Ri.jqq, c11));
      }
      // V <- V J
      for (int e = threadIdx.x; e < nh * np; e += blockDim.x) {
        const int kj = e / np, row = e % np;
        const Rot &Rj = rot[kj];
        if (Rj.mode != 1) continue;
        const size_t ip = (size_t)row * np + Rj.p, iq = (size_t)row * np + Rj.q;
        const double2 vp = V[ip], vq = V[iq];
        V[ip] = cadd(cmul(vp, Rj.jpp), cmul(vq, Rj.jqp));
        V[iq] = cadd(cmul(vp, Rj.jpq), cmul(vq, Rj.jqq));
      }
      __syncthreads();
    }
  }
}

// Descending order of the diagonal of A (first n entries); ties keep index
// order.  perm[k] = index of the k-th largest.  w[k] = its value.
__device__ void sort_desc(const double2 *A, int np, int n, int *perm, double *w) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double wi = A[(size_t)i * np + i].x;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = A[(size_t)j * np + j].x;
      rank += (wj > wi) || (wj == wi && j < i);
    }
    perm[rank] = i;
    w[rank] = wi;
  }
  __syncthreads();
}

// 1 / x and 1 / sqrt(x), x > 0 finite: the hardware approximations refined
// by two Newton steps (each squares the relative error), a handful of
// dependent FMAs against the long correctly-rounded sequences
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ inline double rsq_nr(double x) {
  const double h = 0.5 * x;
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

// Rotation of the pair (p, q) that annihilates b = A_pq, as in jacobi_eigh:
// J = [[c, s], [-s e, c e]] with e = conj(b) / |b| and t = s / c the smaller
// root of t^2 + 2 z t - 1 = 0, z = (A_qq - A_pp) / (2 |b|); mode 0 identity,
// 1 rotate, 2 identity and zero A_pq (|b| negligible against the diagonal).
// t starts in single precision and takes one Newton step in double (error
// ~1e-14 relative, left in A_pq for the next sweep); c and e are exact to
// double rounding, so J is unitary to that level whatever t is.
struct RotW {
  double c, s, ex, ey, ap, aq;
  int mode;
};
__device__ inline RotW make_rot(double ap, double aq, double2 b) {
  RotW R;
  R.c = 1.0;
  R.s = 0.0;
  R.ex = 1.0;
  R.ey = 0.0;
  R.ap = ap;
  R.aq = aq;
  R.mode = 0;
  const double ab2 = b.x * b.x + b.y * b.y;
  if (ab2 > 0.0) {
    if (ab2 <= 1e-36 * fabs(ap * aq)) {
      R.mode = 2;
    } else {
      const double ia = rsq_nr(ab2);  // 1 / |b|
      const double ab = ab2 * ia;
      const double z = (aq - ap) * (0.5 * ia), az = fabs(z);
      double t;
      if (az < 1e18) {
        const float zf = (float)az;
        // (hardware square root and reciprocal: a seed, refined below)
        const float t0 = __builtin_amdgcn_rcpf(zf + __builtin_amdgcn_sqrtf(fmaf(zf, zf, 1.0f)));
        double u = (double)t0;
        const double f = fma(u, u + 2.0 * az, -1.0);
        u = fma(-f, (double)__builtin_amdgcn_rcpf((float)(2.0 * (u + az))), u);
        t = z >= 0.0 ? u : -u;
      } else {
        t = (z >= 0.0 ? 0.5 : -0.5) * rcp_nr(az);
      }
      const double c = rsq_nr(fma(t, t, 1.0));
      R.c = c;
      R.s = t * c;
      R.ex = b.x * ia;
      R.ey = -b.y * ia;
      R.ap = ap - t * ab;
      R.aq = aq + t * ab;
      R.mode = 1;
    }
  }
  return R;
}

// Cyclic Jacobi with the same round-robin ordering and stopping rule as
// jacobi_eigh, on one wave, for a 16 x 16 matrix (ld 16; a smaller matrix
// zero-padded: a rotation against a padding index is the identity, so the
// padding stays zero and the leading block's result is unchanged).  Lane l
// owns the 2x2 block (ki, kj) = (l / 8, l % 8) of the round's pairs and
// rows ki, ki + 8 of V's columns of pair kj.  It forms the rotation of pair
// kj from the round's A and takes c, s and e of pair ki from lane ki (whose
// kj is ki) by cross-lane reads (a diagonal block, ki = kj, has its own
// rotation already), so a round needs no rotation table and no workgroup
// barrier.  The wave's LDS reads and writes are performed in
// program order; the wavefront-scope fences keep the compiler from moving
// them across the read / write split.  Call from all 64 lanes of one wave.
__device__ __forceinline__ int rr16(int pos, int round) {
  int x = pos - 1 + round;
  x = x >= 15 ? x - 15 : x;
  return pos == 0 ? 0 : 1 + x;
}
__device__ __forceinline__ int jacobi_wave16(double2 *A, double2 *V) {
  const int l = threadIdx.x & 63, ki = l >> 3, kj = l & 7;
  for (int sweep = 0;; ++sweep) {
    double off = 0.0, tot = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = l + 64 * u;
      const double2 v = A[e];
      const double a2 = v.x * v.x + v.y * v.y;
      tot += a2;
      if ((e >> 4) != (e & 15)) off += a2;
    }
    // xor butterfly: both partners add the same two operands, so every lane
    // ends with the same sums and the exit is uniform
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      tot += __shfl_xor(tot, o);
    }
    if (off == 0.0 || off <= 1e-30 * tot) return sweep;
    if (sweep == kMaxSweeps) return -1;
    // the round's pairs (pi < qi of pair ki, pj < qj of pair kj); those of
    // the next round are formed during this one (integer work off the
    // round's chain of LDS reads and FP64 operations)
    auto pairs = [&](int round, int &pi, int &qi, int &pj, int &qj) {
      pi = rr16(ki, round);
      qi = rr16(15 - ki, round);
      pj = rr16(kj, round);
      qj = rr16(15 - kj, round);
      const int ti = min(pi, qi), tj = min(pj, qj);
      qi = max(pi, qi);
      pi = ti;
      qj = max(pj, qj);
      pj = tj;
    };
    int pi, qi, pj, qj;
    pairs(0, pi, qi, pj, qj);
    for (int round = 0; round < 15; ++round) {
      const double apj = A[pj * 17].x, aqj = A[qj * 17].x;
      const double2 bj = A[pj * 16 + qj];
      const double2 b00 = A[pi * 16 + pj], b01 = A[pi * 16 + qj];
      const double2 b10 = A[qi * 16 + pj], b11 = A[qi * 16 + qj];
      const double2 vp0 = V[ki * 16 + pj], vq0 = V[ki * 16 + qj];
      const double2 vp1 = V[(ki + 8) * 16 + pj], vq1 = V[(ki + 8) * 16 + qj];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      int npi, nqi, npj, nqj;
      pairs(round + 1 < 15 ? round + 1 : 0, npi, nqi, npj, nqj);
      const RotW Rj = make_rot(apj, aqj, bj);
      // pair ki's rotation: lane ki computed it as its pair kj
      RotW Ri;
      Ri.c = __shfl(Rj.c, ki);
      Ri.s = __shfl(Rj.s, ki);
      Ri.ex = __shfl(Rj.ex, ki);
      Ri.ey = __shfl(Rj.ey, ki);
      // J = [[c, s], [-s e, c e]]: qp = -s e, qq = c e of pair kj
      const double qpx = -Rj.s * Rj.ex, qpy = -Rj.s * Rj.ey;
      const double qqx = Rj.c * Rj.ex, qqy = Rj.c * Rj.ey;
      // C = B J_j
      auto colp = [&](double2 bp, double2 bq) {  // bp c + bq qp
        return make_double2(fma(Rj.c, bp.x, fma(bq.x, qpx, -bq.y * qpy)),
                            fma(Rj.c, bp.y, fma(bq.x, qpy, bq.y * qpx)));
      };
      auto colq = [&](double2 bp, double2 bq) {  // bp s + bq qq
        return make_double2(fma(Rj.s, bp.x, fma(bq.x, qqx, -bq.y * qqy)),
                            fma(Rj.s, bp.y, fma(bq.x, qqy, bq.y * qqx)));
      };
      const double2 c00 = colp(b00, b01), c01 = colq(b00, b01);
      const double2 c10 = colp(b10, b11), c11 = colq(b10, b11);
      // D = J_i^H C: J_i^H = [[c, -s conj(e)], [s, c conj(e)]]
      const double2 w0 = make_double2(fma(Ri.ex, c10.x, Ri.ey * c10.y), fma(Ri.ex, c10.y, -Ri.ey * c10.x));
      const double2 w1 = make_double2(fma(Ri.ex, c11.x, Ri.ey * c11.y), fma(Ri.ex, c11.y, -Ri.ey * c11.x));
      double2 d00 = make_double2(fma(Ri.c, c00.x, -Ri.s * w0.x), fma(Ri.c, c00.y, -Ri.s * w0.y));
      double2 d01 = make_double2(fma(Ri.c, c01.x, -Ri.s * w1.x), fma(Ri.c, c01.y, -Ri.s * w1.y));
      double2 d10 = make_double2(fma(Ri.s, c00.x, Ri.c * w0.x), fma(Ri.s, c00.y, Ri.c * w0.y));
      double2 d11 = make_double2(fma(Ri.s, c01.x, Ri.c * w1.x), fma(Ri.s, c01.y, Ri.c * w1.y));
      if (ki == kj && Rj.mode != 0) {
        // the pair's own 2x2 block (Ri is Rj): the rotated diagonal, A_pq
        // annihilated
        if (Rj.mode == 1) {
          d00 = make_double2(Rj.ap, 0.0);
          d11 = make_double2(Rj.aq, 0.0);
        }
        d01 = make_double2(0.0, 0.0);
        d10 = d01;
      }
      A[pi * 16 + pj] = d00;
      A[pi * 16 + qj] = d01;
      A[qi * 16 + pj] = d10;
      A[qi * 16 + qj] = d11;
      V[ki * 16 + pj] = colp(vp0, vq0);
      V[ki * 16 + qj] = colq(vp0, vq0);
      V[(ki + 8) * 16 + pj] = colp(vp1, vq1);
      V[(ki + 8) * 16 + qj] = colq(vp1, vq1);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      pi = npi;
      qi = nqi;
      pj = npj;
      qj = nqj;
    }
  }
}

// Hermitian eigen-solver of the small kernel: the one-wave Jacobi on the
// 16 x 16 LDS matrices (wave 0 works, the others wait at the barrier), the
// workgroup Jacobi for the wider classes.  Every thread returns the sweep
// count.
template <int NMAX>
__device__ __forceinline__ int eigh_small(double2 *A, double2 *V, int np, Rot *rot, double *red,
                                          int *sweeps) {
  if constexpr (NMAX == 16) {
    if (threadIdx.x < 64) {
      const int sw = jacobi_wave16(A, V);
      if (threadIdx.x == 0) *sweeps = sw;
    }
    __syncthreads();
    return *sweeps;
  } else {
    return jacobi_eigh(A, V, np, rot, red);
  }
}

// Cholesky factor of the leading n x n block of the Hermitian A (ld np) in
// place, right-looking (step j updates the trailing lower triangle, one
// entry per thread, then scales column j), and X = L^-1 (X must hold the
// identity; lower triangle, ld np) by forward substitution, rows of X in
// turn and columns in parallel.  inv[j] receives 1 / L_jj.  Returns false,
// the same in every thread, when a pivot is not above kCholPivot * dmax (A
// is then partly overwritten).  Two barriers per step.
__device__ __forceinline__ bool chol_inv(double2 *A, double2 *X, double *inv, int np, int n, double dmax) {
  for (int j = 0; j < n; ++j) {
    const double d = A[j * np + j].x;
    if (!(d > kCholPivot * dmax)) return false;
    const double il = rsq_nr(d), rd = il * il;
    const int m = n - 1 - j;
    // A_ik -= A_ij conj(A_kj) / d on the trailing lower triangle
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k > i) continue;
      const double2 aij = A[i * np + j], akj = A[k * np + j];
      const double2 p = cmulc(akj, aij);  // A_ij conj(A_kj)
      const double2 a = A[i * np + k];
      A[i * np + k] = make_double2(a.x - p.x * rd, a.y - p.y * rd);
    }
    __syncthreads();
    const double l = d * il;
    for (int i = j + threadIdx.x; i < n; i += blockDim.x) {
      const double2 a = A[i * np + j];
      A[i * np + j] = i == j ? make_double2(l, 0.0) : make_double2(a.x * il, a.y * il);
    }
    if (threadIdx.x == 0) inv[j] = il;
    __syncthreads();
  }
  // L X = I: row i of X is (B_i - sum_k<i L_ik X_k) / L_ii, with B_i kept
  // in X's row i and the sum applied as rows of X are finished
  for (int i = 0; i < n; ++i) {
    const double il = inv[i];
    for (int c = threadIdx.x; c <= i; c += blockDim.x) {
      const double2 b = X[i * np + c];
      X[i * np + c] = make_double2(b.x * il, b.y * il);
    }
    __syncthreads();
    const int m = n - 1 - i;
    for (int e = threadIdx.x; e < m * (i + 1); e += blockDim.x) {
      const int k = i + 1 + e / (i + 1), c = e % (i + 1);
      const double2 x = cmul(A[k * np + i], X[i * np + c]);
      const double2 b = X[k * np + c];
      X[k * np + c] = make_double2(b.x - x.x, b.y - x.y);
    }
    __syncthreads();
  }
  return true;
}

// chol_inv on one wave for the 16 x 16 LDS matrices (ld 16), n <= 16: lane
// l holds entries l + 64 u (u < 4) in registers, row (l >> 4) + 4 u, column
// l & 15.  A step exchanges one column (and, in the substitution, one row)
// through a 32-entry LDS buffer -- one LDS round trip per step, all other
// arithmetic in registers.  The new values are selected branch-free.  The
// wave's LDS accesses are performed in program order, and wavefront-scope
// fences keep the compiler from moving them across the write / read split.
// A is left as it was (the factor stays in registers); X receives L^-1.
// Call from all 64 lanes of one wave; the result is uniform.
// c ? a : b per component (a conditional on the struct itself is lowered
// through private memory)
__device__ __forceinline__ double2 sel2(bool c, double2 a, double2 b) {
  return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
__device__ __forceinline__ bool chol_inv_wave16(const double2 *A, double2 *X, double *inv, int n,
                                                double dmax) {
  __shared__ double2 xch[32];  // [0, 16): a column of L; [16, 32): a row of X
  const int l = threadIdx.x & 63, r0 = l >> 4, k = l & 15;
  double2 a[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) a[u] = A[l + 64 * u];
  for (int j = 0; j < n; ++j) {
    // column j of the updated matrix, from the lanes of column j
    if (k == j) {
#pragma unroll
      for (int u = 0; u < 4; ++u) xch[r0 + 4 * u] = a[u];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const double d = xch[j].x;
    double2 aij[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) aij[u] = xch[r0 + 4 * u];
    const double2 akj = xch[k];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (!(d > kCholPivot * dmax)) return false;
    const double il = rsq_nr(d), rd = il * il;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = r0 + 4 * u;
      // trailing entry (j < k <= i): A_ik - A_ij conj(A_kj) / d
      const double px = aij[u].x * akj.x + aij[u].y * akj.y;
      const double py = aij[u].y * akj.x - aij[u].x * akj.y;
      const double2 t = make_double2(fma(-px, rd, a[u].x), fma(-py, rd, a[u].y));
      // column j (i >= j): L_ij = A_ij / sqrt(d), L_jj = sqrt(d)
      const double2 c = sel2(i == j, make_double2(d * il, 0.0), make_double2(a[u].x * il, a[u].y * il));
      const bool live = i < n && k <= i;
      a[u] = sel2(live && k > j, t, sel2(live && k == j, c, a[u]));
    }
    if (l == 0) inv[j] = il;
  }
  // L X = I, X starting as the identity: at step i row i of X is scaled by
  // 1 / L_ii (the rows above it applied) and applied to the rows below
  double2 x[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) x[u] = make_double2(r0 + 4 * u == k ? 1.0 : 0.0, 0.0);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int i = 0; i < n; ++i) {
    const double il = inv[i];
    const int ui = i >> 2;
    double2 xo = x[0];
#pragma unroll
    for (int u = 1; u < 4; ++u) xo = sel2(u == ui, x[u], xo);
    // row i of X (scaled) from the lanes of row group i & 3, column i of L
    // from the lanes of column i
    if (r0 == (i & 3)) xch[16 + k] = make_double2(xo.x * il, xo.y * il);
    if (k == i) {
#pragma unroll
      for (int u = 0; u < 4; ++u) xch[r0 + 4 * u] = a[u];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const double2 xs = xch[16 + k];
    double2 lk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) lk[u] = xch[r0 + 4 * u];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int row = r0 + 4 * u;
      const double2 t = make_double2(x[u].x - (lk[u].x * xs.x - lk[u].y * xs.y),
                                     x[u].y - (lk[u].x * xs.y + lk[u].y * xs.x));
      const bool live = k <= i && row < n && row >= i;
      x[u] = sel2(live, sel2(row == i, xs, t), x[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) X[l + 64 * u] = x[u];
  return true;
}

// chol_inv of the small kernel: on wave 0 for the 16 x 16 LDS matrices, by
// the workgroup otherwise.  Uniform result in every thread.
template <int NMAX>
__device__ __forceinline__ bool chol_small(double2 *A, double2 *X, double *inv, int np, int n,
                                           double dmax, int *flag) {
  if constexpr (NMAX == 16) {
    if (threadIdx.x < 64) {
      const bool ok = chol_inv_wave16(A, X, inv, n, dmax);
      if (threadIdx.x == 0) *flag = ok;
    }
    __syncthreads();
    return *flag != 0;
  } else {
    return chol_inv(A, X, inv, np, n, dmax);
  }
}

// LDS footprint of the small kernel for matrices up to NMAX (0: global).
template <int NMAX>
struct SmallLds {
  static constexpr int kMat = NMAX > 0 ? NMAX * NMAX : 1;
  // the final step's products Gc, P, Z stay in LDS for n <= 16 (wider
  // classes keep them in global workspace slots, so that several
  // workgroups still share a CU)
  static constexpr bool kProdLds = NMAX > 0 && NMAX <= 16;
  static constexpr int kProd = kProdLds ? NMAX * NMAX : 1;
  double2 A[kMat];
  double2 V[kMat];
  double2 Gc[kProd];
  double2 P[kProd];
  double2 Z[kProd];
  Rot rot[NMAX > 0 ? NMAX / 2 : kMaxN / 2];
  double red[256];
  double w[kMaxN];
  double inv[kMaxN];
  int perm[kMaxN];
  int sweeps;
  int flag;
  int rank;
  unsigned st;
  int chol_ok;
};

// Entries (i, j) and (j, i) of the sum of a frame's Gram partials (slot
// `which` of each chunk) in chunk order; the loads of eight chunks are issued
// before their sums.
__device__ inline void sum_parts(const double2 *part, int nchunk, int which, int n, int i, int j,
                                 double2 &a, double2 &b) {
  for (int c0 = 0; c0 < nchunk; c0 += 8) {
    double2 va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = min(c0 + u, nchunk - 1);
      const FM_GLOBAL double2 *pc =
          (const FM_GLOBAL double2 *)(part + (size_t)(c * 2 + which) * n * n);
      va[u] = pc[(size_t)i * n + j];
      vb[u] = pc[(size_t)j * n + i];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (c0 + u < nchunk) {
        a = cadd(a, va[u]);
        b = cadd(b, vb[u]);
      }
  }
}

// Load a Hermitian matrix: sum of Gram partials (fixed chunk order) or a slot,
// symmetrised, zero padded to np x np; V = I.
__device__ void load_herm(double2 *A, double2 *V, int np, int n, const double2 *part,
                          int nchunk, int which, const double2 *src, int ldsrc) {
  for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
    const int i = e / np, j = e % np;
    double2 v = make_double2(0.0, 0.0);
    if (i < n && j < n) {
      double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
      if (part) {
        sum_parts(part, nchunk, which, n, i, j, a, b);
      } else {
        a = ((const FM_GLOBAL double2 *)src)[(size_t)i * ldsrc + j];
        b = ((const FM_GLOBAL double2 *)src)[(size_t)j * ldsrc + i];
      }
      // (A + A^H) / 2
      v = make_double2(0.5 * (a.x + b.x), i == j ? 0.0 : 0.5 * (a.y - b.y));
    }
    A[e] = v;
    V[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
}

template <int NMAX, bool kBatched>
__global__ __launch_bounds__(256) void small_kernel(FrameDev single, const FrameDev *frames,
                                                    const Item *items, int mode) {
  int unused_a, unused_b;
  const FrameDev &f = frame_of<kBatched>(single, frames, items, unused_a, unused_b);
  __shared__ SmallLds<NMAX> S;
  // LDS matrices of the n <= 16 class are 16 x 16 (zero padding), the
  // one-wave solvers' shape; the wider classes use the frame's even npad
  const int n = f.n, np = NMAX == 16 ? 16 : f.npad;
  double2 *A = NMAX > 0 ? S.A : slot(f, kSlotA);
  double2 *V = NMAX > 0 ? S.V : slot(f, kSlotV);
  if (threadIdx.x == 0) S.st = 0u;

  if (mode == kOrth) {
    load_herm(A, V, np, n, f.part, f.nchunk, 0, nullptr, 0);
    double2 *T = slot(f, kSlotT);
    // V_new = Y L^-H with Gram = L L^H (Cholesky, L^-1 in V).  Only span(V)
    // matters downstream (the Nystrom approximation is the same for any basis
    // of it); a small pivot -- an ill-conditioned or rank-deficient sketch --
    // falls back to the eigen route below.
    {
      double dmax = 0.0;
      for (int i = 0; i < n; ++i) dmax = fmax(dmax, A[(size_t)i * np + i].x);
      if (dmax > 0.0 && chol_small<NMAX>(A, V, S.inv, np, n, dmax, &S.flag)) {
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
          const int i = e / n, k = e % n;  // T[i][k] = conj(Linv[k][i])
          const double2 x = V[(size_t)k * np + i];
          T[e] = make_double2(x.x, -x.y);
        }
        return;
      }
      // the failed attempt overwrote A: reload the Gram for the eigen route
      if (threadIdx.x == 0) *wstat_of(f) |= FM_ST_ORTH_FALLBACK;
      load_herm(A, V, np, n, f.part, f.nchunk, 0, nullptr, 0);
    }
    // V_new = Y E diag(lambda^-1/2): orthonormal basis of the sketch
    const int sw = eigh_small<NMAX>(A, V, np, S.rot, S.red, &S.sweeps);
    sort_desc(A, np, n, S.perm, S.w);
    const double thr = kRcondOrth * S.w[0];
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = e / n, k = e % n;
      const double lam = S.w[k];
      double2 v = make_double2(0.0, 0.0);
      if (lam > 0.0 && lam > thr) {
        const double sc = 1.0 / sqrt(lam);
        const double2 x = V[(size_t)i * np + S.perm[k]];
        v = make_double2(x.x * sc, x.y * sc);
      }
      T[e] = v;
    }
    if (threadIdx.x == 0 && sw < 0) *wstat_of(f) |= FM_ST_EIG_MAXIT;
    return;
  }

  // ---- final: core -> P, H = P^H Gc P -> W, sigma; T_f = P W_K sigma^-1/2 ----
  const bool sample = f.method == FM_METHOD_SAMPLE || f.method == FM_METHOD_SAMPLE_X;
  // Gc (sum of partials, symmetrised) parked in its slot
  constexpr bool kProdLds = SmallLds<NMAX>::kProdLds;
  double2 *Gc = kProdLds ? S.Gc : slot(f, kSlotGc);
  for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
    const int i = e / np, j = e % np;
    double2 v = make_double2(0.0, 0.0);
    if (i < n && j < n) {
      double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
      sum_parts(f.part, f.nchunk, 1, n, i, j, a, b);
      v = make_double2(0.5 * (a.x + b.x), i == j ? 0.0 : 0.5 * (a.y - b.y));
      // a NaN or Inf anywhere in X or R reaches every entry of the sketch's
      // (or the sampled columns') Gram matrix
      if (!isfinite(v.x) || !isfinite(v.y)) atomicOr(&S.st, (unsigned)FM_ST_NONFINITE);
    }
    Gc[e] = v;
  }
  auto load_core = [&]() {
    if (sample) load_herm(A, V, np, n, nullptr, 0, 0, slot(f, kSlotCore), f.npad);
    else load_herm(A, V, np, n, f.part, f.nchunk, 0, nullptr, 0);
  };
  load_core();
  double2 *P = kProdLds ? S.P : slot(f, kSlotP);
  // P with P P^H = core^+ (eq. (8)).  Cholesky route: core = L L^H and
  // P = L^-H, taken when the bounds lambda_min >= 1 / ||L^-1||_F^2 and
  // lambda_max <= trace show that the pseudo-inverse's threshold keeps every
  // direction (then core^+ = core^-1 exactly); otherwise the eigen route
  // P = E_r diag(lambda^-1/2) over the kept eigenpairs.
  bool chol = false;
  {
    double dmax = 0.0, tr = 0.0;
    for (int i = 0; i < n; ++i) {
      const double d = A[(size_t)i * np + i].x;
      dmax = fmax(dmax, d);
      tr += d;
    }
    if (dmax > 0.0 && chol_small<NMAX>(A, V, S.inv, np, n, dmax, &S.flag)) {
      double nrm = 0.0, unused = 0.0;
      for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, c = e % n;
        const double2 x = V[(size_t)i * np + c];
        if (c <= i) nrm += x.x * x.x + x.y * x.y;
      }
      block_sum2(nrm, unused, S.red);
      // (false for NaN: such a core takes the eigen route, which reports it)
      chol = nrm * tr * f.rcond < 0.5;
    }
  }
  int sw = 0;
  if (chol) {
    for (int e = threadIdx.x; e < n * np; e += blockDim.x) {
      const int i = e / np, k = e % np;
      const double2 x = k < n ? V[(size_t)k * np + i] : make_double2(0.0, 0.0);
      P[e] = make_double2(x.x, -x.y);
    }
    if (threadIdx.x == 0) S.rank = n;
    __syncthreads();
  } else {
    load_core();
    sw = eigh_small<NMAX>(A, V, np, S.rot, S.red, &S.sweeps);
    if (threadIdx.x == 0 && sw < 0) S.st |= FM_ST_EIG_MAXIT;
    sort_desc(A, np, n, S.perm, S.w);
    if (threadIdx.x == 0) {
      const double thr = f.rcond * S.w[0];
      int r = 0;
      for (int k = 0; k < n; ++k)
        if (S.w[k] > thr && S.w[k] > 0.0) ++r;
      S.rank = r;
      // the pseudo-inverse of eq. (8) dropped directions of the core
      if (r < n) S.st |= FM_ST_CORE_TRUNCATED;
      if (!isfinite(S.w[0])) S.st |= FM_ST_NONFINITE;
    }
    __syncthreads();
    const int rk = S.rank;
    // P = E_r diag(lambda^-1/2)   (n x r1, ld np)
    for (int e = threadIdx.x; e < n * np; e += blockDim.x) {
      const int i = e / np, k = e % np;
      double2 v = make_double2(0.0, 0.0);
      if (k < rk) {
        const double sc = 1.0 / sqrt(S.w[k]);
        const double2 x = V[(size_t)i * np + S.perm[k]];
        v = make_double2(x.x * sc, x.y * sc);
      }
      P[e] = v;
    }
    __syncthreads();
  }
  const int r1 = S.rank;
  const int rp = NMAX == 16 ? 16 : (r1 + 1) & ~1;
  // Z = Gc P  (n x r1)
  double2 *Z = kProdLds ? S.Z : slot(f, kSlotZ);
  for (int e = threadIdx.x; e < n * r1; e += blockDim.x) {
    const int i = e / r1, k = e % r1;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < n; ++j) acc = cadd(acc, cmul(Gc[(size_t)i * np + j], P[(size_t)j * np + k]));
    Z[(size_t)i * np + k] = acc;
  }
  __syncthreads();
  // H = P^H Z  (r1 x r1, padded to rp), into A; V = I
  for (int e = threadIdx.x; e < rp * rp; e += blockDim.x) {
    const int a = e / rp, b = e % rp;
    double2 acc = make_double2(0.0, 0.0);
    if (a < r1 && b < r1)
      for (int j = 0; j < n; ++j)
        acc = cadd(acc, cmulc(P[(size_t)j * np + a], Z[(size_t)j * np + b]));
    A[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rp * rp; e += blockDim.x) {
    const int a = e / rp, b = e % rp;
    if (a < r1 && b < r1 && a <= b) {
      const double2 x = A[(size_t)a * rp + b], y = A[(size_t)b * rp + a];
      const double2 h = make_double2(0.5 * (x.x + y.x), a == b ? 0.0 : 0.5 * (x.y - y.y));
      A[(size_t)a * rp + b] = h;
      A[(size_t)b * rp + a] = make_double2(h.x, -h.y);
    }
    V[e] = make_double2(a == b ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (rp > 0) {
    sw = eigh_small<NMAX>(A, V, rp, S.rot, S.red, &S.sweeps);
    if (threadIdx.x == 0 && sw < 0) S.st |= FM_ST_EIG_MAXIT;
    sort_desc(A, rp, r1, S.perm, S.w);
  }
  // T_f = P W_K diag(sigma^-1/2)  (n x K, ld K)
  const int K = f.K;
  double2 *Tf = slot(f, kSlotT);
  for (int e = threadIdx.x; e < n * K; e += blockDim.x) {
    const int i = e / K, k = e % K;
    double2 acc = make_double2(0.0, 0.0);
    if (k < r1 && S.w[k] > 0.0) {
      const int col = S.perm[k];
      for (int j = 0; j < r1; ++j) acc = cadd(acc, cmul(P[(size_t)i * np + j], V[(size_t)j * rp + col]));
      const double sc = 1.0 / sqrt(S.w[k]);
      acc = make_double2(acc.x * sc, acc.y * sc);
    }
    Tf[e] = acc;
  }
  __syncthreads();
  // every eigenvalue of S~, for the model-order estimate
  if (f.eig)
    for (int k = threadIdx.x; k < n; k += blockDim.x)
      f.eig[k] = (k < r1 && S.w[k] > 0.0) ? S.w[k] : 0.0;
  if (threadIdx.x == 0) {
    unsigned st = S.st | *wstat_of(f);
    for (int k = 0; k < K; ++k) {
      const bool ok = k < r1 && S.w[k] > 0.0;
      f.sigma[k] = ok ? S.w[k] : 0.0;
      if (!ok) st |= FM_ST_RANK_DEFICIENT;
    }
    *f.status = st;
  }
}

// ---------------------------------------------------------------------------
// apply: V = Y T (ORTH, complex64 [M][n]) or U_s = C T_f (FINAL, complex128
// [K][M] plus the FP32 copy Uf [M][K] used by the spectrum pass)
// ---------------------------------------------------------------------------
// T (n x ncol complex128) and the chunk's rows of Y are staged in LDS when
// T fits (n * ncol <= kApplyTMax); Y is staged column-major so that the
// lanes of a wave (consecutive rows) read consecutive words.
constexpr int kApplyTMax = 1024;
template <bool kBatched>
__global__ __launch_bounds__(256) void apply_kernel(FrameDev single, const FrameDev *frames,
                                                    const Item *items, int mode) {
  __shared__ double2 ts[kApplyTMax];
  __shared__ float2 ys[kApplyRows * kMaxL];
  int chunk, unused;
  const FrameDev &f = frame_of<kBatched>(single, frames, items, chunk, unused);
  const int n = f.n, M = f.M;
  const int m0 = chunk * kApplyRows;
  const int rows = min(M, m0 + kApplyRows) - m0;
  const double2 *Tm = slot(f, kSlotT);
  const float2 *Y = f.Y;
  const int ncol = mode == kApplyV ? n : f.K;
  const bool staged = n * ncol <= kApplyTMax && n <= kMaxL;
  // one output (row m, column c) per thread and pass; the two paths are
  // separate loops so that each reads through its own address space (a
  // select between LDS and global pointers would make every read a flat
  // load with a full wait)
  auto put = [&](int c, int m, double2 acc) {
    if (mode == kApplyV) {
      ((FM_GLOBAL float2 *)f.V)[(size_t)m * n + c] = make_float2((float)acc.x, (float)acc.y);
    } else {
      ((FM_GLOBAL double2 *)f.Us)[(size_t)c * M + m] = acc;
      ((FM_GLOBAL float2 *)f.Uf)[(size_t)m * ncol + c] =
          make_float2((float)acc.x, (float)acc.y);
    }
  };
  auto mac = [](double2 &acc, float2 y, double2 t) {
    acc.x = fma((double)y.x, t.x, acc.x);
    acc.x = fma(-(double)y.y, t.y, acc.x);
    acc.y = fma((double)y.x, t.y, acc.y);
    acc.y = fma((double)y.y, t.x, acc.y);
  };
  if (staged) {
    const gdouble2 *Tg = (const gdouble2 *)Tm;
    const gfloat2 *Yg = (const gfloat2 *)Y;
    for (int e = threadIdx.x; e < n * ncol; e += blockDim.x) ts[e] = Tg[e];
    for (int e = threadIdx.x; e < rows * n; e += blockDim.x) {
      const int m = e / n, j = e % n;
      ys[j * kApplyRows + m] = Yg[(size_t)(m0 + m) * n + j];
    }
    __syncthreads();
    // V ([M][n]) is written with the column fastest across a wave (whole
    // rows: coalesced), U_s ([K][M]) with the row fastest
    const bool cfast = mode == kApplyV;
    for (int e = threadIdx.x; e < rows * ncol; e += blockDim.x) {
      const int c = cfast ? e % ncol : e / rows, ml = cfast ? e / ncol : e % rows;
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
      for (int j = 0; j < n; ++j) mac(acc, ys[j * kApplyRows + ml], ts[j * ncol + c]);
      put(c, m0 + ml, acc);
    }
  } else {
    const gdouble2 *Tg = (const gdouble2 *)Tm;
    const gfloat2 *Yg = (const gfloat2 *)Y;
    for (int e = threadIdx.x; e < rows * ncol; e += blockDim.x) {
      const int c = e / rows, ml = e % rows, m = m0 + ml;
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
      for (int j = 0; j < n; ++j) mac(acc, Yg[(size_t)m * n + j], Tg[(size_t)j * ncol + c]);
      put(c, m, acc);
    }
  }
}

inline dim3 grid1(const FrameDev &single, const Item *items, int n_items, int per_frame) {
  return dim3(items ? n_items : per_frame);
}

}  // namespace

hipError_t launch_omega(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, int to_y, hipStream_t s) {
  const int per = (single.M + kApplyRows - 1) / kApplyRows;
  if (items) hipLaunchKernelGGL(omega_kernel<true>, dim3(n_items), dim3(256), 0, s, single, frames, items, to_y);
  else hipLaunchKernelGGL(omega_kernel<false>, dim3(per), dim3(256), 0, s, single, frames, items, to_y);
  return hipGetLastError();
}

hipError_t launch_sketch(const FrameDev &single, const FrameDev *frames, const Item *items,
                         int n_items, int nb, int round, int split, hipStream_t s) {
  const int S = split == 1 ? sketch_segments(single.M, nb) : 1;
  const dim3 g(items ? n_items : S * ((single.M + kSketchRows - 1) / kSketchRows)), b(256);
  // (every class gets the round: the first product reads the test matrix;
  // only the classes n <= 32 form Gram partials with it)
#define FM_SK(NB)                                                                                           \
  if (items) hipLaunchKernelGGL((sketch_kernel<NB, true>), g, b, 0, s, single, frames, items, round, split); \
  else hipLaunchKernelGGL((sketch_kernel<NB, false>), g, b, 0, s, single, frames, items, round, split);
  switch (nb) {
    case 1: FM_SK(1); break;
    case 2: FM_SK(2); break;
    case 3: FM_SK(3); break;
    default: FM_SK(4); break;
  }
#undef FM_SK
  return hipGetLastError();
}

hipError_t launch_xhv(const FrameDev &single, const FrameDev *frames, const Item *items,
                      int n_items, int nb, hipStream_t s) {
  const dim3 g(items ? n_items : (single.T + kXhvCols - 1) / kXhvCols), b(256);
#define FM_XH(NB)                                                                            \
  if (items) hipLaunchKernelGGL((xhv_kernel<NB, true>), g, b, 0, s, single, frames, items);  \
  else hipLaunchKernelGGL((xhv_kernel<NB, false>), g, b, 0, s, single, frames, items);
  switch (nb) {
    case 1: FM_XH(1); break;
    case 2: FM_XH(2); break;
    case 3: FM_XH(3); break;
    default: FM_XH(4); break;
  }
#undef FM_XH
  return hipGetLastError();
}

hipError_t launch_xz(const FrameDev &single, const FrameDev *frames, const Item *items,
                     int n_items, int nb, int round, hipStream_t s) {
  const dim3 g(items ? n_items : (single.M + kSketchRows - 1) / kSketchRows), b(256);
  const int rd = nb <= 2 ? round : -1;
#define FM_XZ(NB)                                                                                \
  if (items) hipLaunchKernelGGL((xz_kernel<NB, true>), g, b, 0, s, single, frames, items, rd);  \
  else hipLaunchKernelGGL((xz_kernel<NB, false>), g, b, 0, s, single, frames, items, rd);
  switch (nb) {
    case 1: FM_XZ(1); break;
    case 2: FM_XZ(2); break;
    case 3: FM_XZ(3); break;
    default: FM_XZ(4); break;
  }
#undef FM_XZ
  return hipGetLastError();
}

hipError_t launch_zx(const FrameDev &single, const FrameDev *frames, const Item *items,
                     int n_items, hipStream_t s) {
  const dim3 g(items ? n_items : (single.T + kZxCols - 1) / kZxCols), b(256);
  if (items) hipLaunchKernelGGL(zx_kernel<true>, g, b, 0, s, single, frames, items);
  else hipLaunchKernelGGL(zx_kernel<false>, g, b, 0, s, single, frames, items);
  return hipGetLastError();
}

hipError_t launch_xcore(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, hipStream_t s) {
  const dim3 g(items ? n_items : 1), b(256);
  if (items) hipLaunchKernelGGL(xcore_kernel<true>, g, b, 0, s, single, frames, items);
  else hipLaunchKernelGGL(xcore_kernel<false>, g, b, 0, s, single, frames, items);
  return hipGetLastError();
}

hipError_t launch_gather(const FrameDev &single, const FrameDev *frames, const Item *items,
                         int n_items, hipStream_t s) {
  const int per = (single.M + kApplyRows - 1) / kApplyRows;
  if (items) hipLaunchKernelGGL(gather_kernel<true>, dim3(n_items), dim3(256), 0, s, single, frames, items);
  else hipLaunchKernelGGL(gather_kernel<false>, dim3(per), dim3(256), 0, s, single, frames, items);
  return hipGetLastError();
}

hipError_t launch_gram(const FrameDev &single, const FrameDev *frames, const Item *items,
                       int n_items, int mode, hipStream_t s) {
  const int per = (single.M + kGramRows - 1) / kGramRows;
  if (items) hipLaunchKernelGGL(gram_kernel<true>, dim3(n_items), dim3(256), 0, s, single, frames, items, mode);
  else hipLaunchKernelGGL(gram_kernel<false>, dim3(per), dim3(256), 0, s, single, frames, items, mode);
  return hipGetLastError();
}

// The plan sorts frames by n; each launch covers frames of one LDS class.
hipError_t launch_small(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, int mode, hipStream_t s) {
  // class of the launch = the largest n among its frames, passed in single.n
  const int n = single.n;
  const dim3 g(items ? n_items : 1), b(256);
  if (n <= 16) {
    if (items) hipLaunchKernelGGL((small_kernel<16, true>), g, b, 0, s, single, frames, items, mode);
    else hipLaunchKernelGGL((small_kernel<16, false>), g, b, 0, s, single, frames, items, mode);
  } else if (n <= 32) {
    if (items) hipLaunchKernelGGL((small_kernel<32, true>), g, b, 0, s, single, frames, items, mode);
    else hipLaunchKernelGGL((small_kernel<32, false>), g, b, 0, s, single, frames, items, mode);
  } else if (n <= kSmallLdsN) {
    if (items) hipLaunchKernelGGL((small_kernel<kSmallLdsN, true>), g, b, 0, s, single, frames, items, mode);
    else hipLaunchKernelGGL((small_kernel<kSmallLdsN, false>), g, b, 0, s, single, frames, items, mode);
  } else {
    if (items) hipLaunchKernelGGL((small_kernel<0, true>), g, b, 0, s, single, frames, items, mode);
    else hipLaunchKernelGGL((small_kernel<0, false>), g, b, 0, s, single, frames, items, mode);
  }
  return hipGetLastError();
}

hipError_t launch_apply(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, int mode, hipStream_t s) {
  const int per = (single.M + kApplyRows - 1) / kApplyRows;
  if (items) hipLaunchKernelGGL(apply_kernel<true>, dim3(n_items), dim3(256), 0, s, single, frames, items, mode);
  else hipLaunchKernelGGL(apply_kernel<false>, dim3(per), dim3(256), 0, s, single, frames, items, mode);
  return hipGetLastError();
}

}  // namespace fm
