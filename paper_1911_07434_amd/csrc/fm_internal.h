// fm_internal.h -- internal descriptors and launcher declarations of the
// gfx950 fast-MUSIC library (not installed; the public ABI is fastmusic.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "fastmusic.h"

// Global address space for device-side loads through FrameDev's generic
// pointers (global_load instead of flat_load); host passes see a plain type.
#if defined(__HIP_DEVICE_COMPILE__)
#define FM_GLOBAL __attribute__((address_space(1)))
#define FM_LDS __attribute__((address_space(3)))
#else
#define FM_GLOBAL
#define FM_LDS
#endif

namespace fm {

// Everything one frame needs on the device: caller buffers (inputs and
// outputs) plus the frame's slice of workspace.  Batched launches read an
// array of these; single-frame launches pass one by value.
struct FrameDev {
  // stage 1: covariance
  const float2 *X;
  long long ldx;
  int M, T;
  float2 *R;
  long long ldr;
  // stage 2: subspace
  int K, method, n, q;
  double rcond;
  const float *Omega;   // [M][n] real Gaussian (Method 2)
  const int *idx;       // [n] sampled columns (Method 1)
  double2 *Us;          // [K][M] complex128
  double *sigma;        // [K]
  unsigned *status;     // [1]
  // stages 3-4: spectrum and peaks
  int L;
  double theta0, dtheta;
  float *P;
  int *peak_idx;
  float *peak_val;
  int *n_found;
  // workspace (device)
  float2 *Y;            // [M][n] sketch C (= R V, or gathered columns)
  float2 *V;            // [M][n] orthonormal basis fed to the next product
  float2 *Z;            // [T][n] X^H V (products with R formed from X, no R)
  double2 *part;        // [nchunk][2][n][n] Gram partial sums
  double2 *small;       // small dense scratch, kSmallSlots * npad^2
  float2 *Uf;           // FP32 pass: [M][K] FP32 copy of U_s; FP16 pass: scaled
                        // hi and lo planes [K][M] of (re, im) FP16 pairs
  int *rlist;           // [1 + L]: count, then angles whose FP32 denominator needs FP64
  double *eig;          // [n]: every eigenvalue of S~ (descending, 0 past its rank)
  // FP32 spectrum as a polynomial in sin(theta): frames of equal M and grid
  // share a group buffer hgrp [acorr_blocks(M)][M][kPolyRows] (column hslot:
  // this frame's partial sums of conj(h'_d) over each block of kAcorrRows
  // rows); hmem lists the group's frames (plan indices), hcount of them
  float2 *hgrp;
  const int *hmem;
  int hslot, hcount;
  // FP32 covariance with its T segments on separate waves: per unit and
  // segment the wave's (Re, Im) sums, [unit][segment][64 values][64 lanes]
  float *cpart;
  // Method 2 products with their channel segments on separate workgroups:
  // [row block][segment][column block][16][256 threads]
  float *spart;
  // model-order estimate (Sec. V-D); K_hat == null: none
  int *K_hat;           // [1]
  double *order_crit;   // [n + 1] criterion values, or null
  int order_rule;       // FM_ORDER_AIC / FM_ORDER_MDL
  // ESPRIT angles on U_s (degrees, ascending); null: none
  double *doa;
  int or_status;        // 1: OR the order / ESPRIT bits into *status (plans), 0: overwrite
  int nchunk;           // ceil(M / kGramRows)
  int npad;             // n rounded up to even
};

// work item of a batched launch: which frame and which tile of it
struct Item {
  int frame, a, b, c;
};

constexpr int kGramRows = 128;     // rows of the sketch per Gram partial
constexpr int kSmallSlots = 8;     // npad^2 complex128 matrices per frame
// the frame's workspace status word, after the small dense slots: cleared
// by the first launch of the subspace step, or-ed by the orth steps, read
// by the final small solve
__device__ inline unsigned *wstat_of(const FrameDev &f) {
  return reinterpret_cast<unsigned *>(f.small + (size_t)kSmallSlots * f.npad * f.npad);
}
constexpr int kCovTile = 128;      // 16-bit covariance: tile edge (complex entries)
constexpr int kCovBlock = 64;      // FP32 covariance: rows of a wave block (one wave per block)
constexpr int kCovPartFloats = 64 * 64;  // FP32 covariance: one segment's sums of a wave block
constexpr int kCovCols = 32;       // FP32 covariance: columns of a wave block
constexpr int kSketchRows = 128;   // rows of R per sketch workgroup
constexpr int kApplyRows = 64;     // rows per apply / gather workgroup
constexpr int kSpecChunk = 64;     // lags staged in LDS per step of the polynomial pass
constexpr int kPolyRows = 16;      // frames per polynomial-spectrum group (MFMA rows)
constexpr int kAcorrLags = 256;    // lags d per autocorrelation workgroup
constexpr int kAcorrRows = 256;    // rows m per autocorrelation workgroup (partial sums)
__host__ __device__ inline int acorr_blocks(int M) { return (M + kAcorrRows - 1) / kAcorrRows; }
constexpr int kRefineGroups = 8;   // FP64 recompute workgroups per frame
constexpr int kMaxL = 64;          // max sketch width of Method 2 (l)
constexpr int kMaxN = 256;         // max sketch width of Method 1 (p)
constexpr int kMaxK = 64;          // max number of sources
constexpr int kSmallLdsN = 64;     // small dense matrices live in LDS up to this n

// small-dense modes
enum SmallMode { kOrth = 0, kFinal = 1 };
// gram modes
// kGramFinal: Method 2 frames get V^H Y (slot 0) and Y^H Y (slot 1), Method 1
// frames get Y^H Y (slot 1); the method is read from the frame
enum GramMode { kGramSelf = 0, kGramFinal = 1 };
// apply modes
enum ApplyMode { kApplyV = 0, kApplyUs = 1 };

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files); `single` is used when items == null
// ---------------------------------------------------------------------------
hipError_t launch_covariance(const FrameDev &single, const FrameDev *frames,
                             const Item *items, int n_items, fm_prec prec, hipStream_t s);
// 16-bit operand covariance (FM_FP16 / FM_BF16, or split hi + lo with
// FM_FP16X3 / FM_BF16X3), FP32 accumulation
// FP32 covariance, T segments on separate waves: mode 0 writes each
// (unit, segment)'s sums to cpart (items {frame, bi, bj, g}, or a single
// frame's units x segments), mode 1 reduces them in order and stores R
// (items {frame, bi, bj, 0}, or a single frame's units)
hipError_t launch_covariance_split(const FrameDev &single, const FrameDev *frames,
                                   const Item *items, int n_items, int mode, hipStream_t s);
hipError_t launch_covariance16(const FrameDev &single, const FrameDev *frames,
                               const Item *items, int n_items, fm_prec prec, hipStream_t s);
hipError_t launch_omega(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, int to_y, hipStream_t s);
// nb = ceil(2n / 32): MFMA column blocks of the sketch (one launch per class).
// round >= 0: index of this product among the frame's q + 1; for nb <= 2 the
// launch also writes the Gram partials of the step that follows (kGramSelf
// if round < q, else kGramFinal), which then needs no gram launch.  round < 0:
// sketch only.  split (channel segments, sketch_segments): 0 in turn, 1 one
// workgroup per (row block, segment) writing spart (items {frame, block, 0,
// segment}, or a single frame's blocks x segments), 2 the in-order reduction
// and the epilogue (items {frame, block, 0, 0}).
hipError_t launch_sketch(const FrameDev &single, const FrameDev *frames, const Item *items,
                         int n_items, int nb, int round, int split, hipStream_t s);
// whether a sketch of this column class forms its Gram partials itself
inline bool sketch_fuses_gram(int nb) { return nb <= 2; }
// compensated FP16 sketch (16-bit plans and calls), nb <= 2 only; forms the
// Gram partials like launch_sketch
hipError_t launch_sketch16(const FrameDev &single, const FrameDev *frames, const Item *items,
                           int n_items, int nb, int round, int split, hipStream_t s);
inline bool sketch16_ok(int nb) { return nb <= 2; }
// Method 2 products with R sum the M channels in sketch_segments(M, nb)
// fixed segments of whole 32-channel chunks (the ragged chunk in the last):
// each segment's products accumulate from zero and the segment sums are
// added in order.  A workgroup runs the segments in turn, or one workgroup
// per segment writes its sums to spart and a reduction workgroup adds them
// in the same order: the same bits.  The count depends on the frame's shape
// only (at least four chunks per segment, at most 8; one for the wide
// column classes).
inline __host__ __device__ int sketch_segments(int M, int nb) {
  if (nb > 2) return 1;
  const int c = (M >> 5) / 4;
  return c < 1 ? 1 : (c > 8 ? 8 : c);
}
inline __host__ __device__ int sketch_seg_chunk(int s, int S, int nfull) { return s * nfull / S; }
// floats of one sketch workgroup's sums of one segment, per column block
constexpr int kSketchPartFloats = 16 * 256;
// products with R without forming it (Method 2 from X): R V = X (X^H V) / T.
// launch_xhv: Z = X^H V (one workgroup per 128 snapshots); launch_xz:
// Y = X Z / T, Gram partials as launch_sketch (one workgroup per 128 rows)
hipError_t launch_xhv(const FrameDev &single, const FrameDev *frames, const Item *items,
                      int n_items, int nb, hipStream_t s);
hipError_t launch_xz(const FrameDev &single, const FrameDev *frames, const Item *items,
                     int n_items, int nb, int round, hipStream_t s);
constexpr int kXhvCols = 128;  // snapshots per xhv workgroup
// Method 1 without forming R: launch_zx writes Z[t][j] = conj(X[idx_j][t])
// (one workgroup per 64 snapshots), launch_xz (round < 0) forms
// C = R(:, I) = X Z / T, launch_xcore takes core = C(I, :) and checks I
// (one workgroup per frame).  p <= 64.
hipError_t launch_zx(const FrameDev &single, const FrameDev *frames, const Item *items,
                     int n_items, hipStream_t s);
hipError_t launch_xcore(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, hipStream_t s);
constexpr int kZxCols = 64;  // snapshots per zx workgroup
// model order from the eigenvalues f.eig and the trace of f.R (one
// workgroup per frame)
hipError_t launch_order(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, hipStream_t s);
// least-squares ESPRIT on U_s (one 64-lane workgroup per frame, K <= 32)
hipError_t launch_esprit(const FrameDev &single, const FrameDev *frames, const Item *items,
                         int n_items, hipStream_t s);
constexpr int kEspritMaxK = 32;
hipError_t launch_gather(const FrameDev &single, const FrameDev *frames, const Item *items,
                         int n_items, hipStream_t s);
hipError_t launch_gram(const FrameDev &single, const FrameDev *frames, const Item *items,
                       int n_items, int mode, hipStream_t s);
hipError_t launch_small(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, int mode, hipStream_t s);
hipError_t launch_apply(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, int mode, hipStream_t s);
hipError_t launch_uf(const FrameDev &single, hipStream_t s);
// spectrum stage = prep (reset the recompute lists; batched only -- the
// single-frame path resets it in launch_uf), a bulk pass (the FP32
// polynomial pass of fm_poly.hip, or the compensated FP16 pass) and the
// FP64 recompute of the listed angles
hipError_t launch_spec_prep(const FrameDev *frames, const Item *items, int n_items,
                            hipStream_t s);
// compensated FP16 pass: launch_split writes the hi and lo planes of U_s
// (one workgroup per 256 entries; resets the recompute list), then one
// spectrum16 launch per class nb = ceil(K / 8) over tiles of 64 nnb angles
hipError_t launch_split(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, hipStream_t s);
hipError_t launch_spectrum16(const FrameDev &single, const FrameDev *frames, const Item *items,
                             int n_items, int nb, int nnb, hipStream_t s);
// FP32 spectrum as a polynomial in u = sin(theta): launch_acorr writes each
// frame's lag sums h'_d into its group buffer as partial sums over blocks of
// kAcorrRows rows (one two-wave workgroup per 256 lags and row block; reads U_s),
// launch_hsum adds a group's partials in block order into the first block
// (hsum_chunks(M) workgroups per group), launch_poly evaluates a group of up
// to 16 frames over tiles of 64 nnb angles (nnb in {1, 2, 4}); the items of
// the last two name the group's first frame
// wide: one lag per lane, 64 lags per workgroup (four times the
// workgroups, the same bits), for single frames and small plans
hipError_t launch_acorr(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, int wide, hipStream_t s);
inline int acorr_lags(int wide) { return wide ? 64 : kAcorrLags; }
int hsum_chunks(int M);
hipError_t launch_hsum(const FrameDev &single, const FrameDev *frames, const Item *items,
                       int n_items, hipStream_t s);
hipError_t launch_poly(const FrameDev &single, const FrameDev *frames, const Item *items,
                       int n_items, int nnb, hipStream_t s);
hipError_t launch_refine(const FrameDev &single, const FrameDev *frames, const Item *items,
                         int n_items, hipStream_t s);
hipError_t launch_peaks(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, hipStream_t s);

// Covariance work units of one frame.  16-bit: one workgroup per unit of
// 128x128 tiles: off-diagonal tiles (a, b < a), diagonal tiles in pairs
// (a, b > a) and, for an odd number of row tiles, the middle diagonal tile
// alone (kinds below, in Item::c).  FP32: one wave per 64x32 block (bi, bj)
// with bj <= 2 bi + 1 (the blocks of 64-row block bi that reach the
// diagonal), bj < ceil(M / 32).
enum Cov16Kind { kCov16Off = 0, kCov16Diag2 = 1, kCov16Diag1 = 2 };
inline int cov_edge(fm_prec prec) { return prec == FM_FP32 ? kCovBlock : kCovTile; }

// units a single-frame launch covers (FP32: whole block rows; units whose
// columns start past M exit at once)
inline int cov_units(int M, fm_prec prec) {
  const int e = cov_edge(prec);
  const int nt = (M + e - 1) / e;
  return prec == FM_FP32 ? nt * (nt + 1) : nt * (nt - 1) / 2 + (nt + 1) / 2;
}

// The FP32 covariance sums T in cov_segments(M, T) fixed segments of whole
// 8-snapshot chunks (the ragged tail in the last): each segment's Gauss
// products accumulate from zero, and R = (((0 + S_0) + S_1) + ...) / T.  A
// wave runs the segments in turn, or one wave per segment writes S_g and a
// reduction wave adds them in the same order: the same bits either way.  The
// count depends on the frame's shape only: enough segments for about 2048
// waves (two per SIMD) per frame, at most 8, each at least 32 chunks.
inline __host__ __device__ int cov_segments(int M, int T) {
  const int nt = (M + 63) / 64;  // kCovBlock rows per block row
  const int by_waves = 2048 / (nt * (nt + 1));
  const int by_len = (T >> 3) / 32;
  const int g = by_waves < by_len ? by_waves : by_len;
  return g < 1 ? 1 : (g > 8 ? 8 : g);
}
// first chunk of segment g of G over nfull chunks
inline __host__ __device__ int cov_seg_chunk(int g, int G, int nfull) { return g * nfull / G; }
// unit index of FP32 block (bi, bj): block row bi holds units bi (bi + 1) ..
inline __host__ __device__ int cov_unit_index(int bi, int bj) { return bi * (bi + 1) + bj; }

namespace detail {
// 16-bit units of the row tiles [lo, lo + n) of a frame in an order where
// each run of 32 consecutive units touches few row tiles: a triangle of at
// most 8 row tiles is 32 units or fewer (its off-diagonal tiles, then its
// diagonal pairs); a larger one is split into two triangles and the square
// between them, cut into rectangles of at most 32 tiles.  The sub-block
// products do not depend on which tile a diagonal tile is paired with, so
// this order and the single-frame launch's give the same bits.
template <class F>
inline void cov16_square(int r0, int nr, int c0, int nc, F &fn) {
  if (nr * nc <= 32) {
    for (int a = r0; a < r0 + nr; ++a)
      for (int b = c0; b < c0 + nc; ++b) fn(a, b, (int)kCov16Off);
  } else if (nr >= nc) {
    cov16_square(r0, nr / 2, c0, nc, fn);
    cov16_square(r0 + nr / 2, nr - nr / 2, c0, nc, fn);
  } else {
    cov16_square(r0, nr, c0, nc / 2, fn);
    cov16_square(r0, nr, c0 + nc / 2, nc - nc / 2, fn);
  }
}
// `pend`: a diagonal tile left over by an odd triangle, waiting for a partner
template <class F>
inline void cov16_triangle(int lo, int n, int &pend, F &fn) {
  if (n <= 8) {
    for (int a = lo + 1; a < lo + n; ++a)
      for (int b = lo; b < a; ++b) fn(a, b, (int)kCov16Off);
    for (int d = 0; d < n / 2; ++d) fn(lo + d, lo + n - 1 - d, (int)kCov16Diag2);
    if (n % 2) {
      if (pend >= 0) {
        fn(pend, lo + n / 2, (int)kCov16Diag2);
        pend = -1;
      } else {
        pend = lo + n / 2;
      }
    }
    return;
  }
  const int h = n / 2;
  cov16_triangle(lo, h, pend, fn);
  cov16_square(lo + h, n - h, lo, h, fn);
  cov16_triangle(lo + h, n - h, pend, fn);
}
}  // namespace detail

// every non-empty unit (a, b, kind) of a frame: FP32 in row order (kind 0),
// 16-bit in the locality order above
template <class F>
inline void cov_each_unit(int M, fm_prec prec, F &&fn) {
  const int e = cov_edge(prec);
  const int nt = (M + e - 1) / e;
  if (prec == FM_FP32) {
    for (int a = 0; a < nt; ++a)
      for (int b = 0; b <= 2 * a + 1 && b * kCovCols < M; ++b) fn(a, b, 0);
  } else {
    int pend = -1;
    detail::cov16_triangle(0, nt, pend, fn);
    if (pend >= 0) fn(pend, pend, (int)kCov16Diag1);
  }
}

// largest leading dimension of X the 16-bit covariance takes: it addresses
// a 128-row tile of X through 32-bit byte offsets (128 ldx 8 <= 2^32)
constexpr long long kCov16MaxLdx = 1LL << 22;

}  // namespace fm
