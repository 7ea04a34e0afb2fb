// fm_cov16.hip -- stage 1 with 16-bit operands: R = X X^H / T with the
// snapshots rounded to FP16 or BF16 and FP32 accumulation (eqs. (2)-(3)).
//
// v_mfma_f32_32x32x16_{f16,bf16}: K = 16 real values = 8 complex snapshots
// in the interleaved (re, im) order of X, so
//   Re R_ij = x^_i . x^_j          (x^ = the interleaved row)
//   Im R_ij = x'_i . x^_j,  x' = (im, -re) pairs of the row
// and a 32x32 complex sub-block costs two MFMAs per 8 snapshots.
//
// Work units.  A frame's rows form N = ceil(M / 128) row tiles; its lower
// triangle is covered by N (N - 1) / 2 off-diagonal 128x128 tiles (kind
// kOff: row tile a, column tile b < a) and the N diagonal tiles taken in
// pairs (kind kDiag2: tiles a and b, a < b) plus, for odd N, one single
// diagonal tile (kDiag1).  Every unit stages two 128-row planes of
// snapshots (a diagonal pair stages its two tiles), so all units move the
// same bytes, and a frame is N^2 / 2 units (even N): 32 at M = 1024, 128 at
// M = 2048, a power of two whenever N is.
//
// One eight-wave workgroup per unit and per CU.  An off-diagonal tile is 16
// sub-blocks of 32x32, two per wave; a diagonal tile's lower triangle is 10
// sub-blocks, spread 3, 3, 2, 2 over four waves.  The operands come from
// LDS: each stage holds kBK snapshots of both planes, converted to 16 bits
// on the way in, double buffered, with the next two stages' global loads
// in flight in registers; rows are padded by 16 bytes so the 16-byte MFMA
// operand reads of 32 consecutive rows do not collide in a bank.
//
// Batched launches take the units from a list the plan orders so that the
// units of one frame reach one XCD together (its L2 then fetches each
// window of snapshots once for all of them).
//
// Split variant (kSplit, precisions FM_FP16X3 / FM_BF16X3): each snapshot is
// written as hi + lo with hi its 16-bit rounding and lo the 16-bit rounding
// of the remainder, and a sub-block accumulates lo*hi + hi*lo + hi*hi (the
// lo*lo term is below FP32 rounding of the sum), six MFMAs per sub-block per
// 8 snapshots.  The products are exact in FP32, so the result carries
// FP32-level error (FP16: 22 significant bits per operand, BF16: 16).  Both
// halves of a stage sit in LDS; stages hold 16 snapshots.
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

constexpr int kThreads = 512;  // four MFMA waves, then four loader waves
constexpr int kLoaders = 256;  // loader threads
constexpr int kSub = 32;       // MFMA sub-block edge
constexpr int kBufs = 3;       // LDS stage ring

// Stage geometry: kBK snapshots per stage, LDS rows of 2 kBK halves plus 16
// bytes of padding, planes of 128 such rows (A, B, and for the split variant
// A lo, B lo).  Each loader thread loads kPasses float4 (two snapshots) per
// plane and stage.
template <bool kSplit>
struct Geo {
  static constexpr int kBK = kSplit ? 16 : 32;
  static constexpr int kRowHalves = 2 * kBK + 8;
  static constexpr int kPlaneHalves = kCovTile * kRowHalves;
  static constexpr int kPlanes = kSplit ? 4 : 2;
  static constexpr int kStageHalves = kPlanes * kPlaneHalves;
  static constexpr int kTPR = kBK / 2;                        // loader threads per row
  static constexpr int kRowsPerPass = kLoaders / kTPR;
  static constexpr int kPasses = kCovTile / kRowsPerPass;     // per plane
  static constexpr int kLdsHalves = kBufs * kStageHalves;
};
static_assert(Geo<false>::kLdsHalves * 2 <= 160 * 1024, "LDS");
static_assert(Geo<true>::kLdsHalves * 2 <= 160 * 1024, "LDS");

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

// The frame fields a unit needs, copied out of the descriptor once.
struct Src {
  const float2 *X;
  long long ldx;
  int M, T;
};

// Buffer resource over a plane's rows: raw addressing (stride 0), no range
// limit; the byte offsets a plane needs stay below 2^32 (kCov16MaxLdx).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float2 *base) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, -1, 0x00020000);
}

// Global -> registers for one stage of one plane (row tile starting at
// row0, resource `rs` at its first row), loader thread lt: rows lt / kTPR +
// kRowsPerPass j of the plane, snapshots t0 + 2 (lt % kTPR) + {0, 1}.  The
// thread's byte offset within the plane is `off` (a VGPR, fixed for the
// unit), the pass and the stage a uniform offset (an SGPR): buffer loads
// need no per-load address registers.  With kClamp, rows past M read row
// M - 1 (their products are never stored), so each pass has its own lane
// offset.  kTail: snapshots past T read as zero.
template <bool kSplit, bool kClamp, bool kTail>
__device__ __forceinline__ void plane_load(f32x4 *v, __amdgpu_buffer_rsrc_t rs, const Src &x,
                                           int row0, unsigned off, int t0, int lt) {
  typedef Geo<kSplit> G;
  const int tp = t0 + 2 * (lt % G::kTPR);
#pragma unroll
  for (int j = 0; j < G::kPasses; ++j) {
    unsigned vo, so;
    if constexpr (!kClamp) {
      vo = off;
      so = (unsigned)(((long long)G::kRowsPerPass * j * x.ldx + t0) * 8);
    } else {
      const int row = min(row0 + lt / G::kTPR + G::kRowsPerPass * j, x.M - 1) - row0;
      vo = (unsigned)(((long long)row * x.ldx + 2 * (lt % G::kTPR)) * 8);
      so = (unsigned)t0 * 8u;
    }
    if constexpr (!kTail) {
      v[j] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0));
    } else {
      v[j] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (tp + 1 < x.T) {
        v[j] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0));
      } else if (tp < x.T) {
        const f32x2 y = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0));
        v[j].x = y.x;
        v[j].y = y.y;
      }
    }
  }
}

// registers -> LDS plane at `base` (halves), converted to 16 bits; the split
// variant also stores lo = 16-bit rounding of v - hi (exact in FP32) at
// `lo_off` halves past the hi plane
template <class H, bool kSplit>
__device__ __forceinline__ void plane_store(const f32x4 *v, H *lds, int base, int lo_off, int lt) {
  typedef Geo<kSplit> G;
  typedef H h4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int j = 0; j < G::kPasses; ++j) {
    const int row = lt / G::kTPR + G::kRowsPerPass * j;
    const int at = base + row * G::kRowHalves + 4 * (lt % G::kTPR);
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

// (im, -re) pairs of an interleaved row segment
template <class V>
__device__ __forceinline__ V swap_neg(V a) {
  V p;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    p[2 * c] = a[2 * c + 1];
    p[2 * c + 1] = -a[2 * c];
  }
  return p;
}

// MFMA wave roles: NV 32-row operand segments (LDS offsets off[v] in a
// stage) and NP sub-block products, product k = rows of segment A[k] times
// columns of segment B[k] into accumulators k.  A segment's MFMA operand
// layout is the same whether it serves as rows or as columns, so one read
// serves both.
//   Off: a 64x64 quarter (wi, wj) of an off-diagonal tile: segments
//        A[2wi], A[2wi+1], B[2wj], B[2wj+1]
//   DX:  diagonal tile sub-blocks (3,3) (3,0) (3,1) (3,2) (0,0): segments 3, 0, 1, 2
//   DY:  diagonal tile sub-blocks (2,2) (2,1) (2,0) (1,1) (1,0): segments 2, 1, 0
struct RoleOff {
  static constexpr int nv = 4, np = 4;
  static constexpr int a[5] = {0, 0, 1, 1, 0}, b[5] = {2, 3, 2, 3, 0};
};
struct RoleDX {
  static constexpr int nv = 4, np = 5;
  static constexpr int a[5] = {0, 0, 0, 0, 1}, b[5] = {0, 1, 2, 3, 1};
};
struct RoleDY {
  static constexpr int nv = 3, np = 5;
  static constexpr int a[5] = {0, 0, 0, 1, 1}, b[5] = {0, 1, 2, 1, 2};
};
enum Role { kRoleOff = 0, kRoleDX, kRoleDY, kRoleIdle };

template <class H, bool kSplit, class RD>
struct Operands {
  typedef typename Mma<H>::vec vec;
  vec v[RD::nv], vl[kSplit ? RD::nv : 1];
  __device__ __forceinline__ void read(const H *stage, const int (&off)[4], int ks) {
    constexpr int kLo = 2 * Geo<kSplit>::kPlaneHalves;
#pragma unroll
    for (int i = 0; i < RD::nv; ++i) {
      v[i] = *(const vec *)(stage + off[i] + 16 * ks);
      if constexpr (kSplit) vl[i] = *(const vec *)(stage + kLo + off[i] + 16 * ks);
    }
  }
};

// the MFMAs of one k-step (8 snapshots) on operands already in registers
template <class H, bool kSplit, class RD>
__device__ __forceinline__ void kstep(const Operands<H, kSplit, RD> &o, floatx16 (&aR)[5],
                                      floatx16 (&aI)[5]) {
  typedef typename Mma<H>::vec vec;
  vec p[RD::nv];
#pragma unroll
  for (int i = 0; i < RD::nv; ++i) p[i] = swap_neg(o.v[i]);
  if constexpr (kSplit) {
    // lo*hi and hi*lo first, then hi*hi
    vec pl[RD::nv];
#pragma unroll
    for (int i = 0; i < RD::nv; ++i) pl[i] = swap_neg(o.vl[i]);
#pragma unroll
    for (int k = 0; k < RD::np; ++k) {
      aR[k] = Mma<H>::run(o.vl[RD::a[k]], o.v[RD::b[k]], aR[k]);
      aI[k] = Mma<H>::run(pl[RD::a[k]], o.v[RD::b[k]], aI[k]);
    }
#pragma unroll
    for (int k = 0; k < RD::np; ++k) {
      aR[k] = Mma<H>::run(o.v[RD::a[k]], o.vl[RD::b[k]], aR[k]);
      aI[k] = Mma<H>::run(p[RD::a[k]], o.vl[RD::b[k]], aI[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < RD::np; ++k) {
    aR[k] = Mma<H>::run(o.v[RD::a[k]], o.v[RD::b[k]], aR[k]);
    aI[k] = Mma<H>::run(p[RD::a[k]], o.v[RD::b[k]], aI[k]);
  }
}

// An MFMA wave's whole T loop: stage st sits in LDS buffer st % 3 and is
// consumed two barriers after the loaders stored it.  The operands of
// k-step ks live in register slot ks; the reads for k-step ks + kAhead (in
// the next stage once past this one's end: stage st + 1 is published one
// barrier before stage st is consumed) are issued before the MFMAs of
// k-step ks, and a scheduling barrier keeps them there, so the LDS latency
// hides behind kAhead k-steps of MFMAs.  One barrier per stage, plus two
// leading ones, matching the loaders.
template <class H, bool kSplit, class RD>
__device__ __forceinline__ void mfma_loop(const H *lds, const int (&off)[4], int nfull, bool tail,
                                          floatx16 (&aR)[5], floatx16 (&aI)[5]) {
  typedef Geo<kSplit> G;
  constexpr int kSteps = G::kBK / 8;
  constexpr int kAhead = kSteps > 2 ? 2 : 1;
  Operands<H, kSplit, RD> o[kSteps];
  __syncthreads();  // stage 0 is in LDS
  __syncthreads();  // stage 1 is in LDS
  if (nfull > 0) {
#pragma unroll
    for (int ks = 0; ks < kAhead; ++ks) o[ks].read(lds, off, ks);
  }
  int buf = 0;
  for (int st = 0; st < nfull; ++st) {
    const H *stage = lds + buf * G::kStageHalves;
    const int nbuf = buf == kBufs - 1 ? 0 : buf + 1;
    const bool more = st + 1 < nfull;
#pragma unroll
    for (int ks = 0; ks < kSteps; ++ks) {
      const int kn = ks + kAhead;
      if (kn < kSteps) o[kn % kSteps].read(stage, off, kn);
      else if (more) o[kn % kSteps].read(lds + nbuf * G::kStageHalves, off, kn - kSteps);
      __builtin_amdgcn_sched_barrier(0);
      kstep<H, kSplit, RD>(o[ks], aR, aI);
    }
    buf = nbuf;
    __syncthreads();
  }
  if (tail) {
    __syncthreads();  // the ragged stage is in LDS buffer nfull % 3
#pragma unroll
    for (int ks = 0; ks < kSteps; ++ks) {
      o[0].read(lds + buf * G::kStageHalves, off, ks);
      kstep<H, kSplit, RD>(o[0], aR, aI);
    }
  }
}

template <class H, bool kSplit, bool kClamp>
__device__ __forceinline__ void cov16_unit(const FrameDev &f, const Src &x, int a, int b, int kind,
                                           H *lds) {
  typedef Geo<kSplit> G;
  constexpr int kBK = G::kBK, kRowHalves = G::kRowHalves, kPlaneHalves = G::kPlaneHalves;
  constexpr int kStage = G::kStageHalves, kP = G::kPasses;
  const int wave = threadIdx.x >> 6;
  const int T = x.T;
  const int ra = a * kCovTile, rb = b * kCovTile;
  const int nfull = T / kBK;
  const bool tail = nfull * kBK < T;

  if (wave >= 4) {
    // ---- loader waves: stage s goes to LDS buffer s % 3, two stages ahead
    // of the MFMA waves, with the two stages after it in flight in
    // registers.  Both planes are always loaded (a single diagonal tile has
    // b == a) and prefetch indices past the last full stage re-read it:
    // unconditional loads keep the compiler's waits exact.
    const int lt = threadIdx.x - 4 * 64;
    const unsigned lane_off =
        (unsigned)(((long long)(lt / G::kTPR) * x.ldx + 2 * (lt % G::kTPR)) * 8);
    const __amdgpu_buffer_rsrc_t rsa = plane_rsrc(x.X + (long long)ra * x.ldx);
    const __amdgpu_buffer_rsrc_t rsb = plane_rsrc(x.X + (long long)rb * x.ldx);
    auto load = [&](f32x4 (&v)[2 * kP], int st) {
      plane_load<kSplit, kClamp, false>(v, rsa, x, ra, lane_off, st * kBK, lt);
      plane_load<kSplit, kClamp, false>(v + kP, rsb, x, rb, lane_off, st * kBK, lt);
    };
    auto store = [&](const f32x4 (&v)[2 * kP], int buf) {
      plane_store<H, kSplit>(v, lds, buf * kStage, 2 * kPlaneHalves, lt);
      plane_store<H, kSplit>(v + kP, lds, buf * kStage + kPlaneHalves, 2 * kPlaneHalves, lt);
    };
    // Barrier interval g: the loaders store stage g (loaded two intervals
    // earlier) into buffer g % 3 and load stage g + 2; the MFMA waves
    // consume stage g - 2.  The two register sets alternate, and the
    // prologue only loads, so the loop sees the same order of outstanding
    // loads on every entry.
    f32x4 v0[2 * kP], v1[2 * kP];
    if (nfull > 0) {
      const int last = nfull - 1;
      // (scheduling barriers: the two sets' loads must not interleave)
      load(v0, 0);
      __builtin_amdgcn_sched_barrier(0);
      load(v1, min(1, last));
      __builtin_amdgcn_sched_barrier(0);
      // pairs of intervals; no exit between the halves, so the loop header
      // is reached with the same order of outstanding loads from both sides
      int buf = 0;  // buffer of stage g
      int g = 0;
      for (; g + 1 < nfull; g += 2) {
        store(v0, buf);
        load(v0, min(g + 2, last));
        buf = buf == kBufs - 1 ? 0 : buf + 1;
        __syncthreads();
        store(v1, buf);
        load(v1, min(g + 3, last));
        buf = buf == kBufs - 1 ? 0 : buf + 1;
        __syncthreads();
      }
      if (g < nfull) {  // odd count: the last full stage
        store(v0, buf);
        __syncthreads();
      }
    }
    // the MFMA waves' last two full stages
    __syncthreads();
    __syncthreads();
    if (tail) {
      plane_load<kSplit, kClamp, true>(v0, rsa, x, ra, lane_off, nfull * kBK, lt);
      plane_load<kSplit, kClamp, true>(v0 + kP, rsb, x, rb, lane_off, nfull * kBK, lt);
      store(v0, nfull % kBufs);
      __syncthreads();
    }
    return;
  }

  // ---- MFMA waves: this wave's role, LDS segments and the global origin of
  // each sub-block it accumulates
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
  const int lane_lds = r * kRowHalves + 8 * h;
  auto seg = [&](int plane, int s) { return plane * kPlaneHalves + s * kSub * kRowHalves + lane_lds; };
  int role = kRoleIdle, np = 0;
  int off[4] = {0, 0, 0, 0}, gi[5] = {0, 0, 0, 0, 0}, gj[5] = {0, 0, 0, 0, 0};
  if (kind == kCov16Off) {
    const int wi = wave >> 1, wj = wave & 1;
    role = kRoleOff;
    np = 4;
    off[0] = seg(0, 2 * wi);
    off[1] = seg(0, 2 * wi + 1);
    off[2] = seg(1, 2 * wj);
    off[3] = seg(1, 2 * wj + 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      gi[k] = ra + 64 * wi + kSub * (k >> 1);
      gj[k] = rb + 64 * wj + kSub * (k & 1);
    }
  } else if (wave < 2 || kind == kCov16Diag2) {
    const int plane = wave >> 1;
    const int t0 = plane ? rb : ra;
    static constexpr int kSegs[2][4] = {{3, 0, 1, 2}, {2, 1, 0, 0}};
    static constexpr int kBlk[2][5][2] = {{{3, 3}, {3, 0}, {3, 1}, {3, 2}, {0, 0}},
                                          {{2, 2}, {2, 1}, {2, 0}, {1, 1}, {1, 0}}};
    const int v = wave & 1;
    role = v ? kRoleDY : kRoleDX;
    np = 5;
#pragma unroll
    for (int i = 0; i < 4; ++i) off[i] = seg(plane, kSegs[v][i]);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      gi[k] = t0 + kSub * kBlk[v][k][0];
      gj[k] = t0 + kSub * kBlk[v][k][1];
    }
  }

  floatx16 aR[5], aI[5];
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      aR[k][e] = 0.f;
      aI[k][e] = 0.f;
    }
  switch (role) {
    case kRoleOff: mfma_loop<H, kSplit, RoleOff>(lds, off, nfull, tail, aR, aI); break;
    case kRoleDX: mfma_loop<H, kSplit, RoleDX>(lds, off, nfull, tail, aR, aI); break;
    case kRoleDY: mfma_loop<H, kSplit, RoleDY>(lds, off, nfull, tail, aR, aI); break;
    default:
      // no sub-blocks (the second half of a single diagonal tile): the barriers only
      for (int i = 0; i < 2 + nfull + (tail ? 1 : 0); ++i) __syncthreads();
      return;
  }

  // ---- epilogue: lower-triangle entries and their mirror, scaled by 1/T
  const int M = x.M;
  float2 *R = f.R;
  const long long ldr = f.ldr;
  const float Tf = (float)T;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (k >= np) break;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = gi[k] + (e >> 2) * 8 + h * 4 + (e & 3);
      const int j = gj[k] + r;
      if (i >= M || j >= M || i < j) continue;
      const float re = aR[k][e] / Tf;
      const float im = (i == j) ? 0.f : aI[k][e] / Tf;
      *(FM_GLOBAL f32x2 *)(R + (size_t)i * ldr + j) = f32x2{re, im};
      if (i != j) *(FM_GLOBAL f32x2 *)(R + (size_t)j * ldr + i) = f32x2{re, -im};
    }
  }
}

// unit u of a frame of N row tiles in the canonical single-frame order:
// off-diagonal tiles row by row, then the diagonal pairs, then (odd N) the
// middle diagonal tile
__device__ inline void unit_of(int u, int N, int &a, int &b, int &kind) {
  const int noff = N * (N - 1) / 2;
  if (u < noff) {
    int t = (int)((sqrtf(8.0f * (float)u + 1.0f) - 1.0f) * 0.5f);
    while ((t + 1) * (t + 2) / 2 <= u) ++t;
    while (t * (t + 1) / 2 > u) --t;
    a = t + 1;
    b = u - t * (t + 1) / 2;
    kind = kCov16Off;
  } else {
    const int d = u - noff;
    a = d;
    b = N - 1 - d;
    kind = a == b ? kCov16Diag1 : kCov16Diag2;
  }
}

// one eight-wave workgroup per CU: two waves per SIMD, up to 256 registers
// each (the diagonal roles hold three sub-blocks of accumulators)
template <class H, bool kSplit, bool kBatched>
__global__ __launch_bounds__(kThreads, 1) void cov16_kernel(FrameDev single,
                                                            const FrameDev *__restrict__ frames,
                                                            const Item *__restrict__ items) {
  __shared__ __attribute__((aligned(16))) H lds[Geo<kSplit>::kLdsHalves];
  int a, b, kind;
  const FrameDev *fp;
  if constexpr (kBatched) {
    const Item it = items[blockIdx.x];
    fp = &frames[it.frame];
    a = it.a;
    b = it.b;
    kind = it.c;
  } else {
    fp = &single;
    unit_of(blockIdx.x, (single.M + kCovTile - 1) / kCovTile, a, b, kind);
  }
  const Src x{fp->X, fp->ldx, fp->M, fp->T};
  // only the last row tile of a frame has rows past M
  const int top = (kind == kCov16Off ? a : max(a, b)) + 1;
  if (top * kCovTile > x.M) cov16_unit<H, kSplit, true>(*fp, x, a, b, kind, lds);
  else cov16_unit<H, kSplit, false>(*fp, x, a, b, kind, lds);
}

template <class H, bool kSplit>
void launch16(const FrameDev &single, const FrameDev *frames, const Item *items, int n_items,
              hipStream_t s) {
  const dim3 g(items ? n_items : cov_units(single.M, FM_FP16)), b(kThreads);
  if (items) hipLaunchKernelGGL((cov16_kernel<H, kSplit, true>), g, b, 0, s, single, frames, items);
  else hipLaunchKernelGGL((cov16_kernel<H, kSplit, false>), g, b, 0, s, single, frames, items);
}

}  // namespace

hipError_t launch_covariance16(const FrameDev &single, const FrameDev *frames, const Item *items,
                               int n_items, fm_prec prec, hipStream_t s) {
  if (items && n_items <= 0) return hipSuccess;
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
