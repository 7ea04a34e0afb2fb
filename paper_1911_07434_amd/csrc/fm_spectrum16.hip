// fm_spectrum16.hip -- stage 3 on 16-bit matrix cores with compensated
// products (eqs. (5) and (10)): the bulk pass of the pseudo-spectrum of the
// mixed-precision path.
//
// Two-level steering.  With m = m0 + j (m0 a multiple of 32, j = 0..31):
//   a_m(theta) = a_m0(theta) a_j(theta),
//   c_k(theta) = sum_m0 a_m0(theta) Z_k(m0, theta),
//   Z_k(m0, theta) = sum_j conj(U[k][m0 + j]) a_j(theta).
// The 32 twiddles a_j of an angle are exact phasors (64-bit integer phase),
// fixed for the whole angle tile and held in registers as MFMA B operands;
// only one base phasor a_m0 per angle per 32 channels is generated
// (recurrence, resynchronised to the exact phasor every 128 channels).
//
// Z is a complex contraction on v_mfma_f32_16x16x32_f16 whose K = 32 real
// values are 16 channels as interleaved (re, im) pairs.  Row 2k of A holds
// (Ur, Ui) and row 2k+1 holds (-Ui, Ur) of source k, against (ar, ai):
//   row 2k  : Ur ar + Ui ai = Re Z_k,   row 2k+1: Ur ai - Ui ar = Im Z_k,
// so one MFMA yields Re and Im of eight sources for 16 angles.  Operands are
// split hi + lo in FP16 (U scaled by a power of two near sqrt(M) so both
// halves stay normal) and hi.hi + hi.lo + lo.hi accumulate in FP32; the
// dropped lo.lo term is ~2^-22 relative.  c_k += a_m0 Z_k runs in FP32 on
// the vector ALU.  Angles whose denominator falls below M/16 go to the same
// FP64 recompute list as in the FP32 pass.
#include "fm_internal.h"
#include "fm_steer.h"

namespace fm {
namespace {

using namespace steer;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

constexpr int kCh = 32;                   // channels per staged chunk
constexpr int kRowH2 = kCh + 4;           // LDS row stride in (re, im) pairs, 16 B padding
// LDS per buffer: hi and lo planes of 16 NB rows ((Ur, Ui) and (-Ui, Ur) per source)
constexpr int plane_h2(int nb) { return 16 * nb * kRowH2; }

// power of two near sqrt(M): U_s entries scaled to magnitude ~1 in FP16
__device__ inline float u_scale(int M) { return exp2f(rintf(0.5f * log2f((float)M))); }

template <bool kBatched>
__device__ __forceinline__ const FrameDev &frame16(const FrameDev &single, const FrameDev *frames,
                                                   const Item *items, int &tile) {
  if constexpr (kBatched) {
    const Item &it = items[blockIdx.x];
    tile = it.a;
    return frames[it.frame];
  } else {
    tile = blockIdx.x;
    return single;
  }
}

__device__ inline h2 swap_neg(h2 x) {
  h2 y;
  y[0] = -x[1];
  y[1] = x[0];
  return y;
}

// NB: row blocks of 16 (= 8 sources), NNB: angle blocks of 16 per wave
template <int NB, int NNB>
__device__ __forceinline__ void spec16_tile(const FrameDev &f, int tile, const float2 *tab,
                                            h2 *lds) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n = lane & 15, g = lane >> 4;
  const int M = f.M, K = f.K, L = f.L;
  constexpr int kPlaneH2 = plane_h2(NB), kBufH2 = 2 * kPlaneH2;
  constexpr int kWaveAngles = 16 * NNB;
  const int first = tile * (4 * kWaveAngles) + wave * kWaveAngles;
  const h2 *Uh = reinterpret_cast<const h2 *>(f.Uf);  // [K][M] scaled hi
  const h2 *Ul = Uh + (size_t)K * M;                   // [K][M] scaled lo

  unsigned long long F[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb)
    F[nb] = turn_freq(f.theta0, f.dtheta, min(first + 16 * nb + n, L - 1));

  // rows 2K .. 16 NB - 1 of the last row block are never staged: zero them
  // in both buffers once
  {
    const int r0 = 2 * K, nz = (16 * NB - r0) * kRowH2;
    h2 z;
    z[0] = (_Float16)0.f;
    z[1] = (_Float16)0.f;
    for (int e = tid; e < nz; e += 256) {
      const int o = r0 * kRowH2 + e;
      lds[o] = z;
      lds[kPlaneH2 + o] = z;
      lds[kBufH2 + o] = z;
      lds[kBufH2 + kPlaneH2 + o] = z;
    }
  }

  // chunk staging: kCh channels x K sources, hi and lo, <= 8 pairs per thread each
  const int celems = K * kCh;
  const int nchunk = (M + kCh - 1) / kCh;
  h2 sh[8], sl[8];
  auto load_chunk = [&](int cc) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      const int k = e / kCh, m = cc * kCh + e % kCh;
      sh[j][0] = (_Float16)0.f;
      sh[j][1] = (_Float16)0.f;
      sl[j] = sh[j];
      if (e < celems && m < M) {
        sh[j] = Uh[(size_t)k * M + m];
        sl[j] = Ul[(size_t)k * M + m];
      }
    }
  };
  auto store_chunk = [&](int buf) {
    h2 *bh = lds + buf * kBufH2;
    h2 *bl = bh + kPlaneH2;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      if (e < celems) {
        const int k = e / kCh, ch = e % kCh;
        const int o = 2 * k * kRowH2 + ch;
        bh[o] = sh[j];
        bh[o + kRowH2] = swap_neg(sh[j]);
        bl[o] = sl[j];
        bl[o + kRowH2] = swap_neg(sl[j]);
      }
    }
  };
  load_chunk(0);
  store_chunk(0);
  __syncthreads();  // publishes the zero rows, the first chunk and the phasor table

  // twiddles a_j for this lane's B operand: j = 16 half + 4 g + 0..3
  h8 twh[2][NNB], twl[2][NNB];
  float2 w32[NNB], base[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) {
    w32[nb] = phasor32(32u, F[nb], tab);
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const float2 p = phasor32((unsigned)(16 * half + 4 * g + jj), F[nb], tab);
        const _Float16 hr = (_Float16)p.x, hi = (_Float16)p.y;
        twh[half][nb][2 * jj] = hr;
        twh[half][nb][2 * jj + 1] = hi;
        twl[half][nb][2 * jj] = (_Float16)(p.x - (float)hr);
        twl[half][nb][2 * jj + 1] = (_Float16)(p.y - (float)hi);
      }
  }

  floatx4 c[NB][NNB];
#pragma unroll
  for (int rb = 0; rb < NB; ++rb)
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb) c[rb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int cc = 0; cc < nchunk; ++cc) {
    const bool more = cc + 1 < nchunk;
    if (more) load_chunk(cc + 1);
    const h2 *bh = lds + (cc & 1) * kBufH2;
    const h2 *bl = bh + kPlaneH2;
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb)
      base[nb] = (cc & 3) == 0 ? phasor32((unsigned)(cc * kCh), F[nb], tab)
                               : cmulf(base[nb], w32[nb]);
#pragma unroll
    for (int rb = 0; rb < NB; ++rb) {
      h8 ah[2], al[2];
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const int o = (16 * rb + n) * kRowH2 + 16 * half + 4 * g;
        ah[half] = *(const h8 *)(bh + o);
        al[half] = *(const h8 *)(bl + o);
      }
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) {
        floatx4 z = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          z = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[half], twh[half][nb], z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[half], twl[half][nb], z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[half], twh[half][nb], z, 0, 0, 0);
        }
        // rows 4g .. 4g+3: (Re, Im) of sources 8 rb + 2g and 8 rb + 2g + 1
        const float2 b = base[nb];
        c[rb][nb][0] = fmaf(b.x, z[0], fmaf(-b.y, z[1], c[rb][nb][0]));
        c[rb][nb][1] = fmaf(b.x, z[1], fmaf(b.y, z[0], c[rb][nb][1]));
        c[rb][nb][2] = fmaf(b.x, z[2], fmaf(-b.y, z[3], c[rb][nb][2]));
        c[rb][nb][3] = fmaf(b.x, z[3], fmaf(b.y, z[2], c[rb][nb][3]));
      }
    }
    if (more) store_chunk((cc + 1) & 1);
    __syncthreads();
  }

  const float s = u_scale(M);
  const float inv2 = 1.0f / (s * s);
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) {
    float ss = 0.f;
#pragma unroll
    for (int rb = 0; rb < NB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) ss = fmaf(c[rb][nb][v], c[rb][nb][v], ss);
    ss += __shfl_xor(ss, 16);
    ss += __shfl_xor(ss, 32);
    const int gl = first + 16 * nb + n;
    if (g == 0 && gl < L) {
      const float den32 = (float)M - ss * inv2;
      const float floor32 = (float)M * 5.9604644775390625e-08f;  // M * 2^-24
      f.P[gl] = 1.0f / fmaxf(den32, floor32);
      if (den32 < (float)M * 0.0625f) {
        const int slot = atomicAdd(f.rlist, 1);
        f.rlist[1 + slot] = gl;
      }
    }
  }
}

template <int NB, int NNB, bool kBatched>
__global__ __launch_bounds__(256) void spectrum16_kernel(FrameDev single, const FrameDev *frames,
                                                         const Item *items) {
  __shared__ float2 tab[256];
  __shared__ __attribute__((aligned(16))) h2 lds[4 * plane_h2(NB)];
  {
    double sn, cs;
    sincospi((double)threadIdx.x / 128.0, &sn, &cs);
    tab[threadIdx.x] = make_float2((float)cs, (float)sn);
  }
  int tile;
  const FrameDev &f = frame16<kBatched>(single, frames, items, tile);
  spec16_tile<NB, NNB>(f, tile, tab, lds);
}

// U_s (complex128 [K][M]) -> scaled FP16 hi and lo planes ([K][M] (re, im)
// pairs each) in the frame's Uf area; element 0 also resets the recompute list
template <bool kBatched>
__global__ __launch_bounds__(256) void split_kernel(FrameDev single, const FrameDev *frames,
                                                   const Item *items) {
  int part;
  const FrameDev &f = frame16<kBatched>(single, frames, items, part);
  const int M = f.M, K = f.K;
  const double s = (double)u_scale(M);
  h2 *Uh = reinterpret_cast<h2 *>(f.Uf);
  h2 *Ul = Uh + (size_t)K * M;
  const int e = part * 256 + threadIdx.x;
  if (e == 0) f.rlist[0] = 0;
  if (e >= K * M) return;
  const double2 u = f.Us[e];
  const float xr = (float)(u.x * s), xi = (float)(u.y * s);
  h2 hi, lo;
  hi[0] = (_Float16)xr;
  hi[1] = (_Float16)xi;
  lo[0] = (_Float16)(xr - (float)hi[0]);
  lo[1] = (_Float16)(xi - (float)hi[1]);
  Uh[e] = hi;
  Ul[e] = lo;
}

template <int NB, int NNB>
hipError_t launch16(const FrameDev &single, const FrameDev *frames, const Item *items,
                    int n_items, hipStream_t s) {
  if (items) {
    hipLaunchKernelGGL((spectrum16_kernel<NB, NNB, true>), dim3(n_items), dim3(256), 0, s,
                       single, frames, items);
  } else {
    const int per = 64 * NNB;
    hipLaunchKernelGGL((spectrum16_kernel<NB, NNB, false>), dim3((single.L + per - 1) / per),
                       dim3(256), 0, s, single, frames, items);
  }
  return hipGetLastError();
}

template <int NB>
hipError_t launch16_nnb(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, int nnb, hipStream_t s) {
  if constexpr (NB <= 4) {
    if (nnb == 4) return launch16<NB, 4>(single, frames, items, n_items, s);
  }
  if (nnb == 2) return launch16<NB, 2>(single, frames, items, n_items, s);
  return launch16<NB, 1>(single, frames, items, n_items, s);
}

}  // namespace

hipError_t launch_split(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, hipStream_t s) {
  if (items) {
    hipLaunchKernelGGL(split_kernel<true>, dim3(n_items), dim3(256), 0, s, single, frames, items);
  } else {
    const int n = single.K * single.M;
    hipLaunchKernelGGL(split_kernel<false>, dim3((n + 255) / 256), dim3(256), 0, s, single,
                       frames, items);
  }
  return hipGetLastError();
}

hipError_t launch_spectrum16(const FrameDev &single, const FrameDev *frames, const Item *items,
                             int n_items, int nb, int nnb, hipStream_t s) {
  switch (nb) {
    case 1: return launch16_nnb<1>(single, frames, items, n_items, nnb, s);
    case 2: return launch16_nnb<2>(single, frames, items, n_items, nnb, s);
    case 3: return launch16_nnb<3>(single, frames, items, n_items, nnb, s);
    case 4: return launch16_nnb<4>(single, frames, items, n_items, nnb, s);
    case 5: return launch16_nnb<5>(single, frames, items, n_items, nnb, s);
    case 6: return launch16_nnb<6>(single, frames, items, n_items, nnb, s);
    case 7: return launch16_nnb<7>(single, frames, items, n_items, nnb, s);
    default: return launch16_nnb<8>(single, frames, items, n_items, nnb, s);
  }
}

}  // namespace fm
