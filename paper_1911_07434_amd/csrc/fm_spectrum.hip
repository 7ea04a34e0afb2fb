// fm_spectrum.hip -- stage 3: MUSIC pseudo-spectrum (eqs. (5) and (10)).
//
//   den(theta) = ||a||^2 - ||U_s^H a(theta)||^2 = M - sum_k |c_k|^2,
//   c_k = sum_m conj(U[k][m]) a_m(theta),  a_m = exp(-j pi m sin(theta)),
//   P = 1 / den.
//
// Bulk pass on FP32 MFMA (v_mfma_f32_16x16x4_f32): angles on the MFMA N
// dimension (16 per wave), the 2K real outputs (Re c_k, Im c_k) on M, the
// channels m on the contraction index.  With U = Ur + j Ui and a = ar + j ai:
//   Re c = Ur.ar + Ui.ai,   Im c = -Ui.ar + Ur.ai
// so each step is two MFMAs: A1 = [Ur; -Ui] against ar, A2 = [Ui; Ur] against ai.
//
// Steering is generated in registers.  The phase of element m in turns,
// frac(-m sin(theta)/2), is an exact 64-bit integer product m * F mod 2^64,
// F = frac(-sin(theta)/2) * 2^64 computed once per angle in FP64; its top 8
// bits index a 256-entry LDS table of unit phasors and the next 24 bits a
// short polynomial, so each exact phasor has ~1e-7 error for every m.  Lanes
// advance by 4 channels with one complex multiply by a(4) and resynchronise
// to the exact phasor every 64 channels.
//
// Every angle whose FP32 denominator is below M/16 (the cancellation-prone
// main lobes) is recomputed in FP64 from the FP64 U_s by the wave that owns
// it; a denominator below M*2^-53 is clamped (noiseless on-grid pole).
#include "fm_internal.h"

namespace fm {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr double kTwo64 = 18446744073709551616.0;

// F = frac(-sin(theta)/2) * 2^64: turns per element as a 64-bit fraction
__device__ inline unsigned long long turn_freq(double theta0, double dtheta, int l) {
  const double th = theta0 + (double)l * dtheta;
  const double s = sin(th * (3.141592653589793 / 180.0));
  double f = -0.5 * s;
  f = f - floor(f);
  double x = f * kTwo64;
  if (!(x < kTwo64)) x = 0.0;
  return (unsigned long long)x;
}

// exp(2 pi j * (m F mod 2^64) / 2^64) in FP32 from the top 32 phase bits
__device__ inline float2 phasor32(unsigned m, unsigned long long F, const float2 *tab) {
  const unsigned lo = (unsigned)F, hi = (unsigned)(F >> 32);
  const unsigned top = m * hi + __umulhi(m, lo);
  const float d = (float)(top & 0xFFFFFFu) * 1.4629180792671596e-09f;  // 2 pi / 2^32
  const float d2 = d * d;
  const float c = fmaf(d2, fmaf(d2, 1.0f / 24.0f, -0.5f), 1.0f);
  const float s = d * fmaf(d2, fmaf(d2, 1.0f / 120.0f, -1.0f / 6.0f), 1.0f);
  const float2 t = tab[top >> 24];
  return make_float2(t.x * c - t.y * s, t.x * s + t.y * c);
}

// the same phasor in FP64
__device__ inline double2 phasor64(unsigned long long m, unsigned long long F) {
  const unsigned long long ph = m * F;
  const double x = (double)(ph >> 11) * 0x1p-52;  // 2 * ph / 2^64, in [0, 2)
  double s, c;
  sincospi(x, &s, &c);
  return make_double2(c, s);
}

__device__ inline float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <bool kBatched>
__device__ __forceinline__ const FrameDev &spec_frame(const FrameDev &single,
                                                      const FrameDev *frames,
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

// FP64 denominator of one angle, computed by the whole wave
__device__ double den_fp64(const FrameDev &f, unsigned long long F, int lane) {
  const int M = f.M, K = f.K;
  double proj = 0.0;
  const double2 w = phasor64(64, F);
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int kn = min(16, K - k0);
    double2 acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = make_double2(0.0, 0.0);
    double2 a = phasor64((unsigned long long)lane, F);
    for (int m = lane; m < M; m += 64) {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < kn) {
          const double2 u = f.Us[(size_t)(k0 + k) * M + m];
          // conj(u) * a
          acc[k].x = fma(u.x, a.x, fma(u.y, a.y, acc[k].x));
          acc[k].y = fma(u.x, a.y, fma(-u.y, a.x, acc[k].y));
        }
      }
      a = make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      double re = acc[k].x, im = acc[k].y;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o);
        im += __shfl_xor(im, o);
      }
      if (k < kn) proj += re * re + im * im;
    }
  }
  return (double)M - proj;
}

template <int NB>
__device__ __forceinline__ void spectrum_tile(const FrameDev &f, int tile, const float2 *tab) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 15, r = lane >> 4;
  const int M = f.M, K = f.K, L = f.L;
  const int gl = tile * kSpecAngles + wave * 16 + n;
  const unsigned long long F = turn_freq(f.theta0, f.dtheta, min(gl, L - 1));
  const float2 w4 = phasor32(4u, F, tab);

  int kk[NB], part[NB];
  bool okr[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int row = 16 * b + n;
    okr[b] = row < 2 * K;
    part[b] = row < K ? 0 : 1;
    kk[b] = okr[b] ? (row < K ? row : row - K) : 0;
  }
  floatx4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};

  float2 ph = make_float2(1.f, 0.f);
  for (int m0 = 0; m0 < M; m0 += 4) {
    const int m = m0 + r;
    ph = ((m0 & 63) == 0) ? phasor32((unsigned)m, F, tab) : cmulf(ph, w4);
    const bool okm = m < M;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float2 u = (okm && okr[b]) ? f.Uf[(size_t)m * K + kk[b]] : make_float2(0.f, 0.f);
      const float a1 = part[b] == 0 ? u.x : -u.y;
      const float a2 = part[b] == 0 ? u.y : u.x;
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, ph.x, acc[b], 0, 0, 0);
      acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, ph.y, acc[b], 0, 0, 0);
    }
  }
  float ss = 0.f;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) ss = fmaf(acc[b][v], acc[b][v], ss);
  ss += __shfl_xor(ss, 16);
  ss += __shfl_xor(ss, 32);
  const float den32 = (float)M - ss;
  const float floor32 = (float)M * 5.9604644775390625e-08f;  // M * 2^-24
  float pval = 1.0f / fmaxf(den32, floor32);

  // FP64 recompute of the cancellation-prone angles
  const bool flag = (r == 0) && (gl < L) && (den32 < (float)M * 0.0625f);
  unsigned long long mask = __ballot(flag);
  while (mask) {
    const int j = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    const int glj = tile * kSpecAngles + wave * 16 + j;
    const unsigned long long Fj = turn_freq(f.theta0, f.dtheta, glj);
    const double d = den_fp64(f, Fj, lane);
    const double floor64 = (double)M * 1.1102230246251565e-16;  // M * 2^-53
    if (lane == j) pval = (float)(1.0 / fmax(d, floor64));
  }
  if (r == 0 && gl < L) f.P[gl] = pval;
}

template <bool kBatched>
__global__ __launch_bounds__(256) void spectrum_kernel(FrameDev single, const FrameDev *frames,
                                                       const Item *items) {
  __shared__ float2 tab[256];
  {
    double s, c;
    sincospi((double)threadIdx.x / 128.0, &s, &c);
    tab[threadIdx.x] = make_float2((float)c, (float)s);
  }
  __syncthreads();
  int tile;
  const FrameDev &f = spec_frame<kBatched>(single, frames, items, tile);
  const int nb = (2 * f.K + 15) / 16;
  switch (nb) {
    case 1: spectrum_tile<1>(f, tile, tab); break;
    case 2: spectrum_tile<2>(f, tile, tab); break;
    case 3: spectrum_tile<3>(f, tile, tab); break;
    case 4: spectrum_tile<4>(f, tile, tab); break;
    case 5: spectrum_tile<5>(f, tile, tab); break;
    case 6: spectrum_tile<6>(f, tile, tab); break;
    case 7: spectrum_tile<7>(f, tile, tab); break;
    default: spectrum_tile<8>(f, tile, tab); break;
  }
}

// FP32 copy of U_s, transposed to [M][K] so that one channel's K entries are
// contiguous for the MFMA operand loads
__global__ __launch_bounds__(256) void uf_kernel(FrameDev f) {
  const int M = f.M, K = f.K;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * K) return;
  const int m = e / K, k = e % K;
  const double2 u = f.Us[(size_t)k * M + m];
  f.Uf[e] = make_float2((float)u.x, (float)u.y);
}

}  // namespace

hipError_t launch_uf(const FrameDev &single, hipStream_t s) {
  const int n = single.M * single.K;
  hipLaunchKernelGGL(uf_kernel, dim3((n + 255) / 256), dim3(256), 0, s, single);
  return hipGetLastError();
}

hipError_t launch_spectrum(const FrameDev &single, const FrameDev *frames, const Item *items,
                           int n_items, fm_prec prec, hipStream_t s) {
  (void)prec;
  if (items) {
    hipLaunchKernelGGL(spectrum_kernel<true>, dim3(n_items), dim3(256), 0, s, single, frames,
                       items);
  } else {
    const int tiles = (single.L + kSpecAngles - 1) / kSpecAngles;
    hipLaunchKernelGGL(spectrum_kernel<false>, dim3(tiles), dim3(256), 0, s, single, frames,
                       items);
  }
  return hipGetLastError();
}

}  // namespace fm
