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
// main lobes) is appended to a per-frame list, and a second kernel
// recomputes those angles in FP64 from the FP64 U_s (one wave per angle);
// a denominator below M*2^-53 is clamped there (noiseless on-grid pole).
#include "fm_internal.h"
#include "fm_steer.h"

namespace fm {
namespace {

using namespace steer;

typedef float floatx4 __attribute__((ext_vector_type(4)));

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

// FP64 denominators of the four angles Fw (one per wave; a wave with no
// angle passes active = false but still stages and synchronises).  Each lane
// walks every 64th channel with an FP64 phasor recurrence (64 steps at most
// per exact start, error ~1e-14), K accumulated 16 at a time.  U_s is staged
// through LDS 16 sources x 64 channels at a time and shared by the four
// waves, so the workgroup reads it once per four angles.
__device__ double den_fp64_x4(const FrameDev &f, unsigned long long F, bool active, int lane,
                              double2 (*us)[64]) {
  const int M = f.M, K = f.K;
  double proj = 0.0;
  const double2 w = phasor64(64, F);
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int kn = min(16, K - k0);
    double2 acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = make_double2(0.0, 0.0);
    double2 a = phasor64((unsigned long long)lane, F);
    for (int mc = 0; mc < M; mc += 64) {
      __syncthreads();  // the previous chunk has been read by every wave
      for (int e = threadIdx.x; e < 16 * 64; e += blockDim.x) {
        const int k = e >> 6, m = mc + (e & 63);
        us[k][e & 63] = (k < kn && m < M) ? f.Us[(size_t)(k0 + k) * M + m]
                                          : make_double2(0.0, 0.0);
      }
      __syncthreads();
      if (active && mc + lane < M) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          if (k < kn) {
            const double2 u = us[k][lane];
            // conj(u) * a
            acc[k].x = fma(u.x, a.x, fma(u.y, a.y, acc[k].x));
            acc[k].y = fma(u.x, a.y, fma(-u.y, a.x, acc[k].y));
          }
        }
      }
      a = make_double2(fma(a.x, w.x, -(a.y * w.y)), fma(a.x, w.y, a.y * w.x));
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

// FP32 pass over one tile of 64 NNB angles (four waves of 16 NNB).  U_s is
// staged through LDS in chunks of kSpecChunk channels, double buffered: the
// next chunk's global loads are in flight while the matrix cores work on
// the current one.  NB = row blocks of 16 over the 2K stacked outputs; each
// U_s operand read from LDS feeds the NNB angle blocks of the wave.  An
// angle's arithmetic does not depend on NNB.
template <int NB, int NNB>
__device__ __forceinline__ void spectrum_tile(const FrameDev &f, int tile, const float2 *tab,
                                              float2 (*ubuf)[kSpecChunk * 8 * NB]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n = lane & 15, r = lane >> 4;
  const int M = f.M, K = f.K, L = f.L;
  const int first = tile * (64 * NNB) + wave * (16 * NNB);
  unsigned long long F[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb)
    F[nb] = turn_freq(f.theta0, f.dtheta, min(first + 16 * nb + n, L - 1));

  int kk[NB], part[NB];
  bool okr[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int row = 16 * b + n;
    okr[b] = row < 2 * K;
    part[b] = row < K ? 0 : 1;
    kk[b] = okr[b] ? (row < K ? row : row - K) : 0;
  }
  floatx4 acc[NB][NNB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb) acc[b][nb] = floatx4{0.f, 0.f, 0.f, 0.f};

  // cooperative chunk loads: kSpecChunk * K float2, at most 2 * NB per thread
  const int chunk_elems = kSpecChunk * K;
  const int nchunk = (M + kSpecChunk - 1) / kSpecChunk;
  const size_t total = (size_t)M * K;
  float2 stage[2 * NB];
  auto load_chunk = [&](int c) {
    const size_t base = (size_t)c * chunk_elems;
#pragma unroll
    for (int j = 0; j < 2 * NB; ++j) {
      const int e = tid + 256 * j;
      stage[j] = (e < chunk_elems && base + e < total) ? f.Uf[base + e] : make_float2(0.f, 0.f);
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 2 * NB; ++j) {
      const int e = tid + 256 * j;
      if (e < chunk_elems) ubuf[buf][e] = stage[j];
    }
  };
  load_chunk(0);
  store_chunk(0);
  __syncthreads();  // publishes the first chunk and the phasor table
  float2 w4[NNB], ph[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) w4[nb] = phasor32(4u, F[nb], tab);

  for (int c = 0; c < nchunk; ++c) {
    const bool more = c + 1 < nchunk;
    if (more) load_chunk(c + 1);
    const float2 *ub = ubuf[c & 1];
#pragma unroll 4
    for (int s = 0; s < kSpecChunk / 4; ++s) {
      const int m = c * kSpecChunk + 4 * s + r;
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb)
        ph[nb] = (s == 0) ? phasor32((unsigned)m, F[nb], tab) : cmulf(ph[nb], w4[nb]);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float2 u = okr[b] ? ub[(4 * s + r) * K + kk[b]] : make_float2(0.f, 0.f);
        const float a1 = part[b] == 0 ? u.x : -u.y;
        const float a2 = part[b] == 0 ? u.y : u.x;
#pragma unroll
        for (int nb = 0; nb < NNB; ++nb) {
          acc[b][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, ph[nb].x, acc[b][nb], 0, 0, 0);
          acc[b][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, ph[nb].y, acc[b][nb], 0, 0, 0);
        }
      }
    }
    if (more) store_chunk((c + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) {
    float ss = 0.f;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) ss = fmaf(acc[b][nb][v], acc[b][nb][v], ss);
    ss += __shfl_xor(ss, 16);
    ss += __shfl_xor(ss, 32);
    const int gl = first + 16 * nb + n;
    if (r == 0 && gl < L) {
      const float den32 = (float)M - ss;
      const float floor32 = (float)M * 5.9604644775390625e-08f;  // M * 2^-24
      f.P[gl] = 1.0f / fmaxf(den32, floor32);
      // main lobes, where M - ||U^H a||^2 cancels, are recomputed in FP64
      if (den32 < (float)M * 0.0625f) {
        const int slot = atomicAdd(f.rlist, 1);
        f.rlist[1 + slot] = gl;
      }
    }
  }
}

template <int NB, int NNB, bool kBatched>
__global__ __launch_bounds__(256) void spectrum_kernel(FrameDev single, const FrameDev *frames,
                                                       const Item *items) {
  __shared__ float2 tab[256];
  __shared__ float2 ubuf[2][kSpecChunk * 8 * NB];
  {
    double s, c;
    sincospi((double)threadIdx.x / 128.0, &s, &c);
    tab[threadIdx.x] = make_float2((float)c, (float)s);
  }
  // (the first __syncthreads in spectrum_tile also publishes the table)
  int tile;
  const FrameDev &f = spec_frame<kBatched>(single, frames, items, tile);
  spectrum_tile<NB, NNB>(f, tile, tab, ubuf);
}

// FP64 recompute of the listed angles: one wave per angle, the frame's
// kRefineGroups workgroups striding over its list
template <bool kBatched>
__global__ __launch_bounds__(256) void refine_kernel(FrameDev single, const FrameDev *frames,
                                                     const Item *items) {
  __shared__ double2 us[16][64];
  int part;
  const FrameDev &f = spec_frame<kBatched>(single, frames, items, part);
  const int lane = threadIdx.x & 63;
  const int gw = part * 4 + (threadIdx.x >> 6);
  const int cnt = f.rlist[0];
  const double floor64 = (double)f.M * 1.1102230246251565e-16;  // M * 2^-53
  // the four waves take four consecutive list entries per step (uniform loop)
  for (int e0 = part * 4; e0 < cnt; e0 += kRefineGroups * 4) {
    const int e = e0 + (gw - part * 4);
    const bool active = e < cnt;
    const int gl = active ? f.rlist[1 + e] : 0;
    const unsigned long long F = turn_freq(f.theta0, f.dtheta, gl);
    const double d = den_fp64_x4(f, F, active, lane, us);
    if (active && lane == 0) f.P[gl] = (float)(1.0 / fmax(d, floor64));
  }
}

// reset the recompute lists of the frames of a plan
__global__ void spec_prep_kernel(const FrameDev *frames, const Item *items, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) frames[items[i].frame].rlist[0] = 0;
}

// FP32 copy of U_s, transposed to [M][K] so that one channel's K entries are
// contiguous for the MFMA operand loads; also resets the recompute list
__global__ __launch_bounds__(256) void uf_kernel(FrameDev f) {
  const int M = f.M, K = f.K;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) f.rlist[0] = 0;
  if (e >= M * K) return;
  const int m = e / K, k = e % K;
  const double2 u = f.Us[(size_t)k * M + m];
  f.Uf[e] = make_float2((float)u.x, (float)u.y);
}

template <int NB, int NNB>
hipError_t launch_nb(const FrameDev &single, const FrameDev *frames, const Item *items,
                     int n_items, hipStream_t s) {
  if (items) {
    hipLaunchKernelGGL((spectrum_kernel<NB, NNB, true>), dim3(n_items), dim3(256), 0, s, single,
                       frames, items);
  } else {
    const int tiles = (single.L + 64 * NNB - 1) / (64 * NNB);
    hipLaunchKernelGGL((spectrum_kernel<NB, NNB, false>), dim3(tiles), dim3(256), 0, s, single,
                       frames, items);
  }
  return hipGetLastError();
}

template <int NB>
hipError_t launch_nnb(const FrameDev &single, const FrameDev *frames, const Item *items,
                      int n_items, int nnb, hipStream_t s) {
  if constexpr (NB <= 4) {
    if (nnb == 4) return launch_nb<NB, 4>(single, frames, items, n_items, s);
  }
  if (nnb == 2) return launch_nb<NB, 2>(single, frames, items, n_items, s);
  return launch_nb<NB, 1>(single, frames, items, n_items, s);
}

}  // namespace

hipError_t launch_uf(const FrameDev &single, hipStream_t s) {
  const int n = single.M * single.K;
  hipLaunchKernelGGL(uf_kernel, dim3((n + 255) / 256), dim3(256), 0, s, single);
  return hipGetLastError();
}

hipError_t launch_spec_prep(const FrameDev *frames, const Item *items, int n_items,
                            hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(spec_prep_kernel, dim3((n_items + 255) / 256), dim3(256), 0, s, frames,
                     items, n_items);
  return hipGetLastError();
}

hipError_t launch_spectrum(const FrameDev &single, const FrameDev *frames, const Item *items,
                           int n_items, int nb, int nnb, hipStream_t s) {
  switch (nb) {
    case 1: return launch_nnb<1>(single, frames, items, n_items, nnb, s);
    case 2: return launch_nnb<2>(single, frames, items, n_items, nnb, s);
    case 3: return launch_nnb<3>(single, frames, items, n_items, nnb, s);
    case 4: return launch_nnb<4>(single, frames, items, n_items, nnb, s);
    case 5: return launch_nnb<5>(single, frames, items, n_items, nnb, s);
    case 6: return launch_nnb<6>(single, frames, items, n_items, nnb, s);
    case 7: return launch_nnb<7>(single, frames, items, n_items, nnb, s);
    default: return launch_nnb<8>(single, frames, items, n_items, nnb, s);
  }
}

hipError_t launch_refine(const FrameDev &single, const FrameDev *frames, const Item *items,
                         int n_items, hipStream_t s) {
  if (items)
    hipLaunchKernelGGL(refine_kernel<true>, dim3(n_items), dim3(256), 0, s, single, frames, items);
  else
    hipLaunchKernelGGL(refine_kernel<false>, dim3(kRefineGroups), dim3(256), 0, s, single, frames,
                       items);
  return hipGetLastError();
}

}  // namespace fm
