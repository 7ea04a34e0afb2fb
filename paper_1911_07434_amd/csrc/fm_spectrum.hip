// fm_spectrum.hip -- stage 3: MUSIC pseudo-spectrum (eqs. (5) and (10)),
// the parts shared by the bulk passes.
//
//   den(theta) = ||a||^2 - ||U_s^H a(theta)||^2 = M - sum_k |c_k|^2,
//   c_k = sum_m conj(U[k][m]) a_m(theta),  a_m = exp(-j pi m sin(theta)),
//   P = 1 / den.
//
// The bulk of the grid is evaluated in FP32 (fm_poly.hip: the spectrum as a
// polynomial in sin(theta)) or with compensated FP16 products
// (fm_spectrum16.hip).  Both append every angle whose denominator is below
// M/16 (the cancellation-prone main lobes) to a per-frame list, and the
// refine kernel here recomputes those angles in FP64 from the FP64 U_s (one
// wave per angle); a denominator below M*2^-53 is clamped there (noiseless
// on-grid pole).  Also here: the list reset of a plan and the transposed
// FP32 copy of U_s of a single-frame call.
#include "fm_internal.h"
#include "fm_steer.h"

namespace fm {
namespace {

using namespace steer;

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
