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
// refine kernel here recomputes those angles in FP64 from the FP64 U_s (four
// angles per set, a set's sources shared out over up to four waves); a
// denominator below M*2^-53 is clamped there (noiseless on-grid pole).  Also
// here: the list reset of a plan's frames on the FP16 projection pass (the
// lag-sum kernel resets those of the polynomial pass) and the transposed
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

constexpr int kRefAngles = 4;  // angles per wave
constexpr int kRefK = 4;       // sources per pass over the channels
constexpr int kRefU = 4;       // 64-channel blocks fetched together

// FP64 terms |c_k|^2 of kRefAngles angles (phase frequencies F) by one
// wave, for the source groups g0, g0 + gs, ... (kRefK sources a group).
// Each lane walks every 64th channel with an FP64 phasor recurrence,
// restarted exactly every 4096 channels (at most 64 steps per exact start,
// error ~1e-14), and reads U_s straight from memory, kRefU 64-channel blocks
// at a time: the frame's waves share it through the caches, and no wave
// waits for another.  The angles are taken all at once, so every U_s
// element loaded serves kRefAngles angles.  term[k][j] receives |c_k|^2 of
// angle j (written by lane 0).
__device__ void proj_terms_wave(const FrameDev &f, const unsigned long long (&F)[kRefAngles],
                                int lane, int g0, int gs, double (*term)[kRefAngles]) {
  const int M = f.M, K = f.K;
  double2 w[kRefAngles];
#pragma unroll
  for (int j = 0; j < kRefAngles; ++j) w[j] = phasor64(64, F[j]);
  const int mlast = M - 1;
  for (int k0 = g0 * kRefK; k0 < K; k0 += gs * kRefK) {
    const int kn = min(kRefK, K - k0);
    const FM_GLOBAL double2 *u0 = (const FM_GLOBAL double2 *)(f.Us + (size_t)k0 * M);
    // rows past the last source repeat it; their sums are dropped below
    size_t row[kRefK];
#pragma unroll
    for (int k = 0; k < kRefK; ++k) row[k] = (size_t)min(k, kn - 1) * M;
    double2 acc[kRefAngles][kRefK];
    double2 a[kRefAngles];
#pragma unroll
    for (int j = 0; j < kRefAngles; ++j)
#pragma unroll
      for (int k = 0; k < kRefK; ++k) acc[j][k] = make_double2(0.0, 0.0);
    // kRefU channel blocks of 64 are fetched together (kRefU * kRefK loads in
    // flight), then accumulated in channel order
    for (int mg = 0; mg < M; mg += 64 * kRefU) {
      double2 u[kRefU][kRefK];
#pragma unroll
      for (int b = 0; b < kRefU; ++b) {
        const int mb = min(mg + 64 * b + lane, mlast);
#pragma unroll
        for (int k = 0; k < kRefK; ++k) u[b][k] = u0[row[k] + mb];
      }
#pragma unroll
      for (int b = 0; b < kRefU; ++b) {
        const int mc = mg + 64 * b;
        if (mc >= M) break;
        const int m = mc + lane;
        if (m > mlast) {
#pragma unroll
          for (int k = 0; k < kRefK; ++k) u[b][k] = make_double2(0.0, 0.0);
        }
        if ((mc & 4095) == 0) {
#pragma unroll
          for (int j = 0; j < kRefAngles; ++j) a[j] = phasor64((unsigned long long)m, F[j]);
        }
#pragma unroll
        for (int j = 0; j < kRefAngles; ++j)
#pragma unroll
          for (int k = 0; k < kRefK; ++k) {
            // conj(u) * a
            acc[j][k].x = fma(u[b][k].x, a[j].x, fma(u[b][k].y, a[j].y, acc[j][k].x));
            acc[j][k].y = fma(u[b][k].x, a[j].y, fma(-u[b][k].y, a[j].x, acc[j][k].y));
          }
#pragma unroll
        for (int j = 0; j < kRefAngles; ++j)
          a[j] = make_double2(fma(a[j].x, w[j].x, -(a[j].y * w[j].y)),
                              fma(a[j].x, w[j].y, a[j].y * w[j].x));
      }
    }
#pragma unroll
    for (int j = 0; j < kRefAngles; ++j)
#pragma unroll
      for (int k = 0; k < kRefK; ++k) {
        double re = acc[j][k].x, im = acc[j][k].y;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          re += __shfl_xor(re, o);
          im += __shfl_xor(im, o);
        }
        if (k < kn && lane == 0) term[k0 + k][j] = re * re + im * im;
      }
  }
}

// FP64 recompute of the listed angles: each angle set (kRefAngles
// consecutive list entries) takes min(G, 4) waves of a workgroup, G =
// ceil(K / kRefK) source groups, the waves sharing out the groups; the
// terms |c_k|^2 meet in LDS and one wave adds them in source order (the
// order of the sum over k is that of a single wave's, whatever the split).
// The frame's kRefineGroups workgroups stride over its list.
template <bool kBatched>
__global__ __launch_bounds__(256) void refine_kernel(FrameDev single, const FrameDev *frames,
                                                     const Item *items) {
  int part;
  const FrameDev &f = spec_frame<kBatched>(single, frames, items, part);
  __shared__ double term[4][kMaxK][kRefAngles];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const FM_GLOBAL int *rl = (const FM_GLOBAL int *)f.rlist;
  const int cnt = rl[0];
  const int K = f.K;
  const double floor64 = (double)f.M * 1.1102230246251565e-16;  // M * 2^-53
  const int ngrp = (K + kRefK - 1) / kRefK;
  const int wps = min(ngrp, 4);          // waves per angle set
  const int sets = 4 / wps;              // angle sets per workgroup step
  const int set = wave / wps, g0 = wave % wps;
  const bool active = set < sets;
  const int stride = kRefineGroups * sets * kRefAngles;
  for (int e00 = part * sets * kRefAngles; e00 < cnt; e00 += stride) {
    const int e0 = e00 + set * kRefAngles;
    unsigned long long F[kRefAngles];
    int gl[kRefAngles];
    // entries past the end repeat the last one (computed, never stored)
    int r[kRefAngles];
#pragma unroll
    for (int j = 0; j < kRefAngles; ++j) r[j] = rl[1 + min(e0 + j, cnt - 1)];
#pragma unroll
    for (int j = 0; j < kRefAngles; ++j) {
      gl[j] = e0 + j < cnt ? r[j] : -1;
      F[j] = turn_freq(f.theta0, f.dtheta, r[j]);
    }
    if (active && e0 < cnt) proj_terms_wave(f, F, lane, g0, wps, term[set]);
    __syncthreads();
    if (active && g0 == 0 && e0 < cnt && lane < kRefAngles) {
      double proj = 0.0;
      for (int k = 0; k < K; ++k) proj += term[set][k][lane];
      const double d = (double)f.M - proj;
      int g = gl[0];
#pragma unroll
      for (int j = 1; j < kRefAngles; ++j) g = lane == j ? gl[j] : g;
      if (g >= 0) f.P[g] = (float)(1.0 / fmax(d, floor64));
    }
    __syncthreads();
  }
}

// reset the recompute lists of a plan's frames on the FP16 projection pass
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
