// fm_peaks.hip -- stage 4: peak picking (eq. (6)).
//
// l is a peak if P[l] > P[l-1] (l > 0) and P[l] >= P[l+1] (l < L-1), so a
// plateau reports its leftmost point; the K largest peaks are reported in
// the total order (value descending, index ascending).
//
// One 1024-thread workgroup per spectrum.  Each thread marks the peaks of a
// contiguous chunk; the candidates are compacted into LDS with a block scan;
// then K rounds each select the first candidate after the previous winner in
// the total order with a wavefront shuffle reduction and a 16-entry LDS
// reduction.  If a spectrum has more local maxima than the LDS list holds,
// the rounds rescan the spectrum instead (same result, slower).
#include "fm_internal.h"

namespace fm {
namespace {

constexpr int kPeakThreads = 1024;
constexpr int kPeakCap = 8192;

struct Cand {
  float v;
  int i;
};

// a comes before b in the total order
__device__ inline bool before(float av, int ai, float bv, int bi) {
  return av > bv || (av == bv && ai < bi);
}

__device__ inline bool is_peak(const float *P, int L, int l) {
  const float v = P[l];
  const bool left = (l == 0) || (v > P[l - 1]);
  const bool right = (l == L - 1) || (v >= P[l + 1]);
  return left && right;
}

template <bool kBatched>
__global__ __launch_bounds__(kPeakThreads) void peaks_kernel(FrameDev single,
                                                            const FrameDev *frames,
                                                            const Item *items) {
  const FrameDev &f = kBatched ? frames[items[blockIdx.x].frame] : single;
  const float *P = f.P;
  const int L = f.L, K = f.K;
  __shared__ Cand list[kPeakCap];
  __shared__ int wcount[kPeakThreads / 64];
  __shared__ float wv[kPeakThreads / 64];
  __shared__ int wi[kPeakThreads / 64];
  __shared__ int total_s;
  __shared__ float prev_v;
  __shared__ int prev_i;
  __shared__ int found_s;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int chunk = (L + kPeakThreads - 1) / kPeakThreads;
  const int lo = min(L, tid * chunk), hi = min(L, lo + chunk);
  int mine = 0;
  for (int l = lo; l < hi; ++l) mine += is_peak(P, L, l);
  // exclusive scan of the per-thread counts: wave scan, then wave offsets
  int incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wcount[wave] = incl;
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int w = 0; w < kPeakThreads / 64; ++w) {
      const int c = wcount[w];
      wcount[w] = s;
      s += c;
    }
    total_s = s;
    prev_v = __int_as_float(0x7f800000);  // +inf: nothing selected yet
    prev_i = -1;
    found_s = 0;
  }
  __syncthreads();
  const int total = total_s;
  const bool in_lds = total <= kPeakCap;
  if (in_lds) {
    int pos = wcount[wave] + incl - mine;
    for (int l = lo; l < hi; ++l)
      if (is_peak(P, L, l)) list[pos++] = Cand{P[l], l};
  }
  __syncthreads();

  const int rounds = min(K, total);
  for (int k = 0; k < rounds; ++k) {
    const float pv = prev_v;
    const int pi = prev_i;
    float bv = 0.f;
    int bi = -1;
    if (in_lds) {
      for (int e = tid; e < total; e += kPeakThreads) {
        const Cand c = list[e];
        if (before(pv, pi, c.v, c.i) && (bi < 0 || before(c.v, c.i, bv, bi))) {
          bv = c.v;
          bi = c.i;
        }
      }
    } else {
      for (int l = lo; l < hi; ++l) {
        if (!is_peak(P, L, l)) continue;
        const float v = P[l];
        if (before(pv, pi, v, l) && (bi < 0 || before(v, l, bv, bi))) {
          bv = v;
          bi = l;
        }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float ov = __shfl_xor(bv, o);
      const int oi = __shfl_xor(bi, o);
      if (oi >= 0 && (bi < 0 || before(ov, oi, bv, bi))) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      wv[wave] = bv;
      wi[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      float v = 0.f;
      int i = -1;
      for (int w = 0; w < kPeakThreads / 64; ++w)
        if (wi[w] >= 0 && (i < 0 || before(wv[w], wi[w], v, i))) {
          v = wv[w];
          i = wi[w];
        }
      f.peak_idx[k] = i;
      f.peak_val[k] = v;
      prev_v = v;
      prev_i = i;
      found_s = k + 1;
    }
    __syncthreads();
  }
  if (tid == 0) {
    *f.n_found = found_s;
    if (kBatched && found_s < K && f.status) atomicOr(f.status, (unsigned)FM_ST_FEW_PEAKS);
  }
}

}  // namespace

hipError_t launch_peaks(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, hipStream_t s) {
  if (items)
    hipLaunchKernelGGL(peaks_kernel<true>, dim3(n_items), dim3(kPeakThreads), 0, s, single,
                       frames, items);
  else
    hipLaunchKernelGGL(peaks_kernel<false>, dim3(1), dim3(kPeakThreads), 0, s, single, frames,
                       items);
  return hipGetLastError();
}

}  // namespace fm
