// fm_peaks.hip -- stage 4: peak picking (eq. (6)).
//
// l is a peak if P[l] > P[l-1] (l > 0) and P[l] >= P[l+1] (l < L-1), so a
// plateau reports its leftmost point; the K largest peaks are reported in
// the total order (value descending, index ascending).
//
// One 1024-thread workgroup per spectrum.  Thread t marks the peaks among
// l = t, t + 1024, ... (coalesced loads); the candidates are compacted into LDS with a block scan;
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

// l is a peak; l may lie past the end (then false).  The three loads are
// unconditional (clamped), so the scan issues them without waiting on a branch.
__device__ inline bool is_peak(const FM_GLOBAL float *P, int L, int l, float &v) {
  const int c = min(l, L - 1);
  v = P[c];
  const float pl = P[max(c - 1, 0)], pr = P[min(c + 1, L - 1)];
  const bool left = (c == 0) || (v > pl);
  const bool right = (c == L - 1) || (v >= pr);
  return l < L && left && right;
}

template <bool kBatched>
__global__ __launch_bounds__(kPeakThreads) void peaks_kernel(FrameDev single,
                                                            const FrameDev *frames,
                                                            const Item *items) {
  const FrameDev &f = kBatched ? frames[items[blockIdx.x].frame] : single;
  const FM_GLOBAL float *P = (const FM_GLOBAL float *)f.P;
  const int L = f.L, K = f.K;
  __shared__ Cand list[kPeakCap];
  __shared__ int wcount[kPeakThreads / 64];
  __shared__ float wv[kPeakThreads / 64];
  __shared__ int wi[kPeakThreads / 64];
  __shared__ int total_s;
  __shared__ float prev_v;
  __shared__ int prev_i;
  __shared__ int found_s;
  // the K <= kMaxK selections, written out once at the end (a global store
  // before each round's barrier would make every round wait for it)
  __shared__ int sel_i[kMaxK];
  __shared__ float sel_v[kMaxK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // thread tid owns l = tid, tid + 1024, ... (coalesced across the wave)
  const int per = (L + kPeakThreads - 1) / kPeakThreads;
  // up to kKeep scan positions per thread (L <= 32768) keep their flags in a
  // bit mask for the compaction below, which then reloads only the peaks;
  // the loads of eight positions are issued before their tests
  constexpr int kKeep = 32;
  unsigned keep = 0;
  int mine = 0;
  for (int j0 = 0; j0 < per; j0 += 8) {
    float v[8];
    bool pk[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) pk[u] = is_peak(P, L, tid + (j0 + u) * kPeakThreads, v[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (j0 + u < per && pk[u]) {
        ++mine;
        if (j0 + u < kKeep) keep |= 1u << (j0 + u);
      }
  }
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
    if (per <= kKeep) {
      for (unsigned m = keep; m; m &= m - 1) {
        const int l = tid + __builtin_ctz(m) * kPeakThreads;
        list[pos++] = Cand{P[l], l};
      }
    } else {
      for (int j = 0; j < per; ++j) {
        const int l = tid + j * kPeakThreads;
        float v;
        if (is_peak(P, L, l, v)) list[pos++] = Cand{v, l};
      }
    }
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
      for (int j = 0; j < per; ++j) {
        const int l = tid + j * kPeakThreads;
        float v;
        if (!is_peak(P, L, l, v)) continue;
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
      sel_i[k] = i;
      sel_v[k] = v;
      prev_v = v;
      prev_i = i;
      found_s = k + 1;
    }
    __syncthreads();
  }
  for (int k = tid; k < found_s; k += kPeakThreads) {
    f.peak_idx[k] = sel_i[k];
    f.peak_val[k] = sel_v[k];
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
