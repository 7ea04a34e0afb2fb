// fm_peaks.hip -- stage 4: peak picking (eq. (6)).
//
// l is a peak if P[l] > P[l-1] (l > 0) and P[l] >= P[l+1] (l < L-1), so a
// plateau reports its leftmost point; the K largest peaks are reported in
// the total order (value descending, index ascending).
//
// One 1024-thread workgroup per spectrum.  Thread t marks the peaks among
// l = t, t + 1024, ... (coalesced loads); the candidates are compacted into
// LDS with a block scan, each wave's candidates contiguous.  A candidate is
// one 64-bit key whose unsigned order is the total order, so a selection is
// a maximum, reduced across a wave with DPP row shifts and broadcasts (VALU
// moves, no LDS traffic).  Each wave selects its own K best in order (K
// rounds over its part of the list, no workgroup barrier), and one wave
// merges the 16 sorted lists (a 16-lane maximum of the list heads per
// selection).  If a spectrum has more local maxima than the LDS list holds,
// K rounds over the whole workgroup rescan the spectrum instead (same
// result, slower).
#include "fm_internal.h"

namespace fm {
namespace {

constexpr int kPeakThreads = 1024;
constexpr int kPeakCap = 8192;
constexpr int kPeakWaves = kPeakThreads / 64;

// Key of candidate (v, i): the float's bits mapped to an unsigned integer of
// the same order (-0 taken as +0), then the index reversed, so that a larger
// key comes first in the total order.  A key is never 0 (i < 2^31 - 1).
__device__ inline unsigned long long peak_key(float v, int i) {
  unsigned b = __float_as_uint(v);
  if ((b << 1) == 0u) b = 0u;
  const unsigned o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((unsigned long long)o << 32) | (unsigned)(0x7fffffff - i);
}
__device__ inline int key_index(unsigned long long k) {
  return 0x7fffffff - (int)(unsigned)(k & 0xffffffffu);
}

// max(x, x of the lane the DPP control names); lanes without a source (or
// outside the row mask) keep x
template <int kCtrl, int kRowMask>
__device__ inline unsigned long long dpp_max(unsigned long long x) {
  const unsigned lo = (unsigned)x, hi = (unsigned)(x >> 32);
  const unsigned ylo = __builtin_amdgcn_update_dpp(lo, lo, kCtrl, kRowMask, 0xf, false);
  const unsigned yhi = __builtin_amdgcn_update_dpp(hi, hi, kCtrl, kRowMask, 0xf, false);
  const unsigned long long y = ((unsigned long long)yhi << 32) | ylo;
  return y > x ? y : x;
}
__device__ inline unsigned long long readlane64(unsigned long long x, int lane) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)x, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(x >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}
// maximum over lanes 0..15 (row shifts: lane 15 of each row ends with the
// row's maximum), returned to every lane
__device__ inline unsigned long long row0_max(unsigned long long x) {
  x = dpp_max<0x111, 0xf>(x);  // row_shr:1
  x = dpp_max<0x112, 0xf>(x);  // row_shr:2
  x = dpp_max<0x114, 0xf>(x);  // row_shr:4
  x = dpp_max<0x118, 0xf>(x);  // row_shr:8
  return readlane64(x, 15);
}
// maximum over the wave: rows, then row_bcast:15 into rows 1 and 3 and
// row_bcast:31 into rows 2 and 3 leave it in lane 63
__device__ inline unsigned long long wave_max(unsigned long long x) {
  x = dpp_max<0x111, 0xf>(x);
  x = dpp_max<0x112, 0xf>(x);
  x = dpp_max<0x114, 0xf>(x);
  x = dpp_max<0x118, 0xf>(x);
  x = dpp_max<0x142, 0xa>(x);
  x = dpp_max<0x143, 0xc>(x);
  return readlane64(x, 63);
}
// inclusive prefix sum over the wave, the same shifts with zeros shifted in
__device__ inline int wave_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);
  return x;
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
  __shared__ unsigned long long list[kPeakCap];
  __shared__ int wcount[kPeakWaves];
  __shared__ int wtot[kPeakWaves];
  __shared__ unsigned long long wtop[kPeakWaves][kMaxK];
  __shared__ unsigned long long wbest[kPeakWaves];
  __shared__ int total_s;
  __shared__ int found_s;
  // the K <= kMaxK selections, written out once at the end
  __shared__ unsigned long long sel[kMaxK];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // thread tid owns l = tid, tid + 1024, ... (coalesced across the wave)
  const int per = (L + kPeakThreads - 1) / kPeakThreads;
  // Up to kReg positions per thread (L <= 24576): all loads issued at once,
  // the values kept in registers for the compaction, and the neighbours
  // taken from the adjacent lanes (lane 0 and lane 63 load the one outside
  // the wave).  Longer spectra: up to kKeep positions keep their flags in a
  // bit mask and the compaction reloads only the peaks; the loads of eight
  // positions are issued before their tests.
  constexpr int kReg = 24;
  constexpr int kKeep = 32;
  const bool in_reg = per <= kReg;
  float vr[kReg];
  unsigned keep = 0;
  int mine = 0;
  if (in_reg) {
    float ed[kReg];
#pragma unroll
    for (int u = 0; u < kReg; ++u) {
      const int c = min(tid + u * kPeakThreads, L - 1);
      vr[u] = P[c];
      ed[u] = P[lane == 0 ? max(c - 1, 0) : min(c + 1, L - 1)];
    }
#pragma unroll
    for (int u = 0; u < kReg; ++u) {
      const int l = tid + u * kPeakThreads;
      const int c = min(l, L - 1);
      const float up = __shfl_up(vr[u], 1), dn = __shfl_down(vr[u], 1);
      const float pl = lane == 0 ? ed[u] : up;
      const float pr = lane == 63 ? ed[u] : dn;
      const bool left = (c == 0) || (vr[u] > pl);
      const bool right = (c == L - 1) || (vr[u] >= pr);
      if (l < L && left && right) {
        ++mine;
        keep |= 1u << u;
      }
    }
  } else {
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
  }
  // exclusive scan of the per-thread counts: wave scan, then wave offsets
  const int incl = wave_scan(mine);
  if (lane == 63) wcount[wave] = incl;
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int w = 0; w < kPeakWaves; ++w) {
      const int c = wcount[w];
      wtot[w] = c;
      wcount[w] = s;
      s += c;
    }
    total_s = s;
    found_s = 0;
  }
  __syncthreads();
  const int total = total_s;
  const bool in_lds = total <= kPeakCap;
  if (in_lds) {
    int pos = wcount[wave] + incl - mine;
    if (in_reg) {
#pragma unroll
      for (int u = 0; u < kReg; ++u)
        if ((keep >> u) & 1u) list[pos++] = peak_key(vr[u], tid + u * kPeakThreads);
    } else if (per <= kKeep) {
      for (unsigned m = keep; m; m &= m - 1) {
        const int l = tid + __builtin_ctz(m) * kPeakThreads;
        list[pos++] = peak_key(P[l], l);
      }
    } else {
      for (int j = 0; j < per; ++j) {
        const int l = tid + j * kPeakThreads;
        float v;
        if (is_peak(P, L, l, v)) list[pos++] = peak_key(v, l);
      }
    }
  }
  __syncthreads();

  const int rounds = min(K, total);
  if (in_lds) {
    // each wave: its own candidates' K best, in order (wave-uniform loop);
    // round k takes the largest key below the previous winner
    const int ws = wcount[wave], wn = wtot[wave];
    const int rw = min(K, wn);
    unsigned long long prev = ~0ull;
    for (int k = 0; k < rw; ++k) {
      unsigned long long best = 0;
      for (int e = lane; e < wn; e += 64) {
        const unsigned long long c = list[ws + e];
        if (c < prev && c > best) best = c;
      }
      best = wave_max(best);
      if (lane == 0) wtop[wave][k] = best;
      prev = best;
    }
    __syncthreads();
    // wave 0 merges the sorted lists: lane j < 16 holds the head of list j
    if (wave == 0) {
      const int len = lane < kPeakWaves ? min(K, wtot[lane]) : 0;
      int h = 0;
      unsigned long long head = len > 0 ? wtop[lane][0] : 0ull;
      for (int k = 0; k < rounds; ++k) {
        const unsigned long long best = row0_max(head);
        if (lane == 0) sel[k] = best;
        // keys are distinct: exactly one head is the winner
        if (head == best) {
          ++h;
          head = h < len ? wtop[lane][h] : 0ull;
        }
      }
      if (lane == 0) found_s = rounds;
    }
    __syncthreads();
  } else {
    unsigned long long prev = ~0ull;
    for (int k = 0; k < rounds; ++k) {
      unsigned long long best = 0;
      for (int j = 0; j < per; ++j) {
        const int l = tid + j * kPeakThreads;
        float v;
        if (!is_peak(P, L, l, v)) continue;
        const unsigned long long c = peak_key(v, l);
        if (c < prev && c > best) best = c;
      }
      best = wave_max(best);
      if (lane == 0) wbest[wave] = best;
      __syncthreads();
      unsigned long long b = 0;
      for (int w = 0; w < kPeakWaves; ++w) b = wbest[w] > b ? wbest[w] : b;
      if (tid == 0) {
        sel[k] = b;
        found_s = k + 1;
      }
      prev = b;
      __syncthreads();
    }
  }
  for (int k = tid; k < found_s; k += kPeakThreads) {
    const int i = key_index(sel[k]);
    f.peak_idx[k] = i;
    f.peak_val[k] = P[i];
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
