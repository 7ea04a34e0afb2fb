// fm_order.hip -- number of sources from the sketch eigenvalues: the
// pre-estimation of K that Sec. V-D proposes (Akaike's information criterion
// or the minimum description length), for frames whose K is not known.
//
// Criteria for N snapshots of an M-channel array, with noise eigenvalues
// lambda_{k+1..M}:
//   L(k)   = N ((M - k) log(mean of noise) - sum of log(noise))
//   AIC(k) = 2 L(k) + 2 k (2M - k),  MDL(k) = L(k) + k (2M - k) log(N) / 2
// and K_hat the first minimiser.  Only the n eigenvalues of the Nystrom
// approximation S~ are known: those above rcond * eig[0] are used as they
// are (r of them) and the other M - r eigenvalues of R are replaced by their
// mean mu = (tr R - sum of kept) / (M - r), fixed by the exact trace of R;
// k runs over 0..r (0..r-1 when r == M).  mu <= 0 (the kept eigenvalues hold
// the whole trace) gives K_hat = r.  Everything after the trace is FP64 on
// one lane; n <= 64 keeps that O(n^2) loop trivial.
#include "fm_internal.h"

namespace fm {
namespace {

constexpr int kOrderThreads = 256;

template <bool kBatched>
__global__ __launch_bounds__(kOrderThreads) void order_kernel(FrameDev single,
                                                              const FrameDev *frames,
                                                              const Item *items) {
  const FrameDev &fr = kBatched ? frames[items[blockIdx.x].frame] : single;
  const float2 *R = fr.R;
  const long long ldr = fr.ldr;
  const int M = fr.M, n = fr.n, N = fr.T, rule = fr.order_rule;
  const double rcond = fr.rcond;
  const double *eig = fr.eig;
  double *crit = fr.order_crit;
  int *K_hat = fr.K_hat;
  unsigned *status = fr.status;
  const bool or_status = fr.or_status != 0;

  // trace of R: per-thread strided sums, then a fixed-shape tree (the
  // result does not depend on timing)
  __shared__ double part[kOrderThreads];
  double acc = 0.0;
  for (int m = threadIdx.x; m < M; m += kOrderThreads) acc += (double)R[(size_t)m * ldr + m].x;
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kOrderThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double trR = part[0];

  if (crit)
    for (int k = 0; k <= n; ++k) crit[k] = __builtin_inf();
  int r = 0;
  while (r < n && eig[r] > 0.0 && eig[r] > rcond * eig[0]) ++r;
  double kept = 0.0;
  for (int i = 0; i < r; ++i) kept += eig[i];
  const int nc = M - r;
  double mu = 0.0;
  int best = 0;
  bool done = false;
  if (nc > 0) {
    mu = (trR - kept) / nc;
    if (!(mu > 0.0)) {
      best = r;
      done = true;
    }
  }
  if (!done) {
    const int kmax = nc > 0 ? r : r - 1;
    const double logN = log((double)N);
    double cbest = 0.0;
    for (int k = 0; k <= kmax; ++k) {
      double sum = 0.0, lsum = 0.0;
      for (int i = k; i < r; ++i) {
        sum += eig[i];
        lsum += log(eig[i]);
      }
      if (nc > 0) {
        sum += nc * mu;
        lsum += nc * log(mu);
      }
      const int m = M - k;
      const double Lk = (double)N * (m * log(sum / m) - lsum);
      const double pen = (double)k * (2.0 * M - k);
      const double c = rule == FM_ORDER_AIC ? 2.0 * Lk + 2.0 * pen : Lk + 0.5 * pen * logN;
      if (crit) crit[k] = c;
      if (k == 0 || c < cbest) {
        cbest = c;
        best = k;
      }
    }
  }
  *K_hat = best;
  const unsigned bits = best >= n ? FM_ST_ORDER_AT_LIMIT : 0u;
  if (or_status) *status |= bits;
  else *status = bits;
}

}  // namespace

hipError_t launch_order(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, hipStream_t s) {
  if (items) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(order_kernel<true>, dim3(n_items), dim3(kOrderThreads), 0, s, single,
                       frames, items);
  } else {
    hipLaunchKernelGGL(order_kernel<false>, dim3(1), dim3(kOrderThreads), 0, s, single, frames,
                       items);
  }
  return hipGetLastError();
}

}  // namespace fm
