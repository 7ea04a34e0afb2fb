// fm_gram.h -- Gram partials of one row chunk, shared by the sketch kernels
// that form them in their epilogue (device code only).
#pragma once

#include "fm_internal.h"

namespace fm {

// out[a][b] = sum over rows m of conj(A[m][a]) B[m][b] in FP64 (the products
// of FP32 inputs are exact), rows in order: the Gram partial of one chunk,
// one entry per thread at a time.  Same per-entry order as gram_block.
// A and B are typed pointers (FM_LDS or FM_GLOBAL) so every read is an LDS
// or a global load, never a flat one.
template <class PA, class PB>
__device__ __forceinline__ void gram_rows(PA A, PB B, double2 *outp, int n, int rows) {
  FM_GLOBAL double2 *out = (FM_GLOBAL double2 *)outp;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int a = e / n, b = e % n;
    double2 acc = make_double2(0.0, 0.0);
    for (int m = 0; m < rows; ++m) {
      const float2 av = A[(size_t)m * n + a], bv = B[(size_t)m * n + b];
      const double ar = av.x, ai = av.y, br = bv.x, bi = bv.y;
      acc.x = fma(ar, br, acc.x);
      acc.x = fma(ai, bi, acc.x);
      acc.y = fma(ar, bi, acc.y);
      acc.y = fma(-ai, br, acc.y);
    }
    out[e] = acc;
  }
}

}  // namespace fm
