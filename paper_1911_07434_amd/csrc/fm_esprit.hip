// fm_esprit.hip -- ESPRIT on the fast signal subspace: the extension of the
// fast subspace to other subspace estimators that the conclusion proposes
// (Sec. VI), least-squares ESPRIT on the two shifted subarrays of the ULA.
//
// With U1 = rows 0..M-2 and U2 = rows 1..M-1 of U_s (M x K),
//   Psi = (U1^H U1)^-1 U1^H U2,   eig(Psi) = exp(-j pi sin(theta_k))
// for the steering a_m = exp(-j pi m sin(theta)), so
//   theta_k = asin(-arg(phi_k) / pi)  (degrees, reported ascending).
// One 64-lane workgroup per frame, all in FP64: the 2K^2 products over the
// M-1 rows (one pair per lane at a time), Gauss-Jordan elimination with
// partial pivoting on [G | H], Householder reduction of Psi to Hessenberg
// form and implicitly shifted QR (complex Wilkinson shift, Givens bulge
// chase, an exceptional shift every 11th step) -- the row and column
// updates spread over the lanes.  K <= 32 (the matrices live in LDS).
#include "fm_internal.h"

namespace fm {
namespace {

constexpr int kEspMaxK = kEspritMaxK;

__device__ inline double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 zmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 zscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double zabs(double2 a) { return hypot(a.x, a.y); }
__device__ inline double2 zdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ inline double2 zsqrt(double2 z) {
  const double r = zabs(z);
  if (r == 0.0) return make_double2(0.0, 0.0);
  const double t = sqrt(0.5 * (r + fabs(z.x)));
  if (z.x >= 0.0) return make_double2(t, z.y / (2.0 * t));
  return make_double2(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

struct EspLds {
  double2 aug[kEspMaxK][2 * kEspMaxK];  // [G | H] -> [I | Psi]
  double2 A[kEspMaxK][kEspMaxK];        // Psi -> Hessenberg -> triangular
  double2 col[2 * kEspMaxK];            // scratch vector (pivot column, Householder v)
  double2 w[kEspMaxK];                  // eigenvalues
  double deg[kEspMaxK];                 // angles (sorted in place)
  double2 gs;                           // Givens sine
  double gc;                            // Givens cosine
  int piv, skip;
};

// eigenvalues of S.A (n x n, Hessenberg after the reduction) into S.w;
// returns the QR step count or -1
__device__ int esprit_eig(EspLds &S, int n) {
  const int lane = threadIdx.x;
  // Householder reduction to upper Hessenberg form
  for (int c = 0; c + 2 < n; ++c) {
    const int len = n - c - 1;
    if (lane == 0) {
      double nx = 0.0;
      for (int i = 0; i < len; ++i) {
        const double2 x = S.A[c + 1 + i][c];
        S.col[i] = x;
        nx += x.x * x.x + x.y * x.y;
      }
      nx = sqrt(nx);
      S.skip = !(nx > 0.0);
      if (nx > 0.0) {
        const double a0 = zabs(S.col[0]);
        const double2 ph = a0 > 0.0 ? zscale(S.col[0], 1.0 / a0) : make_double2(1.0, 0.0);
        S.col[0] = zadd(S.col[0], zscale(ph, nx));
        double nv = 0.0;
        for (int i = 0; i < len; ++i) nv += S.col[i].x * S.col[i].x + S.col[i].y * S.col[i].y;
        nv = sqrt(nv);
        for (int i = 0; i < len; ++i) S.col[i] = zscale(S.col[i], 1.0 / nv);
      }
    }
    __syncthreads();
    if (!S.skip) {
      // A <- (I - 2 v v^H) A on rows c+1..: column j per lane
      for (int j = lane; j < n; j += 64) {
        double2 s = make_double2(0.0, 0.0);
        for (int i = 0; i < len; ++i) s = zadd(s, zmulc(S.col[i], S.A[c + 1 + i][j]));
        for (int i = 0; i < len; ++i)
          S.A[c + 1 + i][j] = zsub(S.A[c + 1 + i][j], zscale(zmul(S.col[i], s), 2.0));
      }
      __syncthreads();
      // A <- A (I - 2 v v^H) on columns c+1..: row i per lane
      for (int i = lane; i < n; i += 64) {
        double2 s = make_double2(0.0, 0.0);
        for (int j = 0; j < len; ++j) s = zadd(s, zmul(S.A[i][c + 1 + j], S.col[j]));
        for (int j = 0; j < len; ++j)
          S.A[i][c + 1 + j] = zsub(S.A[i][c + 1 + j], zscale(zmul(s, zconj(S.col[j])), 2.0));
      }
    }
    __syncthreads();
  }
  // shifted QR with deflation; the control flow is uniform (lane 0 decides
  // through LDS, every lane reads the same values after a barrier)
  const double eps = 2.220446049250313e-16;
  int steps = 0, hi = n - 1;
  while (hi >= 0) {
    if (hi == 0) {
      if (lane == 0) S.w[0] = S.A[0][0];
      break;
    }
    int l = hi;
    while (l > 0) {
      const double sub = zabs(S.A[l][l - 1]);
      double ref = zabs(S.A[l][l]) + zabs(S.A[l - 1][l - 1]);
      if (ref == 0.0) ref = 1.0;
      if (sub <= eps * ref) break;
      --l;
    }
    if (l == hi) {
      if (lane == 0) S.w[hi] = S.A[hi][hi];
      --hi;
      __syncthreads();
      continue;
    }
    if (++steps > 30 * n) return -1;
    const double2 a = S.A[hi - 1][hi - 1], b = S.A[hi - 1][hi];
    const double2 cc = S.A[hi][hi - 1], d = S.A[hi][hi];
    const double2 tr2 = zscale(zadd(a, d), 0.5);
    const double2 det = zsub(zmul(a, d), zmul(b, cc));
    const double2 disc = zsqrt(zsub(zmul(tr2, tr2), det));
    const double2 e1 = zadd(tr2, disc), e2 = zsub(tr2, disc);
    double2 mu = zabs(zsub(e1, d)) <= zabs(zsub(e2, d)) ? e1 : e2;
    if (steps % 11 == 0) mu = zadd(d, make_double2(zabs(cc), 0.0));
    double2 x = zsub(S.A[l][l], mu), y = S.A[l + 1][l];
    for (int k = l; k < hi; ++k) {
      if (k > l) {
        x = S.A[k][k - 1];
        y = S.A[k + 1][k - 1];
      }
      const double ax = zabs(x);
      const double rho = sqrt(ax * ax + y.x * y.x + y.y * y.y);
      if (rho == 0.0) continue;
      double gc;
      double2 gs;
      if (ax == 0.0) {
        gc = 0.0;
        gs = zscale(zconj(y), 1.0 / zabs(y));
      } else {
        gc = ax / rho;
        gs = zscale(zmul(zscale(x, 1.0 / ax), zconj(y)), 1.0 / rho);
      }
      __syncthreads();  // every lane has read x, y
      // rows k, k+1: [c s; -conj(s) c]
      const int j0 = k > l ? k - 1 : l;
      for (int j = j0 + lane; j <= hi; j += 64) {
        const double2 p = S.A[k][j], q = S.A[k + 1][j];
        S.A[k][j] = zadd(zscale(p, gc), zmul(gs, q));
        S.A[k + 1][j] = zsub(zscale(q, gc), zmul(zconj(gs), p));
      }
      __syncthreads();
      // columns k, k+1: times the conjugate transpose
      const int iend = k + 2 < hi ? k + 2 : hi;
      for (int i = l + lane; i <= iend; i += 64) {
        const double2 p = S.A[i][k], q = S.A[i][k + 1];
        S.A[i][k] = zadd(zscale(p, gc), zmul(zconj(gs), q));
        S.A[i][k + 1] = zsub(zscale(q, gc), zmul(gs, p));
      }
      __syncthreads();
    }
  }
  __syncthreads();
  return steps;
}

template <bool kBatched>
__global__ __launch_bounds__(64) void esprit_kernel(FrameDev single, const FrameDev *frames,
                                                    const Item *items) {
  __shared__ EspLds S;
  const FrameDev *fp = kBatched ? frames + items[blockIdx.x].frame : &single;
  const int M = fp->M, K = fp->K;
  const double2 *U = fp->Us;
  double *doa = fp->doa;
  unsigned *status = fp->status;
  const bool or_status = fp->or_status != 0;
  const int lane = threadIdx.x;

  // G = U1^H U1 and H = U1^H U2, one (a, b) pair per lane at a time
  for (int e = lane; e < K * K; e += 64) {
    const int a = e / K, b = e % K;
    const double2 *ua = U + (size_t)a * M, *ub = U + (size_t)b * M;
    double2 g = make_double2(0.0, 0.0), h = make_double2(0.0, 0.0);
    for (int m = 0; m + 1 < M; ++m) {
      const double2 c = ua[m];
      g = zadd(g, zmulc(c, ub[m]));
      h = zadd(h, zmulc(c, ub[m + 1]));
    }
    S.aug[a][b] = g;
    S.aug[a][K + b] = h;
  }
  __syncthreads();
  // Gauss-Jordan with partial pivoting: [G | H] -> [I | G^-1 H]
  for (int c = 0; c < K; ++c) {
    if (lane == 0) {
      int piv = c;
      for (int r = c + 1; r < K; ++r)
        if (zabs(S.aug[r][c]) > zabs(S.aug[piv][c])) piv = r;
      S.piv = piv;
    }
    __syncthreads();
    const int piv = S.piv;
    if (piv != c)
      for (int j = lane; j < 2 * K; j += 64) {
        const double2 t = S.aug[c][j];
        S.aug[c][j] = S.aug[piv][j];
        S.aug[piv][j] = t;
      }
    __syncthreads();
    const double2 p = S.aug[c][c];
    for (int r = lane; r < K; r += 64) S.col[r] = S.aug[r][c];  // multipliers (before the update)
    __syncthreads();
    for (int j = lane; j < 2 * K; j += 64) S.aug[c][j] = zdiv(S.aug[c][j], p);
    __syncthreads();
    for (int e = lane; e < K * 2 * K; e += 64) {
      const int r = e / (2 * K), j = e % (2 * K);
      if (r != c) S.aug[r][j] = zsub(S.aug[r][j], zmul(S.col[r], S.aug[c][j]));
    }
    __syncthreads();
  }
  for (int e = lane; e < K * K; e += 64) S.A[e / K][e % K] = S.aug[e / K][K + e % K];
  __syncthreads();
  const int st = esprit_eig(S, K);
  if (lane == 0) {
    double *t = S.deg;
    for (int k = 0; k < K; ++k) {
      double u = -atan2(S.w[k].y, S.w[k].x) / 3.141592653589793;
      u = fmin(1.0, fmax(-1.0, u));
      t[k] = asin(u) * (180.0 / 3.141592653589793);
    }
    for (int i = 1; i < K; ++i) {  // ascending
      const double v = t[i];
      int j = i - 1;
      while (j >= 0 && t[j] > v) {
        t[j + 1] = t[j];
        --j;
      }
      t[j + 1] = v;
    }
    for (int k = 0; k < K; ++k) doa[k] = t[k];
    const unsigned bits = st < 0 ? FM_ST_EIG_MAXIT : 0u;
    if (or_status) *status |= bits;
    else *status = bits;
  }
}

}  // namespace

hipError_t launch_esprit(const FrameDev &single, const FrameDev *frames, const Item *items,
                         int n_items, hipStream_t s) {
  if (items) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(esprit_kernel<true>, dim3(n_items), dim3(64), 0, s, single, frames, items);
  } else {
    hipLaunchKernelGGL(esprit_kernel<false>, dim3(1), dim3(64), 0, s, single, frames, items);
  }
  return hipGetLastError();
}

}  // namespace fm
