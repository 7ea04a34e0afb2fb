/*
 * fm_oracle.c -- plain, slow FP64 CPU reference of the fast-MUSIC hot path
 * (Li, Wang, Zhang, Cao, Zhao, "Ultra-Fast Accurate AoA Estimation via
 * Automotive Massive-MIMO Radar", arXiv:1911.07434).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or helper with the HIP library;
 * the two meet only through plain arrays produced by the seeded generators.
 *
 * Everything is computed in IEEE double precision with straightforward loops
 * (no BLAS/LAPACK, no blocking, no reordering beyond what each definition
 * states).  Inputs arrive in the precision the GPU consumes (complex64
 * snapshots, float32 Gaussian test matrix, int32 index set) and are widened
 * to double before any arithmetic, so GPU-vs-oracle differences are purely
 * arithmetic.
 *
 * Storage: complex matrices are row-major arrays of interleaved (re, im)
 * doubles; an n x n matrix A has A[i][j] at element i*n + j.  A subspace
 * U_s with K columns of length M is stored column-contiguous as [K][M]
 * (column k at offset k*M), the layout the library uses as well.
 *
 * Readings of points the paper leaves open (one line each; the full list is
 * in the design notes):
 *  - steering a_m(theta) = exp(-j*pi*m*sin(theta)), m = 0..M-1, d = lambda/2
 *    (Sec. II-B; the conjugation in the definition of a(theta) taken so that
 *    a source synthesised at +theta peaks at +theta);
 *  - grid theta_l = theta0 + l*dtheta in degrees, l = 0..L-1 (Sec. II-B);
 *  - pseudo-inverses keep eigenvalues lambda > rcond * lambda_max (eq. (8));
 *  - the signal subspace keeps the K leading columns of U_c U_B (Alg. 1/2);
 *  - Method 2 uses V = orth(S^q Omega), C = S V, W = (V^H C)^+ (Alg. 2, with
 *    q = 0 meaning V = orth(Omega));
 *  - the pseudo-spectrum denominator is ||a||^2 - ||U^H a||^2 (expansion of
 *    eq. (5)), clamped below at M * 2^-53 so a noiseless pole stays finite;
 *  - a peak is an index whose value exceeds its left neighbour and is not
 *    below its right neighbour (eq. (6)); the K largest win, ties to the
 *    lower index.
 */
#include <complex.h>
#include <stdio.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

#define OM_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

static zc *zalloc(size_t n) { return (zc *)calloc(n ? n : 1, sizeof(zc)); }

static double zabs2(zc z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

/* C (m x n) = A (m x k) * B (k x n), all row-major complex. */
static void zgemm_nn(const zc *A, const zc *B, zc *C, int m, int k, int n) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      zc acc = 0;
      for (int t = 0; t < k; ++t) acc += A[(size_t)i * k + t] * B[(size_t)t * n + j];
      C[(size_t)i * n + j] = acc;
    }
}

/* C (m x n) = A^H * B with A (k x m), B (k x n). */
static void zgemm_hn(const zc *A, const zc *B, zc *C, int m, int k, int n) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      zc acc = 0;
      for (int t = 0; t < k; ++t) acc += conj(A[(size_t)t * m + i]) * B[(size_t)t * n + j];
      C[(size_t)i * n + j] = acc;
    }
}

/* ------------------------------------------------------------------ */
/* 2x2 Hermitian Jacobi rotation                                        */
/* ------------------------------------------------------------------ */
/*
 * For the Hermitian block [[a, b], [conj(b), d]] (a, d real) return the
 * unitary J = diag(1, e^{-i phi}) * [[c, s], [-s, c]] with b = |b| e^{i phi}
 * and the classical choice t = sgn(z)/(|z| + sqrt(1+z^2)), z = (d-a)/(2|b|),
 * c = 1/sqrt(1+t^2), s = t c, which makes J^H [[a,b],[b*,d]] J diagonal with
 * diagonal (a - t|b|, d + t|b|).  Entries: J = [[jpp, jpq], [jqp, jqq]].
 */
static void jacobi_rot(double a, double d, zc b, zc *jpp, zc *jpq, zc *jqp,
                       zc *jqq, double *t_out) {
  double ab = cabs(b);
  double z = (d - a) / (2.0 * ab);
  double t = (z >= 0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
  double c = 1.0 / sqrt(1.0 + t * t);
  double s = t * c;
  zc e = conj(b) / ab; /* e^{-i phi} */
  *jpp = c;
  *jpq = s;
  *jqp = -s * e;
  *jqq = c * e;
  *t_out = t;
}

/* ------------------------------------------------------------------ */
/* Hermitian eigen-decomposition by cyclic two-sided Jacobi             */
/* ------------------------------------------------------------------ */
/*
 * A (n x n Hermitian, overwritten) -> eigenvalues w (descending) and unitary
 * V (n x n, column k = eigenvector of w[k]).  Sweeps run cyclically by rows
 * until the off-diagonal Frobenius norm is below 1e-15 of the full norm.
 * Returns the number of sweeps, or -1 if max_sweeps was reached.  This is
 * the factorisation of eq. (4) for a Hermitian matrix (V = U there).
 */
static int jacobi_eigh(zc *A, int n, double *w, zc *V, int max_sweeps) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int i = 0; i < n; ++i) A[(size_t)i * n + i] = creal(A[(size_t)i * n + i]);
  int sweep = 0, done = 0;
  for (; sweep <= max_sweeps; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double v = zabs2(A[(size_t)i * n + j]);
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot || off == 0.0) { done = 1; break; }
    if (sweep == max_sweeps) break;
    if (n >= 512 && getenv("FM_ORACLE_PROGRESS")) {
      /* long solves report each sweep (timing runs that must show progress) */
      fprintf(stderr, "oracle: Jacobi n=%d sweep %d, off-diagonal/total %.3g\n", n, sweep,
              off / tot);
      fflush(stderr);
    }
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        zc b = A[(size_t)p * n + q];
        if (b == 0) continue;
        double a = creal(A[(size_t)p * n + p]), d = creal(A[(size_t)q * n + q]);
        /* a rotation below the rounding level of the diagonal changes nothing */
        if (cabs(b) <= 1e-18 * sqrt(fabs(a) * fabs(d))) {
          A[(size_t)p * n + q] = 0;
          A[(size_t)q * n + p] = 0;
          continue;
        }
        zc jpp, jpq, jqp, jqq;
        double t;
        jacobi_rot(a, d, b, &jpp, &jpq, &jqp, &jqq, &t);
        /* A <- A J (columns p, q) */
        for (int r = 0; r < n; ++r) {
          zc arp = A[(size_t)r * n + p], arq = A[(size_t)r * n + q];
          A[(size_t)r * n + p] = arp * jpp + arq * jqp;
          A[(size_t)r * n + q] = arp * jpq + arq * jqq;
        }
        /* A <- J^H A (rows p, q) */
        for (int r = 0; r < n; ++r) {
          zc apr = A[(size_t)p * n + r], aqr = A[(size_t)q * n + r];
          A[(size_t)p * n + r] = conj(jpp) * apr + conj(jqp) * aqr;
          A[(size_t)q * n + r] = conj(jpq) * apr + conj(jqq) * aqr;
        }
        double ab = cabs(b);
        A[(size_t)p * n + p] = a - t * ab;
        A[(size_t)q * n + q] = d + t * ab;
        A[(size_t)p * n + q] = 0;
        A[(size_t)q * n + p] = 0;
        /* V <- V J */
        for (int r = 0; r < n; ++r) {
          zc vrp = V[(size_t)r * n + p], vrq = V[(size_t)r * n + q];
          V[(size_t)r * n + p] = vrp * jpp + vrq * jqp;
          V[(size_t)r * n + q] = vrp * jpq + vrq * jqq;
        }
      }
  }
  /* sort descending (stable selection on index order) */
  int *ord = (int *)malloc(sizeof(int) * (n ? n : 1));
  for (int i = 0; i < n; ++i) ord[i] = i;
  for (int i = 0; i < n; ++i) {
    int best = i;
    for (int j = i + 1; j < n; ++j) {
      double vj = creal(A[(size_t)ord[j] * n + ord[j]]);
      double vb = creal(A[(size_t)ord[best] * n + ord[best]]);
      if (vj > vb || (vj == vb && ord[j] < ord[best])) best = j;
    }
    int tmp = ord[i]; ord[i] = ord[best]; ord[best] = tmp;
  }
  zc *Vs = zalloc((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    w[k] = creal(A[(size_t)ord[k] * n + ord[k]]);
    for (int r = 0; r < n; ++r) Vs[(size_t)r * n + k] = V[(size_t)r * n + ord[k]];
  }
  memcpy(V, Vs, sizeof(zc) * (size_t)n * n);
  free(Vs);
  free(ord);
  return done ? sweep : -1;
}

/* ------------------------------------------------------------------ */
/* thin SVD by one-sided (Hestenes) Jacobi                              */
/* ------------------------------------------------------------------ */
/*
 * C (m x n, m >= n) = U diag(s) V^H with U (m x n) orthonormal columns (zero
 * columns where s = 0), s descending, V (n x n) unitary.  Column pairs are
 * rotated until every pair is orthogonal to 1e-15 relative.  Returns sweeps
 * or -1.
 */
static int jacobi_svd(const zc *C, int m, int n, zc *U, double *s, zc *V,
                      int max_sweeps) {
  zc *W = zalloc((size_t)m * n);
  zc *Q = zalloc((size_t)n * n);
  memcpy(W, C, sizeof(zc) * (size_t)m * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
  int sweep = 0, done = 0;
  for (; sweep < max_sweeps; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double alpha = 0, beta = 0;
        zc gam = 0;
        for (int r = 0; r < m; ++r) {
          zc wp = W[(size_t)r * n + p], wq = W[(size_t)r * n + q];
          alpha += zabs2(wp);
          beta += zabs2(wq);
          gam += conj(wp) * wq;
        }
        if (gam == 0 || cabs(gam) <= 1e-15 * sqrt(alpha * beta)) continue;
        rotated = 1;
        zc jpp, jpq, jqp, jqq;
        double t;
        jacobi_rot(alpha, beta, gam, &jpp, &jpq, &jqp, &jqq, &t);
        for (int r = 0; r < m; ++r) {
          zc wp = W[(size_t)r * n + p], wq = W[(size_t)r * n + q];
          W[(size_t)r * n + p] = wp * jpp + wq * jqp;
          W[(size_t)r * n + q] = wp * jpq + wq * jqq;
        }
        for (int r = 0; r < n; ++r) {
          zc qp = Q[(size_t)r * n + p], qq = Q[(size_t)r * n + q];
          Q[(size_t)r * n + p] = qp * jpp + qq * jqp;
          Q[(size_t)r * n + q] = qp * jpq + qq * jqq;
        }
      }
    if (!rotated) { done = 1; break; }
  }
  double *nrm = (double *)malloc(sizeof(double) * (n ? n : 1));
  int *ord = (int *)malloc(sizeof(int) * (n ? n : 1));
  for (int j = 0; j < n; ++j) {
    double a = 0;
    for (int r = 0; r < m; ++r) a += zabs2(W[(size_t)r * n + j]);
    nrm[j] = sqrt(a);
    ord[j] = j;
  }
  for (int i = 0; i < n; ++i) {
    int best = i;
    for (int j = i + 1; j < n; ++j)
      if (nrm[ord[j]] > nrm[ord[best]] ||
          (nrm[ord[j]] == nrm[ord[best]] && ord[j] < ord[best]))
        best = j;
    int tmp = ord[i]; ord[i] = ord[best]; ord[best] = tmp;
  }
  for (int k = 0; k < n; ++k) {
    int j = ord[k];
    s[k] = nrm[j];
    for (int r = 0; r < m; ++r)
      U[(size_t)r * n + k] = nrm[j] > 0 ? W[(size_t)r * n + j] / nrm[j] : 0;
    for (int r = 0; r < n; ++r) V[(size_t)r * n + k] = Q[(size_t)r * n + j];
  }
  free(nrm); free(ord); free(W); free(Q);
  return done ? sweep : -1;
}

/* ------------------------------------------------------------------ */
/* orth(): modified Gram-Schmidt, two passes                             */
/* ------------------------------------------------------------------ */
/*
 * Orthonormal basis of the column space of C (m x n) -> Q (m x r), r <= n.
 * Each column is projected against the accepted ones twice; a column whose
 * remaining norm is at most 1e-10 of its original norm is linearly dependent
 * and dropped.  Returns r.  This is orth() of Alg. 2 / the QR of eq. (11).
 */
static int mgs2_orth(const zc *C, int m, int n, zc *Q) {
  int r = 0;
  zc *v = zalloc((size_t)m);
  for (int j = 0; j < n; ++j) {
    double n0 = 0;
    for (int i = 0; i < m; ++i) {
      v[i] = C[(size_t)i * n + j];
      n0 += zabs2(v[i]);
    }
    n0 = sqrt(n0);
    for (int pass = 0; pass < 2; ++pass)
      for (int k = 0; k < r; ++k) {
        zc h = 0;
        for (int i = 0; i < m; ++i) h += conj(Q[(size_t)i * n + k]) * v[i];
        for (int i = 0; i < m; ++i) v[i] -= h * Q[(size_t)i * n + k];
      }
    double nv = 0;
    for (int i = 0; i < m; ++i) nv += zabs2(v[i]);
    nv = sqrt(nv);
    if (nv > 0 && nv > 1e-10 * n0) {
      for (int i = 0; i < m; ++i) Q[(size_t)i * n + r] = v[i] / nv;
      ++r;
    }
  }
  /* zero the unused trailing columns */
  for (int k = r; k < n; ++k)
    for (int i = 0; i < m; ++i) Q[(size_t)i * n + k] = 0;
  free(v);
  return r;
}

/* ------------------------------------------------------------------ */
/* eigen-based pseudo-inverse of a Hermitian matrix                      */
/* ------------------------------------------------------------------ */
/*
 * A^+ = V diag(1/lambda_i : lambda_i > rcond * lambda_max) V^H for Hermitian
 * PSD A (n x n).  Eigenvalues at or below the threshold (including negative
 * rounding residue) are dropped.  Returns the kept rank.  Eq. (8).
 */
static int pinv_herm(const zc *A, int n, double rcond, zc *Ap) {
  zc *T = zalloc((size_t)n * n), *V = zalloc((size_t)n * n);
  double *w = (double *)malloc(sizeof(double) * (n ? n : 1));
  memcpy(T, A, sizeof(zc) * (size_t)n * n);
  jacobi_eigh(T, n, w, V, 100);
  double thr = rcond * (n ? w[0] : 0);
  int rank = 0;
  for (int k = 0; k < n; ++k)
    if (w[k] > thr && w[k] > 0) ++rank;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      zc acc = 0;
      for (int k = 0; k < rank; ++k)
        acc += V[(size_t)i * n + k] * conj(V[(size_t)j * n + k]) / w[k];
      Ap[(size_t)i * n + j] = acc;
    }
  free(T); free(V); free(w);
  return rank;
}

/* ------------------------------------------------------------------ */
/* rank restriction shared by both methods (Alg. 1 step 2, Alg. 2 step 2) */
/* ------------------------------------------------------------------ */
/*
 * Given the sketch C (m x n) and Nystrom weight W (n x n): SVD C = Uc Sc Vc^H,
 * B = Sc Vc^H W Vc Sc, B = U_B Sigma_B U_B^H (Hermitian PSD, so its SVD is
 * its eigen-decomposition), U~ = Uc U_B.  Writes the K leading columns into
 * Us ([K][m], column-contiguous) and their eigenvalues into sigma.
 */
static void rank_restrict(const zc *C, int m, int n, const zc *W, int K,
                          double *Us, double *sigma) {
  zc *Uc = zalloc((size_t)m * n), *Vc = zalloc((size_t)n * n);
  double *sc = (double *)malloc(sizeof(double) * (n ? n : 1));
  jacobi_svd(C, m, n, Uc, sc, Vc, 100);
  zc *T1 = zalloc((size_t)n * n), *B = zalloc((size_t)n * n);
  /* T1 = W Vc Sc */
  zgemm_nn(W, Vc, T1, n, n, n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T1[(size_t)i * n + j] *= sc[j];
  /* B = Sc Vc^H T1 */
  zgemm_hn(Vc, T1, B, n, n, n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B[(size_t)i * n + j] *= sc[i];
  /* symmetrise the rounding residue (B is Hermitian by construction) */
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      zc h = 0.5 * (B[(size_t)i * n + j] + conj(B[(size_t)j * n + i]));
      B[(size_t)i * n + j] = h;
      B[(size_t)j * n + i] = conj(h);
    }
  zc *UB = zalloc((size_t)n * n);
  double *wB = (double *)malloc(sizeof(double) * (n ? n : 1));
  jacobi_eigh(B, n, wB, UB, 100);
  for (int k = 0; k < K; ++k) {
    if (k < n) {
      sigma[k] = wB[k];
      for (int r = 0; r < m; ++r) {
        zc acc = 0;
        for (int j = 0; j < n; ++j) acc += Uc[(size_t)r * n + j] * UB[(size_t)j * n + k];
        Us[2 * ((size_t)k * m + r)] = creal(acc);
        Us[2 * ((size_t)k * m + r) + 1] = cimag(acc);
      }
    } else {
      sigma[k] = 0;
      for (int r = 0; r < m; ++r) Us[2 * ((size_t)k * m + r)] = Us[2 * ((size_t)k * m + r) + 1] = 0;
    }
  }
  free(Uc); free(Vc); free(sc); free(T1); free(B); free(UB); free(wB);
}

/* ------------------------------------------------------------------ */
/* exported entry points                                                 */
/* ------------------------------------------------------------------ */

/*
 * Sample covariance, eqs. (2)-(3): R = (1/T) X X^H.  X is complex64,
 * row-major [M][ldx] (row m = channel m, column t = snapshot t).  R is
 * complex128 [M][M].  Every entry is the plain sum over t, then divided by T.
 */
OM_EXPORT void om_covariance(const float *X, int M, int T, long ldx, double *R,
                             int nthreads) {
  (void)nthreads;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads > 0 ? nthreads : 1)
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) {
      double sr = 0, si = 0;
      const float *xi = X + 2 * (size_t)i * ldx, *xj = X + 2 * (size_t)j * ldx;
      for (int t = 0; t < T; ++t) {
        double ar = xi[2 * t], ai = xi[2 * t + 1];
        double br = xj[2 * t], bi = -(double)xj[2 * t + 1]; /* conj(x_j) */
        sr += ar * br - ai * bi;
        si += ar * bi + ai * br;
      }
      R[2 * ((size_t)i * M + j)] = sr / T;
      R[2 * ((size_t)i * M + j) + 1] = si / T;
    }
}

/*
 * Hermitian eigen-decomposition (eq. (4) for Hermitian S): w descending,
 * V [n][n] row-major with column k the k-th eigenvector.  Returns sweeps or -1.
 */
OM_EXPORT int om_eigh(const double *A, int n, double *w, double *V) {
  zc *T = zalloc((size_t)n * n);
  memcpy(T, A, sizeof(zc) * (size_t)n * n);
  int sw = jacobi_eigh(T, n, w, (zc *)V, 200);
  free(T);
  return sw;
}

/* Thin SVD C = U diag(s) V^H (one-sided Jacobi); used by Alg. 1/2 step 2. */
OM_EXPORT int om_svd(const double *C, int m, int n, double *U, double *s, double *V) {
  return jacobi_svd((const zc *)C, m, n, (zc *)U, s, (zc *)V, 200);
}

/* orth() of Alg. 2: Q [m][n] (first r columns valid); returns r. */
OM_EXPORT int om_orth(const double *C, int m, int n, double *Q) {
  return mgs2_orth((const zc *)C, m, n, (zc *)Q);
}

/* Eigen-based pseudo-inverse of a Hermitian PSD matrix (eq. (8)); returns rank. */
OM_EXPORT int om_pinv_herm(const double *A, int n, double rcond, double *Ap) {
  return pinv_herm((const zc *)A, n, rcond, (zc *)Ap);
}

/*
 * Standard MUSIC subspace (eq. (4)-(5)): eigen-decomposition of R (M x M,
 * complex128) by Jacobi; Us [K][M] gets the K leading eigenvectors, w all M
 * eigenvalues in descending order.  Returns sweeps or -1.
 */
OM_EXPORT int om_music_subspace(const double *R, int M, int K, double *Us, double *w) {
  zc *A = zalloc((size_t)M * M), *V = zalloc((size_t)M * M);
  memcpy(A, R, sizeof(zc) * (size_t)M * M);
  int sw = jacobi_eigh(A, M, w, V, 200);
  for (int k = 0; k < K; ++k)
    for (int r = 0; r < M; ++r) {
      Us[2 * ((size_t)k * M + r)] = creal(V[(size_t)r * M + k]);
      Us[2 * ((size_t)k * M + r) + 1] = cimag(V[(size_t)r * M + k]);
    }
  free(A); free(V);
  return sw;
}

/*
 * Fast MUSIC Method 1 (Alg. 1; eqs. (8)-(10)): uniform column sampling.
 *   C = R(:, I), W = pinv(R(I, I)), then the rank restriction of step 2.
 * idx: p distinct indices in [0, M).  Us [K][M] complex128, sigma[K].
 * Returns the kept rank of W.
 */
OM_EXPORT int om_fast_music_sample(const double *R, int M, const int32_t *idx, int p,
                                   int K, double rcond, double *Us, double *sigma) {
  const zc *S = (const zc *)R;
  zc *C = zalloc((size_t)M * p), *Cor = zalloc((size_t)p * p), *W = zalloc((size_t)p * p);
  for (int r = 0; r < M; ++r)
    for (int j = 0; j < p; ++j) C[(size_t)r * p + j] = S[(size_t)r * M + idx[j]];
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) Cor[(size_t)i * p + j] = S[(size_t)idx[i] * M + idx[j]];
  int rank = pinv_herm(Cor, p, rcond, W);
  rank_restrict(C, M, p, W, K, Us, sigma);
  free(C); free(Cor); free(W);
  return rank;
}

/*
 * Fast MUSIC Method 2 (Alg. 2; eq. (11)): Gaussian projection with q power
 * iterations.  C = R Omega; repeat q times { V = orth(C); C = R V }
 * (q = 0: V = orth(Omega), C = R V); W = pinv(V^H R V) = pinv(V^H C); then the
 * rank restriction of step 2.  Omega: real float32 [M][l].  Returns the kept
 * rank of W (the number of columns of V may drop below l if the sketch is
 * rank deficient).
 */
OM_EXPORT int om_fast_music_project(const double *R, int M, const float *Omega, int l,
                                    int q, int K, double rcond, double *Us,
                                    double *sigma) {
  const zc *S = (const zc *)R;
  zc *Om = zalloc((size_t)M * l), *C = zalloc((size_t)M * l), *V = zalloc((size_t)M * l);
  for (size_t i = 0; i < (size_t)M * l; ++i) Om[i] = (double)Omega[i];
  int r = l;
  if (q == 0) {
    r = mgs2_orth(Om, M, l, V);
  } else {
    zgemm_nn(S, Om, C, M, M, l); /* C = S Pi */
    for (int it = 0; it < q; ++it) {
      r = mgs2_orth(C, M, l, V); /* V = orth(C) */
      zgemm_nn(S, V, C, M, M, l); /* C = S V (trailing zero columns stay zero) */
    }
  }
  /* Alg. 2 step 2: C = S V and W = (V^H S V)^+ on the r valid columns */
  zc *Vr = zalloc((size_t)M * r), *Cr = zalloc((size_t)M * r);
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < r; ++j) Vr[(size_t)i * r + j] = V[(size_t)i * l + j];
  zgemm_nn(S, Vr, Cr, M, M, r);
  zc *Cor = zalloc((size_t)r * r), *W = zalloc((size_t)r * r);
  zgemm_hn(Vr, Cr, Cor, r, M, r);
  for (int i = 0; i < r; ++i)
    for (int j = i; j < r; ++j) {
      zc h = 0.5 * (Cor[(size_t)i * r + j] + conj(Cor[(size_t)j * r + i]));
      Cor[(size_t)i * r + j] = h;
      Cor[(size_t)j * r + i] = conj(h);
    }
  int rank = pinv_herm(Cor, r, rcond, W);
  rank_restrict(Cr, M, r, W, K, Us, sigma);
  free(Om); free(C); free(V); free(Vr); free(Cr); free(Cor); free(W);
  return rank;
}

/*
 * Pseudo-spectrum, eqs. (5) and (10), over the grid theta_l = theta0 + l*dtheta
 * (degrees).  a_m = exp(-j pi m sin(theta)); the phase m*sin(theta) is reduced
 * modulo 2 in double before cos/sin.  den = ||a||^2 - ||U^H a||^2 with
 * ||a||^2 = M; P = 1 / max(den, M 2^-53).  Us [K][M] complex128.  den may be
 * NULL.
 */
OM_EXPORT void om_pseudospectrum(const double *Us, int M, int K, double theta0_deg,
                                 double dtheta_deg, int L, double *den, double *P,
                                 int nthreads) {
  (void)nthreads;
  const zc *U = (const zc *)Us;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
  for (int l = 0; l < L; ++l) {
    double th = theta0_deg + (double)l * dtheta_deg;
    double s = sin(th * (M_PI / 180.0));
    zc *c = zalloc((size_t)(K > 0 ? K : 1));
    for (int m = 0; m < M; ++m) {
      double ph = fmod((double)m * s, 2.0);
      zc a = cos(M_PI * ph) - I * sin(M_PI * ph);
      for (int k = 0; k < K; ++k) c[k] += conj(U[(size_t)k * M + m]) * a;
    }
    double proj = 0;
    for (int k = 0; k < K; ++k) proj += zabs2(c[k]);
    double d = (double)M - proj;
    if (den) den[l] = d;
    double floor_ = (double)M * ldexp(1.0, -53);
    P[l] = 1.0 / (d > floor_ ? d : floor_);
    free(c);
  }
}

/*
 * Peak picking, eq. (6).  Index l is a peak if P[l] > P[l-1] (when l > 0) and
 * P[l] >= P[l+1] (when l < L-1); a plateau therefore reports its leftmost
 * point.  The K largest peaks are returned in order of decreasing value, ties
 * broken towards the lower index.  Returns n_found <= K.
 */
OM_EXPORT int om_peaks(const double *P, int L, int K, int32_t *idx, double *val) {
  int n = 0;
  int *cand = (int *)malloc(sizeof(int) * (L ? L : 1));
  for (int l = 0; l < L; ++l) {
    int left = (l == 0) || (P[l] > P[l - 1]);
    int right = (l == L - 1) || (P[l] >= P[l + 1]);
    if (left && right) cand[n++] = l;
  }
  int found = 0;
  for (int k = 0; k < K && k < n; ++k) {
    int best = k;
    for (int j = k + 1; j < n; ++j) {
      double vj = P[cand[j]], vb = P[cand[best]];
      if (vj > vb || (vj == vb && cand[j] < cand[best])) best = j;
    }
    int tmp = cand[k]; cand[k] = cand[best]; cand[best] = tmp;
    idx[k] = cand[k];
    val[k] = P[cand[k]];
    ++found;
  }
  free(cand);
  return found;
}

/*
 * Number of sources from the sketch eigenvalues (the pre-estimation of K that
 * Sec. V-D proposes, with Akaike's information criterion or the minimum
 * description length; both in their usual form for N snapshots of an
 * M-channel array, where the noise eigenvalues lambda_{k+1..M} enter through
 * the ratio of their arithmetic to their geometric mean):
 *   L(k)   = N * ((M-k) * log(mean of noise) - sum of log(noise))      >= 0
 *   AIC(k) = 2 L(k) + 2 k (2M - k)             (kind 0)
 *   MDL(k) = L(k) + k (2M - k) log(N) / 2      (kind 1)
 * Only the n eigenvalues of the Nystrom approximation are known (sig,
 * descending).  Reading: those above rcond * sig[0] (and > 0) are kept, r of
 * them; the other M - r eigenvalues of R are taken equal to their mean
 * mu = (trR - sum of kept) / (M - r), which the exact trace of R fixes.
 * k runs over 0..r (0..r-1 when r == M, where nothing is completed).
 * crit[k] gets the criterion for k = 0..n (+INFINITY where not evaluated).
 * Returns the first minimiser; returns r (crit all +INFINITY) when M > r and
 * mu <= 0, i.e. the kept eigenvalues already hold the whole trace.
 */
OM_EXPORT int om_order(const double *sig, int n, int M, int N, double trR, double rcond,
                       int kind, double *crit) {
  for (int k = 0; k <= n; ++k) crit[k] = INFINITY;
  int r = 0;
  while (r < n && sig[r] > 0.0 && sig[r] > rcond * sig[0]) ++r;
  double kept = 0.0;
  for (int i = 0; i < r; ++i) kept += sig[i];
  const int nc = M - r; /* completed eigenvalues */
  double mu = 0.0;
  if (nc > 0) {
    mu = (trR - kept) / nc;
    if (!(mu > 0.0)) return r;
  }
  const int kmax = nc > 0 ? r : r - 1;
  int best = 0;
  for (int k = 0; k <= kmax; ++k) {
    double s = 0.0, ls = 0.0;
    for (int i = k; i < r; ++i) {
      s += sig[i];
      ls += log(sig[i]);
    }
    if (nc > 0) {
      s += nc * mu;
      ls += nc * log(mu);
    }
    const int m = M - k;
    const double Lk = (double)N * (m * log(s / m) - ls);
    const double pen = (double)k * (2.0 * M - k);
    crit[k] = kind == 0 ? 2.0 * Lk + 2.0 * pen : Lk + 0.5 * pen * log((double)N);
    if (crit[k] < crit[best]) best = k;
  }
  return best;
}

/*
 * Eigenvalues of a general complex n x n matrix: Householder reduction to
 * upper Hessenberg form, then implicitly shifted QR (one complex Wilkinson
 * shift per step from the trailing 2x2 of the active block, Givens bulge
 * chase, deflation where a subdiagonal falls below eps * the neighbouring
 * diagonal).  Eigenvalues only.  A is overwritten.  Returns the number of
 * QR steps, or -1 past 30 n steps.
 */
static int hessenberg_qr(zc *A, int n, zc *w) {
  for (int c = 0; c + 2 < n; ++c) {
    const int len = n - c - 1;
    zc *v = zalloc(len);
    double nx = 0;
    for (int i = 0; i < len; ++i) {
      v[i] = A[(size_t)(c + 1 + i) * n + c];
      nx += zabs2(v[i]);
    }
    nx = sqrt(nx);
    if (nx > 0) {
      const double a0 = cabs(v[0]);
      const zc ph = a0 > 0 ? v[0] / a0 : 1.0;
      v[0] += ph * nx; /* v = x + sign(x0) |x| e_0 */
      double nv = 0;
      for (int i = 0; i < len; ++i) nv += zabs2(v[i]);
      nv = sqrt(nv);
      for (int i = 0; i < len; ++i) v[i] /= nv;
      /* A <- (I - 2 v v^H) A on rows c+1.. */
      for (int j = 0; j < n; ++j) {
        zc s = 0;
        for (int i = 0; i < len; ++i) s += conj(v[i]) * A[(size_t)(c + 1 + i) * n + j];
        for (int i = 0; i < len; ++i) A[(size_t)(c + 1 + i) * n + j] -= 2.0 * v[i] * s;
      }
      /* A <- A (I - 2 v v^H) on columns c+1.. */
      for (int i = 0; i < n; ++i) {
        zc s = 0;
        for (int j = 0; j < len; ++j) s += A[(size_t)i * n + c + 1 + j] * v[j];
        for (int j = 0; j < len; ++j) A[(size_t)i * n + c + 1 + j] -= 2.0 * s * conj(v[j]);
      }
    }
    free(v);
  }
  int steps = 0, hi = n - 1;
  const double eps = 2.220446049250313e-16;
  while (hi >= 0) {
    if (hi == 0) {
      w[0] = A[0];
      break;
    }
    int l = hi;
    while (l > 0) {
      const double sub = cabs(A[(size_t)l * n + l - 1]);
      double ref = cabs(A[(size_t)l * n + l]) + cabs(A[(size_t)(l - 1) * n + l - 1]);
      if (ref == 0) ref = 1.0;
      if (sub <= eps * ref) break;
      --l;
    }
    if (l == hi) { /* 1 x 1 block converged */
      w[hi] = A[(size_t)hi * n + hi];
      --hi;
      continue;
    }
    if (++steps > 30 * n) return -1;
    /* Wilkinson shift: the eigenvalue of the trailing 2x2 nearer to its last entry */
    const zc a = A[(size_t)(hi - 1) * n + hi - 1], b = A[(size_t)(hi - 1) * n + hi];
    const zc cc = A[(size_t)hi * n + hi - 1], d = A[(size_t)hi * n + hi];
    const zc tr2 = 0.5 * (a + d), det = a * d - b * cc;
    const zc disc = csqrt(tr2 * tr2 - det);
    const zc e1 = tr2 + disc, e2 = tr2 - disc;
    zc mu = cabs(e1 - d) <= cabs(e2 - d) ? e1 : e2;
    if (steps % 11 == 0) mu = d + cabs(cc); /* exceptional shift against stagnation */
    zc x = A[(size_t)l * n + l] - mu, y = A[(size_t)(l + 1) * n + l];
    for (int k = l; k < hi; ++k) {
      if (k > l) {
        x = A[(size_t)k * n + k - 1];
        y = A[(size_t)(k + 1) * n + k - 1];
      }
      const double ax = cabs(x), rho = sqrt(ax * ax + zabs2(y));
      if (rho == 0) continue;
      double gc;
      zc gs;
      if (ax == 0) {
        gc = 0;
        gs = conj(y) / cabs(y);
      } else {
        gc = ax / rho;
        gs = (x / ax) * conj(y) / rho;
      }
      /* rows k, k+1: [c s; -conj(s) c] */
      for (int j = (k > l ? k - 1 : l); j <= hi; ++j) {
        const zc p = A[(size_t)k * n + j], q = A[(size_t)(k + 1) * n + j];
        A[(size_t)k * n + j] = gc * p + gs * q;
        A[(size_t)(k + 1) * n + j] = -conj(gs) * p + gc * q;
      }
      /* columns k, k+1: times the conjugate transpose */
      const int iend = k + 2 < hi ? k + 2 : hi;
      for (int i = l; i <= iend; ++i) {
        const zc p = A[(size_t)i * n + k], q = A[(size_t)i * n + k + 1];
        A[(size_t)i * n + k] = gc * p + conj(gs) * q;
        A[(size_t)i * n + k + 1] = -gs * p + gc * q;
      }
    }
  }
  return steps;
}

/* Eigenvalues of a general complex matrix (for pinning hessenberg_qr). */
OM_EXPORT int om_eigvals(const double *A, int n, double *w) {
  zc *T = zalloc((size_t)n * n);
  memcpy(T, A, sizeof(zc) * (size_t)n * n);
  int r = hessenberg_qr(T, n, (zc *)w);
  free(T);
  return r;
}

/*
 * ESPRIT on a signal subspace (the extension of the fast subspace to other
 * estimators that the conclusion proposes; reading: least-squares ESPRIT on
 * the two maximally overlapping subarrays of the ULA).  With U1 = rows
 * 0..M-2 and U2 = rows 1..M-1 of U_s (M x K), Psi = (U1^H U1)^-1 U1^H U2
 * (Gaussian elimination with partial pivoting); its eigenvalues are
 * exp(-j pi sin(theta_k)) for a_m = exp(-j pi m sin(theta)), so
 * theta_k = asin(-arg(phi_k) / pi).  Us is [K][M] column-contiguous.
 * doa_deg gets the K angles in degrees, ascending.  Returns the QR step
 * count, or -1 if the eigenvalue iteration did not converge.
 */
OM_EXPORT int om_esprit(const double *Us, int M, int K, double *doa_deg) {
  const zc *U = (const zc *)Us;
  zc *Aug = zalloc((size_t)K * 2 * K);
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) {
      zc g = 0, h = 0;
      for (int m = 0; m + 1 < M; ++m) {
        g += conj(U[(size_t)a * M + m]) * U[(size_t)b * M + m];
        h += conj(U[(size_t)a * M + m]) * U[(size_t)b * M + m + 1];
      }
      Aug[(size_t)a * 2 * K + b] = g;
      Aug[(size_t)a * 2 * K + K + b] = h;
    }
  /* [G | H] -> [I | G^-1 H] */
  for (int c = 0; c < K; ++c) {
    int piv = c;
    for (int r = c + 1; r < K; ++r)
      if (cabs(Aug[(size_t)r * 2 * K + c]) > cabs(Aug[(size_t)piv * 2 * K + c])) piv = r;
    if (piv != c)
      for (int j = 0; j < 2 * K; ++j) {
        const zc t = Aug[(size_t)c * 2 * K + j];
        Aug[(size_t)c * 2 * K + j] = Aug[(size_t)piv * 2 * K + j];
        Aug[(size_t)piv * 2 * K + j] = t;
      }
    const zc p = Aug[(size_t)c * 2 * K + c];
    for (int j = 0; j < 2 * K; ++j) Aug[(size_t)c * 2 * K + j] /= p;
    for (int r = 0; r < K; ++r) {
      if (r == c) continue;
      const zc f = Aug[(size_t)r * 2 * K + c];
      for (int j = 0; j < 2 * K; ++j) Aug[(size_t)r * 2 * K + j] -= f * Aug[(size_t)c * 2 * K + j];
    }
  }
  zc *Psi = zalloc((size_t)K * K), *w = zalloc(K);
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) Psi[(size_t)a * K + b] = Aug[(size_t)a * 2 * K + K + b];
  const int st = hessenberg_qr(Psi, K, w);
  for (int k = 0; k < K; ++k) {
    double u = -carg(w[k]) / 3.141592653589793;
    if (u > 1) u = 1;
    if (u < -1) u = -1;
    doa_deg[k] = asin(u) * (180.0 / 3.141592653589793);
  }
  /* ascending (insertion sort) */
  for (int i = 1; i < K; ++i) {
    const double t = doa_deg[i];
    int j = i - 1;
    while (j >= 0 && doa_deg[j] > t) {
      doa_deg[j + 1] = doa_deg[j];
      --j;
    }
    doa_deg[j + 1] = t;
  }
  free(Aug); free(Psi); free(w);
  return st;
}
