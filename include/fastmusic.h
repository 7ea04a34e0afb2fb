/*
 * fastmusic.h -- C ABI of the MI355X (gfx950) fast-MUSIC angle-of-arrival path.
 *
 * Paper: B. Li, S. Wang, J. Zhang, X. Cao, C. Zhao, "Ultra-Fast Accurate AoA
 * Estimation via Automotive Massive-MIMO Radar", arXiv:1911.07434.
 *
 * The path has four stages, each one entry point:
 *   fm_covariance        R = X X^H / T                    eqs. (2)-(3)
 *   fm_subspace_sample   Method 1: column sampling        Alg. 1, eqs. (8)-(9)
 *   fm_subspace_project  Method 2: projection + power it. Alg. 2, eq. (11)
 *   fm_pseudospectrum    P(theta) = 1/(||a||^2-||U^H a||^2) eqs. (5), (10)
 *   fm_peaks             K largest local maxima of P      eq. (6)
 * plus a batched form (fm_plan_*) that runs many frames of different shapes
 * through the same kernels, one launch per stage.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.  Every array argument is a DEVICE pointer unless stated otherwise;
 *   the caller allocates and owns it.  The library never frees caller memory.
 * Complex.   complex64 = interleaved (re, im) float pairs; complex128 =
 *   interleaved (re, im) double pairs.
 * Streams.   `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream).  Every call only enqueues work on that stream and returns; no
 *   call synchronises.  Outputs are valid once the stream's work completes.
 * Workspace. Scratch memory comes from the context's arena, sized at
 *   fm_create; single-frame calls that need more than the arena return
 *   FM_E_WORKSPACE without launching.  Plans own their own workspace,
 *   allocated once in fm_plan_create.  Hot-path calls never allocate.
 * Errors.    Argument, launch and workspace errors are returned synchronously
 *   as fm_status with a message in fm_last_error; nothing is launched when an
 *   argument is rejected.  Numerical conditions that can only be seen on the
 *   device are OR-ed into a per-frame uint32 status word (FM_ST_* bits).
 * Threads.   A context is used by one host thread at a time.  Calls that
 *   overlap on the same context from different streams are allowed only for
 *   entry points that use no arena workspace (fm_covariance, fm_peaks) or
 *   for plans (each plan owns its workspace).
 * Determinism. The same inputs give bitwise identical outputs whether a frame
 *   runs alone or inside a plan with other frames.
 * Steering.  a_m(theta) = exp(-j*pi*m*sin(theta)), m = 0..M-1 (half-wavelength
 *   ULA, Sec. II-B; the sign chosen so that a source at +theta peaks at
 *   +theta).  Grid theta_l = theta0_deg + l*dtheta_deg, l = 0..L-1.
 */
#ifndef FASTMUSIC_H
#define FASTMUSIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fm_ctx fm_ctx;
typedef struct fm_plan fm_plan;

typedef enum {
  FM_OK = 0,
  FM_E_ARG = 1,          /* invalid argument; nothing launched */
  FM_E_HIP = 2,          /* HIP runtime error (message in fm_last_error) */
  FM_E_WORKSPACE = 3,    /* arena too small for this call */
  FM_E_UNSUPPORTED = 4   /* valid but not supported by this library */
} fm_status;

/* Operand precision of the matrix-core products.  Accumulation is FP32 in
 * every mode.
 *   covariance (fm_covariance, stage 1 of a plan): operands rounded to the
 *     given precision.  FM_FP16X3 and FM_BF16X3 write each snapshot as
 *     hi + lo (hi its 16-bit rounding, lo the 16-bit rounding of the
 *     remainder) and accumulate lo*hi + hi*lo + hi*hi on the 16-bit matrix
 *     cores: FP32-level error (22 significant bits per operand with FP16,
 *     16 with BF16) at three 16-bit products per complex product.  FP16
 *     halves keep 22 bits for snapshots of magnitude >= 2^-3 (below that lo
 *     loses bits: absolute error <= 2^-25 per value); BF16 has FP32's range.
 *   pseudo-spectrum (fm_pseudospectrum): FM_FP32 evaluates the spectrum as a
 *     polynomial in sin(theta) on FP32 products (one length-M product per
 *     angle, see fm_pseudospectrum); FM_FP16 splits U_s and the steering
 *     twiddles into FP16 hi + lo halves and accumulates hi*hi + hi*lo +
 *     lo*hi (~22-bit products), K products per angle; FM_FP16X3 is the
 *     same pass.  fm_pseudospectrum rejects FM_BF16 and FM_BF16X3
 *     (FM_E_UNSUPPORTED).  Plans run each frame's fm_frame.spec_prec pass
 *     (default FM_FP32, the faster and more accurate of the two).
 *   sketch products Y = R V (fm_subspace_project, stage 2 of a plan):
 *     FM_FP32 uses FP32 products; every 16-bit precision splits R and V into
 *     FP16 hi + lo halves (power-of-two scaled) and accumulate hi*hi + hi*lo
 *     + lo*hi, for sketch widths l <= 32 (wider sketches use FP32 products).
 *     A plain 16-bit rounding of R would move the peak-region denominators
 *     by more than 1e-2 dB, so no precision drops the lo halves.  Method 1
 *     (fm_subspace_sample) has no such product.
 * The small dense steps (orthonormalisation, eigen-solves, peak-region
 * denominators) are FP64 in every mode. */
typedef enum {
  FM_FP32 = 0,   /* FP32 operands on FP32 MFMA */
  FM_BF16 = 1,   /* BF16 operands on BF16 MFMA */
  FM_FP16 = 2,   /* FP16 operands on FP16 MFMA */
  FM_FP16X3 = 3, /* FP16 hi + lo operands, three products, on FP16 MFMA */
  FM_BF16X3 = 4  /* BF16 hi + lo operands, three products, on BF16 MFMA */
} fm_prec;

/* Subspace method of a frame in a plan. */
typedef enum {
  FM_METHOD_PROJECT = 0,   /* Method 2, Alg. 2 */
  FM_METHOD_SAMPLE = 1,    /* Method 1, Alg. 1 */
  FM_METHOD_PROJECT_X = 2, /* Method 2 with every product R V formed as
                              X (X^H V) / T: R is never computed (the frame's R
                              may be null); see fm_subspace_project_x */
  FM_METHOD_SAMPLE_X = 3   /* Method 1 with C = R(:, I) formed as
                              X X(I, :)^H / T: R is never computed (R may be
                              null); see fm_subspace_sample_x */
} fm_method;

/* per-frame device status bits, written by the subspace stage (the peak and
 * model-order bits OR-ed in by the stages that find them).  Outputs are
 * meaningful only if status & (FM_ST_NONFINITE | FM_ST_BAD_INDEX) == 0. */
#define FM_ST_NONFINITE      1u  /* NaN/Inf in the final sketch Gram matrix or
                                    its eigenvalues: a NaN or Inf in X or R
                                    reaches every entry of it */
#define FM_ST_ORTH_FALLBACK  2u  /* a Cholesky QR of a sketch (orth() of
                                    Alg. 2) met a pivot below 1e-10 of the
                                    largest diagonal entry; that step used the
                                    Gram eigen-route instead (same span) */
#define FM_ST_EIG_MAXIT      4u  /* a Jacobi eigen-solve hit its sweep limit */
#define FM_ST_RANK_DEFICIENT 8u  /* fewer than K non-zero directions survived */
#define FM_ST_FEW_PEAKS     16u  /* fewer than K local maxima */
#define FM_ST_BAD_INDEX     32u  /* sampled index outside [0, M) or repeated */
#define FM_ST_ORDER_AT_LIMIT 64u  /* model-order estimate equals the sketch width
                                    n: the sketch was too narrow to bound it */
#define FM_ST_CORE_TRUNCATED 128u /* the pseudo-inverse of the core (eq. (8))
                                     kept fewer than n eigen-directions (those
                                     <= rcond * the largest were dropped); the
                                     kept rank is the number of non-zero
                                     entries of the model-order eigenvalue
                                     array (plans) or of sigma when K = n */
/* the bits that describe how a result was reached (expected with noiseless
 * or very high-SNR frames, or T < n), not a failure */
#define FM_ST_NOTES (FM_ST_ORTH_FALLBACK | FM_ST_CORE_TRUNCATED)

/* Default relative threshold of the eigen-based pseudo-inverse, eq. (8):
 * eigenvalues lambda <= rcond * lambda_max of the p x p (or l x l) core are
 * dropped. */
#define FM_RCOND_DEFAULT 1e-6

/* ------------------------------------------------------------------------ */
/* context                                                                  */
/* ------------------------------------------------------------------------ */

/* Create a context on HIP device `device` with a device arena of
 * `workspace_bytes` for single-frame calls (0 = a default of 64 MiB).
 * *out receives the context; on failure *out is NULL. */
fm_status fm_create(int device, size_t workspace_bytes, fm_ctx **out);

/* Release the context and its arena (waits for the device to go idle). */
fm_status fm_destroy(fm_ctx *ctx);

/* Static text of a status code. */
const char *fm_status_string(fm_status s);

/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *fm_last_error(const fm_ctx *ctx);

/* Arena bytes one single-frame call sequence needs for an M-channel frame
 * with sketch width n (l for Method 2, p for Method 1), K sources and an
 * L-angle grid (a plan allocates this much per frame). */
size_t fm_workspace_bytes(int M, int n, int K, int L);

/* ------------------------------------------------------------------------ */
/* stage 1: covariance, eqs. (2)-(3)                                        */
/* ------------------------------------------------------------------------ */

/* R = X X^H / T.
 *   X   complex64 [M][ldx], row m = channel m, column t = snapshot t (ldx >= T)
 *   R   complex64 [M][ldr] (ldr >= M); every entry is written; R is exactly
 *       Hermitian (R[j][i] == conj(R[i][j]) bit for bit, imaginary diagonal 0)
 *   prec operand precision (accumulation FP32; the 1/T scale is applied in
 *       FP32 after accumulation).  FM_FP32 forms each complex product with
 *       three real products (Gauss: (a+b)c, a(c+d), b(c-d)), whose FP32
 *       rounding stays at FP32 level; integer-valued snapshots with exactly
 *       representable partial sums give exact results at every precision.
 * Requires M >= 1, T >= 1.  No workspace. */
fm_status fm_covariance(fm_ctx *ctx, void *stream, const void *X, int M, int T,
                        int64_t ldx, void *R, int64_t ldr, fm_prec prec);

/* ------------------------------------------------------------------------ */
/* stage 2a: Method 1 -- uniform column sampling + Nystrom, Alg. 1           */
/* ------------------------------------------------------------------------ */

/* Signal subspace of S~ = C W C^H with C = R(:, I) and W = pinv(R(I, I))
 * (eqs. (8)-(9)), restricted to its K leading eigen-directions (Alg. 1 step 2).
 *   R      complex64 [M][ldr], Hermitian (rows idx are read)
 *   idx    int32 [p] distinct indices in [0, M) (device)
 *   rcond  pseudo-inverse threshold (FM_RCOND_DEFAULT)
 *   Us     complex128 [K][M]: column k of U_s stored contiguously, ordered by
 *          decreasing sigma.  Column phases are arbitrary: the contract is the
 *          projector U_s U_s^H.
 *   sigma  double [K]: leading eigenvalues of S~ (descending)
 *   status uint32 [1] (device): FM_ST_* bits of this frame (overwritten)
 * Requires 1 <= K <= p <= M.  Uses workspace. */
fm_status fm_subspace_sample(fm_ctx *ctx, void *stream, const void *R, int M, int64_t ldr,
                             const int32_t *idx, int p, int K, double rcond,
                             void *Us, double *sigma, uint32_t *status);

/* ------------------------------------------------------------------------ */
/* stage 2b: Method 2 -- Gaussian projection + power iterations, Alg. 2      */
/* ------------------------------------------------------------------------ */

/* V = orth(R^q Omega), C = R V, W = pinv(V^H C); U_s = K leading
 * eigen-directions of S~ = C W C^H (Alg. 2, eq. (11)); q = 0 means
 * V = orth(Omega).  Exactly q+1 products with R are formed.
 *   Omega  float32 [M][l], real N(0,1) entries (caller-drawn)
 *   prec   operand precision of the products with R
 *   Us, sigma, status as in fm_subspace_sample
 * Requires 1 <= K <= l <= M, 0 <= q <= 16, l <= 64.  Uses workspace. */
fm_status fm_subspace_project(fm_ctx *ctx, void *stream, const void *R, int M, int64_t ldr,
                              const float *Omega, int l, int q, int K, double rcond,
                              fm_prec prec, void *Us, double *sigma, uint32_t *status);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as fm_subspace_project -- the same kernels, bit-identical
 * results -- with its workspace in a fixed device array of
 * FM_NOALLOC_SCRATCH_BYTES that the library holds on each GPU until the
 * process ends (its address is taken once, by fm_create).  The call
 * allocates nothing and does not use the context's arena.  Requires
 * fm_workspace_bytes(M, l, K, 0) <= FM_NOALLOC_SCRATCH_BYTES (FM_E_WORKSPACE
 * otherwise; e.g. M = 4096 with l = K = 64 fits).  Every call on one GPU
 * shares the array: calls that overlap on a GPU (other streams, other
 * contexts, other threads) race and must be serialised by the caller. */
#define FM_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
fm_status fm_subspace_project_noalloc(fm_ctx *ctx, void *stream, const void *R, int M,
                                      int64_t ldr, const float *Omega, int l, int q, int K,
                                      double rcond, fm_prec prec, void *Us, double *sigma,
                                      uint32_t *status);

/* Method 1 straight from the snapshots: the same algorithm as
 * fm_subspace_sample on R = X X^H / T, with the sampled columns formed as
 * C = R(:, I) = X X(I, :)^H / T and the core R(I, I) taken from C(I, :) --
 * 8 M T p real flops instead of 4 M^2 T for R.
 *   X      complex64 [M][ldx] snapshots
 *   other arguments as fm_subspace_sample
 * Requires T >= 1, ldx >= T, 1 <= K <= p <= min(M, 64).  Uses workspace:
 * fm_workspace_bytes(M, p, K, 0) plus T * p * 8 bytes (rounded up to 256). */
fm_status fm_subspace_sample_x(fm_ctx *ctx, void *stream, const void *X, int M, int T,
                               int64_t ldx, const int32_t *idx, int p, int K, double rcond,
                               void *Us, double *sigma, uint32_t *status);

/* Method 2 straight from the snapshots: the same algorithm as
 * fm_subspace_project on R = X X^H / T (eqs. (2)-(3)), with every product
 * R V evaluated as X (X^H V) / T, so R is never formed -- identical in exact
 * arithmetic, (q+1) * 16 M T l real flops instead of 4 M^2 T for R, at the
 * cost of two reads of X per product.
 *   X      complex64 [M][ldx] snapshots (as fm_covariance)
 *   prec   FM_FP32 only (FM_E_UNSUPPORTED otherwise)
 *   other arguments as fm_subspace_project
 * Requires T >= 1, ldx >= T and the fm_subspace_project limits.  Uses
 * workspace: fm_workspace_bytes(M, l, K, 0) plus T * l * 8 bytes (rounded up
 * to 256). */
fm_status fm_subspace_project_x(fm_ctx *ctx, void *stream, const void *X, int M, int T,
                                int64_t ldx, const float *Omega, int l, int q, int K,
                                double rcond, fm_prec prec, void *Us, double *sigma,
                                uint32_t *status);

/* ------------------------------------------------------------------------ */
/* model order: the number of sources when K is not known, Sec. V-D          */
/* ------------------------------------------------------------------------ */

/* Sec. V-D proposes estimating K before the fast method runs (with Akaike's
 * information criterion or the minimum description length) and sizing the
 * sketch from the estimate, p = ceil(1.2 K) in its Fig. 6. */
typedef enum {
  FM_ORDER_AIC = 0,  /* 2 L(k) + 2 k (2M - k) */
  FM_ORDER_MDL = 1   /* L(k) + k (2M - k) log(N) / 2 */
} fm_order_rule;

/* K_hat = argmin over k of the criterion, where for N snapshots of M
 * channels L(k) = N ((M-k) log(mean of noise) - sum of log(noise)) over the
 * noise eigenvalues lambda_{k+1..M} of R.  Of those only the n eigenvalues
 * of the Nystrom approximation are known (run fm_subspace_project, or
 * fm_subspace_sample, with K = n: sigma then holds all n): the ones above
 * rcond * eig[0] are used as they are (r of them) and the other M - r are
 * taken equal to their mean (tr R - sum of kept) / (M - r), which the trace
 * of R fixes; k runs over 0..r (0..r-1 when r == M).  If the kept
 * eigenvalues already hold the whole trace (noiseless data), K_hat = r.
 *   R       complex64 [M][ldr] (its diagonal gives the trace)
 *   T       snapshots behind R (N of the criteria)
 *   eig     double [n] (device): eigenvalues of S~, descending (0 past its
 *           rank), e.g. the sigma of a subspace call with K = n
 *   rule    fm_order_rule
 *   K_hat   int32 [1] (device)
 *   crit    double [n + 1] (device) criterion per k (+inf where not
 *           evaluated), or null
 *   status  uint32 [1] (device): FM_ST_ORDER_AT_LIMIT when K_hat == n
 *           (overwritten)
 * Requires M >= 2, T >= 1, 1 <= n <= min(M, 256).  No workspace. */
fm_status fm_order(fm_ctx *ctx, void *stream, const void *R, int M, int64_t ldr, int T,
                   const double *eig, int n, double rcond, int rule, int32_t *K_hat,
                   double *crit, uint32_t *status);

/* ------------------------------------------------------------------------ */
/* ESPRIT on the fast subspace (the conclusion's extension, Sec. VI)        */
/* ------------------------------------------------------------------------ */

/* Angles of the K sources from a signal subspace by least-squares ESPRIT on
 * the two shifted subarrays of the ULA: with U1 = rows 0..M-2 and U2 = rows
 * 1..M-1 of U_s, Psi = (U1^H U1)^-1 U1^H U2 and its eigenvalues are
 * exp(-j pi sin(theta_k)) for the steering of fm_pseudospectrum, so
 * theta_k = asin(-arg(phi_k) / pi).  Computed in FP64 (Gauss-Jordan with
 * partial pivoting, Householder Hessenberg reduction, shifted QR) by one
 * workgroup; no spectrum and no peak search.
 *   Us       complex128 [K][M] orthonormal columns (stage 2 output)
 *   doa_deg  double [K] (device): the angles in degrees, ascending
 *   status   uint32 [1] (device): FM_ST_EIG_MAXIT if the QR iteration hit
 *            its step limit (overwritten)
 * Requires 1 <= K < M, K <= 32.  No workspace. */
fm_status fm_esprit(fm_ctx *ctx, void *stream, const void *Us, int M, int K, double *doa_deg,
                    uint32_t *status);

/* ------------------------------------------------------------------------ */
/* stage 3: pseudo-spectrum, eqs. (5) and (10)                               */
/* ------------------------------------------------------------------------ */

/* P_l = 1 / (M - ||U_s^H a(theta_l)||^2) on the grid theta_l.  With FM_FP32
 * the bulk of the grid is evaluated through the identity
 * ||U_s^H a||^2 = 2 Re sum_d h'_d a_d(theta), h'_d the lag sums of U_s U_s^H
 * along its d-th diagonal (h'_0 halved): one length-M product per angle on
 * FP32 matrix cores, whatever K is; with FM_FP16 through the K products
 * c_k = u_k^H a with compensated FP16 hi + lo operands.  Every point whose denominator falls
 * below M/16 -- the cancellation-prone region around peaks -- is recomputed
 * in FP64.  A denominator below M*2^-53 is
 * clamped there (the pole of a noiseless on-grid source).
 *   Us  complex128 [K][M] orthonormal columns (stage 2 output)
 *   P   float32 [L] (linear scale)
 * Requires 1 <= K <= 64, K <= M, L >= 1, dtheta_deg > 0.  Uses workspace. */
fm_status fm_pseudospectrum(fm_ctx *ctx, void *stream, const void *Us, int M, int K,
                            double theta0_deg, double dtheta_deg, int L, fm_prec prec,
                            float *P);

/* ------------------------------------------------------------------------ */
/* stage 4: peaks, eq. (6)                                                   */
/* ------------------------------------------------------------------------ */

/* l is a peak if P[l] > P[l-1] (l > 0) and P[l] >= P[l+1] (l < L-1); a
 * plateau reports its leftmost point.  The K largest peaks are written in
 * order of decreasing value, ties to the lower index.
 *   P        float32 [L]
 *   idx      int32 [K]   grid indices (angle = theta0 + idx*dtheta)
 *   val      float32 [K] P at those indices
 *   n_found  int32 [1]   number of peaks written (<= K)
 * Requires 1 <= L <= 1048576, 1 <= K <= 64.  No workspace. */
fm_status fm_peaks(fm_ctx *ctx, void *stream, const float *P, int L, int K,
                   int32_t *idx, float *val, int32_t *n_found);

/* ------------------------------------------------------------------------ */
/* batched frames: one launch per stage for many frames                     */
/* ------------------------------------------------------------------------ */

/* One frame of a plan.  All pointers are device pointers owned by the caller
 * and must stay valid while the plan is used. */
typedef struct {
  const void *X;      /* complex64 [M][ldx] snapshots */
  int64_t ldx;
  int M, T;
  void *R;            /* complex64 [M][ldr] covariance (written by stage 1;
                         not used, may be null, for FM_METHOD_PROJECT_X) */
  int64_t ldr;
  int K;              /* number of sources */
  int method;         /* fm_method */
  int n;              /* sketch width: l (Method 2) or p (Method 1) */
  int q;              /* power iterations (Method 2) */
  double rcond;
  const float *Omega; /* float32 [M][n] (Method 2) */
  const int32_t *idx; /* int32 [n] (Method 1) */
  void *Us;           /* complex128 [K][M] */
  double *sigma;      /* double [K] */
  uint32_t *status;   /* uint32 [1] */
  int L;
  double theta0_deg, dtheta_deg;
  float *P;           /* float32 [L] */
  int32_t *peak_idx;  /* int32 [K] */
  float *peak_val;    /* float32 [K] */
  int32_t *n_found;   /* int32 [1] */
  /* model-order estimate (Sec. V-D), as fm_order, formed at the end of the
   * subspace stage from all n eigenvalues of this frame's S~ and the trace
   * of R; null: none.  Methods 1 and 2 on R only; its FM_ST_ORDER_AT_LIMIT
   * bit is OR-ed into status. */
  int32_t *K_hat;     /* int32 [1] */
  double *order_crit; /* double [n + 1], or null */
  int order_rule;     /* fm_order_rule */
  /* ESPRIT angles of this frame's U_s, as fm_esprit, formed at the end of
   * the subspace stage (K <= 32); null: none.  FM_ST_EIG_MAXIT is OR-ed
   * into status. */
  double *esprit_deg; /* double [K] */
  /* pseudo-spectrum pass of this frame (as fm_pseudospectrum's prec):
   * FM_FP32 (0, the default) the FP32 polynomial pass; FM_FP16 (or
   * FM_FP16X3) the split hi + lo FP16 projection c_k = u_k^H a(theta) on the
   * matrix cores.  Both recompute the peak-region denominators in FP64. */
  int spec_prec;
} fm_frame;

/* Build a plan for n_frames frames (host array, copied): validates every
 * frame, builds the per-stage work lists (longest-first), uploads them and
 * allocates the plan's workspace.  Synchronises the device once.  Each
 * frame is computed exactly as the single-frame entry points compute it:
 * fm_covariance and fm_subspace_project at the plan's precision `prec`,
 * fm_subspace_sample at FM_FP32,
 * fm_pseudospectrum at the frame's spec_prec. */
fm_status fm_plan_create(fm_ctx *ctx, const fm_frame *frames, int n_frames, fm_prec prec,
                         fm_plan **out);
/* Device bytes a plan for these frames needs (workspace, descriptors and
 * work lists); 0 if a frame is invalid.  Pure host computation. */
size_t fm_plan_bytes(fm_ctx *ctx, const fm_frame *frames, int n_frames, fm_prec prec);

/* As fm_plan_create, but for callers that cannot allocate or synchronise
 * (a serving loop with its own device memory pool): the plan lives in the
 * caller's block dev_mem[0, dev_bytes) (>= fm_plan_bytes, 256-byte aligned),
 * its descriptors and work lists are uploaded with asynchronous copies on
 * `stream`, and nothing is allocated on the device or synchronised.  Run it
 * on the same stream (or after it).  The block must stay valid until the
 * plan's work has completed; fm_plan_destroy on such a plan neither
 * synchronises nor frees device memory. */
fm_status fm_plan_create_in(fm_ctx *ctx, const fm_frame *frames, int n_frames, fm_prec prec,
                            void *dev_mem, size_t dev_bytes, void *stream, fm_plan **out);

/* Destroy a plan.  A plan from fm_plan_create first waits for the device to
 * go idle and frees its memory. */
fm_status fm_plan_destroy(fm_plan *plan);

/* Device bytes the plan allocated for its workspace and work lists. */
size_t fm_plan_workspace_bytes(const fm_plan *plan);

/* Stages of all frames of the plan, each one kernel launch (stage 2 is a
 * fixed sequence of launches), enqueued on `stream`. */
fm_status fm_plan_covariance(fm_plan *plan, void *stream);
fm_status fm_plan_subspace(fm_plan *plan, void *stream);
fm_status fm_plan_pseudospectrum(fm_plan *plan, void *stream);
fm_status fm_plan_peaks(fm_plan *plan, void *stream);

/* All four stages.  With use_graph != 0 the sequence is captured once into a
 * HIP graph (on the first call for a given stream) and replayed afterwards. */
fm_status fm_plan_run(fm_plan *plan, void *stream, int use_graph);

/* ------------------------------------------------------------------------ */
/* tuning: kernel variants per shape bucket                                 */
/* ------------------------------------------------------------------------ */

/* A knob selects one of several kernel variants for a shape bucket.  All
 * variants of a knob compute bit-identical results; only their speed
 * differs with the shapes of the batch.  A context starts with built-in
 * defaults; an autotuner times the variants on the caller's frames and
 * installs its choices with fm_set_knob.  Plans built afterwards, and
 * single-frame calls, use the context's current values (a plan keeps the
 * values it was built with).
 *   FM_KNOB_COV_SCHEDULE   bucket = log2(M) - 7 clamped to [0, 5]
 *                          (M <= 128, 256, 512, 1024, 2048, >= 4096).
 *                          0: all covariance tiles of a frame go to one XCD
 *                          (one L2 holds its snapshots); 1: the frame's tiles
 *                          are dealt one by one to the least-loaded XCD;
 *                          2 (built-in default): 1 for FM_FP32 frames with
 *                          M >= 2048, 0 otherwise.
 *   FM_KNOB_SPEC_ANGLES    bucket = ceil(K/8) - 1 (0..7).  Angles per
 *                          workgroup of the FP32 (polynomial) spectrum pass
 *                          of a group of frames of that bucket: 64, 128, or
 *                          256 (buckets 0..3 only).  A plan (or call) whose
 *                          pass would then have fewer than 256 workgroups
 *                          takes 64 angles per workgroup instead.
 *   FM_KNOB_SPEC16_ANGLES  the same for the compensated FP16 spectrum pass. */
typedef enum {
  FM_KNOB_COV_SCHEDULE = 0,
  FM_KNOB_SPEC_ANGLES = 1,
  FM_KNOB_SPEC16_ANGLES = 2
} fm_knob;

/* FM_E_ARG (with a message) for an unknown knob, bucket or value. */
fm_status fm_set_knob(fm_ctx *ctx, int knob, int bucket, int value);
/* Current value, or -1 for an unknown knob or bucket. */
int fm_get_knob(const fm_ctx *ctx, int knob, int bucket);

#ifdef __cplusplus
}
#endif

#endif /* FASTMUSIC_H */
