// fm_api.hip -- the C ABI of fastmusic.h: argument validation, the context
// arena, single-frame stage sequences and batched plans.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "fm_internal.h"

#define FM_API extern "C" __attribute__((visibility("default")))

using fm::FrameDev;
using fm::Item;

// tuning knobs: kernel variants per shape bucket (every variant computes
// bit-identical results)
constexpr int kKnobs = 3, kBuckets = 8;

struct fm_ctx {
  int device = 0;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  // device address of `scratch` (below) on this context's device, from
  // hipGetSymbolAddress at fm_create: the array's host-side name is not a
  // device address
  char *scratch = nullptr;
  std::string err;
  int knob[kKnobs][kBuckets];
};

// Workspace of fm_subspace_project_noalloc: a fixed device array, one copy
// per GPU the library runs on, held until the process ends.  Every call on a
// GPU shares it (concurrent calls on one GPU race); each call's kernels
// initialise what they read, so nothing needs clearing between calls.
constexpr size_t kScratchBytes = (size_t)16 << 20;
static_assert(kScratchBytes == FM_NOALLOC_SCRATCH_BYTES, "header limit");
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

int knob_buckets(int knob) { return knob == FM_KNOB_COV_SCHEDULE ? 6 : 8; }

bool knob_value_ok(int knob, int bucket, int v) {
  if (knob == FM_KNOB_COV_SCHEDULE) return v == 0 || v == 1 || v == 2;
  // spectrum angle tiles: 64 nnb angles, nnb = 4 only for row-block classes <= 4
  return v == 64 || v == 128 || (v == 256 && bucket < 4);
}

// built-in choices (measured on an MI355X): a wider angle tile reuses each
// generated phasor and staged operand for more angles (in the FP16 pass
// until register pressure from the 2K stacked outputs takes over); the best
// polynomial-pass tile depends on how full the groups are -- at full groups
// of equal frames 64, 128 and 256 angles are within 2%, in a batch of mixed
// K 256 is 5-12% slower than 128 -- which the autotuner measures per batch
int knob_default(int knob, int bucket) {
  if (knob == FM_KNOB_COV_SCHEDULE) return 2;
  if (knob == FM_KNOB_SPEC_ANGLES) return bucket < 6 ? 128 : 64;
  return bucket < 2 ? 256 : (bucket < 6 ? 128 : 64);
}

// bucket of a covariance frame: log2(M) - 7 clamped to [0, 5]
int cov_bucket(int M) {
  int b = 0;
  while (b < 5 && (128 << b) < M) ++b;
  return b;
}

}  // namespace

struct fm_plan {
  fm_ctx *ctx = nullptr;
  fm_prec prec = FM_FP32;
  int n_frames = 0;
  std::vector<FrameDev> frames_h;
  FrameDev *frames_d = nullptr;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  Item *items_d = nullptr;
  size_t items_bytes = 0;
  std::vector<Item> items_h;  // host copy (source of the asynchronous upload)
  bool owned = true;          // device memory allocated by the plan itself
  // a launch = (kind, mode/class, offset into items_d, count)
  struct Launch {
    int kind, mode, n_class;
    size_t off;
    int count;
  };
  std::vector<Launch> cov, sub, spec, peaks;
  // the graph is captured once on a private stream (the null stream cannot
  // be captured) and launched on whichever stream the caller passes
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap_stream = nullptr;
};

namespace {

enum Kind { kCov, kCovSplit, kOmega, kGather, kSketch, kSketch16, kSketchSeg, kSketch16Seg,
             kSketchRed, kSketch16Red, kXhv, kXz, kZx, kXcore, kGram, kSmall, kApply,
             kSpecPrep, kRefine, kPeaks, kOrder, kAcorr, kHsum, kPoly, kEsprit, kSplit16, kSpec16 };

fm_status fail(fm_ctx *ctx, fm_status st, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

fm_status hip_fail(fm_ctx *ctx, hipError_t e, const char *where) {
  return fail(ctx, FM_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// A plan runs the FP32 covariance's T segments on separate waves when its
// one-wave blocks number fewer than this (two per SIMD on 1024 SIMDs)
constexpr long long kCovSplitWaves = 2048;
// ... and their segment sums fit in this much workspace
constexpr size_t kCovSplitBytes = (size_t)64 << 20;
// ... and the Method 2 products' channel segments run on separate workgroups
// when its row-block workgroups number fewer than this (two per CU)
constexpr long long kSketchSplitWGs = 512;
// ... and the lag sums take one lag per lane when their workgroups would
// number fewer than this
constexpr long long kAcorrWideWGs = 512;
// ... and the polynomial pass takes 64-angle tiles, whatever the knob, when
// the knob's tiles would number fewer than the compute units (same results:
// a tile's angles do not depend on its width)
constexpr long long kPolyNarrowWGs = 256;

// per-frame workspace layout (shared by single-frame calls and plans)
struct WsLayout {
  size_t y, v, z, part, small, uf, rlist, eig, spart, total;
  bool has_z, has_spart;
};

int sketch_nb(int n);
// bytes of a frame's Method 2 channel-segment sums (0 without segments)
size_t spart_bytes(int M, int n) {
  const int nb = sketch_nb(n), S = fm::sketch_segments(M, nb);
  if (S <= 1) return 0;
  return (size_t)((M + fm::kSketchRows - 1) / fm::kSketchRows) * S * nb * fm::kSketchPartFloats *
         sizeof(float);
}

// Tz > 0: Method 2 from X, with the [T][n] product X^H V; with_spart: room
// for the channel-segment sums (single-frame calls run their products with
// R one workgroup per segment; plans add it only when they do)
WsLayout ws_layout(int M, int n, int K, int L, int Tz = 0, bool with_spart = true) {
  const int np = (n + 1) & ~1;
  const int nchunk = (M + fm::kGramRows - 1) / fm::kGramRows;
  WsLayout w;
  size_t o = 0;
  w.y = o;     o += align256((size_t)M * n * 8);
  w.v = o;     o += align256((size_t)M * n * 8);
  w.z = o;     o += align256((size_t)Tz * n * 8);
  w.has_z = Tz > 0;
  w.part = o;  o += align256((size_t)nchunk * 2 * n * n * 16);
  w.small = o; o += align256(((size_t)fm::kSmallSlots * np * np + 1) * 16);
  w.uf = o;    o += align256((size_t)M * K * 8);
  w.rlist = o; o += align256((size_t)(L + 1) * 4);
  w.eig = o;   o += align256((size_t)n * 8);
  const size_t sp = with_spart && Tz == 0 ? spart_bytes(M, n) : 0;
  w.has_spart = sp > 0;
  w.spart = o; o += align256(sp);
  w.total = o;
  return w;
}

void bind_ws(FrameDev &f, char *base, const WsLayout &w) {
  f.Y = reinterpret_cast<float2 *>(base + w.y);
  f.V = reinterpret_cast<float2 *>(base + w.v);
  f.Z = w.has_z ? reinterpret_cast<float2 *>(base + w.z) : nullptr;
  f.part = reinterpret_cast<double2 *>(base + w.part);
  f.small = reinterpret_cast<double2 *>(base + w.small);
  f.Uf = reinterpret_cast<float2 *>(base + w.uf);
  f.spart = w.has_spart ? reinterpret_cast<float *>(base + w.spart) : nullptr;
  f.rlist = reinterpret_cast<int *>(base + w.rlist);
  f.eig = reinterpret_cast<double *>(base + w.eig);
  f.nchunk = (f.M + fm::kGramRows - 1) / fm::kGramRows;
  f.npad = (f.n + 1) & ~1;
}

FrameDev blank_frame() {
  FrameDev f;
  std::memset(&f, 0, sizeof f);
  return f;
}

bool prec_ok(fm_prec p) {
  return p == FM_FP32 || p == FM_BF16 || p == FM_FP16 || p == FM_FP16X3 || p == FM_BF16X3;
}

fm_status set_dev(fm_ctx *ctx) {
  hipError_t e = hipSetDevice(ctx->device);
  return e == hipSuccess ? FM_OK : hip_fail(ctx, e, "hipSetDevice");
}

#define FM_CHECK_LAUNCH(ctx, call)                                   \
  do {                                                               \
    hipError_t _e = (call);                                          \
    if (_e != hipSuccess) return hip_fail((ctx), _e, #call);         \
  } while (0)

// ---------------------------------------------------------------------------
// validation shared by single-frame calls and plans
// ---------------------------------------------------------------------------
fm_status check_cov(fm_ctx *c, const void *X, int M, int T, int64_t ldx, const void *R,
                    int64_t ldr) {
  if (!X || !R) return fail(c, FM_E_ARG, "covariance: null pointer");
  if (M < 1 || T < 1) return fail(c, FM_E_ARG, "covariance: need M >= 1 and T >= 1 (M=%d T=%d)", M, T);
  if (ldx < T) return fail(c, FM_E_ARG, "covariance: ldx (%lld) < T (%d)", (long long)ldx, T);
  if (ldr < M) return fail(c, FM_E_ARG, "covariance: ldr (%lld) < M (%d)", (long long)ldr, M);
  return FM_OK;
}

// the 16-bit covariance kernels address rows through 32-bit lane offsets
fm_status check_cov16_ldx(fm_ctx *c, int64_t ldx, fm_prec prec) {
  if (prec != FM_FP32 && ldx > fm::kCov16MaxLdx)
    return fail(c, FM_E_UNSUPPORTED, "covariance: ldx (%lld) > %lld for 16-bit operands",
                (long long)ldx, fm::kCov16MaxLdx);
  return FM_OK;
}

fm_status check_sub(fm_ctx *c, const void *R, int M, int64_t ldr, int method, int n, int q,
                    int K, double rcond, const void *rnd, const void *Us, const void *sigma,
                    const void *status) {
  if (!R || !rnd || !Us || !sigma || !status) return fail(c, FM_E_ARG, "subspace: null pointer");
  if (M < 2) return fail(c, FM_E_ARG, "subspace: need M >= 2 (M=%d)", M);
  if (ldr < M) return fail(c, FM_E_ARG, "subspace: ldr (%lld) < M (%d)", (long long)ldr, M);
  if (K < 1 || K > n || n > M)
    return fail(c, FM_E_ARG, "subspace: need 1 <= K <= n <= M (K=%d n=%d M=%d)", K, n, M);
  if (K > fm::kMaxK) return fail(c, FM_E_UNSUPPORTED, "subspace: K=%d > %d", K, fm::kMaxK);
  if (!(rcond >= 0.0) || !std::isfinite(rcond)) return fail(c, FM_E_ARG, "subspace: bad rcond");
  if (method == FM_METHOD_PROJECT || method == FM_METHOD_PROJECT_X) {
    if (n > fm::kMaxL) return fail(c, FM_E_UNSUPPORTED, "subspace_project: l=%d > %d", n, fm::kMaxL);
    if (q < 0 || q > 16) return fail(c, FM_E_ARG, "subspace_project: need 0 <= q <= 16 (q=%d)", q);
  } else if (method == FM_METHOD_SAMPLE) {
    if (n > fm::kMaxN) return fail(c, FM_E_UNSUPPORTED, "subspace_sample: p=%d > %d", n, fm::kMaxN);
  } else if (method == FM_METHOD_SAMPLE_X) {
    if (n > fm::kMaxL) return fail(c, FM_E_UNSUPPORTED, "subspace_sample_x: p=%d > %d", n, fm::kMaxL);
  } else {
    return fail(c, FM_E_ARG, "subspace: unknown method %d", method);
  }
  return FM_OK;
}

fm_status check_spec(fm_ctx *c, const void *Us, int M, int K, double th0, double dth, int L,
                     const void *P) {
  if (!Us || !P) return fail(c, FM_E_ARG, "pseudospectrum: null pointer");
  if (M < 1 || K < 1 || K > M) return fail(c, FM_E_ARG, "pseudospectrum: need 1 <= K <= M (K=%d M=%d)", K, M);
  if (K > fm::kMaxK) return fail(c, FM_E_UNSUPPORTED, "pseudospectrum: K=%d > %d", K, fm::kMaxK);
  if (L < 1) return fail(c, FM_E_ARG, "pseudospectrum: need L >= 1");
  if (!(dth > 0.0) || !std::isfinite(dth) || !std::isfinite(th0))
    return fail(c, FM_E_ARG, "pseudospectrum: need finite theta0 and dtheta > 0");
  return FM_OK;
}

fm_status check_peaks(fm_ctx *c, const void *P, int L, int K, const void *idx, const void *val,
                      const void *nf) {
  if (!P || !idx || !val || !nf) return fail(c, FM_E_ARG, "peaks: null pointer");
  if (L < 1 || L > (1 << 20)) return fail(c, FM_E_ARG, "peaks: need 1 <= L <= 2^20 (L=%d)", L);
  if (K < 1 || K > fm::kMaxK) return fail(c, FM_E_ARG, "peaks: need 1 <= K <= %d (K=%d)", fm::kMaxK, K);
  return FM_OK;
}

// MFMA row/column block classes (one kernel instantiation per class)
// row-block class of both spectrum passes: ceil(2K / 16) = ceil(K / 8)
int spec_nb(int K) { return (K + 7) / 8; }
int sketch_nb(int n) { return (2 * n + 31) / 32; }

// ---------------------------------------------------------------------------
// single-frame stage-2 sequences (identical kernels to the batched plan)
// ---------------------------------------------------------------------------
hipError_t run_project_single(FrameDev &f, hipStream_t s, fm_prec prec) {
  hipError_t e;
  const int nb = sketch_nb(f.n);
  const bool from_x = f.method == FM_METHOD_PROJECT_X;
  const bool s16 = !from_x && prec != FM_FP32 && fm::sketch16_ok(nb);
  auto sketch = [&](int r) -> hipError_t {
    if (from_x) {
      hipError_t e2 = fm::launch_xhv(f, nullptr, nullptr, 0, nb, s);
      return e2 != hipSuccess ? e2 : fm::launch_xz(f, nullptr, nullptr, 0, nb, r, s);
    }
    // channel segments on separate workgroups, then their in-order sum:
    // the same bits as one workgroup running them in turn
    auto launch = [&](int split) {
      return s16 ? fm::launch_sketch16(f, nullptr, nullptr, 0, nb, r, split, s)
                 : fm::launch_sketch(f, nullptr, nullptr, 0, nb, r, split, s);
    };
    if (fm::sketch_segments(f.M, nb) > 1 && f.spart) {
      const hipError_t e2 = launch(1);
      return e2 != hipSuccess ? e2 : launch(2);
    }
    return launch(0);
  };
  const bool fused = fm::sketch_fuses_gram(nb);
  // orth of the current Y; `after_sketch`: the Gram partials came with it
  auto orth = [&](bool after_sketch) -> hipError_t {
    hipError_t r;
    if (!(fused && after_sketch) &&
        (r = fm::launch_gram(f, nullptr, nullptr, 0, fm::kGramSelf, s)) != hipSuccess)
      return r;
    if ((r = fm::launch_small(f, nullptr, nullptr, 0, fm::kOrth, s)) != hipSuccess) return r;
    return fm::launch_apply(f, nullptr, nullptr, 0, fm::kApplyV, s);
  };
  // (with power iterations the first product reads Omega itself)
  if ((from_x || f.q == 0) && (e = fm::launch_omega(f, nullptr, nullptr, 0, 0, s)) != hipSuccess)
    return e;
  if (f.q == 0 && (e = orth(false)) != hipSuccess) return e;
  for (int r = 0; r <= f.q; ++r) {
    if (r > 0 && (e = orth(true)) != hipSuccess) return e;
    if ((e = sketch(r)) != hipSuccess) return e;
  }
  if (!fused && (e = fm::launch_gram(f, nullptr, nullptr, 0, fm::kGramFinal, s)) != hipSuccess)
    return e;
  if ((e = fm::launch_small(f, nullptr, nullptr, 0, fm::kFinal, s)) != hipSuccess) return e;
  return fm::launch_apply(f, nullptr, nullptr, 0, fm::kApplyUs, s);
}

hipError_t run_sample_single(FrameDev &f, hipStream_t s) {
  hipError_t e;
  if (f.method == FM_METHOD_SAMPLE_X) {
    if ((e = fm::launch_zx(f, nullptr, nullptr, 0, s)) != hipSuccess) return e;
    if ((e = fm::launch_xz(f, nullptr, nullptr, 0, sketch_nb(f.n), -1, s)) != hipSuccess) return e;
    if ((e = fm::launch_xcore(f, nullptr, nullptr, 0, s)) != hipSuccess) return e;
  } else if ((e = fm::launch_gather(f, nullptr, nullptr, 0, s)) != hipSuccess) {
    return e;
  }
  if ((e = fm::launch_gram(f, nullptr, nullptr, 0, fm::kGramFinal, s)) != hipSuccess) return e;
  if ((e = fm::launch_small(f, nullptr, nullptr, 0, fm::kFinal, s)) != hipSuccess) return e;
  return fm::launch_apply(f, nullptr, nullptr, 0, fm::kApplyUs, s);
}


int small_class(int n) {
  if (n <= 16) return 16;
  if (n <= 32) return 32;
  if (n <= fm::kSmallLdsN) return fm::kSmallLdsN;
  return fm::kMaxN;
}

}  // namespace

// ===========================================================================
// context
// ===========================================================================

FM_API const char *fm_status_string(fm_status s) {
  switch (s) {
    case FM_OK: return "ok";
    case FM_E_ARG: return "invalid argument";
    case FM_E_HIP: return "HIP runtime error";
    case FM_E_WORKSPACE: return "workspace too small";
    case FM_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

FM_API const char *fm_last_error(const fm_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

FM_API size_t fm_workspace_bytes(int M, int n, int K, int L) {
  if (M < 1 || n < 1 || K < 0 || L < 0) return 0;
  return ws_layout(M, n, K, L).total;
}

FM_API fm_status fm_create(int device, size_t workspace_bytes, fm_ctx **out) {
  if (!out) return FM_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FM_E_ARG;
  fm_ctx *c = new (std::nothrow) fm_ctx;
  if (!c) return FM_E_WORKSPACE;
  c->device = device;
  for (int k = 0; k < kKnobs; ++k)
    for (int b = 0; b < kBuckets; ++b) c->knob[k][b] = knob_default(k, b);
  c->arena_bytes = workspace_bytes ? workspace_bytes : (size_t)64 << 20;
  if (hipSetDevice(device) != hipSuccess ||
      hipMalloc((void **)&c->arena, c->arena_bytes) != hipSuccess) {
    delete c;
    return FM_E_HIP;
  }
  // with the context's device current: this device's copy of `scratch`
  if (hipGetSymbolAddress((void **)&c->scratch, HIP_SYMBOL(scratch)) != hipSuccess ||
      !c->scratch) {
    hipFree(c->arena);
    delete c;
    return FM_E_HIP;
  }
  *out = c;
  return FM_OK;
}

FM_API fm_status fm_destroy(fm_ctx *ctx) {
  if (!ctx) return FM_E_ARG;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  if (ctx->arena) hipFree(ctx->arena);
  delete ctx;
  return FM_OK;
}

// ===========================================================================
// single-frame stages
// ===========================================================================

FM_API fm_status fm_set_knob(fm_ctx *ctx, int knob, int bucket, int value) {
  if (!ctx) return FM_E_ARG;
  if (knob < 0 || knob >= kKnobs) return fail(ctx, FM_E_ARG, "set_knob: unknown knob %d", knob);
  if (bucket < 0 || bucket >= knob_buckets(knob))
    return fail(ctx, FM_E_ARG, "set_knob: knob %d has no bucket %d", knob, bucket);
  if (!knob_value_ok(knob, bucket, value))
    return fail(ctx, FM_E_ARG, "set_knob: value %d not valid for knob %d bucket %d", value, knob,
                bucket);
  ctx->knob[knob][bucket] = value;
  return FM_OK;
}

FM_API int fm_get_knob(const fm_ctx *ctx, int knob, int bucket) {
  if (!ctx || knob < 0 || knob >= kKnobs || bucket < 0 || bucket >= knob_buckets(knob)) return -1;
  return ctx->knob[knob][bucket];
}

FM_API fm_status fm_covariance(fm_ctx *ctx, void *stream, const void *X, int M, int T,
                               int64_t ldx, void *R, int64_t ldr, fm_prec prec) {
  if (!ctx) return FM_E_ARG;
  fm_status st = check_cov(ctx, X, M, T, ldx, R, ldr);
  if (st != FM_OK) return st;
  if (!prec_ok(prec)) return fail(ctx, FM_E_ARG, "covariance: bad precision %d", (int)prec);
  if ((st = check_cov16_ldx(ctx, ldx, prec)) != FM_OK) return st;
  if ((st = set_dev(ctx)) != FM_OK) return st;
  FrameDev f = blank_frame();
  f.X = static_cast<const float2 *>(X);
  f.ldx = ldx;
  f.M = M;
  f.T = T;
  f.R = static_cast<float2 *>(R);
  f.ldr = ldr;
  // FP32 with several T segments: one wave per segment and an in-order
  // reduction when the context's arena holds the segment sums (the same
  // bits as one wave running the segments in turn, four times the waves)
  const size_t part_bytes = (size_t)fm::cov_units(M, FM_FP32) * fm::cov_segments(M, T) *
                            fm::kCovPartFloats * sizeof(float);
  if (prec == FM_FP32 && fm::cov_segments(M, T) > 1 && part_bytes <= ctx->arena_bytes) {
    f.cpart = reinterpret_cast<float *>(ctx->arena);
    FM_CHECK_LAUNCH(ctx, fm::launch_covariance_split(f, nullptr, nullptr, 0, 0, (hipStream_t)stream));
    FM_CHECK_LAUNCH(ctx, fm::launch_covariance_split(f, nullptr, nullptr, 0, 1, (hipStream_t)stream));
    return FM_OK;
  }
  FM_CHECK_LAUNCH(ctx, fm::launch_covariance(f, nullptr, nullptr, 0, prec, (hipStream_t)stream));
  return FM_OK;
}

// `noalloc`: the workspace is this device's `scratch` array instead of the
// context's arena
static fm_status subspace_single(fm_ctx *ctx, void *stream, const void *R, int M, int64_t ldr,
                                 int method, const void *rnd, int n, int q, int K, double rcond,
                                 fm_prec prec, void *Us, double *sigma, uint32_t *status,
                                 bool noalloc = false) {
  if (!ctx) return FM_E_ARG;
  fm_status st = check_sub(ctx, R, M, ldr, method, n, q, K, rcond, rnd, Us, sigma, status);
  if (st != FM_OK) return st;
  if (!prec_ok(prec)) return fail(ctx, FM_E_ARG, "subspace: bad precision %d", (int)prec);

  const WsLayout w = ws_layout(M, n, K, 0);
  char *const ws = noalloc ? ctx->scratch : ctx->arena;
  const size_t ws_bytes = noalloc ? kScratchBytes : ctx->arena_bytes;
  if (w.total > ws_bytes)
    return fail(ctx, FM_E_WORKSPACE, "subspace: needs %zu %s bytes, have %zu", w.total,
                noalloc ? "scratch" : "arena", ws_bytes);
  if ((st = set_dev(ctx)) != FM_OK) return st;
  FrameDev f = blank_frame();
  f.R = static_cast<float2 *>(const_cast<void *>(R));
  f.ldr = ldr;
  f.M = M;
  f.K = K;
  f.method = method;
  f.n = n;
  f.q = q;
  f.rcond = rcond;
  if (method == FM_METHOD_PROJECT) f.Omega = static_cast<const float *>(rnd);
  else f.idx = static_cast<const int *>(rnd);
  f.Us = static_cast<double2 *>(Us);
  f.sigma = sigma;
  f.status = status;
  bind_ws(f, ws, w);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = method == FM_METHOD_PROJECT ? run_project_single(f, s, prec)
                                             : run_sample_single(f, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "subspace launch");
  return FM_OK;
}

FM_API fm_status fm_subspace_sample_x(fm_ctx *ctx, void *stream, const void *X, int M, int T,
                                      int64_t ldx, const int32_t *idx, int p, int K, double rcond,
                                      void *Us, double *sigma, uint32_t *status) {
  if (!ctx) return FM_E_ARG;
  if (!X) return fail(ctx, FM_E_ARG, "subspace_sample_x: null X");
  if (T < 1 || ldx < T)
    return fail(ctx, FM_E_ARG, "subspace_sample_x: need T >= 1 and ldx >= T (T=%d ldx=%lld)", T,
                (long long)ldx);
  fm_status st = check_sub(ctx, X, M, M, FM_METHOD_SAMPLE_X, p, 0, K, rcond, idx, Us, sigma,
                           status);
  if (st != FM_OK) return st;
  const WsLayout w = ws_layout(M, p, K, 0, T);
  if (w.total > ctx->arena_bytes)
    return fail(ctx, FM_E_WORKSPACE, "subspace_sample_x: needs %zu arena bytes, have %zu",
                w.total, ctx->arena_bytes);
  if ((st = set_dev(ctx)) != FM_OK) return st;
  FrameDev f = blank_frame();
  f.X = static_cast<const float2 *>(X);
  f.ldx = ldx;
  f.M = M;
  f.T = T;
  f.K = K;
  f.method = FM_METHOD_SAMPLE_X;
  f.n = p;
  f.q = 0;
  f.rcond = rcond;
  f.idx = idx;
  f.Us = static_cast<double2 *>(Us);
  f.sigma = sigma;
  f.status = status;
  bind_ws(f, ctx->arena, w);
  hipError_t e = run_sample_single(f, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "subspace_sample_x launch");
  return FM_OK;
}

FM_API fm_status fm_subspace_project_x(fm_ctx *ctx, void *stream, const void *X, int M, int T,
                                       int64_t ldx, const float *Omega, int l, int q, int K,
                                       double rcond, fm_prec prec, void *Us, double *sigma,
                                       uint32_t *status) {
  if (!ctx) return FM_E_ARG;
  if (!X) return fail(ctx, FM_E_ARG, "subspace_project_x: null X");
  if (T < 1 || ldx < T)
    return fail(ctx, FM_E_ARG, "subspace_project_x: need T >= 1 and ldx >= T (T=%d ldx=%lld)", T,
                (long long)ldx);
  fm_status st = check_sub(ctx, X, M, M, FM_METHOD_PROJECT_X, l, q, K, rcond, Omega, Us, sigma,
                           status);
  if (st != FM_OK) return st;
  if (!prec_ok(prec)) return fail(ctx, FM_E_ARG, "subspace_project_x: bad precision %d", (int)prec);
  if (prec != FM_FP32)
    return fail(ctx, FM_E_UNSUPPORTED, "subspace_project_x: FM_FP32 products only");
  const WsLayout w = ws_layout(M, l, K, 0, T);
  if (w.total > ctx->arena_bytes)
    return fail(ctx, FM_E_WORKSPACE, "subspace_project_x: needs %zu arena bytes, have %zu",
                w.total, ctx->arena_bytes);
  if ((st = set_dev(ctx)) != FM_OK) return st;
  FrameDev f = blank_frame();
  f.X = static_cast<const float2 *>(X);
  f.ldx = ldx;
  f.M = M;
  f.T = T;
  f.K = K;
  f.method = FM_METHOD_PROJECT_X;
  f.n = l;
  f.q = q;
  f.rcond = rcond;
  f.Omega = Omega;
  f.Us = static_cast<double2 *>(Us);
  f.sigma = sigma;
  f.status = status;
  bind_ws(f, ctx->arena, w);
  hipError_t e = run_project_single(f, (hipStream_t)stream, prec);
  if (e != hipSuccess) return hip_fail(ctx, e, "subspace_project_x launch");
  return FM_OK;
}

FM_API fm_status fm_subspace_sample(fm_ctx *ctx, void *stream, const void *R, int M,
                                    int64_t ldr, const int32_t *idx, int p, int K, double rcond,
                                    void *Us, double *sigma, uint32_t *status) {
  return subspace_single(ctx, stream, R, M, ldr, FM_METHOD_SAMPLE, idx, p, 0, K, rcond, FM_FP32,
                         Us, sigma, status);
}

FM_API fm_status fm_subspace_project(fm_ctx *ctx, void *stream, const void *R, int M,
                                     int64_t ldr, const float *Omega, int l, int q, int K,
                                     double rcond, fm_prec prec, void *Us, double *sigma,
                                     uint32_t *status) {
  return subspace_single(ctx, stream, R, M, ldr, FM_METHOD_PROJECT, Omega, l, q, K, rcond, prec,
                         Us, sigma, status);
}

FM_API fm_status fm_subspace_project_noalloc(fm_ctx *ctx, void *stream, const void *R, int M,
                                             int64_t ldr, const float *Omega, int l, int q, int K,
                                             double rcond, fm_prec prec, void *Us,
                                             double *sigma, uint32_t *status) {
  return subspace_single(ctx, stream, R, M, ldr, FM_METHOD_PROJECT, Omega, l, q, K, rcond, prec,
                         Us, sigma, status, true);
}

FM_API fm_status fm_order(fm_ctx *ctx, void *stream, const void *R, int M, int64_t ldr, int T,
                          const double *eig, int n, double rcond, int rule, int32_t *K_hat,
                          double *crit, uint32_t *status) {
  if (!ctx) return FM_E_ARG;
  if (!R || !eig || !K_hat || !status) return fail(ctx, FM_E_ARG, "order: null pointer");
  if (M < 2 || T < 1) return fail(ctx, FM_E_ARG, "order: need M >= 2 and T >= 1 (M=%d T=%d)", M, T);
  if (ldr < M) return fail(ctx, FM_E_ARG, "order: ldr (%lld) < M (%d)", (long long)ldr, M);
  if (n < 1 || n > M || n > fm::kMaxN)
    return fail(ctx, FM_E_ARG, "order: need 1 <= n <= min(M, %d) (n=%d M=%d)", fm::kMaxN, n, M);
  if (rule != FM_ORDER_AIC && rule != FM_ORDER_MDL)
    return fail(ctx, FM_E_ARG, "order: unknown rule %d", rule);
  if (!(rcond >= 0.0) || !std::isfinite(rcond)) return fail(ctx, FM_E_ARG, "order: bad rcond");
  fm_status st = set_dev(ctx);
  if (st != FM_OK) return st;
  FrameDev f = blank_frame();
  f.R = static_cast<float2 *>(const_cast<void *>(R));
  f.ldr = ldr;
  f.M = M;
  f.T = T;
  f.n = n;
  f.rcond = rcond;
  f.eig = const_cast<double *>(eig);
  f.K_hat = K_hat;
  f.order_crit = crit;
  f.order_rule = rule;
  f.or_status = 0;
  f.status = status;
  FM_CHECK_LAUNCH(ctx, fm::launch_order(f, nullptr, nullptr, 0, (hipStream_t)stream));
  return FM_OK;
}

FM_API fm_status fm_esprit(fm_ctx *ctx, void *stream, const void *Us, int M, int K,
                           double *doa_deg, uint32_t *status) {
  if (!ctx) return FM_E_ARG;
  if (!Us || !doa_deg || !status) return fail(ctx, FM_E_ARG, "esprit: null pointer");
  if (M < 2 || K < 1 || K >= M)
    return fail(ctx, FM_E_ARG, "esprit: need 1 <= K < M (K=%d M=%d)", K, M);
  if (K > fm::kEspritMaxK) return fail(ctx, FM_E_UNSUPPORTED, "esprit: K=%d > %d", K, fm::kEspritMaxK);
  fm_status st = set_dev(ctx);
  if (st != FM_OK) return st;
  FrameDev f = blank_frame();
  f.M = M;
  f.K = K;
  f.Us = static_cast<double2 *>(const_cast<void *>(Us));
  f.doa = doa_deg;
  f.status = status;
  f.or_status = 0;
  FM_CHECK_LAUNCH(ctx, fm::launch_esprit(f, nullptr, nullptr, 0, (hipStream_t)stream));
  return FM_OK;
}

FM_API fm_status fm_pseudospectrum(fm_ctx *ctx, void *stream, const void *Us, int M, int K,
                                   double theta0_deg, double dtheta_deg, int L, fm_prec prec,
                                   float *P) {
  if (!ctx) return FM_E_ARG;
  fm_status st = check_spec(ctx, Us, M, K, theta0_deg, dtheta_deg, L, P);
  if (st != FM_OK) return st;
  if (!prec_ok(prec)) return fail(ctx, FM_E_ARG, "pseudospectrum: bad precision %d", (int)prec);
  if (prec == FM_BF16 || prec == FM_BF16X3)
    return fail(ctx, FM_E_UNSUPPORTED,
                "pseudospectrum: FM_FP32 or FM_FP16 / FM_FP16X3 (compensated) only");
  const size_t uf_bytes = align256((size_t)M * K * 8);
  const size_t rl_bytes = align256((size_t)(L + 1) * 4);
  const size_t need = uf_bytes + rl_bytes +
                      (prec == FM_FP32
                           ? align256((size_t)fm::acorr_blocks(M) * M * fm::kPolyRows * 8)
                           : 0);
  if (need > ctx->arena_bytes)
    return fail(ctx, FM_E_WORKSPACE, "pseudospectrum: needs %zu arena bytes", need);
  if ((st = set_dev(ctx)) != FM_OK) return st;
  FrameDev f = blank_frame();
  f.M = M;
  f.K = K;
  f.Us = static_cast<double2 *>(const_cast<void *>(Us));
  f.Uf = reinterpret_cast<float2 *>(ctx->arena);
  f.rlist = reinterpret_cast<int *>(ctx->arena + uf_bytes);
  f.L = L;
  f.theta0 = theta0_deg;
  f.dtheta = dtheta_deg;
  f.P = P;
  hipStream_t s = (hipStream_t)stream;
  const int nb = spec_nb(K);
  if (prec == FM_FP32) {
    // a group of one: lag sums, then the polynomial pass
    int nnb = ctx->knob[FM_KNOB_SPEC_ANGLES][nb - 1] / 64;
    if ((L + 64 * nnb - 1) / (64 * nnb) < kPolyNarrowWGs) nnb = 1;
    f.hgrp = reinterpret_cast<float2 *>(ctx->arena + uf_bytes + rl_bytes);
    f.hslot = 0;
    f.hcount = 1;
    FM_CHECK_LAUNCH(ctx, fm::launch_uf(f, s));
    FM_CHECK_LAUNCH(ctx, fm::launch_acorr(f, nullptr, nullptr, 0, 1, s));
    if (fm::acorr_blocks(M) > 1) FM_CHECK_LAUNCH(ctx, fm::launch_hsum(f, nullptr, nullptr, 0, s));
    FM_CHECK_LAUNCH(ctx, fm::launch_poly(f, nullptr, nullptr, 0, nnb, s));
  } else {
    const int nnb = ctx->knob[FM_KNOB_SPEC16_ANGLES][nb - 1] / 64;
    FM_CHECK_LAUNCH(ctx, fm::launch_split(f, nullptr, nullptr, 0, s));
    FM_CHECK_LAUNCH(ctx, fm::launch_spectrum16(f, nullptr, nullptr, 0, nb, nnb, s));
  }
  FM_CHECK_LAUNCH(ctx, fm::launch_refine(f, nullptr, nullptr, 0, s));
  return FM_OK;
}

FM_API fm_status fm_peaks(fm_ctx *ctx, void *stream, const float *P, int L, int K, int32_t *idx,
                          float *val, int32_t *n_found) {
  if (!ctx) return FM_E_ARG;
  fm_status st = check_peaks(ctx, P, L, K, idx, val, n_found);
  if (st != FM_OK) return st;
  if ((st = set_dev(ctx)) != FM_OK) return st;
  FrameDev f = blank_frame();
  f.P = const_cast<float *>(P);
  f.L = L;
  f.K = K;
  f.peak_idx = idx;
  f.peak_val = val;
  f.n_found = n_found;
  FM_CHECK_LAUNCH(ctx, fm::launch_peaks(f, nullptr, nullptr, 0, (hipStream_t)stream));
  return FM_OK;
}

// ===========================================================================
// plans
// ===========================================================================

namespace {

hipError_t run_launch(fm_plan *p, const fm_plan::Launch &L, hipStream_t s) {
  if (L.count <= 0) return hipSuccess;
  const Item *it = p->items_d + L.off;
  FrameDev cls = blank_frame();
  cls.n = L.n_class;
  const FrameDev *fr = p->frames_d;
  switch (L.kind) {
    case kCov: return fm::launch_covariance(cls, fr, it, L.count, p->prec, s);
    case kCovSplit: return fm::launch_covariance_split(cls, fr, it, L.count, L.mode, s);
    case kOmega: return fm::launch_omega(cls, fr, it, L.count, 0, s);
    case kGather: return fm::launch_gather(cls, fr, it, L.count, s);
    case kSketch: return fm::launch_sketch(cls, fr, it, L.count, L.n_class, L.mode, 0, s);
    case kSketch16: return fm::launch_sketch16(cls, fr, it, L.count, L.n_class, L.mode, 0, s);
    case kSketchSeg: return fm::launch_sketch(cls, fr, it, L.count, L.n_class, L.mode, 1, s);
    case kSketch16Seg: return fm::launch_sketch16(cls, fr, it, L.count, L.n_class, L.mode, 1, s);
    case kSketchRed: return fm::launch_sketch(cls, fr, it, L.count, L.n_class, L.mode, 2, s);
    case kSketch16Red: return fm::launch_sketch16(cls, fr, it, L.count, L.n_class, L.mode, 2, s);
    case kXhv: return fm::launch_xhv(cls, fr, it, L.count, L.n_class, s);
    case kXz: return fm::launch_xz(cls, fr, it, L.count, L.n_class, L.mode, s);
    case kZx: return fm::launch_zx(cls, fr, it, L.count, s);
    case kXcore: return fm::launch_xcore(cls, fr, it, L.count, s);
    case kGram: return fm::launch_gram(cls, fr, it, L.count, L.mode, s);
    case kSmall: return fm::launch_small(cls, fr, it, L.count, L.mode, s);
    case kApply: return fm::launch_apply(cls, fr, it, L.count, L.mode, s);
    case kSpecPrep: return fm::launch_spec_prep(fr, it, L.count, s);
    case kRefine: return fm::launch_refine(cls, fr, it, L.count, s);
    case kPeaks: return fm::launch_peaks(cls, fr, it, L.count, s);
    case kOrder: return fm::launch_order(cls, fr, it, L.count, s);
    case kAcorr: return fm::launch_acorr(cls, fr, it, L.count, L.mode, s);
    case kHsum: return fm::launch_hsum(cls, fr, it, L.count, s);
    case kPoly: return fm::launch_poly(cls, fr, it, L.count, L.mode, s);
    case kEsprit: return fm::launch_esprit(cls, fr, it, L.count, s);
    case kSplit16: return fm::launch_split(cls, fr, it, L.count, s);
    case kSpec16: return fm::launch_spectrum16(cls, fr, it, L.count, L.n_class, L.mode, s);
  }
  return hipErrorInvalidValue;
}

fm_status run_list(fm_plan *p, const std::vector<fm_plan::Launch> &v, void *stream) {
  for (const auto &L : v) {
    hipError_t e = run_launch(p, L, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "plan launch");
  }
  return FM_OK;
}

}  // namespace

// Builds a plan.  dev == nullptr: the plan allocates its device memory and
// uploads synchronously.  Otherwise everything lives in the caller's block
// [dev, dev + dev_bytes) and the upload is enqueued on `stream`; with
// dry_run only *need is computed.
static fm_status plan_build(fm_ctx *ctx, const fm_frame *frames, int n_frames, fm_prec prec,
                            char *dev, size_t dev_bytes, hipStream_t stream, bool dry_run,
                            size_t *need, fm_plan **out) {
  if (!ctx || (!out && !dry_run)) return FM_E_ARG;
  if (out) *out = nullptr;
  if (!frames || n_frames < 1) return fail(ctx, FM_E_ARG, "plan: need at least one frame");
  if (!prec_ok(prec)) return fail(ctx, FM_E_ARG, "plan: bad precision %d", (int)prec);
  for (int i = 0; i < n_frames; ++i) {
    const fm_frame &a = frames[i];
    // Method 2 from X forms no R: its R may be null
    const bool from_x = a.method == FM_METHOD_PROJECT_X || a.method == FM_METHOD_SAMPLE_X;
    fm_status st = check_cov(ctx, a.X, a.M, a.T, a.ldx, from_x ? a.X : a.R,
                             from_x ? a.M : a.ldr);
    if (st == FM_OK && !from_x) st = check_cov16_ldx(ctx, a.ldx, prec);
    if (st == FM_OK)
      st = check_sub(ctx, from_x ? a.X : a.R, a.M, from_x ? a.M : a.ldr, a.method, a.n, a.q,
                     a.K, a.rcond,
                     (a.method == FM_METHOD_PROJECT || a.method == FM_METHOD_PROJECT_X)
                         ? (const void *)a.Omega : (const void *)a.idx,
                     a.Us, a.sigma, a.status);
    if (st == FM_OK) st = check_spec(ctx, a.Us, a.M, a.K, a.theta0_deg, a.dtheta_deg, a.L, a.P);
    if (st == FM_OK) st = check_peaks(ctx, a.P, a.L, a.K, a.peak_idx, a.peak_val, a.n_found);
    if (st == FM_OK && a.spec_prec != FM_FP32 && a.spec_prec != FM_FP16 &&
        a.spec_prec != FM_FP16X3)
      st = fail(ctx, a.spec_prec == FM_BF16 || a.spec_prec == FM_BF16X3 ? FM_E_UNSUPPORTED
                                                                        : FM_E_ARG,
                "plan: frame %d spectrum precision %d (FM_FP32 or FM_FP16 only)", i,
                a.spec_prec);
    if (st == FM_OK && a.esprit_deg && a.K > fm::kEspritMaxK)
      st = fail(ctx, FM_E_UNSUPPORTED, "ESPRIT: K=%d > %d", a.K, fm::kEspritMaxK);
    if (st == FM_OK && a.K_hat) {
      if (from_x)
        st = fail(ctx, FM_E_ARG, "model order: needs R (Method 1 or 2 on R, method %d)",
                  a.method);
      else if (a.order_rule != FM_ORDER_AIC && a.order_rule != FM_ORDER_MDL)
        st = fail(ctx, FM_E_ARG, "model order: unknown rule %d", a.order_rule);
    }
    if (st != FM_OK) {
      std::string m = ctx->err;
      return fail(ctx, st, "plan frame %d: %s", i, m.c_str());
    }
  }
  fm_status st = dry_run ? FM_OK : set_dev(ctx);
  if (st != FM_OK) return st;
  fm_plan *p = new (std::nothrow) fm_plan;
  if (!p) return fail(ctx, FM_E_WORKSPACE, "plan: out of host memory");
  p->ctx = ctx;
  p->prec = prec;
  p->n_frames = n_frames;
  p->owned = dev == nullptr;

  // workspace: frames packed back to back
  std::vector<WsLayout> lay(n_frames);
  std::vector<size_t> off(n_frames);
  size_t total = 0;
  for (int i = 0; i < n_frames; ++i) {
    const bool fx = frames[i].method == FM_METHOD_PROJECT_X ||
                    frames[i].method == FM_METHOD_SAMPLE_X;
    lay[i] = ws_layout(frames[i].M, frames[i].n, frames[i].K, frames[i].L,
                       fx ? frames[i].T : 0, false);
    off[i] = total;
    total += lay[i].total;
  }
  // spectrum groups of the frames on the FP32 polynomial pass: frames with equal M, angle grid and spectrum knob
  // bucket, up to kPolyRows per group (in frame order), each with a group
  // buffer [M][kPolyRows] placed after the frames' workspaces
  std::vector<int> grp_of(n_frames, -1), slot_of(n_frames, 0);
  std::vector<std::vector<int>> groups;
  std::vector<size_t> goff;
  {
    std::map<std::tuple<int, int, uint64_t, uint64_t, int>, int> open;
    for (int i = 0; i < n_frames; ++i) {
      if (frames[i].spec_prec != FM_FP32) continue;  // the FP16 projection pass needs no group
      uint64_t t0, dt;
      std::memcpy(&t0, &frames[i].theta0_deg, 8);
      std::memcpy(&dt, &frames[i].dtheta_deg, 8);
      const auto key = std::make_tuple(frames[i].M, frames[i].L, t0, dt, spec_nb(frames[i].K));
      auto it = open.find(key);
      if (it == open.end() || (int)groups[it->second].size() == fm::kPolyRows) {
        groups.emplace_back();
        open[key] = (int)groups.size() - 1;
      }
      const int g = open[key];
      slot_of[i] = (int)groups[g].size();
      grp_of[i] = g;
      groups[g].push_back(i);
    }
    for (const auto &g : groups) {
      goff.push_back(total);
      const int Mg = frames[g[0]].M;
      total += align256((size_t)fm::acorr_blocks(Mg) * Mg * fm::kPolyRows * 8);
    }
  }
  // FP32 covariance with its T segments on separate waves when the plan's
  // one-wave blocks would not fill the GPU (same bits as the sequential
  // segments); the segment sums follow the other workspaces
  auto forms_r = [&](int i) {
    return frames[i].method != FM_METHOD_PROJECT_X && frames[i].method != FM_METHOD_SAMPLE_X;
  };
  bool cov_split = false;
  std::vector<size_t> coff(n_frames, 0);
  if (prec == FM_FP32) {
    long long waves = 0;
    bool segs = false;
    for (int i = 0; i < n_frames; ++i)
      if (forms_r(i)) {
        waves += fm::cov_units(frames[i].M, FM_FP32);
        segs |= fm::cov_segments(frames[i].M, frames[i].T) > 1;
      }
    size_t cbytes = 0;
    for (int i = 0; i < n_frames; ++i)
      if (forms_r(i)) {
        coff[i] = total + cbytes;
        cbytes += align256((size_t)fm::cov_units(frames[i].M, FM_FP32) *
                           fm::cov_segments(frames[i].M, frames[i].T) * fm::kCovPartFloats * sizeof(float));
      }
    cov_split = segs && waves < kCovSplitWaves && cbytes <= kCovSplitBytes;
    if (cov_split) total += cbytes;
  }
  // Method 2 products with R, channel segments on separate workgroups when
  // the plan's row-block workgroups are few (same bits as in turn)
  auto seg_r = [&](int i) {
    return frames[i].method == FM_METHOD_PROJECT &&
           fm::sketch_segments(frames[i].M, sketch_nb(frames[i].n)) > 1;
  };
  bool sk_split = false;
  std::vector<size_t> soff(n_frames, 0);
  {
    long long wgs = 0;
    size_t sbytes = 0;
    bool any = false;
    for (int i = 0; i < n_frames; ++i)
      if (frames[i].method == FM_METHOD_PROJECT) {
        wgs += (frames[i].M + fm::kSketchRows - 1) / fm::kSketchRows;
        if (seg_r(i)) {
          any = true;
          soff[i] = total + sbytes;
          sbytes += align256(spart_bytes(frames[i].M, frames[i].n));
        }
      }
    sk_split = any && wgs < kSketchSplitWGs && sbytes <= kCovSplitBytes;
    if (sk_split) total += sbytes;
  }
  p->ws_bytes = total;
  hipError_t e = hipSuccess;
  if (dry_run) {
    p->ws = nullptr;
  } else if (p->owned) {
    e = hipMalloc((void **)&p->ws, std::max<size_t>(total, 256));
    if (e != hipSuccess) {
      delete p;
      return hip_fail(ctx, e, "plan workspace hipMalloc");
    }
  } else {
    p->ws = dev;  // descriptors and work lists follow the workspace
  }
  p->frames_h.resize(n_frames);
  for (int i = 0; i < n_frames; ++i) {
    const fm_frame &a = frames[i];
    FrameDev f = blank_frame();
    f.X = static_cast<const float2 *>(a.X);
    f.ldx = a.ldx;
    f.M = a.M;
    f.T = a.T;
    f.R = static_cast<float2 *>(a.R);
    f.ldr = a.ldr;
    f.K = a.K;
    f.method = a.method;
    f.n = a.n;
    f.q = a.q;
    f.rcond = a.rcond;
    f.Omega = a.Omega;
    f.idx = a.idx;
    f.Us = static_cast<double2 *>(a.Us);
    f.sigma = a.sigma;
    f.status = a.status;
    f.L = a.L;
    f.theta0 = a.theta0_deg;
    f.dtheta = a.dtheta_deg;
    f.P = a.P;
    f.peak_idx = a.peak_idx;
    f.peak_val = a.peak_val;
    f.n_found = a.n_found;
    f.K_hat = a.K_hat;
    f.order_crit = a.order_crit;
    f.order_rule = a.order_rule;
    f.doa = a.esprit_deg;
    f.or_status = 1;
    bind_ws(f, p->ws + off[i], lay[i]);
    if (cov_split && forms_r(i)) f.cpart = reinterpret_cast<float *>(p->ws + coff[i]);
    if (sk_split && seg_r(i)) f.spart = reinterpret_cast<float *>(p->ws + soff[i]);
    if (grp_of[i] >= 0) {
      f.hgrp = reinterpret_cast<float2 *>(p->ws + goff[grp_of[i]]);
      f.hslot = slot_of[i];
      f.hcount = (int)groups[grp_of[i]].size();
    }
    p->frames_h[i] = f;
  }

  // ---- work lists -------------------------------------------------------
  std::vector<Item> items;
  auto begin = [&]() { return items.size(); };
  auto add = [&](std::vector<fm_plan::Launch> &v, int kind, int mode, int cls, size_t b) {
    if (items.size() > b) v.push_back({kind, mode, cls, b, (int)(items.size() - b)});
  };
  // longest frames first (by covariance work), so short frames fill the tail
  std::vector<int> order(n_frames);
  for (int i = 0; i < n_frames; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double wa = (double)frames[a].M * frames[a].M * frames[a].T;
    const double wb = (double)frames[b].M * frames[b].M * frames[b].T;
    return wa > wb;
  });
  auto rows = [](int M, int r) { return (M + r - 1) / r; };

  // Covariance tiles, XCD-aware: workgroup w of a launch is dispatched to XCD
  // w mod 8, each XCD with its own L2.  Frames are dealt to the 8 XCDs
  // (largest first onto the least loaded) and position w of the list takes
  // the next tile of XCD (w mod 8)'s frames, so all tiles of a frame share
  // one L2 and each window of its snapshots is fetched once per XCD.  With
  // the schedule knob at 1 for a frame's M bucket, its tiles are dealt one
  // by one instead (a frame whose snapshots overflow one L2 gains nothing
  // from grouping and loses balance).
  size_t b0 = begin();
  {
    constexpr int kXcd = 8;
    std::vector<std::vector<Item>> q(kXcd);
    std::vector<double> load(kXcd, 0.0);
    for (int i : order) {
      if (frames[i].method == FM_METHOD_PROJECT_X || frames[i].method == FM_METHOD_SAMPLE_X)
        continue;  // forms no R
      // schedule 2 (built-in): the FP32 kernel's one-wave blocks are dealt
      // for M >= 2048 (measured 7-14% faster there), grouped below; the
      // 16-bit kernel's four-wave tiles are grouped at every M
      const int cb = cov_bucket(frames[i].M);
      int sched = ctx->knob[FM_KNOB_COV_SCHEDULE][cb];
      if (sched == 2) sched = (prec == FM_FP32 && cb >= 4) ? 1 : 0;
      // split: each FP32 block once per T segment (Item::c = segment), XCD
      // (8 g + (unit mod 8)) / G, so that an XCD's L2 holds the snapshot
      // windows of one or two segments instead of the whole frame
      const int G = cov_split ? fm::cov_segments(frames[i].M, frames[i].T) : 1;
      if (cov_split) {
        int u = 0;
        fm::cov_each_unit(frames[i].M, prec, [&](int a, int b, int) {
          for (int g = 0; g < G; ++g) {
            const int x = (kXcd * g + u % kXcd) / G;
            load[x] += (double)frames[i].T / G;
            q[x].push_back({i, a, b, g});
          }
          ++u;
        });
      } else if (sched == 0) {
        // the whole frame onto the least-loaded XCD
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        fm::cov_each_unit(frames[i].M, prec, [&](int a, int b, int kind) {
          for (int g = 0; g < G; ++g) {
            load[x] += (double)frames[i].T / G;
            q[x].push_back({i, a, b, cov_split ? g : kind});
          }
        });
      } else {
        // each unit onto the least-loaded XCD
        fm::cov_each_unit(frames[i].M, prec, [&](int a, int b, int kind) {
          for (int g = 0; g < G; ++g) {
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[x] += (double)frames[i].T / G;
            q[x].push_back({i, a, b, cov_split ? g : kind});
          }
        });
      }
    }
    std::vector<size_t> pos(kXcd, 0);
    size_t left = 0;
    for (auto &v : q) left += v.size();
    while (left > 0) {
      for (int x = 0; x < kXcd && left > 0; ++x) {
        int y = x;
        if (pos[y] >= q[y].size()) {  // this XCD's frames are done: take from the fullest
          size_t best = 0;
          for (int z = 0; z < kXcd; ++z)
            if (q[z].size() - pos[z] > best) { best = q[z].size() - pos[z]; y = z; }
          // steal from the back so y's next items keep their positions
          items.push_back(q[y].back());
          q[y].pop_back();
        } else {
          items.push_back(q[y][pos[y]++]);
        }
        --left;
      }
    }
  }
  if (cov_split) {
    add(p->cov, kCovSplit, 0, 0, b0);
    b0 = begin();
    for (int i : order)
      if (forms_r(i))
        fm::cov_each_unit(frames[i].M, prec, [&](int a, int b, int) { items.push_back({i, a, b, 0}); });
    add(p->cov, kCovSplit, 1, 0, b0);
  } else {
    add(p->cov, kCov, 0, 0, b0);
  }

  // stage 2 init: Omega -> V / Y (Method 2 without power iterations, or
  // without R; the first product with R reads Omega itself), gather
  // (Method 1)
  b0 = begin();
  auto is_proj = [&](int i) {
    return frames[i].method == FM_METHOD_PROJECT || frames[i].method == FM_METHOD_PROJECT_X;
  };
  for (int i : order)
    if (is_proj(i) && (frames[i].method == FM_METHOD_PROJECT_X || frames[i].q == 0))
      for (int c = 0; c < rows(frames[i].M, fm::kApplyRows); ++c) items.push_back({i, c, 0, 0});
  add(p->sub, kOmega, 0, 0, b0);
  b0 = begin();
  for (int i : order)
    if (frames[i].method == FM_METHOD_SAMPLE)
      for (int c = 0; c < rows(frames[i].M, fm::kApplyRows); ++c) items.push_back({i, c, 0, 0});
  add(p->sub, kGather, 0, 0, b0);
  // Method 1 without R: Z = conj(X(I, :))^T, C = X Z / T, core = C(I, :)
  auto sample_x = [&](int i) { return frames[i].method == FM_METHOD_SAMPLE_X; };
  b0 = begin();
  for (int i : order)
    if (sample_x(i))
      for (int c = 0; c < rows(frames[i].T, fm::kZxCols); ++c) items.push_back({i, c, 0, 0});
  add(p->sub, kZx, 0, 0, b0);
  for (int nb = 1; nb <= 4; ++nb) {
    b0 = begin();
    for (int i : order)
      if (sample_x(i) && sketch_nb(frames[i].n) == nb)
        for (int c = 0; c < rows(frames[i].M, fm::kSketchRows); ++c) items.push_back({i, c, 0, 0});
    add(p->sub, kXz, -1, nb, b0);
  }
  b0 = begin();
  for (int i : order)
    if (sample_x(i)) items.push_back({i, 0, 0, 0});
  add(p->sub, kXcore, 0, 0, b0);

  const int classes[4] = {16, 32, fm::kSmallLdsN, fm::kMaxN};
  // a sketch of a column class that fuses the Gram step leaves its partials
  auto fused = [&](int i) { return is_proj(i) && fm::sketch_fuses_gram(sketch_nb(frames[i].n)); };
  // after_sketch: this orth follows a product (round >= 1)
  auto orth_round = [&](auto pred, bool after_sketch) {
    size_t b = begin();
    for (int i : order)
      if (pred(i) && !(after_sketch && fused(i)))
        for (int c = 0; c < rows(frames[i].M, fm::kGramRows); ++c) items.push_back({i, c, 0, 0});
    add(p->sub, kGram, fm::kGramSelf, 0, b);
    for (int cl : classes) {
      b = begin();
      for (int i : order)
        if (pred(i) && small_class(frames[i].n) == cl) items.push_back({i, 0, 0, 0});
      add(p->sub, kSmall, fm::kOrth, cl, b);
    }
    b = begin();
    for (int i : order)
      if (pred(i))
        for (int c = 0; c < rows(frames[i].M, fm::kApplyRows); ++c) items.push_back({i, c, 0, 0});
    add(p->sub, kApply, fm::kApplyV, 0, b);
  };
  auto from_x = [&](int i) { return frames[i].method == FM_METHOD_PROJECT_X; };
  auto sketch_round = [&](auto pred, int round) {
    for (int nb = 1; nb <= 4; ++nb) {
      const bool s16 = prec != FM_FP32 && fm::sketch16_ok(nb);
      size_t b = begin();
      for (int i : order)
        if (pred(i) && !from_x(i) && sketch_nb(frames[i].n) == nb) {
          // split: one item per channel segment (Item::c); frames without
          // segments run whole in the same launch
          const int S = sk_split && seg_r(i) ? fm::sketch_segments(frames[i].M, nb) : 1;
          for (int c = 0; c < rows(frames[i].M, fm::kSketchRows); ++c)
            for (int sg = 0; sg < S; ++sg) items.push_back({i, c, 0, sg});
        }
      add(p->sub, sk_split ? (s16 ? kSketch16Seg : kSketchSeg) : (s16 ? kSketch16 : kSketch),
          round, nb, b);
      if (sk_split) {
        b = begin();
        for (int i : order)
          if (pred(i) && !from_x(i) && sketch_nb(frames[i].n) == nb && seg_r(i))
            for (int c = 0; c < rows(frames[i].M, fm::kSketchRows); ++c)
              items.push_back({i, c, 0, 0});
        add(p->sub, s16 ? kSketch16Red : kSketchRed, round, nb, b);
      }
    }
    // without R: Z = X^H V for every such frame, then Y = X Z / T
    for (int nb = 1; nb <= 4; ++nb) {
      size_t b = begin();
      for (int i : order)
        if (pred(i) && from_x(i) && sketch_nb(frames[i].n) == nb)
          for (int c = 0; c < rows(frames[i].T, fm::kXhvCols); ++c) items.push_back({i, c, 0, 0});
      add(p->sub, kXhv, 0, nb, b);
    }
    for (int nb = 1; nb <= 4; ++nb) {
      size_t b = begin();
      for (int i : order)
        if (pred(i) && from_x(i) && sketch_nb(frames[i].n) == nb)
          for (int c = 0; c < rows(frames[i].M, fm::kSketchRows); ++c)
            items.push_back({i, c, 0, 0});
      add(p->sub, kXz, round, nb, b);
    }
  };
  int qmax = 0;
  for (int i = 0; i < n_frames; ++i)
    if (is_proj(i)) qmax = std::max(qmax, frames[i].q);
  // round 0: orth(Omega) for q = 0 frames, then the first product for all
  orth_round([&](int i) { return is_proj(i) && frames[i].q == 0; }, false);
  sketch_round(is_proj, 0);
  for (int r = 1; r <= qmax; ++r) {
    orth_round([&](int i) { return is_proj(i) && frames[i].q >= r; }, true);
    sketch_round([&](int i) { return is_proj(i) && frames[i].q >= r; }, r);
  }
  // final: core and Gram (unless the last product formed them), eigen-solves, U_s
  b0 = begin();
  for (int i : order)
    if (!fused(i))
      for (int c = 0; c < rows(frames[i].M, fm::kGramRows); ++c) items.push_back({i, c, 0, 0});
  add(p->sub, kGram, fm::kGramFinal, 0, b0);
  for (int cl : classes) {
    b0 = begin();
    for (int i : order)
      if (small_class(frames[i].n) == cl) items.push_back({i, 0, 0, 0});
    add(p->sub, kSmall, fm::kFinal, cl, b0);
  }
  b0 = begin();
  for (int i : order)
    for (int c = 0; c < rows(frames[i].M, fm::kApplyRows); ++c) items.push_back({i, c, 0, 0});
  add(p->sub, kApply, fm::kApplyUs, 0, b0);
  // model order of the frames that ask for it (after the status words are set)
  b0 = begin();
  for (int i : order)
    if (frames[i].K_hat) items.push_back({i, 0, 0, 0});
  add(p->sub, kOrder, 0, 0, b0);
  // ESPRIT angles of the frames that ask for them
  b0 = begin();
  for (int i : order)
    if (frames[i].esprit_deg) items.push_back({i, 0, 0, 0});
  add(p->sub, kEsprit, 0, 0, b0);

  // spectrum (every precision): reset the recompute lists (the lag-sum
  // kernel resets those of its frames), lag sums of every frame into its
  // group buffer (row-block partials, then their sums per group), then each
  // group's polynomial pass (tiles of the knob's width for the group's
  // bucket)
  b0 = begin();
  for (int i : order)
    if (grp_of[i] < 0) items.push_back({i, 0, 0, 0});
  add(p->spec, kSpecPrep, 0, 0, b0);
  // one lag per lane (four times the workgroups, the same bits) when the
  // plan's lag-sum workgroups would be few
  long long acw = 0;
  for (int i : order)
    if (grp_of[i] >= 0) acw += (long long)rows(frames[i].M, fm::kAcorrLags) * fm::acorr_blocks(frames[i].M);
  const int ac_wide = acw < kAcorrWideWGs ? 1 : 0;
  b0 = begin();
  for (int i : order)
    if (grp_of[i] >= 0)
      for (int c = 0; c < rows(frames[i].M, fm::acorr_lags(ac_wide)); ++c)
        for (int b = 0; b < fm::acorr_blocks(frames[i].M); ++b) items.push_back({i, c, b, 0});
  add(p->spec, kAcorr, ac_wide, 0, b0);
  b0 = begin();
  for (const auto &g : groups)
    if (fm::acorr_blocks(frames[g[0]].M) > 1)
      for (int c = 0; c < fm::hsum_chunks(frames[g[0]].M); ++c) items.push_back({g[0], c, 0, 0});
  add(p->spec, kHsum, 0, 0, b0);
  long long ptiles = 0;
  for (const auto &g : groups)
    ptiles += rows(frames[g[0]].L, ctx->knob[FM_KNOB_SPEC_ANGLES][spec_nb(frames[g[0]].K) - 1]);
  const bool narrow = ptiles < kPolyNarrowWGs;
  for (int per : {256, 128, 64}) {
    b0 = begin();
    for (const auto &g : groups) {
      const int lead = g[0];
      const int gper = narrow ? 64 : ctx->knob[FM_KNOB_SPEC_ANGLES][spec_nb(frames[lead].K) - 1];
      if (gper != per) continue;
      for (int t = 0; t < rows(frames[lead].L, per); ++t) items.push_back({lead, t, 0, 0});
    }
    add(p->spec, kPoly, per / 64, 0, b0);
  }
  // frames on the split FP16 projection pass: U_s -> hi and lo FP16 planes
  // (one workgroup per 256 entries), then one launch per column class nb and
  // angle tile (64 nnb angles, the context's FM_KNOB_SPEC16_ANGLES)
  auto spec16 = [&](int i) { return frames[i].spec_prec != FM_FP32; };
  b0 = begin();
  for (int i : order)
    if (spec16(i))
      for (int c = 0; c < rows(frames[i].K * frames[i].M, 256); ++c) items.push_back({i, c, 0, 0});
  add(p->spec, kSplit16, 0, 0, b0);
  for (int nb = 1; nb <= 8; ++nb)
    for (int nnb : {4, 2, 1}) {
      b0 = begin();
      for (int i : order) {
        if (!spec16(i) || std::min(spec_nb(frames[i].K), 8) != nb) continue;
        if (ctx->knob[FM_KNOB_SPEC16_ANGLES][nb - 1] / 64 != nnb) continue;
        for (int t = 0; t < rows(frames[i].L, 64 * nnb); ++t) items.push_back({i, t, 0, 0});
      }
      add(p->spec, kSpec16, nnb, nb, b0);
    }
  b0 = begin();
  for (int i : order)
    for (int g = 0; g < fm::kRefineGroups; ++g) items.push_back({i, g, 0, 0});
  add(p->spec, kRefine, 0, 0, b0);
  b0 = begin();
  for (int i : order) items.push_back({i, 0, 0, 0});
  add(p->peaks, kPeaks, 0, 0, b0);

  // member lists of the spectrum groups (16 frame indices, -1 padded) ride
  // at the end of the work-list upload
  std::vector<size_t> gitem(groups.size());
  for (size_t g = 0; g < groups.size(); ++g) {
    gitem[g] = items.size();
    int mem[fm::kPolyRows];
    for (int j = 0; j < fm::kPolyRows; ++j)
      mem[j] = j < (int)groups[g].size() ? groups[g][j] : -1;
    static_assert(fm::kPolyRows % 4 == 0, "member list packs into whole items");
    for (int j = 0; j < fm::kPolyRows; j += 4) items.push_back({mem[j], mem[j + 1], mem[j + 2], mem[j + 3]});
  }
  p->items_bytes = items.size() * sizeof(Item);
  const size_t frames_bytes = align256(sizeof(FrameDev) * n_frames);
  const size_t total_dev = total + frames_bytes + align256(std::max<size_t>(p->items_bytes, 16));
  if (need) *need = total_dev;
  if (dry_run) {
    delete p;
    return FM_OK;
  }
  p->items_h = std::move(items);
  // the member lists' device address, once the work lists have one
  auto bind_members = [&]() {
    for (int i = 0; i < n_frames; ++i)
      if (grp_of[i] >= 0)
        p->frames_h[i].hmem = reinterpret_cast<const int *>(p->items_d + gitem[grp_of[i]]);
  };
  if (p->owned) {
    e = hipMalloc((void **)&p->items_d, std::max<size_t>(p->items_bytes, 256));
    if (e == hipSuccess) bind_members();
    if (e == hipSuccess) e = hipMalloc((void **)&p->frames_d, sizeof(FrameDev) * n_frames);
    if (e == hipSuccess)
      e = hipMemcpy(p->items_d, p->items_h.data(), p->items_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(p->frames_d, p->frames_h.data(), sizeof(FrameDev) * n_frames,
                    hipMemcpyHostToDevice);
  } else {
    if (total_dev > dev_bytes) {
      p->ws = nullptr;
      delete p;
      return fail(ctx, FM_E_WORKSPACE, "plan: needs %zu device bytes, given %zu", total_dev,
                  dev_bytes);
    }
    p->frames_d = reinterpret_cast<FrameDev *>(dev + total);
    p->items_d = reinterpret_cast<Item *>(dev + total + frames_bytes);
    bind_members();
    e = hipMemcpyAsync(p->items_d, p->items_h.data(), p->items_bytes, hipMemcpyHostToDevice,
                       stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p->frames_d, p->frames_h.data(), sizeof(FrameDev) * n_frames,
                         hipMemcpyHostToDevice, stream);
  }
  if (e != hipSuccess) {
    fm_plan_destroy(p);
    return hip_fail(ctx, e, "plan upload");
  }
  *out = p;
  return FM_OK;
}

FM_API fm_status fm_plan_create(fm_ctx *ctx, const fm_frame *frames, int n_frames, fm_prec prec,
                                fm_plan **out) {
  return plan_build(ctx, frames, n_frames, prec, nullptr, 0, nullptr, false, nullptr, out);
}

FM_API size_t fm_plan_bytes(fm_ctx *ctx, const fm_frame *frames, int n_frames, fm_prec prec) {
  size_t need = 0;
  if (plan_build(ctx, frames, n_frames, prec, nullptr, 0, nullptr, true, &need, nullptr) != FM_OK)
    return 0;
  return need;
}

FM_API fm_status fm_plan_create_in(fm_ctx *ctx, const fm_frame *frames, int n_frames,
                                   fm_prec prec, void *dev_mem, size_t dev_bytes, void *stream,
                                   fm_plan **out) {
  if (!dev_mem) return fail(ctx, FM_E_ARG, "plan_create_in: null device memory");
  return plan_build(ctx, frames, n_frames, prec, static_cast<char *>(dev_mem), dev_bytes,
                    (hipStream_t)stream, false, nullptr, out);
}

FM_API fm_status fm_plan_destroy(fm_plan *p) {
  if (!p) return FM_E_ARG;
  hipSetDevice(p->ctx->device);
  if (p->owned) hipDeviceSynchronize();
  if (p->gexec) hipGraphExecDestroy(p->gexec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  if (p->owned) {
    if (p->items_d) hipFree(p->items_d);
    if (p->frames_d) hipFree(p->frames_d);
    if (p->ws) hipFree(p->ws);
  }
  delete p;
  return FM_OK;
}

FM_API size_t fm_plan_workspace_bytes(const fm_plan *p) {
  return p ? p->ws_bytes + p->items_bytes + sizeof(FrameDev) * p->n_frames : 0;
}

FM_API fm_status fm_plan_covariance(fm_plan *p, void *stream) {
  return p ? run_list(p, p->cov, stream) : FM_E_ARG;
}
FM_API fm_status fm_plan_subspace(fm_plan *p, void *stream) {
  return p ? run_list(p, p->sub, stream) : FM_E_ARG;
}
FM_API fm_status fm_plan_pseudospectrum(fm_plan *p, void *stream) {
  return p ? run_list(p, p->spec, stream) : FM_E_ARG;
}
FM_API fm_status fm_plan_peaks(fm_plan *p, void *stream) {
  return p ? run_list(p, p->peaks, stream) : FM_E_ARG;
}

FM_API fm_status fm_plan_run(fm_plan *p, void *stream, int use_graph) {
  if (!p) return FM_E_ARG;
  fm_status st = set_dev(p->ctx);
  if (st != FM_OK) return st;
  if (!use_graph) {
    if ((st = run_list(p, p->cov, stream)) != FM_OK) return st;
    if ((st = run_list(p, p->sub, stream)) != FM_OK) return st;
    if ((st = run_list(p, p->spec, stream)) != FM_OK) return st;
    return run_list(p, p->peaks, stream);
  }
  hipStream_t s = (hipStream_t)stream;
  if (!p->gexec) {
    hipError_t e = hipSuccess;
    if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "hipStreamCreateWithFlags");
    e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "hipStreamBeginCapture");
    void *cs = (void *)p->cap_stream;
    fm_status cst = run_list(p, p->cov, cs);
    if (cst == FM_OK) cst = run_list(p, p->sub, cs);
    if (cst == FM_OK) cst = run_list(p, p->spec, cs);
    if (cst == FM_OK) cst = run_list(p, p->peaks, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &g);
    if (cst != FM_OK) { if (g) hipGraphDestroy(g); return cst; }
    if (e != hipSuccess) return hip_fail(p->ctx, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { hipGraphDestroy(g); return hip_fail(p->ctx, e, "hipGraphInstantiate"); }
    p->graph = g;
  }
  hipError_t e = hipGraphLaunch(p->gexec, s);
  return e == hipSuccess ? FM_OK : hip_fail(p->ctx, e, "hipGraphLaunch");
}
