// fm_poly.hip -- stage 3, FP32 bulk pass: the MUSIC pseudo-spectrum
// (eqs. (5) and (10)) evaluated as a trigonometric polynomial in sin(theta).
//
// With c_k = sum_m conj(U[k][m]) a_m and a_m = exp(-j pi m u), u = sin(theta),
//   sum_k |c_k|^2 = sum_{m,m'} Q[m][m'] a_m conj(a_m'),  Q[m][m'] = sum_k conj(U[k][m]) U[k][m'],
// and a_m conj(a_m') = a_{m-m'} depends on the lag d = m - m' only, so
//   sum_k |c_k|^2 = h_0 + 2 Re sum_{d>=1} h_d a_d,  h_d = sum_k sum_m' conj(U[k][m'+d]) U[k][m']
// (h_{-d} = conj(h_d)).  With h'_0 = h_0 / 2 and h'_d = h_d otherwise,
//   den(theta) = M - 2 Re sum_{d=0}^{M-1} h'_d a_d(theta),   P = 1 / den:
// one length-M inner product per angle whatever K is, against the steering
// vector itself.  This is the same quantity as eq. (5) in exact arithmetic.
//
// acorr: the lag sums h'_d of one frame in FP32 from U_s rounded to FP32, as
//   partial sums over blocks of 256 rows (four adjacent lags per lane with a
//   sliding register window, a four-wave workgroup per 256 lags and row
//   block, each wave over 64 of its rows, so no lane runs longer than
//   4 x 64 K products; the columns staged through LDS; fixed order over k,
//   then m, then the four quarters).
// hsum:  adds each group's row-block partials in block order, once, into the
//   first block, which the polynomial pass then reads.
// poly:  frames with the same M and angle grid form groups of up to 16; the
//   group's conj(h') vectors are the 16 rows of v_mfma_f32_16x16x4_f32 and the
//   angles its columns, so each generated steering phasor and each staged
//   operand serve the whole group.  A frame's rows of the products do not
//   depend on the other rows, so a frame's result is the same in any group
//   (or alone).  Steering, the FP32 floor and the list of main-lobe angles
//   for the FP64 recompute are those of the per-frame pass.
#include "fm_internal.h"
#include "fm_steer.h"

namespace fm {
namespace {

using namespace steer;

typedef float floatx4 __attribute__((ext_vector_type(4)));

// kAcL adjacent lags per lane (4; 1 for single frames and small plans,
// acorr_wide): a wave covers 64 kAcL lags, the workgroup's lag chunk.  A
// lag's sums run in the same order either way (k outer, m ascending within
// a quarter block, then the quarters in order), so both forms give the same
// bits.
constexpr int kAcLanes = 64;                   // lanes per lag chunk (one wave)
constexpr int kAcWaves = 4;                    // waves per row block
constexpr int kAcThreads = kAcLanes * kAcWaves;
constexpr int kAcSub = kAcorrRows / kAcWaves;  // rows per wave
static_assert(kAcorrLags == 4 * kAcLanes, "the 4-lag form covers kAcorrLags");

// One workgroup (four waves): 64 kAcL consecutive lags d0.. of one frame,
// kAcL adjacent lags per lane, over one block of kAcorrRows rows m, each
// wave taking a quarter of the block's rows; the block's partial sums (the
// quarters' sums added in order) go to block `rb` of the group buffer.  A
// lane keeps the kAcL values U[k][m + d] of its lags in registers and slides
// them by one row per step (one new LDS value per kAcL products), reading
// the LDS values of eight steps ahead of their use.  A lag's rows run to
// M - 1 - d: the staged window is zero past M, so the extra products of a
// lane's later lags add exact zeros.  Summation order within a quarter
// block: k outer, m ascending; the blocks are added in order by the
// polynomial pass.
template <int kAcL, bool kBatched>
__global__ __launch_bounds__(kAcThreads) void acorr_kernel(FrameDev single,
                                                           const FrameDev *frames,
                                                           const Item *items) {
  constexpr int kLags = kAcLanes * kAcL;           // lags per workgroup
  constexpr int kPadShift = kAcL == 4 ? 3 : 4;     // lag-window padding period
  __shared__ float2 wa[kAcorrRows];
  // the lag window, one float2 of padding after every 2^kPadShift: lane l
  // reads element kAcL l + c, and without the padding lanes 64 / kAcL apart
  // would hit the same LDS banks (with it, at most two lanes share a bank)
  constexpr int kWbN = kAcorrRows + kLags + kAcL;
  __shared__ float2 wb[kWbN + (kWbN >> kPadShift) + 1];
  __shared__ float2 part[kAcWaves - 1][kAcL][kAcLanes];  // the other waves' sums
  int chunk, rb;
  const FrameDev *fp;
  if constexpr (kBatched) {
    const Item it = items[blockIdx.x];
    chunk = it.a;
    rb = it.b;
    fp = frames + it.frame;
  } else {
    chunk = blockIdx.x;
    rb = blockIdx.y;
    fp = &single;
  }
  const int M = fp->M, K = fp->K;
  // the first workgroup of a frame empties its FP64-recompute list, which
  // the polynomial pass fills next (the previous run's readers are done)
  if (chunk == 0 && rb == 0 && threadIdx.x == 0) fp->rlist[0] = 0;
  const double2 *Us = fp->Us;
  FM_GLOBAL float2 *hg = (FM_GLOBAL float2 *)(fp->hgrp + (size_t)rb * M * kPolyRows);
  const int slot = fp->hslot;
  const int tid = threadIdx.x;
  const int lane = tid & (kAcLanes - 1), wave = tid / kAcLanes;
  const int d0 = chunk * kLags;
  const int dl = d0 + kAcL * lane;          // this lane's first lag
  const int m0 = rb * kAcorrRows;
  const int mw = m0 + wave * kAcSub;        // this wave's first row
  float re[kAcL], im[kAcL];
#pragma unroll
  for (int j = 0; j < kAcL; ++j) re[j] = im[j] = 0.f;
  // column k of U_s in registers, fetched one column ahead with
  // unconditional global loads (rows past M read row M - 1 and are staged as
  // zero), then staged in LDS as FP32 (the values of its FP32 copy)
  constexpr int kWa = kAcorrRows / kAcThreads;
  constexpr int kWb = (kWbN + kAcThreads - 1) / kAcThreads;
  const FM_GLOBAL double2 *Ug = (const FM_GLOBAL double2 *)Us;
  double2 pa[kWa], pb[kWb];
  auto fetch = [&](int k) {
    const FM_GLOBAL double2 *u = Ug + (size_t)min(k, K - 1) * M;
#pragma unroll
    for (int i = 0; i < kWa; ++i) pa[i] = u[min(m0 + tid + kAcThreads * i, M - 1)];
#pragma unroll
    for (int i = 0; i < kWb; ++i) pb[i] = u[min(m0 + d0 + tid + kAcThreads * i, M - 1)];
  };
  auto stage = [&]() {
#pragma unroll
    for (int i = 0; i < kWa; ++i) {
      const int e = tid + kAcThreads * i;
      const double2 v = m0 + e < M ? pa[i] : make_double2(0.0, 0.0);
      wa[e] = make_float2((float)v.x, (float)v.y);
    }
#pragma unroll
    for (int i = 0; i < kWb; ++i) {
      const int e = tid + kAcThreads * i;
      const double2 v = m0 + d0 + e < M ? pb[i] : make_double2(0.0, 0.0);
      if (e < kWbN) wb[e + (e >> kPadShift)] = make_float2((float)v.x, (float)v.y);
    }
  };
  if (m0 + d0 < M) {  // uniform: some lag of this workgroup reaches the block
    fetch(0);
    // rows of this wave's quarter used by the lane's first (longest) lag
    const int cnt = min(kAcSub, M - dl - mw);
    const int base = kAcL * lane + wave * kAcSub;
    const float2 *wah = wa + wave * kAcSub;
    for (int k = 0; k < K; ++k) {
      __syncthreads();  // the previous column has been read
      stage();
      __syncthreads();
      fetch(k + 1);
      if (cnt > 0) {
        float2 x[kAcL];
#pragma unroll
        for (int j = 0; j < kAcL; ++j) x[j] = wb[base + j + ((base + j) >> kPadShift)];
        // one step: conj(U[k][m + d]) * U[k][m], m = mw + i, d = dl + j,
        // then the window slides by the next value xn
        auto step = [&](float2 y, float2 xn) {
#pragma unroll
          for (int j = 0; j < kAcL; ++j) {
            re[j] = fmaf(x[j].x, y.x, fmaf(x[j].y, y.y, re[j]));
            im[j] = fmaf(x[j].x, y.y, fmaf(-x[j].y, y.x, im[j]));
          }
#pragma unroll
          for (int j = 0; j + 1 < kAcL; ++j) x[j] = x[j + 1];
          x[kAcL - 1] = xn;
        };
        int i = 0;
        for (; i + 8 <= cnt; i += 8) {
          float2 y[8], xn[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            y[u] = wah[i + u];
            const int e = base + i + u + kAcL;
            xn[u] = wb[e + (e >> kPadShift)];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) step(y[u], xn[u]);
        }
        for (; i < cnt; ++i) {
          const int e = base + i + kAcL;
          step(wah[i], wb[e + (e >> kPadShift)]);
        }
      }
    }
  }
  // the block's sums: the quarters added in order
  if (wave > 0) {
#pragma unroll
    for (int j = 0; j < kAcL; ++j) part[wave - 1][j][lane] = make_float2(re[j], im[j]);
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int w = 0; w < kAcWaves - 1; ++w)
#pragma unroll
    for (int j = 0; j < kAcL; ++j) {
      const float2 o = part[w][j][lane];
      re[j] += o.x;
      im[j] += o.y;
    }
#pragma unroll
  for (int j = 0; j < kAcL; ++j) {
    const int d = dl + j;
    if (d < M) {
      float r = re[j], q = im[j];
      if (d == 0) {
        r *= 0.5f;  // h'_0 = h_0 / 2 (h_0 is real; halving each partial is exact)
        q = 0.f;
      }
      hg[(size_t)d * kPolyRows + slot] = make_float2(r, -q);  // conj of the partial
    }
  }
}

// Row-block partials of a group buffer added in block order (starting from
// zero, as the sums of the single-block case) into the first block: one
// workgroup per kHsumElems entries of the group's M x kPolyRows lag sums.
constexpr int kHsumElems = 1024;

template <bool kBatched>
__global__ __launch_bounds__(256) void hsum_kernel(FrameDev single, const FrameDev *frames,
                                                   const Item *items) {
  const FrameDev &g = kBatched ? frames[items[blockIdx.x].frame] : single;
  const int chunk = kBatched ? items[blockIdx.x].a : blockIdx.x;
  const size_t total = (size_t)g.M * kPolyRows;
  const int nrb = acorr_blocks(g.M);
  float2 *hg = g.hgrp;
#pragma unroll
  for (int j = 0; j < kHsumElems / 256; ++j) {
    const size_t e = (size_t)chunk * kHsumElems + threadIdx.x + 256 * j;
    if (e < total) {
      float2 v = make_float2(0.f, 0.f);
      for (int b = 0; b < nrb; ++b) {
        const float2 x = hg[(size_t)b * total + e];
        v = make_float2(v.x + x.x, v.y + x.y);
      }
      hg[e] = v;
    }
  }
}

// one tile of 64 NNB angles of a group (four waves of 16 NNB angles); the
// group buffer is staged through LDS in chunks of kSpecChunk lags, double
// buffered like the per-frame pass
template <int NNB, bool kBatched>
__device__ __forceinline__ void poly_tile(const FrameDev &single, const FrameDev *frames,
                                          const FrameDev &g, int tile, const float2 *tab,
                                          float2 (*hbuf)[kSpecChunk * kPolyRows]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n = lane & 15, r = lane >> 4;
  const int M = g.M, L = g.L;
  // global-address loads (a flat load would also count against the LDS
  // waits of the MFMA loop and drain this prefetch every chunk)
  const FM_GLOBAL float2 *hg = (const FM_GLOBAL float2 *)g.hgrp;
  const int first = tile * (64 * NNB) + wave * (16 * NNB);
  unsigned long long F[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb)
    F[nb] = turn_freq(g.theta0, g.dtheta, min(first + 16 * nb + n, L - 1));
  floatx4 acc[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};

  constexpr int kChunkElems = kSpecChunk * kPolyRows;  // 1024 float2, 4 per thread
  const int nchunk = (M + kSpecChunk - 1) / kSpecChunk;
  const size_t total = (size_t)M * kPolyRows;
  float2 stage[kChunkElems / 256];
  // conj(h'_d) of each slot (the sums hsum left in the first block)
  auto load_chunk = [&](int c) {
    const size_t base = (size_t)c * kChunkElems;
#pragma unroll
    for (int j = 0; j < kChunkElems / 256; ++j) {
      const size_t e = base + tid + 256 * j;
      const float2 v = hg[e < total ? e : total - 1];   // unconditional load
      stage[j] = e < total ? v : make_float2(0.f, 0.f);
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int j = 0; j < kChunkElems / 256; ++j) hbuf[buf][tid + 256 * j] = stage[j];
  };
  load_chunk(0);
  store_chunk(0);
  __syncthreads();  // publishes the first chunk and the phasor table
  float2 w4[NNB], ph[NNB];
#pragma unroll
  for (int nb = 0; nb < NNB; ++nb) w4[nb] = phasor32(4u, F[nb], tab);

  for (int c = 0; c < nchunk; ++c) {
    const bool more = c + 1 < nchunk;
    if (more) load_chunk(c + 1);
    const float2 *hb = hbuf[c & 1];
#pragma unroll 4
    for (int s = 0; s < kSpecChunk / 4; ++s) {
      const int d = c * kSpecChunk + 4 * s + r;
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb)
        ph[nb] = (s == 0) ? phasor32((unsigned)d, F[nb], tab) : cmulf(ph[nb], w4[nb]);
      // row n = group slot n: u = conj(h'_d), Re(conj(u) a) = u.x a.x + u.y a.y
      const float2 u = hb[(4 * s + r) * kPolyRows + n];
#pragma unroll
      for (int nb = 0; nb < NNB; ++nb) {
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(u.x, ph[nb].x, acc[nb], 0, 0, 0);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(u.y, ph[nb].y, acc[nb], 0, 0, 0);
      }
    }
    if (more) store_chunk((c + 1) & 1);
    __syncthreads();
  }
  // lane (r, n) holds rows 4r..4r+3 (group slots) of angle column n
  const float Mf = (float)M;
  const float floor32 = Mf * 5.9604644775390625e-08f;  // M * 2^-24
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int slot = 4 * r + v;
    if (slot >= g.hcount) continue;
    const FrameDev &f = kBatched ? frames[g.hmem[slot]] : single;
    float *P = f.P;
    int *rlist = f.rlist;
#pragma unroll
    for (int nb = 0; nb < NNB; ++nb) {
      const int gl = first + 16 * nb + n;
      if (gl < L) {
        const float den32 = fmaf(-2.0f, acc[nb][v], Mf);
        P[gl] = 1.0f / fmaxf(den32, floor32);
        // main lobes, where the denominator cancels, are recomputed in FP64
        if (den32 < Mf * 0.0625f) {
          const int k = atomicAdd(rlist, 1);
          rlist[1 + k] = gl;
        }
      }
    }
  }
}

template <int NNB, bool kBatched>
__global__ __launch_bounds__(256) void poly_kernel(FrameDev single, const FrameDev *frames,
                                                   const Item *items) {
  __shared__ float2 tab[256];
  __shared__ float2 hbuf[2][kSpecChunk * kPolyRows];
  {
    double s, c;
    sincospi((double)threadIdx.x / 128.0, &s, &c);
    tab[threadIdx.x] = make_float2((float)c, (float)s);
  }
  // (the first __syncthreads in poly_tile also publishes the table)
  if constexpr (kBatched) {
    const Item it = items[blockIdx.x];
    poly_tile<NNB, true>(single, frames, frames[it.frame], it.a, tab, hbuf);
  } else {
    poly_tile<NNB, false>(single, frames, single, blockIdx.x, tab, hbuf);
  }
}

template <int NNB>
hipError_t launch_poly_nnb(const FrameDev &single, const FrameDev *frames, const Item *items,
                           int n_items, hipStream_t s) {
  if (items) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL((poly_kernel<NNB, true>), dim3(n_items), dim3(256), 0, s, single, frames,
                       items);
  } else {
    const int tiles = (single.L + 64 * NNB - 1) / (64 * NNB);
    hipLaunchKernelGGL((poly_kernel<NNB, false>), dim3(tiles), dim3(256), 0, s, single, frames,
                       items);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_acorr(const FrameDev &single, const FrameDev *frames, const Item *items,
                        int n_items, int wide, hipStream_t s) {
  if (items) {
    if (n_items <= 0) return hipSuccess;
    if (wide)
      hipLaunchKernelGGL((acorr_kernel<1, true>), dim3(n_items), dim3(kAcThreads), 0, s, single,
                         frames, items);
    else
      hipLaunchKernelGGL((acorr_kernel<4, true>), dim3(n_items), dim3(kAcThreads), 0, s, single,
                         frames, items);
  } else {
    const int chunks = (single.M + acorr_lags(wide) - 1) / acorr_lags(wide);
    if (wide)
      hipLaunchKernelGGL((acorr_kernel<1, false>), dim3(chunks, acorr_blocks(single.M)),
                         dim3(kAcThreads), 0, s, single, frames, items);
    else
      hipLaunchKernelGGL((acorr_kernel<4, false>), dim3(chunks, acorr_blocks(single.M)),
                         dim3(kAcThreads), 0, s, single, frames, items);
  }
  return hipGetLastError();
}

int hsum_chunks(int M) { return (M * kPolyRows + kHsumElems - 1) / kHsumElems; }

hipError_t launch_hsum(const FrameDev &single, const FrameDev *frames, const Item *items,
                       int n_items, hipStream_t s) {
  if (items) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(hsum_kernel<true>, dim3(n_items), dim3(256), 0, s, single, frames, items);
  } else {
    hipLaunchKernelGGL(hsum_kernel<false>, dim3(hsum_chunks(single.M)), dim3(256), 0, s, single,
                       frames, items);
  }
  return hipGetLastError();
}

hipError_t launch_poly(const FrameDev &single, const FrameDev *frames, const Item *items,
                       int n_items, int nnb, hipStream_t s) {
  if (nnb == 4) return launch_poly_nnb<4>(single, frames, items, n_items, s);
  if (nnb == 2) return launch_poly_nnb<2>(single, frames, items, n_items, s);
  return launch_poly_nnb<1>(single, frames, items, n_items, s);
}

}  // namespace fm
