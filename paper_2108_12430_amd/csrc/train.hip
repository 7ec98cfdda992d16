// Training-step kernels for the DeepClean-shaped network: batch-statistics
// normalisation (forward and backward, fused with tanh and its derivative),
// per-channel reductions, deterministic weight gradients, and the band-passed
// MSE loss.  Every reduction has a fixed combination order (chunk partials in
// FP64, then a fixed tree), so results are bitwise reproducible and do not
// depend on scheduling.
#include "internal.h"

#include <algorithm>
#include <initializer_list>

namespace gw {

static constexpr int RCHUNK = 4096;  // (batch, time) elements per reduction chunk

// Fixed-order block reduction of two doubles over 256 lanes.
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sa[256], sb[256];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
  __syncthreads();
}

// Fixed-order block reduction of N doubles per thread over 256 lanes: the
// same pairing tree as block_sum2 for every value, all values per round.
template <int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N]) {
  __shared__ double sv[N][256];
#pragma unroll
  for (int j = 0; j < N; ++j) sv[j][threadIdx.x] = v[j];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int j = 0; j < N; ++j) sv[j][threadIdx.x] += sv[j][threadIdx.x + w];
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = sv[j][0];
  __syncthreads();
}

enum RMode { R_STATS = 0, R_BNBWD = 1, R_SUM = 2 };

struct RedP {
  const float* x;       // z (stats), g (bnbwd), x (sum): [n][C][L]
  const float* a;       // tanh output (bnbwd)
  const float* z;       // pre-normalisation values (bnbwd)
  const float* mean;
  const float* invstd;
  int n, C, L, nchunk;
  double* partial;      // [C][nchunk][2]
};

// Stage 1: chunk partials.  R_STATS sums (z, z^2); R_BNBWD sums (dh, dh*xhat)
// with dh = g (1 - a^2) and xhat = (z - mean) invstd; R_SUM sums (x, 0).
template <int MODE>
__global__ __launch_bounds__(256) void chan_partial(RedP p) {
  const int q = blockIdx.x, c = blockIdx.y;
  const int64_t N = (int64_t)p.n * p.L;
  double s0 = 0.0, s1 = 0.0;
  float mu = 0.f, is = 0.f;
  if (MODE == R_BNBWD) {
    mu = p.mean[c];
    is = p.invstd[c];
  }
  // this thread's elements e = q RCHUNK + 256 r + tid, (b, t) = (e / L, e % L)
  // tracked incrementally; all loads are issued before the in-order sums
  constexpr int NR = RCHUNK / 256;
  const int64_t e0 = (int64_t)q * RCHUNK + threadIdx.x;
  const int nr = (int)std::max<int64_t>(0, std::min<int64_t>(NR, (N - e0 + 255) / 256));
  int64_t b = e0 / p.L;
  int t = (int)(e0 - b * p.L);
  int64_t idx[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    idx[r] = r < nr ? (b * p.C + c) * p.L + t : 0;
    t += 256;
    while (t >= p.L) {
      t -= p.L;
      ++b;
    }
  }
  float xv[NR], av[MODE == R_BNBWD ? NR : 1], zv[MODE == R_BNBWD ? NR : 1];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    xv[r] = p.x[idx[r]];
    if (MODE == R_BNBWD) {
      av[r] = p.a[idx[r]];
      zv[r] = p.z[idx[r]];
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nr) break;
    if (MODE == R_STATS) {
      const double v = xv[r];
      s0 += v;
      s1 += v * v;
    } else if (MODE == R_BNBWD) {
      const float dh = xv[r] * (1.0f - av[r] * av[r]);
      const float xh = (zv[r] - mu) * is;
      s0 += (double)dh;
      s1 += (double)dh * (double)xh;
    } else {
      s0 += (double)xv[r];
    }
  }
  block_sum2(s0, s1);
  if (threadIdx.x == 0) {
    p.partial[((int64_t)c * p.nchunk + q) * 2 + 0] = s0;
    p.partial[((int64_t)c * p.nchunk + q) * 2 + 1] = s1;
  }
}

// Stage 2: one block per channel combines the chunk partials in a fixed tree.
// Outputs (by mode):
//   R_STATS: o0 = mean, o1 = 1/sqrt(var + eps) (biased variance)
//   R_BNBWD: o0 = dbeta = sum dh, o1 = dgamma = sum dh*xhat
//   R_SUM:   o0 = sum
template <int MODE>
__global__ __launch_bounds__(256) void chan_final(const double* partial, int nchunk, int64_t N,
                                                  float* o0, float* o1) {
  const int c = blockIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int q = threadIdx.x; q < nchunk; q += 256) {
    s0 += partial[((int64_t)c * nchunk + q) * 2 + 0];
    s1 += partial[((int64_t)c * nchunk + q) * 2 + 1];
  }
  block_sum2(s0, s1);
  if (threadIdx.x != 0) return;
  if (MODE == R_STATS) {
    const double m = s0 / (double)N;
    double v = s1 / (double)N - m * m;
    if (v < 0.0) v = 0.0;
    o0[c] = (float)m;
    o1[c] = (float)(1.0 / sqrt(v + 1e-5));
  } else if (MODE == R_BNBWD) {
    o0[c] = (float)s0;
    o1[c] = (float)s1;
  } else {
    o0[c] = (float)s0;
  }
}

int red_chunks(int n, int L) { return (int)(((int64_t)n * L + RCHUNK - 1) / RCHUNK); }

hipError_t launch_bn_stats(const float* z, int n, int C, int L, double* partial, int nchunk,
                           float* mean, float* invstd, hipStream_t st) {
  RedP p{};
  p.x = z;
  p.n = n;
  p.C = C;
  p.L = L;
  p.nchunk = nchunk;
  p.partial = partial;
  hipLaunchKernelGGL(chan_partial<R_STATS>, dim3(nchunk, C), dim3(256), 0, st, p);
  hipLaunchKernelGGL(chan_final<R_STATS>, dim3(C), dim3(256), 0, st, partial, nchunk,
                     (int64_t)n * L, mean, invstd);
  return hipGetLastError();
}

hipError_t launch_channel_sum(const float* x, int n, int C, int L, double* partial, int nchunk,
                              float* out, hipStream_t st) {
  RedP p{};
  p.x = x;
  p.n = n;
  p.C = C;
  p.L = L;
  p.nchunk = nchunk;
  p.partial = partial;
  hipLaunchKernelGGL(chan_partial<R_SUM>, dim3(nchunk, C), dim3(256), 0, st, p);
  hipLaunchKernelGGL(chan_final<R_SUM>, dim3(C), dim3(256), 0, st, partial, nchunk,
                     (int64_t)n * L, out, (float*)nullptr);
  return hipGetLastError();
}

// Elementwise kernels over [n][C][L]: grid y = rows (b C + c, strided by
// gridDim.y), x = runs of 1024 positions; 4 positions per thread, as one
// float4 when every row starts 16-byte aligned.
static inline bool rows_vec4(int L, std::initializer_list<const void*> ptrs) {
  if (L % 4) return false;
  for (const void* q : ptrs)
    if (reinterpret_cast<uintptr_t>(q) % 16) return false;
  return true;
}

static inline dim3 rows_grid(int n, int C, int L) {
  const int64_t rows = (int64_t)n * C;
  return dim3((unsigned)((L + 1023) / 1024), (unsigned)std::min<int64_t>(rows, 65535));
}

// a = tanh(gamma (z - mean) invstd + beta)
template <bool V4>
__global__ __launch_bounds__(256) void bn_apply_tanh_kernel(const float* z, const float* mean,
                                                            const float* invstd, const float* gamma,
                                                            const float* beta, float* a, int C,
                                                            int L, int64_t rows) {
  const int t = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (t >= L) return;
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const int c = (int)(row % C);
    const float m = mean[c], is = invstd[c], g = gamma[c], be = beta[c];
    const float* zr = z + row * L + t;
    float* ar = a + row * L + t;
    if (V4) {
      const float4 v = *reinterpret_cast<const float4*>(zr);
      float4 r;
      r.x = tanhf(fmaf(g, (v.x - m) * is, be));
      r.y = tanhf(fmaf(g, (v.y - m) * is, be));
      r.z = tanhf(fmaf(g, (v.z - m) * is, be));
      r.w = tanhf(fmaf(g, (v.w - m) * is, be));
      *reinterpret_cast<float4*>(ar) = r;
    } else {
      for (int j = 0; j < 4 && t + j < L; ++j) ar[j] = tanhf(fmaf(g, (zr[j] - m) * is, be));
    }
  }
}

hipError_t launch_bn_apply_tanh(const float* z, const float* mean, const float* invstd,
                                const float* gamma, const float* beta, float* a, int n, int C,
                                int L, hipStream_t st) {
  const int64_t rows = (int64_t)n * C;
  if (rows < 1 || L < 1) return hipSuccess;
  if (rows_vec4(L, {z, a}))
    hipLaunchKernelGGL(bn_apply_tanh_kernel<true>, rows_grid(n, C, L), dim3(256), 0, st, z, mean, invstd, gamma,
                       beta, a, C, L, rows);
  else
    hipLaunchKernelGGL(bn_apply_tanh_kernel<false>, rows_grid(n, C, L), dim3(256), 0, st, z, mean, invstd, gamma,
                       beta, a, C, L, rows);
  return hipGetLastError();
}

// dz = gamma invstd (dh - sum(dh)/N - xhat sum(dh xhat)/N), dh = g (1 - a^2)
__device__ __forceinline__ float bn_tanh_bwd_one(float g, float av, float zv, float m, float is, float gis,
                                                 float s1, float s2) {
  const float dh = g * (1.0f - av * av);
  const float xh = (zv - m) * is;
  return gis * (dh - s1 - xh * s2);
}

template <bool V4>
__global__ __launch_bounds__(256) void bn_tanh_bwd_kernel(const float* g, const float* a,
                                                          const float* z, const float* mean,
                                                          const float* invstd, const float* gamma,
                                                          const float* sdh, const float* sdhx,
                                                          float* dz, int C, int L, int64_t rows,
                                                          float invN) {
  const int t = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (t >= L) return;
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const int c = (int)(row % C);
    const float m = mean[c], is = invstd[c], gis = gamma[c] * invstd[c];
    const float s1 = sdh[c] * invN, s2 = sdhx[c] * invN;
    const int64_t o = row * L + t;
    if (V4) {
      const float4 gv = *reinterpret_cast<const float4*>(g + o);
      const float4 av = *reinterpret_cast<const float4*>(a + o);
      const float4 zv = *reinterpret_cast<const float4*>(z + o);
      float4 r;
      r.x = bn_tanh_bwd_one(gv.x, av.x, zv.x, m, is, gis, s1, s2);
      r.y = bn_tanh_bwd_one(gv.y, av.y, zv.y, m, is, gis, s1, s2);
      r.z = bn_tanh_bwd_one(gv.z, av.z, zv.z, m, is, gis, s1, s2);
      r.w = bn_tanh_bwd_one(gv.w, av.w, zv.w, m, is, gis, s1, s2);
      *reinterpret_cast<float4*>(dz + o) = r;
    } else {
      for (int j = 0; j < 4 && t + j < L; ++j)
        dz[o + j] = bn_tanh_bwd_one(g[o + j], a[o + j], z[o + j], m, is, gis, s1, s2);
    }
  }
}

hipError_t launch_bn_tanh_backward(const float* g, const float* a, const float* z,
                                   const float* mean, const float* invstd, const float* gamma,
                                   int n, int C, int L, double* partial, int nchunk, float* dz,
                                   float* dgamma, float* dbeta, hipStream_t st) {
  RedP p{};
  p.x = g;
  p.a = a;
  p.z = z;
  p.mean = mean;
  p.invstd = invstd;
  p.n = n;
  p.C = C;
  p.L = L;
  p.nchunk = nchunk;
  p.partial = partial;
  hipLaunchKernelGGL(chan_partial<R_BNBWD>, dim3(nchunk, C), dim3(256), 0, st, p);
  hipLaunchKernelGGL(chan_final<R_BNBWD>, dim3(C), dim3(256), 0, st, partial, nchunk,
                     (int64_t)n * L, dbeta, dgamma);
  const int64_t rows = (int64_t)n * C;
  const float invN = (float)(1.0 / ((double)n * L));
  if (rows_vec4(L, {g, a, z, dz}))
    hipLaunchKernelGGL(bn_tanh_bwd_kernel<true>, rows_grid(n, C, L), dim3(256), 0, st, g, a, z, mean, invstd, gamma,
                       dbeta, dgamma, dz, C, L, rows, invN);
  else
    hipLaunchKernelGGL(bn_tanh_bwd_kernel<false>, rows_grid(n, C, L), dim3(256), 0, st, g, a, z, mean, invstd, gamma,
                       dbeta, dgamma, dz, C, L, rows, invN);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weight gradient: dw[a][c][j] = sum_b sum_t P[b][a][t] * Q[b][c][s t - p + j]
// (Q zero outside [0, Lq)).  For a conv layer P = dL/dz (a = out channel) and
// Q = layer input; for a transposed layer P = layer input and Q = dL/dz.
// Stage 1, a split-K GEMM on the matrix cores: D[a][n] (n = c k + j) summed
// over K = (batch item, time).  Block g walks a fixed run of chunks (batch
// item, WT time steps) in order.  Each thread loads its share of a chunk (P
// rows and the matching window of Q) into registers in one batch of
// independent loads, and the next chunk's loads are issued before the current
// chunk's MFMAs, so memory latency overlaps compute.  The staged chunk sits in
// LDS (FP32) and v_mfma_f32_16x16x4_f32 (exact FP32 products, FP32
// accumulation) runs over WT / 4 K steps of 4 time steps.  Layers with fewer
// accumulator tiles than waves split each chunk's K steps between wave
// groups, whose accumulators are added in a fixed order at the end.  The
// block's sums are written once as block g's FP32 partial.  Stages 2 and 3 add
// the partials of every weight in a fixed two-level tree (groups of 64
// partials, then the groups) in FP64.  Every order is fixed: the result is
// deterministic.
// ---------------------------------------------------------------------------
static constexpr int WG = 64;    // partials per group of the reduction tree
static constexpr int WNW = 8;    // waves per block
static constexpr int WTH = 64 * WNW;
static constexpr int WTPW = 7;   // most accumulator tiles per wave

// chunk configurations, largest chunk first: time steps, the most P and Q
// elements one thread stages per chunk, the most accumulator tiles per wave
struct WgCfg {
  int wt, pmax, qmax, ntmax;
};
static constexpr WgCfg kWgCfg[] = {{1024, 8, 24, 3}, {512, 8, 24, 3}, {256, 8, 24, 3},
                                   {128, 8, 12, 3},  {64, 8, 12, 7},  {64, 16, 24, 7}};

static int wgrad_qs(int span) { return span + ((16 - span % 64) + 64) % 64; }  // row stride = 16 mod 64 banks

static size_t wgrad_lds(int Ca, int Cc, int k, int s, int wt) {
  const size_t need = sizeof(float) * ((size_t)(Ca + 1) * (wt + 4) + (size_t)(Cc + 1) * wgrad_qs(s * (wt - 1) + k) + WTH);
  return std::max(need, sizeof(float) * 8 * 256);  // room to combine the wave groups' accumulators
}

// wave groups splitting a chunk's K steps: as many as the idle waves allow
// (ntile accumulator tiles, ksp * ntile <= 8 when ntile < 8)
__host__ __device__ inline int wgrad_ksp(int ntile) {
  return ntile >= WNW ? 1 : (2 * ntile > WNW ? 1 : (4 * ntile > WNW ? 2 : (8 * ntile > WNW ? 4 : 8)));
}

// the configuration a layer runs with (index into kWgCfg), -1 if none fits
static int wgrad_cfg(int Ca, int Cc, int k, int s) {
  const int ntile = ((Ca + 15) / 16) * ((Cc * k + 15) / 16);
  const int nwk = WNW / wgrad_ksp(ntile), tpw = (ntile + nwk - 1) / nwk;
  for (int i = 0; i < (int)(sizeof(kWgCfg) / sizeof(kWgCfg[0])); ++i) {
    const WgCfg c = kWgCfg[i];
    const int span = s * (c.wt - 1) + k;
    if (Ca * c.wt <= WTH * c.pmax && Cc * span <= WTH * c.qmax && span < 65536 && tpw <= c.ntmax &&
        wgrad_lds(Ca, Cc, k, s, c.wt) <= 64 * 1024)
      return i;
  }
  return -1;
}

static int wgrad_chunks(int n, int Lp, int wt) { return n * ((Lp + wt - 1) / wt); }

// blocks (= partials) of stage 1: one resident round, one 8-wave block per CU
// (the staging registers and the accumulators take up to 256 VGPRs)
static int wgrad_blocks(int nchunk) { return std::max(1, std::min(nchunk, 256)); }

// an upper bound over every configuration (the smallest chunk has the most)
size_t wgrad_scratch_bytes(int n, int Lp, int nw) {
  const size_t G = (size_t)wgrad_blocks(wgrad_chunks(n, Lp, 64));
  const size_t ngroup = (G + WG - 1) / WG;
  size_t a = ((G * nw * sizeof(float)) + 255) & ~(size_t)255;
  return a + ngroup * nw * sizeof(double);
}

struct WgP {
  const float* P;
  const float* Q;
  int Ca, Lp, Cc, Lq, n, k, s, pad, tchunks, nchunk, qs;
  float* partial;  // [blocks][Ca*Cc*k]
};

typedef float wf32x4 __attribute__((ext_vector_type(4)));

// one chunk's K steps for a wave with NT accumulator tiles: K steps slice,
// slice + ksp, ... of 4 time steps each; every operand read is unconditional
// (rows and columns past the GEMM read zero rows)
template <int NT, int WT>
__device__ __forceinline__ void wgrad_mma(const float* Ps, const float* Qs, const int* aoff, const int* boff, int s,
                                          int slice, int ksp, int lk, wf32x4* acc) {
  const int nkk = WT / 4 / ksp;
  const float* pa = Ps + 4 * slice + lk;
  const float* qb = Qs + s * (4 * slice + lk);
  const int da = 4 * ksp, db = 4 * ksp * s;
#pragma unroll 4
  for (int it = 0; it < nkk; ++it) {
#pragma unroll
    for (int u = 0; u < NT; ++u)
      acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[aoff[u]], qb[boff[u]], acc[u], 0, 0, 0);
    pa += da;
    qb += db;
  }
}

template <int WT, int PMAX, int QMAX, int NTMAX>
__global__ __launch_bounds__(WTH, 2) void wgrad_partial(WgP p) {
  extern __shared__ float lds[];
  constexpr int WPS = WT + 4;              // P row stride: rows 4 banks apart
  const int span = p.s * (WT - 1) + p.k;   // Q samples one chunk touches
  float* Ps = lds;                         // [Ca + 1][WPS], row Ca zero
  float* Qs = lds + (p.Ca + 1) * WPS;      // [Cc + 1][qs], row Cc zero
  const int tid = threadIdx.x;
  const int np = p.Ca * WT, nq = p.Cc * span;
  // this thread's Q elements (channel << 16 | position in the span), the
  // same for every chunk; -1 where the thread has none
  int qcu[QMAX];
#pragma unroll
  for (int i = 0; i < QMAX; ++i) {
    const int e = tid + WTH * i;
    const int c = e / span;
    qcu[i] = e < nq ? (c << 16) | (e - c * span) : -1;
  }
  // loads are unconditional, from addresses clamped into the tensors, so that
  // a chunk's loads are all in flight together; the staging store zeroes
  // what lies outside (rows past C, time past L, Q's zero padding)
  float pv[PMAX], qv[QMAX];
  auto fetch = [&](int chunk) {
    const int b = chunk / p.tchunks, t0 = (chunk - b * p.tchunks) * WT;
    const float* Pb = p.P + (int64_t)b * p.Ca * p.Lp;
    const float* Qb = p.Q + (int64_t)b * p.Cc * p.Lq;
#pragma unroll
    for (int i = 0; i < PMAX; ++i) {
      const int e = tid + WTH * i, a = min(e / WT, p.Ca - 1), t = min(t0 + e % WT, p.Lp - 1);
      pv[i] = Pb[(int64_t)a * p.Lp + t];
    }
    const int q0 = p.s * t0 - p.pad;
#pragma unroll
    for (int i = 0; i < QMAX; ++i) {
      const int c = qcu[i] >= 0 ? qcu[i] >> 16 : 0;
      const int q = min(max(q0 + (qcu[i] & 0xffff), 0), p.Lq - 1);
      qv[i] = Qb[(int64_t)c * p.Lq + q];
    }
  };
  // branch-free: a thread's slots past the chunk go to its own sink word, so
  // that every register of the batch is consumed on every path
  float* sink = Qs + (p.Cc + 1) * p.qs + tid;
  for (int e = tid; e < WPS; e += WTH) Ps[p.Ca * WPS + e] = 0.0f;
  for (int e = tid; e < p.qs; e += WTH) Qs[p.Cc * p.qs + e] = 0.0f;
  auto stage = [&](int chunk) {
    const int t0 = (chunk % p.tchunks) * WT, q0 = p.s * t0 - p.pad;
#pragma unroll
    for (int i = 0; i < PMAX; ++i) {
      const int e = tid + WTH * i;
      float* d = e < np ? Ps + (e / WT) * WPS + e % WT : sink;
      *d = t0 + e % WT < p.Lp ? pv[i] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < QMAX; ++i) {
      const int q = q0 + (qcu[i] & 0xffff);
      float* d = qcu[i] >= 0 ? Qs + (qcu[i] >> 16) * p.qs + (qcu[i] & 0xffff) : sink;
      *d = (q >= 0 && q < p.Lq) ? qv[i] : 0.0f;
    }
  };
  const int nk = p.Cc * p.k;               // GEMM columns
  const int MTa = (p.Ca + 15) / 16, NTn = (nk + 15) / 16, ntile = MTa * NTn;
  // wave groups splitting the K steps: as many as the idle waves allow
  const int ksp = wgrad_ksp(ntile);
  const int nwk = WNW / ksp;               // waves per group
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int slice = wave / nwk, wl = wave - slice * nwk;
  const int lr = lane & 15, lk = lane >> 4;
  // this lane's LDS offsets for each of its tiles (tile u of the wave is
  // wl + nwk u): A row a = 16 mt + lr, B column n = 16 nt + lr = (c, j)
  int aoff[NTMAX], boff[NTMAX];
#pragma unroll
  for (int u = 0; u < NTMAX; ++u) {
    const int tile = wl + nwk * u;
    const int mt = tile / NTn, nt = tile - mt * NTn;
    const int a = 16 * mt + lr, nn = 16 * nt + lr;
    aoff[u] = (tile < ntile && a < p.Ca) ? a * WPS : p.Ca * WPS;
    boff[u] = (tile < ntile && nn < nk) ? (nn / p.k) * p.qs + (nn % p.k) : p.Cc * p.qs;
  }
  wf32x4 acc[NTMAX];
#pragma unroll
  for (int u = 0; u < NTMAX; ++u) acc[u] = wf32x4{0.f, 0.f, 0.f, 0.f};
  // this wave's tiles: wl, wl + nwk, ... below ntile
  const int mytiles = wl < ntile ? (ntile - wl + nwk - 1) / nwk : 0;
  const int G = gridDim.x;
  const int c0 = (int)((int64_t)p.nchunk * blockIdx.x / G), c1 = (int)((int64_t)p.nchunk * (blockIdx.x + 1) / G);
  if (c0 < c1) fetch(c0);
  for (int chunk = c0; chunk < c1; ++chunk) {
    __syncthreads();  // the previous chunk's reads are done
    stage(chunk);
    __syncthreads();
    if (chunk + 1 < c1) fetch(chunk + 1);  // in flight during this chunk's MFMAs
#define GW_WG_CASE(N)                                                          \
  case N:                                                                      \
    if constexpr (N <= NTMAX) wgrad_mma<N, WT>(Ps, Qs, aoff, boff, p.s, slice, ksp, lk, acc); \
    break;
    switch (mytiles) {  // wave-uniform
      GW_WG_CASE(1)
      GW_WG_CASE(2)
      GW_WG_CASE(3)
      GW_WG_CASE(4)
      GW_WG_CASE(5)
      GW_WG_CASE(6)
      GW_WG_CASE(7)
      default: break;
    }
#undef GW_WG_CASE
  }
  // groups 1.. hand their accumulators to group 0 through LDS, which adds
  // them in group order
  if (ksp > 1) {
    float* xs = lds;  // [group - 1][wl][u][lane][4]
    const int tpw = (ntile + nwk - 1) / nwk;
    __syncthreads();
    if (slice > 0)
#pragma unroll
      for (int u = 0; u < NTMAX; ++u) {
        if (u >= tpw) break;
        float* d = xs + ((((slice - 1) * nwk + wl) * tpw + u) * 64 + lane) * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) d[r] = acc[u][r];
      }
    __syncthreads();
    if (slice == 0)
      for (int g = 1; g < ksp; ++g)
#pragma unroll
        for (int u = 0; u < NTMAX; ++u) {
          if (u >= tpw) break;
          const float* d = xs + ((((g - 1) * nwk + wl) * tpw + u) * 64 + lane) * 4;
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[u][r] += d[r];
        }
    if (slice > 0) return;
  }
  // D[row = 4 lk + r][col = lr] of tile u: weight (a, n)
  const int nw = p.Ca * nk;
  float* out = p.partial + (int64_t)blockIdx.x * nw;
#pragma unroll
  for (int u = 0; u < NTMAX; ++u) {
    const int tile = wl + nwk * u;
    if (tile >= ntile) break;
    const int mt = tile / NTn, nt = tile - mt * NTn;
    const int nn = 16 * nt + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = 16 * mt + 4 * lk + r;
      if (a < p.Ca && nn < nk) out[(int64_t)a * nk + nn] = acc[u][r];
    }
  }
}

// partials q of group g added in order q = 64 g, 64 g + 1, ...; the loads of
// 16 partials are issued together
__global__ __launch_bounds__(256) void wgrad_group(const float* partial, int nchunk, int nw,
                                                   double* mid) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  if (e >= nw) return;
  double acc = 0.0;
  const int q1 = min(nchunk, (g + 1) * WG);
  int q = g * WG;
  for (; q + 16 <= q1; q += 16) {
    float v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = partial[(int64_t)(q + j) * nw + e];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc += (double)v[j];
  }
  for (; q < q1; ++q) acc += (double)partial[(int64_t)q * nw + e];
  mid[(int64_t)g * nw + e] = acc;
}

__global__ __launch_bounds__(256) void wgrad_final(const double* mid, int ngroup, int nw,
                                                   float* dw) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nw) return;
  double acc = 0.0;
  int g = 0;
  for (; g + 8 <= ngroup; g += 8) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = mid[(int64_t)(g + j) * nw + e];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += v[j];
  }
  for (; g < ngroup; ++g) acc += mid[(int64_t)g * nw + e];
  dw[e] = (float)acc;
}

hipError_t launch_wgrad(const float* P, int Ca, int Lp, const float* Q, int Cc, int Lq, int n,
                        int k, int stride, int pad, void* scratch, float* dw, hipStream_t st) {
  const int cfg = wgrad_cfg(Ca, Cc, k, stride);
  const int nw = Ca * Cc * k;
  // every accumulator tile of the GEMM must have a register slot in its wave
  if (cfg < 0 || ((Ca + 15) / 16) * ((Cc * k + 15) / 16) > WNW * WTPW) return hipErrorInvalidValue;
  const int wt = kWgCfg[cfg].wt;
  WgP p;
  p.P = P;
  p.Q = Q;
  p.Ca = Ca;
  p.Lp = Lp;
  p.Cc = Cc;
  p.Lq = Lq;
  p.n = n;
  p.k = k;
  p.s = stride;
  p.pad = pad;
  p.tchunks = (Lp + wt - 1) / wt;
  p.nchunk = wgrad_chunks(n, Lp, wt);
  p.qs = wgrad_qs(stride * (wt - 1) + k);
  const int G = wgrad_blocks(p.nchunk);
  const int ngroup = (G + WG - 1) / WG;
  p.partial = reinterpret_cast<float*>(scratch);
  double* mid = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) +
                                          ((((size_t)G * nw * sizeof(float)) + 255) & ~(size_t)255));
  const size_t lds = wgrad_lds(Ca, Cc, k, stride, wt);
  switch (cfg) {
    case 0: hipLaunchKernelGGL((wgrad_partial<1024, 8, 24, 3>), dim3(G), dim3(WTH), lds, st, p); break;
    case 1: hipLaunchKernelGGL((wgrad_partial<512, 8, 24, 3>), dim3(G), dim3(WTH), lds, st, p); break;
    case 2: hipLaunchKernelGGL((wgrad_partial<256, 8, 24, 3>), dim3(G), dim3(WTH), lds, st, p); break;
    case 3: hipLaunchKernelGGL((wgrad_partial<128, 8, 12, 3>), dim3(G), dim3(WTH), lds, st, p); break;
    case 4: hipLaunchKernelGGL((wgrad_partial<64, 8, 12, 7>), dim3(G), dim3(WTH), lds, st, p); break;
    default: hipLaunchKernelGGL((wgrad_partial<64, 16, 24, 7>), dim3(G), dim3(WTH), lds, st, p); break;
  }
  hipLaunchKernelGGL(wgrad_group, dim3((nw + 255) / 256, ngroup), dim3(256), 0, st, p.partial,
                     G, nw, mid);
  hipLaunchKernelGGL(wgrad_final, dim3((nw + 255) / 256), dim3(256), 0, st, mid, ngroup, nw, dw);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Band-passed MSE.  With r = strain - noise and the DFT basis
// cos/sin(2 pi k t / W) of the band bins k_lo..k_hi,
//   ||P r||^2 = sum_k c_k (A_k^2 + B_k^2),  A_k = <r, cos_k>, B_k = <r, sin_k>,
//   P r[t]    = sum_k c_k (A_k cos_k[t] + B_k sin_k[t]),
// with c_k = 2/W (c_k = 1/W for k = 0 or k = W/2).  Angles are reduced
// exactly in integers, m = (k t mod W), before the sin/cos evaluation; the
// index advances by a constant per step (one compare and subtract) instead
// of a 64-bit division per sample.
// ---------------------------------------------------------------------------
// Projections A_k, B_k: block (x, y) takes bins [NB x, NB x + NB) of windows
// [NBW y, NBW y + NBW), so each residual sample is read once per NB bins
// and each basis value evaluated once per NBW windows.  A thread keeps FP64
// running sums over samples t = tid, tid + 256, ... for every (window, bin)
// of the block; one fixed block tree adds the threads' sums.
template <int NBW, int NB>
__global__ __launch_bounds__(256) void bp_project(const float* strain, const float* noise, int n, int nb, int W,
                                                  int k_lo, float* proj) {
  const int kb = blockIdx.x * NB, nbk = min(NB, nb - kb);
  const int b0 = blockIdx.y * NBW, nbw = min(NBW, n - b0);
  double acc[2 * NBW * NB];  // (A, B) of (window bb, bin q) at 2 (bb NB + q)
#pragma unroll
  for (int j = 0; j < 2 * NBW * NB; ++j) acc[j] = 0.0;
  const float twoW = 2.0f / (float)W;
  // m[q] = (k_lo + kb + q) t mod W for t = threadIdx.x, threadIdx.x + 256, ...
  int m[NB], step[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int64_t k = k_lo + kb + q;
    m[q] = (int)((k * threadIdx.x) % W);
    step[q] = (int)((k * 256) % W);
  }
  for (int t = threadIdx.x; t < W; t += 256) {
    float r[NBW];
#pragma unroll
    for (int bb = 0; bb < NBW; ++bb) {
      const int64_t o = (int64_t)(b0 + (bb < nbw ? bb : 0)) * W + t;
      r[bb] = strain[o] - noise[o];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      float sn, cs;
      sincospif(twoW * (float)m[q], &sn, &cs);
#pragma unroll
      for (int bb = 0; bb < NBW; ++bb) {
        acc[2 * (bb * NB + q)] += (double)(r[bb] * cs);
        acc[2 * (bb * NB + q) + 1] += (double)(r[bb] * sn);
      }
      m[q] += step[q];
      if (m[q] >= W) m[q] -= W;
    }
  }
  block_sum_n(acc);
  if (threadIdx.x < NBW * NB) {
    const int bb = threadIdx.x / NB, q = threadIdx.x - bb * NB;
    if (bb < nbw && q < nbk) {
      proj[((int64_t)(b0 + bb) * nb + kb + q) * 2 + 0] = (float)acc[2 * (bb * NB + q)];
      proj[((int64_t)(b0 + bb) * nb + kb + q) * 2 + 1] = (float)acc[2 * (bb * NB + q) + 1];
    }
  }
}

__device__ __forceinline__ float bin_weight(int k, int W) {
  return (k == 0 || 2 * k == W) ? 1.0f / (float)W : 2.0f / (float)W;
}

__global__ __launch_bounds__(256) void bp_loss(const float* proj, int n, int nb, int W, int k_lo,
                                               float* loss) {
  double s = 0.0, unused = 0.0;
  for (int e = threadIdx.x; e < n * nb; e += 256) {
    const int kk = e % nb;
    const double a = proj[2 * e], b = proj[2 * e + 1];
    s += (double)bin_weight(k_lo + kk, W) * (a * a + b * b);
  }
  block_sum2(s, unused);
  if (threadIdx.x == 0) loss[0] = (float)(s / ((double)n * W));
}

// dL/dnoise[t] = scale * sum_k c_k (A_k cos_k[t] + B_k sin_k[t]).  Block
// (x, y) covers samples [64 x, 64 x + 64) of windows [NBW y, NBW y + NBW);
// its four waves take a quarter of the bins each (in order), evaluate each
// bin's basis value once per sample for all of the windows, and their four
// partial sums are added in wave order.  The windows' projections are staged
// in LDS bin-major, [bin][window][2], so one bin's values for every window
// are read with 16-byte loads (the same address across the wave: broadcast).
template <int NBW>
__global__ __launch_bounds__(256) void bp_grad(const float* proj, int n, int nb, int W, int k_lo, float scale,
                                               float* dnoise) {
  static_assert(NBW % 2 == 0, "two windows per 16-byte load");
  extern __shared__ __attribute__((aligned(16))) float sp[];  // [nb][NBW][2], then [4][NBW][64] partials
  float* red = sp + (size_t)nb * NBW * 2;
  const int b0 = blockIdx.y * NBW, nbw = min(NBW, n - b0);
  for (int e = threadIdx.x; e < nb * NBW; e += 256) {
    const int kk = e / NBW, bb = e - kk * NBW;
    const bool on = bb < nbw;
    const int64_t o = ((int64_t)(b0 + (on ? bb : 0)) * nb + kk) * 2;
    sp[2 * e] = on ? proj[o] : 0.0f;
    sp[2 * e + 1] = on ? proj[o + 1] : 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + lane;
  const int k0 = nb * wave / 4, k1 = nb * (wave + 1) / 4;
  const float twoW = 2.0f / (float)W;
  float acc[NBW];
#pragma unroll
  for (int bb = 0; bb < NBW; ++bb) acc[bb] = 0.0f;
  if (t < W) {
    int m = (int)(((int64_t)(k_lo + k0) * t) % W);
    for (int kk = k0; kk < k1; ++kk) {
      float sn, cs;
      sincospif(twoW * (float)m, &sn, &cs);
      const float wk = bin_weight(k_lo + kk, W);
      const float4* q = reinterpret_cast<const float4*>(sp + kk * NBW * 2);
#pragma unroll
      for (int j = 0; j < NBW / 2; ++j) {
        const float4 v = q[j];  // (A, B) of windows 2j, 2j + 1
        acc[2 * j] = fmaf(wk, fmaf(v.x, cs, v.y * sn), acc[2 * j]);
        acc[2 * j + 1] = fmaf(wk, fmaf(v.z, cs, v.w * sn), acc[2 * j + 1]);
      }
      m += t;
      if (m >= W) m -= W;
    }
  }
#pragma unroll
  for (int bb = 0; bb < NBW; ++bb) red[(wave * NBW + bb) * 64 + lane] = acc[bb];
  __syncthreads();
  for (int e = threadIdx.x; e < NBW * 64; e += 256) {
    const int bb = e >> 6, ln = e & 63, tt = blockIdx.x * 64 + ln;
    if (bb < nbw && tt < W) {
      float v = red[bb * 64 + ln];
#pragma unroll
      for (int w = 1; w < 4; ++w) v += red[(w * NBW + bb) * 64 + ln];
      dnoise[(int64_t)(b0 + bb) * W + tt] = scale * v;
    }
  }
}

// The same gradient for bands too wide to stage: one window per block, the
// projections read from global memory.
__global__ __launch_bounds__(256) void bp_grad_wide(const float* proj, int nb, int W, int k_lo,
                                               float scale, float* dnoise) {
  const int b = blockIdx.y;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= W) return;
  const float* pr = proj + (int64_t)b * nb * 2;
  const float twoW = 2.0f / (float)W;
  // m = k t mod W for k = k_lo, k_lo + 1, ...: advances by t each bin
  int m = (int)(((int64_t)k_lo * t) % W);
  float acc = 0.0f;
  for (int kk = 0; kk < nb; ++kk) {
    const int k = k_lo + kk;
    float sn, cs;
    sincospif(twoW * (float)m, &sn, &cs);
    acc = fmaf(bin_weight(k, W), fmaf(pr[2 * kk], cs, pr[2 * kk + 1] * sn), acc);
    m += t;
    if (m >= W) m -= W;
  }
  dnoise[(int64_t)b * W + t] = scale * acc;
}

size_t bandpass_ws_floats(int n, int W, int nb) {
  (void)W;
  return (size_t)n * nb * 2;
}

hipError_t launch_bandpass(int n, int W, int k_lo, int k_hi, const float* strain,
                           const float* noise, float* proj, float* loss, float* dnoise,
                           hipStream_t st) {
  const int nb = k_hi - k_lo + 1;
  if (nb <= 0) return hipErrorInvalidValue;
  constexpr int PW = 4, PB = 1;  // windows and bins per projection block
  hipLaunchKernelGGL((bp_project<PW, PB>), dim3((nb + PB - 1) / PB, (n + PW - 1) / PW), dim3(256), 0, st, strain,
                     noise, n, nb, W, k_lo, proj);
  if (loss) hipLaunchKernelGGL(bp_loss, dim3(1), dim3(256), 0, st, proj, n, nb, W, k_lo, loss);
  if (dnoise) {
    const float scale = (float)(-2.0 / ((double)n * W));
    // windows per block: all of a training batch's when the projections fit
    // in LDS, else fewer; LDS = projections + the four waves' partial sums
    const size_t per = sizeof(float) * (2 * (size_t)nb + 4 * 64);
    if (32 * per <= 64 * 1024)
      hipLaunchKernelGGL(bp_grad<32>, dim3((W + 63) / 64, (n + 31) / 32), dim3(256), 32 * per, st, proj, n, nb, W,
                         k_lo, scale, dnoise);
    else if (2 * per <= 64 * 1024)
      hipLaunchKernelGGL(bp_grad<2>, dim3((W + 63) / 64, (n + 1) / 2), dim3(256), 2 * per, st, proj, n, nb, W,
                         k_lo, scale, dnoise);
    else
      hipLaunchKernelGGL(bp_grad_wide, dim3((W + 255) / 256, n), dim3(256), 0, st, proj, nb, W, k_lo, scale,
                         dnoise);
  }
  return hipGetLastError();
}

}  // namespace gw
