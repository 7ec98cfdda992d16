// Training-step kernels for the DeepClean-shaped network: batch-statistics
// normalisation (forward and backward, fused with tanh and its derivative),
// per-channel reductions, deterministic weight gradients, and the band-passed
// MSE loss.  Every reduction has a fixed combination order (chunk partials in
// FP64, then a fixed tree), so results are bitwise reproducible and do not
// depend on scheduling.
#include "internal.h"

#include <algorithm>

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
  for (int r = 0; r < RCHUNK / 256; ++r) {
    const int64_t e = (int64_t)q * RCHUNK + r * 256 + threadIdx.x;
    if (e >= N) break;
    const int64_t b = e / p.L, t = e - b * p.L;
    const int64_t idx = (b * p.C + c) * p.L + t;
    if (MODE == R_STATS) {
      const double v = p.x[idx];
      s0 += v;
      s1 += v * v;
    } else if (MODE == R_BNBWD) {
      const float av = p.a[idx];
      const float dh = p.x[idx] * (1.0f - av * av);
      const float xh = (p.z[idx] - mu) * is;
      s0 += (double)dh;
      s1 += (double)dh * (double)xh;
    } else {
      s0 += (double)p.x[idx];
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

// a = tanh(gamma (z - mean) invstd + beta)
__global__ __launch_bounds__(256) void bn_apply_tanh_kernel(const float* z, const float* mean,
                                                            const float* invstd, const float* gamma,
                                                            const float* beta, float* a, int C,
                                                            int L, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int c = (int)((e / L) % C);
  a[e] = tanhf(fmaf(gamma[c], (z[e] - mean[c]) * invstd[c], beta[c]));
}

hipError_t launch_bn_apply_tanh(const float* z, const float* mean, const float* invstd,
                                const float* gamma, const float* beta, float* a, int n, int C,
                                int L, hipStream_t st) {
  const int64_t total = (int64_t)n * C * L;
  hipLaunchKernelGGL(bn_apply_tanh_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     z, mean, invstd, gamma, beta, a, C, L, total);
  return hipGetLastError();
}

// dz = gamma invstd (dh - sum(dh)/N - xhat sum(dh xhat)/N), dh = g (1 - a^2)
__global__ __launch_bounds__(256) void bn_tanh_bwd_kernel(const float* g, const float* a,
                                                          const float* z, const float* mean,
                                                          const float* invstd, const float* gamma,
                                                          const float* sdh, const float* sdhx,
                                                          float* dz, int C, int L, int64_t total,
                                                          float invN) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int c = (int)((e / L) % C);
  const float av = a[e];
  const float dh = g[e] * (1.0f - av * av);
  const float xh = (z[e] - mean[c]) * invstd[c];
  dz[e] = gamma[c] * invstd[c] * (dh - sdh[c] * invN - xh * (sdhx[c] * invN));
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
  const int64_t total = (int64_t)n * C * L;
  hipLaunchKernelGGL(bn_tanh_bwd_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g,
                     a, z, mean, invstd, gamma, dbeta, dgamma, dz, C, L, total,
                     (float)(1.0 / ((double)n * L)));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weight gradient: dw[a][c][j] = sum_b sum_t P[b][a][t] * Q[b][c][s t - p + j]
// (Q zero outside [0, Lq)).  For a conv layer P = dL/dz (a = out channel) and
// Q = layer input; for a transposed layer P = layer input and Q = dL/dz.
// Stage 1, a split-K GEMM on the matrix cores: D[a][n] (n = c k + j) summed
// over K = (batch item, time).  Block g walks a fixed run of chunks (batch
// item, 64 time steps) in order; per chunk it stages the chunk of P and the
// matching window of Q in LDS (FP32) and runs v_mfma_f32_16x16x4_f32 (exact
// FP32 products, FP32 accumulation) over 16 K steps of 4 time steps; its
// accumulators stay in registers across its chunks and are written once as
// block g's FP32 partial.  Stages 2 and 3 add the partials of every weight in
// a fixed two-level tree (groups of 64 partials, then the groups) in FP64.
// ---------------------------------------------------------------------------
static constexpr int WT = 64;   // time steps per chunk
static constexpr int WG = 64;   // partials per group of the reduction tree
static constexpr int WPS = WT + 1;  // LDS row stride of the P chunk (odd: no bank conflicts down a column)
static constexpr int WNW = 8;       // waves per block
static constexpr int WTPW = 7;      // most accumulator tiles per wave

int wgrad_chunks(int n, int Lp) { return n * ((Lp + WT - 1) / WT); }

// blocks (= partials) of stage 1: enough to fill the chip, few enough that
// the partials of a large layer stay near 16 MB
static int wgrad_blocks(int n, int Lp, int nw) {
  const int nchunk = wgrad_chunks(n, Lp);
  const int cap = std::max(256, (int)std::min<int64_t>(1024, ((int64_t)4 << 20) / std::max(nw, 1)));
  return std::max(1, std::min(nchunk, cap));
}

size_t wgrad_scratch_bytes(int n, int Lp, int nw) {
  const size_t G = (size_t)wgrad_blocks(n, Lp, nw);
  const size_t ngroup = (G + WG - 1) / WG;
  size_t a = ((G * nw * sizeof(float)) + 255) & ~(size_t)255;
  return a + ngroup * nw * sizeof(double);
}

struct WgP {
  const float* P;
  const float* Q;
  int Ca, Lp, Cc, Lq, n, k, s, pad, tchunks, nchunk;
  float* partial;  // [blocks][Ca*Cc*k]
};

typedef float wf32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64 * WNW, 2) void wgrad_partial(WgP p) {
  extern __shared__ float lds[];
  const int span = p.s * (WT - 1) + p.k;  // Q samples touched by one chunk
  float* Ps = lds;                        // [Ca][WPS]
  float* Qs = lds + p.Ca * WPS;           // [Cc][span]
  const int nk = p.Cc * p.k;              // GEMM columns
  const int MTa = (p.Ca + 15) / 16, NTn = (nk + 15) / 16, ntile = MTa * NTn;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  // this lane's LDS offsets for each of its tiles (tile u of the wave is
  // wave + WNW u): A row a = 16 mt + lr, B column n = 16 nt + lr = (c, j)
  int aoff[WTPW], boff[WTPW];
#pragma unroll
  for (int u = 0; u < WTPW; ++u) {
    const int tile = wave + WNW * u;
    const int mt = tile / NTn, nt = tile - mt * NTn;
    const int a = 16 * mt + lr, nn = 16 * nt + lr;
    aoff[u] = (tile < ntile && a < p.Ca) ? a * WPS : -1;
    boff[u] = (tile < ntile && nn < nk) ? (nn / p.k) * span + (nn % p.k) : -1;
  }
  wf32x4 acc[WTPW];
#pragma unroll
  for (int u = 0; u < WTPW; ++u) acc[u] = wf32x4{0.f, 0.f, 0.f, 0.f};
  const int G = gridDim.x;
  const int c0 = (int)((int64_t)p.nchunk * blockIdx.x / G), c1 = (int)((int64_t)p.nchunk * (blockIdx.x + 1) / G);
  for (int chunk = c0; chunk < c1; ++chunk) {
    const int b = chunk / p.tchunks, t0 = (chunk % p.tchunks) * WT;
    const float* Pb = p.P + (int64_t)b * p.Ca * p.Lp;
    const float* Qb = p.Q + (int64_t)b * p.Cc * p.Lq;
    __syncthreads();  // the previous chunk's reads are done
    for (int e = threadIdx.x; e < p.Ca * WT; e += 64 * WNW) {
      const int a = e / WT, t = e - a * WT;
      Ps[a * WPS + t] = (t0 + t < p.Lp) ? Pb[(int64_t)a * p.Lp + t0 + t] : 0.0f;
    }
    const int q0 = p.s * t0 - p.pad;
    for (int e = threadIdx.x; e < p.Cc * span; e += 64 * WNW) {
      const int c = e / span, u = e - c * span;
      const int q = q0 + u;
      Qs[e] = (q >= 0 && q < p.Lq) ? Qb[(int64_t)c * p.Lq + q] : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < WT / 4; ++kk) {
      const int t = 4 * kk + lk;  // this lane's K index
#pragma unroll
      for (int u = 0; u < WTPW; ++u) {
        if (wave + WNW * u >= ntile) break;  // wave-uniform
        const float av = aoff[u] >= 0 ? Ps[aoff[u] + t] : 0.0f;
        const float bv = boff[u] >= 0 ? Qs[boff[u] + p.s * t] : 0.0f;
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[u], 0, 0, 0);
      }
    }
  }
  // D[row = 4 lk + r][col = lr] of tile u: weight (a, n)
  const int nw = p.Ca * nk;
  float* out = p.partial + (int64_t)blockIdx.x * nw;
#pragma unroll
  for (int u = 0; u < WTPW; ++u) {
    const int tile = wave + WNW * u;
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

__global__ __launch_bounds__(256) void wgrad_group(const float* partial, int nchunk, int nw,
                                                   double* mid) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  if (e >= nw) return;
  double acc = 0.0;
  const int q1 = min(nchunk, (g + 1) * WG);
  for (int q = g * WG; q < q1; ++q) acc += (double)partial[(int64_t)q * nw + e];
  mid[(int64_t)g * nw + e] = acc;
}

__global__ __launch_bounds__(256) void wgrad_final(const double* mid, int ngroup, int nw,
                                                   float* dw) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nw) return;
  double acc = 0.0;
  for (int g = 0; g < ngroup; ++g) acc += mid[(int64_t)g * nw + e];
  dw[e] = (float)acc;
}

hipError_t launch_wgrad(const float* P, int Ca, int Lp, const float* Q, int Cc, int Lq, int n,
                        int k, int stride, int pad, void* scratch, float* dw, hipStream_t st) {
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
  p.tchunks = (Lp + WT - 1) / WT;
  p.nchunk = wgrad_chunks(n, Lp);
  const int nw = Ca * Cc * k;
  const int G = wgrad_blocks(n, Lp, nw);
  const int ngroup = (G + WG - 1) / WG;
  p.partial = reinterpret_cast<float*>(scratch);
  double* mid = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) +
                                          ((((size_t)G * nw * sizeof(float)) + 255) & ~(size_t)255));
  const int span = stride * (WT - 1) + k;
  const size_t lds = sizeof(float) * ((size_t)Ca * WPS + (size_t)Cc * span);
  // every accumulator tile of the GEMM must have a register slot in its wave
  if (lds > 64 * 1024 || ((Ca + 15) / 16) * ((Cc * k + 15) / 16) > WNW * WTPW) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wgrad_partial, dim3(G), dim3(64 * WNW), lds, st, p);
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
__global__ __launch_bounds__(256) void bp_project(const float* strain, const float* noise, int W,
                                                  int k_lo, float* proj) {
  const int b = blockIdx.y, kk = blockIdx.x, k = k_lo + kk;
  const float* sr = strain + (int64_t)b * W;
  const float* nr = noise + (int64_t)b * W;
  double sa = 0.0, sb = 0.0;
  const float twoW = 2.0f / (float)W;
  // m = k t mod W for t = threadIdx.x, threadIdx.x + 256, ...
  int m = (int)(((int64_t)k * threadIdx.x) % W);
  const int step = (int)(((int64_t)k * 256) % W);
  for (int t = threadIdx.x; t < W; t += 256) {
    const float r = sr[t] - nr[t];
    float sn, cs;
    sincospif(twoW * (float)m, &sn, &cs);
    sa += (double)(r * cs);
    sb += (double)(r * sn);
    m += step;
    if (m >= W) m -= W;
  }
  block_sum2(sa, sb);
  if (threadIdx.x == 0) {
    proj[((int64_t)b * gridDim.x + kk) * 2 + 0] = (float)sa;
    proj[((int64_t)b * gridDim.x + kk) * 2 + 1] = (float)sb;
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

__global__ __launch_bounds__(256) void bp_grad(const float* proj, int nb, int W, int k_lo,
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
  hipLaunchKernelGGL(bp_project, dim3(nb, n), dim3(256), 0, st, strain, noise, W, k_lo, proj);
  if (loss) hipLaunchKernelGGL(bp_loss, dim3(1), dim3(256), 0, st, proj, n, nb, W, k_lo, loss);
  if (dnoise)
    hipLaunchKernelGGL(bp_grad, dim3((W + 255) / 256, n), dim3(256), 0, st, proj, nb, W, k_lo,
                       (float)(-2.0 / ((double)n * W)), dnoise);
  return hipGetLastError();
}

}  // namespace gw
