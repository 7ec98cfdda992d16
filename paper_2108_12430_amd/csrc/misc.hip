// Bandwidth-bound helpers: snapshot ring update, zero fill, normalisation
// folding, and the classifier head (global average pool + linear).
#include "internal.h"

namespace gw {

// Snapshot update (the stateful model's request): item i writes its [C][s]
// block of new samples at ring positions head, head+1, ... (mod W) of every
// channel, both as the exact FP32 value and as its BF16 shadow.  After the
// write the oldest sample sits at (head + s) mod W, so the ring read from
// there is "previous snapshot ++ new samples, last W kept".
// Grid: x = chunks of 1024 elements of the largest C*s, y = item.
__global__ __launch_bounds__(256) void snapshot_kernel(char* arena, const Item* items,
                                                       const float* samples) {
  const Item it = items[blockIdx.y];
  const int total = it.C * it.s;
  float* ring = reinterpret_cast<float*>(arena) + it.ring;
  uint16_t* sh = reinterpret_cast<uint16_t*>(arena) + it.shadow;
  const float* src = samples + it.src;
  const int e0 = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (e0 >= total) return;
  const bool vec = ((it.s | it.head | it.W) & 3) == 0 && (it.src & 3) == 0 && (it.ring & 3) == 0 &&
                   (it.shadow & 3) == 0 && (reinterpret_cast<uintptr_t>(samples) & 15) == 0;
  if (vec) {
    // four consecutive samples of one channel; head, s and W are multiples of
    // 4, so the group never straddles the wrap point
    const int c = e0 / it.s, q = e0 - c * it.s;
    int ph = it.head + q;
    if (ph >= it.W) ph -= it.W;
    const float4 v = *reinterpret_cast<const float4*>(src + e0);
    *reinterpret_cast<float4*>(ring + (int64_t)c * it.W + ph) = v;
    ushort4 h;
    h.x = f2bf(v.x);
    h.y = f2bf(v.y);
    h.z = f2bf(v.z);
    h.w = f2bf(v.w);
    *reinterpret_cast<ushort4*>(sh + (int64_t)c * it.W + ph) = h;
  } else {
    for (int e = e0; e < min(e0 + 4, total); ++e) {
      const int c = e / it.s, q = e - c * it.s;
      int ph = it.head + q;
      if (ph >= it.W) ph -= it.W;
      const float v = src[e];
      ring[(int64_t)c * it.W + ph] = v;
      sh[(int64_t)c * it.W + ph] = f2bf(v);
    }
  }
}

hipError_t launch_snapshot(void* arena, const Item* items, int n, int max_cs, const float* samples,
                           hipStream_t st) {
  dim3 grid((max_cs + 1023) / 1024, n);
  hipLaunchKernelGGL(snapshot_kernel, grid, dim3(256), 0, st, reinterpret_cast<char*>(arena), items,
                     samples);
  return hipGetLastError();
}

// Zero fill with vector stores (used instead of a memset so that callers may
// capture the work in a graph).  dst and bytes are multiples of 16.
__global__ __launch_bounds__(256) void fill_zero_kernel(uint4* dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
    dst[i] = make_uint4(0, 0, 0, 0);
}

hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t st) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n16 + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     reinterpret_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

// Inference-time normalisation folded into a per-channel affine map applied
// to the raw accumulator: scale = gamma / sqrt(var + eps),
// shift = beta + scale * (bias - mean).  Without normalisation: scale = 1,
// shift = bias.
__global__ void fold_bn_kernel(const float* b, const float* gamma, const float* beta,
                               const float* mean, const float* var, float* scale, float* shift,
                               int C) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= C) return;
  if (gamma) {
    const float sc = gamma[o] / sqrtf(var[o] + 1e-5f);
    scale[o] = sc;
    shift[o] = fmaf(sc, b[o] - mean[o], beta[o]);
  } else {
    scale[o] = 1.0f;
    shift[o] = b[o];
  }
}

hipError_t launch_fold_bn(const float* b, const float* gamma, const float* beta, const float* mean,
                          const float* var, float* scale, float* shift, int C, hipStream_t st) {
  hipLaunchKernelGGL(fold_bn_kernel, dim3((C + 255) / 256), dim3(256), 0, st, b, gamma, beta, mean,
                     var, scale, shift, C);
  return hipGetLastError();
}

// Classifier head: logit[b] = bias + (1/L) sum_c sum_t w[c] a[b][c][t]
// (= bias + w . mean_t a).  One block per window; every lane accumulates a
// fixed strided subset of the window with independent loads, then the block
// combines the lane sums in a fixed tree, so the result does not depend on
// scheduling.
__global__ __launch_bounds__(256) void gap_linear_kernel(const float* a, const float* w,
                                                         const float* bias, float* logits, int C,
                                                         int L) {
  __shared__ float part[256];
  const int b = blockIdx.x;
  const float* ab = a + (int64_t)b * C * L;
  const int total = C * L;
  float s = 0.0f;
  for (int e = threadIdx.x; e < total; e += 256) s = fmaf(w[e / L], ab[e], s);
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) logits[b] = part[0] / (float)L + bias[0];
}

hipError_t launch_gap_linear(const float* a, const float* w, const float* b, float* logits, int n,
                             int C, int L, hipStream_t st) {
  hipLaunchKernelGGL(gap_linear_kernel, dim3(n), dim3(256), 0, st, a, w, b, logits, C, L);
  return hipGetLastError();
}

}  // namespace gw

namespace gw {

// Window fetch: materialise each item's logical window (oldest sample first)
// from its ring, either as FP32 (out) or from the BF16 shadow (outh).
__global__ __launch_bounds__(256) void gather_kernel(const char* arena, const Item* items, int C,
                                                     int W, float* out, uint16_t* outh) {
  const Item it = items[blockIdx.y];
  const int64_t total = (int64_t)C * W;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int c = (int)(e / W), t = (int)(e - (int64_t)c * W);
  int ph = it.head + t;
  if (ph >= W) ph -= W;
  const int64_t dst = (int64_t)blockIdx.y * total + e;
  if (out) out[dst] = reinterpret_cast<const float*>(arena)[it.ring + (int64_t)c * W + ph];
  if (outh) outh[dst] = reinterpret_cast<const uint16_t*>(arena)[it.shadow + (int64_t)c * W + ph];
}

hipError_t launch_gather(const void* arena, const Item* items, int n, int C, int W, float* out,
                         uint16_t* outh, hipStream_t st) {
  const int64_t total = (int64_t)C * W;
  dim3 grid((unsigned)((total + 255) / 256), n);
  hipLaunchKernelGGL(gather_kernel, grid, dim3(256), 0, st, reinterpret_cast<const char*>(arena),
                     items, C, W, out, outh);
  return hipGetLastError();
}

}  // namespace gw

namespace gw {

__global__ __launch_bounds__(256) void zero_floats_kernel(float* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = 0.0f;
}

hipError_t launch_zero_floats(float* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_floats_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, n);
  return hipGetLastError();
}

}  // namespace gw

namespace gw {

__global__ void gap_finalize_kernel(const float* part, int nblk, const float* bias, float* logits, int n,
                                    int L) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= n) return;
  float s = 0.0f;
  for (int k = 0; k < nblk; ++k) s += part[(int64_t)b * nblk + k];
  logits[b] = s / (float)L + bias[0];
}

hipError_t launch_gap_finalize(const float* part, int nblk, const float* bias, float* logits, int n,
                               int L, hipStream_t st) {
  hipLaunchKernelGGL(gap_finalize_kernel, dim3((n + 255) / 256), dim3(256), 0, st, part, nblk, bias, logits,
                     n, L);
  return hipGetLastError();
}

}  // namespace gw

namespace gw {

// Overlap averaging of successive predictions of one stream (App. B.2 notes
// that the output segments of successive windows overlap and could be
// aggregated).  Item fields: s = stride, out = offset of the item's packed
// [s] output block, src = offset (floats) of its state block [depth][s],
// head = request index k mod depth, C = windows averaged, min(depth, k + 1).
// State slot j accumulates the output of the request whose index is j mod
// depth.  Window k contributes to outputs k .. k + depth - 1: to output k + i
// its samples at W - (depth - i) s + t.  One thread per output sample t, so
// the depth slots of a sample are updated by one thread in order.
__global__ __launch_bounds__(256) void overlap_average_kernel(const Item* items, int W, int depth,
                                                              const float* noise, float* state,
                                                              const float* strain, float* clean, float* avg) {
  const Item it = items[blockIdx.y];
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= it.s) return;
  const float* P = noise + (int64_t)blockIdx.y * W;
  float* R = state + it.src;
  for (int i = 0; i < depth; ++i) {
    int slot = it.head + i;
    if (slot >= depth) slot -= depth;
    R[(int64_t)slot * it.s + t] += P[W - (depth - i) * it.s + t];
  }
  float* r0 = R + (int64_t)it.head * it.s + t;
  const float v = *r0 / (float)it.C;
  *r0 = 0.0f;  // the slot starts over for output k + depth
  const int64_t o = it.out + t;
  if (avg) avg[o] = v;
  if (clean) clean[o] = strain[o] - v;
}

hipError_t launch_overlap_average(const Item* items, int n, int max_s, int W, int depth, const float* noise,
                                  float* state, const float* strain, float* clean, float* avg, hipStream_t st) {
  dim3 grid((unsigned)((max_s + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL(overlap_average_kernel, grid, dim3(256), 0, st, items, W, depth, noise, state, strain, clean,
                     avg);
  return hipGetLastError();
}

}  // namespace gw

namespace gw {

// Streaming decimation by 2 with a causal FIR (the end-to-end ensemble's
// step from the cleaned 4096 Hz strain to BBHnet's 2048 Hz input):
// y[m] = sum_j h[j] x[2m + 1 - j] over the stream's samples, zero before its
// first.  One block per (item, channel); the K - 1 inputs before the new
// block come from the item's history, which the block then advances.
__global__ __launch_bounds__(256) void decimate2_kernel(int n, int s, int K, const float* taps, const float* x,
                                                        float* hist, float* y) {
  const int i = blockIdx.x, c = blockIdx.y, C = gridDim.y;
  const float* xb = x + ((int64_t)c * n + i) * s;           // the s new samples
  float* hb = hist + ((int64_t)i * C + c) * (K - 1);        // the K - 1 before them, oldest first
  float* yb = y + ((int64_t)i * C + c) * (s / 2);
  for (int m = threadIdx.x; m < s / 2; m += 256) {
    float acc = 0.0f;
    for (int j = 0; j < K; ++j) {
      const int v = 2 * m + 1 - j;  // input index relative to the new block
      acc = fmaf(taps[j], v >= 0 ? xb[v] : hb[K - 1 + v], acc);
    }
    yb[m] = acc;
  }
  // next history: the last K - 1 samples of (history, block); read before
  // any thread writes (K - 1 <= 256: one sample per thread)
  float h = 0.0f;
  const int e = threadIdx.x;
  if (e < K - 1) {
    const int v = s - (K - 1) + e;
    h = v >= 0 ? xb[v] : hb[K - 1 + v];
  }
  __syncthreads();
  if (e < K - 1) hb[e] = h;
}

hipError_t launch_decimate2(int n, int C, int s, int K, const float* taps, const float* x, float* hist, float* y,
                            hipStream_t st) {
  hipLaunchKernelGGL(decimate2_kernel, dim3((unsigned)n, (unsigned)C), dim3(256), 0, st, n, s, K, taps, x, hist, y);
  return hipGetLastError();
}

}  // namespace gw
