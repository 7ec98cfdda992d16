// Incremental DeepClean forward over per-stream activation caches.
//
// The paper's stateful model turns each request into the full window, which
// the static model then processes from scratch (App. B.1).  Between two
// requests of a stream the window only slides: when the snapshot has advanced
// by a multiple of the network's total stride (16), every layer's activation
// grid slides by whole positions, and an activation keeps its value unless
// its receptive field reaches the newest samples or the window's left edge
// (whose zero padding now replaces what used to be real samples).  A cache
// therefore holds every layer's activations of the stream's last window, as
// rings (layer l: C_{l+1} x L_l, BF16; the output conv: FP32), and an update
// recomputes only each layer's dirty positions: a left zone [0, zl) and a
// right band [zr, L) (cache_band in internal.h).  The rest is reused by
// advancing the ring heads.
//
// Arithmetic per output value: input activations BF16 (the ring's BF16
// shadow for the first layer), weights rounded to BF16 (nearest even), one
// FP32 fused multiply-add chain over (input channel, tap) in that order,
// then the folded normalisation and tanh in FP32, stored as BF16 (FP32 for
// the noise).  Each value depends only on its inputs, never on which
// positions a call recomputes, so an incremental update is bitwise equal to
// recomputing the whole window with the same kernel.
#include "internal.h"

namespace gw {

namespace {

__device__ __forceinline__ uint16_t bf16_of(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  return (uint16_t)((u & 0x7fffffffu) > 0x7f800000u ? ((u >> 16) | 0x40u) : r);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

}  // namespace

// One layer over the dirty positions of every item: grid x = chunks of 64
// dirty positions, y = item; thread (wave w, lane q) computes position
// 64 blockIdx.x + q for output channels w, w + 4, ...
__global__ __launch_bounds__(256) void cache_layer_kernel(const CacheItem* items, const void* arena, CacheLayerP P) {
  const CacheItem it = items[blockIdx.y];
  int zl, zr;
  cache_band(P.geo, P.layer, it.shift, P.W, &zl, &zr);
  const int Lout = P.geo[P.layer].Lout, Lin = P.geo[P.layer].Lin;
  const int nd = zl + (Lout - zr);
  const int q = blockIdx.x * 64 + (threadIdx.x & 63);
  if (q >= nd) return;
  const int pos = q < zl ? q : zr + (q - zl);
  const CacheGeo& g = P.geo[P.layer];
  // input: the snapshot's BF16 shadow (first layer) or the previous layer's ring
  const uint16_t* in;
  int ihead;
  if (P.layer == 0) {
    in = reinterpret_cast<const uint16_t*>(arena) + it.shadow;
    ihead = it.in_head;
  } else {
    in = reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(it.cache) + P.off[P.layer - 1]);
    ihead = it.T / P.geo[P.layer - 1].f;
  }
  const int ohead = it.T / g.f;
  int oslot = ohead + pos;
  if (oslot >= Lout) oslot -= Lout;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  for (int o = wave; o < g.co; o += 4) {
    float acc = 0.0f;
    for (int i = 0; i < g.ci; ++i) {
      const uint16_t* row = in + (int64_t)i * Lin;
      for (int j = 0; j < g.k; ++j) {
        int t;
        float wv;
        if (g.type == 0) {
          t = g.s * pos - g.p + j;
          wv = P.w[((int64_t)o * g.ci + i) * g.k + j];
        } else {
          const int num = pos + g.p - j;  // pos = s t - p + j
          if (num < 0 || num % g.s) continue;
          t = num / g.s;
          wv = P.w[((int64_t)i * g.co + o) * g.k + j];
        }
        if (t < 0 || t >= Lin) continue;
        int sl = ihead + t;
        if (sl >= Lin) sl -= Lin;
        acc = fmaf(bf16_val(row[sl]), bf16_val(bf16_of(wv)), acc);
      }
    }
    const float v = fmaf(acc, P.scale[o], P.shift[o]);
    char* out = reinterpret_cast<char*>(it.cache) + P.off[P.layer];
    if (g.bn)
      reinterpret_cast<uint16_t*>(out)[(int64_t)o * Lout + oslot] = bf16_of(tanhf(v));
    else
      reinterpret_cast<float*>(out)[(int64_t)o * Lout + oslot] = v;
  }
}

// The window's outputs from the cached noise ring: the dense noise window
// (when requested) and the clean output strain - noise over the request's
// span [W - s - delay, W - delay).  grid x = chunks of 256 positions, y = item.
__global__ __launch_bounds__(256) void cache_emit_kernel(const CacheItem* items, int W, size_t off_noise,
                                                         const float* strain, float* noise, float* clean) {
  const CacheItem it = items[blockIdx.y];
  const float* ring = reinterpret_cast<const float*>(reinterpret_cast<const char*>(it.cache) + off_noise);
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= W) return;
  int sl = it.T + k;
  if (sl >= W) sl -= W;
  const float v = ring[sl];
  if (noise) noise[(int64_t)blockIdx.y * W + k] = v;
  if (clean) {
    const int t0 = W - it.s - it.delay;
    if (k >= t0 && k < t0 + it.s) clean[it.out + (k - t0)] = strain[it.out + (k - t0)] - v;
  }
}

hipError_t launch_cache_layer(const CacheItem* items, int n, const void* arena, const CacheLayerP& P, int max_dirty,
                              hipStream_t st) {
  if (n < 1 || max_dirty < 0) return hipErrorInvalidValue;
  if (max_dirty == 0) return hipSuccess;
  hipLaunchKernelGGL(cache_layer_kernel, dim3((max_dirty + 63) / 64, n), dim3(256), 0, st, items, arena, P);
  return hipGetLastError();
}

hipError_t launch_cache_emit(const CacheItem* items, int n, int W, size_t off_noise, const float* strain,
                             float* noise, float* clean, hipStream_t st) {
  if (n < 1 || W < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cache_emit_kernel, dim3((W + 255) / 256, n), dim3(256), 0, st, items, W, off_noise, strain,
                     noise, clean);
  return hipGetLastError();
}

}  // namespace gw
