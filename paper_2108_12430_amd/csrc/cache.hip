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
// Arithmetic per output value: BF16 input activations (the ring's BF16
// shadow for the first layer) and the model's BF16 weights on the matrix
// cores with FP32 accumulation, then the folded normalisation and tanh in
// FP32, stored as BF16 (FP32 for the noise).  Each value depends only on its
// inputs, never on which positions a call recomputes, so an incremental
// update is bitwise equal to recomputing the whole window with the same
// kernel.
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

typedef __bf16 cbf16x8 __attribute__((ext_vector_type(8)));
typedef float cf32x4 __attribute__((ext_vector_type(4)));

// One layer over the dirty positions of every item, as an implicit GEMM on
// the matrix cores: D[o][c] = sum_kappa A[o][kappa] B[kappa][c] with A the
// model's BF16 weight fragments (v_mfma_f32_16x16x32_bf16 lane order, K =
// tap x input channel, transposed layers as two phases of 4 taps) and B the
// input window staged in LDS as [position][channel].  Column c is output
// position c of a conv, or input-aligned position m of a transposed conv
// (outputs 2m and 2m + 1).  grid x = chunks of 64 columns (the left zone's
// chunks, then the right band's), y = item.  An MFMA result element depends
// only on its own row of A and column of B, so a value comes out bitwise the
// same whichever chunk computes it; a chunk may therefore recompute a few
// clean positions next to a dirty range (with the same bits).
template <int CIP, int NPH>
__global__ __launch_bounds__(256) void cache_mfma_kernel(const CacheItem* items, const void* arena, CacheLayerP P) {
  constexpr int RS = CIP + 8;                          // LDS row stride (16-byte multiple, skews banks)
  constexpr int NC = kCacheChunk;                      // columns per block
  constexpr int ROWSMAX = 2 * (NC - 1) + 7;            // a stride-2 k7 conv's window
  __shared__ __attribute__((aligned(16))) uint16_t tile[ROWSMAX * RS];
  const CacheItem it = items[blockIdx.y];
  const CacheGeo& g = P.geo[P.layer];
  int zl, zr;
  cache_band(P.geo, P.layer, it.shift, P.W, &zl, &zr);
  constexpr int CS = NPH == 2 ? 1 : 0;                 // log2 outputs per column
  const int ncols = g.Lout >> CS;
  const int la = (zl + (1 << CS) - 1) >> CS;           // left columns [0, la)
  const int ra = zr >> CS;                             // right columns [ra, ncols)
  const int nl = (la + NC - 1) / NC, nr = (ncols - ra + NC - 1) / NC;
  const int bidx = blockIdx.x;
  if (bidx >= nl + nr) return;  // block-uniform
  const int c0 = bidx < nl ? bidx * NC : ra + (bidx - nl) * NC;
  constexpr int KT = NPH == 2 ? 4 : 7;                // taps per column (k7; transposed: 4 per phase)
  constexpr int KS = (KT * CIP + 31) / 32;             // K steps
  const int SC = NPH == 2 ? 1 : g.s;
  const int t0 = NPH == 2 ? c0 - 1 : SC * c0 - g.p;   // transposed k7 s2 p3: column m reads m - 1 .. m + 2
  const int rows = SC * (NC - 1) + KT;
  const uint16_t* in;
  int ihead;
  if (P.layer == 0) {
    in = reinterpret_cast<const uint16_t*>(arena) + it.shadow;
    ihead = it.in_head;
  } else {
    in = reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(it.cache) + P.off[P.layer - 1]);
    ihead = it.T / P.geo[P.layer - 1].f;
  }
  // stage input positions t0 .. t0 + rows - 1 (zero outside the layer input
  // and for channels past C_in), positions fastest: coalesced ring reads
  for (int e = threadIdx.x; e < rows * CIP; e += 256) {
    const int ch = e / rows, r = e - ch * rows, t = t0 + r;
    uint16_t v = 0;
    if (ch < g.ci && t >= 0 && t < g.Lin) {
      int sl = ihead + t;
      if (sl >= g.Lin) sl -= g.Lin;
      v = in[(int64_t)ch * g.Lin + sl];
    }
    tile[r * RS + ch] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane & 15, lg = lane >> 4;
  const int MT = (g.co + 15) / 16;
  const uint4* wp = reinterpret_cast<const uint4*>(P.wpk);
  char* out = reinterpret_cast<char*>(it.cache) + P.off[P.layer];
  const int ohead = it.T / g.f;
  for (int u = wave; u < MT * (NC / 16); u += 4) {
    const int mt = u / (NC / 16), ct = u - mt * (NC / 16);
    // all of the unit's weight fragments are requested before its first MFMA
    uint4 af[NPH][KS];
#pragma unroll
    for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) af[ph][ks] = wp[((ph * MT + mt) * KS + ks) * 64 + lane];
    cf32x4 acc[NPH];
#pragma unroll
    for (int ph = 0; ph < NPH; ++ph) acc[ph] = cf32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kappa = 32 * ks + 8 * lg, jj = kappa / CIP, i0 = kappa - jj * CIP;
      // K entries past the taps have zero weights: read a row of finite values
      const int row = SC * (16 * ct + lc) + (jj < KT ? jj : KT - 1);
      const cbf16x8 bv = __builtin_bit_cast(cbf16x8, *reinterpret_cast<const uint4*>(&tile[row * RS + i0]));
#pragma unroll
      for (int ph = 0; ph < NPH; ++ph)
        acc[ph] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(cbf16x8, af[ph][ks]), bv, acc[ph], 0,
                                                          0, 0);
    }
    const int c = c0 + 16 * ct + lc;
#pragma unroll
    for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * mt + 4 * lg + r, pos = (c << CS) + ph;
        if (o >= g.co || pos >= g.Lout) continue;
        const float v = fmaf(acc[ph][r], P.scale[o], P.shift[o]);
        int oslot = ohead + pos;
        if (oslot >= g.Lout) oslot -= g.Lout;
        if (g.bn)
          reinterpret_cast<uint16_t*>(out)[(int64_t)o * g.Lout + oslot] = bf16_of(tanhf(v));
        else
          reinterpret_cast<float*>(out)[(int64_t)o * g.Lout + oslot] = v;
      }
  }
}

// The window's outputs from the cached noise ring: the dense noise window
// (when requested) and the clean output strain - noise over the request's
// span [W - s - delay, W - delay).  grid x = chunks of 256 positions of the
// window (or, without the noise output, of the clean span), y = item.
__global__ __launch_bounds__(256) void cache_emit_kernel(const CacheItem* items, int W, size_t off_noise,
                                                         const float* strain, float* noise, float* clean) {
  const CacheItem it = items[blockIdx.y];
  const float* ring = reinterpret_cast<const float*>(reinterpret_cast<const char*>(it.cache) + off_noise);
  const int t0 = W - it.s - it.delay;
  const int k = (noise ? 0 : t0) + (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (k >= (noise ? W : t0 + it.s)) return;
  int sl = it.T + k;
  if (sl >= W) sl -= W;
  const float v = ring[sl];
  if (noise) noise[(int64_t)blockIdx.y * W + k] = v;
  if (clean && k >= t0 && k < t0 + it.s) clean[it.out + (k - t0)] = strain[it.out + (k - t0)] - v;
}

hipError_t launch_cache_layer(const CacheItem* items, int n, const void* arena, const CacheLayerP& P, int max_chunks,
                              hipStream_t st) {
  const CacheGeo& g = P.geo[P.layer];
  if (n < 1 || max_chunks < 0 || !cache_layer_fits(g) || !P.wpk) return hipErrorInvalidValue;
  if (max_chunks == 0) return hipSuccess;
  const dim3 grid((unsigned)max_chunks, n);
  const int cip = (g.ci + 7) / 8 * 8;
#define GW_CACHE_LAUNCH(C_, NP_)                                                              \
  if (cip == C_ && (g.type == 1 ? 2 : 1) == NP_) {                                          \
    hipLaunchKernelGGL((cache_mfma_kernel<C_, NP_>), grid, dim3(256), 0, st, items, arena, P); \
    return hipGetLastError();                                                                \
  }
  GW_CACHE_LAUNCH(8, 1)
  GW_CACHE_LAUNCH(16, 1)
  GW_CACHE_LAUNCH(24, 1)
  GW_CACHE_LAUNCH(32, 1)
  GW_CACHE_LAUNCH(64, 1)
  GW_CACHE_LAUNCH(8, 2)
  GW_CACHE_LAUNCH(16, 2)
  GW_CACHE_LAUNCH(32, 2)
  GW_CACHE_LAUNCH(64, 2)
#undef GW_CACHE_LAUNCH
  return hipErrorNotSupported;
}

hipError_t launch_cache_emit(const CacheItem* items, int n, int W, int max_s, size_t off_noise, const float* strain,
                             float* noise, float* clean, hipStream_t st) {
  if (n < 1 || W < 1 || (!noise && !clean)) return hipErrorInvalidValue;
  const int span = noise ? W : max_s;
  hipLaunchKernelGGL(cache_emit_kernel, dim3((span + 255) / 256, n), dim3(256), 0, st, items, W, off_noise, strain,
                     noise, clean);
  return hipGetLastError();
}

}  // namespace gw
