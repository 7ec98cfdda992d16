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

// One chunk of 64 columns of one layer of one item, as an implicit GEMM on the
// matrix cores: D[o][c] = sum_kappa A[o][kappa] B[kappa][c] with A the model's
// BF16 weight fragments (v_mfma_f32_16x16x32_bf16 lane order, K = tap x input
// channel, transposed layers as two phases of 4 taps) and B the input window
// staged in LDS as [position][channel].  Column c is output position c of a
// conv, or input-aligned position m of a transposed conv (outputs 2m and
// 2m + 1).  Run by a group of 4 waves (gt = thread 0..255 of the group);
// barrier() separates the staging from the MFMAs.  An MFMA result element
// depends only on its own row of A and column of B, so a value comes out
// bitwise the same whichever chunk computes it; a chunk may therefore
// recompute a few clean positions next to a dirty range (with the same bits).
template <int CIP, int NPH>
struct CacheChunk {
  static constexpr int RS = CIP + 8;                  // LDS row stride (16-byte multiple, skews banks)
  static constexpr int NC = kCacheChunk;              // columns per chunk
  static constexpr int ROWSMAX = 2 * (NC - 1) + 7;    // a stride-2 k7 conv's window
  static constexpr int CS = NPH == 2 ? 1 : 0;         // log2 outputs per column
  static constexpr int KT = NPH == 2 ? 4 : 7;         // taps per column (k7; transposed: 4 per phase)
  static constexpr int KS = (KT * CIP + 31) / 32;     // K steps
  static constexpr int RMAX = NPH == 2 ? (NC - 1) + 4 : ROWSMAX;  // rows of a chunk's window, at most
  static constexpr int TILE = RMAX * RS;              // LDS elements
  static constexpr int NE = (RMAX * CIP + 255) / 256;  // staged elements per thread
  static constexpr int NPASS = NE > 20 ? 2 : 1;        // staged in passes of at most NE2 loads
  static constexpr int NE2 = (NE + NPASS - 1) / NPASS;

  // columns [0, la) (left zone) and [ra, ncols) (right band) and their chunks
  __device__ static void zones(const CacheLayerP& P, int layer, const CacheItem& it, int* ra, int* nl, int* nr) {
    const CacheGeo& g = P.geo[layer];
    int zl, zr;
    cache_band(P.geo, layer, it.shift, P.W, &zl, &zr);
    const int ncols = g.Lout >> CS;
    const int la = (zl + (1 << CS) - 1) >> CS;
    *ra = zr >> CS;
    *nl = (la + NC - 1) / NC;
    *nr = (ncols - *ra + NC - 1) / NC;
  }

  // active false: the group takes part in the barrier only
  template <typename Barrier>
  __device__ static void run(uint16_t* tile, const CacheItem& it, const void* arena, const CacheLayerP& P, int layer,
                             int c0, bool active, int gt_in, Barrier barrier) {
    // an opaque copy of the thread index keeps the per-element index
    // arithmetic inside the caller's loops instead of hoisted and live across
    // every layer of the fused kernel
    int gt = gt_in;
    asm volatile("" : "+v"(gt));
    const CacheGeo& g = P.geo[layer];
    const int SC = NPH == 2 ? 1 : g.s;
    const int t0 = NPH == 2 ? c0 - 1 : SC * c0 - g.p;  // transposed k7 s2 p3: column m reads m - 1 .. m + 2
    const int rows = SC * (NC - 1) + KT;
    const uint16_t* in;
    int ihead;
    if (layer == 0) {
      in = reinterpret_cast<const uint16_t*>(arena) + it.shadow;
      ihead = it.in_head;
    } else {
      in = reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(it.cache) + P.off[layer - 1]);
      ihead = it.T / P.geo[layer - 1].f;
    }
    // stage input positions t0 .. t0 + rows - 1 (zero outside the layer input
    // and for channels past C_in), positions fastest: coalesced ring reads.
    // Every load is unconditional, from an address clamped into the ring, so
    // a thread's loads are all in flight together; the store applies the zeros.
    const int lane = gt & 63, wave = gt >> 6;
    const int lc = lane & 15, lg = lane >> 4;
    const int MT = (g.co + 15) / 16;
    const uint4* wp = reinterpret_cast<const uint4*>(P.wpk[layer]);
    // the wave's first unit's weight fragments are requested before the
    // staging, so their latency overlaps it (when they are few enough to stay
    // in registers beside the staged values)
    constexpr bool EARLY = NPH * KS <= 8;
    uint4 af[NPH][KS];
    if (EARLY && active && wave < MT * (NC / 16)) {
      const int mt = wave / (NC / 16);
#pragma unroll
      for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) af[ph][ks] = wp[((ph * MT + mt) * KS + ks) * 64 + lane];
    }
    if (active) {
#pragma unroll
      for (int pass = 0; pass < NPASS; ++pass) {
        uint16_t v[NE2];
#pragma unroll
        for (int j = 0; j < NE2; ++j) {
          const int e = gt + 256 * (pass * NE2 + j);
          const int ch = e / rows, r = e - ch * rows;
          const int tc = min(max(t0 + r, 0), g.Lin - 1);
          int sl = ihead + tc;
          if (sl >= g.Lin) sl -= g.Lin;
          v[j] = in[(int64_t)min(ch, g.ci - 1) * g.Lin + sl];
        }
#pragma unroll
        for (int j = 0; j < NE2; ++j) {
          const int e = gt + 256 * (pass * NE2 + j);
          const int ch = e / rows, r = e - ch * rows, t = t0 + r;
          if (e < rows * CIP) tile[r * RS + ch] = (ch < g.ci && t >= 0 && t < g.Lin) ? v[j] : (uint16_t)0;
        }
      }
    }
    barrier();
    if (!active) return;
    const float* scale = P.scale[layer];
    const float* shift = P.shift[layer];
    char* out = reinterpret_cast<char*>(it.cache) + P.off[layer];
    const int ohead = it.T / g.f;
    for (int u = wave; u < MT * (NC / 16); u += 4) {
      const int mt = u / (NC / 16), ct = u - mt * (NC / 16);
      // the unit's weight fragments (the first unit's were requested above),
      // all in flight before its first MFMA
      if (!EARLY || u != wave) {
#pragma unroll
        for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) af[ph][ks] = wp[((ph * MT + mt) * KS + ks) * 64 + lane];
      }
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
          acc[ph] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(cbf16x8, af[ph][ks]), bv, acc[ph],
                                                            0, 0, 0);
      }
      const int c = c0 + 16 * ct + lc;
#pragma unroll
      for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = 16 * mt + 4 * lg + r, pos = (c << CS) + ph;
          if (o >= g.co || pos >= g.Lout) continue;
          const float val = fmaf(acc[ph][r], scale[o], shift[o]);
          int oslot = ohead + pos;
          if (oslot >= g.Lout) oslot -= g.Lout;
          if (g.bn)
            reinterpret_cast<uint16_t*>(out)[(int64_t)o * g.Lout + oslot] = bf16_of(tanhf(val));
          else
            reinterpret_cast<float*>(out)[(int64_t)o * g.Lout + oslot] = val;
        }
    }
  }
};

// The whole cached forward of one item per block: layer by layer, four groups
// of four waves take the layer's dirty chunks (the left zone's, then the
// right band's) four at a time, with block barriers between the staging and
// the MFMAs and after each round (a layer's ring writes are read by the next
// layer); then the item's outputs from the noise ring: the dense noise window
// (when requested) and the clean output strain - noise over the request's
// span [W - s - delay, W - delay).
constexpr int kCacheGroups = 4;
// the largest tile of any compiled variant: a 32-channel conv's or a
// 64-channel transposed conv's window
constexpr int kCacheTileMax = CacheChunk<32, 1>::TILE > CacheChunk<64, 2>::TILE ? CacheChunk<32, 1>::TILE
                                                                               : CacheChunk<64, 2>::TILE;

template <int CIP, int NPH>
__device__ __forceinline__ void cache_fused_layer(uint16_t* tiles, const CacheItem& it, const void* arena,
                                                  const CacheLayerP& P, int l) {
  using K = CacheChunk<CIP, NPH>;
  static_assert(K::TILE <= kCacheTileMax, "tile fits the group's LDS share");
  const int grp = threadIdx.x >> 8, gt = threadIdx.x & 255;
  int ra, nl, nr;
  K::zones(P, l, it, &ra, &nl, &nr);
  const int nch = nl + nr;
  for (int i = 0; i < nch; i += kCacheGroups) {  // block-uniform
    const int b = i + grp;
    const int c0 = b < nl ? b * K::NC : ra + (b - nl) * K::NC;
    K::run(tiles + grp * kCacheTileMax, it, arena, P, l, c0, b < nch, gt, [] { __syncthreads(); });
    __syncthreads();  // the tiles are free, and this round's ring writes are visible
  }
}

__global__ __launch_bounds__(256 * kCacheGroups) void cache_fused_kernel(const CacheItem* items, const void* arena,
                                                                           CacheLayerP P, const float* strain,
                                                                           float* noise, float* clean) {
  __shared__ __attribute__((aligned(16))) uint16_t tiles[kCacheGroups * kCacheTileMax];
  const CacheItem it = items[blockIdx.x];
  for (int l = 0; l < P.L; ++l) {
    const CacheGeo& g = P.geo[l];
    const int key = 4 * ((g.ci + 7) / 8 * 8) + (g.type == 1 ? 2 : 1);  // block-uniform
#define GW_CACHE_CASE(C_, NP_)                                \
    case 4 * C_ + NP_:                                        \
      cache_fused_layer<C_, NP_>(tiles, it, arena, P, l); \
      break;
    switch (key) {
      GW_CACHE_CASE(8, 1)
      GW_CACHE_CASE(16, 1)
      GW_CACHE_CASE(24, 1)
      GW_CACHE_CASE(32, 1)
      GW_CACHE_CASE(8, 2)
      GW_CACHE_CASE(16, 2)
      GW_CACHE_CASE(32, 2)
      GW_CACHE_CASE(64, 2)
      default: break;  // excluded by cache_layer_fits on the host
    }
#undef GW_CACHE_CASE
  }
  // outputs (the noise ring's writes are visible after the last round's barrier)
  const int W = P.W;
  const float* ring = reinterpret_cast<const float*>(reinterpret_cast<const char*>(it.cache) + P.off[P.L - 1]);
  const int t0 = W - it.s - it.delay;
  const int k0 = noise ? 0 : t0, k1 = noise ? W : t0 + it.s;
  for (int k = k0 + (int)threadIdx.x; k < k1; k += 256 * kCacheGroups) {
    int sl = it.T + k;
    if (sl >= W) sl -= W;
    const float v = ring[sl];
    if (noise) noise[(int64_t)blockIdx.x * W + k] = v;
    if (clean && k >= t0 && k < t0 + it.s) clean[it.out + (k - t0)] = strain[it.out + (k - t0)] - v;
  }
}

hipError_t launch_cache_forward(const CacheItem* items, int n, const void* arena, const CacheLayerP& P,
                                const float* strain, float* noise, float* clean, hipStream_t st) {
  if (n < 1 || P.L < 1 || P.L > kCacheMaxLayers) return hipErrorInvalidValue;
  for (int l = 0; l < P.L; ++l)
    if (!cache_layer_fits(P.geo[l]) || !P.wpk[l]) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cache_fused_kernel, dim3(n), dim3(256 * kCacheGroups), 0, st, items, arena, P, strain, noise,
                     clean);
  return hipGetLastError();
}

}  // namespace gw
