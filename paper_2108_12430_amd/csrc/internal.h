// Internal declarations shared by the ABI layer and the HIP kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace gw {

// Per-item descriptor of a batched call, staged host->device once per call.
// Offsets are in elements of the arena viewed as float (ring) or uint16 (shadow).
struct Item {
  int64_t ring;    // fp32 ring [C][W] of the slot
  int64_t shadow;  // bf16 shadow [C][W] of the slot
  int64_t src;     // snapshot_update: offset of the [C][s] block in `samples`
  int64_t out;     // forward: offset of this item's [s] block in strain/clean
  int32_t head;    // ring index of the oldest sample (update: before writing)
  int32_t s;       // new samples per request (stride)
  int32_t C, W;
  int32_t delay;   // forward: aggregation latency in samples (clean block ends delay before W)
  int32_t pad_;
};
static_assert(sizeof(Item) == 56, "Item layout");

enum Epi : int {
  EPI_AFFINE = 0,       // y = acc*scale[o] + shift[o]
  EPI_AFFINE_TANH = 1,  // y = tanh(acc*scale[o] + shift[o])
  EPI_BIAS = 2,         // y = acc + bias[o]   (bias may be null)
  EPI_RELU = 3,         // y = max(acc + bias[o], 0)
  EPI_RESID_RELU = 4,   // y = max(acc + bias[o] + shortcut(x_stage)[o], 0)
  EPI_OUT = 5,          // y = acc*scale + shift; noise + causal clean outputs
  EPI_RESID_GAP = 6,    // as EPI_RESID_RELU, then sum_o hw[o] * y per block (pooling head)
};

enum Src : int { SRC_DENSE = 0, SRC_RING = 1 };

// One convolution layer launch (direct FP32 or BF16 MFMA).
struct ConvP {
  // input
  const float* x;          // dense fp32 [n][Ci][Lin] (SRC_DENSE)
  const uint16_t* xh;      // dense bf16 [n][Ci][Lin] (BF16 kernels, SRC_DENSE)
  const void* arena;       // pool arena base (SRC_RING)
  const Item* items;       // per-item descriptors (SRC_RING or EPI_OUT)
  // output
  float* y;                // fp32 [n][Co][Lout]
  uint16_t* yh;            // bf16 [n][Co][Lout] (BF16 kernels, intermediate layers)
  // weights: w[o*wso + i*wsi + j] for conv, w[i*wsi + o*wso + j] for transposed
  const float* w;
  int64_t wso, wsi;
  const uint16_t* wpk;     // packed bf16 weights (BF16 kernels)
  const uint16_t* wpk_lo;  // low bf16 terms of the weights (split FP32 input), or null
  const uint16_t* wspk;    // packed bf16 1x1 shortcut weights (BF16 residual epilogue)
  const float* bias;
  const float* scale;
  const float* shift;
  // residual shortcut (EPI_RESID_RELU): 1x1 stride-2 conv of the stage input
  const float* xs;         // stage input fp32 [n][Cs][Ls]
  const uint16_t* xsh;     // stage input bf16
  const float* ws;         // [Co][Cs]
  const float* bs;         // [Co]
  int Cs, Ls;
  // pooling head (EPI_RESID_GAP): per-block partial sums of hw[o] * y[o][t]
  const float* hw;
  float* gap_part;         // [n][gridDim.x]
  // outputs of EPI_OUT
  float* noise;            // [n][W] or null
  const float* strain;     // packed, or null
  float* clean;            // packed, or null
  // shape
  int n, Ci, Co, Lin, Lout, k, stride, pad;
  // row stride (elements) of a dense first-layer input when it differs from
  // Lin (a band at the end of longer windows); 0 means Lin.  Ring inputs wrap
  // at their item's W and read positions [head + q] for q in [0, Lin).
  int ldx;
  // fused snapshot update (ring input, fused kernel only): item i's newest s
  // samples, [C][s] FP32 at upd + items[i].src, are read from here rather
  // than from the ring, and written to the ring and its shadow by the launch
  const float* upd;
};

// ---- incremental DeepClean over per-stream activation caches ----
// Geometry of one layer of the cached network: type 0 conv (output k reads
// inputs s k - p + j), 1 transposed conv (output u = s t - p + j); f is the
// window length over the layer's output length (the grid's step in samples);
// bn: normalisation + tanh, stored BF16; f32: stored FP32 (the output conv).
struct CacheGeo {
  int type, ci, co, k, s, p, op, Lin, Lout, f, bn, f32;
};
constexpr int kCacheMaxLayers = 16;
struct CacheLayerP {
  CacheGeo geo[kCacheMaxLayers];
  size_t off[kCacheMaxLayers];                // byte offset of layer l's ring in a stream's cache
  const uint16_t* wpk[kCacheMaxLayers];       // BF16 weight fragments (the per-layer MFMA kernels' packing)
  const float* scale[kCacheMaxLayers];        // folded normalisation: y = acc * scale + shift
  const float* shift[kCacheMaxLayers];
  int L, W;
};
// Per-item descriptor of a cached call (staged with the pool's item tables).
struct CacheItem {
  void* cache;        // the stream's cache (device)
  int64_t shadow;     // BF16 shadow of the stream's snapshot ring (arena elements)
  int64_t out;        // offset of the item's [s] block in strain/clean
  int32_t in_head;    // ring index of the snapshot's oldest sample
  int32_t T;          // the cache's window start modulo W (a multiple of 16): layer l's ring head is T / f_l
  int32_t shift;      // samples the window advanced since the cache was last made current; -1: recompute all
  int32_t s, delay;   // clean output span [W - s - delay, W - delay)
  int32_t pad_;
};
static_assert(sizeof(CacheItem) == 48, "CacheItem layout");

// float -> bfloat16, round to nearest even (NaN stays NaN): the ring's
// shadow values, written by the snapshot update and by the fused update
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__host__ __device__ inline int cache_cdiv(int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); }
// Dirty output positions of layer `layer` after the window advanced by
// `shift` samples (a multiple of the total stride): [0, *zl) and [*zr, Lout).
// An output keeps its cached value when every input it reads kept its value:
// inputs in the dirty bands of the previous layer change, the first layer's
// newest `shift` samples are new, and inputs before the window's start are
// zero padding now but were real samples before (so the left zone grows
// from the padding inward); inputs past the window's end are padding in both.
// Past the end, the last shift / f positions of a layer did not exist.  The
// bands are a superset of the positions that change (never a subset).
__host__ __device__ inline void cache_band(const CacheGeo* g, int layer, int shift, int W, int* zl, int* zr) {
  const int L = g[layer].Lout;
  if (shift < 0) {  // recompute everything
    *zl = L;
    *zr = L;
    return;
  }
  int lo_in = 0, hi_in = W - shift, Lin = W;
  for (int l = 0; l <= layer; ++l) {
    const CacheGeo& G = g[l];
    const int Lo = G.Lout;
    int lo, hi;
    if (G.type == 0) {
      lo = cache_cdiv(lo_in + G.p, G.s);                                 // s k - p >= lo_in
      hi = hi_in < Lin ? cache_cdiv(hi_in - (G.k - 1 - G.p), G.s) : Lo;  // s k - p + k - 1 >= hi_in
    } else {
      lo = G.s * (lo_in - 1) + G.k - G.p;                                // min input >= lo_in
      hi = hi_in < Lin ? G.s * hi_in - G.p : Lo;                         // max input >= hi_in
    }
    const int fresh = Lo - shift / G.f;
    hi = hi < fresh ? hi : fresh;
    lo = lo < 0 ? 0 : (lo > Lo ? Lo : lo);
    hi = hi < 0 ? 0 : (hi > Lo ? Lo : hi);
    if (hi <= lo) {  // the bands meet: every position is dirty
      lo = Lo;
      hi = Lo;
    }
    lo_in = lo;
    hi_in = hi;
    Lin = Lo;
  }
  *zl = lo_in;
  *zr = hi_in;
}
// A group of the cached kernel covers kCacheChunk consecutive columns at a
// time (output positions of a conv, input-aligned positions of a transposed
// conv) and stages their input window in LDS.
constexpr int kCacheChunk = 64;
// layer shapes the cached kernel takes: k7 p3 convs (stride 1 or 2) and k7
// s2 p3 transposed convs whose C_in rounds up to a compiled channel tile (a
// conv's window of a chunk is twice a transposed conv's, so convs stop at 32
// input channels to keep the fused kernel's staging in registers)
inline bool cache_layer_fits(const CacheGeo& g) {
  const int cip = (g.ci + 7) / 8 * 8;
  const bool tile = g.type == 0 ? (cip == 8 || cip == 16 || cip == 24 || cip == 32)
                                : (cip == 8 || cip == 16 || cip == 32 || cip == 64);
  // the kernel's LDS window holds a stride-1 or stride-2 conv's rows
  return tile && g.k == 7 && g.p == 3 && (g.type == 0 ? (g.s == 1 || g.s == 2) : (g.s == 2 && g.op == 1));
}
// The whole cached forward of n items (one block each: every layer's dirty
// chunks, then the item's noise window and/or clean span; noise NULL: only
// the clean span).
hipError_t launch_cache_forward(const CacheItem* items, int n, const void* arena, const CacheLayerP& P,
                                const float* strain, float* noise, float* clean, hipStream_t st);

// ---- fused BBHnet (reference shape: 2 -> 32 -> 64 -> 128, k7) ----
struct BbFusedP {
  const void* arena;      // pool arena (ring input) or null
  const Item* items;      // ring descriptors (ring input)
  const float* x;         // dense input [n][2][W] or null
  const uint16_t* wa[3];  // packed conv_a fragments per stage
  const uint16_t* wb[3];  // packed conv_b fragments
  const uint16_t* ws[3];  // packed 1x1 shortcut fragments
  const float* ba[3];
  const float* bb[3];
  const float* bs[3];
  const float* hw;        // head weights [128]
  float* part;            // [n][tiles] pooled-head shares
  int n, W, tiles;
};

bool bbh_fused_supported(int c_in, const int* co, int stages);
int bbh_fused_tiles(int W);  // blocks (pooled-head shares) per window
hipError_t launch_bbh_fused(const BbFusedP& p, hipStream_t st);

// ---- launchers (defined in the .hip files) ----
hipError_t launch_conv_fp32(const ConvP& p, bool transposed, int epi, int src, hipStream_t st);
hipError_t launch_conv_bf16(const ConvP& p, bool transposed, int epi, int src, hipStream_t st);
bool conv_bf16_supported(int Ci, int Co, int k, int stride, bool transposed);
int conv_bf16_gap_parts(int Ci, int Co, int Lout, int n);  // GAP partial sums per window (EPI_RESID_GAP), -1 if none
// Fused DeepClean network (21->8->16->32->64 convs, 64->32->16->8->8
// transposed convs, 8->1 output conv, all k7 p3; BN+tanh on all but the last)
bool dc_fused_supported(const int* ci, const int* co, const int* type, const int* k, const int* s,
                        const int* pad, const int* op, const int* bn, int L);
hipError_t launch_dc_fused_bf16(const ConvP& p, const uint16_t* const* wpk, const float* const* scale,
                                const float* const* shift, int W, bool ring, int cu_budget, hipStream_t st,
                                bool f16 = false, bool upd = false);
size_t conv_bf16_packed_elems(int Ci, int Co, int k, bool transposed);
// layers of the fused network whose weights the fused kernel takes in its own
// fragment layout (stacked transposed layers, Toeplitz output conv)
bool dc_fused_special(int l);
size_t dc_fused_special_elems(int l);
hipError_t launch_pack_fused(const float* w, uint16_t* out, int l, hipStream_t st, bool f16);
// mode PACK_BF16: bf16 (RNE); PACK_F16: IEEE half (RNE); PACK_BF16_LO: the
// bf16 rounding of w - bf16(w) (the low term of a two-term split)
enum PackMode : int { PACK_BF16 = 0, PACK_F16 = 1, PACK_BF16_LO = 2 };
hipError_t launch_pack_bf16(const float* w, uint16_t* out, int Ci, int Co, int k, bool transposed,
                            hipStream_t st, int mode = PACK_BF16);

hipError_t launch_snapshot(void* arena, const Item* items, int n, int max_cs, const float* samples,
                           hipStream_t st);
hipError_t launch_fill_zero(void* dst, size_t bytes, hipStream_t st);
hipError_t launch_decimate2(int n, int C, int s, int K, const float* taps, const float* x, float* hist, float* y,
                            hipStream_t st);
hipError_t launch_overlap_average(const Item* items, int n, int max_s, int W, int depth, const float* noise,
                                  float* state, const float* strain, float* clean, float* avg, hipStream_t st);
hipError_t launch_zero_floats(float* dst, int64_t n, hipStream_t st);
// Window fetch: logical window [C][W] of each item's ring into dense [n][C][W].
hipError_t launch_gather(const void* arena, const Item* items, int n, int C, int W, float* out,
                         uint16_t* outh, hipStream_t st);

hipError_t launch_fold_bn(const float* b, const float* gamma, const float* beta, const float* mean,
                          const float* var, float* scale, float* shift, int C, hipStream_t st);

// logits[b] = (sum_k part[b][k]) / L + bias, k < nblk, fixed order
hipError_t launch_gap_finalize(const float* part, int nblk, const float* bias, float* logits, int n,
                               int L, hipStream_t st);
hipError_t launch_gap_linear(const float* a, const float* w, const float* b, float* logits, int n,
                             int C, int L, hipStream_t st);

// Training
int red_chunks(int n, int L);  // chunks of a per-channel (batch, time) reduction
hipError_t launch_bn_stats(const float* z, int n, int C, int L, double* partial, int nchunk,
                           float* mean, float* invstd, hipStream_t st);
hipError_t launch_bn_apply_tanh(const float* z, const float* mean, const float* invstd,
                                const float* gamma, const float* beta, float* a, int n, int C,
                                int L, hipStream_t st);
hipError_t launch_bn_tanh_backward(const float* g, const float* a, const float* z,
                                   const float* mean, const float* invstd, const float* gamma,
                                   int n, int C, int L, double* partial, int nchunk, float* dz,
                                   float* dgamma, float* dbeta, hipStream_t st);
hipError_t launch_channel_sum(const float* x, int n, int C, int L, double* partial, int nchunk,
                              float* out, hipStream_t st);
size_t wgrad_scratch_bytes(int n, int Lp, int nw);
// LDS per block: 4*(Ca*64 + Cc*(stride*63 + k)) bytes, must be <= 64 KiB.
hipError_t launch_wgrad(const float* P, int Ca, int Lp, const float* Q, int Cc, int Lq, int n,
                        int k, int stride, int pad, void* scratch, float* dw, hipStream_t st);
// workspace of the band-passed loss: the n x nb (cos, sin) projections
size_t bandpass_ws_floats(int n, int W, int nb);
hipError_t launch_bandpass(int n, int W, int k_lo, int k_hi, const float* strain,
                           const float* noise, float* proj, float* loss, float* dnoise,
                           hipStream_t st);

}  // namespace gw
