// Fused BBHnet forward (BF16 operands, FP32 accumulation): one block computes
// a tile of 64 positions of the last stage's output for one window through
// all three residual stages, with every intermediate activation in LDS, and
// writes the tile's share of the pooled head (sum over its positions and
// channels of head_w[o] * a3[o][q]); a second launch sums a window's shares
// in a fixed order into its logit.
//
// Network (the reference BBHnet shape): stage s maps C_s -> C_{s+1} channels
// (2 -> 32 -> 64 -> 128) and halves the length:
//   h   = ReLU(conv_a(x) + b_a)                  conv_a: k7, stride 2, pad 3
//   out = ReLU(conv_b(h) + b_b + W_s x[2t] + b_s) conv_b: k7, stride 1, pad 3
// Working back from the tile [q0, q0 + 64) of the last output, every tensor's
// needed rows are a fixed range around its scaled tile start (LO, NR below):
// conv_a output row r reads input rows 2r + j, conv_b output row r reads
// rows r + j, and the shortcut of output row r reads input row 2r + 9.
// Positions outside a tensor's signal are stored as zeros (the next layer's
// padding), so every value equals the layer-by-layer result up to summation
// order.  Tensors read with stride 2 are stored even rows first, then odd
// rows.  Buffers hold every row a padding column may read; rows past a
// tensor's needed range are never written and feed only padding columns
// (an MFMA result column depends only on its own B column), whose outputs
// are discarded.
#include "internal.h"

namespace gw {
namespace bbf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int T3 = 64;     // last-stage positions per block
constexpr int NW = 8;      // waves per block
constexpr int NTHR = 64 * NW;

// per tensor: channels (padded), LDS row stride, row offset LO (row 0 sits at
// scaled tile start + LO), needed rows NR, buffer rows CAP, even/odd split
//                     x     h0    a1    h1    a2    h2    a3
constexpr int CH[7] = {8, 32, 32, 64, 64, 128, 128};
constexpr int RS[7] = {8, 40, 40, 72, 72, 136, 0};
constexpr int LO[7] = {-63, -30, -27, -12, -9, -3, 0};
constexpr int NR[7] = {637, 315, 309, 152, 146, 70, 64};
// CAP: the deepest row a padding column reads, + 1 (x: the a1 shortcut's
// row 2 * 319 + 9; h0: 319 + 6; a1: the a2 shortcut's 2 * 159 + 9; h1: 159 + 6;
// a2: h2's 2 * 79 + 6, rounded up to even for the split; h2: 63 + 6)
constexpr int CAP[7] = {648, 326, 328, 166, 166, 70, 0};
constexpr int SPLIT[7] = {1, 0, 1, 0, 1, 0, 0};
constexpr int HALF(int t) { return SPLIT[t] ? CAP[t] / 2 : 0; }
__host__ __device__ constexpr int prow(int t, int r) { return SPLIT[t] ? (r & 1) * HALF(t) + (r >> 1) : r; }
// scale of tensor t's positions relative to the last stage (x: 8, h0/a1: 4, ...)
constexpr int SCL[7] = {8, 4, 4, 2, 2, 1, 1};

constexpr int mx(int a, int b) { return a > b ? a : b; }
// rows read by a phase's columns (NT column tiles): conv taps and shortcut
constexpr int reach(int sci, int nt, bool sc) { return mx(sci * (16 * nt - 1) + 6, sc ? 2 * (16 * nt - 1) + 9 : 0) + 1; }
static_assert(CAP[0] >= reach(2, 20, false) && CAP[0] >= reach(0, 20, true), "x rows");
static_assert(CAP[1] >= reach(1, 20, false), "h0 rows");
static_assert(CAP[2] >= reach(2, 10, false) && CAP[2] >= reach(0, 10, true), "a1 rows");
static_assert(CAP[3] >= reach(1, 10, false), "h1 rows");
static_assert(CAP[4] >= reach(2, 5, false) && CAP[4] >= reach(0, 4, true), "a2 rows");
static_assert(CAP[5] >= reach(1, 4, false), "h2 rows");
// valid rows read only valid rows
static_assert(2 * (NR[1] - 1) + 6 < NR[0] && NR[2] - 1 + 6 < NR[1] && 2 * (NR[2] - 1) + 9 < NR[0], "stage 0");
static_assert(2 * (NR[3] - 1) + 6 < NR[2] && NR[4] - 1 + 6 < NR[3] && 2 * (NR[4] - 1) + 9 < NR[2], "stage 1");
static_assert(2 * (NR[5] - 1) + 6 < NR[4] && NR[6] - 1 + 6 < NR[5] && 2 * (NR[6] - 1) + 9 < NR[4], "stage 2");

// LDS regions: R0 holds h0 then h1, R1 a1 then h2, R2 x then a2
constexpr int R0 = mx(CAP[1] * RS[1], CAP[3] * RS[3]);
constexpr int R1 = mx(CAP[2] * RS[2], CAP[5] * RS[5]);
constexpr int R2 = mx(CAP[0] * RS[0], CAP[4] * RS[4]);

}  // namespace bbf

namespace bbf {

__device__ __forceinline__ uint16_t rne(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  return (uint16_t)((u & 0x7fffffffu) > 0x7f800000u ? ((u >> 16) | 0x40u) : r);
}

// two floats -> packed BF16 pair by the hardware conversion (round to nearest
// even, the same bits as rne)
__device__ __forceinline__ uint32_t rne2(float lo, float hi) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){lo, hi}, bf16x2_t));
}

// One convolution of the tile: output tensor TO from input tensor TI (taps
// KT, input rows SCI r + jj), optionally with the stage's 1x1 shortcut from
// tensor TS (rows 2 r + 9) added to the same accumulators.  Work unit =
// MTW 16-channel output tiles x NTW column tiles (each B fragment read from
// LDS serves MTW MFMAs, each weight fragment NTW); unit u goes to wave u.
// MODE 0: ReLU, store BF16 rows < NR[TO] (zero outside the signal); MODE 1:
// the last stage, whose ReLU output is pooled: returns this lane's share of
// sum_o hw[o] y[o][q] over valid positions.
template <int TI, int TO, int TS, int SCI, int MT, int MTW, int NT, int NTW, int MODE>
__device__ __forceinline__ float conv_phase(const uint16_t* in, const uint16_t* sin, uint16_t* out, const uint4* wq,
                                            const uint4* wsq, const float* bias, const float* bias2, const float* hw,
                                            int base, int Lout) {
  constexpr int CIP = CH[TI], KT = 7, KS = (KT * CIP + 31) / 32;
  constexpr int CIPS = TS >= 0 ? CH[TS] : 0, KS2 = (CIPS + 31) / 32;
  constexpr int NG = (NT + NTW - 1) / NTW;
  static_assert(MT % MTW == 0 && (MT / MTW) * NG == NW, "one unit per wave");
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lc = lane & 15, lg = lane >> 4;
  const int mt0 = (wave / NG) * MTW, ct0 = (wave % NG) * NTW;
  f32x4 acc[MTW][NTW];
#pragma unroll
  for (int m = 0; m < MTW; ++m)
#pragma unroll
    for (int a = 0; a < NTW; ++a) acc[m][a] = f32x4{0.f, 0.f, 0.f, 0.f};
  // weights: fragment (mt, ks) lane l; four K steps requested ahead
  const uint4* wp = wq + (size_t)mt0 * KS * 64 + lane;
  uint4 ar[4][MTW];
#pragma unroll
  for (int d = 0; d < 4; ++d)
#pragma unroll
    for (int m = 0; m < MTW; ++m) ar[d][m] = d < KS ? wp[(m * KS + d) * 64] : make_uint4(0, 0, 0, 0);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    uint4 av[MTW];
#pragma unroll
    for (int m = 0; m < MTW; ++m) {
      av[m] = ar[ks & 3][m];
      if (ks + 4 < KS) ar[ks & 3][m] = wp[(m * KS + ks + 4) * 64];
    }
    const int kappa = 32 * ks + 8 * lg, jj0 = kappa / CIP, i0 = kappa - jj0 * CIP;
    const int jj = jj0 < KT ? jj0 : KT - 1;  // K padding: zero weights, a row of finite values
#pragma unroll
    for (int a = 0; a < NTW; ++a) {
      if (ct0 + a >= NT) break;
      const int r = (ct0 + a) * 16 + lc;
      const uint4 bv = *reinterpret_cast<const uint4*>(in + prow(TI, SCI * r + jj) * RS[TI] + i0);
#pragma unroll
      for (int m = 0; m < MTW; ++m)
        acc[m][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[m]),
                                                            __builtin_bit_cast(bf16x8, bv), acc[m][a], 0, 0, 0);
    }
  }
  if constexpr (TS >= 0) {
    const uint4* sp = wsq + (size_t)mt0 * KS2 * 64 + lane;
#pragma unroll
    for (int ks = 0; ks < KS2; ++ks) {
      uint4 av[MTW];
#pragma unroll
      for (int m = 0; m < MTW; ++m) av[m] = sp[(m * KS2 + ks) * 64];
      const int kappa = 32 * ks + 8 * lg, i0 = kappa < CIPS ? kappa : 0;
#pragma unroll
      for (int a = 0; a < NTW; ++a) {
        if (ct0 + a >= NT) break;
        const int r = (ct0 + a) * 16 + lc;
        const uint4 bv = *reinterpret_cast<const uint4*>(sin + prow(TS, 2 * r + 9) * RS[TS] + i0);
#pragma unroll
        for (int m = 0; m < MTW; ++m)
          acc[m][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[m]),
                                                              __builtin_bit_cast(bf16x8, bv), acc[m][a], 0, 0, 0);
      }
    }
  }
  // epilogue: D[row = 4 lg + e][col = lc] is channel 16 mt + 4 lg + e of row r
  float gsum = 0.0f;
#pragma unroll
  for (int m = 0; m < MTW; ++m) {
    const int mt = mt0 + m;
    float kb[4], kh[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int o = 16 * mt + 4 * lg + e;
      kb[e] = bias[o] + (TS >= 0 ? bias2[o] : 0.0f);
      kh[e] = MODE == 1 ? hw[o] : 0.0f;
    }
#pragma unroll
    for (int a = 0; a < NTW; ++a) {
      if (ct0 + a >= NT) break;
      const int r = (ct0 + a) * 16 + lc;
      if (r >= NR[TO]) continue;
      const int pos = base + LO[TO] + r;
      const bool live = pos >= 0 && pos < Lout;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = live ? fmaxf(acc[m][a][e] + kb[e], 0.0f) : 0.0f;
      if constexpr (MODE == 1) {
#pragma unroll
        for (int e = 0; e < 4; ++e) gsum = fmaf(kh[e], v[e], gsum);
      } else {
        const uint32_t lo = rne2(v[0], v[1]);
        const uint32_t hi = rne2(v[2], v[3]);
        *reinterpret_cast<uint2*>(out + prow(TO, r) * RS[TO] + 16 * mt + 4 * lg) = make_uint2(lo, hi);
      }
    }
  }
  return gsum;
}

}  // namespace bbf

// two 8-wave blocks per CU (LDS 76 KB each): four waves per SIMD, at most 128 VGPRs
__global__ __launch_bounds__(bbf::NTHR, 4) void bbh_fused(BbFusedP p) {
  using namespace bbf;
  __shared__ __attribute__((aligned(16))) uint16_t r0[R0];
  __shared__ __attribute__((aligned(16))) uint16_t r1[R1];
  __shared__ __attribute__((aligned(16))) uint16_t r2[R2];
  __shared__ float wsum[NW];
  const int b = blockIdx.x / p.tiles, tile = blockIdx.x - b * p.tiles;
  if (b >= p.n) return;
  const int W = p.W, q0 = tile * T3;
  const int L[7] = {W, W / 2, W / 2, W / 4, W / 4, W / 8, W / 8};
  // stage the input rows: positions 8 q0 - 63 + r, r < CAP (channels 2..7 zero)
  {
    const uint16_t* sh = nullptr;
    const float* fx = nullptr;
    int head = 0;
    if (p.items) {
      const Item& it = p.items[b];
      sh = reinterpret_cast<const uint16_t*>(p.arena) + it.shadow;
      head = it.head;
    } else {
      fx = p.x + (int64_t)b * 2 * W;
    }
    const int x0 = SCL[0] * q0 + LO[0];
    for (int r = threadIdx.x; r < CAP[0]; r += NTHR) {
      const int pos = x0 + r;
      uint32_t c01 = 0;
      if (pos >= 0 && pos < W) {
        if (sh) {
          int ph = head + pos;
          if (ph >= W) ph -= W;
          c01 = (uint32_t)sh[ph] | ((uint32_t)sh[W + ph] << 16);
        } else {
          c01 = (uint32_t)bbf::rne(fx[pos]) | ((uint32_t)bbf::rne(fx[W + pos]) << 16);
        }
      }
      *reinterpret_cast<uint4*>(r2 + prow(0, r) * RS[0]) = make_uint4(c01, 0u, 0u, 0u);
    }
  }
  __syncthreads();
  const uint4* const* WA = reinterpret_cast<const uint4* const*>(p.wa);
  const uint4* const* WB = reinterpret_cast<const uint4* const*>(p.wb);
  const uint4* const* WS = reinterpret_cast<const uint4* const*>(p.ws);
  // stage 0: h0 (R0) from x (R2); a1 (R1) from h0 and x
  conv_phase<0, 1, -1, 2, 2, 1, 20, 5, 0>(r2, nullptr, r0, WA[0], nullptr, p.ba[0], nullptr, nullptr,
                                       SCL[1] * q0, L[1]);
  __syncthreads();
  conv_phase<1, 2, 0, 1, 2, 1, 20, 5, 0>(r0, r2, r1, WB[0], WS[0], p.bb[0], p.bs[0], nullptr, SCL[2] * q0, L[2]);
  __syncthreads();
  // stage 1: h1 (R0) from a1 (R1); a2 (R2) from h1 and a1
  conv_phase<2, 3, -1, 2, 4, 1, 10, 5, 0>(r1, nullptr, r0, WA[1], nullptr, p.ba[1], nullptr, nullptr,
                                       SCL[3] * q0, L[3]);
  __syncthreads();
  conv_phase<3, 4, 2, 1, 4, 1, 10, 5, 0>(r0, r1, r2, WB[1], WS[1], p.bb[1], p.bs[1], nullptr, SCL[4] * q0, L[4]);
  __syncthreads();
  // stage 2: h2 (R1) from a2 (R2); the pooled output from h2 and a2
  conv_phase<4, 5, -1, 2, 8, 1, 5, 5, 0>(r2, nullptr, r1, WA[2], nullptr, p.ba[2], nullptr, nullptr,
                                      SCL[5] * q0, L[5]);
  __syncthreads();
  float g = conv_phase<5, 6, 4, 1, 8, 2, 4, 2, 1>(r1, r2, nullptr, WB[2], WS[2], p.bb[2], p.bs[2], p.hw,
                                               SCL[6] * q0, L[6]);
  // fixed-order reduction: lanes of a wave, then the waves in order
  for (int off = 32; off > 0; off >>= 1) g += __shfl_down(g, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = g;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.0f;
    for (int w = 0; w < NW; ++w) s += wsum[w];
    p.part[blockIdx.x] = s;
  }
}

bool bbh_fused_supported(int c_in, const int* co, int stages) {
  return c_in == 2 && stages == 3 && co[0] == 32 && co[1] == 64 && co[2] == 128;
}

int bbh_fused_tiles(int W) { return (W / 8 + bbf::T3 - 1) / bbf::T3; }

hipError_t launch_bbh_fused(const BbFusedP& p, hipStream_t st) {
  if (p.n < 1 || p.W < 8 || p.W % 8 || p.tiles != bbh_fused_tiles(p.W)) return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)p.n * p.tiles;
  if (blocks > ((int64_t)1 << 31) - 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bbh_fused, dim3((unsigned)blocks), dim3(bbf::NTHR), 0, st, p);
  return hipGetLastError();
}

}  // namespace gw
