// BF16 implicit-GEMM 1-D convolutions on the gfx950 matrix cores.
//
// GEMM view of one layer and one window:  Y[o][c] = sum_kappa A[o][kappa] B[kappa][c]
//   o      output channel (M, tiles of 16)
//   c      output column: the output time t for a strided conv, or the input
//          position m for a stride-2 transposed conv (polyphase: column m
//          produces outputs 2m and 2m+1 from two weight sets ("phases"), so the
//          zeros a transposed conv would insert are never multiplied)
//   kappa  = tap * CIP + input channel (K, channel-minor; CIP = C_in rounded up
//          to a multiple of 8 so one lane's 8 consecutive K entries are one
//          tap and 8 consecutive channels)
// A (weights) is pre-packed in the exact per-lane fragment order of
// v_mfma_f32_16x16x32_bf16 (16 bytes per lane per fragment).  B is read from
// an LDS tile that holds the block's input window transposed to
// [time][channel], so each lane's B fragment is one aligned 16-byte LDS read.
// Accumulation is FP32; the epilogue (folded normalisation + tanh, ReLU,
// residual shortcut, causal slice + subtraction) is FP32; intermediate
// activations are stored as BF16 (round to nearest even).
//
// Fragment layout of v_mfma_f32_16x16x32_bf16 (lane l = 0..63):
//   A[row = l % 16][k = 8 (l / 16) + e],  B[k = 8 (l / 16) + e][col = l % 16],
//   D[row = 4 (l / 16) + r][col = l % 16],  e = 0..7, r = 0..3.
#include "internal.h"

namespace gw {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even; NaNs stay (quiet) NaNs.
// Written without a branch so it compiles to straight-line selects.
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  const uint32_t q = (u >> 16) | 0x40u;
  return (uint16_t)((u & 0x7fffffffu) > 0x7f800000u ? q : r);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// IN_RING_F32: fused FP16 kernel only.  IN_F32S: FP32 input split into two
// BF16 terms, x = hi + lo (hi = RNE(x), lo = RNE(x - hi)), staged as two
// tiles; with the weights split the same way each product takes three MFMAs
// (hi*hi + lo_w*hi_x + hi_w*lo_x), which leaves a relative error of about
// 2^-16 per product instead of 2^-8 (the training variant's convolutions).
enum InFmt { IN_F32 = 0, IN_BF16 = 1, IN_RING = 2, IN_RING_F32 = 3, IN_F32S = 4 };

// Geometry of the polyphase/strided column view of a layer (host + device).
struct Geo {
  int nph;    // phases (1 for conv, stride for transposed)
  int kt;     // taps per phase
  int sc;     // input step per column (stride for conv, 1 for transposed)
  int padc;   // input position of tile row 0 is sc*col0 - padc
  int ncol;   // output columns
};

__host__ __device__ inline Geo make_geo(bool tr, int k, int s, int p, int Lout) {
  Geo g;
  if (!tr) {
    g.nph = 1;
    g.kt = k;
    g.sc = s;
    g.padc = p;
    g.ncol = Lout;
  } else {
    // output u = s*m + r uses input m + d with tap j = r + p - s*d, 0 <= j < k
    int dmin = 1 << 30, dmax = -(1 << 30);
    for (int r = 0; r < s; ++r)
      for (int j = 0; j < k; ++j)
        if ((r + p - j) % s == 0) {
          const int d = (r + p - j) / s;
          dmin = d < dmin ? d : dmin;
          dmax = d > dmax ? d : dmax;
        }
    g.nph = s;
    g.kt = dmax - dmin + 1;
    g.sc = 1;
    g.padc = -dmin;
    g.ncol = (Lout + s - 1) / s;
  }
  return g;
}

// ---------------------------------------------------------------------------
// Weight packing: fragment (ph, mt, ks), lane l, element e holds
// W_ph[o = 16 mt + l%16][kappa = 32 ks + 8 (l/16) + e], zero outside.
// ---------------------------------------------------------------------------
static inline int cip_of(int ci) { return (ci + 7) / 8 * 8; }

__global__ void pack_bf16_kernel(const float* w, uint16_t* out, int Ci, int Co, int k, int s, int p,
                                 bool tr, int nph, int kt, int padc, int MT, int KS, int CIP,
                                 int total, int mode) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int e = idx & 7;
  const int l = (idx >> 3) & 63;
  int f = idx >> 9;
  const int ks = f % KS;
  f /= KS;
  const int mt = f % MT;
  const int ph = f / MT;
  const int o = 16 * mt + (l & 15);
  const int kappa = 32 * ks + 8 * (l >> 4) + e;
  const int jj = kappa / CIP, i = kappa % CIP;
  float v = 0.0f;
  if (o < Co && i < Ci && jj < kt) {
    if (!tr) {
      v = w[((int64_t)o * Ci + i) * k + jj];
    } else {
      const int d = jj - padc;
      const int j = ph + p - s * d;
      if (j >= 0 && j < k) v = w[((int64_t)i * Co + o) * k + j];
    }
  }
  if (mode == PACK_F16) {
    out[idx] = __builtin_bit_cast(uint16_t, (_Float16)v);
  } else {
    const uint16_t hi = bf16_rne(v);
    out[idx] = mode == PACK_BF16_LO ? bf16_rne(v - bf16_to_f(hi)) : hi;
  }
}

static void frag_dims(int Ci, int Co, int k, int s, int p, bool tr, int* MT, int* KS, int* CIP,
                      Geo* g) {
  *g = make_geo(tr, k, s, p, 1 << 20);
  *CIP = cip_of(Ci);
  *MT = (Co + 15) / 16;
  *KS = (g->kt * *CIP + 31) / 32;
}

size_t conv_bf16_packed_elems(int Ci, int Co, int k, bool tr) {
  // stride/pad of the supported layers: conv k7 s{1,2} p3, transposed k7 s2 p3
  int MT, KS, CIP;
  Geo g;
  frag_dims(Ci, Co, k, tr ? 2 : 1, 3, tr, &MT, &KS, &CIP, &g);
  return (size_t)g.nph * MT * KS * 512;
}

hipError_t launch_pack_bf16(const float* w, uint16_t* out, int Ci, int Co, int k, bool tr,
                            hipStream_t st, int mode) {
  const int s = tr ? 2 : 1, p = 3;
  int MT, KS, CIP;
  Geo g;
  frag_dims(Ci, Co, k, s, p, tr, &MT, &KS, &CIP, &g);
  const int total = g.nph * MT * KS * 512;
  hipLaunchKernelGGL(pack_bf16_kernel, dim3((total + 255) / 256), dim3(256), 0, st, w, out, Ci, Co, k, s,
                     p, tr, g.nph, g.kt, g.padc, MT, KS, CIP, total, mode);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LDS staging.  Tile row r holds input position q0 + r for every channel
// (time-major, channel-minor, row stride RS).  Work items are (channel,
// 8-position chunk) with the channel varying fastest across lanes, so the
// 2-byte LDS stores of one instruction hit consecutive banks; each item reads
// its 8 positions with one 16-byte load (32 bytes for FP32 input) when the
// chunk is aligned and inside the signal, element by element otherwise.
// ---------------------------------------------------------------------------
template <int CIP, int ROWS, int IN, int NTHR = 256>
struct InRaw {
  static constexpr int NCHMAX = (ROWS + 7 + 7) / 8;             // 8-position chunks per channel
  static constexpr int ITEMS = (NCHMAX * CIP + NTHR - 1) / NTHR;  // (channel, chunk) items per thread
  static constexpr int NV = (IN == IN_F32 || IN == IN_F32S) ? 2 : 1;
  static_assert(ITEMS <= 32, "one mask bit per item");
  uint4 v[ITEMS][NV];  // raw 16-byte pieces (two for FP32 input)
  uint32_t f32mask;    // items whose v[it][0..1] still hold 8 FP32 values (always, for IN_F32S)
};

// Issue the global loads of one tile's input window into registers.  Tile
// row r holds input position q0 + r for every channel; work items are
// (channel, 8-position chunk) with the channel varying fastest across lanes.
// Each item is one 16-byte load (two for FP32 input) when the chunk is
// aligned and inside the signal, element by element otherwise.
template <int CIP, int ROWS, int IN, int NTHR = 256>
__device__ __forceinline__ void load_input(InRaw<CIP, ROWS, IN, NTHR>& R, const ConvP& p, int b, int q0) {
  constexpr int ITEMS = InRaw<CIP, ROWS, IN, NTHR>::ITEMS;
  const int Ci = p.Ci, Lin = p.Lin;  // positions q in [0, Lin) exist; others are zero padding
  const int qa = q0 - (((q0 % 8) + 8) % 8);  // floor to a multiple of 8
  const int nch = (q0 + ROWS - qa + 7) / 8;
  int head = 0;
  int ld = p.ldx ? p.ldx : Lin;  // row stride; a ring wraps at its length
  const uint16_t* hbase = nullptr;
  const float* fbase = nullptr;
  bool vec;
  if (IN == IN_RING) {
    const Item& it = p.items[b];
    head = it.head;
    ld = it.W;
    hbase = reinterpret_cast<const uint16_t*>(p.arena) + it.shadow;
    vec = (ld & 7) == 0 && (head & 7) == 0 && (it.shadow & 7) == 0;
  } else if (IN == IN_BF16) {
    hbase = p.xh + (int64_t)b * Ci * ld;
    vec = (ld & 7) == 0 && (reinterpret_cast<uintptr_t>(p.xh) & 15) == 0;
  } else {
    fbase = p.x + (int64_t)b * Ci * ld;
    vec = (ld & 7) == 0 && (reinterpret_cast<uintptr_t>(p.x) & 15) == 0;
  }
  R.f32mask = 0;
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int e = threadIdx.x + NTHR * it;
    const int i = e % CIP, ch = e / CIP;
    const int qc = qa + 8 * ch;
    R.v[it][0] = make_uint4(0, 0, 0, 0);
    if (IN == IN_F32S) {
      // split staging keeps every item in FP32 (zeros outside the signal)
      R.v[it][R.NV - 1] = make_uint4(0, 0, 0, 0);
      R.f32mask |= 1u << it;
    }
    if (ch < nch && i < Ci) {
      if (vec && qc >= 0 && qc + 8 <= Lin) {
        if (IN == IN_F32 || IN == IN_F32S) {
          const uint4* src = reinterpret_cast<const uint4*>(fbase + (int64_t)i * ld + qc);
          R.v[it][0] = src[0];
          R.v[it][R.NV - 1] = src[1];
          R.f32mask |= 1u << it;
        } else {
          int ph = qc;
          if (IN == IN_RING) {
            ph = head + qc;
            if (ph >= ld) ph -= ld;
          }
          R.v[it][0] = *reinterpret_cast<const uint4*>(hbase + (int64_t)i * ld + ph);
        }
      } else if (IN == IN_F32S) {
        float f[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = qc + k;
          f[k] = (q >= 0 && q < Lin) ? fbase[(int64_t)i * ld + q] : 0.0f;
        }
        R.v[it][0] = make_uint4(__float_as_uint(f[0]), __float_as_uint(f[1]), __float_as_uint(f[2]),
                                __float_as_uint(f[3]));
        R.v[it][R.NV - 1] = make_uint4(__float_as_uint(f[4]), __float_as_uint(f[5]), __float_as_uint(f[6]),
                                       __float_as_uint(f[7]));
      } else {
        uint16_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = qc + k;
          v[k] = 0;
          if (q >= 0 && q < Lin) {
            if (IN == IN_F32) {
              v[k] = bf16_rne(fbase[(int64_t)i * ld + q]);
            } else {
              int ph = q;
              if (IN == IN_RING) {
                ph = head + q;
                if (ph >= ld) ph -= ld;
              }
              v[k] = hbase[(int64_t)i * ld + ph];
            }
          }
        }
        R.v[it][0] = make_uint4((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                                (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16));
      }
    }
  }
}

// Write a loaded tile into LDS ([row][channel], row stride RS) plus the zero
// row used by padded K entries.
// HALF > 0 stores row r at (r & 1) * HALF + (r >> 1): even rows first, then
// odd rows, so a stride-2 reader walks consecutive LDS rows.
// IN_F32S writes the high BF16 terms to `tile` and the low terms to `tile_lo`.
template <int CIP, int ROWS, int RS, int IN, int NTHR = 256, int HALF = 0>
__device__ __forceinline__ void store_input(uint16_t* tile, const InRaw<CIP, ROWS, IN, NTHR>& R, int q0,
                                            uint16_t* tile_lo = nullptr) {
  constexpr int ITEMS = InRaw<CIP, ROWS, IN, NTHR>::ITEMS;
  const int qa = q0 - (((q0 % 8) + 8) % 8);
  const int nch = (q0 + ROWS - qa + 7) / 8;
#pragma unroll
  for (int it = 0; it < ITEMS; ++it) {
    const int e = threadIdx.x + NTHR * it;
    const int i = e % CIP, ch = e / CIP;
    if (ch >= nch) continue;
    uint16_t v[8], vl[8];
    if (IN == IN_F32S) {
      const uint4 a = R.v[it][0], c = R.v[it][R.NV - 1];
      const float f[8] = {__uint_as_float(a.x), __uint_as_float(a.y), __uint_as_float(a.z), __uint_as_float(a.w),
                          __uint_as_float(c.x), __uint_as_float(c.y), __uint_as_float(c.z), __uint_as_float(c.w)};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        v[k] = bf16_rne(f[k]);
        vl[k] = bf16_rne(f[k] - bf16_to_f(v[k]));  // exact difference, rounded
      }
    } else if (IN == IN_F32 && (R.f32mask & (1u << it))) {
      const uint4 a = R.v[it][0], c = R.v[it][R.NV - 1];
      v[0] = bf16_rne(__uint_as_float(a.x)); v[1] = bf16_rne(__uint_as_float(a.y));
      v[2] = bf16_rne(__uint_as_float(a.z)); v[3] = bf16_rne(__uint_as_float(a.w));
      v[4] = bf16_rne(__uint_as_float(c.x)); v[5] = bf16_rne(__uint_as_float(c.y));
      v[6] = bf16_rne(__uint_as_float(c.z)); v[7] = bf16_rne(__uint_as_float(c.w));
    } else {
      const uint4 u = R.v[it][0];
      v[0] = u.x & 0xffff; v[1] = u.x >> 16; v[2] = u.y & 0xffff; v[3] = u.y >> 16;
      v[4] = u.z & 0xffff; v[5] = u.z >> 16; v[6] = u.w & 0xffff; v[7] = u.w >> 16;
    }
    const int r0 = qa + 8 * ch - q0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = r0 + k;
      const int pr = HALF ? (r & 1) * HALF + (r >> 1) : r;
      if (r >= 0 && r < ROWS) {
        tile[pr * RS + i] = v[k];
        if (IN == IN_F32S) tile_lo[pr * RS + i] = vl[k];
      }
    }
  }
  constexpr int PZ = HALF ? (ROWS & 1) * HALF + (ROWS >> 1) : ROWS;
  for (int e = threadIdx.x; e < RS; e += NTHR) {
    tile[PZ * RS + e] = 0;
    if (IN == IN_F32S) tile_lo[PZ * RS + e] = 0;
  }
}

// Shortcut tile for the residual stage: row c holds the stage input at
// position 2 (col0 + c) (1x1 kernel, stride 2), channel-minor.
template <int CSP, int TN>
struct ShortRaw {
  static constexpr int ITEMS = ((TN / 4) * CSP + 255) / 256;  // (channel, 4-row chunk) items per thread
  uint32_t v[ITEMS > 0 ? ITEMS : 1][2];                        // four bf16 per item
};

// Issue the loads of the shortcut tile (row c = stage input at position
// 2 (col0 + c), channel-minor) into registers; stored by store_shortcut.
template <int CSP, int TN, bool XS_F32>
__device__ __forceinline__ void load_shortcut(ShortRaw<CSP, TN>& R, const ConvP& p, int b, int col0) {
  const int Cs = p.Cs, Ls = p.Ls;
  const int p0 = 2 * col0;  // multiple of 8
  const bool vec = (Ls & 7) == 0 &&
                   ((XS_F32 ? reinterpret_cast<uintptr_t>(p.xs) : reinterpret_cast<uintptr_t>(p.xsh)) & 15) == 0;
#pragma unroll
  for (int it = 0; it < ShortRaw<CSP, TN>::ITEMS; ++it) {
    const int e = threadIdx.x + 256 * it;
    const int i = e % CSP, ch = e / CSP;
    const int pc = p0 + 8 * ch;  // positions pc .. pc+7 -> rows 4ch .. 4ch+3 (even positions)
    uint32_t v[4] = {0, 0, 0, 0};
    if (ch < TN / 4 && i < Cs) {
      const int64_t base = ((int64_t)b * Cs + i) * Ls;
      if (vec && pc + 8 <= Ls) {
        if (XS_F32) {
          const float4* src = reinterpret_cast<const float4*>(p.xs + base + pc);
          const float4 a = src[0], c = src[1];
          v[0] = bf16_rne(a.x); v[1] = bf16_rne(a.z); v[2] = bf16_rne(c.x); v[3] = bf16_rne(c.z);
        } else {
          const uint4 u = *reinterpret_cast<const uint4*>(p.xsh + base + pc);
          v[0] = u.x & 0xffff; v[1] = u.y & 0xffff; v[2] = u.z & 0xffff; v[3] = u.w & 0xffff;
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int q = pc + 2 * k;
          if (q < Ls) v[k] = XS_F32 ? bf16_rne(p.xs[base + q]) : p.xsh[base + q];
        }
      }
    }
    R.v[it][0] = v[0] | (v[1] << 16);
    R.v[it][1] = v[2] | (v[3] << 16);
  }
}

template <int CSP, int TN, int RSX>
__device__ __forceinline__ void store_shortcut(uint16_t* xt, const ShortRaw<CSP, TN>& R) {
#pragma unroll
  for (int it = 0; it < ShortRaw<CSP, TN>::ITEMS; ++it) {
    const int e = threadIdx.x + 256 * it;
    const int i = e % CSP, ch = e / CSP;
    if (ch >= TN / 4) continue;
    xt[(4 * ch + 0) * RSX + i] = R.v[it][0] & 0xffff;
    xt[(4 * ch + 1) * RSX + i] = R.v[it][0] >> 16;
    xt[(4 * ch + 2) * RSX + i] = R.v[it][1] & 0xffff;
    xt[(4 * ch + 3) * RSX + i] = R.v[it][1] >> 16;
  }
  for (int e = threadIdx.x; e < RSX; e += 256) xt[TN * RSX + e] = 0;
}

// ---------------------------------------------------------------------------
// The convolution kernel.  Block = 4 waves; a tile = TN = 64*NTW consecutive
// output columns of one window and all output channels.  Blocks are
// persistent: block k processes tiles k, k + gridDim.x, ...; the global loads
// of the next tile's input are issued before the current tile's matrix work,
// so HBM latency overlaps computation.  Weights (when they fit) and the
// epilogue's per-channel constants stay in registers for all tiles.  With
// CSP > 0 (residual stage) the 1x1 stride-2 shortcut of the stage input is
// added to the same accumulators as extra K steps.
// ---------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Request K step `ks` of this block's weight fragments (piece e = fragment
// e >> 6, lane e & 63) into registers; steps past the end are skipped.
template <int MT, int MTB, int KS, int ACH, int APT>
__device__ __forceinline__ void fetch_kstep(u32x4 (&dst)[APT], const u32x4* wp, int ms, int ks) {
#pragma unroll
  for (int k = 0; k < APT; ++k) {
    const int e = threadIdx.x + 256 * k, f = e >> 6, mt = f % MTB, ph = f / MTB;
    if (e < ACH && ks < KS) dst[k] = wp[((ph * MT + ms * MTB + mt) * KS + ks) * 64 + (e & 63)];
  }
}

template <int CIP, int MT, int NPH, int KT, int SC, int NTW, int EPI, int IN, bool OUT_F32, bool XS_F32,
          int CSP, int MS, int AM>
__global__ __launch_bounds__(256) void conv_mfma(ConvP p, int padc, int ncol) {
  static_assert(MT % MS == 0, "the m-split divides the output-channel tiles");
  // AM = 1 (large batches): the block's weight fragments pass through LDS one
  // K step at a time, double-buffered, fetched from L2 while the previous
  // step computes; all four waves share them.
  constexpr int MTB = MT / MS;  // output-channel tiles of this block
  constexpr int TN = 64 * NTW;
  constexpr int ROWS = SC * (TN - 1) + KT;
  constexpr int RS = CIP + 8;  // LDS row stride in bf16 (16-byte multiple, skews banks)
  constexpr int KS = (KT * CIP + 31) / 32;
  constexpr int RSX = CSP + 8;
  constexpr int KS2 = (CSP + 31) / 32;
  constexpr int NFRAG = NPH * MTB * KS;  // weight fragments of this block's channel tiles
  constexpr int TNO = NPH * TN;
  constexpr bool OTILE = EPI != EPI_OUT && EPI != EPI_RESID_GAP && !OUT_F32;
  // the input tile's LDS is reused for the BF16 output tile [C_out][NPH*TN]
  constexpr int TILE = (ROWS + 1) * RS > 16 * MTB * TNO ? (ROWS + 1) * RS : 16 * MTB * TNO;
  // split operands (IN_F32S): a second tile of low terms, weights read per wave
  constexpr bool SPL = IN == IN_F32S;
  static_assert(!SPL || (AM == 0 && CSP == 0 && OUT_F32), "split operands: FP32-output layers, AM = 0");
  // weights staged in LDS once per block when they fit beside the tile; only
  // then is the next tile prefetched (LDS reads do not wait on global loads)
  constexpr bool ALDS = AM == 0 && !SPL && 2 * TILE + NFRAG * 1024 <= 80 * 1024;
  constexpr int ACH = AM ? NPH * MTB * 64 : 1;  // 16-byte pieces of one K step's fragments
  constexpr int APT = (ACH + 255) / 256;        // pieces per thread
  __shared__ __attribute__((aligned(16))) uint16_t tile[TILE];
  __shared__ __attribute__((aligned(16))) uint16_t tile_lo[SPL ? (ROWS + 1) * RS : 8];
  __shared__ __attribute__((aligned(16))) uint16_t xt[CSP > 0 ? (TN + 1) * RSX : 8];
  __shared__ __attribute__((aligned(16))) uint4 alds[ALDS ? NFRAG * 64 : 1];
  __shared__ __attribute__((aligned(16))) uint4 achunk[2 * ACH];
  __shared__ float cst[2][16 * MTB];
  __shared__ float wsum[4];

  // block j computes output-channel tiles [ms MTB, (ms + 1) MTB), ms = j mod MS,
  // of the column tiles j / MS, j / MS + gridDim.x / MS, ... (gridDim.x is a
  // multiple of MS)
  const int ms = (int)blockIdx.x % MS, bi = (int)blockIdx.x / MS, G = (int)gridDim.x / MS;
  const int o_lo = 16 * MTB * ms;  // first output channel of this block
  const int tiles_per = (ncol + TN - 1) / TN;
  const int total = tiles_per * p.n;
  if (bi >= total) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lc = lane & 15, lg = lane >> 4;
  const uint4* wp = reinterpret_cast<const uint4*>(p.wpk);
  const uint4* wpl = reinterpret_cast<const uint4*>(p.wpk_lo);

  if (ALDS)
    for (int e = threadIdx.x; e < (ALDS ? NFRAG * 64 : 0); e += 256) {
      const int f = e >> 6, ks = f % KS, r = f / KS, mtb = r % MTB, ph = r / MTB;
      alds[e] = wp[((ph * MT + ms * MTB + mtb) * KS + ks) * 64 + (e & 63)];
    }
  // per-channel epilogue constants: cst[0] multiplies, cst[1] adds
  for (int o = threadIdx.x; o < 16 * MTB; o += 256) {
    const int oc = min(o_lo + o, p.Co - 1);
    float a = 0.f, c = 0.f;
    if (EPI == EPI_AFFINE || EPI == EPI_OUT || EPI == EPI_AFFINE_TANH) {
      a = p.scale[oc];
      c = p.shift[oc];
    } else if (EPI == EPI_RELU || EPI == EPI_BIAS) {
      c = p.bias ? p.bias[oc] : 0.f;
    } else {
      c = p.bias[oc] + p.bs[oc];
      if (EPI == EPI_RESID_GAP) a = p.hw[oc];
    }
    cst[0][o] = a;
    cst[1][o] = c;
  }

  InRaw<CIP, ROWS, IN> raw;
  ShortRaw<CSP, TN> sraw;
  load_input<CIP, ROWS, IN>(raw, p, bi / tiles_per, SC * ((bi % tiles_per) * TN) - padc);
  if (CSP > 0) load_shortcut<CSP, TN, XS_F32>(sraw, p, bi / tiles_per, (bi % tiles_per) * TN);
  // ALDS: persistent loop over tiles with prefetch; otherwise one tile per block
  const int tstep = ALDS ? G : total;
  for (int t = bi; t < total; t += tstep) {
    const int b = t / tiles_per;
    const int col0 = (t % tiles_per) * TN;
    store_input<CIP, ROWS, RS, IN>(tile, raw, SC * col0 - padc, tile_lo);
    if (CSP > 0) store_shortcut<CSP, TN, RSX>(xt, sraw);
    if constexpr (AM == 1) {
      // K step 0's fragments into buffer 0 (piece e = fragment (e >> 6), lane e & 63)
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        const int e = threadIdx.x + 256 * k, f = e >> 6, mt = f % MTB, ph = f / MTB;
        if (e < ACH) achunk[e] = wp[((ph * MT + ms * MTB + mt) * KS + 0) * 64 + (e & 63)];
      }
    }
    __syncthreads();
    if (ALDS) {
      const int tn = t + tstep;
      if (tn < total) {
        load_input<CIP, ROWS, IN>(raw, p, tn / tiles_per, SC * ((tn % tiles_per) * TN) - padc);
        if (CSP > 0) load_shortcut<CSP, TN, XS_F32>(sraw, p, tn / tiles_per, (tn % tiles_per) * TN);
      }
    }

    f32x4 acc[NTW][NPH][MTB];
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt)
#pragma unroll
      for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
        for (int mt = 0; mt < MTB; ++mt) acc[nt][ph][mt] = f32x4{0.f, 0.f, 0.f, 0.f};

    if constexpr (AM == 1) {
      // register ring of AD stages: the fragments of step ks + AD - 1 are
      // requested while step ks computes, so an L2 round trip has AD - 1
      // steps to complete; one LDS buffer pair holds steps ks and ks + 1
      constexpr int AD = 4;
      const u32x4* wv = reinterpret_cast<const u32x4*>(p.wpk);
      u32x4 an0[APT], an1[APT], an2[APT], an3[APT];
      u32x4(*an[AD])[APT] = {&an0, &an1, &an2, &an3};
      static_assert(AD == 4, "four named ring slots");
      fetch_kstep<MT, MTB, KS, ACH, APT>(an1, wv, ms, 1);  // steps 1 .. 3 (step 0 is in LDS)
      fetch_kstep<MT, MTB, KS, ACH, APT>(an2, wv, ms, 2);
      fetch_kstep<MT, MTB, KS, ACH, APT>(an3, wv, ms, 3);
#pragma unroll 1
      for (int k0 = 0; k0 < KS; k0 += AD) {
#pragma unroll
        for (int d = 0; d < AD; ++d) {
          const int ks = k0 + d;
          if (ks >= KS) break;  // block-uniform
          const uint4* ab = achunk + (ks & 1) * ACH;
          const int kappa = 32 * ks + 8 * lg;
          const int jj = kappa / CIP, i0 = kappa - jj * CIP;
          uint4 af[NPH][MTB];
#pragma unroll
          for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
            for (int mt = 0; mt < MTB; ++mt) af[ph][mt] = ab[(ph * MTB + mt) * 64 + lane];
#pragma unroll
          for (int nt = 0; nt < NTW; ++nt) {
            const int c = (wave * NTW + nt) * 16 + lc;
            const int row = (jj < KT) ? SC * c + jj : ROWS;
            const bf16x8 bb = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&tile[row * RS + i0]));
#pragma unroll
            for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
              for (int mt = 0; mt < MTB; ++mt)
                acc[nt][ph][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[ph][mt]),
                                                                         bb, acc[nt][ph][mt], 0, 0, 0);
          }
          // step ks + 1 (requested AD - 1 steps ago, ring slot (d + 1) mod AD)
          // to the other LDS buffer; then request step ks + AD into the freed slot
          if (ks + 1 < KS) {
            u32x4* dst = reinterpret_cast<u32x4*>(achunk + ((ks + 1) & 1) * ACH);
#pragma unroll
            for (int k = 0; k < APT; ++k)
              if (threadIdx.x + 256 * k < ACH) dst[threadIdx.x + 256 * k] = (*an[(d + 1) % AD])[k];
          }
          fetch_kstep<MT, MTB, KS, ACH, APT>(*an[d], wv, ms, ks + AD);
          __syncthreads();  // step ks + 1 staged; buffer ks & 1 free for step ks + 2
        }
      }
    }
    // few accumulators: unroll so the next K steps' LDS reads are in flight
    // during this step's MFMAs; many accumulators: keep the loop rolled
    constexpr int KUNROLL = NTW * NPH * MTB <= 2 ? 4 : 1;
#pragma unroll KUNROLL
    for (int ks = 0; ks < (AM == 1 ? 0 : KS); ++ks) {
      const int kappa = 32 * ks + 8 * lg;
      const int jj = kappa / CIP, i0 = kappa - jj * CIP;
      uint4 af[NPH][MTB], afl[SPL ? NPH : 1][SPL ? MTB : 1];
#pragma unroll
      for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
        for (int mt = 0; mt < MTB; ++mt) {
          af[ph][mt] = ALDS ? alds[ALDS ? ((ph * MTB + mt) * KS + ks) * 64 + lane : 0]
                            : wp[((ph * MT + ms * MTB + mt) * KS + ks) * 64 + lane];
          if constexpr (SPL) afl[ph][mt] = wpl[((ph * MT + ms * MTB + mt) * KS + ks) * 64 + lane];
        }
#pragma unroll
      for (int nt = 0; nt < NTW; ++nt) {
        const int c = (wave * NTW + nt) * 16 + lc;
        const int row = (jj < KT) ? SC * c + jj : ROWS;
        const uint4 bv = *reinterpret_cast<const uint4*>(&tile[row * RS + i0]);
        const bf16x8 bb = __builtin_bit_cast(bf16x8, bv);
        bf16x8 bl = bb;
        if constexpr (SPL) bl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&tile_lo[row * RS + i0]));
#pragma unroll
        for (int ph = 0; ph < NPH; ++ph)
#pragma unroll
          for (int mt = 0; mt < MTB; ++mt) {
            if constexpr (SPL) {
              // small terms first: lo_w * hi_x + hi_w * lo_x, then hi_w * hi_x
              acc[nt][ph][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  __builtin_bit_cast(bf16x8, afl[ph][mt]), bb, acc[nt][ph][mt], 0, 0, 0);
              acc[nt][ph][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  __builtin_bit_cast(bf16x8, af[ph][mt]), bl, acc[nt][ph][mt], 0, 0, 0);
            }
            acc[nt][ph][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, af[ph][mt]), bb, acc[nt][ph][mt], 0, 0, 0);
          }
      }
    }
    if (CSP > 0) {
      const uint4* sp = reinterpret_cast<const uint4*>(p.wspk);
      for (int ks = 0; ks < KS2; ++ks) {
        const int kappa = 32 * ks + 8 * lg;
        uint4 af[MTB];
#pragma unroll
        for (int mt = 0; mt < MTB; ++mt) af[mt] = sp[((ms * MTB + mt) * KS2 + ks) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
          const int c = (wave * NTW + nt) * 16 + lc;
          const int row = kappa < CSP ? c : TN;
          const uint4 bv = *reinterpret_cast<const uint4*>(&xt[row * RSX + (kappa < CSP ? kappa : 0)]);
          const bf16x8 bb = __builtin_bit_cast(bf16x8, bv);
#pragma unroll
          for (int mt = 0; mt < MTB; ++mt)
            acc[nt][0][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[mt]), bb,
                                                                     acc[nt][0][mt], 0, 0, 0);
        }
      }
    }

    // ---- epilogue
    uint16_t* otile = tile;
    if (OTILE) __syncthreads();  // every wave is done reading the input tile
    float gsum = 0.0f;           // EPI_RESID_GAP: this lane's share of sum_o hw[o] y[o][t]
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
      const int col = col0 + (wave * NTW + nt) * 16 + lc;
      if (col >= ncol) continue;
#pragma unroll
      for (int mt = 0; mt < MTB; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ol = 16 * mt + 4 * lg + r, o = o_lo + ol;  // block-local, global channel
          if (o >= p.Co) continue;
          const float ka = cst[0][ol], kb = cst[1][ol];
          float v[NPH];
#pragma unroll
          for (int ph = 0; ph < NPH; ++ph) {
            const float a = acc[nt][ph][mt][r];
            if (EPI == EPI_AFFINE || EPI == EPI_OUT) {
              v[ph] = fmaf(a, ka, kb);
            } else if (EPI == EPI_AFFINE_TANH) {
              v[ph] = tanhf(fmaf(a, ka, kb));
            } else if (EPI == EPI_BIAS) {
              v[ph] = a + kb;
            } else {  // EPI_RELU, EPI_RESID_RELU, EPI_RESID_GAP (shortcut already accumulated)
              v[ph] = fmaxf(a + kb, 0.0f);
            }
          }
          if (EPI == EPI_RESID_GAP) {
            gsum = fmaf(ka, v[0], gsum);
          } else if (EPI == EPI_OUT) {
#pragma unroll
            for (int ph = 0; ph < NPH; ++ph) {
              const int u = NPH * col + ph;
              if (u >= p.Lout) continue;
              const int W = p.Lout;
              if (p.noise) p.noise[(int64_t)b * W + u] = v[ph];
              if (p.clean) {
                const Item& it = p.items[b];
                const int t0 = W - it.s - it.delay;
                if (u >= t0 && u < t0 + it.s) {
                  const int64_t idx = it.out + (u - t0);
                  p.clean[idx] = p.strain[idx] - v[ph];
                }
              }
            }
          } else if (OUT_F32) {
#pragma unroll
            for (int ph = 0; ph < NPH; ++ph) {
              const int u = NPH * col + ph;
              if (u < p.Lout) p.y[((int64_t)b * p.Co + o) * p.Lout + u] = v[ph];
            }
          } else {
#pragma unroll
            for (int ph = 0; ph < NPH; ++ph) otile[ol * TNO + NPH * (col - col0) + ph] = bf16_rne(v[ph]);
          }
        }
    }
    if (OTILE) {
      // write the tile back with 16-byte stores along time
      __syncthreads();
      const int Co = p.Co, Lout = p.Lout;
      const int u00 = NPH * col0;
      const int nco = min(Co - o_lo, 16 * MTB);  // this block's channels
      uint16_t* yb = p.yh + ((int64_t)b * Co + o_lo) * Lout;
      const bool vec = (Lout & 7) == 0 && (reinterpret_cast<uintptr_t>(p.yh) & 15) == 0;
      for (int e = threadIdx.x; e < nco * (TNO / 8); e += 256) {
        const int o = e / (TNO / 8), cu = e - o * (TNO / 8);
        const int u0 = u00 + 8 * cu;
        if (u0 >= Lout) continue;
        const uint16_t* src = &otile[o * TNO + 8 * cu];
        if (vec && u0 + 8 <= Lout) {
          *reinterpret_cast<uint4*>(yb + (int64_t)o * Lout + u0) = *reinterpret_cast<const uint4*>(src);
        } else {
          for (int k = 0; k < 8 && u0 + k < Lout; ++k) yb[(int64_t)o * Lout + u0 + k] = src[k];
        }
      }
    }
    if (EPI == EPI_RESID_GAP) {
      // fixed-order reduction: lanes of a wave, then the four waves
      for (int off = 32; off > 0; off >>= 1) gsum += __shfl_down(gsum, off, 64);
      if (lane == 0) wsum[wave] = gsum;
      __syncthreads();
      if (threadIdx.x == 0)
        p.gap_part[((int64_t)b * tiles_per + (t % tiles_per)) * MS + ms] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    }
    __syncthreads();  // LDS tiles are rewritten by the next iteration
  }
}

// ---------------------------------------------------------------------------
// Dispatch over the instantiated shapes.
// ---------------------------------------------------------------------------
struct Key {
  int cip, mt, nph, kt, sc, epi, in, out_f32, xs_f32, csp, am;
};

template <int CIP, int MT, int NPH, int KT, int SC, int EPI, int IN, bool OUT_F32, bool XS_F32, int CSP, int NTW,
          int MS, int AM>
static hipError_t launch_t(const ConvP& p, const Geo& g, hipStream_t st) {
  constexpr int TN = 64 * NTW, MTB = MT / MS;
  // same test as the kernel's ALDS: persistent grid only when weights fit in LDS
  constexpr int ROWS = SC * (TN - 1) + KT, RS = CIP + 8, KS = (KT * CIP + 31) / 32;
  constexpr int TILE = (ROWS + 1) * RS > 16 * MTB * NPH * TN ? (ROWS + 1) * RS : 16 * MTB * NPH * TN;
  constexpr bool ALDS = AM == 0 && IN != IN_F32S && 2 * TILE + NPH * MTB * KS * 1024 <= 80 * 1024;
  auto kern = conv_mfma<CIP, MT, NPH, KT, SC, NTW, EPI, IN, OUT_F32, XS_F32, CSP, MS, AM>;
  const int64_t tiles = (int64_t)((g.ncol + TN - 1) / TN) * p.n;
  if (tiles * MS > (int64_t)1 << 30) return hipErrorInvalidValue;
  if (!ALDS) {
    hipLaunchKernelGGL(kern, dim3((unsigned)(tiles * MS)), dim3(256), 0, st, p, g.padc, g.ncol);
    return hipGetLastError();
  }
  // persistent grid: enough blocks to fill every CU at the kernel's occupancy
  static int max_blocks = 0;
  if (max_blocks == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    max_blocks = per_cu * cus;
  }
  // a multiple of MS blocks: each channel share walks the same column tiles
  const int blocks = (int)std::min<int64_t>(tiles, std::max(max_blocks / MS, 1)) * MS;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, st, p, g.padc, g.ncol);
  return hipGetLastError();
}

// (CIP, MT, NPH, KT, SC, EPI, IN, OUT_F32, XS_F32, CSP, NTW, MS, AM) of every
// compiled variant: NTW 16-column tiles per wave (a block covers 64 NTW
// columns), an m-split MS (a block computes MT / MS output-channel tiles) and
// the weight path AM (0: resident in LDS or read per wave; 1: staged per K
// step, for large batches).
// The BBHnet layers are small GEMMs whose weights outweigh a window's
// activations: each block keeps one output-channel tile's weights in LDS and
// streams narrow column tiles past them.
#define GW_BF16_VARIANTS(X)                                                         \
  /* DeepClean-shaped encoder (k7 s2), first layer from FP32 or ring */            \
  X(24, 1, 1, 7, 2, EPI_AFFINE_TANH, IN_F32, false, false, 0, 4, 1, 0)           \
  X(24, 1, 1, 7, 2, EPI_AFFINE_TANH, IN_RING, false, false, 0, 4, 1, 0)          \
  X(8, 1, 1, 7, 2, EPI_AFFINE_TANH, IN_F32, false, false, 0, 4, 1, 0)            \
  X(8, 1, 1, 7, 2, EPI_AFFINE_TANH, IN_RING, false, false, 0, 4, 1, 0)           \
  X(8, 1, 1, 7, 2, EPI_AFFINE_TANH, IN_BF16, false, false, 0, 4, 1, 0)           \
  X(16, 2, 1, 7, 2, EPI_AFFINE_TANH, IN_BF16, false, false, 0, 4, 1, 0)          \
  X(32, 4, 1, 7, 2, EPI_AFFINE_TANH, IN_BF16, false, false, 0, 4, 1, 0)          \
  /* decoder (transposed k7 s2 p3 op1: 2 phases of 4 taps) */                      \
  X(64, 2, 2, 4, 1, EPI_AFFINE_TANH, IN_BF16, false, false, 0, 4, 1, 0)          \
  X(32, 1, 2, 4, 1, EPI_AFFINE_TANH, IN_BF16, false, false, 0, 4, 1, 0)          \
  X(16, 1, 2, 4, 1, EPI_AFFINE_TANH, IN_BF16, false, false, 0, 4, 1, 0)          \
  X(8, 1, 2, 4, 1, EPI_AFFINE_TANH, IN_BF16, false, false, 0, 4, 1, 0)           \
  /* output conv k7 s1 with causal slice + subtraction */                          \
  X(8, 1, 1, 7, 1, EPI_OUT, IN_BF16, true, false, 0, 4, 1, 0)                    \
  /* BBHnet-shaped stages: conv_a, then conv_b + 1x1 stride-2 shortcut */           \
  X(8, 2, 1, 7, 2, EPI_RELU, IN_F32, false, false, 0, 1, 2, 0)                   \
  X(32, 2, 1, 7, 1, EPI_RESID_RELU, IN_BF16, false, true, 8, 1, 2, 0)            \
  X(32, 4, 1, 7, 2, EPI_RELU, IN_BF16, false, false, 0, 1, 4, 0)                 \
  X(64, 4, 1, 7, 1, EPI_RESID_RELU, IN_BF16, false, false, 32, 1, 4, 0)          \
  X(64, 8, 1, 7, 2, EPI_RELU, IN_BF16, false, false, 0, 1, 8, 0)                 \
  X(128, 8, 1, 7, 1, EPI_RESID_RELU, IN_BF16, true, false, 64, 1, 8, 0)          \
  X(128, 8, 1, 7, 1, EPI_RESID_GAP, IN_BF16, true, false, 64, 1, 8, 0)           \
  /* BBHnet layers at large batches: all output channels per block, weights   \
     staged per K step */                                                      \
  X(8, 2, 1, 7, 2, EPI_RELU, IN_F32, false, false, 0, 4, 1, 1)                 \
  X(32, 2, 1, 7, 1, EPI_RESID_RELU, IN_BF16, false, true, 8, 4, 1, 1)          \
  X(32, 4, 1, 7, 2, EPI_RELU, IN_BF16, false, false, 0, 2, 1, 1)               \
  X(64, 4, 1, 7, 1, EPI_RESID_RELU, IN_BF16, false, false, 32, 2, 1, 1)        \
  X(64, 8, 1, 7, 2, EPI_RELU, IN_BF16, false, false, 0, 2, 2, 1)               \
  X(128, 8, 1, 7, 1, EPI_RESID_RELU, IN_BF16, true, false, 64, 2, 1, 1)        \
  X(128, 8, 1, 7, 1, EPI_RESID_GAP, IN_BF16, true, false, 64, 2, 1, 1)         \
  /* FP32-input output conv (a network whose last layer reads FP32) */            \
  X(8, 1, 1, 7, 1, EPI_OUT, IN_F32, true, false, 0, 4, 1, 0)                     \
  X(8, 1, 2, 4, 1, EPI_OUT, IN_F32, true, false, 0, 4, 1, 0)                     \
  /* training forward (BF16 conv variant): FP32 activations in, split into      \
     hi + lo BF16 terms (three MFMAs per product), FP32 z out */                   \
  X(24, 1, 1, 7, 2, EPI_BIAS, IN_F32S, true, false, 0, 2, 1, 0)                  \
  X(8, 1, 1, 7, 2, EPI_BIAS, IN_F32S, true, false, 0, 2, 1, 0)                   \
  X(16, 2, 1, 7, 2, EPI_BIAS, IN_F32S, true, false, 0, 2, 1, 0)                  \
  X(32, 4, 1, 7, 2, EPI_BIAS, IN_F32S, true, false, 0, 2, 1, 0)                  \
  X(64, 2, 2, 4, 1, EPI_BIAS, IN_F32S, true, false, 0, 2, 1, 0)                  \
  X(32, 1, 2, 4, 1, EPI_BIAS, IN_F32S, true, false, 0, 2, 1, 0)                  \
  X(16, 1, 2, 4, 1, EPI_BIAS, IN_F32S, true, false, 0, 2, 1, 0)                  \
  X(8, 1, 2, 4, 1, EPI_BIAS, IN_F32S, true, false, 0, 2, 1, 0)                   \
  X(8, 1, 1, 7, 1, EPI_OUT, IN_F32S, true, false, 0, 2, 1, 0)                    \
  X(8, 1, 2, 4, 1, EPI_OUT, IN_F32S, true, false, 0, 2, 1, 0)                   

// Large layers take the AM = 1 variants where they exist: at least ~4 blocks
// of 128 columns per CU, or, for layers with C_in x C_out >= 4096, at least
// 1.5M output values (columns x C_out).  An AM = 1 block runs the whole K loop
// with a barrier per K step, a floor of ~15-25 us on the BBHnet stages; the
// small-batch kernels grow with the batch and cross that floor near this
// size (measured per layer at 8-256 windows).
static bool large_batch(int n, int ncol, int Ci, int Co) {
  const int64_t cols = (int64_t)n * ncol;
  return cols >= 256 * 128 * 4 || (cols * Co >= 1536 * 1024 && Ci * Co >= 4096);
}

int conv_bf16_gap_parts(int Ci, int Co, int Lout, int n) {
  // partial sums per window written by the pooled (EPI_RESID_GAP) variant
  const int mt = (Co + 15) / 16;
  const int am = large_batch(n, Lout, Ci, Co) ? 1 : 0;
#define GW_GAP(CIP, MT, NPH, KT, SC, EPI, IN, OF, XF, CS, NTW, MS, AM) \
  if (EPI == EPI_RESID_GAP && mt == MT && AM == am) return (Lout + 64 * NTW - 1) / (64 * NTW) * MS;
  GW_BF16_VARIANTS(GW_GAP)
#undef GW_GAP
  return -1;
}

bool conv_bf16_supported(int Ci, int Co, int k, int stride, bool tr) {
  // shape-level check: some variant exists for these channels and geometry
  if (k != 7) return false;
  if (tr && stride != 2) return false;
  const Geo g = make_geo(tr, k, stride, 3, 1 << 20);
  const int cip = cip_of(Ci), mt = (Co + 15) / 16;
#define GW_SHAPE(CIP, MT, NPH, KT, SC, EPI, IN, OF, XF, CS, NTW, MS, AM) \
  if (cip == CIP && mt == MT && g.nph == NPH && g.kt == KT && g.sc == SC) return true;
  GW_BF16_VARIANTS(GW_SHAPE)
#undef GW_SHAPE
  return false;
}

// The ABI passes: input format through p.x (fp32), p.xh (bf16) or ring
// (src == SRC_RING), FP32 input split into hi + lo terms when p.wpk_lo (the
// low weight terms) is set; output fp32 when p.y is set and p.yh is not; residual
// shortcut input through p.xs (fp32) or p.xsh (bf16) with weights p.wspk.
hipError_t launch_conv_bf16(const ConvP& p, bool tr, int epi, int src, hipStream_t st) {
  if (p.k != 7 || p.pad != 3) return hipErrorNotSupported;
  const Geo g = make_geo(tr, p.k, p.stride, p.pad, p.Lout);
  Key k;
  k.cip = cip_of(p.Ci);
  k.mt = (p.Co + 15) / 16;
  k.nph = g.nph;
  k.kt = g.kt;
  k.sc = g.sc;
  k.epi = epi;
  k.in = src == SRC_RING ? IN_RING : (p.xh ? IN_BF16 : (p.wpk_lo ? IN_F32S : IN_F32));
  k.out_f32 = (epi == EPI_OUT || p.yh == nullptr) ? 1 : 0;
  const bool res = epi == EPI_RESID_RELU || epi == EPI_RESID_GAP;
  if (epi == EPI_RESID_GAP) k.out_f32 = 1;
  k.xs_f32 = (res && p.xsh == nullptr) ? 1 : 0;
  k.csp = res ? cip_of(p.Cs) : 0;
  if (res && (!p.wspk || p.Ls != 2 * p.Lout)) return hipErrorInvalidValue;
  if (epi == EPI_RESID_GAP && (!p.hw || !p.gap_part)) return hipErrorInvalidValue;
#define GW_LAUNCH(CIP, MT, NPH, KT, SC, EPI, IN, OF, XF, CS, NTW, MS, AM)                        \
  if (k.cip == CIP && k.mt == MT && k.nph == NPH && k.kt == KT && k.sc == SC && k.epi == EPI && \
      k.in == IN && k.out_f32 == (int)OF && k.xs_f32 == (int)XF && k.csp == CS && k.am == AM)   \
    return launch_t<CIP, MT, NPH, KT, SC, EPI, IN, OF, XF, CS, NTW, MS, AM>(p, g, st);
  // the large-batch variant when one exists, else the general one
  k.am = large_batch(p.n, g.ncol, p.Ci, p.Co) ? 1 : 0;
  GW_BF16_VARIANTS(GW_LAUNCH)
  k.am = 0;
  GW_BF16_VARIANTS(GW_LAUNCH)
#undef GW_LAUNCH
  return hipErrorNotSupported;
}

}  // namespace gw

namespace gw {

// ===========================================================================
// Fused DeepClean forward (BF16 or FP16 operands, FP32 accumulation).  One
// block computes T consecutive output samples of one window through all nine
// layers; every intermediate activation stays in LDS.  Working backwards from
// the output tile [u0, u0+T) each layer's needed output positions are a fixed
// range around its scaled tile start (LO and NR below); the input tile is the window's samples
// [u0 - 93, u0 + T + 93) (the receptive field).  Positions outside a layer's
// signal are stored as zeros, i.e. they are the next layer's zero padding, so
// every output equals the layer-by-layer result up to summation order.
// Layers: four k7 s2 p3 convs (C0 -> C1 -> C2 -> C3 -> C4) with folded BN +
// tanh, four k7 s2 p3 op1 transposed convs (C4 -> C5 -> C6 -> C7 -> C8) as
// two 4-tap phases with folded BN + tanh, and the k7 s1 p3 output conv
// C8 -> 1 whose epilogue writes the noise and the causal clean output.
// ===========================================================================
namespace fused {

#ifndef GW_FUSED_T
#define GW_FUSED_T 768
#endif
constexpr int T = GW_FUSED_T;  // output samples per block (a multiple of 256)
static_assert(T % 256 == 0, "tile must hold whole 16-column MFMA tiles at every layer");
#ifndef GW_FUSED_WAVES
#define GW_FUSED_WAVES 12
#endif
constexpr int NW = GW_FUSED_WAVES;  // waves per block
constexpr int NTHR = 64 * NW;
constexpr int C[10] = {21, 8, 16, 32, 64, 32, 16, 8, 8, 1};
constexpr int cip(int c) { return (c + 7) / 8 * 8; }
// LDS row stride (elements): an odd multiple of 8, so 16 lanes reading 16 B
// from 16 consecutive rows hit 16 distinct 16 B bank groups
constexpr int rs(int c) { return (cip(c) / 8) % 2 ? cip(c) : cip(c) + 8; }
// row counts of the layer outputs a1..a8 (and x); row 0 of a_l sits at
// (tile start scaled to layer l) + LO[l]
constexpr int LO[10] = {-93, -45, -21, -9, -3, -3, -3, -3, -3, 0};
constexpr int NR[10] = {T + 187, T / 2 + 91, T / 4 + 43, T / 8 + 19, T / 16 + 7,
                        T / 8 + 7, T / 4 + 7, T / 2 + 7, T + 6, T};
// output columns of layer l: one per output row for the stride-2 convs L1..L3;
// two output rows (2c, 2c + 1) per column for the first conv, whose MFMA
// rows stack the two output times; one input-aligned position per column
// for the transposed layers (rows 2c - 1 and 2c); one per row for the output
// conv
constexpr int NCOL[9] = {(NR[1] + 1) / 2, NR[2], NR[3], NR[4], T / 16 + 4, T / 8 + 4, T / 4 + 4, T / 2 + 4, T};
constexpr int NT(int l) { return (NCOL[l] + 15) / 16; }
constexpr int SC(int l) { return l < 4 ? 2 : 1; }
// input rows between adjacent columns, and input rows one column reads
constexpr int CSTEP(int l) { return l == 0 ? 4 : SC(l); }
constexpr int KT(int l) { return l == 0 ? 9 : l < 4 || l == 8 ? 7 : 4; }
// rows of layer l's input buffer that its (padded) columns may read
constexpr int rows_read(int l) { return CSTEP(l) * (16 * NT(l) - 1) + KT(l); }
constexpr int cap0(int l) { return (rows_read(l) > NR[l] ? rows_read(l) : NR[l]); }
// inputs read with a column step of 2 or 4 rows are stored split by row
// residue (row r at (r mod F) PART + r / F), so adjacent columns read
// adjacent LDS rows; the others row by row
constexpr int SPLITF(int l) { return l < 9 && CSTEP(l) > 1 ? CSTEP(l) : 1; }
constexpr int PART(int l) { return (cap0(l) + SPLITF(l) - 1) / SPLITF(l); }
// the output conv's input rows are stored with one spare row after every 16
// (row r at r + r / 16): its A-operand reads take rows 16 apart in 16 lanes,
// which the spare rows spread over distinct bank groups
constexpr int prow8(int r) { return r + (r >> 4); }
// LDS row of row r of layer l's input buffer
__host__ __device__ constexpr int phys(int l, int r) {
  return SPLITF(l) > 1 ? (r % SPLITF(l)) * PART(l) + r / SPLITF(l) : l == 8 ? prow8(r) : r;
}
constexpr int cap(int l) {  // LDS rows of layer l's input buffer
  return SPLITF(l) > 1 ? SPLITF(l) * PART(l) : l == 8 ? prow8(cap0(l) - 1) + 1 : cap0(l);
}
constexpr int mx(int a, int b) { return a > b ? a : b; }
// ping-pong: inputs of layers 0,2,4,6,8 in buffer A, of layers 1,3,5,7 in B
constexpr int BUFA = mx(mx(mx(cap(0) * rs(C[0]), cap(2) * rs(C[2])), mx(cap(4) * rs(C[4]), cap(6) * rs(C[6]))),
                        cap(8) * rs(C[8]));
constexpr int BUFB = mx(mx(cap(1) * rs(C[1]), cap(3) * rs(C[3])), mx(cap(5) * rs(C[5]), cap(7) * rs(C[7])));
constexpr int MT(int l) { return (C[l + 1] + 15) / 16; }
constexpr int NPH(int l) { return l >= 4 && l < 8 ? 2 : 1; }
constexpr int KS(int l) { return (KT(l) * cip(C[l]) + 31) / 32; }
// transposed layers with 8 output channels stack their two phases on the
// MFMA rows (row = 8 phase + channel), so no accumulator row is padding
// The first conv (8 output channels) stacks two output times the same way
// (row = 8 n + channel, outputs 2c + n of column c, input offsets d = 2 n + j).
constexpr bool STACK(int l) { return l == 0 || (l >= 4 && l < 8 && C[l + 1] == 8); }
// output row of the stacked tile row block q (phase or time offset) of column c
constexpr int ROFF(int l) { return l == 0 ? 0 : -1; }
// the output conv (one channel) is a Toeplitz product with output time on
// both MFMA dimensions: D[m][n] = noise[16 m + n], A[m][(d, i)] = a8[i][16 m +
// d - 3], B[(d, i)][n] = w[i][d - n] (zero outside the kernel), K = 24
// offsets x 8 channels; one MFMA tile covers 256 outputs
constexpr bool TOEP(int l) { return l == 8; }
constexpr int TB = T / 256;  // 256-output tiles of the output conv
constexpr int KS8 = 6;       // K steps of the Toeplitz product (offsets 22, 23 carry zero weights)
// (phase, channel tile) pairs per column tile
constexpr int QP(int l) { return STACK(l) ? 1 : NPH(l) * MT(l); }

}  // namespace fused

struct FusedP {
  const uint16_t* wpk[9];
  const float* scale[9];
  const float* shift[9];
  int L[10];  // signal length of x and of each layer output (window W, W/2, ...)
};

// tanh for the fused epilogue from z = 2 x log2(e) (the factor is folded into
// the BN scale and shift): 1 - 2 / (2^z + 1) on the hardware exp2 and
// reciprocal.  2^z overflows to +inf for large z, giving exactly 1; relative
// error is far below the BF16 rounding of the stored activations.
__device__ __forceinline__ float tanh_scaled(float z) {
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(z) + 1.0f), 1.0f);
}
constexpr float kTwoLog2e = 2.8853900817779268f;

namespace fused {
constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }
constexpr int mn(int a, int b) { return a < b ? a : b; }
// 8-channel layers: the valid accumulator rows sit in lanes 0..31, so two
// column tiles share one epilogue pass (lanes 32..63 take the second tile)
constexpr bool COMPACT(int l) { return l < 8 && !STACK(l) && MT(l) == 1 && cip(C[l + 1]) == 8; }
// A work unit holds at most FMAX weight fragments (32 VGPRs), so all of its
// fragments are requested at once and the next layer's can be requested
// while this layer's epilogue runs.  Layers with more (phase, channel tile)
// pairs x K steps than that split the pairs over SPL units; the others keep
// every pair in one unit.  Compact and stacked layers have a single pair.
constexpr int FMAX = 8;
constexpr int SPL(int l) {
  return COMPACT(l) || STACK(l) || QP(l) * KS(l) <= FMAX ? 1 : QP(l) / 2 * KS(l) <= FMAX && QP(l) % 2 == 0 ? 2 : 4;
}
// column tiles per work unit: enough that every layer is one round of at
// most NW units (at most 4)
constexpr int NTC(int l) {
  return COMPACT(l) ? mn(4, 2 * cdiv(NT(l), 2 * NW)) : mn(4, cdiv(NT(l), NW / SPL(l)));
}
constexpr int NG(int l) { return cdiv(NT(l), NTC(l)); }
constexpr int NU(int l) { return TOEP(l) ? TB : NG(l) * SPL(l); }              // units of layer l
constexpr int NF(int l) { return TOEP(l) ? KS8 : QP(l) / SPL(l) * KS(l); }   // fragments per unit
// fragments requested during the previous layer: at most 7, so that the
// request fits beside that layer's epilogue without spilling; a unit's
// remaining fragment (the last its MFMAs read) is requested as it starts
constexpr int PF(int l) { return NF(l) < 7 ? NF(l) : 7; }
// per-layer table of B-fragment row offsets: KOFF[l][lg][ks] (elements) for
// the 8 channels at kappa = 32 ks + 8 lg, i.e. tap jj = kappa / C_in and
// channel i0 = kappa mod C_in; taps past the kernel (zero weights) read tap
// K-1 instead, a row that holds finite values
constexpr int KSMAX = 8;
__host__ __device__ constexpr int koff(int l, int lg, int ks) {
  const int kappa = 32 * ks + 8 * lg, jj = kappa / cip(C[l]), i0 = kappa - jj * cip(C[l]);
  const int j = jj < KT(l) ? jj : KT(l) - 1;
  return phys(l, j) * rs(C[l]) + i0;
}
constexpr bool units_fit(int l) {
  return l == 9 || (NU(l) <= NW && NF(l) <= FMAX && QP(l) % SPL(l) == 0 && units_fit(l + 1));
}
static_assert(units_fit(0), "every layer is one round of units of at most FMAX fragments");
}  // namespace fused

// Two floats -> packed bf16 pair, first in the low half: the hardware
// conversion, which rounds to nearest even exactly like bf16_rne (NaNs
// included).
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){lo, hi}, bf16x2_t));
}

// Two floats -> packed IEEE half pair (round to nearest even), first in the
// low half.
__device__ __forceinline__ uint32_t pack_f16x2(float lo, float hi) {
  typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){lo, hi}, f16x2_t));
}

// The fused kernel's 16-bit element type: BF16 (default) or FP16.
template <bool F16>
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
  if constexpr (F16)
    return pack_f16x2(lo, hi);
  else
    return pack_bf16x2(lo, hi);
}

// 16x16x32 MFMA on 8 packed 16-bit values per lane, FP32 accumulation
template <bool F16>
__device__ __forceinline__ f32x4 mfma16(const uint4& a, const uint4& b, const f32x4& c) {
  if constexpr (F16) {
    typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                  0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  }
}

// BN + tanh of channels o0..o0+3 of one output row of layer l (scale and
// shift pre-multiplied by 2 log2 e), stored as four bf16 in one 8 B LDS
// write.  Positions outside the layer's signal are stored as zeros (the next
// layer's padding); only tiles at a window edge (EDGE) have any.  Every
// C_out here is a multiple of 8, so no stored channel is padding.
template <int l, bool EDGE, bool F16>
__device__ __forceinline__ void epi_row(uint16_t* out, int row, int o0, f32x4 v, float4 sc, float4 sh, int pos0,
                                        int Lout) {
  using namespace fused;
  constexpr int RSO = rs(C[l + 1]);
  static_assert(C[l + 1] % 8 == 0, "stored channel groups are never padding");
  if (row < 0 || row >= NR[l + 1]) return;
  float t0 = tanh_scaled(fmaf(v[0], sc.x, sh.x)), t1 = tanh_scaled(fmaf(v[1], sc.y, sh.y));
  float t2 = tanh_scaled(fmaf(v[2], sc.z, sh.z)), t3 = tanh_scaled(fmaf(v[3], sc.w, sh.w));
  if (EDGE) {
    const int u = pos0 + row;
    const bool live = u >= 0 && u < Lout;
    t0 = live ? t0 : 0.0f;
    t1 = live ? t1 : 0.0f;
    t2 = live ? t2 : 0.0f;
    t3 = live ? t3 : 0.0f;
  }
  const int prow = phys(l + 1, row);
  *reinterpret_cast<uint2*>(out + prow * RSO + o0) = make_uint2(pack2<F16>(t0, t1), pack2<F16>(t2, t3));
}

// Epilogue of one work unit (see fused_layer).
template <int l, bool EDGE, int NTCl, int Q, bool F16>
__device__ __forceinline__ void fused_epi(const f32x4 (&acc)[NTCl][Q], int nt0, int sp, int lc, int lg, uint16_t* out,
                                          const float* ksc, const float* ksh, int pos0, int Lout, const ConvP* op,
                                          int b, int Wout) {
  using namespace fused;
  constexpr int CIPO = cip(C[l + 1]), M = MT(l), P = NPH(l), NTn = NT(l), SP = SPL(l);
  (void)op;
  (void)b;
  (void)Wout;
  static_assert(!TOEP(l), "the output conv has its own layer function");
  if constexpr (STACK(l)) {
    // rows 8 ph + o: lanes 0..31 hold phase (time offset) 0, lanes 32..63
    // phase 1, each lane four channels 4 (lg & 1) .. + 3 of column c
    static_assert(SP == 1 && Q == 1, "stacked layers: one (phases x channels) tile per column");
    const int o0 = 4 * (lg & 1), ph = lg >> 1;
    const float4 sc4 = *reinterpret_cast<const float4*>(ksc + o0);
    const float4 sh4 = *reinterpret_cast<const float4*>(ksh + o0);
#pragma unroll
    for (int a = 0; a < NTCl; ++a) {
      if (nt0 + a >= NTn) break;
      const int c = (nt0 + a) * 16 + lc;
      epi_row<l, EDGE, F16>(out, 2 * c + ph + ROFF(l), o0, acc[a][0], sc4, sh4, pos0, Lout);
    }
  } else if constexpr (COMPACT(l)) {
    // tiles a, a+1: lanes 0..31 keep tile a's channels 0..7, lanes 32..63
    // receive tile a+1's (its lanes 0..31) through a 32-lane swap
    static_assert(SP == 1 && Q == P, "compact layers keep both phases in one unit");
    const int o0 = 4 * (lg & 1);
    const float4 sc4 = *reinterpret_cast<const float4*>(ksc + o0);
    const float4 sh4 = *reinterpret_cast<const float4*>(ksh + o0);
#pragma unroll
    for (int a = 0; a < NTCl; a += 2) {
      if (nt0 + a >= NTn) break;
      if (a + 1 < NTCl && nt0 + a + 1 < NTn) {
        const int c = (nt0 + a + (lg >> 1)) * 16 + lc;
#pragma unroll
        for (int ph = 0; ph < P; ++ph) {
          f32x4 v;
#pragma unroll
          for (int r = 0; r < 4; ++r)
            v[r] = __uint_as_float(__builtin_amdgcn_permlane32_swap(__float_as_uint(acc[a][ph][r]),
                                                                    __float_as_uint(acc[a + 1][ph][r]), false,
                                                                    false)[0]);
          epi_row<l, EDGE, F16>(out, P == 1 ? c : 2 * c + ph - 1, o0, v, sc4, sh4, pos0, Lout);
        }
      } else if (lg < 2) {
        const int c = (nt0 + a) * 16 + lc;
#pragma unroll
        for (int ph = 0; ph < P; ++ph)
          epi_row<l, EDGE, F16>(out, P == 1 ? c : 2 * c + ph - 1, o0, acc[a][ph], sc4, sh4, pos0, Lout);
      }
    }
  } else {
    // four consecutive channels per lane and row, one 8 B store each
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int q = sp + k * SP, ph = q / M, mt = q % M;
      const int o0 = 16 * mt + 4 * lg;
      if (o0 >= CIPO) continue;
      const float4 sc4 = *reinterpret_cast<const float4*>(ksc + o0);
      const float4 sh4 = *reinterpret_cast<const float4*>(ksh + o0);
#pragma unroll
      for (int a = 0; a < NTCl; ++a) {
        if (nt0 + a >= NTn) break;
        const int c = (nt0 + a) * 16 + lc;
        epi_row<l, EDGE, F16>(out, P == 1 ? c : 2 * c + ph - 1, o0, acc[a][k], sc4, sh4, pos0, Lout);
      }
    }
  }
}

// One layer of the fused network: LDS in -> LDS out (or global for the last).
// Work units are (group of NTC column tiles, share of the (phase, channel
// tile) pairs); every layer has at most NW units and unit u runs on wave u.
// The 92 KB of packed weights stay in L2, shared by every block; a unit's
// fragments (at most FMAX) arrive in wf, requested while the previous
// layer's epilogue ran, and once its MFMAs have read them the wave requests
// its fragments of the next layer into the same registers.  kt holds the
// layer's row of the B-offset table.
//
// Request wave `wave`'s weight fragments [I0, I1) of layer l into wf:
// fragment i = k KS + ks (pair q = sp + k SPL, K step ks) of unit `wave`,
// sp = wave mod SPL, at [q][ks][lane] in the layer's pack (the output conv:
// fragment ks at [ks][lane]).
template <int l, int I0, int I1>
__device__ __forceinline__ void fused_frags(u32x4 (&wf)[fused::FMAX], const uint4* wg, int wave, int lane) {
  using namespace fused;
  if (I0 >= I1 || wave >= NU(l)) return;  // wave-uniform
  const u32x4* wq = reinterpret_cast<const u32x4*>(wg) + lane;
  if constexpr (TOEP(l)) {
#pragma unroll
    for (int ks = I0; ks < I1; ++ks) wf[ks] = wq[ks * 64];
  } else {
    constexpr int KSn = KS(l), SP = SPL(l);
    const int sp = wave % SP;
#pragma unroll
    for (int i = I0; i < I1; ++i) wf[i] = wq[(sp * KSn + (i / KSn) * SP * KSn + i % KSn) * 64];
  }
}

// The output conv as a Toeplitz product (see TOEP): wave w < TB computes
// outputs [256 w, 256 w + 256) of the tile with KS8 MFMAs whose A operand
// (8 channels at one time offset per lane) comes from LDS and whose B
// operand (the banded weights) from the packed fragments; the epilogue
// writes the noise and the fully-online clean output.  The fragments of the
// next tile's first layer are requested after the MFMAs (wgn).
template <bool F16>
__device__ __forceinline__ void fused_toeplitz(int tid, const uint16_t* in, u32x4 (&wf)[fused::FMAX],
                                               const uint4* wgn, const float* ksc, const float* ksh, int pos0,
                                               const ConvP* op, int b, int Wout) {
  using namespace fused;
  constexpr int RSI = rs(C[8]);
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lc = lane & 15, lg = lane >> 4;
  static_assert(PF(8) == NF(8), "the output conv's fragments all arrive with the previous layer");
  if (wave >= TB) {  // wave-uniform
    fused_frags<0, 0, PF(0)>(wf, wgn, wave, lane);
    return;
  }
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS8; ++ks) {
    // offset d of this lane's eight K entries; offsets past the kernel's
    // reach (zero weights) read the last real one, a row of finite values
    const int d = mn(4 * ks + lg, 21);
    const int r = 256 * wave + 16 * lc + d;
    const uint4 av = *reinterpret_cast<const uint4*>(in + prow8(r) * RSI);
    acc = mfma16<F16>(av, __builtin_bit_cast(uint4, wf[ks]), acc);
  }
  fused_frags<0, 0, PF(0)>(wf, wgn, wave, lane);
  __builtin_amdgcn_s_setprio(1);  // epilogue ahead of MFMA chains, as in fused_layer_mm
  // D[m = 4 lg + q][n = lc]: output 16 m + n of this wave's 256
  const float sc = ksc[0], sh = ksh[0];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int u = pos0 + 256 * wave + 16 * (4 * lg + q) + lc;
    if (u < 0 || u >= Wout) continue;
    const float v = fmaf(acc[q], sc, sh);
    if (op->noise) op->noise[(int64_t)b * Wout + u] = v;
    if (op->clean) {
      const Item& it = op->items[b];
      const int t0 = Wout - it.s - it.delay;
      if (u >= t0 && u < t0 + it.s) {
        const int64_t idx = it.out + (u - t0);
        op->clean[idx] = op->strain[idx] - v;
      }
    }
  }
  __builtin_amdgcn_s_setprio(0);
}

template <int l, bool F16>
__device__ __forceinline__ void fused_layer_mm(int tid, const uint16_t* in, uint16_t* out, u32x4 (&wf)[fused::FMAX],
                                               const uint4* wg, const uint4* wgn, const int* kt, const float* ksc,
                                               const float* ksh, int pos0, int Lout, const ConvP* op, int b,
                                               int Wout) {
  using namespace fused;
  constexpr int RSI = rs(C[l]);
  constexpr int KSn = KS(l), NTn = NT(l);
  constexpr int NTCl = NTC(l), SP = SPL(l), Q = QP(l) / SP;
  constexpr int SX = SPLITF(l) > 1 ? 1 : CSTEP(l);  // LDS rows between adjacent columns
  static_assert(KSn <= KSMAX, "offset table width");
  // the wave index is uniform: in an SGPR, unit selection and the weight
  // addresses are scalar work
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lc = lane & 15, lg = lane >> 4;
  // this lane's B row offsets for the layer's K steps
  int ko[KSMAX];
  {
    const int4 k0 = *reinterpret_cast<const int4*>(kt + KSMAX * lg);
    const int4 k1 = *reinterpret_cast<const int4*>(kt + KSMAX * lg + 4);
    ko[0] = k0.x; ko[1] = k0.y; ko[2] = k0.z; ko[3] = k0.w;
    ko[4] = k1.x; ko[5] = k1.y; ko[6] = k1.z; ko[7] = k1.w;
  }
  // window-edge tiles store zeros outside the signal
  const bool edge = pos0 < 0 || pos0 + NR[l + 1] > Lout;
  if (wave >= NU(l)) {  // wave-uniform
    fused_frags<l + 1, 0, PF(l + 1)>(wf, wgn, wave, lane);
    return;
  }
  fused_frags<l, PF(l), NF(l)>(wf, wg, wave, lane);
  {
    const int unit = wave;
    const int nt0 = (unit / SP) * NTCl, sp = unit % SP;  // wave-uniform
    const uint16_t* colbase = in + ((nt0 * 16 + lc) * SX) * RSI;
    f32x4 acc[NTCl][Q];
#pragma unroll
    for (int a = 0; a < NTCl; ++a)
#pragma unroll
      for (int k = 0; k < Q; ++k) acc[a][k] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KSn; ++ks) {
      const uint16_t* src = colbase + ko[ks];
      // the K step's B fragments of every column tile, read together; tiles
      // past the layer's last re-read that one (their sums are never stored)
      uint4 bb[NTCl];
#pragma unroll
      for (int a = 0; a < NTCl; ++a) {
        const int aa = a < NTn - nt0 ? a : NTn - 1 - nt0;  // wave-uniform
        bb[a] = *reinterpret_cast<const uint4*>(src + aa * 16 * SX * RSI);
      }
#pragma unroll
      for (int a = 0; a < NTCl; ++a)
#pragma unroll
        for (int k = 0; k < Q; ++k)
          acc[a][k] = mfma16<F16>(__builtin_bit_cast(uint4, wf[k * KSn + ks]), bb[a], acc[a][k]);
    }
    fused_frags<l + 1, 0, PF(l + 1)>(wf, wgn, wave, lane);
    // a layer ends when its slowest wave's epilogue does: waves in their
    // epilogue issue ahead of waves still in their MFMA chains
    __builtin_amdgcn_s_setprio(1);
    if (edge)
      fused_epi<l, true, NTCl, Q, F16>(acc, nt0, sp, lc, lg, out, ksc, ksh, pos0, Lout, op, b, Wout);
    else
      fused_epi<l, false, NTCl, Q, F16>(acc, nt0, sp, lc, lg, out, ksc, ksh, pos0, Lout, op, b, Wout);
    __builtin_amdgcn_s_setprio(0);
  }
}

template <int l, bool F16>
__device__ __forceinline__ void fused_layer(int tid, const uint16_t* in, uint16_t* out, u32x4 (&wf)[fused::FMAX],
                                            const uint4* wg, const uint4* wgn, const int* kt, const float* ksc,
                                            const float* ksh, int pos0, int Lout, const ConvP* op, int b, int Wout) {
  if constexpr (fused::TOEP(l))
    fused_toeplitz<F16>(tid, in, wf, wgn, ksc, ksh, pos0, op, b, Wout);
  else
    fused_layer_mm<l, F16>(tid, in, out, wf, wg, wgn, kt, ksc, ksh, pos0, Lout, op, b, Wout);
}

// ---------------------------------------------------------------------------
// Input staging of the fused kernel.  An item is (group of four channels,
// 8-sample chunk): four 16 B loads (one per channel, BF16 ring shadow; two
// per channel for FP32 input) that share one address computation, transposed
// in registers into eight rows of four channels, each written with one 8 B
// LDS store.  Lanes take consecutive channel groups first, so a row's groups
// are contiguous in LDS.  Rows are stored even rows first, then odd rows
// (layer 0 reads with stride 2).
// ---------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
namespace fused {
constexpr int XG = cip(C[0]) / 4;                  // channel groups of x
// staged input rows: every row layer 0's columns read (a column's MFMA rows
// take both output times, so rows past the needed range are read with zero
// weights and must hold finite values: they get the window's real samples)
constexpr int XROWS = cap0(0);
constexpr int XCH = (XROWS + 7 + 7) / 8;           // chunks covering XROWS rows at any alignment
constexpr int XITEMS = cdiv(XG * XCH, NTHR);       // items per thread
}  // namespace fused

template <int IN>
struct XRaw {
  static constexpr int NV = IN == IN_F32 || IN == IN_RING_F32 ? 2 : 1;  // 16 B pieces per channel chunk
  u32x4 v[fused::XITEMS][4][NV];
};

// one channel's 8-sample chunk at positions [qc, qc + 8) of the window; zeros
// outside [0, Lin) and for channels >= Ci
template <int IN>
__device__ __forceinline__ void load_chunk(u32x4 (&d)[XRaw<IN>::NV], const uint16_t* hrow, const float* frow,
                                           int head, int ld, int Lin, int qc, bool vec) {
  constexpr int NV = XRaw<IN>::NV;
  constexpr bool F32SRC = IN == IN_F32 || IN == IN_RING_F32;
#pragma unroll
  for (int k = 0; k < NV; ++k) d[k] = u32x4{0u, 0u, 0u, 0u};
  if (vec && qc >= 0 && qc + 8 <= Lin) {
    if (IN == IN_F32) {
      d[0] = *reinterpret_cast<const u32x4*>(frow + qc);
      d[NV - 1] = *reinterpret_cast<const u32x4*>(frow + qc + 4);
    } else if (IN == IN_RING_F32) {
      // an aligned 8-sample chunk never straddles the ring's wrap point
      int ph = head + qc;
      if (ph >= ld) ph -= ld;
      d[0] = *reinterpret_cast<const u32x4*>(frow + ph);
      d[NV - 1] = *reinterpret_cast<const u32x4*>(frow + ph + 4);
    } else {
      int ph = qc;
      if (IN == IN_RING) {
        ph = head + qc;
        if (ph >= ld) ph -= ld;
      }
      d[0] = *reinterpret_cast<const u32x4*>(hrow + ph);
    }
  } else {
    uint32_t w[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int q = qc + e;
      w[e] = 0;
      if (q >= 0 && q < Lin) {
        if (IN == IN_F32) {
          w[e] = __float_as_uint(frow[q]);
        } else if (IN == IN_RING_F32) {
          int ph = head + q;
          if (ph >= ld) ph -= ld;
          w[e] = __float_as_uint(frow[ph]);
        } else {
          int ph = q;
          if (IN == IN_RING) {
            ph = head + q;
            if (ph >= ld) ph -= ld;
          }
          w[e] = hrow[ph];
        }
      }
    }
    if (F32SRC) {
      d[0] = u32x4{w[0], w[1], w[2], w[3]};
      d[NV - 1] = u32x4{w[4], w[5], w[6], w[7]};
    } else {
      d[0] = u32x4{w[0] | (w[1] << 16), w[2] | (w[3] << 16), w[4] | (w[5] << 16), w[6] | (w[7] << 16)};
    }
  }
}

// Issue the loads of a tile's input rows [q0, q0 + XROWS) of window b
// (tid: the thread index).
template <int IN>
__device__ __forceinline__ void load_x(XRaw<IN>& R, const ConvP& p, int b, int q0, int tid) {
  using namespace fused;
  const int Ci = p.Ci, Lin = p.Lin;
  const int qa = q0 - (((q0 % 8) + 8) % 8);
  const int nch = (q0 + XROWS - qa + 7) / 8;
  int head = 0, ld = p.ldx ? p.ldx : Lin;
  const uint16_t* hbase = nullptr;
  const float* fbase = nullptr;
  bool vec;
  if (IN == IN_RING) {
    const Item& it = p.items[b];
    head = it.head;
    ld = it.W;
    hbase = reinterpret_cast<const uint16_t*>(p.arena) + it.shadow;
    vec = (ld & 7) == 0 && (head & 7) == 0 && (it.shadow & 7) == 0;
  } else if (IN == IN_RING_F32) {
    const Item& it = p.items[b];
    head = it.head;
    ld = it.W;
    fbase = reinterpret_cast<const float*>(p.arena) + it.ring;
    vec = (ld & 7) == 0 && (head & 7) == 0 && (it.ring & 3) == 0;
  } else {
    fbase = p.x + (int64_t)b * Ci * ld;
    vec = (ld & 7) == 0 && (reinterpret_cast<uintptr_t>(p.x) & 15) == 0;
  }
#pragma unroll
  for (int it = 0; it < XITEMS; ++it) {
    const int e = tid + NTHR * it;
    const int g = e % XG, ch = e / XG;
    const int qc = qa + 8 * ch;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = 4 * g + k;
      const bool on = ch < nch && i < Ci;
      const int64_t ro = (int64_t)(on ? i : 0) * ld;
      load_chunk<IN>(R.v[it][k], hbase + (IN == IN_RING ? ro : 0), fbase + (IN != IN_RING ? ro : 0), head, ld,
                     on ? Lin : 0, qc, vec);
    }
  }
}

// Write the staged rows to LDS (row stride RS, split by row residue mod 4).
template <int IN, bool F16>
__device__ __forceinline__ void store_x(uint16_t* tile, const XRaw<IN>& R, int q0, int tid) {
  static_assert(!(F16 && IN == IN_RING), "the ring's 16-bit shadow is BF16");
  using namespace fused;
  constexpr int RS = rs(C[0]), ROWS = XROWS;
  static_assert(SPLITF(0) == 4, "layer 0's columns step four input rows");
  const int qa = q0 - (((q0 % 8) + 8) % 8);
  const int nch = (q0 + ROWS - qa + 7) / 8;
#pragma unroll
  for (int it = 0; it < XITEMS; ++it) {
    const int e = tid + NTHR * it;
    const int g = e % XG, ch = e / XG;
    if (ch >= nch) continue;
    // bf16 pairs of each channel: c[k][d] holds samples 2d, 2d+1
    uint32_t c[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (IN == IN_F32 || IN == IN_RING_F32) {
        const u32x4 a = R.v[it][k][0], z = R.v[it][k][XRaw<IN>::NV - 1];
        c[k][0] = pack2<F16>(__uint_as_float(a.x), __uint_as_float(a.y));
        c[k][1] = pack2<F16>(__uint_as_float(a.z), __uint_as_float(a.w));
        c[k][2] = pack2<F16>(__uint_as_float(z.x), __uint_as_float(z.y));
        c[k][3] = pack2<F16>(__uint_as_float(z.z), __uint_as_float(z.w));
      } else {
        const u32x4 a = R.v[it][k][0];
        c[k][0] = a.x; c[k][1] = a.y; c[k][2] = a.z; c[k][3] = a.w;
      }
    }
    const int r0 = qa + 8 * ch - q0;  // row of the chunk's first sample
    const bool full = r0 >= 0 && r0 + 8 <= ROWS;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int d = t >> 1;
      uint32_t lo, hi;
      if (t & 1) {
        lo = (c[0][d] >> 16) | (c[1][d] & 0xffff0000u);
        hi = (c[2][d] >> 16) | (c[3][d] & 0xffff0000u);
      } else {
        lo = (c[0][d] & 0xffffu) | (c[1][d] << 16);
        hi = (c[2][d] & 0xffffu) | (c[3][d] << 16);
      }
      const int r = r0 + t;
      if (full || (r >= 0 && r < ROWS))
        *reinterpret_cast<uint2*>(tile + phys(0, r) * RS + 4 * g) = make_uint2(lo, hi);
    }
  }
}

// Fused snapshot update: the item carries the head after the update, and
// its [C][s] new samples (FP32 at p.upd + src) belong at window positions
// [W - s, W), ring positions h0, h0+1, ... (mod W), h0 = head - s.  Before a
// tile stages its input rows [q0, q0 + XROWS), the block writes the new
// samples among them (widened to whole groups of four) to the ring and its
// BF16 shadow, exactly as the snapshot update writes them; after a barrier
// the rows are read from the shadow as usual.  Every new position lies in
// some tile's rows, so the launch writes them all; blocks whose rows overlap
// write the same values.  No tile reads the positions the new samples
// replace (they held the oldest samples, which left the window).
// Returns false, writing nothing, when the rows hold no new sample
// (block-uniform).
__device__ __forceinline__ bool upd_stage(const ConvP& p, int b, int q0, int tid) {
  const Item& it = p.items[b];
  const int s = it.s, W = it.W, snew = W - s;
  int lo = q0 > snew ? q0 : snew, hi = q0 + fused::XROWS < W ? q0 + fused::XROWS : W;
  if (lo >= hi) return false;
  // the arena is the pool's device memory; the launch owns these positions
  float* ring = reinterpret_cast<float*>(const_cast<void*>(p.arena)) + it.ring;
  uint16_t* sh = reinterpret_cast<uint16_t*>(const_cast<void*>(p.arena)) + it.shadow;
  const float* src = p.upd + it.src;
  int h0 = it.head - s;
  if (h0 < 0) h0 += W;
  const bool vec = ((s | h0 | W) & 3) == 0 && (it.src & 3) == 0 && (it.ring & 3) == 0 && (it.shadow & 3) == 0 &&
                   (reinterpret_cast<uintptr_t>(p.upd) & 15) == 0;
  if (vec) {
    // groups of four samples of one channel; snew, W, s and h0 are multiples
    // of 4, so a group stays inside [snew, W) and never straddles the wrap
    lo = lo - ((lo - snew) & 3);
    const int n4 = (hi - lo + 3) / 4, total = it.C * n4;
    for (int g = tid; g < total; g += fused::NTHR) {
      const int c = g / n4, q = lo + 4 * (g - c * n4) - snew;  // sample index within the new block
      int ph = h0 + q;
      if (ph >= W) ph -= W;
      const float4 v = *reinterpret_cast<const float4*>(src + (int64_t)c * s + q);
      *reinterpret_cast<float4*>(ring + (int64_t)c * W + ph) = v;
      ushort4 h;
      h.x = f2bf(v.x);
      h.y = f2bf(v.y);
      h.z = f2bf(v.z);
      h.w = f2bf(v.w);
      *reinterpret_cast<ushort4*>(sh + (int64_t)c * W + ph) = h;
    }
  } else {
    const int n1 = hi - lo, total = it.C * n1;
    for (int g = tid; g < total; g += fused::NTHR) {
      const int c = g / n1, q = lo + (g - c * n1) - snew;
      int ph = h0 + q;
      if (ph >= W) ph -= W;
      const float v = src[(int64_t)c * s + q];
      ring[(int64_t)c * W + ph] = v;
      sh[(int64_t)c * W + ph] = f2bf(v);
    }
  }
  return true;
}

#ifndef GW_FUSED_WAVES_PER_SIMD
#define GW_FUSED_WAVES_PER_SIMD 6
#endif
template <int IN, bool F16, bool UPD = false>
__global__ __launch_bounds__(fused::NTHR, GW_FUSED_WAVES_PER_SIMD) void dc_fused(ConvP p, FusedP f, int ntile) {
  using namespace fused;
  __shared__ __attribute__((aligned(16))) uint16_t bufA[BUFA];
  __shared__ __attribute__((aligned(16))) uint16_t bufB[BUFB];
  __shared__ __attribute__((aligned(16))) int ktab[9][4][KSMAX];
  __shared__ __attribute__((aligned(16))) float ksc[9][64];
  __shared__ __attribute__((aligned(16))) float ksh[9][64];

  const int W = f.L[0];
  const int tpw = (W + T - 1) / T;  // tiles per window
  const int G = gridDim.x, j = blockIdx.x;
  const int t0 = (int)((int64_t)ntile * j / G), t1 = (int)((int64_t)ntile * (j + 1) / G);
  if (t0 >= t1) return;  // block-uniform

  XRaw<IN> raw;
  if (UPD && upd_stage(p, t0 / tpw, (t0 % tpw) * T + LO[0], threadIdx.x)) __syncthreads();
  load_x<IN>(raw, p, t0 / tpw, (t0 % tpw) * T + LO[0], threadIdx.x);
  u32x4 wf[FMAX];  // this wave's weight fragments of the current layer
  fused_frags<0, 0, PF(0)>(wf, reinterpret_cast<const uint4*>(f.wpk[0]),
                           __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), threadIdx.x & 63);
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    if (threadIdx.x < 64) {
      const int oc = (int)threadIdx.x < C[l + 1] ? (int)threadIdx.x : C[l + 1] - 1;
      const float g = l < 8 ? kTwoLog2e : 1.0f;  // tanh layers take z = 2 x log2(e)
      ksc[l][threadIdx.x] = f.scale[l][oc] * g;
      ksh[l][threadIdx.x] = f.shift[l][oc] * g;
    }
    if (threadIdx.x < 4 * KSMAX) {
      const int lg = threadIdx.x / KSMAX, ks = threadIdx.x % KSMAX;
      ktab[l][lg][ks] = ks < KS(l) ? koff(l, lg, ks) : 0;
    }
  }
  // input tile rows [u0 - 93, u0 + T + 93) in [time][channel] layout
  store_x<IN, F16>(bufA, raw, (t0 % tpw) * T + LO[0], threadIdx.x);
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const int b = t / tpw, u0 = (t % tpw) * T;
    const bool more = t + 1 < t1;  // block-uniform

    // layer l reads the buffer holding a_l and writes a_{l+1}; u0 scaled per
    // layer; an opaque copy of the thread index keeps each layer's address
    // arithmetic inside the tile loop instead of live across it
#define GW_FUSED_LAYER(l, IN_BUF, OUT_BUF, SCALE_DIV)                                                       \
    {                                                                                                       \
      int tid = threadIdx.x;                                                                                \
      asm volatile("" : "+v"(tid));                                                                         \
      fused_layer<l, F16>(tid, IN_BUF, OUT_BUF, wf, reinterpret_cast<const uint4*>(f.wpk[l]),               \
                          reinterpret_cast<const uint4*>(f.wpk[(l + 1) % 9]), &ktab[l][0][0], ksc[l], ksh[l],  \
                          u0 / (SCALE_DIV) + LO[l + 1], W / (SCALE_DIV), &p, b, W);                         \
      __syncthreads();                                                                                      \
    }
    GW_FUSED_LAYER(0, bufA, bufB, 2)
    GW_FUSED_LAYER(1, bufB, bufA, 4)
    GW_FUSED_LAYER(2, bufA, bufB, 8)
    GW_FUSED_LAYER(3, bufB, bufA, 16)
    GW_FUSED_LAYER(4, bufA, bufB, 8)
    GW_FUSED_LAYER(5, bufB, bufA, 4)
    GW_FUSED_LAYER(6, bufA, bufB, 2)
    GW_FUSED_LAYER(7, bufB, bufA, 1)
    GW_FUSED_LAYER(8, bufA, bufB, 1)
#undef GW_FUSED_LAYER
    if (more) {
      // the next tile's input: the other block on the CU hides its latency
      // (an opaque copy of the thread index, as for the layers)
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      const int nq = ((t + 1) % tpw) * T + LO[0];
      if (UPD && upd_stage(p, (t + 1) / tpw, nq, tid)) __syncthreads();
      __builtin_amdgcn_s_setprio(2);  // ahead of the other block's epilogues
      load_x<IN>(raw, p, (t + 1) / tpw, nq, tid);
      store_x<IN, F16>(bufA, raw, nq, tid);
      __builtin_amdgcn_s_setprio(0);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Weight fragments of the fused kernel's restructured layers: the stacked
// transposed layers (STACK: [ks][lane][8], row lane % 16 = 8 phase + output
// channel, K = tap x input channel as for the per-layer kernels), the stacked
// first conv (row 8 n + output channel, K = input offset x channel) and the
// Toeplitz output conv (TOEP: [ks][lane][8], the B operand W[(d, i)][n] =
// w[0][i][d - n] with n = lane % 16, d = 4 ks + lane / 16, i = element).
// ---------------------------------------------------------------------------
__global__ void pack_fused_kernel(const float* w, uint16_t* out, int kind, int Ci, int Co, int cipi, int kt,
                                  int padc, int total, int f16) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int e = idx & 7, lane = (idx >> 3) & 63, ks = idx >> 9;
  float v = 0.0f;
  if (kind == 2) {
    // stacked stride-2 conv: row 8 n + o, K = input offset d (0..kt-1) x channel; tap j = d - 2 n
    const int row = lane & 15, n = row >> 3, o = row & 7;
    const int kappa = 32 * ks + 8 * (lane >> 4) + e, d = kappa / cipi, i = kappa % cipi, j = d - 2 * n;
    if (o < Co && i < Ci && d < kt && j >= 0 && j < 7) v = w[((int64_t)o * Ci + i) * 7 + j];
  } else if (kind == 1) {
    const int n = lane & 15, d = 4 * ks + (lane >> 4), j = d - n;
    if (e < Ci && j >= 0 && j < 7) v = w[e * 7 + j];
  } else {
    const int row = lane & 15, ph = row >> 3, o = row & 7;
    const int kappa = 32 * ks + 8 * (lane >> 4) + e, jj = kappa / cipi, i = kappa % cipi;
    const int d = jj - padc, j = ph + 3 - 2 * d;  // tap of phase ph at input offset d (k7 s2 p3)
    if (o < Co && i < Ci && jj < kt && j >= 0 && j < 7) v = w[((int64_t)i * Co + o) * 7 + j];
  }
  out[idx] = f16 ? __builtin_bit_cast(uint16_t, (_Float16)v) : bf16_rne(v);
}

bool dc_fused_special(int l) { return l >= 0 && l < 9 && (fused::STACK(l) || fused::TOEP(l)); }

size_t dc_fused_special_elems(int l) {
  return dc_fused_special(l) ? (size_t)(fused::TOEP(l) ? fused::KS8 : fused::KS(l)) * 512 : 0;
}

hipError_t launch_pack_fused(const float* w, uint16_t* out, int l, hipStream_t st, bool f16) {
  using namespace fused;
  if (!dc_fused_special(l)) return hipErrorInvalidValue;
  const Geo g = make_geo(true, 7, 2, 3, 1 << 20);
  const int total = (int)dc_fused_special_elems(l);
  const int kind = TOEP(l) ? 1 : l == 0 ? 2 : 0;
  hipLaunchKernelGGL(pack_fused_kernel, dim3((total + 255) / 256), dim3(256), 0, st, w, out, kind, C[l], C[l + 1],
                     cip(C[l]), l == 0 ? KT(0) : g.kt, g.padc, total, f16 ? 1 : 0);
  return hipGetLastError();
}

bool dc_fused_supported(const int* ci, const int* co, const int* type, const int* k, const int* s,
                        const int* pad, const int* op, const int* bn, int L) {
  using namespace fused;
  if (L != 9) return false;
  for (int l = 0; l < 9; ++l) {
    if (ci[l] != C[l] || co[l] != C[l + 1] || k[l] != 7 || pad[l] != 3) return false;
    const bool tr = l >= 4 && l < 8;
    if (type[l] != (tr ? 1 : 0) || s[l] != (l == 8 ? 1 : 2) || op[l] != (tr ? 1 : 0)) return false;
    if (bn[l] != (l == 8 ? 0 : 1)) return false;
  }
  return true;
}

// p: n, items (ring input or clean outputs), arena, x (+ ldx), noise, clean,
// strain; W = window (or band) length, a multiple of 16.
hipError_t launch_dc_fused_bf16(const ConvP& p, const uint16_t* const* wpk, const float* const* scale,
                                const float* const* shift, int W, bool ring, int cu_budget, hipStream_t st,
                                bool f16, bool upd) {
  using namespace fused;
  if (W < 16 || W % 16) return hipErrorInvalidValue;
  if (upd && (!ring || f16 || !p.upd)) return hipErrorInvalidValue;
  FusedP f;
  for (int l = 0; l < 9; ++l) {
    f.wpk[l] = wpk[l];
    f.scale[l] = scale[l];
    f.shift[l] = shift[l];
  }
  f.L[0] = W;
  f.L[1] = W / 2;
  f.L[2] = W / 4;
  f.L[3] = W / 8;
  f.L[4] = W / 16;
  f.L[5] = W / 8;
  f.L[6] = W / 4;
  f.L[7] = W / 2;
  f.L[8] = W;
  f.L[9] = W;
  ConvP q = p;
  q.Lin = W;
  q.Ci = C[0];
  const int64_t ntile = (int64_t)p.n * ((W + T - 1) / T);
  if (ntile > (int64_t)1 << 30) return hipErrorInvalidValue;
  // one resident grid: (blocks per CU) x CUs, at most one block per tile
  // variants: (ring or dense input) x (BF16 or FP16); the FP16 variant reads
  // the ring's FP32 samples (its 16-bit shadow is BF16)
  // and the ring variant under a fused snapshot update
  void (*kern[5])(ConvP, FusedP, int) = {dc_fused<IN_F32, false>, dc_fused<IN_RING, false>,
                                         dc_fused<IN_F32, true>, dc_fused<IN_RING_F32, true>,
                                         dc_fused<IN_RING, false, true>};
  static int occ[5] = {0, 0, 0, 0, 0}, cus = 0;
  const int v = upd ? 4 : (ring ? 1 : 0) + (f16 ? 2 : 0);
  if (!occ[v]) {
    int dev = 0, n = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern[v], NTHR, 0);
    if (e != hipSuccess) return e;
    occ[v] = n > 0 ? n : 1;
  }
  const int ncu = cu_budget > 0 && cu_budget < cus ? cu_budget : cus;
  const int64_t grid = std::min<int64_t>(ntile, (int64_t)occ[v] * ncu);
  hipLaunchKernelGGL(kern[v], dim3((unsigned)grid), dim3(NTHR), 0, st, q, f, (int)ntile);
  return hipGetLastError();
}

}  // namespace gw
