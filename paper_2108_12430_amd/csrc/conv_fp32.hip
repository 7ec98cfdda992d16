// FP32 direct 1-D convolution / transposed convolution with fused epilogues.
//
// This is the "plain" precision path: one output position per lane, a small
// block of output channels per lane held in registers, weights read through
// wave-uniform (scalar) loads, inputs read straight from HBM/L2 along time so
// neighbouring lanes touch neighbouring addresses.  It is also reused by the
// training path for the adjoint (input-gradient) convolutions: the input
// gradient of a strided conv is the transposed conv with the same weights and
// vice versa, so only the weight strides change.
#include "internal.h"

namespace gw {

__device__ __forceinline__ float tanh_f(float v) { return tanhf(v); }

template <int SRC>
struct In {
  const float* base;
  int head;
  int L;  // row stride; for a ring also its length (wrap point)
  __device__ __forceinline__ float operator()(int i, int q) const {
    if (SRC == SRC_DENSE) return base[(int64_t)i * L + q];
    int ph = head + q;
    if (ph >= L) ph -= L;
    return base[(int64_t)i * L + ph];
  }
};

template <int EPI>
__device__ __forceinline__ void store_out(const ConvP& p, int b, int o, int u, float acc) {
  float v;
  if (EPI == EPI_AFFINE || EPI == EPI_OUT) {
    v = fmaf(acc, p.scale[o], p.shift[o]);
  } else if (EPI == EPI_AFFINE_TANH) {
    v = tanh_f(fmaf(acc, p.scale[o], p.shift[o]));
  } else if (EPI == EPI_BIAS) {
    v = p.bias ? acc + p.bias[o] : acc;
  } else if (EPI == EPI_RELU) {
    v = fmaxf(acc + p.bias[o], 0.0f);
  } else {  // EPI_RESID_RELU: 1x1 stride-2 projection of the stage input
    const float* xs = p.xs + (int64_t)b * p.Cs * p.Ls;
    float sc = 0.0f;
    for (int i = 0; i < p.Cs; ++i) sc = fmaf(p.ws[o * p.Cs + i], xs[(int64_t)i * p.Ls + 2 * u], sc);
    v = fmaxf((acc + p.bias[o]) + (sc + p.bs[o]), 0.0f);
  }
  if (EPI == EPI_OUT) {
    const int W = p.Lout;
    if (p.noise) p.noise[(int64_t)b * W + u] = v;
    if (p.clean) {
      const Item& it = p.items[b];
      const int t0 = W - it.s - it.delay;
      if (u >= t0 && u < t0 + it.s) {
        const int64_t idx = it.out + (u - t0);
        p.clean[idx] = p.strain[idx] - v;
      }
    }
  } else {
    p.y[((int64_t)b * p.Co + o) * p.Lout + u] = v;
  }
}

// Strided convolution: y[o][t] = sum_i sum_j w[o][i][j] * x[i][s t - p + j].
template <int COB, int EPI, int SRC>
__global__ __launch_bounds__(256) void conv_fp32(ConvP p) {
  const int b = blockIdx.z;
  const int o0 = blockIdx.y * COB;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= p.Lout) return;
  In<SRC> in;
  if (SRC == SRC_DENSE) {
    in.L = p.ldx ? p.ldx : p.Lin;
    in.base = p.x + (int64_t)b * p.Ci * in.L;
    in.head = 0;
  } else {
    const Item& it = p.items[b];
    in.L = it.W;
    in.base = reinterpret_cast<const float*>(p.arena) + it.ring;
    in.head = it.head;
  }
  float acc[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc[c] = 0.0f;
  const int q0 = p.stride * t - p.pad;
  for (int i = 0; i < p.Ci; ++i) {
    for (int j = 0; j < p.k; ++j) {
      const int q = q0 + j;
      if (q < 0 || q >= p.Lin) continue;
      const float v = in(i, q);
#pragma unroll
      for (int c = 0; c < COB; ++c) {
        const int o = min(o0 + c, p.Co - 1);
        acc[c] = fmaf(p.w[o * p.wso + i * p.wsi + j], v, acc[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < COB; ++c)
    if (o0 + c < p.Co) store_out<EPI>(p, b, o0 + c, t, acc[c]);
}

// Transposed convolution: y[o][u] = sum_{i,t,j: u = s t - p + j} w[i][o][j] x[i][t].
// Lane m produces the s outputs u = s m + r, r < s (polyphase: only taps with
// j = r + p (mod s) touch phase r, so no inserted zeros are ever multiplied).
template <int COB, int EPI, int SRC>
__global__ __launch_bounds__(256) void convT_fp32(ConvP p) {
  const int b = blockIdx.z;
  const int o0 = blockIdx.y * COB;
  const int m = blockIdx.x * 256 + threadIdx.x;
  const int s = p.stride;
  if (m * s >= p.Lout) return;
  In<SRC> in;
  if (SRC == SRC_DENSE) {
    in.L = p.ldx ? p.ldx : p.Lin;
    in.base = p.x + (int64_t)b * p.Ci * in.L;
    in.head = 0;
  } else {
    const Item& it = p.items[b];
    in.L = it.W;
    in.base = reinterpret_cast<const float*>(p.arena) + it.ring;
    in.head = it.head;
  }
  for (int r = 0; r < s; ++r) {
    const int u = s * m + r;
    if (u >= p.Lout) break;
    float acc[COB];
#pragma unroll
    for (int c = 0; c < COB; ++c) acc[c] = 0.0f;
    const int j0 = (r + p.pad) % s;
    for (int j = j0; j < p.k; j += s) {
      const int t = m + (r + p.pad - j) / s;
      if (t < 0 || t >= p.Lin) continue;
      for (int i = 0; i < p.Ci; ++i) {
        const float v = in(i, t);
#pragma unroll
        for (int c = 0; c < COB; ++c) {
          const int o = min(o0 + c, p.Co - 1);
          acc[c] = fmaf(p.w[i * p.wsi + o * p.wso + j], v, acc[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < COB; ++c)
      if (o0 + c < p.Co) store_out<EPI>(p, b, o0 + c, u, acc[c]);
  }
}

template <int COB, int EPI, int SRC>
static hipError_t launch_one(const ConvP& p, bool transposed, hipStream_t st) {
  const int span = transposed ? (p.Lout + p.stride - 1) / p.stride : p.Lout;
  dim3 grid((span + 255) / 256, (p.Co + COB - 1) / COB, p.n);
  if (transposed)
    hipLaunchKernelGGL((convT_fp32<COB, EPI, SRC>), grid, dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL((conv_fp32<COB, EPI, SRC>), grid, dim3(256), 0, st, p);
  return hipGetLastError();
}

template <int EPI, int SRC>
static hipError_t launch_cob(const ConvP& p, bool transposed, hipStream_t st) {
  if (p.Co == 1) return launch_one<1, EPI, SRC>(p, transposed, st);
  if (p.Co <= 4) return launch_one<4, EPI, SRC>(p, transposed, st);
  return launch_one<8, EPI, SRC>(p, transposed, st);
}

hipError_t launch_conv_fp32(const ConvP& p, bool transposed, int epi, int src, hipStream_t st) {
#define GW_EPI_CASE(E)                                                            \
  case E:                                                                         \
    return src == SRC_RING ? launch_cob<E, SRC_RING>(p, transposed, st)           \
                           : launch_cob<E, SRC_DENSE>(p, transposed, st);
  switch (epi) {
    GW_EPI_CASE(EPI_AFFINE)
    GW_EPI_CASE(EPI_AFFINE_TANH)
    GW_EPI_CASE(EPI_BIAS)
    GW_EPI_CASE(EPI_RELU)
    GW_EPI_CASE(EPI_OUT)
    case EPI_RESID_RELU:
      return launch_cob<EPI_RESID_RELU, SRC_DENSE>(p, transposed, st);
    default:
      return hipErrorInvalidValue;
  }
#undef GW_EPI_CASE
}

}  // namespace gw
