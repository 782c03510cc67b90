// Policy MLP on the matrix cores (gfx950 v_mfma_f32_16x16x32_bf16) for one
// wave of 64 environments: [W<=24 -> 256 -> 128 (-> H3) -> 8], tanh or ELU
// hidden units, BF16 operands, FP32 accumulation. Two networks are built:
// 256-128 tanh (the rollout workload's policy) and 256-128-64 ELU (the
// paper's Table II network).
//
// Formulation: each layer computes Y^T = W X^T, so the MFMA A operand is a
// 16x32 weight tile, B is a 32x16 activation tile (16 environments), and the
// 16x16 result tile D has one environment per column. Lane l = 16 g + j
// holds D rows 4g..4g+3 of column j, exactly the layout it needs as the next
// layer's B fragment (column j, eight K values) if the next layer's K index
// is permuted: in K-block kb (features 32kb..32kb+31) lane group g owns
// features {32kb + 4g + r, 32kb + 16 + 4g + r | r = 0..3}. The weights are
// stored in LDS already permuted and in fragment order, so every operand
// read is one 16-byte ds_read per lane and hidden activations never leave
// the registers. Only the 24-wide input and the 8 outputs pass through LDS
// (a transpose between "one env per lane" and the fragment layout).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kH1 = 256, kH2 = 128, kKin = 32, kOut = 16;  // padded sizes
enum { PACT_TANH = 0, PACT_ELU = 1 };                        // hidden activation
// LDS image of the weights, in 16-byte fragments (uint4):
//   W1: [16 row tiles][64 lanes]          (K = 32 input features, padded)
//   W2: [8 row tiles][8 K-blocks][64 lanes]
//   W3: [H3/16 row tiles][4 K-blocks][64 lanes]   (third hidden layer, if any)
//   Wo: [Ko/32 K-blocks][64 lanes]        (16 rows, outputs >= J+1 zero;
//                                          Ko = H3 or 128)
// and the bias image b1 (256) | b2 (128) | b3 (H3) | bo (16) floats.
constexpr int kW1Frags = 16 * 64, kW2Frags = 8 * 8 * 64;
template <int H3> struct PolicyShape {
  static constexpr int kKo = H3 ? H3 : kH2;
  static constexpr int kW3Frags = (H3 / 16) * (kH2 / 32) * 64;
  static constexpr int kWoFrags = (kKo / 32) * 64;
  static constexpr int kWFrags = kW1Frags + kW2Frags + kW3Frags + kWoFrags;  // 84 KB or 98 KB
  static constexpr int kBias = kH1 + kH2 + H3 + kOut;
};
// the largest image (the weight buffer of a context holds any network)
constexpr int kWFragsMax = PolicyShape<64>::kWFrags;
constexpr int kBiasMax = PolicyShape<64>::kBias;

// fast tanh: 1 - 2 / (exp(2x) + 1) with the hardware exp and reciprocal
// (v_exp_f32, v_rcp_f32: about 1 ulp each) instead of an IEEE division
// sequence; the result is rounded to BF16 before use, far coarser than this
// formula's error. Saturates to +-1 (exp overflow gives rcp(inf) = 0).
__device__ __forceinline__ float tanh_fast(float x) {
  const float e = __expf(2.f * x);
  return 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
}

// ELU with the hardware exponential (about 1 ulp), rounded to BF16 after.
__device__ __forceinline__ float elu_fast(float x) { return x > 0.f ? x : __expf(x) - 1.f; }

template <int ACT> __device__ __forceinline__ float pact(float x) {
  return ACT == PACT_ELU ? elu_fast(x) : tanh_fast(x);
}

__device__ __forceinline__ f32x4 mfma16x16x32(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int ACT> __device__ __forceinline__ bf16x8 pack_act(const f32x4& lo, const f32x4& hi) {
  bf16x8 r;
  r[0] = (__bf16)pact<ACT>(lo[0]); r[1] = (__bf16)pact<ACT>(lo[1]);
  r[2] = (__bf16)pact<ACT>(lo[2]); r[3] = (__bf16)pact<ACT>(lo[3]);
  r[4] = (__bf16)pact<ACT>(hi[0]); r[5] = (__bf16)pact<ACT>(hi[1]);
  r[6] = (__bf16)pact<ACT>(hi[2]); r[7] = (__bf16)pact<ACT>(hi[3]);
  return r;
}

// Stage one env's input row (W floats, lane = env within the wave) into the
// B-fragment image xs: [4 N-tiles][4 groups][16 cols] x 16 B.
__device__ __forceinline__ void stage_input(uint4* xs, int lane, const float* x, int W) {
  const int n = lane >> 4, j = lane & 15;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    bf16x8 v;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = 8 * g + s;
      v[s] = (__bf16)(k < W ? x[k] : 0.f);
    }
    xs[(n * 4 + g) * 16 + j] = *reinterpret_cast<uint4*>(&v);
  }
}

// The forward pass for NT of the 4 staged 16-env tiles, starting at tile
// t0 (a wave computes all four, or each of four waves one). ws: weight
// image, bias: bias image, xs: staged inputs, os: output image [64
// envs][16] floats. With W1G the image in ws starts at W2 and layer 1's
// fragments come from w1 (the global image; all 16 loaded at the start).
// Callers synchronize around it.
template <int H3, int ACT, int NT = 4, bool W1G = false>
__device__ __forceinline__ void mlp_wave(const uint4* __restrict__ ws, const float* __restrict__ bias,
                                         const uint4* __restrict__ xs, float* __restrict__ os, int lane, int t0 = 0,
                                         const uint4* __restrict__ w1 = nullptr) {
  using S = PolicyShape<H3>;
  const int g = lane >> 4, j = lane & 15;
  const uint4* W1 = W1G ? w1 : ws;
  const uint4* W2 = W1G ? ws : ws + kW1Frags;
  const uint4* W3 = W2 + kW2Frags;
  uint4 w1r[W1G ? kW1Frags / 64 : 1];
  if constexpr (W1G) {
#pragma unroll
    for (int m = 0; m < kW1Frags / 64; ++m) w1r[m] = W1[m * 64 + lane];
  }
  const uint4* Wo = W3 + S::kW3Frags;
  const float* bo = bias + kH1 + kH2 + H3;
  bf16x8 xb[NT];
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    uint4 t = xs[((t0 + n) * 4 + g) * 16 + j];
    xb[n] = *reinterpret_cast<bf16x8*>(&t);
  }
  f32x4 acc2[8][NT];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const float4 bb = *reinterpret_cast<const float4*>(bias + kH1 + 16 * m + 4 * g);
#pragma unroll
    for (int n = 0; n < NT; ++n) acc2[m][n] = f32x4{bb.x, bb.y, bb.z, bb.w};
  }
#pragma unroll
  for (int kb = 0; kb < 8; ++kb) {
    f32x4 d1[2][NT];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int m = 2 * kb + h;
      uint4 t = W1G ? w1r[m] : W1[m * 64 + lane];
      const bf16x8 a = *reinterpret_cast<bf16x8*>(&t);
      const float4 bb = *reinterpret_cast<const float4*>(bias + 16 * m + 4 * g);
#pragma unroll
      for (int n = 0; n < NT; ++n) d1[h][n] = mfma16x16x32(a, xb[n], f32x4{bb.x, bb.y, bb.z, bb.w});
    }
    bf16x8 hb[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) hb[n] = pack_act<ACT>(d1[0][n], d1[1][n]);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      uint4 t = W2[(m * 8 + kb) * 64 + lane];
      const bf16x8 a = *reinterpret_cast<bf16x8*>(&t);
#pragma unroll
      for (int n = 0; n < NT; ++n) acc2[m][n] = mfma16x16x32(a, hb[n], acc2[m][n]);
    }
  }
  f32x4 acco[NT];
  {
    const float4 bb = *reinterpret_cast<const float4*>(bo + 4 * g);
#pragma unroll
    for (int n = 0; n < NT; ++n) acco[n] = f32x4{bb.x, bb.y, bb.z, bb.w};
  }
  if constexpr (H3 > 0) {
    // third hidden layer: K-block kb of it is row tiles 2kb, 2kb+1 of layer 2
    constexpr int M3 = H3 / 16;
    f32x4 acc3[M3][NT];
#pragma unroll
    for (int m = 0; m < M3; ++m) {
      const float4 bb = *reinterpret_cast<const float4*>(bias + kH1 + kH2 + 16 * m + 4 * g);
#pragma unroll
      for (int n = 0; n < NT; ++n) acc3[m][n] = f32x4{bb.x, bb.y, bb.z, bb.w};
    }
#pragma unroll
    for (int kb = 0; kb < kH2 / 32; ++kb) {
      bf16x8 hb[NT];
#pragma unroll
      for (int n = 0; n < NT; ++n) hb[n] = pack_act<ACT>(acc2[2 * kb][n], acc2[2 * kb + 1][n]);
#pragma unroll
      for (int m = 0; m < M3; ++m) {
        uint4 t = W3[(m * (kH2 / 32) + kb) * 64 + lane];
        const bf16x8 a = *reinterpret_cast<bf16x8*>(&t);
#pragma unroll
        for (int n = 0; n < NT; ++n) acc3[m][n] = mfma16x16x32(a, hb[n], acc3[m][n]);
      }
    }
#pragma unroll
    for (int kb = 0; kb < H3 / 32; ++kb) {
      uint4 t = Wo[kb * 64 + lane];
      const bf16x8 a = *reinterpret_cast<bf16x8*>(&t);
#pragma unroll
      for (int n = 0; n < NT; ++n) acco[n] = mfma16x16x32(a, pack_act<ACT>(acc3[2 * kb][n], acc3[2 * kb + 1][n]), acco[n]);
    }
  } else {
#pragma unroll
    for (int kb = 0; kb < kH2 / 32; ++kb) {
      uint4 t = Wo[kb * 64 + lane];
      const bf16x8 a = *reinterpret_cast<bf16x8*>(&t);
#pragma unroll
      for (int n = 0; n < NT; ++n) acco[n] = mfma16x16x32(a, pack_act<ACT>(acc2[2 * kb][n], acc2[2 * kb + 1][n]), acco[n]);
    }
  }
  if (g < 2) {
#pragma unroll
    for (int n = 0; n < NT; ++n)
      *reinterpret_cast<float4*>(os + (16 * (t0 + n) + j) * kOut + 4 * g) =
          make_float4(acco[n][0], acco[n][1], acco[n][2], acco[n][3]);
  }
}

// Source of one element of the weight image: fragment f (0 .. kWFrags),
// lane l, slot s -> layer (0 W1, 1 W2, 2 W3, 3 output), row and input k of
// that layer's W [rows][K]; returns false for padding (an input past the
// observation width W, an output row >= O). Shared by the host-visible
// packer kernel so every writer of the image uses one layout.
template <int H3>
__host__ __device__ inline bool img_source(int f, int l, int s, int W, int O, int* layer, int* row, int* k) {
  using S = PolicyShape<H3>;
  const int g = l >> 4, i = l & 15;
  const int kp_lo = s < 4 ? 4 * g + s : 16 + 4 * g + (s - 4);  // permuted K within a 32-block
  if (f < kW1Frags / 64) {
    *layer = 0; *row = 16 * f + i; *k = 8 * g + s;
    return *k < W;
  }
  f -= kW1Frags / 64;
  if (f < kW2Frags / 64) {
    const int m = f / 8, kb = f % 8;
    *layer = 1; *row = 16 * m + i; *k = 32 * kb + kp_lo;
    return true;
  }
  f -= kW2Frags / 64;
  if (f < S::kW3Frags / 64) {
    const int m = f / (kH2 / 32), kb = f % (kH2 / 32);
    *layer = 2; *row = 16 * m + i; *k = 32 * kb + kp_lo;
    return true;
  }
  f -= S::kW3Frags / 64;
  *layer = 3; *row = i; *k = 32 * f + kp_lo;
  return i < O;
}

}  // namespace sgk
