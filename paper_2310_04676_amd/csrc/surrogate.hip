// Learned forward-dynamics surrogate: an ELU MLP (13J -> 256 -> 256 -> 256 ->
// J, J <= 7) predicts the implicit-PD substep's joint accelerations from
// (q, qd, tau~, the 10 standard inertial parameters of every link). The
// prediction is checked by the inverse-dynamics residual
// |RNEA(q, qd, qdd_hat) + arm qdd_hat - tau~| / max(|tau~|, 1e-3); envs
// above the threshold go on a device-wide queue and get the exact ABA solve.
//
// Kernels (the training GEMM, column sums and Adam are the shared ones of
// nn.hpp, with ELU units):
//   k_feat      normalised BF16 features [B][96] of a batch.
//   k_loss      MSE gradient on normalised targets; per-block sums of the
//               output bias gradient and of the loss.
//   k_pack      BF16 fragment image for the fused inference kernel.
//   k_sinfer    fused inference: features -> 4 layers on the matrix cores,
//               hidden activations in registers, weights streamed from L2.
//   k_sstep_a/b/f  surrogate control step: inference + residual + queue,
//               ABA on the queue, integration + episode bookkeeping.
#include "internal.hpp"
#include "mlp.hpp"
#include "nn.hpp"

namespace sgk {

constexpr int kSF = 96;    // padded feature count (13 J <= 91)
constexpr int kSH = 256;   // hidden width
constexpr int kSO = 16;    // padded output count (J <= 7)
constexpr int kSL = 4;     // weight layers
__host__ __device__ constexpr int s_in(int l) { return l == 0 ? kSF : kSH; }
__host__ __device__ constexpr int s_out(int l) { return l == 3 ? kSO : kSH; }

// ---------------------------------------------------------------------------
// Features: x = (q, qd, tau, per joint [m, m c, I_O]) normalised with
// (mu, sd); rows beyond 13 J zero. Samples: q/qd/tau/qdd [J][n_total] with
// env ids; batch rows pick sample idx[r] (or r if idx is null).
struct FeatArgs {
  const float* par;   // context parameter block [P_NFIELDS][J][N]
  const int* nd;
  int N, J;
  const float* q; const float* qd; const float* tau; const int* env;
  int n_total;
  const int* idx;
  int B;
  const float* norm;  // mu_x[96] sd_x[96] mu_y[16] sd_y[16]
  uint16_t* X;        // [B][96] bf16 (normalised)
  float* Xraw;        // optional [96][B] raw features (for the statistics)
};

__device__ __forceinline__ void raw_features(const FeatArgs& a, int s, float* x) {
#pragma unroll 1
  for (int f = 0; f < kSF; ++f) x[f] = 0.f;
  // out-of-range sample or env ids give all-zero features, never a stray read
  if (s < 0 || s >= a.n_total) return;
  const int J = a.J, e = a.env[s];
  if (e < 0 || e >= a.N) return;
  const int n = a.nd[e];
  for (int j = 0; j < J; ++j) {
    if (j >= n) continue;
    x[j] = a.q[(size_t)j * a.n_total + s];
    x[J + j] = a.qd[(size_t)j * a.n_total + s];
    x[2 * J + j] = a.tau[(size_t)j * a.n_total + s];
    const size_t fs = (size_t)J * a.N, b = (size_t)j * a.N + e;
    const int fld[10] = {P_M, P_HX, P_HY, P_HZ, P_IXX, P_IYY, P_IZZ, P_IXY, P_IXZ, P_IYZ};
    for (int k = 0; k < 10; ++k) x[3 * J + 10 * j + k] = a.par[fld[k] * fs + b];
  }
}

// One thread per (row, feature): the same values as raw_features.
// Consecutive threads take consecutive features of a row when writing the
// row-major X, consecutive rows of a feature when writing only the
// feature-major Xraw, so the stores are contiguous either way.
static_assert(P_IYZ == P_M + 9, "link inertial fields are contiguous");
__global__ void __launch_bounds__(256) k_feat(FeatArgs a) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)a.B * kSF) return;
  const bool rows = a.X != nullptr;
  const int r = rows ? (int)(i / kSF) : (int)(i % a.B), f = rows ? (int)(i % kSF) : (int)(i / a.B);
  const int s = a.idx ? a.idx[r] : r;
  const int J = a.J;
  float x = 0.f;
  if (s >= 0 && s < a.n_total) {
    const int e = a.env[s];
    if (e >= 0 && e < a.N) {
      const int n = a.nd[e];
      if (f < 3 * J) {
        const int kind = f / J, j = f % J;
        const float* src = kind == 0 ? a.q : (kind == 1 ? a.qd : a.tau);
        if (j < n) x = src[(size_t)j * a.n_total + s];
      } else if (f < 13 * J) {
        const int g = f - 3 * J, j = g / 10, k = g % 10;
        if (j < n) x = a.par[(size_t)(P_M + k) * J * a.N + (size_t)j * a.N + e];
      }
    }
  }
  if (a.Xraw) a.Xraw[(size_t)f * a.B + r] = x;
  if (a.X) a.X[(size_t)r * kSF + f] = bf16_bits(f < 13 * J ? (x - a.norm[f]) / a.norm[kSF + f] : 0.f);
}

// Mean and standard deviation per row of a [rows][n] array (one block per
// row; the std floor keeps constant features finite).
__global__ void __launch_bounds__(256) k_rowstats(const float* __restrict__ x, int n, float* mu, float* sd) {
  // two passes in double: the mean, then the mean squared deviation from it
  // (no E[x^2] - m^2 cancellation for features with a large mean and a
  // small spread)
  __shared__ double red[256];
  const int row = blockIdx.x;
  const float* xr = x + (size_t)row * n;
  auto block_sum = [&](double a) {
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
  };
  double a = 0;
  for (int i = threadIdx.x; i < n; i += 256) a += (double)xr[i];
  const double m = block_sum(a) / n;
  double b = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double d = (double)xr[i] - m;
    b += d * d;
  }
  const double var = block_sum(b) / n;
  if (threadIdx.x == 0) {
    const double s = var > 1e-12 ? sqrt(var) : 1.0;
    mu[row] = (float)m;
    sd[row] = (float)s;
  }
}

// Loss gradient on normalised targets: G = 2 (z - t) / (B J) for real
// outputs, 0 for padding (BF16 for the GEMMs); per block of 256 rows, the
// column sums of the FP32 G (the output bias gradient) in part[b][0..kSO)
// and the block's share of the loss sum (z - t)^2 / (B J) in part[b][kSO],
// each added in a fixed order.
constexpr int kSLossRow = 32;  // row stride of the k_loss block sums
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ Z, const float* __restrict__ qdd, int n_total,
                                              const int* __restrict__ idx, int B, int J, const float* __restrict__ norm,
                                              uint16_t* __restrict__ Gb, float* __restrict__ part) {
  __shared__ float red[4][kSO + 1];
  const int r = blockIdx.x * 256 + threadIdx.x;
  float g[kSO + 1];
#pragma unroll
  for (int o = 0; o <= kSO; ++o) g[o] = 0.f;
  if (r < B) {
    const int s = idx ? idx[r] : r;
    const bool ok = s >= 0 && s < n_total;
    const float sc = 1.f / ((float)B * (float)J);
#pragma unroll
    for (int o = 0; o < kSO; ++o) {
      if (o < J && ok) {
        const float t = (qdd[(size_t)o * n_total + s] - norm[2 * kSF + o]) / norm[2 * kSF + kSO + o];
        const float d = Z[(size_t)r * kSO + o] - t;
        g[kSO] += d * d * sc;
        g[o] = 2.f * d * sc;
      }
      Gb[(size_t)r * kSO + o] = bf16_bits(g[o]);
    }
  }
#pragma unroll
  for (int o = 0; o <= kSO; ++o)
    for (int off = 32; off > 0; off >>= 1) g[o] += __shfl_xor(g[o], off, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int o = 0; o <= kSO; ++o) red[threadIdx.x >> 6][o] = g[o];
  __syncthreads();
  if (threadIdx.x <= kSO)
    part[(size_t)blockIdx.x * kSLossRow + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}


// ---------------------------------------------------------------------------
// Fragment image for k_sinfer. Layer l has (out/16) M-tiles x (in/32)
// K-blocks; fragment (mt, kb) is 64 lanes x 8 bf16. Layer 0 uses natural K
// order (its inputs are staged in that order); layers 1-3 use the permuted
// order in which the previous layer's results sit in the lanes.
__host__ __device__ constexpr int s_frag_off(int l) {
  return l == 0 ? 0 : s_frag_off(l - 1) + (s_out(l - 1) / 16) * (s_in(l - 1) / 32) * 64;
}
constexpr int kSFrags = s_frag_off(4);

__global__ void __launch_bounds__(64) k_pack(const uint16_t* __restrict__ W0, const uint16_t* __restrict__ W1,
                                             const uint16_t* __restrict__ W2, const uint16_t* __restrict__ W3,
                                             uint16_t* __restrict__ img) {
  const int l = blockIdx.y, f = blockIdx.x, lane = threadIdx.x;
  const int nkb = s_in(l) / 32, nmt = s_out(l) / 16;
  if (f >= nmt * nkb) return;
  const int mt = f / nkb, kb = f % nkb, g = lane >> 4, i = lane & 15;
  const uint16_t* W = l == 0 ? W0 : l == 1 ? W1 : l == 2 ? W2 : W3;
  uint16_t* dst = img + ((size_t)s_frag_off(l) + (size_t)f * 64 + lane) * 8;
  for (int s = 0; s < 8; ++s) {
    const int k = l == 0 ? 32 * kb + 8 * g + s : 32 * kb + (s < 4 ? 4 * g + s : 16 + 4 * g + (s - 4));
    dst[s] = W[(size_t)(16 * mt + i) * s_in(l) + k];
  }
}

// ---------------------------------------------------------------------------
// Fused inference for one wave of 64 samples (two passes of 32: two 16-wide
// N-tiles each). Features are staged through LDS into B fragments; every
// later layer takes the previous layer's D tiles straight from registers.
struct InferWeights {
  const uint4* img;    // fragment image
  const uint4* ch;     // the same fragments in infer_block's chunk order
  const float* b[4];   // biases [out]
  const float* norm;   // mu_x sd_x mu_y sd_y
};

__device__ __forceinline__ bf16x8 pack_elu(const f32x4& lo, const f32x4& hi) {
  bf16x8 r;
  r[0] = (__bf16)elu_f(lo[0]); r[1] = (__bf16)elu_f(lo[1]); r[2] = (__bf16)elu_f(lo[2]); r[3] = (__bf16)elu_f(lo[3]);
  r[4] = (__bf16)elu_f(hi[0]); r[5] = (__bf16)elu_f(hi[1]); r[6] = (__bf16)elu_f(hi[2]); r[7] = (__bf16)elu_f(hi[3]);
  return r;
}
__device__ __forceinline__ bf16x8 ldfrag(const uint4* p) {
  uint4 t = *p;
  return *reinterpret_cast<bf16x8*>(&t);
}
__device__ __forceinline__ f32x4 bias4(const float* b, int row0) {
  return f32x4{b[row0], b[row0 + 1], b[row0 + 2], b[row0 + 3]};
}

// xs: LDS [64 samples][96] bf16 staged as fragments
// ((tile * 3 + kb) * 4 + g) * 16 + j, tile = sample / 16;
// os: LDS [64][16] floats (normalised outputs).
__device__ __forceinline__ void infer_wave(const InferWeights& w, const uint4* xs, float* os, int lane) {
  const int g = lane >> 4, j = lane & 15;
  const uint4* F0 = w.img + s_frag_off(0);
  const uint4* F1 = w.img + s_frag_off(1);
  const uint4* F2 = w.img + s_frag_off(2);
  const uint4* F3 = w.img + s_frag_off(3);
  for (int half = 0; half < 2; ++half) {
    bf16x8 xb[2][3];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kb = 0; kb < 3; ++kb) xb[t][kb] = ldfrag(xs + (((2 * half + t) * 3 + kb) * 4 + g) * 16 + j);
    f32x4 acc2[16][2];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const f32x4 b = bias4(w.b[1], 16 * m + 4 * g);
      acc2[m][0] = b;
      acc2[m][1] = b;
    }
#pragma unroll 1
    for (int kb2 = 0; kb2 < 8; ++kb2) {
      f32x4 d[2][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = 2 * kb2 + h;
        const f32x4 b = bias4(w.b[0], 16 * m + 4 * g);
        d[h][0] = b;
        d[h][1] = b;
#pragma unroll
        for (int kb = 0; kb < 3; ++kb) {
          const bf16x8 a = ldfrag(F0 + (m * 3 + kb) * 64 + lane);
          d[h][0] = mfma16x16x32(a, xb[0][kb], d[h][0]);
          d[h][1] = mfma16x16x32(a, xb[1][kb], d[h][1]);
        }
      }
      const bf16x8 hb0 = pack_elu(d[0][0], d[1][0]), hb1 = pack_elu(d[0][1], d[1][1]);
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const bf16x8 a = ldfrag(F1 + (m * 8 + kb2) * 64 + lane);
        acc2[m][0] = mfma16x16x32(a, hb0, acc2[m][0]);
        acc2[m][1] = mfma16x16x32(a, hb1, acc2[m][1]);
      }
    }
    bf16x8 h2[8][2];
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      h2[kb][0] = pack_elu(acc2[2 * kb][0], acc2[2 * kb + 1][0]);
      h2[kb][1] = pack_elu(acc2[2 * kb][1], acc2[2 * kb + 1][1]);
    }
    f32x4 acc4[2];
    acc4[0] = acc4[1] = bias4(w.b[3], 4 * g);
#pragma unroll 1
    for (int kb3 = 0; kb3 < 8; ++kb3) {
      f32x4 d[2][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int m = 2 * kb3 + h;
        const f32x4 b = bias4(w.b[2], 16 * m + 4 * g);
        d[h][0] = b;
        d[h][1] = b;
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
          const bf16x8 a = ldfrag(F2 + (m * 8 + kb) * 64 + lane);
          d[h][0] = mfma16x16x32(a, h2[kb][0], d[h][0]);
          d[h][1] = mfma16x16x32(a, h2[kb][1], d[h][1]);
        }
      }
      const bf16x8 a = ldfrag(F3 + kb3 * 64 + lane);
      acc4[0] = mfma16x16x32(a, pack_elu(d[0][0], d[1][0]), acc4[0]);
      acc4[1] = mfma16x16x32(a, pack_elu(d[0][1], d[1][1]), acc4[1]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int smp = 32 * half + 16 * t + j;
      *reinterpret_cast<float4*>(os + smp * kSO + 4 * g) = make_float4(acc4[t][0], acc4[t][1], acc4[t][2], acc4[t][3]);
    }
  }
}

__device__ __forceinline__ void stage_features(uint4* xs, int lane, const float* x /*normalised, 96*/) {
  const int tile = lane >> 4, j = lane & 15;
#pragma unroll
  for (int kb = 0; kb < 3; ++kb)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      bf16x8 v;
#pragma unroll
      for (int s = 0; s < 8; ++s) v[s] = (__bf16)x[32 * kb + 8 * g + s];
      xs[((tile * 3 + kb) * 4 + g) * 16 + j] = *reinterpret_cast<uint4*>(&v);
    }
}

// Prediction for a batch of samples: qdd_hat [J][B] (denormalised).
__global__ void __launch_bounds__(64) k_sinfer(FeatArgs a, InferWeights w, float* __restrict__ out) {
  __shared__ __align__(16) uint4 xs[64 * 12];
  __shared__ __align__(16) float os[64 * kSO];
  const int lane = threadIdx.x, r = blockIdx.x * 64 + lane;
  float x[kSF];
  if (r < a.B) {
    raw_features(a, a.idx ? a.idx[r] : r, x);
#pragma unroll
    for (int f = 0; f < kSF; ++f) x[f] = f < 13 * a.J ? (x[f] - a.norm[f]) / a.norm[kSF + f] : 0.f;
  } else {
#pragma unroll
    for (int f = 0; f < kSF; ++f) x[f] = 0.f;
  }
  stage_features(xs, lane, x);
  __syncthreads();
  infer_wave(w, xs, os, lane);
  __syncthreads();
  if (r < a.B)
    for (int o = 0; o < a.J; ++o)
      out[(size_t)o * a.B + r] = os[lane * kSO + o] * a.norm[2 * kSF + kSO + o] + a.norm[2 * kSF + o];
}

// ---------------------------------------------------------------------------
// Surrogate control step.
struct SStepArgs {
  EnvDev<float> E;
  InferWeights w;
  const float* act;   // [J][N]
  float* qddbuf;      // [J][N]
  int* count;         // [S] queue lengths
  int* list;          // [S][N] queued env ids
  float thresh;
  int s;              // substep index
};

template <int J>
__device__ __forceinline__ void drive_terms(const EnvDev<float>& E, const RegPar<float, J>& ps, int n, const float* act,
                                            int e, const float (&q)[J], const float (&qd)[J], float (&tau)[J],
                                            float (&arm)[J]) {
  const float h = E.h;
  const Jp<float>* P = ps.P;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      const float a = clamp1(act[(size_t)j * E.N + e]);
      const float qs = 0.5f * (P[j].hi + P[j].lo) + 0.5f * (P[j].hi - P[j].lo) * a;
      tau[j] = P[j].kp * (qs - q[j] - h * qd[j]) - P[j].kd * qd[j];
      arm[j] = h * P[j].kd + h * h * P[j].kp;
    } else {
      tau[j] = 0.f;
      arm[j] = 0.f;
    }
  }
}

template <int J>
__device__ __forceinline__ void integrate(const EnvDev<float>& E, const RegPar<float, J>& ps, int n,
                                          const float* qddbuf, int e, float (&q)[J], float (&qd)[J]) {
  const Jp<float>* P = ps.P;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      qd[j] = qd[j] + E.h * qddbuf[(size_t)j * E.N + e];
      q[j] = q[j] + E.h * qd[j];
      if (q[j] > P[j].hi) {
        q[j] = P[j].hi;
        if (qd[j] > 0.f) qd[j] = 0.f;
      } else if (q[j] < P[j].lo) {
        q[j] = P[j].lo;
        if (qd[j] < 0.f) qd[j] = 0.f;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Inference with the weights shared through LDS: the kSW waves of one
// workgroup (64 samples each) run infer_wave's sequence of MFMAs on the same
// weight fragments, which the workgroup copies chunk by chunk from the image
// into a double-buffered LDS area (the next chunk's loads in flight while the
// current one is multiplied), so each fragment leaves L2 once per workgroup
// and half instead of once per wave and half. Chunk c of phase A (layers 0
// and 1, c = infer_wave's kb2): W0's fragments of M-tiles 2c and 2c+1 (3
// K-blocks each), then W1's fragments (m, c) of the 16 M-tiles; chunk c of
// phase B (layers 2 and 3, c = kb3): W2's fragments of M-tiles 2c and 2c+1
// (8 K-blocks each), then W3's fragment c. Every MFMA takes the operands of
// infer_wave in the same order: the same results.
constexpr int kSW = 4;
constexpr int kChunkA = (2 * 3 + 16) * 64;  // fragments (uint4 per lane)
constexpr int kChunkB = (2 * 8 + 1) * 64;
constexpr int kChunkIt = (kChunkA + kSW * 64 - 1) / (kSW * 64);  // loads per thread
constexpr int kChunks = 2 * 2 * 8;  // halves x phases x chunks
static_assert(kChunkB <= kChunkA, "phase B chunks fit the buffer");

__device__ __forceinline__ const uint4* chunk_src(const uint4* img, int phase, int c, int i) {
  if (phase == 0) {
    if (i < 6 * 64) {
      const int h = i / 192, r = i % 192;
      return img + s_frag_off(0) + ((2 * c + h) * 3 + r / 64) * 64 + r % 64;
    }
    const int r = i - 6 * 64;
    return img + s_frag_off(1) + ((r / 64) * 8 + c) * 64 + r % 64;
  }
  if (i < 16 * 64) {
    const int h = i / 512, r = i % 512;
    return img + s_frag_off(2) + ((2 * c + h) * 8 + r / 64) * 64 + r % 64;
  }
  return img + s_frag_off(3) + c * 64 + (i - 16 * 64);
}

// The chunk-ordered copy of the image: the 8 phase-A chunks, then the 8
// phase-B chunks, each contiguous (a permutation of the image's fragments).
__host__ __device__ constexpr int chunk_base(int qc) { return qc < 8 ? qc * kChunkA : 8 * kChunkA + (qc - 8) * kChunkB; }
static_assert(chunk_base(16) == kSFrags, "the chunk order is a permutation of the image");

__global__ void __launch_bounds__(256) k_pack_chunks(const uint4* __restrict__ img, uint4* __restrict__ ch) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= kSFrags) return;
  const int ph = t < 8 * kChunkA ? 0 : 1;
  const int r = ph == 0 ? t : t - 8 * kChunkA, n = ph == 0 ? kChunkA : kChunkB;
  ch[t] = *chunk_src(img, ph, r / n, r % n);
}

// chunk q of the sequence: half q / 16, phase (q / 8) % 2, chunk q % 8
__device__ __forceinline__ void chunk_load(const uint4* ch, int q, int tid, uint4 (&r)[kChunkIt]) {
  const int qc = q & 15, n = qc < 8 ? kChunkA : kChunkB;
  const uint4* src = ch + chunk_base(qc);
#pragma unroll
  for (int k = 0; k < kChunkIt; ++k) {
    const int i = tid + k * kSW * 64;
    r[k] = i < n ? src[i] : make_uint4(0u, 0u, 0u, 0u);
  }
}
__device__ __forceinline__ void chunk_store(uint4* buf, int q, int tid, const uint4 (&r)[kChunkIt]) {
  const int n = ((q >> 3) & 1) == 0 ? kChunkA : kChunkB;
#pragma unroll
  for (int k = 0; k < kChunkIt; ++k) {
    const int i = tid + k * kSW * 64;
    if (i < n) buf[i] = r[k];
  }
}

// The biases of the four layers in LDS (so the chunk loop waits on no
// global load but the next chunk's): [256 | 256 | 256 | 16] floats.
constexpr int kSBias = 3 * kSH + kSO;
__device__ __forceinline__ void stage_biases(const InferWeights& w, float* sb, int tid) {
  for (int i = tid; i < kSBias; i += kSW * 64) sb[i] = i < 3 * kSH ? w.b[i / kSH][i % kSH] : w.b[3][i - 3 * kSH];
}
__device__ __forceinline__ f32x4 lbias4(const float* sb, int row0) {
  const float4 v = *reinterpret_cast<const float4*>(sb + row0);
  return f32x4{v.x, v.y, v.z, v.w};
}

// wb: LDS [2][kChunkA] fragment buffers; sb: LDS biases (stage_biases,
// ordered by this function's first barrier); xs: this wave's staged
// features (stage layout of infer_wave); os: this wave's [64][16] outputs.
// Every thread of the workgroup calls it (tid = 0 .. kSW*64-1).
__device__ __forceinline__ void infer_block(const InferWeights& w, uint4* wb, const float* sb, const uint4* xs,
                                            float* os, int lane, int tid) {
  const int g = lane >> 4, j = lane & 15;
  const float* sb0 = sb;
  const float* sb1 = sb + kSH;
  const float* sb2 = sb + 2 * kSH;
  const float* sb3 = sb + 3 * kSH;
  uint4 r[kChunkIt];
  chunk_load(w.ch, 0, tid, r);
  chunk_store(wb, 0, tid, r);
  __syncthreads();
  // one pipeline step: the next chunk's loads issued, this one multiplied,
  // the next one stored, then the workgroup meets (the buffer just read is
  // overwritten only after that barrier)
  auto step = [&](int q, auto&& mul) __attribute__((always_inline)) {
    const bool more = q + 1 < kChunks;
    if (more) chunk_load(w.ch, q + 1, tid, r);
    mul(wb + (q & 1) * kChunkA);
    if (more) chunk_store(wb + ((q + 1) & 1) * kChunkA, q + 1, tid, r);
    __syncthreads();
  };
#pragma unroll 1
  for (int half = 0; half < 2; ++half) {
    bf16x8 xb[2][3];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kb = 0; kb < 3; ++kb) xb[t][kb] = ldfrag(xs + (((2 * half + t) * 3 + kb) * 4 + g) * 16 + j);
    f32x4 acc2[16][2];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const f32x4 b = lbias4(sb1, 16 * m + 4 * g);
      acc2[m][0] = b;
      acc2[m][1] = b;
    }
#pragma unroll 1
    for (int kb2 = 0; kb2 < 8; ++kb2) {
      step(half * 16 + kb2, [&](const uint4* B) __attribute__((always_inline)) {
        f32x4 d[2][2];
        bf16x8 a0[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) a0[i] = ldfrag(B + i * 64 + lane);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const f32x4 b = lbias4(sb0, 16 * (2 * kb2 + h) + 4 * g);
          d[h][0] = b;
          d[h][1] = b;
        }
        // the first W1 fragments in flight while layer 0's tiles finish
        bf16x8 a1[2] = {ldfrag(B + 6 * 64 + lane), ldfrag(B + 7 * 64 + lane)};
#pragma unroll
        for (int kb = 0; kb < 3; ++kb)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            d[h][0] = mfma16x16x32(a0[h * 3 + kb], xb[0][kb], d[h][0]);
            d[h][1] = mfma16x16x32(a0[h * 3 + kb], xb[1][kb], d[h][1]);
          }
        const bf16x8 hb0 = pack_elu(d[0][0], d[1][0]), hb1 = pack_elu(d[0][1], d[1][1]);
#pragma unroll
        for (int m = 0; m < 16; ++m) {
          // two fragments ahead
          const bf16x8 a = a1[m & 1];
          if (m + 2 < 16) a1[m & 1] = ldfrag(B + (6 + m + 2) * 64 + lane);
          acc2[m][0] = mfma16x16x32(a, hb0, acc2[m][0]);
          acc2[m][1] = mfma16x16x32(a, hb1, acc2[m][1]);
        }
      });
    }
    bf16x8 h2[8][2];
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      h2[kb][0] = pack_elu(acc2[2 * kb][0], acc2[2 * kb + 1][0]);
      h2[kb][1] = pack_elu(acc2[2 * kb][1], acc2[2 * kb + 1][1]);
    }
    f32x4 acc4[2];
    acc4[0] = acc4[1] = lbias4(sb3, 4 * g);
#pragma unroll 1
    for (int kb3 = 0; kb3 < 8; ++kb3) {
      step(half * 16 + 8 + kb3, [&](const uint4* B) __attribute__((always_inline)) {
        f32x4 d[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const f32x4 b = lbias4(sb2, 16 * (2 * kb3 + h) + 4 * g);
          d[h][0] = b;
          d[h][1] = b;
        }
        bf16x8 a2[2] = {ldfrag(B + 0 * 64 + lane), ldfrag(B + 1 * 64 + lane)};
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          // fragment i = (h, kb) = (i / 8, i % 8), two ahead
          const bf16x8 a = a2[i & 1];
          if (i + 2 < 16) a2[i & 1] = ldfrag(B + (i + 2) * 64 + lane);
          const int h = i >> 3, kb = i & 7;
          d[h][0] = mfma16x16x32(a, h2[kb][0], d[h][0]);
          d[h][1] = mfma16x16x32(a, h2[kb][1], d[h][1]);
        }
        const bf16x8 a = ldfrag(B + 16 * 64 + lane);
        acc4[0] = mfma16x16x32(a, pack_elu(d[0][0], d[1][0]), acc4[0]);
        acc4[1] = mfma16x16x32(a, pack_elu(d[0][1], d[1][1]), acc4[1]);
      });
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int smp = 32 * half + 16 * t + j;
      *reinterpret_cast<float4*>(os + smp * kSO + 4 * g) = make_float4(acc4[t][0], acc4[t][1], acc4[t][2], acc4[t][3]);
    }
  }
}

// Normalised feature f of this lane's sample into a wave's staged features
// (infer_wave's layout), rounded to BF16 as stage_features does.
__device__ __forceinline__ void put_feature(uint4* xs, int lane, int f, float v) {
  const int kb = f >> 5, g = (f >> 3) & 3, s = f & 7, tile = lane >> 4, j = lane & 15;
  const __bf16 b = (__bf16)v;
  reinterpret_cast<uint16_t*>(xs + ((tile * 3 + kb) * 4 + g) * 16 + j)[s] = *reinterpret_cast<const uint16_t*>(&b);
}

// (a) integrate the previous substep (s > 0), then predict qdd for this
// substep, check the residual, queue the envs that fail. A workgroup of kSW
// waves holds kSW x 64 envs (one per lane) and shares the weights in LDS
// (infer_block); features go straight into LDS.
constexpr size_t kSStepXs = (size_t)kSW * 64 * 12 * 16;     // staged features
constexpr size_t kSStepOs = (size_t)kSW * 64 * kSO * 4;     // outputs
constexpr size_t kSStepWb = (size_t)2 * kChunkA * 16;       // weight chunks
constexpr size_t kSStepLds = kSStepXs + kSStepOs + kSStepWb + kSBias * 4;
static_assert(kSStepLds <= 160 * 1024, "the surrogate step's LDS fits");
template <int J>
__global__ void __launch_bounds__(kSW * 64) k_sstep_a(SStepArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  uint4* xs = reinterpret_cast<uint4*>(smem_raw) + wave * 64 * 12;
  float* os = reinterpret_cast<float*>(smem_raw + kSStepXs) + wave * 64 * kSO;
  uint4* wb = reinterpret_cast<uint4*>(smem_raw + kSStepXs + kSStepOs);
  float* sb = reinterpret_cast<float*>(smem_raw + kSStepXs + kSStepOs + kSStepWb);
  stage_biases(A.w, sb, tid);
  const EnvDev<float>& E = A.E;
  const int e = blockIdx.x * (kSW * 64) + tid;
  const bool active = e < E.N;
  const int n = active ? E.nd[e] : 0;
  float q[J], qd[J], tau[J], arm[J];
  {
    // this lane's features: zeros, then the defined ones
    const int tile = lane >> 4, j16 = lane & 15;
#pragma unroll
    for (int kb = 0; kb < 3; ++kb)
#pragma unroll
      for (int g = 0; g < 4; ++g) xs[((tile * 3 + kb) * 4 + g) * 16 + j16] = make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int j = 0; j < J; ++j) { q[j] = 0.f; qd[j] = 0.f; tau[j] = 0.f; arm[j] = 0.f; }
  if (active) {
    RegPar<float, J> P;
    load_chain<float, J>(E, e, n, P);
    load_state<float, J>(E, e, n, q, qd);
    if (A.s > 0) {
      integrate<J>(E, P, n, A.qddbuf, e, q, qd);
      store_state<float, J>(E, e, n, q, qd, E.prog[e]);
    }
    drive_terms<J>(E, P, n, A.act, e, q, qd, tau, arm);
    const float* nm = A.w.norm;
    const int JE = E.J;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (j < n) {
        put_feature(xs, lane, j, (q[j] - nm[j]) / nm[kSF + j]);
        put_feature(xs, lane, JE + j, (qd[j] - nm[JE + j]) / nm[kSF + JE + j]);
        put_feature(xs, lane, 2 * JE + j, (tau[j] - nm[2 * JE + j]) / nm[kSF + 2 * JE + j]);
        const Jp<float>& pj = P.P[j];
        const float p[10] = {pj.m, pj.hx, pj.hy, pj.hz, pj.ixx, pj.iyy, pj.izz, pj.ixy, pj.ixz, pj.iyz};
#pragma unroll
        for (int k = 0; k < 10; ++k) {
          const int f = 3 * JE + 10 * j + k;
          put_feature(xs, lane, f, (p[k] - nm[f]) / nm[kSF + f]);
        }
      }
    }
  }
  infer_block(A.w, wb, sb, xs, os, lane, tid);  // barriers inside; the first orders features and biases
  if (!active) return;
  // the link parameters again for the residual (not held across the
  // inference: its accumulators need the registers)
  EnvDev<float> E2 = E;
  asm volatile("" : "+s"(E2.par));
  RegPar<float, J> P;
  load_chain<float, J>(E2, e, n, P);
  const float* nm = A.w.norm;
  float qh[J], id[J];
#pragma unroll
  for (int j = 0; j < J; ++j) qh[j] = j < n ? os[lane * kSO + j] * nm[2 * kSF + kSO + j] + nm[2 * kSF + j] : 0.f;
  rnea<float, J>(P, n, q, qd, qh, E.g, id);
  float rr = 0.f, tt = 0.f;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      const float d = id[j] + arm[j] * qh[j] - tau[j];
      rr += d * d;
      tt += tau[j] * tau[j];
      A.qddbuf[(size_t)j * E.N + e] = qh[j];
    }
  }
  const float rel = sqrtf(rr) / fmaxf(sqrtf(tt), 1e-3f);
  if (!(rel <= A.thresh)) {
    const int slot = atomicAdd(&A.count[A.s], 1);
    A.list[(size_t)A.s * E.N + slot] = e;
  }
}

// (b) exact ABA for the queued envs of substep s.
template <int J>
__global__ void __launch_bounds__(256) k_sstep_b(SStepArgs A) {
  const EnvDev<float>& E = A.E;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= A.count[A.s]) return;
  const int e = A.list[(size_t)A.s * E.N + i];
  const int n = E.nd[e];
  RegPar<float, J> P;
  float q[J], qd[J], tau[J], arm[J], qdd[J];
  load_chain<float, J>(E, e, n, P);
  load_state<float, J>(E, e, n, q, qd);
  drive_terms<J>(E, P, n, A.act, e, q, qd, tau, arm);
  aba_lwa<float, J>(P, n, q, qd, tau, arm, E.g, qdd);
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (j < n) A.qddbuf[(size_t)j * E.N + e] = qdd[j];
}

// (f) integrate the last substep, then reward / episode / observation; hand
// the queue lengths out and clear them for the next step.
template <int J>
__global__ void __launch_bounds__(256) k_sstep_f(SStepArgs A, float* __restrict__ obs, float* __restrict__ rew,
                                                 uint8_t* __restrict__ done, int* __restrict__ n_fallback) {
  const EnvDev<float>& E = A.E;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const bool reads = E.task == TASK_TRACK || E.rerand;
  const uint64_t step = reads ? read_counter(E) : 0;
  settle(step);
  __syncthreads();  // every wave of the block has read the counter
  if (threadIdx.x == 0) advance_counter(E, step, reads);
  if (e == 0) {
    for (int s = 0; s < E.S; ++s) {
      if (n_fallback) n_fallback[s] = A.count[s];
      A.count[s] = 0;
    }
  }
  if (e >= E.N) return;
  const int n = E.nd[e];
  RegPar<float, J> P;
  float q[J], qd[J];
  load_chain<float, J>(E, e, n, P);
  load_state<float, J>(E, e, n, q, qd);
  integrate<J>(E, P, n, A.qddbuf, e, q, qd);
  int prog = E.prog[e];
  float r;
  const uint8_t d = post_step<float, J>(E, e, n, P, q, qd, prog, &r, obs, nullptr, nullptr, step);
  store_state<float, J>(E, e, n, q, qd, prog);
  rew[e] = r;
  done[e] = d;
}

}  // namespace sgk

// ===========================================================================
// Host side: the surrogate object and its C interface.
using namespace sgk;

struct sg_surrogate {
  sg_ctx* ctx = nullptr;
  int J = 0, maxB = 0, t = 0;
  float* Wm[kSL] = {};   // FP32 master weights [out][in] (padded)
  float* bm[kSL] = {};
  float* mW[kSL] = {};
  float* vW[kSL] = {};
  float* mb[kSL] = {};
  float* vb[kSL] = {};
  uint16_t* Wb[kSL] = {};  // BF16 copies [out][in]
  uint16_t* img = nullptr; // inference fragment image
  uint16_t* img_ch = nullptr;  // the same in the surrogate step's chunk order
  float* norm = nullptr;   // mu_x[96] sd_x[96] mu_y[16] sd_y[16]
  // training scratch
  uint16_t* X[kSL] = {};   // layer inputs [B][in] bf16
  float* Z[kSL] = {};      // pre-activations [B][out]
  uint16_t* Gb = nullptr;  // gradient [B][256] bf16 of layer 3's outputs (the loss), then of layers 2, 1, 0 in G[]
  uint16_t* G[3] = {nullptr, nullptr, nullptr};  // each layer's output gradient, kept for the grouped weight gradients
  float* ws = nullptr;     // split-K partials of the weight gradients, one kWeightGradWs region per layer
  float* cpart = nullptr;  // per-block column sums of the hidden layers' gradients [kSL - 1][B / 64][256]
  float* lpart = nullptr;  // k_loss block sums [B / 256][kSLossRow]
  float* gW[kSL] = {};
  float* gb[kSL] = {};     // gb[kSL - 1][kSO] holds the batch loss
  float* loss = nullptr;   // = gb[kSL - 1] + kSO
  // control step
  float* qddbuf = nullptr;
  int* count = nullptr;
  int* list = nullptr;
  std::vector<void*> allocs;
};

namespace {

template <typename T> hipError_t dalloc(sg_surrogate* s, T** p, size_t n) {
  hipError_t e = hipMalloc((void**)p, n * sizeof(T) + 16);
  if (e == hipSuccess) {
    s->allocs.push_back(*p);
    e = hipMemset(*p, 0, n * sizeof(T) + 16);
  }
  return e;
}

sg_status sfail(sg_ctx* c, sg_status st, const char* msg) {
  if (c) c->err = msg;
  return st;
}

InferWeights infer_weights(const sg_surrogate* s) {
  InferWeights w;
  w.img = reinterpret_cast<const uint4*>(s->img);
  w.ch = reinterpret_cast<const uint4*>(s->img_ch);
  for (int l = 0; l < kSL; ++l) w.b[l] = s->bm[l];
  w.norm = s->norm;
  return w;
}

hipError_t repack(sg_surrogate* s, hipStream_t st) {
  for (int l = 0; l < kSL; ++l) {
    const int n = s_out(l) * s_in(l);
    k_to_bf16<<<(n + 255) / 256, 256, 0, st>>>(n, s->Wm[l], s->Wb[l]);
  }
  k_pack<<<dim3(16 * 8, kSL), 64, 0, st>>>(s->Wb[0], s->Wb[1], s->Wb[2], s->Wb[3], s->img);
  return hipGetLastError();
}

FeatArgs feat_args(const sg_surrogate* s, const float* q, const float* qd, const float* tau, const int* env,
                   int n_total, const int* idx, int B) {
  FeatArgs a;
  a.par = (const float*)s->ctx->par;
  a.nd = s->ctx->nd;
  a.N = s->ctx->N;
  a.J = s->J;
  a.q = q; a.qd = qd; a.tau = tau; a.env = env;
  a.n_total = n_total;
  a.idx = idx;
  a.B = B;
  a.norm = s->norm;
  a.X = nullptr;
  a.Xraw = nullptr;
  return a;
}

// Forward (training layout) + loss + backward; gradients land in gW/gb.
hipError_t forward_backward(sg_surrogate* s, hipStream_t st, const float* q, const float* qd, const float* tau,
                            const int* env, const float* qdd, int n_total, const int* idx, int B) {
  FeatArgs fa = feat_args(s, q, qd, tau, env, n_total, idx, B);
  fa.X = s->X[0];
  k_feat<<<(unsigned)(((size_t)B * kSF + 255) / 256), 256, 0, st>>>(fa);
  for (int l = 0; l < kSL; ++l) {
    GemmArgs g{};
    g.M = B; g.N = s_out(l); g.K = s_in(l);
    g.A = s->X[l]; g.lda = s_in(l);
    g.B = s->Wb[l]; g.ldb = s_in(l);
    g.C = s->Z[l]; g.ldc = s_out(l);
    g.bias = s->bm[l];
    if (l < kSL - 1) {
      g.Cb = s->X[l + 1];
      launch_gemm<EPI_FWD_HIDDEN, false, true, ACT_ELU>(st, g);
    } else {
      launch_gemm<EPI_FWD_OUT, false, true, ACT_ELU>(st, g);
    }
  }
  uint16_t* Gbc = s->Gb;
  const int gb = (B + 255) / 256, rb = (B + 63) / 64;
  k_loss<<<gb, 256, 0, st>>>(s->Z[kSL - 1], qdd, n_total, idx, B, s->J, s->norm, Gbc, s->lpart);
  // Weight gradients as split-K partials (layer l in region l of ws), all
  // four in one grouped launch once the data gradients are done (each
  // layer's output gradient has a buffer of its own); their sums, the bias
  // sums and the loss (adjacent to the output layer's bias gradient in
  // gb[kSL - 1]) run as one launch of 2 kSL jobs at the end.
  SumJob jobs[2 * kSL];
  int nj = 0;
  WeightGradGroup<ACT_ELU> wg;
  jobs[nj++] = partial_rows(s->lpart, gb, kSO + 1, kSLossRow, s->gb[kSL - 1]);
  const size_t cstride = (size_t)((s->maxB + 63) / 64) * kSH;
  for (int l = kSL - 1; l >= 0; --l) {
    // dW[o][i] = sum_b G[b][o] X[b][i]
    jobs[nj++] = wg.add(s_out(l), s_in(l), B, Gbc, s_out(l), s->X[l], s_in(l), s->gW[l], s_in(l),
                        s->ws + (size_t)l * kWeightGradWs);
    if (l == 0) break;
    uint16_t* Gbn = s->G[l - 1];
    // G_prev[b][i] = (sum_o G[b][o] W[o][i]) * elu'(Z_prev[b][i]), with the
    // per-block column sums of G_prev (the previous layer's bias gradient)
    GemmArgs d{};
    d.M = B; d.N = s_in(l); d.K = s_out(l);
    d.A = Gbc; d.lda = s_out(l);
    d.B = s->Wb[l]; d.ldb = s_in(l);
    d.C = nullptr; d.ldc = s_in(l);
    d.Cb = Gbn;
    d.Zp = s->Z[l - 1];
    d.colpart = s->cpart + (size_t)(l - 1) * cstride;
    launch_gemm<EPI_BWD_DX, false, false, ACT_ELU>(st, d);
    jobs[nj++] = partial_rows(d.colpart, rb, s_out(l - 1), s_out(l - 1), s->gb[l - 1]);
    Gbc = Gbn;
  }
  wg.launch(st);
  launch_sums(st, jobs, nj);
  return hipGetLastError();
}

}  // namespace

extern "C" {

sg_status sg_surrogate_create(sg_ctx* c, int32_t max_batch, sg_surrogate** out) {
  if (!c || !out) return SG_E_INVAL;
  *out = nullptr;
  if (c->dtype != SG_F32) return sfail(c, SG_E_UNSUPPORTED, "sg_surrogate_create: FP32 contexts only");
  if (c->J > 7) return sfail(c, SG_E_UNSUPPORTED, "sg_surrogate_create: max_dof <= 7");
  if (c->prismatic) return sfail(c, SG_E_UNSUPPORTED, "sg_surrogate_create: all-revolute contexts only");
  if (max_batch < 1 || max_batch > (1 << 22)) return sfail(c, SG_E_INVAL, "sg_surrogate_create: max_batch in 1..4M");
  sg_surrogate* s = new sg_surrogate();
  s->ctx = c;
  s->J = c->J;
  s->maxB = max_batch;
  hipError_t e = hipSuccess;
  const size_t B = (size_t)max_batch;
  for (int l = 0; l < kSL && e == hipSuccess; ++l) {
    const size_t nw = (size_t)s_out(l) * s_in(l), nb = s_out(l);
    if (e == hipSuccess) e = dalloc(s, &s->Wm[l], nw);
    if (e == hipSuccess) e = dalloc(s, &s->bm[l], nb);
    if (e == hipSuccess) e = dalloc(s, &s->mW[l], nw);
    if (e == hipSuccess) e = dalloc(s, &s->vW[l], nw);
    if (e == hipSuccess) e = dalloc(s, &s->mb[l], nb);
    if (e == hipSuccess) e = dalloc(s, &s->vb[l], nb);
    if (e == hipSuccess) e = dalloc(s, &s->Wb[l], nw);
    if (e == hipSuccess) e = dalloc(s, &s->gW[l], nw);
    // the output layer's bias gradient is followed by the batch loss
    if (e == hipSuccess) e = dalloc(s, &s->gb[l], l == kSL - 1 ? nb + 1 : nb);
    if (e == hipSuccess) e = dalloc(s, &s->X[l], B * s_in(l));
    if (e == hipSuccess) e = dalloc(s, &s->Z[l], B * s_out(l));
  }
  if (e == hipSuccess) e = dalloc(s, &s->img, (size_t)kSFrags * 8);
  if (e == hipSuccess) e = dalloc(s, &s->img_ch, (size_t)kSFrags * 8);
  if (e == hipSuccess) e = dalloc(s, &s->norm, 2 * kSF + 2 * kSO);
  if (e == hipSuccess) e = dalloc(s, &s->Gb, B * kSH);
  for (int l = 0; l < 3 && e == hipSuccess; ++l) e = dalloc(s, &s->G[l], B * kSH);
  if (e == hipSuccess) e = dalloc(s, &s->ws, kSL * kWeightGradWs);
  if (e == hipSuccess) e = dalloc(s, &s->cpart, (kSL - 1) * ((B + 63) / 64) * (size_t)kSH);
  if (e == hipSuccess) e = dalloc(s, &s->lpart, ((B + 255) / 256) * (size_t)kSLossRow);
  if (e == hipSuccess) s->loss = s->gb[kSL - 1] + kSO;
  if (e == hipSuccess) e = dalloc(s, &s->qddbuf, (size_t)c->J * c->N);
  if (e == hipSuccess) e = dalloc(s, &s->count, 64);
  if (e == hipSuccess) e = dalloc(s, &s->list, (size_t)c->S * c->N);
  if (e != hipSuccess) {
    for (void* p : s->allocs) (void)hipFree(p);
    delete s;
    c->err = std::string("sg_surrogate_create: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  *out = s;
  return SG_OK;
}

void sg_surrogate_destroy(sg_surrogate* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->ctx->stream);
  for (void* p : s->allocs) (void)hipFree(p);
  delete s;
}

// params: host FP32, per layer W [out][in] then b [out] with the unpadded
// sizes (13J -> 256 -> 256 -> 256 -> J); norm: host FP32
// mu_x[13J] sd_x[13J] mu_y[J] sd_y[J] (may be NULL to keep the current).
sg_status sg_surrogate_set_params(sg_surrogate* s, const float* params, const float* norm) {
  if (!s || !params) return SG_E_INVAL;
  sg_ctx* c = s->ctx;
  const int J = s->J, F = 13 * J;
  const int din[kSL] = {F, kSH, kSH, kSH}, dout[kSL] = {kSH, kSH, kSH, J};
  size_t off = 0;
  hipError_t e = hipSuccess;
  for (int l = 0; l < kSL && e == hipSuccess; ++l) {
    std::vector<float> W((size_t)s_out(l) * s_in(l), 0.f), b(s_out(l), 0.f);
    for (int o = 0; o < dout[l]; ++o)
      for (int i = 0; i < din[l]; ++i) W[(size_t)o * s_in(l) + i] = params[off + (size_t)o * din[l] + i];
    off += (size_t)dout[l] * din[l];
    for (int o = 0; o < dout[l]; ++o) b[o] = params[off + o];
    off += dout[l];
    e = hipMemcpy(s->Wm[l], W.data(), W.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->bm[l], b.data(), b.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s->mW[l], 0, W.size() * 4);
    if (e == hipSuccess) e = hipMemset(s->vW[l], 0, W.size() * 4);
    if (e == hipSuccess) e = hipMemset(s->mb[l], 0, b.size() * 4);
    if (e == hipSuccess) e = hipMemset(s->vb[l], 0, b.size() * 4);
  }
  if (e == hipSuccess && norm) {
    std::vector<float> nm(2 * kSF + 2 * kSO, 0.f);
    for (int f = 0; f < kSF; ++f) nm[kSF + f] = 1.f;
    for (int o = 0; o < kSO; ++o) nm[2 * kSF + kSO + o] = 1.f;
    for (int f = 0; f < F; ++f) { nm[f] = norm[f]; nm[kSF + f] = norm[F + f]; }
    for (int o = 0; o < J; ++o) { nm[2 * kSF + o] = norm[2 * F + o]; nm[2 * kSF + kSO + o] = norm[2 * F + J + o]; }
    e = hipMemcpy(s->norm, nm.data(), nm.size() * 4, hipMemcpyHostToDevice);
  }
  s->t = 0;
  if (e == hipSuccess) e = repack(s, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->err = std::string("sg_surrogate_set_params: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

// Copy the FP32 master parameters (same packing as set_params) and the
// normalisation back to the host.
sg_status sg_surrogate_get_params(sg_surrogate* s, float* params, float* norm) {
  if (!s || !params) return SG_E_INVAL;
  sg_ctx* c = s->ctx;
  const int J = s->J, F = 13 * J;
  const int din[kSL] = {F, kSH, kSH, kSH}, dout[kSL] = {kSH, kSH, kSH, J};
  hipError_t e = hipStreamSynchronize(c->stream);
  size_t off = 0;
  for (int l = 0; l < kSL && e == hipSuccess; ++l) {
    std::vector<float> W((size_t)s_out(l) * s_in(l)), b(s_out(l));
    e = hipMemcpy(W.data(), s->Wm[l], W.size() * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(b.data(), s->bm[l], b.size() * 4, hipMemcpyDeviceToHost);
    for (int o = 0; o < dout[l]; ++o)
      for (int i = 0; i < din[l]; ++i) params[off + (size_t)o * din[l] + i] = W[(size_t)o * s_in(l) + i];
    off += (size_t)dout[l] * din[l];
    for (int o = 0; o < dout[l]; ++o) params[off + o] = b[o];
    off += dout[l];
  }
  if (e == hipSuccess && norm) {
    std::vector<float> nm(2 * kSF + 2 * kSO);
    e = hipMemcpy(nm.data(), s->norm, nm.size() * 4, hipMemcpyDeviceToHost);
    for (int f = 0; f < F; ++f) { norm[f] = nm[f]; norm[F + f] = nm[kSF + f]; }
    for (int o = 0; o < J; ++o) { norm[2 * F + o] = nm[2 * kSF + o]; norm[2 * F + J + o] = nm[2 * kSF + kSO + o]; }
  }
  if (e != hipSuccess) {
    c->err = std::string("sg_surrogate_get_params: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

// Normalisation statistics (mean, std per input feature and output) over n
// samples: q, qd, tau, qdd [J][n] device float32, env [n] device int32.
sg_status sg_surrogate_fit_norm(sg_surrogate* s, const float* q, const float* qd, const float* tau, const int32_t* env,
                                const float* qdd, int32_t n) {
  if (!s || !q || !qd || !tau || !env || !qdd || n < 2) return SG_E_INVAL;
  sg_ctx* c = s->ctx;
  float* xr = nullptr;
  hipError_t e = hipMalloc((void**)&xr, (size_t)kSF * n * 4);
  if (e != hipSuccess) return sfail(c, SG_E_NOMEM, "sg_surrogate_fit_norm: out of memory");
  FeatArgs fa = feat_args(s, q, qd, tau, env, n, nullptr, n);
  fa.Xraw = xr;
  k_feat<<<(unsigned)(((size_t)n * kSF + 255) / 256), 256, 0, c->stream>>>(fa);
  k_rowstats<<<kSF, 256, 0, c->stream>>>(xr, n, s->norm, s->norm + kSF);
  k_rowstats<<<s->J, 256, 0, c->stream>>>(qdd, n, s->norm + 2 * kSF, s->norm + 2 * kSF + kSO);
  e = hipStreamSynchronize(c->stream);
  (void)hipFree(xr);
  if (e != hipSuccess) {
    c->err = std::string("sg_surrogate_fit_norm: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

// Loss and gradients of one batch without updating: gW, gb device FP32
// packed like set_params' parameters (unpadded); loss device float.
sg_status sg_surrogate_grad(sg_surrogate* s, const float* q, const float* qd, const float* tau, const int32_t* env,
                            const float* qdd, int32_t n_total, const int32_t* idx, int32_t batch, float* grad,
                            float* loss) {
  if (!s || !q || !qd || !tau || !env || !qdd || batch < 1 || batch > s->maxB) return SG_E_INVAL;
  sg_ctx* c = s->ctx;
  hipError_t e = forward_backward(s, c->stream, q, qd, tau, env, qdd, n_total, idx, batch);
  const int J = s->J, F = 13 * J;
  const int din[kSL] = {F, kSH, kSH, kSH}, dout[kSL] = {kSH, kSH, kSH, J};
  size_t off = 0;
  for (int l = 0; l < kSL && e == hipSuccess && grad; ++l) {
    e = hipMemcpy2DAsync(grad + off, din[l] * 4, s->gW[l], s_in(l) * 4, din[l] * 4, dout[l], hipMemcpyDeviceToDevice,
                         c->stream);
    off += (size_t)dout[l] * din[l];
    if (e == hipSuccess)
      e = hipMemcpyAsync(grad + off, s->gb[l], dout[l] * 4, hipMemcpyDeviceToDevice, c->stream);
    off += dout[l];
  }
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, s->loss, 4, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) {
    c->err = std::string("sg_surrogate_grad: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

// One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on a batch.
sg_status sg_surrogate_train_step(sg_surrogate* s, const float* q, const float* qd, const float* tau,
                                  const int32_t* env, const float* qdd, int32_t n_total, const int32_t* idx,
                                  int32_t batch, float lr, float* loss) {
  if (!s || !q || !qd || !tau || !env || !qdd || batch < 1 || batch > s->maxB || !(lr > 0))
    return SG_E_INVAL;
  sg_ctx* c = s->ctx;
  hipError_t e = forward_backward(s, c->stream, q, qd, tau, env, qdd, n_total, idx, batch);
  s->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)s->t), c2 = 1.f - powf(b2, (float)s->t);
  static_assert(2 * kSL <= kAdamSegs, "one Adam launch covers every layer");
  AdamSegs segs{};
  for (int l = 0; l < kSL; ++l) {
    adam_add(segs, s->Wm[l], s->gW[l], s->mW[l], s->vW[l], s->Wb[l], s_out(l) * s_in(l));
    adam_add(segs, s->bm[l], s->gb[l], s->mb[l], s->vb[l], nullptr, s_out(l));
  }
  if (e == hipSuccess) k_adam_segs<<<segs.blocks, 256, 0, c->stream>>>(segs, lr, b1, b2, 1e-8f, c1, c2);
  if (e == hipSuccess)
    k_pack<<<dim3(16 * 8, kSL), 64, 0, c->stream>>>(s->Wb[0], s->Wb[1], s->Wb[2], s->Wb[3], s->img);
  if (e == hipSuccess && loss) k_copy_f<<<1, 256, 0, c->stream>>>(s->loss, loss, 1);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    c->err = std::string("sg_surrogate_train_step: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

// Prediction with the fused inference kernel: qdd_hat [J][n] device.
sg_status sg_surrogate_predict(sg_surrogate* s, const float* q, const float* qd, const float* tau, const int32_t* env,
                               int32_t n, float* qdd_hat) {
  if (!s || !q || !qd || !tau || !env || !qdd_hat || n < 1) return SG_E_INVAL;
  sg_ctx* c = s->ctx;
  FeatArgs fa = feat_args(s, q, qd, tau, env, n, nullptr, n);
  k_sinfer<<<(n + 63) / 64, 64, 0, c->stream>>>(fa, infer_weights(s), qdd_hat);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    c->err = std::string("sg_surrogate_predict: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

// Control step of the context with the surrogate: per substep, predict,
// check the residual against thresh, solve the failing envs exactly.
// n_fallback (device int32 [S], may be NULL) receives the queue lengths.
sg_status sg_surrogate_step(sg_surrogate* s, const float* actions, float* obs, float* reward, uint8_t* done,
                            float thresh, int32_t* n_fallback) {
  if (!s || !actions || !obs || !reward || !done) return SG_E_INVAL;
  sg_ctx* c = s->ctx;
  if (c->S > 64) return sfail(c, SG_E_UNSUPPORTED, "sg_surrogate_step: substeps <= 64");
  SStepArgs A;
  A.E = env_view<float>(c);
  A.w = infer_weights(s);
  A.act = actions;
  A.qddbuf = s->qddbuf;
  A.count = s->count;
  A.list = s->list;
  A.thresh = thresh;
  const dim3 gw((c->N + kSW * 64 - 1) / (kSW * 64)), gb((c->N + 255) / 256);
  const int b = dof_bucket(c->J);
  {
    const void* fa = b <= 1 ? (const void*)k_sstep_a<1> : b <= 2 ? (const void*)k_sstep_a<2>
                   : b <= 4 ? (const void*)k_sstep_a<4> : (const void*)k_sstep_a<7>;
    hipError_t e = lds_limit(fa, kSStepLds);
    if (e != hipSuccess) {
      c->err = std::string("sg_surrogate_step: ") + hipGetErrorString(e);
      return SG_E_HIP;
    }
  }
  const size_t la = kSStepLds;
  // the chunk-ordered image of the current weights (320 KB, every call, so
  // a captured step follows later training)
  k_pack_chunks<<<(kSFrags + 255) / 256, 256, 0, c->stream>>>(reinterpret_cast<const uint4*>(s->img),
                                                             reinterpret_cast<uint4*>(s->img_ch));
  for (int st = 0; st < c->S; ++st) {
    A.s = st;
    if (b <= 1) { k_sstep_a<1><<<gw, kSW * 64, la, c->stream>>>(A); k_sstep_b<1><<<gb, 256, 0, c->stream>>>(A); }
    else if (b <= 2) { k_sstep_a<2><<<gw, kSW * 64, la, c->stream>>>(A); k_sstep_b<2><<<gb, 256, 0, c->stream>>>(A); }
    else if (b <= 4) { k_sstep_a<4><<<gw, kSW * 64, la, c->stream>>>(A); k_sstep_b<4><<<gb, 256, 0, c->stream>>>(A); }
    else { k_sstep_a<7><<<gw, kSW * 64, la, c->stream>>>(A); k_sstep_b<7><<<gb, 256, 0, c->stream>>>(A); }
  }
  A.E.rng_add = 1;  // the control step's last kernel advances the noise counter
  if (b <= 1) k_sstep_f<1><<<gb, 256, 0, c->stream>>>(A, obs, reward, done, n_fallback);
  else if (b <= 2) k_sstep_f<2><<<gb, 256, 0, c->stream>>>(A, obs, reward, done, n_fallback);
  else if (b <= 4) k_sstep_f<4><<<gb, 256, 0, c->stream>>>(A, obs, reward, done, n_fallback);
  else k_sstep_f<7><<<gb, 256, 0, c->stream>>>(A, obs, reward, done, n_fallback);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    c->err = std::string("sg_surrogate_step: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

}  // extern "C"
