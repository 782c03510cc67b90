// PPO update of the rollout policy on the GPU (the paper trains its policies
// with the GPU PPO of Rudin et al., Sec. III "Policy learning and control";
// objective: the clipped surrogate of Schulman et al., 2017, with a clipped
// value loss and an entropy bonus).
//
// Once per call: advantage mean and standard deviation, the normalised
// advantages, the observations as sample-major BF16 rows and the loss inputs
// (action, old log-probability, advantage, value, return) as sample-major
// FP32 rows (k_ppo_xall).
// One minibatch of B samples (rows) taken from the rollout buffers:
//   k_ppo_gather   the minibatch's rows -> X [B][32] (in sg_ppo_update
//                  only for the first minibatch: later ones are gathered
//                  by extra blocks of the previous k_ppo_norm_adam launch)
//   k_ppo_front    the forward pass, the loss and the gradient down to
//                  hidden layer 1's pre-activations in one launch on the
//                  matrix cores, activations and act' in registers, with
//                  per-chunk column sums (the hidden biases' gradients)
//   backward       weight gradients as split-K GEMMs (nn.hpp; the batch is
//                  the reduction axis), all of a minibatch's in one grouped
//                  launch; every partial is summed in a fixed order --
//                  deterministic; the split sums and bias sums share one
//                  launch (k_sum_jobs)
//   k_ppo_norm_adam  entropy term, global gradient norm, statistics, norm
//                  clip and Adam on the FP32 master weights + BF16 copy (and
//                  the fused kernels' fragment-order weight images), in
//                  one launch (sg_ppo_grad: k_gnorm_part and k_ppo_finish
//                  give the norm and statistics without the Adam step)
// After an update k_ppo_pack rewrites the context's rollout weight image
// (the MFMA fragment order of mlp.hpp), biases and log_std from the master
// weights, so the next rollout samples from the updated policy.
#include <cmath>

#include "internal.hpp"
#include "mlp.hpp"
#include "nn.hpp"

namespace sgk {
// Fragment images of the fused PPO kernels' weights: layout (see img_scatter)
struct PpoImg {
  int W, O, KO, H3;   // inputs, outputs, the output layer's K, hidden-3 width (0: none)
  int oW1, oW2, oW3, oWo;  // weight offsets in the flat parameters
  int fW1, fW2, fW3, fWo, fWoT, fW3T, fW2T, frags;  // image sections (uint4 offsets), total
};
}  // namespace sgk

struct sg_ppo {
  sg_ctx* ctx = nullptr;
  int J = 0, W = 0, O = 0, P = 0;
  // network: hidden layers 256, 128 (, h3), then J + 1 outputs; act the
  // hidden activation (PACT_*); flat parameters per layer W then b, then
  // log_std at oLS
  int h3 = 0, act = 0, nl = 3;
  int oW[4] = {0, 0, 0, 0}, oB[4] = {0, 0, 0, 0}, oLS = 0;
  int max_samples = 0;
  uint64_t* tstep = nullptr; // Adam steps taken (device, so captured updates advance it)
  unsigned* ttick = nullptr; // blocks of the current norm+Adam launch that have read it
  float* p = nullptr;        // master parameters [P]
  uint16_t* pb = nullptr;    // BF16 copy [P]
  uint16_t* img = nullptr;   // fragment images of the fused kernels' weights [im.frags][8]
  float* g = nullptr;        // gradient [P]
  float* m = nullptr;        // Adam moments [P]
  float* v = nullptr;
  float* an = nullptr;       // normalised advantages [max_samples]
  float* scal = nullptr;     // [0] adv mean, [1] adv sd, [2] |g|
  uint16_t* X = nullptr;     // [rows][32]
  uint16_t* Xall = nullptr;  // [max_samples][32] sample-major BF16 observations
  float* Aux = nullptr;      // [max_samples][kAux] sample-major act, logp, adv, value, return
  uint16_t* H1 = nullptr;    // [rows][256] (layer 1's pre-activations are recomputed, not kept)
  uint16_t* H2 = nullptr;
  uint16_t* H3 = nullptr;    // [rows][h3]
  uint16_t* D3b = nullptr;   // [rows][h3]
  float* cpart3 = nullptr;   // per-chunk column sums of dZ3 [loss_blocks(rows)][h3]
  uint16_t* G3b = nullptr;   // [rows][8] dL/d(outputs)
  uint16_t* D2b = nullptr;   // [rows][128]
  uint16_t* D1b = nullptr;   // [rows][256]
  float* ws = nullptr;       // split-K partials, one kWeightGradWs region per layer
  size_t ws_floats = 0;
  float* cpart = nullptr;    // per-chunk column sums of dZ1 [loss_blocks(rows)][256]
  float* cpart2 = nullptr;   // per-chunk column sums of dZ2 [loss_blocks(rows)][128]
  float* lpart = nullptr;    // per-chunk loss sums [loss_blocks(rows)][kLossPart]
  double* gpart = nullptr;   // block sums [kGnormBlocks]: advantage statistics, then gradient norm
  double* npart = nullptr;   // the last minibatch's gradient-norm partials [kNormParts] (from k_sum_jobs)
  int nparts = 0;            // how many (0: k_ppo_norm_adam sums the gradient itself)
  sgk::PpoImg im{};
  std::vector<void*> allocs;
};

namespace sgk {

constexpr int kPX = 32;   // padded input width
// Sample-major per-sample row of the loss inputs: act[0..J), then logp,
// normalised advantage, old value and return at kAux - 4 .. kAux - 1.
constexpr int kAux = 12;
constexpr int kPO = 8;    // padded output width (J + 1 <= 8)
// Loss-sum row (one per chunk of k_ppo_front): dL/d(outputs) sums (O
// columns) then dL/dlog_std sums (J columns), zero to column 16, then the
// four weighted loss sums.
constexpr int kLossPart = 20;
constexpr int kGnormChunk = 1024;  // gradient entries per k_gnorm_part block
constexpr int kGnormBlocks = 128;  // capacity of the partial-sum buffer (norm; advantage statistics)
constexpr int kNormParts = 16384;  // capacity of the sum launch's gradient-norm partials

struct PpoRows {
  const float* obs;   // [T+1][W][N]
  const float* act;   // [T][J][N]
  const float* logp;  // [T][N]
  const float* val;   // [T+1][N]
  const float* ret;   // [T][N]
  const float* an;    // normalised advantages [T N]
  const uint16_t* xall;  // BF16 observations, sample-major [T N][kPX]
  const float* aux;      // loss inputs, sample-major [T N][kAux]
  const int* idx;     // sample of row r (null: r0 + r)
  int r0, rows, N, J, W, total;
};

__device__ __forceinline__ int ppo_sample(const PpoRows& a, int r) { return a.idx ? a.idx[r] : a.r0 + r; }

// The rollout's observations, BF16 and sample-major (one 64-byte row per
// sample s = t N + e, zero past W), so a minibatch gathers whole rows.
__global__ void __launch_bounds__(256) k_ppo_xall(const float* __restrict__ obs, int total, int N, int W,
                                                  uint16_t* __restrict__ xall, PpoRows r, float* __restrict__ aux) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= total) return;
  const int t = s / N, e = s % N;
  {
    // the loss inputs of sample s as one 48-byte row
    float v[kAux];
#pragma unroll
    for (int j = 0; j < kAux - 4; ++j) v[j] = j < r.J ? r.act[((size_t)t * r.J + j) * N + e] : 0.f;
    v[kAux - 4] = r.logp[(size_t)t * N + e];
    v[kAux - 3] = r.an[s];
    v[kAux - 2] = r.val[(size_t)t * N + e];
    v[kAux - 1] = r.ret[(size_t)t * N + e];
    float4* d = reinterpret_cast<float4*>(aux + (size_t)s * kAux);
#pragma unroll
    for (int q = 0; q < kAux / 4; ++q) d[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  }
  uint32_t w[kPX / 2];
#pragma unroll
  for (int k = 0; k < kPX; k += 2) {
    const float x0 = k < W ? obs[((size_t)t * W + k) * N + e] : 0.f;
    const float x1 = k + 1 < W ? obs[((size_t)t * W + k + 1) * N + e] : 0.f;
    w[k / 2] = (uint32_t)bf16_bits(x0) | ((uint32_t)bf16_bits(x1) << 16);
  }
  uint4* dst = reinterpret_cast<uint4*>(xall + (size_t)s * kPX);
#pragma unroll
  for (int q = 0; q < kPX / 8; ++q) dst[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

// Minibatch input rows; a sample id outside [0, T N) gives a zero row.
__device__ __forceinline__ void gather_row(const PpoRows& a, int r, uint16_t* __restrict__ X) {
  const int s = ppo_sample(a, r);
  const bool ok = s >= 0 && s < a.total;
  const uint4* src = reinterpret_cast<const uint4*>(a.xall + (size_t)(ok ? s : 0) * kPX);
  uint4* dst = reinterpret_cast<uint4*>(X + (size_t)r * kPX);
#pragma unroll
  for (int q = 0; q < kPX / 8; ++q) dst[q] = ok ? src[q] : make_uint4(0, 0, 0, 0);
}
__global__ void __launch_bounds__(256) k_ppo_gather(PpoRows a, uint16_t* __restrict__ X) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r < a.rows) gather_row(a, r, X);
}

// Mean and unbiased standard deviation of the n advantages, two passes in
// double over kAdvBlocks blocks: k_adv_sum leaves per-block sums in
// part[0..kAdvBlocks), k_adv_sq the per-block sums of squared deviations
// from the mean in part[kAdvBlocks..2 kAdvBlocks); every reader adds the
// partials in block order. k_adv_norm writes an = (adv - mean) / (sd +
// 1e-8) and, from block 0, scal[0] = mean, scal[1] = sd.
constexpr int kAdvBlocks = 64;
static_assert(2 * kAdvBlocks <= kGnormBlocks, "advantage partials share the partial-sum buffer");

__device__ __forceinline__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  return red[0];
}

__device__ __forceinline__ double adv_mean(const double* part, int n) {
  double s = 0;
  for (int b = 0; b < kAdvBlocks; ++b) s += part[b];
  return s / n;
}

__global__ void __launch_bounds__(256) k_adv_sum(const float* __restrict__ x, int n, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += kAdvBlocks * 256) s += x[i];
  const double t = block_sum256(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_adv_sq(const float* __restrict__ x, int n, double* __restrict__ part) {
  __shared__ double red[256];
  const double mean = adv_mean(part, n);
  double q = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += kAdvBlocks * 256) q += (x[i] - mean) * (x[i] - mean);
  const double t = block_sum256(q, red);
  if (threadIdx.x == 0) part[kAdvBlocks + blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_adv_norm(const float* __restrict__ adv, int n, const double* __restrict__ part,
                                                  float* __restrict__ an, float* __restrict__ scal) {
  const double mean = adv_mean(part, n);
  double q = 0;
  for (int b = 0; b < kAdvBlocks; ++b) q += part[kAdvBlocks + b];
  const float m = (float)mean, sd = n > 1 ? (float)sqrt(q / (n - 1)) : 0.f;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[0] = m;
    scal[1] = sd;
  }
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) an[i] = (adv[i] - m) / (sd + 1e-8f);
}

// One minibatch row with loss inputs x (action, old log-probability,
// normalised advantage, old value, return): log pi(a) under the outputs z
// (mu | V), ratio, clipped objectives; g receives dL/d(outputs), dl the
// log_std terms, and the loss terms lpi, lv, kl and the clip indicator cf.
// A row whose sample id is outside [0, T N) contributes zeros (the caller
// skips it).
// The loss inputs of row r (ppo_row_loss's x); false for a sample id
// outside [0, T N).
__device__ __forceinline__ bool ppo_row_inputs(const PpoRows& R, int r, float (&x)[kAux]) {
  const int s = ppo_sample(R, r);
  if (s < 0 || s >= R.total) return false;
  const float4* src = reinterpret_cast<const float4*>(R.aux + (size_t)s * kAux);
#pragma unroll
  for (int q = 0; q < kAux / 4; ++q) {
    const float4 v = src[q];
    x[4 * q] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
  }
  return true;
}
__device__ __forceinline__ void ppo_row_loss(int J, const float (&x)[kAux], const float* z,
                                             const float* __restrict__ ls, float clip, float c_v, float inv_b,
                                             float (&g)[kPO], float (&dl)[kPO], float& lpi, float& lv, float& kl,
                                             float& cf) {
  float logp = 0.f;
  float u[kPO];
  for (int j = 0; j < J; ++j) {
    const float sig = __expf(ls[j]);
    u[j] = (x[j] - z[j]) / sig;
    logp += -0.5f * u[j] * u[j] - ls[j] - 0.91893853320467274f;
  }
  const float lold = x[kAux - 4];
  const float A = x[kAux - 3];
  const float ratio = __expf(logp - lold);
  const float rc = fminf(fmaxf(ratio, 1.f - clip), 1.f + clip);
  lpi = -fminf(ratio * A, rc * A);
  kl = lold - logp;
  cf = fabsf(ratio - 1.f) > clip ? 1.f : 0.f;
  const bool live = A >= 0.f ? ratio <= 1.f + clip : ratio >= 1.f - clip;
  const float dlogp = live ? -A * ratio * inv_b : 0.f;
  for (int j = 0; j < J; ++j) {
    const float sig = __expf(ls[j]);
    g[j] = dlogp * u[j] / sig;
    dl[j] = dlogp * (u[j] * u[j] - 1.f);
  }
  const float V = z[J], vold = x[kAux - 2], ret = x[kAux - 1];
  const float dv = V - vold;
  const float Vc = vold + fminf(fmaxf(dv, -clip), clip);
  const float e1 = (V - ret) * (V - ret), e2 = (Vc - ret) * (Vc - ret);
  lv = fmaxf(e1, e2);
  float dV;
  if (e1 >= e2) dV = 2.f * (V - ret);
  else dV = fabsf(dv) <= clip ? 2.f * (Vc - ret) : 0.f;
  g[J] = c_v * dV * inv_b;
}

// Fragment images of the fused kernels' weights (BF16, the MFMA operand
// order the kernels stage into LDS, in uint4 units: [fragment row][64
// lanes] x 8 slots), kept next to the flat BF16 copy: the Adam step writes
// every updated weight into its one or two image positions, so a
// workgroup stages its weights with coalesced 16-byte loads. Padding
// positions (inputs past W, outputs past O) stay zero from allocation.
// PpoImg (above) gives the sections.
// permuted position of K index p (0..31) within a 32-wide K block: lane
// group g, slot s (mlp.hpp's layout)
__device__ __forceinline__ void perm_slot(int p, int& g, int& s) {
  if (p < 16) { g = p >> 2; s = p & 3; }
  else { g = (p - 16) >> 2; s = 4 + ((p - 16) & 3); }
}
__device__ __forceinline__ void img_put(uint16_t* img, int base, int row, int lane, int slot, uint16_t v) {
  img[((size_t)(base + row * 64 + lane)) * 8 + slot] = v;
}
// Writes the BF16 value v of flat parameter idx into the images that hold it
__device__ __forceinline__ void img_scatter(const PpoImg& m, int idx, uint16_t v, uint16_t* img) {
  int g, s;
  if (idx >= m.oW1 && idx < m.oW1 + kH1 * m.W) {
    const int r = (idx - m.oW1) / m.W, k = (idx - m.oW1) % m.W;
    img_put(img, m.fW1, r >> 4, 16 * (k >> 3) + (r & 15), k & 7, v);
  } else if (idx >= m.oW2 && idx < m.oW2 + kH2 * kH1) {
    const int u2 = (idx - m.oW2) / kH1, u1 = (idx - m.oW2) % kH1;
    perm_slot(u1 & 31, g, s);
    img_put(img, m.fW2, (u2 >> 4) * (kH1 / 32) + (u1 >> 5), 16 * g + (u2 & 15), s, v);
    perm_slot(u2 & 31, g, s);
    img_put(img, m.fW2T, (u1 >> 4) * (kH2 / 32) + (u2 >> 5), 16 * g + (u1 & 15), s, v);
  } else if (m.H3 && idx >= m.oW3 && idx < m.oW3 + m.H3 * kH2) {
    const int u3 = (idx - m.oW3) / kH2, u2 = (idx - m.oW3) % kH2;
    perm_slot(u2 & 31, g, s);
    img_put(img, m.fW3, (u3 >> 4) * (kH2 / 32) + (u2 >> 5), 16 * g + (u3 & 15), s, v);
    perm_slot(u3 & 31, g, s);
    img_put(img, m.fW3T, (u2 >> 4) * (m.H3 / 32) + (u3 >> 5), 16 * g + (u2 & 15), s, v);
  } else if (idx >= m.oWo && idx < m.oWo + m.O * m.KO) {
    const int o = (idx - m.oWo) / m.KO, k = (idx - m.oWo) % m.KO;
    perm_slot(k & 31, g, s);
    img_put(img, m.fWo, k >> 5, 16 * g + o, s, v);
    img_put(img, m.fWoT, k >> 4, 16 * (o >> 3) + (k & 15), o & 7, v);
  }
}
__global__ void __launch_bounds__(256) k_ppo_img(PpoImg m, int n, const uint16_t* __restrict__ pb,
                                                 uint16_t* __restrict__ img) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) img_scatter(m, i, pb[i], img);
}

// Fused front of a minibatch: per chunk of kFrontRows rows (one 16-row
// tile per wave) the hidden layers (256, 128, and H3 = 64 for the paper's
// Table II network) and the output layer on the matrix cores, the loss of
// ppo_row_loss, and the gradient back through the output layer down to
// hidden layer 1's pre-activations (through hidden layer 3 when there is
// one) -- the work of the forward GEMMs, a per-row loss kernel and the
// data-gradient GEMMs, with the same arithmetic per element: each layer's z = (sum over K) + bias and act(z) rounded to BF16
// as in the GEMM epilogues, the outputs' gradient rounded to BF16 before it
// meets the output weights, dZ = (G_next W_next) act'(Z) from the FP32
// pre-activations, rounded to BF16 for the next product. Within a 32-wide
// K block the matrix cores sum in their own order, so results agree with a
// GEMM formulation to FP32 rounding, not bit for bit. Writes H1, H2 (, H3)
// (the weight gradients' operands), G3b, D2b (, D3b), D1b, and per chunk
// the column sums of dZ2 (, dZ3), dZ1 (cpart2, cpart3, cpart) and the loss
// sums (lpart, kLossPart columns). The weights are staged in LDS once per
// workgroup in the fragment order of mlp.hpp (the K of every layer above
// the first permuted, so a layer's result tile is the next layer's B
// operand straight from registers), plus the transposed output layer (and
// hidden layer 3) for the backward products, whose B operands are gradient
// tiles in the same register layout; for the last product W2^T takes W2's
// place in LDS (and W2 returns before a next chunk). A workgroup walks chunks blockIdx.x,
// blockIdx.x + gridDim.x, ...; eight waves (two per SIMD) hide each other's
// matrix-core and LDS latencies.
constexpr int kFrontWaves = 8;                // one 16-row tile per wave
constexpr int kFrontRows = 16 * kFrontWaves;  // rows per chunk
constexpr int kFrontThreads = 64 * kFrontWaves;
template <int H3> struct FrontShape {
  static constexpr int kKo = H3 ? H3 : kH2;              // the output layer's K
  static constexpr int kW3 = (H3 / 16) * (kH2 / 32) * 64;  // W3 [H3/16 row tiles][4 K-blocks][64 lanes]
  static constexpr int kWo = (kKo / 32) * 64;              // Wo [K-blocks][64 lanes]
  static constexpr int kWoT = (kKo / 16) * 64;             // Wo^T [row tiles of the last hidden layer][64 lanes]
  static constexpr int kW3T = (kH2 / 16) * (H3 / 32) * 64; // W3^T [8 row tiles][H3/32 K-blocks][64 lanes]
  static constexpr int kFrags = kW1Frags + kW2Frags + kW3 + kWo + kWoT + kW3T;
  static constexpr int kBias = kH1 + kH2 + H3 + kOut;
  static constexpr int kCols = kH2 + H3 + kH1;             // column sums per wave (dZ2 | dZ3 | dZ1)
  static constexpr size_t kLds = (size_t)kFrags * 16 + (size_t)kBias * 4 +
                                 (size_t)kFrontWaves * 16 * kPO * 4 +        // outputs, [wave][row][kPO]
                                 (size_t)kFrontWaves * (2 * kPO + 4) * 4 +   // loss sums, [wave][..]
                                 (size_t)kFrontWaves * kCols * 4;            // column sums, [wave][kCols]
};
static_assert(FrontShape<0>::kLds <= 160 * 1024 && FrontShape<64>::kLds <= 160 * 1024, "the fused front fits the LDS");

struct FrontArgs {
  const uint16_t* X;   // [rows][kPX] BF16 inputs
  const uint16_t* pb;  // BF16 parameters: W1 at oW[0] [256][W], W2 at oW[1] [128][256],
                       // W3 at oW[2] [H3][128], Wo at oWo [O][Ko]
  const float* p;      // FP32 parameters (biases at oB[], oBo; log_std at oLS)
  int oW[3], oB[3], oWo, oBo, oLS;
  int W, O;
  const uint4* img;    // the fragment images (PpoImg)
  PpoImg im;
  PpoRows rows;
  float clip, c_v, inv_b, w_stats;
  uint16_t* H1;        // [rows][256]
  uint16_t* H2;        // [rows][128]
  uint16_t* H3;        // [rows][H3]
  uint16_t* G3b;       // [rows][kPO]
  uint16_t* D2b;       // [rows][128]
  uint16_t* D3b;       // [rows][H3]
  uint16_t* D1b;       // [rows][256]
  float* cpart2;       // [chunks][128]
  float* cpart3;       // [chunks][H3]
  float* cpart;        // [chunks][256] (dZ1)
  float* lpart;        // [chunks][kLossPart]
  int nchunks;
};

__device__ __forceinline__ uint2 bf16x4_bits(const bf16x8& v, int h) {
  const uint32_t* u = reinterpret_cast<const uint32_t*>(&v);
  return make_uint2(u[2 * h], u[2 * h + 1]);
}
__device__ __forceinline__ bf16x8 frag(const uint4* s, int i) {
  const uint4 t = s[i];
  return *reinterpret_cast<const bf16x8*>(&t);
}

// Sums over the 16 lanes of a DPP row (lanes 16g .. 16g + 15) of N values
// at once, stage by stage so that no add waits on the one before it; lane
// 16g receives the row's sums (the others partial sums in other orders).
// update_dpp with a zero old value and bound_ctrl lets the compiler fold
// the moves into the adds (v_add_f32 with a DPP source).
template <int N> __device__ __forceinline__ void row16_sums(float (&v)[N]) {
#define SG_DPP_STAGE(ctrl)                                                                            \
  _Pragma("unroll") for (int k = 0; k < N; ++k) v[k] +=                                              \
      __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[k]), ctrl, 0xF, 0xF, true));
  SG_DPP_STAGE(0xB1)   // quad_perm 1,0,3,2
  SG_DPP_STAGE(0x4E)   // quad_perm 2,3,0,1
  SG_DPP_STAGE(0x124)  // row_ror 4
  SG_DPP_STAGE(0x128)  // row_ror 8
#undef SG_DPP_STAGE
}

// Per-element activation, its derivative from the FP32 pre-activation z
template <int ACT> __device__ __forceinline__ float act_and_grad(float z, float& d) {
  if (ACT == ACT_TANH) {
    const float t = tanh_fast(z);
    d = 1.f - t * t;
    return t;
  }
  d = elu_grad_f(z);
  return elu_f(z);
}

template <int ACT, int H3>
__global__ void __launch_bounds__(kFrontThreads) k_ppo_front(FrontArgs a) {
  using S = FrontShape<H3>;
  constexpr int NT = kFrontThreads;
  constexpr int KO = S::kKo;
  extern __shared__ __align__(16) unsigned char lds[];
  uint4* sW1 = reinterpret_cast<uint4*>(lds);
  uint4* sW2 = sW1 + kW1Frags;
  uint4* sW3 = sW2 + kW2Frags;
  uint4* sWo = sW3 + S::kW3;
  uint4* sWoT = sWo + S::kWo;
  uint4* sW3T = sWoT + S::kWoT;
  float* sb1 = reinterpret_cast<float*>(lds + (size_t)S::kFrags * 16);
  float* sb2 = sb1 + kH1;
  float* sb3 = sb2 + kH2;
  float* sbo = sb3 + H3;
  float* sO = sbo + kOut;
  float* sRed = sO + kFrontWaves * 16 * kPO;
  float* sCol = sRed + kFrontWaves * (2 * kPO + 4);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, i = lane & 15;
  const PpoRows& R = a.rows;
  // the first chunk's input tile, in flight during the weight staging
  int c = blockIdx.x;
  uint4 xn = make_uint4(0, 0, 0, 0);
  {
    const int r = c * kFrontRows + 16 * wave + i;
    if (r < R.rows) xn = *reinterpret_cast<const uint4*>(a.X + (size_t)r * kPX + 8 * g);
  }
  // weight images in LDS from their fragment-order copies: every thread
  // issues all of its 16-byte loads before its first LDS store
  {
    constexpr int nW1 = kW1Frags / NT, nW2 = kW2Frags / NT, nW3 = S::kW3 / NT, nWoT = (S::kWoT + NT - 1) / NT,
                  nW3T = S::kW3T / NT;
    static_assert(kW1Frags % NT == 0 && kW2Frags % NT == 0 && S::kW3 % NT == 0 && S::kW3T % NT == 0 &&
                      S::kWo <= NT && kH1 <= NT,
                  "the staging loops are exact");
    const PpoImg& m = a.im;
    uint4 w1[nW1], w2[nW2], w3[nW3 ? nW3 : 1], wo, wt[nWoT], w3t[nW3T ? nW3T : 1];
#pragma unroll
    for (int u = 0; u < nW1; ++u) w1[u] = a.img[m.fW1 + tid + NT * u];
#pragma unroll
    for (int u = 0; u < nW2; ++u) w2[u] = a.img[m.fW2 + tid + NT * u];
#pragma unroll
    for (int u = 0; u < nW3; ++u) w3[u] = a.img[m.fW3 + tid + NT * u];
    wo = tid < S::kWo ? a.img[m.fWo + tid] : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < nWoT; ++u) wt[u] = tid + NT * u < S::kWoT ? a.img[m.fWoT + tid + NT * u] : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < nW3T; ++u) w3t[u] = a.img[m.fW3T + tid + NT * u];
    const float b1 = tid < kH1 ? a.p[a.oB[0] + tid] : 0.f;
    const float b2 = tid < kH2 ? a.p[a.oB[1] + tid] : 0.f;
    const float b3 = tid < H3 ? a.p[a.oB[2] + tid] : 0.f;
    const float bo = tid < a.O ? a.p[a.oBo + tid] : 0.f;
#pragma unroll
    for (int u = 0; u < nW1; ++u) sW1[tid + NT * u] = w1[u];
#pragma unroll
    for (int u = 0; u < nW2; ++u) sW2[tid + NT * u] = w2[u];
#pragma unroll
    for (int u = 0; u < nW3; ++u) sW3[tid + NT * u] = w3[u];
    if (tid < S::kWo) sWo[tid] = wo;
#pragma unroll
    for (int u = 0; u < nWoT; ++u)
      if (tid + NT * u < S::kWoT) sWoT[tid + NT * u] = wt[u];
#pragma unroll
    for (int u = 0; u < nW3T; ++u) sW3T[tid + NT * u] = w3t[u];
    if (tid < kH1) sb1[tid] = b1;
    if (tid < kH2) sb2[tid] = b2;
    if (tid < H3) sb3[tid] = b3;
    if (tid < kOut) sbo[tid] = bo;
  }
  __syncthreads();
  const float* ls = a.p + a.oLS;
  const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};

  for (; c < a.nchunks; c += gridDim.x) {
    // this wave's tile: rows rb .. rb + 15; lane 16 g + i works on row rb + i
    const int rb = c * kFrontRows + 16 * wave, rj = rb + i;
    const bool rv = rj < R.rows;
    bf16x8 xb = *reinterpret_cast<const bf16x8*>(&xn);
    // the next chunk's input tile and this chunk's loss inputs, in flight
    // during the layers
    {
      const int r = rj + gridDim.x * kFrontRows;
      xn = c + (int)gridDim.x < a.nchunks && r < R.rows ? *reinterpret_cast<const uint4*>(a.X + (size_t)r * kPX + 8 * g)
                                                       : make_uint4(0, 0, 0, 0);
    }
    float xa[kAux];
    bool ok = false;
    if (g == 0 && rv) ok = ppo_row_inputs(R, rj, xa);
    // layers 1 and 2: K-block kb of layer 2 is layer 1's row tiles 2kb, 2kb+1;
    // layer 1's act' kept for the gradient at the end
    float dact1[kH1 / 16][4];
    f32x4 acc2[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) acc2[m] = zero4;
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      bf16x8 hb;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f32x4 d = mfma16x16x32(frag(sW1, (2 * kb + h) * 64 + lane), xb, zero4);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          hb[4 * h + r] = (__bf16)act_and_grad<ACT>(d[r] + sb1[32 * kb + 16 * h + 4 * g + r], dact1[2 * kb + h][r]);
      }
      if (rv) {
        uint16_t* dst = a.H1 + (size_t)rj * kH1 + 32 * kb + 4 * g;
        *reinterpret_cast<uint2*>(dst) = bf16x4_bits(hb, 0);
        *reinterpret_cast<uint2*>(dst + 16) = bf16x4_bits(hb, 1);
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) acc2[m] = mfma16x16x32(frag(sW2, (m * 8 + kb) * 64 + lane), hb, acc2[m]);
    }
    // layer 2's activations (BF16, the next layer's B operand) and act'
    float dact2[8][4];
    bf16x8 h2b[4];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        h2b[m >> 1][4 * (m & 1) + r] = (__bf16)act_and_grad<ACT>(acc2[m][r] + sb2[16 * m + 4 * g + r], dact2[m][r]);
    if (rv) {
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        uint16_t* dst = a.H2 + (size_t)rj * kH2 + 32 * kb + 4 * g;
        *reinterpret_cast<uint2*>(dst) = bf16x4_bits(h2b[kb], 0);
        *reinterpret_cast<uint2*>(dst + 16) = bf16x4_bits(h2b[kb], 1);
      }
    }
    // layer 3 (if any), then the output layer on the last hidden layer
    constexpr int M3 = H3 / 16;
    float dact3[M3 ? M3 : 1][4];
    bf16x8 h3b[M3 ? M3 / 2 : 1];
    f32x4 acco = zero4;
    if constexpr (H3 > 0) {
      f32x4 acc3[M3];
#pragma unroll
      for (int m = 0; m < M3; ++m) acc3[m] = zero4;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int m = 0; m < M3; ++m) acc3[m] = mfma16x16x32(frag(sW3, (m * 4 + kb) * 64 + lane), h2b[kb], acc3[m]);
#pragma unroll
      for (int m = 0; m < M3; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          h3b[m >> 1][4 * (m & 1) + r] = (__bf16)act_and_grad<ACT>(acc3[m][r] + sb3[16 * m + 4 * g + r], dact3[m][r]);
      if (rv) {
#pragma unroll
        for (int kb = 0; kb < M3 / 2; ++kb) {
          uint16_t* dst = a.H3 + (size_t)rj * H3 + 32 * kb + 4 * g;
          *reinterpret_cast<uint2*>(dst) = bf16x4_bits(h3b[kb], 0);
          *reinterpret_cast<uint2*>(dst + 16) = bf16x4_bits(h3b[kb], 1);
        }
      }
#pragma unroll
      for (int kb = 0; kb < M3 / 2; ++kb) acco = mfma16x16x32(frag(sWo, kb * 64 + lane), h3b[kb], acco);
    } else {
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acco = mfma16x16x32(frag(sWo, kb * 64 + lane), h2b[kb], acco);
    }
    // outputs to LDS (lane groups 0 and 1 hold outputs 0..7 of row rb + i)
    if (g < 2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) sO[(wave * 16 + i) * kPO + 4 * g + r] = acco[r] + sbo[4 * g + r];
    }
    __syncthreads();
    // the loss, one row per lane of lane group 0
    float lpi = 0.f, lv = 0.f, kl = 0.f, cf = 0.f;
    float gk[kPO], dl[kPO];
#pragma unroll
    for (int k = 0; k < kPO; ++k) { gk[k] = 0.f; dl[k] = 0.f; }
    bf16x8 gb;
#pragma unroll
    for (int k = 0; k < 8; ++k) gb[k] = (__bf16)0.f;
    if (g == 0 && rv) {
      if (ok) {
        float z[kPO];
#pragma unroll
        for (int k = 0; k < kPO; ++k) z[k] = sO[(wave * 16 + i) * kPO + k];
        ppo_row_loss(R.J, xa, z, ls, a.clip, a.c_v, a.inv_b, gk, dl, lpi, lv, kl, cf);
#pragma unroll
        for (int k = 0; k < kPO; ++k) gb[k] = (__bf16)gk[k];
      }
      *reinterpret_cast<uint4*>(a.G3b + (size_t)rj * kPO) = *reinterpret_cast<const uint4*>(&gb);
    }
    // the gradient through the output layer: B operand = the rows' BF16
    // output gradients (K = outputs, held by lane group 0), A = Wo^T; then,
    // with a third hidden layer, through it: B = the BF16 dZ3 tiles, A =
    // W3^T. Column sums over the tile's 16 rows (one DPP row per lane
    // group), then over the waves in order.
    bf16x8 d3b[M3 ? M3 / 2 : 1];
    if constexpr (H3 > 0) {
#pragma unroll
      for (int m = 0; m < M3; ++m) {
        const f32x4 d = mfma16x16x32(frag(sWoT, m * 64 + lane), gb, zero4);
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          v[r] = d[r] * dact3[m][r];
          d3b[m >> 1][4 * (m & 1) + r] = (__bf16)v[r];
        }
        if (rv) *reinterpret_cast<uint2*>(a.D3b + (size_t)rj * H3 + 16 * m + 4 * g) = bf16x4_bits(d3b[m >> 1], m & 1);
        row16_sums(v);
        if (i == 0) *reinterpret_cast<float4*>(sCol + wave * S::kCols + kH2 + 16 * m + 4 * g) = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
    bf16x8 d2b[kH2 / 32];  // dZ2 as the B operand of dZ1's product (permuted K)
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      f32x4 d;
      if constexpr (H3 > 0) {
        d = zero4;
#pragma unroll
        for (int kb = 0; kb < M3 / 2; ++kb) d = mfma16x16x32(frag(sW3T, (m * (M3 / 2) + kb) * 64 + lane), d3b[kb], d);
      } else {
        d = mfma16x16x32(frag(sWoT, m * 64 + lane), gb, zero4);
      }
      bf16x8 o;
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] = d[r] * dact2[m][r];
        o[r] = (__bf16)v[r];
        d2b[m >> 1][4 * (m & 1) + r] = o[r];
      }
      if (rv) *reinterpret_cast<uint2*>(a.D2b + (size_t)rj * kH2 + 16 * m + 4 * g) = bf16x4_bits(o, 0);
      row16_sums(v);
      if (i == 0) *reinterpret_cast<float4*>(sCol + wave * S::kCols + 16 * m + 4 * g) = make_float4(v[0], v[1], v[2], v[3]);
    }
    {
      const float w = a.w_stats * a.inv_b;
      constexpr int L = 2 * kPO + 4;
      float v[L];
#pragma unroll
      for (int k = 0; k < kPO; ++k) { v[k] = gk[k]; v[kPO + k] = dl[k]; }
      v[2 * kPO] = lpi * w; v[2 * kPO + 1] = lv * w; v[2 * kPO + 2] = kl * w; v[2 * kPO + 3] = cf * w;
      row16_sums(v);
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < L; ++k) sRed[wave * L + k] = v[k];
      }
    }
    // hidden layer 1's gradient: W2^T (permuted K) replaces W2 in LDS once
    // every wave is past its last read of the layer images; dZ1^T =
    // W2^T dZ2^T with dZ2's tiles as B operands, times act'(Z1)
    __syncthreads();
    {
      constexpr int nW2 = kW2Frags / NT;
      uint4 w2t[nW2];
#pragma unroll
      for (int u = 0; u < nW2; ++u) w2t[u] = a.img[a.im.fW2T + tid + NT * u];
#pragma unroll
      for (int u = 0; u < nW2; ++u) sW2[tid + NT * u] = w2t[u];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kH1 / 16; ++t) {
      f32x4 d = zero4;
#pragma unroll
      for (int kb = 0; kb < kH2 / 32; ++kb) d = mfma16x16x32(frag(sW2, (t * (kH2 / 32) + kb) * 64 + lane), d2b[kb], d);
      bf16x8 o;
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] = d[r] * dact1[t][r];
        o[r] = (__bf16)v[r];
      }
      if (rv) *reinterpret_cast<uint2*>(a.D1b + (size_t)rj * kH1 + 16 * t + 4 * g) = bf16x4_bits(o, 0);
      row16_sums(v);
      if (i == 0)
        *reinterpret_cast<float4*>(sCol + wave * S::kCols + kH2 + H3 + 16 * t + 4 * g) = make_float4(v[0], v[1], v[2], v[3]);
    }
    __syncthreads();
    for (int col = tid; col < S::kCols; col += NT) {
      float v = 0.f;
#pragma unroll
      for (int w = 0; w < kFrontWaves; ++w) v += sCol[w * S::kCols + col];
      if (col < kH2) a.cpart2[(size_t)c * kH2 + col] = v;
      else if (col < kH2 + H3) a.cpart3[(size_t)c * H3 + col - kH2] = v;
      else a.cpart[(size_t)c * kH1 + col - kH2 - H3] = v;
    }
    if (tid < kLossPart) {
      // column tid of the row: output, log_std, zero, or statistic
      const int cc = tid, O = a.O;
      const int src = cc < O ? cc : (cc < O + R.J ? kPO + cc - O : (cc >= 16 ? 2 * kPO + cc - 16 : -1));
      constexpr int L = 2 * kPO + 4;
      float v = 0.f;
#pragma unroll
      for (int w = 0; w < kFrontWaves; ++w) v += src < 0 ? 0.f : sRed[w * L + src];
      a.lpart[(size_t)c * kLossPart + cc] = v;
    }
    // W2 back in LDS for the next chunk, if any
    if (c + (int)gridDim.x < a.nchunks) {
      constexpr int nW2 = kW2Frags / NT;
      uint4 w2[nW2];
#pragma unroll
      for (int u = 0; u < nW2; ++u) w2[u] = a.img[a.im.fW2 + tid + NT * u];
#pragma unroll
      for (int u = 0; u < nW2; ++u) sW2[tid + NT * u] = w2[u];
    }
    __syncthreads();
  }
}

// Rows per block of the loss sums and the fused front's column sums
static int loss_blocks(int rows) { return (rows + kFrontRows - 1) / kFrontRows; }

// One workgroup per compute unit at most (104 KB or 131 KB of LDS), walking
// the chunks.
template <int ACT, int H3> static hipError_t launch_front(hipStream_t st, const FrontArgs& a, int n_cu) {
  constexpr size_t lds = FrontShape<H3>::kLds;
  hipError_t e = lds_limit((const void*)k_ppo_front<ACT, H3>, lds);
  if (e != hipSuccess) return e;
  const int grid = a.nchunks < n_cu ? a.nchunks : n_cu;
  k_ppo_front<ACT, H3><<<grid, kFrontThreads, lds, st>>>(a);
  return hipGetLastError();
}

// Entropy bonus on the log_std gradient, then per-block sums of squares
// (double) of kGnormChunk gradient entries into gpart[blockIdx.x].
__global__ void __launch_bounds__(256) k_gnorm_part(float* __restrict__ g, int P, int ls0, int J, float c_e,
                                                    double* __restrict__ gpart) {
  __shared__ double red[256];
  double s = 0;
#pragma unroll
  for (int k = 0; k < kGnormChunk / 256; ++k) {
    const int i = blockIdx.x * kGnormChunk + k * 256 + threadIdx.x;
    if (i < P) {
      float gi = g[i];
      if (i >= ls0 && i < ls0 + J) {
        gi -= c_e;
        g[i] = gi;
      }
      s += (double)gi * gi;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) gpart[blockIdx.x] = red[0];
}

// Block-wide: the minibatch's loss statistics (chunk sums of k_ppo_front,
// in a fixed order), entropy and the gradient norm n, added to stats with
// weight w.
__device__ void add_stats(const float* __restrict__ lpart, int lb, const float* __restrict__ ls, int J, float n,
                          float* __restrict__ stats, float w) {
  __shared__ double red[4][256];
  const int t = threadIdx.x;
  if (t < 256) {  // the first 256 threads sum; the others only meet the barriers
    double v[4] = {0, 0, 0, 0};
    for (int b = t; b < lb; b += 256)
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += lpart[(size_t)b * kLossPart + 16 + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][t] = v[k];
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s)
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + s];
    __syncthreads();
  }
  if (t == 0) {
    float H = 0.f;
    for (int j = 0; j < J; ++j) H += ls[j] + 0.5f + 0.91893853320467274f;
    stats[0] += (float)red[0][0];
    stats[1] += (float)red[1][0];
    stats[2] += H * w;
    stats[3] += (float)red[2][0];
    stats[4] += (float)red[3][0];
    stats[5] += n * w;
  }
}

// |g| from the partial sums of k_gnorm_part into scal[2]; with stats, the
// statistics of add_stats. One block.
__global__ void __launch_bounds__(256) k_ppo_finish(const double* __restrict__ gpart, int nb,
                                                    const float* __restrict__ lpart, int lb,
                                                    const float* __restrict__ ls, int J, float* __restrict__ scal,
                                                    float* __restrict__ stats, float w) {
  __shared__ float nsh;
  if (threadIdx.x == 0) {
    double q = 0;
    for (int b = 0; b < nb; ++b) q += gpart[b];
    nsh = (float)sqrt(q);
    scal[2] = nsh;
  }
  __syncthreads();
  if (stats) add_stats(lpart, lb, ls, J, nsh, stats, w);
}

__device__ __forceinline__ void adam_one(int i, float gi, float coef, float* __restrict__ p, float* __restrict__ m,
                                         float* __restrict__ v, float lr, float b1, float b2, float eps, float c1,
                                         float c2, uint16_t* __restrict__ pb) {
  gi *= coef;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = wi;
  pb[i] = bf16_bits(wi);
}

__device__ __forceinline__ float clip_coef(float max_norm, float n) {
  return max_norm > 0.f ? fminf(1.f, max_norm / (n + 1e-6f)) : 1.f;
}

struct NormAdamArgs {
  int P, ls0, J;
  float* p;
  const float* g;
  float* m;
  float* v;
  uint16_t* pb;
  uint16_t* img;    // the fragment images, kept in step with pb
  PpoImg im;
  float* scal;
  float c_e, max_norm, lr, b1, b2, eps;
  uint64_t* tstep;  // Adam steps taken before this one; the launch advances it by one
  unsigned* ttick;
  const float* lpart;
  int lb;
  const double* npart;  // the gradient's squared-norm partials (entropy term included), nparts of them;
  int nparts;           // 0: sum the gradient here
  float* stats;
  float w;
  int nadam;       // blocks [0, nadam) take the Adam step
  PpoRows next;    // blocks from nadam on gather the next minibatch's rows
  uint16_t* X;     // into X (its reads by this minibatch are done)
};

constexpr int kNormAdamThreads = 1024;  // threads per k_ppo_norm_adam block = parameters it updates

// End of a k_ppo_norm_adam Adam block (every thread calls it): once all of
// the block's threads have read the step count, its first thread takes a
// ticket; the last Adam block's ticket stores the new count (the gather
// blocks do not read it).
__device__ __forceinline__ void norm_adam_ticket(const NormAdamArgs& a, uint64_t step) {
  // every wave's read of the count has returned before the ticket is taken
  asm volatile("" ::"v"((uint32_t)step), "v"((uint32_t)(step >> 32)));
  __syncthreads();
  if (threadIdx.x == 0) {
    if (atomicAdd(a.ttick, 1u) == (unsigned)a.nadam - 1) {
      *a.tstep = step;
      *a.ttick = 0u;
    }
  }
}

// The step after a minibatch gradient in one launch (the norm and
// statistics of k_gnorm_part and k_ppo_finish, then Adam): every block sums the squares of the
// whole gradient (entropy term on the log_std entries included) in the same
// fixed order, so each holds the same |g| without a grid-wide barrier, then
// clips and applies Adam to its own kNormAdamThreads parameters. The log_std
// entries (the last J parameters) all belong to the block whose range holds
// the first of them: it stores |g| in scal[2] and adds the statistics
// (which read log_std) before it updates them, and no other block writes
// them. Blocks past the Adam blocks gather the next minibatch's rows.
__global__ void __launch_bounds__(kNormAdamThreads) k_ppo_norm_adam(NormAdamArgs a) {
  constexpr int NT = kNormAdamThreads, NL = 12;
  __shared__ double red[NT / 64];
  __shared__ float nsh;
  __shared__ float csh[2];
  const int t = threadIdx.x;
  // this Adam step's number: every block reads the count; at the end the
  // last block to have read it advances it
  if ((int)blockIdx.x >= a.nadam) {
    const int r = ((int)blockIdx.x - a.nadam) * NT + t;
    if (r < a.next.rows) gather_row(a.next, r, a.X);
    return;
  }
  const uint64_t step = __atomic_load_n(a.tstep, __ATOMIC_RELAXED) + 1;
  double s = 0;
  // the squared norm: from the sum launch's partials when it wrote them,
  // else entries below ls0 as 16-byte vectors, NL loads in flight per
  // thread, the rest (at most 3 + J entries) one per thread
  const int n4 = a.nparts > 0 ? 0 : a.ls0 >> 2;
  for (int i = t; i < a.nparts; i += NT) s += a.npart[i];
  const float4* g4 = reinterpret_cast<const float4*>(a.g);
  for (int base = 0; base < n4; base += NL * NT) {
    float4 x[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int i4 = base + u * NT + t;
      x[u] = i4 < n4 ? g4[i4] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < NL; ++u)
      s += ((double)x[u].x * x[u].x + (double)x[u].y * x[u].y) + ((double)x[u].z * x[u].z + (double)x[u].w * x[u].w);
  }
  for (int i = 4 * n4 + t; a.nparts == 0 && i < a.P; i += NT) {
    float gi = a.g[i];
    if (i >= a.ls0) gi -= a.c_e;
    s += (double)gi * gi;
  }
  // wave sums (xor butterfly), then the 16 wave sums in order: every block
  // adds in the same fixed order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  if (t == 0) {
    double q = 0;
    for (int w = 0; w < NT / 64; ++w) q += red[w];
    nsh = (float)sqrt(q);
    // Adam's bias corrections 1 - beta^step
    csh[0] = 1.f - (float)pow((double)a.b1, (double)step);
    csh[1] = 1.f - (float)pow((double)a.b2, (double)step);
  }
  __syncthreads();
  const float n = nsh;
  const float coef = clip_coef(a.max_norm, n);
  const float c1 = csh[0], c2 = csh[1];
  const int i0 = blockIdx.x * NT;
  const int i = i0 + t;
  if (i < a.ls0) {
    adam_one(i, a.g[i], coef, a.p, a.m, a.v, a.lr, a.b1, a.b2, a.eps, c1, c2, a.pb);
    img_scatter(a.im, i, a.pb[i], a.img);
  }
  if (a.ls0 >= i0 && a.ls0 < i0 + NT) {
    if (t == 0) a.scal[2] = n;
    if (a.stats) add_stats(a.lpart, a.lb, a.p + a.ls0, a.J, n, a.stats, a.w);
    __syncthreads();
    for (int j = a.ls0 + t; j < a.ls0 + a.J; j += NT)
      adam_one(j, a.g[j] - a.c_e, coef, a.p, a.m, a.v, a.lr, a.b1, a.b2, a.eps, c1, c2, a.pb);
  }
  norm_adam_ticket(a, step);
}

// Rollout weight image (fragment order of mlp.hpp, through img_source, as
// sg_set_policy packs it), bias image and log_std from the master
// parameters: per layer l, W at oW[l] ([out][in]) and b at oB[l]; the
// output layer is the last of nl.
struct PackArgs {
  const float* p;
  int W, O, J, nl;
  int oW[4], oB[4], oLS;
  uint16_t* img;
  float* bias;
  float* log_std;
};
template <int H3>
__global__ void __launch_bounds__(256) k_ppo_pack(PackArgs a) {
  using S = PolicyShape<H3>;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < S::kWFrags * 8) {
    const int s = i & 7, l = (i >> 3) & 63, f = i >> 9;
    int layer, row, k;
    float x = 0.f;
    if (img_source<H3>(f, l, s, a.W, a.O, &layer, &row, &k)) {
      const int L = layer == 3 ? a.nl - 1 : layer;
      const int K = L == 0 ? a.W : (L == 1 ? kH1 : (L == 2 && H3 ? kH2 : (H3 ? H3 : kH2)));
      x = a.p[a.oW[L] + row * K + k];
    }
    a.img[i] = bf16_bits(x);
  }
  if (i < S::kBias) {
    float b = 0.f;
    if (i < kH1) b = a.p[a.oB[0] + i];
    else if (i < kH1 + kH2) b = a.p[a.oB[1] + i - kH1];
    else if (i < kH1 + kH2 + H3) b = a.p[a.oB[2] + i - kH1 - kH2];
    else if (i - kH1 - kH2 - H3 < a.O) b = a.p[a.oB[a.nl - 1] + i - kH1 - kH2 - H3];
    a.bias[i] = b;
  }
  if (i < a.J) a.log_std[i] = a.p[a.oLS + i];
}

// A fill kernel rather than a memset node, so the update can be captured.
__global__ void __launch_bounds__(256) k_zero(float* __restrict__ x, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = 0.f;
}

// Gradient of one minibatch into o->g. With `finish`, the entropy term is
// added to o->g, its norm goes to scal[2] and the statistics (weight
// w_stats) to stats; without, k_ppo_norm_adam does both next. ACT: the
// hidden activation (nn.hpp's ACT_TANH / ACT_ELU).
template <int ACT>
static hipError_t minibatch_grad_t(sg_ppo* o, const PpoRows& rows, const sg_ppo_config* cfg, float w_stats,
                                   float* stats, bool finish, bool gathered) {
  sg_ctx* c = o->ctx;
  hipStream_t st = c->stream;
  const int B = rows.rows, W = o->W, O = o->O, J = o->J, h3 = o->h3, L = o->nl - 1;  // L: output layer
  const int gb = (B + 255) / 256, lb = loss_blocks(B);
  // every entry of o->g is written below (weight and bias sums), so no clear
  if (!gathered) k_ppo_gather<<<gb, 256, 0, st>>>(rows, o->X);
  // forward, loss and the gradient down to dZ2 in one launch
  FrontArgs fa;
  fa.X = o->X; fa.pb = o->pb; fa.p = o->p; fa.img = reinterpret_cast<const uint4*>(o->img); fa.im = o->im;
  for (int l = 0; l < 3; ++l) { fa.oW[l] = o->oW[l]; fa.oB[l] = o->oB[l]; }
  fa.oWo = o->oW[L]; fa.oBo = o->oB[L]; fa.oLS = o->oLS;
  fa.W = W; fa.O = O; fa.rows = rows;
  fa.clip = cfg->clip; fa.c_v = cfg->value_coef; fa.inv_b = 1.f / (float)B; fa.w_stats = w_stats;
  fa.H1 = o->H1; fa.H2 = o->H2; fa.H3 = o->H3; fa.G3b = o->G3b; fa.D2b = o->D2b; fa.D3b = o->D3b; fa.D1b = o->D1b;
  fa.cpart2 = o->cpart2; fa.cpart3 = o->cpart3; fa.cpart = o->cpart; fa.lpart = o->lpart;
  fa.nchunks = lb;
  {
    // the two networks sg_ppo_create accepts: 256-128 tanh, 256-128-64 ELU
    if ((ACT == ACT_TANH) != (h3 == 0)) return hipErrorInvalidValue;
    const hipError_t e = ACT == ACT_TANH ? launch_front<ACT_TANH, 0>(st, fa, c->n_cu)
                                         : launch_front<ACT_ELU, 64>(st, fa, c->n_cu);
    if (e != hipSuccess) return e;
  }
  // weight gradients as split-K partials; their sums and the bias sums run
  // in one launch at the end. Output biases and log_std are adjacent in the
  // flat vector (oLS = oB[L] + O).
  SumJob jobs[8];
  int nj = 0;
  WeightGradGroup<ACT_TANH> wg;  // all weight gradients in one launch, after hidden layer 1's gradient
  const int hl = h3 ? h3 : kH2;
  jobs[nj++] = wg.add(O, hl, B, o->G3b, kPO, h3 ? o->H3 : o->H2, hl, o->g + o->oW[L], hl, o->ws + 3 * kWeightGradWs);
  jobs[nj++] = partial_rows(o->lpart, lb, O + J, kLossPart, o->g + o->oB[L]);
  if (h3) {
    jobs[nj++] = wg.add(h3, kH2, B, o->D3b, h3, o->H2, kH2, o->g + o->oW[2], kH2, o->ws + 2 * kWeightGradWs);
    jobs[nj++] = partial_rows(o->cpart3, lb, h3, h3, o->g + o->oB[2]);
  }
  jobs[nj++] = wg.add(kH2, kH1, B, o->D2b, kH2, o->H1, kH1, o->g + o->oW[1], kH1, o->ws + 1 * kWeightGradWs);
  jobs[nj++] = partial_rows(o->cpart2, lb, kH2, kH2, o->g + o->oB[1]);
  // hidden layer 1's weight gradient from the front's D1b
  jobs[nj++] = wg.add(kH1, W, B, o->D1b, kH1, o->X, kPX, o->g + o->oW[0], W, o->ws + 0 * kWeightGradWs);
  jobs[nj++] = partial_rows(o->cpart, lb, kH1, kH1, o->g + o->oB[0]);
  wg.launch(st);
  {
    // with the Adam step next, the sums also leave the gradient's
    // squared-norm partials for it
    SumNorm nm{};
    int blocks = 0;
    for (int k = 0; k < nj; ++k) blocks += sum_job_blocks(jobs[k]);
    if (!finish && blocks <= kNormParts) {
      nm.base = o->g; nm.adj0 = o->oLS; nm.adjn = J; nm.adj = cfg->entropy_coef; nm.npart = o->npart;
    }
    const int nb = launch_sums(st, jobs, nj, nm);
    o->nparts = nm.npart ? nb : 0;
  }
  if (finish) {
    const int nb = (o->P + kGnormChunk - 1) / kGnormChunk;
    k_gnorm_part<<<nb, 256, 0, st>>>(o->g, o->P, o->oLS, J, cfg->entropy_coef, o->gpart);
    k_ppo_finish<<<1, 256, 0, st>>>(o->gpart, nb, o->lpart, lb, o->p + o->oLS, J, o->scal, stats, w_stats);
  }
  return hipGetLastError();
}

static hipError_t minibatch_grad(sg_ppo* o, const PpoRows& rows, const sg_ppo_config* cfg, float w_stats,
                                 float* stats, bool finish, bool gathered = false) {
  return o->act == PACT_ELU ? minibatch_grad_t<ACT_ELU>(o, rows, cfg, w_stats, stats, finish, gathered)
                            : minibatch_grad_t<ACT_TANH>(o, rows, cfg, w_stats, stats, finish, gathered);
}

static PpoRows rows_of(const sg_ppo* o, const sg_rollout_bufs* b, int T) {
  PpoRows r{};
  r.obs = b->obs; r.act = b->act; r.logp = b->logp; r.val = b->val; r.ret = b->ret; r.an = o->an;
  r.xall = o->Xall;
  r.aux = o->Aux;
  r.N = o->ctx->N; r.J = o->J; r.W = o->W; r.total = T * o->ctx->N;
  return r;
}

// Per update: normalised advantages and the sample-major observation rows.
static hipError_t prepare_batch(sg_ppo* o, const sg_rollout_bufs* b, int n) {
  hipStream_t st = o->ctx->stream;
  k_adv_sum<<<kAdvBlocks, 256, 0, st>>>(b->adv, n, o->gpart);
  k_adv_sq<<<kAdvBlocks, 256, 0, st>>>(b->adv, n, o->gpart);
  k_adv_norm<<<(n + 255) / 256, 256, 0, st>>>(b->adv, n, o->gpart, o->an, o->scal);
  PpoRows r{};
  r.act = b->act; r.logp = b->logp; r.val = b->val; r.ret = b->ret; r.an = o->an; r.J = o->J;
  k_ppo_xall<<<(n + 255) / 256, 256, 0, st>>>(b->obs, n, o->ctx->N, o->W, o->Xall, r, o->Aux);
  return hipGetLastError();
}

static hipError_t pack_policy(sg_ppo* o) {
  sg_ctx* c = o->ctx;
  PackArgs a;
  a.p = o->p; a.W = o->W; a.O = o->O; a.J = o->J; a.nl = o->nl; a.oLS = o->oLS;
  for (int l = 0; l < 4; ++l) { a.oW[l] = o->oW[l]; a.oB[l] = o->oB[l]; }
  a.img = c->w_bf16; a.bias = c->bias; a.log_std = c->log_std;
  if (o->h3) {
    const int n = PolicyShape<64>::kWFrags * 8;
    k_ppo_pack<64><<<(n + 255) / 256, 256, 0, c->stream>>>(a);
  } else {
    const int n = PolicyShape<0>::kWFrags * 8;
    k_ppo_pack<0><<<(n + 255) / 256, 256, 0, c->stream>>>(a);
  }
  return hipGetLastError();
}

}  // namespace sgk

using namespace sgk;

namespace {

sg_status pfail(sg_ctx* c, sg_status st, const char* msg) {
  if (c) c->err = msg;
  return st;
}

template <typename T> hipError_t palloc(sg_ppo* o, T** p, size_t n) {
  hipError_t e = hipMalloc((void**)p, n * sizeof(T) + 16);
  if (e == hipSuccess) {
    o->allocs.push_back(*p);
    e = hipMemset(*p, 0, n * sizeof(T) + 16);
  }
  return e;
}

bool ok_cfg(const sg_ppo_config* k) {
  return k && k->clip > 0.f && k->value_coef >= 0.f && k->lr > 0.f && k->beta1 >= 0.f && k->beta1 < 1.f &&
         k->beta2 >= 0.f && k->beta2 < 1.f && k->adam_eps > 0.f && k->epochs >= 1 && k->minibatches >= 1;
}

bool ok_bufs(const sg_rollout_bufs* b) {
  return b && b->obs && b->act && b->logp && b->val && b->adv && b->ret;
}

}  // namespace

extern "C" {

sg_status sg_ppo_create(sg_ctx* c, const sg_policy_arch* arch, const float* params, int32_t max_samples,
                        sg_ppo** out) {
  if (!c || !out) return SG_E_INVAL;
  *out = nullptr;
  if (!params || !arch) return pfail(c, SG_E_INVAL, "sg_ppo_create: null params or arch");
  if (c->dtype != SG_F32) return pfail(c, SG_E_UNSUPPORTED, "sg_ppo_create: FP32 contexts only");
  if (c->J > 7) return pfail(c, SG_E_UNSUPPORTED, "sg_ppo_create: max_dof <= 7");
  const int h3 = policy_h3(arch);
  if (h3 < 0) return pfail(c, SG_E_UNSUPPORTED, "sg_ppo_create: supported are 256-128 tanh and 256-128-64 ELU");
  if (h3 && c->prismatic) return pfail(c, SG_E_UNSUPPORTED, "sg_ppo_create: the 256-128-64 network needs revolute chains");
  if (max_samples < 1 || max_samples > (1 << 24)) return pfail(c, SG_E_INVAL, "sg_ppo_create: max_samples in 1..16M");
  sg_ppo* o = new sg_ppo();
  o->ctx = c;
  o->J = c->J;
  o->W = 2 * c->J + 10;
  o->O = c->J + 1;
  o->h3 = h3;
  o->act = arch->act == SG_ACT_ELU ? PACT_ELU : PACT_TANH;
  o->nl = h3 ? 4 : 3;
  o->max_samples = max_samples;
  {
    const int dims[5] = {o->W, kH1, kH2, h3 ? h3 : o->O, o->O};
    int acc = 0;
    for (int l = 0; l < o->nl; ++l) {
      o->oW[l] = acc;
      acc += dims[l + 1] * dims[l];
      o->oB[l] = acc;
      acc += dims[l + 1];
    }
    o->oLS = acc;
    o->P = acc + o->J;
  }
  {
    PpoImg& m = o->im;
    m.W = o->W; m.O = o->O; m.KO = h3 ? h3 : kH2; m.H3 = h3;
    m.oW1 = o->oW[0]; m.oW2 = o->oW[1]; m.oW3 = h3 ? o->oW[2] : 0; m.oWo = o->oW[o->nl - 1];
    m.fW1 = 0;
    m.fW2 = m.fW1 + kW1Frags;
    m.fW3 = m.fW2 + kW2Frags;
    m.fWo = m.fW3 + (h3 ? FrontShape<64>::kW3 : 0);
    m.fWoT = m.fWo + (m.KO / 32) * 64;
    m.fW3T = m.fWoT + (m.KO / 16) * 64;
    m.fW2T = m.fW3T + (h3 ? FrontShape<64>::kW3T : 0);
    m.frags = m.fW2T + kW2Frags;  // W2^T: as many fragments as W2
  }
  const size_t R = (size_t)max_samples, P = (size_t)o->P;
  // split-K partials: one region per layer (launch_weight_grad_partials bound)
  o->ws_floats = 4 * kWeightGradWs;
  hipError_t e = palloc(o, &o->p, P);
  uint64_t* tcount = nullptr;
  if (e == hipSuccess) e = palloc(o, &tcount, 1);  // the step count and (after it) the completion count, zeroed
  if (e == hipSuccess) { o->tstep = tcount; o->ttick = reinterpret_cast<unsigned*>(tcount + 1); }
  if (e == hipSuccess) e = palloc(o, &o->pb, P);
  if (e == hipSuccess) e = palloc(o, &o->img, (size_t)o->im.frags * 8);
  if (e == hipSuccess) e = palloc(o, &o->g, P);
  if (e == hipSuccess) e = palloc(o, &o->m, P);
  if (e == hipSuccess) e = palloc(o, &o->v, P);
  if (e == hipSuccess) e = palloc(o, &o->an, R);
  if (e == hipSuccess) e = palloc(o, &o->scal, 8);
  if (e == hipSuccess) e = palloc(o, &o->X, R * kPX);
  if (e == hipSuccess) e = palloc(o, &o->Xall, R * kPX);
  if (e == hipSuccess) e = palloc(o, &o->Aux, R * kAux);
  if (e == hipSuccess) e = palloc(o, &o->H1, R * kH1);
  if (e == hipSuccess) e = palloc(o, &o->H2, R * kH2);
  if (e == hipSuccess && h3) e = palloc(o, &o->H3, R * h3);
  if (e == hipSuccess && h3) e = palloc(o, &o->D3b, R * h3);
  if (e == hipSuccess && h3) e = palloc(o, &o->cpart3, (size_t)loss_blocks((int)R) * h3);
  if (e == hipSuccess) e = palloc(o, &o->G3b, R * kPO);
  if (e == hipSuccess) e = palloc(o, &o->D2b, R * kH2);
  if (e == hipSuccess) e = palloc(o, &o->D1b, R * kH1);
  if (e == hipSuccess) e = palloc(o, &o->ws, o->ws_floats);
  if (e == hipSuccess) e = palloc(o, &o->cpart, (size_t)loss_blocks((int)R) * kH1);
  if (e == hipSuccess) e = palloc(o, &o->cpart2, (size_t)loss_blocks((int)R) * kH2);
  if (e == hipSuccess) e = palloc(o, &o->lpart, (size_t)loss_blocks((int)R) * kLossPart);
  if (e == hipSuccess) e = palloc(o, &o->gpart, (size_t)kGnormBlocks);
  if (e == hipSuccess) e = palloc(o, &o->npart, (size_t)kNormParts);
  if (e == hipSuccess && (o->P + kGnormChunk - 1) / kGnormChunk > kGnormBlocks) e = hipErrorInvalidValue;
  if (e == hipSuccess && !c->w_bf16) e = hipMalloc((void**)&c->w_bf16, (size_t)kWFragsMax * 16);
  if (e == hipSuccess && !c->bias) e = hipMalloc((void**)&c->bias, (size_t)kBiasMax * sizeof(float));
  if (e == hipSuccess && !c->log_std) e = hipMalloc((void**)&c->log_std, (size_t)c->J * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(o->p, params, P * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    k_to_bf16<<<(o->P + 255) / 256, 256, 0, c->stream>>>(o->P, o->p, o->pb);
    // (palloc zeroed the images' padding)
    k_ppo_img<<<(o->oLS + 255) / 256, 256, 0, c->stream>>>(o->im, o->oLS, o->pb, o->img);
    e = pack_policy(o);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    for (void* p : o->allocs) (void)hipFree(p);
    delete o;
    c->err = std::string("sg_ppo_create: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  c->has_policy = 1;
  c->h1 = kH1;
  c->h2 = kH2;
  c->h3 = h3;
  c->pact = o->act;
  *out = o;
  return SG_OK;
}

void sg_ppo_destroy(sg_ppo* o) {
  if (!o) return;
  (void)hipStreamSynchronize(o->ctx->stream);
  for (void* p : o->allocs) (void)hipFree(p);
  delete o;
}

int32_t sg_ppo_param_count(const sg_ppo* o) { return o ? o->P : 0; }

sg_status sg_ppo_get_params(sg_ppo* o, float* params) {
  if (!o || !params) return SG_E_INVAL;
  hipError_t e = hipStreamSynchronize(o->ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(params, o->p, (size_t)o->P * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    o->ctx->err = std::string("sg_ppo_get_params: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

sg_status sg_ppo_grad(sg_ppo* o, const sg_rollout_bufs* b, int32_t T, const int32_t* idx, int32_t rows,
                      const sg_ppo_config* cfg, float* grad, float* stats) {
  if (!o) return SG_E_INVAL;
  sg_ctx* c = o->ctx;
  if (!ok_bufs(b) || !ok_cfg(cfg) || !grad) return pfail(c, SG_E_INVAL, "sg_ppo_grad: bad argument");
  const long long total = (long long)T * c->N;
  if (T < 1 || total > o->max_samples || rows < 1 || rows > total)
    return pfail(c, SG_E_INVAL, "sg_ppo_grad: T N must be <= max_samples and 1 <= rows <= T N");
  hipStream_t st = c->stream;
  if (stats) k_zero<<<1, 256, 0, st>>>(stats, 8);
  hipError_t e = prepare_batch(o, b, (int)total);
  PpoRows r = rows_of(o, b, T);
  r.idx = idx;
  r.r0 = 0;
  r.rows = rows;
  if (e == hipSuccess) e = minibatch_grad(o, r, cfg, 1.f, stats, true);
  if (e == hipSuccess)
    e = hipMemcpyAsync(grad, o->g, (size_t)o->P * sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) {
    c->err = std::string("sg_ppo_grad: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

sg_status sg_ppo_update(sg_ppo* o, const sg_rollout_bufs* b, int32_t T, const sg_ppo_config* cfg,
                        const int32_t* perm, float* stats) {
  if (!o) return SG_E_INVAL;
  sg_ctx* c = o->ctx;
  if (!ok_bufs(b) || !ok_cfg(cfg)) return pfail(c, SG_E_INVAL, "sg_ppo_update: bad argument");
  const long long total = (long long)T * c->N;
  if (T < 1 || total > o->max_samples) return pfail(c, SG_E_INVAL, "sg_ppo_update: T N must be <= max_samples");
  if (total % cfg->minibatches != 0) return pfail(c, SG_E_INVAL, "sg_ppo_update: minibatches must divide T N");
  hipStream_t st = c->stream;
  const int mb = (int)(total / cfg->minibatches);
  const float w = 1.f / (float)(cfg->epochs * cfg->minibatches);
  if (stats) k_zero<<<1, 256, 0, st>>>(stats, 8);
  hipError_t e = prepare_batch(o, b, (int)total);
  // minibatch (ep, k) of the update
  auto rows_at = [&](int ep, int k) {
    PpoRows r = rows_of(o, b, T);
    r.rows = mb;
    if (perm) {
      r.idx = perm + (size_t)ep * total + (size_t)k * mb;
      r.r0 = 0;
    } else {
      r.idx = nullptr;
      r.r0 = k * mb;
    }
    return r;
  };
  for (int ep = 0; ep < cfg->epochs && e == hipSuccess; ++ep) {
    for (int k = 0; k < cfg->minibatches && e == hipSuccess; ++k) {
      const PpoRows r = rows_at(ep, k);
      // the rows of every minibatch but the first were gathered by the
      // previous minibatch's k_ppo_norm_adam
      e = minibatch_grad(o, r, cfg, w, stats, false, ep > 0 || k > 0);
      if (e != hipSuccess) break;
      NormAdamArgs na;
      na.P = o->P; na.ls0 = o->oLS; na.J = o->J;
      na.p = o->p; na.g = o->g; na.m = o->m; na.v = o->v; na.pb = o->pb; na.scal = o->scal;
      na.img = o->img; na.im = o->im;
      na.c_e = cfg->entropy_coef; na.max_norm = cfg->max_grad_norm; na.lr = cfg->lr;
      na.b1 = cfg->beta1; na.b2 = cfg->beta2; na.eps = cfg->adam_eps;
      na.tstep = o->tstep; na.ttick = o->ttick;
      na.lpart = o->lpart; na.lb = loss_blocks(mb); na.stats = stats; na.w = w;
      na.npart = o->npart; na.nparts = o->nparts;
      na.nadam = (o->P + kNormAdamThreads - 1) / kNormAdamThreads;
      const bool last = k + 1 == cfg->minibatches && ep + 1 == cfg->epochs;
      na.next = last ? PpoRows{} : rows_at(k + 1 < cfg->minibatches ? ep : ep + 1, (k + 1) % cfg->minibatches);
      na.X = o->X;
      const int ng = last ? 0 : (mb + kNormAdamThreads - 1) / kNormAdamThreads;
      k_ppo_norm_adam<<<na.nadam + ng, kNormAdamThreads, 0, st>>>(na);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = pack_policy(o);
  if (e != hipSuccess) {
    c->err = std::string("sg_ppo_update: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

}  // extern "C"
