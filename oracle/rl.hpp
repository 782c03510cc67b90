// Test infrastructure: part of the FP64 CPU oracle. Only tests/, the smoke
// check and the CPU-baseline leg of the benchmark may load or run anything
// under oracle/; the product path never does.
//
// The learning side of a rollout: the policy network's forward pass, the
// Gaussian exploration noise and the advantage estimate.
//   * Policy: the PPO actor-critic (paper Sec. III "Policy learning and
//     control") as a 3-layer MLP with tanh hidden units whose last layer
//     gives the action mean mu and one extra output, the critic's value V.
//     Weights are BF16 values; in "emulate" mode every layer's input
//     activations are rounded to BF16 (round to nearest, ties to even) as the
//     matrix cores consume them, in "exact" mode they are kept in FP64.
//   * Noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
//     numbers: as easy as 1, 2, 3", SC'11) keyed by the 64-bit seed, counter
//     (env, step lo, step hi, block), then Box-Muller on 24-bit uniforms.
//   * GAE (Schulman et al. 2016, cited by the paper for advantage
//     estimation) with the time-out bootstrap of Sec. III: on a time-out the
//     reward is augmented by gamma * V(s_t).
#pragma once
#include <cmath>
#include <cstdint>

namespace ora {

// ---- BF16 rounding -------------------------------------------------------
// Round x to the nearest value with an 8-bit significand (BF16), ties to
// even, by scaling the significand to [128, 256) and rounding to integer.
// Valid for the normal range of BF16 (all values this project produces).
inline double round_bf16(double x) {
  if (x == 0.0 || !std::isfinite(x)) return x;
  int e;
  double m = std::frexp(x, &e);           // x = m 2^e, 0.5 <= |m| < 1
  double s = std::ldexp(m, 8);            // 128 <= |s| < 256
  double r = std::nearbyint(s);           // default rounding: ties to even
  return std::ldexp(r, e - 8);
}

// ---- Philox4x32-10 -------------------------------------------------------
struct Philox4 {
  uint32_t v[4];
};

inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

inline Philox4 philox4x32_10(Philox4 ctr, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;  // round multipliers
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;  // key schedule (Weyl)
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, ctr.v[0], &hi0, &lo0);
    mulhilo32(M1, ctr.v[2], &hi1, &lo1);
    Philox4 n;
    n.v[0] = hi1 ^ ctr.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ ctr.v[3] ^ k1;
    n.v[3] = lo0;
    ctr = n;
  }
  return ctr;
}

// Uniform in (0, 1) from the top 24 bits: exact in FP32 and FP64 alike.
inline double u24(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

// Standard normals for joints 0..n-1 of (env, step): block b covers joints
// 4b..4b+3 as two Box-Muller pairs (x0, x1) and (x2, x3).
inline void gaussian_noise(uint64_t seed, uint32_t env, uint64_t step, int n, double* eps) {
  const double two_pi = 6.283185307179586476925286766559;
  for (int b = 0; 4 * b < n; ++b) {
    Philox4 c = {{env, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)b}};
    Philox4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int p = 0; p < 2; ++p) {
      double u1 = u24(r.v[2 * p]), u2 = u24(r.v[2 * p + 1]);
      double rad = std::sqrt(-2.0 * std::log(u1));
      double th = two_pi * u2;
      int j0 = 4 * b + 2 * p;
      if (j0 < n) eps[j0] = rad * std::cos(th);
      if (j0 + 1 < n) eps[j0 + 1] = rad * std::sin(th);
    }
  }
}

// Four standard normals from one Philox block (env, step, block): the
// Box-Muller pairs (x0, x1) and (x2, x3) as above.
inline void gaussian_block(uint64_t seed, uint32_t env, uint64_t step, uint32_t block, double* out) {
  const double two_pi = 6.283185307179586476925286766559;
  Philox4 c = {{env, (uint32_t)step, (uint32_t)(step >> 32), block}};
  Philox4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  for (int p = 0; p < 2; ++p) {
    double u1 = u24(r.v[2 * p]), u2 = u24(r.v[2 * p + 1]);
    double rad = std::sqrt(-2.0 * std::log(u1));
    out[2 * p] = rad * std::cos(two_pi * u2);
    out[2 * p + 1] = rad * std::sin(two_pi * u2);
  }
}

// ---- policy MLP ----------------------------------------------------------
// Layer l maps n_in -> n_out with W row-major [n_out][n_in]. A hidden
// activation (tanh, or ELU: z for z > 0, e^z - 1 otherwise) after every
// layer but the last.
struct MlpLayer {
  int n_in, n_out;
  const double* W;
  const double* b;
};

enum { kActTanh = 0, kActElu = 1 };

template <class T> inline T hidden_act(int act, const T& z) {
  using std::exp;
  using std::tanh;
  if (act == kActElu) return val(z) > 0.0 ? z : exp(z) - T(1.0);
  return tanh(z);
}
// d act / dz at z
inline double hidden_act_grad(int act, double z) {
  if (act == kActElu) return z > 0.0 ? 1.0 : std::exp(z);
  const double t = std::tanh(z);
  return 1.0 - t * t;
}

// x: [n_in of layer 0]; out: [n_out of the last layer]. emulate: round each
// layer's input to BF16 before the product.
template <class T>
inline void mlp_forward(const MlpLayer* layers, int n_layers, const T* x, T* out, bool emulate, T* scratch_a,
                        T* scratch_b, int act = kActTanh) {
  const T* in = x;
  T* buf[2] = {scratch_a, scratch_b};
  for (int l = 0; l < n_layers; ++l) {
    const MlpLayer& L = layers[l];
    T* o = (l == n_layers - 1) ? out : buf[l & 1];
    T xin[1024];
    for (int k = 0; k < L.n_in; ++k) xin[k] = emulate ? T(round_bf16(val(in[k]))) : in[k];
    for (int i = 0; i < L.n_out; ++i) {
      T s = T(L.b[i]);
      for (int k = 0; k < L.n_in; ++k) s = s + T(L.W[i * L.n_in + k]) * xin[k];
      o[i] = (l == n_layers - 1) ? s : hidden_act(act, s);
    }
    in = o;
  }
}

// ---- GAE -----------------------------------------------------------------
// One env's backward scan. rew, done: [T][N]; val: [T+1][N]; adv, ret:
// [T][N]; env e. done bit 0 = episode ended, bit 1 = time-out.
inline void gae_env(int T_, int N, int e, const double* rew, const double* val_, const uint8_t* done, double gamma,
                    double lam, double* adv, double* ret) {
  double A = 0.0;
  for (int t = T_ - 1; t >= 0; --t) {
    uint8_t d = done[(size_t)t * N + e];
    double notdone = (d & 1) ? 0.0 : 1.0;
    double r = rew[(size_t)t * N + e];
    if (d & 2) r += gamma * val_[(size_t)t * N + e];
    double delta = r + gamma * val_[(size_t)(t + 1) * N + e] * notdone - val_[(size_t)t * N + e];
    A = delta + gamma * lam * notdone * A;
    adv[(size_t)t * N + e] = A;
    ret[(size_t)t * N + e] = A + val_[(size_t)t * N + e];
  }
}

}  // namespace ora
