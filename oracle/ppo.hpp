// Test infrastructure: part of the FP64 CPU oracle. Only tests/, the smoke
// check and the CPU-baseline leg of the benchmark may load or run anything
// under oracle/; the product path never does.
//
// PPO update of the rollout policy (the paper trains with the GPU PPO of
// Rudin et al., Sec. III "Policy learning and control"; the objective is the
// clipped surrogate of Schulman et al., 2017). Written from the definitions:
//   * network: x -> tanh(W1 x + b1) -> tanh(W2 h1 + b2) -> W3 h2 + b3 =
//     [mu (J) | V]; Gaussian policy with state-independent log_std (J);
//   * log pi(a) = sum_j -0.5 ((a_j - mu_j) / sigma_j)^2 - log sigma_j
//     - 0.5 log(2 pi);
//   * ratio r = exp(log pi(a) - log pi_old(a));
//   * policy loss  L_pi = -mean(min(r A, clip(r, 1 - eps, 1 + eps) A));
//   * value loss   L_v  = mean(max((V - R)^2, (V_c - R)^2)),
//     V_c = V_old + clip(V - V_old, -eps, eps);
//   * entropy      H    = sum_j (log sigma_j + 0.5 + 0.5 log(2 pi));
//   * loss L = L_pi + c_v L_v - c_e H;
//   * gradients by the chain rule; global-norm clipping
//     g <- g min(1, max_norm / (|g|_2 + 1e-6)); Adam.
// Advantages are normalised once per update over the whole batch with the
// mean and the unbiased standard deviation (+1e-8).
// Clip derivatives are taken as 1 on the closed interval (the boundary has
// measure zero). "emulate" rounds every matrix-product operand (weights,
// layer inputs, the backward pass's layer gradients) to BF16 as the matrix
// cores consume them.
#pragma once
#include <cmath>
#include <vector>

#include "rl.hpp"

namespace ora {

struct PpoCfg {
  double clip;       // eps of the ratio and value clips
  double c_v, c_e;   // value-loss and entropy coefficients
  double max_norm;   // global gradient-norm bound (<= 0: no clipping)
  double lr, beta1, beta2, adam_eps;
};

// Flat parameter vector: W1 [h1][n_in], b1, W2 [h2][h1], b2, W3 [J+1][h2],
// b3, log_std [J].
struct PpoNet {
  int n_in, h1, h2, J;
  int off[7];
  int size;
  PpoNet(int n_in_, int h1_, int h2_, int J_) : n_in(n_in_), h1(h1_), h2(h2_), J(J_) {
    const int sz[7] = {h1 * n_in, h1, h2 * h1, h2, (J + 1) * h2, J + 1, J};
    int o = 0;
    for (int i = 0; i < 7; ++i) {
      off[i] = o;
      o += sz[i];
    }
    size = o;
  }
};

struct PpoSample {
  const double* x;   // [n_in] observation
  const double* a;   // [J] sampled action (pre-clamp)
  double logp_old, adv, ret, v_old;
};

struct PpoStats {
  double loss_pi = 0, loss_v = 0, entropy = 0, approx_kl = 0, clip_frac = 0;
};

inline double bf(double x, bool emulate) { return emulate ? round_bf16(x) : x; }

// Loss of one minibatch and its gradient (added into g, size net.size).
inline PpoStats ppo_minibatch(const PpoNet& net, const double* p, const std::vector<PpoSample>& mb,
                              const PpoCfg& cfg, bool emulate, double* g) {
  const int n_in = net.n_in, h1 = net.h1, h2 = net.h2, J = net.J, no = J + 1;
  const double* W1 = p + net.off[0];
  const double* b1 = p + net.off[1];
  const double* W2 = p + net.off[2];
  const double* b2 = p + net.off[3];
  const double* W3 = p + net.off[4];
  const double* b3 = p + net.off[5];
  const double* ls = p + net.off[6];
  const double B = (double)mb.size();
  const double log2pi = std::log(2.0 * M_PI);
  PpoStats st;
  double H = 0;
  for (int j = 0; j < J; ++j) H += ls[j] + 0.5 + 0.5 * log2pi;
  st.entropy = H;
  std::vector<double> x(n_in), z1(h1), a1(h1), z2(h2), a2(h2), out(no), d3(no), d2(h2), d1(h1);
  for (const PpoSample& s : mb) {
    // forward
    for (int k = 0; k < n_in; ++k) x[k] = bf(s.x[k], emulate);
    for (int i = 0; i < h1; ++i) {
      double acc = b1[i];
      for (int k = 0; k < n_in; ++k) acc += bf(W1[i * n_in + k], emulate) * x[k];
      z1[i] = acc;
      a1[i] = bf(std::tanh(acc), emulate);
    }
    for (int i = 0; i < h2; ++i) {
      double acc = b2[i];
      for (int k = 0; k < h1; ++k) acc += bf(W2[i * h1 + k], emulate) * a1[k];
      z2[i] = acc;
      a2[i] = bf(std::tanh(acc), emulate);
    }
    for (int i = 0; i < no; ++i) {
      double acc = b3[i];
      for (int k = 0; k < h2; ++k) acc += bf(W3[i * h2 + k], emulate) * a2[k];
      out[i] = acc;
    }
    // loss terms
    double logp = 0;
    for (int j = 0; j < J; ++j) {
      const double u = (s.a[j] - out[j]) / std::exp(ls[j]);
      logp += -0.5 * u * u - ls[j] - 0.5 * log2pi;
    }
    const double r = std::exp(logp - s.logp_old);
    const double rc = std::fmin(std::fmax(r, 1.0 - cfg.clip), 1.0 + cfg.clip);
    st.loss_pi += -std::fmin(r * s.adv, rc * s.adv) / B;
    st.approx_kl += (s.logp_old - logp) / B;
    st.clip_frac += (std::fabs(r - 1.0) > cfg.clip ? 1.0 : 0.0) / B;
    const double V = out[J];
    const double dv = V - s.v_old;
    const double Vc = s.v_old + std::fmin(std::fmax(dv, -cfg.clip), cfg.clip);
    const double e1 = (V - s.ret) * (V - s.ret), e2 = (Vc - s.ret) * (Vc - s.ret);
    st.loss_v += std::fmax(e1, e2) / B;
    // dL/dlogp: the unclipped term is the minimum unless the ratio has left
    // the interval on the side the advantage favours
    const bool live = s.adv >= 0 ? r <= 1.0 + cfg.clip : r >= 1.0 - cfg.clip;
    const double dlogp = live ? -s.adv * r / B : 0.0;
    for (int j = 0; j < J; ++j) {
      const double sig = std::exp(ls[j]);
      const double u = (s.a[j] - out[j]) / sig;
      d3[j] = dlogp * u / sig;                           // dlogp/dmu = (a - mu) / sigma^2
      g[net.off[6] + j] += dlogp * (u * u - 1.0);        // dlogp/dlog_std
    }
    double dV;
    if (e1 >= e2) dV = 2.0 * (V - s.ret);
    else dV = std::fabs(dv) <= cfg.clip ? 2.0 * (Vc - s.ret) : 0.0;
    d3[J] = cfg.c_v * dV / B;
    // backward through the layers
    for (int i = 0; i < no; ++i) {
      const double gi = bf(d3[i], emulate);
      g[net.off[5] + i] += d3[i];
      for (int k = 0; k < h2; ++k) g[net.off[4] + i * h2 + k] += gi * a2[k];
    }
    for (int k = 0; k < h2; ++k) {
      double acc = 0;
      for (int i = 0; i < no; ++i) acc += bf(d3[i], emulate) * bf(W3[i * h2 + k], emulate);
      const double t = std::tanh(z2[k]);
      d2[k] = acc * (1.0 - t * t);
    }
    for (int i = 0; i < h2; ++i) {
      const double gi = bf(d2[i], emulate);
      g[net.off[3] + i] += d2[i];
      for (int k = 0; k < h1; ++k) g[net.off[2] + i * h1 + k] += gi * a1[k];
    }
    for (int k = 0; k < h1; ++k) {
      double acc = 0;
      for (int i = 0; i < h2; ++i) acc += bf(d2[i], emulate) * bf(W2[i * h1 + k], emulate);
      const double t = std::tanh(z1[k]);
      d1[k] = acc * (1.0 - t * t);
    }
    for (int i = 0; i < h1; ++i) {
      const double gi = bf(d1[i], emulate);
      g[net.off[1] + i] += d1[i];
      for (int k = 0; k < n_in; ++k) g[net.off[0] + i * n_in + k] += gi * x[k];
    }
  }
  // entropy bonus: dL/dlog_std_j = -c_e
  for (int j = 0; j < J; ++j) g[net.off[6] + j] += -cfg.c_e;
  return st;
}

inline double ppo_loss(const PpoStats& s, const PpoCfg& cfg) { return s.loss_pi + cfg.c_v * s.loss_v - cfg.c_e * s.entropy; }

// g <- g min(1, max_norm / (|g| + 1e-6)); returns |g| before clipping.
inline double clip_grad_norm(int n, double* g, double max_norm) {
  double s = 0;
  for (int i = 0; i < n; ++i) s += g[i] * g[i];
  const double norm = std::sqrt(s);
  if (max_norm > 0) {
    const double c = std::fmin(1.0, max_norm / (norm + 1e-6));
    for (int i = 0; i < n; ++i) g[i] *= c;
  }
  return norm;
}

// (adv - mean) / (unbiased std + 1e-8) over n values.
inline void normalise_adv(int n, const double* adv, double* out) {
  double m = 0;
  for (int i = 0; i < n; ++i) m += adv[i];
  m /= n;
  double v = 0;
  for (int i = 0; i < n; ++i) v += (adv[i] - m) * (adv[i] - m);
  const double sd = n > 1 ? std::sqrt(v / (n - 1)) : 0.0;
  for (int i = 0; i < n; ++i) out[i] = (adv[i] - m) / (sd + 1e-8);
}

}  // namespace ora
