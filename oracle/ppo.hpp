// Test infrastructure: part of the FP64 CPU oracle. Only tests/, the smoke
// check and the CPU-baseline leg of the benchmark may load or run anything
// under oracle/; the product path never does.
//
// PPO update of the rollout policy (the paper trains with the GPU PPO of
// Rudin et al., Sec. III "Policy learning and control"; the objective is the
// clipped surrogate of Schulman et al., 2017). Written from the definitions:
//   * network: x -> act(W1 x + b1) -> ... -> act(W_L h + b_L) -> W_o h + b_o =
//     [mu (J) | V], act = tanh or ELU (the rollout workload's 2 x tanh
//     trunk, or the paper's Table II network of 256-128-64 ELU units);
//     Gaussian policy with state-independent log_std (J);
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

// Flat parameter vector: per layer l (hidden layers, then the output layer
// of J + 1 rows) W_l [out][in] then b_l [out]; then log_std [J].
struct PpoNet {
  int n_in, J, act;
  std::vector<int> dims;  // n_in, hidden sizes..., J + 1
  std::vector<int> offW, offB;
  int off_ls = 0, size = 0;
  PpoNet(int n_in_, const std::vector<int>& hidden, int J_, int act_) : n_in(n_in_), J(J_), act(act_) {
    dims.push_back(n_in);
    for (int h : hidden) dims.push_back(h);
    dims.push_back(J + 1);
    int o = 0;
    for (size_t l = 0; l + 1 < dims.size(); ++l) {
      offW.push_back(o);
      o += dims[l + 1] * dims[l];
      offB.push_back(o);
      o += dims[l + 1];
    }
    off_ls = o;
    size = o + J;
  }
  int layers() const { return (int)dims.size() - 1; }
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
  const int L = net.layers(), J = net.J, no = J + 1;
  const double* ls = p + net.off_ls;
  const double B = (double)mb.size();
  const double log2pi = std::log(2.0 * M_PI);
  PpoStats st;
  double H = 0;
  for (int j = 0; j < J; ++j) H += ls[j] + 0.5 + 0.5 * log2pi;
  st.entropy = H;
  // a[l]: input of layer l (a[0] = x), z[l]: its pre-activation
  std::vector<std::vector<double>> a(L + 1), z(L), d(L);
  for (int l = 0; l <= L; ++l) a[l].resize(net.dims[l]);
  for (int l = 0; l < L; ++l) {
    z[l].resize(net.dims[l + 1]);
    d[l].resize(net.dims[l + 1]);
  }
  for (const PpoSample& s : mb) {
    // forward
    for (int k = 0; k < net.n_in; ++k) a[0][k] = bf(s.x[k], emulate);
    for (int l = 0; l < L; ++l) {
      const int ni = net.dims[l], nout = net.dims[l + 1];
      const double* W = p + net.offW[l];
      const double* b = p + net.offB[l];
      for (int i = 0; i < nout; ++i) {
        double acc = b[i];
        for (int k = 0; k < ni; ++k) acc += bf(W[i * ni + k], emulate) * a[l][k];
        z[l][i] = acc;
        if (l + 1 < L) a[l + 1][i] = bf(hidden_act(net.act, acc), emulate);
        else a[l + 1][i] = acc;
      }
    }
    const std::vector<double>& out = a[L];
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
    std::vector<double>& dout = d[L - 1];
    for (int j = 0; j < J; ++j) {
      const double sig = std::exp(ls[j]);
      const double u = (s.a[j] - out[j]) / sig;
      dout[j] = dlogp * u / sig;                          // dlogp/dmu = (a - mu) / sigma^2
      g[net.off_ls + j] += dlogp * (u * u - 1.0);         // dlogp/dlog_std
    }
    double dV;
    if (e1 >= e2) dV = 2.0 * (V - s.ret);
    else dV = std::fabs(dv) <= cfg.clip ? 2.0 * (Vc - s.ret) : 0.0;
    dout[J] = cfg.c_v * dV / B;
    (void)no;
    // backward through the layers: d[l] = dL/dz[l]
    for (int l = L - 1; l >= 0; --l) {
      const int ni = net.dims[l], nout = net.dims[l + 1];
      const double* W = p + net.offW[l];
      for (int i = 0; i < nout; ++i) {
        const double gi = bf(d[l][i], emulate);
        g[net.offB[l] + i] += d[l][i];
        for (int k = 0; k < ni; ++k) g[net.offW[l] + i * ni + k] += gi * a[l][k];
      }
      if (l == 0) break;
      for (int k = 0; k < ni; ++k) {
        double acc = 0;
        for (int i = 0; i < nout; ++i) acc += bf(d[l][i], emulate) * bf(W[i * ni + k], emulate);
        d[l - 1][k] = acc * hidden_act_grad(net.act, z[l - 1][k]);
      }
    }
  }
  // entropy bonus: dL/dlog_std_j = -c_e
  for (int j = 0; j < J; ++j) g[net.off_ls + j] += -cfg.c_e;
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
