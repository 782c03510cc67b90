// Test infrastructure: part of the FP64 CPU oracle. Only tests/, the smoke
// check and the CPU-baseline leg of the benchmark may load or run anything
// under oracle/; the product path never does.
//
// Learned forward-dynamics surrogate: an MLP maps (q, qd, tau~, the 10
// standard inertial parameters of every link) to the joint accelerations of
// the implicit-PD substep, qdd = (H + diag(arm))^-1 (tau~ - C). Its
// prediction is accepted when the inverse-dynamics residual
// r = RNEA(q, qd, qdd_hat) + arm * qdd_hat - tau~ is small relative to tau~,
// otherwise the exact solve (ABA) is used. Written from the definitions:
//   * features: q, qd, tau~ (J each), then per joint (m, m c, I_O) with I_O
//     the rotational inertia about the link origin (xx yy zz xy xz yz);
//   * z-score normalisation of inputs and outputs with given mean/std;
//   * ELU hidden units (elu(x) = x for x > 0, exp(x) - 1 otherwise), linear
//     output layer;
//   * loss: mean squared error over the batch and outputs on normalised
//     targets;
//   * backward pass by the chain rule;
//   * Adam (Kingma & Ba, 2015) with bias correction.
// "emulate" rounds every matrix-product operand (weights and layer inputs,
// and the output gradient in the backward pass) to BF16, as the matrix cores
// consume them; otherwise everything stays FP64.
#pragma once
#include <cmath>
#include <vector>

#include "rl.hpp"

namespace ora {

struct SurrogateNet {
  int n_layers;               // number of weight layers (4: 3 hidden + output)
  std::vector<int> dims;      // n_layers + 1 sizes
  std::vector<const double*> W;  // [dims[l+1]][dims[l]] row-major
  std::vector<const double*> b;  // [dims[l+1]]
};

inline double elu(double x) { return x > 0.0 ? x : std::expm1(x); }
inline double elu_grad(double x) { return x > 0.0 ? 1.0 : std::exp(x); }
inline double maybe_bf16(double x, bool emulate) { return emulate ? round_bf16(x) : x; }

// Forward for one sample. acts[l] holds the (possibly rounded) input of layer
// l, pre[l] its pre-activation output. x is the normalised input.
inline void surrogate_forward(const SurrogateNet& net, const double* x, bool emulate,
                              std::vector<std::vector<double>>& acts, std::vector<std::vector<double>>& pre,
                              double* y) {
  acts.assign(net.n_layers, {});
  pre.assign(net.n_layers, {});
  std::vector<double> in(x, x + net.dims[0]);
  for (int l = 0; l < net.n_layers; ++l) {
    const int ni = net.dims[l], no = net.dims[l + 1];
    acts[l].resize(ni);
    for (int k = 0; k < ni; ++k) acts[l][k] = maybe_bf16(in[k], emulate);
    pre[l].assign(no, 0.0);
    for (int i = 0; i < no; ++i) {
      double s = net.b[l][i];
      for (int k = 0; k < ni; ++k) s += maybe_bf16(net.W[l][i * ni + k], emulate) * acts[l][k];
      pre[l][i] = s;
    }
    in.assign(no, 0.0);
    for (int i = 0; i < no; ++i) in[i] = (l == net.n_layers - 1) ? pre[l][i] : elu(pre[l][i]);
  }
  for (int i = 0; i < net.dims[net.n_layers]; ++i) y[i] = in[i];
}

// Backward for one sample given dL/dy; accumulates into gW, gb (same
// shapes as W, b).
inline void surrogate_backward(const SurrogateNet& net, const std::vector<std::vector<double>>& acts,
                               const std::vector<std::vector<double>>& pre, const double* dy, bool emulate,
                               std::vector<std::vector<double>>& gW, std::vector<std::vector<double>>& gb) {
  const int L = net.n_layers;
  std::vector<double> g(dy, dy + net.dims[L]);  // dL/d(pre) of the last layer
  for (int l = L - 1; l >= 0; --l) {
    const int ni = net.dims[l], no = net.dims[l + 1];
    std::vector<double> ge(no);
    for (int i = 0; i < no; ++i) ge[i] = maybe_bf16(g[i], emulate);
    for (int i = 0; i < no; ++i) {
      gb[l][i] += g[i];
      for (int k = 0; k < ni; ++k) gW[l][i * ni + k] += ge[i] * acts[l][k];
    }
    if (l == 0) break;
    std::vector<double> gin(ni, 0.0);
    for (int k = 0; k < ni; ++k) {
      double s = 0.0;
      for (int i = 0; i < no; ++i) s += maybe_bf16(net.W[l][i * ni + k], emulate) * ge[i];
      gin[k] = s * elu_grad(pre[l - 1][k]);
    }
    g.swap(gin);
  }
}

// Adam step on one parameter array (t = 1-based step count).
inline void adam_update(int n, double* w, const double* g, double* m, double* v, double lr, double beta1,
                        double beta2, double eps, int t) {
  const double c1 = 1.0 - std::pow(beta1, t), c2 = 1.0 - std::pow(beta2, t);
  for (int i = 0; i < n; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
    const double mh = m[i] / c1, vh = v[i] / c2;
    w[i] -= lr * mh / (std::sqrt(vh) + eps);
  }
}

}  // namespace ora
