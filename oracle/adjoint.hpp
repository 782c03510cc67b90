// Test infrastructure: part of the FP64 CPU oracle. Only tests/, the smoke
// check and the CPU-baseline leg of the benchmark may load or run anything
// under oracle/; the product path never does.
//
// Reverse mode (adjoint) of an open-loop rollout: the loss is the summed
// tool-tip distance to the task goal, L = sum_t |tip(q_{t+1}) - goal_t|
// (the negated path-following reward of paper Sec. IV), and the gradients
// are taken with respect to every step's action and every link's mass
// (geometry fixed: the whole spatial inertia of a link scales with its mass).
// Written from the chain rule applied to the forward definitions, with the
// full tape of substep states kept in memory (plain, no checkpointing):
//   * inverse dynamics tau = ID(q, qd, qdd) (RNEA) -> vjp_rnea: the gradient
//     of mu . ID with respect to q, qd and the masses, by reversing the
//     outward (v, a, f) and inward (F) recursions. The joint transform's
//     derivative is dX_j/dq_j = -(S_j x) X_j for both joint kinds.
//   * forward dynamics (H + diag(arm)) qdd = tau - C(q, qd): by the implicit
//     function rule, lambda = (H + diag(arm))^-1 qdd_bar, tau_bar = lambda
//     and (q, qd, m)_bar -= d(lambda . ID)/d(q, qd, m) at the solution qdd
//     (Carpentier and Mansard, RSS 2018, use the same identity).
//   * the implicit-PD torque, semi-implicit Euler and the hard stops (a
//     clamped coordinate passes no gradient; neither does a zeroed velocity).
//   * episodes that end inside the rollout restart from the reset state,
//     which depends on nothing before the reset.
#pragma once
#include <cmath>
#include <vector>

#include "chain.hpp"
#include "env.hpp"

namespace ora {

// Accumulates into gq, gqd, gm the gradients of sum_j mu_j tau_j with
// tau = ID(q, qd, qdd) (gravity included as the base acceleration).
inline void vjp_rnea(const Chain<double>& ch, const double* q, const double* qd, const double* qdd, const double* mu,
                     double* gq, double* gqd, double* gm) {
  const int n = ch.n;
  PX<double> X[kMaxDof];
  SV<double> S[kMaxDof], v[kMaxDof], f[kMaxDof], F[kMaxDof], Xa[kMaxDof], Xv[kMaxDof];
  SV<double> v_par = sv_zero<double>();
  SV<double> a_par = {v3(0.0, 0.0, 0.0), -ch.grav};
  for (int j = 0; j < n; ++j) {
    const Link<double>& l = ch.L[j];
    X[j] = joint_transform(l, q[j]);
    S[j] = motion_subspace(l);
    const SV<double> vJ = scale(S[j], qd[j]);
    Xv[j] = xform_motion(X[j], v_par);
    Xa[j] = xform_motion(X[j], a_par);
    v[j] = Xv[j] + vJ;
    const SV<double> a = Xa[j] + scale(S[j], qdd[j]) + crm(v[j], vJ);
    const SI<double>& I = link_inertia(l);
    f[j] = mul(I, a) + crf(v[j], mul(I, v[j]));
    v_par = v[j];
    a_par = a;
  }
  for (int j = n - 1; j >= 0; --j) F[j] = j == n - 1 ? f[j] : f[j] + xform_force_T(X[j + 1], F[j + 1]);
  // adjoint of the total forces (motion-like), outward: tau_j = S_j . F_j and
  // F_{j-1} = f_{j-1} + X_j^T F_j
  SV<double> Fb[kMaxDof];
  for (int j = 0; j < n; ++j) {
    Fb[j] = scale(S[j], mu[j]);
    if (j > 0) {
      const SV<double> lam = xform_motion(X[j], Fb[j - 1]);
      Fb[j] = Fb[j] + lam;
      gq[j] += sdot(lam, crf(S[j], F[j]));
    }
  }
  // adjoints of a_j and v_j, inward
  SV<double> ab_c = sv_zero<double>(), vb_c = sv_zero<double>();
  for (int j = n - 1; j >= 0; --j) {
    const SI<double>& I = link_inertia(ch.L[j]);
    const SV<double> vJ = scale(S[j], qd[j]);
    const SV<double> ab = mul(I, Fb[j]) + ab_c;
    const SV<double> vb = sv_zero<double>() - crf(Fb[j], mul(I, v[j])) - mul(I, crm(v[j], Fb[j])) + crf(vJ, ab) + vb_c;
    gq[j] += -sdot(crm(S[j], Xa[j]), ab) - sdot(crm(S[j], Xv[j]), vb);
    gqd[j] += sdot(crm(v[j], S[j]), ab) + sdot(S[j], vb);
    gm[j] += sdot(Fb[j], f[j]) / ch.L[j].mass;
    ab_c = xform_force_T(X[j], ab);
    vb_c = xform_force_T(X[j], vb);
  }
}

// lambda = (H(q) + diag(arm))^-1 b by CRBA and Cholesky.
inline void solve_inertia(const Chain<double>& ch, const double* q, const double* arm, const double* b, double* x) {
  const int n = ch.n;
  double H[kMaxDof * kMaxDof];
  crba(ch, q, H);
  for (int j = 0; j < n; ++j) H[j * n + j] += arm[j];
  cholesky_solve(n, H, b, x);
}

// Tool tip and its gradient contribution: qbar += J_tip^T e.
inline void tip_vjp(const Chain<double>& ch, const double* q, const V3<double>& e, double* qbar) {
  Pose<double> P;
  forward_kinematics(ch, q, P);
  for (int j = 0; j < ch.n; ++j) {
    const V3<double> z = mul(P.R[j], ch.L[j].axis);
    const V3<double> col = ch.L[j].type == kPrismatic ? z : cross(z, P.tip - P.p[j]);
    qbar[j] += dot(col, e);
  }
}

struct AdjointOut {
  double loss;
  std::vector<double> g_act;   // [T][n]
  double g_mass[kMaxDof];
};

// Open-loop rollout of T control steps with actions act [T][n] from
// (q, qd, progress); loss and (optionally) its gradients.
inline AdjointOut rollout_adjoint(const Chain<double>& ch, const Drive<double>& dr, double dt, int S,
                                  const TaskSpec& ts, const EnvGoal<double>& g, int T, const double* act,
                                  const double* q_in, const double* qd_in, int progress, bool want_grad) {
  const int n = ch.n;
  const double h = dt / S;
  AdjointOut out;
  out.loss = 0.0;
  out.g_act.assign((size_t)T * n, 0.0);
  for (int j = 0; j < kMaxDof; ++j) out.g_mass[j] = 0.0;
  // forward, keeping every substep's starting state
  std::vector<double> tq((size_t)T * S * n), tqd((size_t)T * S * n), qs_all((size_t)T * n);
  std::vector<V3<double>> edir(T);
  std::vector<double> qend((size_t)T * n);  // post-step state before any reset
  std::vector<uint8_t> reset(T, 0);
  double q[kMaxDof], qd[kMaxDof], arm[kMaxDof], tau[kMaxDof], qdd[kMaxDof];
  for (int j = 0; j < n; ++j) {
    q[j] = q_in[j];
    qd[j] = qd_in[j];
    arm[j] = h * dr.kd[j] + h * h * dr.kp[j];
  }
  for (int t = 0; t < T; ++t) {
    for (int j = 0; j < n; ++j) {
      const double a = act[t * n + j];
      const double ac = a > 1.0 ? 1.0 : (a < -1.0 ? -1.0 : a);
      qs_all[t * n + j] = 0.5 * (dr.hi[j] + dr.lo[j]) + 0.5 * (dr.hi[j] - dr.lo[j]) * ac;
    }
    for (int s = 0; s < S; ++s) {
      for (int j = 0; j < n; ++j) {
        tq[((size_t)t * S + s) * n + j] = q[j];
        tqd[((size_t)t * S + s) * n + j] = qd[j];
        tau[j] = dr.kp[j] * (qs_all[t * n + j] - q[j] - h * qd[j]) - dr.kd[j] * qd[j];
      }
      aba(ch, q, qd, tau, arm, qdd);
      for (int j = 0; j < n; ++j) {
        qd[j] = qd[j] + h * qdd[j];
        q[j] = q[j] + h * qd[j];
        if (q[j] > dr.hi[j]) {
          q[j] = dr.hi[j];
          if (qd[j] > 0.0) qd[j] = 0.0;
        } else if (q[j] < dr.lo[j]) {
          q[j] = dr.lo[j];
          if (qd[j] < 0.0) qd[j] = 0.0;
        }
      }
    }
    for (int j = 0; j < n; ++j) qend[(size_t)t * n + j] = q[j];
    Pose<double> P;
    forward_kinematics(ch, q, P);
    const V3<double> d = P.tip - goal_for(ts, g, progress);
    const double dist = norm3(d);
    out.loss += dist;
    edir[t] = dist > 0.0 ? scale(d, 1.0 / dist) : v3(0.0, 0.0, 0.0);
    ++progress;
    if (ts.ep_len > 0 && progress >= ts.ep_len) {
      reset[t] = 1;
      for (int j = 0; j < n; ++j) {
        q[j] = dr.q0[j];
        qd[j] = 0.0;
      }
      progress = 0;
    }
  }
  if (!want_grad) return out;
  // reverse
  double qb[kMaxDof] = {0}, qdb[kMaxDof] = {0};
  for (int t = T - 1; t >= 0; --t) {
    if (reset[t])
      for (int j = 0; j < n; ++j) qb[j] = qdb[j] = 0.0;
    tip_vjp(ch, &qend[(size_t)t * n], edir[t], qb);
    double qsb[kMaxDof] = {0};
    for (int s = S - 1; s >= 0; --s) {
      const size_t b = ((size_t)t * S + s) * n;
      double q0[kMaxDof], qd0[kMaxDof], q1[kMaxDof], qd1[kMaxDof];
      for (int j = 0; j < n; ++j) {
        q0[j] = tq[b + j];
        qd0[j] = tqd[b + j];
        tau[j] = dr.kp[j] * (qs_all[t * n + j] - q0[j] - h * qd0[j]) - dr.kd[j] * qd0[j];
      }
      aba(ch, q0, qd0, tau, arm, qdd);
      double qddb[kMaxDof], lam[kMaxDof], gq[kMaxDof] = {0}, gqd[kMaxDof] = {0}, gm[kMaxDof] = {0};
      for (int j = 0; j < n; ++j) {
        qd1[j] = qd0[j] + h * qdd[j];
        q1[j] = q0[j] + h * qd1[j];
        double qbj = qb[j], qdbj = qdb[j];
        if (q1[j] > dr.hi[j]) {
          qbj = 0.0;
          if (qd1[j] > 0.0) qdbj = 0.0;
        } else if (q1[j] < dr.lo[j]) {
          qbj = 0.0;
          if (qd1[j] < 0.0) qdbj = 0.0;
        }
        // q1 = q0 + h qd1, qd1 = qd0 + h qdd
        qdbj += h * qbj;
        qb[j] = qbj;
        qdb[j] = qdbj;
        qddb[j] = h * qdbj;
      }
      solve_inertia(ch, q0, arm, qddb, lam);
      vjp_rnea(ch, q0, qd0, qdd, lam, gq, gqd, gm);
      for (int j = 0; j < n; ++j) {
        // q0, qd0 reach q1, qd1 directly; the solve subtracts d(lam . ID)
        qb[j] = qb[j] - gq[j] - dr.kp[j] * lam[j];
        qdb[j] = qdb[j] - gqd[j] - (dr.kp[j] * h + dr.kd[j]) * lam[j];
        qsb[j] += dr.kp[j] * lam[j];
        out.g_mass[j] -= gm[j];
      }
    }
    for (int j = 0; j < n; ++j) {
      const double a = act[t * n + j];
      out.g_act[t * n + j] = (a > -1.0 && a < 1.0) ? 0.5 * (dr.hi[j] - dr.lo[j]) * qsb[j] : 0.0;
    }
  }
  return out;
}

// Scale link j's mass and inertia by s (geometry fixed).
inline void scale_link_mass(Link<double>& l, double s) {
  l.mass *= s;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) l.Ic.m[r][c] *= s;
  finalize_link(l);
}

}  // namespace ora
