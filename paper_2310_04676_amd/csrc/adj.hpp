// Per-lane reverse mode of the chain dynamics (one environment per lane):
//   * vjp_rnea: for tau = ID(q, qd, qdd) (RNEA, gravity as the base
//     acceleration), the gradients of mu . tau with respect to q, qd and
//     each link's mass (every inertial parameter of a link scales with its
//     mass). The reverse sweeps: adjoint total forces outward
//     (Fb_j = mu_j S_j + X_j Fb_{j-1}), then adjoint accelerations and
//     velocities inward; the joint transform's derivative is
//     dX_j/dq_j = -(S_j x) X_j for revolute and prismatic joints alike.
//   * tip_vjp: qbar += J_tip^T e for the tool-tip position.
// Spatial vectors are float[6] (angular; linear) as in dyn.hpp.
#pragma once
#include "dyn.hpp"

namespace sgk {

template <typename T> __device__ __forceinline__ void v6_crm(const T* a, const T* b, T* o) {
  // a x b = (wa x wb; wa x vb + va x wb)
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
  o[3] = (a[1] * b[5] - a[2] * b[4]) + (a[4] * b[2] - a[5] * b[1]);
  o[4] = (a[2] * b[3] - a[0] * b[5]) + (a[5] * b[0] - a[3] * b[2]);
  o[5] = (a[0] * b[4] - a[1] * b[3]) + (a[3] * b[1] - a[4] * b[0]);
}
template <typename T> __device__ __forceinline__ void v6_crf(const T* m, const T* f, T* o) {
  // m x* f = (w x n + v x f; w x f)
  o[0] = (m[1] * f[2] - m[2] * f[1]) + (m[4] * f[5] - m[5] * f[4]);
  o[1] = (m[2] * f[0] - m[0] * f[2]) + (m[5] * f[3] - m[3] * f[5]);
  o[2] = (m[0] * f[1] - m[1] * f[0]) + (m[3] * f[4] - m[4] * f[3]);
  o[3] = m[1] * f[5] - m[2] * f[4];
  o[4] = m[2] * f[3] - m[0] * f[5];
  o[5] = m[0] * f[4] - m[1] * f[3];
}
template <typename T> __device__ __forceinline__ T v6_dot(const T* a, const T* b) {
  return (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) + (a[3] * b[3] + a[4] * b[4] + a[5] * b[5]);
}

// Motion subspace of joint p (after slide()): (axis; 0) or (0; axis).
template <typename T> __device__ __forceinline__ void subspace(const Jp<T>& p, bool pr, T* S) {
  S[0] = pr ? T(0) : p.ax; S[1] = pr ? T(0) : p.ay; S[2] = pr ? T(0) : p.az;
  S[3] = pr ? p.ax : T(0); S[4] = pr ? p.ay : T(0); S[5] = pr ? p.az : T(0);
}

template <typename T, int J, class PS>
__device__ __forceinline__ void vjp_rnea(PS& ps, int n, const T (&q)[J], const T (&qd)[J], const T (&qdd)[J],
                                         const T (&mu)[J], const T* grav, T (&gq)[J], T (&gqd)[J], T (&gm)[J]) {
  T sn[J], cs[J], v[J][6], a[J][6], F[J][6];
  // forward recursion: v, a, f (f held in F)
  {
    T vp[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    T ap[6] = {T(0), T(0), T(0), -grav[0], -grav[1], -grav[2]};
    ps.fence();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (j < n) {
        Jp<T> p = ps.get(j);
        const bool pr = slide<PS>(p, q[j]);
        sc(pr ? T(0) : q[j], &sn[j], &cs[j]);
        T R[9], S[6], vJ[6], c[6], Iv[6], Ia[6], fv[6];
        rodrigues(p, sn[j], cs[j], R);
        subspace(p, pr, S);
#pragma unroll
        for (int k = 0; k < 6; ++k) vJ[k] = S[k] * qd[j];
        xmotion(R, p, vp, v[j]);
        xmotion(R, p, ap, a[j]);
#pragma unroll
        for (int k = 0; k < 6; ++k) v[j][k] += vJ[k];
        v6_crm(v[j], vJ, c);
#pragma unroll
        for (int k = 0; k < 6; ++k) a[j][k] += S[k] * qdd[j] + c[k];
        rigid_mul(p, a[j], Ia);
        rigid_mul(p, v[j], Iv);
        v6_crf(v[j], Iv, fv);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          F[j][k] = Ia[k] + fv[k];
          vp[k] = v[j][k];
          ap[k] = a[j][k];
        }
      }
    }
  }
  // total forces, inward: F_{j-1} += X_j^T F_j
  ps.fence();
#pragma unroll
  for (int j = J - 1; j >= 1; --j) {
    if (j < n) {
      Jp<T> p = ps.get(j);
      slide<PS>(p, q[j]);
      T R[9], t[6];
      rodrigues(p, sn[j], cs[j], R);
      xforce_T(R, p, F[j], t);
#pragma unroll
      for (int k = 0; k < 6; ++k) F[j - 1][k] += t[k];
    }
  }
  // adjoint total forces, outward; F[j] is replaced by Fb_j once used
  ps.fence();
  {
    T prev[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (j < n) {
        Jp<T> p = ps.get(j);
        const bool pr = slide<PS>(p, q[j]);
        T R[9], S[6], lam[6], sf[6];
        rodrigues(p, sn[j], cs[j], R);
        subspace(p, pr, S);
        if (j > 0) {
          xmotion(R, p, prev, lam);
          v6_crf(S, F[j], sf);
          gq[j] += v6_dot(lam, sf);
        } else {
#pragma unroll
          for (int k = 0; k < 6; ++k) lam[k] = T(0);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          F[j][k] = S[k] * mu[j] + lam[k];
          prev[k] = F[j][k];
        }
      }
    }
  }
  // adjoint accelerations and velocities, inward
  ps.fence();
  {
    T abc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    T vbc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int j = J - 1; j >= 0; --j) {
      if (j < n) {
        Jp<T> p = ps.get(j);
        const bool pr = slide<PS>(p, q[j]);
        T R[9], S[6], vJ[6], ab[6], vb[6], Iv[6], t1[6], t2[6], x[6];
        rodrigues(p, sn[j], cs[j], R);
        subspace(p, pr, S);
#pragma unroll
        for (int k = 0; k < 6; ++k) vJ[k] = S[k] * qd[j];
        rigid_mul(p, F[j], ab);
#pragma unroll
        for (int k = 0; k < 6; ++k) ab[k] += abc[k];
        rigid_mul(p, v[j], Iv);
        v6_crf(F[j], Iv, t1);          // Fb x* (I v)
        v6_crm(v[j], F[j], x);         // v x Fb
        rigid_mul(p, x, t2);           // I (v x Fb)
        v6_crf(vJ, ab, x);             // (S qd) x* ab
#pragma unroll
        for (int k = 0; k < 6; ++k) vb[k] = -t1[k] - t2[k] + x[k] + vbc[k];
        // X_j a_{j-1} = a_j - S qdd - v_j x (S qd);  X_j v_{j-1} = v_j - S qd
        T xa[6], xv[6], c[6];
        v6_crm(v[j], vJ, c);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          xa[k] = a[j][k] - S[k] * qdd[j] - c[k];
          xv[k] = v[j][k] - vJ[k];
        }
        v6_crm(S, xa, t1);
        v6_crm(S, xv, t2);
        gq[j] += -v6_dot(t1, ab) - v6_dot(t2, vb);
        v6_crm(v[j], S, t1);
        gqd[j] += v6_dot(t1, ab) + v6_dot(S, vb);
        // link force f_j = I a_j + v_j x* (I v_j); every term scales with m
        rigid_mul(p, a[j], t1);
        v6_crf(v[j], Iv, t2);
#pragma unroll
        for (int k = 0; k < 6; ++k) t1[k] += t2[k];
        gm[j] += v6_dot(F[j], t1) / p.m;
        xforce_T(R, p, ab, abc);
        xforce_T(R, p, vb, vbc);
      }
    }
  }
}

// qbar += J_tip(q)^T e: column j is z_j x (tip - p_j) for a revolute joint
// (world axis z_j through the joint origin p_j) and z_j for a prismatic one.
template <typename T, int J, class PS>
__device__ __forceinline__ void tip_vjp(PS& ps, int n, const T (&q)[J], const T* tipl, const T* e, T (&qbar)[J]) {
  T W[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)};
  T P[3] = {T(0), T(0), T(0)};
  T z[J][3], o[J][3];
  bool isp[J];
  ps.fence();
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      Jp<T> p = ps.get(j);
      const bool pr = slide<PS>(p, q[j]);
      isp[j] = pr;
      P[0] += W[0] * p.ox + W[1] * p.oy + W[2] * p.oz;
      P[1] += W[3] * p.ox + W[4] * p.oy + W[5] * p.oz;
      P[2] += W[6] * p.ox + W[7] * p.oy + W[8] * p.oz;
      T s, c, Rj[9], Wn[9];
      sc(pr ? T(0) : q[j], &s, &c);
      rodrigues(p, s, c, Rj);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          Wn[r * 3 + k] = W[r * 3 + 0] * Rj[0 * 3 + k] + W[r * 3 + 1] * Rj[1 * 3 + k] + W[r * 3 + 2] * Rj[2 * 3 + k];
#pragma unroll
      for (int k = 0; k < 9; ++k) W[k] = Wn[k];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        z[j][r] = W[r * 3 + 0] * p.ax + W[r * 3 + 1] * p.ay + W[r * 3 + 2] * p.az;
        o[j][r] = P[r];
      }
    }
  }
  T tip[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) tip[r] = P[r] + W[r * 3 + 0] * tipl[0] + W[r * 3 + 1] * tipl[1] + W[r * 3 + 2] * tipl[2];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      const T dx = tip[0] - o[j][0], dy = tip[1] - o[j][1], dz = tip[2] - o[j][2];
      T col[3];
      if (isp[j]) {
        col[0] = z[j][0]; col[1] = z[j][1]; col[2] = z[j][2];
      } else {
        col[0] = z[j][1] * dz - z[j][2] * dy;
        col[1] = z[j][2] * dx - z[j][0] * dz;
        col[2] = z[j][0] * dy - z[j][1] * dx;
      }
      qbar[j] += col[0] * e[0] + col[1] * e[1] + col[2] * e[2];
    }
  }
}

}  // namespace sgk
