// Test infrastructure: part of the FP64 CPU oracle. Only tests/, the smoke
// check and the CPU-baseline leg of the benchmark may load or run anything
// under oracle/; the product path never does.
//
// Rigid-body dynamics of a fixed-base serial chain of revolute joints, written
// from Featherstone, "Rigid Body Dynamics Algorithms" (2008):
//   * forward kinematics of the tool tip (the observation's tip position,
//     paper Sec. III "Observation Space");
//   * RNEA, inverse dynamics (Featherstone Table 5.1);
//   * CRBA, the joint-space inertia matrix (Table 6.2), plus a Cholesky solve;
//   * ABA, forward dynamics in three passes (Table 7.1) with a joint
//     "armature" term added to each D_i, which is how the implicit PD drive
//     folds into one forward-dynamics solve.
// The paper states no dynamics algorithm (its engine is a closed GPU solver,
// Sec. III "Simulation Setup"); these are the textbook definitions of the
// quantities that solver produces for a contact-free serial chain.
//
// Chain geometry convention: joint j's origin sits at offset_j in link (j-1)'s
// frame (the base frame for j = 0); link j's frame is that origin rotated by
// q_j about the unit axis_j. So the Pluecker transform from link j-1 to link j
// coordinates is X_j = rot(E_j) xlt(offset_j) with E_j = R(axis_j, q_j)^T and
// the motion subspace of joint j is S_j = (axis_j; 0) in link-j coordinates.
// Gravity enters as a fictitious base acceleration a_0 = (0; -g).
#pragma once
#include <cmath>

#include "spatial.hpp"

namespace ora {

constexpr int kMaxDof = 16;
constexpr int kMaxChains = 4;  // chains per env (multi-tool reaching)

enum { kRevolute = 0, kPrismatic = 1 };

template <class T> struct Link {
  int type;  // kRevolute or kPrismatic
  V3<T> axis, offset, com;
  T mass;
  M3<T> Ic;  // rotational inertia about the centre of mass, link axes
  SI<T> I;   // spatial inertia about the link origin, set by finalize_link
};

template <class T> struct Chain {
  int n;
  Link<T> L[kMaxDof];
  V3<T> tip;   // tool-tip point in the last link's frame
  V3<T> grav;  // gravity vector in base coordinates, e.g. (0, 0, -9.81)
};

// Joint transform X_j = X_J(q) X_T: a revolute joint rotates by q about its
// axis, a prismatic joint translates by q along it (Featherstone Table 4.1).
template <class T> inline PX<T> joint_transform(const Link<T>& l, T q) {
  PX<T> X;
  if (l.type == kPrismatic) {
    X.E = m3_identity<T>();
    X.r = l.offset + scale(l.axis, q);
  } else {
    X.E = transpose(axis_rotation(l.axis, q));
    X.r = l.offset;
  }
  return X;
}

// Motion subspace: (axis; 0) for a revolute joint, (0; axis) for a
// prismatic one (link coordinates).
template <class T> inline SV<T> motion_subspace(const Link<T>& l) {
  const V3<T> z = v3(T(0.0), T(0.0), T(0.0));
  return l.type == kPrismatic ? SV<T>{z, l.axis} : SV<T>{l.axis, z};
}

// The spatial inertia of a link is constant in link coordinates: it is formed
// once when the chain is built, not at every evaluation.
template <class T> inline void finalize_link(Link<T>& l) { l.I = rigid_inertia(l.mass, l.com, l.Ic); }
template <class T> inline const SI<T>& link_inertia(const Link<T>& l) { return l.I; }

// World pose of every link frame and the tool tip.
template <class T> struct Pose {
  M3<T> R[kMaxDof];  // orientation of link j (columns: link axes in base coords)
  V3<T> p[kMaxDof];  // origin of link j (joint j's position) in base coords
  V3<T> tip;
};

template <class T> inline void forward_kinematics(const Chain<T>& ch, const T* q, Pose<T>& out) {
  M3<T> R = m3_identity<T>();
  V3<T> p = v3(T(0.0), T(0.0), T(0.0));
  for (int j = 0; j < ch.n; ++j) {
    if (ch.L[j].type == kPrismatic) {
      p = p + mul(R, ch.L[j].offset + scale(ch.L[j].axis, q[j]));
    } else {
      p = p + mul(R, ch.L[j].offset);
      R = mul(R, axis_rotation(ch.L[j].axis, q[j]));
    }
    out.R[j] = R;
    out.p[j] = p;
  }
  out.tip = p + mul(R, ch.tip);
}

// RNEA: tau = M(q) qdd + C(q, qd) (gravity included in C).
template <class T> inline void rnea(const Chain<T>& ch, const T* q, const T* qd, const T* qdd, T* tau) {
  PX<T> X[kMaxDof];
  SV<T> f[kMaxDof];
  SV<T> v_par = sv_zero<T>();
  SV<T> a_par = {v3(T(0.0), T(0.0), T(0.0)), -ch.grav};
  for (int j = 0; j < ch.n; ++j) {
    const Link<T>& l = ch.L[j];
    X[j] = joint_transform(l, q[j]);
    SV<T> S = motion_subspace(l);
    SV<T> vJ = scale(S, qd[j]);
    SV<T> v = xform_motion(X[j], v_par) + vJ;
    SV<T> a = xform_motion(X[j], a_par) + scale(S, qdd[j]) + crm(v, vJ);
    const SI<T>& I = link_inertia(l);
    f[j] = mul(I, a) + crf(v, mul(I, v));
    v_par = v;
    a_par = a;
  }
  for (int j = ch.n - 1; j >= 0; --j) {
    SV<T> S = motion_subspace(ch.L[j]);
    tau[j] = sdot(S, f[j]);
    if (j > 0) f[j - 1] = f[j - 1] + xform_force_T(X[j], f[j]);
  }
}

// CRBA: joint-space inertia matrix H (n x n, row-major, full).
template <class T> inline void crba(const Chain<T>& ch, const T* q, T* H) {
  const int n = ch.n;
  PX<T> X[kMaxDof];
  SI<T> Ic[kMaxDof];
  for (int j = 0; j < n; ++j) {
    X[j] = joint_transform(ch.L[j], q[j]);
    Ic[j] = link_inertia(ch.L[j]);
  }
  for (int i = n - 1; i >= 0; --i) {
    if (i > 0) Ic[i - 1] = add(Ic[i - 1], congruence(X[i], Ic[i]));
    SV<T> Si = motion_subspace(ch.L[i]);
    SV<T> F = mul(Ic[i], Si);
    H[i * n + i] = sdot(Si, F);
    int j = i;
    while (j > 0) {
      F = xform_force_T(X[j], F);
      j = j - 1;
      SV<T> Sj = motion_subspace(ch.L[j]);
      H[i * n + j] = sdot(Sj, F);
      H[j * n + i] = H[i * n + j];
    }
  }
}

// Solve (A) x = b for symmetric positive-definite A (n x n) by Cholesky
// A = L L^T. Returns false if A is not positive definite.
template <class T> inline bool cholesky_solve(int n, const T* A, const T* b, T* x) {
  using std::sqrt;
  T L[kMaxDof * kMaxDof];
  for (int i = 0; i < n * n; ++i) L[i] = T(0.0);
  for (int j = 0; j < n; ++j) {
    T s = A[j * n + j];
    for (int k = 0; k < j; ++k) s = s - L[j * n + k] * L[j * n + k];
    if (!(val(s) > 0.0)) return false;
    L[j * n + j] = sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      T t = A[i * n + j];
      for (int k = 0; k < j; ++k) t = t - L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  T y[kMaxDof];
  for (int i = 0; i < n; ++i) {
    T t = b[i];
    for (int k = 0; k < i; ++k) t = t - L[i * n + k] * y[k];
    y[i] = t / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    T t = y[i];
    for (int k = i + 1; k < n; ++k) t = t - L[k * n + i] * x[k];
    x[i] = t / L[i * n + i];
  }
  return true;
}

// ABA: qdd = (H(q) + diag(arm))^{-1} (tau - C(q, qd)), in O(n).
template <class T> inline void aba(const Chain<T>& ch, const T* q, const T* qd, const T* tau, const T* arm, T* qdd) {
  const int n = ch.n;
  PX<T> X[kMaxDof];
  SV<T> S[kMaxDof], c[kMaxDof], pA[kMaxDof], U[kMaxDof];
  SI<T> IA[kMaxDof];
  T D[kMaxDof], u[kMaxDof];
  // pass 1, outward: velocities, velocity-product accelerations, bias forces
  SV<T> v_par = sv_zero<T>();
  for (int i = 0; i < n; ++i) {
    const Link<T>& l = ch.L[i];
    X[i] = joint_transform(l, q[i]);
    S[i] = motion_subspace(l);
    SV<T> vJ = scale(S[i], qd[i]);
    SV<T> v = xform_motion(X[i], v_par) + vJ;
    c[i] = crm(v, vJ);
    IA[i] = link_inertia(l);
    pA[i] = crf(v, mul(IA[i], v));
    v_par = v;
  }
  // pass 2, inward: articulated-body inertias and bias forces
  for (int i = n - 1; i >= 0; --i) {
    U[i] = mul(IA[i], S[i]);
    D[i] = sdot(S[i], U[i]) + arm[i];
    u[i] = tau[i] - sdot(S[i], pA[i]);
    if (i > 0) {
      T invD = T(1.0) / D[i];
      SV<T> Ud = scale(U[i], invD);
      // Ia = IA - U U^T / D, block by block (A and C symmetric: upper triangle)
      T ua[3] = {U[i].ang.x, U[i].ang.y, U[i].ang.z}, ul[3] = {U[i].lin.x, U[i].lin.y, U[i].lin.z};
      T da[3] = {Ud.ang.x, Ud.ang.y, Ud.ang.z}, dl[3] = {Ud.lin.x, Ud.lin.y, Ud.lin.z};
      SI<T> Ia;
      for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
          if (s >= r) {
            Ia.A.m[r][s] = IA[i].A.m[r][s] - ua[r] * da[s];
            Ia.A.m[s][r] = Ia.A.m[r][s];
            Ia.C.m[r][s] = IA[i].C.m[r][s] - ul[r] * dl[s];
            Ia.C.m[s][r] = Ia.C.m[r][s];
          }
          Ia.B.m[r][s] = IA[i].B.m[r][s] - ua[r] * dl[s];
        }
      SV<T> pa = pA[i] + mul(Ia, c[i]) + scale(U[i], u[i] * invD);
      IA[i - 1] = add(IA[i - 1], congruence(X[i], Ia));
      pA[i - 1] = pA[i - 1] + xform_force_T(X[i], pa);
    }
  }
  // pass 3, outward: accelerations
  SV<T> a_par = {v3(T(0.0), T(0.0), T(0.0)), -ch.grav};
  for (int i = 0; i < n; ++i) {
    SV<T> a1 = xform_motion(X[i], a_par) + c[i];
    qdd[i] = (u[i] - sdot(a1, U[i])) / D[i];
    a_par = a1 + scale(S[i], qdd[i]);
  }
}

}  // namespace ora
