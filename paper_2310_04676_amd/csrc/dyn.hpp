// Per-lane rigid-body dynamics of a fixed-base serial chain of revolute and
// prismatic joints, for CDNA4 (gfx950): one environment per lane, the whole
// chain in VGPRs.
//
// Algorithms (Featherstone, "Rigid Body Dynamics Algorithms", 2008):
//   * ABA (Table 7.1): pass 1 outward (joint transforms, velocities,
//     velocity-product accelerations c, bias forces p = v x* I v), pass 2
//     inward (articulated inertias IA and bias forces pA; the joint's D gets
//     the drive armature added), pass 3 outward (accelerations, gravity as
//     the base acceleration a0 = (0; -g)).
//   * RNEA (Table 5.1) for inverse dynamics.
// Spatial conventions: motion (w; v), force (n; f), X_j = rot(R_j^T)
// xlt(offset_j) from link j-1 to link j coordinates. Revolute joint:
// R_j = rotation by q_j about axis_j (Rodrigues), S_j = (axis_j; 0).
// Prismatic joint (Featherstone Table 4.1): R_j = 1, the origin slides to
// offset_j + q_j axis_j, S_j = (0; axis_j). Parameter sources whose kPris is
// false compile the revolute-only code.
//
// Link inertias are rigid-body ones held as (m, h = m c, I_O): mass, first
// moment and rotational inertia about the link origin, 10 numbers; the
// articulated inertia of pass 2 is a general symmetric 6x6 held as blocks
// A (sym), B, C (sym) = 21 numbers.
#pragma once
#include <hip/hip_runtime.h>

namespace sgk {

// Parameter fields of the device parameter block [F][J][N].
enum {
  P_AX = 0, P_AY, P_AZ,          // joint axis
  P_OX, P_OY, P_OZ,              // joint origin in the parent frame
  P_M,                           // mass
  P_HX, P_HY, P_HZ,              // first moment m c
  P_IXX, P_IYY, P_IZZ, P_IXY, P_IXZ, P_IYZ,  // inertia about the link origin
  P_KP, P_KD, P_LO, P_HI,
  P_PR,                          // 1 prismatic, 0 revolute
  P_Q0,                          // reset position (not staged)
  P_NFIELDS,
  P_NSTAGE = P_Q0                // fields the kernels read per pass
};

template <typename T> struct Jp {
  T ax, ay, az, ox, oy, oz, m, hx, hy, hz, ixx, iyy, izz, ixy, ixz, iyz, kp, kd, lo, hi, pr;
};

__device__ __forceinline__ void sc(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sc(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ float rsq(float x) { return sqrtf(x); }
__device__ __forceinline__ double rsq(double x) { return sqrt(x); }
// sin and cos of a joint angle for the forward-dynamics solve: the hardware
// v_sin_f32 / v_cos_f32 (argument scaled to revolutions) in FP32, whose
// absolute error (a few 1e-7 for joint angles within a few radians) is below
// the FP32 rounding the rest of the solve accumulates; the library sincos in
// FP64.
__device__ __forceinline__ void sc_hw(float x, float* s, float* c) { *s = __sinf(x); *c = __cosf(x); }
__device__ __forceinline__ void sc_hw(double x, double* s, double* c) { sincos(x, s, c); }
// Reciprocal of an articulated inertia D > 0: the hardware v_rcp_f32 (about
// 1 ulp) in FP32, an exact division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <typename T>
__device__ __forceinline__ void load_joint(const T* __restrict__ par, int J, int N, int j, int e, Jp<T>& p) {
  const T* b = par + (size_t)j * N + e;
  const size_t fs = (size_t)J * N;
  p.ax = b[P_AX * fs]; p.ay = b[P_AY * fs]; p.az = b[P_AZ * fs];
  p.ox = b[P_OX * fs]; p.oy = b[P_OY * fs]; p.oz = b[P_OZ * fs];
  p.m = b[P_M * fs];
  p.hx = b[P_HX * fs]; p.hy = b[P_HY * fs]; p.hz = b[P_HZ * fs];
  p.ixx = b[P_IXX * fs]; p.iyy = b[P_IYY * fs]; p.izz = b[P_IZZ * fs];
  p.ixy = b[P_IXY * fs]; p.ixz = b[P_IXZ * fs]; p.iyz = b[P_IYZ * fs];
  p.kp = b[P_KP * fs]; p.kd = b[P_KD * fs]; p.lo = b[P_LO * fs]; p.hi = b[P_HI * fs];
  p.pr = b[P_PR * fs];
}

// Rotation by angle (s = sin, c = cos) about unit axis a, row-major R[9].
template <typename T>
__device__ __forceinline__ void rodrigues(const Jp<T>& p, T s, T c, T* R) {
  const T t = T(1) - c;
  const T txy = t * p.ax * p.ay, txz = t * p.ax * p.az, tyz = t * p.ay * p.az;
  R[0] = c + t * p.ax * p.ax; R[1] = txy - s * p.az;      R[2] = txz + s * p.ay;
  R[3] = txy + s * p.az;      R[4] = c + t * p.ay * p.ay; R[5] = tyz - s * p.ax;
  R[6] = txz - s * p.ay;      R[7] = tyz + s * p.ax;      R[8] = c + t * p.az * p.az;
}

// X m for X = rot(R^T) xlt(o): w' = R^T w, v' = R^T (v - o x w).
template <typename T>
__device__ __forceinline__ void xmotion(const T* R, const Jp<T>& p, const T* m, T* out) {
  const T tx = m[3] - (p.oy * m[2] - p.oz * m[1]);
  const T ty = m[4] - (p.oz * m[0] - p.ox * m[2]);
  const T tz = m[5] - (p.ox * m[1] - p.oy * m[0]);
  out[0] = R[0] * m[0] + R[3] * m[1] + R[6] * m[2];
  out[1] = R[1] * m[0] + R[4] * m[1] + R[7] * m[2];
  out[2] = R[2] * m[0] + R[5] * m[1] + R[8] * m[2];
  out[3] = R[0] * tx + R[3] * ty + R[6] * tz;
  out[4] = R[1] * tx + R[4] * ty + R[7] * tz;
  out[5] = R[2] * tx + R[5] * ty + R[8] * tz;
}

// X^T f (child -> parent): f' = R f, n' = R n + o x f'.
template <typename T>
__device__ __forceinline__ void xforce_T(const T* R, const Jp<T>& p, const T* f, T* out) {
  const T fx = R[0] * f[3] + R[1] * f[4] + R[2] * f[5];
  const T fy = R[3] * f[3] + R[4] * f[4] + R[5] * f[5];
  const T fz = R[6] * f[3] + R[7] * f[4] + R[8] * f[5];
  out[0] = R[0] * f[0] + R[1] * f[1] + R[2] * f[2] + (p.oy * fz - p.oz * fy);
  out[1] = R[3] * f[0] + R[4] * f[1] + R[5] * f[2] + (p.oz * fx - p.ox * fz);
  out[2] = R[6] * f[0] + R[7] * f[1] + R[8] * f[2] + (p.ox * fy - p.oy * fx);
  out[3] = fx; out[4] = fy; out[5] = fz;
}

// Rigid-body I v with I = [[I_O, h x], [-(h x), m 1]]: n = I_O w + h x v,
// f = m v - h x w.
template <typename T>
__device__ __forceinline__ void rigid_mul(const Jp<T>& p, const T* v, T* out) {
  out[0] = p.ixx * v[0] + p.ixy * v[1] + p.ixz * v[2] + (p.hy * v[5] - p.hz * v[4]);
  out[1] = p.ixy * v[0] + p.iyy * v[1] + p.iyz * v[2] + (p.hz * v[3] - p.hx * v[5]);
  out[2] = p.ixz * v[0] + p.iyz * v[1] + p.izz * v[2] + (p.hx * v[4] - p.hy * v[3]);
  out[3] = p.m * v[3] - (p.hy * v[2] - p.hz * v[1]);
  out[4] = p.m * v[4] - (p.hz * v[0] - p.hx * v[2]);
  out[5] = p.m * v[5] - (p.hx * v[1] - p.hy * v[0]);
}

// Symmetric 3x3 held as (xx, yy, zz, xy, xz, yz).
enum { S00 = 0, S11 = 1, S22 = 2, S01 = 3, S02 = 4, S12 = 5 };

// Articulated inertia blocks.
template <typename T> struct AI {
  T A[6];  // angular-angular, symmetric
  T B[9];  // angular-linear, row-major
  T C[6];  // linear-linear, symmetric
};

template <typename T> __device__ __forceinline__ T sym_at(const T* S, int i, int j) {
  const int k = (i == j) ? i : (i + j == 1 ? S01 : (i + j == 2 ? S02 : S12));
  return S[k];
}

// R S R^T for symmetric S (both as 6-vectors).
template <typename T> __device__ __forceinline__ void sym_rot(const T* R, const T* S, T* out) {
  T RS[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      RS[i * 3 + k] = R[i * 3 + 0] * sym_at(S, 0, k) + R[i * 3 + 1] * sym_at(S, 1, k) + R[i * 3 + 2] * sym_at(S, 2, k);
  auto e = [&](int i, int j) { return RS[i * 3 + 0] * R[j * 3 + 0] + RS[i * 3 + 1] * R[j * 3 + 1] + RS[i * 3 + 2] * R[j * 3 + 2]; };
  out[S00] = e(0, 0); out[S11] = e(1, 1); out[S22] = e(2, 2);
  out[S01] = e(0, 1); out[S02] = e(0, 2); out[S12] = e(1, 2);
}

// X^T Ia X for X = rot(R^T) xlt(o): rotate (R . R^T) then translate:
// C2 = C1, B2 = B1 + ox C1, A2 = A1 + ox B1^T - B2 ox. Accumulates into acc.
template <typename T>
__device__ __forceinline__ void congruence_acc(const T* R, const Jp<T>& p, const AI<T>& I, AI<T>& acc) {
  T A1[6], C1[6], B1[9];
  sym_rot(R, I.A, A1);
  sym_rot(R, I.C, C1);
  {
    T RB[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        RB[i * 3 + k] = R[i * 3 + 0] * I.B[0 * 3 + k] + R[i * 3 + 1] * I.B[1 * 3 + k] + R[i * 3 + 2] * I.B[2 * 3 + k];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        B1[i * 3 + j] = RB[i * 3 + 0] * R[j * 3 + 0] + RB[i * 3 + 1] * R[j * 3 + 1] + RB[i * 3 + 2] * R[j * 3 + 2];
  }
  const T o[3] = {p.ox, p.oy, p.oz};
  // B2 = B1 + o x C1 (column j: o x C1[:, j])
  T B2[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T c0 = sym_at(C1, 0, j), c1 = sym_at(C1, 1, j), c2 = sym_at(C1, 2, j);
    B2[0 * 3 + j] = B1[0 * 3 + j] + (o[1] * c2 - o[2] * c1);
    B2[1 * 3 + j] = B1[1 * 3 + j] + (o[2] * c0 - o[0] * c2);
    B2[2 * 3 + j] = B1[2 * 3 + j] + (o[0] * c1 - o[1] * c0);
  }
  // A2_ij = A1_ij + (o x B1[j, :])_i - (B2[i, :] x o)_j, i <= j
  auto Y = [&](int i, int j) {
    const T b0 = B1[j * 3 + 0], b1 = B1[j * 3 + 1], b2 = B1[j * 3 + 2];
    return i == 0 ? (o[1] * b2 - o[2] * b1) : (i == 1 ? (o[2] * b0 - o[0] * b2) : (o[0] * b1 - o[1] * b0));
  };
  auto Z = [&](int i, int j) {
    const T b0 = B2[i * 3 + 0], b1 = B2[i * 3 + 1], b2 = B2[i * 3 + 2];
    return j == 0 ? (b1 * o[2] - b2 * o[1]) : (j == 1 ? (b2 * o[0] - b0 * o[2]) : (b0 * o[1] - b1 * o[0]));
  };
  acc.A[S00] += A1[S00] + Y(0, 0) - Z(0, 0);
  acc.A[S11] += A1[S11] + Y(1, 1) - Z(1, 1);
  acc.A[S22] += A1[S22] + Y(2, 2) - Z(2, 2);
  acc.A[S01] += A1[S01] + Y(0, 1) - Z(0, 1);
  acc.A[S02] += A1[S02] + Y(0, 2) - Z(0, 2);
  acc.A[S12] += A1[S12] + Y(1, 2) - Z(1, 2);
#pragma unroll
  for (int k = 0; k < 9; ++k) acc.B[k] += B2[k];
#pragma unroll
  for (int k = 0; k < 6; ++k) acc.C[k] += C1[k];
}

// Sources of per-joint link parameters for the dynamics below. RegPar holds
// them in registers; LdsPar reads them from an LDS block [P_NSTAGE][J][64]
// on every use. LdsPar::fence() re-derives the lane offset opaquely, so the
// compiler cannot hoist the reads of one pass into registers held through
// the next: each pass reloads what it needs instead of keeping ~20 values
// per joint live across the whole solve. PR selects chains that may hold
// prismatic joints.
template <typename T, int J, bool PR = false> struct RegPar {
  static constexpr bool kPris = PR;
  Jp<T> P[J];
  __device__ __forceinline__ Jp<T> get(int j) const { return P[j]; }
  __device__ __forceinline__ void fence() {}
};

template <typename T, int J, bool PR = false> struct LdsPar {
  static constexpr bool kPris = PR;
  const T* sp;  // [P_NSTAGE][J][64]
  int lane;
  __device__ __forceinline__ void fence() { asm volatile("" : "+v"(lane)); }
  __device__ __forceinline__ T f(int field, int j) const { return sp[(field * J + j) * 64 + lane]; }
  __device__ __forceinline__ Jp<T> get(int j) const {
    Jp<T> p;
    p.ax = f(P_AX, j); p.ay = f(P_AY, j); p.az = f(P_AZ, j);
    p.ox = f(P_OX, j); p.oy = f(P_OY, j); p.oz = f(P_OZ, j);
    p.m = f(P_M, j);
    p.hx = f(P_HX, j); p.hy = f(P_HY, j); p.hz = f(P_HZ, j);
    p.ixx = f(P_IXX, j); p.iyy = f(P_IYY, j); p.izz = f(P_IZZ, j);
    p.ixy = f(P_IXY, j); p.ixz = f(P_IXZ, j); p.iyz = f(P_IYZ, j);
    p.kp = f(P_KP, j); p.kd = f(P_KD, j); p.lo = f(P_LO, j); p.hi = f(P_HI, j);
    p.pr = PR ? f(P_PR, j) : T(0);
    return p;
  }
};

// Joint kind of p under source PS. For a prismatic joint the origin is moved
// along the axis by q (the joint's rotation is the identity, taken as
// sin 0 = 0, cos 0 = 1). Returns true for a prismatic joint.
template <class PS, typename T> __device__ __forceinline__ bool slide(Jp<T>& p, T q) {
  if constexpr (PS::kPris) {
    const bool pr = p.pr != T(0);
    const T d = pr ? q : T(0);
    p.ox += d * p.ax; p.oy += d * p.ay; p.oz += d * p.az;
    return pr;
  } else {
    return false;
  }
}

// Forward dynamics for one env: qdd = (H + diag(arm))^-1 (tau - C).
// Joints j >= n are skipped. grav = base-frame gravity. Only sin/cos of each
// joint angle is kept between the passes; the joint rotation is rebuilt
// where it is needed (cheaper in registers than holding 9 values per joint).
// STATIC: qd = 0 and no gravity (qd and grav are not read), so the bias
// terms vanish and qdd = (H + diag(arm))^-1 tau.
template <typename T, int J, bool STATIC = false, class PS>
__device__ __forceinline__ void aba(PS& ps, int n, const T (&q)[J], const T (&qd)[J], const T (&tau)[J],
                                    const T (&arm)[J], const T* grav, T (&qdd)[J]) {
  T sn[J], cs[J], cj[J][6], pj[J][6], U[J][6], invD[J], uj[J];
  // pass 1
  ps.fence();
  T v[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      Jp<T> p = ps.get(j);
      const bool pr = slide<PS>(p, q[j]);
      sc(pr ? T(0) : q[j], &sn[j], &cs[j]);
      if constexpr (STATIC) {
#pragma unroll
        for (int k = 0; k < 6; ++k) cj[j][k] = pj[j][k] = T(0);
        continue;
      }
      T R[9];
      rodrigues(p, sn[j], cs[j], R);
      T vn[6];
      xmotion(R, p, v, vn);
      const T qw = pr ? T(0) : qd[j];
      const T wx = p.ax * qw, wy = p.ay * qw, wz = p.az * qw;
      vn[0] += wx; vn[1] += wy; vn[2] += wz;
      // c = v x (S qd) with S qd = (wJ; lJ): (w x wJ; v x wJ + w x lJ)
      cj[j][0] = vn[1] * wz - vn[2] * wy;
      cj[j][1] = vn[2] * wx - vn[0] * wz;
      cj[j][2] = vn[0] * wy - vn[1] * wx;
      cj[j][3] = vn[4] * wz - vn[5] * wy;
      cj[j][4] = vn[5] * wx - vn[3] * wz;
      cj[j][5] = vn[3] * wy - vn[4] * wx;
      if constexpr (PS::kPris) {
        const T qv = pr ? qd[j] : T(0);
        const T lx = p.ax * qv, ly = p.ay * qv, lz = p.az * qv;
        vn[3] += lx; vn[4] += ly; vn[5] += lz;
        cj[j][3] += vn[1] * lz - vn[2] * ly;
        cj[j][4] += vn[2] * lx - vn[0] * lz;
        cj[j][5] += vn[0] * ly - vn[1] * lx;
      }
      T Iv[6];
      rigid_mul(p, vn, Iv);
      // p = v x* (I v) = (w x n + v x f; w x f)
      pj[j][0] = (vn[1] * Iv[2] - vn[2] * Iv[1]) + (vn[4] * Iv[5] - vn[5] * Iv[4]);
      pj[j][1] = (vn[2] * Iv[0] - vn[0] * Iv[2]) + (vn[5] * Iv[3] - vn[3] * Iv[5]);
      pj[j][2] = (vn[0] * Iv[1] - vn[1] * Iv[0]) + (vn[3] * Iv[4] - vn[4] * Iv[3]);
      pj[j][3] = vn[1] * Iv[5] - vn[2] * Iv[4];
      pj[j][4] = vn[2] * Iv[3] - vn[0] * Iv[5];
      pj[j][5] = vn[0] * Iv[4] - vn[1] * Iv[3];
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] = vn[k];
    }
  }
  // pass 2
  ps.fence();
  AI<T> acc;
  T accp[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) { acc.A[k] = T(0); acc.C[k] = T(0); accp[k] = T(0); }
#pragma unroll
  for (int k = 0; k < 9; ++k) acc.B[k] = T(0);
#pragma unroll
  for (int j = J - 1; j >= 0; --j) {
    if (j < n) {
      Jp<T> p = ps.get(j);
      const bool pr = slide<PS>(p, q[j]);
      AI<T> I;
      I.A[S00] = p.ixx + acc.A[S00]; I.A[S11] = p.iyy + acc.A[S11]; I.A[S22] = p.izz + acc.A[S22];
      I.A[S01] = p.ixy + acc.A[S01]; I.A[S02] = p.ixz + acc.A[S02]; I.A[S12] = p.iyz + acc.A[S12];
      I.B[0] = acc.B[0];         I.B[1] = acc.B[1] - p.hz; I.B[2] = acc.B[2] + p.hy;
      I.B[3] = acc.B[3] + p.hz;  I.B[4] = acc.B[4];        I.B[5] = acc.B[5] - p.hx;
      I.B[6] = acc.B[6] - p.hy;  I.B[7] = acc.B[7] + p.hx; I.B[8] = acc.B[8];
      I.C[S00] = p.m + acc.C[S00]; I.C[S11] = p.m + acc.C[S11]; I.C[S22] = p.m + acc.C[S22];
      I.C[S01] = acc.C[S01];       I.C[S02] = acc.C[S02];       I.C[S12] = acc.C[S12];
      T pa[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) pa[k] = pj[j][k] + accp[k];
      if (!pr) {
        // U = IA S = (A a; B^T a)
        U[j][0] = I.A[S00] * p.ax + I.A[S01] * p.ay + I.A[S02] * p.az;
        U[j][1] = I.A[S01] * p.ax + I.A[S11] * p.ay + I.A[S12] * p.az;
        U[j][2] = I.A[S02] * p.ax + I.A[S12] * p.ay + I.A[S22] * p.az;
        U[j][3] = I.B[0] * p.ax + I.B[3] * p.ay + I.B[6] * p.az;
        U[j][4] = I.B[1] * p.ax + I.B[4] * p.ay + I.B[7] * p.az;
        U[j][5] = I.B[2] * p.ax + I.B[5] * p.ay + I.B[8] * p.az;
        invD[j] = recip(U[j][0] * p.ax + U[j][1] * p.ay + U[j][2] * p.az + arm[j]);
        uj[j] = tau[j] - (pa[0] * p.ax + pa[1] * p.ay + pa[2] * p.az);
      } else {
        // prismatic: U = IA (0; a) = (B a; C a)
        U[j][0] = I.B[0] * p.ax + I.B[1] * p.ay + I.B[2] * p.az;
        U[j][1] = I.B[3] * p.ax + I.B[4] * p.ay + I.B[5] * p.az;
        U[j][2] = I.B[6] * p.ax + I.B[7] * p.ay + I.B[8] * p.az;
        U[j][3] = I.C[S00] * p.ax + I.C[S01] * p.ay + I.C[S02] * p.az;
        U[j][4] = I.C[S01] * p.ax + I.C[S11] * p.ay + I.C[S12] * p.az;
        U[j][5] = I.C[S02] * p.ax + I.C[S12] * p.ay + I.C[S22] * p.az;
        invD[j] = recip(U[j][3] * p.ax + U[j][4] * p.ay + U[j][5] * p.az + arm[j]);
        uj[j] = tau[j] - (pa[3] * p.ax + pa[4] * p.ay + pa[5] * p.az);
      }
      if (j > 0) {
        T Ud[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) Ud[k] = U[j][k] * invD[j];
        // Ia = IA - U Ud^T
        I.A[S00] -= U[j][0] * Ud[0]; I.A[S11] -= U[j][1] * Ud[1]; I.A[S22] -= U[j][2] * Ud[2];
        I.A[S01] -= U[j][0] * Ud[1]; I.A[S02] -= U[j][0] * Ud[2]; I.A[S12] -= U[j][1] * Ud[2];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int s2 = 0; s2 < 3; ++s2) I.B[r * 3 + s2] -= U[j][r] * Ud[3 + s2];
        I.C[S00] -= U[j][3] * Ud[3]; I.C[S11] -= U[j][4] * Ud[4]; I.C[S22] -= U[j][5] * Ud[5];
        I.C[S01] -= U[j][3] * Ud[4]; I.C[S02] -= U[j][3] * Ud[5]; I.C[S12] -= U[j][4] * Ud[5];
        // pa += Ia c + U u / D (c = 0 when STATIC)
        const T* c = cj[j];
        const T uD = uj[j] * invD[j];
        T f[6];
        if constexpr (STATIC) {
#pragma unroll
          for (int k = 0; k < 6; ++k) f[k] = pa[k] + U[j][k] * uD;
        } else {
        f[0] = pa[0] + I.A[S00] * c[0] + I.A[S01] * c[1] + I.A[S02] * c[2] + I.B[0] * c[3] + I.B[1] * c[4] + I.B[2] * c[5] + U[j][0] * uD;
        f[1] = pa[1] + I.A[S01] * c[0] + I.A[S11] * c[1] + I.A[S12] * c[2] + I.B[3] * c[3] + I.B[4] * c[4] + I.B[5] * c[5] + U[j][1] * uD;
        f[2] = pa[2] + I.A[S02] * c[0] + I.A[S12] * c[1] + I.A[S22] * c[2] + I.B[6] * c[3] + I.B[7] * c[4] + I.B[8] * c[5] + U[j][2] * uD;
        f[3] = pa[3] + I.B[0] * c[0] + I.B[3] * c[1] + I.B[6] * c[2] + I.C[S00] * c[3] + I.C[S01] * c[4] + I.C[S02] * c[5] + U[j][3] * uD;
        f[4] = pa[4] + I.B[1] * c[0] + I.B[4] * c[1] + I.B[7] * c[2] + I.C[S01] * c[3] + I.C[S11] * c[4] + I.C[S12] * c[5] + U[j][4] * uD;
        f[5] = pa[5] + I.B[2] * c[0] + I.B[5] * c[1] + I.B[8] * c[2] + I.C[S02] * c[3] + I.C[S12] * c[4] + I.C[S22] * c[5] + U[j][5] * uD;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) { acc.A[k] = T(0); acc.C[k] = T(0); }
#pragma unroll
        for (int k = 0; k < 9; ++k) acc.B[k] = T(0);
        T R[9];
        rodrigues(p, sn[j], cs[j], R);
        congruence_acc(R, p, I, acc);
        xforce_T(R, p, f, accp);
      }
    }
  }
  // pass 3
  ps.fence();
  T a[6] = {T(0), T(0), T(0), STATIC ? T(0) : -grav[0], STATIC ? T(0) : -grav[1], STATIC ? T(0) : -grav[2]};
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      Jp<T> p = ps.get(j);
      const bool pr = slide<PS>(p, q[j]);
      T R[9];
      rodrigues(p, sn[j], cs[j], R);
      T an[6];
      xmotion(R, p, a, an);
#pragma unroll
      for (int k = 0; k < 6; ++k) an[k] += cj[j][k];
      T dot = U[j][0] * an[0] + U[j][1] * an[1] + U[j][2] * an[2] + U[j][3] * an[3] + U[j][4] * an[4] + U[j][5] * an[5];
      qdd[j] = (uj[j] - dot) * invD[j];
      const T qw = pr ? T(0) : qdd[j];
      an[0] += p.ax * qw; an[1] += p.ay * qw; an[2] += p.az * qw;
      if constexpr (PS::kPris) {
        const T qv = pr ? qdd[j] : T(0);
        an[3] += p.ax * qv; an[4] += p.ay * qv; an[5] += p.az * qv;
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) a[k] = an[k];
    } else {
      qdd[j] = T(0);
    }
  }
}

// Translation part of a congruence: moves the reference point of a
// symmetric 6x6 inertia I (blocks A, B, C) from the child origin to the
// parent origin, o = child origin - parent origin in the common orientation:
// C' = C, B' = B + o x C, A' = A + o x B^T - B' o x. Written into out.
template <typename T>
__device__ __forceinline__ void shift_inertia(const T* o, const AI<T>& I, AI<T>& out) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T c0 = sym_at(I.C, 0, j), c1 = sym_at(I.C, 1, j), c2 = sym_at(I.C, 2, j);
    out.B[0 * 3 + j] = I.B[0 * 3 + j] + (o[1] * c2 - o[2] * c1);
    out.B[1 * 3 + j] = I.B[1 * 3 + j] + (o[2] * c0 - o[0] * c2);
    out.B[2 * 3 + j] = I.B[2 * 3 + j] + (o[0] * c1 - o[1] * c0);
  }
  auto Y = [&](int i, int j) {
    const T b0 = I.B[j * 3 + 0], b1 = I.B[j * 3 + 1], b2 = I.B[j * 3 + 2];
    return i == 0 ? (o[1] * b2 - o[2] * b1) : (i == 1 ? (o[2] * b0 - o[0] * b2) : (o[0] * b1 - o[1] * b0));
  };
  auto Z = [&](int i, int j) {
    const T b0 = out.B[i * 3 + 0], b1 = out.B[i * 3 + 1], b2 = out.B[i * 3 + 2];
    return j == 0 ? (b1 * o[2] - b2 * o[1]) : (j == 1 ? (b2 * o[0] - b0 * o[2]) : (b0 * o[1] - b1 * o[0]));
  };
  out.A[S00] = I.A[S00] + Y(0, 0) - Z(0, 0);
  out.A[S11] = I.A[S11] + Y(1, 1) - Z(1, 1);
  out.A[S22] = I.A[S22] + Y(2, 2) - Z(2, 2);
  out.A[S01] = I.A[S01] + Y(0, 1) - Z(0, 1);
  out.A[S02] = I.A[S02] + Y(0, 2) - Z(0, 2);
  out.A[S12] = I.A[S12] + Y(1, 2) - Z(1, 2);
#pragma unroll
  for (int k = 0; k < 6; ++k) out.C[k] = I.C[k];
}

// Forward dynamics for one env, the same result as aba() computed in
// world-oriented frames placed at the joint origins (each link's spatial
// quantities are expressed at its own joint origin with the axes of the
// base frame). Pass 1 accumulates the link rotations W_j and rotates each
// link's inertia (m, m c, I_O) into the base orientation once; then passes 2
// and 3 only move reference points between neighbouring joint origins
// (translations by the joint offsets W_{j-1} o_j), so the articulated
// inertia recursion needs no rotations. Per joint the passes keep the
// base-oriented axis, offset, velocity-product acceleration c, bias force
// p and rotated link inertia; offsets stay at link scale, so no precision
// is lost to distant reference points.
//
// Pass 1 splits into a serial part per joint (p1_chain: the joint's axis
// and offset in the base orientation, the velocities carried to its origin,
// c, and the next W) and a part that needs only that joint's W, w and v
// (p1_link: the rotated inertia and the bias force), which other waves can
// take over (aba_lwa_team below).

// Pass 1, serial part for joint j: axis a and offset o in the base
// orientation (from the parent's W), the parent's velocity moved to this
// joint's origin, the joint's velocity added, c = v x (S qd), and W advanced
// to link j's orientation. Returns true for a prismatic joint.
template <class PS, typename T>
__device__ __forceinline__ bool p1_chain(Jp<T>& p, T qj, T qv, T (&W)[9], T (&w)[3], T (&vl)[3], T* a, T* o,
                                         T* cj) {
  const bool pr = slide<PS>(p, qj);
  o[0] = W[0] * p.ox + W[1] * p.oy + W[2] * p.oz;
  o[1] = W[3] * p.ox + W[4] * p.oy + W[5] * p.oz;
  o[2] = W[6] * p.ox + W[7] * p.oy + W[8] * p.oz;
  a[0] = W[0] * p.ax + W[1] * p.ay + W[2] * p.az;
  a[1] = W[3] * p.ax + W[4] * p.ay + W[5] * p.az;
  a[2] = W[6] * p.ax + W[7] * p.ay + W[8] * p.az;
  // the parent's velocity at this joint's origin
  vl[0] += w[1] * o[2] - w[2] * o[1];
  vl[1] += w[2] * o[0] - w[0] * o[2];
  vl[2] += w[0] * o[1] - w[1] * o[0];
  const T sx = a[0] * qv, sy = a[1] * qv, sz = a[2] * qv;
  if (!pr) {
    w[0] += sx; w[1] += sy; w[2] += sz;
    // c = v x (S qd), S qd = (s; 0): (w x s; vl x s)
    cj[0] = w[1] * sz - w[2] * sy;
    cj[1] = w[2] * sx - w[0] * sz;
    cj[2] = w[0] * sy - w[1] * sx;
    cj[3] = vl[1] * sz - vl[2] * sy;
    cj[4] = vl[2] * sx - vl[0] * sz;
    cj[5] = vl[0] * sy - vl[1] * sx;
    T sn, cs, R[9], Wn[9];
    sc_hw(qj, &sn, &cs);
    rodrigues(p, sn, cs, R);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        Wn[r * 3 + k] = W[r * 3 + 0] * R[0 * 3 + k] + W[r * 3 + 1] * R[1 * 3 + k] + W[r * 3 + 2] * R[2 * 3 + k];
#pragma unroll
    for (int k = 0; k < 9; ++k) W[k] = Wn[k];
  } else {
    // prismatic: S qd = (0; s), c = (0; w x s), no rotation
    vl[0] += sx; vl[1] += sy; vl[2] += sz;
    cj[0] = T(0); cj[1] = T(0); cj[2] = T(0);
    cj[3] = w[1] * sz - w[2] * sy;
    cj[4] = w[2] * sx - w[0] * sz;
    cj[5] = w[0] * sy - w[1] * sx;
  }
  return pr;
}

// Pass 1, the part that needs only link j's orientation W and velocity
// (w; vl) at its origin: the link's inertia in the base orientation
// (W I_O W^T, W h) and its bias force p = v x* (I v) with
// I v = (Iw w + h x vl; m vl - h x w).
template <typename T>
__device__ __forceinline__ void p1_link(const Jp<T>& p, const T (&W)[9], const T (&w)[3], const T (&vl)[3], T* Iw,
                                        T* hw, T* pj) {
  {
    const T S6[6] = {p.ixx, p.iyy, p.izz, p.ixy, p.ixz, p.iyz};
    sym_rot(W, S6, Iw);
    hw[0] = W[0] * p.hx + W[1] * p.hy + W[2] * p.hz;
    hw[1] = W[3] * p.hx + W[4] * p.hy + W[5] * p.hz;
    hw[2] = W[6] * p.hx + W[7] * p.hy + W[8] * p.hz;
  }
  const T* I = Iw;
  const T* h = hw;
  const T n0 = I[S00] * w[0] + I[S01] * w[1] + I[S02] * w[2] + (h[1] * vl[2] - h[2] * vl[1]);
  const T n1 = I[S01] * w[0] + I[S11] * w[1] + I[S12] * w[2] + (h[2] * vl[0] - h[0] * vl[2]);
  const T n2 = I[S02] * w[0] + I[S12] * w[1] + I[S22] * w[2] + (h[0] * vl[1] - h[1] * vl[0]);
  const T f0 = p.m * vl[0] - (h[1] * w[2] - h[2] * w[1]);
  const T f1 = p.m * vl[1] - (h[2] * w[0] - h[0] * w[2]);
  const T f2 = p.m * vl[2] - (h[0] * w[1] - h[1] * w[0]);
  pj[0] = (w[1] * n2 - w[2] * n1) + (vl[1] * f2 - vl[2] * f1);
  pj[1] = (w[2] * n0 - w[0] * n2) + (vl[2] * f0 - vl[0] * f2);
  pj[2] = (w[0] * n1 - w[1] * n0) + (vl[0] * f1 - vl[1] * f0);
  pj[3] = w[1] * f2 - w[2] * f1;
  pj[4] = w[2] * f0 - w[0] * f2;
  pj[5] = w[0] * f1 - w[1] * f0;
}

// One step of the base-oriented inward pass (pass 2) for joint j: acc and
// accp hold the articulated inertia and bias force its children hand to
// joint j's origin, and receive this joint's contribution at its parent's
// origin; U, invD and uj of joint j are kept for pass 3.
template <typename T, int J, class PS>
__device__ __forceinline__ void p2_step(PS& ps, int j, int n, const T (&tau)[J], const T (&arm)[J],
                                        const T (&aw)[J][3], const T (&ow)[J][3], const T (&cj)[J][6],
                                        const T (&pj)[J][6], const T (&Iw)[J][6], const T (&hw)[J][3], AI<T>& acc,
                                        T (&accp)[6], T (&U)[J][6], T (&invD)[J], T (&uj)[J]) {
  if (j < n) {
    T m, pr_;
    {
      const Jp<T> p = ps.get(j);
      m = p.m;
      pr_ = p.pr;
    }
    const bool pr = PS::kPris && pr_ != T(0);
    const T* h = hw[j];
    AI<T> I;
#pragma unroll
    for (int k = 0; k < 6; ++k) I.A[k] = Iw[j][k] + acc.A[k];
    I.B[0] = acc.B[0];        I.B[1] = acc.B[1] - h[2]; I.B[2] = acc.B[2] + h[1];
    I.B[3] = acc.B[3] + h[2]; I.B[4] = acc.B[4];        I.B[5] = acc.B[5] - h[0];
    I.B[6] = acc.B[6] - h[1]; I.B[7] = acc.B[7] + h[0]; I.B[8] = acc.B[8];
    I.C[S00] = m + acc.C[S00]; I.C[S11] = m + acc.C[S11]; I.C[S22] = m + acc.C[S22];
    I.C[S01] = acc.C[S01];     I.C[S02] = acc.C[S02];     I.C[S12] = acc.C[S12];
    T pa[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) pa[k] = pj[j][k] + accp[k];
    const T ax = aw[j][0], ay = aw[j][1], az = aw[j][2];
    if (!pr) {
      U[j][0] = I.A[S00] * ax + I.A[S01] * ay + I.A[S02] * az;
      U[j][1] = I.A[S01] * ax + I.A[S11] * ay + I.A[S12] * az;
      U[j][2] = I.A[S02] * ax + I.A[S12] * ay + I.A[S22] * az;
      U[j][3] = I.B[0] * ax + I.B[3] * ay + I.B[6] * az;
      U[j][4] = I.B[1] * ax + I.B[4] * ay + I.B[7] * az;
      U[j][5] = I.B[2] * ax + I.B[5] * ay + I.B[8] * az;
      invD[j] = recip(U[j][0] * ax + U[j][1] * ay + U[j][2] * az + arm[j]);
      uj[j] = tau[j] - (pa[0] * ax + pa[1] * ay + pa[2] * az);
    } else {
      U[j][0] = I.B[0] * ax + I.B[1] * ay + I.B[2] * az;
      U[j][1] = I.B[3] * ax + I.B[4] * ay + I.B[5] * az;
      U[j][2] = I.B[6] * ax + I.B[7] * ay + I.B[8] * az;
      U[j][3] = I.C[S00] * ax + I.C[S01] * ay + I.C[S02] * az;
      U[j][4] = I.C[S01] * ax + I.C[S11] * ay + I.C[S12] * az;
      U[j][5] = I.C[S02] * ax + I.C[S12] * ay + I.C[S22] * az;
      invD[j] = recip(U[j][3] * ax + U[j][4] * ay + U[j][5] * az + arm[j]);
      uj[j] = tau[j] - (pa[3] * ax + pa[4] * ay + pa[5] * az);
    }
    if (j > 0) {
      T Ud[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) Ud[k] = U[j][k] * invD[j];
      I.A[S00] -= U[j][0] * Ud[0]; I.A[S11] -= U[j][1] * Ud[1]; I.A[S22] -= U[j][2] * Ud[2];
      I.A[S01] -= U[j][0] * Ud[1]; I.A[S02] -= U[j][0] * Ud[2]; I.A[S12] -= U[j][1] * Ud[2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2) I.B[r * 3 + s2] -= U[j][r] * Ud[3 + s2];
      I.C[S00] -= U[j][3] * Ud[3]; I.C[S11] -= U[j][4] * Ud[4]; I.C[S22] -= U[j][5] * Ud[5];
      I.C[S01] -= U[j][3] * Ud[4]; I.C[S02] -= U[j][3] * Ud[5]; I.C[S12] -= U[j][4] * Ud[5];
      const T* c = cj[j];
      const T uD = uj[j] * invD[j];
      T f[6];
      f[0] = pa[0] + I.A[S00] * c[0] + I.A[S01] * c[1] + I.A[S02] * c[2] + I.B[0] * c[3] + I.B[1] * c[4] + I.B[2] * c[5] + U[j][0] * uD;
      f[1] = pa[1] + I.A[S01] * c[0] + I.A[S11] * c[1] + I.A[S12] * c[2] + I.B[3] * c[3] + I.B[4] * c[4] + I.B[5] * c[5] + U[j][1] * uD;
      f[2] = pa[2] + I.A[S02] * c[0] + I.A[S12] * c[1] + I.A[S22] * c[2] + I.B[6] * c[3] + I.B[7] * c[4] + I.B[8] * c[5] + U[j][2] * uD;
      f[3] = pa[3] + I.B[0] * c[0] + I.B[3] * c[1] + I.B[6] * c[2] + I.C[S00] * c[3] + I.C[S01] * c[4] + I.C[S02] * c[5] + U[j][3] * uD;
      f[4] = pa[4] + I.B[1] * c[0] + I.B[4] * c[1] + I.B[7] * c[2] + I.C[S01] * c[3] + I.C[S11] * c[4] + I.C[S12] * c[5] + U[j][4] * uD;
      f[5] = pa[5] + I.B[2] * c[0] + I.B[5] * c[1] + I.B[8] * c[2] + I.C[S02] * c[3] + I.C[S12] * c[4] + I.C[S22] * c[5] + U[j][5] * uD;
      // to the parent's origin: translate by o = this joint's offset
      const T* o = ow[j];
      shift_inertia(o, I, acc);
      accp[0] = f[0] + (o[1] * f[5] - o[2] * f[4]);
      accp[1] = f[1] + (o[2] * f[3] - o[0] * f[5]);
      accp[2] = f[2] + (o[0] * f[4] - o[1] * f[3]);
      accp[3] = f[3]; accp[4] = f[4]; accp[5] = f[5];
    }
  }
}

// Pass 3 (outward accelerations) from pass 2's U, invD and uj.
template <typename T, int J, class PS>
__device__ __forceinline__ void p3_pass(PS& ps, int n, const T* grav, const T (&aw)[J][3], const T (&ow)[J][3],
                                        const T (&cj)[J][6], const T (&U)[J][6], const T (&invD)[J],
                                        const T (&uj)[J], T (&qdd)[J]) {
  T a[6] = {T(0), T(0), T(0), -grav[0], -grav[1], -grav[2]};
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      const T* o = ow[j];
      T an[6];
      an[0] = a[0] + cj[j][0];
      an[1] = a[1] + cj[j][1];
      an[2] = a[2] + cj[j][2];
      an[3] = a[3] + (a[1] * o[2] - a[2] * o[1]) + cj[j][3];
      an[4] = a[4] + (a[2] * o[0] - a[0] * o[2]) + cj[j][4];
      an[5] = a[5] + (a[0] * o[1] - a[1] * o[0]) + cj[j][5];
      const T dot = U[j][0] * an[0] + U[j][1] * an[1] + U[j][2] * an[2] + U[j][3] * an[3] + U[j][4] * an[4] +
                    U[j][5] * an[5];
      qdd[j] = (uj[j] - dot) * invD[j];
      bool pr = false;
      if constexpr (PS::kPris) pr = ps.get(j).pr != T(0);
      const T qa = qdd[j];
      if (!pr) {
        an[0] += aw[j][0] * qa; an[1] += aw[j][1] * qa; an[2] += aw[j][2] * qa;
      } else {
        an[3] += aw[j][0] * qa; an[4] += aw[j][1] * qa; an[5] += aw[j][2] * qa;
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) a[k] = an[k];
    } else {
      qdd[j] = T(0);
    }
  }
}


template <typename T> __device__ __forceinline__ void ai_zero(AI<T>& acc, T (&accp)[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) { acc.A[k] = T(0); acc.C[k] = T(0); accp[k] = T(0); }
#pragma unroll
  for (int k = 0; k < 9; ++k) acc.B[k] = T(0);
}

// Passes 2 and 3 of the base-oriented solve from pass 1's per-joint axis aw,
// offset ow, c, bias force pj and rotated inertia (Iw, hw).
template <typename T, int J, class PS>
__device__ __forceinline__ void aba_lwa_io(PS& ps, int n, const T (&tau)[J], const T (&arm)[J], const T* grav,
                                           const T (&aw)[J][3], const T (&ow)[J][3], const T (&cj)[J][6],
                                           const T (&pj)[J][6], const T (&Iw)[J][6], const T (&hw)[J][3],
                                           T (&qdd)[J]) {
  T U[J][6], invD[J], uj[J];
  // pass 2
  ps.fence();
  AI<T> acc;
  T accp[6];
  ai_zero(acc, accp);
#pragma unroll
  for (int j = J - 1; j >= 0; --j) p2_step<T, J>(ps, j, n, tau, arm, aw, ow, cj, pj, Iw, hw, acc, accp, U, invD, uj);
  p3_pass<T, J>(ps, n, grav, aw, ow, cj, U, invD, uj, qdd);
}

template <typename T, int J, class PS>
__device__ __forceinline__ void aba_lwa(PS& ps, int n, const T (&q)[J], const T (&qd)[J], const T (&tau)[J],
                                        const T (&arm)[J], const T* grav, T (&qdd)[J]) {
  T aw[J][3], ow[J][3], cj[J][6], pj[J][6], Iw[J][6], hw[J][3];
  // pass 1
  ps.fence();
  {
    T W[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)};
    T w[3] = {T(0), T(0), T(0)}, vl[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (j < n) {
        Jp<T> p = ps.get(j);
        p1_chain<PS>(p, q[j], qd[j], W, w, vl, aw[j], ow[j], cj[j]);
        p1_link(p, W, w, vl, Iw[j], hw[j], pj[j]);
      }
    }
  }
  aba_lwa_io<T, J>(ps, n, tau, arm, grav, aw, ow, cj, pj, Iw, hw, qdd);
}

// Wave team: kTeam waves of one workgroup hold the same 64 envs (lane l of
// every wave is env l of the block) and share pass 1 of the base-oriented
// solve. Wave 0 owns the envs' state, runs the serial chain of pass 1 and
// passes 2 and 3. The joint-independent work of link j (p1_link: its
// inertia rotated into the base orientation and its bias force, about half
// of pass 1) is done by wave team_owner(j, J): each helper wave recomputes
// the chain up to its links from the state wave 0 publishes in LDS and
// hands back 15 numbers per link through LDS. Two workgroup barriers per
// solve: after the state is published and after the links are handed back.
// Ownership: for 7-joint chains wave 0 keeps the last link, whose inward
// step (the first of pass 2) it then runs before the second barrier while
// the helpers finish, and links 0-5 go to the helpers as {1, 4}, {2, 5},
// {0, 3}; other lengths use j mod kTeam.
// LDS: the state as [(2J+3)/4][64] float4, the links as
// [team_links(J)][4][64] float4 (Iw 0-3 | Iw 4-5, hw 0-1 | hw 2, p 0-2 |
// p 3-5, -); every lane touches only its own env's entries.
constexpr int kTeam = 4;
__host__ __device__ constexpr int team_owner(int j, int J) {
  return J == 7 ? (j == J - 1 ? 0 : 1 + (j + 2) % (kTeam - 1)) : j % kTeam;
}
// index of link j among the links the helpers hand back
__host__ __device__ constexpr int team_slot(int j, int J) { return J == 7 ? j : j - (j + kTeam - 1) / kTeam; }
__host__ __device__ constexpr int team_links(int J) { return J == 7 ? J - 1 : J - (J + kTeam - 1) / kTeam; }
__host__ __device__ constexpr int team_state_slots(int J) { return (2 * J + 3) / 4; }
__host__ __device__ constexpr size_t team_lds_bytes(int J) { return (size_t)team_links(J) * 4 * 64 * 16; }
// the last link of helper wave w (-1: none)
__host__ __device__ constexpr int team_last(int w, int J) {
  int last = -1;
  for (int j = 0; j < J; ++j)
    if (team_owner(j, J) == w) last = j;
  return last;
}

struct TeamLds {
  float4* st;  // [team_state_slots(J)][64]
  float4* lk;  // [team_links(J)][4][64]
  int wave, lane;
};

template <int J>
__device__ __forceinline__ void team_put_state(const TeamLds& t, const float (&q)[J], const float (&qd)[J]) {
  constexpr int S = team_state_slots(J);
  float v[4 * S];
#pragma unroll
  for (int k = 0; k < 4 * S; ++k) v[k] = k < J ? q[k] : (k < 2 * J ? qd[k - J] : 0.f);
#pragma unroll
  for (int s = 0; s < S; ++s) t.st[s * 64 + t.lane] = make_float4(v[4 * s], v[4 * s + 1], v[4 * s + 2], v[4 * s + 3]);
}

template <int J>
__device__ __forceinline__ void team_get_state(const TeamLds& t, float (&q)[J], float (&qd)[J]) {
  constexpr int S = team_state_slots(J);
  float v[4 * S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const float4 x = t.st[s * 64 + t.lane];
    v[4 * s] = x.x; v[4 * s + 1] = x.y; v[4 * s + 2] = x.z; v[4 * s + 3] = x.w;
  }
#pragma unroll
  for (int k = 0; k < J; ++k) { q[k] = v[k]; qd[k] = v[J + k]; }
}

__device__ __forceinline__ void team_put_link(const TeamLds& t, int slot, const float* Iw, const float* hw,
                                              const float* pj) {
  float4* d = t.lk + slot * 256 + t.lane;
  d[0] = make_float4(Iw[0], Iw[1], Iw[2], Iw[3]);
  d[64] = make_float4(Iw[4], Iw[5], hw[0], hw[1]);
  d[128] = make_float4(hw[2], pj[0], pj[1], pj[2]);
  d[192] = make_float4(pj[3], pj[4], pj[5], 0.f);
}

__device__ __forceinline__ void team_get_link(const TeamLds& t, int slot, float* Iw, float* hw, float* pj) {
  const float4* d = t.lk + slot * 256 + t.lane;
  const float4 a = d[0], b = d[64], c = d[128], e = d[192];
  Iw[0] = a.x; Iw[1] = a.y; Iw[2] = a.z; Iw[3] = a.w;
  Iw[4] = b.x; Iw[5] = b.y; hw[0] = b.z; hw[1] = b.w;
  hw[2] = c.x; pj[0] = c.y; pj[1] = c.z; pj[2] = c.w;
  pj[3] = e.x; pj[4] = e.y; pj[5] = e.z;
}

// Wave 0's start of a team solve: the state published to the helpers
// (their aba_team_help starts at this barrier). Work that pass 1 does not
// need (the drive torques) can follow it and overlap the helpers' chain.
template <int J>
__device__ __forceinline__ void team_publish(const TeamLds& t, const float (&q)[J], const float (&qd)[J]) {
  team_put_state<J>(t, q, qd);
  __syncthreads();
}

// The rest of the solve as wave 0 of a team runs it, after team_publish
// (same result as aba_lwa: every quantity is computed by the same
// expressions, only in another wave). Every wave of the workgroup must be in
// the matching aba_team_help call.
template <int J, class PS>
__device__ __forceinline__ void aba_lwa_team(PS& ps, int n, const float (&q)[J], const float (&qd)[J],
                                             const float (&tau)[J], const float (&arm)[J], const float* grav,
                                             float (&qdd)[J], const TeamLds& t) {
  float aw[J][3], ow[J][3], cj[J][6], pj[J][6], Iw[J][6], hw[J][3];
  ps.fence();
  {
    float W[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    float w[3] = {0.f, 0.f, 0.f}, vl[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (j < n) {
        Jp<float> p = ps.get(j);
        p1_chain<PS>(p, q[j], qd[j], W, w, vl, aw[j], ow[j], cj[j]);
        if (team_owner(j, J) == 0) p1_link(p, W, w, vl, Iw[j], hw[j], pj[j]);
      }
    }
  }
  float U[J][6], invD[J], uj[J];
  AI<float> acc;
  float accp[6];
  ps.fence();
  ai_zero(acc, accp);
  // the last link is wave 0's: its inward step needs nothing from the helpers
  constexpr bool kEarly = team_owner(J - 1, J) == 0;
  if constexpr (kEarly) p2_step<float, J>(ps, J - 1, n, tau, arm, aw, ow, cj, pj, Iw, hw, acc, accp, U, invD, uj);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (team_owner(j, J) != 0 && j < n) team_get_link(t, team_slot(j, J), Iw[j], hw[j], pj[j]);
#pragma unroll
  for (int j = kEarly ? J - 2 : J - 1; j >= 0; --j)
    p2_step<float, J>(ps, j, n, tau, arm, aw, ow, cj, pj, Iw, hw, acc, accp, U, invD, uj);
  p3_pass<float, J>(ps, n, grav, aw, ow, cj, U, invD, uj, qdd);
}

// A helper wave's part of one team solve (t.wave = 1 .. kTeam-1): the chain
// up to its last link from the published state, and its links handed back.
template <int J, class PS>
__device__ __forceinline__ void aba_team_help(PS& ps, int n, const TeamLds& t) {
  __syncthreads();
  float q[J], qd[J];
  team_get_state<J>(t, q, qd);
  ps.fence();
  float W[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
  float w[3] = {0.f, 0.f, 0.f}, vl[3] = {0.f, 0.f, 0.f};
  const int last = team_last(t.wave, J);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j <= last && j < n) {
      Jp<float> p = ps.get(j);
      float a[3], o[3], c[6];
      p1_chain<PS>(p, q[j], qd[j], W, w, vl, a, o, c);
      if (team_owner(j, J) != 0 && team_owner(j, J) == t.wave) {
        float Iw[6], hw[3], pj[6];
        p1_link(p, W, w, vl, Iw, hw, pj);
        team_put_link(t, team_slot(j, J), Iw, hw, pj);
      }
    }
  }
  __syncthreads();
}

// Inverse dynamics for one env: tau = H qdd + C (gravity included).
template <typename T, int J, class PS>
__device__ __forceinline__ void rnea(PS& ps, int n, const T (&q)[J], const T (&qd)[J], const T (&qdd)[J],
                                     const T* grav, T (&tau)[J]) {
  T sn[J], cs[J], f[J][6];
  T v[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  T a[6] = {T(0), T(0), T(0), -grav[0], -grav[1], -grav[2]};
  ps.fence();
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      Jp<T> p = ps.get(j);
      const bool pr = slide<PS>(p, q[j]);
      sc(pr ? T(0) : q[j], &sn[j], &cs[j]);
      T R[9];
      rodrigues(p, sn[j], cs[j], R);
      T vn[6], an[6];
      xmotion(R, p, v, vn);
      xmotion(R, p, a, an);
      const T qw = pr ? T(0) : qd[j], qaw = pr ? T(0) : qdd[j];
      const T wx = p.ax * qw, wy = p.ay * qw, wz = p.az * qw;
      vn[0] += wx; vn[1] += wy; vn[2] += wz;
      if constexpr (PS::kPris) {
        const T qv = pr ? qd[j] : T(0), qav = pr ? qdd[j] : T(0);
        const T lx = p.ax * qv, ly = p.ay * qv, lz = p.az * qv;
        vn[3] += lx; vn[4] += ly; vn[5] += lz;
        an[3] += p.ax * qav + (vn[1] * lz - vn[2] * ly);
        an[4] += p.ay * qav + (vn[2] * lx - vn[0] * lz);
        an[5] += p.az * qav + (vn[0] * ly - vn[1] * lx);
      }
      an[0] += p.ax * qaw + (vn[1] * wz - vn[2] * wy);
      an[1] += p.ay * qaw + (vn[2] * wx - vn[0] * wz);
      an[2] += p.az * qaw + (vn[0] * wy - vn[1] * wx);
      an[3] += vn[4] * wz - vn[5] * wy;
      an[4] += vn[5] * wx - vn[3] * wz;
      an[5] += vn[3] * wy - vn[4] * wx;
      T Ia[6], Iv[6];
      rigid_mul(p, an, Ia);
      rigid_mul(p, vn, Iv);
      f[j][0] = Ia[0] + (vn[1] * Iv[2] - vn[2] * Iv[1]) + (vn[4] * Iv[5] - vn[5] * Iv[4]);
      f[j][1] = Ia[1] + (vn[2] * Iv[0] - vn[0] * Iv[2]) + (vn[5] * Iv[3] - vn[3] * Iv[5]);
      f[j][2] = Ia[2] + (vn[0] * Iv[1] - vn[1] * Iv[0]) + (vn[3] * Iv[4] - vn[4] * Iv[3]);
      f[j][3] = Ia[3] + (vn[1] * Iv[5] - vn[2] * Iv[4]);
      f[j][4] = Ia[4] + (vn[2] * Iv[3] - vn[0] * Iv[5]);
      f[j][5] = Ia[5] + (vn[0] * Iv[4] - vn[1] * Iv[3]);
#pragma unroll
      for (int k = 0; k < 6; ++k) { v[k] = vn[k]; a[k] = an[k]; }
    }
  }
  ps.fence();
  T fc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int j = J - 1; j >= 0; --j) {
    if (j < n) {
      Jp<T> p = ps.get(j);
      const bool pr = slide<PS>(p, q[j]);
      T ft[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) ft[k] = f[j][k] + fc[k];
      tau[j] = pr ? p.ax * ft[3] + p.ay * ft[4] + p.az * ft[5] : p.ax * ft[0] + p.ay * ft[1] + p.az * ft[2];
      T R[9];
      rodrigues(p, sn[j], cs[j], R);
      xforce_T(R, p, ft, fc);
    } else {
      tau[j] = T(0);
    }
  }
}

// Tool-tip position: p_j = p_{j-1} + R_{j-1} o_j, R_j = R_{j-1} Rot(a_j, q_j),
// tip = p + R tip_local (prismatic: o_j + q_j a_j, no rotation).
template <typename T, int J, class PS, bool HW = false>
__device__ __forceinline__ void tip_fk(PS& ps, int n, const T (&q)[J], const T* tipl, T* out) {
  // HW: sin and cos from sc_hw (the hardware in FP32) instead of the library
  T W[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)};
  T px = T(0), py = T(0), pz = T(0);
  ps.fence();
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      Jp<T> p = ps.get(j);
      const bool pr = slide<PS>(p, q[j]);
      px += W[0] * p.ox + W[1] * p.oy + W[2] * p.oz;
      py += W[3] * p.ox + W[4] * p.oy + W[5] * p.oz;
      pz += W[6] * p.ox + W[7] * p.oy + W[8] * p.oz;
      T s, c, Rj[9], Wn[9];
      if constexpr (HW) sc_hw(pr ? T(0) : q[j], &s, &c);
      else sc(pr ? T(0) : q[j], &s, &c);
      rodrigues(p, s, c, Rj);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          Wn[r * 3 + k] = W[r * 3 + 0] * Rj[0 * 3 + k] + W[r * 3 + 1] * Rj[1 * 3 + k] + W[r * 3 + 2] * Rj[2 * 3 + k];
#pragma unroll
      for (int k = 0; k < 9; ++k) W[k] = Wn[k];
    }
  }
  out[0] = px + W[0] * tipl[0] + W[1] * tipl[1] + W[2] * tipl[2];
  out[1] = py + W[3] * tipl[0] + W[4] * tipl[1] + W[5] * tipl[2];
  out[2] = pz + W[6] * tipl[0] + W[7] * tipl[1] + W[8] * tipl[2];
}

}  // namespace sgk
