// Test infrastructure: part of the FP64 CPU oracle. Only tests/, the smoke
// check and the CPU-baseline leg of the benchmark may load or run anything
// under oracle/; the product path never does.
//
// Spatial (6-D Pluecker) vector algebra as defined in Featherstone, "Rigid
// Body Dynamics Algorithms" (2008), ch. 2: motion vectors m = (w; v) with v
// the velocity of the body point at the frame origin, force vectors
// f = (n; f) with n the moment about the origin, and Pluecker transforms
// X = rot(E) xlt(r). Every operation is written from its 3x3-block
// definition; tests check each one against the dense 6x6 matrix it stands
// for.
#pragma once
#include <cmath>

#include "counted.hpp"

namespace ora {

template <class T> struct V3 {
  T x, y, z;
};
template <class T> inline V3<T> v3(T x, T y, T z) { return V3<T>{x, y, z}; }
template <class T> inline V3<T> operator+(const V3<T>& a, const V3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> inline V3<T> operator-(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> inline V3<T> operator-(const V3<T>& a) { return {-a.x, -a.y, -a.z}; }
template <class T> inline V3<T> scale(const V3<T>& a, T s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> inline T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> inline V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// 3x3 matrix, row-major m[row][col].
template <class T> struct M3 {
  T m[3][3];
};
template <class T> inline M3<T> m3_zero() {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = T(0.0);
  return r;
}
template <class T> inline M3<T> m3_identity() {
  M3<T> r = m3_zero<T>();
  r.m[0][0] = r.m[1][1] = r.m[2][2] = T(1.0);
  return r;
}
template <class T> inline V3<T> mul(const M3<T>& a, const V3<T>& v) {
  return {a.m[0][0] * v.x + a.m[0][1] * v.y + a.m[0][2] * v.z,
          a.m[1][0] * v.x + a.m[1][1] * v.y + a.m[1][2] * v.z,
          a.m[2][0] * v.x + a.m[2][1] * v.y + a.m[2][2] * v.z};
}
// a^T v
template <class T> inline V3<T> mulT(const M3<T>& a, const V3<T>& v) {
  return {a.m[0][0] * v.x + a.m[1][0] * v.y + a.m[2][0] * v.z,
          a.m[0][1] * v.x + a.m[1][1] * v.y + a.m[2][1] * v.z,
          a.m[0][2] * v.x + a.m[1][2] * v.y + a.m[2][2] * v.z};
}
template <class T> inline M3<T> mul(const M3<T>& a, const M3<T>& b) {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][0] * b.m[0][j] + a.m[i][1] * b.m[1][j] + a.m[i][2] * b.m[2][j];
  return r;
}
template <class T> inline M3<T> transpose(const M3<T>& a) {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[j][i];
  return r;
}
template <class T> inline M3<T> add(const M3<T>& a, const M3<T>& b) {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][j] + b.m[i][j];
  return r;
}
template <class T> inline M3<T> sub(const M3<T>& a, const M3<T>& b) {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][j] - b.m[i][j];
  return r;
}
// r x (the cross-product matrix of r): skew(r) v = r x v
template <class T> inline M3<T> skew(const V3<T>& r) {
  M3<T> s;
  s.m[0][0] = T(0.0); s.m[0][1] = -r.z;  s.m[0][2] = r.y;
  s.m[1][0] = r.z;   s.m[1][1] = T(0.0); s.m[1][2] = -r.x;
  s.m[2][0] = -r.y;  s.m[2][1] = r.x;   s.m[2][2] = T(0.0);
  return s;
}
// skew(r) * a, formed column by column as r x (column of a): 3 flops per entry.
template <class T> inline M3<T> skew_mul(const V3<T>& r, const M3<T>& a) {
  M3<T> out;
  for (int j = 0; j < 3; ++j) {
    V3<T> c = cross(r, v3(a.m[0][j], a.m[1][j], a.m[2][j]));
    out.m[0][j] = c.x; out.m[1][j] = c.y; out.m[2][j] = c.z;
  }
  return out;
}
// a * skew(r): row i of the product is row_i(a) skew(r) = row_i(a) x r.
template <class T> inline M3<T> mul_skew(const M3<T>& a, const V3<T>& r) {
  M3<T> out;
  for (int i = 0; i < 3; ++i) {
    V3<T> c = cross(v3(a.m[i][0], a.m[i][1], a.m[i][2]), r);
    out.m[i][0] = c.x; out.m[i][1] = c.y; out.m[i][2] = c.z;
  }
  return out;
}

// Spatial 6-vector: (top; bottom) = (ang; lin).
template <class T> struct SV {
  V3<T> ang, lin;
};
template <class T> inline SV<T> operator+(const SV<T>& a, const SV<T>& b) { return {a.ang + b.ang, a.lin + b.lin}; }
template <class T> inline SV<T> operator-(const SV<T>& a, const SV<T>& b) { return {a.ang - b.ang, a.lin - b.lin}; }
template <class T> inline SV<T> scale(const SV<T>& a, T s) { return {scale(a.ang, s), scale(a.lin, s)}; }
template <class T> inline SV<T> sv_zero() { return {v3(T(0.0), T(0.0), T(0.0)), v3(T(0.0), T(0.0), T(0.0))}; }
// Pairing of a motion and a force vector (m . f): power.
template <class T> inline T sdot(const SV<T>& m, const SV<T>& f) { return dot(m.ang, f.ang) + dot(m.lin, f.lin); }
// Motion cross product m1 x m2 = (w1 x w2; w1 x v2 + v1 x w2).
template <class T> inline SV<T> crm(const SV<T>& a, const SV<T>& b) {
  return {cross(a.ang, b.ang), cross(a.ang, b.lin) + cross(a.lin, b.ang)};
}
// Force cross product m x* f = (w x n + v x f; w x f).
template <class T> inline SV<T> crf(const SV<T>& m, const SV<T>& f) {
  return {cross(m.ang, f.ang) + cross(m.lin, f.lin), cross(m.ang, f.lin)};
}

// Pluecker transform B_X_A = rot(E) xlt(r): E maps A-coordinates to
// B-coordinates, r is B's origin relative to A's, in A-coordinates.
template <class T> struct PX {
  M3<T> E;
  V3<T> r;
};
// X m = (E w; E (v - r x w))
template <class T> inline SV<T> xform_motion(const PX<T>& X, const SV<T>& m) {
  return {mul(X.E, m.ang), mul(X.E, m.lin - cross(X.r, m.ang))};
}
// X^T f for a force in B-coordinates, giving A-coordinates:
// (E^T n + r x E^T f; E^T f)
template <class T> inline SV<T> xform_force_T(const PX<T>& X, const SV<T>& f) {
  V3<T> ef = mulT(X.E, f.lin);
  return {mulT(X.E, f.ang) + cross(X.r, ef), ef};
}

// Spatial inertia (motion -> force), symmetric 6x6 held as 3x3 blocks
// [[A, B], [B^T, C]]: n = A w + B v, f = B^T w + C v. A and C symmetric.
template <class T> struct SI {
  M3<T> A, B, C;
};
template <class T> inline SV<T> mul(const SI<T>& I, const SV<T>& m) {
  return {mul(I.A, m.ang) + mul(I.B, m.lin), mulT(I.B, m.ang) + mul(I.C, m.lin)};
}
template <class T> inline SI<T> add(const SI<T>& a, const SI<T>& b) { return {add(a.A, b.A), add(a.B, b.B), add(a.C, b.C)}; }

// Rigid body of mass m, centre of mass c (frame coordinates) and rotational
// inertia Ic about the centre of mass (frame axes):
// I = [[Ic + m cx cx^T, m cx], [m cx^T, m 1]]  (Featherstone eq. 2.63).
template <class T> inline SI<T> rigid_inertia(T m, const V3<T>& c, const M3<T>& Ic) {
  M3<T> cx = skew(c);
  M3<T> mcx;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) mcx.m[i][j] = m * cx.m[i][j];
  // cx cx^T = -cx cx
  M3<T> cxcxT = mul(cx, transpose(cx));
  SI<T> I;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      I.A.m[i][j] = Ic.m[i][j] + m * cxcxT.m[i][j];
      I.B.m[i][j] = mcx.m[i][j];
      I.C.m[i][j] = (i == j) ? m : T(0.0);
    }
  return I;
}

// Congruence X^T I X, the inertia I (given in B-coordinates) expressed in
// A-coordinates. First the rotation: A1 = E^T A E, B1 = E^T B E, C1 = E^T C E;
// then the translation xlt(r)^T [.] xlt(r) with xlt(r) = [[1, 0], [-rx, 1]]:
//   C2 = C1,  B2 = B1 + rx C1,  A2 = A1 + rx B1^T - B2 rx.
// A2 and C1 are symmetric; only their upper triangles are formed and then
// mirrored.
template <class T> inline M3<T> sym_congruence(const M3<T>& E, const M3<T>& S) {
  // E^T S E, upper triangle then mirror
  M3<T> SE = mul(S, E);  // full
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      r.m[i][j] = E.m[0][i] * SE.m[0][j] + E.m[1][i] * SE.m[1][j] + E.m[2][i] * SE.m[2][j];
      r.m[j][i] = r.m[i][j];
    }
  return r;
}
template <class T> inline SI<T> congruence(const PX<T>& X, const SI<T>& I) {
  M3<T> A1 = sym_congruence(X.E, I.A);
  M3<T> C1 = sym_congruence(X.E, I.C);
  M3<T> B1 = mul(transpose(X.E), mul(I.B, X.E));
  M3<T> B2 = add(B1, skew_mul(X.r, C1));
  M3<T> Y = skew_mul(X.r, transpose(B1));  // rx B1^T
  M3<T> Z = mul_skew(B2, X.r);             // B2 rx
  SI<T> out;
  out.C = C1;
  out.B = B2;
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      out.A.m[i][j] = A1.m[i][j] + Y.m[i][j] - Z.m[i][j];
      out.A.m[j][i] = out.A.m[i][j];
    }
  return out;
}

// Rotation by angle q (right hand) about the unit axis a (Rodrigues):
// R = cos q 1 + (1 - cos q) a a^T + sin q ax.
template <class T> inline M3<T> axis_rotation(const V3<T>& a, T q) {
  using std::cos;
  using std::sin;
  T c = cos(q), s = sin(q);
  T t = T(1.0) - c;
  M3<T> R;
  R.m[0][0] = c + t * a.x * a.x;     R.m[0][1] = t * a.x * a.y - s * a.z; R.m[0][2] = t * a.x * a.z + s * a.y;
  R.m[1][0] = t * a.y * a.x + s * a.z; R.m[1][1] = c + t * a.y * a.y;     R.m[1][2] = t * a.y * a.z - s * a.x;
  R.m[2][0] = t * a.z * a.x - s * a.y; R.m[2][1] = t * a.z * a.y + s * a.x; R.m[2][2] = c + t * a.z * a.z;
  return R;
}

}  // namespace ora
