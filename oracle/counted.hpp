// Test infrastructure: part of the FP64 CPU oracle. Only tests/, the smoke
// check and the CPU-baseline leg of the benchmark may load or run anything
// under oracle/; the product path never does.
//
// Counted: a double that tallies every arithmetic operation applied to it.
// Instantiating the oracle's templated dynamics with this type yields the
// exact algorithmic operation count of the method as the oracle states it
// (adds/subs, muls, divs, square roots and transcendental calls counted
// separately). A fused multiply-add does not exist at this level: a*b+c is
// one mul plus one add, i.e. two flops, the usual convention.
#pragma once
#include <cmath>

namespace ora {

struct OpTally {
  long long add = 0, mul = 0, div = 0, sqrt = 0, trans = 0;
  long long flops() const { return add + mul + div + sqrt; }
};

inline OpTally& tally() {
  static thread_local OpTally t;
  return t;
}

struct Counted {
  double v;
  Counted() : v(0.0) {}
  Counted(double x) : v(x) {}  // NOLINT: implicit on purpose
  explicit operator double() const { return v; }
  Counted& operator+=(const Counted& o) { tally().add++; v += o.v; return *this; }
  Counted& operator-=(const Counted& o) { tally().add++; v -= o.v; return *this; }
  Counted& operator*=(const Counted& o) { tally().mul++; v *= o.v; return *this; }
  Counted& operator/=(const Counted& o) { tally().div++; v /= o.v; return *this; }
};

inline Counted operator+(Counted a, Counted b) { tally().add++; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { tally().add++; return Counted(a.v - b.v); }
inline Counted operator*(Counted a, Counted b) { tally().mul++; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { tally().div++; return Counted(a.v / b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }  // sign flip: free
inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
inline bool operator>=(Counted a, Counted b) { return a.v >= b.v; }
inline bool operator==(Counted a, Counted b) { return a.v == b.v; }
inline Counted sin(Counted a) { tally().trans++; return Counted(std::sin(a.v)); }
inline Counted cos(Counted a) { tally().trans++; return Counted(std::cos(a.v)); }
inline Counted tanh(Counted a) { tally().trans++; return Counted(std::tanh(a.v)); }
inline Counted exp(Counted a) { tally().trans++; return Counted(std::exp(a.v)); }
inline Counted log(Counted a) { tally().trans++; return Counted(std::log(a.v)); }
inline Counted sqrt(Counted a) { tally().sqrt++; return Counted(std::sqrt(a.v)); }
inline bool isfinite(Counted a) { return std::isfinite(a.v); }
inline double val(Counted a) { return a.v; }
inline double val(double a) { return a; }

}  // namespace ora
