// Scalar types for the CPU oracle: plain double, forward-mode dual numbers and a
// minimal reverse-mode tape.  Test infrastructure only: nothing in the GPU
// renderer includes, links or calls this file.
#pragma once
#include <cmath>
#include <vector>

namespace orc {

// ---------------------------------------------------------------- dual numbers
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() = default;
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return {s, a.d / (2.0 * s)}; }
inline Dual exp(Dual a) { double e = std::exp(a.v); return {e, e * a.d}; }
inline Dual atan2(Dual y, Dual x) {
  double r2 = x.v * x.v + y.v * y.v;
  return {std::atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / r2};
}
inline Dual log1p(Dual a) { return {std::log1p(a.v), a.d / (1.0 + a.v)}; }
// a^p for a constant exponent p (a > 0)
inline Dual pow(Dual a, double p) { double r = std::pow(a.v, p); return {r, p * r / a.v * a.d}; }
inline double val(Dual a) { return a.v; }

// ---------------------------------------------------------------- reverse tape
struct Tape {
  struct Node { int a, b; double da, db; };
  std::vector<Node> nodes;
  void clear() { nodes.clear(); }
  int push(int a, double da, int b, double db) {
    nodes.push_back({a, b, da, db});
    return (int)nodes.size() - 1;
  }
  // adjoint sweep: adj must have nodes.size() entries, seeded by the caller
  void sweep(std::vector<double>& adj) const {
    for (int i = (int)nodes.size() - 1; i >= 0; --i) {
      const Node& n = nodes[i];
      double g = adj[i];
      if (g == 0.0) continue;
      if (n.a >= 0) adj[n.a] += n.da * g;
      if (n.b >= 0) adj[n.b] += n.db * g;
    }
  }
};
extern thread_local Tape* g_tape;

struct Var {
  double v = 0.0;
  int id = -1;  // -1: constant
  Var() = default;
  Var(double x) : v(x), id(-1) {}
  Var(double x, int i) : v(x), id(i) {}
  static Var leaf(double x) { return Var(x, g_tape->push(-1, 0.0, -1, 0.0)); }
};
inline Var mk(double v, int a, double da, int b, double db) {
  if (a < 0 && b < 0) return Var(v);
  return Var(v, g_tape->push(a, da, b, db));
}
inline Var operator+(Var a, Var b) { return mk(a.v + b.v, a.id, 1.0, b.id, 1.0); }
inline Var operator-(Var a, Var b) { return mk(a.v - b.v, a.id, 1.0, b.id, -1.0); }
inline Var operator-(Var a) { return mk(-a.v, a.id, -1.0, -1, 0.0); }
inline Var operator*(Var a, Var b) { return mk(a.v * b.v, a.id, b.v, b.id, a.v); }
inline Var operator/(Var a, Var b) {
  double q = a.v / b.v;
  return mk(q, a.id, 1.0 / b.v, b.id, -q / b.v);
}
inline Var sqrt(Var a) { double s = std::sqrt(a.v); return mk(s, a.id, 0.5 / s, -1, 0.0); }
inline Var exp(Var a) { double e = std::exp(a.v); return mk(e, a.id, e, -1, 0.0); }
inline Var atan2(Var y, Var x) {
  double r2 = x.v * x.v + y.v * y.v;
  return mk(std::atan2(y.v, x.v), y.id, x.v / r2, x.id, -y.v / r2);
}
inline Var log1p(Var a) { return mk(std::log1p(a.v), a.id, 1.0 / (1.0 + a.v), -1, 0.0); }
inline Var pow(Var a, double p) { double r = std::pow(a.v, p); return mk(r, a.id, p * r / a.v, -1, 0.0); }
inline double val(Var a) { return a.v; }

inline double val(double a) { return a; }
inline double log1p(double a) { return std::log1p(a); }
inline double pow(double a, double p) { return std::pow(a, p); }

// mixed arithmetic with plain doubles
#define ORC_MIXED(T)                                                     \
  inline T operator+(T a, double b) { return a + T(b); }                 \
  inline T operator+(double a, T b) { return T(a) + b; }                 \
  inline T operator-(T a, double b) { return a - T(b); }                 \
  inline T operator-(double a, T b) { return T(a) - b; }                 \
  inline T operator*(T a, double b) { return a * T(b); }                 \
  inline T operator*(double a, T b) { return T(a) * b; }                 \
  inline T operator/(T a, double b) { return a / T(b); }                 \
  inline T operator/(double a, T b) { return T(a) / b; }                 \
  inline T& operator+=(T& a, T b) { a = a + b; return a; }               \
  inline T& operator-=(T& a, T b) { a = a - b; return a; }               \
  inline T& operator*=(T& a, T b) { a = a * b; return a; }
ORC_MIXED(Dual)
ORC_MIXED(Var)
#undef ORC_MIXED

}  // namespace orc
