// Automatic-differentiation scalars for the FP64 oracle.
//
// TEST INFRASTRUCTURE ONLY: nothing outside tests/, the smoke check and the
// CPU-baseline leg of the benchmark may use anything under oracle/.
//
// Two scalar types stand in for double in the templated oracle code:
//   Dual<T, N>  forward mode with N tangent directions (nestable: the
//               transport Jacobian of a step is taken with Dual<T, 6> for
//               any T, including another Dual or a tape variable);
//   Rv          reverse mode: every operation is recorded on a tape and a
//               backward sweep gives the adjoint of one output.
// val(x) returns the plain double value of any of them; branches in the
// oracle decide on val() only.
#pragma once

#include <cmath>
#include <vector>

namespace kfo {

inline double val(double x) { return x; }

template <class T, int N>
struct Dual {
  T v;
  T d[N];
  Dual() : v(0.0) {
    for (int i = 0; i < N; ++i) d[i] = T(0.0);
  }
  Dual(double c) : v(c) {  // NOLINT: implicit constants
    for (int i = 0; i < N; ++i) d[i] = T(0.0);
  }
  static Dual make(const T& value, int dir) {
    Dual r;
    r.v = value;
    if (dir >= 0) r.d[dir] = T(1.0);
    return r;
  }
};

template <class T, int N>
inline double val(const Dual<T, N>& x) { return val(x.v); }

// ---- Dual arithmetic (chain rule written out for each operation)
template <class T, int N>
inline Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r;
  r.v = a.v + b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <class T, int N>
inline Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r;
  r.v = a.v - b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <class T, int N>
inline Dual<T, N> operator-(const Dual<T, N>& a) {
  Dual<T, N> r;
  r.v = -a.v;
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <class T, int N>
inline Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r;
  r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <class T, int N>
inline Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r;
  r.v = a.v / b.v;
  T inv = T(1.0) / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
  return r;
}
template <class T, int N>
inline Dual<T, N> operator+(const Dual<T, N>& a, double b) { return a + Dual<T, N>(b); }
template <class T, int N>
inline Dual<T, N> operator+(double a, const Dual<T, N>& b) { return Dual<T, N>(a) + b; }
template <class T, int N>
inline Dual<T, N> operator-(const Dual<T, N>& a, double b) { return a - Dual<T, N>(b); }
template <class T, int N>
inline Dual<T, N> operator-(double a, const Dual<T, N>& b) { return Dual<T, N>(a) - b; }
template <class T, int N>
inline Dual<T, N> operator*(const Dual<T, N>& a, double b) {
  Dual<T, N> r;
  r.v = a.v * b;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <class T, int N>
inline Dual<T, N> operator*(double a, const Dual<T, N>& b) { return b * a; }
template <class T, int N>
inline Dual<T, N> operator/(const Dual<T, N>& a, double b) { return a * (1.0 / b); }
template <class T, int N>
inline Dual<T, N> operator/(double a, const Dual<T, N>& b) { return Dual<T, N>(a) / b; }
template <class T, int N>
inline Dual<T, N>& operator+=(Dual<T, N>& a, const Dual<T, N>& b) { return a = a + b; }
template <class T, int N>
inline Dual<T, N>& operator-=(Dual<T, N>& a, const Dual<T, N>& b) { return a = a - b; }
template <class T, int N>
inline Dual<T, N>& operator*=(Dual<T, N>& a, const Dual<T, N>& b) { return a = a * b; }

// unary function with value f and derivative df (both of type T)
template <class T, int N>
inline Dual<T, N> chain(const Dual<T, N>& a, const T& f, const T& df) {
  Dual<T, N> r;
  r.v = f;
  for (int i = 0; i < N; ++i) r.d[i] = df * a.d[i];
  return r;
}
template <class T, int N>
inline Dual<T, N> sin(const Dual<T, N>& a) { using std::cos; using std::sin; return chain(a, sin(a.v), cos(a.v)); }
template <class T, int N>
inline Dual<T, N> cos(const Dual<T, N>& a) { using std::cos; using std::sin; return chain(a, cos(a.v), -sin(a.v)); }
template <class T, int N>
inline Dual<T, N> sqrt(const Dual<T, N>& a) {
  using std::sqrt;
  T s = sqrt(a.v);
  return chain(a, s, T(0.5) / s);
}
template <class T, int N>
inline Dual<T, N> log(const Dual<T, N>& a) { using std::log; return chain(a, log(a.v), T(1.0) / a.v); }
template <class T, int N>
inline Dual<T, N> fabs(const Dual<T, N>& a) { return val(a) < 0.0 ? -a : a; }
template <class T, int N>
inline Dual<T, N> asin(const Dual<T, N>& a) {
  using std::asin; using std::sqrt;
  return chain(a, asin(a.v), T(1.0) / sqrt(T(1.0) - a.v * a.v));
}
template <class T, int N>
inline Dual<T, N> atan2(const Dual<T, N>& y, const Dual<T, N>& x) {
  using std::atan2;
  Dual<T, N> r;
  r.v = atan2(y.v, x.v);
  T den = T(1.0) / (x.v * x.v + y.v * y.v);
  for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) * den;
  return r;
}

// ---- Reverse mode: a global tape of nodes with up to two parents.
struct Tape {
  std::vector<int> pa, pb;
  std::vector<double> da, db;
  void clear() { pa.clear(); pb.clear(); da.clear(); db.clear(); }
  int push(int a, double dA, int b, double dB) {
    pa.push_back(a); da.push_back(dA);
    pb.push_back(b); db.push_back(dB);
    return static_cast<int>(pa.size()) - 1;
  }
  // adjoints of every node given d(out)/d(out) = 1
  std::vector<double> backward(int out) const {
    std::vector<double> adj(pa.size(), 0.0);
    if (out < 0) return adj;
    adj[out] = 1.0;
    for (int i = out; i >= 0; --i) {
      double g = adj[i];
      if (g == 0.0) continue;
      if (pa[i] >= 0) adj[pa[i]] += g * da[i];
      if (pb[i] >= 0) adj[pb[i]] += g * db[i];
    }
    return adj;
  }
};

Tape& tape();

struct Rv {
  double v;
  int id;  // -1: constant
  Rv() : v(0.0), id(-1) {}
  Rv(double c) : v(c), id(-1) {}  // NOLINT
  static Rv input(double x) {
    Rv r;
    r.v = x;
    r.id = tape().push(-1, 0.0, -1, 0.0);
    return r;
  }
};
inline double val(const Rv& x) { return x.v; }

inline Rv rv_node(double v, const Rv& a, double dA, const Rv& b, double dB) {
  Rv r;
  r.v = v;
  if (a.id < 0 && b.id < 0) return r;
  r.id = tape().push(a.id, dA, b.id, dB);
  return r;
}
inline Rv operator+(const Rv& a, const Rv& b) { return rv_node(a.v + b.v, a, 1.0, b, 1.0); }
inline Rv operator-(const Rv& a, const Rv& b) { return rv_node(a.v - b.v, a, 1.0, b, -1.0); }
inline Rv operator-(const Rv& a) { return rv_node(-a.v, a, -1.0, Rv(), 0.0); }
inline Rv operator*(const Rv& a, const Rv& b) { return rv_node(a.v * b.v, a, b.v, b, a.v); }
inline Rv operator/(const Rv& a, const Rv& b) {
  double q = a.v / b.v;
  return rv_node(q, a, 1.0 / b.v, b, -q / b.v);
}
inline Rv operator+(const Rv& a, double b) { return a + Rv(b); }
inline Rv operator+(double a, const Rv& b) { return Rv(a) + b; }
inline Rv operator-(const Rv& a, double b) { return a - Rv(b); }
inline Rv operator-(double a, const Rv& b) { return Rv(a) - b; }
inline Rv operator*(const Rv& a, double b) { return a * Rv(b); }
inline Rv operator*(double a, const Rv& b) { return Rv(a) * b; }
inline Rv operator/(const Rv& a, double b) { return a / Rv(b); }
inline Rv operator/(double a, const Rv& b) { return Rv(a) / b; }
inline Rv& operator+=(Rv& a, const Rv& b) { return a = a + b; }
inline Rv& operator-=(Rv& a, const Rv& b) { return a = a - b; }
inline Rv& operator*=(Rv& a, const Rv& b) { return a = a * b; }
inline Rv sin(const Rv& a) { return rv_node(std::sin(a.v), a, std::cos(a.v), Rv(), 0.0); }
inline Rv cos(const Rv& a) { return rv_node(std::cos(a.v), a, -std::sin(a.v), Rv(), 0.0); }
inline Rv sqrt(const Rv& a) {
  double s = std::sqrt(a.v);
  return rv_node(s, a, 0.5 / s, Rv(), 0.0);
}
inline Rv log(const Rv& a) { return rv_node(std::log(a.v), a, 1.0 / a.v, Rv(), 0.0); }
inline Rv fabs(const Rv& a) { return a.v < 0.0 ? -a : a; }
inline Rv asin(const Rv& a) {
  return rv_node(std::asin(a.v), a, 1.0 / std::sqrt(1.0 - a.v * a.v), Rv(), 0.0);
}
inline Rv atan2(const Rv& y, const Rv& x) {
  double den = 1.0 / (x.v * x.v + y.v * y.v);
  return rv_node(std::atan2(y.v, x.v), y, x.v * den, x, -y.v * den);
}

}  // namespace kfo
