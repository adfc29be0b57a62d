// TEST INFRASTRUCTURE — part of the CPU oracle. Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load or run anything under oracle/.
//
// Scalar types the oracle is instantiated with:
//   float, double, __float128  — the precision study of the lake-at-rest tables (Sec. 4,
//                                Tables 1-3 print single / double / quadruple errors);
//   Dual<T>                    — forward-mode tangent (exact derivatives of the fluxes, used to
//                                pin the derivative fluxes and the characteristic matrices);
//   Counted                    — a double that counts every +,-,*,/,sqrt it performs, giving the
//                                algorithmic flop count of one right-hand side.
#pragma once
#include <cmath>
#include <cstdint>
#include <limits>
#include <type_traits>
#include <quadmath.h>

namespace orc {

// ---------------------------------------------------------------- __float128 helpers
inline __float128 sqrt_(__float128 x) { return sqrtq(x); }
inline __float128 abs_(__float128 x) { return fabsq(x); }
inline double sqrt_(double x) { return std::sqrt(x); }
inline double abs_(double x) { return std::fabs(x); }
inline float sqrt_(float x) { return std::sqrt(x); }
inline float abs_(float x) { return std::fabs(x); }

template <class T> inline double to_double(const T& x) { return (double)x; }

// ---------------------------------------------------------------- forward-mode dual number
template <class T> struct Dual {
  T v, d;
  Dual() : v(0), d(0) {}
  template <class A, class = std::enable_if_t<std::is_arithmetic<A>::value>>
  Dual(A a) : v(T(a)), d(0) {}
  Dual(T a, T b) : v(a), d(b) {}
};
template <class T> inline Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> inline Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> inline Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <class T> inline Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class T> inline Dual<T> operator/(Dual<T> a, Dual<T> b) {
  T q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class T> inline Dual<T>& operator+=(Dual<T>& a, Dual<T> b) { a = a + b; return a; }
template <class T> inline Dual<T>& operator-=(Dual<T>& a, Dual<T> b) { a = a - b; return a; }
template <class T> inline bool operator<(Dual<T> a, Dual<T> b) { return a.v < b.v; }
template <class T> inline bool operator>(Dual<T> a, Dual<T> b) { return a.v > b.v; }
template <class T> inline bool operator<=(Dual<T> a, Dual<T> b) { return a.v <= b.v; }
template <class T> inline Dual<T> sqrt_(Dual<T> a) {
  T s = sqrt_(a.v);
  return {s, a.d / (T(2) * s)};
}
template <class T> inline Dual<T> abs_(Dual<T> a) { return a.v < T(0) ? -a : a; }
template <class T> inline double to_double(const Dual<T>& x) { return to_double(x.v); }

// ---------------------------------------------------------------- operation-counting double
struct Counted {
  double v;
  static inline long long n_add = 0, n_mul = 0, n_div = 0, n_sqrt = 0, n_cmp = 0;
  Counted() : v(0) {}
  template <class A, class = std::enable_if_t<std::is_arithmetic<A>::value>>
  Counted(A a) : v(double(a)) {}
  static void reset() { n_add = n_mul = n_div = n_sqrt = n_cmp = 0; }
};
inline Counted mk(double x) { Counted c; c.v = x; return c; }
inline Counted operator+(Counted a, Counted b) { ++Counted::n_add; return mk(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { ++Counted::n_add; return mk(a.v - b.v); }
inline Counted operator-(Counted a) { return mk(-a.v); }
inline Counted operator*(Counted a, Counted b) { ++Counted::n_mul; return mk(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { ++Counted::n_div; return mk(a.v / b.v); }
inline Counted& operator+=(Counted& a, Counted b) { a = a + b; return a; }
inline Counted& operator-=(Counted& a, Counted b) { a = a - b; return a; }
inline bool operator<(Counted a, Counted b) { ++Counted::n_cmp; return a.v < b.v; }
inline bool operator>(Counted a, Counted b) { ++Counted::n_cmp; return a.v > b.v; }
inline bool operator<=(Counted a, Counted b) { ++Counted::n_cmp; return a.v <= b.v; }
inline Counted sqrt_(Counted a) { ++Counted::n_sqrt; return mk(std::sqrt(a.v)); }
inline Counted abs_(Counted a) { return mk(std::fabs(a.v)); }
inline double to_double(const Counted& x) { return x.v; }

template <class T> inline T max_(T a, T b) { return (a < b) ? b : a; }
template <class T> inline T sq(T a) { return a * a; }

// a quiet NaN for poisoning ghost corners the cross-shaped stencils never read
template <class T> inline T poison() { return T(0); }
template <> inline float poison<float>() { return std::numeric_limits<float>::quiet_NaN(); }
template <> inline double poison<double>() { return std::numeric_limits<double>::quiet_NaN(); }
template <> inline __float128 poison<__float128>() { return nanq(""); }

// the counted type and duals run single-threaded (static counters, no parallel benefit)
template <class T> struct parallel_ok : std::false_type {};
template <> struct parallel_ok<float> : std::true_type {};
template <> struct parallel_ok<double> : std::true_type {};
template <> struct parallel_ok<__float128> : std::true_type {};

}  // namespace orc
