// Velocity sets of the DDF-QE DVBM (App. G, Tables II and III) and the
// scaled 1-D Hermite polynomials used by the Grad expansions (App. D).
//
// Both sets are tensor products of a 1-D probabilists' Gauss-Hermite rule:
// D2Q16 = 4 x 4 points (exact to degree 7 per direction), D2Q25 = 5 x 5
// points (exact to degree 9).  Population i = a * n + b has the normalised
// velocity (xi_a, xi_b) and weight w_a w_b; the physical velocity is
// sqrt(R T_ref) times the normalised one.  Nodes are ascending.
//
// Table III prints the outer D2Q25 weight factors as 7 +- 2 sqrt(10); the
// 5-point rule needs them divided by 60 (the five weights then sum to one).
#pragma once

#include <hip/hip_runtime.h>

namespace dvbm {

template <int N1>
struct GH;

// 4-point rule: +-sqrt(3 -+ sqrt 6), weights (3 +- sqrt 6) / 12.
template <>
struct GH<4> {
  static constexpr int n = 4;
  static constexpr bool has_zero = false;
  __host__ __device__ static constexpr double xi(int a) {
    return a == 0 ? -2.3344142183389773 : a == 1 ? -0.741963784302726 : a == 2 ? 0.741963784302726
                                                                                : 2.3344142183389773;
  }
  __host__ __device__ static constexpr double w(int a) {
    return (a == 0 || a == 3) ? 0.04587585476806851 : 0.4541241452319315;
  }
};

// 5-point rule: 0, +-sqrt(5 - sqrt 10), +-sqrt(5 + sqrt 10);
// weights 8/15, (7 + 2 sqrt 10)/60, (7 - 2 sqrt 10)/60.
template <>
struct GH<5> {
  static constexpr int n = 5;
  static constexpr bool has_zero = true;
  __host__ __device__ static constexpr double xi(int a) {
    return a == 0   ? -2.8569700138728056
           : a == 1 ? -1.3556261799742657
           : a == 2 ? 0.0
           : a == 3 ? 1.3556261799742657
                    : 2.8569700138728056;
  }
  __host__ __device__ static constexpr double w(int a) {
    return (a == 0 || a == 4) ? 0.011257411327720682 : (a == 1 || a == 3) ? 0.22207592200561266 : 0.5333333333333333;
  }
};

// He_n(x) / n!  (probabilists' Hermite polynomials, App. C), n = 0..4.
__host__ __device__ constexpr double hn(int n, double x) {
  return n == 0   ? 1.0
         : n == 1 ? x
         : n == 2 ? (x * x - 1.0) / 2.0
         : n == 3 ? (x * x * x - 3.0 * x) / 6.0
                  : (x * x * x * x - 6.0 * x * x + 3.0) / 24.0;
}

__host__ __device__ constexpr double ipow(double x, int k) { return k == 0 ? 1.0 : x * ipow(x, k - 1); }

}  // namespace dvbm
