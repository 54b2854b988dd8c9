// Per-node arithmetic of the DDF-QE DVBM update (device code).
//
// Moments, equilibrium and quasi-equilibrium Hermite coefficients, the
// combined two-time relaxation and the limited NND face differences.  The
// 2-D tensors of the paper are handled through the tensor-product structure
// of the velocity sets: every Hermite tensor component H_(p,q) factors into
// He_p(xi_x) He_q(xi_y), so moments and Grad expansions are computed as a
// row pass followed by a column pass over the 1-D nodes, folding the +-xi
// node pairs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"

namespace dvbm {

enum { PR_UNIT = 0, PR_LOW = 1, PR_HIGH = 2 };
enum { BC_PERIODIC = 0, BC_ZERO_GRADIENT = 1, BC_WALL = 2 };

template <int SPLIT>
struct Set {
  static constexpr int N1 = SPLIT == 1 ? 4 : 5;  // 1-D points (App. G)
  static constexpr int Q = N1 * N1;
  static constexpr int NF = SPLIT == 1 ? 3 : 4;  // Grad order of f (Sec. II D 3)
  static constexpr int NG = 2;                   // Grad order of g
};

// Kernel constants (all physical input scaled once on the host).
struct KParams {
  int nx, ny;
  int64_t pitch;         // elements per row of one population plane (nx rounded up to 64)
  int64_t srow, sdist;   // population buffers: elements per row of one distribution (Q pitch)
                         // and per distribution (ny srow)
  double c2;             // R T_ref: square of the lattice velocity scale
  double R, Cv, inv_Cv;
  double kx, ky;         // dt sqrt(R T_ref) / dx, dt sqrt(R T_ref) / dy
  double om_scale;       // CONST_MU: omega_nu = om_scale * p ; CONST_TAU: omega_nu = om_scale
  int const_mu;
  double Pr;
  double beta2;          // 2 beta
  double gr0, gr1;       // rest g per weight: gr0 + gr1 (|xi|^2 - 2)
  double wall_T[2];      // no-slip walls in y (below row 0, above row ny-1): temperature
  double wall_ux[2];     // and x velocity of each wall (physical units)
};

// Element index of population i of distribution d (0: f, 1: g) at cell (x, y)
// in a population buffer.  Buffers are [2][ny][Q][pitch]: a row of one
// distribution holds its Q planes side by side, so the rows a workgroup
// advances together are one contiguous span per distribution.
__host__ __device__ inline int64_t sidx(const KParams& kp, int d, int i, int y, int x) {
  return int64_t(d) * kp.sdist + int64_t(y) * kp.srow + int64_t(i) * kp.pitch + x;
}

// ------------------------------------------------------------ storage formats
// enc: a value computed in the format's arithmetic C -> stored value (the
// value formats); enc_dev: a deviation in units of w, computed in C -> stored
// value (the deviation formats); enc64: a float64 population X of weight w and
// rest value r (per weight) -> stored value, with the deviation X / w - r
// formed in float64 and rounded once to the stored type (initialisation,
// loading, wall ghost rows).
struct StoreF64 {
  using T = double;
  using C = double;
  static constexpr bool dev = false;
  __device__ static C raw(T v) { return v; }
  __device__ static T enc(C x, C /*winv*/, C /*r*/) { return x; }
  __device__ static T enc64(double x, double /*w*/, double /*r*/) { return x; }
};

struct StoreF32 {
  using T = float;
  using C = float;
  static constexpr bool dev = false;
  __device__ static C raw(T v) { return v; }
  __device__ static T enc(C x, C, C) { return x; }
  __device__ static T enc64(double x, double, double) { return float(x); }
};

// bfloat16 deviation (X - X_ref) / w, round to nearest even.
struct StoreBF16 {
  using T = uint16_t;
  using C = float;
  static constexpr bool dev = true;
  __device__ static C raw(T v) { return __uint_as_float(uint32_t(v) << 16); }
  __device__ static T enc_dev(C d) {  // a deviation already in units of w; round to nearest even
    return __builtin_bit_cast(T, __bf16(d));
  }
  __device__ static T enc64(double x, double w, double r) { return __builtin_bit_cast(T, __bf16(x / w - r)); }
};

// IEEE half deviation (X - X_ref) / w, round to nearest even.
struct StoreF16 {
  using T = _Float16;
  using C = float;
  static constexpr bool dev = true;
  __device__ static C raw(T v) { return float(v); }
  __device__ static T enc_dev(C d) { return T(d); }  // a deviation already in units of w
  __device__ static T enc64(double x, double w, double r) { return T(x / w - r); }
};

// float32 deviation (X - X_ref) / w: float32's bytes, with the roundings of
// a value of the deviation's size rather than of X's.
struct StoreF32Dev {
  using T = float;
  using C = float;
  static constexpr bool dev = true;
  __device__ static C raw(T v) { return v; }
  __device__ static T enc_dev(C d) { return d; }  // a deviation already in units of w
  __device__ static T enc64(double x, double w, double r) { return float(x / w - r); }
};

// ------------------------------------------------------------ small helpers
__device__ inline double med3(double a, double b, double c) { return fmax(fmin(a, b), fmin(fmax(a, b), c)); }
__device__ inline float med3(float a, float b, float c) { return __builtin_amdgcn_fmed3f(a, b, c); }

// 4 (b/2) phi(a, b) of the generalised van Leer limiter (Sec. III A 2) in the
// division-free form  2 minmod(beta a, (a + b)/2, beta b);  beta2 = 2 beta.
template <class R>
__device__ inline R lim4(R a, R b, R beta2) {
  return med3(med3(beta2 * a, beta2 * b, R(0)), a + b, R(0));
}

// X_{c+1/2} - X_{c-1/2} of the NND reconstruction for a positive velocity
// component; m2, m1, c0, p1 are the values at c-2 .. c+1:
//   (c0 + L(d1, d2)) - (m1 + L(d0, d1)) = d1 + (L(d1, d2) - L(d0, d1)).
template <class R>
__device__ inline R dface_pos(R m2, R m1, R c0, R p1, R beta2) {
  const R d0 = m1 - m2, d1 = c0 - m1, d2 = p1 - c0;
  return d1 + R(0.25) * (lim4(d1, d2, beta2) - lim4(d0, d1, beta2));
}

// The same for a negative velocity component; m1, c0, p1, p2 at c-1 .. c+2:
//   (p1 + L(p1 - p2, c0 - p1)) - (c0 + L(c0 - p1, m1 - c0)).
template <class R>
__device__ inline R dface_neg(R m1, R c0, R p1, R p2, R beta2) {
  const R e0 = c0 - p1, e1 = p1 - p2, em = m1 - c0;
  return R(0.25) * (lim4(e1, e0, beta2) - lim4(e0, em, beta2)) - e0;
}

// Sums over the 1-D nodes of v, xi v, xi^2 v, xi^3 v, folding +-xi pairs.
template <int N1, class V>
__device__ inline void pair_sums(const V* v, double& s0, double& s1, double& s2, double& s3) {
  using L = GH<N1>;
  constexpr int H = N1 / 2;
  s0 = L::has_zero ? double(v[H]) : 0.0;
  s1 = s2 = s3 = 0.0;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const int pk = N1 - 1 - k;
    const double x = L::xi(pk);
    const double e = double(v[pk]) + double(v[k]);
    const double o = double(v[pk]) - double(v[k]);
    s0 += e;
    s1 += x * o;
    s2 += (x * x) * e;
    s3 += (x * x * x) * o;
  }
}

// Raw moments in normalised velocity units (v = sqrt(R T_ref) xi).
template <class V>
struct MomentsT {
  V rho, jx, jy, pxx, pxy, pyy, qxxx, qxxy, qxyy, qyyy;  // f: orders 0..3
  V g0, qgx, qgy;                                         // g: orders 0..1
};
using NodeMoments = MomentsT<double>;
constexpr int N_MOMENTS = 13;

// Eqs. (eq_quadratur1-3) and the moment notation of Table I, in float64.
template <int N1, class R>
__device__ inline NodeMoments node_moments(const R* f, const R* g) {
  double s[4][N1], t[2][N1], u0, u1, u2, u3;
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    pair_sums<N1>(f + a * N1, s[0][a], s[1][a], s[2][a], s[3][a]);
    pair_sums<N1>(g + a * N1, t[0][a], t[1][a], u2, u3);
  }
  NodeMoments m;
  pair_sums<N1>(s[0], m.rho, m.jx, m.pxx, m.qxxx);
  pair_sums<N1>(s[1], m.jy, m.pxy, m.qxxy, u3);
  pair_sums<N1>(s[2], m.pyy, m.qxyy, u2, u3);
  pair_sums<N1>(s[3], m.qyyy, u1, u2, u3);
  pair_sums<N1>(t[0], m.g0, m.qgx, u2, u3);
  pair_sums<N1>(t[1], m.qgy, u1, u2, u3);
  (void)u0;
  return m;
}

// Float64 moments (Eqs. eq_quadratur1-3, Table I notation) of one
// distribution, accumulated one pair of +-xi_a columns at a time: the ten
// moments of orders 0-3 of f (D = 0) or the three of orders 0-1 of g (D = 1).
template <int D, int N1, class R>
__device__ inline void half_moments(const R* v, double* out) {
  using L = GH<N1>;
  constexpr int NM = D == 0 ? 10 : 3;
  double acc[NM];
  double u1, u2, u3;
  if (L::has_zero) {
    constexpr int a = N1 / 2;
    double s0, s1, s2, s3;
    pair_sums<N1>(v + a * N1, s0, s1, s2, s3);
    if (D == 0) {
      // rho, jx, jy, pxx, pxy, pyy, qxxx, qxxy, qxyy, qyyy
      acc[0] = s0; acc[1] = 0.0; acc[2] = s1; acc[3] = 0.0; acc[4] = 0.0;
      acc[5] = s2; acc[6] = 0.0; acc[7] = 0.0; acc[8] = 0.0; acc[9] = s3;
    } else {
      // g0, qgx, qgy
      acc[0] = s0; acc[1] = 0.0; acc[2] = s1;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NM; ++k) acc[k] = 0.0;
  }
  (void)u1; (void)u2; (void)u3;
#pragma unroll
  for (int k = 0; k < N1 / 2; ++k) {
    const int pa = N1 - 1 - k;
    const double x = L::xi(pa);
    double a0, a1, a2, a3, b0, b1, b2, b3;
    pair_sums<N1>(v + pa * N1, a0, a1, a2, a3);
    pair_sums<N1>(v + k * N1, b0, b1, b2, b3);
    const double e0 = a0 + b0, o0 = a0 - b0, e1 = a1 + b1;
    if (D == 0) {
      const double o1 = a1 - b1, e2 = a2 + b2, o2 = a2 - b2;
      acc[0] += e0;
      acc[1] += x * o0;
      acc[2] += e1;
      acc[3] += (x * x) * e0;
      acc[4] += x * o1;
      acc[5] += e2;
      acc[6] += (x * x * x) * o0;
      acc[7] += (x * x) * e1;
      acc[8] += x * o2;
      acc[9] += a3 + b3;
    } else {
      acc[0] += e0;
      acc[1] += x * o0;
      acc[2] += e1;
    }
  }
#pragma unroll
  for (int k = 0; k < NM; ++k) out[k] = acc[k];
}

// The same moments of w_i v_i, for values v in units of the weight (the
// deviations the 16-bit formats store): the weights enter the float64
// coefficients of the sums, so no value is scaled first.
template <int D, int N1, class R>
__device__ inline void half_moments_w(const R* v, double* out) {
  using L = GH<N1>;
  constexpr int NM = D == 0 ? 10 : 3;
  double acc[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) acc[k] = 0.0;
  // sums over b of w_b v_(a, b) xi_b^k, k = 0..3, folding +-xi_b pairs
  auto psum = [&](int a, double& s0, double& s1, double& s2, double& s3) {
    const R* r = v + a * N1;
    s0 = L::has_zero ? L::w(N1 / 2) * double(r[N1 / 2]) : 0.0;
    s1 = s2 = s3 = 0.0;
#pragma unroll
    for (int k = 0; k < N1 / 2; ++k) {
      const int pk = N1 - 1 - k;
      const double x = L::xi(pk), w = L::w(pk);
      const double e = double(r[pk]) + double(r[k]), o = double(r[pk]) - double(r[k]);
      s0 += w * e;
      s1 += (w * x) * o;
      s2 += (w * x * x) * e;
      s3 += (w * x * x * x) * o;
    }
  };
  if (L::has_zero) {
    const double wz = L::w(N1 / 2);
    double s0, s1, s2, s3;
    psum(N1 / 2, s0, s1, s2, s3);
    acc[0] += wz * s0;
    acc[2] += wz * s1;
    if (D == 0) {
      acc[5] += wz * s2;
      acc[9] += wz * s3;
    }
  }
#pragma unroll
  for (int k = 0; k < N1 / 2; ++k) {
    const int pa = N1 - 1 - k;
    const double x = L::xi(pa), w = L::w(pa);
    double a0, a1, a2, a3, b0, b1, b2, b3;
    psum(pa, a0, a1, a2, a3);
    psum(k, b0, b1, b2, b3);
    const double e0 = a0 + b0, o0 = a0 - b0, e1 = a1 + b1;
    acc[0] += w * e0;
    acc[1] += (w * x) * o0;
    acc[2] += w * e1;
    if (D == 0) {
      const double o1 = a1 - b1, e2 = a2 + b2, o2 = a2 - b2;
      acc[3] += (w * x * x) * e0;
      acc[4] += (w * x) * o1;
      acc[5] += w * e2;
      acc[6] += (w * x * x * x) * o0;
      acc[7] += (w * x * x) * e1;
      acc[8] += (w * x) * o2;
      acc[9] += w * (a3 + b3);
    }
  }
#pragma unroll
  for (int k = 0; k < NM; ++k) out[k] = acc[k];
}

// Hermite moments mu_k(u) = sum_j C(k,2j) (2j-1)!! t^j u^(k-2j) of a Gaussian
// of variance theta relative to the lattice reference (t = theta - 1): the 1-D
// factors of the equilibrium coefficients of App. D,
// a_(p,q) = rho mu_p(u_x) mu_q(u_y).
template <class R>
__device__ inline void gauss_hermite_moments(R u, R t, R* m) {
  const R u2 = u * u;
  m[0] = R(1);
  m[1] = u;
  m[2] = u2 + t;
  m[3] = u * (u2 + R(3) * t);
  m[4] = u2 * (u2 + R(6) * t) + R(3) * t * t;
}

// Collision coefficients of one node:  X_new = (1 - om1) X + w_i sum_k b_k H_k(i) / (p! q!)
// with b = om1 a^eq + (om1 - om2) (a* - a^eq)  (Eq. finalDiscretePDE).
// bf[p][q], bg[p][q] are in normalised units (a_n / sqrt(R T_ref)^n).
// V is the type of the intermediate (moment-level) arithmetic: float64 in the
// step kernels, a dual number in the adjoint kernel; om_scale and Pr are
// passed separately so that the adjoint can differentiate with respect to
// them (kp.om_scale and kp.Pr in the step kernels).
template <int SPLIT, int PRM, class R, class V = double>
__device__ inline void collision_coeffs(const MomentsT<V>& m, const KParams& kp, V om_scale, V Pr,
                                        R (&bf)[5][5], R (&bg)[3][3], R& om1_out) {
  const V rho = m.rho;
  const V irho = 1.0 / rho;
  const V ux = m.jx * irho, uy = m.jy * irho;
  const V E = SPLIT == 2 ? m.g0 + 0.5 * kp.c2 * (m.pxx + m.pyy) : m.g0;
  const V T = (E * irho - 0.5 * kp.c2 * (ux * ux + uy * uy)) * kp.inv_Cv;
  const V RT = kp.R * T;
  const V th = RT / kp.c2;
  const V p = rho * RT;

  // omega = dt / tau (Sec. II C): tau_nu = mu / p or fixed; tau_alpha = tau_nu / Pr.
  const R omn = R(kp.const_mu ? V(om_scale * p) : om_scale);
  R om1, om2;
  if (PRM == PR_HIGH) {
    om1 = omn * R(Pr);
    om2 = omn;
  } else {
    om1 = omn;
    om2 = PRM == PR_LOW ? omn * R(Pr) : omn;
  }
  om1_out = om1;
  const R dw = om1 - om2;

  R mx[5], my[5];
  gauss_hermite_moments(R(ux), R(th - 1.0), mx);
  gauss_hermite_moments(R(uy), R(th - 1.0), my);

  // f: equilibrium part, orders 0..NF
  constexpr int NF = Set<SPLIT>::NF;
  const R rw = om1 * R(rho);
#pragma unroll
  for (int a = 0; a <= NF; ++a)
#pragma unroll
    for (int b = 0; a + b <= NF; ++b) bf[a][b] = rw * mx[a] * my[b];

  // g: equilibrium part, orders 0..2
  if (SPLIT == 2) {
    const R ew = om1 * R(rho * (kp.Cv - kp.R) * T);  // U_ntr = rho (Cv - D R / 2) T
#pragma unroll
    for (int a = 0; a <= 2; ++a)
#pragma unroll
      for (int b = 0; a + b <= 2; ++b) bg[a][b] = ew * mx[a] * my[b];
  } else {
    // G0 = E, G1 = u (E + p), G2 = p uu + (E + p)(uu + RT delta)  (App. A);
    // a2 = G2 - RT_ref G0 delta.
    const R Er = R(E), pr = R(p), Ep = R(E + p), E2p = R(E + 2.0 * p);
    const R diag = R((E + p) * th - E);
    bg[0][0] = om1 * Er;
    bg[1][0] = om1 * R(ux) * Ep;
    bg[0][1] = om1 * R(uy) * Ep;
    bg[2][0] = om1 * (E2p * R(ux * ux) + diag);
    bg[1][1] = om1 * E2p * R(ux * uy);
    bg[0][2] = om1 * (E2p * R(uy * uy) + diag);
    (void)pr;
  }

  if (PRM == PR_UNIT) return;  // Table I: f* = f^eq, g* = g^eq

  // Non-equilibrium second moment, Delta P = M2(f) - M2(f^eq), in float64.
  const V dxx = m.pxx - rho * (ux * ux + th);
  const V dxy = m.pxy - rho * ux * uy;
  const V dyy = m.pyy - rho * (uy * uy + th);

  if (SPLIT == 2) {
    if (PRM == PR_LOW) {
      // M3* = M3(f) - S(u, Delta P),  S = [u A]_cyc - tr A / (D + 2) [u delta]_cyc;  M1(g*) = M1(g).
      const V tr4 = 0.25 * (dxx + dyy);
      const V Sxxx = 3.0 * ux * dxx - 3.0 * tr4 * ux;
      const V Sxxy = 2.0 * ux * dxy + uy * dxx - tr4 * uy;
      const V Sxyy = 2.0 * uy * dxy + ux * dyy - tr4 * ux;
      const V Syyy = 3.0 * uy * dyy - 3.0 * tr4 * uy;
      const V rt = rho * th;
      const V eqxxx = rho * ux * ux * ux + 3.0 * rt * ux;
      const V eqxxy = rho * ux * ux * uy + rt * uy;
      const V eqxyy = rho * ux * uy * uy + rt * ux;
      const V eqyyy = rho * uy * uy * uy + 3.0 * rt * uy;
      bf[3][0] += dw * R(m.qxxx - eqxxx - Sxxx);
      bf[2][1] += dw * R(m.qxxy - eqxxy - Sxxy);
      bf[1][2] += dw * R(m.qxyy - eqxyy - Sxyy);
      bf[0][3] += dw * R(m.qyyy - eqyyy - Syyy);
      const V e = rho * (kp.Cv - kp.R) * T;
      bg[1][0] += dw * R(m.qgx - e * ux);
      bg[0][1] += dw * R(m.qgy - e * uy);
    } else {
      // M2* = M2(f) - tr(Delta P)/D delta, M3* = M3(f^eq) + [u Delta P']_cyc,
      // a4* = a4^eq - [(a2* - a2^eq) delta]_cyc; g* = g^eq.
      const V h = 0.5 * (dxx + dyy);
      const R axx = R(dxx - h), axy = R(dxy), ayy = R(dyy - h);
      const R rux = R(ux), ruy = R(uy);
      bf[2][0] += dw * axx;
      bf[1][1] += dw * axy;
      bf[0][2] += dw * ayy;
      bf[3][0] += dw * (R(3) * rux * axx);
      bf[2][1] += dw * (R(2) * rux * axy + ruy * axx);
      bf[1][2] += dw * (R(2) * ruy * axy + rux * ayy);
      bf[0][3] += dw * (R(3) * ruy * ayy);
      bf[4][0] -= dw * (R(6) * axx);
      bf[3][1] -= dw * (R(3) * axy);
      bf[1][3] -= dw * (R(3) * axy);
      bf[0][4] -= dw * (R(6) * ayy);
      // [(a2* - a2^eq) delta]_(2,2) = axx + ayy = 0 (traceless)
    }
  } else {
    // split I:  u . Delta P  enters the heat flux of g*.
    const V upx = ux * dxx + uy * dxy, upy = ux * dxy + uy * dyy;
    if (PRM == PR_LOW) {
      // f* = f^eq;  M1(g*) = M1(g) - u . Delta P
      const V Ep = E + p;
      bg[1][0] += dw * R(m.qgx - kp.c2 * upx - ux * Ep);
      bg[0][1] += dw * R(m.qgy - kp.c2 * upy - uy * Ep);
    } else {
      // M2(f*) = M2(f);  M1(g*) = M1(g^eq) + u . Delta P
      bf[2][0] += dw * R(dxx);
      bf[1][1] += dw * R(dxy);
      bf[0][2] += dw * R(dyy);
      bg[1][0] += dw * R(kp.c2 * upx);
      bg[0][1] += dw * R(kp.c2 * upy);
    }
  }
}

// The deviation formats update d = X / w - r, where the rest value r (per
// weight) is itself a Grad expansion: r = sum_k a^rest_k He_k / k! with
// a^rest_(0,0) = 1 for f, and for g a^rest_(0,0) = gr0 plus, in split I,
// a^rest_(2,0) = a^rest_(0,2) = 2 gr1.  The relaxation term -om1 X / w of
// Eq. (finalDiscretePDE) is then -om1 d - om1 sum_k a^rest_k He_k / k!, so
// subtracting om1 a^rest from the collision coefficients b leaves
// d' = (1 - om1) d + sum_k (b_k - om1 a^rest_k) He_k / k! (+ flux): no term
// of the size of r is formed per population, and at rest b = om1 a^rest
// cancels exactly.
template <int SPLIT, class R>
__device__ inline void subtract_rest(R (&bf)[5][5], R (&bg)[3][3], R om1, const KParams& kp) {
  // each om1 a^rest is rounded as the coefficient it cancels was (a fused
  // multiply-add would subtract the exact product and leave that rounding)
#pragma clang fp contract(off)
  bf[0][0] -= om1;
  bg[0][0] -= om1 * R(kp.gr0);
  if (SPLIT == 1) {
    const R c = om1 * R(2.0 * kp.gr1);
    bg[2][0] -= c;
    bg[0][2] -= c;
  }
}

// out[i] += w_i sum_{p+q<=N} b[p][q] He_p(xi_a) He_q(xi_b) / (p! q!),  i = a N1 + b
// (Eq. Grad-Hermite-expansion-static in normalised units); without the
// weight w_i when WEIGHTED is false (deviation units X / w).
template <int N1, int N, class R, int BD, bool WEIGHTED = true>
__device__ inline void expand_add(const R (&b)[BD][BD], R* out) {
  using L = GH<N1>;
#pragma unroll
  for (int yb = 0; yb < N1; ++yb) {
    const double xb = L::xi(yb);
    R c[N + 1];
#pragma unroll
    for (int p = 0; p <= N; ++p) {
      c[p] = R(0);
#pragma unroll
      for (int q = 0; p + q <= N; ++q) {
        const double h = hn(q, xb);
        if (h != 0.0) c[p] += b[p][q] * R(h);
      }
    }
#pragma unroll
    for (int xa = 0; xa < N1; ++xa) {
      const double xv = L::xi(xa);
      const double wab = WEIGHTED ? L::w(xa) * L::w(yb) : 1.0;
      R acc = out[xa * N1 + yb];
#pragma unroll
      for (int p = 0; p <= N; ++p) {
        const double h = hn(p, xv);
        if (h != 0.0) acc += R(wab * h) * c[p];
      }
      out[xa * N1 + yb] = acc;
    }
  }
}

}  // namespace dvbm
