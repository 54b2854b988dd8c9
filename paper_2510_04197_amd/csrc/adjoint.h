// Discrete adjoint of the DDF-QE DVBM step (device code).
//
// For one step X' = F(X; tau_ref, Pr) of Eq. (finalDiscretePDE) and a
// cotangent lam' = dL/dX', a thread computes, for its cell c,
//   lam(c) = (dF/dX)^T lam'   restricted to the populations of c,
// and its share of (dF/dtau_ref)^T lam' and (dF/dPr)^T lam'.
//
//  * Relaxation part (local to the cell): F_i = (1 - om1) X_i + w_i sum_k b_k H_k(i).
//    With mu_k = sum_i lam'_i w_i H_k(i) and s = sum_i lam'_i X_i, the
//    cotangent of the moment vector m is  mbar_r = sum_k mu_k db_k/dm_r - s dom1/dm_r,
//    evaluated by forward-mode dual numbers (ADJ_DIRS seed directions per
//    pass) through the same coefficient code the step kernels use.  Moments are
//    linear in X, so lam_j = (1 - om1) lam'_j + sum_r mbar_r dm_r/dX_j.
//  * Flux part: every face value X_{f-1/2} of the NND reconstruction depends
//    on three neighbours; the limiter is differentiated on the branch the
//    forward evaluation selects (at a kink a.b = 0 the derivative is zero).
//    Each cell gathers the contributions of the faces that read it; ghost
//    cells of the zero-gradient rule pass theirs to the interior cell they copy.
#pragma once

#include "step.h"

namespace dvbm {

// ------------------------------------------------------------ dual numbers
struct D1 {
  double v, d;
  __host__ __device__ D1() : v(0.0), d(0.0) {}
  __host__ __device__ D1(double x) : v(x), d(0.0) {}  // NOLINT: implicit constant
  __host__ __device__ D1(double x, double dx) : v(x), d(dx) {}
};
__device__ inline D1 operator+(D1 a, D1 b) { return D1(a.v + b.v, a.d + b.d); }
__device__ inline D1 operator-(D1 a, D1 b) { return D1(a.v - b.v, a.d - b.d); }
__device__ inline D1 operator-(D1 a) { return D1(-a.v, -a.d); }
__device__ inline D1 operator*(D1 a, D1 b) { return D1(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline D1 operator/(D1 a, D1 b) { return D1(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
__device__ inline D1 operator+(D1 a, double b) { return D1(a.v + b, a.d); }
__device__ inline D1 operator+(double a, D1 b) { return D1(a + b.v, b.d); }
__device__ inline D1 operator-(D1 a, double b) { return D1(a.v - b, a.d); }
__device__ inline D1 operator-(double a, D1 b) { return D1(a - b.v, -b.d); }
__device__ inline D1 operator*(D1 a, double b) { return D1(a.v * b, a.d * b); }
__device__ inline D1 operator*(double a, D1 b) { return D1(a * b.v, a * b.d); }
__device__ inline D1 operator/(double a, D1 b) { return D1(a / b.v, -a * b.d / (b.v * b.v)); }
__device__ inline D1 operator/(D1 a, double b) { return D1(a.v / b, a.d / b); }
__device__ inline D1& operator+=(D1& a, D1 b) { return a = a + b; }
__device__ inline D1& operator-=(D1& a, D1 b) { return a = a - b; }
__device__ inline D1& operator*=(D1& a, D1 b) { return a = a * b; }

// Value and N directional derivatives: one pass of the coefficient code
// carries N seed directions, so the value part is evaluated once per N.
template <int N>
struct DN {
  double v, d[N];
  __device__ DN() : v(0.0) {
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = 0.0;
  }
  __device__ DN(double x) : v(x) {  // NOLINT: implicit constant
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = 0.0;
  }
};
template <int N>
__device__ inline DN<N> operator+(const DN<N>& a, const DN<N>& b) {
  DN<N> r(a.v + b.v);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N>
__device__ inline DN<N> operator-(const DN<N>& a, const DN<N>& b) {
  DN<N> r(a.v - b.v);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N>
__device__ inline DN<N> operator-(const DN<N>& a) {
  DN<N> r(-a.v);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N>
__device__ inline DN<N> operator*(const DN<N>& a, const DN<N>& b) {
  DN<N> r(a.v * b.v);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N>
__device__ inline DN<N> operator/(const DN<N>& a, const DN<N>& b) {
  const double inv = 1.0 / b.v;
  DN<N> r(a.v * inv);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * inv;
  return r;
}
template <int N>
__device__ inline DN<N> operator+(const DN<N>& a, double b) {
  DN<N> r = a;
  r.v += b;
  return r;
}
template <int N>
__device__ inline DN<N> operator+(double a, const DN<N>& b) { return b + a; }
template <int N>
__device__ inline DN<N> operator-(const DN<N>& a, double b) { return a + (-b); }
template <int N>
__device__ inline DN<N> operator-(double a, const DN<N>& b) { return (-b) + a; }
template <int N>
__device__ inline DN<N> operator*(const DN<N>& a, double b) {
  DN<N> r(a.v * b);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b;
  return r;
}
template <int N>
__device__ inline DN<N> operator*(double a, const DN<N>& b) { return b * a; }
template <int N>
__device__ inline DN<N> operator/(const DN<N>& a, double b) { return a * (1.0 / b); }
template <int N>
__device__ inline DN<N> operator/(double a, const DN<N>& b) {
  const double inv = 1.0 / b.v;
  DN<N> r(a * inv);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -r.v * b.d[k] * inv;
  return r;
}
template <int N>
__device__ inline DN<N>& operator+=(DN<N>& a, const DN<N>& b) { return a = a + b; }
template <int N>
__device__ inline DN<N>& operator-=(DN<N>& a, const DN<N>& b) { return a = a - b; }
template <int N>
__device__ inline DN<N>& operator*=(DN<N>& a, const DN<N>& b) { return a = a * b; }

// ------------------------------------------------------------ equilibrium of macroscopic fields
// Grad-Hermite equilibria f^eq, g^eq (Sec. II D 2, App. A, App. D) of one
// cell from rho, u (physical units) and T; V is double or D1.
template <int SPLIT, class V>
__device__ inline void equilibrium_cell(V rho, V ux, V uy, V T, const KParams& kp, V* f, V* g) {
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  constexpr int NF = Set<SPLIT>::NF;
  const double isc = 1.0 / sqrt(kp.c2);
  const V vx = ux * isc, vy = uy * isc;
  const V RT = kp.R * T, th = RT / kp.c2, p = rho * RT;
  const V E = rho * kp.Cv * T + 0.5 * rho * kp.c2 * (vx * vx + vy * vy);
  V mx[5], my[5];
  gauss_hermite_moments(vx, th - 1.0, mx);
  gauss_hermite_moments(vy, th - 1.0, my);
  V bf[5][5], bg[3][3];
  for (int a = 0; a <= NF; ++a)
    for (int b = 0; a + b <= NF; ++b) bf[a][b] = rho * mx[a] * my[b];
  if (SPLIT == 2) {
    const V e = rho * (kp.Cv - kp.R) * T;
    for (int a = 0; a <= 2; ++a)
      for (int b = 0; a + b <= 2; ++b) bg[a][b] = e * mx[a] * my[b];
  } else {
    const V diag = (E + p) * th - E;
    bg[0][0] = E;
    bg[1][0] = vx * (E + p);
    bg[0][1] = vy * (E + p);
    bg[2][0] = (E + 2.0 * p) * vx * vx + diag;
    bg[1][1] = (E + 2.0 * p) * vx * vy;
    bg[0][2] = (E + 2.0 * p) * vy * vy + diag;
  }
  for (int i = 0; i < Q; ++i) f[i] = g[i] = V(0.0);
  expand_add<N1, NF>(bf, f);
  expand_add<N1, 2>(bg, g);
}

// ------------------------------------------------------------ limiter partials
// (dL/da, dL/db) of L(a, b) = (b/2) phi(a, b) = 1/2 minmod(beta a, (a+b)/2, beta b)
// on the branch the forward evaluation takes.
__device__ inline void lim_partials(double a, double b, double beta, double& La, double& Lb) {
  La = Lb = 0.0;
  if (!(a * b > 0.0)) return;
  const double t1 = beta * fabs(a), t2 = 0.5 * fabs(a + b), t3 = beta * fabs(b);
  if (t1 <= t2 && t1 <= t3) {
    La = 0.5 * beta;
  } else if (t2 <= t3) {
    La = Lb = 0.25;
  } else {
    Lb = 0.5 * beta;
  }
}

template <int BC>
__device__ inline bool face_exists(int f, int n) {
  return BC == BC_PERIODIC ? true : (f >= 0 && f <= n);
}

// Flux-part cotangent of one population along one axis for cell c.
//   Xs[k]   = population at cell map(c - 3 + k), k = 0..6 (decoded);
//   lam[k]  = lam' at cell map(c - 2 + k), k = 0..4;
//   kv      = (dt / dx) v_alpha (non-zero); F(c) = ... - kv (face(c+1) - face(c)).
template <int BC>
__device__ inline double flux_adjoint(const double* Xs, const double* lam, int c, int n, double kv, double beta) {
  double acc = 0.0;
#pragma unroll
  for (int df = -1; df <= 2; ++df) {  // faces f = c + df (face f lies between cells f-1 and f)
    const int f = c + df;
    if (!face_exists<BC>(f, n)) continue;
    // dL/dface(f) = kv (lam'(f) - lam'(f-1)); cells outside a zero-gradient domain carry no lam'
    const bool in_r = BC == BC_PERIODIC || f <= n - 1;
    const bool in_l = BC == BC_PERIODIC || f >= 1;
    const double lr = in_r ? lam[df + 2] : 0.0;
    const double ll = in_l ? lam[df + 1] : 0.0;
    const double gface = kv * (lr - ll);
    if (gface == 0.0) continue;
    // inputs and partials of face(f)
    double p0, p1, p2;
    int q0;  // position (relative to c) of the first input
    if (kv > 0.0) {  // v >= 0: inputs f-2, f-1, f
      q0 = df - 2;
      const double X0 = Xs[q0 + 3], X1 = Xs[q0 + 4], X2 = Xs[q0 + 5];
      double La, Lb;
      lim_partials(X1 - X0, X2 - X1, beta, La, Lb);
      p0 = -La;
      p1 = 1.0 + La - Lb;
      p2 = Lb;
    } else {  // v < 0: inputs f-1, f, f+1
      q0 = df - 1;
      const double Y0 = Xs[q0 + 3], Y1 = Xs[q0 + 4], Y2 = Xs[q0 + 5];
      double La, Lb;
      lim_partials(Y1 - Y2, Y0 - Y1, beta, La, Lb);
      p0 = Lb;
      p1 = 1.0 + La - Lb;
      p2 = -La;
    }
    // add the partials of the input slots that are cell c (directly or as a ghost copy)
    const double ps[3] = {p0, p1, p2};
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int q = c + q0 + s;
      if (wrap<BC>(q, n) == c) acc += gface * ps[s];
    }
  }
  return acc;
}

// ------------------------------------------------------------ adjoint step in two kernels
// The relaxation part needs the 13 + 2 directional derivatives of the
// coefficient map at every cell; the flux part needs, for every population
// plane, the plane's stencil.  They run as two kernels:
//   relax: one thread per (cell, group of ADJ_DIRS directions) writes
//          mbar_r for its directions and 1 - om1 into a work array
//          work[r][cell] (r = 0..12 moments, 13: 1 - om1) and accumulates its
//          share of d/dtau_ref, d/dPr;
//   flux:  one thread per (population plane, cell) assembles
//          lam(c) = (1 - om1) lam'(c) + sum_r mbar_r dm_r/dX + flux cotangent.
constexpr int ADJ_DIRS = 5;                                       // directions per pass
constexpr int ADJ_GROUPS = (N_MOMENTS + 2 + ADJ_DIRS - 1) / ADJ_DIRS;  // passes per cell
constexpr int ADJ_WORK_ROWS = N_MOMENTS + 1;

// Stored value of population (d, i) at (x, y), decoded to float64.
template <int SPLIT, class S>
__device__ inline double adj_X(const typename S::T* __restrict__ state, const KParams& kp, int d, int i, int y,
                               int x) {
  constexpr int Q = Set<SPLIT>::Q;
  const typename S::T v = state[int64_t(d * Q + i) * kp.plane + int64_t(y) * kp.pitch + x];
  if (!S::dev) return double(S::raw(v));
  const double r = d == 0 ? 1.0 : g_ref_over_w<SPLIT>(kp, i);
  return weight<SPLIT>(i) * (r + double(S::raw(v)));
}

template <int SPLIT, class S, int PRM>
__device__ inline void cell_adjoint_relax(const typename S::T* __restrict__ state, const double* __restrict__ lam1,
                                          double* __restrict__ work, const KParams& kp, int c, int grp,
                                          double tau_ref, double& g_tau, double& g_pr) {
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  constexpr int NF = Set<SPLIT>::NF;
  using L = GH<N1>;
  const int64_t cells = int64_t(kp.nx) * kp.ny;
  const int y = c / kp.nx, x = c - y * kp.nx;

  // moments of the cell and the lam'-weighted Hermite projections
  double f[Q], g[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    f[i] = adj_X<SPLIT, S>(state, kp, 0, i, y, x);
    g[i] = adj_X<SPLIT, S>(state, kp, 1, i, y, x);
  }
  const NodeMoments m = node_moments<N1>(f, g);
  double mu_f[5][5], mu_g[3][3], s = 0.0;
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q < 5; ++q) mu_f[p][q] = 0.0;
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) mu_g[p][q] = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double lf = lam1[int64_t(i) * cells + c], lg = lam1[int64_t(Q + i) * cells + c];
    const double xa = L::xi(i / N1), xb = L::xi(i % N1), w = weight<SPLIT>(i);
#pragma unroll
    for (int p = 0; p <= NF; ++p)
#pragma unroll
      for (int q = 0; p + q <= NF; ++q) mu_f[p][q] += lf * (w * hn(p, xa) * hn(q, xb));
#pragma unroll
    for (int p = 0; p <= 2; ++p)
#pragma unroll
      for (int q = 0; p + q <= 2; ++q) mu_g[p][q] += lg * (w * hn(p, xa) * hn(q, xb));
    s += lf * f[i] + lg * g[i];
  }

  // directions r = grp * ADJ_DIRS + k: moments 0..12, 13: tau_ref, 14: Pr
  using V = DN<ADJ_DIRS>;
  const double mv[N_MOMENTS] = {m.rho, m.jx, m.jy, m.pxx, m.pxy, m.pyy, m.qxxx, m.qxxy, m.qxyy, m.qyyy,
                                m.g0, m.qgx, m.qgy};
  V md[N_MOMENTS];
  V oms(kp.om_scale), prd(kp.Pr);
#pragma unroll
  for (int k = 0; k < N_MOMENTS; ++k) md[k] = V(mv[k]);
#pragma unroll
  for (int k = 0; k < ADJ_DIRS; ++k) {
    const int r = grp * ADJ_DIRS + k;
#pragma unroll
    for (int j = 0; j < N_MOMENTS; ++j)
      if (j == r) md[j].d[k] = 1.0;
    // om_scale = dt / tau_ref [/ p_ref]:  d om_scale / d tau_ref = -om_scale / tau_ref
    if (r == N_MOMENTS) oms.d[k] = -kp.om_scale / tau_ref;
    if (r == N_MOMENTS + 1) prd.d[k] = 1.0;
  }
  const MomentsT<V> mdual = {md[0], md[1], md[2], md[3], md[4], md[5], md[6],
                             md[7], md[8], md[9], md[10], md[11], md[12]};
  V bf[5][5], bg[3][3], o1;
  collision_coeffs<SPLIT, PRM, V, V>(mdual, kp, oms, prd, bf, bg, o1);
  if (grp == 0) work[int64_t(N_MOMENTS) * cells + c] = 1.0 - o1.v;
#pragma unroll
  for (int k = 0; k < ADJ_DIRS; ++k) {
    const int r = grp * ADJ_DIRS + k;
    double t = -s * o1.d[k];
#pragma unroll
    for (int p = 0; p <= NF; ++p)
#pragma unroll
      for (int q = 0; p + q <= NF; ++q) t += mu_f[p][q] * bf[p][q].d[k];
#pragma unroll
    for (int p = 0; p <= 2; ++p)
#pragma unroll
      for (int q = 0; p + q <= 2; ++q) t += mu_g[p][q] * bg[p][q].d[k];
    if (r < N_MOMENTS)
      work[int64_t(r) * cells + c] = t;
    else if (r == N_MOMENTS)
      g_tau += t;
    else if (r == N_MOMENTS + 1)
      g_pr += t;
  }
}

template <int SPLIT, class S, int BCX, int BCY>
__device__ inline void plane_adjoint_flux(const typename S::T* __restrict__ state, const double* __restrict__ lam1,
                                          const double* __restrict__ work, double* __restrict__ lam0,
                                          const KParams& kp, int pl, int x, int y) {
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  using L = GH<N1>;
  const int64_t cells = int64_t(kp.nx) * kp.ny;
  const int64_t c = int64_t(y) * kp.nx + x;
  const int d = pl / Q, i = pl % Q;
  const double xa = L::xi(i / N1), xb = L::xi(i % N1);
  const double* lp = lam1 + int64_t(pl) * cells;
  double out = work[int64_t(N_MOMENTS) * cells + c] * lp[c];
  auto mb = [&](int r) { return work[int64_t(r) * cells + c]; };
  if (d == 0) {
    const double xa2 = xa * xa, xb2 = xb * xb;
    out += mb(0) + mb(1) * xa + mb(2) * xb + mb(3) * xa2 + mb(4) * (xa * xb) + mb(5) * xb2 + mb(6) * (xa2 * xa) +
           mb(7) * (xa2 * xb) + mb(8) * (xa * xb2) + mb(9) * (xb2 * xb);
  } else {
    out += mb(10) + mb(11) * xa + mb(12) * xb;
  }
  const double beta = 0.5 * kp.beta2;
  if (xa != 0.0) {
    double Xs[7], lm[5];
#pragma unroll
    for (int k = 0; k < 7; ++k) Xs[k] = adj_X<SPLIT, S>(state, kp, d, i, y, wrap<BCX>(x - 3 + k, kp.nx));
#pragma unroll
    for (int k = 0; k < 5; ++k) lm[k] = lp[int64_t(y) * kp.nx + wrap<BCX>(x - 2 + k, kp.nx)];
    out += flux_adjoint<BCX>(Xs, lm, x, kp.nx, kp.kx * xa, beta);
  }
  if (xb != 0.0) {
    double Xs[7], lm[5];
#pragma unroll
    for (int k = 0; k < 7; ++k) Xs[k] = adj_X<SPLIT, S>(state, kp, d, i, wrap<BCY>(y - 3 + k, kp.ny), x);
#pragma unroll
    for (int k = 0; k < 5; ++k) lm[k] = lp[int64_t(wrap<BCY>(y - 2 + k, kp.ny)) * kp.nx + x];
    out += flux_adjoint<BCY>(Xs, lm, y, kp.ny, kp.ky * xb, beta);
  }
  lam0[int64_t(pl) * cells + c] = out;
}

// ------------------------------------------------------------ readout adjoint
// lam_j = sum over fields of dfield/dX_j times the field cotangent, for the
// fields rho, u_x, u_y, T of Eqs. (eq_quadratur1-3) and (eq:Total_energy_MB).
template <int SPLIT>
__device__ inline void readout_adjoint_cell(const NodeMoments& m, const KParams& kp, double rb, double uxb,
                                            double uyb, double Tb, double* lf, double* lg) {
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  using L = GH<N1>;
  const double c = sqrt(kp.c2);
  // inputs: rho, jx, jy, pxx + pyy, g0 (normalised moments)
  const double in[5] = {m.rho, m.jx, m.jy, m.pxx + m.pyy, m.g0};
  double bar[5];
  for (int r = 0; r < 5; ++r) {
    D1 v[5];
    for (int k = 0; k < 5; ++k) v[k] = D1(in[k], k == r ? 1.0 : 0.0);
    const D1 rho = v[0];
    const D1 ux = c * v[1] / rho, uy = c * v[2] / rho;
    const D1 E = SPLIT == 2 ? v[4] + 0.5 * kp.c2 * v[3] : v[4];
    const D1 T = (E / rho - 0.5 * (ux * ux + uy * uy)) * kp.inv_Cv;
    bar[r] = rb * rho.d + uxb * ux.d + uyb * uy.d + Tb * T.d;
  }
  for (int i = 0; i < Q; ++i) {
    const double xa = L::xi(i / N1), xb = L::xi(i % N1);
    lf[i] = bar[0] + bar[1] * xa + bar[2] * xb + bar[3] * (xa * xa + xb * xb);
    lg[i] = bar[4];
  }
}

}  // namespace dvbm
