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
//    the gradient of one scalar, taken in reverse mode (coeffs_vjp).  Moments are
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
  // the candidate the forward min selects (ties in the same order), as selects, without branches
  const double t1 = beta * fabs(a), t2 = 0.5 * fabs(a + b), t3 = beta * fabs(b);
  const bool act = a * b > 0.0;
  const bool c1 = t1 <= t2 && t1 <= t3;
  const bool c2 = !c1 && t2 <= t3;
  La = act ? (c1 ? 0.5 * beta : (c2 ? 0.25 : 0.0)) : 0.0;
  Lb = act ? (c1 ? 0.0 : (c2 ? 0.25 : 0.5 * beta)) : 0.0;
}

// ------------------------------------------------------------ reverse mode of the coefficient map
// Gradient of  phi = sum_pq muf[p][q] bf[p][q] + sum_pq mug[p][q] bg[p][q] - s om1
// (bf, bg, om1 as computed by collision_coeffs from the moments m and the
// scalars om_scale, Pr) with respect to the 13 moments (mbar, in the order
// rho, jx, jy, pxx, pxy, pyy, qxxx, qxxy, qxyy, qyyy, g0, qgx, qgy), to
// om_scale (d_oms) and to Pr (d_pr): one forward sweep of the same
// arithmetic, then the chain rule applied backwards, term by term.
template <int SPLIT, int PRM>
__device__ inline void coeffs_vjp(const NodeMoments& m, const KParams& kp, double oms, double Pr,
                                  const double (&muf)[5][5], const double (&mug)[3][3], double s,
                                  double (&mbar)[N_MOMENTS], double& d_oms, double& d_pr, double& om1_out) {
  constexpr int NF = Set<SPLIT>::NF;
  const double c2 = kp.c2;
  // ---- forward
  const double rho = m.rho, irho = 1.0 / rho;
  const double ux = m.jx * irho, uy = m.jy * irho;
  const double E = SPLIT == 2 ? m.g0 + 0.5 * c2 * (m.pxx + m.pyy) : m.g0;
  const double T = (E * irho - 0.5 * c2 * (ux * ux + uy * uy)) * kp.inv_Cv;
  const double RT = kp.R * T, th = RT / c2, p = rho * RT;
  const double omn = kp.const_mu ? oms * p : oms;
  const double om1 = PRM == PR_HIGH ? omn * Pr : omn;
  const double om2 = PRM == PR_LOW ? omn * Pr : omn;
  const double dw = om1 - om2;
  om1_out = om1;
  const double t = th - 1.0;
  double mx[5], my[5];
  gauss_hermite_moments(ux, t, mx);
  gauss_hermite_moments(uy, t, my);
  const double dxx = m.pxx - rho * (ux * ux + th), dxy = m.pxy - rho * ux * uy, dyy = m.pyy - rho * (uy * uy + th);

  // ---- adjoints of the intermediates
  double rho_b = 0, ux_b = 0, uy_b = 0, th_b = 0, T_b = 0, E_b = 0, p_b = 0, om1_b = -s, dw_b = 0;
  double dxx_b = 0, dxy_b = 0, dyy_b = 0;
  double mx_b[5] = {0, 0, 0, 0, 0}, my_b[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < N_MOMENTS; ++k) mbar[k] = 0.0;

  // f equilibrium: bf = om1 rho mx[a] my[b]
  {
    const double rw = om1 * rho;
    double rw_b = 0.0;
#pragma unroll
    for (int a = 0; a <= NF; ++a)
#pragma unroll
      for (int b = 0; a + b <= NF; ++b) {
        rw_b += muf[a][b] * mx[a] * my[b];
        mx_b[a] += rw * muf[a][b] * my[b];
        my_b[b] += rw * muf[a][b] * mx[a];
      }
    om1_b += rw_b * rho;
    rho_b += rw_b * om1;
  }
  // g equilibrium
  if (SPLIT == 2) {
    const double cr = kp.Cv - kp.R, ew = om1 * rho * cr * T;
    double ew_b = 0.0;
#pragma unroll
    for (int a = 0; a <= 2; ++a)
#pragma unroll
      for (int b = 0; a + b <= 2; ++b) {
        ew_b += mug[a][b] * mx[a] * my[b];
        mx_b[a] += ew * mug[a][b] * my[b];
        my_b[b] += ew * mug[a][b] * mx[a];
      }
    om1_b += ew_b * rho * cr * T;
    rho_b += ew_b * om1 * cr * T;
    T_b += ew_b * om1 * rho * cr;
  } else {
    const double Ep = E + p, E2p = E + 2.0 * p, diag = Ep * th - E;
    double Ep_b = 0.0, E2p_b = 0.0, diag_b = 0.0;
    om1_b += mug[0][0] * E + mug[1][0] * ux * Ep + mug[0][1] * uy * Ep + mug[2][0] * (E2p * ux * ux + diag) +
             mug[1][1] * E2p * ux * uy + mug[0][2] * (E2p * uy * uy + diag);
    E_b += mug[0][0] * om1;
    ux_b += mug[1][0] * om1 * Ep + mug[2][0] * om1 * E2p * 2.0 * ux + mug[1][1] * om1 * E2p * uy;
    uy_b += mug[0][1] * om1 * Ep + mug[0][2] * om1 * E2p * 2.0 * uy + mug[1][1] * om1 * E2p * ux;
    Ep_b += (mug[1][0] * ux + mug[0][1] * uy) * om1;
    E2p_b += om1 * (mug[2][0] * ux * ux + mug[1][1] * ux * uy + mug[0][2] * uy * uy);
    diag_b += om1 * (mug[2][0] + mug[0][2]);
    // diag = Ep th - E
    Ep_b += diag_b * th;
    th_b += diag_b * Ep;
    E_b -= diag_b;
    E_b += Ep_b + E2p_b;
    p_b += Ep_b + 2.0 * E2p_b;
  }

  // quasi-equilibrium parts (Table I)
  if (PRM != PR_UNIT) {
    if (SPLIT == 2) {
      if (PRM == PR_LOW) {
        const double tr4 = 0.25 * (dxx + dyy), rt = rho * th, cr = kp.Cv - kp.R, e = rho * cr * T;
        const double Sxxx = 3.0 * ux * dxx - 3.0 * tr4 * ux, Sxxy = 2.0 * ux * dxy + uy * dxx - tr4 * uy;
        const double Sxyy = 2.0 * uy * dxy + ux * dyy - tr4 * ux, Syyy = 3.0 * uy * dyy - 3.0 * tr4 * uy;
        const double eqxxx = rho * ux * ux * ux + 3.0 * rt * ux, eqxxy = rho * ux * ux * uy + rt * uy;
        const double eqxyy = rho * ux * uy * uy + rt * ux, eqyyy = rho * uy * uy * uy + 3.0 * rt * uy;
        dw_b += muf[3][0] * (m.qxxx - eqxxx - Sxxx) + muf[2][1] * (m.qxxy - eqxxy - Sxxy) +
                muf[1][2] * (m.qxyy - eqxyy - Sxyy) + muf[0][3] * (m.qyyy - eqyyy - Syyy) +
                mug[1][0] * (m.qgx - e * ux) + mug[0][1] * (m.qgy - e * uy);
        mbar[6] += dw * muf[3][0];
        mbar[7] += dw * muf[2][1];
        mbar[8] += dw * muf[1][2];
        mbar[9] += dw * muf[0][3];
        mbar[11] += dw * mug[1][0];
        mbar[12] += dw * mug[0][1];
        const double n30 = -dw * muf[3][0], n21 = -dw * muf[2][1], n12 = -dw * muf[1][2], n03 = -dw * muf[0][3];
        // equilibrium third moments
        double rt_b = n30 * 3.0 * ux + n21 * uy + n12 * ux + n03 * 3.0 * uy;
        rho_b += n30 * ux * ux * ux + n21 * ux * ux * uy + n12 * ux * uy * uy + n03 * uy * uy * uy;
        ux_b += n30 * (3.0 * rho * ux * ux + 3.0 * rt) + n21 * 2.0 * rho * ux * uy + n12 * (rho * uy * uy + rt);
        uy_b += n21 * (rho * ux * ux + rt) + n12 * 2.0 * rho * ux * uy + n03 * (3.0 * rho * uy * uy + 3.0 * rt);
        rho_b += rt_b * th;
        th_b += rt_b * rho;
        // S(u, Delta P)
        ux_b += n30 * (3.0 * dxx - 3.0 * tr4) + n21 * 2.0 * dxy + n12 * (dyy - tr4);
        uy_b += n21 * (dxx - tr4) + n12 * 2.0 * dxy + n03 * (3.0 * dyy - 3.0 * tr4);
        dxx_b += n30 * 3.0 * ux + n21 * uy;
        dxy_b += n21 * 2.0 * ux + n12 * 2.0 * uy;
        dyy_b += n12 * ux + n03 * 3.0 * uy;
        const double tr4_b = -(n30 * 3.0 * ux + n21 * uy + n12 * ux + n03 * 3.0 * uy);
        dxx_b += 0.25 * tr4_b;
        dyy_b += 0.25 * tr4_b;
        // g heat flux: - e u
        const double g10 = -dw * mug[1][0], g01 = -dw * mug[0][1];
        const double e_b = g10 * ux + g01 * uy;
        ux_b += g10 * e;
        uy_b += g01 * e;
        rho_b += e_b * cr * T;
        T_b += e_b * rho * cr;
      } else {
        const double h = 0.5 * (dxx + dyy), axx = dxx - h, axy = dxy, ayy = dyy - h;
        dw_b += muf[2][0] * axx + muf[1][1] * axy + muf[0][2] * ayy + muf[3][0] * 3.0 * ux * axx +
                muf[2][1] * (2.0 * ux * axy + uy * axx) + muf[1][2] * (2.0 * uy * axy + ux * ayy) +
                muf[0][3] * 3.0 * uy * ayy - muf[4][0] * 6.0 * axx - muf[3][1] * 3.0 * axy -
                muf[1][3] * 3.0 * axy - muf[0][4] * 6.0 * ayy;
        const double axx_b = dw * (muf[2][0] + 3.0 * ux * muf[3][0] + uy * muf[2][1] - 6.0 * muf[4][0]);
        const double axy_b = dw * (muf[1][1] + 2.0 * ux * muf[2][1] + 2.0 * uy * muf[1][2] - 3.0 * muf[3][1] -
                                   3.0 * muf[1][3]);
        const double ayy_b = dw * (muf[0][2] + ux * muf[1][2] + 3.0 * uy * muf[0][3] - 6.0 * muf[0][4]);
        ux_b += dw * (3.0 * axx * muf[3][0] + 2.0 * axy * muf[2][1] + ayy * muf[1][2]);
        uy_b += dw * (axx * muf[2][1] + 2.0 * axy * muf[1][2] + 3.0 * ayy * muf[0][3]);
        const double h_b = -(axx_b + ayy_b);
        dxx_b += axx_b + 0.5 * h_b;
        dyy_b += ayy_b + 0.5 * h_b;
        dxy_b += axy_b;
      }
    } else {
      const double upx = ux * dxx + uy * dxy, upy = ux * dxy + uy * dyy;
      double upx_b, upy_b;
      if (PRM == PR_LOW) {
        const double Ep = E + p;
        dw_b += mug[1][0] * (m.qgx - c2 * upx - ux * Ep) + mug[0][1] * (m.qgy - c2 * upy - uy * Ep);
        mbar[11] += dw * mug[1][0];
        mbar[12] += dw * mug[0][1];
        upx_b = -dw * mug[1][0] * c2;
        upy_b = -dw * mug[0][1] * c2;
        ux_b -= dw * mug[1][0] * Ep;
        uy_b -= dw * mug[0][1] * Ep;
        const double Ep_b = -dw * (mug[1][0] * ux + mug[0][1] * uy);
        E_b += Ep_b;
        p_b += Ep_b;
      } else {
        dw_b += muf[2][0] * dxx + muf[1][1] * dxy + muf[0][2] * dyy + mug[1][0] * c2 * upx + mug[0][1] * c2 * upy;
        dxx_b += dw * muf[2][0];
        dxy_b += dw * muf[1][1];
        dyy_b += dw * muf[0][2];
        upx_b = dw * mug[1][0] * c2;
        upy_b = dw * mug[0][1] * c2;
      }
      ux_b += upx_b * dxx + upy_b * dxy;
      uy_b += upx_b * dxy + upy_b * dyy;
      dxx_b += upx_b * ux;
      dxy_b += upx_b * uy + upy_b * ux;
      dyy_b += upy_b * uy;
    }
    // Delta P = M2 - M2(f^eq)
    mbar[3] += dxx_b;
    mbar[4] += dxy_b;
    mbar[5] += dyy_b;
    rho_b -= dxx_b * (ux * ux + th) + dxy_b * ux * uy + dyy_b * (uy * uy + th);
    ux_b -= dxx_b * rho * 2.0 * ux + dxy_b * rho * uy;
    uy_b -= dxy_b * rho * ux + dyy_b * rho * 2.0 * uy;
    th_b -= (dxx_b + dyy_b) * rho;
  }

  // Hermite moments mu_k(u, t), t = th - 1
  {
    double t_b = 0.0;
    const double u2x = ux * ux, u2y = uy * uy;
    ux_b += mx_b[1] + mx_b[2] * 2.0 * ux + mx_b[3] * (3.0 * u2x + 3.0 * t) + mx_b[4] * (4.0 * u2x * ux + 12.0 * t * ux);
    uy_b += my_b[1] + my_b[2] * 2.0 * uy + my_b[3] * (3.0 * u2y + 3.0 * t) + my_b[4] * (4.0 * u2y * uy + 12.0 * t * uy);
    t_b += mx_b[2] + mx_b[3] * 3.0 * ux + mx_b[4] * (6.0 * u2x + 6.0 * t);
    t_b += my_b[2] + my_b[3] * 3.0 * uy + my_b[4] * (6.0 * u2y + 6.0 * t);
    th_b += t_b;
  }
  // relaxation rates
  om1_b += dw_b;
  const double om2_b = -dw_b;
  double omn_b;
  if (PRM == PR_HIGH) {
    omn_b = om1_b * Pr + om2_b;
    d_pr = om1_b * omn;
  } else if (PRM == PR_LOW) {
    omn_b = om1_b + om2_b * Pr;
    d_pr = om2_b * omn;
  } else {
    omn_b = om1_b + om2_b;
    d_pr = 0.0;
  }
  if (kp.const_mu) {
    d_oms = omn_b * p;
    p_b += omn_b * oms;
  } else {
    d_oms = omn_b;
  }
  // macroscopic chain: th = R T / c2, p = rho R T, T = (E / rho - c2 |u|^2 / 2) / Cv
  double RT_b = th_b / c2 + p_b * rho;
  rho_b += p_b * RT;
  T_b += kp.R * RT_b;
  E_b += T_b * kp.inv_Cv * irho;
  double irho_b = T_b * kp.inv_Cv * E;
  const double K_b = -T_b * kp.inv_Cv;
  ux_b += K_b * c2 * ux;
  uy_b += K_b * c2 * uy;
  if (SPLIT == 2) {
    mbar[10] += E_b;
    mbar[3] += 0.5 * c2 * E_b;
    mbar[5] += 0.5 * c2 * E_b;
  } else {
    mbar[10] += E_b;
  }
  mbar[1] += ux_b * irho;
  mbar[2] += uy_b * irho;
  irho_b += ux_b * m.jx + uy_b * m.jy;
  rho_b -= irho_b * irho * irho;
  mbar[0] += rho_b;
}

// ------------------------------------------------------------ adjoint step in two kernels
// The relaxation part needs the gradient of the coefficient map at every
// cell; the flux part needs, for every population plane, the plane's
// stencil.  They run as two kernels:
//   relax: one thread per cell takes the reverse pass coeffs_vjp, writes
//          mbar_r and 1 - om1 into a work array work[r][cell] (r = 0..12
//          moments, 13: 1 - om1) and accumulates its share of d/dtau_ref,
//          d/dPr;
//   flux:  one wave per (group of population planes, strip of cells, range
//          of rows) assembles, row after row,
//          lam(c) = (1 - om1) lam'(c) + sum_r mbar_r dm_r/dX + flux cotangent.
constexpr int ADJ_WORK_ROWS = N_MOMENTS + 1;

// Stored value of population (d, i) at (x, y), decoded to float64.
template <int SPLIT, class S>
__device__ inline double adj_X(const typename S::T* __restrict__ state, const KParams& kp, int d, int i, int y,
                               int x) {
  constexpr int Q = Set<SPLIT>::Q;
  const typename S::T v = state[sidx(kp, d, i, y, x)];
  if (!S::dev) return double(S::raw(v));
  const double r = d == 0 ? 1.0 : g_ref_over_w<SPLIT>(kp, i);
  return weight<SPLIT>(i) * (r + double(S::raw(v)));
}

template <int SPLIT, class S, int PRM, class LT>
__device__ inline void cell_adjoint_relax(const typename S::T* __restrict__ state, const LT* __restrict__ lam1,
                                          double* __restrict__ work, const KParams& kp, int c, double tau_ref,
                                          double& g_tau, double& g_pr) {
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
  // mu[p][q] = sum_i lam'_i w_i He_p(xi_a)/p! He_q(xi_b)/q!, factorised over the
  // tensor-product set: t[a][q] = sum_b lam'_(a,b) w_b He_q(xi_b)/q!, then
  // mu[p][q] = sum_a w_a He_p(xi_a)/p! t[a][q]
  double mu_f[5][5], mu_g[3][3], s = 0.0;
  double tf[N1][NF + 1], tg[N1][3];
#pragma unroll
  for (int a = 0; a < N1; ++a) {
#pragma unroll
    for (int q = 0; q <= NF; ++q) tf[a][q] = 0.0;
#pragma unroll
    for (int q = 0; q <= 2; ++q) tg[a][q] = 0.0;
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      const int i = a * N1 + b;
      const double lf = double(lam1[int64_t(i) * cells + c]), lg = double(lam1[int64_t(Q + i) * cells + c]);
      const double xb = L::xi(b), wb = L::w(b);
#pragma unroll
      for (int q = 0; q <= NF; ++q) {
        const double h = wb * hn(q, xb);
        if (h != 0.0) tf[a][q] += lf * h;
      }
#pragma unroll
      for (int q = 0; q <= 2; ++q) {
        const double h = wb * hn(q, xb);
        if (h != 0.0) tg[a][q] += lg * h;
      }
      s += lf * f[i] + lg * g[i];
    }
  }
#pragma unroll
  for (int p = 0; p < 5; ++p)
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      mu_f[p][q] = 0.0;
      if (p + q > NF) continue;
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const double h = L::w(a) * hn(p, L::xi(a));
        if (h != 0.0) mu_f[p][q] += h * tf[a][q];
      }
    }
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      mu_g[p][q] = 0.0;
      if (p + q > 2) continue;
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const double h = L::w(a) * hn(p, L::xi(a));
        if (h != 0.0) mu_g[p][q] += h * tg[a][q];
      }
    }
  double mbar[N_MOMENTS], d_oms, d_pr, om1;
  coeffs_vjp<SPLIT, PRM>(m, kp, kp.om_scale, kp.Pr, mu_f, mu_g, s, mbar, d_oms, d_pr, om1);
#pragma unroll
  for (int r = 0; r < N_MOMENTS; ++r) work[int64_t(r) * cells + c] = mbar[r];
  work[int64_t(N_MOMENTS) * cells + c] = 1.0 - om1;
  // om_scale = dt / tau_ref [/ p_ref]:  d om_scale / d tau_ref = -om_scale / tau_ref
  g_tau += d_oms * (-kp.om_scale / tau_ref);
  g_pr += d_pr;
}

// float64 value held by lane l - 1 (l + 1) of the wave; lane 0 (63) reads 0.
__device__ inline double lane_prev_d(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_mov_dpp(int(uint32_t(b)), 0x138, 0xf, 0xf, true);
  const uint32_t hi = __builtin_amdgcn_mov_dpp(int(uint32_t(b >> 32)), 0x138, 0xf, 0xf, true);
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
__device__ inline double lane_next_d(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_mov_dpp(int(uint32_t(b)), 0x130, 0xf, 0xf, true);
  const uint32_t hi = __builtin_amdgcn_mov_dpp(int(uint32_t(b >> 32)), 0x130, 0xf, 0xf, true);
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// Cells per strip of the flux adjoint: a wave's 64 lanes hold the columns
// x0 - 3 .. x0 + 60 of one row; lanes 3 .. 60 own their cells, the three
// lanes at each end supply the x stencil (radius 3) of their neighbours.
constexpr int ADJ_STRIP = 58;

// ------------------------------------------------------------ flux adjoint, row sweep
// One wave takes the N1 planes (d, a, b), b = 0 .. N1-1, of one distribution
// d and one abscissa xi_a, a strip of ADJ_STRIP columns and the rows
// [ya, yb), and walks the rows upwards.  Along x, lane l forms the face
// between the columns x-1 and x of the row once, and its three partials
// reach their cells through lane shifts.  Along y every face is formed once.  At row c the wave forms face c+2
// (xi_b > 0) or face c+1 (xi_b < 0); in both cases its three inputs are the
// rows c, c+1, c+2 and its three partials belong to the rows c, c+1, c+2, so
// the shares of the rows c+1 and c+2 are carried to the next rows (p1, p2).
// The walk starts two rows early, at ya - 2, to collect the shares of the
// faces below ya.  Under the zero-gradient rule the rows outside the domain
// are copies of the edge rows and carry no lam': their shares (the rows
// -2, -1 and ny, ny+1) go to the edge rows.  A ring of four rows per plane
// holds X and lam' of the rows c .. c+3 (row c+3 in flight).
// The relaxation part comes from the work array, read once per row for all
// N1 planes: with xi_a fixed the Hermite polynomial of the moment cotangents
// is a cubic (f) or linear (g) polynomial in xi_b.
template <int SPLIT, class S, int BCX, int BCY, int D, class LT>
__device__ inline void sweep_adjoint_flux(const typename S::T* __restrict__ state, const LT* __restrict__ lam1,
                                          const double* __restrict__ work, LT* __restrict__ lam0,
                                          const KParams& kp, int a, int x0, int ya, int yb) {
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  constexpr bool ZGY = BCY != BC_PERIODIC;
  using L = GH<N1>;
  const int64_t cells = int64_t(kp.nx) * kp.ny;
  const int lane = threadIdx.x & 63;
  const int x = x0 - 3 + lane;
  const bool own = lane >= 3 && lane < 61 && x < kp.nx;
  const int gx = wrap_any<BCX>(x, kp.nx);
  const double xa = L::xi(a);
  const double beta = 0.5 * kp.beta2;
  const double kvx = kp.kx * xa;
  const int pl0 = D * Q + a * N1;
  const LT* lp = lam1 + int64_t(pl0) * cells + gx;
  // stores of lam through one buffer resource per plane (dense rows of nx
  // values, a plane well below 2 GiB); the stencil-only lanes store to offset
  // 2^31, which the bounds check discards, so no branch guards the stores
  // (a branch there makes every store wait for all loads in flight)
  const uint32_t lrow_bytes = uint32_t(kp.nx) * uint32_t(sizeof(LT));
  const uint32_t lplane_bytes = uint32_t(cells) * uint32_t(sizeof(LT));
  const uint32_t lvo_st = own ? uint32_t(x) * uint32_t(sizeof(LT)) : 0x80000000u;

  constexpr int NW = D == 0 ? 11 : 4;  // work rows read: 0..9 and 13 (f), 10..13 (g)
  double X[N1][4], Lm[N1][4], p1[N1], p2[N1], gs[N1];
  double zf[4];  // 1 inside the domain, 0 for the rows outside (zero-gradient)
#pragma unroll
  for (int b = 0; b < N1; ++b) p1[b] = p2[b] = gs[b] = 0.0;

  auto fill = [&](auto slot, int r) {
    constexpr int s = decltype(slot)::value;
    const int ry = wrap<BCY>(r, kp.ny);
    zf[s] = (!ZGY || (r >= 0 && r < kp.ny)) ? 1.0 : 0.0;
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      X[b][s] = adj_X<SPLIT, S>(state, kp, D, a * N1 + b, ry, gx);
      Lm[b][s] = double(lp[int64_t(b) * cells + int64_t(ry) * kp.nx]);
    }
  };

  // the NW work rows of row r (a start-up row reads an edge row and ignores it)
  auto load_work = [&](double* dst, int r) {
    const int rr = r < 0 ? 0 : (r >= kp.ny ? kp.ny - 1 : r);
    const int64_t cc = int64_t(rr) * kp.nx + gx;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int row = D == 0 ? (k < 10 ? k : N_MOMENTS) : (k < 3 ? 10 + k : N_MOMENTS);
      dst[k] = work[int64_t(row) * cells + cc];
    }
  };

  auto step = [&](auto phase, int c) {
    constexpr int P = decltype(phase)::value;
    constexpr int s0 = P, s1 = (P + 1) & 3, s2 = (P + 2) & 3, s3 = (P + 3) & 3;
    const bool outrow = c >= ya;
    // relaxation part: moment cotangents of the cell (row c; a start-up row
    // reads row 0 and ignores it).  They are loaded before row c+3 is
    // requested: loads complete in order, so waiting for them then does not
    // wait for the new row.
    double w[NW];
    load_work(w, c);
    __builtin_amdgcn_sched_barrier(0);  // keep the row-(c+3) loads after these
    // row c+3 into the slot of row c-1 (past the last needed row, yb+1, a
    // repeat of that row that is never read)
    fill(std::integral_constant<int, s3>(), c + 3 <= yb + 1 ? c + 3 : yb + 1);
    const bool last = ZGY && c == kp.ny - 1;
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      const double xb = L::xi(b);
      // y: the face of this row and the carried shares
      double oy = 0.0;
      if (xb != 0.0) {
        const double kv = kp.ky * xb;
        const double X0 = X[b][s0], X1 = X[b][s1], X2 = X[b][s2];
        double La, Lb, G0, G1, G2;
        if (xb > 0.0) {  // face c+2: inputs c, c+1, c+2; dL/dface = kv (lam'(c+2) - lam'(c+1))
          const double g = kv * (zf[s2] * Lm[b][s2] - zf[s1] * Lm[b][s1]);
          lim_partials(X1 - X0, X2 - X1, beta, La, Lb);
          G0 = -La * g;
          G1 = (1.0 + La - Lb) * g;
          G2 = Lb * g;
        } else {  // face c+1: inputs c, c+1, c+2; dL/dface = kv (lam'(c+1) - lam'(c))
          const double g = kv * (zf[s1] * Lm[b][s1] - zf[s0] * Lm[b][s0]);
          lim_partials(X1 - X2, X0 - X1, beta, La, Lb);
          G0 = Lb * g;
          G1 = (1.0 + La - Lb) * g;
          G2 = -La * g;
        }
        oy = p1[b] + G0;
        p1[b] = p2[b] + G1;
        p2[b] = G2;
        if (last) oy += p1[b] + p2[b];  // shares of the rows ny, ny+1
      }
      if (!outrow) {
        if (ZGY) gs[b] += oy;  // shares of the rows -2, -1 (used when ya == 0)
        continue;
      }
      double out = oy;
      if (ZGY && c == 0) out += gs[b];
      // x: lane l forms face x (between x-1 and x) of row c
      if (kvx != 0.0) {
        const double Xc = X[b][s0], lc = Lm[b][s0];
        const double Xm1 = lane_prev_d(Xc), lm1 = lane_prev_d(lc);
        const bool face_ok = BCX == BC_PERIODIC || (x >= 0 && x <= kp.nx);
        const double lr = (BCX == BC_PERIODIC || x <= kp.nx - 1) ? lc : 0.0;
        const double ll = (BCX == BC_PERIODIC || x >= 1) ? lm1 : 0.0;
        const double gface = face_ok ? kvx * (lr - ll) : 0.0;
        double La, Lb, gsum;
        if (kvx > 0.0) {  // inputs x-2, x-1, x; cell x takes slot 2 of face x, 1 of x+1, 0 of x+2
          const double Xm2 = lane_prev_d(Xm1);
          lim_partials(Xm1 - Xm2, Xc - Xm1, beta, La, Lb);
          const double G0 = -La * gface, G1 = (1.0 + La - Lb) * gface, G2 = Lb * gface;
          gsum = G2 + lane_next_d(G1) + lane_next_d(lane_next_d(G0));
        } else {  // inputs x-1, x, x+1; cell x takes slot 2 of face x-1, 1 of x, 0 of x+1
          const double Xp1 = lane_next_d(Xc);
          lim_partials(Xc - Xp1, Xm1 - Xc, beta, La, Lb);
          const double G0 = Lb * gface, G1 = (1.0 + La - Lb) * gface, G2 = -La * gface;
          gsum = lane_prev_d(G2) + G1 + lane_next_d(G0);
        }
        if (BCX != BC_PERIODIC) {
          // ghost columns (copies of the edge columns) hand their share to the edge column
          const double a1 = lane_prev_d(gsum), a2 = lane_prev_d(a1), b1 = lane_next_d(gsum), b2 = lane_next_d(b1);
          if (x == 0) gsum += a1 + a2;
          if (x == kp.nx - 1) gsum += b1 + b2;
        }
        out += gsum;
      }
      // relaxation: (1 - om1) lam' + sum_r mbar_r dm_r/dX
      if constexpr (D == 0) {
        const double xa2 = xa * xa;
        const double A0 = w[0] + w[1] * xa + w[3] * xa2 + w[6] * (xa2 * xa);
        const double A1 = w[2] + w[4] * xa + w[7] * xa2;
        const double A2 = w[5] + w[8] * xa;
        out += A0 + xb * (A1 + xb * (A2 + xb * w[9])) + w[10] * Lm[b][s0];
      } else {
        out += w[0] + w[1] * xa + w[2] * xb + w[3] * Lm[b][s0];
      }
      Buf<LT>::st(plane_rsrc(lam0, pl0 + b, lplane_bytes), uint32_t(c) * lrow_bytes, lvo_st, LT(out));
    }
  };

  int c = ya - 2;
  fill(std::integral_constant<int, 0>(), c);
  fill(std::integral_constant<int, 1>(), c + 1);
  fill(std::integral_constant<int, 2>(), c + 2);
  for (;;) {
    step(std::integral_constant<int, 0>(), c);
    if (++c >= yb) break;
    step(std::integral_constant<int, 1>(), c);
    if (++c >= yb) break;
    step(std::integral_constant<int, 2>(), c);
    if (++c >= yb) break;
    step(std::integral_constant<int, 3>(), c);
    if (++c >= yb) break;
  }
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
