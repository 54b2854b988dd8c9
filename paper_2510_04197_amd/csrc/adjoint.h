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

template <int BC>
__device__ inline bool face_exists(int f, int n) {
  return BC == BC_PERIODIC ? true : (f >= 0 && f <= n);
}

// Flux-part cotangent of one population along one axis for cell c.
//   Xs[k]   = population at cell map(c - 3 + k), k = 0..6 (decoded);
//   lam[k]  = lam' at cell map(c - 2 + k), k = 0..4;
//   kv      = (dt / dx) v_alpha (non-zero); F(c) = ... - kv (face(c+1) - face(c)).
// Face f lies between cells f-1 and f; with v > 0 its inputs are f-2, f-1, f
// and the faces that read cell c are c, c+1, c+2 (c in slots 2, 1, 0); with
// v < 0 the inputs are f-1, f, f+1 and the faces are c-1, c, c+1.  Under the
// zero-gradient rule the ghost inputs are copies of the edge cell, so at an
// edge cell further slots of the same faces map to it.
template <int BC>
__device__ inline double flux_adjoint(const double* Xs, const double* lam, int c, int n, double kv, double beta) {
  double acc = 0.0;
  const int d0 = kv > 0.0 ? 0 : -1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int df = d0 + k;  // face f = c + df
    const int f = c + df;
    if (BC != BC_PERIODIC && (f < 0 || f > n)) continue;
    // dL/dface(f) = kv (lam'(f) - lam'(f-1)); cells outside a zero-gradient domain carry no lam'
    const double lr = (BC == BC_PERIODIC || f <= n - 1) ? lam[df + 2] : 0.0;
    const double ll = (BC == BC_PERIODIC || f >= 1) ? lam[df + 1] : 0.0;
    const double gface = kv * (lr - ll);
    const int q0 = kv > 0.0 ? df - 2 : df - 1;  // first input of face f, relative to c
    const double X0 = Xs[q0 + 3], X1 = Xs[q0 + 4], X2 = Xs[q0 + 5];
    double La, Lb, p0, p1, p2;
    if (kv > 0.0) {
      lim_partials(X1 - X0, X2 - X1, beta, La, Lb);
      p0 = -La;
      p1 = 1.0 + La - Lb;
      p2 = Lb;
    } else {
      lim_partials(X1 - X2, X0 - X1, beta, La, Lb);
      p0 = Lb;
      p1 = 1.0 + La - Lb;
      p2 = -La;
    }
    const double ps[3] = {p0, p1, p2};
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int q = c + q0 + sl;
      bool hit;
      if (BC == BC_PERIODIC)
        hit = n > 6 ? q == c : wrap_any<BC>(q, n) == c;
      else
        hit = q == c || (c == 0 && q < 0) || (c == n - 1 && q >= n);
      if (hit) acc += gface * ps[sl];
    }
  }
  return acc;
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
//   flux:  one wave per (population plane, row, strip of cells) assembles
//          lam(c) = (1 - om1) lam'(c) + sum_r mbar_r dm_r/dX + flux cotangent.
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
      const double lf = lam1[int64_t(i) * cells + c], lg = lam1[int64_t(Q + i) * cells + c];
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

// lam for plane pl, row y, strip x0 (one wave): the relaxation part from
// the work array plus the flux cotangent.  The x stencil comes from the
// neighbouring lanes, the y stencil from memory.
template <int SPLIT, class S, int BCX, int BCY>
__device__ inline void strip_adjoint_flux(const typename S::T* __restrict__ state, const double* __restrict__ lam1,
                                          const double* __restrict__ work, double* __restrict__ lam0,
                                          const KParams& kp, int pl, int x0, int y) {
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  using L = GH<N1>;
  const int64_t cells = int64_t(kp.nx) * kp.ny;
  const int lane = threadIdx.x & 63;
  const int x = x0 - 3 + lane;
  const bool own = lane >= 3 && lane < 61 && x < kp.nx;
  const int gx = wrap_any<BCX>(x, kp.nx);
  const int d = pl / Q, i = pl % Q;
  const double xa = L::xi(i / N1), xb = L::xi(i % N1);
  const double* lp = lam1 + int64_t(pl) * cells;
  const double beta = 0.5 * kp.beta2;
  double out = 0.0;
  if (xa != 0.0) {  // plane-uniform: every lane takes part in the lane shifts
    // lane l forms face f = x (between x-1 and x) once: G_s = dL/dface * dface/d(input s)
    const double kv = kp.kx * xa;
    const double Xc = adj_X<SPLIT, S>(state, kp, d, i, y, gx);
    const double lc = lp[int64_t(y) * kp.nx + gx];
    const double Xm1 = lane_prev_d(Xc), lm1 = lane_prev_d(lc);
    const bool face_ok = BCX == BC_PERIODIC || (x >= 0 && x <= kp.nx);
    const double lr = (BCX == BC_PERIODIC || x <= kp.nx - 1) ? lc : 0.0;
    const double ll = (BCX == BC_PERIODIC || x >= 1) ? lm1 : 0.0;
    const double gface = face_ok ? kv * (lr - ll) : 0.0;
    double La, Lb, G0, G1, G2;
    if (kv > 0.0) {  // inputs x-2, x-1, x
      const double Xm2 = lane_prev_d(Xm1);
      lim_partials(Xm1 - Xm2, Xc - Xm1, beta, La, Lb);
      G0 = -La * gface;
      G1 = (1.0 + La - Lb) * gface;
      G2 = Lb * gface;
    } else {  // inputs x-1, x, x+1
      const double Xp1 = lane_next_d(Xc);
      lim_partials(Xc - Xp1, Xm1 - Xc, beta, La, Lb);
      G0 = Lb * gface;
      G1 = (1.0 + La - Lb) * gface;
      G2 = -La * gface;
    }
    // cell x gathers slot 2 of face x, 1 of x+1, 0 of x+2 (v > 0) or
    // slot 2 of face x-1, 1 of x, 0 of x+1 (v < 0)
    double gx_sum;
    if (kv > 0.0)
      gx_sum = G2 + lane_next_d(G1) + lane_next_d(lane_next_d(G0));
    else
      gx_sum = lane_prev_d(G2) + G1 + lane_next_d(G0);
    if (BCX != BC_PERIODIC) {
      // ghost cells (copies of the edge cells) hand their share to the edge cell
      const double a1 = lane_prev_d(gx_sum), a2 = lane_prev_d(a1), b1 = lane_next_d(gx_sum), b2 = lane_next_d(b1);
      if (x == 0) gx_sum += a1 + a2;
      if (x == kp.nx - 1) gx_sum += b1 + b2;
    }
    out += gx_sum;
  }
  if (!own) return;
  if (xb != 0.0) {
    double Xs[7], lm[5];
#pragma unroll
    for (int k = 0; k < 7; ++k) Xs[k] = adj_X<SPLIT, S>(state, kp, d, i, wrap<BCY>(y - 3 + k, kp.ny), x);
#pragma unroll
    for (int k = 0; k < 5; ++k) lm[k] = lp[int64_t(wrap<BCY>(y - 2 + k, kp.ny)) * kp.nx + x];
    out += flux_adjoint<BCY>(Xs, lm, y, kp.ny, kp.ky * xb, beta);
  }
  // relaxation part: (1 - om1) lam' + sum_r mbar_r dm_r/dX
  const int64_t c = int64_t(y) * kp.nx + x;
  auto mb = [&](int r) { return work[int64_t(r) * cells + c]; };
  out += mb(N_MOMENTS) * lp[c];
  if (d == 0) {
    const double xa2 = xa * xa, xb2 = xb * xb;
    out += mb(0) + mb(1) * xa + mb(2) * xb + mb(3) * xa2 + mb(4) * (xa * xb) + mb(5) * xb2 + mb(6) * (xa2 * xa) +
           mb(7) * (xa2 * xb) + mb(8) * (xa * xb2) + mb(9) * (xb2 * xb);
  } else {
    out += mb(10) + mb(11) * xa + mb(12) * xb;
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
