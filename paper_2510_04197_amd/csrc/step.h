// One fused DDF-QE DVBM update of a single cell (device code shared by the
// step kernel): decode, moments, two-time QE relaxation, NND flux
// divergence, encode.
#pragma once

#include "node.h"

namespace dvbm {

// Rest reference of the deviation formats, divided by the weight.
template <int SPLIT>
__device__ inline double g_ref_over_w(const KParams& kp, int i) {
  using L = GH<Set<SPLIT>::N1>;
  constexpr int N1 = Set<SPLIT>::N1;
  const double xa = L::xi(i / N1), xb = L::xi(i % N1);
  return kp.gr0 + kp.gr1 * (xa * xa + xb * xb - 2.0);
}

template <int SPLIT>
__device__ inline double weight(int i) {
  using L = GH<Set<SPLIT>::N1>;
  constexpr int N1 = Set<SPLIT>::N1;
  return L::w(i / N1) * L::w(i % N1);
}

template <int BC>
__device__ inline int wrap(int j, int n) {
  if (BC == BC_PERIODIC) return j < 0 ? j + n : (j >= n ? j - n : j);
  return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// One time step of Eq. (finalDiscretePDE) for the cell (x, y): reads the
// populations of the cell and its flux stencil from src, writes the cell's
// new populations to dst.
template <int SPLIT, class S, int BCX, int BCY, int PRM>
__device__ inline void cell_update(const typename S::T* __restrict__ src, typename S::T* __restrict__ dst,
                                   const KParams& kp, int x, int y) {
  using R = typename S::C;
  using T = typename S::T;
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  using L = GH<N1>;

  const int xm2 = wrap<BCX>(x - 2, kp.nx), xm1 = wrap<BCX>(x - 1, kp.nx);
  const int xp1 = wrap<BCX>(x + 1, kp.nx), xp2 = wrap<BCX>(x + 2, kp.nx);
  const int64_t r0 = int64_t(y) * kp.pitch;
  const int64_t rm2 = int64_t(wrap<BCY>(y - 2, kp.ny)) * kp.pitch;
  const int64_t rm1 = int64_t(wrap<BCY>(y - 1, kp.ny)) * kp.pitch;
  const int64_t rp1 = int64_t(wrap<BCY>(y + 1, kp.ny)) * kp.pitch;
  const int64_t rp2 = int64_t(wrap<BCY>(y + 2, kp.ny)) * kp.pitch;

  R xf[Q], xg[Q];  // stored values (deviation units for the 16-bit formats)
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    xf[i] = S::raw(src[int64_t(i) * kp.plane + r0 + x]);
    xg[i] = S::raw(src[int64_t(Q + i) * kp.plane + r0 + x]);
  }
  R f[Q], g[Q];  // decoded populations
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (S::dev) {
      const double w = weight<SPLIT>(i);
      f[i] = R(w) * (R(1) + xf[i]);
      g[i] = R(w) * (R(g_ref_over_w<SPLIT>(kp, i)) + xg[i]);
    } else {
      f[i] = xf[i];
      g[i] = xg[i];
    }
  }

  const NodeMoments m = node_moments<N1>(f, g);
  R bf[5][5], bg[3][3], om1;
  collision_coeffs<SPLIT, PRM, R>(m, kp, bf, bg, om1);

  // collision: (1 - om1) X + expansion of b
  const R keep = R(1) - om1;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    f[i] *= keep;
    g[i] *= keep;
  }
  expand_add<N1, Set<SPLIT>::NF>(bf, f);
  expand_add<N1, 2>(bg, g);

  // advection: -(dt/dx) v_x (X_{x+1/2} - X_{x-1/2}) - (dt/dy) v_y (X_{y+1/2} - X_{y-1/2})
  const R beta2 = R(kp.beta2);
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double xa = L::xi(i / N1), xb = L::xi(i % N1);
      const T* pl = src + int64_t(d * Q + i) * kp.plane;
      const R c0 = d == 0 ? xf[i] : xg[i];
      R div = R(0);
      if (xa > 0.0) {
        div += R(kp.kx * xa) * dface_pos(S::raw(pl[r0 + xm2]), S::raw(pl[r0 + xm1]), c0, S::raw(pl[r0 + xp1]), beta2);
      } else if (xa < 0.0) {
        div += R(kp.kx * xa) * dface_neg(S::raw(pl[r0 + xm1]), c0, S::raw(pl[r0 + xp1]), S::raw(pl[r0 + xp2]), beta2);
      }
      if (xb > 0.0) {
        div += R(kp.ky * xb) * dface_pos(S::raw(pl[rm2 + x]), S::raw(pl[rm1 + x]), c0, S::raw(pl[rp1 + x]), beta2);
      } else if (xb < 0.0) {
        div += R(kp.ky * xb) * dface_neg(S::raw(pl[rm1 + x]), c0, S::raw(pl[rp1 + x]), S::raw(pl[rp2 + x]), beta2);
      }
      const double w = weight<SPLIT>(i);
      const R rr = S::dev ? R(d == 0 ? 1.0 : g_ref_over_w<SPLIT>(kp, i)) : R(0);
      const R xnew = (d == 0 ? f[i] : g[i]) - (S::dev ? R(w) * div : div);
      dst[int64_t(d * Q + i) * kp.plane + r0 + x] = S::enc(xnew, R(1.0 / w), rr);
    }
  }
}

}  // namespace dvbm
