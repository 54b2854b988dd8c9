// Column-sweep form of the fused DDF-QE DVBM step (float32 arithmetic for
// 32-bit and 16-bit storage, float64 for float64 storage).
//
// A strip of SWEEP_OWN columns is advanced by two waves that walk a range of
// rows in +y, one advancing f and the other g; a workgroup holds SWEEP_K
// adjacent strips.  The 64 lanes of a wave hold the columns x0 - 2 .. x0 + 61:
// lanes 2 .. 61 own their cells, the two lanes at each end only supply the x
// stencil of their neighbours.  The x neighbours of a population come from
// the adjacent lanes (DPP wave shifts), the y neighbours from a window of rows
// kept in registers per population plane, so every stored value is read from
// memory once per strip (the 4 overlap columns, and the 2 stencil rows below
// and above each range of rows, aside).
// While a row is being finished, each plane's next row is already in flight.
#pragma once

#include "step.h"

namespace dvbm {

constexpr int SWEEP_OWN = 60;  // cells per strip: 64 lanes minus 2 stencil lanes on each side

// A loaded value kept in a register as its stored bit pattern (the 16-bit
// formats zero-extended into a float32 register), so that the decode, and
// with it the wait for the load, happens at the value's first use rather than
// right after the load.
template <class T>
struct Bits;
template <>
struct Bits<double> {
  __device__ static double keep(double v) { return v; }
  __device__ static double decode(double b) { return b; }
};
template <>
struct Bits<float> {
  __device__ static float keep(float v) { return v; }
  __device__ static float decode(float b) { return b; }
};
template <>
struct Bits<uint16_t> {  // bfloat16: the high half of a float32
  __device__ static float keep(uint16_t v) { return __builtin_bit_cast(float, uint32_t(v)); }
  __device__ static float decode(float b) { return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, b) << 16); }
};
template <>
struct Bits<_Float16> {
  __device__ static float keep(_Float16 v) { return __builtin_bit_cast(float, uint32_t(__builtin_bit_cast(uint16_t, v))); }
  __device__ static float decode(float b) {
    return float(__builtin_bit_cast(_Float16, uint16_t(__builtin_bit_cast(uint32_t, b))));
  }
};

// Value held by lane l - 1 (l + 1) of the wave; lane 0 (63) reads 0.
__device__ inline float lane_prev(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ inline float lane_next(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ inline double lane_prev(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_mov_dpp(int(uint32_t(b)), 0x138, 0xf, 0xf, true);
  const uint32_t hi = __builtin_amdgcn_mov_dpp(int(uint32_t(b >> 32)), 0x138, 0xf, 0xf, true);
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}
__device__ inline double lane_next(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_mov_dpp(int(uint32_t(b)), 0x130, 0xf, 0xf, true);
  const uint32_t hi = __builtin_amdgcn_mov_dpp(int(uint32_t(b >> 32)), 0x130, 0xf, 0xf, true);
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// Moment exchange between the two waves of a strip: 13 float64 moments per
// lane, double-buffered by row parity so one barrier per row suffices.
struct SweepShared {
  double m[2][N_MOMENTS][64];
};

// Strips per workgroup: the 2 SWEEP_K waves of a workgroup advance SWEEP_K
// adjacent strips in lock-step (one barrier per row), so that each plane row
// is read and written as one contiguous span and the overlap columns of
// neighbouring strips are shared through the caches.
#ifndef DVBM_SWEEP_K
#define DVBM_SWEEP_K 4
#endif
constexpr int SWEEP_K = DVBM_SWEEP_K;

// Rows held per plane by the column sweep: the three rows of the stencil
// window plus RING - 3 rows in flight, so a row is requested RING - 2 rows
// before the row step that first reads it.
#ifndef DVBM_SWEEP_RING
#define DVBM_SWEEP_RING 3
#endif

// Rows [ya, yb) of the strip whose first owned column is x0, distribution D
// (0: f, 1: g); yb - ya is a positive multiple of RING.  The other
// distribution of the strip is advanced by the other wave of the workgroup,
// which shares the moments through sh.
//
// Each face value of the NND reconstruction is formed once and used by the
// two cells that share the face: in x the upwind cell's lane forms it and
// its neighbour reads it by a lane shift; in y the value of the face below
// row y is carried over from row y - 1.  Window of plane i (y-node xi_b):
// rows y-1 .. y+1 when xi_b > 0, y .. y+2 when xi_b < 0 (upwind side
// first), row y when xi_b = 0.  The window and the rows in flight behind it
// live in a ring of RING registers per plane whose roles rotate from row to
// row, so the row loop is unrolled RING times and a row's load lands
// directly in the register that the window drops: the row after the ring's
// last one (y + RING - 1 when xi_b > 0, y + RING otherwise).  The moments at
// the start of a row read every plane, so each load has RING - 2 row steps
// of the whole workgroup to arrive.
template <int SPLIT, class S, int BCX, int BCY, int PRM, int D, int RING>
__device__ inline void sweep_update(const typename S::T* __restrict__ src, typename S::T* __restrict__ dst,
                                    const KParams& kp, int x0, int ya, int yb, SweepShared& sh) {
  static_assert(RING >= 3 && RING <= 4, "three window rows, at most four in all (grids have ny >= 4)");
  using R = typename S::C;
  using T = typename S::T;
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  constexpr int N = D == 0 ? Set<SPLIT>::NF : 2;  // Grad order of this distribution
  constexpr uint32_t SZ = sizeof(T);
  using L = GH<N1>;

  const int lane = threadIdx.x & 63;
  const int x = x0 - 2 + lane;
  const bool own = lane >= 2 && lane < 62 && x < kp.nx;
  const uint32_t vo = uint32_t(wrap_any<BCX>(x, kp.nx)) * SZ;
  // stores of the stencil-only lanes go to offset 2^31, which the bounds
  // check of the buffer resource discards: every lane stores, so no branch
  // splits the memory counters.  The resource is the distribution (at most
  // 2^31 bytes) for 32/16-bit storage and the row for float64 storage,
  // whose distributions can exceed 2^31 bytes
  const uint32_t vo_st = own ? vo : 0x80000000u;
  const uint32_t row_bytes = uint32_t(kp.srow) * SZ;     // a buffer row: the Q planes side by side
  const uint32_t plane_bytes = uint32_t(kp.pitch) * SZ;  // plane i + 1 follows plane i in a row
  const uint32_t dist_bytes = uint32_t(kp.sdist) * SZ;
  const rsrc_t rsrc_src = dist_rsrc(src, D, dist_bytes);
  const rsrc_t rsrc_dst = dist_rsrc(dst, D, dist_bytes);
  const int ny = kp.ny;
  const R beta2 = R(kp.beta2);
  const R kx = R(kp.kx), ky = R(kp.ky);
  auto row = [&](int yy) -> uint32_t { return uint32_t(wrap<BCY>(yy, ny)) * row_bytes; };
  // stored bit pattern of plane i at row offset roff; Bits<T>::decode gives the stored value
  auto load = [&](int i, uint32_t roff, uint32_t lo) -> R {
    return Bits<T>::keep(Buf<T>::ld(rsrc_src, uint32_t(i) * plane_bytes + roff, lo));
  };
  // face value between c and n, upwind cell c, far-side cell u: c + L(c - u, n - c) / 4
  auto face = [&](R u, R c, R n) -> R { return c + R(0.25) * lim4(c - u, n - c, beta2); };
  // 16-bit formats: X_i = w_i (r_i + d_i), so a moment is that of w_i r_i
  // (formed here once, in float64) plus that of w_i d_i (formed per row)
  constexpr int NM = D == 0 ? 10 : 3;
  double mref[NM];
  if constexpr (S::dev) {
    double vr[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) vr[i] = D == 0 ? 1.0 : g_ref_over_w<SPLIT>(kp, i);
    half_moments_w<D, N1>(vr, mref);
  }

  // win[i][(P + r) % RING] holds ring row r at phase P = (y - ya) % RING:
  // row y - 1 + r when xi_b > 0, y + r otherwise.  A row enters the ring as
  // its bit pattern and is decoded in place at its first use (y-moving
  // planes: the face above the row two rows earlier; xi_b = 0: as the row's
  // own value)
  R win[Q][RING];
  R fbelow[Q];  // face value below the current row (planes with xi_b != 0)
  {
    // warm-up, issued in the order of first use: rows ya-2 .. ya, then the
    // stencil rows of the first row step, then the rows in flight
    R extra[Q];
#pragma unroll
    for (int dy = -2; dy <= RING - 1; ++dy) {
      const uint32_t ro = row(ya + dy);
      static_for<Q>([&](auto kc) {
        constexpr int i = decltype(kc)::value;
        constexpr double xb = L::xi(i % N1);
        if (xb > 0.0) {
          if (dy == -2) extra[i] = load(i, ro, vo);
          else if (dy <= RING - 2) win[i][dy + 1] = load(i, ro, vo);
        } else if (xb < 0.0) {
          if (dy == -1) extra[i] = load(i, ro, vo);
          else if (dy >= 0) win[i][dy] = load(i, ro, vo);
        } else if (dy >= 0) {
          win[i][dy] = load(i, ro, vo);
        }
      });
    }
    static_for<Q>([&](auto kc) {
      constexpr int i = decltype(kc)::value;
      constexpr double xb = L::xi(i % N1);
      if (xb != 0.0) {
        // window row 2 is decoded by the first row step, at its first use
        win[i][0] = Bits<T>::decode(win[i][0]);
        win[i][1] = Bits<T>::decode(win[i][1]);
        const R e = Bits<T>::decode(extra[i]);
        fbelow[i] = xb > 0.0 ? face(e, win[i][0], win[i][1]) : face(win[i][1], win[i][0], e);
      }
    });
  }

  auto row_step = [&](auto phc, int y) {
    constexpr int P = decltype(phc)::value;
    const uint32_t r_st = uint32_t(y) * row_bytes;
    const uint32_t r_pos = row(y + RING - 1), r_neg = row(y + RING);  // rows entering the ring
    // a row entering the ring is first read RING - 2 row steps later (its
    // face), or RING steps later when xi_b = 0 (its own value); near the end
    // of the range that step lies beyond yb, and the load gets the offset
    // 2^31, which the bounds check of the buffer resource answers with 0
    // and no memory access
    const uint32_t vo_face = y + RING - 2 < yb ? vo : 0x80000000u;
    const uint32_t vo_own = y + RING < yb ? vo : 0x80000000u;

    // the row's populations (stored values), their float64 moments, shared
    R cen[Q];
    static_for<Q>([&](auto kc) {
      constexpr int i = decltype(kc)::value;
      constexpr double xb = L::xi(i % N1);
      if (xb == 0.0) win[i][P] = Bits<T>::decode(win[i][P]);
      cen[i] = xb > 0.0 ? win[i][(P + 1) % RING] : win[i][P];
    });
    NodeMoments m;
    {
      double part[NM];
      if constexpr (S::dev) {
        half_moments_w<D, N1>(cen, part);
#pragma unroll
        for (int k = 0; k < NM; ++k) part[k] += mref[k];
      } else {
        half_moments<D, N1>(cen, part);
      }
      double(*xm)[64] = sh.m[y & 1];
#pragma unroll
      for (int k = 0; k < (D == 0 ? 10 : 3); ++k) xm[(D == 0 ? 0 : 10) + k][lane] = part[k];
      __syncthreads();
      m.rho = xm[0][lane]; m.jx = xm[1][lane]; m.jy = xm[2][lane];
      m.pxx = xm[3][lane]; m.pxy = xm[4][lane]; m.pyy = xm[5][lane];
      m.qxxx = xm[6][lane]; m.qxxy = xm[7][lane]; m.qxyy = xm[8][lane]; m.qyyy = xm[9][lane];
      m.g0 = xm[10][lane]; m.qgx = xm[11][lane]; m.qgy = xm[12][lane];
    }
    R bf[5][5], bg[3][3], om1;
    collision_coeffs<SPLIT, PRM, R>(m, kp, kp.om_scale, kp.Pr, bf, bg, om1);
    if constexpr (S::dev) subtract_rest<SPLIT>(bf, bg, om1, kp);  // the -om1 r term, in the coefficients
    const R keep = R(1) - om1;

    // groups of the N1 populations i = a N1 + b that share the y-node b
    static_for<N1>([&](auto gc) {
      constexpr int ybn = decltype(gc)::value;
      constexpr double xb = L::xi(ybn);
      R c[5];
#pragma unroll
      for (int p = 0; p <= 4; ++p) {
        c[p] = R(0);
        if (p > N) continue;
#pragma unroll
        for (int q = 0; p + q <= N; ++q) {
          const double h = hn(q, xb);
          if (h != 0.0) c[p] += (D == 0 ? bf[p][q] : bg[p][q]) * R(h);
        }
      }
      static_for<N1>([&](auto ac) {
        constexpr int xa = decltype(ac)::value;
        constexpr int i = xa * N1 + ybn;
        constexpr double xv = L::xi(xa);
        constexpr double w = GH<N1>::w(xa) * GH<N1>::w(ybn);
        R* wn = win[i];
        const R c0 = cen[i];
        // collision: (1 - om1) X + w_i sum_p He_p(xi_a)/p! c_p; the deviation formats work in
        // units d = X/w - r, with the rest expansion taken out of c:  d' = (1 - om1) d + sum_p He_p/p! c_p
        R xn;
        if (S::dev) {
          xn = keep * c0;
#pragma unroll
          for (int p = 0; p <= 4; ++p) {
            if (p > N) continue;
            const double h = hn(p, xv);
            if (h != 0.0) xn += R(h) * c[p];
          }
        } else {
          // the small increments are summed first and added to X once: the
          // step changes X by tens of ulps, so every rounding at X's magnitude
          // would be a sizeable share of it
          xn = -om1 * c0;
#pragma unroll
          for (int p = 0; p <= 4; ++p) {
            if (p > N) continue;
            const double h = hn(p, xv);
            if (h != 0.0) xn += R(w * h) * c[p];
          }
        }
        // advection: -(dt/dx) v_x (X_{x+1/2} - X_{x-1/2}) - (dt/dy) v_y (X_{y+1/2} - X_{y-1/2})
        R div = R(0);
        if (xv > 0.0) {
          const R fr = face(lane_prev(c0), c0, lane_next(c0));  // X_{x+1/2}
          div += kx * R(xv) * (fr - lane_prev(fr));
        } else if (xv < 0.0) {
          const R fl = face(lane_next(c0), c0, lane_prev(c0));  // X_{x-1/2}
          div += kx * R(xv) * (lane_next(fl) - fl);
        }
        if (xb != 0.0) {
          wn[(P + 2) % RING] = Bits<T>::decode(wn[(P + 2) % RING]);
          const R r0 = wn[P], r1 = wn[(P + 1) % RING], r2 = wn[(P + 2) % RING];
          const R fa = xb > 0.0 ? face(r0, r1, r2) : face(r2, r1, r0);  // X_{y+1/2}
          div += ky * R(xb) * (fa - fbelow[i]);
          fbelow[i] = fa;
        }
        // stored values and deviations share the flux form (L is homogeneous)
        if constexpr (S::dev)
          xn -= div;
        else
          xn = c0 + (xn - div);
        if constexpr (S::dev)
          Buf<T>::st(rsrc_dst, uint32_t(i) * plane_bytes + r_st, vo_st, S::enc_dev(xn));
        else if constexpr (sizeof(T) == 8)
          Buf<T>::st(row_rsrc(dst, D, dist_bytes, y, row_bytes), uint32_t(i) * plane_bytes, vo_st,
                     S::enc(xn, R(1), R(0)));
        else
          Buf<T>::st(rsrc_dst, uint32_t(i) * plane_bytes + r_st, vo_st, S::enc(xn, R(1), R(0)));
        // the window drops its first row; that register receives the row after the ring's last
        wn[P] = load(i, xb > 0.0 ? r_pos : r_neg, xb != 0.0 ? vo_face : vo_own);
      });
    });
  };

  for (int y = ya; y < yb; y += RING)
    static_for<RING>([&](auto pc) { row_step(pc, y + decltype(pc)::value); });
}

}  // namespace dvbm
