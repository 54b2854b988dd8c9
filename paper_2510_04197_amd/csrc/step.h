// One fused DDF-QE DVBM update of a single cell (device code shared by the
// step kernel): decode, moments, two-time QE relaxation, NND flux
// divergence, encode.
#pragma once

#include <utility>

#include "node.h"

namespace dvbm {

// Rest reference of the deviation formats, divided by the weight.
template <int SPLIT>
__device__ inline double g_ref_over_w(const KParams& kp, int i) {
  using L = GH<Set<SPLIT>::N1>;
  constexpr int N1 = Set<SPLIT>::N1;
  const double xa = L::xi(i / N1), xb = L::xi(i % N1);
  if (SPLIT == 2) return kp.gr0;  // the rest g of split II carries no |xi|^2 term
  return kp.gr0 + kp.gr1 * (xa * xa + xb * xb - 2.0);
}

template <int SPLIT>
__device__ inline double weight(int i) {
  using L = GH<Set<SPLIT>::N1>;
  constexpr int N1 = Set<SPLIT>::N1;
  return L::w(i / N1) * L::w(i % N1);
}

// Float64 moments of one cell's populations X = w (r + d) stored as
// deviations d (units of w): those of w d, with the weights in the float64
// coefficients of the sums, plus those of the rest state w r, so that a state
// at rest has exactly the rest moments (decoding X in float32 first would
// round w r).  The rest state's moments are the Gauss-Hermite rule's exact
// low-order moments: rho = 1 and P = delta for f (r = 1); for g, g0 = gr0 in
// both splits (in split I the |xi|^2 - 2 part of r has weighted mean 0) and a
// zero first moment.
template <int SPLIT, class R>
__device__ inline NodeMoments dev_moments(const R* df, const R* dg, const KParams& kp) {
  constexpr int N1 = Set<SPLIT>::N1;
  double a[10], b[3];
  half_moments_w<0, N1>(df, a);
  half_moments_w<1, N1>(dg, b);
  NodeMoments m;
  m.rho = a[0] + 1.0; m.jx = a[1]; m.jy = a[2];
  m.pxx = a[3] + 1.0; m.pxy = a[4]; m.pyy = a[5] + 1.0;
  m.qxxx = a[6]; m.qxxy = a[7]; m.qxyy = a[8]; m.qyyy = a[9];
  m.g0 = b[0] + kp.gr0; m.qgx = b[1]; m.qgy = b[2];
  return m;
}

template <int BC>
__device__ inline int wrap(int j, int n) {
  if (BC == BC_PERIODIC) return j < 0 ? j + n : (j >= n ? j - n : j);
  return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// One time step of Eq. (finalDiscretePDE) for the cell (x, y): reads the
// populations of the cell and its flux stencil from src, writes the cell's
// new populations to dst.
// Each distribution (Q planes) is addressed through one buffer resource
// (wave-uniform, < 4 GiB), a scalar per-plane offset and a 32-bit per-lane
// byte offset, so the address arithmetic stays out of the vector ALU.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int RSRC_WORD3 = 0x00020000;  // 32-bit data format, raw (untyped) access

__device__ inline rsrc_t dist_rsrc(const void* base, int d, uint32_t dist_bytes) {
  const char* p = static_cast<const char*>(base) + size_t(d) * size_t(dist_bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), 0, dist_bytes, RSRC_WORD3);
}

// One dense plane (index pl) of a cotangent array as its own buffer
// resource: the stencil-only lanes of the adjoint sweep store to offset 2^31,
// beyond any plane, and the row offset plus 2^31 stays below 2^32.
__device__ inline rsrc_t plane_rsrc(const void* base, int pl, uint32_t plane_bytes) {
  const char* p = static_cast<const char*>(base) + size_t(pl) * size_t(plane_bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), 0, plane_bytes, RSRC_WORD3);
}

// Row y of distribution d of a population buffer (its Q planes side by side)
// as its own buffer resource: the stencil-only lanes of the column sweep
// store to offset 2^31, beyond any row, also where a distribution exceeds
// 2^31 bytes (float64 storage).
__device__ inline rsrc_t row_rsrc(const void* base, int d, uint32_t dist_bytes, int y, uint32_t row_bytes) {
  const char* p = static_cast<const char*>(base) + size_t(d) * size_t(dist_bytes) + size_t(y) * size_t(row_bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), 0, row_bytes, RSRC_WORD3);
}

template <class T>
struct Buf;
template <>
struct Buf<float> {
  __device__ static float ld(rsrc_t r, uint32_t so, uint32_t o) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o, so, 0));
  }
  __device__ static void st(rsrc_t r, uint32_t so, uint32_t o, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, o, so, 0);
  }
};
template <>
struct Buf<double> {
  __device__ static double ld(rsrc_t r, uint32_t so, uint32_t o) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, o, so, 0));
  }
  __device__ static void st(rsrc_t r, uint32_t so, uint32_t o, double v) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, o, so, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, o, so, 0);
  }
};
template <>
struct Buf<uint16_t> {
  __device__ static uint16_t ld(rsrc_t r, uint32_t so, uint32_t o) { return __builtin_amdgcn_raw_buffer_load_b16(r, o, so, 0); }
  __device__ static void st(rsrc_t r, uint32_t so, uint32_t o, uint16_t v) { __builtin_amdgcn_raw_buffer_store_b16(v, r, o, so, 0); }
};
template <>
struct Buf<_Float16> {
  __device__ static _Float16 ld(rsrc_t r, uint32_t so, uint32_t o) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, o, so, 0));
  }
  __device__ static void st(rsrc_t r, uint32_t so, uint32_t o, _Float16 v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, o, so, 0);
  }
};

// Compile-time loop: f(std::integral_constant<int, k>) for k = 0 .. N-1.
template <class F, int... K>
__device__ inline void static_for_impl(F&& f, std::integer_sequence<int, K...>) {
  (f(std::integral_constant<int, K>{}), ...);
}
template <int N, class F>
__device__ inline void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// One time step of Eq. (finalDiscretePDE) for the cell (x, y), one thread
// per cell: the cell's 2Q populations stay in registers (moments, then the
// collision of each population), the flux stencil of every population is
// read through the vector L1/L2 caches.
template <int SPLIT, class S, int BCX, int BCY, int PRM>
__device__ inline void cell_update(const typename S::T* __restrict__ src, typename S::T* __restrict__ dst,
                                   const KParams& kp, int x, int y,
                                   const typename S::T* __restrict__ ghost = nullptr) {
  using R = typename S::C;
  using T = typename S::T;
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  constexpr uint32_t SZ = sizeof(T);
  using L = GH<N1>;

  const uint32_t srow = uint32_t(kp.srow);  // a buffer row: the Q planes of one distribution
  const uint32_t row0 = uint32_t(y) * srow;
  const uint32_t o0 = (row0 + uint32_t(x)) * SZ;
  const uint32_t oxm2 = (row0 + uint32_t(wrap<BCX>(x - 2, kp.nx))) * SZ;
  const uint32_t oxm1 = (row0 + uint32_t(wrap<BCX>(x - 1, kp.nx))) * SZ;
  const uint32_t oxp1 = (row0 + uint32_t(wrap<BCX>(x + 1, kp.nx))) * SZ;
  const uint32_t oxp2 = (row0 + uint32_t(wrap<BCX>(x + 2, kp.nx))) * SZ;
  const uint32_t oym2 = (uint32_t(wrap<BCY>(y - 2, kp.ny)) * srow + uint32_t(x)) * SZ;
  const uint32_t oym1 = (uint32_t(wrap<BCY>(y - 1, kp.ny)) * srow + uint32_t(x)) * SZ;
  const uint32_t oyp1 = (uint32_t(wrap<BCY>(y + 1, kp.ny)) * srow + uint32_t(x)) * SZ;
  const uint32_t oyp2 = (uint32_t(wrap<BCY>(y + 2, kp.ny)) * srow + uint32_t(x)) * SZ;
  const uint32_t plane_bytes = uint32_t(kp.pitch) * SZ;  // plane i + 1 follows plane i in a row
  const uint32_t dist_bytes = uint32_t(kp.sdist) * SZ;
  const rsrc_t rsrc_src[2] = {dist_rsrc(src, 0, dist_bytes), dist_rsrc(src, 1, dist_bytes)};
  const rsrc_t rsrc_dst[2] = {dist_rsrc(dst, 0, dist_bytes), dist_rsrc(dst, 1, dist_bytes)};

  R xs[2][Q];  // stored values (deviation units for the 16-bit formats)
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int i = 0; i < Q; ++i) xs[d][i] = S::raw(Buf<T>::ld(rsrc_src[d], i * plane_bytes, o0));
  NodeMoments m;
  if constexpr (S::dev)
    m = dev_moments<SPLIT>(xs[0], xs[1], kp);
  else
    m = node_moments<N1>(xs[0], xs[1]);
  R X[2][Q];  // the increment of each population
  R bf[5][5], bg[3][3], om1;
  collision_coeffs<SPLIT, PRM, R>(m, kp, kp.om_scale, kp.Pr, bf, bg, om1);

  // collision: (1 - om1) X + expansion of b.  X then holds the increment,
  // added to the stored value once at the end (one rounding at the stored
  // value's magnitude): -om1 X + expansion for values, and in deviation units
  // d = X / w - r,  -om1 d + expansion / w of b less om1 times the rest
  // coefficients (subtract_rest) for the deviation formats.
  if constexpr (S::dev) subtract_rest<SPLIT>(bf, bg, om1, kp);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    X[0][i] = -om1 * xs[0][i];
    X[1][i] = -om1 * xs[1][i];
  }
  expand_add<N1, Set<SPLIT>::NF, R, 5, !S::dev>(bf, X[0]);
  expand_add<N1, 2, R, 3, !S::dev>(bg, X[1]);

  // advection: -(dt/dx) v_x (X_{x+1/2} - X_{x-1/2}) - (dt/dy) v_y (X_{y+1/2} - X_{y-1/2})
  const R beta2 = R(kp.beta2);
  const R kx = R(kp.kx), ky = R(kp.ky);
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double xa = L::xi(i / N1), xb = L::xi(i % N1);
      const rsrc_t pl = rsrc_src[d];
      const uint32_t so = i * plane_bytes;
      const R c0 = xs[d][i];
      R div = R(0);
      if (xa > 0.0)
        div += kx * R(xa) * dface_pos(S::raw(Buf<T>::ld(pl, so, oxm2)), S::raw(Buf<T>::ld(pl, so, oxm1)), c0,
                                        S::raw(Buf<T>::ld(pl, so, oxp1)), beta2);
      else if (xa < 0.0)
        div += kx * R(xa) * dface_neg(S::raw(Buf<T>::ld(pl, so, oxm1)), c0, S::raw(Buf<T>::ld(pl, so, oxp1)),
                                        S::raw(Buf<T>::ld(pl, so, oxp2)), beta2);
      // value of the plane at row y + dy; with walls, rows outside the domain
      // come from the ghost rows (ghost[(d Q + i) 4 + r][x], r = 0..3 for the
      // rows -2, -1, ny, ny+1)
      auto ly = [&](uint32_t off, int dy) -> R {
        if constexpr (BCY == BC_WALL) {
          const int yy = y + dy;
          if (yy < 0 || yy >= kp.ny) {
            const int gr = yy < 0 ? yy + 2 : yy - kp.ny + 2;
            return S::raw(ghost[(int64_t(d * Q + i) * 4 + gr) * kp.pitch + x]);
          }
        }
        return S::raw(Buf<T>::ld(pl, so, off));
      };
      if (xb > 0.0)
        div += ky * R(xb) * dface_pos(ly(oym2, -2), ly(oym1, -1), c0, ly(oyp1, 1), beta2);
      else if (xb < 0.0)
        div += ky * R(xb) * dface_neg(ly(oym1, -1), c0, ly(oyp1, 1), ly(oyp2, 2), beta2);
      // the flux of the deviations is that of the values over w (the
      // reconstruction commutes with shifts and scalings)
      const R xnew = c0 + (X[d][i] - div);
      if constexpr (S::dev)
        Buf<T>::st(rsrc_dst[d], so, o0, S::enc_dev(xnew));
      else
        Buf<T>::st(rsrc_dst[d], so, o0, S::enc(xnew, R(1), R(0)));
    }
  }
}

// Neighbour index under the boundary rule, for any integer j.
template <int BC>
__device__ inline int wrap_any(int j, int n) {
  if (BC == BC_PERIODIC) {
    const int r = j % n;
    return r < 0 ? r + n : r;
  }
  return j < 0 ? 0 : (j >= n ? n - 1 : j);
}

// Halo slot s of a (TX + 4) x (TY + 4) tile region (two ghost layers on
// every side): rows 0-1 full, then the two left / two right columns of the
// TY interior rows, then rows TY+2, TY+3 full.
template <int TX, int TY>
__device__ inline void halo_slot(int s, int& hy, int& hx) {
  constexpr int W = TX + 4;
  if (s < 2 * W) {
    hy = s / W;
    hx = s % W;
    return;
  }
  s -= 2 * W;
  if (s < 4 * TY) {
    const int c = s % 4;
    hy = 2 + s / 4;
    hx = c < 2 ? c : TX + c;
    return;
  }
  s -= 4 * TY;
  hy = TY + 2 + s / W;
  hx = s % W;
}

// LDS staging area: G population planes, each the tile plus two ghost
// layers, double-buffered so that one barrier per group of G suffices.
template <class R, int TX, int TY, int G>
struct PlaneTile {
  R v[2][G][TY + 4][TX + 4];
};

// One time step of Eq. (finalDiscretePDE) for the TX x TY cells of tile
// (bx, by), one thread per cell.  Pass 1 reads the cell's 2Q populations
// (coalesced rows) and builds the relaxation coefficients from float64
// moments.  Pass 2 walks the populations: each plane's tile and ghost layers
// are staged in LDS (own value from registers, ghosts from global memory),
// and every thread reads its flux stencil from LDS.  Threads of a partial
// tile hold the values of their wrapped / clamped cells so that every staged
// entry is the one the stencil needs; they store nothing.
template <int SPLIT, class S, int BCX, int BCY, int PRM, int TX, int TY>
__device__ inline void tile_update(const typename S::T* __restrict__ src, typename S::T* __restrict__ dst,
                                   const KParams& kp, int bx, int by,
                                   PlaneTile<typename S::C, TX, TY, Set<SPLIT>::N1>& lds) {
  using R = typename S::C;
  using T = typename S::T;
  constexpr int N1 = Set<SPLIT>::N1;
  constexpr int Q = Set<SPLIT>::Q;
  constexpr int NF = Set<SPLIT>::NF;
  constexpr uint32_t SZ = sizeof(T);
  constexpr int NT = TX * TY;
  constexpr int NH = (TX + 4) * (TY + 4) - TX * TY;
  constexpr int H = (NH + NT - 1) / NT;
  using L = GH<N1>;

  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int x = bx * TX + tx, y = by * TY + ty;
  const bool valid = x < kp.nx && y < kp.ny;
  const uint32_t srow = uint32_t(kp.srow);  // a buffer row: the Q planes of one distribution
  const uint32_t o0 =
      (uint32_t(wrap_any<BCY>(y, kp.ny)) * srow + uint32_t(wrap_any<BCX>(x, kp.nx))) * SZ;
  uint32_t hoff[H];
  int hidx[H];
  bool hval[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const int s = tid + j * NT;
    hval[j] = s < NH;
    int hy = 0, hx = 0;
    if (hval[j]) halo_slot<TX, TY>(s, hy, hx);
    const int gx = wrap_any<BCX>(bx * TX + hx - 2, kp.nx);
    const int gy = wrap_any<BCY>(by * TY + hy - 2, kp.ny);
    hoff[j] = (uint32_t(gy) * srow + uint32_t(gx)) * SZ;
    hidx[j] = hy * (TX + 4) + hx;
  }
  const uint32_t plane_bytes = uint32_t(kp.pitch) * SZ;  // plane i + 1 follows plane i in a row
  const uint32_t dist_bytes = uint32_t(kp.sdist) * SZ;
  const rsrc_t rsrc_src[2] = {dist_rsrc(src, 0, dist_bytes), dist_rsrc(src, 1, dist_bytes)};
  const rsrc_t rsrc_dst[2] = {dist_rsrc(dst, 0, dist_bytes), dist_rsrc(dst, 1, dist_bytes)};

  // Pass 1: the cell's populations (kept in registers for pass 2) and their
  // float64 moments.
  R xs[2][Q];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int i = 0; i < Q; ++i) xs[d][i] = S::raw(Buf<T>::ld(rsrc_src[d], i * plane_bytes, o0));
  NodeMoments m;
  if constexpr (S::dev)
    m = dev_moments<SPLIT>(xs[0], xs[1], kp);
  else
    m = node_moments<N1>(xs[0], xs[1]);
  R bf[5][5], bg[3][3], om1;
  collision_coeffs<SPLIT, PRM, R>(m, kp, kp.om_scale, kp.Pr, bf, bg, om1);
  if constexpr (S::dev) subtract_rest<SPLIT>(bf, bg, om1, kp);  // the -om1 r term, in the coefficients
  const R beta2 = R(kp.beta2);
  const R kx = R(kp.kx), ky = R(kp.ky);

  // Pass 2: groups gk = d N1 + b of the N1 populations i = a N1 + b that share
  // the y-node b (so the Grad expansion factors into
  // sum_p w_a He_p(xi_a)/p! c_p(b)).  A group's planes are staged in LDS with
  // one barrier; the loads of group gk + 1 are issued before that barrier.
  constexpr int W = TX + 4;
  constexpr int PL = (TY + 4) * W;
  constexpr int NMAX = 4;
  const int me = (ty + 2) * W + tx + 2;
  R curh[N1][H];
  auto fetch = [&](int gk, R (&h)[N1][H]) {
    const int d = gk / N1, yb = gk % N1;
#pragma unroll
    for (int xa = 0; xa < N1; ++xa) {
      const uint32_t so = (xa * N1 + yb) * plane_bytes;
#pragma unroll
      for (int j = 0; j < H; ++j) h[xa][j] = hval[j] ? S::raw(Buf<T>::ld(rsrc_src[d], so, hoff[j])) : R(0);
    }
  };
  fetch(0, curh);
  static_for<2 * N1>([&](auto gc) {
    constexpr int gk = decltype(gc)::value;
    constexpr int d = gk / N1, yb = gk % N1;
    constexpr int N = d == 0 ? NF : 2;
    constexpr double xb = L::xi(yb);
    R c[NMAX + 1];
#pragma unroll
    for (int p = 0; p <= NMAX; ++p) {
      c[p] = R(0);
      if (p > N) continue;
#pragma unroll
      for (int q = 0; p + q <= N; ++q) {
        const double h = hn(q, xb);
        if (h != 0.0) c[p] += (d == 0 ? bf[p][q] : bg[p][q]) * R(h);
      }
    }
#pragma unroll
    for (int xa = 0; xa < N1; ++xa) {
      R* buf = &lds.v[gk & 1][xa][0][0];
      buf[me] = xs[d][xa * N1 + yb];
#pragma unroll
      for (int j = 0; j < H; ++j)
        if (hval[j]) buf[hidx[j]] = curh[xa][j];
    }
    if (gk + 1 < 2 * N1) fetch(gk + 1, curh);
    __syncthreads();

    static_for<N1>([&](auto ac) {
      constexpr int xa = decltype(ac)::value;
      constexpr int i = xa * N1 + yb;
      constexpr double xv = L::xi(xa);
      constexpr double w = GH<N1>::w(xa) * GH<N1>::w(yb);
      const R* buf = &lds.v[gk & 1][xa][0][0];
      const R c0 = xs[d][i];
      const uint32_t so = i * plane_bytes;
      // collision: (1 - om1) X + w_i sum_p He_p(xi_a)/p! c_p.  The increment
      // is summed first and added to the stored value once: -om1 X + ... for
      // values, -om1 d + sum_p He_p c_p in deviation units d = X/w - r (the
      // rest expansion taken out of c by subtract_rest)
      R xn = -om1 * c0;
      constexpr double wx = S::dev ? 1.0 : w;
#pragma unroll
      for (int p = 0; p <= NMAX; ++p) {
        if (p > N) continue;
        const double h = hn(p, xv);
        if (h != 0.0) xn += R(wx * h) * c[p];
      }
      // advection: -(dt/dx) v_x (X_{x+1/2} - X_{x-1/2}) - (dt/dy) v_y (X_{y+1/2} - X_{y-1/2})
      R div = R(0);
      if (xv > 0.0)
        div += kx * R(xv) * dface_pos(buf[me - 2], buf[me - 1], c0, buf[me + 1], beta2);
      else if (xv < 0.0)
        div += kx * R(xv) * dface_neg(buf[me - 1], c0, buf[me + 1], buf[me + 2], beta2);
      if (xb > 0.0)
        div += ky * R(xb) * dface_pos(buf[me - 2 * W], buf[me - W], c0, buf[me + W], beta2);
      else if (xb < 0.0)
        div += ky * R(xb) * dface_neg(buf[me - W], c0, buf[me + W], buf[me + 2 * W], beta2);
      xn = c0 + (xn - div);  // deviations share the flux form of the values (over w)
      if (valid) {
        if constexpr (S::dev)
          Buf<T>::st(rsrc_dst[d], so, o0, S::enc_dev(xn));
        else
          Buf<T>::st(rsrc_dst[d], so, o0, S::enc(xn, R(1), R(0)));
      }
    });
  });
  (void)PL;
}

}  // namespace dvbm
