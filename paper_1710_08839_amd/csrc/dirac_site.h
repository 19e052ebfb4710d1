// Per-site pieces of the Wilson-clover operator (Sec. 2.3 of the openQ*D
// paper): link loads with the U(1) phase z^qhat, spin projection of the eight
// hops, colour multiplication, reconstruction, and the 6x6 Pauli blocks.
//
// Hop term of site x:
//   acc(x) = sum_mu [ s (1-g_mu) W(x,mu) psi(x+mu) + s' (1+g_mu) W(x-mu,mu)^dag psi(x-mu) ]
// with W = U exp(i qhat A); D psi = P psi - acc/2.  (1 -+ g_mu) has rank 2:
// with psi = (u, l) in chiral blocks,
//   (1 - g_0) psi = (c, c),          c = u + l
//   (1 + g_0) psi = (c, -c),         c = u - l
//   (1 - g_k) psi = (c, -i s_k c),   c = u + i s_k l
//   (1 + g_k) psi = (c, +i s_k c),   c = u - i s_k l
// so every hop multiplies only a two-spin half spinor by the 3x3 link.
#pragma once

#include "qxd_impl.h"

namespace qxd {

// Link of direction MU (components 9 MU .. 9 MU + 8 of K = 36) of the site
// whose block-major element base is e: the 16-byte groups that cover them.
template <int P, class T, int MU>
QXD_HD void load_link_mu(const typename St<P>::pair_t *links, uint32_t R, uint32_t e, cx<T> u[3][3]) {
  constexpr int W = VW<P>, k0 = 9 * MU, g0 = k0 / W, ng = (k0 + 8) / W - g0 + 1;
  cx<typename St<P>::comp_t> buf[ng * W];
#pragma unroll
  for (int gk = 0; gk < ng; gk++) ld_group<P>(at32(links + (g0 + gk) * W * R, e), buf + gk * W);
#pragma unroll
  for (int rc = 0; rc < 9; rc++) u[rc / 3][rc % 3] = {(T)buf[k0 - g0 * W + rc].re, (T)buf[k0 - g0 * W + rc].im};
}

// Link of direction mu (wavefront-uniform) of the site with element base e.
template <int P, class T>
QXD_HD void load_link_at(const typename St<P>::pair_t *links, const Geom &g, int mu, uint32_t e,
                         cx<T> u[3][3]) {
  const uint32_t R = (uint32_t)g.Vbh;
  switch (mu) {
    case 0: load_link_mu<P, T, 0>(links, R, e, u); break;
    case 1: load_link_mu<P, T, 1>(links, R, e, u); break;
    case 2: load_link_mu<P, T, 2>(links, R, e, u); break;
    default: load_link_mu<P, T, 3>(links, R, e, u); break;
  }
}

template <int P, class T>
QXD_HD void load_link(const typename St<P>::pair_t *links, const Geom &g, int mu, int64_t i, cx<T> u[3][3]) {
  load_link_at<P, T>(links, g, mu, g.rd.base((uint32_t)i, 36, VW<P>), u);
}

template <class T> QXD_HD void sincos_t(T x, T *s, T *c);
template <> QXD_HD void sincos_t<double>(double x, double *s, double *c) { sincos(x, s, c); }
template <> QXD_HD void sincos_t<float>(float x, float *s, float *c) { sincosf(x, s, c); }

// W = U * exp(i qhat A)
template <int P, class T>
QXD_HD void load_w(const typename St<P>::pair_t *links, const typename St<P>::real_t *angles,
                   int qhat, const Geom &g, int mu, int64_t i, cx<T> w[3][3]) {
  load_link<P, T>(links, g, mu, i, w);
  if (qhat != 0) {
    T a = (T)*at32(angles + mu * g.Vbh, g.rd.base((uint32_t)i, 4));
    T sn, cs;
    sincos_t<T>((T)qhat * a, &sn, &cs);
    cx<T> z{cs, sn};
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
      for (int c = 0; c < 3; c++) w[r][c] = w[r][c] * z;
  }
}

// acc += sign * (1 - g_mu) W psi
template <class T>
QXD_HD void hop_fwd(int mu, const cx<T> w[3][3], const cx<T> psi[4][3], T sign, cx<T> acc[4][3]) {
  cx<T> h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    switch (mu) {
      case 0: h0[c] = psi[0][c] + psi[2][c]; h1[c] = psi[1][c] + psi[3][c]; break;
      case 1: h0[c] = psi[0][c] + times_i(psi[3][c]); h1[c] = psi[1][c] + times_i(psi[2][c]); break;
      case 2: h0[c] = psi[0][c] + psi[3][c]; h1[c] = psi[1][c] - psi[2][c]; break;
      default: h0[c] = psi[0][c] + times_i(psi[2][c]); h1[c] = psi[1][c] - times_i(psi[3][c]); break;
    }
  }
  cx<T> g0[3], g1[3];
#pragma unroll
  for (int r = 0; r < 3; r++) {
    cx<T> a{0, 0}, b{0, 0};
#pragma unroll
    for (int c = 0; c < 3; c++) {
      a = fma_acc(a, w[r][c], h0[c]);
      b = fma_acc(b, w[r][c], h1[c]);
    }
    g0[r] = sign * a;
    g1[r] = sign * b;
  }
#pragma unroll
  for (int c = 0; c < 3; c++) {
    acc[0][c] = acc[0][c] + g0[c];
    acc[1][c] = acc[1][c] + g1[c];
    switch (mu) {
      case 0: acc[2][c] = acc[2][c] + g0[c]; acc[3][c] = acc[3][c] + g1[c]; break;
      case 1: acc[2][c] = acc[2][c] + times_mi(g1[c]); acc[3][c] = acc[3][c] + times_mi(g0[c]); break;
      case 2: acc[2][c] = acc[2][c] - g1[c]; acc[3][c] = acc[3][c] + g0[c]; break;
      default: acc[2][c] = acc[2][c] + times_mi(g0[c]); acc[3][c] = acc[3][c] + times_i(g1[c]); break;
    }
  }
}

// acc += sign * (1 + g_mu) W^dag psi
template <class T>
QXD_HD void hop_bwd(int mu, const cx<T> w[3][3], const cx<T> psi[4][3], T sign, cx<T> acc[4][3]) {
  cx<T> h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    switch (mu) {
      case 0: h0[c] = psi[0][c] - psi[2][c]; h1[c] = psi[1][c] - psi[3][c]; break;
      case 1: h0[c] = psi[0][c] - times_i(psi[3][c]); h1[c] = psi[1][c] - times_i(psi[2][c]); break;
      case 2: h0[c] = psi[0][c] - psi[3][c]; h1[c] = psi[1][c] + psi[2][c]; break;
      default: h0[c] = psi[0][c] - times_i(psi[2][c]); h1[c] = psi[1][c] + times_i(psi[3][c]); break;
    }
  }
  cx<T> g0[3], g1[3];
#pragma unroll
  for (int r = 0; r < 3; r++) {
    cx<T> a{0, 0}, b{0, 0};
#pragma unroll
    for (int c = 0; c < 3; c++) {
      // (W^dag)_{rc} = conj(W_{cr})
      a = fma_accc(a, w[c][r], h0[c]);
      b = fma_accc(b, w[c][r], h1[c]);
    }
    g0[r] = sign * a;
    g1[r] = sign * b;
  }
#pragma unroll
  for (int c = 0; c < 3; c++) {
    acc[0][c] = acc[0][c] + g0[c];
    acc[1][c] = acc[1][c] + g1[c];
    switch (mu) {
      case 0: acc[2][c] = acc[2][c] - g0[c]; acc[3][c] = acc[3][c] - g1[c]; break;
      case 1: acc[2][c] = acc[2][c] + times_i(g1[c]); acc[3][c] = acc[3][c] + times_i(g0[c]); break;
      case 2: acc[2][c] = acc[2][c] + g1[c]; acc[3][c] = acc[3][c] - g0[c]; break;
      default: acc[2][c] = acc[2][c] + times_i(g0[c]); acc[3][c] = acc[3][c] - times_i(g1[c]); break;
    }
  }
}

// Packed Hermitian 6x6: pairs 0-2 diagonal (d0,d1),(d2,d3),(d4,d5); pairs
// 3-17 upper triangle row by row.
QXD_HD constexpr int tri_index(int i, int j) { return i * 6 - i * (i + 1) / 2 + (j - i - 1); }

// out = A v for the packed Hermitian block BLK (pairs 18 BLK .. 18 BLK + 17
// of K = 36) of site j, read as the 16-byte groups that cover them.
template <int P, class T, bool NT, int BLK>
QXD_HD void herm6_mul(const typename St<P>::pair_t *pa, const Geom &g, int64_t j, const cx<T> v[6],
                      cx<T> out[6]) {
  constexpr int W = VW<P>, k0 = 18 * BLK, g0 = k0 / W, ng = (k0 + 17) / W - g0 + 1;
  const uint32_t e = g.rd.base((uint32_t)j, 36, W), R = (uint32_t)g.Vbh;
  cx<typename St<P>::comp_t> buf[ng * W];
#pragma unroll
  for (int gk = 0; gk < ng; gk++) ld_group<P, NT>(at32(pa + (g0 + gk) * W * R, e), buf + gk * W);
  auto ldp = [&](int pair) { return buf[k0 - g0 * W + pair]; };
  T d[6];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    auto z = ldp(k);
    d[2 * k] = (T)z.re;
    d[2 * k + 1] = (T)z.im;
  }
#pragma unroll
  for (int i = 0; i < 6; i++) out[i] = d[i] * v[i];
#pragma unroll
  for (int i = 0; i < 6; i++)
#pragma unroll
    for (int k = i + 1; k < 6; k++) {
      auto z = ldp(3 + tri_index(i, k));
      cx<T> a{(T)z.re, (T)z.im};
      out[i] = fma_acc(out[i], a, v[k]);
      out[k] = fma_accc(out[k], a, v[i]);
    }
}

// out = P psi with both chiral blocks; j indexes the sites the array covers
// (all sites for P, the odd sites j = i - V/2 for D_oo^-1).
template <int P, class T, bool NT = false>
QXD_HD void pauli_mul(const typename St<P>::pair_t *pa, const Geom &g, int64_t j,
                      const cx<T> psi[4][3], cx<T> out[4][3]) {
#pragma unroll
  for (int blk = 0; blk < 2; blk++) {
    cx<T> v[6], o[6];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      v[c] = psi[2 * blk][c];
      v[3 + c] = psi[2 * blk + 1][c];
    }
    if (blk == 0)
      herm6_mul<P, T, NT, 0>(pa, g, j, v, o);
    else
      herm6_mul<P, T, NT, 1>(pa, g, j, v, o);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      out[2 * blk][c] = o[c];
      out[2 * blk + 1][c] = o[3 + c];
    }
  }
}

// One hop of site s (native index i): dir = +1 adds (1 - g_mu) W(x,mu)
// psi(x+mu), dir = -1 adds (1 + g_mu) W(x-mu,mu)^dag psi(x-mu).
template <int P, class T>
QXD_HD void hop_one(const Geom &g, const typename St<P>::pair_t *links,
                    const typename St<P>::real_t *angles, int qhat, const Spinor<P> &in,
                    const Site &s, int64_t i, int mu, int dir, cx<T> acc[4][3]) {
  int sg;
  Site t = neighbour(g, s, mu, dir, sg);
  int64_t j = encode(g, t);
  cx<T> psi[4][3], w[3][3];
  load_spinor<P, T>(in, j, psi);
  load_w<P, T>(links, angles, qhat, g, mu, dir > 0 ? i : j, w);
  if (dir > 0)
    hop_fwd<T>(mu, w, psi, (T)sg, acc);
  else
    hop_bwd<T>(mu, w, psi, (T)sg, acc);
}

// Hop sum acc(x) over the eight neighbours of site s (native index i).  The
// hops are issued GROUP at a time (GROUP = 1, 2, 4 or 8): larger groups keep
// more loads in flight per wavefront, smaller ones use fewer registers and
// allow more wavefronts per SIMD.
template <int P, class T, int GROUP = 2>
QXD_HD void hop_sum(const Geom &g, const typename St<P>::pair_t *links,
                    const typename St<P>::real_t *angles, int qhat, const Spinor<P> &in,
                    const Site &s, int64_t i, cx<T> acc[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 3; c++) acc[a][c] = {0, 0};
#pragma unroll 1
  for (int k0 = 0; k0 < 8; k0 += GROUP) {
#pragma unroll
    for (int k = k0; k < k0 + GROUP; k++)
      hop_one<P, T>(g, links, angles, qhat, in, s, i, k >> 1, (k & 1) ? -1 : 1, acc);
  }
}

}  // namespace qxd
