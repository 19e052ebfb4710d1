// Direction-generic form of one hop of the Wilson term (Sec. 2.3 of the
// openQ*D paper), for kernels in which neighbouring lanes of a wavefront hop
// in different directions mu and a switch over mu would serialise them.
//
// In the chiral basis every g_mu maps the upper spins {0, 1} onto the lower
// spins {2, 3}.  Writing p_a (a = 0, 1) for the lower spin that g_mu pairs
// with upper spin a and k_a for a unit complex number,
//   upper part of (1 - g_mu) psi:  c_a = psi_a + k_a psi_{p_a}
//   lower part:                    spin p_a = conj(k_a) c_a
// and (1 + g_mu) flips the sign of both k_a terms.  The pairs are
//   mu = 0: p = (2, 3), k = ( 1,  1)
//   mu = 1: p = (3, 2), k = ( i,  i)
//   mu = 2: p = (3, 2), k = ( 1, -1)
//   mu = 3: p = (2, 3), k = ( i, -i)
// which reproduces the projections of hop_fwd / hop_bwd term by term.  With
// k_a = s_a or i s_a (s_a = +-1), multiplying by k_a is a swap of real and
// imaginary part and a sign, done with selects and fused multiply-adds.
#pragma once

#include "qxd_impl.h"

namespace qxd {

struct SpinProj {
  int p0;       // lower spin paired with upper spin 0 (2 or 3); p1 = 5 - p0
  bool imag;    // k_a imaginary (mu odd)
  float s0, s1; // k_a = s_a (real) or i s_a (imaginary), s_a = +-1
};

QXD_HD SpinProj spin_proj(int mu) {
  SpinProj s;
  s.p0 = (mu == 1 || mu == 2) ? 3 : 2;
  s.imag = mu & 1;
  s.s0 = 1.f;
  s.s1 = mu >= 2 ? -1.f : 1.f;
  return s;
}

// u + sg k z for a unit k = s or i s (two selects, two fused multiply-adds)
template <class T>
QXD_HD cx<T> add_unit(cx<T> u, bool imag, T sg, cx<T> z) {
  T a = imag ? z.im : z.re, b = imag ? z.re : z.im;
  return {fmat(imag ? -sg : sg, a, u.re), fmat(sg, b, u.im)};
}
// sg conj(k) z for a unit k = s or i s
template <class T>
QXD_HD cx<T> mul_unit_conj(bool imag, T sg, cx<T> z) {
  T a = imag ? z.im : z.re, b = imag ? z.re : z.im;
  return {sg * a, (imag ? -sg : sg) * b};
}

// One hop in direction mu:
//   SIGN = +1:  (1 - g_mu) W psi          (forward hop)
//   SIGN = -1:  (1 + g_mu) W^dag psi      (backward hop)
// given the upper spins u0, u1 of psi and its spins q0 = psi_{p0},
// q1 = psi_{p1}.  The result is added to (INIT: written into) au (upper
// spins 0, 1) and al (al[a] = lower spin p_a, i.e. in the lane's own order;
// lower_to_spins maps it back).
template <int SIGN, bool INIT, class T>
QXD_HD void hop_generic(const SpinProj &sp, const cx<T> w[3][3], const cx<T> u0[3], const cx<T> u1[3],
                        const cx<T> q0[3], const cx<T> q1[3], cx<T> au[2][3], cx<T> al[2][3]) {
  const T g0s = (T)(SIGN * sp.s0), g1s = (T)(SIGN * sp.s1);
  cx<T> h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    h0[c] = add_unit(u0[c], sp.imag, g0s, q0[c]);
    h1[c] = add_unit(u1[c], sp.imag, g1s, q1[c]);
  }
#pragma unroll
  for (int r = 0; r < 3; r++) {
    cx<T> a{0, 0}, b{0, 0};
    if (SIGN > 0) {
      a = w[r][0] * h0[0];
      b = w[r][0] * h1[0];
#pragma unroll
      for (int c = 1; c < 3; c++) {
        a = fma_acc(a, w[r][c], h0[c]);
        b = fma_acc(b, w[r][c], h1[c]);
      }
    } else {
      a = cmulc(w[0][r], h0[0]);
      b = cmulc(w[0][r], h1[0]);
#pragma unroll
      for (int c = 1; c < 3; c++) {
        a = fma_accc(a, w[c][r], h0[c]);
        b = fma_accc(b, w[c][r], h1[c]);
      }
    }
    cx<T> l0 = mul_unit_conj(sp.imag, g0s, a), l1 = mul_unit_conj(sp.imag, g1s, b);
    if (INIT) {
      au[0][r] = a;
      au[1][r] = b;
      al[0][r] = l0;
      al[1][r] = l1;
    } else {
      au[0][r] = au[0][r] + a;
      au[1][r] = au[1][r] + b;
      al[0][r] = al[0][r] + l0;
      al[1][r] = al[1][r] + l1;
    }
  }
}

// A hop whose direction is chosen at run time: w is W (forward, sg = +1) or
// W^dag (backward, sg = -1), and the projector is (1 - sg g_mu).  Writes
// (au, al) as hop_generic<SIGN, true> does.
template <class T>
QXD_HD void hop_generic_dir(const SpinProj &sp, T sg, const cx<T> w[3][3], const cx<T> u0[3], const cx<T> u1[3],
                            const cx<T> q0[3], const cx<T> q1[3], cx<T> au[2][3], cx<T> al[2][3]) {
  const T g0s = sg * (T)sp.s0, g1s = sg * (T)sp.s1;
  cx<T> h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    h0[c] = add_unit(u0[c], sp.imag, g0s, q0[c]);
    h1[c] = add_unit(u1[c], sp.imag, g1s, q1[c]);
  }
#pragma unroll
  for (int r = 0; r < 3; r++) {
    cx<T> a = w[r][0] * h0[0], b = w[r][0] * h1[0];
#pragma unroll
    for (int c = 1; c < 3; c++) {
      a = fma_acc(a, w[r][c], h0[c]);
      b = fma_acc(b, w[r][c], h1[c]);
    }
    au[0][r] = a;
    au[1][r] = b;
    al[0][r] = mul_unit_conj(sp.imag, g0s, a);
    al[1][r] = mul_unit_conj(sp.imag, g1s, b);
  }
}

// (au, al) of hop_generic -> acc[4][3] in spin order
template <class T>
QXD_HD void lower_to_spins(const SpinProj &sp, const cx<T> au[2][3], const cx<T> al[2][3], cx<T> acc[4][3]) {
  const bool sw = sp.p0 == 3;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    acc[0][c] = au[0][c];
    acc[1][c] = au[1][c];
    acc[2][c] = sw ? al[1][c] : al[0][c];
    acc[3][c] = sw ? al[0][c] : al[1][c];
  }
}

}  // namespace qxd
