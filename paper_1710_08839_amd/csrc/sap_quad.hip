// SAP block solves with four lanes per site pair (reduced precisions).
//
// The arithmetic is that of the block solver in sap.hip (face update, MR on
// the even-odd preconditioned block operator with Dirichlet boundaries, odd
// reconstruction); only the distribution of the work differs.  Lane rho =
// 0..3 of quad h serves even site h and odd site h of the block (h-th site of
// each parity in native order):
//   * it computes the forward and the backward hop of direction mu = rho;
//   * it holds spin component rho of the site vectors (residual, MR
//     iterate, correction);
//   * it holds rows 3(rho&1) .. 3(rho&1)+2 of chiral block rho>>1 of the
//     Pauli term (P on the even site, D_oo^-1 on the odd site), i.e. exactly
//     the rows that produce spin rho.
// The four partial hop sums of a site are combined with DPP quad
// permutations (no LDS round trip, no barrier): first the two chiral blocks
// are exchanged between lanes rho and rho^2, then the two halves of a block
// between lanes rho and rho^1, so that both lanes of a chiral block end with
// bit-identical sums.  All lanes work in both half steps, and the links and
// Pauli rows of the block stay in registers for the whole block solve; LDS
// holds only the two spinor buffers exchanged between the parities.
#include <atomic>

#include "dirac_site.h"
#include "hop_generic.h"
#include "sap.h"

namespace qxd {

namespace {

constexpr int QP_XOR1 = 0xB1;  // DPP quad_perm(1,0,3,2)
constexpr int QP_XOR2 = 0x4E;  // DPP quad_perm(2,3,0,1)

template <int CTRL>
__device__ __forceinline__ float qperm(float v) {
  // bound_ctrl set: the source lane is always in the same quad, and the four
  // lanes of a quad (one site pair) are active together, so no lane reads a
  // disabled one; it lets the compiler fold the move into the add that uses it
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ cx<float> qperm(cx<float> z) {
  return {qperm<CTRL>(z.re), qperm<CTRL>(z.im)};
}

__device__ __forceinline__ cx<float> csel(bool c, cx<float> a, cx<float> b) { return c ? a : b; }

// Sum over the quad of the partial hop sums acc[4][3]; returns chiral block
// b = rho >> 1 of the total (out[0] = spin 2b, out[1] = spin 2b+1).
__device__ __forceinline__ void quad_sum_block(const cx<float> acc[4][3], bool b, cx<float> out[2][3]) {
#pragma unroll
  for (int s = 0; s < 2; s++)
#pragma unroll
    for (int c = 0; c < 3; c++) {
      cx<float> keep = csel(b, acc[2 + s][c], acc[s][c]);
      cx<float> send = csel(b, acc[s][c], acc[2 + s][c]);
      keep = keep + qperm<QP_XOR2>(send);
      out[s][c] = keep + qperm<QP_XOR1>(keep);
    }
}

// Chiral block of a vector held as one spin per lane: out[0] = spin 2b,
// out[1] = spin 2b+1.
__device__ __forceinline__ void quad_block_of(const cx<float> v[3], bool rh, cx<float> out[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; c++) {
    cx<float> o = qperm<QP_XOR1>(v[c]);
    out[0][c] = csel(rh, o, v[c]);
    out[1][c] = csel(rh, v[c], o);
  }
}

template <int P>
__device__ __forceinline__ cx<float> unpack(typename St<P>::pair_t v) {
  return St<P>::ld(&v, 0);
}
template <int P>
__device__ __forceinline__ typename St<P>::pair_t zero_pair() {
  typename St<P>::pair_t z;
  St<P>::st(&z, 0, cx<float>{0.f, 0.f});
  return z;
}

// Rows of the lane: out[r] = sum_j m[r][j] x[j], x = chiral block (6 entries).
// The rows stay packed between uses: the empty asm makes each use read the
// packed register, so the compiler cannot hoist the unpacked values (twice
// the registers) out of the MR loop.
template <int P>
__device__ __forceinline__ void rows_mul(typename St<P>::pair_t m[3][6], const cx<float> x[2][3],
                                         cx<float> out[3]) {
#pragma unroll
  for (int r = 0; r < 3; r++) {
    cx<float> a{0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 6; j++) {
      __asm__ volatile("" : "+v"(m[r][j]));
      a = fma_acc(a, unpack<P>(m[r][j]), x[j / 3][j % 3]);
    }
    out[r] = a;
  }
}

// Rows 3 rh + r (r = 0..2) of chiral block b of a packed Hermitian Pauli
// field at site j (layout: pairs 18 b + 0..2 real diagonal, 18 b + 3.. upper
// triangle), kept in storage precision: the diagonal entry (d, 0) and the
// conjugates below the diagonal are exact in every storage format.
template <int P>
__device__ __forceinline__ void load_rows(const typename St<P>::pair_t *pa, const Geom &g, uint32_t j, int b,
                                          int rh, typename St<P>::pair_t m[3][6]) {
  constexpr int W = VW<P>;
  const uint32_t e = g.rd.base(j, 36, W);
#pragma unroll
  for (int r = 0; r < 3; r++) {
    const int i = 3 * rh + r;
#pragma unroll
    for (int k = 0; k < 6; k++) {
      const int lo = i < k ? i : k, hi = i < k ? k : i;
      const int pair = 18 * b + (i == k ? (i >> 1) : 3 + tri_index(lo, hi));
      cx<float> z = gld_pair<P>(pa + g.rd.comp_off(pair, W), e);
      cx<float> e;
      if (i == k)
        e = {(i & 1) ? z.im : z.re, 0.f};
      else
        e = {z.re, k > i ? z.im : -z.im};
      St<P>::st(&m[r][k], 0, e);
    }
  }
}

// Spin a (three colours) of a stored spinor at native site i.
template <int P>
__device__ __forceinline__ void load_spin(const Spinor<P> &s, int64_t i, int a, cx<float> out[3]) {
  const uint32_t j = (uint32_t)(i - s.off);
  constexpr int W = VW<P>;
  const uint32_t e = s.rd.base(j, 12, W);
#pragma unroll
  for (int c = 0; c < 3; c++) out[c] = gld_pair<P>(s.data + s.rd.comp_off(a * 3 + c, W), e);
  if constexpr (St<P>::scaled) {
    float f = gld(s.scale, j);
#pragma unroll
    for (int c = 0; c < 3; c++) out[c] = f * out[c];
  }
}

// Store spin a of a site whose four spins are held by the four lanes of the
// quad (all four lanes call this together).  With per-site scales the scale is
// the largest modulus of a real or imaginary part over all 24 reals, as for a
// whole-site store.
template <int P>
__device__ __forceinline__ void store_spin(const Spinor<P> &s, int64_t i, int a, const cx<float> v[3], bool act) {
  const uint32_t j = (uint32_t)(i - s.off);
  constexpr int W = VW<P>;
  const uint32_t e = s.rd.base(j, 12, W);
  float f = 1.f;
  if constexpr (St<P>::scaled) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 3; c++) {
      m = fmaxf(m, fabsf(v[c].re));
      m = fmaxf(m, fabsf(v[c].im));
    }
    m = fmaxf(m, qperm<QP_XOR1>(m));
    m = fmaxf(m, qperm<QP_XOR2>(m));
    if (act && a == 0) gst(s.scale, j, m);
    f = m > 0.f ? 1.0f / m : 0.f;
  }
  if (act) {
#pragma unroll
    for (int c = 0; c < 3; c++)
      gst_pair<P>(s.data + s.rd.comp_off(a * 3 + c, W), e, cx<float>{f * v[c].re, f * v[c].im});
  }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// LDS plane strides are compile-time constants sized for the largest block
// (128 sites of each parity), so that every LDS access is one base register
// plus an immediate offset.  Spinor planes: 128 + 8 complex (the four spin
// planes written by the 32 lanes of a half wavefront fall into disjoint
// banks); link planes: 256 sites + the zero slot, rounded up.
constexpr int QNH_MAX = 128;
constexpr int QNHP = QNH_MAX + 8;
constexpr int QVBP = 2 * QNH_MAX + 4;
constexpr int QZERO = 2 * QNH_MAX;  // zero-link slot

// LDS: per right-hand side two spinor buffers and the reduction scratch (one
// triple per wavefront, at most 8), then the links (shared)
__host__ __device__ constexpr size_t qspin_bytes() { return 2 * 12 * (size_t)QNHP * sizeof(cx<float>); }
__host__ __device__ constexpr size_t qlinks_offset(int nr) {
  return (size_t)nr * (qspin_bytes() + 3 * 8 * sizeof(float));
}

__device__ __forceinline__ int local_lex(const Geom &g, const Site &t) {
  return ((t.y(0) * g.b[1] + t.y(1)) * g.b[2] + t.y(2)) * g.b[3] + t.y(3);
}

// NR right-hand sides (1 or 2) that share the operator are solved on the
// same block by one work-group: the links and Pauli rows are staged once, the
// barriers are shared, and the two solves give independent work between
// barriers.  Each right-hand side's arithmetic is the same as when it is
// solved alone.
template <int P, int NR>
__device__ __forceinline__ void sapq_body(const Geom &g, const SapOp<P> &a, const SapVecs<P> *vvs, int blk,
                                          int first, int skip_face, int nmr, unsigned char *smem) {
  using T = float;
  const int nh = g.Vbh;
  constexpr int nhp = QNHP;
  cx<T> *bufe[NR], *bufo[NR];  // per right-hand side: even- and odd-site vector [12][nhp]
  T *red[NR];
#pragma unroll
  for (int q = 0; q < NR; q++) {
    bufe[q] = (cx<T> *)(smem + q * qspin_bytes());
    bufo[q] = bufe[q] + 12 * nhp;
    red[q] = (T *)(smem + NR * qspin_bytes()) + q * 24;
  }
  using pt = typename St<P>::pair_t;
  pt *lw = (pt *)(smem + qlinks_offset(NR));
  const int tid = threadIdx.x;
  const int h = tid >> 2, rho = tid & 3, mu = rho;
  const bool bb = rho >> 1, rh = rho & 1;
  const bool act = h < nh;
  const int nwaves = (int)(blockDim.x >> 6);
  const SpinProj sp = spin_proj(mu);
  const int p1 = 5 - sp.p0;

  // the lane's even (x = 0) and odd (x = 1) site
  Site st[2];
  {
    int B = blk;
    int B3 = B % g.nb[3];
    B /= g.nb[3];
    int B2 = B % g.nb[2];
    B /= g.nb[2];
    int B1 = B % g.nb[1];
    int B0 = B / g.nb[1];
    int hh = act ? h : 0;
    int q = hh / g.hb3;
    int y3h = hh - q * g.hb3;
    int y2 = q % g.b[2];
    q /= g.b[2];
    int y1 = q % g.b[1];
    int y0 = q / g.b[1];
#pragma unroll
    for (int x = 0; x < 2; x++) {
      st[x].p = x;
      st[x].Bp = pack4(B0, B1, B2, B3);
      st[x].yp = pack4(y0, y1, y2, 2 * y3h + ((x + y0 + y1 + y2) & 1));
    }
  }
  const int64_t ie = (int64_t)blk * nh + (act ? h : 0);
  const int64_t isite[2] = {ie, (int64_t)g.Vh + ie};
  const int bmu = (int)((g.bpk >> (8 * mu)) & 0xff);

  // Links of the block in LDS, [36 (mu, entry)][vbp] in storage precision
  // and indexed by local lexicographic site index; slot vb holds a zero link.
  // A link whose forward neighbour lies outside the block is stored as zero:
  // no in-block hop uses it, and the hops that leave the block read the zero
  // slot, so that every lane runs the same instructions.  Lane (h, mu) loads
  // the links of direction mu of its two sites.
  constexpr int vb = QZERO, vbp = QVBP;
  int lf[2], lb[2], nf[2], nbk[2];
#pragma unroll
  for (int x = 0; x < 2; x++) {
    const int y = st[x].y(mu);
    const bool fin = act && y + 1 < bmu, bin = act && y > 0;
    int sg;
    Site tf = neighbour(g, st[x], mu, 1, sg);
    Site tb = neighbour(g, st[x], mu, -1, sg);
    const int lx = local_lex(g, st[x]);
    nf[x] = fin ? (encode(g, tf) - (1 - x) * g.Vh - blk * nh) : (act ? h : 0);
    nbk[x] = bin ? (encode(g, tb) - (1 - x) * g.Vh - blk * nh) : (act ? h : 0);
    lf[x] = fin ? lx : vb;
    lb[x] = bin ? local_lex(g, tb) : vb;
    if (act) {
      const uint32_t el = g.rd.base((uint32_t)isite[x], 36, VW<P>);
#pragma unroll
      for (int k = 0; k < 9; k++) {
        pt z = gld(a.links, el + g.rd.comp_off(mu * 9 + k, VW<P>));
        lw[(mu * 9 + k) * vbp + lx] = fin ? z : zero_pair<P>();
      }
    }
  }
  if (tid < 36) lw[tid * vbp + vb] = zero_pair<P>();
  // Pauli rows: P on the even site, D_oo^-1 on the odd site
  pt m[2][3][6];
  load_rows<P>(a.pauli, g, (uint32_t)(act ? isite[0] : 0), bb, rh, m[0]);
  load_rows<P>(a.pinv, g, (uint32_t)(act ? ie : 0), bb, rh, m[1]);

  // in-block hops of direction mu of the lane's site of parity x, from the
  // other parity's vector in LDS; partial sums over the quad
  auto hops = [&](const cx<T> *src, int x, cx<T> acc[4][3]) {
    cx<T> u0[3], u1[3], q0[3], q1[3], w[3][3], au[2][3], al[2][3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
      u0[c] = src[(0 * 3 + c) * nhp + nf[x]];
      u1[c] = src[(1 * 3 + c) * nhp + nf[x]];
      q0[c] = src[(sp.p0 * 3 + c) * nhp + nf[x]];
      q1[c] = src[(p1 * 3 + c) * nhp + nf[x]];
    }
#pragma unroll
    for (int k = 0; k < 9; k++) w[k / 3][k % 3] = unpack<P>(lw[(mu * 9 + k) * vbp + lf[x]]);
    hop_generic<1, true, T>(sp, w, u0, u1, q0, q1, au, al);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      u0[c] = src[(0 * 3 + c) * nhp + nbk[x]];
      u1[c] = src[(1 * 3 + c) * nhp + nbk[x]];
      q0[c] = src[(sp.p0 * 3 + c) * nhp + nbk[x]];
      q1[c] = src[(p1 * 3 + c) * nhp + nbk[x]];
    }
#pragma unroll
    for (int k = 0; k < 9; k++) w[k / 3][k % 3] = unpack<P>(lw[(mu * 9 + k) * vbp + lb[x]]);
    hop_generic<-1, false, T>(sp, w, u0, u1, q0, q1, au, al);
    lower_to_spins(sp, au, al, acc);
  };
  auto lds_put = [&](cx<T> *dst, const cx<T> v[3]) {
    if (act) {
#pragma unroll
      for (int c = 0; c < 3; c++) dst[(rho * 3 + c) * nhp + h] = v[c];
    }
  };

  // residual with the face update r -= D v' over the hops that leave the block
  cx<T> r[NR][2][3];
#pragma unroll
  for (int q = 0; q < NR; q++)
#pragma unroll
    for (int x = 0; x < 2; x++) {
      if (act)
        load_spin<P>(first ? vvs[q].rho : vvs[q].r, isite[x], rho, r[q][x]);
      else
#pragma unroll
        for (int c = 0; c < 3; c++) r[q][x][c] = {0.f, 0.f};
    }
  if (!skip_face) {
#pragma unroll
    for (int x = 0; x < 2; x++) {
      // at most one hop of direction mu leaves the block (b_mu >= 2); every
      // lane runs the same instructions, lanes without a face hop read their
      // own site and discard it (select, not a product with zero: the other
      // colour's corrections may not be written yet where no face hop reads)
      const int y = st[x].y(mu);
      const int dir = y == bmu - 1 ? 1 : (y == 0 ? -1 : 0);
      const bool face = act && dir != 0;
      int sg = 0;
      const Site t = neighbour(g, st[x], mu, dir < 0 ? -1 : 1, sg);
      const int64_t j = face ? (int64_t)encode(g, t) : isite[x];
      const uint32_t el = g.rd.base((uint32_t)(dir < 0 && face ? j : isite[x]), 36, VW<P>);
      cx<T> wl[3][3], w[3][3];
#pragma unroll
      for (int k = 0; k < 9; k++) wl[k / 3][k % 3] = gld_pair<P>(a.links + g.rd.comp_off(mu * 9 + k, VW<P>), el);
      // backward hop: W(x - mu, mu)^dag
#pragma unroll
      for (int rr = 0; rr < 3; rr++)
#pragma unroll
        for (int c = 0; c < 3; c++) w[rr][c] = dir < 0 ? conj(wl[c][rr]) : wl[rr][c];
#pragma unroll
      for (int q = 0; q < NR; q++) {
        const Spinor<P> &vq = vvs[q].v;
        const uint32_t jv = (uint32_t)(j - vq.off), ev = vq.rd.base(jv, 12, VW<P>);
        const T f = (T)sg * (St<P>::scaled ? gld(vq.scale, jv) : (T)1);
        const cx<T> z0{0.f, 0.f};
        cx<T> u0[3], u1[3], q0[3], q1[3], au[2][3], al[2][3], acc[4][3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
          u0[c] = csel(face, f * gld_pair<P>(vq.data + vq.rd.comp_off(c, VW<P>), ev), z0);
          u1[c] = csel(face, f * gld_pair<P>(vq.data + vq.rd.comp_off(3 + c, VW<P>), ev), z0);
          q0[c] = csel(face, f * gld_pair<P>(vq.data + vq.rd.comp_off(sp.p0 * 3 + c, VW<P>), ev), z0);
          q1[c] = csel(face, f * gld_pair<P>(vq.data + vq.rd.comp_off(p1 * 3 + c, VW<P>), ev), z0);
        }
        hop_generic_dir<T>(sp, dir < 0 ? (T)-1 : (T)1, w, u0, u1, q0, q1, au, al);
        lower_to_spins(sp, au, al, acc);
        cx<T> blkv[2][3];
        quad_sum_block(acc, bb, blkv);
#pragma unroll
        for (int c = 0; c < 3; c++) r[q][x][c] = r[q][x][c] + (T)0.5 * csel(rh, blkv[1][c], blkv[0][c]);
      }
    }
  }
  // u_o = D_oo^-1 r_o
#pragma unroll
  for (int q = 0; q < NR; q++) {
    cx<T> xb[2][3], u[3];
    quad_block_of(r[q][1], rh, xb);
    rows_mul<P>(m[1], xb, u);
    lds_put(bufo[q], u);
  }
  __syncthreads();
  // s = rho_e = r_e - D_eo^L u_o = r_e + acc_in(u)/2; v_e = 0
  cx<T> s[NR][3], v[NR][3];
#pragma unroll
  for (int q = 0; q < NR; q++) {
    cx<T> acc[4][3], blkv[2][3];
    hops(bufo[q], 0, acc);
    quad_sum_block(acc, bb, blkv);
#pragma unroll
    for (int c = 0; c < 3; c++) {
      s[q][c] = r[q][0][c] + (T)0.5 * csel(rh, blkv[1][c], blkv[0][c]);
      v[q][c] = {0.f, 0.f};
    }
    lds_put(bufe[q], s[q]);
  }
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < nmr; k++) {
    // w_o = D_oo^-1 D_oe^L s = -D_oo^-1 acc_in(s)/2
#pragma unroll
    for (int q = 0; q < NR; q++) {
      cx<T> acc[4][3], blkv[2][3], w[3];
      hops(bufe[q], 1, acc);
      quad_sum_block(acc, bb, blkv);
#pragma unroll
      for (int e = 0; e < 2; e++)
#pragma unroll
        for (int c = 0; c < 3; c++) blkv[e][c] = (T)(-0.5) * blkv[e][c];
      rows_mul<P>(m[1], blkv, w);
      lds_put(bufo[q], w);
    }
    __syncthreads();
    // t = P s - D_eo^L w_o = P s + acc_in(w)/2; alpha = (t,s)/(t,t)
    cx<T> t[NR][3];
#pragma unroll
    for (int q = 0; q < NR; q++) {
      cx<T> acc[4][3], blkv[2][3], sb[2][3];
      hops(bufo[q], 0, acc);
      quad_sum_block(acc, bb, blkv);
      quad_block_of(s[q], rh, sb);
      rows_mul<P>(m[0], sb, t[q]);
#pragma unroll
      for (int c = 0; c < 3; c++) t[q][c] = t[q][c] + (T)0.5 * csel(rh, blkv[1][c], blkv[0][c]);
      T ts_re = 0, ts_im = 0, tt = 0;
      if (act) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
          cx<T> z = cmulc(t[q][c], s[q][c]);
          ts_re += z.re;
          ts_im += z.im;
          tt += norm2(t[q][c]);
        }
      }
      ts_re = wave_sum(ts_re);
      ts_im = wave_sum(ts_im);
      tt = wave_sum(tt);
      if ((tid & 63) == 0) {
        red[q][3 * (tid >> 6)] = ts_re;
        red[q][3 * (tid >> 6) + 1] = ts_im;
        red[q][3 * (tid >> 6) + 2] = tt;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NR; q++) {
      T sr = 0, si = 0, stt = 0;
      for (int w = 0; w < nwaves; w++) {
        sr += red[q][3 * w];
        si += red[q][3 * w + 1];
        stt += red[q][3 * w + 2];
      }
      cx<T> alpha{0.f, 0.f};
      if (stt > (T)0) alpha = {sr / stt, si / stt};
#pragma unroll
      for (int c = 0; c < 3; c++) {
        v[q][c] = v[q][c] + alpha * s[q][c];
        s[q][c] = s[q][c] - alpha * t[q][c];
      }
      lds_put(bufe[q], s[q]);
    }
    __syncthreads();
  }
  // v_o = D_oo^-1 (r_o - D_oe^L v_e) = D_oo^-1 (r_o + acc_in(v_e)/2)
#pragma unroll
  for (int q = 0; q < NR; q++) lds_put(bufo[q], v[q]);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NR; q++) {
    cx<T> vo[3];
    {
      cx<T> acc[4][3], blkv[2][3], rb[2][3];
      hops(bufo[q], 1, acc);
      quad_sum_block(acc, bb, blkv);
      quad_block_of(r[q][1], rh, rb);
#pragma unroll
      for (int e = 0; e < 2; e++)
#pragma unroll
        for (int c = 0; c < 3; c++) rb[e][c] = rb[e][c] + (T)0.5 * blkv[e][c];
      rows_mul<P>(m[1], rb, vo);
    }
    // psi += v; residual on the block: r_e = s, r_o = 0; keep v for the faces
    const SapVecs<P> &vv = vvs[q];
    const cx<T> *vx[2] = {v[q], vo};
#pragma unroll
    for (int x = 0; x < 2; x++) {
      cx<T> p[3];
      if (first) {
#pragma unroll
        for (int c = 0; c < 3; c++) p[c] = vx[x][c];
      } else {
        if (act)
          load_spin<P>(vv.psi, isite[x], rho, p);
        else
#pragma unroll
          for (int c = 0; c < 3; c++) p[c] = {0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 3; c++) p[c] = p[c] + vx[x][c];
      }
      store_spin<P>(vv.psi, isite[x], rho, p, act);
      store_spin<P>(vv.v, isite[x], rho, vx[x], act);
    }
    cx<T> zero[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
    store_spin<P>(vv.r, isite[0], rho, s[q], act);
    store_spin<P>(vv.r, isite[1], rho, zero, act);
  }
}

template <int P>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
sapq_block_kernel(SapArgs<P> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  SapOp<P> op{a.links, a.angles, a.qhat, a.pauli, a.pinv};
  SapVecs<P> vv{a.rho, a.r, a.psi, a.v};
  sapq_body<P, 1>(a.g, op, &vv, a.blocks[xcd_order(blockIdx.x, gridDim.x)], a.first, a.skip_face, a.nmr, smem);
}

template <int P>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
sapq_batch_kernel(Geom g, const int *blocks, const SapSlot<P> *slots, const int *act, int nact, int first,
                  int skip_face, int nmr) {
  extern __shared__ __align__(16) unsigned char smem[];
  int L = xcd_order(blockIdx.x, gridDim.x);
  int bi = L / nact;
  const SapSlot<P> &sl = slots[act[L - bi * nact]];
  sapq_body<P, 1>(g, sl.op, &sl.vec, blocks[bi], first, skip_face, nmr, smem);
}

// Pairs of right-hand sides with the same operator: work-group L solves block
// L / npair for the two slots pairs[2 (L % npair)], pairs[2 (L % npair) + 1].
template <int P>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
sapq_pair_kernel(Geom g, const int *blocks, const SapSlot<P> *slots, const int *pairs, int npair, int first,
                 int skip_face, int nmr) {
  extern __shared__ __align__(16) unsigned char smem[];
  int L = xcd_order(blockIdx.x, gridDim.x);
  int bi = L / npair;
  int pi = L - bi * npair;
  const SapSlot<P> &s0 = slots[pairs[2 * pi]];
  SapVecs<P> vv[2] = {s0.vec, slots[pairs[2 * pi + 1]].vec};
  sapq_body<P, 2>(g, s0.op, vv, blocks[bi], first, skip_face, nmr, smem);
}

int quad_threads(const Geom &g) { return (4 * g.Vbh + 63) / 64 * 64; }

size_t quad_lds(int prec, const Geom &, int nr = 1) {
  return qlinks_offset(nr) + 36 * (size_t)QVBP * pair_bytes(prec);
}

}  // namespace

static int lds_limit() {
  static int limit = -1;
  if (limit < 0) {
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
    limit = v;
  }
  return limit;
}

bool sap_quad_ok(int prec, const Geom &g, int qhat) {
  return prec != QXD_F64 && qhat == 0 && g.Vbh <= QNH_MAX && quad_lds(prec, g) <= (size_t)lds_limit();
}

// Raise a kernel's dynamic LDS limit once (the largest size asked for so far
// per kernel), so that launches issued under graph capture make no
// attribute calls.
template <auto Kernel>
static hipError_t allow_lds(size_t lds) {
  static std::atomic<size_t> granted{65536};
  if (lds <= granted.load()) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)Kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess) granted.store(lds);
  return e;
}

template <int P>
hipError_t launch_sapq_colour(const SapArgs<P> &a, int nblocks_colour, hipStream_t st) {
  size_t lds = quad_lds(P, a.g);
  hipError_t e = allow_lds<sapq_block_kernel<P>>(lds);
  if (e != hipSuccess) return e;
  sapq_block_kernel<P><<<nblocks_colour, quad_threads(a.g), lds, st>>>(a);
  return hipGetLastError();
}

template <int P>
hipError_t launch_sapq_batch(const Geom &g, const int *blocks, int nblocks_colour, const SapSlot<P> *slots,
                             const int *act, int nact, int first, int skip_face, int nmr, hipStream_t st) {
  if (nact < 1) return hipSuccess;
  size_t lds = quad_lds(P, g);
  hipError_t e = allow_lds<sapq_batch_kernel<P>>(lds);
  if (e != hipSuccess) return e;
  sapq_batch_kernel<P><<<(unsigned)nblocks_colour * nact, quad_threads(g), lds, st>>>(
      g, blocks, slots, act, nact, first, skip_face, nmr);
  return hipGetLastError();
}

bool sap_quad_pairs_ok(int prec, const Geom &g) {
  return sap_quad_ok(prec, g, 0) && quad_lds(prec, g, 2) <= (size_t)lds_limit();
}

template <int P>
hipError_t launch_sapq_pairs(const Geom &g, const int *blocks, int nblocks_colour, const SapSlot<P> *slots,
                             const int *pairs, int npair, int first, int skip_face, int nmr, hipStream_t st) {
  if (npair < 1) return hipSuccess;
  size_t lds = quad_lds(P, g, 2);
  hipError_t e = allow_lds<sapq_pair_kernel<P>>(lds);
  if (e != hipSuccess) return e;
  sapq_pair_kernel<P><<<(unsigned)nblocks_colour * npair, quad_threads(g), lds, st>>>(
      g, blocks, slots, pairs, npair, first, skip_face, nmr);
  return hipGetLastError();
}

#define QXD_INST(P)                                                                                      \
  template hipError_t launch_sapq_colour<P>(const SapArgs<P> &, int, hipStream_t);                        \
  template hipError_t launch_sapq_batch<P>(const Geom &, const int *, int, const SapSlot<P> *, const int *, \
                                           int, int, int, int, hipStream_t);                              \
  template hipError_t launch_sapq_pairs<P>(const Geom &, const int *, int, const SapSlot<P> *, const int *, \
                                           int, int, int, int, hipStream_t);
QXD_INST(QXD_F32)
QXD_INST(QXD_F16S)
QXD_INST(QXD_BF16)
#undef QXD_INST

}  // namespace qxd
