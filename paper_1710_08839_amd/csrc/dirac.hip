// Wilson-clover operator kernels: full D, hopping part, Pauli term, and the
// two half-lattice passes of the even-odd Schur complement (Sec. 2.4):
//   odd pass   t_o = D_oo^-1 (self_o + c * acc(in_e))
//   even pass  out_e = P self_e + c * acc(t_o)      (or self_e + c acc)
// so that D^ psi_e = P_e psi_e + acc(t_o)/2 with t_o = -D_oo^-1 acc(psi_e)/2.
// One thread per site; every operand is a structure-of-arrays field in native
// order, so the 64 lanes of a wavefront read consecutive sites.
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "dirac_site.h"
#include "launch.h"

namespace qxd {

namespace {

constexpr int LDS_VARIANT = 16;
constexpr int NT_VARIANT = 32;
constexpr int MIRROR_VARIANT = 64;
constexpr int WAVE_VARIANT = 128;

template <int P, int KIND, int GROUP>
__global__ void __launch_bounds__(256) dirac_kernel(Geom g, const typename St<P>::pair_t *links,
                                                    const typename St<P>::real_t *angles, int qhat,
                                                    const typename St<P>::pair_t *pauli,
                                                    const typename St<P>::pair_t *pinv,
                                                    Spinor<P> in, Spinor<P> self, Spinor<P> out,
                                                    typename St<P>::comp_t c) {
  using T = typename St<P>::comp_t;
  // A work-group owns whole lattice blocks (both parities for the full-lattice
  // kinds, one parity for the half-lattice passes), in XCD-aware order, so
  // that the even/odd neighbours of a site and the blocks next to it are read
  // through the same L2.
  constexpr bool half = KIND == DK_ODD || KIND == DK_EVEN || KIND == DK_EVEN_ID;
  const int per_block = half ? g.Vbh : 2 * g.Vbh;
  const int wg = xcd_order(blockIdx.x, gridDim.x);
  int blk, r;
  if (per_block <= (int)blockDim.x) {  // whole blocks per work-group
    const int bpw = blockDim.x / per_block;
    blk = wg * bpw + threadIdx.x / per_block;
    r = threadIdx.x % per_block;
  } else {                             // a block spread over several work-groups
    const int wpb = per_block / blockDim.x;
    blk = wg / wpb;
    r = (wg % wpb) * blockDim.x + threadIdx.x;
  }
  if (blk >= g.nblocks) return;
  int par = half ? (KIND == DK_ODD ? 1 : 0) : (r >= g.Vbh);
  int i = par * g.Vh + blk * g.Vbh + (r >= g.Vbh ? r - g.Vbh : r);
  cx<T> res[4][3];
  if (KIND != DK_PAULI) {
    Site s = decode(g, i);
    hop_sum<P, T, GROUP>(g, links, angles, qhat, in, s, i, res);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) res[a][b] = c * res[a][b];
  } else {
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) res[a][b] = {0, 0};
  }
  if (KIND == DK_FULL || KIND == DK_PAULI || KIND == DK_EVEN) {
    cx<T> v[4][3], pv[4][3];
    load_spinor<P, T>(self, i, v);
    pauli_mul<P, T>(pauli, g, i, v, pv);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) res[a][b] = res[a][b] + pv[a][b];
  } else if (KIND == DK_EVEN_ID || KIND == DK_ODD) {
    if (self.data != nullptr) {
      cx<T> v[4][3];
      load_spinor<P, T>(self, i, v);
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) res[a][b] = res[a][b] + v[a][b];
    }
  }
  if (KIND == DK_ODD) {
    cx<T> pv[4][3];
    pauli_mul<P, T>(pinv, g, i - g.Vh, res, pv);
    store_spinor<P, T>(out, i, pv);
  } else {
    store_spinor<P, T>(out, i, res);
  }
}

// Variant with the hop neighbours' input spinors staged in LDS.  Each thread
// first copies one site of its block(s) into LDS -- its own site for the
// full-lattice kinds, the site of the other parity with the same half index
// for the half-lattice passes -- so that every input spinor of the block is
// read from memory once; the hops then take in-block neighbours from LDS and
// only the neighbours across the block faces from memory.  The links and the
// Pauli term are read as in dirac_kernel.  Requires whole blocks per
// work-group and hopping links with the U(1) phase folded in (qhat = 0);
// LDS: 12 complex per staged site.
//
// Mirror-fused link reads (mb > 0, C* lattices only): the orbifold makes the
// link of a mirror site x + L1 e1 the complex conjugate of the link of x
// (Sec. 2.1), also with the U(1) phase folded in (the mirror angle is -A).
// Consecutive logical blocks are then a block of the physical half and its
// mirror (mb = L1 / b1 blocks further in direction 1), and every link of a
// mirror site is read at its physical partner and conjugated: the two reads
// of a link line come from neighbouring work-groups of one XCD, so the second
// is served by its L2, and the mirror half of the link array is never read.
template <int P, int KIND, int GROUP, bool NT>
__global__ void __launch_bounds__(256) dirac_lds_kernel(Geom g, const typename St<P>::pair_t *links,
                                                        const typename St<P>::real_t *angles, int qhat,
                                                        const typename St<P>::pair_t *pauli,
                                                        const typename St<P>::pair_t *pinv,
                                                        Spinor<P> in, Spinor<P> self, Spinor<P> out,
                                                        typename St<P>::comp_t c, int mb) {
  using T = typename St<P>::comp_t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *lds = (cx<T> *)smem_raw;
  constexpr bool half = KIND == DK_ODD || KIND == DK_EVEN || KIND == DK_EVEN_ID;
  const int per_block = half ? g.Vbh : 2 * g.Vbh;  // threads (and staged sites) per block
  const int bpw = blockDim.x / per_block;
  const int ns = bpw * per_block;                   // LDS plane length
  const int wg = xcd_order(blockIdx.x, gridDim.x);
  const int lb = threadIdx.x / per_block;
  const int r = threadIdx.x - lb * per_block;
  const int lblk = wg * bpw + lb;
  const bool valid = lblk < g.nblocks;
  const int n23 = g.nb[2] * g.nb[3];
  int blk = lblk;
  if (mb) {
    // logical pair m = (B0, B1 < mb, B2, B3) lexicographic: the block, then its mirror
    const int m = lblk >> 1, q = m / n23;
    blk = ((q / mb) * g.nb[1] + q % mb + (lblk & 1) * mb) * n23 + (m - q * n23);
  }
  const int par = half ? (KIND == DK_ODD ? 1 : 0) : (r >= g.Vbh);
  const int h = r >= g.Vbh ? r - g.Vbh : r;
  const int i = par * g.Vh + blk * g.Vbh + h;
  // The Pauli self term (full D, the even pass) is computed first, straight
  // into the result, and the hops are then added with the factor c folded
  // into their sign: no second 12-component buffer is live at any point.
  constexpr bool pauli_first = KIND == DK_FULL || KIND == DK_PAULI || KIND == DK_EVEN;
  // the own site is the staged one when self is the input field
  const bool self_in_lds = !half && self.data == in.data && self.off == in.off;
  cx<T> res[4][3];
  // stage one input site: own site (full kinds) or the other parity's site
  if (valid) {
    const int spar = half ? 1 - par : par;
    cx<T> v[4][3];
    load_spinor<P, T>(in, (int64_t)spar * g.Vh + (int64_t)blk * g.Vbh + h, v);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) lds[(a * 3 + b) * ns + threadIdx.x] = v[a][b];
    if constexpr (pauli_first) {
      if (!self_in_lds) load_spinor<P, T>(self, i, v);
      pauli_mul<P, T, NT>(pauli, g, i, v, res);
    }
  }
  __syncthreads();
  if (!valid) return;
  const int base = lb * per_block;  // LDS slot of the block's first staged site
  if constexpr (!pauli_first) {
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) res[a][b] = {0, 0};
  }
  if (KIND != DK_PAULI) {
    const Site s = decode(g, i);
#pragma unroll 1
    for (int k0 = 0; k0 < 8; k0 += GROUP) {
#pragma unroll
      for (int k = k0; k < k0 + GROUP; k++) {
        // odd sites of a full-lattice block take the backward hop of each
        // direction first: in every step both parities then read the same
        // links (the forward links of one parity are the backward links of
        // the other), so each link line is fetched once per work-group
        const int mu = k >> 1, dir = ((k & 1) ^ (half ? 0 : par)) ? -1 : 1;
        int sg;
        const Site t = neighbour(g, s, mu, dir, sg);
        const int y = s.y(mu) + dir;
        const bool inside = y >= 0 && y < (int)((g.bpk >> (8 * mu)) & 0xff);
        const int j = encode(g, t);
        cx<T> psi[4][3], w[3][3];
        if (inside) {
          const int l = ((t.y(0) * g.b[1] + t.y(1)) * g.b[2] + t.y(2)) * g.b[3] + t.y(3);
          const int slot = base + (half ? 0 : t.p * g.Vbh) + (l >> 1);
#pragma unroll
          for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) psi[a][b] = lds[(a * 3 + b) * ns + slot];
        } else {
          load_spinor<P, T>(in, j, psi);
        }
        int64_t li = dir > 0 ? (int64_t)i : (int64_t)j;
        bool cj = false;
        if (mb && (dir > 0 ? s.B(1) : t.B(1)) >= mb) {
          li -= (int64_t)mb * n23 * g.Vbh;  // the physical partner, same parity and block position
          cj = true;
        }
        load_link<P, T>(links, g, mu, li, w);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++) w[a][b].im = cj ? -w[a][b].im : w[a][b].im;
        if (dir > 0)
          hop_fwd<T>(mu, w, psi, c * (T)sg, res);
        else
          hop_bwd<T>(mu, w, psi, c * (T)sg, res);
      }
    }
  }
  if (KIND == DK_EVEN_ID || KIND == DK_ODD) {
    if (self.data != nullptr) {
      cx<T> v[4][3];
      load_spinor<P, T>(self, i, v);
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) res[a][b] = res[a][b] + v[a][b];
    }
  }
  if (KIND == DK_ODD) {
    cx<T> pv[4][3];
    pauli_mul<P, T, NT>(pinv, g, i - g.Vh, res, pv);
    store_spinor<P, T, NT>(out, i, pv);
  } else {
    store_spinor<P, T, NT>(out, i, res);
  }
}


// The LDS-staged kernel for 4^4 lattice blocks with wavefront-uniform
// addressing.  A wavefront then lies inside one block and one parity (128
// sites of each parity per block, 64 lanes per wavefront), so everything a
// hop needs beyond the lane's local coordinates is the same for the whole
// wavefront and is computed once in scalar registers: the block across the
// face in direction (mu, dir) with its wrap, the fermion sign of the time
// boundary and the C* shift in directions 2 and 3 (Sec. 2.1), the block
// runs of the neighbour spinors and of the links, and the physical partner
// block for mirror-fused link reads.  A lane finds its neighbour by adding
// +-stride_mu to its local lexicographic index (wrapping across the face),
// with no division.  Neighbour spinors read from memory are loaded as stored
// and the FP16 site scale is folded into the hop's sign.  Same results as
// dirac_lds_kernel up to the order of additions.
template <int P, int KIND, int GROUP, bool NT>
__global__ void __launch_bounds__(256) dirac_wave_kernel(Geom g, const typename St<P>::pair_t *links,
                                                         const typename St<P>::pair_t *pauli,
                                                         const typename St<P>::pair_t *pinv,
                                                         Spinor<P> in, Spinor<P> self, Spinor<P> out,
                                                         typename St<P>::comp_t c, int mb) {
  using T = typename St<P>::comp_t;
  using C = typename St<P>::comp_t;
  constexpr int W = VW<P>;
  constexpr int R = 128;  // sites of one parity of a 4^4 block
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *lds = (cx<T> *)smem_raw;
  constexpr bool half = KIND == DK_ODD || KIND == DK_EVEN || KIND == DK_EVEN_ID;
  constexpr int per_block = half ? R : 2 * R;
  const int bpw = blockDim.x / per_block;
  const int ns = bpw * per_block;
  const int wg = xcd_order(blockIdx.x, gridDim.x);
  const int lb = (int)threadIdx.x / per_block;
  const int r = (int)threadIdx.x - lb * per_block;
  const int lblk = wg * bpw + lb;
  const bool valid = lblk < g.nblocks;
  const int n23 = g.nb[2] * g.nb[3];
  int blk = lblk;
  if (mb) {
    const int m = lblk >> 1, q = m / n23;
    blk = ((q / mb) * g.nb[1] + q % mb + (lblk & 1) * mb) * n23 + (m - q * n23);
  }
  blk = __builtin_amdgcn_readfirstlane(blk);
  const int par = half ? (KIND == DK_ODD ? 1 : 0) : __builtin_amdgcn_readfirstlane(r >> 7);
  const int h = r & (R - 1);
  const int i = par * g.Vh + blk * R + h;
  constexpr bool pauli_first = KIND == DK_FULL || KIND == DK_PAULI || KIND == DK_EVEN;
  const bool self_in_lds = !half && self.data == in.data && self.off == in.off;
  cx<T> res[4][3];
  if (valid) {
    const int spar = half ? 1 - par : par;
    cx<T> v[4][3];
    load_spinor<P, T>(in, (int64_t)spar * g.Vh + (int64_t)blk * R + h, v);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) lds[(a * 3 + b) * ns + threadIdx.x] = v[a][b];
    if constexpr (pauli_first) {
      if (!self_in_lds) load_spinor<P, T>(self, i, v);
      pauli_mul<P, T, NT>(pauli, g, i, v, res);
    }
  }
  __syncthreads();
  if (!valid) return;
  const int base = lb * per_block;
  if constexpr (!pauli_first) {
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) res[a][b] = {0, 0};
  }
  if (KIND != DK_PAULI) {
    // the lane's local coordinates in its 4^4 block and its local index
    const int q = h >> 1;
    const int y2 = q & 3, y1 = (q >> 2) & 3, y0 = q >> 4;
    const int y3 = 2 * (h & 1) + ((par + y0 + y1 + y2) & 1);
    const int l = (y0 << 6) | (y1 << 4) | (y2 << 2) | y3;
    const uint32_t ypk = pack4(y0, y1, y2, y3);
    // the block's coordinates (wavefront-uniform)
    int bb = blk;
    const int B3 = bb % g.nb[3];
    bb /= g.nb[3];
    const int B2 = bb % g.nb[2];
    bb /= g.nb[2];
    const int B1 = bb % g.nb[1];
    const int B0 = bb / g.nb[1];
    const uint32_t Bpk = pack4(B0, B1, B2, B3);
    const int npar = 1 - par;
    const int in_run0 = (int)(in.off / R);
    const uint32_t mshift = (uint32_t)mb * (uint32_t)n23;  // block-index offset of a mirror block's partner
#pragma unroll 1
    for (int k0 = 0; k0 < 8; k0 += GROUP) {
#pragma unroll
      for (int k = k0; k < k0 + GROUP; k++) {
        const int mu = k >> 1, dir = ((k & 1) ^ (half ? 0 : par)) ? -1 : 1;
        // wavefront-uniform: the block across the face, sign and C* shift
        int nb_mu = (int)((Bpk >> (8 * mu)) & 0xff) + dir;
        const int nbm = (int)((g.nbpk >> (8 * mu)) & 0xff);
        int sg = 1;
        uint32_t nBpk = Bpk;
        bool wrap = false;
        if (nb_mu == nbm) {
          nb_mu = 0;
          wrap = true;
        } else if (nb_mu < 0) {
          nb_mu = nbm - 1;
          wrap = true;
        }
        nBpk = (nBpk & ~(0xffu << (8 * mu))) | ((uint32_t)nb_mu << (8 * mu));
        if (wrap) {
          if (mu == 0) {
            sg = g.time_bc == 0 ? -1 : 0;
          } else if ((g.shift_mask >> mu) & 1) {
            int b1 = (int)((nBpk >> 8) & 0xff) + g.L1b;
            if (b1 >= g.nb[1]) b1 -= g.nb[1];
            nBpk = (nBpk & ~0xff00u) | ((uint32_t)b1 << 8);
          }
        }
        const int nB1 = (int)((nBpk >> 8) & 0xff);
        const int nbk = ((int)(nBpk & 0xff) * g.nb[1] + nB1) * n23 + (int)((nBpk >> 16) & 0xff) * g.nb[3] +
                        (int)(nBpk >> 24);
        // the lane's neighbour: inside the block (LDS) or across the face
        const int ym = (int)((ypk >> (8 * mu)) & 0xff);
        const bool inside = (unsigned)(ym + dir) < 4u;
        const int stride = 1 << (6 - 2 * mu);
        const int lp = inside ? l + dir * stride : l - 3 * dir * stride;
        const int hn = lp >> 1;
        cx<T> psi[4][3];
        T hs = (T)1;
        if (inside) {
          const int slot = base + (half ? 0 : npar * R) + hn;
#pragma unroll
          for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) psi[a][b] = lds[(a * 3 + b) * ns + slot];
        } else {
          const uint32_t jrel = (uint32_t)((npar * g.nblocks + nbk - in_run0) * R + hn);
          const uint32_t e = (uint32_t)((npar * g.nblocks + nbk - in_run0) * 12 * R) + (uint32_t)hn * W;
#pragma unroll
          for (int gk = 0; gk < 12 / W; gk++) {
            cx<C> z[W];
            ld_group<P>(at32(in.data + gk * W * R, e), z);
#pragma unroll
            for (int w = 0; w < W; w++) psi[(gk * W + w) / 3][(gk * W + w) % 3] = {(T)z[w].re, (T)z[w].im};
          }
          if constexpr (St<P>::scaled) hs = (T)*at32(in.scale, jrel);
          hs *= (T)sg;
        }
        // the link: the site's own for a forward hop, the neighbour's for a
        // backward one; a mirror block's links are read at its physical
        // partner and conjugated
        int lblkk, lrun_par, lh;
        bool cj = false;
        if (dir > 0) {
          lblkk = blk;
          lrun_par = par;
          lh = h;
          if (mb && B1 >= mb) {
            lblkk -= (int)mshift;
            cj = true;
          }
        } else {
          const int ob1 = inside ? B1 : nB1;
          lblkk = inside ? blk : nbk;
          lrun_par = npar;
          lh = hn;
          if (mb && ob1 >= mb) {
            lblkk -= (int)mshift;
            cj = true;
          }
        }
        const uint32_t el = (uint32_t)((lrun_par * g.nblocks + lblkk) * 36 * R) + (uint32_t)lh * W;
        cx<T> w[3][3];
        load_link_at<P, T>(links, g, mu, el, w);
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++) w[a][b].im = cj ? -w[a][b].im : w[a][b].im;
        if (dir > 0)
          hop_fwd<T>(mu, w, psi, c * hs, res);
        else
          hop_bwd<T>(mu, w, psi, c * hs, res);
      }
    }
  }
  if (KIND == DK_EVEN_ID || KIND == DK_ODD) {
    if (self.data != nullptr) {
      cx<T> v[4][3];
      load_spinor<P, T>(self, i, v);
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) res[a][b] = res[a][b] + v[a][b];
    }
  }
  if (KIND == DK_ODD) {
    cx<T> pv[4][3];
    pauli_mul<P, T, NT>(pinv, g, i - g.Vh, res, pv);
    store_spinor<P, T, NT>(out, i, pv);
  } else {
    store_spinor<P, T, NT>(out, i, res);
  }
}

template <int P, int KIND, int G>
void launch_k(unsigned gr, int threads, size_t lds, bool nt, bool wave, hipStream_t st, const Geom &g,
              const typename St<P>::pair_t *links, const typename St<P>::real_t *angles, int qhat,
              const typename St<P>::pair_t *pauli, const typename St<P>::pair_t *pinv, Spinor<P> vin,
              Spinor<P> vself, Spinor<P> vout, typename St<P>::comp_t c, int mb) {
  if (lds && wave && nt)
    dirac_wave_kernel<P, KIND, G, true><<<gr, threads, lds, st>>>(g, links, pauli, pinv, vin, vself, vout, c, mb);
  else if (lds && wave)
    dirac_wave_kernel<P, KIND, G, false><<<gr, threads, lds, st>>>(g, links, pauli, pinv, vin, vself, vout, c, mb);
  else if (lds && nt)
    dirac_lds_kernel<P, KIND, G, true><<<gr, threads, lds, st>>>(g, links, angles, qhat, pauli, pinv, vin, vself, vout, c, mb);
  else if (lds)
    dirac_lds_kernel<P, KIND, G, false><<<gr, threads, lds, st>>>(g, links, angles, qhat, pauli, pinv, vin, vself, vout, c, mb);
  else
    dirac_kernel<P, KIND, G><<<gr, threads, 0, st>>>(g, links, angles, qhat, pauli, pinv, vin, vself, vout, c);
}

template <int P, int KIND>
void launch_g(int group, unsigned gr, int threads, size_t lds, bool nt, bool wave, hipStream_t st, const Geom &g,
              const typename St<P>::pair_t *links, const typename St<P>::real_t *angles, int qhat,
              const typename St<P>::pair_t *pauli, const typename St<P>::pair_t *pinv, Spinor<P> vin,
              Spinor<P> vself, Spinor<P> vout, typename St<P>::comp_t c, int mb) {
  switch (group) {
    case 1: launch_k<P, KIND, 1>(gr, threads, lds, nt, wave, st, g, links, angles, qhat, pauli, pinv, vin, vself, vout, c, mb); break;
    case 4: launch_k<P, KIND, 4>(gr, threads, lds, nt, wave, st, g, links, angles, qhat, pauli, pinv, vin, vself, vout, c, mb); break;
    case 8: launch_k<P, KIND, 8>(gr, threads, lds, nt, wave, st, g, links, angles, qhat, pauli, pinv, vin, vself, vout, c, mb); break;
    default: launch_k<P, KIND, 2>(gr, threads, lds, nt, wave, st, g, links, angles, qhat, pauli, pinv, vin, vself, vout, c, mb); break;
  }
}

template <int P>
hipError_t launch_p(DiracKind kind, int choice, const Geom &g, const OpFields &f, SpinorArg in,
                    SpinorArg self, SpinorArg out, double c, hipStream_t st) {
  using pt = typename St<P>::pair_t;
  using rt = typename St<P>::real_t;
  using T = typename St<P>::comp_t;
  auto links = (const pt *)f.links;
  auto angles = (const rt *)f.angles;
  auto pauli = (const pt *)f.pauli;
  auto pinv = (const pt *)f.pinv;
  Spinor<P> vin = spinor_view<P>(in.ptr, in.sites, in.off, g);
  Spinor<P> vself = self.ptr ? spinor_view<P>(self.ptr, self.sites, self.off, g) : Spinor<P>{nullptr, nullptr, 0, g.rd};
  Spinor<P> vout = spinor_view<P>(out.ptr, out.sites, out.off, g);
  // work-group size: whole blocks, about 256 threads
  bool half = kind == DK_ODD || kind == DK_EVEN || kind == DK_EVEN_ID;
  int per_block = half ? g.Vbh : 2 * g.Vbh;
  int threads;
  unsigned gr;
  if (per_block <= 256) {
    int bpw = 256 / per_block;
    threads = bpw * per_block;
    gr = grid_for(g.nblocks, bpw);
  } else {
    // block sites are a multiple of 16, so per_block is a multiple of 8: use
    // the largest power-of-two divisor of per_block up to 256 threads
    threads = 256;
    while (per_block % threads) threads >>= 1;
    gr = (unsigned)g.nblocks * (per_block / threads);
  }
  T cc = (T)c;
  // choice = hop group size, + LDS_VARIANT for the LDS-staged kernel (whole
  // blocks per work-group only)
  const bool use_lds = (choice & LDS_VARIANT) && per_block <= 256 && kind != DK_PAULI && f.qhat == 0;
  const bool nt = use_lds && (choice & NT_VARIANT);
  // mirror-fused link reads: C* lattices (extended direction 1 twice L1), pairs of whole blocks
  const int mb = use_lds && (choice & MIRROR_VARIANT) && g.N[1] == 2 * g.L1 ? g.L1b : 0;
  const int group = choice & (LDS_VARIANT - 1);
  const size_t lds = use_lds ? 12 * (size_t)threads * sizeof(cx<T>) : 0;
  // wavefront-uniform addressing: LDS-staged kernel on 4^4 blocks
  const bool wave = use_lds && (choice & WAVE_VARIANT) && g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4;
  switch (kind) {
    case DK_FULL: launch_g<P, DK_FULL>(group, gr, threads, lds, nt, wave, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc, mb); break;
    case DK_HOP: launch_g<P, DK_HOP>(group, gr, threads, lds, nt, wave, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc, mb); break;
    case DK_PAULI: launch_g<P, DK_PAULI>(1, gr, threads, 0, false, false, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc, mb); break;
    case DK_ODD: launch_g<P, DK_ODD>(group, gr, threads, lds, nt, wave, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc, mb); break;
    case DK_EVEN: launch_g<P, DK_EVEN>(group, gr, threads, lds, nt, wave, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc, mb); break;
    case DK_EVEN_ID: launch_g<P, DK_EVEN_ID>(group, gr, threads, lds, nt, wave, st, g, links, angles, f.qhat, pauli, pinv, vin, vself, vout, cc, mb); break;
  }
  return hipGetLastError();
}

hipError_t launch_any(int prec, DiracKind kind, int choice, const Geom &g, const OpFields &f, SpinorArg in,
                      SpinorArg self, SpinorArg out, double c, hipStream_t st) {
  switch (prec) {
    case QXD_F64: return launch_p<QXD_F64>(kind, choice, g, f, in, self, out, c, st);
    case QXD_F32: return launch_p<QXD_F32>(kind, choice, g, f, in, self, out, c, st);
    case QXD_F16S: return launch_p<QXD_F16S>(kind, choice, g, f, in, self, out, c, st);
    case QXD_BF16: return launch_p<QXD_BF16>(kind, choice, g, f, in, self, out, c, st);
  }
  return hipErrorInvalidValue;
}

// Autotuned choice of the kernel variant (hop group size, LDS staging of the
// input spinor), per (precision, kernel kind, volume, U(1) phase on the
// fly): the first call times every candidate on the caller's own operands
// (all candidates compute the same result up to rounding) and keeps the
// fastest, or the first in candidate order within 2% of it.
struct TuneKey {
  int prec, kind, V, phase;
  bool operator<(const TuneKey &o) const {
    return std::tie(prec, kind, V, phase) < std::tie(o.prec, o.kind, o.V, o.phase);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;

int tune_group(int prec, DiracKind kind, const Geom &g, const OpFields &f, SpinorArg in, SpinorArg self,
               SpinorArg out, double c, hipStream_t st) {
  TuneKey key{prec, (int)kind, g.V, f.qhat != 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  constexpr int L = LDS_VARIANT, N = NT_VARIANT;
  constexpr int M = MIRROR_VARIANT, Wv = WAVE_VARIANT;
  const bool half = kind == DK_ODD || kind == DK_EVEN || kind == DK_EVEN_ID;
  const bool fits = (half ? g.Vbh : 2 * g.Vbh) <= 256;
  const bool cstar = g.N[1] == 2 * g.L1;
  const bool b44 = g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4;
  // FP64 with groups of 8 hops exceeds the register file and spills to
  // private memory (slower, and that memory is allocated at dispatch): it is
  // left out of the search
  std::vector<int> cands = {1, 2, 4};
  if (prec != QXD_F64) cands.push_back(8);
  if (fits) {
    for (int c : {L | 1, L | 2, L | 4, L | N | 1, L | N | 2, L | N | 4}) cands.push_back(c);
    if (cstar)
      for (int c : {L | M | 1, L | N | M | 1, L | N | M | 2}) cands.push_back(c);
    if (b44) {
      for (int c : {L | N | Wv | 1, L | N | Wv | 2, L | N | Wv | 4}) cands.push_back(c);
      if (cstar)
        for (int c : {L | N | M | Wv | 1, L | N | M | Wv | 2, L | N | M | Wv | 4}) cands.push_back(c);
    }
  }
  const int ncand = (int)cands.size();
  const int *cand = cands.data();
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 2;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return 2;
  }
  std::vector<float> ms_of(cands.size());
  for (float &m : ms_of) m = 1e30f;
  for (int ci = 0; ci < ncand; ci++) {
    const int gsz = cand[ci];
    // warm-up; a candidate that cannot launch here is skipped
    if (launch_any(prec, kind, gsz, g, f, in, self, out, c, st) != hipSuccess) continue;
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 3; r++) (void)launch_any(prec, kind, gsz, g, f, in, self, out, c, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms_of[ci] = ms;
  }
  // the first candidate within 2% of the fastest: near-ties resolve the same
  // way in every process
  float best_ms = 1e30f;
  for (int ci = 0; ci < ncand; ci++) best_ms = ms_of[ci] < best_ms ? ms_of[ci] : best_ms;
  int best = 2;
  for (int ci = 0; ci < ncand; ci++)
    if (ms_of[ci] <= 1.02f * best_ms) {
      best = cand[ci];
      break;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

}  // namespace

std::atomic<int> g_forced_choice{0};

hipError_t launch_dirac(int prec, DiracKind kind, const Geom &g, const OpFields &f, SpinorArg in,
                        SpinorArg self, SpinorArg out, double c, hipStream_t st, bool may_tune) {
  if (prec < QXD_F64 || prec > QXD_BF16) return hipErrorInvalidValue;
  const int forced = g_forced_choice.load(std::memory_order_relaxed);
  int choice = 1;
  if (kind != DK_PAULI) {
    if (forced) {
      choice = forced;
    } else if (may_tune) {
      choice = tune_group(prec, kind, g, f, in, self, out, c, st);
    } else {
      choice = tuned_group(prec, (int)kind, g.V, f.qhat != 0);
      if (!choice) choice = 2;
    }
  }
  return launch_any(prec, kind, choice, g, f, in, self, out, c, st);
}

bool force_dirac_variant(int choice) {
  const int group = choice & (LDS_VARIANT - 1);
  if (choice != 0 && ((choice & ~(WAVE_VARIANT | MIRROR_VARIANT | NT_VARIANT | LDS_VARIANT | 15)) ||
                      (group != 1 && group != 2 && group != 4 && group != 8)))
    return false;
  g_forced_choice.store(choice);
  return true;
}

int tuned_group(int prec, int kind, int V, int phase) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(TuneKey{prec, kind, V, phase});
  return it == g_tuned.end() ? 0 : it->second;
}

}  // namespace qxd
