// Schwarz alternating procedure: block solves of one colour (SAP preconditioner
// of the GCR solver named in the openQ*D paper's abstract and Sec. 2).
//
// One work-group per block Lambda of the colour, one thread per (even site,
// odd site) pair of the block.  On entry the thread pair first applies the
// face update left over from the other colour's last pass,
//     r(x) -= (D v')(x) = +acc_out(v')(x)/2,
// where acc_out sums the hops from sites outside Lambda and v' holds the other
// colour's latest block corrections.  Then the even-odd block problem is
// solved approximately:
//     u_o   = D_oo^-1 r_o
//     rho_e = r_e - D_eo^L u_o                     (L: hops inside Lambda only)
//     nmr MR steps on D^_L = D_ee - D_eo^L D_oo^-1 D_oe^L:
//         t = D^_L s, alpha = (t,s)/(t,t), v_e += alpha s, s -= alpha t
//     v_o   = D_oo^-1 (r_o - D_oe^L v_e)
// after which the residual on Lambda is exactly r_e = s, r_o = 0, psi += v and
// v is kept for the face update of the neighbouring blocks.  The half spinors
// exchanged between the even and the odd sites of the block live in LDS.
#include "dirac_site.h"
#include "sap.h"

namespace qxd {

namespace {

template <class T>
struct Lds {
  cx<T> *buf0;   // [12][nh] even-site vector
  cx<T> *buf1;   // [12][nh] odd-site vector
  T *red;        // reduction scratch
  int nh;
};

template <class T>
__device__ __forceinline__ void lds_store(cx<T> *buf, int nh, int h, const cx<T> v[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 3; c++) buf[(a * 3 + c) * nh + h] = v[a][c];
}
template <class T>
__device__ __forceinline__ void lds_load(const cx<T> *buf, int nh, int h, cx<T> v[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 3; c++) v[a][c] = buf[(a * 3 + c) * nh + h];
}

__device__ __forceinline__ int local_half(const Geom &g, const int y[4]) {
  return (((y[0] * g.b[1] + y[1]) * g.b[2] + y[2]) * g.b[3] + y[3]) >> 1;
}

// acc over the hops of site s that stay inside its block, neighbours from LDS
template <int P, class T>
__device__ void acc_inside(const Geom &g, const typename St<P>::pair_t *links,
                           const typename St<P>::real_t *angles, int qhat, const Site &s, int64_t i,
                           const cx<T> *buf, int nh, cx<T> acc[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 3; c++) acc[a][c] = {0, 0};
#pragma unroll
  for (int mu = 0; mu < 4; mu++) {
    if (s.y[mu] + 1 < g.b[mu]) {
      int y[4] = {s.y[0], s.y[1], s.y[2], s.y[3]};
      y[mu] += 1;
      cx<T> psi[4][3], w[3][3];
      lds_load<T>(buf, nh, local_half(g, y), psi);
      load_w<P, T>(links, angles, qhat, g.V, mu, i, w);
      hop_fwd<T>(mu, w, psi, (T)1, acc);
    }
    if (s.y[mu] > 0) {
      int sg;
      Site t = neighbour(g, s, mu, -1, sg);
      int64_t j = encode(g, t);
      cx<T> psi[4][3], w[3][3];
      lds_load<T>(buf, nh, local_half(g, t.y), psi);
      load_w<P, T>(links, angles, qhat, g.V, mu, j, w);
      hop_bwd<T>(mu, w, psi, (T)1, acc);
    }
  }
}

// acc over the hops of site s that leave its block, neighbours from global v
template <int P, class T>
__device__ void acc_outside(const Geom &g, const typename St<P>::pair_t *links,
                            const typename St<P>::real_t *angles, int qhat, const Site &s, int64_t i,
                            const Spinor<P> &v, cx<T> acc[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 3; c++) acc[a][c] = {0, 0};
#pragma unroll
  for (int mu = 0; mu < 4; mu++) {
    int sg;
    if (s.y[mu] + 1 == g.b[mu]) {
      Site t = neighbour(g, s, mu, +1, sg);
      cx<T> psi[4][3], w[3][3];
      load_spinor<P, T>(v, encode(g, t), psi);
      load_w<P, T>(links, angles, qhat, g.V, mu, i, w);
      hop_fwd<T>(mu, w, psi, (T)sg, acc);
    }
    if (s.y[mu] == 0) {
      Site t = neighbour(g, s, mu, -1, sg);
      int64_t j = encode(g, t);
      cx<T> psi[4][3], w[3][3];
      load_spinor<P, T>(v, j, psi);
      load_w<P, T>(links, angles, qhat, g.V, mu, j, w);
      hop_bwd<T>(mu, w, psi, (T)sg, acc);
    }
  }
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int P>
__global__ void sap_block_kernel(SapArgs<P> a) {
  using T = typename St<P>::comp_t;
  extern __shared__ __align__(16) unsigned char smem[];
  const Geom &g = a.g;
  const int nh = g.Vbh;
  cx<T> *buf0 = (cx<T> *)smem;
  cx<T> *buf1 = buf0 + 12 * nh;
  T *red = (T *)(buf1 + 12 * nh);
  const int h = threadIdx.x;
  const bool act = h < nh;
  const int nwaves = (blockDim.x + 63) >> 6;

  int blk = a.blocks[blockIdx.x];
  Site se, so;
  {
    int B = blk;
    int Bc[4];
    Bc[3] = B % g.nb[3];
    B /= g.nb[3];
    Bc[2] = B % g.nb[2];
    B /= g.nb[2];
    Bc[1] = B % g.nb[1];
    Bc[0] = B / g.nb[1];
    int hh = act ? h : 0;
    int q = hh / g.hb3;
    int y3h = hh - q * g.hb3;
    int y[3];
    y[2] = q % g.b[2];
    q /= g.b[2];
    y[1] = q % g.b[1];
    y[0] = q / g.b[1];
    for (int m = 0; m < 4; m++) se.B[m] = so.B[m] = Bc[m];
    for (int m = 0; m < 3; m++) se.y[m] = so.y[m] = y[m];
    int par = (y[0] + y[1] + y[2]) & 1;
    se.p = 0;
    se.y[3] = 2 * y3h + par;
    so.p = 1;
    so.y[3] = 2 * y3h + (par ^ 1);
  }
  const int64_t ie = (int64_t)blk * nh + h;
  const int64_t io = (int64_t)g.Vh + ie;

  cx<T> re[4][3], ro[4][3], s[4][3], ve[4][3], tmp[4][3], acc[4][3];
  if (act) {
    const Spinor<P> &src = a.first ? a.rho : a.r;
    load_spinor<P, T>(src, ie, re);
    load_spinor<P, T>(src, io, ro);
    if (!a.skip_face) {
      acc_outside<P, T>(g, a.links, a.angles, a.qhat, se, ie, a.v, acc);
#pragma unroll
      for (int x = 0; x < 4; x++)
#pragma unroll
        for (int c = 0; c < 3; c++) re[x][c] = re[x][c] + (T)0.5 * acc[x][c];
      acc_outside<P, T>(g, a.links, a.angles, a.qhat, so, io, a.v, acc);
#pragma unroll
      for (int x = 0; x < 4; x++)
#pragma unroll
        for (int c = 0; c < 3; c++) ro[x][c] = ro[x][c] + (T)0.5 * acc[x][c];
    }
    // u_o = D_oo^-1 r_o
    pauli_mul<P, T>(a.pinv, g.Vh, ie, ro, tmp);
    lds_store<T>(buf1, nh, h, tmp);
  }
  __syncthreads();
  if (act) {
    // rho_e = r_e - D_eo^L u_o = r_e + acc_in(u)/2
    acc_inside<P, T>(g, a.links, a.angles, a.qhat, se, ie, buf1, nh, acc);
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int c = 0; c < 3; c++) {
        s[x][c] = re[x][c] + (T)0.5 * acc[x][c];
        ve[x][c] = {0, 0};
      }
    lds_store<T>(buf0, nh, h, s);
  }
  __syncthreads();
  for (int k = 0; k < a.nmr; k++) {
    if (act) {
      // odd: w_o = D_oo^-1 D_oe^L s = -D_oo^-1 acc_in(s)/2
      acc_inside<P, T>(g, a.links, a.angles, a.qhat, so, io, buf0, nh, acc);
#pragma unroll
      for (int x = 0; x < 4; x++)
#pragma unroll
        for (int c = 0; c < 3; c++) acc[x][c] = (T)(-0.5) * acc[x][c];
      pauli_mul<P, T>(a.pinv, g.Vh, ie, acc, tmp);
      lds_store<T>(buf1, nh, h, tmp);
    }
    __syncthreads();
    T ts_re = 0, ts_im = 0, tt = 0;
    if (act) {
      // even: t = P s - D_eo^L w_o = P s + acc_in(w)/2
      acc_inside<P, T>(g, a.links, a.angles, a.qhat, se, ie, buf1, nh, acc);
      pauli_mul<P, T>(a.pauli, g.V, ie, s, tmp);
#pragma unroll
      for (int x = 0; x < 4; x++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
          tmp[x][c] = tmp[x][c] + (T)0.5 * acc[x][c];
          cx<T> z = cmulc(tmp[x][c], s[x][c]);
          ts_re += z.re;
          ts_im += z.im;
          tt += norm2(tmp[x][c]);
        }
    }
    ts_re = wave_sum(ts_re);
    ts_im = wave_sum(ts_im);
    tt = wave_sum(tt);
    if ((h & 63) == 0) {
      red[3 * (h >> 6)] = ts_re;
      red[3 * (h >> 6) + 1] = ts_im;
      red[3 * (h >> 6) + 2] = tt;
    }
    __syncthreads();
    ts_re = ts_im = tt = 0;
    for (int w = 0; w < nwaves; w++) {
      ts_re += red[3 * w];
      ts_im += red[3 * w + 1];
      tt += red[3 * w + 2];
    }
    cx<T> alpha{0, 0};
    if (tt > (T)0) alpha = {ts_re / tt, ts_im / tt};
    if (act) {
#pragma unroll
      for (int x = 0; x < 4; x++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
          ve[x][c] = ve[x][c] + alpha * s[x][c];
          s[x][c] = s[x][c] - alpha * tmp[x][c];
        }
    }
    __syncthreads();  // everyone has read red and buf0 (s) of this step
    if (act) lds_store<T>(buf0, nh, h, k + 1 < a.nmr ? s : ve);
    __syncthreads();
  }
  if (a.nmr == 0) {
    if (act) lds_store<T>(buf0, nh, h, ve);
    __syncthreads();
  }
  if (act) {
    // v_o = D_oo^-1 (r_o - D_oe^L v_e) = D_oo^-1 (r_o + acc_in(v_e)/2)
    acc_inside<P, T>(g, a.links, a.angles, a.qhat, so, io, buf0, nh, acc);
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int c = 0; c < 3; c++) acc[x][c] = ro[x][c] + (T)0.5 * acc[x][c];
    cx<T> vo[4][3];
    pauli_mul<P, T>(a.pinv, g.Vh, ie, acc, vo);
    // psi += v; r_e = s; r_o = 0; keep v for the neighbours' face update
    if (a.first) {
      store_spinor<P, T>(a.psi, ie, ve);
      store_spinor<P, T>(a.psi, io, vo);
    } else {
      cx<T> pe[4][3], po[4][3];
      load_spinor<P, T>(a.psi, ie, pe);
      load_spinor<P, T>(a.psi, io, po);
#pragma unroll
      for (int x = 0; x < 4; x++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
          pe[x][c] = pe[x][c] + ve[x][c];
          po[x][c] = po[x][c] + vo[x][c];
        }
      store_spinor<P, T>(a.psi, ie, pe);
      store_spinor<P, T>(a.psi, io, po);
    }
    cx<T> zero[4][3];
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int c = 0; c < 3; c++) zero[x][c] = {0, 0};
    store_spinor<P, T>(a.r, ie, s);
    store_spinor<P, T>(a.r, io, zero);
    store_spinor<P, T>(a.v, ie, ve);
    store_spinor<P, T>(a.v, io, vo);
  }
}

}  // namespace

size_t sap_lds_bytes(int prec, const Geom &g) {
  size_t cs = prec == QXD_F64 ? 16 : 8;
  size_t rs = prec == QXD_F64 ? 8 : 4;
  int nthreads = (g.Vbh + 63) / 64 * 64;
  return 2 * 12 * (size_t)g.Vbh * cs + 3 * (size_t)(nthreads / 64) * rs;
}

template <int P>
hipError_t launch_sap_colour(const SapArgs<P> &a, int nblocks_colour, hipStream_t st) {
  int nthreads = (a.g.Vbh + 63) / 64 * 64;
  size_t lds = sap_lds_bytes(P, a.g);
  sap_block_kernel<P><<<nblocks_colour, nthreads, lds, st>>>(a);
  return hipGetLastError();
}

template hipError_t launch_sap_colour<QXD_F64>(const SapArgs<QXD_F64> &, int, hipStream_t);
template hipError_t launch_sap_colour<QXD_F32>(const SapArgs<QXD_F32> &, int, hipStream_t);
template hipError_t launch_sap_colour<QXD_F16S>(const SapArgs<QXD_F16S> &, int, hipStream_t);
template hipError_t launch_sap_colour<QXD_BF16>(const SapArgs<QXD_BF16> &, int, hipStream_t);

}  // namespace qxd
