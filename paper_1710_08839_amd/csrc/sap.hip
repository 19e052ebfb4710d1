// Schwarz alternating procedure: block solves of one colour (SAP preconditioner
// of the GCR solver named in the openQ*D paper's abstract and Sec. 2).
//
// This file: one work-group per block Lambda of the colour, one thread per
// site (FP64, and blocks of more than 256 sites); the reduced precisions use
// the four-lanes-per-site variant in sap_quad.hip.  On entry each site first
// applies the face update left over from the other colour's last pass,
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

__device__ __forceinline__ int local_half(const Geom &g, const Site &t) {
  return (((t.y(0) * g.b[1] + t.y(1)) * g.b[2] + t.y(2)) * g.b[3] + t.y(3)) >> 1;
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
#pragma unroll 1
  for (int k = 0; k < 8; k++) {
    int mu = k >> 1, dir = (k & 1) ? -1 : 1;
    int y = s.y(mu) + dir;
    if (y < 0 || y >= (int)((g.bpk >> (8 * mu)) & 0xff)) continue;
    int sg;
    Site t = neighbour(g, s, mu, dir, sg);
    cx<T> psi[4][3], w[3][3];
    lds_load<T>(buf, nh, local_half(g, t), psi);
    load_w<P, T>(links, angles, qhat, g, mu, dir > 0 ? i : (int64_t)encode(g, t), w);
    if (dir > 0)
      hop_fwd<T>(mu, w, psi, (T)1, acc);
    else
      hop_bwd<T>(mu, w, psi, (T)1, acc);
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
#pragma unroll 1
  for (int k = 0; k < 8; k++) {
    int mu = k >> 1, dir = (k & 1) ? -1 : 1;
    int y = s.y(mu) + dir;
    if (y >= 0 && y < (int)((g.bpk >> (8 * mu)) & 0xff)) continue;
    int sg;
    Site t = neighbour(g, s, mu, dir, sg);
    int64_t j = encode(g, t);
    cx<T> psi[4][3], w[3][3];
    load_spinor<P, T>(v, j, psi);
    load_w<P, T>(links, angles, qhat, g, mu, dir > 0 ? i : j, w);
    if (dir > 0)
      hop_fwd<T>(mu, w, psi, (T)sg, acc);
    else
      hop_bwd<T>(mu, w, psi, (T)sg, acc);
  }
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Thread t < nh works on even site t of the block, thread nh + t on odd site
// t (nh = sites of one parity per block, a multiple of 64 for the usual 4^4
// blocks so that no wavefront mixes parities).
template <int P>
__device__ __forceinline__ void sap_block_body(const Geom &g, const SapOp<P> &a, const SapVecs<P> &vv,
                                               int blk, int first, int skip_face, int nmr,
                                               unsigned char *smem) {
  using T = typename St<P>::comp_t;
  const int nh = g.Vbh;
  cx<T> *buf0 = (cx<T> *)smem;        // even-site vector s
  cx<T> *buf1 = buf0 + 12 * nh;       // odd-site vector
  cx<T> *bufv = buf1 + 12 * nh;       // even-site MR solution v_e
  T *red = (T *)(bufv + 12 * nh);     // per-wavefront partial sums
  const int tid = threadIdx.x;
  const bool odd = tid >= nh;
  const int h = odd ? tid - nh : tid;
  const bool act = h < nh && tid < 2 * nh;
  const int even_waves = (nh + 63) >> 6;

  Site st;
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
    st.p = odd ? 1 : 0;
    st.Bp = pack4(B0, B1, B2, B3);
    st.yp = pack4(y0, y1, y2, 2 * y3h + ((st.p + y0 + y1 + y2) & 1));
  }
  const int64_t ie = (int64_t)blk * nh + h;      // native index of the even site / odd half index
  const int64_t i = odd ? (int64_t)g.Vh + ie : ie;

  cx<T> r[4][3], s[4][3], tmp[4][3], acc[4][3];
  if (act) {
    load_spinor<P, T>(first ? vv.rho : vv.r, i, r);
    if (!skip_face) {
      acc_outside<P, T>(g, a.links, a.angles, a.qhat, st, i, vv.v, acc);
#pragma unroll
      for (int x = 0; x < 4; x++)
#pragma unroll
        for (int c = 0; c < 3; c++) r[x][c] = r[x][c] + (T)0.5 * acc[x][c];
    }
    if (odd) {
      // u_o = D_oo^-1 r_o; r_o is parked in the residual field until the end
      store_spinor<P, T>(vv.r, i, r);
      pauli_mul<P, T>(a.pinv, g, ie, r, tmp);
      lds_store<T>(buf1, nh, h, tmp);
    }
  }
  __syncthreads();
  if (act && !odd) {
    // rho_e = r_e - D_eo^L u_o = r_e + acc_in(u)/2
    acc_inside<P, T>(g, a.links, a.angles, a.qhat, st, i, buf1, nh, acc);
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int c = 0; c < 3; c++) {
        s[x][c] = r[x][c] + (T)0.5 * acc[x][c];
        tmp[x][c] = {0, 0};
      }
    lds_store<T>(buf0, nh, h, s);
    lds_store<T>(bufv, nh, h, tmp);
  }
  __syncthreads();
  for (int k = 0; k < nmr; k++) {
    if (act && odd) {
      // w_o = D_oo^-1 D_oe^L s = -D_oo^-1 acc_in(s)/2
      acc_inside<P, T>(g, a.links, a.angles, a.qhat, st, i, buf0, nh, acc);
#pragma unroll
      for (int x = 0; x < 4; x++)
#pragma unroll
        for (int c = 0; c < 3; c++) acc[x][c] = (T)(-0.5) * acc[x][c];
      pauli_mul<P, T>(a.pinv, g, ie, acc, tmp);
      lds_store<T>(buf1, nh, h, tmp);
    }
    __syncthreads();
    // (t, s) and (t, t) over the even sites; every lane takes part in the
    // wavefront reductions (odd and idle lanes add zero)
    T ts_re = 0, ts_im = 0, tt = 0;
    if (!odd) {
      if (act) {
        // t = P s - D_eo^L w_o = P s + acc_in(w)/2
        acc_inside<P, T>(g, a.links, a.angles, a.qhat, st, i, buf1, nh, acc);
        pauli_mul<P, T>(a.pauli, g, i, s, tmp);
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
    }
    ts_re = wave_sum(ts_re);
    ts_im = wave_sum(ts_im);
    tt = wave_sum(tt);
    if ((tid & 63) == 0) {
      red[3 * (tid >> 6)] = ts_re;
      red[3 * (tid >> 6) + 1] = ts_im;
      red[3 * (tid >> 6) + 2] = tt;
    }
    __syncthreads();
    if (!odd) {
      T sr = 0, si = 0, stt = 0;
      for (int w = 0; w < even_waves; w++) {
        sr += red[3 * w];
        si += red[3 * w + 1];
        stt += red[3 * w + 2];
      }
      cx<T> alpha{0, 0};
      if (stt > (T)0) alpha = {sr / stt, si / stt};
      if (act) {
#pragma unroll
        for (int x = 0; x < 4; x++)
#pragma unroll
          for (int c = 0; c < 3; c++) {
            int e = (x * 3 + c) * nh + h;
            bufv[e] = bufv[e] + alpha * s[x][c];
            s[x][c] = s[x][c] - alpha * tmp[x][c];
          }
        lds_store<T>(buf0, nh, h, s);
      }
    }
    __syncthreads();
  }
  if (!act) return;
  cx<T> v[4][3];
  if (odd) {
    // v_o = D_oo^-1 (r_o - D_oe^L v_e) = D_oo^-1 (r_o + acc_in(v_e)/2)
    load_spinor<P, T>(vv.r, i, r);
    acc_inside<P, T>(g, a.links, a.angles, a.qhat, st, i, bufv, nh, acc);
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int c = 0; c < 3; c++) acc[x][c] = r[x][c] + (T)0.5 * acc[x][c];
    pauli_mul<P, T>(a.pinv, g, ie, acc, v);
  } else {
    lds_load<T>(bufv, nh, h, v);
  }
  // psi += v; residual on the block: r_e = s, r_o = 0; keep v for the faces
  if (first) {
    store_spinor<P, T>(vv.psi, i, v);
  } else {
    load_spinor<P, T>(vv.psi, i, tmp);
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int c = 0; c < 3; c++) tmp[x][c] = tmp[x][c] + v[x][c];
    store_spinor<P, T>(vv.psi, i, tmp);
  }
  if (odd) {
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
      for (int c = 0; c < 3; c++) s[x][c] = {0, 0};
  }
  store_spinor<P, T>(vv.r, i, s);
  store_spinor<P, T>(vv.v, i, v);
}

template <int P>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
sap_block_kernel(SapArgs<P> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  SapOp<P> op{a.links, a.angles, a.qhat, a.pauli, a.pinv};
  SapVecs<P> vv{a.rho, a.r, a.psi, a.v};
  sap_block_body<P>(a.g, op, vv, a.blocks[xcd_order(blockIdx.x, gridDim.x)], a.first, a.skip_face,
                    a.nmr, smem);
}

// Batched: work-group L (in XCD-aware order) solves block L / nact of the
// colour for right-hand side slot act[L % nact]; the blocks of the batch that
// share a lattice block run next to each other, so their links and Pauli
// terms are read through the same L2.
template <int P>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
sap_batch_kernel(Geom g, const int *blocks, const SapSlot<P> *slots, const int *act, int nact,
                 int first, int skip_face, int nmr) {
  extern __shared__ __align__(16) unsigned char smem[];
  int L = xcd_order(blockIdx.x, gridDim.x);
  int bi = L / nact;
  const SapSlot<P> &sl = slots[act[L - bi * nact]];
  sap_block_body<P>(g, sl.op, sl.vec, blocks[bi], first, skip_face, nmr, smem);
}

}  // namespace

static int sap_threads(const Geom &g) {
  // even sites in waves [0, ceil(nh/64)), odd sites from thread nh on
  return ((2 * g.Vbh) + 63) / 64 * 64;
}

size_t sap_lds_bytes(int prec, const Geom &g) {
  size_t cs = prec == QXD_F64 ? 16 : 8;
  size_t rs = prec == QXD_F64 ? 8 : 4;
  return 3 * 12 * (size_t)g.Vbh * cs + 3 * (size_t)(sap_threads(g) / 64) * rs;
}

template <int P>
hipError_t launch_sap_colour(const SapArgs<P> &a, int nblocks_colour, hipStream_t st) {
  if constexpr (P != QXD_F64) {
    if (sap_quad_ok(P, a.g, a.qhat)) return launch_sapq_colour<P>(a, nblocks_colour, st);
  }
  int nthreads = sap_threads(a.g);
  size_t lds = sap_lds_bytes(P, a.g);
  sap_block_kernel<P><<<nblocks_colour, nthreads, lds, st>>>(a);
  return hipGetLastError();
}

template <int P>
hipError_t launch_sap_batch(const Geom &g, const int *blocks, int nblocks_colour, const SapSlot<P> *slots,
                            const int *act, int nact, int first, int skip_face, int nmr, hipStream_t st) {
  if (nact < 1) return hipSuccess;
  if constexpr (P != QXD_F64) {
    if (sap_quad_ok(P, g, 0))
      return launch_sapq_batch<P>(g, blocks, nblocks_colour, slots, act, nact, first, skip_face, nmr, st);
  }
  int nthreads = sap_threads(g);
  size_t lds = sap_lds_bytes(P, g);
  sap_batch_kernel<P><<<(unsigned)nblocks_colour * nact, nthreads, lds, st>>>(g, blocks, slots, act, nact,
                                                                            first, skip_face, nmr);
  return hipGetLastError();
}

#define QXD_INST(P)                                                                                  \
  template hipError_t launch_sap_batch<P>(const Geom &, const int *, int, const SapSlot<P> *, const int *, \
                                          int, int, int, int, hipStream_t);
QXD_INST(QXD_F64)
QXD_INST(QXD_F32)
QXD_INST(QXD_F16S)
QXD_INST(QXD_BF16)
#undef QXD_INST

template hipError_t launch_sap_colour<QXD_F64>(const SapArgs<QXD_F64> &, int, hipStream_t);
template hipError_t launch_sap_colour<QXD_F32>(const SapArgs<QXD_F32> &, int, hipStream_t);
template hipError_t launch_sap_colour<QXD_F16S>(const SapArgs<QXD_F16S> &, int, hipStream_t);
template hipError_t launch_sap_colour<QXD_BF16>(const SapArgs<QXD_BF16> &, int, hipStream_t);

}  // namespace qxd
