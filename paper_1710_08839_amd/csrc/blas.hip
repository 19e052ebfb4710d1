// Linear algebra on native spinors for the Krylov solvers: multi-dot products,
// multi-axpys with fused norms, residual updates and precision conversion.
//
// Every reduction accumulates in FP64 (GCR orthogonalisation and norms are
// FP64 whatever the storage precision) and is deterministic: a fixed grid of
// at most RED_BLOCKS work-groups writes per-group partial sums, and one
// work-group adds them in a fixed tree order.  Results depend only on the
// vector length and the data, never on what else runs on the GPU.
#include "blas.h"
#include "qxd_impl.h"

namespace qxd {

namespace {

constexpr int BT = 256;

__device__ __forceinline__ double block_sum(double v, double *sh) {
  // wavefront reduction then across the 4 wavefronts of the group
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;
}

// K block sums at once, each in the order of block_sum (wavefront tree, then
// the four wavefronts pairwise) but with a single barrier; partial[k * stride]
// receives sum k (written by thread k)
template <int K>
__device__ __forceinline__ void block_sums(const double (&v)[K], double *sh, double *partial, int64_t stride) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; k++) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) sh[4 * k + w] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    const int k = threadIdx.x;
    partial[k * stride] = (sh[4 * k] + sh[4 * k + 1]) + (sh[4 * k + 2] + sh[4 * k + 3]);
  }
}

inline unsigned red_grid(int64_t n) {
  int64_t g = (n + BT - 1) / BT;
  return (unsigned)(g < RED_BLOCKS ? (g < 1 ? 1 : g) : RED_BLOCKS);
}

template <int P>
__device__ __forceinline__ void ld(const Spinor<P> &v, int64_t i, cx<double> a[4][3]) {
  load_spinor<P, double>(v, i, a);
}

// partial[k][blk] for k < nred
__global__ void __launch_bounds__(BT) finish_kernel(const double *partial, int nblk, int nred, double *out,
                              const double *div, int div_stride) {
  __shared__ double sh[4];
  for (int k = 0; k < nred; k++) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += BT) v += partial[(int64_t)k * nblk + b];
    double s = block_sum(v, sh);
    if (threadIdx.x == 0) {
      if (div) s /= div[(k / 2) * div_stride];
      out[k] = s;
    }
    __syncthreads();
  }
}

// partial[(base + 2l (+1)) * grid + blk] = block sums of (y_l, x), l < N
template <int P, int N>
__global__ void __launch_bounds__(BT) mdot_kernel(VecList<P> ys, Spinor<P> x, int64_t first, int64_t count,
                            double *partial, int base) {
  __shared__ double sh[4];
  double acc[2 * N];
#pragma unroll
  for (int k = 0; k < 2 * N; k++) acc[k] = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < count; t += (int64_t)gridDim.x * BT) {
    int64_t i = first + t;
    cx<double> xv[4][3];
    ld<P>(x, i, xv);
#pragma unroll
    for (int l = 0; l < N; l++) {
      cx<double> yv[4][3];
      ld<P>(ys.v[l], i, yv);
      double re = 0, im = 0;
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
          cx<double> z = cmulc(yv[a][c], xv[a][c]);
          re += z.re;
          im += z.im;
        }
      acc[2 * l] += re;
      acc[2 * l + 1] += im;
    }
  }
#pragma unroll
  for (int k = 0; k < 2 * N; k++) {
    double s = block_sum(acc[k], sh);
    if (threadIdx.x == 0) partial[(int64_t)(base + k) * gridDim.x + blockIdx.x] = s;
  }
}

template <int P>
struct MaxpyArgs {
  int ntriples;
  Spinor<P> src[2];
  Spinor<P> dst[2];
  VecList<P> ys[2];
  const double *coef;   // complex, element l + coef_base
  const double *div;
  int div_stride;
  int coef_base;
  int want_norms;
  int has_w;
  Spinor<P> w;
};

// One triple of maxpy_kernel at site i.  TR is a template argument so that
// the kernel-argument arrays are indexed by constants: a run-time index
// would copy them to private memory.
template <int P, int N, int TR>
__device__ __forceinline__ void maxpy_triple(const MaxpyArgs<P> &a, int64_t i, const cx<double> *cf, double &nn,
                                             double &wr, double &wi) {
  cx<double> z[4][3];
  ld<P>(a.src[TR], i, z);
#pragma unroll
  for (int l = 0; l < N; l++) {
    cx<double> y[4][3];
    ld<P>(a.ys[TR].v[l], i, y);
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
      for (int k = 0; k < 3; k++) z[s][k] = z[s][k] - cf[l] * y[s][k];
  }
  store_spinor<P, double>(a.dst[TR], i, z);
  if (TR == 0 && a.want_norms) {
    // re-read what was stored so that the norms match the stored vector
    ld<P>(a.dst[0], i, z);
    cx<double> w[4][3];
    if (a.has_w) ld<P>(a.w, i, w);
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        nn += norm2(z[s][k]);
        if (a.has_w) {
          cx<double> q = cmulc(z[s][k], w[s][k]);
          wr += q.re;
          wi += q.im;
        }
      }
  }
}

// z_t = src_t - sum_{l<N} coef[l] / div[l] * ys_t[l] for t < ntriples; then
// partial sums of (z_0, z_0) and (z_0, w).
template <int P, int N>
__global__ void __launch_bounds__(BT) maxpy_kernel(MaxpyArgs<P> a, int64_t first, int64_t count, double *partial) {
  __shared__ double sh[4];
  cx<double> cf[N > 0 ? N : 1];
#pragma unroll
  for (int l = 0; l < N; l++) {
    int L = a.coef_base + l;
    double d = a.div ? a.div[L * a.div_stride] : 1.0;
    cf[l] = {a.coef[2 * L] / d, a.coef[2 * L + 1] / d};
  }
  double nn = 0.0, wr = 0.0, wi = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < count; t += (int64_t)gridDim.x * BT) {
    int64_t i = first + t;
    maxpy_triple<P, N, 0>(a, i, cf, nn, wr, wi);
    if (a.ntriples > 1) maxpy_triple<P, N, 1>(a, i, cf, nn, wr, wi);
  }
  if (a.want_norms) {
    double s0 = block_sum(nn, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s0;
    double s1 = block_sum(wr, sh);
    if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = s1;
    double s2 = block_sum(wi, sh);
    if (threadIdx.x == 0) partial[2 * gridDim.x + blockIdx.x] = s2;
  }
}

// y -= (num / den) x  with num complex (device), den real (device); then |y|^2.
template <int P>
__global__ void __launch_bounds__(BT) update_kernel(Spinor<P> y, Spinor<P> x, const double *num, const double *den,
                              int negate, int64_t first, int64_t count, double *partial) {
  __shared__ double sh[4];
  double d = den ? *den : 1.0;
  cx<double> c{num[0] / d, num[1] / d};
  if (negate) c = -c;
  double nn = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < count; t += (int64_t)gridDim.x * BT) {
    int64_t i = first + t;
    cx<double> yv[4][3], xv[4][3];
    ld<P>(y, i, yv);
    ld<P>(x, i, xv);
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
      for (int k = 0; k < 3; k++) yv[s][k] = yv[s][k] - c * xv[s][k];
    store_spinor<P, double>(y, i, yv);
    ld<P>(y, i, yv);
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
      for (int k = 0; k < 3; k++) nn += norm2(yv[s][k]);
  }
  double s0 = block_sum(nn, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s0;
}

// y_Q = a * y_Q + b * x_P (a, b real; y may be absent: a = 0 and y not read);
// optional |y|^2.
template <int Q, int P>
__global__ void __launch_bounds__(BT) axpby_kernel(Spinor<Q> y, double a, Spinor<P> x, double b, int64_t first,
                             int64_t count, double *partial) {
  __shared__ double sh[4];
  double nn = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < count; t += (int64_t)gridDim.x * BT) {
    int64_t i = first + t;
    cx<double> yv[4][3], xv[4][3];
    ld<P>(x, i, xv);
    if (a != 0.0) {
      ld<Q>(y, i, yv);
#pragma unroll
      for (int s = 0; s < 4; s++)
#pragma unroll
        for (int k = 0; k < 3; k++) yv[s][k] = a * yv[s][k] + b * xv[s][k];
    } else {
#pragma unroll
      for (int s = 0; s < 4; s++)
#pragma unroll
        for (int k = 0; k < 3; k++) yv[s][k] = b * xv[s][k];
    }
    store_spinor<Q, double>(y, i, yv);
    if (partial) {
      ld<Q>(y, i, yv);
#pragma unroll
      for (int s = 0; s < 4; s++)
#pragma unroll
        for (int k = 0; k < 3; k++) nn += norm2(yv[s][k]);
    }
  }
  if (partial) {
    double s0 = block_sum(nn, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s0;
  }
}

// |x|^2 and a finiteness check
template <int P>
__global__ void __launch_bounds__(BT) norm_kernel(Spinor<P> x, int64_t first, int64_t count, double *partial) {
  __shared__ double sh[4];
  double nn = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < count; t += (int64_t)gridDim.x * BT) {
    cx<double> xv[4][3];
    ld<P>(x, first + t, xv);
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
      for (int k = 0; k < 3; k++) nn += norm2(xv[s][k]);
  }
  double s0 = block_sum(nn, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s0;
}

template <int P>
Spinor<P> view(const SpinorArg &a) {
  return spinor_view<P>(a.ptr, a.sites, a.off, a.rd);
}

// ---- flat forms --------------------------------------------------------------
// For whole runs of sites (first and count multiples of the run length) the
// elements of a site range are one contiguous stretch in the block-major
// layout, and every vector of a call shares the layout, so dot products and
// axpys can run over 16-byte groups of components in storage order: one
// 16-byte load per vector and group, few registers, fully contiguous
// streams.  Not for FP16S (per-site scales).

template <int P>
__device__ __forceinline__ void ldg_group(const typename St<P>::pair_t *base, int64_t gi,
                                          cx<double> out[VW<P>]) {
  cx<typename St<P>::comp_t> z[VW<P>];
  ld_group<P>(base + gi * VW<P>, z);
#pragma unroll
  for (int w = 0; w < VW<P>; w++) out[w] = {(double)z[w].re, (double)z[w].im};
}

// partial[(base + 2l (+1)) * grid + blk] = block sums of (y_l, x) over groups [g0, g0 + ng)
template <int P, int N>
__global__ void __launch_bounds__(BT) mdot_flat_kernel(VecList<P> ys, Spinor<P> x, int64_t g0, int64_t ng, double *partial,
                                 int base) {
  constexpr int W = VW<P>;
  __shared__ double sh[4 * 2 * N];
  double acc[2 * N];
#pragma unroll
  for (int k = 0; k < 2 * N; k++) acc[k] = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < ng; t += (int64_t)gridDim.x * BT) {
    cx<double> xv[W];
    ldg_group<P>(x.data, g0 + t, xv);
#pragma unroll
    for (int l = 0; l < N; l++) {
      cx<double> yv[W];
      ldg_group<P>(ys.v[l].data, g0 + t, yv);
#pragma unroll
      for (int w = 0; w < W; w++) {
        acc[2 * l] = fmat(yv[w].re, xv[w].re, acc[2 * l]);
        acc[2 * l] = fmat(yv[w].im, xv[w].im, acc[2 * l]);
        acc[2 * l + 1] = fmat(yv[w].re, xv[w].im, acc[2 * l + 1]);
        acc[2 * l + 1] = fmat(-yv[w].im, xv[w].re, acc[2 * l + 1]);
      }
    }
  }
  block_sums<2 * N>(acc, sh, partial + (int64_t)base * gridDim.x + blockIdx.x, gridDim.x);
}

// z_t = src_t - sum_l cf_l ys_t[l] over groups; norms of the stored z_0 (the
// value rounded to the storage precision, as a later read would see it)
template <int P, int N>
__global__ void __launch_bounds__(BT) maxpy_flat_kernel(MaxpyArgs<P> a, int64_t g0, int64_t ng, double *partial) {
  constexpr int W = VW<P>;
  using C = typename St<P>::comp_t;
  __shared__ double sh[12];
  cx<double> cf[N > 0 ? N : 1];
#pragma unroll
  for (int l = 0; l < N; l++) {
    int L = a.coef_base + l;
    double d = a.div ? a.div[L * a.div_stride] : 1.0;
    cf[l] = {a.coef[2 * L] / d, a.coef[2 * L + 1] / d};
  }
  double nn = 0.0, wr = 0.0, wi = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < ng; t += (int64_t)gridDim.x * BT) {
    const int64_t gi = g0 + t;
    for (int tr = 0; tr < a.ntriples; tr++) {
      cx<double> z[W];
      ldg_group<P>(a.src[tr].data, gi, z);
#pragma unroll
      for (int l = 0; l < N; l++) {
        cx<double> y[W];
        ldg_group<P>(a.ys[tr].v[l].data, gi, y);
#pragma unroll
        for (int w = 0; w < W; w++) z[w] = z[w] - cf[l] * y[w];
      }
      cx<C> zs[W];
#pragma unroll
      for (int w = 0; w < W; w++) {
        typename St<P>::pair_t v;
        St<P>::st(&v, 0, cx<C>{(C)z[w].re, (C)z[w].im});
        zs[w] = St<P>::ld(&v, 0);
      }
      st_group<P>(a.dst[tr].data + gi * W, zs);
      if (tr == 0 && a.want_norms) {
        cx<double> wv[W];
        if (a.has_w) ldg_group<P>(a.w.data, gi, wv);
#pragma unroll
        for (int w = 0; w < W; w++) {
          cx<double> q{(double)zs[w].re, (double)zs[w].im};
          nn += norm2(q);
          if (a.has_w) {
            cx<double> c = cmulc(q, wv[w]);
            wr += c.re;
            wi += c.im;
          }
        }
      }
    }
  }
  if (a.want_norms) {
    const double v3[3] = {nn, wr, wi};
    block_sums<3>(v3, sh, partial + blockIdx.x, gridDim.x);
  }
}

// the site range [first, first + count) of views starting at site `off` is
// whole runs: the flat forms apply (group range returned)
template <int P>
bool flat_range(const SpinorArg &x, int64_t first, int64_t count, int64_t *g0, int64_t *ng) {
  if (St<P>::scaled) return false;
  const int64_t R = x.rd.R;
  const int64_t j0 = first - x.off;
  if (R < 1 || j0 < 0 || j0 % R || count % R) return false;
  *g0 = j0 * 12 / VW<P>;
  *ng = count * 12 / VW<P>;
  return true;
}
template <int P>
bool same_offset(const SpinorArg &a, const SpinorArg &x) {
  return a.off == x.off && a.rd.R == x.rd.R;
}

// --- batched Gram-Schmidt (GsSlot) ------------------------------------------

// one 16-byte group of a flat vector whose base pointer was read from a table
template <int P>
__device__ __forceinline__ void gld_grp(const typename St<P>::pair_t *base, int64_t gi, cx<double> out[VW<P>]) {
  using R = typename RawOf<16>::type;
  const R r = gld((const R *)base, gi);
  typename St<P>::pair_t v[VW<P>];
  __builtin_memcpy(v, &r, 16);
#pragma unroll
  for (int w = 0; w < VW<P>; w++) {
    const auto z = St<P>::ld(v, w);
    out[w] = {(double)z.re, (double)z.im};
  }
}
// store a group rounded to the storage precision; `stored` = what was written
template <int P>
__device__ __forceinline__ void gst_grp(typename St<P>::pair_t *base, int64_t gi, const cx<double> in[VW<P>],
                                        cx<double> stored[VW<P>]) {
  using R = typename RawOf<16>::type;
  using C = typename St<P>::comp_t;
  typename St<P>::pair_t v[VW<P>];
#pragma unroll
  for (int w = 0; w < VW<P>; w++) {
    St<P>::st(v, w, cx<C>{(C)in[w].re, (C)in[w].im});
    const auto z = St<P>::ld(v, w);
    stored[w] = {(double)z.re, (double)z.im};
  }
  R r;
  __builtin_memcpy(&r, v, 16);
  gst((R *)base, gi, r);
}

constexpr int GS_CH = 8;  // vectors per sweep of the dot kernel

template <int P>
__device__ __forceinline__ typename St<P>::pair_t *vec_at(const GsSlot<P> &s, int l) {
  return (typename St<P>::pair_t *)((char *)s.chi0 + (int64_t)l * s.vstride_bytes);
}
template <int P>
__device__ __forceinline__ Spinor<P> vec_view(const GsSlot<P> &s, int l, int64_t nsites, const RunDiv &rd) {
  return spinor_view<P>(vec_at(s, l), nsites, 0, rd);
}

// partial[(y * 2 MAXV + 2l (+1)) * gx + bx] = block sums of (chi_l, chi_k)
template <int P>
__global__ void __launch_bounds__(BT) gs_dot_kernel(const GsSlot<P> *slots, int64_t ng, double *partial) {
  constexpr int W = VW<P>;
  __shared__ double sh[4 * 2 * GS_CH];
  const GsSlot<P> s = slots[blockIdx.y];
  const int k = s.k, gx = gridDim.x;
  double *pp = partial + (int64_t)blockIdx.y * 2 * MAXV * gx + blockIdx.x;
  const typename St<P>::pair_t *xk = vec_at(s, k);
  for (int c0 = 0; c0 < k; c0 += GS_CH) {
    const int m = k - c0 < GS_CH ? k - c0 : GS_CH;
    double acc[2 * GS_CH];
#pragma unroll
    for (int j = 0; j < 2 * GS_CH; j++) acc[j] = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < ng; t += (int64_t)gx * BT) {
      cx<double> xv[W];
      gld_grp<P>(xk, t, xv);
#pragma unroll
      for (int l = 0; l < GS_CH; l++) {
        if (l < m) {
          cx<double> yv[W];
          gld_grp<P>(vec_at(s, c0 + l), t, yv);
#pragma unroll
          for (int w = 0; w < W; w++) {
            acc[2 * l] = fmat(yv[w].re, xv[w].re, acc[2 * l]);
            acc[2 * l] = fmat(yv[w].im, xv[w].im, acc[2 * l]);
            acc[2 * l + 1] = fmat(yv[w].re, xv[w].im, acc[2 * l + 1]);
            acc[2 * l + 1] = fmat(-yv[w].im, xv[w].re, acc[2 * l + 1]);
          }
        }
      }
    }
    // block sums of the 2m values (wavefront trees, then the 4 wavefronts)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 2 * GS_CH; j++) {
      double x = acc[j];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (lane == 0) sh[4 * j + wv] = x;
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * m) {
      const int j = threadIdx.x;
      pp[(int64_t)(2 * c0 + j) * gx] = (sh[4 * j] + sh[4 * j + 1]) + (sh[4 * j + 2] + sh[4 * j + 3]);
    }
    __syncthreads();
  }
}

// chi_k -= sum_l ak_l chi_l (second: ak2_l); partial values 0..2 = |chi_k|^2, (chi_k, rho)
template <int P>
__global__ void __launch_bounds__(BT) gs_axpy_kernel(const GsSlot<P> *slots, int64_t ng, double *partial, int second) {
  constexpr int W = VW<P>;
  __shared__ double sh[12];
  __shared__ double cfs[2 * MAXV];  // the coefficients ak, read once per work-group
  const GsSlot<P> s = slots[blockIdx.y];
  const int k = s.k, gx = gridDim.x;
  typename St<P>::pair_t *xk = vec_at(s, k);
  const double *cf_src = second ? s.ak2 : s.ak;
  for (int j = threadIdx.x; j < 2 * k; j += BT) cfs[j] = gld(cf_src, j);
  __syncthreads();
  double nn = 0.0, wr = 0.0, wi = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < ng; t += (int64_t)gx * BT) {
    cx<double> z[W];
    gld_grp<P>(xk, t, z);
#pragma unroll 4
    for (int l = 0; l < k; l++) {
      const cx<double> cf{cfs[2 * l], cfs[2 * l + 1]};
      cx<double> y[W];
      gld_grp<P>(vec_at(s, l), t, y);
#pragma unroll
      for (int w = 0; w < W; w++) z[w] = z[w] - cf * y[w];
    }
    cx<double> zs[W], rv[W];
    gst_grp<P>(xk, t, z, zs);
    gld_grp<P>(s.rho, t, rv);
#pragma unroll
    for (int w = 0; w < W; w++) {
      nn += norm2(zs[w]);
      const cx<double> c = cmulc(zs[w], rv[w]);
      wr += c.re;
      wi += c.im;
    }
  }
  const double v3[3] = {nn, wr, wi};
  block_sums<3>(v3, sh, partial + (int64_t)blockIdx.y * 2 * MAXV * gx + blockIdx.x, gx);
}

// rho -= (rec[3k+1..2] / rec[3k]) chi_k; partial value 0 = |rho|^2
template <int P>
__global__ void __launch_bounds__(BT) gs_update_kernel(const GsSlot<P> *slots, int64_t ng, double *partial) {
  constexpr int W = VW<P>;
  __shared__ double sh[4];
  const GsSlot<P> s = slots[blockIdx.y];
  const int k = s.k, gx = gridDim.x;
  const typename St<P>::pair_t *xk = vec_at(s, k);
  const double d = gld(s.rec, 3 * k);
  const cx<double> c{gld(s.rec, 3 * k + 1) / d, gld(s.rec, 3 * k + 2) / d};
  double nn = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * BT + threadIdx.x; t < ng; t += (int64_t)gx * BT) {
    cx<double> r[W], x[W], rs[W];
    gld_grp<P>(s.rho, t, r);
    gld_grp<P>(xk, t, x);
#pragma unroll
    for (int w = 0; w < W; w++) r[w] = r[w] - c * x[w];
    gst_grp<P>(s.rho, t, r, rs);
#pragma unroll
    for (int w = 0; w < W; w++) nn += norm2(rs[w]);
  }
  const double v1[1] = {nn};
  block_sums<1>(v1, sh, partial + (int64_t)blockIdx.y * 2 * MAXV * gx + blockIdx.x, gx);
}

// One site per thread (vectors with per-site scales): the three phases of
// gs_dot_kernel, gs_axpy_kernel and gs_update_kernel, with whole spinors
// loaded and stored through the scaled format.
template <int P>
__global__ void __launch_bounds__(BT) gs_dot_site_kernel(const GsSlot<P> *slots, int64_t nsites, RunDiv rd, double *partial) {
  __shared__ double sh[4 * 2 * GS_CH];
  const GsSlot<P> s = slots[blockIdx.y];
  const int k = s.k, gx = gridDim.x;
  double *pp = partial + (int64_t)blockIdx.y * 2 * MAXV * gx + blockIdx.x;
  const Spinor<P> xk = vec_view(s, k, nsites, rd);
  for (int c0 = 0; c0 < k; c0 += GS_CH) {
    const int m = k - c0 < GS_CH ? k - c0 : GS_CH;
    double acc[2 * GS_CH];
#pragma unroll
    for (int j = 0; j < 2 * GS_CH; j++) acc[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < nsites; i += (int64_t)gx * BT) {
      cx<double> x[4][3];
      load_spinor<P, double>(xk, i, x);
#pragma unroll
      for (int l = 0; l < GS_CH; l++) {
        if (l < m) {
          cx<double> y[4][3];
          load_spinor<P, double>(vec_view(s, c0 + l, nsites, rd), i, y);
#pragma unroll
          for (int a = 0; a < 4; a++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
              acc[2 * l] = fmat(y[a][c].re, x[a][c].re, acc[2 * l]);
              acc[2 * l] = fmat(y[a][c].im, x[a][c].im, acc[2 * l]);
              acc[2 * l + 1] = fmat(y[a][c].re, x[a][c].im, acc[2 * l + 1]);
              acc[2 * l + 1] = fmat(-y[a][c].im, x[a][c].re, acc[2 * l + 1]);
            }
        }
      }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 2 * GS_CH; j++) {
      double x = acc[j];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (lane == 0) sh[4 * j + wv] = x;
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * m) {
      const int j = threadIdx.x;
      pp[(int64_t)(2 * c0 + j) * gx] = (sh[4 * j] + sh[4 * j + 1]) + (sh[4 * j + 2] + sh[4 * j + 3]);
    }
    __syncthreads();
  }
}

template <int P>
__global__ void __launch_bounds__(BT) gs_axpy_site_kernel(const GsSlot<P> *slots, int64_t nsites, RunDiv rd, double *partial,
                                                           int second) {
  __shared__ double sh[12];
  __shared__ double cfs[2 * MAXV];
  const GsSlot<P> s = slots[blockIdx.y];
  const int k = s.k, gx = gridDim.x;
  const Spinor<P> xk = vec_view(s, k, nsites, rd);
  const Spinor<P> rho = spinor_view<P>(s.rho, nsites, 0, rd);
  const double *cf_src = second ? s.ak2 : s.ak;
  for (int j = threadIdx.x; j < 2 * k; j += BT) cfs[j] = gld(cf_src, j);
  __syncthreads();
  double nn = 0.0, wr = 0.0, wi = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < nsites; i += (int64_t)gx * BT) {
    cx<double> z[4][3];
    load_spinor<P, double>(xk, i, z);
    for (int l = 0; l < k; l++) {
      const cx<double> cf{cfs[2 * l], cfs[2 * l + 1]};
      cx<double> y[4][3];
      load_spinor<P, double>(vec_view(s, l, nsites, rd), i, y);
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) z[a][c] = z[a][c] - cf * y[a][c];
    }
    store_spinor<P, double>(xk, i, z);
    cx<double> zs[4][3], rv[4][3];
    load_spinor<P, double>(xk, i, zs);  // the stored value, as a later read sees it
    load_spinor<P, double>(rho, i, rv);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int c = 0; c < 3; c++) {
        nn += norm2(zs[a][c]);
        const cx<double> q = cmulc(zs[a][c], rv[a][c]);
        wr += q.re;
        wi += q.im;
      }
  }
  const double v3[3] = {nn, wr, wi};
  block_sums<3>(v3, sh, partial + (int64_t)blockIdx.y * 2 * MAXV * gx + blockIdx.x, gx);
}

template <int P>
__global__ void __launch_bounds__(BT) gs_update_site_kernel(const GsSlot<P> *slots, int64_t nsites, RunDiv rd, double *partial) {
  __shared__ double sh[4];
  const GsSlot<P> s = slots[blockIdx.y];
  const int k = s.k, gx = gridDim.x;
  const Spinor<P> xk = vec_view(s, k, nsites, rd);
  const Spinor<P> rho = spinor_view<P>(s.rho, nsites, 0, rd);
  const double d = gld(s.rec, 3 * k);
  const cx<double> c{gld(s.rec, 3 * k + 1) / d, gld(s.rec, 3 * k + 2) / d};
  double nn = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < nsites; i += (int64_t)gx * BT) {
    cx<double> r[4][3], x[4][3];
    load_spinor<P, double>(rho, i, r);
    load_spinor<P, double>(xk, i, x);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) r[a][b] = r[a][b] - c * x[a][b];
    store_spinor<P, double>(rho, i, r);
    load_spinor<P, double>(rho, i, r);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) nn += norm2(r[a][b]);
  }
  const double v1[1] = {nn};
  block_sums<1>(v1, sh, partial + (int64_t)blockIdx.y * 2 * MAXV * gx + blockIdx.x, gx);
}

// Per slot (one work-group each): add the partial sums of a phase in a fixed
// order and write the results.  phase 0: ak_l = dot_l / rec[3l] (l < k);
// phase 1: rec[3k..3k+2]; phase 2: *norm; phase 3: ak2_l = dot_l / rec[3l]
// and ak_l += ak2_l (l < k).
template <int P>
__global__ void __launch_bounds__(BT) gs_finish_kernel(const GsSlot<P> *slots, int gx, const double *partial, int phase) {
  constexpr int K = 16;
  __shared__ double sh[4 * K], res[K];
  const GsSlot<P> s = slots[blockIdx.x];
  const int k = s.k;
  const int nval = (phase == 0 || phase == 3) ? 2 * k : (phase == 1 ? 3 : 1);
  const double *pp = partial + (int64_t)blockIdx.x * 2 * MAXV * gx;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int v0 = 0; v0 < nval; v0 += K) {
    const int m = nval - v0 < K ? nval - v0 : K;
#pragma unroll
    for (int j = 0; j < K; j++) {
      double x = 0.0;
      if (j < m)
        for (int b = threadIdx.x; b < gx; b += BT) x += pp[(int64_t)(v0 + j) * gx + b];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (lane == 0) sh[4 * j + wv] = x;
    }
    __syncthreads();
    if ((int)threadIdx.x < m) {
      const int j = threadIdx.x;
      res[j] = (sh[4 * j] + sh[4 * j + 1]) + (sh[4 * j + 2] + sh[4 * j + 3]);
    }
    __syncthreads();
    if ((int)threadIdx.x < m) {
      const int j = threadIdx.x, v = v0 + j;
      if (phase == 0) {
        gst(s.ak, v, res[j] / gld(s.rec, 3 * (v >> 1)));
      } else if (phase == 3) {
        const double a2 = res[j] / gld(s.rec, 3 * (v >> 1));
        gst(s.ak2, v, a2);
        gst(s.ak, v, gld(s.ak, v) + a2);
      } else if (phase == 1)
        gst(s.rec, 3 * k + v, res[j]);
      else
        gst(s.norm, 0, res[j]);
    }
    __syncthreads();
  }
}

// Shaped like one FP64 spinor site of the block-major fields: thread (c, t)
// of 4 KB-plane chunk c reads the 12 NR planes of src chunk c at position t
// and writes 12 planes of dst chunk c, plane p = xor of input planes
// p, p + 12, ..., p + 12 (NR - 1); every byte read or written once, streamed
template <int NR>
__global__ void __launch_bounds__(256) stream_kernel(const typename RawOf<16>::type *src,
                                                     typename RawOf<16>::type *dst, int64_t nchunk) {
  using R = typename RawOf<16>::type;
  const int64_t c = blockIdx.x;
  if (c >= nchunk) return;
  const R *s = src + c * 12 * NR * 256 + threadIdx.x;
  R acc[12];
#pragma unroll
  for (int p = 0; p < 12; p++) acc[p] = __builtin_nontemporal_load(s + p * 256);
#pragma unroll
  for (int k = 12; k < 12 * NR; k++) acc[k % 12] ^= __builtin_nontemporal_load(s + k * 256);
  R *d = dst + c * 12 * 256 + threadIdx.x;
#pragma unroll
  for (int p = 0; p < 12; p++) __builtin_nontemporal_store(acc[p], d + p * 256);
}

}  // namespace

hipError_t launch_stream(const void *src, void *dst, size_t dst_bytes, int reads_per_write, hipStream_t st) {
  using R = typename RawOf<16>::type;
  const int64_t nchunk = (int64_t)(dst_bytes / (12 * 4096));
  if (nchunk == 0) return hipSuccess;
  if (nchunk > 0x7fffffff) return hipErrorInvalidValue;
  const R *s = (const R *)src;
  R *d = (R *)dst;
  const unsigned grid = (unsigned)nchunk;
  switch (reads_per_write) {
    case 1: stream_kernel<1><<<grid, 256, 0, st>>>(s, d, nchunk); break;
    case 2: stream_kernel<2><<<grid, 256, 0, st>>>(s, d, nchunk); break;
    case 4: stream_kernel<4><<<grid, 256, 0, st>>>(s, d, nchunk); break;
    case 5: stream_kernel<5><<<grid, 256, 0, st>>>(s, d, nchunk); break;
    case 6: stream_kernel<6><<<grid, 256, 0, st>>>(s, d, nchunk); break;
    case 7: stream_kernel<7><<<grid, 256, 0, st>>>(s, d, nchunk); break;
    case 8: stream_kernel<8><<<grid, 256, 0, st>>>(s, d, nchunk); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t finish(const double *partial, int nblk, int nred, double *out, const double *div,
                  int div_stride, hipStream_t st) {
  finish_kernel<<<1, BT, 0, st>>>(partial, nblk, nred, out, div, div_stride);
  return hipGetLastError();
}

template <int P>
hipError_t blas_mdot(const SpinorArg *ys, int n, SpinorArg x, int64_t first, int64_t count,
                     double *partial, double *out, const double *div, int div_stride, hipStream_t st) {
  if (n < 1 || n > MAXV) return hipErrorInvalidValue;
  unsigned g = red_grid(count);
  Spinor<P> xv = view<P>(x);
  int64_t g0 = 0, ng = 0;
  bool flat = flat_range<P>(x, first, count, &g0, &ng);
  for (int k = 0; k < n && flat; k++) flat = same_offset<P>(ys[k], x);
  if (flat) g = red_grid(ng);  // one thread per 16-byte group where the vector is short
  for (int c0 = 0; c0 < n; c0 += CHUNK) {
    int m = n - c0 < CHUNK ? n - c0 : CHUNK;
    VecList<P> l;
    for (int k = 0; k < m; k++) l.v[k] = view<P>(ys[c0 + k]);
    int base = 2 * c0;
    if (flat) {
      switch (m) {
#define QXD_CASE(N) case N: mdot_flat_kernel<P, N><<<g, BT, 0, st>>>(l, xv, g0, ng, partial, base); break;
        QXD_CASE(1) QXD_CASE(2) QXD_CASE(3) QXD_CASE(4) QXD_CASE(5) QXD_CASE(6) QXD_CASE(7) QXD_CASE(8)
#undef QXD_CASE
      }
      continue;
    }
    switch (m) {
#define QXD_CASE(N) case N: mdot_kernel<P, N><<<g, BT, 0, st>>>(l, xv, first, count, partial, base); break;
      QXD_CASE(1) QXD_CASE(2) QXD_CASE(3) QXD_CASE(4) QXD_CASE(5) QXD_CASE(6) QXD_CASE(7) QXD_CASE(8)
#undef QXD_CASE
    }
  }
  return finish(partial, g, 2 * n, out, div, div_stride, st);
}

template <int P>
hipError_t blas_maxpy(const MaxpyHost &h, int64_t first, int64_t count, double *partial, double *out,
                      hipStream_t st) {
  if (h.n < 0 || h.n > MAXV || h.ntriples < 1 || h.ntriples > 2) return hipErrorInvalidValue;
  unsigned g = red_grid(count);
  int64_t g0 = 0, ng = 0;
  bool flat = flat_range<P>(h.dst[0], first, count, &g0, &ng);
  for (int tr = 0; tr < h.ntriples && flat; tr++) {
    flat = same_offset<P>(h.src[tr], h.dst[0]) && same_offset<P>(h.dst[tr], h.dst[0]);
    for (int k = 0; k < h.n && flat; k++) flat = same_offset<P>(h.ys[tr][k], h.dst[0]);
  }
  if (flat && h.w.ptr) flat = same_offset<P>(h.w, h.dst[0]);
  if (flat) g = red_grid(ng);  // one thread per 16-byte group where the vector is short
  int c0 = 0;
  do {
    int m = h.n - c0 < CHUNK ? h.n - c0 : CHUNK;
    bool last = c0 + m >= h.n;
    MaxpyArgs<P> a;
    a.ntriples = h.ntriples;
    for (int tr = 0; tr < h.ntriples; tr++) {
      a.src[tr] = view<P>(c0 == 0 ? h.src[tr] : h.dst[tr]);
      a.dst[tr] = view<P>(h.dst[tr]);
      for (int k = 0; k < m; k++) a.ys[tr].v[k] = view<P>(h.ys[tr][c0 + k]);
    }
    a.coef = h.coef;
    a.div = h.div;
    a.div_stride = h.div_stride;
    a.coef_base = c0;
    a.want_norms = last && out != nullptr;
    a.has_w = h.w.ptr != nullptr;
    a.w = a.has_w ? view<P>(h.w) : Spinor<P>{nullptr, nullptr, 0, RunDiv{}};
    if (flat) {
      switch (m) {
#define QXD_CASE(N) case N: maxpy_flat_kernel<P, N><<<g, BT, 0, st>>>(a, g0, ng, partial); break;
        QXD_CASE(0) QXD_CASE(1) QXD_CASE(2) QXD_CASE(3) QXD_CASE(4) QXD_CASE(5) QXD_CASE(6) QXD_CASE(7) QXD_CASE(8)
#undef QXD_CASE
      }
      c0 += m;
      continue;
    }
    switch (m) {
#define QXD_CASE(N) case N: maxpy_kernel<P, N><<<g, BT, 0, st>>>(a, first, count, partial); break;
      QXD_CASE(0) QXD_CASE(1) QXD_CASE(2) QXD_CASE(3) QXD_CASE(4) QXD_CASE(5) QXD_CASE(6) QXD_CASE(7) QXD_CASE(8)
#undef QXD_CASE
    }
    c0 += m;
  } while (c0 < h.n);
  if (!out) return hipGetLastError();
  return finish(partial, g, 3, out, nullptr, 0, st);
}

template <int P>
hipError_t blas_update(SpinorArg y, SpinorArg x, const double *num, const double *den, int negate,
                       int64_t first, int64_t count, double *partial, double *out, hipStream_t st) {
  unsigned g = red_grid(count);
  update_kernel<P><<<g, BT, 0, st>>>(view<P>(y), view<P>(x), num, den, negate, first, count, partial);
  return finish(partial, g, 1, out, nullptr, 0, st);
}

template <int Q, int P>
hipError_t blas_axpby(SpinorArg y, double a, SpinorArg x, double b, int64_t first, int64_t count,
                      double *partial, double *out, hipStream_t st) {
  unsigned g = red_grid(count);
  axpby_kernel<Q, P><<<g, BT, 0, st>>>(view<Q>(y), a, view<P>(x), b, first, count, out ? partial : nullptr);
  if (!out) return hipGetLastError();
  return finish(partial, g, 1, out, nullptr, 0, st);
}

template <int P>
hipError_t blas_norm2(SpinorArg x, int64_t first, int64_t count, double *partial, double *out,
                      hipStream_t st) {
  unsigned g = red_grid(count);
  norm_kernel<P><<<g, BT, 0, st>>>(view<P>(x), first, count, partial);
  return finish(partial, g, 1, out, nullptr, 0, st);
}

#define QXD_INST(P)                                                                              \
  template hipError_t blas_mdot<P>(const SpinorArg *, int, SpinorArg, int64_t, int64_t, double *, \
                                   double *, const double *, int, hipStream_t);                   \
  template hipError_t blas_maxpy<P>(const MaxpyHost &, int64_t, int64_t, double *, double *,     \
                                    hipStream_t);                                                \
  template hipError_t blas_update<P>(SpinorArg, SpinorArg, const double *, const double *, int,  \
                                     int64_t, int64_t, double *, double *, hipStream_t);          \
  template hipError_t blas_norm2<P>(SpinorArg, int64_t, int64_t, double *, double *, hipStream_t);
QXD_INST(QXD_F64)
QXD_INST(QXD_F32)
QXD_INST(QXD_F16S)
QXD_INST(QXD_BF16)
#undef QXD_INST

#define QXD_INST2(Q, P)                                                                       \
  template hipError_t blas_axpby<Q, P>(SpinorArg, double, SpinorArg, double, int64_t, int64_t, \
                                       double *, double *, hipStream_t);
QXD_INST2(QXD_F64, QXD_F64)
QXD_INST2(QXD_F64, QXD_F32)
QXD_INST2(QXD_F64, QXD_F16S)
QXD_INST2(QXD_F64, QXD_BF16)
QXD_INST2(QXD_F32, QXD_F64)
QXD_INST2(QXD_F16S, QXD_F64)
QXD_INST2(QXD_BF16, QXD_F64)
QXD_INST2(QXD_F32, QXD_F32)
QXD_INST2(QXD_F16S, QXD_F16S)
QXD_INST2(QXD_BF16, QXD_BF16)
#undef QXD_INST2

// flat forms: one 16-byte group per thread; scaled vectors: one site per thread
unsigned gs_batch_grid(int prec, int64_t nsites) {
  if (prec == QXD_F16S) return red_grid(nsites);
  const int w = prec == QXD_F64 ? 1 : (prec == QXD_F32 ? 2 : 4);
  return red_grid(nsites * 12 / w);
}

template <int P>
hipError_t blas_gs_batch(const GsSlot<P> *slots, int n, int64_t nsites, const RunDiv &rd, double *partial,
                         int passes, hipStream_t st) {
  if (n < 1) return hipSuccess;
  if (passes != 1 && passes != 2) return hipErrorInvalidValue;
  const unsigned gx = gs_batch_grid(P, nsites);
  const dim3 grid(gx, (unsigned)n);
  if constexpr (St<P>::scaled) {
    gs_dot_site_kernel<P><<<grid, BT, 0, st>>>(slots, nsites, rd, partial);
    gs_finish_kernel<P><<<(unsigned)n, BT, 0, st>>>(slots, (int)gx, partial, 0);
    gs_axpy_site_kernel<P><<<grid, BT, 0, st>>>(slots, nsites, rd, partial, 0);
    if (passes == 2) {
      gs_dot_site_kernel<P><<<grid, BT, 0, st>>>(slots, nsites, rd, partial);
      gs_finish_kernel<P><<<(unsigned)n, BT, 0, st>>>(slots, (int)gx, partial, 3);
      gs_axpy_site_kernel<P><<<grid, BT, 0, st>>>(slots, nsites, rd, partial, 1);
    }
    gs_finish_kernel<P><<<(unsigned)n, BT, 0, st>>>(slots, (int)gx, partial, 1);
    gs_update_site_kernel<P><<<grid, BT, 0, st>>>(slots, nsites, rd, partial);
    gs_finish_kernel<P><<<(unsigned)n, BT, 0, st>>>(slots, (int)gx, partial, 2);
  } else {
    const int64_t ng = nsites * 12 / VW<P>;
    gs_dot_kernel<P><<<grid, BT, 0, st>>>(slots, ng, partial);
    gs_finish_kernel<P><<<(unsigned)n, BT, 0, st>>>(slots, (int)gx, partial, 0);
    gs_axpy_kernel<P><<<grid, BT, 0, st>>>(slots, ng, partial, 0);
    if (passes == 2) {
      gs_dot_kernel<P><<<grid, BT, 0, st>>>(slots, ng, partial);
      gs_finish_kernel<P><<<(unsigned)n, BT, 0, st>>>(slots, (int)gx, partial, 3);
      gs_axpy_kernel<P><<<grid, BT, 0, st>>>(slots, ng, partial, 1);
    }
    gs_finish_kernel<P><<<(unsigned)n, BT, 0, st>>>(slots, (int)gx, partial, 1);
    gs_update_kernel<P><<<grid, BT, 0, st>>>(slots, ng, partial);
    gs_finish_kernel<P><<<(unsigned)n, BT, 0, st>>>(slots, (int)gx, partial, 2);
  }
  return hipGetLastError();
}
#define QXD_INST(P)                                                                                       \
  template hipError_t blas_gs_batch<P>(const GsSlot<P> *, int, int64_t, const RunDiv &, double *, int, hipStream_t);
QXD_INST(QXD_F64)
QXD_INST(QXD_F32)
QXD_INST(QXD_F16S)
QXD_INST(QXD_BF16)
#undef QXD_INST

}  // namespace qxd
