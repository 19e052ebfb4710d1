// Kernels of the local deflation (declarations and the method in dfl.h).
//
// The basis fields are FP32 native spinors; every reduction is FP64 and
// deterministic (fixed work-group shapes, fixed summation order).  Block
// kernels run one work-group of DT threads per SAP block, one site per
// thread (blocks of at most DT sites).
#include "dfl.h"
#include "dirac_site.h"

namespace qxd {
namespace {

constexpr int DT = 256;          // threads of a block work-group
constexpr int NW = DT / 64;      // its wavefronts
constexpr int LVG = 256;         // work-groups of a little-vector reduction
constexpr int LV_MAXK = 64;      // most little Krylov vectors

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum of v over the work-group (every thread gets it); sh: NW doubles
__device__ __forceinline__ double wg_sum(double v, double *sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; w++) s += sh[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ void zero_sp(cx<double> v[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 3; c++) v[a][c] = {0.0, 0.0};
}

__device__ __forceinline__ cx<double> sp_dot(const cx<double> u[4][3], const cx<double> v[4][3]) {
  cx<double> d{0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 3; c++) d = d + cmulc(u[a][c], v[a][c]);
  return d;
}

__device__ __forceinline__ Spinor<QXD_F32> field_at(const Geom &g, const void *basis, size_t vbytes, int k) {
  return spinor_view<QXD_F32>((char *)basis + (size_t)k * vbytes, g.V, 0, g.rd);
}

// the native index of the site handled by thread t of block blk (both
// parities: t < Vbh even run, then odd run); false past the block
__device__ __forceinline__ bool block_site(const Geom &g, int blk, int t, int64_t &i) {
  if (t >= 2 * g.Vbh) return false;
  const int par = t >= g.Vbh;
  i = (int64_t)par * g.Vh + (int64_t)blk * g.Vbh + (t - par * g.Vbh);
  return true;
}

// splitmix64 (Steele, Lea, Flood 2014): a bijective mixing of a 64-bit counter
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(DT) dfl_random_kernel(Geom g, char *basis, size_t vbytes, int k, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * DT + threadIdx.x;
  if (i >= g.V) return;
  cx<double> v[4][3];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int c = 0; c < 3; c++) {
      // Box-Muller from two uniforms in (0, 1]
      const uint64_t ctr = (((uint64_t)k * (uint64_t)g.V + (uint64_t)i) * 12 + (uint64_t)(a * 3 + c));
      const uint64_t h1 = splitmix64(seed ^ splitmix64(2 * ctr)), h2 = splitmix64(seed ^ splitmix64(2 * ctr + 1));
      const double u1 = ((double)(h1 >> 11) + 1.0) * 0x1.0p-53, u2 = (double)(h2 >> 11) * 0x1.0p-53;
      const double r = sqrt(-2.0 * log(u1));
      double s, co;
      sincos(6.283185307179586 * u2, &s, &co);
      v[a][c] = {r * co, r * s};
    }
  store_spinor<QXD_F32, double>(field_at(g, basis, vbytes, k), i, v);
}

// modified Gram-Schmidt on one block: field k minus its projections on the
// (already orthonormal) fields j < k, then normalised
__global__ void __launch_bounds__(DT) dfl_ortho_kernel(Geom g, char *basis, size_t vbytes, int ns, int *bad) {
  __shared__ double sh[NW];
  const int blk = blockIdx.x;
  int64_t i = 0;
  const bool on = block_site(g, blk, threadIdx.x, i);
  bool vanished = false;
  for (int k = 0; k < ns; k++) {
    const Spinor<QXD_F32> fk = field_at(g, basis, vbytes, k);
    cx<double> v[4][3];
    if (on)
      load_spinor<QXD_F32, double>(fk, i, v);
    else
      zero_sp(v);
    for (int j = 0; j < k; j++) {
      cx<double> u[4][3];
      if (on)
        load_spinor<QXD_F32, double>(field_at(g, basis, vbytes, j), i, u);
      else
        zero_sp(u);
      const cx<double> d = sp_dot(u, v);
      const cx<double> c{wg_sum(d.re, sh), wg_sum(d.im, sh)};
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) v[a][b] = v[a][b] - c * u[a][b];
    }
    double n2 = 0.0;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) n2 += norm2(v[a][b]);
    n2 = wg_sum(n2, sh);
    const double f = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    if (!(n2 > 0.0)) vanished = true;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) v[a][b] = f * v[a][b];
    if (on) store_spinor<QXD_F32, double>(fk, i, v);
  }
  if (vanished && threadIdx.x == 0) atomicAdd(bad, 1);
}

// per-block dots of all ns basis vectors with the thread's vector h; the
// work-group sums land in sh_out[2k], sh_out[2k + 1] (after the barrier)
__device__ __forceinline__ void block_dots(const Geom &g, const void *basis, size_t vbytes, int ns, bool on,
                                           int64_t i, const cx<double> h[4][3], double *sh, double *sh_out) {
  for (int k = 0; k < ns; k++) {
    cx<double> u[4][3];
    if (on)
      load_spinor<QXD_F32, double>(field_at(g, basis, vbytes, k), i, u);
    else
      zero_sp(u);
    cx<double> d = sp_dot(u, h);
    d.re = wave_sum(d.re);
    d.im = wave_sum(d.im);
    if ((threadIdx.x & 63) == 0) {
      sh[(threadIdx.x >> 6) * 2 * DFL_NSMAX + 2 * k] = d.re;
      sh[(threadIdx.x >> 6) * 2 * DFL_NSMAX + 2 * k + 1] = d.im;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * ns) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; w++) s += sh[w * 2 * DFL_NSMAX + threadIdx.x];
    sh_out[threadIdx.x] = s;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(DT) dfl_restrict_kernel(Geom g, const char *basis, size_t vbytes, int ns,
                                                          const void *r, const int *vpos, double *c) {
  __shared__ double sh[NW * 2 * DFL_NSMAX];
  __shared__ double out[2 * DFL_NSMAX];
  const int blk = blockIdx.x;
  int64_t i = 0;
  const bool on = block_site(g, blk, threadIdx.x, i);
  cx<double> h[4][3];
  if (on)
    load_spinor<QXD_F32, double>(spinor_view<QXD_F32>((void *)r, g.V, 0, g.rd), i, h);
  else
    zero_sp(h);
  block_dots(g, basis, vbytes, ns, on, i, h, sh, out);
  if ((int)threadIdx.x < 2 * ns) c[(int64_t)vpos[blk] * 2 * ns + threadIdx.x] = out[threadIdx.x];
}

__global__ void __launch_bounds__(DT) dfl_prolong_kernel(Geom g, const char *basis, size_t vbytes, int ns,
                                                         const double2 *c, const int *vpos, void *out) {
  const int64_t i = (int64_t)blockIdx.x * DT + threadIdx.x;
  if (i >= g.V) return;
  const int64_t r = i >= g.Vh ? i - g.Vh : i;
  const int blk = (int)g.rd.div((uint32_t)r);
  const int64_t vb = vpos[blk];
  cx<double> acc[4][3];
  zero_sp(acc);
  for (int k = 0; k < ns; k++) {
    const double2 ck = c[vb * ns + k];
    const cx<double> cc{ck.x, ck.y};
    cx<double> u[4][3];
    load_spinor<QXD_F32, double>(field_at(g, basis, vbytes, k), i, u);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) acc[a][b] = acc[a][b] + cc * u[a][b];
  }
  store_spinor<QXD_F32, double>(spinor_view<QXD_F32>(out, g.V, 0, g.rd), i, acc);
}

// work-group (blk, d): the hops of D through face d = 2 mu + s of block blk
// (s = 0: to x + mu, s = 1: to x - mu) applied to basis field l, dotted with
// every basis vector of the block
__global__ void __launch_bounds__(DT) dfl_face_kernel(Geom g, const double2 *wl, const char *basis, size_t vbytes,
                                                      int ns, int l, double *a, int *nbr) {
  __shared__ double sh[NW * 2 * DFL_NSMAX];
  __shared__ double out[2 * DFL_NSMAX];
  const int blk = blockIdx.x, d = blockIdx.y;
  const int mu = d >> 1, dir = (d & 1) ? -1 : 1;
  const int bmu = (g.bpk >> (8 * mu)) & 0xff;
  int64_t i = 0;
  const bool in_block = block_site(g, blk, threadIdx.x, i);
  cx<double> h[4][3];
  zero_sp(h);
  bool on = false;
  if (in_block) {
    const Site s = decode(g, (int)i);
    if (s.y(mu) == (dir > 0 ? bmu - 1 : 0)) {
      int sg;
      const Site t = neighbour(g, s, mu, dir, sg);
      const int64_t j = encode(g, t);
      cx<double> psi[4][3], w[3][3];
      load_spinor<QXD_F32, double>(field_at(g, basis, vbytes, l), j, psi);
      load_link<QXD_F64, double>(wl, g, mu, dir > 0 ? i : j, w);
      if (dir > 0)
        hop_fwd<double>(mu, w, psi, -0.5 * sg, h);
      else
        hop_bwd<double>(mu, w, psi, -0.5 * sg, h);
      on = true;
    }
  }
  block_dots(g, basis, vbytes, ns, on, i, h, sh, out);
  const int64_t base = (((int64_t)blk * DFL_SLOTS + 1 + d) * ns) * ns;
  if ((int)threadIdx.x < 2 * ns) {
    const int k = threadIdx.x >> 1;
    a[2 * (base + (int64_t)k * ns + l) + (threadIdx.x & 1)] = out[threadIdx.x];
  }
  if (threadIdx.x == 0) {
    // the block across the face, from a face site of this block
    Site s = decode(g, (int)((int64_t)blk * g.Vbh));
    s.sety(mu, dir > 0 ? bmu - 1 : 0);
    int sg;
    nbr[blk * DFL_SLOTS + 1 + d] = block_index(g, neighbour(g, s, mu, dir, sg));
  }
}

__global__ void __launch_bounds__(DT) dfl_diag_kernel(Geom g, const char *basis, size_t vbytes, int ns, int l,
                                                      const void *y64, double *a, int *nbr) {
  __shared__ double sh[NW * 2 * DFL_NSMAX];
  __shared__ double out[2 * DFL_NSMAX];
  const int blk = blockIdx.x;
  int64_t i = 0;
  const bool on = block_site(g, blk, threadIdx.x, i);
  cx<double> h[4][3];
  if (on)
    load_spinor<QXD_F64, double>(spinor_view<QXD_F64>((void *)y64, g.V, 0, g.rd), i, h);
  else
    zero_sp(h);
  block_dots(g, basis, vbytes, ns, on, i, h, sh, out);
  if ((int)threadIdx.x < 2 * ns) {
    const int k = threadIdx.x >> 1, part = threadIdx.x & 1;
    double v = out[threadIdx.x];
    for (int d = 1; d < DFL_SLOTS; d++)
      v -= a[2 * ((((int64_t)blk * DFL_SLOTS + d) * ns + k) * ns + l) + part];
    a[2 * ((((int64_t)blk * DFL_SLOTS) * ns + k) * ns + l) + part] = v;
  }
  if (threadIdx.x == 0) nbr[blk * DFL_SLOTS] = blk;
}

// Gauss-Jordan with partial pivoting of the ns x ns block a[b][0] in LDS
__global__ void __launch_bounds__(DT) little_invert_kernel(int ns, const double2 *a, double2 *ainv, int *bad) {
  __shared__ double2 m[DFL_NSMAX][2 * DFL_NSMAX];
  __shared__ double2 col[DFL_NSMAX];
  __shared__ int piv;
  __shared__ double2 pinv;
  const int blk = blockIdx.x;
  const int w = 2 * ns;
  const double2 *ab = a + (int64_t)blk * DFL_SLOTS * ns * ns;
  for (int e = threadIdx.x; e < ns * w; e += DT) {
    const int r = e / w, c = e - r * w;
    m[r][c] = c < ns ? ab[r * ns + c] : make_double2(c - ns == r ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  bool singular = false;
  for (int p = 0; p < ns; p++) {
    if (threadIdx.x == 0) {
      int best = p;
      double bv = -1.0;
      for (int r = p; r < ns; r++) {
        const double v = m[r][p].x * m[r][p].x + m[r][p].y * m[r][p].y;
        if (v > bv) {
          bv = v;
          best = r;
        }
      }
      piv = best;
    }
    __syncthreads();
    const int q = piv;
    if (q != p)
      for (int c = threadIdx.x; c < w; c += DT) {
        const double2 t = m[p][c];
        m[p][c] = m[q][c];
        m[q][c] = t;
      }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double2 v = m[p][p];
      const double n = v.x * v.x + v.y * v.y;
      pinv = n > 0.0 ? make_double2(v.x / n, -v.y / n) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (pinv.x == 0.0 && pinv.y == 0.0) singular = true;
    for (int c = threadIdx.x; c < w; c += DT) {
      const double2 v = m[p][c];
      m[p][c] = make_double2(v.x * pinv.x - v.y * pinv.y, v.x * pinv.y + v.y * pinv.x);
    }
    for (int r = threadIdx.x; r < ns; r += DT) col[r] = m[r][p];
    __syncthreads();
    for (int e = threadIdx.x; e < ns * w; e += DT) {
      const int r = e / w, c = e - r * w;
      if (r == p) continue;
      const double2 f = col[r], v = m[p][c];
      m[r][c].x -= f.x * v.x - f.y * v.y;
      m[r][c].y -= f.x * v.y + f.y * v.x;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < ns * ns; e += DT) {
    const int r = e / ns, c = e - r * ns;
    ainv[(int64_t)blk * ns * ns + e] = m[r][ns + c];
  }
  if (singular && threadIdx.x == 0) atomicAdd(bad, 1);
}

// The little solve reads FP32 (or FP16) copies of A and FP32 copies of the
// inverse diagonal blocks, transposed within each ns x ns block (element
// (k, l) at l * ns + k), so that the threads of consecutive rows k read
// consecutive words.
__device__ __forceinline__ void to_mt(double2 v, float2 *d) { *d = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ void to_mt(double2 v, h2_t *d) {
  h2_t h;
  h.x = (_Float16)v.x;
  h.y = (_Float16)v.y;
  *d = h;
}
template <class MT>
__global__ void __launch_bounds__(DT) little_pack_kernel(int64_t nmat, int ns, const double2 *src, MT *dst) {
  const int64_t t = (int64_t)blockIdx.x * DT + threadIdx.x;
  if (t >= nmat * ns * ns) return;
  const int64_t m = t / (ns * ns);
  const int e = (int)(t - m * ns * ns), k = e / ns, l = e - k * ns;
  to_mt(src[t], dst + m * ns * ns + (int64_t)l * ns + k);
}

// Little products in column-streaming form: one work-group per block b of
// `list`, made of G = blockDim.x / ns groups of ns threads.  The block's
// transposed matrices are columns of ns complex numbers (FP32 or FP16),
// column c of slot d at c = d * ns + l holding A[b][d][k][l] for k = 0 ..
// ns-1; thread
// (g, k) takes the columns c = g, g + G, ... for its row k, so that the
// work-group reads the block's matrices front to back, and the G partial
// sums of a row are added in the order g = 0 .. G-1.  The vector entries
// the columns multiply are staged in LDS first.

// h_b = (xa ? A[b][0] xa_b : (w ? w_b : 0)) - sum_{d >= 1} A[b][d] xh[nbr[b][d]];
// y_b = h_b, or with INV y_b = s ainv[b] h_b (at: the transposed FP32 or
// FP16 copy of A; ait: the transposed FP32 copy of the inverse diagonal
// blocks)
template <bool DIAG, bool INV, class MT>
__global__ void __launch_bounds__(DT) lt_hop_kernel(const int *list, int vbase, int ns, const MT *at,
                                                    const int *nbrv, const double2 *xa, const double2 *w,
                                                    const double2 *xh, const float2 *ait, double s, double2 *y) {
  __shared__ double2 xs[DFL_SLOTS * DFL_NSMAX];
  __shared__ double2 red[DT];
  const int blk = list[blockIdx.x];               // the block (its matrices)
  const int64_t vb = vbase + (int64_t)blockIdx.x;  // its entries in the little vectors
  const int G = blockDim.x / ns, g = threadIdx.x / ns, k = threadIdx.x - g * ns;
  // column c multiplies xs[c]: xa_b for the diagonal slot, -xh at the block
  // across face d for the others
  for (int i = threadIdx.x; i < DFL_SLOTS * ns; i += blockDim.x) {
    const int d = i / ns, l = i - d * ns;
    double2 v = make_double2(0.0, 0.0);
    if (d == 0) {
      if (DIAG) v = xa[vb * ns + l];
    } else {
      v = xh[(int64_t)nbrv[blk * DFL_SLOTS + d] * ns + l];
      v.x = -v.x;
      v.y = -v.y;
    }
    xs[i] = v;
  }
  __syncthreads();
  const MT *m = at + (int64_t)blk * DFL_SLOTS * ns * ns + k;
  double re = 0.0, im = 0.0;
#pragma unroll 8
  for (int c = (DIAG ? 0 : ns) + g; c < DFL_SLOTS * ns; c += G) {
    const MT a = m[(int64_t)c * ns];
    const double2 v = xs[c];
    re += (double)a.x * v.x - (double)a.y * v.y;
    im += (double)a.x * v.y + (double)a.y * v.x;
  }
  red[threadIdx.x] = make_double2(re, im);
  __syncthreads();
  if (g == 0) {
    double2 h = make_double2(0.0, 0.0);
    if (!DIAG && w) h = w[vb * ns + k];
    for (int q = 0; q < G; q++) {
      h.x += red[q * ns + k].x;
      h.y += red[q * ns + k].y;
    }
    if (INV)
      xs[k] = h;  // every read of xs and red is done (the barrier above)
    else
      y[vb * ns + k] = h;
  }
  if (INV) {
    __syncthreads();
    const float2 *mi = ait + (int64_t)blk * ns * ns + k;
    re = 0.0;
    im = 0.0;
    for (int c = g; c < ns; c += G) {
      const float2 a = mi[(int64_t)c * ns];
      const double2 v = xs[c];
      re += (double)a.x * v.x - (double)a.y * v.y;
      im += (double)a.x * v.y + (double)a.y * v.x;
    }
    red[threadIdx.x] = make_double2(re, im);
    __syncthreads();
    if (g == 0) {
      double2 t = make_double2(0.0, 0.0);
      for (int q = 0; q < G; q++) {
        t.x += red[q * ns + k].x;
        t.y += red[q * ns + k].y;
      }
      y[vb * ns + k] = make_double2(s * t.x, s * t.y);
    }
  }
}

// y_b = s ainv[b] x_b for the blocks b of `list` (x and y distinct); ait:
// the transposed FP32 copy of the inverse diagonal blocks
__global__ void __launch_bounds__(DT) lt_jacobi_kernel(const int *list, int vbase, int ns, const float2 *ait,
                                                       double s, const double2 *x, double2 *y) {
  __shared__ double2 xs[DFL_NSMAX];
  __shared__ double2 red[DT];
  const int blk = list[blockIdx.x];
  const int64_t vb = vbase + (int64_t)blockIdx.x;
  const int G = blockDim.x / ns, g = threadIdx.x / ns, k = threadIdx.x - g * ns;
  if (threadIdx.x < ns) xs[threadIdx.x] = x[vb * ns + threadIdx.x];
  __syncthreads();
  const float2 *m = ait + (int64_t)blk * ns * ns + k;
  double re = 0.0, im = 0.0;
  for (int c = g; c < ns; c += G) {
    const float2 a = m[(int64_t)c * ns];
    const double2 v = xs[c];
    re += (double)a.x * v.x - (double)a.y * v.y;
    im += (double)a.x * v.y + (double)a.y * v.x;
  }
  red[threadIdx.x] = make_double2(re, im);
  __syncthreads();
  if (g == 0) {
    double2 t = make_double2(0.0, 0.0);
    for (int h = 0; h < G; h++) {
      t.x += red[h * ns + k].x;
      t.y += red[h * ns + k].y;
    }
    y[vb * ns + k] = make_double2(s * t.x, s * t.y);
  }
}

// ---- little-vector reductions: LVG work-groups, partial sums per group ------
// work-group (g, j): its share of (W_j, x)
__global__ void __launch_bounds__(DT) lv_dots_kernel(const double2 *W, int64_t n, const double2 *x,
                                                     double *partial) {
  __shared__ double sh[NW];
  const int j = blockIdx.y;
  const double2 *wj = W + (int64_t)j * n;
  double re = 0.0, im = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * DT + threadIdx.x; e < n; e += (int64_t)LVG * DT) {
    const double2 u = wj[e], v = x[e];
    re += u.x * v.x + u.y * v.y;
    im += u.x * v.y - u.y * v.x;
  }
  re = wg_sum(re, sh);
  im = wg_sum(im, sh);
  if (threadIdx.x == 0) {
    partial[(int64_t)(2 * j) * LVG + blockIdx.x] = re;
    partial[(int64_t)(2 * j + 1) * LVG + blockIdx.x] = im;
  }
}

__global__ void __launch_bounds__(DT) lv_dot2_kernel(const double2 *w, const double2 *r, int64_t n, double *partial) {
  __shared__ double sh[NW];
  double ww = 0.0, re = 0.0, im = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * DT + threadIdx.x; e < n; e += (int64_t)LVG * DT) {
    const double2 u = w[e], v = r[e];
    ww += u.x * u.x + u.y * u.y;
    re += u.x * v.x + u.y * v.y;
    im += u.x * v.y - u.y * v.x;
  }
  ww = wg_sum(ww, sh);
  re = wg_sum(re, sh);
  im = wg_sum(im, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = ww;
    partial[LVG + blockIdx.x] = re;
    partial[2 * LVG + blockIdx.x] = im;
  }
}

// out[v] = sum over the LVG groups of partial[v * LVG + group], in order
__global__ void __launch_bounds__(64) lv_finish_kernel(const double *partial, int nval, double *out) {
  const int v = blockIdx.x;
  double s = 0.0;
  for (int gi = threadIdx.x; gi < LVG; gi += 64) s += partial[(int64_t)v * LVG + gi];
  s = wave_sum(s);
  if (threadIdx.x == 0 && v < nval) out[v] = s;
}

// the same multi-axpy on two vector sets: x1 -= sum_j c_j W1_j, x2 -= sum_j c_j W2_j
__global__ void __launch_bounds__(DT) lv_maxpy2_kernel(double2 *x1, const double2 *W1, double2 *x2,
                                                       const double2 *W2, int k, int64_t n, const double *d,
                                                       const double *wn) {
  // the coefficients, once per work-group; wn[j] = |w_j|^2 is 0 only for
  // steps on a zero residual: no update
  __shared__ double cf[2 * LV_MAXK];
  for (int j = threadIdx.x; j < k; j += DT) {
    const double q = wn[j];
    cf[2 * j] = q != 0.0 ? d[2 * j] / q : 0.0;
    cf[2 * j + 1] = q != 0.0 ? d[2 * j + 1] / q : 0.0;
  }
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * DT + threadIdx.x;
  if (e >= n) return;
  double2 v1 = x1[e], v2 = x2[e];
  for (int j = 0; j < k; j++) {
    const double cr = cf[2 * j], ci = cf[2 * j + 1];
    const double2 u1 = W1[(int64_t)j * n + e], u2 = W2[(int64_t)j * n + e];
    v1.x -= cr * u1.x - ci * u1.y;
    v1.y -= cr * u1.y + ci * u1.x;
    v2.x -= cr * u2.x - ci * u2.y;
    v2.y -= cr * u2.y + ci * u2.x;
  }
  x1[e] = v1;
  x2[e] = v2;
}

// the sums of lv_dot2_kernel's partials (as lv_finish_kernel adds them) are
// formed by every work-group's first wavefront; the update's own partial
// sums of |r|^2 go to rpart
__global__ void __launch_bounds__(DT) lv_update_kernel(double2 *x, const double2 *z, double2 *r, const double2 *w,
                                                       int64_t n, const double *spart, double *wn, double *rpart) {
  __shared__ double sh[NW];
  __shared__ double s[3];
  if (threadIdx.x < 64) {
    for (int v = 0; v < 3; v++) {
      double t = 0.0;
      for (int gi = threadIdx.x; gi < LVG; gi += 64) t += spart[(int64_t)v * LVG + gi];
      t = wave_sum(t);
      if (threadIdx.x == 0) s[v] = t;
    }
  }
  __syncthreads();
  // s[0] = |w|^2 is 0 only for a step on a zero residual: no update
  const double ar = s[0] != 0.0 ? s[1] / s[0] : 0.0, ai = s[0] != 0.0 ? s[2] / s[0] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *wn = s[0];
  double rr = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * DT + threadIdx.x; e < n; e += (int64_t)LVG * DT) {
    const double2 zv = z[e], wv = w[e];
    double2 xv = x[e], rv = r[e];
    xv.x += ar * zv.x - ai * zv.y;
    xv.y += ar * zv.y + ai * zv.x;
    rv.x -= ar * wv.x - ai * wv.y;
    rv.y -= ar * wv.y + ai * wv.x;
    x[e] = xv;
    r[e] = rv;
    rr += rv.x * rv.x + rv.y * rv.y;
  }
  rr = wg_sum(rr, sh);
  if (threadIdx.x == 0) rpart[blockIdx.x] = rr;
}

bool fits(const Geom &g) { return 2 * g.Vbh <= DT; }

}  // namespace

size_t lv_partial_doubles() { return (size_t)2 * LV_MAXK * LVG + 8; }
static_assert(2 * LV_MAXK >= 4, "lv_update's partial sums follow lv_dot2's");

hipError_t launch_dfl_random(const Geom &g, void *basis, size_t vbytes, int ns, uint64_t seed, hipStream_t st) {
  for (int k = 0; k < ns; k++)
    dfl_random_kernel<<<grid_for(g.V, DT), DT, 0, st>>>(g, (char *)basis, vbytes, k, seed);
  return hipGetLastError();
}

hipError_t launch_dfl_ortho(const Geom &g, void *basis, size_t vbytes, int ns, int *bad, hipStream_t st) {
  if (!fits(g) || ns > DFL_NSMAX) return hipErrorInvalidValue;
  dfl_ortho_kernel<<<g.nblocks, DT, 0, st>>>(g, (char *)basis, vbytes, ns, bad);
  return hipGetLastError();
}

hipError_t launch_dfl_restrict(const Geom &g, const void *basis, size_t vbytes, int ns, const void *r,
                               const int *vpos, double2 *c, hipStream_t st) {
  if (!fits(g) || ns > DFL_NSMAX) return hipErrorInvalidValue;
  dfl_restrict_kernel<<<g.nblocks, DT, 0, st>>>(g, (const char *)basis, vbytes, ns, r, vpos, (double *)c);
  return hipGetLastError();
}

hipError_t launch_dfl_prolong(const Geom &g, const void *basis, size_t vbytes, int ns, const double2 *c,
                              const int *vpos, void *out, hipStream_t st) {
  dfl_prolong_kernel<<<grid_for(g.V, DT), DT, 0, st>>>(g, (const char *)basis, vbytes, ns, c, vpos, out);
  return hipGetLastError();
}

hipError_t launch_dfl_face(const Geom &g, const double2 *wl64, const void *basis, size_t vbytes, int ns, int l,
                           double2 *a, int *nbr, hipStream_t st) {
  if (!fits(g) || ns > DFL_NSMAX) return hipErrorInvalidValue;
  dfl_face_kernel<<<dim3(g.nblocks, 8), DT, 0, st>>>(g, wl64, (const char *)basis, vbytes, ns, l, (double *)a, nbr);
  return hipGetLastError();
}

hipError_t launch_dfl_diag(const Geom &g, const void *basis, size_t vbytes, int ns, int l, const void *y64,
                           double2 *a, int *nbr, hipStream_t st) {
  if (!fits(g) || ns > DFL_NSMAX) return hipErrorInvalidValue;
  dfl_diag_kernel<<<g.nblocks, DT, 0, st>>>(g, (const char *)basis, vbytes, ns, l, y64, (double *)a, nbr);
  return hipGetLastError();
}

hipError_t launch_little_invert(int nb, int ns, const double2 *a, double2 *ainv, int *bad, hipStream_t st) {
  if (ns > DFL_NSMAX) return hipErrorInvalidValue;
  little_invert_kernel<<<nb, DT, 0, st>>>(ns, a, ainv, bad);
  return hipGetLastError();
}

template <class MT>
hipError_t launch_little_pack(int64_t nmat, int ns, const double2 *src, MT *dst, hipStream_t st) {
  little_pack_kernel<MT><<<grid_for(nmat * ns * ns, DT), DT, 0, st>>>(nmat, ns, src, dst);
  return hipGetLastError();
}
template hipError_t launch_little_pack<float2>(int64_t, int, const double2 *, float2 *, hipStream_t);
template hipError_t launch_little_pack<h2_t>(int64_t, int, const double2 *, h2_t *, hipStream_t);

// work-group size of the column-streaming little products: a whole number
// of ns-thread groups, at most DT threads
static int lt_threads(int ns) { return (DT / ns) * ns; }

template <class MT>
hipError_t launch_lt_hop(const int *list, int nlist, int vbase, int ns, const MT *at, const int *nbrv,
                         const double2 *xa, const double2 *w, const double2 *xh, const float2 *ait, double s,
                         double2 *y, hipStream_t st) {
  if (ns < 1 || ns > DFL_NSMAX) return hipErrorInvalidValue;
  if (nlist < 1) return hipSuccess;
  const int nt = lt_threads(ns);
  if (xa && ait)
    lt_hop_kernel<true, true, MT><<<nlist, nt, 0, st>>>(list, vbase, ns, at, nbrv, xa, w, xh, ait, s, y);
  else if (xa)
    lt_hop_kernel<true, false, MT><<<nlist, nt, 0, st>>>(list, vbase, ns, at, nbrv, xa, w, xh, ait, s, y);
  else if (ait)
    lt_hop_kernel<false, true, MT><<<nlist, nt, 0, st>>>(list, vbase, ns, at, nbrv, xa, w, xh, ait, s, y);
  else
    lt_hop_kernel<false, false, MT><<<nlist, nt, 0, st>>>(list, vbase, ns, at, nbrv, xa, w, xh, ait, s, y);
  return hipGetLastError();
}
template hipError_t launch_lt_hop<float2>(const int *, int, int, int, const float2 *, const int *, const double2 *,
                                          const double2 *, const double2 *, const float2 *, double, double2 *,
                                          hipStream_t);
template hipError_t launch_lt_hop<h2_t>(const int *, int, int, int, const h2_t *, const int *, const double2 *,
                                        const double2 *, const double2 *, const float2 *, double, double2 *,
                                        hipStream_t);

hipError_t launch_lt_jacobi(const int *list, int nlist, int vbase, int ns, const float2 *ait, double s,
                            const double2 *x, double2 *y, hipStream_t st) {
  if (ns < 1 || ns > DFL_NSMAX) return hipErrorInvalidValue;
  if (nlist < 1) return hipSuccess;
  // about four columns per thread: a block's inverse is only ns x ns
  lt_jacobi_kernel<<<nlist, ns * ((ns + 3) / 4), 0, st>>>(list, vbase, ns, ait, s, x, y);
  return hipGetLastError();
}

hipError_t launch_lv_dots(const double2 *W, int k, int64_t n, const double2 *x, double *partial, double *out,
                          hipStream_t st) {
  if (k < 1 || k > LV_MAXK) return hipErrorInvalidValue;
  lv_dots_kernel<<<dim3(LVG, k), DT, 0, st>>>(W, n, x, partial);
  lv_finish_kernel<<<2 * k, 64, 0, st>>>(partial, 2 * k, out);
  return hipGetLastError();
}

hipError_t launch_lv_maxpy2(double2 *x1, const double2 *W1, double2 *x2, const double2 *W2, int k, int64_t n,
                            const double *d, const double *wn, hipStream_t st) {
  if (k < 1) return hipSuccess;
  if (k > LV_MAXK) return hipErrorInvalidValue;
  lv_maxpy2_kernel<<<grid_for(n, DT), DT, 0, st>>>(x1, W1, x2, W2, k, n, d, wn);
  return hipGetLastError();
}

hipError_t launch_lv_dot2(const double2 *w, const double2 *r, int64_t n, double *partial, double *s,
                          hipStream_t st) {
  lv_dot2_kernel<<<LVG, DT, 0, st>>>(w, r, n, partial);
  if (s) lv_finish_kernel<<<3, 64, 0, st>>>(partial, 3, s);
  return hipGetLastError();
}

hipError_t launch_lv_update(double2 *x, const double2 *z, double2 *r, const double2 *w, int64_t n, double *wn,
                            double *partial, double *out, hipStream_t st) {
  lv_update_kernel<<<LVG, DT, 0, st>>>(x, z, r, w, n, partial, wn, partial + 3 * LVG);
  lv_finish_kernel<<<1, 64, 0, st>>>(partial + 3 * LVG, 1, out);
  return hipGetLastError();
}

}  // namespace qxd
