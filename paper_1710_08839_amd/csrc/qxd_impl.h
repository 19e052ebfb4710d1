// Internal types of libqxd: device geometry of the extended lattice, storage
// precisions, complex arithmetic and the spinor/link/Pauli layouts.
//
// Device layout ("native order").  The extended lattice (Sec. 2.1 of the
// openQ*D paper) is cut into blocks of b0 x b1 x b2 x b3 sites (all even).
// A site x has parity p = (x0+x1+x2+x3) & 1, block coordinates B_mu =
// x_mu / b_mu (block index lexicographic, B0 slowest) and local coordinates
// y_mu = x_mu mod b_mu with local lexicographic index l.  Its native index is
//     i = p * V/2 + block * Vb/2 + (l >> 1),
// so even sites come first, and inside one parity every block is contiguous
// (the SAP block solver reads its block as one contiguous range).
//
// Fields are stored block-major: the sites of one parity of one block form a
// run of R = Vb/2 consecutive native indices, and an array with K components
// per site keeps the components of a run together, W at a time: W = 16 bytes
// / (bytes of one stored complex) consecutive components of a site form one
// 16-byte group (W = 1 in FP64, 2 in FP32, 4 with 16-bit storage), and each
// group index of a run is contiguous over the run's sites,
//   element (site j, component k) at
//       (j / R) K R + (k / W) W R + (j % R) W + k % W,
// where j is the site's index in the range of sites the array covers (the
// whole lattice, or one parity half).  A work-group that processes a block
// therefore reads a few contiguous stretches of memory per field, and a lane
// fetches W components with one 16-byte load.
//   spinor    K = 12 (spin*3 + colour)    (+ [sites] fp32 scale for F16S)
//   links     K = 36 (mu*9 + row*3 + col) forward links U(x,mu), all sites
//   angles    K = 4  (mu)                 U(1) potential A(x,mu), all sites
//   pauli     K = 36 pairs, all sites: two 6x6 Hermitian blocks, 18 pairs
//             each: pairs 0-2 hold the 6 real diagonal entries, pairs 3-17
//             the upper triangle (0,1),(0,2)...(0,5),(1,2)...(4,5) as (re, im)
//   pauli_inv K = 36 pairs over the odd sites (j = i - V/2): D_oo^-1
// Block 0 acts on spins 0,1 (gamma5 = +1), block 1 on spins 2,3; inside a
// block the index is s*3 + colour.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qxd.h"

#define QXD_HD __host__ __device__ __forceinline__

namespace qxd {

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------
template <class T>
struct cx {
  T re, im;
};
template <class T> QXD_HD cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <class T> QXD_HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> QXD_HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> QXD_HD cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <class T> QXD_HD cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> QXD_HD cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T> QXD_HD cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <class T> QXD_HD cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class T> QXD_HD cx<T> times_i(cx<T> a) { return {-a.im, a.re}; }
template <class T> QXD_HD cx<T> times_mi(cx<T> a) { return {a.im, -a.re}; }
template <class T> QXD_HD T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <class T> QXD_HD T fmat(T a, T b, T c);
template <> QXD_HD float fmat<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> QXD_HD double fmat<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc + a b, as four fused multiply-adds
template <class T> QXD_HD cx<T> fma_acc(cx<T> acc, cx<T> a, cx<T> b) {
  acc.re = fmat(a.re, b.re, acc.re);
  acc.re = fmat(-a.im, b.im, acc.re);
  acc.im = fmat(a.re, b.im, acc.im);
  acc.im = fmat(a.im, b.re, acc.im);
  return acc;
}
// acc + conj(a) b, as four fused multiply-adds
template <class T> QXD_HD cx<T> fma_accc(cx<T> acc, cx<T> a, cx<T> b) {
  acc.re = fmat(a.re, b.re, acc.re);
  acc.re = fmat(a.im, b.im, acc.re);
  acc.im = fmat(a.re, b.im, acc.im);
  acc.im = fmat(-a.im, b.re, acc.im);
  return acc;
}

// ---------------------------------------------------------------------------
// storage precisions
// ---------------------------------------------------------------------------
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

template <int P> struct St;
template <> struct St<QXD_F64> {
  using pair_t = double2;
  using real_t = double;   // storage of single reals (angles)
  using comp_t = double;   // arithmetic
  static constexpr bool scaled = false;
  QXD_HD static cx<double> ld(const pair_t *p, int64_t i) {
    pair_t v = p[i];
    return {v.x, v.y};
  }
  QXD_HD static void st(pair_t *p, int64_t i, cx<double> z) { p[i] = make_double2(z.re, z.im); }
  QXD_HD static double ldr(const real_t *p, int64_t i) { return p[i]; }
  QXD_HD static void str(real_t *p, int64_t i, double v) { p[i] = v; }
};
template <> struct St<QXD_F32> {
  using pair_t = float2;
  using real_t = float;
  using comp_t = float;
  static constexpr bool scaled = false;
  QXD_HD static cx<float> ld(const pair_t *p, int64_t i) {
    pair_t v = p[i];
    return {v.x, v.y};
  }
  QXD_HD static void st(pair_t *p, int64_t i, cx<float> z) { p[i] = make_float2(z.re, z.im); }
  QXD_HD static float ldr(const real_t *p, int64_t i) { return p[i]; }
  QXD_HD static void str(real_t *p, int64_t i, float v) { p[i] = v; }
};
template <> struct St<QXD_F16S> {
  using pair_t = h2_t;
  using real_t = float;    // angles stay fp32
  using comp_t = float;
  static constexpr bool scaled = true;
  QXD_HD static cx<float> ld(const pair_t *p, int64_t i) {
    pair_t v = p[i];
    return {(float)v.x, (float)v.y};
  }
  QXD_HD static void st(pair_t *p, int64_t i, cx<float> z) {
    pair_t v;
    v.x = (_Float16)z.re;
    v.y = (_Float16)z.im;
    p[i] = v;
  }
  QXD_HD static float ldr(const real_t *p, int64_t i) { return p[i]; }
  QXD_HD static void str(real_t *p, int64_t i, float v) { p[i] = v; }
};
// bfloat16 pairs stored as one uint32: low half = real part, high half = imag
template <> struct St<QXD_BF16> {
  using pair_t = uint32_t;
  using real_t = float;
  using comp_t = float;
  static constexpr bool scaled = false;
  QXD_HD static float bf2f(uint32_t bits16) { return __builtin_bit_cast(float, bits16 << 16); }
  QXD_HD static uint32_t f2bf(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return u >> 16;
  }
  QXD_HD static cx<float> ld(const pair_t *p, int64_t i) {
    uint32_t v = p[i];
    return {bf2f(v & 0xffffu), bf2f(v >> 16)};
  }
  QXD_HD static void st(pair_t *p, int64_t i, cx<float> z) {
#if defined(__HIP_DEVICE_COMPILE__)
    // one packed conversion instruction of gfx950 (round to nearest even)
    typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
    typedef float f32x2_t __attribute__((ext_vector_type(2)));
    p[i] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){z.re, z.im}, bf16x2_t));
#else
    p[i] = f2bf(z.re) | (f2bf(z.im) << 16);
#endif
  }
  QXD_HD static float ldr(const real_t *p, int64_t i) { return p[i]; }
  QXD_HD static void str(real_t *p, int64_t i, float v) { p[i] = v; }
};

// Loads and stores through the global address space.  Pointers that a kernel
// reads from memory (the per-slot tables of the batched kernels) are generic
// to the compiler, which then emits flat instructions (they also count against
// the LDS wait counter); these casts give global ones.  Only for pointers into
// device memory.
template <int N> struct RawOf;
template <> struct RawOf<4> { using type = uint32_t; };
template <> struct RawOf<8> { using type = uint64_t; };
template <> struct RawOf<16> { typedef uint32_t type __attribute__((ext_vector_type(4))); };

template <class T>
__device__ __forceinline__ T gld(const T *p, int64_t i) {
  using R = typename RawOf<sizeof(T)>::type;
  R r = ((const __attribute__((address_space(1))) R *)p)[i];
  return __builtin_bit_cast(T, r);
}
template <class T>
__device__ __forceinline__ void gst(T *p, int64_t i, T v) {
  using R = typename RawOf<sizeof(T)>::type;
  ((__attribute__((address_space(1))) R *)p)[i] = __builtin_bit_cast(R, v);
}
// Non-temporal (streaming) load and store of one stored pair, for data that
// a kernel touches exactly once: they keep such data from displacing lines
// that are read again (neighbour spinors, links) in the caches.
template <int P>
QXD_HD cx<typename St<P>::comp_t> ld_nt(const typename St<P>::pair_t *p) {
  using R = typename RawOf<sizeof(typename St<P>::pair_t)>::type;
  R r = __builtin_nontemporal_load((const R *)p);
  typename St<P>::pair_t v = __builtin_bit_cast(typename St<P>::pair_t, r);
  return St<P>::ld(&v, 0);
}
template <int P>
QXD_HD void st_nt(typename St<P>::pair_t *p, cx<typename St<P>::comp_t> z) {
  using R = typename RawOf<sizeof(typename St<P>::pair_t)>::type;
  typename St<P>::pair_t v;
  St<P>::st(&v, 0, z);
  __builtin_nontemporal_store(__builtin_bit_cast(R, v), (R *)p);
}

// Components per 16-byte group of the block-major layout.
template <int P>
constexpr int VW = 16 / (int)sizeof(typename St<P>::pair_t);

// One 16-byte group (VW<P> stored complex numbers) at p, 16-byte aligned.
template <int P, bool NT = false>
QXD_HD void ld_group(const typename St<P>::pair_t *p, cx<typename St<P>::comp_t> out[VW<P>]) {
  using R = typename RawOf<16>::type;
  R r;
  if constexpr (NT)
    r = __builtin_nontemporal_load((const R *)p);
  else
    r = *(const R *)p;
  typename St<P>::pair_t v[VW<P>];
  __builtin_memcpy(v, &r, 16);
#pragma unroll
  for (int w = 0; w < VW<P>; w++) out[w] = St<P>::ld(v, w);
}
template <int P, bool NT = false>
QXD_HD void st_group(typename St<P>::pair_t *p, const cx<typename St<P>::comp_t> in[VW<P>]) {
  using R = typename RawOf<16>::type;
  typename St<P>::pair_t v[VW<P>];
#pragma unroll
  for (int w = 0; w < VW<P>; w++) St<P>::st(v, w, in[w]);
  R r;
  __builtin_memcpy(&r, v, 16);
  if constexpr (NT)
    __builtin_nontemporal_store(r, (R *)p);
  else
    *(R *)p = r;
}

// pair i of a device array in storage format, as complex
template <int P>
__device__ __forceinline__ cx<typename St<P>::comp_t> gld_pair(const typename St<P>::pair_t *p, int64_t i) {
  typename St<P>::pair_t v = gld(p, i);
  return St<P>::ld(&v, 0);
}
template <int P>
__device__ __forceinline__ void gst_pair(typename St<P>::pair_t *p, int64_t i, cx<typename St<P>::comp_t> z) {
  typename St<P>::pair_t v;
  St<P>::st(&v, 0, z);
  gst(p, i, v);
}

// Element i of a field plane addressed as (plane base) + (32-bit byte
// offset).  With a wavefront-uniform plane base the compiler can use the
// scalar-base + 32-bit-offset form of the global memory instructions: one
// address register per lane instead of a 64-bit address.  Every plane is
// smaller than 4 GiB (the lattice volume is checked when a field is created).
template <class T>
QXD_HD const T *at32(const T *p, uint32_t i) {
  return (const T *)((const char *)p + i * (uint32_t)sizeof(T));
}
template <class T>
QXD_HD T *at32(T *p, uint32_t i) {
  return (T *)((char *)p + i * (uint32_t)sizeof(T));
}

inline size_t pair_bytes(int prec) {
  switch (prec) {
    case QXD_F64: return 16;
    case QXD_F32: return 8;
    default: return 4;
  }
}
inline size_t real_bytes(int prec) { return prec == QXD_F64 ? 8 : 4; }

// Bytes of one native spinor over `sites` sites.
inline size_t spinor_bytes(int prec, int64_t sites) {
  size_t b = 12 * pair_bytes(prec) * (size_t)sites;
  if (prec == QXD_F16S) b += 4 * (size_t)sites;
  return b;
}

// ---------------------------------------------------------------------------
// geometry of the extended lattice (Sec. 2.1)
// ---------------------------------------------------------------------------
// Division by the run length R of the block-major layout by multiplication:
// with l = ceil(log2 R) and m = ceil(2^(32+l) / R), floor(j m / 2^(32+l)) =
// floor(j / R) for every 0 <= j < 2^31 (the error term j (m R - 2^(32+l)) /
// (R 2^(32+l)) is below 2^-(l+1) <= 1/(2R)).
struct RunDiv {
  uint64_t m;
  uint32_t shift;
  uint32_t R;
  QXD_HD uint32_t div(uint32_t j) const { return (uint32_t)(((uint64_t)j * m) >> shift); }
  // element index of component 0 of site j in an array with K components
  // per site packed W at a time; component k is at + comp_off(k, W)
  QXD_HD uint32_t base(uint32_t j, int K, int W = 1) const {
    uint32_t q = div(j);
    return q * (uint32_t)K * R + (j - q * R) * (uint32_t)W;
  }
  QXD_HD uint32_t comp_off(int k, int W) const { return (uint32_t)(k / W) * (uint32_t)W * R + (uint32_t)(k % W); }
};

inline RunDiv make_rundiv(uint32_t R) {
  uint32_t l = 0;
  while (((uint64_t)1 << l) < R) l++;
  RunDiv d;
  d.R = R;
  d.shift = 32 + l;
  d.m = (uint64_t)((((unsigned __int128)1 << d.shift) + R - 1) / R);
  return d;
}

struct Geom {
  int N[4];        // extended extents T, N1, L2, L3
  int b[4];        // block extents
  int nb[4];       // blocks per direction
  int L1;          // physical extent of direction 1
  int L1b;         // L1 / b1: block shift of the C* shifted boundary
  int shift_mask;  // bit k (k = 2, 3): direction k has shifted (C*) boundaries
  int time_bc;     // 0 antiperiodic fermions, 1 open
  int V, Vh;       // sites, half of them
  int Vb, Vbh;     // sites per block, half of them
  int hb3;         // b3 / 2
  int nblocks;
  uint32_t bpk;    // b[0..3] packed 8 bits each (indexed at run time)
  uint32_t nbpk;   // nb[0..3] packed 8 bits each
  RunDiv rd;       // runs of Vbh sites (block-major field layout)
};

// Decoded site: block coordinates B, local coordinates y (8 bits each, packed
// into one word so that a direction chosen at run time needs no array
// indexing), parity p.
struct Site {
  uint32_t Bp;
  uint32_t yp;
  int p;
  QXD_HD int B(int m) const { return (Bp >> (8 * m)) & 0xff; }
  QXD_HD int y(int m) const { return (yp >> (8 * m)) & 0xff; }
  QXD_HD void setB(int m, int v) { Bp = (Bp & ~(0xffu << (8 * m))) | ((uint32_t)v << (8 * m)); }
  QXD_HD void sety(int m, int v) { yp = (yp & ~(0xffu << (8 * m))) | ((uint32_t)v << (8 * m)); }
};

QXD_HD uint32_t pack4(int a0, int a1, int a2, int a3) {
  return (uint32_t)a0 | ((uint32_t)a1 << 8) | ((uint32_t)a2 << 16) | ((uint32_t)a3 << 24);
}

inline void finish_geom(Geom &g) {
  g.bpk = pack4(g.b[0], g.b[1], g.b[2], g.b[3]);
  g.nbpk = pack4(g.nb[0], g.nb[1], g.nb[2], g.nb[3]);
  g.rd = make_rundiv((uint32_t)g.Vbh);
}

QXD_HD Site decode(const Geom &g, int i) {
  Site s;
  s.p = i >= g.Vh;
  int r = i - s.p * g.Vh;
  int blk = r / g.Vbh;
  int h = r - blk * g.Vbh;
  int B3 = blk % g.nb[3];
  blk /= g.nb[3];
  int B2 = blk % g.nb[2];
  blk /= g.nb[2];
  int B1 = blk % g.nb[1];
  int B0 = blk / g.nb[1];
  int q = h / g.hb3;
  int y3h = h - q * g.hb3;
  int y2 = q % g.b[2];
  q /= g.b[2];
  int y1 = q % g.b[1];
  int y0 = q / g.b[1];
  int e = (s.p + y0 + y1 + y2) & 1;
  s.Bp = pack4(B0, B1, B2, B3);
  s.yp = pack4(y0, y1, y2, 2 * y3h + e);
  return s;
}

QXD_HD int block_index(const Geom &g, const Site &s) {
  return ((s.B(0) * g.nb[1] + s.B(1)) * g.nb[2] + s.B(2)) * g.nb[3] + s.B(3);
}

QXD_HD int encode(const Geom &g, const Site &s) {
  int l = ((s.y(0) * g.b[1] + s.y(1)) * g.b[2] + s.y(2)) * g.b[3] + s.y(3);
  return s.p * g.Vh + block_index(g, s) * g.Vbh + (l >> 1);
}

// Element index of component 0 of site s in a block-major array with K
// components over all sites (runs: even blocks, then odd blocks).
QXD_HD uint32_t site_base(const Geom &g, const Site &s, int K) {
  int l = ((s.y(0) * g.b[1] + s.y(1)) * g.b[2] + s.y(2)) * g.b[3] + s.y(3);
  uint32_t run = (uint32_t)(s.p * g.nblocks + block_index(g, s));
  return run * (uint32_t)K * (uint32_t)g.Vbh + (uint32_t)(l >> 1);
}

QXD_HD void global_coords(const Geom &g, const Site &s, int x[4]) {
#pragma unroll
  for (int m = 0; m < 4; m++) x[m] = s.B(m) * g.b[m] + s.y(m);
}

// Neighbour x + mu (dir = +1) or x - mu (dir = -1).  `sign` receives the
// fermion factor of the hop: -1 across the antiperiodic time boundary, 0 across
// an open one, else 1.  Shifted C* boundaries move x1 by L1 (mod 2 L1).
QXD_HD Site neighbour(const Geom &g, const Site &s, int mu, int dir, int &sign) {
  Site t = s;
  t.p = s.p ^ 1;
  sign = 1;
  int y = s.y(mu) + dir;
  int bmu = (g.bpk >> (8 * mu)) & 0xff;
  if (y >= 0 && y < bmu) {
    t.sety(mu, y);
    return t;
  }
  t.sety(mu, dir > 0 ? 0 : bmu - 1);
  int nbm = (g.nbpk >> (8 * mu)) & 0xff;
  int B = s.B(mu) + dir;
  bool wrap = false;
  if (B == nbm) {
    B = 0;
    wrap = true;
  } else if (B < 0) {
    B = nbm - 1;
    wrap = true;
  }
  t.setB(mu, B);
  if (wrap) {
    if (mu == 0) {
      sign = g.time_bc == 0 ? -1 : 0;
    } else if ((g.shift_mask >> mu) & 1) {
      int b1 = t.B(1) + g.L1b;
      if (b1 >= g.nb[1]) b1 -= g.nb[1];
      t.setB(1, b1);
    }
  }
  return t;
}

// Physical-lattice lexicographic index of the site (mirror sites map to their
// physical partner); `mirror` tells which half the site lies in.
QXD_HD int64_t phys_lex(const Geom &g, const int x[4], bool &mirror) {
  int x1 = x[1];
  mirror = x1 >= g.L1;
  if (mirror) x1 -= g.L1;
  return (((int64_t)x[0] * g.L1 + x1) * g.N[2] + x[2]) * g.N[3] + x[3];
}

QXD_HD int64_t ext_lex(const Geom &g, const int x[4]) {
  return (((int64_t)x[0] * g.N[1] + x[1]) * g.N[2] + x[2]) * g.N[3] + x[3];
}

// ---------------------------------------------------------------------------
// spinor views
// ---------------------------------------------------------------------------
// A spinor view over the sites [off, off + sites) of the native order:
// component c (= spin * 3 + colour) of native site i is the block-major
// element of (j = i - off, c) with K = 12; F16S keeps one fp32 scale per site
// after the 12 * sites pairs.
template <int P>
struct Spinor {
  typename St<P>::pair_t *data;
  float *scale;   // F16S only: one fp32 scale per site, index j
  int64_t off;
  RunDiv rd;
};

template <int P>
QXD_HD Spinor<P> spinor_view(void *base, int64_t sites, int64_t off, const RunDiv &rd) {
  Spinor<P> s;
  s.data = (typename St<P>::pair_t *)base;
  s.scale = St<P>::scaled ? (float *)((char *)base + 12 * sizeof(typename St<P>::pair_t) * sites) : nullptr;
  s.off = off;
  s.rd = rd;
  return s;
}
template <int P>
QXD_HD Spinor<P> spinor_view(void *base, int64_t sites, int64_t off, const Geom &g) {
  return spinor_view<P>(base, sites, off, g.rd);
}

// Components are addressed as (wavefront-uniform base of the component) +
// (32-bit element offset of the site), so that the 12 loads of a spinor share
// one address register.
template <int P, class T>
QXD_HD void load_spinor(const Spinor<P> &s, int64_t i, cx<T> psi[4][3]) {
  constexpr int W = VW<P>;
  uint32_t j = (uint32_t)(i - s.off);
  uint32_t e = s.rd.base(j, 12, W);
#pragma unroll
  for (int gk = 0; gk < 12 / W; gk++) {
    cx<typename St<P>::comp_t> z[W];
    ld_group<P>(at32(s.data + gk * W * s.rd.R, e), z);
#pragma unroll
    for (int w = 0; w < W; w++) psi[(gk * W + w) / 3][(gk * W + w) % 3] = {(T)z[w].re, (T)z[w].im};
  }
  if constexpr (St<P>::scaled) {
    T f = (T)*at32(s.scale, j);
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int c = 0; c < 3; c++) psi[a][c] = f * psi[a][c];
  }
}

template <int P, class T, bool NT = false>
QXD_HD void store_spinor(const Spinor<P> &s, int64_t i, const cx<T> psi[4][3]) {
  constexpr int W = VW<P>;
  int64_t j = i - s.off;
  uint32_t e = s.rd.base((uint32_t)j, 12, W);
  using C = typename St<P>::comp_t;
  C f = (C)1;
  if constexpr (St<P>::scaled) {
    // largest magnitude (fmax ignores a NaN operand, as the comparison did;
    // one max with an abs modifier per component)
    T m = 0;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int c = 0; c < 3; c++) m = fmax(fmax(m, fabs(psi[a][c].re)), fabs(psi[a][c].im));
    *at32(s.scale, (uint32_t)j) = (float)m;
    f = m > 0 ? (C)(1.0f / (float)m) : (C)0;
  }
#pragma unroll
  for (int gk = 0; gk < 12 / W; gk++) {
    cx<C> z[W];
#pragma unroll
    for (int w = 0; w < W; w++) {
      const cx<T> &x = psi[(gk * W + w) / 3][(gk * W + w) % 3];
      z[w] = {(C)(f * (C)x.re), (C)(f * (C)x.im)};
    }
    st_group<P, NT>(at32(s.data + gk * W * s.rd.R, e), z);
  }
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
inline unsigned grid_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// The GPU hands work-group w to XCD (w mod 8); each XCD has its own L2.  Map
// work-groups to a logical order in which XCD x owns one contiguous range of
// the logical index space, so that neighbouring lattice blocks are processed
// by the same XCD at about the same time.  A bijection on [0, n).
constexpr int N_XCD = 8;
QXD_HD int xcd_order(int w, int n) {
  int x = w % N_XCD, k = w / N_XCD;
  int q = n / N_XCD, r = n % N_XCD;
  return x * q + (x < r ? x : r) + k;
}

}  // namespace qxd
