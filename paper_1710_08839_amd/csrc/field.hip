// Gauge-field ingest with the C* orbifold, clover/Pauli construction, the
// inverse of the odd-site Pauli blocks, and layout/precision conversions.
#include "dirac_site.h"
#include "launch.h"

namespace qxd {

namespace {

struct M3 {
  cx<double> m[3][3];
};

__device__ __forceinline__ M3 ld_u(const double2 *links, const Geom &g, int mu, int64_t i) {
  M3 r;
  load_link<QXD_F64, double>(links, g, mu, i, r.m);
  return r;
}
__device__ __forceinline__ M3 mul(const M3 &a, const M3 &b) {
  M3 r;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      cx<double> s{0, 0};
      for (int k = 0; k < 3; k++) s = fma_acc(s, a.m[i][k], b.m[k][j]);
      r.m[i][j] = s;
    }
  return r;
}
__device__ __forceinline__ M3 dag(const M3 &a) {
  M3 r;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) r.m[i][j] = conj(a.m[j][i]);
  return r;
}

// ---- orbifold build (Sec. 2.1, eq. orbi:gauge) ------------------------------
__global__ void orbifold_kernel(Geom g, const double *u_phs, const double *a_phs, double2 *links,
                                double *angles) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  Site s = decode(g, i);
  int x[4];
  global_coords(g, s, x);
  bool mirror;
  int64_t j = phys_lex(g, x, mirror);
  const uint32_t el = g.rd.base((uint32_t)i, 36), ea = g.rd.base((uint32_t)i, 4);
  for (int mu = 0; mu < 4; mu++) {
    // an open time end (open, open-SF) cuts the links across x0 = T-1 -> 0
    bool cut = (g.time_bc == 1 || g.time_bc == 3) && mu == 0 && x[0] == g.N[0] - 1;
    const double *u = u_phs + (j * 4 + mu) * 18;
    for (int k = 0; k < 9; k++) {
      double re = u[2 * k], im = u[2 * k + 1];
      if (mirror) im = -im;
      if (cut) re = im = 0.0;
      links[el + (mu * 9 + k) * g.Vbh] = make_double2(re, im);
    }
    double a = a_phs ? a_phs[j * 4 + mu] : 0.0;
    angles[ea + mu * g.Vbh] = mirror ? -a : a;
  }
}

// ---- clover and Pauli term (Sec. 2.3) ---------------------------------------
__device__ __forceinline__ cx<double> zlink(const Geom &g, const double *angles, int mu,
                                            int64_t i, const Site &s) {
  int x0 = s.B(0) * g.b[0] + s.y(0);
  if ((g.time_bc == 1 || g.time_bc == 3) && mu == 0 && x0 == g.N[0] - 1) return {0.0, 0.0};
  double sn, cs;
  sincos(angles[g.rd.base((uint32_t)i, 4) + mu * g.Vbh], &sn, &cs);
  return {cs, sn};
}

__global__ void __launch_bounds__(128) pauli_build_kernel(Geom g, const double2 *links, const double *angles, int has_u1,
                                   double kappa, double csw, double u1coef, double cF, double cFp,
                                   double2 *pauli) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  Site s = decode(g, i);
  const int x0 = s.B(0) * g.b[0] + s.y(0), t1 = g.N[0] - 1;
  if ((g.time_bc == 2 || g.time_bc == 3) && x0 == 0) {
    // the fixed slice of SF / open-SF: identity
    const uint32_t e = g.rd.base((uint32_t)i, 36);
    for (int blk = 0; blk < 2; blk++) {
      for (int k = 0; k < 3; k++) pauli[e + (18 * blk + k) * g.Vbh] = make_double2(1.0, 1.0);
      for (int k = 3; k < 18; k++) pauli[e + (18 * blk + k) * g.Vbh] = make_double2(0.0, 0.0);
    }
    return;
  }
  // dD_b = (c_F - 1) on x0 = 0, T-1 (open); x0 = 1, T-1 (SF); (c_F - 1) on
  // x0 = 1 and (c_F' - 1) on x0 = T-1 (open-SF)
  double dbt = 0.0;
  if (g.time_bc == 1 && (x0 == 0 || x0 == t1)) dbt = cF - 1.0;
  if (g.time_bc == 2 && (x0 == 1 || x0 == t1)) dbt = cF - 1.0;
  if (g.time_bc == 3) dbt = x0 == t1 ? cFp - 1.0 : (x0 == 1 ? cF - 1.0 : 0.0);
  // The chiral blocks are A = d + [[h3, h1 - i h2], [h1 + i h2, -h3]] with
  // h_l = (i/2) M_l and M_l = +-G_0l - B_l, B = (G_23, -G_13, G_12), where
  // G_p = csw F_p + u1coef * Ahat'_p.  The planes (01,02,03,12,13,23) are
  // taken one at a time (a rolled loop: one plane's links live at once) and
  // each adds its share to the upper triangles of both blocks, held in
  // registers under compile-time indices (no private memory).
  cx<double> ul[2][3][3], lr[2][3][3], ur[2][3][3];  // upper-left, lower-right (a <= b), upper-right
#pragma unroll
  for (int blk = 0; blk < 2; blk++)
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) ul[blk][a][b] = lr[blk][a][b] = ur[blk][a][b] = cx<double>{0.0, 0.0};
#pragma unroll 1
  for (int p = 0; p < 6; p++) {
    const int mu = p < 3 ? 0 : (p < 5 ? 1 : 2);
    const int nu = p < 3 ? p + 1 : (p < 5 ? p - 1 : 3);
    M3 gp;
    {
      int sg;
      Site xpm = neighbour(g, s, mu, 1, sg), xpn = neighbour(g, s, nu, 1, sg);
      Site xmm = neighbour(g, s, mu, -1, sg), xmn = neighbour(g, s, nu, -1, sg);
      Site xmm_pn = neighbour(g, xmm, nu, 1, sg), xmm_mn = neighbour(g, xmm, nu, -1, sg);
      Site xpm_mn = neighbour(g, xmn, mu, 1, sg);
      int64_t ixpm = encode(g, xpm), ixpn = encode(g, xpn), ixmm = encode(g, xmm),
              ixmn = encode(g, xmn), ixmm_pn = encode(g, xmm_pn), ixmm_mn = encode(g, xmm_mn),
              ixpm_mn = encode(g, xpm_mn);
      // clover leaves q1..q4 (anticlockwise from x in the (mu, nu) plane),
      // each the product of four links; the sixteen factors are taken in a
      // rolled loop so that one link, the running product and the leaf sum
      // are all that live at once
      M3 qsum, prod;
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) qsum.m[a][b] = prod.m[a][b] = cx<double>{0.0, 0.0};
#pragma unroll 1
      for (int t = 0; t < 16; t++) {
        const int leaf = t >> 2, fct = t & 3;
        int64_t y;
        int dir;
        bool dg;
        if (leaf == 0) {         // U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
          y = fct == 0 ? (int64_t)i : fct == 1 ? ixpm : fct == 2 ? ixpn : (int64_t)i;
          dir = (fct & 1) ? nu : mu;
          dg = fct >= 2;
        } else if (leaf == 1) {  // U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
          y = fct == 0 ? (int64_t)i : fct == 1 ? ixmm_pn : ixmm;
          dir = (fct & 1) ? mu : nu;
          dg = fct == 1 || fct == 2;
        } else if (leaf == 2) {  // U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
          y = fct == 0 ? ixmm : fct == 3 ? ixmn : ixmm_mn;
          dir = (fct & 1) ? nu : mu;
          dg = fct <= 1;
        } else {                 // U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
          y = fct <= 1 ? ixmn : fct == 2 ? ixpm_mn : (int64_t)i;
          dir = (fct & 1) ? mu : nu;
          dg = fct == 0 || fct == 3;
        }
        M3 u = ld_u(links, g, dir, y);
        if (dg) u = dag(u);
        prod = fct == 0 ? u : mul(prod, u);
        if (fct == 3) {
#pragma unroll
          for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) qsum.m[a][b] = qsum.m[a][b] + prod.m[a][b];
        }
      }
      double ah = 0.0;  // Ahat' = i * ah
      if (has_u1) {
        auto zp = [&](int64_t y, const Site &sy, int64_t ypm, const Site &sypm, int64_t ypn,
                      const Site &sypn) {
          return zlink(g, angles, mu, y, sy) * zlink(g, angles, nu, ypm, sypm) *
                 conj(zlink(g, angles, mu, ypn, sypn)) * conj(zlink(g, angles, nu, y, sy));
        };
        cx<double> zs = zp(i, s, ixpm, xpm, ixpn, xpn) + zp(ixmm, xmm, i, s, ixmm_pn, xmm_pn) +
                        zp(ixmn, xmn, ixpm_mn, xpm_mn, i, s) +
                        zp(ixmm_mn, xmm_mn, ixmn, xmn, ixmm, xmm);
        ah = 0.25 * zs.im;
      }
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
          cx<double> f = 0.125 * (qsum.m[a][b] - conj(qsum.m[b][a]));
          gp.m[a][b] = csw * f;
        }
#pragma unroll
      for (int a = 0; a < 3; a++) gp.m[a][a].im += u1coef * ah;
    }
    // plane p enters M_l (l = 1, 2, 3 for 01/23, 02/13, 03/12) with weight
    // +-1 (the sign of the block) for the planes 0l, and -1, +1, -1 for
    // 12, 13, 23
    const int l = (p == 0 || p == 5) ? 1 : ((p == 1 || p == 4) ? 2 : 3);
#pragma unroll
    for (int blk = 0; blk < 2; blk++) {
      const double c = p < 3 ? (blk == 0 ? 0.5 : -0.5) : (p == 4 ? 0.5 : -0.5);
      const double w3 = l == 3 ? c : 0.0, w1 = l == 1 ? c : 0.0, w2 = l == 2 ? c : 0.0;
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
          const cx<double> ig = times_i(gp.m[a][b]);
          if (a <= b) {
            ul[blk][a][b] = ul[blk][a][b] + w3 * ig;
            lr[blk][a][b] = lr[blk][a][b] - w3 * ig;
          }
          ur[blk][a][b] = ur[blk][a][b] + w1 * ig + w2 * gp.m[a][b];
        }
    }
  }
  const double d = 0.5 / kappa + dbt;
  const uint32_t e = g.rd.base((uint32_t)i, 36);
#pragma unroll
  for (int blk = 0; blk < 2; blk++) {
    // A[r][c] for r <= c: rows/columns 0..2 upper, 3..5 lower chirality-block spin
    auto entry = [&](int r, int c) -> cx<double> {
      if (c < 3) return ul[blk][r][c];
      if (r >= 3) return lr[blk][r - 3][c - 3];
      return ur[blk][r][c - 3];
    };
    const int base = 18 * blk;
#pragma unroll
    for (int k = 0; k < 3; k++)
      pauli[e + (base + k) * g.Vbh] = make_double2(d + entry(2 * k, 2 * k).re, d + entry(2 * k + 1, 2 * k + 1).re);
#pragma unroll
    for (int r = 0; r < 6; r++)
#pragma unroll
      for (int c = r + 1; c < 6; c++) {
        const cx<double> v = entry(r, c);
        pauli[e + (base + 3 + tri_index(r, c)) * g.Vbh] = make_double2(v.re, v.im);
      }
  }
}

// In-place Gauss-Jordan inverse of a Hermitian positive-definite 6x6 block
// (no pivoting is needed for positive-definite matrices; a non-positive or
// tiny pivot is reported as singular).
__global__ void __launch_bounds__(128) pauli_invert_kernel(Geom g, const double2 *pauli, double2 *pinv, int *bad) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * g.Vh) return;
  int blk = t / g.Vh;
  int j = t - blk * g.Vh;      // odd-site half index
  int64_t i = (int64_t)g.Vh + j;
  int base = 18 * blk;
  const uint32_t ep = g.rd.base((uint32_t)i, 36), eq = g.rd.base((uint32_t)j, 36);
  cx<double> a[6][6];
  for (int k = 0; k < 3; k++) {
    double2 v = pauli[ep + (base + k) * g.Vbh];
    a[2 * k][2 * k] = {v.x, 0.0};
    a[2 * k + 1][2 * k + 1] = {v.y, 0.0};
  }
  for (int r = 0; r < 6; r++)
    for (int c = r + 1; c < 6; c++) {
      double2 v = pauli[ep + (base + 3 + tri_index(r, c)) * g.Vbh];
      a[r][c] = {v.x, v.y};
      a[c][r] = {v.x, -v.y};
    }
  double scale = 0.0;
  for (int r = 0; r < 6; r++) scale = fmax(scale, a[r][r].re);
  bool ok = scale > 0.0;
  for (int k = 0; k < 6; k++) {
    cx<double> p = a[k][k];
    double n2 = norm2(p);
    if (!(n2 > 1e-28 * scale * scale)) ok = false;
    cx<double> pi{p.re / n2, -p.im / n2};
    a[k][k] = {1.0, 0.0};
    for (int c = 0; c < 6; c++) a[k][c] = a[k][c] * pi;
    for (int r = 0; r < 6; r++) {
      if (r == k) continue;
      cx<double> f = a[r][k];
      a[r][k] = {0.0, 0.0};
      for (int c = 0; c < 6; c++) a[r][c] = a[r][c] - f * a[k][c];
    }
  }
  if (!ok) atomicAdd(bad, 1);
  for (int k = 0; k < 3; k++)
    pinv[eq + (base + k) * g.Vbh] = make_double2(a[2 * k][2 * k].re, a[2 * k + 1][2 * k + 1].re);
  for (int r = 0; r < 6; r++)
    for (int c = r + 1; c < 6; c++) {
      // symmetrise the rounding of the two triangles
      cx<double> v = 0.5 * (a[r][c] + conj(a[c][r]));
      pinv[eq + (base + 3 + tri_index(r, c)) * g.Vbh] = make_double2(v.re, v.im);
    }
}

// FP64 block-major field (K pairs per site, packing 1) -> storage precision P
// (packing VW<P>); one thread per (site, 16-byte group).
template <int P>
__global__ void convert_field_kernel(RunDiv rd, int K, int64_t sites, const double2 *src,
                                     typename St<P>::pair_t *dst) {
  constexpr int W = VW<P>;
  const int ng = K / W;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= sites * ng) return;
  const uint32_t j = (uint32_t)(t / ng);
  const int gk = (int)(t - (int64_t)j * ng);
  const uint32_t e1 = rd.base(j, K, 1), ew = rd.base(j, K, W);
  using C = typename St<P>::comp_t;
  cx<C> z[W];
#pragma unroll
  for (int w = 0; w < W; w++) {
    double2 v = src[e1 + rd.comp_off(gk * W + w, 1)];
    z[w] = {(C)v.x, (C)v.y};
  }
  st_group<P>(dst + ew + (uint32_t)gk * W * rd.R, z);
}

__global__ void convert_reals_kernel(const double *src, float *dst, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = (float)src[k];
}

// ---- spinor layout conversion ---------------------------------------------
template <int P>
__global__ void pack_kernel(Geom g, const double *api, void *native, size_t bytes) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (i >= g.V) return;
  Site s = decode(g, i);
  int x[4];
  global_coords(g, s, x);
  int64_t l = ext_lex(g, x);
  const double *src = api + ((int64_t)r * g.V + l) * 24;
  cx<double> psi[4][3];
  for (int a = 0; a < 4; a++)
    for (int c = 0; c < 3; c++) psi[a][c] = {src[(a * 3 + c) * 2], src[(a * 3 + c) * 2 + 1]};
  Spinor<P> out = spinor_view<P>((char *)native + r * bytes, g.V, 0, g);
  store_spinor<P, double>(out, i, psi);
}

template <int P>
__global__ void unpack_kernel(Geom g, const void *native, double *api, size_t bytes) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (i >= g.V) return;
  Site s = decode(g, i);
  int x[4];
  global_coords(g, s, x);
  int64_t l = ext_lex(g, x);
  Spinor<P> in = spinor_view<P>((char *)const_cast<void *>(native) + r * bytes, g.V, 0, g);
  cx<double> psi[4][3];
  load_spinor<P, double>(in, i, psi);
  double *dst = api + ((int64_t)r * g.V + l) * 24;
  for (int a = 0; a < 4; a++)
    for (int c = 0; c < 3; c++) {
      dst[(a * 3 + c) * 2] = psi[a][c].re;
      dst[(a * 3 + c) * 2 + 1] = psi[a][c].im;
    }
}

struct Theta {
  double t[4];
};

// W(x,mu) = U(x,mu) exp(i qhat A(x,mu)) in FP64, times exp(+-i theta_mu) on
// the links whose forward hop crosses the boundary of direction mu (the sign
// is - on the C* mirror half, x1 >= L1 of an extended direction 1); one
// thread per (site, mu)
__global__ void fold_phase_kernel(Geom g, const double2 *links, const double *angles, int qhat, Theta th,
                                  double2 *w) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * (int64_t)g.V) return;
  int mu = (int)(t / g.V);
  uint32_t i = (uint32_t)(t - (int64_t)mu * g.V);
  const uint32_t el = g.rd.base(i, 36);
  double phase = qhat * angles[g.rd.base(i, 4) + mu * g.Vbh];
  const Site s = decode(g, (int)i);
  int x[4];
  global_coords(g, s, x);
  if (th.t[mu] != 0.0 && x[mu] == g.N[mu] - 1) phase += (g.N[1] != g.L1 && x[1] >= g.L1) ? -th.t[mu] : th.t[mu];
  double sn, cs;
  sincos(phase, &sn, &cs);
  cx<double> z{cs, sn};
  // SF / open-SF: no hop enters or leaves the fixed slice x0 = 0
  if ((g.time_bc == 2 || g.time_bc == 3) && x[0] == 0) z = {0.0, 0.0};
  for (int k = 0; k < 9; k++) {
    double2 u = links[el + (mu * 9 + k) * g.Vbh];
    cx<double> r = cx<double>{u.x, u.y} * z;
    w[el + (mu * 9 + k) * g.Vbh] = make_double2(r.re, r.im);
  }
}

template <int P>
__global__ void zero_sites_kernel(Spinor<P> v, int64_t first, int64_t count) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  int64_t i = first + k;
  cx<typename St<P>::comp_t> z[4][3];
  for (int a = 0; a < 4; a++)
    for (int c = 0; c < 3; c++) z[a][c] = {0, 0};
  store_spinor<P, typename St<P>::comp_t>(v, i, z);
}

// gamma5 of the chiral basis, diag(1, 1, -1, -1) in spin, in place: flips the
// sign of the stored components 6..11 (spins 2 and 3); exact in every storage
// format, and the FP16 site scale (a magnitude) is unchanged.  Thread t
// handles component 6 + t / count of site first + t % count.
template <int P>
__global__ void g5_sites_kernel(Spinor<P> v, int64_t first, int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 6 * count) return;
  const int k = 6 + (int)(t / count);
  const int64_t i = first + t % count;
  const uint32_t j = (uint32_t)(i - v.off);
  typename St<P>::pair_t *p = v.data + v.rd.base(j, 12, VW<P>) + v.rd.comp_off(k, VW<P>);
  const auto z = St<P>::ld(p, 0);
  St<P>::st(p, 0, {-z.re, -z.im});
}

}  // namespace

hipError_t launch_g5_sites(int prec, SpinorArg v, int64_t first, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  unsigned gr = grid_for(6 * count, 256);
  switch (prec) {
    case QXD_F64: g5_sites_kernel<QXD_F64><<<gr, 256, 0, st>>>(spinor_view<QXD_F64>(v.ptr, v.sites, v.off, v.rd), first, count); break;
    case QXD_F32: g5_sites_kernel<QXD_F32><<<gr, 256, 0, st>>>(spinor_view<QXD_F32>(v.ptr, v.sites, v.off, v.rd), first, count); break;
    case QXD_F16S: g5_sites_kernel<QXD_F16S><<<gr, 256, 0, st>>>(spinor_view<QXD_F16S>(v.ptr, v.sites, v.off, v.rd), first, count); break;
    case QXD_BF16: g5_sites_kernel<QXD_BF16><<<gr, 256, 0, st>>>(spinor_view<QXD_BF16>(v.ptr, v.sites, v.off, v.rd), first, count); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero_sites(int prec, SpinorArg v, int64_t first, int64_t count, hipStream_t st) {
  unsigned gr = grid_for(count, 256);
  switch (prec) {
    case QXD_F64: zero_sites_kernel<QXD_F64><<<gr, 256, 0, st>>>(spinor_view<QXD_F64>(v.ptr, v.sites, v.off, v.rd), first, count); break;
    case QXD_F32: zero_sites_kernel<QXD_F32><<<gr, 256, 0, st>>>(spinor_view<QXD_F32>(v.ptr, v.sites, v.off, v.rd), first, count); break;
    case QXD_F16S: zero_sites_kernel<QXD_F16S><<<gr, 256, 0, st>>>(spinor_view<QXD_F16S>(v.ptr, v.sites, v.off, v.rd), first, count); break;
    case QXD_BF16: zero_sites_kernel<QXD_BF16><<<gr, 256, 0, st>>>(spinor_view<QXD_BF16>(v.ptr, v.sites, v.off, v.rd), first, count); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fold_phase(const Geom &g, const double2 *links, const double *angles, int qhat,
                             const double theta[4], double2 *w, hipStream_t st) {
  Theta th;
  for (int m = 0; m < 4; m++) th.t[m] = theta ? theta[m] : 0.0;
  fold_phase_kernel<<<grid_for(4 * (int64_t)g.V, 256), 256, 0, st>>>(g, links, angles, qhat, th, w);
  return hipGetLastError();
}

namespace {
// out = ca G_a a + cb G_b b per site (G = gamma5 or 1), one thread per site
template <int P>
__global__ void lincomb_sites_kernel(Spinor<P> out, Spinor<P> a, cx<typename St<P>::comp_t> ca, int g5a,
                                     Spinor<P> b, cx<typename St<P>::comp_t> cb, int g5b, int64_t first,
                                     int64_t count) {
  using T = typename St<P>::comp_t;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int64_t i = first + k;
  cx<T> va[4][3], res[4][3];
  load_spinor<P, T>(a, i, va);
  for (int s = 0; s < 4; s++)
    for (int c = 0; c < 3; c++) res[s][c] = ca * ((g5a && s >= 2) ? -va[s][c] : va[s][c]);
  if (b.data) {
    cx<T> vb[4][3];
    load_spinor<P, T>(b, i, vb);
    for (int s = 0; s < 4; s++)
      for (int c = 0; c < 3; c++) res[s][c] = res[s][c] + cb * ((g5b && s >= 2) ? -vb[s][c] : vb[s][c]);
  }
  store_spinor<P, T>(out, i, res);
}

template <int P>
hipError_t lincomb_p(SpinorArg out, SpinorArg a, double car, double cai, bool g5a, SpinorArg b, double cbr,
                     double cbi, bool g5b, int64_t first, int64_t count, hipStream_t st) {
  using T = typename St<P>::comp_t;
  Spinor<P> vo = spinor_view<P>(out.ptr, out.sites, out.off, out.rd);
  Spinor<P> va = spinor_view<P>(a.ptr, a.sites, a.off, a.rd);
  Spinor<P> vb = b.ptr ? spinor_view<P>(b.ptr, b.sites, b.off, b.rd) : Spinor<P>{nullptr, nullptr, 0, out.rd};
  lincomb_sites_kernel<P><<<grid_for(count, 256), 256, 0, st>>>(vo, va, cx<T>{(T)car, (T)cai}, g5a, vb,
                                                                cx<T>{(T)cbr, (T)cbi}, g5b, first, count);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_lincomb_sites(int prec, SpinorArg out, SpinorArg a, double ca_re, double ca_im, bool g5a,
                                SpinorArg b, double cb_re, double cb_im, bool g5b, int64_t first, int64_t count,
                                hipStream_t st) {
  if (count <= 0) return hipSuccess;
  switch (prec) {
    case QXD_F64: return lincomb_p<QXD_F64>(out, a, ca_re, ca_im, g5a, b, cb_re, cb_im, g5b, first, count, st);
    case QXD_F32: return lincomb_p<QXD_F32>(out, a, ca_re, ca_im, g5a, b, cb_re, cb_im, g5b, first, count, st);
    case QXD_F16S: return lincomb_p<QXD_F16S>(out, a, ca_re, ca_im, g5a, b, cb_re, cb_im, g5b, first, count, st);
    case QXD_BF16: return lincomb_p<QXD_BF16>(out, a, ca_re, ca_im, g5a, b, cb_re, cb_im, g5b, first, count, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_orbifold(const Geom &g, const double *u_phs, const double *a_phs, double2 *links,
                           double *angles, hipStream_t st) {
  orbifold_kernel<<<grid_for(g.V, 256), 256, 0, st>>>(g, u_phs, a_phs, links, angles);
  return hipGetLastError();
}

hipError_t launch_pauli_build(const Geom &g, const double2 *links, const double *angles, int has_u1,
                              double kappa, double csw, double u1coef, double cF, double cFp,
                              double2 *pauli, hipStream_t st) {
  pauli_build_kernel<<<grid_for(g.V, 128), 128, 0, st>>>(g, links, angles, has_u1, kappa, csw,
                                                         u1coef, cF, cFp, pauli);
  return hipGetLastError();
}

hipError_t launch_pauli_invert(const Geom &g, const double2 *pauli, double2 *pinv, int *bad,
                               hipStream_t st) {
  pauli_invert_kernel<<<grid_for(2 * (int64_t)g.Vh, 128), 128, 0, st>>>(g, pauli, pinv, bad);
  return hipGetLastError();
}

hipError_t launch_convert_field(int prec, const Geom &g, int K, int64_t sites, const double2 *src, void *dst,
                                hipStream_t st) {
  const RunDiv rd = g.rd;
  switch (prec) {
    case QXD_F64: return hipMemcpyAsync(dst, src, (size_t)K * sites * 16, hipMemcpyDeviceToDevice, st);
    case QXD_F32:
      convert_field_kernel<QXD_F32><<<grid_for(sites * K / 2, 256), 256, 0, st>>>(rd, K, sites, src, (float2 *)dst);
      break;
    case QXD_F16S:
      convert_field_kernel<QXD_F16S><<<grid_for(sites * K / 4, 256), 256, 0, st>>>(rd, K, sites, src, (h2_t *)dst);
      break;
    case QXD_BF16:
      convert_field_kernel<QXD_BF16><<<grid_for(sites * K / 4, 256), 256, 0, st>>>(rd, K, sites, src, (uint32_t *)dst);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_convert_reals(const double *src, float *dst, int64_t n, hipStream_t st) {
  convert_reals_kernel<<<grid_for(n, 256), 256, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_pack(int prec, const Geom &g, const double *api, void *native, int nrhs,
                       hipStream_t st) {
  dim3 gr(grid_for(g.V, 256), nrhs);
  size_t bytes = spinor_bytes(prec, g.V);
  switch (prec) {
    case QXD_F64: pack_kernel<QXD_F64><<<gr, 256, 0, st>>>(g, api, native, bytes); break;
    case QXD_F32: pack_kernel<QXD_F32><<<gr, 256, 0, st>>>(g, api, native, bytes); break;
    case QXD_F16S: pack_kernel<QXD_F16S><<<gr, 256, 0, st>>>(g, api, native, bytes); break;
    case QXD_BF16: pack_kernel<QXD_BF16><<<gr, 256, 0, st>>>(g, api, native, bytes); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_unpack(int prec, const Geom &g, const void *native, double *api, int nrhs,
                         hipStream_t st) {
  dim3 gr(grid_for(g.V, 256), nrhs);
  size_t bytes = spinor_bytes(prec, g.V);
  switch (prec) {
    case QXD_F64: unpack_kernel<QXD_F64><<<gr, 256, 0, st>>>(g, native, api, bytes); break;
    case QXD_F32: unpack_kernel<QXD_F32><<<gr, 256, 0, st>>>(g, native, api, bytes); break;
    case QXD_F16S: unpack_kernel<QXD_F16S><<<gr, 256, 0, st>>>(g, native, api, bytes); break;
    case QXD_BF16: unpack_kernel<QXD_BF16><<<gr, 256, 0, st>>>(g, native, api, bytes); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qxd
