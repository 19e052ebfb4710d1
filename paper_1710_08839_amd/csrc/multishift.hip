// Multi-shift conjugate gradient on the even-odd normal operator and rational
// functions of it (qxd_multishift_solve, qxd_rational_apply).
//
// Sec. 2.4 of the openQ*D paper writes the pseudofermion action with a
// rational function R = A prod_j (D^dag D^ + nu_j^2) / (D^dag D^ + mu_j^2)
// and its frequency-splitting factors; every pole is a shifted system
// (X + sigma) x = b with X = D^dag D^ + mu^2 (mu a twisted mass), which the
// multi-shift CG the paper names (Sec. 2 feature list, Table 2) solves for
// all shifts in one Krylov space:
//   CG on X + sigma_0 (sigma_0 the smallest shift) gives a_k, b_k, r_k, p_k;
//   for shift j, with s = sigma_j - sigma_0, the residual is zeta_k r_k with
//     zeta_{k+1} = zeta_k zeta_{k-1} a_{k-1}
//                  / (a_k b_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} a_{k-1} (1 + s a_k)),
//   zeta_0 = zeta_{-1} = 1, a_{-1} = 1, b_{-1} = 0, and
//     x_j += a_k zeta_{k+1} / zeta_k p_j,
//     p_j = zeta_{k+1} r_{k+1} + b_k (zeta_{k+1} / zeta_k)^2 p_j.
// FP64 throughout.  X p = gamma5 D^ gamma5 D^ p + mu^2 p (D^dag = gamma5 D^
// gamma5, the gamma5-hermiticity of D carried to the even-odd blocks).  The
// per-shift updates of a step are one streaming kernel over all active
// shifts (the vectors are read once per step); dot products and norms are
// the library's deterministic FP64 reductions.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "blas.h"
#include "host.h"
#include "launch.h"
#include "solver.h"

namespace qxd {

namespace {

constexpr int MS_MAX = 64;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// coefficients of one step for the active shifts (passed by value)
struct MsStep {
  double alpha[MS_MAX], zeta[MS_MAX], beta[MS_MAX];
  int idx[MS_MAX];
  int n;
  double beta0;  // p = r + beta0 p
};

// One step of the shifted recurrences over the even half (npairs FP64
// complex numbers per vector, every vector in the same native layout):
//   x_j += alpha_j p_j;  p_j = zeta_j r + beta_j p_j  (active j);  p = r + beta0 p
__global__ void __launch_bounds__(256) ms_update_kernel(const double2 *__restrict__ r, double2 *__restrict__ p,
                                                        double2 *__restrict__ x, int64_t xstride,
                                                        double2 *__restrict__ ps, int64_t pstride,
                                                        int64_t npairs, MsStep c) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < npairs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double2 rv = r[e];
    const double2 pv = p[e];
    for (int k = 0; k < c.n; k++) {
      const int j = c.idx[k];
      double2 *xj = x + j * xstride + e;
      double2 *pj = ps + j * pstride + e;
      const double2 pjv = *pj;
      double2 xv = *xj;
      xv.x = fma(c.alpha[k], pjv.x, xv.x);
      xv.y = fma(c.alpha[k], pjv.y, xv.y);
      *xj = xv;
      double2 np;
      np.x = fma(c.beta[k], pjv.x, c.zeta[k] * rv.x);
      np.y = fma(c.beta[k], pjv.y, c.zeta[k] * rv.y);
      *pj = np;
    }
    double2 nq;
    nq.x = fma(c.beta0, pv.x, rv.x);
    nq.y = fma(c.beta0, pv.y, rv.y);
    p[e] = nq;
  }
}

// out = a0 (b + sum_j rho_j x_j) over the even half
struct MsComb {
  double rho[MS_MAX];
  int n;
  double a0;
};
__global__ void __launch_bounds__(256) ms_combine_kernel(const double2 *__restrict__ b, const double2 *__restrict__ x,
                                                         int64_t xstride, double2 *__restrict__ out,
                                                         int64_t npairs, MsComb c) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < npairs;
       e += (int64_t)gridDim.x * blockDim.x) {
    double2 s = b[e];
    for (int j = 0; j < c.n; j++) {
      const double2 v = x[j * xstride + e];
      s.x = fma(c.rho[j], v.x, s.x);
      s.y = fma(c.rho[j], v.y, s.y);
    }
    out[e] = make_double2(c.a0 * s.x, c.a0 * s.y);
  }
}

unsigned stream_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::min<int64_t>(std::max<int64_t>(g, 1), 8192);
}

#define MCK(...)                                                                      \
  do {                                                                                \
    hipError_t _e = (__VA_ARGS__);                                                    \
    if (_e != hipSuccess) {                                                           \
      set_error("HIP error %s at %s:%d", hipGetErrorString(_e), __FILE__, __LINE__); \
      return _e == hipErrorOutOfMemory ? QXD_ENOMEM : QXD_EDEVICE;                    \
    }                                                                                 \
  } while (0)
#define MCS(...)                   \
  do {                             \
    qxd_status _s = (__VA_ARGS__); \
    if (_s != QXD_OK) return _s;   \
  } while (0)

struct Ms {
  Field *f;
  const Operator *op;
  double mu2 = 0.0;  // the caller's twisted mass squared (not part of the cached operator)
  hipStream_t st;
  OpFields of;
  size_t fb = 0;      // bytes of a full FP64 native spinor
  void *tmp = nullptr, *u = nullptr, *v = nullptr;
  double *partial = nullptr, *scal = nullptr;
  SpinorArg F(void *p) const { return SpinorArg{p, f->g.V, 0, f->g.rd}; }

  qxd_status fetch(double *h, const double *d, int n) {
    MCK(hipMemcpyAsync(h, d, n * sizeof(double), hipMemcpyDeviceToHost, st));
    MCK(hipStreamSynchronize(st));
    return QXD_OK;
  }
  // q = (D^dag D^ + s) p on the even half of full-lattice native spinors
  qxd_status normal(void *p, void *q, double s) {
    const Geom &g = f->g;
    SpinorArg none{nullptr, 0, 0, g.rd};
    MCK(schur_tm(f, of, QXD_F64, 0.0, F(p), F(u), tmp, st, true));
    MCK(launch_lincomb_sites(QXD_F64, F(u), F(u), 1.0, 0.0, true, none, 0, 0, false, 0, g.Vh, st));
    MCK(schur_tm(f, of, QXD_F64, 0.0, F(u), F(v), tmp, st, true));
    MCK(launch_lincomb_sites(QXD_F64, F(q), F(v), 1.0, 0.0, true, F(p), s, 0.0, false, 0, g.Vh, st));
    return QXD_OK;
  }
};

// The multi-shift CG core: x_j (full native FP64 spinors with zero odd half,
// n of them at xbuf with stride fb) solve (X + shifts[j]) x_j = b_e, b the
// even half of the native spinor bnat.  its[j], res[j]: iterations and true
// relative residual of shift j.
qxd_status ms_core(Ms &m, const double *shifts, int n, double tol, int maxiter, void *bnat, char *xbuf,
                   std::vector<int> &its, std::vector<double> &res, bool *converged) {
  Field *f = m.f;
  const Geom &g = f->g;
  const double mu2 = m.mu2;
  const size_t fb = m.fb, hb = spinor_bytes(QXD_F64, g.Vh);
  hipError_t e;
  char *pbuf = (char *)f->workspace("ms_p", hb * n, &e);
  MCK(e);
  void *r = f->workspace("ms_r", fb, &e);
  MCK(e);
  void *p = f->workspace("ms_pbase", fb, &e);
  MCK(e);
  void *q = f->workspace("ms_q", fb, &e);
  MCK(e);
  double *sc = m.scal;
  auto H = [&](void *ptr) { return SpinorArg{ptr, g.Vh, 0, g.rd}; };
  its.assign(n, 0);
  res.assign(n, 0.0);
  *converged = false;
  // |b|
  MCK(blas_norm2<QXD_F64>(m.F(bnat), 0, g.Vh, m.partial, sc, m.st));
  double bn2;
  MCS(m.fetch(&bn2, sc, 1));
  if (!isfinite(bn2)) {
    set_error("source contains NaN/Inf");
    return QXD_EFLOAT;
  }
  MCK(hipMemsetAsync(xbuf, 0, fb * n, m.st));
  if (bn2 == 0.0) {
    *converged = true;
    return QXD_OK;
  }
  const double bn = sqrt(bn2);
  // r = p = p_j = b
  MCK(hipMemsetAsync(r, 0, fb, m.st));
  MCK(hipMemsetAsync(p, 0, fb, m.st));
  MCK(hipMemsetAsync(q, 0, fb, m.st));
  MCK(hipMemcpyAsync(r, bnat, hb, hipMemcpyDeviceToDevice, m.st));
  MCK(hipMemcpyAsync(p, bnat, hb, hipMemcpyDeviceToDevice, m.st));
  for (int j = 0; j < n; j++) MCK(hipMemcpyAsync(pbuf + j * hb, bnat, hb, hipMemcpyDeviceToDevice, m.st));
  double s0 = INFINITY;
  for (int j = 0; j < n; j++) s0 = std::min(s0, shifts[j] + mu2);
  std::vector<double> ds(n), zeta(n, 1.0), zeta_old(n, 1.0), zeta_new(n, 1.0);
  std::vector<char> active(n, 1);
  for (int j = 0; j < n; j++) ds[j] = shifts[j] + mu2 - s0;
  double rr = bn2, a_old = 1.0, b_old = 0.0;
  const int64_t npairs = (int64_t)12 * g.Vh;
  int nact = n, it = 0;
  while (it < maxiter && nact > 0) {
    MCS(m.normal(p, q, s0));
    SpinorArg pa = m.F(p);
    MCK(blas_mdot<QXD_F64>(&pa, 1, m.F(q), 0, g.Vh, m.partial, sc, nullptr, 0, m.st));
    double pq[2];
    MCS(m.fetch(pq, sc, 2));
    const double a = rr / pq[0];
    if (!isfinite(a) || !(pq[0] > 0.0)) {
      set_error("multi-shift CG breakdown: (p, X p) = %g (X must be positive definite)", pq[0]);
      return QXD_EFLOAT;
    }
    MsStep c;
    c.n = 0;
    for (int j = 0; j < n; j++) {
      if (!active[j]) continue;
      const double den = a * b_old * (zeta_old[j] - zeta[j]) + zeta_old[j] * a_old * (1.0 + ds[j] * a);
      zeta_new[j] = zeta[j] * zeta_old[j] * a_old / den;
      c.idx[c.n] = j;
      c.alpha[c.n] = a * zeta_new[j] / zeta[j];
      c.n++;
    }
    MCK(blas_axpby<QXD_F64, QXD_F64>(H(r), 1.0, H(q), -a, 0, g.Vh, m.partial, sc, m.st));
    double rr_new;
    MCS(m.fetch(&rr_new, sc, 1));
    if (!isfinite(rr_new)) {
      set_error("multi-shift CG residual is NaN/Inf");
      return QXD_EFLOAT;
    }
    const double beta = rr_new / rr;
    for (int k = 0; k < c.n; k++) {
      const int j = c.idx[k];
      const double z = zeta_new[j] / zeta[j];
      c.zeta[k] = zeta_new[j];
      c.beta[k] = beta * z * z;
    }
    c.beta0 = beta;
    ms_update_kernel<<<stream_grid(npairs), 256, 0, m.st>>>((const double2 *)r, (double2 *)p, (double2 *)xbuf,
                                                           (int64_t)(fb / 16), (double2 *)pbuf,
                                                           (int64_t)(hb / 16), npairs, c);
    MCK(hipGetLastError());
    it++;
    for (int k = 0; k < c.n; k++) {
      const int j = c.idx[k];
      zeta_old[j] = zeta[j];
      zeta[j] = zeta_new[j];
      its[j] = it;
      if (fabs(zeta[j]) * sqrt(rr_new) <= tol * bn) {
        active[j] = 0;
        nact--;
      }
    }
    a_old = a;
    b_old = beta;
    rr = rr_new;
  }
  *converged = nact == 0;
  // true residuals |b - (X + shift_j) x_j| / |b|
  for (int j = 0; j < n; j++) {
    MCS(m.normal(xbuf + j * fb, q, shifts[j] + mu2));
    MCK(blas_axpby<QXD_F64, QXD_F64>(H(q), -1.0, H(bnat), 1.0, 0, g.Vh, m.partial, sc, m.st));
    double r2;
    MCS(m.fetch(&r2, sc, 1));
    res[j] = sqrt(r2) / bn;
  }
  return QXD_OK;
}

qxd_status ms_setup(Field *f, const qxd_quark &quark, hipStream_t st, Ms *m) {
  m->f = f;
  m->st = st;
  Operator *op;
  MCS(f->get_op(quark, QXD_F64, &op, st));
  m->op = op;
  m->mu2 = quark.mu * quark.mu;
  m->of = f->op_fields(*op, QXD_F64);
  const Geom &g = f->g;
  m->fb = spinor_bytes(QXD_F64, g.V);
  hipError_t e;
  m->tmp = f->workspace("dhat_tmp", spinor_bytes(QXD_F64, g.Vh), &e);
  MCK(e);
  m->u = f->workspace("ms_u", m->fb, &e);
  MCK(e);
  m->v = f->workspace("ms_v", m->fb, &e);
  MCK(e);
  m->partial = (double *)f->workspace("partial", blas_partial_doubles() * 8, &e);
  MCK(e);
  m->scal = (double *)f->workspace("ms_scalars", 64 * 8, &e);
  MCK(e);
  // odd halves of the work vectors stay zero
  MCK(hipMemsetAsync(m->u, 0, m->fb, st));
  MCK(hipMemsetAsync(m->v, 0, m->fb, st));
  return QXD_OK;
}

void fill_info(qxd_solve_info *info, int n, const std::vector<int> &its, const std::vector<double> &res,
               double tol, double t0) {
  if (!info) return;
  const double dt = now_s() - t0;
  for (int j = 0; j < n; j++) {
    info[j].status = res[j] <= tol ? QXD_OK : QXD_ENOCONV;
    info[j].outer_iters = 1;
    info[j].inner_iters = its[j];
    info[j].true_resid = res[j];
    info[j].seconds = dt;
  }
}

}  // namespace

qxd_status multishift_solve(Field *f, const qxd_quark &quark, const double *shifts, int n, double tol,
                            int maxiter, const double *eta_api, double *psi_api, qxd_solve_info *info,
                            hipStream_t st) {
  const double t0 = now_s();
  Ms m;
  MCS(ms_setup(f, quark, st, &m));
  const Geom &g = f->g;
  hipError_t e;
  void *bnat = f->workspace("ms_b", m.fb, &e);
  MCK(e);
  char *xbuf = (char *)f->workspace("ms_x", m.fb * n, &e);
  MCK(e);
  MCK(launch_pack(QXD_F64, g, eta_api, bnat, 1, st));
  std::vector<int> its;
  std::vector<double> res;
  bool conv;
  MCS(ms_core(m, shifts, n, tol, maxiter > 0 ? maxiter : 100000, bnat, xbuf, its, res, &conv));
  for (int j = 0; j < n; j++) MCK(launch_unpack(QXD_F64, g, xbuf + j * m.fb, psi_api + (int64_t)j * 24 * g.V, 1, st));
  MCK(hipStreamSynchronize(st));
  fill_info(info, n, its, res, tol, t0);
  return conv ? QXD_OK : QXD_ENOCONV;
}

qxd_status rational_apply(Field *f, const qxd_quark &quark, double A, const double *nu, const double *mu, int n,
                          double tol, int maxiter, const double *eta_api, double *out_api, qxd_solve_info *info,
                          hipStream_t st) {
  const double t0 = now_s();
  // partial fractions: R(t) / A = 1 + sum_j rho_j / (t + mu_j^2), rho_j the
  // residue of prod_k (t + nu_k^2) / (t + mu_k^2) at t = -mu_j^2
  MsComb c;
  c.n = n;
  c.a0 = A;
  std::vector<double> poles(n);
  for (int j = 0; j < n; j++) {
    const double bj = mu[j] * mu[j];
    poles[j] = bj;
    double num = 1.0, den = 1.0;
    for (int k = 0; k < n; k++) {
      num *= nu[k] * nu[k] - bj;
      if (k != j) den *= mu[k] * mu[k] - bj;
    }
    if (den == 0.0 || !isfinite(num / den)) {
      set_error("the poles mu_j^2 of a rational function must be distinct");
      return QXD_EINVAL;
    }
    c.rho[j] = num / den;
  }
  Ms m;
  MCS(ms_setup(f, quark, st, &m));
  const Geom &g = f->g;
  hipError_t e;
  void *bnat = f->workspace("ms_b", m.fb, &e);
  MCK(e);
  char *xbuf = (char *)f->workspace("ms_x", m.fb * n, &e);
  MCK(e);
  void *out = f->workspace("ms_out", m.fb, &e);
  MCK(e);
  MCK(launch_pack(QXD_F64, g, eta_api, bnat, 1, st));
  std::vector<int> its;
  std::vector<double> res;
  bool conv;
  MCS(ms_core(m, poles.data(), n, tol, maxiter > 0 ? maxiter : 100000, bnat, xbuf, its, res, &conv));
  MCK(hipMemsetAsync(out, 0, m.fb, st));
  const int64_t npairs = (int64_t)12 * g.Vh;
  ms_combine_kernel<<<stream_grid(npairs), 256, 0, st>>>((const double2 *)bnat, (const double2 *)xbuf,
                                                        (int64_t)(m.fb / 16), (double2 *)out, npairs, c);
  MCK(hipGetLastError());
  MCK(launch_unpack(QXD_F64, g, out, out_api, 1, st));
  MCK(hipStreamSynchronize(st));
  fill_info(info, n, its, res, tol, t0);
  return conv ? QXD_OK : QXD_ENOCONV;
}

}  // namespace qxd
