// Local deflation of the SAP-GCR, host side (the method in dfl.h).
#include <math.h>

#include <chrono>
#include <memory>
#include <vector>

#include "blas.h"
#include "dfl.h"
#include "qxd_debug.h"
#include "sap.h"
#include "solver.h"

namespace qxd {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

#define DCK(...)                                                                      \
  do {                                                                                 \
    hipError_t _e = (__VA_ARGS__);                                                          \
    if (_e != hipSuccess) {                                                            \
      set_error("HIP error %s at %s:%d", hipGetErrorString(_e), __FILE__, __LINE__);  \
      return _e == hipErrorOutOfMemory ? QXD_ENOMEM : QXD_EDEVICE;                     \
    }                                                                                  \
  } while (0)
#define DCS(...)                        \
  do {                                   \
    qxd_status _s = (__VA_ARGS__);            \
    if (_s != QXD_OK) return _s;         \
  } while (0)

qxd_status fetch(double *host, const double *dev, int n, hipStream_t st) {
  DCK(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, st));
  DCK(hipStreamSynchronize(st));
  return QXD_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// the field's workspace `name` of at least `bytes`
qxd_status ws(Field *f, const char *name, size_t bytes, void **p) {
  hipError_t e;
  *p = f->workspace(name, bytes, &e);
  if (e != hipSuccess) {
    set_error("workspace allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? QXD_ENOMEM : QXD_EDEVICE;
  }
  return QXD_OK;
}

SpinorArg full(const Geom &g, void *p) { return SpinorArg{p, g.V, 0, g.rd}; }

// scalars of the little GCR on the device
constexpr int LS_DOTS = 8, LS_WN = 8 + 2 * 64, LS_N = LS_WN + 64 + 8;

// x = A^-1 b approximately, on the even-block Schur complement
//   Ahat = A_ee - A_eo A_oo^-1 A_oe,   Ahat x_e = b_e - A_eo A_oo^-1 b_o,
//   x_o = A_oo^-1 (b_o - A_oe x_e),
// by GCR right-preconditioned with A_ee^-1: z_k = A_ee^-1 r and w_k = Ahat z_k
// made orthogonal to the earlier w, x and r updated at every step; stops at
// |r| <= tol |b_e - A_eo A_oo^-1 b_o| or maxiter iterations.  In the little
// vectors the even blocks come first (positions 0 .. ne - 1), so r, z, w
// and the Gram-Schmidt work on the first ne * ns entries only; b, x and u
// are full length.
// The host reads the residual norm of step j while step j + 1 is already
// queued, so the device never waits for the host; the step queued past
// convergence is kept (it only lowers the residual further).
template <class MT>
qxd_status little_solve_t(Dfl &d, const MT *A, const double2 *b, double2 *x, double tol, int *iters,
                          hipStream_t st) {
  const int nkv = d.p.little_nkv, ns = d.ns, maxiter = d.p.little_maxiter, ne = d.ne;
  const int64_t n = (int64_t)ne * ns;  // entries of the even blocks
  double2 *Z = d.lz.as<double2>(), *W = d.lw.as<double2>(), *r = d.lr.as<double2>();
  double2 *u = d.lu.as<double2>();
  double *part = d.lpart.as<double>(), *sc = d.lscal.as<double>();
  const float2 *Ai = d.ait32.as<float2>();
  const int *nbrv = d.nbrv.as<int>(), *ev = d.even.as<int>(), *od = d.odd.as<int>();
  // x starts at 0 (x_o is written at the end); r, z_k and w_k are written
  // whole before they are read
  DCK(hipMemsetAsync(x, 0, (size_t)d.nb * ns * sizeof(double2), st));
  // r_e = b_e - A_eo A_oo^-1 b_o
  DCK(launch_lt_jacobi(od, d.no, ne, ns, Ai, 1.0, b, u, st));
  DCK(launch_lt_hop(ev, ne, 0, ns, A, nbrv, nullptr, b, u, nullptr, 1.0, r, st));
  // |r_0|^2 goes to host slot 2; the host reads it after the first step
  // (a zero residual makes every step a no-op)
  DCK(launch_lv_dot2(r, r, n, part, d.sync.dev + 2, st));
  // step j: Krylov slot j mod nkv (a restart every nkv steps); its |r|^2 goes
  // to host slot j mod 2
  auto step = [&](int j) -> qxd_status {
    const int k = j % nkv;
    double2 *zk = Z + (int64_t)k * n, *wk = W + (int64_t)k * n;
    DCK(launch_lt_jacobi(ev, ne, 0, ns, Ai, 1.0, r, zk, st));
    // w_e = A_ee z - A_eo u_o with u_o = A_oo^-1 A_oe z (-A_oe z is what
    // the hop makes)
    DCK(launch_lt_hop(od, d.no, ne, ns, A, nbrv, nullptr, nullptr, zk, Ai, -1.0, u, st));
    DCK(launch_lt_hop(ev, ne, 0, ns, A, nbrv, zk, nullptr, u, nullptr, 1.0, wk, st));
    if (k > 0) {
      DCK(launch_lv_dots(W, k, n, wk, part, sc + LS_DOTS, st));
      DCK(launch_lv_maxpy2(wk, W, zk, Z, k, n, sc + LS_DOTS, sc + LS_WN, st));
    }
    DCK(launch_lv_dot2(wk, r, n, part, nullptr, st));
    DCK(launch_lv_update(x, zk, r, wk, n, sc + LS_WN + k, part, d.sync.dev + (j & 1), st));
    DCK(hipEventRecord(d.sync.ev[j & 1], st));
    return QXD_OK;
  };
  int launched = 0;
  double bn2 = 0.0;
  DCS(step(launched++));
  for (int j = 0;; j++) {
    if (launched < maxiter) DCS(step(launched++));
    DCK(hipEventSynchronize(d.sync.ev[j & 1]));
    if (j == 0) {
      bn2 = d.sync.host[2];
      if (!isfinite(bn2)) {
        DCK(hipStreamSynchronize(st));
        set_error("little system: right-hand side is NaN/Inf");
        return QXD_EFLOAT;
      }
    }
    const double rr = d.sync.host[j & 1];
    if (!isfinite(rr)) {
      DCK(hipStreamSynchronize(st));
      set_error("little system: residual is NaN/Inf");
      return QXD_EFLOAT;
    }
    if (rr <= tol * tol * bn2 || j + 1 >= launched) break;
  }
  // x_o = A_oo^-1 (b_o - A_oe x_e)
  DCK(launch_lt_hop(od, d.no, ne, ns, A, nbrv, nullptr, b, x, Ai, 1.0, x, st));
  if (iters) *iters = launched;
  return QXD_OK;
}

// Little solves to a relative residual of at least HALF_LITTLE_TOL read the
// FP16 copy of A (half the bytes of the two hops that dominate a step; its
// 11-bit mantissa perturbs the little operator far below such a tolerance),
// tighter ones the FP32 copy.
constexpr double HALF_LITTLE_TOL = 1e-2;

qxd_status little_solve(Dfl &d, const double2 *b, double2 *x, double tol, int *iters, hipStream_t st) {
  if (tol >= HALF_LITTLE_TOL) return little_solve_t(d, d.at16.as<h2_t>(), b, x, tol, iters, st);
  return little_solve_t(d, d.at32.as<float2>(), b, x, tol, iters, st);
}

qxd_status fill_params(qxd_dfl_params *p) {
  if (p->ns == 0) p->ns = 16;
  if (p->ninv == 0) p->ninv = 30;
  if (p->ncy == 0) p->ncy = 4;
  if (p->nmr == 0) p->nmr = 4;
  if (p->little_tol == 0.0) p->little_tol = 0.2;
  if (p->little_nkv == 0) p->little_nkv = 48;
  if (p->little_maxiter == 0) p->little_maxiter = 256;
  if (p->ns < 1 || p->ns > DFL_NSMAX || p->ninv < 0 || p->ncy < 1 || p->nmr < 0 || !(p->little_tol > 0.0) ||
      p->little_tol >= 1.0 || p->little_nkv < 1 || p->little_nkv > 64 || p->little_maxiter < 1) {
    set_error("invalid deflation parameters (ns 1..%d, ncy >= 1, 0 < little_tol < 1, little_nkv 1..64)",
              DFL_NSMAX);
    return QXD_EINVAL;
  }
  return QXD_OK;
}

// the quark's operator with its deflation subspace, or QXD_EINVAL
qxd_status op_with_dfl(Field *f, const qxd_quark &q, Operator **op, hipStream_t st) {
  DCS(f->get_op(q, QXD_F64, op, st));
  DCS(f->get_op(q, QXD_F32, op, st));
  if (!(*op)->dfl) {
    set_error("no deflation subspace for this quark: call qxd_dfl_setup first");
    return QXD_EINVAL;
  }
  return QXD_OK;
}

}  // namespace

size_t Dfl::bytes() const {
  return basis.n + a.n + ainv.n + at32.n + ait32.n + at16.n + nbr.n + even.n + odd.n + vpos.n + nbrv.n + lz.n + lw.n +
         lx.n + lr.n + lb.n + lu.n + lpart.n + lscal.n;
}

qxd_status dfl_setup(Field *f, const qxd_quark &q, const qxd_dfl_params *pin, const double *init_api,
                     hipStream_t st) {
  qxd_dfl_params p = pin ? *pin : qxd_dfl_params{};
  DCS(fill_params(&p));
  DCS(check_sap_blocks(f));
  const Geom &g = f->g;
  if (2 * g.Vbh > 256) {
    set_error("deflation needs SAP blocks of at most 256 sites");
    return QXD_EINVAL;
  }
  Operator *op;
  DCS(f->get_op(q, QXD_F64, &op, st));
  DCS(f->get_op(q, QXD_F32, &op, st));
  op->dfl.reset();  // free an earlier subspace first
  std::shared_ptr<Dfl> d = std::make_shared<Dfl>();
  d->p = p;
  d->ns = p.ns;
  d->nb = g.nblocks;
  d->vbytes = align256(spinor_bytes(QXD_F32, g.V));
  const int ns = d->ns;
  DCK(d->basis.ensure(d->vbytes * ns));
  char *basis = (char *)d->basis.p;
  void *t32, *partial, *scal;
  DCS(ws(f, "dfl_t32", spinor_bytes(QXD_F32, g.V), &t32));
  DCS(ws(f, "partial", blas_partial_doubles() * 8, &partial));
  DCS(ws(f, "dfl_scal", 64 * 8, &scal));
  double *misc = (double *)scal;
  // start fields
  if (init_api) {
    for (int k = 0; k < ns; k++)
      DCK(launch_pack(QXD_F32, g, init_api + (int64_t)k * 24 * g.V, basis + (size_t)k * d->vbytes, 1, st));
  } else {
    DCK(launch_dfl_random(g, basis, d->vbytes, ns, p.seed, st));
  }
  // SAP-smoothed inverse iteration: psi <- psi / |psi|, then ninv times
  // psi <- M_sap psi / |M_sap psi|
  auto field = [&](int k) -> void * { return basis + (size_t)k * d->vbytes; };
  // v_k = src / |src| (with a zero coefficient the old v_k is not read)
  auto normalise = [&](int k, void *src) -> qxd_status {
    void *v = field(k);
    DCK(blas_norm2<QXD_F32>(full(g, src), 0, g.V, (double *)partial, misc, st));
    double n2;
    DCS(fetch(&n2, misc, 1, st));
    if (!(n2 > 0.0) || !isfinite(n2)) {
      set_error("deflation field %d vanished or is not finite in inverse iteration", k);
      return QXD_EFLOAT;
    }
    const double sc = 1.0 / sqrt(n2);
    DCK(blas_axpby<QXD_F32, QXD_F32>(full(g, v), src == v ? sc : 0.0, full(g, src), src == v ? 0.0 : sc, 0, g.V,
                                     (double *)partial, nullptr, st));
    return QXD_OK;
  };
  int k0 = 0;
  if (ns > 1 && sap_quad_pairs_ok(QXD_F32, g)) {
    // two fields at a time through the paired SAP block solver (links and
    // Pauli rows staged once per block for both; per field the same
    // arithmetic as sap_apply): slot k reads field k and writes t32 (k even)
    // or t32b (k odd), with its own two work vectors
    const size_t fb = spinor_bytes(QXD_F32, g.V);
    void *t32b, *rv, *dslots, *dpairs;
    DCS(ws(f, "dfl_t32b", fb, &t32b));
    DCS(ws(f, "dfl_pair_rv", 4 * fb, &rv));
    DCS(ws(f, "dfl_pair_slots", (size_t)ns * sizeof(SapSlot<QXD_F32>), &dslots));
    DCS(ws(f, "dfl_pair_idx", (size_t)ns * sizeof(int), &dpairs));
    const OpFields of = f->op_fields(*op, QXD_F32);
    using PT = typename St<QXD_F32>::pair_t;
    std::vector<SapSlot<QXD_F32>> hs(ns);
    std::vector<int> hp(ns);
    for (int k = 0; k < ns; k++) {
      char *w = (char *)rv + (size_t)2 * (k & 1) * fb;
      hs[k].op = SapOp<QXD_F32>{(const PT *)of.links, nullptr, 0, (const PT *)of.pauli, (const PT *)of.pinv};
      hs[k].vec = SapVecs<QXD_F32>{spinor_view<QXD_F32>(field(k), g.V, 0, g), spinor_view<QXD_F32>(w, g.V, 0, g),
                                   spinor_view<QXD_F32>(k & 1 ? t32b : t32, g.V, 0, g),
                                   spinor_view<QXD_F32>(w + fb, g.V, 0, g)};
      hp[k] = k;
    }
    DCK(hipMemcpyAsync(dslots, hs.data(), hs.size() * sizeof(SapSlot<QXD_F32>), hipMemcpyHostToDevice, st));
    DCK(hipMemcpyAsync(dpairs, hp.data(), hp.size() * sizeof(int), hipMemcpyHostToDevice, st));
    DCK(hipStreamSynchronize(st));
    const int *lists[2];
    int nper;
    DCS(sap_block_lists(f, lists, &nper));
    for (; k0 + 1 < ns; k0 += 2) {
      for (int it = 0; it <= p.ninv; it++) {
        if (it > 0) {
          for (int cy = 0; cy < p.ncy; cy++)
            for (int c = 0; c < 2; c++)
              DCK(launch_sapq_pairs<QXD_F32>(g, lists[c], nper, (const SapSlot<QXD_F32> *)dslots,
                                             (const int *)dpairs + k0, 1, cy == 0, cy == 0 && c == 0, p.nmr, st));
        }
        DCS(normalise(k0, it > 0 ? t32 : field(k0)));
        DCS(normalise(k0 + 1, it > 0 ? t32b : field(k0 + 1)));
      }
    }
  }
  for (int k = k0; k < ns; k++) {
    for (int it = 0; it <= p.ninv; it++) {
      void *src = field(k);  // the field to normalise into v_k: v_k itself, then M_sap v_k
      if (it > 0) {
        DCS(sap_apply(f, *op, QXD_F32, p.ncy, p.nmr, field(k), t32, st));
        src = t32;
      }
      DCS(normalise(k, src));
    }
  }
  // block orthonormalisation
  int *bad = (int *)misc;
  DCK(hipMemsetAsync(bad, 0, sizeof(int), st));
  DCK(launch_dfl_ortho(g, basis, d->vbytes, ns, bad, st));
  int nbad = 0;
  DCK(hipMemcpyAsync(&nbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  DCK(hipStreamSynchronize(st));
  if (nbad) {
    set_error("a deflation field vanishes on %d blocks (ns too large for the block?)", nbad);
    return QXD_EFLOAT;
  }
  // little operator in FP64
  const size_t nn = (size_t)ns * ns;
  DCK(d->a.ensure((size_t)d->nb * DFL_SLOTS * nn * sizeof(double2)));
  DCK(d->nbr.ensure((size_t)d->nb * DFL_SLOTS * sizeof(int)));
  DCK(d->ainv.ensure((size_t)d->nb * nn * sizeof(double2)));
  void *x64, *y64;
  DCS(ws(f, "dfl_x64", spinor_bytes(QXD_F64, g.V), &x64));
  DCS(ws(f, "dfl_y64", spinor_bytes(QXD_F64, g.V), &y64));
  const OpFields of64 = f->op_fields(*op, QXD_F64);
  for (int l = 0; l < ns; l++) {
    const void *bl = basis + (size_t)l * d->vbytes;
    DCK(launch_dfl_face(g, (const double2 *)of64.links, basis, d->vbytes, ns, l, d->a.as<double2>(),
                        d->nbr.as<int>(), st));
    DCK(blas_axpby<QXD_F64, QXD_F32>(full(g, x64), 0.0, full(g, (void *)bl), 1.0, 0, g.V, (double *)partial,
                                     nullptr, st));
    DCS(apply_native(f, *op, 0.0, QXD_OP_D, QXD_F64, x64, y64, st));
    DCK(launch_dfl_diag(g, basis, d->vbytes, ns, l, y64, d->a.as<double2>(), d->nbr.as<int>(), st));
  }
  DCK(hipMemsetAsync(bad, 0, sizeof(int), st));
  DCK(launch_little_invert(d->nb, ns, d->a.as<double2>(), d->ainv.as<double2>(), bad, st));
  DCK(hipMemcpyAsync(&nbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  DCK(hipStreamSynchronize(st));
  if (nbad) {
    set_error("the little operator has %d singular diagonal blocks", nbad);
    return QXD_EFLOAT;
  }
  DCK(d->at32.ensure((size_t)d->nb * DFL_SLOTS * nn * sizeof(float2)));
  DCK(d->ait32.ensure((size_t)d->nb * nn * sizeof(float2)));
  DCK(d->at16.ensure((size_t)d->nb * DFL_SLOTS * nn * sizeof(h2_t)));
  DCK(launch_little_pack((int64_t)d->nb * DFL_SLOTS, ns, d->a.as<double2>(), d->at32.as<float2>(), st));
  DCK(launch_little_pack((int64_t)d->nb * DFL_SLOTS, ns, d->a.as<double2>(), d->at16.as<h2_t>(), st));
  DCK(launch_little_pack((int64_t)d->nb, ns, d->ainv.as<double2>(), d->ait32.as<float2>(), st));
  // the blocks of each colour: the parity of the block coordinates, as for
  // SAP (the two-colour check guarantees that neighbours differ)
  {
    std::vector<int> ev, od;
    for (int b = 0; b < d->nb; b++) {
      int c = b, sum = 0;
      for (int m = 3; m >= 0; m--) {
        sum += c % g.nb[m];
        c /= g.nb[m];
      }
      (sum & 1 ? od : ev).push_back(b);
    }
    d->ne = (int)ev.size();
    d->no = (int)od.size();
    DCK(d->even.ensure(ev.size() * sizeof(int)));
    DCK(d->odd.ensure(od.size() * sizeof(int)));
    DCK(hipMemcpyAsync(d->even.p, ev.data(), ev.size() * sizeof(int), hipMemcpyHostToDevice, st));
    DCK(hipMemcpyAsync(d->odd.p, od.data(), od.size() * sizeof(int), hipMemcpyHostToDevice, st));
    // positions in the little vectors: the even blocks, then the odd ones;
    // the neighbour table in those positions
    std::vector<int> vpos(d->nb), nbr((size_t)d->nb * DFL_SLOTS), nbrv((size_t)d->nb * DFL_SLOTS);
    for (int i = 0; i < d->ne; i++) vpos[ev[i]] = i;
    for (int i = 0; i < d->no; i++) vpos[od[i]] = d->ne + i;
    DCK(hipMemcpyAsync(nbr.data(), d->nbr.p, nbr.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    DCK(hipStreamSynchronize(st));
    for (size_t i = 0; i < nbr.size(); i++) {
      if (nbr[i] < 0 || nbr[i] >= d->nb) {
        set_error("little operator: neighbour table out of range");
        return QXD_EDEVICE;
      }
      nbrv[i] = vpos[nbr[i]];
    }
    DCK(d->vpos.ensure(vpos.size() * sizeof(int)));
    DCK(d->nbrv.ensure(nbrv.size() * sizeof(int)));
    DCK(hipMemcpyAsync(d->vpos.p, vpos.data(), vpos.size() * sizeof(int), hipMemcpyHostToDevice, st));
    DCK(hipMemcpyAsync(d->nbrv.p, nbrv.data(), nbrv.size() * sizeof(int), hipMemcpyHostToDevice, st));
    DCK(hipStreamSynchronize(st));
  }
  // little GCR workspace
  const size_t n = (size_t)d->nb * ns;
  DCK(d->lu.ensure(n * sizeof(double2)));
  DCK(d->lz.ensure((size_t)p.little_nkv * n * sizeof(double2)));
  DCK(d->lw.ensure((size_t)p.little_nkv * n * sizeof(double2)));
  DCK(d->lx.ensure(n * sizeof(double2)));
  DCK(d->lr.ensure(n * sizeof(double2)));
  DCK(d->lb.ensure(n * sizeof(double2)));
  DCK(d->lpart.ensure(lv_partial_doubles() * sizeof(double)));
  DCK(d->lscal.ensure(LS_N * sizeof(double)));
  DCK(d->sync.init());
  op->dfl = d;
  return QXD_OK;
}

qxd_status dfl_precond(Field *f, Operator &op, double little_tol, int ncy, int nmr, void *r32, void *out32,
                       hipStream_t st, int *little_iters) {
  Dfl &d = *op.dfl;
  const Geom &g = f->g;
  void *u, *t, *partial;
  DCS(ws(f, "dfl_u", spinor_bytes(QXD_F32, g.V), &u));
  DCS(ws(f, "dfl_t", spinor_bytes(QXD_F32, g.V), &t));
  DCS(ws(f, "partial", blas_partial_doubles() * 8, &partial));
  // u = V A^-1 V^dag r
  DCK(launch_dfl_restrict(g, d.basis.p, d.vbytes, d.ns, r32, d.vpos.as<int>(), d.lb.as<double2>(), st));
  int lit = 0;
  DCS(little_solve(d, d.lb.as<double2>(), d.lx.as<double2>(), little_tol > 0.0 ? little_tol : d.p.little_tol,
                   &lit, st));
  if (little_iters) *little_iters = lit;
  d.applications++;
  d.little_iters += lit;
  if (lit > d.little_max) d.little_max = lit;
  DCK(launch_dfl_prolong(g, d.basis.p, d.vbytes, d.ns, d.lx.as<double2>(), d.vpos.as<int>(), u, st));
  // out = u + M_sap (r - D u)
  DCS(apply_native(f, op, 0.0, QXD_OP_D, QXD_F32, u, t, st));
  DCK(blas_axpby<QXD_F32, QXD_F32>(full(g, t), -1.0, full(g, r32), 1.0, 0, g.V, (double *)partial, nullptr, st));
  DCS(sap_apply(f, op, QXD_F32, ncy, nmr, t, out32, st));
  DCK(blas_axpby<QXD_F32, QXD_F32>(full(g, out32), 1.0, full(g, u), 1.0, 0, g.V, (double *)partial, nullptr,
                                   st));
  return QXD_OK;
}

qxd_status dfl_solve(Field *f, Operator &op, const qxd_solver &s, void *eta, void *psi, bool guess,
                     qxd_solve_info *info, hipStream_t st) {
  const Geom &g = f->g;
  const int nkv = s.nkv > 0 ? s.nkv : 32;
  const int ncy = s.ncy > 0 ? s.ncy : 4, nmr = s.nmr > 0 ? s.nmr : 4;
  const double inner_tol = s.inner_tol > 0.0 ? s.inner_tol : 1e-5;
  const int maxiter = s.maxiter > 0 ? s.maxiter : 100000;
  const int max_outer = s.max_outer > 0 ? s.max_outer : 100;
  if (nkv > MAXV) {
    set_error("nkv must be <= %d", MAXV);
    return QXD_EINVAL;
  }
  const size_t fb32 = spinor_bytes(QXD_F32, g.V), fb64 = spinor_bytes(QXD_F64, g.V);
  void *pv, *qv, *x32, *rho, *rho0, *z, *r64, *t64, *partial, *scal;
  DCS(ws(f, "dfl_p", fb32 * nkv, &pv));
  DCS(ws(f, "dfl_q", fb32 * nkv, &qv));
  DCS(ws(f, "dfl_x32", fb32, &x32));
  DCS(ws(f, "dfl_rho", fb32, &rho));
  DCS(ws(f, "dfl_rho0", fb32, &rho0));
  DCS(ws(f, "dfl_z", fb32, &z));
  DCS(ws(f, "dfl_r64", fb64, &r64));
  DCS(ws(f, "dfl_t64", fb64, &t64));
  DCS(ws(f, "partial", blas_partial_doubles() * 8, &partial));
  DCS(ws(f, "dfl_solve_scal", (size_t)(2 * MAXV + 3 * MAXV + 16) * 8, &scal));
  double *beta = (double *)scal, *rec = beta + 2 * MAXV, *rn2 = rec + 3 * MAXV, *misc = rn2 + 4;
  double *part = (double *)partial;
  std::vector<SpinorArg> ps(nkv), qs(nkv);
  for (int k = 0; k < nkv; k++) {
    ps[k] = full(g, (char *)pv + k * fb32);
    qs[k] = full(g, (char *)qv + k * fb32);
  }
  const SpinorArg E = full(g, eta), X = full(g, psi), R64 = full(g, r64), T64 = full(g, t64);
  const SpinorArg X32 = full(g, x32), RHO = full(g, rho), RHO0 = full(g, rho0), Z = full(g, z);
  DCK(blas_norm2<QXD_F64>(E, 0, g.V, part, misc, st));
  double eta2;
  DCS(fetch(&eta2, misc, 1, st));
  if (!isfinite(eta2)) {
    set_error("source contains NaN/Inf");
    return QXD_EFLOAT;
  }
  if (eta2 == 0.0) {
    DCK(hipMemsetAsync(psi, 0, fb64, st));
    if (info) *info = qxd_solve_info{QXD_OK, 0, 0, 0.0, 0.0};
    return QXD_OK;
  }
  const double eta_n = sqrt(eta2);
  if (!guess) DCK(hipMemsetAsync(psi, 0, fb64, st));
  int outer = 0, inner = 0;
  double res = INFINITY;
  for (;;) {
    // r = eta - D psi in FP64
    DCS(apply_native(f, op, 0.0, QXD_OP_D, QXD_F64, psi, t64, st));
    DCK(blas_axpby<QXD_F64, QXD_F64>(R64, 0.0, E, 1.0, 0, g.V, part, nullptr, st));
    DCK(blas_axpby<QXD_F64, QXD_F64>(R64, 1.0, T64, -1.0, 0, g.V, part, misc, st));
    double r2;
    DCS(fetch(&r2, misc, 1, st));
    if (!isfinite(r2)) {
      set_error("residual is NaN/Inf");
      return QXD_EFLOAT;
    }
    res = sqrt(r2) / eta_n;
    if (res <= s.tol || outer >= max_outer || inner >= maxiter) break;
    // inner: D x = r / |r| by flexible GCR(M_dfl) in FP32, to inner_tol
    const double sc = sqrt(r2);
    DCK(blas_axpby<QXD_F32, QXD_F64>(RHO0, 0.0, R64, 1.0 / sc, 0, g.V, part, nullptr, st));
    DCK(blas_axpby<QXD_F32, QXD_F32>(RHO, 0.0, RHO0, 1.0, 0, g.V, part, rn2, st));
    DCK(hipMemsetAsync(x32, 0, fb32, st));
    double rr;
    DCS(fetch(&rr, rn2, 1, st));
    while (sqrt(rr) > inner_tol && inner < maxiter) {
      for (int k = 0; k < nkv && inner < maxiter; k++) {
        DCS(dfl_precond(f, op, 0.0, ncy, nmr, rho, z, st));
        DCS(apply_native(f, op, 0.0, QXD_OP_D, QXD_F32, z, qs[k].ptr, st));
        if (k > 0) DCK(blas_mdot<QXD_F32>(qs.data(), k, qs[k], 0, g.V, part, beta, rec, 3, st));
        MaxpyHost m;
        m.n = k;
        m.ntriples = 2;
        m.src[0] = qs[k];
        m.dst[0] = qs[k];
        m.ys[0] = qs.data();
        m.src[1] = Z;
        m.dst[1] = ps[k];
        m.ys[1] = ps.data();
        m.coef = beta;
        m.w = RHO;
        DCK(blas_maxpy<QXD_F32>(m, 0, g.V, part, rec + 3 * k, st));
        DCK(blas_update<QXD_F32>(X32, ps[k], rec + 3 * k + 1, rec + 3 * k, 1, 0, g.V, part, misc, st));
        DCK(blas_update<QXD_F32>(RHO, qs[k], rec + 3 * k + 1, rec + 3 * k, 0, 0, g.V, part, rn2, st));
        DCS(fetch(&rr, rn2, 1, st));
        inner++;
        if (!isfinite(rr)) {
          set_error("inner GCR residual is NaN/Inf");
          return QXD_EFLOAT;
        }
        if (sqrt(rr) <= inner_tol) break;
      }
      // restart: rho = rho0 - D x
      DCS(apply_native(f, op, 0.0, QXD_OP_D, QXD_F32, x32, z, st));
      DCK(blas_axpby<QXD_F32, QXD_F32>(RHO, 0.0, RHO0, 1.0, 0, g.V, part, nullptr, st));
      DCK(blas_axpby<QXD_F32, QXD_F32>(RHO, 1.0, Z, -1.0, 0, g.V, part, rn2, st));
      DCS(fetch(&rr, rn2, 1, st));
    }
    // psi += |r| x
    DCK(blas_axpby<QXD_F64, QXD_F32>(X, 1.0, X32, sc, 0, g.V, part, nullptr, st));
    outer++;
  }
  if (info) {
    info->outer_iters = outer;
    info->inner_iters = inner;
    info->true_resid = res;
  }
  return res <= s.tol ? QXD_OK : QXD_ENOCONV;
}

}  // namespace qxd

using namespace qxd;

extern "C" {

qxd_status qxd_dfl_setup(qxd_field *field, const qxd_quark *quark, const qxd_dfl_params *params,
                         const double *init_dev, void *stream) {
  if (!field || !quark) {
    set_error("field or quark is NULL");
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  DCK(hipSetDevice(field->ctx->device));
  return dfl_setup(field, *quark, params, init_dev, (hipStream_t)stream);
}

qxd_status qxd_debug_dfl_basis(qxd_field *field, const qxd_quark *quark, int k, double *out_dev, void *stream) {
  if (!field || !quark || !out_dev) {
    set_error("invalid arguments to qxd_debug_dfl_basis");
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  hipStream_t st = (hipStream_t)stream;
  DCK(hipSetDevice(field->ctx->device));
  Operator *op;
  DCS(op_with_dfl(field, *quark, &op, st));
  const Dfl &d = *op->dfl;
  if (k < 0 || k >= d.ns) {
    set_error("basis field %d out of range (ns = %d)", k, d.ns);
    return QXD_EINVAL;
  }
  DCK(launch_unpack(QXD_F32, field->g, (const char *)d.basis.p + (size_t)k * d.vbytes, out_dev, 1, st));
  DCK(hipStreamSynchronize(st));
  return QXD_OK;
}

qxd_status qxd_debug_dfl_little(qxd_field *field, const qxd_quark *quark, int *ns, int *nblocks, double *a,
                                int *nbr) {
  if (!field || !quark || !ns || !nblocks) {
    set_error("invalid arguments to qxd_debug_dfl_little");
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  DCK(hipSetDevice(field->ctx->device));
  Operator *op;
  DCS(op_with_dfl(field, *quark, &op, nullptr));
  const Dfl &d = *op->dfl;
  *ns = d.ns;
  *nblocks = d.nb;
  DCK(hipDeviceSynchronize());
  if (a) DCK(hipMemcpy(a, d.a.p, (size_t)d.nb * DFL_SLOTS * d.ns * d.ns * sizeof(double2), hipMemcpyDeviceToHost));
  if (nbr) DCK(hipMemcpy(nbr, d.nbr.p, (size_t)d.nb * DFL_SLOTS * sizeof(int), hipMemcpyDeviceToHost));
  return QXD_OK;
}

qxd_status qxd_debug_dfl_stats(qxd_field *field, const qxd_quark *quark, int64_t out[3]) {
  if (!field || !quark || !out) {
    set_error("invalid arguments to qxd_debug_dfl_stats");
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  DCK(hipSetDevice(field->ctx->device));
  Operator *op;
  DCS(op_with_dfl(field, *quark, &op, nullptr));
  Dfl &d = *op->dfl;
  out[0] = d.applications;
  out[1] = d.little_iters;
  out[2] = d.little_max;
  d.applications = d.little_iters = d.little_max = 0;
  return QXD_OK;
}

qxd_status qxd_debug_dfl_precond(qxd_field *field, const qxd_quark *quark, double little_tol, int ncy, int nmr,
                                 const double *in_dev, double *out_dev, void *stream) {
  if (!field || !quark || !in_dev || !out_dev || ncy < 1 || nmr < 0 || little_tol < 0.0 || little_tol >= 1.0) {
    set_error("invalid arguments to qxd_debug_dfl_precond");
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  hipStream_t st = (hipStream_t)stream;
  DCK(hipSetDevice(field->ctx->device));
  Operator *op;
  DCS(op_with_dfl(field, *quark, &op, st));
  void *r32, *o32;
  DCS(ws(field, "dfl_dbg_in", spinor_bytes(QXD_F32, field->g.V), &r32));
  DCS(ws(field, "dfl_dbg_out", spinor_bytes(QXD_F32, field->g.V), &o32));
  DCK(launch_pack(QXD_F32, field->g, in_dev, r32, 1, st));
  DCS(dfl_precond(field, *op, little_tol, ncy, nmr, r32, o32, st));
  DCK(launch_unpack(QXD_F32, field->g, o32, out_dev, 1, st));
  DCK(hipStreamSynchronize(st));
  return QXD_OK;
}

}  // extern "C"
