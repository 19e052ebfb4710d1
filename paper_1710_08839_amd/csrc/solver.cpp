// Solvers for D psi = eta (qxd_solve): the plain even-odd GCR in FP64 and the
// SAP-preconditioned flexible GCR with FP64 outer defect correction.
//
// The paper names these solvers (abstract, Sec. 2) without printing their
// steps; the steps follow the standard Schwarz-preconditioned GCR:
//   * EO_GCR: restarted GCR on D^ psi_e = eta^_e with eta^_e = eta_e -
//     D_eo D_oo^-1 eta_o, then psi_o = D_oo^-1 (eta_o - D_oe psi_e) (Sec. 2.4).
//   * SAP_GCR: x += s * delta with s = |r|, r = eta - D x in FP64, where delta
//     solves D delta = r / s approximately by flexible GCR in the inner
//     precision, right-preconditioned by ncy cycles of the Schwarz alternating
//     procedure (block solves by nmr minimal-residual steps on the even-odd
//     block operator).
// Gram-Schmidt coefficients and norms are FP64 and stay on the device; the host
// reads one residual norm per iteration.
#include <math.h>

#include <chrono>
#include <vector>

#include <algorithm>

#include "batch_solver.h"
#include "blas.h"
#include "dfl.h"
#include "sap.h"
#include "solver.h"

namespace qxd {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Ws {
  Field *f;
  hipStream_t st;
  qxd_status err = QXD_OK;
  void *get(const std::string &name, size_t bytes) {
    hipError_t e;
    void *p = f->workspace(name, bytes, &e);
    if (e != hipSuccess) {
      set_error("workspace allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
      err = QXD_ENOMEM;
    }
    return p;
  }
};

#define CK(...)                                                                       \
  do {                                                                                 \
    hipError_t _e = (__VA_ARGS__);                                                          \
    if (_e != hipSuccess) {                                                            \
      set_error("HIP error %s at %s:%d", hipGetErrorString(_e), __FILE__, __LINE__);  \
      return QXD_EDEVICE;                                                              \
    }                                                                                  \
  } while (0)
#define CS(...)                         \
  do {                                   \
    qxd_status _s = (__VA_ARGS__);            \
    if (_s != QXD_OK) return _s;         \
  } while (0)

// read `n` doubles from device (synchronises the stream)
qxd_status fetch(double *host, const double *dev, int n, hipStream_t st) {
  CK(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  return QXD_OK;
}

// ---------------------------------------------------------------------------
// D^ on even-half FP64 vectors
// ---------------------------------------------------------------------------
struct Schur {
  Field *f;
  OpFields of;
  int prec;
  void *tmp;  // odd-half temporary
  qxd_status apply(void *in_e, void *out_e, hipStream_t st) {
    const Geom &g = f->g;
    SpinorArg in{in_e, g.Vh, 0, g.rd}, out{out_e, g.Vh, 0, g.rd}, t{tmp, g.Vh, g.Vh, g.rd}, none{nullptr, 0, 0, g.rd};
    CK(launch_dirac(prec, DK_ODD, g, of, in, none, t, -0.5, st));
    CK(launch_dirac(prec, DK_EVEN, g, of, t, in, out, 0.5, st));
    return QXD_OK;
  }
};

// ---------------------------------------------------------------------------
// plain even-odd GCR, FP64
// ---------------------------------------------------------------------------
qxd_status eo_gcr(Field *f, const Operator &op, const qxd_solver &s, void *eta, void *psi, bool guess,
                  qxd_solve_info *info, hipStream_t st) {
  const Geom &g = f->g;
  const int P = QXD_F64;
  const int nkv = s.nkv > 0 ? s.nkv : 16;
  if (nkv > MAXV) {
    set_error("nkv must be <= %d", MAXV);
    return QXD_EINVAL;
  }
  Ws w{f, st};
  size_t hb = spinor_bytes(P, g.Vh), fb = spinor_bytes(P, g.V);
  char *pv = (char *)w.get("gcr_p", hb * nkv);
  char *qv = (char *)w.get("gcr_q", hb * nkv);
  void *x = w.get("gcr_x", hb), *r = w.get("gcr_r", hb), *b = w.get("gcr_b", hb);
  void *tmp = w.get("gcr_tmp", hb), *full = w.get("gcr_full", fb);
  double *partial = (double *)w.get("partial", blas_partial_doubles() * 8);
  double *scal = (double *)w.get("scalars", (size_t)(2 * MAXV + 3 * MAXV + 16) * 8);
  if (w.err) return w.err;
  double *beta = scal, *rec = scal + 2 * MAXV, *rn2 = rec + 3 * MAXV, *misc = rn2 + 4;
  Schur A{f, f->op_fields(op, P), P, tmp};
  auto H = [&](void *p) { return SpinorArg{p, g.Vh, 0, g.rd}; };
  SpinorArg FULL_eta{eta, g.V, 0}, FULL_psi{psi, g.V, 0}, FULL{full, g.V, 0}, none{nullptr, 0, 0};
  OpFields of = f->op_fields(op, P);

  // |eta|
  CK(blas_norm2<P>(FULL_eta, 0, g.V, partial, misc, st));
  double eta2;
  CS(fetch(&eta2, misc, 1, st));
  if (!isfinite(eta2)) {
    set_error("source contains NaN/Inf");
    return QXD_EFLOAT;
  }
  if (eta2 == 0.0) {
    CK(hipMemsetAsync(psi, 0, fb, st));
    if (info) info->true_resid = 0.0;
    return QXD_OK;
  }
  const double eta_n = sqrt(eta2);
  // b = eta^_e = eta_e + acc(D_oo^-1 eta_o)/2
  SpinorArg t_o{tmp, g.Vh, g.Vh, g.rd};
  CK(launch_dirac(P, DK_ODD, g, of, FULL_eta, FULL_eta, t_o, 0.0, st));
  CK(launch_dirac(P, DK_EVEN_ID, g, of, t_o, FULL_eta, H(b), 0.5, st));
  // x = guess_e or 0; r = b - D^ x
  if (guess) {
    CK(blas_axpby<P, P>(H(x), 0.0, FULL_psi, 1.0, 0, g.Vh, partial, nullptr, st));
    CS(A.apply(x, r, st));
    CK(blas_axpby<P, P>(H(r), -1.0, H(b), 1.0, 0, g.Vh, partial, rn2, st));
  } else {
    CK(hipMemsetAsync(x, 0, hb, st));
    CK(blas_axpby<P, P>(H(r), 0.0, H(b), 1.0, 0, g.Vh, partial, rn2, st));
  }
  double r2;
  CS(fetch(&r2, rn2, 1, st));
  int it = 0;
  const int maxiter = s.maxiter > 0 ? s.maxiter : 100000;
  double target = 0.5 * s.tol * eta_n;
  double true_res = INFINITY;
  std::vector<SpinorArg> ps(nkv), qs(nkv);
  for (int k = 0; k < nkv; k++) {
    ps[k] = H(pv + k * hb);
    qs[k] = H(qv + k * hb);
  }
  for (int refine = 0; refine < 8; refine++) {
    while (sqrt(r2) > target && it < maxiter) {
      for (int k = 0; k < nkv && it < maxiter; k++, it++) {
        // q_k = D^ r; orthogonalise against q_0..q_{k-1} (and p_k = r - sum beta p_l)
        CS(A.apply(r, qs[k].ptr, st));
        if (k > 0) CK(blas_mdot<P>(qs.data(), k, qs[k], 0, g.Vh, partial, beta, rec, 3, st));
        MaxpyHost m;
        m.n = k;
        m.ntriples = 2;
        m.src[0] = qs[k];
        m.dst[0] = qs[k];
        m.ys[0] = qs.data();
        m.src[1] = H(r);
        m.dst[1] = ps[k];
        m.ys[1] = ps.data();
        m.coef = beta;
        m.w = H(r);
        CK(blas_maxpy<P>(m, 0, g.Vh, partial, rec + 3 * k, st));
        // alpha = (q_k, r) / |q_k|^2: x += alpha p_k, r -= alpha q_k
        CK(blas_update<P>(H(x), ps[k], rec + 3 * k + 1, rec + 3 * k, 1, 0, g.Vh, partial, misc, st));
        CK(blas_update<P>(H(r), qs[k], rec + 3 * k + 1, rec + 3 * k, 0, 0, g.Vh, partial, rn2, st));
        CS(fetch(&r2, rn2, 1, st));
        if (!isfinite(r2)) {
          set_error("GCR residual is NaN/Inf");
          return QXD_EFLOAT;
        }
        if (sqrt(r2) <= target) {
          it++;
          break;
        }
      }
      // restart: r = b - D^ x
      CS(A.apply(x, r, st));
      CK(blas_axpby<P, P>(H(r), -1.0, H(b), 1.0, 0, g.Vh, partial, rn2, st));
      CS(fetch(&r2, rn2, 1, st));
    }
    // psi_e = x, psi_o = D_oo^-1 (eta_o + acc(x)/2); true residual in FP64
    CK(blas_axpby<P, P>(SpinorArg{psi, g.V, 0, g.rd}, 0.0, H(x), 1.0, 0, g.Vh, partial, nullptr, st));
    CK(launch_dirac(P, DK_ODD, g, of, H(x), FULL_eta, FULL_psi, 0.5, st));
    CK(launch_dirac(P, DK_FULL, g, of, FULL_psi, FULL_psi, FULL, -0.5, st));
    CK(blas_axpby<P, P>(FULL, -1.0, FULL_eta, 1.0, 0, g.V, partial, misc, st));
    double res2;
    CS(fetch(&res2, misc, 1, st));
    true_res = sqrt(res2) / eta_n;
    if (true_res <= s.tol || it >= maxiter) break;
    target *= 0.25;
  }
  if (info) {
    info->outer_iters = 1;
    info->inner_iters = it;
    info->true_resid = true_res;
  }
  return true_res <= s.tol ? QXD_OK : QXD_ENOCONV;
}

// ---------------------------------------------------------------------------
// SAP preconditioner
// ---------------------------------------------------------------------------
}  // namespace

qxd_status sap_block_lists(Field *f, const int **lists, int *per_colour) {
  const Geom &g = f->g;
  hipError_t e;
  int *d = (int *)f->workspace("sap_blocks", sizeof(int) * g.nblocks, &e);
  if (e != hipSuccess) {
    set_error("workspace allocation failed");
    return QXD_ENOMEM;
  }
  if (!f->work.count("sap_blocks_ready")) {
    std::vector<int> h;
    h.reserve(g.nblocks);
    for (int c = 0; c < 2; c++)
      for (int B0 = 0; B0 < g.nb[0]; B0++)
        for (int B1 = 0; B1 < g.nb[1]; B1++)
          for (int B2 = 0; B2 < g.nb[2]; B2++)
            for (int B3 = 0; B3 < g.nb[3]; B3++)
              if (((B0 + B1 + B2 + B3) & 1) == c) h.push_back(((B0 * g.nb[1] + B1) * g.nb[2] + B2) * g.nb[3] + B3);
    CK(hipMemcpy(d, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice));
    f->work["sap_blocks_ready"].reset(new DevBuf());
  }
  lists[0] = d;
  lists[1] = d + g.nblocks / 2;
  *per_colour = g.nblocks / 2;
  return QXD_OK;
}

namespace {

template <int P>
qxd_status sap_apply_t(Field *f, const Operator &op, int ncy, int nmr, void *rho, void *psi, hipStream_t st) {
  const Geom &g = f->g;
  CS(check_sap_blocks(f));
  const int *lists[2];
  int nper;
  CS(sap_block_lists(f, lists, &nper));
  Ws w{f, st};
  size_t fb = spinor_bytes(P, g.V);
  void *r = w.get("sap_r", fb), *v = w.get("sap_v", fb);
  if (w.err) return w.err;
  OpFields of = f->op_fields(op, P);
  SapArgs<P> a;
  a.g = g;
  a.links = (const typename St<P>::pair_t *)of.links;
  a.angles = (const typename St<P>::real_t *)of.angles;
  a.qhat = of.qhat;
  a.pauli = (const typename St<P>::pair_t *)of.pauli;
  a.pinv = (const typename St<P>::pair_t *)of.pinv;
  a.rho = spinor_view<P>(rho, g.V, 0, g);
  a.r = spinor_view<P>(r, g.V, 0, g);
  a.psi = spinor_view<P>(psi, g.V, 0, g);
  a.v = spinor_view<P>(v, g.V, 0, g);
  a.nmr = nmr;
  for (int cy = 0; cy < ncy; cy++)
    for (int c = 0; c < 2; c++) {
      a.blocks = lists[c];
      a.first = cy == 0;
      a.skip_face = cy == 0 && c == 0;
      CK(launch_sap_colour<P>(a, nper, st));
    }
  return QXD_OK;
}

}  // namespace

namespace {
template <int P>
qxd_status sap_pair_pass_t(Field *f, const Operator &op, int nmr, int npair, int reps, float *ms, hipStream_t st) {
  const Geom &g = f->g;
  if (!sap_quad_pairs_ok(P, g)) {
    set_error("the paired SAP kernel does not run on this lattice");
    return QXD_EINVAL;
  }
  const int *lists[2];
  int nper;
  CS(sap_block_lists(f, lists, &nper));
  const int nslot = 2 * npair;
  const size_t fb = spinor_bytes(P, g.V);
  Ws w{f, st};
  char *vecs = (char *)w.get("sap_probe_vecs", fb * 4 * nslot);
  SapSlot<P> *dslots = (SapSlot<P> *)w.get("sap_probe_slots", sizeof(SapSlot<P>) * nslot);
  int *dpairs = (int *)w.get("sap_probe_pairs", sizeof(int) * nslot);
  if (w.err) return w.err;
  // finite, normal values in every storage format (bytes 0x3c: fp16 1.06,
  // bfloat16 0.011, fp32 0.011; the FP16 site scales read 0.011)
  CK(hipMemsetAsync(vecs, 0x3c, fb * 4 * nslot, st));
  OpFields of = f->op_fields(op, P);
  std::vector<SapSlot<P>> hs(nslot);
  std::vector<int> hp(nslot);
  for (int k = 0; k < nslot; k++) {
    char *v = vecs + (size_t)4 * k * fb;
    hs[k].op = SapOp<P>{(const typename St<P>::pair_t *)of.links, nullptr, 0,
                        (const typename St<P>::pair_t *)of.pauli, (const typename St<P>::pair_t *)of.pinv};
    hs[k].vec = SapVecs<P>{spinor_view<P>(v, g.V, 0, g), spinor_view<P>(v + fb, g.V, 0, g),
                           spinor_view<P>(v + 2 * fb, g.V, 0, g), spinor_view<P>(v + 3 * fb, g.V, 0, g)};
    hp[k] = k;
  }
  CK(hipMemcpyAsync(dslots, hs.data(), sizeof(SapSlot<P>) * nslot, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(dpairs, hp.data(), sizeof(int) * nslot, hipMemcpyHostToDevice, st));
  // one untimed pass, then reps passes of colour 0 with the face update
  CK(launch_sapq_pairs<P>(g, lists[0], nper, dslots, dpairs, npair, 0, 0, nmr, st));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventRecord(e0, st));
  for (int r = 0; r < reps; r++) CK(launch_sapq_pairs<P>(g, lists[0], nper, dslots, dpairs, npair, 0, 0, nmr, st));
  CK(hipEventRecord(e1, st));
  CK(hipEventSynchronize(e1));
  float t = 0;
  CK(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return QXD_OK;
}
}  // namespace

qxd_status debug_sap_pair_pass(Field *f, const qxd_quark &q, int prec, int nmr, int npair, int reps, float *ms,
                               hipStream_t st) {
  CS(check_sap_blocks(f));
  Operator *op;
  CS(f->get_op(q, prec, &op, st));
  switch (prec) {
    case QXD_F32: return sap_pair_pass_t<QXD_F32>(f, *op, nmr, npair, reps, ms, st);
    case QXD_F16S: return sap_pair_pass_t<QXD_F16S>(f, *op, nmr, npair, reps, ms, st);
    case QXD_BF16: return sap_pair_pass_t<QXD_BF16>(f, *op, nmr, npair, reps, ms, st);
  }
  set_error("the paired SAP kernel runs in FP32, FP16+scale and BF16 storage");
  return QXD_EINVAL;
}

qxd_status check_sap_blocks(const Field *f) {
  const Geom &g = f->g;
  for (int m = 0; m < 4; m++)
    if (g.nb[m] < 2 || g.nb[m] % 2) {
      set_error("SAP needs an even number (>= 2) of blocks in every direction (direction %d has %d)", m, g.nb[m]);
      return QXD_EINVAL;
    }
  if (g.Vbh > 256) {
    set_error("SAP blocks may hold at most 512 sites");
    return QXD_EINVAL;
  }
  if (g.shift_mask && (g.L1b % 2)) {
    set_error("with shifted C* boundaries SAP needs L1 / b1 even for a two-colour block decomposition");
    return QXD_EINVAL;
  }
  return QXD_OK;
}

qxd_status sap_apply(Field *f, const Operator &op, int prec, int ncy, int nmr, void *rho, void *psi,
                     hipStream_t st) {
  switch (prec) {
    case QXD_F64: return sap_apply_t<QXD_F64>(f, op, ncy, nmr, rho, psi, st);
    case QXD_F32: return sap_apply_t<QXD_F32>(f, op, ncy, nmr, rho, psi, st);
    case QXD_F16S: return sap_apply_t<QXD_F16S>(f, op, ncy, nmr, rho, psi, st);
    case QXD_BF16: return sap_apply_t<QXD_BF16>(f, op, ncy, nmr, rho, psi, st);
  }
  set_error("invalid precision");
  return QXD_EINVAL;
}

qxd_status solve(Field *f, const qxd_quark *quarks, int nquark, const qxd_solver &s, const double *eta_dev,
                 double *psi_dev, int nrhs, int use_guess, qxd_solve_info *info, hipStream_t st) {
  if (!(s.tol > 0.0) || s.tol >= 1.0 ||
      (s.kind != QXD_SOLVER_EO_GCR && s.kind != QXD_SOLVER_SAP_GCR && s.kind != QXD_SOLVER_DFL_SAP_GCR) ||
      s.inner_prec < QXD_F64 || s.inner_prec > QXD_BF16 || s.nkv < 0 || s.nkv > MAXV || s.ncy < 0 ||
      s.nmr < 0 || s.maxiter < 0 || s.max_outer < 0 || !(s.inner_tol >= 0.0 && s.inner_tol < 1.0)) {
    set_error("invalid solver parameters");
    return QXD_EINVAL;
  }
  const Geom &g = f->g;
  int per = nrhs / nquark;
  qxd_status worst = QXD_OK;
  if (s.kind == QXD_SOLVER_SAP_GCR) {
    CS(check_sap_blocks(f));
    if (2 * g.Vbh > 256) {
      set_error("the batched SAP-GCR needs blocks of at most 128 sites");
      return QXD_EINVAL;
    }
    // every right-hand side gets a slot of the batch while device memory
    // allows; the others join as slots free up (continuous batching).  The
    // operators of the call's quarks are built as their right-hand sides
    // join, so the memory of those not built yet is set aside first (built
    // ones are already out of the free memory).
    size_t freeb = 0, totalb = 0;
    CK(hipMemGetInfo(&freeb, &totalb));
    size_t per_slot = BatchSolver::slot_bytes(f, s.inner_prec, s);
    size_t avail = (size_t)(0.8 * freeb);
    const size_t ops_b = f->pending_op_bytes(quarks, nquark, s.inner_prec);
    avail = avail > ops_b ? avail - ops_b : 0;
    int cap = (int)std::min<size_t>((size_t)nrhs, std::max<size_t>(1, avail / per_slot));
    BatchSolver bs(f, s.inner_prec, s, st);
    CS(bs.reserve(cap));
    int next = 0, finished = 0;
    while (finished < nrhs) {
      while (next < nrhs && bs.free_slots() > 0) {
        const qxd_quark &q = quarks[next / per];
        CS(bs.add(q, eta_dev + (int64_t)next * 24 * g.V, psi_dev + (int64_t)next * 24 * g.V, use_guess,
                  (void *)(intptr_t)next));
        next++;
      }
      qxd_status ss = bs.step();
      if (ss != QXD_OK) {
        // report the right-hand sides still in flight with the error
        bs.abort_all(ss);
        for (auto &fin : bs.take_finished())
          if (info) info[(int)(intptr_t)fin.tag] = fin.info;
        return ss;
      }
      for (auto &fin : bs.take_finished()) {
        int r = (int)(intptr_t)fin.tag;
        if (info) info[r] = fin.info;
        if (fin.info.status != QXD_OK) {
          if (fin.info.status == QXD_EFLOAT || worst == QXD_OK) worst = (qxd_status)fin.info.status;
        }
        finished++;
      }
    }
    return worst;
  }
  if (s.kind == QXD_SOLVER_DFL_SAP_GCR && s.inner_prec != QXD_F32) {
    set_error("the deflated SAP-GCR runs with FP32 inner storage only");
    return QXD_EINVAL;
  }
  Ws w{f, st};
  size_t fb = spinor_bytes(QXD_F64, g.V);
  void *eta = w.get("solve_eta", fb), *psi = w.get("solve_psi", fb);
  if (w.err) return w.err;
  for (int r = 0; r < nrhs; r++) {
    double t0 = now_s();
    const qxd_quark &q = quarks[r / per];
    Operator *op;
    CS(f->get_op(q, QXD_F64, &op, st));
    if (s.kind == QXD_SOLVER_DFL_SAP_GCR) {
      CS(f->get_op(q, QXD_F32, &op, st));
      if (!op->dfl) {
        set_error("no deflation subspace for this quark: call qxd_dfl_setup first");
        return QXD_EINVAL;
      }
    }
    const double *src = eta_dev + (int64_t)r * 24 * g.V;
    double *dst = psi_dev + (int64_t)r * 24 * g.V;
    CK(launch_pack(QXD_F64, g, src, eta, 1, st));
    if (use_guess) CK(launch_pack(QXD_F64, g, dst, psi, 1, st));
    qxd_solve_info inf{};
    qxd_status rs = s.kind == QXD_SOLVER_DFL_SAP_GCR ? dfl_solve(f, *op, s, eta, psi, use_guess, &inf, st)
                                                     : eo_gcr(f, *op, s, eta, psi, use_guess, &inf, st);
    if (rs != QXD_OK && rs != QXD_ENOCONV && rs != QXD_EFLOAT) return rs;
    CK(launch_unpack(QXD_F64, g, psi, dst, 1, st));
    CK(hipStreamSynchronize(st));
    inf.status = rs;
    inf.seconds = now_s() - t0;
    if (info) info[r] = inf;
    if (rs != QXD_OK && (rs == QXD_EFLOAT || worst == QXD_OK)) worst = rs;
  }
  return worst;
}

}  // namespace qxd
