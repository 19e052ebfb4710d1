// Batched SAP-GCR (see batch_solver.h).  Per right-hand side the iteration is
// the flexible GCR of the defect-correction inner solve:
//   phi_k = M_SAP rho_k,  chi_k = D phi_k,
//   chi_k -= sum_l a_lk chi_l  with a_lk = (chi_l, chi_k) / |chi_l|^2,
//   c_k = (chi_k, rho_k) / |chi_k|^2,  rho_{k+1} = rho_k - c_k chi_k,
// and at the end of a cycle the triangular system R beta = c (R_lk = a_lk,
// R_kk = 1) gives delta += sum beta_k phi_k.  The outer loop is
// x += |r| delta, r = eta - D x in FP64 until |r| <= tol |eta|.
#include "batch_solver.h"

#include <math.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <tuple>
#include <vector>

#include "batch.h"
#include "blas.h"
#include "sap.h"
#include "solver.h"

namespace qxd {

// Gram-Schmidt passes of batch solvers constructed from now on (1 or 2)
std::atomic<int> g_gs_passes{1};

namespace {
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
}  // namespace

#define BCK(...)                                                                       \
  do {                                                                                 \
    hipError_t _e = (__VA_ARGS__);                                                     \
    if (_e != hipSuccess) {                                                            \
      set_error("HIP error %s at %s:%d", hipGetErrorString(_e), __FILE__, __LINE__);  \
      return _e == hipErrorOutOfMemory ? QXD_ENOMEM : QXD_EDEVICE;                     \
    }                                                                                  \
  } while (0)
#define BCS(...)                         \
  do {                                   \
    qxd_status _s = (__VA_ARGS__);       \
    if (_s != QXD_OK) return _s;         \
  } while (0)

struct BatchSolver::Slot {
  bool active = false;
  void *tag = nullptr;
  const double *eta_api = nullptr;
  double *psi_api = nullptr;
  qxd_quark q{};
  Operator *op64 = nullptr, *opP = nullptr;
  DevBuf f64, inner, scal;
  size_t fb64 = 0, fbP = 0;
  int k = 0, inner_it = 0, total_it = 0, outer = 0;
  double eta_n = 0, s_norm = 0, bn = 0, r2 = 0;
  double t0 = 0;
  // FP64 vectors
  void *eta() { return f64.p; }
  void *x() { return (char *)f64.p + fb64; }
  void *r() { return (char *)f64.p + 2 * fb64; }
  void *tmp() { return (char *)f64.p + 3 * fb64; }
  // inner-precision vectors
  void *b() { return inner.p; }
  void *rho() { return (char *)inner.p + fbP; }
  void *delta() { return (char *)inner.p + 2 * fbP; }
  void *sap_r() { return (char *)inner.p + 3 * fbP; }
  void *sap_v() { return (char *)inner.p + 4 * fbP; }
  void *phi(int k) { return (char *)inner.p + (5 + k) * fbP; }
  void *chi(int nkv, int k) { return (char *)inner.p + (5 + nkv + k) * fbP; }
  // scalars: amat[2*nkv*nkv], rec[3*nkv], coef[2*nkv], misc[8], ak2[2*nkv]
  double *amat() { return (double *)scal.p; }
  double *rec(int nkv) { return amat() + 2 * nkv * nkv; }
  double *coef(int nkv) { return rec(nkv) + 3 * nkv; }
  double *misc(int nkv) { return coef(nkv) + 2 * nkv; }
  double *ak2(int nkv) { return misc(nkv) + 8; }
};

static size_t scal_doubles(int nkv) { return (size_t)2 * nkv * nkv + 3 * nkv + 2 * nkv + 8 + 2 * nkv; }

BatchSolver::BatchSolver(Field *f, int prec, const qxd_solver &s, hipStream_t st)
    : f_(f), prec_(prec), s_(s), st_(st) {
  nkv_ = s.nkv > 0 ? s.nkv : kDefaultNkv;
  if (nkv_ > MAXV) nkv_ = MAXV;
  ncy_ = s.ncy > 0 ? s.ncy : kDefaultNcy;
  nmr_ = s.nmr > 0 ? s.nmr : kDefaultNmr;
  inner_tol_ = s.inner_tol > 0 ? s.inner_tol : kDefaultInnerTol[prec >= QXD_F64 && prec <= QXD_BF16 ? prec : 0];
  gs_passes_ = g_gs_passes.load();
}

BatchSolver::~BatchSolver() {
  (void)hipStreamSynchronize(st_);
  {
    std::lock_guard<std::recursive_mutex> lk(f_->mu);
    for (auto &s : slots_) release_ops(*s);
  }
  drop_graphs();
  if (cap_st_) (void)hipStreamDestroy(cap_st_);
  if (h_stage_) (void)hipHostFree(h_stage_);
  if (h_norms_) (void)hipHostFree(h_norms_);
}

size_t BatchSolver::slot_bytes(const Field *f, int prec, const qxd_solver &s) {
  int nkv = s.nkv > 0 ? s.nkv : kDefaultNkv;
  if (nkv > MAXV) nkv = MAXV;
  return 4 * spinor_bytes(QXD_F64, f->g.V) + (size_t)(5 + 2 * nkv) * spinor_bytes(prec, f->g.V) +
         scal_doubles(nkv) * 8;
}

int BatchSolver::active() const {
  int n = 0;
  for (auto &s : slots_) n += s->active;
  return n;
}

qxd_status BatchSolver::reserve(int n) {
  const Geom &g = f_->g;
  while ((int)slots_.size() < n) {
    std::unique_ptr<Slot> sl(new Slot());
    sl->fb64 = spinor_bytes(QXD_F64, g.V);
    sl->fbP = spinor_bytes(prec_, g.V);
    BCK(sl->f64.ensure(4 * sl->fb64));
    BCK(sl->inner.ensure((5 + 2 * nkv_) * sl->fbP));
    BCK(sl->scal.ensure(scal_doubles(nkv_) * 8));
    slots_.push_back(std::move(sl));
  }
  size_t nslot = slots_.size();
  size_t stage =
      nslot * (sizeof(SapSlot<QXD_F64>) + sizeof(DSlot<QXD_F64>) + 2 * sizeof(int) + sizeof(GsSlot<QXD_F64>)) + 256;
  if (stage > h_stage_bytes_) {
    BCK(hipStreamSynchronize(st_));
    if (h_stage_) (void)hipHostFree(h_stage_);
    h_stage_ = nullptr;
    BCK(hipHostMalloc(&h_stage_, stage, hipHostMallocDefault));
    h_stage_bytes_ = stage;
    if (h_norms_) (void)hipHostFree(h_norms_);
    h_norms_ = nullptr;
    BCK(hipHostMalloc((void **)&h_norms_, nslot * sizeof(double) + 64, hipHostMallocDefault));
  }
  const void *old[5] = {dslots_.p, sslots_.p, act_.p, gsslots_.p, gspart_.p};
  BCK(dslots_.ensure(nslot * sizeof(DSlot<QXD_F64>)));
  BCK(sslots_.ensure(nslot * sizeof(SapSlot<QXD_F64>)));
  BCK(act_.ensure(2 * nslot * sizeof(int)));
  BCK(gsslots_.ensure(nslot * sizeof(GsSlot<QXD_F64>)));
  BCK(gspart_.ensure(gs_batch_partial_doubles((int)nslot, prec_, g.V) * 8));
  // graphs name the tables by address: none survives a reallocation
  if (old[0] != dslots_.p || old[1] != sslots_.p || old[2] != act_.p || old[3] != gsslots_.p ||
      old[4] != gspart_.p)
    drop_graphs();
  BCK(d_norms_.ensure(nslot * sizeof(double)));
  BCK(partial_.ensure(blas_partial_doubles() * 8));
  return QXD_OK;
}

// ---------------------------------------------------------------------------
// per-precision pieces
// ---------------------------------------------------------------------------
template <int P>
struct BImpl {
  static SpinorArg F(const Geom &g, void *p) { return SpinorArg{p, g.V, 0, g.rd}; }

  // b = r / |r| (inner precision), rho = b, delta = 0
  static qxd_status new_inner(BatchSolver::Slot &sl, const Geom &g, double *partial, int nkv,
                              hipStream_t st) {
    sl.s_norm = sqrt(sl.r2);
    BCK(blas_axpby<P, QXD_F64>(F(g, sl.b()), 0.0, F(g, sl.r()), 1.0 / sl.s_norm, 0, g.V, partial,
                               sl.misc(nkv) + 1, st));
    BCK(blas_axpby<P, P>(F(g, sl.rho()), 0.0, F(g, sl.b()), 1.0, 0, g.V, partial, nullptr, st));
    BCK(hipMemsetAsync(sl.delta(), 0, sl.fbP, st));
    double b2 = 0;
    BCK(hipMemcpyAsync(&b2, sl.misc(nkv) + 1, 8, hipMemcpyDeviceToHost, st));
    BCK(hipStreamSynchronize(st));
    sl.bn = sqrt(b2);
    sl.r2 = b2;
    sl.k = 0;
    sl.inner_it = 0;
    return QXD_OK;
  }

  // end of a cycle: delta += sum beta_k phi_k (kused = sl.k vectors)
  static qxd_status cycle_end(BatchSolver::Slot &sl, const Geom &g, double *partial, int nkv,
                              hipStream_t st) {
    int kused = sl.k;
    if (kused == 0) return QXD_OK;
    std::vector<double> hv(2 * nkv * nkv + 3 * nkv);
    BCK(hipMemcpyAsync(hv.data(), sl.amat(), hv.size() * 8, hipMemcpyDeviceToHost, st));
    BCK(hipStreamSynchronize(st));
    const double *rec = hv.data() + 2 * nkv * nkv;
    std::vector<double> br(kused), bi(kused), hc(2 * kused);
    for (int k = kused - 1; k >= 0; k--) {
      double n = rec[3 * k];
      double cr = rec[3 * k + 1] / n, ci = rec[3 * k + 2] / n;
      for (int j = k + 1; j < kused; j++) {
        double ar = hv[2 * (j * nkv + k)], ai = hv[2 * (j * nkv + k) + 1];
        cr -= ar * br[j] - ai * bi[j];
        ci -= ar * bi[j] + ai * br[j];
      }
      br[k] = cr;
      bi[k] = ci;
    }
    for (int k = 0; k < kused; k++) {
      hc[2 * k] = -br[k];
      hc[2 * k + 1] = -bi[k];
    }
    BCK(hipMemcpyAsync(sl.coef(nkv), hc.data(), hc.size() * 8, hipMemcpyHostToDevice, st));
    std::vector<SpinorArg> phi(kused);
    for (int l = 0; l < kused; l++) phi[l] = F(g, sl.phi(l));
    MaxpyHost m;
    m.n = kused;
    m.src[0] = F(g, sl.delta());
    m.dst[0] = F(g, sl.delta());
    m.ys[0] = phi.data();
    m.coef = sl.coef(nkv);
    BCK(blas_maxpy<P>(m, 0, g.V, partial, nullptr, st));
    BCK(hipStreamSynchronize(st));  // hc lives on this stack frame
    return QXD_OK;
  }

  // rho = b - D delta (restart inside the inner solve)
  static qxd_status restart(BatchSolver::Slot &sl, Field *f, double *partial, int nkv, hipStream_t st) {
    const Geom &g = f->g;
    OpFields of = f->op_fields(*sl.opP, P);
    BCK(launch_dirac(P, DK_FULL, g, of, F(g, sl.delta()), F(g, sl.delta()), F(g, sl.chi(nkv, 0)), -0.5, st));
    BCK(blas_axpby<P, P>(F(g, sl.rho()), 0.0, F(g, sl.b()), 1.0, 0, g.V, partial, nullptr, st));
    BCK(blas_axpby<P, P>(F(g, sl.rho()), 1.0, F(g, sl.chi(nkv, 0)), -1.0, 0, g.V, partial, sl.misc(nkv), st));
    BCK(hipMemcpyAsync(&sl.r2, sl.misc(nkv), 8, hipMemcpyDeviceToHost, st));
    BCK(hipStreamSynchronize(st));
    sl.k = 0;
    return QXD_OK;
  }

  // x += |r| delta; r = eta - D x (FP64); r2 = |r|^2
  static qxd_status outer_update(BatchSolver::Slot &sl, Field *f, double *partial, int nkv, hipStream_t st) {
    const Geom &g = f->g;
    auto F64 = [&](void *p) { return SpinorArg{p, g.V, 0, g.rd}; };
    BCK(blas_axpby<QXD_F64, P>(F64(sl.x()), 1.0, F(g, sl.delta()), sl.s_norm, 0, g.V, partial, nullptr, st));
    OpFields of = f->op_fields(*sl.op64, QXD_F64);
    BCK(launch_dirac(QXD_F64, DK_FULL, g, of, F64(sl.x()), F64(sl.x()), F64(sl.tmp()), -0.5, st));
    BCK(blas_axpby<QXD_F64, QXD_F64>(F64(sl.r()), 0.0, F64(sl.eta()), 1.0, 0, g.V, partial, nullptr, st));
    BCK(blas_axpby<QXD_F64, QXD_F64>(F64(sl.r()), 1.0, F64(sl.tmp()), -1.0, 0, g.V, partial, sl.misc(nkv), st));
    BCK(hipMemcpyAsync(&sl.r2, sl.misc(nkv), 8, hipMemcpyDeviceToHost, st));
    BCK(hipStreamSynchronize(st));
    return QXD_OK;
  }

  // the batched part of a step: phi_k = M_SAP rho, chi_k = D phi_k
  static qxd_status batched(BatchSolver &bs, std::vector<BatchSolver::Slot *> &act, hipStream_t st,
                            DevBuf &sslots, DevBuf &dslots, DevBuf &actbuf, DevBuf &gsslots, DevBuf &gspart,
                            double *norms, void *stage, int ncy, int nmr, int nkv) {
    Field *f = bs.field();
    const Geom &g = f->g;
    int n = (int)act.size();
    SapSlot<P> *hs = (SapSlot<P> *)stage;
    DSlot<P> *hd = (DSlot<P> *)(hs + n);
    int *ha = (int *)(hd + n);
    for (int j = 0; j < n; j++) {
      BatchSolver::Slot &sl = *act[j];
      OpFields of = f->op_fields(*sl.opP, P);
      hs[j].op = SapOp<P>{(const typename St<P>::pair_t *)of.links, nullptr, 0,
                          (const typename St<P>::pair_t *)of.pauli, (const typename St<P>::pair_t *)of.pinv};
      hs[j].vec = SapVecs<P>{spinor_view<P>(sl.rho(), g.V, 0, g), spinor_view<P>(sl.sap_r(), g.V, 0, g),
                             spinor_view<P>(sl.phi(sl.k), g.V, 0, g), spinor_view<P>(sl.sap_v(), g.V, 0, g)};
      hd[j].links = hs[j].op.links;
      hd[j].pauli = hs[j].op.pauli;
      hd[j].in = spinor_view<P>(sl.phi(sl.k), g.V, 0, g);
      hd[j].out = spinor_view<P>(sl.chi(nkv, sl.k), g.V, 0, g);
      ha[j] = j;
    }
    // pair up right-hand sides with the same operator (two per work-group in
    // the block solver); the rest go one per work-group.  ha: [0, n) for the
    // Dirac launch, then the single slots, then the pairs.
    int *hsingle = ha + n, nsingle = 0, npair = 0;
    std::vector<int> order(n);
    for (int j = 0; j < n; j++) order[j] = j;
    const bool pairs_ok = P != QXD_F64 && sap_quad_pairs_ok(P, g);
    if (pairs_ok)
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return std::make_tuple(hs[x].op.links, hs[x].op.pauli) < std::make_tuple(hs[y].op.links, hs[y].op.pauli);
      });
    std::vector<int> pairs;
    for (int k = 0; k < n;) {
      if (pairs_ok && k + 1 < n && hs[order[k]].op.links == hs[order[k + 1]].op.links &&
          hs[order[k]].op.pauli == hs[order[k + 1]].op.pauli && hs[order[k]].op.pinv == hs[order[k + 1]].op.pinv) {
        pairs.push_back(order[k]);
        pairs.push_back(order[k + 1]);
        k += 2;
      } else {
        hsingle[nsingle++] = order[k++];
      }
    }
    npair = (int)pairs.size() / 2;
    int *hpair = hsingle + nsingle;
    for (size_t k = 0; k < pairs.size(); k++) hpair[k] = pairs[k];
    BCK(hipMemcpyAsync(sslots.p, hs, n * sizeof(SapSlot<P>), hipMemcpyHostToDevice, st));
    BCK(hipMemcpyAsync(dslots.p, hd, n * sizeof(DSlot<P>), hipMemcpyHostToDevice, st));
    BCK(hipMemcpyAsync(actbuf.p, ha, 2 * n * sizeof(int), hipMemcpyHostToDevice, st));
    // Gram-Schmidt table (chi_k = D phi_k is orthogonalised in the same step)
    GsSlot<P> *hg = (GsSlot<P> *)(((uintptr_t)(ha + 2 * n) + 15) & ~(uintptr_t)15);
    for (int j = 0; j < n; j++) {
      BatchSolver::Slot &sl = *act[j];
      hg[j].chi0 = (typename St<P>::pair_t *)sl.chi(nkv, 0);
      hg[j].vstride_bytes = (int64_t)sl.fbP;
      hg[j].rho = (typename St<P>::pair_t *)sl.rho();
      hg[j].ak = sl.amat() + 2 * sl.k * nkv;
      hg[j].ak2 = sl.ak2(nkv);
      hg[j].rec = sl.rec(nkv);
      hg[j].norm = norms + j;
      hg[j].k = sl.k;
    }
    BCK(hipMemcpyAsync(gsslots.p, hg, n * sizeof(GsSlot<P>), hipMemcpyHostToDevice, st));
    const int *dsingle = actbuf.as<int>() + n, *dpair = dsingle + nsingle;
    const int *lists[2];
    int nper;
    BCS(sap_block_lists(f, lists, &nper));
    auto issue = [&](hipStream_t st) -> qxd_status {
      for (int cy = 0; cy < ncy; cy++)
        for (int c = 0; c < 2; c++) {
          if constexpr (P != QXD_F64) {
            if (npair > 0)
              BCK(launch_sapq_pairs<P>(g, lists[c], nper, sslots.as<SapSlot<P>>(), dpair, npair, cy == 0,
                                       cy == 0 && c == 0, nmr, st));
          }
          if (nsingle > 0)
            BCK(launch_sap_batch<P>(g, lists[c], nper, sslots.as<SapSlot<P>>(), dsingle, nsingle, cy == 0,
                                    cy == 0 && c == 0, nmr, st));
        }
      BCK(launch_dirac_batch<P>(g, dslots.as<DSlot<P>>(), actbuf.as<int>(), n, 2, st));
      BCK(blas_gs_batch<P>(gsslots.as<GsSlot<P>>(), n, g.V, g.rd, gspart.as<double>(), bs.gs_passes(), st));
      return QXD_OK;
    };
    const std::array<int64_t, 10> key{P, n, npair, (int64_t)ncy * 256 + nmr, (int64_t)(intptr_t)sslots.p,
                                      (int64_t)(intptr_t)dslots.p, (int64_t)(intptr_t)actbuf.p, nper,
                                      (int64_t)(intptr_t)gsslots.p, (int64_t)(intptr_t)gspart.p};
    // FP64 inner solves (not a performance path) launch directly
    if constexpr (P == QXD_F64) return issue(st);
    return bs.run_step_launches(key, issue);
    return QXD_OK;
  }
};

std::atomic<bool> g_step_graphs{true};
std::atomic<int> g_inject_failures{0};
std::atomic<int64_t> g_graph_captures{0}, g_graph_replays{0};

#define DISPATCH(call)                                          \
  switch (prec_) {                                              \
    case QXD_F64: return BImpl<QXD_F64>::call;                  \
    case QXD_F32: return BImpl<QXD_F32>::call;                  \
    case QXD_F16S: return BImpl<QXD_F16S>::call;                \
    default: return BImpl<QXD_BF16>::call;                      \
  }

void set_step_graphs(bool on) { g_step_graphs.store(on); }
void set_gs_passes(int passes) { g_gs_passes.store(passes); }
void inject_step_failures(int n) { g_inject_failures.store(n > 0 ? n : 0); }
void step_graph_counts(int64_t *captures, int64_t *replays) {
  *captures = g_graph_captures.load();
  *replays = g_graph_replays.load();
}

void BatchSolver::drop_graphs() {
  if (!graphs_.empty()) (void)hipStreamSynchronize(st_);
  for (auto &ge : graphs_) (void)hipGraphExecDestroy(ge.second);
  graphs_.clear();
  seen_.clear();
}

qxd_status BatchSolver::run_step_launches(const StepKey &key,
                                          const std::function<qxd_status(hipStream_t)> &issue) {
  constexpr size_t MAX_GRAPHS = 16, MAX_SEEN = 64;
  if (!graphs_ok_ || !g_step_graphs.load()) return issue(st_);
  for (size_t k = 0; k < graphs_.size(); k++)
    if (graphs_[k].first == key) {
      std::rotate(graphs_.begin() + k, graphs_.begin() + k + 1, graphs_.end());
      BCK(hipGraphLaunch(graphs_.back().second, st_));
      g_graph_replays.fetch_add(1);
      return QXD_OK;
    }
  if (std::find(seen_.begin(), seen_.end(), key) == seen_.end()) {
    // first sight of this configuration: run eagerly (also sets up kernel
    // attributes outside any capture); capture when it comes again
    if (seen_.size() == MAX_SEEN) seen_.erase(seen_.begin());
    seen_.push_back(key);
    return issue(st_);
  }
  if (!cap_st_ && hipStreamCreateWithFlags(&cap_st_, hipStreamNonBlocking) != hipSuccess) {
    cap_st_ = nullptr;
    graphs_ok_ = false;
    return issue(st_);
  }
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(cap_st_, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    graphs_ok_ = false;
    return issue(st_);
  }
  qxd_status s = issue(cap_st_);
  hipError_t e = hipStreamEndCapture(cap_st_, &graph);
  if (s != QXD_OK || e != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    graphs_ok_ = false;
    return issue(st_);  // nothing ran during the failed capture
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    graphs_ok_ = false;
    return issue(st_);
  }
  if (graphs_.size() == MAX_GRAPHS) {
    // the least recently used graph may still be queued on st_
    BCK(hipStreamSynchronize(st_));
    (void)hipGraphExecDestroy(graphs_.front().second);
    graphs_.erase(graphs_.begin());
  }
  graphs_.emplace_back(key, exec);
  g_graph_captures.fetch_add(1);
  BCK(hipGraphLaunch(exec, st_));
  g_graph_replays.fetch_add(1);
  return QXD_OK;
}

qxd_status BatchSolver::new_inner(Slot &sl) {
  DISPATCH(new_inner(sl, f_->g, partial_.as<double>(), nkv_, st_));
}
qxd_status BatchSolver::cycle_end(Slot &sl) {
  DISPATCH(cycle_end(sl, f_->g, partial_.as<double>(), nkv_, st_));
}
qxd_status BatchSolver::outer_update(Slot &sl) {
  DISPATCH(outer_update(sl, f_, partial_.as<double>(), nkv_, st_));
}

qxd_status BatchSolver::finish(Slot &sl, int status) {
  const Geom &g = f_->g;
  BCK(launch_unpack(QXD_F64, g, sl.x(), sl.psi_api, 1, st_));
  BCK(hipStreamSynchronize(st_));
  Finished fin;
  fin.slot = -1;
  fin.tag = sl.tag;
  fin.info.status = status;
  fin.info.outer_iters = sl.outer;
  fin.info.inner_iters = sl.total_it;
  fin.info.true_resid = sl.eta_n > 0 ? sqrt(sl.r2) / sl.eta_n : 0.0;
  fin.info.seconds = now_s() - sl.t0;
  for (size_t j = 0; j < slots_.size(); j++)
    if (slots_[j].get() == &sl) fin.slot = (int)j;
  done_.push_back(fin);
  sl.active = false;
  release_ops(sl);
  return QXD_OK;
}

void BatchSolver::release_ops(Slot &sl) {
  if (sl.op64) sl.op64->users--;
  if (sl.opP && sl.opP != sl.op64) sl.opP->users--;
  sl.op64 = sl.opP = nullptr;
}

qxd_status BatchSolver::release_slots() {
  if (active() != 0) {
    set_error("release_slots with right-hand sides in flight");
    return QXD_EBUSY;
  }
  BCK(hipStreamSynchronize(st_));
  slots_.clear();
  return QXD_OK;
}

qxd_status BatchSolver::add(const qxd_quark &q, const double *eta_api, double *psi_api, bool use_guess,
                            void *tag) {
  Slot *sl = nullptr;
  for (auto &s : slots_)
    if (!s->active) {
      sl = s.get();
      break;
    }
  if (!sl) {
    set_error("no free slot in the batch");
    return QXD_EBUSY;
  }
  const Geom &g = f_->g;
  BCS(f_->get_op(q, QXD_F64, &sl->op64, st_));
  sl->op64->users++;  // held until finish(): the operator cache keeps it
  qxd_status so = f_->get_op(q, prec_, &sl->opP, st_);
  if (so != QXD_OK) {
    release_ops(*sl);
    return so;
  }
  if (sl->opP != sl->op64) sl->opP->users++;
  sl->q = q;
  sl->tag = tag;
  sl->eta_api = eta_api;
  sl->psi_api = psi_api;
  sl->k = sl->inner_it = sl->total_it = sl->outer = 0;
  sl->t0 = now_s();
  sl->active = true;
  double *partial = partial_.as<double>();
  auto F64 = [&](void *p) { return SpinorArg{p, g.V, 0, g.rd}; };
  BCK(launch_pack(QXD_F64, g, eta_api, sl->eta(), 1, st_));
  BCK(blas_norm2<QXD_F64>(F64(sl->eta()), 0, g.V, partial, sl->misc(nkv_), st_));
  double e2 = 0;
  BCK(hipMemcpyAsync(&e2, sl->misc(nkv_), 8, hipMemcpyDeviceToHost, st_));
  BCK(hipStreamSynchronize(st_));
  if (!isfinite(e2)) {
    sl->eta_n = 0;
    sl->r2 = 0;
    BCK(hipMemsetAsync(sl->x(), 0, sl->fb64, st_));
    return finish(*sl, QXD_EFLOAT);
  }
  sl->eta_n = sqrt(e2);
  if (e2 == 0.0) {
    sl->r2 = 0;
    BCK(hipMemsetAsync(sl->x(), 0, sl->fb64, st_));
    return finish(*sl, QXD_OK);
  }
  if (use_guess) {
    BCK(launch_pack(QXD_F64, g, psi_api, sl->x(), 1, st_));
    OpFields of = f_->op_fields(*sl->op64, QXD_F64);
    BCK(launch_dirac(QXD_F64, DK_FULL, g, of, F64(sl->x()), F64(sl->x()), F64(sl->tmp()), -0.5, st_));
    BCK(blas_axpby<QXD_F64, QXD_F64>(F64(sl->r()), 0.0, F64(sl->eta()), 1.0, 0, g.V, partial, nullptr, st_));
    BCK(blas_axpby<QXD_F64, QXD_F64>(F64(sl->r()), 1.0, F64(sl->tmp()), -1.0, 0, g.V, partial, sl->misc(nkv_), st_));
    BCK(hipMemcpyAsync(&sl->r2, sl->misc(nkv_), 8, hipMemcpyDeviceToHost, st_));
    BCK(hipStreamSynchronize(st_));
    if (!isfinite(sl->r2)) return finish(*sl, QXD_EFLOAT);
  } else {
    BCK(hipMemsetAsync(sl->x(), 0, sl->fb64, st_));
    BCK(blas_axpby<QXD_F64, QXD_F64>(F64(sl->r()), 0.0, F64(sl->eta()), 1.0, 0, g.V, partial, nullptr, st_));
    sl->r2 = e2;
  }
  if (sqrt(sl->r2) <= s_.tol * sl->eta_n) return finish(*sl, QXD_OK);
  return new_inner(*sl);
}

void BatchSolver::abort_all(int status) {
  for (size_t j = 0; j < slots_.size(); j++) {
    Slot &sl = *slots_[j];
    if (!sl.active) continue;
    Finished fin;
    fin.slot = (int)j;
    fin.tag = sl.tag;
    fin.info.status = status;
    fin.info.outer_iters = sl.outer;
    fin.info.inner_iters = sl.total_it;
    fin.info.true_resid = INFINITY;
    fin.info.seconds = now_s() - sl.t0;
    done_.push_back(fin);
    sl.active = false;
    release_ops(sl);
  }
}

qxd_status BatchSolver::step() {
  std::vector<Slot *> act;
  for (auto &s : slots_)
    if (s->active) act.push_back(s.get());
  if (act.empty()) return QXD_OK;
  for (int left = g_inject_failures.load(); left > 0;)
    if (g_inject_failures.compare_exchange_weak(left, left - 1)) {
      set_error("injected failure of a batched solver step (testing hook)");
      return QXD_EDEVICE;
    }
  const Geom &g = f_->g;
  int n = (int)act.size();
  // batched: phi_k = M_SAP rho, chi_k = D phi_k
  switch (prec_) {
    case QXD_F64: BCS(BImpl<QXD_F64>::batched(*this, act, st_, sslots_, dslots_, act_, gsslots_, gspart_, d_norms_.as<double>(), h_stage_, ncy_, nmr_, nkv_)); break;
    case QXD_F32: BCS(BImpl<QXD_F32>::batched(*this, act, st_, sslots_, dslots_, act_, gsslots_, gspart_, d_norms_.as<double>(), h_stage_, ncy_, nmr_, nkv_)); break;
    case QXD_F16S: BCS(BImpl<QXD_F16S>::batched(*this, act, st_, sslots_, dslots_, act_, gsslots_, gspart_, d_norms_.as<double>(), h_stage_, ncy_, nmr_, nkv_)); break;
    default: BCS(BImpl<QXD_BF16>::batched(*this, act, st_, sslots_, dslots_, act_, gsslots_, gspart_, d_norms_.as<double>(), h_stage_, ncy_, nmr_, nkv_)); break;
  }
  // the batched Gram-Schmidt of the step left |rho|^2 of right-hand side j in
  // d_norms_[j]
  double *dn = d_norms_.as<double>();
  BCK(hipMemcpyAsync(h_norms_, dn, n * sizeof(double), hipMemcpyDeviceToHost, st_));
  BCK(hipStreamSynchronize(st_));
  const int maxiter = s_.maxiter > 0 ? s_.maxiter : 100000;
  const int max_outer = s_.max_outer > 0 ? s_.max_outer : 50;
  for (int j = 0; j < n; j++) {
    Slot &sl = *act[j];
    sl.r2 = h_norms_[j];
    sl.k++;
    sl.inner_it++;
    sl.total_it++;
    if (!isfinite(sl.r2)) {
      BCS(finish(sl, QXD_EFLOAT));
      continue;
    }
    bool inner_done = sqrt(sl.r2) <= inner_tol_ * sl.bn;
    bool budget = sl.total_it >= maxiter;
    if (!(inner_done || budget || sl.k == nkv_)) continue;
    BCS(cycle_end(sl));
    // an inner solve that has not converged after kMaxInnerCycles cycles is
    // cut short: the FP64 correction restarts it from the true residual
    constexpr int kMaxInnerCycles = 16;
    if (inner_done || budget || sl.inner_it >= kMaxInnerCycles * nkv_) {
      BCS(outer_update(sl));
      sl.outer++;
      if (!isfinite(sl.r2)) {
        BCS(finish(sl, QXD_EFLOAT));
      } else if (sqrt(sl.r2) <= s_.tol * sl.eta_n) {
        BCS(finish(sl, QXD_OK));
      } else if (budget || sl.outer >= max_outer) {
        BCS(finish(sl, QXD_ENOCONV));
      } else {
        BCS(new_inner(sl));
      }
    } else {
      switch (prec_) {
        case QXD_F64: BCS(BImpl<QXD_F64>::restart(sl, f_, partial_.as<double>(), nkv_, st_)); break;
        case QXD_F32: BCS(BImpl<QXD_F32>::restart(sl, f_, partial_.as<double>(), nkv_, st_)); break;
        case QXD_F16S: BCS(BImpl<QXD_F16S>::restart(sl, f_, partial_.as<double>(), nkv_, st_)); break;
        default: BCS(BImpl<QXD_BF16>::restart(sl, f_, partial_.as<double>(), nkv_, st_)); break;
      }
    }
  }
  return QXD_OK;
}

std::vector<Finished> BatchSolver::take_finished() {
  std::vector<Finished> out;
  out.swap(done_);
  return out;
}

}  // namespace qxd
