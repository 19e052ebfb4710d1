// The C ABI of libqxd (include/qxd.h): argument checks, gauge-field upload,
// operator cache, Dirac-operator application and layout conversion.  Solvers
// live in solver.cpp and the serving scheduler in serve.cpp.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/qxd_debug.h"
#include "host.h"
#include "batch_solver.h"
#include "blas.h"
#include "launch.h"
#include "solver.h"

namespace qxd {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int qhat_of(double q, double q_el, bool *ok) {
  double qh = q / q_el;
  double r = nearbyint(qh);
  *ok = fabs(qh - r) < 1e-9 && fabs(r) < 1e6;
  return (int)r;
}

// Validate the lattice (Sec. 2.1 geometry) and fill the device geometry.
static qxd_status make_geom(const qxd_lattice *lat, Geom *g) {
  if (!lat) {
    set_error("lattice is NULL");
    return QXD_EINVAL;
  }
  if (lat->cstar < 0 || lat->cstar > 3) {
    set_error("cstar must be 0..3 (got %d)", lat->cstar);
    return QXD_EINVAL;
  }
  if (lat->time_bc < 0 || lat->time_bc > 3) {
    set_error("time_bc must be 0 (antiperiodic), 1 (open), 2 (SF) or 3 (open-SF)");
    return QXD_EINVAL;
  }
  if (!isfinite(lat->cF) || !isfinite(lat->cF_prime)) {
    set_error("cF and cF_prime must be finite");
    return QXD_EINVAL;
  }
  int N[4] = {lat->dims[0], lat->cstar ? 2 * lat->dims[1] : lat->dims[1], lat->dims[2], lat->dims[3]};
  int64_t V = 1;
  for (int m = 0; m < 4; m++) {
    if (lat->dims[m] < 2 || lat->dims[m] % 2) {
      set_error("lattice extent %d of direction %d must be even and >= 2", lat->dims[m], m);
      return QXD_EINVAL;
    }
    int b = lat->block[m] ? lat->block[m] : 4;
    if (b < 2 || b % 2 || N[m] % b) {
      set_error("block extent %d must be even and divide the extended extent %d (direction %d)", b, N[m], m);
      return QXD_EINVAL;
    }
    g->N[m] = N[m];
    g->b[m] = b;
    g->nb[m] = N[m] / b;
    V *= N[m];
  }
  // fields are addressed with 32-bit byte offsets: the largest array (36
  // FP64 pairs per site) must stay below 4 GiB
  if (V * 36 * 16 >= ((int64_t)1 << 32)) {
    set_error("extended volume %lld exceeds the %lld sites addressable with 32-bit offsets", (long long)V,
              (long long)((((int64_t)1 << 32) - 1) / (36 * 16)));
    return QXD_EINVAL;
  }
  g->L1 = lat->dims[1];
  if (lat->cstar && g->L1 % g->b[1]) {
    set_error("under C* the block extent in direction 1 must divide L1");
    return QXD_EINVAL;
  }
  g->L1b = g->L1 / g->b[1];
  g->shift_mask = 0;
  for (int k = 2; k <= lat->cstar; k++) g->shift_mask |= 1 << k;
  g->time_bc = lat->time_bc;
  g->V = (int)V;
  g->Vh = (int)(V / 2);
  g->Vb = g->b[0] * g->b[1] * g->b[2] * g->b[3];
  g->Vbh = g->Vb / 2;
  g->hb3 = g->b[3] / 2;
  g->nblocks = g->nb[0] * g->nb[1] * g->nb[2] * g->nb[3];
  for (int m = 0; m < 4; m++)
    if (g->b[m] > 255 || g->nb[m] > 255) {
      set_error("at most 255 blocks and block sites per direction");
      return QXD_EINVAL;
    }
  finish_geom(*g);
  return QXD_OK;
}

void *Field::workspace(const std::string &name, size_t bytes, hipError_t *err) {
  auto &slot = work[name];
  if (!slot) slot.reset(new DevBuf());
  *err = slot->ensure(bytes);
  return *err == hipSuccess ? slot->p : nullptr;
}

qxd_status Field::ensure_links(int prec, hipStream_t st) {
  if (links_ready[prec]) return QXD_OK;
  int64_t n_pairs = (int64_t)36 * g.V;
  QXD_HIP_CHECK(links[prec].ensure(n_pairs * pair_bytes(prec)));
  QXD_HIP_CHECK(launch_convert_field(prec, g, 36, g.V, links[QXD_F64].as<double2>(), links[prec].p, st));
  QXD_HIP_CHECK(angles[prec].ensure((size_t)4 * g.V * sizeof(float)));
  QXD_HIP_CHECK(launch_convert_reals(angles[QXD_F64].as<double>(), angles[prec].as<float>(), (int64_t)4 * g.V, st));
  links_ready[prec] = true;
  return QXD_OK;
}

size_t Field::op_bytes(int prec) const {
  // Pauli term (all sites), its odd-site inverse and the folded links, in FP64
  // and (if different) in precision prec
  size_t b = (size_t)36 * (2 * g.V + g.Vh) * 16;
  if (prec != QXD_F64) b += (size_t)36 * (2 * g.V + g.Vh) * pair_bytes(prec);
  return b;
}

Field::OpKey Field::op_key(const qxd_quark &q) const {
  return OpKey{q.kappa, has_u1 ? q.q : 0.0, q.csw, has_u1 ? q.csw_u1 : 0.0,
               q.theta[0], q.theta[1], q.theta[2], q.theta[3]};
}

size_t Field::pending_op_bytes(const qxd_quark *quarks, int n, int prec) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  size_t b = 0;
  std::vector<OpKey> seen;
  for (int k = 0; k < n; k++) {
    const qxd_quark &q = quarks[k];
    const OpKey key = op_key(q);
    if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
    seen.push_back(key);
    auto it = ops.find(key);
    if (it == ops.end())
      b += op_bytes(prec);
    else if (!it->second->ready[prec])
      b += (size_t)36 * (2 * g.V + g.Vh) * pair_bytes(prec);
  }
  return b;
}

// Quark parameters that the lattice admits: finite values, kappa > 0, theta
// only in periodic directions (not C*, not open time).
static qxd_status check_quark(const Field &f, const qxd_quark &q) {
  bool fin = isfinite(q.kappa) && isfinite(q.csw) && isfinite(q.csw_u1) && isfinite(q.q) && isfinite(q.mu);
  for (int m = 0; m < 4; m++) fin = fin && isfinite(q.theta[m]);
  if (!fin || !(q.kappa > 0.0)) {
    set_error("quark parameters must be finite with kappa > 0");
    return QXD_EINVAL;
  }
  for (int m = 0; m < 4; m++) {
    if (q.theta[m] == 0.0) continue;
    const bool cstar_dir = m >= 1 && m <= f.lat.cstar;
    if (cstar_dir || (m == 0 && f.lat.time_bc != 0)) {
      set_error("theta[%d] must be 0: direction %d has %s boundaries", m, m, cstar_dir ? "C*" : "open");
      return QXD_EINVAL;
    }
  }
  return QXD_OK;
}

size_t Field::pending_op_bytes_nowait(const qxd_quark &q, int prec) {
  if (!mu.try_lock()) return op_bytes(prec);
  size_t b = pending_op_bytes(&q, 1, prec);
  mu.unlock();
  return b;
}

qxd_status Field::get_op(const qxd_quark &q, int prec, Operator **out, hipStream_t st) {
  {
    qxd_status cs = check_quark(*this, q);
    if (cs != QXD_OK) return cs;
  }
  int qhat = 0;
  if (has_u1) {
    bool ok;
    qhat = qhat_of(q.q, q_el, &ok);
    if (!ok) {
      set_error("charge q = %g is not an integer multiple of q_el = %g", q.q, q_el);
      return QXD_EINVAL;
    }
  }
  const OpKey key = op_key(q);
  auto it = ops.find(key);
  Operator *op;
  if (it == ops.end()) {
    // bounded cache: drop the least recently used operators no solver slot
    // holds (freeing device memory synchronises the device, so no queued
    // kernel still reads them)
    while (ops.size() >= kMaxCachedOps) {
      auto victim = ops.end();
      for (auto jt = ops.begin(); jt != ops.end(); ++jt)
        if (jt->second->users == 0 && (victim == ops.end() || jt->second->last_use < victim->second->last_use))
          victim = jt;
      if (victim == ops.end()) break;
      op_mem -= victim->second->bytes;
      ops.erase(victim);
    }
    std::unique_ptr<Operator> nop(new Operator());
    nop->quark = q;
    nop->qhat = qhat;
    QXD_HIP_CHECK(nop->pauli[QXD_F64].ensure((size_t)36 * g.V * 16));
    QXD_HIP_CHECK(nop->pinv[QXD_F64].ensure((size_t)36 * g.Vh * 16));
    QXD_HIP_CHECK(launch_pauli_build(g, links[QXD_F64].as<double2>(), angles[QXD_F64].as<double>(), has_u1,
                                     q.kappa, q.csw, has_u1 ? qhat * q.csw_u1 : 0.0,
                                     lat.cF == 0.0 ? 1.0 : lat.cF, lat.cF_prime == 0.0 ? 1.0 : lat.cF_prime,
                                     nop->pauli[QXD_F64].as<double2>(), st));
    hipError_t e;
    int *bad = (int *)workspace("bad_count", sizeof(int), &e);
    QXD_HIP_CHECK(e);
    QXD_HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(int), st));
    QXD_HIP_CHECK(launch_pauli_invert(g, nop->pauli[QXD_F64].as<double2>(), nop->pinv[QXD_F64].as<double2>(), bad, st));
    int nbad = 0;
    QXD_HIP_CHECK(hipMemcpyAsync(&nbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    QXD_HIP_CHECK(hipStreamSynchronize(st));
    if (nbad) {
      set_error("%d odd-site Pauli blocks are not positive definite (kappa=%g, csw=%g)", nbad, q.kappa, q.csw);
      return QXD_EFLOAT;
    }
    QXD_HIP_CHECK(nop->wl[QXD_F64].ensure((size_t)36 * g.V * 16));
    QXD_HIP_CHECK(launch_fold_phase(g, links[QXD_F64].as<double2>(), angles[QXD_F64].as<double>(), qhat,
                                    q.theta, nop->wl[QXD_F64].as<double2>(), st));
    nop->ready[QXD_F64] = true;
    nop->bytes = (size_t)36 * (2 * g.V + g.Vh) * 16;
    op_mem += nop->bytes;
    op = nop.get();
    ops[key] = std::move(nop);
  } else {
    op = it->second.get();
  }
  if (!op->ready[prec]) {
    QXD_HIP_CHECK(op->pauli[prec].ensure((size_t)36 * g.V * pair_bytes(prec)));
    QXD_HIP_CHECK(op->pinv[prec].ensure((size_t)36 * g.Vh * pair_bytes(prec)));
    QXD_HIP_CHECK(launch_convert_field(prec, g, 36, g.V, op->pauli[QXD_F64].as<double2>(), op->pauli[prec].p, st));
    QXD_HIP_CHECK(launch_convert_field(prec, g, 36, g.Vh, op->pinv[QXD_F64].as<double2>(), op->pinv[prec].p, st));
    QXD_HIP_CHECK(op->wl[prec].ensure((size_t)36 * g.V * pair_bytes(prec)));
    QXD_HIP_CHECK(launch_convert_field(prec, g, 36, g.V, op->wl[QXD_F64].as<double2>(), op->wl[prec].p, st));
    op->ready[prec] = true;
    const size_t nb = (size_t)36 * (2 * g.V + g.Vh) * pair_bytes(prec);
    op->bytes += nb;
    op_mem += nb;
  }
  qxd_status s = ensure_links(prec, st);
  if (s != QXD_OK) return s;
  op->last_use = ++op_clock;
  *out = op;
  return QXD_OK;
}

Operator *Field::find_op(const qxd_quark &q, int prec) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  if (!links_ready[prec]) return nullptr;
  auto it = ops.find(op_key(q));
  if (it == ops.end() || !it->second->ready[prec]) return nullptr;
  return it->second.get();
}

OpFields Field::op_fields(const Operator &op, int prec) const {
  OpFields f;
  f.links = op.wl[prec].p;
  f.angles = nullptr;
  f.pauli = op.pauli[prec].p;
  f.pinv = op.pinv[prec].p;
  f.qhat = 0;
  return f;
}

OpFields Field::op_fields_u(const Operator &op, int prec) const {
  OpFields f;
  f.links = links[prec].p;
  f.angles = angles[prec].p;
  f.pauli = op.pauli[prec].p;
  f.pinv = op.pinv[prec].p;
  f.qhat = op.qhat;
  return f;
}

// out_e = (D^ + i mu gamma5) in_e on the even half of full-lattice native
// spinors (odd half of out untouched); tmp: an odd-half spinor.
hipError_t schur_tm(Field *fd, const OpFields &f, int prec, double mu, SpinorArg in, SpinorArg out, void *tmp,
                    hipStream_t st, bool may_tune) {
  const Geom &g = fd->g;
  SpinorArg t_o{tmp, g.Vh, g.Vh, g.rd}, none{nullptr, 0, 0, g.rd};
  hipError_t e = launch_dirac(prec, DK_ODD, g, f, in, none, t_o, -0.5, st, may_tune);
  if (e == hipSuccess) e = launch_dirac(prec, DK_EVEN, g, f, t_o, in, out, 0.5, st, may_tune);
  if (e == hipSuccess && mu != 0.0)
    e = launch_lincomb_sites(prec, out, out, 1.0, 0.0, false, in, 0.0, mu, true, 0, g.Vh, st);
  return e;
}

// Apply `op` to one native spinor (full-lattice buffers).
qxd_status apply_native(Field *fd, const Operator &op, double mu, qxd_op which, int prec, void *in, void *out,
                        hipStream_t st, void *dhat_tmp, bool may_tune) {
  const Geom &g = fd->g;
  OpFields f = fd->op_fields(op, prec);
  SpinorArg full_in{in, g.V, 0, g.rd}, full_out{out, g.V, 0, g.rd}, none{nullptr, 0, 0, g.rd};
  const bool mt = may_tune;
  switch (which) {
    case QXD_OP_D:
      QXD_HIP_CHECK(launch_dirac(prec, DK_FULL, g, f, full_in, full_in, full_out, -0.5, st, mt));
      break;
    case QXD_OP_HOP:
      QXD_HIP_CHECK(launch_dirac(prec, DK_HOP, g, f, full_in, none, full_out, -0.5, st, mt));
      break;
    case QXD_OP_PAULI:
      QXD_HIP_CHECK(launch_dirac(prec, DK_PAULI, g, f, full_in, full_in, full_out, 0.0, st, mt));
      break;
    case QXD_OP_DHAT: {
      void *tmp = dhat_tmp;
      if (!tmp) {
        hipError_t e;
        tmp = fd->workspace("dhat_tmp", spinor_bytes(prec, g.Vh), &e);
        QXD_HIP_CHECK(e);
      }
      QXD_HIP_CHECK(schur_tm(fd, f, prec, mu, full_in, full_out, tmp, st, mt));
      QXD_HIP_CHECK(launch_zero_sites(prec, full_out, g.Vh, g.Vh, st));
      break;
    }
    case QXD_OP_DHAT_DAG:
    case QXD_OP_NORMAL: {
      hipError_t e;
      void *tmp = fd->workspace("dhat_tmp", spinor_bytes(prec, g.Vh), &e);
      QXD_HIP_CHECK(e);
      void *t2 = fd->workspace("normal_tmp", spinor_bytes(prec, g.V), &e);
      QXD_HIP_CHECK(e);
      SpinorArg full_t2{t2, g.V, 0, g.rd};
      const double m = mu;
      SpinorArg src = full_in;
      if (which == QXD_OP_NORMAL) {  // t2 = (D^ + i mu g5) in
        QXD_HIP_CHECK(schur_tm(fd, f, prec, m, full_in, full_t2, tmp, st, mt));
        src = full_t2;
      }
      // (D^ + i mu g5)^dag src = g5 (D^ - i mu g5) g5 src: out = g5 src,
      // out = (D^ - i mu g5) out through t2, out = g5 out
      QXD_HIP_CHECK(launch_lincomb_sites(prec, full_out, src, 1.0, 0.0, true, none, 0, 0, false, 0, g.Vh, st));
      QXD_HIP_CHECK(schur_tm(fd, f, prec, -m, full_out, full_t2, tmp, st, mt));
      QXD_HIP_CHECK(launch_lincomb_sites(prec, full_out, full_t2, 1.0, 0.0, true, none, 0, 0, false, 0, g.Vh, st));
      QXD_HIP_CHECK(launch_zero_sites(prec, full_out, g.Vh, g.Vh, st));
      break;
    }
    case QXD_OP_OOINV:
      QXD_HIP_CHECK(launch_dirac(prec, DK_ODD, g, f, full_in, full_in, full_out, 0.0, st, mt));
      QXD_HIP_CHECK(launch_zero_sites(prec, full_out, 0, g.Vh, st));
      break;
    case QXD_OP_G5D:
      QXD_HIP_CHECK(launch_dirac(prec, DK_FULL, g, f, full_in, full_in, full_out, -0.5, st, mt));
      QXD_HIP_CHECK(launch_g5_sites(prec, full_out, 0, g.V, st));
      break;
    default:
      set_error("unknown operator %d", (int)which);
      return QXD_EINVAL;
  }
  return QXD_OK;
}

// ---------------------------------------------------------------------------
// Scratch memory of the allocation-free entry point (qxd_dirac_apply_noalloc):
// one buffer per GPU, part of the library's code object, so the runtime
// creates it when the code is loaded on a device and it lives until the
// process ends.  Host code never passes `scratch` itself to a kernel (in host
// code the name is only a stand-in for the symbol): qxd_init resolves the
// device address of each GPU's copy once, with that GPU current, and every
// later use goes through that address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[QXD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Resolve this device's copy of the scratch array (the device is current).
static qxd_status init_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device %d beyond the %d devices the library supports", device, kMaxDevices);
    return QXD_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return QXD_OK;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    set_error("cannot resolve the scratch buffer of device %d: %s", device, hipGetErrorString(e));
    return QXD_EDEVICE;
  }
  g_scratch_ptr[device] = ptr;
  return QXD_OK;
}

static void *scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace qxd

using namespace qxd;

static bool valid_prec(int p) { return p >= QXD_F64 && p <= QXD_BF16; }

extern "C" {

int qxd_abi_version(void) { return QXD_ABI_VERSION; }

qxd_status qxd_debug_get_dirac_variant(const qxd_field *field, qxd_prec prec, int *choice) {
  if (!field || !choice || prec < QXD_F64 || prec > QXD_BF16) {
    set_error("field and choice must be non-NULL and prec valid");
    return QXD_EINVAL;
  }
  *choice = tuned_group((int)prec, (int)DK_FULL, field->g.V, 0);
  return QXD_OK;
}

qxd_status qxd_debug_set_step_graphs(int enable) {
  set_step_graphs(enable != 0);
  return QXD_OK;
}

qxd_status qxd_debug_set_gs_passes(int passes) {
  if (passes != 1 && passes != 2) {
    set_error("qxd_debug_set_gs_passes: passes must be 1 or 2");
    return QXD_EINVAL;
  }
  set_gs_passes(passes);
  return QXD_OK;
}

qxd_status qxd_debug_sap_pair_pass(qxd_field *field, const qxd_quark *quark, qxd_prec prec, int nmr, int npair,
                                   int reps, float *ms, void *stream) {
  if (!field || !quark || !ms || nmr < 0 || npair < 1 || reps < 1) {
    set_error("invalid arguments to qxd_debug_sap_pair_pass");
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  QXD_HIP_CHECK(hipSetDevice(field->ctx->device));
  return debug_sap_pair_pass(field, *quark, (int)prec, nmr, npair, reps, ms, (hipStream_t)stream);
}

qxd_status qxd_debug_fail_steps(int n) {
  if (n < 0) {
    set_error("n must be >= 0");
    return QXD_EINVAL;
  }
  inject_step_failures(n);
  return QXD_OK;
}

qxd_status qxd_debug_step_graph_counts(int64_t *captures, int64_t *replays) {
  if (!captures || !replays) {
    set_error("captures and replays must be non-NULL");
    return QXD_EINVAL;
  }
  step_graph_counts(captures, replays);
  return QXD_OK;
}

qxd_status qxd_debug_stream(const void *src_dev, void *dst_dev, size_t dst_bytes, int reads_per_write,
                            void *stream) {
  const int r = reads_per_write;
  if (!src_dev || !dst_dev || (((uintptr_t)src_dev | (uintptr_t)dst_dev) & 15) || dst_bytes % 49152 ||
      !(r == 1 || r == 2 || (r >= 4 && r <= 8))) {
    set_error("stream probe needs non-NULL 16-byte-aligned buffers, a multiple of 49152 bytes and "
              "reads_per_write in {1, 2, 4, 5, 6, 7, 8}");
    return QXD_EINVAL;
  }
  QXD_HIP_CHECK(launch_stream(src_dev, dst_dev, dst_bytes, r, (hipStream_t)stream));
  return QXD_OK;
}

qxd_status qxd_debug_set_dirac_variant(int choice) {
  if (!force_dirac_variant(choice)) {
    set_error("invalid Dirac kernel variant %d", choice);
    return QXD_EINVAL;
  }
  return QXD_OK;
}

const char *qxd_last_error(void) { return g_err; }

qxd_status qxd_init(int device, qxd_ctx **ctx) {
  if (!ctx) {
    set_error("ctx is NULL");
    return QXD_EINVAL;
  }
  int n = 0;
  QXD_HIP_CHECK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) {
    set_error("device %d out of range (%d devices)", device, n);
    return QXD_EINVAL;
  }
  QXD_HIP_CHECK(hipSetDevice(device));
  qxd_status ss = init_scratch(device);
  if (ss != QXD_OK) return ss;
  qxd_ctx *c = new qxd_ctx();
  c->device = device;
  *ctx = c;
  return QXD_OK;
}

qxd_status qxd_finalize(qxd_ctx *ctx) {
  if (!ctx) {
    set_error("ctx is NULL");
    return QXD_EINVAL;
  }
  if (ctx->serve) qxd_serve_stop(ctx);
  if (ctx->n_fields) {
    set_error("%d fields of this context are still alive", ctx->n_fields);
    return QXD_EINVAL;
  }
  delete ctx;
  return QXD_OK;
}

qxd_status qxd_field_upload(qxd_ctx *ctx, const qxd_lattice *lat, const double *U_host,
                            const double *A_host, qxd_field **field) {
  if (!ctx || !field || !U_host) {
    set_error("ctx, U_host and field must be non-NULL");
    return QXD_EINVAL;
  }
  Geom g;
  qxd_status s = make_geom(lat, &g);
  if (s != QXD_OK) return s;
  double q_el = lat->q_el == 0.0 ? 1.0 / 6.0 : lat->q_el;
  if (!(q_el > 0.0) || !isfinite(q_el)) {
    set_error("q_el must be positive");
    return QXD_EINVAL;
  }
  QXD_HIP_CHECK(hipSetDevice(ctx->device));
  std::unique_ptr<qxd_field> f(new qxd_field());
  f->ctx = ctx;
  f->lat = *lat;
  f->g = g;
  f->q_el = q_el;
  f->has_u1 = A_host != nullptr;
  int64_t vph = (int64_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  DevBuf u_st, a_st;
  QXD_HIP_CHECK(u_st.ensure(vph * 4 * 18 * sizeof(double)));
  QXD_HIP_CHECK(hipMemcpy(u_st.p, U_host, vph * 4 * 18 * sizeof(double), hipMemcpyHostToDevice));
  if (A_host) {
    QXD_HIP_CHECK(a_st.ensure(vph * 4 * sizeof(double)));
    QXD_HIP_CHECK(hipMemcpy(a_st.p, A_host, vph * 4 * sizeof(double), hipMemcpyHostToDevice));
  }
  QXD_HIP_CHECK(f->links[QXD_F64].ensure((size_t)36 * g.V * 16));
  QXD_HIP_CHECK(f->angles[QXD_F64].ensure((size_t)4 * g.V * 8));
  QXD_HIP_CHECK(launch_orbifold(g, u_st.as<double>(), a_st.as<double>(), f->links[QXD_F64].as<double2>(),
                                f->angles[QXD_F64].as<double>(), 0));
  QXD_HIP_CHECK(hipDeviceSynchronize());
  f->links_ready[QXD_F64] = true;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->n_fields++;
  }
  *field = f.release();
  return QXD_OK;
}

qxd_status qxd_field_release(qxd_field *field) {
  if (!field) {
    set_error("field is NULL");
    return QXD_EINVAL;
  }
  qxd_ctx *ctx = field->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  delete field;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->n_fields--;
  return QXD_OK;
}

qxd_status qxd_field_volume(const qxd_field *field, int64_t *v_ext) {
  if (!field || !v_ext) {
    set_error("field and v_ext must be non-NULL");
    return QXD_EINVAL;
  }
  *v_ext = field->g.V;
  return QXD_OK;
}

qxd_status qxd_spinor_bytes(const qxd_field *field, qxd_prec prec, size_t *bytes) {
  if (!field || !bytes || !valid_prec(prec)) {
    set_error("invalid arguments to qxd_spinor_bytes");
    return QXD_EINVAL;
  }
  *bytes = field->spinor_bytes(prec);
  return QXD_OK;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

qxd_status qxd_spinor_pack(qxd_field *field, qxd_prec prec, const double *in_dev, void *out_dev,
                           int nrhs, void *stream) {
  if (!field || !in_dev || !out_dev || nrhs < 1 || !valid_prec(prec)) {
    set_error("invalid arguments to qxd_spinor_pack");
    return QXD_EINVAL;
  }
  if (!aligned16(out_dev)) {
    set_error("native spinors must be 16-byte aligned");
    return QXD_EINVAL;
  }
  QXD_HIP_CHECK(hipSetDevice(field->ctx->device));
  QXD_HIP_CHECK(launch_pack(prec, field->g, in_dev, out_dev, nrhs, (hipStream_t)stream));
  return QXD_OK;
}

qxd_status qxd_spinor_unpack(qxd_field *field, qxd_prec prec, const void *in_dev, double *out_dev,
                             int nrhs, void *stream) {
  if (!field || !in_dev || !out_dev || nrhs < 1 || !valid_prec(prec)) {
    set_error("invalid arguments to qxd_spinor_unpack");
    return QXD_EINVAL;
  }
  if (!aligned16(in_dev)) {
    set_error("native spinors must be 16-byte aligned");
    return QXD_EINVAL;
  }
  QXD_HIP_CHECK(hipSetDevice(field->ctx->device));
  QXD_HIP_CHECK(launch_unpack(prec, field->g, in_dev, out_dev, nrhs, (hipStream_t)stream));
  return QXD_OK;
}

qxd_status qxd_dirac_apply(qxd_field *field, const qxd_quark *quarks, int nquark, qxd_op op,
                           qxd_prec prec, const void *in_dev, void *out_dev, int nrhs, unsigned flags,
                           void *stream) {
  if (!field || !quarks || !in_dev || !out_dev || nquark < 1 || nrhs < 1 || nrhs % nquark ||
      !valid_prec(prec) || op < QXD_OP_D || op > QXD_OP_NORMAL || (flags & ~QXD_NATIVE)) {
    set_error("invalid arguments to qxd_dirac_apply");
    return QXD_EINVAL;
  }
  if (in_dev == out_dev) {
    set_error("in and out must not overlap");
    return QXD_EINVAL;
  }
  if ((flags & QXD_NATIVE) && (!aligned16(in_dev) || !aligned16(out_dev))) {
    set_error("native spinors must be 16-byte aligned");
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  hipStream_t st = (hipStream_t)stream;
  QXD_HIP_CHECK(hipSetDevice(field->ctx->device));
  size_t nb = field->spinor_bytes(prec);
  const bool native = flags & QXD_NATIVE;
  void *nin = nullptr, *nout = nullptr;
  if (!native) {
    hipError_t e;
    nin = field->workspace("apply_in", nb, &e);
    QXD_HIP_CHECK(e);
    nout = field->workspace("apply_out", nb, &e);
    QXD_HIP_CHECK(e);
  }
  int per = nrhs / nquark;
  for (int r = 0; r < nrhs; r++) {
    Operator *o;
    qxd_status s = field->get_op(quarks[r / per], prec, &o, st);
    if (s != QXD_OK) return s;
    if (native) {
      s = apply_native(field, *o, quarks[r / per].mu, op, prec, (char *)in_dev + r * nb, (char *)out_dev + r * nb,
                       st);
    } else {
      const double *src = (const double *)in_dev + (int64_t)r * 24 * field->g.V;
      double *dst = (double *)out_dev + (int64_t)r * 24 * field->g.V;
      QXD_HIP_CHECK(launch_pack(prec, field->g, src, nin, 1, st));
      s = apply_native(field, *o, quarks[r / per].mu, op, prec, nin, nout, st);
      if (s == QXD_OK) QXD_HIP_CHECK(launch_unpack(prec, field->g, nout, dst, 1, st));
    }
    if (s != QXD_OK) return s;
  }
  return QXD_OK;
}

static size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

qxd_status qxd_dirac_apply_noalloc(qxd_field *field, const qxd_quark *quarks, int nquark, qxd_op op,
                                   qxd_prec prec, const void *in_dev, void *out_dev, int nrhs, unsigned flags,
                                   void *stream) {
  if (!field || !quarks || !in_dev || !out_dev || nquark < 1 || nrhs < 1 || nrhs % nquark ||
      !valid_prec(prec) || op < QXD_OP_D || op > QXD_OP_G5D || (flags & ~QXD_NATIVE)) {
    set_error("invalid arguments to qxd_dirac_apply_noalloc");
    return QXD_EINVAL;
  }
  if (in_dev == out_dev) {
    set_error("in and out must not overlap");
    return QXD_EINVAL;
  }
  const bool native = flags & QXD_NATIVE;
  if (native && (!aligned16(in_dev) || !aligned16(out_dev))) {
    set_error("native spinors must be 16-byte aligned");
    return QXD_EINVAL;
  }
  const Geom &g = field->g;
  const size_t nb = field->spinor_bytes(prec);
  // scratch layout: [API staging in | API staging out] [odd-site temporary of D^]
  const size_t stage = native ? 0 : 2 * align256(nb);
  const size_t need = stage + (op == QXD_OP_DHAT ? spinor_bytes(prec, g.Vh) : 0);
  if (need > QXD_NOALLOC_SCRATCH_BYTES) {
    set_error("qxd_dirac_apply_noalloc needs %zu bytes of scratch on this lattice, more than the %zu it has",
              need, (size_t)QXD_NOALLOC_SCRATCH_BYTES);
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  const int device = field->ctx->device;
  char *ptr = (char *)scratch_of(device);
  if (!ptr) {
    set_error("the scratch buffer of device %d is not resolved (no qxd_init on it)", device);
    return QXD_EDEVICE;
  }
  // every operator must exist already: building one allocates
  const int per = nrhs / nquark;
  for (int k = 0; k < nquark; k++)
    if (!field->find_op(quarks[k], prec)) {
      set_error("the operator of quark %d (kappa %g, q %g) is not built in precision %d on this field; "
                "apply it once with qxd_dirac_apply first",
                k, quarks[k].kappa, quarks[k].q, (int)prec);
      return QXD_EINVAL;
    }
  hipStream_t st = (hipStream_t)stream;
  QXD_HIP_CHECK(hipSetDevice(device));
  void *nin = ptr, *nout = ptr + align256(nb);
  void *tmp = op == QXD_OP_DHAT ? ptr + stage : nullptr;
  for (int r = 0; r < nrhs; r++) {
    Operator *o = field->find_op(quarks[r / per], prec);
    qxd_status s;
    if (native) {
      s = apply_native(field, *o, quarks[r / per].mu, op, prec, (char *)const_cast<void *>(in_dev) + r * nb,
                       (char *)out_dev + r * nb, st, tmp, false);
    } else {
      const double *src = (const double *)in_dev + (int64_t)r * 24 * g.V;
      double *dst = (double *)out_dev + (int64_t)r * 24 * g.V;
      QXD_HIP_CHECK(launch_pack(prec, g, src, nin, 1, st));
      s = apply_native(field, *o, quarks[r / per].mu, op, prec, nin, nout, st, tmp, false);
      if (s == QXD_OK) QXD_HIP_CHECK(launch_unpack(prec, g, nout, dst, 1, st));
    }
    if (s != QXD_OK) return s;
  }
  return QXD_OK;
}

qxd_status qxd_solve(qxd_field *field, const qxd_quark *quarks, int nquark, const qxd_solver *s,
                     const double *eta_dev, double *psi_dev, int nrhs, int use_guess,
                     qxd_solve_info *info, void *stream) {
  if (!field || !quarks || !s || !eta_dev || !psi_dev || nquark < 1 || nrhs < 1 || nrhs % nquark) {
    set_error("invalid arguments to qxd_solve");
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  QXD_HIP_CHECK(hipSetDevice(field->ctx->device));
  return solve(field, quarks, nquark, *s, eta_dev, psi_dev, nrhs, use_guess, info, (hipStream_t)stream);
}

qxd_status qxd_multishift_solve(qxd_field *field, const qxd_quark *quark, const double *shifts, int nshift,
                                double tol, int maxiter, const double *eta_dev, double *psi_dev,
                                qxd_solve_info *info, void *stream) {
  if (!field || !quark || !shifts || !eta_dev || !psi_dev || nshift < 1 || nshift > 64 || !(tol > 0.0) ||
      tol >= 1.0 || maxiter < 0) {
    set_error("invalid arguments to qxd_multishift_solve");
    return QXD_EINVAL;
  }
  for (int j = 0; j < nshift; j++)
    if (!(shifts[j] >= 0.0) || !isfinite(shifts[j])) {
      set_error("shift %d must be finite and >= 0", j);
      return QXD_EINVAL;
    }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  QXD_HIP_CHECK(hipSetDevice(field->ctx->device));
  return multishift_solve(field, *quark, shifts, nshift, tol, maxiter, eta_dev, psi_dev, info,
                          (hipStream_t)stream);
}

qxd_status qxd_rational_apply(qxd_field *field, const qxd_quark *quark, double A, const double *nu,
                              const double *mu, int n, double tol, int maxiter, const double *eta_dev,
                              double *out_dev, qxd_solve_info *info, void *stream) {
  if (!field || !quark || !nu || !mu || !eta_dev || !out_dev || n < 1 || n > 64 || !isfinite(A) ||
      !(tol > 0.0) || tol >= 1.0 || maxiter < 0) {
    set_error("invalid arguments to qxd_rational_apply");
    return QXD_EINVAL;
  }
  for (int j = 0; j < n; j++)
    if (!isfinite(nu[j]) || !isfinite(mu[j])) {
      set_error("zeros and poles must be finite");
      return QXD_EINVAL;
    }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  QXD_HIP_CHECK(hipSetDevice(field->ctx->device));
  return rational_apply(field, *quark, A, nu, mu, n, tol, maxiter, eta_dev, out_dev, info, (hipStream_t)stream);
}

qxd_status qxd_sap_apply(qxd_field *field, const qxd_quark *quark, qxd_prec prec, int ncy, int nmr,
                         const double *in_dev, double *out_dev, int nrhs, void *stream) {
  if (!field || !quark || !in_dev || !out_dev || nrhs < 1 || ncy < 1 || nmr < 0 || !valid_prec(prec)) {
    set_error("invalid arguments to qxd_sap_apply");
    return QXD_EINVAL;
  }
  std::lock_guard<std::recursive_mutex> lk(field->mu);
  hipStream_t st = (hipStream_t)stream;
  QXD_HIP_CHECK(hipSetDevice(field->ctx->device));
  qxd_status s = check_sap_blocks(field);
  if (s != QXD_OK) return s;
  Operator *o;
  s = field->get_op(*quark, prec, &o, st);
  if (s != QXD_OK) return s;
  size_t nb = field->spinor_bytes(prec);
  hipError_t e;
  void *nin = field->workspace("precond_in", nb, &e);
  QXD_HIP_CHECK(e);
  void *nout = field->workspace("precond_out", nb, &e);
  QXD_HIP_CHECK(e);
  for (int r = 0; r < nrhs; r++) {
    QXD_HIP_CHECK(launch_pack(prec, field->g, in_dev + (int64_t)r * 24 * field->g.V, nin, 1, st));
    s = sap_apply(field, *o, prec, ncy, nmr, nin, nout, st);
    if (s != QXD_OK) return s;
    QXD_HIP_CHECK(launch_unpack(prec, field->g, nout, out_dev + (int64_t)r * 24 * field->g.V, 1, st));
  }
  return QXD_OK;
}

}  // extern "C"
