// Host-side objects behind the C ABI: contexts, gauge fields, cached
// operators (Pauli terms per quark), device buffers and error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "launch.h"
#include "qxd_impl.h"

struct qxd_serve;  // serve.cpp

namespace qxd {

void set_error(const char *fmt, ...);

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  // grow to at least `bytes` (contents are not preserved)
  hipError_t ensure(size_t bytes) {
    if (n >= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
    if (e == hipSuccess) n = bytes;
    else p = nullptr;
    return e;
  }
  template <class T> T *as() const { return (T *)p; }
};

struct Dfl;  // deflation subspace of an operator (dfl.h)

// One Dirac operator (one quark flavour) on one gauge field: its Pauli term
// and the inverse odd-site blocks, in FP64 and in each storage precision.
struct Operator {
  qxd_quark quark;         // the quark that built it (its mu is not part of the operator)
  int qhat = 0;
  int users = 0;           // solver slots holding it (guarded by the field's mutex)
  uint64_t last_use = 0;   // for least-recently-used eviction
  size_t bytes = 0;        // device bytes of its fields built so far
  DevBuf pauli[4];   // indexed by qxd_prec
  DevBuf pinv[4];
  DevBuf wl[4];      // hopping links W = U z^qhat with the phase folded in
  bool ready[4] = {false, false, false, false};
  std::shared_ptr<Dfl> dfl;  // local deflation subspace (qxd_dfl_setup), if built
};

struct Field {
  qxd_ctx *ctx = nullptr;
  qxd_lattice lat;
  Geom g;
  bool has_u1 = false;
  double q_el = 1.0 / 6.0;
  DevBuf links[4];   // indexed by qxd_prec (links[F64] is the master copy)
  DevBuf angles[4];  // F64: double, others: float (same buffer for F32/F16S/BF16)
  bool links_ready[4] = {false, false, false, false};
  // operators by (kappa, q, c_sw, c_sw^U(1), theta[4]); at most
  // kMaxCachedOps are kept once unused (a serve stream draws a new kappa per
  // request, and at 64x32^3 one operator holds several GB)
  using OpKey = std::array<double, 8>;
  OpKey op_key(const qxd_quark &q) const;
  std::map<OpKey, std::unique_ptr<Operator>> ops;
  uint64_t op_clock = 0;
  static constexpr size_t kMaxCachedOps = 4;
  // device bytes one operator of this field holds in FP64 plus precision prec
  size_t op_bytes(int prec) const;
  // device bytes still to be allocated for the operators of these quarks
  // (distinct ones, not yet built in FP64 and precision prec)
  size_t pending_op_bytes(const qxd_quark *quarks, int n, int prec);
  // as pending_op_bytes for one quark without waiting for the field's lock:
  // if another thread holds it, the whole operator counts as pending (for
  // callers that hold other locks the field's users may take after it)
  size_t pending_op_bytes_nowait(const qxd_quark &q, int prec);
  // device bytes of the operators resident on this field (built and cached),
  // readable without the field's lock
  std::atomic<size_t> op_mem{0};
  std::map<std::string, std::unique_ptr<DevBuf>> work;  // named workspaces
  std::recursive_mutex mu;

  // workspace of at least `bytes` under `name`
  void *workspace(const std::string &name, size_t bytes, hipError_t *err);
  // operator for a quark in precision prec (built on first use)
  qxd_status get_op(const qxd_quark &q, int prec, Operator **out, hipStream_t st);
  // the operator if it is already built in precision prec (nothing is
  // allocated), else nullptr
  Operator *find_op(const qxd_quark &q, int prec);
  qxd_status ensure_links(int prec, hipStream_t st);
  // operator fields for the kernels: links with the U(1) phase folded in
  OpFields op_fields(const Operator &op, int prec) const;
  // variant reading the shared SU(3) links and the U(1) angles
  OpFields op_fields_u(const Operator &op, int prec) const;
  size_t spinor_bytes(int prec) const { return qxd::spinor_bytes(prec, g.V); }
};

int qhat_of(double q, double q_el, bool *ok);

}  // namespace qxd

struct qxd_field : public qxd::Field {};

struct qxd_ctx {
  int device = 0;
  std::mutex mu;
  int n_fields = 0;
  qxd_serve *serve = nullptr;
};

#define QXD_HIP_CHECK(...)                                                          \
  do {                                                                               \
    hipError_t _e = (__VA_ARGS__);                                                          \
    if (_e != hipSuccess) {                                                          \
      qxd::set_error("HIP error %s at %s:%d", hipGetErrorString(_e), __FILE__, __LINE__); \
      return _e == hipErrorOutOfMemory ? QXD_ENOMEM : QXD_EDEVICE;                   \
    }                                                                                \
  } while (0)
