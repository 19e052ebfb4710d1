// Batched SAP-preconditioned GCR with FP64 defect correction: many right-hand
// sides (each with its own quark) on one gauge field advance together, one
// inner FGCR iteration per step.  The Schwarz block solves and the Dirac
// operator of a step run as one batched launch over all active right-hand
// sides; Gram-Schmidt, restarts and the outer FP64 correction are per
// right-hand side.  A right-hand side's arithmetic never depends on which
// others share its steps, so a solve gives the same bits alone or batched.
#pragma once

#include <memory>
#include <vector>

#include "host.h"

namespace qxd {

struct Finished {
  int slot;
  void *tag;
  qxd_solve_info info;
};

class BatchSolver {
 public:
  BatchSolver(Field *f, int prec, const qxd_solver &s, hipStream_t st);
  ~BatchSolver();
  BatchSolver(const BatchSolver &) = delete;
  BatchSolver &operator=(const BatchSolver &) = delete;

  // device bytes one right-hand side needs (for admission control)
  static size_t slot_bytes(const Field *f, int prec, const qxd_solver &s);
  // make room for n right-hand sides (allocates their workspaces)
  qxd_status reserve(int n);
  int capacity() const { return (int)slots_.size(); }
  int active() const;
  int free_slots() const { return capacity() - active(); }
  // start solving D psi = eta for one right-hand side (API-layout FP64
  // device buffers); may finish at once (zero or converged guess)
  qxd_status add(const qxd_quark &q, const double *eta_api, double *psi_api, bool use_guess, void *tag);
  // one inner iteration for every active right-hand side
  qxd_status step();
  // right-hand sides finished since the last call
  std::vector<Finished> take_finished();
  // the solver parameters this batch runs with
  const qxd_solver &params() const { return s_; }
  int prec() const { return prec_; }
  Field *field() const { return f_; }

  struct Slot;  // one right-hand side in flight (batch_solver.cpp)

 private:
  qxd_status finish(Slot &sl, int status);
  qxd_status new_inner(Slot &sl);
  qxd_status cycle_end(Slot &sl);
  qxd_status outer_update(Slot &sl);
  Field *f_;
  int prec_;
  qxd_solver s_;
  hipStream_t st_;
  int nkv_, ncy_, nmr_;
  double inner_tol_;
  std::vector<std::unique_ptr<Slot>> slots_;
  std::vector<Finished> done_;
  // device/pinned staging of slot descriptors and the active list
  DevBuf dslots_, sslots_, act_, partial_;
  void *h_stage_ = nullptr;
  size_t h_stage_bytes_ = 0;
  double *h_norms_ = nullptr;
  DevBuf d_norms_;
};

}  // namespace qxd
