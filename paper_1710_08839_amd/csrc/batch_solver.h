// Batched SAP-preconditioned GCR with FP64 defect correction: many right-hand
// sides (each with its own quark) on one gauge field advance together, one
// inner FGCR iteration per step.  The Schwarz block solves and the Dirac
// operator of a step run as one batched launch over all active right-hand
// sides; Gram-Schmidt, restarts and the outer FP64 correction are per
// right-hand side.  A right-hand side's arithmetic never depends on which
// others share its steps, so a solve gives the same bits alone or batched.
#pragma once

#include <array>
#include <functional>
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
  // free every slot's memory (no right-hand side may be in flight)
  qxd_status release_slots();
  // start solving D psi = eta for one right-hand side (API-layout FP64
  // device buffers); may finish at once (zero or converged guess)
  qxd_status add(const qxd_quark &q, const double *eta_api, double *psi_api, bool use_guess, void *tag);
  // one inner iteration for every active right-hand side
  qxd_status step();
  // end every active right-hand side with `status` after a failed step: no
  // device work (the device may be unusable), the solutions are not written
  // back, their operators are released and take_finished() reports them
  void abort_all(int status);
  // right-hand sides finished since the last call
  std::vector<Finished> take_finished();
  // the solver parameters this batch runs with
  const qxd_solver &params() const { return s_; }
  int prec() const { return prec_; }
  Field *field() const { return f_; }
  // classical Gram-Schmidt passes per step (1, or 2 with re-orthogonalisation)
  int gs_passes() const { return gs_passes_; }

  struct Slot;  // one right-hand side in flight (batch_solver.cpp)

  // Issue the fixed launch sequence of a step (the batched SAP passes, D and
  // the batched Gram-Schmidt)
  // on the solver's stream: eagerly the first time a configuration `key` is
  // seen, then captured once into a HIP graph (on a private stream: the
  // caller's may be the legacy default stream, which cannot be captured) and
  // replayed whenever the configuration comes again (a few graphs are kept:
  // the number of active and paired right-hand sides changes as they pass
  // through cycle ends).  The sequence reads its per-step data from device
  // tables written before it.
  qxd_status run_step_launches(const std::array<int64_t, 10> &key,
                               const std::function<qxd_status(hipStream_t)> &issue);

 private:
  qxd_status finish(Slot &sl, int status);
  void release_ops(Slot &sl);
  qxd_status new_inner(Slot &sl);
  qxd_status cycle_end(Slot &sl);
  qxd_status outer_update(Slot &sl);
  Field *f_;
  int prec_;
  qxd_solver s_;
  hipStream_t st_;
  int nkv_, ncy_, nmr_, gs_passes_ = 1;
  double inner_tol_;
  std::vector<std::unique_ptr<Slot>> slots_;
  std::vector<Finished> done_;
  // device/pinned staging of slot descriptors and the active list
  DevBuf dslots_, sslots_, act_, partial_;
  // batched Gram-Schmidt: per-slot table and partial sums
  DevBuf gsslots_, gspart_;
  void *h_stage_ = nullptr;
  size_t h_stage_bytes_ = 0;
  double *h_norms_ = nullptr;
  DevBuf d_norms_;
  // graphs of the step's launch sequence, most recently used last, and the
  // configurations seen once
  using StepKey = std::array<int64_t, 10>;
  std::vector<std::pair<StepKey, hipGraphExec_t>> graphs_;
  std::vector<StepKey> seen_;
  hipStream_t cap_st_ = nullptr;
  bool graphs_ok_ = true;
  void drop_graphs();
};

// SAP-GCR parameters taken when the caller passes 0: the measured best of
// sweeps on the hardest synthetic operators (48x24^3 C*, q = -1/3)
constexpr int kDefaultNkv = 32, kDefaultNcy = 4, kDefaultNmr = 4;
// relative residual reduction per inner solve by inner precision (F64, F32,
// F16+scale, BF16), measured best on the same operators
constexpr double kDefaultInnerTol[4] = {1e-6, 1e-5, 2e-2, 1e-2};

// Process-wide switch for graph capture of the batched steps (testing hook).
void set_step_graphs(bool on);
// Gram-Schmidt passes (1 or 2) of batch solvers constructed from now on
// (measurement hook).
void set_gs_passes(int passes);
// Make the next n batched steps of any solver fail before any launch
// (testing hook for the error paths of qxd_solve and the serve loop).
void inject_step_failures(int n);
// process-wide totals: step graphs captured, and step graphs launched
void step_graph_counts(int64_t *captures, int64_t *replays);

}  // namespace qxd
