// Solvers behind qxd_solve (solver.cpp).
#pragma once

#include "host.h"

namespace qxd {

qxd_status solve(Field *f, const qxd_quark *quarks, int nquark, const qxd_solver &s,
                 const double *eta_dev, double *psi_dev, int nrhs, int use_guess,
                 qxd_solve_info *info, hipStream_t st);

// Apply the operator `which` to one native spinor (abi.cpp); mu: the twisted
// mass of the even-odd operators (the caller's quark: an operator is shared
// by quarks that differ only in mu).  The odd-site
// temporary of the Schur complement is dhat_tmp if given (a half-lattice
// spinor of precision prec), else a field workspace; with may_tune = false
// no kernel variant is timed.
qxd_status apply_native(Field *fd, const Operator &op, double mu, qxd_op which, int prec, void *in, void *out,
                        hipStream_t st, void *dhat_tmp = nullptr, bool may_tune = true);

// out_e = (D^ + i mu gamma5) in_e on the even half of full-lattice native
// spinors of precision prec (odd half of out untouched); tmp: an odd-half
// native spinor (abi.cpp).
hipError_t schur_tm(Field *fd, const OpFields &f, int prec, double mu, SpinorArg in, SpinorArg out, void *tmp,
                    hipStream_t st, bool may_tune = true);

// Multi-shift CG (X + shifts[j]) psi_j = eta_e, X = D^dag D^ + mu^2, and the
// rational function A prod (X + nu^2)/(X + mu^2) eta_e (multishift.hip);
// API-layout FP64 device buffers.
qxd_status multishift_solve(Field *f, const qxd_quark &quark, const double *shifts, int n, double tol,
                            int maxiter, const double *eta_api, double *psi_api, qxd_solve_info *info,
                            hipStream_t st);
qxd_status rational_apply(Field *f, const qxd_quark &quark, double A, const double *nu, const double *mu, int n,
                          double tol, int maxiter, const double *eta_api, double *out_api, qxd_solve_info *info,
                          hipStream_t st);

// M_SAP on native spinors of precision prec: psi = M_SAP rho (ncy cycles,
// nmr MR steps per block solve).
qxd_status sap_apply(Field *f, const Operator &op, int prec, int ncy, int nmr, void *rho, void *psi,
                     hipStream_t st);

// Time one colour pass of the paired SAP block solver (two right-hand sides
// per work-group, as in the batched solve) for npair pairs of synthetic
// vectors: *ms = average over reps launches (HIP events on st).
qxd_status debug_sap_pair_pass(Field *f, const qxd_quark &q, int prec, int nmr, int npair, int reps, float *ms,
                               hipStream_t st);

// Device lists of the block indices of each SAP colour (built on first use).
qxd_status sap_block_lists(Field *f, const int **lists, int *per_colour);

// Check that the layout blocks admit the two-colour SAP decomposition.
qxd_status check_sap_blocks(const Field *f);

}  // namespace qxd
