// Solvers behind qxd_solve (solver.cpp).
#pragma once

#include "host.h"

namespace qxd {

qxd_status solve(Field *f, const qxd_quark *quarks, int nquark, const qxd_solver &s,
                 const double *eta_dev, double *psi_dev, int nrhs, int use_guess,
                 qxd_solve_info *info, hipStream_t st);

// Apply the operator `which` to one native spinor (abi.cpp).  The odd-site
// temporary of the Schur complement is dhat_tmp if given (a half-lattice
// spinor of precision prec), else a field workspace; with may_tune = false
// no kernel variant is timed.
qxd_status apply_native(Field *fd, const Operator &op, qxd_op which, int prec, void *in, void *out,
                        hipStream_t st, void *dhat_tmp = nullptr, bool may_tune = true);

// M_SAP on native spinors of precision prec: psi = M_SAP rho (ncy cycles,
// nmr MR steps per block solve).
qxd_status sap_apply(Field *f, const Operator &op, int prec, int ncy, int nmr, void *rho, void *psi,
                     hipStream_t st);

// Device lists of the block indices of each SAP colour (built on first use).
qxd_status sap_block_lists(Field *f, const int **lists, int *per_colour);

// Check that the layout blocks admit the two-colour SAP decomposition.
qxd_status check_sap_blocks(const Field *f);

}  // namespace qxd
