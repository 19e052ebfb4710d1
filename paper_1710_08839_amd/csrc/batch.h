// Batched kernels over right-hand-side slots (batch.hip, sap.hip).
#pragma once

#include "qxd_impl.h"
#include "sap.h"

namespace qxd {

// one right-hand side of a batched D application (kept in device memory)
template <int P>
struct DSlot {
  const typename St<P>::pair_t *links;   // W = U z^qhat of the slot's charge
  const typename St<P>::pair_t *pauli;   // Pauli term of the slot's operator
  Spinor<P> in, out;                     // full-lattice native spinors
};

// out = D in for the active slots act[0..nact) (requires 2 * block sites <= 256)
template <int P>
hipError_t launch_dirac_batch(const Geom &g, const DSlot<P> *slots, const int *act, int nact, int group,
                              hipStream_t st);

}  // namespace qxd
