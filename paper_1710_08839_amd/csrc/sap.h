// Schwarz alternating procedure (sap.hip).
#pragma once

#include "qxd_impl.h"

namespace qxd {

template <int P>
struct SapArgs {
  Geom g;
  const typename St<P>::pair_t *links;   // W or U (with angles/qhat)
  const typename St<P>::real_t *angles;
  int qhat;
  const typename St<P>::pair_t *pauli;   // [36][V]
  const typename St<P>::pair_t *pinv;    // [36][V/2]
  const int *blocks;                      // block indices of this colour
  Spinor<P> rho;                          // SAP input, read when first != 0
  Spinor<P> r;                            // residual (full lattice)
  Spinor<P> psi;                          // accumulated solution (full lattice)
  Spinor<P> v;                            // latest block corrections (full lattice)
  int first;       // first cycle: r := rho, psi := v
  int skip_face;   // the other colour has no correction yet
  int nmr;
};

size_t sap_lds_bytes(int prec, const Geom &g);

template <int P>
hipError_t launch_sap_colour(const SapArgs<P> &a, int nblocks_colour, hipStream_t st);

}  // namespace qxd
