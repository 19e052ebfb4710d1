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

template <int P>
struct SapOp {
  const typename St<P>::pair_t *links;
  const typename St<P>::real_t *angles;
  int qhat;
  const typename St<P>::pair_t *pauli;
  const typename St<P>::pair_t *pinv;
};

template <int P>
struct SapVecs {
  Spinor<P> rho, r, psi, v;
};

// one right-hand side of a batched SAP pass (kept in device memory)
template <int P>
struct SapSlot {
  SapOp<P> op;
  SapVecs<P> vec;
};

size_t sap_lds_bytes(int prec, const Geom &g);

// One colour pass of SAP for the active slots act[0..nact) of a batch.
template <int P>
hipError_t launch_sap_batch(const Geom &g, const int *blocks, int nblocks_colour, const SapSlot<P> *slots,
                            const int *act, int nact, int first, int skip_face, int nmr, hipStream_t st);

template <int P>
hipError_t launch_sap_colour(const SapArgs<P> &a, int nblocks_colour, hipStream_t st);

// Four-lanes-per-site block solver (sap_quad.hip): reduced precisions, links
// with the phase folded in, at most 128 sites of each parity per block.
bool sap_quad_ok(int prec, const Geom &g, int qhat);
template <int P>
hipError_t launch_sapq_colour(const SapArgs<P> &a, int nblocks_colour, hipStream_t st);
template <int P>
hipError_t launch_sapq_batch(const Geom &g, const int *blocks, int nblocks_colour, const SapSlot<P> *slots,
                             const int *act, int nact, int first, int skip_face, int nmr, hipStream_t st);

// Pairs of slots that share the operator, two right-hand sides per
// work-group (links and Pauli rows staged once): pairs[2 p], pairs[2 p + 1].
bool sap_quad_pairs_ok(int prec, const Geom &g);
template <int P>
hipError_t launch_sapq_pairs(const Geom &g, const int *blocks, int nblocks_colour, const SapSlot<P> *slots,
                             const int *pairs, int npair, int first, int skip_face, int nmr, hipStream_t st);

}  // namespace qxd
