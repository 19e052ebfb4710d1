// Host-side launchers of the libqxd kernels (precision-erased interfaces).
#pragma once

#include <hip/hip_runtime.h>

#include "qxd_impl.h"

namespace qxd {

// ---- fields (field.hip) ----------------------------------------------------
// Extended-lattice links/angles in native order from physical API-layout
// arrays, with the orbifold constraint on the mirror half (Sec. 2.1) and the
// links across an open time boundary set to zero.
hipError_t launch_orbifold(const Geom &g, const double *u_phs, const double *a_phs,
                           double2 *links, double *angles, hipStream_t st);

// Pauli term P = 4 + m0 + dD_sw + dD_b (Sec. 2.3) in FP64, packed Hermitian
// blocks; dD_b from the time boundary type of g with the coefficients cF, cFp;
// the identity on the fixed slice x0 = 0 of SF and open-SF boundaries.
hipError_t launch_pauli_build(const Geom &g, const double2 *links, const double *angles,
                              int has_u1, double kappa, double csw, double u1coef, double cF, double cFp,
                              double2 *pauli, hipStream_t st);

// Inverse blocks of P on odd sites (D_oo^-1); *bad counts singular blocks.
hipError_t launch_pauli_invert(const Geom &g, const double2 *pauli, double2 *pinv,
                               int *bad, hipStream_t st);

// W = U exp(i qhat A) in FP64 ([4][9][V] pairs), times the fermion boundary
// phase e^{+-i theta_mu} on the links whose forward hop crosses the boundary
// of direction mu (+ on the physical half, - on the C* mirror half).
hipError_t launch_fold_phase(const Geom &g, const double2 *links, const double *angles, int qhat,
                             const double theta[4], double2 *w, hipStream_t st);

// FP64 pairs -> storage precision `prec` (n pairs).
// FP64 block-major field with K pairs per site over `sites` sites -> the
// storage precision and component packing of prec.
hipError_t launch_convert_field(int prec, const Geom &g, int K, int64_t sites, const double2 *src, void *dst,
                                hipStream_t st);
hipError_t launch_convert_reals(const double *src, float *dst, int64_t n, hipStream_t st);

// API-layout FP64 spinors <-> native spinors of precision prec (nrhs each).
hipError_t launch_pack(int prec, const Geom &g, const double *api, void *native, int nrhs,
                       hipStream_t st);
hipError_t launch_unpack(int prec, const Geom &g, const void *native, double *api, int nrhs,
                         hipStream_t st);

struct SpinorArg;
// Zero native sites [first, first + count) of a spinor.
hipError_t launch_zero_sites(int prec, SpinorArg v, int64_t first, int64_t count, hipStream_t st);
// v = gamma5 v on sites [first, first + count), in place
hipError_t launch_g5_sites(int prec, SpinorArg v, int64_t first, int64_t count, hipStream_t st);
// out = ca G_a a + cb G_b b on sites [first, first + count), G = gamma5 if
// the flag is set else 1, complex coefficients; b may be null (cb ignored);
// out may be a or b (site-local)
hipError_t launch_lincomb_sites(int prec, SpinorArg out, SpinorArg a, double ca_re, double ca_im, bool g5a,
                                SpinorArg b, double cb_re, double cb_im, bool g5b, int64_t first, int64_t count,
                                hipStream_t st);

// ---- Dirac operator (dirac.hip) -----------------------------------------
struct OpFields {
  const void *links;    // [4][9][V] pairs of precision prec
  const void *angles;   // [4][V] reals (double for F64, float otherwise)
  const void *pauli;    // [36][V] pairs
  const void *pinv;     // [36][V/2] pairs (odd sites)
  int qhat;
};

enum DiracKind {
  DK_FULL = 0,     // out = P in - acc(in)/2           (all sites)
  DK_HOP = 1,      // out = -acc(in)/2                  (all sites)
  DK_PAULI = 2,    // out = P in                        (all sites)
  DK_ODD = 3,      // out_o = Pinv (self_o + c acc(in_e))   (odd sites)
  DK_EVEN = 4,     // out_e = P self_e + c acc(in_o)        (even sites)
  DK_EVEN_ID = 5,  // out_e = self_e + c acc(in_o)          (even sites)
};

// Spinor operands: pointer to a native spinor with `sites` sites whose first
// site has native index `off` (full field: sites = V, off = 0; even half:
// sites = V/2, off = 0; odd half: sites = V/2, off = V/2).
// A native spinor over the sites [off, off + sites) (block-major runs rd).
struct SpinorArg {
  void *ptr;
  int64_t sites;
  int64_t off;
  RunDiv rd;
};

// Autotuned on first use per (prec, kind, volume, phase-on-the-fly): the
// first call times the hop-group variants on its own operands.  With
// may_tune = false nothing is timed: the variant already chosen for the key
// is used, or a fixed default if none has been chosen yet.
hipError_t launch_dirac(int prec, DiracKind kind, const Geom &g, const OpFields &f,
                        SpinorArg in, SpinorArg self, SpinorArg out, double c, hipStream_t st,
                        bool may_tune = true);

// Kernel variant chosen by the autotuner for a key (0 if not tuned yet):
// hop group size, plus 16 for the LDS-staged variant.
int tuned_group(int prec, int kind, int V, int phase);

// Force a variant for every later launch (0: back to the autotuner); false
// for an invalid choice.
bool force_dirac_variant(int choice);

}  // namespace qxd
