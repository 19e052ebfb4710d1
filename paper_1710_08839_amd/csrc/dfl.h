// Local deflation of the SAP-GCR solver (qxd_dfl_setup, QXD_SOLVER_DFL_SAP_GCR):
// kernels in dfl.hip, host side in dfl_solver.cpp.
//
// The paper names the locally deflated SAP-GCR (abstract; Sec. 2 feature
// list; Appendix A and Table 2, where it serves the expensive factors) and
// cites the published method for its steps:
//   - deflation fields: ns random fields refined by SAP-smoothed inverse
//     iteration, psi <- M_sap psi / |M_sap psi|;
//   - basis: on every SAP block the restricted fields, orthonormalised by
//     modified Gram-Schmidt; V maps coefficients c[block][k] to fields;
//   - little operator A = V^dag D V: per block its couplings to itself and,
//     through each of its eight faces, to the block across;
//   - preconditioner M_dfl r = V A^-1 V^dag r + M_sap (r - D V A^-1 V^dag r),
//     A^-1 by GCR on the even-block Schur complement A_ee - A_eo A_oo^-1 A_oe
//     (blocks coloured as for SAP, so A_ee and A_oo are block diagonal),
//     right-preconditioned with the inverse diagonal blocks A_ee^-1.
#pragma once

#include "host.h"

namespace qxd {

constexpr int DFL_NSMAX = 32;  // basis vectors per block
constexpr int DFL_SLOTS = 9;   // couplings of a block: itself, then faces 2 mu + (0 fwd, 1 bwd)

// Pinned host slots (mapped and coherent: the last kernel of a step writes
// them) and events through which the little GCR reads the residual norm of a
// step while the device already runs the next one.
struct LittleSync {
  // host[0..1]: |r|^2 of a step, by step parity; host[2]: |r_0|^2 of the
  // solve (host[3..4] the other sums of the same reduction)
  static constexpr int NSLOT = 8;
  double *host = nullptr;
  double *dev = nullptr;  // their device address (mapped pinned memory)
  hipEvent_t ev[2] = {nullptr, nullptr};
  LittleSync() = default;
  LittleSync(const LittleSync &) = delete;
  LittleSync &operator=(const LittleSync &) = delete;
  ~LittleSync() {
    // a copy into the slots may still be queued (a solve that stopped on an
    // error): wait for the events recorded after the copies before freeing
    for (hipEvent_t e : ev)
      if (e) (void)hipEventSynchronize(e);
    if (host) (void)hipHostFree(host);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  hipError_t init() {
    hipError_t e = hipSuccess;
    if (!host) {
      e = hipHostMalloc((void **)&host, NSLOT * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent);
      if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&dev, host, 0);
    }
    for (int i = 0; i < 2 && e == hipSuccess; i++)
      if (!ev[i]) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    return e;
  }
};

struct Dfl {
  qxd_dfl_params p{};     // with the defaults filled in
  int ns = 0;
  int nb = 0;              // blocks
  size_t vbytes = 0;       // bytes of one basis field (FP32 native spinor)
  DevBuf basis;            // ns FP32 native spinors; field k holds basis vector k of every block
  DevBuf a;                // little operator [nb][9][ns][ns] double2
  DevBuf ainv;             // inverses of the diagonal blocks A[b][0] [nb][ns][ns] double2
  DevBuf at32, ait32;      // FP32 copies of a and ainv for the little solve, transposed per block
  DevBuf at16;             // FP16 copy of a, transposed per block (little solves to a loose tolerance)
  DevBuf nbr;              // [nb][9] int: the block each slot couples to
  DevBuf even, odd;        // the blocks of each SAP colour (neighbours have opposite colours)
  DevBuf vpos;             // [nb] int: a block's position in the little vectors (even blocks first)
  DevBuf nbrv;             // [nb][9] int: vpos of the block each slot couples to
  int ne = 0, no = 0;
  // little GCR: Krylov vectors z_k (preconditioned) and w_k = A z_k (even
  // blocks only, ne * ns entries each), work vectors, scalars
  DevBuf lz, lw, lx, lr, lb, lu, lpart, lscal;
  LittleSync sync;
  // counters since the last read: preconditioner applications, little GCR
  // iterations (total and the largest of one solve)
  int64_t applications = 0, little_iters = 0, little_max = 0;
  size_t bytes() const;
};

// ---- kernels (dfl.hip) ----------------------------------------------------
// basis field k of `basis` is at basis + k * vbytes (FP32 native spinors)

// ns Gaussian start fields (N(0,1) real and imaginary parts) from a
// counter-based generator (splitmix64 of seed, field, site, component)
hipError_t launch_dfl_random(const Geom &g, void *basis, size_t vbytes, int ns, uint64_t seed, hipStream_t st);
// modified Gram-Schmidt of the ns restricted fields on every block, in place;
// *bad counts blocks on which a field vanished
hipError_t launch_dfl_ortho(const Geom &g, void *basis, size_t vbytes, int ns, int *bad, hipStream_t st);
// Little vectors hold block b's ns entries at position vpos[b] (entries
// vpos[b] * ns ... + ns - 1): the blocks of the first colour first, in the
// order of their list, then those of the second, so that the Krylov vectors
// of the even-block system are the first ne * ns entries.
// c[vpos[b] * ns + k] = (phi_{b,k}, r)_b for an FP32 native spinor r
hipError_t launch_dfl_restrict(const Geom &g, const void *basis, size_t vbytes, int ns, const void *r,
                               const int *vpos, double2 *c, hipStream_t st);
// out = sum_{b,k} c[vpos[b] * ns + k] phi_{b,k} (FP32 native spinor)
hipError_t launch_dfl_prolong(const Geom &g, const void *basis, size_t vbytes, int ns, const double2 *c,
                              const int *vpos, void *out, hipStream_t st);
// face couplings of basis field l: a[b][1 + d][k][l] = (phi_{b,k}, H_d phi_l)_b for the
// eight faces d of every block (H_d: the hops of D through that face), and nbr[b][1 + d]
hipError_t launch_dfl_face(const Geom &g, const double2 *wl64, const void *basis, size_t vbytes, int ns, int l,
                           double2 *a, int *nbr, hipStream_t st);
// couplings inside the blocks: a[b][0][k][l] = (phi_{b,k}, y)_b - sum_d a[b][1 + d][k][l]
// with y = D phi_l (FP64 native spinor); nbr[b][0] = b
hipError_t launch_dfl_diag(const Geom &g, const void *basis, size_t vbytes, int ns, int l, const void *y64,
                           double2 *a, int *nbr, hipStream_t st);
// ainv[b] = a[b][0]^-1 (Gauss-Jordan with partial pivoting); *bad counts singular blocks
hipError_t launch_little_invert(int nb, int ns, const double2 *a, double2 *ainv, int *bad, hipStream_t st);
// FP32 (MT = float2) or FP16 (MT = h2_t) copies of nmat ns x ns blocks,
// transposed within each block
template <class MT>
hipError_t launch_little_pack(int64_t nmat, int ns, const double2 *src, MT *dst, hipStream_t st);
// for the i-th block b = list[i] of `list`, whose little-vector entries are
// at position v = vbase + i: h_v = (xa ? A[b][0] xa_v : (w ? w_v : 0)) -
// sum_{d >= 1} A[b][d] xh[nbrv[b][d]] (the couplings to the blocks across the
// faces; nbrv: their positions), y_v = h_v, or y_v = s ainv[b] h_v if ait is
// given; at: the transposed FP32 (MT = float2) or FP16 (MT = h2_t) copy of A,
// ait: the transposed FP32 copy of the inverse diagonal blocks.  y must not
// overlap the entries of xa, w and xh the blocks of `list` read.
template <class MT>
hipError_t launch_lt_hop(const int *list, int nlist, int vbase, int ns, const MT *at, const int *nbrv,
                         const double2 *xa, const double2 *w, const double2 *xh, const float2 *ait, double s,
                         double2 *y, hipStream_t st);
// for the i-th block b = list[i] of `list`: y_v = s ainv[b] x_v with v =
// vbase + i (x and y distinct); ait: the transposed FP32 copy of the inverse
// diagonal blocks
hipError_t launch_lt_jacobi(const int *list, int nlist, int vbase, int ns, const float2 *ait, double s,
                            const double2 *x, double2 *y, hipStream_t st);
// out[2j..2j+1] = (W_j, x) for j < k, W_j = W + j * n (complex vectors of length n)
hipError_t launch_lv_dots(const double2 *W, int k, int64_t n, const double2 *x, double *partial, double *out,
                          hipStream_t st);
// x1 -= sum_{j<k} c_j W1_j and x2 -= sum_{j<k} c_j W2_j with
// c_j = (d[2j] + i d[2j+1]) / wn[j] (0 if wn[j] = 0)
hipError_t launch_lv_maxpy2(double2 *x1, const double2 *W1, double2 *x2, const double2 *W2, int k, int64_t n,
                            const double *d, const double *wn, hipStream_t st);
// partial sums of s[0] = |w|^2, s[1..2] = (w, r) into the partial-sum
// scratch, and, if s is given, their totals into s
hipError_t launch_lv_dot2(const double2 *w, const double2 *r, int64_t n, double *partial, double *s,
                          hipStream_t st);
// with s the totals of the partial sums launch_lv_dot2 left in `partial`:
// alpha = (s[1] + i s[2]) / s[0] (0 if s[0] = 0): x += alpha z, r -= alpha w; *wn = s[0];
// out[0] = |r|^2 (out may be the device address of mapped host memory)
hipError_t launch_lv_update(double2 *x, const double2 *z, double2 *r, const double2 *w, int64_t n, double *wn,
                            double *partial, double *out, hipStream_t st);
// partial-sum scratch of the little reductions (doubles)
size_t lv_partial_doubles();

// ---- host side (dfl_solver.cpp) ---------------------------------------------------
// build the subspace and little operator of the quark's operator (replacing
// any earlier one); init_api: ns API-layout FP64 start fields or null
qxd_status dfl_setup(Field *f, const qxd_quark &q, const qxd_dfl_params *params, const double *init_api,
                     hipStream_t st);
// out = M_dfl r on FP32 native full-lattice spinors; little_tol 0: the setup's
qxd_status dfl_precond(Field *f, Operator &op, double little_tol, int ncy, int nmr, void *r32, void *out32,
                       hipStream_t st, int *little_iters = nullptr);
// D psi = eta (FP64 native) by defect correction around flexible GCR(M_dfl) in FP32
qxd_status dfl_solve(Field *f, Operator &op, const qxd_solver &s, void *eta64, void *psi64, bool guess,
                     qxd_solve_info *info, hipStream_t st);

}  // namespace qxd
