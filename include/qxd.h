/*
 * qxd.h -- C ABI of libqxd: the O(a)-improved Wilson-clover Dirac operator on
 * an SU(3) x U(1) gauge field with C* spatial boundaries, and its even-odd /
 * SAP-preconditioned GCR solvers, on one AMD MI355X (gfx950).
 *
 * The operations follow Campos et al., "openQ*D simulation code for QCD+QED"
 * (Lattice 2017, arXiv:1710.08839):
 *   - extended lattice, orbifold constraint, shifted boundaries: Sec. 2.1
 *   - D = m0 + Dw + dD_sw, charges qhat = q / q_el, clover tensors: Sec. 2.3
 *   - even-odd blocks and the Schur complement D^: Sec. 2.4
 *   - SAP-preconditioned GCR: named in the abstract and Sec. 2.
 *
 * Conventions shared by every entry point
 *   Axes: mu = 0 is time, 1..3 are space.  C* needs direction 1; under C* the
 *   extended lattice is T x 2L1 x L2 x L3 and sites with x1 >= L1 form the
 *   mirror lattice.
 *   Site order ("API order"): ((x0*N1 + x1)*L2 + x2)*L3 + x3, N1 = 2L1 under
 *   C*, else L1.  x3 runs fastest.
 *   Gamma matrices: chiral basis, gamma_0 = [[0,-1],[-1,0]],
 *   gamma_k = [[0,-i s_k],[i s_k,0]], gamma_5 = diag(1,1,-1,-1).
 *   Spinors in API layout: double [nrhs][V_ext][4 spin][3 colour][re,im].
 *   D = (4 + m0) + dD_sw + dD_b - 1/2 sum_mu [(1-g_mu) W(x,mu) psi(x+mu)
 *       + (1+g_mu) W(x-mu,mu)^dag psi(x-mu)],  W = U exp(i qhat A),
 *   m0 = 1/(2 kappa) - 4.  Fermions are antiperiodic in time (time_bc = 0)
 *   or the time hop is absent (open, SF, open-SF: qxd_lattice.time_bc).
 *   Clover: F = (Q_munu - Q_munu^dag)/8 from the four plaquette leaves;
 *   Ahat = i/(4 q_el) Im(sum of the four U(1) plaquettes).
 *
 * Memory: pointers named *_host are host memory, *_dev device memory on the
 * context's GPU.  The caller owns every buffer it passes; the library owns
 * field and context handles and their workspaces.  Calls return a
 * qxd_status; on error nothing has been written unless stated, and
 * qxd_last_error() gives a message (thread-local).  Arguments are checked on
 * the host before any device work.  Device work is queued on the stream
 * passed as `stream` (a hipStream_t, NULL = the default stream); entry points
 * that return results to the host synchronise that stream.
 *
 * Native layout: for speed, spinors can be kept in the library's private
 * device layout and precision (qxd_spinor_bytes / qxd_spinor_pack /
 * qxd_spinor_unpack); pass QXD_NATIVE to qxd_dirac_apply to use it.  Native
 * buffers must be 16-byte aligned (QXD_EINVAL otherwise); their content is
 * opaque (lattice blocks stored one after another, components grouped per
 * 16 bytes) and may change between library versions.
 */
#ifndef QXD_H
#define QXD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QXD_ABI_VERSION 3

typedef enum {
  QXD_OK = 0,
  QXD_EINVAL = -1,   /* invalid argument (checked before any device work)   */
  QXD_ENOMEM = -2,   /* device or host allocation failed                     */
  QXD_ENOCONV = -3,  /* solver hit maxiter; best iterate and info written    */
  QXD_EFLOAT = -4,   /* NaN/Inf in the input or the iteration                */
  QXD_EDEVICE = -5,  /* HIP runtime error                                     */
  QXD_EBUSY = -6,    /* serve request still pending                           */
  QXD_ENOTFOUND = -7 /* unknown serve ticket                                  */
} qxd_status;

/* Storage precision of spinors, links and Pauli terms.  F64 computes in FP64;
 * the others compute in FP32.  F16S stores spinors as FP16 with one FP32
 * scale per site (the site's largest component magnitude). */
typedef enum { QXD_F64 = 0, QXD_F32 = 1, QXD_F16S = 2, QXD_BF16 = 3 } qxd_prec;

typedef enum {
  QXD_OP_D = 0,      /* full D on all of the extended lattice (Sec. 2.3)      */
  QXD_OP_DHAT = 1,   /* D^ + i mu gamma5 on even sites, D^ = D_ee - D_eo
                        D_oo^-1 D_oe (Sec. 2.4) and mu the quark's twisted
                        mass (0: plain D^); odd sites of the output are 0    */
  QXD_OP_HOP = 2,    /* hopping part of D only (D minus its diagonal)         */
  QXD_OP_PAULI = 3,  /* diagonal part P(x) = 4 + m0 + dD_sw only              */
  QXD_OP_OOINV = 4,  /* D_oo^-1 on odd sites, even sites set to 0             */
  QXD_OP_G5D = 5,    /* gamma5 D (Hermitian: D is gamma5-hermitian, Sec. 2.3;
                        gamma5 = diag(1, 1, -1, -1) in the chiral basis)     */
  QXD_OP_DHAT_DAG = 6, /* (D^ + i mu gamma5)^dag = gamma5 (D^ - i mu gamma5)
                        gamma5 on even sites, odd sites 0                    */
  QXD_OP_NORMAL = 7  /* (D^ + i mu gamma5)^dag (D^ + i mu gamma5) = D^dag D^ +
                        mu^2 on even sites (Sec. 2.4: the operator of the
                        twisted-mass regulator and of the rational
                        approximation), odd sites 0                           */
} qxd_op;

#define QXD_NATIVE 1u  /* in/out are native-layout buffers of precision prec */

typedef struct {
  int dims[4];    /* physical T, L1, L2, L3; all even                        */
  int time_bc;    /* 0: periodic gauge, antiperiodic fermions; 1: open;
                     2: Schroedinger functional (SF): the fermion field is
                     fixed to zero on x0 = 0 (D is the identity on that slice,
                     no hop enters or leaves it) and the hop across x0 = T-1
                     -> T is absent, the time links into x0 = T staying in
                     the clover term with the x0 = 0 slice's spatial links as
                     the upper boundary field; 3: open-SF (SF at x0 = 0, open
                     at x0 = T-1).  Sec. 2 feature list                      */
  int cstar;      /* 0: periodic space; k = 1..3: directions 1..k are C*    */
  double q_el;    /* elementary charge (Sec. 2.2); 1/6 is required with C*
                     for charged hadrons; 0 means 1/6                         */
  int block[4];   /* block size of the device layout and of SAP; each even,
                     dividing the extended extent (and L1); 0 means 4          */
  double cF;      /* time-boundary improvement coefficient c_F of dD_b (Sec.
                     2.3): dD_b = (c_F - 1) on x0 = 0 and T-1 (open), on x0 = 1
                     and T-1 (SF), on x0 = 1 (open-SF); 0 means 1            */
  double cF_prime;/* c_F' on x0 = T-1 of open-SF; 0 means 1                  */
} qxd_lattice;

typedef struct {
  double kappa;   /* hopping parameter, m0 = 1/(2 kappa) - 4               */
  double q;       /* charge in units of e; q / q_el must be an integer       */
  double csw;     /* SU(3) clover coefficient                                */
  double csw_u1;  /* U(1) clover coefficient                                 */
  double mu;      /* twisted mass of the even-odd operators QXD_OP_DHAT,
                     QXD_OP_DHAT_DAG, QXD_OP_NORMAL and of the multi-shift
                     solver and rational functions (Sec. 2.4); D itself and
                     the D solvers do not use it                             */
  double theta[4];/* fermion boundary phases psi(x + L_mu e_mu) =
                     e^{i theta_mu} psi(x) in periodic directions (Sec. 2
                     feature list), entering as e^{i theta_mu} on the links
                     whose forward hop crosses the boundary; on a C* lattice
                     the mirror half carries e^{-i theta_mu} (the orbifold
                     conjugates every U(1) field).  theta_0 multiplies the
                     antiperiodic sign of the time hop.  Must be 0 in C*
                     directions and, with open time, for mu = 0 (QXD_EINVAL) */
} qxd_quark;

typedef enum { QXD_SOLVER_EO_GCR = 0, QXD_SOLVER_SAP_GCR = 1, QXD_SOLVER_DFL_SAP_GCR = 2 } qxd_solver_kind;

typedef struct {
  int kind;           /* qxd_solver_kind                                       */
  double tol;         /* target |eta - D psi| / |eta| in FP64 (e.g. 1e-10)     */
  int maxiter;        /* EO_GCR: GCR iterations; SAP_GCR, DFL_SAP_GCR: inner
                         iterations                                            */
  int nkv;            /* Krylov vectors per restart cycle (0: 32 for SAP_GCR,
                         16 for EO_GCR)                                        */
  int ncy;            /* SAP cycles per preconditioner application (0: 4)      */
  int nmr;            /* MR steps per SAP block solve (0: 4)                   */
  int inner_prec;     /* qxd_prec of the SAP-GCR inner solver (DFL_SAP_GCR:
                         QXD_F32 only)                                         */
  double inner_tol;   /* relative residual reduction per inner solve (0: 1e-6
                         F64, 1e-5 F32, 2e-2 F16S, 1e-2 BF16)                  */
  int max_outer;      /* outer defect-correction steps (SAP_GCR)              */
} qxd_solver;

typedef struct {
  int status;         /* qxd_status of this right-hand side                    */
  int outer_iters;    /* defect-correction steps                               */
  int inner_iters;    /* GCR iterations (sum over outer steps)                 */
  double true_resid;  /* |eta - D psi| / |eta| computed in FP64 at the end     */
  double seconds;     /* wall time of this solve                               */
} qxd_solve_info;

typedef struct qxd_ctx qxd_ctx;
typedef struct qxd_field qxd_field;

/* Version of this ABI (QXD_ABI_VERSION). */
int qxd_abi_version(void);

/* Thread-local message describing the last error of this thread. */
const char *qxd_last_error(void);

/* Open a context on HIP device `device`.  *ctx receives the handle. */
qxd_status qxd_init(int device, qxd_ctx **ctx);

/* Release a context.  All its fields must have been released. */
qxd_status qxd_finalize(qxd_ctx *ctx);

/* Upload a gauge field (Sec. 2.1, 2.3).  U_host: double
 * [V_phs][4 mu][3][3][re,im], U(x,mu) row-major, physical sites in API order
 * with extent L1 in direction 1.  A_host: double [V_phs][4] U(1) potential
 * with z = exp(iA), or NULL for an SU(3)-only field.  Under C* the library
 * builds the mirror half by the orbifold constraint U(x+L1 e1) = U(x)^*,
 * A(x+L1 e1) = -A(x).  The host arrays may be freed after return. */
qxd_status qxd_field_upload(qxd_ctx *ctx, const qxd_lattice *lat,
                            const double *U_host, const double *A_host,
                            qxd_field **field);

/* Release a field and every operator (Pauli term) cached on it. */
qxd_status qxd_field_release(qxd_field *field);

/* Number of extended-lattice sites V_ext of the field. */
qxd_status qxd_field_volume(const qxd_field *field, int64_t *v_ext);

/* Bytes of one native-layout spinor of precision prec (nrhs = 1). */
qxd_status qxd_spinor_bytes(const qxd_field *field, qxd_prec prec, size_t *bytes);

/* API-layout FP64 spinors (device) -> native layout of precision prec. */
qxd_status qxd_spinor_pack(qxd_field *field, qxd_prec prec, const double *in_dev,
                           void *out_dev, int nrhs, void *stream);

/* Native layout of precision prec -> API-layout FP64 spinors (device). */
qxd_status qxd_spinor_unpack(qxd_field *field, qxd_prec prec, const void *in_dev,
                             double *out_dev, int nrhs, void *stream);

/* out = op(in) for nrhs spinors: D = m0 + Dw + dD_sw with the covariant
 * derivatives carrying U z^qhat and the SW term of both gauge groups (Sec.
 * 2.3), its diagonal and hopping parts, the even-odd blocks and the Schur
 * complement D^ = D_ee - D_eo D_oo^-1 D_oe (Sec. 2.4), or gamma5 D.
 * quarks: nquark entries; right-hand side r
 * uses quarks[r * nquark / nrhs] (nrhs must be a multiple of nquark).  With
 * flags & QXD_NATIVE, in_dev/out_dev are nrhs consecutive native spinors of
 * precision prec; otherwise they are API-layout FP64 buffers and the operator
 * is applied in precision prec.  in and out must not overlap.  Asynchronous
 * on `stream`. */
qxd_status qxd_dirac_apply(qxd_field *field, const qxd_quark *quarks, int nquark,
                           qxd_op op, qxd_prec prec, const void *in_dev, void *out_dev,
                           int nrhs, unsigned flags, void *stream);

/* Bytes of the device scratch buffer of qxd_dirac_apply_noalloc, one per GPU. */
#define QXD_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments and results as qxd_dirac_apply for the operators
 * QXD_OP_D to QXD_OP_G5D, but the call performs no hipMalloc, hipFree or
 * other allocation (QXD_OP_DHAT_DAG and QXD_OP_NORMAL: QXD_EINVAL).  Limits:
 *   - every quark's operator must already be built on this field in precision
 *     prec (an earlier qxd_dirac_apply or qxd_solve in that precision builds
 *     it); otherwise QXD_EINVAL and nothing is queued;
 *   - its temporaries live in one library-owned device buffer of
 *     QXD_NOALLOC_SCRATCH_BYTES per GPU, created when the library's code is
 *     loaded on that GPU (resolved by qxd_init) and held until the process
 *     ends.  Needed: nothing for native-layout D, HOP, PAULI, OOINV and G5D;
 *     one half-lattice native spinor of precision prec for QXD_OP_DHAT; two
 *     full-lattice native spinors of precision prec (each rounded up to 256
 *     bytes) more for API-layout buffers.  A call that needs more returns
 *     QXD_EINVAL before any device work;
 *   - all calls on one GPU share that buffer and it keeps the last call's
 *     contents: calls queued on one stream are ordered, but calls that
 *     overlap in time on one GPU (other streams, other threads) race;
 *   - the kernel variant is the one the autotuner already chose for the
 *     lattice and precision (a fixed default if none was chosen); nothing is
 *     timed.
 * Asynchronous on `stream`. */
qxd_status qxd_dirac_apply_noalloc(qxd_field *field, const qxd_quark *quarks, int nquark, qxd_op op,
                                   qxd_prec prec, const void *in_dev, void *out_dev, int nrhs,
                                   unsigned flags, void *stream);

/* Solve D psi = eta for nrhs right-hand sides (API-layout FP64, device), each
 * to |eta - D psi| / |eta| <= s->tol with the residual computed in FP64.  D
 * is the operator of qxd_dirac_apply (Sec. 2.3); psi lives on the whole
 * extended lattice (Sec. 2.1).  The solvers are the ones the paper names in
 * its abstract and in the feature list of Sec. 2: QXD_SOLVER_EO_GCR is GCR on
 * the even-odd preconditioned D^ of Sec. 2.4 with psi_o reconstructed from
 * psi_e; QXD_SOLVER_SAP_GCR is flexible GCR right-preconditioned by the
 * Schwarz alternating procedure (qxd_sap_apply) inside an FP64 defect
 * correction; QXD_SOLVER_DFL_SAP_GCR is the same with the deflated
 * preconditioner of qxd_dfl_setup (one right-hand side at a time; QXD_EINVAL
 * if no subspace was built for the quark).
 * quarks as in qxd_dirac_apply.  psi_dev is the initial guess if use_guess,
 * else it is overwritten.  info: nrhs entries (may be NULL).  Returns
 * QXD_ENOCONV if any right-hand side missed tol (best iterate written),
 * QXD_EFLOAT on NaN/Inf.  Synchronises `stream`. */
qxd_status qxd_solve(qxd_field *field, const qxd_quark *quarks, int nquark,
                     const qxd_solver *s, const double *eta_dev, double *psi_dev,
                     int nrhs, int use_guess, qxd_solve_info *info, void *stream);

/* Parameters of the local deflation of the SAP-GCR (QXD_SOLVER_DFL_SAP_GCR).
 * Zero means the default given in brackets. */
typedef struct {
  int ns;             /* deflation fields, i.e. basis vectors per SAP block
                         (1..32) [16]                                          */
  int ninv;           /* SAP-smoothed inverse-iteration steps that refine the
                         random start fields [30]                              */
  int ncy, nmr;       /* SAP cycles and MR steps of each such step [4, 4]      */
  double little_tol;  /* relative residual of each little-system solve [0.2]  */
  int little_nkv;     /* Krylov vectors of the little GCR (<= 64) [48]         */
  int little_maxiter; /* iterations of one little solve [256]                  */
  uint64_t seed;      /* seed of the random start fields                       */
} qxd_dfl_params;

/* Build the deflation subspace of the locally deflated SAP-GCR (the solver
 * the paper inherits and uses for its most expensive factors: abstract,
 * Sec. 2 feature list, Appendix A, Table 2) for one quark on this field, and
 * its little Dirac operator:
 *   - ns global fields, random (or the caller's start fields init_dev: ns
 *     API-layout FP64 spinors, may be NULL), each refined by ninv steps
 *     psi <- M_sap psi / |M_sap psi| with the Schwarz preconditioner (ncy,
 *     nmr; FP32 storage) standing in for D^-1;
 *   - on every SAP block the restricted fields are orthonormalised by
 *     modified Gram-Schmidt in the order of the fields: the subspace has ns
 *     basis vectors per block (stored FP32);
 *   - the little operator A = V^dag D V on it (V: coefficients -> fields),
 *     assembled in FP64: per block its ns x ns couplings to itself and to
 *     its eight neighbours.
 * A later qxd_solve with QXD_SOLVER_DFL_SAP_GCR for this quark then uses the
 * preconditioner M_dfl r = V A^-1 V^dag r + M_sap (r - D V A^-1 V^dag r),
 * with A^-1 applied by GCR on the even-block Schur complement of A (blocks
 * coloured as for SAP), right-preconditioned by the inverse diagonal blocks,
 * to little_tol, with FP16 copies of the little matrices when little_tol is
 * 1e-2 or more (the default) and FP32 copies otherwise (the inverse diagonal
 * blocks in FP32 either way).
 * A new call for the same quark replaces the subspace.  The subspace lives
 * with the quark's operator in the field's operator cache (freed with it).
 * Needs SAP blocks of at most 256 sites that admit the two-colour
 * decomposition.  Synchronises `stream`. */
qxd_status qxd_dfl_setup(qxd_field *field, const qxd_quark *quark, const qxd_dfl_params *params,
                         const double *init_dev, void *stream);

/* Multi-shift conjugate gradient (the paper's solver for the factors of the
 * rational approximation, feature list of Sec. 2 and Table 2): solves
 *     (D^dag D^ + mu^2 + shifts[j]) psi_j = eta_e,   j < nshift,
 * on the even sites for one quark (mu its twisted mass, Sec. 2.4), all shifts
 * in one Krylov space: CG on the smallest shift, the others from the
 * collinear residuals.  FP64 throughout.  eta_dev: one API-layout FP64
 * spinor (its odd sites are ignored); psi_dev: nshift API-layout FP64
 * spinors, written with zero odd sites.  shifts >= 0, 1 <= nshift <= 64.
 * Shift j stops once its residual |eta_e - (X + shift_j) psi_j| <= tol
 * |eta_e| (X = D^dag D^ + mu^2); info (nshift entries, may be NULL) gets each
 * shift's iterations and true FP64 residual.  QXD_ENOCONV if maxiter (0:
 * 100000) ends first (iterates written).  Synchronises `stream`. */
qxd_status qxd_multishift_solve(qxd_field *field, const qxd_quark *quark, const double *shifts, int nshift,
                                double tol, int maxiter, const double *eta_dev, double *psi_dev,
                                qxd_solve_info *info, void *stream);

/* Rational function of the even-odd normal operator (Sec. 2.4):
 *     out_e = A prod_{j<n} (X + nu_j^2) / (X + mu_j^2) eta_e,  X = D^dag D^ + mu^2
 * (mu the quark's twisted mass), evaluated as A (eta_e + sum_j rho_j (X +
 * mu_j^2)^-1 eta_e) with the partial-fraction residues rho_j and one
 * multi-shift CG over the poles.  A whole approximation R (Table 2) or one
 * frequency-splitting factor P_k (A = 1 and the zeros and poles of its index
 * range) or a twisted-mass Hasenbusch ratio (n = 1) are all of this form.
 * The mu_j must be distinct; 1 <= n <= 64.  tol, maxiter, info (n entries,
 * one per pole) as for qxd_multishift_solve.  eta_dev, out_dev: API-layout
 * FP64 spinors (odd sites of eta ignored, of out set to 0).  Synchronises
 * `stream`. */
qxd_status qxd_rational_apply(qxd_field *field, const qxd_quark *quark, double A, const double *nu,
                              const double *mu, int n, double tol, int maxiter, const double *eta_dev,
                              double *out_dev, qxd_solve_info *info, void *stream);

/* Apply the SAP preconditioner M_SAP of the SAP_GCR solver (the Schwarz
 * preconditioner the paper's SAP-GCR is named after, abstract and Sec. 2):
 * ncy cycles of black and white block solves, each by nmr minimal-residual
 * steps on the even-odd (Sec. 2.4) block operator with Dirichlet faces, to
 * nrhs API-layout FP64 spinors, computing in precision prec with the field's
 * blocks.  out = M in.
 * Asynchronous on `stream`. */
qxd_status qxd_sap_apply(qxd_field *field, const qxd_quark *quark, qxd_prec prec, int ncy,
                         int nmr, const double *in_dev, double *out_dev, int nrhs, void *stream);

/* ---- serving: continuous batching of solve requests ------------------- */

typedef struct {
  qxd_field *field;        /* resident gauge field                           */
  qxd_quark quark;         /* operator of every right-hand side              */
  qxd_solver solver;       /* solver parameters                              */
  const double *eta_dev;   /* nrhs API-layout FP64 sources (device)          */
  double *psi_dev;         /* nrhs API-layout FP64 solutions (device)        */
  int nrhs;
} qxd_request;

typedef struct {
  int status;              /* qxd_status of the request                      */
  int nrhs;
  double latency_s;        /* submit -> completion                            */
  double queue_s;          /* submit -> admission                             */
  int inner_iters;         /* max over right-hand sides                       */
  double true_resid;       /* max over right-hand sides                       */
} qxd_result;

/* Start the serving scheduler of ctx with a device-memory budget (bytes);
 * 0 means 70% of the device memory free at this call.  Charged against it:
 * per group of requests (same field, inner precision and solver parameters)
 * the larger of the solver workspaces the group holds and those its admitted
 * right-hand sides need; the operators (clover term, its inverse, hopping
 * links) the fields build or keep cached beyond what they held when their
 * first request arrived; and for every admitted request whose operator is
 * not built yet, that operator until it is built.  Requests are admitted in
 * arrival order, each right-hand side while the charge fits and the
 * device's free memory, less what admitted work has still to allocate,
 * covers its allocations plus a floor of 4 GiB + 2% of the device; a
 * request that does not fit whole is admitted in pieces (later requests
 * wait until all of its right-hand sides are in); one right-hand side always
 * runs when no other work is charged (QXD_ENOMEM as the request's status if
 * the device cannot hold it).  max_active (0 = no limit) caps the
 * right-hand sides in flight. */
qxd_status qxd_serve_start(qxd_ctx *ctx, size_t budget_bytes, int max_active);

/* Queue a request; *ticket identifies it.  Buffers must stay valid until
 * qxd_serve_poll reports completion. */
qxd_status qxd_serve_submit(qxd_ctx *ctx, const qxd_request *req, uint64_t *ticket);

/* QXD_EBUSY while pending; otherwise fills *out (status of the solve) and
 * forgets the ticket; if the request failed, qxd_last_error() of the calling
 * thread then says why.  QXD_ENOTFOUND for unknown tickets. */
qxd_status qxd_serve_poll(qxd_ctx *ctx, uint64_t ticket, qxd_result *out);

/* Stop the scheduler after finishing admitted requests. */
qxd_status qxd_serve_stop(qxd_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* QXD_H */
