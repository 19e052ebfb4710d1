/* Testing hooks of libqxd (not needed by applications).
 *
 * The Dirac kernels come in several variants that compute the same operator
 * (Sec. 2.3 of the openQ*D paper) up to the order of floating-point
 * additions: the number of hops whose loads are issued together (1, 2, 4 or
 * 8), whether the input spinors of a lattice block are first staged in
 * LDS, and whether the Pauli term and the output are streamed with
 * non-temporal loads and stores, and whether the links of the C* mirror half
 * are read at their physical partners.  An autotuner picks the fastest variant per (precision, kernel,
 * lattice volume) on first use.  Tests force each variant in turn to check
 * all of them against the reference.
 */
#ifndef QXD_DEBUG_H
#define QXD_DEBUG_H

#include "qxd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Force the Dirac kernel variant of every later application in this process:
 * choice = group (1, 2, 4 or 8), plus 16 for the LDS-staged variant (ignored
 * where a block does not fit one work-group), plus 32 for non-temporal Pauli
 * and output streams, plus 64 for mirror-fused link reads on C* lattices
 * (links of the mirror half read at the physical partner and conjugated,
 * Sec. 2.1), plus 128 for wavefront-uniform addressing on 4^4 blocks (the
 * neighbour blocks, boundary signs and C* shifts of each hop computed once
 * per wavefront; ignored on other block shapes); 32, 64 and 128 with the
 * LDS-staged variant only; 0 returns to the autotuner.
 * Process-wide; not synchronised with applications in flight on other
 * threads.  QXD_EINVAL for any other value. */
qxd_status qxd_debug_set_dirac_variant(int choice);

/* Batched SAP-GCR steps replay the fixed launch sequence of a step (block
 * solves of every colour pass and the batched D) from a HIP graph captured
 * the second time a batch configuration occurs.  enable = 0 issues every
 * launch directly instead (the results are the same bits); process-wide. */
qxd_status qxd_debug_set_step_graphs(int enable);

/* Classical Gram-Schmidt passes per step of the batched SAP-GCR (qxd_solve
 * with QXD_SOLVER_SAP_GCR, and the serve loop): 1 (the default) orthogonalises
 * the new direction chi_k = D phi_k once against the stored chi_l; 2 repeats
 * the projection against the stored vectors and adds the second coefficients
 * to the first (equal in exact arithmetic).  Applies to solvers created after
 * the call; process-wide.  QXD_EINVAL for any other value. */
qxd_status qxd_debug_set_gs_passes(int passes);

/* Process-wide totals since load: step graphs captured, and step graphs
 * launched (each capture is launched once at once, then replayed while its
 * configuration repeats).  QXD_EINVAL if either pointer is NULL. */
qxd_status qxd_debug_step_graph_counts(int64_t *captures, int64_t *replays);

/* Make the next n steps of the batched SAP-GCR solver (qxd_solve with
 * QXD_SOLVER_SAP_GCR, and the serve loop) fail with QXD_EDEVICE before any
 * device work; 0 cancels.  For testing the error paths: qxd_solve returns the
 * error with every unfinished right-hand side's info.status set to it, and a
 * serve request whose batch fails completes with that status (its psi is not
 * written).  Process-wide.  QXD_EINVAL for n < 0. */
qxd_status qxd_debug_fail_steps(int n);

/* Measurement hook: time one colour pass (the blocks of colour 0, with the
 * face update) of the SAP block solver that the batched SAP-GCR runs on pairs
 * of right-hand sides sharing an operator, for npair pairs of synthetic
 * vectors in storage precision prec (QXD_F32, QXD_F16S or QXD_BF16), with nmr
 * MR steps per block; *ms receives the average over reps launches, timed
 * with HIP events on `stream`.  Builds the quark's operator if needed;
 * allocates its vectors on the field.  Synchronises `stream`. */
qxd_status qxd_debug_sap_pair_pass(qxd_field *field, const qxd_quark *quark, qxd_prec prec, int nmr, int npair,
                                   int reps, float *ms, void *stream);

/* Streaming probe on the current device, the practical bandwidth ceiling the
 * benchmark reports next to the kernels, shaped like the spinor traffic of
 * the block-major fields.  dst is cut into chunks of 12 planes of 4 KB, src
 * into chunks of 12 r planes (r = reads_per_write: 1, 2 or 4 to 8); plane p
 * of dst chunk c is the bytewise xor of planes p, p + 12, ..., p + 12 (r - 1)
 * of src chunk c, with non-temporal loads and stores, so r bytes are read
 * per byte written (the FP64 Dirac operator reads about 7 per byte it
 * writes, 5.5 with the mirror-fused link reads).  src holds r * dst_bytes bytes; both buffers are device memory,
 * 16-byte aligned and disjoint; dst_bytes a multiple of 49152 (QXD_EINVAL
 * otherwise).  Asynchronous on `stream` (a hipStream_t, NULL =
 * default stream). */
qxd_status qxd_debug_stream(const void *src_dev, void *dst_dev, size_t dst_bytes, int reads_per_write,
                            void *stream);

/* The serve loop's memory accounting on ctx (a snapshot): out[0] = operator
 * bytes that admitted requests have still to build, out[1] = operator bytes
 * the fields of its requests hold beyond what they held when first seen,
 * out[2] = solver slot bytes charged to its groups, out[3] = the budget.
 * QXD_EINVAL if out is NULL or serving is not started on ctx. */
qxd_status qxd_debug_serve_charges(qxd_ctx *ctx, size_t out[4]);

/* Deflation subspace that qxd_dfl_setup built for this quark: basis field k
 * (its basis vector k on every SAP block) as one API-layout FP64 spinor on
 * the device.  QXD_EINVAL if no subspace was built or k is out of range.
 * Synchronises `stream`. */
qxd_status qxd_debug_dfl_basis(qxd_field *field, const qxd_quark *quark, int k, double *out_dev, void *stream);

/* Its little operator, copied to host memory: with the blocks numbered
 * ((B0 nb1 + B1) nb2 + B2) nb3 + B3 over the extended lattice,
 * a[2 (((b * 9 + d) * ns + k) * ns + l)] (re, im) = (phi_{b,k}, D phi_{n,l})
 * restricted to the couplings of slot d, n = nbr[b * 9 + d]: d = 0 the
 * couplings inside block b (n = b), d = 1 + 2 mu + s those through the
 * face of b in direction mu, forward (s = 0) or backward (s = 1), n the
 * block across it (the same block may appear in several slots).  a and nbr
 * may be NULL to read *ns and *nblocks only.  QXD_EINVAL if no subspace was
 * built. */
qxd_status qxd_debug_dfl_little(qxd_field *field, const qxd_quark *quark, int *ns, int *nblocks, double *a,
                                int *nbr);

/* Counters of the deflated preconditioner of this quark since the last call
 * (then reset): out[0] applications, out[1] little-system GCR iterations in
 * total, out[2] the most iterations of one little solve.  QXD_EINVAL if no
 * subspace was built. */
qxd_status qxd_debug_dfl_stats(qxd_field *field, const qxd_quark *quark, int64_t out[3]);

/* out = M_dfl in for one API-layout FP64 spinor: the deflated preconditioner
 * of the DFL_SAP_GCR solver (FP32 storage inside), with the little system
 * solved to relative residual little_tol (0: the setup's) and ncy, nmr SAP
 * cycles and MR steps.  Synchronises `stream`. */
qxd_status qxd_debug_dfl_precond(qxd_field *field, const qxd_quark *quark, double little_tol, int ncy, int nmr,
                                 const double *in_dev, double *out_dev, void *stream);

/* The variant the autotuner chose for the full operator D (phase folded into
 * the links) on this field's lattice in precision prec, in the encoding of
 * qxd_debug_set_dirac_variant; 0 if D has not been applied yet. */
qxd_status qxd_debug_get_dirac_variant(const qxd_field *field, qxd_prec prec, int *choice);

#ifdef __cplusplus
}
#endif

#endif
