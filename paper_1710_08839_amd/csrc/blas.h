// Solver linear algebra on native spinors (blas.hip).  All reductions are in
// FP64 and deterministic (fixed grid, fixed summation order).
#pragma once

#include "launch.h"
#include "qxd_impl.h"

namespace qxd {

constexpr int RED_BLOCKS = 1024;  // work-groups of a reduction (upper bound)
constexpr int CHUNK = 8;          // vectors handled per multi-vector launch
constexpr int MAXV = 64;          // most vectors in one multi-dot / multi-axpy

template <int P>
struct VecList {
  Spinor<P> v[CHUNK];
};

// host description of z_t = src_t - sum_l coef[l] / div[l] * ys_t[l], t < ntriples
struct MaxpyHost {
  int n = 0;
  int ntriples = 1;
  SpinorArg src[2];
  SpinorArg dst[2];
  const SpinorArg *ys[2];
  const double *coef = nullptr;   // device, complex [n]
  const double *div = nullptr;    // device, real, element l at div[l * div_stride]
  int div_stride = 1;
  SpinorArg w{nullptr, 0, 0, RunDiv{}};     // optional: also (z_0, w)
};

// Streaming probe, the reference point for the kernels' bandwidth: per 48 KB
// chunk (12 planes of 4 KB) of dst (16-byte aligned, dst_bytes a multiple of
// 49152), plane p = xor of planes p, p + 12, ... of the 12 reads_per_write
// planes of the matching src chunk (reads_per_write 1, 2, 4, 7 or 8)
hipError_t launch_stream(const void *src, void *dst, size_t dst_bytes, int reads_per_write, hipStream_t st);

// Partial-sum scratch needed by any call: 3 * 2 * MAXV * RED_BLOCKS doubles
inline size_t blas_partial_doubles() { return (size_t)2 * MAXV * RED_BLOCKS + 8; }

// out[2l], out[2l+1] = (ys[l], x) [/ div[l*div_stride] if div]; complex results
template <int P>
hipError_t blas_mdot(const SpinorArg *ys, int n, SpinorArg x, int64_t first, int64_t count,
                     double *partial, double *out, const double *div, int div_stride, hipStream_t st);

// multi-axpy; if out != null: out[0] = |z_0|^2, out[1..2] = (z_0, w)
template <int P>
hipError_t blas_maxpy(const MaxpyHost &h, int64_t first, int64_t count, double *partial, double *out,
                      hipStream_t st);

// y -= (+-)(num/den) x; out[0] = |y|^2
template <int P>
hipError_t blas_update(SpinorArg y, SpinorArg x, const double *num, const double *den, int negate,
                       int64_t first, int64_t count, double *partial, double *out, hipStream_t st);

// y = a y + b x (precisions Q <- P); out[0] = |y|^2 if out != null
template <int Q, int P>
hipError_t blas_axpby(SpinorArg y, double a, SpinorArg x, double b, int64_t first, int64_t count,
                      double *partial, double *out, hipStream_t st);

// out[0] = |x|^2
template <int P>
hipError_t blas_norm2(SpinorArg x, int64_t first, int64_t count, double *partial, double *out,
                      hipStream_t st);

// Batched Gram-Schmidt step of the flexible GCR for many right-hand sides at
// once (one launch per phase for the whole batch; flat 16-byte streams, or
// one site per thread for FP16 + scale vectors with their per-site scales).
// For each slot, with k = slot.k:
//   ak_l = (chi_l, chi_k) / |chi_l|^2            (l < k; |chi_l|^2 = rec[3l])
//   chi_k -= sum_l ak_l chi_l                     (stored in place)
//   with passes = 2, once more (classical Gram-Schmidt with one
//   re-orthogonalisation against the stored vectors):
//     ak2_l = (chi_l, chi_k) / |chi_l|^2, chi_k -= sum_l ak2_l chi_l,
//     ak_l += ak2_l
//   rec[3k] = |chi_k|^2, rec[3k+1..2] = (chi_k, rho)
//   rho -= (rec[3k+1..2] / rec[3k]) chi_k,  *norm = |rho|^2
// Sums are FP64 over a grid fixed by the vector length, so a slot's results do
// not depend on the other slots of the batch.
template <int P>
struct GsSlot {
  typename St<P>::pair_t *chi0;  // chi_0 (full-lattice native vector)
  int64_t vstride_bytes;         // bytes from chi_l to chi_l+1
  typename St<P>::pair_t *rho;
  double *ak;                    // complex, l < k
  double *ak2;                   // second-pass coefficients (complex, l < k)
  double *rec;                   // 3 per vector
  double *norm;                  // |rho|^2 out
  int k;
};
// work-groups per slot of the batched kernels for vectors of nsites sites,
// and the partial-sum scratch they need for n slots
unsigned gs_batch_grid(int prec, int64_t nsites);
inline size_t gs_batch_partial_doubles(int n, int prec, int64_t nsites) {
  return (size_t)n * 2 * MAXV * gs_batch_grid(prec, nsites) + 8;
}
template <int P>
hipError_t blas_gs_batch(const GsSlot<P> *slots, int n, int64_t nsites, const RunDiv &rd, double *partial,
                         int passes, hipStream_t st);

}  // namespace qxd
