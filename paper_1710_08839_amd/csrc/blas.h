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

}  // namespace qxd
