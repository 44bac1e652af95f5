// Vector kernels of the implicit (Newton-Krylov) time step.  Every
// reduction has a fixed assignment of elements to work-groups and a fixed
// summation order for a given length, so results are bitwise reproducible.
// The multi-dot and multi-axpy kernels take two consecutive elements per
// access: their FP64 vectors must be 16-byte aligned, FP32 basis vectors
// (base and stride) 8-byte aligned.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace dgbgk {

// Most vectors one multi-dot or multi-axpy call takes.
constexpr int kMaxBasis = 72;

// out = a x + b y + c z; a term is skipped when its pointer is null.  out may
// alias any input (element-wise update).
hipError_t launch_lincomb(size_t n, double a, const double *x, double b, const double *y, double c,
                          const double *z, double *out, hipStream_t stream);

// Doubles of scratch that launch_multi_dot needs for length n and nv vectors.
size_t multi_dot_scratch(size_t n, int nv);

// result[k] = V_k . w for k < nv, V_k = V + k * stride (nv <= kMaxBasis).
// scratch holds multi_dot_scratch(n, nv) doubles; result is device memory.
hipError_t launch_multi_dot(size_t n, int nv, const double *V, size_t stride, const double *w,
                            double *scratch, double *result, hipStream_t stream);

// out = scale (w + alpha sum_{k < nv} coef[k] V_k), coef in device memory
// (nv <= kMaxBasis); out may alias w.
hipError_t launch_multi_axpy(size_t n, int nv, const double *V, size_t stride, const double *coef,
                             double alpha, const double *w, double scale, double *out,
                             hipStream_t stream);

// The same operations with the Krylov basis V stored in FP32 (w, coef and
// out stay FP64).  lincomb_mixed: out = a x + b y + c z with y in FP32.
hipError_t launch_lincomb_mixed(size_t n, double a, const double *x, double b, const float *y,
                                double c, const double *z, double *out, hipStream_t stream);

// result[k] = V_k . w for k < nv and result[nv] = w . w (nv + 1 <= kMaxBasis);
// scratch holds multi_dot_scratch(n, nv + 1) doubles.
hipError_t launch_multi_dot32(size_t n, int nv, const float *V, size_t stride, const double *w,
                              double *scratch, double *result, hipStream_t stream);

// out = scale (w + alpha sum_{k < nv} coef[k] V_k); out32, when not null,
// receives out rounded to FP32.  out may alias w.
hipError_t launch_multi_axpy32(size_t n, int nv, const float *V, size_t stride, const double *coef,
                               double alpha, const double *w, double scale, double *out,
                               float *out32, hipStream_t stream);

}  // namespace dgbgk
