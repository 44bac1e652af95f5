// Vector kernels of the implicit time step (FP64 vectors; the Krylov basis in
// FP64 or FP32): a fused linear combination,
// a deterministic multi-vector dot product (Gram-Schmidt projections of the
// Krylov basis) and the matching multi-vector update with scaling.  All are HBM-bound
// streams; the dot kernel reads w once per four basis vectors.
#include "linalg.hpp"

namespace dgbgk {

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;     // elements per thread per pass of the dot kernel
constexpr int kVecs = 4;      // basis vectors per dot work-group
constexpr int kMaxGroups = 1024;

__global__ __launch_bounds__(kBlock) void lincomb_kernel(size_t n, double a, const double *x, double b,
                                                         const double *y, double c, const double *z,
                                                         double *out) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double v = x ? a * x[i] : 0.0;
    if (y) v += b * y[i];
    if (z) v += c * z[i];
    out[i] = v;
  }
}

// out = a x + b y + c z with y in FP32 (a Krylov vector of the FP32 basis).
__global__ __launch_bounds__(kBlock) void lincomb_mixed_kernel(size_t n, double a, const double *x,
                                                               double b, const float *y, double c,
                                                               const double *z, double *out) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double v = x ? a * x[i] : 0.0;
    if (y) v += b * (double)y[i];
    if (z) v += c * z[i];
    out[i] = v;
  }
}

// Sum of v over the work-group, valid in thread 0; red is reusable on return.
__device__ inline double block_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// Work-group (g, j) sums V_k . w for k = kVecs j ... kVecs j + kVecs - 1 over
// the chunks g, g + G, g + 2G, ... of kBlock * kItems elements.
__global__ __launch_bounds__(kBlock) void multi_dot_partial_kernel(size_t n, int nv, const double *V,
                                                                   size_t vstride, const double *w,
                                                                   double *partial) {
  __shared__ double red[kBlock / 64];
  const int k0 = blockIdx.y * kVecs;
  const int G = gridDim.x;
  double acc[kVecs];
#pragma unroll
  for (int t = 0; t < kVecs; ++t) acc[t] = 0.0;
  // two consecutive elements per access (16-byte loads)
  const size_t chunk = (size_t)kBlock * kItems * 2;
  for (size_t base = (size_t)blockIdx.x * chunk; base < n; base += (size_t)G * chunk) {
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const size_t i = base + 2 * ((size_t)it * kBlock + threadIdx.x);
      if (i + 1 < n) {
        const double2 wi = *reinterpret_cast<const double2 *>(w + i);
#pragma unroll
        for (int t = 0; t < kVecs; ++t)
          if (k0 + t < nv) {
            const double2 v = *reinterpret_cast<const double2 *>(V + (size_t)(k0 + t) * vstride + i);
            acc[t] += v.x * wi.x + v.y * wi.y;
          }
      } else if (i < n) {
        const double wi = w[i];
#pragma unroll
        for (int t = 0; t < kVecs; ++t)
          if (k0 + t < nv) acc[t] += V[(size_t)(k0 + t) * vstride + i] * wi;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kVecs; ++t) {
    const double s = block_sum(acc[t], red);
    if (threadIdx.x == 0 && k0 + t < nv) partial[(size_t)(k0 + t) * G + blockIdx.x] = s;
  }
}

// The FP32-basis form: as above with two consecutive elements per access
// (float2 basis loads, double2 loads of w), and vector nv taken as w itself.
__global__ __launch_bounds__(kBlock) void multi_dot32_partial_kernel(size_t n, int nv, const float *V,
                                                                     size_t vstride, const double *w,
                                                                     double *partial) {
  __shared__ double red[kBlock / 64];
  const int k0 = blockIdx.y * kVecs;
  const int G = gridDim.x;
  double acc[kVecs];
#pragma unroll
  for (int t = 0; t < kVecs; ++t) acc[t] = 0.0;
  const size_t chunk = (size_t)kBlock * kItems * 2;
  for (size_t base = (size_t)blockIdx.x * chunk; base < n; base += (size_t)G * chunk) {
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const size_t i = base + 2 * ((size_t)it * kBlock + threadIdx.x);
      if (i + 1 < n) {
        const double2 wi = *reinterpret_cast<const double2 *>(w + i);
#pragma unroll
        for (int t = 0; t < kVecs; ++t) {
          if (k0 + t < nv) {
            const float2 v = *reinterpret_cast<const float2 *>(V + (size_t)(k0 + t) * vstride + i);
            acc[t] += (double)v.x * wi.x + (double)v.y * wi.y;
          } else if (k0 + t == nv) {
            acc[t] += wi.x * wi.x + wi.y * wi.y;
          }
        }
      } else if (i < n) {
        const double wi = w[i];
#pragma unroll
        for (int t = 0; t < kVecs; ++t) {
          if (k0 + t < nv) acc[t] += (double)V[(size_t)(k0 + t) * vstride + i] * wi;
          else if (k0 + t == nv) acc[t] += wi * wi;
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kVecs; ++t) {
    const double s = block_sum(acc[t], red);
    if (threadIdx.x == 0 && k0 + t <= nv) partial[(size_t)(k0 + t) * G + blockIdx.x] = s;
  }
}

// Work-group k sums the G partials of vector k in a fixed order.
__global__ __launch_bounds__(kBlock) void multi_dot_final_kernel(int G, const double *partial,
                                                                 double *result) {
  __shared__ double red[kBlock / 64];
  const double *p = partial + (size_t)blockIdx.x * G;
  double acc = 0.0;
  for (int g = threadIdx.x; g < G; g += kBlock) acc += p[g];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) result[blockIdx.x] = s;
}

// Two consecutive elements per thread (16-byte loads).
__global__ __launch_bounds__(kBlock) void multi_axpy_kernel(size_t n, int nv, const double *V,
                                                            size_t vstride, const double *coef,
                                                            double alpha, const double *w,
                                                            double scale, double *out) {
  const size_t stride = 2 * (size_t)gridDim.x * blockDim.x;
  for (size_t i = 2 * ((size_t)blockIdx.x * blockDim.x + threadIdx.x); i < n; i += stride) {
    if (i + 1 < n) {
      double s0 = 0.0, s1 = 0.0;
      for (int k = 0; k < nv; ++k) {
        const double2 v = *reinterpret_cast<const double2 *>(V + (size_t)k * vstride + i);
        s0 += coef[k] * v.x;
        s1 += coef[k] * v.y;
      }
      const double2 wi = *reinterpret_cast<const double2 *>(w + i);
      double2 r;
      r.x = scale * (wi.x + alpha * s0);
      r.y = scale * (wi.y + alpha * s1);
      *reinterpret_cast<double2 *>(out + i) = r;
    } else {
      double s0 = 0.0;
      for (int k = 0; k < nv; ++k) s0 += coef[k] * V[(size_t)k * vstride + i];
      out[i] = scale * (w[i] + alpha * s0);
    }
  }
}

// The FP32-basis form, two consecutive elements per thread (float2 basis
// loads); out32 (optional) receives out rounded to FP32.
__global__ __launch_bounds__(kBlock) void multi_axpy32_kernel(size_t n, int nv, const float *V,
                                                              size_t vstride, const double *coef,
                                                              double alpha, const double *w,
                                                              double scale, double *out, float *out32) {
  const size_t stride = 2 * (size_t)gridDim.x * blockDim.x;
  for (size_t i = 2 * ((size_t)blockIdx.x * blockDim.x + threadIdx.x); i < n; i += stride) {
    if (i + 1 < n) {
      double s0 = 0.0, s1 = 0.0;
      for (int k = 0; k < nv; ++k) {
        const float2 v = *reinterpret_cast<const float2 *>(V + (size_t)k * vstride + i);
        s0 += coef[k] * (double)v.x;
        s1 += coef[k] * (double)v.y;
      }
      const double2 wi = *reinterpret_cast<const double2 *>(w + i);
      double2 r;
      r.x = scale * (wi.x + alpha * s0);
      r.y = scale * (wi.y + alpha * s1);
      *reinterpret_cast<double2 *>(out + i) = r;
      if (out32) {
        float2 r32;
        r32.x = (float)r.x;
        r32.y = (float)r.y;
        *reinterpret_cast<float2 *>(out32 + i) = r32;
      }
    } else {
      double s0 = 0.0;
      for (int k = 0; k < nv; ++k) s0 += coef[k] * (double)V[(size_t)k * vstride + i];
      const double r = scale * (w[i] + alpha * s0);
      out[i] = r;
      if (out32) out32[i] = (float)r;
    }
  }
}

int dot_groups(size_t n) {
  const size_t chunk = (size_t)kBlock * kItems;
  size_t g = (n + chunk - 1) / chunk;
  if (g < 1) g = 1;
  return (int)(g > (size_t)kMaxGroups ? kMaxGroups : g);
}

unsigned stream_blocks(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (unsigned)(b > 8192 ? 8192 : b);
}

}  // namespace

hipError_t launch_lincomb(size_t n, double a, const double *x, double b, const double *y, double c,
                          const double *z, double *out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(lincomb_kernel, dim3(stream_blocks(n)), dim3(kBlock), 0, st, n, a, x, b, y, c,
                     z, out);
  return hipGetLastError();
}

size_t multi_dot_scratch(size_t n, int nv) { return (size_t)dot_groups(n) * (size_t)nv; }

hipError_t launch_multi_dot(size_t n, int nv, const double *V, size_t vstride, const double *w,
                            double *scratch, double *result, hipStream_t st) {
  if (nv < 1 || nv > kMaxBasis) return hipErrorInvalidValue;
  const int G = dot_groups((n + 1) / 2);  // within multi_dot_scratch(n, nv)
  const unsigned gy = (unsigned)((nv + kVecs - 1) / kVecs);
  hipLaunchKernelGGL(multi_dot_partial_kernel, dim3((unsigned)G, gy), dim3(kBlock), 0, st, n, nv, V,
                     vstride, w, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(multi_dot_final_kernel, dim3((unsigned)nv), dim3(kBlock), 0, st, G, scratch,
                     result);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(size_t n, int nv, const double *V, size_t vstride, const double *coef,
                             double alpha, const double *w, double scale, double *out,
                             hipStream_t st) {
  if (nv < 0 || nv > kMaxBasis) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(stream_blocks((n + 1) / 2)), dim3(kBlock), 0, st, n, nv,
                     V, vstride, coef, alpha, w, scale, out);
  return hipGetLastError();
}

hipError_t launch_lincomb_mixed(size_t n, double a, const double *x, double b, const float *y,
                                double c, const double *z, double *out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(lincomb_mixed_kernel, dim3(stream_blocks(n)), dim3(kBlock), 0, st, n, a, x, b, y,
                     c, z, out);
  return hipGetLastError();
}

hipError_t launch_multi_dot32(size_t n, int nv, const float *V, size_t vstride, const double *w,
                              double *scratch, double *result, hipStream_t st) {
  if (nv < 0 || nv + 1 > kMaxBasis) return hipErrorInvalidValue;
  // half the groups of the FP64 form (two elements per access): within
  // the scratch that multi_dot_scratch(n, nv + 1) sizes
  const int G = dot_groups((n + 1) / 2);
  const int nt = nv + 1;
  const unsigned gy = (unsigned)((nt + kVecs - 1) / kVecs);
  hipLaunchKernelGGL(multi_dot32_partial_kernel, dim3((unsigned)G, gy), dim3(kBlock), 0, st, n, nv, V,
                     vstride, w, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(multi_dot_final_kernel, dim3((unsigned)nt), dim3(kBlock), 0, st, G, scratch,
                     result);
  return hipGetLastError();
}

hipError_t launch_multi_axpy32(size_t n, int nv, const float *V, size_t vstride, const double *coef,
                               double alpha, const double *w, double scale, double *out, float *out32,
                               hipStream_t st) {
  if (nv < 0 || nv > kMaxBasis) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(multi_axpy32_kernel, dim3(stream_blocks((n + 1) / 2)), dim3(kBlock), 0, st, n, nv,
                     V, vstride, coef, alpha, w, scale, out, out32);
  return hipGetLastError();
}

}  // namespace dgbgk
