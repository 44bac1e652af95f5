// Initial states from node moments: the equilibrium of eq. (5) with each
// node's own density and velocity, written in the element-major device
// layout f[k][q][n].
#include "init.hpp"

namespace dgbgk {

namespace {

__device__ inline double feq_node(const double *vel, const double *mom, size_t KNP, size_t node, int Q,
                                  int q, double theta) {
  const double rho = mom[node], ux = mom[KNP + node], uy = mom[2 * KNP + node];
  const double cx = vel[q], cy = vel[Q + q], w = vel[2 * Q + q];
  const double eu = cx * ux + cy * uy, usq = ux * ux + uy * uy;
  return w * rho * (1.0 + eu / theta + eu * eu / (2.0 * theta * theta) - usq / (2.0 * theta));
}

// Thread (node, q): node = k Np + n in x, velocity q in y.
__global__ __launch_bounds__(256) void init_moments_kernel(double *f, const double *vel, const double *mom,
                                                           size_t KNP, int Np, int Q, double theta) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= KNP) return;
  f[((i / Np) * Q + q) * Np + i % Np] = feq_node(vel, mom, KNP, i, Q, q, theta);
}

__global__ __launch_bounds__(256) void init_moments32_kernel(float *g, const double *vel, const double *mom,
                                                             size_t KNP, int Np, int Q, double theta,
                                                             double rho_ref) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= KNP) return;
  const double w = vel[2 * Q + q];
  g[((i / Np) * Q + q) * Np + i % Np] = (float)(feq_node(vel, mom, KNP, i, Q, q, theta) - w * rho_ref);
}

}  // namespace

hipError_t launch_init_moments(double *f, const double *vel, const double *mom, int K, int Np, int Q,
                               double theta, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  if (KNP == 0 || Q <= 0) return hipSuccess;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(init_moments_kernel, grid, dim3(256), 0, st, f, vel, mom, KNP, Np, Q, theta);
  return hipGetLastError();
}

hipError_t launch_init_moments32(float *g, const double *vel, const double *mom, int K, int Np, int Q,
                                 double theta, double rho_ref, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  if (KNP == 0 || Q <= 0) return hipSuccess;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(init_moments32_kernel, grid, dim3(256), 0, st, g, vel, mom, KNP, Np, Q, theta,
                     rho_ref);
  return hipGetLastError();
}

}  // namespace dgbgk
