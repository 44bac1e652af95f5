// Initial states from node moments (device kernels).
#pragma once

#include <hip/hip_runtime.h>

namespace dgbgk {

// f[k][q][n] = f^eq_q(rho, u) of eq. (5) at every node, from device arrays
// mom = [rho | ux | uy], each K*Np doubles (node k*Np + n).  vel: [3][Q]
// (e_x, e_y, w).  FP64 state.
hipError_t launch_init_moments(double *f, const double *vel, const double *mom, int K, int Np, int Q,
                               double theta, hipStream_t stream);

// The same for the FP32 deviation state g = f^eq - w rho_ref (f^eq in FP64).
hipError_t launch_init_moments32(float *g, const double *vel, const double *mom, int K, int Np, int Q,
                                 double theta, double rho_ref, hipStream_t stream);

}  // namespace dgbgk
