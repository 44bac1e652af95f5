// Device kernels of the FP32-storage precision path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "kernels.hpp"

namespace dgbgk {

// One launch of the FP32 stage kernel.  The state arrays hold the deviation
// g = f - w_q rho_ref in FP32, element-major g[k][q][n]; the moments, the
// diffuse-wall densities and the wall exterior states are formed in FP64.
struct Stage32Args {
  const float *fs;      // stage input g_s
  const float *fn;      // g at the start of the step
  float *acc;           // RK4 accumulator (deviation form)
  float *out;           // stage output (g_{s+1}, g_{n+1}, or L(f_s) when stage 0)
  const double *vel;    // [3][Q]: e_x, e_y, w
  const double *feqb;   // [4][Q]: f^eq_q(1, u_b) of each side's wall velocity
  const double *wmom;   // [Q][16]: moment weights 1, e_x, e_y, outgoing |e.n| per side, 0...
  const uint16_t *dmat;  // [2 Np][32] bf16 rows of Dr and Ds (contraction variant only)
  double *rhow_out;     // optional [K][4][Nfp] copy of the wall densities
  // reference form (DGBGK_FP32_REF): the state is f = f_r + g with an FP64
  // reference f_r; rref = L(f_r) in FP32 ([k][q][n]), mref = rho, u_x, u_y of
  // f_r per node ([3][K Np], FP64).  NULL otherwise.
  const float *rref;
  const double *mref;
  // moments handed between stages (one-element blocks of orders 1 and 3): the
  // input's seven moment sums per node ([K][7][Np], FP64, of g) and the
  // output's, written by the update pass; NULL: the block reduces its own
  const double *pin;
  double *pout;
  float D1[kMaxN1 * kMaxN1];
  float lift_lo[kMaxN1], lift_hi[kMaxN1];
  float rx, sy, fsx, fsy;
  float theta_inv, half_theta2_inv, inv_tau;
  double half_theta_inv;
  double wall_den_inv[4];
  double mconst[7];      // rho_ref sum_q W[q][c] w_q: moments of the w_q rho_ref part of f
  double rho_ref;
  float c_acc, c_out;    // RK4 coefficients of this stage (times dt)
  int nx, ny, K, Q;
  int E;                 // elements per work-group
  int nblk;              // element blocks (grid x)
  int stage;             // 0: out = L(f_s); 1..4: classical RK4 stage
  int wall_mask;
  int periodic_x, periodic_y;
  int stream_nt;         // 1: x and the accumulator move with non-temporal hints
};

// Whether the bf16 matrix-core contraction variant is built for order p.
bool bf16_contraction_available(int p);

// Whether the reference form is built for order p (and contraction variant).
bool ref_form_available(int p, int contract);

// LDS bytes of the FP32 stage kernel for (p, E, Q).
size_t stage32_lds_bytes(int p, int E, int Q, bool bf16, bool ref);

// contract: 0 FP32 vector contractions, 1 BF16 matrix-core contractions of
// the volume term (FP32 accumulation).  ref: the reference form (a.rref,
// a.mref set).
hipError_t launch_stage32(int p, const Stage32Args &a, size_t lds_bytes, int contract, int ref,
                          hipStream_t stream);

// Batched FP32 stage over problems of order p with the same access width cw
// (4 when Q Np is a multiple of 4, else 1), contraction variant and form;
// items and descs as for launch_batch_stage.  ho: every member has one
// element per block and hands its moments between stages (a.pin, a.pout).
hipError_t launch_batch_stage32(int p, int stage, int cw, int contract, int ref, int ho,
                                const Stage32Args *descs, const int2 *items, int nitems,
                                size_t lds_bytes, int groups, hipStream_t stream);

// Reference form helpers (element-major arrays of n = K Np Q values):
// fold: f_r += g, g = 0;  to_f32: dst = (float) src;  sum: dst = f_r + g;
// from_ref: dst[q][k][n] (host order) = f_r + g;  to_ref: g = src (host
// order) - f_r.
hipError_t launch_ref_fold(double *fref, float *g, size_t n, hipStream_t stream);
hipError_t launch_f64_to_f32(const double *src, float *dst, size_t n, hipStream_t stream);
hipError_t launch_ref_sum(const double *fref, const float *g, double *dst, size_t n,
                          hipStream_t stream);
hipError_t launch_from_ref(const double *fref, const float *g, double *dst, int K, int Np, int Q,
                           hipStream_t stream);
hipError_t launch_to_ref(const double *src, const double *fref, float *g, int K, int Np, int Q,
                         hipStream_t stream);

// f (double, host order f[q][k][n]) <-> g (float, element-major), with
// g = f - offset * w_q (offset = rho_ref for states, 0 for rates).
hipError_t launch_to_dev32(const double *src, float *dst, const double *vel, int K, int Np, int Q,
                           double offset, hipStream_t stream);
hipError_t launch_from_dev32(const float *src, double *dst, const double *vel, int K, int Np, int Q,
                             double offset, hipStream_t stream);

// g = f^eq(rho0, u0) - w rho_ref everywhere.
hipError_t launch_init_equilibrium32(float *g, const double *vel, int K, int Np, int Q, double rho0,
                                     double ux0, double uy0, double theta, double rho_ref,
                                     hipStream_t stream);

// rho, ux, uy of f = g + w rho_ref at every node (FP64 sums).
hipError_t launch_moments32(const float *g, const double *vel, int K, int Np, int Q,
                            double rho_ref, double *rho, double *ux, double *uy, hipStream_t stream);

// Moment rows of an FP32 state g (element-major): out[k][7][Np] = sum over
// velocities of (1, e_x, e_y, outgoing normal speed at the bottom, right,
// top, left wall) times g, in FP64: the input moments of the stages that read
// them (a.pin).
hipError_t launch_moment_rows32(const float *g, const double *vel, int K, int Np, int Q, double *out,
                                hipStream_t stream);

// Residual of a rate k (float, element-major), as launch_residual.
hipError_t launch_residual32(const float *k, const double *vel, int K, int Np, int Q, double scale,
                             unsigned long long *result, hipStream_t stream);

}  // namespace dgbgk
