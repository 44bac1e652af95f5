// Device kernels of the DG-BGK library and their launch parameters.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace dgbgk {

constexpr int kMaxP = 8;
constexpr int kMaxN1 = kMaxP + 1;
constexpr int kBlock = 256;  // threads per work-group of the stage kernel
constexpr int kStreamDoubles = 16;  // f doubles per thread and block in the persistent kernel
constexpr int kStreamMaxP = 3;      // higher orders hold too many nodal values per row

// Everything one launch of the fused RK-stage kernel needs.  Passed by value:
// the reference-element tables ride in the kernel-argument segment.
// Device states are element-major, f[k][q][n] (element k, velocity q, node n).
struct StageArgs {
  const double *fs;    // stage input state f_s[k][q][n]
  const double *fn;    // state at the start of the step f_n
  double *acc;         // RK4 accumulator
  double *out;         // stage output (f_{s+1}, f_{n+1}, or L(f_s) when stage 0)
  const double *vel;   // [3][Q]: e_x, e_y, w
  const double *feqb;  // [4][Q]: f^eq_q(1, u_b) of each side's wall velocity
  const double *mom;   // [3][K*Np]: rho, ux, uy  (tiled mode only)
  const double *rhow;  // [K][4][Nfp]: diffuse-wall densities (tiled mode only)
  const double *wmom;  // [Q][16]: moment weights 1, e_x, e_y, outgoing |e.n| per side, 0...
  double *rhow_out;    // optional [K][4][Nfp] copy of the wall densities (fused mode)
  // velocity-tiled mode: moment partials [tile][K][7][Np] (rho, rho u_x, rho u_y
  // and the outgoing wall fluxes summed over each velocity tile).  pin: those
  // of fs, read instead of mom / rhow (NULL: use mom / rhow); pout: those of
  // out, written by stages 1..4 (NULL: none).
  const double *pin;
  double *pout;
  double D1[kMaxN1 * kMaxN1];  // 1-D GLL differentiation matrix
  double lift_lo[kMaxN1];      // M1^{-1} e_0: lift of a flux on the left / bottom face
  double lift_hi[kMaxN1];      // M1^{-1} e_p: lift of a flux on the right / top face
  double rx, sy;               // 2/hx, 2/hy (reference-to-physical derivative scale)
  double fsx, fsy;             // face-to-volume Jacobian ratio of x-faces / y-faces
  double theta_inv;            // 1/theta
  double half_theta2_inv;      // 1/(2 theta^2)
  double half_theta_inv;       // 1/(2 theta)
  double inv_tau;              // 1/tau (0 for tau = +inf)
  double wall_den_inv[4];      // 1 / sum_{e.n<0} |e.n| f^eq(1,u_b) per side
  double c_acc, c_out;         // RK4 coefficients of this stage (times dt)
  int nx, ny, K, Q;
  int E, log2E;                // elements per work-group (power of two)
  int Qt;                      // velocities per work-group
  int nblk;                    // element blocks (grid x)
  int stage;                   // 0: out = L(f_s); 1..4: classical RK4 stage
  int wall_mask;               // bit s: side s is a diffuse wall
  int periodic_x, periodic_y;
  int fused;                   // 1: moments and wall densities computed in-block
  int stream_nt;               // 1: x and the accumulator move with non-temporal hints
};

// Velocity tiles for which the tiled stage kernels exchange moment partials.
constexpr int kMaxPartialTiles = 4;

// LDS bytes of the stage kernel for (p, E, Qt).
size_t stage_lds_bytes(int p, int E, int Qt);

hipError_t launch_stage(int p, const StageArgs &a, size_t lds_bytes, int ntiles,
                        hipStream_t stream);

// Batched stage: problems of order p (fused blocks), one work item per
// (problem, element block) in items (.x problem index into descs, .y block);
// groups work-groups stride over the items.  descs (device) must hold the
// stage's arguments of every problem for the duration of the launch.
hipError_t launch_batch_stage(int p, int stage, const StageArgs *descs, const int2 *items,
                              int nitems, size_t lds_bytes, int groups, hipStream_t stream);

// The persistent pipelined stage kernel applies to fused blocks with at most
// kBlock velocity rows (E * Q) and at most kStreamDoubles * kBlock f values,
// p <= kStreamMaxP, and f arrays below 4 GiB (32-bit offsets).
bool stream_applicable(int p, int E, int Q, int64_t K);
size_t stream_lds_bytes(int p, int E, int Q);
hipError_t launch_stream(int p, const StageArgs &a, size_t lds_bytes, int groups,
                         hipStream_t stream);

// rho, ux, uy of f at every node (any output may be null) and, when rhow is
// non-null, the diffuse-wall densities of every wall face node.
hipError_t launch_moments(const double *f, const double *vel, int K, int p, int Q, int nx,
                          int ny, int wall_mask, const double *wall_den_inv4, double *rho,
                          double *ux, double *uy, double *rhow, hipStream_t stream);

// Whether one-element fused work-groups of order p hand the moments of their
// output to the next stage (a.pin / a.pout of the fused form).
__host__ __device__ constexpr bool handoff_moments(int p) { return p == 1 || p == 3; }

// Moment rows of an FP64 state (element-major): out[k][7][Np] = sum over
// velocities of (1, e_x, e_y, outgoing normal speed at the bottom, right, top,
// left wall) times f, the input moments of the stages that read them (a.pin),
// then zeros in the slots of tiles 1..ntiles-1.
hipError_t launch_moment_rows(const double *f, const double *vel, int K, int Np, int Q, int ntiles,
                              double *out, hipStream_t stream);

// Scaled max-norm of the moment rates of k = L(f): atomically max-reduced into
// *result (bit pattern of a non-negative double; must be zeroed first).
hipError_t launch_residual(const double *k, const double *vel, int K, int Np, int Q,
                           double scale, unsigned long long *result, hipStream_t stream);

// f_q = f_q^eq(rho0, u0) everywhere.
hipError_t launch_init_equilibrium(double *f, const double *vel, int K, int Np, int Q,
                                   double rho0, double ux0, double uy0, double theta,
                                   hipStream_t stream);

// f[q][k][n] -> f[k][q][n] (to_element_major = 1) or back (0).
hipError_t launch_transpose(const double *src, double *dst, int K, int Np, int Q,
                            int to_element_major, hipStream_t stream);

hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v,
                           hipStream_t stream);

hipError_t launch_u64_to_f64(const unsigned long long *src, double *dst, hipStream_t stream);

}  // namespace dgbgk
