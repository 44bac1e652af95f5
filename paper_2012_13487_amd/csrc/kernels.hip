// Device kernels of the DG-BGK library (gfx950).
//
// The hot path is one fused kernel per RK4 stage.  A work-group owns a block
// of E consecutive elements and a tile of Qt velocities (Qt = Q in fused
// mode) and, in one pass over HBM:
//   1. stages f_s[q][k][n] of its block in LDS (coalesced: consecutive lanes
//      read consecutive nodes of one velocity row);
//   2. reduces the node moments rho, rho u (Sec. II.A) over the velocities in
//      LDS, and the diffuse-wall densities of eq. (8) at wall face nodes;
//      in tiled mode both come from a separate moments pass instead;
//   3. forms the upwind face jumps (e.n)(f^- - f^+) on inflow faces, with f^+
//      the neighbour trace or the wall exterior state rho_w f^eq(1, u_b);
//   4. per (velocity, node): volume term -e.grad f by the 1-D derivative
//      matrix along the node's grid line (sum factorisation of Dr = I x D1,
//      Ds = D1 x I), lift of the two inflow-face jumps (LIFT = M^{-1} E is a
//      rank-one outer product per face on tensor GLL elements), BGK collision
//      with the second-order equilibrium eq. (5), and the RK4 register update.
// The path is HBM-bound (about 2.5-5 flop per byte in FP64), so the small
// contractions run on the FP64 vector units from registers and LDS rather
// than being padded out to matrix-core tiles.
#include "kernels.hpp"

#include <cmath>

namespace dgbgk {

namespace {

template <int P>
struct Shape {
  static constexpr int N1 = P + 1;
  static constexpr int NP = N1 * N1;
  static constexpr int NFP = N1;
  static constexpr int S = (NP % 2 == 0) ? NP + 1 : NP;  // odd LDS row stride (doubles)
  static constexpr int G = kBlock / NP;                   // node groups per work-group
  static constexpr int T = G * NP;                        // threads with a node
};

struct LdsLayout {
  int jump, mom, rw, total;  // offsets / size in doubles; the tile starts at 0
};

__host__ __device__ inline LdsLayout lds_layout(int NP, int NFP, int S, int T, int E, int Qt) {
  LdsLayout L;
  const int tile_sz = Qt * E * S;
  int jump_sz = Qt * E * 2 * NFP;
  const int part_sz = 7 * T;  // moment partials alias the jump buffer
  if (part_sz > jump_sz) jump_sz = part_sz;
  L.jump = tile_sz;
  L.mom = L.jump + jump_sz;
  L.rw = L.mom + E * NP * 4;
  L.total = L.rw + E * 4 * NFP;
  return L;
}

// Work-groups are handed to the 8 XCDs round-robin; give each XCD a
// contiguous run of element blocks so that neighbour traces re-read by the
// next block are still in that XCD's L2.
__device__ inline int xcd_block(int b, int nblk) {
  const int per = nblk >> 3, rem = nblk & 7, x = b & 7;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

__device__ inline int neighbour(int k, int face, const StageArgs &a) {
  const int ex = k % a.nx, ey = k / a.nx;
  switch (face) {
    case 0: return ey > 0 ? k - a.nx : (a.periodic_y ? k + a.nx * (a.ny - 1) : -1);
    case 1: return ex < a.nx - 1 ? k + 1 : (a.periodic_x ? k - (a.nx - 1) : -1);
    case 2: return ey < a.ny - 1 ? k + a.nx : (a.periodic_y ? k - a.nx * (a.ny - 1) : -1);
    default: return ex > 0 ? k - 1 : (a.periodic_x ? k + (a.nx - 1) : -1);
  }
}

template <int P>
__global__ __launch_bounds__(kBlock) void stage_kernel(const StageArgs a) {
  using Sh = Shape<P>;
  constexpr int N1 = Sh::N1, NP = Sh::NP, NFP = Sh::NFP, S = Sh::S, G = Sh::G, T = Sh::T;
  extern __shared__ double lds[];
  const int E = a.E, log2E = a.log2E;
  const LdsLayout L = lds_layout(NP, NFP, S, T, E, a.Qt);
  double *tile = lds;
  double *jump = lds + L.jump;
  double *part = jump;
  double *mom = lds + L.mom;
  double *rw = lds + L.rw;

  const int tid = threadIdx.x;
  const int blk = xcd_block(blockIdx.x, a.nblk);
  const int k0 = blk * E;
  const int Eb = min(E, a.K - k0);
  const int q0 = blockIdx.y * a.Qt;
  const int Qb = min(a.Qt, a.Q - q0);
  const int rows = Qb * E;  // LDS row r = q_local * E + e
  const size_t KNP = (size_t)a.K * NP;
  const double *vex = a.vel;
  const double *vey = a.vel + a.Q;
  const double *vw = a.vel + 2 * a.Q;

  const int n = tid % NP;  // each thread keeps one node for the whole kernel
  const int g = tid / NP;
  const bool active = tid < T;

  // ---- 1. stage f_s of the block --------------------------------------------
  if (active) {
    for (int r = g; r < rows; r += G) {
      const int q = r >> log2E, e = r & (E - 1);
      if (e < Eb) tile[r * S + n] = a.fs[(size_t)(q0 + q) * KNP + (size_t)(k0 + e) * NP + n];
    }
  }
  __syncthreads();

  // ---- 2. node moments and diffuse-wall densities ----------------------------
  const bool walls = a.wall_mask != 0;
  if (a.fused) {
    const int Gp = G >> log2E;  // groups per (element, node)
    const int e = g & (E - 1), gp = g >> log2E;
    if (active && gp < Gp) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, hb = 0.0, hr = 0.0, ht = 0.0, hl = 0.0;
      if (e < Eb) {
        for (int q = gp; q < Qb; q += Gp) {
          const double v = tile[(q * E + e) * S + n];
          const double cx = vex[q0 + q], cy = vey[q0 + q];
          s0 += v;
          s1 += cx * v;
          s2 += cy * v;
          if (walls) {  // outgoing (e.n > 0) flux per wall side
            hb += cy < 0.0 ? -cy * v : 0.0;
            hr += cx > 0.0 ? cx * v : 0.0;
            ht += cy > 0.0 ? cy * v : 0.0;
            hl += cx < 0.0 ? -cx * v : 0.0;
          }
        }
      }
      double *pp = part + ((gp * E + e) * NP + n) * 7;
      pp[0] = s0; pp[1] = s1; pp[2] = s2;
      pp[3] = hb; pp[4] = hr; pp[5] = ht; pp[6] = hl;
    }
    __syncthreads();
    if (tid < E * NP) {
      const int e2 = tid / NP, n2 = tid % NP;
      if (e2 < Eb) {
        double s[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int gp2 = 0; gp2 < Gp; ++gp2) {
          const double *pp = part + ((gp2 * E + e2) * NP + n2) * 7;
#pragma unroll
          for (int c = 0; c < 7; ++c) s[c] += pp[c];
        }
        const double rho = s[0], ux = s[1] / rho, uy = s[2] / rho;
        double *m = mom + (e2 * NP + n2) * 4;
        m[0] = ux;
        m[1] = uy;
        m[2] = rho;
        m[3] = 1.0 - (ux * ux + uy * uy) * a.half_theta_inv;
        if (walls) {
          const int k = k0 + e2, kx = k % a.nx, ky = k / a.nx;
          const int i2 = n2 % N1, j2 = n2 / N1;
          const bool on[4] = {(a.wall_mask & 1) && ky == 0 && j2 == 0,
                              (a.wall_mask & 2) && kx == a.nx - 1 && i2 == P,
                              (a.wall_mask & 4) && ky == a.ny - 1 && j2 == P,
                              (a.wall_mask & 8) && kx == 0 && i2 == 0};
          const int fm[4] = {i2, j2, i2, j2};
#pragma unroll
          for (int fc = 0; fc < 4; ++fc)
            if (on[fc]) {
              const double v = s[3 + fc] * a.wall_den_inv[fc];
              rw[(e2 * 4 + fc) * NFP + fm[fc]] = v;
              if (a.rhow_out) a.rhow_out[((size_t)k * 4 + fc) * NFP + fm[fc]] = v;
            }
        }
      }
    }
  } else {
    if (tid < E * NP) {
      const int e2 = tid / NP, n2 = tid % NP;
      if (e2 < Eb) {
        const size_t node = (size_t)(k0 + e2) * NP + n2;
        const double rho = a.mom[node], ux = a.mom[KNP + node], uy = a.mom[2 * KNP + node];
        double *m = mom + (e2 * NP + n2) * 4;
        m[0] = ux;
        m[1] = uy;
        m[2] = rho;
        m[3] = 1.0 - (ux * ux + uy * uy) * a.half_theta_inv;
      }
    }
    if (walls) {
      for (int u = tid; u < E * 4 * NFP; u += blockDim.x) {
        const int e2 = u / (4 * NFP);
        if (e2 < Eb) rw[u] = a.rhow[(size_t)(k0 + e2) * 4 * NFP + (u - e2 * 4 * NFP)];
      }
    }
  }
  __syncthreads();

  // ---- 3. upwind jumps on the inflow faces -------------------------------------
  for (int u = tid; u < rows * 2 * NFP; u += blockDim.x) {
    const int m = u % NFP;
    const int rest = u / NFP;
    const int d = rest & 1;  // 0: x-face, 1: y-face
    const int r = rest >> 1;
    const int q = r >> log2E, e = r & (E - 1);
    if (e >= Eb) continue;
    const int qg = q0 + q;
    const int k = k0 + e;
    const double c = d == 0 ? vex[qg] : vey[qg];
    double J = 0.0;
    if (c != 0.0) {
      int face, own, nbnode;
      if (d == 0) {
        if (c > 0.0) { face = 3; own = N1 * m; nbnode = N1 * m + P; }
        else         { face = 1; own = N1 * m + P; nbnode = N1 * m; }
      } else {
        if (c > 0.0) { face = 0; own = m; nbnode = m + N1 * P; }
        else         { face = 2; own = m + N1 * P; nbnode = m; }
      }
      const int nb = neighbour(k, face, a);
      const double fm = tile[r * S + own];
      const double fp = nb >= 0 ? a.fs[(size_t)qg * KNP + (size_t)nb * NP + nbnode]
                                : rw[(e * 4 + face) * NFP + m] * a.feqb[face * a.Q + qg];
      J = (d == 0 ? a.fsx : a.fsy) * (-fabs(c)) * (fm - fp);  // e.n = -|c| on inflow
    }
    jump[r * 2 * NFP + d * NFP + m] = J;
  }
  __syncthreads();

  // ---- 4. volume + surface + collision + RK4 update ----------------------------
  if (!active) return;
  const int i = n % N1, j = n / N1;
  double dri[N1], dsj[N1];
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    dri[m] = a.D1[i * N1 + m];
    dsj[m] = a.D1[j * N1 + m];
  }
  const double llo_i = a.lift_lo[i], lhi_i = a.lift_hi[i];
  const double llo_j = a.lift_lo[j], lhi_j = a.lift_hi[j];
  for (int r = g; r < rows; r += G) {
    const int q = r >> log2E, e = r & (E - 1);
    if (e >= Eb) continue;
    const int qg = q0 + q;
    const double cx = vex[qg], cy = vey[qg], wq = vw[qg];
    const double *row = tile + r * S;
    double dr = 0.0, ds = 0.0;
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      dr += dri[m] * row[m + N1 * j];
      ds += dsj[m] * row[i + N1 * m];
    }
    const double fq = row[n];
    const double vol = -(cx * a.rx * dr + cy * a.sy * ds);
    const double *jr = jump + r * 2 * NFP;
    const double surf = (cx > 0.0 ? llo_i : lhi_i) * jr[j] + (cy > 0.0 ? llo_j : lhi_j) * jr[NFP + i];
    const double *mm = mom + (e * NP + n) * 4;
    const double eu = cx * mm[0] + cy * mm[1];
    const double feq = wq * mm[2] * (mm[3] + eu * (a.theta_inv + eu * a.half_theta2_inv));
    const double coll = (feq - fq) * a.inv_tau;
    const double kv = vol + surf + coll;
    const size_t gi = (size_t)qg * KNP + (size_t)(k0 + e) * NP + n;
    switch (a.stage) {
      case 0:
        a.out[gi] = kv;
        break;
      case 1:
        a.acc[gi] = fq + a.c_acc * kv;
        a.out[gi] = fq + a.c_out * kv;
        break;
      case 2:
      case 3: {
        const double ac = a.acc[gi];
        const double f0 = a.fn[gi];
        a.acc[gi] = ac + a.c_acc * kv;
        a.out[gi] = f0 + a.c_out * kv;
        break;
      }
      default:
        a.out[gi] = a.acc[gi] + a.c_acc * kv;
        break;
    }
  }
}

__global__ __launch_bounds__(256) void moments_kernel(const double *f, const double *vel, int K,
                                                      int P, int Q, int nx, int ny, int wall_mask,
                                                      double d0, double d1, double d2, double d3,
                                                      double *rho, double *ux, double *uy,
                                                      double *rhow) {
  const int N1 = P + 1, NP = N1 * N1;
  const size_t KNP = (size_t)K * NP;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KNP) return;
  const int k = (int)(i / NP), n = (int)(i % NP);
  const int kx = k % nx, ky = k / nx, ii = n % N1, jj = n / N1;
  const bool wb = rhow && (wall_mask & 1) && ky == 0 && jj == 0;
  const bool wr = rhow && (wall_mask & 2) && kx == nx - 1 && ii == P;
  const bool wt = rhow && (wall_mask & 4) && ky == ny - 1 && jj == P;
  const bool wl = rhow && (wall_mask & 8) && kx == 0 && ii == 0;
  const bool anyw = wb || wr || wt || wl;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, hb = 0.0, hr = 0.0, ht = 0.0, hl = 0.0;
  for (int q = 0; q < Q; ++q) {
    const double v = f[(size_t)q * KNP + i];
    const double cx = vel[q], cy = vel[Q + q];
    s0 += v;
    s1 += cx * v;
    s2 += cy * v;
    if (anyw) {
      hb += cy < 0.0 ? -cy * v : 0.0;
      hr += cx > 0.0 ? cx * v : 0.0;
      ht += cy > 0.0 ? cy * v : 0.0;
      hl += cx < 0.0 ? -cx * v : 0.0;
    }
  }
  if (rho) rho[i] = s0;
  if (ux) ux[i] = s1 / s0;
  if (uy) uy[i] = s2 / s0;
  const int NFP = N1;
  if (wb) rhow[((size_t)k * 4 + 0) * NFP + ii] = hb * d0;
  if (wr) rhow[((size_t)k * 4 + 1) * NFP + jj] = hr * d1;
  if (wt) rhow[((size_t)k * 4 + 2) * NFP + ii] = ht * d2;
  if (wl) rhow[((size_t)k * 4 + 3) * NFP + jj] = hl * d3;
}

// max that keeps NaN
__device__ inline double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

__global__ __launch_bounds__(256) void residual_kernel(const double *k, const double *vel, int KNP,
                                                       int Q, double scale,
                                                       unsigned long long *result) {
  __shared__ double red[256 / 64];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double m = 0.0;
  if (i < KNP) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = 0; q < Q; ++q) {
      const double v = k[(size_t)q * KNP + i];
      s0 += v;
      s1 += vel[q] * v;
      s2 += vel[Q + q] * v;
    }
    m = nan_max(nan_max(fabs(s0), fabs(s1)), fabs(s2)) * scale;
  }
  for (int off = 32; off > 0; off >>= 1) m = nan_max(m, __shfl_xor(m, off));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = nan_max(b, red[w]);
    atomicMax(result, (unsigned long long)__double_as_longlong(fabs(b)));
  }
}

__global__ void init_equilibrium_kernel(double *f, const double *vel, size_t KNP, int Q,
                                        double rho0, double ux0, double uy0, double theta) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= KNP) return;
  const double cx = vel[q], cy = vel[Q + q], w = vel[2 * Q + q];
  const double eu = cx * ux0 + cy * uy0, usq = ux0 * ux0 + uy0 * uy0;
  f[(size_t)q * KNP + i] =
      w * rho0 * (1.0 + eu / theta + eu * eu / (2.0 * theta * theta) - usq / (2.0 * theta));
}

__global__ void fill_u64_kernel(unsigned long long *p, size_t n, unsigned long long v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void u64_to_f64_kernel(const unsigned long long *src, double *dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = __longlong_as_double((long long)src[0]);
}

template <int P>
hipError_t launch_stage_p(const StageArgs &a, size_t lds, int ntiles, hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)stage_kernel<P>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)a.nblk, (unsigned)ntiles);
  hipLaunchKernelGGL(stage_kernel<P>, grid, dim3(kBlock), lds, st, a);
  return hipGetLastError();
}

}  // namespace

size_t stage_lds_bytes(int p, int E, int Qt) {
  const int N1 = p + 1, NP = N1 * N1;
  const int S = (NP % 2 == 0) ? NP + 1 : NP;
  const int G = kBlock / NP, T = G * NP;
  return (size_t)lds_layout(NP, N1, S, T, E, Qt).total * sizeof(double);
}

hipError_t launch_stage(int p, const StageArgs &a, size_t lds, int ntiles, hipStream_t st) {
  switch (p) {
    case 1: return launch_stage_p<1>(a, lds, ntiles, st);
    case 2: return launch_stage_p<2>(a, lds, ntiles, st);
    case 3: return launch_stage_p<3>(a, lds, ntiles, st);
    case 4: return launch_stage_p<4>(a, lds, ntiles, st);
    case 5: return launch_stage_p<5>(a, lds, ntiles, st);
    case 6: return launch_stage_p<6>(a, lds, ntiles, st);
    case 7: return launch_stage_p<7>(a, lds, ntiles, st);
    case 8: return launch_stage_p<8>(a, lds, ntiles, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_moments(const double *f, const double *vel, int K, int p, int Q, int nx, int ny,
                          int wall_mask, const double *den, double *rho, double *ux, double *uy,
                          double *rhow, hipStream_t st) {
  const size_t KNP = (size_t)K * (p + 1) * (p + 1);
  const unsigned nb = (unsigned)((KNP + 255) / 256);
  hipLaunchKernelGGL(moments_kernel, dim3(nb), dim3(256), 0, st, f, vel, K, p, Q, nx, ny,
                     wall_mask, den[0], den[1], den[2], den[3], rho, ux, uy, rhow);
  return hipGetLastError();
}

hipError_t launch_residual(const double *k, const double *vel, int K, int Np, int Q, double scale,
                           unsigned long long *result, hipStream_t st) {
  const int KNP = K * Np;
  const unsigned nb = (unsigned)((KNP + 255) / 256);
  hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(256), 0, st, k, vel, KNP, Q, scale, result);
  return hipGetLastError();
}

hipError_t launch_init_equilibrium(double *f, const double *vel, int K, int Np, int Q, double rho0,
                                   double ux0, double uy0, double theta, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(init_equilibrium_kernel, grid, dim3(256), 0, st, f, vel, KNP, Q, rho0, ux0,
                     uy0, theta);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, size_t n, unsigned long long v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_u64_to_f64(const unsigned long long *src, double *dst, hipStream_t st) {
  hipLaunchKernelGGL(u64_to_f64_kernel, dim3(1), dim3(64), 0, st, src, dst);
  return hipGetLastError();
}

}  // namespace dgbgk
