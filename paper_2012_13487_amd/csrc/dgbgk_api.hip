// C ABI of the DG-BGK library (declared in include/dgbgk.h).
//
// Host side: validation, reference-element and wall tables, device memory,
// and the order of kernel launches for one RK4 step.  All arithmetic of the
// time step runs in the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dgbgk.h"
#include "host_math.hpp"
#include "kernels.hpp"
#include "init.hpp"
#include "kernels32.hpp"
#include "linalg.hpp"

using namespace dgbgk;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kFusedLdsLimit = 80 * 1024;  // keeps >= 2 work-groups per CU
constexpr size_t kStreamLdsLimit = 160 * 1024;  // one persistent work-group per CU
constexpr int kMaxQ = 4096;

size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// MI355X last-level cache (Infinity Cache).  A stage touches four state
// arrays; when they fit, the streams read once per stage are left cached
// (the next stages find them there); above it they move with non-temporal
// hints so that the neighbour tiles stay in L2 (measured both ways).
constexpr size_t kLastLevelCacheBytes = (size_t)256 << 20;
int stream_nt_for(size_t state_bytes) { return 4 * state_bytes > kLastLevelCacheBytes ? 1 : 0; }

struct Layout {
  size_t fn, acc, a, b, xfer, vel, feqb, wmom, dmat, mom, rhow, u64, fref, rref, mref, part, total;
};

bool is_fp32(int precision) {
  return precision == DGBGK_FP32 || precision == DGBGK_FP32_BF16MMA || precision == DGBGK_FP32_REF ||
         precision == DGBGK_FP32_BF16MMA_REF;
}
bool is_bf(int precision) { return precision == DGBGK_FP32_BF16MMA || precision == DGBGK_FP32_BF16MMA_REF; }
bool is_ref(int precision) { return precision == DGBGK_FP32_REF || precision == DGBGK_FP32_BF16MMA_REF; }
bool valid_precision(int precision) { return precision == DGBGK_FP64 || is_fp32(precision); }

// Velocity tiles whose moment partials a state of this precision keeps.
int part_tiles(int precision, int Np) {
  if (precision == DGBGK_FP64) return kMaxPartialTiles;
  return (Np == 4 || Np == 16) ? 1 : 0;  // the orders that hand moments over (1 and 3)
}

// State registers (FP64, or the FP32 deviation), an FP64 transfer buffer for
// the FP32 precisions, then the small tables.
Layout make_layout(int64_t K, int Np, int Nfp, int Q, int precision) {
  Layout L{};
  const size_t ndof = (size_t)K * Np * Q;
  const size_t dof = ndof * (is_fp32(precision) ? sizeof(float) : sizeof(double));
  size_t off = 0;
  L.fn = off;   off += round_up(dof);
  L.acc = off;  off += round_up(dof);
  L.a = off;    off += round_up(dof);
  L.b = off;    off += round_up(dof);
  L.xfer = off; off += is_fp32(precision) ? round_up(ndof * sizeof(double)) : 0;
  L.vel = off;  off += round_up((size_t)3 * Q * sizeof(double));
  L.feqb = off; off += round_up((size_t)4 * Q * sizeof(double));
  L.wmom = off; off += round_up((size_t)16 * Q * sizeof(double));
  L.mom = off;  off += round_up((size_t)3 * K * Np * sizeof(double));
  L.rhow = off; off += round_up((size_t)K * 4 * Nfp * sizeof(double));
  L.u64 = off;  off += round_up(8 * sizeof(unsigned long long));
  L.dmat = off; off += round_up((size_t)((2 * Np + 15) / 16) * 16 * 32 * sizeof(uint16_t));
  // reference form: the FP64 reference state, its right-hand side in FP32 and its node moments
  const bool ref = is_ref(precision);
  L.fref = off; off += ref ? round_up(ndof * sizeof(double)) : 0;
  L.rref = off; off += ref ? round_up(ndof * sizeof(float)) : 0;
  L.mref = off; off += ref ? round_up((size_t)3 * K * Np * sizeof(double)) : 0;
  // moment partials of two states (the state a stage reads, the one it
  // writes): FP64 up to kMaxPartialTiles velocity tiles each; FP32 storage one
  // (one-element blocks of orders 1 and 3)
  L.part = off;
  off += 2 * round_up((size_t)part_tiles(precision, Np) * K * 7 * Np * sizeof(double));
  L.total = off;
  return L;
}

thread_local std::string g_create_error;

// Size (DOF) from which a batch member runs its own single-problem stage
// kernels, in its own decomposition, instead of joining a persistent class
// launch: 2^22 DOF fill the GPU with 1024 or more work-groups.
constexpr int64_t kSoloDof = (int64_t)1 << 22;

// Streams a batch spreads its independent chains over (the hardware queues
// a process gets by default).
constexpr size_t kBatchLanes = 4;

}  // namespace

struct dgbgk_solver {
  dgbgk_problem pb{};
  std::vector<double> ex, ey, w;
  int64_t K = 0;
  int Np = 0, Nfp = 0, Q = 0, p = 0;
  double hx = 0, hy = 0;
  std::vector<double> r, D1, M1, lift_lo, lift_hi;
  std::vector<double> feqb;  // [4][Q]
  double wall_den[4] = {0, 0, 0, 0};
  double wall_den_inv[4] = {0, 0, 0, 0};
  int wall_mask = 0;
  double resid_scale = 1.0;
  hipStream_t stream = nullptr;
  // device
  bool dev_ready = false;
  int device = -1;  // the device holding the solver's memory
  void *base = nullptr;
  bool owns = false;
  Layout lay{};
  double *d_fn = nullptr, *d_acc = nullptr, *d_a = nullptr, *d_b = nullptr;  // FP64 states
  float *g_fn = nullptr, *g_acc = nullptr, *g_a = nullptr, *g_b = nullptr;   // FP32 deviations
  double *d_xfer = nullptr;  // FP64 staging of host transfers (FP32 precisions)
  uint16_t *d_dmat = nullptr;  // bf16 [Dr; Ds] rows, 32 columns (FP32_BF16MMA)
  int prec = DGBGK_FP64;
  double rho_ref = 1.0;      // reference density of the FP32 deviation g = f - w rho_ref
  double mconst[7] = {0, 0, 0, 0, 0, 0, 0};
  double *d_vel = nullptr, *d_feqb = nullptr, *d_wmom = nullptr, *d_mom = nullptr, *d_rhow = nullptr;
  unsigned long long *d_u64 = nullptr;
  // velocity-tiled FP64 stages: moment partials (two slots; slot 0 holds f_n's
  // between steps) and whether slot 0 holds those of the current f_n
  double *d_part[2] = {nullptr, nullptr};
  bool part_valid = false;
  // reference form: f = f_ref + g (FP64 reference, FP32 correction in the registers)
  double *d_fref = nullptr, *d_mref = nullptr;
  float *g_rref = nullptr;
  struct Cfg64 {
    int fused = 1, E = 1, log2E = 0, Qt = 0, ntiles = 1, nblk = 1;
    size_t lds = 0;
  } ref64;  // FP64 decomposition of the reference's right-hand side
  // launch configuration
  int fused = 1, E = 1, log2E = 0, Qt = 0, ntiles = 1, nblk = 1;
  int persistent = 0;  // fused blocks run by the persistent pipelined kernel
  int num_cu = 256;
  size_t lds = 0;
  int tiling_mode = 0, tiling_qt = 0;
  int forced_E = 0;  // elements per work-group set by the caller or the autotuner (0: automatic)
  // RK4 steps replayed from a captured hipGraph (0: eager launches)
  int graph_steps = 0;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;  // capture stream (the solver's may be the null stream)
  double graph_dt = 0.0;             // dt and launch configuration the graph was captured with
  int graph_cfg[5] = {0, 0, 0, 0, 0};
  bool graph_partials = false;       // the captured first stage reads f_n's partials
  // implicit-step workspace (allocated at the first implicit step)
  double *imp_ws = nullptr;
  size_t imp_bytes = 0;
  // state
  bool have_state = false;
  int64_t steps = 0;
  std::string err;
};

namespace {

int fail(dgbgk_solver *s, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (s) s->err = buf;
  else g_create_error = buf;
  return code;
}

int hip_fail(dgbgk_solver *s, hipError_t e, const char *what) {
  return fail(s, DGBGK_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is_finite_d(double v) { return std::isfinite(v); }

int validate(const dgbgk_problem *pb, dgbgk_solver *s) {
  if (!pb) return fail(s, DGBGK_EINVAL, "problem is NULL");
  if (pb->nx < 1 || pb->ny < 1) return fail(s, DGBGK_EINVAL, "nx, ny must be >= 1");
  if ((int64_t)pb->nx * pb->ny > (int64_t)1 << 30)
    return fail(s, DGBGK_EINVAL, "too many elements");
  if (pb->p < 1 || pb->p > kMaxP) return fail(s, DGBGK_EINVAL, "p must be in 1..%d", kMaxP);
  if (pb->q < 1 || pb->q > kMaxQ) return fail(s, DGBGK_EINVAL, "q must be in 1..%d", kMaxQ);
  if (!pb->ex || !pb->ey || !pb->w) return fail(s, DGBGK_EINVAL, "velocity arrays are NULL");
  if (!(pb->lx > 0) || !(pb->ly > 0) || !is_finite_d(pb->lx) || !is_finite_d(pb->ly) || !is_finite_d(pb->x0) ||
      !is_finite_d(pb->y0))
    return fail(s, DGBGK_EINVAL, "domain must be finite with lx, ly > 0");
  if (!(pb->theta > 0) || !is_finite_d(pb->theta)) return fail(s, DGBGK_EINVAL, "theta must be > 0");
  if (!(pb->tau > 0)) return fail(s, DGBGK_EINVAL, "tau must be > 0 (or +inf)");
  for (int i = 0; i < pb->q; ++i)
    if (!is_finite_d(pb->ex[i]) || !is_finite_d(pb->ey[i]) || !is_finite_d(pb->w[i]))
      return fail(s, DGBGK_EINVAL, "velocity set entry %d is not finite", i);
  for (int sd = 0; sd < 4; ++sd) {
    if (pb->bc[sd] != DGBGK_BC_PERIODIC && pb->bc[sd] != DGBGK_BC_DIFFUSE_WALL)
      return fail(s, DGBGK_EINVAL, "bc[%d] is not a dgbgk_bc", sd);
    if (!is_finite_d(pb->wall_u[sd][0]) || !is_finite_d(pb->wall_u[sd][1]))
      return fail(s, DGBGK_EINVAL, "wall_u[%d] is not finite", sd);
  }
  if ((pb->bc[0] == DGBGK_BC_PERIODIC) != (pb->bc[2] == DGBGK_BC_PERIODIC) ||
      (pb->bc[1] == DGBGK_BC_PERIODIC) != (pb->bc[3] == DGBGK_BC_PERIODIC))
    return fail(s, DGBGK_EINVAL, "periodic sides must come in pairs (0,2) and (1,3)");
  // sides 0, 2 have normals along y; 1, 3 along x: the wall velocity must be tangential
  for (int sd = 0; sd < 4; ++sd) {
    if (pb->bc[sd] != DGBGK_BC_DIFFUSE_WALL) continue;
    const double un = (sd % 2 == 0) ? pb->wall_u[sd][1] : pb->wall_u[sd][0];
    if (un != 0.0) return fail(s, DGBGK_EINVAL, "wall_u[%d] has a normal component", sd);
  }
  return DGBGK_OK;
}

// FP32 precisions: always the fused form; E elements per work-group while
// the tile stays within 64 KB of LDS (at least one element, up to 160 KB).
// Largest block, in DOF, the automatic choice gives one work-group (32 KB
// of FP64 state): on the 64x64 p = 3 NC 16x16 cavity one element per
// work-group (4096 DOF) measured faster than two once element blocks run in
// strips (126 vs 129 us FP64, 68.5 vs 69.5 us FP32).
constexpr int64_t kMaxBlockDof = 4096;

void choose_tiling32(dgbgk_solver *s) {
  const int NP = s->Np;
  const bool bf = is_bf(s->prec), ref = is_ref(s->prec);
  int E = 1;
  while ((int64_t)E * 2 * s->Q * NP <= kMaxBlockDof && E * 2 <= s->K &&
         stage32_lds_bytes(s->p, E * 2, s->Q, bf, ref) <= kFusedLdsLimit)
    E *= 2;
  if (s->forced_E > 0) E = s->forced_E;
  s->E = E;
  s->log2E = 0;
  while ((1 << s->log2E) < E) ++s->log2E;
  s->fused = 1;
  s->persistent = 0;
  s->Qt = s->Q;
  s->ntiles = 1;
  s->nblk = (int)((s->K + E - 1) / E);
  s->lds = stage32_lds_bytes(s->p, E, s->Q, bf, ref);
}

// Launch configuration: fused (all velocities of E elements per work-group)
// when its LDS fits, else velocity tiles with a separate moments pass.
void choose_tiling(dgbgk_solver *s) {
  s->part_valid = false;  // the tile decomposition of any partials changes
  if (is_fp32(s->prec)) {
    choose_tiling32(s);
    return;
  }
  const int NP = s->Np;
  const int G = kBlock / NP;
  int E = 1;
  // the persistent kernel takes one velocity row per thread
  const bool row_cap = s->tiling_mode == 4 && s->p <= kStreamMaxP;
  while (E * 2 <= G && (int64_t)E * 2 * s->Q * NP <= kMaxBlockDof && E * 2 <= s->K &&
         (!row_cap || (int64_t)E * 2 * s->Q <= kBlock) &&
         stage_lds_bytes(s->p, E * 2, s->Q) <= kFusedLdsLimit)
    E *= 2;
  if (s->forced_E > 0) E = s->forced_E;
  size_t lds = stage_lds_bytes(s->p, E, s->Q);
  bool fused = lds <= kFusedLdsLimit;
  if (s->tiling_mode == 1 || s->tiling_mode == 3 || s->tiling_mode == 4 || s->forced_E > 0)
    fused = true;
  if (s->tiling_mode == 2) fused = false;
  if (fused) {
    s->fused = 1;
    s->Qt = s->Q;
    s->ntiles = 1;
  } else {
    E = 1;
    int qt = s->tiling_qt > 0 ? s->tiling_qt : s->Q;
    if (qt > s->Q) qt = s->Q;
    if (s->tiling_qt <= 0) {
      while (qt > 1 && stage_lds_bytes(s->p, E, qt) > kFusedLdsLimit) qt = (qt + 1) / 2;
      // the same number of tiles with a multiple of 64 velocity rows per tile,
      // where it fits: the row phase then runs whole wavefronts (576 velocities
      // at p = 4: 320 + 256 rows measured 2127 us per stage against 2190 for 288 + 288)
      const int nt = (s->Q + qt - 1) / qt, q64 = (qt + 63) / 64 * 64;
      if (q64 < s->Q && (s->Q + q64 - 1) / q64 == nt && stage_lds_bytes(s->p, E, q64) <= kFusedLdsLimit)
        qt = q64;
    }
    s->fused = 0;
    s->Qt = qt;
    s->ntiles = (s->Q + qt - 1) / qt;
    lds = stage_lds_bytes(s->p, E, qt);
  }
  s->E = E;
  s->log2E = 0;
  while ((1 << s->log2E) < E) ++s->log2E;
  s->nblk = (int)((s->K + E - 1) / E);
  s->persistent = s->fused && s->tiling_mode == 4 && stream_applicable(s->p, E, s->Q, s->K) &&
                  stream_lds_bytes(s->p, E, s->Q) <= kStreamLdsLimit;
  if (s->persistent) lds = stream_lds_bytes(s->p, E, s->Q);
  s->lds = lds;
}

int ensure_device(dgbgk_solver *s) {
  if (s->dev_ready) return DGBGK_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(s, e, "hipGetDevice (no usable GPU)");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(s, e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(s, DGBGK_EDEVICE, "device %d is %s; this library is built for gfx950", dev,
                prop.gcnArchName);
  if (prop.multiProcessorCount > 0) s->num_cu = prop.multiProcessorCount;
  s->device = dev;
  if (s->lds > prop.sharedMemPerBlock && s->lds > 65536)
    return fail(s, DGBGK_EDEVICE, "stage kernel needs %zu B of LDS, device allows %zu", s->lds,
                (size_t)prop.sharedMemPerBlock);
  if (!s->base) {
    void *p = nullptr;
    e = hipMalloc(&p, s->lay.total);
    if (e != hipSuccess) return fail(s, DGBGK_ENOMEM, "hipMalloc(%zu): %s", s->lay.total,
                                     hipGetErrorString(e));
    s->base = p;
    s->owns = true;
  }
  char *b = (char *)s->base;
  s->d_fn = (double *)(b + s->lay.fn);
  s->d_acc = (double *)(b + s->lay.acc);
  s->d_a = (double *)(b + s->lay.a);
  s->d_b = (double *)(b + s->lay.b);
  s->g_fn = (float *)(b + s->lay.fn);
  s->g_acc = (float *)(b + s->lay.acc);
  s->g_a = (float *)(b + s->lay.a);
  s->g_b = (float *)(b + s->lay.b);
  s->d_xfer = is_fp32(s->prec) ? (double *)(b + s->lay.xfer) : nullptr;
  s->d_vel = (double *)(b + s->lay.vel);
  s->d_feqb = (double *)(b + s->lay.feqb);
  s->d_wmom = (double *)(b + s->lay.wmom);
  s->d_dmat = (uint16_t *)(b + s->lay.dmat);
  s->d_mom = (double *)(b + s->lay.mom);
  s->d_rhow = (double *)(b + s->lay.rhow);
  s->d_u64 = (unsigned long long *)(b + s->lay.u64);
  if (const int pt = part_tiles(s->prec, s->Np)) {
    s->d_part[0] = (double *)(b + s->lay.part);
    s->d_part[1] = (double *)(b + s->lay.part + round_up((size_t)pt * s->K * 7 * s->Np * sizeof(double)));
  }
  if (is_ref(s->prec)) {
    s->d_fref = (double *)(b + s->lay.fref);
    s->g_rref = (float *)(b + s->lay.rref);
    s->d_mref = (double *)(b + s->lay.mref);
  }
  std::vector<double> vel((size_t)3 * s->Q);
  for (int q = 0; q < s->Q; ++q) {
    vel[q] = s->ex[q];
    vel[s->Q + q] = s->ey[q];
    vel[2 * s->Q + q] = s->w[q];
  }
  // moment weights per velocity: 1, e_x, e_y, then the outgoing normal speed
  // e.n > 0 at a bottom, right, top and left wall (for eq. (8)); rest zero
  std::vector<double> wm((size_t)16 * s->Q, 0.0);
  for (int q = 0; q < s->Q; ++q) {
    const double cx = s->ex[q], cy = s->ey[q];
    double *r = &wm[(size_t)16 * q];
    r[0] = 1.0;
    r[1] = cx;
    r[2] = cy;
    r[3] = cy < 0.0 ? -cy : 0.0;
    r[4] = cx > 0.0 ? cx : 0.0;
    r[5] = cy > 0.0 ? cy : 0.0;
    r[6] = cx < 0.0 ? -cx : 0.0;
  }
  e = hipMemcpyAsync(s->d_vel, vel.data(), vel.size() * sizeof(double), hipMemcpyHostToDevice,
                     s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_wmom, wm.data(), wm.size() * sizeof(double), hipMemcpyHostToDevice,
                       s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_feqb, s->feqb.data(), s->feqb.size() * sizeof(double),
                       hipMemcpyHostToDevice, s->stream);
  std::vector<uint16_t> dm;
  if (is_bf(s->prec)) {
    // [Dr; Ds] (2 Np x Np, node n = i + N1 j), rows padded to 16-row tiles and
    // columns to 32, rounded to bf16 (nearest, ties to even)
    const int N1 = s->Nfp, Np = s->Np, rows = (2 * Np + 15) / 16 * 16;
    dm.assign((size_t)rows * 32, 0);
    auto bf = [](double v) {
      float x = (float)v;
      uint32_t u;
      std::memcpy(&u, &x, 4);
      u += 0x7fffu + ((u >> 16) & 1u);
      return (uint16_t)(u >> 16);
    };
    for (int n = 0; n < Np; ++n)
      for (int m = 0; m < Np; ++m) {
        const int in = n % N1, jn = n / N1, im = m % N1, jm = m / N1;
        if (jn == jm) dm[(size_t)n * 32 + m] = bf(s->D1[in * N1 + im]);
        if (in == im) dm[(size_t)(Np + n) * 32 + m] = bf(s->D1[jn * N1 + jm]);
      }
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->d_dmat, dm.data(), dm.size() * sizeof(uint16_t), hipMemcpyHostToDevice,
                         s->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "uploading tables");
  s->dev_ready = true;
  return DGBGK_OK;
}

StageArgs base_args(const dgbgk_solver *s) {
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  const int N1 = s->p + 1;
  for (int i = 0; i < N1 * N1; ++i) a.D1[i] = s->D1[i];
  for (int i = 0; i < N1; ++i) {
    a.lift_lo[i] = s->lift_lo[i];
    a.lift_hi[i] = s->lift_hi[i];
  }
  a.vel = s->d_vel;
  a.feqb = s->d_feqb;
  a.wmom = s->d_wmom;
  a.mom = s->d_mom;
  a.rhow = s->d_rhow;
  a.rx = 2.0 / s->hx;
  a.sy = 2.0 / s->hy;
  a.fsx = 2.0 / s->hx;  // face Jacobian hy/2 over volume Jacobian hx hy/4
  a.fsy = 2.0 / s->hy;
  a.theta_inv = 1.0 / s->pb.theta;
  a.half_theta2_inv = 1.0 / (2.0 * s->pb.theta * s->pb.theta);
  a.half_theta_inv = 1.0 / (2.0 * s->pb.theta);
  a.inv_tau = std::isinf(s->pb.tau) ? 0.0 : 1.0 / s->pb.tau;
  for (int sd = 0; sd < 4; ++sd) a.wall_den_inv[sd] = s->wall_den_inv[sd];
  a.nx = s->pb.nx;
  a.ny = s->pb.ny;
  a.K = (int)s->K;
  a.Q = s->Q;
  a.E = s->E;
  a.log2E = s->log2E;
  a.Qt = s->Qt;
  a.nblk = s->nblk;
  a.wall_mask = s->wall_mask;
  a.periodic_x = s->pb.bc[1] == DGBGK_BC_PERIODIC;
  a.periodic_y = s->pb.bc[0] == DGBGK_BC_PERIODIC;
  a.fused = s->fused;
  a.stream_nt = stream_nt_for((size_t)s->K * s->Np * s->Q * sizeof(double));
  return a;
}

Stage32Args base_args32(const dgbgk_solver *s) {
  Stage32Args a;
  std::memset(&a, 0, sizeof a);
  const int N1 = s->p + 1;
  for (int i = 0; i < N1 * N1; ++i) a.D1[i] = (float)s->D1[i];
  for (int i = 0; i < N1; ++i) {
    a.lift_lo[i] = (float)s->lift_lo[i];
    a.lift_hi[i] = (float)s->lift_hi[i];
  }
  a.vel = s->d_vel;
  a.feqb = s->d_feqb;
  a.wmom = s->d_wmom;
  a.dmat = is_bf(s->prec) ? s->d_dmat : nullptr;
  a.rref = is_ref(s->prec) ? s->g_rref : nullptr;
  a.mref = is_ref(s->prec) ? s->d_mref : nullptr;
  a.rx = (float)(2.0 / s->hx);
  a.sy = (float)(2.0 / s->hy);
  a.fsx = (float)(2.0 / s->hx);
  a.fsy = (float)(2.0 / s->hy);
  a.theta_inv = (float)(1.0 / s->pb.theta);
  a.half_theta2_inv = (float)(1.0 / (2.0 * s->pb.theta * s->pb.theta));
  a.half_theta_inv = 1.0 / (2.0 * s->pb.theta);
  a.inv_tau = std::isinf(s->pb.tau) ? 0.0f : (float)(1.0 / s->pb.tau);
  for (int sd = 0; sd < 4; ++sd) a.wall_den_inv[sd] = s->wall_den_inv[sd];
  for (int c = 0; c < 7; ++c) a.mconst[c] = s->mconst[c];
  a.rho_ref = s->rho_ref;
  a.nx = s->pb.nx;
  a.ny = s->pb.ny;
  a.K = (int)s->K;
  a.Q = s->Q;
  a.E = s->E;
  a.nblk = s->nblk;
  a.wall_mask = s->wall_mask;
  a.periodic_x = s->pb.bc[1] == DGBGK_BC_PERIODIC;
  a.periodic_y = s->pb.bc[0] == DGBGK_BC_PERIODIC;
  a.stream_nt = stream_nt_for((size_t)s->K * s->Np * s->Q * sizeof(float));
  return a;
}

void rk_coefficients(int stage, double dt, double &ca, double &co) {
  ca = co = 0.0;
  switch (stage) {
    case 1: ca = dt / 6.0; co = dt / 2.0; break;
    case 2: ca = dt / 3.0; co = dt / 2.0; break;
    case 3: ca = dt / 3.0; co = dt; break;
    case 4: ca = dt / 6.0; co = 0.0; break;
    default: break;
  }
}

// One FP32 stage on deviation arrays.
int run_stage32(dgbgk_solver *s, int stage, const float *fs, float *out, double dt,
                double *rhow_out, const double *pin = nullptr, double *pout = nullptr) {
  Stage32Args a = base_args32(s);
  a.fs = fs;
  a.fn = s->g_fn;
  a.acc = s->g_acc;
  a.out = out;
  a.stage = stage;
  a.rhow_out = rhow_out;
  a.pin = pin;
  a.pout = pout;
  double ca, co;
  rk_coefficients(stage, dt, ca, co);
  a.c_acc = (float)ca;
  a.c_out = (float)co;
  hipError_t e = launch_stage32(s->p, a, s->lds, is_bf(s->prec), is_ref(s->prec), s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "FP32 stage kernel");
  return DGBGK_OK;
}

// One stage: L(fs) combined into the RK4 registers (stage 1..4) or written to
// out (stage 0).  Tiled mode first reduces the moments of fs.  The state
// pointers are FP64 arrays, or FP32 deviation arrays for the FP32 precisions.
int run_stage(dgbgk_solver *s, int stage, const void *fs_, void *out_, double dt,
              double *rhow_out = nullptr, const double *pin = nullptr, double *pout = nullptr) {
  if (is_fp32(s->prec))
    return run_stage32(s, stage, (const float *)fs_, (float *)out_, dt, rhow_out, pin, pout);
  const double *fs = (const double *)fs_;
  double *out = (double *)out_;
  hipError_t e;
  if (!s->fused && !pin) {
    e = launch_moments(fs, s->d_vel, (int)s->K, s->p, s->Q, s->pb.nx, s->pb.ny, s->wall_mask,
                       s->wall_den_inv, s->d_mom, s->d_mom + s->K * s->Np,
                       s->d_mom + 2 * s->K * s->Np, s->wall_mask ? s->d_rhow : nullptr, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "moments kernel");
  }
  StageArgs a = base_args(s);
  a.fs = fs;
  a.fn = s->d_fn;
  a.acc = s->d_acc;
  a.out = out;
  a.stage = stage;
  a.rhow_out = rhow_out;
  a.pin = pin;
  a.pout = pout;
  rk_coefficients(stage, dt, a.c_acc, a.c_out);
  if (s->persistent) {
    const int groups = (int)std::min<int64_t>(s->nblk, (int64_t)s->num_cu);
    e = launch_stream(s->p, a, s->lds, groups, s->stream);
  } else {
    e = launch_stage(s->p, a, s->lds, s->ntiles, s->stream);
  }
  if (e != hipSuccess) return hip_fail(s, e, "stage kernel");
  return DGBGK_OK;
}

// Reference form: r = L(f_ref) by the FP64 stage kernel (into the FP64
// transfer buffer, then rounded to FP32), and the node moments of f_ref.
int ref_refresh(dgbgk_solver *s) {
  const dgbgk_solver::Cfg64 &c = s->ref64;
  const int K = (int)s->K;
  const size_t KN = (size_t)s->K * s->Np, n = KN * s->Q;
  hipError_t e = hipSuccess;
  if (!c.fused)
    e = launch_moments(s->d_fref, s->d_vel, K, s->p, s->Q, s->pb.nx, s->pb.ny, s->wall_mask,
                       s->wall_den_inv, s->d_mom, s->d_mom + KN, s->d_mom + 2 * KN,
                       s->wall_mask ? s->d_rhow : nullptr, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "reference moments pass");
  StageArgs a = base_args(s);
  a.E = c.E;
  a.log2E = c.log2E;
  a.Qt = c.Qt;
  a.nblk = c.nblk;
  a.fused = c.fused;
  a.stream_nt = stream_nt_for(n * sizeof(double));
  a.fs = s->d_fref;
  a.fn = s->d_fref;
  a.acc = nullptr;
  a.out = s->d_xfer;
  a.stage = 0;
  e = launch_stage(s->p, a, c.lds, c.ntiles, s->stream);
  if (e == hipSuccess) e = launch_f64_to_f32(s->d_xfer, s->g_rref, n, s->stream);
  if (e == hipSuccess)
    e = launch_moments(s->d_fref, s->d_vel, K, s->p, s->Q, s->pb.nx, s->pb.ny, 0, s->wall_den_inv,
                       s->d_mref, s->d_mref + KN, s->d_mref + 2 * KN, nullptr, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "reference right-hand side");
  return DGBGK_OK;
}

// g = 0 (graph-safe fill kernel; the region is padded to 256 bytes).
hipError_t zero_f32(dgbgk_solver *s, float *g) {
  const size_t n = (size_t)s->K * s->Np * s->Q;
  return launch_fill_u64((unsigned long long *)g, (n * sizeof(float) + 7) / 8, 0ull, s->stream);
}

// Reference form: the state just written to f_ref becomes the reference,
// with a zero correction.
int ref_reset(dgbgk_solver *s) {
  hipError_t e = zero_f32(s, s->g_fn);
  if (e != hipSuccess) return hip_fail(s, e, "fill kernel");
  return ref_refresh(s);
}

}  // namespace

extern "C" {

const char *dgbgk_version(void) { return "dgbgk 0.2 (gfx950; FP64, FP32 storage)"; }

const char *dgbgk_last_error(const dgbgk_solver *s) {
  if (!s) return g_create_error.c_str();
  return s->err.c_str();
}

int dgbgk_velset_gh(int32_t n1d, double *ex, double *ey, double *w, double *theta) {
  if (!ex || !ey || !w) return fail(nullptr, DGBGK_EINVAL, "NULL output");
  std::vector<double> x, wt;
  if (!gauss_hermite_rule(n1d, x, wt)) return fail(nullptr, DGBGK_EINVAL, "n1d must be 1..40");
  for (int b = 0; b < n1d; ++b)
    for (int a = 0; a < n1d; ++a) {
      ex[a + n1d * b] = x[a];
      ey[a + n1d * b] = x[b];
      w[a + n1d * b] = wt[a] * wt[b];
    }
  if (theta) *theta = 1.0;
  return DGBGK_OK;
}

int dgbgk_velset_nc(int32_t m1d, double vmax, double *ex, double *ey, double *w, double *theta) {
  if (!ex || !ey || !w) return fail(nullptr, DGBGK_EINVAL, "NULL output");
  std::vector<double> x, wt;
  if (!newton_cotes_rule(m1d, vmax, x, wt))
    return fail(nullptr, DGBGK_EINVAL, "m1d must be 2..64 and vmax > 0");
  double th = 0.0;
  for (int b = 0; b < m1d; ++b)
    for (int a = 0; a < m1d; ++a) {
      const int q = a + m1d * b;
      ex[q] = x[a];
      ey[q] = x[b];
      w[q] = wt[a] * wt[b];
    }
  for (int q = 0; q < m1d * m1d; ++q) th += w[q] * ex[q] * ex[q];
  if (theta) *theta = th;
  return DGBGK_OK;
}

int dgbgk_tau_from_kn(double kn, double L, int32_t convention, double *tau) {
  if (!tau || !(kn > 0) || !(L > 0)) return fail(nullptr, DGBGK_EINVAL, "kn, L must be > 0");
  if (convention == 0) *tau = kn * L / std::sqrt(3.0);
  else if (convention == 1) *tau = kn * L / std::sqrt(M_PI / 2.0);
  else return fail(nullptr, DGBGK_EINVAL, "convention must be 0 or 1");
  return DGBGK_OK;
}

int dgbgk_required_bytes(const dgbgk_problem *pb, int32_t precision, size_t *bytes) {
  if (!bytes) return fail(nullptr, DGBGK_EINVAL, "bytes is NULL");
  int rc = validate(pb, nullptr);
  if (rc) return rc;
  if (!valid_precision(precision))
    return fail(nullptr, DGBGK_EINVAL, "unknown precision %d", precision);
  const int N1 = pb->p + 1;
  *bytes = make_layout((int64_t)pb->nx * pb->ny, N1 * N1, N1, pb->q, precision).total;
  return DGBGK_OK;
}

int dgbgk_create(const dgbgk_problem *pb, int32_t precision, void *hip_stream,
                 dgbgk_solver **out) {
  if (!out) return fail(nullptr, DGBGK_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(pb, nullptr);
  if (rc) return rc;
  if (!valid_precision(precision))
    return fail(nullptr, DGBGK_EINVAL, "unknown precision %d", precision);
  if (is_bf(precision) && !bf16_contraction_available(pb->p))
    return fail(nullptr, DGBGK_ENOTSUP, "bf16 contractions are built for p <= 4");
  if (is_ref(precision) && !ref_form_available(pb->p, is_bf(precision)))
    return fail(nullptr, DGBGK_ENOTSUP, "the reference form is built for p <= 4");
  if (is_fp32(precision) && (int64_t)pb->nx * pb->ny * pb->q * (pb->p + 1) * (pb->p + 1) >= ((int64_t)1 << 31))
    return fail(nullptr, DGBGK_ENOTSUP, "FP32 path: more than 2^31 degrees of freedom");
  dgbgk_solver *s = new (std::nothrow) dgbgk_solver;
  if (!s) return fail(nullptr, DGBGK_ENOMEM, "out of host memory");
  s->prec = precision;
  s->pb = *pb;
  s->Q = pb->q;
  s->ex.assign(pb->ex, pb->ex + pb->q);
  s->ey.assign(pb->ey, pb->ey + pb->q);
  s->w.assign(pb->w, pb->w + pb->q);
  s->pb.ex = s->ex.data();
  s->pb.ey = s->ey.data();
  s->pb.w = s->w.data();
  s->p = pb->p;
  s->Nfp = pb->p + 1;
  s->Np = s->Nfp * s->Nfp;
  s->K = (int64_t)pb->nx * pb->ny;
  s->hx = pb->lx / pb->nx;
  s->hy = pb->ly / pb->ny;
  s->stream = (hipStream_t)hip_stream;
  // reference element
  gll_points(s->p, s->r);
  differentiation_matrix(s->r, s->D1);
  mass_matrix(s->r, s->M1);
  std::vector<double> e0(s->Nfp, 0.0), ep(s->Nfp, 0.0);
  e0[0] = 1.0;
  ep[s->p] = 1.0;
  if (!spd_solve(s->Nfp, s->M1, e0, s->lift_lo) || !spd_solve(s->Nfp, s->M1, ep, s->lift_hi)) {
    delete s;
    return fail(nullptr, DGBGK_EINVAL, "mass matrix is not positive definite");
  }
  // walls: exterior equilibria f^eq(1, u_b) and the incoming-flux normalisation of eq. (8)
  const double nrm[4][2] = {{0, -1}, {1, 0}, {0, 1}, {-1, 0}};
  const double th = pb->theta;
  s->feqb.assign((size_t)4 * s->Q, 0.0);
  double umax = 0.0;
  for (int sd = 0; sd < 4; ++sd) {
    const double ubx = pb->wall_u[sd][0], uby = pb->wall_u[sd][1];
    const double usq = ubx * ubx + uby * uby;
    double den = 0.0;
    for (int q = 0; q < s->Q; ++q) {
      const double eu = s->ex[q] * ubx + s->ey[q] * uby;
      const double fe = s->w[q] * (1.0 + eu / th + eu * eu / (2.0 * th * th) - usq / (2.0 * th));
      s->feqb[(size_t)sd * s->Q + q] = fe;
      const double cn = s->ex[q] * nrm[sd][0] + s->ey[q] * nrm[sd][1];
      if (cn < 0.0) den += -cn * fe;
    }
    s->wall_den[sd] = den;
    s->wall_den_inv[sd] = den > 0.0 ? 1.0 / den : 0.0;
    if (pb->bc[sd] == DGBGK_BC_DIFFUSE_WALL) {
      s->wall_mask |= 1 << sd;
      if (!(den > 0.0)) {
        delete s;
        return fail(nullptr, DGBGK_EINVAL, "wall %d has no incoming velocity", sd);
      }
      umax = std::fmax(umax, std::sqrt(usq));
    }
  }
  const double uref = umax > 0.0 ? umax : 1.0;
  s->resid_scale = std::fmin(pb->lx, pb->ly) / uref;
  // constant part of the moments of f = g + w rho_ref (FP32 precisions)
  for (int q = 0; q < s->Q; ++q) {
    const double cx = s->ex[q], cy = s->ey[q], wr = s->w[q] * s->rho_ref;
    const double W[7] = {1.0, cx, cy, cy < 0.0 ? -cy : 0.0, cx > 0.0 ? cx : 0.0,
                         cy > 0.0 ? cy : 0.0, cx < 0.0 ? -cx : 0.0};
    for (int c = 0; c < 7; ++c) s->mconst[c] += W[c] * wr;
  }
  s->lay = make_layout(s->K, s->Np, s->Nfp, s->Q, precision);
  if (is_ref(precision)) {
    // the reference's right-hand side runs the FP64 kernel in its own decomposition
    s->prec = DGBGK_FP64;
    choose_tiling(s);
    s->ref64.fused = s->fused;
    s->ref64.E = s->E;
    s->ref64.log2E = s->log2E;
    s->ref64.Qt = s->Qt;
    s->ref64.ntiles = s->ntiles;
    s->ref64.nblk = s->nblk;
    s->ref64.lds = s->lds;
    s->prec = precision;
  }
  choose_tiling(s);
  if (is_fp32(precision) && s->lds > 160 * 1024) {
    delete s;
    return fail(nullptr, DGBGK_ENOTSUP, "FP32 path: one element's velocities do not fit in LDS");
  }
  *out = s;
  return DGBGK_OK;
}

int dgbgk_bind_buffers(dgbgk_solver *s, void *device_ptr, size_t bytes) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (s->dev_ready || s->base) return fail(s, DGBGK_ESTATE, "device memory already in use");
  if (!device_ptr) return fail(s, DGBGK_EINVAL, "device_ptr is NULL");
  if ((uintptr_t)device_ptr % kAlign) return fail(s, DGBGK_EINVAL, "device_ptr must be 256-byte aligned");
  if (bytes < s->lay.total)
    return fail(s, DGBGK_EINVAL, "buffer of %zu B is smaller than the %zu B required", bytes,
                s->lay.total);
  s->base = device_ptr;
  s->owns = false;
  return ensure_device(s);
}

int dgbgk_set_stream(dgbgk_solver *s, void *hip_stream) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  hipStream_t ns = (hipStream_t)hip_stream;
  if (ns != s->stream && s->dev_ready) {
    // work enqueued on the new stream must not overtake the stages still in
    // flight on the old one (they read and write the same registers)
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, s->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(ns, ev, 0);
    if (ev) (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(s, e, "ordering the new stream after the old one");
  }
  s->stream = ns;
  return DGBGK_OK;
}

void dgbgk_destroy(dgbgk_solver *s) {
  if (!s) return;
  if (s->gexec) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipGraphExecDestroy(s->gexec);
  }
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->owns && s->base) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->base);
  }
  if (s->imp_ws) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->imp_ws);
  }
  delete s;
}

int dgbgk_sizes(const dgbgk_solver *s, int64_t *K, int32_t *Np, int32_t *Nfp, int32_t *Q) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (K) *K = s->K;
  if (Np) *Np = s->Np;
  if (Nfp) *Nfp = s->Nfp;
  if (Q) *Q = s->Q;
  return DGBGK_OK;
}

int dgbgk_stable_dt(const dgbgk_solver *s, double cfl, double *dt) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  dgbgk_solver *m = const_cast<dgbgk_solver *>(s);
  if (!dt || !(cfl > 0) || !is_finite_d(cfl)) return fail(m, DGBGK_EINVAL, "cfl must be > 0");
  double dr = 2.0;
  for (int i = 0; i < s->p; ++i) dr = std::fmin(dr, s->r[i + 1] - s->r[i]);
  double vmax = 0.0;
  for (int q = 0; q < s->Q; ++q) vmax = std::fmax(vmax, std::fabs(s->ex[q]) + std::fabs(s->ey[q]));
  if (!(vmax > 0)) return fail(m, DGBGK_EINVAL, "all velocities are zero");
  *dt = cfl * (0.5 * std::fmin(s->hx, s->hy)) * dr / vmax;
  return DGBGK_OK;
}

int dgbgk_node_coords(const dgbgk_solver *s, double *x, double *y) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!x || !y) return fail(const_cast<dgbgk_solver *>(s), DGBGK_EINVAL, "NULL output");
  const int N1 = s->Nfp;
  for (int64_t k = 0; k < s->K; ++k) {
    const int64_t kx = k % s->pb.nx, ky = k / s->pb.nx;
    for (int n = 0; n < s->Np; ++n) {
      const int i = n % N1, j = n / N1;
      x[k * s->Np + n] = s->pb.x0 + s->hx * ((double)kx + 0.5 * (1.0 + s->r[i]));
      y[k * s->Np + n] = s->pb.y0 + s->hy * ((double)ky + 0.5 * (1.0 + s->r[j]));
    }
  }
  return DGBGK_OK;
}

int dgbgk_get_operator(const dgbgk_solver *s, int32_t which, double *out) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!out) return fail(const_cast<dgbgk_solver *>(s), DGBGK_EINVAL, "NULL output");
  const int N1 = s->Nfp, Np = s->Np, Nfp = s->Nfp;
  switch (which) {
    case 0:  // Dr = I (x) D1 acting on i
    case 1:  // Ds = D1 (x) I acting on j
      for (int a = 0; a < Np; ++a)
        for (int b = 0; b < Np; ++b) {
          const int ia = a % N1, ja = a / N1, ib = b % N1, jb = b / N1;
          double v = 0.0;
          if (which == 0 && ja == jb) v = s->D1[ia * N1 + ib];
          if (which == 1 && ia == ib) v = s->D1[ja * N1 + jb];
          out[a * Np + b] = v;
        }
      return DGBGK_OK;
    case 2:
      for (int a = 0; a < Np; ++a)
        for (int b = 0; b < Np; ++b)
          out[a * Np + b] = s->M1[(a % N1) * N1 + (b % N1)] * s->M1[(a / N1) * N1 + (b / N1)];
      return DGBGK_OK;
    case 3:
      for (int a = 0; a < Np * 4 * Nfp; ++a) out[a] = 0.0;
      for (int nd = 0; nd < Np; ++nd) {
        const int i = nd % N1, j = nd / N1;
        out[nd * 4 * Nfp + 0 * Nfp + i] = s->lift_lo[j];  // bottom face, node i of the face
        out[nd * 4 * Nfp + 1 * Nfp + j] = s->lift_hi[i];  // right face
        out[nd * 4 * Nfp + 2 * Nfp + i] = s->lift_hi[j];  // top face
        out[nd * 4 * Nfp + 3 * Nfp + j] = s->lift_lo[i];  // left face
      }
      return DGBGK_OK;
    case 4: std::memcpy(out, s->r.data(), sizeof(double) * N1); return DGBGK_OK;
    case 5: std::memcpy(out, s->M1.data(), sizeof(double) * N1 * N1); return DGBGK_OK;
    case 6:
      out[0] = 2.0 / s->hy; out[1] = 2.0 / s->hx; out[2] = 2.0 / s->hy; out[3] = 2.0 / s->hx;
      return DGBGK_OK;
    case 7: std::memcpy(out, s->D1.data(), sizeof(double) * N1 * N1); return DGBGK_OK;
    default: return fail(const_cast<dgbgk_solver *>(s), DGBGK_EINVAL, "unknown operator %d", which);
  }
}

int dgbgk_init_equilibrium(dgbgk_solver *s, double rho0, double ux0, double uy0) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!(rho0 > 0) || !is_finite_d(rho0) || !is_finite_d(ux0) || !is_finite_d(uy0))
    return fail(s, DGBGK_EINVAL, "rho0 must be > 0 and u0 finite");
  int rc = ensure_device(s);
  if (rc) return rc;
  hipError_t e =
      is_ref(s->prec)
          ? launch_init_equilibrium(s->d_fref, s->d_vel, (int)s->K, s->Np, s->Q, rho0, ux0, uy0,
                                    s->pb.theta, s->stream)
      : is_fp32(s->prec)
          ? launch_init_equilibrium32(s->g_fn, s->d_vel, (int)s->K, s->Np, s->Q, rho0, ux0, uy0,
                                      s->pb.theta, s->rho_ref, s->stream)
          : launch_init_equilibrium(s->d_fn, s->d_vel, (int)s->K, s->Np, s->Q, rho0, ux0, uy0,
                                    s->pb.theta, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "init kernel");
  if (is_ref(s->prec) && (rc = ref_reset(s))) return rc;
  s->have_state = true;
  s->part_valid = false;
  s->steps = 0;
  return DGBGK_OK;
}

int dgbgk_init_moments(dgbgk_solver *s, const double *rho, const double *ux, const double *uy,
                       size_t count) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  const size_t KN = (size_t)s->K * s->Np;
  if (!rho || !ux || !uy || count != KN) return fail(s, DGBGK_EINVAL, "arrays need %zu doubles", KN);
  for (size_t i = 0; i < KN; ++i)
    if (!(rho[i] > 0) || !is_finite_d(rho[i]) || !is_finite_d(ux[i]) || !is_finite_d(uy[i]))
      return fail(s, DGBGK_EINVAL, "node %zu: rho must be > 0 and u finite", i);
  int rc = ensure_device(s);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(s->d_mom, rho, KN * sizeof(double), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_mom + KN, ux, KN * sizeof(double), hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_mom + 2 * KN, uy, KN * sizeof(double), hipMemcpyHostToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "moments copy");
  e = is_ref(s->prec)
          ? launch_init_moments(s->d_fref, s->d_vel, s->d_mom, (int)s->K, s->Np, s->Q, s->pb.theta,
                                s->stream)
      : is_fp32(s->prec)
          ? launch_init_moments32(s->g_fn, s->d_vel, s->d_mom, (int)s->K, s->Np, s->Q, s->pb.theta,
                                  s->rho_ref, s->stream)
          : launch_init_moments(s->d_fn, s->d_vel, s->d_mom, (int)s->K, s->Np, s->Q, s->pb.theta,
                                s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // the host arrays may go away
  if (e != hipSuccess) return hip_fail(s, e, "init kernel");
  if (is_ref(s->prec)) {
    int rc2 = ref_reset(s);
    if (!rc2) {
      e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) rc2 = hip_fail(s, e, "reference set-up");
    }
    if (rc2) return rc2;
  }
  s->have_state = true;
  s->part_valid = false;
  s->steps = 0;
  return DGBGK_OK;
}

int dgbgk_set_state(dgbgk_solver *s, const double *f, size_t count) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  const size_t need = (size_t)s->K * s->Np * s->Q;
  if (!f || count != need) return fail(s, DGBGK_EINVAL, "state needs %zu doubles", need);
  int rc = ensure_device(s);
  if (rc) return rc;
  // host order f[q][k][n] into a staging buffer, then element-major into f_n
  hipError_t e;
  if (is_ref(s->prec)) {
    e = hipMemcpyAsync(s->d_xfer, f, need * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = launch_transpose(s->d_xfer, s->d_fref, (int)s->K, s->Np, s->Q, 1, s->stream);
    if (e == hipSuccess) {
      // the transfer buffer is reused by the reference's right-hand side
      e = hipStreamSynchronize(s->stream);
      if (e == hipSuccess && (rc = ref_reset(s))) return rc;
    }
  } else if (is_fp32(s->prec)) {
    e = hipMemcpyAsync(s->d_xfer, f, need * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
      e = launch_to_dev32(s->d_xfer, s->g_fn, s->d_vel, (int)s->K, s->Np, s->Q, s->rho_ref, s->stream);
  } else {
    e = hipMemcpyAsync(s->d_b, f, need * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = launch_transpose(s->d_b, s->d_fn, (int)s->K, s->Np, s->Q, 1, s->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "set_state copy");
  s->have_state = true;
  s->part_valid = false;
  s->steps = 0;
  return DGBGK_OK;
}

int dgbgk_get_state(dgbgk_solver *s, double *f, size_t count) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  const size_t need = (size_t)s->K * s->Np * s->Q;
  if (!f || count != need) return fail(s, DGBGK_EINVAL, "state needs %zu doubles", need);
  if (!s->have_state) return fail(s, DGBGK_ESTATE, "no state: call init or set_state first");
  double *stage = is_fp32(s->prec) ? s->d_xfer : s->d_b;
  hipError_t e = is_ref(s->prec)
                     ? launch_from_ref(s->d_fref, s->g_fn, stage, (int)s->K, s->Np, s->Q, s->stream)
                 : is_fp32(s->prec)
                     ? launch_from_dev32(s->g_fn, stage, s->d_vel, (int)s->K, s->Np, s->Q, s->rho_ref,
                                         s->stream)
                     : launch_transpose(s->d_fn, stage, (int)s->K, s->Np, s->Q, 0, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(f, stage, need * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "get_state copy");
  return DGBGK_OK;
}

int dgbgk_state_device_ptr(dgbgk_solver *s, void **ptr) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!ptr) return fail(s, DGBGK_EINVAL, "ptr is NULL");
  int rc = ensure_device(s);
  if (rc) return rc;
  *ptr = is_fp32(s->prec) ? (void *)s->g_fn : (void *)s->d_fn;
  return DGBGK_OK;
}

}  // extern "C"

namespace {

// Whether the stages hand moment partials to the next (see stage_partials).
bool uses_partials(const dgbgk_solver *s) {
  if (!s->d_part[0]) return false;
  if (is_fp32(s->prec))  // (16-byte rows: Q Np is a multiple of 4 at these orders)
    return s->fused && s->E == 1 && handoff_moments(s->p) && ((int64_t)s->Q * s->Np) % 4 == 0;
  if (!s->fused) return s->ntiles <= kMaxPartialTiles;
  return s->E == 1 && !s->persistent && handoff_moments(s->p);
}

// Velocity-tiled FP64 stages, and fused ones of one element per work-group
// (orders 1 and 3), hand the moment partials of their output to the next
// stage.  Slots: stage 1 reads P0 and writes P1, then P1 -> P0, P0 -> P1,
// P1 -> P0, so P0 holds the partials of f_n between steps (stage 0 reads it).
void stage_partials(const dgbgk_solver *s, int stage, const double *&pin, double *&pout) {
  pin = nullptr;
  pout = nullptr;
  if (!uses_partials(s)) return;
  double *P0 = s->d_part[0], *P1 = s->d_part[1];
  const bool odd = stage == 1 || stage == 3;
  pin = stage == 2 || stage == 4 ? P1 : P0;
  if (stage != 0) pout = odd ? P1 : P0;
}

// The partials of f_n in P0 (the full moment rows in tile 0, zeros in the
// others) where they are stale: after f_n was set from outside a step.
int ensure_partials(dgbgk_solver *s) {
  if (!uses_partials(s) || s->part_valid) return DGBGK_OK;
  hipError_t e =
      is_fp32(s->prec)
          ? launch_moment_rows32(s->g_fn, s->d_vel, (int)s->K, s->Np, s->Q, s->d_part[0], s->stream)
          : launch_moment_rows(s->d_fn, s->d_vel, (int)s->K, s->Np, s->Q, s->fused ? 1 : s->ntiles,
                               s->d_part[0], s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "moment rows kernel");
  s->part_valid = true;
  return DGBGK_OK;
}

// One RK4 step.  Registers: f_n, acc, and two stage buffers A/B so that a
// stage never overwrites the state its neighbours still read.
int enqueue_rk4_step(dgbgk_solver *s, double dt) {
  int rc;
  void *fn = s->d_fn, *A = s->d_a, *B = s->d_b;
  if (uses_partials(s)) {
    if ((rc = ensure_partials(s))) return rc;
    void *const io[5] = {fn, A, B, A, fn};
    for (int st = 1; st <= 4; ++st) {
      const double *pin;
      double *pout;
      stage_partials(s, st, pin, pout);
      if ((rc = run_stage(s, st, io[st - 1], io[st], dt, nullptr, pin, pout))) {
        s->part_valid = false;
        return rc;
      }
    }
    return DGBGK_OK;
  }
  if ((rc = run_stage(s, 1, fn, A, dt))) return rc;
  if ((rc = run_stage(s, 2, A, B, dt))) return rc;
  if ((rc = run_stage(s, 3, B, A, dt))) return rc;
  return run_stage(s, 4, A, fn, dt);
}

void drop_solver_graph(dgbgk_solver *s) {
  if (s->gexec) {
    (void)hipStreamSynchronize(s->stream);  // replays in flight still use it
    (void)hipGraphExecDestroy(s->gexec);
  }
  s->gexec = nullptr;
}

// Captures graph_steps RK4 steps of size dt on the capture stream.
int capture_solver_graph(dgbgk_solver *s, double dt) {
  drop_solver_graph(s);
  hipError_t e = hipSuccess;
  if (!s->cap_stream) e = hipStreamCreate(&s->cap_stream);
  if (e != hipSuccess) return hip_fail(s, e, "capture stream");
  // the capture stream starts after the solver's stream (set-up work on it)
  hipEvent_t ev = nullptr;
  e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev, s->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(s->cap_stream, ev, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(s->cap_stream);
  if (ev) (void)hipEventDestroy(ev);
  if (e != hipSuccess) return hip_fail(s, e, "capture stream ordering");
  hipStream_t own = s->stream;
  s->stream = s->cap_stream;
  e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
  int rc = DGBGK_OK;
  if (e == hipSuccess)
    for (int i = 0; i < s->graph_steps && !rc; ++i) rc = enqueue_rk4_step(s, dt);
  hipGraph_t g = nullptr;
  hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(s->cap_stream, &g) : e;
  s->stream = own;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e2 == hipSuccess) e2 = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) {
    s->gexec = nullptr;
    return hip_fail(s, e2, "graph capture");
  }
  s->graph_dt = dt;
  const int cfg[5] = {s->fused, s->E, s->Qt, s->persistent, s->prec};
  std::memcpy(s->graph_cfg, cfg, sizeof cfg);
  s->graph_partials = uses_partials(s);
  return DGBGK_OK;
}

}  // namespace

extern "C" {

int dgbgk_set_graph(dgbgk_solver *s, int32_t steps_per_graph) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (steps_per_graph < 0 || steps_per_graph > 1000)
    return fail(s, DGBGK_EINVAL, "steps_per_graph must be in 0..1000");
  if (steps_per_graph != s->graph_steps) drop_solver_graph(s);
  s->graph_steps = steps_per_graph;
  return DGBGK_OK;
}

int dgbgk_step(dgbgk_solver *s, int64_t nsteps, double dt) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (nsteps < 0 || !(dt > 0) || !is_finite_d(dt)) return fail(s, DGBGK_EINVAL, "need nsteps >= 0, dt > 0");
  if (!s->have_state) return fail(s, DGBGK_ESTATE, "no state: call init or set_state first");
  int rc = ensure_device(s);
  if (rc) return rc;
  int64_t it = 0;
  if (s->graph_steps > 0 && nsteps >= s->graph_steps) {
    const int cfg[5] = {s->fused, s->E, s->Qt, s->persistent, s->prec};
    if (!s->gexec || s->graph_dt != dt || std::memcmp(cfg, s->graph_cfg, sizeof cfg) != 0 ||
        (s->graph_partials && !s->part_valid)) {
      // one eager step first: it sets the kernels' LDS attributes outside the capture
      if ((rc = enqueue_rk4_step(s, dt))) return rc;
      ++s->steps;
      ++it;
      if ((rc = capture_solver_graph(s, dt))) return rc;
    }
    for (; it + s->graph_steps <= nsteps; it += s->graph_steps) {
      hipError_t e = hipGraphLaunch(s->gexec, s->stream);
      if (e != hipSuccess) return hip_fail(s, e, "graph launch");
      s->steps += s->graph_steps;
    }
  }
  for (; it < nsteps; ++it) {
    if ((rc = enqueue_rk4_step(s, dt))) return rc;
    ++s->steps;
  }
  return DGBGK_OK;
}

int dgbgk_rhs(dgbgk_solver *s, const double *f, double *k, size_t count) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  const size_t need = (size_t)s->K * s->Np * s->Q;
  if (!f || !k || count != need) return fail(s, DGBGK_EINVAL, "arrays need %zu doubles", need);
  int rc = ensure_device(s);
  if (rc) return rc;
  hipError_t e;
  if (is_fp32(s->prec)) {
    if (is_ref(s->prec) && !s->have_state)
      return fail(s, DGBGK_ESTATE, "the reference form evaluates L(f) as a correction to its "
                                   "reference: call init or set_state first");
    e = hipMemcpyAsync(s->d_xfer, f, need * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
      e = is_ref(s->prec)
              ? launch_to_ref(s->d_xfer, s->d_fref, s->g_a, (int)s->K, s->Np, s->Q, s->stream)
              : launch_to_dev32(s->d_xfer, s->g_a, s->d_vel, (int)s->K, s->Np, s->Q, s->rho_ref,
                                s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "rhs input copy");
    if ((rc = run_stage(s, 0, s->g_a, s->g_b, 0.0))) return rc;
    e = launch_from_dev32(s->g_b, s->d_xfer, s->d_vel, (int)s->K, s->Np, s->Q, 0.0, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(k, s->d_xfer, need * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  } else {
    e = hipMemcpyAsync(s->d_b, f, need * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = launch_transpose(s->d_b, s->d_a, (int)s->K, s->Np, s->Q, 1, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "rhs input copy");
    if ((rc = run_stage(s, 0, s->d_a, s->d_b, 0.0))) return rc;
    e = launch_transpose(s->d_b, s->d_a, (int)s->K, s->Np, s->Q, 0, s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(k, s->d_a, need * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "rhs output copy");
  return DGBGK_OK;
}

int dgbgk_wall_density(dgbgk_solver *s, const double *f, double *out, size_t count) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  const size_t need = (size_t)s->K * s->Np * s->Q;
  const size_t nout = (size_t)s->K * 4 * s->Nfp;
  if (!f || !out || count != need) return fail(s, DGBGK_EINVAL, "state needs %zu doubles", need);
  if (is_ref(s->prec))
    return fail(s, DGBGK_ENOTSUP, "the reference form forms wall densities of its correction only");
  int rc = ensure_device(s);
  if (rc) return rc;
  const bool f32 = is_fp32(s->prec);
  hipError_t e = hipMemcpyAsync(f32 ? s->d_xfer : s->d_b, f, need * sizeof(double),
                                hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = f32 ? launch_to_dev32(s->d_xfer, s->g_a, s->d_vel, (int)s->K, s->Np, s->Q, s->rho_ref,
                              s->stream)
            : launch_transpose(s->d_b, s->d_a, (int)s->K, s->Np, s->Q, 1, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "wall_density input copy");
  e = launch_fill_u64((unsigned long long *)s->d_rhow, nout, 0ull, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "fill kernel");
  if ((rc = run_stage(s, 0, f32 ? (void *)s->g_a : (void *)s->d_a, f32 ? (void *)s->g_b : (void *)s->d_b,
                      0.0, s->fused ? s->d_rhow : nullptr)))
    return rc;
  e = hipMemcpyAsync(out, s->d_rhow, nout * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "wall_density output copy");
  return DGBGK_OK;
}

static int residual_enqueue(dgbgk_solver *s) {
  int rc = ensure_partials(s);
  if (rc) return rc;
  const double *pin;
  double *pout;
  stage_partials(s, 0, pin, pout);
  if ((rc = run_stage(s, 0, s->d_fn, s->d_b, 0.0, nullptr, pin))) return rc;
  hipError_t e = launch_fill_u64(s->d_u64, 1, 0ull, s->stream);
  if (e == hipSuccess)
    e = is_fp32(s->prec)
            ? launch_residual32(s->g_b, s->d_vel, (int)s->K, s->Np, s->Q, s->resid_scale, s->d_u64,
                                s->stream)
            : launch_residual(s->d_b, s->d_vel, (int)s->K, s->Np, s->Q, s->resid_scale, s->d_u64,
                              s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "residual kernel");
  return DGBGK_OK;
}

int dgbgk_residual(dgbgk_solver *s, double *r) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!r) return fail(s, DGBGK_EINVAL, "r is NULL");
  if (!s->have_state) return fail(s, DGBGK_ESTATE, "no state: call init or set_state first");
  int rc = residual_enqueue(s);
  if (rc) return rc;
  unsigned long long bits = 0;
  hipError_t e = hipMemcpyAsync(&bits, s->d_u64, sizeof bits, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "residual copy");
  double v;
  std::memcpy(&v, &bits, sizeof v);
  *r = v;
  if (!std::isfinite(v)) {
    *r = NAN;
    return fail(s, DGBGK_ENONFINITE, "residual is not finite");
  }
  return DGBGK_OK;
}

int dgbgk_residual_async(dgbgk_solver *s, double *device_out) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!device_out) return fail(s, DGBGK_EINVAL, "device_out is NULL");
  if (!s->have_state) return fail(s, DGBGK_ESTATE, "no state: call init or set_state first");
  int rc = residual_enqueue(s);
  if (rc) return rc;
  hipError_t e = launch_u64_to_f64(s->d_u64, device_out, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "residual convert kernel");
  return DGBGK_OK;
}

int dgbgk_moments(dgbgk_solver *s, double *rho, double *ux, double *uy) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!rho || !ux || !uy) return fail(s, DGBGK_EINVAL, "NULL output");
  if (!s->have_state) return fail(s, DGBGK_ESTATE, "no state: call init or set_state first");
  const size_t KN = (size_t)s->K * s->Np;
  hipError_t e = hipSuccess;
  if (is_ref(s->prec)) {  // f = f_ref + g in FP64 (transfer buffer), then the FP64 moments
    e = launch_ref_sum(s->d_fref, s->g_fn, s->d_xfer, KN * s->Q, s->stream);
    if (e == hipSuccess)
      e = launch_moments(s->d_xfer, s->d_vel, (int)s->K, s->p, s->Q, s->pb.nx, s->pb.ny, 0,
                         s->wall_den_inv, s->d_mom, s->d_mom + KN, s->d_mom + 2 * KN, nullptr,
                         s->stream);
  } else
    e =
      is_fp32(s->prec)
          ? launch_moments32(s->g_fn, s->d_vel, (int)s->K, s->Np, s->Q, s->rho_ref, s->d_mom,
                             s->d_mom + KN, s->d_mom + 2 * KN, s->stream)
          : launch_moments(s->d_fn, s->d_vel, (int)s->K, s->p, s->Q, s->pb.nx, s->pb.ny, 0,
                           s->wall_den_inv, s->d_mom, s->d_mom + KN, s->d_mom + 2 * KN, nullptr,
                           s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(rho, s->d_mom, KN * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(ux, s->d_mom + KN, KN * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(uy, s->d_mom + 2 * KN, KN * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "moments");
  for (size_t i = 0; i < KN; ++i)
    if (!std::isfinite(rho[i]) || !std::isfinite(ux[i]) || !std::isfinite(uy[i]))
      return fail(s, DGBGK_ENONFINITE, "moment at node %zu is not finite", i);
  return DGBGK_OK;
}

int dgbgk_fold(dgbgk_solver *s) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!is_ref(s->prec)) return fail(s, DGBGK_ENOTSUP, "only the reference form has a correction to fold");
  if (!s->have_state) return fail(s, DGBGK_ESTATE, "no state: call init or set_state first");
  hipError_t e = launch_ref_fold(s->d_fref, s->g_fn, (size_t)s->K * s->Np * s->Q, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "fold kernel");
  s->part_valid = false;  // the correction is zero now
  return ref_refresh(s);
}

int dgbgk_synchronize(dgbgk_solver *s) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!s->dev_ready) return DGBGK_OK;
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "synchronize");
  return DGBGK_OK;
}

int dgbgk_steps_taken(const dgbgk_solver *s, int64_t *steps) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (!steps) return fail(const_cast<dgbgk_solver *>(s), DGBGK_EINVAL, "steps is NULL");
  *steps = s->steps;
  return DGBGK_OK;
}

int dgbgk_set_tiling(dgbgk_solver *s, int32_t mode, int32_t velocities_per_tile) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (mode < 0 || mode > 4) return fail(s, DGBGK_EINVAL, "mode must be 0..4");
  if (is_fp32(s->prec) && (mode == 2 || mode == 4))
    return fail(s, DGBGK_ENOTSUP, "the FP32 precisions run the fused per-block form only");
  if (velocities_per_tile < 0) return fail(s, DGBGK_EINVAL, "velocities_per_tile must be >= 0");
  const int saved_mode = s->tiling_mode, saved_qt = s->tiling_qt;
  s->tiling_mode = mode;
  s->tiling_qt = velocities_per_tile;
  choose_tiling(s);
  if (mode == 4 && !s->persistent) {
    s->tiling_mode = saved_mode;
    s->tiling_qt = saved_qt;
    choose_tiling(s);
    return fail(s, DGBGK_EINVAL, "the persistent kernel does not apply to this problem");
  }
  if (s->fused && s->lds > 160 * 1024) {
    s->tiling_mode = saved_mode;
    s->tiling_qt = saved_qt;
    choose_tiling(s);
    return fail(s, DGBGK_EINVAL, "fused tile does not fit in LDS");
  }
  return DGBGK_OK;
}

int dgbgk_get_tiling(const dgbgk_solver *s, int32_t *fused, int32_t *elems_per_group,
                     int32_t *velocities_per_tile, size_t *lds_bytes) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (fused) *fused = s->fused ? (s->persistent ? 2 : 1) : 0;
  if (elems_per_group) *elems_per_group = s->E;
  if (velocities_per_tile) *velocities_per_tile = s->Qt;
  if (lds_bytes) *lds_bytes = s->lds;
  return DGBGK_OK;
}

}  // extern "C"

// ---- block size, autotuner -----------------------------------------------------

namespace {

// Whether the current configuration of s is one the kernels accept.
bool tiling_admissible(const dgbgk_solver *s) {
  if (s->lds > 160 * 1024) return false;
  if (s->E < 1 || s->E > s->K || (s->E & (s->E - 1)) != 0) return false;
  if (!is_fp32(s->prec) && s->fused && (int64_t)s->E * s->Np > kBlock) return false;
  return true;
}

}  // namespace

extern "C" {

int dgbgk_set_block_elements(dgbgk_solver *s, int32_t elems_per_group) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (elems_per_group < 0) return fail(s, DGBGK_EINVAL, "elems_per_group must be >= 0");
  const int saved = s->forced_E;
  s->forced_E = elems_per_group;
  choose_tiling(s);
  if (!tiling_admissible(s)) {
    s->forced_E = saved;
    choose_tiling(s);
    return fail(s, DGBGK_EINVAL, "%d elements per work-group: the tile does not fit",
                elems_per_group);
  }
  return DGBGK_OK;
}

int dgbgk_autotune(dgbgk_solver *s, int32_t launches, double *best_us) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  if (launches < 1) return fail(s, DGBGK_EINVAL, "launches must be >= 1");
  if (!s->have_state) return fail(s, DGBGK_ESTATE, "no state: call init or set_state first");
  int rc = ensure_device(s);
  if (rc) return rc;
  // candidates: (forced_E, tiling_mode, tiling_qt)
  struct Cand { int E, mode, qt; };
  std::vector<Cand> cands;
  // a caller that forced the fused form (mode 1 or 3) keeps it
  const bool fused_only = s->tiling_mode == 1 || s->tiling_mode == 3;
  const int fmode = fused_only ? s->tiling_mode : 0;
  for (int E = 1; E <= s->K && E <= 64; E *= 2) cands.push_back({E, fmode, 0});
  if (!is_fp32(s->prec) && !fused_only)
    for (int qt = s->Q; qt >= 8; qt = (qt + 1) / 2) cands.push_back({0, 2, qt});
  const int sE = s->forced_E, sm = s->tiling_mode, sq = s->tiling_qt;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(s, e, "autotune events");
  double best = -1.0;
  Cand pick{sE, sm, sq};
  void *out = s->d_b;  // stage buffer: the state is only read
  for (const Cand &c : cands) {
    s->forced_E = c.E;
    s->tiling_mode = c.mode;
    s->tiling_qt = c.qt;
    choose_tiling(s);
    if (!tiling_admissible(s)) continue;
    if (c.mode == 2 && s->fused) continue;
    if ((rc = run_stage(s, 0, s->d_fn, out, 0.0))) break;  // warm-up
    e = hipEventRecord(e0, s->stream);
    for (int i = 0; i < launches && e == hipSuccess && !rc; ++i) rc = run_stage(s, 0, s->d_fn, out, 0.0);
    if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess || rc) break;
    const double us = 1000.0 * ms / launches;
    if (best < 0.0 || us < best) {
      best = us;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->forced_E = pick.E;
  s->tiling_mode = pick.mode;
  s->tiling_qt = pick.qt;
  choose_tiling(s);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(s, e, "autotune timing");
  if (best < 0.0) return fail(s, DGBGK_ENOTSUP, "no admissible configuration");
  if (best_us) *best_us = best;
  return DGBGK_OK;
}

}  // extern "C"

// ---- implicit SDIRK steps: Newton's method with matrix-free GMRES ---------

namespace {

// Stiffly accurate SDIRK tableaus (lower triangle of A, diagonal gamma);
// f_{n+1} is the last stage value.
struct Sdirk {
  int stages = 0;
  double gamma = 0.0;
  double a[5][5] = {};
};

bool sdirk_tableau(int scheme, Sdirk &t) {
  t = Sdirk{};
  switch (scheme) {
    case DGBGK_BACKWARD_EULER:
      t.stages = 1;
      t.gamma = 1.0;
      break;
    case DGBGK_SDIRK2: {  // Alexander (1977), two stages, L-stable
      const double g = 1.0 - std::sqrt(0.5);
      t.stages = 2;
      t.gamma = g;
      t.a[1][0] = 1.0 - g;
      break;
    }
    case DGBGK_SDIRK4:  // Hairer-Wanner, five stages, order 4, L-stable
      t.stages = 5;
      t.gamma = 0.25;
      t.a[1][0] = 0.5;
      t.a[2][0] = 17.0 / 50.0;
      t.a[2][1] = -1.0 / 25.0;
      t.a[3][0] = 371.0 / 1360.0;
      t.a[3][1] = -137.0 / 2720.0;
      t.a[3][2] = 15.0 / 544.0;
      t.a[4][0] = 25.0 / 24.0;
      t.a[4][1] = -49.0 / 48.0;
      t.a[4][2] = 125.0 / 16.0;
      t.a[4][3] = -85.0 / 12.0;
      break;
    default:
      return false;
  }
  for (int i = 0; i < t.stages; ++i) t.a[i][i] = t.gamma;
  return true;
}

// Relative step of the forward differences J v ~ (L(y + e v) - L(y)) / e.
// The rounding error of an evaluation of L is relative to its transport terms
// (|D f|), which near uniform or steady states exceed |L| by orders of
// magnitude, so the usual sqrt(machine epsilon) would leave that error
// amplified by 1e8; 1e-6 balances it against the truncation error of the
// quadratic equilibrium.
constexpr double kFdStep = 1e-6;

// First GMRES cycle length.  On the 64x64 p = 3 cavity the Krylov iteration
// count barely depends on the cycle length between 3 and 45 at moderate
// steps, while each iteration's Gram-Schmidt traffic grows with it; at very
// large steps short cycles stagnate, hence the doubling in gmres().
constexpr int kShortCycle = 8;

// Device workspace of one implicit step, in doubles: the stage rates, the
// Newton vectors, the Krylov basis and the small reduction buffers.
struct ImplicitWs {
  size_t n = 0, stride = 0;
  double *K = nullptr;  // stages x stride: L(y_i)
  double *y = nullptr, *b = nullptr, *F = nullptr, *T = nullptr, *X = nullptr;
  double *V = nullptr;  // (m + 1) x stride (FP64 basis)
  double *W = nullptr;  // the vector being orthogonalised (FP32 basis)
  float *V32 = nullptr;  // (m + 1) x stride floats (FP32 basis)
  double *dots = nullptr;   // multi-dot scratch
  double *small = nullptr;  // h1[m+1], h2[m+1], |w|^2, spare
  double *coef = nullptr;   // kMaxBasis coefficients uploaded from the host
};

size_t implicit_ws_bytes(size_t n, int stages, int m, bool v32, size_t *stride) {
  const size_t st = (n + 31) / 32 * 32;
  if (stride) *stride = st;
  const size_t vecs = (size_t)stages + 5 + (v32 ? 1 : (size_t)(m + 1));
  const size_t basis32 = v32 ? (size_t)(m + 1) * st / 2 : 0;  // st is even
  const size_t small = multi_dot_scratch(n, m + 1) + 2 * (size_t)(m + 1) + 8 + kMaxBasis;
  return (vecs * st + basis32 + small) * sizeof(double);
}

struct Implicit {
  dgbgk_solver *s;
  ImplicitWs w;
  int m;
  double h = 0.0;         // dt gamma of the current stage
  double eps = 0.0;       // finite-difference step for a unit vector
  int rhs_evals = 0;
  std::vector<double> host_small, host_coef;

  double *Vk(int k) const { return w.V + (size_t)k * w.stride; }
  float *Vk32(int k) const { return w.V32 + (size_t)k * w.stride; }

  int check(hipError_t e, const char *what) { return e == hipSuccess ? DGBGK_OK : hip_fail(s, e, what); }

  // x . y, synchronised to the host.
  int dot(const double *x, const double *y, double &out) {
    int rc = check(launch_multi_dot(w.n, 1, x, w.stride, y, w.dots, w.small + 2 * (m + 1), s->stream),
                   "dot kernel");
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(host_small.data(), w.small + 2 * (m + 1), sizeof(double),
                                  hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "dot copy");
    out = host_small[0];
    return DGBGK_OK;
  }

  int rhs(const double *in, double *out) {
    ++rhs_evals;
    return run_stage(s, 0, in, out, 0.0);
  }

  // out = v - h (L(y + e v) - L(y)) / e with e = eps / vnorm: the product of
  // (I - h J(y)) with v by a forward difference.  Ly = L(y); out != v.
  int apply(const double *v, double vnorm, const double *Ly, double *out) {
    const double e = eps / vnorm;
    int rc = check(launch_lincomb(w.n, 1.0, w.y, e, v, 0.0, nullptr, w.T, s->stream), "lincomb");
    if (!rc) rc = rhs(w.T, out);
    if (!rc)
      rc = check(launch_lincomb(w.n, -h / e, out, h / e, Ly, 1.0, v, out, s->stream), "lincomb");
    return rc;
  }

  // GMRES(m) for (I - h J) X = -F from X = 0, Givens rotations on the host.
  int gmres(const double *Ly, double fnorm2, double tol2, int max_it, int &iters) {
    const size_t n = w.n;
    std::vector<double> R((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), yv(m);
    int rc = check(launch_lincomb(n, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, w.X, s->stream), "zero");
    if (rc) return rc;
    double beta = fnorm2;
    // cycle length: short cycles while they make progress, doubled (up to
    // m) after a cycle that reduces the residual by less than 10%
    int mc = std::min(kShortCycle, m);
    rc = check(launch_lincomb(n, -1.0 / beta, w.F, 0.0, nullptr, 0.0, nullptr, Vk(0), s->stream),
               "lincomb");
    if (rc) return rc;
    bool done = false;
    while (!done) {
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int jn = 0;
      const double beta_cycle = beta;
      for (int j = 0; j < mc; ++j) {
        double *v1 = Vk(j + 1);
        if ((rc = apply(Vk(j), 1.0, Ly, v1))) return rc;
        // Classical Gram-Schmidt, repeated only when the first pass cancels
        // more than half of |w| (the "twice is enough" criterion).  V_0..V_j
        // and w = V_{j+1} are consecutive, so one multi-dot over j + 2
        // vectors gives the projections and |w|^2; without a second pass
        // |w'|^2 = |w|^2 - |h|^2 and the normalisation joins the update.
        double *h1 = w.small, *h2 = w.small + (m + 1);
        hipError_t e = launch_multi_dot(n, j + 2, w.V, w.stride, v1, w.dots, h1, s->stream);
        if (e == hipSuccess)
          e = hipMemcpyAsync(host_small.data(), h1, (size_t)(j + 2) * sizeof(double),
                             hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "Arnoldi projections");
        double *col = &R[(size_t)j * (m + 1)];
        double hh = 0.0;
        for (int i = 0; i <= j; ++i) {
          col[i] = host_small[i];
          hh += col[i] * col[i];
        }
        const double ww = host_small[j + 1];
        if (!std::isfinite(ww) || !std::isfinite(hh))
          return fail(s, DGBGK_ENONFINITE, "Krylov vector is not finite");
        double hn;
        if (ww - hh > 0.5 * ww) {
          hn = std::sqrt(ww - hh);
          e = launch_multi_axpy(n, j + 1, w.V, w.stride, h1, -1.0, v1, 1.0 / hn, v1, s->stream);
        } else {
          e = launch_multi_axpy(n, j + 1, w.V, w.stride, h1, -1.0, v1, 1.0, v1, s->stream);
          if (e == hipSuccess) e = launch_multi_dot(n, j + 2, w.V, w.stride, v1, w.dots, h2, s->stream);
          if (e == hipSuccess)
            e = hipMemcpyAsync(host_small.data(), h2, (size_t)(j + 2) * sizeof(double),
                               hipMemcpyDeviceToHost, s->stream);
          if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
          if (e != hipSuccess) return hip_fail(s, e, "Arnoldi reorthogonalisation");
          double hh2 = 0.0;
          for (int i = 0; i <= j; ++i) {
            col[i] += host_small[i];
            hh2 += host_small[i] * host_small[i];
          }
          hn = std::sqrt(std::max(host_small[j + 1] - hh2, 0.0));
          e = launch_multi_axpy(n, j + 1, w.V, w.stride, h2, -1.0, v1, hn > 0.0 ? 1.0 / hn : 1.0, v1,
                                s->stream);
        }
        if (e != hipSuccess) return hip_fail(s, e, "Arnoldi update");
        for (int i = 0; i < j; ++i) {
          const double a = col[i], b = col[i + 1];
          col[i] = cs[i] * a + sn[i] * b;
          col[i + 1] = -sn[i] * a + cs[i] * b;
        }
        const double den = std::hypot(col[j], hn);
        cs[j] = den > 0 ? col[j] / den : 1.0;
        sn[j] = den > 0 ? hn / den : 0.0;
        col[j] = den;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++iters;
        jn = j + 1;
        const bool breakdown = !(hn > 0.0);
        if (std::fabs(g[j + 1]) <= tol2 || breakdown || iters >= max_it) {
          done = true;
          break;
        }
      }
      // X += V y with R y = g (upper triangular, jn columns)
      for (int i = jn - 1; i >= 0; --i) {
        double t = g[i];
        for (int k = i + 1; k < jn; ++k) t -= R[(size_t)k * (m + 1) + i] * yv[k];
        const double d = R[(size_t)i * (m + 1) + i];
        yv[i] = d != 0.0 ? t / d : 0.0;
      }
      for (int i = 0; i < jn; ++i) host_coef[i] = yv[i];
      hipError_t e = hipMemcpyAsync(w.coef, host_coef.data(), jn * sizeof(double),
                                    hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess)
        e = launch_multi_axpy(n, jn, w.V, w.stride, w.coef, 1.0, w.X, 1.0, w.X, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // host_coef is reused
      if (e != hipSuccess) return hip_fail(s, e, "GMRES update");
      if (done) break;
      // restart from the true residual -F - (I - h J) X
      double xn2 = 0.0;
      if ((rc = dot(w.X, w.X, xn2))) return rc;
      const double xn = std::sqrt(xn2);
      if (!(xn > 0.0)) break;
      if ((rc = apply(w.X, xn, Ly, Vk(0)))) return rc;
      if ((rc = check(launch_lincomb(n, -1.0, Vk(0), -1.0, w.F, 0.0, nullptr, Vk(0), s->stream),
                      "lincomb")))
        return rc;
      double r2 = 0.0;
      if ((rc = dot(Vk(0), Vk(0), r2))) return rc;
      beta = std::sqrt(r2);
      if (!std::isfinite(beta)) return fail(s, DGBGK_ENONFINITE, "GMRES residual is not finite");
      if (beta <= tol2) break;
      if (beta > 0.9 * beta_cycle) mc = std::min(2 * mc, m);
      if ((rc = check(launch_lincomb(n, 1.0 / beta, Vk(0), 0.0, nullptr, 0.0, nullptr, Vk(0), s->stream),
                      "lincomb")))
        return rc;
    }
    return DGBGK_OK;
  }

  // apply() for a vector v of the FP32 basis; out (FP64) != T.
  int apply32(const float *v, double vnorm, const double *Ly, double *out) {
    const double e = eps / vnorm;
    int rc = check(launch_lincomb_mixed(w.n, 1.0, w.y, e, v, 0.0, nullptr, w.T, s->stream), "lincomb");
    if (!rc) rc = rhs(w.T, out);
    if (!rc)
      rc = check(launch_lincomb_mixed(w.n, -h / e, out, 1.0, v, h / e, Ly, out, s->stream), "lincomb");
    return rc;
  }

  // GMRES as above with the basis stored in FP32: each new Krylov vector is
  // formed and orthogonalised in FP64 (w.W) against the FP32 basis, and
  // stored in FP32 once normalised; restarts form the true residual in FP64.
  int gmres32(const double *Ly, double fnorm2, double tol2, int max_it, int &iters) {
    const size_t n = w.n;
    std::vector<double> R((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), yv(m);
    int rc = check(launch_lincomb(n, 0.0, nullptr, 0.0, nullptr, 0.0, nullptr, w.X, s->stream), "zero");
    if (rc) return rc;
    double beta = fnorm2;
    int mc = std::min(kShortCycle, m);
    rc = check(launch_multi_axpy32(n, 0, w.V32, w.stride, w.coef, 0.0, w.F, -1.0 / beta, w.W, Vk32(0),
                                   s->stream),
               "basis vector");
    if (rc) return rc;
    bool done = false;
    while (!done) {
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int jn = 0;
      const double beta_cycle = beta;
      for (int j = 0; j < mc; ++j) {
        if ((rc = apply32(Vk32(j), 1.0, Ly, w.W))) return rc;
        // projections on V_0..V_j and |w|^2 in one pass
        double *h1 = w.small, *h2 = w.small + (m + 1);
        hipError_t e = launch_multi_dot32(n, j + 1, w.V32, w.stride, w.W, w.dots, h1, s->stream);
        if (e == hipSuccess)
          e = hipMemcpyAsync(host_small.data(), h1, (size_t)(j + 2) * sizeof(double),
                             hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(s, e, "Arnoldi projections");
        double *col = &R[(size_t)j * (m + 1)];
        double hh = 0.0;
        for (int i = 0; i <= j; ++i) {
          col[i] = host_small[i];
          hh += col[i] * col[i];
        }
        const double ww = host_small[j + 1];
        if (!std::isfinite(ww) || !std::isfinite(hh))
          return fail(s, DGBGK_ENONFINITE, "Krylov vector is not finite");
        double hn;
        if (ww - hh > 0.5 * ww) {
          hn = std::sqrt(ww - hh);
          e = launch_multi_axpy32(n, j + 1, w.V32, w.stride, h1, -1.0, w.W, 1.0 / hn, w.W, Vk32(j + 1),
                                  s->stream);
        } else {
          e = launch_multi_axpy32(n, j + 1, w.V32, w.stride, h1, -1.0, w.W, 1.0, w.W, nullptr, s->stream);
          if (e == hipSuccess) e = launch_multi_dot32(n, j + 1, w.V32, w.stride, w.W, w.dots, h2, s->stream);
          if (e == hipSuccess)
            e = hipMemcpyAsync(host_small.data(), h2, (size_t)(j + 2) * sizeof(double),
                               hipMemcpyDeviceToHost, s->stream);
          if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
          if (e != hipSuccess) return hip_fail(s, e, "Arnoldi reorthogonalisation");
          double hh2 = 0.0;
          for (int i = 0; i <= j; ++i) {
            col[i] += host_small[i];
            hh2 += host_small[i] * host_small[i];
          }
          hn = std::sqrt(std::max(host_small[j + 1] - hh2, 0.0));
          e = launch_multi_axpy32(n, j + 1, w.V32, w.stride, h2, -1.0, w.W, hn > 0.0 ? 1.0 / hn : 1.0, w.W,
                                  Vk32(j + 1), s->stream);
        }
        if (e != hipSuccess) return hip_fail(s, e, "Arnoldi update");
        for (int i = 0; i < j; ++i) {
          const double a = col[i], b = col[i + 1];
          col[i] = cs[i] * a + sn[i] * b;
          col[i + 1] = -sn[i] * a + cs[i] * b;
        }
        const double den = std::hypot(col[j], hn);
        cs[j] = den > 0 ? col[j] / den : 1.0;
        sn[j] = den > 0 ? hn / den : 0.0;
        col[j] = den;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++iters;
        jn = j + 1;
        const bool breakdown = !(hn > 0.0);
        if (std::fabs(g[j + 1]) <= tol2 || breakdown || iters >= max_it) {
          done = true;
          break;
        }
      }
      for (int i = jn - 1; i >= 0; --i) {
        double t = g[i];
        for (int k = i + 1; k < jn; ++k) t -= R[(size_t)k * (m + 1) + i] * yv[k];
        const double d = R[(size_t)i * (m + 1) + i];
        yv[i] = d != 0.0 ? t / d : 0.0;
      }
      for (int i = 0; i < jn; ++i) host_coef[i] = yv[i];
      hipError_t e = hipMemcpyAsync(w.coef, host_coef.data(), jn * sizeof(double),
                                    hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess)
        e = launch_multi_axpy32(n, jn, w.V32, w.stride, w.coef, 1.0, w.X, 1.0, w.X, nullptr, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // host_coef is reused
      if (e != hipSuccess) return hip_fail(s, e, "GMRES update");
      if (done) break;
      double xn2 = 0.0;
      if ((rc = dot(w.X, w.X, xn2))) return rc;
      const double xn = std::sqrt(xn2);
      if (!(xn > 0.0)) break;
      if ((rc = apply(w.X, xn, Ly, w.W))) return rc;
      if ((rc = check(launch_lincomb(n, -1.0, w.W, -1.0, w.F, 0.0, nullptr, w.W, s->stream), "lincomb")))
        return rc;
      double r2 = 0.0;
      if ((rc = dot(w.W, w.W, r2))) return rc;
      beta = std::sqrt(r2);
      if (!std::isfinite(beta)) return fail(s, DGBGK_ENONFINITE, "GMRES residual is not finite");
      if (beta <= tol2) break;
      if (beta > 0.9 * beta_cycle) mc = std::min(2 * mc, m);
      if ((rc = check(launch_multi_axpy32(n, 0, w.V32, w.stride, w.coef, 0.0, w.W, 1.0 / beta, w.W,
                                          Vk32(0), s->stream),
                      "basis vector")))
        return rc;
    }
    return DGBGK_OK;
  }

  // F = y - b - h Ly and its 2-norm.
  int newton_residual(const double *Ly, double &fn2) {
    int rc = check(launch_lincomb(w.n, 1.0, w.y, -1.0, w.b, -h, Ly, w.F, s->stream), "lincomb");
    double ff = 0.0;
    if (!rc) rc = dot(w.F, w.F, ff);
    if (rc) return rc;
    fn2 = std::sqrt(ff);
    if (!std::isfinite(fn2)) return fail(s, DGBGK_ENONFINITE, "Newton residual is not finite");
    return DGBGK_OK;
  }
};

}  // namespace

// Static workspace of the allocation-free implicit step: one array per device
// (each device that runs the library holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel: its device
// address comes from hipGetSymbolAddress, once per device, with that device
// current.
constexpr size_t kStaticWsBytes = (size_t)64 << 20;
static __device__ __align__(256) double scratch[kStaticWsBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of the static workspace on the solver's device (which must
// be current).
int static_workspace(dgbgk_solver *s, double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(s, e, "hipGetDevice");
  if (dev != s->device)
    return fail(s, DGBGK_EDEVICE, "device %d is current; the solver's memory is on device %d", dev,
                s->device);
  if (dev < 0 || dev >= kMaxDevices)
    return fail(s, DGBGK_EDEVICE, "device %d: the static workspace covers devices 0..%d", dev,
                kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(s, e, "hipGetSymbolAddress(static workspace)");
    if (!p || (uintptr_t)p % kAlign) return fail(s, DGBGK_EDEVICE, "static workspace address %p", p);
    g_scratch_ptr[dev] = (double *)p;
  }
  *out = g_scratch_ptr[dev];
  return DGBGK_OK;
}

int implicit_steps(dgbgk_solver *s, int32_t scheme, int64_t nsteps, double dt,
                   const dgbgk_implicit_options *opt, dgbgk_implicit_report *report,
                   bool static_ws) {
  if (!s) return fail(nullptr, DGBGK_EINVAL, "solver is NULL");
  Sdirk tab;
  if (!sdirk_tableau(scheme, tab)) return fail(s, DGBGK_EINVAL, "unknown implicit scheme %d", scheme);
  if (nsteps < 0 || !(dt > 0) || !is_finite_d(dt)) return fail(s, DGBGK_EINVAL, "need nsteps >= 0, dt > 0");
  dgbgk_implicit_options o{20, 1e-10, 1e-14, 30, 300, 1e-6, 0};
  if (opt) o = *opt;
  if (o.max_newton < 1 || o.max_newton > 1000 || o.restart < 1 || o.restart > 64 || o.max_krylov < 1 ||
      !(o.newton_rtol >= 0) || !(o.newton_atol >= 0) || !is_finite_d(o.newton_rtol) ||
      !is_finite_d(o.newton_atol) || !(o.krylov_rtol > 0 && o.krylov_rtol < 1) ||
      (o.krylov_fp32 != 0 && o.krylov_fp32 != 1))
    return fail(s, DGBGK_EINVAL, "implicit options out of range");
  if (o.krylov_fp32 && o.krylov_rtol < 1e-5)
    return fail(s, DGBGK_EINVAL, "an FP32 Krylov basis needs krylov_rtol >= 1e-5");
  if (s->prec != DGBGK_FP64) return fail(s, DGBGK_ENOTSUP, "implicit steps need FP64 precision");
  if (!s->have_state) return fail(s, DGBGK_ESTATE, "no state: call init or set_state first");
  // a state implies the solver's device memory exists (nothing is allocated here)
  if (static_ws && !s->dev_ready) return fail(s, DGBGK_ESTATE, "solver has no device memory");
  int rc = ensure_device(s);
  if (rc) return rc;

  Implicit im{s, ImplicitWs{}, o.restart};
  const size_t n = (size_t)s->K * s->Np * s->Q;
  size_t stride = 0;
  const bool v32 = o.krylov_fp32 != 0;
  const size_t bytes = implicit_ws_bytes(n, tab.stages, im.m, v32, &stride);
  double *ws = nullptr;
  if (static_ws) {
    if (bytes > kStaticWsBytes)
      return fail(s, DGBGK_EINVAL,
                  "implicit workspace of %zu B exceeds the %zu B static workspace (a shorter "
                  "GMRES restart, the FP32 Krylov basis or a smaller problem fits)",
                  bytes, kStaticWsBytes);
    if ((rc = static_workspace(s, &ws))) return rc;
  }
  if (report) *report = dgbgk_implicit_report{0, 0, 0, 0.0, 1};
  if (!static_ws && bytes > s->imp_bytes) {
    if (s->imp_ws) {
      (void)hipStreamSynchronize(s->stream);
      (void)hipFree(s->imp_ws);
      s->imp_ws = nullptr;
      s->imp_bytes = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(s, DGBGK_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    s->imp_ws = (double *)p;
    s->imp_bytes = bytes;
  }
  if (!static_ws) ws = s->imp_ws;
  ImplicitWs &w = im.w;
  w.n = n;
  w.stride = stride;
  double *q = ws;
  w.K = q;  q += (size_t)tab.stages * stride;
  w.y = q;  q += stride;
  w.b = q;  q += stride;
  w.F = q;  q += stride;
  w.T = q;  q += stride;
  w.X = q;  q += stride;
  if (v32) {
    w.W = q;  q += stride;
    w.V32 = (float *)q;  q += (size_t)(im.m + 1) * stride / 2;
  } else {
    w.V = q;  q += (size_t)(im.m + 1) * stride;
  }
  w.dots = q;  q += multi_dot_scratch(n, im.m + 1);
  w.small = q;  q += 2 * (size_t)(im.m + 1) + 8;
  w.coef = q;
  im.host_small.assign(2 * (size_t)(im.m + 1) + 8, 0.0);
  im.host_coef.assign(kMaxBasis, 0.0);

  const double rms = std::sqrt((double)n);  // 2-norm -> RMS
  int newton_total = 0, krylov_total = 0;
  double worst = 0.0;
  bool all_conv = true;
  for (int64_t step = 0; step < nsteps; ++step) {
    for (int i = 0; i < tab.stages; ++i) {
      // b_i = f_n + dt sum_{j<i} a_ij k_j
      for (int j = 0; j < i; ++j) im.host_coef[j] = dt * tab.a[i][j];
      hipError_t e = hipSuccess;
      if (i > 0)
        e = hipMemcpyAsync(w.coef, im.host_coef.data(), i * sizeof(double), hipMemcpyHostToDevice,
                           s->stream);
      if (e == hipSuccess)
        e = launch_multi_axpy(n, i, w.K, stride, w.coef, 1.0, s->d_fn, 1.0, w.b, s->stream);
      if (e == hipSuccess && i == 0)
        e = launch_lincomb(n, 1.0, s->d_fn, 0.0, nullptr, 0.0, nullptr, w.y, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);  // host_coef is reused
      if (e != hipSuccess) return hip_fail(s, e, "stage set-up");
      im.h = dt * tab.gamma;
      double *Ly = w.K + (size_t)i * stride;
      if ((rc = im.rhs(w.y, Ly))) return rc;
      double fn2 = 0.0;
      if ((rc = im.newton_residual(Ly, fn2))) return rc;
      const double target = std::max(o.newton_rtol * fn2, o.newton_atol * rms);
      bool conv = fn2 <= target;
      for (int it = 0; it < o.max_newton && !conv; ++it) {
        double yy = 0.0;
        if ((rc = im.dot(w.y, w.y, yy))) return rc;
        im.eps = kFdStep * (1.0 + std::sqrt(yy));
        int kit = 0;
        // inexact Newton: no linear solve tighter than the Newton target needs
        const double ktol = std::max(o.krylov_rtol * fn2, 0.1 * target);
        if ((rc = v32 ? im.gmres32(Ly, fn2, ktol, o.max_krylov, kit)
                      : im.gmres(Ly, fn2, ktol, o.max_krylov, kit)))
          return rc;
        krylov_total += kit;
        ++newton_total;
        if ((rc = im.check(launch_lincomb(n, 1.0, w.y, 1.0, w.X, 0.0, nullptr, w.y, s->stream), "lincomb")))
          return rc;
        if ((rc = im.rhs(w.y, Ly))) return rc;
        if ((rc = im.newton_residual(Ly, fn2))) return rc;
        conv = fn2 <= target;
      }
      all_conv = all_conv && conv;
      worst = std::max(worst, fn2 / rms);
    }
    // stiffly accurate: f_{n+1} is the last stage value
    s->part_valid = false;
    hipError_t e = launch_lincomb(n, 1.0, w.y, 0.0, nullptr, 0.0, nullptr, s->d_fn, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "lincomb");
    ++s->steps;
  }
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "implicit step");
  if (report) {
    report->newton_iterations = newton_total;
    report->krylov_iterations = krylov_total;
    report->rhs_evaluations = im.rhs_evals;
    report->max_final_residual = worst;
    report->converged = all_conv ? 1 : 0;
  }
  return DGBGK_OK;
}

}  // namespace

extern "C" {

int dgbgk_implicit_step(dgbgk_solver *s, int32_t scheme, int64_t nsteps, double dt,
                        const dgbgk_implicit_options *opt, dgbgk_implicit_report *report) {
  return implicit_steps(s, scheme, nsteps, dt, opt, report, false);
}

int dgbgk_implicit_step_noalloc(dgbgk_solver *s, int32_t scheme, int64_t nsteps, double dt,
                                const dgbgk_implicit_options *opt, dgbgk_implicit_report *report) {
  return implicit_steps(s, scheme, nsteps, dt, opt, report, true);
}

}  // extern "C"

// ---- batches ---------------------------------------------------------------------

struct dgbgk_batch {
  struct Class {
    int prec = DGBGK_FP64, p = 1, cw = 0, contract = 0, ref = 0, lds_bin = 0;
    int ho = 0;  // FP32: one-element members that hand their moments between stages
    std::vector<int> members;  // indices into s
    std::vector<int2> items;   // (member index within the class, element block)
    size_t lds = 0;
    int groups = 0;
    size_t off_items = 0, off_desc = 0;  // byte offsets into dev
    size_t desc_size = 0;                // bytes of one descriptor
  };
  std::vector<dgbgk_solver *> s;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<Class> cls;
  std::vector<int> solo;           // members large enough to run their own stage kernels
  char *dev = nullptr;
  std::vector<char> host;          // staging of the descriptor tables
  std::vector<double> dt_loaded;   // dt each member's descriptors hold (NaN: none)
  std::vector<int> E_built;        // each member's elements per block when the lists were built
  std::vector<int> fused_built;    // and its fused flag
  // independent chains (a class, or a large member) are spread over up to
  // kBatchLanes streams forked from and joined to `stream` around each call
  // (or captured graph), so that small kernels run beside large ones
  std::vector<hipStream_t> lanes;
  std::vector<hipEvent_t> lane_done;
  hipEvent_t fork = nullptr;
  std::vector<int> class_lane, solo_lane;
  int graph_steps = 0;                // RK4 steps per captured graph (0: eager)
  hipGraphExec_t exec = nullptr;      // graph_steps steps
  hipGraphExec_t exec1 = nullptr;     // one step (the remainder of a call)
  size_t off_res = 0;                 // byte offset of the residual accumulators in dev
  std::vector<unsigned long long> res_host;
  std::string err;
};

namespace {

int bfail(dgbgk_batch *b, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) b->err = buf;
  else g_create_error = buf;
  return code;
}

// State buffers a stage reads and writes: 1: fn -> A, 2: A -> B, 3: B -> A,
// 4: A -> fn, 0 (right-hand side): fn -> B.
void stage_buffers(dgbgk_solver *s, int stage, void *&fs, void *&out) {
  void *fn = s->d_fn, *A = s->d_a, *B = s->d_b;
  switch (stage) {
    case 1: fs = fn; out = A; break;
    case 2: fs = A; out = B; break;
    case 3: fs = B; out = A; break;
    case 4: fs = A; out = fn; break;
    default: fs = fn; out = B; break;
  }
}

// Fills the host copy of the descriptors of every class, stage and member.
void fill_descriptors(dgbgk_batch *b, const double *dt) {
  // the cache policy follows the whole batch's state, which a step sweeps
  size_t total = 0;
  for (dgbgk_solver *s : b->s) total += (size_t)s->K * s->Np * s->Q * (is_fp32(s->prec) ? 4 : 8);
  const int nt = stream_nt_for(total);
  for (auto &c : b->cls) {
    const size_t nm = c.members.size();
    for (int stage = 0; stage <= 4; ++stage)
      for (size_t i = 0; i < nm; ++i) {
        dgbgk_solver *s = b->s[c.members[i]];
        const double h = dt ? dt[c.members[i]] : 0.0;
        void *fs, *out;
        stage_buffers(s, stage, fs, out);
        char *dst = b->host.data() + c.off_desc + ((size_t)stage * nm + i) * c.desc_size;
        double ca, co;
        rk_coefficients(stage, h, ca, co);
        if (is_fp32(s->prec)) {
          Stage32Args a = base_args32(s);
          a.fs = (const float *)fs;
          a.fn = s->g_fn;
          a.acc = s->g_acc;
          a.out = (float *)out;
          a.stage = stage;
          a.c_acc = (float)ca;
          a.c_out = (float)co;
          a.stream_nt = nt;
          stage_partials(s, stage, a.pin, a.pout);
          std::memcpy(dst, &a, sizeof a);
        } else {
          StageArgs a = base_args(s);
          a.fs = (const double *)fs;
          a.fn = s->d_fn;
          a.acc = s->d_acc;
          a.out = (double *)out;
          a.stage = stage;
          a.c_acc = ca;
          a.c_out = co;
          a.stream_nt = nt;
          stage_partials(s, stage, a.pin, a.pout);
          std::memcpy(dst, &a, sizeof a);
        }
      }
  }
}

// The members' stages read the partials of f_n from P0: fill those that are
// stale, on the batch's stream.
int batch_partials(dgbgk_batch *b) {
  for (size_t i = 0; i < b->s.size(); ++i) {
    dgbgk_solver *s = b->s[i];
    hipStream_t own = s->stream;
    s->stream = b->stream;
    const int rc = ensure_partials(s);
    s->stream = own;
    if (rc) return bfail(b, rc, "member %zu: %s", i, s->err.c_str());
  }
  return DGBGK_OK;
}

int upload_descriptors(dgbgk_batch *b) {
  hipError_t e = hipMemcpyAsync(b->dev, b->host.data(), b->host.size(), hipMemcpyHostToDevice,
                                b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "descriptor upload: %s", hipGetErrorString(e));
  return DGBGK_OK;
}

int launch_class(dgbgk_batch *b, const dgbgk_batch::Class &c, int stage, hipStream_t st) {
  const size_t nm = c.members.size();
  const void *descs = b->dev + c.off_desc + (size_t)stage * nm * c.desc_size;
  const int2 *items = (const int2 *)(b->dev + c.off_items);
  hipError_t e;
  if (is_fp32(c.prec))
    e = launch_batch_stage32(c.p, stage, c.cw, c.contract, c.ref, c.ho, (const Stage32Args *)descs, items,
                             (int)c.items.size(), c.lds, c.groups, st);
  else
    e = launch_batch_stage(c.p, stage, (const StageArgs *)descs, items, (int)c.items.size(), c.lds,
                           c.groups, st);
  if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "batched stage kernel: %s", hipGetErrorString(e));
  return DGBGK_OK;
}

// A member of kSoloDof or more fills the GPU on its own: the batch launches
// its single-problem stage kernels, in its own decomposition (same results as
// stepping it alone), and packs only the smaller members into the persistent
// kernels, which pay off where launches dominate.
int launch_solo(dgbgk_batch *b, int i, int stage, hipStream_t st) {
  dgbgk_solver *s = b->s[i];
  void *fs, *out;
  stage_buffers(s, stage, fs, out);
  hipStream_t own = s->stream;
  s->stream = st;
  const double *pin;
  double *pout;
  stage_partials(s, stage, pin, pout);  // P0 is current: the batch filled it before its steps
  const int rc = run_stage(s, stage, fs, out, b->dt_loaded[i], nullptr, pin, pout);
  s->stream = own;
  if (rc) return bfail(b, rc, "member %d: %s", i, s->err.c_str());
  return DGBGK_OK;
}

// nsteps RK4 steps of every chain; with lanes, each chain on its own lane
// stream between a fork from and a join to the batch's stream.
int enqueue_steps(dgbgk_batch *b, int64_t nsteps) {
  const bool multi = !b->lanes.empty();
  hipError_t e = hipSuccess;
  if (multi) {
    e = hipEventRecord(b->fork, b->stream);
    for (size_t k = 0; k < b->lanes.size() && e == hipSuccess; ++k)
      e = hipStreamWaitEvent(b->lanes[k], b->fork, 0);
    if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "lane fork: %s", hipGetErrorString(e));
  }
  int rc = DGBGK_OK;
  for (int64_t it = 0; it < nsteps && !rc; ++it)
    for (int stage = 1; stage <= 4 && !rc; ++stage) {
      for (size_t c = 0; c < b->cls.size() && !rc; ++c)
        rc = launch_class(b, b->cls[c], stage, multi ? b->lanes[b->class_lane[c]] : b->stream);
      for (size_t j = 0; j < b->solo.size() && !rc; ++j)
        rc = launch_solo(b, b->solo[j], stage, multi ? b->lanes[b->solo_lane[j]] : b->stream);
    }
  if (multi) {  // join (also after a failed launch, so that a capture can end)
    for (size_t k = 0; k < b->lanes.size() && e == hipSuccess; ++k) {
      e = hipEventRecord(b->lane_done[k], b->lanes[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->lane_done[k], 0);
    }
    if (e != hipSuccess && !rc) rc = bfail(b, DGBGK_EDEVICE, "lane join: %s", hipGetErrorString(e));
  }
  return rc;
}

int enqueue_step(dgbgk_batch *b) { return enqueue_steps(b, 1); }

void drop_graph(dgbgk_batch *b) {
  if (b->exec || b->exec1) (void)hipStreamSynchronize(b->stream);  // replays in flight
  if (b->exec && b->exec != b->exec1) (void)hipGraphExecDestroy(b->exec);
  if (b->exec1) (void)hipGraphExecDestroy(b->exec1);
  b->exec = nullptr;
  b->exec1 = nullptr;
}

// Captures `steps` RK4 steps of the batch into *out.
int capture_batch(dgbgk_batch *b, int steps, hipGraphExec_t *out) {
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "begin capture: %s", hipGetErrorString(e));
  int rc = enqueue_steps(b, steps);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *out = nullptr;
    return bfail(b, DGBGK_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  }
  return DGBGK_OK;
}

}  // namespace

extern "C" {

int dgbgk_batch_create(dgbgk_solver *const *solvers, int32_t n, void *hip_stream,
                       dgbgk_batch **out) {
  if (!out) return bfail(nullptr, DGBGK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!solvers || n < 1) return bfail(nullptr, DGBGK_EINVAL, "need at least one solver");
  for (int i = 0; i < n; ++i) {
    if (!solvers[i]) return bfail(nullptr, DGBGK_EINVAL, "solver %d is NULL", i);
    for (int j = 0; j < i; ++j)
      if (solvers[j] == solvers[i]) return bfail(nullptr, DGBGK_EINVAL, "solver %d appears twice", i);
  }
  dgbgk_batch *b = new (std::nothrow) dgbgk_batch;
  if (!b) return bfail(nullptr, DGBGK_ENOMEM, "out of host memory");
  b->s.assign(solvers, solvers + n);
  b->stream = (hipStream_t)hip_stream;
  int rc = DGBGK_OK;
  for (int i = 0; i < n && !rc; ++i) {
    dgbgk_solver *s = b->s[i];
    if ((int64_t)s->K * s->Np * s->Q >= kSoloDof) {  // keeps its own decomposition
      b->solo.push_back(i);
      if ((rc = ensure_device(s))) bfail(nullptr, rc, "solver %d: %s", i, s->err.c_str());
      continue;
    }
    if (!s->fused || s->persistent) {  // members run the fused per-block body
      s->tiling_mode = 1;
      choose_tiling(s);
    }
    if (!s->fused || !tiling_admissible(s))
      rc = bfail(nullptr, DGBGK_ENOTSUP, "solver %d: its fused tile does not fit in LDS", i);
    else if ((rc = ensure_device(s)))
      bfail(nullptr, rc, "solver %d: %s", i, s->err.c_str());
  }
  if (rc) {
    delete b;
    return rc;
  }
  // classes of (precision, p, access width, contraction, LDS bin)
  const size_t bins[4] = {40 * 1024, 64 * 1024, 80 * 1024, 160 * 1024};
  for (int i = 0; i < n; ++i) {
    dgbgk_solver *s = b->s[i];
    if (std::find(b->solo.begin(), b->solo.end(), i) != b->solo.end()) continue;
    const bool f32 = is_fp32(s->prec);
    const int cw = f32 ? (((int64_t)s->Q * s->Np) % 4 == 0 ? 4 : 1) : 0;
    const int contract = is_bf(s->prec) ? 1 : 0;
    const int ref = is_ref(s->prec) ? 1 : 0;
    const int ho = f32 && uses_partials(s) ? 1 : 0;
    int bin = 0;
    while (bin < 3 && s->lds > bins[bin]) ++bin;
    const int prec_class = f32 ? DGBGK_FP32 : DGBGK_FP64;
    size_t k = 0;
    for (; k < b->cls.size(); ++k) {
      const auto &c = b->cls[k];
      if (c.prec == prec_class && c.p == s->p && c.cw == cw && c.contract == contract && c.ref == ref &&
          c.ho == ho && c.lds_bin == bin)
        break;
    }
    if (k == b->cls.size()) {
      dgbgk_batch::Class c;
      c.prec = prec_class;
      c.p = s->p;
      c.cw = cw;
      c.contract = contract;
      c.ref = ref;
      c.ho = ho;
      c.lds_bin = bin;
      b->cls.push_back(c);
    }
    auto &c = b->cls[k];
    const int li = (int)c.members.size();
    c.members.push_back(i);
    for (int blk = 0; blk < s->nblk; ++blk) c.items.push_back(make_int2(li, blk));
    c.lds = std::max(c.lds, s->lds);
  }
  // device layout: per class its items, then its descriptors (5 stages x members)
  size_t off = 0;
  for (auto &c : b->cls) {
    // the kernels index the table as an array of the argument struct: the
    // stride must be exactly its size
    c.desc_size = is_fp32(c.prec) ? sizeof(Stage32Args) : sizeof(StageArgs);
    c.off_items = off;
    off += round_up(c.items.size() * sizeof(int2));
    c.off_desc = off;
    off += round_up(5 * c.members.size() * c.desc_size);
    const int per_cu = std::max(1, std::min(is_fp32(c.prec) ? 3 : 2, (int)((160 * 1024) / c.lds)));
    c.groups = (int)std::min<size_t>(c.items.size(), (size_t)per_cu * b->s[c.members[0]]->num_cu);
  }
  b->off_res = off;  // one accumulator per member for the batched residuals
  off += round_up((size_t)n * sizeof(unsigned long long));
  b->host.assign(off, 0);
  for (auto &c : b->cls)
    std::memcpy(b->host.data() + c.off_items, c.items.data(), c.items.size() * sizeof(int2));
  hipError_t e = hipMalloc((void **)&b->dev, off);
  if (e != hipSuccess) {
    delete b;
    return bfail(nullptr, DGBGK_ENOMEM, "hipMalloc(%zu): %s", off, hipGetErrorString(e));
  }
  if (!b->stream) {
    // a stream of its own (ordered with the null stream), needed for graph capture
    e = hipStreamCreate(&b->stream);
    if (e != hipSuccess) {
      (void)hipFree(b->dev);
      delete b;
      return bfail(nullptr, DGBGK_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    b->own_stream = true;
  }
  // lanes: chains balanced by DOF, largest first onto the least loaded lane
  {
    struct Chain { int64_t dof; int cls; int solo; };
    std::vector<Chain> ch;
    for (size_t c = 0; c < b->cls.size(); ++c) {
      int64_t d = 0;
      for (int m : b->cls[c].members) d += b->s[m]->K * b->s[m]->Np * b->s[m]->Q;
      ch.push_back({d, (int)c, -1});
    }
    for (size_t j = 0; j < b->solo.size(); ++j) {
      const dgbgk_solver *m = b->s[b->solo[j]];
      ch.push_back({m->K * m->Np * m->Q, -1, (int)j});
    }
    const int nl = (int)std::min<size_t>(ch.size(), kBatchLanes);
    if (nl >= 2) {
      std::sort(ch.begin(), ch.end(), [](const Chain &x, const Chain &y) { return x.dof > y.dof; });
      std::vector<int64_t> load(nl, 0);
      b->class_lane.assign(b->cls.size(), 0);
      b->solo_lane.assign(b->solo.size(), 0);
      for (const Chain &c : ch) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[k] += c.dof;
        if (c.cls >= 0) b->class_lane[c.cls] = k;
        else b->solo_lane[c.solo] = k;
      }
      e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
      for (int k = 0; k < nl && e == hipSuccess; ++k) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) b->lanes.push_back(st);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->lane_done.push_back(ev);
      }
      if (e != hipSuccess) {
        dgbgk_batch_destroy(b);
        return bfail(nullptr, DGBGK_EDEVICE, "lane streams: %s", hipGetErrorString(e));
      }
    }
  }
  b->dt_loaded.assign(n, std::nan(""));
  b->E_built.resize(n);
  b->fused_built.resize(n);
  for (int i = 0; i < n; ++i) {
    b->E_built[i] = b->s[i]->E;
    b->fused_built[i] = b->s[i]->fused;
  }
  fill_descriptors(b, nullptr);
  if ((rc = upload_descriptors(b))) {
    const std::string msg = b->err;
    dgbgk_batch_destroy(b);
    return bfail(nullptr, rc, "%s", msg.c_str());
  }
  *out = b;
  return DGBGK_OK;
}

int dgbgk_batch_set_graph(dgbgk_batch *b, int32_t use_graph) {
  if (!b) return bfail(nullptr, DGBGK_EINVAL, "batch is NULL");
  if (use_graph < 0 || use_graph > 1000) return bfail(b, DGBGK_EINVAL, "use_graph must be 0..1000");
  if (use_graph != b->graph_steps) drop_graph(b);
  b->graph_steps = use_graph;
  return DGBGK_OK;
}

int dgbgk_batch_step(dgbgk_batch *b, int64_t nsteps, const double *dt) {
  if (!b) return bfail(nullptr, DGBGK_EINVAL, "batch is NULL");
  if (nsteps < 0 || !dt) return bfail(b, DGBGK_EINVAL, "need nsteps >= 0 and dt");
  const size_t n = b->s.size();
  for (size_t i = 0; i < n; ++i) {
    if (!(dt[i] > 0) || !std::isfinite(dt[i])) return bfail(b, DGBGK_EINVAL, "dt[%zu] must be > 0", i);
    if (!b->s[i]->have_state) return bfail(b, DGBGK_ESTATE, "member %zu has no state", i);
    if (b->s[i]->E != b->E_built[i] || b->s[i]->fused != b->fused_built[i])
      return bfail(b, DGBGK_ESTATE, "member %zu was re-tiled after the batch was built", i);
  }
  bool changed = false;
  for (size_t i = 0; i < n; ++i) changed |= !(b->dt_loaded[i] == dt[i]);
  int rc;
  if (changed) {
    // the stream may still run replays that read the tables: wait before rewriting them
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "synchronize: %s", hipGetErrorString(e));
    fill_descriptors(b, dt);
    if ((rc = upload_descriptors(b))) return rc;
    for (size_t i = 0; i < n; ++i) b->dt_loaded[i] = dt[i];
    // the single-problem launches of large members carry dt in their arguments
    if (!b->solo.empty()) drop_graph(b);
  }
  if (nsteps == 0) return DGBGK_OK;
  if ((rc = batch_partials(b))) return rc;
  for (auto *s : b->s) s->part_valid = false;  // until every step is enqueued
  const int k = b->graph_steps;
  if (k > 0 && ((nsteps >= k && !b->exec) || (nsteps % k != 0 && !b->exec1))) {
    // one eager step first: it sets the kernels' LDS attributes outside the capture
    if ((rc = enqueue_step(b))) return rc;
    --nsteps;
    for (auto *s : b->s) ++s->steps;
    if (!b->exec && k > 1 && (rc = capture_batch(b, k, &b->exec))) return rc;
    if (!b->exec1 && (rc = capture_batch(b, 1, &b->exec1))) return rc;
    if (k == 1) b->exec = b->exec1;
  }
  int64_t it = 0;
  if (k > 0) {
    for (; it + k <= nsteps; it += k) {
      hipError_t e = hipGraphLaunch(b->exec, b->stream);
      if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "graph launch: %s", hipGetErrorString(e));
    }
    for (; it < nsteps; ++it) {
      hipError_t e = hipGraphLaunch(b->exec1, b->stream);
      if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "graph launch: %s", hipGetErrorString(e));
    }
  } else if ((rc = enqueue_steps(b, nsteps - it))) {
    return rc;
  }
  for (auto *s : b->s) {
    s->steps += nsteps;
    s->part_valid = uses_partials(s);  // each step ends with the partials of f_n in P0
  }
  return DGBGK_OK;
}

int dgbgk_batch_residuals(dgbgk_batch *b, double *r) {
  if (!b) return bfail(nullptr, DGBGK_EINVAL, "batch is NULL");
  if (!r) return bfail(b, DGBGK_EINVAL, "r is NULL");
  const size_t n = b->s.size();
  for (size_t i = 0; i < n; ++i) {
    if (!b->s[i]->have_state) return bfail(b, DGBGK_ESTATE, "member %zu has no state", i);
    if (b->s[i]->E != b->E_built[i] || b->s[i]->fused != b->fused_built[i])
      return bfail(b, DGBGK_ESTATE, "member %zu was re-tiled after the batch was built", i);
  }
  // L(f) of every member (one stage-0 launch per class, the members' own
  // kernels for large members), then one reduction launch per member into the
  // batch's accumulators and a single copy to the host
  unsigned long long *acc = (unsigned long long *)(b->dev + b->off_res);
  int rc = batch_partials(b);
  if (rc) return rc;
  hipError_t e = launch_fill_u64(acc, n, 0ull, b->stream);
  if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "fill kernel: %s", hipGetErrorString(e));
  for (const auto &c : b->cls)
    if ((rc = launch_class(b, c, 0, b->stream))) return rc;
  for (int i : b->solo)
    if ((rc = launch_solo(b, i, 0, b->stream))) return rc;
  for (size_t i = 0; i < n; ++i) {
    dgbgk_solver *s = b->s[i];
    void *fs, *out;
    stage_buffers(s, 0, fs, out);
    e = is_fp32(s->prec)
            ? launch_residual32((const float *)out, s->d_vel, (int)s->K, s->Np, s->Q, s->resid_scale,
                                acc + i, b->stream)
            : launch_residual((const double *)out, s->d_vel, (int)s->K, s->Np, s->Q, s->resid_scale,
                              acc + i, b->stream);
    if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "residual kernel: %s", hipGetErrorString(e));
  }
  b->res_host.assign(n, 0ull);
  e = hipMemcpyAsync(b->res_host.data(), acc, n * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                     b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(b, DGBGK_EDEVICE, "residual copy: %s", hipGetErrorString(e));
  for (size_t i = 0; i < n; ++i) {
    double v;
    std::memcpy(&v, &b->res_host[i], sizeof v);
    if (!std::isfinite(v)) {
      v = NAN;
      rc = bfail(b, DGBGK_ENONFINITE, "member %zu: residual is not finite", i);
    }
    r[i] = v;
  }
  return rc;
}

int dgbgk_batch_launches_per_step(const dgbgk_batch *b, int32_t *launches) {
  if (!b) return bfail(nullptr, DGBGK_EINVAL, "batch is NULL");
  if (!launches) return bfail(const_cast<dgbgk_batch *>(b), DGBGK_EINVAL, "launches is NULL");
  *launches = (int32_t)(4 * (b->cls.size() + b->solo.size()));
  return DGBGK_OK;
}

const char *dgbgk_batch_last_error(const dgbgk_batch *b) {
  if (!b) return g_create_error.c_str();
  return b->err.c_str();
}

void dgbgk_batch_destroy(dgbgk_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  if (b->dev) (void)hipFree(b->dev);
  for (hipStream_t st : b->lanes) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t ev : b->lane_done) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
