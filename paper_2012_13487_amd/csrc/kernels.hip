// Device kernels of the DG-BGK library (gfx950).
//
// The hot path is one fused kernel per RK4 stage.  A work-group owns a block
// of E consecutive elements and a tile of Qt velocities (Qt = Q in fused
// mode) and, in one pass over HBM:
//   1. stages f_s[q][k][n] of its block in LDS with coalesced 16-byte loads;
//   2. reduces the node moments rho, rho u (Sec. II.A) over the velocities in
//      LDS, and the diffuse-wall densities of eq. (8) at wall face nodes;
//      in tiled mode both come from a separate moments pass instead;
//   3. per (velocity, element) row, in registers: the volume term -e.grad f
//      by sum factorisation (Dr = I x D1, Ds = D1 x I, D1 uniform across the
//      wavefront), the upwind jumps (e.n)(f^- - f^+) on the two inflow faces
//      lifted by LIFT = M^{-1} E (a rank-one outer product per face on tensor
//      GLL elements), with f^+ the neighbour trace or the wall exterior state
//      rho_w f^eq(1, u_b), and the BGK collision with the second-order
//      equilibrium eq. (5); L(f) goes back into the row in LDS;
//   4. the classical RK4 register update, streaming f_n / acc / outputs with
//      coalesced 16-byte accesses.
// The path is HBM-bound (about 2.5-5 flop per byte in FP64), so the small
// contractions run on the FP64 vector units from registers and LDS rather
// than being padded out to matrix-core tiles.
#include "kernels.hpp"

#include <cstdint>
#include <cmath>
#include <type_traits>

namespace dgbgk {

namespace {

typedef double double4v __attribute__((ext_vector_type(4)));
typedef double double2v __attribute__((ext_vector_type(2)));  // native 16-byte vector

template <int P>
struct Shape {
  static constexpr int N1 = P + 1;
  static constexpr int NP = N1 * N1;
  static constexpr int NFP = N1;
  static constexpr int S = (NP % 2 == 0) ? NP + 2 : NP;
  static constexpr int G = kBlock / NP;                   // node groups per work-group
  static constexpr int T = G * NP;                        // threads with a node
  static constexpr bool VEC = (NP % 2 == 0);              // 16-byte loads of f
};

struct LdsLayout {
  int part, mom, rw, nbr, total;  // offsets / size in doubles; the tile starts at 0
};

__host__ __device__ inline LdsLayout lds_layout(int NP, int NFP, int S, int E, int Qt) {
  LdsLayout L;
  const int tile_sz = Qt * E * S;
  const int tasks = E * ((NP + 15) / 16);
  const int pairs = tasks >= 4 ? tasks : 4;  // (task, K slice) partial products
  L.part = tile_sz;
  L.mom = (L.part + pairs * 7 * 16 + 3) / 4 * 4;  // 32-byte aligned (read as double4)
  L.rw = L.mom + E * NP * 4;
  L.nbr = L.rw + E * 4 * NFP;
  L.total = L.nbr + (E * 4 + 1) / 2;  // E*4 ints
  return L;
}

// out / new accumulator of one stage of classical RK4 from k = L(f_s), with
// the accumulator written once per step, in the second stage (f_1 - f_n =
// dt/2 k1 and f_3 - f_n = dt k3 stand for the first and third rates), so that
// stages 1 and 3 move no accumulator; where the row phase holds f_s and k it
// forms the stage's share itself (row_rhs), and kv is that value:
//   MODE 1 (stage 1): out = kv = f_s + dt/2 k
//   MODE 3 (stage 2): acc = f_n + (f_s - f_n) / 3 + dt/3 k,
//                     out = f_n + dt/2 k                          (x = f_n, y = f_s)
//   MODE 2 (stage 3): out = f_n + dt k                            (x = f_n)
//   MODE 4 (stage 4): out = acc - f_n / 3 + kv, kv = f_s / 3 + dt/6 k  (x = acc, y = f_n)
//   MODE 0: out = k
template <int MODE>
__device__ inline double rk_one(double kv, double x, double y, double ca, double co, double &an) {
  if (MODE == 0 || MODE == 1) return kv;
  if (MODE == 3) { an = x + (y - x) * (1.0 / 3.0) + ca * kv; return x + co * kv; }
  if (MODE == 2) return x + co * kv;
  return x - y * (1.0 / 3.0) + kv;
}

// The update's operands for a stage MODE, as above: x, y (y read only where
// rk_reads_y), and whether the accumulator is written.
template <int MODE>
__device__ __forceinline__ const double *rk_x(const StageArgs &a) {
  return MODE == 1 ? a.fs : (MODE == 2 || MODE == 3) ? a.fn : a.acc;
}
template <int MODE>
__device__ __forceinline__ const double *rk_y(const StageArgs &a) {
  return MODE == 3 ? a.fs : a.fn;
}
__host__ __device__ constexpr bool rk_reads_x(int mode) { return mode == 2 || mode == 3 || mode == 4; }
__host__ __device__ constexpr bool rk_reads_y(int mode) { return mode == 3 || mode == 4; }
__host__ __device__ constexpr bool rk_writes_acc(int mode) { return mode == 3; }
template <int MODE>
__device__ inline void rk_update(double kv, double x, double y, double ca, double co, double &o,
                                 double &an) {
  o = rk_one<MODE>(kv, x, y, ca, co, an);
}
template <int MODE>
__device__ inline void rk_update(const double2v &kv, const double2v &x, const double2v &y, double ca,
                                 double co, double2v &o, double2v &an) {
  double o0, o1, a0 = 0.0, a1 = 0.0;
  o0 = rk_one<MODE>(kv[0], x[0], y[0], ca, co, a0);
  o1 = rk_one<MODE>(kv[1], x[1], y[1], ca, co, a1);
  o = double2v{o0, o1};
  an = double2v{a0, a1};
}

// Work-groups are handed to the 8 XCDs round-robin; give each XCD a
// contiguous run of element blocks so that neighbour traces re-read by the
// next block are still in that XCD's L2.
__device__ inline int xcd_block(int b, int nblk) {
  const int per = nblk >> 3, rem = nblk & 7, x = b & 7;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

// Elements per strip of the strip order below (measured best on the
// 64 x 64 p = 3 cavity in FP64 and FP32 and on the 128 x 128 p = 4 cavity).
constexpr int kStripElems = 16;

// The t-th element block in strip order: the block grid (rows of bpr blocks)
// is cut into strips of kStripElems elements, each swept row by row, so that the
// work-groups resident on one XCD at a time cover a compact patch and find
// the faces of their neighbours above and below in L2.  Applies when the
// blocks tile whole mesh rows (E divides nx); otherwise the identity.
__device__ inline int strip_block(int t, int nx, int log2E, int nblk) {
  if (nx & ((1 << log2E) - 1)) return t;
  const int W = kStripElems >> log2E > 0 ? kStripElems >> log2E : 1;  // blocks per strip
  const int bpr = nx >> log2E, rows = nblk / bpr;
  const int full = bpr - bpr % W;  // columns in full-width strips
  int row, col;
  if (t < full * rows) {
    const int per = W * rows, s = t / per, in = t - s * per;
    row = in / W;
    col = s * W + in % W;
  } else {
    const int wr = bpr - full, t2 = t - full * rows;
    row = t2 / wr;
    col = full + t2 % wr;
  }
  return row * bpr + col;
}

// LDS rows have an odd stride, so 16-byte values move as two 8-byte halves.
__device__ __forceinline__ void lds_put(double *p, double v) { *p = v; }
__device__ __forceinline__ void lds_put(double *p, const double2v &v) { *reinterpret_cast<double2v *>(p) = v; }
template <typename V>
__device__ __forceinline__ V lds_get(const double *p);
template <>
__device__ __forceinline__ double lds_get<double>(const double *p) { return *p; }
template <>
__device__ __forceinline__ double2v lds_get<double2v>(const double *p) { return *reinterpret_cast<const double2v *>(p); }

// n / d for 0 <= n < 2^22, d >= 1: a reciprocal estimate, then one exact
// correction step.
__device__ __forceinline__ int div_small(int n, int d) {
  int t = (int)(((float)n + 0.5f) * __builtin_amdgcn_rcpf((float)d));
  if (t * d > n) --t;
  if ((t + 1) * d <= n) ++t;
  return t;
}

// f is stored element-major, f[k][q][n]: the Q velocity rows of an element are
// consecutive, each NP contiguous nodes.  A block tile (E elements, Qb
// velocities from q0) is read in memory order: access c (CW doubles; CPE per
// velocity row) is element e, velocity q, access w within the row, at offset
// e * Q * NP + q * NP + CW * w from the tile origin.
template <int CPE>
__device__ __forceinline__ void split_access(int c, int Qb, int E, int &q, int &e, int &w) {
  const int cq = c / CPE;
  w = c - cq * CPE;
  e = E == 1 ? 0 : div_small(cq, Qb);
  q = cq - e * Qb;
}

// Exterior traces of the two inflow faces of one velocity row: a column of the
// x-neighbour (stride N1) and a contiguous row of the y-neighbour (two nodes
// per 16-byte access when N1 is even: that row then starts 16-byte aligned).
template <int N1, int NFP>
__device__ __forceinline__ void load_face_traces(const double *sx, const double *sy, bool gx, bool gy,
                                                 double (&px)[NFP], double (&py)[NFP]) {
#pragma unroll
  for (int m = 0; m < NFP; ++m) px[m] = gx ? sx[N1 * m] : 0.0;
  if (N1 % 2 == 0) {
#pragma unroll
    for (int m = 0; m < NFP; m += 2) {
      double2v v = {0.0, 0.0};
      if (gy) v = *reinterpret_cast<const double2v *>(sy + m);
      py[m] = v[0];
      py[m + 1] = v[1];
    }
  } else {
#pragma unroll
    for (int m = 0; m < NFP; ++m) py[m] = gy ? sy[m] : 0.0;
  }
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

// Global accesses at a wave-uniform base plus a 32-bit per-lane offset (in
// doubles; the caller guarantees offset * 8 < 2^32), so that each access
// needs one offset register rather than a 64-bit address.
template <typename V>
__device__ __forceinline__ V ld32(const double *base, uint32_t off) {
  return *reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + (off << 3));
}
template <typename V>
__device__ __forceinline__ void st32(double *base, uint32_t off, const V &v) {
  *reinterpret_cast<V *>(reinterpret_cast<char *>(base) + (off << 3)) = v;
}

// Coalesced copy of a block's f tile (E elements x Qb velocities) between HBM
// and registers: access u of a thread is c = tid + u * nthr.
template <int CPE, int CW, int NP, int PF, typename V>
__device__ __forceinline__ void load_tile(V (&pf)[PF], const double *src, int tid, int nthr, int nch,
                                          int Qb, int E, int Eb, uint32_t QNP) {
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const int c = tid + u * nthr;
    int q, e, w;
    split_access<CPE>(c, Qb, E, q, e, w);
    if (c < nch && e < Eb) pf[u] = ld32<V>(src, (uint32_t)e * QNP + (uint32_t)(q * NP + CW * w));
  }
}

// Node moments and diffuse-wall densities of a block whose f tile is in LDS.
// C[c][n] = sum_q W[q][c] f[q][n] with W[q] = (1, e_x, e_y, outgoing normal
// speed at the bottom, right, top, left wall): a dense (7 x Q) x (Q x NP)
// product per element, on FP64 matrix cores (16x16x4 steps; K split over the
// wavefronts, partial products summed through LDS).  wsrc points at the
// weights of the block's first velocity ([q][16]).  Threads 0..nthr-1 take
// part; this writes the partial products, and block_moments_combine (after a
// barrier) sums them.  KB 4-velocity steps have their operands loaded
// together.
__host__ __device__ inline int moment_slices(int P, int E) {
  const int tasks = E * (((P + 1) * (P + 1) + 15) / 16);
  return tasks >= 4 ? 1 : 4 / tasks;
}

// Moment weight c of a velocity (the columns of W above): 1, e_x, e_y, then
// the outgoing normal speed at the bottom, right, top and left wall.
__device__ __forceinline__ double moment_weight(int c, double cx, double cy) {
  switch (c) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return cy < 0.0 ? -cy : 0.0;
    case 4: return cx > 0.0 ? cx : 0.0;
    case 5: return cy > 0.0 ? cy : 0.0;
    case 6: return cx < 0.0 ? -cx : 0.0;
    default: return 0.0;
  }
}

// WV: wsrc holds the velocities (e_x[Qb] then e_y[Qb]) and the weights are
// formed in registers; otherwise wsrc is the [q][16] weight table.
template <int P, int KB, bool WV = false>
__device__ __forceinline__ void block_moments_mfma(const double *tile, double *part, const double *wsrc,
                                                   int E, int Qb, int Eb, int tid, int nthr) {
  using Sh = Shape<P>;
  constexpr int NP = Sh::NP, S = Sh::S;
  constexpr int NB = (NP + 15) / 16;  // 16-node column blocks of the moment product
  const int wave = tid >> 6, lane = tid & 63;
  const int tasks = E * NB;                     // (element, 16-node block)
  const int ks = moment_slices(P, E);           // K slices per task
  const int qper = ((Qb + ks - 1) / ks + 3) / 4 * 4;
  for (int pr = wave; pr < tasks * ks; pr += nthr >> 6) {
    const int t = pr / ks, sl = pr % ks;
    const int e = t / NB, nb = t % NB;
    const int node = nb * 16 + (lane & 15);
    const int qa = sl * qper, qe = min(Qb, qa + qper);
    double4v acc = {0.0, 0.0, 0.0, 0.0}, acc1 = acc, acc2 = acc, acc3 = acc;
    if (e < Eb) {
#pragma unroll 1
      for (int qb = qa; qb < qe; qb += 4 * KB) {
        double av[KB], bv[KB];
#pragma unroll
        for (int t2 = 0; t2 < KB; ++t2) {
          const int q = qb + 4 * t2 + (lane >> 4);
          const bool in = q < qe;
          if (WV) av[t2] = in ? moment_weight(lane & 15, wsrc[q], wsrc[Qb + q]) : 0.0;
          else av[t2] = in ? wsrc[(size_t)q * 16 + (lane & 15)] : 0.0;
          bv[t2] = (in && node < NP) ? tile[(q * E + e) * S + node] : 0.0;
        }
#pragma unroll
        for (int t2 = 0; t2 < KB; t2 += 4) {  // four independent accumulation chains
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t2], bv[t2], acc, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t2 + 1], bv[t2 + 1], acc1, 0, 0, 0);
          acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t2 + 2], bv[t2 + 2], acc2, 0, 0, 0);
          acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t2 + 3], bv[t2 + 3], acc3, 0, 0, 0);
        }
      }
    }
    acc += acc1 + acc2 + acc3;
    // register v of a lane holds C[4 v + lane / 16][lane % 16]; rows 0..6 are used
    if (node < NP) {
      double *pp = part + ((size_t)pr * 7) * 16;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int row = 4 * v + (lane >> 4);
        if (row < 7) pp[row * 16 + (lane & 15)] = acc[v];
      }
    }
  }
}

// Sums the partial products into mom (ux, uy, rho, 1 - |u|^2 / (2 theta) per
// node) and the wall densities rw ([e][face][NFP]); the caller synchronises
// afterwards.
template <int P>
__device__ __forceinline__ void block_moments_combine(const StageArgs &a, const double *part,
                                                      double *mom, double *rw, const int *nbr,
                                                      int E, int Eb, int k0, int tid) {
  using Sh = Shape<P>;
  constexpr int N1 = Sh::N1, NP = Sh::NP, NFP = Sh::NFP;
  constexpr int NB = (NP + 15) / 16;
  const int ks = moment_slices(P, E);
  if (tid < E * NP) {
    const int e2 = tid / NP, n2 = tid % NP;
    if (e2 < Eb) {
      const int t = e2 * NB + n2 / 16, col = n2 % 16;
      double sm[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int sl = 0; sl < ks; ++sl) {
        const double *pp = part + ((size_t)(t * ks + sl) * 7) * 16;
#pragma unroll
        for (int c = 0; c < 7; ++c) sm[c] += pp[c * 16 + col];
      }
      const double rho = sm[0], ux = sm[1] / rho, uy = sm[2] / rho;
      double *m = mom + (e2 * NP + n2) * 4;
      m[0] = ux;
      m[1] = uy;
      m[2] = rho;
      m[3] = 1.0 - (ux * ux + uy * uy) * a.half_theta_inv;
      if (a.wall_mask != 0) {
        const int i2 = n2 % N1, j2 = n2 / N1;
        const bool on[4] = {nbr[e2 * 4 + 0] < 0 && j2 == 0, nbr[e2 * 4 + 1] < 0 && i2 == P,
                            nbr[e2 * 4 + 2] < 0 && j2 == P, nbr[e2 * 4 + 3] < 0 && i2 == 0};
        const int fm[4] = {i2, j2, i2, j2};
#pragma unroll
        for (int fc = 0; fc < 4; ++fc)
          if (on[fc]) {
            const double v = sm[3 + fc] * a.wall_den_inv[fc];
            rw[(e2 * 4 + fc) * NFP + fm[fc]] = v;
            if (a.rhow_out) a.rhow_out[((size_t)(k0 + e2) * 4 + fc) * NFP + fm[fc]] = v;
          }
      }
    }
  }
}

// Exterior traces of the two inflow faces of velocity qg at element k (zero
// where the face is a wall or the velocity is parallel to it).
template <int P>
__device__ __forceinline__ void row_traces(const StageArgs &a, int qg, int k, int nbx, int nby,
                                           double (&px)[P + 1], double (&py)[P + 1]) {
  constexpr int N1 = P + 1, NP = N1 * N1;
  const double cx = a.vel[qg], cy = a.vel[a.Q + qg];
  const bool gx = cx != 0.0 && nbx >= 0, gy = cy != 0.0 && nby >= 0;
  const double *sx = a.fs + ((size_t)(nbx >= 0 ? nbx : 0) * a.Q + qg) * NP + (cx > 0.0 ? P : 0);
  const double *sy = a.fs + ((size_t)(nby >= 0 ? nby : 0) * a.Q + qg) * NP + (cy > 0.0 ? N1 * P : 0);
  load_face_traces<N1, N1>(sx, sy, gx, gy, px, py);
  (void)k;
}

// As row_traces, with 32-bit offsets from the base of f_s.
template <int P>
__device__ __forceinline__ void row_traces32(const StageArgs &a, double cx, double cy, int qg, int nbx,
                                             int nby, double (&px)[P + 1], double (&py)[P + 1]) {
  constexpr int N1 = P + 1, NP = N1 * N1;
  const bool gx = cx != 0.0 && nbx >= 0, gy = cy != 0.0 && nby >= 0;
  const uint32_t ox = ((uint32_t)(nbx >= 0 ? nbx : 0) * a.Q + qg) * NP + (cx > 0.0 ? P : 0);
  const uint32_t oy = ((uint32_t)(nby >= 0 ? nby : 0) * a.Q + qg) * NP + (cy > 0.0 ? N1 * P : 0);
#pragma unroll
  for (int m = 0; m < N1; ++m) px[m] = gx ? ld32<double>(a.fs, ox + N1 * m) : 0.0;
  if (N1 % 2 == 0) {
#pragma unroll
    for (int m = 0; m < N1; m += 2) {
      double2v v = {0.0, 0.0};
      if (gy) v = ld32<double2v>(a.fs, oy + m);
      py[m] = v[0];
      py[m + 1] = v[1];
    }
  } else {
#pragma unroll
    for (int m = 0; m < N1; ++m) py[m] = gy ? ld32<double>(a.fs, oy + m) : 0.0;
  }
}

// L(f) of one (velocity, element) row held in LDS: its NP nodal values go to
// registers; the derivative and lift tables are wave-uniform scalars.  mm is
// the element's moment table, rwe its wall densities ([face][NFP]).  The
// result overwrites the row.
// RowVel: the velocity data of one row (e_x, e_y, w and the wall exterior
// states f^eq(1, u_b) of its two inflow faces).
struct RowVel {
  double cx, cy, wq, gbx, gby;
};

__device__ __forceinline__ RowVel row_vel(const StageArgs &a, int qg) {
  RowVel v;
  v.cx = a.vel[qg];
  v.cy = a.vel[a.Q + qg];
  v.wq = a.vel[2 * a.Q + qg];
  v.gbx = a.feqb[(v.cx > 0.0 ? 3 : 1) * a.Q + qg];
  v.gby = a.feqb[(v.cy > 0.0 ? 0 : 2) * a.Q + qg];
  return v;
}

template <int P, int MODE = 0>
__device__ __forceinline__ void row_rhs(const StageArgs &a, double *row, const double *mm,
                                        const double *rwe, const RowVel &rv, int nbx, int nby,
                                        const double (&px)[P + 1], const double (&py)[P + 1]) {
  using Sh = Shape<P>;
  constexpr int N1 = Sh::N1, NP = Sh::NP, NFP = Sh::NFP;
  const double cx = rv.cx, cy = rv.cy, wq = rv.wq;
  const int fxc = cx > 0.0 ? 3 : 1, fyc = cy > 0.0 ? 0 : 2;  // inflow faces
  double f[NP];
  if (Sh::VEC) {
#pragma unroll
    for (int c = 0; c < NP / 2; ++c) {
      const double2v v = *reinterpret_cast<const double2v *>(row + 2 * c);
      f[2 * c] = v[0];
      f[2 * c + 1] = v[1];
    }
  } else {
#pragma unroll
    for (int c = 0; c < NP; ++c) f[c] = row[c];
  }
  double kk[NP];
  const double ax = cx * a.rx, ay = cy * a.sy;
#pragma unroll
  for (int j = 0; j < N1; ++j)
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      double dr = 0.0, ds = 0.0;
#pragma unroll
      for (int m = 0; m < N1; ++m) {
        dr += a.D1[i * N1 + m] * f[m + N1 * j];
        ds += a.D1[j * N1 + m] * f[i + N1 * m];
      }
      kk[i + N1 * j] = -(ax * dr + ay * ds);
    }
  if (cx != 0.0) {
    const double wx = a.fsx * (-fabs(cx));
    const double gbx = rv.gbx;
    const double *rwx = rwe + fxc * NFP;
#pragma unroll
    for (int jj = 0; jj < N1; ++jj) {
      const double own = cx > 0.0 ? f[N1 * jj] : f[N1 * jj + P];
      const double ext = nbx >= 0 ? px[jj] : rwx[jj] * gbx;
      const double J = wx * (own - ext);
#pragma unroll
      for (int ii = 0; ii < N1; ++ii) kk[ii + N1 * jj] += (cx > 0.0 ? a.lift_lo[ii] : a.lift_hi[ii]) * J;
    }
  }
  if (cy != 0.0) {
    const double wy = a.fsy * (-fabs(cy));
    const double gby = rv.gby;
    const double *rwy = rwe + fyc * NFP;
#pragma unroll
    for (int ii = 0; ii < N1; ++ii) {
      const double own = cy > 0.0 ? f[ii] : f[ii + N1 * P];
      const double ext = nby >= 0 ? py[ii] : rwy[ii] * gby;
      const double J = wy * (own - ext);
#pragma unroll
      for (int jj = 0; jj < N1; ++jj) kk[ii + N1 * jj] += (cy > 0.0 ? a.lift_lo[jj] : a.lift_hi[jj]) * J;
    }
  }
#pragma unroll
  for (int nn = 0; nn < NP; ++nn) {
    const double4v m4 = *reinterpret_cast<const double4v *>(mm + 4 * nn);
    const double eu = cx * m4[0] + cy * m4[1];
    const double feq = wq * m4[2] * (m4[3] + eu * (a.theta_inv + eu * a.half_theta2_inv));
    kk[nn] += (feq - f[nn]) * a.inv_tau;
  }
  if constexpr (MODE == 1) {  // the first RK4 stage's output, f_s + dt/2 L(f_s)
#pragma unroll
    for (int c = 0; c < NP; ++c) kk[c] = f[c] + a.c_out * kk[c];
  } else if constexpr (MODE == 4) {  // the last stage's share, f_3 / 3 + dt/6 L(f_3)
#pragma unroll
    for (int c = 0; c < NP; ++c) kk[c] = f[c] * (1.0 / 3.0) + a.c_acc * kk[c];
  }
  if (Sh::VEC) {
#pragma unroll
    for (int c = 0; c < NP / 2; ++c)
      *reinterpret_cast<double2v *>(row + 2 * c) = double2v{kk[2 * c], kk[2 * c + 1]};
  } else {
#pragma unroll
    for (int c = 0; c < NP; ++c) row[c] = kk[c];
  }
}

// Loads and stores of the streams that are touched once per stage, with or
// without non-temporal hints.
template <bool NT, typename V>
__device__ __forceinline__ V ld_once(const double *p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
  return *reinterpret_cast<const V *>(p);
}
template <bool NT, typename V>
__device__ __forceinline__ void st_once(double *p, const V &v) {
  if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
  else *reinterpret_cast<V *>(p) = v;
}

// Phase 4 of a stage: the RK4 register update of the block, coalesced over
// each velocity row; L(f) of the block is in the LDS tile.  With NT, x and
// the accumulator, read once per stage and not again before the next
// launch, move with non-temporal hints so that they do not evict the tiles
// neighbours still gather from (used when the state arrays exceed the
// last-level cache); the stage output, the next stage's input, is always
// stored normally.
template <int P, int MODE, bool NT>
__device__ __forceinline__ void update_rows(const StageArgs &a, const double *tile, size_t boff, int Qb,
                                            int E, int Eb, int nch, bool full, int tid, int nthr) {
  using Sh = Shape<P>;
  constexpr int NP = Sh::NP, S = Sh::S;
  constexpr int CW = Sh::VEC ? 2 : 1;
  constexpr int CPE = NP / CW;
  constexpr int U = 8;
  using V = typename std::conditional<Sh::VEC, double2v, double>::type;
  const size_t QNP = (size_t)a.Q * NP;
  const double cacc = a.c_acc, cout = a.c_out;
  // x: f_n (stages 2, 3), acc (stage 4); y: f_s (stage 2), f_n (stage 4)
  const double *xr = rk_x<MODE>(a) + boff;
  const double *yr = rk_y<MODE>(a) + boff;
  double *accr = a.acc + boff;
  double *outr = a.out + boff;
  for (int c0 = tid; c0 < nch; c0 += nthr * U) {
    V kv[U], x[U], y[U];
    size_t go[U];
    bool ok[U];
    const bool all = full && c0 - tid + U * nthr <= nch;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * nthr;
      int q, e, w;
      split_access<CPE>(c, Qb, E, q, e, w);
      ok[u] = all || (c < nch && e < Eb);
      go[u] = e * QNP + q * NP + CW * w;
      if (ok[u]) kv[u] = lds_get<V>(tile + (q * E + e) * S + CW * w);
    }
    if (rk_reads_x(MODE)) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) x[u] = ld_once<NT, V>(xr + go[u]);
    }
    if (rk_reads_y(MODE)) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) y[u] = ld_once<NT, V>(yr + go[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      V o, an;
      rk_update<MODE>(kv[u], x[u], y[u], cacc, cout, o, an);
      *reinterpret_cast<V *>(outr + go[u]) = o;
      if (rk_writes_acc(MODE)) st_once<NT, V>(accr + go[u], an);
    }
  }
}

// One pass of phase 4 (16 accesses per thread from c0), the same update as
// update_rows; the velocity-tiled block loops over passes itself, a code
// layout that measured faster there.
template <int P, int MODE, bool NT>
__device__ __forceinline__ void update_pass(const StageArgs &a, const double *tile, const double *xr,
                                            double *accr, double *outr, int c0, int Qb, int E, int Eb,
                                            int nch, bool full, int tid, int nthr, double *keep) {
  using Sh = Shape<P>;
  constexpr int NP = Sh::NP, S = Sh::S;
  constexpr int CW = Sh::VEC ? 2 : 1;
  constexpr int CPE = NP / CW;
  constexpr int U = Sh::VEC ? 8 : 16;  // (as stage_block: its pass loop steps by this)
  using V = typename std::conditional<Sh::VEC, double2v, double>::type;
  const size_t QNP = (size_t)a.Q * NP;
  const double cacc = a.c_acc, cout = a.c_out;
  const double *yr = rk_y<MODE>(a) + (accr - a.acc);  // (at the tile's offset)
  V kv[U], x[U], y[U];
  size_t go[U];
  bool ok[U];
  const bool all = full && c0 - tid + U * nthr <= nch;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int c = c0 + u * nthr;
    int q, e, w;
    split_access<CPE>(c, Qb, E, q, e, w);
    ok[u] = all || (c < nch && e < Eb);
    go[u] = e * QNP + q * NP + CW * w;
    if (ok[u]) kv[u] = lds_get<V>(tile + (q * E + e) * S + CW * w);
  }
  if (rk_reads_x(MODE)) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) x[u] = ld_once<NT, V>(xr + go[u]);
  }
  if (rk_reads_y(MODE)) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) y[u] = ld_once<NT, V>(yr + go[u]);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (!ok[u]) continue;
    V o, an;
    rk_update<MODE>(kv[u], x[u], y[u], cacc, cout, o, an);
    *reinterpret_cast<V *>(outr + go[u]) = o;
    if (rk_writes_acc(MODE)) st_once<NT, V>(accr + go[u], an);
    if (keep) {  // the output replaces L(f) at the same LDS position (this thread's own)
      const int c = c0 + u * nthr;
      int q, e, w;
      split_access<CPE>(c, Qb, E, q, e, w);
      lds_put(keep + (q * E + e) * S + CW * w, o);
    }
  }
}

// Phase 4 of a velocity tile whose output's moment partials the next stage
// reads.  Thread t takes node n = t % NP of the velocity rows g, g + G, g + 2G,
// ... (g = t / NP, G = nthr / NP groups): a wavefront's lanes cover
// consecutive nodes of consecutive rows, so the accesses stay coalesced, and
// each thread sums the moment weights (1, e_x, e_y, the outgoing normal
// speeds) times its outputs in registers; the groups' sums are then added in
// LDS in a fixed order and written to pout.  The tile must hold 7 G NP
// doubles (the caller checks).
template <int P, int MODE, bool NT>
__device__ __forceinline__ void update_columns(const StageArgs &a, double *tile, const double *xr,
                                               double *accr, double *outr, int Qb, int q0, int tid,
                                               int nthr, double *po) {
  using Sh = Shape<P>;
  constexpr int NP = Sh::NP, S = Sh::S;
  constexpr int U = 8;
  const int G = nthr / NP;
  const int g = tid / NP, n = tid - g * NP;
  const double cacc = a.c_acc, cout = a.c_out;
  const double *yr = rk_y<MODE>(a) + (accr - a.acc);  // (at the tile's offset)
  double sm[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (g < G) {
    for (int qa = g; qa < Qb; qa += G * U) {
      double kv[U], x[U], y[U], cx[U], cy[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = qa + u * G;
        if (q < Qb) {
          kv[u] = tile[q * S + n];
          cx[u] = a.vel[q0 + q];
          cy[u] = a.vel[a.Q + q0 + q];
        }
      }
      if (rk_reads_x(MODE)) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = qa + u * G;
          if (q < Qb) x[u] = ld_once<NT, double>(xr + (size_t)q * NP + n);
        }
      }
      if (rk_reads_y(MODE)) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = qa + u * G;
          if (q < Qb) y[u] = ld_once<NT, double>(yr + (size_t)q * NP + n);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = qa + u * G;
        if (q >= Qb) continue;
        double o, an = 0.0;
        rk_update<MODE>(kv[u], x[u], y[u], cacc, cout, o, an);
        outr[(size_t)q * NP + n] = o;
        if (rk_writes_acc(MODE)) st_once<NT, double>(accr + (size_t)q * NP + n, an);
        const double ex = cx[u], ey = cy[u];
        sm[0] += o;
        sm[1] += ex * o;
        sm[2] += ey * o;
        sm[3] += (ey < 0.0 ? -ey : 0.0) * o;
        sm[4] += (ex > 0.0 ? ex : 0.0) * o;
        sm[5] += (ey > 0.0 ? ey : 0.0) * o;
        sm[6] += (ex < 0.0 ? -ex : 0.0) * o;
      }
    }
  }
  __syncthreads();  // every tile value is consumed: the groups' sums go there
  if (g < G) {
#pragma unroll
    for (int c = 0; c < 7; ++c) tile[(g * 7 + c) * NP + n] = sm[c];
  }
  __syncthreads();
  if (tid < 7 * NP) {
    const int c = tid / NP, n2 = tid - c * NP;
    double v = 0.0;
    for (int gg = 0; gg < G; ++gg) v += tile[(gg * 7 + c) * NP + n2];
    po[c * NP + n2] = v;
  }
}

// Whether one-element fused blocks of order P hand their output's moments to
// the next stage: each thread's accesses of phase 4 then stay on one column
// of CW nodes, and the four wavefronts' sums fit the partial-product area.
template <int P>
__host__ __device__ constexpr bool handoff_order() {
  constexpr int NP = (P + 1) * (P + 1), CPE = NP % 2 == 0 ? NP / 2 : NP;
  return kBlock % CPE == 0 && 64 % CPE == 0 && 4 * 7 * NP <= 4 * 7 * 16;
}

static_assert(handoff_order<1>() == handoff_moments(1) && handoff_order<2>() == handoff_moments(2) &&
                  handoff_order<3>() == handoff_moments(3) && handoff_order<4>() == handoff_moments(4) &&
                  handoff_order<5>() == handoff_moments(5) && handoff_order<6>() == handoff_moments(6) &&
                  handoff_order<7>() == handoff_moments(7) && handoff_order<8>() == handoff_moments(8),
              "the host's choice of orders that hand over moments matches the kernel's");

// Phase 4 of a one-element fused block (the accesses of update_rows) that
// also sums the moments of its output over the velocities, per node, for the
// next stage: rows 0..2 of po (1, e_x, e_y), and rows 3..6 (the outgoing
// normal speed at each wall) when WALL.  Each thread keeps one column of CW
// nodes; the column sums are reduced across the lanes of a wavefront, then
// across the wavefronts in red (4 x 7 x NP doubles).
template <int P, int MODE, bool NT, bool WALL>
__device__ __forceinline__ void update_rows_handoff(const StageArgs &a, const double *tile, size_t boff,
                                                    int Qb, int tid, int nthr, double *red,
                                                    double *po) {
  using Sh = Shape<P>;
  constexpr int NP = Sh::NP, S = Sh::S;
  constexpr int CW = Sh::VEC ? 2 : 1;
  constexpr int CPE = NP / CW;
  constexpr int U = 4;  // (8 measured slower: more registers, fewer resident work-groups)
  constexpr int W = WALL ? 7 : 3;
  using V = typename std::conditional<Sh::VEC, double2v, double>::type;
  const double cacc = a.c_acc, cout = a.c_out;
  const double *xr = rk_x<MODE>(a) + boff;
  const double *yr = rk_y<MODE>(a) + boff;
  double *accr = a.acc + boff;
  double *outr = a.out + boff;
  const int w = tid % CPE;  // nthr is a multiple of CPE: the column never changes
  const int nch = Qb * CPE;
  double sm[W][CW];
#pragma unroll
  for (int c = 0; c < W; ++c)
#pragma unroll
    for (int j = 0; j < CW; ++j) sm[c][j] = 0.0;
  for (int c0 = tid; c0 < nch; c0 += nthr * U) {
    V kv[U], x[U], y[U];
    double ex[U], ey[U];
    int go[U];
    bool ok[U];
    const bool all = c0 - tid + U * nthr <= nch;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * nthr;
      const int q = c / CPE;
      ok[u] = all || c < nch;
      go[u] = q * NP + CW * w;
      if (ok[u]) {
        kv[u] = lds_get<V>(tile + q * S + CW * w);
        ex[u] = a.vel[q];
        ey[u] = a.vel[a.Q + q];
      }
    }
    if (rk_reads_x(MODE)) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) x[u] = ld_once<NT, V>(xr + go[u]);
    }
    if (rk_reads_y(MODE)) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) y[u] = ld_once<NT, V>(yr + go[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!ok[u]) continue;
      V o, an;
      rk_update<MODE>(kv[u], x[u], y[u], cacc, cout, o, an);
      *reinterpret_cast<V *>(outr + go[u]) = o;
      if (rk_writes_acc(MODE)) st_once<NT, V>(accr + go[u], an);
      const double *ov = reinterpret_cast<const double *>(&o);
      double wt[W];
      wt[0] = 1.0;
      wt[1] = ex[u];
      wt[2] = ey[u];
      if (WALL) {
        wt[3 % W] = ey[u] < 0.0 ? -ey[u] : 0.0;
        wt[4 % W] = ex[u] > 0.0 ? ex[u] : 0.0;
        wt[5 % W] = ey[u] > 0.0 ? ey[u] : 0.0;
        wt[6 % W] = ex[u] < 0.0 ? -ex[u] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < W; ++c)
#pragma unroll
        for (int j = 0; j < CW; ++j) sm[c][j] += wt[c] * ov[j];
    }
  }
  // lanes with the same column are CPE apart within a wavefront
#pragma unroll
  for (int m = CPE; m < 64; m <<= 1)
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
      for (int j = 0; j < CW; ++j) sm[c][j] += __shfl_xor(sm[c][j], m);
  const int wave = tid >> 6, lane = tid & 63;
  if (lane < CPE) {
#pragma unroll
    for (int c = 0; c < W; ++c)
#pragma unroll
      for (int j = 0; j < CW; ++j) red[(wave * 7 + c) * NP + CW * lane + j] = sm[c][j];
  }
  __syncthreads();
  if (tid < W * NP) {
    const int c = tid / NP, n = tid - c * NP;
    double v = 0.0;
    for (int wv = 0; wv < (nthr >> 6); ++wv) v += red[(wv * 7 + c) * NP + n];
    po[c * NP + n] = v;
  }
}

// MODE: 0 writes L(f_s); 1 first RK4 stage; 3 second; 2 third; 4 fourth (see rk_one).
// FUSED: the block reduces its own moments and wall densities (a.fused).
// One element block blk and velocity tile tile_y of the stage, by one
// work-group; the body of the general kernel and of the batched kernel.
// NTM: 0 the cache policy of phase 4 is chosen at run time (a.stream_nt);
// 1 / 2 it is fixed to non-temporal / normal at compile time.
// EFIX: elements per work-group fixed at compile time (0: a.E at run time).
template <int P, int MODE, bool FUSED, int NTM, int EFIX = 0, bool HO = false>
__device__ __forceinline__ void stage_block(const StageArgs &a, int blk, int tile_y) {
  using Sh = Shape<P>;
  constexpr int NP = Sh::NP, NFP = Sh::NFP, S = Sh::S;
  constexpr int CW = Sh::VEC ? 2 : 1;  // doubles per global access
  constexpr int CPE = NP / CW;         // accesses per element per velocity
  // global accesses in flight per thread (measured: 8 for fused blocks,
  // 16 for velocity tiles: 2850 -> 2640 us on the 128x128 p = 4 cavity)
  constexpr int U = (FUSED || Sh::VEC) ? 8 : 16;
  using V = typename std::conditional<Sh::VEC, double2v, double>::type;
  extern __shared__ double lds[];
  const int E = EFIX > 0 ? EFIX : a.E, log2E = EFIX == 1 ? 0 : a.log2E;
  const LdsLayout L = lds_layout(NP, NFP, S, E, a.Qt);
  double *tile = lds;
  double *part = lds + L.part;
  double *mom = lds + L.mom;
  double *rw = lds + L.rw;
  int *nbr = (int *)(lds + L.nbr);

  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int k0 = blk * E;
  const int Eb = min(E, a.K - k0);
  const int q0 = tile_y * a.Qt;
  const int Qb = min(a.Qt, a.Q - q0);
  const int rows = Qb * E;  // LDS row r = q_local * E + e
  const int nch = rows * CPE;
  const size_t KN = (size_t)a.K * NP;
  const size_t QNP = (size_t)a.Q * NP;
  const size_t boff = (size_t)k0 * QNP + (size_t)q0 * NP;  // tile origin in f

  // ---- 0. neighbours of the block's elements (-1: wall) -----------------------
  if (tid < E * 4) {
    const int e = tid >> 2, fc = tid & 3;
    nbr[tid] = e < Eb ? neighbour(k0 + e, fc, a) : -1;
  }
  // one-element fused blocks read the moments of f_s handed over by the stage
  // that wrote it; the loads are issued before the tile's
  const bool handoff = FUSED && E == 1 && handoff_order<P>();
  const bool pin1 = HO || (handoff && a.pin != nullptr);
  // (rows 3..6 of the moments, the wall sums, exist only where the element
  // has a wall face; the flag is formed by every thread: measured faster than
  // by the loading threads alone)
  const bool we = handoff && a.wall_mask != 0 &&
                  (neighbour(k0, 0, a) < 0 || neighbour(k0, 1, a) < 0 || neighbour(k0, 2, a) < 0 ||
                   neighbour(k0, 3, a) < 0);
  double pv[7];
  if (pin1 && tid < NP) {
    const double *pp = a.pin + (size_t)k0 * 7 * NP + tid;
#pragma unroll
    for (int c = 0; c < 3; ++c) pv[c] = pp[c * NP];
    if (we) {
#pragma unroll
      for (int c = 3; c < 7; ++c) pv[c] = pp[c * NP];
    }
  }

  // ---- 1. f_s of the block into LDS (coalesced, U accesses in flight) ----------
  const bool full = Eb == E;
  {
    const double *src = a.fs + boff;
    for (int c0 = tid; c0 < nch; c0 += nthr * U) {
      V v[U];
      const bool all = full && c0 - tid + U * nthr <= nch;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * nthr;
        int q, e, w;
        split_access<CPE>(c, Qb, E, q, e, w);
        if (all || (c < nch && e < Eb)) v[u] = *reinterpret_cast<const V *>(src + e * QNP + q * NP + CW * w);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * nthr;
        int q, e, w;
        split_access<CPE>(c, Qb, E, q, e, w);
        if (all || (c < nch && e < Eb)) lds_put(tile + (q * E + e) * S + CW * w, v[u]);
      }
    }
  }
  __syncthreads();

  // ---- 2. node moments and diffuse-wall densities ----------------------------
  if (pin1) {
    if (tid < NP) {
      const int n2 = tid;
      const double rho = pv[0], ux = pv[1] / rho, uy = pv[2] / rho;
      double *m = mom + n2 * 4;
      m[0] = ux;
      m[1] = uy;
      m[2] = rho;
      m[3] = 1.0 - (ux * ux + uy * uy) * a.half_theta_inv;
      if (a.wall_mask != 0) {
        constexpr int N1 = Sh::N1;
        const int i2 = n2 % N1, j2 = n2 / N1;
        const bool on[4] = {nbr[0] < 0 && j2 == 0, nbr[1] < 0 && i2 == P, nbr[2] < 0 && j2 == P,
                            nbr[3] < 0 && i2 == 0};
        const int fm[4] = {i2, j2, i2, j2};
#pragma unroll
        for (int fc = 0; fc < 4; ++fc)
          if (on[fc]) rw[fc * NFP + fm[fc]] = pv[3 + fc] * a.wall_den_inv[fc];
      }
    }
  } else if (a.pin) {
    // the moments of f_s summed from the velocity tiles' partials (one tile in
    // the fused form), written by the stage that produced f_s
    if (tid < E * NP) {
      const int e2 = tid / NP, n2 = tid % NP;
      if (e2 < Eb) {
        double sm[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const int ntl = (int)gridDim.y;
        for (int t = 0; t < ntl; ++t) {
          const double *pp = a.pin + (((size_t)t * a.K + k0 + e2) * 7) * NP + n2;
#pragma unroll
          for (int c = 0; c < 7; ++c) sm[c] += pp[c * NP];
        }
        const double rho = sm[0], ux = sm[1] / rho, uy = sm[2] / rho;
        double *m = mom + (e2 * NP + n2) * 4;
        m[0] = ux;
        m[1] = uy;
        m[2] = rho;
        m[3] = 1.0 - (ux * ux + uy * uy) * a.half_theta_inv;
        if (a.wall_mask != 0) {
          constexpr int N1 = Sh::N1;
          const int i2 = n2 % N1, j2 = n2 / N1;
          const bool on[4] = {nbr[e2 * 4 + 0] < 0 && j2 == 0, nbr[e2 * 4 + 1] < 0 && i2 == P,
                              nbr[e2 * 4 + 2] < 0 && j2 == P, nbr[e2 * 4 + 3] < 0 && i2 == 0};
          const int fm[4] = {i2, j2, i2, j2};
#pragma unroll
          for (int fc = 0; fc < 4; ++fc)
            if (on[fc]) rw[(e2 * 4 + fc) * NFP + fm[fc]] = sm[3 + fc] * a.wall_den_inv[fc];
        }
      }
    }
  } else if (FUSED && !HO) {
    block_moments_mfma<P, 16>(tile, part, a.wmom + (size_t)q0 * 16, E, Qb, Eb, tid, nthr);
    __syncthreads();
    block_moments_combine<P>(a, part, mom, rw, nbr, E, Eb, k0, tid);
  } else {
    if (tid < E * NP) {
      const int e2 = tid / NP, n2 = tid % NP;
      if (e2 < Eb) {
        const size_t node = (size_t)(k0 + e2) * NP + n2;
        const double rho = a.mom[node], ux = a.mom[KN + node], uy = a.mom[2 * KN + node];
        double *m = mom + (e2 * NP + n2) * 4;
        m[0] = ux;
        m[1] = uy;
        m[2] = rho;
        m[3] = 1.0 - (ux * ux + uy * uy) * a.half_theta_inv;
      }
    }
    if (a.wall_mask != 0) {
      for (int u = tid; u < E * 4 * NFP; u += nthr) {
        const int e2 = u / (4 * NFP);
        if (e2 < Eb) rw[u] = a.rhow[(size_t)(k0 + e2) * 4 * NFP + (u - e2 * 4 * NFP)];
      }
    }
  }
  __syncthreads();

  // ---- 3. per velocity row: L(f) = volume + lifted inflow jumps + collision ----
  for (int r = tid; r < rows; r += nthr) {
    const int q = r >> log2E, e = r & (E - 1);
    if (e >= Eb) continue;
    const int qg = q0 + q;
    const RowVel rv = row_vel(a, qg);
    const int nbx = nbr[e * 4 + (rv.cx > 0.0 ? 3 : 1)], nby = nbr[e * 4 + (rv.cy > 0.0 ? 0 : 2)];
    double px[NFP], py[NFP];
    row_traces<P>(a, qg, k0 + e, nbx, nby, px, py);
    row_rhs<P, MODE>(a, tile + r * S, mom + e * NP * 4, rw + e * 4 * NFP, rv, nbx, nby, px, py);
  }
  __syncthreads();

  // ---- 4. RK4 register update, coalesced over each velocity row -----------------
  if constexpr (NTM != 0) {
    const double *xr = rk_x<MODE>(a) + boff;
    double *accr = a.acc + boff;
    double *outr = a.out + boff;
    if (MODE != 0 && a.pout && E == 1 && 7 * (nthr / NP) * NP <= Qb * S) {
      update_columns<P, MODE, NTM == 1>(a, tile, xr, accr, outr, Qb, q0, tid, nthr,
                                        a.pout + (((size_t)tile_y * a.K + k0) * 7) * NP);
      return;
    }
    double *keep = (MODE != 0 && a.pout) ? tile : nullptr;
    for (int c0 = tid; c0 < nch; c0 += nthr * U)
      update_pass<P, MODE, NTM == 1>(a, tile, xr, accr, outr, c0, Qb, E, Eb, nch, full, tid, nthr,
                                     keep);
    if (keep) {
      // moment partials of the stage output over this velocity tile, for the
      // next stage (its output values replaced L(f) in the LDS tile)
      __syncthreads();
      block_moments_mfma<P, 16>(tile, part, a.wmom + (size_t)q0 * 16, E, Qb, Eb, tid, nthr);
      __syncthreads();
      const int ks = moment_slices(P, E);
      constexpr int NB = (NP + 15) / 16;
      if (tid < E * NP) {
        const int e2 = tid / NP, n2 = tid % NP;
        if (e2 < Eb) {
          const int t = e2 * NB + n2 / 16, col = n2 % 16;
          double sm[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
          for (int sl = 0; sl < ks; ++sl) {
            const double *pp = part + ((size_t)(t * ks + sl) * 7) * 16;
#pragma unroll
            for (int c = 0; c < 7; ++c) sm[c] += pp[c * 16 + col];
          }
          double *po = a.pout + (((size_t)tile_y * a.K + k0 + e2) * 7) * NP + n2;
#pragma unroll
          for (int c = 0; c < 7; ++c) po[c * NP] = sm[c];
        }
      }
    }
  } else if (MODE != 0 && handoff && a.pout) {
    // one-element blocks handing their output's moments to the next stage
    double *po = a.pout + ((size_t)k0 * 7) * NP;
    const bool wall_el = we;
    if constexpr (handoff_order<P>()) {
      if (a.stream_nt) {
        if (wall_el) update_rows_handoff<P, MODE, true, true>(a, tile, boff, Qb, tid, nthr, part, po);
        else update_rows_handoff<P, MODE, true, false>(a, tile, boff, Qb, tid, nthr, part, po);
      } else {
        if (wall_el) update_rows_handoff<P, MODE, false, true>(a, tile, boff, Qb, tid, nthr, part, po);
        else update_rows_handoff<P, MODE, false, false>(a, tile, boff, Qb, tid, nthr, part, po);
      }
    }
  } else if (a.stream_nt) {
    update_rows<P, MODE, true>(a, tile, boff, Qb, E, Eb, nch, full, tid, nthr);
  } else {
    update_rows<P, MODE, false>(a, tile, boff, Qb, E, Eb, nch, full, tid, nthr);
  }
}

// One work-group per (element block, velocity tile); the general kernel.
// FK: 0 velocity-tiled blocks, 1 fused blocks, 2 fused blocks of one element.
template <int P, int MODE, int FK>
// Fused blocks of orders 1-3 with the moment product ask for three resident
// wavefronts per SIMD: the compiler then keeps the product's accumulators in
// ordinary VGPRs (168 at most, no spills) instead of 32 extra accumulation
// registers, which had capped these kernels at two (measured: 256x256 p = 2
// Couette, 16 elements per block, 199 -> 157 us per stage; 128x128 p = 2
// NC 16x16, one element, 448 -> 380 us); so do velocity tiles of order 3
// (64x64 p = 3 NC 24x24, tiles of 320 + 256: 318 -> 285 us; order 1 measured
// slower, 805 -> 874 us).  The handover kernel (FK = 3) has no product and
// measured slower with the request (91 -> 102 us per stage on the 64x64 p = 3
// cavity).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(((FK == 1 || FK == 2) && P <= 3) || (FK == 0 && P == 3) ? 3 : 1)))
void stage_kernel(const StageArgs a) {
  const int blk = strip_block(xcd_block(blockIdx.x, a.nblk), a.nx, a.log2E, a.nblk);
  // Code layouts chosen by measurement: the fused block with the run-time
  // cache policy, the velocity-tiled block with one copy per policy.
  if constexpr (FK == 3)
    stage_block<P, MODE, true, 0, 1, true>(a, blk, blockIdx.y);
  else if constexpr (FK == 2)
    stage_block<P, MODE, true, 0, 1>(a, blk, blockIdx.y);
  else if constexpr (FK == 1)
    stage_block<P, MODE, true, 0>(a, blk, blockIdx.y);
  else if (a.stream_nt)  // (velocity tiles hold one element, but the run-time E measured faster)
    stage_block<P, MODE, false, 1>(a, blk, blockIdx.y);
  else
    stage_block<P, MODE, false, 2>(a, blk, blockIdx.y);
}

// Batched stage over several problems of the same order P: work item i is
// (problem, element block); work-groups stride over the items.  The
// per-problem arguments are read from a descriptor table in the constant
// address space (scalar loads), written before the launch and unchanged
// during it.  Fused blocks only (all velocities of a block per work-group).
typedef __attribute__((address_space(4))) const StageArgs ConstStageArgs;

template <int P, int MODE>
// (two resident wavefronts per SIMD asked for at order 4: its body then fits
// 256 VGPRs with the accumulators, instead of one wavefront; lower orders run
// two either way)
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(P == 4 ? 2 : 1)))
void batch_stage_kernel(const StageArgs *descs, const int2 *items, int nitems) {
#if defined(__HIP_DEVICE_COMPILE__)
  ConstStageArgs *cd = (ConstStageArgs *)descs;
#endif
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int2 it = items[i];
    const int inst = __builtin_amdgcn_readfirstlane(it.x);
    const int blk = __builtin_amdgcn_readfirstlane(it.y);
#if defined(__HIP_DEVICE_COMPILE__)
    const StageArgs a = cd[inst];  // scalar loads from the constant address space
#else
    const StageArgs a = descs[inst];  // host pass: the body is never run on the host
#endif
    stage_block<P, MODE, true, 0>(a, blk, 0);
    __syncthreads();  // LDS is reused by the next item
  }
}

// LDS layout of the pipelined kernel, in doubles: three f tiles (staged,
// computed, updated), two trace buffers (staged, computed), then the moment
// scratch of the block being computed.
struct PipeLayout {
  int tile, trace, part, mom, rw, nbr, total;
};

__host__ __device__ inline PipeLayout pipe_layout(int NP, int NFP, int S, int E, int Q) {
  PipeLayout L;
  L.tile = Q * E * S;
  L.trace = Q * E * (2 * NFP + 1);  // odd row stride: 8-byte accesses without bank conflicts
  const int tasks = E * ((NP + 15) / 16);
  const int pairs = tasks >= 4 ? tasks : 4;
  L.part = 3 * L.tile + 2 * L.trace;
  L.mom = (L.part + pairs * 7 * 16 + 3) / 4 * 4;  // 32-byte aligned (read as double4)
  L.rw = L.mom + E * NP * 4;
  L.nbr = L.rw + E * 4 * NFP;
  L.total = L.nbr + (E * 4 + 1) / 2;
  return L;
}

// Loads a memory thread of the pipelined kernel issues in iteration t - 1
// for iteration t: the f tile and the row's inflow traces of the block staged
// in t (index t of the run) and the RK operands of the block updated in t
// (index t - 2).
template <int P, int MODE, int PF, typename V>
__device__ __forceinline__ void pipe_issue(const StageArgs &a, int t, int first, int nl, int nb,
                                           int tid, double cx, double cy, V (&tl)[PF], V (&x)[PF],
                                           V (&y)[PF], double (&px)[P + 1], double (&py)[P + 1]) {
  using Sh = Shape<P>;
  constexpr int NP = Sh::NP;
  constexpr int CW = Sh::VEC ? 2 : 1;
  constexpr int CPE = NP / CW;
  const int E = a.E, Q = a.Q, rows = Q * E, nch = rows * CPE;
  const uint32_t QNP = (uint32_t)Q * NP;
  const int rq = tid >> a.log2E, re = tid & (E - 1);
  if (t < nb) {
    const int bs = first + t * nl, Ebs = min(E, a.K - bs * E);
    load_tile<CPE, CW, NP, PF>(tl, a.fs + (size_t)bs * E * QNP, tid, kBlock, nch, Q, E, Ebs, QNP);
    if (tid < rows && re < Ebs) {
      const int nbx = neighbour(bs * E + re, cx > 0.0 ? 3 : 1, a);
      const int nby = neighbour(bs * E + re, cy > 0.0 ? 0 : 2, a);
      row_traces32<P>(a, cx, cy, rq, nbx, nby, px, py);
    }
  }
  if (rk_reads_x(MODE) && t >= 2 && t - 2 < nb) {
    const int bu = first + (t - 2) * nl, Ebu = min(E, a.K - bu * E);
    const size_t boff = (size_t)bu * E * QNP;
    const double *xr = rk_x<MODE>(a) + boff;
    const double *yr = rk_y<MODE>(a) + boff;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int c = tid + u * kBlock;
      int q, e, w;
      split_access<CPE>(c, Q, E, q, e, w);
      if (c < nch && e < Ebu) {
        const uint32_t go = (uint32_t)e * QNP + (uint32_t)(q * NP + CW * w);
        x[u] = ld32<V>(xr, go);
        if (rk_reads_y(MODE)) y[u] = ld32<V>(yr, go);
      }
    }
  }
}

// Persistent, wave-specialised form of the fused stage, for blocks whose
// velocity rows fit one per thread and whose f tile fits kStreamDoubles
// doubles per thread.  A work-group of 2 x kBlock threads walks a run of
// element blocks as a three-deep pipeline: in iteration t its four memory
// wavefronts put the f tile and the inflow traces of block t into LDS, apply
// the RK4 update of block t-2 and issue the loads of iteration t+1, so that
// every load has a whole iteration to arrive, while its four compute
// wavefronts reduce the moments of block t-1 on the matrix cores and
// evaluate L(f) of its rows.  HBM traffic and the LDS /
// register work of neighbouring blocks thus overlap inside each work-group.
// Blocks are dealt to the XCDs (work-group w runs on XCD w mod 8) in
// contiguous runs, so the neighbour traces are mostly read from that XCD's
// L2.  The arithmetic per block is that of stage_kernel, in the same order.
template <int P, int MODE>
__global__ __launch_bounds__(2 * kBlock) void pipe_kernel(const StageArgs a) {
  using Sh = Shape<P>;
  constexpr int NP = Sh::NP, NFP = Sh::NFP, S = Sh::S, TS = 2 * NFP + 1;
  constexpr int CW = Sh::VEC ? 2 : 1;
  constexpr int CPE = NP / CW;
  constexpr int PF = kStreamDoubles / CW;  // tile accesses per memory thread
  using V = typename std::conditional<Sh::VEC, double2v, double>::type;
  extern __shared__ double lds[];
  const int E = a.E, log2E = a.log2E, Q = a.Q;
  const PipeLayout L = pipe_layout(NP, NFP, S, E, Q);
  double *part = lds + L.part;
  double *mom = lds + L.mom;
  double *rw = lds + L.rw;
  int *nbr = (int *)(lds + L.nbr);
  const int rows = Q * E, nch = rows * CPE;
  const uint32_t QNP = (uint32_t)Q * NP;

  // block run of this work-group: the blocks are split into contiguous runs,
  // one per XCD that has work-groups, and the work-groups of an XCD take
  // every nl-th block of its run
  const int nx8 = min(8, (int)gridDim.x);
  const int xcd = blockIdx.x & 7, l = blockIdx.x >> 3;
  const int nl = ((int)gridDim.x - xcd + 7) >> 3;  // work-groups on this XCD
  const int per = a.nblk / nx8, rem = a.nblk - per * nx8;
  const int b1 = xcd * per + min(xcd, rem) + per + (xcd < rem ? 1 : 0);
  const int first = xcd * per + min(xcd, rem) + l;
  if (first >= b1) return;
  const int nb = (b1 - first + nl - 1) / nl;  // blocks of this work-group
  const bool memory = threadIdx.x >= kBlock;  // wavefronts 4..7

  // The memory wavefronts' gather addresses depend on the velocity of the
  // thread's row: it is loaded once, since a global load inside the loop would
  // make the gathers wait for every load issued before it (loads complete in
  // order).
  const int tid0 = (int)(threadIdx.x & (kBlock - 1));
  const int rq0 = min(tid0 >> log2E, Q - 1);
  double mcx = 0.0, mcy = 0.0;
  if (memory) {
    mcx = a.vel[rq0];
    mcy = a.vel[Q + rq0];
  }

  // operands in flight from one iteration to the next (memory wavefronts)
  V tl[PF], x[PF], y[PF];
  double px[NFP], py[NFP];
  if (memory) pipe_issue<P, MODE, PF>(a, 0, first, nl, nb, tid0, mcx, mcy, tl, x, y, px, py);

  for (int t = 0; t < nb + 2; ++t) {
    // The thread index is made opaque once per iteration so that the
    // per-access index arithmetic is recomputed rather than held in
    // registers across the loop.
    int tid = (int)(threadIdx.x & (kBlock - 1));
    asm volatile("" : "+v"(tid));
    const int bs = first + t * nl;  // block staged in this iteration
    const int bc = bs - nl;         // block computed
    const int bu = bs - 2 * nl;     // block updated
    const bool do_s = t < nb, do_c = t >= 1 && t <= nb, do_u = t >= 2;
    const int Ebs = min(E, a.K - bs * E), Ebc = min(E, a.K - bc * E), Ebu = min(E, a.K - bu * E);
    double *tile_s = lds + (t % 3) * L.tile;
    double *tile_c = lds + ((t + 2) % 3) * L.tile;
    double *tile_u = lds + ((t + 1) % 3) * L.tile;
    double *trace_s = lds + 3 * L.tile + (t & 1) * L.trace;
    const double *trace_c = lds + 3 * L.tile + ((t + 1) & 1) * L.trace;
    const int rq = tid >> log2E, re = tid & (E - 1);

    // A. compute: moment partials (the memory wavefronts' loads are in flight)
    if (!memory && do_c) {
      if (tid < E * 4) {
        const int e = tid >> 2, fc = tid & 3;
        nbr[tid] = e < Ebc ? neighbour(bc * E + e, fc, a) : -1;
      }
      block_moments_mfma<P, 8>(tile_c, part, a.wmom, E, Q, Ebc, tid, kBlock);
    }
    __syncthreads();
    if (!memory && do_c) block_moments_combine<P>(a, part, mom, rw, nbr, E, Ebc, bc * E, tid);
    __syncthreads();

    // C. memory: the staged tile and traces into LDS, the RK4 update of block
    // bu; compute: L(f) of the rows of block bc
    if (memory) {
      if (do_s) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int c = tid + u * kBlock;
          int q, e, w;
          split_access<CPE>(c, Q, E, q, e, w);
          if (c < nch && e < Ebs) lds_put(tile_s + (q * E + e) * S + CW * w, tl[u]);
        }
        if (tid < rows && re < Ebs) {
          double *tr = trace_s + tid * TS;
#pragma unroll
          for (int m = 0; m < NFP; ++m) {
            tr[m] = px[m];
            tr[NFP + m] = py[m];
          }
        }
      }
      if (do_u) {
        const size_t boff = (size_t)bu * E * QNP;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int c = tid + u * kBlock;
          int q, e, w;
          split_access<CPE>(c, Q, E, q, e, w);
          if (c < nch && e < Ebu) {
            const V kv = lds_get<V>(tile_u + (q * E + e) * S + CW * w);
            const uint32_t go = (uint32_t)e * QNP + (uint32_t)(q * NP + CW * w);
            V o, an;
            rk_update<MODE>(kv, x[u], y[u], a.c_acc, a.c_out, o, an);
            st32<V>(a.out + boff, go, o);
            if (rk_writes_acc(MODE)) st32<V>(a.acc + boff, go, an);
          }
        }
      }
      pipe_issue<P, MODE, PF>(a, t + 1, first, nl, nb, tid, mcx, mcy, tl, x, y, px, py);
    } else if (do_c && tid < rows && re < Ebc) {
      const RowVel rv = row_vel(a, rq);
      const int nbx = nbr[re * 4 + (rv.cx > 0.0 ? 3 : 1)], nby = nbr[re * 4 + (rv.cy > 0.0 ? 0 : 2)];
      double qx[NFP], qy[NFP];
      const double *tr = trace_c + tid * TS;
#pragma unroll
      for (int m = 0; m < NFP; ++m) {
        qx[m] = tr[m];
        qy[m] = tr[NFP + m];
      }
      row_rhs<P, MODE>(a, tile_c + tid * S, mom + re * NP * 4, rw + re * 4 * NFP, rv, nbx, nby, qx, qy);
    }
    __syncthreads();
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
    const double v = f[((size_t)k * Q + q) * NP + n];
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

// Moment rows of a state for the stages that read their input's moments:
// out[(k 7 + c) Np + n] = sum_q W[q][c] f[k][q][n] with W = (1, e_x, e_y, the
// outgoing normal speed at the bottom, right, top, left wall), then zeros for
// the partial slots of further velocity tiles.
__global__ __launch_bounds__(256) void moment_rows_kernel(const double *f, const double *vel, int K, int Np,
                                                          int Q, int ntiles, double *out) {
  const size_t KNP = (size_t)K * Np;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KNP) return;
  const size_t k = i / Np, n = i % Np;
  double s[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int q = 0; q < Q; ++q) {
    const double v = f[(k * Q + q) * Np + n];
    const double cx = vel[q], cy = vel[Q + q];
    s[0] += v;
    s[1] += cx * v;
    s[2] += cy * v;
    s[3] += (cy < 0.0 ? -cy : 0.0) * v;
    s[4] += (cx > 0.0 ? cx : 0.0) * v;
    s[5] += (cy > 0.0 ? cy : 0.0) * v;
    s[6] += (cx < 0.0 ? -cx : 0.0) * v;
  }
  for (int c = 0; c < 7; ++c) out[(k * 7 + c) * Np + n] = s[c];
  for (int t = 1; t < ntiles; ++t)
    for (int c = 0; c < 7; ++c) out[(((size_t)t * K + k) * 7 + c) * Np + n] = 0.0;
}

// max that keeps NaN
__device__ inline double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

__global__ __launch_bounds__(256) void residual_kernel(const double *k, const double *vel, int KNP,
                                                       int Np, int Q, double scale,
                                                       unsigned long long *result) {
  __shared__ double red[256 / 64];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double m = 0.0;
  if (i < KNP) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = 0; q < Q; ++q) {
      const double v = k[((size_t)(i / Np) * Q + q) * Np + i % Np];
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

__global__ void init_equilibrium_kernel(double *f, const double *vel, size_t KNP, int Np, int Q,
                                        double rho0, double ux0, double uy0, double theta) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= KNP) return;
  const double cx = vel[q], cy = vel[Q + q], w = vel[2 * Q + q];
  const double eu = cx * ux0 + cy * uy0, usq = ux0 * ux0 + uy0 * uy0;
  f[((i / Np) * Q + q) * Np + i % Np] =
      w * rho0 * (1.0 + eu / theta + eu * eu / (2.0 * theta * theta) - usq / (2.0 * theta));
}

// f[q][k][n] <-> f[k][q][n] (to_element_major selects the direction).
__global__ void transpose_kernel(const double *src, double *dst, size_t KNP, int Np, int Q,
                                 int to_element_major) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // k * Np + n
  const int q = blockIdx.y;
  if (i >= KNP) return;
  const size_t qmaj = (size_t)q * KNP + i;
  const size_t emaj = ((i / Np) * Q + q) * Np + i % Np;
  if (to_element_major) dst[emaj] = src[qmaj];
  else dst[qmaj] = src[emaj];
}

__global__ void fill_u64_kernel(unsigned long long *p, size_t n, unsigned long long v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void u64_to_f64_kernel(const unsigned long long *src, double *dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = __longlong_as_double((long long)src[0]);
}

template <int P, int MODE, int FK>
hipError_t launch_stage_pmf(const StageArgs &a, size_t lds, int ntiles, hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)stage_kernel<P, MODE, FK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)a.nblk, (unsigned)ntiles);
  hipLaunchKernelGGL((stage_kernel<P, MODE, FK>), grid, dim3(kBlock), lds, st, a);
  return hipGetLastError();
}

template <int P, int MODE>
hipError_t launch_stage_pm(const StageArgs &a, size_t lds, int ntiles, hipStream_t st) {
  if (!a.fused) {
    if (a.E != 1) return hipErrorInvalidValue;  // velocity tiles hold one element
    return launch_stage_pmf<P, MODE, 0>(a, lds, ntiles, st);
  }
  if constexpr (handoff_order<P>()) {
    // one-element blocks that read their input's moments (and, in RK4 stages,
    // write their output's): a kernel without the matrix-core moment product,
    // whose accumulators would cost a resident work-group per compute unit
    if (a.E == 1 && a.pin && (MODE == 0 || a.pout)) return launch_stage_pmf<P, MODE, 3>(a, lds, ntiles, st);
  }
  return a.E == 1 ? launch_stage_pmf<P, MODE, 2>(a, lds, ntiles, st)
                  : launch_stage_pmf<P, MODE, 1>(a, lds, ntiles, st);
}



template <int P, int MODE>
hipError_t launch_stream_pm(const StageArgs &a, size_t lds, int groups, hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)pipe_kernel<P, MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((pipe_kernel<P, MODE>), dim3((unsigned)groups), dim3(2 * kBlock), lds, st, a);
  return hipGetLastError();
}

template <int P>
hipError_t launch_stream_p(const StageArgs &a, size_t lds, int groups, hipStream_t st) {
  switch (a.stage) {
    case 0: return launch_stream_pm<P, 0>(a, lds, groups, st);
    case 1: return launch_stream_pm<P, 1>(a, lds, groups, st);
    case 2: return launch_stream_pm<P, 3>(a, lds, groups, st);
    case 3: return launch_stream_pm<P, 2>(a, lds, groups, st);
    case 4: return launch_stream_pm<P, 4>(a, lds, groups, st);
    default: return hipErrorInvalidValue;
  }
}

template <int P, int MODE>
hipError_t launch_batch_pm(const StageArgs *descs, const int2 *items, int nitems, size_t lds,
                           int groups, hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)batch_stage_kernel<P, MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((batch_stage_kernel<P, MODE>), dim3((unsigned)groups), dim3(kBlock), lds, st,
                     descs, items, nitems);
  return hipGetLastError();
}

template <int P>
hipError_t launch_batch_p(int stage, const StageArgs *descs, const int2 *items, int nitems,
                          size_t lds, int groups, hipStream_t st) {
  switch (stage) {
    case 0: return launch_batch_pm<P, 0>(descs, items, nitems, lds, groups, st);
    case 1: return launch_batch_pm<P, 1>(descs, items, nitems, lds, groups, st);
    case 2: return launch_batch_pm<P, 3>(descs, items, nitems, lds, groups, st);
    case 3: return launch_batch_pm<P, 2>(descs, items, nitems, lds, groups, st);
    case 4: return launch_batch_pm<P, 4>(descs, items, nitems, lds, groups, st);
    default: return hipErrorInvalidValue;
  }
}

template <int P>
hipError_t launch_stage_p(const StageArgs &a, size_t lds, int ntiles, hipStream_t st) {
  switch (a.stage) {
    case 0: return launch_stage_pm<P, 0>(a, lds, ntiles, st);
    case 1: return launch_stage_pm<P, 1>(a, lds, ntiles, st);
    case 2: return launch_stage_pm<P, 3>(a, lds, ntiles, st);
    case 3: return launch_stage_pm<P, 2>(a, lds, ntiles, st);
    case 4: return launch_stage_pm<P, 4>(a, lds, ntiles, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t stage_lds_bytes(int p, int E, int Qt) {
  const int N1 = p + 1, NP = N1 * N1;
  const int S = (NP % 2 == 0) ? NP + 2 : NP;
  return (size_t)lds_layout(NP, N1, S, E, Qt).total * sizeof(double);
}

bool stream_applicable(int p, int E, int Q, int64_t K) {
  const int NP = (p + 1) * (p + 1);
  return p >= 1 && p <= kStreamMaxP && (int64_t)E * Q <= kBlock &&
         (int64_t)E * Q * NP <= (int64_t)kStreamDoubles * kBlock &&
         (int64_t)Q * K * NP * 8 < ((int64_t)1 << 32);
}

size_t stream_lds_bytes(int p, int E, int Q) {
  const int N1 = p + 1, NP = N1 * N1;
  const int S = (NP % 2 == 0) ? NP + 2 : NP;
  return (size_t)pipe_layout(NP, N1, S, E, Q).total * sizeof(double);
}

hipError_t launch_stream(int p, const StageArgs &a, size_t lds, int groups, hipStream_t st) {
  if (!a.fused || !stream_applicable(p, a.E, a.Q, a.K) || groups < 1 || groups > a.nblk)
    return hipErrorInvalidValue;
  switch (p) {
    case 1: return launch_stream_p<1>(a, lds, groups, st);
    case 2: return launch_stream_p<2>(a, lds, groups, st);
    case 3: return launch_stream_p<3>(a, lds, groups, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_stage(int p, int stage, const StageArgs *descs, const int2 *items,
                              int nitems, size_t lds, int groups, hipStream_t st) {
  if (nitems <= 0 || groups <= 0) return hipSuccess;
  switch (p) {
    case 1: return launch_batch_p<1>(stage, descs, items, nitems, lds, groups, st);
    case 2: return launch_batch_p<2>(stage, descs, items, nitems, lds, groups, st);
    case 3: return launch_batch_p<3>(stage, descs, items, nitems, lds, groups, st);
    case 4: return launch_batch_p<4>(stage, descs, items, nitems, lds, groups, st);
    case 5: return launch_batch_p<5>(stage, descs, items, nitems, lds, groups, st);
    case 6: return launch_batch_p<6>(stage, descs, items, nitems, lds, groups, st);
    case 7: return launch_batch_p<7>(stage, descs, items, nitems, lds, groups, st);
    case 8: return launch_batch_p<8>(stage, descs, items, nitems, lds, groups, st);
    default: return hipErrorInvalidValue;
  }
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

hipError_t launch_moment_rows(const double *f, const double *vel, int K, int Np, int Q, int ntiles,
                              double *out, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  hipLaunchKernelGGL(moment_rows_kernel, dim3((unsigned)((KNP + 255) / 256)), dim3(256), 0, st,
                     f, vel, K, Np, Q, ntiles, out);
  return hipGetLastError();
}

hipError_t launch_residual(const double *k, const double *vel, int K, int Np, int Q, double scale,
                           unsigned long long *result, hipStream_t st) {
  const int KNP = K * Np;
  const unsigned nb = (unsigned)((KNP + 255) / 256);
  hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(256), 0, st, k, vel, KNP, Np, Q, scale, result);
  return hipGetLastError();
}

hipError_t launch_init_equilibrium(double *f, const double *vel, int K, int Np, int Q, double rho0,
                                   double ux0, double uy0, double theta, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(init_equilibrium_kernel, grid, dim3(256), 0, st, f, vel, KNP, Np, Q, rho0, ux0,
                     uy0, theta);
  return hipGetLastError();
}

hipError_t launch_transpose(const double *src, double *dst, int K, int Np, int Q,
                            int to_element_major, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, src, dst, KNP, Np, Q,
                     to_element_major);
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
