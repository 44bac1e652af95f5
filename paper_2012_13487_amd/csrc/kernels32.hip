// FP32-storage precision path of the RK stage (gfx950).
//
// The state is stored as the deviation g = f - w_q rho_ref in FP32,
// element-major g[k][q][n].  Since w_q rho_ref is constant in space and time,
// the RK update, the volume term (D1 annihilates constants) and the jumps
// between neighbours are the same on g as on f; FP32 rounding is then relative
// to the deviation rather than to f ~ w_q.  Following the method's split of
// work, the node moments rho, rho u (Sec. II.A) and the diffuse-wall densities
// of eq. (8) are reduced in FP64 (on the FP64 matrix cores, from the FP32
// values converted exactly), and the wall exterior states
// rho_w f^eq(1, u_b) - w rho_ref are formed in FP64; the volume term, the
// lifted upwind jumps, the BGK collision with the second-order equilibrium of
// eq. (5) and the RK4 update (classical RK4 in increment form, see rk32) run
// in FP32.
//
// One work-group owns E elements and all Q velocities (the fused form of the
// FP64 kernel): the block's tile is one contiguous run of E Q Np floats,
// streamed with 16-byte accesses.
//
// Reference form (REF): the state is f = f_r + g with an FP64 reference f_r
// (any state, refreshed from time to time by folding g into it) and the FP32
// correction g.  Transport (volume term, upwind jumps and the wall exterior
// state, whose density of eq. (8) is linear in the outgoing values) is linear
// in f, so L(f_r + g) = L(f_r) + T(g) - g / tau + [f^eq(m_r + m_g) - f^eq(m_r)] / tau
// with m the node moments; L(f_r) is computed in FP64 when the reference is
// set and streamed in FP32, and the difference of equilibria is expanded in
// the moment increments with FP64 node factors, so every FP32 quantity is
// rounded relative to the correction or to the current rate, which both
// vanish as a solve approaches its steady state.
#include "kernels32.hpp"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace dgbgk {

namespace {

typedef double double4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBlock32 = 256;

template <int P>
struct Shape32 {
  static constexpr int N1 = P + 1;
  static constexpr int NP = N1 * N1;
  static constexpr int NFP = N1;
  static constexpr int S = NP | 1;  // odd LDS row stride: row-per-thread reads without conflicts
  static constexpr int NB = (NP + 15) / 16;
};

// LDS layout in doubles: float tile, FP64 partial products, FP32 node
// moments (8 per node), FP64 wall densities, neighbour table, and (bf16
// variant) the contraction outputs of one 16-velocity group per wavefront.
struct Lds32 {
  int part, mom, rw, nbr, vol, total;
};

__host__ __device__ inline Lds32 lds32_layout(int NP, int NFP, int S, int E, int Q, bool bf16,
                                               bool ref) {
  Lds32 L;
  const int tile_d = (E * Q * S + 1) / 2;
  const int tasks = E * ((NP + 15) / 16);
  const int pairs = tasks >= 4 ? tasks : 4;
  L.part = (tile_d + 3) / 4 * 4;
  L.mom = L.part + pairs * 7 * 16;      // float [E*NP][8] (reference form [12]) per node
  L.rw = L.mom + E * NP * (ref ? 6 : 4);
  L.nbr = L.rw + E * 4 * NFP;
  L.vol = (L.nbr + (E * 4 + 1) / 2 + 3) / 4 * 4;
  // bf16: per wavefront a [2 NP][16] float block (Dr g and Ds g of 16
  // velocity rows) and the 64 row means of its rows
  L.total = L.vol + (bf16 ? (4 * (2 * NP * 16) + 4 * 64) / 2 : 0);
  return L;
}

__device__ inline int xcd_block32(int b, int nblk) {
  const int per = nblk >> 3, rem = nblk & 7, x = b & 7;
  return x * per + (x < rem ? x : rem) + (b >> 3);
}

constexpr int kStripElems32 = 16;  // elements per strip (measured best)

// The t-th element block in strip order: strips of kStripElems32 elements,
// each swept row by row, so that the work-groups resident on one XCD cover a
// compact patch and find their neighbours' faces in L2.  Applies when the
// blocks tile whole mesh rows (E divides nx); otherwise the identity.
__device__ inline int strip_block32(int t, int nx, int E, int nblk) {
  if (nx % E) return t;
  const int W = kStripElems32 / E > 0 ? kStripElems32 / E : 1;  // blocks per strip
  const int bpr = nx / E, rows = nblk / bpr;
  const int full = bpr - bpr % W;
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

__device__ inline int neighbour32(int k, int face, const Stage32Args &a) {
  const int ex = k % a.nx, ey = k / a.nx;
  switch (face) {
    case 0: return ey > 0 ? k - a.nx : (a.periodic_y ? k + a.nx * (a.ny - 1) : -1);
    case 1: return ex < a.nx - 1 ? k + 1 : (a.periodic_x ? k - (a.nx - 1) : -1);
    case 2: return ey < a.ny - 1 ? k + a.nx : (a.periodic_y ? k - a.nx * (a.ny - 1) : -1);
    default: return ex > 0 ? k - 1 : (a.periodic_x ? k + (a.nx - 1) : -1);
  }
}

// Classical RK4 in increment form: acc holds d = sum_i b_i dt k_i (small, so
// its FP32 rounding is relative to the increment, not to the state), and the
// state is rounded once per step, g_{n+1} = g_n + (d + dt/6 k_4).
//   MODE 1: d = dt/6 k,     out = g_n + dt/2 k      (x = g_n = g_s)
//   MODE 2: d += dt/3 k,    out = g_n + c dt k      (x = g_n, y = d)
//   MODE 4: out = g_n + (d + dt/6 k)                (x = g_n, y = d)
//   MODE 0: out = k
template <int MODE>
__device__ __forceinline__ float rk32(float kv, float x, float y, float ca, float co, float &an) {
  if (MODE == 0) return kv;
  if (MODE == 1) { an = ca * kv; return x + co * kv; }
  if (MODE == 2) { an = y + ca * kv; return x + co * kv; }
  return x + (y + ca * kv);
}

typedef float float4m __attribute__((ext_vector_type(4)));

// Volume term of the wavefront's 64 rows r0 + 64 w + lane on bf16 matrix
// cores.  The rows go in four groups of 16 velocity rows (the N dimension of
// v_mfma_f32_16x16x32_bf16); the M dimension runs over the 2 NP output nodes of
// [Dr; Ds] (MT tiles of 16), the K dimension over the NP input nodes (padded to
// 32).  Each row's mean is subtracted before rounding to bf16 (Dr and Ds
// annihilate constants), so the rounding is relative to the variation of g
// within the element.  Lane layout (established with an in-bounds probe):
// A: lane l holds A[l % 16][8 (l / 16) + t]; B: B[8 (l / 16) + t][l % 16];
// D: register v of lane l is D[4 (l / 16) + v][l % 16].  Results go through a
// per-wavefront LDS block to the lane that owns the row; the LDS accesses of
// one wavefront execute in order, so no barrier is needed.
template <int NP, int MT>
__device__ __forceinline__ void volume_bf16(const float *tile, int S, int r0w, int rows, bool own_valid,
                                            const float (&f)[NP], float ax, float ay,
                                            const bf16x8 (&dA)[MT], float *cm, float *vs,
                                            float (&kk)[NP]) {
  const int lane = threadIdx.x & 63;
  float mean = 0.0f;
  if (own_valid) {
#pragma unroll
    for (int n = 0; n < NP; ++n) mean += f[n];
    mean *= 1.0f / NP;
  }
  cm[lane] = mean;
  const int col = lane & 15, kg = lane >> 4;
#pragma unroll
  for (int gi = 0; gi < 4; ++gi) {
    const int rb = r0w + 16 * gi + col;  // row of this lane's B column
    bf16x8 bop;
    const float cmb = cm[16 * gi + col];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int n = 8 * kg + t;
      const float v = (rb < rows && n < NP) ? tile[rb * S + n] - cmb : 0.0f;
      bop[t] = (__bf16)v;
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      float4m d = {0.0f, 0.0f, 0.0f, 0.0f};
      d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(dA[mt], bop, d, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * mt + 4 * kg + v;
        if (row < 2 * NP) vs[row * 16 + col] = d[v];
      }
    }
    if (kg == gi && own_valid) {
#pragma unroll
      for (int n = 0; n < NP; ++n) kk[n] = -(ax * vs[n * 16 + col] + ay * vs[(NP + n) * 16 + col]);
    }
  }
}

// Loads and stores of the streams touched once per stage, with or without
// non-temporal hints.
template <bool NT, typename V>
__device__ __forceinline__ V ld_once32(const float *p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
  return *reinterpret_cast<const V *>(p);
}
template <bool NT, typename V>
__device__ __forceinline__ void st_once32(float *p, const V &v) {
  if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
  else *reinterpret_cast<V *>(p) = v;
}

// Phase 4 of an FP32 stage: the RK4 update of the block (contiguous floats),
// L(g) in the LDS tile.  With NT, x and the accumulator, read once per stage
// and not again before the next launch, move with non-temporal hints so that
// they do not evict the tiles neighbours still gather from (used when the
// state arrays exceed the last-level cache); the stage output, the next
// stage's input, is always stored normally.
template <int P, int MODE, int CW, bool NT, bool REF>
__device__ __forceinline__ void update32(const Stage32Args &a, const float *tile, size_t boff, int nch,
                                         int tid, int nthr) {
  using Sh = Shape32<P>;
  constexpr int NP = Sh::NP, S = Sh::S;
  // measured: p = 4 (25 nodes) 1188 -> 1150 us, p = 3 prefers 8; the reference
  // form's third stream (L(f_r)) takes registers: 8 at p = 4 (16 takes all 256;
  // 4 measured 1332 against 1319 us), 4 below (p = 3: 79.6 against 92.1 us with 8,
  // three work-groups per CU instead of two)
  constexpr int U = REF ? (P == 4 ? 8 : 4) : (P == 4 ? 16 : 8);
  using V = typename std::conditional<CW == 4, float4v, float>::type;
  const float cacc = a.c_acc, cout = a.c_out;
  const float *xr = (MODE == 1 ? a.fs : a.fn) + boff;
  float *accr = a.acc + boff;
  float *outr = a.out + boff;
  const float *rr = REF ? a.rref + boff : nullptr;
  for (int c0 = tid; c0 < nch; c0 += nthr * U) {
    V x[U], y[U], rv[REF ? U : 1];
    if constexpr (REF) {  // L(f_r), added to the tile's T(g) + collision difference
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * nthr;
        if (c < nch) rv[u] = ld_once32<NT, V>(rr + (size_t)c * CW);
      }
    }
    if (MODE != 0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * nthr;
        if (c < nch) x[u] = ld_once32<NT, V>(xr + (size_t)c * CW);
      }
    }
    if (MODE == 2 || MODE == 4) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * nthr;
        if (c < nch) y[u] = ld_once32<NT, V>(accr + (size_t)c * CW);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * nthr;
      if (c >= nch) continue;
      V o, an;
#pragma unroll
      for (int i = 0; i < CW; ++i) {
        const int j = c * CW + i, r = j / NP, n = j - r * NP;
        float kv = tile[r * S + n];
        if constexpr (REF) {
          if constexpr (CW == 4) kv += rv[u][i];
          else kv += rv[u];
        }
        float xi = 0.0f, yi = 0.0f, ai = 0.0f, oi;
        if constexpr (CW == 4) {
          if (MODE != 0) xi = x[u][i];
          if (MODE == 2 || MODE == 4) yi = y[u][i];
        } else {
          if (MODE != 0) xi = x[u];
          if (MODE == 2 || MODE == 4) yi = y[u];
        }
        oi = rk32<MODE>(kv, xi, yi, cacc, cout, ai);
        if constexpr (CW == 4) {
          o[i] = oi;
          an[i] = ai;
        } else {
          o = oi;
          an = ai;
        }
      }
      *reinterpret_cast<V *>(outr + (size_t)c * CW) = o;
      if (MODE == 1 || MODE == 2) st_once32<NT, V>(accr + (size_t)c * CW, an);
    }
  }
}

// Whether one-element blocks of order P hand their output's moments to the
// next stage: with 16-byte accesses (4 nodes of one velocity row) each
// thread's accesses stay on one column of 4 nodes, and the four wavefronts'
// sums fit the partial-product area.
template <int P>
__host__ __device__ constexpr bool handoff32_order() {
  constexpr int NP = (P + 1) * (P + 1);
  return NP % 4 == 0 && 64 % (NP / 4) == 0 && NP <= 16;
}

static_assert(handoff32_order<1>() == handoff_moments(1) && handoff32_order<2>() == handoff_moments(2) &&
                  handoff32_order<3>() == handoff_moments(3) && handoff32_order<4>() == handoff_moments(4) &&
                  handoff32_order<5>() == handoff_moments(5) && handoff32_order<6>() == handoff_moments(6) &&
                  handoff32_order<7>() == handoff_moments(7) && handoff32_order<8>() == handoff_moments(8),
              "the host's choice of orders that hand over moments matches the kernel's");

// Sum of a double over the lanes of each 16-lane row that are m, 2m, ... apart
// (m = 1, 2, 4, 8): rotations within the row (DPP).
template <int M>
__device__ __forceinline__ double row_rotate_add(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const int rlo = __builtin_amdgcn_update_dpp(0, lo, 0x120 + M, 0xf, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(0, hi, 0x120 + M, 0xf, 0xf, false);
  const long long r = ((long long)rhi << 32) | (unsigned int)rlo;
  return v + __builtin_bit_cast(double, r);
}

// Sum of v over the lanes of the wavefront congruent to this lane modulo G
// (G = 1, 2, 4): rotations within 16-lane rows, then shuffles across rows.
template <int G>
__device__ __forceinline__ double lane_group_sum(double v) {
  static_assert(G == 1 || G == 2 || G == 4, "lane groups of 1, 2 or 4");
  if constexpr (G <= 1) v = row_rotate_add<1>(v);
  if constexpr (G <= 2) v = row_rotate_add<2>(v);
  v = row_rotate_add<4>(v);
  v = row_rotate_add<8>(v);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Phase 4 of a one-element block (the accesses of update32, 16 bytes) that
// also sums the moments of its output over the velocities per node, in FP64,
// for the next stage: rows 0..2 of po (1, e_x, e_y) from each thread's column
// of 4 nodes (reduced across the lanes of a wavefront, then across the
// wavefronts in red, 4 x 7 x NP doubles).  WALL: the element has wall faces;
// its outputs also go to the LDS tile, from which the outgoing normal speed
// times the output is summed for the nodes of each wall face (rows 3..6).
template <int P, int MODE, bool NT, bool REF, bool WALL>
__device__ __forceinline__ void update32_handoff(const Stage32Args &a, float *tile, size_t boff, int nch,
                                                 int tid, int nthr, const int *nbr, double *red,
                                                 double *po) {
  using Sh = Shape32<P>;
  constexpr int N1 = Sh::N1, NP = Sh::NP, S = Sh::S;
  constexpr int CPE = NP / 4;  // 16-byte accesses per velocity row
  constexpr int U = REF ? 2 : 1;  // (measured: 4 / 2 / 1 -> 59.1 / 57.7 / 57.0 us, reference form 78.1 / 74.0 / 75.1)
  const float cacc = a.c_acc, cout = a.c_out;
  const float *xr = (MODE == 1 ? a.fs : a.fn) + boff;
  float *accr = a.acc + boff;
  float *outr = a.out + boff;
  const float *rr = REF ? a.rref + boff : nullptr;
  const int w = tid % CPE;  // nthr is a multiple of CPE: the column never changes
  double sm[3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) sm[c][i] = 0.0;
  for (int c0 = tid; c0 < nch; c0 += nthr * U) {
    float4v x[U], y[U], rv[REF ? U : 1];
    if constexpr (REF) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * nthr;
        if (c < nch) rv[u] = ld_once32<NT, float4v>(rr + (size_t)c * 4);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * nthr;
      if (c < nch) x[u] = ld_once32<NT, float4v>(xr + (size_t)c * 4);
    }
    if (MODE == 2 || MODE == 4) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * nthr;
        if (c < nch) y[u] = ld_once32<NT, float4v>(accr + (size_t)c * 4);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * nthr;
      if (c >= nch) continue;
      const int q = c / CPE;
      float4v o, an;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float kv = tile[q * S + 4 * w + i];
        if constexpr (REF) kv += rv[u][i];
        float ai = 0.0f;
        const float yi = (MODE == 2 || MODE == 4) ? y[u][i] : 0.0f;
        o[i] = rk32<MODE>(kv, x[u][i], yi, cacc, cout, ai);
        an[i] = ai;
        if (WALL) tile[q * S + 4 * w + i] = o[i];  // (the position this thread read)
      }
      *reinterpret_cast<float4v *>(outr + (size_t)c * 4) = o;
      if (MODE == 1 || MODE == 2) st_once32<NT, float4v>(accr + (size_t)c * 4, an);
      const double ex = a.vel[q], ey = a.vel[a.Q + q];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double ov = (double)o[i];
        sm[0][i] += ov;
        sm[1][i] += ex * ov;
        sm[2][i] += ey * ov;
      }
    }
  }
  // lanes with the same column are congruent modulo CPE
#pragma unroll
  for (int cc = 0; cc < 3; ++cc)
#pragma unroll
    for (int i = 0; i < 4; ++i) sm[cc][i] = lane_group_sum<CPE>(sm[cc][i]);
  const int wave = tid >> 6, lane = tid & 63;
  if (lane < CPE) {
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[(wave * 7 + cc) * NP + 4 * lane + i] = sm[cc][i];
  }
  __syncthreads();
  if constexpr (WALL) {
    // face node m of this thread, velocity rows tid / N1, + nthr / N1, ...
    const int m = tid % N1;
    const int nd[4] = {m, m * N1 + P, P * N1 + m, m * N1};  // bottom, right, top, left
    double ws[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = tid / N1; q < a.Q; q += nthr / N1) {
      const double ex = a.vel[q], ey = a.vel[a.Q + q];
      const double wt[4] = {ey < 0.0 ? -ey : 0.0, ex > 0.0 ? ex : 0.0, ey > 0.0 ? ey : 0.0,
                            ex < 0.0 ? -ex : 0.0};
#pragma unroll
      for (int fc = 0; fc < 4; ++fc)
        if (nbr[fc] < 0) ws[fc] += wt[fc] * (double)tile[q * S + nd[fc]];
    }
#pragma unroll
    for (int fc = 0; fc < 4; ++fc) ws[fc] = lane_group_sum<N1>(ws[fc]);
    if (lane < N1) {
#pragma unroll
      for (int fc = 0; fc < 4; ++fc) red[(wave * 7 + 3 + fc) * NP + nd[fc]] = ws[fc];
    }
    __syncthreads();
  }
  constexpr int W = WALL ? 7 : 3;  // (rows 3..6 hold sums at the wall faces' nodes only)
  if (tid < W * NP) {
    const int cc = tid / NP, n = tid - cc * NP;
    double v = 0.0;
    for (int wv = 0; wv < (nthr >> 6); ++wv) v += red[(wv * 7 + cc) * NP + n];
    po[cc * NP + n] = v;
  }
}

// MODE: 0 writes L(f_s); 1 first RK4 stage; 2 second and third; 4 fourth.
// CW: floats per global access (4 when Q Np is a multiple of 4, else 1).
// BF: the volume term's contractions Dr g, Ds g on bf16 matrix cores.
// EFIX: elements per work-group fixed at compile time (0: a.E at run time);
// the one-element form drops the block's index arithmetic.
// HO: a one-element block that reads its input's moments (a.pin) and writes
// its output's (a.pout), compiled without the matrix-core moment product.
template <int P, int MODE, int CW, bool BF, int EFIX = 0, bool REF = false, bool HO = false>
__device__ __forceinline__ void stage32_block(const Stage32Args &a, int blk) {
  using Sh = Shape32<P>;
  constexpr int N1 = Sh::N1, NP = Sh::NP, NFP = Sh::NFP, S = Sh::S, NB = Sh::NB;
  constexpr int U = P == 4 ? 16 : 8;  // global accesses in flight per thread (as update32)
  using V = typename std::conditional<CW == 4, float4v, float>::type;
  extern __shared__ double lds[];
  const int E = EFIX > 0 ? EFIX : a.E, Q = a.Q;
  const Lds32 L = lds32_layout(NP, NFP, S, E, Q, BF, REF);
  constexpr int MS = REF ? 12 : 8;  // floats per node in the moment table
  float *tile = (float *)lds;
  double *part = lds + L.part;
  float *mom = (float *)(lds + L.mom);
  double *rw = lds + L.rw;
  int *nbr = (int *)(lds + L.nbr);

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int k0 = blk * E;
  const int Eb = min(E, a.K - k0);
  const int QNP = Q * NP;
  const int nflt = Eb * QNP;  // floats of this block (contiguous)
  const int nch = nflt / CW;
  const size_t boff = (size_t)k0 * QNP;

  // ---- 0. neighbours (-1: wall) ------------------------------------------------
  if (tid < E * 4) {
    const int e = tid >> 2, fc = tid & 3;
    nbr[tid] = e < Eb ? neighbour32(k0 + e, fc, a) : -1;
  }

  // one-element blocks of orders 1 and 3 read the moments of g_s handed over
  // by the stage that wrote it (rows 3..6, the wall sums, only where the
  // element has a wall face); the loads are issued before the tile's
  static_assert(!HO || (CW == 4 && handoff32_order<P>()), "moment handover: orders 1 and 3, 16-byte rows");
  constexpr bool pin1 = HO;  // (the host sets a.pin, a.pout and one element per block)
  const bool we = HO && a.wall_mask != 0 &&
                  (neighbour32(k0, 0, a) < 0 || neighbour32(k0, 1, a) < 0 ||
                   neighbour32(k0, 2, a) < 0 || neighbour32(k0, 3, a) < 0);
  double pv[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (pin1 && tid < NP) {
    const double *pp = a.pin + (size_t)k0 * 7 * NP + tid;
#pragma unroll
    for (int c = 0; c < 3; ++c) pv[c] = pp[c * NP];
    if (we) {
#pragma unroll
      for (int c = 3; c < 7; ++c) pv[c] = pp[c * NP];
    }
  }

  // reference form: the reference moments of this thread's node are loaded
  // before the tile (they arrive first; loads complete in order) and used in
  // phase 2, instead of a dependent load after the moment product
  const bool mref_pre = REF && E * NP <= nthr;
  double pre_rr = 0.0, pre_ux = 0.0, pre_uy = 0.0;
  if constexpr (REF) {
    if (mref_pre && tid < Eb * NP) {
      const size_t KN = (size_t)a.K * NP, node = (size_t)k0 * NP + tid;
      pre_rr = a.mref[node];
      pre_ux = a.mref[KN + node];
      pre_uy = a.mref[2 * KN + node];
    }
  }

  // ---- 1. the block's tile into LDS: row r = e Q + q, node n at r S + n --------
  for (int c0 = tid; c0 < nch; c0 += nthr * U) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * nthr;
      if (c < nch) v[u] = *reinterpret_cast<const V *>(a.fs + boff + (size_t)c * CW);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * nthr;
      if (c >= nch) continue;
#pragma unroll
      for (int i = 0; i < CW; ++i) {
        const int j = c * CW + i, r = j / NP, n = j - r * NP;
        float x;
        if constexpr (CW == 4) x = v[u][i];
        else x = v[u];
        tile[r * S + n] = x;
      }
    }
  }
  __syncthreads();

  // ---- 2. FP64 moments and wall densities (matrix cores) -----------------------
  {
    const int wave = tid >> 6, lane = tid & 63;
    const int tasks = E * NB;
    const int ks = tasks >= 4 ? 1 : 4 / tasks;
    const int qper = ((Q + ks - 1) / ks + 3) / 4 * 4;
    for (int pr = wave; !pin1 && pr < tasks * ks; pr += nthr >> 6) {
      const int t = pr / ks, sl = pr % ks;
      const int e = t / NB, nb = t % NB;
      const int node = nb * 16 + (lane & 15);
      const int qa = sl * qper, qe = min(Q, qa + qper);
      double4v acc = {0.0, 0.0, 0.0, 0.0}, acc1 = acc, acc2 = acc, acc3 = acc;
      if (e < Eb) {
        constexpr int KB = 8;
        for (int qb = qa; qb < qe; qb += 4 * KB) {
          double av[KB], bv[KB];
#pragma unroll
          for (int t2 = 0; t2 < KB; ++t2) {
            const int q = qb + 4 * t2 + (lane >> 4);
            const bool in = q < qe;
            av[t2] = in ? a.wmom[(size_t)q * 16 + (lane & 15)] : 0.0;
            bv[t2] = (in && node < NP) ? (double)tile[(e * Q + q) * S + node] : 0.0;
          }
#pragma unroll
          for (int t2 = 0; t2 < KB; t2 += 4) {
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t2], bv[t2], acc, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t2 + 1], bv[t2 + 1], acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t2 + 2], bv[t2 + 2], acc2, 0, 0, 0);
            acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t2 + 3], bv[t2 + 3], acc3, 0, 0, 0);
          }
        }
      }
      acc += acc1 + acc2 + acc3;
      // register v of a lane holds C[4 v + lane / 16][lane % 16]
      if (node < NP) {
        double *pp = part + ((size_t)pr * 7) * 16;
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const int row = 4 * v + (lane >> 4);
          if (row < 7) pp[row * 16 + (lane & 15)] = acc[v];
        }
      }
    }
    __syncthreads();
    for (int idx = tid; idx < E * NP; idx += nthr) {
      const int e2 = idx / NP, n2 = idx % NP;
      if (e2 < Eb) {
        const int t = e2 * NB + n2 / 16, col = n2 % 16;
        double sm[7];
#pragma unroll
        for (int c = 0; c < 7; ++c) sm[c] = 0.0;
        if (pin1) {
#pragma unroll
          for (int c = 0; c < 7; ++c) sm[c] = pv[c];  // (one element: idx == tid < NP)
        } else {
          for (int sl = 0; sl < ks; ++sl) {
            const double *pp = part + ((size_t)(t * ks + sl) * 7) * 16;
#pragma unroll
            for (int c = 0; c < 7; ++c) sm[c] += pp[c * 16 + col];
          }
        }
        float *m = mom + (e2 * NP + n2) * MS;
        if constexpr (REF) {
          // moments of g are the increments over the reference's (FP64)
          const size_t KN = (size_t)a.K * NP, node = (size_t)(k0 + e2) * NP + n2;
          const double rr = mref_pre ? pre_rr : a.mref[node];
          const double urx = mref_pre ? pre_ux : a.mref[KN + node];
          const double ury = mref_pre ? pre_uy : a.mref[2 * KN + node];
          const double drho = sm[0], rho = rr + drho;
          const double ux = (rr * urx + sm[1]) / rho, uy = (rr * ury + sm[2]) / rho;
          const double dux = ux - urx, duy = uy - ury;
          const double h1 = a.half_theta_inv, th_inv = 2.0 * h1, h2 = h1 * th_inv;
          // rho |u|^2 - rho_r |u_r|^2 = drho |u|^2 + rho_r (u + u_r).(u - u_r)
          const double dq = drho * (ux * ux + uy * uy) + rr * ((ux + urx) * dux + (uy + ury) * duy);
          m[0] = (float)(drho - dq * h1);
          m[1] = (float)(sm[1] * th_inv);
          m[2] = (float)(sm[2] * th_inv);
          m[3] = (float)urx;
          m[4] = (float)ury;
          m[5] = (float)dux;
          m[6] = (float)duy;
          m[7] = (float)(drho * h2);
          m[8] = (float)(rho * h2);
        } else {
#pragma unroll
          for (int c = 0; c < 7; ++c) sm[c] += a.mconst[c];
          const double rho = sm[0], ux = sm[1] / rho, uy = sm[2] / rho;
          m[0] = (float)ux;
          m[1] = (float)uy;
          m[2] = (float)rho;
          m[3] = (float)(rho - a.rho_ref);
          m[4] = (float)((ux * ux + uy * uy) * a.half_theta_inv);
        }
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
  __syncthreads();

  // ---- 3. per velocity row: L(f) in FP32 ------------------------------------------
  const int rows = E * Q;
  constexpr int MT = (2 * NP + 15) / 16;  // bf16: M tiles of [Dr; Ds]
  bf16x8 dA[BF ? MT : 1];
  if constexpr (BF) {
    const int lane = tid & 63;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      dA[mt] = *reinterpret_cast<const bf16x8 *>(a.dmat + (size_t)(16 * mt + (lane & 15)) * 32 +
                                                 8 * (lane >> 4));
  }
  for (int r0 = 0; r0 < rows; r0 += nthr) {
    const int r = r0 + tid;
    const int e = r / Q, q = r - e * Q;
    const bool valid = r < rows && e < Eb;
    float f[NP];
    float kk[NP];
    if (valid) {
      const float *row = tile + r * S;
#pragma unroll
      for (int c = 0; c < NP; ++c) f[c] = row[c];
    }
    const int qv = valid ? q : 0;
    const float cx = (float)a.vel[qv], cy = (float)a.vel[Q + qv], wq = (float)a.vel[2 * Q + qv];
    const float ax = cx * a.rx, ay = cy * a.sy;
    if constexpr (BF) {
      // all lanes take part in the matrix-core products
      const int wave = tid >> 6;
      float *vs = (float *)(lds + L.vol) + wave * (2 * NP * 16);
      float *cm = (float *)(lds + L.vol) + 4 * (2 * NP * 16) + wave * 64;
      volume_bf16<NP, MT>(tile, S, r0 + 64 * wave, rows, valid, f, ax, ay, dA, cm, vs, kk);
    }
    if (!valid) continue;
    const int fxc = cx > 0.0f ? 3 : 1, fyc = cy > 0.0f ? 0 : 2;  // inflow faces
    const int nbx = nbr[e * 4 + fxc], nby = nbr[e * 4 + fyc];
    // exterior traces of the two inflow faces
    float px[NFP], py[NFP];
    {
      const bool gx = cx != 0.0f && nbx >= 0, gy = cy != 0.0f && nby >= 0;
      const float *sx = a.fs + ((size_t)(nbx >= 0 ? nbx : 0) * Q + q) * NP + (cx > 0.0f ? P : 0);
      const float *sy = a.fs + ((size_t)(nby >= 0 ? nby : 0) * Q + q) * NP + (cy > 0.0f ? N1 * P : 0);
#pragma unroll
      for (int m = 0; m < NFP; ++m) {
        px[m] = gx ? sx[N1 * m] : 0.0f;
        py[m] = gy ? sy[m] : 0.0f;
      }
    }
    if constexpr (!BF) {
#pragma unroll
      for (int j = 0; j < N1; ++j)
#pragma unroll
        for (int i = 0; i < N1; ++i) {
          float dr = 0.0f, ds = 0.0f;
#pragma unroll
          for (int m = 0; m < N1; ++m) {
            dr += a.D1[i * N1 + m] * f[m + N1 * j];
            ds += a.D1[j * N1 + m] * f[i + N1 * m];
          }
          kk[i + N1 * j] = -(ax * dr + ay * ds);
        }
    }
    // wall exterior state in deviation form, rho_w f^eq_q(1, u_b) - w_q rho_ref
    // (FP64); in the reference form rho_w(g) f^eq_q(1, u_b), the wall density
    // being that of the correction alone
    const double wrr = REF ? 0.0 : a.vel[2 * Q + q] * a.rho_ref;
    if (cx != 0.0f) {
      const float wx = a.fsx * (-fabsf(cx));
      const double gb = a.feqb[fxc * Q + q];
      const double *rwx = rw + (e * 4 + fxc) * NFP;
#pragma unroll
      for (int jj = 0; jj < N1; ++jj) {
        const float own = cx > 0.0f ? f[N1 * jj] : f[N1 * jj + P];
        const float ext = nbx >= 0 ? px[jj] : (float)(rwx[jj] * gb - wrr);
        const float J = wx * (own - ext);
#pragma unroll
        for (int ii = 0; ii < N1; ++ii) kk[ii + N1 * jj] += (cx > 0.0f ? a.lift_lo[ii] : a.lift_hi[ii]) * J;
      }
    }
    if (cy != 0.0f) {
      const float wy = a.fsy * (-fabsf(cy));
      const double gb = a.feqb[fyc * Q + q];
      const double *rwy = rw + (e * 4 + fyc) * NFP;
#pragma unroll
      for (int ii = 0; ii < N1; ++ii) {
        const float own = cy > 0.0f ? f[ii] : f[ii + N1 * P];
        const float ext = nby >= 0 ? py[ii] : (float)(rwy[ii] * gb - wrr);
        const float J = wy * (own - ext);
#pragma unroll
        for (int jj = 0; jj < N1; ++jj) kk[ii + N1 * jj] += (cy > 0.0f ? a.lift_lo[jj] : a.lift_hi[jj]) * J;
      }
    }
    const float *mm = mom + e * NP * MS;
    if constexpr (REF) {
      // collision difference: f^eq(m_r + m_g) - f^eq(m_r) - g, with
      // f^eq / w = rho + e.j/theta + [rho (e.u)^2 / theta - rho |u|^2] / (2 theta):
      // a = e.u_r, b = e.(u - u_r); rho (e.u)^2 - rho_r a^2 = drho a^2 + rho b (2a + b)
#pragma unroll
      for (int nn = 0; nn < NP; ++nn) {
        const float *m = mm + MS * nn;
        const float av = cx * m[3] + cy * m[4], bv = cx * m[5] + cy * m[6];
        const float dev =
            wq * (m[0] + cx * m[1] + cy * m[2] + m[7] * av * av + m[8] * bv * (2.0f * av + bv));
        kk[nn] += (dev - f[nn]) * a.inv_tau;
      }
    } else {
      // collision: f^eq - f = w [(rho - rho_ref) + rho (e.u/theta + (e.u)^2/(2 theta^2)
      //                          - |u|^2/(2 theta))] - g
#pragma unroll
      for (int nn = 0; nn < NP; ++nn) {
        const float4v m4 = *reinterpret_cast<const float4v *>(mm + 8 * nn);
        const float usq = mm[8 * nn + 4];
        const float eu = cx * m4[0] + cy * m4[1];
        const float dev = wq * (m4[3] + m4[2] * (eu * (a.theta_inv + eu * a.half_theta2_inv) - usq));
        kk[nn] += (dev - f[nn]) * a.inv_tau;
      }
    }
    float *roww = tile + r * S;
#pragma unroll
    for (int c = 0; c < NP; ++c) roww[c] = kk[c];
  }
  __syncthreads();

  // ---- 4. RK4 update, coalesced over the contiguous block -----------------------
  if constexpr (HO && MODE != 0) {
    {
      // one-element blocks handing their output's moments to the next stage
      double *po = a.pout + (size_t)k0 * 7 * NP;
      if (a.stream_nt) {
        if (we) update32_handoff<P, MODE, true, REF, true>(a, tile, boff, nch, tid, nthr, nbr, part, po);
        else update32_handoff<P, MODE, true, REF, false>(a, tile, boff, nch, tid, nthr, nbr, part, po);
      } else {
        if (we) update32_handoff<P, MODE, false, REF, true>(a, tile, boff, nch, tid, nthr, nbr, part, po);
        else update32_handoff<P, MODE, false, REF, false>(a, tile, boff, nch, tid, nthr, nbr, part, po);
      }
      return;
    }
  }
  if (a.stream_nt)
    update32<P, MODE, CW, true, REF>(a, tile, boff, nch, tid, nthr);
  else
    update32<P, MODE, CW, false, REF>(a, tile, boff, nch, tid, nthr);
}

template <int P, int MODE, int CW, bool BF, int EFIX, bool REF, bool HO = false>
// Orders up to 3 (except the handover and bf16 forms) ask for four resident
// wavefronts per SIMD: the moment product's accumulators then live in ordinary
// VGPRs (128 at most, no spills) instead of 32 extra accumulation registers
// that had held these kernels at three (measured, reference form: 256x256
// p = 2 Couette 65.9 -> 60.2 us per stage, 128x128 p = 2 NC 16x16 194.7 ->
// 177.0 us).
__global__ __launch_bounds__(kBlock32) __attribute__((amdgpu_waves_per_eu((HO || BF) ? 1 : P <= 3 ? 4 : 1)))
void stage32_kernel(const Stage32Args a) {
  stage32_block<P, MODE, CW, BF, EFIX, REF, HO>(
      a, strip_block32(xcd_block32(blockIdx.x, a.nblk), a.nx, EFIX > 0 ? EFIX : a.E, a.nblk));
}

// Batched FP32 stage over problems of the same order P and access width CW:
// work item i is (problem, element block); the per-problem arguments come from
// a descriptor table in the constant address space (see batch_stage_kernel).
typedef __attribute__((address_space(4))) const Stage32Args ConstStage32Args;

template <int P, int MODE, int CW, bool BF, bool REF, bool HO>
__global__ __launch_bounds__(kBlock32) __attribute__((amdgpu_waves_per_eu((HO || BF) ? 1 : P <= 3 ? 4 : 1)))
void batch_stage32_kernel(const Stage32Args *descs,
                                                                  const int2 *items, int nitems) {
#if defined(__HIP_DEVICE_COMPILE__)
  ConstStage32Args *cd = (ConstStage32Args *)descs;
#endif
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int2 it = items[i];
    const int inst = __builtin_amdgcn_readfirstlane(it.x);
    const int blk = __builtin_amdgcn_readfirstlane(it.y);
#if defined(__HIP_DEVICE_COMPILE__)
    const Stage32Args a = cd[inst];  // scalar loads from the constant address space
#else
    const Stage32Args a = descs[inst];  // host pass: the body is never run on the host
#endif
    stage32_block<P, MODE, CW, BF, HO ? 1 : 0, REF, HO>(a, blk);
    __syncthreads();  // LDS is reused by the next item
  }
}

__global__ void to_dev32_kernel(const double *src, float *dst, const double *vel, size_t KNP, int Np,
                                int Q, double offset) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // k * Np + n
  const int q = blockIdx.y;
  if (i >= KNP) return;
  const double w = vel[2 * Q + q];
  dst[((i / Np) * Q + q) * Np + i % Np] = (float)(src[(size_t)q * KNP + i] - offset * w);
}

__global__ void from_dev32_kernel(const float *src, double *dst, const double *vel, size_t KNP,
                                  int Np, int Q, double offset) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= KNP) return;
  const double w = vel[2 * Q + q];
  dst[(size_t)q * KNP + i] = (double)src[((i / Np) * Q + q) * Np + i % Np] + offset * w;
}

__global__ void init_equilibrium32_kernel(float *g, const double *vel, size_t KNP, int Np, int Q,
                                          double rho0, double ux0, double uy0, double theta,
                                          double rho_ref) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= KNP) return;
  const double cx = vel[q], cy = vel[Q + q], w = vel[2 * Q + q];
  const double eu = cx * ux0 + cy * uy0, usq = ux0 * ux0 + uy0 * uy0;
  const double feq = w * rho0 * (1.0 + eu / theta + eu * eu / (2.0 * theta * theta) - usq / (2.0 * theta));
  g[((i / Np) * Q + q) * Np + i % Np] = (float)(feq - w * rho_ref);
}

__global__ __launch_bounds__(256) void moments32_kernel(const float *g, const double *vel, size_t KNP,
                                                        int Np, int Q, double rho_ref, double *rho,
                                                        double *ux, double *uy) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KNP) return;
  const size_t k = i / Np, n = i % Np;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int q = 0; q < Q; ++q) {
    const double cx = vel[q], cy = vel[Q + q], w = vel[2 * Q + q];
    const double v = (double)g[(k * Q + q) * Np + n] + w * rho_ref;
    s0 += v;
    s1 += cx * v;
    s2 += cy * v;
  }
  if (rho) rho[i] = s0;
  if (ux) ux[i] = s1 / s0;
  if (uy) uy[i] = s2 / s0;
}

// Reference form: f_r += g, g = 0 (both element-major).
__global__ __launch_bounds__(256) void ref_fold_kernel(double *fref, float *g, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    fref[i] += (double)g[i];
    g[i] = 0.0f;
  }
}

__global__ __launch_bounds__(256) void f64_to_f32_kernel(const double *src, float *dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = (float)src[i];
}

__global__ __launch_bounds__(256) void ref_sum_kernel(const double *fref, const float *g, double *dst,
                                                      size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = fref[i] + (double)g[i];
}

// host order [q][k][n] <-> element-major [k][q][n]
__global__ void from_ref_kernel(const double *fref, const float *g, double *dst, size_t KNP, int Np,
                                int Q) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // k * Np + n
  const int q = blockIdx.y;
  if (i >= KNP) return;
  const size_t d = ((i / Np) * Q + q) * Np + i % Np;
  dst[(size_t)q * KNP + i] = fref[d] + (double)g[d];
}

__global__ void to_ref_kernel(const double *src, const double *fref, float *g, size_t KNP, int Np,
                              int Q) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (i >= KNP) return;
  const size_t d = ((i / Np) * Q + q) * Np + i % Np;
  g[d] = (float)(src[(size_t)q * KNP + i] - fref[d]);
}

// out[(k 7 + c) Np + n] = sum_q W[q][c] g[k][q][n] in FP64, W = (1, e_x,
// e_y, the outgoing normal speed at the bottom, right, top, left wall).
__global__ __launch_bounds__(256) void moment_rows32_kernel(const float *g, const double *vel, int K,
                                                            int Np, int Q, double *out) {
  const size_t KNP = (size_t)K * Np;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KNP) return;
  const size_t k = i / Np, n = i % Np;
  double s[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int q = 0; q < Q; ++q) {
    const double v = (double)g[(k * Q + q) * Np + n];
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
}

__device__ inline double nan_max32(double a, double b) { return (b > a || b != b) ? b : a; }

__global__ __launch_bounds__(256) void residual32_kernel(const float *k, const double *vel, size_t KNP,
                                                         int Np, int Q, double scale,
                                                         unsigned long long *result) {
  __shared__ double red[4];
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double m = 0.0;
  if (i < KNP) {
    const size_t kk = i / Np, n = i % Np;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = 0; q < Q; ++q) {
      const double v = (double)k[(kk * Q + q) * Np + n];
      s0 += v;
      s1 += vel[q] * v;
      s2 += vel[Q + q] * v;
    }
    m = nan_max32(nan_max32(fabs(s0), fabs(s1)), fabs(s2)) * scale;
  }
  for (int off = 32; off > 0; off >>= 1) m = nan_max32(m, __shfl_xor(m, off));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = nan_max32(b, red[w]);
    atomicMax(result, (unsigned long long)__double_as_longlong(fabs(b)));
  }
}

template <int P, int MODE, int CW, bool BF, bool REF, bool HO>
hipError_t launch_batch32_pmcb(const Stage32Args *descs, const int2 *items, int nitems, size_t lds,
                               int groups, hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)batch_stage32_kernel<P, MODE, CW, BF, REF, HO>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((batch_stage32_kernel<P, MODE, CW, BF, REF, HO>), dim3((unsigned)groups),
                     dim3(kBlock32), lds, st, descs, items, nitems);
  return hipGetLastError();
}

template <int P, int CW, bool BF, bool REF, bool HO>
hipError_t launch_batch32_pcb(int stage, const Stage32Args *descs, const int2 *items, int nitems,
                              size_t lds, int groups, hipStream_t st) {
  switch (stage) {
    case 0: return launch_batch32_pmcb<P, 0, CW, BF, REF, HO>(descs, items, nitems, lds, groups, st);
    case 1: return launch_batch32_pmcb<P, 1, CW, BF, REF, HO>(descs, items, nitems, lds, groups, st);
    case 2:
    case 3: return launch_batch32_pmcb<P, 2, CW, BF, REF, HO>(descs, items, nitems, lds, groups, st);
    case 4: return launch_batch32_pmcb<P, 4, CW, BF, REF, HO>(descs, items, nitems, lds, groups, st);
    default: return hipErrorInvalidValue;
  }
}

// ho: a class of one-element members that hand their moments between stages.
template <int P, bool BF, bool REF>
hipError_t launch_batch32_pb(int stage, int cw, int ho, const Stage32Args *descs, const int2 *items,
                             int nitems, size_t lds, int groups, hipStream_t st) {
  if (ho) {
    if constexpr (handoff32_order<P>())
      if (cw == 4) return launch_batch32_pcb<P, 4, BF, REF, true>(stage, descs, items, nitems, lds, groups, st);
    return hipErrorInvalidValue;
  }
  if (cw == 4) return launch_batch32_pcb<P, 4, BF, REF, false>(stage, descs, items, nitems, lds, groups, st);
  return launch_batch32_pcb<P, 1, BF, REF, false>(stage, descs, items, nitems, lds, groups, st);
}

// The reference form and the bf16 contractions are built for p <= 4.
constexpr int kMaxRefP = 4;

template <bool BF, bool REF>
hipError_t launch_batch32_b(int p, int stage, int cw, int ho, const Stage32Args *descs, const int2 *items,
                            int nitems, size_t lds, int groups, hipStream_t st) {
  switch (p) {
    case 1: return launch_batch32_pb<1, BF, REF>(stage, cw, ho, descs, items, nitems, lds, groups, st);
    case 2: return launch_batch32_pb<2, BF, REF>(stage, cw, ho, descs, items, nitems, lds, groups, st);
    case 3: return launch_batch32_pb<3, BF, REF>(stage, cw, ho, descs, items, nitems, lds, groups, st);
    case 4: return launch_batch32_pb<4, BF, REF>(stage, cw, ho, descs, items, nitems, lds, groups, st);
    default: break;
  }
  if constexpr (!BF && !REF) {
    switch (p) {
      case 5: return launch_batch32_pb<5, false, false>(stage, cw, ho, descs, items, nitems, lds, groups, st);
      case 6: return launch_batch32_pb<6, false, false>(stage, cw, ho, descs, items, nitems, lds, groups, st);
      case 7: return launch_batch32_pb<7, false, false>(stage, cw, ho, descs, items, nitems, lds, groups, st);
      case 8: return launch_batch32_pb<8, false, false>(stage, cw, ho, descs, items, nitems, lds, groups, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <int P, int MODE, int CW, bool BF, int EFIX, bool REF, bool HO = false>
hipError_t launch32_pmcbe(const Stage32Args &a, size_t lds, hipStream_t st) {
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)stage32_kernel<P, MODE, CW, BF, EFIX, REF, HO>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((stage32_kernel<P, MODE, CW, BF, EFIX, REF, HO>), dim3((unsigned)a.nblk),
                     dim3(kBlock32), lds, st, a);
  return hipGetLastError();
}

template <int P, int MODE, int CW, bool BF, bool REF>
hipError_t launch32_pmcb(const Stage32Args &a, size_t lds, hipStream_t st) {
  if constexpr (CW == 4 && handoff32_order<P>()) {
    // one-element blocks that read their input's moments (and, in RK4 stages,
    // write their output's): a kernel without the matrix-core moment product
    if (a.E == 1 && a.pin && (MODE == 0 || a.pout))
      return launch32_pmcbe<P, MODE, CW, BF, 1, REF, true>(a, lds, st);
  }
  if constexpr (P <= 4)
    if (a.E == 1) return launch32_pmcbe<P, MODE, CW, BF, 1, REF>(a, lds, st);
  return launch32_pmcbe<P, MODE, CW, BF, 0, REF>(a, lds, st);
}

template <int P, int MODE, bool BF, bool REF>
hipError_t launch32_pmb(const Stage32Args &a, size_t lds, hipStream_t st) {
  if ((a.Q * (P + 1) * (P + 1)) % 4 == 0) return launch32_pmcb<P, MODE, 4, BF, REF>(a, lds, st);
  return launch32_pmcb<P, MODE, 1, BF, REF>(a, lds, st);
}

template <int P, bool BF, bool REF>
hipError_t launch32_pb(const Stage32Args &a, size_t lds, hipStream_t st) {
  switch (a.stage) {
    case 0: return launch32_pmb<P, 0, BF, REF>(a, lds, st);
    case 1: return launch32_pmb<P, 1, BF, REF>(a, lds, st);
    case 2:
    case 3: return launch32_pmb<P, 2, BF, REF>(a, lds, st);
    case 4: return launch32_pmb<P, 4, BF, REF>(a, lds, st);
    default: return hipErrorInvalidValue;
  }
}

template <bool BF, bool REF>
hipError_t launch32_b(int p, const Stage32Args &a, size_t lds, hipStream_t st) {
  switch (p) {
    case 1: return launch32_pb<1, BF, REF>(a, lds, st);
    case 2: return launch32_pb<2, BF, REF>(a, lds, st);
    case 3: return launch32_pb<3, BF, REF>(a, lds, st);
    case 4: return launch32_pb<4, BF, REF>(a, lds, st);
    default: break;
  }
  if constexpr (!BF && !REF) {
    switch (p) {
      case 5: return launch32_pb<5, false, false>(a, lds, st);
      case 6: return launch32_pb<6, false, false>(a, lds, st);
      case 7: return launch32_pb<7, false, false>(a, lds, st);
      case 8: return launch32_pb<8, false, false>(a, lds, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <typename K, typename... A>
hipError_t launch_stream_kernel(K kern, size_t n, hipStream_t st, A... args) {
  const size_t groups = std::min<size_t>((n + 255) / 256, 8192);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3((unsigned)groups), dim3(256), 0, st, args..., n);
  return hipGetLastError();
}

}  // namespace

size_t stage32_lds_bytes(int p, int E, int Q, bool bf16, bool ref) {
  const int N1 = p + 1, NP = N1 * N1;
  return (size_t)lds32_layout(NP, N1, NP | 1, E, Q, bf16, ref).total * sizeof(double);
}

bool bf16_contraction_available(int p) { return p >= 1 && p <= 4; }

bool ref_form_available(int p, int contract) {
  (void)contract;
  return p >= 1 && p <= kMaxRefP;
}

hipError_t launch_batch_stage32(int p, int stage, int cw, int contract, int ref, int ho,
                                const Stage32Args *descs, const int2 *items, int nitems, size_t lds,
                                int groups, hipStream_t st) {
  if (nitems <= 0 || groups <= 0) return hipSuccess;
  if (contract && ref) return launch_batch32_b<true, true>(p, stage, cw, ho, descs, items, nitems, lds, groups, st);
  if (contract) return launch_batch32_b<true, false>(p, stage, cw, ho, descs, items, nitems, lds, groups, st);
  if (ref) return launch_batch32_b<false, true>(p, stage, cw, ho, descs, items, nitems, lds, groups, st);
  return launch_batch32_b<false, false>(p, stage, cw, ho, descs, items, nitems, lds, groups, st);
}

hipError_t launch_stage32(int p, const Stage32Args &a, size_t lds, int contract, int ref,
                          hipStream_t st) {
  if (contract && !a.dmat) return hipErrorInvalidValue;
  if (ref && (!a.rref || !a.mref)) return hipErrorInvalidValue;
  if (contract && ref) return launch32_b<true, true>(p, a, lds, st);
  if (contract) return launch32_b<true, false>(p, a, lds, st);
  if (ref) return launch32_b<false, true>(p, a, lds, st);
  return launch32_b<false, false>(p, a, lds, st);
}

hipError_t launch_ref_fold(double *fref, float *g, size_t n, hipStream_t st) {
  return launch_stream_kernel(ref_fold_kernel, n, st, fref, g);
}

hipError_t launch_f64_to_f32(const double *src, float *dst, size_t n, hipStream_t st) {
  return launch_stream_kernel(f64_to_f32_kernel, n, st, src, dst);
}

hipError_t launch_ref_sum(const double *fref, const float *g, double *dst, size_t n, hipStream_t st) {
  return launch_stream_kernel(ref_sum_kernel, n, st, fref, g, dst);
}

hipError_t launch_from_ref(const double *fref, const float *g, double *dst, int K, int Np, int Q,
                           hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(from_ref_kernel, grid, dim3(256), 0, st, fref, g, dst, KNP, Np, Q);
  return hipGetLastError();
}

hipError_t launch_to_ref(const double *src, const double *fref, float *g, int K, int Np, int Q,
                         hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(to_ref_kernel, grid, dim3(256), 0, st, src, fref, g, KNP, Np, Q);
  return hipGetLastError();
}

hipError_t launch_to_dev32(const double *src, float *dst, const double *vel, int K, int Np, int Q,
                           double offset, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(to_dev32_kernel, grid, dim3(256), 0, st, src, dst, vel, KNP, Np, Q, offset);
  return hipGetLastError();
}

hipError_t launch_from_dev32(const float *src, double *dst, const double *vel, int K, int Np, int Q,
                             double offset, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(from_dev32_kernel, grid, dim3(256), 0, st, src, dst, vel, KNP, Np, Q, offset);
  return hipGetLastError();
}

hipError_t launch_init_equilibrium32(float *g, const double *vel, int K, int Np, int Q, double rho0,
                                     double ux0, double uy0, double theta, double rho_ref,
                                     hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  dim3 grid((unsigned)((KNP + 255) / 256), (unsigned)Q);
  hipLaunchKernelGGL(init_equilibrium32_kernel, grid, dim3(256), 0, st, g, vel, KNP, Np, Q, rho0,
                     ux0, uy0, theta, rho_ref);
  return hipGetLastError();
}

hipError_t launch_moment_rows32(const float *g, const double *vel, int K, int Np, int Q, double *out,
                                hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  hipLaunchKernelGGL(moment_rows32_kernel, dim3((unsigned)((KNP + 255) / 256)), dim3(256), 0, st, g,
                     vel, K, Np, Q, out);
  return hipGetLastError();
}

hipError_t launch_moments32(const float *g, const double *vel, int K, int Np, int Q, double rho_ref,
                            double *rho, double *ux, double *uy, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  hipLaunchKernelGGL(moments32_kernel, dim3((unsigned)((KNP + 255) / 256)), dim3(256), 0, st, g,
                     vel, KNP, Np, Q, rho_ref, rho, ux, uy);
  return hipGetLastError();
}

hipError_t launch_residual32(const float *k, const double *vel, int K, int Np, int Q, double scale,
                             unsigned long long *result, hipStream_t st) {
  const size_t KNP = (size_t)K * Np;
  hipLaunchKernelGGL(residual32_kernel, dim3((unsigned)((KNP + 255) / 256)), dim3(256), 0, st, k,
                     vel, KNP, Np, Q, scale, result);
  return hipGetLastError();
}

}  // namespace dgbgk
