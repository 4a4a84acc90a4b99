// Q1 cell loops (the fast path of the Jacobian and the smoother operator, Sec. 4.1) for 2D and
// 3D, FP64 and FP32: the marching tiles (bodies in q1_tiles.h), one thread per cell with atomic
// scatter, two work items per cell and LDS bricks (the residual and the diagonal are in
// cell_q1_aux.hip).
//
// The cell work is split into a displacement part (test functions w:
// g(phi~) sigma(du) : e(w)) and a phase-field part (test functions psi), each
// sum-factorized with q1_math.h, which keeps the live register set small.
//
// The block operator B~ (the smoother's operator, applied far more often than
// G~) reads its phase-field coefficient c_phi JxW per Gauss point from a
// per-level array written once per linearization (k_q1_block_coef), so its
// cells load neither U nor form the gradient of u; every B~ shape below does.
#include "q1_tiles.h"

namespace pff {

// Workgroups are dealt to the chip's 8 XCDs round-robin (workgroup b to XCD b mod 8), each
// XCD with its own L2.  xcd_tile maps b to a tile index so that every XCD receives one
// contiguous range of tiles (a bijection of [0, nb) for any nb): tiles that share node
// planes and columns then read them through the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t q = nb / kXcds, r = nb % kXcds;
  const int64_t xcd = b % kXcds, k = b / kXcds;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// one wavefront per tile; tiles ordered x fastest, then y, then z-chunk (ntx x nty tiles of
// TX x TY cells, nzc chunks), launched as a 1D grid of ntx * nty * nzc workgroups: an XCD's range
// holds neighbouring tiles of a chunk layer, which share their edge lines in one L2
// CHEB (block operator only): instead of y, apply the Chebyshev step cf at every owned node.
template <typename T, int MODE, int TX, int TY, bool CHEB = false>
__global__ __launch_bounds__(64) void k_q1_3d(CellParams cp, int zc, int ntx, int nzc, const T* __restrict__ x,
                                              const T* __restrict__ U, const T* __restrict__ phit,
                                              const uint8_t* __restrict__ mask, T* __restrict__ y,
                                              ChebFuse<T> cf = ChebFuse<T>{}) {
  const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t tiles = (int64_t)gridDim.x / nzc;
  const int bx = (int)(t % ntx);
  const int by = (int)((t / ntx) % (tiles / ntx));
  const int bz = (int)(t / tiles);
  q1_tile3<T, MODE, TX, TY, CHEB>(cp, zc, bx, by, bz, x, U, phit, mask, y, cf);
}

// one wavefront per 2D row tile; tiles ordered x fastest (ntx strips per y-chunk), launched as a
// 1D grid: an XCD's range holds neighbouring strips of a chunk row, which share the cache lines at
// their common edge (a strip's 64-node row segments do not start on a line boundary)
template <typename T, int MODE>
__global__ __launch_bounds__(64) void k_q1_2d(CellParams cp, int zc, int ntx, const T* __restrict__ x,
                                              const T* __restrict__ U, const T* __restrict__ phit,
                                              const uint8_t* __restrict__ mask, T* __restrict__ y) {
  const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
  q1_tile2<T, MODE>(cp, zc, (int)(t % ntx), (int)(t / ntx), x, U, phit, mask, y);
}

// One Q1 cell of the block operator B~ with the phase-field coefficients stored per point
// (qcb[q * n_cells + cid]); contributions added atomically on the free DoFs.  part: 0 = all
// rows, 1 = displacement rows, 2 = phase-field rows.
template <int D, typename T>
__device__ __forceinline__ void q1_block_stored(const CellParams& cp, int64_t g0, int64_t cid,
                                                const T* __restrict__ x, const T* __restrict__ phit,
                                                const uint8_t* __restrict__ mask, const T* __restrict__ qcb,
                                                T* __restrict__ y, int part) {
  constexpr int NL = D == 2 ? 4 : 8;
  const int64_t nn = cp.n_nodes, sy = cp.ns[1], sz = cp.ns[2];
  int64_t gi[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) gi[a] = g0 + (a & 1) + ((a >> 1) & 1) * sy + (D == 3 ? (a >> 2) * sz : 0);
  const Consts<T> kc(cp, NL);
  uint8_t mk[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) mk[a] = mask[gi[a]];
  if (part != 2) {
    T du[D][NL], pt[NL], outu[D][NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      pt[a] = phit[gi[a]];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const T v = x[c * nn + gi[a]];
        du[c][a] = (mk[a] & (1 << c)) ? T(0) : v;
      }
    }
    if constexpr (D == 3)
      cell3_u<T>(kc, du, pt, outu);
    else
      cell2_u<T>(kc, du, pt, outu);
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int a = 0; a < NL; ++a)
        if (!(mk[a] & (1 << c))) atomicAdd(&y[c * nn + gi[a]], outu[c][a]);
  }
  if (part == 1) return;
  T dp[NL], cq[NL], outp[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) {
    const T v = x[D * nn + gi[a]];
    dp[a] = (mk[a] & kMaskPhi) ? T(0) : v;
    cq[a] = qcb[a * cp.n_cells + cid];
  }
  if constexpr (D == 3)
    cell3_phi_stored<T>(kc, dp, cq, outp);
  else
    cell2_phi_stored<T>(kc, dp, cq, outp);
#pragma unroll
  for (int a = 0; a < NL; ++a)
    if (!(mk[a] & kMaskPhi)) atomicAdd(&y[D * nn + gi[a]], outp[a]);
}

// ----------------------------------------------------------------------------------- atomic variant
// One thread per cell with the same sum-factorized cell math; contributions are
// added with device atomics into y pre-set to Pi_C x.  No halo recompute, so it
// wins on levels too small to fill the chip with marching tiles.
template <typename T, int MODE>
__global__ __launch_bounds__(128) void k_q1_3d_atomic(CellParams cp, const T* __restrict__ x,
                                                      const T* __restrict__ U, const T* __restrict__ phit,
                                                      const uint8_t* __restrict__ mask, T* __restrict__ y) {
  constexpr bool COUPLE = (MODE == MODE_APPLY);
  // one contiguous range of cells per XCD (neighbouring cells share nodes)
  const int64_t cid = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (cid >= cp.n_cells) return;
  const int cx = (int)(cid % cp.N[0]);
  const int cy = (int)((cid / cp.N[0]) % cp.N[1]);
  const int cz = (int)(cid / ((int64_t)cp.N[0] * cp.N[1]));
  if (cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) return;
  const int64_t nn = cp.n_nodes, sy = cp.ns[1], sz = cp.ns[2];
  const int64_t g0 = (int64_t)cx + (int64_t)cy * sy + (int64_t)cz * sz;
  if constexpr (MODE == MODE_BLOCK) {
    q1_block_stored<3, T>(cp, g0, cid, x, phit, mask, (const T*)cp.qcb, y, 0);
    return;
  }
  int64_t gi[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) gi[a] = g0 + (a & 1) + ((a >> 1) & 1) * sy + (a >> 2) * sz;
  const Consts<T> kc(cp, 8);
  uint8_t mk[8];
  T du[3][8], pt[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    mk[a] = mask[gi[a]];
    pt[a] = phit[gi[a]];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T v = x[c * nn + gi[a]];
      du[c][a] = (mk[a] & (1 << c)) ? T(0) : v;
    }
  }
  {
    T outu[3][8];
    cell3_u<T>(kc, du, pt, outu);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (!(mk[a] & (1 << c))) atomicAdd(&y[c * nn + gi[a]], outu[c][a]);
  }
  T dp[8], uu[3][8], ph[8], outp[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T v = x[3 * nn + gi[a]];
    dp[a] = (mk[a] & kMaskPhi) ? T(0) : v;
#pragma unroll
    for (int c = 0; c < 3; ++c) uu[c][a] = U[c * nn + gi[a]];
    ph[a] = COUPLE ? U[3 * nn + gi[a]] : T(0);
  }
  cell3_phi<T, COUPLE>(kc, du, dp, uu, ph, outp);
#pragma unroll
  for (int a = 0; a < 8; ++a)
    if (!(mk[a] & kMaskPhi)) atomicAdd(&y[3 * nn + gi[a]], outp[a]);
}

template <typename T, int MODE>
__global__ __launch_bounds__(128) void k_q1_2d_atomic(CellParams cp, const T* __restrict__ x,
                                                      const T* __restrict__ U, const T* __restrict__ phit,
                                                      const uint8_t* __restrict__ mask, T* __restrict__ y) {
  constexpr bool COUPLE = (MODE == MODE_APPLY);
  const int64_t cid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cid >= cp.n_cells) return;
  const int cx = (int)(cid % cp.N[0]);
  const int cy = (int)(cid / cp.N[0]);
  if (cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) return;
  const int64_t nn = cp.n_nodes, sy = cp.ns[1];
  const int64_t g0 = (int64_t)cx + (int64_t)cy * sy;
  if constexpr (MODE == MODE_BLOCK) {
    q1_block_stored<2, T>(cp, g0, cid, x, phit, mask, (const T*)cp.qcb, y, 0);
    return;
  }
  int64_t gi[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) gi[a] = g0 + (a & 1) + (a >> 1) * sy;
  const Consts<T> kc(cp, 4);
  uint8_t mk[4];
  T du[2][4], pt[4], outu[2][4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    mk[a] = mask[gi[a]];
    pt[a] = phit[gi[a]];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const T v = x[c * nn + gi[a]];
      du[c][a] = (mk[a] & (1 << c)) ? T(0) : v;
    }
  }
  cell2_u<T>(kc, du, pt, outu);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (!(mk[a] & (1 << c))) atomicAdd(&y[c * nn + gi[a]], outu[c][a]);
  T dp[4], uu[2][4], ph[4], outp[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const T v = x[2 * nn + gi[a]];
    dp[a] = (mk[a] & kMaskPhi) ? T(0) : v;
    uu[0][a] = U[gi[a]];
    uu[1][a] = U[nn + gi[a]];
    ph[a] = COUPLE ? U[2 * nn + gi[a]] : T(0);
  }
  cell2_phi<T, COUPLE>(kc, du, dp, uu, ph, outp);
#pragma unroll
  for (int a = 0; a < 4; ++a)
    if (!(mk[a] & kMaskPhi)) atomicAdd(&y[2 * nn + gi[a]], outp[a]);
}

// ----------------------------------------------------------------------------------- 3D bricks
// One 256-thread workgroup per brick of kBX x kBY x kBZ cells.  The brick's
// (kBX+1)(kBY+1)(kBZ+1) nodes of x, U (Jacobian only), phi~ and the mask are first copied to
// LDS with row-contiguous loads (each node value read from HBM once per
// brick instead of once per adjacent cell), then every thread evaluates one
// cell from LDS and scatters with atomics as the atomic variant does.  The
// FP64 cell needs ~250 VGPRs (two waves per SIMD); two co-resident bricks per
// CU overlap one brick's staging with the other's arithmetic.
constexpr int kBX = 16, kBY = 4, kBZ = 4;
constexpr int kBNX = kBX + 1, kBNY = kBY + 1, kBNZ = kBZ + 1, kBN = kBNX * kBNY * kBNZ;

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_q1_3d_brick(CellParams cp, const T* __restrict__ x,
                                                     const T* __restrict__ U, const T* __restrict__ phit,
                                                     const uint8_t* __restrict__ mask, T* __restrict__ y) {
  constexpr bool COUPLE = (MODE == MODE_APPLY);
  constexpr int NU = COUPLE ? 4 : 1;  // U components the cell reads (none for B~: stored coefficients)
  __shared__ T sx[4][kBN];
  __shared__ T sU[NU][kBN];
  __shared__ T sp[kBN];
  __shared__ uint8_t sm[kBN];
  const int nbx = (cp.N[0] + kBX - 1) / kBX, nby = (cp.N[1] + kBY - 1) / kBY;
  const int bx = (int)(blockIdx.x % nbx), by = (int)((blockIdx.x / nbx) % nby), bz = (int)(blockIdx.x / (nbx * nby));
  const int x0 = bx * kBX, y0 = by * kBY, z0 = bz * kBZ;
  const int64_t nn = cp.n_nodes, sy = cp.ns[1], sz = cp.ns[2];
  for (int t = threadIdx.x; t < kBN; t += blockDim.x) {
    const int ix = t % kBNX, iy = (t / kBNX) % kBNY, iz = t / (kBNX * kBNY);
    const int gx = x0 + ix, gy = y0 + iy, gz = z0 + iz;
    const bool in = gx < cp.nn[0] && gy < cp.nn[1] && gz < cp.nn[2];
    const int64_t g = in ? (int64_t)gx + (int64_t)gy * sy + (int64_t)gz * sz : 0;
    sm[t] = in ? mask[g] : (uint8_t)0xFF;
    sp[t] = in ? phit[g] : T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c) sx[c][t] = in ? x[c * nn + g] : T(0);
    if constexpr (COUPLE) {
#pragma unroll
      for (int c = 0; c < NU; ++c) sU[c][t] = in ? U[c * nn + g] : T(0);
    }
  }
  __syncthreads();
  const int lx = threadIdx.x % kBX, ly = (threadIdx.x / kBX) % kBY, lz = threadIdx.x / (kBX * kBY);
  const int cx = x0 + lx, cy = y0 + ly, cz = z0 + lz;
  if (cx >= cp.N[0] || cy >= cp.N[1] || cz >= cp.N[2] || cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) return;
  const int64_t g0 = (int64_t)cx + (int64_t)cy * sy + (int64_t)cz * sz;
  const int l0 = lx + ly * kBNX + lz * kBNX * kBNY;
  int li[8];
  int64_t gi[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    li[a] = l0 + (a & 1) + ((a >> 1) & 1) * kBNX + (a >> 2) * kBNX * kBNY;
    gi[a] = g0 + (a & 1) + ((a >> 1) & 1) * sy + (a >> 2) * sz;
  }
  const Consts<T> kc(cp, 8);
  uint8_t mk[8];
  T du[3][8];
  {
    T pt[8], outu[3][8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      mk[a] = sm[li[a]];
      pt[a] = sp[li[a]];
#pragma unroll
      for (int c = 0; c < 3; ++c) du[c][a] = (mk[a] & (1 << c)) ? T(0) : sx[c][li[a]];
    }
    cell3_u<T>(kc, du, pt, outu);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (!(mk[a] & (1 << c))) atomicAdd(&y[c * nn + gi[a]], outu[c][a]);
  }
  T dp[8], outp[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) dp[a] = (mk[a] & kMaskPhi) ? T(0) : sx[3][li[a]];
  if constexpr (COUPLE) {
    T uu[3][8], ph[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
#pragma unroll
      for (int c = 0; c < 3; ++c) uu[c][a] = sU[c][li[a]];
      ph[a] = sU[3][li[a]];
    }
    cell3_phi<T, true>(kc, du, dp, uu, ph, outp);
  } else {
    const T* __restrict__ qcb = (const T*)cp.qcb;
    const int64_t cid = (int64_t)cx + (int64_t)cy * cp.N[0] + (int64_t)cz * cp.N[0] * cp.N[1];
    T cq[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) cq[q] = qcb[q * cp.n_cells + cid];
    cell3_phi_stored<T>(kc, dp, cq, outp);
  }
#pragma unroll
  for (int a = 0; a < 8; ++a)
    if (!(mk[a] & kMaskPhi)) atomicAdd(&y[3 * nn + gi[a]], outp[a]);
}

// ----------------------------------------------------------------------------------- split cells
// Two work items per cell: the displacement rows and the phase-field rows are
// evaluated by different wavefronts (each wave is uniform in its part, so
// there is no divergence), halving the serial chain per lane.  For levels
// too small to fill the chip, where a cell's latency is the cost.
template <int D, typename T, int MODE>
__global__ __launch_bounds__(128) void k_q1_split(CellParams cp, const T* __restrict__ x, const T* __restrict__ U,
                                                  const T* __restrict__ phit, const uint8_t* __restrict__ mask,
                                                  T* __restrict__ y) {
  constexpr bool COUPLE = (MODE == MODE_APPLY);
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int part = 1 + (int)((w >> 6) & 1);
  const int64_t cid = (w >> 7) * 64 + (w & 63);
  if (cid >= cp.n_cells) return;
  const int cx = (int)(cid % cp.N[0]);
  const int cy = (int)((cid / cp.N[0]) % cp.N[1]);
  const int cz = D == 3 ? (int)(cid / ((int64_t)cp.N[0] * cp.N[1])) : 0;
  if (cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) return;
  const int64_t g0 = (int64_t)cx + (int64_t)cy * cp.ns[1] + (int64_t)cz * cp.ns[2];
  if constexpr (MODE == MODE_BLOCK)
    q1_block_stored<D, T>(cp, g0, cid, x, phit, mask, (const T*)cp.qcb, y, part);
  else
    q1_cell_atomic<D, T, COUPLE>(cp, g0, x, U, phit, mask, y, part);
}

// ----------------------------------------------------------------------------------- B~ coefficients
// c[q * n_cells + cid] = ((1-kappa) E_s(u) + 2 p div u + G_c/eps) JxW at Gauss point q of cell
// cid, from the level's linearization point U (FP64), stored in FP64 and FP32; 0 in hole cells.
template <int D>
__global__ __launch_bounds__(128) void k_q1_block_coef(CellParams cp, const double* __restrict__ U,
                                                       double* __restrict__ c64, float* __restrict__ c32) {
  constexpr int NL = D == 3 ? 8 : 4;
  const int64_t cid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cid >= cp.n_cells) return;
  const int cx = (int)(cid % cp.N[0]);
  const int cy = (int)((cid / cp.N[0]) % cp.N[1]);
  const int cz = D == 3 ? (int)(cid / ((int64_t)cp.N[0] * cp.N[1])) : 0;
  double cph[NL];
  if (cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) {
#pragma unroll
    for (int q = 0; q < NL; ++q) cph[q] = 0.0;
  } else {
    const int64_t nn = cp.n_nodes;
    const int64_t g0 = (int64_t)cx + (int64_t)cy * cp.ns[1] + (int64_t)cz * cp.ns[2];
    double uu[D][NL], pt[NL], gw[NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      const int64_t gi = g0 + (a & 1) + ((a >> 1) & 1) * cp.ns[1] + (D == 3 ? (a >> 2) * cp.ns[2] : 0);
      pt[a] = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) uu[c][a] = U[c * nn + gi];
    }
    const Consts<double> kc(cp, NL);
    if constexpr (D == 3)
      cell3_diag_coef<double>(kc, uu, pt, gw, cph);
    else
      cell2_diag_coef<double>(kc, uu, pt, gw, cph);
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    c64[q * cp.n_cells + cid] = cph[q];
    c32[q * cp.n_cells + cid] = (float)cph[q];
  }
}

int q1_block_coef_values(int d) { return d == 3 ? 8 : 4; }

pf_status launch_block_coef(const Geom& g, const CellParams& cp, const double* U, double* c64, float* c32,
                            hipStream_t s) {
  if (g.p != 1 || !(g.d == 2 || g.d == 3) || !c64 || !c32) {
    set_error("block coefficients: Q1 levels with coefficient storage only");
    return PF_ERR_UNSUPPORTED;
  }
  if (g.n_cells == 0) return PF_OK;
  const int64_t nb = (g.n_cells + 127) / 128;
  if (g.d == 3)
    k_q1_block_coef<3><<<nb, 128, 0, s>>>(cp, U, c64, c32);
  else
    k_q1_block_coef<2><<<nb, 128, 0, s>>>(cp, U, c64, c32);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

// ----------------------------------------------------------------------------------- dispatch
// Variant per level: 0 = marching 8x8 tiles, 1 = marching 16x4 tiles, 2 = atomic,
// 3 = LDS-staged bricks (3D; 2D maps it to 2), 4 = split cells (two work items per cell),
// 5 = LDS-staged marching slabs of 16x16 cells (cell_q1_slab.hip; 3D, 2D maps it to 0).
// q1_set_tile forces a variant / z-chunk (tuning and tests); -1 restores the heuristic.
static int64_t q1_tiles_xy(const Geom& g, int tile) {
  if (g.d == 2) return q1_tiles2(g.nn[0]);
  const int tx = tile == 1 ? 16 : 8, ty = 64 / tx;
  return (int64_t)((g.nn[0] + tx - 2) / (tx - 1)) * ((g.nn[1] + ty - 2) / (ty - 1));
}

int q1_chunk(const Geom& g, int variant, int requested_zc) {
  if (requested_zc > 0) return requested_zc;
  const int64_t tiles = q1_tiles_xy(g, variant);
  const int nplanes = g.nn[g.d - 1];
  const int cand[] = {32, 16, 8};
  for (int z : cand)
    if (tiles * ((nplanes + z - 1) / z) >= 4096) return z;
  return 8;
}

// Size heuristic (the autotuner overrides it per level): marching tiles only
// where they fill the chip with chunks of >= 8 planes.
int q1_variant(const Geom& g, int mode, int requested) {
  if (!(g.p == 1 && (mode == MODE_APPLY || mode == MODE_BLOCK) && (g.d == 2 || g.d == 3))) return -1;
  if (requested >= 0 && requested < kQ1Variants) {
    if (g.d == 2 && requested == 1) return 0;
    if (g.d == 2 && requested == 3) return 2;
    if (g.d == 2 && requested == 5) return 0;
    return requested;
  }
  const int nplanes = g.nn[g.d - 1];
  return q1_tiles_xy(g, 0) * ((nplanes + 7) / 8) >= 4096 ? 0 : 2;
}

bool q1_tiled_handles(const Geom& g, int mode, int requested) {
  const int v = q1_variant(g, mode, requested);
  return v == 0 || v == 1 || v == 5;
}

template <typename T>
static pf_status launch_q1(const Geom& g, const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                           const uint8_t* mask, T* y, hipStream_t s) {
  if (mode == MODE_BLOCK && !cp.qcb) {
    set_error("Q1 block operator: the level's stored coefficients are missing");
    return PF_ERR_UNSUPPORTED;
  }
  const int variant = q1_variant(g, mode, cp.variant);
  if (variant == 5) return launch_q1_slab<T>(g, cp, mode, x, U, phit, mask, y, nullptr, s);
  if (variant == 4) {
    const int64_t nb = (2 * ((g.n_cells + 63) / 64) * 64 + 127) / 128;
    if (g.d == 3) {
      if (mode == MODE_APPLY)
        k_q1_split<3, T, MODE_APPLY><<<nb, 128, 0, s>>>(cp, x, U, phit, mask, y);
      else
        k_q1_split<3, T, MODE_BLOCK><<<nb, 128, 0, s>>>(cp, x, U, phit, mask, y);
    } else {
      if (mode == MODE_APPLY)
        k_q1_split<2, T, MODE_APPLY><<<nb, 128, 0, s>>>(cp, x, U, phit, mask, y);
      else
        k_q1_split<2, T, MODE_BLOCK><<<nb, 128, 0, s>>>(cp, x, U, phit, mask, y);
    }
    PFF_CHECK_LAUNCH();
    return PF_OK;
  }
  if (variant == 3) {
    const int64_t nb = (int64_t)((g.N[0] + kBX - 1) / kBX) * ((g.N[1] + kBY - 1) / kBY) * ((g.N[2] + kBZ - 1) / kBZ);
    if (mode == MODE_APPLY)
      k_q1_3d_brick<T, MODE_APPLY><<<nb, 256, 0, s>>>(cp, x, U, phit, mask, y);
    else
      k_q1_3d_brick<T, MODE_BLOCK><<<nb, 256, 0, s>>>(cp, x, U, phit, mask, y);
    PFF_CHECK_LAUNCH();
    return PF_OK;
  }
  if (variant == 2) {
    const int64_t nb = (g.n_cells + 127) / 128;
    if (g.d == 3) {
      if (mode == MODE_APPLY)
        k_q1_3d_atomic<T, MODE_APPLY><<<nb, 128, 0, s>>>(cp, x, U, phit, mask, y);
      else
        k_q1_3d_atomic<T, MODE_BLOCK><<<nb, 128, 0, s>>>(cp, x, U, phit, mask, y);
    } else {
      if (mode == MODE_APPLY)
        k_q1_2d_atomic<T, MODE_APPLY><<<nb, 128, 0, s>>>(cp, x, U, phit, mask, y);
      else
        k_q1_2d_atomic<T, MODE_BLOCK><<<nb, 128, 0, s>>>(cp, x, U, phit, mask, y);
    }
    PFF_CHECK_LAUNCH();
    return PF_OK;
  }
  if (g.d == 3) {
    const int tile = variant;
    const int tx = tile == 1 ? 16 : 8;
    const int64_t ntx = (g.nn[0] + tx - 2) / (tx - 1), nty = (g.nn[1] + 64 / tx - 2) / (64 / tx - 1);
    const int zc = q1_chunk(g, tile, cp.zc);
    const int nzc = (g.nn[2] + zc - 1) / zc;
    const int64_t nb = ntx * nty * nzc;
    if (nb > 0x7fffffff) {
      set_error("Q1 marching tiles: too many tiles for one launch");
      return PF_ERR_UNSUPPORTED;
    }
    const unsigned grid = (unsigned)nb;
    if (tile == 1) {
      if (mode == MODE_APPLY)
        k_q1_3d<T, MODE_APPLY, 16, 4><<<grid, 64, 0, s>>>(cp, zc, (int)ntx, nzc, x, U, phit, mask, y);
      else
        k_q1_3d<T, MODE_BLOCK, 16, 4><<<grid, 64, 0, s>>>(cp, zc, (int)ntx, nzc, x, U, phit, mask, y);
    } else {
      if (mode == MODE_APPLY)
        k_q1_3d<T, MODE_APPLY, 8, 8><<<grid, 64, 0, s>>>(cp, zc, (int)ntx, nzc, x, U, phit, mask, y);
      else
        k_q1_3d<T, MODE_BLOCK, 8, 8><<<grid, 64, 0, s>>>(cp, zc, (int)ntx, nzc, x, U, phit, mask, y);
    }
  } else {
    const int64_t ntx = q1_tiles2(g.nn[0]);
    const int zc = q1_chunk(g, 0, cp.zc);
    const unsigned grid = (unsigned)(ntx * ((g.nn[1] + zc - 1) / zc));
    if (mode == MODE_APPLY)
      k_q1_2d<T, MODE_APPLY><<<grid, 64, 0, s>>>(cp, zc, (int)ntx, x, U, phit, mask, y);
    else
      k_q1_2d<T, MODE_BLOCK><<<grid, 64, 0, s>>>(cp, zc, (int)ntx, x, U, phit, mask, y);
  }
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

bool q1_block_cheb_fusable(const Geom& g, const CellParams& cp) {
  if (g.d != 3 || g.p != 1 || cp.split || !cp.qcb) return false;
  const int v = q1_variant(g, MODE_BLOCK, cp.variant);
  return v == 0 || v == 1 || v == 5;
}

template <typename T>
pf_status launch_q1_block_cheb(const Geom& g, const CellParams& cp, const T* d, const T* U, const T* phit,
                               const uint8_t* mask, const ChebFuse<T>& cf, hipStream_t s, bool* handled) {
  *handled = q1_block_cheb_fusable(g, cp);
  if (!*handled || g.n_cells == 0) return PF_OK;
  const int tile = q1_variant(g, MODE_BLOCK, cp.variant);
  if (tile == 5) return launch_q1_slab<T>(g, cp, MODE_BLOCK, d, U, phit, mask, nullptr, &cf, s);
  const int tx = tile == 1 ? 16 : 8;
  const int64_t ntx = (g.nn[0] + tx - 2) / (tx - 1), nty = (g.nn[1] + 64 / tx - 2) / (64 / tx - 1);
  const int zc = q1_chunk(g, tile, cp.zc);
  const int nzc = (g.nn[2] + zc - 1) / zc;
  const int64_t nb = ntx * nty * nzc;
  if (nb > 0x7fffffff) {
    set_error("Q1 marching tiles: too many tiles for one launch");
    return PF_ERR_UNSUPPORTED;
  }
  if (tile == 1)
    k_q1_3d<T, MODE_BLOCK, 16, 4, true><<<(unsigned)nb, 64, 0, s>>>(cp, zc, (int)ntx, nzc, d, U, phit, mask, nullptr, cf);
  else
    k_q1_3d<T, MODE_BLOCK, 8, 8, true><<<(unsigned)nb, 64, 0, s>>>(cp, zc, (int)ntx, nzc, d, U, phit, mask, nullptr, cf);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}
template pf_status launch_q1_block_cheb<double>(const Geom&, const CellParams&, const double*, const double*,
                                                const double*, const uint8_t*, const ChebFuse<double>&, hipStream_t,
                                                bool*);
template pf_status launch_q1_block_cheb<float>(const Geom&, const CellParams&, const float*, const float*, const float*,
                                               const uint8_t*, const ChebFuse<float>&, hipStream_t, bool*);

pf_status launch_cell_q1_d(const Geom& g, const CellParams& cp, int mode, const double* x, const double* U,
                           const double* phit, const uint8_t* mask, double* y, hipStream_t s, bool* handled) {
  if (q1_aux_handles(g, mode)) {
    *handled = true;
    return launch_q1_aux(g, cp, mode, U, phit, y, s);
  }
  *handled = q1_variant(g, mode, cp.variant) >= 0;
  if (!*handled) return PF_OK;
  return launch_q1<double>(g, cp, mode, x, U, phit, mask, y, s);
}
pf_status launch_cell_q1_f(const Geom& g, const CellParams& cp, int mode, const float* x, const float* U,
                           const float* phit, const uint8_t* mask, float* y, hipStream_t s, bool* handled) {
  *handled = q1_variant(g, mode, cp.variant) >= 0;
  if (!*handled) return PF_OK;
  return launch_q1<float>(g, cp, mode, x, U, phit, mask, y, s);
}

}  // namespace pff
