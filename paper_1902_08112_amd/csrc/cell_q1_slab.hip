// LDS-staged marching slabs for the 3D Q1 cell loop (the tensor-product apply of Sec. 4.1):
// the Jacobian G~ and the smoother's block operator B~, FP64 and FP32.
//
// One 256-thread workgroup (four wavefronts) per tile of 16 x 16 cells, one cell per lane,
// marching along z through a chunk of node planes.  The node data of the tile's 17 x 17 node
// plane (x and, for G~, U in every component, phi~, the constraint mask) go through a ring of
// three planes in LDS: while the lanes evaluate the cells of layer k from planes k and k+1,
// the plane k+2 streams in with direct global-to-LDS loads (global_load_lds: no registers held
// for the prefetch), one row of 17 nodes per 34 (FP64) or 17 (FP32) lanes, coalesced.  The
// cell math reads each field's eight corners from LDS right where it needs them, so the
// corner values are not held across the displacement and phase-field parts.
//
// The 2^3 corner contributions of a cell are combined without atomics, as in the one-wave
// marching tiles: along x with a one-lane shuffle inside each 16-lane row, along y with a
// 16-lane shuffle inside a wavefront and, across the three wavefront boundaries of the tile,
// through a small double-buffered LDS exchange, and along z with a register carry.  Tiles
// overlap by one cell in x and y (and chunks by one cell layer in z); a lane whose node has a
// neighbouring cell outside the tile owns nothing.  Every node is written once with a plain
// store, identity rows included; the result is deterministic.  One barrier per cell layer.
#include "q1_tiles.h"

namespace pff {

namespace {

constexpr int kSX = 16, kSY = 16;                 // cells of a tile (one per lane)
constexpr int kSNX = kSX + 1, kSNY = kSY + 1;     // nodes of the tile's plane
constexpr int kSPlane = kSNX * kSNY;              // 289
constexpr int kSThreads = kSX * kSY;              // 256
constexpr int kSWaves = kSThreads / 64;           // 4
constexpr int kSMaskPad = 292;                    // mask bytes per plane, dword-padded
constexpr int kSPlanePad = 320;                   // values per LDS plane: 289 padded to whole wavefronts

template <int MODE>
struct SlabFields {
  // x (4 components), then for G~ U (4 components), then phi~
  static constexpr int NF = MODE == MODE_APPLY ? 9 : 5;
  static constexpr int U0 = 4;
  static constexpr int PT = MODE == MODE_APPLY ? 8 : 4;
};

constexpr int kXcdsS = 8;
__device__ __forceinline__ int64_t xcd_tile_s(int64_t b, int64_t nb) {
  const int64_t q = nb / kXcdsS, r = nb % kXcdsS;
  const int64_t xcd = b % kXcdsS, k = b / kXcdsS;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

typedef __attribute__((address_space(3))) void lds_void;

// Streaming of one node plane of one field into LDS rows of 17 values with global_load_lds, a
// dword per lane: the plane's dword e (row jj = e / ROW) comes from the lattice node
// (gx0 + ii, gy0 + jj) of the plane and lands at LDS dword e.  The LDS plane is padded to whole
// wavefronts (kSPlanePad values), so every lane of a streaming wavefront loads: a lane past the
// plane fills padding, and a lane whose node lies outside the lattice reads the plane's node
// (0, 0) into a slot that only cells outside the mesh ever read (they contribute nothing).  The
// per-lane byte offsets within a plane are the same for every field and every plane, so they are
// computed once; the per-field, per-plane base is uniform.
template <typename T>
struct PlaneStream {
  static constexpr int W = (int)(sizeof(T) / 4);         // dwords per value
  static constexpr int ROW = kSNX * W;                   // dwords per row
  static constexpr int TOT = kSNY * ROW;                 // dwords per plane
  static constexpr int TOTW = (TOT + 63) / 64 * 64;      // streamed dwords (whole wavefronts)
  static constexpr int R = (TOTW + kSThreads - 1) / kSThreads;
  static_assert(TOTW <= kSPlanePad * W, "padded LDS plane");
  uint32_t off[R];                                       // byte offset within the plane
  __device__ __forceinline__ void init(int gx0, int gy0, const CellParams& cp, int tid) {
    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = r * kSThreads + wave * 64 + lane;
      const int jj = e / ROW, col = e - jj * ROW;
      const int ii = col / W;
      const int gx = gx0 + ii, gy = gy0 + jj;
      const bool ok = e < TOT && gx >= 0 && gx < cp.nn[0] && gy >= 0 && gy < cp.nn[1];
      off[r] = ok ? (uint32_t)(((int64_t)gx + (int64_t)gy * cp.ns[1]) * (int64_t)sizeof(T) + 4 * (col - ii * W)) : 0u;
    }
  }
  // plane: the field's array at node plane kz (uniform); wave: the wavefront index (uniform)
  __device__ __forceinline__ void fetch(const T* __restrict__ plane, T* dst, int wave) const {
    const char* base = reinterpret_cast<const char*>(plane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e0 = r * kSThreads + wave * 64;
      uint32_t o = off[r];
      // an opaque copy per call: keeps the compiler from hoisting 64-bit addresses out of the
      // layer loop (it would hold, or spill, one pair per load); uniform base + 32-bit offset
      __asm__ __volatile__("" : "+v"(o));
      if (e0 < TOTW)
        __builtin_amdgcn_global_load_lds(base + o, (lds_void*)(reinterpret_cast<char*>(dst) + 4 * e0), 4, 0, 0);
    }
  }
};

// the eight corner values of one field for the lane's cell: node (i, j) of planes lo and hi
template <typename T>
__device__ __forceinline__ void corners(const T* lo, const T* hi, int ln, T f[8]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int o = ln + (a & 1) + (a >> 1) * kSNX;
    f[a] = lo[o];
    f[a + 4] = hi[o];
  }
}

// x- and (in-wave) y-combine of one component's corner contributions; X1[az] keeps the
// contributions of the cell's upper y-row (az = 0, 1) for the cross-wave exchange
template <typename T>
__device__ __forceinline__ void combine_xy(const T out[8], bool first_row, T Y[2], T X1[2]) {
#pragma unroll
  for (int az = 0; az < 2; ++az) {
    const T x0 = out[4 * az] + __shfl_up(out[1 + 4 * az], 1, 16);
    const T x1 = out[2 + 4 * az] + __shfl_up(out[3 + 4 * az], 1, 16);
    const T up = __shfl_up(x1, 16, 64);
    Y[az] = x0 + (first_row ? T(0) : up);
    X1[az] = x1;
  }
}

// Gradient tables of a field restricted to the Gauss layer qz = h (the Q1 interpolant's
// derivative along j does not depend on the j-coordinate): g0[qy] = d/dx at (qy, h), g1[qx] =
// d/dy at (qx, h), g2[qx + 2 qy] = d/dz (the same for both layers).  Lerps along z first.
template <typename T>
__device__ __forceinline__ void grad3_layer(const T f[8], const T ih[3], int h, T g0[2], T g1[2], T g2[4]) {
  const T xz = h ? T(q1::XI1) : T(q1::XI0);
  const T x0 = T(q1::XI0), x1 = T(q1::XI1);
  {
    T e[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) e[r] = (f[2 * r + 1] - f[2 * r]) * ih[0];  // r = ay + 2 az
    const T a0 = e[0] + xz * (e[2] - e[0]), a1 = e[1] + xz * (e[3] - e[1]);
    g0[0] = a0 + x0 * (a1 - a0);
    g0[1] = a0 + x1 * (a1 - a0);
  }
  {
    T e[4];
#pragma unroll
    for (int az = 0; az < 2; ++az)
#pragma unroll
      for (int ax = 0; ax < 2; ++ax) e[ax + 2 * az] = (f[ax + 2 + 4 * az] - f[ax + 4 * az]) * ih[1];
    const T a0 = e[0] + xz * (e[2] - e[0]), a1 = e[1] + xz * (e[3] - e[1]);
    g1[0] = a0 + x0 * (a1 - a0);
    g1[1] = a0 + x1 * (a1 - a0);
  }
  {
    T e[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) e[r] = (f[r + 4] - f[r]) * ih[2];  // r = ax + 2 ay
    const T t0 = e[0] + x0 * (e[1] - e[0]), t1 = e[0] + x1 * (e[1] - e[0]);
    const T t2 = e[2] + x0 * (e[3] - e[2]), t3 = e[2] + x1 * (e[3] - e[2]);
    g2[0] = t0 + x0 * (t2 - t0);
    g2[1] = t1 + x0 * (t3 - t1);
    g2[2] = t0 + x1 * (t2 - t0);
    g2[3] = t1 + x1 * (t3 - t1);
  }
}

// values at the four Gauss points of layer qz = h: v[qx + 2 qy]
template <typename T>
__device__ __forceinline__ void val3_layer(const T f[8], int h, T v[4]) {
  const T xz = h ? T(q1::XI1) : T(q1::XI0);
  const T x0 = T(q1::XI0), x1 = T(q1::XI1);
  T z[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) z[r] = f[r] + xz * (f[r + 4] - f[r]);
  const T a0 = z[0] + x0 * (z[1] - z[0]), a1 = z[0] + x1 * (z[1] - z[0]);
  const T b0 = z[2] + x0 * (z[3] - z[2]), b1 = z[2] + x1 * (z[3] - z[2]);
  v[0] = a0 + x0 * (b0 - a0);
  v[1] = a1 + x0 * (b1 - a1);
  v[2] = a0 + x1 * (b0 - a0);
  v[3] = a1 + x1 * (b1 - a1);
}

// All rows of G~ for one cell (FP64), the Gauss points one z-layer at a time, the corners of u, du
// and phi re-read from LDS for each layer, so that the gradient tables of u and of du are never
// both whole in registers (the whole-cell form spills at two waves per SIMD).  Each layer's tables
// of du serve both the displacement rows (their stress tables accumulate over the two layers
// before one backward contraction, as in cell3_u of q1_cell.h) and the coupled phase-field rows
// (cell3_phi), so du is interpolated once per cell.
//   phase-field rows: f(q) = ((1-kappa) E_s(u) + 2 p div u + G_c/eps) dphi
//                            + phi ((1-kappa) sigma(u):e(du) + 2 p div du),
//   out[a] = sum_q f(q) JxW N_a(q) + G_c eps grad dphi . grad N_a JxW
template <typename T, int NF>
__device__ __forceinline__ void g_rows_layers(const Consts<T>& k, const T (*plo)[kSPlanePad], const T (*phi_)[kSPlanePad],
                                              int ln, const uint8_t mk[8], int u0, int ptf, const T dp[8],
                                              T outu[3][8], T outp[8]) {
  T P[3][3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[c][j][r] = T(0);
  T fv[8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __asm__ __volatile__("" ::: "memory");
    T gd0[3][2], gd1[3][2], gd2[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T f[8];
      corners<T>(&plo[c][0], &phi_[c][0], ln, f);
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (mk[a] & (1 << c)) f[a] = T(0);
      grad3_layer<T>(f, k.ih, h, gd0[c], gd1[c], gd2[c]);
    }
    T pq[4];
    {
      T f[8];
      corners<T>(&plo[ptf][0], &phi_[ptf][0], ln, f);
      val3_layer<T>(f, h, pq);
    }
    // displacement rows: g(phi~) sigma(du) at the layer's points into the stress tables
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int qx = qq & 1, qy = qq >> 1;
      const int r0 = qy + 2 * h, r1 = qx + 2 * h, r2 = qq;
      const T g00 = gd0[0][qy], g01 = gd1[0][qx], g02 = gd2[0][qq];
      const T g10 = gd0[1][qy], g11 = gd1[1][qx], g12 = gd2[1][qq];
      const T g20 = gd0[2][qy], g21 = gd1[2][qx], g22 = gd2[2][qq];
      const T gw = ((T(1) - k.kap) * pq[qq] * pq[qq] + k.kap) * k.jxw;
      const T lt = k.lam * (g00 + g11 + g22);
      const T tm = T(2) * k.mu;
      const T s00 = gw * (tm * g00 + lt), s11 = gw * (tm * g11 + lt), s22 = gw * (tm * g22 + lt);
      const T s01 = gw * k.mu * (g01 + g10), s02 = gw * k.mu * (g02 + g20), s12 = gw * k.mu * (g12 + g21);
      P[0][0][r0] += s00;
      P[0][1][r1] += s01;
      P[0][2][r2] += s02;
      P[1][0][r0] += s01;
      P[1][1][r1] += s11;
      P[1][2][r2] += s12;
      P[2][0][r0] += s02;
      P[2][1][r1] += s12;
      P[2][2][r2] += s22;
    }
    __asm__ __volatile__("" ::: "memory");
    T gu0[3][2], gu1[3][2], gu2[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T f[8];
      corners<T>(&plo[u0 + c][0], &phi_[u0 + c][0], ln, f);
      grad3_layer<T>(f, k.ih, h, gu0[c], gu1[c], gu2[c]);
    }
    T pv[4], dv[4];
    {
      T f[8];
      corners<T>(&plo[u0 + 3][0], &phi_[u0 + 3][0], ln, f);
      val3_layer<T>(f, h, pv);
    }
    val3_layer<T>(dp, h, dv);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int qx = qq & 1, qy = qq >> 1;
      const T e00 = gu0[0][qy], e11 = gu1[1][qx], e22 = gu2[2][qq];
      const T e01 = T(0.5) * (gu1[0][qx] + gu0[1][qy]);
      const T e02 = T(0.5) * (gu2[0][qq] + gu0[2][qy]);
      const T e12 = T(0.5) * (gu2[1][qq] + gu1[2][qx]);
      const T tru = e00 + e11 + e22;
      const T ee = e00 * e00 + e11 * e11 + e22 * e22 + T(2) * (e01 * e01 + e02 * e02 + e12 * e12);
      const T Es = T(0.5) * k.lam * tru * tru + k.mu * ee;
      const T cphi = (T(1) - k.kap) * Es + T(2) * k.pres * tru + k.gce;
      const T d00 = gd0[0][qy], d11 = gd1[1][qx], d22 = gd2[2][qq];
      const T d01 = T(0.5) * (gd1[0][qx] + gd0[1][qy]);
      const T d02 = T(0.5) * (gd2[0][qq] + gd0[2][qy]);
      const T d12 = T(0.5) * (gd2[1][qq] + gd1[2][qx]);
      const T trd = d00 + d11 + d22;
      const T eed = e00 * d00 + e11 * d11 + e22 * d22 + T(2) * (e01 * d01 + e02 * d02 + e12 * d12);
      const T sde = T(2) * k.mu * eed + k.lam * tru * trd;
      fv[qq + 4 * h] = (cphi * dv[qq] + pv[qq] * ((T(1) - k.kap) * sde + T(2) * k.pres * trd)) * k.jxw;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int a = 0; a < 8; ++a) outu[c][a] = T(0);
    q1::grad3T(P[c], k.ih, outu[c]);
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) outp[a] = T(0);
  q1::val3T(fv, outp);
  T Gp[3][4];
  q1::grad3(dp, k.ih, Gp);
  const T s = T(2) * k.gcx * k.jxw;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) Gp[j][r] *= s;
  q1::grad3T(Gp, k.ih, outp);
}

}  // namespace

// Occupancy: the FP64 Jacobian and the FP64 fused step keep 256 registers at 2 waves per SIMD
// (at 3 they spill heavily); the FP32 kernels and the plain FP64 B~ fit 168 registers with at
// most 40 B of spill and run at 3 waves (FP32 G~ 10% and FP64 B~ 3% faster on 256^3).
template <typename T, int MODE, bool CHEB>
__global__ __launch_bounds__(kSThreads)
__attribute__((amdgpu_waves_per_eu((sizeof(T) == 8 && (MODE == MODE_APPLY || CHEB)) ? 2 : 3))) void k_q1_3d_slab(
    CellParams cp, int zc, int ntx, int nzc, const T* __restrict__ x, const T* __restrict__ U,
    const T* __restrict__ phit, const uint8_t* __restrict__ mask, T* __restrict__ y, ChebFuse<T> cf) {
  static_assert(!CHEB || MODE == MODE_BLOCK, "the fused Chebyshev step follows the block operator");
  using F = SlabFields<MODE>;
  constexpr bool COUPLE = (MODE == MODE_APPLY);
  __shared__ T sv[3][F::NF][kSPlanePad];
  __shared__ uint8_t sm[3][kSMaskPad];
  __shared__ T sx[2][kSWaves - 1][kSX][8];  // cross-wave y exchange (double-buffered by layer parity)

  // the fused step's coefficients, read once (device memory: captured launches follow new bounds)
  T cc[4] = {T(0), T(0), T(0), T(0)};
  if constexpr (CHEB) {
#pragma unroll
    for (int k = 0; k < 4; ++k) cc[k] = (T)cf.dc[k];
  }
  // tiles x-fastest, then y, then z-chunk: an XCD's range holds neighbouring slabs of a chunk
  // layer, which share the cache lines of their common edge rows and columns in one L2
  const int64_t t = xcd_tile_s(blockIdx.x, gridDim.x);
  const int64_t tiles = (int64_t)gridDim.x / nzc;
  const int bx = (int)(t % ntx);
  const int by = (int)((t / ntx) % (tiles / ntx));
  const int bz = (int)(t / tiles);
  const int tid = threadIdx.x;
  const int i = tid % kSX, j = tid / kSX;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool first_row = (j & 3) == 0, last_row = (j & 3) == 3;
  const int gx0 = bx * (kSX - 1) - 1, gy0 = by * (kSY - 1) - 1;
  const int cx = gx0 + i, cy = gy0 + j;
  const int z_lo = bz * zc;
  const int z_hi = min(z_lo + zc, cp.nn[2]);
  const int64_t nn = cp.n_nodes, sy = cp.ns[1], sz = cp.ns[2];
  const bool own_xy = i >= 1 && j >= 1 && cx <= cp.nn[0] - 1 && cy <= cp.nn[1] - 1;
  if (q1_hole_tile(cp, gx0, gy0)) {  // uniform over the workgroup: no barrier has run yet
    q1_hole_rows3<T, CHEB>(cp, own_xy, cx, cy, z_lo, z_hi, x, mask, y, cf, cc);
    return;
  }
  const bool cell_xy = cx >= 0 && cx < cp.N[0] && cy >= 0 && cy < cp.N[1] &&
                       !cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1]);
  const int ln = i + j * kSNX;  // the lane's node (lower corner of its cell) in the tile plane
  const Consts<T> kc(cp, 8);
  const T* __restrict__ qcb = (const T*)cp.qcb;

  // stream plane kz (all fields and the mask) into ring slot kz mod 3
  PlaneStream<T> ps;
  ps.init(gx0, gy0, cp, tid);
  // the mask bytes go through registers: the lane's (at most two) nodes of the plane
  uint32_t moff[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + h * kSThreads;
    const int jj = e / kSNX, ii = e - jj * kSNX;
    const int gx = gx0 + ii, gy = gy0 + jj;
    moff[h] = (e < kSPlane && gx >= 0 && gx < cp.nn[0] && gy >= 0 && gy < cp.nn[1])
                  ? (uint32_t)((int64_t)gx + (int64_t)gy * sy) : ~0u;
  }
  auto fetch = [&](int kz, uint8_t& m0, uint8_t& m1) {
    const int slot = (kz + 3) % 3;
    const int64_t zo = (int64_t)kz * sz;
#pragma unroll
    for (int c = 0; c < 4; ++c) ps.fetch(x + c * nn + zo, &sv[slot][c][0], wave);
    if constexpr (COUPLE) {
#pragma unroll
      for (int c = 0; c < 4; ++c) ps.fetch(U + c * nn + zo, &sv[slot][F::U0 + c][0], wave);
    }
    ps.fetch(phit + zo, &sv[slot][F::PT][0], wave);
    const uint8_t* mp = mask + zo;
    uint32_t o0 = moff[0], o1 = moff[1];
    __asm__ __volatile__("" : "+v"(o0), "+v"(o1));
    m0 = mp[o0 != ~0u ? o0 : 0u];
    m1 = mp[o1 != ~0u ? o1 : 0u];
  };
  auto put_mask = [&](int kz, uint8_t m0, uint8_t m1) {
    const int slot = (kz + 3) % 3;
    sm[slot][tid] = m0;
    if (tid + kSThreads < kSPlane) sm[slot][tid + kSThreads] = m1;
  };

  // prologue: planes z_lo - 1 and z_lo
  {
    uint8_t a0, a1, b0, b1;
    const bool pa = z_lo - 1 >= 0, pb = z_lo < cp.nn[2];
    if (pa) fetch(z_lo - 1, a0, a1);
    if (pb) fetch(z_lo, b0, b1);
    __builtin_amdgcn_s_waitcnt(0);
    if (pa) put_mask(z_lo - 1, a0, a1);
    if (pb) put_mask(z_lo, b0, b1);
    __syncthreads();
  }

  T carry[4] = {T(0), T(0), T(0), T(0)};
  for (int kz = z_lo - 1; kz < z_hi; ++kz) {
    const int par = kz & 1;
    // the plane after next streams in while this layer computes
    const int kn = kz + 2;
    const bool pre = kn <= z_hi && kn < cp.nn[2];
    uint8_t n0 = 0xFF, n1 = 0xFF;
    if (pre) fetch(kn, n0, n1);
    // the fused step's operands at the lane's own node of plane kz, requested early so that the
    // layer's cell math covers their latency: residual and diagonal here, the iterate before the
    // phase-field rows
    T fr[4] = {T(0), T(0), T(0), T(0)}, fd[4] = {T(1), T(1), T(1), T(1)};
    if constexpr (CHEB) {
      if (own_xy && kz >= z_lo) {
        const int64_t go = (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          fr[c] = cf.res[c * nn + go];
          fd[c] = cf.diag[c * nn + go];
        }
      }
    }

    const bool cell = cell_xy && kz >= 0 && kz < cp.N[2];
    const int lo = (kz + 3) % 3, hi = (kz + 4) % 3;
    uint8_t mk[8];
    if (cell) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int o = ln + (a & 1) + (a >> 1) * kSNX;
        mk[a] = sm[lo][o];
        mk[a + 4] = sm[hi][o];
      }
    }
    T Y[4][2];
    T fx[4] = {T(0), T(0), T(0), T(0)};  // the fused step's iterate at the own node (requested below)
    if constexpr (MODE == MODE_APPLY && sizeof(T) == 8) {
      // FP64 G~: displacement and phase-field rows from the same per-layer tables of du
      T outu[3][8], outp[8];
      if (cell) {
        T dp[8];
        corners<T>(&sv[lo][3][0], &sv[hi][3][0], ln, dp);
#pragma unroll
        for (int a = 0; a < 8; ++a)
          if (mk[a] & kMaskPhi) dp[a] = T(0);
        g_rows_layers<T, F::NF>(kc, sv[lo], sv[hi], ln, mk, F::U0, F::PT, dp, outu, outp);
      } else {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
#pragma unroll
          for (int c = 0; c < 3; ++c) outu[c][a] = T(0);
          outp[a] = T(0);
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T X1[2];
        combine_xy<T>(c < 3 ? outu[c] : outp, first_row, Y[c], X1);
        if (last_row && wave < kSWaves - 1) {
          sx[par][wave][i][2 * c] = X1[0];
          sx[par][wave][i][2 * c + 1] = X1[1];
        }
      }
    } else {
      // displacement rows
      {
        T outu[3][8];
        if (cell) {
          T du[3][8], pt[8];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            corners<T>(&sv[lo][c][0], &sv[hi][c][0], ln, du[c]);
#pragma unroll
            for (int a = 0; a < 8; ++a)
              if (mk[a] & (1 << c)) du[c][a] = T(0);
          }
          corners<T>(&sv[lo][F::PT][0], &sv[hi][F::PT][0], ln, pt);
          cell3_u<T>(kc, du, pt, outu);
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < 8; ++a) outu[c][a] = T(0);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T X1[2];
          combine_xy<T>(outu[c], first_row, Y[c], X1);
          if (last_row && wave < kSWaves - 1) {
            sx[par][wave][i][2 * c] = X1[0];
            sx[par][wave][i][2 * c + 1] = X1[1];
          }
        }
      }
      // keep the compiler from carrying the corner values of the first part into the second
      __asm__ __volatile__("" ::: "memory");
      if constexpr (CHEB) {
        if (own_xy && kz >= z_lo) {
          const int64_t go = (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz;
#pragma unroll
          for (int c = 0; c < 4; ++c) fx[c] = cf.x[c * nn + go];
        }
      }
      // phase-field rows
      {
        T outp[8];
        if (cell) {
          T dp[8];
          corners<T>(&sv[lo][3][0], &sv[hi][3][0], ln, dp);
#pragma unroll
          for (int a = 0; a < 8; ++a)
            if (mk[a] & kMaskPhi) dp[a] = T(0);
          if constexpr (MODE == MODE_BLOCK) {
            const int64_t cid = (int64_t)cx + (int64_t)cy * cp.N[0] + (int64_t)kz * cp.N[0] * cp.N[1];
            T cq[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) cq[q] = qcb[q * cp.n_cells + cid];
            cell3_phi_stored<T>(kc, dp, cq, outp);
          } else {
            // FP32 G~ (FP64 takes g_rows_layers above): the whole-cell tables fit its registers
            T du[3][8], uu[3][8], ph[8];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              corners<T>(&sv[lo][c][0], &sv[hi][c][0], ln, du[c]);
#pragma unroll
              for (int a = 0; a < 8; ++a)
                if (mk[a] & (1 << c)) du[c][a] = T(0);
              corners<T>(&sv[lo][F::U0 + c][0], &sv[hi][F::U0 + c][0], ln, uu[c]);
            }
            corners<T>(&sv[lo][F::U0 + 3][0], &sv[hi][F::U0 + 3][0], ln, ph);
            cell3_phi<T, COUPLE>(kc, du, dp, uu, ph, outp);
          }
        } else {
#pragma unroll
          for (int a = 0; a < 8; ++a) outp[a] = T(0);
        }
        T X1[2];
        combine_xy<T>(outp, first_row, Y[3], X1);
        if (last_row && wave < kSWaves - 1) {
          sx[par][wave][i][6] = X1[0];
          sx[par][wave][i][7] = X1[1];
        }
      }
    }
    // the own node's input values and mask on plane kz, read before the barrier: after it the
    // ring slot of plane kz is refilled with plane kz + 3 by waves that run ahead
    T xo[4];
    uint8_t mo = 0;
    if (own_xy && kz >= z_lo) {
#pragma unroll
      for (int c = 0; c < 4; ++c) xo[c] = sv[lo][c][ln];
      mo = sm[lo][ln];
    }
    // the streamed plane and this layer's exchange are complete and visible after this point
    __builtin_amdgcn_s_waitcnt(0);
    if (pre) put_mask(kn, n0, n1);
    __syncthreads();
    if (first_row && wave > 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        Y[c][0] += sx[par][wave - 1][i][2 * c];
        Y[c][1] += sx[par][wave - 1][i][2 * c + 1];
      }
    }
    if (own_xy && kz >= z_lo) {
      const int64_t go = (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz;
      const uint8_t m = mo;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T val = Y[c][0] + carry[c];
        const int64_t o = c * nn + go;
        const bool con = m & mask_bit(c, 3);
        if constexpr (CHEB) {
          const T c1 = c == 3 ? cc[2] : cc[0], c2 = c == 3 ? cc[3] : cc[1];
          const T d = xo[c];
          const T r = fr[c] - (con ? d : val);
          cf.res[o] = r;
          const T dn = c1 * d + c2 * r / fd[c];
          const T xn = fx[c] + dn;
          cf.x[o] = xn;
          if (cf.d_out) cf.d_out[o] = dn;
          if (cf.t_next) cf.t_next[o] = con ? (cf.next_of_x ? xn : dn) : T(0);
        } else {
          y[o] = con ? xo[c] : val;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) carry[c] = Y[c][1];
  }
}

// ----------------------------------------------------------------------------------- launch
static int64_t slab_tiles(const Geom& g, int64_t* ntx) {
  *ntx = (g.nn[0] + kSX - 2) / (kSX - 1);
  const int64_t nty = (g.nn[1] + kSY - 2) / (kSY - 1);
  return *ntx * nty;
}

int q1_slab_chunk(const Geom& g, int requested_zc) {
  if (requested_zc > 0) return requested_zc;
  int64_t ntx;
  const int64_t tiles = slab_tiles(g, &ntx);
  const int cand[] = {64, 32, 16};
  for (int z : cand)
    if (tiles * ((g.nn[2] + z - 1) / z) >= 1024) return z;
  return 8;
}

template <typename T>
pf_status launch_q1_slab(const Geom& g, const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                         const uint8_t* mask, T* y, const ChebFuse<T>* cf, hipStream_t s) {
  if (g.d != 3 || g.p != 1) {
    set_error("Q1 slabs: 3D Q1 levels only");
    return PF_ERR_UNSUPPORTED;
  }
  if (g.n_cells == 0) return PF_OK;
  int64_t ntx;
  const int64_t tiles = slab_tiles(g, &ntx);
  const int zc = q1_slab_chunk(g, cp.zc);
  const int nzc = (g.nn[2] + zc - 1) / zc;
  const int64_t nb = tiles * nzc;
  if (nb > 0x7fffffff) {
    set_error("Q1 slabs: too many tiles for one launch");
    return PF_ERR_UNSUPPORTED;
  }
  const unsigned grid = (unsigned)nb;
  const ChebFuse<T> none{};
  if (cf) {
    if (mode != MODE_BLOCK) {
      set_error("Q1 slabs: the fused Chebyshev step follows the block operator");
      return PF_ERR_UNSUPPORTED;
    }
    k_q1_3d_slab<T, MODE_BLOCK, true><<<grid, kSThreads, 0, s>>>(cp, zc, (int)ntx, nzc, x, U, phit, mask, nullptr, *cf);
  } else if (mode == MODE_APPLY) {
    k_q1_3d_slab<T, MODE_APPLY, false><<<grid, kSThreads, 0, s>>>(cp, zc, (int)ntx, nzc, x, U, phit, mask, y, none);
  } else {
    k_q1_3d_slab<T, MODE_BLOCK, false><<<grid, kSThreads, 0, s>>>(cp, zc, (int)ntx, nzc, x, U, phit, mask, y, none);
  }
  PFF_CHECK_LAUNCH();
  return PF_OK;
}
template pf_status launch_q1_slab<double>(const Geom&, const CellParams&, int, const double*, const double*,
                                          const double*, const uint8_t*, double*, const ChebFuse<double>*, hipStream_t);
template pf_status launch_q1_slab<float>(const Geom&, const CellParams&, int, const float*, const float*, const float*,
                                         const uint8_t*, float*, const ChebFuse<float>*, hipStream_t);

}  // namespace pff
