// Marching-tile bodies of the Q1 cell loop (Sec. 4.1), shared by the single-instance kernels
// (cell_q1.hip) and the batched work-table kernel (batch.hip).
//
// One wavefront per tile.  3D: a TX x TY patch of cells (one cell per lane) marches along z
// through a chunk of node planes; 2D: 64 cells along x march along y.  Each lane owns the node
// at the lower corner of its cell.  Per cell layer the 2^d corner contributions are combined
// without atomics: along x with a one-lane shuffle, along y (3D) with a TX-lane shuffle, and
// along the marching axis with a register carry from the previous layer.  Tiles overlap by one
// cell column in x and y (and one layer per chunk), so a lane with i = 0 or j = 0 computes a halo
// cell and owns nothing; every node is written exactly once, with plain stores, including the
// identity rows of the constrained DoFs.  The result is deterministic.
#pragma once

#include "q1_cell.h"

namespace pff {

// combine the corner contributions of a TX x TY patch: value at the lane's own node of
// plane k (layers k-1 and k) and the carry into plane k+1
template <typename T, int TX>
__device__ __forceinline__ void combine3(const T out[8], T carry, T& val, T& ncarry) {
  T X[2][2];
#pragma unroll
  for (int az = 0; az < 2; ++az)
#pragma unroll
    for (int ay = 0; ay < 2; ++ay) X[ay][az] = out[2 * ay + 4 * az] + __shfl_up(out[1 + 2 * ay + 4 * az], 1, TX);
  const T y0 = X[0][0] + __shfl_up(X[1][0], TX, 64);
  const T y1 = X[0][1] + __shfl_up(X[1][1], TX, 64);
  val = y0 + carry;
  ncarry = y1;
}

// One TX x TY marching tile (bx, by) and z-chunk bz of a 3D Q1 level (the body of k_q1_3d; the
// batched solver runs it for one instance's tile per work item).  One wavefront, lane = threadIdx.x.
// STORED (block operator): read c_phi JxW per Gauss point from cp.qcb; otherwise form it from U.
// A 3D tile whose cells all lie in the L-shape's hole (2 cx >= N0 and 2 cy >= N1 from its first
// cell on) has no cell work: its owned nodes are hole nodes, and the cell loop over no cells leaves
// each row at its identity (constrained) or 0 -- written here without streaming anything else.
// cx0, cy0: the tile's first cell.
__device__ __forceinline__ bool q1_hole_tile(const CellParams& cp, int cx0, int cy0) {
  return cp.lshape && cx0 >= 0 && cy0 >= 0 && 2 * cx0 >= cp.N[0] && 2 * cy0 >= cp.N[1];
}
template <typename T, bool CHEB>
__device__ __forceinline__ void q1_hole_rows3(const CellParams& cp, bool own_xy, int cx, int cy, int z_lo, int z_hi,
                                              const T* __restrict__ x, const uint8_t* __restrict__ mask,
                                              T* __restrict__ y, const ChebFuse<T>& cf, const T (&cc)[4]) {
  if (!own_xy) return;
  const int64_t nn = cp.n_nodes, sy = cp.ns[1], sz = cp.ns[2];
  for (int kz = z_lo; kz < z_hi; ++kz) {
    const int64_t go = (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz;
    const uint8_t m = mask[go];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t o = c * nn + go;
      const bool con = m & mask_bit(c, 3);
      if constexpr (CHEB) {
        // the fused Chebyshev step with (B~ d)(node) = Pi_C d
        const T c1 = c == 3 ? cc[2] : cc[0], c2 = c == 3 ? cc[3] : cc[1];
        const T d = x[o];
        const T r = cf.res[o] - (con ? d : T(0));
        cf.res[o] = r;
        const T dn = c1 * d + c2 * r / cf.diag[o];
        const T xn = cf.x[o] + dn;
        cf.x[o] = xn;
        if (cf.d_out) cf.d_out[o] = dn;
        if (cf.t_next) cf.t_next[o] = con ? (cf.next_of_x ? xn : dn) : T(0);
      } else {
        y[o] = con ? x[o] : T(0);
      }
    }
  }
}

template <typename T, int MODE, int TX, int TY, bool CHEB, bool STORED = true>
__device__ __forceinline__ void q1_tile3(const CellParams& cp, int zc, int bx, int by, int bz, const T* __restrict__ x,
                                         const T* __restrict__ U, const T* __restrict__ phit,
                                         const uint8_t* __restrict__ mask, T* __restrict__ y, const ChebFuse<T>& cf) {
  static_assert(TX * TY == 64, "one wavefront per tile");
  static_assert(!CHEB || MODE == MODE_BLOCK, "the fused Chebyshev step follows the block operator");
  constexpr bool COUPLE = (MODE == MODE_APPLY);
  const int lane = threadIdx.x;
  const int i = lane % TX, j = lane / TX;
  const int cx = bx * (TX - 1) - 1 + i;
  const int cy = by * (TY - 1) - 1 + j;
  const int z_lo = bz * zc;
  const int z_hi = min(z_lo + zc, cp.nn[2]);
  const int64_t nn = cp.n_nodes, sy = cp.ns[1], sz = cp.ns[2];
  const bool own_xy = i >= 1 && j >= 1 && cx <= cp.nn[0] - 1 && cy <= cp.nn[1] - 1;
  const bool cell_xy = cx >= 0 && cx < cp.N[0] && cy >= 0 && cy < cp.N[1] &&
                       !cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1]);
  const Consts<T> kc(cp, 8);
  const T* __restrict__ qcb = (const T*)cp.qcb;  // block operator: stored c_phi JxW per point
  // the fused step's coefficients, read once (device memory: captured launches follow new bounds)
  T cc[4] = {T(0), T(0), T(0), T(0)};
  if constexpr (CHEB) {
#pragma unroll
    for (int k = 0; k < 4; ++k) cc[k] = (T)cf.dc[k];
  }
  if (q1_hole_tile(cp, bx * (TX - 1) - 1, by * (TY - 1) - 1)) {
    q1_hole_rows3<T, CHEB>(cp, own_xy, cx, cy, z_lo, z_hi, x, mask, y, cf, cc);
    return;
  }
  T carry[4] = {T(0), T(0), T(0), T(0)};
  for (int kz = z_lo - 1; kz < z_hi; ++kz) {
    const bool cell = cell_xy && kz >= 0 && kz < cp.N[2];
    const int64_t g0 = cell ? (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz : 0;
    int64_t gi[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) gi[a] = g0 + (a & 1) + ((a >> 1) & 1) * sy + (a >> 2) * sz;
    uint8_t mk[8];
    T du[3][8];
    T outu[3][8];
    if (cell) {
      T pt[8];
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
      cell3_u<T>(kc, du, pt, outu);
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 8; ++a) outu[c][a] = T(0);
    }
    T val[4], nc[4];
#pragma unroll
    for (int c = 0; c < 3; ++c) combine3<T, TX>(outu[c], carry[c], val[c], nc[c]);
    // the fused step's operands at the lane's own node of plane kz (residual, diagonal, iterate),
    // requested before the phase-field rows so that their math covers the latency
    T fr[4] = {T(0), T(0), T(0), T(0)}, fd[4] = {T(1), T(1), T(1), T(1)}, fx[4] = {T(0), T(0), T(0), T(0)};
    if constexpr (CHEB) {
      if (own_xy && kz >= z_lo) {
        const int64_t go = (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          fr[c] = cf.res[c * nn + go];
          fd[c] = cf.diag[c * nn + go];
          fx[c] = cf.x[c * nn + go];
        }
      }
    }
    T outp[8];
    if (cell) {
      if constexpr (MODE == MODE_BLOCK && STORED) {
        T dp[8], cq[8];
        const int64_t cid = (int64_t)cx + (int64_t)cy * cp.N[0] + (int64_t)kz * cp.N[0] * cp.N[1];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const T v = x[3 * nn + gi[a]];
          dp[a] = (mk[a] & kMaskPhi) ? T(0) : v;
          cq[a] = qcb[a * cp.n_cells + cid];
        }
        cell3_phi_stored<T>(kc, dp, cq, outp);
      } else {
        T dp[8], uu[3][8], ph[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const T v = x[3 * nn + gi[a]];
          dp[a] = (mk[a] & kMaskPhi) ? T(0) : v;
#pragma unroll
          for (int c = 0; c < 3; ++c) uu[c][a] = U[c * nn + gi[a]];
          ph[a] = COUPLE ? U[3 * nn + gi[a]] : T(0);
        }
        cell3_phi<T, COUPLE>(kc, du, dp, uu, ph, outp);
      }
    } else {
#pragma unroll
      for (int a = 0; a < 8; ++a) outp[a] = T(0);
    }
    combine3<T, TX>(outp, carry[3], val[3], nc[3]);
    if (own_xy && kz >= z_lo) {
      const int64_t go = (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz;
      const uint8_t m = mask[go];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t o = c * nn + go;
        const bool con = m & mask_bit(c, 3);
        if constexpr (CHEB) {
          const T c1 = c == 3 ? cc[2] : cc[0], c2 = c == 3 ? cc[3] : cc[1];
          const T d = x[o];
          const T r = fr[c] - (con ? d : val[c]);
          cf.res[o] = r;
          const T dn = c1 * d + c2 * r / fd[c];
          const T xn = fx[c] + dn;
          cf.x[o] = xn;
          if (cf.d_out) cf.d_out[o] = dn;
          if (cf.t_next) cf.t_next[o] = con ? (cf.next_of_x ? xn : dn) : T(0);
        } else {
          y[o] = con ? x[o] : val[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) carry[c] = nc[c];
  }
}

template <typename T>
__device__ __forceinline__ void combine2(const T out[4], T carry, T& val, T& ncarry) {
  const T x0 = out[0] + __shfl_up(out[1], 1, 64);
  const T x1 = out[2] + __shfl_up(out[3], 1, 64);
  val = x0 + carry;
  ncarry = x1;
}

// 2D row tiles: lane i of the wavefront holds node column bx * kT2Cells - 1 + i and, for i < 63, the
// cell to its right; lanes 1..62 own their nodes, lane 0 is the left halo and lane 63 only lends
// its node values to lane 62.
constexpr int kT2Cells = 62;
__host__ __device__ constexpr int64_t q1_tiles2(int nodes_x) { return (nodes_x + kT2Cells - 1) / kT2Cells; }

// One row tile bx and y-chunk by of a 2D Q1 level (the body of k_q1_2d; the batched solver runs
// it for one instance's tile per work item).  One wavefront, lane = threadIdx.x.  The wavefront
// marches up the node rows: each lane loads its own node of each row once (a contiguous
// 64-node segment per field), takes the right-hand corners from lane i + 1 by a shuffle and the
// lower row from the registers of the previous step.  (Loading one row further ahead measured
// 1.5-3% slower: three waves per SIMD already cover the load latency.)  STORED as for q1_tile3.
template <typename T, int MODE, bool STORED = true>
__device__ __forceinline__ void q1_tile2(const CellParams& cp, int zc, int bx, int by, const T* __restrict__ x,
                                         const T* __restrict__ U, const T* __restrict__ phit,
                                         const uint8_t* __restrict__ mask, T* __restrict__ y) {
  constexpr bool COUPLE = (MODE == MODE_APPLY);
  constexpr bool SB = MODE == MODE_BLOCK && STORED;  // phase-field rows from stored coefficients
  constexpr int NU = SB ? 0 : (COUPLE ? 3 : 2);      // U components the cell reads
  const int i = threadIdx.x;
  const int cx = bx * kT2Cells - 1 + i;
  const int y_lo = by * zc;
  const int y_hi = min(y_lo + zc, cp.nn[1]);
  const int64_t nn = cp.n_nodes, sy = cp.ns[1];
  const bool node_x = cx >= 0 && cx <= cp.nn[0] - 1;
  const bool own_x = i >= 1 && i <= kT2Cells && node_x;
  const bool cell_x = i <= kT2Cells && cx >= 0 && cx < cp.N[0];
  const Consts<T> kc(cp, 4);
  const T* __restrict__ qcb = (const T*)cp.qcb;  // block operator: stored c_phi JxW per point

  // a node row's values at this lane's column: mask, phi~, x (u, phi), U (u[, phi]); zero off the lattice
  struct Row {
    int m;
    T p, xv[3], uv[NU > 0 ? NU : 1];
  };
  auto load = [&](int ky, Row& r) {
    const bool in = node_x && ky >= 0 && ky < cp.nn[1];
    const int64_t g = in ? (int64_t)cx + (int64_t)ky * sy : 0;
    r.m = in ? (int)mask[g] : 0;
    r.p = in ? phit[g] : T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) r.xv[c] = in ? x[c * nn + g] : T(0);
#pragma unroll
    for (int c = 0; c < NU; ++c) r.uv[c] = in ? U[c * nn + g] : T(0);
  };
  auto right = [&](const Row& r, Row& n) {
    n.m = __shfl_down(r.m, 1, 64);
    n.p = __shfl_down(r.p, 1, 64);
#pragma unroll
    for (int c = 0; c < 3; ++c) n.xv[c] = __shfl_down(r.xv[c], 1, 64);
#pragma unroll
    for (int c = 0; c < NU; ++c) n.uv[c] = __shfl_down(r.uv[c], 1, 64);
  };
  Row lo, lon, hi, hin;
  load(y_lo - 1, lo);
  right(lo, lon);
  T carry[3] = {T(0), T(0), T(0)};
  for (int ky = y_lo - 1; ky < y_hi; ++ky) {
    load(ky + 1, hi);
    right(hi, hin);
    const bool cell = cell_x && ky >= 0 && ky < cp.N[1] && !cell_in_hole(cp.lshape, cx, ky, cp.N[0], cp.N[1]);
    // corners a = 0 (cx, ky), 1 (cx + 1, ky), 2 (cx, ky + 1), 3 (cx + 1, ky + 1)
    const int ma[4] = {lo.m, lon.m, hi.m, hin.m};
    const T pt[4] = {lo.p, lon.p, hi.p, hin.p};
    T du[2][4], outu[2][4], dp[4], ua[NU > 0 ? NU : 1][4];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const T xa[4] = {lo.xv[c], lon.xv[c], hi.xv[c], hin.xv[c]};
#pragma unroll
      for (int a = 0; a < 4; ++a) du[c][a] = (ma[a] & (1 << c)) ? T(0) : xa[a];
    }
    {
      const T xa[4] = {lo.xv[2], lon.xv[2], hi.xv[2], hin.xv[2]};
#pragma unroll
      for (int a = 0; a < 4; ++a) dp[a] = (ma[a] & kMaskPhi) ? T(0) : xa[a];
    }
#pragma unroll
    for (int c = 0; c < NU; ++c) {
      ua[c][0] = lo.uv[c];
      ua[c][1] = lon.uv[c];
      ua[c][2] = hi.uv[c];
      ua[c][3] = hin.uv[c];
    }
    if (cell) {
      cell2_u<T>(kc, du, pt, outu);
    } else {
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int a = 0; a < 4; ++a) outu[c][a] = T(0);
    }
    T val[3], nc[3];
    combine2<T>(outu[0], carry[0], val[0], nc[0]);
    combine2<T>(outu[1], carry[1], val[1], nc[1]);
    T outp[4];
    if (cell) {
      if constexpr (SB) {
        T cq[4];
        const int64_t cid = (int64_t)cx + (int64_t)ky * cp.N[0];
#pragma unroll
        for (int a = 0; a < 4; ++a) cq[a] = qcb[a * cp.n_cells + cid];
        cell2_phi_stored<T>(kc, dp, cq, outp);
      } else {
        T uu[2][4], ph[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          uu[0][a] = ua[0][a];
          uu[1][a] = ua[NU > 1 ? 1 : 0][a];
          ph[a] = COUPLE ? ua[NU > 2 ? 2 : 0][a] : T(0);
        }
        cell2_phi<T, COUPLE>(kc, du, dp, uu, ph, outp);
      }
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a) outp[a] = T(0);
    }
    combine2<T>(outp, carry[2], val[2], nc[2]);
    if (own_x && ky >= y_lo) {
      const int64_t go = (int64_t)cx + (int64_t)ky * sy;
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c * nn + go] = (lo.m & mask_bit(c, 2)) ? lo.xv[c] : val[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) carry[c] = nc[c];
    lo = hi;
    lon = hin;
  }
}

}  // namespace pff
