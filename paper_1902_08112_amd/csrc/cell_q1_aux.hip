// The Q1 cell loops that run once per Newton step, FP64, 2D and 3D: the residual -A(U) (Sec. 2.3)
// and the diagonal of G on every level (the Jacobi part of the smoother, Sec. 4.2).  (The
// unconstrained G x of the lift is the Jacobian's own kernel with an all-free mask.)
//
// They use the marching tiles of the Jacobian (q1_tiles.h): one wavefront per tile, one cell per
// lane, the 2^d corner contributions of each cell combined by lane shuffles along x (and y in
// 3D) and a register carry along the marching axis.  Every node of y is written once with a plain
// store -- no atomics, no pre-zeroed output -- and the result does not depend on the schedule.
// No constraint is applied here: the caller sets the constrained rows of the diagonal afterwards.
#include "q1_tiles.h"

namespace pff {

namespace {

constexpr int kXcdsA = 8;
// workgroup b -> tile, one contiguous range of tiles per XCD (workgroups go to XCD b mod 8)
__device__ __forceinline__ int64_t xcd_tile_a(int64_t b, int64_t nb) {
  const int64_t q = nb / kXcdsA, r = nb % kXcdsA;
  const int64_t xcd = b % kXcdsA, k = b / kXcdsA;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// one cell's residual (RESID) or diagonal (DIAG) contributions from its corner values
// (uu: u, ph: phi, pt: phi~)
template <int MODE>
__device__ __forceinline__ void aux_cell3(const Consts<double>& kc, const double (&uu)[3][8], const double (&ph)[8],
                                          const double (&pt)[8], double (&ou)[3][8], double (&op)[8]) {
  if constexpr (MODE == MODE_RESID) {
    cell3_resid<double>(kc, uu, ph, pt, ou, op);
  } else {
    double gw[8], cph[8];
    cell3_diag_coef<double>(kc, uu, pt, gw, cph);
    cell_diag<3, double>(kc, gw, cph, ou, op);
  }
}

}  // namespace

// 3D: TX x TY tiles ordered x fastest, then y, then z-chunk (nzc chunks of zc node planes)
template <int MODE, int TX, int TY>
__global__ __launch_bounds__(64) void k_q1_aux3(CellParams cp, int zc, int ntx, int nzc, const double* __restrict__ U,
                                                const double* __restrict__ phit, double* __restrict__ y) {
  static_assert(TX * TY == 64, "one wavefront per tile");
  const int64_t t = xcd_tile_a(blockIdx.x, gridDim.x);
  const int64_t tiles = (int64_t)gridDim.x / nzc;
  const int bx = (int)(t % ntx);
  const int by = (int)((t / ntx) % (tiles / ntx));
  const int bz = (int)(t / tiles);
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
  if (q1_hole_tile(cp, bx * (TX - 1) - 1, by * (TY - 1) - 1)) {
    // every cell of the tile lies in the hole: its owned rows get no contribution
    if (own_xy)
      for (int kz = z_lo; kz < z_hi; ++kz) {
        const int64_t go = (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz;
#pragma unroll
        for (int c = 0; c < 4; ++c) y[c * nn + go] = 0.0;
      }
    return;
  }
  const Consts<double> kc(cp, 8);
  double carry[4] = {0.0, 0.0, 0.0, 0.0};
  for (int kz = z_lo - 1; kz < z_hi; ++kz) {
    const bool cell = cell_xy && kz >= 0 && kz < cp.N[2];
    double ou[3][8], op[8];
    if (cell) {
      const int64_t g0 = (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz;
      double uu[3][8], ph[8], pt[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int64_t gi = g0 + (a & 1) + ((a >> 1) & 1) * sy + (a >> 2) * sz;
#pragma unroll
        for (int c = 0; c < 3; ++c) uu[c][a] = U[c * nn + gi];
        ph[a] = MODE == MODE_DIAG ? 0.0 : U[3 * nn + gi];
        pt[a] = phit[gi];
      }
      aux_cell3<MODE>(kc, uu, ph, pt, ou, op);
    } else {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
#pragma unroll
        for (int c = 0; c < 3; ++c) ou[c][a] = 0.0;
        op[a] = 0.0;
      }
    }
    double val[4], nc[4];
#pragma unroll
    for (int c = 0; c < 3; ++c) combine3<double, TX>(ou[c], carry[c], val[c], nc[c]);
    combine3<double, TX>(op, carry[3], val[3], nc[3]);
    if (own_xy && kz >= z_lo) {
      const int64_t go = (int64_t)cx + (int64_t)cy * sy + (int64_t)kz * sz;
#pragma unroll
      for (int c = 0; c < 4; ++c) y[c * nn + go] = val[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) carry[c] = nc[c];
  }
}

// 2D: row tiles of kT2Cells owned node columns (lane 0 the left halo, lane 63 lends its node to
// lane 62) marching up a chunk of zc node rows; tiles ordered x fastest.  Each lane loads its
// node of each row once and takes the right-hand corners from lane i + 1.
template <int MODE>
__global__ __launch_bounds__(64) void k_q1_aux2(CellParams cp, int zc, int ntx, const double* __restrict__ U,
                                                const double* __restrict__ phit, double* __restrict__ y) {
  const int64_t t = xcd_tile_a(blockIdx.x, gridDim.x);
  const int bx = (int)(t % ntx), by = (int)(t / ntx);
  const int i = threadIdx.x;
  const int cx = bx * kT2Cells - 1 + i;
  const int y_lo = by * zc;
  const int y_hi = min(y_lo + zc, cp.nn[1]);
  const int64_t nn = cp.n_nodes, sy = cp.ns[1];
  const bool node_x = cx >= 0 && cx <= cp.nn[0] - 1;
  const bool own_x = i >= 1 && i <= kT2Cells && node_x;
  const bool cell_x = i <= kT2Cells && cx >= 0 && cx < cp.N[0];
  const Consts<double> kc(cp, 4);

  // a node row at this lane's column: phi~, U (u, phi); zero off the lattice
  struct Row {
    double p, uv[3];
  };
  auto load = [&](int ky, Row& r) {
    const bool in = node_x && ky >= 0 && ky < cp.nn[1];
    const int64_t g = in ? (int64_t)cx + (int64_t)ky * sy : 0;
    r.p = in ? phit[g] : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) r.uv[c] = in ? U[c * nn + g] : 0.0;
  };
  auto right = [&](const Row& r, Row& n) {
    n.p = __shfl_down(r.p, 1, 64);
#pragma unroll
    for (int c = 0; c < 3; ++c) n.uv[c] = __shfl_down(r.uv[c], 1, 64);
  };
  Row lo, lon, hi, hin;
  load(y_lo - 1, lo);
  right(lo, lon);
  double carry[3] = {0.0, 0.0, 0.0};
  for (int ky = y_lo - 1; ky < y_hi; ++ky) {
    load(ky + 1, hi);
    right(hi, hin);
    const bool cell = cell_x && ky >= 0 && ky < cp.N[1] && !cell_in_hole(cp.lshape, cx, ky, cp.N[0], cp.N[1]);
    // corners a = 0 (cx, ky), 1 (cx + 1, ky), 2 (cx, ky + 1), 3 (cx + 1, ky + 1)
    double ou[2][4], op[4];
    if (cell) {
      const double pt[4] = {lo.p, lon.p, hi.p, hin.p};
      double uu[2][4], ph[4];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        uu[c][0] = lo.uv[c];
        uu[c][1] = lon.uv[c];
        uu[c][2] = hi.uv[c];
        uu[c][3] = hin.uv[c];
      }
      ph[0] = lo.uv[2];
      ph[1] = lon.uv[2];
      ph[2] = hi.uv[2];
      ph[3] = hin.uv[2];
      if constexpr (MODE == MODE_RESID) {
        cell2_resid<double>(kc, uu, ph, pt, ou, op);
      } else {
        double gw[4], cph[4];
        cell2_diag_coef<double>(kc, uu, pt, gw, cph);
        cell_diag<2, double>(kc, gw, cph, ou, op);
      }
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        ou[0][a] = ou[1][a] = 0.0;
        op[a] = 0.0;
      }
    }
    double val[3], nc[3];
    combine2<double>(ou[0], carry[0], val[0], nc[0]);
    combine2<double>(ou[1], carry[1], val[1], nc[1]);
    combine2<double>(op, carry[2], val[2], nc[2]);
    if (own_x && ky >= y_lo) {
      const int64_t go = (int64_t)cx + (int64_t)ky * sy;
#pragma unroll
      for (int c = 0; c < 3; ++c) y[c * nn + go] = val[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) carry[c] = nc[c];
    lo = hi;
    lon = hin;
  }
}

namespace {

template <int MODE>
pf_status launch_aux_mode(const Geom& g, const CellParams& cp, const double* U, const double* phit, double* y,
                          hipStream_t s) {
  if (g.d == 3) {
    constexpr int TX = 8, TY = 8;
    const int64_t ntx = (g.nn[0] + TX - 2) / (TX - 1), nty = (g.nn[1] + TY - 2) / (TY - 1);
    const int zc = q1_chunk(g, 0, 0);
    const int nzc = (g.nn[2] + zc - 1) / zc;
    const int64_t nb = ntx * nty * nzc;
    if (nb > 0x7fffffff) {
      set_error("Q1 residual/diagonal tiles: too many tiles for one launch");
      return PF_ERR_UNSUPPORTED;
    }
    k_q1_aux3<MODE, TX, TY><<<(unsigned)nb, 64, 0, s>>>(cp, zc, (int)ntx, nzc, U, phit, y);
  } else {
    const int64_t ntx = q1_tiles2(g.nn[0]);
    const int zc = q1_chunk(g, 0, 0);
    const int64_t nb = ntx * ((g.nn[1] + zc - 1) / zc);
    if (nb > 0x7fffffff) {
      set_error("Q1 residual/diagonal tiles: too many tiles for one launch");
      return PF_ERR_UNSUPPORTED;
    }
    k_q1_aux2<MODE><<<(unsigned)nb, 64, 0, s>>>(cp, zc, (int)ntx, U, phit, y);
  }
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

}  // namespace

bool q1_aux_handles(const Geom& g, int mode) {
  return g.p == 1 && (g.d == 2 || g.d == 3) && (mode == MODE_RESID || mode == MODE_DIAG);
}

pf_status launch_q1_aux(const Geom& g, const CellParams& cp, int mode, const double* U, const double* phit,
                        double* y, hipStream_t s) {
  if (!q1_aux_handles(g, mode) || cp.split) {
    set_error("Q1 residual/diagonal tiles: a 2D or 3D Q1 level without the energy split");
    return PF_ERR_UNSUPPORTED;
  }
  if (g.n_nodes == 0) return PF_OK;
  if (mode == MODE_RESID) return launch_aux_mode<MODE_RESID>(g, cp, U, phit, y, s);
  return launch_aux_mode<MODE_DIAG>(g, cp, U, phit, y, s);
}

}  // namespace pff
