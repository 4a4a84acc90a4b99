// Coarse-grid solve in one launch: the Chebyshev method used as the solver on
// the coarsest level (Sec. 3.2.2) -- sweeps of r = b - G~ x, x += Cheb_B(r)
// with the per-block interval [0.9 lam_min, 1.2 lam_max] -- run by a single
// workgroup of Q1 cells.
//
// The coarsest level has a few hundred cells, so each operator apply is a
// latency-bound sliver of work; issuing the ~40 applies and ~40 vector updates
// of a coarse solve as separate kernels costs more in launch and drain time
// than the arithmetic.  Here one workgroup loops over all steps.  The operand
// and the result of each apply live in LDS (cell contributions are LDS
// atomics, workgroup barriers order the steps, no device-scope fences); x and
// r stay in global memory, each entry owned by one thread for the whole solve.
// Q1 cells are split into a displacement and a phase-field work item.
#include "q1_cell.h"

namespace pff {

constexpr int kCoarseThreads = 512;
constexpr int kCoarseMaxDegree = 64;
constexpr int64_t kCoarseMaxDofs = 4096;  // two LDS vectors of doubles: 64 KiB

// y = Pi_C x + sum over cells of the masked cell operator (full G~ if COUPLE, else B~); x, y in LDS
template <int D, bool COUPLE>
__device__ void wg_apply(const CellParams& cp, const double* x, double* y, const double* U, const double* phit,
                         const uint8_t* mask) {
  const int64_t nn = cp.n_nodes, n = (int64_t)(D + 1) * nn;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const int c = (int)(i / nn);
    y[i] = (mask[i - (int64_t)c * nn] & mask_bit(c, D)) ? x[i] : 0.0;
  }
  __syncthreads();
  for (int64_t w = threadIdx.x; w < 2 * cp.n_cells; w += blockDim.x) {
    const int64_t cid = w >> 1;
    const int cx = (int)(cid % cp.N[0]);
    const int cy = (int)((cid / cp.N[0]) % cp.N[1]);
    const int cz = D == 3 ? (int)(cid / ((int64_t)cp.N[0] * cp.N[1])) : 0;
    if (cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) continue;
    const int64_t g0 = (int64_t)cx + (int64_t)cy * cp.ns[1] + (int64_t)cz * cp.ns[2];
    q1_cell_atomic<D, double, COUPLE>(cp, g0, x, U, phit, mask, y, 1 + (int)(w & 1));
  }
  __syncthreads();
}

// COUPLE: the sweep residuals b - A x use the full G~ (P_full) or the block-diagonal B~ (P_diag).
// COLUMNS: workgroup j solves for b = e_j (0 if DoF j is constrained) and writes x to column j of
// the dense coarse-solve matrix x = S b (column-major, x + j n; r + j n is its scratch).
template <int D, bool COUPLE, bool COLUMNS>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_solve(CellParams cp, const double* __restrict__ dc, int degree,
                                                                 int sweeps, const double* U,
                                                                 const double* phit, const uint8_t* mask,
                                                                 const double* diag, const double* b, double* x,
                                                                 double* r) {
  extern __shared__ double lds[];
  const int64_t nn = cp.n_nodes, n = (int64_t)(D + 1) * nn, nu = (int64_t)D * nn;
  double* vd = lds;      // apply operand: the Chebyshev direction, or x at a sweep start
  double* vt = lds + n;  // apply result
  int64_t col = -1;
  if (COLUMNS) {
    col = blockIdx.x;
    x += col * n;
    r += col * n;
    const int cc_ = (int)(col / nn);
    if (mask[col - (int64_t)cc_ * nn] & mask_bit(cc_, D)) col = -1;  // constrained: the zero column
  }
  auto bval = [&](int64_t i) -> double { return COLUMNS ? (i == col ? 1.0 : 0.0) : b[i]; };
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) x[i] = 0.0;
  // dc[4 k ..] = {c1, c2} of step k for the displacement block, then the phase-field block; the
  // next step's values are fetched one step ahead, so their latency hides behind an apply
  double cn[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) cn[q] = dc[q];
  for (int sw = 0; sw < sweeps; ++sw) {
    if (sw == 0) {
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) r[i] = bval(i);
    } else {
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) vd[i] = x[i];
      __syncthreads();
      wg_apply<D, COUPLE>(cp, vd, vt, U, phit, mask);
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) r[i] = bval(i) - vt[i];
    }
    for (int k = 0; k < degree; ++k) {
      double cs[4];
      const int kn = k + 1 < degree ? k + 1 : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cs[q] = cn[q];
        cn[q] = dc[4 * kn + q];
      }
      if (k > 0) wg_apply<D, false>(cp, vd, vt, U, phit, mask);
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int blk = i >= nu ? 1 : 0;
        const double c1 = cs[2 * blk], c2 = cs[2 * blk + 1];
        double ri = r[i], dn;
        if (k == 0) {
          dn = c2 * ri / diag[i];
        } else {
          ri -= vt[i];
          r[i] = ri;
          dn = c1 * vd[i] + c2 * ri / diag[i];
        }
        vd[i] = dn;
        x[i] += dn;
      }
      __syncthreads();
    }
  }
}

// Q1 levels up to kCoarseMaxDofs and degrees up to kCoarseMaxDegree; *handled = false otherwise.
// couple: sweep residuals with G~ (P_full) or with B~ (P_diag).  columns: build the dense matrix of
// the solve instead (n workgroups; x and r hold n x n doubles each, b unused).
pf_status launch_coarse_solve(const Geom& g, const CellParams& cp, int degree, int sweeps, const double* dcoef,
                              const double* U, const double* phit, const uint8_t* mask, const double* diag,
                              const double* b, double* x, double* r, bool couple, hipStream_t s, bool* handled,
                              bool columns) {
  *handled = false;
  if (g.p != 1 || degree > kCoarseMaxDegree || degree < 1 || g.n_dofs > kCoarseMaxDofs) return PF_OK;
  const size_t lds = 2 * (size_t)g.n_dofs * sizeof(double);
  const unsigned nwg = columns ? (unsigned)g.n_dofs : 1u;
  if (columns) {
    // many concurrent columns: two wavefronts per column keep the chip full in one round (the
    // single solve uses kCoarseThreads to finish one column fast)
    const int bt = 128;
    if (g.d == 2 && couple)
      k_coarse_solve<2, true, true><<<nwg, bt, lds, s>>>(cp, dcoef, degree, sweeps, U, phit, mask, diag, b, x, r);
    else if (g.d == 2)
      k_coarse_solve<2, false, true><<<nwg, bt, lds, s>>>(cp, dcoef, degree, sweeps, U, phit, mask, diag, b, x, r);
    else if (couple)
      k_coarse_solve<3, true, true><<<nwg, bt, lds, s>>>(cp, dcoef, degree, sweeps, U, phit, mask, diag, b, x, r);
    else
      k_coarse_solve<3, false, true><<<nwg, bt, lds, s>>>(cp, dcoef, degree, sweeps, U, phit, mask, diag, b, x, r);
  } else {
    if (g.d == 2 && couple)
      k_coarse_solve<2, true, false><<<1, kCoarseThreads, lds, s>>>(
          cp, dcoef, degree, sweeps, U, phit, mask, diag, b, x, r);
    else if (g.d == 2)
      k_coarse_solve<2, false, false><<<1, kCoarseThreads, lds, s>>>(
          cp, dcoef, degree, sweeps, U, phit, mask, diag, b, x, r);
    else if (couple)
      k_coarse_solve<3, true, false><<<1, kCoarseThreads, lds, s>>>(
          cp, dcoef, degree, sweeps, U, phit, mask, diag, b, x, r);
    else
      k_coarse_solve<3, false, false><<<1, kCoarseThreads, lds, s>>>(
          cp, dcoef, degree, sweeps, U, phit, mask, diag, b, x, r);
  }
  PFF_CHECK_LAUNCH();
  *handled = true;
  return PF_OK;
}

// T = transpose of the column-major n x n matrix C (T row-major = C column-major read by rows)
__global__ __launch_bounds__(256) void k_coarse_transpose(const double* __restrict__ C, double* __restrict__ T,
                                                          int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * n) return;
  const int64_t i = k / n, j = k - i * n;  // T[i][j] = C[j * n + i]
  T[k] = C[j * n + i];
}

pf_status coarse_transpose(const double* C, double* T, int64_t n, hipStream_t s) {
  if (n <= 0) return PF_OK;
  k_coarse_transpose<<<(unsigned)((n * n + 255) / 256), 256, 0, s>>>(C, T, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

// x = S b with the row-major dense coarse-solve matrix S (n x n): one wavefront per row, lanes
// stride the columns (independent loads), a shuffle reduction ends the row
__global__ __launch_bounds__(256) void k_coarse_matvec(const double* __restrict__ S, const double* __restrict__ b,
                                                       double* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const double* row = S + i * n;
  double acc = 0.0;
  for (int64_t j = lane; j < n; j += 64) acc += row[j] * b[j];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) x[i] = acc;
}

pf_status coarse_matvec(const double* S, const double* b, double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return PF_OK;
  k_coarse_matvec<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(S, b, x, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

}  // namespace pff
