// Q1 cell loops of the Miehe split (Sec. 2.1) from stored per-point eigen-data.
//
// k_split_data runs once per linearization and level: one work item per (Gauss
// point, cell) computes e(U) at the point, its eigenpairs by Jacobi rotations in
// FP64 (split.h) and writes the record of q1_split.h in FP64 and FP32.  The
// apply kernels then stream the records with the direction: the displacement rows
// form C e(du) - (1 - g(phi~)) C^+ e(du) in registers, the phase-field rows need the
// eigenvalues only (and the eigenvectors for the coupling block).  Two shapes, as
// for the unsplit Q1 loop: one work item per cell (variant 2), or the displacement
// and phase-field rows of a cell in two different wavefronts (variant 4); both
// scatter with device atomics into y pre-set to Pi_C x.
#include "q1_split.h"

namespace pff {

template <int D>
__global__ __launch_bounds__(256) void k_split_data(CellParams cp, const double* __restrict__ U,
                                                    double* __restrict__ rec64, float* __restrict__ rec32) {
  using Lt = q1s::Layout<D>;
  constexpr int NL = D == 3 ? 8 : 4;
  const int64_t nc = cp.n_cells;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * Lt::NQ) return;
  const int q = (int)(t / nc);
  const int64_t cid = t - (int64_t)q * nc;
  const int cx = (int)(cid % cp.N[0]);
  const int cy = (int)((cid / cp.N[0]) % cp.N[1]);
  const int cz = D == 3 ? (int)(cid / ((int64_t)cp.N[0] * cp.N[1])) : 0;
  double v[Lt::NV];
  if (cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) {
#pragma unroll
    for (int k = 0; k < Lt::NV; ++k) v[k] = 0.0;
  } else {
    const int64_t nn = cp.n_nodes;
    const int64_t g0 = (int64_t)cx + (int64_t)cy * cp.ns[1] + (int64_t)cz * cp.ns[2];
    double uc[D][NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      const int64_t gi = g0 + (a & 1) + ((a >> 1) & 1) * cp.ns[1] + (D == 3 ? (a >> 2) * cp.ns[2] : 0);
#pragma unroll
      for (int c = 0; c < D; ++c) uc[c][a] = U[c * nn + gi];
    }
    q1s::cell_records<D>(cp, uc, q, v);
  }
#pragma unroll
  for (int k = 0; k < Lt::NV; ++k) {
    const int64_t o = (int64_t)(k * Lt::NQ + q) * nc + cid;
    rec64[o] = v[k];
    rec32[o] = (float)v[k];
  }
}

// PARTS = 1: one work item per cell; PARTS = 2: displacement rows in even, phase-field rows in odd
// wavefronts of a block of 128 (64 cells per block)
template <int D, typename T, int MODE, int PARTS>
__global__ __launch_bounds__(128) void k_q1s(CellParams cp, const T* __restrict__ rec, const T* __restrict__ x,
                                             const T* __restrict__ U, const T* __restrict__ phit,
                                             const uint8_t* __restrict__ mask, T* __restrict__ y) {
  constexpr bool COUPLE = (MODE == MODE_APPLY);
  constexpr int NL = D == 3 ? 8 : 4;
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int part = PARTS == 1 ? 0 : 1 + (int)((w >> 6) & 1);
  const int64_t cid = PARTS == 1 ? w : (w >> 7) * 64 + (w & 63);
  if (cid >= cp.n_cells) return;
  const int cx = (int)(cid % cp.N[0]);
  const int cy = (int)((cid / cp.N[0]) % cp.N[1]);
  const int cz = D == 3 ? (int)(cid / ((int64_t)cp.N[0] * cp.N[1])) : 0;
  if (cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) return;
  const int64_t nn = cp.n_nodes, nc = cp.n_cells;
  const int64_t g0 = (int64_t)cx + (int64_t)cy * cp.ns[1] + (int64_t)cz * cp.ns[2];
  int64_t gi[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) gi[a] = g0 + (a & 1) + ((a >> 1) & 1) * cp.ns[1] + (D == 3 ? (a >> 2) * cp.ns[2] : 0);
  const q1s::CK<T> k(cp, NL);
  const T* rb = rec + cid;
  uint8_t mk[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) mk[a] = mask[gi[a]];
  T du[D][NL];
  if (part != 2 || COUPLE) {
#pragma unroll
    for (int a = 0; a < NL; ++a)
#pragma unroll
      for (int c = 0; c < D; ++c) du[c][a] = (mk[a] & (1 << c)) ? T(0) : x[c * nn + gi[a]];
  } else {
#pragma unroll
    for (int a = 0; a < NL; ++a)
#pragma unroll
      for (int c = 0; c < D; ++c) du[c][a] = T(0);
  }
  if (part != 2) {
    T pt[NL], ou[D][NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) pt[a] = phit[gi[a]];
    if constexpr (D == 3)
      q1s::cell3_u<T>(k, du, pt, rb, nc, ou);
    else
      q1s::cell2_u<T>(k, du, pt, rb, nc, ou);
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int a = 0; a < NL; ++a)
        if (!(mk[a] & (1 << c))) atomicAdd(&y[c * nn + gi[a]], ou[c][a]);
  }
  if (part == 1) return;
  T dp[NL], ph[NL], op[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) {
    dp[a] = (mk[a] & kMaskPhi) ? T(0) : x[D * nn + gi[a]];
    ph[a] = COUPLE ? U[D * nn + gi[a]] : T(0);
  }
  if constexpr (D == 3)
    q1s::cell3_phi<T, COUPLE>(k, du, dp, ph, rb, nc, op);
  else
    q1s::cell2_phi<T, COUPLE>(k, du, dp, ph, rb, nc, op);
#pragma unroll
  for (int a = 0; a < NL; ++a)
    if (!(mk[a] & kMaskPhi)) atomicAdd(&y[D * nn + gi[a]], op[a]);
}

int split_record_values(int d) { return d == 3 ? q1s::Layout<3>::NV * q1s::Layout<3>::NQ : q1s::Layout<2>::NV * q1s::Layout<2>::NQ; }

pf_status launch_split_data(const Geom& g, const CellParams& cp, const double* U, double* rec64, float* rec32,
                            hipStream_t s) {
  if (g.p != 1 || !rec64 || !rec32) {
    set_error("split records: Q1 levels with record storage only");
    return PF_ERR_UNSUPPORTED;
  }
  const int nq = g.d == 3 ? q1s::Layout<3>::NQ : q1s::Layout<2>::NQ;
  const int64_t n = g.n_cells * nq;
  if (n == 0) return PF_OK;
  const int64_t nb = (n + 255) / 256;
  if (g.d == 3)
    k_split_data<3><<<nb, 256, 0, s>>>(cp, U, rec64, rec32);
  else
    k_split_data<2><<<nb, 256, 0, s>>>(cp, U, rec64, rec32);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <int D, typename T, int PARTS>
static void launch_q1s_dp(const CellParams& cp, int mode, const T* rec, const T* x, const T* U, const T* phit,
                          const uint8_t* mask, T* y, hipStream_t s) {
  const int64_t nb = PARTS == 1 ? (cp.n_cells + 127) / 128 : (2 * ((cp.n_cells + 63) / 64) * 64 + 127) / 128;
  if (mode == MODE_APPLY)
    k_q1s<D, T, MODE_APPLY, PARTS><<<nb, 128, 0, s>>>(cp, rec, x, U, phit, mask, y);
  else
    k_q1s<D, T, MODE_BLOCK, PARTS><<<nb, 128, 0, s>>>(cp, rec, x, U, phit, mask, y);
}

// the split's Q1 apply (MODE_APPLY / MODE_BLOCK, y pre-set to Pi_C x) from the records cp.qpd
template <typename T>
static pf_status launch_q1s(const Geom& g, const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                            const uint8_t* mask, T* y, hipStream_t s, bool* handled) {
  *handled = false;
  if (!(g.p == 1 && cp.qpd && (mode == MODE_APPLY || mode == MODE_BLOCK) && (g.d == 2 || g.d == 3)))
    return PF_OK;
  *handled = true;
  if (g.n_cells == 0) return PF_OK;
  const T* rec = (const T*)cp.qpd;
  const bool parts = cp.variant != 2;  // 4 (two wavefronts per cell) unless the one-item shape is asked for
  if (g.d == 3) {
    if (parts)
      launch_q1s_dp<3, T, 2>(cp, mode, rec, x, U, phit, mask, y, s);
    else
      launch_q1s_dp<3, T, 1>(cp, mode, rec, x, U, phit, mask, y, s);
  } else {
    if (parts)
      launch_q1s_dp<2, T, 2>(cp, mode, rec, x, U, phit, mask, y, s);
    else
      launch_q1s_dp<2, T, 1>(cp, mode, rec, x, U, phit, mask, y, s);
  }
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

pf_status launch_cell_q1s_d(const Geom& g, const CellParams& cp, int mode, const double* x, const double* U,
                            const double* phit, const uint8_t* mask, double* y, hipStream_t s, bool* handled) {
  return launch_q1s<double>(g, cp, mode, x, U, phit, mask, y, s, handled);
}
pf_status launch_cell_q1s_f(const Geom& g, const CellParams& cp, int mode, const float* x, const float* U,
                            const float* phit, const uint8_t* mask, float* y, hipStream_t s, bool* handled) {
  return launch_q1s<float>(g, cp, mode, x, U, phit, mask, y, s, handled);
}

}  // namespace pff
