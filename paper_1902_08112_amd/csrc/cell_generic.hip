// Generic matrix-free cell loop: one thread per cell, any (dim, degree).
//
// Computes, cell by cell, the local contribution C^T P_k^T G_k P_k C x of the
// Jacobian (Sec. 4.1), the residual -A(U) or the diagonal of G with the
// integrands of generic_cell.h, and scatters with device atomics.  The Q1
// kernels of cell_q1.hip are the fast path; this kernel covers Q2, the
// residual and diagonal modes, the unmasked (lift) apply, and every mode of the
// Miehe split (SPLIT: the split evaluated on the fly at each point).
#include "generic_cell.h"

namespace pff {

template <int D, int P, typename T, int MODE, bool SPLIT>
__global__ __launch_bounds__(128) void k_cell_generic(CellParams cp, const T* __restrict__ x,
                                                      const T* __restrict__ U, const T* __restrict__ phit,
                                                      const uint8_t* __restrict__ mask, T* __restrict__ y) {
  using TT = Tens<D, P>;
  constexpr int NL = TT::NL;
  const int64_t cid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cid >= cp.n_cells) return;
  int c[3] = {0, 0, 0};
  {
    int64_t r = cid;
    c[0] = (int)(r % cp.N[0]);
    r /= cp.N[0];
    c[1] = (int)(r % cp.N[1]);
    r /= cp.N[1];
    c[2] = (int)r;
  }
  if (cell_in_hole(cp.lshape, c[0], c[1], cp.N[0], cp.N[1])) return;
  const int64_t nn = cp.n_nodes;
  int64_t g[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) {
    int64_t v = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) v += (int64_t)(P * c[k] + TT::idx(a, k)) * cp.ns[k];
    g[a] = v;
  }
  constexpr bool kDir = (MODE == MODE_APPLY || MODE == MODE_BLOCK || MODE == MODE_RAW);
  constexpr bool kMasked = (MODE == MODE_APPLY || MODE == MODE_BLOCK);
  // arithmetic type: the split is evaluated in FP64 whatever the storage type T (FP32 levels
  // read and write FP32 vectors)
  using TC = typename std::conditional<SPLIT, double, T>::type;
  TC xv[D + 1][NL];
  TC uv[D + 1][NL];
  TC pv[NL];
  uint8_t mk[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) {
    mk[a] = kMasked ? mask[g[a]] : 0;
    pv[a] = (TC)phit[g[a]];
#pragma unroll
    for (int i = 0; i <= D; ++i) {
      uv[i][a] = (TC)U[i * nn + g[a]];
      TC v = kDir ? (TC)x[i * nn + g[a]] : TC(0);
      xv[i][a] = (kMasked && (mk[a] & mask_bit(i, D))) ? TC(0) : v;
    }
  }
  TC out[D + 1][NL];
  generic_cell<D, P, TC, MODE, SPLIT>(cp, xv, uv, pv, out);
#pragma unroll
  for (int a = 0; a < NL; ++a)
#pragma unroll
    for (int i = 0; i <= D; ++i) {
      if (kMasked && (mk[a] & mask_bit(i, D))) continue;
      atomicAdd(&y[i * nn + g[a]], (T)out[i][a]);
    }
}

CellParams make_cell_params(const Geom& g, const Material& m) {
  CellParams cp;
  for (int k = 0; k < 3; ++k) {
    cp.N[k] = g.N[k];
    cp.nn[k] = g.nn[k];
    cp.ns[k] = g.ns[k];
    cp.inv_h[k] = k < g.d ? 1.0 / g.h[k] : 0.0;
  }
  cp.n_nodes = g.n_nodes;
  cp.n_cells = g.n_cells;
  cp.lshape = g.lshape;
  cp.vol = 1.0;
  for (int k = 0; k < g.d; ++k) cp.vol *= g.h[k];
  cp.mu = m.mu;
  cp.lam = m.lam;
  cp.kappa = m.kappa;
  cp.pres = m.p;
  cp.gc_over_eps = m.Gc / m.eps;
  cp.gc_eps = m.Gc * m.eps;
  cp.variant = -1;
  cp.zc = -1;
  cp.d = g.d;
  cp.p = g.p;
  cp.split = m.split;
  cp.qpd = nullptr;
  cp.qcb = nullptr;
  return cp;
}

template <int D, int P, typename T, bool SPLIT>
static pf_status launch_dps(const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                            const uint8_t* mask, T* y, hipStream_t s) {
  const int bs = 128;
  const int64_t nb = (cp.n_cells + bs - 1) / bs;
  if (nb == 0) return PF_OK;
  switch (mode) {
    case MODE_APPLY:
      k_cell_generic<D, P, T, MODE_APPLY, SPLIT><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
      break;
    case MODE_BLOCK:
      k_cell_generic<D, P, T, MODE_BLOCK, SPLIT><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
      break;
    default:
      if constexpr (std::is_same<T, double>::value) {
        if (mode == MODE_RAW)
          k_cell_generic<D, P, T, MODE_RAW, SPLIT><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
        else if (mode == MODE_RESID)
          k_cell_generic<D, P, T, MODE_RESID, SPLIT><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
        else if (mode == MODE_DIAG)
          k_cell_generic<D, P, T, MODE_DIAG, SPLIT><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
        else {
          set_error("unknown cell mode");
          return PF_ERR_INVALID_ARG;
        }
      } else {
        set_error("FP32 cell loop supports the apply modes only");
        return PF_ERR_UNSUPPORTED;
      }
  }
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <int D, int P, typename T>
static pf_status launch_dp(const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                           const uint8_t* mask, T* y, hipStream_t s) {
  return cp.split ? launch_dps<D, P, T, true>(cp, mode, x, U, phit, mask, y, s)
                  : launch_dps<D, P, T, false>(cp, mode, x, U, phit, mask, y, s);
}

pf_status launch_cell_generic_d(const Geom& g, const CellParams& cp, int mode, const double* x, const double* U,
                                const double* phit, const uint8_t* mask, double* y, hipStream_t s) {
  if (g.d == 2 && g.p == 1) return launch_dp<2, 1, double>(cp, mode, x, U, phit, mask, y, s);
  if (g.d == 2 && g.p == 2) return launch_dp<2, 2, double>(cp, mode, x, U, phit, mask, y, s);
  if (g.d == 3 && g.p == 1) return launch_dp<3, 1, double>(cp, mode, x, U, phit, mask, y, s);
  if (g.d == 3 && g.p == 2) return launch_dp<3, 2, double>(cp, mode, x, U, phit, mask, y, s);
  set_error("unsupported dim/degree");
  return PF_ERR_UNSUPPORTED;
}

pf_status launch_cell_generic_f(const Geom& g, const CellParams& cp, int mode, const float* x, const float* U,
                                const float* phit, const uint8_t* mask, float* y, hipStream_t s) {
  if (g.d == 2 && g.p == 1) return launch_dp<2, 1, float>(cp, mode, x, U, phit, mask, y, s);
  if (g.d == 2 && g.p == 2) return launch_dp<2, 2, float>(cp, mode, x, U, phit, mask, y, s);
  if (g.d == 3 && g.p == 1) return launch_dp<3, 1, float>(cp, mode, x, U, phit, mask, y, s);
  if (g.d == 3 && g.p == 2) return launch_dp<3, 2, float>(cp, mode, x, U, phit, mask, y, s);
  set_error("unsupported dim/degree");
  return PF_ERR_UNSUPPORTED;
}

}  // namespace pff
