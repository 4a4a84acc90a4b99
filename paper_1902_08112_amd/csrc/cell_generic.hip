// Generic matrix-free cell loop: one thread per cell, any (dim, degree).
//
// Computes, cell by cell, the local contribution C^T P_k^T G_k P_k C x of the
// Jacobian (Sec. 4.1), the residual -A(U) or the diagonal of G, with the
// integrands of the semi-linear form (Sec. 2.3, eq. semilinear, no split):
//   u rows:   g(phi~) sigma(du) : e(w)
//   phi rows: [(1-kappa) phi sigma(u):e(du) + 2 p phi div du
//              + ((1-kappa) E_s(e(u)) + 2 p div u + G_c/eps) dphi] psi
//             + G_c eps grad dphi . grad psi
// (the factor 1/2 in front of d_phi g_kappa E_s taken literally; phi~ in the
// displacement equation, so the u-phi block vanishes, Sec. 3.3).
// Gauss quadrature with p+1 points per direction on affine box cells.
// Contributions are scattered with device atomics; the tiled Q1 kernels in
// cell_q1.hip are the fast path, this kernel covers Q2 and is the fallback.
#include "common.h"

namespace pff {

// 1D Lagrange basis on the nodes {0, 1} / {0, 1/2, 1} at the Gauss points of [0, 1].
template <int P>
struct B1;

template <>
struct B1<1> {
  static constexpr int n = 2;
  __device__ static constexpr double pt(int q) { return q == 0 ? 0.21132486540518711775 : 0.78867513459481288225; }
  __device__ static constexpr double wt(int) { return 0.5; }
  __device__ static constexpr double val(int a, double t) { return a == 0 ? 1.0 - t : t; }
  __device__ static constexpr double der(int a, double) { return a == 0 ? -1.0 : 1.0; }
};

template <>
struct B1<2> {
  static constexpr int n = 3;
  __device__ static constexpr double pt(int q) {
    return q == 0 ? 0.11270166537925831148 : (q == 1 ? 0.5 : 0.88729833462074168852);
  }
  __device__ static constexpr double wt(int q) { return q == 1 ? 8.0 / 18.0 : 5.0 / 18.0; }
  __device__ static constexpr double val(int a, double t) {
    return a == 0 ? 2.0 * (t - 0.5) * (t - 1.0) : (a == 1 ? 4.0 * t * (1.0 - t) : 2.0 * t * (t - 0.5));
  }
  __device__ static constexpr double der(int a, double t) {
    return a == 0 ? 4.0 * t - 3.0 : (a == 1 ? 4.0 - 8.0 * t : 4.0 * t - 1.0);
  }
};

template <int D, int P>
struct Tens {
  static constexpr int n = P + 1;
  static constexpr int NL = D == 2 ? n * n : n * n * n;
  __device__ static constexpr int idx(int a, int k) { return k == 0 ? a % n : (k == 1 ? (a / n) % n : a / (n * n)); }
  // shape value N_a at quadrature point q
  __device__ static constexpr double N(int q, int a) {
    double v = 1.0;
    for (int k = 0; k < D; ++k) v *= B1<P>::val(idx(a, k), B1<P>::pt(idx(q, k)));
    return v;
  }
  // reference derivative d N_a / d xi_j at q
  __device__ static constexpr double dN(int q, int a, int j) {
    double v = 1.0;
    for (int k = 0; k < D; ++k)
      v *= (k == j) ? B1<P>::der(idx(a, k), B1<P>::pt(idx(q, k))) : B1<P>::val(idx(a, k), B1<P>::pt(idx(q, k)));
    return v;
  }
  __device__ static constexpr double w(int q) {
    double v = 1.0;
    for (int k = 0; k < D; ++k) v *= B1<P>::wt(idx(q, k));
    return v;
  }
};

template <int D, int P, typename T, int MODE>
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
  T xv[D + 1][NL];
  T uv[D + 1][NL];
  T pv[NL];
  uint8_t mk[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) {
    mk[a] = kMasked ? mask[g[a]] : 0;
    pv[a] = phit[g[a]];
#pragma unroll
    for (int i = 0; i <= D; ++i) {
      uv[i][a] = U[i * nn + g[a]];
      if (kDir) {
        T v = x[i * nn + g[a]];
        xv[i][a] = (kMasked && (mk[a] & mask_bit(i, D))) ? T(0) : v;
      } else {
        xv[i][a] = T(0);
      }
    }
  }

  const T mu = T(cp.mu), lam = T(cp.lam), kap = T(cp.kappa), pres = T(cp.pres);
  const T gce = T(cp.gc_over_eps), gcx = T(cp.gc_eps);
  T ih[3] = {T(cp.inv_h[0]), T(cp.inv_h[1]), T(cp.inv_h[2])};

  T out[D + 1][NL];
#pragma unroll
  for (int i = 0; i <= D; ++i)
#pragma unroll
    for (int a = 0; a < NL; ++a) out[i][a] = T(0);

#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const T jxw = T(TT::w(q) * cp.vol);
    // linearization point at q
    T gu[D][D];
    T phi = T(0), pt = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) gu[i][j] = T(0);
    T gphi[D];
#pragma unroll
    for (int j = 0; j < D; ++j) gphi[j] = T(0);
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      const T Na = T(TT::N(q, a));
      phi += Na * uv[D][a];
      pt += Na * pv[a];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const T dNa = T(TT::dN(q, a, j)) * ih[j];
#pragma unroll
        for (int i = 0; i < D; ++i) gu[i][j] += dNa * uv[i][a];
        gphi[j] += dNa * uv[D][a];
      }
    }
    T tr_u = T(0), ee = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) tr_u += gu[i][i];
    T su[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const T e = T(0.5) * (gu[i][j] + gu[j][i]);
        ee += e * e;
        su[i][j] = T(2) * mu * e + (i == j ? lam * tr_u : T(0));
      }
    const T Es = T(0.5) * lam * tr_u * tr_u + mu * ee;
    const T gdeg = (T(1) - kap) * pt * pt + kap;

    if (MODE == MODE_DIAG) {
      const T cphi = (T(1) - kap) * Es + T(2) * pres * tr_u + gce;
#pragma unroll
      for (int a = 0; a < NL; ++a) {
        const T Na = T(TT::N(q, a));
        T dn[D];
        T g2 = T(0);
#pragma unroll
        for (int j = 0; j < D; ++j) {
          dn[j] = T(TT::dN(q, a, j)) * ih[j];
          g2 += dn[j] * dn[j];
        }
#pragma unroll
        for (int i = 0; i < D; ++i) out[i][a] += jxw * gdeg * (mu * (g2 + dn[i] * dn[i]) + lam * dn[i] * dn[i]);
        out[D][a] += jxw * (cphi * Na * Na + gcx * g2);
      }
      continue;
    }

    T tau[D][D];
    T fval, zeta[D];
    if (MODE == MODE_RESID) {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) tau[i][j] = -(gdeg * su[i][j] + (i == j ? pt * pt * pres : T(0)));
      fval = -((T(1) - kap) * phi * Es + T(2) * phi * pres * tr_u - gce * (T(1) - phi));
#pragma unroll
      for (int j = 0; j < D; ++j) zeta[j] = -gcx * gphi[j];
    } else {
      // direction at q
      T gd[D][D];
      T dphi = T(0);
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) gd[i][j] = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) zeta[j] = T(0);
#pragma unroll
      for (int a = 0; a < NL; ++a) {
        const T Na = T(TT::N(q, a));
        dphi += Na * xv[D][a];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const T dNa = T(TT::dN(q, a, j)) * ih[j];
#pragma unroll
          for (int i = 0; i < D; ++i) gd[i][j] += dNa * xv[i][a];
          zeta[j] += dNa * xv[D][a];
        }
      }
      T tr_d = T(0), se = T(0);
#pragma unroll
      for (int i = 0; i < D; ++i) tr_d += gd[i][i];
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const T e = T(0.5) * (gd[i][j] + gd[j][i]);
          se += su[i][j] * e;
          tau[i][j] = gdeg * (T(2) * mu * e + (i == j ? lam * tr_d : T(0)));
        }
      const T cphi = (T(1) - kap) * Es + T(2) * pres * tr_u + gce;
      fval = cphi * dphi;
      if (MODE != MODE_BLOCK) fval += (T(1) - kap) * phi * se + T(2) * pres * phi * tr_d;
#pragma unroll
      for (int j = 0; j < D; ++j) zeta[j] *= gcx;
    }
    // test functions
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      const T Na = T(TT::N(q, a));
      T acc = fval * Na;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const T dNa = T(TT::dN(q, a, j)) * ih[j];
        acc += zeta[j] * dNa;
#pragma unroll
        for (int i = 0; i < D; ++i) out[i][a] += jxw * tau[i][j] * dNa;
      }
      out[D][a] += jxw * acc;
    }
  }

#pragma unroll
  for (int a = 0; a < NL; ++a)
#pragma unroll
    for (int i = 0; i <= D; ++i) {
      if (kMasked && (mk[a] & mask_bit(i, D))) continue;
      atomicAdd(&y[i * nn + g[a]], out[i][a]);
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
  return cp;
}

template <int D, int P, typename T>
static pf_status launch_dp(const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                           const uint8_t* mask, T* y, hipStream_t s) {
  const int bs = 128;
  const int64_t nb = (cp.n_cells + bs - 1) / bs;
  if (nb == 0) return PF_OK;
  switch (mode) {
    case MODE_APPLY:
      k_cell_generic<D, P, T, MODE_APPLY><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
      break;
    case MODE_BLOCK:
      k_cell_generic<D, P, T, MODE_BLOCK><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
      break;
    default:
      if constexpr (std::is_same<T, double>::value) {
        if (mode == MODE_RAW)
          k_cell_generic<D, P, T, MODE_RAW><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
        else if (mode == MODE_RESID)
          k_cell_generic<D, P, T, MODE_RESID><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
        else if (mode == MODE_DIAG)
          k_cell_generic<D, P, T, MODE_DIAG><<<nb, bs, 0, s>>>(cp, x, U, phit, mask, y);
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
