// Per-cell operator math for any (dim, degree) by direct evaluation at the
// (p+1)^d Gauss points: Jacobian (full or smoother block), residual -A(U),
// or the diagonal of G.  Integrands of the semi-linear form (Sec. 2.3, phi~ in
// the displacement equation, the 1/2 of the phase-field equation read literally):
//   u rows:   g(phi~) sigma(du) : e(w)                     [residual: + phi~^2 p div w]
//   phi rows: [(1-kappa) phi sigma(u):e(du) + 2 p phi div du
//              + ((1-kappa) E_s(e(u)) + 2 p div u + G_c/eps) dphi] psi
//             + G_c eps grad dphi . grad psi
// With SPLIT (Miehe split, Sec. 2.1, split.h) E_s and sigma(u) of the phase-field rows
// become E_s^+ and sigma^+(u), and the displacement rows use g sigma^+ + sigma^- =
// sigma - (1 - g) sigma^+ with the tangent C - (1 - g) C^+ at e(u); the split at each
// point is evaluated on the fly in FP64.
#pragma once

#include "common.h"
#include "split.h"

namespace pff {

// 1D Lagrange basis on the nodes {0, 1} / {0, 1/2, 1} at the Gauss points of [0, 1].
template <int P>
struct B1;

template <>
struct B1<1> {
  static constexpr int n = 2;
  __host__ __device__ static constexpr double pt(int q) {
    return q == 0 ? 0.21132486540518711775 : 0.78867513459481288225;
  }
  __host__ __device__ static constexpr double wt(int) { return 0.5; }
  __host__ __device__ static constexpr double val(int a, double t) { return a == 0 ? 1.0 - t : t; }
  __host__ __device__ static constexpr double der(int a, double) { return a == 0 ? -1.0 : 1.0; }
};

template <>
struct B1<2> {
  static constexpr int n = 3;
  __host__ __device__ static constexpr double pt(int q) {
    return q == 0 ? 0.11270166537925831148 : (q == 1 ? 0.5 : 0.88729833462074168852);
  }
  __host__ __device__ static constexpr double wt(int q) { return q == 1 ? 8.0 / 18.0 : 5.0 / 18.0; }
  __host__ __device__ static constexpr double val(int a, double t) {
    return a == 0 ? 2.0 * (t - 0.5) * (t - 1.0) : (a == 1 ? 4.0 * t * (1.0 - t) : 2.0 * t * (t - 0.5));
  }
  __host__ __device__ static constexpr double der(int a, double t) {
    return a == 0 ? 4.0 * t - 3.0 : (a == 1 ? 4.0 - 8.0 * t : 4.0 * t - 1.0);
  }
};

template <int D, int P>
struct Tens {
  static constexpr int n = P + 1;
  static constexpr int NL = D == 2 ? n * n : n * n * n;
  __host__ __device__ static constexpr int idx(int a, int k) {
    return k == 0 ? a % n : (k == 1 ? (a / n) % n : a / (n * n));
  }
  __host__ __device__ static constexpr double N(int q, int a) {
    double v = 1.0;
    for (int k = 0; k < D; ++k) v *= B1<P>::val(idx(a, k), B1<P>::pt(idx(q, k)));
    return v;
  }
  __host__ __device__ static constexpr double dN(int q, int a, int j) {
    double v = 1.0;
    for (int k = 0; k < D; ++k)
      v *= (k == j) ? B1<P>::der(idx(a, k), B1<P>::pt(idx(q, k))) : B1<P>::val(idx(a, k), B1<P>::pt(idx(q, k)));
    return v;
  }
  __host__ __device__ static constexpr double w(int q) {
    double v = 1.0;
    for (int k = 0; k < D; ++k) v *= B1<P>::wt(idx(q, k));
    return v;
  }
};

// out[i][a] = contributions of one cell; xv: direction (already masked), uv: U, pv: phi~
template <int D, int P, typename T, int MODE, bool SPLIT = false>
__device__ __forceinline__ void generic_cell(const CellParams& cp, const T (&xv)[D + 1][Tens<D, P>::NL],
                                             const T (&uv)[D + 1][Tens<D, P>::NL], const T (&pv)[Tens<D, P>::NL],
                                             T (&out)[D + 1][Tens<D, P>::NL]) {
  using TT = Tens<D, P>;
  constexpr int NL = TT::NL;
  const T mu = T(cp.mu), lam = T(cp.lam), kap = T(cp.kappa), pres = T(cp.pres);
  const T gce = T(cp.gc_over_eps), gcx = T(cp.gc_eps);
  const T ih[3] = {T(cp.inv_h[0]), T(cp.inv_h[1]), T(cp.inv_h[2])};
#pragma unroll
  for (int i = 0; i <= D; ++i)
#pragma unroll
    for (int a = 0; a < NL; ++a) out[i][a] = T(0);

#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const T jxw = T(TT::w(q) * cp.vol);
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
    const T omg = T(1) - gdeg;  // 1 - g(phi~)
    // E_s^+ and sigma^+(u): the split at this point, or E_s and sigma(u) without one
    split::QP<D> sq;
    T EsP = Es;
    T sp[D][D];
    if constexpr (SPLIT) {
      double ed[D][D];
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) ed[i][j] = 0.5 * ((double)gu[i][j] + (double)gu[j][i]);
      split::eval<D>(ed, cp.mu, cp.lam, sq);
      EsP = T(sq.Es_pos);
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) sp[i][j] = T(sq.sig[i][j]);
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) sp[i][j] = su[i][j];
    }

    if (MODE == MODE_DIAG) {
      const T cphi = (T(1) - kap) * EsP + T(2) * pres * tr_u + gce;
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
        double dnd[D];
#pragma unroll
        for (int j = 0; j < D; ++j) dnd[j] = (double)dn[j];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          const T ece = mu * (g2 + dn[i] * dn[i]) + lam * dn[i] * dn[i];  // e(w):C e(w), w = N_a e_i
          if constexpr (SPLIT)
            out[i][a] += jxw * (ece - omg * T(split::test_energy<D>(sq, cp.mu, cp.lam, i, dnd)));
          else
            out[i][a] += jxw * gdeg * ece;
        }
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
        for (int j = 0; j < D; ++j) {
          const T sg = SPLIT ? su[i][j] - omg * sp[i][j] : gdeg * su[i][j];
          tau[i][j] = -(sg + (i == j ? pt * pt * pres : T(0)));
        }
      fval = -((T(1) - kap) * phi * EsP + T(2) * phi * pres * tr_u - gce * (T(1) - phi));
#pragma unroll
      for (int j = 0; j < D; ++j) zeta[j] = -gcx * gphi[j];
    } else {
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
      double hd[D][D], cpd[D][D];
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const T e = T(0.5) * (gd[i][j] + gd[j][i]);
          se += sp[i][j] * e;
          tau[i][j] = T(2) * mu * e + (i == j ? lam * tr_d : T(0));
          hd[i][j] = (double)e;
        }
      if constexpr (SPLIT) {
        split::tangent<D>(sq, cp.mu, cp.lam, hd, cpd);  // C^+ e(du)
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) tau[i][j] -= omg * T(cpd[i][j]);
      } else {
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) tau[i][j] *= gdeg;
      }
      const T cphi = (T(1) - kap) * EsP + T(2) * pres * tr_u + gce;
      fval = cphi * dphi;
      if (MODE != MODE_BLOCK) fval += (T(1) - kap) * phi * se + T(2) * pres * phi * tr_d;
#pragma unroll
      for (int j = 0; j < D; ++j) zeta[j] *= gcx;
    }
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
}

}  // namespace pff
