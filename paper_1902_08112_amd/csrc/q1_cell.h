// Per-cell Q1 operator math shared by the single-instance and batched cell loops.
//
// Displacement part: out[c][a] = sum_q g(phi~) sigma(du) : grad(N_a e_c) JxW.
// Phase-field part: out[a] = sum_q [f(q) N_a + G_c eps grad dphi . grad N_a] JxW with
// f = ((1-kappa) E_s(u) + 2 p div u + G_c/eps) dphi [+ (1-kappa) phi sigma(u):e(du) + 2 p phi div du]
// (the Jacobian of the semi-linear form, Sec. 2.3, with the factor 1/2 of the
// phase-field equation read literally).  Sum-factorized with q1_math.h.
#pragma once

#include "common.h"
#include "q1_math.h"

namespace pff {

using q1::grad2;
using q1::grad2T;
using q1::grad3;
using q1::grad3T;
using q1::val2;
using q1::val2T;
using q1::val3;
using q1::val3T;

template <typename T>
struct Consts {
  T mu, lam, kap, pres, gce, gcx, jxw, ih[3];
  __device__ Consts(const CellParams& cp, int nq) {
    mu = T(cp.mu);
    lam = T(cp.lam);
    kap = T(cp.kappa);
    pres = T(cp.pres);
    gce = T(cp.gc_over_eps);
    gcx = T(cp.gc_eps);
    jxw = T(cp.vol / nq);
    ih[0] = T(cp.inv_h[0]);
    ih[1] = T(cp.inv_h[1]);
    ih[2] = T(cp.inv_h[2]);
  }
};

// ----------------------------------------------------------------------------------- 3D
// displacement rows of one cell: out[c][a] = sum_q g(phi~) sigma(du):grad(N_a e_c) JxW
template <typename T>
__device__ __forceinline__ void cell3_u(const Consts<T>& k, const T du[3][8], const T pt[8], T out[3][8]) {
  T G[3][3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c) grad3(du[c], k.ih, G[c]);
  T pq[8];
  val3(pt, pq);
  T P[3][3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[c][j][r] = T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int qx = q & 1, qy = (q >> 1) & 1, qz = q >> 2;
    const int r0 = qy + 2 * qz, r1 = qx + 2 * qz, r2 = qx + 2 * qy;
    const T g00 = G[0][0][r0], g01 = G[0][1][r1], g02 = G[0][2][r2];
    const T g10 = G[1][0][r0], g11 = G[1][1][r1], g12 = G[1][2][r2];
    const T g20 = G[2][0][r0], g21 = G[2][1][r1], g22 = G[2][2][r2];
    const T gw = ((T(1) - k.kap) * pq[q] * pq[q] + k.kap) * k.jxw;
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
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int a = 0; a < 8; ++a) out[c][a] = T(0);
    grad3T(P[c], k.ih, out[c]);
  }
}

// phase-field rows: out[a] = sum_q [f(q) N_a + G_c eps grad dphi . grad N_a] JxW
// f = ((1-kappa) E_s(u) + 2 p div u + G_c/eps) dphi [+ (1-kappa) phi sigma(u):e(du) + 2 p phi div du]
template <typename T, bool COUPLE>
__device__ __forceinline__ void cell3_phi(const Consts<T>& k, const T du[3][8], const T dp[8], const T uu[3][8],
                                          const T ph[8], T out[8]) {
  T Gu[3][3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c) grad3(uu[c], k.ih, Gu[c]);
  T Gd[3][3][4];
  T pv[8];
  if (COUPLE) {
#pragma unroll
    for (int c = 0; c < 3; ++c) grad3(du[c], k.ih, Gd[c]);
    val3(ph, pv);
  }
  T dv[8];
  val3(dp, dv);
  T fv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int qx = q & 1, qy = (q >> 1) & 1, qz = q >> 2;
    const int r0 = qy + 2 * qz, r1 = qx + 2 * qz, r2 = qx + 2 * qy;
    const T e00 = Gu[0][0][r0], e11 = Gu[1][1][r1], e22 = Gu[2][2][r2];
    const T e01 = T(0.5) * (Gu[0][1][r1] + Gu[1][0][r0]);
    const T e02 = T(0.5) * (Gu[0][2][r2] + Gu[2][0][r0]);
    const T e12 = T(0.5) * (Gu[1][2][r2] + Gu[2][1][r1]);
    const T tru = e00 + e11 + e22;
    const T ee = e00 * e00 + e11 * e11 + e22 * e22 + T(2) * (e01 * e01 + e02 * e02 + e12 * e12);
    const T Es = T(0.5) * k.lam * tru * tru + k.mu * ee;
    const T cphi = (T(1) - k.kap) * Es + T(2) * k.pres * tru + k.gce;
    T f = cphi * dv[q];
    if (COUPLE) {
      const T d00 = Gd[0][0][r0], d11 = Gd[1][1][r1], d22 = Gd[2][2][r2];
      const T d01 = T(0.5) * (Gd[0][1][r1] + Gd[1][0][r0]);
      const T d02 = T(0.5) * (Gd[0][2][r2] + Gd[2][0][r0]);
      const T d12 = T(0.5) * (Gd[1][2][r2] + Gd[2][1][r1]);
      const T trd = d00 + d11 + d22;
      const T eed = e00 * d00 + e11 * d11 + e22 * d22 + T(2) * (e01 * d01 + e02 * d02 + e12 * d12);
      const T sde = T(2) * k.mu * eed + k.lam * tru * trd;
      f += pv[q] * ((T(1) - k.kap) * sde + T(2) * k.pres * trd);
    }
    fv[q] = f * k.jxw;
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) out[a] = T(0);
  val3T(fv, out);
  T Gp[3][4];
  grad3(dp, k.ih, Gp);
  const T s = T(2) * k.gcx * k.jxw;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) Gp[j][r] *= s;
  grad3T(Gp, k.ih, out);
}

// ----------------------------------------------------------------------------------- 2D
template <typename T>
__device__ __forceinline__ void cell2_u(const Consts<T>& k, const T du[2][4], const T pt[4], T out[2][4]) {
  T G[2][2][2];
  grad2(du[0], k.ih, G[0]);
  grad2(du[1], k.ih, G[1]);
  T pq[4];
  val2(pt, pq);
  T P[2][2][2] = {{{T(0), T(0)}, {T(0), T(0)}}, {{T(0), T(0)}, {T(0), T(0)}}};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int qx = q & 1, qy = q >> 1;
    const T g00 = G[0][0][qy], g01 = G[0][1][qx], g10 = G[1][0][qy], g11 = G[1][1][qx];
    const T gw = ((T(1) - k.kap) * pq[q] * pq[q] + k.kap) * k.jxw;
    const T lt = k.lam * (g00 + g11);
    const T s00 = gw * (T(2) * k.mu * g00 + lt), s11 = gw * (T(2) * k.mu * g11 + lt);
    const T s01 = gw * k.mu * (g01 + g10);
    P[0][0][qy] += s00;
    P[0][1][qx] += s01;
    P[1][0][qy] += s01;
    P[1][1][qx] += s11;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int a = 0; a < 4; ++a) out[c][a] = T(0);
    grad2T(P[c], k.ih, out[c]);
  }
}

template <typename T, bool COUPLE>
__device__ __forceinline__ void cell2_phi(const Consts<T>& k, const T du[2][4], const T dp[4], const T uu[2][4],
                                          const T ph[4], T out[4]) {
  T Gu[2][2][2], Gd[2][2][2];
  grad2(uu[0], k.ih, Gu[0]);
  grad2(uu[1], k.ih, Gu[1]);
  T pv[4];
  if (COUPLE) {
    grad2(du[0], k.ih, Gd[0]);
    grad2(du[1], k.ih, Gd[1]);
    val2(ph, pv);
  }
  T dv[4];
  val2(dp, dv);
  T fv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int qx = q & 1, qy = q >> 1;
    const T e00 = Gu[0][0][qy], e11 = Gu[1][1][qx];
    const T e01 = T(0.5) * (Gu[0][1][qx] + Gu[1][0][qy]);
    const T tru = e00 + e11;
    const T Es = T(0.5) * k.lam * tru * tru + k.mu * (e00 * e00 + e11 * e11 + T(2) * e01 * e01);
    const T cphi = (T(1) - k.kap) * Es + T(2) * k.pres * tru + k.gce;
    T f = cphi * dv[q];
    if (COUPLE) {
      const T d00 = Gd[0][0][qy], d11 = Gd[1][1][qx];
      const T d01 = T(0.5) * (Gd[0][1][qx] + Gd[1][0][qy]);
      const T trd = d00 + d11;
      const T sde = T(2) * k.mu * (e00 * d00 + e11 * d11 + T(2) * e01 * d01) + k.lam * tru * trd;
      f += pv[q] * ((T(1) - k.kap) * sde + T(2) * k.pres * trd);
    }
    fv[q] = f * k.jxw;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) out[a] = T(0);
  val2T(fv, out);
  T Gp[2][2];
  grad2(dp, k.ih, Gp);
  const T s = T(2) * k.gcx * k.jxw;
  Gp[0][0] *= s;
  Gp[0][1] *= s;
  Gp[1][0] *= s;
  Gp[1][1] *= s;
  grad2T(Gp, k.ih, out);
}

// ----------------------------------------------------------------------------------- stored coefficients
// Phase-field rows of the block operator B~ (no phi-u coupling) from per-point coefficients
// fixed by the linearization point: cq[q] = ((1-kappa) E_s(u) + 2 p div u + G_c/eps) JxW at
// Gauss point q (the same c_phi as cell3_phi / cell2_phi).  out[a] = sum_q cq[q] dphi(q)
// N_a(q) + the gradient term of cell3_phi / cell2_phi.
template <typename T>
__device__ __forceinline__ void cell3_phi_stored(const Consts<T>& k, const T dp[8], const T cq[8], T out[8]) {
  T dv[8];
  val3(dp, dv);
#pragma unroll
  for (int q = 0; q < 8; ++q) dv[q] *= cq[q];
#pragma unroll
  for (int a = 0; a < 8; ++a) out[a] = T(0);
  val3T(dv, out);
  T Gp[3][4];
  grad3(dp, k.ih, Gp);
  const T s = T(2) * k.gcx * k.jxw;
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) Gp[j][r] *= s;
  grad3T(Gp, k.ih, out);
}

template <typename T>
__device__ __forceinline__ void cell2_phi_stored(const Consts<T>& k, const T dp[4], const T cq[4], T out[4]) {
  T dv[4];
  val2(dp, dv);
#pragma unroll
  for (int q = 0; q < 4; ++q) dv[q] *= cq[q];
#pragma unroll
  for (int a = 0; a < 4; ++a) out[a] = T(0);
  val2T(dv, out);
  T Gp[2][2];
  grad2(dp, k.ih, Gp);
  const T s = T(2) * k.gcx * k.jxw;
  Gp[0][0] *= s;
  Gp[0][1] *= s;
  Gp[1][0] *= s;
  Gp[1][1] *= s;
  grad2T(Gp, k.ih, out);
}

// ----------------------------------------------------------------------------------- residual
// -A(U) on one cell (Sec. 2.3): displacement rows -(g(phi~) sigma(u) + phi~^2 p I) : grad(N_a e_c);
// phase-field rows -[((1-kappa) phi E_s + 2 phi p div u - G_c/eps (1 - phi)) N_a
//                    + G_c eps grad phi . grad N_a]
template <typename T>
__device__ __forceinline__ void cell3_resid(const Consts<T>& k, const T uu[3][8], const T ph[8], const T pt[8],
                                            T outu[3][8], T outp[8]) {
  T G[3][3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c) grad3(uu[c], k.ih, G[c]);
  T pq[8], fq[8];
  val3(pt, pq);
  val3(ph, fq);
  T P[3][3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[c][j][r] = T(0);
  T fv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int qx = q & 1, qy = (q >> 1) & 1, qz = q >> 2;
    const int r0 = qy + 2 * qz, r1 = qx + 2 * qz, r2 = qx + 2 * qy;
    const T g00 = G[0][0][r0], g01 = G[0][1][r1], g02 = G[0][2][r2];
    const T g10 = G[1][0][r0], g11 = G[1][1][r1], g12 = G[1][2][r2];
    const T g20 = G[2][0][r0], g21 = G[2][1][r1], g22 = G[2][2][r2];
    const T tr = g00 + g11 + g22;
    const T e01 = T(0.5) * (g01 + g10), e02 = T(0.5) * (g02 + g20), e12 = T(0.5) * (g12 + g21);
    const T ee = g00 * g00 + g11 * g11 + g22 * g22 + T(2) * (e01 * e01 + e02 * e02 + e12 * e12);
    const T Es = T(0.5) * k.lam * tr * tr + k.mu * ee;
    const T gw = ((T(1) - k.kap) * pq[q] * pq[q] + k.kap) * k.jxw;
    const T dg = gw * k.lam * tr + pq[q] * pq[q] * k.pres * k.jxw;  // diagonal part of g sigma + phi~^2 p I
    const T tm = T(2) * k.mu * gw;
    P[0][0][r0] -= tm * g00 + dg;
    P[1][1][r1] -= tm * g11 + dg;
    P[2][2][r2] -= tm * g22 + dg;
    const T s01 = tm * e01, s02 = tm * e02, s12 = tm * e12;
    P[0][1][r1] -= s01;
    P[1][0][r0] -= s01;
    P[0][2][r2] -= s02;
    P[2][0][r0] -= s02;
    P[1][2][r2] -= s12;
    P[2][1][r1] -= s12;
    const T f = fq[q];
    fv[q] = -((T(1) - k.kap) * f * Es + T(2) * f * k.pres * tr - k.gce * (T(1) - f)) * k.jxw;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int a = 0; a < 8; ++a) outu[c][a] = T(0);
    grad3T(P[c], k.ih, outu[c]);
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) outp[a] = T(0);
  val3T(fv, outp);
  T Gp[3][4];
  grad3(ph, k.ih, Gp);
  const T sg = -T(2) * k.gcx * k.jxw;  // each gradient-table entry stands for two Gauss points
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) Gp[j][r] *= sg;
  grad3T(Gp, k.ih, outp);
}

template <typename T>
__device__ __forceinline__ void cell2_resid(const Consts<T>& k, const T uu[2][4], const T ph[4], const T pt[4],
                                            T outu[2][4], T outp[4]) {
  T G[2][2][2];
  grad2(uu[0], k.ih, G[0]);
  grad2(uu[1], k.ih, G[1]);
  T pq[4], fq[4];
  val2(pt, pq);
  val2(ph, fq);
  T P[2][2][2] = {{{T(0), T(0)}, {T(0), T(0)}}, {{T(0), T(0)}, {T(0), T(0)}}};
  T fv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int qx = q & 1, qy = q >> 1;
    const T g00 = G[0][0][qy], g01 = G[0][1][qx], g10 = G[1][0][qy], g11 = G[1][1][qx];
    const T tr = g00 + g11;
    const T e01 = T(0.5) * (g01 + g10);
    const T Es = T(0.5) * k.lam * tr * tr + k.mu * (g00 * g00 + g11 * g11 + T(2) * e01 * e01);
    const T gw = ((T(1) - k.kap) * pq[q] * pq[q] + k.kap) * k.jxw;
    const T dg = gw * k.lam * tr + pq[q] * pq[q] * k.pres * k.jxw;
    const T tm = T(2) * k.mu * gw;
    P[0][0][qy] -= tm * g00 + dg;
    P[1][1][qx] -= tm * g11 + dg;
    P[0][1][qx] -= tm * e01;
    P[1][0][qy] -= tm * e01;
    const T f = fq[q];
    fv[q] = -((T(1) - k.kap) * f * Es + T(2) * f * k.pres * tr - k.gce * (T(1) - f)) * k.jxw;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int a = 0; a < 4; ++a) outu[c][a] = T(0);
    grad2T(P[c], k.ih, outu[c]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) outp[a] = T(0);
  val2T(fv, outp);
  T Gp[2][2];
  grad2(ph, k.ih, Gp);
  const T sg = -T(2) * k.gcx * k.jxw;
  Gp[0][0] *= sg;
  Gp[0][1] *= sg;
  Gp[1][0] *= sg;
  Gp[1][1] *= sg;
  grad2T(Gp, k.ih, outp);
}

// ----------------------------------------------------------------------------------- diagonal
// diag(G) on one cell, every row: displacement rows sum_q JxW g(phi~) (mu (|grad N_a|^2 + (d_c N_a)^2)
// + lam (d_c N_a)^2); phase-field rows sum_q JxW (c_phi N_a^2 + G_c eps |grad N_a|^2) with
// c_phi = (1-kappa) E_s + 2 p div u + G_c/eps.  N_a at a Gauss point is a product of the 1D
// values XI1 (same side) or XI0 (opposite side); d_j N_a replaces factor j by -+1/h_j.
template <int D, typename T>
__device__ __forceinline__ void cell_diag(const Consts<T>& k, const T (&gw)[D == 3 ? 8 : 4],
                                          const T (&cph)[D == 3 ? 8 : 4], T (&outu)[D][D == 3 ? 8 : 4],
                                          T (&outp)[D == 3 ? 8 : 4]) {
  constexpr int NL = D == 3 ? 8 : 4;
  const T x0 = T(q1::XI0), x1 = T(q1::XI1);
#pragma unroll
  for (int a = 0; a < NL; ++a) {
    T su[D], sp = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) su[c] = T(0);
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      T f[D], dn[D];
#pragma unroll
      for (int j = 0; j < D; ++j) f[j] = (((a >> j) & 1) == ((q >> j) & 1)) ? x1 : x0;
      T n = T(1);
#pragma unroll
      for (int j = 0; j < D; ++j) n *= f[j];
      T g2 = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        T v = k.ih[j];
#pragma unroll
        for (int m = 0; m < D; ++m)
          if (m != j) v *= f[m];
        dn[j] = v;  // |d_j N_a|; the sign squares away
        g2 += v * v;
      }
#pragma unroll
      for (int c = 0; c < D; ++c) su[c] += gw[q] * (k.mu * (g2 + dn[c] * dn[c]) + k.lam * dn[c] * dn[c]);
      sp += cph[q] * n * n + k.gcx * k.jxw * g2;
    }
#pragma unroll
    for (int c = 0; c < D; ++c) outu[c][a] = su[c];
    outp[a] = sp;
  }
}

// Gauss-point coefficients of the diagonal: JxW g(phi~) and JxW c_phi
template <typename T>
__device__ __forceinline__ void cell3_diag_coef(const Consts<T>& k, const T uu[3][8], const T pt[8], T gw[8], T cph[8]) {
  T G[3][3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c) grad3(uu[c], k.ih, G[c]);
  T pq[8];
  val3(pt, pq);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int qx = q & 1, qy = (q >> 1) & 1, qz = q >> 2;
    const int r0 = qy + 2 * qz, r1 = qx + 2 * qz, r2 = qx + 2 * qy;
    const T g00 = G[0][0][r0], g11 = G[1][1][r1], g22 = G[2][2][r2];
    const T e01 = T(0.5) * (G[0][1][r1] + G[1][0][r0]);
    const T e02 = T(0.5) * (G[0][2][r2] + G[2][0][r0]);
    const T e12 = T(0.5) * (G[1][2][r2] + G[2][1][r1]);
    const T tr = g00 + g11 + g22;
    const T ee = g00 * g00 + g11 * g11 + g22 * g22 + T(2) * (e01 * e01 + e02 * e02 + e12 * e12);
    const T Es = T(0.5) * k.lam * tr * tr + k.mu * ee;
    gw[q] = ((T(1) - k.kap) * pq[q] * pq[q] + k.kap) * k.jxw;
    cph[q] = ((T(1) - k.kap) * Es + T(2) * k.pres * tr + k.gce) * k.jxw;
  }
}

template <typename T>
__device__ __forceinline__ void cell2_diag_coef(const Consts<T>& k, const T uu[2][4], const T pt[4], T gw[4], T cph[4]) {
  T G[2][2][2];
  grad2(uu[0], k.ih, G[0]);
  grad2(uu[1], k.ih, G[1]);
  T pq[4];
  val2(pt, pq);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int qx = q & 1, qy = q >> 1;
    const T g00 = G[0][0][qy], g11 = G[1][1][qx];
    const T e01 = T(0.5) * (G[0][1][qx] + G[1][0][qy]);
    const T tr = g00 + g11;
    const T Es = T(0.5) * k.lam * tr * tr + k.mu * (g00 * g00 + g11 * g11 + T(2) * e01 * e01);
    gw[q] = ((T(1) - k.kap) * pq[q] * pq[q] + k.kap) * k.jxw;
    cph[q] = ((T(1) - k.kap) * Es + T(2) * k.pres * tr + k.gce) * k.jxw;
  }
}

// One Q1 cell (corner node g0 of a lattice with strides sy, sz): masked
// Jacobian (COUPLE) or block apply, contributions added atomically to y on
// the free DoFs.  x, U, phit, mask, y are the instance's own arrays.
// part: 0 = both parts, 1 = displacement rows only, 2 = phase-field rows only
template <int D, typename T, bool COUPLE>
__device__ __forceinline__ void q1_cell_atomic(const CellParams& cp, int64_t g0, const T* __restrict__ x,
                                               const T* __restrict__ U, const T* __restrict__ phit,
                                               const uint8_t* __restrict__ mask, T* __restrict__ y,
                                               int part = 0) {
  constexpr int NL = D == 2 ? 4 : 8;
  const int64_t nn = cp.n_nodes, sy = cp.ns[1], sz = cp.ns[2];
  int64_t gi[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) gi[a] = g0 + (a & 1) + ((a >> 1) & 1) * sy + (D == 3 ? (a >> 2) * sz : 0);
  const Consts<T> kc(cp, NL);
  uint8_t mk[NL];
  T du[D][NL], pt[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) {
    mk[a] = mask[gi[a]];
    pt[a] = phit[gi[a]];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const T v = x[c * nn + gi[a]];
      du[c][a] = (mk[a] & (1 << c)) ? T(0) : v;
    }
  }
  if (part != 2) {
    T outu[D][NL];
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
  T dp[NL], uu[D][NL], ph[NL], outp[NL];
#pragma unroll
  for (int a = 0; a < NL; ++a) {
    const T v = x[D * nn + gi[a]];
    dp[a] = (mk[a] & kMaskPhi) ? T(0) : v;
#pragma unroll
    for (int c = 0; c < D; ++c) uu[c][a] = U[c * nn + gi[a]];
    ph[a] = COUPLE ? U[D * nn + gi[a]] : T(0);
  }
  if constexpr (D == 3)
    cell3_phi<T, COUPLE>(kc, du, dp, uu, ph, outp);
  else
    cell2_phi<T, COUPLE>(kc, du, dp, uu, ph, outp);
#pragma unroll
  for (int a = 0; a < NL; ++a)
    if (!(mk[a] & kMaskPhi)) atomicAdd(&y[D * nn + gi[a]], outp[a]);
}

}  // namespace pff
