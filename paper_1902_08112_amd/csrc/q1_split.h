// Q1 cell operator with the Miehe split from stored per-point eigen-data.
//
// The split's tangent at the linearization point (split.h) depends on e(u) at each
// Gauss point only, which is fixed during a Newton step, so the eigenpairs are
// computed once per linearization (k_split_data) and every apply reads them:
// per point tr e, the eigenvalues (snapped as in split.h) and the eigenvectors as
// a unit quaternion (3D) or the first eigenvector (2D).  Layout of a level's
// record: value k of point q of lattice cell c at [(k * NQ + q) * n_cells + c]
// (consecutive cells adjacent: the loads of a wavefront are contiguous).
//
// Displacement rows: tau = C e(du) - (1 - g(phi~)) C^+ e(du), C^+ h = lam H(tr e) tr h I
// + 2 mu N (F o (N^T h N)) N^T.  Phase-field rows: E_s^+ and sigma^+ : e(du) from the
// eigenvalues, sigma^+ : h = lam <tr e>_+ tr h + 2 mu sum_i <lam_i>_+ n_i . h n_i.
//
// Since C h = lam tr h I + 2 mu N (1 o (N^T h N)) N^T for the orthonormal N, the displacement
// tangent is formed as one spectral sum with the weights g F + (1 - F) and g H + (1 - H),
// each in [g, 1]: no difference of two O(|C|) terms.  Written as C h - (1 - g) C^+ h, a fully
// broken point in tension (g = kappa, F = H = 1) is kappa |C h| left over from cancelling
// terms, which FP32 rounding (1e-7 |C h|) swamps: the FP32 operator's rows there turn
// indefinite, 100-1000 times the true diagonal, and the Chebyshev smoother, whose interval
// comes from the FP64 operator, amplifies them without bound.
#pragma once

#include "common.h"
#include "q1_math.h"
#include "split.h"

namespace pff {
namespace q1s {

template <int D>
struct Layout {
  static constexpr int NQ = D == 3 ? 8 : 4;
  static constexpr int NV = D == 3 ? 8 : 5;  // values per point
  // value slots
  static constexpr int TR = 0;               // tr e
  static constexpr int LAM = 1;              // eigenvalues: LAM .. LAM + D - 1
  static constexpr int ROT = 1 + D;          // 3D: quaternion (w, x, y, z); 2D: first eigenvector (c, s)
};

// rotation matrix (columns = eigenvectors) from a unit quaternion (w, x, y, z)
template <typename T>
__host__ __device__ __forceinline__ void quat_to_rot(T w, T x, T y, T z, T (&R)[3][3]) {
  R[0][0] = T(1) - T(2) * (y * y + z * z);
  R[0][1] = T(2) * (x * y - z * w);
  R[0][2] = T(2) * (x * z + y * w);
  R[1][0] = T(2) * (x * y + z * w);
  R[1][1] = T(1) - T(2) * (x * x + z * z);
  R[1][2] = T(2) * (y * z - x * w);
  R[2][0] = T(2) * (x * z - y * w);
  R[2][1] = T(2) * (y * z + x * w);
  R[2][2] = T(1) - T(2) * (x * x + y * y);
}

// unit quaternion of a rotation matrix (Shepperd's method: the largest of the four
// squared components is taken from the diagonal, the others from off-diagonal sums)
__host__ __device__ __forceinline__ void rot_to_quat(const double (&R)[3][3], double (&q)[4]) {
  const double t = R[0][0] + R[1][1] + R[2][2];
  double w, x, y, z;
  if (t > R[0][0] && t > R[1][1] && t > R[2][2]) {
    const double s = 2.0 * sqrt(fmax(1.0 + t, 0.0));
    w = 0.25 * s;
    x = (R[2][1] - R[1][2]) / s;
    y = (R[0][2] - R[2][0]) / s;
    z = (R[1][0] - R[0][1]) / s;
  } else if (R[0][0] >= R[1][1] && R[0][0] >= R[2][2]) {
    const double s = 2.0 * sqrt(fmax(1.0 + R[0][0] - R[1][1] - R[2][2], 0.0));
    w = (R[2][1] - R[1][2]) / s;
    x = 0.25 * s;
    y = (R[0][1] + R[1][0]) / s;
    z = (R[0][2] + R[2][0]) / s;
  } else if (R[1][1] >= R[2][2]) {
    const double s = 2.0 * sqrt(fmax(1.0 + R[1][1] - R[0][0] - R[2][2], 0.0));
    w = (R[0][2] - R[2][0]) / s;
    x = (R[0][1] + R[1][0]) / s;
    y = 0.25 * s;
    z = (R[1][2] + R[2][1]) / s;
  } else {
    const double s = 2.0 * sqrt(fmax(1.0 + R[2][2] - R[0][0] - R[1][1], 0.0));
    w = (R[1][0] - R[0][1]) / s;
    x = (R[0][2] + R[2][0]) / s;
    y = (R[1][2] + R[2][1]) / s;
    z = 0.25 * s;
  }
  const double n = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  q[0] = w * n;
  q[1] = x * n;
  q[2] = y * n;
  q[3] = z * n;
}

// the stored record of one point from its strain (FP64): v[0..NV)
template <int D>
__host__ __device__ __forceinline__ void point_record(const double (&e)[D][D], double mu, double lame,
                                                      double (&v)[Layout<D>::NV]) {
  using Lt = Layout<D>;
  split::QP<D> s;
  split::eval<D>(e, mu, lame, s);
  v[Lt::TR] = s.tr;
#pragma unroll
  for (int i = 0; i < D; ++i) v[Lt::LAM + i] = s.lam[i];
  if constexpr (D == 3) {
    double N[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) N[i][j] = s.N[i][j];
    // a product of plane rotations is proper; guard the sign anyway
    const double det = N[0][0] * (N[1][1] * N[2][2] - N[1][2] * N[2][1]) -
                       N[0][1] * (N[1][0] * N[2][2] - N[1][2] * N[2][0]) +
                       N[0][2] * (N[1][0] * N[2][1] - N[1][1] * N[2][0]);
    if (det < 0.0)
#pragma unroll
      for (int i = 0; i < 3; ++i) N[i][2] = -N[i][2];
    double q[4];
    rot_to_quat(N, q);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[Lt::ROT + k] = q[k];
  } else {
    v[Lt::ROT] = s.N[0][0];
    v[Lt::ROT + 1] = s.N[1][0];
  }
}

// eigenvectors (columns) of a stored record
template <int D, typename T>
__host__ __device__ __forceinline__ void record_rot(const T* v, T (&N)[D][D]) {
  using Lt = Layout<D>;
  if constexpr (D == 3) {
    quat_to_rot<T>(v[Lt::ROT], v[Lt::ROT + 1], v[Lt::ROT + 2], v[Lt::ROT + 3], N);
  } else {
    const T c = v[Lt::ROT], s = v[Lt::ROT + 1];
    N[0][0] = c;
    N[1][0] = s;
    N[0][1] = -s;
    N[1][1] = c;
  }
}

template <typename T>
__host__ __device__ __forceinline__ T tpos(T x) { return x > T(0) ? x : T(0); }
template <typename T>
__host__ __device__ __forceinline__ T theav(T x) { return x > T(0) ? T(1) : T(0); }
template <typename T>
__host__ __device__ __forceinline__ T tdd(T a, T b) {
  if (a > T(0) && b > T(0)) return T(1);
  if (a <= T(0) && b <= T(0)) return T(0);
  return (tpos(a) - tpos(b)) / (a - b);
}

// tau = C h - (1 - g) C^+ h for the symmetric increment h (of the displacement direction), as
// lam w(H) tr h I + 2 mu N (w(F) o (N^T h N)) N^T with w(f) = g f + (1 - f)
template <int D, typename T>
__host__ __device__ __forceinline__ void split_stress(T mu, T lam, T g, const T* v, const T (&h)[D][D],
                                                      T (&tau)[D][D]) {
  using Lt = Layout<D>;
  T N[D][D];
  record_rot<D, T>(v, N);
  T l[D];
#pragma unroll
  for (int i = 0; i < D; ++i) l[i] = v[Lt::LAM + i];
  const T tre = v[Lt::TR];
  T hN[D][D], M[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T x = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) x += h[i][j] * N[j][b];
      hN[i][b] = x;
    }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a; b < D; ++b) {
      T x = T(0);
#pragma unroll
      for (int i = 0; i < D; ++i) x += N[i][a] * hN[i][b];
      const T f = a == b ? theav(l[a]) : tdd(l[a], l[b]);
      M[a][b] = (g * f + (T(1) - f)) * x;
      M[b][a] = M[a][b];
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T x = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) x += N[i][a] * M[a][b];
      hN[i][b] = x;  // N M
    }
  T trh = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) trh += h[i][i];
  const T ht = theav(tre);
  const T ltp = lam * (g * ht + (T(1) - ht)) * trh;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      T x = T(0);
#pragma unroll
      for (int b = 0; b < D; ++b) x += hN[i][b] * N[j][b];
      tau[i][j] = T(2) * mu * x + (i == j ? ltp : T(0));
      tau[j][i] = tau[i][j];
    }
}

// E_s^+ at a point from its record
template <int D, typename T>
__host__ __device__ __forceinline__ T split_energy(T mu, T lam, const T* v) {
  using Lt = Layout<D>;
  const T trp = tpos(v[Lt::TR]);
  T s = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const T p = tpos(v[Lt::LAM + i]);
    s += p * p;
  }
  return T(0.5) * lam * trp * trp + mu * s;
}

// sigma^+ : h at a point from its record
template <int D, typename T>
__host__ __device__ __forceinline__ T split_stress_dot(T mu, T lam, const T* v, const T (&h)[D][D]) {
  using Lt = Layout<D>;
  T N[D][D];
  record_rot<D, T>(v, N);
  T trh = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) trh += h[i][i];
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const T p = tpos(v[Lt::LAM + a]);
    T q = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      T hn = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) hn += h[i][j] * N[j][a];
      q += N[i][a] * hn;
    }
    acc += p * q;
  }
  return lam * tpos(v[Lt::TR]) * trh + T(2) * mu * acc;
}

}  // namespace q1s
}  // namespace pff

namespace pff {
namespace q1s {

// constants of one cell (affine box): Lame, kappa, pressure, G_c/eps, G_c eps, JxW, 1/h
template <typename T>
struct CK {
  T mu, lam, kap, pres, gce, gcx, jxw, ih[3];
  __host__ __device__ CK(const CellParams& cp, int nq) {
    mu = T(cp.mu);
    lam = T(cp.lam);
    kap = T(cp.kappa);
    pres = T(cp.pres);
    gce = T(cp.gc_over_eps);
    gcx = T(cp.gc_eps);
    jxw = T(cp.vol / nq);
    for (int k = 0; k < 3; ++k) ih[k] = T(cp.inv_h[k]);
  }
};

// load the record of point q of a cell: rb = record base + cell index, stride = n_cells
template <int D, typename T>
__host__ __device__ __forceinline__ void load_record(const T* __restrict__ rb, int64_t stride, int q, T (&v)[Layout<D>::NV],
                                                     bool with_rot) {
  using Lt = Layout<D>;
#pragma unroll
  for (int k = 0; k < Lt::NV; ++k) {
    if (!with_rot && k >= Lt::ROT) {
      v[k] = T(0);
      continue;
    }
    v[k] = rb[(int64_t)(k * Lt::NQ + q) * stride];
  }
}

// ---------------------------------------------------------------------------- 3D
// displacement rows: out[c][a] = sum_q tau(q) : grad(N_a e_c) JxW with the split tangent
template <typename T>
__host__ __device__ __forceinline__ void cell3_u(const CK<T>& k, const T (&du)[3][8], const T (&pt)[8],
                                                 const T* __restrict__ rb, int64_t stride, T (&out)[3][8]) {
  T G[3][3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c) q1::grad3(du[c], k.ih, G[c]);
  T pq[8];
  q1::val3(pt, pq);
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
    const int rj[3] = {qy + 2 * qz, qx + 2 * qz, qx + 2 * qy};
    T h[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) h[i][j] = T(0.5) * (G[i][j][rj[j]] + G[j][i][rj[i]]);
    T v[Layout<3>::NV];
    load_record<3, T>(rb, stride, q, v, true);
    const T gq = k.kap + (T(1) - k.kap) * pq[q] * pq[q];  // g(phi~)
    T tau[3][3];
    split_stress<3, T>(k.mu, k.lam, gq, v, h, tau);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < 3; ++j) P[c][j][rj[j]] += k.jxw * tau[c][j];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int a = 0; a < 8; ++a) out[c][a] = T(0);
    q1::grad3T(P[c], k.ih, out[c]);
  }
}

// phase-field rows: f(q) = ((1-kappa) E_s^+ + 2 p tr e + G_c/eps) dphi
//                          [+ (1-kappa) phi sigma^+ : e(du) + 2 p phi div du], + G_c eps grad dphi . grad psi
template <typename T, bool COUPLE>
__host__ __device__ __forceinline__ void cell3_phi(const CK<T>& k, const T (&du)[3][8], const T (&dp)[8],
                                                   const T (&ph)[8], const T* __restrict__ rb, int64_t stride,
                                                   T (&out)[8]) {
  T Gd[3][3][4];
  T pv[8];
  if (COUPLE) {
#pragma unroll
    for (int c = 0; c < 3; ++c) q1::grad3(du[c], k.ih, Gd[c]);
    q1::val3(ph, pv);
  }
  T dv[8];
  q1::val3(dp, dv);
  T fv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    T v[Layout<3>::NV];
    load_record<3, T>(rb, stride, q, v, COUPLE);
    const T cphi = (T(1) - k.kap) * split_energy<3, T>(k.mu, k.lam, v) + T(2) * k.pres * v[Layout<3>::TR] + k.gce;
    T f = cphi * dv[q];
    if (COUPLE) {
      const int qx = q & 1, qy = (q >> 1) & 1, qz = q >> 2;
      const int rj[3] = {qy + 2 * qz, qx + 2 * qz, qx + 2 * qy};
      T h[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) h[i][j] = T(0.5) * (Gd[i][j][rj[j]] + Gd[j][i][rj[i]]);
      const T trd = h[0][0] + h[1][1] + h[2][2];
      f += pv[q] * ((T(1) - k.kap) * split_stress_dot<3, T>(k.mu, k.lam, v, h) + T(2) * k.pres * trd);
    }
    fv[q] = f * k.jxw;
  }
#pragma unroll
  for (int a = 0; a < 8; ++a) out[a] = T(0);
  q1::val3T(fv, out);
  T Gp[3][4];
  q1::grad3(dp, k.ih, Gp);
  const T s = T(2) * k.gcx * k.jxw;  // each gradient-table entry stands for two Gauss points
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) Gp[j][r] *= s;
  q1::grad3T(Gp, k.ih, out);
}

// ---------------------------------------------------------------------------- 2D
template <typename T>
__host__ __device__ __forceinline__ void cell2_u(const CK<T>& k, const T (&du)[2][4], const T (&pt)[4],
                                                 const T* __restrict__ rb, int64_t stride, T (&out)[2][4]) {
  T G[2][2][2];
  q1::grad2(du[0], k.ih, G[0]);
  q1::grad2(du[1], k.ih, G[1]);
  T pq[4];
  q1::val2(pt, pq);
  T P[2][2][2] = {{{T(0), T(0)}, {T(0), T(0)}}, {{T(0), T(0)}, {T(0), T(0)}}};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int qx = q & 1, qy = q >> 1;
    const int rj[2] = {qy, qx};
    T h[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) h[i][j] = T(0.5) * (G[i][j][rj[j]] + G[j][i][rj[i]]);
    T v[Layout<2>::NV];
    load_record<2, T>(rb, stride, q, v, true);
    const T gq = k.kap + (T(1) - k.kap) * pq[q] * pq[q];  // g(phi~)
    T tau[2][2];
    split_stress<2, T>(k.mu, k.lam, gq, v, h, tau);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 2; ++j) P[c][j][rj[j]] += k.jxw * tau[c][j];
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int a = 0; a < 4; ++a) out[c][a] = T(0);
    q1::grad2T(P[c], k.ih, out[c]);
  }
}

template <typename T, bool COUPLE>
__host__ __device__ __forceinline__ void cell2_phi(const CK<T>& k, const T (&du)[2][4], const T (&dp)[4],
                                                   const T (&ph)[4], const T* __restrict__ rb, int64_t stride,
                                                   T (&out)[4]) {
  T Gd[2][2][2];
  T pv[4];
  if (COUPLE) {
    q1::grad2(du[0], k.ih, Gd[0]);
    q1::grad2(du[1], k.ih, Gd[1]);
    q1::val2(ph, pv);
  }
  T dv[4];
  q1::val2(dp, dv);
  T fv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T v[Layout<2>::NV];
    load_record<2, T>(rb, stride, q, v, COUPLE);
    const T cphi = (T(1) - k.kap) * split_energy<2, T>(k.mu, k.lam, v) + T(2) * k.pres * v[Layout<2>::TR] + k.gce;
    T f = cphi * dv[q];
    if (COUPLE) {
      const int qx = q & 1, qy = q >> 1;
      const int rj[2] = {qy, qx};
      T h[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) h[i][j] = T(0.5) * (Gd[i][j][rj[j]] + Gd[j][i][rj[i]]);
      const T trd = h[0][0] + h[1][1];
      f += pv[q] * ((T(1) - k.kap) * split_stress_dot<2, T>(k.mu, k.lam, v, h) + T(2) * k.pres * trd);
    }
    fv[q] = f * k.jxw;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) out[a] = T(0);
  q1::val2T(fv, out);
  T Gp[2][2];
  q1::grad2(dp, k.ih, Gp);
  const T s = T(2) * k.gcx * k.jxw;
  Gp[0][0] *= s;
  Gp[0][1] *= s;
  Gp[1][0] *= s;
  Gp[1][1] *= s;
  q1::grad2T(Gp, k.ih, out);
}

// the record of every Gauss point of one cell from the nodal displacements uc[c][a] (FP64)
template <int D>
__host__ __device__ __forceinline__ void cell_records(const CellParams& cp, const double (&uc)[D][D == 3 ? 8 : 4],
                                                      int q, double (&v)[Layout<D>::NV]) {
  const double ih[3] = {cp.inv_h[0], cp.inv_h[1], cp.inv_h[2]};
  double e[D][D];
  if constexpr (D == 3) {
    double G[3][3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c) q1::grad3(uc[c], ih, G[c]);
    const int qx = q & 1, qy = (q >> 1) & 1, qz = q >> 2;
    const int rj[3] = {qy + 2 * qz, qx + 2 * qz, qx + 2 * qy};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) e[i][j] = 0.5 * (G[i][j][rj[j]] + G[j][i][rj[i]]);
  } else {
    double G[2][2][2];
    q1::grad2(uc[0], ih, G[0]);
    q1::grad2(uc[1], ih, G[1]);
    const int rj[2] = {q >> 1, q & 1};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) e[i][j] = 0.5 * (G[i][j][rj[j]] + G[j][i][rj[i]]);
  }
  point_record<D>(e, cp.mu, cp.lam, v);
}

}  // namespace q1s
}  // namespace pff
