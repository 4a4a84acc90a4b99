// Miehe spectral split of the elastic energy (Sec. 2.1) at one quadrature point.
//
// With the strain e = sum_i lam_i n_i n_i^T (symmetric D x D; in 2D the in-plane
// strain of plane strain, whose out-of-plane eigenvalue 0 adds nothing):
//   E_s^+ = lam/2 <tr e>_+^2 + mu sum_i <lam_i>_+^2
//   sigma^+ = dE_s^+/de = lam <tr e>_+ I + 2 mu e_+,   e_+ = sum_i <lam_i>_+ n_i n_i^T
// and its derivative, applied to a strain increment h,
//   C^+[h] = lam H(tr e) tr(h) I + 2 mu N (F o (N^T h N)) N^T,
// the derivative of the spectral function e -> e_+ (Daleckii-Krein), with F_ij the
// divided difference of <.>_+ at (lam_i, lam_j) and H(lam_i) on a tie.  The step
// H = d<x>_+/dx is taken as 0 at x = 0, and an eigenvalue or tr e within kSnap times
// the spectral radius of e of zero counts as zero (its sign is rounding noise of the
// eigensolver, and the tangent jumps there).  The displacement equation uses
// g sigma^+ + sigma^- = sigma - (1 - g) sigma^+, so its tangent is C - (1 - g) C^+.
//
// Eigenpairs by cyclic Jacobi rotations in FP64 (each rotation zeroes one
// off-diagonal entry with the smaller rotation angle; quadratic convergence),
// a published method written here from its definition.  The arithmetic is FP64
// whatever the type of the surrounding cell loop.
#pragma once

#include <hip/hip_runtime.h>

namespace pff {
namespace split {

constexpr int kJacobiMaxSweeps = 16;
constexpr double kSnap = 1e-13;

__host__ __device__ __forceinline__ double pos(double x) { return x > 0.0 ? x : 0.0; }
__host__ __device__ __forceinline__ double heav(double x) { return x > 0.0 ? 1.0 : 0.0; }
// divided difference of <.>_+ at (a, b); H(a) when a == b.  Both positive: (a-b)/(a-b) = 1
// exactly, both non-positive: 0; only a sign change needs the quotient.
__host__ __device__ __forceinline__ double dd_pos(double a, double b) {
  if (a > 0.0 && b > 0.0) return 1.0;
  if (a <= 0.0 && b <= 0.0) return 0.0;
  return (pos(a) - pos(b)) / (a - b);
}

// one rotation in the (p, q) plane that zeroes A[p][q]; the columns of V collect the rotations
template <int D>
__host__ __device__ __forceinline__ void jacobi_rotate(double (&A)[D][D], double (&V)[D][D], int p, int q) {
  const double apq = A[p][q];
  if (apq == 0.0) return;
  const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
  // t = tan(angle): the root of t^2 + 2 theta t - 1 = 0 of smaller magnitude
  const double at = fabs(theta);
  const double t = at > 1e150 ? 0.5 / theta : copysign(1.0, theta) / (at + sqrt(theta * theta + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
  A[p][p] -= t * apq;
  A[q][q] += t * apq;
  A[p][q] = 0.0;
  A[q][p] = 0.0;
#pragma unroll
  for (int r = 0; r < D; ++r) {
    if (r == p || r == q) continue;
    const double arp = A[r][p], arq = A[r][q];
    A[r][p] = A[p][r] = c * arp - s * arq;
    A[r][q] = A[q][r] = s * arp + c * arq;
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double vkp = V[k][p], vkq = V[k][q];
    V[k][p] = c * vkp - s * vkq;
    V[k][q] = s * vkp + c * vkq;
  }
}

// eigenvalues lam (diagonal of the rotated A) and eigenvectors N (columns) of the symmetric e
template <int D>
__host__ __device__ __forceinline__ void sym_eig(const double (&e)[D][D], double (&lam)[D], double (&N)[D][D]) {
  double A[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      A[i][j] = 0.5 * (e[i][j] + e[j][i]);
      N[i][j] = i == j ? 1.0 : 0.0;
    }
  if constexpr (D == 2) {
    jacobi_rotate<2>(A, N, 0, 1);  // one rotation diagonalizes a 2x2
  } else {
    for (int sw = 0; sw < kJacobiMaxSweeps; ++sw) {
      const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
      const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
      if (off == 0.0 || off <= 1e-40 * dia) break;
      jacobi_rotate<3>(A, N, 0, 1);
      jacobi_rotate<3>(A, N, 0, 2);
      jacobi_rotate<3>(A, N, 1, 2);
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) lam[i] = A[i][i];
}

// What the operators need at one point: eigenpairs, divided differences, H(tr e),
// E_s^+ and sigma^+.
template <int D>
struct QP {
  double lam[D];
  double N[D][D];
  double F[D][D];
  double tr, htr, Es_pos;
  double sig[D][D];
};

// from eigenpairs (tr = tr e as computed by the caller); applies the snap to zero
template <int D>
__host__ __device__ __forceinline__ void finish(QP<D>& s, double mu, double lame) {
  double rad = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) rad = fmax(rad, fabs(s.lam[i]));
  const double tiny = kSnap * rad;
#pragma unroll
  for (int i = 0; i < D; ++i)
    if (fabs(s.lam[i]) <= tiny) s.lam[i] = 0.0;
  if (fabs(s.tr) <= tiny) s.tr = 0.0;
  double lp[D];
  double sl2 = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    lp[i] = pos(s.lam[i]);
    sl2 += lp[i] * lp[i];
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) s.F[i][j] = i == j ? heav(s.lam[i]) : dd_pos(s.lam[i], s.lam[j]);
  const double trp = pos(s.tr);
  s.htr = heav(s.tr);
  s.Es_pos = 0.5 * lame * trp * trp + mu * sl2;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double ep = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) ep += s.N[i][k] * lp[k] * s.N[j][k];
      s.sig[i][j] = 2.0 * mu * ep + (i == j ? lame * trp : 0.0);
    }
}

// the split at a strain e (symmetric part taken)
template <int D>
__host__ __device__ __forceinline__ void eval(const double (&e)[D][D], double mu, double lame, QP<D>& s) {
  sym_eig<D>(e, s.lam, s.N);
  s.tr = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) s.tr += e[i][i];
  finish<D>(s, mu, lame);
}

// out = C^+[h] for a symmetric increment h
template <int D>
__host__ __device__ __forceinline__ void tangent(const QP<D>& s, double mu, double lame, const double (&h)[D][D],
                                                 double (&out)[D][D]) {
  double hN[D][D], ht[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) v += h[i][j] * s.N[j][b];
      hN[i][b] = v;
    }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) v += s.N[i][a] * hN[i][b];
      ht[a][b] = s.F[a][b] * v;  // F o (N^T h N)
    }
  double trh = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) trh += h[i][i];
  const double lt = lame * s.htr * trh;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) v += s.N[i][a] * ht[a][b];
      hN[i][b] = v;
    }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) v += hN[i][b] * s.N[j][b];
      out[i][j] = 2.0 * mu * v + (i == j ? lt : 0.0);
    }
}

// h : C^+[h] for the strain of a displacement test function N_a e_i, h = sym(e_i (x) g)
// with g = grad N_a: lam H tr(h)^2 + 2 mu sum_ab F_ab ht_ab^2, ht = N^T h N
template <int D>
__host__ __device__ __forceinline__ double test_energy(const QP<D>& s, double mu, double lame, int i,
                                                       const double (&g)[D]) {
  double v[D], w[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    v[a] = s.N[i][a];
    double x = 0.0;
#pragma unroll
    for (int m = 0; m < D; ++m) x += s.N[m][a] * g[m];
    w[a] = x;
  }
  double q = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const double ht = 0.5 * (v[a] * w[b] + w[a] * v[b]);
      q += s.F[a][b] * ht * ht;
    }
  return lame * s.htr * g[i] * g[i] + 2.0 * mu * q;
}

}  // namespace split
}  // namespace pff
