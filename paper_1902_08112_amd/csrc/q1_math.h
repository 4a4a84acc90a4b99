// Sum-factorized Q1 interpolation at the 2-point Gauss points and its adjoint.
//
// On an affine box cell the trilinear (bilinear) interpolant has derivative
// d/dx_j that does not depend on the quadrature coordinate along j, so the
// gradient of a field at the 2^d Gauss points is a table of 2^(d-1) values per
// direction: g[j][r] with r the index over the other coordinates.  Values,
// gradient tables and their transposes cost a few lerps per cell (the
// tensor-product factorization of Sec. 4.1, O(p^{d+1} d^2) per element).
//
// Local numbering: node a = ax + 2 ay (+ 4 az), quadrature point q likewise.
// Gauss points on [0,1]: xi0 = (1 - 1/sqrt 3)/2, xi1 = (1 + 1/sqrt 3)/2.
#pragma once

#include <hip/hip_runtime.h>

namespace pff {
namespace q1 {

constexpr double XI0 = 0.21132486540518711775;
constexpr double XI1 = 0.78867513459481288225;

// values at xi0, xi1 of the linear interpolant through (0, a), (1, b)
template <typename T>
__host__ __device__ __forceinline__ void lerp2(T a, T b, T& o0, T& o1) {
  const T d = b - a;
  o0 = a + T(XI0) * d;
  o1 = a + T(XI1) * d;
}
// adjoint of lerp2: coefficients c0, c1 of the two point values -> coefficients of a, b
template <typename T>
__host__ __device__ __forceinline__ void lerp2T(T c0, T c1, T& a, T& b) {
  a = T(XI1) * c0 + T(XI0) * c1;
  b = T(XI0) * c0 + T(XI1) * c1;
}

// ---------------------------------------------------------------- 3D
// gradient tables: g[0][qy + 2 qz], g[1][qx + 2 qz], g[2][qx + 2 qy]; ih = 1/h
template <typename T>
__host__ __device__ __forceinline__ void grad3(const T f[8], const T ih[3], T g[3][4]) {
  T e[4], t[4];
  // d/dx: edges along x at (ay, az), interpolate in y then z
  for (int r = 0; r < 4; ++r) e[r] = (f[2 * r + 1] - f[2 * r]) * ih[0];  // r = ay + 2 az
  lerp2(e[0], e[1], t[0], t[1]);                                          // az = 0: t[qy]
  lerp2(e[2], e[3], t[2], t[3]);                                          // az = 1: t[2 + qy]
  lerp2(t[0], t[2], g[0][0], g[0][2]);
  lerp2(t[1], t[3], g[0][1], g[0][3]);
  // d/dy: edges along y at (ax, az), interpolate in x then z
  for (int az = 0; az < 2; ++az)
    for (int ax = 0; ax < 2; ++ax) e[ax + 2 * az] = (f[ax + 2 + 4 * az] - f[ax + 4 * az]) * ih[1];
  lerp2(e[0], e[1], t[0], t[1]);
  lerp2(e[2], e[3], t[2], t[3]);
  lerp2(t[0], t[2], g[1][0], g[1][2]);
  lerp2(t[1], t[3], g[1][1], g[1][3]);
  // d/dz: edges along z at (ax, ay), interpolate in x then y
  for (int r = 0; r < 4; ++r) e[r] = (f[r + 4] - f[r]) * ih[2];           // r = ax + 2 ay
  lerp2(e[0], e[1], t[0], t[1]);
  lerp2(e[2], e[3], t[2], t[3]);
  lerp2(t[0], t[2], g[2][0], g[2][2]);
  lerp2(t[1], t[3], g[2][1], g[2][3]);
}

// adjoint of grad3: out[a] += sum_j sum_r P[j][r] * (dN_a/dx_j at r)
template <typename T>
__host__ __device__ __forceinline__ void grad3T(const T P[3][4], const T ih[3], T out[8]) {
  T e[4], t[4];
  lerp2T(P[0][0], P[0][2], t[0], t[2]);
  lerp2T(P[0][1], P[0][3], t[1], t[3]);
  lerp2T(t[0], t[1], e[0], e[1]);
  lerp2T(t[2], t[3], e[2], e[3]);
  for (int r = 0; r < 4; ++r) {
    const T v = e[r] * ih[0];
    out[2 * r + 1] += v;
    out[2 * r] -= v;
  }
  lerp2T(P[1][0], P[1][2], t[0], t[2]);
  lerp2T(P[1][1], P[1][3], t[1], t[3]);
  lerp2T(t[0], t[1], e[0], e[1]);
  lerp2T(t[2], t[3], e[2], e[3]);
  for (int az = 0; az < 2; ++az)
    for (int ax = 0; ax < 2; ++ax) {
      const T v = e[ax + 2 * az] * ih[1];
      out[ax + 2 + 4 * az] += v;
      out[ax + 4 * az] -= v;
    }
  lerp2T(P[2][0], P[2][2], t[0], t[2]);
  lerp2T(P[2][1], P[2][3], t[1], t[3]);
  lerp2T(t[0], t[1], e[0], e[1]);
  lerp2T(t[2], t[3], e[2], e[3]);
  for (int r = 0; r < 4; ++r) {
    const T v = e[r] * ih[2];
    out[r + 4] += v;
    out[r] -= v;
  }
}

// values at the 8 Gauss points, v[qx + 2 qy + 4 qz]
template <typename T>
__host__ __device__ __forceinline__ void val3(const T f[8], T v[8]) {
  T a[8], b[8];
  for (int r = 0; r < 4; ++r) lerp2(f[2 * r], f[2 * r + 1], a[2 * r], a[2 * r + 1]);
  for (int az = 0; az < 2; ++az)
    for (int qx = 0; qx < 2; ++qx) lerp2(a[qx + 4 * az], a[qx + 2 + 4 * az], b[qx + 4 * az], b[qx + 2 + 4 * az]);
  for (int m = 0; m < 4; ++m) lerp2(b[m], b[m + 4], v[m], v[m + 4]);
}
// adjoint of val3: out[a] += sum_q N_a(q) c[q]
template <typename T>
__host__ __device__ __forceinline__ void val3T(const T c[8], T out[8]) {
  T a[8], b[8], f[8];
  for (int m = 0; m < 4; ++m) lerp2T(c[m], c[m + 4], b[m], b[m + 4]);
  for (int az = 0; az < 2; ++az)
    for (int qx = 0; qx < 2; ++qx) lerp2T(b[qx + 4 * az], b[qx + 2 + 4 * az], a[qx + 4 * az], a[qx + 2 + 4 * az]);
  for (int r = 0; r < 4; ++r) lerp2T(a[2 * r], a[2 * r + 1], f[2 * r], f[2 * r + 1]);
  for (int i = 0; i < 8; ++i) out[i] += f[i];
}

// ---------------------------------------------------------------- 2D
// g[0][qy], g[1][qx]
template <typename T>
__host__ __device__ __forceinline__ void grad2(const T f[4], const T ih[2], T g[2][2]) {
  lerp2((f[1] - f[0]) * ih[0], (f[3] - f[2]) * ih[0], g[0][0], g[0][1]);
  lerp2((f[2] - f[0]) * ih[1], (f[3] - f[1]) * ih[1], g[1][0], g[1][1]);
}
template <typename T>
__host__ __device__ __forceinline__ void grad2T(const T P[2][2], const T ih[2], T out[4]) {
  T e0, e1;
  lerp2T(P[0][0], P[0][1], e0, e1);  // e0: edge ay=0, e1: edge ay=1
  e0 *= ih[0];
  e1 *= ih[0];
  out[1] += e0;
  out[0] -= e0;
  out[3] += e1;
  out[2] -= e1;
  lerp2T(P[1][0], P[1][1], e0, e1);  // e0: edge ax=0, e1: edge ax=1
  e0 *= ih[1];
  e1 *= ih[1];
  out[2] += e0;
  out[0] -= e0;
  out[3] += e1;
  out[1] -= e1;
}
template <typename T>
__host__ __device__ __forceinline__ void val2(const T f[4], T v[4]) {
  T a[4];
  lerp2(f[0], f[1], a[0], a[1]);
  lerp2(f[2], f[3], a[2], a[3]);
  lerp2(a[0], a[2], v[0], v[2]);
  lerp2(a[1], a[3], v[1], v[3]);
}
template <typename T>
__host__ __device__ __forceinline__ void val2T(const T c[4], T out[4]) {
  T a[4], f[4];
  lerp2T(c[0], c[2], a[0], a[2]);
  lerp2T(c[1], c[3], a[1], a[3]);
  lerp2T(a[0], a[1], f[0], f[1]);
  lerp2T(a[2], a[3], f[2], f[3]);
  for (int i = 0; i < 4; ++i) out[i] += f[i];
}

}  // namespace q1
}  // namespace pff
