// Per-node operations on the Q_p node lattice, shared by the single-instance
// (grid.hip) and batched (batch.hip) kernels: Dirichlet/hole masks, nodal
// injection (Sec. 4.2), prolongation and restriction (Sec. 3.2), the
// Gauss-Lobatto lumped mass (Sec. 3.1 remark).  Node-centric gathers.
#pragma once

#include "common.h"

namespace pff {

struct G3 {
  int d, p;
  int N[3], nn[3];
  int64_t ns[3];
  int64_t n_nodes;
  int lshape;
  double h[3];
};

__host__ __device__ inline G3 g3_of(const CellParams& cp) {
  G3 r;
  r.d = cp.d;
  r.p = cp.p;
  for (int k = 0; k < 3; ++k) {
    r.N[k] = cp.N[k];
    r.nn[k] = cp.nn[k];
    r.ns[k] = cp.ns[k];
    r.h[k] = cp.inv_h[k] > 0.0 ? 1.0 / cp.inv_h[k] : 1.0;
  }
  r.n_nodes = cp.n_nodes;
  r.lshape = cp.lshape;
  return r;
}

__device__ inline void node_idx(const G3& g, int64_t i, int idx[3]) {
  idx[0] = (int)(i % g.nn[0]);
  const int64_t r = i / g.nn[0];
  idx[1] = (int)(r % g.nn[1]);
  idx[2] = (int)(r / g.nn[1]);
}

// cells adjacent to lattice index i along one axis and the node's local index in each
__device__ inline int adj_cells(int p, int i, int N, int cell[2], int loc[2]) {
  int m = 0;
  if (p == 1) {
    if (i - 1 >= 0 && i - 1 < N) {
      cell[m] = i - 1;
      loc[m++] = 1;
    }
    if (i < N) {
      cell[m] = i;
      loc[m++] = 0;
    }
  } else {
    if (i & 1) {
      cell[m] = (i - 1) / 2;
      loc[m++] = 1;
    } else {
      if (i / 2 - 1 >= 0) {
        cell[m] = i / 2 - 1;
        loc[m++] = 2;
      }
      if (i / 2 < N) {
        cell[m] = i / 2;
        loc[m++] = 0;
      }
    }
  }
  return m;
}

// Dirichlet face bits (all displacement components) and hole nodes (every component)
__device__ inline uint8_t base_mask_node(const G3& g, unsigned faces, int64_t i) {
  int idx[3];
  node_idx(g, i, idx);
  uint8_t m = 0;
  const uint8_t ubits = (uint8_t)((1 << g.d) - 1);
  for (int k = 0; k < g.d; ++k) {
    if ((faces & (1u << (2 * k))) && idx[k] == 0) m |= ubits;
    if ((faces & (1u << (2 * k + 1))) && idx[k] == g.nn[k] - 1) m |= ubits;
  }
  int cx[2], cy[2], cz[2], l[2];
  const int mx = adj_cells(g.p, idx[0], g.N[0], cx, l);
  const int my = adj_cells(g.p, idx[1], g.N[1], cy, l);
  const int mz = g.d == 3 ? adj_cells(g.p, idx[2], g.N[2], cz, l) : 1;
  bool used = false;
  for (int a = 0; a < mx; ++a)
    for (int b = 0; b < my; ++b)
      for (int c = 0; c < mz; ++c)
        if (!cell_in_hole(g.lshape, cx[a], cy[b], g.N[0], g.N[1])) used = true;
  if (!used) m |= (uint8_t)(ubits | kMaskPhi);
  return m;
}

__device__ inline int64_t inj_fine_index(const G3& c, const G3& f, int64_t j) {
  int idx[3];
  node_idx(c, j, idx);
  int64_t r = 0;
  for (int k = 0; k < c.d; ++k) r += (int64_t)(2 * idx[k]) * f.ns[k];
  return r;
}

// 1D weight of coarse node j in the coarse Q_p interpolant evaluated at fine node f
__device__ inline double w1d(int p, int f, int j, int Nc) {
  if (p == 1) {
    const int e = f - 2 * j;
    return e == 0 ? 1.0 : ((e == 1 || e == -1) ? 0.5 : 0.0);
  }
  int c = f / 4;
  if (c > Nc - 1) c = Nc - 1;
  const int a = j - 2 * c;
  if (a < 0 || a > 2) return 0.0;
  const double t = 0.25 * (double)(f - 4 * c);
  return a == 0 ? 2.0 * (t - 0.5) * (t - 1.0) : (a == 1 ? 4.0 * t * (1.0 - t) : 2.0 * t * (t - 0.5));
}

// out_f[i] (all components) = (add ? out_f : 0) + [mask_f] (P in_c)[i]
template <typename Tin, typename Tout>
__device__ inline void prolong_node(const G3& c, const G3& f, int64_t i, const Tin* in_c, Tout* out_f,
                                    const uint8_t* mask_f, int add) {
  int idx[3];
  node_idx(f, i, idx);
  int js[3][3];
  double ws[3][3];
  int m[3] = {1, 1, 1};
  for (int k = 0; k < 3; ++k) {
    js[k][0] = 0;
    ws[k][0] = 1.0;
  }
  for (int k = 0; k < f.d; ++k) {
    int cnt = 0;
    if (f.p == 1) {
      const int j0 = idx[k] / 2;
      js[k][cnt] = j0;
      ws[k][cnt++] = w1d(1, idx[k], j0, c.N[k]);
      if (idx[k] & 1) {
        js[k][cnt] = j0 + 1;
        ws[k][cnt++] = w1d(1, idx[k], j0 + 1, c.N[k]);
      }
    } else {
      int cc = idx[k] / 4;
      if (cc > c.N[k] - 1) cc = c.N[k] - 1;
      for (int a = 0; a < 3; ++a) {
        const double w = w1d(2, idx[k], 2 * cc + a, c.N[k]);
        if (w != 0.0) {
          js[k][cnt] = 2 * cc + a;
          ws[k][cnt++] = w;
        }
      }
    }
    m[k] = cnt;
  }
  const int d = f.d;
  for (int comp = 0; comp <= d; ++comp) {
    double acc = 0.0;
    for (int a = 0; a < m[0]; ++a)
      for (int b = 0; b < m[1]; ++b)
        for (int e = 0; e < m[2]; ++e) {
          const int64_t jc = js[0][a] * c.ns[0] + js[1][b] * c.ns[1] + (d == 3 ? js[2][e] * c.ns[2] : 0);
          acc += ws[0][a] * ws[1][b] * ws[2][e] * (double)in_c[comp * c.n_nodes + jc];
        }
    const int64_t o = comp * f.n_nodes + i;
    const bool con = mask_f && (mask_f[i] & mask_bit(comp, d));
    const double v = con ? 0.0 : acc;
    out_f[o] = add ? (Tout)((double)out_f[o] + v) : (Tout)v;
  }
}

// out_c[j] (all components) = [mask_c] (P^T in_f)[j]
template <typename Tin, typename Tout>
__device__ inline void restrict_node(const G3& c, const G3& f, int64_t j, const Tin* in_f, Tout* out_c,
                                     const uint8_t* mask_c) {
  int idx[3];
  node_idx(c, j, idx);
  int fs[3][7];
  double ws[3][7];
  int m[3] = {1, 1, 1};
  for (int k = 0; k < 3; ++k) {
    fs[k][0] = 0;
    ws[k][0] = 1.0;
  }
  const int reach = 2 * f.p - 1;
  for (int k = 0; k < f.d; ++k) {
    int cnt = 0;
    for (int o = -reach; o <= reach; ++o) {
      const int fi = 2 * idx[k] + o;
      if (fi < 0 || fi >= f.nn[k]) continue;
      const double w = w1d(f.p, fi, idx[k], c.N[k]);
      if (w != 0.0) {
        fs[k][cnt] = fi;
        ws[k][cnt++] = w;
      }
    }
    m[k] = cnt;
  }
  const int d = f.d;
  for (int comp = 0; comp <= d; ++comp) {
    double acc = 0.0;
    for (int a = 0; a < m[0]; ++a)
      for (int b = 0; b < m[1]; ++b)
        for (int e = 0; e < m[2]; ++e) {
          const int64_t fi = fs[0][a] * f.ns[0] + fs[1][b] * f.ns[1] + (d == 3 ? fs[2][e] * f.ns[2] : 0);
          acc += ws[0][a] * ws[1][b] * ws[2][e] * (double)in_f[comp * f.n_nodes + fi];
        }
    const bool con = mask_c && (mask_c[j] & mask_bit(comp, d));
    out_c[comp * c.n_nodes + j] = (Tout)(con ? 0.0 : acc);
  }
}

// Fixed-shape forms of the two transfers for one (node, component): the 1D
// stencils are unrolled per axis (3 fine nodes per coarse node and axis for
// Q1, 7 for Q2 in restriction; 2 resp. 3 coarse nodes in prolongation) and
// out-of-lattice taps get weight 0 at a clamped, in-bounds address.
template <int P>
__device__ inline void restrict_taps(int ic, int nnf, int Nc, int64_t stride, double w[4 * P - 1],
                                     int64_t off[4 * P - 1]) {
#pragma unroll
  for (int t = 0; t < 4 * P - 1; ++t) {
    const int fi = 2 * ic + t - (2 * P - 1);
    const bool in = fi >= 0 && fi < nnf;
    w[t] = in ? w1d(P, fi, ic, Nc) : 0.0;
    off[t] = in ? (int64_t)fi * stride : 0;
  }
}
template <int P>
__device__ inline void prolong_taps(int fi, int Nc, int64_t stride, double w[P + 1], int64_t off[P + 1]) {
  if constexpr (P == 1) {
    const int j0 = fi >> 1;
    const bool odd = fi & 1;
    w[0] = odd ? 0.5 : 1.0;
    off[0] = (int64_t)j0 * stride;
    w[1] = odd ? 0.5 : 0.0;
    off[1] = (int64_t)(odd ? j0 + 1 : j0) * stride;
  } else {
    int cc = fi / 4;
    if (cc > Nc - 1) cc = Nc - 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      w[a] = w1d(2, fi, 2 * cc + a, Nc);
      off[a] = (int64_t)(2 * cc + a) * stride;
    }
  }
}

// (P^T v) at coarse node j, component comp; v = in_f, or in_f - sub_f (formed in Tin) if sub_f
template <int D, int P, typename Tin>
__device__ inline double restrict_dof(const G3& c, const G3& f, int64_t j, int comp, const Tin* __restrict__ in_f,
                                      const Tin* __restrict__ sub_f = nullptr) {
  constexpr int T = 4 * P - 1;
  int idx[3];
  node_idx(c, j, idx);
  double wx[T], wy[T], wz[T];
  int64_t ox[T], oy[T], oz[T];
  restrict_taps<P>(idx[0], f.nn[0], c.N[0], f.ns[0], wx, ox);
  restrict_taps<P>(idx[1], f.nn[1], c.N[1], f.ns[1], wy, oy);
  if constexpr (D == 3) restrict_taps<P>(idx[2], f.nn[2], c.N[2], f.ns[2], wz, oz);
  const Tin* src = in_f + (int64_t)comp * f.n_nodes;
  const Tin* sub = sub_f ? sub_f + (int64_t)comp * f.n_nodes : nullptr;
  auto val = [&](int64_t k) -> double { return sub ? (double)(Tin)(src[k] - sub[k]) : (double)src[k]; };
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      const double wab = wx[a] * wy[b];
      if constexpr (D == 3) {
#pragma unroll
        for (int e = 0; e < T; ++e)
          if (wab * wz[e] != 0.0) acc += wab * wz[e] * val(ox[a] + oy[b] + oz[e]);
      } else {
        if (wab != 0.0) acc += wab * val(ox[a] + oy[b]);
      }
    }
  return acc;
}

// (P in_c) at fine node i, component comp
template <int D, int P, typename Tin>
__device__ inline double prolong_dof(const G3& c, const G3& f, int64_t i, int comp, const Tin* __restrict__ in_c) {
  constexpr int T = P + 1;
  int idx[3];
  node_idx(f, i, idx);
  double wx[T], wy[T], wz[T];
  int64_t ox[T], oy[T], oz[T];
  prolong_taps<P>(idx[0], c.N[0], c.ns[0], wx, ox);
  prolong_taps<P>(idx[1], c.N[1], c.ns[1], wy, oy);
  if constexpr (D == 3) prolong_taps<P>(idx[2], c.N[2], c.ns[2], wz, oz);
  const Tin* src = in_c + (int64_t)comp * c.n_nodes;
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      const double wab = wx[a] * wy[b];
      if constexpr (D == 3) {
#pragma unroll
        for (int e = 0; e < T; ++e)
          if (wab * wz[e] != 0.0) acc += wab * wz[e] * (double)src[ox[a] + oy[b] + oz[e]];
      } else {
        if (wab != 0.0) acc += wab * (double)src[ox[a] + oy[b]];
      }
    }
  return acc;
}

// lumped mass: sum over adjacent active cells of the product of 1D Gauss-Lobatto weights times h
__device__ inline double lumped_node(const G3& g, int64_t i) {
  int idx[3];
  node_idx(g, i, idx);
  int cx[2], cy[2], cz[2], lx[2], ly[2], lz[2];
  const int mx = adj_cells(g.p, idx[0], g.N[0], cx, lx);
  const int my = adj_cells(g.p, idx[1], g.N[1], cy, ly);
  int mz = 1;
  cz[0] = 0;
  lz[0] = 0;
  if (g.d == 3) mz = adj_cells(g.p, idx[2], g.N[2], cz, lz);
  double acc = 0.0;
  for (int a = 0; a < mx; ++a)
    for (int b = 0; b < my; ++b)
      for (int c = 0; c < mz; ++c) {
        if (cell_in_hole(g.lshape, cx[a], cy[b], g.N[0], g.N[1])) continue;
        auto w = [&](int loc, double h) {
          return g.p == 1 ? 0.5 * h : (loc == 1 ? (4.0 / 6.0) * h : (1.0 / 6.0) * h);
        };
        double v = w(lx[a], g.h[0]) * w(ly[b], g.h[1]);
        if (g.d == 3) v *= w(lz[c], g.h[2]);
        acc += v;
      }
  return acc;
}

}  // namespace pff
