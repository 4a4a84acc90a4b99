// Structured-grid kernels on the Q_p node lattice: Dirichlet/hole masks,
// nodal injection of the linearization point and the active set to coarser
// levels (Sec. 4.2), prolongation P / restriction P^T (Sec. 3.2), the
// Gauss-Lobatto lumped mass (Sec. 3.1 remark) and the active-set decision
// (Algorithm 1 step 3).  All node-centric gathers: deterministic, no atomics.
#include "common.h"

namespace pff {

static inline int64_t nblk(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return b < 1 ? 1 : b;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

struct G3 {
  int d, p;
  int N[3], nn[3];
  int64_t ns[3];
  int64_t n_nodes;
  int lshape;
};
static G3 g3(const Geom& g) {
  G3 r;
  r.d = g.d;
  r.p = g.p;
  for (int k = 0; k < 3; ++k) {
    r.N[k] = g.N[k];
    r.nn[k] = g.nn[k];
    r.ns[k] = g.ns[k];
  }
  r.n_nodes = g.n_nodes;
  r.lshape = g.lshape;
  return r;
}

__device__ inline void node_idx(const G3& g, int64_t i, int idx[3]) {
  idx[0] = (int)(i % g.nn[0]);
  int64_t r = i / g.nn[0];
  idx[1] = (int)(r % g.nn[1]);
  idx[2] = (int)(r / g.nn[1]);
}

// cells adjacent to lattice index i along one axis and the node's local index in each
__device__ inline int adj_cells(int p, int i, int N, int cell[2], int loc[2]) {
  int m = 0;
  if (p == 1) {
    if (i - 1 >= 0 && i - 1 < N) { cell[m] = i - 1; loc[m++] = 1; }
    if (i < N) { cell[m] = i; loc[m++] = 0; }
  } else {
    if (i & 1) {
      cell[m] = (i - 1) / 2; loc[m++] = 1;
    } else {
      if (i / 2 - 1 >= 0) { cell[m] = i / 2 - 1; loc[m++] = 2; }
      if (i / 2 < N) { cell[m] = i / 2; loc[m++] = 0; }
    }
  }
  return m;
}

__global__ void k_base_mask(G3 g, unsigned faces, uint8_t* mask) {
  GRID_STRIDE(i, g.n_nodes) {
    int idx[3];
    node_idx(g, i, idx);
    uint8_t m = 0;
    const uint8_t ubits = (uint8_t)((1 << g.d) - 1);
    for (int k = 0; k < g.d; ++k) {
      if ((faces & (1u << (2 * k))) && idx[k] == 0) m |= ubits;
      if ((faces & (1u << (2 * k + 1))) && idx[k] == g.nn[k] - 1) m |= ubits;
    }
    // hole: no adjacent active cell
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
    mask[i] = m;
  }
}
pf_status build_base_mask(const Geom& g, unsigned faces, uint8_t* mask, hipStream_t s) {
  k_base_mask<<<nblk(g.n_nodes), 256, 0, s>>>(g3(g), faces, mask);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__device__ inline int64_t inj_fine_index(const G3& c, const G3& f, int64_t j) {
  int idx[3];
  node_idx(c, j, idx);
  int64_t r = 0;
  for (int k = 0; k < c.d; ++k) r += (int64_t)(2 * idx[k]) * f.ns[k];
  return r;
}

template <typename T>
__global__ void k_inject(G3 c, G3 f, const T* fine, T* coarse, int ncomp) {
  GRID_STRIDE(j, c.n_nodes) {
    const int64_t fi = inj_fine_index(c, f, j);
    for (int k = 0; k < ncomp; ++k) coarse[k * c.n_nodes + j] = fine[k * f.n_nodes + fi];
  }
}
template <typename T>
pf_status inject(const Geom& gc, const Geom& gf, const T* fine, T* coarse, int ncomp, hipStream_t s) {
  k_inject<T><<<nblk(gc.n_nodes), 256, 0, s>>>(g3(gc), g3(gf), fine, coarse, ncomp);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}
template pf_status inject<double>(const Geom&, const Geom&, const double*, double*, int, hipStream_t);

__global__ void k_inject_mask(G3 c, G3 f, const uint8_t* fine, const uint8_t* base, uint8_t* coarse) {
  GRID_STRIDE(j, c.n_nodes) coarse[j] = (uint8_t)(fine[inj_fine_index(c, f, j)] | base[j]);
}
pf_status inject_mask(const Geom& gc, const Geom& gf, const uint8_t* fine, const uint8_t* base, uint8_t* coarse,
                      hipStream_t s) {
  k_inject_mask<<<nblk(gc.n_nodes), 256, 0, s>>>(g3(gc), g3(gf), fine, base, coarse);
  PFF_CHECK_LAUNCH();
  return PF_OK;
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

// prolongation: per fine node, the coarse nodes of the containing coarse cell
template <typename Tin, typename Tout>
__global__ void k_prolong(G3 c, G3 f, const Tin* in_c, Tout* out_f, const uint8_t* mask_f, int add) {
  GRID_STRIDE(i, f.n_nodes) {
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
}

// restriction P^T: per coarse node, the fine nodes within one coarse cell
template <typename Tin, typename Tout>
__global__ void k_restrict(G3 c, G3 f, const Tin* in_f, Tout* out_c, const uint8_t* mask_c) {
  GRID_STRIDE(j, c.n_nodes) {
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
}

template <typename Tin, typename Tout>
pf_status restrict_vec(const Geom& gc, const Geom& gf, const Tin* in_f, Tout* out_c, const uint8_t* mask_c,
                       hipStream_t s) {
  k_restrict<Tin, Tout><<<nblk(gc.n_nodes), 256, 0, s>>>(g3(gc), g3(gf), in_f, out_c, mask_c);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}
template <typename Tin, typename Tout>
pf_status prolong_vec(const Geom& gc, const Geom& gf, const Tin* in_c, Tout* out_f, const uint8_t* mask_f, int add,
                      hipStream_t s) {
  k_prolong<Tin, Tout><<<nblk(gf.n_nodes), 256, 0, s>>>(g3(gc), g3(gf), in_c, out_f, mask_f, add);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}
#define INST_TR(A, B)                                                                                    \
  template pf_status restrict_vec<A, B>(const Geom&, const Geom&, const A*, B*, const uint8_t*, hipStream_t); \
  template pf_status prolong_vec<A, B>(const Geom&, const Geom&, const A*, B*, const uint8_t*, int, hipStream_t);
INST_TR(double, double)
INST_TR(float, float)
INST_TR(float, double)
INST_TR(double, float)

// lumped mass: sum over adjacent active cells of the product of 1D Gauss-Lobatto weights times h
__global__ void k_lumped_mass(G3 g, double hx, double hy, double hz, double* M) {
  GRID_STRIDE(i, g.n_nodes) {
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
          double v = w(lx[a], hx) * w(ly[b], hy);
          if (g.d == 3) v *= w(lz[c], hz);
          acc += v;
        }
    M[i] = acc;
  }
}
pf_status lumped_mass(const Geom& g, double* M, hipStream_t s) {
  k_lumped_mass<<<nblk(g.n_nodes), 256, 0, s>>>(g3(g), g.h[0], g.h[1], g.d == 3 ? g.h[2] : 1.0, M);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__global__ void k_pdas(int64_t nn, int d, const double* R, const double* U, const double* Uold, const double* M,
                       const uint8_t* base, double c, uint8_t* active, double* v) {
  GRID_STRIDE(i, nn) {
    double val = 0.0;
    uint8_t a = 0;
    if (!(base[i] & kMaskPhi)) {
      const int64_t k = (int64_t)d * nn + i;
      val = R[k] / M[i] + c * (U[k] - Uold[k]);
      a = val > 0.0 ? 1 : 0;
    }
    active[i] = a;
    if (v) v[i] = val;
  }
}
pf_status pdas_decide(const Geom& g, const double* R, const double* U, const double* Uold, const double* M,
                      const uint8_t* base_mask, double c, uint8_t* active, double* v, hipStream_t s) {
  k_pdas<<<nblk(g.n_nodes), 256, 0, s>>>(g.n_nodes, g.d, R, U, Uold, M, base_mask, c, active, v);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__device__ inline double block_sum_g(double v) {
  __shared__ double sh[4];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}
__global__ void k_count(const uint8_t* a, int64_t n, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) acc += a[i] ? 1.0 : 0.0;
  const double b = block_sum_g(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = b;
}
__global__ void k_sum1(const double* partials, int n, double* out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partials[i];
  const double b = block_sum_g(acc);
  if (threadIdx.x == 0) *out = b;
}
pf_status count_bytes(const uint8_t* a, int64_t n, double* d_part, int64_t* h_out, hipStream_t s) {
  int nb = (int)((n + 255) / 256);
  if (nb > kRedMaxBlocks) nb = kRedMaxBlocks;
  if (nb < 1) nb = 1;
  k_count<<<nb, 256, 0, s>>>(a, n, d_part);
  PFF_CHECK_LAUNCH();
  k_sum1<<<1, 256, 0, s>>>(d_part, nb, d_part + 2 * kRedMaxBlocks);
  PFF_CHECK_LAUNCH();
  double h = 0;
  PFF_HIP(hipMemcpyAsync(&h, d_part + 2 * kRedMaxBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
  PFF_HIP(hipStreamSynchronize(s));
  *h_out = (int64_t)h;
  return PF_OK;
}

__global__ void k_combine_mask(const uint8_t* base, const uint8_t* extra, const uint8_t* active, uint8_t* mask,
                               int64_t n) {
  GRID_STRIDE(i, n) {
    uint8_t m = base[i];
    if (extra) m |= extra[i] & 7;
    if (active && active[i]) m |= kMaskPhi;
    mask[i] = m;
  }
}
pf_status combine_mask(const uint8_t* base, const uint8_t* extra, const uint8_t* active, uint8_t* mask, int64_t n,
                       hipStream_t s) {
  k_combine_mask<<<nblk(n), 256, 0, s>>>(base, extra, active, mask, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__global__ void k_lift(int64_t nn, int d, const double* U, const double* Uold, const uint8_t* active, double* dl) {
  const int64_t n = (int64_t)(d + 1) * nn;
  const int64_t nu = (int64_t)d * nn;
  GRID_STRIDE(i, n) {
    double v = 0.0;
    if (i >= nu && active[i - nu]) v = Uold[i] - U[i];
    dl[i] = v;
  }
}
pf_status build_lift(const Geom& g, const double* U, const double* Uold, const uint8_t* active, double* dl,
                     hipStream_t s) {
  k_lift<<<nblk(g.n_dofs), 256, 0, s>>>(g.n_nodes, g.d, U, Uold, active, dl);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__global__ void k_constrain_rhs(int64_t nn, int d, const double* R, const double* t, const double* dl,
                                const uint8_t* mask, double* Rt) {
  const int64_t n = (int64_t)(d + 1) * nn;
  GRID_STRIDE(i, n) {
    const int c = (int)(i / nn);
    const int64_t node = i - (int64_t)c * nn;
    Rt[i] = (mask[node] & mask_bit(c, d)) ? dl[i] : R[i] - (t ? t[i] : 0.0);
  }
}
pf_status constrain_rhs(const Geom& g, const double* R, const double* t, const double* dl, const uint8_t* mask,
                        double* Rt, hipStream_t s) {
  k_constrain_rhs<<<nblk(g.n_dofs), 256, 0, s>>>(g.n_nodes, g.d, R, t, dl, mask, Rt);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

}  // namespace pff
