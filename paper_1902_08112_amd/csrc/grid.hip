// Structured-grid kernels of one instance on the Q_p node lattice: Dirichlet
// and hole masks, nodal injection of the linearization point and the active
// set to coarser levels (Sec. 4.2), prolongation P / restriction P^T
// (Sec. 3.2), the Gauss-Lobatto lumped mass (Sec. 3.1 remark), the active-set
// decision (Algorithm 1 step 3), the lift and the constrained right-hand side
// (step 4).  Node-centric gathers (grid_ops.h): deterministic, no atomics.
#include "grid_ops.h"

namespace pff {

static inline int64_t nblk(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return b < 1 ? 1 : b;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

static G3 g3(const Geom& g) {
  G3 r;
  r.d = g.d;
  r.p = g.p;
  for (int k = 0; k < 3; ++k) {
    r.N[k] = g.N[k];
    r.nn[k] = g.nn[k];
    r.ns[k] = g.ns[k];
    r.h[k] = g.h[k];
  }
  r.n_nodes = g.n_nodes;
  r.lshape = g.lshape;
  return r;
}

__global__ void k_base_mask(G3 g, unsigned faces, uint8_t* mask) {
  GRID_STRIDE(i, g.n_nodes) mask[i] = base_mask_node(g, faces, i);
}
pf_status build_base_mask(const Geom& g, unsigned faces, uint8_t* mask, hipStream_t s) {
  k_base_mask<<<nblk(g.n_nodes), 256, 0, s>>>(g3(g), faces, mask);
  PFF_CHECK_LAUNCH();
  return PF_OK;
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

// one thread per (node, component), node fastest: neighbouring threads read
// neighbouring lattice points of one component block
template <int D, int P, typename Tin, typename Tout>
__global__ void k_prolong(G3 c, G3 f, const Tin* __restrict__ in_c, Tout* __restrict__ out_f,
                          const uint8_t* __restrict__ mask_f, int add) {
  const int64_t n = (int64_t)(D + 1) * f.n_nodes;
  GRID_STRIDE(t, n) {
    const int comp = (int)(t / f.n_nodes);
    const int64_t i = t - (int64_t)comp * f.n_nodes;
    const bool con = mask_f && (mask_f[i] & mask_bit(comp, D));
    if (add) {
      if (!con) out_f[t] = (Tout)((double)out_f[t] + prolong_dof<D, P, Tin>(c, f, i, comp, in_c));
    } else {
      out_f[t] = (Tout)(con ? 0.0 : prolong_dof<D, P, Tin>(c, f, i, comp, in_c));
    }
  }
}
template <int D, int P, typename Tin, typename Tout>
__global__ void k_restrict(G3 c, G3 f, const Tin* __restrict__ in_f, const Tin* __restrict__ sub_f,
                           Tout* __restrict__ out_c, const uint8_t* __restrict__ mask_c) {
  const int64_t n = (int64_t)(D + 1) * c.n_nodes;
  GRID_STRIDE(t, n) {
    const int comp = (int)(t / c.n_nodes);
    const int64_t j = t - (int64_t)comp * c.n_nodes;
    const bool con = mask_c && (mask_c[j] & mask_bit(comp, D));
    out_c[t] = (Tout)(con ? 0.0 : restrict_dof<D, P, Tin>(c, f, j, comp, in_f, sub_f));
  }
}

template <typename Tin, typename Tout>
pf_status restrict_vec(const Geom& gc, const Geom& gf, const Tin* in_f, const Tin* sub_f, Tout* out_c,
                       const uint8_t* mask_c, hipStream_t s) {
  const int64_t n = gc.n_dofs;
  const G3 c = g3(gc), f = g3(gf);
  if (gf.d == 2 && gf.p == 1)
    k_restrict<2, 1, Tin, Tout><<<nblk(n), 256, 0, s>>>(c, f, in_f, sub_f, out_c, mask_c);
  else if (gf.d == 2)
    k_restrict<2, 2, Tin, Tout><<<nblk(n), 256, 0, s>>>(c, f, in_f, sub_f, out_c, mask_c);
  else if (gf.p == 1)
    k_restrict<3, 1, Tin, Tout><<<nblk(n), 256, 0, s>>>(c, f, in_f, sub_f, out_c, mask_c);
  else
    k_restrict<3, 2, Tin, Tout><<<nblk(n), 256, 0, s>>>(c, f, in_f, sub_f, out_c, mask_c);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}
template <typename Tin, typename Tout>
pf_status prolong_vec(const Geom& gc, const Geom& gf, const Tin* in_c, Tout* out_f, const uint8_t* mask_f, int add,
                      hipStream_t s) {
  const int64_t n = gf.n_dofs;
  const G3 c = g3(gc), f = g3(gf);
  if (gf.d == 2 && gf.p == 1)
    k_prolong<2, 1, Tin, Tout><<<nblk(n), 256, 0, s>>>(c, f, in_c, out_f, mask_f, add);
  else if (gf.d == 2)
    k_prolong<2, 2, Tin, Tout><<<nblk(n), 256, 0, s>>>(c, f, in_c, out_f, mask_f, add);
  else if (gf.p == 1)
    k_prolong<3, 1, Tin, Tout><<<nblk(n), 256, 0, s>>>(c, f, in_c, out_f, mask_f, add);
  else
    k_prolong<3, 2, Tin, Tout><<<nblk(n), 256, 0, s>>>(c, f, in_c, out_f, mask_f, add);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}
#define INST_TR(A, B)                                                                                    \
  template pf_status restrict_vec<A, B>(const Geom&, const Geom&, const A*, const A*, B*, const uint8_t*, hipStream_t); \
  template pf_status prolong_vec<A, B>(const Geom&, const Geom&, const A*, B*, const uint8_t*, int, hipStream_t);
INST_TR(double, double)
INST_TR(float, float)
INST_TR(float, double)
INST_TR(double, float)

__global__ void k_lumped_mass(G3 g, double* M) {
  GRID_STRIDE(i, g.n_nodes) M[i] = lumped_node(g, i);
}
pf_status lumped_mass(const Geom& g, double* M, hipStream_t s) {
  k_lumped_mass<<<nblk(g.n_nodes), 256, 0, s>>>(g3(g), M);
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
// number of positions where two byte masks differ (as flags: nonzero = set)
__global__ void k_count_diff(const uint8_t* a, const uint8_t* b, int64_t n, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) acc += ((a[i] != 0) != (b[i] != 0)) ? 1.0 : 0.0;
  const double r = block_sum_g(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}
pf_status count_diff_bytes(const uint8_t* a, const uint8_t* b, int64_t n, double* d_part, int64_t* h_out,
                           hipStream_t s) {
  int nb = (int)((n + 255) / 256);
  if (nb > kRedMaxBlocks) nb = kRedMaxBlocks;
  if (nb < 1) nb = 1;
  k_count_diff<<<nb, 256, 0, s>>>(a, b, n, d_part);
  PFF_CHECK_LAUNCH();
  k_sum1<<<1, 256, 0, s>>>(d_part, nb, d_part + 2 * kRedMaxBlocks);
  PFF_CHECK_LAUNCH();
  double h = 0;
  PFF_HIP(hipMemcpyAsync(&h, d_part + 2 * kRedMaxBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
  PFF_HIP(hipStreamSynchronize(s));
  *h_out = (int64_t)h;
  return PF_OK;
}

// time-lagged extrapolation phi~ = phi_1 + theta (phi_1 - phi_2) (hole nodes: phi_1)
__global__ void k_extrapolate(const double* phi_1, const double* phi_2, double theta, const uint8_t* base,
                              int64_t n, double* out) {
  GRID_STRIDE(i, n) {
    const double a = phi_1[i];
    out[i] = (base[i] & kMaskPhi) ? a : a + theta * (a - phi_2[i]);
  }
}
pf_status extrapolate_phase(const double* phi_1, const double* phi_2, double theta, const uint8_t* base, int64_t n,
                            double* out, hipStream_t s) {
  k_extrapolate<<<nblk(n), 256, 0, s>>>(phi_1, phi_2, theta, base, n, out);
  PFF_CHECK_LAUNCH();
  return PF_OK;
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
