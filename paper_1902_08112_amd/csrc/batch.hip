// Batched solver: many independent instances (each with its own mesh size,
// material, crack and linearization point; common dim, degree and level count)
// advanced by one Newton/active-set step together.
//
// Level data are packed level-major: for each level, the instances' vectors
// (component-major blocks over each instance's own node lattice) are
// concatenated.  Per-instance geometry and material records and prefix
// offsets (DoFs, nodes, cells) live in device memory; every stage is one
// grid-stride launch over the (instance, cell) or (instance, DoF/node) index
// space of the whole batch, the instance found by binary search over the
// offsets.  So a V-cycle costs the same number of launches for 1 or 1000
// instances, the chip is filled by the union of the instances, and no stage
// waits for the host (the V-cycle is graph-capturable).  Per-instance scalars
// (Chebyshev coefficients, CG and Arnoldi coefficients) are device arrays.
// FGMRES advances all unconverged instances in lockstep with per-instance
// Hessenberg matrices on the host; each instance stops at its own tolerance.
//
// The Q1 cell loop also runs from a per-level work table of (instance, tile) items
// (pf_batch_autotune picks the shape per level, precision and operator): one launch per
// stage whose workgroups loop over the table, each item one marching tile of one instance
// (the single-instance bodies of q1_tiles.h, no atomics) or 64 consecutive cells of one
// instance with atomic scatter.  The instance of an item is uniform across its workgroup,
// so its geometry and material come through scalar loads, with no per-cell search.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "generic_cell.h"
#include "grid_ops.h"
#include "q1_cell.h"
#include "q1_tiles.h"

namespace pff {

struct BInst {
  CellParams cp;
  int64_t dof_off, node_off, cell_off;
  unsigned faces;
};

struct BView {
  const BInst* inst;
  const int64_t* dof_off;   // B+1
  const int64_t* node_off;  // B+1
  const int64_t* cell_off;  // B+1
  int B, d, p;
  int split;  // PF_SPLIT_MIEHE: every mode evaluates the split on the fly (generic cell math, FP64)
  int64_t n_dofs, n_nodes, n_cells;
};

__device__ inline int find_seg(const int64_t* off, int B, int64_t i) {
  int lo = 0, hi = B;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

#define GSTRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

static inline int64_t bgrid(int64_t n, int bs = 256) {
  int64_t b = (n + bs - 1) / bs;
  if (b > 65536) b = 65536;
  return b < 1 ? 1 : b;
}

// ---------------------------------------------------------------------------- cell loop
template <int D, int P, typename T, int MODE, bool SPLIT>
__global__ __launch_bounds__(128) void k_b_cell(BView v, const T* __restrict__ x, const T* __restrict__ U,
                                                const T* __restrict__ phit, const uint8_t* __restrict__ mask,
                                                T* __restrict__ y) {
  for (int64_t gc = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gc < v.n_cells;
       gc += (int64_t)gridDim.x * blockDim.x) {
    const int b = find_seg(v.cell_off, v.B, gc);
    const CellParams cp = v.inst[b].cp;
    const int64_t lc = gc - v.cell_off[b];
    const int cx = (int)(lc % cp.N[0]);
    const int cy = (int)((lc / cp.N[0]) % cp.N[1]);
    const int cz = D == 3 ? (int)(lc / ((int64_t)cp.N[0] * cp.N[1])) : 0;
    if (cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) continue;
    const int64_t dof = v.dof_off[b], node = v.node_off[b];
    const T* xo = x ? x + dof : nullptr;
    const T* Uo = U + dof;
    const T* po = phit + node;
    const uint8_t* mo = mask + node;
    T* yo = y + dof;
    if constexpr (!SPLIT && P == 1 && (MODE == MODE_APPLY || MODE == MODE_BLOCK)) {
      const int64_t g0 = (int64_t)cx + (int64_t)cy * cp.ns[1] + (int64_t)cz * cp.ns[2];
      q1_cell_atomic<D, T, MODE == MODE_APPLY>(cp, g0, xo, Uo, po, mo, yo);
    } else {
      using TT = Tens<D, P>;
      constexpr int NL = TT::NL;
      constexpr bool kDir = (MODE == MODE_APPLY || MODE == MODE_BLOCK || MODE == MODE_RAW);
      constexpr bool kMasked = (MODE == MODE_APPLY || MODE == MODE_BLOCK);
      const int c3[3] = {cx, cy, cz};
      const int64_t nn = cp.n_nodes;
      int64_t g[NL];
#pragma unroll
      for (int a = 0; a < NL; ++a) {
        int64_t w = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) w += (int64_t)(P * c3[k] + TT::idx(a, k)) * cp.ns[k];
        g[a] = w;
      }
      // the split is evaluated in FP64 whatever the storage type
      using TC = typename std::conditional<SPLIT, double, T>::type;
      TC xv[D + 1][NL], uv[D + 1][NL], pv[NL];
      uint8_t mk[NL];
#pragma unroll
      for (int a = 0; a < NL; ++a) {
        mk[a] = kMasked ? mo[g[a]] : 0;
        pv[a] = (TC)po[g[a]];
#pragma unroll
        for (int i = 0; i <= D; ++i) {
          uv[i][a] = (TC)Uo[i * nn + g[a]];
          const TC val = kDir ? (TC)xo[i * nn + g[a]] : TC(0);
          xv[i][a] = (kMasked && (mk[a] & mask_bit(i, D))) ? TC(0) : val;
        }
      }
      TC out[D + 1][NL];
      generic_cell<D, P, TC, MODE, SPLIT>(cp, xv, uv, pv, out);
#pragma unroll
      for (int a = 0; a < NL; ++a)
#pragma unroll
        for (int i = 0; i <= D; ++i) {
          if (kMasked && (mk[a] & mask_bit(i, D))) continue;
          atomicAdd(&yo[i * nn + g[a]], (T)out[i][a]);
        }
    }
  }
}

template <int D, int P, typename T, bool SPLIT>
static pf_status b_cell_dps(const BView& v, int mode, const T* x, const T* U, const T* phit, const uint8_t* mask,
                            T* y, hipStream_t s) {
  const int64_t nb = bgrid(v.n_cells, 128);
  switch (mode) {
    case MODE_APPLY:
      k_b_cell<D, P, T, MODE_APPLY, SPLIT><<<nb, 128, 0, s>>>(v, x, U, phit, mask, y);
      break;
    case MODE_BLOCK:
      k_b_cell<D, P, T, MODE_BLOCK, SPLIT><<<nb, 128, 0, s>>>(v, x, U, phit, mask, y);
      break;
    default:
      if constexpr (std::is_same<T, double>::value) {
        if (mode == MODE_RAW)
          k_b_cell<D, P, T, MODE_RAW, SPLIT><<<nb, 128, 0, s>>>(v, x, U, phit, mask, y);
        else if (mode == MODE_RESID)
          k_b_cell<D, P, T, MODE_RESID, SPLIT><<<nb, 128, 0, s>>>(v, x, U, phit, mask, y);
        else
          k_b_cell<D, P, T, MODE_DIAG, SPLIT><<<nb, 128, 0, s>>>(v, x, U, phit, mask, y);
      } else {
        set_error("FP32 batched cell loop supports the apply modes only");
        return PF_ERR_UNSUPPORTED;
      }
  }
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <int D, int P, typename T>
static pf_status b_cell_dp(const BView& v, int mode, const T* x, const T* U, const T* phit, const uint8_t* mask,
                           T* y, hipStream_t s) {
  return v.split ? b_cell_dps<D, P, T, true>(v, mode, x, U, phit, mask, y, s)
                 : b_cell_dps<D, P, T, false>(v, mode, x, U, phit, mask, y, s);
}

template <typename T>
static pf_status b_cell(const BView& v, int mode, const T* x, const T* U, const T* phit, const uint8_t* mask, T* y,
                        hipStream_t s) {
  if (v.d == 2 && v.p == 1) return b_cell_dp<2, 1, T>(v, mode, x, U, phit, mask, y, s);
  if (v.d == 2 && v.p == 2) return b_cell_dp<2, 2, T>(v, mode, x, U, phit, mask, y, s);
  if (v.d == 3 && v.p == 1) return b_cell_dp<3, 1, T>(v, mode, x, U, phit, mask, y, s);
  return b_cell_dp<3, 2, T>(v, mode, x, U, phit, mask, y, s);
}

// ---------------------------------------------------------------------------- work-table cell loop
// Shapes of a work item (kBShape*): 64 consecutive cells of one instance with atomic scatter into y
// preset to Pi_C x; a 3D 8x8 or 16x4 marching tile / 2D 64-cell marching row of one instance
// (every node written once).  items[w] = {instance, tile index within the instance}; the
// workgroups loop over the table (a grid of at most kBItemsGrid workgroups).
constexpr int kBShapeAtomic = 2, kBShapeMarch = 0, kBShapeMarch16 = 1;
constexpr int kBItemsGrid = 4096;

template <int D, typename T, int MODE, int SHAPE>
__global__ __launch_bounds__(64) void k_b_items(BView v, const int2* __restrict__ items, int n_items, int zc,
                                                const T* __restrict__ x, const T* __restrict__ U,
                                                const T* __restrict__ phit, const uint8_t* __restrict__ mask,
                                                T* __restrict__ y) {
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const int2 it = items[w];
    const int b = it.x, tl = it.y;
    const CellParams cp = v.inst[b].cp;
    const int64_t dof = v.dof_off[b], node = v.node_off[b];
    const T* xo = x + dof;
    const T* Uo = U + dof;
    const T* po = phit + node;
    const uint8_t* mo = mask + node;
    T* yo = y + dof;
    if constexpr (SHAPE == kBShapeAtomic) {
      const int64_t lc = (int64_t)tl * 64 + threadIdx.x;
      if (lc < cp.n_cells) {
        const int cx = (int)(lc % cp.N[0]);
        const int cy = (int)((lc / cp.N[0]) % cp.N[1]);
        const int cz = D == 3 ? (int)(lc / ((int64_t)cp.N[0] * cp.N[1])) : 0;
        if (!cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1])) {
          const int64_t g0 = (int64_t)cx + (int64_t)cy * cp.ns[1] + (int64_t)cz * cp.ns[2];
          q1_cell_atomic<D, T, MODE == MODE_APPLY>(cp, g0, xo, Uo, po, mo, yo);
        }
      }
    } else if constexpr (D == 3) {
      constexpr int TX = SHAPE == kBShapeMarch16 ? 16 : 8, TY = 64 / TX;
      const int ntx = (cp.nn[0] + TX - 2) / (TX - 1);
      const int nzc = (cp.nn[2] + zc - 1) / zc;
      const int bz = tl % nzc, bx = (tl / nzc) % ntx, by = tl / (nzc * ntx);
      q1_tile3<T, MODE, TX, TY, false, false>(cp, zc, bx, by, bz, xo, Uo, po, mo, yo, ChebFuse<T>{});
    } else {
      const int nyc = (cp.nn[1] + zc - 1) / zc;
      q1_tile2<T, MODE, false>(cp, zc, tl / nyc, tl % nyc, xo, Uo, po, mo, yo);
    }
  }
}

// items of one instance for a shape (and chunk zc of the marching shapes)
static int64_t b_items_of(const CellParams& cp, int d, int shape, int zc) {
  if (shape == kBShapeAtomic) return (cp.n_cells + 63) / 64;
  if (d == 3) {
    const int tx = shape == kBShapeMarch16 ? 16 : 8, ty = 64 / tx;
    return (int64_t)((cp.nn[0] + tx - 2) / (tx - 1)) * ((cp.nn[1] + ty - 2) / (ty - 1)) * ((cp.nn[2] + zc - 1) / zc);
  }
  return (int64_t)q1_tiles2(cp.nn[0]) * ((cp.nn[1] + zc - 1) / zc);
}

template <int D, typename T, int SHAPE>
static pf_status b_items_launch(const BView& v, int mode, const int2* items, int n, int zc, const T* x, const T* U,
                                const T* phit, const uint8_t* mask, T* y, hipStream_t s) {
  const int grid = std::min(n, kBItemsGrid);
  if (mode == MODE_APPLY)
    k_b_items<D, T, MODE_APPLY, SHAPE><<<grid, 64, 0, s>>>(v, items, n, zc, x, U, phit, mask, y);
  else
    k_b_items<D, T, MODE_BLOCK, SHAPE><<<grid, 64, 0, s>>>(v, items, n, zc, x, U, phit, mask, y);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <typename T>
static pf_status b_items(const BView& v, int mode, int shape, const int2* items, int n, int zc, const T* x,
                         const T* U, const T* phit, const uint8_t* mask, T* y, hipStream_t s) {
  if (n <= 0) return PF_OK;
  if (v.d == 3) {
    if (shape == kBShapeAtomic) return b_items_launch<3, T, kBShapeAtomic>(v, mode, items, n, zc, x, U, phit, mask, y, s);
    if (shape == kBShapeMarch16) return b_items_launch<3, T, kBShapeMarch16>(v, mode, items, n, zc, x, U, phit, mask, y, s);
    return b_items_launch<3, T, kBShapeMarch>(v, mode, items, n, zc, x, U, phit, mask, y, s);
  }
  if (shape == kBShapeAtomic) return b_items_launch<2, T, kBShapeAtomic>(v, mode, items, n, zc, x, U, phit, mask, y, s);
  return b_items_launch<2, T, kBShapeMarch>(v, mode, items, n, zc, x, U, phit, mask, y, s);
}

// ---------------------------------------------------------------------------- DoF-wise kernels
struct Dec {
  int b, c;
  int64_t node;  // instance-local node
};
__device__ inline Dec decode(const BView& v, int64_t i) {
  Dec r;
  r.b = find_seg(v.dof_off, v.B, i);
  const int64_t j = i - v.dof_off[r.b];
  const int64_t nn = v.node_off[r.b + 1] - v.node_off[r.b];
  r.c = (int)(j / nn);
  r.node = j - (int64_t)r.c * nn;
  return r;
}

template <typename T>
__global__ void k_b_init_constrained(BView v, T* y, const T* x, const uint8_t* mask) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    const bool con = mask[v.node_off[e.b] + e.node] & mask_bit(e.c, v.d);
    y[i] = (con && x) ? x[i] : T(0);
  }
}
template <typename T>
__global__ void k_b_set_constrained(BView v, T* y, T val, const uint8_t* mask) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    if (mask[v.node_off[e.b] + e.node] & mask_bit(e.c, v.d)) y[i] = val;
  }
}
template <typename Tin, typename Tout>
__global__ void k_b_mask_free(BView v, Tout* y, const Tin* x, const uint8_t* mask) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    y[i] = (mask[v.node_off[e.b] + e.node] & mask_bit(e.c, v.d)) ? Tout(0) : (Tout)x[i];
  }
}
__global__ void k_b_jacobi(BView v, double* y, const double* x, const double* diag, const uint8_t* mask) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    y[i] = (mask[v.node_off[e.b] + e.node] & mask_bit(e.c, v.d)) ? 0.0 : x[i] / diag[i];
  }
}
// coef[b*4 + 0..3] = c1 (u), c2 (u), c1 (phi), c2 (phi) of this Chebyshev step
template <typename T>
__global__ void k_b_cheb_step(BView v, T* res, const T* t, T* dv, T* x, const T* diag, const double* coef,
                              int first) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    const int k = e.c < v.d ? 0 : 2;
    const T c1 = (T)coef[4 * e.b + k], c2 = (T)coef[4 * e.b + k + 1];
    T r = res[i];
    T dn;
    if (first) {
      dn = c2 * r / diag[i];
    } else {
      r -= t[i];
      res[i] = r;
      dn = c1 * dv[i] + c2 * r / diag[i];
    }
    dv[i] = dn;
    x[i] += dn;
  }
}
// y += a_b x  (a per instance and block: a[2b] u, a[2b+1] phi)
__global__ void k_b_axpy_blocks(BView v, double* y, const double* x, const double* a) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    y[i] += a[2 * e.b + (e.c < v.d ? 0 : 1)] * x[i];
  }
}
// y = x + beta_b y
__global__ void k_b_xpby_blocks(BView v, double* y, const double* x, const double* beta) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    y[i] = x[i] + beta[2 * e.b + (e.c < v.d ? 0 : 1)] * y[i];
  }
}
__device__ inline uint64_t sm64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// SplitMix64 start vector with the same per-(level, block) streams as a single instance
__global__ void k_b_eig_start(BView v, double* s, const uint8_t* mask, uint64_t seed_u, uint64_t seed_p) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    const int64_t nn = v.node_off[e.b + 1] - v.node_off[e.b];
    const bool phi = e.c >= v.d;
    const uint64_t ctr = (uint64_t)(phi ? e.node : (int64_t)e.c * nn + e.node);
    const uint64_t z = sm64((phi ? seed_p : seed_u) + (ctr + 1ull) * 0x9E3779B97F4A7C15ull);
    const double u = (double)(z >> 11) * 0x1.0p-53;
    s[i] = (mask[v.node_off[e.b] + e.node] & mask_bit(e.c, v.d)) ? 0.0 : 2.0 * u - 1.0;
  }
}
__global__ void k_b_lift(BView v, const double* U, const double* Uold, const uint8_t* active, double* dl) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    dl[i] = (e.c == v.d && active[v.node_off[e.b] + e.node]) ? Uold[i] - U[i] : 0.0;
  }
}
__global__ void k_b_constrain_rhs(BView v, const double* R, const double* t, const double* dl, const uint8_t* mask,
                                  double* Rt) {
  GSTRIDE(i, v.n_dofs) {
    const Dec e = decode(v, i);
    Rt[i] = (mask[v.node_off[e.b] + e.node] & mask_bit(e.c, v.d)) ? dl[i] : R[i] - (t ? t[i] : 0.0);
  }
}
// per-instance scale: y = x / sqrt(nrm2[b])  (0 where the norm is 0)
__global__ void k_b_scale_inv_sqrt(BView v, double* y, const double* x, const double* nrm2) {
  GSTRIDE(i, v.n_dofs) {
    const int b = find_seg(v.dof_off, v.B, i);
    const double nr = sqrt(nrm2[b]);
    y[i] = nr > 0.0 ? x[i] / nr : 0.0;
  }
}
// w += sign * sum_i h[i*B + b] V_i  (per-instance coefficients)
__global__ void k_b_multi_axpy(BView v, double* w, const double* V, int64_t ld, int k, const double* h,
                               double sign) {
  GSTRIDE(t, v.n_dofs) {
    const int b = find_seg(v.dof_off, v.B, t);
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += h[(int64_t)i * v.B + b] * V[(int64_t)i * ld + t];
    w[t] += sign * acc;
  }
}

// ---------------------------------------------------------------------------- node kernels
__global__ void k_b_base_mask(BView v, uint8_t* mask) {
  GSTRIDE(i, v.n_nodes) {
    const int b = find_seg(v.node_off, v.B, i);
    const BInst& in = v.inst[b];
    mask[i] = base_mask_node(g3_of(in.cp), in.faces, i - v.node_off[b]);
  }
}
__global__ void k_b_lumped(BView v, double* M) {
  GSTRIDE(i, v.n_nodes) {
    const int b = find_seg(v.node_off, v.B, i);
    M[i] = lumped_node(g3_of(v.inst[b].cp), i - v.node_off[b]);
  }
}
// coarse <- fine nodal injection; ncomp == 1: node-indexed field, else DoF-indexed vector
__global__ void k_b_inject(BView vc, BView vf, const double* fine, double* coarse, int ncomp) {
  GSTRIDE(i, vc.n_nodes) {
    const int b = find_seg(vc.node_off, vc.B, i);
    const G3 c = g3_of(vc.inst[b].cp), f = g3_of(vf.inst[b].cp);
    const int64_t j = i - vc.node_off[b];
    const int64_t fi = inj_fine_index(c, f, j);
    if (ncomp == 1) {
      coarse[vc.node_off[b] + j] = fine[vf.node_off[b] + fi];
    } else {
      for (int k = 0; k < ncomp; ++k)
        coarse[vc.dof_off[b] + k * c.n_nodes + j] = fine[vf.dof_off[b] + k * f.n_nodes + fi];
    }
  }
}
__global__ void k_b_inject_mask(BView vc, BView vf, const uint8_t* fine, const uint8_t* base, uint8_t* coarse) {
  GSTRIDE(i, vc.n_nodes) {
    const int b = find_seg(vc.node_off, vc.B, i);
    const G3 c = g3_of(vc.inst[b].cp), f = g3_of(vf.inst[b].cp);
    const int64_t j = i - vc.node_off[b];
    coarse[i] = (uint8_t)(fine[vf.node_off[b] + inj_fine_index(c, f, j)] | base[i]);
  }
}
template <typename Tin, typename Tout>
__global__ void k_b_restrict(BView vc, BView vf, const Tin* in_f, Tout* out_c, const uint8_t* mask_c) {
  GSTRIDE(i, vc.n_nodes) {
    const int b = find_seg(vc.node_off, vc.B, i);
    const G3 c = g3_of(vc.inst[b].cp), f = g3_of(vf.inst[b].cp);
    restrict_node<Tin, Tout>(c, f, i - vc.node_off[b], in_f + vf.dof_off[b], out_c + vc.dof_off[b],
                             mask_c ? mask_c + vc.node_off[b] : nullptr);
  }
}
template <typename Tin, typename Tout>
__global__ void k_b_prolong(BView vc, BView vf, const Tin* in_c, Tout* out_f, const uint8_t* mask_f, int add) {
  GSTRIDE(i, vf.n_nodes) {
    const int b = find_seg(vf.node_off, vf.B, i);
    const G3 c = g3_of(vc.inst[b].cp), f = g3_of(vf.inst[b].cp);
    prolong_node<Tin, Tout>(c, f, i - vf.node_off[b], in_c + vc.dof_off[b], out_f + vf.dof_off[b],
                            mask_f ? mask_f + vf.node_off[b] : nullptr, add);
  }
}
__global__ void k_b_pdas(BView v, const double* R, const double* U, const double* Uold, const double* M,
                         const uint8_t* base, double c, uint8_t* active) {
  GSTRIDE(i, v.n_nodes) {
    const int b = find_seg(v.node_off, v.B, i);
    const int64_t node = i - v.node_off[b];
    const int64_t nn = v.node_off[b + 1] - v.node_off[b];
    uint8_t a = 0;
    if (!(base[i] & kMaskPhi)) {
      const int64_t k = v.dof_off[b] + (int64_t)v.d * nn + node;
      a = (R[k] / M[i] + c * (U[k] - Uold[k])) > 0.0 ? 1 : 0;
    }
    active[i] = a;
  }
}

// ---------------------------------------------------------------------------- reductions
__device__ inline double bsum(double v) {
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
// grid (nblk, nseg, nvec): partial of V_k . w over segment s -> partials[((k*nseg)+s)*nblk + blk]
__global__ void k_b_seg_dot(const double* V, int64_t ld, const double* w, const int64_t* lo, const int64_t* hi,
                            double* partials) {
  const int s = blockIdx.y, k = blockIdx.z;
  const double* vk = V + (int64_t)k * ld;
  double acc = 0.0;
  for (int64_t t = lo[s] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < hi[s];
       t += (int64_t)gridDim.x * blockDim.x)
    acc += vk[t] * w[t];
  const double r = bsum(acc);
  if (threadIdx.x == 0) partials[((int64_t)k * gridDim.y + s) * gridDim.x + blockIdx.x] = r;
}
__global__ void k_b_seg_count(const uint8_t* a, const int64_t* off, double* partials) {
  const int s = blockIdx.y;
  double acc = 0.0;
  for (int64_t t = off[s] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < off[s + 1];
       t += (int64_t)gridDim.x * blockDim.x)
    acc += a[t] ? 1.0 : 0.0;
  const double r = bsum(acc);
  if (threadIdx.x == 0) partials[(int64_t)s * gridDim.x + blockIdx.x] = r;
}
__global__ void k_b_rows(const double* partials, int nparts, double* out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partials[(int64_t)blockIdx.x * nparts + i];
  const double r = bsum(acc);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

}  // namespace pff

using namespace pff;

namespace {

constexpr int kSegBlocks = 16;  // blocks per segment in segmented reductions

// autotuner candidates of the batched Q1 cell loop: (shape, chunk); -1 = the grid-stride kernel over
// all cells (also the only shape with the split and on Q2)
static const int kBCand[][2] = {{-1, 0}, {kBShapeAtomic, 0}, {kBShapeMarch, 4}, {kBShapeMarch, 8}, {kBShapeMarch, 16},
                                {kBShapeMarch, 32}, {kBShapeMarch16, 4}, {kBShapeMarch16, 8}, {kBShapeMarch16, 16}};
static const int kBNCand = 9;

struct BLevel {
  std::vector<BInst> h_inst;
  std::vector<int64_t> h_dof, h_node, h_cell;
  BInst* d_inst = nullptr;
  int64_t *d_dof = nullptr, *d_node = nullptr, *d_cell = nullptr;
  int64_t *d_seg2_lo = nullptr, *d_seg2_hi = nullptr;  // 2B segments: u-block, phi-block per instance
  int64_t *d_seg1_lo = nullptr, *d_seg1_hi = nullptr;  // B segments: whole instance vector
  int64_t n_dofs = 0, n_nodes = 0, n_cells = 0;
  double *U = nullptr, *phit = nullptr, *diag = nullptr;
  float *U32 = nullptr, *phit32 = nullptr, *diag32 = nullptr;
  uint8_t *base = nullptr, *mask = nullptr;
  void *vb = nullptr, *vx = nullptr, *vr = nullptr, *vt = nullptr, *vd = nullptr;
  double* d_coef_s = nullptr;  // [cheb_degree][B][4]
  double* d_coef_c = nullptr;  // [coarse_degree][B][4] (level 0)
  std::vector<double> eig;     // [B][4]
  std::vector<double> eig_fix; // [B][4]: bounds fixed by pf_batch_set_eig_bounds (0: estimate)
  // cell-loop shape per [precision][operator] (-1: grid-stride over all cells) with its chunk and
  // work table (items[pi][mi], capacity item_cap each); tune_us: the autotuner's timings
  int shape[2][2] = {{-1, -1}, {-1, -1}};
  int zc[2][2] = {{0, 0}, {0, 0}};
  int n_items[2][2] = {{0, 0}, {0, 0}};
  int2* items[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int64_t item_cap = 0;
  double tune_us[2][2][16] = {};
  int d = 0, p = 0, B = 0;
  int split = PF_SPLIT_NONE;
  BView view() const {
    BView v;
    v.inst = d_inst;
    v.dof_off = d_dof;
    v.node_off = d_node;
    v.cell_off = d_cell;
    v.B = B;
    v.d = d;
    v.p = p;
    v.split = split;
    v.n_dofs = n_dofs;
    v.n_nodes = n_nodes;
    v.n_cells = n_cells;
    return v;
  }
};

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T) + 256;
    return p;
  }
};

}  // namespace

struct pf_batch {
  int B = 0, d = 0, p = 0, L = 0;
  pf_options opt;
  int vprec = PF_F64;
  std::vector<pf_mesh> meshes;
  std::vector<Material> mats;
  std::vector<BLevel> lev;
  double *M = nullptr, *R = nullptr, *dl = nullptr, *Rt = nullptr, *dU = nullptr, *t = nullptr;
  uint8_t *extra = nullptr, *active = nullptr;
  double *V = nullptr, *Z = nullptr;
  double *part = nullptr, *dscal = nullptr;
  double *d_alpha = nullptr, *d_beta = nullptr, *d_y = nullptr;
  bool has_extra = false, has_lin = false;
  std::vector<double> h_coef;  // staging for coefficient uploads (kept alive for async copies)
  // captured batched V-cycle per precision: every coefficient it uses is read from
  // device memory, so one capture stays valid for the lifetime of the batch
  double *vin = nullptr, *vout = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t vgraph[2] = {nullptr, nullptr};
  hipGraphExec_t vexec[2] = {nullptr, nullptr};
  bool use_graphs = true;
  void drop_graphs() {
    for (int k = 0; k < 2; ++k) {
      if (vexec[k]) (void)hipGraphExecDestroy(vexec[k]);
      if (vgraph[k]) (void)hipGraphDestroy(vgraph[k]);
      vexec[k] = nullptr;
      vgraph[k] = nullptr;
    }
  }
  ~pf_batch() {
    for (int k = 0; k < 2; ++k) {
      if (vexec[k]) hipGraphExecDestroy(vexec[k]);
      if (vgraph[k]) hipGraphDestroy(vgraph[k]);
    }
    if (cap_stream) hipStreamDestroy(cap_stream);
  }
};

namespace {

hipStream_t bst(void* s) { return reinterpret_cast<hipStream_t>(s); }

pf_status validate_batch(const pf_mesh* meshes, const double* mats, int n, const pf_options* o) {
  if (!meshes || n < 1 || n > 4096) {
    set_error("need 1 <= n <= 4096 meshes");
    return PF_ERR_INVALID_ARG;
  }
  (void)o;
  for (int b = 0; b < n; ++b) {
    if (meshes[b].dim != meshes[0].dim || meshes[b].degree != meshes[0].degree ||
        meshes[b].n_levels != meshes[0].n_levels) {
      set_error("all instances of a batch need the same dim, degree and n_levels");
      return PF_ERR_INVALID_ARG;
    }
  }
  if (mats) {
    for (int b = 0; b < n; ++b) {
      const double* m = mats + 6 * b;
      const double E = m[0], nu = m[1], Gc = m[2], eps = m[3], kappa = m[4], p = m[5];
      if (!(E > 0.0) || !std::isfinite(E) || !(nu > -1.0 && nu < 0.5) || !(Gc > 0.0) || !std::isfinite(Gc) ||
          !(eps > 0.0) || !std::isfinite(eps) || !(kappa >= 0.0 && kappa < 1.0) || !std::isfinite(p)) {
        set_error("material of instance " + std::to_string(b) + " out of range");
        return PF_ERR_INVALID_ARG;
      }
    }
  }
  return PF_OK;
}

// geometry of instance b on level l (same rules as a single context)
Geom inst_geom(const pf_mesh& m, int l) {
  Geom g;
  std::memset(&g, 0, sizeof(g));
  g.d = m.dim;
  g.p = m.degree;
  const int sh = m.n_levels - 1 - l;
  int64_t stride = 1;
  g.n_cells = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < m.dim) {
      g.N[k] = m.n_cells[k] >> sh;
      g.nn[k] = m.degree * g.N[k] + 1;
      g.h[k] = m.extent[k] / g.N[k];
      g.ext[k] = m.extent[k];
    } else {
      g.N[k] = 1;
      g.nn[k] = 1;
      g.h[k] = 1.0;
      g.ext[k] = 1.0;
    }
    g.ns[k] = stride;
    stride *= g.nn[k];
    g.n_cells *= g.N[k];
  }
  g.n_nodes = stride;
  g.n_dofs = (int64_t)(m.dim + 1) * stride;
  g.lshape = m.domain == PF_LSHAPE;
  return g;
}

size_t bcarve(pf_batch* c, const pf_mesh* meshes, int n, const pf_options& o, char* base,
              const std::vector<Material>* mats) {
  Carver cv{base};
  const int L = meshes[0].n_levels;
  const int d = meshes[0].dim;
  std::vector<BLevel> lev(L);
  for (int l = 0; l < L; ++l) {
    BLevel& bl = lev[l];
    bl.B = n;
    bl.d = d;
    bl.p = meshes[0].degree;
    bl.split = o.stress_split;
    bl.h_dof.assign(n + 1, 0);
    bl.h_node.assign(n + 1, 0);
    bl.h_cell.assign(n + 1, 0);
    bl.h_inst.resize(n);
    for (int b = 0; b < n; ++b) {
      const Geom g = inst_geom(meshes[b], l);
      Material m = mats ? (*mats)[b] : Material{1, 1, 1, 1, 0, 0, PF_SPLIT_NONE};
      bl.h_inst[b].cp = make_cell_params(g, m);
      bl.h_inst[b].faces = meshes[b].dirichlet_faces;
      bl.h_inst[b].dof_off = bl.h_dof[b];
      bl.h_inst[b].node_off = bl.h_node[b];
      bl.h_inst[b].cell_off = bl.h_cell[b];
      bl.h_dof[b + 1] = bl.h_dof[b] + g.n_dofs;
      bl.h_node[b + 1] = bl.h_node[b] + g.n_nodes;
      bl.h_cell[b + 1] = bl.h_cell[b] + g.n_cells;
    }
    bl.n_dofs = bl.h_dof[n];
    bl.n_nodes = bl.h_node[n];
    bl.n_cells = bl.h_cell[n];
    const size_t nd = bl.n_dofs, nn = bl.n_nodes;
    bl.d_inst = cv.take<BInst>(n);
    bl.d_dof = cv.take<int64_t>(n + 1);
    bl.d_node = cv.take<int64_t>(n + 1);
    bl.d_cell = cv.take<int64_t>(n + 1);
    bl.d_seg2_lo = cv.take<int64_t>(2 * n);
    bl.d_seg2_hi = cv.take<int64_t>(2 * n);
    bl.d_seg1_lo = cv.take<int64_t>(n);
    bl.d_seg1_hi = cv.take<int64_t>(n);
    bl.U = cv.take<double>(nd);
    bl.phit = cv.take<double>(nn);
    bl.diag = cv.take<double>(nd);
    bl.U32 = cv.take<float>(nd);
    bl.phit32 = cv.take<float>(nn);
    bl.diag32 = cv.take<float>(nd);
    bl.base = cv.take<uint8_t>(nn);
    bl.mask = cv.take<uint8_t>(nn);
    bl.vb = cv.take<double>(nd);
    bl.vx = cv.take<double>(nd);
    bl.vr = cv.take<double>(nd);
    bl.vt = cv.take<double>(nd);
    bl.vd = cv.take<double>(nd);
    bl.d_coef_s = cv.take<double>((size_t)o.cheb_degree * n * 4);
    bl.d_coef_c = cv.take<double>((size_t)o.coarse_degree * n * 4);
    // work tables: room for the largest table of any autotuner candidate
    int64_t cap = 0;
    if (bl.p == 1) {
      for (int k = 0; k < kBNCand; ++k) {
        if (kBCand[k][0] < 0 || (kBCand[k][0] == kBShapeMarch16 && d != 3)) continue;
        int64_t m = 0;
        for (int b = 0; b < n; ++b) m += b_items_of(bl.h_inst[b].cp, d, kBCand[k][0], kBCand[k][1]);
        cap = std::max(cap, m);
      }
    }
    bl.item_cap = cap;
    for (int pi = 0; pi < 2; ++pi)
      for (int mi = 0; mi < 2; ++mi) bl.items[pi][mi] = cap ? cv.take<int2>((size_t)cap) : nullptr;
    bl.eig.assign(4 * n, 1.0);
    bl.eig_fix.assign(4 * n, 0.0);
  }
  const BLevel& f = lev[L - 1];
  const size_t nd = f.n_dofs, nn = f.n_nodes;
  const int mr = o.gmres_restart;
  double* M = cv.take<double>(nn);
  double* R = cv.take<double>(nd);
  double* dl = cv.take<double>(nd);
  double* Rt = cv.take<double>(nd);
  double* dU = cv.take<double>(nd);
  double* t = cv.take<double>(nd);
  uint8_t* extra = cv.take<uint8_t>(nn);
  uint8_t* active = cv.take<uint8_t>(nn);
  double* V = cv.take<double>((size_t)(mr + 1) * nd);
  double* Z = cv.take<double>((size_t)mr * nd);
  double* part = cv.take<double>((size_t)kSegBlocks * 2 * n * (mr + 2) + 1024);
  double* dscal = cv.take<double>((size_t)4 * n * (mr + 4) + 1024);
  double* alpha = cv.take<double>(2 * n);
  double* beta = cv.take<double>(2 * n);
  double* y = cv.take<double>((size_t)n * mr);
  double* vin = cv.take<double>(nd);
  double* vout = cv.take<double>(nd);
  (void)d;
  if (c) {
    c->lev = lev;
    c->M = M;
    c->R = R;
    c->dl = dl;
    c->Rt = Rt;
    c->dU = dU;
    c->t = t;
    c->extra = extra;
    c->active = active;
    c->V = V;
    c->Z = Z;
    c->part = part;
    c->dscal = dscal;
    c->d_alpha = alpha;
    c->d_beta = beta;
    c->d_y = y;
    c->vin = vin;
    c->vout = vout;
  }
  return cv.off + 256;
}

int blevel_prec(int l, int vprec) { return l == 0 ? PF_F64 : vprec; }

// ---------------------------------------------------------------------------- launch helpers
template <typename T>
pf_status b_init_constrained(const BLevel& bl, T* y, const T* x, hipStream_t s) {
  k_b_init_constrained<T><<<bgrid(bl.n_dofs), 256, 0, s>>>(bl.view(), y, x, bl.mask);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}
template <typename T>
pf_status b_fill(T* y, T v, int64_t n, hipStream_t s) {
  return vec_fill<T>(y, v, n, s);
}

pf_status bapply(pf_batch* c, int l, int prec, int mode, const void* x, void* y, hipStream_t s) {
  BLevel& bl = c->lev[l];
  const BView v = bl.view();
  const int pi = prec == PF_F64 ? 0 : 1;
  if ((mode == MODE_APPLY || mode == MODE_BLOCK) && !bl.split && bl.p == 1 && bl.shape[pi][mode] >= 0) {
    const int sh = bl.shape[pi][mode];
    // marching tiles write every node; one thread per cell adds into Pi_C x
    if (prec == PF_F64) {
      if (sh == kBShapeAtomic) PFF_TRY(b_init_constrained<double>(bl, (double*)y, (const double*)x, s));
      return b_items<double>(v, mode, sh, bl.items[pi][mode], bl.n_items[pi][mode], bl.zc[pi][mode], (const double*)x,
                             bl.U, bl.phit, bl.mask, (double*)y, s);
    }
    if (sh == kBShapeAtomic) PFF_TRY(b_init_constrained<float>(bl, (float*)y, (const float*)x, s));
    return b_items<float>(v, mode, sh, bl.items[pi][mode], bl.n_items[pi][mode], bl.zc[pi][mode], (const float*)x,
                          bl.U32, bl.phit32, bl.mask, (float*)y, s);
  }
  if (prec == PF_F64) {
    if (mode == MODE_APPLY || mode == MODE_BLOCK)
      PFF_TRY(b_init_constrained<double>(bl, (double*)y, (const double*)x, s));
    else
      PFF_TRY(vec_fill<double>((double*)y, 0.0, bl.n_dofs, s));
    PFF_TRY(b_cell<double>(v, mode, (const double*)x, bl.U, bl.phit, bl.mask, (double*)y, s));
    if (mode == MODE_DIAG) {
      k_b_set_constrained<double><<<bgrid(bl.n_dofs), 256, 0, s>>>(v, (double*)y, 1.0, bl.mask);
      PFF_CHECK_LAUNCH();
    }
  } else {
    PFF_TRY(b_init_constrained<float>(bl, (float*)y, (const float*)x, s));
    PFF_TRY(b_cell<float>(v, mode, (const float*)x, bl.U32, bl.phit32, bl.mask, (float*)y, s));
  }
  return PF_OK;
}

// Chebyshev coefficients (three-term recurrence, Sec. 3.2.1) per instance and block
void cheb_coefs(double lo, double hi, int degree, std::vector<double>& c1, std::vector<double>& c2) {
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  c1.assign(degree, 0.0);
  c2.assign(degree, 0.0);
  c2[0] = 1.0 / theta;
  for (int k = 1; k < degree; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    c1[k] = rn * rho;
    c2[k] = 2.0 * rn / delta;
    rho = rn;
  }
}

pf_status upload_cheb(pf_batch* c, hipStream_t s) {
  const pf_options& o = c->opt;
  for (int l = 0; l < c->L; ++l) {
    BLevel& bl = c->lev[l];
    const int deg = l == 0 ? o.coarse_degree : o.cheb_degree;
    c->h_coef.assign((size_t)deg * c->B * 4, 0.0);
    std::vector<double> c1, c2;
    for (int b = 0; b < c->B; ++b)
      for (int blk = 0; blk < 2; ++blk) {
        const double lmin = bl.eig[4 * b + 2 * blk], lmax = bl.eig[4 * b + 2 * blk + 1];
        const double hi = o.cheb_safety * lmax;
        const double lo = l == 0 ? o.coarse_lo_factor * lmin : hi / o.cheb_ratio;
        cheb_coefs(lo, hi, deg, c1, c2);
        for (int k = 0; k < deg; ++k) {
          c->h_coef[((size_t)k * c->B + b) * 4 + 2 * blk] = c1[k];
          c->h_coef[((size_t)k * c->B + b) * 4 + 2 * blk + 1] = c2[k];
        }
      }
    double* dst = l == 0 ? bl.d_coef_c : bl.d_coef_s;
    PFF_HIP(hipMemcpyAsync(dst, c->h_coef.data(), c->h_coef.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PFF_HIP(hipStreamSynchronize(s));
    // the smoother on level 0 is never used; level 0 also needs smoothing coefficients only if L == 1
  }
  return PF_OK;
}

template <typename T>
pf_status bcheb(pf_batch* c, int l, int prec, T* res, T* x, const double* coef, int degree, hipStream_t s) {
  BLevel& bl = c->lev[l];
  T* dv = (T*)bl.vd;
  T* t = (T*)bl.vt;
  const T* diag = prec == PF_F64 ? (const T*)bl.diag : (const T*)bl.diag32;
  for (int k = 0; k < degree; ++k) {
    if (k > 0) PFF_TRY(bapply(c, l, prec, MODE_BLOCK, dv, t, s));
    k_b_cheb_step<T><<<bgrid(bl.n_dofs), 256, 0, s>>>(bl.view(), res, t, dv, x, diag, coef + (size_t)k * c->B * 4,
                                                     k == 0 ? 1 : 0);
    PFF_CHECK_LAUNCH();
  }
  return PF_OK;
}

// residual operator of the V-cycle: G~ (P_full) or the block-diagonal B~ (P_diag), Sec. 3.3
int bcycle_mode(const pf_batch* c) { return c->opt.preconditioner == PF_PREC_DIAG ? MODE_BLOCK : MODE_APPLY; }

template <typename T>
pf_status bsmooth(pf_batch* c, int l, int prec, bool x_zero, hipStream_t s) {
  BLevel& bl = c->lev[l];
  T* bb = (T*)bl.vb;
  T* x = (T*)bl.vx;
  T* r = (T*)bl.vr;
  if (x_zero) {
    PFF_TRY(vec_sub<T>(r, bb, x, bl.n_dofs, s));  // x == 0: r = b
  } else {
    PFF_TRY(bapply(c, l, prec, bcycle_mode(c), x, bl.vt, s));
    PFF_TRY(vec_sub<T>(r, bb, (T*)bl.vt, bl.n_dofs, s));
  }
  return bcheb<T>(c, l, prec, r, x, bl.d_coef_s, c->opt.cheb_degree, s);
}

pf_status bcoarse(pf_batch* c, hipStream_t s) {
  BLevel& bl = c->lev[0];
  double* bb = (double*)bl.vb;
  double* x = (double*)bl.vx;
  double* r = (double*)bl.vr;
  PFF_TRY(vec_fill<double>(x, 0.0, bl.n_dofs, s));
  for (int sw = 0; sw < c->opt.coarse_sweeps; ++sw) {
    if (sw == 0) {
      PFF_TRY(vec_sub<double>(r, bb, x, bl.n_dofs, s));
    } else {
      PFF_TRY(bapply(c, 0, PF_F64, bcycle_mode(c), x, bl.vt, s));
      PFF_TRY(vec_sub<double>(r, bb, (double*)bl.vt, bl.n_dofs, s));
    }
    PFF_TRY(bcheb<double>(c, 0, PF_F64, r, x, bl.d_coef_c, c->opt.coarse_degree, s));
  }
  return PF_OK;
}

template <typename Tf, typename Tc>
pf_status brestrict(pf_batch* c, int l, hipStream_t s) {
  BLevel& f = c->lev[l];
  BLevel& co = c->lev[l - 1];
  k_b_restrict<Tf, Tc><<<bgrid(co.n_nodes), 256, 0, s>>>(co.view(), f.view(), (const Tf*)f.vr, (Tc*)co.vb, co.mask);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}
template <typename Tc, typename Tf>
pf_status bprolong(pf_batch* c, int l, hipStream_t s) {
  BLevel& f = c->lev[l];
  BLevel& co = c->lev[l - 1];
  k_b_prolong<Tc, Tf><<<bgrid(f.n_nodes), 256, 0, s>>>(co.view(), f.view(), (const Tc*)co.vx, (Tf*)f.vx, f.mask, 1);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

pf_status bvcycle_level(pf_batch* c, int l, int vprec, hipStream_t s) {
  if (l == 0) return bcoarse(c, s);
  const int pl = blevel_prec(l, vprec), pc = blevel_prec(l - 1, vprec);
  BLevel& bl = c->lev[l];
  if (pl == PF_F64) {
    PFF_TRY(vec_fill<double>((double*)bl.vx, 0.0, bl.n_dofs, s));
    PFF_TRY(bsmooth<double>(c, l, pl, true, s));
    PFF_TRY(bapply(c, l, pl, bcycle_mode(c), bl.vx, bl.vt, s));
    PFF_TRY(vec_sub<double>((double*)bl.vr, (double*)bl.vb, (double*)bl.vt, bl.n_dofs, s));
    PFF_TRY(pc == PF_F64 ? brestrict<double, double>(c, l, s) : brestrict<double, float>(c, l, s));
  } else {
    PFF_TRY(vec_fill<float>((float*)bl.vx, 0.0f, bl.n_dofs, s));
    PFF_TRY(bsmooth<float>(c, l, pl, true, s));
    PFF_TRY(bapply(c, l, pl, bcycle_mode(c), bl.vx, bl.vt, s));
    PFF_TRY(vec_sub<float>((float*)bl.vr, (float*)bl.vb, (float*)bl.vt, bl.n_dofs, s));
    PFF_TRY(pc == PF_F64 ? brestrict<float, double>(c, l, s) : brestrict<float, float>(c, l, s));
  }
  PFF_TRY(bvcycle_level(c, l - 1, vprec, s));
  if (pl == PF_F64) {
    PFF_TRY(pc == PF_F64 ? bprolong<double, double>(c, l, s) : bprolong<float, double>(c, l, s));
    PFF_TRY(bsmooth<double>(c, l, pl, false, s));
  } else {
    PFF_TRY(pc == PF_F64 ? bprolong<double, float>(c, l, s) : bprolong<float, float>(c, l, s));
    PFF_TRY(bsmooth<float>(c, l, pl, false, s));
  }
  return PF_OK;
}

pf_status bvcycle(pf_batch* c, int vprec, const double* r, double* z, hipStream_t s) {
  BLevel& f = c->lev[c->L - 1];
  const BView v = f.view();
  const int pl = blevel_prec(c->L - 1, vprec);
  if (pl == PF_F64)
    k_b_mask_free<double, double><<<bgrid(f.n_dofs), 256, 0, s>>>(v, (double*)f.vb, r, f.mask);
  else
    k_b_mask_free<double, float><<<bgrid(f.n_dofs), 256, 0, s>>>(v, (float*)f.vb, r, f.mask);
  PFF_CHECK_LAUNCH();
  PFF_TRY(bvcycle_level(c, c->L - 1, vprec, s));
  if (pl == PF_F64)
    k_b_mask_free<double, double><<<bgrid(f.n_dofs), 256, 0, s>>>(v, z, (const double*)f.vx, f.mask);
  else
    k_b_mask_free<float, double><<<bgrid(f.n_dofs), 256, 0, s>>>(v, z, (const float*)f.vx, f.mask);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

pf_status bvcycle_graph(pf_batch* c, int vprec, const double* r, double* z, hipStream_t s) {
  const int k = vprec == PF_F64 ? 0 : 1;
  const int64_t n = c->lev[c->L - 1].n_dofs;
  if (!c->vexec[k]) {
    if (!c->cap_stream) PFF_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    PFF_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const pf_status st = bvcycle(c, vprec, c->vin, c->vout, c->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != PF_OK || e != hipSuccess) {
      if (g) hipGraphDestroy(g);
      if (st == PF_OK) set_error(std::string("batched V-cycle capture: ") + hipGetErrorString(e));
      return st != PF_OK ? st : PF_ERR_DEVICE;
    }
    c->vgraph[k] = g;
    PFF_HIP(hipGraphInstantiate(&c->vexec[k], g, nullptr, nullptr, 0));
  }
  PFF_TRY(vec_copy<double>(c->vin, r, n, s));
  PFF_HIP(hipGraphLaunch(c->vexec[k], s));
  PFF_TRY(vec_copy<double>(z, c->vout, n, s));
  return PF_OK;
}

pf_status bvcycle_any(pf_batch* c, int vprec, const double* r, double* z, hipStream_t s) {
  return c->use_graphs ? bvcycle_graph(c, vprec, r, z, s) : bvcycle(c, vprec, r, z, s);
}

// segmented dots: out[k*nseg + s] = V_k . w over segment s (host copy, synchronizes)
pf_status seg_dots(pf_batch* c, const double* V, int64_t ld, int nvec, const double* w, const int64_t* lo,
                   const int64_t* hi, int nseg, double* d_out, double* h_out, hipStream_t s) {
  dim3 grid(kSegBlocks, nseg, nvec);
  k_b_seg_dot<<<grid, 256, 0, s>>>(V, ld, w, lo, hi, c->part);
  PFF_CHECK_LAUNCH();
  k_b_rows<<<nseg * nvec, 256, 0, s>>>(c->part, kSegBlocks, d_out);
  PFF_CHECK_LAUNCH();
  if (h_out) {
    PFF_HIP(hipMemcpyAsync(h_out, d_out, sizeof(double) * nseg * nvec, hipMemcpyDeviceToHost, s));
    PFF_HIP(hipStreamSynchronize(s));
  }
  return PF_OK;
}

// symmetric tridiagonal eigenvalue by Sturm bisection (k-th smallest)
double tri_eig(const std::vector<double>& a, const std::vector<double>& b, int k) {
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
      q = a[i] - mid - (i ? b[i - 1] * b[i - 1] / q : 0.0);
      if (q == 0.0) q = 1e-300;
      if (q < 0) ++cnt;
    }
    if (cnt > k)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

// lockstep PCG on every instance and block (Sec. 3.2.1), Lanczos tridiagonals per (instance, block)
pf_status bestimate_eigs(pf_batch* c, int l, hipStream_t s) {
  BLevel& bl = c->lev[l];
  const BView v = bl.view();
  const int B = c->B;
  double* r = (double*)bl.vr;
  double* z = (double*)bl.vd;
  double* p = (double*)bl.vb;
  double* Ap = (double*)bl.vt;
  const uint64_t seed = c->opt.eig_seed;
  const uint64_t su = seed + (uint64_t)l * 0x1000003ull, sp = su + 0x10001ull;
  k_b_eig_start<<<bgrid(bl.n_dofs), 256, 0, s>>>(v, r, bl.mask, su, sp);
  PFF_CHECK_LAUNCH();
  k_b_jacobi<<<bgrid(bl.n_dofs), 256, 0, s>>>(v, z, r, bl.diag, bl.mask);
  PFF_CHECK_LAUNCH();
  PFF_TRY(vec_copy<double>(p, z, bl.n_dofs, s));
  const int ns = 2 * B;
  std::vector<double> rz(ns), rz0(ns), pAp(ns), rzn(ns), alpha(ns), beta(ns);
  double* dd = c->dscal;
  PFF_TRY(seg_dots(c, r, 0, 1, z, bl.d_seg2_lo, bl.d_seg2_hi, ns, dd, rz.data(), s));
  rz0 = rz;
  std::vector<char> done(ns);
  for (int k = 0; k < ns; ++k) done[k] = !(rz0[k] > 0);
  std::vector<std::vector<double>> al(ns), be(ns);
  for (int it = 0; it < c->opt.eig_cg_steps; ++it) {
    bool all = true;
    for (int k = 0; k < ns; ++k) {
      if (!done[k] && (rz[k] <= 0.0 || rz[k] <= 1e-24 * rz0[k])) done[k] = 1;
      all = all && done[k];
    }
    if (all) break;
    PFF_TRY(bapply(c, l, PF_F64, MODE_BLOCK, p, Ap, s));
    PFF_TRY(seg_dots(c, p, 0, 1, Ap, bl.d_seg2_lo, bl.d_seg2_hi, ns, dd, pAp.data(), s));
    for (int k = 0; k < ns; ++k) {
      alpha[k] = 0.0;
      if (done[k]) continue;
      if (!(pAp[k] > 0.0)) {
        done[k] = 1;
        continue;
      }
      alpha[k] = rz[k] / pAp[k];
      al[k].push_back(alpha[k]);
    }
    for (int k = 0; k < ns; ++k) alpha[k] = -alpha[k];
    PFF_HIP(hipMemcpyAsync(c->d_alpha, alpha.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
    k_b_axpy_blocks<<<bgrid(bl.n_dofs), 256, 0, s>>>(v, r, Ap, c->d_alpha);
    PFF_CHECK_LAUNCH();
    k_b_jacobi<<<bgrid(bl.n_dofs), 256, 0, s>>>(v, z, r, bl.diag, bl.mask);
    PFF_CHECK_LAUNCH();
    PFF_TRY(seg_dots(c, r, 0, 1, z, bl.d_seg2_lo, bl.d_seg2_hi, ns, dd, rzn.data(), s));
    for (int k = 0; k < ns; ++k) {
      beta[k] = 0.0;
      if (done[k]) continue;
      beta[k] = rzn[k] / rz[k];
      be[k].push_back(beta[k]);
      rz[k] = rzn[k];
    }
    PFF_HIP(hipMemcpyAsync(c->d_beta, beta.data(), sizeof(double) * ns, hipMemcpyHostToDevice, s));
    k_b_xpby_blocks<<<bgrid(bl.n_dofs), 256, 0, s>>>(v, p, z, c->d_beta);
    PFF_CHECK_LAUNCH();
    PFF_HIP(hipStreamSynchronize(s));
  }
  for (int k = 0; k < ns; ++k) {
    const size_t n = al[k].size();
    const int b = k / 2, blk = k % 2;
    if (n == 0) {
      bl.eig[4 * b + 2 * blk] = 1.0;
      bl.eig[4 * b + 2 * blk + 1] = 1.0;
      continue;
    }
    std::vector<double> a(n), off(n > 1 ? n - 1 : 0);
    for (size_t j = 0; j < n; ++j) {
      a[j] = 1.0 / al[k][j] + (j ? be[k][j - 1] / al[k][j - 1] : 0.0);
      if (j + 1 < n) off[j] = std::sqrt(be[k][j]) / al[k][j];
    }
    bl.eig[4 * b + 2 * blk] = tri_eig(a, off, 0);
    bl.eig[4 * b + 2 * blk + 1] = tri_eig(a, off, (int)n - 1);
  }
  for (int b = 0; b < B; ++b)
    if (bl.eig_fix[4 * b] > 0.0)
      for (int k = 0; k < 4; ++k) bl.eig[4 * b + k] = bl.eig_fix[4 * b + k];
  return PF_OK;
}

pf_status bset_linearization(pf_batch* c, const double* U, const double* phit, const uint8_t* active,
                             hipStream_t s) {
  const int L = c->L;
  BLevel& f = c->lev[L - 1];
  PFF_TRY(vec_copy<double>(f.U, U, f.n_dofs, s));
  PFF_TRY(vec_copy<double>(f.phit, phit, f.n_nodes, s));
  PFF_TRY(combine_mask(f.base, c->has_extra ? c->extra : nullptr, active, f.mask, f.n_nodes, s));
  for (int l = L - 2; l >= 0; --l) {
    BLevel& co = c->lev[l];
    BLevel& fi = c->lev[l + 1];
    const int64_t gb = bgrid(co.n_nodes);
    k_b_inject<<<gb, 256, 0, s>>>(co.view(), fi.view(), fi.U, co.U, c->d + 1);
    k_b_inject<<<gb, 256, 0, s>>>(co.view(), fi.view(), fi.phit, co.phit, 1);
    k_b_inject_mask<<<gb, 256, 0, s>>>(co.view(), fi.view(), fi.mask, co.base, co.mask);
    PFF_CHECK_LAUNCH();
  }
  for (int l = 0; l < L; ++l) {
    BLevel& bl = c->lev[l];
    PFF_TRY(bapply(c, l, PF_F64, MODE_DIAG, nullptr, bl.diag, s));
    PFF_TRY(vec_cast<double, float>(bl.U32, bl.U, bl.n_dofs, s));
    PFF_TRY(vec_cast<double, float>(bl.phit32, bl.phit, bl.n_nodes, s));
    PFF_TRY(vec_cast<double, float>(bl.diag32, bl.diag, bl.n_dofs, s));
  }
  for (int l = 0; l < L; ++l) PFF_TRY(bestimate_eigs(c, l, s));
  PFF_TRY(upload_cheb(c, s));
  PFF_HIP(hipStreamSynchronize(s));
  c->has_lin = true;
  return PF_OK;
}

// Lockstep FGMRES(m) with CGS2 for every instance; instance b stops at its own tolerance.
pf_status bfgmres(pf_batch* c, const double* b, double* x, int vprec, std::vector<int>& iters,
                  std::vector<double>& rel, std::vector<double>& bnorm, hipStream_t s) {
  const int L = c->L, B = c->B, m = c->opt.gmres_restart;
  BLevel& f = c->lev[L - 1];
  const BView v = f.view();
  const int64_t n = f.n_dofs;
  double* dd = c->dscal;                   // [0, 4B(m+2)) scratch rows
  double* h1 = dd;                         // [m+1][B]
  double* h2 = dd + (size_t)(m + 1) * B;   // [m+1][B]
  double* nr = dd + (size_t)2 * (m + 1) * B;  // [B]
  std::vector<double> hb(B);
  PFF_TRY(seg_dots(c, b, 0, 1, b, f.d_seg1_lo, f.d_seg1_hi, B, nr, hb.data(), s));
  bnorm.assign(B, 0.0);
  std::vector<double> tol(B);
  for (int i = 0; i < B; ++i) {
    bnorm[i] = std::sqrt(hb[i]);
    tol[i] = std::max(c->opt.gmres_rtol * bnorm[i], c->opt.gmres_atol);
  }
  auto true_res = [&](std::vector<double>& beta) -> pf_status {
    PFF_TRY(bapply(c, L - 1, PF_F64, MODE_APPLY, x, c->t, s));
    PFF_TRY(vec_sub<double>(c->V, b, c->t, n, s));
    std::vector<double> r2(B);
    PFF_TRY(seg_dots(c, c->V, 0, 1, c->V, f.d_seg1_lo, f.d_seg1_hi, B, nr, r2.data(), s));
    beta.resize(B);
    for (int i = 0; i < B; ++i) beta[i] = std::sqrt(r2[i]);
    return PF_OK;
  };
  std::vector<double> beta;
  PFF_TRY(true_res(beta));
  iters.assign(B, 0);
  std::vector<char> conv(B);
  for (int i = 0; i < B; ++i) conv[i] = !(beta[i] > tol[i]);
  int total = 0;
  std::vector<double> H((size_t)B * (m + 1) * m), g((size_t)B * (m + 1)), cs((size_t)B * m), sn((size_t)B * m),
      y((size_t)B * m), hbuf((size_t)2 * (m + 1) * B + B);
  std::vector<int> jend(B);
  auto Hb = [&](int bb, int i, int j) -> double& { return H[((size_t)bb * (m + 1) + i) * m + j]; };
  while (total < c->opt.gmres_max_iter) {
    bool any = false;
    for (int i = 0; i < B; ++i) any = any || !conv[i];
    if (!any) break;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    std::vector<char> active_cycle(B);
    for (int i = 0; i < B; ++i) {
      active_cycle[i] = !conv[i];
      g[(size_t)i * (m + 1)] = beta[i];
      jend[i] = 0;
      hb[i] = beta[i] * beta[i];
    }
    PFF_HIP(hipMemcpyAsync(nr, hb.data(), sizeof(double) * B, hipMemcpyHostToDevice, s));
    k_b_scale_inv_sqrt<<<bgrid(n), 256, 0, s>>>(v, c->V, c->V, nr);
    PFF_CHECK_LAUNCH();
    std::vector<char> running = active_cycle;
    for (int j = 0; j < m; ++j) {
      double* vj = c->V + (int64_t)j * n;
      double* zj = c->Z + (int64_t)j * n;
      double* w = c->V + (int64_t)(j + 1) * n;
      PFF_TRY(bvcycle_any(c, vprec, vj, zj, s));
      PFF_TRY(bapply(c, L - 1, PF_F64, MODE_APPLY, zj, w, s));
      PFF_TRY(seg_dots(c, c->V, n, j + 1, w, f.d_seg1_lo, f.d_seg1_hi, B, h1, nullptr, s));
      k_b_multi_axpy<<<bgrid(n), 256, 0, s>>>(v, w, c->V, n, j + 1, h1, -1.0);
      PFF_CHECK_LAUNCH();
      PFF_TRY(seg_dots(c, c->V, n, j + 1, w, f.d_seg1_lo, f.d_seg1_hi, B, h2, nullptr, s));
      k_b_multi_axpy<<<bgrid(n), 256, 0, s>>>(v, w, c->V, n, j + 1, h2, -1.0);
      PFF_CHECK_LAUNCH();
      PFF_TRY(seg_dots(c, w, 0, 1, w, f.d_seg1_lo, f.d_seg1_hi, B, nr, nullptr, s));
      k_b_scale_inv_sqrt<<<bgrid(n), 256, 0, s>>>(v, w, w, nr);
      PFF_CHECK_LAUNCH();
      PFF_HIP(hipMemcpyAsync(hbuf.data(), dd, sizeof(double) * ((size_t)2 * (m + 1) * B + B), hipMemcpyDeviceToHost,
                             s));
      PFF_HIP(hipStreamSynchronize(s));
      ++total;
      bool any_running = false;
      for (int bb = 0; bb < B; ++bb) {
        if (!running[bb]) continue;
        for (int i = 0; i <= j; ++i)
          Hb(bb, i, j) = hbuf[(size_t)i * B + bb] + hbuf[(size_t)(m + 1) * B + (size_t)i * B + bb];
        Hb(bb, j + 1, j) = std::sqrt(std::max(0.0, hbuf[(size_t)2 * (m + 1) * B + bb]));
        double* csb = &cs[(size_t)bb * m];
        double* snb = &sn[(size_t)bb * m];
        double* gb = &g[(size_t)bb * (m + 1)];
        for (int i = 0; i < j; ++i) {
          const double a = Hb(bb, i, j), q = Hb(bb, i + 1, j);
          Hb(bb, i, j) = csb[i] * a + snb[i] * q;
          Hb(bb, i + 1, j) = -snb[i] * a + csb[i] * q;
        }
        const double a = Hb(bb, j, j), q = Hb(bb, j + 1, j);
        const double den = std::hypot(a, q);
        csb[j] = den == 0.0 ? 1.0 : a / den;
        snb[j] = den == 0.0 ? 0.0 : q / den;
        Hb(bb, j, j) = den;
        Hb(bb, j + 1, j) = 0.0;
        gb[j + 1] = -snb[j] * gb[j];
        gb[j] = csb[j] * gb[j];
        jend[bb] = j + 1;
        iters[bb] += 1;
        if (!std::isfinite(gb[j + 1])) {
          set_error("batched FGMRES produced a non-finite residual estimate");
          return PF_ERR_NONFINITE;
        }
        if (std::fabs(gb[j + 1]) <= tol[bb] || den == 0.0) running[bb] = 0;
        any_running = any_running || running[bb];
      }
      if (!any_running || total >= c->opt.gmres_max_iter) break;
    }
    // per-instance back substitution; instances not in this cycle get y = 0
    std::fill(y.begin(), y.end(), 0.0);
    int jmax = 0;
    for (int bb = 0; bb < B; ++bb) {
      if (!active_cycle[bb]) continue;
      const int je = jend[bb];
      jmax = std::max(jmax, je);
      for (int i = je - 1; i >= 0; --i) {
        double acc = g[(size_t)bb * (m + 1) + i];
        for (int k = i + 1; k < je; ++k) acc -= Hb(bb, i, k) * y[(size_t)k * B + bb];
        y[(size_t)i * B + bb] = Hb(bb, i, i) != 0.0 ? acc / Hb(bb, i, i) : 0.0;
      }
    }
    if (jmax > 0) {
      PFF_HIP(hipMemcpyAsync(c->d_y, y.data(), sizeof(double) * (size_t)jmax * B, hipMemcpyHostToDevice, s));
      k_b_multi_axpy<<<bgrid(n), 256, 0, s>>>(v, x, c->Z, n, jmax, c->d_y, 1.0);
      PFF_CHECK_LAUNCH();
    }
    PFF_HIP(hipStreamSynchronize(s));
    PFF_TRY(true_res(beta));
    for (int i = 0; i < B; ++i) conv[i] = !(beta[i] > tol[i]);
  }
  rel.assign(B, 0.0);
  for (int i = 0; i < B; ++i) rel[i] = bnorm[i] > 0 ? beta[i] / bnorm[i] : 0.0;
  return PF_OK;
}

double now() { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); }

}  // namespace

extern "C" {

pf_status pf_batch_workspace_size(const pf_mesh* meshes, int n, const pf_options* opt, size_t* bytes) {
  if (!bytes) {
    set_error("bytes is NULL");
    return PF_ERR_INVALID_ARG;
  }
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  PFF_TRY(validate_batch(meshes, nullptr, n, &o));
  for (int b = 0; b < n; ++b) {
    size_t tmp = 0;
    PFF_TRY(pf_workspace_size(&meshes[b], &o, &tmp));
  }
  *bytes = bcarve(nullptr, meshes, n, o, nullptr, nullptr);
  return PF_OK;
}

pf_status pf_batch_setup(const pf_mesh* meshes, const double* materials, int n, const pf_options* opt,
                         void* d_workspace, size_t ws_bytes, void* stream, pf_batch** out) {
  if (!out || !materials) {
    set_error("out and materials must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  *out = nullptr;
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  PFF_TRY(validate_batch(meshes, materials, n, &o));
  for (int b = 0; b < n; ++b) {
    size_t tmp = 0;
    PFF_TRY(pf_workspace_size(&meshes[b], &o, &tmp));
  }
  const size_t need = bcarve(nullptr, meshes, n, o, nullptr, nullptr);
  if (!d_workspace || ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return PF_ERR_WORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) {
    set_error("workspace must be 256-byte aligned");
    return PF_ERR_WORKSPACE;
  }
  pf_batch* c = new pf_batch();
  c->B = n;
  c->d = meshes[0].dim;
  c->p = meshes[0].degree;
  c->L = meshes[0].n_levels;
  c->opt = o;
  c->vprec = o.vcycle_precision;
  c->meshes.assign(meshes, meshes + n);
  for (int b = 0; b < n; ++b) {
    const double* m = materials + 6 * b;
    Material mm;
    mm.mu = m[0] / (2.0 * (1.0 + m[1]));
    mm.lam = m[0] * m[1] / ((1.0 + m[1]) * (1.0 - 2.0 * m[1]));
    mm.Gc = m[2];
    mm.eps = m[3];
    mm.kappa = m[4];
    mm.p = m[5];
    mm.split = o.stress_split;
    c->mats.push_back(mm);
  }
  bcarve(c, meshes, n, o, reinterpret_cast<char*>(d_workspace), &c->mats);
  hipStream_t s = bst(stream);
  pf_status st = PF_OK;
  for (int l = 0; l < c->L && st == PF_OK; ++l) {
    BLevel& bl = c->lev[l];
    std::vector<int64_t> s2lo(2 * n), s2hi(2 * n), s1lo(n), s1hi(n);
    for (int b = 0; b < n; ++b) {
      const int64_t nn = bl.h_node[b + 1] - bl.h_node[b];
      s2lo[2 * b] = bl.h_dof[b];
      s2hi[2 * b] = bl.h_dof[b] + (int64_t)c->d * nn;
      s2lo[2 * b + 1] = s2hi[2 * b];
      s2hi[2 * b + 1] = bl.h_dof[b + 1];
      s1lo[b] = bl.h_dof[b];
      s1hi[b] = bl.h_dof[b + 1];
    }
    auto h2d = [&](void* dst, const void* src, size_t bytes) {
      return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    hipError_t e = h2d(bl.d_inst, bl.h_inst.data(), sizeof(BInst) * n);
    if (e == hipSuccess) e = h2d(bl.d_dof, bl.h_dof.data(), sizeof(int64_t) * (n + 1));
    if (e == hipSuccess) e = h2d(bl.d_node, bl.h_node.data(), sizeof(int64_t) * (n + 1));
    if (e == hipSuccess) e = h2d(bl.d_cell, bl.h_cell.data(), sizeof(int64_t) * (n + 1));
    if (e == hipSuccess) e = h2d(bl.d_seg2_lo, s2lo.data(), sizeof(int64_t) * 2 * n);
    if (e == hipSuccess) e = h2d(bl.d_seg2_hi, s2hi.data(), sizeof(int64_t) * 2 * n);
    if (e == hipSuccess) e = h2d(bl.d_seg1_lo, s1lo.data(), sizeof(int64_t) * n);
    if (e == hipSuccess) e = h2d(bl.d_seg1_hi, s1hi.data(), sizeof(int64_t) * n);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host staging vectors end with this iteration
    if (e != hipSuccess) {
      set_error(std::string("batch setup copy: ") + hipGetErrorString(e));
      st = PF_ERR_DEVICE;
      break;
    }
    k_b_base_mask<<<bgrid(bl.n_nodes), 256, 0, s>>>(bl.view(), bl.base);
    if (hipGetLastError() != hipSuccess) st = PF_ERR_DEVICE;
    if (st == PF_OK) st = vec_copy<uint8_t>(bl.mask, bl.base, bl.n_nodes, s);
  }
  if (st == PF_OK) {
    BLevel& f = c->lev[c->L - 1];
    k_b_lumped<<<bgrid(f.n_nodes), 256, 0, s>>>(f.view(), c->M);
    if (hipGetLastError() != hipSuccess) st = PF_ERR_DEVICE;
  }
  if (st == PF_OK && hipStreamSynchronize(s) != hipSuccess) st = PF_ERR_DEVICE;
  if (st != PF_OK) {
    if (st == PF_ERR_DEVICE && std::string(pf_last_error()).empty()) set_error("batch setup failed on the device");
    delete c;
    return st;
  }
  *out = c;
  return PF_OK;
}

void pf_batch_destroy(pf_batch* b) { delete b; }

#define NEED_BATCH()                  \
  if (!bt) {                          \
    set_error("batch is NULL");       \
    return PF_ERR_INVALID_ARG;        \
  }

pf_status pf_batch_layout(pf_batch* bt, int level, int64_t* dof_offsets, int64_t* node_offsets) {
  NEED_BATCH();
  if (level < 0 || level >= bt->L) {
    set_error("level out of range");
    return PF_ERR_INVALID_ARG;
  }
  const BLevel& bl = bt->lev[level];
  if (dof_offsets) std::memcpy(dof_offsets, bl.h_dof.data(), sizeof(int64_t) * (bt->B + 1));
  if (node_offsets) std::memcpy(node_offsets, bl.h_node.data(), sizeof(int64_t) * (bt->B + 1));
  return PF_OK;
}

pf_status pf_batch_set_constraints(pf_batch* bt, const uint8_t* d_bits, void* stream) {
  NEED_BATCH();
  if (!d_bits) {
    bt->has_extra = false;
    return PF_OK;
  }
  PFF_TRY(vec_copy<uint8_t>(bt->extra, d_bits, bt->lev[bt->L - 1].n_nodes, bst(stream)));
  bt->has_extra = true;
  return PF_OK;
}

pf_status pf_batch_set_linearization(pf_batch* bt, const double* d_U, const double* d_phi_tilde,
                                     const uint8_t* d_active, void* stream) {
  NEED_BATCH();
  if (!d_U || !d_phi_tilde) {
    set_error("U and phi_tilde must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  return bset_linearization(bt, d_U, d_phi_tilde, d_active, bst(stream));
}

pf_status pf_batch_jacobian_apply(pf_batch* bt, int level, int prec, const void* d_x, void* d_y, void* stream) {
  NEED_BATCH();
  if (!bt->has_lin) {
    set_error("no linearization point: call pf_batch_set_linearization");
    return PF_ERR_INVALID_ARG;
  }
  if (level < 0 || level >= bt->L || (prec != PF_F64 && prec != PF_F32) || !d_x || !d_y || d_x == d_y) {
    set_error("bad level, precision or vectors");
    return PF_ERR_INVALID_ARG;
  }
  return bapply(bt, level, prec, MODE_APPLY, d_x, d_y, bst(stream));
}

pf_status pf_batch_vcycle(pf_batch* bt, int prec, const double* d_r, double* d_z, void* stream) {
  NEED_BATCH();
  if (!bt->has_lin) {
    set_error("no linearization point: call pf_batch_set_linearization");
    return PF_ERR_INVALID_ARG;
  }
  if ((prec != PF_F64 && prec != PF_F32) || !d_r || !d_z || d_r == d_z) {
    set_error("bad precision or vectors");
    return PF_ERR_INVALID_ARG;
  }
  return bvcycle_any(bt, prec, d_r, d_z, bst(stream));
}

pf_status pf_batch_get_eig_bounds(pf_batch* bt, int level, int inst, double out[4]) {
  NEED_BATCH();
  if (level < 0 || level >= bt->L || inst < 0 || inst >= bt->B || !out) {
    set_error("bad level, instance or output");
    return PF_ERR_INVALID_ARG;
  }
  for (int k = 0; k < 4; ++k) out[k] = bt->lev[level].eig[4 * inst + k];
  return PF_OK;
}

pf_status pf_batch_set_eig_bounds(pf_batch* bt, int level, int inst, const double in[4]) {
  NEED_BATCH();
  if (level < 0 || level >= bt->L || inst < 0 || inst >= bt->B) {
    set_error("bad level or instance");
    return PF_ERR_INVALID_ARG;
  }
  BLevel& bl = bt->lev[level];
  if (!in) {
    for (int k = 0; k < 4; ++k) bl.eig_fix[4 * inst + k] = 0.0;
    return PF_OK;
  }
  for (int k = 0; k < 4; ++k)
    if (!(in[k] > 0.0) || !std::isfinite(in[k])) {
      set_error("eigenvalue bounds must be positive and finite");
      return PF_ERR_INVALID_ARG;
    }
  if (in[0] > in[1] || in[2] > in[3]) {
    set_error("need lam_min <= lam_max per block");
    return PF_ERR_INVALID_ARG;
  }
  for (int k = 0; k < 4; ++k) bl.eig_fix[4 * inst + k] = bl.eig[4 * inst + k] = in[k];
  // the Chebyshev coefficients live in device memory (captured V-cycles read them there)
  if (bt->has_lin) PFF_TRY(upload_cheb(bt, nullptr));
  return PF_OK;
}

// the work table of level l, precision index pi and operator mi for a shape and chunk
static pf_status b_build_items(pf_batch* c, int l, int pi, int mi, int shape, int zc, hipStream_t s) {
  BLevel& bl = c->lev[l];
  bl.shape[pi][mi] = -1;
  bl.zc[pi][mi] = 0;
  bl.n_items[pi][mi] = 0;
  if (shape < 0) return PF_OK;
  if (bl.p != 1 || bl.split || !bl.items[pi][mi] || (shape == kBShapeMarch16 && bl.d != 3) ||
      (shape != kBShapeAtomic && zc < 1)) {
    set_error("batched cell loop: no work table of this shape on this level");
    return PF_ERR_UNSUPPORTED;
  }
  std::vector<int2> h;
  for (int b = 0; b < bl.B; ++b) {
    const int64_t m = b_items_of(bl.h_inst[b].cp, bl.d, shape, zc);
    for (int64_t k = 0; k < m; ++k) h.push_back(make_int2(b, (int)k));
  }
  if ((int64_t)h.size() > bl.item_cap || h.size() > (size_t)0x7fffffff) {
    set_error("batched cell loop: the work table does not fit (chunk below the autotuner's smallest?)");
    return PF_ERR_WORKSPACE;
  }
  if (!h.empty()) {
    PFF_HIP(hipMemcpyAsync(bl.items[pi][mi], h.data(), h.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    PFF_HIP(hipStreamSynchronize(s));
  }
  bl.shape[pi][mi] = shape;
  bl.zc[pi][mi] = shape == kBShapeAtomic ? 0 : zc;
  bl.n_items[pi][mi] = (int)h.size();
  return PF_OK;
}

pf_status pf_batch_autotune(pf_batch* bt, int reps, void* stream) {
  NEED_BATCH();
  if (!bt->has_lin) {
    set_error("no linearization point: call pf_batch_set_linearization");
    return PF_ERR_INVALID_ARG;
  }
  if (reps < 1 || reps > 10000) {
    set_error("reps must be in [1, 10000]");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = bst(stream);
  bt->drop_graphs();
  hipEvent_t e0, e1;
  PFF_HIP(hipEventCreate(&e0));
  PFF_HIP(hipEventCreate(&e1));
  pf_status st = PF_OK;
  for (int l = 0; l < bt->L && st == PF_OK; ++l) {
    BLevel& bl = bt->lev[l];
    if (bl.p != 1 || bl.split) continue;
    for (int pi = 0; pi < 2 && st == PF_OK; ++pi) {
      const int prec = pi == 0 ? PF_F64 : PF_F32;
      st = prec == PF_F64 ? vec_fill<double>((double*)bl.vb, 1.0, bl.n_dofs, s)
                          : vec_fill<float>((float*)bl.vb, 1.0f, bl.n_dofs, s);
      for (int mi = 0; mi < 2 && st == PF_OK; ++mi) {
        double best = 1e300;
        for (int k = 0; k < kBNCand && st == PF_OK; ++k) {
          bl.tune_us[pi][mi][k] = -1.0;
          if (kBCand[k][0] == kBShapeMarch16 && bl.d != 3) continue;
          st = b_build_items(bt, l, pi, mi, kBCand[k][0], kBCand[k][1], s);
          for (int w = 0; w < 2 && st == PF_OK; ++w) st = bapply(bt, l, prec, mi, bl.vb, bl.vt, s);
          if (st != PF_OK) break;
          float ms = 0.f;
          if (hipEventRecord(e0, s) != hipSuccess) st = PF_ERR_DEVICE;
          for (int r = 0; r < reps && st == PF_OK; ++r) st = bapply(bt, l, prec, mi, bl.vb, bl.vt, s);
          if (st != PF_OK) break;
          if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            set_error("batched autotune timing failed");
            st = PF_ERR_DEVICE;
            break;
          }
          bl.tune_us[pi][mi][k] = 1e3 * ms / reps;
          best = std::min(best, bl.tune_us[pi][mi][k]);
        }
        if (st != PF_OK) break;
        // the earliest candidate within 3% of the fastest (timing noise does not flip the choice)
        int pick = 0;
        for (int k = 0; k < kBNCand; ++k)
          if (bl.tune_us[pi][mi][k] > 0.0 && bl.tune_us[pi][mi][k] <= best * 1.03) {
            pick = k;
            break;
          }
        st = b_build_items(bt, l, pi, mi, kBCand[pick][0], kBCand[pick][1], s);
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

pf_status pf_batch_get_tuning(pf_batch* bt, int level, int prec, int mode, int* shape, int* zc, double* us) {
  NEED_BATCH();
  if (level < 0 || level >= bt->L || (prec != PF_F64 && prec != PF_F32) || (mode != 0 && mode != 1) || !shape ||
      !zc) {
    set_error("bad level, precision, mode or output pointer");
    return PF_ERR_INVALID_ARG;
  }
  const BLevel& bl = bt->lev[level];
  const int pi = prec == PF_F64 ? 0 : 1;
  *shape = bl.shape[pi][mode];
  *zc = bl.zc[pi][mode];
  if (us)
    for (int k = 0; k < kBNCand; ++k) us[k] = bl.tune_us[pi][mode][k];
  return PF_OK;
}

pf_status pf_batch_set_tuning(pf_batch* bt, int level, int prec, int mode, int shape, int zc) {
  NEED_BATCH();
  if (level < 0 || level >= bt->L || (prec != PF_F64 && prec != PF_F32) || (mode != 0 && mode != 1) ||
      shape < -1 || shape > kBShapeAtomic) {
    set_error("bad level, precision, mode or shape");
    return PF_ERR_INVALID_ARG;
  }
  bt->drop_graphs();
  return b_build_items(bt, level, prec == PF_F64 ? 0 : 1, mode, shape, zc, nullptr);
}

pf_status pf_batch_set_graphs(pf_batch* bt, int enable) {
  NEED_BATCH();
  bt->use_graphs = enable != 0;
  return PF_OK;
}

pf_status pf_batch_set_vcycle_precision(pf_batch* bt, int prec) {
  NEED_BATCH();
  if (prec != PF_F64 && prec != PF_F32) {
    set_error("prec must be PF_F64 or PF_F32");
    return PF_ERR_INVALID_ARG;
  }
  bt->vprec = prec;
  return PF_OK;
}

pf_status pf_batch_newton_step(pf_batch* bt, double* d_U, const double* d_U_old, const double* d_phi_tilde,
                               pf_newton_report* reps, void* stream) {
  NEED_BATCH();
  if (!d_U || !d_U_old || !d_phi_tilde) {
    set_error("U, U_old and phi_tilde must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = bst(stream);
  const int L = bt->L, B = bt->B;
  BLevel& f = bt->lev[L - 1];
  const BView v = f.view();
  const double t0 = now();
  // 1. residual of every instance
  PFF_TRY(vec_fill<double>(bt->R, 0.0, f.n_dofs, s));
  // the residual reads the caller's U and phi~ (same packed layout as the finest level)
  PFF_TRY(b_cell<double>(v, MODE_RESID, nullptr, d_U, d_phi_tilde, f.mask, bt->R, s));
  double bad = 0;
  PFF_TRY(count_nonfinite(bt->R, f.n_dofs, bt->part, &bad, s));
  if (bad > 0) {
    set_error("non-finite residual (check U, U_old, phi_tilde)");
    return PF_ERR_NONFINITE;
  }
  const double t1 = now();
  // 2-4. active sets, lifts, level data
  k_b_pdas<<<bgrid(f.n_nodes), 256, 0, s>>>(v, bt->R, d_U, d_U_old, bt->M, f.base, bt->opt.pdas_c, bt->active);
  PFF_CHECK_LAUNCH();
  std::vector<double> nact(B);
  {
    dim3 grid(kSegBlocks, B);
    k_b_seg_count<<<grid, 256, 0, s>>>(bt->active, f.d_node, bt->part);
    PFF_CHECK_LAUNCH();
    k_b_rows<<<B, 256, 0, s>>>(bt->part, kSegBlocks, bt->dscal);
    PFF_CHECK_LAUNCH();
    PFF_HIP(hipMemcpyAsync(nact.data(), bt->dscal, sizeof(double) * B, hipMemcpyDeviceToHost, s));
    PFF_HIP(hipStreamSynchronize(s));
  }
  double nact_total = 0;
  for (double a : nact) nact_total += a;
  k_b_lift<<<bgrid(f.n_dofs), 256, 0, s>>>(v, d_U, d_U_old, bt->active, bt->dl);
  PFF_CHECK_LAUNCH();
  PFF_TRY(bset_linearization(bt, d_U, d_phi_tilde, bt->active, s));
  const double* tl = nullptr;
  if (nact_total > 0) {
    PFF_TRY(bapply(bt, L - 1, PF_F64, MODE_RAW, bt->dl, bt->t, s));
    tl = bt->t;
  }
  k_b_constrain_rhs<<<bgrid(f.n_dofs), 256, 0, s>>>(v, bt->R, tl, bt->dl, f.mask, bt->Rt);
  PFF_CHECK_LAUNCH();
  PFF_HIP(hipStreamSynchronize(s));
  const double t2 = now();
  // 5. FGMRES from the lift; 6. update
  PFF_TRY(vec_copy<double>(bt->dU, bt->dl, f.n_dofs, s));
  std::vector<int> iters;
  std::vector<double> rel, bn;
  PFF_TRY(bfgmres(bt, bt->Rt, bt->dU, bt->vprec, iters, rel, bn, s));
  PFF_TRY(vec_axpby<double>(d_U, 1.0, bt->dU, 1.0, f.n_dofs, s));
  PFF_HIP(hipStreamSynchronize(s));
  const double t3 = now();
  bool all = true;
  for (int b = 0; b < B; ++b) {
    const bool conv = rel[b] * bn[b] <= std::max(bt->opt.gmres_rtol * bn[b], bt->opt.gmres_atol);
    all = all && conv;
    if (reps) {
      pf_newton_report& r = reps[b];
      std::memset(&r, 0, sizeof(r));
      r.gmres_iters = iters[b];
      r.converged = conv ? 1 : 0;
      r.rel_residual = rel[b];
      r.rhs_norm = bn[b];
      r.n_active = (int64_t)nact[b];
      r.t_residual_s = t1 - t0;
      r.t_setup_s = t2 - t1;
      r.t_solve_s = t3 - t2;
      r.t_total_s = t3 - t0;
    }
  }
  if (!all) {
    set_error("batched FGMRES reached gmres_max_iter before the tolerance on some instance");
    return PF_ERR_NOT_CONVERGED;
  }
  return PF_OK;
}

}  // extern "C"
