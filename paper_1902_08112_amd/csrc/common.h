// Internal declarations of the pff library (gfx950 HIP).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pff.h"

namespace pff {

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);

#define PFF_HIP(...)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (__VA_ARGS__);                                                                  \
    if (e_ != hipSuccess) {                                                                    \
      ::pff::set_error(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));                     \
      return PF_ERR_DEVICE;                                                                    \
    }                                                                                          \
  } while (0)

#define PFF_CHECK_LAUNCH()                                                                     \
  do {                                                                                         \
    hipError_t e_ = hipGetLastError();                                                         \
    if (e_ != hipSuccess) {                                                                    \
      ::pff::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));                \
      return PF_ERR_DEVICE;                                                                    \
    }                                                                                          \
  } while (0)

#define PFF_TRY(...)                                                                           \
  do {                                                                                         \
    pf_status s_ = (__VA_ARGS__);                                                                   \
    if (s_ != PF_OK) return s_;                                                                \
  } while (0)

constexpr int kMaskPhi = 8;

__host__ __device__ inline int mask_bit(int comp, int d) { return comp < d ? (1 << comp) : kMaskPhi; }

// ---------------------------------------------------------------------------
// level geometry and cell-operator parameters
// ---------------------------------------------------------------------------
struct Geom {
  int d, p;
  int N[3];        // cells per axis (1 for unused axes)
  int nn[3];       // nodes per axis (1 for unused axes)
  int64_t ns[3];   // node strides (x fastest)
  int64_t n_nodes, n_dofs, n_cells;
  double h[3];
  double ext[3];
  int lshape;
};

// Parameters of every cell-loop kernel (passed by value).
struct CellParams {
  int N[3];
  int nn[3];
  int64_t ns[3];
  int64_t n_nodes;
  int64_t n_cells;
  int lshape;
  double inv_h[3];
  double vol;          // cell volume (JxW = w_q * vol)
  double mu, lam, kappa, pres, gc_over_eps, gc_eps;
  int variant;         // Q1 cell-loop variant (-1: size heuristic), see cell_q1.hip
  int zc;              // node planes per marching chunk (<= 0: heuristic)
  int d, p;            // dimension and degree
  int split;           // PF_SPLIT_NONE or PF_SPLIT_MIEHE (Sec. 2.1)
  const void* qpd;     // split: the level's per-point eigen-records in the apply's precision (or null)
  const void* qcb;     // Q1 block operator: per-point c_phi JxW of the level in the apply's precision (or null)
};

// Material constants (Sec. 2.1): mu, lambda from E, nu; G_c, eps, kappa, p; energy split.
struct Material {
  double mu, lam, Gc, eps, kappa, p;
  int split;
};

CellParams make_cell_params(const Geom& g, const Material& m);

__host__ __device__ inline bool cell_in_hole(int lshape, int cx, int cy, int Nx, int Ny) {
  return lshape && (2 * cx >= Nx) && (2 * cy >= Ny);
}

// Cell-loop modes.
enum CellMode {
  MODE_APPLY = 0,  // y += Pi_F G Pi_F x   (y pre-set to Pi_C x)
  MODE_BLOCK = 1,  // same with the phi-u coupling removed (smoother operator B)
  MODE_RAW = 2,    // y += G x, no constraints
  MODE_RESID = 3,  // y += -A(U)
  MODE_DIAG = 4,   // y += diag(G) (constrained rows set to 1 afterwards)
};

// Launch the cell loop on level data.  T = double or float.  For MODE_RESID
// and MODE_DIAG x is ignored.  y is accumulated into (callers pre-set it).
template <typename T>
pf_status launch_cell(const Geom& g, const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                      const uint8_t* mask, T* y, hipStream_t s);

// Miehe split on Q1 levels (cell_split.hip): records of the per-point eigen-data
// (split_record_values(d) values per cell), computed from the level's U
int split_record_values(int d);
// One Chebyshev step of the smoother fused into the block-operator apply (3D Q1 marching
// tiles, which write every node once): at each node, with t = (B~ d)(node),
//   r -= t;  d' = c1 d + c2 r / diag;  x += d';  [d_out = d'];  [t_next = Pi_C (next_of_x ? x : d')]
// with (c1, c2) of the displacement block on u rows and of the phase-field block on phi rows.
// d (the apply's input) is only read; d_out is a different buffer, or null.
template <typename T>
struct ChebFuse {
  T* res;
  const T* diag;
  T* x;
  T* d_out;
  T* t_next;
  const double* dc;  // device: {c1, c2} of the displacement block, then of the phase-field block
  int next_of_x;
};
// *handled = false when the level's block operator is not a 3D Q1 marching-tile shape
template <typename T>
pf_status launch_q1_block_cheb(const Geom& g, const CellParams& cp, const T* d, const T* U, const T* phit,
                               const uint8_t* mask, const ChebFuse<T>& cf, hipStream_t s, bool* handled);
bool q1_block_cheb_fusable(const Geom& g, const CellParams& cp);
// 3D Q1 LDS-staged marching slabs (variant 5): G~ or B~ into y, or B~ with the fused
// Chebyshev step when cf is non-null; q1_slab_chunk: node planes per chunk
template <typename T>
pf_status launch_q1_slab(const Geom& g, const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                         const uint8_t* mask, T* y, const ChebFuse<T>* cf, hipStream_t s);
int q1_slab_chunk(const Geom& g, int requested_zc);

// Q1 block operator coefficients: values per cell, and the per-linearization pass that writes them
int q1_block_coef_values(int d);
pf_status launch_block_coef(const Geom& g, const CellParams& cp, const double* U, double* c64, float* c32,
                            hipStream_t s);
// 3D Q2 block operator coefficients: g(phi~) JxW and c_phi at the 27 Gauss points (54 values per cell)
constexpr int kQ2BlockCoefValues = 54;
pf_status launch_block_coef_q2(const Geom& g, const CellParams& cp, const double* U, const double* phit, double* c64,
                               float* c32, hipStream_t s);
pf_status launch_split_data(const Geom& g, const CellParams& cp, const double* U, double* rec64, float* rec32,
                            hipStream_t s);

// Q1 cell-loop variants: 0 = marching 8x8 tiles, 1 = marching 16x4 tiles (both
// write every node of y themselves), 2 = one thread per cell with atomics (y pre-set),
// 3 = LDS-staged bricks of cells with atomics (3D, y pre-set), 4 = two work items
// (displacement / phase-field rows) per cell with atomics (y pre-set).
constexpr int kQ1Variants = 6;
int q1_variant(const Geom& g, int mode, int requested);
bool q1_tiled_handles(const Geom& g, int mode, int requested);
// marching chunk the tiled kernels use for this level and request
int q1_chunk(const Geom& g, int variant, int requested_zc);
// FP64 residual -A(U) (MODE_RESID) and diag(G) (MODE_DIAG) on 2D / 3D Q1 levels without the
// energy split (cell_q1_aux.hip): marching tiles that write every entry of y (no constraint
// applied, no pre-set y)
bool q1_aux_handles(const Geom& g, int mode);
pf_status launch_q1_aux(const Geom& g, const CellParams& cp, int mode, const double* U, const double* phit,
                        double* y, hipStream_t s);

// ---------------------------------------------------------------------------
// vector kernels (vec.hip)
// ---------------------------------------------------------------------------
template <typename T>
pf_status vec_fill(T* y, T v, int64_t n, hipStream_t s);
template <typename T>
pf_status vec_copy(T* y, const T* x, int64_t n, hipStream_t s);
template <typename Tin, typename Tout>
pf_status vec_cast(Tout* y, const Tin* x, int64_t n, hipStream_t s);
// y_i = constrained ? x_i : 0   (x may be null -> 0)
template <typename T>
pf_status vec_init_constrained(T* y, const T* x, const uint8_t* mask, int64_t nn, int d, hipStream_t s);
// y_i = constrained ? v : y_i
template <typename T>
pf_status vec_set_constrained(T* y, T v, const uint8_t* mask, int64_t nn, int d, hipStream_t s);
// y = a*x + b*y
template <typename T>
pf_status vec_axpby(T* y, T a, const T* x, T b, int64_t n, hipStream_t s);
// z = x - y
template <typename T>
pf_status vec_sub(T* z, const T* x, const T* y, int64_t n, hipStream_t s);
// Chebyshev step (per block coefficients c1[2], c2[2]; blocks u / phi):
//   mode 0: res -= t;      d = c1*d + c2*Dinv*res; x += d
//   mode 1: res = b;       d = c2*Dinv*res;        x = d    (x = 0 before)
//   mode 2: res = b - t;   d = c2*Dinv*res;        x += d   (t = G~ x)
//   mode 3: res as given;  d = c2*Dinv*res;        x += d
// t_next (may alias t, or nullptr): t_next = Pi_C d (Pi_C x_new if next_of_x), the
// starting value of the next operator apply.  dc: device array {c1, c2} of the displacement
// block then {c1, c2} of the phase-field block
template <typename T>
pf_status vec_cheb_step(T* res, const T* t, T* dv, T* x, const T* diag, const double* dc, int mode, int64_t nn,
                        int d, const uint8_t* mask, T* t_next, int next_of_x, const T* b, hipStream_t s);
// dst[0..n) = src[0..n) from host memory, in stream order, through kernel arguments (src may be
// reused as soon as the call returns)
pf_status vec_put(double* dst, const double* src, int64_t n, hipStream_t s);
// dots per block: out[0] = sum over u-block of x*y, out[1] over the phi-block (FP64 accumulation)
pf_status dot_blocks(const double* x, const double* y, int64_t nn, int d, double* d_partials, double* h_out,
                     hipStream_t s);
// ||x||^2 (FP64) into host
pf_status dot_host(const double* x, const double* y, int64_t n, double* d_partials, double* h_out, hipStream_t s);
// h_dev[i] = V_i . w for i < k (V rows of length n, stride ld); FP64
pf_status multi_dot(const double* V, int64_t ld, int k, const double* w, int64_t n, double* d_partials,
                    double* d_h, hipStream_t s);
// w -= sum_i h[i] V_i   (h on device)
pf_status multi_axpy(double* w, const double* V, int64_t ld, int k, const double* d_h, int64_t n, double sign,
                     hipStream_t s);
// One Gram-Schmidt pass fused with the reduction that follows it, for k <= kMultiDotRows:
// w -= sum_i h[i] V_i, and in the same pass over w either d_out[i] = V_i . w (norm false) or
// d_out[0] = |w|^2 (norm true), both of the updated w.  w and the dots take the values of
// multi_axpy followed by multi_dot (the same reduction grid and order).
pf_status axpy_then_dot(double* w, const double* V, int64_t ld, int k, const double* d_h, int64_t n, bool norm,
                        double* d_partials, double* d_out, hipStream_t s);
// y = x * (1/sqrt(*d_nrm2))
pf_status vec_scale_inv_sqrt(double* y, const double* x, const double* d_nrm2, int64_t n, hipStream_t s);
// sum of squares into d_out (device scalar)
pf_status nrm2_dev(const double* x, int64_t n, double* d_partials, double* d_out, hipStream_t s);
// count of non-finite entries (host)
pf_status count_nonfinite(const double* x, int64_t n, double* d_partials, double* h_out, hipStream_t s);
// SplitMix64 start vector of the eigenvalue estimate (block-local counters), masked
template <typename T>
pf_status eig_start_vector(T* v, const uint8_t* mask, int64_t nn, int d, uint64_t seed_u, uint64_t seed_phi,
                           hipStream_t s);
// y_i = x_i * dinv_i where dinv = 1/diag (constrained rows: 0)
pf_status vec_jacobi(double* y, const double* x, const double* diag, const uint8_t* mask, int64_t nn, int d,
                     hipStream_t s);
// per block: y_b = x_b + beta_b * y_b / y_b -= alpha_b * x_b
pf_status vec_xpby_blocks(double* y, const double* x, const double beta[2], int64_t nn, int d, hipStream_t s);
pf_status vec_axpy_blocks(double* y, const double* x, const double alpha[2], int64_t nn, int d, hipStream_t s);

// Jacobi-PCG of the eigenvalue estimate with its scalars on the device: the
// per-block coefficients alpha_k, beta_k accumulate in an EigDev record that
// the host reads once after every level has run (no round trip per step).
constexpr int kEigMaxSteps = 100;
struct EigDev {
  double rz[2], rz0[2], alpha[2], beta[2];
  int done[2], n_al[2], n_be[2];
  double al[2][kEigMaxSteps], be[2][kEigMaxSteps];
};
// z = p = D^-1 r (masked), then rz = rz0 = (r, z) per block
// (T = double or float vectors; the dots accumulate in FP64, the coefficients are FP64)
template <typename T>
pf_status eig_cg_begin(const T* r, T* z, T* p, const T* diag, const uint8_t* mask, int64_t nn,
                       int d, double* d_partials, EigDev* st, hipStream_t s);
// alpha_b = rz_b / (p, Ap)_b (a block with (p, Ap)_b <= 0 stops)
template <typename T>
pf_status eig_cg_alpha(const T* p, const T* Ap, int64_t nn, int d, double* d_partials, EigDev* st,
                       hipStream_t s);
// r -= alpha Ap, z = D^-1 r, beta_b = (r, z)_b / rz_b, p = z + beta p; a block stops once rz_b <= 1e-24 rz0_b
template <typename T>
pf_status eig_cg_beta(T* r, const T* Ap, T* z, T* p, const T* diag, const uint8_t* mask,
                      int64_t nn, int d, double* d_partials, EigDev* st, hipStream_t s);

// ---------------------------------------------------------------------------
// structured grid kernels (grid.hip)
// ---------------------------------------------------------------------------
// masks: Dirichlet faces and hole
pf_status build_base_mask(const Geom& g, unsigned faces, uint8_t* mask, hipStream_t s);
// coarse[j] = fine[inj(j)] for ncomp components (fine -> coarse nodal injection)
template <typename T>
pf_status inject(const Geom& gc, const Geom& gf, const T* fine, T* coarse, int ncomp, hipStream_t s);
// coarse_mask[j] = fine_mask[inj(j)] | base[j]
pf_status inject_mask(const Geom& gc, const Geom& gf, const uint8_t* fine, const uint8_t* base, uint8_t* coarse,
                      hipStream_t s);
// restriction out_c = [mask_c] P^T v with v = in_f, or v = in_f - sub_f (formed in Tin) when sub_f
// is set (the residual b - G~ x restricted without storing it)
template <typename Tin, typename Tout>
pf_status restrict_vec(const Geom& gc, const Geom& gf, const Tin* in_f, const Tin* sub_f, Tout* out_c,
                       const uint8_t* mask_c, hipStream_t s);
// prolongation: out_f = (add ? out_f : 0) + [mask_f] P in_c
template <typename Tin, typename Tout>
pf_status prolong_vec(const Geom& gc, const Geom& gf, const Tin* in_c, Tout* out_f, const uint8_t* mask_f, int add,
                      hipStream_t s);
// lumped mass on the node lattice
pf_status lumped_mass(const Geom& g, double* M, hipStream_t s);
// active set decision; active bytes, v values, and mask |= 8 for active nodes
pf_status pdas_decide(const Geom& g, const double* R, const double* U, const double* Uold, const double* M,
                      const uint8_t* base_mask, double c, uint8_t* active, double* v, hipStream_t s);
// count of nonzero bytes (host result)
pf_status count_bytes(const uint8_t* a, int64_t n, double* d_partials, int64_t* h_out, hipStream_t s);
// positions where two masks differ as flags (host result)
pf_status count_diff_bytes(const uint8_t* a, const uint8_t* b, int64_t n, double* d_partials, int64_t* h_out,
                           hipStream_t s);
// phi~ = phi_1 + theta (phi_1 - phi_2) on nodes; nodes whose base mask constrains phi (hole) copy phi_1
pf_status extrapolate_phase(const double* phi_1, const double* phi_2, double theta, const uint8_t* base, int64_t n,
                            double* out, hipStream_t s);
// mask = base | extra | (active ? 8 : 0)
pf_status combine_mask(const uint8_t* base, const uint8_t* extra, const uint8_t* active, uint8_t* mask, int64_t n,
                       hipStream_t s);
// lift d = Pi_C,phi-active (Uold - U) (only phi block on active nodes), else 0
pf_status build_lift(const Geom& g, const double* U, const double* Uold, const uint8_t* active, double* dl,
                     hipStream_t s);
// Rt_i = constrained ? dl_i : R_i - t_i
pf_status constrain_rhs(const Geom& g, const double* R, const double* t, const double* dl, const uint8_t* mask,
                        double* Rt, hipStream_t s);

constexpr int kRedBlock = 256;
constexpr int kRedMaxBlocks = 4096;  // enough wavefronts in flight to stream a 50M-value vector
// multi_dot: rows per launch, and workgroups per launch (its partials need kMultiDotBlocks per row)
constexpr int kMultiDotRows = 8;
constexpr int kMultiDotBlocks = 2048;

}  // namespace pff
