// Host orchestration and the C ABI: context and workspace carve-up, level data
// (Sec. 4.2), eigenvalue estimates (Sec. 3.2.1), the V-cycle (Sec. 3.2, 3.3),
// FGMRES with CGS2 (Sec. 3, 5) and one active-set Newton step (Algorithm 1).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <limits>
#include <vector>

#include "common.h"

namespace pff {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

pf_status launch_cell_generic_d(const Geom&, const CellParams&, int, const double*, const double*, const double*,
                                const uint8_t*, double*, hipStream_t);
pf_status launch_cell_generic_f(const Geom&, const CellParams&, int, const float*, const float*, const float*,
                                const uint8_t*, float*, hipStream_t);
pf_status launch_cell_q1s_d(const Geom&, const CellParams&, int, const double*, const double*, const double*,
                            const uint8_t*, double*, hipStream_t, bool*);
pf_status launch_cell_q1s_f(const Geom&, const CellParams&, int, const float*, const float*, const float*,
                            const uint8_t*, float*, hipStream_t, bool*);
pf_status launch_cell_q1_d(const Geom&, const CellParams&, int, const double*, const double*, const double*,
                           const uint8_t*, double*, hipStream_t, bool* handled);
pf_status launch_cell_q1_f(const Geom&, const CellParams&, int, const float*, const float*, const float*,
                           const uint8_t*, float*, hipStream_t, bool* handled);
pf_status launch_cell_q2_d(const Geom&, const CellParams&, int, const double*, const double*, const double*,
                           const uint8_t*, double*, hipStream_t, bool* handled);
pf_status launch_cell_q2_f(const Geom&, const CellParams&, int, const float*, const float*, const float*,
                           const uint8_t*, float*, hipStream_t, bool* handled);
pf_status quantity_energies(const Geom& gm, const CellParams& cp, double Gc, double eps, const double* U,
                            double* d_part, double out[2], hipStream_t s);
pf_status quantity_scratch_init(int device);
pf_status quantity_energies_noalloc(const Geom& gm, const CellParams& cp, double Gc, double eps, const double* U,
                                    int device, double* d_out, hipStream_t s);
pf_status quantity_face_traction(const Geom& gm, const CellParams& cp, int face, const double* U, double* d_part,
                                 double* out, hipStream_t s);
pf_status launch_coarse_solve(const Geom& g, const CellParams& cp, int degree, int sweeps, const double* dcoef,
                              const double* U, const double* phit, const uint8_t* mask, const double* diag,
                              const double* b, double* x, double* r, bool couple, hipStream_t s, bool* handled,
                              bool columns = false);
pf_status coarse_matvec(const double* S, const double* b, double* x, int64_t n, hipStream_t s);
pf_status coarse_transpose(const double* C, double* T, int64_t n, hipStream_t s);

template <>
pf_status launch_cell<double>(const Geom& g, const CellParams& cp, int mode, const double* x, const double* U,
                              const double* phit, const uint8_t* mask, double* y, hipStream_t s) {
  bool handled = false;
  if (cp.split) {
    // Q1 apply modes from the stored eigen-records, everything else on the fly
    const pf_status sq = launch_cell_q1s_d(g, cp, mode, x, U, phit, mask, y, s, &handled);
    if (handled) return sq;
    return launch_cell_generic_d(g, cp, mode, x, U, phit, mask, y, s);
  }
  pf_status st = launch_cell_q1_d(g, cp, mode, x, U, phit, mask, y, s, &handled);
  if (handled) return st;
  st = launch_cell_q2_d(g, cp, mode, x, U, phit, mask, y, s, &handled);
  if (handled) return st;
  return launch_cell_generic_d(g, cp, mode, x, U, phit, mask, y, s);
}
template <>
pf_status launch_cell<float>(const Geom& g, const CellParams& cp, int mode, const float* x, const float* U,
                             const float* phit, const uint8_t* mask, float* y, hipStream_t s) {
  bool handled = false;
  if (cp.split) {
    const pf_status sq = launch_cell_q1s_f(g, cp, mode, x, U, phit, mask, y, s, &handled);
    if (handled) return sq;
    return launch_cell_generic_f(g, cp, mode, x, U, phit, mask, y, s);
  }
  pf_status st = launch_cell_q1_f(g, cp, mode, x, U, phit, mask, y, s, &handled);
  if (handled) return st;
  st = launch_cell_q2_f(g, cp, mode, x, U, phit, mask, y, s, &handled);
  if (handled) return st;
  return launch_cell_generic_f(g, cp, mode, x, U, phit, mask, y, s);
}

// modes whose output starts from Pi_C x (identity rows on constrained DoFs)
static bool starts_from_constrained(int mode) { return mode == MODE_APPLY || mode == MODE_BLOCK; }

// the cell loop for (cp, mode) is a tiled Q1 kernel, which writes every entry of y itself
static bool tiled_writes_all(const Geom& g, const CellParams& cp, int mode) {
  return !cp.split && q1_tiled_handles(g, mode, cp.variant);
}

// overwrite y with the operator result on one level's data
template <typename T>
pf_status apply_op(const Geom& g, const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                   const uint8_t* mask, T* y, hipStream_t s, bool y_preset = false) {
  if (tiled_writes_all(g, cp, mode) || (sizeof(T) == 8 && !cp.split && q1_aux_handles(g, mode))) {
    // the tiled kernels write every entry, identity rows included
  } else if (starts_from_constrained(mode)) {
    // y = Pi_C x, unless the producer of x already wrote it
    if (!y_preset) PFF_TRY(vec_init_constrained<T>(y, x, mask, g.n_nodes, g.d, s));
  } else {
    PFF_TRY(vec_fill<T>(y, T(0), g.n_dofs, s));
  }
  PFF_TRY(launch_cell<T>(g, cp, mode, x, U, phit, mask, y, s));
  if (mode == MODE_DIAG) PFF_TRY(vec_set_constrained<T>(y, T(1), mask, g.n_nodes, g.d, s));
  return PF_OK;
}

// y = constrained ? 0 : x  (with type conversion)
template <typename Tin, typename Tout>
__global__ void k_mask_free(Tout* y, const Tin* x, const uint8_t* mask, int64_t nn, int d) {
  // node-major: one mask byte per node, the components without a 64-bit division per value
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nn; j += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t m = mask[j];
    for (int c = 0; c <= d; ++c) {
      const int64_t i = (int64_t)c * nn + j;
      y[i] = (m & mask_bit(c, d)) ? Tout(0) : (Tout)x[i];
    }
  }
}
template <typename Tin, typename Tout>
pf_status mask_free(Tout* y, const Tin* x, const uint8_t* mask, int64_t nn, int d, hipStream_t s) {
  int64_t nb = std::min<int64_t>(65536, std::max<int64_t>(1, (nn + 255) / 256));
  k_mask_free<Tin, Tout><<<nb, 256, 0, s>>>(y, x, mask, nn, d);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

// eigenvalues of a symmetric tridiagonal matrix by Sturm-sequence bisection
static int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    q = a[i] - x - (i ? bb / q : 0.0);
    if (q == 0.0) q = 1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}
static double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int k) {
  // k-th smallest eigenvalue (0-based)
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < a.size(); ++i) {
    double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(a, b, mid) > k)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace pff

using namespace pff;

// reduction scratch of one concurrent level task (partials of two segments + results)
constexpr size_t kPartStride = 2 * kRedMaxBlocks + 256;
// FGMRES scalars per Arnoldi step, device dscal[0 .. kHostScal): h1 at 0, h2 at 256, |w|^2 at 512
constexpr int kHostScal = 520;
constexpr int kKernelTimerMax = 1024;  // timed launches kept per pf_set_kernel_timing period

// autotuner candidates measured per level, precision and operator
constexpr int kTuneSlots = 20;

struct LevelBuf {
  Geom g;
  double *U = nullptr, *phit = nullptr, *diag = nullptr;
  float *U32 = nullptr, *phit32 = nullptr, *diag32 = nullptr;
  double* rec64 = nullptr;  // split: per-point eigen-records of U (Q1 levels), FP64 and FP32
  float* rec32 = nullptr;
  double* cb64 = nullptr;   // without the split: B~'s per-point coefficients (Q1: c_phi JxW; 3D Q2:
                            // g(phi~) JxW and c_phi), FP64 and FP32
  float* cb32 = nullptr;
  double cb_pres = std::numeric_limits<double>::quiet_NaN();  // pressure the coefficients hold
  uint8_t *base = nullptr, *mask = nullptr;
  void *vb = nullptr, *vx = nullptr, *vr = nullptr, *vt = nullptr, *vd = nullptr;
  double eig[4] = {1, 1, 1, 1};
  bool eig_fixed = false;
  int64_t n_active_cells = 0;
  int64_t n_domain_nodes = 0;
  // cell-loop choice per [precision][mode APPLY/BLOCK]: variant and marching chunk (-1: heuristic)
  int variant[2][2] = {{-1, -1}, {-1, -1}};
  int zc[2][2] = {{-1, -1}, {-1, -1}};
  double tune_us[2][2][kTuneSlots] = {};  // measured candidates (autotune report)
  // per precision: whether the smoother's Chebyshev steps run fused into the marching-tile B~
  // (PF_FUSE_TUNED), and the autotuner's times of one step unfused / fused (us, 0 = not timed)
  bool fuse[2] = {false, false};
  double fuse_us[2][2] = {};
};

struct pf_ctx {
  pf_mesh mesh;
  int device = 0;  // the HIP device current at pf_setup
  Material mat;
  pf_options opt;
  std::vector<LevelBuf> lev;
  double *M = nullptr, *R = nullptr, *dl = nullptr, *Rt = nullptr, *dU = nullptr, *t = nullptr;
  uint8_t *extra = nullptr, *active = nullptr, *prev_active = nullptr;
  uint8_t* free_mask = nullptr;  // finest level, all zero: no DoF constrained
  double *V = nullptr, *Z = nullptr;
  double *part = nullptr, *part_md = nullptr, *dscal = nullptr;
  EigDev* eigdev = nullptr;  // one record per level
  // Chebyshev coefficients in device memory, 4 per step ({c1, c2} of the displacement block, then of
  // the phase-field block): the smoother of each level (cheb_degree steps), then the coarse solve
  // (coarse_degree steps), then one step of the autotuner's timing runs.  Kernels read them there,
  // so a captured V-cycle stays valid when the eigenvalue bounds change.
  double* dcoef = nullptr;
  bool coef_stale = true;    // host bounds changed since the last upload
  bool dense_stale = false;  // level-0 bounds changed: the dense coarse matrix is rebuilt before the next V-cycle
  // captured V-cycles per precision (finest-level vb -> vx); invalid after any change of
  // operator parameters, kernel tuning or the path of the coarse solve
  hipStream_t cap_stream = nullptr;
  // per-level helper streams of the linearization set-up (diagonals and eigenvalue CGs of
  // all levels run concurrently), their join events, and per-level reduction scratch
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> aux_ev;
  hipEvent_t fork_ev = nullptr;
  double* part_lev = nullptr;
  double* qpart = nullptr;      // reduction scratch of the quantities of interest
  double* host_scal = nullptr;  // pinned host copy of the FGMRES scalars (kHostScal doubles)
  // optional HIP-event timing of the finest-level FP64 cell kernels (pf_set_kernel_timing):
  // record 0 = Jacobian G~, record 1 = block operator B~
  // record 2 = B~ applies that carry a fused Chebyshev step
  int ktime_mask = 0;
  int ktime_every = 1;               // bracket every ktime_every-th launch of a record
  int64_t ktime_seen[3] = {0, 0, 0};  // launches seen since the record was cleared
  int ktime_n[3] = {0, 0, 0};
  std::vector<hipEvent_t> ktime_ev[3];  // pairs (start, end), kKernelTimerMax of them per record
  int cheb_fusion = PF_FUSE_TUNED;  // Chebyshev steps fused into marching-tile B~ applies (pf_set_smoother_fusion)
  hipGraph_t vgraph[2] = {nullptr, nullptr};
  hipGraphExec_t vexec[2] = {nullptr, nullptr};
  bool vvalid[2] = {false, false};
  bool use_graphs = false;
  int64_t n_captures = 0;
  // coarse solve: PF_COARSE_AUTO = the dense matrix of the fixed Chebyshev solve (small Q1 coarse
  // levels, built once per linearization) else the single-workgroup kernel; PF_COARSE_FUSED;
  // PF_COARSE_STEPS = one launch per operator apply and vector step
  int coarse_mode = PF_COARSE_AUTO;
  double* Sc = nullptr;  // dense coarse-solve matrix: built column-major here (Rc: per-column scratch),
  double* Rc = nullptr;  // then transposed into Rc, which the V-cycle reads row by row
  bool coarse_dense_ok = false;
  void drop_graphs() {
    for (int k = 0; k < 2; ++k) {
      if (vexec[k]) hipGraphExecDestroy(vexec[k]);
      if (vgraph[k]) hipGraphDestroy(vgraph[k]);
      vexec[k] = nullptr;
      vgraph[k] = nullptr;
      vvalid[k] = false;
    }
  }
  ~pf_ctx() {
    drop_graphs();
    if (cap_stream) hipStreamDestroy(cap_stream);
    for (hipStream_t a : aux) hipStreamDestroy(a);
    for (hipEvent_t e : aux_ev) hipEventDestroy(e);
    if (fork_ev) hipEventDestroy(fork_ev);
    if (host_scal) hipHostFree(host_scal);
    for (int k = 0; k < 3; ++k)
      for (hipEvent_t e : ktime_ev[k]) hipEventDestroy(e);
  }
  bool has_extra = false, has_lin = false;
  size_t ws_bytes = 0;
  int vprec = PF_F64;
};

namespace {

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

pf_status validate_mesh(const pf_mesh* m) {
  if (!m) {
    set_error("mesh is NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (m->dim != 2 && m->dim != 3) {
    set_error("dim must be 2 or 3");
    return PF_ERR_UNSUPPORTED;
  }
  if (m->degree != 1 && m->degree != 2) {
    set_error("degree must be 1 or 2");
    return PF_ERR_UNSUPPORTED;
  }
  if (m->n_levels < 1 || m->n_levels > 16) {
    set_error("n_levels must be in [1, 16]");
    return PF_ERR_INVALID_ARG;
  }
  if (m->domain != PF_BOX && m->domain != PF_LSHAPE) {
    set_error("domain must be PF_BOX or PF_LSHAPE");
    return PF_ERR_INVALID_ARG;
  }
  const int s = 1 << (m->n_levels - 1);
  for (int k = 0; k < m->dim; ++k) {
    if (m->n_cells[k] < 1 || m->n_cells[k] % s != 0) {
      set_error("n_cells must be positive and divisible by 2^(n_levels-1)");
      return PF_ERR_INVALID_ARG;
    }
    if (!(m->extent[k] > 0.0) || !std::isfinite(m->extent[k])) {
      set_error("extent must be positive and finite");
      return PF_ERR_INVALID_ARG;
    }
    if ((int64_t)m->n_cells[k] * m->degree + 1 > (1 << 24)) {
      set_error("too many nodes per axis");
      return PF_ERR_INVALID_ARG;
    }
  }
  if (m->domain == PF_LSHAPE) {
    for (int k = 0; k < 2; ++k)
      if ((m->n_cells[k] / s) % 2 != 0) {
        set_error("L-shape needs an even number of coarsest-level cells in x and y");
        return PF_ERR_INVALID_ARG;
      }
  }
  if (m->dirichlet_faces >> (2 * m->dim)) {
    set_error("dirichlet_faces has bits beyond 2*dim");
    return PF_ERR_INVALID_ARG;
  }
  return PF_OK;
}

pf_status validate_opts(const pf_options* o) {
  if (o->vcycle_precision != PF_F64 && o->vcycle_precision != PF_F32) {
    set_error("vcycle_precision must be PF_F64 or PF_F32");
    return PF_ERR_INVALID_ARG;
  }
  if (o->cheb_degree < 1 || o->cheb_degree > 64 || o->coarse_degree < 1 || o->coarse_degree > 256 ||
      o->coarse_sweeps < 1 || o->coarse_sweeps > 64) {
    set_error("Chebyshev degrees / sweeps out of range");
    return PF_ERR_INVALID_ARG;
  }
  if (!(o->cheb_ratio > 1.0) || !(o->cheb_safety > 0.0) || !(o->coarse_lo_factor > 0.0)) {
    set_error("Chebyshev range factors out of range");
    return PF_ERR_INVALID_ARG;
  }
  if (o->eig_cg_steps < 1 || o->eig_cg_steps > 100) {
    set_error("eig_cg_steps must be in [1, 100]");
    return PF_ERR_INVALID_ARG;
  }
  if (o->gmres_restart < 1 || o->gmres_restart > 200 || o->gmres_max_iter < 1 || !(o->gmres_rtol > 0.0)) {
    set_error("FGMRES settings out of range (restart in [1, 200])");
    return PF_ERR_INVALID_ARG;
  }
  if (!std::isfinite(o->gmres_atol) || !(o->gmres_atol >= 0.0)) {
    set_error("gmres_atol must be finite and >= 0");
    return PF_ERR_INVALID_ARG;
  }
  if (!std::isfinite(o->pdas_c) || !(o->pdas_c >= 0.0)) {
    set_error("pdas_c must be finite and >= 0");
    return PF_ERR_INVALID_ARG;
  }
  if (o->preconditioner != PF_PREC_FULL && o->preconditioner != PF_PREC_DIAG) {
    set_error("preconditioner must be PF_PREC_FULL or PF_PREC_DIAG");
    return PF_ERR_INVALID_ARG;
  }
  if (o->stress_split != PF_SPLIT_NONE && o->stress_split != PF_SPLIT_MIEHE) {
    set_error("stress_split must be PF_SPLIT_NONE or PF_SPLIT_MIEHE");
    return PF_ERR_INVALID_ARG;
  }
  return PF_OK;
}

Geom level_geom(const pf_mesh& m, int l) {
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

// The coarse solve is a fixed linear map during a Newton step (a Chebyshev polynomial with
// coefficients fixed by the level's lambda bounds).  For a small Q1 coarsest level it is
// cheaper to form its matrix once per linearization, one workgroup per unit vector, and apply
// it as one dense matvec per V-cycle than to run 2 x 20 latency-bound steps every time.
constexpr int64_t kDenseCoarseMaxDofs = 1024;
bool dense_coarse_eligible(const Geom& g0, const pf_options& o) {
  return g0.p == 1 && g0.n_dofs <= kDenseCoarseMaxDofs && o.stress_split == PF_SPLIT_NONE &&
         o.coarse_degree <= 64;
}

// Carve every device buffer; with base == nullptr only the size is computed.
size_t carve(pf_ctx* c, const pf_mesh& m, const pf_options& o, char* base) {
  Carver cv{base};
  const int L = m.n_levels;
  std::vector<LevelBuf> lev(L);
  for (int l = 0; l < L; ++l) {
    LevelBuf& b = lev[l];
    b.g = level_geom(m, l);
    const size_t nn = b.g.n_nodes, nd = b.g.n_dofs;
    b.U = cv.take<double>(nd);
    b.phit = cv.take<double>(nn);
    b.diag = cv.take<double>(nd);
    b.U32 = cv.take<float>(nd);
    b.phit32 = cv.take<float>(nn);
    b.diag32 = cv.take<float>(nd);
    b.base = cv.take<uint8_t>(nn);
    b.mask = cv.take<uint8_t>(nn);
    b.vb = cv.take<double>(nd);
    b.vx = cv.take<double>(nd);
    b.vr = cv.take<double>(nd);
    b.vt = cv.take<double>(nd);
    b.vd = cv.take<double>(nd);
    if (o.stress_split == PF_SPLIT_MIEHE && b.g.p == 1) {
      const size_t nr = (size_t)split_record_values(b.g.d) * (size_t)b.g.n_cells;
      b.rec64 = cv.take<double>(nr);
      b.rec32 = cv.take<float>(nr);
    }
    if (o.stress_split == PF_SPLIT_NONE && (b.g.p == 1 || b.g.d == 3)) {
      const size_t per = b.g.p == 1 ? (size_t)q1_block_coef_values(b.g.d) : (size_t)kQ2BlockCoefValues;
      const size_t nq = per * (size_t)b.g.n_cells;
      b.cb64 = cv.take<double>(nq);
      b.cb32 = cv.take<float>(nq);
    }
  }
  const Geom& gf = lev[L - 1].g;
  const size_t nn = gf.n_nodes, nd = gf.n_dofs;
  const int mr = o.gmres_restart;
  double* M = cv.take<double>(nn);
  double* R = cv.take<double>(nd);
  double* dl = cv.take<double>(nd);
  double* Rt = cv.take<double>(nd);
  double* dU = cv.take<double>(nd);
  double* t = cv.take<double>(nd);
  uint8_t* extra = cv.take<uint8_t>(nn);
  uint8_t* active = cv.take<uint8_t>(nn);
  uint8_t* prev_active = cv.take<uint8_t>(nn);
  uint8_t* free_mask = cv.take<uint8_t>(nn);
  double* V = cv.take<double>((size_t)(mr + 1) * nd);
  double* Z = cv.take<double>((size_t)mr * nd);
  double* part = cv.take<double>(2 * kRedMaxBlocks + 256);
  double* part_md = cv.take<double>((size_t)kMultiDotBlocks * (mr + 2));
  double* dscal = cv.take<double>(1024);
  EigDev* eigdev = cv.take<EigDev>(L);
  double* part_lev = cv.take<double>((size_t)L * kPartStride);
  double* qpart = cv.take<double>(3 * 1024 + 64);
  double* dcoef = cv.take<double>(4 * ((size_t)L * o.cheb_degree + o.coarse_degree + 1));
  double *Sc = nullptr, *Rc = nullptr;
  if (dense_coarse_eligible(lev[0].g, o)) {
    const size_t n0 = (size_t)lev[0].g.n_dofs;
    Sc = cv.take<double>(n0 * n0);
    Rc = cv.take<double>(n0 * n0);
  }
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
    c->prev_active = prev_active;
    c->free_mask = free_mask;
    c->V = V;
    c->Z = Z;
    c->part = part;
    c->part_md = part_md;
    c->dscal = dscal;
    c->eigdev = eigdev;
    c->part_lev = part_lev;
    c->qpart = qpart;
    c->dcoef = dcoef;
    c->Sc = Sc;
    c->Rc = Rc;
  }
  return cv.off + 256;
}

CellParams cparams(pf_ctx* c, int l) { return make_cell_params(c->lev[l].g, c->mat); }

int level_prec(pf_ctx* c, int l, int vprec) { return l == 0 ? PF_F64 : vprec; }

// ---------------------------------------------------------------------------
// operator on level l in precision prec (x, y point to that precision)
// ---------------------------------------------------------------------------
CellParams level_params(pf_ctx* c, int l, int prec, int mode) {
  LevelBuf& b = c->lev[l];
  CellParams cp = cparams(c, l);
  if (mode == MODE_APPLY || mode == MODE_BLOCK) {
    const int pi = prec == PF_F64 ? 0 : 1, mi = mode == MODE_APPLY ? 0 : 1;
    cp.variant = b.variant[pi][mi];
    cp.zc = b.zc[pi][mi];
    if (cp.split) cp.qpd = prec == PF_F64 ? (const void*)b.rec64 : (const void*)b.rec32;
    if (mode == MODE_BLOCK && b.cb64) cp.qcb = prec == PF_F64 ? (const void*)b.cb64 : (const void*)b.cb32;
  }
  return cp;
}

// the per-point coefficients of B~ on a level from its linearization point and the current pressure
pf_status refresh_block_coef(pf_ctx* c, int l, hipStream_t s) {
  LevelBuf& b = c->lev[l];
  if (!b.cb64) return PF_OK;
  if (b.g.p == 1)
    PFF_TRY(launch_block_coef(b.g, cparams(c, l), b.U, b.cb64, b.cb32, s));
  else
    PFF_TRY(launch_block_coef_q2(b.g, cparams(c, l), b.U, b.phit, b.cb64, b.cb32, s));
  b.cb_pres = c->mat.p;
  return PF_OK;
}

// whether the (level, prec, mode) operator starts from y = Pi_C x written by a separate pass
bool apply_needs_preset(pf_ctx* c, int l, int prec, int mode) {
  const CellParams cp = level_params(c, l, prec, mode);
  return !tiled_writes_all(c->lev[l].g, cp, mode);
}

// y_preset: the caller already stored y = Pi_C x (fused into the kernel that produced x)
pf_status level_apply(pf_ctx* c, int l, int prec, int mode, const void* x, void* y, hipStream_t s,
                      bool y_preset = false) {
  LevelBuf& b = c->lev[l];
  // a pressure set since the linearization reaches B~ through its coefficients
  if (mode == MODE_BLOCK && b.cb64 && !(b.cb_pres == c->mat.p)) PFF_TRY(refresh_block_coef(c, l, s));
  const CellParams cp = level_params(c, l, prec, mode);
  const int kop = mode == MODE_APPLY ? 0 : (mode == MODE_BLOCK ? 1 : -1);
  if (kop >= 0 && ((c->ktime_mask >> kop) & 1) && prec == PF_F64 && l == (int)c->lev.size() - 1 &&
      c->ktime_seen[kop]++ % c->ktime_every == 0 && c->ktime_n[kop] < kKernelTimerMax) {
    // the Pi_C start (when needed) outside, the cell kernel alone between the two events
    if (!y_preset && !tiled_writes_all(b.g, cp, mode))
      PFF_TRY(vec_init_constrained<double>((double*)y, (const double*)x, b.mask, b.g.n_nodes, b.g.d, s));
    hipEvent_t* ev = &c->ktime_ev[kop][2 * c->ktime_n[kop]++];
    PFF_HIP(hipEventRecord(ev[0], s));
    PFF_TRY(launch_cell<double>(b.g, cp, mode, (const double*)x, b.U, b.phit, b.mask, (double*)y, s));
    PFF_HIP(hipEventRecord(ev[1], s));
    return PF_OK;
  }
  if (prec == PF_F64)
    return apply_op<double>(b.g, cp, mode, (const double*)x, b.U, b.phit, b.mask, (double*)y, s, y_preset);
  return apply_op<float>(b.g, cp, mode, (const float*)x, b.U32, b.phit32, b.mask, (float*)y, s, y_preset);
}

// Chebyshev coefficients of step k for one block: interval [lo, hi]
struct ChebCoef {
  std::vector<double> c1, c2;
};
ChebCoef cheb_coefs(double lo, double hi, int degree) {
  ChebCoef r;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  r.c1.push_back(0.0);
  r.c2.push_back(1.0 / theta);
  for (int k = 1; k < degree; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    r.c1.push_back(rn * rho);
    r.c2.push_back(2.0 * rn / delta);
    rho = rn;
  }
  return r;
}

// the device coefficient blocks (pf_ctx::dcoef)
double* smooth_coefs(pf_ctx* c, int l) { return c->dcoef + (size_t)4 * l * c->opt.cheb_degree; }
double* coarse_coefs(pf_ctx* c) { return smooth_coefs(c, (int)c->lev.size()); }
double* tune_coefs(pf_ctx* c) { return coarse_coefs(c) + (size_t)4 * c->opt.coarse_degree; }

// steps of both blocks interleaved as the kernels read them: {c1, c2} (u), {c1, c2} (phi) per step
std::vector<double> interleave(const ChebCoef& u, const ChebCoef& p) {
  std::vector<double> h(4 * u.c1.size());
  for (size_t k = 0; k < u.c1.size(); ++k) {
    h[4 * k] = u.c1[k];
    h[4 * k + 1] = u.c2[k];
    h[4 * k + 2] = p.c1[k];
    h[4 * k + 3] = p.c2[k];
  }
  return h;
}

// Level l's smoother coefficients for its current bounds -- the interval [lam_max / ratio, lam_max]
// scaled by the safety factor per block -- and on level 0 those of the coarse solve, whose
// interval reaches down to a fraction of lam_min (Sec. 3.2.1, 3.2.2); written in stream order.
pf_status put_level_coefs(pf_ctx* c, int l, hipStream_t s) {
  const LevelBuf& b = c->lev[l];
  const pf_options& o = c->opt;
  const double hi[2] = {o.cheb_safety * b.eig[1], o.cheb_safety * b.eig[3]};
  const double lo[2] = {hi[0] / o.cheb_ratio, hi[1] / o.cheb_ratio};
  std::vector<double> h =
      interleave(cheb_coefs(lo[0], hi[0], o.cheb_degree), cheb_coefs(lo[1], hi[1], o.cheb_degree));
  PFF_TRY(vec_put(smooth_coefs(c, l), h.data(), (int64_t)h.size(), s));
  if (l == 0) {
    const double clo[2] = {o.coarse_lo_factor * b.eig[0], o.coarse_lo_factor * b.eig[2]};
    h = interleave(cheb_coefs(clo[0], hi[0], o.coarse_degree), cheb_coefs(clo[1], hi[1], o.coarse_degree));
    PFF_TRY(vec_put(coarse_coefs(c), h.data(), (int64_t)h.size(), s));
  }
  return PF_OK;
}
pf_status put_all_coefs(pf_ctx* c, hipStream_t s) {
  for (int l = 0; l < (int)c->lev.size(); ++l) PFF_TRY(put_level_coefs(c, l, s));
  c->coef_stale = false;
  return PF_OK;
}

// x += Cheb_B(r) with per-block intervals, starting from r as selected by first_mode
// (vec_cheb_step: 1 = b with x = 0, 2 = b - t with t = G~ x, 3 = res as given); res is
// overwritten; uses vd, vt of the level.  tail_init: the last step leaves t = Pi_C x, the
// start of a following G~ x apply.  dcoef: the degree steps' coefficients in device memory.
template <typename T>
pf_status cheb_run(pf_ctx* c, int l, int prec, T* res, T* x, const double* dcoef, int degree, int first_mode,
                   const T* bvec, bool tail_init, hipStream_t s) {
  LevelBuf& b = c->lev[l];
  T* dv = (T*)b.vd;
  T* t = (T*)b.vt;
  const T* diag = prec == PF_F64 ? (const T*)b.diag : (const T*)b.diag32;
  // the step that produces the next direction also writes t = Pi_C dv for the next apply
  const bool fuse = apply_needs_preset(c, l, prec, MODE_BLOCK);
  // Marching tiles write every node once, so the block-operator apply of steps k >= 1 can carry
  // the step's vector update itself; the direction then alternates between vd (odd k) and vt
  // (even k), and the last step (odd when the degree is even) may leave Pi_C x in vt.
  if (b.cb64 && !(b.cb_pres == c->mat.p)) PFF_TRY(refresh_block_coef(c, l, s));
  const CellParams bcp = level_params(c, l, prec, MODE_BLOCK);
  const bool want = c->cheb_fusion == PF_FUSE_ALWAYS || (c->cheb_fusion == PF_FUSE_TUNED && b.fuse[prec == PF_F64 ? 0 : 1]);
  const bool fused = want && degree >= 2 && (degree % 2 == 0 || !tail_init) && q1_block_cheb_fusable(b.g, bcp);
  const T* Ul = prec == PF_F64 ? (const T*)b.U : (const T*)b.U32;
  const T* pl = prec == PF_F64 ? (const T*)b.phit : (const T*)b.phit32;
  T* din = dv;
  for (int k = 0; k < degree; ++k) {
    if (k > 0 && fused) {
      const bool last = k + 1 == degree;
      ChebFuse<T> cf;
      cf.res = res;
      cf.diag = diag;
      cf.x = x;
      cf.d_out = last ? nullptr : (din == dv ? t : dv);
      cf.t_next = last && tail_init ? t : nullptr;
      cf.dc = dcoef + 4 * k;
      cf.next_of_x = 1;
      bool handled = false;
      const bool timed = ((c->ktime_mask >> 2) & 1) && prec == PF_F64 && l == (int)c->lev.size() - 1 &&
                         c->ktime_seen[2]++ % c->ktime_every == 0 && c->ktime_n[2] < kKernelTimerMax;
      hipEvent_t* ev = timed ? &c->ktime_ev[2][2 * c->ktime_n[2]++] : nullptr;
      if (ev) PFF_HIP(hipEventRecord(ev[0], s));
      PFF_TRY(launch_q1_block_cheb<T>(b.g, bcp, din, Ul, pl, b.mask, cf, s, &handled));
      if (ev) PFF_HIP(hipEventRecord(ev[1], s));
      if (!handled) {
        set_error("fused Chebyshev step: the level's block operator is not a marching-tile shape");
        return PF_ERR_UNSUPPORTED;
      }
      din = cf.d_out;
      continue;
    }
    if (k > 0) PFF_TRY(level_apply(c, l, prec, MODE_BLOCK, dv, t, s, fuse));
    T* t_next = nullptr;
    int next_of_x = 0;
    if (k + 1 < degree) {
      if (fuse) t_next = t;
    } else if (tail_init) {
      t_next = t;
      next_of_x = 1;
    }
    PFF_TRY(vec_cheb_step<T>(res, t, dv, x, diag, dcoef + 4 * k, k == 0 ? first_mode : 0, b.g.n_nodes, b.g.d,
                             b.mask, t_next, next_of_x, bvec, s));
  }
  return PF_OK;
}

// The operator the V-cycle forms its residuals with: G~ for P_full = MG(G~), the
// block-diagonal B~ for P_diag = diag(MG(U~), MG(P~)) (Sec. 3.3).  The transfers, the
// smoother and the coarse Chebyshev work per block in both, so with B~ the two block
// multigrids run side by side without ever mixing.
int cycle_mode(const pf_ctx* c) { return c->opt.preconditioner == PF_PREC_DIAG ? MODE_BLOCK : MODE_APPLY; }

// one smoothing step x += Cheb_B(b - G~ x); x_zero: x = 0 on entry (x is not read).
// tail_init: leave t = Pi_C x for a following G~ x apply.
template <typename T>
pf_status smooth(pf_ctx* c, int l, int prec, bool x_zero, bool tail_init, hipStream_t s) {
  LevelBuf& b = c->lev[l];
  T* bb = (T*)b.vb;
  T* x = (T*)b.vx;
  T* r = (T*)b.vr;
  if (!x_zero) PFF_TRY(level_apply(c, l, prec, cycle_mode(c), x, b.vt, s));
  return cheb_run<T>(c, l, prec, r, x, smooth_coefs(c, l), c->opt.cheb_degree, x_zero ? 1 : 2, bb, tail_init, s);
}

pf_status coarse_solve(pf_ctx* c, hipStream_t s) {
  LevelBuf& b = c->lev[0];
  double* bb = (double*)b.vb;
  double* x = (double*)b.vx;
  double* r = (double*)b.vr;
  const pf_options& o = c->opt;
  if (c->coarse_mode == PF_COARSE_AUTO && c->coarse_dense_ok) return coarse_matvec(c->Rc, bb, x, b.g.n_dofs, s);
  if (c->coarse_mode != PF_COARSE_STEPS && !c->mat.split) {
    bool handled = false;
    PFF_TRY(launch_coarse_solve(b.g, cparams(c, 0), o.coarse_degree, o.coarse_sweeps, coarse_coefs(c), b.U, b.phit,
                                b.mask, b.diag, bb, x, r, cycle_mode(c) == MODE_APPLY, s, &handled));
    if (handled) return PF_OK;
  }
  for (int sw = 0; sw < o.coarse_sweeps; ++sw) {
    if (sw > 0) PFF_TRY(level_apply(c, 0, PF_F64, cycle_mode(c), x, b.vt, s));
    // sweep 0 starts from x = 0 (r = b), later sweeps from r = b - G~ x
    PFF_TRY(cheb_run<double>(c, 0, PF_F64, r, x, coarse_coefs(c), o.coarse_degree, sw == 0 ? 1 : 2, bb, false, s));
  }
  return PF_OK;
}

// the dense matrix of the coarse solve for the current level-0 data and lambda bounds (the
// coarse coefficients must have been written on stream s)
pf_status build_coarse_dense(pf_ctx* c, hipStream_t s) {
  c->coarse_dense_ok = false;
  if (!c->Sc || c->coarse_mode != PF_COARSE_AUTO || c->mat.split) return PF_OK;
  LevelBuf& b = c->lev[0];
  const pf_options& o = c->opt;
  bool handled = false;
  PFF_TRY(launch_coarse_solve(b.g, cparams(c, 0), o.coarse_degree, o.coarse_sweeps, coarse_coefs(c), b.U, b.phit,
                              b.mask, b.diag, nullptr, c->Sc, c->Rc, cycle_mode(c) == MODE_APPLY, s, &handled,
                              true));
  if (handled) PFF_TRY(coarse_transpose(c->Sc, c->Rc, b.g.n_dofs, s));
  c->coarse_dense_ok = handled;
  return PF_OK;
}

template <typename Tf, typename Tc>
pf_status restrict_to(pf_ctx* c, int l, hipStream_t s) {
  LevelBuf& f = c->lev[l];
  LevelBuf& co = c->lev[l - 1];
  // residual r = b - G~ x of the level (b in vb, G~ x in vt), restricted without being stored
  return restrict_vec<Tf, Tc>(co.g, f.g, (const Tf*)f.vb, (const Tf*)f.vt, (Tc*)co.vb, co.mask, s);
}
template <typename Tc, typename Tf>
pf_status prolong_add(pf_ctx* c, int l, hipStream_t s) {
  LevelBuf& f = c->lev[l];
  LevelBuf& co = c->lev[l - 1];
  return prolong_vec<Tc, Tf>(co.g, f.g, (const Tc*)co.vx, (Tf*)f.vx, f.mask, 1, s);
}

pf_status vcycle_level(pf_ctx* c, int l, int vprec, hipStream_t s) {
  if (l == 0) return coarse_solve(c, s);
  const int pl = level_prec(c, l, vprec), pc = level_prec(c, l - 1, vprec);
  LevelBuf& b = c->lev[l];
  // pre-smoothing from x = 0; its last step leaves t = Pi_C x when the residual apply needs it,
  // and the residual b - G~ x is formed inside the restriction
  const int cm = cycle_mode(c);
  const bool pre_init = apply_needs_preset(c, l, pl, cm);
  if (pl == PF_F64) {
    PFF_TRY(smooth<double>(c, l, pl, true, pre_init, s));
    PFF_TRY(level_apply(c, l, pl, cm, b.vx, b.vt, s, pre_init));
    PFF_TRY(pc == PF_F64 ? restrict_to<double, double>(c, l, s) : restrict_to<double, float>(c, l, s));
  } else {
    PFF_TRY(smooth<float>(c, l, pl, true, pre_init, s));
    PFF_TRY(level_apply(c, l, pl, cm, b.vx, b.vt, s, pre_init));
    PFF_TRY(pc == PF_F64 ? restrict_to<float, double>(c, l, s) : restrict_to<float, float>(c, l, s));
  }
  PFF_TRY(vcycle_level(c, l - 1, vprec, s));
  if (pl == PF_F64) {
    PFF_TRY(pc == PF_F64 ? prolong_add<double, double>(c, l, s) : prolong_add<float, double>(c, l, s));
    PFF_TRY(smooth<double>(c, l, pl, false, false, s));
  } else {
    PFF_TRY(pc == PF_F64 ? prolong_add<double, float>(c, l, s) : prolong_add<float, float>(c, l, s));
    PFF_TRY(smooth<float>(c, l, pl, false, false, s));
  }
  return PF_OK;
}

// the finest level's right-hand side vb = Pi_F r (in the level's precision), and z = Pi_F vx
pf_status vcycle_in(pf_ctx* c, int vprec, const double* r, hipStream_t s) {
  const int L = (int)c->lev.size() - 1;
  LevelBuf& f = c->lev[L];
  if (level_prec(c, L, vprec) == PF_F64)
    return mask_free<double, double>((double*)f.vb, r, f.mask, f.g.n_nodes, f.g.d, s);
  return mask_free<double, float>((float*)f.vb, r, f.mask, f.g.n_nodes, f.g.d, s);
}
pf_status vcycle_out(pf_ctx* c, int vprec, double* z, hipStream_t s) {
  const int L = (int)c->lev.size() - 1;
  LevelBuf& f = c->lev[L];
  if (level_prec(c, L, vprec) == PF_F64)
    return mask_free<double, double>(z, (const double*)f.vx, f.mask, f.g.n_nodes, f.g.d, s);
  return mask_free<float, double>(z, (const float*)f.vx, f.mask, f.g.n_nodes, f.g.d, s);
}

pf_status vcycle(pf_ctx* c, int vprec, const double* r, double* z, hipStream_t s) {
  PFF_TRY(vcycle_in(c, vprec, r, s));
  PFF_TRY(vcycle_level(c, (int)c->lev.size() - 1, vprec, s));
  return vcycle_out(c, vprec, z, s);
}

// The V-cycle has no host decision inside, and every value that changes with the
// linearization (level data, diagonals, Chebyshev coefficients, the dense coarse
// matrix) is read from device buffers that keep their addresses, so it is
// captured once into a hipGraph (per precision) on a private stream and replayed
// on the caller's stream across linearizations: one launch instead of ~10 per
// level per smoothing step.  The capture covers the levels only (finest-level
// vb -> vx); the masked copies in and out, whose vectors change with every call,
// run as ordinary launches around the replay.  A new pressure, kernel tuning or
// coarse-solve path changes kernel arguments or the launch sequence and drops
// the capture.
pf_status vcycle_graph(pf_ctx* c, int vprec, const double* r, double* z, hipStream_t s) {
  const int k = vprec == PF_F64 ? 0 : 1;
  if (!c->vvalid[k]) {
    // B~'s per-point coefficients follow a pressure set since the linearization here, on the
    // caller's stream, so that the capture does not record their refresh
    for (int l = 0; l < (int)c->lev.size(); ++l)
      if (c->lev[l].cb64 && !(c->lev[l].cb_pres == c->mat.p)) PFF_TRY(refresh_block_coef(c, l, s));
    if (!c->cap_stream) PFF_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (c->vexec[k]) hipGraphExecDestroy(c->vexec[k]);
    if (c->vgraph[k]) hipGraphDestroy(c->vgraph[k]);
    c->vexec[k] = nullptr;
    c->vgraph[k] = nullptr;
    PFF_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const pf_status st = vcycle_level(c, (int)c->lev.size() - 1, vprec, c->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != PF_OK || e != hipSuccess) {
      if (g) hipGraphDestroy(g);
      if (st == PF_OK) set_error(std::string("V-cycle capture: ") + hipGetErrorString(e));
      return st != PF_OK ? st : PF_ERR_DEVICE;
    }
    c->vgraph[k] = g;
    PFF_HIP(hipGraphInstantiate(&c->vexec[k], g, nullptr, nullptr, 0));
    c->vvalid[k] = true;
    ++c->n_captures;
  }
  PFF_TRY(vcycle_in(c, vprec, r, s));
  PFF_HIP(hipGraphLaunch(c->vexec[k], s));
  return vcycle_out(c, vprec, z, s);
}

pf_status vcycle_any(pf_ctx* c, int vprec, const double* r, double* z, hipStream_t s) {
  if (c->coef_stale) PFF_TRY(put_all_coefs(c, s));
  if (c->dense_stale) {
    // same path, new matrix (in place): a captured V-cycle stays valid
    PFF_TRY(build_coarse_dense(c, s));
    c->dense_stale = false;
    if (!c->coarse_dense_ok) c->drop_graphs();
  }
  // kernel timing records events between launches: timed runs launch eagerly
  return c->use_graphs && !c->ktime_mask ? vcycle_graph(c, vprec, r, z, s) : vcycle(c, vprec, r, z, s);
}

// ---------------------------------------------------------------------------
// eigenvalue estimates: PCG on D^{-1} B~_bb per block (both blocks in one apply)
// ---------------------------------------------------------------------------
// Launch the Jacobi-PCG of level l (both diagonal blocks, lockstep); the
// coefficients stay in c->eigdev[l] until eig_from_cg reads them.
template <typename T>
static pf_status eig_cg_run(pf_ctx* c, int l, int prec, double* part, hipStream_t s) {
  LevelBuf& b = c->lev[l];
  const Geom& g = b.g;
  T* r = (T*)b.vr;
  T* z = (T*)b.vd;
  T* p = (T*)b.vb;
  T* Ap = (T*)b.vt;
  const T* diag = prec == PF_F64 ? (const T*)b.diag : (const T*)b.diag32;
  EigDev* st = c->eigdev + l;
  const uint64_t seed = c->opt.eig_seed;
  const uint64_t su = seed + (uint64_t)l * 0x1000003ull + 0ull * 0x10001ull;
  const uint64_t sp = seed + (uint64_t)l * 0x1000003ull + 1ull * 0x10001ull;
  PFF_TRY(eig_start_vector<T>(r, b.mask, g.n_nodes, g.d, su, sp, s));
  PFF_TRY(eig_cg_begin<T>(r, z, p, diag, b.mask, g.n_nodes, g.d, part, st, s));
  for (int it = 0; it < c->opt.eig_cg_steps; ++it) {
    PFF_TRY(level_apply(c, l, prec, MODE_BLOCK, p, Ap, s));
    PFF_TRY(eig_cg_alpha<T>(p, Ap, g.n_nodes, g.d, part, st, s));
    PFF_TRY(eig_cg_beta<T>(r, Ap, z, p, diag, b.mask, g.n_nodes, g.d, part, st, s));
  }
  return PF_OK;
}

// The eigenvalue CG of a level runs in the precision the V-cycle applies that level's operator
// in: FP64 for FP64 V-cycles and the coarsest level, FP32 on the other levels of FP32 V-cycles
// (the bounds only place the Chebyshev interval, which carries a 1.2 safety factor).
pf_status launch_eig_cg(pf_ctx* c, int l, double* part, hipStream_t s) {
  const int prec = level_prec(c, l, c->vprec);
  return prec == PF_F64 ? eig_cg_run<double>(c, l, prec, part, s) : eig_cg_run<float>(c, l, prec, part, s);
}

// Lanczos tridiagonal of the CG coefficients -> extreme eigenvalues per block
void eig_from_cg(const EigDev& e, double eig[4]) {
  for (int k = 0; k < 2; ++k) {
    const int n = e.n_al[k];
    if (n == 0) {
      eig[2 * k] = 1.0;
      eig[2 * k + 1] = 1.0;
      continue;
    }
    std::vector<double> a(n), off(n > 1 ? n - 1 : 0);
    for (int j = 0; j < n; ++j) {
      a[j] = 1.0 / e.al[k][j] + (j ? e.be[k][j - 1] / e.al[k][j - 1] : 0.0);
      if (j + 1 < n) off[j] = std::sqrt(e.be[k][j]) / e.al[k][j];
    }
    eig[2 * k] = tridiag_eig(a, off, 0);
    eig[2 * k + 1] = tridiag_eig(a, off, n - 1);
  }
}

// read back the CG coefficients of every level without fixed bounds (after the level tasks)
pf_status eig_readback(pf_ctx* c, hipStream_t s) {
  const int L = (int)c->lev.size();
  bool any = false;
  for (int l = 0; l < L; ++l) any = any || !c->lev[l].eig_fixed;
  if (!any) return PF_OK;
  std::vector<EigDev> h(L);
  PFF_HIP(hipMemcpyAsync(h.data(), c->eigdev, sizeof(EigDev) * L, hipMemcpyDeviceToHost, s));
  PFF_HIP(hipStreamSynchronize(s));
  for (int l = 0; l < L; ++l)
    if (!c->lev[l].eig_fixed) eig_from_cg(h[l], c->lev[l].eig);
  return PF_OK;
}

// the eigenvalue bounds of one level from its CG record (waits for stream s)
pf_status eig_readback_level(pf_ctx* c, int l, hipStream_t s) {
  if (c->lev[l].eig_fixed) return PF_OK;
  EigDev h;
  PFF_HIP(hipMemcpyAsync(&h, c->eigdev + l, sizeof(EigDev), hipMemcpyDeviceToHost, s));
  PFF_HIP(hipStreamSynchronize(s));
  eig_from_cg(h, c->lev[l].eig);
  return PF_OK;
}

// helper streams and events of the level tasks (created on first use)
pf_status ensure_aux(pf_ctx* c) {
  const size_t L = c->lev.size();
  if (!c->fork_ev) PFF_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  while (c->aux.size() < L) {
    hipStream_t a;
    PFF_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
    c->aux.push_back(a);
  }
  while (c->aux_ev.size() < L) {
    hipEvent_t e;
    PFF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->aux_ev.push_back(e);
  }
  return PF_OK;
}

// per-level set-up task: split eigen-records or B~ coefficients, diagonal of B~, FP32 copies,
// eigenvalue CG
pf_status level_task(pf_ctx* c, int l, hipStream_t s) {
  LevelBuf& b = c->lev[l];
  if (b.rec64) PFF_TRY(launch_split_data(b.g, cparams(c, l), b.U, b.rec64, b.rec32, s));
  PFF_TRY(refresh_block_coef(c, l, s));
  PFF_TRY(apply_op<double>(b.g, cparams(c, l), MODE_DIAG, nullptr, b.U, b.phit, b.mask, b.diag, s));
  PFF_TRY(vec_cast<double, float>(b.U32, b.U, b.g.n_dofs, s));
  PFF_TRY(vec_cast<double, float>(b.phit32, b.phit, b.g.n_nodes, s));
  PFF_TRY(vec_cast<double, float>(b.diag32, b.diag, b.g.n_dofs, s));
  if (!b.eig_fixed) PFF_TRY(launch_eig_cg(c, l, c->part_lev + (size_t)l * kPartStride, s));
  return PF_OK;
}

pf_status set_linearization(pf_ctx* c, const double* U, const double* phit, const uint8_t* active, hipStream_t s) {
  const int L = (int)c->lev.size() - 1;
  LevelBuf& f = c->lev[L];
  PFF_TRY(vec_copy<double>(f.U, U, f.g.n_dofs, s));
  PFF_TRY(vec_copy<double>(f.phit, phit, f.g.n_nodes, s));
  PFF_TRY(combine_mask(f.base, c->has_extra ? c->extra : nullptr, active, f.mask, f.g.n_nodes, s));
  for (int l = L - 1; l >= 0; --l) {
    LevelBuf& co = c->lev[l];
    LevelBuf& fi = c->lev[l + 1];
    PFF_TRY(inject<double>(co.g, fi.g, fi.U, co.U, co.g.d + 1, s));
    PFF_TRY(inject<double>(co.g, fi.g, fi.phit, co.phit, 1, s));
    PFF_TRY(inject_mask(co.g, fi.g, fi.mask, co.base, co.mask, s));
  }
  // the levels are independent from here on: one task per level on its own stream, the
  // finest on the caller's stream, joined before the coefficients are read back
  PFF_TRY(ensure_aux(c));
  PFF_HIP(hipEventRecord(c->fork_ev, s));
  for (int l = 0; l < L; ++l) {
    PFF_HIP(hipStreamWaitEvent(c->aux[l], c->fork_ev, 0));
    PFF_TRY(level_task(c, l, c->aux[l]));
    PFF_HIP(hipEventRecord(c->aux_ev[l], c->aux[l]));
  }
  PFF_TRY(level_task(c, L, s));
  const bool dense_before = c->coarse_dense_ok;
  if (L > 0) {
    // the dense coarse-solve matrix needs level 0 only: it is built on level 0's stream while
    // the finest level's task (queued above) still runs
    PFF_TRY(eig_readback_level(c, 0, c->aux[0]));
    PFF_TRY(put_level_coefs(c, 0, c->aux[0]));
    PFF_TRY(build_coarse_dense(c, c->aux[0]));
    PFF_HIP(hipEventRecord(c->aux_ev[0], c->aux[0]));
  }
  for (int l = 0; l < L; ++l) PFF_HIP(hipStreamWaitEvent(s, c->aux_ev[l], 0));
  PFF_TRY(eig_readback(c, s));
  for (int l = L > 0 ? 1 : 0; l <= L; ++l) PFF_TRY(put_level_coefs(c, l, s));
  if (L == 0) PFF_TRY(build_coarse_dense(c, s));
  PFF_HIP(hipStreamSynchronize(s));
  c->coef_stale = false;
  c->dense_stale = false;
  c->has_lin = true;
  // a captured V-cycle reads everything above in place; only a change of the coarse path
  // (dense matrix or Chebyshev kernel) changes its launch sequence
  if (c->coarse_dense_ok != dense_before) c->drop_graphs();
  return PF_OK;
}

// Givens-based FGMRES(m), right preconditioned by the V-cycle, CGS2 Arnoldi.
pf_status fgmres(pf_ctx* c, const double* b, double* x, int vprec, int* iters, double* rel, double* bnorm_out,
                 hipStream_t s) {
  const int L = (int)c->lev.size() - 1;
  LevelBuf& f = c->lev[L];
  const int64_t n = f.g.n_dofs;
  const int m = c->opt.gmres_restart;
  double bn2 = 0;
  PFF_TRY(dot_host(b, b, n, c->part, &bn2, s));
  const double bnorm = std::sqrt(bn2);
  *bnorm_out = bnorm;
  const double tol = std::max(c->opt.gmres_rtol * bnorm, c->opt.gmres_atol);
  auto true_res = [&](double* beta) -> pf_status {
    PFF_TRY(level_apply(c, L, PF_F64, MODE_APPLY, x, c->t, s));
    PFF_TRY(vec_sub<double>(c->V, b, c->t, n, s));
    double r2 = 0;
    PFF_TRY(dot_host(c->V, c->V, n, c->part, &r2, s));
    *beta = std::sqrt(r2);
    return PF_OK;
  };
  double beta = 0;
  PFF_TRY(true_res(&beta));
  int total = 0;
  std::vector<double> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), y(m);
  std::vector<double> hbuf(2);
  if (!c->host_scal) PFF_HIP(hipHostMalloc((void**)&c->host_scal, sizeof(double) * kHostScal, hipHostMallocDefault));
  double* hs = c->host_scal;
  while (beta > tol && total < c->opt.gmres_max_iter) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    // V_0 = r / beta (r already in V_0)
    double* dnorm = c->dscal + 520;
    hbuf[0] = beta * beta;
    PFF_HIP(hipMemcpyAsync(dnorm, hbuf.data(), sizeof(double), hipMemcpyHostToDevice, s));
    PFF_TRY(vec_scale_inv_sqrt(c->V, c->V, dnorm, n, s));
    PFF_HIP(hipStreamSynchronize(s));
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = c->V + (int64_t)j * n;
      double* zj = c->Z + (int64_t)j * n;
      double* w = c->V + (int64_t)(j + 1) * n;
      PFF_TRY(vcycle_any(c, vprec, vj, zj, s));
      PFF_TRY(level_apply(c, L, PF_F64, MODE_APPLY, zj, w, s));
      double* h1 = c->dscal;
      double* h2 = c->dscal + 256;
      double* nr = c->dscal + 512;
      PFF_TRY(multi_dot(c->V, n, j + 1, w, n, c->part_md, h1, s));
      if (j + 1 <= kMultiDotRows) {
        // each subtraction shares its pass over w with the reduction after it
        PFF_TRY(axpy_then_dot(w, c->V, n, j + 1, h1, n, false, c->part_md, h2, s));
        PFF_TRY(axpy_then_dot(w, c->V, n, j + 1, h2, n, true, c->part_md, nr, s));
      } else {
        PFF_TRY(multi_axpy(w, c->V, n, j + 1, h1, n, -1.0, s));
        PFF_TRY(multi_dot(c->V, n, j + 1, w, n, c->part_md, h2, s));
        PFF_TRY(multi_axpy(w, c->V, n, j + 1, h2, n, -1.0, s));
        PFF_TRY(nrm2_dev(w, n, c->part, nr, s));
      }
      PFF_TRY(vec_scale_inv_sqrt(w, w, nr, n, s));
      // one copy of both Gram-Schmidt passes and the norm into pinned memory
      PFF_HIP(hipMemcpyAsync(hs, c->dscal, sizeof(double) * kHostScal, hipMemcpyDeviceToHost, s));
      PFF_HIP(hipStreamSynchronize(s));
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hs[i] + hs[256 + i];
      H[(size_t)(j + 1) * m + j] = std::sqrt(std::max(0.0, hs[512]));
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], bq = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * bq;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bq;
      }
      const double a = H[(size_t)j * m + j], bq = H[(size_t)(j + 1) * m + j];
      const double den = std::hypot(a, bq);
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = a / den;
        sn[j] = bq / den;
      }
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      jend = j + 1;
      if (!std::isfinite(g[j + 1])) {
        set_error("FGMRES produced a non-finite residual estimate");
        return PF_ERR_NONFINITE;
      }
      if (std::fabs(g[j + 1]) <= tol || total >= c->opt.gmres_max_iter || den == 0.0) break;
    }
    // back substitution H y = g
    for (int i = jend - 1; i >= 0; --i) {
      double acc = g[i];
      for (int k = i + 1; k < jend; ++k) acc -= H[(size_t)i * m + k] * y[k];
      y[i] = H[(size_t)i * m + i] != 0.0 ? acc / H[(size_t)i * m + i] : 0.0;
    }
    double* dy = c->dscal + 640;
    PFF_HIP(hipMemcpyAsync(dy, y.data(), sizeof(double) * jend, hipMemcpyHostToDevice, s));
    PFF_TRY(multi_axpy(x, c->Z, n, jend, dy, n, 1.0, s));
    PFF_HIP(hipStreamSynchronize(s));
    PFF_TRY(true_res(&beta));
  }
  *iters = total;
  *rel = bnorm > 0 ? beta / bnorm : 0.0;
  return PF_OK;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

hipStream_t st(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

void pf_default_options(pf_options* o) {
  if (!o) return;
  o->vcycle_precision = PF_F64;
  o->cheb_degree = 4;
  o->cheb_ratio = 5.0;
  o->cheb_safety = 1.2;
  o->eig_cg_steps = 10;
  o->coarse_degree = 20;
  o->coarse_sweeps = 2;
  o->coarse_lo_factor = 0.9;
  o->gmres_restart = 50;
  o->gmres_max_iter = 500;
  o->gmres_rtol = 1e-8;
  o->gmres_atol = 0.0;
  o->pdas_c = 100.0;
  o->eig_seed = 12345;
  o->preconditioner = PF_PREC_FULL;
  o->stress_split = PF_SPLIT_NONE;
}

const char* pf_status_string(pf_status s) {
  switch (s) {
    case PF_OK: return "PF_OK";
    case PF_ERR_INVALID_ARG: return "PF_ERR_INVALID_ARG";
    case PF_ERR_UNSUPPORTED: return "PF_ERR_UNSUPPORTED";
    case PF_ERR_DEVICE: return "PF_ERR_DEVICE";
    case PF_ERR_WORKSPACE: return "PF_ERR_WORKSPACE";
    case PF_ERR_NOT_CONVERGED: return "PF_ERR_NOT_CONVERGED";
    case PF_ERR_NONFINITE: return "PF_ERR_NONFINITE";
    default: return "PF_ERR_UNKNOWN";
  }
}

const char* pf_last_error(void) { return g_err.c_str(); }

pf_status pf_workspace_size(const pf_mesh* mesh, const pf_options* opt, size_t* bytes) {
  if (!bytes) {
    set_error("bytes is NULL");
    return PF_ERR_INVALID_ARG;
  }
  PFF_TRY(validate_mesh(mesh));
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  PFF_TRY(validate_opts(&o));
  *bytes = carve(nullptr, *mesh, o, nullptr);
  return PF_OK;
}

pf_status pf_setup(const pf_mesh* mesh, double E, double nu, double G_c, double eps, double kappa, double pressure,
                   const pf_options* opt, void* d_workspace, size_t ws_bytes, void* stream, pf_ctx** out) {
  if (!out) {
    set_error("out is NULL");
    return PF_ERR_INVALID_ARG;
  }
  *out = nullptr;
  PFF_TRY(validate_mesh(mesh));
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  PFF_TRY(validate_opts(&o));
  if (!(E > 0.0) || !std::isfinite(E) || !(nu > -1.0 && nu < 0.5) || !(G_c > 0.0) || !std::isfinite(G_c) ||
      !(eps > 0.0) || !std::isfinite(eps) || !(kappa >= 0.0 && kappa < 1.0) || !std::isfinite(pressure)) {
    set_error("material parameters out of range (E>0, -1<nu<0.5, G_c>0, eps>0, 0<=kappa<1, finite p)");
    return PF_ERR_INVALID_ARG;
  }
  const size_t need = carve(nullptr, *mesh, o, nullptr);
  if (!d_workspace || ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return PF_ERR_WORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) {
    set_error("workspace must be 256-byte aligned");
    return PF_ERR_WORKSPACE;
  }
  int device = 0;
  PFF_HIP(hipGetDevice(&device));
  // the allocation-free entry point's scratch address on this device, resolved at set-up
  PFF_TRY(quantity_scratch_init(device));
  pf_ctx* c = new pf_ctx();
  c->device = device;
  c->mesh = *mesh;
  c->opt = o;
  c->vprec = o.vcycle_precision;
  c->mat.mu = E / (2.0 * (1.0 + nu));
  c->mat.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  c->mat.Gc = G_c;
  c->mat.eps = eps;
  c->mat.kappa = kappa;
  c->mat.p = pressure;
  c->mat.split = o.stress_split;
  c->ws_bytes = ws_bytes;
  carve(c, *mesh, o, reinterpret_cast<char*>(d_workspace));
  hipStream_t s = st(stream);
  const int L = mesh->n_levels;
  for (int l = 0; l < L; ++l) {
    LevelBuf& b = c->lev[l];
    int64_t act = 0;
    for (int64_t cy = 0; cy < b.g.N[1]; ++cy)
      for (int64_t cx = 0; cx < b.g.N[0]; ++cx) act += cell_in_hole(b.g.lshape, (int)cx, (int)cy, b.g.N[0], b.g.N[1]) ? 0 : 1;
    b.n_active_cells = act * b.g.N[2];
    // hole nodes: strictly inside the removed quadrant (all adjacent cells in the hole)
    int64_t hole = 0;
    if (b.g.lshape)
      hole = (int64_t)(b.g.nn[0] - 1 - b.g.p * (b.g.N[0] / 2)) * (b.g.nn[1] - 1 - b.g.p * (b.g.N[1] / 2)) * b.g.nn[2];
    b.n_domain_nodes = b.g.n_nodes - hole;
    pf_status r = build_base_mask(b.g, mesh->dirichlet_faces, b.base, s);
    if (r == PF_OK) r = vec_copy<uint8_t>(b.mask, b.base, b.g.n_nodes, s);
    if (r != PF_OK) {
      delete c;
      return r;
    }
  }
  pf_status r = lumped_mass(c->lev[L - 1].g, c->M, s);
  if (r == PF_OK && hipMemsetAsync(c->free_mask, 0, (size_t)c->lev[L - 1].g.n_nodes, s) != hipSuccess) {
    set_error("clearing the all-free mask failed");
    r = PF_ERR_DEVICE;
  }
  if (r != PF_OK) {
    delete c;
    return r;
  }
  *out = c;
  return PF_OK;
}

void pf_destroy(pf_ctx* ctx) { delete ctx; }

#define NEED_CTX()                     \
  if (!ctx) {                          \
    set_error("context is NULL");      \
    return PF_ERR_INVALID_ARG;         \
  }
#define NEED_LIN()                                                    \
  if (!ctx->has_lin) {                                                \
    set_error("no linearization point: call pf_set_linearization"); \
    return PF_ERR_INVALID_ARG;                                        \
  }
#define NEED_LEVEL(l)                                   \
  if ((l) < 0 || (l) >= (int)ctx->lev.size()) {         \
    set_error("level out of range");                    \
    return PF_ERR_INVALID_ARG;                          \
  }

pf_status pf_set_constraints(pf_ctx* ctx, const uint8_t* d_bits, void* stream) {
  NEED_CTX();
  if (!d_bits) {
    ctx->has_extra = false;
    return PF_OK;
  }
  LevelBuf& f = ctx->lev.back();
  PFF_TRY(vec_copy<uint8_t>(ctx->extra, d_bits, f.g.n_nodes, st(stream)));
  ctx->has_extra = true;
  return PF_OK;
}

pf_status pf_set_linearization(pf_ctx* ctx, const double* d_U, const double* d_phi_tilde, const uint8_t* d_active,
                               void* stream) {
  NEED_CTX();
  if (!d_U || !d_phi_tilde) {
    set_error("U and phi_tilde must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  return set_linearization(ctx, d_U, d_phi_tilde, d_active, st(stream));
}

static pf_status apply_entry(pf_ctx* ctx, int level, int prec, int mode, const void* d_x, void* d_y, void* stream) {
  NEED_CTX();
  NEED_LIN();
  NEED_LEVEL(level);
  if (prec != PF_F64 && prec != PF_F32) {
    set_error("prec must be PF_F64 or PF_F32");
    return PF_ERR_INVALID_ARG;
  }
  if (!d_x || !d_y) {
    set_error("x and y must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (d_x == d_y) {
    set_error("x and y must not alias");
    return PF_ERR_INVALID_ARG;
  }
  return level_apply(ctx, level, prec, mode, d_x, d_y, st(stream));
}

pf_status pf_jacobian_apply(pf_ctx* ctx, int level, int prec, const void* d_x, void* d_y, void* stream) {
  return apply_entry(ctx, level, prec, MODE_APPLY, d_x, d_y, stream);
}

pf_status pf_set_kernel_timing(pf_ctx* ctx, int enable, int every) {
  NEED_CTX();
  if (enable < 0 || enable > (PF_KTIME_JACOBIAN | PF_KTIME_BLOCK | PF_KTIME_BLOCK_CHEB)) {
    set_error("enable must be 0 or a combination of PF_KTIME_JACOBIAN, PF_KTIME_BLOCK and PF_KTIME_BLOCK_CHEB");
    return PF_ERR_INVALID_ARG;
  }
  if (every < 1 || every > 1000000) {
    set_error("every must be in [1, 1000000]");
    return PF_ERR_INVALID_ARG;
  }
  for (int k = 0; k < 3 && enable; ++k)
    if (((enable >> k) & 1) && ctx->ktime_ev[k].empty()) {
      ctx->ktime_ev[k].resize(2 * kKernelTimerMax, nullptr);
      for (auto& e : ctx->ktime_ev[k]) PFF_HIP(hipEventCreate(&e));
    }
  ctx->ktime_mask = enable;
  if (enable) {
    ctx->ktime_every = every;
    for (int k = 0; k < 3; ++k) ctx->ktime_n[k] = 0, ctx->ktime_seen[k] = 0;
  }
  return PF_OK;
}

pf_status pf_get_kernel_timing_op(pf_ctx* ctx, int op, int64_t* launches, int* count, double* avg_s, double* min_s,
                                  double* max_s) {
  NEED_CTX();
  if (!launches || !count || !avg_s || !min_s || !max_s) {
    set_error("launches, count, avg_s, min_s and max_s must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (op != PF_KTIME_JACOBIAN && op != PF_KTIME_BLOCK && op != PF_KTIME_BLOCK_CHEB) {
    set_error("op must be PF_KTIME_JACOBIAN, PF_KTIME_BLOCK or PF_KTIME_BLOCK_CHEB");
    return PF_ERR_INVALID_ARG;
  }
  const int k = op == PF_KTIME_JACOBIAN ? 0 : (op == PF_KTIME_BLOCK ? 1 : 2);
  double sum = 0.0, lo = 0.0, hi = 0.0;
  for (int i = 0; i < ctx->ktime_n[k]; ++i) {
    PFF_HIP(hipEventSynchronize(ctx->ktime_ev[k][2 * i + 1]));
    float ms = 0.f;
    PFF_HIP(hipEventElapsedTime(&ms, ctx->ktime_ev[k][2 * i], ctx->ktime_ev[k][2 * i + 1]));
    const double t = 1e-3 * ms;
    sum += t;
    lo = i ? std::min(lo, t) : t;
    hi = i ? std::max(hi, t) : t;
  }
  *launches = ctx->ktime_seen[k];
  *count = ctx->ktime_n[k];
  *avg_s = ctx->ktime_n[k] ? sum / ctx->ktime_n[k] : 0.0;
  *min_s = lo;
  *max_s = hi;
  return PF_OK;
}

pf_status pf_set_smoother_fusion(pf_ctx* ctx, int mode) {
  NEED_CTX();
  if (mode != PF_FUSE_OFF && mode != PF_FUSE_TUNED && mode != PF_FUSE_ALWAYS) {
    set_error("mode must be PF_FUSE_OFF, PF_FUSE_TUNED or PF_FUSE_ALWAYS");
    return PF_ERR_INVALID_ARG;
  }
  ctx->cheb_fusion = mode;
  ctx->drop_graphs();
  return PF_OK;
}

pf_status pf_set_level_fusion(pf_ctx* ctx, int level, int prec, int fused) {
  NEED_CTX();
  NEED_LEVEL(level);
  if ((prec != PF_F64 && prec != PF_F32) || (fused != 0 && fused != 1)) {
    set_error("prec must be PF_F64 or PF_F32 and fused 0 or 1");
    return PF_ERR_INVALID_ARG;
  }
  ctx->lev[level].fuse[prec == PF_F64 ? 0 : 1] = fused != 0;
  ctx->drop_graphs();
  return PF_OK;
}

pf_status pf_get_kernel_timing(pf_ctx* ctx, int* count, double* avg_s, double* min_s, double* max_s) {
  int64_t launches = 0;
  return pf_get_kernel_timing_op(ctx, PF_KTIME_JACOBIAN, &launches, count, avg_s, min_s, max_s);
}

pf_status pf_block_apply(pf_ctx* ctx, int level, int prec, const void* d_x, void* d_y, void* stream) {
  return apply_entry(ctx, level, prec, MODE_BLOCK, d_x, d_y, stream);
}

pf_status pf_residual(pf_ctx* ctx, const double* d_U, const double* d_phi_tilde, double* d_R, void* stream) {
  NEED_CTX();
  if (!d_U || !d_phi_tilde || !d_R) {
    set_error("U, phi_tilde and R must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  LevelBuf& f = ctx->lev.back();
  return apply_op<double>(f.g, cparams(ctx, (int)ctx->lev.size() - 1), MODE_RESID, nullptr, d_U, d_phi_tilde,
                          f.mask, d_R, st(stream));
}

pf_status pf_get_diagonal(pf_ctx* ctx, int level, double* d_diag, void* stream) {
  NEED_CTX();
  NEED_LIN();
  NEED_LEVEL(level);
  if (!d_diag) {
    set_error("diag is NULL");
    return PF_ERR_INVALID_ARG;
  }
  LevelBuf& b = ctx->lev[level];
  return vec_copy<double>(d_diag, b.diag, b.g.n_dofs, st(stream));
}

pf_status pf_get_lumped_mass(pf_ctx* ctx, double* d_M, void* stream) {
  NEED_CTX();
  if (!d_M) {
    set_error("M is NULL");
    return PF_ERR_INVALID_ARG;
  }
  return vec_copy<double>(d_M, ctx->M, ctx->lev.back().g.n_nodes, st(stream));
}

pf_status pf_get_level_data(pf_ctx* ctx, int level, double* d_U, double* d_phi_tilde, uint8_t* d_mask,
                            void* stream) {
  NEED_CTX();
  NEED_LEVEL(level);
  LevelBuf& b = ctx->lev[level];
  hipStream_t s = st(stream);
  if ((d_U || d_phi_tilde) && !ctx->has_lin) {
    set_error("no linearization point: call pf_set_linearization");
    return PF_ERR_INVALID_ARG;
  }
  if (d_U) PFF_TRY(vec_copy<double>(d_U, b.U, b.g.n_dofs, s));
  if (d_phi_tilde) PFF_TRY(vec_copy<double>(d_phi_tilde, b.phit, b.g.n_nodes, s));
  if (d_mask) PFF_TRY(vec_copy<uint8_t>(d_mask, b.mask, b.g.n_nodes, s));
  return PF_OK;
}

pf_status pf_active_set(pf_ctx* ctx, const double* d_R, const double* d_U, const double* d_U_old, uint8_t* d_active,
                        double* d_v, int64_t* n_active, void* stream) {
  NEED_CTX();
  if (!d_R || !d_U || !d_U_old || !d_active) {
    set_error("R, U, U_old and active must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  LevelBuf& f = ctx->lev.back();
  hipStream_t s = st(stream);
  PFF_TRY(pdas_decide(f.g, d_R, d_U, d_U_old, ctx->M, f.base, ctx->opt.pdas_c, d_active, d_v, s));
  if (n_active) PFF_TRY(count_bytes(d_active, f.g.n_nodes, ctx->part, n_active, s));
  return PF_OK;
}

pf_status pf_transfer(pf_ctx* ctx, int level, int op, const double* d_in, double* d_out, void* stream) {
  NEED_CTX();
  if (level < 1 || level >= (int)ctx->lev.size()) {
    set_error("transfer level must be in [1, n_levels-1]");
    return PF_ERR_INVALID_ARG;
  }
  if (!d_in || !d_out || d_in == d_out) {
    set_error("in/out must be non-NULL and distinct");
    return PF_ERR_INVALID_ARG;
  }
  const Geom& gf = ctx->lev[level].g;
  const Geom& gc = ctx->lev[level - 1].g;
  hipStream_t s = st(stream);
  if (op == 0) return restrict_vec<double, double>(gc, gf, d_in, nullptr, d_out, nullptr, s);
  if (op == 1) return prolong_vec<double, double>(gc, gf, d_in, d_out, nullptr, 0, s);
  if (op == 2) return inject<double>(gc, gf, d_in, d_out, gf.d + 1, s);
  set_error("op must be 0 (restrict), 1 (prolong) or 2 (inject)");
  return PF_ERR_INVALID_ARG;
}

pf_status pf_get_eig_bounds(pf_ctx* ctx, int level, double out[4]) {
  NEED_CTX();
  NEED_LEVEL(level);
  if (!out) {
    set_error("out is NULL");
    return PF_ERR_INVALID_ARG;
  }
  for (int k = 0; k < 4; ++k) out[k] = ctx->lev[level].eig[k];
  return PF_OK;
}

pf_status pf_set_eig_bounds(pf_ctx* ctx, int level, const double in[4]) {
  NEED_CTX();
  NEED_LEVEL(level);
  LevelBuf& b = ctx->lev[level];
  if (!in) {
    b.eig_fixed = false;
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
  for (int k = 0; k < 4; ++k) b.eig[k] = in[k];
  b.eig_fixed = true;
  // written on the stream of the next V-cycle, which also rebuilds the dense coarse matrix for
  // new level-0 bounds
  ctx->coef_stale = true;
  if (level == 0 && ctx->coarse_dense_ok) ctx->dense_stale = true;
  return PF_OK;
}

pf_status pf_vcycle(pf_ctx* ctx, int prec, const double* d_r, double* d_z, void* stream) {
  NEED_CTX();
  NEED_LIN();
  if (prec != PF_F64 && prec != PF_F32) {
    set_error("prec must be PF_F64 or PF_F32");
    return PF_ERR_INVALID_ARG;
  }
  if (!d_r || !d_z || d_r == d_z) {
    set_error("r and z must be non-NULL and distinct");
    return PF_ERR_INVALID_ARG;
  }
  return vcycle_any(ctx, prec, d_r, d_z, st(stream));
}

// Steps 1, 3 and 4 of Algorithm 1 at U_k: R = -A(U_k), the active set, the lift and
// R~ = Pi_F (R - G d) + d on the finest level (no level data yet).
pf_status newton_prepare(pf_ctx* ctx, const double* d_U, const double* d_U_old, const double* d_phi_tilde,
                         int64_t* n_active, double* rt_norm, hipStream_t s, double* t_resid = nullptr) {
  const int L = (int)ctx->lev.size() - 1;
  LevelBuf& f = ctx->lev[L];
  const Geom& g = f.g;
  const double t0 = now_s();
  PFF_TRY(apply_op<double>(g, cparams(ctx, L), MODE_RESID, nullptr, d_U, d_phi_tilde, f.mask, ctx->R, s));
  double bad = 0;
  PFF_TRY(count_nonfinite(ctx->R, g.n_dofs, ctx->part, &bad, s));  // synchronizes
  if (t_resid) *t_resid = now_s() - t0;
  if (bad > 0) {
    set_error("non-finite residual (check U, U_old, phi_tilde)");
    return PF_ERR_NONFINITE;
  }
  PFF_TRY(pdas_decide(g, ctx->R, d_U, d_U_old, ctx->M, f.base, ctx->opt.pdas_c, ctx->active, nullptr, s));
  PFF_TRY(count_bytes(ctx->active, g.n_nodes, ctx->part, n_active, s));
  PFF_TRY(build_lift(g, d_U, d_U_old, ctx->active, ctx->dl, s));
  PFF_TRY(combine_mask(f.base, ctx->has_extra ? ctx->extra : nullptr, ctx->active, f.mask, g.n_nodes, s));
  const double* tlift = nullptr;
  if (*n_active > 0) {
    // t = G d_lift with no constraint applied: on Q1 cells without the energy split the Jacobian's
    // own (tuned) kernel with the all-free mask, else the unmasked mode of the cell loop
    const CellParams cpa = level_params(ctx, L, PF_F64, MODE_APPLY);
    if (g.p == 1 && !cpa.split)
      PFF_TRY(apply_op<double>(g, cpa, MODE_APPLY, ctx->dl, d_U, d_phi_tilde, ctx->free_mask, ctx->t, s));
    else
      PFF_TRY(apply_op<double>(g, cparams(ctx, L), MODE_RAW, ctx->dl, d_U, d_phi_tilde, f.mask, ctx->t, s));
    tlift = ctx->t;
  }
  PFF_TRY(constrain_rhs(g, ctx->R, tlift, ctx->dl, f.mask, ctx->Rt, s));
  double r2 = 0;
  PFF_TRY(dot_host(ctx->Rt, ctx->Rt, g.n_dofs, ctx->part, &r2, s));
  *rt_norm = std::sqrt(r2);
  return PF_OK;
}

// Steps 2, 5 and 6 after newton_prepare: level data, FGMRES from the lift, U += dU.
pf_status newton_solve(pf_ctx* ctx, double* d_U, const double* d_phi_tilde, int* iters, double* rel, double* bn,
                       hipStream_t s) {
  const Geom& g = ctx->lev.back().g;
  PFF_TRY(set_linearization(ctx, d_U, d_phi_tilde, ctx->active, s));
  PFF_TRY(vec_copy<double>(ctx->dU, ctx->dl, g.n_dofs, s));
  PFF_TRY(fgmres(ctx, ctx->Rt, ctx->dU, ctx->vprec, iters, rel, bn, s));
  PFF_TRY(vec_axpby<double>(d_U, 1.0, ctx->dU, 1.0, g.n_dofs, s));
  PFF_HIP(hipStreamSynchronize(s));
  return PF_OK;
}

bool fgmres_converged(const pf_ctx* ctx, double rel, double bn) {
  return rel * bn <= std::max(ctx->opt.gmres_rtol * bn, ctx->opt.gmres_atol);
}

pf_status pf_newton_step(pf_ctx* ctx, double* d_U, const double* d_U_old, const double* d_phi_tilde,
                         pf_newton_report* rep, void* stream) {
  NEED_CTX();
  if (!d_U || !d_U_old || !d_phi_tilde) {
    set_error("U, U_old and phi_tilde must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = st(stream);
  pf_newton_report r;
  std::memset(&r, 0, sizeof(r));
  const double t0 = now_s();
  double rt = 0, t_res = 0;
  const pf_status sp = newton_prepare(ctx, d_U, d_U_old, d_phi_tilde, &r.n_active, &rt, s, &t_res);
  if (sp != PF_OK) {
    if (rep) *rep = r;
    return sp;
  }
  PFF_HIP(hipStreamSynchronize(s));
  const double t2 = now_s();
  int iters = 0;
  double rel = 0, bn = 0;
  PFF_TRY(newton_solve(ctx, d_U, d_phi_tilde, &iters, &rel, &bn, s));
  const double t3 = now_s();
  r.gmres_iters = iters;
  r.rel_residual = rel;
  r.rhs_norm = bn;
  r.converged = fgmres_converged(ctx, rel, bn) ? 1 : 0;
  r.t_residual_s = t_res;
  r.t_setup_s = t2 - t0 - t_res;
  r.t_solve_s = t3 - t2;
  r.t_total_s = t3 - t0;
  if (rep) *rep = r;
  if (!r.converged) {
    set_error("FGMRES reached gmres_max_iter before the tolerance");
    return PF_ERR_NOT_CONVERGED;
  }
  return PF_OK;
}

pf_status pf_pdas_solve(pf_ctx* ctx, double* d_U, const double* d_U_old, const double* d_phi_tilde, int max_iter,
                        double tol_as, pf_pdas_report* rep, void* stream) {
  NEED_CTX();
  if (!d_U || !d_U_old || !d_phi_tilde) {
    set_error("U, U_old and phi_tilde must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (max_iter < 1 || !(tol_as >= 0.0) || !std::isfinite(tol_as)) {
    set_error("max_iter must be >= 1 and tol_as finite and >= 0");
    return PF_ERR_INVALID_ARG;
  }
  hipStream_t s = st(stream);
  const Geom& g = ctx->lev.back().g;
  pf_pdas_report r;
  std::memset(&r, 0, sizeof(r));
  r.n_changed = -1;
  const double t0 = now_s();
  pf_status status = PF_ERR_NOT_CONVERGED;
  bool gmres_failed = false;
  for (int k = 0; k <= max_iter; ++k) {
    double rt = 0;
    const pf_status sp = newton_prepare(ctx, d_U, d_U_old, d_phi_tilde, &r.n_active, &rt, s);
    if (sp != PF_OK) {
      status = sp;
      break;
    }
    r.residual_norm = rt;
    r.n_changed = -1;
    if (k > 0) PFF_TRY(count_diff_bytes(ctx->active, ctx->prev_active, g.n_nodes, ctx->part, &r.n_changed, s));
    if (k > 0 && r.n_changed == 0 && rt <= tol_as) {
      r.converged = 1;
      status = PF_OK;
      break;
    }
    if (k == max_iter) break;
    int iters = 0;
    double rel = 0, bn = 0;
    PFF_TRY(newton_solve(ctx, d_U, d_phi_tilde, &iters, &rel, &bn, s));
    r.iterations = k + 1;
    r.gmres_iters_total += iters;
    if (!fgmres_converged(ctx, rel, bn)) {
      set_error("FGMRES reached gmres_max_iter before the tolerance in a PDAS correction");
      gmres_failed = true;
      break;
    }
    PFF_TRY(vec_copy<uint8_t>(ctx->prev_active, ctx->active, g.n_nodes, s));
  }
  PFF_HIP(hipStreamSynchronize(s));
  r.t_total_s = now_s() - t0;
  if (rep) *rep = r;
  if (status == PF_ERR_NOT_CONVERGED && !gmres_failed)
    set_error("the active set did not settle within max_iter corrections");
  return status;
}

pf_status pf_extrapolate(pf_ctx* ctx, const double* d_phi_1, const double* d_phi_2, double theta, double* d_out,
                         void* stream) {
  NEED_CTX();
  if (!d_phi_1 || !d_phi_2 || !d_out) {
    set_error("phi_1, phi_2 and out must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (!std::isfinite(theta)) {
    set_error("theta must be finite");
    return PF_ERR_INVALID_ARG;
  }
  if (d_out == d_phi_1 || d_out == d_phi_2) {
    set_error("out may not alias phi_1 or phi_2");
    return PF_ERR_INVALID_ARG;
  }
  const LevelBuf& f = ctx->lev.back();
  return extrapolate_phase(d_phi_1, d_phi_2, theta, f.base, f.g.n_nodes, d_out, st(stream));
}

pf_status pf_energies(pf_ctx* ctx, const double* d_U, double out[2], void* stream) {
  NEED_CTX();
  if (!d_U || !out) {
    set_error("U and out must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  const int L = (int)ctx->lev.size() - 1;
  return quantity_energies(ctx->lev[L].g, cparams(ctx, L), ctx->mat.Gc, ctx->mat.eps, d_U, ctx->qpart, out,
                           st(stream));
}

pf_status pf_energies_noalloc(pf_ctx* ctx, const double* d_U, double* d_out, void* stream) {
  NEED_CTX();
  if (!d_U || !d_out) {
    set_error("U and out must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  int device = -1;
  PFF_HIP(hipGetDevice(&device));
  if (device != ctx->device) {
    set_error("the current device is not the context's");
    return PF_ERR_INVALID_ARG;
  }
  const int L = (int)ctx->lev.size() - 1;
  return quantity_energies_noalloc(ctx->lev[L].g, cparams(ctx, L), ctx->mat.Gc, ctx->mat.eps, d_U, device, d_out,
                                   st(stream));
}

pf_status pf_boundary_traction(pf_ctx* ctx, const double* d_U, int face, double* out, void* stream) {
  NEED_CTX();
  const int L = (int)ctx->lev.size() - 1;
  const Geom& g = ctx->lev[L].g;
  if (!d_U || !out) {
    set_error("U and out must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  if (face < 0 || face >= 2 * g.d) {
    set_error("face must be in [0, 2 dim)");
    return PF_ERR_INVALID_ARG;
  }
  return quantity_face_traction(g, cparams(ctx, L), face, d_U, ctx->qpart, out, st(stream));
}

pf_status pf_set_pressure(pf_ctx* ctx, double pressure) {
  NEED_CTX();
  if (!std::isfinite(pressure)) {
    set_error("pressure must be finite");
    return PF_ERR_INVALID_ARG;
  }
  ctx->mat.p = pressure;
  ctx->coarse_dense_ok = false;  // the operator changed: the fused kernel serves until the next set-up
  ctx->drop_graphs();
  return PF_OK;
}

pf_status pf_get_level_info(pf_ctx* ctx, int level, pf_level_info* info) {
  NEED_CTX();
  NEED_LEVEL(level);
  if (!info) {
    set_error("info is NULL");
    return PF_ERR_INVALID_ARG;
  }
  const LevelBuf& b = ctx->lev[level];
  for (int k = 0; k < 3; ++k) {
    info->n_cells[k] = b.g.N[k];
    info->n_nodes_axis[k] = b.g.nn[k];
    info->h[k] = b.g.h[k];
  }
  info->n_nodes = b.g.n_nodes;
  info->n_dofs = b.g.n_dofs;
  info->n_active_cells = b.n_active_cells;
  info->precision = level_prec(ctx, level, ctx->vprec);
  info->n_domain_nodes = b.n_domain_nodes;
  return PF_OK;
}

// ---------------------------------------------------------------------------------- autotuner
// Candidates of the Q1 cell loop: (variant, chunk).  Variants 1 (16x4 tiles), 3 (LDS bricks) and 5
// (LDS-staged slabs) are 3D only.
// Small chunks suit levels that barely fill the chip, long ones (fewer recomputed halo
// layers) the large levels.
static const int kCand[][2] = {{2, -1}, {4, -1}, {3, -1}, {0, 4}, {0, 8}, {0, 16}, {0, 32}, {0, 64},
                               {1, 4}, {1, 8}, {1, 16}, {1, 32}, {0, 2}, {0, 3}, {1, 2},
                               {5, 16}, {5, 32}, {5, 64}};
static const int kNCand = 18;
static_assert(kNCand <= kTuneSlots, "tune_us holds kTuneSlots candidates");
static const double kTuneTie = 0.03;

extern "C++" {
// One Chebyshev smoother step of level l in precision prec, fused into the marching-tile B~ apply or
// as the apply followed by the vector pass, timed over reps launches (us per step).  Works on the
// level's V-cycle scratch vectors with bounded coefficients.
template <typename T>
static pf_status time_cheb_step(pf_ctx* c, int l, int prec, bool fused, int reps, hipEvent_t e0, hipEvent_t e1,
                                hipStream_t s, double* us) {
  LevelBuf& b = c->lev[l];
  const int64_t nd = b.g.n_dofs;
  T* d = (T*)b.vd;
  T* t = (T*)b.vt;
  T* res = (T*)b.vr;
  T* x = (T*)b.vx;
  T* dout = (T*)b.vb;
  const T* diag = prec == PF_F64 ? (const T*)b.diag : (const T*)b.diag32;
  const T* Ul = prec == PF_F64 ? (const T*)b.U : (const T*)b.U32;
  const T* pl = prec == PF_F64 ? (const T*)b.phit : (const T*)b.phit32;
  const CellParams bcp = level_params(c, l, prec, MODE_BLOCK);
  const double hc[4] = {0.5, 1e-3, 0.5, 1e-3};
  double* dc = tune_coefs(c);
  PFF_TRY(vec_put(dc, hc, 4, s));
  for (T* v : {d, res, x, dout}) PFF_TRY(vec_fill<T>(v, T(1), nd, s));
  auto step = [&]() -> pf_status {
    if (fused) {
      ChebFuse<T> cf;
      cf.res = res;
      cf.diag = diag;
      cf.x = x;
      cf.d_out = dout;
      cf.t_next = nullptr;
      cf.dc = dc;
      cf.next_of_x = 0;
      bool handled = false;
      PFF_TRY(launch_q1_block_cheb<T>(b.g, bcp, d, Ul, pl, b.mask, cf, s, &handled));
      if (!handled) {
        set_error("fused Chebyshev step: not a marching-tile level");
        return PF_ERR_UNSUPPORTED;
      }
      return PF_OK;
    }
    PFF_TRY(level_apply(c, l, prec, MODE_BLOCK, d, t, s));
    return vec_cheb_step<T>(res, t, d, x, diag, dc, 0, b.g.n_nodes, b.g.d, b.mask, nullptr, 0, nullptr, s);
  };
  for (int w = 0; w < 2; ++w) PFF_TRY(step());
  PFF_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) PFF_TRY(step());
  PFF_HIP(hipEventRecord(e1, s));
  PFF_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  PFF_HIP(hipEventElapsedTime(&ms, e0, e1));
  *us = 1e3 * ms / reps;
  return PF_OK;
}
}  // extern "C++"

static pf_status autotune_level(pf_ctx* c, int l, int reps, hipStream_t s) {
  LevelBuf& b = c->lev[l];
  if (b.g.p != 1) return PF_OK;
  // the split has two shapes of its own (one work item per cell, or two wavefronts per cell)
  const bool split = c->mat.split != PF_SPLIT_NONE;
  hipEvent_t e0, e1;
  PFF_HIP(hipEventCreate(&e0));
  PFF_HIP(hipEventCreate(&e1));
  pf_status st = PF_OK;
  for (int pi = 0; pi < 2 && st == PF_OK; ++pi) {
    const int prec = pi == 0 ? PF_F64 : PF_F32;
    if (prec == PF_F64)
      st = vec_fill<double>((double*)b.vb, 1.0, b.g.n_dofs, s);
    else
      st = vec_fill<float>((float*)b.vb, 1.0f, b.g.n_dofs, s);
    for (int mi = 0; mi < 2 && st == PF_OK; ++mi) {
      const int mode = mi == 0 ? MODE_APPLY : MODE_BLOCK;
      double best = 1e300;
      int bv = -1, bz = -1;
      for (int k = 0; k < kNCand && st == PF_OK; ++k) {
        if (((kCand[k][0] == 1 || kCand[k][0] == 3 || kCand[k][0] == 5) && b.g.d != 3) ||
            (split && !(kCand[k][0] == 2 || kCand[k][0] == 4))) {
          b.tune_us[pi][mi][k] = -1.0;
          continue;
        }
        b.variant[pi][mi] = kCand[k][0];
        b.zc[pi][mi] = kCand[k][1];
        for (int w = 0; w < 2 && st == PF_OK; ++w) st = level_apply(c, l, prec, mode, b.vb, b.vt, s);
        if (st != PF_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) st = PF_ERR_DEVICE;
        for (int r = 0; r < reps && st == PF_OK; ++r) st = level_apply(c, l, prec, mode, b.vb, b.vt, s);
        if (st != PF_OK) break;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          set_error("autotune timing failed");
          st = PF_ERR_DEVICE;
          break;
        }
        const double us = 1e3 * ms / reps;
        b.tune_us[pi][mi][k] = us;
        best = std::min(best, us);
      }
      // the earliest candidate within kTuneTie of the fastest: timing noise between near-equal
      // shapes does not flip the choice from run to run
      for (int k = 0; k < kNCand && st == PF_OK; ++k) {
        const double us = b.tune_us[pi][mi][k];
        if (us > 0.0 && us <= best * (1.0 + kTuneTie)) {
          bv = kCand[k][0];
          bz = kCand[k][1];
          break;
        }
      }
      b.variant[pi][mi] = bv;
      b.zc[pi][mi] = bz;
      if (mi == 1 && st == PF_OK) {
        // with B~ on marching tiles, time one smoother step fused and unfused; fuse only when
        // that is clearly faster (the fused vector update is not a coalesced stream)
        b.fuse[pi] = false;
        b.fuse_us[pi][0] = b.fuse_us[pi][1] = 0.0;
        if (q1_block_cheb_fusable(b.g, level_params(c, l, prec, MODE_BLOCK))) {
          for (int f = 0; f < 2 && st == PF_OK; ++f)
            st = prec == PF_F64 ? time_cheb_step<double>(c, l, prec, f == 1, reps, e0, e1, s, &b.fuse_us[pi][f])
                                : time_cheb_step<float>(c, l, prec, f == 1, reps, e0, e1, s, &b.fuse_us[pi][f]);
          if (st == PF_OK) b.fuse[pi] = b.fuse_us[pi][1] < b.fuse_us[pi][0] * (1.0 - kTuneTie);
        }
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return st;
}

pf_status pf_autotune(pf_ctx* ctx, int reps, void* stream) {
  NEED_CTX();
  NEED_LIN();
  if (reps < 1 || reps > 10000) {
    set_error("reps must be in [1, 10000]");
    return PF_ERR_INVALID_ARG;
  }
  ctx->drop_graphs();
  for (int l = 0; l < (int)ctx->lev.size(); ++l) PFF_TRY(autotune_level(ctx, l, reps, st(stream)));
  return PF_OK;
}

static pf_status tuning_index(pf_ctx* ctx, int level, int prec, int mode, int* pi, int* mi) {
  NEED_LEVEL(level);
  if ((prec != PF_F64 && prec != PF_F32) || (mode != 0 && mode != 1)) {
    set_error("prec must be PF_F64/PF_F32 and mode 0 (Jacobian) or 1 (block)");
    return PF_ERR_INVALID_ARG;
  }
  *pi = prec == PF_F64 ? 0 : 1;
  *mi = mode;
  return PF_OK;
}

pf_status pf_get_tuning(pf_ctx* ctx, int level, int prec, int mode, int* variant, int* zc) {
  NEED_CTX();
  int pi, mi;
  PFF_TRY(tuning_index(ctx, level, prec, mode, &pi, &mi));
  if (!variant || !zc) {
    set_error("variant and zc must be non-NULL");
    return PF_ERR_INVALID_ARG;
  }
  *variant = ctx->lev[level].variant[pi][mi];
  *zc = ctx->lev[level].zc[pi][mi];
  return PF_OK;
}

pf_status pf_set_tuning(pf_ctx* ctx, int level, int prec, int mode, int variant, int zc) {
  NEED_CTX();
  int pi, mi;
  PFF_TRY(tuning_index(ctx, level, prec, mode, &pi, &mi));
  if (variant < -1 || variant >= kQ1Variants || zc > 4096) {
    set_error("variant must be in [-1, 5] and zc <= 4096");
    return PF_ERR_INVALID_ARG;
  }
  ctx->lev[level].variant[pi][mi] = variant;
  ctx->lev[level].zc[pi][mi] = zc;
  ctx->drop_graphs();
  return PF_OK;
}

pf_status pf_tuning_report(pf_ctx* ctx, char* buf, size_t len) {
  NEED_CTX();
  if (!buf || len == 0) {
    set_error("buf must be non-NULL with len > 0");
    return PF_ERR_INVALID_ARG;
  }
  std::string o = "{\"levels\": [";
  for (size_t l = 0; l < ctx->lev.size(); ++l) {
    const LevelBuf& b = ctx->lev[l];
    if (l) o += ", ";
    o += "{\"level\": " + std::to_string(l) + ", \"cells\": " + std::to_string(b.g.n_cells) + ", \"choices\": [";
    for (int pi = 0; pi < 2; ++pi)
      for (int mi = 0; mi < 2; ++mi) {
        if (pi || mi) o += ", ";
        o += "{\"prec\": \"" + std::string(pi ? "f32" : "f64") + "\", \"mode\": \"" + (mi ? "block" : "jacobian") +
             "\", \"variant\": " + std::to_string(b.variant[pi][mi]) + ", \"zc\": " + std::to_string(b.zc[pi][mi]);
        if (mi) {
          char tmp[96];
          snprintf(tmp, sizeof(tmp), ", \"fused\": %d, \"step_us\": [%.3f, %.3f]", b.fuse[pi] ? 1 : 0,
                   b.fuse_us[pi][0], b.fuse_us[pi][1]);
          o += tmp;
        }
        o += ", \"us\": [";
        for (int k = 0; k < kNCand; ++k) {
          if (k) o += ", ";
          char tmp[64];
          snprintf(tmp, sizeof(tmp), "[%d, %d, %.3f]", kCand[k][0], kCand[k][1], b.tune_us[pi][mi][k]);
          o += tmp;
        }
        o += "]}";
      }
    o += "]}";
  }
  o += "]}";
  if (o.size() + 1 > len) {
    set_error("report buffer too small: need " + std::to_string(o.size() + 1));
    return PF_ERR_INVALID_ARG;
  }
  std::memcpy(buf, o.c_str(), o.size() + 1);
  return PF_OK;
}

pf_status pf_set_coarse_mode(pf_ctx* ctx, int mode) {
  NEED_CTX();
  if (mode != PF_COARSE_AUTO && mode != PF_COARSE_FUSED && mode != PF_COARSE_STEPS) {
    set_error("mode must be PF_COARSE_AUTO, PF_COARSE_FUSED or PF_COARSE_STEPS");
    return PF_ERR_INVALID_ARG;
  }
  if (mode != ctx->coarse_mode) ctx->coarse_dense_ok = false;  // AUTO builds its matrix at the next set-up
  ctx->coarse_mode = mode;
  ctx->drop_graphs();
  return PF_OK;
}

pf_status pf_set_graphs(pf_ctx* ctx, int enable) {
  NEED_CTX();
  ctx->use_graphs = enable != 0;
  if (!ctx->use_graphs) ctx->drop_graphs();
  return PF_OK;
}

pf_status pf_get_graph_captures(pf_ctx* ctx, int64_t* n) {
  NEED_CTX();
  if (!n) {
    set_error("n must not be null");
    return PF_ERR_INVALID_ARG;
  }
  *n = ctx->n_captures;
  return PF_OK;
}

pf_status pf_set_vcycle_precision(pf_ctx* ctx, int prec) {
  NEED_CTX();
  if (prec != PF_F64 && prec != PF_F32) {
    set_error("prec must be PF_F64 or PF_F32");
    return PF_ERR_INVALID_ARG;
  }
  ctx->vprec = prec;
  return PF_OK;
}

}  // extern "C"
