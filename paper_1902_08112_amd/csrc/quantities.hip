// Quantities of interest of Sec. 5 as fused reductions over the cells of the
// finest level, state U = (u, phi):
//   crack energy  E_c = int G_c/2 ((1 - phi)^2 / eps + eps |grad phi|^2)
//   bulk energy   E_b = int g_kappa(phi) E_s^+(e(u)) + E_s^-(e(u)) + phi^2 p div u
//   face load     L = int_face (g_kappa(phi) sigma^+(u) + sigma^-(u)) n ds on one box face
// (without a split E_s^+ = E_s, sigma^+ = sigma; with the Miehe split the parts of split.h)
// evaluated at the cell's (p+1)^d Gauss points (the facet's (p+1)^(d-1)).
// One thread per cell; per-block partial sums in a fixed grid, then one final
// block, so the sums are deterministic.
#include <mutex>

#include "generic_cell.h"

namespace pff {

namespace {

constexpr int kQBlock = 256;
constexpr int kQMaxBlocks = 1024;

__device__ inline double qsum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

template <int D, int P>
__device__ inline void cell_nodes(const CellParams& cp, int64_t cid, int64_t g[Tens<D, P>::NL], bool* active) {
  using TT = Tens<D, P>;
  int c[3] = {(int)(cid % cp.N[0]), (int)((cid / cp.N[0]) % cp.N[1]),
              D == 3 ? (int)(cid / ((int64_t)cp.N[0] * cp.N[1])) : 0};
  *active = !cell_in_hole(cp.lshape, c[0], c[1], cp.N[0], cp.N[1]);
#pragma unroll
  for (int a = 0; a < TT::NL; ++a) {
    int64_t v = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) v += (int64_t)(P * c[k] + TT::idx(a, k)) * cp.ns[k];
    g[a] = v;
  }
}

}  // namespace

// partials[2 * nb]: per block (E_c, E_b)
template <int D, int P>
__global__ __launch_bounds__(kQBlock) void k_energies(CellParams cp, double Gc, double eps, const double* U,
                                                      double* partials) {
  using TT = Tens<D, P>;
  constexpr int NL = TT::NL;
  __shared__ double sh[kQBlock / 64];
  const int64_t nn = cp.n_nodes;
  const double mu = cp.mu, lam = cp.lam, kap = cp.kappa, pres = cp.pres;
  const double ih[3] = {cp.inv_h[0], cp.inv_h[1], cp.inv_h[2]};
  double ec = 0.0, eb = 0.0;
  for (int64_t cid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cid < cp.n_cells;
       cid += (int64_t)gridDim.x * blockDim.x) {
    int64_t g[NL];
    bool act;
    cell_nodes<D, P>(cp, cid, g, &act);
    if (!act) continue;
#pragma unroll 1
    for (int q = 0; q < NL; ++q) {
      const double jxw = TT::w(q) * cp.vol;
      double gu[D][D], gp[D], phi = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        gp[i] = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) gu[i][j] = 0.0;
      }
#pragma unroll
      for (int a = 0; a < NL; ++a) {
        const double pa = U[D * nn + g[a]];
        phi += TT::N(q, a) * pa;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const double dn = TT::dN(q, a, j) * ih[j];
          gp[j] += dn * pa;
#pragma unroll
          for (int i = 0; i < D; ++i) gu[i][j] += dn * U[i * nn + g[a]];
        }
      }
      double tr = 0.0, ee = 0.0, g2 = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        tr += gu[i][i];
        g2 += gp[i] * gp[i];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const double e = 0.5 * (gu[i][j] + gu[j][i]);
          ee += e * e;
        }
      }
      const double Es = 0.5 * lam * tr * tr + mu * ee;
      const double gd = (1.0 - kap) * phi * phi + kap;
      ec += jxw * 0.5 * Gc * ((1.0 - phi) * (1.0 - phi) / eps + eps * g2);
      if (cp.split) {
        // g E_s^+ + E_s^- = E_s - (1 - g) E_s^+
        double ed[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) ed[i][j] = 0.5 * (gu[i][j] + gu[j][i]);
        split::QP<D> sq;
        split::eval<D>(ed, mu, lam, sq);
        eb += jxw * (Es - (1.0 - gd) * sq.Es_pos + phi * phi * pres * tr);
      } else {
        eb += jxw * (gd * Es + phi * phi * pres * tr);
      }
    }
  }
  const double bc = qsum(ec, sh);
  const double bb = qsum(eb, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = bc;
    partials[gridDim.x + blockIdx.x] = bb;
  }
}

// partials[D * nb]: per block the traction components over the face cells
template <int D, int P>
__global__ __launch_bounds__(kQBlock) void k_face_traction(CellParams cp, int face, const double* U,
                                                           double* partials) {
  using TT = Tens<D, P>;
  constexpr int NL = TT::NL, n1 = P + 1;
  constexpr int NQ = D == 2 ? n1 : n1 * n1;
  __shared__ double sh[kQBlock / 64];
  const int k = face / 2, side = face % 2;
  const double nsign = side ? 1.0 : -1.0;
  // the face's cells form an (N_a x N_b) slab over the two (one) tangential axes
  const int ta = k == 0 ? 1 : 0, tb = k == 2 ? 1 : 2;
  const int64_t ncell_face = (int64_t)cp.N[ta] * (D == 3 ? cp.N[tb] : 1);
  const int64_t nn = cp.n_nodes;
  const double mu = cp.mu, lam = cp.lam, kap = cp.kappa;
  const double ih[3] = {cp.inv_h[0], cp.inv_h[1], cp.inv_h[2]};
  double hta = 1.0 / ih[ta], htb = D == 3 ? 1.0 / ih[tb] : 1.0;
  double acc[D];
#pragma unroll
  for (int i = 0; i < D; ++i) acc[i] = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell_face;
       t += (int64_t)gridDim.x * blockDim.x) {
    int c[3] = {0, 0, 0};
    c[ta] = (int)(t % cp.N[ta]);
    if (D == 3) c[tb] = (int)(t / cp.N[ta]);
    c[k] = side ? cp.N[k] - 1 : 0;
    if (cell_in_hole(cp.lshape, c[0], c[1], cp.N[0], cp.N[1])) continue;
    int64_t g[NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) {
      int64_t v = 0;
#pragma unroll
      for (int kk = 0; kk < D; ++kk) v += (int64_t)(P * c[kk] + TT::idx(a, kk)) * cp.ns[kk];
      g[a] = v;
    }
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      // reference point: t_k = side, tangential Gauss points
      double tp[3] = {0.0, 0.0, 0.0};
      double w = 1.0;
      const int qa = q % n1, qb = q / n1;
      tp[k] = (double)side;
      tp[ta] = B1<P>::pt(qa);
      w *= B1<P>::wt(qa) * hta;
      if (D == 3) {
        tp[tb] = B1<P>::pt(qb);
        w *= B1<P>::wt(qb) * htb;
      }
      double gu[D][D], phi = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) gu[i][j] = 0.0;
#pragma unroll
      for (int a = 0; a < NL; ++a) {
        double val = 1.0, dv[D];
#pragma unroll
        for (int j = 0; j < D; ++j) dv[j] = 1.0;
#pragma unroll
        for (int kk = 0; kk < D; ++kk) {
          const int ak = TT::idx(a, kk);
          const double l = B1<P>::val(ak, tp[kk]), dl = B1<P>::der(ak, tp[kk]) * ih[kk];
          val *= l;
#pragma unroll
          for (int j = 0; j < D; ++j) dv[j] *= (j == kk) ? dl : l;
        }
        phi += val * U[D * nn + g[a]];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          const double ui = U[i * nn + g[a]];
#pragma unroll
          for (int j = 0; j < D; ++j) gu[i][j] += dv[j] * ui;
        }
      }
      double tr = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) tr += gu[i][i];
      const double gd = (1.0 - kap) * phi * phi + kap;
      // (sigma n)_i = sigma_ik * nsign; with the split sigma - (1 - g) sigma^+
      if (cp.split) {
        double ed[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
          for (int j = 0; j < D; ++j) ed[i][j] = 0.5 * (gu[i][j] + gu[j][i]);
        split::QP<D> sq;
        split::eval<D>(ed, mu, lam, sq);
#pragma unroll
        for (int i = 0; i < D; ++i) {
          const double sik = mu * (gu[i][k] + gu[k][i]) + (i == k ? lam * tr : 0.0);
          acc[i] += w * (sik - (1.0 - gd) * sq.sig[i][k]) * nsign;
        }
      } else {
#pragma unroll
        for (int i = 0; i < D; ++i) {
          const double sik = mu * (gu[i][k] + gu[k][i]) + (i == k ? lam * tr : 0.0);
          acc[i] += w * gd * sik * nsign;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double b = qsum(acc[i], sh);
    if (threadIdx.x == 0) partials[i * gridDim.x + blockIdx.x] = b;
  }
}

__global__ void k_qfinal(const double* partials, int nb, int nval, double* out) {
  __shared__ double sh[kQBlock / 64];
  for (int v = 0; v < nval; ++v) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) a += partials[v * nb + i];
    const double b = qsum(a, sh);
    if (threadIdx.x == 0) out[v] = b;
  }
}

static int qblocks(int64_t n) {
  int64_t b = (n + kQBlock - 1) / kQBlock;
  if (b > kQMaxBlocks) b = kQMaxBlocks;
  return (int)(b < 1 ? 1 : b);
}

// out (host): {E_c, E_b}; d_part: 2 * kQMaxBlocks + 8 doubles of device scratch
pf_status quantity_energies(const Geom& gm, const CellParams& cp, double Gc, double eps, const double* U,
                            double* d_part, double out[2], hipStream_t s) {
  const int nb = qblocks(gm.n_cells);
  if (gm.d == 2 && gm.p == 1)
    k_energies<2, 1><<<nb, kQBlock, 0, s>>>(cp, Gc, eps, U, d_part);
  else if (gm.d == 2)
    k_energies<2, 2><<<nb, kQBlock, 0, s>>>(cp, Gc, eps, U, d_part);
  else if (gm.p == 1)
    k_energies<3, 1><<<nb, kQBlock, 0, s>>>(cp, Gc, eps, U, d_part);
  else
    k_energies<3, 2><<<nb, kQBlock, 0, s>>>(cp, Gc, eps, U, d_part);
  PFF_CHECK_LAUNCH();
  double* d_out = d_part + 2 * kQMaxBlocks;
  k_qfinal<<<1, kQBlock, 0, s>>>(d_part, nb, 2, d_out);
  PFF_CHECK_LAUNCH();
  PFF_HIP(hipMemcpyAsync(out, d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  PFF_HIP(hipStreamSynchronize(s));
  return PF_OK;
}

// out (host): d traction components; d_part: 3 * kQMaxBlocks + 8 doubles of device scratch
pf_status quantity_face_traction(const Geom& gm, const CellParams& cp, int face, const double* U, double* d_part,
                                 double* out, hipStream_t s) {
  const int k = face / 2;
  const int ta = k == 0 ? 1 : 0, tb = k == 2 ? 1 : 2;
  const int64_t ncf = (int64_t)gm.N[ta] * (gm.d == 3 ? gm.N[tb] : 1);
  const int nb = qblocks(ncf);
  if (gm.d == 2 && gm.p == 1)
    k_face_traction<2, 1><<<nb, kQBlock, 0, s>>>(cp, face, U, d_part);
  else if (gm.d == 2)
    k_face_traction<2, 2><<<nb, kQBlock, 0, s>>>(cp, face, U, d_part);
  else if (gm.p == 1)
    k_face_traction<3, 1><<<nb, kQBlock, 0, s>>>(cp, face, U, d_part);
  else
    k_face_traction<3, 2><<<nb, kQBlock, 0, s>>>(cp, face, U, d_part);
  PFF_CHECK_LAUNCH();
  double* d_out = d_part + 3 * kQMaxBlocks;
  k_qfinal<<<1, kQBlock, 0, s>>>(d_part, nb, gm.d, d_out);
  PFF_CHECK_LAUNCH();
  PFF_HIP(hipMemcpyAsync(out, d_out, gm.d * sizeof(double), hipMemcpyDeviceToHost, s));
  PFF_HIP(hipStreamSynchronize(s));
  return PF_OK;
}


// ----------------------------------------------------------------------------------- allocation-free
// Device scratch of pf_energies_noalloc: the per-block partial sums of the energies and the two
// final values, in a file-scope array that every GPU the library runs on holds until the process
// ends.  Host code never passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): quantity_scratch_init resolves its address once per device, with that device
// current, and the kernels take that address.  Every call on one GPU shares the array, so calls
// that overlap on one GPU (two streams, two host threads) race; each call writes every partial it
// reads, so nothing has to start at zero.
constexpr int kNoAllocScratch = 2 * kQMaxBlocks + 8;  // doubles: 16,448 B
static __device__ __align__(256) double scratch[kNoAllocScratch];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

pf_status quantity_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device index beyond the scratch table");
    return PF_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return PF_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return PF_ERR_DEVICE;
  }
  g_scratch_ptr[device] = static_cast<double*>(p);
  return PF_OK;
}

// The energies of quantity_energies into d_out (device, 2 doubles), with the partial sums in the
// device's static scratch: no read-back, no synchronization, no allocation.
pf_status quantity_energies_noalloc(const Geom& gm, const CellParams& cp, double Gc, double eps, const double* U,
                                    int device, double* d_out, hipStream_t s) {
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device >= 0 && device < kMaxDevices) part = g_scratch_ptr[device];
  }
  if (!part) {
    set_error("no scratch address for this device (the context was set up on another device)");
    return PF_ERR_DEVICE;
  }
  const int nb = qblocks(gm.n_cells);
  if (2 * nb > kNoAllocScratch) {
    set_error("energies need " + std::to_string(2 * nb) + " scratch doubles, the static scratch holds " +
              std::to_string(kNoAllocScratch));
    return PF_ERR_WORKSPACE;
  }
  if (gm.d == 2 && gm.p == 1)
    k_energies<2, 1><<<nb, kQBlock, 0, s>>>(cp, Gc, eps, U, part);
  else if (gm.d == 2)
    k_energies<2, 2><<<nb, kQBlock, 0, s>>>(cp, Gc, eps, U, part);
  else if (gm.p == 1)
    k_energies<3, 1><<<nb, kQBlock, 0, s>>>(cp, Gc, eps, U, part);
  else
    k_energies<3, 2><<<nb, kQBlock, 0, s>>>(cp, Gc, eps, U, part);
  PFF_CHECK_LAUNCH();
  k_qfinal<<<1, kQBlock, 0, s>>>(part, nb, 2, d_out);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

}  // namespace pff
