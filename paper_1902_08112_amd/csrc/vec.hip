// Vector kernels: fills, casts, constraint masks, the fused Chebyshev step,
// deterministic two-stage reductions (block dots, multi-dots for the FGMRES
// Gram-Schmidt passes), multi-axpy, and the SplitMix64 start vector.
// All are HBM streams: grid-stride loops, 256-thread blocks, FP64 accumulation.
#include <type_traits>

#include "common.h"

namespace pff {

static inline int64_t nblocks(int64_t n, int bs = 256, int64_t cap = 65536) {
  int64_t b = (n + bs - 1) / bs;
  if (b > cap) b = cap;
  return b < 1 ? 1 : b;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

template <typename T>
__global__ void k_fill(T* y, T v, int64_t n) {
  GRID_STRIDE(i, n) y[i] = v;
}
template <typename T>
pf_status vec_fill(T* y, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return PF_OK;
  k_fill<T><<<nblocks(n), 256, 0, s>>>(y, v, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <typename T>
pf_status vec_copy(T* y, const T* x, int64_t n, hipStream_t s) {
  if (n <= 0) return PF_OK;
  PFF_HIP(hipMemcpyAsync(y, x, n * sizeof(T), hipMemcpyDeviceToDevice, s));
  return PF_OK;
}

template <typename Tin, typename Tout>
__global__ void k_cast(Tout* y, const Tin* x, int64_t n) {
  GRID_STRIDE(i, n) y[i] = (Tout)x[i];
}
template <typename Tin, typename Tout>
pf_status vec_cast(Tout* y, const Tin* x, int64_t n, hipStream_t s) {
  if (n <= 0) return PF_OK;
  k_cast<Tin, Tout><<<nblocks(n), 256, 0, s>>>(y, x, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <typename T>
__global__ void k_init_constrained(T* y, const T* x, const uint8_t* mask, int64_t nn, int d) {
  const int64_t n = (int64_t)(d + 1) * nn;
  GRID_STRIDE(i, n) {
    const int c = (int)(i / nn);
    const int64_t node = i - (int64_t)c * nn;
    const bool con = mask[node] & mask_bit(c, d);
    y[i] = (con && x) ? x[i] : T(0);
  }
}
template <typename T>
pf_status vec_init_constrained(T* y, const T* x, const uint8_t* mask, int64_t nn, int d, hipStream_t s) {
  k_init_constrained<T><<<nblocks((d + 1) * nn), 256, 0, s>>>(y, x, mask, nn, d);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <typename T>
__global__ void k_set_constrained(T* y, T v, const uint8_t* mask, int64_t nn, int d) {
  const int64_t n = (int64_t)(d + 1) * nn;
  GRID_STRIDE(i, n) {
    const int c = (int)(i / nn);
    const int64_t node = i - (int64_t)c * nn;
    if (mask[node] & mask_bit(c, d)) y[i] = v;
  }
}
template <typename T>
pf_status vec_set_constrained(T* y, T v, const uint8_t* mask, int64_t nn, int d, hipStream_t s) {
  k_set_constrained<T><<<nblocks((d + 1) * nn), 256, 0, s>>>(y, v, mask, nn, d);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <typename T>
__global__ void k_axpby(T* y, T a, const T* x, T b, int64_t n) {
  GRID_STRIDE(i, n) y[i] = a * x[i] + b * y[i];
}
template <typename T>
pf_status vec_axpby(T* y, T a, const T* x, T b, int64_t n, hipStream_t s) {
  k_axpby<T><<<nblocks(n), 256, 0, s>>>(y, a, x, b, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <typename T>
__global__ void k_sub(T* z, const T* x, const T* y, int64_t n) {
  GRID_STRIDE(i, n) z[i] = x[i] - y[i];
}
template <typename T>
pf_status vec_sub(T* z, const T* x, const T* y, int64_t n, hipStream_t s) {
  k_sub<T><<<nblocks(n), 256, 0, s>>>(z, x, y, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

// Chebyshev-Jacobi step of the smoother (three-term recurrence, Sec. 3.2.1).
// diag holds diag(B~) (1 on constrained rows).  mode selects the residual the
// step starts from: 0 = res - t (t = B~ d of the previous direction);
// 1 = b with x = 0 (x is written, not read); 2 = b - t with t = G~ x;
// 3 = res as given.  t_next, if set, receives Pi_C of the new direction (or of
// the new x when next_of_x) as the starting value of the next operator apply.
// dc holds the step's coefficients in device memory, {c1, c2} of the
// displacement block then of the phase-field block, so that a captured launch
// stays valid when the eigenvalue bounds change.
template <typename T>
__global__ void k_cheb_step(T* res, const T* t, T* dv, T* x, const T* diag, const double* __restrict__ dc, int mode,
                            int64_t nn, int d, const uint8_t* mask, T* t_next, int next_of_x, const T* b) {
  const int64_t n = (int64_t)(d + 1) * nn;
  const int64_t nu = (int64_t)d * nn;
  const T c1u = (T)dc[0], c2u = (T)dc[1], c1p = (T)dc[2], c2p = (T)dc[3];
  GRID_STRIDE(i, n) {
    const bool phi = i >= nu;
    const T c1 = phi ? c1p : c1u, c2 = phi ? c2p : c2u;
    T r, dn, xn;
    if (mode == 0) {
      r = res[i] - t[i];
      res[i] = r;
      dn = c1 * dv[i] + c2 * r / diag[i];
      xn = x[i] + dn;
    } else {
      r = mode == 1 ? b[i] : (mode == 2 ? b[i] - t[i] : res[i]);
      if (mode != 3) res[i] = r;
      dn = c2 * r / diag[i];
      xn = mode == 1 ? dn : x[i] + dn;
    }
    dv[i] = dn;
    x[i] = xn;
    if (t_next) {
      const int c = (int)(i / nn);
      t_next[i] = (mask[i - (int64_t)c * nn] & mask_bit(c, d)) ? (next_of_x ? xn : dn) : T(0);
    }
  }
}
template <typename T>
pf_status vec_cheb_step(T* res, const T* t, T* dv, T* x, const T* diag, const double* dc, int mode, int64_t nn,
                        int d, const uint8_t* mask, T* t_next, int next_of_x, const T* b, hipStream_t s) {
  k_cheb_step<T><<<nblocks((d + 1) * nn), 256, 0, s>>>(res, t, dv, x, diag, dc, mode, nn, d, mask, t_next,
                                                       next_of_x, b);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

// Small host arrays (solver coefficients) written into device memory in stream order: the values
// travel as kernel arguments, so the host copy may change as soon as the call returns.
constexpr int kPutChunk = 256;
struct PutChunk {
  double v[kPutChunk];
};
__global__ void k_put(double* dst, PutChunk p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = p.v[i];
}
pf_status vec_put(double* dst, const double* src, int64_t n, hipStream_t s) {
  for (int64_t o = 0; o < n; o += kPutChunk) {
    const int m = (int)std::min<int64_t>(kPutChunk, n - o);
    PutChunk p;
    for (int i = 0; i < m; ++i) p.v[i] = src[o + i];
    k_put<<<1, 256, 0, s>>>(dst + o, p, m);
    PFF_CHECK_LAUNCH();
  }
  return PF_OK;
}

// ---------------------------------------------------------------------------
// reductions (deterministic: fixed grid, per-block partials, one final block)
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v) {
  __shared__ double sh[kRedBlock / 64];
  // wave64 reduction
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// partials[k * gridDim.x + block] for segment k = [b_k, b_{k+1}), k < nseg <= 2
template <typename T>
__global__ void k_dot_segments(const T* x, const T* y, int64_t b0, int64_t b1, int64_t b2, int nseg,
                               double* partials) {
  for (int k = 0; k < nseg; ++k) {
    const int64_t lo = k == 0 ? b0 : b1, hi = k == 0 ? b1 : b2;
    double acc = 0.0;
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += (int64_t)gridDim.x * blockDim.x)
      acc += (double)x[i] * (double)y[i];
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = b;
  }
}

__global__ void k_finalize(const double* partials, int nparts, int nseg, double* out) {
  for (int k = 0; k < nseg; ++k) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partials[k * nparts + i];
    const double b = block_sum(acc);
    if (threadIdx.x == 0) out[k] = b;
  }
}

// dot products over up to 2 segments; partials in d_part[0 .. 2*kRedMaxBlocks)
static pf_status dot_segments(const double* x, const double* y, const int64_t bounds[3], int nseg, double* d_part,
                              double* d_out, hipStream_t s) {
  const int64_t n = bounds[nseg];
  int nb = (int)nblocks(n, kRedBlock, kRedMaxBlocks);
  k_dot_segments<double><<<nb, kRedBlock, 0, s>>>(x, y, bounds[0], bounds[1], bounds[2], nseg, d_part);
  PFF_CHECK_LAUNCH();
  k_finalize<<<1, kRedBlock, 0, s>>>(d_part, nb, nseg, d_out);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

pf_status dot_blocks(const double* x, const double* y, int64_t nn, int d, double* d_part, double* h_out,
                     hipStream_t s) {
  const int64_t b[3] = {0, (int64_t)d * nn, (int64_t)(d + 1) * nn};
  double* d_out = d_part + 2 * kRedMaxBlocks;
  PFF_TRY(dot_segments(x, y, b, 2, d_part, d_out, s));
  PFF_HIP(hipMemcpyAsync(h_out, d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  PFF_HIP(hipStreamSynchronize(s));
  return PF_OK;
}

pf_status dot_host(const double* x, const double* y, int64_t n, double* d_part, double* h_out, hipStream_t s) {
  const int64_t b[3] = {0, n, n};
  double* d_out = d_part + 2 * kRedMaxBlocks;
  PFF_TRY(dot_segments(x, y, b, 1, d_part, d_out, s));
  PFF_HIP(hipMemcpyAsync(h_out, d_out, sizeof(double), hipMemcpyDeviceToHost, s));
  PFF_HIP(hipStreamSynchronize(s));
  return PF_OK;
}

pf_status nrm2_dev(const double* x, int64_t n, double* d_part, double* d_out, hipStream_t s) {
  const int64_t b[3] = {0, n, n};
  return dot_segments(x, x, b, 1, d_part, d_out, s);
}

// multi-dot: h[i] = V_i . w for i < k.  A thread reads w once and accumulates up to kMultiDotRows
// dots; partials[i * nb + block] (rows beyond one launch's kMultiDotRows take further launches).
__global__ void k_multi_dot(const double* V, int64_t ld, int k, const double* w, int64_t n, double* partials) {
  double acc[kMultiDotRows];
#pragma unroll
  for (int i = 0; i < kMultiDotRows; ++i) acc[i] = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    const double wt = w[t];
#pragma unroll
    for (int i = 0; i < kMultiDotRows; ++i)
      if (i < k) acc[i] += V[(int64_t)i * ld + t] * wt;
  }
  for (int i = 0; i < k; ++i) {
    const double b = block_sum(acc[i]);
    if (threadIdx.x == 0) partials[(int64_t)i * gridDim.x + blockIdx.x] = b;
  }
}

__global__ void k_finalize_rows(const double* partials, int nparts, double* out) {
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partials[(int64_t)k * nparts + i];
  const double b = block_sum(acc);
  if (threadIdx.x == 0) out[k] = b;
}

// d_part holds kMultiDotBlocks * k doubles
pf_status multi_dot(const double* V, int64_t ld, int k, const double* w, int64_t n, double* d_part, double* d_h,
                    hipStream_t s) {
  // at least 8 values per thread (small vectors: fewer partials to finish), at most kMultiDotBlocks
  const int nb = (int)nblocks(n, kRedBlock * 8, kMultiDotBlocks);
  for (int r0 = 0; r0 < k; r0 += kMultiDotRows) {
    const int kr = std::min(kMultiDotRows, k - r0);
    k_multi_dot<<<nb, kRedBlock, 0, s>>>(V + (int64_t)r0 * ld, ld, kr, w, n, d_part + (int64_t)r0 * nb);
    PFF_CHECK_LAUNCH();
  }
  k_finalize_rows<<<k, kRedBlock, 0, s>>>(d_part, nb, d_h);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__global__ void k_multi_axpy(double* w, const double* V, int64_t ld, int k, const double* h, int64_t n, double sign) {
  GRID_STRIDE(t, n) {
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += h[i] * V[(int64_t)i * ld + t];
    w[t] += sign * acc;
  }
}
pf_status multi_axpy(double* w, const double* V, int64_t ld, int k, const double* d_h, int64_t n, double sign,
                     hipStream_t s) {
  k_multi_axpy<<<nblocks(n), 256, 0, s>>>(w, V, ld, k, d_h, n, sign);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

// w -= sum_i h[i] V_i, then per-row partial dots of the new w with V_i (NORM false) or of w with
// itself (NORM true); the grid and the per-thread order are those of k_multi_dot
template <bool NORM>
__global__ void k_axpy_dot(double* w, const double* V, int64_t ld, int k, const double* h, int64_t n,
                           double* partials) {
  double hh[kMultiDotRows], acc[kMultiDotRows];
#pragma unroll
  for (int i = 0; i < kMultiDotRows; ++i) {
    hh[i] = i < k ? h[i] : 0.0;
    acc[i] = 0.0;
  }
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double v[kMultiDotRows];
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < kMultiDotRows; ++i) {
      v[i] = i < k ? V[(int64_t)i * ld + t] : 0.0;
      if (i < k) a += hh[i] * v[i];
    }
    const double wt = w[t] + -1.0 * a;
    w[t] = wt;
    if (NORM) {
      acc[0] += wt * wt;
    } else {
#pragma unroll
      for (int i = 0; i < kMultiDotRows; ++i)
        if (i < k) acc[i] += v[i] * wt;
    }
  }
  const int rows = NORM ? 1 : k;
  for (int i = 0; i < rows; ++i) {
    const double b = block_sum(acc[i]);
    if (threadIdx.x == 0) partials[(int64_t)i * gridDim.x + blockIdx.x] = b;
  }
}

pf_status axpy_then_dot(double* w, const double* V, int64_t ld, int k, const double* d_h, int64_t n, bool norm,
                        double* d_part, double* d_out, hipStream_t s) {
  if (k < 1 || k > kMultiDotRows) {
    set_error("axpy_then_dot: 1 to kMultiDotRows rows");
    return PF_ERR_INVALID_ARG;
  }
  const int nb = (int)nblocks(n, kRedBlock * 8, kMultiDotBlocks);
  if (norm)
    k_axpy_dot<true><<<nb, kRedBlock, 0, s>>>(w, V, ld, k, d_h, n, d_part);
  else
    k_axpy_dot<false><<<nb, kRedBlock, 0, s>>>(w, V, ld, k, d_h, n, d_part);
  PFF_CHECK_LAUNCH();
  k_finalize_rows<<<norm ? 1 : k, kRedBlock, 0, s>>>(d_part, nb, d_out);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__global__ void k_scale_inv_sqrt(double* y, const double* x, const double* nrm2, int64_t n) {
  const double nr = sqrt(*nrm2);
  const double f = nr > 0.0 ? 1.0 / nr : 0.0;
  GRID_STRIDE(i, n) y[i] = x[i] * f;
}
pf_status vec_scale_inv_sqrt(double* y, const double* x, const double* d_nrm2, int64_t n, hipStream_t s) {
  k_scale_inv_sqrt<<<nblocks(n), 256, 0, s>>>(y, x, d_nrm2, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__global__ void k_nonfinite(const double* x, int64_t n, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) acc += isfinite(x[i]) ? 0.0 : 1.0;
  const double b = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = b;
}
pf_status count_nonfinite(const double* x, int64_t n, double* d_part, double* h_out, hipStream_t s) {
  int nb = (int)nblocks(n, kRedBlock, kRedMaxBlocks);
  double* d_out = d_part + 2 * kRedMaxBlocks;
  k_nonfinite<<<nb, kRedBlock, 0, s>>>(x, n, d_part);
  PFF_CHECK_LAUNCH();
  k_finalize<<<1, kRedBlock, 0, s>>>(d_part, nb, 1, d_out);
  PFF_CHECK_LAUNCH();
  PFF_HIP(hipMemcpyAsync(h_out, d_out, sizeof(double), hipMemcpyDeviceToHost, s));
  PFF_HIP(hipStreamSynchronize(s));
  return PF_OK;
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014): state s + (i+1)*gamma through the
// variant-13 finalizer; doubles in [-1, 1) from the top 53 bits.
// ---------------------------------------------------------------------------
__device__ inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void k_eig_start(T* v, const uint8_t* mask, int64_t nn, int d, uint64_t seed_u, uint64_t seed_p) {
  const int64_t n = (int64_t)(d + 1) * nn;
  const int64_t nu = (int64_t)d * nn;
  GRID_STRIDE(i, n) {
    const int c = (int)(i / nn);
    const int64_t node = i - (int64_t)c * nn;
    const bool phi = i >= nu;
    const uint64_t ctr = (uint64_t)(phi ? i - nu : i);
    const uint64_t z = sm64_mix((phi ? seed_p : seed_u) + (ctr + 1ull) * 0x9E3779B97F4A7C15ull);
    const double u = (double)(z >> 11) * 0x1.0p-53;
    v[i] = (T)((mask[node] & mask_bit(c, d)) ? 0.0 : 2.0 * u - 1.0);
  }
}
template <typename T>
pf_status eig_start_vector(T* v, const uint8_t* mask, int64_t nn, int d, uint64_t seed_u, uint64_t seed_phi,
                           hipStream_t s) {
  k_eig_start<T><<<nblocks((d + 1) * nn), 256, 0, s>>>(v, mask, nn, d, seed_u, seed_phi);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__global__ void k_jacobi(double* y, const double* x, const double* diag, const uint8_t* mask, int64_t nn, int d) {
  const int64_t n = (int64_t)(d + 1) * nn;
  GRID_STRIDE(i, n) {
    const int c = (int)(i / nn);
    const int64_t node = i - (int64_t)c * nn;
    y[i] = (mask[node] & mask_bit(c, d)) ? 0.0 : x[i] / diag[i];
  }
}
pf_status vec_jacobi(double* y, const double* x, const double* diag, const uint8_t* mask, int64_t nn, int d,
                     hipStream_t s) {
  k_jacobi<<<nblocks((d + 1) * nn), 256, 0, s>>>(y, x, diag, mask, nn, d);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__global__ void k_xpby_blocks(double* y, const double* x, double bu, double bp, int64_t nu, int64_t n) {
  GRID_STRIDE(i, n) y[i] = x[i] + (i >= nu ? bp : bu) * y[i];
}
pf_status vec_xpby_blocks(double* y, const double* x, const double beta[2], int64_t nn, int d, hipStream_t s) {
  const int64_t n = (int64_t)(d + 1) * nn;
  k_xpby_blocks<<<nblocks(n), 256, 0, s>>>(y, x, beta[0], beta[1], (int64_t)d * nn, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

__global__ void k_axpy_blocks(double* y, const double* x, double au, double ap, int64_t nu, int64_t n) {
  GRID_STRIDE(i, n) y[i] += (i >= nu ? ap : au) * x[i];
}
pf_status vec_axpy_blocks(double* y, const double* x, const double alpha[2], int64_t nn, int d, hipStream_t s) {
  const int64_t n = (int64_t)(d + 1) * nn;
  k_axpy_blocks<<<nblocks(n), 256, 0, s>>>(y, x, alpha[0], alpha[1], (int64_t)d * nn, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

// ---------------------------------------------------------------------------
// device-resident Jacobi-PCG for the eigenvalue estimate.  The reductions use
// the same grid, loop order and final block as dot_blocks, so the
// coefficients equal those of a host-driven loop bit for bit.
// ---------------------------------------------------------------------------
// z = D^-1 (r - alpha q) on free DoFs (r updated when q != nullptr), p = z if
// p != nullptr; partials of (r, z) per block
template <typename T>
__global__ void k_eig_precond(T* r, const T* q, const EigDev* st, T* z, T* p, const T* diag,
                              const uint8_t* mask, int64_t nn, int d, double* partials) {
  // node-major: a thread takes a node and the components of one block, so the component of an
  // index needs no 64-bit division
  for (int k = 0; k < 2; ++k) {
    const int c0 = k == 0 ? 0 : d, c1 = k == 0 ? d : d + 1;
    const T na = q ? T(-st->alpha[k]) : T(0);
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nn; j += (int64_t)gridDim.x * blockDim.x) {
      const uint8_t m = mask[j];
      for (int c = c0; c < c1; ++c) {
        const int64_t i = (int64_t)c * nn + j;
        T ri = r[i];
        if (q) {
          ri += na * q[i];
          r[i] = ri;
        }
        const T zi = (m & mask_bit(c, d)) ? T(0) : ri / diag[i];
        z[i] = zi;
        if (p) p[i] = zi;
        acc += (double)ri * (double)zi;
      }
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partials[k * gridDim.x + blockIdx.x] = b;
  }
}

__global__ void k_eig_update(const double* partials, int nparts, EigDev* st, int phase) {
  double tot[2];
  for (int k = 0; k < 2; ++k) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partials[k * nparts + i];
    tot[k] = block_sum(acc);
  }
  if (threadIdx.x != 0) return;
  for (int k = 0; k < 2; ++k) {
    if (phase == 0) {
      st->rz[k] = st->rz0[k] = tot[k];
      st->done[k] = !(tot[k] > 0.0);
      st->n_al[k] = st->n_be[k] = 0;
      st->alpha[k] = st->beta[k] = 0.0;
    } else if (phase == 1) {
      double a = 0.0;
      if (!st->done[k]) {
        if (!(tot[k] > 0.0)) {
          st->done[k] = 1;
        } else {
          a = st->rz[k] / tot[k];
          st->al[k][st->n_al[k]++] = a;
        }
      }
      st->alpha[k] = a;
    } else {
      double b = 0.0;
      if (!st->done[k]) {
        b = tot[k] / st->rz[k];
        st->be[k][st->n_be[k]++] = b;
        st->rz[k] = tot[k];
        if (st->rz[k] <= 0.0 || st->rz[k] <= 1e-24 * st->rz0[k]) st->done[k] = 1;
      }
      st->beta[k] = b;
    }
  }
}

template <typename T>
__global__ void k_eig_xpby(T* p, const T* z, const EigDev* st, int64_t nu, int64_t n) {
  const T bu = T(st->beta[0]), bp = T(st->beta[1]);
  GRID_STRIDE(i, n) p[i] = z[i] + (i >= nu ? bp : bu) * p[i];
}

template <typename T>
pf_status eig_cg_begin(const T* r, T* z, T* p, const T* diag, const uint8_t* mask, int64_t nn,
                       int d, double* d_part, EigDev* st, hipStream_t s) {
  const int nb = (int)nblocks(nn, kRedBlock, kRedMaxBlocks);
  k_eig_precond<T><<<nb, kRedBlock, 0, s>>>(const_cast<T*>(r), nullptr, st, z, p, diag, mask, nn, d, d_part);
  PFF_CHECK_LAUNCH();
  k_eig_update<<<1, kRedBlock, 0, s>>>(d_part, nb, st, 0);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <typename T>
pf_status eig_cg_alpha(const T* p, const T* Ap, int64_t nn, int d, double* d_part, EigDev* st,
                       hipStream_t s) {
  const int64_t n = (int64_t)(d + 1) * nn;
  const int nb = (int)nblocks(n, kRedBlock, kRedMaxBlocks);
  k_dot_segments<T><<<nb, kRedBlock, 0, s>>>(p, Ap, 0, (int64_t)d * nn, n, 2, d_part);
  PFF_CHECK_LAUNCH();
  k_eig_update<<<1, kRedBlock, 0, s>>>(d_part, nb, st, 1);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

template <typename T>
pf_status eig_cg_beta(T* r, const T* Ap, T* z, T* p, const T* diag, const uint8_t* mask,
                      int64_t nn, int d, double* d_part, EigDev* st, hipStream_t s) {
  const int64_t n = (int64_t)(d + 1) * nn;
  const int nb = (int)nblocks(nn, kRedBlock, kRedMaxBlocks);
  k_eig_precond<T><<<nb, kRedBlock, 0, s>>>(r, Ap, st, z, nullptr, diag, mask, nn, d, d_part);
  PFF_CHECK_LAUNCH();
  k_eig_update<<<1, kRedBlock, 0, s>>>(d_part, nb, st, 2);
  PFF_CHECK_LAUNCH();
  k_eig_xpby<T><<<nblocks(n), 256, 0, s>>>(p, z, st, (int64_t)d * nn, n);
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

// explicit instantiations
#define INST_T(T)                                                                                             \
  template pf_status vec_fill<T>(T*, T, int64_t, hipStream_t);                                                 \
  template pf_status vec_copy<T>(T*, const T*, int64_t, hipStream_t);                                          \
  template pf_status vec_init_constrained<T>(T*, const T*, const uint8_t*, int64_t, int, hipStream_t);         \
  template pf_status vec_set_constrained<T>(T*, T, const uint8_t*, int64_t, int, hipStream_t);                 \
  template pf_status vec_axpby<T>(T*, T, const T*, T, int64_t, hipStream_t);                                   \
  template pf_status vec_sub<T>(T*, const T*, const T*, int64_t, hipStream_t);                                 \
  template pf_status vec_cheb_step<T>(T*, const T*, T*, T*, const T*, const double*, int, int64_t, int,          \
                                      const uint8_t*, T*, int, const T*, hipStream_t);
INST_T(double)
INST_T(float)
#define INST_EIG(T)                                                                                            \
  template pf_status eig_start_vector<T>(T*, const uint8_t*, int64_t, int, uint64_t, uint64_t, hipStream_t);   \
  template pf_status eig_cg_begin<T>(const T*, T*, T*, const T*, const uint8_t*, int64_t, int, double*, EigDev*, \
                                     hipStream_t);                                                              \
  template pf_status eig_cg_alpha<T>(const T*, const T*, int64_t, int, double*, EigDev*, hipStream_t);          \
  template pf_status eig_cg_beta<T>(T*, const T*, T*, T*, const T*, const uint8_t*, int64_t, int, double*,      \
                                    EigDev*, hipStream_t);
INST_EIG(double)
INST_EIG(float)
template pf_status vec_cast<double, float>(float*, const double*, int64_t, hipStream_t);
template pf_status vec_cast<float, double>(double*, const float*, int64_t, hipStream_t);

}  // namespace pff

namespace pff {
template pf_status vec_copy<uint8_t>(uint8_t*, const uint8_t*, int64_t, hipStream_t);
}  // namespace pff
