// Sum-factorized Q2 cell loop in 3D (the tensor-product apply of Sec. 4.1 for
// p = 2): nine threads per cell, one per (x, y) column of the 3x3x3 node and
// Gauss-point lattices.  A thread holds the three z-values of its column; the
// contractions along x and y exchange values through LDS, the one along z
// stays in registers.  Seven cells share a 64-thread workgroup (one
// wavefront, so the LDS barriers are cheap).
//
// Forward: nodal values -> values and gradients at the 27 Gauss points
// (three 3x3 contractions per direction instead of 27x27 direct sums).
// Pointwise: the integrands of the semi-linear form (no split, phi~ in the
// displacement equation, the 1/2 of the phase-field equation read literally).
// Backward: the adjoint contractions give the 27 nodal contributions, which
// are scattered with atomics (y pre-set for the masked modes).
#include "generic_cell.h"

namespace pff {

namespace {

constexpr int kQ2Cells = 7;  // cells per 64-thread workgroup (63 active threads)

// 1D tables on the Gauss points t_q: B[q][a] = L_a(t_q), D[q][a] = L_a'(t_q), weights W[q].
// Entries with compile-time indices fold into immediates; the lane-dependent rows and
// columns are read from a copy in LDS (one table per workgroup, broadcast reads), which
// keeps them out of the register file.
template <typename T>
struct Q2Tab {
  T B[3][3], D[3][3], W[3];
  // squared: B^2 and D^2 (the diagonal of the element matrices)
  __device__ explicit Q2Tab(bool squared = false) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      W[q] = T(B1<2>::wt(q));
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double b = B1<2>::val(a, B1<2>::pt(q)), d = B1<2>::der(a, B1<2>::pt(q));
        B[q][a] = T(squared ? b * b : b);
        D[q][a] = T(squared ? d * d : d);
      }
    }
  }
};

// the LDS copy of the (squared) tables, written by the first nine threads
template <typename T>
__device__ __forceinline__ void q2_fill_tables(T (&tb)[3][3], T (&td)[3][3], int tid, bool squared) {
  if (tid < 9) {
    const int q = tid / 3, a = tid % 3;
    const double t = B1<2>::pt(q), b = B1<2>::val(a, t), d = B1<2>::der(a, t);
    tb[q][a] = T(squared ? b * b : b);
    td[q][a] = T(squared ? d * d : d);
  }
}

// per-workgroup exchange buffers: [buffer][cell slot][az][ay][ax]; slot kQ2Cells belongs to
// the idle lane 63, which runs the same code (barriers) on its own data
template <typename T>
struct Q2Lds {
  T tb[3][3], td[3][3];  // B and D (or their squares for the diagonal)
  T s[3][kQ2Cells + 1][3][3][3];
  // per thread and Gauss point: g(phi~) JxW, the phase-field coefficient, the coupling tensor
  // (6); written and read by the same thread only (parked here to bound live registers).
  // Lane index fastest: a wavefront's accesses are 64 consecutive values, free of bank
  // conflicts (a per-thread row of 24 values put every lane on the same two banks).
  T q[3][8][64];
};

// Forward contraction of one scalar field.  col[az] = f(tx, ty, az).  Output at the
// thread's Gauss points (qx = tx, qy = ty, qz): val[qz] and, if GRAD, the physical
// gradient g[j][qz].
template <typename T, bool GRAD>
__device__ __forceinline__ void q2_forward(Q2Lds<T>& L, const Q2Tab<T>& k, int cs, int tx, int ty, const T col[3],
                                           const T ih[3], T val[3], T g[3][3]) {
  T (&S0)[3][3][3] = L.s[0][cs];
  T (&S1)[3][3][3] = L.s[1][cs];
#pragma unroll
  for (int az = 0; az < 3; ++az) S0[az][ty][tx] = col[az];
  __syncthreads();
  T bx[3], dx[3];
#pragma unroll
  for (int az = 0; az < 3; ++az) {
    bx[az] = L.tb[tx][0] * S0[az][ty][0] + L.tb[tx][1] * S0[az][ty][1] + L.tb[tx][2] * S0[az][ty][2];
    if (GRAD) dx[az] = L.td[tx][0] * S0[az][ty][0] + L.td[tx][1] * S0[az][ty][1] + L.td[tx][2] * S0[az][ty][2];
  }
  __syncthreads();
#pragma unroll
  for (int az = 0; az < 3; ++az) {
    S0[az][ty][tx] = bx[az];
    if (GRAD) S1[az][ty][tx] = dx[az];
  }
  __syncthreads();
  T bb[3], bd[3], db[3];
#pragma unroll
  for (int az = 0; az < 3; ++az) {
    bb[az] = L.tb[ty][0] * S0[az][0][tx] + L.tb[ty][1] * S0[az][1][tx] + L.tb[ty][2] * S0[az][2][tx];
    if (GRAD) {
      bd[az] = L.td[ty][0] * S0[az][0][tx] + L.td[ty][1] * S0[az][1][tx] + L.td[ty][2] * S0[az][2][tx];
      db[az] = L.tb[ty][0] * S1[az][0][tx] + L.tb[ty][1] * S1[az][1][tx] + L.tb[ty][2] * S1[az][2][tx];
    }
  }
  __syncthreads();
#pragma unroll
  for (int qz = 0; qz < 3; ++qz) {
    val[qz] = k.B[qz][0] * bb[0] + k.B[qz][1] * bb[1] + k.B[qz][2] * bb[2];
    if (GRAD) {
      g[0][qz] = ih[0] * (k.B[qz][0] * db[0] + k.B[qz][1] * db[1] + k.B[qz][2] * db[2]);
      g[1][qz] = ih[1] * (k.B[qz][0] * bd[0] + k.B[qz][1] * bd[1] + k.B[qz][2] * bd[2]);
      g[2][qz] = ih[2] * (k.D[qz][0] * bb[0] + k.D[qz][1] * bb[1] + k.D[qz][2] * bb[2]);
    }
  }
}

// Backward (adjoint) contraction: coefficients at the thread's Gauss points of the
// test value (cv, if VAL) and of the physical test gradient (c[j], already scaled by
// 1/h_j) -> out[az] at node (tx, ty, az).
template <typename T, bool VAL>
__device__ __forceinline__ void q2_backward(Q2Lds<T>& L, const Q2Tab<T>& k, int cs, int tx, int ty, const T cv[3],
                                            const T c[3][3], T out[3]) {
  T (&S0)[3][3][3] = L.s[0][cs];
  T (&S1)[3][3][3] = L.s[1][cs];
  T (&S2)[3][3][3] = L.s[2][cs];
  T z0[3], zx[3], zy[3];
#pragma unroll
  for (int az = 0; az < 3; ++az) {
    T a0 = T(0), ax = T(0), ay = T(0);
#pragma unroll
    for (int qz = 0; qz < 3; ++qz) {
      a0 += k.D[qz][az] * c[2][qz];
      if (VAL) a0 += k.B[qz][az] * cv[qz];
      ax += k.B[qz][az] * c[0][qz];
      ay += k.B[qz][az] * c[1][qz];
    }
    z0[az] = a0;
    zx[az] = ax;
    zy[az] = ay;
  }
#pragma unroll
  for (int az = 0; az < 3; ++az) {
    S0[az][ty][tx] = z0[az];
    S1[az][ty][tx] = zy[az];
    S2[az][ty][tx] = zx[az];
  }
  __syncthreads();
  T y0[3], yx[3];
#pragma unroll
  for (int az = 0; az < 3; ++az) {
    y0[az] = L.tb[0][ty] * S0[az][0][tx] + L.tb[1][ty] * S0[az][1][tx] + L.tb[2][ty] * S0[az][2][tx] +
             L.td[0][ty] * S1[az][0][tx] + L.td[1][ty] * S1[az][1][tx] + L.td[2][ty] * S1[az][2][tx];
    yx[az] = L.tb[0][ty] * S2[az][0][tx] + L.tb[1][ty] * S2[az][1][tx] + L.tb[2][ty] * S2[az][2][tx];
  }
  __syncthreads();
#pragma unroll
  for (int az = 0; az < 3; ++az) {
    S0[az][ty][tx] = y0[az];
    S1[az][ty][tx] = yx[az];
  }
  __syncthreads();
#pragma unroll
  for (int az = 0; az < 3; ++az)
    out[az] = L.tb[0][tx] * S0[az][ty][0] + L.tb[1][tx] * S0[az][ty][1] + L.tb[2][tx] * S0[az][ty][2] +
              L.td[0][tx] * S1[az][ty][0] + L.td[1][tx] * S1[az][ty][1] + L.td[2][tx] * S1[az][ty][2];
  __syncthreads();
}

}  // namespace

// Template-only mode: write the block operator's per-point coefficients g(phi~) JxW and c_phi
// of the linearization point, [k][point][cell] with k = 0, 1 and point = x + 3 y + 9 z, to y
// (FP64) instead of applying anything.
constexpr int kModeQ2Coef = 17;

// MODE: MODE_APPLY / MODE_BLOCK (masked direction, y pre-set to Pi_C x), MODE_RAW
// (unmasked G x), MODE_RESID (-A(U); x unused), MODE_DIAG (diag G, every row; x unused).
// The diagonal entry of node a is a sum over Gauss points of products of squared 1D
// basis values / derivatives, i.e. the backward contraction with the tables B^2, D^2.
// MODE_BLOCK reads g(phi~) JxW and c_phi per Gauss point from cp.qcb (kModeQ2Coef's
// output) and loads neither phi~ nor U.
template <typename T, int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_q2_3d(CellParams cp, const T* __restrict__ x, const T* __restrict__ U,
                                              const T* __restrict__ phit, const uint8_t* __restrict__ mask,
                                              T* __restrict__ y) {
  constexpr bool kMasked = (MODE == MODE_APPLY || MODE == MODE_BLOCK);
  constexpr bool kCouple = (MODE == MODE_APPLY || MODE == MODE_RAW);
  constexpr bool kResid = (MODE == MODE_RESID);
  constexpr bool kDiag = (MODE == MODE_DIAG);
  constexpr bool kStored = (MODE == MODE_BLOCK);
  constexpr bool kCoef = (MODE == kModeQ2Coef);
  __shared__ Q2Lds<T> L;
  const int tid = threadIdx.x;
  const int cs = tid / 9;  // 0 .. kQ2Cells (the last slot is the idle lane's)
  const int tx = (tid % 9) % 3, ty = (tid % 9) / 3;
  const Q2Tab<T> k;
  q2_fill_tables(L.tb, L.td, tid, false);
  __syncthreads();
  // workgroups are dealt to the 8 XCDs round-robin: give each XCD one contiguous range of cell
  // groups, so that neighbouring cells read their shared nodes through one L2
  const int64_t nb = gridDim.x, qq = nb / 8, rr = nb % 8, xcd = blockIdx.x % 8;
  const int64_t grp = xcd * qq + (xcd < rr ? xcd : rr) + blockIdx.x / 8;
  const int64_t cid = grp * kQ2Cells + tid / 9;
  bool active = tid < 9 * kQ2Cells && cid < cp.n_cells;
  int cx = 0, cy = 0, cz = 0;
  if (active) {
    cx = (int)(cid % cp.N[0]);
    cy = (int)((cid / cp.N[0]) % cp.N[1]);
    cz = (int)(cid / ((int64_t)cp.N[0] * cp.N[1]));
    active = !cell_in_hole(cp.lshape, cx, cy, cp.N[0], cp.N[1]);
  }
  const int64_t nn = cp.n_nodes;
  int64_t gi[3];
#pragma unroll
  for (int az = 0; az < 3; ++az)
    gi[az] = active ? (int64_t)(2 * cx + tx) + (int64_t)(2 * cy + ty) * cp.ns[1] + (int64_t)(2 * cz + az) * cp.ns[2]
                    : 0;
  uint8_t mk[3];
#pragma unroll
  for (int az = 0; az < 3; ++az) mk[az] = (active && kMasked) ? mask[gi[az]] : (uint8_t)0;
  const T ih[3] = {T(cp.inv_h[0]), T(cp.inv_h[1]), T(cp.inv_h[2])};
  const T mu = T(cp.mu), lam = T(cp.lam), kap = T(cp.kappa), pres = T(cp.pres);
  const T gce = T(cp.gc_over_eps), gcx = T(cp.gc_eps);
  T jxw[3];
#pragma unroll
  for (int qz = 0; qz < 3; ++qz) jxw[qz] = T(cp.vol * B1<2>::wt(tx) * B1<2>::wt(ty)) * k.W[qz];

  // linearization point at the Gauss points: g(phi~), and the phase-field coefficients
  T col[3], tmp[3][3];
  T pt[3] = {T(0), T(0), T(0)};
  T phv[3], gphi[3][3];
  T gdeg[3], cphi[3], Ksym[3][6], rf[3], rsu[3][6];
  if constexpr (kStored) {
    // g(phi~) JxW and c_phi of the thread's three Gauss points, written at the linearization
    const T* qc = (const T*)cp.qcb;
    const int64_t nc = cp.n_cells, q0 = tid % 9;
#pragma unroll
    for (int qz = 0; qz < 3; ++qz) {
      gdeg[qz] = active ? qc[(q0 + 9 * qz) * nc + cid] : T(0);
      cphi[qz] = active ? qc[(27 + q0 + 9 * qz) * nc + cid] : T(0);
    }
  } else {
#pragma unroll
    for (int az = 0; az < 3; ++az) col[az] = active ? phit[gi[az]] : T(0);
    q2_forward<T, false>(L, k, cs, tx, ty, col, ih, pt, tmp);
    if (kCouple || kResid) {
#pragma unroll
      for (int az = 0; az < 3; ++az) col[az] = active ? U[3 * nn + gi[az]] : T(0);
      if (kResid)
        q2_forward<T, true>(L, k, cs, tx, ty, col, ih, phv, gphi);
      else
        q2_forward<T, false>(L, k, cs, tx, ty, col, ih, phv, gphi);
    }
    T gu[3][3][3];  // [component][direction][qz]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int az = 0; az < 3; ++az) col[az] = active ? U[c * nn + gi[az]] : T(0);
      T v[3];
      q2_forward<T, true>(L, k, cs, tx, ty, col, ih, v, gu[c]);
    }
    // per Gauss point: gdeg, cphi = (1-kappa) E_s + 2 p div u + G_c/eps, and the coupling
    // tensor K = (1-kappa) phi sigma(u) + 2 p phi I (APPLY / RAW) or the residual terms
#pragma unroll
    for (int qz = 0; qz < 3; ++qz) {
      const T e00 = gu[0][0][qz], e11 = gu[1][1][qz], e22 = gu[2][2][qz];
      const T e01 = T(0.5) * (gu[0][1][qz] + gu[1][0][qz]);
      const T e02 = T(0.5) * (gu[0][2][qz] + gu[2][0][qz]);
      const T e12 = T(0.5) * (gu[1][2][qz] + gu[2][1][qz]);
      const T tr = e00 + e11 + e22;
      const T ee = e00 * e00 + e11 * e11 + e22 * e22 + T(2) * (e01 * e01 + e02 * e02 + e12 * e12);
      const T Es = T(0.5) * lam * tr * tr + mu * ee;
      gdeg[qz] = (T(1) - kap) * pt[qz] * pt[qz] + kap;
      cphi[qz] = (T(1) - kap) * Es + T(2) * pres * tr + gce;
      const T s00 = T(2) * mu * e00 + lam * tr, s11 = T(2) * mu * e11 + lam * tr, s22 = T(2) * mu * e22 + lam * tr;
      const T s01 = T(2) * mu * e01, s02 = T(2) * mu * e02, s12 = T(2) * mu * e12;
      if (kCouple) {
        const T a = (T(1) - kap) * phv[qz], b = T(2) * pres * phv[qz];
        Ksym[qz][0] = a * s00 + b;
        Ksym[qz][1] = a * s11 + b;
        Ksym[qz][2] = a * s22 + b;
        Ksym[qz][3] = a * s01;
        Ksym[qz][4] = a * s02;
        Ksym[qz][5] = a * s12;
      }
      if (kResid) {
        const T ph = phv[qz], p2 = pt[qz] * pt[qz] * pres;
        rsu[qz][0] = -(gdeg[qz] * s00 + p2);
        rsu[qz][1] = -(gdeg[qz] * s11 + p2);
        rsu[qz][2] = -(gdeg[qz] * s22 + p2);
        rsu[qz][3] = -gdeg[qz] * s01;
        rsu[qz][4] = -gdeg[qz] * s02;
        rsu[qz][5] = -gdeg[qz] * s12;
        rf[qz] = -((T(1) - kap) * ph * Es + T(2) * ph * pres * tr - gce * (T(1) - ph));
      }
    }
  }

  if constexpr (kCoef) {
    // the block operator's coefficients of this thread's Gauss points (every cell of the level)
    const int64_t nc = cp.n_cells, q0 = tid % 9;
    if (tid < 9 * kQ2Cells && cid < nc)
#pragma unroll
      for (int qz = 0; qz < 3; ++qz) {
        y[(q0 + 9 * qz) * nc + cid] = gdeg[qz] * jxw[qz];
        y[(27 + q0 + 9 * qz) * nc + cid] = cphi[qz];
      }
    return;
  }

  if constexpr (kDiag) {
    const Q2Tab<T> k2(true);
    __syncthreads();  // every read of the plain tables is done
    q2_fill_tables(L.tb, L.td, tid, true);
    __syncthreads();
    T cv[3], cg[3][3], out[3];
    // u_c rows: gdeg (mu |grad N_a|^2 + (mu + lambda) (d_c N_a)^2)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int qz = 0; qz < 3; ++qz) {
          cv[qz] = T(0);
          cg[j][qz] = jxw[qz] * gdeg[qz] * (j == c ? T(2) * mu + lam : mu) * ih[j] * ih[j];
        }
      q2_backward<T, false>(L, k2, cs, tx, ty, cv, cg, out);
      if (active)
#pragma unroll
        for (int az = 0; az < 3; ++az) atomicAdd(&y[c * nn + gi[az]], out[az]);
    }
    // phase-field row: cphi N_a^2 + G_c eps |grad N_a|^2
#pragma unroll
    for (int qz = 0; qz < 3; ++qz) {
      cv[qz] = jxw[qz] * cphi[qz];
#pragma unroll
      for (int j = 0; j < 3; ++j) cg[j][qz] = jxw[qz] * gcx * ih[j] * ih[j];
    }
    q2_backward<T, true>(L, k2, cs, tx, ty, cv, cg, out);
    if (active)
#pragma unroll
      for (int az = 0; az < 3; ++az) atomicAdd(&y[3 * nn + gi[az]], out[az]);
    return;
  }

  // displacement rows: test-gradient coefficients per component
  T tau[3][6];  // symmetric tau per Gauss point: 00 11 22 01 02 12 (times JxW)
  T fcpl[3] = {T(0), T(0), T(0)};
  if (kResid) {
#pragma unroll
    for (int qz = 0; qz < 3; ++qz)
#pragma unroll
      for (int m = 0; m < 6; ++m) tau[qz][m] = rsu[qz][m] * jxw[qz];
  } else {
    // park the linearization data of the thread's Gauss points; tau and the coupling term
    // accumulate one direction component at a time (tau is linear in grad du)
    auto Q = [&](int qz, int m) -> T& { return L.q[qz][m][tid]; };
#pragma unroll
    for (int qz = 0; qz < 3; ++qz) {
      Q(qz, 0) = kStored ? gdeg[qz] : gdeg[qz] * jxw[qz];
      Q(qz, 1) = cphi[qz];
      if (kCouple)
#pragma unroll
        for (int m = 0; m < 6; ++m) Q(qz, 2 + m) = Ksym[qz][m];
#pragma unroll
      for (int m = 0; m < 6; ++m) tau[qz][m] = T(0);
    }
    constexpr int kSym[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int az = 0; az < 3; ++az) {
        T v = active ? x[c * nn + gi[az]] : T(0);
        col[az] = (mk[az] & (1 << c)) ? T(0) : v;
      }
      T v[3], gdc[3][3];
      q2_forward<T, true>(L, k, cs, tx, ty, col, ih, v, gdc);
#pragma unroll
      for (int qz = 0; qz < 3; ++qz) {
        const T w = Q(qz, 0);
        const T tl = w * lam * gdc[c][qz];
        tau[qz][0] += tl;
        tau[qz][1] += tl;
        tau[qz][2] += tl;
        tau[qz][c] += w * T(2) * mu * gdc[c][qz];
#pragma unroll
        for (int j = 0; j < 3; ++j)
          if (j != c) tau[qz][kSym[c][j]] += w * mu * gdc[j][qz];
        if (kCouple) {
          T f = T(0);
#pragma unroll
          for (int j = 0; j < 3; ++j) f += Q(qz, 2 + kSym[c][j]) * gdc[j][qz];
          fcpl[qz] += f;
        }
      }
    }
  }
  // the symmetric tau row of component c: (c, 0), (c, 1), (c, 2)
  constexpr int kRow[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T cg[3][3], cv0[3] = {T(0), T(0), T(0)}, out[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int qz = 0; qz < 3; ++qz) cg[j][qz] = tau[qz][kRow[c][j]] * ih[j];
    q2_backward<T, false>(L, k, cs, tx, ty, cv0, cg, out);
    if (active)
#pragma unroll
      for (int az = 0; az < 3; ++az)
        if (!(mk[az] & (1 << c))) atomicAdd(&y[c * nn + gi[az]], out[az]);
  }

  // phase-field row
  T cv[3], cg[3][3], out[3];
  if (kResid) {
#pragma unroll
    for (int qz = 0; qz < 3; ++qz) {
      cv[qz] = rf[qz] * jxw[qz];
#pragma unroll
      for (int j = 0; j < 3; ++j) cg[j][qz] = -gcx * gphi[j][qz] * jxw[qz] * ih[j];
    }
  } else {
#pragma unroll
    for (int az = 0; az < 3; ++az) {
      T v = active ? x[3 * nn + gi[az]] : T(0);
      col[az] = (mk[az] & kMaskPhi) ? T(0) : v;
    }
    T dpv[3], gdp[3][3];
    q2_forward<T, true>(L, k, cs, tx, ty, col, ih, dpv, gdp);
#pragma unroll
    for (int qz = 0; qz < 3; ++qz) {
      cv[qz] = (L.q[qz][1][tid] * dpv[qz] + fcpl[qz]) * jxw[qz];
#pragma unroll
      for (int j = 0; j < 3; ++j) cg[j][qz] = gcx * gdp[j][qz] * jxw[qz] * ih[j];
    }
  }
  q2_backward<T, true>(L, k, cs, tx, ty, cv, cg, out);
  if (active)
#pragma unroll
    for (int az = 0; az < 3; ++az)
      if (!(mk[az] & kMaskPhi)) atomicAdd(&y[3 * nn + gi[az]], out[az]);
}

// 3D Q2 apply / raw / residual modes; *handled = false for other shapes and modes
template <typename T>
pf_status launch_cell_q2(const Geom& g, const CellParams& cp, int mode, const T* x, const T* U, const T* phit,
                         const uint8_t* mask, T* y, hipStream_t s, bool* handled) {
  *handled = false;
  if (g.d != 3 || g.p != 2) return PF_OK;
  const bool fp64 = sizeof(T) == 8;
  if (!(mode == MODE_APPLY || mode == MODE_BLOCK || (fp64 && (mode == MODE_RAW || mode == MODE_RESID || mode == MODE_DIAG))))
    return PF_OK;
  *handled = true;
  if (mode == MODE_BLOCK && !cp.qcb) {
    set_error("Q2 block operator: the level's stored coefficients are missing");
    return PF_ERR_UNSUPPORTED;
  }
  const int64_t nb = (g.n_cells + kQ2Cells - 1) / kQ2Cells;
  if (nb == 0) return PF_OK;
  switch (mode) {
    case MODE_APPLY:
      k_q2_3d<T, MODE_APPLY><<<nb, 64, 0, s>>>(cp, x, U, phit, mask, y);
      break;
    case MODE_BLOCK:
      k_q2_3d<T, MODE_BLOCK><<<nb, 64, 0, s>>>(cp, x, U, phit, mask, y);
      break;
    case MODE_RAW:
      k_q2_3d<T, MODE_RAW><<<nb, 64, 0, s>>>(cp, x, U, phit, mask, y);
      break;
    case MODE_DIAG:
      k_q2_3d<T, MODE_DIAG><<<nb, 64, 0, s>>>(cp, x, U, phit, mask, y);
      break;
    default:
      k_q2_3d<T, MODE_RESID><<<nb, 64, 0, s>>>(cp, x, U, phit, mask, y);
      break;
  }
  PFF_CHECK_LAUNCH();
  return PF_OK;
}

// the block operator's per-point coefficients of a 3D Q2 level: g(phi~) JxW and c_phi, FP64 and FP32
pf_status launch_block_coef_q2(const Geom& g, const CellParams& cp, const double* U, const double* phit, double* c64,
                               float* c32, hipStream_t s) {
  if (g.d != 3 || g.p != 2 || !c64 || !c32) {
    set_error("block coefficients: 3D Q2 levels with coefficient storage only");
    return PF_ERR_UNSUPPORTED;
  }
  const int64_t nb = (g.n_cells + kQ2Cells - 1) / kQ2Cells;
  if (nb == 0) return PF_OK;
  k_q2_3d<double, kModeQ2Coef><<<nb, 64, 0, s>>>(cp, nullptr, U, phit, nullptr, c64);
  PFF_CHECK_LAUNCH();
  return vec_cast<double, float>(c32, c64, (int64_t)54 * g.n_cells, s);
}

pf_status launch_cell_q2_d(const Geom& g, const CellParams& cp, int mode, const double* x, const double* U,
                           const double* phit, const uint8_t* mask, double* y, hipStream_t s, bool* handled) {
  return launch_cell_q2<double>(g, cp, mode, x, U, phit, mask, y, s, handled);
}
pf_status launch_cell_q2_f(const Geom& g, const CellParams& cp, int mode, const float* x, const float* U,
                           const float* phit, const uint8_t* mask, float* y, hipStream_t s, bool* handled) {
  return launch_cell_q2<float>(g, cp, mode, x, U, phit, mask, y, s, handled);
}

}  // namespace pff
