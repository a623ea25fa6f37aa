// Device code shared by the per-stage kernels: the structured application of
// the cluster Hamiltonian to a column of a cluster matrix and the arguments
// of one Runge-Kutta stage.
#pragma once

#include "common.hpp"

namespace cdtwa {

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for the thread's outstanding global loads and stores, so
// loads issued before it stay in flight across it.  For barriers whose only
// purpose is LDS data exchanged between the waves of a workgroup.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Structured application of the cluster Hamiltonian
//   H_mu = U sum_l h_l - J sum_{intra bonds (l,m)} (a_l^+ a_m + a_m^+ a_l)
//          - J sum_l (conj(phi_l) a_l + phi_l a_l^+)
// (Sec. II Eq. (cluster_mf); App. B.1 Gamma^intra and Phi^inter) to column q
// of Y: every term shifts the Kronecker digits of the row index.
// ---------------------------------------------------------------------------
template <int CX, int CY>
struct Bonds;
template <>
struct Bonds<1, 1> {
  static constexpr int n = 0;
  __device__ static int l(int) { return 0; }
  __device__ static int m(int) { return 0; }
};
template <>
struct Bonds<2, 1> {
  static constexpr int n = 1;
  __device__ static int l(int) { return 0; }
  __device__ static int m(int) { return 1; }
};
template <>
struct Bonds<1, 2> {
  static constexpr int n = 1;
  __device__ static int l(int) { return 0; }
  __device__ static int m(int) { return 1; }
};
// 2x2: local index x*2+y; bonds 1-2, 1-3, 2-4, 3-4 of App. B.1 (0-based)
template <>
struct Bonds<2, 2> {
  static constexpr int n = 4;
  __device__ static int l(int b) { return b == 3 ? 2 : (b == 2 ? 1 : 0); }
  __device__ static int m(int b) { return b == 0 ? 1 : (b == 1 ? 2 : 3); }
};

// explicit fused multiply-add: the per-stage arithmetic must not depend on
// where the compiler chooses to contract a*b + c, so that every kernel that
// runs it (any workgroup size, any clusters per workgroup) rounds alike
__device__ inline double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int d>
__device__ inline double sqrt_int(int n) {
  // sqrt(n) for 0 <= n < d, exact to rounding
  return n == 0 ? 0.0 : (n == 1 ? 1.0 : (n == 2 ? 1.4142135623730951 : 1.7320508075688772));
}

// M[p][q] = (H Y)[p][q] from a copy Yc of the columns of one cluster matrix
// that holds row r of column q at Yc[r * LD + q] (LD = D: the whole matrix)
template <typename R, int d, int CX, int CY, int LD = cluster_dim<d, CX * CY>()>
__device__ inline cpx<R> apply_h(const cpx<R>* __restrict__ Yc, int p, int q, const cpx<R>* phi, R J, R U) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  int nd[NLOC];
#pragma unroll
  for (int l = 0; l < NLOC; ++l) nd[l] = digit<d, NLOC>(p, l);
  R diag = 0;
#pragma unroll
  for (int l = 0; l < NLOC; ++l) diag += R(0.5) * R(nd[l] * (nd[l] - 1));
  diag *= U;
  const cpx<R> y0 = Yc[p * LD + q];
  R re = diag * y0.re, im = diag * y0.im;
#pragma unroll
  for (int b = 0; b < Bonds<CX, CY>::n; ++b) {
    const int l = Bonds<CX, CY>::l(b), m = Bonds<CX, CY>::m(b);
    const int sl = kron_stride<d, NLOC>(l), sm = kron_stride<d, NLOC>(m);
    if (nd[l] >= 1 && nd[m] <= d - 2) {  // a_l^+ a_m
      const R c = -J * R(sqrt_int<d>(nd[l]) * sqrt_int<d>(nd[m] + 1));
      const cpx<R> y = Yc[(p - sl + sm) * LD + q];
      re = fma_r(c, y.re, re);
      im = fma_r(c, y.im, im);
    }
    if (nd[m] >= 1 && nd[l] <= d - 2) {  // a_m^+ a_l
      const R c = -J * R(sqrt_int<d>(nd[m]) * sqrt_int<d>(nd[l] + 1));
      const cpx<R> y = Yc[(p - sm + sl) * LD + q];
      re = fma_r(c, y.re, re);
      im = fma_r(c, y.im, im);
    }
  }
#pragma unroll
  for (int l = 0; l < NLOC; ++l) {
    const int sl = kron_stride<d, NLOC>(l);
    if (nd[l] <= d - 2) {  // -J conj(phi_l) a_l
      const R c = -J * R(sqrt_int<d>(nd[l] + 1));
      const cpx<R> y = Yc[(p + sl) * LD + q];
      const R fr = c * phi[l].re, fi = -c * phi[l].im;
      re = fma_r(fr, y.re, re);
      re = fma_r(-fi, y.im, re);
      im = fma_r(fr, y.im, im);
      im = fma_r(fi, y.re, im);
    }
    if (nd[l] >= 1) {  // -J phi_l a_l^+
      const R c = -J * R(sqrt_int<d>(nd[l]));
      const cpx<R> y = Yc[(p - sl) * LD + q];
      const R fr = c * phi[l].re, fi = c * phi[l].im;
      re = fma_r(fr, y.re, re);
      re = fma_r(-fi, y.im, re);
      im = fma_r(fr, y.im, im);
      im = fma_r(fi, y.re, im);
    }
  }
  return cmake(re, im);
}

// Local Lindblad dissipator (the open-system extension: channels
// L = sqrt(gd) n_l and L = sqrt(gl) a_l on every site l of the cluster) at
// entry (p, q):  sum_l [ gl sqrt((n_l(p)+1)(n_l(q)+1)) Y[p+s_l][q+s_l]
//                        - (gd/2 (n_l(p) - n_l(q))^2 + gl/2 (n_l(p) + n_l(q))) Y[p][q] ]
template <typename R, int d, int CX, int CY>
__device__ inline cpx<R> dissipate(const cpx<R>* __restrict__ Yc, int p, int q, R gd, R gl) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  R re = 0, im = 0, diag = 0;
#pragma unroll
  for (int l = 0; l < NLOC; ++l) {
    const int np = digit<d, NLOC>(p, l), nq = digit<d, NLOC>(q, l);
    diag = fma_r(R(-0.5) * gd, R((np - nq) * (np - nq)), diag);
    diag = fma_r(R(-0.5) * gl, R(np + nq), diag);
    if (np <= d - 2 && nq <= d - 2) {
      const int sl = kron_stride<d, NLOC>(l);
      const R c = gl * R(sqrt_int<d>(np + 1) * sqrt_int<d>(nq + 1));
      const cpx<R> u = Yc[(p + sl) * D + q + sl];
      re = fma_r(c, u.re, re);
      im = fma_r(c, u.im, im);
    }
  }
  const cpx<R> y = Yc[p * D + q];
  return cmake(fma_r(diag, y.re, re), fma_r(diag, y.im, im));
}

// ---------------------------------------------------------------------------
// Arguments of one classical RK4 stage (mode 1..4) or of the bare commutator
// (mode 0):
//   mode 0: Y = rho,              K written to kout
//   mode 1: Y = rho,              K1 -> kout, b(rho + dt/2 K1) -> b_out
//   mode 2: Y = rho + dt/2 K1,    K2 -> kout, b(rho + dt/2 K2) -> b_out
//   mode 3: Y = rho + dt/2 K2,    K3 -> kout, b(rho + dt K3)   -> b_out
//   mode 4: Y = rho + dt K3,      rho += dt/6 (K1 + 2K2 + 2K3 + K4), b(rho) -> b_out
// b_in holds the mean fields of Y for every site of every trajectory.
// ---------------------------------------------------------------------------
template <typename R>
struct StageArgs {
  Geom g;
  cpx<R>* rho;
  const cpx<R>* kprev;  // K_{s-1} (modes 2..4)
  const cpx<R>* k1;     // mode 4
  const cpx<R>* k2;     // mode 4
  cpx<R>* kout;         // modes 0..3
  const cpx<R>* b_in;
  cpx<R>* b_out;        // modes 1..4
  R dt;
  int mode;
};

// One stage for the CPB clusters first .. first+CPB-1 (flat (trajectory,
// cluster) indices) with NT threads; sY: CPB*D*D entries of LDS, sPhi:
// CPB*NLOC entries of LDS.  DISS: add the local Lindblad dissipator.
template <typename R, int d, int CX, int CY, int CPB, int NT, bool DISS = false>
__device__ inline void stage_body(const StageArgs<R>& a, const int64_t first, cpx<R>* __restrict__ sY,
                                  cpx<R>* __restrict__ sPhi) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  constexpr int DD = D * D;
  constexpr int NE = CPB * DD;
  constexpr int EPT = (NE + NT - 1) / NT;
  const Geom& g = a.g;
  const int64_t total = g.n_traj * g.nc;
  const R J = R(g.J), U = R(g.U);
  const int mode = a.mode;
  const R cin = mode == 4 ? a.dt : R(0.5) * a.dt;        // Y_s = rho + cin K_{s-1}
  const R cout = mode == 3 ? a.dt : R(0.5) * a.dt;       // Y_{s+1} = rho + cout K_s

  cpx<R> rv[EPT], kp[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e >= NE || first + e / DD >= total) continue;
    const int64_t gidx = first * DD + e;
    rv[i] = a.rho[gidx];
    cpx<R> y = rv[i];
    if (mode >= 2) {
      kp[i] = a.kprev[gidx];
      y.re = fma_r(cin, kp[i].re, y.re);
      y.im = fma_r(cin, kp[i].im, y.im);
    }
    sY[e] = y;
  }
  // boundary fields of the clusters of this block
  for (int i = threadIdx.x; i < CPB * NLOC; i += NT) {
    const int gi = i / NLOC, l = i % NLOC;
    const int64_t flat = first + gi;
    if (flat >= total) continue;
    const int64_t t = flat / g.nc;
    const int mu = (int)(flat % g.nc);
    const int j = g.cluster_site[mu * NLOC + l];
    R re = 0, im = 0;
    for (int k = 0; k < 4; ++k) {
      const int n = g.ext_nbr[j * 4 + k];
      if (n < 0) continue;
      const cpx<R> v = a.b_in[t * g.Ns + n];
      re += v.re;
      im += v.im;
    }
    sPhi[gi * NLOC + l] = cmake(re, im);
  }
  __syncthreads();
  cpx<R> m[EPT], dv[DISS ? EPT : 1];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e >= NE) continue;
    const int gi = e / DD, pq = e % DD;
    m[i] = apply_h<R, d, CX, CY>(sY + gi * DD, pq / D, pq % D, sPhi + gi * NLOC, J, U);
    if constexpr (DISS) dv[i] = dissipate<R, d, CX, CY>(sY + gi * DD, pq / D, pq % D, R(g.gdeph), R(g.gloss));
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < NE) sY[e] = m[i];
  }
  __syncthreads();
  // K = -i (M - M^+):  K.re = Im M_pq + Im M_qp,  K.im = Re M_qp - Re M_pq
  cpx<R> yn[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e >= NE || first + e / DD >= total) continue;
    const int gi = e / DD, pq = e % DD, p = pq / D, q = pq % D;
    const cpx<R> mt = sY[gi * DD + q * D + p];
    cpx<R> kk = cmake(m[i].im + mt.im, mt.re - m[i].re);
    if constexpr (DISS) {
      kk.re += dv[i].re;
      kk.im += dv[i].im;
    }
    const int64_t gidx = first * DD + e;
    if (mode <= 3) {
      a.kout[gidx] = kk;
      yn[i] = cmake(fma_r(cout, kk.re, rv[i].re), fma_r(cout, kk.im, rv[i].im));
    } else {
      const cpx<R> q1 = a.k1[gidx], q2 = a.k2[gidx];
      const R h6 = a.dt / R(6);
      const R sr = fma_r(R(2), kp[i].re, fma_r(R(2), q2.re, q1.re)) + kk.re;
      const R si = fma_r(R(2), kp[i].im, fma_r(R(2), q2.im, q1.im)) + kk.im;
      yn[i] = cmake(fma_r(h6, sr, rv[i].re), fma_r(h6, si, rv[i].im));
      a.rho[gidx] = yn[i];
    }
  }
  if (mode == 0) return;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < NE && first + e / DD < total) sY[e] = yn[i];
  }
  __syncthreads();
  // mean fields of Y_{s+1}: b_l = sum_q sqrt(n_l(q)+1) Y[q+s_l][q]
  for (int i = threadIdx.x; i < CPB * NLOC; i += NT) {
    const int gi = i / NLOC, l = i % NLOC;
    const int64_t flat = first + gi;
    if (flat >= total) continue;
    const int64_t t = flat / g.nc;
    const int mu = (int)(flat % g.nc);
    const int sl = kron_stride<d, NLOC>(l);
    R re = 0, im = 0;
    for (int q = 0; q < D; ++q) {
      const int n = digit<d, NLOC>(q, l);
      if (n > d - 2) continue;
      const R c = R(sqrt_int<d>(n + 1));
      const cpx<R> y = sY[gi * DD + (q + sl) * D + q];
      re = fma_r(c, y.re, re);
      im = fma_r(c, y.im, im);
    }
    a.b_out[t * g.Ns + g.cluster_site[mu * NLOC + l]] = cmake(re, im);
  }
}

}  // namespace cdtwa
