// Device code shared by the per-stage kernels: the structured application of
// the cluster Hamiltonian to a column of a cluster matrix and the arguments
// of one Runge-Kutta stage.
#pragma once

#include "common.hpp"

namespace cdtwa {

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
      re += c * y.re;
      im += c * y.im;
    }
    if (nd[m] >= 1 && nd[l] <= d - 2) {  // a_m^+ a_l
      const R c = -J * R(sqrt_int<d>(nd[m]) * sqrt_int<d>(nd[l] + 1));
      const cpx<R> y = Yc[(p - sm + sl) * LD + q];
      re += c * y.re;
      im += c * y.im;
    }
  }
#pragma unroll
  for (int l = 0; l < NLOC; ++l) {
    const int sl = kron_stride<d, NLOC>(l);
    if (nd[l] <= d - 2) {  // -J conj(phi_l) a_l
      const R c = -J * R(sqrt_int<d>(nd[l] + 1));
      const cpx<R> y = Yc[(p + sl) * LD + q];
      const R fr = c * phi[l].re, fi = -c * phi[l].im;
      re += fr * y.re - fi * y.im;
      im += fr * y.im + fi * y.re;
    }
    if (nd[l] >= 1) {  // -J phi_l a_l^+
      const R c = -J * R(sqrt_int<d>(nd[l]));
      const cpx<R> y = Yc[(p - sl) * LD + q];
      const R fr = c * phi[l].re, fi = c * phi[l].im;
      re += fr * y.re - fi * y.im;
      im += fr * y.im + fi * y.re;
    }
  }
  return cmake(re, im);
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

}  // namespace cdtwa
