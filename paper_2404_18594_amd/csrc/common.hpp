// Shared device/host definitions of the C-dTWA library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdtwa {

constexpr int kMaxD = 4;        // local dimension d
constexpr int kMaxGen = 15;     // d*d - 1
constexpr int kMaxLoc = 4;      // sites per cluster
constexpr int kNObs = 15;       // per-trajectory observables

template <typename R>
struct cpx {
  R re, im;
};

template <typename R>
__host__ __device__ inline cpx<R> cmake(R re, R im) {
  cpx<R> c;
  c.re = re;
  c.im = im;
  return c;
}

// Constant tables of one plan, passed to kernels by value.
struct Geom {
  int Lx, Ly, cx, cy, d, periodic;
  int Ns, ncx, ncy, nc, nloc, D, n_gen;
  int model;                 // 0 Bose-Hubbard, 1 transverse-field Ising (d = 2)
  int init_state;            // 1: two onsite states on the (x+y) sublattices
  int layout;                // storage of rho: 0 full D x D, 1 packed upper 16x16 tiles (D = 256)
  double J, U, h;
  double gdeph, gloss;       // local Lindblad rates (L = n_j, L = a_j), model 0
  int64_t n_traj;
  const int* cluster_site;   // [nc][nloc]      global site of (cluster, local)
  const int* ext_nbr;        // [Ns][4]         neighbour in another cluster (+x,-x,+y,-y), -1 if none
  const int* site_cluster;   // [Ns]
  const int* site_local;     // [Ns]
  const double* gen;         // [n_gen][d][d][2] generator matrices T_a
  // sampling tables of every onsite-state class c (site_class), generator a
  // at index c * n_gen + a
  const int* n_out;          // [n_class][n_gen]         distinct outcomes of T_a
  const double* val;         // [n_class][n_gen][kMaxD]  outcome values (ascending)
  const uint64_t* thr;       // [n_class][n_gen][kMaxD]  cumulative thresholds * 2^32
  double g_norm;             // Tr(T_a^2)
};

// onsite-state class of site j: 0 everywhere, or (x + y) mod 2 for a state
// with two sublattices (the Neel start of the Ising chain, App. A)
__host__ __device__ inline int site_class(const Geom& g, int j) {
  return g.init_state == 1 ? ((j % g.Lx) + (j / g.Lx)) & 1 : 0;
}

// Philox-4x32-10 block function (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64-bit
// multiplies with the Weyl-sequence key schedule.
__device__ inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                     uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// Digit of local site l in the Kronecker index p of a cluster with nloc
// sites of dimension d (local 0 most significant).
template <int d, int NLOC>
__host__ __device__ constexpr int kron_stride(int l) {
  int s = 1;
  for (int i = l + 1; i < NLOC; ++i) s *= d;
  return s;
}

template <int d, int NLOC>
__host__ __device__ constexpr int cluster_dim() {
  int D = 1;
  for (int i = 0; i < NLOC; ++i) D *= d;
  return D;
}

template <int d, int NLOC>
__device__ inline int digit(int p, int l) {
  return (p / kron_stride<d, NLOC>(l)) % d;
}

}  // namespace cdtwa
