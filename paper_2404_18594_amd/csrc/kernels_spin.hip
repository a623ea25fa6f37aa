// Transverse-field Ising chain/lattice (App. A Eq. (Hising)) on the C-dTWA
// hot path: spin-1/2 sites (d = 2), clusters of 1, 2 or 4 sites (D <= 16).
//
// The cluster Hamiltonian is J sum_{intra bonds} s^z_l s^z_m + h sum_l s^x_l
// plus, for every bond to a site k of another cluster, J s^z_l Re(b_k) with
// b_k = Tr(s^z_k rho_nu) (Sec. II Eq. (cluster_mf): the neighbour replaced by
// its cluster mean field).  In the product basis (|0> = |up>, local site 0
// the most significant bit) s^z is diagonal and s^x flips one bit, so
//   (H Y - Y H)[p][q] = (E_p - E_q) Y[p][q] + h sum_l (Y[p ^ bit_l][q] - Y[p][q ^ bit_l])
// with E_p the diagonal energy of basis state p; the stage kernel evaluates
// this directly, one matrix entry per thread, without forming H Y.
// Stage scheme, field buffers and RK4 update are those of the per-stage path
// (App. B.1, classical RK4 with the fields recomputed at every stage).
#include "launch.hpp"
#include "pairs.hpp"
#include "structured.hpp"

namespace cdtwa {

namespace {

template <int NLOC>
__device__ inline int spin_bit(int l) {
  return 1 << (NLOC - 1 - l);
}
template <int NLOC, typename R>
__device__ inline R spin_z(int p, int l) {
  return (p & spin_bit<NLOC>(l)) ? R(-1) : R(1);
}

// b_j = Tr(s^z_j rho_C) = sum_p z_l(p) rho[p][p], one thread per (trajectory, site)
template <typename R, int NLOC>
__global__ void __launch_bounds__(256) k_spin_fields(Geom g, const cpx<R>* __restrict__ rho, cpx<R>* __restrict__ b) {
  constexpr int D = 1 << NLOC;
  const int64_t flat = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (flat >= g.n_traj * g.Ns) return;
  const int64_t t = flat / g.Ns;
  const int j = (int)(flat % g.Ns);
  const int mu = g.site_cluster[j], l = g.site_local[j];
  const cpx<R>* Y = rho + (t * g.nc + mu) * D * D;
  R re = 0, im = 0;
#pragma unroll
  for (int p = 0; p < D; ++p) {
    const cpx<R> y = Y[p * D + p];
    const R z = spin_z<NLOC, R>(p, l);
    re = fma_r(z, y.re, re);
    im = fma_r(z, y.im, im);
  }
  b[flat] = cmake(re, im);
}

// One RK4 stage (modes 1..4) or the bare commutator (mode 0) for CPB
// clusters per workgroup; modes as in StageArgs.
template <typename R, int CX, int CY, int CPB, int NT>
__global__ void __launch_bounds__(NT) k_spin_stage(StageArgs<R> a) {
  constexpr int NLOC = CX * CY;
  constexpr int D = 1 << NLOC;
  constexpr int DD = D * D;
  constexpr int NE = CPB * DD;
  constexpr int EPT = (NE + NT - 1) / NT;
  __shared__ cpx<R> sY[NE];
  __shared__ R sE[CPB * D];
  __shared__ R sF[CPB * NLOC];
  const Geom& g = a.g;
  const int64_t first = (int64_t)blockIdx.x * CPB;
  const int64_t total = g.n_traj * g.nc;
  const int nvalid = total - first < CPB ? (int)(total - first) : CPB;
  const R J = R(g.J), h = R(g.h);
  const int mode = a.mode;
  const R cin = mode == 4 ? a.dt : R(0.5) * a.dt;
  const R cout = mode == 3 ? a.dt : R(0.5) * a.dt;

  cpx<R> rv[EPT], kp[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e >= nvalid * DD) continue;
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
  // field on each boundary site: J times the sum of Re b_k over its
  // neighbours in other clusters
  for (int i = threadIdx.x; i < nvalid * NLOC; i += NT) {
    const int gi = i / NLOC, l = i % NLOC;
    const int64_t flat = first + gi;
    const int64_t t = flat / g.nc;
    const int mu = (int)(flat % g.nc);
    const int j = g.cluster_site[mu * NLOC + l];
    R f = 0;
    for (int k = 0; k < 4; ++k) {
      const int n = g.ext_nbr[j * 4 + k];
      if (n >= 0) f += a.b_in[t * g.Ns + n].re;
    }
    sF[i] = J * f;
  }
  __syncthreads();
  // diagonal energy of every basis state
  for (int i = threadIdx.x; i < nvalid * D; i += NT) {
    const int gi = i / D, p = i % D;
    R e = 0;
#pragma unroll
    for (int b = 0; b < Bonds<CX, CY>::n; ++b)
      e = fma_r(J, spin_z<NLOC, R>(p, Bonds<CX, CY>::l(b)) * spin_z<NLOC, R>(p, Bonds<CX, CY>::m(b)), e);
#pragma unroll
    for (int l = 0; l < NLOC; ++l) e = fma_r(sF[gi * NLOC + l], spin_z<NLOC, R>(p, l), e);
    sE[i] = e;
  }
  __syncthreads();
  // K = -i [H, Y]:  K.re = Im X,  K.im = -Re X  with X = (H Y - Y H)[p][q]
  cpx<R> yn[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e >= nvalid * DD) continue;
    const int gi = e / DD, pq = e % DD, p = pq / D, q = pq % D;
    const cpx<R>* Y = sY + gi * DD;
    const R de = sE[gi * D + p] - sE[gi * D + q];
    const cpx<R> y0 = Y[pq];
    R sr = 0, si = 0;
#pragma unroll
    for (int l = 0; l < NLOC; ++l) {
      const cpx<R> u = Y[(p ^ spin_bit<NLOC>(l)) * D + q], v = Y[p * D + (q ^ spin_bit<NLOC>(l))];
      sr += u.re - v.re;
      si += u.im - v.im;
    }
    const R xr = fma_r(de, y0.re, h * sr), xi = fma_r(de, y0.im, h * si);
    const cpx<R> kk = cmake(xi, -xr);
    const int64_t gidx = first * DD + e;
    if (mode <= 3) {
      a.kout[gidx] = kk;
      yn[i] = cmake(fma_r(cout, kk.re, rv[i].re), fma_r(cout, kk.im, rv[i].im));
    } else {
      const cpx<R> q1 = a.k1[gidx], q2 = a.k2[gidx];
      const R h6 = a.dt / R(6);
      const R tr = fma_r(R(2), kp[i].re, fma_r(R(2), q2.re, q1.re)) + kk.re;
      const R ti = fma_r(R(2), kp[i].im, fma_r(R(2), q2.im, q1.im)) + kk.im;
      yn[i] = cmake(fma_r(h6, tr, rv[i].re), fma_r(h6, ti, rv[i].im));
      a.rho[gidx] = yn[i];
    }
  }
  if (mode == 0) return;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * NT;
    if (e < nvalid * DD) sY[e] = yn[i];
  }
  __syncthreads();
  // mean fields of Y_{s+1}
  for (int i = threadIdx.x; i < nvalid * NLOC; i += NT) {
    const int gi = i / NLOC, l = i % NLOC;
    const int64_t flat = first + gi;
    const int64_t t = flat / g.nc;
    const int mu = (int)(flat % g.nc);
    R re = 0, im = 0;
#pragma unroll
    for (int p = 0; p < D; ++p) {
      const cpx<R> y = sY[gi * DD + p * D + p];
      const R z = spin_z<NLOC, R>(p, l);
      re = fma_r(z, y.re, re);
      im = fma_r(z, y.im, im);
    }
    a.b_out[t * g.Ns + g.cluster_site[mu * NLOC + l]] = cmake(re, im);
  }
}

// ---------------------------------------------------------------------------
// Observables (FP64).  Cluster record: [0,n) <s^z_l>, [n,2n) <s^x_l>,
// [2n,3n) <s^y_l>, [3n, 3n+n^2) <s^z_l s^z_m>, then Re Tr, Tr rho^2, max
// Hermiticity deviation, Tr(Gamma^intra rho), Im Tr.  One thread per cluster.
// ---------------------------------------------------------------------------
template <int NLOC>
__host__ __device__ constexpr int spin_rec() {
  return 3 * NLOC + NLOC * NLOC + 5;
}

template <typename R, int CX, int CY>
__global__ void __launch_bounds__(256) k_spin_obs_cluster(Geom g, const cpx<R>* __restrict__ rho,
                                                          double* __restrict__ rec) {
  constexpr int NLOC = CX * CY;
  constexpr int D = 1 << NLOC;
  constexpr int NR = spin_rec<NLOC>();
  const int64_t flat = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (flat >= g.n_traj * g.nc) return;
  const cpx<R>* Y = rho + flat * D * D;
  double acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0;
  double hmax = 0, eint = 0;
  for (int p = 0; p < D; ++p) {
    const double ypp = (double)Y[p * D + p].re;
    acc[3 * NLOC + NLOC * NLOC] += ypp;
    acc[3 * NLOC + NLOC * NLOC + 4] += (double)Y[p * D + p].im;
    double ebond = 0;
#pragma unroll
    for (int b = 0; b < Bonds<CX, CY>::n; ++b)
      ebond += spin_z<NLOC, double>(p, Bonds<CX, CY>::l(b)) * spin_z<NLOC, double>(p, Bonds<CX, CY>::m(b));
    eint += g.J * ebond * ypp;
#pragma unroll
    for (int l = 0; l < NLOC; ++l) {
      const double zl = spin_z<NLOC, double>(p, l);
      acc[l] += zl * ypp;
      const cpx<R> f = Y[(p ^ spin_bit<NLOC>(l)) * D + p];
      acc[NLOC + l] += (double)f.re;
      acc[2 * NLOC + l] += (p & spin_bit<NLOC>(l)) ? -(double)f.im : (double)f.im;
#pragma unroll
      for (int m = 0; m < NLOC; ++m) acc[3 * NLOC + l * NLOC + m] += zl * spin_z<NLOC, double>(p, m) * ypp;
    }
    for (int q = 0; q < D; ++q) {
      const cpx<R> u = Y[p * D + q], v = Y[q * D + p];
      acc[3 * NLOC + NLOC * NLOC + 1] += (double)u.re * v.re - (double)u.im * v.im;
      const double dr = (double)u.re - (double)v.re, di = (double)u.im + (double)v.im;
      hmax = fmax(hmax, sqrt(dr * dr + di * di));
    }
  }
  double sx = 0;
#pragma unroll
  for (int l = 0; l < NLOC; ++l) sx += acc[NLOC + l];
  acc[3 * NLOC + NLOC * NLOC + 2] = hmax;
  acc[3 * NLOC + NLOC * NLOC + 3] = eint + g.h * sx;
#pragma unroll
  for (int k = 0; k < NR; ++k) rec[flat * NR + k] = acc[k];
}

// per-trajectory observables from the cluster records, one block per trajectory
template <int NLOC>
__global__ void __launch_bounds__(256) k_spin_obs_traj(Geom g, const double* __restrict__ rec, double* __restrict__ out) {
  constexpr int NR = spin_rec<NLOC>();
  constexpr int NA = 10;   // staggered, z, x, y, zz classes 0..4, inter-cluster bond energy
  const int64_t t = blockIdx.x;
  const double* R0 = rec + t * g.nc * NR;
  __shared__ double part[256][NA];
  double acc[NA];
  for (int k = 0; k < NA; ++k) acc[k] = 0;
  for (int i = threadIdx.x; i < g.Ns; i += 256) {
    const int mi = g.site_cluster[i], li = g.site_local[i];
    const double zi = R0[mi * NR + li];
    acc[0] += (((i % g.Lx) + (i / g.Lx)) & 1) ? -zi : zi;
    acc[1] += zi;
    acc[2] += R0[mi * NR + NLOC + li];
    acc[3] += R0[mi * NR + 2 * NLOC + li];
    for_each_class_pair(g, i, [&](int j, int cls) {
      const int mj = g.site_cluster[j], lj = g.site_local[j];
      acc[4 + cls] += mi == mj ? R0[mi * NR + 3 * NLOC + li * NLOC + lj] : zi * R0[mj * NR + lj];
    });
    for (int k = 0; k < 4; k += 2) {   // +x and +y neighbours in other clusters: each bond once
      const int j = g.ext_nbr[i * 4 + k];
      if (j >= 0) acc[9] += g.J * zi * R0[g.site_cluster[j] * NR + g.site_local[j]];
    }
  }
  for (int k = 0; k < NA; ++k) part[threadIdx.x][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < NA) {
    double s = 0;
    for (int u = 0; u < 256; ++u) s += part[u][threadIdx.x];
    part[0][threadIdx.x] = s;   // only thread k touches column k
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = out + t * kNObs;
    const double inv = 1.0 / g.Ns;
    for (int k = 0; k < 4; ++k) o[k] = part[0][k] * inv;
    o[4] = 0;
    for (int c = 0; c < 5; ++c) o[5 + c] = part[0][4 + c] * inv;
    o[10] = 0;
    double e = part[0][9], pur = 0, trd = 0, hd = 0;
    const int base = 3 * NLOC + NLOC * NLOC;
    for (int mu = 0; mu < g.nc; ++mu) {
      e += R0[mu * NR + base + 3];
      pur += R0[mu * NR + base + 1];
      trd = fmax(trd, hypot(R0[mu * NR + base] - 1.0, R0[mu * NR + base + 4]));   // |Tr - 1|, complex
      hd = fmax(hd, R0[mu * NR + base + 2]);
    }
    o[11] = e * inv;
    o[12] = pur / g.nc;
    o[13] = trd;
    o[14] = hd;
  }
}

template <typename R, int CX, int CY>
struct Spin {
  static constexpr int NLOC = CX * CY;
  static constexpr int D = 1 << NLOC;
  static constexpr int NT = 256;
  static constexpr int CPB = 2048 / (D * D);

  static hipError_t fields(const Geom& g, const void* rho, void* b, hipStream_t s) {
    const int64_t n = g.n_traj * g.Ns;
    hipLaunchKernelGGL((k_spin_fields<R, NLOC>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                       (const cpx<R>*)rho, (cpx<R>*)b);
    return hipGetLastError();
  }
  static hipError_t stage(const Geom& g, void* rho, const void* kprev, const void* k1, const void* k2, void* kout,
                          const void* b_in, void* b_out, double dt, int mode, hipStream_t s) {
    const StageArgs<R> a{g, (cpx<R>*)rho, (const cpx<R>*)kprev, (const cpx<R>*)k1, (const cpx<R>*)k2, (cpx<R>*)kout,
                         (const cpx<R>*)b_in, (cpx<R>*)b_out, (R)dt, mode};
    const int64_t total = g.n_traj * g.nc;
    hipLaunchKernelGGL((k_spin_stage<R, CX, CY, CPB, NT>), dim3((unsigned)((total + CPB - 1) / CPB)), dim3(NT), 0, s,
                       a);
    return hipGetLastError();
  }
  static hipError_t observables(const Geom& g, const void* rho, double* rec, double* per_traj, hipStream_t s) {
    static_assert(spin_rec<NLOC>() <= cluster_rec<NLOC>(), "record fits the observable workspace");
    const int64_t n = g.n_traj * g.nc;
    hipLaunchKernelGGL((k_spin_obs_cluster<R, CX, CY>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                       (const cpx<R>*)rho, rec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_spin_obs_traj<NLOC>), dim3((unsigned)g.n_traj), dim3(256), 0, s, g, (const double*)rec,
                       per_traj);
    return hipGetLastError();
  }
};

template <typename F>
hipError_t spin_dispatch(const Geom& g, int dtype, F&& f) {
  if (g.model != 1 || g.d != 2) return hipErrorInvalidValue;
#define CDTWA_SPIN(RT)                                          \
  if (g.cx == 1 && g.cy == 1) return f(Spin<RT, 1, 1>());       \
  if (g.cx == 2 && g.cy == 1) return f(Spin<RT, 2, 1>());       \
  if (g.cx == 1 && g.cy == 2) return f(Spin<RT, 1, 2>());       \
  if (g.cx == 2 && g.cy == 2) return f(Spin<RT, 2, 2>());
  if (dtype == 1) {
    CDTWA_SPIN(double)
  } else {
    CDTWA_SPIN(float)
  }
#undef CDTWA_SPIN
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t spin_site_fields(const Geom& g, int dtype, const void* rho, void* b, hipStream_t s) {
  return spin_dispatch(g, dtype, [&](auto k) { return decltype(k)::fields(g, rho, b, s); });
}

hipError_t spin_stage(const Geom& g, int dtype, void* rho, const void* kprev, const void* k1, const void* k2,
                      void* kout, const void* b_in, void* b_out, double dt, int mode, hipStream_t s) {
  return spin_dispatch(g, dtype, [&](auto k) {
    return decltype(k)::stage(g, rho, kprev, k1, k2, kout, b_in, b_out, dt, mode, s);
  });
}

hipError_t spin_observables(const Geom& g, int dtype, const void* rho, double* rec, double* per_traj, hipStream_t s) {
  return spin_dispatch(g, dtype, [&](auto k) { return decltype(k)::observables(g, rho, rec, per_traj, s); });
}

}  // namespace cdtwa
