// Generic HIP kernels of the C-dTWA hot path for every cluster shape:
// discrete sampling, cluster mean fields and the per-trajectory observables
// for every D, and one Runge-Kutta stage of the cluster mean-field equation
// for cluster matrices that fit in LDS (D <= 81; larger ones in
// kernels_big.hip).  One workgroup holds CPB cluster matrices; a
// stage streams the state through HBM once per stage.
#include <algorithm>

#include "launch.hpp"
#include "pairs.hpp"
#include "structured.hpp"

namespace cdtwa {

// ---------------------------------------------------------------------------
// a1: sampling.  One workgroup per group of CPB clusters of one trajectory.
// ---------------------------------------------------------------------------
template <typename R, int d, int CX, int CY, int CPB, int NT>
__global__ void __launch_bounds__(NT) k_sample(Geom g, uint64_t seed, int64_t traj_offset, int8_t* __restrict__ noise,
                                               cpx<R>* __restrict__ rho) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  constexpr int NG = d * d - 1;
  __shared__ double s_r[CPB][NLOC][NG];
  __shared__ double s_A[CPB][NLOC][d * d][2];
  const int64_t first = (int64_t)blockIdx.x * CPB;  // flat (traj, cluster) index
  const int64_t total = g.n_traj * g.nc;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int i = threadIdx.x; i < CPB * NLOC * NG; i += NT) {
    const int gi = i / (NLOC * NG), l = (i / NG) % NLOC, a = i % NG;
    const int64_t flat = first + gi;
    if (flat >= total) continue;
    const int64_t t = flat / g.nc;
    const int mu = (int)(flat % g.nc);
    const int j = g.cluster_site[mu * NLOC + l];
    const uint64_t tg = (uint64_t)(traj_offset + t);
    uint32_t w[4];
    philox4x32_10((uint32_t)(a / 4), (uint32_t)j, (uint32_t)tg, (uint32_t)(tg >> 32), k0, k1, w);
    const uint32_t x = w[a % 4];
    const int ca = site_class(g, j) * NG + a;
    int n = 0;
    while (n < g.n_out[ca] - 1 && !((uint64_t)x < g.thr[ca * kMaxD + n])) ++n;
    if (noise) noise[(t * g.Ns + j) * NG + a] = (int8_t)n;
    s_r[gi][l][a] = g.val[ca * kMaxD + n];
  }
  __syncthreads();
  // A_j = I/d + (1/g) sum_a r^a T_a
  for (int i = threadIdx.x; i < CPB * NLOC * d * d; i += NT) {
    const int gi = i / (NLOC * d * d), l = (i / (d * d)) % NLOC, e = i % (d * d);
    double re = (e / d == e % d) ? 1.0 / d : 0.0, im = 0.0;
    for (int a = 0; a < NG; ++a) {
      const double c = s_r[gi][l][a] / g.g_norm;
      re += c * g.gen[(a * d * d + e) * 2];
      im += c * g.gen[(a * d * d + e) * 2 + 1];
    }
    s_A[gi][l][e][0] = re;
    s_A[gi][l][e][1] = im;
  }
  __syncthreads();
  // rho[p][q] = prod_l A_l[n_l(p)][n_l(q)]
  for (int i = threadIdx.x; i < CPB * D * D; i += NT) {
    const int gi = i / (D * D), pq = i % (D * D), p = pq / D, q = pq % D;
    const int64_t flat = first + gi;
    if (flat >= total) continue;
    double re = 1.0, im = 0.0;
#pragma unroll
    for (int l = 0; l < NLOC; ++l) {
      const int e = digit<d, NLOC>(p, l) * d + digit<d, NLOC>(q, l);
      const double ar = s_A[gi][l][e][0], ai = s_A[gi][l][e][1];
      const double nr = re * ar - im * ai, ni = re * ai + im * ar;
      re = nr;
      im = ni;
    }
    if (g.layout == 1) {
      // packed upper 16 x 16 tiles (D = 256): entries of the lower tiles are
      // not stored
      const int I = p / 16, Jt = q / 16;
      if (I > Jt) continue;
      const int64_t at = (int64_t)(I * 16 - I * (I - 1) / 2 + (Jt - I)) * 256 + (p % 16) * 16 + q % 16;
      rho[flat * (int64_t)(136 * 256) + at] = cmake(R(re), R(im));
    } else {
      rho[flat * D * D + pq] = cmake(R(re), R(im));
    }
  }
}

// ---------------------------------------------------------------------------
// a2: cluster mean fields b_j = Tr(a_j rho_C) = sum_q sqrt(n_l(q)+1) rho[q+s_l][q]
// ---------------------------------------------------------------------------
template <typename R, int d, int CX, int CY>
__global__ void __launch_bounds__(64) k_site_fields(Geom g, const cpx<R>* __restrict__ rho, cpx<R>* __restrict__ b) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  const int64_t flat = (int64_t)blockIdx.x * 64 + threadIdx.x;  // (traj, site)
  if (flat >= g.n_traj * g.Ns) return;
  const int64_t t = flat / g.Ns;
  const int j = (int)(flat % g.Ns);
  const int mu = g.site_cluster[j], l = g.site_local[j];
  const cpx<R>* Y = rho + (t * g.nc + mu) * D * D;
  const int sl = kron_stride<d, NLOC>(l);
  R re = 0, im = 0;
  for (int q = 0; q < D; ++q) {
    const int n = digit<d, NLOC>(q, l);
    if (n > d - 2) continue;
    const R c = R(sqrt_int<d>(n + 1));
    const cpx<R> y = Y[(q + sl) * D + q];
    re += c * y.re;
    im += c * y.im;
  }
  b[flat] = cmake(re, im);
}

// phi_j = sum of b_k over neighbours k of j in other clusters (+x,-x,+y,-y order)
template <typename R>
__global__ void __launch_bounds__(256) k_boundary_fields(Geom g, const cpx<R>* __restrict__ b, cpx<R>* __restrict__ phi) {
  const int64_t flat = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (flat >= g.n_traj * g.Ns) return;
  const int64_t t = flat / g.Ns;
  const int j = (int)(flat % g.Ns);
  R re = 0, im = 0;
  for (int k = 0; k < 4; ++k) {
    const int n = g.ext_nbr[j * 4 + k];
    if (n < 0) continue;
    const cpx<R> v = b[t * g.Ns + n];
    re += v.re;
    im += v.im;
  }
  phi[flat] = cmake(re, im);
}

// ---------------------------------------------------------------------------
// a3 + a4: one classical RK4 stage (mode 1..4) or the bare commutator (mode 0)
// for CPB clusters per workgroup.
//   mode 0: Y = rho,              K written to kout
//   mode 1: Y = rho,              K1 -> kout, b(rho + dt/2 K1) -> b_out
//   mode 2: Y = rho + dt/2 K1,    K2 -> kout, b(rho + dt/2 K2) -> b_out
//   mode 3: Y = rho + dt/2 K2,    K3 -> kout, b(rho + dt K3)   -> b_out
//   mode 4: Y = rho + dt K3,      rho += dt/6 (K1 + 2K2 + 2K3 + K4), b(rho) -> b_out
// b_in holds the mean fields of Y for every site of every trajectory.
// ---------------------------------------------------------------------------

template <typename R, int d, int CX, int CY, int CPB, int NT, bool DISS>
__global__ void __launch_bounds__(NT) k_stage(StageArgs<R> a) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  __shared__ cpx<R> sY[CPB * D * D];
  __shared__ cpx<R> sPhi[CPB * NLOC];
  stage_body<R, d, CX, CY, CPB, NT, DISS>(a, (int64_t)blockIdx.x * CPB, sY, sPhi);
}

// ---------------------------------------------------------------------------
// a5: observables.  Per cluster (FP64 from the state precision), then per
// trajectory, then the ordered FP64 Neumaier sums over trajectories.
// Cluster record layout: cluster_rec (launch.hpp).
// ---------------------------------------------------------------------------

// NW waves per cluster, which split its rows (band quantities) and its 8x8
// block pairs (purity, Hermiticity) between them; the partial results of the
// waves are combined in wave order, so every sum has a fixed order.
//
// Band quantities (b_l, Tr(a_l^+ a_m rho), the diagonal ones): each lane owns
// one quantity, which fixes the offset delta = row - column of the entries it
// sums; a wave walks its rows together, so one load instruction reads
// entries of a single row (a few cache lines) instead of one line per lane.
// Lane roles, in order: b_l (re, im) for every site; G[l][m] = sum_p
// sqrt(n_l) sqrt(n_m + 1) Re rho[p - s_l + s_m][p] for l != m; n_l; NN[l][m]
// for l != m; Re Tr rho; the diagonal energy U sum_l n_l (n_l - 1) / 2;
// Im Tr rho (the trace deviation |Tr rho - 1| is taken as a complex modulus).
// The intra-cluster hopping energy is -J sum over bonds of G[l][m] + G[m][l].
template <int D>
constexpr int obs_waves() {
  return D >= 27 ? 4 : 1;
}

// The band quantity of a lane: kind, sites L and M, offset delta = row -
// column of the entries it sums, and its record slot; weight(c) is the weight
// of entry (c + delta, c) (zero where the quantity has no term).
template <int d, int NLOC>
struct BandRole {
  static constexpr int QB = 2 * NLOC, QG = NLOC * (NLOC - 1);
  static constexpr int Q = QB + QG + NLOC + QG + 3;
  static_assert(Q <= 64, "one lane per band quantity");
  int kind = -1, L = 0, M = 0, delta = 0, slot = 0;
  bool take_im = false;
  static __device__ int stride(int l) {
    int s = 1;
    for (int k = NLOC - 1; k > l; --k) s *= d;
    return s;
  }
  static __device__ void pair_of(int idx, int& l, int& m) {   // idx-th ordered pair l != m
    constexpr int den = NLOC > 1 ? NLOC - 1 : 1;
    l = idx / den;
    const int mm = idx % den;
    m = mm < l ? mm : mm + 1;
  }
  __device__ explicit BandRole(int lane) {
    constexpr int base = 3 * NLOC + 2 * NLOC * NLOC;
    if (lane < QB) {
      kind = 0;
      L = lane >> 1;
      delta = stride(L);
      slot = lane;
    } else if (lane < QB + QG) {
      kind = 1;
      pair_of(lane - QB, L, M);
      delta = stride(M) - stride(L);
      slot = 3 * NLOC + L * NLOC + M;
    } else if (lane < QB + QG + NLOC) {
      kind = 2;
      L = lane - QB - QG;
      slot = 2 * NLOC + L;
    } else if (lane < QB + 2 * QG + NLOC) {
      kind = 3;
      pair_of(lane - QB - QG - NLOC, L, M);
      slot = 3 * NLOC + NLOC * NLOC + L * NLOC + M;
    } else if (lane == Q - 3) {
      kind = 4;   // Re Tr
      slot = base;
    } else if (lane == Q - 2) {
      kind = 5;   // diagonal energy
      slot = base + 3;
    } else if (lane == Q - 1) {
      kind = 6;   // Im Tr
      slot = base + 4;
    }
    take_im = (kind == 0 && (lane & 1)) || kind == 6;
  }
  __device__ double weight(int c, double hU) const {
    int nd[NLOC];
#pragma unroll
    for (int l = 0; l < NLOC; ++l) nd[l] = digit<d, NLOC>(c, l);
    int nl = nd[0], nm = nd[0], h = nd[0] * (nd[0] - 1);
#pragma unroll
    for (int l = 1; l < NLOC; ++l) {
      nl = L == l ? nd[l] : nl;
      nm = M == l ? nd[l] : nm;
      h += nd[l] * (nd[l] - 1);
    }
    if (kind == 0) return nl <= d - 2 ? sqrt_int<d>(nl + 1) : 0.0;
    if (kind == 1) return (nl >= 1 && nm <= d - 2) ? sqrt_int<d>(nl) * sqrt_int<d>(nm + 1) : 0.0;
    if (kind == 2) return nl;
    if (kind == 3) return nl * nm;
    if (kind == 4 || kind == 6) return 1.0;
    return hU * h;
  }
};

// The record of one cluster from the per-wave partial results part[w] (band
// sum of every lane, purity, Hermiticity), combined in wave order: the band
// values, Tr rho^2, the Hermiticity deviation and the energy, then written to
// rec.  Called by every thread of the block.
template <int CX, int CY, int NW>
__device__ inline void obs_finish(const Geom& g, int kind, int slot, const double (*part)[64 + 2], double* vals,
                                  double* rec_out) {
  constexpr int NLOC = CX * CY;
  constexpr int NR = cluster_rec<NLOC>();
  constexpr int base = 3 * NLOC + 2 * NLOC * NLOC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  lds_barrier();
  if (wave == 0) {
    double bs = 0, ps = 0, hm = 0;
    for (int w = 0; w < NW; ++w) {
      bs += part[w][lane];
      ps += part[w][64];
      hm = fmax(hm, part[w][65]);
    }
    if (kind >= 0) vals[slot] = bs;
    if (lane == 0) {
      vals[base + 1] = ps;
      vals[base + 2] = hm;
    }
  }
  lds_barrier();
  if (threadIdx.x == 0) {
    double e = 0;
#pragma unroll
    for (int b = 0; b < Bonds<CX, CY>::n; ++b) {
      const int l = Bonds<CX, CY>::l(b), m = Bonds<CX, CY>::m(b);
      e += vals[3 * NLOC + l * NLOC + m] + vals[3 * NLOC + m * NLOC + l];
    }
    vals[base + 3] -= g.J * e;
  }
  lds_barrier();
  for (int k = threadIdx.x; k < NR; k += 64 * NW) rec_out[k] = vals[k];
}

template <typename R, int d, int CX, int CY, int NW = obs_waves<cluster_dim<d, CX * CY>()>()>
__global__ void __launch_bounds__(64 * NW) k_obs_cluster(Geom g, const cpx<R>* __restrict__ rho, double* __restrict__ rec) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  constexpr int NR = cluster_rec<NLOC>();
  constexpr int NB = (D + 7) / 8;   // 8x8 blocks per side
  const int64_t flat = blockIdx.x;  // (traj, cluster)
  const cpx<R>* Y = rho + flat * D * D;
  __shared__ double vals[NR];
  __shared__ double part[NW][64 + 2];   // per wave: band sum of each lane, purity, Hermiticity
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < NR; k += 64 * NW) vals[k] = 0;

  const BandRole<d, NLOC> role(lane);
  const double hU = 0.5 * g.U;
  double band = 0;
#pragma unroll 8
  for (int r = wave; r < D; r += NW) {
    const int c = r - role.delta;
    if (role.kind >= 0 && c >= 0 && c < D) {
      const cpx<R> v = Y[r * D + c];
      band += role.weight(c, hU) * (double)(role.take_im ? v.im : v.re);
    }
  }
  // Tr rho^2 = sum Re(Y_pq Y_qp) and max |Y_pq - conj(Y_qp)| over 8x8 block
  // pairs (I, J), I <= J: lane (i, j) reads Y[8I+i][8J+j] and Y[8J+j][8I+i],
  // both 8 rows of 8 consecutive entries, so every cache line is used while
  // it is loaded; an off-diagonal pair stands for both of its blocks
  double pur = 0, hmax = 0;
  {
    // block pairs t = wave, wave + NW, ... in row-major order over I <= J
    const int i = lane >> 3, j = lane & 7;
    int I = 0, Jb = 0;
    for (int k = 0; k < wave; ++k)
      if (++Jb == NB) {
        ++I;
        Jb = I;
      }
#pragma unroll 4
    for (int t = wave; t < NB * (NB + 1) / 2; t += NW) {
      const int p = 8 * I + i, q = 8 * Jb + j;
      if (p < D && q < D) {
        const cpx<R> a = Y[p * D + q], b = Y[q * D + p];
        const double w = I == Jb ? 1.0 : 2.0;
        pur += w * ((double)a.re * b.re - (double)a.im * b.im);
        const double dr = (double)a.re - (double)b.re, di = (double)a.im + (double)b.im;
        hmax = fmax(hmax, sqrt(dr * dr + di * di));
      }
      for (int k = 0; k < NW; ++k)
        if (++Jb == NB) {
          ++I;
          Jb = I;
        }
    }
  }
  // purity and Hermiticity over the wave (butterfly: the same order on every
  // lane)
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    pur += __shfl_xor(pur, o);
    hmax = fmax(hmax, __shfl_xor(hmax, o));
  }
  part[wave][lane] = band;
  if (lane == 0) {
    part[wave][64] = pur;
    part[wave][65] = hmax;
  }
  obs_finish<CX, CY, NW>(g, role.kind, role.slot, part, vals, rec + flat * NR);
}

// Workgroups of a persistent kernel that fits per_cu of them on a CU: that
// many on every CU of the current device (256 CUs if the count cannot be read).
static int obs_lds_slots(int per_cu) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  return cus * per_cu;
}

// D = 81 (2x2 clusters, d = 3): each cluster matrix is staged through LDS
// once (105 KB in FP64, 52 KB in FP32) with coalesced loads, and the band
// quantities, Tr rho^2 and the Hermiticity deviation read it from there.  The
// kernel above reads the matrix twice from global memory (by rows for the
// band quantities, by 8x8 block pairs for the rest), and at this size the
// second read misses the caches.  Only one (FP64) or two (FP32) such
// workgroups fit on a CU, so the kernel is persistent: a workgroup walks the
// clusters blockIdx.x, blockIdx.x + gridDim.x, ... and loads the next one
// into registers while it works on the current one from LDS.  The lane
// weights of the band quantities are formed once per workgroup.
template <typename R, int d, int CX, int CY>
__global__ void __launch_bounds__(512, sizeof(R) == 4 ? 4 : 2) k_obs_cluster_lds(Geom g, const cpx<R>* __restrict__ rho,
                                                         double* __restrict__ rec, int64_t total) {
  constexpr int NW = 8, NT = 64 * NW;
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  constexpr int E = D * D;
  constexpr int PER = (E + NT - 1) / NT;   // entries per thread
  constexpr int NRW = (D + NW - 1) / NW;   // band rows per wave
  constexpr int NR = cluster_rec<NLOC>();
  __shared__ cpx<R> sY[E];
  __shared__ double vals[NR];
  __shared__ double part[NW][64 + 2];   // per wave: band sum of each lane, purity, Hermiticity
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const BandRole<d, NLOC> role(lane);
  // weights of this lane's band entries, rows r = wave + NW k (0 where the
  // row has no entry of the quantity)
  double wr[NRW];
  int cr[NRW];
  {
    const double hU = 0.5 * g.U;
#pragma unroll
    for (int k = 0; k < NRW; ++k) {
      const int r = wave + NW * k, c = r - role.delta;
      const bool ok = role.kind >= 0 && r < D && c >= 0 && c < D;
      cr[k] = ok ? r * D + c : -1;
      wr[k] = ok ? role.weight(c, hU) : 0.0;
    }
  }
  // (p, q) of entry e = tid + k NT, and the position of (q, p)
  int et[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + k * NT, p = e / D, q = e - p * D;
    et[k] = q * D + p;
  }
  // the cluster's entries, loaded one cluster ahead (written out at both
  // load sites: through a lambda the array went to scratch memory)
  cpx<R> own[PER];
  int64_t f = blockIdx.x;
  if (f < total) {
    const cpx<R>* Y = rho + f * E;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * NT;
      own[k] = e < E ? Y[e] : cmake(R(0), R(0));
    }
  }
  for (; f < total; f += gridDim.x) {
    lds_barrier();   // the previous cluster's readers of sY, vals and part are done
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * NT;
      if (e < E) sY[e] = own[k];
    }
    for (int k = tid; k < NR; k += NT) vals[k] = 0;
    lds_barrier();
    if (f + gridDim.x < total) {   // in flight until sY is next written
      const cpx<R>* Y = rho + (f + gridDim.x) * E;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = tid + k * NT;
        own[k] = e < E ? Y[e] : cmake(R(0), R(0));
      }
    }
    double band = 0;
#pragma unroll
    for (int k = 0; k < NRW; ++k) {
      // entries outside the band stay out of the sum (no 0 x value term)
      const cpx<R> v = sY[cr[k] >= 0 ? cr[k] : 0];
      const double t = wr[k] * (double)(role.take_im ? v.im : v.re);
      band = cr[k] >= 0 ? band + t : band;
    }
    // Tr rho^2 = sum over every (p, q) of Re(Y_pq Y_qp); the largest
    // |Y_pq - conj(Y_qp)|^2, its square root taken once at the end
    double pur = 0, h2 = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + k * NT;
      if (e < E) {
        const cpx<R> a = sY[e], b = sY[et[k]];
        pur += (double)a.re * b.re - (double)a.im * b.im;
        const double dr = (double)a.re - (double)b.re, di = (double)a.im + (double)b.im;
        h2 = fmax(h2, dr * dr + di * di);
      }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      pur += __shfl_xor(pur, o);
      h2 = fmax(h2, __shfl_xor(h2, o));
    }
    part[wave][lane] = band;
    if (lane == 0) {
      part[wave][64] = pur;
      part[wave][65] = sqrt(h2);
    }
    obs_finish<CX, CY, NW>(g, role.kind, role.slot, part, vals, rec + f * NR);
  }
}

// per-trajectory observables from the cluster records (one block per trajectory)
template <int NLOC>
__global__ void __launch_bounds__(256) k_obs_traj(Geom g, const double* __restrict__ rec, double* __restrict__ out) {
  constexpr int NR = cluster_rec<NLOC>();
  const int64_t t = blockIdx.x;
  const double* R0 = rec + t * g.nc * NR;
  __shared__ double part[256][12];
  double acc[12];
  for (int k = 0; k < 12; ++k) acc[k] = 0;
  for (int i = threadIdx.x; i < g.Ns; i += 256) {
    const int mi = g.site_cluster[i], li = g.site_local[i];
    const double bir = R0[mi * NR + 2 * li], bii = R0[mi * NR + 2 * li + 1];
    const double ni = R0[mi * NR + 2 * NLOC + li];
    for_each_class_pair(g, i, [&](int j, int cls) {
      const int mj = g.site_cluster[j], lj = g.site_local[j];
      double gij, nij;
      if (mi == mj) {
        gij = R0[mi * NR + 3 * NLOC + li * NLOC + lj];
        nij = R0[mi * NR + 3 * NLOC + NLOC * NLOC + li * NLOC + lj];
      } else {
        const double bjr = R0[mj * NR + 2 * lj], bji = R0[mj * NR + 2 * lj + 1];
        gij = bir * bjr + bii * bji;
        nij = ni * R0[mj * NR + 2 * NLOC + lj];
      }
      acc[cls] += gij;
      acc[5 + cls] += nij;
    });
    acc[10] += ni;
    // inter-cluster bonds, +x and +y neighbours (each bond once)
    for (int k = 0; k < 4; k += 2) {
      const int j = g.ext_nbr[i * 4 + k];
      if (j < 0) continue;
      const int mj = g.site_cluster[j], lj = g.site_local[j];
      acc[11] += -g.J * 2.0 * (bir * R0[mj * NR + 2 * lj] + bii * R0[mj * NR + 2 * lj + 1]);
    }
  }
  for (int k = 0; k < 12; ++k) part[threadIdx.x][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < 12) {
    double s = 0;
    for (int u = 0; u < 256; ++u) s += part[u][threadIdx.x];
    part[0][threadIdx.x] = s;  // only thread k touches column k
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = out + t * kNObs;
    for (int k = 0; k < 11; ++k) o[k] = part[0][k] / g.Ns;
    double e = part[0][11], pur = 0, trd = 0, hd = 0;
    const int base = 3 * NLOC + 2 * NLOC * NLOC;
    for (int mu = 0; mu < g.nc; ++mu) {
      e += R0[mu * NR + base + 3];
      pur += R0[mu * NR + base + 1];
      trd = fmax(trd, hypot(R0[mu * NR + base] - 1.0, R0[mu * NR + base + 4]));   // |Tr - 1|, complex
      hd = fmax(hd, R0[mu * NR + base + 2]);
    }
    o[11] = e / g.Ns;
    o[12] = pur / g.nc;
    o[13] = trd;
    o[14] = hd;
  }
}

// Sums over trajectories, deterministic for a given trajectory count:
// chunks of OBS_CHUNK consecutive trajectories are summed in index order
// (Neumaier: sum, compensation; and the sum of squares), then the chunk
// partials are added in chunk order into sums[k] = (s, c, sum of squares).
constexpr int OBS_CHUNK = 64;

__device__ inline void neumaier_add(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

__global__ void __launch_bounds__(256) k_obs_chunks(const double* __restrict__ per_traj, int64_t n_traj,
                                                    double* __restrict__ part) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t chunk = idx / 16;
  const int k = (int)(idx % 16);
  const int64_t t0 = chunk * OBS_CHUNK;
  if (k >= kNObs || t0 >= n_traj) return;
  const int64_t t1 = t0 + OBS_CHUNK < n_traj ? t0 + OBS_CHUNK : n_traj;
  double s = 0, c = 0, q = 0;
  for (int64_t t = t0; t < t1; ++t) {
    const double x = per_traj[t * kNObs + k];
    neumaier_add(s, c, x);
    q += x * x;
  }
  part[(chunk * kNObs + k) * 3] = s;
  part[(chunk * kNObs + k) * 3 + 1] = c;
  part[(chunk * kNObs + k) * 3 + 2] = q;
}

__global__ void __launch_bounds__(64) k_obs_sum(const double* __restrict__ part, int64_t n_chunks,
                                                double* __restrict__ sums) {
  const int k = threadIdx.x;
  if (k >= kNObs) return;
  double s = sums[3 * k], c = sums[3 * k + 1], q = sums[3 * k + 2];
  for (int64_t ch = 0; ch < n_chunks; ++ch) {
    const double* v = part + (ch * kNObs + k) * 3;
    neumaier_add(s, c, v[0]);
    c += v[1];
    q += v[2];
  }
  sums[3 * k] = s;
  sums[3 * k + 1] = c;
  sums[3 * k + 2] = q;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int d, int NLOC>
constexpr int clusters_per_block() {
  constexpr int DD = cluster_dim<d, NLOC>() * cluster_dim<d, NLOC>();
  return DD >= 4096 ? 1 : 4096 / DD;
}

template <typename R, int d, int CX, int CY>
struct Generic {
  using Real = R;
  static constexpr int NLOC = CX * CY;
  static constexpr int D = cluster_dim<d, NLOC>();
  static constexpr int CPB = clusters_per_block<d, NLOC>();
  static constexpr int NT = 512;

  static hipError_t sample(const Geom& g, uint64_t seed, int64_t off, int8_t* noise, void* rho, hipStream_t s) {
    const int64_t total = g.n_traj * g.nc;
    constexpr int SCPB = CPB > 64 ? 64 : CPB;
    const int64_t blocks = (total + SCPB - 1) / SCPB;
    hipLaunchKernelGGL((k_sample<R, d, CX, CY, SCPB, NT>), dim3((unsigned)blocks), dim3(NT), 0, s, g, seed, off, noise,
                       (cpx<R>*)rho);
    return hipGetLastError();
  }
  static hipError_t site_fields(const Geom& g, const void* rho, void* b, hipStream_t s) {
    const int64_t n = g.n_traj * g.Ns;
    hipLaunchKernelGGL((k_site_fields<R, d, CX, CY>), dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, g,
                       (const cpx<R>*)rho, (cpx<R>*)b);
    return hipGetLastError();
  }
  static hipError_t boundary_fields(const Geom& g, const void* b, void* phi, hipStream_t s) {
    const int64_t n = g.n_traj * g.Ns;
    hipLaunchKernelGGL((k_boundary_fields<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                       (const cpx<R>*)b, (cpx<R>*)phi);
    return hipGetLastError();
  }
  static hipError_t stage(const StageArgs<R>& a, hipStream_t s) {
    if constexpr (D * D > 4096 * 2) {
      // the cluster matrix does not fit in LDS: kernels_big.hip
      (void)a;
      (void)s;
      return hipErrorInvalidValue;
    } else {
      const int64_t total = a.g.n_traj * a.g.nc;
      const int64_t blocks = (total + CPB - 1) / CPB;
      if (a.g.gdeph != 0 || a.g.gloss != 0)
        hipLaunchKernelGGL((k_stage<R, d, CX, CY, CPB, NT, true>), dim3((unsigned)blocks), dim3(NT), 0, s, a);
      else
        hipLaunchKernelGGL((k_stage<R, d, CX, CY, CPB, NT, false>), dim3((unsigned)blocks), dim3(NT), 0, s, a);
      return hipGetLastError();
    }
  }
  static hipError_t observables(const Geom& g, const void* rho, double* rec, double* per_traj, hipStream_t s) {
    constexpr int D = cluster_dim<d, CX * CY>();
    constexpr int NW = obs_waves<D>();
    if constexpr (D == 81) {
      // persistent: as many workgroups as fit on the device at once
      const int64_t total = g.n_traj * g.nc;
      const int64_t grid = std::min<int64_t>(total, (int64_t)obs_lds_slots(sizeof(R) == 4 ? 2 : 1));
      hipLaunchKernelGGL((k_obs_cluster_lds<R, d, CX, CY>), dim3((unsigned)grid), dim3(512), 0, s, g,
                         (const cpx<R>*)rho, rec, total);
    } else {
      hipLaunchKernelGGL((k_obs_cluster<R, d, CX, CY>), dim3((unsigned)(g.n_traj * g.nc)), dim3(64 * NW), 0, s, g,
                         (const cpx<R>*)rho, rec);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_obs_traj<NLOC>), dim3((unsigned)g.n_traj), dim3(256), 0, s, g, (const double*)rec, per_traj);
    return hipGetLastError();
  }
};

size_t obs_sum_scratch_doubles(int64_t n_traj) { return (size_t)((n_traj + OBS_CHUNK - 1) / OBS_CHUNK) * kNObs * 3; }

hipError_t launch_obs_sum(const double* per_traj, int64_t n_traj, double* sums, double* scratch, hipStream_t s) {
  const int64_t n_chunks = (n_traj + OBS_CHUNK - 1) / OBS_CHUNK;
  const int64_t threads = n_chunks * 16;
  hipLaunchKernelGGL(k_obs_chunks, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, per_traj, n_traj, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_obs_sum, dim3(1), dim3(64), 0, s, (const double*)scratch, n_chunks, sums);
  return hipGetLastError();
}

size_t obs_record_doubles(int nloc) {
  switch (nloc) {
    case 1: return cluster_rec<1>();
    case 2: return cluster_rec<2>();
    default: return cluster_rec<4>();
  }
}

// Dispatch on (precision, d, shape)
template <typename F>
static hipError_t dispatch(const Geom& g, int dtype, F&& f) {
#define CDTWA_CASE(RT, DV, X, Y)                                   \
  if (g.d == DV && g.cx == X && g.cy == Y) return f(Generic<RT, DV, X, Y>());
#define CDTWA_SHAPES(RT, DV) \
  CDTWA_CASE(RT, DV, 1, 1)   \
  CDTWA_CASE(RT, DV, 2, 1)   \
  CDTWA_CASE(RT, DV, 1, 2)   \
  CDTWA_CASE(RT, DV, 2, 2)
  if (dtype == 1) {
    CDTWA_SHAPES(double, 2)
    CDTWA_SHAPES(double, 3)
    CDTWA_CASE(double, 4, 1, 1)
    CDTWA_CASE(double, 4, 2, 1)
    CDTWA_CASE(double, 4, 1, 2)
    CDTWA_CASE(double, 4, 2, 2)
  } else {
    CDTWA_SHAPES(float, 2)
    CDTWA_SHAPES(float, 3)
    CDTWA_CASE(float, 4, 1, 1)
    CDTWA_CASE(float, 4, 2, 1)
    CDTWA_CASE(float, 4, 1, 2)
    CDTWA_CASE(float, 4, 2, 2)
  }
#undef CDTWA_SHAPES
#undef CDTWA_CASE
  return hipErrorInvalidValue;
}

bool generic_supported(int d, int cx, int cy) { return d >= 2 && d <= 4 && (cx == 1 || cx == 2) && (cy == 1 || cy == 2); }

hipError_t generic_sample(const Geom& g, int dtype, uint64_t seed, int64_t off, int8_t* noise, void* rho, hipStream_t s) {
  return dispatch(g, dtype, [&](auto k) { return decltype(k)::sample(g, seed, off, noise, rho, s); });
}
hipError_t generic_site_fields(const Geom& g, int dtype, const void* rho, void* b, hipStream_t s) {
  return dispatch(g, dtype, [&](auto k) { return decltype(k)::site_fields(g, rho, b, s); });
}
hipError_t generic_boundary_fields(const Geom& g, int dtype, const void* b, void* phi, hipStream_t s) {
  return dispatch(g, dtype, [&](auto k) { return decltype(k)::boundary_fields(g, b, phi, s); });
}
hipError_t generic_stage(const Geom& g, int dtype, void* rho, const void* kprev, const void* k1, const void* k2,
                         void* kout, const void* b_in, void* b_out, double dt, int mode, hipStream_t s) {
  return dispatch(g, dtype, [&](auto k) {
    using K = decltype(k);
    using RT = typename K::Real;
    StageArgs<RT> a;
    a.g = g;
    a.rho = (cpx<RT>*)rho;
    a.kprev = (const cpx<RT>*)kprev;
    a.k1 = (const cpx<RT>*)k1;
    a.k2 = (const cpx<RT>*)k2;
    a.kout = (cpx<RT>*)kout;
    a.b_in = (const cpx<RT>*)b_in;
    a.b_out = (cpx<RT>*)b_out;
    a.dt = (RT)dt;
    a.mode = mode;
    return K::stage(a, s);
  });
}
hipError_t generic_observables(const Geom& g, int dtype, const void* rho, double* rec, double* per_traj, hipStream_t s) {
  return dispatch(g, dtype, [&](auto k) { return decltype(k)::observables(g, rho, rec, per_traj, s); });
}

}  // namespace cdtwa
