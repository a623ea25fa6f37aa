// Trajectory-resident RK4 for small clusters (d = 3; 1x1, 2x1 and 1x2
// clusters, D = 3 and 9): one workgroup holds whole trajectories of one
// lattice on chip -- every cluster matrix in registers, the mean fields in
// LDS -- and integrates all the steps of a call without touching HBM
// between the initial load and the final store.  Sec. II Eq. (cluster_mf);
// App. B.1 Gamma^intra, Phi^inter and the RK4 remark.
//
// A work item is a block of trajectories of one member problem; a
// persistent grid pulls items from an atomic counter, so one launch advances
// every member of a batch (any mix of these cluster shapes, lattice sizes,
// couplings and trajectory counts) and the larger items, queued first, keep
// the tail short.  Thread t of the workgroup owns the columns
// i = t, t + NT, ... (i = (traj * nc + cluster) * D + q) of the stage
// matrix Y, of rho_n and of the running RK4 sum S.  Per stage:
//   A. the boundary fields phi of the owned clusters' sites from the mean
//      fields b of the lattice (LDS), and M = H Y on the owned column
//      (register-local: H acts on the row index), written to LDS;
//   B. K = -i (M - M^+) from the column and its transpose in LDS, the
//      classical RK4 update in registers, and every column's share of the
//      band sums b_l = sum_q sqrt(n_l(q)+1) Y[q + s_l][q] of the next
//      stage matrix;
//   C. b of every site, the band shares of its cluster added in column order.
#include <cstring>
#include <type_traits>

#include "launch.hpp"
#include "structured.hpp"

namespace cdtwa {

namespace {

constexpr int TNT = 512;              // threads per workgroup
constexpr int TLDS = 128 * 1024;      // LDS bytes for M, band shares and fields

// columns per thread for cluster dimension D: the state (3 arrays of IPT x D
// complex entries) and the temporaries of H Y fit in the 256 VGPRs of two
// waves per SIMD without spilling
template <typename R, int D>
constexpr int traj_ipt() {
  return sizeof(R) == 4 ? (D == 3 ? 6 : 2) : (D == 3 ? 3 : 1);
}

template <typename R>
struct TrajMember {
  cpx<R>* rho;        // [n_traj][nc][D][D]
  int64_t n_traj;
  int Lx, Ly, cx, cy, periodic;
  int Ns, ncx, nc;
  int ntr;            // trajectories per work item
  R J, U;
};

template <typename R>
struct TrajArgs {
  const TrajMember<R>* members;   // nullable: single member m0
  TrajMember<R> m0;
  const int2* work;               // (member, first trajectory); nullable: member 0, item k -> k * ntr
  int64_t n_work;
  int* counter;                   // zero at launch
  R dt;
  int n_steps;
};

// site of local index l (l = x_loc * cy + y_loc) of cluster mu
template <typename M>
__device__ inline int cluster_site_of(const M& m, int mu, int l) {
  const int mx = mu % m.ncx, my = mu / m.ncx;
  const int xl = l / m.cy, yl = l % m.cy;
  return (my * m.cy + yl) * m.Lx + mx * m.cx + xl;
}
// neighbour of site j in direction k (+x, -x, +y, -y) that lies in another
// cluster, -1 if none (open edge or same cluster)
template <typename M>
__device__ inline int ext_neighbour(const M& m, int j, int k) {
  const int x = j % m.Lx, y = j / m.Lx;
  int xx = x + (k == 0 ? 1 : (k == 1 ? -1 : 0)), yy = y + (k == 2 ? 1 : (k == 3 ? -1 : 0));
  if (m.periodic) {
    xx = (xx + m.Lx) % m.Lx;
    yy = (yy + m.Ly) % m.Ly;
  } else if (xx < 0 || xx >= m.Lx || yy < 0 || yy >= m.Ly) {
    return -1;
  }
  if (xx / m.cx == x / m.cx && yy / m.cy == y / m.cy) return -1;
  return yy * m.Lx + xx;
}

// One work item: trajectories t0 .. t0 + ntr - 1 of member m, n_steps steps.
template <typename R, int CX, int CY>
__device__ void traj_item(const TrajMember<R>& m, int64_t t0, R dt, int n_steps, char* smem) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<3, NLOC>();
  constexpr int DD = D * D;
  constexpr int IPT = traj_ipt<R, D>();
  const int tid = threadIdx.x;
  const int ntr = (int)(m.n_traj - t0 < m.ntr ? m.n_traj - t0 : m.ntr);
  const int nc = m.nc;
  const int n_items = ntr * nc * D;
  // LDS: M [ntr*nc][D][D], band shares [n_items][NLOC], phi [ntr*nc][NLOC],
  // and the lattice's neighbour table [nc*NLOC][4]: for site l of cluster mu
  // and direction +x, -x, +y, -y, the offset (mu' D) NLOC + l' of the band
  // shares of the neighbouring site l' of cluster mu' within a trajectory,
  // -1 where the neighbour is in the same cluster or beyond an open edge
  cpx<R>* sM = (cpx<R>*)smem;
  cpx<R>* sC = sM + (size_t)ntr * nc * DD;
  cpx<R>* sP = sC + (size_t)n_items * NLOC;
  int* sN = (int*)(sP + (size_t)ntr * nc * NLOC);
  const int per = nc * NLOC;
  const R J = m.J, U = m.U;
  const R h6 = dt / R(6);
  cpx<R> y[IPT][D], rr[IPT][D], ss[IPT][D];
  // load rho (column q of the cluster matrix of each owned item)
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const int i = tid + k * TNT;
    const bool act = i < n_items;
    const int ic = act ? i : 0;
    const int64_t base = (t0 * nc + ic / D) * DD + ic % D;   // (t0 nc + tc) DD + q
#pragma unroll
    for (int p = 0; p < D; ++p) {
      rr[k][p] = act ? m.rho[base + p * D] : cmake(R(0), R(0));
      y[k][p] = rr[k][p];
      ss[k][p] = cmake(R(0), R(0));
    }
  }
  // band shares of the column items: site l gets sqrt(n_l(q)+1) Y[q + s_l][q]
  auto band_shares = [&]() {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const int i = tid + k * TNT;
      if (i < n_items) {
        const int q = i % D;
#pragma unroll
        for (int l = 0; l < NLOC; ++l) {
          const int sl = kron_stride<3, NLOC>(l);
          const int n = digit<3, NLOC>(q, l);
          cpx<R> v = cmake(R(0), R(0));
#pragma unroll
          for (int p = 0; p < D; ++p)
            if (p == q + sl) v = y[k][p];
          const R c = n <= 1 ? R(sqrt_int<3>(n + 1)) : R(0);
          sC[(size_t)i * NLOC + l] = cmake(c * v.re, c * v.im);
        }
      }
    }
  };
  // phi of every cluster site (trajectory tau, site s = cluster * NLOC + l):
  // the mean fields b of its neighbours in other clusters, each b the band
  // shares of its cluster in column order
  auto site_phi = [&]() {
    int tau = tid / per, sl = tid - tau * per;
    for (int s2 = tid; s2 < ntr * per; s2 += TNT) {
      const cpx<R>* sh = sC + (size_t)tau * nc * D * NLOC;
      R re = 0, im = 0;
#pragma unroll
      for (int dir = 0; dir < 4; ++dir) {
        const int off = sN[sl * 4 + dir];
        if (off < 0) continue;
        R br = 0, bi = 0;
#pragma unroll
        for (int q = 0; q < D; ++q) {
          br += sh[off + q * NLOC].re;
          bi += sh[off + q * NLOC].im;
        }
        re += br;
        im += bi;
      }
      sP[s2] = cmake(re, im);
      sl += TNT;
      while (sl >= per) {
        sl -= per;
        ++tau;
      }
    }
  };
  for (int sl = tid; sl < per; sl += TNT) {
    const int j = cluster_site_of(m, sl / NLOC, sl % NLOC);
    for (int dir = 0; dir < 4; ++dir) {
      const int n = ext_neighbour(m, j, dir);
      int off = -1;
      if (n >= 0) {
        const int x = n % m.Lx, yy = n / m.Lx;
        off = ((yy / m.cy) * m.ncx + x / m.cx) * D * NLOC + (x % m.cx) * m.cy + yy % m.cy;
      }
      sN[sl * 4 + dir] = off;
    }
  }
  band_shares();
  __syncthreads();   // band shares and the neighbour table
  site_phi();
  __syncthreads();
  for (int st = 0; st < 4 * n_steps; ++st) {
    const int stage = st & 3;
    // ---- A: M = H Y on the owned columns, with phi of the cluster's sites
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const int i = tid + k * TNT;
      if (i < n_items) {
        const int tc = i / D, q = i % D;
        cpx<R> phi[NLOC];
#pragma unroll
        for (int l = 0; l < NLOC; ++l) phi[l] = sP[tc * NLOC + l];
        cpx<R>* mc = sM + (size_t)tc * DD + q;
#pragma unroll
        for (int p = 0; p < D; ++p) mc[p * D] = apply_h<R, 3, CX, CY, 1>(y[k], p, 0, phi, J, U);
      }
    }
    __syncthreads();
    // ---- B: K = -i (M - M^+) and the classical RK4 update, one loop per
    // kind of stage (0: the first, 1: the second and third, 3: the last)
    const R hin = stage == 2 ? dt : R(0.5) * dt;
    auto update = [&](auto kind) {
      constexpr int KS = decltype(kind)::value;
#pragma unroll
      for (int k = 0; k < IPT; ++k) {
        const int i = tid + k * TNT;
        const int ic = i < n_items ? i : 0;
        const int tc = ic / D, q = ic % D;
        const cpx<R>* mc = sM + (size_t)tc * DD;
#pragma unroll
        for (int p = 0; p < D; ++p) {
          const cpx<R> mpq = mc[p * D + q], mqp = mc[q * D + p];
          const R kr = mpq.im + mqp.im, ki = mqp.re - mpq.re;
          if constexpr (KS == 0) {
            ss[k][p] = cmake(kr, ki);
          } else if constexpr (KS == 1) {
            ss[k][p] = cmake(fma_r(R(2), kr, ss[k][p].re), fma_r(R(2), ki, ss[k][p].im));
          }
          if constexpr (KS < 3) {
            y[k][p] = cmake(fma_r(hin, kr, rr[k][p].re), fma_r(hin, ki, rr[k][p].im));
          } else {
            rr[k][p] = cmake(fma_r(h6, ss[k][p].re + kr, rr[k][p].re), fma_r(h6, ss[k][p].im + ki, rr[k][p].im));
            y[k][p] = rr[k][p];
          }
        }
      }
    };
    if (stage == 0)
      update(std::integral_constant<int, 0>{});
    else if (stage < 3)
      update(std::integral_constant<int, 1>{});
    else
      update(std::integral_constant<int, 3>{});
    band_shares();
    __syncthreads();
    // ---- C: phi of every site for the next stage
    site_phi();
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const int i = tid + k * TNT;
    if (i >= n_items) continue;
    const int64_t base = (t0 * nc + i / D) * DD + i % D;
#pragma unroll
    for (int p = 0; p < D; ++p) m.rho[base + p * D] = rr[k][p];
  }
}

template <typename R>
__global__ void __launch_bounds__(TNT, 1) k_traj(TrajArgs<R> a) {
  __shared__ __align__(16) char smem[TLDS];
  __shared__ int sItem;
  for (;;) {
    __syncthreads();   // the previous item's last LDS reads are done
    if (threadIdx.x == 0) sItem = atomicAdd(a.counter, 1);
    __syncthreads();
    const int64_t item = sItem;
    if (item >= a.n_work) break;
    int mi = 0;
    int64_t t0;
    if (a.work) {
      const int2 w = a.work[item];
      mi = w.x;
      t0 = w.y;
    } else {
      t0 = item * a.m0.ntr;
    }
    const TrajMember<R> m = a.members ? a.members[mi] : a.m0;
    if (m.cx == 1 && m.cy == 1)
      traj_item<R, 1, 1>(m, t0, a.dt, a.n_steps, smem);
    else if (m.cx == 2)
      traj_item<R, 2, 1>(m, t0, a.dt, a.n_steps, smem);
    else
      traj_item<R, 1, 2>(m, t0, a.dt, a.n_steps, smem);
  }
}

__global__ void k_traj_zero(int* p) { *p = 0; }

}  // namespace

bool traj_supported(int model, int d, int cx, int cy, bool diss) {
  return model == 0 && d == 3 && !diss && ((cx == 1 && cy == 1) || (cx == 2 && cy == 1) || (cx == 1 && cy == 2));
}

// Trajectories one workgroup holds for this lattice (0 if not even one fits):
// limited by the columns its registers hold and by the LDS for M, the band
// shares and the fields of each trajectory next to the neighbour table.
int traj_per_item(const Geom& g, int dtype) {
  if (!traj_supported(g.model, g.d, g.cx, g.cy, g.gdeph > 0 || g.gloss > 0)) return 0;
  const int D = g.D, nloc = g.nloc;
  const int cs = dtype == 1 ? 16 : 8;
  const int ipt = dtype == 1 ? (D == 3 ? traj_ipt<double, 3>() : traj_ipt<double, 9>())
                             : (D == 3 ? traj_ipt<float, 3>() : traj_ipt<float, 9>());
  const int64_t per_traj_items = (int64_t)g.nc * D;
  const int64_t per_traj_lds = ((int64_t)g.nc * D * D + per_traj_items * nloc + g.Ns) * cs;
  const int64_t table = (int64_t)g.Ns * 4 * sizeof(int);
  if (table >= TLDS) return 0;
  int64_t n = (int64_t)TNT * ipt / per_traj_items;
  const int64_t nl = (TLDS - table) / per_traj_lds;
  if (nl < n) n = nl;
  if (n > g.n_traj) n = g.n_traj;
  return n < 1 ? 0 : (int)n;
}

template <typename R>
static TrajMember<R> traj_member(const Geom& g, void* rho, int ntr, double J, double U) {
  TrajMember<R> m;
  m.rho = (cpx<R>*)rho;
  m.n_traj = g.n_traj;
  m.Lx = g.Lx;
  m.Ly = g.Ly;
  m.cx = g.cx;
  m.cy = g.cy;
  m.periodic = g.periodic;
  m.Ns = g.Ns;
  m.ncx = g.ncx;
  m.nc = g.nc;
  m.ntr = ntr;
  m.J = (R)J;
  m.U = (R)U;
  return m;
}

size_t traj_member_bytes(int dtype) { return dtype == 1 ? sizeof(TrajMember<double>) : sizeof(TrajMember<float>); }

void traj_member_fill(const Geom& g, int dtype, void* rho, int ntr, void* out) {
  if (dtype == 1) {
    const TrajMember<double> m = traj_member<double>(g, rho, ntr, g.J, g.U);
    std::memcpy(out, &m, sizeof(m));
  } else {
    const TrajMember<float> m = traj_member<float>(g, rho, ntr, g.J, g.U);
    std::memcpy(out, &m, sizeof(m));
  }
}

static int traj_grid(int64_t n_work) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return (int)(n_work < cus ? n_work : cus);
}

template <typename R>
static hipError_t traj_launch(const TrajArgs<R>& a, hipStream_t s) {
  hipLaunchKernelGGL(k_traj_zero, dim3(1), dim3(1), 0, s, a.counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.n_work == 0) return e;
  hipLaunchKernelGGL((k_traj<R>), dim3((unsigned)traj_grid(a.n_work)), dim3(TNT), 0, s, a);
  return hipGetLastError();
}

hipError_t traj_rk4(const Geom& g, int dtype, void* rho, int* counter, double dt, int n_steps, hipStream_t s) {
  const int ntr = traj_per_item(g, dtype);
  if (ntr < 1) return hipErrorInvalidValue;
  const int64_t n_work = (g.n_traj + ntr - 1) / ntr;
  if (dtype == 1) {
    TrajArgs<double> a{};
    a.m0 = traj_member<double>(g, rho, ntr, g.J, g.U);
    a.n_work = n_work;
    a.counter = counter;
    a.dt = dt;
    a.n_steps = n_steps;
    return traj_launch<double>(a, s);
  }
  TrajArgs<float> a{};
  a.m0 = traj_member<float>(g, rho, ntr, g.J, g.U);
  a.n_work = n_work;
  a.counter = counter;
  a.dt = (float)dt;
  a.n_steps = n_steps;
  return traj_launch<float>(a, s);
}

hipError_t traj_batch_rk4(int dtype, const void* members, const int2* work, int64_t n_work, int* counter, double dt,
                          int n_steps, hipStream_t s) {
  if (dtype == 1) {
    TrajArgs<double> a{};
    a.members = (const TrajMember<double>*)members;
    a.work = work;
    a.n_work = n_work;
    a.counter = counter;
    a.dt = dt;
    a.n_steps = n_steps;
    return traj_launch<double>(a, s);
  }
  TrajArgs<float> a{};
  a.members = (const TrajMember<float>*)members;
  a.work = work;
  a.n_work = n_work;
  a.counter = counter;
  a.dt = (float)dt;
  a.n_steps = n_steps;
  return traj_launch<float>(a, s);
}

}  // namespace cdtwa
