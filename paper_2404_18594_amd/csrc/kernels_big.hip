// Per-stage path for cluster matrices larger than the LDS: 2x2 clusters with
// d = 4 (D = 256; 1 MB per cluster in FP64).  One RK4 stage (or the bare
// commutator) is three launches:
//   k_big_apply    M = (H_C + H_MF) Y for a block of QB columns per workgroup
//                  (Y = rho + c K_{s-1} formed on load, staged in LDS),
//                  written to a scratch matrix in HBM;
//   k_big_combine  K = -i (M - M^+) on a pair of 32x32 tiles, (i, j) and its
//                  mirror (j, i), both staged in LDS so that M is read from
//                  HBM once and every read is row-contiguous, and the
//                  classical RK4 update;
//   k_big_fields   mean fields b_l of the next stage matrix from its bands.
// Sec. II Eq. (cluster_mf); App. B.1 Gamma^intra, Phi^inter and the RK4 remark.
#include "launch.hpp"
#include "structured.hpp"

namespace cdtwa {

namespace {

// columns per apply workgroup: 8 (FP64: 32 KB of LDS, so that more
// workgroups per CU keep loads in flight; 0.186 vs 0.155 M cluster-steps/s
// with 16)
template <typename R>
constexpr int big_qb() {
  return 8;
}

// Workgroups are dealt to the 8 XCDs in turn (block b to XCD b % 8).  This
// renumbering gives XCD x a contiguous range of logical blocks, so that the
// workgroups of one cluster matrix run on one XCD and its L2 rather than
// spread over all eight (bijective for any grid size).
__device__ inline int64_t xcd_block() {
  constexpr int64_t NX = 8;
  const int64_t G = gridDim.x, b = blockIdx.x;
  const int64_t q = G / NX, r = G % NX, x = b % NX, i = b / NX;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}
constexpr int BTB = 32;   // combine tile side
constexpr int BNT = 256;  // threads per workgroup

template <typename R, int d, int CX, int CY>
__global__ void __launch_bounds__(BNT) k_big_apply(StageArgs<R> a, cpx<R>* __restrict__ M) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  constexpr int DD = D * D;
  constexpr int BQB = big_qb<R>();
  constexpr int NB = D / BQB;
  __shared__ cpx<R> sY[D * BQB];
  __shared__ cpx<R> sPhi[NLOC];
  const Geom& g = a.g;
  const int64_t bid = xcd_block();
  const int64_t flat = bid / NB;   // (trajectory, cluster)
  const int q0 = (int)(bid % NB) * BQB;
  const int mode = a.mode;
  const R cin = mode == 4 ? a.dt : R(0.5) * a.dt;
  const cpx<R>* rho = a.rho + flat * DD;
  const cpx<R>* kp = a.kprev ? a.kprev + flat * DD : nullptr;
  // every load of the block issued before the first LDS store
  constexpr int EPT = D * BQB / BNT;
  static_assert(EPT * BNT == D * BQB, "apply block shape");
  if (mode >= 2) {
    cpx<R> y[EPT], k[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * BNT, p = e / BQB, c = e % BQB;
      y[i] = rho[p * D + q0 + c];
      k[i] = kp[p * D + q0 + c];
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      y[i].re += cin * k[i].re;
      y[i].im += cin * k[i].im;
      sY[threadIdx.x + i * BNT] = y[i];
    }
  } else {
    cpx<R> y[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * BNT, p = e / BQB, c = e % BQB;
      y[i] = rho[p * D + q0 + c];
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) sY[threadIdx.x + i * BNT] = y[i];
  }
  if (threadIdx.x < NLOC) {
    const int l = threadIdx.x;
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
    sPhi[l] = cmake(re, im);
  }
  __syncthreads();
  const R J = R(g.J), U = R(g.U);
  cpx<R>* out = M + flat * DD;
  for (int e = threadIdx.x; e < D * BQB; e += BNT) {
    const int p = e / BQB, c = e % BQB;
    out[p * D + q0 + c] = apply_h<R, d, CX, CY, BQB>(sY, p, c, sPhi, J, U);
  }
}

// Tile pair number t of NT (NT + 1) / 2 (i <= j, row-major over the upper
// triangle of tiles) -> (i, j)
template <int NT>
__device__ inline void tile_pair(int t, int& i, int& j) {
  i = 0;
  while (t >= NT - i) {
    t -= NT - i;
    ++i;
  }
  j = i + t;
}

template <typename R, int d, int CX, int CY>
__global__ void __launch_bounds__(BNT) k_big_combine(StageArgs<R> a, const cpx<R>* __restrict__ M) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  constexpr int DD = D * D;
  constexpr int NT = D / BTB;              // tiles per side
  constexpr int NP = NT * (NT + 1) / 2;    // tile pairs (i <= j)
  constexpr int EPT = BTB * BTB / BNT;     // entries of one tile per thread
  static_assert(EPT * BNT == BTB * BTB, "combine tile shape");
  __shared__ cpx<R> sP[2][BTB][BTB + 1];   // [0]: tile (i, j), [1]: tile (j, i)
  const int64_t cbid = xcd_block();
  const int64_t flat = cbid / NP;
  int ti, tj;
  tile_pair<NT>((int)(cbid % NP), ti, tj);
  const bool diag = ti == tj;
  const int r0 = ti * BTB, c0 = tj * BTB;  // sP[0][r][c] = M[r0 + r][c0 + c], sP[1][r][c] = M[c0 + r][r0 + c]
  const cpx<R>* m = M + flat * DD;
  {
    // both tiles loaded unconditionally (a diagonal tile twice, the second
    // read from L2): a load under a branch kept its array in scratch memory
    // and waited for every load before the next
    cpx<R> va[EPT], vb[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * BNT, r = e / BTB, c = e % BTB;
      va[i] = m[(r0 + r) * D + c0 + c];
      vb[i] = m[(c0 + r) * D + r0 + c];
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * BNT, r = e / BTB, c = e % BTB;
      sP[0][r][c] = va[i];
      sP[1][r][c] = vb[i];
    }
  }
  __syncthreads();
  const int mode = a.mode;
  const R h6 = a.dt / R(6);
  // half 0: entries (r0 + r, c0 + c), own tile sP[0], mirror sP[1];
  // half 1: entries (c0 + r, r0 + c), own sP[1], mirror sP[0] (off-diagonal
  // pairs only: a diagonal tile is its own mirror, sP[1] = sP[0])
  for (int half = 0; half < (diag ? 1 : 2); ++half) {
    const int own = half, mir = 1 - half;
    const int p0 = half == 0 ? r0 : c0, q0 = half == 0 ? c0 : r0;
    if (mode <= 3) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * BNT, r = e / BTB, c = e % BTB;
        const cpx<R> mpq = sP[own][r][c], mqp = sP[mir][c][r];
        // K = -i (M - M^+):  K.re = Im M_pq + Im M_qp,  K.im = Re M_qp - Re M_pq
        a.kout[flat * DD + (int64_t)(p0 + r) * D + q0 + c] = cmake(mpq.im + mqp.im, mqp.re - mpq.re);
      }
    } else {
      cpx<R> r_[EPT], k1[EPT], k2[EPT], k3[EPT];
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * BNT, r = e / BTB, c = e % BTB;
        const int64_t gi = flat * DD + (int64_t)(p0 + r) * D + q0 + c;
        r_[i] = a.rho[gi];
        k1[i] = a.k1[gi];
        k2[i] = a.k2[gi];
        k3[i] = a.kprev[gi];
      }
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * BNT, r = e / BTB, c = e % BTB;
        const int64_t gi = flat * DD + (int64_t)(p0 + r) * D + q0 + c;
        const cpx<R> mpq = sP[own][r][c], mqp = sP[mir][c][r];
        const cpx<R> k = cmake(mpq.im + mqp.im, mqp.re - mpq.re);
        const R sr = k1[i].re + R(2) * k2[i].re + R(2) * k3[i].re + k.re;
        const R si = k1[i].im + R(2) * k2[i].im + R(2) * k3[i].im + k.im;
        a.rho[gi] = cmake(r_[i].re + h6 * sr, r_[i].im + h6 * si);
      }
    }
  }
}

// b_l of Y_{s+1} = rho + cout K_s (modes 1..3) or of the new rho (mode 4):
// sum over rows q with digit_l(q) <= d-2 of sqrt(digit_l(q)+1) Y[q + s_l][q],
// added in a fixed order (per thread in row order, then a tree over threads)
template <typename R, int d, int CX, int CY>
__global__ void __launch_bounds__(BNT) k_big_fields(StageArgs<R> a) {
  constexpr int NLOC = CX * CY;
  constexpr int D = cluster_dim<d, NLOC>();
  constexpr int DD = D * D;
  __shared__ R sRe[NLOC][BNT], sIm[NLOC][BNT];
  const Geom& g = a.g;
  const int64_t flat = blockIdx.x;
  const int mode = a.mode;
  const R cout = mode == 3 ? a.dt : R(0.5) * a.dt;
  const cpx<R>* rho = a.rho + flat * DD;
  const cpx<R>* k = mode <= 3 ? a.kout + flat * DD : nullptr;
#pragma unroll
  for (int l = 0; l < NLOC; ++l) {
    const int sl = kron_stride<d, NLOC>(l);
    R re = 0, im = 0;
    for (int q = threadIdx.x; q < D; q += BNT) {
      const int n = digit<d, NLOC>(q, l);
      if (n > d - 2) continue;
      const R c = R(sqrt_int<d>(n + 1));
      cpx<R> y = rho[(q + sl) * D + q];
      if (mode <= 3) {
        const cpx<R> kk = k[(q + sl) * D + q];
        y.re += cout * kk.re;
        y.im += cout * kk.im;
      }
      re += c * y.re;
      im += c * y.im;
    }
    sRe[l][threadIdx.x] = re;
    sIm[l][threadIdx.x] = im;
  }
  __syncthreads();
  for (int w = BNT / 2; w > 0; w /= 2) {
    if (threadIdx.x < w)
#pragma unroll
      for (int l = 0; l < NLOC; ++l) {
        sRe[l][threadIdx.x] += sRe[l][threadIdx.x + w];
        sIm[l][threadIdx.x] += sIm[l][threadIdx.x + w];
      }
    __syncthreads();
  }
  if (threadIdx.x < NLOC) {
    const int l = threadIdx.x;
    const int64_t t = flat / g.nc;
    const int mu = (int)(flat % g.nc);
    a.b_out[t * g.Ns + g.cluster_site[mu * NLOC + l]] = cmake(sRe[l][0], sIm[l][0]);
  }
}

template <typename R, int d, int CX, int CY>
hipError_t big_stage_t(const StageArgs<R>& a, cpx<R>* M, hipStream_t s) {
  constexpr int D = cluster_dim<d, CX * CY>();
  constexpr int BQB = big_qb<R>();
  static_assert(D % BQB == 0 && D % BTB == 0, "tile shape");
  const int64_t clusters = a.g.n_traj * a.g.nc;
  hipLaunchKernelGGL((k_big_apply<R, d, CX, CY>), dim3((unsigned)(clusters * (D / BQB))), dim3(BNT), 0, s, a, M);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int NT = D / BTB;
  hipLaunchKernelGGL((k_big_combine<R, d, CX, CY>), dim3((unsigned)(clusters * (NT * (NT + 1) / 2))), dim3(BNT), 0,
                     s, a, (const cpx<R>*)M);
  e = hipGetLastError();
  if (e != hipSuccess || a.mode == 0) return e;
  hipLaunchKernelGGL((k_big_fields<R, d, CX, CY>), dim3((unsigned)clusters), dim3(BNT), 0, s, a);
  return hipGetLastError();
}

}  // namespace

bool big_supported(int d, int cx, int cy) { return d == 4 && cx == 2 && cy == 2; }

hipError_t big_stage(const Geom& g, int dtype, void* rho, const void* kprev, const void* k1, const void* k2,
                     void* kout, const void* b_in, void* b_out, double dt, int mode, void* M, hipStream_t s) {
  if (!big_supported(g.d, g.cx, g.cy)) return hipErrorInvalidValue;
  if (dtype == 1) {
    StageArgs<double> a{g, (cpx<double>*)rho, (const cpx<double>*)kprev, (const cpx<double>*)k1,
                        (const cpx<double>*)k2, (cpx<double>*)kout, (const cpx<double>*)b_in, (cpx<double>*)b_out,
                        dt, mode};
    return big_stage_t<double, 4, 2, 2>(a, (cpx<double>*)M, s);
  }
  StageArgs<float> a{g, (cpx<float>*)rho, (const cpx<float>*)kprev, (const cpx<float>*)k1, (const cpx<float>*)k2,
                     (cpx<float>*)kout, (const cpx<float>*)b_in, (cpx<float>*)b_out, (float)dt, mode};
  return big_stage_t<float, 4, 2, 2>(a, (cpx<float>*)M, s);
}

}  // namespace cdtwa
