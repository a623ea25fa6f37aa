// Dense-GEMM variant of one RK4 stage for 2x2 clusters with d = 3 (D = 81),
// FP32 state: the cluster Hamiltonian H = H_C + H_MF (Sec. II
// Eq. (cluster_mf); App. B.1 Gamma^intra, Phi^inter) is built as a dense
// 81x81 complex matrix in LDS next to Y, and M = H Y is a complex matrix
// product on the matrix cores (v_mfma_f32_16x16x4_f32; Re M = Hr Yr - Hi Yi,
// Im M = Hr Yi + Hi Yr on 16x16 tiles of the matrices padded to 96).  The
// rest of the stage (K = -i (M - M^+), the RK4 update with K1..K3 in HBM, the
// next stage's mean fields) is the per-stage path's.  This route does ~9.7x
// the flops of the structured operator; it exists to be measured against it.
#include "launch.hpp"
#include "structured.hpp"

namespace cdtwa {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int DD_D = 81;
constexpr int DD_P = 96;    // padded side: 6 tiles of 16
constexpr int DD_L = 81;    // LDS row stride (complex entries)
constexpr int DD_NT = 256;  // 4 waves

__global__ void __launch_bounds__(DD_NT) k_dense_stage(StageArgs<float> a) {
  constexpr int D = DD_D, DDn = D * D, NLOC = 4;
  __shared__ cpx<float> sY[D * DD_L];   // Y, then M
  __shared__ cpx<float> sH[D * DD_L];   // dense H
  __shared__ cpx<float> sPhi[NLOC];
  const Geom& g = a.g;
  const int64_t flat = blockIdx.x;
  const int mode = a.mode;
  const float cin = mode == 4 ? a.dt : 0.5f * a.dt;
  const float cout = mode == 3 ? a.dt : 0.5f * a.dt;
  const float J = (float)g.J, U = (float)g.U;
  const cpx<float>* rho = a.rho + flat * DDn;
  // Y = rho + cin K_{s-1}
  for (int e = threadIdx.x; e < DDn; e += DD_NT) {
    cpx<float> y = rho[e];
    if (mode >= 2) {
      const cpx<float> k = a.kprev[flat * DDn + e];
      y.re = fma_r(cin, k.re, y.re);
      y.im = fma_r(cin, k.im, y.im);
    }
    sY[(e / D) * DD_L + e % D] = y;
  }
  if (threadIdx.x < NLOC) {
    const int l = threadIdx.x;
    const int64_t t = flat / g.nc;
    const int mu = (int)(flat % g.nc);
    const int j = g.cluster_site[mu * NLOC + l];
    float re = 0, im = 0;
    for (int k = 0; k < 4; ++k) {
      const int n = g.ext_nbr[j * 4 + k];
      if (n < 0) continue;
      const cpx<float> v = a.b_in[t * g.Ns + n];
      re += v.re;
      im += v.im;
    }
    sPhi[l] = cmake(re, im);
  }
  __syncthreads();
  // dense H, one row per thread pass: H[p][p'] for every p'
  for (int p = threadIdx.x; p < D; p += DD_NT) {
    cpx<float>* row = sH + p * DD_L;
    for (int c = 0; c < D; ++c) row[c] = cmake(0.f, 0.f);
    int nd[NLOC];
    for (int l = 0; l < NLOC; ++l) nd[l] = digit<3, NLOC>(p, l);
    float diag = 0;
    for (int l = 0; l < NLOC; ++l) diag += 0.5f * (float)(nd[l] * (nd[l] - 1));
    row[p].re = U * diag;
    for (int b = 0; b < Bonds<2, 2>::n; ++b) {
      const int l = Bonds<2, 2>::l(b), m = Bonds<2, 2>::m(b);
      const int sl = kron_stride<3, NLOC>(l), sm = kron_stride<3, NLOC>(m);
      if (nd[l] >= 1 && nd[m] <= 1) row[p - sl + sm].re = -J * (float)(sqrt_int<3>(nd[l]) * sqrt_int<3>(nd[m] + 1));
      if (nd[m] >= 1 && nd[l] <= 1) row[p - sm + sl].re = -J * (float)(sqrt_int<3>(nd[m]) * sqrt_int<3>(nd[l] + 1));
    }
    for (int l = 0; l < NLOC; ++l) {
      const int sl = kron_stride<3, NLOC>(l);
      if (nd[l] <= 1) {   // -J conj(phi_l) a_l: column p + s_l
        const float c = -J * (float)sqrt_int<3>(nd[l] + 1);
        row[p + sl] = cmake(c * sPhi[l].re, -c * sPhi[l].im);
      }
      if (nd[l] >= 1) {   // -J phi_l a_l^+: column p - s_l
        const float c = -J * (float)sqrt_int<3>(nd[l]);
        row[p - sl] = cmake(c * sPhi[l].re, c * sPhi[l].im);
      }
    }
  }
  __syncthreads();
  // M = H Y on the matrix cores: wave w owns the 16x16 output tiles w, w+4, ...
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int NTI = DD_P / 16;
  f32x4 accr[9], acci[9];
#pragma unroll
  for (int s = 0; s < 9; ++s) {
    const int tile = wave + 4 * s;
    const int i0 = (tile / NTI) * 16, j0 = (tile % NTI) * 16;
    f32x4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    for (int k0 = 0; k0 < DD_P; k0 += 4) {
      const int i = i0 + li, k = k0 + lk, j = j0 + li;
      const cpx<float> h = (i < D && k < D) ? sH[i * DD_L + k] : cmake(0.f, 0.f);   // A[i][k]
      const cpx<float> y = (k < D && j < D) ? sY[k * DD_L + j] : cmake(0.f, 0.f);   // B[k][j]
      cr = __builtin_amdgcn_mfma_f32_16x16x4f32(h.re, y.re, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_16x16x4f32(-h.im, y.im, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x4f32(h.re, y.im, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x4f32(h.im, y.re, ci, 0, 0, 0);
    }
    accr[s] = cr;
    acci[s] = ci;
  }
  __syncthreads();   // every wave is done reading Y
#pragma unroll
  for (int s = 0; s < 9; ++s) {
    const int tile = wave + 4 * s;
    const int i0 = (tile / NTI) * 16, j0 = (tile % NTI) * 16;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + 4 * lk + e, j = j0 + li;
      if (i < D && j < D) sY[i * DD_L + j] = cmake(accr[s][e], acci[s][e]);
    }
  }
  __syncthreads();
  // K = -i (M - M^+) and the RK4 update (K-store scheme of the per-stage
  // path); Y_{s+1} kept in registers, then staged through LDS for the fields
  constexpr int EPT = (DDn + DD_NT - 1) / DD_NT;
  const float h6 = a.dt / 6.f;
  cpx<float> yn[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * DD_NT;
    if (e >= DDn) continue;
    const int p = e / D, q = e % D;
    const cpx<float> m = sY[p * DD_L + q], mt = sY[q * DD_L + p];
    const cpx<float> kk = cmake(m.im + mt.im, mt.re - m.re);
    const int64_t gi = flat * DDn + e;
    const cpx<float> r0 = a.rho[gi];
    if (mode <= 3) {
      a.kout[gi] = kk;
      yn[i] = cmake(fma_r(cout, kk.re, r0.re), fma_r(cout, kk.im, r0.im));
    } else {
      const cpx<float> q1 = a.k1[gi], q2 = a.k2[gi], q3 = a.kprev[gi];
      const float sr = fma_r(2.f, q3.re, fma_r(2.f, q2.re, q1.re)) + kk.re;
      const float si = fma_r(2.f, q3.im, fma_r(2.f, q2.im, q1.im)) + kk.im;
      yn[i] = cmake(fma_r(h6, sr, r0.re), fma_r(h6, si, r0.im));
      a.rho[gi] = yn[i];
    }
  }
  if (mode == 0) return;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * DD_NT;
    if (e < DDn) sY[(e / D) * DD_L + e % D] = yn[i];
  }
  __syncthreads();
  if (threadIdx.x < NLOC) {
    const int l = threadIdx.x;
    const int sl = kron_stride<3, NLOC>(l);
    float re = 0, im = 0;
    for (int q = 0; q < D; ++q) {
      const int n = digit<3, NLOC>(q, l);
      if (n > 1) continue;
      const float c = (float)sqrt_int<3>(n + 1);
      const cpx<float> y = sY[(q + sl) * DD_L + q];
      re = fma_r(c, y.re, re);
      im = fma_r(c, y.im, im);
    }
    const int64_t t = flat / g.nc;
    const int mu = (int)(flat % g.nc);
    a.b_out[t * g.Ns + g.cluster_site[mu * NLOC + l]] = cmake(re, im);
  }
}

}  // namespace

bool dense_supported(int d, int cx, int cy, int dtype) { return d == 3 && cx == 2 && cy == 2 && dtype == 0; }

hipError_t dense_stage(const Geom& g, int dtype, void* rho, const void* kprev, const void* k1, const void* k2,
                       void* kout, const void* b_in, void* b_out, double dt, int mode, hipStream_t s) {
  if (!dense_supported(g.d, g.cx, g.cy, dtype)) return hipErrorInvalidValue;
  StageArgs<float> a{g, (cpx<float>*)rho, (const cpx<float>*)kprev, (const cpx<float>*)k1, (const cpx<float>*)k2,
                     (cpx<float>*)kout, (const cpx<float>*)b_in, (cpx<float>*)b_out, (float)dt, mode};
  hipLaunchKernelGGL(k_dense_stage, dim3((unsigned)(g.n_traj * g.nc)), dim3(DD_NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace cdtwa
