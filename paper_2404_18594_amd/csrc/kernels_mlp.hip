// Control variate for the C-dTWA estimator: a small MLP g(noise of a site
// patch) trained to predict the nearest-neighbour correlation carried by the
// central cluster of the patch, with BF16 weights and FP32 accumulation.
// Dense products run on MFMA (v_mfma_f32_16x16x16_bf16); everything else is
// elementwise or a fixed-order reduction.
#include "launch.hpp"

namespace cdtwa {

namespace {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest, ties to even
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan kept
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C[m][n] = sum_{k in [k0,k1)} A[m][k] B[k][n] for a 32x32 tile per wave,
// A element (m,k) at a[m*sam + k*sak], B element (k,n) at b[k*sbk + n*sbn]
// (BF16), C element at c[m*ldc + n] (FP32, overwritten). K range must be a
// multiple of 16; M and N edges are masked.
struct GemmArgs {
  const uint16_t* a;
  const uint16_t* b;
  float* c;
  int64_t sam, sak, sbk, sbn, ldc;
  int M, N, K;
  int ksplit;          // number of K slices (partials at c + slice*M*ldc)
};

__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  const int wave = (blockIdx.x * 4) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tiles_n = (g.N + 31) / 32;
  const int tiles_m = (g.M + 31) / 32;
  const int tiles = tiles_m * tiles_n;
  const int slice = wave / tiles;
  if (slice >= g.ksplit) return;
  const int t = wave % tiles;
  const int m0 = (t / tiles_n) * 32, n0 = (t % tiles_n) * 32;
  const int kper = ((g.K / 16 + g.ksplit - 1) / g.ksplit) * 16;
  const int k0 = slice * kper, k1 = min(g.K, k0 + kper);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
  const int row = lane & 15, kq = (lane >> 4) * 4;
  for (int kk = k0; kk < k1; kk += 16) {
    s16x4 av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = m0 + 16 * i + row;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        av[i][e] = (short)(m < g.M ? g.a[(int64_t)m * g.sam + (int64_t)(kk + kq + e) * g.sak] : 0);
      const int n = n0 + 16 * i + row;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        bv[i][e] = (short)(n < g.N ? g.b[(int64_t)(kk + kq + e) * g.sbk + (int64_t)n * g.sbn] : 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[i], bv[j], acc[i][j], 0, 0, 0);
  }
  float* c = g.c + (int64_t)slice * g.M * g.ldc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + 16 * i + kq + e, n = n0 + 16 * j + row;
        if (m < g.M && n < g.N) c[(int64_t)m * g.ldc + n] = acc[i][j][e];
      }
}

// sum of ksplit partial products in slice order, then bias / activation:
// mode 0: out = sum (+ bias); mode 1: z = sum + bias, keep z, act = bf16(relu(z))
__global__ void k_gemm_epilogue(const float* part, int ksplit, int64_t MN, int N, const float* bias, float* out,
                                uint16_t* act_bf16, int mode) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MN) return;
  float s = 0;
  for (int sl = 0; sl < ksplit; ++sl) s += part[(int64_t)sl * MN + i];
  if (bias) s += bias[i % N];
  if (out) out[i] = s;
  if (mode == 1) act_bf16[i] = to_bf16(s > 0.f ? s : 0.f);
}

__global__ void k_to_bf16(const float* x, uint16_t* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// dz = dact * (z > 0), also as BF16
__global__ void k_relu_back(const float* dact, const float* z, float* dz, uint16_t* dz_bf16, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = z[i] > 0.f ? dact[i] : 0.f;
  dz[i] = v;
  dz_bf16[i] = to_bf16(v);
}

// column sums of x [rows][N] times `scale`, in a fixed order for a given
// row count: pass 1 splits the rows into P contiguous chunks (at most 256,
// of at least 64 rows) and sums each chunk per column (64 columns x 4 row
// groups per workgroup; group g adds rows g, g+4, ... of the chunk in order,
// then the 4 group sums are added in group order) into part[p][n]; pass 2
// adds the P chunk sums in chunk order.  A 4096-row batch with 256 columns
// runs on 256 workgroups.
constexpr int CS_GROUPS = 4;
__global__ void __launch_bounds__(256) k_colsum_part(const float* x, int64_t rows, int N, int64_t ch, float* part) {
  __shared__ float red[CS_GROUPS][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int64_t r0 = (int64_t)blockIdx.y * ch;
  const int64_t r1 = r0 + ch < rows ? r0 + ch : rows;
  float s = 0;
  if (n < N)
    for (int64_t r = r0 + g; r < r1; r += CS_GROUPS) s += x[r * N + n];
  red[g][c] = s;
  __syncthreads();
  if (g == 0 && n < N) {
    float t = 0;
    for (int k = 0; k < CS_GROUPS; ++k) t += red[k][c];
    part[(int64_t)blockIdx.y * N + n] = t;
  }
}
__global__ void __launch_bounds__(64) k_colsum_final(const float* part, int P, int N, float scale, float* out) {
  const int n = blockIdx.x * 64 + threadIdx.x;
  if (n >= N) return;
  float t = 0;
  // unrolled so that the loads are issued ahead of the (ordered) additions
#pragma unroll 16
  for (int p = 0; p < P; ++p) t += part[(int64_t)p * N + n];
  out[n] = t * scale;
}

// mean-squared-error gradient dy = 2 (y - t) / (rows * N) and the loss
// terms (summed per column, then over columns, by the column-sum passes)
__global__ void k_mse_grad(const float* y, const float* t, float* dy, uint16_t* dy_bf16, float* sq, int64_t n,
                           float scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float d = y[i] - t[i];
  dy[i] = 2.f * d * scale;
  dy_bf16[i] = to_bf16(2.f * d * scale);
  sq[i] = d * d;
}

// Adam (Kingma & Ba) on the FP32 master weights, then the BF16 copy
__global__ void k_adam(float* w, uint16_t* w_bf16, const float* grad, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (w_bf16) w_bf16[i] = to_bf16(wi);
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t gemm_bf16(const uint16_t* a, int64_t sam, int64_t sak, const uint16_t* b, int64_t sbk, int64_t sbn,
                     float* c, int64_t ldc, int M, int N, int K, int ksplit, hipStream_t s) {
  GemmArgs g{a, b, c, sam, sak, sbk, sbn, ldc, M, N, K, ksplit};
  const int64_t waves = (int64_t)((M + 31) / 32) * ((N + 31) / 32) * ksplit;
  hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, g);
  return hipGetLastError();
}
hipError_t gemm_epilogue(const float* part, int ksplit, int64_t MN, int N, const float* bias, float* out,
                         uint16_t* act, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_gemm_epilogue, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, s, part, ksplit, MN, N, bias,
                     out, act, mode);
  return hipGetLastError();
}
hipError_t to_bf16_array(const float* x, uint16_t* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}
hipError_t relu_back(const float* dact, const float* z, float* dz, uint16_t* dzb, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_relu_back, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dact, z, dz, dzb, n);
  return hipGetLastError();
}
hipError_t colsum(const float* x, int64_t rows, int N, float scale, float* out, float* scratch, hipStream_t s) {
  if (N < 1 || rows < 0) return hipErrorInvalidValue;
  const int64_t ch = std::max<int64_t>(COLSUM_MIN_CHUNK, (rows + COLSUM_MAX_CHUNKS - 1) / COLSUM_MAX_CHUNKS);
  const int64_t P = std::max<int64_t>(1, (rows + ch - 1) / ch);
  hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)((N + 63) / 64), (unsigned)P), dim3(256), 0, s, x, rows, N, ch,
                     scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum_final, dim3((unsigned)((N + 63) / 64)), dim3(64), 0, s, (const float*)scratch, (int)P,
                     N, scale, out);
  return hipGetLastError();
}
hipError_t mse_grad(const float* y, const float* t, float* dy, uint16_t* dyb, float* sq, int64_t n, float scale,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_mse_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, t, dy, dyb, sq, n, scale);
  return hipGetLastError();
}
hipError_t adam_update(float* w, uint16_t* wb, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, wb, g, m, v, n, lr, b1, b2, eps, c1,
                     c2);
  return hipGetLastError();
}

}  // namespace cdtwa

// ---------------------------------------------------------------------------
// Features and targets of the control variate
// ---------------------------------------------------------------------------
namespace cdtwa {
namespace {

// Patch of cluster mu: the 4x4 sites x in [x0-1, x0+2], y in [y0-1, y0+2]
// around the cluster's 2x2 block (x0, y0) = (2 mx, 2 my); patch site
// s = 4 (y - y0 + 1) + (x - x0 + 1); feature 8 s + a = r^a of that site
// (0 outside an open lattice).
__global__ void k_cv_features(Geom g, const int8_t* __restrict__ noise, float* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (traj, cluster, s)
  const int64_t total = g.n_traj * g.nc * 16;
  if (i >= total) return;
  const int s = (int)(i % 16);
  const int64_t tc = i / 16;
  const int64_t t = tc / g.nc;
  const int mu = (int)(tc % g.nc);
  const int x0 = (mu % g.ncx) * g.cx, y0 = (mu / g.ncx) * g.cy;
  int x = x0 - 1 + s % 4, y = y0 - 1 + s / 4;
  bool inside = true;
  if (g.periodic) {
    x = (x + g.Lx) % g.Lx;
    y = (y + g.Ly) % g.Ly;
  } else {
    inside = x >= 0 && x < g.Lx && y >= 0 && y < g.Ly;
  }
  float* f = feat + tc * (16 * g.n_gen) + s * g.n_gen;
  for (int a = 0; a < g.n_gen; ++a) {
    float v = 0.f;
    if (inside) {
      const int j = y * g.Lx + x;
      v = (float)g.val[a * kMaxD + noise[(t * g.Ns + j) * g.n_gen + a]];
    }
    f[a] = v;
  }
}

// i.i.d. patch features drawn from the site noise distribution: patch
// p = first + row, site s, generator a uses Philox counter (a/4, s, p_lo,
// p_hi) with key (seed, seed >> 32) xor 0x5bd1e995 in the upper key word, so
// the stream is disjoint from the trajectory draws of the same seed.
__global__ void k_cv_sample_features(Geom g, uint64_t seed, int64_t first, int64_t n, float* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (patch, s, a)
  const int64_t total = n * 16 * g.n_gen;
  if (i >= total) return;
  const int a = (int)(i % g.n_gen);
  const int s = (int)((i / g.n_gen) % 16);
  const uint64_t p = (uint64_t)(first + i / (16 * g.n_gen));
  uint32_t w[4];
  philox4x32_10((uint32_t)(a / 4), (uint32_t)s, (uint32_t)p, (uint32_t)(p >> 32), (uint32_t)seed,
                (uint32_t)(seed >> 32) ^ 0x5bd1e995u, w);
  const uint32_t x = w[a % 4];
  int o = 0;
  while (o < g.n_out[a] - 1 && !((uint64_t)x < g.thr[a * kMaxD + o])) ++o;
  feat[i] = (float)g.val[a * kMaxD + o];
}

// t_mu = sum over the sites i of cluster mu of Re<a_i^+ a_{i+x}> + Re<a_i^+ a_{i+y}>
// (the nearest-neighbour correlation carried by the cluster), from the
// observable cluster records (b, n, intra-cluster pairs)
template <int NLOC>
__global__ void k_cv_targets(Geom g, const double* __restrict__ rec, float* __restrict__ out, int ldo, int col) {
  constexpr int NR = cluster_rec<NLOC>();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (traj, cluster)
  if (i >= g.n_traj * g.nc) return;
  const int64_t t = i / g.nc;
  const int mu = (int)(i % g.nc);
  const double* R0 = rec + t * g.nc * NR;
  double s = 0;
  for (int l = 0; l < NLOC; ++l) {
    const int j = g.cluster_site[mu * NLOC + l];
    const int xi = j % g.Lx, yi = j / g.Lx;
    const double bir = R0[mu * NR + 2 * l], bii = R0[mu * NR + 2 * l + 1];
    for (int dir = 0; dir < 2; ++dir) {
      int xj = xi + (dir == 0), yj = yi + (dir == 1);
      if (g.periodic) {
        xj %= g.Lx;
        yj %= g.Ly;
      } else if (xj >= g.Lx || yj >= g.Ly) {
        continue;
      }
      const int jj = yj * g.Lx + xj;
      const int mj = g.site_cluster[jj], lj = g.site_local[jj];
      if (mj == mu)
        s += R0[mu * NR + 3 * NLOC + l * NLOC + lj];
      else
        s += bir * R0[mj * NR + 2 * lj] + bii * R0[mj * NR + 2 * lj + 1];
    }
  }
  out[i * ldo + col] = (float)s;
}

// FP64 column moments of y [rows][N], N <= 64: block b covers rows
// [b*per, (b+1)*per); 4 row groups per block summed in group order;
// part[b][n] = (sum y, sum y^2)
__global__ void __launch_bounds__(256) k_colmom_part(const float* y, int64_t rows, int N, int64_t per,
                                                     double* part) {
  __shared__ double s1[4][64], s2[4][64];
  const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(rows, r0 + per);
  double a = 0, q = 0;
  if (c < N)
    for (int64_t r = r0 + rg; r < r1; r += 4) {
      const double v = (double)y[r * N + c];
      a += v;
      q += v * v;
    }
  s1[rg][c] = a;
  s2[rg][c] = q;
  __syncthreads();
  if (rg == 0 && c < N) {
    double ta = 0, tq = 0;
    for (int k = 0; k < 4; ++k) {
      ta += s1[k][c];
      tq += s2[k][c];
    }
    part[((int64_t)blockIdx.x * N + c) * 2] = ta;
    part[((int64_t)blockIdx.x * N + c) * 2 + 1] = tq;
  }
}

// adds the block partials in block order into out[n] = (Neumaier sum,
// compensation, sum of squares)
__global__ void k_colmom_final(const double* part, int nblk, int N, double* out) {
  const int c = threadIdx.x;
  if (c >= N) return;
  double sum = out[3 * c], comp = out[3 * c + 1], sq = out[3 * c + 2];
  for (int b = 0; b < nblk; ++b) {
    const double v = part[((int64_t)b * N + c) * 2];
    const double t = sum + v;
    comp += fabs(sum) >= fabs(v) ? (sum - t) + v : (v - t) + sum;
    sum = t;
    sq += part[((int64_t)b * N + c) * 2 + 1];
  }
  out[3 * c] = sum;
  out[3 * c + 1] = comp;
  out[3 * c + 2] = sq;
}

// out[t][n] = scale * sum over the rows_per_traj rows of trajectory t (in
// row order) of y[t][row][n], FP64
__global__ void k_traj_sums(const float* y, int rows_per_traj, int N, double scale, double* out) {
  const int64_t t = blockIdx.x;
  for (int c = threadIdx.x; c < N; c += blockDim.x) {
    double s = 0;
    const float* yt = y + t * rows_per_traj * N;
    for (int r = 0; r < rows_per_traj; ++r) s += (double)yt[(int64_t)r * N + c];
    out[t * N + c] = s * scale;
  }
}

// parameter initialisation: weight (layer l, index i) uniform in
// [-bound_l, bound_l) from Philox counter (i_lo, i_hi, l, 0x4d4c50) keyed by
// the seed; biases zero; the BF16 copy is the rounded FP32 value
__global__ void k_mlp_init(float* w, uint16_t* wb, int64_t n, float bound, int layer, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t r[4];
  philox4x32_10((uint32_t)i, (uint32_t)(i >> 32), (uint32_t)layer, 0x4d4c50u, (uint32_t)seed, (uint32_t)(seed >> 32),
                r);
  const float u = (float)(r[0] >> 8) * (1.0f / 16777216.0f);
  const float v = (2.f * u - 1.f) * bound;
  w[i] = v;
  if (wb) wb[i] = to_bf16(v);
}

__global__ void k_fill_zero(float* w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = 0.f;
}

}  // namespace

hipError_t cv_features(const Geom& g, const int8_t* noise, float* feat, hipStream_t s) {
  const int64_t n = g.n_traj * g.nc * 16;
  hipLaunchKernelGGL(k_cv_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, noise, feat);
  return hipGetLastError();
}
hipError_t cv_sample_features(const Geom& g, uint64_t seed, int64_t first, int64_t n, float* feat, hipStream_t s) {
  const int64_t tot = n * 16 * g.n_gen;
  hipLaunchKernelGGL(k_cv_sample_features, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g, seed, first, n,
                     feat);
  return hipGetLastError();
}
hipError_t cv_targets(const Geom& g, const double* rec, float* out, int ldo, int col, hipStream_t s) {
  const int64_t n = g.n_traj * g.nc;
  if (g.nloc == 4)
    hipLaunchKernelGGL(k_cv_targets<4>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, rec, out, ldo, col);
  else if (g.nloc == 2)
    hipLaunchKernelGGL(k_cv_targets<2>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, rec, out, ldo, col);
  else
    hipLaunchKernelGGL(k_cv_targets<1>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, rec, out, ldo, col);
  return hipGetLastError();
}
hipError_t colmoments(const float* y, int64_t rows, int N, double* part, int nblk_max, double* out, hipStream_t s) {
  int64_t per = std::max<int64_t>(256, (rows + nblk_max - 1) / nblk_max);
  const int nblk = (int)((rows + per - 1) / per);
  hipLaunchKernelGGL(k_colmom_part, dim3((unsigned)nblk), dim3(256), 0, s, y, rows, N, per, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colmom_final, dim3(1), dim3(64), 0, s, part, nblk, N, out);
  return hipGetLastError();
}
hipError_t traj_sums(const float* y, int64_t n_traj, int rows_per_traj, int N, double scale, double* out,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_traj_sums, dim3((unsigned)n_traj), dim3(64), 0, s, y, rows_per_traj, N, scale, out);
  return hipGetLastError();
}
hipError_t mlp_init_layer(float* w, uint16_t* wb, int64_t n, float bound, int layer, uint64_t seed, hipStream_t s) {
  if (bound > 0)
    hipLaunchKernelGGL(k_mlp_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, wb, n, bound, layer, seed);
  else
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, n);
  return hipGetLastError();
}

}  // namespace cdtwa
