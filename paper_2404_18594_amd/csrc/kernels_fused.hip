// Fused persistent RK4 kernel for 2x2 clusters with d = 3 (D = 81).
//
// One workgroup owns one cluster of one trajectory for a whole call and keeps
// its matrices on chip: thread (q, k) holds rows 27k..27k+26 of column q of
// the stage matrix Y, of rho_n and of the running sum S of the stage
// derivatives (243 active threads of 256).  All clusters of G trajectories
// run concurrently (cooperative launch, so every workgroup is resident) and
// exchange their mean fields b_j = Tr(a_j rho_C) through tagged 64-bit words
// in global memory: every word carries the stage number in its upper half, so
// a reader that sees the right tag has the value, with no fence.
//
// A stage (Sec. II Eq. (cluster_mf); App. B.1 Gamma^intra, Phi^inter and the
// RK4 remark):
//   A. M  = H_0 Y on the thread's own rows (interaction + the hops between
//      sites 2,3,4), written to LDS          -- needs no neighbour data
//   B. wave 0 waits for the neighbours' b of this stage -> phi
//   C. M += (field terms) Y + (terms that move the site-1 digit), the latter
//      exchanged between the three threads of a column with DPP lane shifts
//   D. K = -i (M - M^+) from LDS, classical RK4 update in registers
//   E. b of the next stage matrix from the K band in LDS, published by wave 0
#include "launch.hpp"

namespace cdtwa {

namespace {

constexpr int FD = 81;     // cluster dimension
constexpr int FB = 27;     // rows per thread
constexpr int FNT = 256;   // threads per workgroup
constexpr int LS = 81;     // LDS row stride (complex entries)

template <typename R>
struct FusedArgs {
  cpx<R>* rho;          // [n_traj][nc][81][81]
  uint64_t* xch;        // [G][nc][2][16] tagged words
  int* status;          // bit 0: neighbour wait timed out
  const int* legs;      // [nc][4][4]: neighbour (cluster*4 + local) of local l in direction dir, -1 if none
  int64_t n_traj;
  int nc, G, n_steps;
  R J, U, dt;
  int spin_limit;
};

// lane i <- lane i+1 (wave_shl:1) and lane i <- lane i-1 (wave_shr:1); lanes
// with no source read 0
__device__ inline int dpp_next_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true); }
__device__ inline int dpp_prev_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true); }
__device__ inline float dpp_next(float v) { return __int_as_float(dpp_next_i(__float_as_int(v))); }
__device__ inline float dpp_prev(float v) { return __int_as_float(dpp_prev_i(__float_as_int(v))); }
__device__ inline double dpp_next(double v) {
  return __hiloint2double(dpp_next_i(__double2hiint(v)), dpp_next_i(__double2loint(v)));
}
__device__ inline double dpp_prev(double v) {
  return __hiloint2double(dpp_prev_i(__double2hiint(v)), dpp_prev_i(__double2loint(v)));
}

__device__ constexpr double sq(int n) {
  return n == 0 ? 0.0 : (n == 1 ? 1.0 : 1.4142135623730951);
}

// payload words per real: FP64 splits into two 32-bit halves
template <typename R>
struct Words;
template <>
struct Words<double> {
  static constexpr int per_real = 2;
  __device__ static uint32_t half(double v, int w) {
    return (uint32_t)(w == 0 ? __double2loint(v) : __double2hiint(v));
  }
  __device__ static double join(uint32_t lo, uint32_t hi) { return __hiloint2double((int)hi, (int)lo); }
};
template <>
struct Words<float> {
  static constexpr int per_real = 1;
  __device__ static uint32_t half(float v, int) { return (uint32_t)__float_as_int(v); }
  __device__ static float join(uint32_t lo, uint32_t) { return __int_as_float((int)lo); }
};

// FP64 keeps one cluster per compute unit; FP32 fits two
template <typename R>
__global__ void __launch_bounds__(FNT, sizeof(R) == 8 ? 1 : 2) k_fused(FusedArgs<R> a) {
  constexpr int WPR = Words<R>::per_real;
  constexpr int WPB = 2 * WPR;  // words per complex b
  __shared__ cpx<R> sM[FD * LS];
  __shared__ cpx<R> sBand[4][64];
  __shared__ cpx<R> sPhi[4];
  __shared__ int sBail;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int q = wave * 21 + lane / 3;
  const int k = lane % 3;
  const bool active = lane < 63 && q < FD;
  const int g = blockIdx.x / a.nc;
  const int mu = blockIdx.x % a.nc;
  const R J = a.J, U = a.U, dt = a.dt;
  const R hk = (k == 2) ? R(1) : R(0);                  // h(n1) = n1 (n1-1)/2
  const R cdn = k <= 1 ? R(sq(k + 1)) : R(0);           // from block k+1: sqrt(k+1)
  const R cup = R(sq(k));                                // from block k-1: sqrt(k)
  const int* legs = a.legs + mu * 16;
  uint64_t* xout = a.xch + ((size_t)g * a.nc + mu) * 32;
  if (tid == 0) sBail = 0;

  cpx<R> y[FB], rr[FB], ss[FB];
  uint32_t tag = 0;

  for (int64_t round = 0;; ++round) {
    const int64_t t = round * a.G + g;
    if (t >= a.n_traj) break;
    cpx<R>* rho = a.rho + ((size_t)t * a.nc + mu) * FD * FD;
#pragma unroll
    for (int r = 0; r < FB; ++r) {
      rr[r] = active ? rho[(27 * k + r) * FD + q] : cmake(R(0), R(0));
      y[r] = rr[r];
      ss[r] = cmake(R(0), R(0));
    }
    // b(rho) from the band of rho in global memory (216 terms)
    cpx<R> bR = cmake(R(0), R(0)), bS = cmake(R(0), R(0));
    {
      __syncthreads();
      if (tid < 216) {
        const int l = tid / 54, j = tid % 54;
        const int s = l == 0 ? 27 : (l == 1 ? 9 : (l == 2 ? 3 : 1));
        const int lo = j % s, dl = (j / s) % 2, hi = j / (2 * s);
        const int qq = hi * 3 * s + dl * s + lo;
        const cpx<R> v = rho[(qq + s) * FD + qq];
        const R c = R(sq(dl + 1));
        sBand[l][j] = cmake(c * v.re, c * v.im);
      } else if (tid < 256 && (tid - 216) < 40) {
        const int u = tid - 216;
        sBand[u / 10][54 + u % 10] = cmake(R(0), R(0));
      }
      __syncthreads();
    }
    // wave 0: reduce the band terms, publish b(rho)
    auto reduce_band = [&](void) -> cpx<R> {
      // lane -> (l = lane/16, part = lane%16); four terms each, then a 16-lane tree
      const int l = lane >> 4, part = lane & 15;
      R re = 0, im = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const cpx<R> v = sBand[l][part + 16 * u];
        re += v.re;
        im += v.im;
      }
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) {
        re += __shfl_xor(re, off, 16);
        im += __shfl_xor(im, off, 16);
      }
      return cmake(re, im);  // valid in every lane of row l
    };
    auto publish = [&](cpx<R> bl, uint32_t tg) {
      // lanes 16l..16l+15 hold b_l; lanes 0..4*WPB-1 store one word each
      const int l = lane / WPB, w = lane % WPB;
      cpx<R> v;
      v.re = __shfl(bl.re, l * 16);
      v.im = __shfl(bl.im, l * 16);
      if (lane < 4 * WPB) {
        const R comp = (w / WPR) == 0 ? v.re : v.im;
        const uint32_t payload = Words<R>::half(comp, w % WPR);
        const uint64_t word = ((uint64_t)tg << 32) | payload;
        __hip_atomic_store(&xout[(tg & 1) * 16 + lane], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    };
    // wave 0: wait until every neighbour leg carries tag `want`; the leg
    // values (re, im) end up in the leader lane e*WPB of leg e = 4*l + dir
    auto wait_legs = [&](uint32_t want, R& lre, R& lim) {
      lre = R(0);
      lim = R(0);
      if (sBail) return;
      const int e = lane / WPB, w = lane % WPB;
      const int nb = e < 16 ? legs[e] : -1;
      bool done = nb < 0;
      uint32_t payload = 0;
      uint64_t* src = nullptr;
      if (nb >= 0) src = a.xch + ((size_t)g * a.nc + (nb >> 2)) * 32 + (want & 1) * 16 + (nb & 3) * WPB + w;
      int spins = 0;
      while (true) {
        if (!done) {
          const uint64_t word = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if ((uint32_t)(word >> 32) == want) {
            done = true;
            payload = (uint32_t)word;
          }
        }
        if (__all(done)) break;
        if (++spins > a.spin_limit) {
          if (lane == 0) {
            atomicOr(a.status, 1);
            sBail = 1;
          }
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      const uint32_t w0 = __shfl(payload, (e * WPB + 0) & 63);
      const uint32_t w1 = __shfl(payload, (e * WPB + (WPR == 2 ? 1 : 0)) & 63);
      const uint32_t w2 = __shfl(payload, (e * WPB + WPR) & 63);
      const uint32_t w3 = __shfl(payload, (e * WPB + WPR + (WPR == 2 ? 1 : 0)) & 63);
      lre = (nb >= 0) ? Words<R>::join(w0, w1) : R(0);
      lim = (nb >= 0) ? Words<R>::join(w2, w3) : R(0);
    };
    if (round > 0 && wave != 0) ++tag;
    if (wave == 0) {
      if (round > 0) {
        // the neighbours' last publish of the previous trajectory: once seen,
        // they have consumed our last words and the slot may be reused
        R lre, lim;
        wait_legs(tag + 1, lre, lim);
        ++tag;
      }
      bR = reduce_band();
      publish(bR, tag + 1);
    }

    const int total_stages = 4 * a.n_steps;
    for (int st = 0; st < total_stages; ++st) {
      const int stage = st & 3;
      const uint32_t want = tag + 1;
      // ---- A: M = H0 Y restricted to the thread's rows (no site-1 moves)
#pragma unroll
      for (int r = 0; r < FB; ++r) {
        const int n2 = r / 9, n3 = (r / 3) % 3, n4 = r % 3;
        const R dg = U * (hk + R((n2 == 2) + (n3 == 2) + (n4 == 2)));
        R mr = dg * y[r].re, mi = dg * y[r].im;
        // bond sites 2-4 (locals 1,3; strides 9,1)
        if (n2 >= 1 && n4 <= 1) { const R c = -J * R(sq(n2) * sq(n4 + 1)); mr += c * y[r - 9 + 1].re; mi += c * y[r - 9 + 1].im; }
        if (n4 >= 1 && n2 <= 1) { const R c = -J * R(sq(n4) * sq(n2 + 1)); mr += c * y[r - 1 + 9].re; mi += c * y[r - 1 + 9].im; }
        // bond sites 3-4 (locals 2,3; strides 3,1)
        if (n3 >= 1 && n4 <= 1) { const R c = -J * R(sq(n3) * sq(n4 + 1)); mr += c * y[r - 3 + 1].re; mi += c * y[r - 3 + 1].im; }
        if (n4 >= 1 && n3 <= 1) { const R c = -J * R(sq(n4) * sq(n3 + 1)); mr += c * y[r - 1 + 3].re; mi += c * y[r - 1 + 3].im; }
        if (active) sM[(27 * k + r) * LS + q] = cmake(mr, mi);
      }
      // ---- B: neighbour mean fields of this stage -> phi
      if (wave == 0) {
        R lre, lim;
        wait_legs(want, lre, lim);
        // phi_l = sum over dir 0..3 (+x,-x,+y,-y) of the leg values
        R pr = 0, pi = 0;
#pragma unroll
        for (int dir = 0; dir < 4; ++dir) {
          pr += __shfl(lre, (4 * (lane & 3) + dir) * WPB);
          pi += __shfl(lim, (4 * (lane & 3) + dir) * WPB);
        }
        if (lane < 4) sPhi[lane] = cmake(pr, pi);
      }
      __syncthreads();
      if (sBail) break;
      const cpx<R> f0 = sPhi[0], f1 = sPhi[1], f2 = sPhi[2], f3 = sPhi[3];
      // ---- C: field terms and the moves of the site-1 digit
#pragma unroll
      for (int r = 0; r < FB; ++r) {
        const int n2 = r / 9, n3 = (r / 3) % 3, n4 = r % 3;
        // what this block sends to block k-1 (a_1 applied there): -J [conj(phi0) y + a_2^+ y + a_3^+ y]
        R dr = f0.re * y[r].re + f0.im * y[r].im, di = f0.re * y[r].im - f0.im * y[r].re;
        if (n2 >= 1) { const R c = R(sq(n2)); dr += c * y[r - 9].re; di += c * y[r - 9].im; }
        if (n3 >= 1) { const R c = R(sq(n3)); dr += c * y[r - 3].re; di += c * y[r - 3].im; }
        // what this block sends to block k+1 (a_1^+ applied there): -J [phi0 y + a_2 y + a_3 y]
        R ur = f0.re * y[r].re - f0.im * y[r].im, ui = f0.re * y[r].im + f0.im * y[r].re;
        if (n2 <= 1) { const R c = R(sq(n2 + 1)); ur += c * y[r + 9].re; ui += c * y[r + 9].im; }
        if (n3 <= 1) { const R c = R(sq(n3 + 1)); ur += c * y[r + 3].re; ui += c * y[r + 3].im; }
        const R rdr = dpp_next(dr), rdi = dpp_next(di);   // from block k+1
        const R rur = dpp_prev(ur), rui = dpp_prev(ui);   // from block k-1
        R mr = -J * (cdn * rdr + cup * rur), mi = -J * (cdn * rdi + cup * rui);
        // fields on sites 2,3,4: -J (conj(phi_l) a_l + phi_l a_l^+)
        auto field = [&](const cpx<R>& f, int n, int s) {
          if (n <= 1) {  // conj(f) sqrt(n+1) y[r+s]
            const R c = -J * R(sq(n + 1));
            const cpx<R> v = y[r + s];
            mr += c * (f.re * v.re + f.im * v.im);
            mi += c * (f.re * v.im - f.im * v.re);
          }
          if (n >= 1) {  // f sqrt(n) y[r-s]
            const R c = -J * R(sq(n));
            const cpx<R> v = y[r - s];
            mr += c * (f.re * v.re - f.im * v.im);
            mi += c * (f.re * v.im + f.im * v.re);
          }
        };
        field(f1, n2, 9);
        field(f2, n3, 3);
        field(f3, n4, 1);
        if (active) {
          cpx<R>& m = sM[(27 * k + r) * LS + q];
          m.re += mr;
          m.im += mi;
        }
      }
      __syncthreads();
      // ---- band of K for the next mean fields
      if (tid < 216) {
        const int l = tid / 54, j = tid % 54;
        const int s = l == 0 ? 27 : (l == 1 ? 9 : (l == 2 ? 3 : 1));
        const int lo = j % s, dl = (j / s) % 2, hi = j / (2 * s);
        const int qq = hi * 3 * s + dl * s + lo;
        const cpx<R> mpq = sM[(qq + s) * LS + qq], mqp = sM[qq * LS + qq + s];
        const R c = R(sq(dl + 1));
        sBand[l][j] = cmake(c * (mpq.im + mqp.im), c * (mqp.re - mpq.re));
      }
      // ---- D: K = -i (M - M^+) and the RK4 update
      const R hin = stage == 2 ? dt : R(0.5) * dt;
#pragma unroll
      for (int r = 0; r < FB; ++r) {
        const int p = 27 * k + r;
        const cpx<R> mpq = active ? sM[p * LS + q] : cmake(R(0), R(0));
        const cpx<R> mqp = active ? sM[q * LS + p] : cmake(R(0), R(0));
        const cpx<R> kk = cmake(mpq.im + mqp.im, mqp.re - mpq.re);
        if (stage == 0) {
          ss[r] = kk;
        } else if (stage < 3) {
          ss[r].re += R(2) * kk.re;
          ss[r].im += R(2) * kk.im;
        }
        if (stage < 3) {
          y[r].re = rr[r].re + hin * kk.re;
          y[r].im = rr[r].im + hin * kk.im;
        } else {
          const R h6 = dt / R(6);
          rr[r].re = rr[r].re + h6 * (ss[r].re + kk.re);
          rr[r].im = rr[r].im + h6 * (ss[r].im + kk.im);
          y[r] = rr[r];
        }
      }
      __syncthreads();
      ++tag;
      if (wave == 0) {
        const cpx<R> bK = reduce_band();
        cpx<R> bn;
        if (stage == 0) {
          bS = bK;
        } else if (stage < 3) {
          bS.re += R(2) * bK.re;
          bS.im += R(2) * bK.im;
        }
        if (stage < 3) {
          bn = cmake(bR.re + hin * bK.re, bR.im + hin * bK.im);
        } else {
          const R h6 = dt / R(6);
          bR = cmake(bR.re + h6 * (bS.re + bK.re), bR.im + h6 * (bS.im + bK.im));
          bn = bR;
        }
        publish(bn, tag + 1);
      }
    }
    if (sBail) {
      // poison this cluster so that a timed-out call cannot pass unnoticed
      const R nan = __builtin_nan("");
#pragma unroll
      for (int r = 0; r < FB; ++r)
        if (active) rho[(27 * k + r) * FD + q] = cmake(nan, nan);
      break;
    }
#pragma unroll
    for (int r = 0; r < FB; ++r)
      if (active) rho[(27 * k + r) * FD + q] = rr[r];
  }
}

__global__ void k_zero_words(uint64_t* p, size_t n, int* status) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
  if (i == 0 && status) *status = 0;
}

}  // namespace

size_t fused_exchange_words(int nc, int G) { return (size_t)G * nc * 32; }

// Largest number of trajectories the fused kernel can keep resident at once
// for nc clusters each (0 if not even one fits).
int fused_slots(int nc, int dtype) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e = dtype == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<double>, FNT, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<float>, FNT, 0);
  if (e != hipSuccess || per_cu <= 0) return 0;
  return (cus * per_cu) / nc;
}

hipError_t fused_rk4(const Geom& g, int dtype, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                     double dt, int n_steps, int spin_limit, hipStream_t s) {
  const size_t nw = fused_exchange_words(g.nc, G);
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, xch, nw, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)(g.nc * G)), block(FNT);
  if (dtype == 1) {
    FusedArgs<double> a{(cpx<double>*)rho, xch, status, legs, g.n_traj, g.nc, G, n_steps, g.J, g.U, dt, spin_limit};
    void* args[] = {&a};
    return hipLaunchCooperativeKernel((const void*)k_fused<double>, grid, block, args, 0, s);
  }
  FusedArgs<float> a{(cpx<float>*)rho, xch, status, legs, g.n_traj, g.nc, G, n_steps, (float)g.J, (float)g.U,
                     (float)dt, spin_limit};
  void* args[] = {&a};
  return hipLaunchCooperativeKernel((const void*)k_fused<float>, grid, block, args, 0, s);
}

}  // namespace cdtwa
