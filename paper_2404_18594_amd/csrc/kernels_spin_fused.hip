// Fused persistent RK4 kernel for the transverse-field Ising model with 2x2
// clusters (D = 16): one wave per cluster, the whole cluster state on chip.
//
// Lane L holds row p = L / 4 and columns q = 4 (L % 4) + c, c = 0..3, of the
// stage matrix Y and of the running sum S of the stage derivatives in
// registers; its entries of rho_n and of K sit in LDS.  In the product basis (|0> = |up>, local site 0 the
// most significant bit) s^z is diagonal and s^x flips one bit, so
//   [H, Y][p][q] = (E_p - E_q) Y[p][q] + h sum_l (Y[p ^ bit_l][q] - Y[p][q ^ bit_l])
// (App. A Eq. (Hising) with the cluster mean field of Sec. II Eq.
// (cluster_mf): E_p = J sum over intra bonds z_l z_m + sum_l F_l z_l, F_l = J
// times the sum of Re b_k over the neighbours k of site l in other clusters,
// b_k = Tr(s^z_k rho)).  Flipping a bit of p is a lane exchange (xor 32, 16,
// 8, 4 for sites 0..3), flipping bit 8 or 4 of q a lane exchange within the
// quad (xor 2, 1), flipping bit 2 or 1 of q a register exchange.  All lane
// exchanges within a row of 16 lanes are DPP moves.
//
// All clusters of G trajectories run concurrently (cooperative launch) and
// exchange b through tagged 64-bit words in global memory, as the fused
// Bose-Hubbard kernels do: every word carries the stage number in its upper
// half, so a reader that sees the right tag has the value.  A stage:
//   A. wait for the neighbours' words of this stage, form F_l
//   B. K = -i [H, Y] entry by entry, the classical RK4 update in registers
//   C. b of the next stage matrix from its diagonal, published for the
//      neighbours
#include "launch.hpp"

namespace cdtwa {

namespace {

constexpr int SD = 16;    // cluster dimension
constexpr int SNT = 64;   // one wave per cluster

template <typename R>
struct SpinFusedArgs {
  cpx<R>* rho;          // [n_traj][nc][16][16]
  uint64_t* xch;        // [G][nc][32] tagged words: slot (tag parity) * 16 + site * words + word
  int* status;          // bit 0: neighbour wait timed out
  const int* legs;      // [nc][4][4]: neighbour (cluster*4 + local) of local l in direction dir, -1 if none
  int64_t n_traj;
  int nc, G, n_steps;
  R J, h, dt;
  int spin_limit;
  int sched;                          // 1: J and h of every stage from sJ, sH
  R sJ[kSchedVals], sH[kSchedVals];   // at every half step of this launch
};

// payload words per real: FP64 splits into two 32-bit halves
template <typename R>
struct SWords;
template <>
struct SWords<double> {
  static constexpr int per_real = 2;
  __device__ static uint32_t half(double v, int w) {
    return (uint32_t)(w == 0 ? __double2loint(v) : __double2hiint(v));
  }
  __device__ static double join(uint32_t lo, uint32_t hi) { return __hiloint2double((int)hi, (int)lo); }
};
template <>
struct SWords<float> {
  static constexpr int per_real = 1;
  __device__ static uint32_t half(float v, int) { return (uint32_t)__float_as_int(v); }
  __device__ static float join(uint32_t lo, uint32_t) { return __int_as_float((int)lo); }
};

__device__ inline double sfm(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float sfm(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// s^z eigenvalue of local site l in basis state p (site 0 the bit 8)
template <typename R>
__device__ inline R zl(int p, int l) {
  return (p & (8 >> l)) ? R(-1) : R(1);
}

// diagonal energy of basis state p: J sum over the bonds (0,1), (0,2), (1,3),
// (2,3) of z_l z_m, then the fields, in the order of the per-stage kernels
template <typename R>
__device__ inline R energy(int p, R J, const R F[4]) {
  R e = 0;
  e = sfm(J, zl<R>(p, 0) * zl<R>(p, 1), e);
  e = sfm(J, zl<R>(p, 0) * zl<R>(p, 2), e);
  e = sfm(J, zl<R>(p, 1) * zl<R>(p, 3), e);
  e = sfm(J, zl<R>(p, 2) * zl<R>(p, 3), e);
#pragma unroll
  for (int l = 0; l < 4; ++l) e = sfm(F[l], zl<R>(p, l), e);
  return e;
}

// value of lane L ^ M.  M = 1, 2 (quad permutations), 8 (rotation of a
// 16-lane row by 8) and 4 (row shifts by 4 into alternate banks of 4 lanes)
// are DPP moves; 16 and 32 cross rows and go through ds_bpermute.
template <int CTRL, int BANK>
__device__ inline int dpp_x(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xF, BANK, false);
}
template <int M>
__device__ inline int xlane_i(int v) {
  if constexpr (M == 1) return dpp_x<0xB1, 0xF>(v, v);          // quad_perm [1,0,3,2]
  else if constexpr (M == 2) return dpp_x<0x4E, 0xF>(v, v);     // quad_perm [2,3,0,1]
  else if constexpr (M == 8) return dpp_x<0x128, 0xF>(v, v);    // row_ror:8
  else if constexpr (M == 4) {
    const int t = dpp_x<0x114, 0xA>(v, v);                       // banks 1, 3 <- lane - 4
    return dpp_x<0x104, 0x5>(t, v);                              // banks 0, 2 <- lane + 4
  } else {
    return __shfl_xor(v, M);
  }
}
template <int M>
__device__ inline float xlane_r(float v) {
  return __int_as_float(xlane_i<M>(__float_as_int(v)));
}
template <int M>
__device__ inline double xlane_r(double v) {
  return __hiloint2double(xlane_i<M>(__double2hiint(v)), xlane_i<M>(__double2loint(v)));
}
template <int M, typename R>
__device__ inline cpx<R> xlane(const cpx<R>& v) {
  return cmake(xlane_r<M>(v.re), xlane_r<M>(v.im));
}

template <typename R>
__global__ void __launch_bounds__(SNT) k_spin_fused(SpinFusedArgs<R> a) {
  constexpr int WPR = SWords<R>::per_real;
  __shared__ R sPart[4][SD];   // z_l(p) Y[p][p] of the 16 diagonal entries
  __shared__ R sE[SD];         // diagonal energies E_p of this stage

  const int lane = threadIdx.x;
  const int p = lane >> 2, jq = lane & 3;         // row p, columns 4 jq .. 4 jq + 3
  const bool diag = jq == (p >> 2);               // this lane holds Y[p][p] at c = p & 3
  const int dc = p & 3;
  const int g = blockIdx.x / a.nc;
  const int mu = blockIdx.x % a.nc;
  R J = a.J, h = a.h;
  const R dt = a.dt;
  const int* legs = a.legs + mu * 16;
  uint64_t* xout = a.xch + ((size_t)g * a.nc + mu) * 32;

  // lane -> leg e = 4 l + dir (lane / WPR) and payload word w (lane % WPR)
  const int pe = lane / WPR, pw = lane % WPR;
  const int pnb = pe < 16 ? legs[pe] : -1;
  uint64_t* const psrc = pnb >= 0 ? a.xch + ((size_t)g * a.nc + (pnb >> 2)) * 32 + (pnb & 3) * WPR + pw : nullptr;
  uint32_t leg_mask = 0;
#pragma unroll
  for (int e = 0; e < 16; ++e) leg_mask |= (legs[e] >= 0 ? 1u : 0u) << e;

  bool bail = false;
  uint32_t tag = 0;
  auto load_word = [&](uint32_t want) -> uint64_t {
    return psrc ? __hip_atomic_load(psrc + (want & 1) * 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
  };
  // spin until every leg word carries tag `want` (`first`: an issued load of
  // this lane's word); returns this lane's payload
  auto poll = [&](uint32_t want, uint64_t first) -> uint32_t {
    if (bail) return 0u;
    bool done = psrc == nullptr || (uint32_t)(first >> 32) == want;
    uint32_t payload = (uint32_t)first;
    int spins = 0;
    // two loads in flight: the next one is issued before the older one is
    // looked at, so a word that lands just after a load was issued is seen
    // about half a round trip sooner
    uint64_t next = done ? 0 : load_word(want);
    while (!__all(done)) {
      if (++spins > a.spin_limit) {
        if (lane == 0) atomicOr(a.status, 1);
        bail = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      const uint64_t cur = next;
      if (!done) next = load_word(want);
      if (!done && (uint32_t)(cur >> 32) == want) {
        done = true;
        payload = (uint32_t)cur;
      }
    }
    return payload;
  };
  // F_l = J * sum over the present legs of site l (directions in order)
  auto fields = [&](uint32_t payload, R F[4]) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      R f = 0;
#pragma unroll
      for (int dir = 0; dir < 4; ++dir) {
        const int e = 4 * l + dir;
        if (leg_mask & (1u << e)) {
          const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)payload, e * WPR);
          const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)payload, e * WPR + WPR - 1);
          f += SWords<R>::join(lo, hi);
        }
      }
      F[l] = J * f;
    }
  };
  // b_l = sum_p z_l(p) Re Y[p][p] in lane l (l < 4), p in order
  auto site_b = [&](const cpx<R> y[4]) -> R {
    const R v = dc == 0 ? y[0].re : (dc == 1 ? y[1].re : (dc == 2 ? y[2].re : y[3].re));
    __syncthreads();
    if (diag) {
#pragma unroll
      for (int l = 0; l < 4; ++l) sPart[l][p] = zl<R>(p, l) * v;
    }
    __syncthreads();
    R b = 0;
    if (lane < 4) {
#pragma unroll
      for (int q = 0; q < SD; ++q) b += sPart[lane][q];
    }
    return b;
  };
  // publish b_l (held by lane l) as tagged words
  auto publish = [&](R b, uint32_t tg) {
    const int l = lane / WPR, w = lane % WPR;
    const R v = __shfl(b, lane < 4 * WPR ? l : 0);
    if (lane < 4 * WPR) {
      const uint64_t word = ((uint64_t)tg << 32) | SWords<R>::half(v, w);
      __hip_atomic_store(&xout[(tg & 1) * 16 + l * WPR + w], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };

  // Y and the RK4 sum S in registers; rho_n and the stage derivative K in
  // LDS, entry-major (entry c of lane L at c * 64 + L, so that a load
  // instruction touches consecutive banks).  With all of them in registers
  // the FP64 kernel needs ~200 VGPRs and runs two waves per SIMD; this
  // split runs four, which hides more of the neighbours' round trip.
  cpx<R> y[4], ss[4];
  __shared__ cpx<R> sRR[4 * SNT], sK[4 * SNT];
  for (int64_t round = 0;; ++round) {
    const int64_t t = round * a.G + g;
    if (t >= a.n_traj) break;
    cpx<R>* rho = a.rho + ((size_t)t * a.nc + mu) * SD * SD + p * SD + 4 * jq;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      y[c] = rho[c];
      sRR[c * SNT + lane] = y[c];
      ss[c] = cmake(R(0), R(0));
    }
    const R b0 = site_b(y);
    if (round > 0) {
      // the neighbours' last words of the previous trajectory: once seen,
      // they have consumed ours and the slots may be reused
      (void)poll(tag + 1, load_word(tag + 1));
      ++tag;
    }
    publish(b0, tag + 1);
    uint64_t pre = load_word(tag + 1);

    const int total_stages = 4 * a.n_steps;
    for (int st = 0; st < total_stages; ++st) {
      const int stage = st & 3;
      if (a.sched) {
        // stage 1 at t, stages 2 and 3 at t + dt/2, stage 4 at t + dt
        const int hs = 2 * (st >> 2) + (stage == 0 ? 0 : (stage == 3 ? 2 : 1));
        J = a.sJ[hs];
        h = a.sH[hs];
      }
      R F[4];
      fields(poll(tag + 1, pre), F);
      if (bail) break;
      // the diagonal energies of the 16 basis states, one per lane, shared
      // through LDS
      if (lane < SD) sE[lane] = energy<R>(lane, J, F);
      __syncthreads();
      const R ep = sE[p];
      const R hin = stage == 2 ? dt : R(0.5) * dt;
      const R h6 = dt / R(6);
      // S = sa S + sb K, rho_n += sc S, Y = rho_n + sy K
      const R sa = stage == 0 ? R(0) : R(1), sb = (stage == 1 || stage == 2) ? R(2) : R(1);
      const R sc = stage == 3 ? h6 : R(0), sy = stage < 3 ? hin : R(0);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const cpx<R> y0 = y[c];
        // sum over sites l of Y[p ^ bit_l][q] - Y[p][q ^ bit_l], l in order,
        // each pair added as soon as it is exchanged
        R sr = 0, si = 0;
        auto acc = [&](const cpx<R>& u, const cpx<R>& v) {
          sr += u.re - v.re;
          si += u.im - v.im;
        };
        acc(xlane<32>(y0), xlane<2>(y0));
        acc(xlane<16>(y0), xlane<1>(y0));
        acc(xlane<8>(y0), y[c ^ 2]);
        acc(xlane<4>(y0), y[c ^ 1]);
        const R de = ep - sE[4 * jq + c];
        const R xr = sfm(de, y0.re, h * sr), xi = sfm(de, y0.im, h * si);
        sK[c * SNT + lane] = cmake(xi, -xr);   // K = -i [H, Y]
        // one entry at a time: the exchanged values of all four entries at
        // once would cost registers, and occupancy hides the latencies
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const cpx<R> kc = sK[c * SNT + lane];
        cpx<R> sv = ss[c], rv = sRR[c * SNT + lane];
        sv.re = sfm(sb, kc.re, sa * sv.re);
        sv.im = sfm(sb, kc.im, sa * sv.im);
        rv.re = sfm(sc, sv.re, rv.re);
        rv.im = sfm(sc, sv.im, rv.im);
        y[c].re = sfm(sy, kc.re, rv.re);
        y[c].im = sfm(sy, kc.im, rv.im);
        ss[c] = sv;
        if (stage == 3) sRR[c * SNT + lane] = rv;
      }
      ++tag;
      publish(site_b(y), tag + 1);
      pre = load_word(tag + 1);
    }
    if (bail) {
      // poison this cluster so that a timed-out call cannot pass unnoticed
      const R nan = __builtin_nan("");
#pragma unroll
      for (int c = 0; c < 4; ++c) rho[c] = cmake(nan, nan);
      break;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) rho[c] = sRR[c * SNT + lane];
  }
}

template <typename R>
static hipError_t spin_fused_launch(const Geom& g, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                                    double dt, int n_steps, int spin_limit, const double* sJ, const double* sH,
                                    hipStream_t s) {
  if (sJ && n_steps > kSchedSteps) return hipErrorInvalidValue;
  SpinFusedArgs<R> a{};
  a.rho = (cpx<R>*)rho;
  a.xch = xch;
  a.status = status;
  a.legs = legs;
  a.n_traj = g.n_traj;
  a.nc = g.nc;
  a.G = G;
  a.n_steps = n_steps;
  a.J = (R)g.J;
  a.h = (R)g.h;
  a.dt = (R)dt;
  a.spin_limit = spin_limit;
  a.sched = sJ ? 1 : 0;
  if (sJ)
    for (int i = 0; i <= 2 * n_steps; ++i) {
      a.sJ[i] = (R)sJ[i];
      a.sH[i] = (R)sH[i];
    }
  void* args[] = {&a};
  return hipLaunchCooperativeKernel((const void*)k_spin_fused<R>, dim3((unsigned)(g.nc * G)), dim3(SNT), args, 0, s);
}

}  // namespace

bool spin_fused_supported(int model, int d, int cx, int cy) { return model == 1 && d == 2 && cx == 2 && cy == 2; }

// Largest number of trajectories the fused spin kernel can keep resident at
// once for nc clusters each (0 if not even one fits).
int spin_fused_slots(int nc, int dtype) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* f = dtype == 1 ? (const void*)k_spin_fused<double> : (const void*)k_spin_fused<float>;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, SNT, 0);
  if (e != hipSuccess || per_cu <= 0) return 0;
  return (cus * per_cu) / nc;
}

hipError_t spin_fused_rk4(const Geom& g, int dtype, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                          double dt, int n_steps, int spin_limit, const double* sJ, const double* sH,
                          bool zero_status, hipStream_t s) {
  hipError_t e = fused_zero_words(xch, fused_exchange_words(g.nc, G), zero_status ? status : nullptr, s);
  if (e != hipSuccess) return e;
  return dtype == 1 ? spin_fused_launch<double>(g, rho, xch, status, legs, G, dt, n_steps, spin_limit, sJ, sH, s)
                    : spin_fused_launch<float>(g, rho, xch, status, legs, G, dt, n_steps, spin_limit, sJ, sH, s);
}

}  // namespace cdtwa
