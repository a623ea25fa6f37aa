// Fused persistent RK4 kernel for 2x2 clusters (plaquettes) with d = 3,
// D = 81, at three waves per SIMD.
//
// Cluster row index p = 27 n1 + 9 n2 + 3 n3 + n4 (n_l the occupation digit of
// local site l; sites 1 and 4 sit on a diagonal of the plaquette, so every
// bond joins one of them to site 2 or 3; App. B.1 Gamma^intra).  One
// workgroup of 12 waves owns one cluster of one trajectory for a whole call.
// Column q of the stage matrix Y is split over 9 threads, one per value of
// the two diagonal digits (n1, n4); the thread keeps the 9 rows
// p = 27 n1 + n4 + 3 j, j = 3 n2 + n3, of Y, rho_n and the RK4 sum S in
// registers.  In a wave, 7 columns of 9 lanes each: lane = 9 c + 3 n1 + n4.
//
// Every term of H Y that changes n1 or n4 (the site-1 and site-4 fields and
// all four bonds) is formed by the thread that owns the source row, from its
// own rows only, and moved to the owner of the target row: n4 +- 1 is a lane
// shift by 1 (DPP), n1 +- 1 a shift by 3 (ds_bpermute).  The site-2 and
// site-3 fields and the interaction act within the thread's rows.
//
// A stage (Sec. II Eq. (cluster_mf); App. B.1 Phi^inter and the RK4 remark):
//   1. every wave waits for the neighbour clusters' b of this stage -> phi
//   2. M = (H_C + H_MF) Y on the thread's rows, written to LDS
//   3. K = -i (M - M^+) and the classical RK4 update in registers; waves 0-3
//      form b_l of the next stage matrix from the band of K and publish it
// Mean fields travel between clusters as tagged 64-bit words (stage tag in
// the upper half), double-buffered by tag parity, exactly as in the 27-row
// kernel.
#include "launch.hpp"

namespace cdtwa {

namespace {

constexpr int PD = 81;    // cluster dimension
constexpr int PR = 9;     // rows per thread
constexpr int PNT = 768;  // threads per workgroup (12 waves)
constexpr int PLS = 81;   // LDS row stride (complex entries)
// variant switches, bit 0: FP32, bit 1: FP64
#ifndef PLAQ_UNI
#define PLAQ_UNI 2      // field constants forced into scalar registers
#endif
#ifndef PLAQ_SH4P
#define PLAQ_SH4P 0     // site-4 exchange by ds_bpermute instead of DPP (measured slower)
#endif

template <typename R>
struct PlaqArgs {
  cpx<R>* rho;          // [n_traj][nc][81][81]
  uint64_t* xch;        // [G][nc][2][16] tagged words
  int* status;          // bit 0: neighbour wait timed out
  const int* legs;      // [nc][4][4]: neighbour (cluster*4 + local) of local l in direction dir, -1 if none
  int64_t n_traj;
  int nc, G, n_steps;
  R J, U, dt;
  int spin_limit;
  int sched;                      // 1: J and U of every stage from sJ, sU
  R sJ[kSchedVals], sU[kSchedVals];   // at every half step of this launch
};

__device__ constexpr double sqn(int n) { return n <= 0 ? 0.0 : (n == 1 ? 1.0 : 1.4142135623730951); }
__device__ constexpr int hn(int n) { return n == 2 ? 1 : 0; }   // n (n - 1) / 2 for n <= 2

// lane i <- lane i-1 (wave_shr:1) and lane i <- lane i+1 (wave_shl:1); the
// lane without a source reads 0
__device__ inline int sh_prev_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true); }
__device__ inline int sh_next_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true); }
__device__ inline float sh_prev(float v) { return __int_as_float(sh_prev_i(__float_as_int(v))); }
__device__ inline float sh_next(float v) { return __int_as_float(sh_next_i(__float_as_int(v))); }
__device__ inline double sh_prev(double v) {
  return __hiloint2double(sh_prev_i(__double2hiint(v)), sh_prev_i(__double2loint(v)));
}
__device__ inline double sh_next(double v) {
  return __hiloint2double(sh_next_i(__double2hiint(v)), sh_next_i(__double2loint(v)));
}
// value of lane addr/4 (ds_bpermute)
__device__ inline float perm(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ inline double perm(int addr, double v) {
  return __hiloint2double(__builtin_amdgcn_ds_bpermute(addr, __double2hiint(v)),
                          __builtin_amdgcn_ds_bpermute(addr, __double2loint(v)));
}

__device__ inline double fm(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fm(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// a value that is the same in every lane, moved to scalar registers
__device__ inline float uni(float v) {
  return (PLAQ_UNI & 1) ? __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))) : v;
}
__device__ inline double uni(double v) {
  return (PLAQ_UNI & 2) ? __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                                           __builtin_amdgcn_readfirstlane(__double2loint(v)))
                        : v;
}

template <typename R>
struct PWords;
template <>
struct PWords<double> {
  static constexpr int per_real = 2;
  __device__ static uint32_t half(double v, int w) {
    return (uint32_t)(w == 0 ? __double2loint(v) : __double2hiint(v));
  }
  __device__ static double join(uint32_t lo, uint32_t hi) { return __hiloint2double((int)hi, (int)lo); }
};
template <>
struct PWords<float> {
  static constexpr int per_real = 1;
  __device__ static uint32_t half(float v, int) { return (uint32_t)__float_as_int(v); }
  __device__ static float join(uint32_t lo, uint32_t) { return __int_as_float((int)lo); }
};

// sum over the 64 lanes in a fixed order; the total ends up in lane 63
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, BOUND);
}
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ inline float dpp_r(float v) {
  return __int_as_float(dpp_i<CTRL, ROW_MASK, BOUND>(__float_as_int(v)));
}
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ inline double dpp_r(double v) {
  return __hiloint2double(dpp_i<CTRL, ROW_MASK, BOUND>(__double2hiint(v)),
                          dpp_i<CTRL, ROW_MASK, BOUND>(__double2loint(v)));
}
template <typename R>
__device__ inline R lane_sum(R v) {
  v += dpp_r<0x111, 0xF, true>(v);   // row_shr:1
  v += dpp_r<0x112, 0xF, true>(v);   // row_shr:2
  v += dpp_r<0x114, 0xF, true>(v);   // row_shr:4
  v += dpp_r<0x118, 0xF, true>(v);   // row_shr:8
  v += dpp_r<0x142, 0xA, false>(v);  // row_bcast:15
  v += dpp_r<0x143, 0xC, false>(v);  // row_bcast:31
  return v;
}

template <typename R>
__global__ void __launch_bounds__(PNT, 1) k_plaq(PlaqArgs<R> a) {
  constexpr int WPR = PWords<R>::per_real;
  constexpr int WPB = 2 * WPR;  // words per complex b
  __shared__ cpx<R> sM[PD * PLS];
  __shared__ R sBand[4][4];   // per site: b of rho_n (re, im), RK4 sum of the band of K (re, im)
  __shared__ int sBail;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int grp = lane / 9, blk = lane % 9;
  const int q0 = wave * 7 + grp;
  // lanes without a column of their own (lane 63, and columns past 80 in the
  // last wave) start from 0 and read column 0's K from LDS, so they carry
  // column 0's state minus its value at the start of the round: bounded and
  // finite.  They never store, and what they send reaches only lanes that
  // weight it by 0.
  const bool active = lane < 63 && q0 < PD;
  const int q = active ? q0 : 0;
  const int n1 = blk / 3, n4 = blk % 3;
  const int base = 27 * n1 + n4;                  // row of j = 0
  const int g = blockIdx.x / a.nc;
  const int mu = blockIdx.x % a.nc;
  R U = a.U, mJ = -a.J;
  const R dt = a.dt;
  // receive coefficients: a_1^+ (sqrt n1), a_1 (sqrt(n1+1), n1 <= 1), same for site 4
  const R c1u = R(sqn(n1)), c1d = n1 <= 1 ? R(sqn(n1 + 1)) : R(0);
  const R c4u = R(sqn(n4)), c4d = n4 <= 1 ? R(sqn(n4 + 1)) : R(0);
  const R hd = R(hn(n1) + hn(n4));
  const int addr_m3 = ((lane + 61) & 63) << 2;    // lane - 3
  const int addr_p3 = ((lane + 3) & 63) << 2;     // lane + 3
  const int addr_m1 = ((lane + 63) & 63) << 2;    // lane - 1
  const int addr_p1 = ((lane + 1) & 63) << 2;     // lane + 1
  const int* legs = a.legs + mu * 16;
  uint64_t* xout = a.xch + ((size_t)g * a.nc + mu) * 32;
  if (tid == 0) sBail = 0;
  __syncthreads();

  // polling: lane -> leg e = 4 l + dir (lane / WPB), payload word (lane % WPB)
  const int pe = lane / WPB, pw = lane % WPB;
  const int pnb = pe < 16 ? legs[pe] : -1;
  uint64_t* const psrc = pnb >= 0 ? a.xch + ((size_t)g * a.nc + (pnb >> 2)) * 32 + (pnb & 3) * WPB + pw : nullptr;
  uint32_t leg_mask = 0;
#pragma unroll
  for (int e = 0; e < 16; ++e) leg_mask |= (legs[e] >= 0 ? 1u : 0u) << e;

  // band of site bl = wave (waves 0-3): term i (lane i < 54) is the entry
  // (bqq + bs, bqq) with digit_l(bqq) = bdl, weight sqrt(bdl + 1)
  const int bl = wave < 4 ? wave : 0;
  const int bs = bl == 0 ? 27 : (bl == 1 ? 9 : (bl == 2 ? 3 : 1));
  const int bj = lane < 54 ? lane : 0;
  const int bdl = (bj / bs) % 2;
  const int bqq = (bj / (2 * bs)) * 3 * bs + bdl * bs + bj % bs;
  const R bc = lane < 54 ? R(sqn(bdl + 1)) : R(0);

  cpx<R> y[PR], rr[PR], ss[PR];
  uint32_t tag = 0;

  auto publish = [&](R bre, R bim, uint32_t tg) {
    const R vre = __shfl(bre, 63), vim = __shfl(bim, 63);
    if (lane < WPB) {
      const R comp = (lane / WPR) == 0 ? vre : vim;
      const uint64_t word = ((uint64_t)tg << 32) | PWords<R>::half(comp, lane % WPR);
      __hip_atomic_store(&xout[(tg & 1) * 16 + bl * WPB + lane], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  auto load_word = [&](uint32_t want) -> uint64_t {
    return psrc ? __hip_atomic_load(psrc + (want & 1) * 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
  };
  // spin until every leg word carries tag `want` (`first`: an already issued
  // load of this lane's word); returns this lane's payload, sets sBail on a
  // timeout
  auto poll = [&](uint32_t want, uint64_t first) -> uint32_t {
    bool done = psrc == nullptr || (uint32_t)(first >> 32) == want;
    uint32_t payload = (uint32_t)first;
    int spins = 0;
    while (!__all(done)) {
      if (sBail || ++spins > a.spin_limit) {
        if (lane == 0) {
          atomicOr(a.status, 1);
          sBail = 1;
        }
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      if (!done) {
        const uint64_t word = load_word(want);
        if ((uint32_t)(word >> 32) == want) {
          done = true;
          payload = (uint32_t)word;
        }
      }
    }
    return payload;
  };
  auto leg_value = [&](uint32_t payload, int e, int comp) -> R {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)payload, e * WPB + comp * WPR);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)payload, e * WPB + comp * WPR + WPR - 1);
    return PWords<R>::join(lo, hi);
  };
  auto gather_phi = [&](uint32_t payload, cpx<R> phi[4]) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      R pr = 0, pi = 0;
#pragma unroll
      for (int dir = 0; dir < 4; ++dir) {
        const int e = 4 * l + dir;
        if (leg_mask & (1u << e)) {
          pr += leg_value(payload, e, 0);
          pi += leg_value(payload, e, 1);
        }
      }
      phi[l] = cmake(pr, pi);
    }
  };

  for (int64_t round = 0;; ++round) {
    const int64_t t = round * a.G + g;
    if (t >= a.n_traj) break;
    cpx<R>* rho = a.rho + ((size_t)t * a.nc + mu) * PD * PD;
#pragma unroll
    for (int j = 0; j < PR; ++j) {
      rr[j] = active ? rho[(base + 3 * j) * PD + q] : cmake(R(0), R(0));
      y[j] = rr[j];
      ss[j] = cmake(R(0), R(0));
    }
    // b_l(rho) from the band of rho in global memory (waves 0-3)
    if (wave < 4) {
      const cpx<R> v = rho[(bqq + bs) * PD + bqq];
      const R br = lane_sum(bc * v.re), bi = lane_sum(bc * v.im);
      if (lane == 63) {
        sBand[bl][0] = br;
        sBand[bl][1] = bi;
      }
    }
    if (round > 0) {
      // the neighbours' last words of the previous trajectory: once seen, they
      // have consumed ours and the slots may be reused
      (void)poll(tag + 1, load_word(tag + 1));
      ++tag;
      // every wave must have seen those words before any wave publishes the
      // next ones: a neighbour that sees them may run a stage and overwrite
      // the slot a slower wave here is still waiting on
      __syncthreads();
    }
    if (wave < 4) publish(sBand[bl][0], sBand[bl][1], tag + 1);
    uint64_t pre = load_word(tag + 1);

    const int total_stages = 4 * a.n_steps;
    for (int st = 0; st < total_stages; ++st) {
      const int stage = st & 3;
      if (a.sched) {
        // stage 1 at t, stages 2 and 3 at t + dt/2, stage 4 at t + dt
        const int hs = 2 * (st >> 2) + (stage == 0 ? 0 : (stage == 3 ? 2 : 1));
        mJ = -a.sJ[hs];
        U = a.sU[hs];
      }
      // ---- 1. neighbour mean fields of this stage
      cpx<R> phi[4];
      gather_phi(poll(tag + 1, pre), phi);
      // -J phi_l; the site-2 and site-3 field terms with their sqrt(n) factors
      // (wave-uniform: kept in scalar registers)
      const R sq2 = R(1.4142135623730951);
      const cpx<R> P1 = cmake(uni(mJ * phi[0].re), uni(mJ * phi[0].im));
      const cpx<R> P4 = cmake(uni(mJ * phi[3].re), uni(mJ * phi[3].im));
      const cpx<R> P2[3] = {cmake(R(0), R(0)), cmake(uni(mJ * phi[1].re), uni(mJ * phi[1].im)),
                            cmake(uni(sq2 * mJ * phi[1].re), uni(sq2 * mJ * phi[1].im))};
      const cpx<R> P3[3] = {cmake(R(0), R(0)), cmake(uni(mJ * phi[2].re), uni(mJ * phi[2].im)),
                            cmake(uni(sq2 * mJ * phi[2].re), uni(sq2 * mJ * phi[2].im))};
      // ---- 2. M = H Y on the thread's rows
#pragma unroll
      for (int j = 0; j < PR; ++j) {
        const int n2 = j / 3, n3 = j % 3;
        const cpx<R> v = y[j];
        // bond parts shared by the site-1 and site-4 terms: raising (a_l^+ a_2,
        // a_l^+ a_3) and lowering (a_2^+ a_l, a_3^+ a_l), times -J
        R bur = 0, bui = 0, bdr = 0, bdi = 0;
        if (n2 <= 1) { const R c = mJ * R(sqn(n2 + 1)); bur = c * y[j + 3].re; bui = c * y[j + 3].im; }
        if (n3 <= 1) { const R c = mJ * R(sqn(n3 + 1)); bur = fm(c, y[j + 1].re, bur); bui = fm(c, y[j + 1].im, bui); }
        if (n2 >= 1) { const R c = mJ * R(sqn(n2)); bdr = c * y[j - 3].re; bdi = c * y[j - 3].im; }
        if (n3 >= 1) { const R c = mJ * R(sqn(n3)); bdr = fm(c, y[j - 1].re, bdr); bdi = fm(c, y[j - 1].im, bdi); }
        // V_l = Bu + P_l v (sent to n_l + 1), W_l = Bd + conj(P_l) v (sent to n_l - 1)
        R v1r = fm(P1.re, v.re, bur), v1i = fm(P1.re, v.im, bui);
        v1r = fm(-P1.im, v.im, v1r);
        v1i = fm(P1.im, v.re, v1i);
        R w1r = fm(P1.re, v.re, bdr), w1i = fm(P1.re, v.im, bdi);
        w1r = fm(P1.im, v.im, w1r);
        w1i = fm(-P1.im, v.re, w1i);
        R v4r = fm(P4.re, v.re, bur), v4i = fm(P4.re, v.im, bui);
        v4r = fm(-P4.im, v.im, v4r);
        v4i = fm(P4.im, v.re, v4i);
        R w4r = fm(P4.re, v.re, bdr), w4i = fm(P4.re, v.im, bdi);
        w4r = fm(P4.im, v.im, w4r);
        w4i = fm(-P4.im, v.re, w4i);
        const R x1r = perm(addr_m3, v1r), x1i = perm(addr_m3, v1i);   // from n1 - 1
        const R z1r = perm(addr_p3, w1r), z1i = perm(addr_p3, w1i);   // from n1 + 1
        R x4r, x4i, z4r, z4i;                                         // from n4 -+ 1
        if (PLAQ_SH4P & (sizeof(R) == 8 ? 2 : 1)) {
          x4r = perm(addr_m1, v4r);
          x4i = perm(addr_m1, v4i);
          z4r = perm(addr_p1, w4r);
          z4i = perm(addr_p1, w4i);
        } else {
          x4r = sh_prev(v4r);
          x4i = sh_prev(v4i);
          z4r = sh_next(w4r);
          z4i = sh_next(w4i);
        }
        // interaction
        const R dg = U * (hd + R(hn(n2) + hn(n3)));
        R mr = dg * v.re, mi = dg * v.im;
        // site-2 and site-3 fields: conj(P) sqrt(n+1) y[n+e] + P sqrt(n) y[n-e]
        // (P[k] = sqrt(k) (-J phi))
#define CDTWA_PFIELD(P, N, S)                                                      \
  if (N <= 1) {                                                                    \
    const cpx<R> f = P[N + 1];                                                     \
    const cpx<R> u = y[j + S];                                                     \
    mr = fm(f.re, u.re, mr);                                                       \
    mr = fm(f.im, u.im, mr);                                                       \
    mi = fm(f.re, u.im, mi);                                                       \
    mi = fm(-f.im, u.re, mi);                                                      \
  }                                                                                \
  if (N >= 1) {                                                                    \
    const cpx<R> f = P[N];                                                         \
    const cpx<R> u = y[j - S];                                                     \
    mr = fm(f.re, u.re, mr);                                                       \
    mr = fm(-f.im, u.im, mr);                                                      \
    mi = fm(f.re, u.im, mi);                                                       \
    mi = fm(f.im, u.re, mi);                                                       \
  }
        CDTWA_PFIELD(P2, n2, 3)
        CDTWA_PFIELD(P3, n3, 1)
#undef CDTWA_PFIELD
        // terms that changed n1 or n4, received from the neighbouring blocks
        mr = fm(c1u, x1r, mr);
        mi = fm(c1u, x1i, mi);
        mr = fm(c1d, z1r, mr);
        mi = fm(c1d, z1i, mi);
        mr = fm(x4r, c4u, mr);
        mi = fm(x4i, c4u, mi);
        mr = fm(z4r, c4d, mr);
        mi = fm(z4i, c4d, mi);
        if (active) sM[(base + 3 * j) * PLS + q] = cmake(mr, mi);
        __builtin_amdgcn_sched_barrier(0);
      }
      __syncthreads();
      if (sBail) break;
      ++tag;
      const R hin = stage == 2 ? dt : R(0.5) * dt;
      const R h6 = dt / R(6);
      // ---- 3. b_l of the next stage matrix from the band of K (waves 0-3);
      // lane 63 holds the sums and keeps the running values in LDS
      if (wave < 4) {
        const cpx<R> mpq = sM[(bqq + bs) * PLS + bqq], mqp = sM[bqq * PLS + bqq + bs];
        const R kr = lane_sum(bc * (mpq.im + mqp.im));
        const R ki = lane_sum(bc * (mqp.re - mpq.re));
        R nr = 0, ni = 0;
        if (lane == 63) {
          const R bRr = sBand[bl][0], bRi = sBand[bl][1];
          R bSr = sBand[bl][2], bSi = sBand[bl][3];
          if (stage == 0) {
            bSr = kr;
            bSi = ki;
          } else if (stage < 3) {
            bSr = fm(R(2), kr, bSr);
            bSi = fm(R(2), ki, bSi);
          }
          if (stage < 3) {
            nr = fm(hin, kr, bRr);
            ni = fm(hin, ki, bRi);
          } else {
            nr = fm(h6, bSr + kr, bRr);
            ni = fm(h6, bSi + ki, bRi);
            sBand[bl][0] = nr;
            sBand[bl][1] = ni;
          }
          sBand[bl][2] = bSr;
          sBand[bl][3] = bSi;
        }
        publish(nr, ni, tag + 1);
      }
      // ---- K = -i (M - M^+) and the classical RK4 update
#pragma unroll
      for (int j = 0; j < PR; ++j) {
        // K[p][q] = -i (M[p][q] - conj(M[q][p]))
        const cpx<R> m0 = sM[(base + 3 * j) * PLS + q];
        const cpx<R> m1 = sM[q * PLS + base + 3 * j];
        const R kr = m0.im + m1.im, ki = m1.re - m0.re;
        if (stage == 0) {
          ss[j] = cmake(kr, ki);
        } else if (stage < 3) {
          ss[j].re = fm(R(2), kr, ss[j].re);
          ss[j].im = fm(R(2), ki, ss[j].im);
        }
        if (stage < 3) {
          y[j].re = fm(hin, kr, rr[j].re);
          y[j].im = fm(hin, ki, rr[j].im);
        } else {
          rr[j].re = fm(h6, ss[j].re + kr, rr[j].re);
          rr[j].im = fm(h6, ss[j].im + ki, rr[j].im);
          y[j] = rr[j];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      pre = load_word(tag + 1);
      __syncthreads();
    }
    if (sBail) {
      // poison this cluster so that a timed-out call cannot pass unnoticed
      const R nan = __builtin_nan("");
#pragma unroll
      for (int j = 0; j < PR; ++j)
        if (active) rho[(base + 3 * j) * PD + q] = cmake(nan, nan);
      break;
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < PR; ++j) rho[(base + 3 * j) * PD + q] = rr[j];
    }
  }
}

}  // namespace

// Largest number of trajectories the plaquette kernel keeps resident at once
// for nc clusters each (0 if not even one fits).
int plaq_slots(int nc, int dtype) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e = dtype == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_plaq<double>, PNT, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_plaq<float>, PNT, 0);
  if (e != hipSuccess || per_cu <= 0) return 0;
  return (cus * per_cu) / nc;
}

template <typename R>
static hipError_t plaq_launch(const Geom& g, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                             double dt, int n_steps, int spin_limit, const double* sJ, const double* sU,
                             hipStream_t s) {
  if (sJ && n_steps > kSchedSteps) return hipErrorInvalidValue;
  PlaqArgs<R> a{};
  a.rho = (cpx<R>*)rho;
  a.xch = xch;
  a.status = status;
  a.legs = legs;
  a.n_traj = g.n_traj;
  a.nc = g.nc;
  a.G = G;
  a.n_steps = n_steps;
  a.J = (R)g.J;
  a.U = (R)g.U;
  a.dt = (R)dt;
  a.spin_limit = spin_limit;
  a.sched = sJ ? 1 : 0;
  if (sJ)
    for (int i = 0; i <= 2 * n_steps; ++i) {
      a.sJ[i] = (R)sJ[i];
      a.sU[i] = (R)sU[i];
    }
  void* args[] = {&a};
  return hipLaunchCooperativeKernel((const void*)k_plaq<R>, dim3((unsigned)(g.nc * G)), dim3(PNT), args, 0, s);
}

hipError_t plaq_rk4(const Geom& g, int dtype, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                    double dt, int n_steps, int spin_limit, const double* sJ, const double* sU, bool zero_status,
                    hipStream_t s) {
  hipError_t e = fused_zero_words(xch, fused_exchange_words(g.nc, G), zero_status ? status : nullptr, s);
  if (e != hipSuccess) return e;
  return dtype == 1 ? plaq_launch<double>(g, rho, xch, status, legs, G, dt, n_steps, spin_limit, sJ, sU, s)
                    : plaq_launch<float>(g, rho, xch, status, legs, G, dt, n_steps, spin_limit, sJ, sU, s);
}

}  // namespace cdtwa
