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
//   A. every wave waits for the neighbours' tagged words of this stage and
//      forms the fields phi of the four sites
//   B. M = H Y on the thread's own rows: interaction, the hops among sites
//      2, 3, 4 and their fields; the terms that move the site-1 digit are
//      formed by the neighbouring block and shifted in with DPP lane shifts;
//      M is written to LDS
//   C. after a barrier, K = -i (M - M^+) from LDS and the classical RK4
//      update in registers (one loop per kind of stage)
//   D. wave l forms b_l of the next stage matrix from the band of K and
//      publishes it, early in C so that the neighbours' wait is short
//
// With local Lindblad channels (the extension named in Sec. IV and App. B.1;
// dephasing L = n_j and loss L = a_j on every site) the dissipator D(Y)
// enters through M: adding (i/2) D(Y) to M adds (D + D^+)/2 = D to
// K = -i (M - M^+), since D maps a Hermitian Y to a Hermitian matrix.  Its
// diagonal part is local to a thread's entries; the jump terms
// gamma_loss sqrt((n_l(p)+1)(n_l(q)+1)) Y[p+s_l][q+s_l] read the stage matrix
// from a second LDS array that holds its lower triangle, written during the
// update of the previous stage.
#include <cstring>
#include <type_traits>

#include "launch.hpp"

namespace cdtwa {

namespace {

constexpr int FD = 81;     // cluster dimension
constexpr int FB = 27;     // rows per thread
constexpr int FNT = 256;   // threads per workgroup
constexpr int LS = 81;     // LDS row stride (complex entries)
constexpr int FT = FD * (FD + 1) / 2;   // lower triangle p >= q, row-major: (p, q) -> p (p + 1) / 2 + q

// One member problem of a batch launch: its state, exchange words and
// neighbour table, trajectory and cluster counts, the G gangs of nc
// workgroups it owns (workgroups slot0 .. slot0 + G nc - 1) and couplings.
template <typename R>
struct FusedMember {
  cpx<R>* rho;
  uint64_t* xch;
  const int* legs;
  int64_t n_traj;
  int nc, G, slot0;
  R J, U;
};

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
  R gd, gl;             // dephasing and loss rates (the DISS kernel only)
  int sched;                      // 1: J and U of every stage from sJ, sU
  R sJ[kSchedVals], sU[kSchedVals];   // at every half step of this launch
  const FusedMember<R>* members;   // batch launch: the member table (else unused)
  int n_members;
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

__device__ inline double fm(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fm(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Sum over the 64 lanes of a wave in a fixed order (DPP row shifts, then the
// row broadcasts); the total ends up in lane 63.
__device__ inline float wave_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));  // row_shr:1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));  // row_shr:2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));  // row_shr:4
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));  // row_shr:8
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false)); // row_bcast:15
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false)); // row_bcast:31
  return v;
}
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ inline double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, BOUND);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, BOUND);
  return __hiloint2double(hi, lo);
}
__device__ inline double wave_sum(double v) {
  v += dpp_d<0x111, 0xF, true>(v);
  v += dpp_d<0x112, 0xF, true>(v);
  v += dpp_d<0x114, 0xF, true>(v);
  v += dpp_d<0x118, 0xF, true>(v);
  v += dpp_d<0x142, 0xA, false>(v);
  v += dpp_d<0x143, 0xC, false>(v);
  return v;
}

// a value read from memory that is the same in every lane, in scalar registers
__device__ inline int64_t uniform_i64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ inline const void* uniform_ptr(const void* p) { return (const void*)uniform_i64((int64_t)p); }
__device__ inline float uniform_real(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ inline double uniform_real(double v) { return __longlong_as_double(uniform_i64(__double_as_longlong(v))); }

// One workgroup per cluster (one per compute unit in FP64, two in FP32).
// WPC: workgroups per CU the register budget is sized for (one in FP64, two
// in FP32; three in FP32 for lattices whose clusters do not fit at two).
// MULTI: a batch launch, the workgroups split into the gangs of several
// member problems (closed systems, constant couplings); each workgroup takes
// its member's parameters from the table and runs the same body.
template <typename R, bool DISS, int WPC = (sizeof(R) == 8 ? 1 : 2), bool MULTI = false>
__global__ void __launch_bounds__(FNT, WPC) k_fused(FusedArgs<R> a) {
  constexpr int WPR = Words<R>::per_real;
  constexpr int WPB = 2 * WPR;  // words per complex b
  __shared__ cpx<R> sM[FD * LS];      // M = H Y of the current stage
  __shared__ cpx<R> sT[DISS ? FT : 1];  // lower triangle of the stage matrix Y
  __shared__ int sBail;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int q0 = wave * 21 + lane / 3;
  const bool active = lane < 63 && q0 < FD;
  const int q = active ? q0 : FD - 1;
  const int k = lane % 3;
  unsigned blk = blockIdx.x;
  cpx<R>* rho_all = a.rho;
  uint64_t* xch = a.xch;
  const int* legs_all = a.legs;
  int64_t n_traj = a.n_traj;
  int nc = a.nc, G = a.G;
  R J = a.J, U = a.U;
  if constexpr (MULTI) {
    // the member of this workgroup; every value is uniform over the
    // workgroup and is kept in scalar registers
    int m = 0;
    while (m + 1 < a.n_members && blk >= (unsigned)a.members[m + 1].slot0) ++m;
    m = __builtin_amdgcn_readfirstlane(m);
    const FusedMember<R>& e = a.members[m];
    blk -= (unsigned)__builtin_amdgcn_readfirstlane(e.slot0);
    rho_all = (cpx<R>*)uniform_ptr(e.rho);
    xch = (uint64_t*)uniform_ptr(e.xch);
    legs_all = (const int*)uniform_ptr(e.legs);
    n_traj = uniform_i64(e.n_traj);
    nc = __builtin_amdgcn_readfirstlane(e.nc);
    G = __builtin_amdgcn_readfirstlane(e.G);
    J = uniform_real(e.J);
    U = uniform_real(e.U);
  }
  const int g = blk / nc;
  const int mu = blk % nc;
  const R dt = a.dt;
  const R hk = (k == 2) ? R(1) : R(0);                  // h(n1) = n1 (n1-1)/2
  R jdn = k <= 1 ? -J * R(sq(k + 1)) : R(0);            // scale of what block k+1 sends
  R jup = -J * R(sq(k));                                 // scale of what block k-1 sends
  const int* legs = legs_all + mu * 16;
  uint64_t* xout = xch + ((size_t)g * nc + mu) * 32;
  cpx<R>* const mown = sM + (27 * k) * LS + q;           // M[27k + r][q] = mown[r * LS]
  const cpx<R>* const mtr = sM + q * LS + 27 * k;        // M[q][27k + r] = mtr[r]
  if (tid == 0) sBail = 0;
  __syncthreads();

  // Every wave polls all neighbour legs itself: lane -> leg e = 4 l + dir
  // (lane / WPB) and payload word w (lane % WPB).
  const int pe = lane / WPB, pw = lane % WPB;
  const int pnb = pe < 16 ? legs[pe] : -1;
  uint64_t* const psrc = pnb >= 0 ? xch + ((size_t)g * nc + (pnb >> 2)) * 32 + (pnb & 3) * WPB + pw : nullptr;
  uint32_t leg_mask = 0;
#pragma unroll
  for (int e = 0; e < 16; ++e) leg_mask |= (legs[e] >= 0 ? 1u : 0u) << e;

  // Site whose mean field this wave publishes: l = wave.  Band term j (lane
  // j < 54) of site l is the entry (qq + s_l, qq) with digit_l(qq) = dl.
  const int bl = wave;
  const int bs = bl == 0 ? 27 : (bl == 1 ? 9 : (bl == 2 ? 3 : 1));
  const int bj = lane < 54 ? lane : 0;
  const int bdl = (bj / bs) % 2;
  const int bqq = (bj / (2 * bs)) * 3 * bs + bdl * bs + bj % bs;
  const R bc = lane < 54 ? R(sq(bdl + 1)) : R(0);

  // Dissipator (DISS): rows p = 27k + r of column q; the lower triangle of
  // Y sits at T(p) + q for p >= q, T(x) = x (x+1) / 2.  Every index and
  // coefficient is derived from opaque copies of q and k where it is used:
  // kept live across the whole kernel they do not fit in registers.
  auto tri_row0 = [](int qq, int kk) { return (27 * kk) * (27 * kk + 1) / 2 + qq; };   // T(27k) + q
  const R gd4 = R(0.25) * a.gd, gl4 = R(0.25) * a.gl, gl2 = R(0.5) * a.gl;
  (void)tri_row0; (void)gd4; (void)gl4; (void)gl2;

  cpx<R> y[FB], rr[FB], ss[FB];
  uint32_t tag = 0;

  // publish b_l (valid in lane 63 after wave_sum) as tagged words
  auto publish = [&](R bre, R bim, uint32_t tg) {
    const R vre = __shfl(bre, 63), vim = __shfl(bim, 63);
    if (lane < WPB) {
      const R comp = (lane / WPR) == 0 ? vre : vim;
      const uint64_t word = ((uint64_t)tg << 32) | Words<R>::half(comp, lane % WPR);
      __hip_atomic_store(&xout[(tg & 1) * 16 + bl * WPB + lane], word, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  auto load_word = [&](uint32_t want) -> uint64_t {
    return psrc ? __hip_atomic_load(psrc + (want & 1) * 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
  };
  // spin until every leg word carries tag `want` (`first` is an already
  // issued load of this lane's word); returns this lane's payload
  auto poll = [&](uint32_t want, uint64_t first) -> uint32_t {
    if (sBail) return 0u;
    bool done = psrc == nullptr || (uint32_t)(first >> 32) == want;
    uint32_t payload = (uint32_t)first;
    int spins = 0;
    while (!__all(done)) {
      if (++spins > a.spin_limit) {
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
  // phi_l = sum over dir (+x,-x,+y,-y) of the legs of site l present
  auto leg_value = [&](uint32_t payload, int e, int comp) -> R {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)payload, e * WPB + comp * WPR);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)payload, e * WPB + comp * WPR + WPR - 1);
    return Words<R>::join(lo, hi);
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
    const int64_t t = round * G + g;
    if (t >= n_traj) break;
    cpx<R>* rho = rho_all + ((size_t)t * nc + mu) * FD * FD;
    const cpx<R>* rown = rho + (27 * k) * FD + q;
#pragma unroll
    for (int r = 0; r < FB; ++r) {
      rr[r] = rown[r * FD];
      y[r] = rr[r];
      ss[r] = cmake(R(0), R(0));
    }
    if constexpr (DISS) {
      int qo = q, ko = k;
      asm volatile("" : "+v"(qo), "+v"(ko));
      const int t0 = tri_row0(qo, ko), k27 = 27 * ko, qk = qo - k27;
#pragma unroll
      for (int r = 0; r < FB; ++r)
        if (active && r >= qk) sT[t0 + r * k27 + r * (r + 1) / 2] = y[r];
      __syncthreads();
    }
    // b_l(rho) from the band of rho in global memory
    R bRr, bRi, bSr = 0, bSi = 0;
    {
      const cpx<R> v = rho[(bqq + bs) * FD + bqq];
      bRr = wave_sum(bc * v.re);
      bRi = wave_sum(bc * v.im);
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
    publish(bRr, bRi, tag + 1);
    uint64_t pre = load_word(tag + 1);

    const int total_stages = 4 * a.n_steps;
    for (int st = 0; st < total_stages; ++st) {
      const int stage = st & 3;
      const uint32_t want = tag + 1;
      if (a.sched) {
        // stage 1 at t, stages 2 and 3 at t + dt/2, stage 4 at t + dt
        const int hs = 2 * (st >> 2) + (stage == 0 ? 0 : (stage == 3 ? 2 : 1));
        J = a.sJ[hs];
        U = a.sU[hs];
        jdn = k <= 1 ? -J * R(sq(k + 1)) : R(0);
        jup = -J * R(sq(k));
      }
      // ---- neighbour mean fields of this stage
      cpx<R> phi[4];
      gather_phi(poll(want, pre), phi);
      const cpx<R> f0 = phi[0];
      cpx<R> F1[3], F2[3];   // -J c phi_l, c = 1 and sqrt(2), sites 2,3,4
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        F1[l] = cmake(-J * phi[l + 1].re, -J * phi[l + 1].im);
        F2[l] = cmake(R(-1.4142135623730951) * J * phi[l + 1].re, R(-1.4142135623730951) * J * phi[l + 1].im);
      }
      // ---- M = H Y on the thread's rows; the terms that move the site-1
      // digit are formed by the neighbouring block and shifted in with DPP
      if (active) {
        // dissipator terms of this thread, formed afresh in every stage
        int qo = q, ko = k;
        if constexpr (DISS) asm volatile("" : "+v"(qo), "+v"(ko));
        const int c0 = qo / 27, c1 = (qo / 9) % 3, c2 = (qo / 3) % 3, c3 = qo % 3;
        const int k27 = 27 * ko, tlo = tri_row0(qo, ko), qk = qo - k27;
        const int d0sq = (ko - c0) * (ko - c0), d0sum = ko + c0 + c1 + c2 + c3;
        // jump of site l at (p, q): (gl/2) sqrt(n_l(p)+1) sqrt(c_l+1) Y[p+s_l][q+s_l],
        // read as T(p+s_l) + q+s_l for p >= q, else conj of T(q+s_l) + p+s_l
        int thi[4];
        R cj[4];
        {
          const int cl[4] = {c0, c1, c2, c3}, sl[4] = {27, 9, 3, 1};
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            const int b = qo + sl[l];
            thi[l] = cl[l] <= 1 ? b * (b + 1) / 2 + k27 : 0;     // 0 keeps unused reads in range
            cj[l] = cl[l] <= 1 ? (cl[l] == 0 ? gl2 : gl2 * R(1.4142135623730951)) : R(0);
          }
          // site 1 also needs k <= 1 (its row p + 27 exists)
          cj[0] = ko == 0 ? cj[0] : (ko == 1 ? cj[0] * R(1.4142135623730951) : R(0));
        }
        (void)d0sq; (void)d0sum; (void)tlo; (void)qk;
        // FP32: the sending block scales what it sends by the receiver's
        // factor -J sqrt(n_1) -- its own jup for what goes to block k-1, its
        // own jdn for what goes to block k+1 (both 0 where no receiver
        // exists) -- so that the receiver only adds the shifted value, and
        // the lane shift folds into that add (a DPP source operand; a
        // multiply-add cannot take one).  FP64 scales on receipt.
        constexpr bool PRE = sizeof(R) == 4;
        const R sd = PRE ? jup : R(1), su = PRE ? jdn : R(1);
        const cpx<R> fd = cmake(sd * f0.re, sd * f0.im), fu = cmake(su * f0.re, su * f0.im);
        const R dq[3] = {R(0), sd, sd * R(1.4142135623730951)}, uq[3] = {su, su * R(1.4142135623730951), R(0)};
#pragma unroll
        for (int r = 0; r < FB; ++r) {
          const int n2 = r / 9, n3 = (r / 3) % 3, n4 = r % 3;
          // to block k-1 (a_1 there): conj(phi_1) y + a_2^+ y + a_3^+ y
          R dr = fd.re * y[r].re, di = fd.re * y[r].im;
          dr = fm(fd.im, y[r].im, dr);
          di = fm(-fd.im, y[r].re, di);
          if (n2 >= 1) { const R c = dq[n2]; dr = fm(c, y[r - 9].re, dr); di = fm(c, y[r - 9].im, di); }
          if (n3 >= 1) { const R c = dq[n3]; dr = fm(c, y[r - 3].re, dr); di = fm(c, y[r - 3].im, di); }
          // to block k+1 (a_1^+ there): phi_1 y + a_2 y + a_3 y
          R ur = fu.re * y[r].re, ui = fu.re * y[r].im;
          ur = fm(-fu.im, y[r].im, ur);
          ui = fm(fu.im, y[r].re, ui);
          if (n2 <= 1) { const R c = uq[n2]; ur = fm(c, y[r + 9].re, ur); ui = fm(c, y[r + 9].im, ui); }
          if (n3 <= 1) { const R c = uq[n3]; ur = fm(c, y[r + 3].re, ur); ui = fm(c, y[r + 3].im, ui); }
          const R rdr = dpp_next(dr), rdi = dpp_next(di);   // from block k+1
          const R rur = dpp_prev(ur), rui = dpp_prev(ui);   // from block k-1
          // interaction
          const R dg = U * (hk + R((n2 == 2) + (n3 == 2) + (n4 == 2)));
          R mr, mi;
          if constexpr (PRE) {
            mr = rdr + rur;
            mi = rdi + rui;
            mr = fm(dg, y[r].re, mr);
            mi = fm(dg, y[r].im, mi);
          } else {
            mr = dg * y[r].re;
            mi = dg * y[r].im;
            mr = fm(jdn, rdr, mr);
            mi = fm(jdn, rdi, mi);
            mr = fm(jup, rur, mr);
            mi = fm(jup, rui, mi);
          }
          // hops between sites 2-4 (strides 9, 1) and 3-4 (strides 3, 1)
          if (n2 >= 1 && n4 <= 1) { const R c = -J * R(sq(n2) * sq(n4 + 1)); mr = fm(c, y[r - 8].re, mr); mi = fm(c, y[r - 8].im, mi); }
          if (n4 >= 1 && n2 <= 1) { const R c = -J * R(sq(n4) * sq(n2 + 1)); mr = fm(c, y[r + 8].re, mr); mi = fm(c, y[r + 8].im, mi); }
          if (n3 >= 1 && n4 <= 1) { const R c = -J * R(sq(n3) * sq(n4 + 1)); mr = fm(c, y[r - 2].re, mr); mi = fm(c, y[r - 2].im, mi); }
          if (n4 >= 1 && n3 <= 1) { const R c = -J * R(sq(n4) * sq(n3 + 1)); mr = fm(c, y[r + 2].re, mr); mi = fm(c, y[r + 2].im, mi); }
          // fields on sites 2,3,4: -J sqrt(n+1) conj(phi) y[r+s] and -J sqrt(n) phi y[r-s]
#define CDTWA_FIELD(L, N, S)                                                                 \
  if (N <= 1) {                                                                              \
    const cpx<R> F = N == 0 ? F1[L] : F2[L];                                                 \
    const cpx<R> v = y[r + S];                                                               \
    mr = fm(F.re, v.re, mr);                                                                 \
    mr = fm(F.im, v.im, mr);                                                                 \
    mi = fm(F.re, v.im, mi);                                                                 \
    mi = fm(-F.im, v.re, mi);                                                                \
  }                                                                                          \
  if (N >= 1) {                                                                              \
    const cpx<R> F = N == 1 ? F1[L] : F2[L];                                                 \
    const cpx<R> v = y[r - S];                                                               \
    mr = fm(F.re, v.re, mr);                                                                 \
    mr = fm(-F.im, v.im, mr);                                                                \
    mi = fm(F.re, v.im, mi);                                                                 \
    mi = fm(F.im, v.re, mi);                                                                 \
  }
          CDTWA_FIELD(0, n2, 9)
          CDTWA_FIELD(1, n3, 3)
          CDTWA_FIELD(2, n4, 1)
#undef CDTWA_FIELD
          if constexpr (DISS) {
            // (i/2) D(Y): diagonal part -(A/2) i Y with
            // A/2 = gd/4 sum_l (n_l(p) - n_l(q))^2 + gl/4 sum_l (n_l(p) + n_l(q))
            const int dsq = d0sq + (n2 - c1) * (n2 - c1) + (n3 - c2) * (n3 - c2) + (n4 - c3) * (n4 - c3);
            const R ha = fm(gd4, R(dsq), gl4 * R(d0sum + n2 + n3 + n4));
            mr = fm(ha, y[r].im, mr);
            mi = fm(-ha, y[r].re, mi);
            // jumps, times i/2 (the 1/2 is in cj)
            const bool lo = r >= qk;
#define CDTWA_JUMP(L, S, C)                                                                  \
  {                                                                                          \
    const int m = r + S;                                                                     \
    const int ix = lo ? tlo + m * k27 + m * (m + 1) / 2 + S : thi[L] + m;                    \
    const cpx<R> v = sT[L == 0 ? (ko <= 1 ? ix : 0) : ix];                                   \
    const R cc = C * cj[L];                                                                  \
    mr = fm(lo ? -cc : cc, v.im, mr);                                                        \
    mi = fm(cc, v.re, mi);                                                                   \
  }
            CDTWA_JUMP(0, 27, R(1))
            if (n2 <= 1) CDTWA_JUMP(1, 9, R(sq(n2 + 1)))
            if (n3 <= 1) CDTWA_JUMP(2, 3, R(sq(n3 + 1)))
            if (n4 <= 1) CDTWA_JUMP(3, 1, R(sq(n4 + 1)))
#undef CDTWA_JUMP
          }
          mown[r * LS] = cmake(mr, mi);
          // keep the triangle reads of a row with that row (hoisted reads
          // of every row do not fit in registers)
          if constexpr (DISS) __builtin_amdgcn_sched_barrier(0);
        }
      }
      __syncthreads();
      if (sBail) break;   // read after the barrier: the same value in every wave
      ++tag;
      const R hin = stage == 2 ? dt : R(0.5) * dt;
      const R h6 = dt / R(6);
      // ---- wave l forms b_l of the next stage matrix from the band of
      // K = -i (M - M^+) and publishes it (interleaved with the first rows of
      // the update below so that its latency is hidden)
      auto band_publish = [&]() {
        const cpx<R> mpq = sM[(bqq + bs) * LS + bqq], mqp = sM[bqq * LS + bqq + bs];
        const R kr = wave_sum(bc * (mpq.im + mqp.im));
        const R ki = wave_sum(bc * (mqp.re - mpq.re));
        R nr, ni;
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
          bRr = fm(h6, bSr + kr, bRr);
          bRi = fm(h6, bSi + ki, bRi);
          nr = bRr;
          ni = bRi;
        }
        publish(nr, ni, tag + 1);
      };
      // ---- K = -i (M - M^+) and the classical RK4 update.  Rows are
      // processed in order with the LDS reads PF rows ahead (a software
      // pipeline; the scheduling fences keep the compiler from hoisting every
      // read of the loop, which would not fit in registers).
      int qo = q, ko = k;    // opaque copies for the triangle writes
      if constexpr (DISS) asm volatile("" : "+v"(qo), "+v"(ko));
      const int k27_k = 27 * ko, tlo_k = tri_row0(qo, ko), qk_k = qo - k27_k;
      (void)k27_k; (void)tlo_k; (void)qk_k;
      // The loop is instantiated once per kind of stage (KS = 0: the first,
      // 1: the second and third, 3: the last) behind a uniform branch: with
      // a run-time stage the compiler forms every alternative and selects.
      // The dissipator kernel runs one branch-free loop instead (KS = -1)
      // with the RK4 coefficients as uniform values, S = sa S + sb K,
      // rho_n += sc S, Y = rho_n + sy K (the same roundings as the
      // specialised loops): its three specialised copies spill, and a loop
      // that tests the stage in every row branches and copies registers at
      // every join.
      const R sa = stage == 0 ? R(0) : R(1), sb = (stage == 1 || stage == 2) ? R(2) : R(1);
      const R sc = stage == 3 ? h6 : R(0), sy = stage < 3 ? hin : R(0);
      auto kstep = [&](auto kind) {
        constexpr int KS = decltype(kind)::value;
        constexpr int PF = 4;
        cpx<R> pa[PF], pb[PF];
#pragma unroll
        for (int i = 0; i < PF; ++i) {
          pa[i] = mown[i * LS];
          pb[i] = mtr[i];
        }
#pragma unroll
        for (int r = 0; r < FB; ++r) {
          const cpx<R> a0 = pa[r % PF], b0 = pb[r % PF];
          if (r + PF < FB) {
            pa[r % PF] = mown[(r + PF) * LS];
            pb[r % PF] = mtr[r + PF];
          }
          const R kr = a0.im + b0.im, ki = b0.re - a0.re;
          if constexpr (KS < 0) {
            ss[r].re = fm(sb, kr, sa * ss[r].re);
            ss[r].im = fm(sb, ki, sa * ss[r].im);
            rr[r].re = fm(sc, ss[r].re, rr[r].re);
            rr[r].im = fm(sc, ss[r].im, rr[r].im);
            y[r].re = fm(sy, kr, rr[r].re);
            y[r].im = fm(sy, ki, rr[r].im);
          } else {
            if constexpr (KS == 0) {
              ss[r] = cmake(kr, ki);
            } else if constexpr (KS == 1) {
              ss[r].re = fm(R(2), kr, ss[r].re);
              ss[r].im = fm(R(2), ki, ss[r].im);
            }
            if constexpr (KS < 3) {
              y[r].re = fm(hin, kr, rr[r].re);
              y[r].im = fm(hin, ki, rr[r].im);
            } else {
              rr[r].re = fm(h6, ss[r].re + kr, rr[r].re);
              rr[r].im = fm(h6, ss[r].im + ki, rr[r].im);
              y[r] = rr[r];
            }
          }
          // the next stage's jump terms read Y from the triangle; stage A of
          // this stage read it before the barrier above
          if (DISS && active && r >= qk_k) sT[tlo_k + r * k27_k + r * (r + 1) / 2] = y[r];
          if (r == 1) band_publish();
          if (r == 18) pre = load_word(tag + 1);   // the neighbours have published by now
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      if (DISS)
        kstep(std::integral_constant<int, -1>{});
      else if (stage == 0)
        kstep(std::integral_constant<int, 0>{});
      else if (stage < 3)
        kstep(std::integral_constant<int, 1>{});
      else
        kstep(std::integral_constant<int, 3>{});
      __syncthreads();
    }
    if (sBail) {
      // poison this cluster so that a timed-out call cannot pass unnoticed
      const R nan = __builtin_nan("");
#pragma unroll
      for (int r = 0; r < FB; ++r)
        if (active) rho[(27 * k + r) * FD + q] = cmake(nan, nan);
      break;
    }
    if (active) {
#pragma unroll
      for (int r = 0; r < FB; ++r) rho[(27 * k + r) * FD + q] = rr[r];
    }
  }
}

__global__ void k_zero_words(uint64_t* p, size_t n, int* status) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
  if (i == 0 && status) *status = 0;
}

}  // namespace

size_t fused_exchange_words(int nc, int G) { return (size_t)G * nc * 32; }

// Largest number of trajectories the fused kernel (with the dissipator when
// diss; the three-workgroups-per-CU FP32 build when wide) can keep resident
// at once for nc clusters each (0 if not even one fits).
int fused_slots(int nc, int dtype, bool diss, bool wide) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (wide && (dtype == 1 || diss)) return 0;
  const void* f = wide ? (const void*)k_fused<float, false, 3>
                  : dtype == 1 ? (diss ? (const void*)k_fused<double, true> : (const void*)k_fused<double, false>)
                               : (diss ? (const void*)k_fused<float, true> : (const void*)k_fused<float, false>);
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, FNT, 0);
  if (e != hipSuccess || per_cu <= 0) return 0;
  return (cus * per_cu) / nc;
}

hipError_t fused_zero_words(uint64_t* xch, size_t nw, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, xch, nw, status);
  return hipGetLastError();
}

template <typename R>
static hipError_t fused_launch(const Geom& g, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                              double dt, int n_steps, int spin_limit, const double* sJ, const double* sU, bool wide,
                              hipStream_t s) {
  if (sJ && n_steps > kSchedSteps) return hipErrorInvalidValue;
  FusedArgs<R> a{};
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
  a.gd = (R)g.gdeph;
  a.gl = (R)g.gloss;
  a.sched = sJ ? 1 : 0;
  if (sJ)
    for (int i = 0; i <= 2 * n_steps; ++i) {
      a.sJ[i] = (R)sJ[i];
      a.sU[i] = (R)sU[i];
    }
  void* args[] = {&a};
  const bool diss = g.gdeph > 0 || g.gloss > 0;
  const void* f = diss ? (const void*)k_fused<R, true> : (const void*)k_fused<R, false>;
  if constexpr (sizeof(R) == 4) {
    if (wide) {
      if (diss) return hipErrorInvalidValue;
      f = (const void*)k_fused<float, false, 3>;
    }
  } else {
    if (wide) return hipErrorInvalidValue;
  }
  return hipLaunchCooperativeKernel(f, dim3((unsigned)(g.nc * G)), dim3(FNT), args, 0, s);
}

hipError_t fused_rk4(const Geom& g, int dtype, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                     double dt, int n_steps, int spin_limit, const double* sJ, const double* sU, bool zero_status,
                     bool wide, hipStream_t s) {
  hipError_t e = fused_zero_words(xch, fused_exchange_words(g.nc, G), zero_status ? status : nullptr, s);
  if (e != hipSuccess) return e;
  return dtype == 1 ? fused_launch<double>(g, rho, xch, status, legs, G, dt, n_steps, spin_limit, sJ, sU, wide, s)
                    : fused_launch<float>(g, rho, xch, status, legs, G, dt, n_steps, spin_limit, sJ, sU, wide, s);
}

// ---------------------------------------------------------------------------
// Batch launch: the gangs of several member problems in one cooperative
// launch (closed systems, constant couplings, the builds for one and two
// workgroups per CU).
// ---------------------------------------------------------------------------
size_t fused_member_bytes(int dtype) { return dtype == 1 ? sizeof(FusedMember<double>) : sizeof(FusedMember<float>); }

template <typename R>
static void member_fill_t(const Geom& g, void* rho, uint64_t* xch, const int* legs, int G, int slot0, void* out) {
  FusedMember<R> m{};
  m.rho = (cpx<R>*)rho;
  m.xch = xch;
  m.legs = legs;
  m.n_traj = g.n_traj;
  m.nc = g.nc;
  m.G = G;
  m.slot0 = slot0;
  m.J = (R)g.J;
  m.U = (R)g.U;
  std::memcpy(out, &m, sizeof(m));
}

void fused_member_fill(const Geom& g, int dtype, void* rho, uint64_t* xch, const int* legs, int G, int slot0,
                       void* out) {
  if (dtype == 1)
    member_fill_t<double>(g, rho, xch, legs, G, slot0, out);
  else
    member_fill_t<float>(g, rho, xch, legs, G, slot0, out);
}

// Workgroups of the batch kernel that the device keeps resident at once.
int fused_multi_slots(int dtype) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* f = dtype == 1 ? (const void*)k_fused<double, false, 1, true> : (const void*)k_fused<float, false, 2, true>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, FNT, 0) != hipSuccess || per_cu <= 0) return 0;
  return cus * per_cu;
}

template <typename R>
static hipError_t multi_launch(const void* members, int n_members, int grid, int* status, double dt, int n_steps,
                               int spin_limit, hipStream_t s) {
  FusedArgs<R> a{};
  a.status = status;
  a.n_steps = n_steps;
  a.dt = (R)dt;
  a.spin_limit = spin_limit;
  a.members = (const FusedMember<R>*)members;
  a.n_members = n_members;
  void* args[] = {&a};
  const void* f = sizeof(R) == 8 ? (const void*)k_fused<double, false, 1, true> : (const void*)k_fused<float, false, 2, true>;
  return hipLaunchCooperativeKernel(f, dim3((unsigned)grid), dim3(FNT), args, 0, s);
}

hipError_t fused_multi_rk4(int dtype, const void* members, int n_members, int grid, uint64_t* xch, size_t n_words,
                           int* status, double dt, int n_steps, int spin_limit, hipStream_t s) {
  if (grid < 1 || grid > fused_multi_slots(dtype)) return hipErrorInvalidValue;
  hipError_t e = fused_zero_words(xch, n_words, status, s);
  if (e != hipSuccess) return e;
  return dtype == 1 ? multi_launch<double>(members, n_members, grid, status, dt, n_steps, spin_limit, s)
                    : multi_launch<float>(members, n_members, grid, status, dt, n_steps, spin_limit, s);
}

}  // namespace cdtwa
