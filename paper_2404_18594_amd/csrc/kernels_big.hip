// Per-stage path for cluster matrices larger than the LDS: 2x2 clusters with
// d = 4 (D = 256; 1 MB per cluster in FP64).  Sec. II Eq. (cluster_mf);
// App. B.1 Gamma^intra, Phi^inter and the RK4 remark.
//
// The Kronecker index p = 64 n1 + 16 n2 + 4 n3 + n4 of the four site digits
// cuts the matrix into 16 x 16 tiles (I, J): row block I holds the rows whose
// leading digits (n1, n2) = (I / 4, I % 4) are fixed, and the trailing digits
// (n3, n4) run inside it.  K = -i [H, Y] is Hermitian, so a stage forms the
// 136 upper tiles I <= J.  Every term of H moves one or two digits by one,
// so (H Y)_pq for p in block I needs the rows of I and of its neighbour
// blocks, (n1, n2) shifted by (+-1, 0), (0, +-1), (+1, -1), (-1, +1).  How a
// stage splits this over workgroups, waves and lanes is described at
// k_big_strip below; neither K nor M = H Y ever reaches memory.
//
// RK4 with three packed arrays in the workspace (each tile (I, J), I <= J,
// stored as 256 contiguous entries, tiles in row-major order over I <= J):
//   stage 1: K1 from rho;  Y2 = rho + dt/2 K1,  A = dt/6 K1
//   stage 2: K2 from Y2;   Y3 = rho + dt/2 K2,  A += dt/3 K2
//   stage 3: K3 from Y3;   Y4 = rho + dt K3,    A += dt/3 K3
//   stage 4: K4 from Y4;   rho += A + dt/6 K4
// (classical RK4, fields recomputed at every stage).  A holds the increment
// of the step, not rho plus it: rho is rounded once per step, as in the
// other paths (an accumulator of rho's size, rounded at every stage,
// quadruples the FP32 rounding of the state).  The compensated FP32 step
// (stage mode 5 in place of 4) also carries the rounding error of rho in a
// packed array of low parts: rho + lo + A is formed with an error-free sum
// (Knuth's TwoSum), the sum rounded to FP32 becomes rho and its exact
// remainder the new lo, so that rho + lo follows the FP32 increments without
// a rounding of the state at every step.  The halo of stage 1 reads
// rho, which only stage 4 writes; stage 4 reads rho only at the entries its
// own threads then overwrite.  The mean fields b_l of the next stage matrix
// come from its band entries Y[q + s_l][q] = conj(Y[q][q + s_l]), which lie
// in the tiles (I, I) (sites 3, 4), (I, I + 1) (site 2) and (I, I + 4)
// (site 1): the workgroup that updates such a tile writes its band sum, and
// k_big_band_sum adds the tile sums of a site in tile order.
#include "launch.hpp"
#include "structured.hpp"

namespace cdtwa {

namespace {

constexpr int BD = 256;                        // cluster dimension
constexpr int BT = 16;                         // tile side
constexpr int BNB = BD / BT;                   // tiles per side
constexpr int BNTILE = BNB * (BNB + 1) / 2;    // upper tiles (136)
constexpr int BTE = BT * BT;                   // entries per tile
constexpr int64_t BPACK = (int64_t)BNTILE * BTE;   // entries of a packed cluster matrix
constexpr int BNT = 256;                       // threads of the unpack kernel (one per tile entry)
constexpr int BBAND = 56;                      // band tile sums per cluster

__host__ __device__ constexpr int tile_index(int I, int J) { return I * BNB - I * (I - 1) / 2 + (J - I); }

// entry (r, c) of the stored upper tile (A, B), A <= B, relative to the
// cluster's base: full layout (row-major D x D) or packed tiles
template <bool FULL>
__device__ inline int64_t tile_addr(int A, int B, int r, int c) {
  if constexpr (FULL)
    return (int64_t)(BT * A + r) * BD + BT * B + c;
  else
    return (int64_t)tile_index(A, B) * BTE + r * BT + c;
}
template <bool FULL>
constexpr int64_t cluster_elems() {
  return FULL ? (int64_t)BD * BD : BPACK;
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

// upper tile number t -> (I, J), row-major over I <= J
__device__ inline void tile_of(int t, int& I, int& J) {
  I = 0;
  while (t >= BNB - I) {
    t -= BNB - I;
    ++I;
  }
  J = I + t;
}

// -v where f, v where not: the sign bit flipped (f is the same in every lane)
__device__ inline double flip_sign(double v, bool f) {
  return __hiloint2double(__double2hiint(v) ^ (f ? (int)0x80000000u : 0), __double2loint(v));
}
__device__ inline float flip_sign(float v, bool f) {
  return __int_as_float(__float_as_int(v) ^ (f ? (int)0x80000000u : 0));
}

// sqrt(n) for 0 <= n < 4 and 0 for n = 4 (a raising operator on the top
// level): the constants of sqrt_int as a sum of selects (at most one term is
// nonzero), so that a per-lane n compiles to selects rather than branches
__device__ inline double sqz(int n) {
  return (n == 1 ? 1.0 : 0.0) + (n == 2 ? 1.4142135623730951 : 0.0) + (n == 3 ? 1.7320508075688772 : 0.0);
}

template <typename R>
struct BigArgs {
  Geom g;
  const cpx<R>* src;    // halo source: rho (modes 0, 1) or the packed stage matrix (2..5)
  const cpx<R>* rho;    // modes 2..5: rho at the tile (user layout)
  cpx<R>* ynext;        // modes 1..3: next stage matrix (packed)
  cpx<R>* acc;          // modes 1..5: RK4 increment dt/6 K1 + dt/3 K2 + dt/3 K3 (packed)
  cpx<R>* out;          // mode 0: K; modes 4, 5: rho (user layout)
  cpx<R>* lo;           // mode 5: low parts of rho (packed), read and written
  const cpx<R>* phi;    // [clusters][4] boundary fields of this stage's matrix
  cpx<R>* band;         // [clusters][BBAND] band tile sums of the next stage matrix
  R dt;
  R dt3, dt6;          // dt / 3 and dt / 6, rounded once on the host as on the device
  R J, U;
};

// ---------------------------------------------------------------------------
// Stage kernel k_big_strip: the work split so that the operator needs no lane
// shifts and no per-lane coefficients.
//
// Rows and columns are grouped in four super blocks of 64 (the leading digit
// n1).  A wave computes M = H Y on the 16 rows of one row block B (digits
// n1, n2 fixed) and the 64 columns of one super block C: each lane owns one
// column and holds the 16 rows (trailing digits n3, n4) in registers, so every
// in-block shift of the operator (+-1, +-3, +-4) is a register index known at
// compile time, every coefficient depends only on (n1, n2), J, U and the
// cluster's fields (the same in every lane), and a term that leaves the
// truncated space is dropped at compile time.  The six neighbour blocks of B
// are read the same way, one block of 16 rows at a time.
//
// A workgroup of 8 waves owns one of 8 units of a cluster:
//   units 0..5, a super pair (SI, SJ), SI < SJ: waves 0..3 compute the rows
//     of B = 4 SI + w on the columns of SJ, waves 4..7 the rows of
//     B = 4 SJ + w - 4 on the columns of SI.  The workgroup then holds
//     M_(I,J) and M_(J,I) of its 16 tiles (I, J), I in SI, J in SJ.
//   units 6 and 7: waves 4h .. 4h + 3 the diagonal super block
//     S = 2 (u - 6) + h, rows B = 4 S + w % 4 on the columns of S: the 10
//     upper tiles of that super block.
// Every entry of M is formed once per stage.  M goes to LDS, and each entry
// (p, q) of an upper tile takes K = -i (M_pq - conj(M_qp)) from there before
// the RK4 stage above.
constexpr int SNT = 512;                     // threads per workgroup (8 waves)
constexpr int SUNITS = 8;                    // workgroups per cluster
constexpr int SPAD = 65;                     // LDS row of M: 64 columns + 1 (bank spread)
constexpr int SBROWS = 22;                   // band rows of the diagonal units

// sqrt(n) for n = 0..3, 0 for n = 4: sqz on a compile-time digit
constexpr double SQC[5] = {0.0, 1.0, 1.4142135623730951, 1.7320508075688772, 0.0};

// super pair of unit u < 6
__device__ inline void super_pair(int u, int& si, int& sj) {
  si = u < 3 ? 0 : (u < 5 ? 1 : 2);
  sj = u < 3 ? u + 1 : (u < 5 ? u - 1 : 3);
}
// upper tile t' = 0..9 of a diagonal super block, row-major over a <= b
__device__ __host__ constexpr int diag_a(int t) { return t < 4 ? 0 : (t < 7 ? 1 : (t < 9 ? 2 : 3)); }
__device__ __host__ constexpr int diag_b(int t) { return t - (t < 4 ? 0 : (t < 7 ? 3 : (t < 9 ? 5 : 6))); }

template <typename R>
__device__ inline void mac_r(cpx<R>& a, R c, const cpx<R>& y) {
  a.re = fma_r(c, y.re, a.re);
  a.im = fma_r(c, y.im, a.im);
}
// a += (cr + i ci) y: the real part's two products first, then the imaginary part's
template <typename R>
__device__ inline void mac_c(cpx<R>& a, R cr, R ci, const cpx<R>& y) {
  a.re = fma_r(cr, y.re, a.re);
  a.re = fma_r(-ci, y.im, a.re);
  a.im = fma_r(cr, y.im, a.im);
  a.im = fma_r(ci, y.re, a.im);
}

// entry at a 32-bit byte offset from a base that is the same in every lane
template <typename R>
__device__ inline cpx<R> ld_off(const cpx<R>* __restrict__ base, uint32_t bytes) {
  return *(const cpx<R>*)((const char*)base + bytes);
}
template <typename R>
__device__ inline void st_off(cpx<R>* __restrict__ base, uint32_t bytes, const cpx<R>& v) {
  *(cpx<R>*)((char*)base + bytes) = v;
}

// y[k] = Y[16 X + k][64 C + lane], k = 0..15, from the cluster's halo source:
// the full user matrix (SF), or the packed upper tiles.  Lane group g (16
// lanes) reads the 16 x 16 tile (X, 4 C + g); a lower one is stored as the
// conjugate of its mirror (4 C + g, X).  Every load reads rows of the stored
// tile (16 consecutive entries per group), so that lane cq holds entry
// (k, cq) of it; for a mirrored tile that is the value lane k needs as row
// cq, and fix_block transposes it through the wave's own LDS slice sT
// (16 x 65, the slice that later holds its M rows) once the loads have
// arrived.  Whether a group is mirrored depends on the group only.
template <typename R, bool SF>
__device__ inline void load_block(const cpx<R>* __restrict__ src, int X, int C, int lane, cpx<R> (&y)[BT]) {
  constexpr uint32_t CS = sizeof(cpx<R>);
  if constexpr (SF) {
    const uint32_t base = ((uint32_t)(BT * X) * BD + 64 * C + lane) * CS;
#pragma unroll
    for (int k = 0; k < BT; ++k) y[k] = ld_off(src, base + (uint32_t)(k * BD) * CS);
  } else {
    const int g = lane >> 4, cq = lane & 15, Jq = 4 * C + g;
    const bool lo = X > Jq;
    const uint32_t base = ((uint32_t)tile_index(lo ? Jq : X, lo ? X : Jq) * BTE + (uint32_t)cq) * CS;
#pragma unroll
    for (int k = 0; k < BT; ++k) {
      const cpx<R> v = ld_off(src, base + (uint32_t)(k * BT) * CS);
      y[k] = cmake(v.re, flip_sign(v.im, lo));
    }
  }
}
// the transpose of the mirrored groups' values, once they have arrived.  It
// runs for every block: with a branch around it (skipping blocks with no
// mirrored group) the compiler kept both copies of the block live and
// spilled.
template <typename R, bool SF>
__device__ inline void fix_block(int X, int C, int lane, cpx<R> (*sT)[SPAD], cpx<R> (&y)[BT]) {
  if constexpr (!SF) {
    {
      const int g = lane >> 4, cq = lane & 15;
      const bool lo = X > 4 * C + g;
#pragma unroll
      for (int k = 0; k < BT; ++k) sT[k][lane] = y[k];
      // (a wave's LDS operations run in order, and the reads may alias the
      // writes, so the compiler keeps them after the writes)
      // lane (g, cq), row k: entry (cq, k) of the stored tile = sT[cq][16 g + k];
      // a lane of an unmirrored group reads back its own entry sT[k][lane]
      const cpx<R>* flat = &sT[0][0];
      const int base = lo ? cq * SPAD + 16 * g : lane, stride = lo ? 1 : SPAD;
#pragma unroll
      for (int k = 0; k < BT; ++k) y[k] = flat[base + k * stride];
    }
  }
}

// The terms of (H Y)_pq, p = 16 B + k, grouped by the block of the source
// row p' (Sec. II Eq. (cluster_mf), App. B.1): the interaction U n (n - 1) / 2,
// the hops -J sqrt(n_l) sqrt(n_m + 1) a_l^+ a_m of the bonds 1-2, 1-3, 2-4,
// 3-4, and the fields -J conj(phi_l) a_l and -J phi_l a_l^+ (digits of p):
//   kind 0, p' in B: interaction, bond 3-4 (rows k -+ 3), fields of sites 3
//     and 4 (rows k +- 4, k +- 1)
//   kind 1, n1 + 1: a_3^+ a_1 (row k - 4), -J conj(phi_1) a_1 (row k)
//   kind 2, n1 - 1: a_1^+ a_3 (row k + 4), -J phi_1 a_1^+ (row k)
//   kind 3, n2 + 1: a_4^+ a_2 (row k - 1), -J conj(phi_2) a_2
//   kind 4, n2 - 1: a_2^+ a_4 (row k + 1), -J phi_2 a_2^+
//   kind 5, (n1 + 1, n2 - 1): a_2^+ a_1;  kind 6, (n1 - 1, n2 + 1): a_1^+ a_2
// A term whose source row leaves the truncated space has a zero factor
// (sqz(0) = sqz(4) = 0): dropped at compile time for the in-block digits,
// multiplied by 0 for n1, n2 (the block of such a kind does not exist; its
// stand-in values are finite).
template <typename R>
__device__ inline void apply_k0(cpx<R> (&acc)[BT], const cpx<R> (&y)[BT], int n1, int n2, R J, R U,
                                const cpx<R>& p3, const cpx<R>& p4) {
  const int cB = (n1 * (n1 - 1) + n2 * (n2 - 1)) / 2;
#pragma unroll
  for (int k = 0; k < BT; ++k) {
    const int n3 = k >> 2, n4 = k & 3;
    const R dk = U * R(cB + (n3 * (n3 - 1) + n4 * (n4 - 1)) / 2);
    acc[k] = cmake(dk * y[k].re, dk * y[k].im);
    if (n3 >= 1 && n4 <= 2) mac_r(acc[k], -J * R(SQC[n3] * SQC[n4 + 1]), y[k - 3]);
    if (n4 >= 1 && n3 <= 2) mac_r(acc[k], -J * R(SQC[n4] * SQC[n3 + 1]), y[k + 3]);
    if (n3 <= 2) {
      const R cu = -J * R(SQC[n3 + 1]);
      mac_c(acc[k], cu * p3.re, -cu * p3.im, y[k + 4]);
    }
    if (n3 >= 1) {
      const R cd = -J * R(SQC[n3]);
      mac_c(acc[k], cd * p3.re, cd * p3.im, y[k - 4]);
    }
    if (n4 <= 2) {
      const R cu = -J * R(SQC[n4 + 1]);
      mac_c(acc[k], cu * p4.re, -cu * p4.im, y[k + 1]);
    }
    if (n4 >= 1) {
      const R cd = -J * R(SQC[n4]);
      mac_c(acc[k], cd * p4.re, cd * p4.im, y[k - 1]);
    }
  }
}
// kinds 1..4: one hop whose in-block digit moves by DK rows (the block digit
// factor sb), and one field term on the unshifted row (c_re + i c_im)
template <typename R, int KIND>
__device__ inline void apply_k14(cpx<R> (&acc)[BT], const cpx<R> (&y)[BT], double sb, R J, R fr, R fi) {
#pragma unroll
  for (int k = 0; k < BT; ++k) {
    const int n3 = k >> 2, n4 = k & 3;
    if constexpr (KIND == 1) {
      if (n3 >= 1) mac_r(acc[k], -J * R(SQC[n3] * sb), y[k - 4]);
    } else if constexpr (KIND == 2) {
      if (n3 <= 2) mac_r(acc[k], -J * R(sb * SQC[n3 + 1]), y[k + 4]);
    } else if constexpr (KIND == 3) {
      if (n4 >= 1) mac_r(acc[k], -J * R(SQC[n4] * sb), y[k - 1]);
    } else {
      if (n4 <= 2) mac_r(acc[k], -J * R(sb * SQC[n4 + 1]), y[k + 1]);
    }
    mac_c(acc[k], fr, fi, y[k]);
  }
}
template <typename R>
__device__ inline void apply_k56(cpx<R> (&acc)[BT], const cpx<R> (&y)[BT], R h) {
#pragma unroll
  for (int k = 0; k < BT; ++k) mac_r(acc[k], h, y[k]);
}

// neighbour block of kind 1 (n1 + 1), B itself where it does not exist
__device__ inline int kind1_block(int B) { return (B >> 2) < 3 ? B + 4 : B; }

// M = H Y on rows 16 B .. 16 B + 15, column 64 C + lane, block by block with
// the next block's loads in flight; ya holds block B on entry (issued by the
// caller, during the previous unit's update)
template <typename R, bool SF>
__device__ inline void strip_apply(const cpx<R>* __restrict__ src, int B, int C, int lane, R J, R U,
                                   const cpx<R>* ph, cpx<R> (*sT)[SPAD], cpx<R> (&ya)[BT], cpx<R> (&acc)[BT]) {
  const int n1 = B >> 2, n2 = B & 3;
  // neighbour block of each kind, B itself where it does not exist
  const int X1 = kind1_block(B), X2 = n1 > 0 ? B - 4 : B;
  const int X3 = n2 < 3 ? B + 1 : B, X4 = n2 > 0 ? B - 1 : B;
  const int X5 = n1 < 3 && n2 > 0 ? B + 3 : B, X6 = n1 > 0 && n2 < 3 ? B - 3 : B;
  cpx<R> yb[BT];
  load_block<R, SF>(src, X1, C, lane, yb);
  fix_block<R, SF>(B, C, lane, sT, ya);
  apply_k0<R>(acc, ya, n1, n2, J, U, ph[2], ph[3]);
  load_block<R, SF>(src, X2, C, lane, ya);
  fix_block<R, SF>(X1, C, lane, sT, yb);
  {
    const double s = sqz(n1 + 1);
    const R cu = -J * R(s);
    apply_k14<R, 1>(acc, yb, s, J, cu * ph[0].re, -cu * ph[0].im);
  }
  load_block<R, SF>(src, X3, C, lane, yb);
  fix_block<R, SF>(X2, C, lane, sT, ya);
  {
    const double s = sqz(n1);
    const R cd = -J * R(s);
    apply_k14<R, 2>(acc, ya, s, J, cd * ph[0].re, cd * ph[0].im);
  }
  load_block<R, SF>(src, X4, C, lane, ya);
  fix_block<R, SF>(X3, C, lane, sT, yb);
  {
    const double s = sqz(n2 + 1);
    const R cu = -J * R(s);
    apply_k14<R, 3>(acc, yb, s, J, cu * ph[1].re, -cu * ph[1].im);
  }
  load_block<R, SF>(src, X5, C, lane, yb);
  fix_block<R, SF>(X4, C, lane, sT, ya);
  {
    const double s = sqz(n2);
    const R cd = -J * R(s);
    apply_k14<R, 4>(acc, ya, s, J, cd * ph[1].re, cd * ph[1].im);
  }
  load_block<R, SF>(src, X6, C, lane, ya);
  fix_block<R, SF>(X5, C, lane, sT, yb);
  apply_k56<R>(acc, yb, -J * R(sqz(n2) * sqz(n1 + 1)));
  fix_block<R, SF>(X6, C, lane, sT, ya);
  apply_k56<R>(acc, ya, -J * R(sqz(n1) * sqz(n2 + 1)));
}

// rows of block B on the columns of super block C: the role of wave w in unit u
__device__ inline void unit_roles(int u, int w, int& B, int& C) {
  if (u < 6) {
    int si, sj;
    super_pair(u, si, sj);
    B = w < 4 ? 4 * si + w : 4 * sj + (w - 4);
    C = w < 4 ? sj : si;
  } else {
    const int S = 2 * (u - 6) + (w >> 2);
    B = 4 * S + (w & 3);
    C = S;
  }
}

// Tile of update iteration j in a unit: t = 2 j + hi, the same in every lane
// of a wave (hi = thread >> 8).  M_pq lies in wave w1 (row r, lane 16 cb + c),
// M_qp in wave w2 (row c, lane 16 ca + r).  DIAG: units 6, 7 (20 tiles).
struct UTile {
  int I, J, w1, w2, ca, cb, h;
};
template <bool DIAG>
__device__ inline UTile utile(int u, int j, int hi) {
  UTile t;
  const int t0 = 2 * j + hi;
  if constexpr (DIAG) {
    t.h = t0 >= 10 ? 1 : 0;
    const int tt = t0 - 10 * t.h, S = 2 * (u - 6) + t.h;
    t.ca = diag_a(tt);
    t.cb = diag_b(tt);
    t.I = 4 * S + t.ca;
    t.J = 4 * S + t.cb;
    t.w1 = 4 * t.h + t.ca;
    t.w2 = 4 * t.h + t.cb;
  } else {
    int si, sj;
    super_pair(u, si, sj);
    t.h = 0;
    t.ca = t0 >> 2;
    t.cb = t0 & 3;
    t.I = 4 * si + t.ca;
    t.J = 4 * sj + t.cb;
    t.w1 = t.ca;
    t.w2 = 4 + t.cb;
  }
  return t;
}
constexpr int SNJ = 10;   // update iterations of a diagonal unit (8 elsewhere)

// the update's own entries of rho and of the accumulator
template <typename R, int MODE, bool FULL, bool DIAG>
__device__ inline void strip_own_loads(const BigArgs<R>& a, int64_t flat, int u, int tid, cpx<R> (&rho_o)[SNJ],
                                       cpx<R> (&acc_o)[SNJ], cpx<R> (&lo_o)[SNJ]) {
  if constexpr (MODE >= 1) {   // (mode 0, the bare commutator, reads neither)
    constexpr int NJ = DIAG ? 10 : 8;
    const int r = (tid >> 4) & 15, c = tid & 15, hi = tid >> 8;
    constexpr uint32_t CS = sizeof(cpx<R>);
    const cpx<R>* rho = (MODE == 1 ? a.src : a.rho) + flat * cluster_elems<FULL>();
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const UTile t = utile<DIAG>(u, j, hi);
      rho_o[j] = ld_off(rho, (uint32_t)tile_addr<FULL>(t.I, t.J, r, c) * CS);
      if constexpr (MODE >= 2) acc_o[j] = ld_off(a.acc + flat * BPACK, (uint32_t)tile_addr<false>(t.I, t.J, r, c) * CS);
      if constexpr (MODE == 5) lo_o[j] = ld_off(a.lo + flat * BPACK, (uint32_t)tile_addr<false>(t.I, t.J, r, c) * CS);
    }
  }
}

// K = -i (M - M^+) from LDS and the RK4 stage on the unit's
// upper tiles; the band entries of the next matrix go to sBand
template <typename R, int MODE, bool FULL, bool DIAG>
__device__ inline void strip_update(const BigArgs<R>& a, int64_t flat, int u, int tid, const cpx<R> (&rho_o)[SNJ],
                                    const cpx<R> (&acc_o)[SNJ], const cpx<R> (&lo_o)[SNJ], cpx<R> (*sM)[BT][SPAD],
                                    cpx<R> (*sBand)[BT]) {
  constexpr int NJ = DIAG ? 10 : 8;
  constexpr uint32_t CS = sizeof(cpx<R>);
  const int r = (tid >> 4) & 15, c = tid & 15, hi = tid >> 8;
  // the packed workspace arrays of this cluster (modes 1..3 write both, 4 reads
  // the accumulator through acc_o, 0 uses neither)
  cpx<R>* accb = MODE >= 1 && MODE <= 3 ? a.acc + flat * BPACK : nullptr;
  cpx<R>* ynb = MODE >= 1 && MODE <= 3 ? a.ynext + flat * BPACK : nullptr;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const UTile t = utile<DIAG>(u, j, hi);
    const int I = t.I, J = t.J;
    const cpx<R> hpq = sM[t.w1][r][16 * t.cb + c];
    const cpx<R> hqp = sM[t.w2][c][16 * t.ca + r];
    // K = -i (M - M^+):  K.re = Im M_pq + Im M_qp,  K.im = Re M_qp - Re M_pq
    const cpx<R> K = cmake(hpq.im + hqp.im, hqp.re - hpq.re);
    // byte offsets within the cluster (a D x D matrix is at most 1 MiB)
    const uint32_t pk = (uint32_t)tile_addr<false>(I, J, r, c) * CS;
    auto store_user = [&](cpx<R>* base, const cpx<R>& x) {
      if constexpr (FULL) {
        st_off(base, (uint32_t)tile_addr<true>(I, J, r, c) * CS, x);
        if (I != J) st_off(base, (uint32_t)((BT * J + c) * BD + BT * I + r) * CS, cmake(x.re, -x.im));
      } else {
        st_off(base, pk, x);
      }
    };
    if constexpr (MODE == 0) {
      store_user(a.out + flat * cluster_elems<FULL>(), K);
    } else {
      const R dt = a.dt;
      const cpx<R> rho_own = rho_o[j];
      cpx<R> nxt;
      if constexpr (MODE == 1) {
        const R h2 = R(0.5) * dt, h6 = a.dt6;
        nxt = cmake(fma_r(h2, K.re, rho_own.re), fma_r(h2, K.im, rho_own.im));
        st_off(accb, pk, cmake(h6 * K.re, h6 * K.im));
        st_off(ynb, pk, nxt);
      } else if constexpr (MODE == 2 || MODE == 3) {
        const cpx<R> acc_own = acc_o[j];
        const R hy = MODE == 2 ? R(0.5) * dt : dt, h3 = a.dt3;
        nxt = cmake(fma_r(hy, K.re, rho_own.re), fma_r(hy, K.im, rho_own.im));
        st_off(accb, pk, cmake(fma_r(h3, K.re, acc_own.re), fma_r(h3, K.im, acc_own.im)));
        st_off(ynb, pk, nxt);
      } else {
        // the increment of the step first, then rho rounded once
        const cpx<R> acc_own = acc_o[j];
        const R h6 = a.dt6;
        const cpx<R> inc = cmake(fma_r(h6, K.re, acc_own.re), fma_r(h6, K.im, acc_own.im));
        if constexpr (MODE == 5) {
          // rho + (inc + lo): TwoSum gives the rounded sum and its exact error
          const cpx<R> lo = lo_o[j];
          const R yr = inc.re + lo.re, yi = inc.im + lo.im;
          const R sr = rho_own.re + yr, si = rho_own.im + yi;
          const R vr = sr - rho_own.re, vi = si - rho_own.im;
          const R er = (rho_own.re - (sr - vr)) + (yr - vr), ei = (rho_own.im - (si - vi)) + (yi - vi);
          nxt = cmake(sr, si);
          st_off(a.lo + flat * BPACK, pk, cmake(er, ei));
        } else {
          nxt = cmake(rho_own.re + inc.re, rho_own.im + inc.im);
        }
        store_user(a.out + flat * cluster_elems<FULL>(), nxt);
      }
      // band entries (q, q + s_l) of the next matrix
      const int i1 = I >> 2, i2 = I & 3;
      if constexpr (DIAG) {
        if (J == I) {
          const int n3 = r >> 2, n4 = r & 3;
          if (c == r + 4 && n3 <= 2) {
            const R wgt = R(sqz(n3 + 1));
            sBand[11 * t.h + 2 * t.ca][r] = cmake(wgt * nxt.re, -wgt * nxt.im);
          }
          if (c == r + 1 && n4 <= 2) {
            const R wgt = R(sqz(n4 + 1));
            sBand[11 * t.h + 2 * t.ca + 1][r] = cmake(wgt * nxt.re, -wgt * nxt.im);
          }
        } else if (J == I + 1 && i2 <= 2 && c == r) {
          const R wgt = R(sqz(i2 + 1));
          sBand[11 * t.h + 8 + t.ca][r] = cmake(wgt * nxt.re, -wgt * nxt.im);
        }
      } else {
        if (J == I + 4 && c == r) {
          const R wgt = R(sqz(i1 + 1));
          sBand[t.ca][r] = cmake(wgt * nxt.re, -wgt * nxt.im);
        }
      }
    }
  }
}

// band tile sums, one thread per band row (k = 0..15 in order); the row is
// cleared for the next unit
template <typename R, bool DIAG>
__device__ inline void strip_band_sums(const BigArgs<R>& a, int64_t flat, int u, int tid, cpx<R> (*sBand)[BT]) {
  int si = 0, sj = 0;
  if constexpr (!DIAG) super_pair(u, si, sj);
  const int nrows = DIAG ? SBROWS : (sj == si + 1 ? 4 : 0);
  if (tid >= nrows) return;
  int slot;
  if constexpr (DIAG) {
    const int h = tid / 11, x = tid % 11, S = 2 * (u - 6) + h;
    slot = x < 8 ? 24 + 4 * S + (x >> 1) + 16 * (x & 1) : 12 + 3 * S + (x - 8);
  } else {
    slot = 4 * si + tid;
  }
  R sr = 0, sim = 0;
  for (int k = 0; k < BT; ++k) {
    sr += sBand[tid][k].re;
    sim += sBand[tid][k].im;
    sBand[tid][k] = cmake(R(0), R(0));
  }
  a.band[flat * BBAND + slot] = cmake(sr, sim);
}

// the rest of a unit after its M phase: own loads, barrier, K and the RK4
// stage, barrier, band sums
template <typename R, int MODE, bool FULL, bool DIAG>
__device__ inline void strip_finish(const BigArgs<R>& a, int64_t flat, int u, int tid, cpx<R> (*sM)[BT][SPAD],
                                    cpx<R> (*sBand)[BT]) {
  cpx<R> rho_o[SNJ], acc_o[SNJ], lo_o[SNJ];
  strip_own_loads<R, MODE, FULL, DIAG>(a, flat, u, tid, rho_o, acc_o, lo_o);
  __syncthreads();
  strip_update<R, MODE, FULL, DIAG>(a, flat, u, tid, rho_o, acc_o, lo_o, sM, sBand);
  if constexpr (MODE != 0) {
    __syncthreads();
    strip_band_sums<R, DIAG>(a, flat, u, tid, sBand);
  }
}

// One workgroup per unit, numbered so that the 8 units of a cluster run
// together on one XCD and share its L2 for the halo reads.  The own entries
// of rho and of the accumulator are loading while the workgroup waits for
// the last M rows.  FP32: two workgroups per CU (at most 128 registers).
template <typename R, int MODE, bool FULL>
__global__ void __launch_bounds__(SNT, sizeof(R) == 4 ? 4 : 2) k_big_strip(BigArgs<R> a) {
  __shared__ cpx<R> sM[8][BT][SPAD];
  __shared__ cpx<R> sBand[SBROWS][BT];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  constexpr bool SF = FULL && MODE <= 1;
  constexpr int64_t CE = SF ? cluster_elems<true>() : BPACK;
  const int64_t L = xcd_block();
  const int64_t flat = L / SUNITS;
  const int u = (int)(L % SUNITS);
  const cpx<R>* src = a.src + flat * CE;
  int B, C;
  unit_roles(u, w, B, C);
  cpx<R> ya[BT];
  load_block<R, SF>(src, B, C, lane, ya);
  for (int i = tid; i < SBROWS * BT; i += SNT) sBand[i / BT][i % BT] = cmake(R(0), R(0));
  cpx<R> ph[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) ph[l] = a.phi[flat * 4 + l];
  {
    cpx<R> acc[BT];
    strip_apply<R, SF>(src, B, C, lane, a.J, a.U, ph, sM[w], ya, acc);
#pragma unroll
    for (int k = 0; k < BT; ++k) sM[w][k][lane] = acc[k];
  }
  if (u < 6)
    strip_finish<R, MODE, FULL, false>(a, flat, u, tid, sM, sBand);
  else
    strip_finish<R, MODE, FULL, true>(a, flat, u, tid, sM, sBand);
}

// band tile sums of site l in tile order -> b[t][site]
template <typename R>
__global__ void __launch_bounds__(256) k_big_band_sum(Geom g, const cpx<R>* __restrict__ band, cpx<R>* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_traj * g.nc * 4) return;
  const int l = (int)(i % 4);
  const int64_t flat = i / 4;
  const int first = l == 0 ? 0 : (l == 1 ? 12 : (l == 2 ? 24 : 40));
  const int n = l <= 1 ? 12 : 16;
  R sr = 0, si = 0;
  for (int k = 0; k < n; ++k) {
    const cpx<R> v = band[flat * BBAND + first + k];
    sr += v.re;
    si += v.im;
  }
  const int64_t t = flat / g.nc;
  const int mu = (int)(flat % g.nc);
  b[t * g.Ns + g.cluster_site[mu * 4 + l]] = cmake(sr, si);
}

// boundary fields of every cluster site: phi[flat][l] = sum of b over the
// lattice neighbours of site l in other clusters (directions +x, -x, +y, -y
// in that order)
template <typename R>
__global__ void __launch_bounds__(256) k_big_phi(Geom g, const cpx<R>* __restrict__ b, cpx<R>* __restrict__ phi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_traj * g.nc * 4) return;
  const int l = (int)(i % 4);
  const int64_t flat = i / 4;
  const int64_t t = flat / g.nc;
  const int mu = (int)(flat % g.nc);
  const int j = g.cluster_site[mu * 4 + l];
  R re = 0, im = 0;
  for (int k = 0; k < 4; ++k) {
    const int n = g.ext_nbr[j * 4 + k];
    if (n < 0) continue;
    const cpx<R> v = b[t * g.Ns + n];
    re += v.re;
    im += v.im;
  }
  phi[i] = cmake(re, im);
}

// b_l = Tr(a_l rho) = sum_q sqrt(n_l(q)+1) conj(rho[q][q + s_l]) from the
// state itself, summed per band tile in row order and then over tiles in tile
// order (the order of k_big_strip and k_big_band_sum, so that the fields at
// the start of a call equal those the last stage of the previous call left)
template <typename R, bool FULL>
__global__ void __launch_bounds__(256) k_big_rho_fields(Geom g, const cpx<R>* __restrict__ rho, cpx<R>* __restrict__ b) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_traj * g.nc * 4) return;
  const int l = (int)(i % 4);
  const int64_t flat = i / 4;
  const cpx<R>* m = rho + flat * cluster_elems<FULL>();
  R br = 0, bi = 0;
  for (int I = 0; I < BNB; ++I) {
    const int i1 = I >> 2, i2 = I & 3;
    int J = I;
    if (l == 0) {
      if (i1 > 2) continue;
      J = I + 4;
    } else if (l == 1) {
      if (i2 > 2) continue;
      J = I + 1;
    }
    R tr = 0, ti = 0;
    for (int r = 0; r < BT; ++r) {
      int cc, n;
      if (l <= 1) {
        cc = r;
        n = l == 0 ? i1 : i2;
      } else if (l == 2) {
        cc = r + 4;
        n = r >> 2;
      } else {
        cc = r + 1;
        n = r & 3;
      }
      if (n > 2) continue;
      const cpx<R> v = m[tile_addr<FULL>(I, J, r, cc)];
      const R w = R(sqz(n + 1));
      tr += w * v.re;
      ti += -w * v.im;
    }
    br += tr;
    bi += ti;
  }
  const int64_t t = flat / g.nc;
  const int mu = (int)(flat % g.nc);
  b[t * g.Ns + g.cluster_site[mu * 4 + l]] = cmake(br, bi);
}

// packed -> full: one workgroup per upper tile, the tile and its mirror
template <typename R>
__global__ void __launch_bounds__(BNT) k_big_unpack(int64_t clusters, const cpx<R>* __restrict__ pk,
                                                    cpx<R>* __restrict__ full) {
  const int64_t L = blockIdx.x;
  const int64_t flat = L / BNTILE;
  int I, J;
  tile_of((int)(L % BNTILE), I, J);
  const int r = threadIdx.x / BT, c = threadIdx.x % BT;
  const cpx<R> v = pk[flat * BPACK + tile_addr<false>(I, J, r, c)];
  cpx<R>* m = full + flat * cluster_elems<true>();
  m[tile_addr<true>(I, J, r, c)] = v;
  if (I != J) m[(int64_t)(BT * J + c) * BD + BT * I + r] = cmake(v.re, -v.im);
}

template <typename R, int MODE, bool FULL>
hipError_t launch_stage(const BigArgs<R>& a, hipStream_t s) {
  const int64_t units = a.g.n_traj * a.g.nc * SUNITS;
  hipLaunchKernelGGL((k_big_strip<R, MODE, FULL>), dim3((unsigned)units), dim3(SNT), 0, s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_band_sum(const Geom& g, const cpx<R>* band, cpx<R>* b, hipStream_t s) {
  const int64_t n = g.n_traj * g.nc * 4;
  hipLaunchKernelGGL((k_big_band_sum<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, band, b);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_phi(const Geom& g, const cpx<R>* b, cpx<R>* phi, hipStream_t s) {
  const int64_t n = g.n_traj * g.nc * 4;
  hipLaunchKernelGGL((k_big_phi<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, b, phi);
  return hipGetLastError();
}

template <typename R, bool FULL>
hipError_t launch_rho_fields(const Geom& g, const cpx<R>* rho, cpx<R>* b, hipStream_t s) {
  const int64_t n = g.n_traj * g.nc * 4;
  hipLaunchKernelGGL((k_big_rho_fields<R, FULL>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, rho, b);
  return hipGetLastError();
}

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

template <typename R>
struct BigWs {
  cpx<R>*ya, *yb, *acc, *band, *b, *phi;
};
template <typename R>
BigWs<R> big_ws(const Geom& g, void* ws) {
  const size_t pk = a256((size_t)g.n_traj * g.nc * BPACK * sizeof(cpx<R>));
  const size_t bd = a256((size_t)g.n_traj * g.nc * BBAND * sizeof(cpx<R>));
  const size_t fb = a256((size_t)g.n_traj * g.Ns * sizeof(cpx<R>));
  char* w = (char*)ws;
  BigWs<R> o;
  o.ya = (cpx<R>*)w;
  o.yb = (cpx<R>*)(w + pk);
  o.acc = (cpx<R>*)(w + 2 * pk);
  o.band = (cpx<R>*)(w + 3 * pk);
  o.b = (cpx<R>*)(w + 3 * pk + bd);
  o.phi = (cpx<R>*)(w + 3 * pk + bd + fb);   // [clusters][4] = [n_traj][Ns] entries
  return o;
}

// band tile sums -> b -> boundary fields of every cluster
template <typename R>
hipError_t fields_from_band(const Geom& g, const BigWs<R>& w, hipStream_t s) {
  hipError_t e = launch_band_sum<R>(g, w.band, w.b, s);
  return e == hipSuccess ? launch_phi<R>(g, w.b, w.phi, s) : e;
}

template <typename R, bool FULL>
hipError_t big_rk4_t(const Geom& g0, void* rho_v, void* lo, void* ws, double dt, int n_steps, const double* c1,
                     const double* c2, hipStream_t s) {
  cpx<R>* rho = (cpx<R>*)rho_v;
  const BigWs<R> w = big_ws<R>(g0, ws);
  hipError_t e = launch_rho_fields<R, FULL>(g0, rho, w.b, s);
  if (e == hipSuccess) e = launch_phi<R>(g0, w.b, w.phi, s);
  auto coupl = [&](int64_t hs, R& J, R& U) {
    J = R(c1 ? c1[hs] : g0.J);
    U = R(c2 ? c2[hs] : g0.U);
  };
  for (int it = 0; it < n_steps && e == hipSuccess; ++it) {
    BigArgs<R> a{};
    a.g = g0;
    a.dt = R(dt);
    a.dt3 = a.dt / R(3);
    a.dt6 = a.dt / R(6);
    a.band = w.band;
    a.acc = w.acc;
    a.phi = w.phi;
    // stage 1: rho -> Y2
    coupl(2 * (int64_t)it, a.J, a.U);
    a.src = rho;
    a.ynext = w.ya;
    e = launch_stage<R, 1, FULL>(a, s);
    if (e == hipSuccess) e = fields_from_band<R>(g0, w, s);
    // stage 2: Y2 -> Y3
    coupl(2 * (int64_t)it + 1, a.J, a.U);
    a.src = w.ya;
    a.rho = rho;
    a.ynext = w.yb;
    if (e == hipSuccess) e = launch_stage<R, 2, FULL>(a, s);
    if (e == hipSuccess) e = fields_from_band<R>(g0, w, s);
    // stage 3: Y3 -> Y4
    a.src = w.yb;
    a.ynext = w.ya;
    if (e == hipSuccess) e = launch_stage<R, 3, FULL>(a, s);
    if (e == hipSuccess) e = fields_from_band<R>(g0, w, s);
    // stage 4: Y4 -> rho
    coupl(2 * (int64_t)it + 2, a.J, a.U);
    a.src = w.ya;
    a.out = rho;
    if constexpr (sizeof(R) == 4) {
      a.lo = (cpx<R>*)lo;
      if (e == hipSuccess) e = lo ? launch_stage<R, 5, FULL>(a, s) : launch_stage<R, 4, FULL>(a, s);
    } else {
      if (e == hipSuccess) e = launch_stage<R, 4, FULL>(a, s);
    }
    if (e == hipSuccess) e = fields_from_band<R>(g0, w, s);
  }
  return e;
}

template <typename R, bool FULL>
hipError_t big_commutator_t(const Geom& g, const void* rho, void* K, void* ws, hipStream_t s) {
  const BigWs<R> w = big_ws<R>(g, ws);
  hipError_t e = launch_rho_fields<R, FULL>(g, (const cpx<R>*)rho, w.b, s);
  if (e == hipSuccess) e = launch_phi<R>(g, w.b, w.phi, s);
  if (e != hipSuccess) return e;
  BigArgs<R> a{};
  a.g = g;
  a.src = (const cpx<R>*)rho;
  a.out = (cpx<R>*)K;
  a.phi = w.phi;
  a.J = R(g.J);
  a.U = R(g.U);
  return launch_stage<R, 0, FULL>(a, s);
}

}  // namespace

bool big_supported(int d, int cx, int cy) { return d == 4 && cx == 2 && cy == 2; }

int64_t big_packed_elems() { return BPACK; }

size_t big_workspace_bytes(const Geom& g, int dtype) {
  const size_t cs = dtype == 1 ? 16 : 8;
  return 3 * a256((size_t)g.n_traj * g.nc * BPACK * cs) + a256((size_t)g.n_traj * g.nc * BBAND * cs) +
         2 * a256((size_t)g.n_traj * g.Ns * cs);
}

hipError_t big_rk4(const Geom& g, int dtype, int layout, void* rho, void* lo, void* ws, double dt, int n_steps,
                   const double* c1, const double* c2, hipStream_t s) {
  if (!big_supported(g.d, g.cx, g.cy)) return hipErrorInvalidValue;
  if (lo && dtype == 1) return hipErrorInvalidValue;   // low parts: FP32 state only
  const bool full = layout == 0;
  if (dtype == 1)
    return full ? big_rk4_t<double, true>(g, rho, nullptr, ws, dt, n_steps, c1, c2, s)
                : big_rk4_t<double, false>(g, rho, nullptr, ws, dt, n_steps, c1, c2, s);
  return full ? big_rk4_t<float, true>(g, rho, lo, ws, dt, n_steps, c1, c2, s)
              : big_rk4_t<float, false>(g, rho, lo, ws, dt, n_steps, c1, c2, s);
}

hipError_t big_commutator(const Geom& g, int dtype, int layout, const void* rho, void* K, void* ws, hipStream_t s) {
  if (!big_supported(g.d, g.cx, g.cy)) return hipErrorInvalidValue;
  const bool full = layout == 0;
  if (dtype == 1)
    return full ? big_commutator_t<double, true>(g, rho, K, ws, s) : big_commutator_t<double, false>(g, rho, K, ws, s);
  return full ? big_commutator_t<float, true>(g, rho, K, ws, s) : big_commutator_t<float, false>(g, rho, K, ws, s);
}

hipError_t big_unpack(const Geom& g, int dtype, const void* packed, void* full, hipStream_t s) {
  const int64_t clusters = g.n_traj * g.nc;
  if (dtype == 1)
    hipLaunchKernelGGL((k_big_unpack<double>), dim3((unsigned)(clusters * BNTILE)), dim3(BNT), 0, s, clusters,
                       (const cpx<double>*)packed, (cpx<double>*)full);
  else
    hipLaunchKernelGGL((k_big_unpack<float>), dim3((unsigned)(clusters * BNTILE)), dim3(BNT), 0, s, clusters,
                       (const cpx<float>*)packed, (cpx<float>*)full);
  return hipGetLastError();
}

hipError_t big_site_fields(const Geom& g, int dtype, int layout, const void* rho, void* b, hipStream_t s) {
  if (!big_supported(g.d, g.cx, g.cy)) return hipErrorInvalidValue;
  const bool full = layout == 0;
  if (dtype == 1)
    return full ? launch_rho_fields<double, true>(g, (const cpx<double>*)rho, (cpx<double>*)b, s)
                : launch_rho_fields<double, false>(g, (const cpx<double>*)rho, (cpx<double>*)b, s);
  return full ? launch_rho_fields<float, true>(g, (const cpx<float>*)rho, (cpx<float>*)b, s)
              : launch_rho_fields<float, false>(g, (const cpx<float>*)rho, (cpx<float>*)b, s);
}

}  // namespace cdtwa
