// Host side of the C-dTWA library: plan construction (geometry, generator
// basis and discrete sampling tables), argument validation, workspace layout
// and the launch sequences behind the C ABI declared in include/cdtwa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/cdtwa.h"
#include "launch.hpp"
#include "plan.hpp"

using namespace cdtwa;

namespace {

thread_local std::string g_last_error;

cdtwa_status fail(cdtwa_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

cdtwa_status hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return CDTWA_EHIP;
}

// ---------------------------------------------------------------------------
// Generator bases.  d = 3: the eight matrices T_1..T_8 of App. B.1 (not the
// Gell-Mann set).  d = 2: Pauli matrices (App. A).  d = 4: generalised
// Gell-Mann matrices (pairs j<k lexicographic, symmetric then antisymmetric,
// then the diagonal ones), normalised to Tr(T_a T_b) = 2 delta_ab.
// Stored as [a][row][col][re,im].
// ---------------------------------------------------------------------------
std::vector<double> generator_basis(int d) {
  const int ng = d * d - 1;
  std::vector<double> T((size_t)ng * d * d * 2, 0.0);
  auto set = [&](int a, int r, int c, double re, double im) {
    T[(((size_t)a * d + r) * d + c) * 2] = re;
    T[(((size_t)a * d + r) * d + c) * 2 + 1] = im;
  };
  if (d == 3) {
    const double s = 1.0 / std::sqrt(2.0), t = 1.0 / std::sqrt(3.0);
    // T_1 = (1/sqrt2) [[0,1,0],[1,0,1],[0,1,0]]
    set(0, 0, 1, s, 0); set(0, 1, 0, s, 0); set(0, 1, 2, s, 0); set(0, 2, 1, s, 0);
    // T_2 = (1/sqrt2) [[0,-i,0],[i,0,-i],[0,i,0]]
    set(1, 0, 1, 0, -s); set(1, 1, 0, 0, s); set(1, 1, 2, 0, -s); set(1, 2, 1, 0, s);
    // T_3 = diag(1, 0, -1)
    set(2, 0, 0, 1, 0); set(2, 2, 2, -1, 0);
    // T_4 = [[0,0,1],[0,0,0],[1,0,0]]
    set(3, 0, 2, 1, 0); set(3, 2, 0, 1, 0);
    // T_5 = [[0,0,-i],[0,0,0],[i,0,0]]
    set(4, 0, 2, 0, -1); set(4, 2, 0, 0, 1);
    // T_6 = (1/sqrt2) [[0,-1,0],[-1,0,1],[0,1,0]]
    set(5, 0, 1, -s, 0); set(5, 1, 0, -s, 0); set(5, 1, 2, s, 0); set(5, 2, 1, s, 0);
    // T_7 = (1/sqrt2) [[0,i,0],[-i,0,-i],[0,i,0]]
    set(6, 0, 1, 0, s); set(6, 1, 0, 0, -s); set(6, 1, 2, 0, -s); set(6, 2, 1, 0, s);
    // T_8 = (1/sqrt3) diag(-1, 2, -1)
    set(7, 0, 0, -t, 0); set(7, 1, 1, 2 * t, 0); set(7, 2, 2, -t, 0);
    return T;
  }
  if (d == 2) {
    set(0, 0, 1, 1, 0); set(0, 1, 0, 1, 0);
    set(1, 0, 1, 0, -1); set(1, 1, 0, 0, 1);
    set(2, 0, 0, 1, 0); set(2, 1, 1, -1, 0);
    return T;
  }
  int a = 0;
  for (int j = 0; j < d; ++j)
    for (int k = j + 1; k < d; ++k) {
      set(a, j, k, 1, 0); set(a, k, j, 1, 0); ++a;
      set(a, j, k, 0, -1); set(a, k, j, 0, 1); ++a;
    }
  for (int m = 1; m < d; ++m) {
    const double c = std::sqrt(2.0 / (m * (m + 1.0)));
    for (int i = 0; i < m; ++i) set(a, i, i, c, 0);
    set(a, m, m, -m * c, 0);
    ++a;
  }
  return T;
}

// Eigen-decomposition of a complex Hermitian d x d matrix through the real
// symmetric 2d x 2d embedding [[A,-B],[B,A]] and cyclic Jacobi rotations.
// Returns eigenvalues and the real eigenvectors (columns) of the embedding.
void jacobi_eigen(std::vector<double>& S, int n, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += S[p * n + q] * S[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = S[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (S[q * n + q] - S[p * n + p]) / (2 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        const double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double skp = S[k * n + p], skq = S[k * n + q];
          S[k * n + p] = c * skp - s * skq;
          S[k * n + q] = s * skp + c * skq;
        }
        for (int k = 0; k < n; ++k) {
          const double spk = S[p * n + k], sqk = S[q * n + k];
          S[p * n + k] = c * spk - s * sqk;
          S[q * n + k] = s * spk + c * sqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = S[i * n + i];
}

// Tomography sampling tables for every generator with the site in the Fock
// state |f> (Sec. II; App. B.1): distinct eigenvalues ascending, probability
// p(lambda) = <f|P_lambda|f>, thresholds round(2^32 * cumulative p).
void sampling_tables(const std::vector<double>& T, int d, int f, std::vector<int>& n_out, std::vector<double>& val,
                     std::vector<uint64_t>& thr) {
  const int ng = d * d - 1, n = 2 * d;
  n_out.assign(ng, 0);
  val.assign((size_t)ng * kMaxD, 0.0);
  thr.assign((size_t)ng * kMaxD, (uint64_t)1 << 32);
  for (int a = 0; a < ng; ++a) {
    std::vector<double> S((size_t)n * n, 0.0);
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) {
        const double re = T[(((size_t)a * d + r) * d + c) * 2], im = T[(((size_t)a * d + r) * d + c) * 2 + 1];
        S[r * n + c] = re;
        S[(r + d) * n + (c + d)] = re;
        S[r * n + (c + d)] = -im;
        S[(r + d) * n + c] = im;
      }
    std::vector<double> w, V;
    jacobi_eigen(S, n, w, V);
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    for (int i = 0; i < n; ++i)
      for (int k = i + 1; k < n; ++k)
        if (w[idx[k]] < w[idx[i]]) std::swap(idx[i], idx[k]);
    // group eigenvalues of the embedding (each complex eigenvalue appears twice)
    int no = 0;
    double cum = 0;
    int i = 0;
    while (i < n) {
      const double lam = w[idx[i]];
      double p = 0, sum = 0;
      int cnt = 0;
      while (i < n && std::fabs(w[idx[i]] - lam) < 1e-9) {
        const int col = idx[i];
        const double x1 = V[(size_t)f * n + col], x2 = V[(size_t)(f + d) * n + col];
        p += 0.5 * (x1 * x1 + x2 * x2);
        sum += w[col];
        ++cnt;
        ++i;
      }
      val[(size_t)a * kMaxD + no] = sum / cnt;
      cum += p;
      const double scaled = std::floor(cum * 4294967296.0 + 0.5);
      thr[(size_t)a * kMaxD + no] = scaled >= 4294967296.0 ? ((uint64_t)1 << 32) : (uint64_t)scaled;
      ++no;
    }
    thr[(size_t)a * kMaxD + no - 1] = (uint64_t)1 << 32;
    n_out[a] = no;
  }
}

}  // namespace

struct cdtwa_plan_s {
  cdtwa_problem p;
  Geom g;
  int path = 0;              // 0: per-stage, 1: fused 27-row, 2: fused plaquette, 3: per-stage dense MFMA,
                             // 4: per-stage spin (Ising), 5: fused spin, 6: trajectory-resident
  int G = 0;                 // trajectories resident at once on the fused paths; per workgroup on path 6
  bool wide = false;         // path 1 with three workgroups per CU (FP32, lattices too large for two)
  int spin_limit = 1 << 22;  // polls a fused kernel's neighbour wait may take
  const int* legs = nullptr; // fused path: [nc][4][4] neighbour (cluster*4 + local)
  void* dev = nullptr;       // one device block holding every table
  size_t state_bytes = 0;    // one copy of rho for all trajectories
  size_t field_bytes = 0;    // [n_traj][Ns] complex
  size_t rec_bytes = 0;      // observable cluster records
  size_t ptraj_bytes = 0;    // [n_traj][kNObs] doubles
  int real_bytes = 8;
};

namespace cdtwa {
size_t step_workspace_bytes(cdtwa_plan P);
cdtwa_status set_error(cdtwa_status st, const std::string& msg) { return fail(st, msg); }
const Geom* plan_geom(cdtwa_plan P) { return P ? &P->g : nullptr; }
bool plan_layout(cdtwa_plan P, PlanLayout* out) {
  if (!P || !out) return false;
  *out = PlanLayout{P->state_bytes, P->field_bytes, P->p.dtype, P->path, P->legs, P->wide ? 1 : 0, P->spin_limit};
  return true;
}
}  // namespace cdtwa

extern "C" {

const char* cdtwa_status_string(cdtwa_status s) {
  switch (s) {
    case CDTWA_OK: return "ok";
    case CDTWA_EINVAL: return "invalid argument";
    case CDTWA_EUNSUPPORTED: return "unsupported problem";
    case CDTWA_EHIP: return "HIP error";
    case CDTWA_ENOMEM: return "out of host memory";
  }
  return "unknown status";
}

const char* cdtwa_last_error(void) { return g_last_error.c_str(); }

cdtwa_status cdtwa_plan_create(const cdtwa_problem* pp, int64_t n_traj, cdtwa_plan* out) {
  if (!pp || !out) return fail(CDTWA_EINVAL, "plan_create: NULL argument");
  *out = nullptr;
  const cdtwa_problem p = *pp;
  if (n_traj < 1) return fail(CDTWA_EINVAL, "plan_create: n_traj must be >= 1");
  if (p.Lx < 1 || p.Ly < 1) return fail(CDTWA_EINVAL, "plan_create: lattice sides must be >= 1");
  if (p.cx < 1 || p.cx > 2 || p.cy < 1 || p.cy > 2) return fail(CDTWA_EINVAL, "plan_create: cluster sides must be 1 or 2");
  if (p.Lx % p.cx || p.Ly % p.cy) return fail(CDTWA_EINVAL, "plan_create: lattice not divisible into clusters");
  if (p.d < 2 || p.d > 4) return fail(CDTWA_EINVAL, "plan_create: d must be 2, 3 or 4");
  if (p.periodic && (p.Lx / p.cx < 2 || p.Ly / p.cy < 2 || p.Lx < 3 || p.Ly < 3))
    return fail(CDTWA_EINVAL, "plan_create: a periodic side needs two clusters and three sites");
  if (!(std::isfinite(p.J) && std::isfinite(p.U) && std::isfinite(p.h)))
    return fail(CDTWA_EINVAL, "plan_create: J, U and h must be finite");
  if (p.dtype != CDTWA_F32 && p.dtype != CDTWA_F64) return fail(CDTWA_EINVAL, "plan_create: bad dtype");
  if (p.model != 0 && p.model != 1) return fail(CDTWA_EINVAL, "plan_create: model must be 0 or 1");
  if (p.layout != CDTWA_LAYOUT_FULL && p.layout != CDTWA_LAYOUT_PACKED_UPPER)
    return fail(CDTWA_EINVAL, "plan_create: layout must be CDTWA_LAYOUT_FULL or CDTWA_LAYOUT_PACKED_UPPER");
  if (p.layout == CDTWA_LAYOUT_PACKED_UPPER && (p.model != 0 || !big_supported(p.d, p.cx, p.cy)))
    return fail(CDTWA_EUNSUPPORTED, "plan_create: the packed layout is built for 2x2 clusters with d = 4 only");
  if (p.model == 1 && p.d != 2) return fail(CDTWA_EINVAL, "plan_create: the Ising model needs d = 2");
  if (p.model == 0 && p.h != 0.0) return fail(CDTWA_EINVAL, "plan_create: h is defined for the Ising model only");
  if (p.model == 0 && p.init_state != 0)
    return fail(CDTWA_EUNSUPPORTED, "plan_create: only the unit-filling Mott state for the Bose-Hubbard model");
  if (p.model == 1 && p.init_state != 0 && p.init_state != 1)
    return fail(CDTWA_EUNSUPPORTED, "plan_create: Ising initial state must be 0 (all up) or 1 (Neel)");
  if (!(std::isfinite(p.gamma_deph) && std::isfinite(p.gamma_loss) && p.gamma_deph >= 0 && p.gamma_loss >= 0))
    return fail(CDTWA_EINVAL, "plan_create: Lindblad rates must be finite and >= 0");
  const bool open_system = p.gamma_deph != 0 || p.gamma_loss != 0;
  if (open_system && p.model != 0)
    return fail(CDTWA_EUNSUPPORTED, "plan_create: Lindblad channels are built for the Bose-Hubbard model only");
  if (open_system && big_supported(p.d, p.cx, p.cy))
    return fail(CDTWA_EUNSUPPORTED, "plan_create: Lindblad channels need D <= 81");
  if (!generic_supported(p.d, p.cx, p.cy)) return fail(CDTWA_EUNSUPPORTED, "plan_create: unsupported d or cluster shape");
  if ((int64_t)p.Lx * p.Ly > (1 << 24)) return fail(CDTWA_EINVAL, "plan_create: lattice too large");
  // every launch grid (one thread per trajectory and site at most) must stay
  // below 2^31 work items
  if (n_traj > (int64_t)INT32_MAX / ((int64_t)p.Lx * p.Ly))
    return fail(CDTWA_EINVAL, "plan_create: n_traj x sites exceeds 2^31; split the trajectories into batches");

  cdtwa_plan_s* P = new (std::nothrow) cdtwa_plan_s();
  if (!P) return fail(CDTWA_ENOMEM, "plan_create: allocation failed");
  P->p = p;
  Geom& g = P->g;
  g.Lx = p.Lx; g.Ly = p.Ly; g.cx = p.cx; g.cy = p.cy; g.d = p.d; g.periodic = p.periodic ? 1 : 0;
  g.Ns = p.Lx * p.Ly;
  g.ncx = p.Lx / p.cx;
  g.ncy = p.Ly / p.cy;
  g.nc = g.ncx * g.ncy;
  g.nloc = p.cx * p.cy;
  g.D = 1;
  for (int i = 0; i < g.nloc; ++i) g.D *= p.d;
  g.n_gen = p.d * p.d - 1;
  g.model = p.model;
  g.init_state = p.init_state;
  g.layout = p.layout;
  g.J = p.J;
  g.U = p.U;
  g.h = p.h;
  g.gdeph = p.gamma_deph;
  g.gloss = p.gamma_loss;
  g.n_traj = n_traj;

  std::vector<int> cluster_site((size_t)g.nc * g.nloc), site_cluster(g.Ns), site_local(g.Ns), ext((size_t)g.Ns * 4);
  for (int y = 0; y < p.Ly; ++y)
    for (int x = 0; x < p.Lx; ++x) {
      const int j = y * p.Lx + x;
      const int mu = (y / p.cy) * g.ncx + x / p.cx;
      const int l = (x % p.cx) * p.cy + (y % p.cy);
      site_cluster[j] = mu;
      site_local[j] = l;
      cluster_site[(size_t)mu * g.nloc + l] = j;
    }
  const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
  for (int j = 0; j < g.Ns; ++j) {
    const int x = j % p.Lx, y = j / p.Lx;
    for (int k = 0; k < 4; ++k) {
      int xx = x + dx[k], yy = y + dy[k];
      int n = -1;
      if (g.periodic) {
        xx = (xx + p.Lx) % p.Lx;
        yy = (yy + p.Ly) % p.Ly;
        n = yy * p.Lx + xx;
      } else if (xx >= 0 && xx < p.Lx && yy >= 0 && yy < p.Ly) {
        n = yy * p.Lx + xx;
      }
      if (n >= 0 && site_cluster[n] == site_cluster[j]) n = -1;
      ext[(size_t)j * 4 + k] = n;
    }
  }
  // neighbour legs of every cluster: for local l and direction dir
  // (+x,-x,+y,-y) the neighbouring site in another cluster as cluster*4+local
  std::vector<int> legs((size_t)g.nc * 16, -1);
  if (g.nloc <= 4)
    for (int mu = 0; mu < g.nc; ++mu)
      for (int l = 0; l < g.nloc; ++l)
        for (int k = 0; k < 4; ++k) {
          const int n = ext[(size_t)cluster_site[(size_t)mu * g.nloc + l] * 4 + k];
          if (n >= 0) legs[(size_t)mu * 16 + l * 4 + k] = site_cluster[n] * 4 + site_local[n];
        }
  std::vector<double> T = generator_basis(p.d);
  // one table per onsite-state class: the Mott state |1>, or for the Ising
  // model |up> = |0> (and |down> = |1> on the odd sublattice of the Neel state)
  std::vector<int> n_out;
  std::vector<double> val;
  std::vector<uint64_t> thr;
  const int n_class = p.model == 1 && p.init_state == 1 ? 2 : 1;
  for (int c = 0; c < n_class; ++c) {
    std::vector<int> no;
    std::vector<double> va;
    std::vector<uint64_t> th;
    sampling_tables(T, p.d, p.model == 1 ? c : 1, no, va, th);
    n_out.insert(n_out.end(), no.begin(), no.end());
    val.insert(val.end(), va.begin(), va.end());
    thr.insert(thr.end(), th.begin(), th.end());
  }
  g.g_norm = 2.0;

  // the fused kernels' wait bound; a tiny value makes waits time out (the
  // test of the timeout path sets it)
  if (const char* sl = std::getenv("CDTWA_SPIN_LIMIT")) {
    char* end = nullptr;
    const long v = std::strtol(sl, &end, 10);
    if (end == sl || *end != '\0' || v < 0 || v > INT32_MAX) {
      delete P;
      return fail(CDTWA_EINVAL, "plan_create: CDTWA_SPIN_LIMIT must be an integer in [0, 2^31)");
    }
    P->spin_limit = (int)v;
  }
  // path choice (before any device memory is taken, so that a rejection
  // leaks nothing): the fused paths keep every cluster of G trajectories
  // resident on the chip.  Default: the 27-row kernel in both precisions
  // (measured faster than the plaquette kernel: FP64 11.3 vs 9.6, FP32 with
  // two trajectories resident 20.8 vs 16.1 M cluster-steps/s on 32x32);
  // CDTWA_PATH = generic | fused27 | plaq | dense | spin | traj overrides it.
  // Small clusters (d = 3; 1x1, 2x1, 1x2) run trajectory-resident whenever
  // one trajectory fits a workgroup
  const char* force = std::getenv("CDTWA_PATH");
  const std::string want = force ? force : "";
  if (p.model == 1) {
    // transverse-field Ising: the fused spin kernel for 2x2 clusters when
    // one trajectory fits on the chip, else the spin per-stage kernels
    if (force && want != "spin" && want != "spinfused") {
      delete P;
      return fail(CDTWA_EUNSUPPORTED, "plan_create: the Ising model runs on the spin paths only");
    }
    P->path = 4;
    if (want != "spin" && spin_fused_supported(p.model, p.d, p.cx, p.cy)) {
      const int slots = spin_fused_slots(g.nc, p.dtype);
      if (slots >= 1) {
        P->path = 5;
        P->G = (int)(n_traj < slots ? n_traj : slots);
      }
    }
  } else if (want == "spin" || want == "spinfused") {
    delete P;
    return fail(CDTWA_EUNSUPPORTED, "plan_create: the spin paths need the Ising model");
  } else if (open_system && force && want != "generic" && want != "fused27") {
    // the dissipator lives in the per-stage kernels and the 27-row kernel
    delete P;
    return fail(CDTWA_EUNSUPPORTED, "plan_create: an open system runs on the per-stage or the 27-row path only");
  } else if (want == "dense") {
    // dense-GEMM per-stage variant (FP32, 2x2, d = 3 only)
    if (!dense_supported(p.d, p.cx, p.cy, p.dtype)) {
      delete P;
      return fail(CDTWA_EUNSUPPORTED, "plan_create: the dense path needs an FP32 state, 2x2 clusters and d = 3");
    }
    P->path = 3;
  } else if (want == "traj" || (want != "generic" && traj_supported(p.model, p.d, p.cx, p.cy, open_system))) {
    // small clusters: whole trajectories on chip when one fits a workgroup
    const int ntr = traj_per_item(g, p.dtype);
    if (ntr >= 1) {
      P->path = 6;
      P->G = ntr;
    } else if (want == "traj") {
      delete P;
      return fail(CDTWA_EUNSUPPORTED,
                  "plan_create: the trajectory-resident path needs d = 3, 1x1, 2x1 or 1x2 clusters, a closed "
                  "Bose-Hubbard system and one trajectory that fits a workgroup");
    }
  } else if (want != "generic" && p.d == 3 && p.cx == 2 && p.cy == 2) {
    const bool use_plaq = want == "plaq";
    const int slots = use_plaq ? plaq_slots(g.nc, p.dtype) : fused_slots(g.nc, p.dtype, open_system, false);
    if (slots >= 1) {
      P->path = use_plaq ? 2 : 1;
      P->G = (int)(n_traj < slots ? n_traj : slots);
    } else if (!use_plaq && p.dtype == 0 && !open_system) {
      // FP32 lattices with more clusters than two workgroups per CU hold:
      // the build sized for three (it spills, yet beats the per-stage path)
      const int wslots = fused_slots(g.nc, p.dtype, false, true);
      if (wslots >= 1) {
        P->path = 1;
        P->wide = true;
        P->G = (int)(n_traj < wslots ? n_traj : wslots);
      }
    }
  }

  // one device block: ints, then doubles and uint64 (8-byte aligned)
  const size_t n_int = cluster_site.size() + site_cluster.size() + site_local.size() + ext.size() + n_out.size() +
                       legs.size();
  const size_t off_dbl = ((n_int * sizeof(int) + 255) / 256) * 256;
  const size_t bytes = off_dbl + (T.size() + val.size()) * sizeof(double) + thr.size() * sizeof(uint64_t);
  hipError_t e = hipMalloc(&P->dev, bytes);
  if (e != hipSuccess) {
    delete P;
    return hip_fail(e, "plan_create: hipMalloc");
  }
  std::vector<char> host(bytes, 0);
  size_t o = 0;
  auto put_int = [&](const std::vector<int>& v) {
    std::memcpy(host.data() + o, v.data(), v.size() * sizeof(int));
    const size_t at = o;
    o += v.size() * sizeof(int);
    return (const int*)((char*)P->dev + at);
  };
  g.cluster_site = put_int(cluster_site);
  g.site_cluster = put_int(site_cluster);
  g.site_local = put_int(site_local);
  g.ext_nbr = put_int(ext);
  g.n_out = put_int(n_out);
  P->legs = put_int(legs);
  o = off_dbl;
  std::memcpy(host.data() + o, T.data(), T.size() * sizeof(double));
  g.gen = (const double*)((char*)P->dev + o);
  o += T.size() * sizeof(double);
  std::memcpy(host.data() + o, val.data(), val.size() * sizeof(double));
  g.val = (const double*)((char*)P->dev + o);
  o += val.size() * sizeof(double);
  std::memcpy(host.data() + o, thr.data(), thr.size() * sizeof(uint64_t));
  g.thr = (const uint64_t*)((char*)P->dev + o);
  e = hipMemcpy(P->dev, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(P->dev);
    delete P;
    return hip_fail(e, "plan_create: hipMemcpy");
  }
  P->real_bytes = p.dtype == CDTWA_F64 ? 8 : 4;
  P->state_bytes = (size_t)n_traj * g.nc * (p.layout == CDTWA_LAYOUT_PACKED_UPPER ? big_packed_elems() : (int64_t)g.D * g.D) *
                   2 * P->real_bytes;
  P->field_bytes = (size_t)n_traj * g.Ns * 2 * P->real_bytes;
  // cluster records, whose space later holds the partial sums over trajectories
  P->rec_bytes = std::max((size_t)n_traj * g.nc * obs_record_doubles(g.nloc), obs_sum_scratch_doubles(n_traj)) *
                 sizeof(double);
  P->ptraj_bytes = (size_t)n_traj * kNObs * sizeof(double);
  *out = P;
  return CDTWA_OK;
}

cdtwa_status cdtwa_plan_destroy(cdtwa_plan P) {
  if (!P) return fail(CDTWA_EINVAL, "plan_destroy: NULL plan");
  if (P->dev) (void)hipFree(P->dev);
  delete P;
  return CDTWA_OK;
}

cdtwa_status cdtwa_plan_info(cdtwa_plan P, int32_t* n_sites, int32_t* n_clusters, int32_t* n_local, int32_t* D,
                             int32_t* n_gen, int32_t* real_bytes) {
  if (!P) return fail(CDTWA_EINVAL, "plan_info: NULL plan");
  if (n_sites) *n_sites = P->g.Ns;
  if (n_clusters) *n_clusters = P->g.nc;
  if (n_local) *n_local = P->g.nloc;
  if (D) *D = P->g.D;
  if (n_gen) *n_gen = P->g.n_gen;
  if (real_bytes) *real_bytes = P->real_bytes;
  return CDTWA_OK;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }
// bytes of a full-layout copy of the state of a packed plan (0 otherwise)
static size_t unpacked_bytes(cdtwa_plan P) {
  return P->p.layout == CDTWA_LAYOUT_PACKED_UPPER
             ? align256((size_t)P->g.n_traj * P->g.nc * P->g.D * P->g.D * 2 * P->real_bytes)
             : 0;
}

// the fused paths' status word lives in the first 256 bytes of a workspace;
// the observable scratch starts after them
static constexpr size_t kStatusBytes = 256;

cdtwa_status cdtwa_workspace_bytes(cdtwa_plan P, size_t* bytes) {
  if (!P || !bytes) return fail(CDTWA_EINVAL, "workspace_bytes: NULL argument");
  // per-stage path: K1, K2, K3, two field buffers, and for D = 256 the
  // scratch matrix M of the big-cluster kernels; fused paths: the status
  // word (first 256 bytes, kept intact by every other call) and the
  // exchange words; observables: records and per-trajectory values after
  // the first 256 bytes
  const size_t rk = cdtwa::step_workspace_bytes(P);
  // a packed plan's observables run on an unpacked copy of the state
  const size_t ob = kStatusBytes + align256(P->rec_bytes) + align256(P->ptraj_bytes) + unpacked_bytes(P);
  *bytes = rk > ob ? rk : ob;
  return CDTWA_OK;
}

cdtwa_status cdtwa_sample_noise(cdtwa_plan P, uint64_t seed, int64_t traj_offset, int8_t* noise, void* rho,
                                void* stream) {
  if (!P || !rho) return fail(CDTWA_EINVAL, "sample_noise: NULL argument");
  if (traj_offset < 0) return fail(CDTWA_EINVAL, "sample_noise: negative trajectory offset");
  hipError_t e = generic_sample(P->g, P->p.dtype, seed, traj_offset, noise, rho, (hipStream_t)stream);
  return e == hipSuccess ? CDTWA_OK : hip_fail(e, "sample_noise");
}

// b_j = Tr(a_j rho_C) (model 0) or Tr(s^z_j rho_C) (model 1)
static hipError_t site_fields(cdtwa_plan P, const void* rho, void* b, hipStream_t s) {
  if (P->p.model == 1) return spin_site_fields(P->g, P->p.dtype, rho, b, s);
  if (big_supported(P->g.d, P->g.cx, P->g.cy)) return big_site_fields(P->g, P->p.dtype, P->p.layout, rho, b, s);
  return generic_site_fields(P->g, P->p.dtype, rho, b, s);
}

cdtwa_status cdtwa_gather_boundary_fields(cdtwa_plan P, const void* rho, void* b, void* phi, void* stream) {
  if (!P || !rho || !b || !phi) return fail(CDTWA_EINVAL, "gather_boundary_fields: NULL argument");
  hipError_t e = site_fields(P, rho, b, (hipStream_t)stream);
  if (e == hipSuccess) e = generic_boundary_fields(P->g, P->p.dtype, b, phi, (hipStream_t)stream);
  return e == hipSuccess ? CDTWA_OK : hip_fail(e, "gather_boundary_fields");
}

cdtwa_status cdtwa_commutator(cdtwa_plan P, const void* rho, void* K, void* ws, void* stream) {
  if (!P || !rho || !K || !ws) return fail(CDTWA_EINVAL, "commutator: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if (big_supported(P->g.d, P->g.cx, P->g.cy)) {
    const hipError_t eb = big_commutator(P->g, P->p.dtype, P->p.layout, rho, K, ws, s);
    return eb == hipSuccess ? CDTWA_OK : hip_fail(eb, "commutator");
  }
  void* b = ws;
  hipError_t e = site_fields(P, rho, b, s);
  if (e == hipSuccess && P->p.model == 1) {
    e = spin_stage(P->g, P->p.dtype, const_cast<void*>(rho), nullptr, nullptr, nullptr, K, b, nullptr, 0.0, 0, s);
  } else if (e == hipSuccess && P->path == 3) {
    e = dense_stage(P->g, P->p.dtype, const_cast<void*>(rho), nullptr, nullptr, nullptr, K, b, nullptr, 0.0, 0, s);
  } else if (e == hipSuccess) {
    e = generic_stage(P->g, P->p.dtype, const_cast<void*>(rho), nullptr, nullptr, nullptr, K, b, nullptr, 0.0, 0, s);
  }
  return e == hipSuccess ? CDTWA_OK : hip_fail(e, "commutator");
}

// n_steps RK4 steps; c1, c2 (nullable): the couplings (J, U) -- (J, h) for
// the Ising model -- at every half step, 2 n_steps + 1 values each
static cdtwa_status step_impl(cdtwa_plan P, void* rho, void* ws, double dt, int32_t n_steps, const double* c1,
                              const double* c2, hipStream_t s) {
  char* w = (char*)ws;
  if (P->path == 1 || P->path == 2 || P->path == 5) {
    int* status = (int*)w;
    uint64_t* xch = (uint64_t*)(w + kStatusBytes);
    auto launch = [&](int32_t first, int32_t m) {
      const double* sJ = c1 ? c1 + 2 * first : nullptr;
      const double* sU = c2 ? c2 + 2 * first : nullptr;
      if (P->path == 5)
        return spin_fused_rk4(P->g, P->p.dtype, rho, xch, status, P->legs, P->G, dt, m, P->spin_limit, sJ, sU,
                              first == 0, s);
      return P->path == 2
                 ? plaq_rk4(P->g, P->p.dtype, rho, xch, status, P->legs, P->G, dt, m, P->spin_limit, sJ, sU,
                            first == 0, s)
                 : fused_rk4(P->g, P->p.dtype, rho, xch, status, P->legs, P->G, dt, m, P->spin_limit, sJ, sU,
                             first == 0, P->wide, s);
    };
    hipError_t e = hipSuccess;
    if (!c1) {
      e = launch(0, n_steps);
    } else {
      // the schedule travels in the kernel arguments: launches of at most
      // kSchedSteps steps
      for (int32_t first = 0; first < n_steps && e == hipSuccess; first += kSchedSteps)
        e = launch(first, std::min<int32_t>(kSchedSteps, n_steps - first));
    }
    return e == hipSuccess ? CDTWA_OK : hip_fail(e, "step_rk4 (fused)");
  }
  if (P->path == 6 && !c1) {
    // the counter of the work queue sits where the per-stage path keeps K1
    const hipError_t et = traj_rk4(P->g, P->p.dtype, rho, (int*)w, dt, n_steps, s);
    return et == hipSuccess ? CDTWA_OK : hip_fail(et, "step_rk4 (trajectory-resident)");
  }
  if (big_supported(P->g.d, P->g.cx, P->g.cy)) {
    const hipError_t eb = big_rk4(P->g, P->p.dtype, P->p.layout, rho, nullptr, ws, dt, n_steps, c1, c2, s);
    return eb == hipSuccess ? CDTWA_OK : hip_fail(eb, "step_rk4");
  }
  const size_t S = align256(P->state_bytes), F = align256(P->field_bytes);
  // couplings of half step hs (the plan's own without a schedule)
  auto geom_at = [&](int64_t hs) {
    Geom g = P->g;
    if (c1) {
      g.J = c1[hs];
      if (P->g.model == 1)
        g.h = c2[hs];
      else
        g.U = c2[hs];
    }
    return g;
  };
  auto stage = [&](const Geom& g, void* kp, void* q1, void* q2, void* ko, void* bi, void* bo, int mode) {
    if (P->path == 3) return dense_stage(g, P->p.dtype, rho, kp, q1, q2, ko, bi, bo, dt, mode, s);
    if (P->path == 4) return spin_stage(g, P->p.dtype, rho, kp, q1, q2, ko, bi, bo, dt, mode, s);
    return generic_stage(g, P->p.dtype, rho, kp, q1, q2, ko, bi, bo, dt, mode, s);
  };
  void* K1 = w;
  void* K2 = w + S;
  void* K3 = w + 2 * S;
  void* bA = w + 3 * S;
  void* bB = w + 3 * S + F;
  hipError_t e = site_fields(P, rho, bA, s);
  for (int32_t it = 0; it < n_steps && e == hipSuccess; ++it) {
    const Geom g0 = geom_at(2 * (int64_t)it), gh = geom_at(2 * (int64_t)it + 1), g1 = geom_at(2 * (int64_t)it + 2);
    e = stage(g0, nullptr, nullptr, nullptr, K1, bA, bB, 1);
    if (e == hipSuccess) e = stage(gh, K1, nullptr, nullptr, K2, bB, bA, 2);
    if (e == hipSuccess) e = stage(gh, K2, nullptr, nullptr, K3, bA, bB, 3);
    if (e == hipSuccess) e = stage(g1, K3, K1, K2, nullptr, bB, bA, 4);
  }
  return e == hipSuccess ? CDTWA_OK : hip_fail(e, "step_rk4");
}

cdtwa_status cdtwa_step_rk4(cdtwa_plan P, void* rho, void* ws, double dt, int32_t n_steps, void* stream) {
  if (!P || !rho || !ws) return fail(CDTWA_EINVAL, "step_rk4: NULL argument");
  if (!(std::isfinite(dt) && dt > 0)) return fail(CDTWA_EINVAL, "step_rk4: dt must be finite and positive");
  if (n_steps < 0) return fail(CDTWA_EINVAL, "step_rk4: negative n_steps");
  if (n_steps == 0) return CDTWA_OK;
  return step_impl(P, rho, ws, dt, n_steps, nullptr, nullptr, (hipStream_t)stream);
}

cdtwa_status cdtwa_step_rk4_compensated(cdtwa_plan P, void* rho, void* rho_lo, void* ws, double dt, int32_t n_steps,
                                        void* stream) {
  if (!P || !rho || !rho_lo || !ws) return fail(CDTWA_EINVAL, "step_rk4_compensated: NULL argument");
  if (!(std::isfinite(dt) && dt > 0)) return fail(CDTWA_EINVAL, "step_rk4_compensated: dt must be finite and positive");
  if (n_steps < 0) return fail(CDTWA_EINVAL, "step_rk4_compensated: negative n_steps");
  if (P->p.dtype != CDTWA_F32 || !big_supported(P->g.d, P->g.cx, P->g.cy))
    return fail(CDTWA_EUNSUPPORTED, "step_rk4_compensated: needs an FP32 plan with 2x2 clusters and d = 4");
  if (n_steps == 0) return CDTWA_OK;
  const hipError_t e =
      big_rk4(P->g, P->p.dtype, P->p.layout, rho, rho_lo, ws, dt, n_steps, nullptr, nullptr, (hipStream_t)stream);
  return e == hipSuccess ? CDTWA_OK : hip_fail(e, "step_rk4_compensated");
}

}  // extern "C"

namespace cdtwa {
// Bytes of workspace that the RK4 steps alone use (the status word and the
// exchange words of the fused paths; K1, K2, K3, the field buffers and, for
// D = 256, the scratch matrix M of the per-stage paths).
size_t step_workspace_bytes(cdtwa_plan P) {
  if (big_supported(P->g.d, P->g.cx, P->g.cy)) return big_workspace_bytes(P->g, P->p.dtype);
  const bool fused = P->path == 1 || P->path == 2 || P->path == 5;
  return fused ? kStatusBytes + align256(fused_exchange_words(P->g.nc, P->G) * 8)
               : 3 * align256(P->state_bytes) + 2 * align256(P->field_bytes);
}
// cdtwa_step_rk4 on a workspace the caller has already validated
cdtwa_status step_rk4_checked(cdtwa_plan P, void* rho, void* ws, double dt, int32_t n_steps, hipStream_t s) {
  return step_impl(P, rho, ws, dt, n_steps, nullptr, nullptr, s);
}
}  // namespace cdtwa

extern "C" {

cdtwa_status cdtwa_step_rk4_schedule(cdtwa_plan P, void* rho, void* ws, double dt, int32_t n_steps,
                                     const double* c1_half, const double* c2_half, void* stream) {
  if (!P || !rho || !ws || !c1_half || !c2_half) return fail(CDTWA_EINVAL, "step_rk4_schedule: NULL argument");
  if (!(std::isfinite(dt) && dt > 0)) return fail(CDTWA_EINVAL, "step_rk4_schedule: dt must be finite and positive");
  if (n_steps < 0) return fail(CDTWA_EINVAL, "step_rk4_schedule: negative n_steps");
  for (int64_t k = 0; k <= 2 * (int64_t)n_steps; ++k)
    if (!(std::isfinite(c1_half[k]) && std::isfinite(c2_half[k])))
      return fail(CDTWA_EINVAL, "step_rk4_schedule: couplings must be finite");
  if (n_steps == 0) return CDTWA_OK;
  return step_impl(P, rho, ws, dt, n_steps, c1_half, c2_half, (hipStream_t)stream);
}

cdtwa_status cdtwa_plan_path(cdtwa_plan P, int32_t* path, int32_t* resident) {
  if (!P || !path) return fail(CDTWA_EINVAL, "plan_path: NULL argument");
  *path = P->path;
  if (resident) *resident = P->G;
  return CDTWA_OK;
}

cdtwa_status cdtwa_device_status(cdtwa_plan P, const void* ws, int32_t* status, void* stream) {
  if (!P || !ws || !status) return fail(CDTWA_EINVAL, "device_status: NULL argument");
  *status = 0;
  if (P->path != 1 && P->path != 2 && P->path != 5) return CDTWA_OK;
  const char* w = (const char*)ws;
  const int* dev = (const int*)w;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(status, dev, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? CDTWA_OK : hip_fail(e, "device_status");
}

cdtwa_status cdtwa_accumulate_observables(cdtwa_plan P, const void* rho, int32_t t_index, double* sums,
                                          double* per_traj, void* ws, void* stream) {
  if (!P || !rho || !sums || !ws) return fail(CDTWA_EINVAL, "accumulate_observables: NULL argument");
  if (t_index < 0) return fail(CDTWA_EINVAL, "accumulate_observables: negative t_index");
  hipStream_t s = (hipStream_t)stream;
  double* rec = (double*)((char*)ws + kStatusBytes);
  double* pt = per_traj ? per_traj : (double*)((char*)ws + kStatusBytes + align256(P->rec_bytes));
  hipError_t e = hipSuccess;
  if (P->p.layout == CDTWA_LAYOUT_PACKED_UPPER) {
    // the observable kernels read full matrices: unpack into the workspace
    void* full = (char*)ws + kStatusBytes + align256(P->rec_bytes) + align256(P->ptraj_bytes);
    e = big_unpack(P->g, P->p.dtype, rho, full, s);
    rho = full;
  }
  if (e == hipSuccess)
    e = P->p.model == 1 ? spin_observables(P->g, P->p.dtype, rho, rec, pt, s)
                        : generic_observables(P->g, P->p.dtype, rho, rec, pt, s);
  // the cluster records are consumed by now: their space holds the chunk partials
  if (e == hipSuccess) e = launch_obs_sum(pt, P->g.n_traj, sums + (size_t)t_index * kNObs * 3, rec, s);
  return e == hipSuccess ? CDTWA_OK : hip_fail(e, "accumulate_observables");
}

cdtwa_status cdtwa_cv_targets(cdtwa_plan P, const void* rho, int32_t column, float* targets, void* ws,
                              void* stream) {
  if (!P || !rho || !targets || !ws) return fail(CDTWA_EINVAL, "cv_targets: NULL argument");
  if (P->g.cx != 2 || P->g.cy != 2 || P->g.model != 0 || P->p.layout != CDTWA_LAYOUT_FULL)
    return fail(CDTWA_EUNSUPPORTED, "cv_targets: needs the Bose-Hubbard model with 2x2 clusters (full layout)");
  if (column < 0 || column >= CDTWA_MLP_OUT) return fail(CDTWA_EINVAL, "cv_targets: column out of range");
  hipStream_t s = (hipStream_t)stream;
  double* rec = (double*)((char*)ws + kStatusBytes);
  double* pt = (double*)((char*)ws + kStatusBytes + align256(P->rec_bytes));
  hipError_t e = generic_observables(P->g, P->p.dtype, rho, rec, pt, s);
  if (e == hipSuccess) e = cv_targets(P->g, rec, targets, CDTWA_MLP_OUT, column, s);
  return e == hipSuccess ? CDTWA_OK : hip_fail(e, "cv_targets");
}

}  // extern "C"
