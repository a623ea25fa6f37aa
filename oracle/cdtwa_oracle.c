/*
 * cdtwa_oracle.c -- plain FP64 CPU oracle for the cluster discrete truncated
 * Wigner approximation (C-dTWA) of Nagao & Yunoki, arXiv:2404.18594, applied to
 * the Bose-Hubbard model truncated to d levels per site.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
 * that the GPU library is checked against.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header or table with the GPU library.
 *
 * What it computes, in the paper's order:
 *   1. discrete phase-point sampling of every site (Sec. II, onsite expansion of
 *      A_j and the tomography probabilities; App. B.1, "ansatz" A_j = I/3 +
 *      (1/2) sum_a r^a T_a and the eigen-decomposition rule p^a_j(n)),
 *   2. cluster phase-point matrices as Kronecker products of the onsite A_j
 *      (Sec. II Eq. (rho_t); App. B.1, factorised initial cluster matrices),
 *   3. the cluster mean-field equation of motion
 *        d/dt A_mu = -i [ Gamma^intra_mu + Phi^inter_mu , A_mu ]
 *      (Sec. II Eq. (cluster_mf); App. B.1 Eq. (app:eom_cdtwa)) with
 *      Gamma^intra the on-site interaction plus the intra-cluster hops and
 *      Phi^inter the hops to neighbouring clusters with the neighbour replaced
 *      by its cluster mean field <a_k> = Tr(a_k A_nu),
 *   4. classical fourth-order Runge-Kutta on all clusters of a trajectory
 *      jointly (App. B.1, last paragraph),
 *   5. per-trajectory estimators of <a_i^dag a_j> and <n_i n_j> whose average
 *      over trajectories approximates the quantum expectation (Sec. II,
 *      rho(t) ~ average of the product of cluster matrices; Sec. III,
 *      definition of C^sp).
 *
 * Everything is dense: operators are D x D matrices built from Kronecker
 * products of d x d matrices; the commutator is two matrix products H Y and
 * Y H (zero entries of H are skipped, nothing else is restructured).
 *
 * Conventions (readings where the paper is silent; each is also listed in the
 * design notes):
 *   - site j = y*Lx + x; cluster (mx,my) = (x/cx, y/cy), index my*(Lx/cx)+mx;
 *     local index l = (x%cx)*cy + (y%cy), local 0 is the most significant
 *     Kronecker factor.  For 2x2 clusters this puts paper sites 1..4 at local
 *     (x,y) = (0,0),(0,1),(1,0),(1,1), the only placement consistent with the
 *     eight legs of Phi^inter in App. B.1.
 *   - random draws: Philox-4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (a/4, site, traj_lo, traj_hi), word a%4 for generator a.
 *     The outcome is the first distinct eigenvalue n of T_a (ascending) with
 *     x < thr[a][n], thr = round(2^32 * cumulative probability).
 *   - each generator of a site is drawn independently.
 *   - observables use minimum-image displacements on periodic lattices.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_MAXD 4      /* local dimension d                     */
#define ORC_MAXGEN 15   /* d*d - 1                               */
#define ORC_MAXLOC 4    /* sites per cluster                     */
#define ORC_NOBS 15     /* per-trajectory observables, see below */

enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ENOMEM = -4
};

/* ------------------------------------------------------------------------ */
/* Problem and derived geometry                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
  int Lx, Ly;     /* lattice sides                               */
  int cx, cy;     /* cluster shape                               */
  int d;          /* local dimension n_max + 1                   */
  int periodic;   /* 1 periodic, 0 open                          */
  double J, U;    /* model 0: H = -J sum_<ij> (a_i^+ a_j + h.c.) + U/2 sum n(n-1) */
  int model;      /* 0 Bose-Hubbard (Sec. III), 1 transverse-field Ising (App. A) */
  double h;       /* model 1: H = J sum_<ij> s^z_i s^z_j + h sum_i s^x_i (d = 2)  */
  int init_state; /* 0 the same onsite state everywhere (Mott |1>, or |up>);
                     1 Neel: |up> where x+y is even, |down> elsewhere (model 1)   */
  double gdeph;   /* model 0: Lindblad rate of on-site dephasing, L_j = n_j       */
  double gloss;   /* model 0: Lindblad rate of on-site particle loss, L_j = a_j   */
} orc_problem;

typedef struct {
  orc_problem p;
  int Ns, ncx, ncy, nc, nloc, D;
  int *site_cluster;   /* [Ns]            cluster of each site            */
  int *site_local;     /* [Ns]            local index of each site        */
  int *cluster_site;   /* [nc][nloc]      site of (cluster, local)        */
  int *nbr;            /* [Ns][4]         lattice neighbours, -1 if none  */
  int nbond_intra;     /* intra-cluster bonds (local pairs)               */
  int bond_intra[16][2];
  /* embedded operators, D x D, real entries stored as complex              */
  cplx *Bl;            /* [nloc][D*D]  a_l   (annihilation on local l)     */
  cplx *Bdl;           /* [nloc][D*D]  a_l^dagger                         */
  cplx *Nl;            /* [nloc][D*D]  n_l                                */
  cplx *H0;            /* [D*D]        Gamma^intra at the problem's couplings */
  cplx *Hc1, *Hc2;     /* [D*D]        Gamma^intra = c1 Hc1 + c2 Hc2 with
                          (c1, c2) = (J, U): Hc1 = -(intra hops), Hc2 = sum_l h_l;
                          (c1, c2) = (J, h): Hc1 = sum_bonds s^z s^z, Hc2 = sum_l s^x */
  cplx *Sy;            /* [nloc][D*D]  model 1: s^y_l (observables)        */
} orc_geom;

static int valid_problem(const orc_problem *p) {
  if (p->Lx < 1 || p->Ly < 1) return 0;
  if (p->cx < 1 || p->cx > 2 || p->cy < 1 || p->cy > 2) return 0;
  if (p->Lx % p->cx || p->Ly % p->cy) return 0;
  if (p->d < 2 || p->d > ORC_MAXD) return 0;
  if (p->model < 0 || p->model > 1 || p->init_state < 0 || p->init_state > 1) return 0;
  if (p->model == 1 && p->d != 2) return 0;
  if (p->model == 0 && p->init_state != 0) return 0;
  if (!(p->gdeph >= 0) || !(p->gloss >= 0)) return 0;
  if (p->model == 1 && (p->gdeph != 0 || p->gloss != 0)) return 0;
  if (p->periodic) {
    /* a periodic direction needs two clusters and three sites, otherwise a
       cluster couples to itself through the mean field or a bond repeats */
    if (p->Lx / p->cx < 2 || p->Ly / p->cy < 2) return 0;
    if (p->Lx < 3 || p->Ly < 3) return 0;
  }
  return 1;
}

/* the second coupling of the model: U (Bose-Hubbard) or h (Ising) */
static double coupling2(const orc_problem *p) { return p->model == 1 ? p->h : p->U; }

/* dense Kronecker product C = A (m x m) (x) B (n x n) */
static void kron(const cplx *A, int m, const cplx *B, int n, cplx *C) {
  int mn = m * n;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      for (int k = 0; k < n; ++k)
        for (int l = 0; l < n; ++l)
          C[(i * n + k) * mn + (j * n + l)] = A[i * m + j] * B[k * n + l];
}

/* I (x) ... (x) O (x) ... (x) I with O at position pos of nloc factors */
static void embed(const cplx *O, int d, int pos, int nloc, cplx *out) {
  int D = 1;
  for (int i = 0; i < nloc; ++i) D *= d;
  cplx *cur = calloc((size_t)D * D, sizeof(cplx));
  cplx *nxt = calloc((size_t)D * D, sizeof(cplx));
  cplx Id[ORC_MAXD * ORC_MAXD];
  memset(Id, 0, sizeof(Id));
  for (int i = 0; i < d; ++i) Id[i * d + i] = 1.0;
  int dim = 1;
  cur[0] = 1.0;
  for (int f = 0; f < nloc; ++f) {
    const cplx *F = (f == pos) ? O : Id;
    kron(cur, dim, F, d, nxt);
    dim *= d;
    cplx *t = cur; cur = nxt; nxt = t;
  }
  memcpy(out, cur, (size_t)D * D * sizeof(cplx));
  free(cur);
  free(nxt);
}

/* C = A B for D x D matrices */
static void matmul(const cplx *A, const cplx *B, cplx *C, int D) {
  for (int i = 0; i < D * D; ++i) C[i] = 0;
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k) {
      cplx a = A[i * D + k];
      if (a == 0) continue;
      for (int j = 0; j < D; ++j) C[i * D + j] += a * B[k * D + j];
    }
}

static void geom_free(orc_geom *g) {
  free(g->site_cluster); free(g->site_local); free(g->cluster_site); free(g->nbr);
  free(g->Bl); free(g->Bdl); free(g->Nl); free(g->H0); free(g->Sy); free(g->Hc1); free(g->Hc2);
  memset(g, 0, sizeof(*g));
}

static int geom_init(const orc_problem *p, orc_geom *g) {
  memset(g, 0, sizeof(*g));
  if (!valid_problem(p)) return ORC_EINVAL;
  g->p = *p;
  g->Ns = p->Lx * p->Ly;
  g->ncx = p->Lx / p->cx;
  g->ncy = p->Ly / p->cy;
  g->nc = g->ncx * g->ncy;
  g->nloc = p->cx * p->cy;
  g->D = 1;
  for (int i = 0; i < g->nloc; ++i) g->D *= p->d;
  int D = g->D, d = p->d;

  g->site_cluster = malloc(sizeof(int) * g->Ns);
  g->site_local = malloc(sizeof(int) * g->Ns);
  g->cluster_site = malloc(sizeof(int) * g->nc * g->nloc);
  g->nbr = malloc(sizeof(int) * g->Ns * 4);
  for (int y = 0; y < p->Ly; ++y)
    for (int x = 0; x < p->Lx; ++x) {
      int j = y * p->Lx + x;
      int mu = (y / p->cy) * g->ncx + (x / p->cx);
      int l = (x % p->cx) * p->cy + (y % p->cy);
      g->site_cluster[j] = mu;
      g->site_local[j] = l;
      g->cluster_site[mu * g->nloc + l] = j;
      int dx[4] = {+1, -1, 0, 0}, dy[4] = {0, 0, +1, -1};
      for (int k = 0; k < 4; ++k) {
        int xx = x + dx[k], yy = y + dy[k];
        if (p->periodic) {
          xx = (xx + p->Lx) % p->Lx;
          yy = (yy + p->Ly) % p->Ly;
        } else if (xx < 0 || xx >= p->Lx || yy < 0 || yy >= p->Ly) {
          g->nbr[j * 4 + k] = -1;
          continue;
        }
        g->nbr[j * 4 + k] = yy * p->Lx + xx;
      }
    }
  /* intra-cluster bonds: pairs of local sites at unit distance */
  g->nbond_intra = 0;
  for (int l = 0; l < g->nloc; ++l)
    for (int m = l + 1; m < g->nloc; ++m) {
      int xl = l / p->cy, yl = l % p->cy, xm = m / p->cy, ym = m % p->cy;
      if (abs(xl - xm) + abs(yl - ym) == 1) {
        g->bond_intra[g->nbond_intra][0] = l;
        g->bond_intra[g->nbond_intra][1] = m;
        g->nbond_intra++;
      }
    }

  /* local operators: a = sum_n sqrt(n)|n-1><n|, a^dagger, n, h = n(n-1)/2 */
  cplx a[ORC_MAXD * ORC_MAXD], ad[ORC_MAXD * ORC_MAXD], nn[ORC_MAXD * ORC_MAXD], hint[ORC_MAXD * ORC_MAXD];
  memset(a, 0, sizeof(a)); memset(ad, 0, sizeof(ad)); memset(nn, 0, sizeof(nn)); memset(hint, 0, sizeof(hint));
  for (int n = 1; n < d; ++n) {
    a[(n - 1) * d + n] = sqrt((double)n);
    ad[n * d + (n - 1)] = sqrt((double)n);
  }
  for (int n = 0; n < d; ++n) {
    nn[n * d + n] = n;
    hint[n * d + n] = 0.5 * n * (n - 1);
  }
  size_t DD = (size_t)D * D;
  g->Bl = calloc(DD * g->nloc, sizeof(cplx));
  g->Bdl = calloc(DD * g->nloc, sizeof(cplx));
  g->Nl = calloc(DD * g->nloc, sizeof(cplx));
  g->H0 = calloc(DD, sizeof(cplx));
  g->Hc1 = calloc(DD, sizeof(cplx));
  g->Hc2 = calloc(DD, sizeof(cplx));
  cplx *tmp = calloc(DD, sizeof(cplx));
  cplx *tmp2 = calloc(DD, sizeof(cplx));
  for (int l = 0; l < g->nloc; ++l) {
    embed(a, d, l, g->nloc, g->Bl + DD * l);
    embed(ad, d, l, g->nloc, g->Bdl + DD * l);
    embed(nn, d, l, g->nloc, g->Nl + DD * l);
    embed(hint, d, l, g->nloc, tmp);
    for (size_t i = 0; i < DD; ++i) g->Hc2[i] += tmp[i];
  }
  for (int b = 0; b < g->nbond_intra; ++b) {
    int l = g->bond_intra[b][0], m = g->bond_intra[b][1];
    matmul(g->Bdl + DD * l, g->Bl + DD * m, tmp, D);   /* a_l^+ a_m */
    matmul(g->Bdl + DD * m, g->Bl + DD * l, tmp2, D);  /* a_m^+ a_l */
    for (size_t i = 0; i < DD; ++i) g->Hc1[i] += -(tmp[i] + tmp2[i]);
  }
  free(tmp);
  free(tmp2);
  if (p->model == 1) {
    /* Pauli operators, basis |0> = |up> (s^z = +1), |1> = |down>:
       B = B^+ = s^z (the mean field is <s^z>), N = s^x, Sy = s^y,
       Gamma^intra = J sum_bonds s^z s^z + h sum_l s^x                       */
    cplx sz[4] = {1, 0, 0, -1}, sx[4] = {0, 1, 1, 0}, sy[4] = {0, -I, I, 0};
    g->Sy = calloc(DD * g->nloc, sizeof(cplx));
    memset(g->Hc1, 0, DD * sizeof(cplx));
    memset(g->Hc2, 0, DD * sizeof(cplx));
    cplx *t3 = calloc(DD, sizeof(cplx));
    for (int l = 0; l < g->nloc; ++l) {
      embed(sz, 2, l, g->nloc, g->Bl + DD * l);
      embed(sz, 2, l, g->nloc, g->Bdl + DD * l);
      embed(sx, 2, l, g->nloc, g->Nl + DD * l);
      embed(sy, 2, l, g->nloc, g->Sy + DD * l);
      for (size_t i = 0; i < DD; ++i) g->Hc2[i] += g->Nl[DD * l + i];
    }
    for (int b = 0; b < g->nbond_intra; ++b) {
      int l = g->bond_intra[b][0], m = g->bond_intra[b][1];
      matmul(g->Bl + DD * l, g->Bl + DD * m, t3, D);
      for (size_t i = 0; i < DD; ++i) g->Hc1[i] += t3[i];
    }
    free(t3);
  }
  for (size_t i = 0; i < DD; ++i) g->H0[i] = p->J * g->Hc1[i] + coupling2(p) * g->Hc2[i];
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                        */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Sampling tables (built by the Python side from the generator basis)      */
/* ------------------------------------------------------------------------ */

typedef struct {
  int n_gen;                          /* number of generators T_a                    */
  const double *T;                    /* [n_gen][d][d][2] generator matrices         */
  const int *n_out;                   /* [n_class][n_gen] distinct outcomes          */
  const double *val;                  /* [n_class][n_gen][ORC_MAXD] outcome values   */
  const uint64_t *thr;                /* [n_class][n_gen][ORC_MAXD] thresholds       */
  double g_norm;                      /* g = Tr(T_a^2)                               */
} orc_tables;

/* onsite-state class of a site: 0 everywhere, or the Neel sublattice */
static int site_class(const orc_geom *g, int j) {
  if (g->p.init_state != 1) return 0;
  return ((j % g->p.Lx) + (j / g->p.Lx)) % 2;
}

/* Draw every generator of every site of one trajectory and build the onsite
   phase-point matrices A_j = I/d + (1/g) sum_a r^a T_a.                     */
static void sample_sites(const orc_geom *g, const orc_tables *tb, uint64_t seed, int64_t traj,
                         int8_t *codes /* [Ns][n_gen] or NULL */, cplx *A /* [Ns][d*d] */) {
  int d = g->p.d;
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int j = 0; j < g->Ns; ++j) {
    cplx *Aj = A + (size_t)j * d * d;
    for (int i = 0; i < d * d; ++i) Aj[i] = 0;
    for (int i = 0; i < d; ++i) Aj[i * d + i] = 1.0 / d;
    const int c = site_class(g, j);
    for (int a = 0; a < tb->n_gen; ++a) {
      const int ca = c * tb->n_gen + a;
      uint32_t ctr[4] = {(uint32_t)(a / 4), (uint32_t)j, (uint32_t)((uint64_t)traj), (uint32_t)((uint64_t)traj >> 32)};
      uint32_t w[4];
      orc_philox4x32_10(ctr, key, w);
      uint32_t x = w[a % 4];
      int n = 0;
      while (n < tb->n_out[ca] - 1 && !((uint64_t)x < tb->thr[ca * ORC_MAXD + n])) ++n;
      if (codes) codes[(size_t)j * tb->n_gen + a] = (int8_t)n;
      double r = tb->val[ca * ORC_MAXD + n];
      const double *Ta = tb->T + (size_t)a * d * d * 2;
      for (int i = 0; i < d * d; ++i) Aj[i] += (r / tb->g_norm) * (Ta[2 * i] + I * Ta[2 * i + 1]);
    }
  }
}

/* A_mu = A_{site(mu,0)} (x) A_{site(mu,1)} (x) ... */
static void cluster_product(const orc_geom *g, const cplx *A, int mu, cplx *out) {
  int d = g->p.d, D = g->D;
  cplx *cur = calloc((size_t)D * D, sizeof(cplx));
  cplx *nxt = calloc((size_t)D * D, sizeof(cplx));
  int dim = 1;
  cur[0] = 1.0;
  for (int l = 0; l < g->nloc; ++l) {
    int j = g->cluster_site[mu * g->nloc + l];
    kron(cur, dim, A + (size_t)j * d * d, d, nxt);
    dim *= d;
    cplx *t = cur; cur = nxt; nxt = t;
  }
  memcpy(out, cur, (size_t)D * D * sizeof(cplx));
  free(cur);
  free(nxt);
}

/* ------------------------------------------------------------------------ */
/* Cluster mean fields and the equation of motion                            */
/* ------------------------------------------------------------------------ */

/* Tr(O Y) for D x D matrices */
static cplx trace_prod(const cplx *O, const cplx *Y, int D) {
  cplx s = 0;
  for (int p = 0; p < D; ++p)
    for (int q = 0; q < D; ++q) {
      cplx o = O[p * D + q];
      if (o == 0) continue;
      s += o * Y[q * D + p];
    }
  return s;
}

/* b_j = Tr(a_j A_mu(j)) for every site of one trajectory (Sec. II, cluster
   mean fields <s_j>_{S_nu} = Tr[s_j A_nu]).                                 */
static void site_fields(const orc_geom *g, const cplx *rho /* [nc][D*D] */, cplx *b /* [Ns] */) {
  size_t DD = (size_t)g->D * g->D;
  for (int j = 0; j < g->Ns; ++j) {
    int mu = g->site_cluster[j], l = g->site_local[j];
    b[j] = trace_prod(g->Bl + DD * l, rho + DD * mu, g->D);
  }
}

/* phi_j = sum of b_k over lattice neighbours k of j in other clusters */
static void boundary_fields(const orc_geom *g, const cplx *b, cplx *phi) {
  for (int j = 0; j < g->Ns; ++j) {
    phi[j] = 0;
    for (int k = 0; k < 4; ++k) {
      int nb = g->nbr[j * 4 + k];
      if (nb < 0) continue;
      if (g->site_cluster[nb] == g->site_cluster[j]) continue;
      phi[j] += b[nb];
    }
  }
}

/* Gamma^intra_mu + Phi^inter_mu as a dense matrix.  Each leg
   -J a_i <a_k^dagger> + H.c. of App. B.1 equals -J (conj(b_k) a_i + b_k a_i^dagger). */
/* Model 1 (App. A): each bond to a site k of another cluster contributes
   J s^z_i <s^z_k>, i.e. kappa (conj(b_k) B_i + b_k B_i^+) with B = s^z,
   kappa = J/2 and b_k real. */
/* (c1, c2) = (J, U) for model 0, (J, h) for model 1, at the stage's time */
static void cluster_hamiltonian(const orc_geom *g, const cplx *phi, int mu, cplx *H, double c1, double c2) {
  size_t DD = (size_t)g->D * g->D;
  const double kappa = g->p.model == 1 ? 0.5 * c1 : -c1;
  for (size_t i = 0; i < DD; ++i) H[i] = c1 * g->Hc1[i] + c2 * g->Hc2[i];
  for (int l = 0; l < g->nloc; ++l) {
    int j = g->cluster_site[mu * g->nloc + l];
    cplx f = phi[j];
    const cplx *B = g->Bl + DD * l, *Bd = g->Bdl + DD * l;
    for (size_t i = 0; i < DD; ++i) H[i] += kappa * (conj(f) * B[i] + f * Bd[i]);
  }
}

/* K = -i (H Y - Y H) */
static void commutator_rhs(const cplx *H, const cplx *Y, cplx *K, cplx *work, int D) {
  cplx *HY = work, *YH = work + (size_t)D * D;
  matmul(H, Y, HY, D);
  for (int i = 0; i < D * D; ++i) YH[i] = 0;
  for (int r = 0; r < D; ++r)
    for (int q = 0; q < D; ++q) {
      cplx h = H[r * D + q];
      if (h == 0) continue;
      for (int p = 0; p < D; ++p) YH[p * D + q] += Y[p * D + r] * h;
    }
  for (int i = 0; i < D * D; ++i) K[i] = -I * (HY[i] - YH[i]);
}

/* Local Lindblad dissipator of the cluster matrix (the extension to open
   systems that the paper names, Sec. IV and App. B.1): for every site l of the
   cluster and channel L in {sqrt(gdeph) n_l, sqrt(gloss) a_l},
   K += L Y L^+ - (1/2) (L^+ L Y + Y L^+ L).  Dense products. */
static void dissipator_add(const orc_geom *g, const cplx *Y, cplx *K, cplx *work) {
  const int D = g->D;
  const size_t DD = (size_t)D * D;
  cplx *T1 = work, *T2 = work + DD;
  for (int l = 0; l < g->nloc; ++l)
    for (int ch = 0; ch < 2; ++ch) {
      const double gam = ch == 0 ? g->p.gdeph : g->p.gloss;
      if (gam == 0) continue;
      const cplx *L = ch == 0 ? g->Nl + DD * l : g->Bl + DD * l;
      const cplx *Ld = ch == 0 ? g->Nl + DD * l : g->Bdl + DD * l;
      matmul(L, Y, T1, D);             /* L Y          */
      matmul(T1, Ld, T2, D);           /* L Y L^+      */
      for (size_t i = 0; i < DD; ++i) K[i] += gam * T2[i];
      matmul(Ld, L, T1, D);            /* L^+ L        */
      matmul(T1, Y, T2, D);            /* L^+ L Y      */
      for (size_t i = 0; i < DD; ++i) K[i] -= 0.5 * gam * T2[i];
      matmul(Y, T1, T2, D);            /* Y L^+ L      */
      for (size_t i = 0; i < DD; ++i) K[i] -= 0.5 * gam * T2[i];
    }
}

static int has_dissipation(const orc_geom *g) { return g->p.gdeph != 0 || g->p.gloss != 0; }

/* right-hand side of the coupled cluster equations for one trajectory; the
   clusters are independent once the fields are known, so they may be spread
   over `inner` threads (each with its own H and scratch).                   */
static int g_inner_threads = 1;

static void trajectory_rhs(const orc_geom *g, const cplx *rho, cplx *K, cplx *b, cplx *phi, cplx *H, cplx *work,
                           double c1, double c2) {
  size_t DD = (size_t)g->D * g->D;
  site_fields(g, rho, b);
  boundary_fields(g, b, phi);
  int inner = g_inner_threads;
  if (inner <= 1) {
    for (int mu = 0; mu < g->nc; ++mu) {
      cluster_hamiltonian(g, phi, mu, H, c1, c2);
      commutator_rhs(H, rho + DD * mu, K + DD * mu, work, g->D);
      if (has_dissipation(g)) dissipator_add(g, rho + DD * mu, K + DD * mu, work);
    }
    return;
  }
#pragma omp parallel num_threads(inner)
  {
    cplx *Ht = malloc(sizeof(cplx) * DD), *wt = malloc(sizeof(cplx) * 2 * DD);
#pragma omp for schedule(static)
    for (int mu = 0; mu < g->nc; ++mu) {
      cluster_hamiltonian(g, phi, mu, Ht, c1, c2);
      commutator_rhs(Ht, rho + DD * mu, K + DD * mu, wt, g->D);
      if (has_dissipation(g)) dissipator_add(g, rho + DD * mu, K + DD * mu, wt);
    }
    free(Ht);
    free(wt);
  }
}

/* one classical RK4 step of all clusters of one trajectory; the couplings
   c1[k], c2[k] are those at t, t + dt/2 and t + dt (k = 0, 1, 2): stage 1
   at t, stages 2 and 3 at t + dt/2, stage 4 at t + dt (RK4 for a
   time-dependent right-hand side) */
static void trajectory_rk4(const orc_geom *g, cplx *rho, double dt, cplx *ws /* 5*nc*DD + scratch */,
                           const double c1[3], const double c2[3]) {
  size_t n = (size_t)g->nc * g->D * g->D;
  size_t DD = (size_t)g->D * g->D;
  cplx *K1 = ws, *K2 = ws + n, *K3 = ws + 2 * n, *K4 = ws + 3 * n, *Y = ws + 4 * n;
  cplx *b = ws + 5 * n, *phi = b + g->Ns, *H = phi + g->Ns, *work = H + DD;
  trajectory_rhs(g, rho, K1, b, phi, H, work, c1[0], c2[0]);
  for (size_t i = 0; i < n; ++i) Y[i] = rho[i] + 0.5 * dt * K1[i];
  trajectory_rhs(g, Y, K2, b, phi, H, work, c1[1], c2[1]);
  for (size_t i = 0; i < n; ++i) Y[i] = rho[i] + 0.5 * dt * K2[i];
  trajectory_rhs(g, Y, K3, b, phi, H, work, c1[1], c2[1]);
  for (size_t i = 0; i < n; ++i) Y[i] = rho[i] + dt * K3[i];
  trajectory_rhs(g, Y, K4, b, phi, H, work, c1[2], c2[2]);
  for (size_t i = 0; i < n; ++i) rho[i] = rho[i] + (dt / 6.0) * (K1[i] + 2.0 * K2[i] + 2.0 * K3[i] + K4[i]);
}

static size_t rk4_ws_elems(const orc_geom *g) {
  size_t DD = (size_t)g->D * g->D;
  return 5 * (size_t)g->nc * DD + 2 * (size_t)g->Ns + DD + 2 * DD;
}

/* ------------------------------------------------------------------------ */
/* Per-trajectory observables                                                */
/* ------------------------------------------------------------------------ */
/* Output layout (ORC_NOBS doubles):
 *   0..4   C^sp at (dx,dy) = (1,0),(0,1),(1,1),(2,0),(0,2):
 *          (1/Ns) sum over ordered site pairs (i,j) with |x_i-x_j| = dx and
 *          |y_i-y_j| = dy of Re <a_i^dag a_j>   (Sec. III definition)
 *   5..9   the same sums of <n_i n_j>
 *   10     (1/Ns) sum_j <n_j>
 *   11     mean-field energy per site
 *   12     mean over clusters of Tr(A_mu^2)
 *   13     max over clusters of |Tr A_mu - 1|
 *   14     max over clusters and entries of |A_pq - conj(A_qp)|
 * Pairs inside one cluster use the cluster matrix, Tr(a_i^dag a_j A_mu) and
 * Tr(n_i n_j A_mu); pairs in different clusters use the product of the
 * cluster mean fields, conj(b_i) b_j and n_i n_j, because the trajectory
 * state is the Kronecker product of its cluster matrices.                  */
static const int orc_class_dx[5] = {1, 0, 1, 2, 0};
static const int orc_class_dy[5] = {0, 1, 1, 0, 2};

static int min_image(int d, int L, int periodic) {
  if (!periodic) return abs(d);
  int m = ((d % L) + L) % L;
  if (L - m < m) m = L - m;
  return m;
}

/* obs 12..14: mean purity, trace and Hermiticity deviations */
static void invariants(const orc_geom *g, const cplx *rho, double *obs) {
  size_t DD = (size_t)g->D * g->D;
  int D = g->D;
  double pur = 0, trdev = 0, hdev = 0;
  for (int mu = 0; mu < g->nc; ++mu) {
    const cplx *Y = rho + DD * mu;
    pur += creal(trace_prod(Y, Y, D));
    cplx tr = 0;
    for (int q = 0; q < D; ++q) tr += Y[q * D + q];
    if (cabs(tr - 1.0) > trdev) trdev = cabs(tr - 1.0);
    for (int q = 0; q < D; ++q)
      for (int r = 0; r < D; ++r) {
        double h = cabs(Y[q * D + r] - conj(Y[r * D + q]));
        if (h > hdev) hdev = h;
      }
  }
  obs[12] = pur / g->nc;
  obs[13] = trdev;
  obs[14] = hdev;
}

/* Model 1 (transverse-field Ising, App. A):
 *   0      (1/Ns) sum_j (-1)^(x_j+y_j) <s^z_j>   (staggered magnetisation;
 *          App. A's M_z = Ns times this on the four-site chain)
 *   1..3   (1/Ns) sum_j <s^z_j>, <s^x_j>, <s^y_j>
 *   5..9   (1/Ns) sum over ordered pairs of the displacement classes above of
 *          <s^z_i s^z_j> (same cluster: Tr(s^z_i s^z_j A_mu); else the product)
 *   11     mean-field energy per site; 12..14 as for model 0; 4 and 10 zero. */
static void spin_observables(const orc_geom *g, const cplx *rho, double *obs, cplx *work) {
  size_t DD = (size_t)g->D * g->D;
  int D = g->D, Ns = g->Ns;
  const orc_problem *p = &g->p;
  cplx *T = work;
  double *sz = malloc(sizeof(double) * Ns);
  for (int k = 0; k < ORC_NOBS; ++k) obs[k] = 0;
  for (int j = 0; j < Ns; ++j) {
    int mu = g->site_cluster[j], l = g->site_local[j];
    sz[j] = creal(trace_prod(g->Bl + DD * l, rho + DD * mu, D));
    int x = j % p->Lx, y = j / p->Lx;
    obs[0] += ((x + y) % 2 ? -sz[j] : sz[j]) / Ns;
    obs[1] += sz[j] / Ns;
    obs[2] += creal(trace_prod(g->Nl + DD * l, rho + DD * mu, D)) / Ns;
    obs[3] += creal(trace_prod(g->Sy + DD * l, rho + DD * mu, D)) / Ns;
  }
  for (int i = 0; i < Ns; ++i) {
    int xi = i % p->Lx, yi = i / p->Lx;
    for (int j = 0; j < Ns; ++j) {
      if (j == i) continue;
      int xj = j % p->Lx, yj = j / p->Lx;
      int ax = min_image(xj - xi, p->Lx, p->periodic);
      int ay = min_image(yj - yi, p->Ly, p->periodic);
      int cls = -1;
      for (int c = 0; c < 5; ++c)
        if (ax == orc_class_dx[c] && ay == orc_class_dy[c]) cls = c;
      if (cls < 0) continue;
      double zz;
      int mi = g->site_cluster[i], mj = g->site_cluster[j];
      if (mi == mj) {
        matmul(g->Bl + DD * g->site_local[i], g->Bl + DD * g->site_local[j], T, D);
        zz = creal(trace_prod(T, rho + DD * mi, D));
      } else {
        zz = sz[i] * sz[j];
      }
      obs[5 + cls] += zz / Ns;
    }
  }
  double e = 0;
  for (int mu = 0; mu < g->nc; ++mu) e += creal(trace_prod(g->H0, rho + DD * mu, D));
  for (int i = 0; i < Ns; ++i)
    for (int k = 0; k < 4; k += 2) {
      int j = g->nbr[i * 4 + k];
      if (j < 0) continue;
      if (g->site_cluster[j] == g->site_cluster[i]) continue;
      e += p->J * sz[i] * sz[j];
    }
  obs[11] = e / Ns;
  free(sz);
}

static void trajectory_observables(const orc_geom *g, const cplx *rho, double *obs, cplx *work) {
  size_t DD = (size_t)g->D * g->D;
  int D = g->D, Ns = g->Ns;
  const orc_problem *p = &g->p;
  cplx *b = work, *T = work + Ns;
  if (p->model == 1) {
    spin_observables(g, rho, obs, T);
    invariants(g, rho, obs);
    return;
  }
  double *nloc_ = malloc(sizeof(double) * Ns);
  for (int k = 0; k < ORC_NOBS; ++k) obs[k] = 0;
  for (int j = 0; j < Ns; ++j) {
    int mu = g->site_cluster[j], l = g->site_local[j];
    b[j] = trace_prod(g->Bl + DD * l, rho + DD * mu, D);
    nloc_[j] = creal(trace_prod(g->Nl + DD * l, rho + DD * mu, D));
  }
  for (int i = 0; i < Ns; ++i) {
    int xi = i % p->Lx, yi = i / p->Lx;
    for (int j = 0; j < Ns; ++j) {
      if (j == i) continue;
      int xj = j % p->Lx, yj = j / p->Lx;
      int ax = min_image(xj - xi, p->Lx, p->periodic);
      int ay = min_image(yj - yi, p->Ly, p->periodic);
      int cls = -1;
      for (int c = 0; c < 5; ++c)
        if (ax == orc_class_dx[c] && ay == orc_class_dy[c]) cls = c;
      if (cls < 0) continue;
      double gij, nij;
      int mi = g->site_cluster[i], mj = g->site_cluster[j];
      if (mi == mj) {
        int li = g->site_local[i], lj = g->site_local[j];
        matmul(g->Bdl + DD * li, g->Bl + DD * lj, T, D);
        gij = creal(trace_prod(T, rho + DD * mi, D));
        matmul(g->Nl + DD * li, g->Nl + DD * lj, T, D);
        nij = creal(trace_prod(T, rho + DD * mi, D));
      } else {
        gij = creal(conj(b[i]) * b[j]);
        nij = nloc_[i] * nloc_[j];
      }
      obs[cls] += gij / Ns;
      obs[5 + cls] += nij / Ns;
    }
  }
  double ntot = 0;
  for (int j = 0; j < Ns; ++j) ntot += nloc_[j];
  obs[10] = ntot / Ns;
  /* mean-field energy: sum_mu Tr(Gamma^intra_mu A_mu) - J sum over lattice
     bonds between clusters of (conj(b_i) b_j + c.c.), each bond once */
  double e = 0;
  for (int mu = 0; mu < g->nc; ++mu) e += creal(trace_prod(g->H0, rho + DD * mu, D));
  for (int i = 0; i < Ns; ++i)
    for (int k = 0; k < 4; k += 2) { /* +x and +y neighbours: each bond once */
      int j = g->nbr[i * 4 + k];
      if (j < 0) continue;
      if (g->site_cluster[j] == g->site_cluster[i]) continue;
      e += -p->J * 2.0 * creal(conj(b[i]) * b[j]);
    }
  obs[11] = e / Ns;
  invariants(g, rho, obs);
  free(nloc_);
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (all arrays are C-contiguous, complex as re,im)     */
/* ------------------------------------------------------------------------ */

static int nthreads_or_default(int n) {
#ifdef _OPENMP
  return n > 0 ? n : omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* threads over trajectories; any surplus goes to clusters inside a stage */
static int split_threads(int nthreads, int64_t n_traj) {
  int total = nthreads_or_default(nthreads);
  int outer = n_traj < total ? (int)(n_traj > 0 ? n_traj : 1) : total;
  g_inner_threads = total / outer;
#ifdef _OPENMP
  if (g_inner_threads > 1) omp_set_max_active_levels(2);
#endif
  return outer;
}

int orc_geometry(const orc_problem *p, int *out /* [4] Ns, nc, nloc, D */) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  out[0] = g.Ns; out[1] = g.nc; out[2] = g.nloc; out[3] = g.D;
  geom_free(&g);
  return ORC_OK;
}

/* neighbour table and cluster maps, for the geometry pins */
int orc_maps(const orc_problem *p, int *site_cluster, int *site_local, int *nbr, int *bonds /* [16][2] */, int *nbond) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  memcpy(site_cluster, g.site_cluster, sizeof(int) * g.Ns);
  memcpy(site_local, g.site_local, sizeof(int) * g.Ns);
  memcpy(nbr, g.nbr, sizeof(int) * g.Ns * 4);
  memcpy(bonds, g.bond_intra, sizeof(int) * 2 * g.nbond_intra);
  *nbond = g.nbond_intra;
  geom_free(&g);
  return ORC_OK;
}

/* embedded operators a_l, a_l^dag, n_l and Gamma^intra, for the pins */
int orc_operators(const orc_problem *p, double *Bl, double *Bdl, double *Nl, double *H0) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  size_t DD = (size_t)g.D * g.D;
  memcpy(Bl, g.Bl, sizeof(cplx) * DD * g.nloc);
  memcpy(Bdl, g.Bdl, sizeof(cplx) * DD * g.nloc);
  memcpy(Nl, g.Nl, sizeof(cplx) * DD * g.nloc);
  memcpy(H0, g.H0, sizeof(cplx) * DD);
  geom_free(&g);
  return ORC_OK;
}

static orc_tables make_tables(int n_gen, const double *T, const int *n_out, const double *val, const uint64_t *thr, double g_norm) {
  orc_tables tb;
  tb.n_gen = n_gen; tb.T = T; tb.n_out = n_out; tb.val = val; tb.thr = thr; tb.g_norm = g_norm;
  return tb;
}

/* sampling: codes [n_traj][Ns][n_gen] (nullable), rho [n_traj][nc][D][D] complex */
int orc_sample(const orc_problem *p, int n_gen, const double *T, const int *n_out, const double *val,
               const uint64_t *thr, double g_norm, uint64_t seed, int64_t traj_offset, int64_t n_traj,
               int8_t *codes, double *rho_out, int nthreads) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  orc_tables tb = make_tables(n_gen, T, n_out, val, thr, g_norm);
  size_t DD = (size_t)g.D * g.D;
  int d = p->d;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads_or_default(nthreads))
  for (int64_t t = 0; t < n_traj; ++t) {
    cplx *A = malloc(sizeof(cplx) * g.Ns * d * d);
    sample_sites(&g, &tb, seed, traj_offset + t, codes ? codes + (size_t)t * g.Ns * n_gen : NULL, A);
    cplx *rho = (cplx *)rho_out + (size_t)t * g.nc * DD;
    for (int mu = 0; mu < g.nc; ++mu) cluster_product(&g, A, mu, rho + DD * mu);
    free(A);
  }
  geom_free(&g);
  return ORC_OK;
}

/* cluster matrices from given noise codes [n_traj][Ns][n_gen] instead of
   random draws: rho [n_traj][nc][D][D] (used to enumerate the noise).      */
int orc_build_rho(const orc_problem *p, int n_gen, const double *T, const int *n_out, const double *val,
                  double g_norm, const int8_t *codes, int64_t n_traj, double *rho_out) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  size_t DD = (size_t)g.D * g.D;
  int d = p->d;
  cplx *A = malloc(sizeof(cplx) * g.Ns * d * d);
  for (int64_t t = 0; t < n_traj; ++t) {
    for (int j = 0; j < g.Ns; ++j) {
      cplx *Aj = A + (size_t)j * d * d;
      const int c = site_class(&g, j);
      for (int i = 0; i < d * d; ++i) Aj[i] = 0;
      for (int i = 0; i < d; ++i) Aj[i * d + i] = 1.0 / d;
      for (int a = 0; a < n_gen; ++a) {
        const int ca = c * n_gen + a;
        int n = codes[((size_t)t * g.Ns + j) * n_gen + a];
        if (n < 0 || n >= n_out[ca]) { free(A); geom_free(&g); return ORC_EINVAL; }
        double r = val[ca * ORC_MAXD + n];
        const double *Ta = T + (size_t)a * d * d * 2;
        for (int i = 0; i < d * d; ++i) Aj[i] += (r / g_norm) * (Ta[2 * i] + I * Ta[2 * i + 1]);
      }
    }
    cplx *rho = (cplx *)rho_out + (size_t)t * g.nc * DD;
    for (int mu = 0; mu < g.nc; ++mu) cluster_product(&g, A, mu, rho + DD * mu);
  }
  free(A);
  geom_free(&g);
  return ORC_OK;
}

/* cluster mean fields b [n_traj][Ns] and boundary fields phi [n_traj][Ns] */
int orc_fields(const orc_problem *p, const double *rho_in, int64_t n_traj, double *b_out, double *phi_out) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  size_t DD = (size_t)g.D * g.D;
  for (int64_t t = 0; t < n_traj; ++t) {
    const cplx *rho = (const cplx *)rho_in + (size_t)t * g.nc * DD;
    cplx *b = (cplx *)b_out + (size_t)t * g.Ns, *phi = (cplx *)phi_out + (size_t)t * g.Ns;
    site_fields(&g, rho, b);
    boundary_fields(&g, b, phi);
  }
  geom_free(&g);
  return ORC_OK;
}

/* right-hand side K = -i[H_mu, A_mu] for every cluster of n_traj trajectories */
int orc_rhs(const orc_problem *p, const double *rho_in, int64_t n_traj, double *K_out, int nthreads) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  size_t DD = (size_t)g.D * g.D;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads_or_default(nthreads))
  for (int64_t t = 0; t < n_traj; ++t) {
    cplx *b = malloc(sizeof(cplx) * 2 * g.Ns), *H = malloc(sizeof(cplx) * DD), *work = malloc(sizeof(cplx) * 2 * DD);
    trajectory_rhs(&g, (const cplx *)rho_in + (size_t)t * g.nc * DD, (cplx *)K_out + (size_t)t * g.nc * DD, b, b + g.Ns, H, work,
                   g.p.J, coupling2(&g.p));
    free(b); free(H); free(work);
  }
  geom_free(&g);
  return ORC_OK;
}

/* n_steps classical RK4 steps in place */
int orc_rk4(const orc_problem *p, double *rho_io, int64_t n_traj, double dt, int n_steps, int nthreads) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  size_t DD = (size_t)g.D * g.D;
  int outer = split_threads(nthreads, n_traj);
#pragma omp parallel for schedule(dynamic) num_threads(outer)
  for (int64_t t = 0; t < n_traj; ++t) {
    cplx *ws = malloc(sizeof(cplx) * rk4_ws_elems(&g));
    cplx *rho = (cplx *)rho_io + (size_t)t * g.nc * DD;
    const double c1[3] = {g.p.J, g.p.J, g.p.J}, c2[3] = {coupling2(&g.p), coupling2(&g.p), coupling2(&g.p)};
    for (int s = 0; s < n_steps; ++s) trajectory_rk4(&g, rho, dt, ws, c1, c2);
    free(ws);
  }
  geom_free(&g);
  return ORC_OK;
}

/* n_steps RK4 steps with time-dependent couplings sampled every half step:
   c1_half[k], c2_half[k] (k = 0 .. 2 n_steps) are (J, U) -- or (J, h) for
   model 1 -- at t0 + k dt/2; step s uses entries 2s, 2s+1, 2s+2.          */
int orc_rk4_schedule(const orc_problem *p, double *rho_io, int64_t n_traj, double dt, int n_steps,
                     const double *c1_half, const double *c2_half, int nthreads) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  size_t DD = (size_t)g.D * g.D;
  int outer = split_threads(nthreads, n_traj);
#pragma omp parallel for schedule(dynamic) num_threads(outer)
  for (int64_t t = 0; t < n_traj; ++t) {
    cplx *ws = malloc(sizeof(cplx) * rk4_ws_elems(&g));
    cplx *rho = (cplx *)rho_io + (size_t)t * g.nc * DD;
    for (int s = 0; s < n_steps; ++s) trajectory_rk4(&g, rho, dt, ws, c1_half + 2 * s, c2_half + 2 * s);
    free(ws);
  }
  geom_free(&g);
  return ORC_OK;
}

/* per-trajectory observables obs [n_traj][ORC_NOBS] */
int orc_observables(const orc_problem *p, const double *rho_in, int64_t n_traj, double *obs, int nthreads) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  size_t DD = (size_t)g.D * g.D;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads_or_default(nthreads))
  for (int64_t t = 0; t < n_traj; ++t) {
    cplx *work = malloc(sizeof(cplx) * (g.Ns + DD));
    trajectory_observables(&g, (const cplx *)rho_in + (size_t)t * g.nc * DD, obs + (size_t)t * ORC_NOBS, work);
    free(work);
  }
  geom_free(&g);
  return ORC_OK;
}

/* Whole method for n_traj trajectories: sample, then n_steps RK4 steps,
   recording observables before the first step and after every step listed
   in record_steps (ascending, values in 0..n_steps; 0 = initial state).
   obs [n_traj][n_record][ORC_NOBS]; codes [n_traj][Ns][n_gen] (nullable);
   rho_final [n_traj][nc][D][D] complex (nullable).                          */
int orc_run(const orc_problem *p, int n_gen, const double *T, const int *n_out, const double *val,
            const uint64_t *thr, double g_norm, uint64_t seed, int64_t traj_offset, int64_t n_traj,
            double dt, int n_steps, const int *record_steps, int n_record, double *obs,
            int8_t *codes, double *rho_final, int nthreads) {
  orc_geom g;
  int st = geom_init(p, &g);
  if (st) return st;
  for (int r = 0; r < n_record; ++r)
    if (record_steps[r] < 0 || record_steps[r] > n_steps || (r > 0 && record_steps[r] <= record_steps[r - 1])) {
      geom_free(&g);
      return ORC_EINVAL;
    }
  orc_tables tb = make_tables(n_gen, T, n_out, val, thr, g_norm);
  size_t DD = (size_t)g.D * g.D;
  int d = p->d;
  int outer = split_threads(nthreads, n_traj);
#pragma omp parallel for schedule(dynamic) num_threads(outer)
  for (int64_t t = 0; t < n_traj; ++t) {
    cplx *A = malloc(sizeof(cplx) * g.Ns * d * d);
    cplx *rho = malloc(sizeof(cplx) * g.nc * DD);
    cplx *ws = malloc(sizeof(cplx) * rk4_ws_elems(&g));
    cplx *work = malloc(sizeof(cplx) * (g.Ns + DD));
    sample_sites(&g, &tb, seed, traj_offset + t, codes ? codes + (size_t)t * g.Ns * n_gen : NULL, A);
    for (int mu = 0; mu < g.nc; ++mu) cluster_product(&g, A, mu, rho + DD * mu);
    int rec = 0;
    const double c1[3] = {g.p.J, g.p.J, g.p.J}, c2[3] = {coupling2(&g.p), coupling2(&g.p), coupling2(&g.p)};
    for (int s = 0; s <= n_steps; ++s) {
      if (s > 0) trajectory_rk4(&g, rho, dt, ws, c1, c2);
      if (rec < n_record && record_steps[rec] == s) {
        trajectory_observables(&g, rho, obs + ((size_t)t * n_record + rec) * ORC_NOBS, work);
        ++rec;
      }
    }
    if (rho_final) memcpy((cplx *)rho_final + (size_t)t * g.nc * DD, rho, sizeof(cplx) * g.nc * DD);
    free(A); free(rho); free(ws); free(work);
  }
  geom_free(&g);
  return ORC_OK;
}

/* Outcome values of i.i.d. 4x4 site patches (the control variate's patch
   sampler): patch p = first + i, site s, generator a drawn from Philox with
   counter (a/4, s, p_lo, p_hi), key (seed_lo, seed_hi ^ 0x5bd1e995), word
   a % 4, by the same outcome rule as the trajectory sites.
   out: [n][16][n_gen] outcome values.                                      */
int orc_patch_samples(int n_gen, const int *n_out, const double *val, const uint64_t *thr, uint64_t seed,
                      int64_t first, int64_t n, double *out) {
  if (n_gen < 1 || n < 0 || first < 0) return ORC_EINVAL;
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ 0x5bd1e995u};
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t p = (uint64_t)(first + i);
    for (int s = 0; s < 16; ++s)
      for (int a = 0; a < n_gen; ++a) {
        const uint32_t ctr[4] = {(uint32_t)(a / 4), (uint32_t)s, (uint32_t)p, (uint32_t)(p >> 32)};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        const uint32_t x = w[a % 4];
        int o = 0;
        while (o < n_out[a] - 1 && !((uint64_t)x < thr[a * ORC_MAXD + o])) ++o;
        out[(i * 16 + s) * n_gen + a] = val[a * ORC_MAXD + o];
      }
  }
  return ORC_OK;
}
