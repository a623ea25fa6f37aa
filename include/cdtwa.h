/*
 * cdtwa.h -- C ABI of the MI355X (gfx950) library for the cluster discrete
 * truncated Wigner approximation (C-dTWA) of Nagao & Yunoki,
 * arXiv:2404.18594, for the Bose-Hubbard model truncated to d levels per site.
 *
 * The method (Sec. II and App. B.1): every site j of a trajectory gets a
 * random onsite phase-point matrix A_j = I/d + (1/2) sum_a r^a_j T_a with the
 * r^a_j drawn from the tomography rule; the sites are grouped into clusters
 * (cx x cy sites), each cluster carries the D x D matrix rho_C = (x)_j A_j
 * (D = d^(cx*cy)), and every cluster evolves under its cluster mean-field
 * equation  d rho_C/dt = -i [ H_C + H_MF , rho_C ]  (Sec. II Eq. (cluster_mf),
 * App. B.1 Eq. (app:eom_cdtwa)), where H_MF couples the boundary sites to the
 * mean fields b_k = Tr(a_k rho_nu) of the neighbouring clusters.  Averages
 * over trajectories of products of cluster expectations estimate the quantum
 * correlations (Sec. II, Sec. III definition of C^sp).
 *
 * Conventions shared by every entry point:
 *   - site j = y*Lx + x.  Cluster (mx,my) = (x/cx, y/cy), index my*(Lx/cx)+mx.
 *     Local index l = (x%cx)*cy + (y%cy); local 0 is the most significant
 *     Kronecker factor of rho_C (for 2x2 clusters: the paper's sites 1..4 at
 *     (x,y) = (0,0),(0,1),(1,0),(1,1), App. B.1).
 *   - complex numbers are stored as (re, im) pairs of the state precision.
 *   - rho: [n_traj][n_clusters][D][D] complex, row-major, Hermitian.
 *   - all device pointers are allocated and owned by the caller; the library
 *     never frees them.  The plan owns only its constant tables.
 *   - every call is asynchronous on the given HIP stream (NULL = legacy
 *     default stream); results are valid after the stream synchronises.  One
 *     plan is used by one stream at a time.
 *   - every call returns a status; nothing aborts or throws across the ABI.
 *     Argument errors are reported before anything is enqueued.
 */
#ifndef CDTWA_H
#define CDTWA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CDTWA_OK = 0,
  CDTWA_EINVAL = -1,       /* bad argument (NULL pointer, bad shape, bad size) */
  CDTWA_EUNSUPPORTED = -2, /* valid problem this build does not implement      */
  CDTWA_EHIP = -3,         /* HIP runtime or launch error                      */
  CDTWA_ENOMEM = -4        /* host allocation failed                           */
} cdtwa_status;

typedef enum { CDTWA_F32 = 0, CDTWA_F64 = 1 } cdtwa_dtype;

/* Problem definition.
 * H = -J sum_<ij> (a_i^+ a_j + h.c.) + U/2 sum_i n_i (n_i - 1)   (Sec. III Eq. (H_bose))
 * with occupations truncated to 0..d-1 (d = n_max + 1, Sec. III).          */
typedef struct {
  int32_t Lx, Ly;        /* lattice sides                                              */
  int32_t cx, cy;        /* cluster shape, each 1 or 2; Lx % cx == Ly % cy == 0         */
  int32_t d;             /* local dimension: 2, 3 or 4                                 */
  int32_t periodic;      /* 1 periodic (needs >= 2 clusters and >= 3 sites per side)   */
  double J, U;           /* hopping and interaction                                    */
  int32_t init_state;    /* 0 = unit-filling Mott state |1> on every site (Sec. III)   */
  int32_t dtype;         /* cdtwa_dtype of the trajectory state                        */
} cdtwa_problem;

typedef struct cdtwa_plan_s *cdtwa_plan;

/* Number of per-trajectory observables written by cdtwa_accumulate_observables. */
#define CDTWA_NOBS 15
/* Observable order (every value a double):
 *   0..4   C^sp_(dx,dy) for (dx,dy) = (1,0),(0,1),(1,1),(2,0),(0,2):
 *          (1/Ns) sum over ordered site pairs (i,j) with |x_i-x_j| = dx and
 *          |y_i-y_j| = dy (minimum image if periodic) of Re <a_i^+ a_j>
 *          (Sec. III definition of C^sp)
 *   5..9   the same sums of <n_i n_j>
 *   10     (1/Ns) sum_j <n_j>
 *   11     mean-field energy per site
 *   12     mean over clusters of Tr(rho_C^2)
 *   13     max over clusters of |Tr rho_C - 1|
 *   14     max over clusters and entries of |rho_pq - conj(rho_qp)|
 * Pairs in one cluster use Tr(a_i^+ a_j rho_C), Tr(n_i n_j rho_C); pairs in
 * different clusters use conj(b_i) b_j and n_i n_j.                        */

/* Create a plan for n_traj trajectories (n_traj >= 1).  Validates the
 * problem (CDTWA_EINVAL for inconsistent shapes, CDTWA_EUNSUPPORTED for a
 * valid shape this build does not implement), builds the geometry and the
 * sampling tables, and uploads them to the current HIP device. */
cdtwa_status cdtwa_plan_create(const cdtwa_problem *p, int64_t n_traj, cdtwa_plan *out);
cdtwa_status cdtwa_plan_destroy(cdtwa_plan plan);

/* Sizes derived from the problem: number of sites, clusters, sites per
 * cluster, cluster dimension D, generators per site (d*d-1), bytes of one
 * real of the state precision. Any output pointer may be NULL. */
cdtwa_status cdtwa_plan_info(cdtwa_plan plan, int32_t *n_sites, int32_t *n_clusters, int32_t *n_local,
                             int32_t *D, int32_t *n_gen, int32_t *real_bytes);

/* Device workspace that cdtwa_step_rk4 needs for this plan, in bytes. */
cdtwa_status cdtwa_workspace_bytes(cdtwa_plan plan, size_t *bytes);

/* a1: discrete phase-point sampling (Sec. II onsite expansion and tomography
 * rule; App. B.1 ansatz and eigen-decomposition rule; App. B.1 factorised
 * initial cluster matrices).
 * For trajectory t (global index traj_offset + t) and site j, generator a is
 * drawn from Philox-4x32-10 keyed by `seed` with counter
 * (a/4, j, traj_lo, traj_hi), word a%4: the outcome is the first distinct
 * eigenvalue n of T_a (ascending) with x < round(2^32 * sum_{m<=n} p_m).
 *   noise (nullable): int8 [n_traj][Ns][n_gen], the outcome index n.
 *   rho: written, [n_traj][n_clusters][D][D] complex.                      */
cdtwa_status cdtwa_sample_noise(cdtwa_plan plan, uint64_t seed, int64_t traj_offset, int8_t *noise, void *rho,
                                void *stream);

/* a2: cluster mean fields and boundary fields (Sec. II, <s_j>_nu = Tr[s_j rho_nu]
 * and Phi^inter; App. B.1, the eight legs of Phi^inter).
 *   b:   written, [n_traj][Ns] complex, b_j = Tr(a_j rho_C(j)).
 *   phi: written, [n_traj][Ns] complex, phi_j = sum of b_k over lattice
 *        neighbours k of j that lie in another cluster.                    */
cdtwa_status cdtwa_gather_boundary_fields(cdtwa_plan plan, const void *rho, void *b, void *phi, void *stream);

/* a3 alone: K_C = -i [H_C + H_MF, rho_C] for every cluster of every
 * trajectory, with the fields taken from rho itself (Sec. II Eq. (cluster_mf)).
 *   K: written, same layout as rho. */
cdtwa_status cdtwa_commutator(cdtwa_plan plan, const void *rho, void *K, void *workspace, void *stream);

/* a3 + a4: n_steps steps of classical fourth-order Runge-Kutta of the coupled
 * cluster equations (App. B.1), fields recomputed at every stage for all
 * clusters, in place on rho.  workspace: device buffer of at least
 * cdtwa_workspace_bytes bytes, contents undefined on return. */
cdtwa_status cdtwa_step_rk4(cdtwa_plan plan, void *rho, void *workspace, double dt, int32_t n_steps, void *stream);

/* a5: per-trajectory observables (CDTWA_NOBS values, order above) computed in
 * FP64 from rho, and their sums over the plan's trajectories added into
 * sums[t_index][CDTWA_NOBS][3] = (Neumaier sum, Neumaier compensation, sum of
 * squares); trajectories are added in index order (deterministic).
 *   sums:     device double array of at least (t_index+1)*CDTWA_NOBS*3.
 *   per_traj: nullable device double [n_traj][CDTWA_NOBS] (this time only).
 *   workspace: the cdtwa_step_rk4 workspace (any contents).                */
cdtwa_status cdtwa_accumulate_observables(cdtwa_plan plan, const void *rho, int32_t t_index, double *sums,
                                          double *per_traj, void *workspace, void *stream);

/* Which implementation cdtwa_step_rk4 uses for this plan: *path = 0 for the
 * per-stage kernels (state streamed through HBM every stage), 1 for the fused
 * persistent kernel (2x2 clusters with d = 3: every cluster of *resident
 * trajectories kept on chip for a whole call, neighbours exchanging their
 * mean fields through global memory).  The choice is made at plan creation
 * from the device occupancy; setting the environment variable
 * CDTWA_PATH=generic before plan creation forces path 0. resident nullable. */
cdtwa_status cdtwa_plan_path(cdtwa_plan plan, int32_t *path, int32_t *resident);

/* Synchronises `stream` and reads the device status word of the last
 * cdtwa_step_rk4 on `workspace`: 0 = fine; bit 0 = a workgroup of the fused
 * kernel waited for its neighbours longer than its spin limit, in which case
 * the affected clusters were overwritten with NaN.  Always 0 on path 0. */
cdtwa_status cdtwa_device_status(cdtwa_plan plan, const void *workspace, int32_t *status, void *stream);

const char *cdtwa_status_string(cdtwa_status s);
/* Detail of the last error on the calling thread (e.g. the HIP error string). */
const char *cdtwa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CDTWA_H */
