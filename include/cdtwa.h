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
 *   - rho: [n_traj][n_clusters][D][D] complex, row-major, Hermitian.  The
 *     stepping, commutator and field calls rely on it: they form
 *     K = -i (M - M^+) with M = H rho, which equals -i [H, rho] only for
 *     Hermitian rho, and the packed layout stores the upper tiles alone.
 *     The observables read every entry and follow their definitions for any
 *     matrix (Tr rho^2 = sum rho_pq rho_qp, |Tr rho - 1| with the complex
 *     trace, max |rho_pq - conj(rho_qp)|).
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
  CDTWA_EUNSUPPORTED = -2, /* valid problem the library does not implement     */
  CDTWA_EHIP = -3,         /* HIP runtime or launch error                      */
  CDTWA_ENOMEM = -4        /* host allocation failed                           */
} cdtwa_status;

typedef enum { CDTWA_F32 = 0, CDTWA_F64 = 1 } cdtwa_dtype;

/* Storage of the cluster matrices rho (and of K from cdtwa_commutator).
 * FULL: [D][D] row-major per cluster.  PACKED_UPPER (2x2 clusters with
 * d = 4 only, D = 256): the upper triangle of 16 x 16 tiles -- tile (I, J),
 * 0 <= I <= J < 16, holds rows 16 I .. 16 I + 15 and columns 16 J .. 16 J + 15
 * as 256 contiguous entries (row-major inside the tile); tiles follow each
 * other in row-major order over I <= J, tile (I, J) at position
 * 16 I - I (I - 1) / 2 + (J - I); a diagonal tile holds all 256 of its
 * entries.  The lower tiles are the conjugate transposes (rho is Hermitian).
 * CDTWA_PACKED_ELEMS entries per cluster, 0.53 of the full layout.          */
typedef enum { CDTWA_LAYOUT_FULL = 0, CDTWA_LAYOUT_PACKED_UPPER = 1 } cdtwa_layout;
#define CDTWA_PACKED_TILE 16
#define CDTWA_PACKED_ELEMS 34816

/* Problem definition.
 * model 0 (Bose-Hubbard, Sec. III Eq. (H_bose)):
 *   H = -J sum_<ij> (a_i^+ a_j + h.c.) + U/2 sum_i n_i (n_i - 1)
 *   with occupations truncated to 0..d-1 (d = n_max + 1, Sec. III).
 * model 1 (transverse-field Ising, App. A Eq. (Hising); d must be 2):
 *   H = J sum_<ij> s^z_i s^z_j + h sum_i s^x_i  (Pauli matrices; basis
 *   |0> = |up>, s^z = +1).  The mean field of a site is b_j = <s^z_j>
 *   (stored as a complex number with the imaginary part of Tr(s^z rho_C));
 *   a bond to another cluster adds J s^z_i Re(b_k) to the cluster
 *   Hamiltonian.  U is ignored.
 * Onsite initial states:
 *   model 0, init_state 0: unit-filling Mott state |1> on every site (Sec. III)
 *   model 1, init_state 0: |up> on every site
 *   model 1, init_state 1: Neel state, |up> where x + y is even, |down>
 *                          elsewhere (App. A: s^x, s^y = +-1 with probability
 *                          1/2 each, s^z fixed).
 * Open system (model 0; the extension to the Lindblad master equation that
 * Sec. IV and App. B.1 name): local channels L_j = sqrt(gamma_deph) n_j and
 * L_j = sqrt(gamma_loss) a_j on every site; every cluster matrix then obeys
 *   d rho_C/dt = -i [H_C + H_MF, rho_C]
 *                + sum_{j in C, L} (L rho_C L^+ - (L^+ L rho_C + rho_C L^+ L)/2).
 * Rates must be finite and >= 0; a nonzero rate needs clusters with D <= 81
 * (CDTWA_EUNSUPPORTED otherwise) and runs on the fused 27-row path for 2x2
 * clusters with d = 3 when they fit on the chip, else on the per-stage path.
 * The 80-byte layout below is part of the ABI.                              */
typedef struct {
  int32_t Lx, Ly;        /* lattice sides                                              */
  int32_t cx, cy;        /* cluster shape, each 1 or 2; Lx % cx == Ly % cy == 0         */
  int32_t d;             /* local dimension: 2, 3 or 4                                 */
  int32_t periodic;      /* 1 periodic (needs >= 2 clusters and >= 3 sites per side)   */
  double J, U;           /* hopping (model 1: zz coupling) and interaction             */
  int32_t init_state;    /* onsite initial state, see above                            */
  int32_t dtype;         /* cdtwa_dtype of the trajectory state                        */
  int32_t model;         /* 0 Bose-Hubbard, 1 transverse-field Ising                   */
  int32_t layout;        /* cdtwa_layout of rho; PACKED_UPPER needs model 0, 2x2, d = 4  */
  double h;              /* model 1: transverse field; must be 0 for model 0           */
  double gamma_deph;     /* model 0: on-site dephasing rate (0: closed system)         */
  double gamma_loss;     /* model 0: on-site particle-loss rate (0: closed system)     */
} cdtwa_problem;

typedef struct cdtwa_plan_s *cdtwa_plan;

/* Number of per-trajectory observables written by cdtwa_accumulate_observables. */
#define CDTWA_NOBS 15
/* Observable order for model 0 (every value a double):
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

/* Observable order for model 1 (same slots):
 *   0      (1/Ns) sum_j (-1)^(x_j + y_j) <s^z_j>   (staggered magnetisation;
 *          App. A's M_z on the four-site chain is Ns times this)
 *   1..3   (1/Ns) sum_j <s^z_j>, <s^x_j>, <s^y_j>
 *   4, 10  zero
 *   5..9   the ordered-pair sums of slots 5..9 above for <s^z_i s^z_j>
 *          (same cluster: Tr(s^z_i s^z_j rho_C); else the product)
 *   11     mean-field energy per site; 12..14 as for model 0.              */

/* Create a plan for n_traj trajectories (n_traj >= 1).  Validates the
 * problem (CDTWA_EINVAL for inconsistent shapes, CDTWA_EUNSUPPORTED for a
 * valid shape the library does not implement), builds the geometry and the
 * sampling tables, and uploads them to the current HIP device. */
cdtwa_status cdtwa_plan_create(const cdtwa_problem *p, int64_t n_traj, cdtwa_plan *out);
cdtwa_status cdtwa_plan_destroy(cdtwa_plan plan);

/* Sizes derived from the problem: number of sites, clusters, sites per
 * cluster, cluster dimension D, generators per site (d*d-1), bytes of one
 * real of the state precision. Any output pointer may be NULL.  A cluster
 * matrix holds D*D complex entries in the full layout and
 * CDTWA_PACKED_ELEMS in the packed one. */
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
 * trajectory, with the fields taken from rho itself (Sec. II Eq. (cluster_mf));
 * plus the dissipator when the problem has Lindblad rates.
 *   K: written, same layout as rho. */
cdtwa_status cdtwa_commutator(cdtwa_plan plan, const void *rho, void *K, void *workspace, void *stream);

/* a3 + a4: n_steps steps of classical fourth-order Runge-Kutta of the coupled
 * cluster equations (App. B.1), fields recomputed at every stage for all
 * clusters, in place on rho.  workspace: device buffer of at least
 * cdtwa_workspace_bytes bytes, contents undefined on return. */
cdtwa_status cdtwa_step_rk4(cdtwa_plan plan, void *rho, void *workspace, double dt, int32_t n_steps, void *stream);

/* cdtwa_step_rk4 without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The RK4 workspace comes from a static
 * device buffer of CDTWA_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device it runs on until the process ends; the call itself allocates
 * nothing.  Same arithmetic and results as cdtwa_step_rk4 (the same kernels).
 * Returns CDTWA_EINVAL, before anything is enqueued, when the plan's RK4
 * workspace exceeds the buffer: the fused paths (2x2 clusters resident on
 * the chip) need a few hundred KB at most; the per-stage paths need three
 * state copies and fit only small problems.  Every call on one device shares
 * that device's buffer: calls that overlap on one device (different streams
 * or host threads) race and must be serialised by the caller.  The device
 * status word (cdtwa_device_status) of these calls lives in the shared
 * buffer and is not readable through the ABI.                               */
#define CDTWA_NOALLOC_SCRATCH_BYTES (4u << 20)
cdtwa_status cdtwa_step_rk4_noalloc(cdtwa_plan plan, void *rho, double dt, int32_t n_steps, void *stream);

/* a3 + a4 with time-dependent couplings (the ramped lattice of Sec. III,
 * Fig. 2 protocol, with the schedule supplied by the caller): n_steps
 * classical RK4 steps as cdtwa_step_rk4, the couplings of every stage taken
 * from host arrays sampled at every half step,
 *   c1_half[k] = J(t0 + k dt/2),  c2_half[k] = U(t0 + k dt/2)  (model 1: h),
 *   k = 0 .. 2 n_steps;
 * stage 1 of step s uses entry 2s, stages 2 and 3 entry 2s+1, stage 4 entry
 * 2s+2 (classical RK4 for a time-dependent right-hand side).  The arrays are
 * read before the call returns (the caller may reuse them at once); every
 * value must be finite (CDTWA_EINVAL otherwise).  The problem's own J, U (h)
 * are not used by this call; the energy slot of the observables keeps using
 * them.  Same workspace as cdtwa_step_rk4.  On the fused paths the schedule
 * travels in the kernel arguments, so a call runs as launches of at most 16
 * steps. */
cdtwa_status cdtwa_step_rk4_schedule(cdtwa_plan plan, void *rho, void *workspace, double dt, int32_t n_steps,
                                     const double *c1_half, const double *c2_half, void *stream);

/* a4 with a compensated FP32 state (project choice of an FP32 trajectory
 * state; App. B.1 RK4): n_steps steps of cdtwa_step_rk4, the same stages and
 * roundings, except that the state is rho + rho_lo.  rho_lo holds the part of
 * every entry that FP32 rho cannot represent.  The last stage forms
 * rho + (rho_lo + increment) as an exact two-term sum (TwoSum); the rounded
 * sum is written to rho and its remainder to rho_lo.  So the state is not
 * rounded to FP32 at every step, and only the stage arithmetic is FP32.
 * Fields, observables and the commutator read rho alone.
 *   rho:    as for cdtwa_step_rk4 (the plan's layout), updated in place.
 *   rho_lo: device FP32 complex [n_traj][n_clusters][CDTWA_PACKED_ELEMS],
 *           the packed layout in either plan layout, updated in place.  A
 *           state fresh from cdtwa_sample_noise starts from rho_lo = 0 (the
 *           Mott-state phase points are exact in FP32); a caller holding an
 *           FP64 state x passes rho = fp32(x), rho_lo = fp32(x - rho).
 *   workspace: as for cdtwa_step_rk4.
 * Needs an FP32 plan with 2x2 clusters and d = 4 (D = 256);
 * CDTWA_EUNSUPPORTED otherwise.  Costs one more read and write of an FP32
 * packed state per step. */
cdtwa_status cdtwa_step_rk4_compensated(cdtwa_plan plan, void *rho, void *rho_lo, void *workspace, double dt,
                                        int32_t n_steps, void *stream);

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
 * per-stage kernels (state streamed through HBM every stage); 1 and 2 for the
 * fused persistent kernels of 2x2 clusters with d = 3, which keep every
 * cluster of *resident trajectories on chip for a whole call, neighbours
 * exchanging their mean fields through global memory: 1 = one column of 27
 * rows per thread (4 waves per cluster), 2 = 9 rows per thread (12 waves per
 * cluster).  The choice is made at plan creation from the device occupancy
 * (default: 1 whenever it fits; for FP32 closed systems whose clusters do not
 * fit at two workgroups per CU, path 1 runs a build sized for three); the
 * environment variable
 * CDTWA_PATH = generic | fused27 | plaq set before plan creation forces
 * path 0, 1 or 2.  CDTWA_PATH = dense selects path 3: the per-stage path
 * with M = H Y as a dense complex matrix product on the matrix cores (FP32
 * state, 2x2 clusters, d = 3 only; plan creation fails with
 * CDTWA_EUNSUPPORTED otherwise), kept for measurement against the
 * structured operator.  Paths 4 and 5 belong to the Ising model (model 1):
 * 5 = the fused persistent spin kernel for 2x2 clusters (one wave per
 * cluster, the cluster state in registers, mean fields exchanged as on paths
 * 1 and 2), chosen whenever the clusters of one trajectory fit on the chip;
 * 4 = the per-stage spin kernels otherwise.  CDTWA_PATH, if set, must then be
 * "spinfused" or "spin" ("spin" forces path 4).  An
 * open system (nonzero Lindblad rate) runs on path 1 or 0 only; CDTWA_PATH,
 * if set, must then be "fused27" or "generic".  Path 6 (the default for the
 * closed Bose-Hubbard model with d = 3 and 1x1, 2x1 or 1x2 clusters whenever
 * one trajectory fits a workgroup; CDTWA_PATH = traj forces it and fails with
 * CDTWA_EUNSUPPORTED where it cannot run) is trajectory-resident: a
 * persistent grid of one workgroup per CU pulls blocks of *resident
 * trajectories from a work queue and integrates every step of the call with
 * the whole trajectory on chip (matrices in registers, mean fields in LDS),
 * reading rho once and writing it once (Sec. II Eq. (cluster_mf); App. B.1).
 * cdtwa_step_rk4_schedule on a path-6 plan runs the per-stage kernels.
 * resident nullable: trajectories held at once (paths 1, 2, 5) or per
 * workgroup (path 6). */
cdtwa_status cdtwa_plan_path(cdtwa_plan plan, int32_t *path, int32_t *resident);

/* Synchronises `stream` and reads the device status word of the last
 * cdtwa_step_rk4 on `workspace`: 0 = fine; bit 0 = a workgroup of the fused
 * kernel waited for its neighbours longer than its spin limit (4194304 polls,
 * or the value of the environment variable CDTWA_SPIN_LIMIT at plan creation;
 * a tiny value makes the waits time out, which tests this path), in which case
 * the affected clusters were overwritten with NaN.  Always 0 on paths other
 * than 1, 2 and 5.  The status word sits in the first 256 bytes of the
 * workspace, which no other call writes: it stays readable after
 * cdtwa_accumulate_observables or cdtwa_cv_targets on the same workspace. */
cdtwa_status cdtwa_device_status(cdtwa_plan plan, const void *workspace, int32_t *status, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many independent problems (plans) advanced together, in groups:
 * - members on the trajectory-resident path (cdtwa_plan_path 6: d = 3 with
 *   1x1, 2x1 or 1x2 clusters, whatever their lattices, couplings and
 *   trajectory counts) in one persistent launch per call: a work queue of
 *   (member, block of trajectories) items, the costliest first, each
 *   integrating all the call's steps on chip;
 * - members on the fused 27-row path (2x2 clusters, d = 3, closed, the
 *   build for one workgroup per CU in FP64 and two in FP32) packed side by
 *   side into as few cooperative launches per call as fit (first fit by
 *   decreasing footprint): each member keeps the gangs of nc workgroups its
 *   own launch would use (min(trajectories, co-resident workgroups / nc)),
 *   and each gang integrates the member's trajectories in turn with every
 *   step of the call on chip (Sec. II Eq. (cluster_mf); App. B.1).  A member
 *   alone in its launch (one that fills the device) runs its own path, so
 *   batching gains where several members would each leave most of the
 *   device idle;
 * - the other members with d = 3 whose clusters are 1x1, 2x1, 1x2 (and 2x2
 *   members on the per-stage path, or every 2x2 member with
 *   CDTWA_BATCH_MIX_ALL) by one launch per RK4 stage that covers every
 *   cluster of every such member; the four launches of a step are captured
 *   in a HIP graph at the first call (and again when dt changes) and
 *   replayed once per step.  At the first call the workgroup size and, per
 *   cluster shape, the number of clusters per workgroup of that launch are
 *   chosen by timing candidates on commutator launches (they write only
 *   workspace);
 * - the remaining members (2x2 on the fused build for three workgroups per
 *   CU, open systems, d = 2 or 4) run their own cdtwa_step_rk4 on the same
 *   stream.
 * Results equal those of cdtwa_step_rk4 on each plan (bit for bit): with its
 * own path for resident, fused and remaining members, with the per-stage
 * path for members of the per-stage launch.  A fused member whose neighbour
 * wait times out has its clusters overwritten with NaN.
 * ------------------------------------------------------------------------ */
typedef struct cdtwa_batch_s *cdtwa_batch;
#define CDTWA_BATCH_MIX_ALL 1

/* plans: n plans of the same state precision; they must outlive the batch.
 * flags: 0 or CDTWA_BATCH_MIX_ALL.  Allocates the batch's device tables. */
cdtwa_status cdtwa_batch_create(const cdtwa_plan *plans, int32_t n, int32_t flags, cdtwa_batch *out);
cdtwa_status cdtwa_batch_destroy(cdtwa_batch batch);

/* Workspace the batch needs for member `member` (at least that member's own
 * cdtwa_workspace_bytes; the per-stage layout for members of the mixed launch). */
cdtwa_status cdtwa_batch_workspace_bytes(cdtwa_batch batch, int32_t member, size_t *bytes);

/* n_steps classical RK4 steps of every member.  rho[i], workspace[i]: member
 * i's state and workspace (device pointers).  Changing the pointers between
 * calls is allowed (the batch then synchronises the stream once to rewrite
 * its tables). */
cdtwa_status cdtwa_batch_step_rk4(cdtwa_batch batch, void *const *rho, void *const *workspace, double dt,
                                  int32_t n_steps, void *stream);

/* Members in the per-stage mixed launch, its chosen workgroup size (0
 * before the first step), chosen variant per shape (variants[3]: 1x1, 2x1,
 * 1x2; 0 = most clusters per workgroup, 1 = a quarter of that), workgroups
 * per stage launch; members in the trajectory-resident launch and its work
 * items; members in the fused launches and the workgroups of the largest.
 * Any output may be NULL. */
cdtwa_status cdtwa_batch_info(cdtwa_batch batch, int32_t *n_mixed, int32_t *threads, int32_t *variants,
                              int64_t *workgroups, int32_t *n_resident, int64_t *resident_items, int32_t *n_fused,
                              int32_t *fused_workgroups);

/* ------------------------------------------------------------------------
 * a6: learned control variate.  This is an addition to the paper's method,
 * not part of it: the paper estimates every observable by the plain sample
 * mean over trajectories (Sec. II).  For 2x2 clusters with d = 3, a small
 * network g maps the noise of the 4x4 site patch around a cluster mu (the
 * cluster's 2x2 block and a ring of one site) to the cluster's share of the
 * nearest-neighbour correlation at up to CDTWA_MLP_OUT recorded times,
 *   t_mu = sum over sites i of mu of Re<a_i^+ a_(i+x)> + Re<a_i^+ a_(i+y)>,
 * so that (1/Ns) sum_mu t_mu = (C^sp_(1,0) + C^sp_(0,1)) / 2.  With
 * G = (1/Ns) sum_mu g(patch_mu) per trajectory, the estimate
 *   mean over trajectories of (O - G)  +  (n_clusters/Ns) E[g]
 * is unbiased for any fixed g, because every patch of a trajectory has the
 * distribution of an i.i.d. patch (independent, identically distributed site
 * noise); E[g] comes from fresh i.i.d. patches (cdtwa_cv_expectation).
 *
 * Network: x[128] -> relu(x W1 + b1)[256] -> relu(. W2 + b2)[256] ->
 * (. W3 + b3)[64].  Products take BF16 operands (weights: a BF16 copy of the
 * FP32 master weights; activations rounded to BF16 before each product) and
 * accumulate in FP32 on the matrix cores; biases, activations and gradients
 * are FP32.  Loss: mean over all n*64 outputs of (y - target)^2.
 *   params: FP32 [CDTWA_MLP_PARAMS] = W1 [128][256], b1 [256], W2 [256][256],
 *           b2 [256], W3 [256][64], b3 [64]  (row-major, W[in][out]).
 *   wbf16:  BF16 bit patterns [CDTWA_MLP_WBF16] = W1, W2, W3, the rounded
 *           (nearest, ties to even) copies of the FP32 weights.
 * Feature 8*s + a of a patch is the value r^a (a = 0..7) of patch site
 * s = 4*(y - y0 + 1) + (x - x0 + 1), x in [x0-1, x0+2], y in [y0-1, y0+2],
 * (x0, y0) the cluster's lower-left site, wrapped on a periodic lattice and
 * 0 for a site outside an open one.
 * ------------------------------------------------------------------------ */
#define CDTWA_MLP_IN 128
#define CDTWA_MLP_HIDDEN 256
#define CDTWA_MLP_OUT 64
#define CDTWA_MLP_PARAMS 115264
#define CDTWA_MLP_WBF16 114688

/* Device workspace bytes of cdtwa_mlp_forward / cdtwa_mlp_backward for n rows. */
cdtwa_status cdtwa_mlp_workspace_bytes(int64_t n, size_t *bytes);

/* Weights uniform in [-b, b) with b = sqrt(6/fan_in) (hidden layers) and
 * sqrt(3/fan_in) (output layer), from Philox-4x32-10 keyed by seed; biases 0;
 * writes params and wbf16. */
cdtwa_status cdtwa_mlp_init(float *params, uint16_t *wbf16, uint64_t seed, void *stream);

/* y [n][64] = g(x [n][128]) (FP32 rows).  The activations are kept in the
 * workspace (cdtwa_mlp_workspace_bytes(n)) for a following backward pass. */
cdtwa_status cdtwa_mlp_forward(const float *params, const uint16_t *wbf16, const float *x, float *y, int64_t n,
                               void *workspace, void *stream);

/* Gradient of the mean squared error of y (the output of the last
 * cdtwa_mlp_forward on this workspace with the same n and weights) against
 * target [n][64].  grad: FP32 [CDTWA_MLP_PARAMS], overwritten, same layout as
 * params.  loss: nullable device float, overwritten.  n: multiple of 16. */
cdtwa_status cdtwa_mlp_backward(const uint16_t *wbf16, const float *y, const float *target, float *grad, float *loss,
                                int64_t n, void *workspace, void *stream);

/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected with step >= 1) on params with moments m, v (FP32
 * [CDTWA_MLP_PARAMS], zero before step 1), then the BF16 copy. */
cdtwa_status cdtwa_mlp_adam(float *params, uint16_t *wbf16, const float *grad, float *m, float *v, float lr,
                            int32_t step, void *stream);

/* features: written, FP32 [n_traj][n_clusters][128], from the noise codes
 * that cdtwa_sample_noise wrote for the plan's trajectories. */
cdtwa_status cdtwa_cv_features(cdtwa_plan plan, const int8_t *noise, float *features, void *stream);

/* targets[(t*n_clusters + mu)*64 + column] = t_mu of trajectory t, from rho
 * (FP32, computed in FP64).  workspace: the cdtwa_step_rk4 workspace. */
cdtwa_status cdtwa_cv_targets(cdtwa_plan plan, const void *rho, int32_t column, float *targets, void *workspace,
                              void *stream);

/* gtraj: written, FP64 [n_traj][64], gtraj[t][o] = (1/Ns) sum_mu y[t][mu][o]
 * (clusters added in index order) for y [n_traj][n_clusters][64]. */
cdtwa_status cdtwa_cv_traj_sums(cdtwa_plan plan, const float *y, double *gtraj, void *stream);

/* Features of n i.i.d. patches with indices first .. first+n-1: patch p,
 * site s, generator a drawn like a trajectory site (same outcome rule) from
 * Philox-4x32-10 with counter (a/4, s, p_lo, p_hi) and key (seed_lo,
 * seed_hi ^ 0x5bd1e995).  features: written, FP32 [n][128]. */
cdtwa_status cdtwa_cv_sample_features(cdtwa_plan plan, uint64_t seed, int64_t first, int64_t n, float *features,
                                      void *stream);

/* Device workspace bytes of cdtwa_cv_expectation. */
cdtwa_status cdtwa_cv_workspace_bytes(size_t *bytes);

/* Adds the moments of g over the i.i.d. patches 0 .. n_samples-1 of `seed`
 * into moments [64][3] (Neumaier sum, compensation, sum of squares; FP64,
 * patches added in index order). */
cdtwa_status cdtwa_cv_expectation(cdtwa_plan plan, const float *params, const uint16_t *wbf16, uint64_t seed,
                                  int64_t n_samples, double *moments, void *workspace, void *stream);

const char *cdtwa_status_string(cdtwa_status s);
/* Detail of the last error on the calling thread (e.g. the HIP error string). */
const char *cdtwa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CDTWA_H */
