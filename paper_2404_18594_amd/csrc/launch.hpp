// Internal interface between the host library and the kernel translation units.
#pragma once

#include "common.hpp"

namespace cdtwa {

// Doubles in the observable record of one Bose-Hubbard cluster of NLOC
// sites: [0,2nloc) b, [2nloc,3nloc) n, then G[l][m] (nloc^2), NN[l][m]
// (nloc^2), Re Tr, Tr rho^2, Hermiticity deviation, E_intra, Im Tr.
template <int NLOC>
__host__ __device__ constexpr int cluster_rec() {
  return 3 * NLOC + 2 * NLOC * NLOC + 5;
}

bool generic_supported(int d, int cx, int cy);
size_t obs_record_doubles(int nloc);
hipError_t generic_sample(const Geom& g, int dtype, uint64_t seed, int64_t off, int8_t* noise, void* rho, hipStream_t s);
hipError_t generic_site_fields(const Geom& g, int dtype, const void* rho, void* b, hipStream_t s);
hipError_t generic_boundary_fields(const Geom& g, int dtype, const void* b, void* phi, hipStream_t s);
// mode 0: bare commutator; modes 1..4: classical RK4 stages
hipError_t generic_stage(const Geom& g, int dtype, void* rho, const void* kprev, const void* k1, const void* k2,
                         void* kout, const void* b_in, void* b_out, double dt, int mode, hipStream_t s);
// 2x2 clusters with d = 4 (D = 256): one launch per RK4 stage; layout 0 full,
// 1 packed upper tiles (g.layout)
bool big_supported(int d, int cx, int cy);
int64_t big_packed_elems();
size_t big_workspace_bytes(const Geom& g, int dtype);
// n_steps classical RK4 steps; c1, c2 (nullable): J, U at every half step;
// lo (nullable, FP32 state only): packed low parts of rho, carried by the
// compensated final stage
hipError_t big_rk4(const Geom& g, int dtype, int layout, void* rho, void* lo, void* ws, double dt, int n_steps,
                   const double* c1, const double* c2, hipStream_t s);
hipError_t big_commutator(const Geom& g, int dtype, int layout, const void* rho, void* K, void* ws, hipStream_t s);
hipError_t big_site_fields(const Geom& g, int dtype, int layout, const void* rho, void* b, hipStream_t s);
// packed cluster matrices -> full D x D matrices (the lower tiles as conjugate transposes)
hipError_t big_unpack(const Geom& g, int dtype, const void* packed, void* full, hipStream_t s);
hipError_t generic_observables(const Geom& g, int dtype, const void* rho, double* rec, double* per_traj, hipStream_t s);
// fused persistent RK4 for 2x2 clusters, d = 3.  sJ, sU (nullable): the
// couplings at every half step of this launch (2 n_steps + 1 values, n_steps
// <= kSchedSteps), passed by value in the kernel arguments; zero_status:
// clear the status word with the exchange words (the first launch of a call)
constexpr int kSchedSteps = 16;
constexpr int kSchedVals = 2 * kSchedSteps + 1;
size_t fused_exchange_words(int nc, int G);
int fused_slots(int nc, int dtype, bool diss, bool wide);
hipError_t fused_rk4(const Geom& g, int dtype, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                     double dt, int n_steps, int spin_limit, const double* sJ, const double* sU, bool zero_status,
                     bool wide, hipStream_t s);
hipError_t fused_zero_words(uint64_t* xch, size_t n_words, int* status, hipStream_t s);
// fused persistent RK4 for the transverse-field Ising model with 2x2
// clusters (one wave per cluster, state in registers)
bool spin_fused_supported(int model, int d, int cx, int cy);
int spin_fused_slots(int nc, int dtype);
hipError_t spin_fused_rk4(const Geom& g, int dtype, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                          double dt, int n_steps, int spin_limit, const double* sJ, const double* sH,
                          bool zero_status, hipStream_t s);
// fused persistent RK4 for 2x2 clusters, d = 3, 9 rows per thread (12 waves)
int plaq_slots(int nc, int dtype);
hipError_t plaq_rk4(const Geom& g, int dtype, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                    double dt, int n_steps, int spin_limit, const double* sJ, const double* sU, bool zero_status,
                    hipStream_t s);
// dense-GEMM (matrix-core) variant of one stage: FP32, 2x2 clusters, d = 3
bool dense_supported(int d, int cx, int cy, int dtype);
hipError_t dense_stage(const Geom& g, int dtype, void* rho, const void* kprev, const void* k1, const void* k2,
                       void* kout, const void* b_in, void* b_out, double dt, int mode, hipStream_t s);
// Batches of problems with mixed cluster shapes (d = 3): one stage launch for
// all members.  shape: 0 = 1x1, 1 = 2x1, 2 = 1x2, 3 = 2x2; variant: 0 or 1
// (clusters per workgroup, batch_cpb).  Field buffers A, B as in the
// single-problem stage loop.
template <typename R>
struct BatchMember {
  Geom g;
  cpx<R>* rho;
  cpx<R>* k1;
  cpx<R>* k2;
  cpx<R>* k3;
  cpx<R>* bA;
  cpx<R>* bB;
  int shape, variant;
};
struct BatchWork {
  int32_t member, pad;
  int64_t first;   // first flat (trajectory, cluster) index of the workgroup
};
int batch_cpb(int shape, int variant);
hipError_t batch_stage(int dtype, int nt, const void* members, const BatchWork* work, int64_t n_work, int mode,
                       double dt, hipStream_t s);
// batch launch of the fused 27-row kernel: the gangs of several member
// problems (2x2, d = 3, closed, the one- and two-per-CU builds) in one
// cooperative launch; members is a device array of fused_member_bytes(dtype)
// records written by fused_member_fill (slot0: first workgroup of the
// member's G gangs of nc workgroups), xch the members' exchange words
// (n_words in all, cleared by the call), grid <= fused_multi_slots(dtype)
size_t fused_member_bytes(int dtype);
void fused_member_fill(const Geom& g, int dtype, void* rho, uint64_t* xch, const int* legs, int G, int slot0,
                       void* out);
int fused_multi_slots(int dtype);
hipError_t fused_multi_rk4(int dtype, const void* members, int n_members, int grid, uint64_t* xch, size_t n_words,
                           int* status, double dt, int n_steps, int spin_limit, hipStream_t s);
// trajectory-resident RK4 (d = 3; 1x1, 2x1, 1x2 clusters; closed
// Bose-Hubbard): one workgroup keeps whole trajectories on chip for a call.
// traj_per_item: trajectories one workgroup holds (0: not even one fits).
// counter: one device int (cleared by the call).  Batches: members is a device
// array of traj_member_bytes(dtype)-sized records written by
// traj_member_fill, work a device array of (member, first trajectory).
bool traj_supported(int model, int d, int cx, int cy, bool diss);
int traj_per_item(const Geom& g, int dtype);
size_t traj_member_bytes(int dtype);
void traj_member_fill(const Geom& g, int dtype, void* rho, int ntr, void* out);
hipError_t traj_rk4(const Geom& g, int dtype, void* rho, int* counter, double dt, int n_steps, hipStream_t s);
hipError_t traj_batch_rk4(int dtype, const void* members, const int2* work, int64_t n_work, int* counter, double dt,
                          int n_steps, hipStream_t s);
// sums over trajectories of the per-trajectory observables; scratch: at
// least obs_sum_scratch_doubles(n_traj) doubles
size_t obs_sum_scratch_doubles(int64_t n_traj);
hipError_t launch_obs_sum(const double* per_traj, int64_t n_traj, double* sums, double* scratch, hipStream_t s);
// transverse-field Ising (model 1, d = 2), any cluster shape: mean fields
// b_j = Tr(s^z_j rho_C), one RK4 stage (modes as generic_stage), observables
hipError_t spin_site_fields(const Geom& g, int dtype, const void* rho, void* b, hipStream_t s);
hipError_t spin_stage(const Geom& g, int dtype, void* rho, const void* kprev, const void* k1, const void* k2,
                      void* kout, const void* b_in, void* b_out, double dt, int mode, hipStream_t s);
hipError_t spin_observables(const Geom& g, int dtype, const void* rho, double* rec, double* per_traj, hipStream_t s);

}  // namespace cdtwa

namespace cdtwa {
// MLP and control-variate kernels
hipError_t gemm_bf16(const uint16_t* a, int64_t sam, int64_t sak, const uint16_t* b, int64_t sbk, int64_t sbn,
                     float* c, int64_t ldc, int M, int N, int K, int ksplit, hipStream_t s);
hipError_t gemm_epilogue(const float* part, int ksplit, int64_t MN, int N, const float* bias, float* out,
                         uint16_t* act, int mode, hipStream_t s);
hipError_t to_bf16_array(const float* x, uint16_t* y, int64_t n, hipStream_t s);
hipError_t relu_back(const float* dact, const float* z, float* dz, uint16_t* dzb, int64_t n, hipStream_t s);
// column sums of x [rows][N] times scale into out[N]; scratch holds
// COLSUM_MAX_CHUNKS x N floats of chunk sums
constexpr int64_t COLSUM_MAX_CHUNKS = 256, COLSUM_MIN_CHUNK = 64;
hipError_t colsum(const float* x, int64_t rows, int N, float scale, float* out, float* scratch, hipStream_t s);
hipError_t mse_grad(const float* y, const float* t, float* dy, uint16_t* dyb, float* sq, int64_t n, float scale,
                    hipStream_t s);
hipError_t adam_update(float* w, uint16_t* wb, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t cv_features(const Geom& g, const int8_t* noise, float* feat, hipStream_t s);
hipError_t cv_sample_features(const Geom& g, uint64_t seed, int64_t first, int64_t n, float* feat, hipStream_t s);
hipError_t cv_targets(const Geom& g, const double* rec, float* out, int ldo, int col, hipStream_t s);
// FP64 column moments of y [rows][N] (N <= 64) added into out [N][3]
// (Neumaier sum, compensation, sum of squares); part: nblk_max*N*2 doubles
hipError_t colmoments(const float* y, int64_t rows, int N, double* part, int nblk_max, double* out, hipStream_t s);
hipError_t traj_sums(const float* y, int64_t n_traj, int rows_per_traj, int N, double scale, double* out,
                     hipStream_t s);
// bound > 0: uniform weights; bound == 0: zeros (wb unused)
hipError_t mlp_init_layer(float* w, uint16_t* wb, int64_t n, float bound, int layer, uint64_t seed, hipStream_t s);
}  // namespace cdtwa
