// Internal interface between the host library and the kernel translation units.
#pragma once

#include "common.hpp"

namespace cdtwa {

bool generic_supported(int d, int cx, int cy);
size_t obs_record_doubles(int nloc);
hipError_t generic_sample(const Geom& g, int dtype, uint64_t seed, int64_t off, int8_t* noise, void* rho, hipStream_t s);
hipError_t generic_site_fields(const Geom& g, int dtype, const void* rho, void* b, hipStream_t s);
hipError_t generic_boundary_fields(const Geom& g, int dtype, const void* b, void* phi, hipStream_t s);
// mode 0: bare commutator; modes 1..4: classical RK4 stages
hipError_t generic_stage(const Geom& g, int dtype, void* rho, const void* kprev, const void* k1, const void* k2,
                         void* kout, const void* b_in, void* b_out, double dt, int mode, hipStream_t s);
hipError_t generic_observables(const Geom& g, int dtype, const void* rho, double* rec, double* per_traj, hipStream_t s);
// fused persistent RK4 for 2x2 clusters, d = 3
size_t fused_exchange_words(int nc, int G);
int fused_slots(int nc, int dtype);
hipError_t fused_rk4(const Geom& g, int dtype, void* rho, uint64_t* xch, int* status, const int* legs, int G,
                     double dt, int n_steps, int spin_limit, hipStream_t s);
hipError_t launch_obs_sum(const double* per_traj, int64_t n_traj, double* sums, hipStream_t s);

}  // namespace cdtwa
