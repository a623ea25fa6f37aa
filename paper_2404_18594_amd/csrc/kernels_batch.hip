// One RK4 stage for every cluster of many independent problems at once
// (mixed cluster shapes 1x1, 2x1, 1x2 and 2x2 with d = 3, mixed lattices,
// couplings and trajectory counts): a work table maps each workgroup to
// (member problem, first cluster); the workgroup runs the per-stage body of
// that member's shape with the clusters-per-workgroup variant the batch chose
// for it.  Same arithmetic per cluster as the single-problem stage kernel.
#include "launch.hpp"
#include "structured.hpp"

namespace cdtwa {

namespace {

template <int CX, int CY>
constexpr int cpb_max() {
  constexpr int D = cluster_dim<3, CX * CY>();
  return D * D >= 4096 ? 1 : 4096 / (D * D);
}
// variant 0: as many clusters as fit (4096 entries of LDS); variant 1: a
// quarter of that (more workgroups, fewer entries per thread)
template <int CX, int CY, int V>
constexpr int cpb_of() {
  return V == 0 ? cpb_max<CX, CY>() : (cpb_max<CX, CY>() / 4 > 0 ? cpb_max<CX, CY>() / 4 : 1);
}

template <typename R, int NT>
__global__ void __launch_bounds__(NT) k_stage_multi(const BatchMember<R>* __restrict__ members,
                                                    const BatchWork* __restrict__ work, int mode, R dt) {
  __shared__ cpx<R> sY[81 * 81];   // one 2x2 cluster, or up to 4096 entries of smaller ones
  __shared__ cpx<R> sPhi[512];
  const BatchWork w = work[blockIdx.x];
  const BatchMember<R>& mb = members[w.member];
  StageArgs<R> a;
  a.g = mb.g;
  a.rho = mb.rho;
  a.k1 = mb.k1;
  a.k2 = mb.k2;
  a.kprev = mode == 2 ? mb.k1 : (mode == 3 ? mb.k2 : (mode == 4 ? mb.k3 : nullptr));
  a.kout = mode <= 1 ? mb.k1 : (mode == 2 ? mb.k2 : (mode == 3 ? mb.k3 : nullptr));
  // field buffers ping-pong as in the single-problem loop: stages 1 and 3
  // read A and write B, stages 2 and 4 read B and write A
  const bool odd = mode == 0 || mode == 1 || mode == 3;
  a.b_in = odd ? mb.bA : mb.bB;
  a.b_out = odd ? mb.bB : mb.bA;
  a.dt = dt;
  a.mode = mode;
  switch (mb.shape * 2 + mb.variant) {
    case 0: stage_body<R, 3, 1, 1, cpb_of<1, 1, 0>(), NT>(a, w.first, sY, sPhi); break;
    case 1: stage_body<R, 3, 1, 1, cpb_of<1, 1, 1>(), NT>(a, w.first, sY, sPhi); break;
    case 2: stage_body<R, 3, 2, 1, cpb_of<2, 1, 0>(), NT>(a, w.first, sY, sPhi); break;
    case 3: stage_body<R, 3, 2, 1, cpb_of<2, 1, 1>(), NT>(a, w.first, sY, sPhi); break;
    case 4: stage_body<R, 3, 1, 2, cpb_of<1, 2, 0>(), NT>(a, w.first, sY, sPhi); break;
    case 5: stage_body<R, 3, 1, 2, cpb_of<1, 2, 1>(), NT>(a, w.first, sY, sPhi); break;
    default: stage_body<R, 3, 2, 2, 1, NT>(a, w.first, sY, sPhi); break;
  }
}

}  // namespace

int batch_cpb(int shape, int variant) {
  switch (shape * 2 + variant) {
    case 0: return cpb_of<1, 1, 0>();
    case 1: return cpb_of<1, 1, 1>();
    case 2: return cpb_of<2, 1, 0>();
    case 3: return cpb_of<2, 1, 1>();
    case 4: return cpb_of<1, 2, 0>();
    case 5: return cpb_of<1, 2, 1>();
    default: return 1;
  }
}

hipError_t batch_stage(int dtype, int nt, const void* members, const BatchWork* work, int64_t n_work, int mode,
                       double dt, hipStream_t s) {
  if (n_work < 1) return hipSuccess;
  const dim3 grid((unsigned)n_work);
  if (dtype == 1) {
    if (nt == 1024)
      hipLaunchKernelGGL((k_stage_multi<double, 1024>), grid, dim3(1024), 0, s, (const BatchMember<double>*)members,
                         work, mode, dt);
    else
      hipLaunchKernelGGL((k_stage_multi<double, 512>), grid, dim3(512), 0, s, (const BatchMember<double>*)members,
                         work, mode, dt);
  } else {
    if (nt == 1024)
      hipLaunchKernelGGL((k_stage_multi<float, 1024>), grid, dim3(1024), 0, s, (const BatchMember<float>*)members,
                         work, mode, (float)dt);
    else
      hipLaunchKernelGGL((k_stage_multi<float, 512>), grid, dim3(512), 0, s, (const BatchMember<float>*)members, work,
                         mode, (float)dt);
  }
  return hipGetLastError();
}

}  // namespace cdtwa
