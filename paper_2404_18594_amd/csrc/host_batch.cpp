// Host side of problem batches (C ABI in include/cdtwa.h).  Members on the
// trajectory-resident path (d = 3 small clusters whose trajectories fit a
// workgroup) advance in ONE persistent launch per call: a work queue of
// (member, block of trajectories) items, the costliest first, pulled by a
// grid of one workgroup per CU, every item integrating all the call's steps
// on chip.  Members on the fused 27-row path (2x2, d = 3) advance packed
// side by side, with the gangs of their own launches, into as few
// cooperative launches per call as fit (waves), the co-resident workgroups
// split into the gangs of each member's clusters.  Members with small clusters that do not fit
// a workgroup (and 2x2 ones on the per-stage path, or every 2x2 member on
// request) advance together through one launch per RK4 stage for all of
// them, the four launches of a step captured once in a HIP graph and
// replayed; the clusters-per-workgroup variant of every shape and the
// workgroup size are chosen by timing.  Other members run their own
// cdtwa_step_rk4.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/cdtwa.h"
#include "launch.hpp"
#include "plan.hpp"

using namespace cdtwa;

struct cdtwa_batch_s {
  std::vector<cdtwa_plan> plans;
  std::vector<int> resident;    // members in the trajectory-resident launch
  void* d_tmembers = nullptr;   // their records (traj_member_fill)
  int2* d_twork = nullptr;      // (member, first trajectory), costliest first
  int* d_counter = nullptr;     // the work queue's counter
  int64_t n_twork = 0;
  std::vector<const void*> last_trho;
  std::vector<int> fused;       // members in the batch launch of the fused 27-row kernel
  std::vector<int> fusedG;      // gangs of each
  struct Wave {
    int first, count, grid;     // members fused[first .. first + count - 1], workgroups
  };
  std::vector<Wave> fwave;      // one cooperative launch each
  void* d_fmembers = nullptr;   // their records (fused_member_fill)
  uint64_t* d_fxch = nullptr;   // their exchange words
  int* d_fstatus = nullptr;     // bit 0: a neighbour wait timed out (clusters set to NaN)
  int fgrid = 0, fspin = 0;
  std::vector<const void*> last_frho;
  std::vector<int> mixed;       // members in the mixed launch
  std::vector<int> own;         // members stepped through their own plan
  std::vector<int> shape;       // per member (mixed only): 0 1x1, 1 2x1, 2 1x2, 3 2x2
  int dtype = 1;
  int nt = 512;
  int variant[4] = {0, 0, 0, 0};
  bool tuned = false;
  void* d_members = nullptr;    // BatchMember<R>[n_mixed]
  BatchWork* d_work = nullptr;  // capacity work_cap
  int64_t work_cap = 0, n_work = 0;
  std::vector<const void*> last_rho, last_ws;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  double graph_dt = 0;
  int dev = 0;
};

namespace {

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

cdtwa_status hip_err(hipError_t e, const char* where) {
  return set_error(CDTWA_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

int shape_code(const Geom& g) {
  if (g.cx == 1 && g.cy == 1) return 0;
  if (g.cx == 2 && g.cy == 1) return 1;
  if (g.cx == 1 && g.cy == 2) return 2;
  return 3;
}

std::vector<BatchWork> work_table(const cdtwa_batch_s& b, const int variant[4]) {
  std::vector<BatchWork> w;
  for (size_t i = 0; i < b.mixed.size(); ++i) {
    const Geom* g = plan_geom(b.plans[b.mixed[i]]);
    const int cpb = batch_cpb(b.shape[i], b.shape[i] == 3 ? 0 : variant[b.shape[i]]);
    const int64_t total = g->n_traj * g->nc;
    for (int64_t f = 0; f < total; f += cpb) w.push_back(BatchWork{(int32_t)i, 0, f});
  }
  return w;
}

template <typename R>
std::vector<BatchMember<R>> member_table(const cdtwa_batch_s& b, void* const* rho, void* const* ws,
                                         const int variant[4]) {
  std::vector<BatchMember<R>> m;
  for (size_t i = 0; i < b.mixed.size(); ++i) {
    const int k = b.mixed[i];
    PlanLayout L;
    plan_layout(b.plans[k], &L);
    const size_t S = a256(L.state_bytes), F = a256(L.field_bytes);
    char* w = (char*)ws[k];
    BatchMember<R> e;
    e.g = *plan_geom(b.plans[k]);
    e.rho = (cpx<R>*)rho[k];
    e.k1 = (cpx<R>*)w;
    e.k2 = (cpx<R>*)(w + S);
    e.k3 = (cpx<R>*)(w + 2 * S);
    e.bA = (cpx<R>*)(w + 3 * S);
    e.bB = (cpx<R>*)(w + 3 * S + F);
    e.shape = b.shape[i];
    e.variant = b.shape[i] == 3 ? 0 : variant[b.shape[i]];
    m.push_back(e);
  }
  return m;
}

hipError_t upload_tables(cdtwa_batch_s& b, void* const* rho, void* const* ws, const int variant[4]) {
  hipError_t e;
  if (b.dtype == 1) {
    auto m = member_table<double>(b, rho, ws, variant);
    e = hipMemcpy(b.d_members, m.data(), m.size() * sizeof(m[0]), hipMemcpyHostToDevice);
  } else {
    auto m = member_table<float>(b, rho, ws, variant);
    e = hipMemcpy(b.d_members, m.data(), m.size() * sizeof(m[0]), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return e;
  const auto w = work_table(b, variant);
  if ((int64_t)w.size() > b.work_cap) return hipErrorInvalidValue;
  b.n_work = (int64_t)w.size();
  return hipMemcpy(b.d_work, w.data(), w.size() * sizeof(BatchWork), hipMemcpyHostToDevice);
}

// work items of the resident members, the costliest first (longest
// processing time first keeps the tail of the persistent grid short); the
// cost of an item is its trajectories times the entries of their matrices
std::vector<int2> resident_work(const cdtwa_batch_s& b) {
  struct Item {
    int64_t cost;
    int member, first;
  };
  std::vector<Item> it;
  for (size_t i = 0; i < b.resident.size(); ++i) {
    const cdtwa_plan p = b.plans[b.resident[i]];
    const Geom* g = plan_geom(p);
    const int ntr = traj_per_item(*g, b.dtype);
    for (int64_t t = 0; t < g->n_traj; t += ntr) {
      const int64_t n = std::min<int64_t>(ntr, g->n_traj - t);
      it.push_back(Item{n * g->nc * g->D * g->D, (int)i, (int)t});
    }
  }
  std::stable_sort(it.begin(), it.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
  std::vector<int2> w(it.size());
  for (size_t k = 0; k < it.size(); ++k) w[k] = make_int2(it[k].member, it[k].first);
  return w;
}

hipError_t upload_resident(cdtwa_batch_s& b, void* const* rho) {
  const size_t rb = traj_member_bytes(b.dtype);
  std::vector<char> rec(rb * b.resident.size());
  for (size_t i = 0; i < b.resident.size(); ++i) {
    const int k = b.resident[i];
    const Geom* g = plan_geom(b.plans[k]);
    traj_member_fill(*g, b.dtype, rho[k], traj_per_item(*g, b.dtype), rec.data() + i * rb);
  }
  return hipMemcpy(b.d_tmembers, rec.data(), rec.size(), hipMemcpyHostToDevice);
}

// Gangs of the fused members: each member gets the gangs its own launch
// would use (G = min(trajectories, co-resident workgroups / clusters)), and
// the members are packed into waves, first fit by decreasing footprint
// G x clusters, each wave one cooperative launch of members side by side.
// A member alone in its wave (one that fills the device, or that nothing
// fits next to) runs its own path, which is the same thing.  So the batch
// never runs a member with fewer gangs than its own launch would, and it
// gains where several members would each leave most of the device idle.
void plan_gangs(cdtwa_batch_s& b, std::vector<int>& cand) {
  const int slots = fused_multi_slots(b.dtype);
  auto alone = [&](int k) {
    const Geom* g = plan_geom(b.plans[k]);
    const int64_t cap = g->nc > 0 ? slots / g->nc : 0;
    return (int)std::min<int64_t>(g->n_traj, cap);
  };
  auto foot = [&](int k) { return (int64_t)alone(k) * plan_geom(b.plans[k])->nc; };
  std::stable_sort(cand.begin(), cand.end(), [&](int x, int y) { return foot(x) > foot(y); });
  std::vector<std::vector<int>> waves;
  std::vector<int64_t> used;
  for (int k : cand) {
    if (alone(k) < 1) {
      b.own.push_back(k);
      continue;
    }
    size_t w = 0;
    while (w < waves.size() && used[w] + foot(k) > slots) ++w;
    if (w == waves.size()) {
      waves.emplace_back();
      used.push_back(0);
    }
    waves[w].push_back(k);
    used[w] += foot(k);
  }
  for (size_t w = 0; w < waves.size(); ++w) {
    if (waves[w].size() < 2) {
      b.own.push_back(waves[w][0]);
      continue;
    }
    b.fwave.push_back({(int)b.fused.size(), (int)waves[w].size(), (int)used[w]});
    for (int k : waves[w]) {
      b.fused.push_back(k);
      b.fusedG.push_back(alone(k));
    }
    b.fgrid = std::max(b.fgrid, (int)used[w]);
  }
}

// member records, wave by wave; the waves run one after the other and share
// the exchange words
hipError_t upload_fused(cdtwa_batch_s& b, void* const* rho) {
  const size_t rb = fused_member_bytes(b.dtype);
  std::vector<char> rec(rb * b.fused.size());
  for (const auto& wv : b.fwave) {
    int slot = 0;
    for (int i = wv.first; i < wv.first + wv.count; ++i) {
      const int k = b.fused[i];
      PlanLayout L;
      plan_layout(b.plans[k], &L);
      fused_member_fill(*plan_geom(b.plans[k]), b.dtype, rho[k], b.d_fxch + (size_t)slot * 32, L.legs,
                        b.fusedG[i], slot, rec.data() + i * rb);
      slot += b.fusedG[i] * plan_geom(b.plans[k])->nc;
    }
  }
  return hipMemcpy(b.d_fmembers, rec.data(), rec.size(), hipMemcpyHostToDevice);
}

void drop_graph(cdtwa_batch_s& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  b.exec = nullptr;
}

// time candidate (threads, variants) on commutator-mode launches (they write
// only the K1 scratch of every member) and keep the fastest
hipError_t autotune(cdtwa_batch_s& b, void* const* rho, void* const* ws, hipStream_t s) {
  bool present[4] = {false, false, false, false};
  for (int sc : b.shape) present[sc] = true;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return e;
  float best = 1e30f;
  int best_nt = 512, best_v[4] = {0, 0, 0, 0};
  for (int nt : {512, 1024}) {
    for (int mask = 0; mask < 8 && e == hipSuccess; ++mask) {
      int v[4] = {mask & 1, (mask >> 1) & 1, (mask >> 2) & 1, 0};
      bool redundant = false;
      for (int sc = 0; sc < 3; ++sc)
        if (!present[sc] && v[sc]) redundant = true;
      if (redundant) continue;
      e = upload_tables(b, rho, ws, v);
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) e = batch_stage(b.dtype, nt, b.d_members, b.d_work, b.n_work, 0, 0.0, s);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = batch_stage(b.dtype, nt, b.d_members, b.d_work, b.n_work, 0, 0.0, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms < best) {
        best = ms;
        best_nt = nt;
        std::memcpy(best_v, v, sizeof(v));
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  b.nt = best_nt;
  std::memcpy(b.variant, best_v, sizeof(best_v));
  b.tuned = true;
  return upload_tables(b, rho, ws, b.variant);
}

hipError_t capture(cdtwa_batch_s& b, double dt) {
  drop_graph(b);
  hipError_t e = hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal);
  for (int mode = 1; mode <= 4 && e == hipSuccess; ++mode)
    e = batch_stage(b.dtype, b.nt, b.d_members, b.d_work, b.n_work, mode, dt, b.cap);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b.cap, &graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&b.exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e == hipSuccess) b.graph_dt = dt;
  return e;
}

}  // namespace

extern "C" {

cdtwa_status cdtwa_batch_create(const cdtwa_plan* plans, int32_t n, int32_t flags, cdtwa_batch* out) {
  if (!plans || !out || n < 1) return set_error(CDTWA_EINVAL, "batch_create: bad argument");
  *out = nullptr;
  cdtwa_batch_s* b = new (std::nothrow) cdtwa_batch_s;
  if (!b) return set_error(CDTWA_ENOMEM, "batch_create: out of host memory");
  int64_t work = 0;
  std::vector<int> fused_cand;
  for (int32_t i = 0; i < n; ++i) {
    PlanLayout L;
    if (!plans[i] || !plan_layout(plans[i], &L)) {
      delete b;
      return set_error(CDTWA_EINVAL, "batch_create: NULL plan");
    }
    if (i == 0) b->dtype = L.dtype;
    if (L.dtype != b->dtype) {
      delete b;
      return set_error(CDTWA_EINVAL, "batch_create: members differ in state precision");
    }
    const Geom* g = plan_geom(plans[i]);
    b->plans.push_back(plans[i]);
    if (L.path == 6) {
      b->resident.push_back(i);
      continue;
    }
    if (L.path == 1 && !L.wide && g->gdeph == 0 && g->gloss == 0 && !(flags & CDTWA_BATCH_MIX_ALL)) {
      fused_cand.push_back(i);
      b->fspin = std::max(b->fspin, L.spin_limit);
      continue;
    }
    const int sc = shape_code(*g);
    const bool mixable = g->d == 3 && g->model == 0 && g->gdeph == 0 && g->gloss == 0 && (sc != 3 || (flags & CDTWA_BATCH_MIX_ALL) || L.path == 0);
    if (mixable) {
      b->mixed.push_back(i);
      b->shape.push_back(sc);
      // work items of the smallest clusters-per-workgroup variant bound every table
      const int cpb = batch_cpb(sc, sc == 3 ? 0 : 1);
      work += (g->n_traj * g->nc + cpb - 1) / cpb;
    } else {
      b->own.push_back(i);
    }
  }
  if (!fused_cand.empty()) plan_gangs(*b, fused_cand);
  hipError_t e = hipGetDevice(&b->dev);
  const size_t msz = b->dtype == 1 ? sizeof(BatchMember<double>) : sizeof(BatchMember<float>);
  if (e == hipSuccess && !b->mixed.empty()) e = hipMalloc(&b->d_members, msz * b->mixed.size());
  if (e == hipSuccess && !b->mixed.empty()) e = hipMalloc((void**)&b->d_work, sizeof(BatchWork) * (size_t)work);
  b->work_cap = work;
  if (e == hipSuccess && !b->resident.empty()) {
    const auto w = resident_work(*b);
    b->n_twork = (int64_t)w.size();
    e = hipMalloc(&b->d_tmembers, traj_member_bytes(b->dtype) * b->resident.size());
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_twork, sizeof(int2) * w.size());
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_counter, 256);
    if (e == hipSuccess) e = hipMemcpy(b->d_twork, w.data(), sizeof(int2) * w.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && !b->fused.empty()) {
    e = hipMalloc(&b->d_fmembers, fused_member_bytes(b->dtype) * b->fused.size());
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_fxch, sizeof(uint64_t) * 32 * (size_t)b->fgrid);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_fstatus, 256);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    if (b->d_fmembers) (void)hipFree(b->d_fmembers);
    if (b->d_fxch) (void)hipFree(b->d_fxch);
    if (b->d_fstatus) (void)hipFree(b->d_fstatus);
    if (b->d_members) (void)hipFree(b->d_members);
    if (b->d_work) (void)hipFree(b->d_work);
    if (b->d_tmembers) (void)hipFree(b->d_tmembers);
    if (b->d_twork) (void)hipFree(b->d_twork);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
    return hip_err(e, "batch_create");
  }
  *out = b;
  return CDTWA_OK;
}

cdtwa_status cdtwa_batch_destroy(cdtwa_batch b) {
  if (!b) return CDTWA_OK;
  drop_graph(*b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_members) (void)hipFree(b->d_members);
  if (b->d_work) (void)hipFree(b->d_work);
  if (b->d_tmembers) (void)hipFree(b->d_tmembers);
  if (b->d_twork) (void)hipFree(b->d_twork);
  if (b->d_counter) (void)hipFree(b->d_counter);
  if (b->d_fmembers) (void)hipFree(b->d_fmembers);
  if (b->d_fxch) (void)hipFree(b->d_fxch);
  if (b->d_fstatus) (void)hipFree(b->d_fstatus);
  delete b;
  return CDTWA_OK;
}

cdtwa_status cdtwa_batch_workspace_bytes(cdtwa_batch b, int32_t member, size_t* bytes) {
  if (!b || !bytes || member < 0 || member >= (int32_t)b->plans.size())
    return set_error(CDTWA_EINVAL, "batch_workspace_bytes: bad argument");
  cdtwa_plan p = b->plans[member];
  size_t own = 0;
  cdtwa_status st = cdtwa_workspace_bytes(p, &own);
  if (st != CDTWA_OK) return st;
  if (std::find(b->mixed.begin(), b->mixed.end(), member) != b->mixed.end()) {
    PlanLayout L;
    plan_layout(p, &L);
    own = std::max(own, 3 * a256(L.state_bytes) + 2 * a256(L.field_bytes));
  }
  *bytes = own;
  return CDTWA_OK;
}

cdtwa_status cdtwa_batch_info(cdtwa_batch b, int32_t* n_mixed, int32_t* threads, int32_t* variants,
                              int64_t* workgroups, int32_t* n_resident, int64_t* resident_items, int32_t* n_fused,
                              int32_t* fused_workgroups) {
  if (!b) return set_error(CDTWA_EINVAL, "batch_info: NULL batch");
  if (n_fused) *n_fused = (int32_t)b->fused.size();
  if (fused_workgroups) *fused_workgroups = b->fgrid;
  if (n_resident) *n_resident = (int32_t)b->resident.size();
  if (resident_items) *resident_items = b->n_twork;
  if (n_mixed) *n_mixed = (int32_t)b->mixed.size();
  if (threads) *threads = b->tuned ? b->nt : 0;
  if (variants)
    for (int i = 0; i < 3; ++i) variants[i] = b->variant[i];
  if (workgroups) *workgroups = b->n_work;
  return CDTWA_OK;
}

cdtwa_status cdtwa_batch_step_rk4(cdtwa_batch b, void* const* rho, void* const* ws, double dt, int32_t n_steps,
                                  void* stream) {
  if (!b || !rho || !ws) return set_error(CDTWA_EINVAL, "batch_step_rk4: NULL argument");
  if (!(std::isfinite(dt) && dt > 0)) return set_error(CDTWA_EINVAL, "batch_step_rk4: dt must be finite and positive");
  if (n_steps < 0) return set_error(CDTWA_EINVAL, "batch_step_rk4: negative n_steps");
  for (size_t i = 0; i < b->plans.size(); ++i)
    if (!rho[i] || !ws[i]) return set_error(CDTWA_EINVAL, "batch_step_rk4: NULL state or workspace");
  if (n_steps == 0) return CDTWA_OK;
  hipStream_t s = (hipStream_t)stream;
  // members on their own path
  for (int k : b->own) {
    cdtwa_status st = cdtwa_step_rk4(b->plans[k], rho[k], ws[k], dt, n_steps, stream);
    if (st != CDTWA_OK) return st;
  }
  hipError_t e = hipSuccess;
  std::vector<const void*> r(rho, rho + b->plans.size()), w(ws, ws + b->plans.size());
  // the resident members: one persistent launch for all their steps
  if (!b->resident.empty()) {
    if (r != b->last_trho) {
      // earlier launches may still read the member records
      e = hipStreamSynchronize(s);
      if (e == hipSuccess) e = upload_resident(*b, rho);
      if (e != hipSuccess) return hip_err(e, "batch_step_rk4 (resident tables)");
      b->last_trho = r;
    }
    e = traj_batch_rk4(b->dtype, b->d_tmembers, b->d_twork, b->n_twork, b->d_counter, dt, n_steps, s);
    if (e != hipSuccess) return hip_err(e, "batch_step_rk4 (resident)");
  }
  // the fused members: one cooperative launch for all their steps
  if (!b->fused.empty()) {
    if (r != b->last_frho) {
      e = hipStreamSynchronize(s);
      if (e == hipSuccess) e = upload_fused(*b, rho);
      if (e != hipSuccess) return hip_err(e, "batch_step_rk4 (fused tables)");
      b->last_frho = r;
    }
    for (const auto& wv : b->fwave) {
      e = fused_multi_rk4(b->dtype, (const char*)b->d_fmembers + fused_member_bytes(b->dtype) * wv.first, wv.count,
                          wv.grid, b->d_fxch, 32 * (size_t)wv.grid, b->d_fstatus, dt, n_steps, b->fspin, s);
      if (e != hipSuccess) return hip_err(e, "batch_step_rk4 (fused)");
    }
  }
  if (b->mixed.empty()) return CDTWA_OK;
  if (!b->tuned) {
    e = autotune(*b, rho, ws, s);
    if (e != hipSuccess) return hip_err(e, "batch_step_rk4 (tuning)");
    b->last_rho = r;
    b->last_ws = w;
  } else if (r != b->last_rho || w != b->last_ws) {
    // the graph reads the member table at run time: wait for earlier work
    // that may still read it, then rewrite it
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = upload_tables(*b, rho, ws, b->variant);
    if (e != hipSuccess) return hip_err(e, "batch_step_rk4 (tables)");
    b->last_rho = r;
    b->last_ws = w;
  }
  if (!b->exec || b->graph_dt != dt) {
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = capture(*b, dt);
    if (e != hipSuccess) return hip_err(e, "batch_step_rk4 (graph capture)");
  }
  // mean fields of every mixed member's rho, then the captured steps
  for (size_t i = 0; i < b->mixed.size() && e == hipSuccess; ++i) {
    const int k = b->mixed[i];
    PlanLayout L;
    plan_layout(b->plans[k], &L);
    char* bA = (char*)ws[k] + 3 * a256(L.state_bytes);
    e = generic_site_fields(*plan_geom(b->plans[k]), b->dtype, rho[k], bA, s);
  }
  for (int32_t it = 0; it < n_steps && e == hipSuccess; ++it) e = hipGraphLaunch(b->exec, s);
  return e == hipSuccess ? CDTWA_OK : hip_err(e, "batch_step_rk4");
}

}  // extern "C"
