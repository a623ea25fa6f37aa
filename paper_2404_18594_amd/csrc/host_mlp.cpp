// Host side of the learned control variate (C ABI in include/cdtwa.h):
// MLP workspace layout, argument checks and the launch sequences of the
// forward pass, the backward pass, the Adam step, the patch features and the
// expectation of g over i.i.d. patches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/cdtwa.h"
#include "launch.hpp"

using namespace cdtwa;

namespace cdtwa {
// defined in host.cpp
cdtwa_status set_error(cdtwa_status st, const std::string& msg);
const Geom* plan_geom(cdtwa_plan plan);
}  // namespace cdtwa

namespace {

constexpr int NI = CDTWA_MLP_IN, NH = CDTWA_MLP_HIDDEN, NO = CDTWA_MLP_OUT;
// FP32 parameter offsets: W1 [NI][NH], b1, W2 [NH][NH], b2, W3 [NH][NO], b3
constexpr int64_t OW1 = 0, OB1 = OW1 + NI * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
                  OB3 = OW3 + NH * NO, NPAR = OB3 + NO;
// BF16 weight offsets (same matrices, no biases)
constexpr int64_t QW1 = 0, QW2 = QW1 + NI * NH, QW3 = QW2 + NH * NH, NQ = QW3 + NH * NO;
static_assert(NPAR == CDTWA_MLP_PARAMS, "parameter count");
static_assert(NQ == CDTWA_MLP_WBF16, "bf16 weight count");
constexpr int KSPLIT_MAX = 64;
constexpr int64_t CV_CHUNK = 32768;  // patches per forward pass of cdtwa_cv_expectation
constexpr int MOM_BLOCKS = 256;      // partial blocks of the column moments
constexpr int64_t MAX_ROWS = (int64_t)1 << 28;

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

struct MlpWs {
  uint16_t *x0b, *a1b, *a2b, *dyb, *dz2b, *dz1b;
  float *z1, *z2, *dy, *sq, *da2, *dz2, *da1, *dz1, *part, *tmp;
};

// carve the workspace of an n-row batch; base == nullptr only sizes it
size_t mlp_ws_layout(int64_t n, char* base, MlpWs* w) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + o : nullptr;
    o += a256(bytes);
    return p;
  };
  MlpWs t;
  t.x0b = (uint16_t*)take(n * NI * 2);
  t.z1 = (float*)take(n * NH * 4);
  t.a1b = (uint16_t*)take(n * NH * 2);
  t.z2 = (float*)take(n * NH * 4);
  t.a2b = (uint16_t*)take(n * NH * 2);
  t.dy = (float*)take(n * NO * 4);
  t.dyb = (uint16_t*)take(n * NO * 2);
  t.sq = (float*)take(n * NO * 4);
  t.da2 = (float*)take(n * NH * 4);
  t.dz2 = (float*)take(n * NH * 4);
  t.dz2b = (uint16_t*)take(n * NH * 2);
  t.da1 = (float*)take(n * NH * 4);
  t.dz1 = (float*)take(n * NH * 4);
  t.dz1b = (uint16_t*)take(n * NH * 2);
  // split-K partial products of the weight gradients; also the chunk sums
  // of the column sums (which run after each weight gradient is reduced)
  static_assert((size_t)KSPLIT_MAX * NH * NH >= (size_t)COLSUM_MAX_CHUNKS * NH, "column-sum scratch");
  t.part = (float*)take((size_t)KSPLIT_MAX * NH * NH * 4);
  t.tmp = (float*)take(NO * 4);
  if (w) *w = t;
  return o;
}

// expectation workspace: features, outputs, moment partials, then an MLP
// workspace of CV_CHUNK rows
struct CvWs {
  float *feat, *y;
  double* part;
  char* mlp;
};
size_t cv_ws_layout(char* base, CvWs* w) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + o : nullptr;
    o += a256(bytes);
    return p;
  };
  CvWs t;
  t.feat = (float*)take(CV_CHUNK * NI * 4);
  t.y = (float*)take(CV_CHUNK * NO * 4);
  t.part = (double*)take((size_t)MOM_BLOCKS * NO * 2 * 8);
  t.mlp = take(mlp_ws_layout(CV_CHUNK, nullptr, nullptr));
  if (w) *w = t;
  return o;
}

cdtwa_status hip_err(hipError_t e, const char* where) {
  return set_error(CDTWA_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// dW [Mo][No] = A^T dZ with the n batch rows as the reduction, split into
// slices whose partial products are then added in slice order
hipError_t weight_grad(const uint16_t* a, int Mo, const uint16_t* dz, int No, int64_t n, float* part, float* out,
                       hipStream_t s) {
  const int tiles = ((Mo + 31) / 32) * ((No + 31) / 32);
  int64_t ksplit = std::min<int64_t>(KSPLIT_MAX, std::max<int64_t>(1, 1024 / tiles));
  ksplit = std::max<int64_t>(1, std::min<int64_t>(ksplit, n / 16));
  hipError_t e = gemm_bf16(a, 1, Mo, dz, No, 1, part, No, Mo, No, (int)n, (int)ksplit, s);
  if (e == hipSuccess) e = gemm_epilogue(part, (int)ksplit, (int64_t)Mo * No, No, nullptr, out, nullptr, 0, s);
  return e;
}

hipError_t forward(const float* params, const uint16_t* wbf16, const float* x, float* y, int64_t n, const MlpWs& w,
                   hipStream_t s) {
  hipError_t e = to_bf16_array(x, w.x0b, n * NI, s);
  if (e == hipSuccess) e = gemm_bf16(w.x0b, NI, 1, wbf16 + QW1, NH, 1, w.z1, NH, (int)n, NH, NI, 1, s);
  if (e == hipSuccess) e = gemm_epilogue(w.z1, 1, n * NH, NH, params + OB1, w.z1, w.a1b, 1, s);
  if (e == hipSuccess) e = gemm_bf16(w.a1b, NH, 1, wbf16 + QW2, NH, 1, w.z2, NH, (int)n, NH, NH, 1, s);
  if (e == hipSuccess) e = gemm_epilogue(w.z2, 1, n * NH, NH, params + OB2, w.z2, w.a2b, 1, s);
  if (e == hipSuccess) e = gemm_bf16(w.a2b, NH, 1, wbf16 + QW3, NO, 1, y, NO, (int)n, NO, NH, 1, s);
  if (e == hipSuccess) e = gemm_epilogue(y, 1, n * NO, NO, params + OB3, y, nullptr, 0, s);
  return e;
}

// control-variate problems: d = 3 (8 generators) and 2x2 clusters, so that a
// 4x4 patch carries 16 x 8 = CDTWA_MLP_IN features
cdtwa_status check_cv_plan(const Geom* g, const char* where) {
  if (!g) return set_error(CDTWA_EINVAL, std::string(where) + ": NULL plan");
  if (g->n_gen * 16 != NI || g->cx != 2 || g->cy != 2 || g->model != 0)
    return set_error(CDTWA_EUNSUPPORTED, std::string(where) + ": needs the Bose-Hubbard model, d = 3, 2x2 clusters");
  return CDTWA_OK;
}

}  // namespace

extern "C" {

cdtwa_status cdtwa_mlp_workspace_bytes(int64_t n, size_t* bytes) {
  if (n < 1 || n > MAX_ROWS || !bytes) return set_error(CDTWA_EINVAL, "mlp_workspace_bytes: bad argument");
  *bytes = mlp_ws_layout(n, nullptr, nullptr);
  return CDTWA_OK;
}

cdtwa_status cdtwa_mlp_init(float* params, uint16_t* wbf16, uint64_t seed, void* stream) {
  if (!params || !wbf16) return set_error(CDTWA_EINVAL, "mlp_init: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const float bw[3] = {std::sqrt(6.0f / NI), std::sqrt(6.0f / NH), std::sqrt(3.0f / NH)};
  const int64_t wo[3] = {OW1, OW2, OW3}, wn[3] = {NI * NH, NH * NH, NH * NO}, qo[3] = {QW1, QW2, QW3};
  const int64_t bo[3] = {OB1, OB2, OB3}, bn[3] = {NH, NH, NO};
  hipError_t e = hipSuccess;
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    e = mlp_init_layer(params + wo[l], wbf16 + qo[l], wn[l], bw[l], l, seed, s);
    if (e == hipSuccess) e = mlp_init_layer(params + bo[l], nullptr, bn[l], 0.f, l, seed, s);
  }
  return e == hipSuccess ? CDTWA_OK : hip_err(e, "mlp_init");
}

cdtwa_status cdtwa_mlp_forward(const float* params, const uint16_t* wbf16, const float* x, float* y, int64_t n,
                               void* ws, void* stream) {
  if (!params || !wbf16 || !x || !y || !ws) return set_error(CDTWA_EINVAL, "mlp_forward: NULL argument");
  if (n < 1 || n > MAX_ROWS) return set_error(CDTWA_EINVAL, "mlp_forward: bad row count");
  MlpWs w;
  mlp_ws_layout(n, (char*)ws, &w);
  hipError_t e = forward(params, wbf16, x, y, n, w, (hipStream_t)stream);
  return e == hipSuccess ? CDTWA_OK : hip_err(e, "mlp_forward");
}

cdtwa_status cdtwa_mlp_backward(const uint16_t* wbf16, const float* y, const float* target, float* grad, float* loss,
                                int64_t n, void* ws, void* stream) {
  if (!wbf16 || !y || !target || !grad || !ws) return set_error(CDTWA_EINVAL, "mlp_backward: NULL argument");
  if (n < 16 || n % 16 != 0 || n > MAX_ROWS)
    return set_error(CDTWA_EINVAL, "mlp_backward: the row count must be a positive multiple of 16");
  hipStream_t s = (hipStream_t)stream;
  MlpWs w;
  mlp_ws_layout(n, (char*)ws, &w);
  const float scale = 1.0f / (float)(n * NO);
  hipError_t e = mse_grad(y, target, w.dy, w.dyb, w.sq, n * NO, scale, s);
  if (e == hipSuccess && loss) e = colsum(w.sq, n, NO, 1.0f, w.tmp, w.part, s);
  if (e == hipSuccess && loss) e = colsum(w.tmp, NO, 1, scale, loss, w.part, s);
  // layer 3
  if (e == hipSuccess) e = weight_grad(w.a2b, NH, w.dyb, NO, n, w.part, grad + OW3, s);
  if (e == hipSuccess) e = colsum(w.dy, n, NO, 1.0f, grad + OB3, w.part, s);
  if (e == hipSuccess) e = gemm_bf16(w.dyb, NO, 1, wbf16 + QW3, 1, NO, w.da2, NH, (int)n, NH, NO, 1, s);
  if (e == hipSuccess) e = relu_back(w.da2, w.z2, w.dz2, w.dz2b, n * NH, s);
  // layer 2
  if (e == hipSuccess) e = weight_grad(w.a1b, NH, w.dz2b, NH, n, w.part, grad + OW2, s);
  if (e == hipSuccess) e = colsum(w.dz2, n, NH, 1.0f, grad + OB2, w.part, s);
  if (e == hipSuccess) e = gemm_bf16(w.dz2b, NH, 1, wbf16 + QW2, 1, NH, w.da1, NH, (int)n, NH, NH, 1, s);
  if (e == hipSuccess) e = relu_back(w.da1, w.z1, w.dz1, w.dz1b, n * NH, s);
  // layer 1
  if (e == hipSuccess) e = weight_grad(w.x0b, NI, w.dz1b, NH, n, w.part, grad + OW1, s);
  if (e == hipSuccess) e = colsum(w.dz1, n, NH, 1.0f, grad + OB1, w.part, s);
  return e == hipSuccess ? CDTWA_OK : hip_err(e, "mlp_backward");
}

cdtwa_status cdtwa_mlp_adam(float* params, uint16_t* wbf16, const float* grad, float* m, float* v, float lr,
                            int32_t step, void* stream) {
  if (!params || !wbf16 || !grad || !m || !v) return set_error(CDTWA_EINVAL, "mlp_adam: NULL argument");
  if (step < 1 || !(lr > 0) || !std::isfinite(lr)) return set_error(CDTWA_EINVAL, "mlp_adam: bad step or rate");
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, step)), c2 = (float)(1.0 - std::pow(b2, step));
  hipStream_t s = (hipStream_t)stream;
  const int64_t wo[3] = {OW1, OW2, OW3}, wn[3] = {NI * NH, NH * NH, NH * NO}, qo[3] = {QW1, QW2, QW3};
  const int64_t bo[3] = {OB1, OB2, OB3}, bn[3] = {NH, NH, NO};
  hipError_t e = hipSuccess;
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    e = adam_update(params + wo[l], wbf16 + qo[l], grad + wo[l], m + wo[l], v + wo[l], wn[l], lr, (float)b1,
                    (float)b2, 1e-8f, c1, c2, s);
    if (e == hipSuccess)
      e = adam_update(params + bo[l], nullptr, grad + bo[l], m + bo[l], v + bo[l], bn[l], lr, (float)b1, (float)b2,
                      1e-8f, c1, c2, s);
  }
  return e == hipSuccess ? CDTWA_OK : hip_err(e, "mlp_adam");
}

cdtwa_status cdtwa_cv_features(cdtwa_plan plan, const int8_t* noise, float* features, void* stream) {
  const Geom* g = plan_geom(plan);
  cdtwa_status st = check_cv_plan(g, "cv_features");
  if (st != CDTWA_OK) return st;
  if (!noise || !features) return set_error(CDTWA_EINVAL, "cv_features: NULL argument");
  hipError_t e = cv_features(*g, noise, features, (hipStream_t)stream);
  return e == hipSuccess ? CDTWA_OK : hip_err(e, "cv_features");
}

cdtwa_status cdtwa_cv_sample_features(cdtwa_plan plan, uint64_t seed, int64_t first, int64_t n, float* features,
                                      void* stream) {
  const Geom* g = plan_geom(plan);
  cdtwa_status st = check_cv_plan(g, "cv_sample_features");
  if (st != CDTWA_OK) return st;
  if (!features || n < 1 || n > MAX_ROWS || first < 0)
    return set_error(CDTWA_EINVAL, "cv_sample_features: bad argument");
  hipError_t e = cv_sample_features(*g, seed, first, n, features, (hipStream_t)stream);
  return e == hipSuccess ? CDTWA_OK : hip_err(e, "cv_sample_features");
}

cdtwa_status cdtwa_cv_traj_sums(cdtwa_plan plan, const float* y, double* gtraj, void* stream) {
  const Geom* g = plan_geom(plan);
  cdtwa_status st = check_cv_plan(g, "cv_traj_sums");
  if (st != CDTWA_OK) return st;
  if (!y || !gtraj) return set_error(CDTWA_EINVAL, "cv_traj_sums: NULL argument");
  hipError_t e = traj_sums(y, g->n_traj, g->nc, NO, 1.0 / g->Ns, gtraj, (hipStream_t)stream);
  return e == hipSuccess ? CDTWA_OK : hip_err(e, "cv_traj_sums");
}

cdtwa_status cdtwa_cv_workspace_bytes(size_t* bytes) {
  if (!bytes) return set_error(CDTWA_EINVAL, "cv_workspace_bytes: NULL argument");
  *bytes = cv_ws_layout(nullptr, nullptr);
  return CDTWA_OK;
}

cdtwa_status cdtwa_cv_expectation(cdtwa_plan plan, const float* params, const uint16_t* wbf16, uint64_t seed,
                                  int64_t n_samples, double* moments, void* ws, void* stream) {
  const Geom* g = plan_geom(plan);
  cdtwa_status st = check_cv_plan(g, "cv_expectation");
  if (st != CDTWA_OK) return st;
  if (!params || !wbf16 || !moments || !ws) return set_error(CDTWA_EINVAL, "cv_expectation: NULL argument");
  if (n_samples < 1) return set_error(CDTWA_EINVAL, "cv_expectation: n_samples must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  CvWs w;
  cv_ws_layout((char*)ws, &w);
  MlpWs mw;
  mlp_ws_layout(CV_CHUNK, w.mlp, &mw);
  hipError_t e = hipSuccess;
  for (int64_t first = 0; first < n_samples && e == hipSuccess; first += CV_CHUNK) {
    const int64_t n = std::min<int64_t>(CV_CHUNK, n_samples - first);
    e = cv_sample_features(*g, seed, first, n, w.feat, s);
    if (e == hipSuccess) e = forward(params, wbf16, w.feat, w.y, n, mw, s);
    if (e == hipSuccess) e = colmoments(w.y, n, NO, w.part, MOM_BLOCKS, moments, s);
  }
  return e == hipSuccess ? CDTWA_OK : hip_err(e, "cv_expectation");
}

}  // extern "C"
