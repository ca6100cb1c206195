// C-ABI of the regression: cva_regress_fit / cva_regress_predict.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/hsim.h"
#include "abi_internal.hpp"
#include "regress.hpp"

using namespace hsim;

namespace {

int check_cfg(const cva_mlp_cfg* c) {
  if (!c) return fail(HSIM_EINVAL, "cfg is NULL");
  if (!mlp_supported(c->width, c->hidden))
    return fail(HSIM_EUNSUPPORTED, "no kernel built for width=%d hidden=%d", c->width, c->hidden);
  if (c->d_in < 1 || c->d_in > kMlpDin) return fail(HSIM_ERANGE, "d_in=%d out of [1,%d]", c->d_in, kMlpDin);
  if (c->epochs < 1 || c->batch < 1) return fail(HSIM_EINVAL, "epochs and batch must be >= 1");
  if (!(c->lr > 0.0f) || !(c->beta1 >= 0.0f && c->beta1 < 1.0f) || !(c->beta2 >= 0.0f && c->beta2 < 1.0f) ||
      !(c->eps > 0.0f))
    return fail(HSIM_EINVAL, "bad Adam hyper-parameters");
  return HSIM_OK;
}

int fill_args(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int32_t n_dates_total, int64_t M,
              int32_t n_feat, MlpArgs& a) {
  int rc = check_cfg(c);
  if (rc) return rc;
  if (n_reg < 1 || n_reg > kMaxRegDates) return fail(HSIM_ERANGE, "n_reg=%d out of [1,%d]", n_reg, kMaxRegDates);
  if (!dates) return fail(HSIM_EINVAL, "dates is NULL");
  if (M < 1) return fail(HSIM_EINVAL, "M must be >= 1");
  if (n_feat < c->d_in) return fail(HSIM_EINVAL, "n_feat=%d < d_in=%d", n_feat, c->d_in);
  for (int j = 0; j < n_reg; ++j)
    if (dates[j] < 0 || dates[j] >= n_dates_total) return fail(HSIM_EINVAL, "date %d out of [0,%d)", dates[j], n_dates_total);
  memset(&a, 0, sizeof(a));
  a.U = c->width;
  a.H = c->hidden;
  a.d_in = c->d_in;
  a.epochs = c->epochs;
  a.batch = c->batch;
  a.lr = c->lr;
  a.beta1 = c->beta1;
  a.beta2 = c->beta2;
  a.eps = c->eps;
  a.n_reg = n_reg;
  a.M = M;
  a.n_feat = n_feat;
  a.init_tag = c->init_tag;
  for (int j = 0; j < n_reg; ++j) a.dates[j] = dates[j];
  return HSIM_OK;
}

int n_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return n;
}

__global__ void copy_params(const float* src, float* dst, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

}  // namespace

extern "C" {

int cva_regress_record_floats(const cva_mlp_cfg* c) {
  int rc = check_cfg(c);
  if (rc) return rc;
  return MlpLayout{c->width, c->hidden}.record();
}

size_t cva_regress_workspace_bytes(const cva_mlp_cfg* c, int32_t n_reg, int64_t M) {
  (void)M;
  if (!c || n_reg < 1) return 0;
  const MlpLayout L{c->width, c->hidden};
  const size_t np = (size_t)L.n_params();
  return align256(3 * np * n_reg * sizeof(float)) +
         align256((size_t)(c->width + 1) * (c->width + 2) * n_reg * sizeof(double)) + 256;
}

int cva_regress_fit(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int32_t n_dates_total, int64_t M,
                    int32_t n_feat, const float* X_dev, const float* Y_dev, uint64_t seed, float* model_dev,
                    float* loss_hist_dev, void* workspace_dev, size_t ws_bytes, void* stream) {
  MlpArgs a;
  int rc = fill_args(c, n_reg, dates, n_dates_total, M, n_feat, a);
  if (rc) return rc;
  if (!X_dev || !Y_dev || !model_dev) return fail(HSIM_EINVAL, "X, Y and model must not be NULL");
  const size_t need = cva_regress_workspace_bytes(c, n_reg, M);
  if (!workspace_dev || ws_bytes < need) return fail(HSIM_ENOWS, "workspace %zu < %zu bytes", ws_bytes, need);
  const MlpLayout L{c->width, c->hidden};
  const size_t np = (size_t)L.n_params();
  char* w = (char*)workspace_dev;
  a.cur = (float*)w;
  a.adam_m = a.cur + np * n_reg;
  a.adam_v = a.adam_m + np * n_reg;
  w += align256(3 * np * n_reg * sizeof(float));
  a.gram = (double*)w;
  w += align256((size_t)(c->width + 1) * (c->width + 2) * n_reg * sizeof(double));
  a.queue = (int32_t*)w;
  a.X = X_dev;
  a.Y = Y_dev;
  a.model = model_dev;
  a.loss_hist = loss_hist_dev;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_mlp_stats(a, s);
  if (e != hipSuccess) return device_error(e, "regression statistics launch");
  if (!c->warm_start) {
    a.use_init = 0;
    int ncu = n_cus();
    if (ncu <= 0) return fail(HSIM_EDEVICE, "cannot query the number of compute units");
    e = launch_mlp_train(a, n_reg < ncu ? n_reg : ncu, s);
    if (e != hipSuccess) return device_error(e, "regression training launch");
    return HSIM_OK;
  }
  // Backward learning: dates in the given order, each started from the previous result.
  for (int j = 0; j < n_reg; ++j) {
    MlpArgs b = a;
    b.n_reg = 1;
    b.dates[0] = a.dates[j];
    b.model = a.model + (size_t)j * L.record();
    b.cur = a.cur + np * j;
    b.adam_m = a.adam_m + np * j;
    b.adam_v = a.adam_v + np * j;
    b.gram = a.gram + (size_t)(c->width + 1) * (c->width + 2) * j;
    b.loss_hist = a.loss_hist ? a.loss_hist + (size_t)c->epochs * j : nullptr;
    b.use_init = j > 0;
    if (j > 0) {
      hipLaunchKernelGGL(copy_params, dim3(1), dim3(256), 0, s, a.model + (size_t)(j - 1) * L.record(),
                         b.model, (int)np);
      if ((e = hipGetLastError()) != hipSuccess) return device_error(e, "warm-start copy");
    }
    e = launch_mlp_train(b, 1, s);
    if (e != hipSuccess) return device_error(e, "regression training launch");
  }
  return HSIM_OK;
}

int cva_regress_predict(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int32_t n_dates_total, int64_t M,
                        int32_t n_feat, const float* X_dev, const float* model_dev, float* out_dev, void* stream) {
  MlpArgs a;
  int rc = fill_args(c, n_reg, dates, n_dates_total, M, n_feat, a);
  if (rc) return rc;
  if (!X_dev || !model_dev || !out_dev) return fail(HSIM_EINVAL, "X, model and out must not be NULL");
  a.X = X_dev;
  a.Y = nullptr;
  a.model = (float*)model_dev;
  hipError_t e = launch_mlp_predict(a, out_dev, (hipStream_t)stream);
  return e == hipSuccess ? HSIM_OK : device_error(e, "prediction launch");
}

}  // extern "C"
