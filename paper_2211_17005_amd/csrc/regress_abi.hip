// C-ABI of the regression: cva_regress_fit / cva_regress_predict.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>

#include "../../include/hsim.h"
#include "abi_internal.hpp"
#include "regress.hpp"
#include "regress_plain.hpp"

using namespace hsim;

namespace {

bool plain(const cva_mlp_cfg* c) { return c->dtype == HSIM_REG_FP32 || c->dtype == HSIM_REG_FP64; }
size_t elem_bytes(const cva_mlp_cfg* c) { return c->dtype == HSIM_REG_FP64 ? sizeof(double) : sizeof(float); }

int check_cfg(const cva_mlp_cfg* c) {
  if (!c) return fail(HSIM_EINVAL, "cfg is NULL");
  if (c->dtype != HSIM_REG_BF16 && !plain(c)) return fail(HSIM_EINVAL, "unknown regression dtype %d", c->dtype);
  if (plain(c)) {
    if (c->width < 1 || c->width > kPlainMaxWidth || c->hidden < 1 || c->hidden > 3)
      return fail(HSIM_EUNSUPPORTED, "width=%d hidden=%d outside 1..%d x 1..3", c->width, c->hidden, kPlainMaxWidth);
  } else if (!mlp_supported(c->width, c->hidden)) {
    return fail(HSIM_EUNSUPPORTED, "no kernel built for width=%d hidden=%d", c->width, c->hidden);
  }
  const int dmax = plain(c) ? kMlpDinWide : kMlpDin;
  if (c->d_in < 1 || c->d_in > dmax) return fail(HSIM_ERANGE, "d_in=%d out of [1,%d]", c->d_in, dmax);
  if (c->epochs < 1 || c->batch < 1) return fail(HSIM_EINVAL, "epochs and batch must be >= 1");
  if (c->team < 0 || c->team > 32) return fail(HSIM_ERANGE, "team=%d out of [0,32]", c->team);
  if (c->tile < 0 || c->tile >= kMlpTiles || (plain(c) && c->tile != 0))
    return fail(HSIM_ERANGE, "tile=%d out of [0,%d) (0 for the FP32 / FP64 form)", c->tile, kMlpTiles);
  if (!(c->lr >= 0.0) || !(c->beta1 >= 0.0 && c->beta1 < 1.0) || !(c->beta2 >= 0.0 && c->beta2 < 1.0) ||
      !(c->eps > 0.0))
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
  a.lr = (float)c->lr;
  a.beta1 = (float)c->beta1;
  a.beta2 = (float)c->beta2;
  a.eps = (float)c->eps;
  a.n_reg = n_reg;
  a.M = M;
  a.n_feat = n_feat;
  a.init_tag = c->init_tag;
  a.tile = c->tile;
  for (int j = 0; j < n_reg; ++j) a.dates[j] = dates[j];
  return HSIM_OK;
}

// Team size (workgroups per date) and number of teams of one training launch over n_dates dates:
// the configured size, else as many workgroups per date as the device holds for all dates at
// once, at most one per four chunks of a batch and at most 32 (one XCD).
bool choose_team(const cva_mlp_cfg* c, int n_dates, int& G, int& n_teams) {
  const int chunks = (c->batch + kMlpRows - 1) / kMlpRows;
  const int resident = mlp_max_teams(c->width, c->hidden, 1);
  if (resident <= 0) return false;
  if (c->team > 0) {
    G = c->team;
  } else {
    G = resident / n_dates;
    G = G < chunks / 4 ? G : chunks / 4;
    G = G < 32 ? G : 32;
    G = G > 1 ? G : 1;
  }
  const int max_teams = mlp_max_teams(c->width, c->hidden, G);
  if (max_teams <= 0) return false;
  n_teams = n_dates < max_teams ? n_dates : max_teams;
  return true;
}

// Loss helpers run when every date has its team in the one launch and the device holds more
// workgroups than the teams use (batched mode only).
bool use_loss_helpers(const cva_mlp_cfg* c, int n_reg, int G, int n_teams) {
  if (c->warm_start || n_teams != n_reg) return false;
  const int capacity = mlp_max_teams(c->width, c->hidden, 1);
  return capacity > G * n_teams;
}

struct RegWs {
  size_t params, partial, gram, loss, ctr, snaps, flags, losses, total;
};

RegWs reg_ws(const cva_mlp_cfg* c, int n_reg, int G, int n_teams) {
  const MlpLayout L{c->width, c->hidden};
  const size_t np = (size_t)L.n_params();
  const bool helpers = use_loss_helpers(c, n_reg, G, n_teams);
  const size_t ne = (size_t)n_reg * c->epochs;
  RegWs w;
  w.params = align256(3 * np * n_reg * sizeof(float));
  w.partial = align256(G > 1 ? np * G * n_teams * sizeof(float) : 0);
  w.gram = align256((size_t)(c->width + 1) * (c->width + 2) * G * n_teams * sizeof(double));
  w.loss = align256((size_t)G * n_teams * sizeof(double));
  w.ctr = align256((size_t)(n_teams + 1) * sizeof(int32_t));   // team counters, then the status word
  w.snaps = helpers ? align256(ne * np * sizeof(float)) : 0;
  w.flags = helpers ? align256((ne + n_reg + 1) * sizeof(int32_t)) : 0;    // ready, done, queue
  w.losses = helpers ? align256(ne * sizeof(float)) : 0;
  w.total = w.params + w.partial + w.gram + w.loss + w.ctr + w.snaps + w.flags + w.losses;
  return w;
}

__global__ void copy_params(const float* src, float* dst, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

__global__ void zero_word(int32_t* p) { *p = 0; }

// Polls of the bounded waits (team barriers, loss helpers) before they give up; 0: the default.
std::atomic<int32_t> g_wait_limit{0};

int32_t wait_limit() {
  const int32_t v = g_wait_limit.load(std::memory_order_relaxed);
  return v > 0 ? v : kTeamSpinLimit;
}

// Waits for the fit and maps its status word: a bounded wait that gave up is HSIM_ETIMEOUT.
int read_status(const int32_t* status_dev, hipStream_t s) {
  int32_t st = 0;
  hipError_t e = hipMemcpyAsync(&st, status_dev, sizeof(st), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return device_error(e, "regression status read");
  if (st != 0)
    return fail(HSIM_ETIMEOUT, "a bounded wait of the regression gave up (%s): the fit is incomplete",
                (st & 1) ? "team barrier" : "loss snapshot");
  return HSIM_OK;
}

}  // namespace

extern "C" {

int hsim_set_wait_limit(int32_t polls) {
  if (polls < 0) return fail(HSIM_EINVAL, "polls must be >= 0");
  g_wait_limit.store(polls, std::memory_order_relaxed);
  return HSIM_OK;
}

int cva_regress_adam_state(const cva_mlp_cfg* c, int32_t n_reg, int64_t M, const void* workspace_dev, size_t ws_bytes,
                           void* params_dev, void* m_dev, void* v_dev, void* stream) {
  if (cva_regress_workspace_bytes(c, n_reg, M) == 0) return fail(HSIM_EINVAL, "bad cfg or n_reg");
  if (!workspace_dev || ws_bytes < cva_regress_workspace_bytes(c, n_reg, M))
    return fail(HSIM_ENOWS, "workspace smaller than the fit's");
  // both paths keep the parameters, then m, then v of every date at the head of the workspace
  const size_t bytes = (size_t)MlpLayout{c->width, c->hidden, din_pad(c->d_in)}.n_params() * n_reg * elem_bytes(c);
  const char* src = (const char*)workspace_dev;
  void* dst[3] = {params_dev, m_dev, v_dev};
  for (int k = 0; k < 3; ++k) {
    if (!dst[k]) continue;
    const hipError_t e = hipMemcpyAsync(dst[k], (const char*)src + k * bytes, bytes, hipMemcpyDeviceToDevice,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return device_error(e, "Adam state copy");
  }
  return HSIM_OK;
}

int cva_regress_param_floats(const cva_mlp_cfg* c) {
  int rc = check_cfg(c);
  if (rc) return rc;
  return MlpLayout{c->width, c->hidden, din_pad(c->d_in)}.n_params();
}

int cva_regress_record_floats(const cva_mlp_cfg* c) {
  int rc = check_cfg(c);
  if (rc) return rc;
  return MlpLayout{c->width, c->hidden, din_pad(c->d_in)}.record();
}

size_t cva_regress_workspace_bytes(const cva_mlp_cfg* c, int32_t n_reg, int64_t M) {
  if (!c || n_reg < 1 || check_cfg(c) != HSIM_OK) return 0;
  if (plain(c)) return M >= 1 ? plain_workspace_bytes(c, n_reg, M) : 0;
  int G = 0, n_teams = 0;
  if (!choose_team(c, c->warm_start ? 1 : n_reg, G, n_teams)) return 0;
  return reg_ws(c, n_reg, G, n_teams).total;
}

int cva_regress_fit(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int32_t n_dates_total, int64_t M,
                    int32_t n_feat, const void* X_dev, const void* Y_dev, const void* W_dev, uint64_t seed,
                    void* model_dev, void* loss_hist_dev, void* workspace_dev, size_t ws_bytes, void* stream) {
  MlpArgs a;
  int rc = fill_args(c, n_reg, dates, n_dates_total, M, n_feat, a);
  if (rc) return rc;
  if (!X_dev || !Y_dev || !model_dev) return fail(HSIM_EINVAL, "X, Y and model must not be NULL");
  if (!plain(c) && ((uintptr_t)model_dev & 7u))
    return fail(HSIM_EINVAL, "model must be 8-byte aligned (weights are read in pairs)");
  if (plain(c))
    return plain_fit(c, n_reg, dates, M, n_feat, X_dev, Y_dev, W_dev, seed, model_dev, loss_hist_dev, workspace_dev,
                     ws_bytes, (hipStream_t)stream);
  int G = 0, n_teams = 0;
  if (!choose_team(c, c->warm_start ? 1 : n_reg, G, n_teams))
    return fail(HSIM_EDEVICE, "no team of %d workgroups fits on the device", c->team);
  const RegWs ws = reg_ws(c, n_reg, G, n_teams);
  if (!workspace_dev || ws_bytes < ws.total) return fail(HSIM_ENOWS, "workspace %zu < %zu bytes", ws_bytes, ws.total);
  const MlpLayout L{c->width, c->hidden};
  const size_t np = (size_t)L.n_params();
  char* w = (char*)workspace_dev;
  a.cur = (float*)w;
  a.adam_m = a.cur + np * n_reg;
  a.adam_v = a.adam_m + np * n_reg;
  w += ws.params;
  a.partial = (float*)w;
  w += ws.partial;
  a.gram = (double*)w;
  w += ws.gram;
  a.loss_part = (double*)w;
  w += ws.loss;
  a.team_ctr = (int32_t*)w;
  a.status = a.team_ctr + n_teams;
  a.spin_limit = wait_limit();
  w += ws.ctr;
  a.G = G;
  a.n_teams = n_teams;
  a.snaps = nullptr;
  a.n_blocks = 0;
  if (ws.snaps) {
    a.snaps = (float*)w;
    w += ws.snaps;
    a.ready = (int32_t*)w;
    a.done = a.ready + (size_t)n_reg * c->epochs;
    a.lqueue = a.done + n_reg;
    w += ws.flags;
    a.losses = (float*)w;
    a.n_blocks = mlp_max_teams(c->width, c->hidden, 1);
  }
  a.X = (const float*)X_dev;
  a.Y = (const float*)Y_dev;
  a.Wt = (const float*)W_dev;
  a.model = (float*)model_dev;
  a.loss_hist = (float*)loss_hist_dev;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(zero_word, dim3(1), dim3(1), 0, s, a.status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return device_error(e, "status reset");
  e = launch_mlp_stats(a, s);
  if (e != hipSuccess) return device_error(e, "regression statistics launch");
  if (!c->warm_start) {
    a.use_init = 0;
    e = launch_mlp_train(a, s);
    if (e != hipSuccess) return device_error(e, "regression training launch");
    return read_status(a.status, s);
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
    b.loss_hist = a.loss_hist ? a.loss_hist + (size_t)c->epochs * j : nullptr;
    b.use_init = j > 0;
    if (j > 0) {
      hipLaunchKernelGGL(copy_params, dim3(1), dim3(256), 0, s, a.model + (size_t)(j - 1) * L.record(),
                         b.model, (int)np);
      if ((e = hipGetLastError()) != hipSuccess) return device_error(e, "warm-start copy");
    }
    e = launch_mlp_train(b, s);
    if (e != hipSuccess) return device_error(e, "regression training launch");
  }
  return read_status(a.status, s);
}

int cva_regress_predict(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int32_t n_dates_total, int64_t M,
                        int32_t n_feat, const void* X_dev, const void* model_dev, void* out_dev, void* stream) {
  MlpArgs a;
  int rc = fill_args(c, n_reg, dates, n_dates_total, M, n_feat, a);
  if (rc) return rc;
  if (!X_dev || !model_dev || !out_dev) return fail(HSIM_EINVAL, "X, model and out must not be NULL");
  if (!plain(c) && ((uintptr_t)model_dev & 7u))
    return fail(HSIM_EINVAL, "model must be 8-byte aligned (weights are read in pairs)");
  if (plain(c)) return plain_predict(c, n_reg, dates, M, n_feat, X_dev, model_dev, out_dev, (hipStream_t)stream);
  a.X = (const float*)X_dev;
  a.Y = nullptr;
  a.Wt = nullptr;
  a.model = (float*)model_dev;
  hipError_t e = launch_mlp_predict(a, (float*)out_dev, (hipStream_t)stream);
  return e == hipSuccess ? HSIM_OK : device_error(e, "prediction launch");
}

}  // extern "C"
