// Internal interface of the FP32 / FP64 regression path (rocBLAS products, date after date).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hsim.h"

namespace hsim {

constexpr int kPlainMaxWidth = 128;   // units per hidden layer (up to three hidden layers)

size_t plain_workspace_bytes(const cva_mlp_cfg* c, int32_t n_reg, int64_t M);
// Element type of X, Y, W, model and loss history: float (HSIM_REG_FP32) or double (HSIM_REG_FP64).
int plain_fit(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int64_t M, int32_t n_feat, const void* X,
              const void* Y, const void* W, uint64_t seed, void* model, void* loss_hist, void* ws, size_t ws_bytes,
              hipStream_t s);
int plain_predict(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int64_t M, int32_t n_feat,
                  const void* X, const void* model, void* out, hipStream_t s);

}  // namespace hsim
