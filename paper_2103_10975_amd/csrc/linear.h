// Single-layer linear guess model: host-side interface.
#pragma once

#include "common.h"

namespace mlg {

size_t lin_param_bytes(const mlg_grid* grid);
size_t lin_workspace_bytes(const mlg_grid* grid, int batch);
int lin_init(const mlg_grid* grid, void* params, hipStream_t stream);
int lin_infer(const mlg_grid* grid, const void* params, int batch, const double* b, double* x0,
              hipStream_t stream);
int lin_train_step(const mlg_grid* grid, void* params, float lr, int batch,
                   const double* const* b, const double* const* x, void* ws, size_t ws_bytes,
                   float* loss, hipStream_t stream);

}  // namespace mlg
