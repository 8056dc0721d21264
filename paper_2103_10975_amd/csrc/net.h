// Guess network: host-side interface.
#pragma once

#include "common.h"

namespace mlg {

int64_t net_param_count(const guess_net_cfg* cfg);
int64_t net_param_offset(const guess_net_cfg* cfg, int index);
size_t net_param_bytes(const guess_net_cfg* cfg);
size_t net_workspace_bytes(const guess_net_cfg* cfg, const mlg_grid* grid, int batch, int train);
int net_init(const guess_net_cfg* cfg, void* params, hipStream_t stream);
int net_refresh(const guess_net_cfg* cfg, void* params, hipStream_t stream);
int net_infer(const guess_net_cfg* cfg, const void* params, const mlg_grid* grid, int batch,
              const double* f, const double* u_prev, double* guess, void* ws, size_t ws_bytes,
              hipStream_t stream);
int net_train_step(const guess_net_cfg* cfg, void* params, const mlg_grid* grid, int batch,
                   const double* const* f, const double* const* u_prev,
                   const double* const* u_target, void* ws, size_t ws_bytes, float* loss,
                   hipStream_t stream);

int64_t fluid_param_count(const fluid_net_cfg* cfg);
int64_t fluid_param_offset(const fluid_net_cfg* cfg, int index);
size_t fluid_param_bytes(const fluid_net_cfg* cfg);
size_t fluid_workspace_bytes(const fluid_net_cfg* cfg, const mlg_grid* grid, int batch, int train);
int fluid_init(const fluid_net_cfg* cfg, void* params, hipStream_t stream);
int fluid_refresh(const fluid_net_cfg* cfg, void* params, hipStream_t stream);
int fluid_infer(const fluid_net_cfg* cfg, const void* params, int blocks, const mlg_grid* grid,
                int batch, const double* f, const double* u_prev, double* guess, void* ws,
                size_t ws_bytes, hipStream_t stream);
int fluid_train_step(const fluid_net_cfg* cfg, void* params, int blocks, const mlg_grid* grid,
                     int batch, const double* const* f, const double* const* u_prev,
                     const double* const* u_target, void* ws, size_t ws_bytes, float* loss,
                     hipStream_t stream);

}  // namespace mlg
