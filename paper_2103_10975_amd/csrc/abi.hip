// extern "C" boundary: argument checks, exception-to-status translation and
// the thread-local error message.
#include <string>

#include "engine.h"
#include "net.h"
#include "linear.h"
#include "batched.h"

namespace mlg {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace mlg

using namespace mlg;

template <class F>
static int guarded(F&& f) {
  try {
    return f();
  } catch (const ArgError& e) {
    set_error(e.msg);
    return e.code;
  } catch (const HipError& e) {
    set_error(std::string(hipGetErrorString(e.code)) + " in " + e.where);
    return MLG_ERR_HIP;
  } catch (const std::exception& e) {
    set_error(e.what());
    return MLG_ERR_HIP;
  } catch (...) {
    set_error("unknown error");
    return MLG_ERR_HIP;
  }
}

extern "C" {

const char* mlg_last_error(void) { return g_last_error.c_str(); }

void mlg_shutdown(void) {
  try {
    runtime_shutdown();
    batched_shutdown();
    autotune_clear();
  } catch (...) {
  }
}

size_t gmres_workspace_bytes(const mlg_grid* grid, const mlg_opts* opts) {
  size_t out = 0;
  int rc = guarded([&] {
    out = solve_workspace_bytes(grid, opts);
    return 0;
  });
  return rc == 0 ? out : 0;
}

int gmres_solve(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts, void* ws,
                size_t ws_bytes, mlg_stats* stats, void* stream) {
  return guarded([&] { return solve(grid, b, x, opts, ws, ws_bytes, stats, (hipStream_t)stream); });
}

int gmres_solve_static(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts,
                       mlg_stats* stats, void* stream) {
  return guarded([&] { return solve_static(grid, b, x, opts, stats, (hipStream_t)stream); });
}

size_t gmres_batched_workspace_bytes(int32_t nsys, const mlg_system* sys, const mlg_opts* opts) {
  size_t out = 0;
  int rc = guarded([&] {
    out = batched_workspace_bytes(nsys, sys, opts);
    return 0;
  });
  return rc == 0 ? out : 0;
}

int gmres_solve_batched(int32_t nsys, const mlg_system* sys, const mlg_opts* opts, void* ws,
                        size_t ws_bytes, mlg_stats* stats, void* stream) {
  return guarded(
      [&] { return batched_solve(nsys, sys, opts, ws, ws_bytes, stats, (hipStream_t)stream); });
}

int mlg_apply_operator(const mlg_grid* grid, const double* u, double* y, void* stream) {
  return guarded([&] { return apply_operator(grid, u, y, (hipStream_t)stream); });
}

size_t mlg_kernel_bench_scratch_bytes(int32_t reps) {
  return reps > 0 ? kernel_bench_scratch_bytes(reps) : 0;
}

int mlg_kernel_bench(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes,
                     void* scratch, size_t scratch_bytes, int32_t kind, int32_t step, int32_t reps,
                     double* avg_us, void* stream) {
  return guarded([&] {
    if (!avg_us) throw ArgError{MLG_ERR_ARG, "avg_us is NULL"};
    *avg_us = kernel_bench(grid, opts, ws, ws_bytes, scratch, scratch_bytes, kind, step, reps,
                           (hipStream_t)stream);
    return 0;
  });
}

size_t mlg_autotune_workspace_bytes(const mlg_grid* grid, const mlg_opts* opts) {
  size_t out = 0;
  int rc = guarded([&] {
    out = autotune_workspace_bytes(grid, opts);
    return 0;
  });
  return rc == 0 ? out : 0;
}

int mlg_autotune(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes,
                 int32_t* tile, uint64_t* fused, uint64_t* split, int32_t* launch,
                 void* stream) {
  return guarded([&] {
    int t = 0, l = 0;
    unsigned long long f = 0, sp = 0;
    const int rc = autotune(grid, opts, ws, ws_bytes, &t, &f, &sp, &l, (hipStream_t)stream);
    if (tile) *tile = t;
    if (fused) *fused = (uint64_t)f;
    if (split) *split = (uint64_t)sp;
    if (launch) *launch = l;
    return rc;
  });
}

int32_t mlg_tile_count(int32_t dim) { return (dim == 2 || dim == 3) ? tile_count(dim) : 0; }

int mlg_tile_shape(int32_t dim, int32_t index, int32_t* tx, int32_t* ty, int32_t* tz) {
  return guarded([&] {
    if ((dim != 2 && dim != 3) || index < 0 || index >= tile_count(dim) || !tx || !ty || !tz)
      throw ArgError{MLG_ERR_ARG, "bad tile query"};
    TileDesc t = tile_desc(dim, index);
    *tx = t.tx;
    *ty = t.ty;
    *tz = t.tz;
    return 0;
  });
}

int64_t guess_net_param_count(const guess_net_cfg* cfg) {
  int64_t out = -1;
  guarded([&] {
    out = net_param_count(cfg);
    return 0;
  });
  return out;
}

int64_t guess_net_param_offset(const guess_net_cfg* cfg, int32_t index) {
  int64_t out = -1;
  guarded([&] {
    out = net_param_offset(cfg, index);
    return 0;
  });
  return out;
}

size_t guess_net_param_bytes(const guess_net_cfg* cfg) {
  size_t out = 0;
  guarded([&] {
    out = net_param_bytes(cfg);
    return 0;
  });
  return out;
}

size_t guess_net_workspace_bytes(const guess_net_cfg* cfg, const mlg_grid* grid, int32_t batch,
                                 int32_t train) {
  size_t out = 0;
  guarded([&] {
    out = net_workspace_bytes(cfg, grid, batch, train);
    return 0;
  });
  return out;
}

int guess_net_init(const guess_net_cfg* cfg, void* params, void* stream) {
  return guarded([&] { return net_init(cfg, params, (hipStream_t)stream); });
}

int guess_net_refresh(const guess_net_cfg* cfg, void* params, void* stream) {
  return guarded([&] { return net_refresh(cfg, params, (hipStream_t)stream); });
}

int guess_net_infer(const guess_net_cfg* cfg, const void* params, const mlg_grid* grid,
                    int32_t batch, const double* f, const double* u_prev, double* guess, void* ws,
                    size_t ws_bytes, void* stream) {
  return guarded([&] {
    return net_infer(cfg, params, grid, batch, f, u_prev, guess, ws, ws_bytes, (hipStream_t)stream);
  });
}

int guess_net_train_step(const guess_net_cfg* cfg, void* params, const mlg_grid* grid,
                         int32_t batch, const double* const* f, const double* const* u_prev,
                         const double* const* u_target, void* ws, size_t ws_bytes, float* loss,
                         void* stream) {
  return guarded([&] {
    return net_train_step(cfg, params, grid, batch, f, u_prev, u_target, ws, ws_bytes, loss,
                          (hipStream_t)stream);
  });
}

int64_t fluid_net_param_count(const fluid_net_cfg* cfg) {
  int64_t out = -1;
  guarded([&] {
    out = fluid_param_count(cfg);
    return 0;
  });
  return out;
}

int64_t fluid_net_param_offset(const fluid_net_cfg* cfg, int32_t index) {
  int64_t out = -1;
  guarded([&] {
    out = fluid_param_offset(cfg, index);
    return 0;
  });
  return out;
}

size_t fluid_net_param_bytes(const fluid_net_cfg* cfg) {
  size_t out = 0;
  guarded([&] {
    out = fluid_param_bytes(cfg);
    return 0;
  });
  return out;
}

size_t fluid_net_workspace_bytes(const fluid_net_cfg* cfg, const mlg_grid* grid, int32_t batch,
                                 int32_t train) {
  size_t out = 0;
  guarded([&] {
    out = fluid_workspace_bytes(cfg, grid, batch, train);
    return 0;
  });
  return out;
}

int fluid_net_init(const fluid_net_cfg* cfg, void* params, void* stream) {
  return guarded([&] { return fluid_init(cfg, params, (hipStream_t)stream); });
}

int fluid_net_refresh(const fluid_net_cfg* cfg, void* params, void* stream) {
  return guarded([&] { return fluid_refresh(cfg, params, (hipStream_t)stream); });
}

int fluid_net_infer(const fluid_net_cfg* cfg, const void* params, int32_t blocks,
                    const mlg_grid* grid, int32_t batch, const double* f, const double* u_prev,
                    double* guess, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    return fluid_infer(cfg, params, blocks, grid, batch, f, u_prev, guess, ws, ws_bytes,
                       (hipStream_t)stream);
  });
}

int fluid_net_train_step(const fluid_net_cfg* cfg, void* params, int32_t blocks,
                         const mlg_grid* grid, int32_t batch, const double* const* f,
                         const double* const* u_prev, const double* const* u_target, void* ws,
                         size_t ws_bytes, float* loss, void* stream) {
  return guarded([&] {
    return fluid_train_step(cfg, params, blocks, grid, batch, f, u_prev, u_target, ws, ws_bytes,
                            loss, (hipStream_t)stream);
  });
}

size_t linear_guess_param_bytes(const mlg_grid* grid) {
  size_t out = 0;
  guarded([&] {
    out = lin_param_bytes(grid);
    return 0;
  });
  return out;
}

size_t linear_guess_workspace_bytes(const mlg_grid* grid, int32_t batch) {
  size_t out = 0;
  guarded([&] {
    out = lin_workspace_bytes(grid, batch);
    return 0;
  });
  return out;
}

int linear_guess_init(const mlg_grid* grid, void* params, void* stream) {
  return guarded([&] { return lin_init(grid, params, (hipStream_t)stream); });
}

int linear_guess_infer(const mlg_grid* grid, const void* params, int32_t batch, const double* b,
                       double* x0, void* stream) {
  return guarded([&] { return lin_infer(grid, params, batch, b, x0, (hipStream_t)stream); });
}

int linear_guess_train_step(const mlg_grid* grid, void* params, float lr, int32_t batch,
                            const double* const* b, const double* const* x, void* ws,
                            size_t ws_bytes, float* loss, void* stream) {
  return guarded([&] {
    return lin_train_step(grid, params, lr, batch, b, x, ws, ws_bytes, loss, (hipStream_t)stream);
  });
}

}  // extern "C"
