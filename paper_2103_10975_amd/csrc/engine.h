// Host-side interfaces shared by the library's translation units.
#pragma once

#include "common.h"

namespace mlg {

struct TileDesc {
  int tx, ty, tz;
};

int tile_count(int dim);
TileDesc tile_desc(int dim, int idx);
void check_grid(const mlg_grid* grid);
void check_opts(const mlg_opts* o, int dim);
int default_tile(const mlg_grid& gr, const mlg_opts& o);

// tuned tile index for (grid, opts), or -1 when the tuner has no entry
int autotune_lookup(const mlg_grid& gr, const mlg_opts& o);

size_t solve_workspace_bytes(const mlg_grid* grid, const mlg_opts* opts);
int solve(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts, void* ws,
          size_t ws_bytes, mlg_stats* stats, hipStream_t stream);
int apply_operator(const mlg_grid* grid, const double* u, double* y, hipStream_t stream);

double kernel_bench(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes,
                    void* scratch, size_t scratch_bytes, int kind, int j, int reps,
                    hipStream_t stream);
size_t kernel_bench_scratch_bytes(int reps);

void runtime_shutdown();

}  // namespace mlg
