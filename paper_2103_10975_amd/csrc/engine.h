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

// Tuned choices for one (grid, precision, restart length): the fastest tile
// and, for every tile, the steps that run fused (bit j) and those of them
// whose sums run in the split form.
constexpr int kMaxTiles = 8;
struct TuneEntry {
  int tile;
  unsigned long long fused[kMaxTiles];    // bit j: step j runs as the fused sweep
  unsigned long long split[kMaxTiles];    // bit j: ... with sums(j), coefficients in the sweep
  bool direct;                            // restart cycles launched directly, not as graph replays
};
bool autotune_find(const mlg_grid& g, const mlg_opts& o, TuneEntry* e);
void autotune_store(const mlg_grid& g, const mlg_opts& o, const TuneEntry& e);
void autotune_clear();
size_t autotune_workspace_bytes(const mlg_grid* grid, const mlg_opts* opts);
int autotune(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes, int* tile,
             unsigned long long* fused, unsigned long long* split, int* launch,
             hipStream_t stream);

size_t solve_workspace_bytes(const mlg_grid* grid, const mlg_opts* opts);
int solve(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts, void* ws,
          size_t ws_bytes, mlg_stats* stats, hipStream_t stream);
int apply_operator(const mlg_grid* grid, const double* u, double* y, hipStream_t stream);

// solve() with its workspace in a static per-device array of this many bytes.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
int solve_static(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts,
                 mlg_stats* stats, hipStream_t stream);

double kernel_bench(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes,
                    void* scratch, size_t scratch_bytes, int kind, int j, int reps,
                    hipStream_t stream);
size_t kernel_bench_scratch_bytes(int reps);

void runtime_shutdown();

}  // namespace mlg
