// Batched solves (sequential placeholder over gmres_solve until the
// multi-system engine lands).
#include "batched.h"
#include "engine.h"

namespace mlg {

size_t batched_workspace_bytes(int nsys, const mlg_system* sys, const mlg_opts* opts) {
  if (nsys < 1 || !sys) throw ArgError{MLG_ERR_ARG, "need at least one system"};
  size_t best = 0;
  for (int i = 0; i < nsys; ++i) {
    check_grid(&sys[i].grid);
    check_opts(opts, sys[i].grid.dim);
    best = std::max(best, plan_layout(sys[i].grid, *opts).total);
  }
  return best;
}

int batched_solve(int nsys, const mlg_system* sys, const mlg_opts* opts, void* ws, size_t ws_bytes,
                  mlg_stats* stats, hipStream_t stream) {
  batched_workspace_bytes(nsys, sys, opts);
  int worst = MLG_OK, idx = 0;
  for (int i = 0; i < nsys; ++i) {
    const mlg_grid& g = sys[i].grid;
    const size_t n = (size_t)g.nx * g.ny * (g.dim == 3 ? g.nz : 1);
    for (int t = 0; t < sys[i].nrhs; ++t, ++idx) {
      double* x = sys[i].x + t * n;
      if (t > 0) {
        if (sys[i].guess == 1)
          MLG_HIP(hipMemcpyAsync(x, x - n, n * 8, hipMemcpyDeviceToDevice, stream));
        else
          MLG_HIP(hipMemsetAsync(x, 0, n * 8, stream));
      }
      int rc = solve(&g, sys[i].b + t * n, x, opts, ws, ws_bytes, stats ? &stats[idx] : nullptr,
                     stream);
      if (rc < 0) return rc;
      if (rc > worst) worst = rc;
    }
  }
  return worst;
}

void batched_shutdown() {}

}  // namespace mlg
