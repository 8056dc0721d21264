// Batched solver over many independent systems: host-side interface.
#pragma once

#include "common.h"

namespace mlg {

size_t batched_workspace_bytes(int nsys, const mlg_system* sys, const mlg_opts* opts);
int batched_solve(int nsys, const mlg_system* sys, const mlg_opts* opts, void* ws, size_t ws_bytes,
                  mlg_stats* stats, hipStream_t stream);
void batched_shutdown();

}  // namespace mlg
