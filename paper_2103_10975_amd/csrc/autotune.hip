// Tile autotuner cache (filled by the tuner; empty means use the heuristic).
#include "engine.h"

namespace mlg {

int autotune_lookup(const mlg_grid&, const mlg_opts&) { return -1; }

}  // namespace mlg
