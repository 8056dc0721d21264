// Process-wide table of tuned tile shapes and step schedules.
#include <map>
#include <mutex>
#include <tuple>

#include "engine.h"

namespace mlg {

namespace {
using Key = std::tuple<int, int, int, int, int, int>;   // dim, nx, ny, nz, precision, m
Key key_of(const mlg_grid& g, const mlg_opts& o) {
  return Key{g.dim, g.nx, g.ny, g.dim == 3 ? g.nz : 1, o.precision, o.restart_m};
}
std::mutex& mu() {
  static std::mutex m;
  return m;
}
std::map<Key, TuneEntry>& table() {
  static std::map<Key, TuneEntry> t;
  return t;
}
}  // namespace

bool autotune_find(const mlg_grid& g, const mlg_opts& o, TuneEntry* e) {
  std::lock_guard<std::mutex> lk(mu());
  auto it = table().find(key_of(g, o));
  if (it == table().end()) return false;
  *e = it->second;
  return true;
}

void autotune_store(const mlg_grid& g, const mlg_opts& o, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(mu());
  table()[key_of(g, o)] = e;
}

void autotune_clear() {
  std::lock_guard<std::mutex> lk(mu());
  table().clear();
}

}  // namespace mlg
