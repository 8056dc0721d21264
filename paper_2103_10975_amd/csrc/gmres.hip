// Host engine of restarted GMRES(m): workspace plan, kernel dispatch over the
// tile table, per-cycle HIP graphs and the host polling loop.
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "engine.h"
#include "gmres_kernels.h"

namespace mlg {

// ------------------------------------------------------------------ tiles
// Tile shapes (points per workgroup; 256 threads each).  2D tiles are 64 or
// 128 points wide so that one wavefront reads a contiguous 512 B (FP64) row
// segment of every basis vector.
static const TileDesc kTiles2[] = {{64, 16, 1}, {64, 8, 1}, {128, 8, 1}, {64, 4, 1}};
static const TileDesc kTiles3[] = {{64, 4, 4}, {32, 8, 4}, {64, 2, 4}};
static constexpr int kNumTiles2 = sizeof(kTiles2) / sizeof(kTiles2[0]);
static constexpr int kNumTiles3 = sizeof(kTiles3) / sizeof(kTiles3[0]);

int tile_count(int dim) { return dim == 3 ? kNumTiles3 : kNumTiles2; }
TileDesc tile_desc(int dim, int idx) { return dim == 3 ? kTiles3[idx] : kTiles2[idx]; }

static int ceil_div(int a, int b) { return (a + b - 1) / b; }

Geo make_geo(const mlg_grid& gr, int tile) {
  TileDesc t = tile_desc(gr.dim, tile);
  Geo g{};
  g.nx = gr.nx;
  g.ny = gr.ny;
  g.nz = gr.dim == 3 ? gr.nz : 1;
  g.tcx = ceil_div(g.nx, t.tx);
  g.tcy = ceil_div(g.ny, t.ty);
  g.tcz = ceil_div(g.nz, t.tz);
  g.ntiles = g.tcx * g.tcy * g.tcz;
  double hx = 1.0 / (g.nx + 1.0), hy = 1.0 / (g.ny + 1.0), hz = 1.0 / (g.nz + 1.0);
  g.cx = 1.0 / (hx * hx);
  g.cy = 1.0 / (hy * hy);
  g.cz = 1.0 / (hz * hz);
  g.n = (long long)g.nx * g.ny * g.nz;
  g.ldv = (long long)align_up((size_t)g.n, 64);
  return g;
}

int max_tiles(const mlg_grid& gr) {
  int best = 0;
  for (int i = 0; i < tile_count(gr.dim); ++i) best = std::max(best, make_geo(gr, i).ntiles);
  return best;
}

void check_grid(const mlg_grid* grid) {
  if (!grid) throw ArgError{MLG_ERR_ARG, "grid is NULL"};
  if (grid->dim != 2 && grid->dim != 3) throw ArgError{MLG_ERR_ARG, "grid.dim must be 2 or 3"};
  if (grid->nx < 1 || grid->ny < 1 || (grid->dim == 3 && grid->nz < 1))
    throw ArgError{MLG_ERR_ARG, "grid sizes must be >= 1"};
  long long n = (long long)grid->nx * grid->ny * (grid->dim == 3 ? grid->nz : 1);
  if (n > (1LL << 31)) throw ArgError{MLG_ERR_ARG, "grid has more than 2^31 points"};
}

void check_opts(const mlg_opts* o, int dim) {
  if (!o) throw ArgError{MLG_ERR_ARG, "opts is NULL"};
  if (o->restart_m < 1 || o->restart_m > kMaxRestart)
    throw ArgError{MLG_ERR_ARG, "restart_m must be in 1..64"};
  if (o->precision != MLG_FP64 && o->precision != MLG_FP32_IR)
    throw ArgError{MLG_ERR_ARG, "precision must be MLG_FP64 or MLG_FP32_IR"};
  if (!(o->rtol >= 0.0)) throw ArgError{MLG_ERR_ARG, "rtol must be >= 0"};
  if (o->max_iters < 0 || o->fixed_iters < 0) throw ArgError{MLG_ERR_ARG, "negative iteration cap"};
  if (o->tile < 0 || o->tile > tile_count(dim)) throw ArgError{MLG_ERR_ARG, "tile index out of range"};
}

Layout plan_layout(const mlg_grid& gr, const mlg_opts& o) {
  Layout L{};
  const size_t n = (size_t)gr.nx * gr.ny * (gr.dim == 3 ? gr.nz : 1);
  const size_t ldv = align_up(n, 64);
  const size_t s = o.precision == MLG_FP64 ? 8 : 4;
  L.off_ctrl = 0;
  L.off_part = align_up(sizeof(Ctrl), 256);
  L.off_r = align_up(L.off_part + (size_t)(kMaxRestart + 2) * max_tiles(gr) * 8, 256);
  L.off_V = align_up(L.off_r + n * 8, 256);
  L.total = align_up(L.off_V + (size_t)(o.restart_m + 1) * ldv * s, 256);
  return L;
}

// ------------------------------------------------------------------ dispatch
template <class T, class TL, int MM>
static void enqueue_cycle(hipStream_t s, const Geo& g, Ctrl* C, double* r, double* part, void* Vv,
                          int m) {
  T* V = (T*)Vv;
  const dim3 grid(g.ntiles), block(kBlock);
  k_start<T, TL><<<grid, block, 0, s>>>(g, C, r, V);
  for (int j = 0; j < m; ++j) {
    k_proj1<T, TL, MM><<<grid, block, 0, s>>>(g, C, V, part, j);
    k_proj2<T, TL, MM><<<grid, block, 0, s>>>(g, C, V, part, j);
    if (j + 1 < m) k_proj3<T, TL><<<grid, block, 0, s>>>(g, C, V, j);
  }
  k_update<T, TL><<<grid, block, 0, s>>>(g, C, V);
  k_residual<TL><<<grid, block, 0, s>>>(g, C, r, part);
}

template <class TL>
static void enqueue_init(hipStream_t s, const Geo& g, Ctrl* C, double* r, double* part) {
  k_init<TL><<<g.ntiles, kBlock, 0, s>>>(g, C, r, part);
  k_zero_if_needed<TL><<<g.ntiles, kBlock, 0, s>>>(g, C);
}

template <class TL>
static void enqueue_apply(hipStream_t s, const Geo& g, const double* u, double* y) {
  k_apply<TL><<<g.ntiles, kBlock, 0, s>>>(g, u, y);
}

using CycleFn = void (*)(hipStream_t, const Geo&, Ctrl*, double*, double*, void*, int);
using InitFn = void (*)(hipStream_t, const Geo&, Ctrl*, double*, double*);
using ApplyFn = void (*)(hipStream_t, const Geo&, const double*, double*);

template <class T, class TL>
static CycleFn pick_mm(int m) {
  if (m <= 16) return &enqueue_cycle<T, TL, 16>;
  if (m <= 32) return &enqueue_cycle<T, TL, 32>;
  if (m <= 40) return &enqueue_cycle<T, TL, 40>;
  return &enqueue_cycle<T, TL, 64>;
}

template <class TL>
struct TileFns {
  static CycleFn cycle(int prec, int m) {
    return prec == MLG_FP64 ? pick_mm<double, TL>(m) : pick_mm<float, TL>(m);
  }
  static InitFn init() { return &enqueue_init<TL>; }
  static ApplyFn apply() { return &enqueue_apply<TL>; }
};

#define MLG_TILE_SWITCH(DIM, IDX, EXPR_TL)                      \
  if (DIM == 2) {                                               \
    switch (IDX) {                                              \
      case 0: { using TL = TileT<2, 64, 16, 1>; EXPR_TL; }      \
      case 1: { using TL = TileT<2, 64, 8, 1>; EXPR_TL; }       \
      case 2: { using TL = TileT<2, 128, 8, 1>; EXPR_TL; }      \
      default: { using TL = TileT<2, 64, 4, 1>; EXPR_TL; }      \
    }                                                           \
  } else {                                                      \
    switch (IDX) {                                              \
      case 0: { using TL = TileT<3, 64, 4, 4>; EXPR_TL; }       \
      case 1: { using TL = TileT<3, 32, 8, 4>; EXPR_TL; }       \
      default: { using TL = TileT<3, 64, 2, 4>; EXPR_TL; }      \
    }                                                           \
  }

static CycleFn cycle_fn(int dim, int tile, int prec, int m) {
  MLG_TILE_SWITCH(dim, tile, return TileFns<TL>::cycle(prec, m));
}
static InitFn init_fn(int dim, int tile) { MLG_TILE_SWITCH(dim, tile, return TileFns<TL>::init()); }
static ApplyFn apply_fn(int dim, int tile) { MLG_TILE_SWITCH(dim, tile, return TileFns<TL>::apply()); }

// Default tile when the caller leaves the choice to the library: the widest
// tile that still yields >= 2 workgroups per CU (or the smallest tile).
int default_tile(const mlg_grid& gr, const mlg_opts& o) {
  int pick = autotune_lookup(gr, o);
  if (pick >= 0) return pick;
  if (gr.dim == 3) return 0;
  if (make_geo(gr, 0).ntiles >= 512) return 0;
  if (make_geo(gr, 1).ntiles >= 256) return 1;
  return 3;
}

// ------------------------------------------------------------------ caches
struct GraphKey {
  int dev;
  const void* ws;
  int dim, nx, ny, nz, m, prec, tile;
  bool operator<(const GraphKey& o) const {
    return std::tie(dev, ws, dim, nx, ny, nz, m, prec, tile) <
           std::tie(o.dev, o.ws, o.dim, o.nx, o.ny, o.nz, o.m, o.prec, o.tile);
  }
};

struct Runtime {
  std::mutex mu;
  std::map<GraphKey, std::pair<hipGraphExec_t, unsigned long long>> graphs;
  unsigned long long tick = 0;
  std::map<int, hipStream_t> capture_streams;
  std::vector<Summary*> pinned_free;
  std::vector<Summary*> pinned_all;
};

static Runtime& rt() {
  static Runtime* r = new Runtime();
  return *r;
}

static hipStream_t capture_stream(int dev) {
  auto& R = rt();
  auto it = R.capture_streams.find(dev);
  if (it != R.capture_streams.end()) return it->second;
  hipStream_t s;
  MLG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  R.capture_streams[dev] = s;
  return s;
}

// Captured graph of one restart cycle for this workspace and shape.
static hipGraphExec_t cycle_graph(const GraphKey& key, const Geo& g, Ctrl* C, double* r,
                                  double* part, void* V) {
  auto& R = rt();
  std::lock_guard<std::mutex> lk(R.mu);
  auto it = R.graphs.find(key);
  if (it != R.graphs.end()) {
    it->second.second = ++R.tick;
    return it->second.first;
  }
  if (R.graphs.size() >= 32) {                      // evict the least recently used
    auto victim = R.graphs.begin();
    for (auto i = R.graphs.begin(); i != R.graphs.end(); ++i)
      if (i->second.second < victim->second.second) victim = i;
    hipGraphExecDestroy(victim->second.first);
    R.graphs.erase(victim);
  }
  hipStream_t cs = capture_stream(key.dev);
  hipGraph_t graph;
  MLG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  cycle_fn(key.dim, key.tile, key.prec, key.m)(cs, g, C, r, part, V, key.m);
  MLG_HIP(hipStreamEndCapture(cs, &graph));
  hipGraphExec_t exec;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  MLG_HIP(e);
  R.graphs[key] = {exec, ++R.tick};
  return exec;
}

struct PinnedPair {
  Summary* p = nullptr;
  PinnedPair() {
    auto& R = rt();
    std::lock_guard<std::mutex> lk(R.mu);
    if (!R.pinned_free.empty()) {
      p = R.pinned_free.back();
      R.pinned_free.pop_back();
    } else {
      MLG_HIP(hipHostMalloc((void**)&p, 2 * sizeof(Summary), hipHostMallocDefault));
      R.pinned_all.push_back(p);
    }
  }
  ~PinnedPair() {
    auto& R = rt();
    std::lock_guard<std::mutex> lk(R.mu);
    R.pinned_free.push_back(p);
  }
};

void runtime_shutdown() {
  auto& R = rt();
  std::lock_guard<std::mutex> lk(R.mu);
  for (auto& kv : R.graphs) hipGraphExecDestroy(kv.second.first);
  R.graphs.clear();
  for (auto& kv : R.capture_streams) hipStreamDestroy(kv.second);
  R.capture_streams.clear();
  for (auto* p : R.pinned_all) hipHostFree(p);
  R.pinned_all.clear();
  R.pinned_free.clear();
}

// ------------------------------------------------------------------ solve
static void fill_stats(mlg_stats* st, const Summary& s, double secs) {
  if (!st) return;
  st->status = s.status;
  st->cycles = s.cycles;
  st->iters = s.iters;
  st->relres_init = s.relres_init;
  st->relres_first_cycle = s.relres_first;
  st->relres_est = s.relres_est;
  st->relres_true = s.relres_true;
  st->seconds = secs;
}

int solve(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts, void* ws,
          size_t ws_bytes, mlg_stats* stats, hipStream_t stream) {
  auto t0 = std::chrono::steady_clock::now();
  check_grid(grid);
  check_opts(opts, grid->dim);
  if (!b || !x) throw ArgError{MLG_ERR_ARG, "b and x must be device pointers"};
  if (!ws) throw ArgError{MLG_ERR_WORKSPACE, "workspace is NULL"};
  if ((uintptr_t)ws % 256 != 0) throw ArgError{MLG_ERR_ARG, "workspace must be 256-byte aligned"};
  const Layout L = plan_layout(*grid, *opts);
  if (ws_bytes < L.total)
    throw ArgError{MLG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(L.total) +
                                          " bytes, got " + std::to_string(ws_bytes)};
  const int tile = opts->tile > 0 ? opts->tile - 1 : default_tile(*grid, *opts);
  const Geo g = make_geo(*grid, tile);
  char* base = (char*)ws;
  Ctrl* C = (Ctrl*)(base + L.off_ctrl);
  double* part = (double*)(base + L.off_part);
  double* r = (double*)(base + L.off_r);
  void* V = base + L.off_V;
  const int m = opts->restart_m;
  const long long limit = opts->fixed_iters > 0 ? opts->fixed_iters
                          : (opts->max_iters > 0 ? opts->max_iters : 1000000000LL);
  int dev = 0;
  MLG_HIP(hipGetDevice(&dev));

  PinnedPair pin;
  Summary* host = pin.p;
  hipEvent_t ev[2];
  MLG_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  MLG_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { hipEventDestroy(e[0]); hipEventDestroy(e[1]); }
  } evg{ev};

  k_reset<<<1, 64, 0, stream>>>(C, b, x, m, opts->fixed_iters > 0 ? 1 : 0, limit, opts->rtol);
  init_fn(grid->dim, tile)(stream, g, C, r, part);
  MLG_HIP(hipGetLastError());
  MLG_HIP(hipMemcpyAsync(&host[0], &C->s, sizeof(Summary), hipMemcpyDeviceToHost, stream));
  MLG_HIP(hipStreamSynchronize(stream));
  Summary fin = host[0];
  if (!fin.finished) {
    GraphKey key{dev, ws, grid->dim, grid->nx, grid->ny, grid->dim == 3 ? grid->nz : 1, m,
                 opts->precision, tile};
    hipGraphExec_t exec = cycle_graph(key, g, C, r, part, V);
    const int poll = opts->poll_cycles > 0 ? opts->poll_cycles : 1;
    // Every cycle takes >= 1 Arnoldi step until the device marks the solve
    // finished, so this many cycles always suffice; the cap only guards the host.
    const long long max_groups = limit / poll + 4;
    int slot = 0, pending = -1;
    long long last_iters = -1;
    for (long long grp = 0; grp < max_groups; ++grp) {
      for (int c = 0; c < poll; ++c) MLG_HIP(hipGraphLaunch(exec, stream));
      MLG_HIP(hipMemcpyAsync(&host[slot], &C->s, sizeof(Summary), hipMemcpyDeviceToHost, stream));
      MLG_HIP(hipEventRecord(ev[slot], stream));
      if (pending >= 0) {
        MLG_HIP(hipEventSynchronize(ev[pending]));
        if (host[pending].finished) break;
        // every unfinished cycle takes at least one Arnoldi step
        if (host[pending].iters <= last_iters)
          throw HipError{hipErrorUnknown, "solver made no progress in a restart cycle"};
        last_iters = host[pending].iters;
      }
      pending = slot;
      slot ^= 1;
    }
    // final state (the device state is frozen once finished)
    MLG_HIP(hipMemcpyAsync(&host[0], &C->s, sizeof(Summary), hipMemcpyDeviceToHost, stream));
    MLG_HIP(hipStreamSynchronize(stream));
    fin = host[0];
    if (!fin.finished) throw HipError{hipErrorUnknown, "solver did not report completion"};
  }
  double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_stats(stats, fin, secs);
  return fin.status;
}

// ------------------------------------------------------------------ kernel timing
template <class T, class TL, int MM>
static void enqueue_one(hipStream_t s, const Geo& g, Ctrl* C, double* r, double* part, void* Vv,
                        int kind, int j) {
  T* V = (T*)Vv;
  const dim3 grid(g.ntiles), block(kBlock);
  switch (kind) {
    case MLG_K_PROJ1: k_proj1<T, TL, MM><<<grid, block, 0, s>>>(g, C, V, part, j); break;
    case MLG_K_PROJ2: k_proj2<T, TL, MM><<<grid, block, 0, s>>>(g, C, V, part, j); break;
    case MLG_K_PROJ3: k_proj3<T, TL><<<grid, block, 0, s>>>(g, C, V, j); break;
    case MLG_K_UPDATE: k_update<T, TL><<<grid, block, 0, s>>>(g, C, V); break;
    default: k_residual<TL><<<grid, block, 0, s>>>(g, C, r, part); break;
  }
}

using OneFn = void (*)(hipStream_t, const Geo&, Ctrl*, double*, double*, void*, int, int);

template <class T, class TL>
static OneFn pick_one_mm(int m) {
  if (m <= 16) return &enqueue_one<T, TL, 16>;
  if (m <= 32) return &enqueue_one<T, TL, 32>;
  if (m <= 40) return &enqueue_one<T, TL, 40>;
  return &enqueue_one<T, TL, 64>;
}

template <class TL>
static OneFn pick_one(int prec, int m) {
  return prec == MLG_FP64 ? pick_one_mm<double, TL>(m) : pick_one_mm<float, TL>(m);
}

static OneFn one_fn(int dim, int tile, int prec, int m) {
  MLG_TILE_SWITCH(dim, tile, return pick_one<TL>(prec, m));
}

double kernel_bench(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes,
                    void* scratch, size_t scratch_bytes, int kind, int j, int reps,
                    hipStream_t stream) {
  check_grid(grid);
  check_opts(opts, grid->dim);
  if (kind < MLG_K_PROJ1 || kind > MLG_K_RESIDUAL) throw ArgError{MLG_ERR_ARG, "unknown kernel kind"};
  if (j < 0 || j >= opts->restart_m || (kind == MLG_K_PROJ3 && j + 1 >= opts->restart_m))
    throw ArgError{MLG_ERR_ARG, "step index out of range"};
  if (reps < 1 || reps > 4096) throw ArgError{MLG_ERR_ARG, "reps must be in 1..4096"};
  const Layout L = plan_layout(*grid, *opts);
  if (!ws || ws_bytes < L.total) throw ArgError{MLG_ERR_WORKSPACE, "workspace too small"};
  if (!scratch || scratch_bytes < (size_t)reps * sizeof(Ctrl) || (uintptr_t)scratch % 256)
    throw ArgError{MLG_ERR_WORKSPACE, "scratch must hold reps control blocks (mlg_kernel_bench_scratch_bytes)"};
  const int tile = opts->tile > 0 ? opts->tile - 1 : default_tile(*grid, *opts);
  const Geo g = make_geo(*grid, tile);
  char* base = (char*)ws;
  Ctrl* C = (Ctrl*)(base + L.off_ctrl);
  Ctrl* copies = (Ctrl*)scratch;
  k_bench_setup<<<reps, 256, 0, stream>>>(C, copies, reps);
  MLG_HIP(hipGetLastError());
  OneFn fn = one_fn(grid->dim, tile, opts->precision, opts->restart_m);
  hipEvent_t e0, e1;
  MLG_HIP(hipEventCreate(&e0));
  MLG_HIP(hipEventCreate(&e1));
  struct G {
    hipEvent_t a, b;
    ~G() { hipEventDestroy(a); hipEventDestroy(b); }
  } guard{e0, e1};
  // one untimed launch, then the timed ones
  fn(stream, g, copies, (double*)(base + L.off_r), (double*)(base + L.off_part), base + L.off_V,
     kind, j);
  k_bench_setup<<<reps, 256, 0, stream>>>(C, copies, reps);
  MLG_HIP(hipEventRecord(e0, stream));
  for (int i = 0; i < reps; ++i)
    fn(stream, g, copies + i, (double*)(base + L.off_r), (double*)(base + L.off_part),
       base + L.off_V, kind, j);
  MLG_HIP(hipEventRecord(e1, stream));
  MLG_HIP(hipGetLastError());
  MLG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  MLG_HIP(hipEventElapsedTime(&ms, e0, e1));
  return 1000.0 * ms / reps;
}

size_t kernel_bench_scratch_bytes(int reps) { return (size_t)reps * sizeof(Ctrl) + 256; }

int apply_operator(const mlg_grid* grid, const double* u, double* y, hipStream_t stream) {
  check_grid(grid);
  if (!u || !y) throw ArgError{MLG_ERR_ARG, "u and y must be device pointers"};
  const int tile = grid->dim == 3 ? 0 : 1;
  const Geo g = make_geo(*grid, tile);
  apply_fn(grid->dim, tile)(stream, g, u, y);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

}  // namespace mlg
