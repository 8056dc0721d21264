// Host engine of restarted GMRES(m) for one or many systems: workspace plan,
// job tables, kernel dispatch over the tile table, HIP graphs of restart
// cycles (or parts of them) and the host polling loop.  gmres_solve is the
// batched engine with one system and one right-hand side.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "batched.h"
#include "engine.h"
#include "dispatch.h"

namespace mlg {

// ------------------------------------------------------------------ tiles
template <int DIM, int IDX>
constexpr TileDesc tile_of() {
  using TL = typename TileOf<DIM, IDX>::type;
  return TileDesc{TL::TX, TL::TY, TL::TZ};
}
static const TileDesc kTiles2[kNumTiles2] = {tile_of<2, 0>(), tile_of<2, 1>(), tile_of<2, 2>(),
                                             tile_of<2, 3>(), tile_of<2, 4>()};
static const TileDesc kTiles3[kNumTiles3] = {tile_of<3, 0>(), tile_of<3, 1>(), tile_of<3, 2>(),
                                             tile_of<3, 3>(), tile_of<3, 4>()};

int tile_count(int dim) { return dim == 3 ? kNumTiles3 : kNumTiles2; }
TileDesc tile_desc(int dim, int idx) { return dim == 3 ? kTiles3[idx] : kTiles2[idx]; }

static int ceil_div(int a, int b) { return (a + b - 1) / b; }
static size_t npoints(const mlg_grid& g) {
  return (size_t)g.nx * g.ny * (g.dim == 3 ? g.nz : 1);
}

static Geo make_geo(const mlg_grid& gr, int tile, int nblk) {
  TileDesc t = tile_desc(gr.dim, tile);
  Geo g{};
  g.nx = gr.nx;
  g.ny = gr.ny;
  g.nz = gr.dim == 3 ? gr.nz : 1;
  g.tcx = ceil_div(g.nx, t.tx);
  g.tcy = ceil_div(g.ny, t.ty);
  g.tcz = ceil_div(g.nz, t.tz);
  g.ntiles = g.tcx * g.tcy * g.tcz;
  g.nblk = std::max(1, std::min({nblk, g.ntiles, kMaxGrid}));
  double hx = 1.0 / (g.nx + 1.0), hy = 1.0 / (g.ny + 1.0), hz = 1.0 / (g.nz + 1.0);
  g.cx = 1.0 / (hx * hx);
  g.cy = 1.0 / (hy * hy);
  g.cz = 1.0 / (hz * hz);
  g.n = (long long)g.nx * g.ny * g.nz;
  g.ldv = (long long)align_up((size_t)g.n, 64);
  return g;
}

static int tiles_of(const mlg_grid& gr, int tile) { return make_geo(gr, tile, 1).ntiles; }

void check_grid(const mlg_grid* grid) {
  if (!grid) throw ArgError{MLG_ERR_ARG, "grid is NULL"};
  if (grid->dim != 2 && grid->dim != 3) throw ArgError{MLG_ERR_ARG, "grid.dim must be 2 or 3"};
  if (grid->nx < 1 || grid->ny < 1 || (grid->dim == 3 && grid->nz < 1))
    throw ArgError{MLG_ERR_ARG, "grid sizes must be >= 1"};
  long long n = (long long)grid->nx * grid->ny * (grid->dim == 3 ? grid->nz : 1);
  // the sweeps address a field with 32-bit byte offsets (8-byte elements)
  if (n > (1LL << 29)) throw ArgError{MLG_ERR_ARG, "grid has more than 2^29 points"};
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
  if (o->schedule < 0 || o->schedule > 3) throw ArgError{MLG_ERR_ARG, "schedule must be in 0..3"};
  if (o->launch < 0 || o->launch > 2) throw ArgError{MLG_ERR_ARG, "launch must be in 0..2"};
}

// Default tile when the caller leaves the choice to the library and the
// autotuner has no entry: the widest tile that still yields >= 2 workgroups
// per CU (or the smallest tile).
int default_tile(const mlg_grid& gr, const mlg_opts&) {
  if (gr.dim == 3) return 0;
  if (tiles_of(gr, 0) >= 512) return 0;
  if (tiles_of(gr, 1) >= 256) return 1;
  return 3;
}

// ------------------------------------------------------------------ plan
struct Group {
  int dim, tile;
  unsigned long long fused;         // bit j: step j runs as the fused sweep
  unsigned long long split;         // bit j: ... in the split form (sums + sweep)
  int maxblk;                       // most workgroups of one of its systems
  std::vector<int> systems;
  std::vector<Job> jobs;
  size_t off_jobs, off_list;        // device job table, device list of its systems
};

struct Plan {
  int nsys;
  size_t s;                         // basis element size
  std::vector<Geo> geo;
  std::vector<size_t> off_ctrl, off_part, off_r, off_V;
  std::vector<Group> groups;
  size_t off_hdr, off_stats, off_desc, off_init, off_plan_end, total;
  int total_rhs;
  bool direct;                      // launch cycles directly (tuned), else replay a graph
};

struct SysInit {                    // per-call fields of a system's control block
  const double* b0;
  double* x0;
  int nrhs, guess;
  Summary* stats;
  int m, fixed;                     // restart length; 1 = run exactly `limit` steps
  long long limit;                  // step cap
  double rtol;
};

static Plan make_plan(int nsys, const mlg_system* sys, const mlg_opts& o) {
  Plan P{};
  P.nsys = nsys;
  P.s = o.precision == MLG_FP64 ? 8 : 4;
  P.total_rhs = 0;
  for (int i = 0; i < nsys; ++i) P.total_rhs += sys[i].nrhs;
  int ngroups = 0, ndirect = 0;
  // one group per dimension (all systems of a group share the tile shape)
  for (int dim = 2; dim <= 3; ++dim) {
    Group G{};
    G.dim = dim;
    int biggest = -1;
    for (int i = 0; i < nsys; ++i)
      if (sys[i].grid.dim == dim) {
        G.systems.push_back(i);
        if (biggest < 0 || npoints(sys[i].grid) > npoints(sys[biggest].grid)) biggest = i;
      }
    if (G.systems.empty()) continue;
    TuneEntry te;
    const bool tuned = autotune_find(sys[biggest].grid, o, &te);
    G.tile = o.tile > 0 ? o.tile - 1 : (tuned ? te.tile : default_tile(sys[biggest].grid, o));
    if (G.tile >= tile_count(dim)) G.tile = tile_count(dim) - 1;
    // the fused sweep exists for 2D grids only (in 3D its halo ring would
    // exceed the tile)
    G.fused = G.split = 0;
    if (dim == 2 && o.schedule >= 2) {
      G.fused = ~0ULL;
      G.split = o.schedule == 3 ? ~0ULL : 0;
    } else if (dim == 2 && o.schedule == 0 && tuned) {
      G.fused = te.fused[G.tile];
      G.split = te.split[G.tile] & G.fused;
    }
    ++ngroups;
    ndirect += (tuned && te.direct) ? 1 : 0;
    P.groups.push_back(G);
  }
  // as tuned: direct launches only when every group's entry chose them
  P.direct = o.launch == 2 || (o.launch == 0 && ngroups > 0 && ndirect == ngroups);
  P.geo.resize(nsys);
  for (auto& G : P.groups) {
    long long total_tiles = 0;
    for (int i : G.systems) total_tiles += tiles_of(sys[i].grid, G.tile);
    // one system: up to kMaxGrid workgroups; several systems share a larger
    // launch (each system still has at most kMaxGrid partials per column)
    const long long budget =
        std::min<long long>(total_tiles, G.systems.size() > 1 ? 4 * kMaxGrid : kMaxGrid);
    for (int i : G.systems) {
      const int t = tiles_of(sys[i].grid, G.tile);
      const int nb = (int)std::max<long long>(1, (budget * t + total_tiles - 1) / total_tiles);
      P.geo[i] = make_geo(sys[i].grid, G.tile, nb);
      const Geo& g = P.geo[i];
      G.maxblk = std::max(G.maxblk, g.nblk);
      for (int b = 0; b < g.nblk; ++b) {
        Job J{};
        J.sys = i;
        J.t0 = (int)((long long)b * g.ntiles / g.nblk);
        J.t1 = (int)((long long)(b + 1) * g.ntiles / g.nblk);
        J.lblk = b;
        G.jobs.push_back(J);
      }
    }
  }
  size_t o_ = 0;
  auto take = [&](size_t bytes) {
    size_t r = o_;
    o_ = align_up(o_ + bytes, 256);
    return r;
  };
  P.off_hdr = take(256);
  P.off_stats = take((size_t)P.total_rhs * sizeof(Summary));
  P.off_desc = take((size_t)nsys * sizeof(SysDesc));
  P.off_init = take((size_t)nsys * sizeof(SysInit));
  for (auto& G : P.groups) {
    G.off_jobs = take(G.jobs.size() * sizeof(Job));
    G.off_list = take(G.systems.size() * sizeof(int));
  }
  P.off_plan_end = o_;              // descriptors .. lists: one contiguous upload
  P.off_ctrl.resize(nsys);
  P.off_part.resize(nsys);
  P.off_r.resize(nsys);
  P.off_V.resize(nsys);
  for (int i = 0; i < nsys; ++i) {
    const Geo& g = P.geo[i];
    P.off_ctrl[i] = take(sizeof(Ctrl));
    P.off_part[i] = take((size_t)(2 * kMaxRestart + 2) * g.nblk * 8);
    P.off_r[i] = take((size_t)g.n * 8);
    // m basis vectors v_0..v_{m-1}, then the two directions u_j, u_{j+1};
    // the sweeps address the region with 32-bit byte offsets
    const size_t vbytes = (size_t)(o.restart_m + 2) * g.ldv * P.s;
    if (vbytes >= (1ULL << 32))
      throw ArgError{MLG_ERR_ARG, "a system's Krylov basis would exceed 4 GiB: use a smaller "
                                  "restart length, the FP32 basis or a smaller grid"};
    P.off_V[i] = take(vbytes);
  }
  P.total = o_;
  return P;
}

static void check_systems(int nsys, const mlg_system* sys, const mlg_opts* opts) {
  if (nsys < 1 || !sys) throw ArgError{MLG_ERR_ARG, "need at least one system"};
  if (!opts) throw ArgError{MLG_ERR_ARG, "opts is NULL"};
  for (int i = 0; i < nsys; ++i) {
    check_grid(&sys[i].grid);
    check_opts(opts, sys[i].grid.dim);
    if (sys[i].nrhs < 1) throw ArgError{MLG_ERR_ARG, "every system needs nrhs >= 1"};
    if (sys[i].guess != 0 && sys[i].guess != 1) throw ArgError{MLG_ERR_ARG, "guess must be 0 or 1"};
  }
}

size_t workspace_bytes(int nsys, const mlg_system* sys, const mlg_opts* opts) {
  check_systems(nsys, sys, opts);
  return make_plan(nsys, sys, *opts).total;
}

// ------------------------------------------------------------------ dispatch
// Partial blocks per lane for sums over at most maxblk workgroups.
#define MLG_NB_SWITCH(MAXBLK, EXPR_NB)                              \
  if ((MAXBLK) <= 256) { constexpr int NB = 4; EXPR_NB; }           \
  else if ((MAXBLK) <= 512) { constexpr int NB = 8; EXPR_NB; }      \
  else { constexpr int NB = 16; EXPR_NB; }

// coef(j) / sums(j) for `count` systems (those in `list`, or all when null)
// whose partials come from at most maxblk workgroups.
static void launch_coef(hipStream_t s, int count, const int* list, int maxblk, const SysDesc* sd,
                        int j) {
  MLG_NB_SWITCH(maxblk, (k_coef<NB><<<count, kReduceThreads, 0, s>>>(sd, list, j)));
}
static void launch_sums(hipStream_t s, int count, const int* list, int maxblk, const SysDesc* sd,
                        int j) {
  const dim3 grid((2 * j + 2 + kBlock / 64 - 1) / (kBlock / 64), count);
  MLG_NB_SWITCH(maxblk, (k_sums<NB><<<grid, kBlock, 0, s>>>(sd, list, j)));
}

GroupFn group_fn(int dim, int tile, int prec) {
  const int p = prec == MLG_FP64 ? 0 : 1;
#define MLG_SWEEP_PICK(P, D, T) \
  if (p == P && dim == D && tile == T) return MLG_SWEEP_NAME(P, D, T)();
  MLG_SWEEP_ALL(MLG_SWEEP_PICK)
#undef MLG_SWEEP_PICK
  throw ArgError{MLG_ERR_ARG, "no sweep kernels for this tile"};
}

struct DevPlan {                    // device pointers of a plan inside a workspace
  char* base;
  unsigned int* hdr;
  Summary* stats;
  SysDesc* desc;
  SysInit* init;
  std::vector<const Job*> jobs;
  std::vector<const int*> lists;
};

static DevPlan dev_plan(const Plan& P, void* ws) {
  DevPlan D;
  D.base = (char*)ws;
  D.hdr = (unsigned int*)(D.base + P.off_hdr);
  D.stats = (Summary*)(D.base + P.off_stats);
  D.desc = (SysDesc*)(D.base + P.off_desc);
  D.init = (SysInit*)(D.base + P.off_init);
  for (auto& G : P.groups) {
    D.jobs.push_back((const Job*)(D.base + G.off_jobs));
    D.lists.push_back((const int*)(D.base + G.off_list));
  }
  return D;
}

// Per-call set-up of every control block (pointers, counts, options), and of
// the shared counters.  One workgroup per system.
__global__ void k_setup(const SysInit* init, const SysDesc* sd, unsigned int* hdr) {
  const SysDesc* S = sd + blockIdx.x;
  Ctrl* C = S->C;
  if (threadIdx.x != 0) return;
  const SysInit& I = init[blockIdx.x];
  const int m = I.m, fixed = I.fixed;
  const long long limit = I.limit;
  const double rtol = I.rtol;
  C->s = Summary{MLG_OK, 0, 0, 0.0, 0.0, 0.0, 0.0, 0.0};
  C->phase = PH_INIT;
  C->cycle_end = 0;
  C->tail_done = 0;
  C->k = 0;
  C->m = m;
  C->fixed = fixed;
  C->guess = I.guess;
  C->rhs = 0;
  C->nrhs = I.nrhs;
  C->limit = limit;
  C->rtol = rtol;
  C->b0 = I.b0;
  C->x0 = I.x0;
  C->stats = I.stats;
  C->done = hdr;
  if (blockIdx.x == 0) {
    hdr[0] = 0u;
    hdr[1] = 0u;
    hdr[2] = 0u;
    hdr[3] = 0u;
  }
}

// A part of a restart cycle of every system: with `head`, the cycle's start
// (new right-hand sides, initial residual, first direction); steps j0..j1-1;
// then the end of the cycle (after the final coefficients when j1 = m),
// which the device runs only once the cycle has stopped stepping.  `setup`
// first sets up the control blocks from the uploaded init records (the first
// part of a call).  A whole cycle is part(head, 0, m).  A call with a single
// right-hand side leaves out of the head what cannot act on it: the guess of a
// later right-hand side (`begin`), and after its first cycle the initial
// residual of a new one (`resid0`).
struct CyclePart {
  bool setup, head;
  int j0, j1;
  bool begin = true, resid0 = true;
};

static void enqueue_part(hipStream_t s, const Plan& P, const DevPlan& D, int prec, int m,
                         CyclePart cp) {
  std::vector<GroupFn> fns;
  for (auto& G : P.groups) fns.push_back(group_fn(G.dim, G.tile, prec));
  const size_t ng = P.groups.size();
  auto each = [&](int kind, int j) {
    for (size_t gi = 0; gi < ng; ++gi)
      fns[gi](s, kind, (int)P.groups[gi].jobs.size(), D.jobs[gi], D.desc, j);
  };
  const int ns = P.nsys;
  int maxblk = 1;
  for (auto& G : P.groups) maxblk = std::max(maxblk, G.maxblk);
  if (cp.setup) k_setup<<<ns, 64, 0, s>>>(D.init, D.desc, D.hdr);
  if (cp.head) {
    if (cp.begin) each(G_BEGIN, 0);
    if (cp.resid0) each(G_RESID0, 0);
    k_rsum<true><<<ns, kReduceThreads, 0, s>>>(D.desc);
    each(G_START, 0);
    each(G_DOTS, 0);
  }
  for (int j = cp.j0; j < cp.j1; ++j) {
    // the grid-wide sums of step j: coef(j), or sums(j) for groups whose step
    // runs in the split form (one launch over all systems when every group
    // takes the same form)
    int nsplit = 0;
    for (auto& G : P.groups) nsplit += (int)((G.split >> j) & 1ULL);
    if (nsplit == 0) {
      launch_coef(s, ns, nullptr, maxblk, D.desc, j);
    } else if (nsplit == (int)ng) {
      launch_sums(s, ns, nullptr, maxblk, D.desc, j);
    } else {
      for (size_t gi = 0; gi < ng; ++gi) {
        const Group& G = P.groups[gi];
        const int cnt = (int)G.systems.size();
        if ((G.split >> j) & 1ULL) launch_sums(s, cnt, D.lists[gi], G.maxblk, D.desc, j);
        else launch_coef(s, cnt, D.lists[gi], G.maxblk, D.desc, j);
      }
    }
    for (size_t gi = 0; gi < ng; ++gi) {
      const Group& G = P.groups[gi];
      const int nb = (int)G.jobs.size();
      if ((G.fused >> j) & 1ULL) {
        fns[gi](s, ((G.split >> j) & 1ULL) ? G_SPLIT : G_STEP, nb, D.jobs[gi], D.desc, j);
      } else {
        fns[gi](s, G_EXTEND, nb, D.jobs[gi], D.desc, j);
        fns[gi](s, G_DOTS, nb, D.jobs[gi], D.desc, j + 1);
      }
    }
  }
  if (cp.j1 == m) launch_coef(s, ns, nullptr, maxblk, D.desc, m);
  each(G_UPDATE, m);
  each(G_RESID, 0);
  k_rsum<false><<<ns, kReduceThreads, 0, s>>>(D.desc);
}

static void enqueue_cycle(hipStream_t s, const Plan& P, const DevPlan& D, int prec, int m,
                          bool setup = false) {
  enqueue_part(s, P, D, prec, m, CyclePart{setup, true, 0, m});
}

// ------------------------------------------------------------------ caches
struct Runtime {
  std::mutex mu;
  std::map<std::string, std::pair<hipGraphExec_t, unsigned long long>> graphs;
  // Arnoldi steps each restart cycle of the last single right-hand side
  // solved with a plan (by plan key): where the next solve splits its cycles
  std::map<std::string, std::vector<int>> steps_hist;
  unsigned long long tick = 0;
  std::map<int, hipStream_t> capture_streams;
  std::vector<std::pair<void*, size_t>> pinned_free;
  std::vector<void*> pinned_all;
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

static std::string plan_key(int dev, const void* ws, const Plan& P, int prec, int m) {
  std::string k = std::to_string(dev) + ":" + std::to_string((uintptr_t)ws) + ":" +
                  std::to_string(prec) + ":" + std::to_string(m) + ":" + std::to_string(P.total);
  for (size_t i = 0; i < P.geo.size(); ++i) {
    const Geo& g = P.geo[i];
    k += "|" + std::to_string(g.nx) + "," + std::to_string(g.ny) + "," + std::to_string(g.nz) +
         "," + std::to_string(g.ntiles) + "," + std::to_string(g.nblk);
  }
  for (auto& G : P.groups)
    k += "#" + std::to_string(G.dim) + "," + std::to_string(G.tile) + "," + std::to_string(G.fused) +
         "," + std::to_string(G.split);
  return k;
}

// Captured graph of a cycle part for this workspace and plan.
static hipGraphExec_t part_graph(const std::string& key0, int dev, const Plan& P, const DevPlan& D,
                                 int prec, int m, CyclePart cp) {
  const std::string key = key0 + "/" + std::to_string(cp.setup) + std::to_string(cp.head) +
                          std::to_string(cp.begin) + std::to_string(cp.resid0) + "," +
                          std::to_string(cp.j0) + "," + std::to_string(cp.j1);
  auto& R = rt();
  std::lock_guard<std::mutex> lk(R.mu);
  auto it = R.graphs.find(key);
  if (it != R.graphs.end()) {
    it->second.second = ++R.tick;
    return it->second.first;
  }
  if (R.graphs.size() >= 128) {                     // evict the least recently used
    auto victim = R.graphs.begin();
    for (auto i = R.graphs.begin(); i != R.graphs.end(); ++i)
      if (i->second.second < victim->second.second) victim = i;
    (void)hipGraphExecDestroy(victim->second.first);
    R.graphs.erase(victim);
  }
  hipStream_t cs = capture_stream(dev);
  hipGraph_t graph;
  MLG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  enqueue_part(cs, P, D, prec, m, cp);
  hipError_t ce = hipStreamEndCapture(cs, &graph);
  MLG_HIP(ce);
  hipGraphExec_t exec;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  MLG_HIP(e);
  R.graphs[key] = {exec, ++R.tick};
  return exec;
}

// Pinned host staging buffer of at least `bytes` bytes, returned on scope exit.
struct Pinned {
  void* p = nullptr;
  size_t n = 0;
  explicit Pinned(size_t bytes) {
    auto& R = rt();
    std::lock_guard<std::mutex> lk(R.mu);
    for (size_t i = 0; i < R.pinned_free.size(); ++i)
      if (R.pinned_free[i].second >= bytes) {
        p = R.pinned_free[i].first;
        n = R.pinned_free[i].second;
        R.pinned_free.erase(R.pinned_free.begin() + i);
        return;
      }
    n = std::max<size_t>(align_up(bytes, 4096), 4096);
    MLG_HIP(hipHostMalloc(&p, n, hipHostMallocDefault));
    R.pinned_all.push_back(p);
  }
  ~Pinned() {
    auto& R = rt();
    std::lock_guard<std::mutex> lk(R.mu);
    R.pinned_free.push_back({p, n});
  }
};

void runtime_shutdown() {
  auto& R = rt();
  std::lock_guard<std::mutex> lk(R.mu);
  for (auto& kv : R.graphs) (void)hipGraphExecDestroy(kv.second.first);
  R.graphs.clear();
  R.steps_hist.clear();
  for (auto& kv : R.capture_streams) (void)hipStreamDestroy(kv.second);
  R.capture_streams.clear();
  for (auto* p : R.pinned_all) (void)hipHostFree(p);
  R.pinned_all.clear();
  R.pinned_free.clear();
}

void batched_shutdown() {}

// ------------------------------------------------------------------ solve
// `h`: host staging memory of at least stage_bytes(P) bytes that stays
// untouched until the stream has passed the copies.
static void upload_plan(const Plan& P, const DevPlan& D, int nsys, const mlg_system* sys,
                        const mlg_opts& o, hipStream_t stream, char* h) {
  // host image of the descriptors, init records and job tables, laid out as
  // in the workspace, and one copy of it
  const size_t base = P.off_desc;
  std::memset(h, 0, P.off_plan_end - base);
  auto put = [&](const void* src, size_t bytes, size_t off) { std::memcpy(h + (off - base), src, bytes); };
  const long long limit = o.fixed_iters > 0 ? o.fixed_iters
                          : (o.max_iters > 0 ? o.max_iters : 1000000000LL);
  std::vector<SysDesc> desc(nsys);
  std::vector<SysInit> init(nsys);
  int stat_base = 0;
  for (int i = 0; i < nsys; ++i) {
    desc[i].g = P.geo[i];
    desc[i].C = (Ctrl*)(D.base + P.off_ctrl[i]);
    desc[i].V = D.base + P.off_V[i];
    desc[i].r = (double*)(D.base + P.off_r[i]);
    desc[i].part = (double*)(D.base + P.off_part[i]);
    init[i].b0 = sys[i].b;
    init[i].x0 = sys[i].x;
    init[i].nrhs = sys[i].nrhs;
    init[i].guess = sys[i].guess;
    init[i].stats = D.stats + stat_base;
    init[i].m = o.restart_m;
    init[i].fixed = o.fixed_iters > 0 ? 1 : 0;
    init[i].limit = limit;
    init[i].rtol = o.rtol;
    stat_base += sys[i].nrhs;
  }
  put(desc.data(), desc.size() * sizeof(SysDesc), P.off_desc);
  put(init.data(), init.size() * sizeof(SysInit), P.off_init);
  for (size_t gi = 0; gi < P.groups.size(); ++gi) {
    std::vector<Job> jobs = P.groups[gi].jobs;
    for (Job& J : jobs) {
      J.m = o.restart_m;
      J.g = desc[J.sys].g;
      J.V = desc[J.sys].V;
      J.r = desc[J.sys].r;
      J.part = desc[J.sys].part;
    }
    put(jobs.data(), jobs.size() * sizeof(Job), P.groups[gi].off_jobs);
    put(P.groups[gi].systems.data(), P.groups[gi].systems.size() * sizeof(int),
        P.groups[gi].off_list);
  }
  MLG_HIP(hipMemcpyAsync(D.desc, h, P.off_plan_end - base, hipMemcpyHostToDevice, stream));
}

static size_t stage_bytes(const Plan& P) { return P.off_plan_end - P.off_desc; }

static int report(const Plan& P, const std::vector<Summary>& res, double secs, mlg_stats* stats);

int batched_solve(int nsys, const mlg_system* sys, const mlg_opts* opts, void* ws, size_t ws_bytes,
                  mlg_stats* stats, hipStream_t stream) {
  auto t0 = std::chrono::steady_clock::now();
  check_systems(nsys, sys, opts);
  for (int i = 0; i < nsys; ++i)
    if (!sys[i].b || !sys[i].x) throw ArgError{MLG_ERR_ARG, "b and x must be device pointers"};
  if (!ws) throw ArgError{MLG_ERR_WORKSPACE, "workspace is NULL"};
  if ((uintptr_t)ws % 256 != 0) throw ArgError{MLG_ERR_ARG, "workspace must be 256-byte aligned"};
  const Plan P = make_plan(nsys, sys, *opts);
  if (ws_bytes < P.total)
    throw ArgError{MLG_ERR_WORKSPACE, "workspace too small: need " + std::to_string(P.total) +
                                          " bytes, got " + std::to_string(ws_bytes)};
  const DevPlan D = dev_plan(P, ws);
  int dev = 0;
  MLG_HIP(hipGetDevice(&dev));
  const int m = opts->restart_m;
  const long long limit = opts->fixed_iters > 0 ? opts->fixed_iters
                          : (opts->max_iters > 0 ? opts->max_iters : 1000000000LL);

  Pinned stage(stage_bytes(P));
  upload_plan(P, D, nsys, sys, *opts, stream, (char*)stage.p);
  const std::string key = plan_key(dev, ws, P, opts->precision, m);
  // Each poll copies the header -- and, for up to kStatsInPoll right-hand
  // sides, the statistics behind it in the workspace -- into one of two
  // pinned slots, so that a finished solve needs no further round trip.
  constexpr int kStatsInPoll = 64;
  const bool stats_in_poll = P.total_rhs <= kStatsInPoll;
  const size_t stats_bytes = (size_t)P.total_rhs * sizeof(Summary);
  const size_t poll_bytes = (P.off_stats - P.off_hdr) + (stats_in_poll ? stats_bytes : 0);
  const size_t slot_bytes = align_up(poll_bytes, 256);
  Pinned pin(2 * slot_bytes + stats_bytes);
  auto slot_ptr = [&](int sl) { return (char*)pin.p + sl * slot_bytes; };
  auto slot_hdr = [&](int sl) { return (volatile unsigned int*)slot_ptr(sl); };
  hipEvent_t ev[2];
  MLG_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  MLG_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
  } evg{ev};

  const int poll = opts->poll_cycles > 0 ? opts->poll_cycles : 1;
  // Every cycle completes at least one Arnoldi step or one right-hand side of
  // some unfinished system, so this many cycles always suffice; the cap only
  // guards the host against a solver that stopped making progress.
  long long rhs_total = P.total_rhs;
  const long long max_groups = (limit + 2) * rhs_total / poll + 8;
  int slot = 0, queue[2] = {0, 0}, nq = 0;
  bool first = true;
  // enqueue cycle parts (graph replays, or direct launches), then the poll
  auto launch_parts = [&](const CyclePart* parts, int n) {
    for (int c = 0; c < n; ++c) {
      CyclePart cp = parts[c];
      cp.setup = first;
      first = false;
      if (P.direct) {
        enqueue_part(stream, P, D, opts->precision, m, cp);
        MLG_HIP(hipGetLastError());
      } else {
        MLG_HIP(hipGraphLaunch(part_graph(key, dev, P, D, opts->precision, m, cp), stream));
      }
    }
    MLG_HIP(hipMemcpyAsync(slot_ptr(slot), D.hdr, poll_bytes, hipMemcpyDeviceToHost, stream));
    MLG_HIP(hipEventRecord(ev[slot], stream));
    queue[nq++] = slot;
    slot ^= 1;
  };
  const CyclePart whole{false, true, 0, m};
  std::vector<CyclePart> group(poll, whole);
  auto launch = [&]() { launch_parts(group.data(), poll); };
  int done_slot = -1;
  if (P.total_rhs == 1) {
    // A single right-hand side.  A cycle that the plan's previous solve ended
    // early is split after the steps it took then (plus a margin): the first
    // part ends with the cycle's end, which the device runs only if the cycle
    // stopped within it, and the rest of the cycle is launched only if the
    // header shows that it did not -- so the steps that a stopped cycle would
    // skip are rarely launched at all.  Whole cycles are launched one ahead
    // of the one whose header the host reads, unless that read forecasts
    // (header [2]) that the cycle in flight finishes the right-hand side (the
    // first cycle is read before the next is launched: a good initial guess
    // finishes in one).
    constexpr int kSplitMargin = 2;
    std::vector<int> hist;
    {
      std::lock_guard<std::mutex> lk(rt().mu);
      auto it = rt().steps_hist.find(key);
      if (it != rt().steps_hist.end()) hist = it->second;
    }
    std::vector<int> took;
    unsigned int progress = 0;
    struct Entry {
      int slot, cyc;
      bool first_part;              // the first part of a split cycle
    };
    std::vector<Entry> q;
    long long next = 0;
    auto split_of = [&](long long c) { return c < (long long)hist.size() ? hist[c] + kSplitMargin : m; };
    auto launch_cycle = [&](long long c) {
      const int sp = split_of(c);
      CyclePart part = sp < m ? CyclePart{false, true, 0, sp} : whole;
      part.begin = false;
      part.resid0 = c == 0;
      launch_parts(&part, 1);
      q.push_back(Entry{queue[nq - 1], (int)c, sp < m});
      --nq;                         // this path keeps its own queue
    };
    bool ahead_ok = false;
    launch_cycle(next++);
    while (true) {
      if (q.size() == 1 && !q[0].first_part && ahead_ok && next < max_groups)
        launch_cycle(next++);
      const Entry e = q.front();
      q.erase(q.begin());
      MLG_HIP(hipEventSynchronize(ev[e.slot]));
      volatile unsigned int* host = slot_hdr(e.slot);
      const unsigned int fin = host[0], prog = host[1], fc = host[2], ends = host[3];
      const bool over = fin >= 1u || ends >= (unsigned)(e.cyc + 1);
      if (over) took.push_back((int)(prog - progress));
      if (fin >= 1u) {
        done_slot = e.slot;
        break;
      }
      if (prog == progress)
        throw HipError{hipErrorUnknown, "solver made no progress in a restart cycle"};
      if (over) progress = prog;
      ahead_ok = fin + fc < 1u;
      if (!over) {
        // a split cycle still stepping: its rest (nothing was launched
        // behind its first part)
        const CyclePart rest{false, false, split_of(e.cyc), m};
        launch_parts(&rest, 1);
        q.push_back(Entry{queue[nq - 1], e.cyc, false});
        --nq;
      } else if (q.empty()) {
        if (next >= max_groups) break;
        launch_cycle(next++);
      }
    }
    // a cycle launched ahead runs idle; it must pass before the slots are reused
    if (!q.empty()) MLG_HIP(hipStreamSynchronize(stream));
    if (done_slot >= 0) {
      std::lock_guard<std::mutex> lk(rt().mu);
      auto& H = rt().steps_hist;
      // a bounded table (callers may use a new workspace for every call)
      if (H.size() >= 256 && H.find(key) == H.end()) H.erase(H.begin());
      H[key] = took;
    }
  } else {
    // Groups of `poll` cycles are launched one ahead of the group whose
    // header the host reads, so the device never waits for the host --
    // except when the group read forecasts (header [2]) that the group in
    // flight finishes every system: then the host waits for it before
    // launching more, which saves a whole cycle of no-op kernels at the end
    // of a solve, and costs one host round trip when the forecast was wrong.
    bool forecast = false;
    unsigned int last_progress = 0;
    long long grp = 0, reads = 0;
    launch();
    ++grp;
    while (true) {
      if (!forecast && nq < 2 && grp < max_groups) {
        launch();
        ++grp;
      }
      const int p = queue[0];
      queue[0] = queue[1];
      --nq;
      MLG_HIP(hipEventSynchronize(ev[p]));
      volatile unsigned int* host = slot_hdr(p);
      const unsigned int fin = host[0], prog = host[1], fc = host[2];
      if (fin >= (unsigned)nsys) {
        done_slot = p;
        break;
      }
      if (reads > 0 && prog == last_progress)
        throw HipError{hipErrorUnknown, "solver made no progress in a restart cycle"};
      ++reads;
      last_progress = prog;
      forecast = fin + fc >= (unsigned)nsys;
      if (nq == 0) {
        if (grp >= max_groups) break;
        launch();
        ++grp;
      }
    }
  }
  // a group still in flight (launched ahead) runs idle; it must pass before
  // the pinned slots are reused
  if (nq > 0) MLG_HIP(hipStreamSynchronize(stream));
  if (done_slot < 0) throw HipError{hipErrorUnknown, "solver did not finish"};
  std::vector<Summary> res(P.total_rhs);
  if (stats_in_poll) {
    std::memcpy(res.data(), slot_ptr(done_slot) + (P.off_stats - P.off_hdr), stats_bytes);
  } else {
    char* sp = (char*)pin.p + 2 * slot_bytes;
    MLG_HIP(hipMemcpyAsync(sp, D.stats, stats_bytes, hipMemcpyDeviceToHost, stream));
    MLG_HIP(hipStreamSynchronize(stream));
    std::memcpy(res.data(), sp, stats_bytes);
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return report(P, res, secs, stats);
}

// Status of a finished solve (the most severe over its right-hand sides) and
// the per-RHS statistics.
static int report(const Plan& P, const std::vector<Summary>& res, double secs, mlg_stats* stats) {
  int worst = MLG_OK;
  for (int i = 0; i < P.total_rhs; ++i) {
    const Summary& s = res[i];
    if (s.status < 0 && (worst >= 0 || s.status < worst)) worst = s.status;
    else if (worst >= 0 && s.status > worst) worst = s.status;
    if (stats) {
      stats[i].status = s.status;
      stats[i].cycles = s.cycles;
      stats[i].iters = s.iters;
      stats[i].relres_init = s.relres_init;
      stats[i].relres_first_cycle = s.relres_first;
      stats[i].relres_est = s.relres_est;
      stats[i].relres_true = s.relres_true;
      stats[i].seconds = P.total_rhs == 1 ? secs : 0.0;
      stats[i].relres_iter5 = s.relres5;
    }
  }
  return worst;
}

size_t batched_workspace_bytes(int nsys, const mlg_system* sys, const mlg_opts* opts) {
  return workspace_bytes(nsys, sys, opts);
}

static mlg_system single(const mlg_grid* grid, const double* b, double* x) {
  mlg_system s{};
  s.grid = *grid;
  s.nrhs = 1;
  s.guess = 0;
  s.b = b;
  s.x = x;
  return s;
}

size_t solve_workspace_bytes(const mlg_grid* grid, const mlg_opts* opts) {
  check_grid(grid);
  mlg_system s = single(grid, nullptr, nullptr);
  return workspace_bytes(1, &s, opts);
}

int solve(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts, void* ws,
          size_t ws_bytes, mlg_stats* stats, hipStream_t stream) {
  check_grid(grid);
  if (!b || !x) throw ArgError{MLG_ERR_ARG, "b and x must be device pointers"};
  mlg_system s = single(grid, b, x);
  return batched_solve(1, &s, opts, ws, ws_bytes, stats, stream);
}

// ------------------------------------------------------------------ solve without allocation
// Workspace of solve_static: a file-scope array that every device holds from
// the load of this code object until the process ends.  Host code never
// passes `scratch` itself (on the host it is only a stand-in); it uses the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct StaticScratch {
  std::mutex mu;           // held for a whole call: calls on one device never overlap
  void* ptr = nullptr;     // device address of `scratch` on this device
};

static StaticScratch& static_scratch(int dev) {
  static std::mutex mu;
  static std::map<int, StaticScratch*> per_dev;
  std::lock_guard<std::mutex> lk(mu);
  StaticScratch*& e = per_dev[dev];
  if (!e) e = new StaticScratch();
  return *e;
}

int solve_static(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts,
                 mlg_stats* stats, hipStream_t stream) {
  auto t0 = std::chrono::steady_clock::now();
  check_grid(grid);
  if (!b || !x) throw ArgError{MLG_ERR_ARG, "b and x must be device pointers"};
  mlg_system sys = single(grid, b, x);
  check_systems(1, &sys, opts);
  const Plan P = make_plan(1, &sys, *opts);
  if (P.total > kStaticScratchBytes)
    throw ArgError{MLG_ERR_WORKSPACE,
                   "gmres_solve_static: this grid and restart length need " +
                       std::to_string(P.total) + " bytes of workspace, the static scratch holds " +
                       std::to_string(kStaticScratchBytes) + " (gmres_solve takes a workspace)"};
  int dev = 0;
  MLG_HIP(hipGetDevice(&dev));
  StaticScratch& S = static_scratch(dev);
  std::lock_guard<std::mutex> lk(S.mu);
  if (!S.ptr) MLG_HIP(hipGetSymbolAddress((void**)&S.ptr, HIP_SYMBOL(scratch)));
  const DevPlan D = dev_plan(P, S.ptr);
  // pageable staging: the copies below complete before this call returns
  std::vector<char> stage(stage_bytes(P));
  upload_plan(P, D, 1, &sys, *opts, stream, stage.data());
  const int m = opts->restart_m;
  const int poll = opts->poll_cycles > 0 ? opts->poll_cycles : 1;
  const long long limit = opts->fixed_iters > 0 ? opts->fixed_iters
                          : (opts->max_iters > 0 ? opts->max_iters : 1000000000LL);
  // the same bound on restart cycles as the graph path; cycles are enqueued
  // directly (no graph: instantiating one allocates)
  const long long max_groups = (limit + 2) * P.total_rhs / poll + 8;
  unsigned int hdr[3] = {0u, 0u, 0u};
  unsigned int last_progress = 0;
  bool finished = false;
  for (long long grp = 0; grp < max_groups; ++grp) {
    for (int c = 0; c < poll; ++c) enqueue_cycle(stream, P, D, opts->precision, m, grp == 0 && c == 0);
    MLG_HIP(hipGetLastError());
    MLG_HIP(hipMemcpyAsync(hdr, D.hdr, sizeof(hdr), hipMemcpyDeviceToHost, stream));
    MLG_HIP(hipStreamSynchronize(stream));
    if (hdr[0] >= 1u) {
      finished = true;
      break;
    }
    if (grp > 0 && hdr[1] == last_progress)
      throw HipError{hipErrorUnknown, "solver made no progress in a restart cycle"};
    last_progress = hdr[1];
  }
  if (!finished) throw HipError{hipErrorUnknown, "solver did not finish"};
  std::vector<Summary> res(P.total_rhs);
  MLG_HIP(hipMemcpyAsync(res.data(), D.stats, (size_t)P.total_rhs * sizeof(Summary),
                         hipMemcpyDeviceToHost, stream));
  MLG_HIP(hipStreamSynchronize(stream));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return report(P, res, secs, stats);
}

// ------------------------------------------------------------------ kernel timing
// Replicate a system's state into `n` independent copies for kernel timing:
// each keeps the coefficients of the finished solve but is marked running
// with a zero tolerance, so every timed launch does its full work.
// descs[i] is the system descriptor pointing at copy i.
__global__ void k_bench_setup(const SysDesc* src_desc, SysDesc* descs, Ctrl* copies, int n,
                              int j, int tail) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const unsigned int* s = (const unsigned int*)src_desc->C;
  unsigned int* d = (unsigned int*)(copies + i);
  for (int e = threadIdx.x; e < (int)(sizeof(Ctrl) / 4); e += blockDim.x) d[e] = s[e];
  __syncthreads();
  Ctrl* c = copies + i;
  // column sums of a unit direction orthogonal to the basis (alpha = 1), so a
  // split step at j runs its full sweep
  for (int e = threadIdx.x; e < 2 * kMaxRestart + 2; e += blockDim.x)
    c->sums[e] = e == 2 * j ? 1.0 : 0.0;
  if (threadIdx.x == 0) {
    c->phase = PH_RUN;
    c->rhs = 0;
    // the cycle-end kernels (update, residual) run on a stopped cycle whose
    // end is pending; the step kernels on a running one
    c->cycle_end = tail;
    c->tail_done = 0;
    c->tol_abs = 0.0;
    c->fixed = 1;
    c->limit = 1LL << 62;
    c->k = c->m;
    if (!(c->alpha > 0.0)) c->alpha = 1.0;
    descs[i] = *src_desc;
    descs[i].C = c;
  }
}

// One launch of a solver kernel in the solve's configuration (kind: MLG_K_*;
// j: step index, the restart length for MLG_K_UPDATE).
static void enqueue_one(GroupFn fn, hipStream_t s, int kind, int nb, const Job* jobs,
                        const SysDesc* sd, int j) {
  switch (kind) {
    case MLG_K_DOTS: fn(s, G_DOTS, nb, jobs, sd, j); break;
    case MLG_K_COEF: launch_coef(s, 1, nullptr, nb, sd, j); break;
    case MLG_K_SUMS: launch_sums(s, 1, nullptr, nb, sd, j); break;
    case MLG_K_STEPC: fn(s, G_SPLIT, nb, jobs, sd, j); break;
    case MLG_K_EXTEND: fn(s, G_EXTEND, nb, jobs, sd, j); break;
    case MLG_K_UPDATE: fn(s, G_UPDATE, nb, jobs, sd, j); break;
    case MLG_K_STEP: fn(s, G_STEP, nb, jobs, sd, j); break;
    default: fn(s, G_RESID, nb, jobs, sd, j); break;
  }
}

size_t kernel_bench_scratch_bytes(int reps) {
  return (size_t)reps * (sizeof(Ctrl) + sizeof(SysDesc)) + 512;
}

double kernel_bench(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes,
                    void* scratch, size_t scratch_bytes, int kind, int j, int reps,
                    hipStream_t stream) {
  check_grid(grid);
  check_opts(opts, grid->dim);
  if (kind < MLG_K_DOTS || kind > MLG_K_STEPC) throw ArgError{MLG_ERR_ARG, "unknown kernel kind"};
  if (j < 0 || j > opts->restart_m ||
      ((kind == MLG_K_EXTEND || kind == MLG_K_STEP || kind == MLG_K_STEPC) &&
       j >= opts->restart_m))
    throw ArgError{MLG_ERR_ARG, "step index out of range"};
  if (reps < 1 || reps > 4096) throw ArgError{MLG_ERR_ARG, "reps must be in 1..4096"};
  mlg_system s1 = single(grid, nullptr, nullptr);
  const Plan P = make_plan(1, &s1, *opts);
  if (!ws || ws_bytes < P.total) throw ArgError{MLG_ERR_WORKSPACE, "workspace too small"};
  if (!scratch || scratch_bytes < kernel_bench_scratch_bytes(reps) || (uintptr_t)scratch % 256)
    throw ArgError{MLG_ERR_WORKSPACE,
                   "scratch must hold reps control blocks (mlg_kernel_bench_scratch_bytes)"};
  const DevPlan D = dev_plan(P, ws);
  Ctrl* copies = (Ctrl*)scratch;
  SysDesc* descs = (SysDesc*)align_up((uintptr_t)((char*)scratch + (size_t)reps * sizeof(Ctrl)), 256);
  const Group& G = P.groups[0];
  GroupFn fn = group_fn(G.dim, G.tile, opts->precision);
  const int nb = (int)G.jobs.size();
  hipEvent_t e0, e1;
  MLG_HIP(hipEventCreate(&e0));
  MLG_HIP(hipEventCreate(&e1));
  struct Gd {
    hipEvent_t a, b;
    ~Gd() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } guard{e0, e1};
  const int jj = kind == MLG_K_UPDATE ? opts->restart_m : j;
  const int tail = kind == MLG_K_UPDATE || kind == MLG_K_RESIDUAL ? 1 : 0;
  k_bench_setup<<<reps, 256, 0, stream>>>(D.desc, descs, copies, reps, jj, tail);
  enqueue_one(fn, stream, kind, nb, D.jobs[0], descs, jj);    // untimed warm-up launch
  k_bench_setup<<<reps, 256, 0, stream>>>(D.desc, descs, copies, reps, jj, tail);
  MLG_HIP(hipEventRecord(e0, stream));
  for (int i = 0; i < reps; ++i) enqueue_one(fn, stream, kind, nb, D.jobs[0], descs + i, jj);
  MLG_HIP(hipEventRecord(e1, stream));
  MLG_HIP(hipGetLastError());
  MLG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  MLG_HIP(hipEventElapsedTime(&ms, e0, e1));
  return 1000.0 * ms / reps;
}

// ------------------------------------------------------------------ autotuner
constexpr int kTuneReps = 5;

// Synthetic right-hand side for tuning (a fixed smooth field plus a hashed
// perturbation) and a zero initial guess.
__global__ void k_tune_fill(double* b, double* x, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  unsigned int h = (unsigned int)p * 2654435761u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  b[p] = 1.0 + 0.5 * ((double)(h & 0xffff) / 65536.0 - 0.5);
  x[p] = 0.0;
}

static size_t tune_solve_bytes(const mlg_grid* grid, const mlg_opts* opts) {
  size_t mx = 0;
  for (int t = 0; t < tile_count(grid->dim); ++t) {
    mlg_opts o = *opts;
    o.tile = t + 1;
    mlg_system s1 = single(grid, nullptr, nullptr);
    mx = std::max(mx, make_plan(1, &s1, o).total);
  }
  return align_up(mx, 256);
}

size_t autotune_workspace_bytes(const mlg_grid* grid, const mlg_opts* opts) {
  check_grid(grid);
  check_opts(opts, grid->dim);
  const size_t n = npoints(*grid);
  return tune_solve_bytes(grid, opts) + 2 * align_up(n * 8, 256) +
         align_up(kernel_bench_scratch_bytes(kTuneReps), 256);
}

int autotune(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes, int* tile_out,
             unsigned long long* fused_out, unsigned long long* split_out, int* launch_out,
             hipStream_t stream) {
  check_grid(grid);
  check_opts(opts, grid->dim);
  if (!ws || ws_bytes < autotune_workspace_bytes(grid, opts) || (uintptr_t)ws % 256)
    throw ArgError{MLG_ERR_WORKSPACE, "autotune workspace too small or misaligned"};
  const size_t n = npoints(*grid);
  const size_t solve_bytes = tune_solve_bytes(grid, opts);
  char* base = (char*)ws;
  double* b = (double*)(base + solve_bytes);
  double* x = (double*)(base + solve_bytes + align_up(n * 8, 256));
  char* scratch = base + solve_bytes + 2 * align_up(n * 8, 256);
  const size_t scratch_bytes = align_up(kernel_bench_scratch_bytes(kTuneReps), 256);
  const int m = opts->restart_m;
  const bool two_d = grid->dim == 2;
  // step indices sampled; costs in between are interpolated linearly
  std::vector<int> js;
  for (int q = 0; q <= 4; ++q) js.push_back(std::min(m - 1, q * (m - 1) / 4));
  js.push_back(std::min(1, m - 1));
  std::sort(js.begin(), js.end());
  js.erase(std::unique(js.begin(), js.end()), js.end());
  auto interp = [&](const std::vector<double>& v, int j) {
    size_t i = 0;
    while (i + 1 < js.size() && js[i + 1] < j) ++i;
    if (i + 1 >= js.size() || js[i] >= j) return v[i];
    const double w = double(j - js[i]) / double(js[i + 1] - js[i]);
    return (1.0 - w) * v[i] + w * v[i + 1];
  };
  // stage 1: per tile, the per-step choice between the separate and the
  // fused sweeps, from kernel timings
  TuneEntry te{};
  for (int t = 0; t < tile_count(grid->dim); ++t) {
    mlg_opts o = *opts;
    o.tile = t + 1;
    o.schedule = 1;
    o.launch = 1;
    o.fixed_iters = m;                         // one full cycle fills the basis
    o.max_iters = 0;
    k_tune_fill<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(b, x, (long long)n);
    MLG_HIP(hipGetLastError());
    solve(grid, b, x, &o, ws, solve_bytes, nullptr, stream);
    auto bench = [&](int kind, int j) {
      return kernel_bench(grid, &o, ws, solve_bytes, scratch, scratch_bytes, kind, j, kTuneReps,
                          stream);
    };
    unsigned long long mask = 0;
    if (two_d) {
      std::vector<double> sep, fus;
      for (int j : js) {
        sep.push_back(bench(MLG_K_EXTEND, j) + bench(MLG_K_DOTS, j + 1));
        fus.push_back(bench(MLG_K_STEP, j));
      }
      for (int j = 0; j < m; ++j)
        if (interp(fus, j) < interp(sep, j)) mask |= 1ULL << j;
    }
    te.fused[t] = mask;
    te.split[t] = 0;
  }
  // stage 2: the tile, and for its fused steps the form of their sums (one
  // workgroup's coef launch, or sums spread over workgroups with the
  // coefficients formed in the sweep), whose whole restart cycles (graph
  // launches, every kernel, the host poll) are fastest.  The form is timed
  // whole because its cost is the cross-XCD traffic of freshly written
  // partials, which repeated launches of one kernel do not show.  The default
  // tile is kept unless another is at least 5% faster, so that timing noise
  // does not flip the choice between near-equal tiles.
  const int dflt = default_tile(*grid, *opts);
  const int nt = tile_count(grid->dim);
  std::vector<double> cyc(2 * nt, 1e300);      // [tile][form: 0 coef, 1 split]
  for (int t = 0; t < nt; ++t)
    for (int form = 0; form < (two_d ? 2 : 1); ++form) {
      te.tile = t;
      te.split[t] = form ? te.fused[t] : 0;
      autotune_store(*grid, *opts, te);
      mlg_opts o = *opts;
      o.tile = t + 1;
      o.schedule = 0;                          // the entry just stored
      o.launch = 1;
      o.fixed_iters = 2 * m;
      o.max_iters = 0;
      o.poll_cycles = 2;
      for (int rep = 0; rep < 5; ++rep) {      // the first run also captures the graph
        k_tune_fill<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(b, x, (long long)n);
        MLG_HIP(hipGetLastError());
        MLG_HIP(hipStreamSynchronize(stream));
        const auto t0 = std::chrono::steady_clock::now();
        solve(grid, b, x, &o, ws, solve_bytes, nullptr, stream);
        const auto t1 = std::chrono::steady_clock::now();
        if (rep > 0)
          cyc[2 * t + form] = std::min(cyc[2 * t + form], std::chrono::duration<double>(t1 - t0).count());
      }
    }
  for (int t = 0; t < nt; ++t) te.split[t] = cyc[2 * t + 1] < cyc[2 * t] ? te.fused[t] : 0;
  auto best = [&](int t) { return std::min(cyc[2 * t], cyc[2 * t + 1]); };
  int fastest = 0;
  for (int t = 1; t < nt; ++t)
    if (best(t) < best(fastest)) fastest = t;
  te.tile = best(fastest) < 0.95 * best(dflt) ? fastest : dflt;
  // stage 3: the chosen configuration's restart cycles replayed as captured
  // graphs or launched directly (a graph node starts later after its
  // predecessor than a directly launched kernel does on some sizes, while
  // direct launches cost host time per kernel); direct only when at least
  // 3% faster
  te.direct = false;
  autotune_store(*grid, *opts, te);
  double lm[2] = {1e300, 1e300};
  for (int direct = 0; direct < 2; ++direct) {
    mlg_opts o = *opts;
    o.tile = 0;
    o.schedule = 0;
    o.launch = direct ? 2 : 1;
    o.fixed_iters = 2 * m;
    o.max_iters = 0;
    o.poll_cycles = 1;
    for (int rep = 0; rep < 5; ++rep) {        // the first run also captures the graph
      k_tune_fill<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(b, x, (long long)n);
      MLG_HIP(hipGetLastError());
      MLG_HIP(hipStreamSynchronize(stream));
      const auto t0 = std::chrono::steady_clock::now();
      solve(grid, b, x, &o, ws, solve_bytes, nullptr, stream);
      const auto t1 = std::chrono::steady_clock::now();
      if (rep > 0) lm[direct] = std::min(lm[direct], std::chrono::duration<double>(t1 - t0).count());
    }
  }
  te.direct = lm[1] < 0.97 * lm[0];
  autotune_store(*grid, *opts, te);
  if (tile_out) *tile_out = te.tile + 1;
  if (fused_out) *fused_out = te.fused[te.tile];
  if (split_out) *split_out = te.split[te.tile];
  if (launch_out) *launch_out = te.direct ? 2 : 1;
  return MLG_OK;
}

// ------------------------------------------------------------------ operator
template <class TL>
static void enqueue_apply(hipStream_t s, const Geo& g, const double* u, double* y) {
  k_apply<TL><<<g.nblk, kBlock, 0, s>>>(g, u, y);
}
using ApplyFn = void (*)(hipStream_t, const Geo&, const double*, double*);
static ApplyFn apply_fn(int dim, int tile) { MLG_TILE_SWITCH(dim, tile, return &enqueue_apply<TL>); }

int apply_operator(const mlg_grid* grid, const double* u, double* y, hipStream_t stream) {
  check_grid(grid);
  if (!u || !y) throw ArgError{MLG_ERR_ARG, "u and y must be device pointers"};
  const int tile = grid->dim == 3 ? 0 : 1;
  const Geo g = make_geo(*grid, tile, kMaxGrid);
  apply_fn(grid->dim, tile)(stream, g, u, y);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

}  // namespace mlg
