// Device side of restarted GMRES(m) on the zero-Dirichlet Poisson operator,
// for one or many independent systems at once.
//
// One restart cycle (Section 1.3 of the paper: GMRES(k) minimises the residual
// over K_k(A, r0) and restarts from the last iterate) is a fixed sequence of
// kernels that a HIP graph replays.  The Arnoldi process is classical
// Gram-Schmidt applied twice (CGS2) with the second pass delayed by one step,
// so each step needs ONE grid-wide reduction and TWO sweeps over the basis:
//
//   begin        systems starting a right-hand side: initial guess x0
//   resid0/rsum0 r = b - A x0, |r|, |b| for those systems; a zero right-hand
//                side or an already converged guess ends the RHS here
//   start        u_0 = r
//   dots(j)      w = A u_j (LDS-tiled stencil); per-workgroup partials of
//                s = V_{j-1}^T u_j, t = V_{j-1}^T w, u_j^T u_j, u_j^T w
//   coef(j)      one workgroup per system: sums the partials; second
//                projection of u_j (alpha = |u_j - V s|, Hessenberg column
//                j-1 = h_{j-1} + s, H[j, j-1] = alpha); Givens rotation,
//                residual estimate, stop test; first-projection coefficients
//                h_j of A v_j from the Arnoldi relation A V_{j-1} = V_j Hbar
//   extend(j)    v_j = (u_j - V_{j-1} s) / alpha;
//                u_{j+1} = A v_j - V_j h_j = w/alpha - V_j (Hbar s/alpha + h_j)
//   update       x += V_k y                     (FP64)
//   resid/rsum   r = b - A x, beta = |r| (FP64): acceptance on the true
//                residual; a finished system records its statistics and moves
//                on to its next right-hand side (or is done)
//
// Grid-wide sums never use atomics or fences inside a kernel: every sweep
// writes one partial per workgroup and a one-workgroup-per-system kernel sums
// them in a fixed order after the kernel boundary, which makes the partials
// visible across XCDs.  Runs are bitwise reproducible.
//
// Work distribution: a launch covers the tiles of every system of one tile
// shape; workgroup b takes job xcd_tile(b) -- a contiguous tile range of one
// system -- so each XCD owns contiguous bands of the grids and a workgroup
// keeps the same tiles (and their basis chunks in L2) for the whole solve.
#pragma once

#include <type_traits>

#include "common.h"

namespace mlg {

enum Phase { PH_INIT = 0, PH_RUN = 1, PH_ZERO = 2, PH_DONE = 3 };

// Packed column storage of the small dense matrices: Hessenberg column c
// holds rows 0..c+1, the rotated (upper triangular) column c rows 0..c.
__host__ __device__ constexpr int hu_off(int c) { return c * (c + 3) / 2; }
__host__ __device__ constexpr int r_off(int c) { return c * (c + 1) / 2; }

// Statistics of one right-hand side (copied to the host at the end).
struct Summary {
  int status;
  int cycles;
  long long iters;
  double relres_init, relres_first, relres_est, relres_true;
  double relres5;       // Givens estimate after Arnoldi step min(5, iters)
};

struct Ctrl {
  Summary s;            // statistics of the current right-hand side
  int phase;
  int cycle_end;        // the current cycle stopped stepping (until the next cycle opens)
  int tail_done;        // the current cycle's end (update, true residual) has run
  int k;                // Arnoldi columns of the current cycle
  int m, fixed, guess;
  int rhs, nrhs;        // current / total right-hand sides of this system
  long long limit;
  double rtol, bnorm, tol_abs, beta;
  double alpha;         // |u_j - V_{j-1} s| of the current step
  const double* b0;     // right-hand sides [nrhs][n]
  double* x0;           // solutions [nrhs][n]
  Summary* stats;       // this system's slots of the statistics array
  unsigned int* done;   // [0]: systems with every right-hand side solved,
                        // [1]: progress count (Arnoldi columns + finished RHS),
                        // [2]: systems forecast to finish in the next cycle
                        //      (counted by this cycle's k_rsum<false>),
                        // [3]: cycle ends run (update + true residual), all systems
  // first-projection coefficients h_{j-1}: step j reads row j & 1 and writes
  // row (j + 1) & 1, so a launch may read and write them at once
  double hprev[2][kMaxRestart + 1];
  double sums[2 * kMaxRestart + 2];        // column sums of step j's partials (k_sums)
  double sY[kMaxRestart + 1];              // second-projection coefficients (extend)
  double cY[kMaxRestart + 1];              // coefficients of V_j in u_{j+1} (extend)
  double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart];
  double Hu[hu_off(kMaxRestart)];          // Hessenberg, packed by column
  double R[r_off(kMaxRestart)];            // rotated Hessenberg, packed by column
};

struct Geo {
  int nx, ny, nz;                  // nz = 1 in 2D
  int tcx, tcy, tcz, ntiles;       // tile counts per axis, total
  int nblk;                        // workgroups this system gets per launch
  double cx, cy, cz;               // 1 / h^2 per axis
  long long n, ldv;                // points; stride between basis vectors
};

// Everything a workgroup needs to know about its system.
struct SysDesc {
  Geo g;
  Ctrl* C;
  void* V;        // basis: m vectors v_0..v_{m-1}, then u_even, u_odd (stride ldv)
  double* r;      // FP64 residual
  double* part;   // reduction partials, column c at part[c * nblk]
};

// One workgroup's share of a launch: a contiguous tile range of one system,
// with a copy of that system's geometry and buffers so that a workgroup can
// issue its data loads after a single table read (the control block, which
// differs between kernel timing copies, is reached through the descriptor).
struct Job {
  int sys;
  int t0, t1;
  int lblk;       // index of this workgroup among its system's workgroups
  int m;          // restart length (the directions follow the m basis vectors)
  int pad;
  Geo g;
  void* V;
  double* r;
  double* part;
};

template <int DIM_, int TX_, int TY_, int TZ_>
struct TileT {
  static constexpr int DIM = DIM_, TX = TX_, TY = TY_, TZ = TZ_;
  static constexpr int P = TX * TY * TZ;
  static constexpr int PPT = P / kBlock;
  static constexpr int LX = TX + 2, LY = TY + 2, LZ = DIM == 3 ? TZ + 2 : 1;
  static constexpr int LSZ = LX * LY * LZ;
  static_assert(P % kBlock == 0, "tile must be a multiple of the block");
  static_assert(DIM == 3 || TZ == 1, "2D tiles have TZ = 1");
};

template <class TL>
struct PointRef {
  int qx, qy, qz;
  bool valid;
  long long p;
};

template <class TL>
__device__ __forceinline__ void tile_origin(const Geo& g, int tile, int& ox, int& oy, int& oz) {
  int tx = tile % g.tcx;
  int r = tile / g.tcx;
  int ty = r % g.tcy;
  int tz = r / g.tcy;
  ox = tx * TL::TX;
  oy = ty * TL::TY;
  oz = tz * TL::TZ;
}

// Point i (0 <= i < PPT) of this thread inside the tile at (ox, oy, oz).
template <class TL>
__device__ __forceinline__ PointRef<TL> point(const Geo& g, int ox, int oy, int oz, int i) {
  PointRef<TL> pr;
  int q = threadIdx.x + kBlock * i;
  pr.qx = q % TL::TX;
  pr.qy = (q / TL::TX) % TL::TY;
  pr.qz = q / (TL::TX * TL::TY);
  int gx = ox + pr.qx, gy = oy + pr.qy, gz = oz + pr.qz;
  pr.valid = gx < g.nx && gy < g.ny && gz < g.nz;
  pr.p = ((long long)gz * g.ny + gy) * g.nx + gx;
  return pr;
}

// A tile with a RING-point halo as laid out in LDS.
template <class TL, int RING>
struct Halo {
  static constexpr int X = TL::TX + 2 * RING, Y = TL::TY + 2 * RING;
  static constexpr int Z = TL::DIM == 3 ? TL::TZ + 2 * RING : 1;
  static constexpr int SZ = X * Y * Z;
  // LDS index of tile-relative point (qx, qy, qz), which may lie in the halo
  static __device__ __forceinline__ int at(int qx, int qy, int qz) {
    return ((TL::DIM == 3 ? qz + RING : 0) * Y + (qy + RING)) * X + (qx + RING);
  }
};

// ---------------------------------------------------------------- buffer access
// The sweeps read and write the basis vectors (and the FP64 iterate) through
// raw buffer descriptors: a vector's base address and size live in scalar
// registers and each access takes a 32-bit element offset in one vector
// register, shared by every vector at the same point.  Global loads would
// each need a 64-bit address in two vector registers (and 64-bit address
// arithmetic per basis vector); with up to 40 vectors in flight per point
// that, not the data, set the register footprint and the occupancy of the
// long steps.  Fields hold fewer than 2^29 points, so byte offsets fit 32 bits.
constexpr int kBufDword3 = 0x00020000;   // word 3 of a raw buffer descriptor (gfx9 family)
using Rsrc = __amdgpu_buffer_rsrc_t;

// Descriptor of `count` elements from `base` (accesses past the end read 0).
template <class T>
__device__ __forceinline__ Rsrc vec_rsrc(const T* base, long long count) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, (int)(unsigned)(count * sizeof(T)),
                                           kBufDword3);
}
// Element e of the vector that starts `vo` bytes into the descriptor's
// region (vo in a scalar register: the range check covers e only).
__device__ __forceinline__ float buf_ld(Rsrc r, unsigned e, unsigned vo, float) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, e * 4u, vo, 0));
}
__device__ __forceinline__ double buf_ld(Rsrc r, unsigned e, unsigned vo, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8u, vo, 0));
}
template <class T>
__device__ __forceinline__ T buf_load(Rsrc r, unsigned e, unsigned vo = 0) {
  return buf_ld(r, e, vo, T{});
}
__device__ __forceinline__ void buf_store(Rsrc r, unsigned e, float v, unsigned vo = 0) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, e * 4u, vo, 0);
}
__device__ __forceinline__ void buf_store(Rsrc r, unsigned e, double v, unsigned vo = 0) {
  __builtin_amdgcn_raw_buffer_store_b64(
      __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r, e * 8u,
      vo, 0);
}

// The basis region of a system: one descriptor over all m + 2 vectors;
// vector k starts k * ldv elements in, selected by the scalar offset.  The
// region is smaller than 4 GiB (checked on the host), so every byte offset
// fits 32 bits and every access passes the descriptor's range check.
template <class T>
struct BasisBuf {
  Rsrc r;
  unsigned vb;                      // bytes between vectors
  __device__ __forceinline__ BasisBuf(const T* V, const Geo& g, int m)
      : r(vec_rsrc(V, (long long)(m + 2) * g.ldv)), vb((unsigned)(g.ldv * (long long)sizeof(T))) {}
  __device__ __forceinline__ T load(int k, unsigned e) const {
    return buf_load<T>(r, e, (unsigned)k * vb);
  }
  __device__ __forceinline__ void store(int k, unsigned e, T v) const {
    buf_store(r, e, v, (unsigned)k * vb);
  }
};

// Stage the tile of `src` plus a RING-point halo into LDS as FP64; points
// outside the grid read as 0 (the Dirichlet boundary).
template <class TL, int RING = 1, class P>
__device__ __forceinline__ void load_tile(double* L, P src, const Geo& g, int ox, int oy, int oz) {
  using H = Halo<TL, RING>;
  constexpr int NPT = (H::SZ + kBlock - 1) / kBlock;
  // every load is issued unconditionally (out-of-grid points read element 0
  // and are replaced by 0 afterwards), so no branch separates them
  double v[NPT];
  bool in[NPT];
#pragma unroll
  for (int h = 0; h < NPT; ++h) {
    const int e = threadIdx.x + kBlock * h;
    const int lx = e % H::X, r = e / H::X, ly = r % H::Y, lz = r / H::Y;
    const int gx = ox + lx - RING, gy = oy + ly - RING, gz = TL::DIM == 3 ? oz + lz - RING : 0;
    in[h] = e < H::SZ && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
    v[h] = (double)src[in[h] ? ((long long)gz * g.ny + gy) * g.nx + gx : 0];
  }
#pragma unroll
  for (int h = 0; h < NPT; ++h) {
    const int e = threadIdx.x + kBlock * h;
    if (e < H::SZ) L[e] = in[h] ? v[h] : 0.0;
  }
}

// A tile of a basis slot plus a RING-point halo, staged in two parts: issue()
// starts the loads into registers and write() later stores the values into
// LDS as FP64 (points outside the grid as 0, the Dirichlet boundary).  Loads
// issued in between stay in flight across write(): the memory counter is in
// order, so write() waits for the halo alone when the halo loads went first.
// Every halo load is unconditional (out-of-grid points read element 0); the
// empty asm at write() keeps the compiler from turning the masking select
// into a branch around each load, which would move the loads past the
// barrier that precedes write() and serialise them.
template <class TL, class T, int RING = 1>
struct HaloStage {
  using H = Halo<TL, RING>;
  static constexpr int NPT = (H::SZ + kBlock - 1) / kBlock;
  T v[NPT];
  bool in[NPT];
  __device__ __forceinline__ void issue(const BasisBuf<T>& B, int k, const Geo& g, int ox, int oy,
                                        int oz) {
#pragma unroll
    for (int h = 0; h < NPT; ++h) {
      const int e = threadIdx.x + kBlock * h;
      const int lx = e % H::X, r = e / H::X, ly = r % H::Y, lz = r / H::Y;
      const int gx = ox + lx - RING, gy = oy + ly - RING, gz = TL::DIM == 3 ? oz + lz - RING : 0;
      in[h] = e < H::SZ && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
      v[h] = B.load(k, in[h] ? (unsigned)(((long long)gz * g.ny + gy) * g.nx + gx) : 0u);
    }
  }
  __device__ __forceinline__ void write(double* L) {
#pragma unroll
    for (int h = 0; h < NPT; ++h) {
      asm volatile("" : "+v"(v[h]));
      const int e = threadIdx.x + kBlock * h;
      if (e < H::SZ) L[e] = in[h] ? (double)v[h] : 0.0;
    }
  }
};

// (A u) at LDS index i of a staged tile with row pitch px and plane pitch pxy:
// sum over axes of (2 u - u_minus - u_plus) / h^2.  Not contracted, so that
// every evaluation of the same point rounds identically wherever it is
// inlined (the fused step recomputes halo points that another workgroup owns).
template <int DIM>
__device__ __forceinline__ double stencil_at(const double* L, const Geo& g, int i, int px, int pxy) {
#pragma clang fp contract(off)
  const double c = L[i];
  double a = (2.0 * c - L[i - 1] - L[i + 1]) * g.cx + (2.0 * c - L[i - px] - L[i + px]) * g.cy;
  if (DIM == 3) a += (2.0 * c - L[i - pxy] - L[i + pxy]) * g.cz;
  return a;
}

// (A u) at a tile point from a tile staged with a one-point halo.
template <class TL>
__device__ __forceinline__ double stencil(const double* L, const Geo& g, int qx, int qy, int qz) {
  using H = Halo<TL, 1>;
  return stencil_at<TL::DIM>(L, g, H::at(qx, qy, qz), H::X, H::X * H::Y);
}

// The tile point itself from a tile staged with a one-point halo.
template <class TL>
__device__ __forceinline__ double centre(const double* L, int qx, int qy, int qz) {
  return L[Halo<TL, 1>::at(qx, qy, qz)];
}

// Tile-relative position of ring point r (0 <= r < LSZ - P) of the one-point
// halo: in 3D the two z faces first, then per interior z plane the rows above
// and below the tile, then its left and right columns.
template <class TL>
__device__ __forceinline__ void ring_point(int r, int& qx, int& qy, int& qz) {
  constexpr int LX = TL::LX, LY = TL::LY;
  qz = 0;
  if (TL::DIM == 3) {
    constexpr int F = LX * LY;
    if (r < 2 * F) {
      qz = r < F ? -1 : TL::TZ;
      const int q = r < F ? r : r - F;
      qx = q % LX - 1;
      qy = q / LX - 1;
      return;
    }
    r -= 2 * F;
    constexpr int SR = 2 * LX + 2 * TL::TY;
    qz = r / SR;
    r -= qz * SR;
  }
  if (r < 2 * LX) {
    qy = r < LX ? -1 : TL::TY;
    qx = (r < LX ? r : r - LX) - 1;
  } else {
    r -= 2 * LX;
    qy = r >> 1;
    qx = (r & 1) ? TL::TX : -1;
  }
}

// v_j and u_{j+1} at one point from u_j, (A u_j) and the basis sums
// a = V_{j-1} s, b = V_{j-1} cY there.  Explicit FMAs only: the fused step
// evaluates this both for its own points and for halo points of its
// neighbours, and both must round the same way.
template <class T>
__device__ __forceinline__ void extend_point(double uu, double ww, double a, double b, double ainv,
                                             double cyj, T& vj, T& un) {
#pragma clang fp contract(off)
  vj = (T)((uu - a) * ainv);
  un = (T)fma(-cyj, (double)vj, fma(ww, ainv, -b));
}

// This workgroup's job (by value) and its system's descriptor.
struct Mine {
  Job job;
  const SysDesc* S;
};
__device__ __forceinline__ Mine mine(const Job* jobs, const SysDesc* sd) {
  Mine me;
  me.job = jobs[xcd_tile(blockIdx.x, gridDim.x)];
  me.S = sd + me.job.sys;
  return me;
}

// The end of a cycle (update, true residual and its test) runs once, after
// the cycle stopped stepping: a launch sequence may place it after any step.
template <class CP>
__device__ __forceinline__ bool cycle_tail_pending(const CP& C) {
  return C->phase == PH_RUN && C->cycle_end && !C->tail_done;
}

// A finished right-hand side: record its statistics and move on to the next
// one (phase INIT) or mark the system done.  One thread.
__device__ inline void finish_rhs(gptr<Ctrl> C) {
  atomicAdd(C->done + 1, 1u);
  const gptr<Summary> st = gmem(C->stats) + C->rhs;
  st->status = C->s.status;
  st->cycles = C->s.cycles;
  st->iters = C->s.iters;
  st->relres_init = C->s.relres_init;
  st->relres_first = C->s.relres_first;
  st->relres_est = C->s.relres_est;
  st->relres_true = C->s.relres_true;
  st->relres5 = C->s.relres5;
  C->rhs += 1;
  C->cycle_end = 1;
  if (C->rhs >= C->nrhs) {
    C->phase = PH_DONE;
    atomicAdd(C->done, 1u);
  } else {
    C->phase = PH_INIT;
  }
}

// Broadcast lane `src` of a wavefront's FP64 value (src wave-uniform).
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Slots k0 .. k0 + KC - 1 of the basis at this thread's points, every load of
// the chunk issued at once and unconditionally: slots k >= `live` re-read the
// last live vector (vector `spare` when none is live), so no branch separates
// the loads.  Those slots may meet zero coefficients (an exact no-op) but are
// otherwise unused; they must hold finite data, which written vectors do (a
// slot not yet written in this cycle may not).  The sweeps stream the basis
// through registers one chunk at a time, the next chunk's loads in flight
// while the current one is used, so their register use does not grow with
// the restart length and larger tiles stay resident.
// Chunks of basis slots in flight ahead of the one in use (chunk buffers
// minus one) in the dot-product and extension sweeps.
#ifndef MLG_SWEEP_NB
#define MLG_SWEEP_NB 2
#endif
constexpr int kSweepBufs = MLG_SWEEP_NB;

template <int KC, int N, class T>
__device__ __forceinline__ void load_basis_chunk(T (&v)[KC][N], const BasisBuf<T>& B,
                                                 const long long (&p)[N], int k0, int live,
                                                 int spare) {
  const int last = live > 0 ? live - 1 : spare;
#pragma unroll
  for (int q = 0; q < KC; ++q) {
    const int k = k0 + q;
#pragma unroll
    for (int i = 0; i < N; ++i) v[q][i] = B.load(k < live ? k : last, (unsigned)p[i]);
  }
}

// Block sums of the folded products into this workgroup's partial columns.
// Sum index k < 16 * (MM / 8): basis slot 8 * (k / 16) + (k % 8), the x
// product for k % 16 < 8, else the y product; then the 4 `last` sums.
// col(slot, is_y) / col_last(f) give the partial column, or -1 for none.
template <int MM, class ColFn, class LastFn>
__device__ __forceinline__ void store_folded(const double (&acc)[MM / 8 + 1], double* red,
                                             gptr<double> part, int nblk, int lblk, ColFn col,
                                             LastFn col_last) {
  constexpr int NCH = MM / 8, NS = 16 * NCH + 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if ((lane & 3) == 0) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) red[wave * NS + 16 * c + rs16_slot(lane)] = acc[c];
  }
  if ((lane & 15) == 0) red[wave * NS + 16 * NCH + rs4_slot(lane)] = acc[NCH];
  __syncthreads();
  for (int k = threadIdx.x; k < NS; k += kBlock) {
    const int cl = k < 16 * NCH ? col(8 * (k >> 4) + (k & 7), (k & 15) >= 8) : col_last(k - 16 * NCH);
    if (cl >= 0)
      part[(size_t)cl * nblk + lblk] = ((red[k] + red[NS + k]) + red[2 * NS + k]) + red[3 * NS + k];
  }
}

// ---------------------------------------------------------------- kernels

// begin: initial guess of a system that starts a right-hand side other than
// its first (whose guess the caller provides): zero, or the previous solution.
template <class T, class TL>
__global__ __launch_bounds__(kBlock) void k_begin(const Job* jobs, const SysDesc* sd) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_INIT || C->rhs == 0) return;
  const Geo g = me.job.g;
  gptr<double> x = gmem(C->x0) + (size_t)C->rhs * g.n;
  gptr<const double> xp = x - g.n;
  const bool prev = C->guess == 1;
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
#pragma unroll
    for (int i = 0; i < TL::PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      if (pr.valid) x[pr.p] = prev ? xp[pr.p] : 0.0;
    }
  }
}

// r = b - A x: partials of |r|^2 and, when starting a right-hand side, |b|^2.
template <class T, class TL, bool INIT>
__global__ __launch_bounds__(kBlock) void k_resid(const Job* jobs, const SysDesc* sd) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (INIT ? C->phase != PH_INIT : !cycle_tail_pending(C)) return;
  constexpr int PPT = TL::PPT;
  __shared__ double L[TL::LSZ];
  __shared__ double red[4 * 4];
  const Geo g = me.job.g;
  gptr<const double> b = gmem(C->b0) + (size_t)C->rhs * g.n;
  gptr<const double> x = gmem((const double*)C->x0) + (size_t)C->rhs * g.n;
  gptr<double> r = gmem(me.job.r);
  double acc[1] = {0.0};
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
    long long pp[PPT];
    bool ok[PPT];
    int qc[PPT][3];
    double bv[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      ok[i] = pr.valid;
      pp[i] = pr.valid ? pr.p : 0;
      qc[i][0] = pr.qx;
      qc[i][1] = pr.qy;
      qc[i][2] = pr.qz;
      bv[i] = b[pp[i]];
    }
    __syncthreads();
    load_tile<TL>(L, x, g, ox, oy, oz);
    __syncthreads();
    double last[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < PPT; ++i)
      if (ok[i]) {
        const double ri = bv[i] - stencil<TL>(L, g, qc[i][0], qc[i][1], qc[i][2]);
        r[pp[i]] = ri;
        last[0] = fma(ri, ri, last[0]);
        last[1] = fma(bv[i], bv[i], last[1]);
      }
    acc[0] += rs4(last);
  }
  store_folded<0>(acc, red, gmem(me.job.part), g.nblk, me.job.lblk,
                  [](int, bool) { return -1; },
                  [](int f) { return f == 0 || (INIT && f == 1) ? f : -1; });
}

// beta = |r| (and |b| when starting): one workgroup per system.
template <bool INIT>
__global__ __launch_bounds__(kReduceThreads) void k_rsum(const SysDesc* sd) {
  const SysDesc* S = sd + blockIdx.x;
  const gptr<Ctrl> C = gmem(S->C);
  // k_rsum<true> opens every cycle: clear the cycle's forecast count, and
  // let a system that continues its right-hand side step again
  if (INIT && blockIdx.x == 0 && threadIdx.x == 0) C->done[2] = 0u;
  if (INIT && C->phase == PH_RUN) {
    if (threadIdx.x == 0) {
      C->cycle_end = 0;
      C->tail_done = 0;
    }
    return;
  }
  if (INIT ? C->phase != PH_INIT : !cycle_tail_pending(C)) return;
  __shared__ double fin[2];
  reduce_partials(gmem((const double*)S->part), S->g.nblk, INIT ? 2 : 1, fin);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(fin[0]);
  C->beta = beta;
  C->g[0] = beta;
  C->k = 0;
  if (INIT) {
    C->cycle_end = 0;
    C->tail_done = 0;
  } else {
    // the cycle stays stopped (its remaining steps, if launched, do nothing)
    // until the next cycle opens it
    C->tail_done = 1;
    atomicAdd(C->done + 3, 1u);
  }
  if (INIT) {
    const double bnorm = sqrt(fin[1]);
    C->s.status = MLG_OK;
    C->s.cycles = 0;
    C->s.iters = 0;
    C->bnorm = bnorm;
    C->tol_abs = C->rtol * bnorm;
    if (bnorm == 0.0) {                     // A x = 0: x = 0 (written by start)
      C->s.relres_init = C->s.relres_first = C->s.relres_est = C->s.relres_true = 0.0;
      C->s.relres5 = 0.0;
      C->phase = PH_ZERO;
      return;
    }
    const double rr = beta / bnorm;
    C->s.relres_init = rr;
    C->s.relres_first = rr;
    C->s.relres_est = rr;
    C->s.relres_true = rr;
    C->s.relres5 = rr;
    if (!isfinite(beta)) {
      C->s.status = MLG_ERR_NONFINITE;
      finish_rhs(C);
    } else if ((!C->fixed && beta <= C->tol_abs) || beta == 0.0 || C->limit <= 0) {
      finish_rhs(C);
    } else {
      C->phase = PH_RUN;
    }
    return;
  }
  const int cycles = C->s.cycles + 1;
  C->s.cycles = cycles;
  const double rr = beta / C->bnorm;
  const double rr_prev = C->s.relres_true;     // at the start of this cycle
  C->s.relres_true = rr;
  if (cycles == 1) C->s.relres_first = rr;
  if (!isfinite(beta)) {
    C->s.status = MLG_ERR_NONFINITE;
    finish_rhs(C);
    return;
  }
  const bool conv = !C->fixed && beta <= C->tol_abs;
  if (conv || C->s.iters >= C->limit || beta == 0.0) {
    C->s.status = (conv || C->fixed || beta == 0.0) ? MLG_OK : MLG_NOT_CONVERGED;
    finish_rhs(C);
  } else if (!C->fixed && C->rhs + 1 >= C->nrhs && rr * (rr / rr_prev) <= C->rtol) {
    // forecast for the host's scheduling only: the last right-hand side, its
    // residual extrapolated by this cycle's reduction factor, reaches the
    // tolerance in the next cycle
    atomicAdd(C->done + 2, 1u);
  }
}

// start: u_0 = r (in the basis precision T); x = 0 for a zero right-hand side.
template <class T, class TL>
__global__ __launch_bounds__(kBlock) void k_start(const Job* jobs, const SysDesc* sd) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_RUN && C->phase != PH_ZERO) return;
  const bool zero = C->phase == PH_ZERO;
  const Geo g = me.job.g;
  gptr<T> U0 = gmem((T*)me.job.V) + (size_t)me.job.m * g.ldv;
  const gptr<double> r = gmem(me.job.r);
  gptr<double> x = gmem(C->x0) + (size_t)C->rhs * g.n;
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
#pragma unroll
    for (int i = 0; i < TL::PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      if (pr.valid) {
        if (zero) x[pr.p] = 0.0;
        else U0[pr.p] = (T)r[pr.p];
      }
    }
  }
}

// dots(j): w = A u_j; partials of s = V_{j-1}^T u_j (columns 0..j-1),
// t = V_{j-1}^T w (columns j..2j-1), u^T u (column 2j), u^T w (column 2j+1).
// MM >= j bounds the basis slots held in registers; all loads of a tile are
// issued before any is used.
template <class T, class TL, int MM>
__global__ __launch_bounds__(kBlock) void k_dots(const Job* jobs, const SysDesc* sd, int j) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_RUN || C->cycle_end) return;
  constexpr int PPT = TL::PPT;
  constexpr int NS = 16 * (MM / 8) + 4;
  __shared__ double L[TL::LSZ];
  __shared__ double red[4 * NS];
  const Geo g = me.job.g;
  const BasisBuf<T> VB((const T*)me.job.V, g, me.job.m);
  const int kU = me.job.m + (j & 1);
  double acc[MM / 8 + 1];
#pragma unroll
  for (int c = 0; c <= MM / 8; ++c) acc[c] = 0.0;
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
    long long pp[PPT];
    bool ok[PPT];
    int qc[PPT][3];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      ok[i] = pr.valid;
      pp[i] = pr.valid ? pr.p : 0;
      qc[i][0] = pr.qx;
      qc[i][1] = pr.qy;
      qc[i][2] = pr.qz;
    }
    constexpr int KC = 8, NCH = MM / KC, NB = kSweepBufs;
    // the halo of u_j first, then the first chunks of the basis: those stay
    // in flight while the halo is written to LDS and the stencil applied
    HaloStage<TL, T> hs;
    hs.issue(VB, kU, g, ox, oy, oz);
    T vb[NB][KC][PPT];
    __builtin_amdgcn_sched_barrier(0);
    load_basis_chunk<KC, PPT, T>(vb[0], VB, pp, 0, j, kU);
#pragma unroll
    for (int c = 1; c < NB - 1; ++c)
      if (c < NCH && KC * c < j) load_basis_chunk<KC, PPT, T>(vb[c], VB, pp, KC * c, j, kU);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    hs.write(L);
    __syncthreads();
    double uu[PPT], ww[PPT], last[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      uu[i] = ok[i] ? centre<TL>(L, qc[i][0], qc[i][1], qc[i][2]) : 0.0;
      ww[i] = ok[i] ? stencil<TL>(L, g, qc[i][0], qc[i][1], qc[i][2]) : 0.0;
      last[0] = fma(uu[i], uu[i], last[0]);
      last[1] = fma(uu[i], ww[i], last[1]);
    }
    // products per chunk of 8 slots, folded across the wavefront (16 sums)
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      // the scheduler keeps each chunk's loads here (NB - 1 chunks ahead),
      // not hoisted to the top, so only NB chunks occupy registers
      __builtin_amdgcn_sched_barrier(0);
      if (c + NB - 1 < NCH && KC * (c + NB - 1) < j)
        load_basis_chunk<KC, PPT, T>(vb[(c + NB - 1) % NB], VB, pp, KC * (c + NB - 1), j, kU);
      if (KC * c < j) {
        double prod[16];
#pragma unroll
        for (int q = 0; q < KC; ++q) {
          prod[q] = 0.0;
          prod[KC + q] = 0.0;
#pragma unroll
          for (int i = 0; i < PPT; ++i) {
            prod[q] = fma((double)vb[c % NB][q][i], uu[i], prod[q]);
            prod[KC + q] = fma((double)vb[c % NB][q][i], ww[i], prod[KC + q]);
          }
        }
        acc[c] += rs16(prod);
      }
    }
    acc[NCH] += rs4(last);
  }
  store_folded<MM>(acc, red, gmem(me.job.part), g.nblk, me.job.lblk,
                   [j](int slot, bool y) { return slot < j ? (y ? j + slot : slot) : -1; },
                   [j](int f) { return f < 2 ? 2 * j + f : -1; });
}

// ------------------------------------------------ coefficient update of step j
// Wavefront 0 of a workgroup, lane i owning row i (j <= 64).  fin holds the
// column sums of the step's partials (s: 0..j-1, t: j..2j-1, u^T u, u^T w),
// HuS the Hessenberg columns 0..j-2 (packed); hpi is h_{j-1} at this lane.
struct StepCoef {
  double nu, si, hpl, alpha, coli, h, cy;
};

// Second projection of u_j and the coefficients of the next sweep: alpha =
// |u_j - V s|, Hessenberg column j-1 = h_{j-1} + s with subdiagonal alpha
// (stored into HuS), z = Hbar_{j-1} s, h_j = (V_j^T A v_j) from the Arnoldi
// relation, cY = z / alpha + h_j, sY = s.
__device__ __forceinline__ StepCoef coef_project(const double* fin, double* HuS, int j,
                                                 double hpi) {
  const int lane = threadIdx.x & 63;
  StepCoef q;
  q.nu = fin[2 * j];
  const double mu = fin[2 * j + 1];
  q.si = lane < j ? fin[lane] : 0.0;
  const double ti = lane < j ? fin[j + lane] : 0.0;
  q.hpl = lane < j ? hpi : 0.0;
  const double ss = wave_sum(q.si * q.si);
  const double st = wave_sum(q.si * ti);
  q.coli = 0.0;
  if (j == 0) {
    q.alpha = sqrt(q.nu);
  } else {
    // |u_j - V s|^2 = |u_j|^2 - |s|^2 (V orthonormal)
    q.alpha = sqrt(fmax(q.nu - ss, 0.0));
    q.coli = lane < j ? q.hpl + q.si : (lane == j ? q.alpha : 0.0);
    if (lane <= j) HuS[hu_off(j - 1) + lane] = q.coli;
  }
  // h_i = v_i^T A v_j with A v_j = (w - V_j z) / alpha, z = Hbar_{j-1} s
  double z = 0.0;
  if (lane <= j)
    for (int c2 = (lane > 0 ? lane - 1 : 0); c2 < j; ++c2) z += HuS[hu_off(c2) + lane] * fin[c2];
  const double vw = lane < j ? ti : (mu - st) / q.alpha;
  q.h = (vw - z) / q.alpha;
  q.cy = z / q.alpha + q.h;
  return q;
}

// Fields of the control block the stop test reads (loaded at kernel start).
struct StopState {
  long long iters, limit;
  double tol_abs, bnorm;
  int fixed, m;
};
__device__ __forceinline__ StopState stop_state(gptr<const Ctrl> C) {
  return StopState{C->s.iters, C->limit, C->tol_abs, C->bnorm, C->fixed, C->m};
}

// The system's own state for step j >= 1 (one workgroup per system calls
// this): stores Hessenberg column j-1 and h_j, applies the Givens rotations
// G_0..G_{j-2} to the column and forms G_{j-1}, updates the residual
// estimate and tests for the end of the cycle.  Returns 0 to continue, 1 at
// the end of the cycle, 2 on a non-finite value (status set; the caller
// finishes the RHS); rot is this lane's entry of the rotated column, gnew the
// rotated g_{j-1}.
__device__ __forceinline__ int coef_rotate(gptr<Ctrl> C, const StepCoef& q, int j,
                                           const StopState& ss, double csl, double snl, double gc,
                                           double& rot, double& gnew) {
  const int lane = threadIdx.x & 63;
  const int c = j - 1;
  if (lane <= j) {
    C->Hu[hu_off(c) + lane] = q.coli;
    C->hprev[(j + 1) & 1][lane] = q.h;
  }
  const double hh = wave_sum(q.hpl * q.hpl);
  // rotations G_0..G_{c-1}: carry the running entry down the column
  const double csv = lane < c ? csl : 0.0, snv = lane < c ? snl : 0.0;
  double carry = lane_bcast(q.coli, 0);
  rot = 0.0;
  for (int i = 0; i < c; ++i) {
    const double a = carry, bb = lane_bcast(q.coli, i + 1);
    const double ci = lane_bcast(csv, i), sni = lane_bcast(snv, i);
    if (lane == i) rot = ci * a + sni * bb;
    carry = -sni * a + ci * bb;
  }
  const double den = hypot(carry, q.alpha);
  double cc = 1.0, sn = 0.0;
  if (den != 0.0) {
    cc = carry / den;
    sn = q.alpha / den;
  }
  if (lane == c) rot = den;
  if (lane <= c) C->R[r_off(c) + lane] = rot;
  gnew = cc * gc;
  const double est = fabs(sn * gc);
  const long long iters = ss.iters + 1;
  // breakdown: the new direction is rounding noise relative to A v_{j-1}
  // (|A v_{j-1}|^2 = |u_j|^2 + |h_{j-1}|^2)
  const bool breakdown = q.alpha <= 1e-14 * sqrt(q.nu + hh);
  const bool bad = !isfinite(q.alpha) || !isfinite(est);
  const bool stop = bad || iters >= ss.limit || breakdown || (!ss.fixed && est <= ss.tol_abs) ||
                    j == ss.m;
  if (lane == 0) {
    C->cs[c] = cc;
    C->sn[c] = sn;
    C->g[c + 1] = -sn * gc;
    C->g[c] = gnew;
    C->s.iters = iters;
    C->k = j;
    C->s.relres_est = est / ss.bnorm;
    if (iters <= 5) C->s.relres5 = est / ss.bnorm;
    atomicAdd(C->done + 1, 1u);
    if (bad) C->s.status = MLG_ERR_NONFINITE;
  }
  return bad ? 2 : (stop ? 1 : 0);
}

// End of a cycle after step j: back substitution R y = g (R: j x j upper
// triangular, packed in Rs), row i on lane i of wavefront 0.
__device__ __forceinline__ void back_substitute(gptr<Ctrl> C, const double* Rs, int j, double gl) {
  const int lane = threadIdx.x & 63;
  double accl = 0.0, yl = 0.0;
  for (int i = j - 1; i >= 0; --i) {
    const double yi = lane_bcast((gl - accl) / (lane < j ? Rs[r_off(lane) + lane] : 1.0), i);
    if (lane == i) yl = yi;
    if (lane < i) accl += Rs[r_off(i) + lane] * yi;
  }
  if (lane < j) C->y[lane] = yl;
  if (lane == 0) C->cycle_end = 1;
}

// coef(j): one workgroup per system (those in `list`, or system blockIdx.x).
// Every global load of the launch (the first round of partials, the
// Hessenberg columns, wavefront 0's per-row state) is issued at once and
// consumed before the state is tested, so their latencies overlap.
// Wavefront 0 then runs the coefficient update; at the end of a cycle R is
// staged by all threads for the back substitution.  For a zero right-hand
// side, coef(0) ends the RHS.
template <int NB>
__global__ __launch_bounds__(kReduceThreads) void k_coef(const SysDesc* sd, const int* list,
                                                         int j) {
  constexpr int HPT = (hu_off(kMaxRestart) + kReduceThreads - 1) / kReduceThreads;
  constexpr int RPT = (r_off(kMaxRestart) + kReduceThreads - 1) / kReduceThreads;
  __shared__ double fin[2 * kMaxRestart + 2];
  // Hessenberg columns (for z) or, at the end of a cycle, the rotated R
  __shared__ double HuS[hu_off(kMaxRestart)];
  __shared__ int flag;
  double* Rs = HuS;
  const SysDesc* S = sd + (list ? list[blockIdx.x] : (int)blockIdx.x);
  const gptr<Ctrl> C = gmem(S->C);
  const gptr<const double> part = gmem((const double*)S->part);
  const int nblk = S->g.nblk;
  const int ncols = 2 * j + 2;
  const int tid = threadIdx.x, lane = tid;
  const bool w0 = tid < 64;
  const int c = j - 1;
  // ---- all loads at once
  PartialsRound<NB> r0;
  partials_load(r0, part, nblk, ncols, 0);
  const int hlim = j > 1 ? hu_off(j - 1) : 0;          // columns 0..j-2
  double hv[HPT];
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    const int e = tid + kReduceThreads * k;
    hv[k] = 0.0;
    if (e < hlim) hv[k] = C->Hu[e];
  }
  const double hpi = C->hprev[j & 1][w0 && lane < j ? lane : 0];
  const double csl = C->cs[w0 && lane < c ? lane : 0];
  const double snl = C->sn[w0 && lane < c ? lane : 0];
  const double gc = C->g[j > 0 ? c : 0];
  const double glane = C->g[w0 && lane < j ? lane : 0];
  const StopState ss = stop_state(C);
  partials_sum(r0, nblk, ncols, 0, fin);
#pragma unroll
  for (int k = 0; k < HPT; ++k) {
    const int e = tid + kReduceThreads * k;
    if (e < hlim) HuS[e] = hv[k];
  }
  for (int c0 = PartialsRound<NB>::kCols; c0 < ncols; c0 += PartialsRound<NB>::kCols) {
    PartialsRound<NB> r;
    partials_load(r, part, nblk, ncols, c0);
    partials_sum(r, nblk, ncols, c0, fin);
  }
  if (j == 0 && C->phase == PH_ZERO) {
    if (tid == 0) finish_rhs(C);
    return;
  }
  if (C->phase != PH_RUN || C->cycle_end) return;
  __syncthreads();
  StepCoef q{};
  double rot = 0.0, gnew = 0.0;
  if (w0) {
    q = coef_project(fin, HuS, j, hpi);
    int fl = 0;
    if (j > 0) {
      fl = coef_rotate(C, q, j, ss, csl, snl, gc, rot, gnew);
    } else if (lane == 0) {
      C->hprev[1][0] = q.h;
    }
    if (lane == 0) flag = fl;
  }
  __syncthreads();
  const int fl = flag;
  if (fl == 2) {
    if (tid == 0) finish_rhs(C);
    return;
  }
  if (fl == 1) {
    // columns 0..c-1 of R from memory (staged by all threads), column c from
    // wavefront 0's registers
    const int rlim = r_off(c);
    double rv[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int e = tid + kReduceThreads * k;
      rv[k] = 0.0;
      if (e < rlim) rv[k] = C->R[e];
    }
    __syncthreads();                                  // HuS is no longer read
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int e = tid + kReduceThreads * k;
      if (e < rlim) Rs[e] = rv[k];
    }
    if (w0 && lane <= c) Rs[rlim + lane] = rot;
    __syncthreads();
    if (w0) back_substitute(C, Rs, j, lane < j ? (lane == c ? gnew : glane) : 0.0);
    return;
  }
  if (!w0) return;
  if (lane <= j) {
    C->cY[lane] = q.cy;
    C->sY[lane] = q.si;
  }
  if (lane == 0) C->alpha = q.alpha;
}

// sums(j): the column sums of step j's partials into the control block, one
// wavefront per column (columns spread over blockIdx.x, systems over
// blockIdx.y: those in `list`, or all), in the order coef(j) sums them.
// sums(0) also ends a zero right-hand side.
template <int NB>
__global__ __launch_bounds__(kBlock) void k_sums(const SysDesc* sd, const int* list, int j) {
  constexpr int NW = kBlock / 64;
  const SysDesc* S = sd + (list ? list[blockIdx.y] : (int)blockIdx.y);
  const int lane = threadIdx.x & 63, c = blockIdx.x * NW + (threadIdx.x >> 6);
  const int nblk = S->g.nblk;
  // a zero right-hand side ends here, as at coef(0) in the other forms
  if (j == 0 && blockIdx.x == 0 && threadIdx.x == 0 && gmem(S->C)->phase == PH_ZERO)
    finish_rhs(gmem(S->C));
  if (c >= 2 * j + 2) return;                         // wavefront-uniform
  const gptr<const double> part = gmem((const double*)S->part) + (size_t)c * nblk;
  double v[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = lane + 64 * i;
    v[i] = b < nblk ? part[b] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NB; ++i) s += v[i];
  s = wave_sum(s);
  if (lane == 0) gmem(S->C)->sums[c] = s;
}

// extend(j): v_j = (u_j - V_{j-1} s) / alpha, u_{j+1} = w/alpha - V_j cY.
template <class T, class TL, int MM>
__global__ __launch_bounds__(kBlock) void k_extend(const Job* jobs, const SysDesc* sd, int j) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_RUN || C->cycle_end) return;
  constexpr int PPT = TL::PPT;
  __shared__ double L[TL::LSZ];
  // coefficients zero beyond j, so every register slot takes an
  // unconditional FMA (adding exact zeros) instead of a per-slot select
  __shared__ double sY[MM], cY[MM];
  for (int k = threadIdx.x; k < MM; k += kBlock) {
    sY[k] = k < j ? C->sY[k] : 0.0;
    cY[k] = k < j ? C->cY[k] : 0.0;
  }
  const Geo g = me.job.g;
  const BasisBuf<T> VB((const T*)me.job.V, g, me.job.m);
  const int kU = me.job.m + (j & 1), kUn = me.job.m + ((j + 1) & 1);
  const double ainv = 1.0 / C->alpha;
  const double cyj = C->cY[j];
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
    long long pp[PPT];
    bool ok[PPT];
    int qc[PPT][3];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      ok[i] = pr.valid;
      pp[i] = pr.valid ? pr.p : 0;
      qc[i][0] = pr.qx;
      qc[i][1] = pr.qy;
      qc[i][2] = pr.qz;
    }
    constexpr int KC = 8, NCH = MM / KC, NB = kSweepBufs;
    // the halo of u_j first, then the first chunks (in flight across the
    // LDS write)
    HaloStage<TL, T> hs;
    hs.issue(VB, kU, g, ox, oy, oz);
    T vb[NB][KC][PPT];
    __builtin_amdgcn_sched_barrier(0);
    load_basis_chunk<KC, PPT, T>(vb[0], VB, pp, 0, j, kU);
#pragma unroll
    for (int c = 1; c < NB - 1; ++c)
      if (c < NCH && KC * c < j) load_basis_chunk<KC, PPT, T>(vb[c], VB, pp, KC * c, j, kU);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    hs.write(L);
    __syncthreads();
    // a = V s, b = V cY at this thread's points, slot by slot in order (the
    // chunks past j hold zero coefficients only and are skipped)
    double a[PPT], b[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) a[i] = b[i] = 0.0;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      // the scheduler keeps each chunk's loads here (NB - 1 chunks ahead),
      // not hoisted to the top, so only NB chunks occupy registers
      __builtin_amdgcn_sched_barrier(0);
      if (c + NB - 1 < NCH && KC * (c + NB - 1) < j)
        load_basis_chunk<KC, PPT, T>(vb[(c + NB - 1) % NB], VB, pp, KC * (c + NB - 1), j, kU);
      if (KC * c < j) {
#pragma unroll
        for (int q = 0; q < KC; ++q)
#pragma unroll
          for (int i = 0; i < PPT; ++i) {
            a[i] = fma((double)vb[c % NB][q][i], sY[KC * c + q], a[i]);
            b[i] = fma((double)vb[c % NB][q][i], cY[KC * c + q], b[i]);
          }
      }
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i)
      if (ok[i]) {
        const double uu = centre<TL>(L, qc[i][0], qc[i][1], qc[i][2]);
        const double ww = stencil<TL>(L, g, qc[i][0], qc[i][1], qc[i][2]);
        T vj, un;
        extend_point<T>(uu, ww, a[i], b[i], ainv, cyj, vj, un);
        VB.store(j, (unsigned)pp[i], vj);
        VB.store(kUn, (unsigned)pp[i], un);
      }
  }
}

// step(j) = extend(j) followed by dots(j+1), one sweep over the basis.
// extend(j) needs u_j only at the workgroup's own points, but dots(j+1) needs
// w = A u_{j+1}, i.e. u_{j+1} on a one-point halo around the tile as well.
// The workgroup therefore recomputes u_{j+1} on that ring itself (u_j staged
// with a two-point halo, the basis read at the ring points) -- bitwise the
// values the owning workgroup stores, since both evaluate the same
// uncontracted expressions in the same order.  The basis values of its own
// points stay in registers between the extension and the products, so
// V_{j-1} is read once per step:
//   v_j = (u_j - V_{j-1} s) / alpha,  u_{j+1} = w_j/alpha - V_{j-1} cY - cY_j v_j
//   partials of s' = V_j^T u_{j+1} (columns 0..j), t' = V_j^T w_{j+1}
//   (j+1..2j+1), u_{j+1}^T u_{j+1} (2j+2), u_{j+1}^T w_{j+1} (2j+3).
// The products of each tile are folded across the wavefront at once (chunks
// of 8 basis vectors, 16 sums, reduce-scatter), so a lane carries only one
// running sum per chunk and the kernel keeps its occupancy.
template <class T, class TL, int MM, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_step(const Job* jobs, const SysDesc* sd, int j) {
  const Mine me = mine(jobs, sd);
  const gptr<Ctrl> C = gmem((Ctrl*)me.S->C);
  // a system that is not stepping leaves before any load: the steps after
  // its cycle ended are replayed as part of the cycle, and must cost no
  // more than the launch (uniform: the whole workgroup leaves)
  if (C->phase != PH_RUN || C->cycle_end) return;
  const int tid = threadIdx.x;
  using H1 = Halo<TL, 1>;
  using H2 = Halo<TL, 2>;
  constexpr int PPT = TL::PPT;
  constexpr int KC = 8;
  static_assert(MM % KC == 0, "register bound must be a multiple of the chunk");
  constexpr int NCH = MM / KC;                       // chunks of 16 sums
  constexpr int NS = 16 * NCH + 4;                   // sums per wavefront
  constexpr int RS = H1::SZ - TL::P;                 // ring points
  constexpr int RPT = (RS + kBlock - 1) / kBlock;
  constexpr int HPT = (H2::SZ + kBlock - 1) / kBlock;
  // split form: Hessenberg columns 0..j-1 (j < MM), later R, share L1's space
  constexpr int HUS = SPLIT ? hu_off(MM - 1) : 0;
  constexpr int HT = (hu_off(MM - 2) + kBlock - 1) / kBlock;
  constexpr int RT = (r_off(MM - 2) + kBlock - 1) / kBlock;
  constexpr int L1SZ = H1::SZ > HUS ? H1::SZ : HUS;
  // staged coefficient inputs (split form, first tile only) share red's space
  constexpr int CF = 0, CH = 2 * MM + 2, CC = CH + MM, CSN = CC + MM, CG = CSN + MM;
  static_assert(CG + MM + 1 <= 4 * NS, "coefficient staging exceeds the reduction buffer");
  __shared__ double L2[H2::SZ];
  __shared__ double L1[L1SZ];
  __shared__ double red[4 * NS];
  // coefficients zero beyond j (see k_extend); cY_j kept apart
  __shared__ double sY[MM], cY[MM];
  __shared__ double sCyj;
  __shared__ double sAlpha;
  __shared__ int sFlag;
  const Geo g = me.job.g;
  const BasisBuf<T> VB((const T*)me.job.V, g, me.job.m);
  const int kU = me.job.m + (j & 1), kUn = me.job.m + ((j + 1) & 1);
  const bool writer = me.job.lblk == 0;
  const int c = j - 1;
  double ainv = 0.0, sYl = 0.0, cYl = 0.0;
  double stA = 0.0, stB = 0.0, hs[SPLIT ? HT : 1];
  StopState ss{};
  if constexpr (!SPLIT) {
    // coefficients from coef(j)
    ainv = 1.0 / C->alpha;
    sYl = tid < j ? C->sY[tid] : 0.0;
    cYl = tid <= j ? C->cY[tid] : 0.0;
  } else {
    // inputs of the coefficient update, loaded unconditionally at clamped
    // indices: A = column sums (2j+2) then h_{j-1} (j); B (used by the
    // system's first workgroup only) = cs, sn (j-1 each) then g (j); the
    // Hessenberg columns 0..j-2
    const int nA = 3 * j + 2, nB = 3 * j - 2, hlim = j > 1 ? hu_off(j - 1) : 0;
    const int a = tid < nA ? tid : 0;
    const gptr<const double> pa = a < 2 * j + 2 ? C->sums + a : C->hprev[j & 1] + (a - (2 * j + 2));
    stA = *pa;
    const int b = tid < nB ? tid : 0;
    const gptr<const double> pb = b < c ? C->cs + b : (b < 2 * c ? C->sn + (b - c) : C->g + (b - 2 * c));
    stB = *pb;
#pragma unroll
    for (int k = 0; k < HT; ++k) {
      const int e = tid + kBlock * k;
      hs[k] = C->Hu[e < hlim ? e : 0];
    }
    ss = stop_state(C);
  }
  double accw[NCH + 1];
#pragma unroll
  for (int cc = 0; cc <= NCH; ++cc) accw[cc] = 0.0;
  // the first tile is peeled off the tile loop (a straight-line copy of the
  // body), so that no loop-carried register reuse makes its data loads wait
  // for the coefficient inputs issued before them
  auto sweep = [&](const int tile, auto first_c) -> bool {
    constexpr bool FIRST = decltype(first_c)::value;
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
    // ---- every global load of the tile is issued here, before any is used,
    // unconditionally: indices are clamped into valid memory (basis slots
    // >= j re-read v_{j-1}, points outside the grid read element 0) and the
    // extra values are never used, so no branch splits the loads
    T hv[HPT];                                        // u_j with a two-point halo
    bool hin[HPT];
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
      const int e = threadIdx.x + kBlock * h;
      const int lx = e % H2::X, r = e / H2::X, ly = r % H2::Y, lz = r / H2::Y;
      const int gx = ox + lx - 2, gy = oy + ly - 2, gz = TL::DIM == 3 ? oz + lz - 2 : 0;
      hin[h] = e < H2::SZ && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 &&
               gz < g.nz;
      hv[h] = VB.load(kU, hin[h] ? (unsigned)(((long long)gz * g.ny + gy) * g.nx + gx) : 0u);
    }
    long long pp[PPT];
    bool ok[PPT];
    int q2[PPT], q1[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      ok[i] = pr.valid;
      pp[i] = pr.valid ? pr.p : 0;
      q2[i] = H2::at(pr.qx, pr.qy, pr.qz);
      q1[i] = H1::at(pr.qx, pr.qy, pr.qz);
    }
    int rq[RPT][3];
    bool rin[RPT];
    long long rp[RPT];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int e = threadIdx.x + kBlock * rr;
      ring_point<TL>(e < RS ? e : 0, rq[rr][0], rq[rr][1], rq[rr][2]);
      const int gx = ox + rq[rr][0], gy = oy + rq[rr][1], gz = oz + rq[rr][2];
      rin[rr] = e < RS && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
      rp[rr] = rin[rr] ? ((long long)gz * g.ny + gy) * g.nx + gx : 0;
    }
    T vr[MM][PPT];                                    // basis at this thread's points
    T vg[MM][RPT];                                    // basis at this thread's ring points
    // padded slots: v_{j-1}, or at j = 0 (no basis vector written yet in
    // this cycle) the direction u_j itself
    const int jl = j > 0 ? j - 1 : kU;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
      const int kk = k < j ? k : jl;
#pragma unroll
      for (int i = 0; i < PPT; ++i) vr[k][i] = VB.load(kk, (unsigned)pp[i]);
#pragma unroll
      for (int rr = 0; rr < RPT; ++rr) vg[k][rr] = VB.load(kk, (unsigned)rp[rr]);
    }
    // (the previous tile's readers of L2/L1 are done)
    __syncthreads();
    // ---- the step's coefficients first (first tile): their inputs were
    // loaded before the tile's data, so the update runs while the tile's
    // loads are in flight
    if constexpr (FIRST) {
      if constexpr (SPLIT) {
        // the coefficient inputs go to LDS before any branch, so that waiting
        // for them does not wait for the tile's data loads
        const int nA = 3 * j + 2, nB = 3 * j - 2, hlim = j > 1 ? hu_off(j - 1) : 0;
        if (tid < nA) red[tid < 2 * j + 2 ? CF + tid : CH + tid - (2 * j + 2)] = stA;
        if (tid < nB) red[tid < c ? CC + tid : (tid < 2 * c ? CSN + tid - c : CG + tid - 2 * c)] = stB;
#pragma unroll
        for (int k = 0; k < HT; ++k) {
          const int e = tid + kBlock * k;
          if (e < hlim) L1[e] = hs[k];
        }
      }
      if constexpr (!SPLIT) {
        if (tid < MM) {
          sY[tid] = tid < j ? sYl : 0.0;
          cY[tid] = tid < j ? cYl : 0.0;
        }
        if (tid == j) sCyj = cYl;
      } else {
        // ---- coefficient update of step j (this workgroup's own copy; the
        // system's first workgroup also advances the system's state)
        double* fin = red + CF;
        __syncthreads();
        double rot = 0.0, gnew = 0.0;
        if (tid < 64) {
          const int lane = tid;
          const StepCoef q = coef_project(fin, L1, j, red[CH + (lane < j ? lane : 0)]);
          if (lane < MM) {
            sY[lane] = lane < j ? q.si : 0.0;
            cY[lane] = lane < j ? q.cy : 0.0;
          }
          if (lane == j) sCyj = q.cy;
          if (lane == 0) sAlpha = q.alpha;
          int fl = 0;
          if (writer) {
            if (j > 0)
              fl = coef_rotate(C, q, j, ss, red[CC + (lane < c ? lane : 0)],
                               red[CSN + (lane < c ? lane : 0)], red[CG + c], rot, gnew);
            else if (lane == 0)
              C->hprev[1][0] = q.h;
          }
          if (lane == 0) sFlag = fl;
        }
        __syncthreads();
        // only the system's first workgroup can stop here; the others finish
        // the sweep, whose results no later step reads
        const int fl = sFlag;
        if (fl != 0) {
          if (fl == 2 && tid == 0) finish_rhs(C);
          if (fl == 1) {
            // end of the cycle: R in L1's space (columns 0..c-1 from memory,
            // column c from wavefront 0's registers), then y
            const int rlim = r_off(c);
            double rv[RT];
#pragma unroll
            for (int k = 0; k < RT; ++k) {
              const int e = tid + kBlock * k;
              rv[k] = C->R[e < rlim ? e : 0];
            }
#pragma unroll
            for (int k = 0; k < RT; ++k) {
              const int e = tid + kBlock * k;
              if (e < rlim) L1[e] = rv[k];
            }
            if (tid <= c) L1[rlim + tid] = rot;
            __syncthreads();
            if (tid < 64) back_substitute(C, L1, j, tid < j ? (tid == c ? gnew : red[CG + tid]) : 0.0);
          }
          return false;
        }
        ainv = 1.0 / sAlpha;
      }
    }
    // ---- stage u_j
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
      const int e = threadIdx.x + kBlock * h;
      if (e < H2::SZ) L2[e] = hin[h] ? (double)hv[h] : 0.0;
    }
    __syncthreads();
    const double cyj = sCyj;
    // u_{j+1} on the ring (zero outside the grid)
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
      const int e = threadIdx.x + kBlock * rr;
      if (e < RS) {
        double un = 0.0;
        if (rin[rr]) {
          const int i2 = H2::at(rq[rr][0], rq[rr][1], rq[rr][2]);
          const double uu = L2[i2];
          const double ww = stencil_at<TL::DIM>(L2, g, i2, H2::X, H2::X * H2::Y);
          double a = 0.0, b = 0.0;
#pragma unroll
          for (int k = 0; k < MM; ++k) {
            a = fma((double)vg[k][rr], sY[k], a);
            b = fma((double)vg[k][rr], cY[k], b);
          }
          T vj, unT;
          extend_point<T>(uu, ww, a, b, ainv, cyj, vj, unT);
          un = (double)unT;
        }
        L1[H1::at(rq[rr][0], rq[rr][1], rq[rr][2])] = un;
      }
    }
    // v_j and u_{j+1} at this thread's points
    double vjd[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      vjd[i] = 0.0;
      double un = 0.0;
      if (ok[i]) {
        const double uu = L2[q2[i]];
        const double ww = stencil_at<TL::DIM>(L2, g, q2[i], H2::X, H2::X * H2::Y);
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int k = 0; k < MM; ++k) {
          a = fma((double)vr[k][i], sY[k], a);
          b = fma((double)vr[k][i], cY[k], b);
        }
        T vj, unT;
        extend_point<T>(uu, ww, a, b, ainv, cyj, vj, unT);
        VB.store(j, (unsigned)pp[i], vj);
        VB.store(kUn, (unsigned)pp[i], unT);
        vjd[i] = (double)vj;
        un = (double)unT;
      }
      L1[q1[i]] = un;
    }
    __syncthreads();
    // products for step j+1, folded across the wavefront per chunk
    double u1[PPT], w1[PPT];
    double last[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      u1[i] = ok[i] ? L1[q1[i]] : 0.0;
      w1[i] = ok[i] ? stencil_at<TL::DIM>(L1, g, q1[i], H1::X, H1::X * H1::Y) : 0.0;
      last[0] = fma(u1[i], u1[i], last[0]);
      last[1] = fma(u1[i], w1[i], last[1]);
      last[2] = fma(vjd[i], u1[i], last[2]);
      last[3] = fma(vjd[i], w1[i], last[3]);
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c)
      if (KC * c < j) {
        double prod[16];
#pragma unroll
        for (int q = 0; q < KC; ++q) {
          prod[q] = 0.0;
          prod[KC + q] = 0.0;
#pragma unroll
          for (int i = 0; i < PPT; ++i) {
            prod[q] = fma((double)vr[KC * c + q][i], u1[i], prod[q]);
            prod[KC + q] = fma((double)vr[KC * c + q][i], w1[i], prod[KC + q]);
          }
        }
        accw[c] += rs16(prod);
      }
    accw[NCH] += rs4(last);
    return true;
  };
  if (!sweep(me.job.t0, std::true_type{})) return;
  for (int tile = me.job.t0 + 1; tile < me.job.t1; ++tile) sweep(tile, std::false_type{});
  // per-wavefront sums -> LDS -> block sums -> this workgroup's partials
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if ((lane & 3) == 0) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) red[wave * NS + 16 * c + rs16_slot(lane)] = accw[c];
  }
  if ((lane & 15) == 0) red[wave * NS + 16 * NCH + rs4_slot(lane)] = accw[NCH];
  __syncthreads();
  const int jn = j + 1;
  for (int k = threadIdx.x; k < NS; k += kBlock) {
    int col = -1;
    if (k < 16 * NCH) {
      const int q = k & 15, bi = KC * (k >> 4) + (q & 7);
      if (bi < j) col = q < KC ? bi : jn + bi;
    } else {
      const int f = k - 16 * NCH;                 // nu, mu, s_j, t_j
      col = f == 0 ? 2 * jn : (f == 1 ? 2 * jn + 1 : (f == 2 ? j : jn + j));
    }
    if (col >= 0)
      gmem(me.job.part)[(size_t)col * g.nblk + me.job.lblk] =
          ((red[k] + red[NS + k]) + red[2 * NS + k]) + red[3 * NS + k];
  }
}

// x += V_k y (FP64 accumulation into the FP64 iterate); MM >= k.
template <class T, class TL, int MM>
__global__ __launch_bounds__(kBlock) void k_update(const Job* jobs, const SysDesc* sd) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (!cycle_tail_pending(C)) return;
  constexpr int PPT = TL::PPT;
  __shared__ double ys[MM];
  const int k = C->k;
  for (int l = threadIdx.x; l < MM; l += kBlock) ys[l] = l < k ? C->y[l] : 0.0;
  __syncthreads();
  const Geo g = me.job.g;
  const BasisBuf<T> VB((const T*)me.job.V, g, me.job.m);
  const Rsrc rx = vec_rsrc(C->x0 + (size_t)C->rhs * g.n, g.n);
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
    long long pp[PPT];
    bool ok[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      ok[i] = pr.valid;
      pp[i] = pr.valid ? pr.p : 0;
    }
    constexpr int KC = 8, NCH = MM / KC;
    T vb[2][KC][PPT];
    load_basis_chunk<KC, PPT, T>(vb[0], VB, pp, 0, k, me.job.m);
    double acc[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) acc[i] = buf_load<double>(rx, (unsigned)pp[i]);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      // the scheduler keeps each chunk's loads here (one chunk ahead), not
      // hoisted to the top, so only two chunks occupy registers
      __builtin_amdgcn_sched_barrier(0);
      if (c + 1 < NCH && KC * (c + 1) < k)
        load_basis_chunk<KC, PPT, T>(vb[(c + 1) & 1], VB, pp, KC * (c + 1), k, me.job.m);
      if (KC * c < k) {
#pragma unroll
        for (int q = 0; q < KC; ++q)
#pragma unroll
          for (int i = 0; i < PPT; ++i) acc[i] = fma(ys[KC * c + q], (double)vb[c & 1][q][i], acc[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i)
      if (ok[i]) buf_store(rx, (unsigned)pp[i], acc[i]);
  }
}

// y = A u (standalone operator application): workgroup b takes an equal
// share of the tiles.
template <class TL>
__global__ __launch_bounds__(kBlock) void k_apply(Geo g, const double* u, double* y) {
  __shared__ double L[TL::LSZ];
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int t0 = (int)((long long)b * g.ntiles / gridDim.x);
  const int t1 = (int)((long long)(b + 1) * g.ntiles / gridDim.x);
  for (int tile = t0; tile < t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
    __syncthreads();
    load_tile<TL>(L, u, g, ox, oy, oz);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TL::PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      if (pr.valid) y[pr.p] = stencil<TL>(L, g, pr.qx, pr.qy, pr.qz);
    }
  }
}

}  // namespace mlg
