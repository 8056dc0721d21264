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

#include "common.h"

namespace mlg {

enum Phase { PH_INIT = 0, PH_RUN = 1, PH_ZERO = 2, PH_DONE = 3 };

// Statistics of one right-hand side (copied to the host at the end).
struct Summary {
  int status;
  int cycles;
  long long iters;
  double relres_init, relres_first, relres_est, relres_true;
};

struct Ctrl {
  Summary s;            // statistics of the current right-hand side
  int phase;
  int cycle_end;        // the current cycle stopped stepping
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
                        // [1]: progress count (Arnoldi columns + finished RHS)
  double hprev[kMaxRestart + 1];           // first-projection coefficients h_{j-1}
  double sY[kMaxRestart + 1];              // second-projection coefficients (extend)
  double cY[kMaxRestart + 1];              // coefficients of V_j in u_{j+1} (extend)
  double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart];
  double Hu[kMaxRestart * (kMaxRestart + 1)];  // Hessenberg, column c at Hu[c*(kMaxRestart+1)]
  double R[kMaxRestart * kMaxRestart];         // rotated Hessenberg, column c at R[c*kMaxRestart]
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

// One workgroup's share of a launch: a contiguous tile range of one system.
struct Job {
  int sys;
  int t0, t1;
  int lblk;       // index of this workgroup among its system's workgroups
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

// This workgroup's job and system.
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

// Block sums of the live slots of acc (slot k lands in column col(k)); each
// workgroup writes its own entry of every live partial column.  Per chunk of
// 16 slots a wavefront transposes its lanes' values through LDS (tr: 64 x 17
// doubles per wavefront), four lanes sum 16 lanes each in a fixed order and
// two lane exchanges combine them -- the same sums in every lane, so the
// result is bitwise reproducible; then the four wavefronts are added.
constexpr int kTrPitch = 17;
template <int NV, class Live, class Col>
__device__ __forceinline__ void store_partials(const double (&acc)[NV], Live live, Col col,
                                               double* red, double* tr, gptr<double> part, int nblk,
                                               int lblk) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* trw = tr + wave * 64 * kTrPitch;
  const int sl = lane & 15, pq = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < NV; k0 += 16) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (k0 + q < NV) any = any || live(k0 + q);
    if (!any) continue;
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (k0 + q < NV) trw[lane * kTrPitch + q] = acc[k0 + q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) v += trw[(pq * 16 + i) * kTrPitch + sl];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (pq == 0 && k0 + sl < NV && live(k0 + sl)) red[wave * NV + k0 + sl] = v;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += kBlock)
    if (live(k))
      part[(size_t)col(k) * nblk + lblk] =
          ((red[k] + red[NV + k]) + red[2 * NV + k]) + red[3 * NV + k];
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

// ---------------------------------------------------------------- kernels

// begin: initial guess of a system that starts a right-hand side other than
// its first (whose guess the caller provides): zero, or the previous solution.
template <class TL>
__global__ __launch_bounds__(kBlock) void k_begin(const Job* jobs, const SysDesc* sd) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_INIT || C->rhs == 0) return;
  const Geo g = me.S->g;
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
template <class TL, bool INIT>
__global__ __launch_bounds__(kBlock) void k_resid(const Job* jobs, const SysDesc* sd) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != (INIT ? PH_INIT : PH_RUN)) return;
  __shared__ double L[TL::LSZ];
  __shared__ double red[4 * 2];
  __shared__ double tr[4 * 64 * kTrPitch];
  const Geo g = me.S->g;
  gptr<const double> b = gmem(C->b0) + (size_t)C->rhs * g.n;
  const gptr<double> x = gmem(C->x0) + (size_t)C->rhs * g.n;
  gptr<double> r = gmem(me.S->r);
  double acc[2] = {0.0, 0.0};
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
    __syncthreads();
    load_tile<TL>(L, x, g, ox, oy, oz);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TL::PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      if (pr.valid) {
        const double bi = b[pr.p];
        const double ri = bi - stencil<TL>(L, g, pr.qx, pr.qy, pr.qz);
        r[pr.p] = ri;
        acc[0] += ri * ri;
        acc[1] += bi * bi;
      }
    }
  }
  store_partials<2>(acc, [](int k) { return INIT || k == 0; }, [](int k) { return k; }, red, tr,
                    gmem(me.S->part), g.nblk, me.job.lblk);
}

// beta = |r| (and |b| when starting): one workgroup per system.
template <bool INIT>
__global__ __launch_bounds__(kReduceThreads) void k_rsum(const SysDesc* sd) {
  const SysDesc* S = sd + blockIdx.x;
  const gptr<Ctrl> C = gmem(S->C);
  if (C->phase != (INIT ? PH_INIT : PH_RUN)) return;
  __shared__ double fin[2];
  reduce_partials(gmem((const double*)S->part), S->g.nblk, INIT ? 2 : 1, fin);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(fin[0]);
  C->beta = beta;
  C->g[0] = beta;
  C->k = 0;
  C->cycle_end = 0;
  if (INIT) {
    const double bnorm = sqrt(fin[1]);
    C->s.status = MLG_OK;
    C->s.cycles = 0;
    C->s.iters = 0;
    C->bnorm = bnorm;
    C->tol_abs = C->rtol * bnorm;
    if (bnorm == 0.0) {                     // A x = 0: x = 0 (written by start)
      C->s.relres_init = C->s.relres_first = C->s.relres_est = C->s.relres_true = 0.0;
      C->phase = PH_ZERO;
      return;
    }
    const double rr = beta / bnorm;
    C->s.relres_init = rr;
    C->s.relres_first = rr;
    C->s.relres_est = rr;
    C->s.relres_true = rr;
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
  }
}

// start: u_0 = r (in the basis precision T); x = 0 for a zero right-hand side.
template <class T, class TL>
__global__ __launch_bounds__(kBlock) void k_start(const Job* jobs, const SysDesc* sd) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_RUN && C->phase != PH_ZERO) return;
  const bool zero = C->phase == PH_ZERO;
  const Geo g = me.S->g;
  gptr<T> U0 = gmem((T*)me.S->V) + (size_t)C->m * g.ldv;
  const gptr<double> r = gmem(me.S->r);
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
// The basis is read in chunks of KC vectors whose loads are all issued before
// any is consumed (indices clamped into the live range, so no branch splits a
// chunk), which keeps KC x PPT loads in flight per lane.
template <class T, class TL, int MM>
__global__ __launch_bounds__(kBlock) void k_dots(const Job* jobs, const SysDesc* sd, int j) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_RUN || C->cycle_end) return;
  constexpr int NV = 2 * MM + 2;     // s in 0..MM-1, t in MM..2MM-1, nu, mu
  constexpr int PPT = TL::PPT;
  constexpr int KC0 = PPT >= 4 ? 8 : (PPT == 2 ? 16 : 32);
  constexpr int KC = KC0 < MM ? KC0 : MM;
  __shared__ double L[TL::LSZ];
  __shared__ double red[4 * NV];
  __shared__ double tr[4 * 64 * kTrPitch];
  const Geo g = me.S->g;
  const gptr<const T> V = gmem((const T*)me.S->V);
  const gptr<const T> U = V + (size_t)(C->m + (j & 1)) * g.ldv;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
    __syncthreads();
    load_tile<TL>(L, U, g, ox, oy, oz);
    __syncthreads();
    double uu[PPT], ww[PPT];
    long long pp[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      pp[i] = pr.valid ? pr.p : 0;
      uu[i] = pr.valid ? centre<TL>(L, pr.qx, pr.qy, pr.qz) : 0.0;
      ww[i] = pr.valid ? stencil<TL>(L, g, pr.qx, pr.qy, pr.qz) : 0.0;
      acc[2 * MM] += uu[i] * uu[i];
      acc[2 * MM + 1] += uu[i] * ww[i];
    }
#pragma unroll
    for (int kc = 0; kc < MM; kc += KC) {
      if (kc >= j) break;
      double v[KC][PPT];
#pragma unroll
      for (int q = 0; q < KC; ++q) {
        const int ks = kc + q < j ? kc + q : j - 1;
#pragma unroll
        for (int i = 0; i < PPT; ++i) v[q][i] = (double)V[(size_t)ks * g.ldv + pp[i]];
      }
#pragma unroll
      for (int q = 0; q < KC; ++q)
        if (kc + q < j && kc + q < MM) {
#pragma unroll
          for (int i = 0; i < PPT; ++i) {
            acc[kc + q] += v[q][i] * uu[i];
            acc[MM + kc + q] += v[q][i] * ww[i];
          }
        }
    }
  }
  store_partials<NV>(
      acc, [j](int k) { return (k < MM && k < j) || (k >= MM && k < MM + j) || k >= 2 * MM; },
      [j](int k) { return k < MM ? k : (k < 2 * MM ? j + (k - MM) : 2 * j + (k - 2 * MM)); }, red,
      tr, gmem(me.S->part), g.nblk, me.job.lblk);
}

// coef(j): one workgroup per system.  All threads stage the small per-cycle
// state into LDS while they sum the partials; wavefront 0 then completes
// Hessenberg column j-1 (second projection), applies the Givens rotations
// (lane-parallel data, uniform loop with lane broadcasts), tests for the end
// of the cycle (back substitution if so) and prepares the coefficients of
// extend(j).  For a zero right-hand side, coef(0) ends the RHS.
__global__ __launch_bounds__(kReduceThreads) void k_coef(const SysDesc* sd, int j) {
  const SysDesc* S = sd + blockIdx.x;
  const gptr<Ctrl> C = gmem(S->C);
  if (j == 0 && C->phase == PH_ZERO) {
    if (threadIdx.x == 0) finish_rhs(C);
    return;
  }
  if (C->phase != PH_RUN || C->cycle_end) return;
  constexpr int LDH = kMaxRestart + 1;
  __shared__ double fin[2 * kMaxRestart + 2];
  // Hessenberg columns (for z) or, at the end of a cycle, the rotated R
  __shared__ double HuS[kMaxRestart * LDH];
  double* Rs = HuS;
  // Hessenberg columns 0..j-2 (rows <= c+1) for z = Hbar s
  for (int e = threadIdx.x; e < (j > 1 ? (j - 1) * LDH : 0); e += kReduceThreads)
    HuS[e] = C->Hu[e];
  // wavefront 0's per-row state, loaded together with the partials
  const int lane = threadIdx.x;
  const bool w0 = threadIdx.x < 64;
  const int c = j - 1;
  const double hpi = (w0 && lane < j) ? C->hprev[lane] : 0.0;
  const double csl = (w0 && lane < c) ? C->cs[lane] : 0.0;
  const double snl = (w0 && lane < c) ? C->sn[lane] : 0.0;
  const double gc = (w0 && j > 0) ? C->g[c] : 0.0;
  const double glane = (w0 && lane < j) ? C->g[lane] : 0.0;
  reduce_partials(gmem((const double*)S->part), S->g.nblk, 2 * j + 2, fin);
  if (!w0) return;
  // ---- wavefront 0: lane i owns row i (j <= 64)
  const double nu = fin[2 * j], mu = fin[2 * j + 1];
  const double si = lane < j ? fin[lane] : 0.0;
  const double ti = lane < j ? fin[j + lane] : 0.0;
  const double ss = wave_sum(si * si), hh = wave_sum(hpi * hpi), st = wave_sum(si * ti);
  double alpha;
  if (j == 0) {
    alpha = sqrt(nu);
  } else {
    // |u_j - V s|^2 = |u_j|^2 - |s|^2 (V orthonormal)
    alpha = sqrt(fmax(nu - ss, 0.0));
    // Hessenberg column c: first + second projection, subdiagonal alpha
    const double coli = lane < j ? hpi + si : (lane == j ? alpha : 0.0);
    if (lane <= j) {
      C->Hu[(size_t)c * LDH + lane] = coli;
      HuS[(size_t)c * LDH + lane] = coli;
    }
    // rotations G_0..G_{c-1}: carry the running entry down the column
    double carry = lane_bcast(coli, 0);
    double rot = 0.0;                 // rotated entry of this lane's row
    for (int i = 0; i < c; ++i) {
      const double a = carry, bb = lane_bcast(coli, i + 1);
      const double ci = lane_bcast(csl, i), sni = lane_bcast(snl, i);
      if (lane == i) rot = ci * a + sni * bb;
      carry = -sni * a + ci * bb;
    }
    const double den = hypot(carry, alpha);
    double cc = 1.0, sn = 0.0;
    if (den != 0.0) {
      cc = carry / den;
      sn = alpha / den;
    }
    if (lane == c) rot = den;
    if (lane <= c) C->R[c * kMaxRestart + lane] = rot;
    const double est = fabs(sn * gc);
    const long long iters = C->s.iters + 1;
    // breakdown: the new direction is rounding noise relative to A v_{j-1}
    // (|A v_{j-1}|^2 = |u_j|^2 + |h_{j-1}|^2)
    const bool breakdown = alpha <= 1e-14 * sqrt(nu + hh);
    const bool bad = !isfinite(alpha) || !isfinite(est);
    const bool stop = bad || iters >= C->limit || breakdown ||
                      (!C->fixed && est <= C->tol_abs) || j == C->m;
    if (lane == 0) {
      C->cs[c] = cc;
      C->sn[c] = sn;
      C->g[c + 1] = -sn * gc;
      C->g[c] = cc * gc;
      C->s.iters = iters;
      C->k = j;
      C->s.relres_est = est / C->bnorm;
      atomicAdd(C->done + 1, 1u);
      if (bad) {
        C->s.status = MLG_ERR_NONFINITE;
        finish_rhs(C);
      }
    }
    if (bad) return;
    if (stop) {
      // back substitution R y = g (R: j x j upper triangular), row i on lane i
      for (int e = lane; e < j * kMaxRestart; e += 64) Rs[e] = C->R[e];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      const double gl = lane < j ? (lane == c ? cc * gc : glane) : 0.0;
      double accl = 0.0, yl = 0.0;
      for (int i = j - 1; i >= 0; --i) {
        const double yi = lane_bcast((gl - accl) / (lane < j ? Rs[lane * kMaxRestart + lane] : 1.0), i);
        if (lane == i) yl = yi;
        if (lane < i) accl += Rs[i * kMaxRestart + lane] * yi;
      }
      if (lane < j) C->y[lane] = yl;
      if (lane == 0) C->cycle_end = 1;
      return;
    }
  }
  // h_i = v_i^T A v_j with A v_j = (w - V_j z) / alpha, z = Hbar_{j-1} s
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  double z = 0.0;
  if (lane <= j)
    for (int c = (lane > 0 ? lane - 1 : 0); c < j; ++c) z += HuS[(size_t)c * LDH + lane] * fin[c];
  if (lane <= j) {
    const double vw = lane < j ? ti : (mu - st) / alpha;
    const double h = (vw - z) / alpha;
    C->hprev[lane] = h;
    C->cY[lane] = z / alpha + h;
    C->sY[lane] = si;
  }
  if (lane == 0) C->alpha = alpha;
}

// extend(j): v_j = (u_j - V_{j-1} s) / alpha, u_{j+1} = w/alpha - V_j cY.
template <class T, class TL>
__global__ __launch_bounds__(kBlock) void k_extend(const Job* jobs, const SysDesc* sd, int j) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_RUN || C->cycle_end) return;
  __shared__ double L[TL::LSZ];
  __shared__ double sY[kMaxRestart + 1], cY[kMaxRestart + 1];
  for (int k = threadIdx.x; k <= j; k += kBlock) {
    sY[k] = C->sY[k];
    cY[k] = C->cY[k];
  }
  const Geo g = me.S->g;
  const gptr<T> V = gmem((T*)me.S->V);
  const gptr<const T> U = V + (size_t)(C->m + (j & 1)) * g.ldv;
  const gptr<T> Unext = V + (size_t)(C->m + ((j + 1) & 1)) * g.ldv;
  const double ainv = 1.0 / C->alpha;
  constexpr int PPT = TL::PPT;
  constexpr int KC = PPT >= 4 ? 8 : (PPT == 2 ? 16 : 32);
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
    __syncthreads();
    load_tile<TL>(L, U, g, ox, oy, oz);
    __syncthreads();
    double uu[PPT], ww[PPT], a[PPT], bs[PPT];
    long long pp[PPT];
    bool ok[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      ok[i] = pr.valid;
      pp[i] = pr.valid ? pr.p : 0;
      uu[i] = pr.valid ? centre<TL>(L, pr.qx, pr.qy, pr.qz) : 0.0;
      ww[i] = pr.valid ? stencil<TL>(L, g, pr.qx, pr.qy, pr.qz) : 0.0;
      a[i] = 0.0;
      bs[i] = 0.0;
    }
    // all loads of a chunk are issued before any is used (clamped indices)
    for (int kc = 0; kc < j; kc += KC) {
      double v[KC][PPT];
#pragma unroll
      for (int q = 0; q < KC; ++q) {
        const int ks = kc + q < j ? kc + q : j - 1;
#pragma unroll
        for (int i = 0; i < PPT; ++i) v[q][i] = (double)V[(size_t)ks * g.ldv + pp[i]];
      }
#pragma unroll
      for (int q = 0; q < KC; ++q)
        if (kc + q < j) {
          const double sq = sY[kc + q], cq = cY[kc + q];
#pragma unroll
          for (int i = 0; i < PPT; ++i) {
            a[i] += v[q][i] * sq;
            bs[i] += v[q][i] * cq;
          }
        }
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i)
      if (ok[i]) {
        const T vj = (T)((uu[i] - a[i]) * ainv);
        V[(size_t)j * g.ldv + pp[i]] = vj;
        Unext[pp[i]] = (T)(ww[i] * ainv - bs[i] - cY[j] * (double)vj);
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
template <class T, class TL, int MM>
__global__ __launch_bounds__(kBlock) void k_step(const Job* jobs, const SysDesc* sd, int j) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_RUN || C->cycle_end) return;
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
  __shared__ double L2[H2::SZ];
  __shared__ double L1[H1::SZ];
  __shared__ double red[4 * NS];
  __shared__ double sY[MM], cY[MM];
  for (int k = threadIdx.x; k <= j; k += kBlock) {
    if (k < j) sY[k] = C->sY[k];
    cY[k] = C->cY[k];
  }
  const Geo g = me.S->g;
  const gptr<T> V = gmem((T*)me.S->V);
  const gptr<const T> U = V + (size_t)(C->m + (j & 1)) * g.ldv;
  const gptr<T> Unext = V + (size_t)(C->m + ((j + 1) & 1)) * g.ldv;
  const double ainv = 1.0 / C->alpha;
  double accw[NCH + 1];
#pragma unroll
  for (int c = 0; c <= NCH; ++c) accw[c] = 0.0;
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
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
      hv[h] = U[hin[h] ? ((long long)gz * g.ny + gy) * g.nx + gx : 0];
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
    const int jl = j > 0 ? j - 1 : 0;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
      const gptr<const T> Vk = V + (size_t)(k < j ? k : jl) * g.ldv;
#pragma unroll
      for (int i = 0; i < PPT; ++i) vr[k][i] = Vk[pp[i]];
#pragma unroll
      for (int rr = 0; rr < RPT; ++rr) vg[k][rr] = Vk[rp[rr]];
    }
    // ---- stage u_j (the previous tile's readers of L2/L1 are done)
    __syncthreads();
#pragma unroll
    for (int h = 0; h < HPT; ++h) {
      const int e = threadIdx.x + kBlock * h;
      if (e < H2::SZ) L2[e] = hin[h] ? (double)hv[h] : 0.0;
    }
    __syncthreads();
    const double cyj = cY[j];
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
          for (int k = 0; k < MM; ++k)
            if (k < j) {
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
        for (int k = 0; k < MM; ++k)
          if (k < j) {
            a = fma((double)vr[k][i], sY[k], a);
            b = fma((double)vr[k][i], cY[k], b);
          }
        T vj, unT;
        extend_point<T>(uu, ww, a, b, ainv, cyj, vj, unT);
        V[(size_t)j * g.ldv + pp[i]] = vj;
        Unext[pp[i]] = unT;
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
  }
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
      gmem(me.S->part)[(size_t)col * g.nblk + me.job.lblk] =
          ((red[k] + red[NS + k]) + red[2 * NS + k]) + red[3 * NS + k];
  }
}

// x += V_k y (FP64 accumulation into the FP64 iterate).
template <class T, class TL>
__global__ __launch_bounds__(kBlock) void k_update(const Job* jobs, const SysDesc* sd) {
  const Mine me = mine(jobs, sd);
  const gptr<const Ctrl> C = gmem((const Ctrl*)me.S->C);
  if (C->phase != PH_RUN) return;
  __shared__ double ys[kMaxRestart];
  const int k = C->k;
  for (int l = threadIdx.x; l < k; l += kBlock) ys[l] = C->y[l];
  __syncthreads();
  const Geo g = me.S->g;
  const gptr<const T> V = gmem((const T*)me.S->V);
  gptr<double> x = gmem(C->x0) + (size_t)C->rhs * g.n;
  for (int tile = me.job.t0; tile < me.job.t1; ++tile) {
    int ox, oy, oz;
    tile_origin<TL>(g, tile, ox, oy, oz);
#pragma unroll
    for (int i = 0; i < TL::PPT; ++i) {
      auto pr = point<TL>(g, ox, oy, oz, i);
      if (pr.valid) {
        double s = x[pr.p];
        for (int l = 0; l < k; ++l) s += ys[l] * (double)V[(size_t)l * g.ldv + pr.p];
        x[pr.p] = s;
      }
    }
  }
}

// Replicate a system's state into `n` independent copies for kernel timing:
// each keeps the coefficients of the finished solve but is marked running
// with a zero tolerance, so every timed launch does its full work.
// descs[i] is the system descriptor pointing at copy i.
__global__ void k_bench_setup(const SysDesc* src_desc, SysDesc* descs, Ctrl* copies, int n) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const unsigned int* s = (const unsigned int*)src_desc->C;
  unsigned int* d = (unsigned int*)(copies + i);
  for (int e = threadIdx.x; e < (int)(sizeof(Ctrl) / 4); e += blockDim.x) d[e] = s[e];
  __syncthreads();
  if (threadIdx.x == 0) {
    Ctrl* c = copies + i;
    c->phase = PH_RUN;
    c->rhs = 0;
    c->cycle_end = 0;
    c->tol_abs = 0.0;
    c->limit = 1LL << 62;
    c->k = c->m;
    if (!(c->alpha > 0.0)) c->alpha = 1.0;
    descs[i] = *src_desc;
    descs[i].C = c;
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
