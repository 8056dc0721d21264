// Device side of restarted GMRES(m) on the zero-Dirichlet Poisson operator.
//
// One restart cycle (Section 1.3 of the paper: GMRES(k) minimises the residual
// over K_k(A, r0) and restarts from the last iterate) is a fixed sequence of
// kernels that a HIP graph replays:
//
//   start        v_0 = r / beta
//   proj1(j)     w = A v_j (LDS-tiled stencil), h1 = V_j^T w, |w|^2
//   proj2(j)     w' = w - V_j h1, h2 = V_j^T w', |w'|^2; last block: Hessenberg
//                column c = h1 + h2, H[j+1,j] = sqrt(|w'|^2 - |h2|^2), Givens
//                rotation, residual estimate, stop test, back substitution
//   proj3(j)     v_{j+1} = (w - V_j c) / H[j+1,j]
//   update       x += V_k y                     (FP64)
//   residual     r = b - A x, beta = |r|        (FP64), convergence test
//
// proj1..proj3 form classical Gram-Schmidt applied twice (CGS2); w is
// recomputed from the LDS tile of v_j in every pass instead of being stored.
// Every grid-wide sum is a fixed-order two-level reduction (DPP wave sums,
// per-block partials, last-block sum), so runs are bitwise reproducible.
// Device-side control state (Ctrl) lets every kernel of a replayed cycle
// become a no-op once the cycle or the solve has ended.
#pragma once

#include "common.h"

namespace mlg {

struct Summary {
  int finished;
  int status;
  int cycles;
  int k;
  long long iters;
  double relres_init, relres_first, relres_est, relres_true;
};

struct Ctrl {
  Summary s;
  unsigned int ticket[8];
  int cycle_end;
  int m;
  int fixed;
  int zero_rhs;
  long long limit;
  double rtol, bnorm, tol_abs, beta;
  double wnorm2, wp2, rho;
  const double* b;
  double* x;
  double h1[kMaxRestart + 2];
  double c[kMaxRestart + 2];
  double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart];
  double R[kMaxRestart * kMaxRestart];   // rotated Hessenberg, column j at R[j*kMaxRestart]
};

struct Geo {
  int nx, ny, nz;                  // nz = 1 in 2D
  int tcx, tcy, tcz, ntiles;       // tile counts per axis, total
  double cx, cy, cz;               // 1 / h^2 per axis
  long long n, ldv;                // points; stride between basis vectors
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

// Point i (0 <= i < PPT) of this thread inside a tile.
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

// Stage the tile of `src` plus a one-point halo into LDS as FP64; points
// outside the grid read as 0 (the Dirichlet boundary).
template <class TL, class S>
__device__ __forceinline__ void load_tile(double* L, const S* __restrict__ src, const Geo& g,
                                          int ox, int oy, int oz) {
  for (int e = threadIdx.x; e < TL::LSZ; e += kBlock) {
    int lx = e % TL::LX;
    int r = e / TL::LX;
    int ly = r % TL::LY;
    int lz = r / TL::LY;
    int gx = ox + lx - 1, gy = oy + ly - 1, gz = TL::DIM == 3 ? oz + lz - 1 : 0;
    double v = 0.0;
    if (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz)
      v = (double)src[((long long)gz * g.ny + gy) * g.nx + gx];
    L[e] = v;
  }
}

// (A u) at a tile point from the LDS tile: sum over axes of
// (2 u - u_minus - u_plus) / h^2.
template <class TL>
__device__ __forceinline__ double stencil(const double* L, const Geo& g, int qx, int qy, int qz) {
  const int i = ((TL::DIM == 3 ? qz + 1 : 0) * TL::LY + (qy + 1)) * TL::LX + (qx + 1);
  const double c = L[i];
  double a = (2.0 * c - L[i - 1] - L[i + 1]) * g.cx + (2.0 * c - L[i - TL::LX] - L[i + TL::LX]) * g.cy;
  if (TL::DIM == 3)
    a += (2.0 * c - L[i - TL::LX * TL::LY] - L[i + TL::LX * TL::LY]) * g.cz;
  return a;
}

// ---------------------------------------------------------------- kernels

__global__ void k_reset(Ctrl* C, const double* b, double* x, int m, int fixed, long long limit,
                        double rtol) {
  if (threadIdx.x < 8) C->ticket[threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    C->s.finished = 0;
    C->s.status = 0;
    C->s.cycles = 0;
    C->s.k = 0;
    C->s.iters = 0;
    C->s.relres_init = C->s.relres_first = C->s.relres_est = C->s.relres_true = 0.0;
    C->cycle_end = 0;
    C->m = m;
    C->fixed = fixed;
    C->zero_rhs = 0;
    C->limit = limit;
    C->rtol = rtol;
    C->b = b;
    C->x = x;
  }
}

// r = b - A x0, |r|^2, |b|^2; last block decides whether any cycle is needed.
template <class TL>
__global__ __launch_bounds__(kBlock) void k_init(Geo g, Ctrl* C, double* r, double* part) {
  __shared__ double L[TL::LSZ];
  __shared__ double red[4 * 2];
  const int tile = xcd_tile(blockIdx.x, g.ntiles);
  int ox, oy, oz;
  tile_origin<TL>(g, tile, ox, oy, oz);
  const double* b = C->b;
  const double* x = C->x;
  load_tile<TL>(L, x, g, ox, oy, oz);
  __syncthreads();
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < TL::PPT; ++i) {
    auto pr = point<TL>(g, ox, oy, oz, i);
    if (pr.valid) {
      double bi = b[pr.p];
      double ri = bi - stencil<TL>(L, g, pr.qx, pr.qy, pr.qz);
      r[pr.p] = ri;
      acc[0] += ri * ri;
      acc[1] += bi * bi;
    }
  }
  double tot;
  block_sums<2>(acc, 2, red, tot);
  if (threadIdx.x < 2) part[threadIdx.x * g.ntiles + blockIdx.x] = tot;
  if (!last_block(&C->ticket[0], g.ntiles)) return;
  __shared__ double fin[2];
  reduce_partials(part, g.ntiles, 2, fin);
  if (threadIdx.x == 0) {
    double beta = sqrt(fin[0]), bnorm = sqrt(fin[1]);
    C->bnorm = bnorm;
    C->beta = beta;
    C->tol_abs = C->rtol * bnorm;
    C->g[0] = beta;
    C->s.k = 0;
    C->cycle_end = 0;
    if (bnorm == 0.0) {
      C->zero_rhs = 1;
      C->s.finished = 1;
      return;
    }
    double rr = beta / bnorm;
    C->s.relres_init = rr;
    C->s.relres_first = rr;
    C->s.relres_est = rr;
    C->s.relres_true = rr;
    if (!isfinite(beta)) {
      C->s.status = MLG_ERR_NONFINITE;
      C->s.finished = 1;
    } else if ((!C->fixed && beta <= C->tol_abs) || beta == 0.0 || C->limit <= 0) {
      C->s.finished = 1;
    }
  }
}

// x = 0 when b = 0 (the solution of A x = 0).
template <class TL>
__global__ __launch_bounds__(kBlock) void k_zero_if_needed(Geo g, Ctrl* C) {
  if (!C->zero_rhs) return;
  double* x = C->x;
  const int tile = xcd_tile(blockIdx.x, g.ntiles);
  int ox, oy, oz;
  tile_origin<TL>(g, tile, ox, oy, oz);
#pragma unroll
  for (int i = 0; i < TL::PPT; ++i) {
    auto pr = point<TL>(g, ox, oy, oz, i);
    if (pr.valid) x[pr.p] = 0.0;
  }
}

// v_0 = r / beta (stored in the basis precision T).
template <class T, class TL>
__global__ __launch_bounds__(kBlock) void k_start(Geo g, Ctrl* C, const double* r, T* V) {
  if (C->s.finished) return;
  const double beta = C->beta;
  const int tile = xcd_tile(blockIdx.x, g.ntiles);
  int ox, oy, oz;
  tile_origin<TL>(g, tile, ox, oy, oz);
#pragma unroll
  for (int i = 0; i < TL::PPT; ++i) {
    auto pr = point<TL>(g, ox, oy, oz, i);
    if (pr.valid) V[pr.p] = (T)(r[pr.p] / beta);
  }
}

// proj1(j): w = A v_j, partial sums of V_j^T w and |w|^2.
template <class T, class TL, int MM>
__global__ __launch_bounds__(kBlock) void k_proj1(Geo g, Ctrl* C, const T* __restrict__ V,
                                                  double* part, int j) {
  if (C->s.finished || C->cycle_end) return;
  constexpr int NV = MM + 2;                      // dots 0..MM, norm in slot NV-1
  __shared__ double L[TL::LSZ];
  __shared__ double red[4 * NV];
  const int tile = xcd_tile(blockIdx.x, g.ntiles);
  int ox, oy, oz;
  tile_origin<TL>(g, tile, ox, oy, oz);
  load_tile<TL>(L, V + (size_t)j * g.ldv, g, ox, oy, oz);
  __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
#pragma unroll
  for (int i = 0; i < TL::PPT; ++i) {
    auto pr = point<TL>(g, ox, oy, oz, i);
    if (pr.valid) {
      const double w = stencil<TL>(L, g, pr.qx, pr.qy, pr.qz);
#pragma unroll
      for (int k = 0; k <= MM; ++k)
        if (k <= j) acc[k] += (double)V[(size_t)k * g.ldv + pr.p] * w;
      acc[NV - 1] += w * w;
    }
  }
  // block sums of the live slots (0..j and the norm)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k <= j || k == NV - 1) {
      double s = wave_sum(acc[k]);
      if (lane == 0) red[wave * NV + k] = s;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += kBlock)
    if (k <= j || k == NV - 1)
      part[(size_t)k * g.ntiles + blockIdx.x] =
          ((red[k] + red[NV + k]) + red[2 * NV + k]) + red[3 * NV + k];
  if (!last_block(&C->ticket[1], g.ntiles)) return;
  __shared__ double fin[NV];
  reduce_partials(part, g.ntiles, j + 1, fin);
  reduce_partials(part + (size_t)(NV - 1) * g.ntiles, g.ntiles, 1, fin + NV - 1);
  for (int k = threadIdx.x; k <= j; k += kBlock) C->h1[k] = fin[k];
  if (threadIdx.x == 0) C->wnorm2 = fin[NV - 1];
}

// proj2(j): second projection, then the Hessenberg column, Givens rotation,
// stop test and (at the end of the cycle) back substitution.
template <class T, class TL, int MM>
__global__ __launch_bounds__(kBlock) void k_proj2(Geo g, Ctrl* C, const T* __restrict__ V,
                                                  double* part, int j) {
  if (C->s.finished || C->cycle_end) return;
  constexpr int NV = MM + 2;
  __shared__ double L[TL::LSZ];
  __shared__ double red[4 * NV];
  __shared__ double hs[MM + 1];
  const int tile = xcd_tile(blockIdx.x, g.ntiles);
  int ox, oy, oz;
  tile_origin<TL>(g, tile, ox, oy, oz);
  for (int k = threadIdx.x; k <= j; k += kBlock) hs[k] = C->h1[k];
  load_tile<TL>(L, V + (size_t)j * g.ldv, g, ox, oy, oz);
  __syncthreads();
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
#pragma unroll
  for (int i = 0; i < TL::PPT; ++i) {
    auto pr = point<TL>(g, ox, oy, oz, i);
    if (pr.valid) {
      double vk[MM + 1];
      double wp = stencil<TL>(L, g, pr.qx, pr.qy, pr.qz);
#pragma unroll
      for (int k = 0; k <= MM; ++k)
        if (k <= j) vk[k] = (double)V[(size_t)k * g.ldv + pr.p];
#pragma unroll
      for (int k = 0; k <= MM; ++k)
        if (k <= j) wp -= vk[k] * hs[k];
#pragma unroll
      for (int k = 0; k <= MM; ++k)
        if (k <= j) acc[k] += vk[k] * wp;
      acc[NV - 1] += wp * wp;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k <= j || k == NV - 1) {
      double s = wave_sum(acc[k]);
      if (lane == 0) red[wave * NV + k] = s;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += kBlock)
    if (k <= j || k == NV - 1)
      part[(size_t)k * g.ntiles + blockIdx.x] =
          ((red[k] + red[NV + k]) + red[2 * NV + k]) + red[3 * NV + k];
  if (!last_block(&C->ticket[2], g.ntiles)) return;
  __shared__ double fin[NV];
  __shared__ double col[kMaxRestart + 2];
  reduce_partials(part, g.ntiles, j + 1, fin);
  reduce_partials(part + (size_t)(NV - 1) * g.ntiles, g.ntiles, 1, fin + NV - 1);
  if (threadIdx.x != 0) return;

  // ---- one thread: Hessenberg column, Givens, stop test
  double h2sq = 0.0;
  for (int i = 0; i <= j; ++i) {
    double h2 = fin[i];
    h2sq += h2 * h2;
    double ci = C->h1[i] + h2;
    C->c[i] = ci;
    col[i] = ci;
  }
  // |w''|^2 = |w'|^2 - |h2|^2 (w'' orthogonal to V_j)
  const double rho = sqrt(fmax(fin[NV - 1] - h2sq, 0.0));
  C->rho = rho;
  col[j + 1] = rho;
  for (int i = 0; i < j; ++i) {
    double a = col[i], bb = col[i + 1];
    col[i] = C->cs[i] * a + C->sn[i] * bb;
    col[i + 1] = -C->sn[i] * a + C->cs[i] * bb;
  }
  const double den = hypot(col[j], col[j + 1]);
  double cj = 1.0, sj = 0.0;
  if (den != 0.0) {
    cj = col[j] / den;
    sj = col[j + 1] / den;
  }
  C->cs[j] = cj;
  C->sn[j] = sj;
  col[j] = den;
  const double gj = C->g[j];
  C->g[j + 1] = -sj * gj;
  C->g[j] = cj * gj;
  for (int i = 0; i <= j; ++i) C->R[j * kMaxRestart + i] = col[i];

  const long long iters = C->s.iters + 1;
  C->s.iters = iters;
  C->s.k = j + 1;
  const double est = fabs(C->g[j + 1]);
  C->s.relres_est = est / C->bnorm;
  const bool breakdown = rho <= 1e-14 * sqrt(C->wnorm2);
  if (!isfinite(rho) || !isfinite(est)) {
    C->s.status = MLG_ERR_NONFINITE;
    C->s.finished = 1;
    C->cycle_end = 1;
    return;
  }
  const bool end = iters >= C->limit || breakdown || (!C->fixed && est <= C->tol_abs) ||
                   j + 1 == C->m;
  if (end) {
    C->cycle_end = 1;
    const int k = j + 1;
    for (int i = k - 1; i >= 0; --i) {
      double s = C->g[i];
      for (int l = i + 1; l < k; ++l) s -= C->R[l * kMaxRestart + i] * C->y[l];
      C->y[i] = s / C->R[i * kMaxRestart + i];
    }
  }
}

// proj3(j): v_{j+1} = (w - V_j c) / rho.
template <class T, class TL>
__global__ __launch_bounds__(kBlock) void k_proj3(Geo g, Ctrl* C, T* __restrict__ V, int j) {
  if (C->s.finished || C->cycle_end) return;
  __shared__ double L[TL::LSZ];
  __shared__ double cs[kMaxRestart + 1];
  const int tile = xcd_tile(blockIdx.x, g.ntiles);
  int ox, oy, oz;
  tile_origin<TL>(g, tile, ox, oy, oz);
  for (int k = threadIdx.x; k <= j; k += kBlock) cs[k] = C->c[k];
  const double rho = C->rho;
  load_tile<TL>(L, V + (size_t)j * g.ldv, g, ox, oy, oz);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < TL::PPT; ++i) {
    auto pr = point<TL>(g, ox, oy, oz, i);
    if (pr.valid) {
      double w = stencil<TL>(L, g, pr.qx, pr.qy, pr.qz);
      for (int k = 0; k <= j; ++k) w -= (double)V[(size_t)k * g.ldv + pr.p] * cs[k];
      V[(size_t)(j + 1) * g.ldv + pr.p] = (T)(w / rho);
    }
  }
}

// x += V_k y (FP64 accumulation into the FP64 iterate).
template <class T, class TL>
__global__ __launch_bounds__(kBlock) void k_update(Geo g, Ctrl* C, const T* __restrict__ V) {
  if (C->s.finished) return;
  __shared__ double ys[kMaxRestart];
  const int k = C->s.k;
  for (int l = threadIdx.x; l < k; l += kBlock) ys[l] = C->y[l];
  __syncthreads();
  double* x = C->x;
  const int tile = xcd_tile(blockIdx.x, g.ntiles);
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

// r = b - A x, beta = |r|; last block: acceptance test on the true residual
// and set-up of the next cycle.
template <class TL>
__global__ __launch_bounds__(kBlock) void k_residual(Geo g, Ctrl* C, double* r, double* part) {
  if (C->s.finished) return;
  __shared__ double L[TL::LSZ];
  __shared__ double red[4];
  const int tile = xcd_tile(blockIdx.x, g.ntiles);
  int ox, oy, oz;
  tile_origin<TL>(g, tile, ox, oy, oz);
  const double* b = C->b;
  load_tile<TL>(L, C->x, g, ox, oy, oz);
  __syncthreads();
  double acc[1] = {0.0};
#pragma unroll
  for (int i = 0; i < TL::PPT; ++i) {
    auto pr = point<TL>(g, ox, oy, oz, i);
    if (pr.valid) {
      double ri = b[pr.p] - stencil<TL>(L, g, pr.qx, pr.qy, pr.qz);
      r[pr.p] = ri;
      acc[0] += ri * ri;
    }
  }
  double tot;
  block_sums<1>(acc, 1, red, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
  if (!last_block(&C->ticket[3], g.ntiles)) return;
  __shared__ double fin[1];
  reduce_partials(part, g.ntiles, 1, fin);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(fin[0]);
  const int cycles = C->s.cycles + 1;
  C->s.cycles = cycles;
  const double rr = beta / C->bnorm;
  C->s.relres_true = rr;
  if (cycles == 1) C->s.relres_first = rr;
  if (!isfinite(beta)) {
    C->s.status = MLG_ERR_NONFINITE;
    C->s.finished = 1;
    return;
  }
  const bool conv = !C->fixed && beta <= C->tol_abs;
  if (conv || C->s.iters >= C->limit || beta == 0.0) {
    C->s.finished = 1;
    C->s.status = (conv || C->fixed || beta == 0.0) ? MLG_OK : MLG_NOT_CONVERGED;
    return;
  }
  C->beta = beta;
  C->g[0] = beta;
  C->s.k = 0;
  C->cycle_end = 0;
}

// Replicate the solver state into `copies` independent control blocks for
// kernel timing: each copy keeps the basis coefficients of the finished solve
// but is marked running with a zero tolerance, so every timed launch does its
// full work.
__global__ void k_bench_setup(const Ctrl* src, Ctrl* dst, int copies) {
  const int i = blockIdx.x;
  if (i >= copies) return;
  const unsigned int* s = (const unsigned int*)src;
  unsigned int* d = (unsigned int*)(dst + i);
  for (int e = threadIdx.x; e < (int)(sizeof(Ctrl) / 4); e += blockDim.x) d[e] = s[e];
  __syncthreads();
  if (threadIdx.x == 0) {
    Ctrl* c = dst + i;
    for (int t = 0; t < 8; ++t) c->ticket[t] = 0u;
    c->s.finished = 0;
    c->s.status = 0;
    c->cycle_end = 0;
    c->tol_abs = 0.0;
    c->limit = 1LL << 62;
    c->s.k = c->m;
    if (!(c->beta > 0.0)) c->beta = 1.0;
    if (!(c->rho > 0.0)) c->rho = 1.0;
  }
}

// y = A u (standalone operator application).
template <class TL>
__global__ __launch_bounds__(kBlock) void k_apply(Geo g, const double* u, double* y) {
  __shared__ double L[TL::LSZ];
  const int tile = xcd_tile(blockIdx.x, g.ntiles);
  int ox, oy, oz;
  tile_origin<TL>(g, tile, ox, oy, oz);
  load_tile<TL>(L, u, g, ox, oy, oz);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < TL::PPT; ++i) {
    auto pr = point<TL>(g, ox, oy, oz, i);
    if (pr.valid) y[pr.p] = stencil<TL>(L, g, pr.qx, pr.qy, pr.qz);
  }
}

}  // namespace mlg
