// Launch table of the per-tile sweep kernels.
//
// The sweeps are templates over the basis precision T, the tile shape TL and
// the register bound MM; their instantiations are spread over translation
// units (sweeps.hip, compiled once per precision, dimension and tile index)
// so that the library builds in parallel.  Each unit exports one launcher
// function; group_fn picks it for a (dim, tile, precision) triple.
#pragma once

#include "gmres_kernels.h"

namespace mlg {

// Tile shapes (points per workgroup; 256 threads each), by dimension and
// index.  2D tiles are 32 to 128 points wide so that a wavefront reads whole
// 128 B lines of every basis vector; the narrow tall 32 x 8 tile has the
// smallest halo ring of the one-point-per-thread tiles, which the fused
// Arnoldi step recomputes.
template <int DIM, int IDX>
struct TileOf;
template <> struct TileOf<2, 0> { using type = TileT<2, 64, 16, 1>; };
template <> struct TileOf<2, 1> { using type = TileT<2, 64, 8, 1>; };
template <> struct TileOf<2, 2> { using type = TileT<2, 128, 8, 1>; };
template <> struct TileOf<2, 3> { using type = TileT<2, 64, 4, 1>; };
template <> struct TileOf<2, 4> { using type = TileT<2, 32, 8, 1>; };
template <> struct TileOf<3, 0> { using type = TileT<3, 64, 2, 4>; };
template <> struct TileOf<3, 1> { using type = TileT<3, 64, 2, 2>; };
template <> struct TileOf<3, 2> { using type = TileT<3, 32, 4, 2>; };
template <> struct TileOf<3, 3> { using type = TileT<3, 64, 4, 4>; };
// 32 wide: rows of a multiple of 32 (but not of 64) points leave no
// half-empty tile column, whose loads cost as much as full ones
template <> struct TileOf<3, 4> { using type = TileT<3, 32, 8, 4>; };
constexpr int kNumTiles2 = 5;
constexpr int kNumTiles3 = 5;

#define MLG_TILE_SWITCH(DIM, IDX, EXPR_TL)                                   \
  if ((DIM) == 2) {                                                          \
    switch (IDX) {                                                           \
      case 0: { using TL = TileOf<2, 0>::type; EXPR_TL; }                    \
      case 1: { using TL = TileOf<2, 1>::type; EXPR_TL; }                    \
      case 2: { using TL = TileOf<2, 2>::type; EXPR_TL; }                    \
      case 3: { using TL = TileOf<2, 3>::type; EXPR_TL; }                    \
      default: { using TL = TileOf<2, 4>::type; EXPR_TL; }                   \
    }                                                                        \
  } else {                                                                   \
    switch (IDX) {                                                           \
      case 0: { using TL = TileOf<3, 0>::type; EXPR_TL; }                    \
      case 1: { using TL = TileOf<3, 1>::type; EXPR_TL; }                    \
      case 2: { using TL = TileOf<3, 2>::type; EXPR_TL; }                    \
      case 3: { using TL = TileOf<3, 3>::type; EXPR_TL; }                    \
      default: { using TL = TileOf<3, 4>::type; EXPR_TL; }                   \
    }                                                                        \
  }

// Sweep kinds of one launcher: begin, initial residual, start, dots(j),
// extend(j), update (j = restart length m), residual, fused step(j), fused
// step in the split form (coefficients from sums(j)).
enum { G_BEGIN = 0, G_RESID0 = 1, G_START = 2, G_DOTS = 3, G_EXTEND = 4, G_UPDATE = 5, G_RESID = 6,
       G_STEP = 7, G_SPLIT = 8 };

// Launch one sweep kind over `nb` workgroups of a job table.
using GroupFn = void (*)(hipStream_t, int kind, int nb, const Job*, const SysDesc*, int j);

// The launcher for a tile shape and basis precision (MLG_FP64 / MLG_FP32_IR).
GroupFn group_fn(int dim, int tile, int prec);

// One launcher per (precision, dim, tile), each defined in its own unit.
#define MLG_SWEEP_NAME(P, D, T) sweeps_p##P##_d##D##_t##T
#define MLG_SWEEP_DECL(P, D, T) GroupFn MLG_SWEEP_NAME(P, D, T)();
#define MLG_SWEEP_ALL(X)                                                          \
  X(0, 2, 0) X(0, 2, 1) X(0, 2, 2) X(0, 2, 3) X(0, 2, 4) X(0, 3, 0) X(0, 3, 1)    \
  X(0, 3, 2) X(0, 3, 3) X(0, 3, 4) X(1, 2, 0) X(1, 2, 1) X(1, 2, 2) X(1, 2, 3)    \
  X(1, 2, 4) X(1, 3, 0) X(1, 3, 1) X(1, 3, 2) X(1, 3, 3) X(1, 3, 4)
MLG_SWEEP_ALL(MLG_SWEEP_DECL)

}  // namespace mlg
