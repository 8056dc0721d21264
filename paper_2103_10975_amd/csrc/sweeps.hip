// Instantiations of the per-tile sweep kernels for one basis precision, grid
// dimension and tile index, selected by MLG_SWEEP_PREC (0 FP64, 1 FP32),
// MLG_SWEEP_DIM and MLG_SWEEP_TILE at compile time.  The build compiles this
// unit once per triple; without the three macros it defines nothing.
#include "dispatch.h"

#if defined(MLG_SWEEP_PREC) && defined(MLG_SWEEP_DIM) && defined(MLG_SWEEP_TILE)

namespace mlg {
namespace {

// Sweeps keep the basis values of their points in registers, MM slots of
// them; MM is the smallest of 8, 16, 24, 32, 40, 64 that covers the step, so
// early steps of a cycle run at high occupancy.
#define MLG_MM_SWITCH(N, EXPR_MM)                                   \
  if ((N) <= 8) { constexpr int MM = 8; EXPR_MM; }                  \
  else if ((N) <= 16) { constexpr int MM = 16; EXPR_MM; }           \
  else if ((N) <= 24) { constexpr int MM = 24; EXPR_MM; }           \
  else if ((N) <= 32) { constexpr int MM = 32; EXPR_MM; }           \
  else if ((N) <= 40) { constexpr int MM = 40; EXPR_MM; }           \
  else { constexpr int MM = 64; EXPR_MM; }

template <class T, class TL>
void enqueue_group_step(hipStream_t s, int kind, int nb, const Job* jobs, const SysDesc* sd,
                        int j) {
  switch (kind) {
    case G_BEGIN: k_begin<T, TL><<<nb, kBlock, 0, s>>>(jobs, sd); break;
    case G_RESID0: k_resid<T, TL, true><<<nb, kBlock, 0, s>>>(jobs, sd); break;
    case G_START: k_start<T, TL><<<nb, kBlock, 0, s>>>(jobs, sd); break;
    case G_DOTS: MLG_MM_SWITCH(j, (k_dots<T, TL, MM><<<nb, kBlock, 0, s>>>(jobs, sd, j))); break;
    case G_EXTEND: MLG_MM_SWITCH(j, (k_extend<T, TL, MM><<<nb, kBlock, 0, s>>>(jobs, sd, j))); break;
    case G_UPDATE: MLG_MM_SWITCH(j, (k_update<T, TL, MM><<<nb, kBlock, 0, s>>>(jobs, sd))); break;
    case G_STEP:
      if constexpr (TL::DIM == 2)
        MLG_MM_SWITCH(j + 1, (k_step<T, TL, MM, false><<<nb, kBlock, 0, s>>>(jobs, sd, j)));
      break;
    case G_SPLIT:
      if constexpr (TL::DIM == 2)
        MLG_MM_SWITCH(j + 1, (k_step<T, TL, MM, true><<<nb, kBlock, 0, s>>>(jobs, sd, j)));
      break;
    default: k_resid<T, TL, false><<<nb, kBlock, 0, s>>>(jobs, sd); break;
  }
}

}  // namespace

#define MLG_SWEEP_DEF(P, D, T)                                                       \
  GroupFn MLG_SWEEP_NAME(P, D, T)() {                                                \
    using Prec = std::conditional_t<P == 0, double, float>;                         \
    return &enqueue_group_step<Prec, TileOf<D, T>::type>;                            \
  }
#define MLG_SWEEP_DEF_X(P, D, T) MLG_SWEEP_DEF(P, D, T)
MLG_SWEEP_DEF_X(MLG_SWEEP_PREC, MLG_SWEEP_DIM, MLG_SWEEP_TILE)

}  // namespace mlg

#endif
