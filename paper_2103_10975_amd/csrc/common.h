// Shared device/host helpers of the MI355X (gfx950) MLGMRES library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/mlgmres.h"

namespace mlg {

// ------------------------------------------------------------------ errors
// Thread-local message behind mlg_last_error().
void set_error(const std::string& msg);

struct HipError {
  hipError_t code;
  std::string where;
};

#define MLG_HIP(expr)                                                          \
  do {                                                                         \
    hipError_t _e = (expr);                                                    \
    if (_e != hipSuccess)                                                      \
      throw ::mlg::HipError{_e, std::string(#expr) + " @ " + __FILE__ + ":" + \
                                    std::to_string(__LINE__)};                 \
  } while (0)

struct ArgError {
  int code;
  std::string msg;
};

// ------------------------------------------------------------------ sizes
constexpr int kBlock = 256;         // threads per workgroup for every sweep kernel
constexpr int kMaxRestart = 64;     // largest supported restart length m
constexpr int kXcds = 8;            // MI355X: 8 accelerator complex dies
constexpr int kMaxGrid = 1024;      // workgroups per sweep kernel (4 per CU)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Map a hardware workgroup index to a tile index so that each XCD (which the
// dispatcher feeds round-robin: workgroup b runs on XCD b % 8) owns one
// contiguous band of tiles.  Neighbouring tiles then share that XCD's L2 for
// their stencil halos.  Bijective for any count.
__device__ __forceinline__ int xcd_tile(int b, int count) {
  int q = count / kXcds, rem = count % kXcds;
  int xcd = b % kXcds, i = b / kXcds;
  int base = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
  return base + i;
}

// ------------------------------------------------------------------ global pointers
// A pointer the kernel loads from memory (the per-system descriptors) is
// generic to the compiler, which then emits flat instructions; those also
// count against the LDS counter, so every LDS wait would wait for them too.
// Everything the kernels reach through the descriptors is device memory;
// these casts make those accesses global ones.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> gmem(T* p) {
  return (gptr<T>)p;
}

// ------------------------------------------------------------------ wave sums
// Deterministic full-wavefront FP64 sum with DPP lane moves (no LDS): pairs,
// quads, half-rows, rows, then the two row broadcasts; lane 63 ends with the
// total, which is broadcast through a scalar register.  Same order on every
// call, so results are bitwise reproducible.
template <int CTRL, int RM = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, RM, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, RM, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);        // row_half_mirror
  v += dpp_f64<0x140>(v);        // row_mirror
  v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Wavefront reduce-scatters (fixed pairings, so bitwise reproducible): each
// step sends half of a lane's remaining values to its partner across one lane
// bit and adds the partner's copy of the half it keeps; once one value is
// left, the remaining bits are summed outright.
// rs16: 16 values per lane -> lane l holds the 64-lane sum of value
// 8*b5 + 4*b4 + 2*b3 + b2 (b = bits of l); lanes differing in bits 0..1 agree.
__device__ __forceinline__ double rs16(const double (&v)[16]) {
  const int lane = threadIdx.x & 63;
  double a[8], b[4], c[2];
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
#pragma unroll
  for (int i = 0; i < 8; ++i)
    a[i] = (h5 ? v[8 + i] : v[i]) + __shfl_xor(h5 ? v[i] : v[8 + i], 32, 64);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    b[i] = (h4 ? a[4 + i] : a[i]) + __shfl_xor(h4 ? a[i] : a[4 + i], 16, 64);
#pragma unroll
  for (int i = 0; i < 2; ++i)
    c[i] = (h3 ? b[2 + i] : b[i]) + dpp_f64<0x128>(h3 ? b[i] : b[2 + i]);   // row_ror:8
  double d = (h2 ? c[1] : c[0]) + dpp_f64<0x141>(h2 ? c[0] : c[1]);      // row_half_mirror
  d += dpp_f64<0x4E>(d);
  d += dpp_f64<0xB1>(d);
  return d;
}
__device__ __forceinline__ int rs16_slot(int lane) {
  return ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
}
// rs4: 4 values per lane -> lane l holds the 64-lane sum of value 2*b5 + b4.
__device__ __forceinline__ double rs4(const double (&v)[4]) {
  const int lane = threadIdx.x & 63;
  const bool h5 = lane & 32, h4 = lane & 16;
  double a[2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
    a[i] = (h5 ? v[2 + i] : v[i]) + __shfl_xor(h5 ? v[i] : v[2 + i], 32, 64);
  double d = (h4 ? a[1] : a[0]) + __shfl_xor(h4 ? a[0] : a[1], 16, 64);
  d += dpp_f64<0x128>(d);
  d += dpp_f64<0x141>(d);
  d += dpp_f64<0x4E>(d);
  d += dpp_f64<0xB1>(d);
  return d;
}
__device__ __forceinline__ int rs4_slot(int lane) { return ((lane >> 5) & 1) * 2 + ((lane >> 4) & 1); }

__device__ __forceinline__ float wave_sum_f32(float v) {
  // float variant with the same lane schedule
  int iv;
  iv = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false); v += __int_as_float(iv);
  iv = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xf, 0xf, false); v += __int_as_float(iv);
  iv = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xf, 0xf, false); v += __int_as_float(iv);
  iv = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xf, 0xf, false); v += __int_as_float(iv);
  iv = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false); v += __int_as_float(iv);
  iv = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false); v += __int_as_float(iv);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sum of partials part[col * nblocks + b] over b (fixed order) for cols <
// ncols, by one workgroup of kReduceThreads threads (nblocks <= kMaxGrid).
// Every lane issues 32 independent loads per round (2 columns x 16 blocks),
// so the latency of the partials is paid once per round, not once per load.
constexpr int kReduceThreads = 1024;
__device__ __forceinline__ void reduce_partials(gptr<const double> part, int nblocks, int ncols,
                                                double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kReduceThreads / 64;
  for (int c0 = wave; c0 < ncols; c0 += 2 * NW) {
    double v[2][16];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int c = c0 + NW * q;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int b = lane + 64 * i;
        v[q][i] = (c < ncols && b < nblocks) ? part[(size_t)c * nblocks + b] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int c = c0 + NW * q;
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 16; i += 4) s += (v[q][i] + v[q][i + 1]) + (v[q][i + 2] + v[q][i + 3]);
      s = wave_sum(s);
      if (lane == 0 && c < ncols) out[c] = s;
    }
  }
  __syncthreads();
}

// The same sums split into rounds whose loads can be issued early: NB
// blocks per lane per column (nblocks <= 64 NB), 32 / NB columns per
// wavefront, so a round covers 16 * 32 / NB columns with 32 loads per lane.
template <int NB>
struct PartialsRound {
  static constexpr int kPerWave = 32 / NB;
  static constexpr int kCols = (kReduceThreads / 64) * kPerWave;
  double v[kPerWave][NB];
};
template <int NB>
__device__ __forceinline__ void partials_load(PartialsRound<NB>& r, gptr<const double> part,
                                              int nblocks, int ncols, int c0) {
  // only live columns are loaded (a wavefront-uniform test), and only live
  // blocks (lanes past the last block are masked off): a single workgroup
  // moves all the partials, so its load instruction count is its cost
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kReduceThreads / 64;
#pragma unroll
  for (int q = 0; q < PartialsRound<NB>::kPerWave; ++q) {
    const int c = c0 + q * NW + wave;
#pragma unroll
    for (int i = 0; i < NB; ++i) r.v[q][i] = 0.0;
    if (c < ncols) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int b = lane + 64 * i;
        if (b < nblocks) r.v[q][i] = part[(size_t)c * nblocks + b];
      }
    }
  }
}
template <int NB>
__device__ __forceinline__ void partials_sum(const PartialsRound<NB>& r, int nblocks, int ncols,
                                             int c0, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kReduceThreads / 64;
#pragma unroll
  for (int q = 0; q < PartialsRound<NB>::kPerWave; ++q) {
    const int c = c0 + q * NW + wave;
    if (c >= ncols) continue;                       // wavefront-uniform
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i) s += r.v[q][i];
    s = wave_sum(s);
    if (lane == 0) out[c] = s;
  }
}

}  // namespace mlg
