// Guess network of the learned initial guess: forward (inference), and one
// training step (forward with saved activations, squared-error loss,
// back-propagation, Adam), all as HIP kernels for gfx950.
//
// Section 2 of the paper feeds the network output to GMRES(k) as x0 and trains
// the network in situ on the (RHS, solution) pairs the solver produces with the
// loss |x_tilde - x|^2 (Section 2.3) by back-propagation and ADAM; Section 2.1
// asks for a network that captures non-local relations without reducing
// resolution.  Architecture (C channels, M x M sine modes in L3, K x K in the
// skip band):
//   x0 = (r/s_r, f/s_f), r = f - A u_prev (FP64)       BF16 NHWC, 2 channels
//   a1 = ReLU(conv3x3(x0))          a2 = ReLU(conv3x3(a1))
//   a3 = ReLU(W1 a2 + b + S^-1[Wk . S[a2]])           (spectral mixing)
//   a4 = ReLU(conv3x3(a3))          a5 = ReLU(conv3x3(a4))
//   c6 = conv3x3(a5) (1 channel, FP32)
//   out = g (c6 - P_K c6) + S^-1[w_kl S[r/s_r]_kl]    (band path, FP64; K = 0: out = c6)
//       (P_K: projection on the K x K band; the band path alone sets the
//       output there.  Its per-mode weights w = sxt / sxx are learned from the
//       training pairs by least squares: every train step adds the batch's
//       sums of X T and X^2, X and T the band coefficients of A d and of the
//       target c_u d / s_r for the correction d = u_t - u_prev -- u_t solves
//       A u_t = f - r_fin exactly, so (A d, d) is an exact pair -- the
//       minimiser of the loss over w on those pairs; g, the output gain of
//       the convolutional branch, is the least-squares scale of its off-band
//       output against the off-band targets of recent batches, applied at
//       inference only)
//   guess = u_prev + (s_r/c_u) out
// The 3x3 convolutions with C -> C channels (forward, input gradient and
// weight gradient) and C -> 1 run on MFMA (v_mfma_f32_16x16x32_bf16) as
// implicit GEMMs over LDS tiles, the 2 -> C input layer per pixel block; the
// spectral layer's sine transforms on the BF16 and FP32 matrix cores; the
// band path's four FP64 transforms on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64; the row and output transforms also in a vector
// form for launches that fill the device); the element-wise work on the
// vector ALUs.  Activations and gradients are BF16, accumulation FP32, master
// weights and Adam state FP32, the band path FP64.
#include <algorithm>
#include <cmath>
#include <vector>

#include "net.h"

namespace mlg {
namespace {

constexpr double kCu = 19.739208802178717;   // 2 pi^2
constexpr int kMaxBatch = 64;
constexpr int kNumTensors = 13;
enum { T_C1W, T_C1B, T_C2W, T_C2B, T_SW1, T_SB, T_SWK, T_C4W, T_C4B, T_C5W, T_C5B, T_C6W, T_C6B };
constexpr int kRmsBlocks = 128;       // chunks per field of the RMS sums

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16;

// round-to-nearest-even FP32 -> BF16
__device__ __forceinline__ bf16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16)0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float((uint32_t)h << 16); }

struct Ptrs {
  const double* p[kMaxBatch];
};
struct MPtrs {
  double* p[kMaxBatch];
};

// ------------------------------------------------------------------ sizes
struct Dims {
  int B, H, W, C, M, K;          // K: skip band modes
  long long HW;
};

void tensor_sizes(const guess_net_cfg* cfg, int64_t* sz) {
  const int64_t C = cfg->channels, M = cfg->modes;
  int64_t s[kNumTensors] = {C * 2 * 9, C, C * C * 9, C, C * C, C, M * M * C * C,
                            C * C * 9, C, C * C * 9, C, C * 9, 1};
  for (int i = 0; i < kNumTensors; ++i) sz[i] = s[i];
}

void check_cfg(const guess_net_cfg* cfg) {
  if (!cfg) throw ArgError{MLG_ERR_ARG, "cfg is NULL"};
  if (cfg->channels != 32) throw ArgError{MLG_ERR_ARG, "channels must be 32"};
  if (cfg->modes < 1 || cfg->modes > 32) throw ArgError{MLG_ERR_ARG, "modes must be in 1..32"};
  if (cfg->skip_modes < 0 || cfg->skip_modes > 128)
    throw ArgError{MLG_ERR_ARG, "skip_modes must be in 0..128"};
}

struct ParamLayout {
  int64_t P;
  int64_t off[kNumTensors + 1];
  size_t master, grad, m, v, bf, step, band, gate, total;
};

ParamLayout param_layout(const guess_net_cfg* cfg) {
  check_cfg(cfg);
  ParamLayout L{};
  int64_t sz[kNumTensors];
  tensor_sizes(cfg, sz);
  L.off[0] = 0;
  for (int i = 0; i < kNumTensors; ++i) L.off[i + 1] = L.off[i] + (sz[i] + 63) / 64 * 64;
  L.P = L.off[kNumTensors];
  const size_t f = align_up((size_t)L.P * 4, 256);
  L.master = 0;
  L.grad = f;
  L.m = 2 * f;
  L.v = 3 * f;
  L.bf = 4 * f;
  L.step = L.bf + align_up((size_t)L.P * 2, 256);
  // the band's least-squares state: FP64 sums of X T, then of X^2, [K][K] each
  L.band = L.step + 256;
  // the output gain's least-squares state: FP64 sums of <c, t> and |c|^2
  L.gate = L.band + align_up((size_t)2 * cfg->skip_modes * cfg->skip_modes * 8, 256);
  L.total = L.gate + 256;
  return L;
}

Dims check_grid_net(const guess_net_cfg* cfg, const mlg_grid* grid, int batch) {
  check_cfg(cfg);
  if (!grid || grid->dim != 2) throw ArgError{MLG_ERR_ARG, "the guess network takes 2D grids"};
  const int mx = std::max(cfg->modes, cfg->skip_modes);
  if (grid->nx < mx || grid->ny < mx)
    throw ArgError{MLG_ERR_ARG, "grid must have at least max(modes, skip_modes) points per axis"};
  if (batch < 1 || batch > kMaxBatch) throw ArgError{MLG_ERR_ARG, "batch must be in 1..64"};
  Dims d{batch, grid->ny, grid->nx, cfg->channels, cfg->modes, cfg->skip_modes,
         (long long)grid->nx * grid->ny};
  return d;
}

// Padded extents of the spectral layer's x basis: modes to a multiple of 16
// (MFMA tiles), columns to a multiple of the row transform's chunk.
inline int spec_mp(const Dims& d) { return (d.M + 15) / 16 * 16; }
inline int spec_wp(const Dims& d) { return (d.W + 255) / 256 * 256; }

struct WsLayout {
  size_t s, r0, x0, act[5], out, dout, dz[2], T, X, Y, Z, Sx, Sxh, Sxl, Sy, part, loss;
  size_t kT, kT2, kX, kC, kZ, kZ2, kdY, kdY2, kTc, kXa, ad, kSx, kSxT, kSy, rms, total;   // band path (FP64)
  int wgrad_blocks;
};

WsLayout ws_layout(const Dims& d, bool train) {
  WsLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  const size_t act = (size_t)d.B * d.HW * d.C * 2;
  L.s = take((size_t)d.B * 8 * 3);        // s_r (raw), s_in, s_f
  L.r0 = take((size_t)d.B * d.HW * 8);
  L.x0 = take((size_t)d.B * d.HW * 2 * 2);
  const int nact = train ? 5 : 2;
  for (int i = 0; i < 5; ++i) L.act[i] = i < nact ? take(act) : L.act[i % 2];
  L.out = take((size_t)d.B * d.HW * 4);
  L.T = take((size_t)d.B * d.H * d.M * d.C * 4);
  L.X = take((size_t)d.B * d.M * d.M * d.C * 4);
  L.Y = take((size_t)d.B * d.M * d.M * d.C * 4);
  L.Z = take((size_t)d.B * d.H * d.M * d.C * 4);
  L.Sx = take((size_t)spec_mp(d) * spec_wp(d) * 4);
  L.Sxh = take((size_t)spec_mp(d) * spec_wp(d) * 2);
  L.Sxl = take((size_t)spec_mp(d) * spec_wp(d) * 2);
  L.Sy = take((size_t)d.M * d.H * 4);
  L.kT = take((size_t)d.B * d.H * d.K * 8);
  L.kT2 = take((size_t)d.B * d.H * d.K * 8);
  L.kX = take((size_t)d.B * d.K * d.K * 8);
  L.kC = take((size_t)d.B * d.K * d.K * 8);
  L.kZ = take((size_t)d.B * d.H * d.K * 8);
  L.kZ2 = train ? take((size_t)d.B * d.H * d.K * 8) : 0;
  L.kdY = train ? take((size_t)d.B * d.K * d.K * 8) : 0;
  L.kdY2 = train ? take((size_t)d.B * d.K * d.K * 8) : 0;
  L.kTc = train ? take((size_t)d.B * d.K * d.K * 8) : 0;
  L.kXa = train ? take((size_t)d.B * d.K * d.K * 8) : 0;
  L.ad = train && d.K > 0 ? take((size_t)d.B * d.HW * 8) : 0;
  L.kSx = take((size_t)d.K * d.W * 8);
  L.kSxT = take((size_t)d.K * d.W * 8);
  L.kSy = take((size_t)d.K * d.H * 8);
  L.rms = take((size_t)2 * d.B * kRmsBlocks * 8);
  L.wgrad_blocks = 0;
  if (train) {
    L.dout = take((size_t)d.B * d.HW * 4);
    L.dz[0] = take(act);
    L.dz[1] = take(act);
    L.wgrad_blocks = 512;
    L.part = take((size_t)L.wgrad_blocks * (9 * d.C * d.C + d.C) * 4);
    L.loss = take(4096 * 8);
  }
  L.total = o;
  return L;
}

// ------------------------------------------------------------------ small kernels

// Sine bases (DST-I): S[k][j] = sin((k+1) pi (j+1) / (n+1)), the slowest modes.
// Every basis one pass needs (filled beside the network input, see k_resid_sumsq):
//   Sx       FP32 [MP][WP]  x direction of the spectral layer, zero for k >= M
//            or j >= W (MP = M rounded up to 16, WP = W rounded up to 256)
//   Sxh, Sxl BF16 [MP][WP]  Sx = Sxh + Sxl to within 2^-17 |Sx| (the two BF16
//            halves of the MFMA row transform)
//   Sy       FP32 [M][H]    y direction of the spectral layer
//   kSx      FP64 [K][W], kSxT FP64 [W][K], kSy FP64 [K][H]  the band path
struct Bases {
  float* Sx;
  bf16* Sxh;
  bf16* Sxl;
  float* Sy;
  double* kSx;
  double* kSxT;
  double* kSy;
  int M, MP, W, WP, H, K;
};

__device__ __forceinline__ double sine_mode(int k, int j, int n) {
  return sin((double)(k + 1) * M_PI * (double)(j + 1) / (double)(n + 1));
}

// Element e of the concatenated bases (Sx with its BF16 halves, Sy, kSx with
// kSxT, kSy).
__device__ __forceinline__ void bases_at(const Bases& o, long long e) {
  const long long n1 = (long long)o.MP * o.WP, n2 = (long long)o.M * o.H;
  const long long n3 = (long long)o.K * o.W, n4 = (long long)o.K * o.H;
  if (e < n1) {
    const int k = (int)(e / o.WP), j = (int)(e % o.WP);
    const float f = (k < o.M && j < o.W) ? (float)sine_mode(k, j, o.W) : 0.f;
    const bf16 h = f2bf(f);
    o.Sx[e] = f;
    o.Sxh[e] = h;
    o.Sxl[e] = f2bf(f - bf2f(h));
    return;
  }
  e -= n1;
  if (e < n2) {
    o.Sy[e] = (float)sine_mode((int)(e / o.H), (int)(e % o.H), o.H);
    return;
  }
  e -= n2;
  if (e < n3) {
    const int k = (int)(e / o.W), j = (int)(e % o.W);
    const double v = sine_mode(k, j, o.W);
    o.kSx[e] = v;
    o.kSxT[(size_t)j * o.K + k] = v;
    return;
  }
  e -= n3;
  if (e < n4) o.kSy[e] = sine_mode((int)(e / o.H), (int)(e % o.H), o.H);
}

inline long long bases_count(const Bases& o) {
  return (long long)o.MP * o.WP + (long long)o.M * o.H + (long long)o.K * (o.W + o.H);
}

// The residual r_b = f_b - A u_b of each image (FP64, the 5-point operator
// of the solver) written out, with the sums of squares of the B residuals
// and the B sources over kRmsBlocks contiguous chunks per field (blockIdx.y:
// field r_0..r_{B-1}, f_0..f_{B-1}); each chunk's sum in a fixed order.  A
// plane blockIdx.y = 2B, when launched, fills the network's sine bases
// (nbases elements), which depend on nothing else.
__global__ __launch_bounds__(256) void k_resid_sumsq(Ptrs f, Ptrs u, double* r, int B, int H, int W,
                                                     double* part, Bases o, long long nbases) {
  __shared__ double red[4];
  const int fi = blockIdx.y;
  if (fi == 2 * B) {                                     // the extra plane: the sine bases
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < nbases;
         e += (long long)gridDim.x * 256)
      bases_at(o, e);
    return;
  }
  const long long n = (long long)H * W;
  const long long c0 = n * blockIdx.x / kRmsBlocks, c1 = n * (blockIdx.x + 1) / kRmsBlocks;
  double acc = 0.0;
  if (fi < B) {
    const double* ub = u.p[fi];
    const double* fb = f.p[fi];
    double* rb = r + (size_t)fi * n;
    const double cx = (double)(W + 1) * (W + 1), cy = (double)(H + 1) * (H + 1);
    for (long long p = c0 + threadIdx.x; p < c1; p += 256) {
      const int y = (int)(p / W), x = (int)(p % W);
      const double c = ub[p];
      const double w = x > 0 ? ub[p - 1] : 0.0, e = x < W - 1 ? ub[p + 1] : 0.0;
      const double sN = y > 0 ? ub[p - W] : 0.0, nN = y < H - 1 ? ub[p + W] : 0.0;
      const double v = fb[p] - ((2.0 * c - w - e) * cx + (2.0 * c - sN - nN) * cy);
      rb[p] = v;
      acc += v * v;
    }
  } else {
    const double* x = f.p[fi - B];
    for (long long p = c0 + threadIdx.x; p < c1; p += 256) acc += x[p] * x[p];
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    part[(size_t)fi * kRmsBlocks + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// RMS of field fi from its kRmsBlocks chunk sums, added in a fixed order by
// one wavefront (every lane returns it).
__device__ __forceinline__ double rms_of(const double* part, int fi, long long n) {
  double v = 0.0;
  for (int k = threadIdx.x & 63; k < kRmsBlocks; k += 64) v += part[(size_t)fi * kRmsBlocks + k];
  v = wave_sum(v);
  return sqrt(v / (double)n);
}

// x0[b][p] = (r/s_r, f/s_f) in BF16 (2 channels), s_r and s_f the
// division-safe RMS of r_b and f_b (1 where the RMS is 0), formed in every
// workgroup from the chunk sums (wavefront 0: r_b, wavefront 1: f_b); the
// first workgroup of each image also stores sv[b] = RMS(r_b) (raw),
// sv[B + b] = s_r and sv[2B + b] = s_f.
__global__ __launch_bounds__(256) void k_norm_in(const double* r, Ptrs f, const double* part,
                                                 double* sv, int B, bf16* x0, long long HW) {
  __shared__ double sc[2];
  const int b = blockIdx.y, wv = threadIdx.x >> 6;
  if (wv < 2) {
    const double rms = rms_of(part, wv == 0 ? b : B + b, HW);
    const double safe = rms > 0.0 ? rms : 1.0;
    if ((threadIdx.x & 63) == 0) {
      sc[wv] = safe;
      if (blockIdx.x == 0) {
        if (wv == 0) {
          sv[b] = rms;
          sv[B + b] = safe;
        } else {
          sv[2 * B + b] = safe;
        }
      }
    }
  }
  __syncthreads();
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  bf16* o = x0 + ((size_t)b * HW + p) * 2;
  o[0] = f2bf((float)(r[(size_t)b * HW + p] / sc[0]));
  o[1] = f2bf((float)(f.p[b][p] / sc[1]));
}

// guess = u_prev + (s_r / c_u) out
__global__ void k_guess(const float* out, Ptrs u, const double* s, MPtrs g, long long HW) {
  const int b = blockIdx.y;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  g.p[b][p] = u.p[b][p] + (s[b] / kCu) * (double)out[(size_t)b * HW + p];
}

// loss = (1/B) sum_b |out_b - t_b|^2, t = c_u (u_t - u_prev)/s; dout = (2/B)(out - t).
// Per-workgroup partial sums of the squared error; k_loss_sum adds them.
__global__ __launch_bounds__(256) void k_loss(const float* out, Ptrs ut, Ptrs up, const double* s,
                                              float* dout, double* part, long long HW, int B) {
  __shared__ double red[4];
  double acc = 0.0;
  const long long total = (long long)B * HW;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (long long)gridDim.x * 256) {
    const int b = (int)(e / HW);
    const long long p = e % HW;
    const double t = (ut.p[b][p] - up.p[b][p]) * (kCu / s[b]);
    const double diff = (double)out[e] - t;
    dout[e] = (float)(2.0 * diff / B);
    acc += diff * diff;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(kReduceThreads) void k_loss_sum(const double* part, int nblk,
                                                            float* loss_dev, float* loss_user,
                                                            int B) {
  __shared__ double fin[1];
  reduce_partials(gmem(part), nblk, 1, fin);
  if (threadIdx.x == 0) {
    const float L = (float)(fin[0] / B);
    *loss_dev = L;
    if (loss_user) *loss_user = L;
  }
}

// ------------------------------------------------------------------ thin convolutions (VALU)
// out[p][co] = epilogue(sum_{tap,ci} w[tap][co][ci] in[p + off(tap)][ci]) with the weight
// tensor staged as w[tap][co][ci]; DGRAD stages the flipped transpose of the forward
// weights (input gradient of the forward layer) and multiplies by (mask > 0).
// A pixel's channel vector in 16-byte pieces when the channel count allows
// (8 BF16 or 4 FP32 per piece), else element by element.
template <int N>
__device__ __forceinline__ void load_ch(const bf16* p, float (&v)[N]) {
  if constexpr (N % 8 == 0) {
#pragma unroll
    for (int q = 0; q < N / 8; ++q) {
      const uint4 u = reinterpret_cast<const uint4*>(p)[q];
      const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        v[8 * q + 2 * h] = __uint_as_float(w[h] << 16);
        v[8 * q + 2 * h + 1] = __uint_as_float(w[h] & 0xffff0000u);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = bf2f(p[i]);
  }
}
template <int N>
__device__ __forceinline__ void load_ch(const float* p, float (&v)[N]) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (int q = 0; q < N / 4; ++q) {
      const float4 u = reinterpret_cast<const float4*>(p)[q];
      v[4 * q] = u.x;
      v[4 * q + 1] = u.y;
      v[4 * q + 2] = u.z;
      v[4 * q + 3] = u.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = p[i];
  }
}
template <int N>
__device__ __forceinline__ void store_ch(bf16* p, const float (&v)[N]) {
  if constexpr (N % 8 == 0) {
#pragma unroll
    for (int q = 0; q < N / 8; ++q) {
      uint32_t w[4];
#pragma unroll
      for (int h = 0; h < 4; ++h)
        w[h] = (uint32_t)f2bf(v[8 * q + 2 * h]) | ((uint32_t)f2bf(v[8 * q + 2 * h + 1]) << 16);
      reinterpret_cast<uint4*>(p)[q] = make_uint4(w[0], w[1], w[2], w[3]);
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = f2bf(v[i]);
  }
}
template <int N>
__device__ __forceinline__ void store_ch(float* p, const float (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) p[i] = v[i];
}

// ------------------------------------------------------------------ thin convolutions on MFMA
// The input (2 -> C) and output (C -> 1) convolutions and the output
// convolution's input gradient, on the matrix cores although one side of each
// contraction is thin: a workgroup takes 256 consecutive pixels of one image
// (each wavefront four 16-pixel steps), every tap read at a clamped position
// with all of a step's loads in flight, taps outside the grid zeroed by a
// select.  The weights are read once per thread as the 32-bit words that hold
// them.
__device__ __forceinline__ uint32_t bf16_word_pick(const bf16* base, long long e) {
  const uint32_t w = *reinterpret_cast<const uint32_t*>(base + (e & ~1LL));
  return (e & 1) ? (w >> 16) : (w & 0xffffu);
}

// Block index of this workgroup along x (n = gridDim.x blocks): workgroup g
// runs on XCD g mod 8 (each XCD has its own L2), so when 8 divides n the
// blocks are dealt out as 8 contiguous ranges, one per XCD; the 3 x 3
// neighbourhoods of adjacent rows then come from the L2 that already holds
// them instead of being fetched again by another XCD (a per-pixel 3 x 3
// read of 32 channels fetched 3.2x its input without this).  With a y dimension the
// workgroup's linear index is x + n y, so the XCD is still x mod 8.
__device__ __forceinline__ int xcd_block() {
  const int n = gridDim.x, g = blockIdx.x;
  return n % 8 ? g : (g % 8) * (n / 8) + g / 8;
}

// out[p][co] = ReLU(bias[co] + sum_{t, ci} W[co][ci][t] in[p + off(t)][ci]) for
// 2 input channels, v_mfma_f32_16x16x32_bf16 with K = 9 taps x 2 channels
// (padded to 32): A = W (16 channels x 32), B = the 18 tap values of 16
// pixels (a lane: four taps x both channels, four 4-byte reads).
template <int C>
__global__ __launch_bounds__(256) void k_conv_in_mfma(const bf16* in, const bf16* wt,
                                                      const bf16* bias, bf16* out, int H, int W) {
  static_assert(C == 32, "two 16-channel tiles");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int b = blockIdx.y;
  const long long HW = (long long)H * W;
  // A[co][k], k = 8 lg + e: tap t = 4 lg + e / 2, channel e % 2 (zero for t >= 9)
  bf16x8 wa[2];
  float bl[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int co = mt * 16 + li;
    uint32_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int tt = 4 * lg + e / 2, ci = e % 2;
      const uint32_t v = bf16_word_pick(wt, (long long)(co * 2 + ci) * 9 + min(tt, 8));
      h[e] = tt < 9 ? v : 0u;
    }
    wa[mt] = __builtin_bit_cast(bf16x8, make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16),
                                                   h[4] | (h[5] << 16), h[6] | (h[7] << 16)));
#pragma unroll
    for (int r = 0; r < 4; ++r) bl[mt][r] = bf2f(bias[mt * 16 + 4 * lg + r]);
  }
  const uint32_t* inw = reinterpret_cast<const uint32_t*>(in) + (size_t)b * HW;   // one word per pixel
  const long long nblk = (HW + 255) / 256;
  for (long long blk = xcd_block(); blk < nblk; blk += gridDim.x) {
    // the neighbourhoods of all four 16-pixel steps of this wavefront are
    // loaded first, at clamped positions (no branch between the loads); the
    // out-of-grid taps are zeroed afterwards (the empty asm keeps the compiler
    // from turning that select into a branch around each load)
    uint32_t v[4][4];
    bool in_tap[4][4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const long long p = blk * 256 + wv * 64 + st * 16 + li;
      const long long pc = p < HW ? p : HW - 1;
      const int y = (int)(pc / W), x = (int)(pc % W);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tt = 4 * lg + q, dy = tt / 3 - 1, dx = tt % 3 - 1;
        const int yy = y + dy, xx = x + dx;
        v[st][q] = inw[(long long)min(max(yy, 0), H - 1) * W + min(max(xx, 0), W - 1)];
        in_tap[st][q] = tt < 9 && yy >= 0 && yy < H && xx >= 0 && xx < W;
      }
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const long long p = blk * 256 + wv * 64 + st * 16 + li;
      if (blk * 256 + wv * 64 + st * 16 >= HW) break;                     // wavefront-uniform
      uint32_t vm[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t w = v[st][q];
        asm volatile("" : "+v"(w));
        vm[q] = in_tap[st][q] ? w : 0u;
      }
      const bf16x8 bx = __builtin_bit_cast(bf16x8, make_uint4(vm[0], vm[1], vm[2], vm[3]));
      floatx4 acc[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[mt], bx, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      if (p < HW) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          float o[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) o[r] = fmaxf(acc[mt][r] + bl[mt][r], 0.f);
          uint2 w2;
          w2.x = (uint32_t)f2bf(o[0]) | ((uint32_t)f2bf(o[1]) << 16);
          w2.y = (uint32_t)f2bf(o[2]) | ((uint32_t)f2bf(o[3]) << 16);
          *reinterpret_cast<uint2*>(out + ((size_t)b * HW + p) * C + mt * 16 + 4 * lg) = w2;
        }
      }
    }
  }
}

// dz[p][co] = (mask[p][co] > 0) * sum_t W[0][co][8 - t] dout[p + off(t)]: the
// input gradient of the C -> 1 convolution from the FP32 output gradient, on
// v_mfma_f32_16x16x4_f32 (K = 4 taps per step, three steps): A = the flipped
// weights (16 channels x 4 taps), B = the output gradient at the taps (4 x 16
// pixels), in FP32.
template <int C>
__global__ __launch_bounds__(256) void k_conv_outT_mfma(const float* dout, const bf16* wt,
                                                        const bf16* mask, bf16* dz, int H, int W) {
  static_assert(C == 32, "two 16-channel tiles");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int b = blockIdx.y;
  const long long HW = (long long)H * W;
  float wa[3][2];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int tt = 4 * s + lg, co = mt * 16 + li;
      const float v = bf2f((bf16)bf16_word_pick(wt, (long long)co * 9 + (8 - min(tt, 8))));
      wa[s][mt] = tt < 9 ? v : 0.f;
    }
  const float* db = dout + (size_t)b * HW;
  const long long nblk = (HW + 255) / 256;
  for (long long blk = xcd_block(); blk < nblk; blk += gridDim.x) {
#pragma unroll 1
    for (int st = 0; st < 4; ++st) {
      const long long p0 = blk * 256 + wv * 64 + st * 16;
      if (p0 >= HW) break;                                   // wavefront-uniform
      const long long p = p0 + li, pc = p < HW ? p : HW - 1;
      const int y = (int)(pc / W), x = (int)(pc % W);
      float bvv[3];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int tt = 4 * s + lg, yy = y + tt / 3 - 1, xx = x + tt % 3 - 1;
        const float v = db[(long long)min(max(yy, 0), H - 1) * W + min(max(xx, 0), W - 1)];
        bvv[s] = (tt < 9 && yy >= 0 && yy < H && xx >= 0 && xx < W) ? v : 0.f;
      }
      const size_t base = ((size_t)b * HW + pc) * C;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 3; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[s][mt], bvv[s], acc, 0, 0, 0);
        // lane holds channels mt*16 + 4 lg + r of pixel p
        const uint2 mu = *reinterpret_cast<const uint2*>(mask + base + mt * 16 + 4 * lg);
        if (p >= HW) continue;
        const float m4[4] = {__uint_as_float(mu.x << 16), __uint_as_float(mu.x & 0xffff0000u),
                             __uint_as_float(mu.y << 16), __uint_as_float(mu.y & 0xffff0000u)};
        float o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = m4[r] > 0.f ? acc[r] : 0.f;
        uint2 w2;
        w2.x = (uint32_t)f2bf(o[0]) | ((uint32_t)f2bf(o[1]) << 16);
        w2.y = (uint32_t)f2bf(o[2]) | ((uint32_t)f2bf(o[3]) << 16);
        *reinterpret_cast<uint2*>(dz + base + mt * 16 + 4 * lg) = w2;
      }
    }
  }
}

// Weight gradient of the C -> 1 output convolution (C = 32):
// dW[t][c] = sum_p dout[p] a[p + off(t)][c], db = sum_p dout[p].  With
// q = p + off(t) every input pixel q is read once (its 8-channel chunk, 16
// bytes) and multiplied by the 3x3 neighbourhood of dout around it (from
// LDS); a thread keeps its 9 x 8 running sums over every pixel it visits
// (persistent over 64 x 4 tiles), and each wavefront (one channel chunk)
// sums its lanes at the end.  part[blk][t * C + c], bias at [9 C].
template <int C>
__global__ __launch_bounds__(256) void k_wgrad_out(const bf16* a, const float* dout, float* part,
                                                   int B, int H, int W) {
  static_assert(C == 32, "four wavefronts, one 8-channel chunk each");
  constexpr int TX = 64, TY = 4, LX = TX + 2, LY = TY + 2;
  __shared__ float dl[LY * LX];
  const int lane = threadIdx.x & 63, cg = threadIdx.x >> 6;
  float acc[9][8];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[t][e] = 0.f;
  float bacc = 0.f;
  const int tilesx = (W + TX - 1) / TX, tilesy = (H + TY - 1) / TY;
  const int per_img = tilesx * tilesy, ntiles = B * per_img;
  const long long HW = (long long)H * W;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int b = tile / per_img, r0 = tile % per_img;
    const int ox = (r0 % tilesx) * TX, oy = (r0 / tilesx) * TY;
    // every load of the tile first, at clamped addresses: this thread's
    // 8-channel chunk on each row, then the halo of the output gradient
    const int x = ox + lane;
    uint4 av[TY];
    bool okr[TY];
#pragma unroll
    for (int r = 0; r < TY; ++r) {
      const int y = oy + r;
      okr[r] = y < H && x < W;
      const long long pix = (long long)min(y, H - 1) * W + min(x, W - 1);
      av[r] = *reinterpret_cast<const uint4*>(a + ((size_t)b * HW + pix) * C + cg * 8);
    }
    constexpr int NH = (LY * LX + 255) / 256;
    float hv[NH];
    bool hin[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int e = threadIdx.x + 256 * h;
      const int gy = oy + e / LX - 1, gx = ox + e % LX - 1;
      hin[h] = e < LY * LX && gy >= 0 && gy < H && gx >= 0 && gx < W;
      hv[h] = dout[(size_t)b * HW + (hin[h] ? (long long)gy * W + gx : 0)];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int e = threadIdx.x + 256 * h;
      if (e < LY * LX) dl[e] = hin[h] ? hv[h] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < TY; ++r) {
      if (!okr[r]) continue;
      float v[8];
      {
        const uint32_t w4[4] = {av[r].x, av[r].y, av[r].z, av[r].w};
#pragma unroll
        for (int h2 = 0; h2 < 4; ++h2) {
          v[2 * h2] = __uint_as_float(w4[h2] << 16);
          v[2 * h2 + 1] = __uint_as_float(w4[h2] & 0xffff0000u);
        }
      }
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        // dout at q - off(t): halo row r + 2 - ky, column lane + 2 - kx
        const float w = dl[(r + 2 - t / 3) * LX + lane + 2 - t % 3];
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[t][e] = fmaf(w, v[e], acc[t][e]);
      }
      if (cg == 0) bacc += dl[(r + 1) * LX + lane + 1];
    }
  }
  float* pb = part + (size_t)blockIdx.x * (9 * C + 1);
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float sum = wave_sum_f32(acc[t][e]);
      if (lane == 0) pb[t * C + cg * 8 + e] = sum;
    }
  const float bs = wave_sum_f32(bacc);
  if (threadIdx.x == 0) pb[9 * C] = bs;
}

// Weight gradient of the 2 -> C input convolution (C = 32):
// dW[t][d][c] = sum_p dz[p][d] x[p + off(t)][c] (c < 2), db[d] = sum_p dz[p][d].
// A thread takes 4 output channels of one tile column (tiles of 32 x 8
// pixels, persistent): per pixel one 8-byte read of dz and the 3x3 x 2
// neighbourhood of x from LDS, 4 x 9 x 2 running sums; the 32 lanes of a
// channel group sum at the end.  part[blk][(t * C + d) * 2 + c], bias at
// [18 C + d].
template <int C>
__global__ __launch_bounds__(256) void k_wgrad_in(const bf16* x, const bf16* dz, float* part,
                                                  int B, int H, int W) {
  static_assert(C == 32, "eight channel groups of four");
  constexpr int TX = 32, TY = 8, LX = TX + 2, LY = TY + 2;
  __shared__ float xl[LY * LX * 2];
  const int l32 = threadIdx.x & 31, dg = threadIdx.x >> 5;
  float acc[4][9][2], bacc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    bacc[q] = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[q][t][0] = acc[q][t][1] = 0.f;
  }
  const int tilesx = (W + TX - 1) / TX, tilesy = (H + TY - 1) / TY;
  const int per_img = tilesx * tilesy, ntiles = B * per_img;
  const long long HW = (long long)H * W;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int b = tile / per_img, r0 = tile % per_img;
    const int ox = (r0 % tilesx) * TX, oy = (r0 / tilesx) * TY;
    // every load of the tile first, at clamped addresses (no branch between
    // them): this thread's four gradient channels on each of the tile's rows,
    // then the input halo as 32-bit words (both channels of a pixel)
    const int gx = ox + l32;
    uint2 dv[TY];
    bool okr[TY];
#pragma unroll
    for (int r = 0; r < TY; ++r) {
      const int gy = oy + r;
      okr[r] = gy < H && gx < W;
      const long long pix = (long long)min(gy, H - 1) * W + min(gx, W - 1);
      dv[r] = *reinterpret_cast<const uint2*>(dz + ((size_t)b * HW + pix) * C + dg * 4);
    }
    constexpr int NH = (LY * LX + 255) / 256;
    unsigned int hw[NH];
    bool hin[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int e = threadIdx.x + 256 * h;
      const int gy = oy + e / LX - 1, gx2 = ox + e % LX - 1;
      hin[h] = e < LY * LX && gy >= 0 && gy < H && gx2 >= 0 && gx2 < W;
      const long long pix = hin[h] ? (long long)gy * W + gx2 : 0;
      hw[h] = *reinterpret_cast<const unsigned int*>(x + ((size_t)b * HW + pix) * 2);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int e = threadIdx.x + 256 * h;
      if (e < LY * LX) {
        xl[2 * e] = hin[h] ? __uint_as_float(hw[h] << 16) : 0.f;
        xl[2 * e + 1] = hin[h] ? __uint_as_float(hw[h] & 0xffff0000u) : 0.f;
      }
    }
    __syncthreads();
#pragma unroll 2
    for (int r = 0; r < TY; ++r) {
      // rows outside the grid add exact zeros (finite inputs)
      const uint2 du = okr[r] ? dv[r] : make_uint2(0u, 0u);
      const float d4[4] = {__uint_as_float(du.x << 16), __uint_as_float(du.x & 0xffff0000u),
                           __uint_as_float(du.y << 16), __uint_as_float(du.y & 0xffff0000u)};
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        // x at p + off(t): halo row r + ky, column l32 + kx
        const int o = 2 * ((r + t / 3) * LX + l32 + t % 3);
        const float x0 = xl[o], x1 = xl[o + 1];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[q][t][0] = fmaf(d4[q], x0, acc[q][t][0]);
          acc[q][t][1] = fmaf(d4[q], x1, acc[q][t][1]);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) bacc[q] += d4[q];
    }
  }
  // sum the 32 lanes of this channel group (fixed pairing)
  auto half_sum = [](float v) {
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
  };
  float* pb = part + (size_t)blockIdx.x * (18 * C + C);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int d = dg * 4 + q;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float sum = half_sum(acc[q][t][c]);
        if (l32 == 0) pb[(t * C + d) * 2 + c] = sum;
      }
    const float bs = half_sum(bacc[q]);
    if (l32 == 0) pb[18 * C + d] = bs;
  }
}

// grad[...] = sum over blocks of the partials (fixed order).  Partial element
// e = (t*COUT + d)*CIN + c maps to the torch layout (d*CIN + c)*ntap + t; the
// trailing COUT elements are bias gradients.  A workgroup takes 64 elements
// (lanes); its four wavefronts sum a quarter of the blocks each (eight
// independent running sums), and the quarters are added in a fixed order.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* part, int nblk, int ntap,
                                                      int cout, int cin, float* gw, float* gb) {
  __shared__ float red[4][64];
  const int nw = ntap * cout * cin, stride = nw + cout;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int ka = nblk * w / 4, kb = nblk * (w + 1) / 4;
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (e < stride) {
    int k = ka;
    for (; k + 8 <= kb; k += 8) {
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] += part[(size_t)(k + q) * stride + e];
    }
    for (; k < kb; ++k) a[0] += part[(size_t)k * stride + e];
  }
  red[w][lane] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  if (w != 0 || e >= stride) return;
  const float s = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
  if (e < nw) {
    const int t = e / (cout * cin), r = e % (cout * cin), d = r / cin, c = r % cin;
    gw[(d * cin + c) * ntap + t] = s;
  } else {
    gb[e - nw] = s;
  }
}

// ------------------------------------------------------------------ MFMA convolutions
// 3x3 convolution C -> C (C = 32), persistent over 64 x 8 pixel tiles of all
// B images, on v_mfma_f32_16x16x32_bf16 with the roles
//   A = weights (16 output channels x 32 input channels of one tap), held in
//       registers for the whole launch (9 taps x 2 output tiles);
//   B = input (32 input channels x 16 pixels), read from the LDS tile (one
//       16-byte read per lane, a contiguous 1 KB per wavefront);
//   D = 16 output channels x 16 pixels: a lane holds 4 consecutive channels
//       of one pixel, written as one 8-byte store.
// Wavefront w computes rows 2w, 2w+1 of the tile; the next tile's input is
// loaded into registers while the current one is computed.  Forward: bias +
// ReLU epilogue.  DGRAD: flipped-transposed weights, epilogue multiplies by
// (mask > 0).  RES: a linear epilogue (bias in the forward form) that adds
// `mask` as a residual (none when it is NULL); each output element reads only
// its own residual element, so `out` may alias it.
constexpr int kConvTX = 64, kConvTY = 8;

template <int C, bool DGRAD, bool RES = false>
__global__ __launch_bounds__(256) void k_conv_mfma(const bf16* in, const bf16* wt, const bf16* bias,
                                                   const bf16* mask, bf16* out, int B, int H, int W) {
  static_assert(C == 32, "the MFMA convolution is laid out for 32 channels");
  constexpr int TX = kConvTX, TY = kConvTY, LX = TX + 2, LY = TY + 2;
  constexpr int CH = C / 8;                              // 16-byte chunks per pixel
  constexpr int NLD = (LY * LX * CH + 255) / 256;        // staged chunks per thread
  constexpr bool EPI = (DGRAD && !RES) || RES;           // the epilogue reads `mask`
  __shared__ __attribute__((aligned(16))) bf16 tin[LY * LX * C];
  // weights: A[i = output channel mt*16 + li][k = input channel lg*8 + e] of
  // tap t (32-bit word reads).  With a masked epilogue they are gathered once
  // per workgroup into LDS and read per row (the registers hold the masks);
  // the forward keeps them in registers for the whole launch.
  __shared__ uint4 wfr[EPI ? 9 : 1][2][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  auto frag = [&](int t, int mt, int ln) {
    const int co = mt * 16 + (ln & 15), cb = (ln >> 4) * 8;
    uint32_t h[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ci = cb + q;
      h[q] = bf16_word_pick(wt, DGRAD ? (long long)(ci * C + co) * 9 + (8 - t) : (long long)(co * C + ci) * 9 + t);
    }
    return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
  };
  const int tilesx = (W + TX - 1) / TX, tilesy = (H + TY - 1) / TY;
  const int per_img = tilesx * tilesy, ntiles = B * per_img;
  // one tile per workgroup (a single image): the output goes out with
  // non-temporal stores, written back while the kernel runs instead of at its
  // end (batch 1: 14.7 -> 13.1 us; with several tiles per workgroup the plain
  // stores are faster)
  const bool nt_out = ntiles <= (int)gridDim.x;
  const long long HW = (long long)H * W;
  // staged chunk e of a tile: halo pixel e / CH (row-major in the halo), chunk e % CH
  auto fetch = [&](int tile, uint4 (&pre)[NLD]) {
    const int b = tile / per_img, r0 = tile % per_img;
    const int ox = (r0 % tilesx) * TX, oy = (r0 / tilesx) * TY;
    const bf16* inb = in + (size_t)b * HW * C;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int e = threadIdx.x + 256 * k;
      const int pix = e / CH, ch = e % CH;
      const int ly = pix / LX, lx = pix % LX;
      const int gy = oy + ly - 1, gx = ox + lx - 1;
      const bool ok = e < LY * LX * CH && gy >= 0 && gy < H && gx >= 0 && gx < W;
      pre[k] = ok ? *reinterpret_cast<const uint4*>(inb + ((long long)gy * W + gx) * C + ch * 8)
                  : make_uint4(0, 0, 0, 0);
    }
  };
  uint4 pre[NLD];
  int tile = blockIdx.x;
  if (tile < ntiles) fetch(tile, pre);              // the first tile's loads go out first
  bf16x8 wa[EPI ? 1 : 9][2];
  if constexpr (EPI) {
    for (int e = threadIdx.x; e < 9 * 2 * 64; e += 256) wfr[e / 128][(e / 64) % 2][e % 64] = frag(e / 128, (e / 64) % 2, e % 64);
  } else {
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        bf16 v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = wt[((mt * 16 + li) * C + lg * 8 + e) * 9 + t];
        wa[t][mt] = __builtin_bit_cast(bf16x8, v);
      }
  }
  // the bias, loaded unconditionally (from the weights when there is none)
  // and selected afterwards: a load under the null test compiled to a branch
  // and a full wait per value
  const bool has_bias = !DGRAD && bias != nullptr;
  const bf16* bsrc = has_bias ? bias : wt;
  uint32_t braw[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) braw[mt][r] = bf16_word_pick(bsrc, mt * 16 + lg * 4 + r);
  float bl[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint32_t v = braw[mt][r];
      asm volatile("" : "+v"(v));
      bl[mt][r] = has_bias ? bf2f((bf16)v) : 0.f;
    }
  for (; tile < ntiles; tile += gridDim.x) {
    __syncthreads();                                     // the previous tile's reads are done
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < LY * LX * CH) *reinterpret_cast<uint4*>(&tin[e * 8]) = pre[k];
    }
    __syncthreads();
    const int b = tile / per_img, r0 = tile % per_img;
    const int ox = (r0 % tilesx) * TX, oy = (r0 / tilesx) * TY;
    // the epilogue's mask (or residual) of both rows, read before the next
    // tile's loads so that waiting for it leaves those in flight (clamped
    // positions; entries outside the grid are never used)
    uint2 mk[2][4][2];
    if constexpr (EPI) {
      if (mask) {
#pragma unroll
        for (int r2 = 0; r2 < 2; ++r2) {
          const int y = min(oy + wv * 2 + r2, H - 1);
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) {
            const int x = min(ox + nt * 16 + li, W - 1);
            const size_t base = ((size_t)b * HW + (long long)y * W + x) * C;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) mk[r2][nt][mt] = *reinterpret_cast<const uint2*>(mask + base + mt * 16 + lg * 4);
          }
        }
      }
    }
    const int next = tile + gridDim.x;
    if (next < ntiles) fetch(next, pre);                 // in flight during the MFMAs
    // one output row at a time (its accumulators only); the row's masks are
    // picked by a select, so both rows' stay in registers
#pragma unroll 1
    for (int r2 = 0; r2 < 2; ++r2) {
      // with a masked epilogue, an index the compiler cannot see to be
      // `lane`, so that the weight fragments are read from LDS per row (the
      // registers hold the masks); the forward keeps them in registers
      int wl = lane;
      if constexpr (EPI) asm volatile("" : "+v"(wl));
      floatx4 acc[4][2];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) acc[nt][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int ly = wv * 2 + r2 + t / 3, kx = t % 3;
        bf16x8 wa0, wa1;
        if constexpr (EPI) {
          wa0 = __builtin_bit_cast(bf16x8, wfr[t][0][wl]);
          wa1 = __builtin_bit_cast(bf16x8, wfr[t][1][wl]);
        } else {
          wa0 = wa[t][0];
          wa1 = wa[t][1];
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const int lx = nt * 16 + li + kx;
          const bf16x8 bx = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const uint4*>(&tin[(ly * LX + lx) * C + lg * 8]));
          acc[nt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa0, bx, acc[nt][0], 0, 0, 0);
          acc[nt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa1, bx, acc[nt][1], 0, 0, 0);
        }
      }
      // epilogue: lane holds channels mt*16 + lg*4 + r (r < 4) of pixel nt*16 + li
      const int y = oy + wv * 2 + r2;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int x = ox + nt * 16 + li;
        if (y >= H || x >= W) continue;
        const size_t base = ((size_t)b * HW + (long long)y * W + x) * C;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          const size_t o = base + mt * 16 + lg * 4;
          float v[4];
          float m4[4] = {0.f, 0.f, 0.f, 0.f};
          // the ReLU mask of the input gradient, or the residual (optional)
          if (EPI && mask) {
            const uint2 mu = r2 ? mk[1][nt][mt] : mk[0][nt][mt];
            m4[0] = __uint_as_float(mu.x << 16);
            m4[1] = __uint_as_float(mu.x & 0xffff0000u);
            m4[2] = __uint_as_float(mu.y << 16);
            m4[3] = __uint_as_float(mu.y & 0xffff0000u);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float a = acc[nt][mt][r];
            if constexpr (RES) a = a + bl[mt][r] + m4[r];
            else if constexpr (!DGRAD) a = fmaxf(a + bl[mt][r], 0.f);
            else a = m4[r] > 0.f ? a : 0.f;
            v[r] = a;
          }
          uint2 w2;
          w2.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
          w2.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
          if (nt_out)
            __builtin_nontemporal_store((unsigned long long)w2.x | ((unsigned long long)w2.y << 32),
                                        reinterpret_cast<unsigned long long*>(out + o));
          else
            *reinterpret_cast<uint2*>(out + o) = w2;
        }
      }
    }
  }
}

// out[p] = bias + sum_{t, ci} W[0][ci][t] in[p + off(t)][ci] (C -> 1, FP32
// out), persistent over 64 x 8 pixel tiles staged in LDS with their halo as in
// k_conv_mfma (the next tile's input in flight during the MFMAs): a pixel's
// 3 x 3 neighbourhood then comes from LDS instead of nine 64-byte reads from
// the caches.  v_mfma_f32_16x16x32_bf16 per tap and 16 pixels: A = the tap's
// weights in row 0 (rows 1..15 zero), B = the input (32 channels x 16 pixels);
// row 0 of D (register 0 of lanes 0..15) holds the 16 outputs.  Wavefront w
// computes rows 2w, 2w+1 of the tile.
template <int C>
__global__ __launch_bounds__(256) void k_conv_out_tile(const bf16* in, const bf16* wt,
                                                       const bf16* bias, float* out, int B, int H,
                                                       int W) {
  static_assert(C == 32, "one K = 32 step per tap");
  constexpr int TX = kConvTX, TY = kConvTY, LX = TX + 2, LY = TY + 2;
  constexpr int CH = C / 8;                              // 16-byte chunks per pixel
  constexpr int NLD = (LY * LX * CH + 255) / 256;        // staged chunks per thread
  __shared__ __attribute__((aligned(16))) bf16 tin[LY * LX * C];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int tilesx = (W + TX - 1) / TX, tilesy = (H + TY - 1) / TY;
  const int per_img = tilesx * tilesy, ntiles = B * per_img;
  const long long HW = (long long)H * W;
  auto fetch = [&](int tile, uint4 (&pre)[NLD]) {
    const int b = tile / per_img, r0 = tile % per_img;
    const int ox = (r0 % tilesx) * TX, oy = (r0 / tilesx) * TY;
    const bf16* inb = in + (size_t)b * HW * C;
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int e = threadIdx.x + 256 * k;
      const int pix = e / CH, ch = e % CH;
      const int ly = pix / LX, lx = pix % LX;
      const int gy = oy + ly - 1, gx = ox + lx - 1;
      const bool ok = e < LY * LX * CH && gy >= 0 && gy < H && gx >= 0 && gx < W;
      pre[k] = ok ? *reinterpret_cast<const uint4*>(inb + ((long long)gy * W + gx) * C + ch * 8)
                  : make_uint4(0, 0, 0, 0);
    }
  };
  uint4 pre[NLD];
  int tile = blockIdx.x;
  if (tile < ntiles) fetch(tile, pre);                   // the first tile's loads go out first
  // A[i][k] = W[0][lg*8 + e][t] in row i = 0 (lanes li == 0), zero in the others
  bf16x8 wa[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    uint32_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = bf16_word_pick(wt, (long long)(lg * 8 + e) * 9 + t);
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = li == 0 ? h[e] : 0u;
    wa[t] = __builtin_bit_cast(bf16x8, make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16),
                                                  h[4] | (h[5] << 16), h[6] | (h[7] << 16)));
  }
  const float bv = bf2f((bf16)bf16_word_pick(bias, 0));
  for (; tile < ntiles; tile += gridDim.x) {
    __syncthreads();                                     // the previous tile's reads are done
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < LY * LX * CH) *reinterpret_cast<uint4*>(&tin[e * 8]) = pre[k];
    }
    __syncthreads();
    const int b = tile / per_img, r0 = tile % per_img;
    const int ox = (r0 % tilesx) * TX, oy = (r0 / tilesx) * TY;
    const int next = tile + gridDim.x;
    if (next < ntiles) fetch(next, pre);                 // in flight during the MFMAs
#pragma unroll 1
    for (int r2 = 0; r2 < 2; ++r2) {
      floatx4 acc[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int ly = wv * 2 + r2 + t / 3, kx = t % 3;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const int lx = nt * 16 + li + kx;
          const bf16x8 bx = __builtin_bit_cast(
              bf16x8, *reinterpret_cast<const uint4*>(&tin[(ly * LX + lx) * C + lg * 8]));
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[t], bx, acc[nt], 0, 0, 0);
        }
      }
      // D[i][p]: lane li + 16 lg holds rows 4 lg + r of pixel li; output channel 0
      // is register 0 of lanes 0..15
      const int y = oy + wv * 2 + r2;
      if (lg == 0 && y < H) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const int x = ox + nt * 16 + li;
          if (x < W) out[(size_t)b * HW + (long long)y * W + x] = acc[nt][0] + bv;
        }
      }
    }
  }
}

// Workgroups of a persistent MFMA convolution over B images of H x W.
inline int conv_grid(int B, int H, int W) {
  const long long tiles = (long long)B * ((W + kConvTX - 1) / kConvTX) * ((H + kConvTY - 1) / kConvTY);
  return (int)std::max<long long>(1, std::min<long long>(tiles, 512));
}

// Weight gradient of a C -> C convolution with NTAP taps (9: 3x3, 1: 1x1):
// per workgroup the partial dW[t][d][c] = sum_p dz[p][d] in[p + off(t)][c]
// over its tiles (persistent over 64 x 4 pixel tiles of all images) and the
// bias sums, on v_mfma_f32_16x16x32_bf16 with K = 32 pixels: A = dz^T (16
// output channels x 32 pixels), B = the shifted input (32 pixels x 16 input
// channels).  A lane's 8 K-elements are 8 consecutive pixels of one channel,
// so the tile is staged transposed ([channel][pixel]); the input twice,
// shifted by 0 and by 1 column, so that the fragment of every tap starts at
// an even column (four 4-byte LDS reads), the output gradient once (one
// 16-byte read).  Wavefront w accumulates output tile (d-tile w/2, c-tile
// w%2) for every tap.
template <int C, int NTAP>
__global__ __launch_bounds__(256) void k_wgrad_mfma(const bf16* in, const bf16* dz, float* part,
                                                    int B, int H, int W) {
  static_assert(C == 32, "the MFMA weight gradient is laid out for 32 channels");
  constexpr int TX = 64, TY = 4, LY = TY + 2;
  constexpr int NP = TX * TY;                    // tile pixels
  constexpr int PD = NP + 8;                     // dz^T pitch (elements)
  constexpr int PX = 74;                         // input row pitch: 66 columns + padding
  constexpr int PC = LY * PX;                    // input channel pitch
  __shared__ __attribute__((aligned(16))) bf16 dzT[C * PD];
  __shared__ __attribute__((aligned(16))) bf16 inT[2][C * PC];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int dt = wv >> 1, ct = wv & 1;
  floatx4 acc[NTAP];
#pragma unroll
  for (int t = 0; t < NTAP; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  const int tilesx = (W + TX - 1) / TX, tilesy = (H + TY - 1) / TY;
  const int per_img = tilesx * tilesy, ntiles = B * per_img;
  const long long HW = (long long)H * W;
  constexpr int CH = C / 8;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int b = tile / per_img, r0 = tile % per_img;
    const int ox = (r0 % tilesx) * TX, oy = (r0 / tilesx) * TY;
    const bf16* dzb = dz + (size_t)b * HW * C;
    const bf16* inb = in + (size_t)b * HW * C;
    // Every global load of the tile is issued before the first LDS write, at
    // clamped positions (values outside the grid replaced by zero).
    // dz^T: a unit = two adjacent pixels x 8 channels -> 8 channel rows, one dword each
    constexpr int UD = (NP / 2) * CH / 256;              // dz units per thread
    constexpr int NUI = NTAP == 9 ? LY * 33 * CH : TY * 32 * CH;
    constexpr int UI = (NUI + 255) / 256;                // input units per thread
    constexpr int LI = NTAP == 9 ? 3 : 2;                // loads per input unit
    static_assert((NP / 2) * CH % 256 == 0, "whole dz units per thread");
    uint4 dv[UD][2], iv[UI][LI];
#pragma unroll
    for (int s = 0; s < UD; ++s) {
      const int u = threadIdx.x + 256 * s;
      const int pr = u / CH, ch = u % CH;
      const int q = 2 * pr, qy = q / TX, qx = q % TX;
      const int gy = min(oy + qy, H - 1);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int gx = min(ox + qx + e, W - 1);
        dv[s][e] = *reinterpret_cast<const uint4*>(dzb + ((long long)gy * W + gx) * C + ch * 8);
      }
    }
#pragma unroll
    for (int s = 0; s < UI; ++s) {
      const int u = min(threadIdx.x + 256 * s, NUI - 1);
      const int ch = u % CH;
      if constexpr (NTAP == 9) {
        const int rk = u / CH, ly = rk / 33, k = rk % 33;
        const int gy = min(max(oy + ly - 1, 0), H - 1);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int gx = min(max(ox + 2 * k + e - 1, 0), W - 1);
          iv[s][e] = *reinterpret_cast<const uint4*>(inb + ((long long)gy * W + gx) * C + ch * 8);
        }
      } else {
        const int rk = u / CH, r = rk / 32, k = rk % 32;
        const int gy = min(oy + r, H - 1);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int gx = min(ox + 2 * k + e, W - 1);
          iv[s][e] = *reinterpret_cast<const uint4*>(inb + ((long long)gy * W + gx) * C + ch * 8);
        }
      }
    }
    __syncthreads();                                     // the previous tile's readers are done
#pragma unroll
    for (int s = 0; s < UD; ++s) {
      const int u = threadIdx.x + 256 * s;
      const int pr = u / CH, ch = u % CH;
      const int q = 2 * pr, qy = q / TX, qx = q % TX;
      const int gy = oy + qy, gx = ox + qx;
      const uint4 z = make_uint4(0, 0, 0, 0);
      const uint4 v0 = (gy < H && gx < W) ? dv[s][0] : z, v1 = (gy < H && gx + 1 < W) ? dv[s][1] : z;
      const uint32_t a0[4] = {v0.x, v0.y, v0.z, v0.w}, a1[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        // channels ch*8 + 2h (low halves) and ch*8 + 2h + 1 (high halves)
        *reinterpret_cast<uint32_t*>(&dzT[(ch * 8 + 2 * h) * PD + q]) = (a0[h] & 0xffffu) | (a1[h] << 16);
        *reinterpret_cast<uint32_t*>(&dzT[(ch * 8 + 2 * h + 1) * PD + q]) = (a0[h] >> 16) | (a1[h] & 0xffff0000u);
      }
    }
    // input^T.  1x1: the tile's own pixels only, in copy 1 (image column ox + h
    // at position h, the position the tap reads), two columns x 8 channels a
    // unit.  3x3: halo columns -1..64 of rows -1..TY: copy 0 holds halo column
    // h at position h, copy 1 at position h - 1; a unit = halo columns 2k,
    // 2k+1, 2k+2 of one row x 8 channels.
#pragma unroll
    for (int s = 0; s < UI; ++s) {
      const int u = threadIdx.x + 256 * s;
      if (u >= NUI) break;
      const int ch = u % CH;
      const uint4 z = make_uint4(0, 0, 0, 0);
      if constexpr (NTAP == 9) {
        const int rk = u / CH, ly = rk / 33, k = rk % 33;
        const int gy = oy + ly - 1;
        uint4 v[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int gx = ox + 2 * k + e - 1;
          v[e] = (2 * k + e < TX + 2 && gy >= 0 && gy < H && gx >= 0 && gx < W) ? iv[s][e] : z;
        }
        const uint32_t w0[4] = {v[0].x, v[0].y, v[0].z, v[0].w}, w1[4] = {v[1].x, v[1].y, v[1].z, v[1].w},
                       w2[4] = {v[2].x, v[2].y, v[2].z, v[2].w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int c0 = ch * 8 + 2 * h;
          const int o = ly * PX + 2 * k;
          *reinterpret_cast<uint32_t*>(&inT[0][c0 * PC + o]) = (w0[h] & 0xffffu) | (w1[h] << 16);
          *reinterpret_cast<uint32_t*>(&inT[0][(c0 + 1) * PC + o]) = (w0[h] >> 16) | (w1[h] & 0xffff0000u);
          *reinterpret_cast<uint32_t*>(&inT[1][c0 * PC + o]) = (w1[h] & 0xffffu) | (w2[h] << 16);
          *reinterpret_cast<uint32_t*>(&inT[1][(c0 + 1) * PC + o]) = (w1[h] >> 16) | (w2[h] & 0xffff0000u);
        }
      } else {
        const int rk = u / CH, r = rk / 32, k = rk % 32;
        const int gy = oy + r, gx = ox + 2 * k;
        const uint4 v1 = (gy < H && gx < W) ? iv[s][0] : z, v2 = (gy < H && gx + 1 < W) ? iv[s][1] : z;
        const uint32_t w1[4] = {v1.x, v1.y, v1.z, v1.w}, w2[4] = {v2.x, v2.y, v2.z, v2.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int c0 = ch * 8 + 2 * h, o = (r + 1) * PX + 2 * k;
          *reinterpret_cast<uint32_t*>(&inT[1][c0 * PC + o]) = (w1[h] & 0xffffu) | (w2[h] << 16);
          *reinterpret_cast<uint32_t*>(&inT[1][(c0 + 1) * PC + o]) = (w1[h] >> 16) | (w2[h] & 0xffff0000u);
        }
      }
    }
    __syncthreads();
    // K loop over chunks of 32 pixels (one tile row holds two)
#pragma unroll 1
    for (int chk = 0; chk < NP / 32; ++chk) {
      const int qy = chk >> 1, qx = (chk & 1) * 32 + lg * 8;     // this lane's 8 pixels
      const bf16x8 a = __builtin_bit_cast(
          bf16x8, *reinterpret_cast<const uint4*>(&dzT[(dt * 16 + li) * PD + qy * TX + qx]));
      if (ct == 0) {                                 // bias sums, once per output channel
        const uint4 au = __builtin_bit_cast(uint4, a);
        const uint32_t aw[4] = {au.x, au.y, au.z, au.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) bacc += __uint_as_float(aw[h] << 16) + __uint_as_float(aw[h] & 0xffff0000u);
      }
#pragma unroll
      for (int t = 0; t < NTAP; ++t) {
        const int ky = NTAP == 9 ? t / 3 : 1, kx = NTAP == 9 ? t % 3 : 1;
        // halo column of pixel qx under tap kx is qx + kx: copy kx & 1 at qx + (kx & 2)
        const bf16* src = &inT[kx & 1][(ct * 16 + li) * PC + (qy + ky) * PX + qx + (kx & 2)];
        const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src);
        const uint4 bu = make_uint4(s32[0], s32[1], s32[2], s32[3]);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, bu), acc[t], 0, 0, 0);
      }
    }
  }
  // D[i][j]: lane holds rows (d) dt*16 + 4*lg + r, column (c) ct*16 + li
  constexpr int STRIDE = NTAP * C * C + C;
  float* pb = part + (size_t)blockIdx.x * STRIDE;
#pragma unroll
  for (int t = 0; t < NTAP; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int d = dt * 16 + lg * 4 + r, c = ct * 16 + li;
      pb[(t * C + d) * C + c] = acc[t][r];
    }
  // bias: sum the four lane groups of channel dt*16 + li
  bacc += __shfl_xor(bacc, 16, 64);
  bacc += __shfl_xor(bacc, 32, 64);
  if (ct == 0 && lg == 0) pb[NTAP * C * C + dt * 16 + li] = bacc;
}

// ------------------------------------------------------------------ spectral layer
constexpr int kRowChunk = 256;                   // columns per staged chunk (WP's multiple)

// T[r][l][c] = sum_j Sx[l][j] x[r][j][c] for l < M (r = b H + i): the row
// transform of the spectral layer on v_mfma_f32_16x16x32_bf16, the FP32 basis
// taken as Sxh + Sxl (two BF16 products into FP32 accumulators; the split
// leaves 2^-17 of the basis, below the FP32 rounding of a row sum).  A = basis
// (16 modes x 32 columns, one 16-byte read per lane), B = the row (32 columns
// x 16 channels) from an LDS copy transposed to [channel][column], staged in
// chunks of 256 columns.  The four wavefronts take a quarter of every chunk;
// their partial products are added in a fixed order.  One workgroup per row.
template <int C>
__global__ __launch_bounds__(256) void k_spec_rows(const bf16* in, const bf16* Sxh, const bf16* Sxl,
                                                   float* T, int W, int WP, int M) {
  static_assert(C == 32, "two 16-channel tiles");
  constexpr int JC = kRowChunk, PJ = JC + 8, CH = C / 8, MTM = 2;
  __shared__ __attribute__((aligned(16))) bf16 xT[C * PJ];
  __shared__ float red[4][MTM * 2 * 4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int MT = (M + 15) / 16;
  const size_t row = blockIdx.x;
  const bf16* ip = in + row * W * C;
  floatx4 acc[MTM][2];
#pragma unroll
  for (int mt = 0; mt < MTM; ++mt)
    for (int ct = 0; ct < 2; ++ct) acc[mt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int j0 = 0; j0 < W; j0 += JC) {
    __syncthreads();                               // the previous chunk's reads are done
    // a unit = two adjacent columns x 8 channels -> 8 channel rows, one dword each
    for (int u = threadIdx.x; u < (JC / 2) * CH; u += 256) {
      const int pr = u / CH, ch = u % CH, q = 2 * pr, j = j0 + q;
      uint4 v0 = make_uint4(0, 0, 0, 0), v1 = v0;
      if (j < W) v0 = *reinterpret_cast<const uint4*>(ip + (size_t)j * C + ch * 8);
      if (j + 1 < W) v1 = *reinterpret_cast<const uint4*>(ip + (size_t)(j + 1) * C + ch * 8);
      const uint32_t a0[4] = {v0.x, v0.y, v0.z, v0.w}, a1[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        *reinterpret_cast<uint32_t*>(&xT[(ch * 8 + 2 * h) * PJ + q]) = (a0[h] & 0xffffu) | (a1[h] << 16);
        *reinterpret_cast<uint32_t*>(&xT[(ch * 8 + 2 * h + 1) * PJ + q]) =
            (a0[h] >> 16) | (a1[h] & 0xffff0000u);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < JC / 128; ++s) {           // this wavefront's 32-column steps
      const int jl = (wv * (JC / 128) + s) * 32;
      bf16x8 bx[2];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
        bx[ct] = __builtin_bit_cast(bf16x8,
                                    *reinterpret_cast<const uint4*>(&xT[(ct * 16 + li) * PJ + jl + 8 * lg]));
#pragma unroll
      for (int mt = 0; mt < MTM; ++mt) {
        if (mt >= MT) break;                       // uniform
        const size_t ao = (size_t)(mt * 16 + li) * WP + j0 + jl + 8 * lg;
        const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(Sxh + ao));
        const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(Sxl + ao));
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          acc[mt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bx[ct], acc[mt][ct], 0, 0, 0);
          acc[mt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bx[ct], acc[mt][ct], 0, 0, 0);
        }
      }
    }
  }
  // D[mode][channel]: lane holds modes mt*16 + 4 lg + r, channel ct*16 + li
#pragma unroll
  for (int mt = 0; mt < MTM; ++mt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wv][(mt * 2 + ct) * 4 + r][lane] = acc[mt][ct][r];
  __syncthreads();
  for (int e = threadIdx.x; e < MT * 2 * 4 * 64; e += 256) {
    const int ln = e & 63, slot = e >> 6;
    const int mt = slot >> 3, ct = (slot >> 2) & 1, r = slot & 3;
    const int mode = mt * 16 + 4 * (ln >> 4) + r, c = ct * 16 + (ln & 15);
    const float v = ((red[0][slot][ln] + red[1][slot][ln]) + red[2][slot][ln]) + red[3][slot][ln];
    if (mode < M) T[(row * M + mode) * C + c] = v;
  }
}

// Column transform of the spectral layer: X[b][k][q] = scale sum_i Sy[k][i]
// T[b][i][q] for q = l C + c < M C (the row-transformed activations), on the
// FP32 matrix cores (v_mfma_f32_16x16x4f32: lane t holds A[t % 16][t / 16]
// and B[t / 16][t % 16], register r of the result D[4 (t / 16) + r][t % 16]).
// A workgroup takes 16 modes k x 16 columns q of one image, its wavefront w
// the rows w*128.. of every chunk of 512 (A = the basis, zero past H; B =
// T), every load of a chunk issued before the first MFMA; the four partial
// tiles are added in LDS in a fixed order.  X ([b][k][l][c]) is kept for the
// mode mixing and its weight gradient.
__global__ __launch_bounds__(256) void k_spec_cols(const float* T, const float* Sy, float* X, int H,
                                                   int M, int LQ, float scale) {
  constexpr int NS = 32, IC = 16 * NS;
  __shared__ float part[4][16][16];
  const int nqb = (LQ + 15) / 16, nkb = (M + 15) / 16;
  const int qb = blockIdx.x % nqb, kb = (blockIdx.x / nqb) % nkb, b = blockIdx.x / (nqb * nkb);
  const int k0 = kb * 16, q0 = qb * 16;
  const int t = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = t % 16, kq = t / 16;
  const float* sr = Sy + (size_t)min(k0 + m, M - 1) * H;
  const float* tq = T + (size_t)b * H * LQ + min(q0 + m, LQ - 1);
  floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < H; c0 += IC) {
    const int iw = c0 + w * 4 * NS + kq;
    float a[NS], bb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = min(iw + 4 * s, H - 1);
      a[s] = sr[i];
      bb[s] = tq[(size_t)i * LQ];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) asm volatile("" : "+v"(a[s]), "+v"(bb[s]));
#pragma unroll
    for (int s = 0; s < NS; ++s)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(iw + 4 * s < H ? a[s] : 0.f, bb[s], acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) part[w][4 * kq + r][m] = acc[r];
  __syncthreads();
  const int mm = threadIdx.x / 16, nn = threadIdx.x % 16;
  const int k = k0 + mm, q = q0 + nn;
  if (k < M && q < LQ) {
    const float v = (part[0][mm][nn] + part[1][mm][nn]) + (part[2][mm][nn] + part[3][mm][nn]);
    X[((size_t)b * M + k) * LQ + q] = scale * v;
  }
}

// Mode mixing and inverse column transform of the spectral layer, one
// workgroup per (b, l, block of 64 rows), l the mode along x:
//   Y[k][n] = sum_m w[k][l][n][m] X[b][k][l][m]   (BWD: the transpose w[k][l][m][n])
//   Z[b][i][l][n] = alpha sum_k Sy[k][i] Y[k][n]  for the block's rows i.
// Every workgroup of a (b, l) forms the same Y (a few thousand operations),
// so that the rows spread over many workgroups.
template <int C, bool BWD>
__global__ __launch_bounds__(256) void k_spec_minv(const float* X, const bf16* wk, const float* Sy,
                                                   float* Z, int H, int M, float alpha) {
  static_assert(C == 32, "a channel per lane of a half-wavefront");
  constexpr int MM = 32, RB = 64, KPT = MM / 8;
  __shared__ float xl[MM][C];
  __shared__ float yl[MM][C];
  __shared__ float syl[MM][RB];
  const int nrb = (H + RB - 1) / RB;
  const int rb = blockIdx.x % nrb, bl = blockIdx.x / nrb;
  const int b = bl / M, l = bl % M, i0 = rb * RB;
  const int c = threadIdx.x & 31, ig = threadIdx.x >> 5;
  // X[b][k][l][:] and Sy[k][i0 .. i0 + 63] (zero past M or H), and this
  // thread's mixing weights, all loads issued together
  float xv[KPT], sv[MM * RB / 256];
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int k = ig + 8 * u;
    xv[u] = X[(((size_t)b * M + min(k, M - 1)) * M + l) * C + c];
  }
#pragma unroll
  for (int u = 0; u < MM * RB / 256; ++u) {
    const int e = threadIdx.x + 256 * u, k = e / RB, ii = e % RB;
    sv[u] = Sy[(size_t)min(k, M - 1) * H + min(i0 + ii, H - 1)];
  }
  uint32_t wv[KPT][16];
  uint32_t wb[KPT][C];
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int k = min(ig + 8 * u, M - 1);
    const bf16* wp = wk + ((size_t)k * M + l) * C * C;
    if constexpr (!BWD) {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const uint4 u4 = reinterpret_cast<const uint4*>(wp + c * C)[h];
        wv[u][4 * h] = u4.x;
        wv[u][4 * h + 1] = u4.y;
        wv[u][4 * h + 2] = u4.z;
        wv[u][4 * h + 3] = u4.w;
      }
    } else {
#pragma unroll
      for (int m = 0; m < C; ++m) wb[u][m] = *reinterpret_cast<const uint32_t*>(wp + m * C + (c & ~1));
    }
  }
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int k = ig + 8 * u;
    xl[k][c] = k < M ? xv[u] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < MM * RB / 256; ++u) {
    const int e = threadIdx.x + 256 * u, k = e / RB, ii = e % RB;
    syl[k][ii] = (k < M && i0 + ii < H) ? sv[u] : 0.f;
  }
  __syncthreads();
  // mixing: thread (n = c, modes k = ig + 8 u)
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int k = ig + 8 * u;
    float y = 0.f;
#pragma unroll
    for (int m = 0; m < C; ++m) {
      float wf;
      if constexpr (!BWD) {
        const uint32_t wd = wv[u][m >> 1];
        wf = __uint_as_float((m & 1) ? (wd & 0xffff0000u) : (wd << 16));
      } else {
        const uint32_t wd = wb[u][m];
        wf = __uint_as_float((c & 1) ? (wd & 0xffff0000u) : (wd << 16));
      }
      y = fmaf(wf, xl[k][m], y);
    }
    yl[k][c] = k < M ? y : 0.f;
  }
  __syncthreads();
  float yv[MM];
#pragma unroll
  for (int k = 0; k < MM; ++k) yv[k] = yl[k][c];
  const size_t tstride = (size_t)M * C;
  float* zb = Z + ((size_t)b * H * M + l) * C + c;
#pragma unroll 2
  for (int ii = ig; ii < RB; ii += 8) {
    if (i0 + ii >= H) break;
    float z = 0.f;
#pragma unroll
    for (int k = 0; k < MM; ++k) z = fmaf(syl[k][ii], yv[k], z);
    zb[(size_t)(i0 + ii) * tstride] = alpha * z;
  }
}

// dWk[k][l][d][c] = sum_b dY[b][k][l][d] X[b][k][l][c]
__global__ void k_spec_dwk(const float* dY, const float* X, float* gwk, int B, int M, int C) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)M * M * C * C;
  if (e >= total) return;
  const int c = (int)(e % C), d = (int)((e / C) % C);
  const long long kl = e / ((long long)C * C);
  float s = 0.f;
  for (int b = 0; b < B; ++b) {
    const long long base = ((long long)b * M * M + kl) * C;
    s += dY[base + d] * X[base + c];
  }
  gwk[e] = s;
}

// out[r][j][n] = epi( sum_m W1'[n][m] in[r][j][m] (+ bias[n]) + beta sum_l Sx[l][j] Z[r][l][n] )
// (r = b H + i): the spectral layer's output, 16 pixels x 32 channels per
// wavefront step, both terms into the same FP32 accumulators: the 1x1
// convolution on v_mfma_f32_16x16x32_bf16 (A = W1', 16 channels x 32 input
// channels; B = the input, 32 channels x 16 pixels, one 16-byte read per
// lane), the inverse row transform on v_mfma_f32_16x16x4_f32 (A = beta Z of
// the row, 16 channels x 4 modes; B = Sx, 4 modes x 16 pixels), in FP32.
// Forward: W1' = W1, bias, ReLU.  BWD: W1' = W1^T, no bias, times (mask > 0).
// A workgroup takes 64 pixels of one row.
template <int C, bool BWD, int MS>
__global__ __launch_bounds__(256) void k_spec_out(const bf16* in, const bf16* w1, const bf16* bias,
                                                  const float* Z, const float* Sx, const bf16* mask,
                                                  bf16* out, int W, int WP, int M, float beta) {
  static_assert(C == 32, "two 16-channel tiles");
  static_assert(MS >= 1 && MS <= 8, "modes <= 32 in steps of 4");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int tilesx = (W + 63) / 64;
  const size_t row = blockIdx.x / tilesx;
  const int j0 = (blockIdx.x % tilesx) * 64 + wv * 16;
  // A: W1'[n][m], n = nt*16 + li, m = 8 lg .. 8 lg + 7
  bf16x8 wa[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int n = nt * 16 + li;
    if constexpr (!BWD) {
      wa[nt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(w1 + n * C + 8 * lg));
    } else {
      // element n of rows 8 lg .. 8 lg + 7, read as the 32-bit words that hold it
      uint32_t wd[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) wd[e] = *reinterpret_cast<const uint32_t*>(w1 + (8 * lg + e) * C + (n & ~1));
      uint32_t pk[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const uint32_t lo = (n & 1) ? (wd[2 * h] >> 16) : (wd[2 * h] & 0xffffu);
        const uint32_t hi = (n & 1) ? (wd[2 * h + 1] >> 16) : (wd[2 * h + 1] & 0xffffu);
        pk[h] = lo | (hi << 16);
      }
      wa[nt] = __builtin_bit_cast(bf16x8, make_uint4(pk[0], pk[1], pk[2], pk[3]));
    }
  }
  // A2: beta Z[row][mode][n], mode = 4 s + lg (zero past M; loads at clamped
  // modes, all in flight together)
  float za[MS][2];
#pragma unroll
  for (int s = 0; s < MS; ++s)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int mode = 4 * s + lg;
      const float zv = Z[(row * M + min(mode, M - 1)) * C + nt * 16 + li];
      za[s][nt] = mode < M ? beta * zv : 0.f;
    }
  if (j0 >= W) return;                           // wavefront-uniform
  // B: input channels 8 lg .. 8 lg + 7 of pixel j0 + li (zero past the row)
  const int j = j0 + li;
  const size_t px = (row * W + (j < W ? j : W - 1)) * C;
  const bf16x8 bx = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(in + px + 8 * lg));
  floatx4 acc[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[nt], bx, acc[nt], 0, 0, 0);
  }
#pragma unroll
  for (int s = 0; s < MS; ++s) {
    const float sb = Sx[(size_t)(4 * s + lg) * WP + j];   // in bounds: WP >= W rounded to 64
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(za[s][nt], sb, acc[nt], 0, 0, 0);
  }
  if (j >= W) return;
  // D[n][p]: lane holds channels nt*16 + 4 lg + r of pixel j0 + li
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const size_t o = px + nt * 16 + 4 * lg;
    float m4[4] = {0.f, 0.f, 0.f, 0.f};
    if constexpr (BWD) {
      const uint2 mu = *reinterpret_cast<const uint2*>(mask + o);
      m4[0] = __uint_as_float(mu.x << 16);
      m4[1] = __uint_as_float(mu.x & 0xffff0000u);
      m4[2] = __uint_as_float(mu.y << 16);
      m4[3] = __uint_as_float(mu.y & 0xffff0000u);
    }
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float a = acc[nt][r];
      if constexpr (!BWD) a = fmaxf(a + bf2f(bias[nt * 16 + 4 * lg + r]), 0.f);
      else a = m4[r] > 0.f ? a : 0.f;
      v[r] = a;
    }
    uint2 w2;
    w2.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
    w2.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
    if constexpr (!BWD)   // the forward layer's output goes out non-temporal (faster at batch 1
                          // and 8; the input-gradient form is slower with it)
      __builtin_nontemporal_store((unsigned long long)w2.x | ((unsigned long long)w2.y << 32),
                                  reinterpret_cast<unsigned long long*>(out + o));
    else
      *reinterpret_cast<uint2*>(out + o) = w2;
  }
}

// k_spec_out for M modes (4-mode steps as a template argument, so that the
// step loop has no early exit and its loads are issued together).
template <int C, bool BWD>
void launch_spec_out(dim3 grid, hipStream_t s, const bf16* in, const bf16* w1, const bf16* bias,
                     const float* Z, const float* Sx, const bf16* mask, bf16* out, int W, int WP,
                     int M, float beta) {
  switch ((M + 3) / 4) {
#define MLG_SPEC_OUT(MS)                                                                        \
  case MS:                                                                                      \
    k_spec_out<C, BWD, MS><<<grid, 256, 0, s>>>(in, w1, bias, Z, Sx, mask, out, W, WP, M, beta); \
    break;
    MLG_SPEC_OUT(1) MLG_SPEC_OUT(2) MLG_SPEC_OUT(3) MLG_SPEC_OUT(4)
    MLG_SPEC_OUT(5) MLG_SPEC_OUT(6) MLG_SPEC_OUT(7) MLG_SPEC_OUT(8)
#undef MLG_SPEC_OUT
    default: throw ArgError{MLG_ERR_ARG, "modes must be in 1..32"};
  }
}

// ------------------------------------------------------------------ band path (FP64)
// FP64 throughout: the residual of a slowly moving source is dipole-like, so
// its projection on the slowest modes cancels heavily, and FP32 sums (or an
// FP32-rounded basis) leave errors in the mode coefficients comparable to the
// coefficients themselves; trained on such inputs the gains settle below the
// exact inverse.  The four transforms of the band (rows, columns, inverse
// with the band weights, output) are dense FP64 products of the field with
// the sine basis, run on the FP64 matrix cores in 16 x 16 tiles: both
// operands come from registers (loaded straight from memory, every load of
// a wavefront's batch issued before its first MFMA), which leaves the LDS to
// the fixed-order sum of the wavefronts' partial tiles.  The row and output
// transforms also have a vector form (8 rows per workgroup, all modes),
// faster once a launch has enough rows to fill the device.  Up to two
// independent fields per launch (blockIdx.y).
typedef double doublex4 __attribute__((ext_vector_type(4)));

// D(16 x 16) += A(16 x 4) B(4 x 16) in FP64 on the matrix cores: lane t holds
// A[t % 16][t / 16] and B[t / 16][t % 16]; register r of D holds
// D[4 r + t / 16][t % 16] (rows interleaved over the four lane groups).
__device__ __forceinline__ doublex4 mfma_f64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// MFMA steps (4 terms each) per wavefront and batch of loads.
constexpr int kBandSteps = 32;

// Every value of a batch of loads counts as used here, in order, before the
// first MFMA: the whole batch is in flight at once (left to itself the
// compiler issues each load next to its MFMA and waits for it there).
template <int N>
__device__ __forceinline__ void band_batch_fence(double (&a)[N], double (&b)[N]) {
#pragma unroll
  for (int s = 0; s < N; ++s) asm volatile("" : "+v"(a[s]), "+v"(b[s]));
}

// One field's operand of a band launch: the data, its per-image divisor (or
// NULL), the result, a scale.
template <class X>
struct BandIn {
  const X* x;
  const double* div;
  double* out;
  double scale;
};

// The four wavefronts' 16 x 16 partial tiles (register r of lane t of
// wavefront w at part[w][4 r + t / 16][t % 16]), summed in a fixed order:
// returns element (e / 16, e % 16) for e = threadIdx.x.
__device__ __forceinline__ double band_tile_sum(double (*part)[16][16], const doublex4& acc) {
  const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < 4; ++r) part[w][4 * r + t / 16][t % 16] = acc[r];
  __syncthreads();
  const int m = threadIdx.x / 16, n = threadIdx.x % 16;
  return (part[0][m][n] + part[1][m][n]) + (part[2][m][n] + part[3][m][n]);
}

// T[b][i][l] = scale (sum_j x[b][i][j] SxT[j][l]) / div[b]: a workgroup takes
// 16 rows x 16 modes of one image, its wavefront w the columns w*128.. of
// every chunk of 512 (32 steps: A = the rows' values, zero past the grid;
// B = the basis).
template <class X0, class X1>
__global__ __launch_bounds__(256) void k_band_rows(BandIn<X0> f0, BandIn<X1> f1, const double* SxT,
                                                   int H, int W, int K) {
  constexpr int NS = kBandSteps, JC = 16 * NS;
  __shared__ double part[4][16][16];
  const int nlb = (K + 15) / 16, nrb = (H + 15) / 16;
  const int lb = blockIdx.x % nlb, rb = (blockIdx.x / nlb) % nrb, b = blockIdx.x / (nlb * nrb);
  const int i0 = rb * 16, l0 = lb * 16;
  const int t = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = t % 16, kq = t / 16;
  auto run = [&](const auto& f) {
    const auto* xr = f.x + ((size_t)b * H + min(i0 + m, H - 1)) * W;
    const double* sb = SxT + min(l0 + m, K - 1);
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int j0 = 0; j0 < W; j0 += JC) {
      const int jw = j0 + w * 4 * NS + kq;
      double a[NS], bb[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int j = min(jw + 4 * s, W - 1);
        a[s] = (double)xr[j];
        bb[s] = sb[(size_t)j * K];
      }
      band_batch_fence(a, bb);
#pragma unroll
      for (int s = 0; s < NS; ++s) acc = mfma_f64(jw + 4 * s < W ? a[s] : 0.0, bb[s], acc);
    }
    const double v = band_tile_sum(part, acc);
    const int i = i0 + threadIdx.x / 16, l = l0 + threadIdx.x % 16;
    if (i < H && l < K) {
      double o = v;
      if (f.div) o /= f.div[b];
      f.out[((size_t)b * H + i) * K + l] = f.scale * o;
    }
  };
  if (blockIdx.y == 0) run(f0);
  else run(f1);
}

// The row transform on the vector units, for launches with enough rows to
// fill the device (a batch of training pairs): a workgroup takes 8 rows of
// one image and all modes, so every basis value it loads serves all 8 rows.
constexpr int kBandRows = 8;

// T[b][i][l] = sum_j SxT[j][l] x[b][i][j] / div[b]: a workgroup takes 8 rows
// of one image; lanes are the modes l (64 per pass, two passes at most), the
// four wavefronts a quarter of every chunk of 256 columns.  The rows are
// staged in LDS (FP64, zero past the grid), so the inner loop reads basis
// values (16 independent coalesced loads issued together, at clamped
// indices) and broadcast LDS values, eight running sums per lane and pass;
// the quarters are added in a fixed order.
constexpr int kBandChunk = 256;

template <class X0, class X1>
__global__ __launch_bounds__(256) void k_band_rows_vec(BandIn<X0> f0, BandIn<X1> f1,
                                                       const double* SxT, int H, int W, int K) {
  constexpr int JC = kBandChunk, JQ = JC / 4, NB = 16, PER = kBandRows * JC / 256;
  __shared__ double xs[kBandRows][JC];
  __shared__ double part[4][kBandRows][64];
  const int nrb = (H + kBandRows - 1) / kBandRows;
  const int b = blockIdx.x / nrb, i0 = (blockIdx.x % nrb) * kBandRows;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rlast = min(kBandRows, H - i0) - 1;
  const int np = (K + 63) / 64;
  auto run = [&](const auto& f) {
    const auto* xb = f.x + ((size_t)b * H + i0) * W;
    double s[2][kBandRows];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int r = 0; r < kBandRows; ++r) s[p][r] = 0.0;
    for (int j0 = 0; j0 < W; j0 += JC) {
      double xv[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + 256 * u, r = e / JC, jj = e % JC;
        xv[u] = (double)xb[(size_t)min(r, rlast) * W + min(j0 + jj, W - 1)];
      }
      __syncthreads();                                   // the previous chunk's readers are done
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + 256 * u, r = e / JC, jj = e % JC;
        xs[r][jj] = (r <= rlast && j0 + jj < W) ? xv[u] : 0.0;
      }
      __syncthreads();
      const int ja = j0 + w * JQ;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if (p >= np) break;                              // uniform
        const int lc = min(p * 64 + lane, K - 1);
#pragma unroll 1
        for (int jb = 0; jb < JQ; jb += NB) {
          double bv[NB];
#pragma unroll
          for (int u = 0; u < NB; ++u) bv[u] = SxT[(size_t)min(ja + jb + u, W - 1) * K + lc];
#pragma unroll
          for (int u = 0; u < NB; ++u)
#pragma unroll
            for (int r = 0; r < kBandRows; ++r) s[p][r] = fma(bv[u], xs[r][w * JQ + jb + u], s[p][r]);
        }
      }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p >= np) break;
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kBandRows; ++r) part[w][r][lane] = s[p][r];
      __syncthreads();
      for (int e = threadIdx.x; e < kBandRows * 64; e += 256) {
        const int r = e / 64, ln = e % 64, ll = p * 64 + ln;
        if (r > rlast || ll >= K) continue;
        double v = (part[0][r][ln] + part[1][r][ln]) + (part[2][r][ln] + part[3][r][ln]);
        if (f.div) v /= f.div[b];
        f.out[((size_t)b * H + i0 + r) * K + ll] = f.scale * v;
      }
    }
  };
  if (blockIdx.y == 0) run(f0);
  else run(f1);
}

// X[b][k][q] = scale sum_i Sy[k][i] T[b][i][q] (k, q < K): a workgroup takes
// 16 x 16 of (k, q) of one image, its wavefront w the rows w*128.. of every
// chunk of 512 (A = the basis, zero past the grid; B = T).
__global__ __launch_bounds__(256) void k_band_cols(BandIn<double> f0, BandIn<double> f1,
                                                   const double* Sy, int H, int K) {
  constexpr int NS = kBandSteps, IC = 16 * NS;
  __shared__ double part[4][16][16];
  const int nkb = (K + 15) / 16;
  const int qb = blockIdx.x % nkb, kb = (blockIdx.x / nkb) % nkb, b = blockIdx.x / (nkb * nkb);
  const int k0 = kb * 16, q0 = qb * 16;
  const int t = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = t % 16, kq = t / 16;
  const BandIn<double>& f = blockIdx.y == 0 ? f0 : f1;
  const double* sr = Sy + (size_t)min(k0 + m, K - 1) * H;
  const double* tq = f.x + (size_t)b * H * K + min(q0 + m, K - 1);
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < H; c0 += IC) {
    const int iw = c0 + w * 4 * NS + kq;
    double a[NS], bb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = min(iw + 4 * s, H - 1);
      a[s] = sr[i];
      bb[s] = tq[(size_t)i * K];
    }
    band_batch_fence(a, bb);
#pragma unroll
    for (int s = 0; s < NS; ++s) acc = mfma_f64(iw + 4 * s < H ? a[s] : 0.0, bb[s], acc);
  }
  const double v = band_tile_sum(part, acc);
  const int k = k0 + threadIdx.x / 16, q = q0 + threadIdx.x % 16;
  if (k < K && q < K) f.out[((size_t)b * K + k) * K + q] = f.scale * v;
}

// The convolutional branch's output gain: sct / scc, 1 before any data (or
// without a gain: gate == NULL).
__device__ __forceinline__ double gate_of(const double* gate) {
  return gate && gate[1] > 0.0 ? gate[0] / gate[1] : 1.0;
}

// Z[b][i][l] = alpha sum_k Sy[k][i] Y[b][k][l], with the band applied on the
// way in when `band` is given: Y = w_kl X - g Cc (w = sxt / sxx, 0 where sxx =
// 0; g the output gain), else Y = X.  A workgroup takes 16 rows x 16 modes l
// of one image, its wavefront w the modes k = w*16.. of every chunk of 64 (A
// = the basis, B = Y, zero past the band).
__global__ __launch_bounds__(256) void k_band_inv(const double* X, const double* Cc,
                                                  const double* band, const double* gate,
                                                  const double* Sy, double* Z, int H, int K,
                                                  double alpha) {
  constexpr int NS = 4, KC = 16 * NS;
  __shared__ double part[4][16][16];
  const int nlb = (K + 15) / 16, nrb = (H + 15) / 16;
  const int lb = blockIdx.x % nlb, rb = (blockIdx.x / nlb) % nrb, b = blockIdx.x / (nlb * nrb);
  const int i0 = rb * 16, l0 = lb * 16;
  const int t = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = t % 16, kq = t / 16;
  const double g = gate_of(gate);
  const int ic = min(i0 + m, H - 1), lc = min(l0 + m, K - 1);
  const double* Xb = X + (size_t)b * K * K;
  const double* Cb = Cc ? Cc + (size_t)b * K * K : nullptr;
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < K; c0 += KC) {
    const int kw = c0 + w * 4 * NS + kq;
    double a[NS], y[NS];
    if (band) {
      double cv[NS], tv[NS], qv[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int k = min(kw + 4 * s, K - 1);
        a[s] = Sy[(size_t)k * H + ic];
        y[s] = Xb[k * K + lc];
        cv[s] = Cb[k * K + lc];
        tv[s] = band[k * K + lc];
        qv[s] = band[K * K + k * K + lc];
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double wk = qv[s] > 0.0 ? tv[s] / qv[s] : 0.0;
        y[s] = wk * y[s] - g * cv[s];
      }
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int k = min(kw + 4 * s, K - 1);
        a[s] = Sy[(size_t)k * H + ic];
        y[s] = Xb[k * K + lc];
      }
    }
    band_batch_fence(a, y);
#pragma unroll
    for (int s = 0; s < NS; ++s) acc = mfma_f64(a[s], kw + 4 * s < K ? y[s] : 0.0, acc);
  }
  const double v = band_tile_sum(part, acc);
  const int i = i0 + threadIdx.x / 16, l = l0 + threadIdx.x % 16;
  if (i < H && l < K) Z[((size_t)b * H + i) * K + l] = alpha * v;
}

// out[b][i][j] = g out[b][i][j] + beta sum_l Sx[l][j] Z[b][i][l] (sum and add in
// FP64; g the output gain, 1 without one): a workgroup takes 16 rows x 64
// columns of one image, its wavefront w the 16 columns w*16.., lane group g
// the 16 consecutive modes 16g.. of every 64 (A = the rows' Z, read along
// the row and zero past the band; B = the basis); the output values and a
// band of up to 64 modes are loaded in one batch.  Up to two fields
// (blockIdx.y).
struct BandOut {
  const double* Z;
  float* out;
  const double* gate;
  double beta;
};

// The guess written by the output transform's epilogue (inference): guess =
// u_prev + (s_r / c_u) out, from the stored FP32 output value (the same
// arithmetic as k_guess).
struct GuessOut {
  Ptrs u;
  MPtrs g;
  const double* s;
};
struct NoGuess {};

template <bool GUESS>
__global__ __launch_bounds__(256) void k_band_out(BandOut f0, BandOut f1, const double* Sx, int H,
                                                  int W, int K,
                                                  std::conditional_t<GUESS, GuessOut, NoGuess> go) {
  constexpr int NS = 16;
  const BandOut& f = blockIdx.y == 0 ? f0 : f1;
  const int ncb = (W + 63) / 64, nrb = (H + 15) / 16;
  const int cb = blockIdx.x % ncb, rb = (blockIdx.x / ncb) % nrb, b = blockIdx.x / (ncb * nrb);
  const int t = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int m = t % 16, kq = t / 16;
  const int i0 = rb * 16, j = cb * 64 + w * 16 + m;
  const int jc = min(j, W - 1);
  float ov[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) ov[r] = f.out[((size_t)b * H + min(i0 + 4 * r + kq, H - 1)) * W + jc];
  const double* zr = f.Z + ((size_t)b * H + min(i0 + m, H - 1)) * K;
  const double* sc = Sx + jc;
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < K; c0 += 4 * NS) {
    double a[NS], bb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int l = min(c0 + 4 * s + kq, K - 1);
      a[s] = zr[l];
      bb[s] = sc[(size_t)l * W];
    }
    band_batch_fence(a, bb);
#pragma unroll
    for (int s = 0; s < NS; ++s) acc = mfma_f64(c0 + 4 * s + kq < K ? a[s] : 0.0, bb[s], acc);
  }
  if (j >= W) return;
  const double g = gate_of(f.gate);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 4 * r + kq;
    if (i < H) {
      const float o = (float)(g * (double)ov[r] + f.beta * acc[r]);
      f.out[((size_t)b * H + i) * W + j] = o;
      if constexpr (GUESS) {
        const size_t q = (size_t)i * W + j;
        go.g.p[b][q] = go.u.p[b][q] + (go.s[b] / kCu) * (double)o;
      }
    }
  }
}

// The output transform on the vector units, for launches with enough rows
// to fill the device: a workgroup takes 8 rows x 256 columns of one image, a
// thread one column and its eight rows (eight running sums, so every basis
// value serves eight rows); the rows' Z values come through LDS.
__global__ __launch_bounds__(256) void k_band_out_vec(BandOut f0, BandOut f1, const double* Sx,
                                                      int H, int W, int K) {
  constexpr int KMAX = 128, NB = 16, PZ = kBandRows * KMAX / 256;
  __shared__ double zl[kBandRows][KMAX];
  const BandOut& f = blockIdx.y == 0 ? f0 : f1;
  const int ncb = (W + 255) / 256, nrb = (H + kBandRows - 1) / kBandRows;
  const int cb = blockIdx.x % ncb, rb = (blockIdx.x / ncb) % nrb, b = blockIdx.x / (ncb * nrb);
  const int j = cb * 256 + threadIdx.x, i0 = rb * kBandRows;
  const int jc = j < W ? j : W - 1;
  const int rlast = min(kBandRows, H - i0) - 1;
  const double* zb = f.Z + ((size_t)b * H + i0) * K;
  double zv[PZ];
#pragma unroll
  for (int u = 0; u < PZ; ++u) {
    const int e = threadIdx.x + 256 * u, r = e / KMAX, l = e % KMAX;
    zv[u] = zb[(size_t)min(r, rlast) * K + min(l, K - 1)];
  }
#pragma unroll
  for (int u = 0; u < PZ; ++u) {
    const int e = threadIdx.x + 256 * u, r = e / KMAX, l = e % KMAX;
    zl[r][l] = (r <= rlast && l < K) ? zv[u] : 0.0;         // zero past K: padded steps add 0
  }
  __syncthreads();
  double s[kBandRows];
#pragma unroll
  for (int r = 0; r < kBandRows; ++r) s[r] = 0.0;
  const double* sx = Sx + jc;
  const int KP = (K + NB - 1) / NB * NB;
#pragma unroll 1
  for (int l0 = 0; l0 < KP; l0 += NB) {
    double sv[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) sv[u] = sx[(size_t)min(l0 + u, K - 1) * W];
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
      for (int r = 0; r < kBandRows; ++r) s[r] = fma(zl[r][l0 + u], sv[u], s[r]);
  }
  if (j >= W) return;
  const double g = gate_of(f.gate);
  float* ob = f.out + ((size_t)b * H + i0) * W + j;
  float ov[kBandRows];
#pragma unroll
  for (int r = 0; r < kBandRows; ++r) ov[r] = ob[(size_t)min(r, rlast) * W];
#pragma unroll
  for (int r = 0; r < kBandRows; ++r)
    if (r <= rlast) ob[(size_t)r * W] = (float)(g * (double)ov[r] + f.beta * s[r]);
}

// Least-squares state of the band: sxt_kl += sum_b X[b][k][l] T[b][k][l],
// sxx_kl += sum_b X[b][k][l]^2 (samples added in order)
__global__ void k_band_fit(const double* X, const double* T, double* band, int B, int K) {
  const int kl = blockIdx.x * blockDim.x + threadIdx.x;
  if (kl >= K * K) return;
  double xt = band[kl], xx = band[K * K + kl];
  for (int b = 0; b < B; ++b) {
    const double x = X[(size_t)b * K * K + kl];
    xt += x * T[(size_t)b * K * K + kl];
    xx += x * x;
  }
  band[kl] = xt;
  band[K * K + kl] = xx;
}

// Sums of c c and c d over a batch of fields (per-workgroup partials; the
// first 2 * gridDim.x entries of part).
__global__ __launch_bounds__(256) void k_gate_sums(const float* c, const float* d, long long n,
                                                   double* part) {
  __shared__ double red[2][4];
  double cc = 0.0, cd = 0.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n;
       e += (long long)gridDim.x * 256) {
    const double x = c[e];
    cc += x * x;
    cd += x * (double)d[e];
  }
  cc = wave_sum(cc);
  cd = wave_sum(cd);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = cc;
    red[1][threadIdx.x >> 6] = cd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
    part[2 * blockIdx.x + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  }
}

// Output gain state: with cc = sum |c|^2 and cd = sum <c, dout> of this
// batch (dout = (2/B)(c - t) off the band), sum <c, t> = cc - (B/2) cd; both
// running sums decay by kGateDecay per training step, so that the gain
// follows the branch as it trains.
constexpr double kGateDecay = 0.9;
__global__ void k_gate_fin(const double* part, int nblk, double* gate, int B) {
  // one wavefront: lane l sums partials l, l + 64, ... in order, then the
  // lanes are added in a fixed tree
  const int lane = threadIdx.x & 63;
  if (blockIdx.x != 0 || threadIdx.x >= 64) return;
  double cc = 0.0, cd = 0.0;
  for (int b = lane; b < nblk; b += 64) {
    cc += part[2 * b];
    cd += part[2 * b + 1];
  }
  cc = wave_sum(cc);
  cd = wave_sum(cd);
  if (lane == 0) {
    gate[0] = kGateDecay * gate[0] + (cc - 0.5 * B * cd);
    gate[1] = kGateDecay * gate[1] + cc;
  }
}

// The exact training pair of the band for the correction d = u_t - u_prev:
// t = c_u d (the target before its division by s_r) and a = A d with the
// solver's operator (zero Dirichlet, h = 1/(N+1)), d formed in FP64.
__global__ void k_pair(Ptrs ut, Ptrs up, double* t, double* a, int H, int W) {
  const int b = blockIdx.y;
  const long long HW = (long long)H * W;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HW) return;
  const int y = (int)(p / W), x = (int)(p % W);
  const double* u1 = ut.p[b];
  const double* u0 = up.p[b];
  auto d = [&](long long q) { return u1[q] - u0[q]; };
  const double cx = (double)(W + 1) * (W + 1), cy = (double)(H + 1) * (H + 1);
  const double c = d(p);
  const double w = x > 0 ? d(p - 1) : 0.0, e = x < W - 1 ? d(p + 1) : 0.0;
  const double sN = y > 0 ? d(p - W) : 0.0, nN = y < H - 1 ? d(p + W) : 0.0;
  t[(size_t)b * HW + p] = kCu * c;
  a[(size_t)b * HW + p] = (2.0 * c - w - e) * cx + (2.0 * c - sN - nN) * cy;
}

// ------------------------------------------------------------------ parameters
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

template <int NT>
struct InitSpecT {
  int64_t off[NT + 1];
  int64_t size[NT];
  float bound[NT];    // 0 -> zero tensor
};
using InitSpec = InitSpecT<kNumTensors>;

// He-uniform weights from a counter-based generator (SplitMix64 of seed and
// element index), zero biases and output layer, zero Adam state and grads.
template <int NT>
__global__ void k_init_params(float* master, float* grad, float* m, float* v, bf16* bf,
                              long long* step, InitSpecT<NT> spec, int ntensors, int64_t P,
                              uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) *step = 0;
  if (e >= P) return;
  int t = 0;
  while (t < ntensors - 1 && e >= spec.off[t + 1]) ++t;
  float val = 0.f;
  if (spec.bound[t] > 0.f && e < spec.off[t] + spec.size[t]) {
    const uint64_t r = splitmix64(seed * 0x100000001B3ull + (uint64_t)e);
    const double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);   // [0, 1)
    val = (float)((2.0 * u - 1.0) * spec.bound[t]);
  }
  master[e] = val;
  grad[e] = 0.f;
  m[e] = 0.f;
  v[e] = 0.f;
  bf[e] = f2bf(val);
}

__global__ void k_refresh(const float* master, float* grad, float* m, float* v, bf16* bf,
                          long long* step, int64_t P) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) *step = 0;
  if (e >= P) return;
  grad[e] = 0.f;
  m[e] = 0.f;
  v[e] = 0.f;
  bf[e] = f2bf(master[e]);
}

__global__ void k_step_inc(long long* step) {
  if (threadIdx.x == 0) *step += 1;
}

// Adam (Kingma & Ba) with bias correction on the FP32 master weights; the BF16
// working copy is refreshed in the same pass.
__global__ void k_adam(float* master, const float* grad, float* m, float* v, bf16* bf,
                       const long long* step, int64_t P, float lr, float b1, float b2, float eps) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P) return;
  const double t = (double)*step;
  const float c1 = (float)(1.0 - pow((double)b1, t));
  const float c2 = (float)(1.0 - pow((double)b2, t));
  const float g = grad[e];
  const float mm = b1 * m[e] + (1.f - b1) * g;
  const float vv = b2 * v[e] + (1.f - b2) * g * g;
  m[e] = mm;
  v[e] = vv;
  const float p = master[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  master[e] = p;
  bf[e] = f2bf(p);
}

// ------------------------------------------------------------------ host helpers
inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// Workgroups per image of the input convolution, which loops over the
// image's 256-pixel blocks: at most 2048 over the batch (measured at 512²: a
// batch of 8 with 256 per image ran it in 49 µs against 61 µs with one
// workgroup per block, while a single image keeps one per block, 1024).  The
// output-gradient convolution keeps one workgroup per block (capped it ran
// 78 against 69 µs).
constexpr int kPixelBlocksTotal = 2048;
inline int pixel_blocks(long long hw, int B) {
  return (int)std::max<long long>(1, std::min<long long>(cdiv(hw, 256), kPixelBlocksTotal / B));
}

// The network inputs of a batch: residuals r0 (FP64), their and the sources'
// RMS in sv, and the normalised two-channel BF16 input x0; with `bases`, the
// same launch fills the sine bases.
static void normalise_inputs(const Ptrs& f, const Ptrs& u, double* r0, double* rms_part, double* sv,
                             bf16* x0, int B, int H, int W, hipStream_t s,
                             const Bases* bases = nullptr) {
  const long long HW = (long long)H * W;
  const Bases o = bases ? *bases : Bases{};
  const long long nb = bases ? bases_count(o) : 0;
  k_resid_sumsq<<<dim3(kRmsBlocks, 2 * B + (bases ? 1 : 0)), 256, 0, s>>>(f, u, r0, B, H, W,
                                                                          rms_part, o, nb);
  k_norm_in<<<dim3(cdiv(HW, 256), B), 256, 0, s>>>(r0, f, rms_part, sv, B, x0, HW);
}

struct Net {
  Dims d;
  ParamLayout pl;
  WsLayout wl;
  char* params;
  char* ws;
  const bf16* bfw(int t) const { return (const bf16*)(params + pl.bf) + pl.off[t]; }
  const float* master(int t) const { return (const float*)(params + pl.master) + pl.off[t]; }
  float* grad(int t) const { return (float*)(params + pl.grad) + pl.off[t]; }
  template <class T>
  T* w(size_t off) const { return (T*)(ws + off); }
};

// The band path's workspace views.
struct BandSpace {
  double *kT, *kT2, *kX, *kC, *kZ, *kZ2, *kdY, *kdY2, *kTc, *kXa, *kSx, *kSxT, *kSy;
};

BandSpace band_space(const Net& n) {
  auto p = [&](size_t off) { return n.w<double>(off); };
  return BandSpace{p(n.wl.kT),   p(n.wl.kT2), p(n.wl.kX),  p(n.wl.kC),   p(n.wl.kZ),
                   p(n.wl.kZ2),  p(n.wl.kdY), p(n.wl.kdY2), p(n.wl.kTc), p(n.wl.kXa),
                   p(n.wl.kSx),  p(n.wl.kSxT), p(n.wl.kSy)};
}

// Launch shapes of the band kernels: 16 x 16 tiles (rows x modes, modes x
// modes), 16 x 64 output tiles; up to two fields as blockIdx.y.
inline dim3 band_rows_grid(const Dims& d) { return dim3(d.B * cdiv(d.H, 16) * cdiv(d.K, 16), 2); }
inline dim3 band_cols_grid(const Dims& d) { return dim3(d.B * cdiv(d.K, 16) * cdiv(d.K, 16), 2); }
inline dim3 band_inv_grid(const Dims& d) { return dim3(d.B * cdiv(d.H, 16) * cdiv(d.K, 16)); }
inline dim3 band_out_grid(const Dims& d, int fields) {
  return dim3(d.B * cdiv(d.H, 16) * cdiv(d.W, 64), fields);
}

// The row and output transforms run on the vector units when their 8-row
// workgroups alone fill the 256 compute units (a training batch at the
// benchmark's size), and on the matrix cores otherwise (inference of one
// field, where the vector form would leave most of the device idle).
inline bool band_vector(const Dims& d) { return (long long)d.B * cdiv(d.H, kBandRows) >= 256; }

// With `go` (inference of one field), the matrix-core form also writes the
// guess; returns whether it did.
bool launch_band_out(hipStream_t s, const Dims& d, int fields, BandOut f0, BandOut f1,
                     const double* Sx, const GuessOut* go = nullptr) {
  if (band_vector(d)) {
    k_band_out_vec<<<dim3(d.B * cdiv(d.H, kBandRows) * cdiv(d.W, 256), fields), 256, 0, s>>>(
        f0, f1, Sx, d.H, d.W, d.K);
    return false;
  }
  if (go) {
    k_band_out<true><<<band_out_grid(d, fields), 256, 0, s>>>(f0, f1, Sx, d.H, d.W, d.K, *go);
    return true;
  }
  k_band_out<false><<<band_out_grid(d, fields), 256, 0, s>>>(f0, f1, Sx, d.H, d.W, d.K, NoGuess{});
  return false;
}

// Mode coefficients of two fields, X_q = scale_q S_y (x_q / div_q) S_x^T
// (K x K per image): the row transforms of both fields in one launch (into
// kT, kT2), then the column transforms of both.
template <class X0, class X1>
void band_project_rows_cols(const Net& n, BandIn<X0> f0, BandIn<X1> f1, double* X0out,
                            double* X1out, double scale0, double scale1, hipStream_t s) {
  const Dims& d = n.d;
  const BandSpace b = band_space(n);
  f0.out = b.kT;
  f1.out = b.kT2;
  if (band_vector(d))
    k_band_rows_vec<X0, X1><<<dim3(d.B * cdiv(d.H, kBandRows), 2), 256, 0, s>>>(f0, f1, b.kSxT, d.H,
                                                                              d.W, d.K);
  else
    k_band_rows<X0, X1><<<band_rows_grid(d), 256, 0, s>>>(f0, f1, b.kSxT, d.H, d.W, d.K);
  k_band_cols<<<band_cols_grid(d), 256, 0, s>>>(
      BandIn<double>{b.kT, nullptr, X0out, scale0}, BandIn<double>{b.kT2, nullptr, X1out, scale1},
      b.kSy, d.H, d.K);
}

// gated: apply the convolutional branch's output gain (inference); training
// runs with gain 1.
template <int C>
bool forward(const Net& n, const Ptrs& f, const Ptrs& u, hipStream_t s, bool gated,
             const GuessOut* go = nullptr) {
  const Dims& d = n.d;
  const long long HW = d.HW;
  bf16* x0 = n.w<bf16>(n.wl.x0);
  bf16* a[5];
  for (int i = 0; i < 5; ++i) a[i] = n.w<bf16>(n.wl.act[i]);
  float* Sx = n.w<float>(n.wl.Sx);
  float* Sy = n.w<float>(n.wl.Sy);
  double* sv = n.w<double>(n.wl.s);            // s_r[B], s_in[B], s_f[B]
  double* r0 = n.w<double>(n.wl.r0);
  const int WP = spec_wp(d);
  const Bases bs{Sx, n.w<bf16>(n.wl.Sxh), n.w<bf16>(n.wl.Sxl), Sy, n.w<double>(n.wl.kSx),
                 n.w<double>(n.wl.kSxT), n.w<double>(n.wl.kSy), d.M, spec_mp(d), d.W, WP, d.H, d.K};
  normalise_inputs(f, u, r0, n.w<double>(n.wl.rms), sv, x0, d.B, d.H, d.W, s, &bs);
  // L1, L2
  k_conv_in_mfma<C><<<dim3(pixel_blocks(HW, d.B), d.B), 256, 0, s>>>(
      x0, n.bfw(T_C1W), n.bfw(T_C1B), a[0], d.H, d.W);
  k_conv_mfma<C, false><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(a[0], n.bfw(T_C2W), n.bfw(T_C2B), nullptr, a[1], d.B, d.H, d.W);
  // L3 spectral
  float* T = n.w<float>(n.wl.T);
  float* X = n.w<float>(n.wl.X);
  float* Z = n.w<float>(n.wl.Z);
  k_spec_rows<C><<<d.B * d.H, 256, 0, s>>>(a[1], n.w<bf16>(n.wl.Sxh), n.w<bf16>(n.wl.Sxl), T, d.W,
                                           WP, d.M);
  k_spec_cols<<<d.B * cdiv(d.M, 16) * cdiv(d.M * C, 16), 256, 0, s>>>(T, Sy, X, d.H, d.M, d.M * C, 1.f);
  k_spec_minv<C, false><<<d.B * d.M * cdiv(d.H, 64), 256, 0, s>>>(X, n.bfw(T_SWK), Sy, Z, d.H, d.M,
                                                                  (float)(2.0 / (d.H + 1)));
  launch_spec_out<C, false>(dim3(d.B * d.H * cdiv(d.W, 64)), s, a[1], n.bfw(T_SW1), n.bfw(T_SB), Z, Sx,
                            nullptr, a[2], d.W, WP, d.M, (float)(2.0 / (d.W + 1)));
  // L4, L5, L6
  k_conv_mfma<C, false><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(a[2], n.bfw(T_C4W), n.bfw(T_C4B), nullptr, a[3], d.B, d.H, d.W);
  k_conv_mfma<C, false><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(a[3], n.bfw(T_C5W), n.bfw(T_C5B), nullptr, a[4], d.B, d.H, d.W);
  k_conv_out_tile<C><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(a[4], n.bfw(T_C6W), n.bfw(T_C6B),
                                                              n.w<float>(n.wl.out), d.B, d.H, d.W);
  // band path from the FP64 residual, replacing the band of the
  // convolutional output: out += norm S^T (w X - S out S^T) S (FP64); with
  // `go`, the output transform may also write the guess (returns whether)
  if (d.K == 0) return false;
  float* out = n.w<float>(n.wl.out);
  const double* gate = gated ? (const double*)(n.params + n.pl.gate) : nullptr;
  const BandSpace bsp = band_space(n);
  band_project_rows_cols<double, float>(n, {r0, sv + d.B, bsp.kT, 1.0},
                                        {out, nullptr, bsp.kT2, 1.0}, bsp.kX, bsp.kC, 1.0, 1.0, s);
  k_band_inv<<<band_inv_grid(d), 256, 0, s>>>(bsp.kX, bsp.kC, (const double*)(n.params + n.pl.band),
                                               gate, bsp.kSy, bsp.kZ, d.H, d.K, 2.0 / (d.H + 1));
  return launch_band_out(s, d, 1, BandOut{bsp.kZ, out, gate, 2.0 / (d.W + 1)}, BandOut{}, bsp.kSx,
                         go);
}

template <int C>
void wgrad_conv(const Net& n, const bf16* in, const bf16* dz, int tw, int tb, hipStream_t s,
                int ntap) {
  const Dims& d = n.d;
  float* part = n.w<float>(n.wl.part);
  const int G = n.wl.wgrad_blocks;
  if (ntap == 9)
    k_wgrad_mfma<C, 9><<<G, 256, 0, s>>>(in, dz, part, d.B, d.H, d.W);
  else
    k_wgrad_mfma<C, 1><<<G, 256, 0, s>>>(in, dz, part, d.B, d.H, d.W);
  const int nout = ntap * C * C + C;
  k_wgrad_reduce<<<cdiv(nout, 64), 256, 0, s>>>(part, G, ntap, C, C, n.grad(tw), n.grad(tb));
}

template <int C>
void train(const Net& n, const Ptrs& f, const Ptrs& up, const Ptrs& ut, float* loss,
           const guess_net_cfg* cfg, hipStream_t s) {
  forward<C>(n, f, up, s, false);
  const Dims& d = n.d;
  const long long HW = d.HW;
  bf16* x0 = n.w<bf16>(n.wl.x0);
  bf16* a[5];
  for (int i = 0; i < 5; ++i) a[i] = n.w<bf16>(n.wl.act[i]);
  bf16* dz[2] = {n.w<bf16>(n.wl.dz[0]), n.w<bf16>(n.wl.dz[1])};
  float* out = n.w<float>(n.wl.out);
  float* dout = n.w<float>(n.wl.dout);
  double* sv = n.w<double>(n.wl.s);
  float* Sx = n.w<float>(n.wl.Sx);
  float* Sy = n.w<float>(n.wl.Sy);
  float* part = n.w<float>(n.wl.part);
  const int G = n.wl.wgrad_blocks;
  // loss
  double* lpart = n.w<double>(n.wl.loss) + 8;
  float* ldev = (float*)n.w<double>(n.wl.loss);
  {
    const int nb = (int)std::min<long long>(kMaxGrid, cdiv((long long)d.B * HW, 1024));
    k_loss<<<nb, 256, 0, s>>>(out, ut, up, sv + d.B, dout, lpart, HW, d.B);
    k_loss_sum<<<1, kReduceThreads, 0, s>>>(lpart, nb, ldev, loss, d.B);
  }
  // band path (K > 0): its least-squares state takes the batch's sums of
  // X T and X^2 (X = S[A d/s_r], T = S[t] of the target t = c_u d/s_r,
  // d = u_t - u_prev); the convolutional branch's gradient is dout off the
  // band: dout -= norm S^T S[dout] S
  if (d.K > 0) {
    const BandSpace bsp = band_space(n);
    double* tbuf = n.w<double>(n.wl.r0);          // the residual input is no longer needed
    double* abuf = n.w<double>(n.wl.ad);
    const int K = d.K;
    k_pair<<<dim3(cdiv(HW, 256), d.B), 256, 0, s>>>(ut, up, tbuf, abuf, d.H, d.W);
    band_project_rows_cols<double, double>(n, {tbuf, sv + d.B, nullptr, 1.0},
                                           {abuf, sv + d.B, nullptr, 1.0}, bsp.kTc, bsp.kXa, 1.0,
                                           1.0, s);
    k_band_fit<<<cdiv((long long)K * K, 256), 256, 0, s>>>(bsp.kXa, bsp.kTc,
                                                          (double*)(n.params + n.pl.band), d.B, K);
    // dout -= P_K dout, and (output gain) c = out - P_K out, the branch's
    // output off the band (out is no longer needed), against dout = (2/B)(c -
    // t) off the band; P_K x = nrm S^T S[x] S
    const double nrm = (2.0 / (d.H + 1)) * (2.0 / (d.W + 1));
    band_project_rows_cols<float, float>(n, {dout, nullptr, nullptr, 1.0}, {out, nullptr, nullptr, 1.0},
                                         bsp.kdY, bsp.kdY2, nrm, nrm, s);
    k_band_inv<<<band_inv_grid(d), 256, 0, s>>>(bsp.kdY, nullptr, nullptr, nullptr, bsp.kSy, bsp.kZ,
                                                 d.H, K, 1.0);
    k_band_inv<<<band_inv_grid(d), 256, 0, s>>>(bsp.kdY2, nullptr, nullptr, nullptr, bsp.kSy,
                                                 bsp.kZ2, d.H, K, 1.0);
    launch_band_out(s, d, 2, BandOut{bsp.kZ, dout, nullptr, -1.0},
                    BandOut{bsp.kZ2, out, nullptr, -1.0}, bsp.kSx);
    double* gpart = n.w<double>(n.wl.loss) + 8 + 2048;
    k_gate_sums<<<256, 256, 0, s>>>(out, dout, (long long)d.B * HW, gpart);
    k_gate_fin<<<1, 64, 0, s>>>(gpart, 256, (double*)(n.params + n.pl.gate), d.B);
  }
  // L6: weight grad from (a5, dout); input grad masked by a5 -> dz5
  k_wgrad_out<C><<<G, 256, 0, s>>>(a[4], dout, part, d.B, d.H, d.W);
  k_wgrad_reduce<<<cdiv(9 * C + 1, 64), 256, 0, s>>>(part, G, 9, 1, C, n.grad(T_C6W), n.grad(T_C6B));
  k_conv_outT_mfma<C><<<dim3(cdiv(HW, 256), d.B), 256, 0, s>>>(
      dout, n.bfw(T_C6W), a[4], dz[0], d.H, d.W);
  // L5
  wgrad_conv<C>(n, a[3], dz[0], T_C5W, T_C5B, s, 9);
  k_conv_mfma<C, true><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(dz[0], n.bfw(T_C5W), nullptr, a[3], dz[1], d.B, d.H, d.W);
  // L4
  wgrad_conv<C>(n, a[2], dz[1], T_C4W, T_C4B, s, 9);
  k_conv_mfma<C, true><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(dz[1], n.bfw(T_C4W), nullptr, a[2], dz[0], d.B, d.H, d.W);
  // L3 spectral: dz3 = dz[0]
  wgrad_conv<C>(n, a[1], dz[0], T_SW1, T_SB, s, 1);
  float* T = n.w<float>(n.wl.T);
  float* X = n.w<float>(n.wl.X);
  float* dY = n.w<float>(n.wl.Y);
  float* Z = n.w<float>(n.wl.Z);
  const float nrm = (float)((2.0 / (d.H + 1)) * (2.0 / (d.W + 1)));
  const int WP = spec_wp(d);
  k_spec_rows<C><<<d.B * d.H, 256, 0, s>>>(dz[0], n.w<bf16>(n.wl.Sxh), n.w<bf16>(n.wl.Sxl), T, d.W,
                                           WP, d.M);
  k_spec_cols<<<d.B * cdiv(d.M, 16) * cdiv(d.M * C, 16), 256, 0, s>>>(T, Sy, dY, d.H, d.M, d.M * C, nrm);
  k_spec_minv<C, true><<<d.B * d.M * cdiv(d.H, 64), 256, 0, s>>>(dY, n.bfw(T_SWK), Sy, Z, d.H, d.M, 1.f);
  k_spec_dwk<<<cdiv((long long)d.M * d.M * C * C, 256), 256, 0, s>>>(dY, X, n.grad(T_SWK), d.B, d.M, C);
  launch_spec_out<C, true>(dim3(d.B * d.H * cdiv(d.W, 64)), s, dz[0], n.bfw(T_SW1), nullptr, Z, Sx,
                           a[1], dz[1], d.W, WP, d.M, 1.f);
  // L2: dz2 = dz[1]
  wgrad_conv<C>(n, a[0], dz[1], T_C2W, T_C2B, s, 9);
  k_conv_mfma<C, true><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(dz[1], n.bfw(T_C2W), nullptr, a[0], dz[0], d.B, d.H, d.W);
  // L1: dz1 = dz[0]
  k_wgrad_in<C><<<G, 256, 0, s>>>(x0, dz[0], part, d.B, d.H, d.W);
  k_wgrad_reduce<<<cdiv(9 * C * 2 + C, 64), 256, 0, s>>>(part, G, 9, C, 2, n.grad(T_C1W),
                                                          n.grad(T_C1B));
  // Adam
  long long* step = (long long*)(n.params + n.pl.step);
  k_step_inc<<<1, 64, 0, s>>>(step);
  k_adam<<<cdiv(n.pl.P, 256), 256, 0, s>>>((float*)(n.params + n.pl.master),
                                           (const float*)(n.params + n.pl.grad),
                                           (float*)(n.params + n.pl.m), (float*)(n.params + n.pl.v),
                                           (bf16*)(n.params + n.pl.bf), step, n.pl.P, cfg->lr,
                                           cfg->beta1, cfg->beta2, cfg->eps);
}


// ------------------------------------------------------------------ multi-scale network
// The FluidNet-variant guess network (Section 2.1): a 2x2 average-pooling
// pyramid of the input, per level conv3x3 2->C + ReLU and conv3x3 C->C + ReLU,
// the levels upsampled (nearest) to the full grid and summed, R residual
// blocks S += conv3x3(ReLU(conv3x3(S))), then conv3x3 C->C + ReLU and
// conv3x3 C->1.  Every convolution runs on the kernels above; the pyramid adds
// three small bandwidth-bound kernels.
constexpr int kFluidC = 32;
constexpr int kFluidMaxLevels = 6;
constexpr int kFluidMaxBlocks = 8;
constexpr int kFluidMaxTensors = 4 * kFluidMaxLevels + 4 * kFluidMaxBlocks + 4;

struct LvlPtrs {
  const bf16* p[kFluidMaxLevels];
};

// Coarse input X_c = avgpool2(X_f) of the 2-channel BF16 input, one thread per
// coarse pixel, FP32 sum rounded once.
__global__ void k_pool_in(const bf16* xf, bf16* xc, int Hc, int Wc) {
  const int b = blockIdx.y;
  const long long HWc = (long long)Hc * Wc;
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= HWc) return;
  const int i = (int)(p / Wc), j = (int)(p % Wc);
  const long long Wf = 2LL * Wc;
  const bf16* base = xf + ((size_t)b * 4 * HWc + (size_t)(2 * i) * Wf + 2 * j) * 2;
  float s0 = 0.f, s1 = 0.f;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const bf16* px = base + ((size_t)dy * Wf + dx) * 2;
      s0 += bf2f(px[0]);
      s1 += bf2f(px[1]);
    }
  bf16* o = xc + ((size_t)b * HWc + p) * 2;
  o[0] = f2bf(0.25f * s0);
  o[1] = f2bf(0.25f * s1);
}

// S[p] = sum over levels l (in order) of y_l[p >> l]: nearest upsampling of
// every level and their sum, one thread per 8 channels of a full-grid pixel.
template <int C>
__global__ __launch_bounds__(256) void k_upsum(LvlPtrs y, int L, bf16* S, int H, int W) {
  constexpr int CH = C / 8;
  const int b = blockIdx.y;
  const long long HW = (long long)H * W;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= HW * CH) return;
  const long long pix = e / CH;
  const int ch = (int)(e % CH);
  const int yy = (int)(pix / W), xx = (int)(pix % W);
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int l = 0; l < L; ++l) {
    const int Hl = H >> l, Wl = W >> l;
    float v[8];
    load_ch<8>(y.p[l] + (((size_t)b * Hl + (yy >> l)) * Wl + (xx >> l)) * C + ch * 8, v);
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] += v[k];
  }
  store_ch<8>(S + ((size_t)b * HW + pix) * C + ch * 8, acc);
}

// Adjoint of the upsampling, one level down: Pc = the sum of each 2x2 block of
// Pf (FP32; Pc may be NULL at the coarsest level), and dz = Pc (Y > 0) in BF16
// (the gradient of that level's ReLU output).
template <int C, class TI>
__global__ __launch_bounds__(256) void k_sumpool_mask(const TI* Pf, float* Pc, const bf16* Y,
                                                      bf16* dz, int Hc, int Wc) {
  constexpr int CH = C / 8;
  const int b = blockIdx.y;
  const long long HWc = (long long)Hc * Wc;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= HWc * CH) return;
  const long long pix = e / CH;
  const int ch = (int)(e % CH);
  const int i = (int)(pix / Wc), j = (int)(pix % Wc);
  const long long Wf = 2LL * Wc;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      float v[8];
      load_ch<8>(Pf + (((size_t)b * 2 * Hc + 2 * i + dy) * Wf + 2 * j + dx) * C + ch * 8, v);
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] += v[k];
    }
  const size_t o = ((size_t)b * HWc + pix) * C + ch * 8;
  if (Pc) store_ch<8>(Pc + o, acc);
  float m[8];
  load_ch<8>(Y + o, m);
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = m[k] > 0.f ? acc[k] : 0.f;
  store_ch<8>(dz + o, acc);
}

// dz = d (Y > 0), 8 elements per thread.
__global__ void k_mask8(const bf16* d, const bf16* Y, bf16* dz, long long n8) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n8) return;
  float v[8], m[8];
  load_ch<8>(d + e * 8, v);
  load_ch<8>(Y + e * 8, m);
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = m[k] > 0.f ? v[k] : 0.f;
  store_ch<8>(dz + e * 8, v);
}

__global__ void k_fill0(float* p, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0.f;
}

struct FDims {
  int B, H, W, L, R;   // R: blocks with storage (cfg->max_blocks)
  long long HW;
};

void check_fluid_cfg(const fluid_net_cfg* cfg) {
  if (!cfg) throw ArgError{MLG_ERR_ARG, "cfg is NULL"};
  if (cfg->channels != kFluidC) throw ArgError{MLG_ERR_ARG, "channels must be 32"};
  if (cfg->levels < 1 || cfg->levels > kFluidMaxLevels)
    throw ArgError{MLG_ERR_ARG, "levels must be in 1..6"};
  if (cfg->max_blocks < 0 || cfg->max_blocks > kFluidMaxBlocks)
    throw ArgError{MLG_ERR_ARG, "max_blocks must be in 0..8"};
}

int fl_ntensors(const fluid_net_cfg* cfg) { return 4 * cfg->levels + 4 * cfg->max_blocks + 4; }
inline int fl_lvl(int l, int k) { return 4 * l + k; }
inline int fl_blk(const FDims& d, int i, int k) { return 4 * d.L + 4 * i + k; }
inline int fl_head(const FDims& d, int k) { return 4 * d.L + 4 * d.R + k; }

// element counts and He-uniform fan-ins (0: zero-initialised) per tensor
void fluid_sizes(const fluid_net_cfg* cfg, int64_t* sz, float* fan) {
  const int64_t C = kFluidC;
  int t = 0;
  auto put = [&](int64_t n, float f) {
    sz[t] = n;
    fan[t] = f;
    ++t;
  };
  for (int l = 0; l < cfg->levels; ++l) {
    put(C * 2 * 9, 18.f);
    put(C, 0.f);
    put(C * C * 9, 9.f * C);
    put(C, 0.f);
  }
  for (int i = 0; i < cfg->max_blocks; ++i) {
    put(C * C * 9, 9.f * C);
    put(C, 0.f);
    put(C * C * 9, 0.f);      // a new block starts as the identity
    put(C, 0.f);
  }
  put(C * C * 9, 9.f * C);
  put(C, 0.f);
  put(C * 9, 0.f);            // zero output layer: the untrained network returns u_prev
  put(1, 0.f);
}

struct FLayout {
  int n;
  int64_t P;
  int64_t off[kFluidMaxTensors + 1];
  size_t master, grad, m, v, bf, step, total;
};

FLayout fluid_layout(const fluid_net_cfg* cfg) {
  check_fluid_cfg(cfg);
  FLayout L{};
  int64_t sz[kFluidMaxTensors];
  float fan[kFluidMaxTensors];
  fluid_sizes(cfg, sz, fan);
  L.n = fl_ntensors(cfg);
  L.off[0] = 0;
  for (int i = 0; i < L.n; ++i) L.off[i + 1] = L.off[i] + (sz[i] + 63) / 64 * 64;
  L.P = L.off[L.n];
  const size_t f = align_up((size_t)L.P * 4, 256);
  L.master = 0;
  L.grad = f;
  L.m = 2 * f;
  L.v = 3 * f;
  L.bf = 4 * f;
  L.step = L.bf + align_up((size_t)L.P * 2, 256);
  L.total = L.step + 256;
  return L;
}

FDims check_fluid_grid(const fluid_net_cfg* cfg, const mlg_grid* grid, int batch) {
  check_fluid_cfg(cfg);
  if (!grid || grid->dim != 2) throw ArgError{MLG_ERR_ARG, "the guess network takes 2D grids"};
  const int q = 1 << (cfg->levels - 1);
  if (grid->nx < 1 || grid->ny < 1 || grid->nx % q || grid->ny % q)
    throw ArgError{MLG_ERR_ARG, "grid sides must be multiples of 2^(levels-1)"};
  if (batch < 1 || batch > kMaxBatch) throw ArgError{MLG_ERR_ARG, "batch must be in 1..64"};
  return FDims{batch, grid->ny, grid->nx, cfg->levels, cfg->max_blocks,
               (long long)grid->nx * grid->ny};
}

struct FWs {
  size_t s, r0, rms, X[kFluidMaxLevels], A[kFluidMaxLevels], Y[kFluidMaxLevels];
  size_t S[kFluidMaxBlocks + 1], Hb[kFluidMaxBlocks], o, out;
  size_t dout, dS, d1, d2, P[2], part, loss, total;
  int wgrad_blocks;
};

FWs fluid_ws(const FDims& d, bool train) {
  FWs L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  const size_t full = (size_t)d.B * d.HW * kFluidC * 2;
  L.s = take((size_t)d.B * 8 * 3);
  L.r0 = take((size_t)d.B * d.HW * 8);
  L.rms = take((size_t)2 * d.B * kRmsBlocks * 8);
  for (int l = 0; l < d.L; ++l) {
    const size_t hw = (size_t)(d.H >> l) * (d.W >> l);
    L.X[l] = take((size_t)d.B * hw * 2 * 2);
    L.A[l] = take((size_t)d.B * hw * kFluidC * 2);
    L.Y[l] = take((size_t)d.B * hw * kFluidC * 2);
  }
  for (int i = 0; i <= d.R; ++i) L.S[i] = take(full);
  for (int i = 0; i < d.R; ++i) L.Hb[i] = take(full);
  L.o = take(full);
  L.out = take((size_t)d.B * d.HW * 4);
  if (train) {
    L.dout = take((size_t)d.B * d.HW * 4);
    L.dS = take(full);
    L.d1 = take(full);
    L.d2 = take(full);
    const size_t q = (size_t)d.B * (d.HW / 4) * kFluidC * 4;
    L.P[0] = take(q);
    L.P[1] = take(q);
    L.wgrad_blocks = 512;
    L.part = take((size_t)L.wgrad_blocks * (9 * kFluidC * kFluidC + kFluidC) * 4);
    L.loss = take(4096 * 8);
  }
  L.total = o;
  return L;
}

struct FNet {
  FDims d;
  FLayout pl;
  FWs wl;
  char* params;
  char* ws;
  const bf16* bfw(int t) const { return (const bf16*)(params + pl.bf) + pl.off[t]; }
  float* grad(int t) const { return (float*)(params + pl.grad) + pl.off[t]; }
  template <class T>
  T* w(size_t off) const { return (T*)(ws + off); }
};

void fluid_forward(const FNet& n, const Ptrs& f, const Ptrs& u, int blocks, hipStream_t s) {
  constexpr int C = kFluidC;
  const FDims& d = n.d;
  const long long HW = d.HW;
  double* sv = n.w<double>(n.wl.s);
  double* r0 = n.w<double>(n.wl.r0);
  normalise_inputs(f, u, r0, n.w<double>(n.wl.rms), sv, n.w<bf16>(n.wl.X[0]), d.B, d.H, d.W, s);
  for (int l = 1; l < d.L; ++l) {
    const int Hl = d.H >> l, Wl = d.W >> l;
    k_pool_in<<<dim3(cdiv((long long)Hl * Wl, 256), d.B), 256, 0, s>>>(
        n.w<bf16>(n.wl.X[l - 1]), n.w<bf16>(n.wl.X[l]), Hl, Wl);
  }
  LvlPtrs yp{};
  for (int l = 0; l < d.L; ++l) {
    const int Hl = d.H >> l, Wl = d.W >> l;
    const long long hw = (long long)Hl * Wl;
    k_conv_in_mfma<C><<<dim3(pixel_blocks(hw, d.B), d.B), 256, 0, s>>>(
        n.w<bf16>(n.wl.X[l]), n.bfw(fl_lvl(l, 0)), n.bfw(fl_lvl(l, 1)), n.w<bf16>(n.wl.A[l]), Hl,
        Wl);
    k_conv_mfma<C, false><<<conv_grid(d.B, Hl, Wl), 256, 0, s>>>(n.w<bf16>(n.wl.A[l]), n.bfw(fl_lvl(l, 2)), n.bfw(fl_lvl(l, 3)), nullptr, n.w<bf16>(n.wl.Y[l]), d.B, Hl, Wl);
    yp.p[l] = n.w<bf16>(n.wl.Y[l]);
  }
  k_upsum<C><<<dim3(cdiv(HW * (C / 8), 256), d.B), 256, 0, s>>>(yp, d.L, n.w<bf16>(n.wl.S[0]),
                                                                d.H, d.W);
  for (int i = 0; i < blocks; ++i) {
    k_conv_mfma<C, false><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(n.w<bf16>(n.wl.S[i]), n.bfw(fl_blk(d, i, 0)), n.bfw(fl_blk(d, i, 1)), nullptr, n.w<bf16>(n.wl.Hb[i]), d.B, d.H, d.W);
    k_conv_mfma<C, false, true><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(n.w<bf16>(n.wl.Hb[i]), n.bfw(fl_blk(d, i, 2)), n.bfw(fl_blk(d, i, 3)), n.w<bf16>(n.wl.S[i]), n.w<bf16>(n.wl.S[i + 1]), d.B, d.H, d.W);
  }
  k_conv_mfma<C, false><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(n.w<bf16>(n.wl.S[blocks]), n.bfw(fl_head(d, 0)), n.bfw(fl_head(d, 1)), nullptr, n.w<bf16>(n.wl.o), d.B, d.H, d.W);
  k_conv_out_tile<C><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(
      n.w<bf16>(n.wl.o), n.bfw(fl_head(d, 2)), n.bfw(fl_head(d, 3)), n.w<float>(n.wl.out), d.B, d.H,
      d.W);
}

void fl_wgrad9(const FNet& n, const bf16* in, const bf16* dz, int tw, int tb, int H, int W,
               hipStream_t s) {
  constexpr int C = kFluidC;
  float* part = n.w<float>(n.wl.part);
  const int G = n.wl.wgrad_blocks;
  k_wgrad_mfma<C, 9><<<G, 256, 0, s>>>(in, dz, part, n.d.B, H, W);
  k_wgrad_reduce<<<cdiv(9 * C * C + C, 64), 256, 0, s>>>(part, G, 9, C, C, n.grad(tw), n.grad(tb));
}

void fluid_train(const FNet& n, const Ptrs& f, const Ptrs& up, const Ptrs& ut, int blocks,
                 float* loss, const fluid_net_cfg* cfg, hipStream_t s) {
  constexpr int C = kFluidC;
  fluid_forward(n, f, up, blocks, s);
  const FDims& d = n.d;
  const long long HW = d.HW;
  double* sv = n.w<double>(n.wl.s);
  float* out = n.w<float>(n.wl.out);
  float* dout = n.w<float>(n.wl.dout);
  float* part = n.w<float>(n.wl.part);
  const int G = n.wl.wgrad_blocks;
  bf16* dS = n.w<bf16>(n.wl.dS);
  bf16* d1 = n.w<bf16>(n.wl.d1);
  bf16* d2 = n.w<bf16>(n.wl.d2);
  {
    double* lpart = n.w<double>(n.wl.loss) + 8;
    float* ldev = (float*)n.w<double>(n.wl.loss);
    const int nb = (int)std::min<long long>(kMaxGrid, cdiv((long long)d.B * HW, 1024));
    k_loss<<<nb, 256, 0, s>>>(out, ut, up, sv + d.B, dout, lpart, HW, d.B);
    k_loss_sum<<<1, kReduceThreads, 0, s>>>(lpart, nb, ldev, loss, d.B);
  }
  // head: out = conv(o), o = ReLU(conv(S_R))
  bf16* o = n.w<bf16>(n.wl.o);
  k_wgrad_out<C><<<G, 256, 0, s>>>(o, dout, part, d.B, d.H, d.W);
  k_wgrad_reduce<<<cdiv(9 * C + 1, 64), 256, 0, s>>>(part, G, 9, 1, C, n.grad(fl_head(d, 2)),
                                                       n.grad(fl_head(d, 3)));
  k_conv_outT_mfma<C><<<dim3(cdiv(HW, 256), d.B), 256, 0, s>>>(
      dout, n.bfw(fl_head(d, 2)), o, d1, d.H, d.W);
  fl_wgrad9(n, n.w<bf16>(n.wl.S[blocks]), d1, fl_head(d, 0), fl_head(d, 1), d.H, d.W, s);
  k_conv_mfma<C, true, true><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(d1, n.bfw(fl_head(d, 0)), nullptr, nullptr, dS, d.B, d.H, d.W);
  // residual blocks, last first: dS accumulates in place
  for (int i = blocks - 1; i >= 0; --i) {
    bf16* hb = n.w<bf16>(n.wl.Hb[i]);
    fl_wgrad9(n, hb, dS, fl_blk(d, i, 2), fl_blk(d, i, 3), d.H, d.W, s);
    k_conv_mfma<C, true><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(dS, n.bfw(fl_blk(d, i, 2)), nullptr, hb, d1, d.B, d.H, d.W);
    fl_wgrad9(n, n.w<bf16>(n.wl.S[i]), d1, fl_blk(d, i, 0), fl_blk(d, i, 1), d.H, d.W, s);
    k_conv_mfma<C, true, true><<<conv_grid(d.B, d.H, d.W), 256, 0, s>>>(d1, n.bfw(fl_blk(d, i, 0)), nullptr, dS, dS, d.B, d.H, d.W);
  }
  // levels: the gradient of y_l is the 2^l x 2^l block sum of dS, masked
  float* P[2] = {n.w<float>(n.wl.P[0]), n.w<float>(n.wl.P[1])};
  for (int l = 0; l < d.L; ++l) {
    const int Hl = d.H >> l, Wl = d.W >> l;
    const long long hw = (long long)Hl * Wl;
    const bf16* Y = n.w<bf16>(n.wl.Y[l]);
    float* pc = l + 1 < d.L ? P[l & 1] : nullptr;
    if (l == 0)
      k_mask8<<<cdiv((long long)d.B * HW * C / 8, 256), 256, 0, s>>>(dS, Y, d1,
                                                                    (long long)d.B * HW * C / 8);
    else if (l == 1)
      k_sumpool_mask<C, bf16><<<dim3(cdiv(hw * (C / 8), 256), d.B), 256, 0, s>>>(dS, pc, Y, d1, Hl,
                                                                                Wl);
    else
      k_sumpool_mask<C, float><<<dim3(cdiv(hw * (C / 8), 256), d.B), 256, 0, s>>>(
          P[(l - 1) & 1], pc, Y, d1, Hl, Wl);
    bf16* A = n.w<bf16>(n.wl.A[l]);
    fl_wgrad9(n, A, d1, fl_lvl(l, 2), fl_lvl(l, 3), Hl, Wl, s);
    k_conv_mfma<C, true><<<conv_grid(d.B, Hl, Wl), 256, 0, s>>>(d1, n.bfw(fl_lvl(l, 2)), nullptr, A, d2, d.B, Hl, Wl);
    k_wgrad_in<C><<<G, 256, 0, s>>>(n.w<bf16>(n.wl.X[l]), d2, part, d.B, Hl, Wl);
    k_wgrad_reduce<<<cdiv(9 * C * 2 + C, 64), 256, 0, s>>>(part, G, 9, C, 2, n.grad(fl_lvl(l, 0)),
                                                            n.grad(fl_lvl(l, 1)));
  }
  // blocks beyond the active ones take no step
  const int64_t z0 = n.pl.off[fl_blk(d, blocks, 0)], z1 = n.pl.off[fl_head(d, 0)];
  if (z1 > z0)
    k_fill0<<<cdiv(z1 - z0, 256), 256, 0, s>>>((float*)(n.params + n.pl.grad) + z0, z1 - z0);
  long long* step = (long long*)(n.params + n.pl.step);
  k_step_inc<<<1, 64, 0, s>>>(step);
  k_adam<<<cdiv(n.pl.P, 256), 256, 0, s>>>((float*)(n.params + n.pl.master),
                                           (const float*)(n.params + n.pl.grad),
                                           (float*)(n.params + n.pl.m), (float*)(n.params + n.pl.v),
                                           (bf16*)(n.params + n.pl.bf), step, n.pl.P, cfg->lr,
                                           cfg->beta1, cfg->beta2, cfg->eps);
}

}  // namespace

// ------------------------------------------------------------------ entry points
int64_t net_param_offset(const guess_net_cfg* cfg, int index) {
  if (index < 0 || index > kNumTensors) throw ArgError{MLG_ERR_ARG, "tensor index out of range"};
  return param_layout(cfg).off[index];
}

int64_t net_param_count(const guess_net_cfg* cfg) { return param_layout(cfg).P; }

size_t net_param_bytes(const guess_net_cfg* cfg) { return param_layout(cfg).total; }

size_t net_workspace_bytes(const guess_net_cfg* cfg, const mlg_grid* grid, int batch, int train) {
  Dims d = check_grid_net(cfg, grid, batch);
  return ws_layout(d, train != 0).total;
}

int net_init(const guess_net_cfg* cfg, void* params, hipStream_t s) {
  ParamLayout pl = param_layout(cfg);
  if (!params) throw ArgError{MLG_ERR_ARG, "params is NULL"};
  InitSpec spec{};
  for (int i = 0; i <= kNumTensors; ++i) spec.off[i] = pl.off[i];
  int64_t sz[kNumTensors];
  tensor_sizes(cfg, sz);
  const float C = (float)cfg->channels;
  const float fan[kNumTensors] = {18.f, 0, 9 * C, 0, 2 * C, 0, 2 * C, 9 * C, 0, 9 * C, 0, 0, 0};
  for (int i = 0; i < kNumTensors; ++i) {
    spec.bound[i] = fan[i] > 0 ? sqrtf(6.f / fan[i]) : 0.f;
    spec.size[i] = sz[i];
  }
  char* p = (char*)params;
  k_init_params<kNumTensors><<<cdiv(pl.P, 256), 256, 0, s>>>((float*)(p + pl.master), (float*)(p + pl.grad),
                                                (float*)(p + pl.m), (float*)(p + pl.v),
                                                (bf16*)(p + pl.bf), (long long*)(p + pl.step), spec,
                                                kNumTensors, pl.P, cfg->seed);
  // the band's least-squares state starts empty (w = 0)
  const long long nb = 4LL * cfg->skip_modes * cfg->skip_modes;
  if (nb > 0) k_fill0<<<cdiv(nb, 256), 256, 0, s>>>((float*)(p + pl.band), nb);
  k_fill0<<<1, 64, 0, s>>>((float*)(p + pl.gate), 4);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

int net_refresh(const guess_net_cfg* cfg, void* params, hipStream_t s) {
  ParamLayout pl = param_layout(cfg);
  if (!params) throw ArgError{MLG_ERR_ARG, "params is NULL"};
  char* p = (char*)params;
  k_refresh<<<cdiv(pl.P, 256), 256, 0, s>>>((const float*)(p + pl.master), (float*)(p + pl.grad),
                                            (float*)(p + pl.m), (float*)(p + pl.v),
                                            (bf16*)(p + pl.bf), (long long*)(p + pl.step), pl.P);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

int net_infer(const guess_net_cfg* cfg, const void* params, const mlg_grid* grid, int batch,
              const double* f, const double* u_prev, double* guess, void* ws, size_t ws_bytes,
              hipStream_t s) {
  Dims d = check_grid_net(cfg, grid, batch);
  if (!params || !f || !u_prev || !guess) throw ArgError{MLG_ERR_ARG, "NULL pointer"};
  WsLayout wl = ws_layout(d, false);
  if (!ws || ws_bytes < wl.total) throw ArgError{MLG_ERR_WORKSPACE, "network workspace too small"};
  Net n{d, param_layout(cfg), wl, (char*)params, (char*)ws};
  Ptrs fp{}, up{};
  MPtrs gp{};
  for (int b = 0; b < d.B; ++b) {
    fp.p[b] = f + (size_t)b * d.HW;
    up.p[b] = u_prev + (size_t)b * d.HW;
    gp.p[b] = guess + (size_t)b * d.HW;
  }
  const GuessOut go{up, gp, n.w<double>(wl.s)};
  if (!forward<32>(n, fp, up, s, true, &go))
    k_guess<<<dim3(cdiv(d.HW, 256), d.B), 256, 0, s>>>(n.w<float>(wl.out), up, n.w<double>(wl.s), gp,
                                                        d.HW);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

int net_train_step(const guess_net_cfg* cfg, void* params, const mlg_grid* grid, int batch,
                   const double* const* f, const double* const* u_prev,
                   const double* const* u_target, void* ws, size_t ws_bytes, float* loss,
                   hipStream_t s) {
  Dims d = check_grid_net(cfg, grid, batch);
  if (!params || !f || !u_prev || !u_target) throw ArgError{MLG_ERR_ARG, "NULL pointer"};
  WsLayout wl = ws_layout(d, true);
  if (!ws || ws_bytes < wl.total) throw ArgError{MLG_ERR_WORKSPACE, "network workspace too small"};
  Net n{d, param_layout(cfg), wl, (char*)params, (char*)ws};
  Ptrs fp{}, up{}, tp{};
  for (int b = 0; b < d.B; ++b) {
    if (!f[b] || !u_prev[b] || !u_target[b]) throw ArgError{MLG_ERR_ARG, "NULL sample pointer"};
    fp.p[b] = f[b];
    up.p[b] = u_prev[b];
    tp.p[b] = u_target[b];
  }
  train<32>(n, fp, up, tp, loss, cfg, s);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

// ------------------------------------------------------------------ multi-scale network entry points
int64_t fluid_param_offset(const fluid_net_cfg* cfg, int index) {
  FLayout pl = fluid_layout(cfg);
  if (index < 0 || index > pl.n) throw ArgError{MLG_ERR_ARG, "tensor index out of range"};
  return pl.off[index];
}

int64_t fluid_param_count(const fluid_net_cfg* cfg) { return fluid_layout(cfg).P; }

size_t fluid_param_bytes(const fluid_net_cfg* cfg) { return fluid_layout(cfg).total; }

size_t fluid_workspace_bytes(const fluid_net_cfg* cfg, const mlg_grid* grid, int batch, int train) {
  return fluid_ws(check_fluid_grid(cfg, grid, batch), train != 0).total;
}

int fluid_init(const fluid_net_cfg* cfg, void* params, hipStream_t s) {
  FLayout pl = fluid_layout(cfg);
  if (!params) throw ArgError{MLG_ERR_ARG, "params is NULL"};
  InitSpecT<kFluidMaxTensors> spec{};
  int64_t sz[kFluidMaxTensors];
  float fan[kFluidMaxTensors];
  fluid_sizes(cfg, sz, fan);
  for (int i = 0; i <= pl.n; ++i) spec.off[i] = pl.off[i];
  for (int i = 0; i < pl.n; ++i) {
    spec.size[i] = sz[i];
    spec.bound[i] = fan[i] > 0.f ? sqrtf(6.f / fan[i]) : 0.f;
  }
  char* p = (char*)params;
  k_init_params<kFluidMaxTensors><<<cdiv(pl.P, 256), 256, 0, s>>>(
      (float*)(p + pl.master), (float*)(p + pl.grad), (float*)(p + pl.m), (float*)(p + pl.v),
      (bf16*)(p + pl.bf), (long long*)(p + pl.step), spec, pl.n, pl.P, cfg->seed);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

int fluid_refresh(const fluid_net_cfg* cfg, void* params, hipStream_t s) {
  FLayout pl = fluid_layout(cfg);
  if (!params) throw ArgError{MLG_ERR_ARG, "params is NULL"};
  char* p = (char*)params;
  k_refresh<<<cdiv(pl.P, 256), 256, 0, s>>>((const float*)(p + pl.master), (float*)(p + pl.grad),
                                            (float*)(p + pl.m), (float*)(p + pl.v),
                                            (bf16*)(p + pl.bf), (long long*)(p + pl.step), pl.P);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

static void check_blocks(const fluid_net_cfg* cfg, int blocks) {
  if (blocks < 0 || blocks > cfg->max_blocks)
    throw ArgError{MLG_ERR_ARG, "blocks must be in 0..max_blocks"};
}

int fluid_infer(const fluid_net_cfg* cfg, const void* params, int blocks, const mlg_grid* grid,
                int batch, const double* f, const double* u_prev, double* guess, void* ws,
                size_t ws_bytes, hipStream_t s) {
  FDims d = check_fluid_grid(cfg, grid, batch);
  check_blocks(cfg, blocks);
  if (!params || !f || !u_prev || !guess) throw ArgError{MLG_ERR_ARG, "NULL pointer"};
  FWs wl = fluid_ws(d, false);
  if (!ws || ws_bytes < wl.total) throw ArgError{MLG_ERR_WORKSPACE, "network workspace too small"};
  FNet n{d, fluid_layout(cfg), wl, (char*)params, (char*)ws};
  Ptrs fp{}, up{};
  MPtrs gp{};
  for (int b = 0; b < d.B; ++b) {
    fp.p[b] = f + (size_t)b * d.HW;
    up.p[b] = u_prev + (size_t)b * d.HW;
    gp.p[b] = guess + (size_t)b * d.HW;
  }
  fluid_forward(n, fp, up, blocks, s);
  k_guess<<<dim3(cdiv(d.HW, 256), d.B), 256, 0, s>>>(n.w<float>(wl.out), up, n.w<double>(wl.s), gp,
                                                      d.HW);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

int fluid_train_step(const fluid_net_cfg* cfg, void* params, int blocks, const mlg_grid* grid,
                     int batch, const double* const* f, const double* const* u_prev,
                     const double* const* u_target, void* ws, size_t ws_bytes, float* loss,
                     hipStream_t s) {
  FDims d = check_fluid_grid(cfg, grid, batch);
  check_blocks(cfg, blocks);
  if (!params || !f || !u_prev || !u_target) throw ArgError{MLG_ERR_ARG, "NULL pointer"};
  FWs wl = fluid_ws(d, true);
  if (!ws || ws_bytes < wl.total) throw ArgError{MLG_ERR_WORKSPACE, "network workspace too small"};
  FNet n{d, fluid_layout(cfg), wl, (char*)params, (char*)ws};
  Ptrs fp{}, up{}, tp{};
  for (int b = 0; b < d.B; ++b) {
    if (!f[b] || !u_prev[b] || !u_target[b]) throw ArgError{MLG_ERR_ARG, "NULL sample pointer"};
    fp.p[b] = f[b];
    up.p[b] = u_prev[b];
    tp.p[b] = u_target[b];
  }
  fluid_train(n, fp, up, tp, blocks, loss, cfg, s);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

}  // namespace mlg
