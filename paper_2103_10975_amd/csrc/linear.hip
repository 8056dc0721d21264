// Single-layer linear model of the initial guess (Section 3, "Understanding
// the AI accelerator through a simplified model"): x0 = T b with one dense
// n x n matrix T, trained on the solver's (b, x) pairs with the Section 2.3
// loss L = (1/B) sum_i |T b_i - x_i|^2 by gradient descent,
// T <- T - lr (2/B) sum_i (T b_i - x_i) b_i^T.
//
// T is FP32 (row-major, n = points of the grid); products accumulate in FP64.
// The matrix-vector products read T once per call for the whole batch (one
// wavefront per row, coalesced along the row), so a call is one pass over T:
// bound by HBM (or L2 while n^2 * 4 B fits) at any batch size up to 16.
#include "linear.h"

namespace mlg {
namespace {

constexpr int kLinMaxBatch = 16;
constexpr long long kLinMaxN = 16384;

struct LinIn {
  const double* p[kLinMaxBatch];
};
struct LinOut {
  double* p[kLinMaxBatch];
};

// out_i[r] = sum_c T[r][c] b_i[c] - (x_i ? x_i[r] : 0), i < B; 4 rows per workgroup.
__global__ __launch_bounds__(256) void k_lin_apply(const float* T, LinIn b, LinIn x, LinOut out,
                                                   int n, int B) {
  const int lane = threadIdx.x & 63;
  const long long r = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  double acc[kLinMaxBatch];
#pragma unroll
  for (int i = 0; i < kLinMaxBatch; ++i) acc[i] = 0.0;
  const float* row = T + r * n;
  for (int c = lane; c < n; c += 64) {
    const double t = row[c];
#pragma unroll
    for (int i = 0; i < kLinMaxBatch; ++i)
      if (i < B) acc[i] += t * b.p[i][c];
  }
#pragma unroll
  for (int i = 0; i < kLinMaxBatch; ++i) {
    if (i >= B) break;
    const double s = wave_sum(acc[i]);
    if (lane == 0) out.p[i][r] = s - (x.p[i] ? x.p[i][r] : 0.0);
  }
}

// loss = (1/B) sum of e^2 over e [B * n], one workgroup in a fixed order.
__global__ __launch_bounds__(256) void k_lin_loss(const double* e, long long m, int B,
                                                  float* loss) {
  __shared__ double red[4];
  double acc = 0.0;
  for (long long k = threadIdx.x; k < m; k += 256) acc += e[k] * e[k];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) *loss = (float)((((red[0] + red[1]) + red[2]) + red[3]) / B);
}

// grad[r][c] = (2/B) sum_i e_i[r] b_i[c]; T[r][c] -= lr grad[r][c].
__global__ __launch_bounds__(256) void k_lin_step(float* T, float* grad, const double* e, LinIn b,
                                                  int n, int B, float lr) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= (long long)n * n) return;
  const int r = (int)(k / n), c = (int)(k % n);
  double g = 0.0;
  for (int i = 0; i < B; ++i) g += e[(size_t)i * n + r] * b.p[i][c];
  g *= 2.0 / B;
  grad[k] = (float)g;
  T[k] = (float)((double)T[k] - (double)lr * g);
}

__global__ void k_lin_zero(float* p, long long m) {
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k < m) p[k] = 0.f;
}

inline int cdivl(long long a, long long b) { return (int)((a + b - 1) / b); }

long long lin_n(const mlg_grid* grid) {
  if (!grid || (grid->dim != 2 && grid->dim != 3)) throw ArgError{MLG_ERR_ARG, "bad grid"};
  const long long n = (long long)grid->nx * grid->ny * (grid->dim == 3 ? grid->nz : 1);
  if (grid->nx < 1 || grid->ny < 1 || (grid->dim == 3 && grid->nz < 1) || n > kLinMaxN)
    throw ArgError{MLG_ERR_ARG, "the linear model takes grids of 1..16384 points"};
  return n;
}

void check_batch(int batch) {
  if (batch < 1 || batch > kLinMaxBatch) throw ArgError{MLG_ERR_ARG, "batch must be in 1..16"};
}

size_t t_bytes(long long n) { return align_up((size_t)n * n * 4, 256); }

}  // namespace

size_t lin_param_bytes(const mlg_grid* grid) { return 2 * t_bytes(lin_n(grid)); }

size_t lin_workspace_bytes(const mlg_grid* grid, int batch) {
  const long long n = lin_n(grid);
  check_batch(batch);
  return align_up((size_t)batch * n * 8, 256);
}

int lin_init(const mlg_grid* grid, void* params, hipStream_t s) {
  const long long n = lin_n(grid);
  if (!params) throw ArgError{MLG_ERR_ARG, "params is NULL"};
  const long long m = 2 * (long long)(t_bytes(n) / 4);
  k_lin_zero<<<cdivl(m, 256), 256, 0, s>>>((float*)params, m);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

int lin_infer(const mlg_grid* grid, const void* params, int batch, const double* b, double* x0,
              hipStream_t s) {
  const long long n = lin_n(grid);
  check_batch(batch);
  if (!params || !b || !x0) throw ArgError{MLG_ERR_ARG, "NULL pointer"};
  LinIn bp{}, none{};
  LinOut op{};
  for (int i = 0; i < batch; ++i) {
    bp.p[i] = b + (size_t)i * n;
    op.p[i] = x0 + (size_t)i * n;
  }
  k_lin_apply<<<cdivl(n, 4), 256, 0, s>>>((const float*)params, bp, none, op, (int)n, batch);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

int lin_train_step(const mlg_grid* grid, void* params, float lr, int batch, const double* const* b,
                   const double* const* x, void* ws, size_t ws_bytes, float* loss, hipStream_t s) {
  const long long n = lin_n(grid);
  check_batch(batch);
  if (!params || !b || !x) throw ArgError{MLG_ERR_ARG, "NULL pointer"};
  if (!ws || ws_bytes < lin_workspace_bytes(grid, batch))
    throw ArgError{MLG_ERR_WORKSPACE, "workspace too small"};
  LinIn bp{}, xp{};
  LinOut ep{};
  double* e = (double*)ws;
  for (int i = 0; i < batch; ++i) {
    if (!b[i] || !x[i]) throw ArgError{MLG_ERR_ARG, "NULL sample pointer"};
    bp.p[i] = b[i];
    xp.p[i] = x[i];
    ep.p[i] = e + (size_t)i * n;
  }
  float* T = (float*)params;
  float* grad = (float*)((char*)params + t_bytes(n));
  k_lin_apply<<<cdivl(n, 4), 256, 0, s>>>(T, bp, xp, ep, (int)n, batch);
  k_lin_loss<<<1, 256, 0, s>>>(e, (long long)batch * n, batch, loss);
  k_lin_step<<<cdivl(n * n, 256), 256, 0, s>>>(T, grad, e, bp, (int)n, batch, lr);
  MLG_HIP(hipGetLastError());
  return MLG_OK;
}

}  // namespace mlg
