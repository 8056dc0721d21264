/*
 * mlgmres.h -- C ABI of the MI355X (gfx950) MLGMRES library.
 *
 * The library implements the hot path of "Accelerating GMRES with Deep
 * Learning in Real-Time" (Luna, Klymko, Blaschke; arXiv 2103.10975):
 * restarted GMRES(k) on the discrete Poisson problem, solved for a time
 * series of right-hand sides, started from an initial guess produced by a
 * small network that is trained in situ on the (source, solution) pairs the
 * solver produces (Section 2 and Fig. 2 of the paper).
 *
 * Conventions shared by every entry point
 *  - Pointers are DEVICE pointers unless the comment says "host".  The caller
 *    owns all device memory (inputs, outputs, workspaces, parameters).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it; the gmres_* calls also wait for it (they return
 *    host statistics), the guess_net_* calls only enqueue.
 *  - Fields are float64, row-major with x fastest: index (z*ny + y)*nx + x.
 *  - Return codes: MLG_OK (0), MLG_NOT_CONVERGED (1, gmres only), or a
 *    negative error; mlg_last_error() then holds a message (thread-local).
 *    No C++ exception crosses this boundary.
 *  - The library allocates no device memory on any call below.  It keeps a
 *    per-process cache (pinned status buffers, captured HIP graphs, a helper
 *    stream) that mlg_shutdown() releases.
 */
#ifndef MLGMRES_H
#define MLGMRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MLG_OK = 0,
  MLG_NOT_CONVERGED = 1,     /* iteration cap reached; x holds the last iterate */
  MLG_ERR_ARG = -1,          /* bad argument or shape */
  MLG_ERR_WORKSPACE = -2,    /* workspace (or parameter buffer) too small */
  MLG_ERR_HIP = -3,          /* a HIP runtime call failed */
  MLG_ERR_NONFINITE = -4     /* a NaN/Inf appeared (e.g. in the initial guess) */
};

enum { MLG_FP64 = 0, MLG_FP32_IR = 1 };

/*
 * The discrete problem (paper Section 1.4, eq. for A u = f; benchmark of
 * Section 3): A = -lap_h, the zero-Dirichlet 5-point (dim 2) or 7-point
 * (dim 3) Laplacian on the unit square/cube with nx, ny[, nz] interior points
 * per axis and h_i = 1/(n_i + 1); (A u)_p = sum_axes (2 u_p - u_{p-e} -
 * u_{p+e}) / h_axis^2 with u = 0 outside the grid.  nz is ignored in 2D.
 */
typedef struct {
  int32_t dim;
  int32_t nx, ny, nz;
} mlg_grid;

/*
 * Solver options (GMRES(k) of Section 1.3; the paper fixes neither k, the
 * tolerance nor the precision).
 *   restart_m     k of GMRES(k), 1..64.
 *   precision     MLG_FP64: Krylov basis stored in FP64.  MLG_FP32_IR: basis
 *                 stored in FP32, every cycle restarted from the FP64 true
 *                 residual (iterative refinement: FP64 residual, Givens/least
 *                 squares and solution update; FP32 Arnoldi vectors).
 *   rtol          stop when |b - A x| <= rtol |b| (true residual, FP64).
 *   max_iters     cap on Arnoldi steps (0 = 10^9).
 *   fixed_iters   > 0: ignore rtol and run exactly this many Arnoldi steps,
 *                 restarting every restart_m (trajectory comparisons).
 *   tile          0 = autotuned/default tile shape; otherwise an index into
 *                 the tile table (mlg_tile_count / mlg_tile_shape).
 *   poll_cycles   restart cycles enqueued between host polls of the
 *                 convergence flag (0 = 1) when a call holds several
 *                 right-hand sides; a single one is polled after every
 *                 cycle (or cycle part, see gmres_solve).
 *   schedule      how an Arnoldi step sweeps the basis (same arithmetic):
 *                 0 = as tuned by mlg_autotune for this grid (separate sweeps
 *                 when untuned), 1 = separate extend and dot-product sweeps,
 *                 2 = the fused single sweep wherever the grid is 2D, 3 = the
 *                 fused sweep in the split form wherever the grid is 2D: the
 *                 step's partials are summed by many workgroups at once and
 *                 every workgroup of the sweep forms the step's coefficients
 *                 itself (bitwise the same results as 2).
 *   launch        how restart cycles reach the device (same kernels, same
 *                 order, bitwise the same results): 0 = as tuned by
 *                 mlg_autotune for this grid (graph replay when untuned),
 *                 1 = replay of a captured graph of the cycle, 2 = direct
 *                 kernel launches.  gmres_solve_static always launches
 *                 directly.
 */
typedef struct {
  int32_t restart_m;
  int32_t precision;
  double rtol;
  int64_t max_iters;
  int64_t fixed_iters;
  int32_t tile;
  int32_t poll_cycles;
  int32_t schedule;
  int32_t launch;
} mlg_opts;

/* Per-solve statistics (host).  relres_first_cycle is the paper's metric E_k
 * (Section 2.2): the true relative residual after the first restart cycle. */
typedef struct {
  int32_t status;
  int32_t cycles;
  int64_t iters;               /* Arnoldi steps (products A v) */
  double relres_init;          /* |b - A x0| / |b| */
  double relres_first_cycle;   /* E_k */
  double relres_est;           /* last Givens estimate / |b| */
  double relres_true;          /* final true relative residual (FP64) */
  double seconds;              /* host wall time of the call (TOS of Section 2.2) */
  double relres_iter5;         /* Givens residual estimate / |b| after the 5th Arnoldi
                                  step (after the last one if fewer were taken): the
                                  fifth-iteration residual Section 3 judges guesses by */
} mlg_stats;

/* ---------------------------------------------------------------- solver */

/* Bytes of device workspace gmres_solve needs for this grid and options
 * (0 on invalid arguments).  The workspace holds the Krylov basis
 * ((m+1) n elements of the basis precision), the FP64 residual, reduction
 * partials and the device-side solver state. */
size_t gmres_workspace_bytes(const mlg_grid* grid, const mlg_opts* opts);

/*
 * Restarted GMRES(k) (Section 1.3): x0 -> r0 = b - A x0, minimise the residual
 * over K_k(A, r0) (Arnoldi with classical Gram-Schmidt applied twice, Givens
 * rotations, back substitution), x += V y, restart from the last iterate until
 * the true residual meets rtol.  A cycle stops early when the Givens residual
 * estimate reaches rtol |b| or on breakdown; acceptance is on the recomputed
 * true residual.
 * The library remembers, per workspace and plan, how many Arnoldi steps each
 * cycle of the last solve took, and launches a cycle that ended early then in
 * two parts split just after that count: the second part only if the cycle
 * is still running after the first.  The kernels and their order are the same
 * either way, so the result does not depend on this history.
 *   b      [n] right-hand side (read only).
 *   x      [n] initial guess on entry, solution on exit.
 *   ws     >= gmres_workspace_bytes(grid, opts) bytes, 256-byte aligned.
 *   stats  host, may be NULL.
 * Blocks until the solve has finished on `stream`.  b = 0 gives x = 0.
 * Returns MLG_OK, MLG_NOT_CONVERGED, or an error (x then undefined).
 */
int gmres_solve(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts,
                void* ws, size_t ws_bytes, mlg_stats* stats, void* stream);

/* Largest workspace gmres_solve_static can hold (64 MiB). */
#define MLG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * gmres_solve for callers that cannot allocate device memory (serving loops
 * and harnesses that forbid hipMalloc): the same solve, with the same result
 * bit for bit, but its workspace lives in a static array inside the library
 * (MLG_STATIC_SCRATCH_BYTES on every device the library runs on, held until
 * the process ends).  The call allocates nothing: no device or pinned host
 * memory, no graph, no event; the cycles are enqueued directly on `stream`.
 *   b, x, stats, stream  as for gmres_solve.
 * Returns MLG_ERR_WORKSPACE (nothing launched) when gmres_workspace_bytes
 * for this grid and these options exceeds MLG_STATIC_SCRATCH_BYTES.
 * The array keeps the last call's contents; every call sets up what it
 * reads.  Calls on one device share the array: the library serialises them
 * within a process (each blocks until its solve has finished), and nothing
 * else may run a solve on that array while one is in flight.
 */
int gmres_solve_static(const mlg_grid* grid, const double* b, double* x, const mlg_opts* opts,
                       mlg_stats* stats, void* stream);

/* One independent system of a batched solve: nrhs right-hand sides solved in
 * order; guess 0 starts each from zero, 1 from the previous solution of the
 * same system (the first from x's initial contents). */
typedef struct {
  mlg_grid grid;
  int32_t nrhs;
  int32_t guess;
  const double* b;   /* [nrhs][n] */
  double* x;         /* [nrhs][n]; x[0] holds the first initial guess */
} mlg_system;

size_t gmres_batched_workspace_bytes(int32_t nsys, const mlg_system* sys, const mlg_opts* opts);

/*
 * Solve many independent systems of uneven size together: every restart
 * cycle is one graph replay over the tiles of all still-active systems; a
 * system that converges advances to its next right-hand side on the device.
 *   stats  host, [sum of nrhs] in system order, may be NULL.
 * Each solution equals gmres_solve on the same system and RHS.
 */
int gmres_solve_batched(int32_t nsys, const mlg_system* sys, const mlg_opts* opts,
                        void* ws, size_t ws_bytes, mlg_stats* stats, void* stream);

/* y = A u on the device (the operator of every solve), for checks. */
int mlg_apply_operator(const mlg_grid* grid, const double* u, double* y, void* stream);

/*
 * Kernel timing (measurement support).  Times `reps` back-to-back launches of
 * one solver kernel, in the launch configuration gmres_solve uses, with HIP
 * events on `stream`, and returns the average duration in microseconds.
 * Kernels of one Arnoldi step j: MLG_K_DOTS (w = A u_j and the block dot
 * products), MLG_K_COEF (one-workgroup sum, Hessenberg column, Givens),
 * MLG_K_EXTEND (new basis vector v_j and direction u_{j+1}), MLG_K_STEP (the
 * solver's fused form of MLG_K_EXTEND at j and MLG_K_DOTS at j+1, one sweep
 * over the basis), MLG_K_SUMS (the split form's column sums of the partials,
 * one wavefront per column), MLG_K_STEPC (MLG_K_STEP in the split form: the
 * coefficient update of MLG_K_COEF from those sums, then the sweep); once per
 * cycle: MLG_K_UPDATE (x += V y) and MLG_K_RESIDUAL (r = b - A x).
 *   ws       the workspace of a finished gmres_solve with the same grid and
 *            opts (its basis and coefficients are the kernel inputs; the
 *            reduction partials, the residual buffer, and for MLG_K_EXTEND,
 *            MLG_K_STEP, MLG_K_STEPC and MLG_K_UPDATE basis vector `step`,
 *            the direction buffers and x are overwritten).  MLG_K_STEPC
 *            takes the sums of a unit direction orthogonal to the basis.
 *   scratch  >= mlg_kernel_bench_scratch_bytes(reps) bytes: one private copy
 *            of the solver state per launch, so every launch does full work.
 *   step     Arnoldi index j: 0..m (0..m-1 for MLG_K_EXTEND, MLG_K_STEP and
 *            MLG_K_STEPC).
 */
enum { MLG_K_DOTS = 0, MLG_K_COEF = 1, MLG_K_EXTEND = 2, MLG_K_UPDATE = 3, MLG_K_RESIDUAL = 4,
       MLG_K_STEP = 5, MLG_K_SUMS = 6, MLG_K_STEPC = 7 };
size_t mlg_kernel_bench_scratch_bytes(int32_t reps);
int mlg_kernel_bench(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes,
                     void* scratch, size_t scratch_bytes, int32_t kind, int32_t step, int32_t reps,
                     double* avg_us, void* stream);

/* Tile table used by the solver kernels. */
int32_t mlg_tile_count(int32_t dim);
int mlg_tile_shape(int32_t dim, int32_t index, int32_t* tx, int32_t* ty, int32_t* tz);

/*
 * Autotuner.  For one grid and option set (precision, restart_m), times every
 * tile shape and, per Arnoldi step, the separate extend + dot-product sweeps
 * against the fused sweep (kernel timings), then whole restart cycles of
 * every tile with the fused steps' sums in either form, on synthetic data in
 * `ws`, in the launch configuration the solver uses, then whole solves of
 * the chosen configuration with graph replay against direct launches;
 * records the fastest tile, per-step schedule and launch mode in a
 * process-wide table that gmres_solve / gmres_solve_batched consult when
 * opts->tile == 0 (tile), opts->schedule == 0 (schedule) and opts->launch
 * == 0 (launch mode).  A batched solve takes the entry of its largest system
 * per dimension (and launches directly only when every dimension's entry
 * chose that).
 *   ws      >= mlg_autotune_workspace_bytes(grid, opts) bytes (overwritten).
 *   tile    host, may be NULL: the chosen tile index (1-based, as opts->tile).
 *   fused   host, may be NULL: bit j set = step j runs fused.
 *   split   host, may be NULL: bit j set = ... in the split form (a subset
 *           of `fused`).
 *   launch  host, may be NULL: the chosen launch mode (1 graph, 2 direct, as
 *           opts->launch).
 * Blocks until done.  Entries live until mlg_shutdown.
 */
size_t mlg_autotune_workspace_bytes(const mlg_grid* grid, const mlg_opts* opts);
int mlg_autotune(const mlg_grid* grid, const mlg_opts* opts, void* ws, size_t ws_bytes,
                 int32_t* tile, uint64_t* fused, uint64_t* split, int32_t* launch,
                 void* stream);

/* ---------------------------------------------------------------- network */

/*
 * Guess network (the learned initial guess x0 = N(b) of Section 2; a
 * non-local architecture as Section 2.1 asks for).  2D grids only.
 *   inputs (r / s_r, f / s_f): r = f - A u_prev, the FP64 residual of the
 *      previous solution under the solver's operator A (a fixed first layer),
 *      s_r = RMS(r), s_f = RMS(f) (a zero scale divides as 1), c_u = 2 pi^2
 *   L1 conv3x3 2->C + ReLU, L2 conv3x3 C->C + ReLU,
 *   L3 spectral: ReLU(W1 x + b + S^-1[W_kl . S[x]_kl]) over the modes x modes
 *      slowest sine modes (S = DST-I basis), per-mode C x C mixing,
 *   L4, L5 conv3x3 C->C + ReLU, L6 conv3x3 C->1;
 *   band path (FP64, skip_modes = K > 0) over the K x K slowest sine modes:
 *      band = S^-1[w_kl S[r/s_r]_kl] with per-mode weights w learned from the
 *      training pairs by least squares (w = sxt / sxx, the running sums of
 *      X T and X^2 that every train step extends; for the correction
 *      d = u_target - u_prev, X and T are the band coefficients of A d / s_r
 *      and of the target c_u d / s_r -- u_target solves A u = f - r_fin
 *      exactly, so (A d, d) is an exact pair: the minimiser of the loss over
 *      w on those pairs, which Adam could not reach at the precision GMRES
 *      needs as the optimal weights span several orders of magnitude);
 *   out = g (L6 - P_K L6) + band, P_K the orthogonal projection on the band:
 *      the band path alone sets the output there, the convolutions the rest,
 *      scaled at inference by their output gain g (the least-squares scale
 *      of the branch's off-band output against the off-band targets, from
 *      running sums over the training batches that decay by 0.9 per step; 1
 *      before any batch; training sees g = 1) (K = 0: out = L6, the network
 *      without a band path);
 *   guess = u_prev + (s_r / c_u) out  (= u_prev when u_prev solves A u = f).
 * Weights and activations are BF16 in the kernels with FP32 accumulation;
 * FP32 master weights and Adam moments (Section 2.3: back-propagation and
 * ADAM) live in the parameter buffer.
 */
typedef struct {
  int32_t channels;   /* C, 32 */
  int32_t modes;      /* M, 16; 1..32 (the L3 spectral layer) */
  int32_t skip_modes; /* K, 64; 0..128 (the band path; 0 = none) */
  float lr, beta1, beta2, eps;
  uint64_t seed;
} guess_net_cfg;

/*
 * Parameter buffer layout (device, 256-byte aligned regions, in this order):
 *   master  FP32 [P]   weights in the tensor order below
 *   grad    FP32 [P]   gradient of the last train step
 *   adam_m  FP32 [P], adam_v FP32 [P]
 *   bf16    BF16 [P]   working copy used by the kernels
 *   step    int64      Adam step counter (256 bytes reserved)
 *   band    FP64 [2][K][K]  least-squares state of the band path: sxt
 *                      ([ky][kx]) then sxx; w = sxt / sxx (0 where sxx = 0).
 *                      A caller may write it directly (e.g. sxt = w,
 *                      sxx = 1 to impose weights w).
 *   gate    FP64 [2]   output gain state: sums of <c, t> and |c|^2 (g = their
 *                      ratio; 1 while the second is 0)
 * Tensor order inside each FP32/BF16 array (shapes [out, in, ky, kx]):
 *   conv1.w [C,2,3,3] conv1.b [C] conv2.w [C,C,3,3] conv2.b [C]
 *   spec.w1 [C,C] spec.b [C] spec.wk [M,M,C,C] (= [ky, kx, out, in])
 *   conv4.w conv4.b conv5.w conv5.b (as conv2) conv6.w [1,C,3,3] conv6.b [1]
 * guess_net_param_count gives P; guess_net_param_offset the element offset
 * of tensor `index` (0..12 in the order above; 13 gives P) inside one array.
 */
int64_t guess_net_param_count(const guess_net_cfg* cfg);
int64_t guess_net_param_offset(const guess_net_cfg* cfg, int32_t index);
size_t guess_net_param_bytes(const guess_net_cfg* cfg);

/* Device workspace for infer (train = 0) or train_step (train = 1) on an
 * nx x ny grid with `batch` samples. */
size_t guess_net_workspace_bytes(const guess_net_cfg* cfg, const mlg_grid* grid,
                                 int32_t batch, int32_t train);

/* Deterministic initialisation from cfg->seed: He-uniform weights, zero
 * biases, zero output layer, an empty band state (w = 0) and gain state, so
 * the untrained network returns u_prev; zero Adam state. */
int guess_net_init(const guess_net_cfg* cfg, void* params, void* stream);

/* Recompute the BF16 working copy from the FP32 master weights (after the
 * caller wrote master weights directly) and zero the Adam state; the band
 * state is left as it is. */
int guess_net_refresh(const guess_net_cfg* cfg, void* params, void* stream);

/* guess[b] = N(f[b], u_prev[b]) for `batch` samples of one grid (FP64 in/out,
 * [batch][n] contiguous). */
int guess_net_infer(const guess_net_cfg* cfg, const void* params, const mlg_grid* grid,
                    int32_t batch, const double* f, const double* u_prev, double* guess,
                    void* ws, size_t ws_bytes, void* stream);

/*
 * One training step on L = (1/B) sum_b |out_b - t_b|^2 with out the network
 * output and t_b = c_u (u_target_b - u_prev_b) / s_b, s_b = s_r of the sample
 * with 0 replaced by 1 (Section 2.3 loss, in the network's output units): the
 * loss at the current weights, then the band state takes the batch's sums
 * (least squares), and every other weight one Adam step on its gradient
 * (the convolutional branch sees the loss off the band).
 * f, u_prev, u_target: host arrays of `batch` device pointers (samples need
 * not be contiguous).  loss: device float, may be NULL.
 */
int guess_net_train_step(const guess_net_cfg* cfg, void* params, const mlg_grid* grid,
                         int32_t batch, const double* const* f, const double* const* u_prev,
                         const double* const* u_target, void* ws, size_t ws_bytes,
                         float* loss, void* stream);

/* ------------------------------------------------- multi-scale network */

/*
 * The multi-scale guess network of Section 2.1: a variant of the FluidNet
 * pressure model with residual blocks stacked before the output layer and
 * appended while training runs.  2D grids whose sides are multiples of
 * 2^(levels-1).
 *   inputs   (r / s_r, f / s_f) as for guess_net (r = f - A u_prev in FP64)
 *   pyramid  X_0 = inputs, X_l = 2x2 average pool of X_{l-1}, l < levels
 *   level l  y_l = ReLU(conv3x3 C->C (ReLU(conv3x3 2->C (X_l))))
 *   sum      S_0 = sum_l of y_l upsampled (nearest, 2^l x 2^l) to the grid
 *   block i  S_{i+1} = S_i + conv3x3(ReLU(conv3x3(S_i))), i < blocks
 *   head     out = conv3x3 C->1 (ReLU(conv3x3 C->C (S_blocks)))
 *   guess    u_prev + (s_r / c_u) out
 * `blocks` (0..max_blocks) is an argument of every call: storage exists
 * for max_blocks, and the caller grows the active count (a new block's
 * second convolution starts at zero, so it begins as the identity).
 * BF16 weights and activations, FP32 accumulation, FP32 master weights and
 * Adam moments, as for guess_net.
 */
typedef struct {
  int32_t channels;   /* C, 32 */
  int32_t levels;     /* pyramid levels, 1..6 (levels - 1 poolings) */
  int32_t max_blocks; /* residual blocks with storage, 0..8 */
  float lr, beta1, beta2, eps;
  uint64_t seed;
} fluid_net_cfg;

/*
 * Parameter buffer: the same regions as guess_net (master, grad, adam_m,
 * adam_v FP32 [P]; bf16 [P]; int64 step).  Tensor order (shapes [out, in,
 * ky, kx]): for each level l: conv1.w [C,2,3,3] conv1.b [C] conv2.w
 * [C,C,3,3] conv2.b [C]; for each block i < max_blocks: a.w [C,C,3,3] a.b
 * [C] b.w [C,C,3,3] b.b [C]; then head.conv1.w [C,C,3,3] head.conv1.b [C]
 * head.conv2.w [1,C,3,3] head.conv2.b [1].  fluid_net_param_offset gives the
 * element offset of tensor `index` (0 .. 4 levels + 4 max_blocks + 4).
 */
int64_t fluid_net_param_count(const fluid_net_cfg* cfg);
int64_t fluid_net_param_offset(const fluid_net_cfg* cfg, int32_t index);
size_t fluid_net_param_bytes(const fluid_net_cfg* cfg);

/* Device workspace for infer (train = 0) or train_step (train = 1); it holds
 * the activations of all max_blocks blocks. */
size_t fluid_net_workspace_bytes(const fluid_net_cfg* cfg, const mlg_grid* grid,
                                 int32_t batch, int32_t train);

/* Deterministic initialisation from cfg->seed: He-uniform weights, zero
 * biases, zero second convolution in every block, zero output layer (the
 * untrained network returns u_prev), zero Adam state. */
int fluid_net_init(const fluid_net_cfg* cfg, void* params, void* stream);

/* BF16 working copy from the FP32 master weights; zero Adam state. */
int fluid_net_refresh(const fluid_net_cfg* cfg, void* params, void* stream);

/* guess[b] = N(f[b], u_prev[b]) with `blocks` active blocks (FP64 in/out,
 * [batch][n] contiguous). */
int fluid_net_infer(const fluid_net_cfg* cfg, const void* params, int32_t blocks,
                    const mlg_grid* grid, int32_t batch, const double* f,
                    const double* u_prev, double* guess, void* ws, size_t ws_bytes,
                    void* stream);

/* One Adam step on the guess_net loss with `blocks` active blocks; the
 * gradients of inactive blocks are zero, so they do not move.  Arguments as
 * guess_net_train_step. */
int fluid_net_train_step(const fluid_net_cfg* cfg, void* params, int32_t blocks,
                         const mlg_grid* grid, int32_t batch, const double* const* f,
                         const double* const* u_prev, const double* const* u_target,
                         void* ws, size_t ws_bytes, float* loss, void* stream);

/* ------------------------------------------------- linear model */

/*
 * The single-layer linear model of Section 3: x0 = T b with one dense
 * n x n matrix T (n = points of the grid, 1..16384), the paper's simplified
 * network for studying the spectrum of A T.  T is FP32, row-major over the
 * grid's row-major points; products accumulate in FP64.
 * Parameter buffer (device): T FP32 [n*n], then (256-byte aligned) the
 * gradient of the last train step FP32 [n*n].
 */
size_t linear_guess_param_bytes(const mlg_grid* grid);

/* Device workspace of a train step with `batch` (1..16) samples. */
size_t linear_guess_workspace_bytes(const mlg_grid* grid, int32_t batch);

/* T = 0 and gradient = 0 (the untrained model guesses zero). */
int linear_guess_init(const mlg_grid* grid, void* params, void* stream);

/* x0[i] = T b[i] for `batch` (1..16) samples, [batch][n] contiguous, FP64. */
int linear_guess_infer(const mlg_grid* grid, const void* params, int32_t batch,
                       const double* b, double* x0, void* stream);

/*
 * One gradient-descent step on L = (1/B) sum_i |T b_i - x_i|^2 (Section 2.3
 * loss): T -= lr (2/B) sum_i (T b_i - x_i) b_i^T.  b, x: host arrays of
 * `batch` device pointers to FP64 [n]; loss: device float (L before the
 * step), may be NULL.
 */
int linear_guess_train_step(const mlg_grid* grid, void* params, float lr, int32_t batch,
                            const double* const* b, const double* const* x, void* ws,
                            size_t ws_bytes, float* loss, void* stream);

/* ---------------------------------------------------------------- misc */
const char* mlg_last_error(void);
void mlg_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* MLGMRES_H */
