/*
 * tvpd.h -- C ABI of the MI355X (gfx950) primal-dual image-sweep library.
 *
 * Problem.  The paper's regularised inverse problem (Section 6, eq. opt:
 * data misfit plus lam times a regulariser) with the identity as forward
 * operator and the isotropic total variation as regulariser:
 *
 *     minimise_f  E(f) = 1/2 ||f - g||^2 + lam * sum_i |(grad f)_i|_2
 *
 * over images f (2D) or volumes (3D).  grad is the forward difference with
 * Neumann boundary (zero difference at the last index of every axis), and
 * div = -grad^T, the adjoint relation the paper states for its operator pair
 * (Section 1, eq. adjoint).  The solver is the first-order primal-dual
 * iteration (Chambolle & Pock 2011, Algorithm 1) with extrapolation theta:
 *
 *     fbar    = f^k + theta (f^k - f^{k-1})
 *     p^{k+1} = projection of p^k + sigma grad fbar onto {|p_i|_2 <= lam}
 *     f^{k+1} = (f^k + tau div p^{k+1} + tau g) / (1 + tau)
 *
 * from f^0 = f^{-1} = g, p^0 = 0.  The plain and batched 2D solvers form
 * the extrapolation as fbar = f^k + theta tau' (g + div p^k - f^k), tau' the
 * step that produced f^k, the same value (the data prox gives f^{k-1} =
 * (1 + tau') f^k - tau' (g + div p^k)), so their workspaces keep no f^{k-1};
 * the plain workspace records tau' for steps whose coefficients change
 * between calls.
 * Convergence needs tau sigma ||grad||^2 < 1;
 * ||grad||^2 < 8 in 2D and < 12 in 3D, so tau = sigma = 1/sqrt(8) (2D) and
 * 1/sqrt(12) (3D) are always admissible.  The duality gap of a pair (f, p) is
 *     gap = sum_i 1/2 (f_i - g_i - (div p)_i)^2 + lam |(grad f)_i| - <(grad f)_i, p_i>
 * (= P(f) - D(p) with P = E and D(p) = -1/2 ||div p||^2 - <g, div p>).
 *
 * Conventions.
 *   - Arrays are float32, dense and row-major: [ny][nx] (2D), [nz][ny][nx]
 *     (3D), batches lead: [batch][...].  x is the fastest axis.
 *   - A dual field is planar: [ndim][...], component 0 along x, 1 along y,
 *     2 along z.
 *   - "device" pointers point to memory of the current HIP device; "host"
 *     pointers to ordinary host memory.  The caller owns every buffer,
 *     including the workspace, whose size the *_workspace_size calls give;
 *     the library never allocates device memory.  A workspace must be
 *     256-byte aligned.  It holds the solver state between calls (f ring,
 *     dual ring, a padded copy of g, reduction partials and a small header).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work on it and return at once, except where a function
 *     says it synchronises the stream (those that return host results).
 *   - Every function returns a status: TVPD_OK (0) or a negative error code;
 *     tvpd_status_string() names it.  Arguments are validated before any
 *     device work is enqueued, so an error leaves the workspace untouched.
 *     Non-convergence is not an error: it is reported in tvpd_result.
 *   - Calls that share a workspace must not overlap in time.
 */
#ifndef TVPD_H
#define TVPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TVPD_OK = 0,
  TVPD_ERR_INVALID_ARG = -1, /* null pointer, bad count or parameter */
  TVPD_ERR_SHAPE = -2,       /* ndim not 2 or 3, or a non-positive size */
  TVPD_ERR_ALIGNMENT = -3,   /* workspace not 256-byte aligned */
  TVPD_ERR_WORKSPACE = -4,   /* workspace smaller than required */
  TVPD_ERR_HIP = -5,         /* a HIP runtime call failed */
  TVPD_ERR_UNSUPPORTED = -6, /* valid request the library does not handle */
  TVPD_ERR_STEP = -7,        /* tau * sigma * ||grad||^2 >= 1 (or <= 0) */
  TVPD_ERR_DEVICE = -8,      /* a device-side check failed (see string) */
  TVPD_ERR_SCRATCH = -9      /* request larger than a static scratch area */
};

/* Image or volume shape.  ndim = 2: nz must be 1.  Sizes >= 1. */
typedef struct tvpd_shape {
  int32_t ndim;
  int32_t nz, ny, nx;
} tvpd_shape;

/* Coefficients of one iteration: weight lam >= 0 on the regulariser, primal
 * step tau > 0, dual step sigma > 0, extrapolation theta in [0, 1]. */
typedef struct tvpd_coeffs {
  float lam, tau, sigma, theta;
} tvpd_coeffs;

/* Solve parameters.  The gap of (f^k, p^k) is evaluated during iteration k
 * whenever check_every > 0 and k % check_every == 0; the solve stops at the
 * first such k with gap <= gap_tol * P(f^k) and returns f^k.  gap_tol < 0
 * never stops (fixed max_iter iterations).  use_graph: 1 replays the
 * iterations as HIP graphs, 0 launches them one by one, -1 decides (graphs
 * for images of up to 2^20 pixels run one iteration per launch, else
 * direct launches). */
typedef struct tvpd_params {
  tvpd_coeffs c;
  int32_t max_iter;
  int32_t check_every;
  double gap_tol;
  int32_t use_graph;
  int32_t reserved;
} tvpd_params;

/* Result of a solve: iters = k of the returned iterate; converged = 1 if a
 * check passed; primal = P(f), dual = D(p), gap = their difference, for the
 * returned pair (evaluated at the passing check, or at the final pair when
 * no check passed). */
typedef struct tvpd_result {
  int32_t iters;
  int32_t converged;
  double primal, dual, gap;
} tvpd_result;

/* Name of a status code (static string, never NULL). */
const char* tvpd_status_string(int status);

/* Library version as 10000*major + 100*minor + patch. */
int tvpd_version(void);

/* Release the host resources the calling thread's solver drivers keep
 * between calls: pinned staging buffers, events and the stream used for
 * graph capture (tvpd_solve and tvpd_solve_batched create them on their
 * first call on a device and reuse them).  Call it before the thread or the
 * process ends, while the HIP runtime is still up; later calls recreate what
 * they need.  Must not overlap a running solve of the same thread.  Always
 * returns TVPD_OK. */
int tvpd_release_thread_resources(void);

/* A plain device copy dst[i] = src[i], i < n (16-byte loads and stores;
 * src, dst device, 16-byte aligned, not overlapping; n a multiple of 4):
 * a kernel (tvpd_copy_kernel) that moves a known number of bytes, against
 * which profilers' HBM byte counters are scaled.  TVPD_ERR_INVALID_ARG for
 * null or misaligned pointers or n not a positive multiple of 4. */
int tvpd_stream_copy(const float* src, float* dst, int64_t n, void* stream);

/* ---------------------------------------------------------------------
 * Plain solver (one image or volume).
 * ------------------------------------------------------------------- */

/* Bytes of workspace the plain solver needs for `shape` (host out). */
int tvpd_workspace_size(const tvpd_shape* shape, size_t* bytes);

/* Start a solve: f^0 = f^{-1} = g, p^0 = 0, k = 0.  g: device, dense. */
int tvpd_init(const tvpd_shape* shape, const float* g, void* ws,
              size_t ws_bytes, void* stream);

/* Run n_iter iterations with coefficients c from the current state, without
 * gap checks.  Resumable: the state stays in the workspace. */
int tvpd_step(const tvpd_shape* shape, const tvpd_coeffs* c, int32_t n_iter,
              void* ws, size_t ws_bytes, void* stream);

/* Copy the current iterate f^k (device, dense, [ny][nx] / [nz][ny][nx]) and,
 * if p_out is not NULL, the dual p^k (device, dense, [ndim][...]). */
int tvpd_read_state(const tvpd_shape* shape, const void* ws, size_t ws_bytes,
                    float* f_out, float* p_out, void* stream);

/* Current iteration index k (host out).  Synchronises the stream. */
int tvpd_iteration(const tvpd_shape* shape, const void* ws, size_t ws_bytes,
                   int32_t* k, void* stream);

/* Primal energy, dual energy and duality gap of the current pair
 * (f^k, p^k) for weight lam, accumulated in float64: out[0] = P,
 * out[1] = D, out[2] = gap (host out).  Synchronises the stream.
 * TVPD_ERR_DEVICE if a pipelined pass since the last tvpd_init recorded a
 * timed-out wait (the state is then not a valid iterate). */
int tvpd_energy_gap(const tvpd_shape* shape, float lam, void* ws,
                    size_t ws_bytes, double out[3], void* stream);

/* Full solve: init from g (device), iterate with the stopping rule of
 * tvpd_params, write the returned iterate to f_out (device, dense).  res is
 * host memory.  Synchronises the stream.  TVPD_ERR_DEVICE: a wait inside a
 * pipelined pass (tile order 2) timed out, so f_out is not valid. */
int tvpd_solve(const tvpd_shape* shape, const float* g, float* f_out,
               const tvpd_params* prm, void* ws, size_t ws_bytes,
               tvpd_result* res, void* stream);

/* ---------------------------------------------------------------------
 * Tiling of the fused 2D sweep.  A wave walks a band of `th` rows of a
 * 256-column strip; a block holds `wpb` consecutive wave tiles, numbered
 * band by band (order 0: a block's waves sit side by side) or strip by
 * strip (order 1: stacked).  order 2 selects the pipelined passes instead:
 * one block per band of `th` rows of a 232-column strip, whose waves run one
 * iteration of the pass each and hand their rows on through LDS (wpb is not
 * used; never the default, the autotuner tries it).  The iterates do not depend on the tile (halo values are
 * recomputed with the owner's arithmetic), only the speed and the summation
 * order of the gap do.
 * ------------------------------------------------------------------- */

/* Use this tile for the 2D `shape` from now on in this process (overrides
 * the default and any autotuned choice).  th in [1, 65536], order in
 * {0, 1, 2}, wpb in {1, 2, 4} for orders 0 and 1 (any value for order 2).
 * TVPD_ERR_UNSUPPORTED for a 3D shape. */
int tvpd_set_tile(const tvpd_shape* shape, int32_t th, int32_t wpb,
                  int32_t order);

/* Tile the library will use for the 2D `shape` (host out). */
int tvpd_get_tile(const tvpd_shape* shape, int32_t* th, int32_t* wpb,
                  int32_t* order);

/* Tiling of the fused 3D sweep.  A wave owns a 256-column strip and a band
 * of th rows (2 or 4) and marches through a segment of tz planes (it
 * recomputes the dual of the plane above its segment); a block holds wpb
 * consecutive wave tiles (strip fastest, then band, then segment).  The
 * iterates do not depend on the tile.  set: th in {2, 4}, tz in
 * [1, 65536], wpb in {1, 2, 4}; TVPD_ERR_UNSUPPORTED for a 2D shape. */
int tvpd_set_tile3d(const tvpd_shape* shape, int32_t th, int32_t tz,
                    int32_t wpb);
int tvpd_get_tile3d(const tvpd_shape* shape, int32_t* th, int32_t* tz,
                    int32_t* wpb);

/* Temporal blocking of the 2D solvers.  The plain solver runs its
 * iterations as passes of up to `depth` iterations per launch (f^k, p^k, g
 * read once; f^{k+n}, p^{k+n} written once: 28 bytes per n pixel-iterations,
 * against 32 per pixel-iteration for one pass per iteration that reads
 * f^{k-1}); a gap check
 * only ever falls on a pass's first iteration, so passes end before the next
 * check.  depth 0 (the default) lets each kernel take its own longest pass,
 * 5 for the strip walks and 10 for the pipelined passes; depth 1 .. 10 sets
 * it for both, the strip walks capping it at 6.  The batched solver uses
 * passes of 1, 2 and (with a walk depth >= 5) 5 iterations, the unrolled
 * solver at most 5.  The iterates are bit-identical for every depth.
 * Process-wide setting.  tvpd_set_blocking(0) is depth 1,
 * tvpd_set_blocking(1) depth 0. */
int tvpd_set_blocking(int32_t on);
int tvpd_set_pass_depth(int32_t depth);
int tvpd_get_pass_depth(int32_t* depth);

/* The longest pass (iterations per launch) the plain solver takes for the
 * 2D `shape` under the current tile and depth settings. */
int tvpd_pass_length(const tvpd_shape* shape, int32_t* n);

/* Polls after which a wait between the waves of a pipelined pass (tile
 * order 2) gives up, process-wide; 0 (the default) means 2^24 polls, about
 * half a second.  A wait that gives up lets the pass finish with invalid
 * iterates and makes tvpd_solve and tvpd_energy_gap return TVPD_ERR_DEVICE
 * until the next tvpd_init: a small limit exercises that path.  polls >= 0,
 * else TVPD_ERR_INVALID_ARG. */
int tvpd_set_wait_limit(int64_t polls);

/* Autotuner.  Times every candidate tile of the sweep on `ws`, an
 * initialised workspace of this shape, and keeps the fastest for `shape` in
 * this process.  2D: th from 2 to 256, wpb 1/2/4, orders 0 and 1, and the
 * pipelined passes (order 2) on bands of one to three tiles per CU and of
 * 64, 128 and 256 rows, timing passes of the pass depth in use.  3D: th 2/4, tz from 2 to 128,
 * wpb 1/2/4; the chosen tz is returned in *order.  The workspace state is
 * advanced by the timing runs: call tvpd_init before solving with it.  If
 * cache_path is not NULL the choice is appended to that text file (one line
 * per shape: arch ndim nz ny nx th wpb order-or-tz microseconds).  Outputs
 * (host, each may be NULL): the chosen tile and its time per iteration in
 * microseconds.  Synchronises the stream. */
int tvpd_autotune(const tvpd_shape* shape, void* ws, size_t ws_bytes,
                  const char* cache_path, int32_t* th, int32_t* wpb,
                  int32_t* order, float* us, void* stream);

/* Read tiles recorded by tvpd_autotune for the current device's
 * architecture from cache_path; later lines override earlier ones.
 * *count (host) receives the number of entries taken. */
int tvpd_tune_load(const char* cache_path, int32_t* count);

/* ---------------------------------------------------------------------
 * Batched solver: n images of different sizes (2D), each solved exactly as
 * tvpd_solve would solve it alone -- same iterates, same stopping iteration
 * -- but together on the device.  Images are packed in caller-owned arenas:
 * image i occupies ny_i * nx_i floats starting at element offsets[i] of both
 * g_arena (input) and f_arena (output).
 * ------------------------------------------------------------------- */

/* Driver and tiling of a batched solve.  mode 0: one persistent cooperative
 * launch runs every iteration (grid barriers between passes, per-image
 * stopping on the device); mode 1: one launch per pass, replayed from HIP
 * graphs of whole check intervals with the host polling a flag; mode 2:
 * plain launches, one per pass (reference driver).  Passes hold 1, 2 or 5
 * iterations (tvpd_set_pass_depth).  th: rows per wave band (0 = the
 * autotuned or default value); wpb: waves per block (0 = autotuned or
 * default, else 1, 2, 4 or 8); th_short: rows per band of the second tile
 * table, used once the running images no longer fill the grid (0 = default
 * 8; at most th); two more tables halve the band (at least 1 row) and take
 * over as images stop, whenever their tiles still fit the grid's waves.  The
 * tiling never changes the iterates. */
typedef struct tvpd_batch_opts {
  int32_t mode;
  int32_t th;
  int32_t wpb;
  int32_t th_short;
} tvpd_batch_opts;

/* Workspace bytes for a batch of n shapes (host arrays; ndim must be 2).
 * TVPD_ERR_UNSUPPORTED when the tile tables would need more than 2^31 - 1
 * entries (4 per image row and 256-column strip). */
int tvpd_batch_workspace_size(int32_t n, const tvpd_shape* shapes,
                              size_t* bytes);

/* Solve n images.  shapes, offsets (element offsets into the arenas), prm
 * (one tvpd_params per image; max_iter and check_every must agree) and res
 * (n results) are host arrays; g_arena, f_arena and ws are device memory.
 * opts may be NULL (mode 0, autotuned tiles).  Synchronises the stream.
 * TVPD_ERR_DEVICE: a grid barrier of the persistent driver timed out (the
 * grid could not be made co-resident); results are then invalid. */
int tvpd_solve_batched(int32_t n, const tvpd_shape* shapes,
                       const int64_t* offsets, const float* g_arena,
                       float* f_arena, const tvpd_params* prm,
                       const tvpd_batch_opts* opts, void* ws, size_t ws_bytes,
                       tvpd_result* res, void* stream);

/* Batch tile autotuner: times 30 iterations of the persistent driver on this
 * batch for th in {8, 16, 32, 64, 128} and wpb in {1, 2, 4}, and makes the
 * fastest the default of later batched solves in this process.  f_arena is
 * overwritten.  Outputs (host, may be NULL): th, wpb, milliseconds of the
 * 30 iterations.  Synchronises the stream. */
int tvpd_batch_autotune(int32_t n, const tvpd_shape* shapes,
                        const int64_t* offsets, const float* g_arena,
                        float* f_arena, const tvpd_params* prm, void* ws,
                        size_t ws_bytes, int32_t* th, int32_t* wpb,
                        float* ms, void* stream);

/* ---------------------------------------------------------------------
 * Unrolled (differentiable) solver.  `batch` images or volumes of one shape
 * ([batch][ny][nx] or [batch][nz][ny][nx], dense) run K iterations of the
 * method from f^0 = f^{-1} = g, p^0 = 0, each with its own coefficients
 * (lam_k, tau_k, sigma_k) = coeffs[3k .. 3k+2] (device, float32, shared by
 * the batch; theta fixed).  The output is f^K.  The backward call returns
 * dL/dg and dL/dcoeffs for a given dL/df^K by the reverse-mode adjoint of
 * the iteration (the derivative of the projection at |q| = lam is taken
 * from the identity branch).
 *
 * Checkpointing: iterations are grouped in segments of ckpt_every; the
 * forward keeps one checkpoint (f^s, f^{s-1}, p^s) per segment start and the
 * states of the last segment; the backward recomputes each earlier segment
 * from its checkpoint.  Memory grows like K/ckpt_every + ckpt_every state
 * planes; ckpt_every >= K stores every iterate and recomputes nothing.
 * ckpt_every must be >= 2 (or >= K).  No step-size check is made: the
 * coefficients are the caller's (learnable) parameters.
 * ------------------------------------------------------------------- */

/* Workspace bytes of an unrolled forward/backward pair (host out). */
int tvpd_unrolled_workspace_size(const tvpd_shape* shape, int32_t batch,
                                 int32_t K, int32_t ckpt_every, size_t* bytes);

/* Forward: g (device, dense) -> f_out = f^K (device, dense).  Leaves the
 * checkpoints in ws for tvpd_unrolled_backward. */
int tvpd_unrolled_forward(const tvpd_shape* shape, int32_t batch,
                          const float* g, const float* coeffs, int32_t K,
                          int32_t ckpt_every, float theta, float* f_out,
                          void* ws, size_t ws_bytes, void* stream);

/* Backward: needs the workspace of a forward call with the same shape,
 * batch, coeffs, K, ckpt_every and theta.  grad_f = dL/df^K (device, dense);
 * outputs grad_g (device, dense, same shape as g) and grad_coeffs (device,
 * float32 [K][3], summed over the batch).  The workspace's checkpoints stay
 * valid, so the backward may be called again. */
int tvpd_unrolled_backward(const tvpd_shape* shape, int32_t batch,
                           const float* coeffs, int32_t K, int32_t ckpt_every,
                           float theta, const float* grad_f, float* grad_g,
                           float* grad_coeffs, void* ws, size_t ws_bytes,
                           void* stream);

/* Adjoint steps of the unrolled solver: with on = 1 (the default) each step
 * is one fused pass over the data (reads f^k, f^{k-1}, p^k, g, a, b, r,
 * gbar; writes a', b', r', gbar: 60 bytes per pixel in 2D, 72 per voxel in
 * 3D); with on = 0 it is a forward-difference pass that stores p^{k+1} and t
 * followed by a backward-difference pass (92 / 116 bytes).  Both give the
 * same a', b', r' and dL/dg bit for bit; the coefficient gradients differ
 * only in summation order.  Process-wide setting. */
int tvpd_set_fused_adjoint(int32_t on);

/* ---------------------------------------------------------------------
 * Tomographic data term.  The paper's reconstruction problem (Section 6,
 * eq. opt) with its Radon transform as forward operator:
 *
 *     minimise_f  1/2 ||A f - g||^2 + lam TV(f)             (TVPD_REG_TV)
 *     minimise_f  1/2 ||A f - g||^2 + lam/2 ||f||^2         (TVPD_REG_TIKHONOV)
 *
 * (the Tikhonov form is half of eq. opt; its optimality condition is the
 * normal equation (A^T A + lam I) f = A^T g of Section 6, eq. neq2).
 *
 * Geometry, in pixel units with detector spacing 1: image f is [ny][nx]
 * (dense, row-major), pixel (a, b) centred at x = b + 1/2 - nx/2 (along
 * columns), y = a + 1/2 - ny/2 (along rows); angles theta_k = k pi / n_angles
 * (k < n_angles, the angle mesh of Section 5); bins t_i = i + 1/2 - n_det/2;
 * a sinogram is [n_angles][n_det] (dense, t fastest).
 *
 *   A f    [k][i] = sum_ab f[a][b] max(0, 1 - |x cos theta_k + y sin theta_k - t_i|)
 *              (the Radon transform, Section 1 eq. P_theta, with the line's
 *               delta replaced by the unit hat: pixel-driven, linear weights)
 *   A^T s  [a][b] = sum_k (linear interpolation of s[k][.] at x cos + y sin,
 *              zero beyond the detector's ends)
 *              (its exact transpose: the backprojection of Section 2,
 *               eq. bp_app, without the factor pi / n_angles)
 *
 * Iteration (Chambolle & Pock 2011, Algorithm 1, with the operator
 * (A, grad) and dual steps sigma_r for the sinogram dual r, sigma_p for the
 * gradient dual p):
 *     fbar    = f^k + theta (f^k - f^{k-1})
 *     r^{k+1} = (r^k + sigma_r (A fbar - g)) / (1 + sigma_r)
 *     p^{k+1} = projection of p^k + sigma_p grad fbar onto {|p_i|_2 <= lam}   (TV)
 *     f^{k+1} = f^k - tau A^T r^{k+1} + tau div p^{k+1}                       (TV)
 *     f^{k+1} = (f^k - tau A^T r^{k+1}) / (1 + tau lam)                        (Tikhonov)
 * from f^0 = f^{-1} = f0 (or 0), r^0 = 0, p^0 = 0; grad, div as above.
 * Convergence needs tau (sigma_r ||A||^2 + sigma_p ||grad||^2) <= 1 (TV) or
 * tau sigma_r ||A||^2 <= 1 (Tikhonov); tvpd_tomo_opnorm estimates ||A||^2.
 * The library does not check this condition.
 *
 * All tomography calls share one workspace type, sized by
 * tvpd_tomo_workspace_size for the geometry; it holds the iteration state
 * (k, f ring, r, p ring), padded copies of the extrapolated image and its
 * transpose, an angle table and reduction partials.
 * ------------------------------------------------------------------- */

typedef struct tvpd_tomo_geom {
  int32_t ny, nx;      /* image rows and columns, >= 1 */
  int32_t n_angles;    /* >= 1 */
  int32_t n_det;       /* >= 1 */
} tvpd_tomo_geom;

enum { TVPD_REG_TV = 0, TVPD_REG_TIKHONOV = 1 };

/* lam >= 0; tau, sigma_r > 0; sigma_p > 0 for TV (unused for Tikhonov);
 * theta in [0, 1]; reg one of TVPD_REG_*. */
typedef struct tvpd_tomo_params {
  float lam, tau, sigma_r, sigma_p, theta;
  int32_t reg;
} tvpd_tomo_params;

/* Workspace bytes for `geom` (host out).  Sizes are limited so that every
 * index fits in int32: ny, nx, n_det <= 32768, n_angles <= 65535. */
int tvpd_tomo_workspace_size(const tvpd_tomo_geom* geom, size_t* bytes);

/* sino = A f.  f: device [ny][nx]; sino: device [n_angles][n_det].  Uses the
 * workspace's scratch planes only (the iteration state is left alone). */
int tvpd_radon_forward(const tvpd_tomo_geom* geom, const float* f, float* sino,
                       void* ws, size_t ws_bytes, void* stream);

/* How A gathers the image, process-wide: with on = 1 (the default) a
 * block of 8 angles stages each image row's window of 256 columns in LDS
 * once for all 8 (blocks whose angles straddle a diagonal, or whose columns
 * spread wider, gather from memory); with on = 0 every lane gathers its
 * three columns from memory.  Both give A f bit for bit.  on in {0, 1}. */
int tvpd_set_projection_staging(int32_t on);

/* img = A^T sino.  sino: device [n_angles][n_det]; img: device [ny][nx].
 * Uses no workspace state except the angle table (rebuilt by the call). */
int tvpd_radon_backward(const tvpd_tomo_geom* geom, const float* sino,
                        float* img, void* ws, size_t ws_bytes, void* stream);

/* Start an iteration: f^0 = f^{-1} = f0 (device [ny][nx], or NULL for 0),
 * r^0 = 0, p^0 = 0, k = 0. */
int tvpd_tomo_init(const tvpd_tomo_geom* geom, const float* f0, void* ws,
                   size_t ws_bytes, void* stream);

/* n_iter >= 0 iterations from the workspace's state.  g: device
 * [n_angles][n_det], the measured sinogram. */
int tvpd_tomo_step(const tvpd_tomo_geom* geom, const float* g,
                   const tvpd_tomo_params* prm, int32_t n_iter, void* ws,
                   size_t ws_bytes, void* stream);

/* Copy the current state out (device buffers, each may be NULL): f = f^k
 * [ny][nx], r = r^k [n_angles][n_det], p = p^k [2][ny][nx] (x component
 * first).  k (host, may be NULL) receives the iteration count and
 * synchronises the stream. */
int tvpd_tomo_read(const tvpd_tomo_geom* geom, const void* ws, size_t ws_bytes,
                   float* f, float* r, float* p, int32_t* k, void* stream);

/* Energies of the current f^k (host out[3]: data term 1/2 ||A f - g||^2,
 * regulariser term, their sum), accumulated in float64.  Synchronises. */
int tvpd_tomo_energy(const tvpd_tomo_geom* geom, const float* g, float lam,
                     int32_t reg, void* ws, size_t ws_bytes, double* out,
                     void* stream);

/* ||A||^2 by `iters` >= 1 steps of the power iteration on A^T A from the
 * constant image (host out: the last Rayleigh quotient).  Uses scratch
 * planes only.  Synchronises. */
int tvpd_tomo_opnorm(const tvpd_tomo_geom* geom, int32_t iters, void* ws,
                     size_t ws_bytes, double* out, void* stream);

/* Regularised filtered backprojection (Section 6, eq. reg_sol and the
 * filter after it): f_out = (pi / n_angles) A^T F_lam g, where F_lam filters
 * every projection in t with the frequency response |nu| / (1 + lam |nu|)
 * (nu in cycles per pixel, lam >= 0 in pixels; lam = 0 is the ramp filter of
 * the standard inversion formula), as a linear convolution over the
 * detector: the circular convolution on the zero-padded grid of length L,
 * the smallest power of two >= 2 n_det.  g: device [n_angles][n_det];
 * f_out: device [ny][nx].  For L <= 4096 the filtering runs through FFTs of
 * length L (two projections per transform, O(L log L) each); beyond, as a
 * direct convolution with taps formed on the device in O(L n_det) work
 * (n_det^2 per projection).  Uses the workspace's scratch sinogram and its
 * filter region only. */
int tvpd_fbp(const tvpd_tomo_geom* geom, const float* g, float lam, float* f_out,
             void* ws, size_t ws_bytes, void* stream);

/* tvpd_fbp without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same result as tvpd_fbp, bit for bit (the same
 * kernels); g and f_out as there.  The angle table, the filter's twiddles or
 * taps and the filtered sinogram live in a static device array of 32 MiB that the library
 * holds on each device it runs on until the process ends; the call allocates
 * nothing.  Limit: n_angles * n_det <= 8093696 (TVPD_ERR_SCRATCH beyond), the
 * other limits as for tvpd_fbp.  Every call on one device shares that array:
 * calls that overlap in time on one device (other streams or threads) race
 * and must be serialised by the caller. */
int tvpd_fbp_noalloc(const tvpd_tomo_geom* geom, const float* g, float lam,
                     float* f_out, void* stream);

/* Fast backprojection by the backprojection slice theorem (Section 3, eq.
 * bst; the algorithm of Section 5).  In the cycles convention the 2D Fourier
 * transform of B g on the line at angle theta is G(nu, theta) / |nu|, G the 1D
 * transform of the projection; for sampled data B = (pi / n_angles) A^T.
 * Steps: the DFT of each zero-padded projection (length M, a power of two
 * >= 2 n_det) times K(nu) = 1/|nu|, with 1/dnu = M at nu = 0; bilinear
 * interpolation of these polar samples at the frequencies (p, q)/Q of a
 * Q x Q grid (Q a power of two >= 2 max(ny, nx)), zero beyond |nu| = 1/2;
 * the 2D inverse DFT at the pixel centres.  The result approximates
 * (pi / n_angles) A^T g; the origin rule makes it differ by about a constant
 * (which halves when the grids double).  Lengths are limited to M, Q <= 4096
 * (n_det <= 2048, ny, nx <= 2048): TVPD_ERR_UNSUPPORTED beyond.  The BST has
 * its own workspace. */
int tvpd_bst_lengths(const tvpd_tomo_geom* geom, int32_t* M, int32_t* Q);
int tvpd_bst_workspace_size(const tvpd_tomo_geom* geom, size_t* bytes);
/* img = BST backprojection of g (device [n_angles][n_det] -> [ny][nx]). */
int tvpd_bst_backproject(const tvpd_tomo_geom* geom, const float* g, float* img,
                         void* ws, size_t ws_bytes, void* stream);
/* Regularised filtered backprojection f_lam = B F_lam g (Section 6, eq.
 * reg_sol) with B computed by the BST: the steps of tvpd_bst_backproject with
 * K(nu) = 1/(1 + lam |nu|) in the second step, because the Fourier transform
 * of F_lam g on a line is G(nu) |nu| / (1 + lam |nu|) and the theorem divides
 * by |nu| (eq. reg_fst).  The kernel is finite at nu = 0, so no origin rule
 * enters and the mean of the image is kept.  g: device [n_angles][n_det];
 * img: device [ny][nx], overwritten; ws: the BST workspace
 * (tvpd_bst_workspace_size), caller-owned; nothing is allocated.  lam >= 0
 * and finite, else TVPD_ERR_INVALID_ARG; lam = 0 is the plain ramp-filtered
 * backprojection (eq. reg_fbp with lam = 0).  The same length limits as
 * tvpd_bst_backproject.  Asynchronous on `stream`. */
int tvpd_fbp_bst(const tvpd_tomo_geom* geom, const float* g, float lam, float* img,
                 void* ws, size_t ws_bytes, void* stream);
/* The polar samples of the second step, spec[k][j + M/2] = K(nu_j) G_k(nu_j)
 * for nu_j = j / M, j = -M/2 .. M/2-1 (device, complex as interleaved
 * float pairs, [n_angles][M][2]). */
int tvpd_bst_spectra(const tvpd_tomo_geom* geom, const float* g, float* spec,
                     void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Log-polar backprojection: Andersson's formula (Section 2.1, eq.
 * and_approach and and_kernel) by the algorithm of Section 5.  In log-polar
 * coordinates x = R e^rho xi_theta (R = n_det / 2, the detector's half width
 * as the paper's unit disc) the backprojection is the convolution of the
 * semi-polar sinogram [g]_L(mu, phi) (2 n_angles rays phi_j = j pi / n_angles
 * over [0, 2 pi), ray j carrying row j mod n_angles at t = +s for
 * j < n_angles, at t = -s beyond) with K(a, b) = delta(1 - e^a cos b):
 *   Step 1  [g]_L at the mesh nodes rho_i = rho_0 + (i + 1) drho, i < N_rho,
 *           by linear interpolation in t (zero beyond the detector's ends);
 *   Step 2  the kernel on the lags a_l = l drho: for each angle offset b
 *           with cos b > 0, weights 1 - |a_l - a*| / drho at the two lags
 *           around the root a* = -ln cos b (the hat form of eq.
 *           calc_and_kernel; its weights sum to one);
 *   Step 3  the convolution, periodic in the angle and linear in rho, by
 *           FFTs, with the weights drho dphi (dphi = pi / n_angles);
 *   Step 4  bilinear interpolation in (rho, theta) at the pixel centres
 *           (pixels nearer the origin than the first node take its value).
 * Mesh (table of symbols, eq. N_rho with the adaptive rho_0 of "Problem near
 * the origin"): rho_0 = ln(1 / n_det) (half a pixel from the origin),
 * N_rho = ceil((rho_top - rho_0) / -ln(1 - 2 / n_det)), drho = (rho_top -
 * rho_0) / N_rho, rho_top = max(0, ln(r_max / R)) with r_max the farthest
 * pixel centre.  The result approximates (pi / n_angles) A^T g without the
 * lines that pass within half a pixel of the origin (a fraction
 * (2/pi) asin(1 / (2 r)) of the angles at radius r: the method's loss near
 * the origin).  Limits: n_det >= 4, N_rho <= 8192 (the rho transforms have
 * length L <= 16384, the smallest power of two >= 2 N_rho - 1) and 2 n_angles
 * <= 4096 with no prime factor other than 2, 3, 5: TVPD_ERR_UNSUPPORTED
 * otherwise.  The geometry conventions are those of the tomography calls. */

/* The mesh for `geom` (host outs): N_rho, the ray count 2 n_angles, the
 * transform length L, rho_0 and drho.  Returns TVPD_ERR_UNSUPPORTED (after
 * filling the outs) for a geometry beyond the limits. */
int tvpd_lp_mesh(const tvpd_tomo_geom* geom, int32_t* n_rho, int32_t* n_phi, int32_t* L,
                 double* rho0, double* drho);

/* Workspace bytes for `geom` (host out): node and twiddle tables, the
 * kernel's spectrum and the data's ((L/2 + 1) x 2 n_angles complex values
 * each, rounded up to whole tiles), and [B g]_L (2 n_angles x N_rho floats). */
int tvpd_lp_workspace_size(const tvpd_tomo_geom* geom, size_t* bytes);

/* Prepare a workspace for `geom`: node and twiddle tables and the kernel's
 * 2D spectrum (Step 2 and its transforms), once per geometry.  Asynchronous
 * on `stream`. */
int tvpd_lp_plan(const tvpd_tomo_geom* geom, void* ws, size_t ws_bytes, void* stream);

/* img = B g by Steps 1-4 (g: device [n_angles][n_det]; img: device
 * [ny][nx]); lp_out (device, may be NULL) receives [B g]_L as
 * [2 n_angles][N_rho] floats, ray-major.  The workspace must have been
 * prepared by tvpd_lp_plan for the same geometry; otherwise img is NaN.
 * Asynchronous on `stream`. */
int tvpd_lp_backproject(const tvpd_tomo_geom* geom, const float* g, float* img,
                        float* lp_out, void* ws, size_t ws_bytes, void* stream);

/* tvpd_tomo_init(f0 = NULL) + tvpd_tomo_step(n_iter) + f_out = f^n_iter. */
int tvpd_tomo_solve(const tvpd_tomo_geom* geom, const float* g,
                    const tvpd_tomo_params* prm, int32_t n_iter, float* f_out,
                    void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TVPD_H */
