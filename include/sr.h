/*
 * sr.h -- C ABI of the structured random phase retrieval library (libsrpr.so).
 *
 * The library applies the structured sensing operator of Hu, Tachella, Unser
 * and Dong, "Structured Random Model for Fast and Robust Phase Retrieval"
 * (arXiv 2409.05734), section III, Eq. (5):
 *
 *     A = S F D_L ... F D_1 U,    y = |A x|^2                       (Eq. (1))
 *
 * The transforms run on a grid of G_k = max(N_k, M_k) points per axis.  U
 * zero-pads the signal (n = N1*N2 entries) into the centred window of the
 * grid (oversampling, M > N), S keeps the centred M1 x M2 window of it
 * (undersampling, M < N; the identity when M = G), both at offset
 * floor((G-N)/2) resp. floor((G-M)/2) per axis.  D_l = diag(exp(i theta_l))
 * are the random phase diagonals on the grid and F is the unitary DFT (1D,
 * or the separable 2D DFT for images).  On top of A and A^H it runs the paper's two
 * solvers: the spectral initialisation (shifted power iteration on
 * A^H diag(T(y)) A, section II-B.2, Eq. (3)-(4)) and gradient descent on the
 * l2 intensity loss (section II-B.1, Eq. (2)), and it also provides the dense
 * i.i.d. complex Gaussian model (section II-A) as an MFMA baseline.
 *
 * Conventions shared by every call:
 *  - Complex numbers are interleaved float pairs (re, im) ("complex64"),
 *    arrays are row-major and contiguous.
 *  - Every data pointer is a DEVICE pointer owned by the caller unless the
 *    comment says "host".  The library never frees caller memory.
 *  - Calls are asynchronous and ordered on the plan's HIP stream (a call may
 *    run part of its work on a second stream the plan owns, forked from and
 *    joined back into the plan's stream within the call, so the ordering
 *    holds); argument and shape errors are reported synchronously by the
 *    return value, before any work is enqueued.  Device-side failures
 *    surface at sr_plan_sync().
 *  - A plan holds several problems; per-problem arrays are concatenated in
 *    problem order (offsets from sr_plan_offsets).
 *  - No call aborts the process and no C++ exception crosses this boundary.
 *    sr_last_error() gives a thread-local description of the last failure.
 *  - A plan must not be used from two host threads at the same time.
 */
#ifndef SR_H_
#define SR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sr_plan_s* sr_plan;

typedef enum {
  SR_OK = 0,
  SR_E_ARG = -1,          /* null pointer, bad count or value */
  SR_E_SHAPE = -2,        /* inconsistent shapes (M < N, theta out of range, ...) */
  SR_E_UNSUPPORTED = -3,  /* valid but not implemented (e.g. an FFT length with a prime factor > 3) */
  SR_E_HIP = -4,          /* a HIP runtime call failed */
  SR_E_NONFINITE = -5,    /* a solve produced NaN or Inf (reported by sr_plan_sync), or a step is not finite */
  SR_E_STATE = -6,        /* call not valid for this plan (e.g. structured call on a dense plan) */
  SR_E_NOMEM = -7         /* device allocation failed, or a caller workspace is too small */
} sr_status;

typedef enum {
  SR_STRUCTURED = 0,  /* A = S F D_L ... F D_1 U (section III, Eq. (5); any alpha: U pads, S trims) */
  SR_DENSE = 1        /* i.i.d. complex Gaussian A given as an explicit m x n matrix (section II-A) */
} sr_kind;

typedef enum {
  SR_LOSS_L2 = 0,          /* l2 intensity loss || |Ax|^2 - y ||^2 (section II-B.1, Eq. (2)) */
  SR_LOSS_POISSON = 1      /* Poisson negative log-likelihood of the intensities (see sr_plan_set_loss) */
} sr_loss;

/* SR_SCHED_AUTO: a structured plan whose problems share one 2D geometry
 * (phase blocks all one block, or evenly spaced at least one block apart) runs
 * as a stack: each fused pass of every problem in one launch, with results
 * bitwise equal to SR_SCHED_LOOP (A, A^H, both VJPs, GD, and power
 * iteration; GD with a loss trace and power iteration only where the tiles of
 * the pass that sums per-problem partials hold whole problems, else the
 * loop); the first stacked call allocates two grids per problem (plus
 * small per-problem arrays) beside the workspace, kept until sr_plan_destroy.
 * Other plans of 8 or more problems take the batched schedule.
 * SR_SCHED_BATCHED: every 2D problem advances one fused pass per launch
 * (one launch per pass level over all problems: A, A^H, GD, power
 * iteration and both derivatives, the latter where no two problems share
 * a phase block);
 * GD and power iteration run the problems with a 96-, 192- or 384-point axis
 * on a second stream beside the others; with SR_LDS_RESIDENT=1, problems
 * whose grid fits one workgroup's LDS solve there instead, beside the
 * levels.                                                                   */
typedef enum {
  SR_SCHED_AUTO = 0,       /* library's choice (above) */
  SR_SCHED_LOOP = 1,       /* one problem after another, one launch per fused pass */
  SR_SCHED_BATCHED = 2     /* all problems together (level launches, above) */
} sr_schedule;

/* One phase-retrieval problem.
 *  ndim      1 (vector) or 2 (image)
 *  n[0..1]   signal shape N1 (, N2); n[1] ignored for ndim == 1
 *  m[0..1]   measurement shape M1 (, M2); per axis M >= N pads the signal
 *            (oversampling) and M < N trims the transformed grid (undersampling)
 *  layers    L >= 1 phase layers (structured only)
 *  kind      sr_kind; all problems of a plan have the same kind
 *  theta_offset  offset, in floats, of this problem's L phase grids (L*g
 *            floats, g = G1*G2 grid points) inside the plan's theta buffer
 *            (problems may share a set of phases)                            */
typedef struct {
  int32_t ndim;
  int32_t n[2];
  int32_t m[2];
  int32_t layers;
  int32_t kind;
  int64_t theta_offset;
} sr_problem;

/* Create a plan for nprob problems.
 *  probs        host array of nprob problem descriptors
 *  theta_host   host, theta_len floats: phases theta_l of every problem, each
 *               problem's block is L consecutive G1 x G2 grids (layer-major,
 *               row-major grid) starting at probs[p].theta_offset.  Copied into
 *               the plan.
 *               Must be NULL (theta_len 0) for SR_DENSE plans.
 *  dense_A      SR_DENSE only: device pointer to the m x n complex64 matrix,
 *               row-major, shared by all problems of the plan (all problems
 *               must then have the same shape); the caller keeps it alive
 *               until sr_plan_destroy.  NULL for SR_STRUCTURED.
 *  hip_stream   hipStream_t to order all work on (NULL = default stream)
 * Grid lengths G_k must be one of 16, 32, 64, 96, 128, 192, 256, 384, 512,
 * 768, 1024, 2048 (2D), or one of those or 4096 with L*G <= 4096 (1D).
 * Dense problems (any m, n) need an even signal length n; otherwise
 * SR_E_UNSUPPORTED.  Allocates the plan's device workspace.                 */
sr_status sr_plan_create(sr_plan* out, const sr_problem* probs, int32_t nprob, const float* theta_host,
                         int64_t theta_len, const void* dense_A, void* hip_stream);

/* Replace the plan's phases by theta_len floats read from DEVICE memory
 * (stream-ordered copy; same layout as at creation).                          */
sr_status sr_plan_set_theta(sr_plan plan, const float* theta_dev, int64_t theta_len);

/* Bytes of device workspace the plan uses (allocated by sr_plan_create).      */
sr_status sr_plan_workspace_size(sr_plan plan, size_t* bytes);

/* Move the plan's workspace (phases and their exp(i theta) table, twiddles,
 * pass buffers, reduction scratch) into caller-owned device memory, e.g. a
 * tensor of the caller's allocator.
 *  dev_ptr  device pointer, 256-byte aligned, at least
 *           sr_plan_workspace_size bytes, not overlapping the current
 *           workspace; the caller keeps it alive until sr_plan_destroy (or
 *           the next sr_plan_set_workspace) and frees it afterwards.
 * Waits for the plan's queued work, copies the contents, releases the
 * plan's own allocation (the caller's earlier memory is left alone) and
 * drops recorded schedules and captured graphs (they are rebuilt on use).
 * Memory the plan allocates on first use of some schedules (stacks, batched
 * levels, derivatives) stays the plan's.  SR_E_ARG on NULL, short or
 * misaligned memory.                                                       */
sr_status sr_plan_set_workspace(sr_plan plan, void* dev_ptr, size_t bytes);

/* Per-problem offsets (in complex elements) into concatenated signal arrays
 * (x_off, n-sized) and measurement arrays (y_off, m-sized).  Both are host
 * arrays of nprob + 1 entries; either may be NULL.                           */
sr_status sr_plan_offsets(sr_plan plan, int64_t* x_off, int64_t* y_off);

/* Choose how multi-problem plans are scheduled (sr_schedule).                */
sr_status sr_plan_set_schedule(sr_plan plan, int32_t schedule);

/* Choose the loss sr_gd_solve descends, for every problem of the plan and
 * every later call (default SR_LOSS_L2).  Section II-B.1 notes that the loss
 * can follow the noise model; SR_LOSS_POISSON is the negative Poisson
 * log-likelihood of the intensities, sum_i |z_i|^2 - y_i log(|z_i|^2 + eps)
 * (z = A x), whose gradient step replaces the residual (|z|^2 - y) . z by
 * (1 - y / (|z|^2 + eps)) . z; eps > 0 guards the logarithm and the division
 * and is ignored for SR_LOSS_L2.  The step keeps its meaning (x <- x - eta
 * A^H r / m); for the Poisson loss a step of order mu / c (c as for
 * sr_spectral_init) plays the part of mu / (c mean(y)).  The loss trace
 * records the chosen loss.  SR_E_ARG for an unknown loss, or for
 * SR_LOSS_POISSON with eps not finite and positive.                          */
sr_status sr_plan_set_loss(sr_plan plan, int32_t loss, float eps);

/* Wait for all work of the plan's stream; reports device-side failures:
 *  SR_E_HIP        a HIP call failed, or a grid-wide barrier wait of the
 *                  persistent solver exceeded its bound;
 *  SR_E_NONFINITE  a GD or spectral solve since the previous sync returned a
 *                  NaN or Inf entry (final iterate, spectral estimate, or an
 *                  entry of a loss trace): the solve diverged (step too large)
 *                  or its inputs held NaN / Inf.  The results are still
 *                  written; the flag is cleared once reported.                */
sr_status sr_plan_sync(sr_plan plan);

/* Free the plan and its workspace (after waiting for its stream).             */
sr_status sr_plan_destroy(sr_plan plan);

/* z = A x and/or y = |A x|^2 (Eq. (1), Eq. (5)).
 *  x  complex64, concatenated signals (x_off layout)
 *  z  complex64, concatenated m-grids (y_off layout), or NULL
 *  y  float, concatenated m-grids (y_off layout), or NULL                    */
sr_status sr_forward(sr_plan plan, const void* x, void* z, float* y);

/* x_out = A^H r (adjoint of Eq. (5)).  r: complex64 (y_off layout);
 * x_out: complex64 (x_off layout).                                            */
sr_status sr_adjoint(sr_plan plan, const void* r, void* x_out);

/* Spectral initialisation (section II-B.2, Eq. (3)-(4)).  With y~ = y/mean(y),
 * T(y~) = max(1 - 1/y~, lambda) (T = lambda where y = 0), the shifted power
 * iteration v <- B v / ||B v||, B = A^H diag(T) A / (m c) - 2 lambda I, with
 * m the number of measurements and c the mean squared entry of A (1/g for
 * SR_STRUCTURED, g = G1*G2 grid points; 1 for SR_DENSE), runs `iters` times from
 * v0/||v0||; x0_out = sqrt(sum(y)/(m c)) * v_iters.
 *  y       float, measurements (y_off layout)
 *  v0      complex64 start vectors (x_off layout), not modified
 *  lambda  threshold, lambda < 0
 *  x0_out  complex64 (x_off layout); must not alias v0                        */
sr_status sr_spectral_init(sr_plan plan, const float* y, const void* v0, int32_t iters, float lambda,
                           void* x0_out);

/* Gradient descent on the intensity loss || |Ax|^2 - y ||^2 (section II-B.1,
 * Eq. (2) read with diag(A x)): x <- x - eta * A^H((|Ax|^2 - y) . Ax) / m,
 * `iters` times, in place (or on the loss chosen with sr_plan_set_loss).
 *  y           float measurements (y_off layout)
 *  x_inout     complex64 iterates (x_off layout), updated in place
 *  eta_host    HOST array of nprob raw step sizes (no hidden normalisation)
 *  loss_trace  device float[iters * nprob] (problem-major) receiving the loss
 *              before each step, or NULL                                       */
sr_status sr_gd_solve(sr_plan plan, const float* y, void* x_inout, int32_t iters, const float* eta_host,
                      float* loss_trace);

/* sr_gd_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same GD iterations as sr_gd_solve (same kernels, same results), with the
 * two ping-pong grids in a fixed device array of the library (16 MiB per GPU,
 * reserved when the library loads and held until the process ends) instead
 * of the plan's workspace.  The call itself allocates nothing: no hipMalloc,
 * no graph instantiation (every pass is launched directly), nothing but
 * kernel launches on the plan's stream.
 *  Limits: structured plans of 2D problems only (1D problems need no scratch;
 *  use sr_gd_solve), each grid of at most 2^20 points (M1 * M2 <= 1048576,
 *  e.g. 1024 x 1024); larger grids return SR_E_ARG, 1D problems
 *  SR_E_UNSUPPORTED, dense plans SR_E_STATE.  No loss trace.
 *  The array is shared by every call on one GPU: calls that overlap on the
 *  same GPU (other streams, other threads) race; serialise them.
 *  Arguments as for sr_gd_solve.                                              */
sr_status sr_gd_solve_noalloc(sr_plan plan, const float* y, void* x_inout, int32_t iters, const float* eta_host);

/* Reverse-mode derivatives (gradients follow PyTorch's complex convention
 * dL/dRe + i dL/dIm), for differentiating through A and A^H.
 * sr_forward_vjp: given x and a cotangent gz of z = A x, writes
 *   gx_out = A^H gz and ADDS d<gz, A x>/d theta into gtheta_accum (theta layout,
 *   problems sharing a set of phases accumulate into the same entries).
 * sr_adjoint_vjp: given r and a cotangent gv of v = A^H r, writes gr_out = A gv
 *   and ADDS the phase cotangent into gtheta_accum.
 * gx_out / gr_out may be NULL.  Structured plans only.                         */
sr_status sr_forward_vjp(sr_plan plan, const void* x, const void* gz, void* gx_out, float* gtheta_accum);
sr_status sr_adjoint_vjp(sr_plan plan, const void* r, const void* gv, void* gr_out, float* gtheta_accum);

/* Reverse mode through one GD step and through the intensities, for
 * differentiating an unrolled solve with respect to the phase masks (e.g. mask
 * design: a loss on the iterate after T steps, with y = |A(theta) x*|^2).
 * sr_gd_step_vjp: the step x+ = x - (eta/m) A^H((|Ax|^2 - y) . Ax) of
 *   sr_gd_solve (section II-B.1, Eq. (2); l2 loss only).  Given x (the step's
 *   input), y, eta (HOST array, one raw step per problem) and the cotangent
 *   gx_next of x+, writes gx_out = d<gx_next, x+>/dx (must not alias gx_next)
 *   and ADDS d<gx_next, x+>/dy into gy_accum (measurement layout, nullable)
 *   and d<gx_next, x+>/dtheta into gtheta_accum.  Nothing of the forward step
 *   needs to be kept: A x and the residual are recomputed.
 * sr_intensity_vjp: y = |A x|^2 (Eq. (1)).  Given x and the cotangent gy of
 *   y, writes gx_out = d<gy, y>/dx (nullable) and ADDS d<gy, y>/dtheta into
 *   gtheta_accum.
 * Structured plans; the first call allocates 3 measurement-sized and 2
 * signal-sized complex64 temporaries for the plan's lifetime.                 */
sr_status sr_gd_step_vjp(sr_plan plan, const float* y, const void* x, const float* eta_host, const void* gx_next,
                         void* gx_out, float* gy_accum, float* gtheta_accum);
sr_status sr_intensity_vjp(sr_plan plan, const void* x, const float* gy, void* gx_out, float* gtheta_accum);

/* Static description of a status code.                                        */
const char* sr_status_string(sr_status s);

/* Thread-local description of the last failure on this thread ("" if none).  */
const char* sr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SR_H_ */
