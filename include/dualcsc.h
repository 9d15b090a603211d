/*
 * dualcsc.h -- C ABI of the dual-domain convolutional sparse coding library
 * for AMD Instinct MI355X (gfx950).
 *
 * The library solves the two convex subproblems of convolutional sparse
 * coding (CSC) in their dual form, as in Affara, Ghanem and Wonka, "Fast
 * Convolutional Sparse Coding in the Dual Domain":
 *
 *   min_{d,z} 1/2 || x - sum_k d_k * z_k ||_2^2 + beta sum_k ||z_k||_1
 *   s.t. ||d_k||_2 <= 1                                     (eq:CSC, Sec. 3.1)
 *
 * for N images x (each with J correlated channels, Sec. 3.3) sharing K
 * filters d_k of fixed support M.  Convolutions are circular on a padded
 * power-of-two grid and are diagonalised by the DFT (Sec. 3.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer to C-contiguous float32 unless
 *    stated otherwise.  Shapes use the grid (H, W) or (T, H, W):
 *        b     [N][J][grid]          images (zero-padded by the caller)
 *        d     [K][J][fsupp]         filters; tap m sits at grid index m
 *        z     [N][K][grid]          sparse codes
 *        theta [N][K][grid]          ADMM split variable theta = D^T lambda
 *  - The caller owns all memory.  The library never allocates or frees, and
 *    never calls hipMalloc: scratch space is the caller's workspace `ws`
 *    (device memory, 256-byte aligned, at least csc_workspace_bytes()).
 *  - All work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *    and is asynchronous: outputs are valid once the stream has synchronised.
 *  - Host-side argument checks run before anything is enqueued, so an error
 *    return leaves every output untouched.
 *  - Calls on distinct workspaces are independent; two calls that share a
 *    workspace must be ordered on one stream.
 *  - Supported geometry: ndim 2 or 3; every grid side a power of two, H and W
 *    in [8, 256], T in [2, 64]; 1 <= fsupp <= grid per axis; J in [1, 3];
 *    K >= 1; N >= 1.
 */
#ifndef DUALCSC_H
#define DUALCSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSC_ABI_VERSION 2

/* Return codes. */
#define CSC_OK 0
#define CSC_EINVAL (-1)       /* bad shape or argument (see each entry point) */
#define CSC_EWORKSPACE (-2)   /* workspace NULL, too small or not 256-B aligned */
#define CSC_EUNSUPPORTED (-3) /* geometry outside the supported set */
#define CSC_EHIP (-4)         /* a HIP runtime call failed */
#define CSC_ENONFINITE (-5)   /* NaN or infinity found (csc_check_finite's flag, raised by the binding) */
#define CSC_ESCRATCH (-6)     /* csc_code_noalloc: the problem needs more than the static scratch holds */

/* Workspace query operations. */
#define CSC_OP_CODE 1
#define CSC_OP_LEARN 2
#define CSC_OP_OBJECTIVE 3
#define CSC_OP_DCT 4          /* csc_code_dct and csc_objective_dct */

/* Flags. */
#define CSC_ADAPTIVE_RHO 0x1u /* csc_code: residual-balancing step size */
#define CSC_Z_ZERO 0x2u       /* csc_code: start from z = 0 (z is output only) */
#define CSC_THETA_ZERO 0x4u   /* csc_code: start from theta = 0 (theta output only) */
#define CSC_GAMMA_ZERO 0x8u   /* csc_learn: start from gamma = 0 (gamma output only) */
#define CSC_USE_GRAPH 0x10u   /* csc_code, csc_learn, csc_code_batched: capture the call
                                 once into a hipGraph, replay it on later calls with
                                 identical arguments (pointers, sizes, scalars, stream);
                                 ignored on the NULL stream.  Buffer contents may change
                                 between replays, pointers may not. */
#define CSC_NUCLEAR 0x20u     /* csc_code, csc_code_tol, csc_code_noalloc, csc_objective_reg,
                                 csc_workspace_bytes: the regulariser is beta sum_k ||z_k||_*,
                                 the nuclear norm of each code map as an H x W matrix, in place
                                 of the l1 norm (Sec. 5: low-rank maps).  The projection of
                                 eq:Inference_solution becomes the projection onto the
                                 beta-ball of the spectral norm, i.e. the z step is singular
                                 value thresholding of z - rho D^T lambda at rho beta, map by
                                 map.  2-D grids with 8 <= H, W <= 128 (CSC_EUNSUPPORTED
                                 otherwise); theta, resid, adaptive rho and the stopping rule
                                 keep their meaning. */

#define CSC_LEARN_DIRECT 0x40u /* csc_learn: apply the operator of eq:Learning_gamma to the
                                  full CG vectors in every step (two passes over the code
                                  spectra), instead of carrying the CG in the span of x, the
                                  warm start and the code-filter products, which is otherwise
                                  chosen where it is modelled to be cheaper; both give the
                                  same iterates up to rounding. */
#define CSC_LEARN_SPAN 0x80u   /* csc_learn: the span form wherever the plan allows it (2-D
                                  grids up to 256 x 256, supports up to 16 x 16), whatever
                                  the cost model says; with CSC_LEARN_DIRECT, CSC_EINVAL. */

typedef struct csc_shape {
  int32_t abi_version; /* must equal CSC_ABI_VERSION */
  int32_t n;           /* images N */
  int32_t j;           /* correlated channels J (1 = grayscale CSC) */
  int32_t k;           /* filters K */
  int32_t ndim;        /* 2: grid = (H, W); 3: grid = (T, H, W) */
  int32_t grid[3];     /* padded FFT grid, first ndim entries used */
  int32_t fsupp[3];    /* filter support, first ndim entries used */
} csc_shape;

/* Bytes of workspace needed by `op` (CSC_OP_*) for `shape` and `flags`
 * (CSC_NUCLEAR changes the coding and objective workspaces; other flags do
 * not matter); 0 if the shape is invalid or unsupported. */
size_t csc_workspace_bytes(const csc_shape* shape, int op, unsigned flags);

/*
 * Coding subproblem (eq:Inference) solved by ADMM on its dual
 * (eq:Inference_Dual, eq:Inference_ADMM) with the updates of
 * eq:Inference_solution, in the Fourier domain, for exactly `iters`
 * iterations per image (images are independent, Sec. 3.1):
 *
 *   lambda <- (D D^T + I/rho)^-1 (D theta + D z/rho - x/rho)
 *   theta  <- Pi_C(D^T lambda - z/rho),  C = { ||theta||_inf <= beta }
 *   z      <- z + rho (theta - D^T lambda)
 *
 * For J > 1 (Sec. 3.3) the lambda system is block diagonal with one J x J
 * Hermitian block per frequency and is solved exactly per frequency.
 *
 *   b      [N][J][grid]  images.
 *   d      [K][J][fsupp] filters.
 *   beta   sparsity weight (>= 0).
 *   rho    [N] ADMM step per image (> 0); read at entry, and with
 *          CSC_ADAPTIVE_RHO overwritten with the step for the next iteration
 *          (residual balancing of Boyd et al. 2011 Sec. 3.4.1: double when
 *          r_pri > 10 r_dual, halve when r_dual > 10 r_pri).
 *   iters  number of ADMM iterations (>= 0).
 *   z      [N][K][grid] in/out: warm start (ignored with CSC_Z_ZERO), result.
 *   theta  [N][K][grid] in/out, or NULL (start from 0, not returned).  With
 *          CSC_THETA_ZERO the input contents are ignored.
 *   resid  NULL or [iters][N][3] float64: r_pri = ||theta' - D^T lambda'||,
 *          r_dual = rho ||D (theta' - theta)||, and the rho used.
 *   flags  CSC_ADAPTIVE_RHO, CSC_Z_ZERO, CSC_THETA_ZERO, CSC_USE_GRAPH,
 *          CSC_NUCLEAR.
 *   Errors: CSC_EINVAL for a bad shape, beta < 0, iters < 0, NULL b/d/rho/z,
 *           unknown flags; CSC_EUNSUPPORTED (CSC_NUCLEAR on a grid it does
 *           not cover); CSC_EWORKSPACE; CSC_EHIP.
 */
int csc_code(const csc_shape* shape, const float* b, const float* d, float beta,
             float* rho, int iters, unsigned flags, float* z, float* theta,
             double* resid, void* ws, size_t ws_bytes, void* stream);

/*
 * csc_code for callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation).  Same
 * operation, arguments, flags (except CSC_USE_GRAPH) and results as csc_code,
 * bit for bit, but without a workspace argument: the scratch comes from one
 * static device array of CSC_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on every device it runs on until the process ends (its address is
 * looked up once per device, on the first call there).  The call allocates
 * nothing and frees nothing.
 *   Every call on one device shares that device's array and leaves its
 *   contents behind: two calls that overlap on one device (different
 *   streams, or different host threads without ordering) race and give
 *   wrong results.  Order them on one stream.
 *   Errors: as csc_code; CSC_ESCRATCH when csc_workspace_bytes(shape,
 *           CSC_OP_CODE, flags) exceeds CSC_NOALLOC_SCRATCH_BYTES (nothing
 *           is enqueued); CSC_EINVAL for CSC_USE_GRAPH.
 */
#define CSC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int csc_code_noalloc(const csc_shape* shape, const float* b, const float* d, float beta,
                     float* rho, int iters, unsigned flags, float* z, float* theta,
                     double* resid, void* stream);

/*
 * Coding with symmetric boundaries: the DCT-domain variant (Sec. 3 notes,
 * after Bristow et al., that the DCT can replace the DFT where the circular
 * boundary is a problem).  Images and code maps are extended half-sample
 * symmetrically at both ends of each axis, and every filter is whole-sample
 * symmetric about its centre: `q` holds one quadrant of each,
 *   h_kj[m1][m2] = q[k][j][|m1|][|m2|],  |m1| < fsupp[0], |m2| < fsupp[1],
 * a (2 fsupp[0] - 1) x (2 fsupp[1] - 1) filter.  The 2-D DCT-II then
 * diagonalises each convolution with real eigenvalues and the updates of
 * eq:Inference_solution (as csc_code: eq:Inference_Dual, eq:Inference_ADMM,
 * J x J blocks for J > 1) run with the DCT in place of the DFT:
 *   min_z 1/2 || x - sum_k h_k *_s z_k ||^2 + beta sum_k ||z_k||_1.
 *   shape  ndim 2; grid sides powers of two in [8, 128] with H W <= 16384;
 *          fsupp = quadrant size, 1 <= fsupp <= min(grid, 16) per axis.
 *   q      [K][J][fsupp] quadrants (device).
 *   Other arguments, flags (CSC_ADAPTIVE_RHO, CSC_Z_ZERO, CSC_THETA_ZERO) and
 *   resid as csc_code; workspace: csc_workspace_bytes(shape, CSC_OP_DCT, 0).
 *   Errors: CSC_EINVAL, CSC_EUNSUPPORTED (geometry), CSC_EWORKSPACE, CSC_EHIP.
 */
int csc_code_dct(const csc_shape* shape, const float* b, const float* q, float beta,
                 float* rho, int iters, unsigned flags, float* z, float* theta,
                 double* resid, void* ws, size_t ws_bytes, void* stream);

/* Objective of the symmetric-boundary problem above, per image and total
 * (out: device float64 [N + 1]); arguments as csc_code_dct, workspace
 * csc_workspace_bytes(shape, CSC_OP_DCT, 0).  Errors as csc_code_dct. */
int csc_objective_dct(const csc_shape* shape, const float* b, const float* q,
                      const float* z, float beta, double* out, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * csc_code with a stopping rule (the convergence-driven mode; the paper runs
 * its solvers to convergence rather than for a fixed count).  Iterates as
 * csc_code for at most max_iters iterations and stops after the first
 * iteration at which every image has
 *   r_pri  <= tol sqrt(K * grid size)   and   r_dual <= tol sqrt(J * grid size)
 * (r_pri, r_dual as in `resid`: the primal and dual residual norms of the
 * ADMM of eq:Inference_ADMM; i.e. both RMS residuals below tol, the
 * criterion of Boyd et al. 2011, Sec. 3.3.1, with zero relative tolerance).
 * The decision is taken on the device; the launches after it return at once.
 *   tol         > 0, finite.
 *   theta       if given, holds theta after the last iteration carried out.
 *   resid       if given, rows [0, iterations done) are written.
 *   iters_done  NULL or a device int: the number of iterations carried out
 *               (max_iters if the rule never fired).
 *   flags       CSC_ADAPTIVE_RHO, CSC_Z_ZERO, CSC_THETA_ZERO, CSC_NUCLEAR.
 *   Errors: as csc_code, and CSC_EINVAL for tol <= 0 or not finite.
 */
int csc_code_tol(const csc_shape* shape, const float* b, const float* d, float beta,
                 float* rho, int max_iters, float tol, unsigned flags, float* z,
                 float* theta, double* resid, int* iters_done, void* ws,
                 size_t ws_bytes, void* stream);

/*
 * Learning subproblem (eq:Learning) in the dual: for fixed multipliers mu,
 *   gamma = -(I + sum_k 1/(2 mu_k) Z_k S^T S Z_k^T)^-1 x      (eq:Learning_gamma)
 * by `cg_iters` conjugate-gradient iterations warm-started from gamma, then
 *   d_k = -1/(2 mu_k) S Z_k^T gamma                      (eq:Learning_Solution)
 *   mu_k <- mu_k ||d_k||_2                                   (eq:mu_update)
 * repeated `inner_iters` times; finally d_k <- d_k / max(1, ||d_k||).  The
 * images are coupled through the shared filters; for J > 1 each channel has
 * its own gamma_j with one shared operator, and mu_k and ||d_k|| span all
 * channels (Sec. 3.3).  A filter whose norm is exactly 0 keeps its mu.
 *
 *   b      [N][J][grid] images.   z [N][K][grid] codes.
 *   d      [K][J][fsupp] output filters.
 *   mu     [K] in/out multipliers (> 0 on entry).
 *   gamma  [N][J][grid] in/out dual variable (warm start unless
 *          CSC_GAMMA_ZERO).
 *   flags  CSC_GAMMA_ZERO, CSC_USE_GRAPH, CSC_LEARN_DIRECT, CSC_LEARN_SPAN.
 * On 2-D grids (up to 256 x 256, supports up to 16 x 16) the CG is carried,
 * where that is modelled to be cheaper, in the span of x, the warm start and
 * the products Z S^T w (w a filter-support vector): a CG step is then one
 * product of the filter-space vector with the lag correlations of the code
 * maps, in float64, and gamma is formed once at the end.
 *   Errors: CSC_EINVAL for a bad shape, inner_iters < 1, cg_iters < 0, NULL
 *           pointers; CSC_EWORKSPACE; CSC_EHIP.
 */
int csc_learn(const csc_shape* shape, const float* b, const float* z, float* d,
              float* mu, float* gamma, int inner_iters, int cg_iters,
              unsigned flags, void* ws, size_t ws_bytes, void* stream);

/*
 * csc_learn with a CG stopping rule: each multiplier step runs at most max_cg
 * CG iterations and stops once ||r_j|| <= cg_tol ||x_j|| for every channel j
 * (the residual of eq:Learning_gamma relative to its right-hand side; warm
 * starts make this fire after a few iterations, which the paper reports as
 * the reason the CG cost is negligible).  cg_tol = 0 runs max_cg iterations.
 *   cg_counts  NULL or a device int array [inner_iters]: the CG iterations
 *              carried out in each multiplier step.
 *   flags      CSC_GAMMA_ZERO.
 *   Errors: as csc_learn, and CSC_EINVAL for cg_tol < 0 or not finite.
 */
int csc_learn_tol(const csc_shape* shape, const float* b, const float* z, float* d,
                  float* mu, float* gamma, int inner_iters, int max_cg, float cg_tol,
                  unsigned flags, int* cg_counts, void* ws, size_t ws_bytes,
                  void* stream);

/*
 * Objective of eq:CSC for given (d, z), summed over channels:
 *   out[n] = 1/2 sum_j ||x_j^n - sum_k d_jk * z_k^n||^2 + beta ||z^n||_1,
 *   out[N] = sum_n out[n]  (fixed summation order).
 *   out: device float64 [N + 1].
 *   Errors: CSC_EINVAL, CSC_EWORKSPACE, CSC_EHIP.
 */
int csc_objective(const csc_shape* shape, const float* b, const float* d,
                  const float* z, float beta, double* out, void* ws,
                  size_t ws_bytes, void* stream);

/*
 * csc_objective with the regulariser chosen by `flags`: 0 (the l1 norm, as
 * csc_objective) or CSC_NUCLEAR (beta sum_k ||z_k||_*, the nuclear norm of
 * each map, its singular values found by the Jacobi method in float64).
 * Arguments, workspace (csc_workspace_bytes(shape, CSC_OP_OBJECTIVE, flags))
 * and errors as csc_objective, plus CSC_EINVAL for other flags and
 * CSC_EUNSUPPORTED as for csc_code.
 */
int csc_objective_reg(const csc_shape* shape, const float* b, const float* d,
                      const float* z, float beta, unsigned flags, double* out,
                      void* ws, size_t ws_bytes, void* stream);

/*
 * Differentiable coding (grayscale, J = 1; J > 1 gives CSC_EUNSUPPORTED).
 *
 * csc_code_unrolled runs `iters` iterations of eq:Inference_solution from
 * z = theta = 0 at the fixed per-image steps rho [N] (device) and writes z^T
 * (the iteration of csc_code, so z^T equals csc_code's result bit for bit).
 * If `ckpt` is non-NULL it receives the solver state at iterations 0, every,
 * 2 every, ... : ceil(iters / every) consecutive records of
 * csc_unrolled_record_floats(shape) floats each (device, caller-owned;
 * opaque apart from its first [2][N][K][grid] floats, z then theta).
 *
 * csc_code_backward is the reverse pass of that solve: given the same
 * inputs, the checkpoints and zbar = dL/dz^T [N][K][grid], it writes
 * dd = dL/dd [K][1][fsupp] and *dbeta = dL/dbeta (device float64) through
 * every iteration (the filters enter each iteration through D and
 * (D D^T + I/rho)^-1).  It replays `every` iterations at a time from their
 * record, reproducing the forward's states exactly, so the result does not
 * depend on `every`.  Kinks: the branch of the clip at each code is the
 * forward's own (gradient passes where its soft threshold returned zero,
 * i.e. |u| <= beta in its float arithmetic, and sign(u) enters dL/dbeta
 * elsewhere); the measure-zero ties |u| = beta count as passed.
 *
 * csc_loss_grad evaluates the objective of eq:CSC, loss [N + 1] (as
 * csc_objective), and its gradients: zbar = D^T (D z - x) + beta sign(z)
 * (sign(0) = 0) [N][K][grid], dd [K][1][fsupp] and *dbeta = ||z||_1.
 *
 * All three share one workspace size, csc_unrolled_workspace_bytes(shape,
 * every) (use every = 1 for csc_loss_grad).
 * Errors: CSC_EINVAL (NULL pointers, iters < 0, every < 1, beta < 0),
 *         CSC_EUNSUPPORTED, CSC_EWORKSPACE, CSC_EHIP.
 */
size_t csc_unrolled_workspace_bytes(const csc_shape* shape, int every);

/* Floats in one checkpoint record of csc_code_unrolled for `shape`
 * (N (2K + 6) grid); 0 for an invalid or J > 1 shape. */
int64_t csc_unrolled_record_floats(const csc_shape* shape);

int csc_code_unrolled(const csc_shape* shape, const float* b, const float* d,
                      float beta, const float* rho, int iters, int every,
                      float* z, float* ckpt, void* ws, size_t ws_bytes,
                      void* stream);

int csc_code_backward(const csc_shape* shape, const float* b, const float* d,
                      float beta, const float* rho, int iters, int every,
                      const float* ckpt, const float* zbar, float* dd,
                      double* dbeta, void* ws, size_t ws_bytes, void* stream);

int csc_loss_grad(const csc_shape* shape, const float* b, const float* d,
                  const float* z, float beta, double* loss, float* zbar,
                  float* dd, double* dbeta, void* ws, size_t ws_bytes,
                  void* stream);

/*
 * Batched coding: many grayscale images of uneven sizes share K filters
 * (the coding problem separates over images, Sec. 3.1, so each image is
 * coded exactly as by csc_code with J = 1 and a fixed rho).
 *
 *   batch->grid   host [n][2] padded grid (H, W) of each image (powers of two,
 *                 as for csc_code); images are grouped by grid internally.
 *   batch->b_off  host [n] element offset of image i's H x W block in `b`.
 *   batch->z_off  host [n] element offset of image i's K x H x W codes in `z`.
 *   batch->ppg    NULL, or host [classes] filter pairs per workgroup for each
 *                 grid class (classes in increasing (H, W) order, see
 *                 csc_batch_classes); 0 entries keep the built-in choice.
 *   b, d, z       device buffers; d [K][1][fsupp]; z in/out (warm start
 *                 unless CSC_Z_ZERO).
 *   flags         CSC_Z_ZERO, CSC_USE_GRAPH.  With CSC_USE_GRAPH (and a
 *                 non-NULL stream) the first call for a given set of
 *                 arguments captures the whole call into a hipGraph; later
 *                 calls with identical arguments (pointers, sizes, beta, rho,
 *                 iters) replay it.  Buffer contents may change between
 *                 replays; pointers may not.
 *   Errors: CSC_EINVAL (bad table, grid, K, beta < 0, rho <= 0, iters < 0,
 *           flags), CSC_EUNSUPPORTED, CSC_EWORKSPACE, CSC_EHIP.
 */
typedef struct csc_batch {
  int32_t abi_version; /* CSC_ABI_VERSION */
  int32_t n;           /* images */
  int32_t k;           /* filters */
  int32_t fsupp[2];    /* filter support (2-D) */
  const int32_t* grid;
  const int64_t* b_off;
  const int64_t* z_off;
  const int32_t* ppg;
} csc_batch;

size_t csc_batch_workspace_bytes(const csc_batch* batch);

/* Grid classes of a batch in processing order: grids [classes][2] and image
 * counts [classes] (either may be NULL; at most max_classes written).
 * Returns the number of classes, or a negative error code. */
int csc_batch_classes(const csc_batch* batch, int32_t* grids, int32_t* counts,
                      int max_classes);

int csc_code_batched(const csc_batch* batch, const float* b, const float* d,
                     float beta, float rho, int iters, unsigned flags, float* z,
                     void* ws, size_t ws_bytes, void* stream);

/* Measured choice of filter pairs per workgroup for each single-tile grid
 * class: runs `iters` coding iterations of each class per candidate (z is
 * overwritten) and writes the fastest into ppg_out [classes] (host).
 * Synchronises the stream.  Errors as csc_code_batched. */
int csc_batch_autotune(const csc_batch* batch, const float* b, const float* d,
                       float beta, float rho, int iters, float* z, void* ws,
                       size_t ws_bytes, void* stream, int32_t* ppg_out,
                       int max_classes);

/*
 * Launch tracing (for benchmarks and profiling).  csc_trace_enable(n), n >= 1,
 * clears the record and starts bracketing every n-th launch of each traced
 * kernel class (the 1st, (n+1)-th, ...) with HIP events on the stream it is
 * launched on (at most 8192 records; later launches are not recorded).  Each
 * bracket costs a few microseconds of stream time, so benchmarks sample with
 * n > 1.  csc_trace_enable(0) stops recording; n < 0 is CSC_EINVAL.
 * csc_trace_read waits for the recorded events and returns the summed
 * duration in milliseconds and the number of records of class `cls`:
 *   0 = coding map kernel (back-projection, inverse FFT, soft threshold,
 *       forward FFT: one launch per ADMM iteration on single-tile grids),
 *   1 = coding per-frequency kernels (spectral reduce and dual solve),
 *   2 = learning pass A kernel (sum over images of conj(zhat) times the CG
 *       vector, eq:Learning_gamma; one record per launch),
 *   3 = learning pass B kernel (sum over filters of zhat times the projected
 *       filter spectra; one record per launch),
 *   4 = learning span form, row stage of the code-map correlation table
 *       (one launch per learning call),
 *   5 = learning span form, product of a filter-space vector with the
 *       correlation table (one launch per CG step and per multiplier step).
 * Calls captured into a hipGraph (CSC_USE_GRAPH) record nothing.
 * Errors: CSC_EINVAL (bad class or NULL outputs), CSC_EHIP.
 */
int csc_trace_enable(int on);
int csc_trace_read(int cls, double* total_ms, int* count);

/*
 * Non-finite detection.  The library never synchronises with the device,
 * so a NaN or infinity in a result (diverging iterations, bad inputs) is
 * found by a check the caller enqueues and reads: csc_check_finite writes
 * *flag = 1 if any of x[0 .. n) is NaN or +-infinity, else 0, on `stream`
 * after the work already enqueued there.  x, flag: device pointers
 * (caller-owned; x may be NULL when n = 0); n >= 0 (n = 0 writes 0).  A
 * caller that finds the flag set reports CSC_ENONFINITE (the Python binding
 * raises it).
 * Errors: CSC_EINVAL (NULL flag, NULL x with n > 0, n < 0), CSC_EHIP.
 */
int csc_check_finite(const float* x, int64_t n, int* flag, void* stream);

/* Static description of a return code. */
const char* csc_strerror(int code);

/* CSC_ABI_VERSION of the loaded library. */
int csc_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DUALCSC_H */
