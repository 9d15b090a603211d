// Host-side plan and launch helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/dualcsc.h"

namespace dcsc {

// Geometry of one call.  Grids are stored as (T, H, W) with T = 1 for 2-D.
// Filters are handled in pairs p = (2p, 2p+1): two real maps travel as the
// real and imaginary parts of one complex grid.
struct Plan {
  int n = 0, j = 0, k = 0, p = 0;  // images, channels, filters, filter pairs
  int nd = 2;
  int g[3] = {1, 1, 1};            // T, H, W
  int fs[3] = {1, 1, 1};           // filter support, same axis order
  int64_t dsz = 0;                 // pixels per grid
  int64_t msz = 0;                 // taps per filter channel
  bool lds = false;                // whole grid fits one LDS tile (fused path)
  bool split = false;              // 2-D grid beyond one tile: row / column / row phases
  bool nuclear = false;            // nuclear-norm regulariser (maps through the global path)
  bool vol = false;                // 3-D grid, T <= 16 frames of a single-tile plane (volume.hip)
  int ng = 1;                      // pair groups per image in the fused kernel
  int ppg = 1;                     // pairs per group
  // Optional device tables (batched form): element offset of image n's
  // block in b ([J][grid]) and in z / theta ([K][grid]).  NULL = dense.
  const int64_t* boff = nullptr;
  const int64_t* zoff = nullptr;
};

// Pairs per group for a tile-path plan (fills the chip with one or a few
// workgroups per CU); ppg_override > 0 replaces the heuristic.
void set_grouping(Plan* pl, int ppg_override);

// Largest grid (complex elements) that one LDS tile holds.
constexpr int kTileMax = 16384;

int make_plan(const csc_shape* s, Plan* pl);
// make_plan, then the plan changes that `flags` ask for (CSC_NUCLEAR).
int make_plan_flags(const csc_shape* s, unsigned flags, Plan* pl);

// Nuclear-norm regulariser (nuclear.hip): 2-D grids with 8 <= H, W <= 128.
bool nuclear_supported(int T, int H, int W);
// mode 0: the ADMM z step by singular value thresholding of every map
// (buf holds D * (D^T lam) pairs and receives the new pairs; rmap [N][K]
// gets sum (z' - z)^2 per map); mode 1: rmap [N][K] = nuclear norms of z.
hipError_t launch_svt(const Plan& pl, float2* buf, float* z, const float* zin, float* theta, const float* rho,
                      float beta, double* rmap, int mode, hipStream_t st, const int* stop);

// Large 2-D grids (128 x 256, 256 x 128, 256 x 256): the coding map work in
// three phases (split.hip).  Column / row workgroups per grid:
bool split_supported(int T, int H, int W);
int split_col_blocks(const Plan& pl);
int split_row_blocks(const Plan& pl);
// mode 0: one ADMM map iteration (z, theta as in the fused kernel, residual
// partials to rpart [N][P * col_blocks]); mode 1: forward transform of the
// maps z and reduction into part (l1 partials to rpart).
// With `stop` (tolerance mode) the kernels return at once when stop[0] is set.
hipError_t split_maps(const Plan& pl, const float2* E, const float2* lam, float2* buf, float* z, float* theta,
                      const float* rho, float beta, float2* part, double* rpart, int mode, hipStream_t st,
                      const int* stop, const float* zin = nullptr);

// 3-D grids with 2 <= T <= 16 frames of a plane that fits one LDS tile: the
// coding map work in three launches per iteration (volume.hip).  Residual
// partials go to rpart [N][P * nblk(D)] (one slot per 256 grid points of a
// pair, as on the axis-pass path; the unused slots hold zeros).
bool vol_supported(int T, int H, int W);
hipError_t vol_maps(const Plan& pl, const float2* E, const float2* lam, float2* buf, float* z, float* theta,
                    const float* rho, float beta, double* rpart, hipStream_t st, const int* stop);

// Workspace carving: aligned sub-buffers of one caller-provided block.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// In-place unnormalised DFT (dir = -1 forward, +1 inverse) of `count`
// complex grids of shape g (T, H, W), contiguous one after the other.
hipError_t fft_grids(float2* data, int64_t count, const int g[3], int dir, hipStream_t st);

// Whether the fused single-tile kernels exist for this (H, W).
bool tile_supported(int h, int w);

// Learning in the span form (learnspan.hip): the CG vectors of a learning
// call carried as coordinates on {x, gamma_0} plus a filter-space vector,
// the operator applied through the lag correlations of the code maps.
// Eligible plans: 2-D grids up to 256 x 256, supports up to 16 x 16.
bool span_eligible(const Plan& pl);
// Whether the span form's modelled cost is below the direct form's.
bool span_preferred(const Plan& pl, int inner_iters, int cg_iters);
size_t span_ws_bytes(const Plan& pl);
// From the code, image and warm-start spectra (Zh pair-packed, xh, gh full
// grids): inner_iters multiplier steps of cg_iters CG steps each; writes d,
// mu, and for the final gamma the spectrum a xhat + b gammahat_0 to vout and
// the pair-unpacked canonical spectra of its filter-space part to Uc (pass B
// of Uc onto vout then gives gammahat).
hipError_t run_span(const Plan& pl, const float2* Zh, const float2* xh, const float2* gh, float2* vout, float4* Uc,
                    float* d, float* mu, int inner_iters, int cg_iters, void* span_ws, hipStream_t st);

// Workspace of the coding / objective paths (carved from the caller's block).
struct CodeWs {
  float2 *E, *G, *xh, *yh, *Th, *lam, *part, *buf;
  double *rpri, *rdual, *opart;
  double* rres;  // per-image r_pri, r_dual of the last iteration (tolerance mode)
  double* rmap;  // nuclear-norm plans: per-map partials [N][K]
  int* stop;     // tolerance mode: [0] converged flag, [1] iterations carried out
  float* rho;
  float* rho2;   // adaptive rho: the other buffer (k_solve_rho reads one, writes the other)
  int npri, ndual, ngp;  // partial counts per image; pair groups written to part
};
size_t carve_code(const Plan& pl, void* base, CodeWs* w);
// Filter pair spectra E, Gram blocks G and image spectra xhat.
hipError_t setup_spectra(const Plan& pl, const float* b, const float* d, CodeWs& w, hipStream_t st);
// Everything run_code does before its iteration loop: set-up spectra, rho,
// z zeroed (CSC_Z_ZERO) or its spectra, theta's spectra (zero when theta is
// null or CSC_THETA_ZERO), and with `solve` the first lam.
hipError_t code_prepare(const Plan& pl, const float* b, const float* d, const float* rho, unsigned flags, float* z,
                        const float* theta, bool solve, CodeWs& w, hipStream_t st);
// ADMM coding of eq:Inference_solution (csc_code / csc_code_tol).  tol > 0
// selects the stopping rule; iters_done receives the count.  With `ckpt`
// (dense maps, fixed steps and count only) the state after 0, every,
// 2 every, ... (< iters) iterations is written to consecutive records of
// code_record_floats(pl) floats: z [N][K][grid], theta [N][K][grid], then
// yhat, Thhat and lam ([N][J][grid] complex each) as the next iteration
// reads them.
int run_code(const Plan& pl, const float* b, const float* d, float beta, float* rho, int iters, unsigned flags,
             float* z, float* theta, double* resid, void* ws, hipStream_t st, float tol = 0.0f,
             int* iters_done = nullptr, float* ckpt = nullptr, int every = 0);
int64_t code_record_floats(const Plan& pl);
// Resumes run_code's fixed-step loop from a record: seg[i - 1]
// ([2][N][K][grid], z then theta) receives the state after i more
// iterations, 0 < i < nstates, equal bit for bit to the states the
// uninterrupted loop passes through (the state after 0 iterations is the
// record's own first [2][N][K][grid] floats).  E, G and xh of `w` must hold
// the spectra of the same images and filters.
hipError_t replay_code(const Plan& pl, CodeWs& w, const float* rho, float beta, const float* rec, int nstates, float* seg,
                       hipStream_t st);
// part <- per-group spectral contributions sum_p DFT(maps pair) conj(E_p);
// l1 <- partial sums of |maps| ([N][npri]).
hipError_t forward_maps(const Plan& pl, const float* maps, CodeWs& w, double* l1, hipStream_t st);
// buf[n][p] = sum_j lam[n][j] E[j][p]
void launch_make_v(const Plan& pl, const float2* E, const float2* lam, float2* buf, hipStream_t st);
// dst[n][j](f) = (Y(f) + conj(Y(-f)))/2, Y = sum of the ng groups of part
void launch_sym_reduce(const Plan& pl, const float2* part, int ng, float2* dst, hipStream_t st);
// objective from part (after forward_maps) and l1 partials in w.rpri
void launch_objective_tail(const Plan& pl, CodeWs& w, float beta, double* out, hipStream_t st);

// Residual norms and the residual-balancing step per image (k_rho), and
// the objective's final sums (k_obj_final, k_obj_total), for other paths.
void launch_rho(const double* rpri, int npri, const double* rdual, int ndual, float* rho, double* resid, int it,
                int N, int64_t D, int adaptive, hipStream_t st);
void launch_obj_final(const double* opart, int nopart, const double* l1, int nl1, double* out, int N, int64_t D,
                      float beta, hipStream_t st);

// DCT-domain variant (dct.hip): 2-D grids with 8 <= H, W <= 128 and
// H W <= 16384.
bool dct_supported(int T, int H, int W);
size_t dct_ws_bytes(const Plan& pl);
int run_code_dct(const Plan& pl, const float* b, const float* q, float beta, float* rho, int iters, unsigned flags,
                 float* z, float* theta, double* resid, void* ws, hipStream_t st);
int run_objective_dct(const Plan& pl, const float* b, const float* q, const float* z, float beta, double* out,
                      void* ws, hipStream_t st);

// hipGraph capture/replay keyed by every argument of a call.  `enqueue`
// enqueues the call on `st`; the first call with a key captures it, later
// calls replay the executable graph.  Returns a CSC_* code.
int graph_call(const std::vector<int64_t>& key, hipStream_t st, int (*enqueue)(void*), void* ctx);

// *flag = 1 if any of x[0 .. n) is NaN or +-infinity, else 0 (enqueued).
hipError_t launch_check_finite(const float* x, int64_t n, int* flag, hipStream_t st);

// Launch tracing.  While enabled (csc_trace_enable), a sampled TraceScope
// times the launches made in its lifetime with a pair of HIP events on the
// launching stream; csc_trace_read sums the elapsed times per class.  A
// scope that covers several kernels records the events around them.  A
// scope made with own_launch covers exactly one kernel, which the caller
// launches with hipExtLaunchKernelGGL and the scope's events (events()):
// the runtime then stamps them at that kernel's own start and end, so the
// time excludes the dispatch around it.
enum TraceClass {
  kTraceCodeMaps = 0,
  kTraceCodeSpec = 1,
  kTraceLearnA = 2,
  kTraceLearnB = 3,
  kTraceLearnSpanRows = 4,
  kTraceLearnSpanApply = 5,
  kTraceClasses = 6
};
struct TraceScope {
  TraceScope(int cls, hipStream_t st, bool own_launch = false);
  ~TraceScope();
  // own-launch scopes: the events to launch the kernel with; false when the
  // scope is not sampled (launch it normally)
  bool events(hipEvent_t* start, hipEvent_t* stop) const;
  int cls_;
  hipStream_t st_;
  int slot_;
  bool own_;
};

// Launch KERNEL<J> (J = 1, 2, 3) under an own-launch TraceScope `tr`.
#define LAUNCH_J_TRACED(tr, KERNEL, J, grid, block, st, ...)                                          \
  do {                                                                                                \
    hipEvent_t e0_, e1_;                                                                              \
    if ((tr).events(&e0_, &e1_)) {                                                                    \
      if ((J) == 1) hipExtLaunchKernelGGL(KERNEL<1>, grid, block, 0, st, e0_, e1_, 0, __VA_ARGS__);      \
      else if ((J) == 2) hipExtLaunchKernelGGL(KERNEL<2>, grid, block, 0, st, e0_, e1_, 0, __VA_ARGS__); \
      else hipExtLaunchKernelGGL(KERNEL<3>, grid, block, 0, st, e0_, e1_, 0, __VA_ARGS__);             \
    } else {                                                                                          \
      if ((J) == 1) hipLaunchKernelGGL(KERNEL<1>, grid, block, 0, st, __VA_ARGS__);                      \
      else if ((J) == 2) hipLaunchKernelGGL(KERNEL<2>, grid, block, 0, st, __VA_ARGS__);                 \
      else hipLaunchKernelGGL(KERNEL<3>, grid, block, 0, st, __VA_ARGS__);                               \
    }                                                                                                 \
  } while (0)

}  // namespace dcsc
