// Coding subproblem: ADMM on the dual of the lasso (eq:Inference_Dual,
// eq:Inference_ADMM) with the updates of eq:Inference_solution, evaluated in
// the Fourier domain (Sec. 3.2), plus the objective of eq:CSC.
//
// Restructuring used on the GPU (identical iterates in exact arithmetic):
// theta is never stored.  From the z update, theta' = D^T lam' + (z' - z)/rho,
// so DFT(D theta') = G lam' + (DFT(D z') - DFT(D z))/rho.  Per image the
// library keeps yhat = DFT(D z) and Thhat = DFT(D theta) (J channels each),
// and one iteration is
//   lam'   = (G + I/rho)^-1 (Thhat + (yhat - xhat)/rho)          [k_solve]
//   z'     = soft(z - rho D^T lam', rho beta)                     [k_fused]
//   yhat'  = DFT(D z')                                            [k_fused + k_spec]
//   Thhat' = G lam' + (yhat' - yhat)/rho                          [k_spec]
// The soft threshold is the Moreau form of the theta/z pair of
// eq:Inference_solution.  Only z streams through HBM each iteration.
//
// Filter pairs.  Filters (2p, 2p+1) travel together: with
// E_jp(f) = conj(dhat_j,2p(f)) + i conj(dhat_j,2p+1(f)), which equals the
// unnormalised inverse DFT of S^T d_2p + i S^T d_2p+1, one complex inverse FFT
// of sum_j lamhat_j E_jp yields D^T lam for both maps (real and imaginary
// part), and one complex forward FFT C of (z_2p + i z_2p+1) gives their
// contribution to yhat as (Y(f) + conj(Y(-f)))/2 with Y = C conj(E).
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"
#include "tiles.hpp"

namespace dcsc {

constexpr int kEW = 256;  // threads of the elementwise kernels



// ------------------------------------------------------------------ set-up

// Pair grids of the filters: E[j][p] = S^T d_{2p,j} + i S^T d_{2p+1,j}.
__global__ void k_pack_filters(const float* __restrict__ d, float2* __restrict__ E, int K, int J, int P,
                               int T, int H, int W, int ft, int fh, int fw) {
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= D) return;
  const int p = blockIdx.y, j = blockIdx.z;
  const int t = (int)(f / (int64_t(H) * W)), h = (int)((f / W) % H), w = (int)(f % W);
  float2 v = make_float2(0.f, 0.f);
  if (t < ft && h < fh && w < fw) {
    const int64_t m = (int64_t(t) * fh + h) * fw + w, msz = int64_t(ft) * fh * fw;
    v.x = d[(int64_t(2 * p) * J + j) * msz + m];
    if (2 * p + 1 < K) v.y = d[(int64_t(2 * p + 1) * J + j) * msz + m];
  }
  E[(int64_t(j) * P + p) * D + f] = v;
}

// Images -> complex planes with zero imaginary part: dst[n][j] = b of image n
// (dense [N][J][grid], or at boff[n] when a table is given).
__global__ void k_pack_images(const float* __restrict__ b, const int64_t* __restrict__ boff,
                              float2* __restrict__ dst, int J, int64_t D) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int j = blockIdx.y, n = blockIdx.z;
  if (f >= D) return;
  const int64_t base = boff ? boff[n] : int64_t(n) * J * D;
  dst[(int64_t(n) * J + j) * D + f] = make_float2(b[base + int64_t(j) * D + f], 0.f);
}

// Zero the code maps of every image (dense or through the offset table).
__global__ void k_zero_maps(float* __restrict__ z, const int64_t* __restrict__ zoff, int K, int64_t D) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (i < int64_t(K) * D) z[map_base(zoff, n, K, D) + i] = 0.f;
}

// Map pairs -> complex planes; l1 partial sums of |maps| per (image, block).
__global__ void k_pack_maps(const float* __restrict__ z, const int64_t* __restrict__ zoff, float2* __restrict__ buf,
                            double* __restrict__ l1, int K, int P, int64_t D) {
  __shared__ double red[kEW / 64];
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, n = blockIdx.z;
  double s = 0.0;
  if (f < D) {
    const float* zn = z + map_base(zoff, n, K, D);
    const float a = zn[int64_t(2 * p) * D + f];
    const float b = (2 * p + 1 < K) ? zn[int64_t(2 * p + 1) * D + f] : 0.f;
    buf[(int64_t(n) * P + p) * D + f] = make_float2(a, b);
    s = (double)fabsf(a) + (double)fabsf(b);
  }
  const double t = block_sum(s, red);
  if (l1 && threadIdx.x == 0) l1[(int64_t(n) * P + p) * gridDim.x + blockIdx.x] = t;
}

// G_f = sum_k dhat_.k(f) dhat_.k(f)^H, J x J per frequency (Sec. 3.2, 3.3),
// from the pair spectra: dhat_j,2p(f) = (conj(E(f)) + E(-f))/2 and
// dhat_j,2p+1(f) = i (conj(E(f)) - E(-f))/2.  Stored [D][J][J].
template <int J>
__global__ void k_gram(const float2* __restrict__ E, float2* __restrict__ G, int P, int T, int H, int W) {
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= D) return;
  const int64_t fn = neg_index(f, T, H, W);
  double gr[J][J], gi[J][J];
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int c = 0; c < J; ++c) gr[a][c] = gi[a][c] = 0.0;
  // a batch of pairs' loads in flight at a time (8 / 4 / 3 pairs for J = 1 /
  // 2 / 3), unconditionally (a pair past P loads pair P - 1 again with
  // weight 0; the sums keep their order)
  constexpr int kB = J == 1 ? 8 : (J == 2 ? 4 : 3);
  for (int p0 = 0; p0 < P; p0 += kB) {
    float2 le[kB][J], lm[kB][J];
#pragma unroll
    for (int u = 0; u < kB; ++u)
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int64_t o = (int64_t(j) * P + min(p0 + u, P - 1)) * D;
        le[u][j] = E[o + f];
        lm[u][j] = E[o + fn];
      }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const double w = p0 + u < P ? 0.5 : 0.0;
      double ar[J], ai[J], br[J], bi[J];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const float2 e = le[u][j], m = lm[u][j];
        ar[j] = w * ((double)e.x + m.x);
        ai[j] = w * (-(double)e.y + m.y);
        // i (conj(e) - m) / 2 = i ((e.x - m.x) + i(-e.y - m.y)) / 2
        br[j] = w * ((double)e.y + m.y);
        bi[j] = w * ((double)e.x - m.x);
      }
#pragma unroll
      for (int a = 0; a < J; ++a)
#pragma unroll
        for (int c = 0; c < J; ++c) {
          // x conj(y) for x = a-row, y = c-row
          gr[a][c] += ar[a] * ar[c] + ai[a] * ai[c] + br[a] * br[c] + bi[a] * bi[c];
          gi[a][c] += ai[a] * ar[c] - ar[a] * ai[c] + bi[a] * br[c] - br[a] * bi[c];
        }
    }
  }
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int c = 0; c < J; ++c) G[(f * J + a) * J + c] = make_float2((float)gr[a][c], (float)gi[a][c]);
}

__global__ void k_fill_f2(float2* __restrict__ dst, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) dst[i] = make_float2(0.f, 0.f);
}
__global__ void k_copy_f(float* __restrict__ dst, const float* __restrict__ src, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

// dst[n][j](f) = (Y(f) + conj(Y(-f)))/2 with Y = sum_g part[n][g][j].  The
// thread of the lower index of each pair (f, -f) writes both values (the
// second is the conjugate of the first), so part is read once.
template <int J>
__global__ void k_sym_reduce(const float2* __restrict__ part, float2* __restrict__ dst, int ng, int T, int H,
                             int W) {
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (f >= D) return;
  const int64_t fn = neg_index(f, T, H, W);
  if (fn < f) return;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    float2 y, ym;
    group_sums<8>(part + (int64_t(n) * ng * J + j) * D, int64_t(J) * D, ng, f, fn, y, ym);
    const float2 s = make_float2(0.5f * (y.x + ym.x), 0.5f * (y.y - ym.y));
    dst[(int64_t(n) * J + j) * D + f] = s;
    dst[(int64_t(n) * J + j) * D + fn] = cconj(s);
  }
}

// --------------------------------------------- per-frequency dual solve

template <int J>
__global__ void k_solve(const float2* __restrict__ G, const float2* __restrict__ xh, const float2* __restrict__ yh,
                        const float2* __restrict__ Th, const float* __restrict__ rho_cur, float2* __restrict__ lam,
                        int64_t D, const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (f >= D) return;
  const float inv_rho = 1.0f / rho_cur[n];
  float2 r[J], l[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t o = (int64_t(n) * J + j) * D + f;
    const float2 y = yh[o], x = xh[o], th = Th[o];
    r[j] = make_float2(th.x + (y.x - x.x) * inv_rho, th.y + (y.y - x.y) * inv_rho);
  }
  dual_solve<J>(G + f * J * J, inv_rho, r, l);
#pragma unroll
  for (int j = 0; j < J; ++j) lam[(int64_t(n) * J + j) * D + f] = l[j];
}

#define SPEC_KERNEL(NAME, U)                                                                                   \
  template <int J>                                                                                             \
  __global__ __launch_bounds__(kSpecT) void NAME(                                                              \
      const float2* __restrict__ part, const float2* __restrict__ G, const float2* __restrict__ xh,           \
      float2* __restrict__ yh, float2* __restrict__ Th, float2* __restrict__ lam,                              \
      const float* __restrict__ rho_cur, double* __restrict__ rdual, int ng, int T, int H, int W,             \
      int solve_next, const int* __restrict__ stop) {                                                          \
    if (stop && stop[0]) return;                                                                               \
    __shared__ double red[kSpecT / 64];                                                                        \
    spec_item<J, U>(red, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, part, G, xh, yh, Th, lam, rho_cur,  \
                    rdual, ng, T, H, W, solve_next);                                                           \
  }
// k_spec sums the group partials with 8 accumulators; k_spec_wide, for
// single-tile plans with many groups, with 16 (more loads in flight, more
// registers)
SPEC_KERNEL(k_spec, 8)
SPEC_KERNEL(k_spec_wide, 16)
#undef SPEC_KERNEL

// Residual norms per image (Boyd et al. 2011, Sec. 3.3) and the residual
// balancing rule (Sec. 3.4.1): r_pri = ||z' - z|| / rho, r_dual = rho
// sqrt(sum |dThhat|^2 / D).  Partial sums are added in a fixed order.
__global__ __launch_bounds__(64) void k_rho(const double* __restrict__ rpri, int npri,
                                            const double* __restrict__ rdual, int ndual, float* __restrict__ rho_cur,
                                            double* __restrict__ resid, int it, int N, int64_t D, int adaptive,
                                            const int* __restrict__ stop, double* __restrict__ rres) {
  if (stop && stop[0]) return;
  const int n = blockIdx.x, lane = threadIdx.x;
  double sp = 0.0, sd = 0.0;
  for (int i = lane; i < npri; i += 64) sp += rpri[int64_t(n) * npri + i];
  for (int i = lane; i < ndual; i += 64) sd += rdual[int64_t(n) * ndual + i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sp += __shfl_down(sp, off, 64);
    sd += __shfl_down(sd, off, 64);
  }
  if (lane != 0) return;
  const float rho = rho_cur[n];
  const double r_pri = sqrt(sp) / (double)rho;
  const double r_dual = (double)rho * sqrt(sd / (double)D);
  if (resid) {
    double* o = resid + (int64_t(it) * N + n) * 3;
    o[0] = r_pri;
    o[1] = r_dual;
    o[2] = (double)rho;
  }
  if (rres) {
    rres[2 * n] = r_pri;
    rres[2 * n + 1] = r_dual;
  }
  if (adaptive) {
    float nr = rho;
    if (r_pri > 10.0 * r_dual) nr = rho * 2.0f;
    else if (r_dual > 10.0 * r_pri) nr = rho * 0.5f;
    rho_cur[n] = nr;
  }
}

// k_rho and k_solve in one launch (adaptive rho between two iterations):
// every wavefront of a block reduces image n's residual partials in k_rho's
// order, takes the residual-balancing step from rho_cur, and solves for
// lam with the new rho; block (0, n) records the residuals and writes the
// new rho to rho_next (a separate buffer, since the other blocks still read
// rho_cur).  Results equal k_rho followed by k_solve bit for bit.
template <int J>
__global__ __launch_bounds__(kEW) void k_solve_rho(const float2* __restrict__ G, const float2* __restrict__ xh,
                                                    const float2* __restrict__ yh, const float2* __restrict__ Th,
                                                    const double* __restrict__ rpri, int npri,
                                                    const double* __restrict__ rdual, int ndual,
                                                    const float* __restrict__ rho_cur, float* __restrict__ rho_next,
                                                    double* __restrict__ resid, int it, int N, float2* __restrict__ lam,
                                                    int64_t D) {
  const int n = blockIdx.y, lane = threadIdx.x & 63;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // the spectra do not depend on rho: their loads go out first
  float2 y[J], x[J], th[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t o = (int64_t(n) * J + j) * D + (f < D ? f : 0);
    y[j] = yh[o];
    x[j] = xh[o];
    th[j] = Th[o];
  }
  double sp = 0.0, sd = 0.0;
  for (int i = lane; i < npri; i += 64) sp += rpri[int64_t(n) * npri + i];
  for (int i = lane; i < ndual; i += 64) sd += rdual[int64_t(n) * ndual + i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sp += __shfl_down(sp, off, 64);
    sd += __shfl_down(sd, off, 64);
  }
  sp = __shfl(sp, 0, 64);
  sd = __shfl(sd, 0, 64);
  const float rho = rho_cur[n];
  const double r_pri = sqrt(sp) / (double)rho;
  const double r_dual = (double)rho * sqrt(sd / (double)D);
  float nr = rho;
  if (r_pri > 10.0 * r_dual) nr = rho * 2.0f;
  else if (r_dual > 10.0 * r_pri) nr = rho * 0.5f;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    rho_next[n] = nr;
    if (resid) {
      double* o = resid + (int64_t(it) * N + n) * 3;
      o[0] = r_pri;
      o[1] = r_dual;
      o[2] = (double)rho;
    }
  }
  if (f >= D) return;
  const float inv_rho = 1.0f / nr;
  float2 r[J], l[J];
#pragma unroll
  for (int j = 0; j < J; ++j)
    r[j] = make_float2(th[j].x + (y[j].x - x[j].x) * inv_rho, th[j].y + (y[j].y - x[j].y) * inv_rho);
  dual_solve<J>(G + f * J * J, inv_rho, r, l);
#pragma unroll
  for (int j = 0; j < J; ++j) lam[(int64_t(n) * J + j) * D + f] = l[j];
}

// Stopping rule of the tolerance mode (Boyd et al. 2011, Sec. 3.3.1 with a
// zero relative tolerance): every image has r_pri <= thr_pri and r_dual <=
// thr_dual (the RMS residuals times sqrt of the entry counts).  stop[0] is
// the flag every later kernel of the call checks; stop[1] counts the
// iterations carried out.
__global__ void k_stop(const double* __restrict__ rres, int N, double thr_pri, double thr_dual,
                       int* __restrict__ stop) {
  if (blockIdx.x != 0 || threadIdx.x != 0 || stop[0]) return;
  stop[1] += 1;
  bool done = true;
  for (int n = 0; n < N; ++n) done = done && rres[2 * n] <= thr_pri && rres[2 * n + 1] <= thr_dual;
  if (done) stop[0] = 1;
}

__global__ void k_stop_init(int* __restrict__ stop) {
  if (blockIdx.x == 0 && threadIdx.x == 0) stop[0] = stop[1] = 0;
}

__global__ void k_stop_out(const int* __restrict__ stop, int* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = stop[1];
}

__global__ void k_fill_i(int* __restrict__ out, int v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = v;
}

// ------------------------------------------------------- fused tile kernel

// The kernel: one workgroup per (pair group g, image n), handed out by
// xcd_item so that the workgroups of one XCD share pair groups (and their
// filter spectra in that XCD's L2) across the images.
template <int H, int W, int J, int MODE>
__global__ __launch_bounds__(fused_threads(H * W, J)) void k_fused(
    const float2* __restrict__ E, const float2* __restrict__ lam, float* __restrict__ z,
    float* __restrict__ theta, const int64_t* __restrict__ zoff, const float* __restrict__ rho_cur, float beta,
    float2* __restrict__ part, double* __restrict__ rpart, int K, int P, int ppg, int ng,
    const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int D = H * W, NT = fused_threads(D, J), WP = tile_stride(W);
  __shared__ float2 tile[H * WP];
  __shared__ float2 tw[256];
  __shared__ double red[NT / 64];
  const int N = (int)(gridDim.x / ng), item = xcd_item((int)blockIdx.x, (int)gridDim.x);
  const int g = item / N, n = item % N;
  load_twiddles(tw);
#include "fused_body.inc"
}

// ------------------------------------------------ global path (large grids)

// buf[n][p](f) = sum_j lam_j(f) E_jp(f)
template <int J>
__global__ void k_make_v(const float2* __restrict__ E, const float2* __restrict__ lam, float2* __restrict__ buf,
                         int P, int64_t D, const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, n = blockIdx.z;
  if (f >= D) return;
  float2 v = make_float2(0.f, 0.f);
#pragma unroll
  for (int j = 0; j < J; ++j) v = cadd(v, cmul(lam[(int64_t(n) * J + j) * D + f], E[(int64_t(j) * P + p) * D + f]));
  buf[(int64_t(n) * P + p) * D + f] = v;
}

// Soft-threshold step on buf (holding D * (D^T lam) for the pair); writes the
// new pair back into buf for the forward FFT.  rpart [N][P * gridDim.x].
__global__ __launch_bounds__(kEW) void k_spatial(float2* __restrict__ buf, float* __restrict__ z,
                                                 float* __restrict__ theta, const int64_t* __restrict__ zoff,
                                                 const float* __restrict__ rho_cur,
                                                 float beta, double* __restrict__ rpart, int K, int P, int64_t D,
                                                 const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  __shared__ double red[kEW / 64];
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, n = blockIdx.z;
  const float rho = rho_cur[n], thr = rho * beta, inv_rho = 1.0f / rho, invD = 1.0f / (float)D;
  double s = 0.0;
  if (f < D) {
    const int ka = 2 * p, kb = 2 * p + 1;
    const bool hb = kb < K;
    float2* bp = buf + (int64_t(n) * P + p) * D + f;
    const float2 c = *bp;
    const float va = c.x * invD, vb = c.y * invD;
    const int64_t zbase = map_base(zoff, n, K, D);
    float* za = z + zbase + int64_t(ka) * D + f;
    float* zb = z + zbase + int64_t(hb ? kb : ka) * D + f;
    const float a0 = *za, b0 = hb ? *zb : 0.f;
    const float a1 = soft_thresh(fmaf(-rho, va, a0), thr);
    const float b1 = hb ? soft_thresh(fmaf(-rho, vb, b0), thr) : 0.f;
    const double da = (double)a1 - a0, db = (double)b1 - b0;
    s = da * da + db * db;
    *za = a1;
    if (hb) *zb = b1;
    if (theta) {
      theta[zbase + int64_t(ka) * D + f] = va + (a1 - a0) * inv_rho;
      if (hb) theta[zbase + int64_t(kb) * D + f] = vb + (b1 - b0) * inv_rho;
    }
    *bp = make_float2(a1, b1);
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) rpart[(int64_t(n) * P + p) * gridDim.x + blockIdx.x] = t;
}

// part[n][0][j](f) = sum_p buf[n][p](f) conj(E_jp(f))
template <int J>
__global__ void k_accum(const float2* __restrict__ buf, const float2* __restrict__ E, float2* __restrict__ part,
                        int P, int64_t D, const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (f >= D) return;
  float2 y[J];
#pragma unroll
  for (int j = 0; j < J; ++j) y[j] = make_float2(0.f, 0.f);
  for (int p = 0; p < P; ++p) {
    const float2 c = buf[(int64_t(n) * P + p) * D + f];
#pragma unroll
    for (int j = 0; j < J; ++j) y[j] = cadd(y[j], cmulc(c, E[(int64_t(j) * P + p) * D + f]));
  }
#pragma unroll
  for (int j = 0; j < J; ++j) part[(int64_t(n) * J + j) * D + f] = y[j];
}

// ---------------------------------------------------------------- objective

// opart[n][blk] = sum_f sum_j |xhat_j - yhat_j|^2 (yhat = sym(sum_g part)).
template <int J>
__global__ __launch_bounds__(kEW) void k_obj_spec(const float2* __restrict__ part, const float2* __restrict__ xh,
                                                  double* __restrict__ opart, int ng, int T, int H, int W) {
  __shared__ double red[kEW / 64];
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  double s = 0.0;
  const int64_t fn = f < D ? neg_index(f, T, H, W) : 0;
  if (f < D && fn >= f) {  // the pair (f, -f) once, by its lower index
#pragma unroll
    for (int j = 0; j < J; ++j) {
      float2 y, ym;
      group_sums<8>(part + (int64_t(n) * ng * J + j) * D, int64_t(J) * D, ng, f, fn, y, ym);
      const double sx = 0.5 * ((double)y.x + ym.x), sy = 0.5 * ((double)y.y - ym.y);  // yhat at f
      const float2 x = xh[(int64_t(n) * J + j) * D + f];
      double rx = (double)x.x - sx, ry = (double)x.y - sy;
      s += rx * rx + ry * ry;
      if (fn != f) {  // yhat(-f) = conj(yhat(f))
        const float2 xm = xh[(int64_t(n) * J + j) * D + fn];
        rx = (double)xm.x - sx;
        ry = (double)xm.y + sy;
        s += rx * rx + ry * ry;
      }
    }
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) opart[int64_t(n) * gridDim.x + blockIdx.x] = t;
}

// out[n] = 0.5 sum(opart[n]) / D + beta sum(l1[n]): one workgroup per image,
// partials summed in a fixed order.
__global__ __launch_bounds__(kEW) void k_obj_final(const double* __restrict__ opart, int nopart,
                                                   const double* __restrict__ l1, int nl1, double* __restrict__ out,
                                                   int N, int64_t D, float beta) {
  __shared__ double red[kEW / 64];
  const int n = blockIdx.x;
  double r = 0.0, a = 0.0;
  for (int i = threadIdx.x; i < nopart; i += kEW) r += opart[int64_t(n) * nopart + i];
  for (int i = threadIdx.x; i < nl1; i += kEW) a += l1[int64_t(n) * nl1 + i];
  r = block_sum(r, red);
  a = block_sum(a, red);
  if (threadIdx.x == 0) out[n] = 0.5 * r / (double)D + (double)beta * a;
}

// out[N] = sum over images of out[n], in image order
__global__ void k_obj_total(double* __restrict__ out, int N) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double tot = 0.0;
  for (int n = 0; n < N; ++n) tot += out[n];
  out[N] = tot;
}

// ================================================================== host side

static unsigned nblk(int64_t n, int b = kEW) { return (unsigned)((n + b - 1) / b); }

#define LAUNCH_J(KERNEL, J, grid, block, st, ...)                                          \
  do {                                                                                     \
    if ((J) == 1) hipLaunchKernelGGL(KERNEL<1>, grid, block, 0, st, __VA_ARGS__);          \
    else if ((J) == 2) hipLaunchKernelGGL(KERNEL<2>, grid, block, 0, st, __VA_ARGS__);     \
    else hipLaunchKernelGGL(KERNEL<3>, grid, block, 0, st, __VA_ARGS__);                   \
  } while (0)

template <int J, int MODE>
static bool fused_launch(const Plan& pl, const float2* E, const float2* lam, float* z, float* theta,
                         const float* rho, float beta, float2* part, double* rpart, hipStream_t st,
                         const int* stop, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid(pl.ng * pl.n);
  const int h = pl.g[1], w = pl.g[2];
#define FL(HH, WW)                                                                                         \
  if (h == HH && w == WW) {                                                                                \
    if (e0)                                                                                                \
      hipExtLaunchKernelGGL((k_fused<HH, WW, J, MODE>), grid, dim3(fused_threads(HH * WW, J)), 0, st, e0, \
                            e1, 0, E, lam, z, theta, pl.zoff, rho, beta, part, rpart, pl.k, pl.p, pl.ppg,   \
                            pl.ng, stop);                                                                  \
    else                                                                                                   \
      hipLaunchKernelGGL((k_fused<HH, WW, J, MODE>), grid, dim3(fused_threads(HH * WW, J)), 0, st, E, lam,  \
                         z, theta, pl.zoff, rho, beta, part, rpart, pl.k, pl.p, pl.ppg, pl.ng, stop);      \
    return true;                                                                                           \
  }
  FL(16, 16) FL(16, 32) FL(16, 64) FL(16, 128) FL(16, 256)
  FL(32, 16) FL(32, 32) FL(32, 64) FL(32, 128) FL(32, 256)
  FL(64, 16) FL(64, 32) FL(64, 64) FL(64, 128) FL(64, 256)
  FL(128, 16) FL(128, 32) FL(128, 64) FL(128, 128)
  FL(256, 16) FL(256, 32) FL(256, 64)
#undef FL
  return false;
}

// e0, e1: events to launch with (an own-launch TraceScope's), or null
template <int MODE>
static bool fused_dispatch(const Plan& pl, const float2* E, const float2* lam, float* z, float* theta,
                           const float* rho, float beta, float2* part, double* rpart, hipStream_t st,
                           const int* stop = nullptr, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  if (pl.j == 1) return fused_launch<1, MODE>(pl, E, lam, z, theta, rho, beta, part, rpart, st, stop, e0, e1);
  if (pl.j == 2) return fused_launch<2, MODE>(pl, E, lam, z, theta, rho, beta, part, rpart, st, stop, e0, e1);
  return fused_launch<3, MODE>(pl, E, lam, z, theta, rho, beta, part, rpart, st, stop, e0, e1);
}

size_t carve_code(const Plan& pl, void* base, CodeWs* w) {
  Carver c(base);
  const int64_t D = pl.dsz, N = pl.n, J = pl.j, P = pl.p;
  // single-tile plans with J > 1 write pair spectra to buf and reduce them
  // with k_accum into one partial per image
  const bool tile1 = pl.lds && pl.j == 1;
  w->ngp = (tile1 || pl.split) ? pl.ng : 1;
  w->npri = pl.lds ? pl.ng : pl.split ? int(P * split_col_blocks(pl)) : int(P * nblk(D));
  w->ndual = (int)nblk(D);
  w->E = c.take<float2>(J * P * D);
  w->G = c.take<float2>(D * J * J);
  w->xh = c.take<float2>(N * J * D);
  w->yh = c.take<float2>(N * J * D);
  w->Th = c.take<float2>(N * J * D);
  w->lam = c.take<float2>(N * J * D);
  w->part = c.take<float2>(N * w->ngp * J * D);
  w->buf = tile1 ? nullptr : c.take<float2>(N * P * D);
  w->rpri = c.take<double>(N * w->npri);
  w->rdual = c.take<double>(N * w->ndual);
  w->opart = c.take<double>(N * w->ndual);
  w->rho = c.take<float>(N);
  w->rho2 = c.take<float>(N);
  w->rres = c.take<double>(2 * N);
  w->stop = c.take<int>(2);
  w->rmap = pl.nuclear ? c.take<double>(N * int64_t(pl.k)) : nullptr;
  return c.off;
}

static size_t code_ws_bytes(const Plan& pl) {
  CodeWs w;
  return carve_code(pl, nullptr, &w);
}

// Filter pair spectra E and the Gram blocks G; image spectra xhat.
hipError_t setup_spectra(const Plan& pl, const float* b, const float* d, CodeWs& w, hipStream_t st) {
  const int64_t D = pl.dsz;
  const int T = pl.g[0], H = pl.g[1], W = pl.g[2];
  hipLaunchKernelGGL(k_pack_filters, dim3(nblk(D), pl.p, pl.j), dim3(kEW), 0, st, d, w.E, pl.k, pl.j, pl.p, T, H,
                     W, pl.fs[0], pl.fs[1], pl.fs[2]);
  hipError_t e = fft_grids(w.E, int64_t(pl.j) * pl.p, pl.g, +1, st);
  if (e != hipSuccess) return e;
  LAUNCH_J(k_gram, pl.j, dim3(nblk(D)), dim3(kEW), st, w.E, w.G, pl.p, T, H, W);
  hipLaunchKernelGGL(k_pack_images, dim3(nblk(D), pl.j, pl.n), dim3(kEW), 0, st, b, pl.boff, w.xh, pl.j, D);
  e = fft_grids(w.xh, int64_t(pl.n) * pl.j, pl.g, -1, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// part <- contributions of the given maps (forward FFT, times conj(E)); the
// per-image l1 norms go to `l1` ([N][npri]).
hipError_t forward_maps(const Plan& pl, const float* maps, CodeWs& w, double* l1, hipStream_t st) {
  const int64_t D = pl.dsz;
  if (pl.lds) {
    if (!fused_dispatch<kModeForward>(pl, w.E, w.lam, const_cast<float*>(maps), nullptr, w.rho, 0.f,
                                      pl.j == 1 ? w.part : w.buf, l1, st))
      return hipErrorInvalidValue;
    if (pl.j > 1) LAUNCH_J(k_accum, pl.j, dim3(nblk(D), pl.n), dim3(kEW), st, w.buf, w.E, w.part, pl.p, D, nullptr);
    return hipGetLastError();
  }
  if (pl.split)
    return split_maps(pl, w.E, w.lam, w.buf, const_cast<float*>(maps), nullptr, w.rho, 0.f, w.part, l1, 1, st,
                      nullptr);
  hipLaunchKernelGGL(k_pack_maps, dim3(nblk(D), pl.p, pl.n), dim3(kEW), 0, st, maps, pl.zoff, w.buf, l1, pl.k,
                     pl.p, D);
  hipError_t e = fft_grids(w.buf, int64_t(pl.n) * pl.p, pl.g, -1, st);
  if (e != hipSuccess) return e;
  LAUNCH_J(k_accum, pl.j, dim3(nblk(D), pl.n), dim3(kEW), st, w.buf, w.E, w.part, pl.p, D, nullptr);
  return hipGetLastError();
}

// One ADMM iteration's map work: back-projection, soft threshold, forward.
// One ADMM iteration's map kernels.  zin: the codes to start from (null: z,
// updated in place); the split path reads them directly, the others copy
// them into z first.
static hipError_t iterate_maps(const Plan& pl, CodeWs& w, float* z, float* theta, float beta, hipStream_t st,
                               const int* stop, const float* zin = nullptr) {
  const int64_t D = pl.dsz;
  if (zin && pl.zoff) return hipErrorInvalidValue;  // dense layouts only
  if (zin && !pl.split)
    hipLaunchKernelGGL(k_copy_f, dim3(nblk(int64_t(pl.n) * pl.k * D)), dim3(kEW), 0, st, z, zin,
                       int64_t(pl.n) * pl.k * D);
  // one kernel on the single-tile path (timed at its own start and end),
  // several otherwise (timed around them)
  TraceScope trace(kTraceCodeMaps, st, pl.lds);
  if (pl.lds) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    trace.events(&e0, &e1);
    if (!fused_dispatch<kModeIter>(pl, w.E, w.lam, z, theta, w.rho, beta, pl.j == 1 ? w.part : w.buf, w.rpri, st,
                                   stop, e0, e1))
      return hipErrorInvalidValue;
    if (pl.j > 1) LAUNCH_J(k_accum, pl.j, dim3(nblk(D), pl.n), dim3(kEW), st, w.buf, w.E, w.part, pl.p, D, stop);
    return hipGetLastError();
  }
  if (pl.split) return split_maps(pl, w.E, w.lam, w.buf, z, theta, w.rho, beta, w.part, w.rpri, 0, st, stop, zin);
  hipError_t e;
  if (pl.vol) {
    if ((e = vol_maps(pl, w.E, w.lam, w.buf, z, theta, w.rho, beta, w.rpri, st, stop)) != hipSuccess) return e;
    LAUNCH_J(k_accum, pl.j, dim3(nblk(D), pl.n), dim3(kEW), st, w.buf, w.E, w.part, pl.p, D, stop);
    return hipGetLastError();
  }
  LAUNCH_J(k_make_v, pl.j, dim3(nblk(D), pl.p, pl.n), dim3(kEW), st, w.E, w.lam, w.buf, pl.p, D, stop);
  e = fft_grids(w.buf, int64_t(pl.n) * pl.p, pl.g, +1, st);
  if (e != hipSuccess) return e;
  if (pl.nuclear) {
    // z holds the input codes (copied from zin above when given)
    if ((e = launch_svt(pl, w.buf, z, nullptr, theta, w.rho, beta, w.rmap, 0, st, stop)) != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_spatial, dim3(nblk(D), pl.p, pl.n), dim3(kEW), 0, st, w.buf, z, theta, pl.zoff, w.rho,
                       beta, w.rpri, pl.k, pl.p, D, stop);
  }
  e = fft_grids(w.buf, int64_t(pl.n) * pl.p, pl.g, -1, st);
  if (e != hipSuccess) return e;
  LAUNCH_J(k_accum, pl.j, dim3(nblk(D), pl.n), dim3(kEW), st, w.buf, w.E, w.part, pl.p, D, stop);
  return hipGetLastError();
}

hipError_t code_prepare(const Plan& pl, const float* b, const float* d, const float* rho, unsigned flags, float* z,
                        const float* theta, bool solve, CodeWs& w, hipStream_t st) {
  const int64_t D = pl.dsz, N = pl.n, J = pl.j;
  const int T = pl.g[0], H = pl.g[1], W = pl.g[2];
  const bool z_zero = (flags & CSC_Z_ZERO) != 0;
  const bool th_zero = theta == nullptr || (flags & CSC_THETA_ZERO) != 0;
  const int64_t ns = N * J * D;
  hipError_t e;
  if ((e = setup_spectra(pl, b, d, w, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_f, dim3(nblk(N)), dim3(kEW), 0, st, w.rho, rho, N);
  if (z_zero) {
    hipLaunchKernelGGL(k_zero_maps, dim3(nblk(int64_t(pl.k) * D), N), dim3(kEW), 0, st, z, pl.zoff, pl.k, D);
    hipLaunchKernelGGL(k_fill_f2, dim3(nblk(ns)), dim3(kEW), 0, st, w.yh, ns);
  } else {
    if ((e = forward_maps(pl, z, w, w.rpri, st)) != hipSuccess) return e;
    LAUNCH_J(k_sym_reduce, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.part, w.yh, w.ngp, T, H, W);
  }
  if (th_zero) {
    hipLaunchKernelGGL(k_fill_f2, dim3(nblk(ns)), dim3(kEW), 0, st, w.Th, ns);
  } else {
    if ((e = forward_maps(pl, theta, w, w.rpri, st)) != hipSuccess) return e;
    LAUNCH_J(k_sym_reduce, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.part, w.Th, w.ngp, T, H, W);
  }
  if (solve) LAUNCH_J(k_solve, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.G, w.xh, w.yh, w.Th, w.rho, w.lam, D, nullptr);
  return hipGetLastError();
}

int run_code(const Plan& pl, const float* b, const float* d, float beta, float* rho, int iters, unsigned flags,
             float* z, float* theta, double* resid, void* ws, hipStream_t st, float tol, int* iters_done, float* ckpt,
             int every) {
  const bool adaptive = (flags & CSC_ADAPTIVE_RHO) != 0;
  if (ckpt && (tol > 0.0f || adaptive || every < 1 || pl.zoff)) return CSC_EINVAL;
  CodeWs w;
  carve_code(pl, ws, &w);
  const int64_t D = pl.dsz, N = pl.n, J = pl.j;
  const int T = pl.g[0], H = pl.g[1], W = pl.g[2];
  const bool z_zero = (flags & CSC_Z_ZERO) != 0;
  const bool th_zero = theta == nullptr || (flags & CSC_THETA_ZERO) != 0;
  const int64_t ns = N * J * D;
  hipError_t e;
  if ((e = setup_spectra(pl, b, d, w, st)) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(k_copy_f, dim3(nblk(N)), dim3(kEW), 0, st, w.rho, rho, N);
  if (z_zero) {
    hipLaunchKernelGGL(k_zero_maps, dim3(nblk(int64_t(pl.k) * D), N), dim3(kEW), 0, st, z, pl.zoff, pl.k, D);
    hipLaunchKernelGGL(k_fill_f2, dim3(nblk(ns)), dim3(kEW), 0, st, w.yh, ns);
  } else {
    if ((e = forward_maps(pl, z, w, w.rpri, st)) != hipSuccess) return CSC_EHIP;
    LAUNCH_J(k_sym_reduce, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.part, w.yh, w.ngp, T, H, W);
  }
  if (th_zero) {
    hipLaunchKernelGGL(k_fill_f2, dim3(nblk(ns)), dim3(kEW), 0, st, w.Th, ns);
    if (theta && iters == 0)
      hipLaunchKernelGGL(k_zero_maps, dim3(nblk(int64_t(pl.k) * D), N), dim3(kEW), 0, st, theta, pl.zoff, pl.k, D);
  } else {
    if ((e = forward_maps(pl, theta, w, w.rpri, st)) != hipSuccess) return CSC_EHIP;
    LAUNCH_J(k_sym_reduce, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.part, w.Th, w.ngp, T, H, W);
  }
  // tolerance mode: every launch of the iteration loop checks the stop flag,
  // so iterations after convergence cost a launch each and no work
  const bool tol_mode = tol > 0.0f;
  const int* stop = tol_mode ? w.stop : nullptr;
  if (tol_mode) hipLaunchKernelGGL(k_stop_init, dim3(1), dim3(64), 0, st, w.stop);
  if (iters > 0)
    LAUNCH_J(k_solve, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.G, w.xh, w.yh, w.Th, w.rho, w.lam, D, nullptr);
  const bool need_rho = adaptive || resid != nullptr || tol_mode;
  const double thr_pri = (double)tol * sqrt((double)pl.k * (double)D);
  const double thr_dual = (double)tol * sqrt((double)J * (double)D);
  // a record holds z and theta, then the spectral state the next iteration
  // starts from (yhat, Thhat and lam), so that replay_code resumes the loop
  // exactly where it was
  const int64_t nz = N * pl.k * D, rec_floats = code_record_floats(pl);
  auto save_spec = [&](float* rec) {
    float* s = rec + 2 * nz;
    hipLaunchKernelGGL(k_copy_f, dim3(nblk(2 * ns)), dim3(kEW), 0, st, s, (const float*)w.yh, 2 * ns);
    hipLaunchKernelGGL(k_copy_f, dim3(nblk(2 * ns)), dim3(kEW), 0, st, s + 2 * ns, (const float*)w.Th, 2 * ns);
    hipLaunchKernelGGL(k_copy_f, dim3(nblk(2 * ns)), dim3(kEW), 0, st, s + 4 * ns, (const float*)w.lam, 2 * ns);
  };
  if (ckpt && iters > 0) {
    hipLaunchKernelGGL(k_fill_f2, dim3(nblk(nz)), dim3(kEW), 0, st, (float2*)ckpt, nz);
    save_spec(ckpt);
  }
  // on the split path a record iteration writes its codes straight into the
  // record and the next iteration reads them from there (records are never
  // at the last iteration, so z ends with the final codes); elsewhere they
  // are copied
  const float* zsrc = nullptr;  // where the current codes are, when not in z
  for (int it = 0; it < iters; ++it) {
    const bool last = it == iters - 1;
    // theta is written by the last iteration, or by every one when the loop may stop early
    float* th_out = (last || tol_mode) ? theta : nullptr;
    float* rec = (ckpt && !last && (it + 1) % every == 0) ? ckpt + int64_t((it + 1) / every) * rec_floats : nullptr;
    if (rec) th_out = rec + nz;
    const bool into_rec = rec && pl.split;
    // the input is wherever the current codes are (z unless a record holds them)
    const float* zin = into_rec ? (zsrc ? zsrc : z) : zsrc;
    if ((e = iterate_maps(pl, w, into_rec ? rec : z, th_out, beta, st, stop, zin)) != hipSuccess) return CSC_EHIP;
    zsrc = into_rec ? rec : nullptr;
    if (rec && !into_rec) hipLaunchKernelGGL(k_copy_f, dim3(nblk(nz)), dim3(kEW), 0, st, rec, z, nz);
    const int solve_next = (!last && !adaptive) ? 1 : 0;
    {
      TraceScope trace(kTraceCodeSpec, st, true);
      if (pl.j == 1 && w.ngp > 8)
        LAUNCH_J_TRACED(trace, k_spec_wide, 1, dim3(nblk(D), N), dim3(kEW), st, w.part, w.G, w.xh, w.yh, w.Th,
                        w.lam, w.rho, w.rdual, w.ngp, T, H, W, solve_next, stop);
      else
        LAUNCH_J_TRACED(trace, k_spec, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.part, w.G, w.xh, w.yh, w.Th, w.lam,
                        w.rho, w.rdual, w.ngp, T, H, W, solve_next, stop);
    }
    if (rec) save_spec(rec);
    if (adaptive && !last && !tol_mode) {
      // residual-balancing step and the next solve in one launch; the new
      // rho goes to the other buffer, which the next iteration reads
      LAUNCH_J(k_solve_rho, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.G, w.xh, w.yh, w.Th,
               pl.nuclear ? w.rmap : w.rpri, pl.nuclear ? pl.k : w.npri, w.rdual, w.ndual, w.rho, w.rho2, resid, it,
               (int)N, w.lam, D);
      std::swap(w.rho, w.rho2);
      continue;
    }
    if (need_rho)
      hipLaunchKernelGGL(k_rho, dim3((unsigned)N), dim3(64), 0, st, pl.nuclear ? w.rmap : w.rpri,
                         pl.nuclear ? pl.k : w.npri, w.rdual, w.ndual, w.rho, resid, it, (int)N, D, adaptive ? 1 : 0,
                         stop, tol_mode ? w.rres : nullptr);
    if (tol_mode) hipLaunchKernelGGL(k_stop, dim3(1), dim3(64), 0, st, w.rres, (int)N, thr_pri, thr_dual, w.stop);
    if (adaptive && !last)
      LAUNCH_J(k_solve, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.G, w.xh, w.yh, w.Th, w.rho, w.lam, D, stop);
  }
  if (adaptive) hipLaunchKernelGGL(k_copy_f, dim3(nblk(N)), dim3(kEW), 0, st, rho, w.rho, N);
  if (iters_done) {
    if (tol_mode) hipLaunchKernelGGL(k_stop_out, dim3(1), dim3(64), 0, st, w.stop, iters_done);
    else hipLaunchKernelGGL(k_fill_i, dim3(1), dim3(64), 0, st, iters_done, iters);
  }
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

int64_t code_record_floats(const Plan& pl) {
  return int64_t(pl.n) * pl.dsz * (2 * int64_t(pl.k) + 6 * int64_t(pl.j));
}

hipError_t replay_code(const Plan& pl, CodeWs& w, const float* rho, float beta, const float* rec, int nstates,
                       float* seg, hipStream_t st) {
  const int64_t D = pl.dsz, N = pl.n, nz = N * pl.k * D, ns = N * pl.j * D;
  const int T = pl.g[0], H = pl.g[1], W = pl.g[2];
  const float* s = rec + 2 * nz;
  hipLaunchKernelGGL(k_copy_f, dim3(nblk(N)), dim3(kEW), 0, st, w.rho, rho, N);
  hipLaunchKernelGGL(k_copy_f, dim3(nblk(2 * ns)), dim3(kEW), 0, st, (float*)w.yh, s, 2 * ns);
  hipLaunchKernelGGL(k_copy_f, dim3(nblk(2 * ns)), dim3(kEW), 0, st, (float*)w.Th, s + 2 * ns, 2 * ns);
  hipLaunchKernelGGL(k_copy_f, dim3(nblk(2 * ns)), dim3(kEW), 0, st, (float*)w.lam, s + 4 * ns, 2 * ns);
  for (int i = 1; i < nstates; ++i) {
    // the iteration updates z in place: start from the previous state's codes
    float* zi = seg + int64_t(i - 1) * 2 * nz;
    const float* zprev = i == 1 ? rec : zi - 2 * nz;
    hipError_t e = iterate_maps(pl, w, zi, zi + nz, beta, st, nullptr, zprev);
    if (e != hipSuccess) return e;
    if (i < nstates - 1)
      {
        // the same kernel as the forward loop, so the states agree bit for bit
        if (pl.j == 1 && w.ngp > 8)
          LAUNCH_J(k_spec_wide, 1, dim3(nblk(D), N), dim3(kEW), st, w.part, w.G, w.xh, w.yh, w.Th, w.lam, w.rho,
                   w.rdual, w.ngp, T, H, W, 1, nullptr);
        else
          LAUNCH_J(k_spec, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.part, w.G, w.xh, w.yh, w.Th, w.lam, w.rho,
                   w.rdual, w.ngp, T, H, W, 1, nullptr);
      }
  }
  return hipGetLastError();
}

__global__ void k_flag_zero(int* __restrict__ flag) {
  if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = 0;
}
// Every workgroup that sees a NaN or an infinity stores 1 (the same value
// from any number of workgroups, so no atomics and no ordering are needed).
__global__ __launch_bounds__(kEW) void k_check_finite(const float* __restrict__ x, int64_t n, int* __restrict__ flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    mine |= !isfinite(x[i]);
  if (mine) bad = 1;
  __syncthreads();
  if (threadIdx.x == 0 && bad) flag[0] = 1;
}

hipError_t launch_check_finite(const float* x, int64_t n, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_flag_zero, dim3(1), dim3(64), 0, st, flag);
  if (n > 0) {
    const int64_t blocks = std::min<int64_t>((n + kEW - 1) / kEW, 4096);
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(kEW), 0, st, x, n, flag);
  }
  return hipGetLastError();
}

size_t run_code_ws(const Plan& pl) { return code_ws_bytes(pl); }

void launch_rho(const double* rpri, int npri, const double* rdual, int ndual, float* rho, double* resid, int it,
                int N, int64_t D, int adaptive, hipStream_t st) {
  hipLaunchKernelGGL(k_rho, dim3((unsigned)N), dim3(64), 0, st, rpri, npri, rdual, ndual, rho, resid, it, N, D,
                     adaptive, nullptr, nullptr);
}

void launch_obj_final(const double* opart, int nopart, const double* l1, int nl1, double* out, int N, int64_t D,
                      float beta, hipStream_t st) {
  hipLaunchKernelGGL(k_obj_final, dim3((unsigned)N), dim3(kEW), 0, st, opart, nopart, l1, nl1, out, N, D, beta);
  hipLaunchKernelGGL(k_obj_total, dim3(1), dim3(64), 0, st, out, N);
}

void launch_make_v(const Plan& pl, const float2* E, const float2* lam, float2* buf, hipStream_t st) {
  LAUNCH_J(k_make_v, pl.j, dim3(nblk(pl.dsz), pl.p, pl.n), dim3(kEW), st, E, lam, buf, pl.p, pl.dsz, nullptr);
}

void launch_sym_reduce(const Plan& pl, const float2* part, int ng, float2* dst, hipStream_t st) {
  LAUNCH_J(k_sym_reduce, pl.j, dim3(nblk(pl.dsz), pl.n), dim3(kEW), st, part, dst, ng, pl.g[0], pl.g[1], pl.g[2]);
}

void launch_objective_tail(const Plan& pl, CodeWs& w, float beta, double* out, hipStream_t st) {
  LAUNCH_J(k_obj_spec, pl.j, dim3(nblk(pl.dsz), pl.n), dim3(kEW), st, w.part, w.xh, w.opart, w.ngp, pl.g[0], pl.g[1],
           pl.g[2]);
  hipLaunchKernelGGL(k_obj_final, dim3((unsigned)pl.n), dim3(kEW), 0, st, w.opart, w.ndual, w.rpri, w.npri, out, pl.n,
                     pl.dsz, beta);
  hipLaunchKernelGGL(k_obj_total, dim3(1), dim3(64), 0, st, out, pl.n);
}

int run_objective(const Plan& pl, const float* b, const float* d, const float* z, float beta, double* out, void* ws,
                  hipStream_t st) {
  CodeWs w;
  carve_code(pl, ws, &w);
  const int64_t D = pl.dsz, N = pl.n;
  const int T = pl.g[0], H = pl.g[1], W = pl.g[2];
  if (setup_spectra(pl, b, d, w, st) != hipSuccess) return CSC_EHIP;
  if (forward_maps(pl, z, w, w.rpri, st) != hipSuccess) return CSC_EHIP;
  LAUNCH_J(k_obj_spec, pl.j, dim3(nblk(D), N), dim3(kEW), st, w.part, w.xh, w.opart, w.ngp, T, H, W);
  if (pl.nuclear &&
      launch_svt(pl, nullptr, const_cast<float*>(z), nullptr, nullptr, nullptr, 0.f, w.rmap, 1, st, nullptr) !=
          hipSuccess)
    return CSC_EHIP;
  hipLaunchKernelGGL(k_obj_final, dim3((unsigned)N), dim3(kEW), 0, st, w.opart, w.ndual,
                     pl.nuclear ? w.rmap : w.rpri, pl.nuclear ? pl.k : w.npri, out, (int)N, D, beta);
  hipLaunchKernelGGL(k_obj_total, dim3(1), dim3(64), 0, st, out, (int)N);
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

}  // namespace dcsc
