// Learning subproblem in the dual (eq:Learning_Dual .. eq:mu_update).
//
// For fixed multipliers mu, gamma solves (eq:Learning_gamma)
//     A gamma = -x,   A = I + sum_k 1/(2 mu_k) Z_k S^T S Z_k^T,
// by conjugate gradient.  All CG vectors live in the Fourier domain (full
// complex grids, one per image and channel): the operator is
//     t_k   = sum_n conj(zhat_k^n) phat^n            (pass A, Z_k^T p)
//     u_k   = S^T S IDFT(t_k) / (2 mu_k)              (support projection)
//     qhat^n = phat^n + sum_k zhat_k^n DFT(u_k)       (pass B)
// and inner products follow from Parseval (the common 1/D factor cancels in
// the CG ratios).  Scalars are float64 and every reduction runs in a fixed
// order.  Maps and filters travel in pairs (2p, 2p+1) as the real and
// imaginary parts of one complex grid; a pair spectrum C unpacks as
//     zhat_2p(f) = (C(f) + conj(C(-f)))/2,  zhat_2p+1(f) = -i (C(f) - conj(C(-f)))/2.
#include "common.hpp"
#include "internal.hpp"

namespace dcsc {

hipError_t fft_grids(float2* data, int64_t count, const int g[3], int dir, hipStream_t st);

constexpr int kLW = 256;

static unsigned lblk(int64_t n, int b = kLW) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ int64_t lneg(int64_t fl, int T, int H, int W) {
  const int f = (int)fl;
  const int lw = __builtin_ctz(W), lh = __builtin_ctz(H);
  const int w = f & (W - 1), h = (f >> lw) & (H - 1), t = f >> (lw + lh);
  return (((((T - t) & (T - 1)) << lh) | ((H - h) & (H - 1))) << lw) | ((W - w) & (W - 1));
}

__device__ __forceinline__ void unpack_pair(float2 c, float2 cm, float2& a, float2& b) {
  // a = (c + conj(cm))/2 ; b = -i (c - conj(cm))/2
  a = make_float2(0.5f * (c.x + cm.x), 0.5f * (c.y - cm.y));
  const float dx = c.x - cm.x, dy = c.y + cm.y;
  b = make_float2(0.5f * dy, -0.5f * dx);
}

__global__ void l_pack_maps(const float* __restrict__ z, float2* __restrict__ Zh, int K, int P, int64_t D) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, n = blockIdx.z;
  if (f >= D) return;
  const float a = z[(int64_t(n) * K + 2 * p) * D + f];
  const float b = (2 * p + 1 < K) ? z[(int64_t(n) * K + 2 * p + 1) * D + f] : 0.f;
  Zh[(int64_t(n) * P + p) * D + f] = make_float2(a, b);
}

__global__ void l_real_to_complex(const float* __restrict__ src, float2* __restrict__ dst, int64_t count, int zero) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) dst[i] = make_float2(zero ? 0.f : src[i], 0.f);
}

__global__ void l_complex_to_real(const float2* __restrict__ src, float* __restrict__ dst, int64_t count, float s) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i].x * s;
}

// Tp[j][p](f) = t_2p,j(f) + i t_2p+1,j(f),  t_k,j(f) = sum_n conj(zhat_k^n(f)) v_j^n(f)
template <int J>
__global__ __launch_bounds__(kLW) void l_passA(const float2* __restrict__ Zh, const float2* __restrict__ v,
                                               float2* __restrict__ Tp, int N, int P, int T, int H, int W) {
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (f >= D) return;
  const int64_t fn = lneg(f, T, H, W);
  float2 ta[J], tb[J];
#pragma unroll
  for (int j = 0; j < J; ++j) ta[j] = tb[j] = make_float2(0.f, 0.f);
  for (int n = 0; n < N; ++n) {
    const float2* zp = Zh + (int64_t(n) * P + p) * D;
    float2 za, zb;
    unpack_pair(zp[f], zp[fn], za, zb);
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const float2 x = v[(int64_t(n) * J + j) * D + f];
      ta[j] = cadd(ta[j], cmulc(x, za));
      tb[j] = cadd(tb[j], cmulc(x, zb));
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j)
    Tp[(int64_t(j) * P + p) * D + f] = make_float2(ta[j].x - tb[j].y, ta[j].y + tb[j].x);
}

// In place on D * (t_2p + i t_2p+1) (spatial): keep the support, scale by
// 1/(2 mu_k D), zero elsewhere.
__global__ void l_crop_scale(float2* __restrict__ Tp, const float* __restrict__ mu, int K, int P, int T, int H,
                             int W, int ft, int fh, int fw) {
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, j = blockIdx.z;
  if (f >= D) return;
  const int t = (int)(f / (int64_t(H) * W)), h = (int)((f / W) % H), w = (int)(f % W);
  float2* e = Tp + (int64_t(j) * P + p) * D + f;
  float2 o = make_float2(0.f, 0.f);
  if (t < ft && h < fh && w < fw) {
    const float2 c = *e;
    const float invD = 1.0f / (float)D;
    o.x = c.x * invD / (2.0f * mu[2 * p]);
    o.y = (2 * p + 1 < K) ? c.y * invD / (2.0f * mu[2 * p + 1]) : 0.f;
  }
  *e = o;
}

constexpr int lt_threads(int d) { return d >= 16384 ? 1024 : d <= 1024 ? 64 : d / 16; }

// Single-tile version of (inverse FFT, crop/scale, forward FFT) for grids
// that fit LDS.  One workgroup per (pair, channel).
template <int H, int W>
__global__ __launch_bounds__(lt_threads(H * W)) void l_crop_tile(float2* __restrict__ Tp, const float* __restrict__ mu,
                                                                int K, int P, int fh, int fw) {
  constexpr int D = H * W, NT = lt_threads(D), WP = W + 1;
  __shared__ float2 tile[H * WP];
  __shared__ float2 tw[256];
  const int p = blockIdx.x, j = blockIdx.y;
  float2* g = Tp + (int64_t(j) * P + p) * D;
  load_twiddles(tw);
  for (int e = threadIdx.x; e < D; e += NT) tile[(e / W) * WP + (e % W)] = g[e];
  __syncthreads();
  fft2d_tile<H, W, WP, NT, 1>(tile, tw);
  const float invD = 1.0f / (float)D;
  const float sa = invD / (2.0f * mu[2 * p]);
  const float sb = (2 * p + 1 < K) ? invD / (2.0f * mu[2 * p + 1]) : 0.f;
  for (int e = threadIdx.x; e < D; e += NT) {
    const int h = e / W, w = e % W;
    float2* a = tile + h * WP + w;
    const float2 c = *a;
    *a = (h < fh && w < fw) ? make_float2(c.x * sa, c.y * sb) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft2d_tile<H, W, WP, NT, -1>(tile, tw);
  for (int e = threadIdx.x; e < D; e += NT) g[e] = tile[(e / W) * WP + (e % W)];
}

// q^n_j = v^n_j + sum_p (zhat_2p^n uhat_2p,j + zhat_2p+1^n uhat_2p+1,j); dot
// partials sum_f Re(v conj(q)) per (channel, image, block).  With `sub`,
// q is replaced by -x - q (the initial residual of the warm start), and the
// partials are |q|^2.
template <int J>
__global__ __launch_bounds__(kLW) void l_passB(const float2* __restrict__ Zh, const float2* __restrict__ Up,
                                               const float2* __restrict__ v, float2* __restrict__ q,
                                               const float2* __restrict__ xh, double* __restrict__ dots, int N,
                                               int P, int T, int H, int W) {
  __shared__ double red[kLW / 64];
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  double s[J];
#pragma unroll
  for (int j = 0; j < J; ++j) s[j] = 0.0;
  if (f < D) {
    const int64_t fn = lneg(f, T, H, W);
    float2 acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = make_float2(0.f, 0.f);
    for (int p = 0; p < P; ++p) {
      const float2* zp = Zh + (int64_t(n) * P + p) * D;
      float2 za, zb;
      unpack_pair(zp[f], zp[fn], za, zb);
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const float2* up = Up + (int64_t(j) * P + p) * D;
        float2 ua, ub;
        unpack_pair(up[f], up[fn], ua, ub);
        acc[j] = cadd(acc[j], cadd(cmul(za, ua), cmul(zb, ub)));
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t o = (int64_t(n) * J + j) * D + f;
      const float2 vv = v[o];
      float2 qq = cadd(vv, acc[j]);
      if (xh) {
        const float2 x = xh[o];
        qq = make_float2(-x.x - qq.x, -x.y - qq.y);
        s[j] = (double)qq.x * qq.x + (double)qq.y * qq.y;
      } else {
        s[j] = (double)vv.x * qq.x + (double)vv.y * qq.y;
      }
      q[o] = qq;
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const double t = block_sum(s[j], red);
    if (threadIdx.x == 0) dots[(int64_t(j) * N + n) * gridDim.x + blockIdx.x] = t;
  }
}

// Fixed-order sum of `cnt` partials by one block (all threads get the total).
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int cnt, double* red, double* bcast) {
  double s = 0.0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) s += p[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) *bcast = t;
  __syncthreads();
  return *bcast;
}

// gamma += alpha p ; r -= alpha q ; partials of |r|^2.  alpha = rr / pAp.
// `rr` is the running |r|^2 per channel (float64), `pap` the partials.
template <int J>
__global__ __launch_bounds__(kLW) void l_cg_step(float2* __restrict__ g, float2* __restrict__ r,
                                                 const float2* __restrict__ p, const float2* __restrict__ q,
                                                 const double* __restrict__ rr, const double* __restrict__ pap,
                                                 int npart, double* __restrict__ rrpart, int N, int64_t D) {
  __shared__ double red[kLW / 64];
  __shared__ double bc;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  double alpha[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const double pa = sum_partials(pap + int64_t(j) * npart, npart, red, &bc);
    alpha[j] = pa > 0.0 ? rr[j] / pa : 0.0;
  }
  double s[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    s[j] = 0.0;
    if (f < D) {
      const int64_t o = (int64_t(n) * J + j) * D + f;
      const float a = (float)alpha[j];
      const float2 pp = p[o], qq = q[o];
      float2 gg = g[o], rv = r[o];
      gg = make_float2(fmaf(a, pp.x, gg.x), fmaf(a, pp.y, gg.y));
      rv = make_float2(fmaf(-a, qq.x, rv.x), fmaf(-a, qq.y, rv.y));
      g[o] = gg;
      r[o] = rv;
      s[j] = (double)rv.x * rv.x + (double)rv.y * rv.y;
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const double t = block_sum(s[j], red);
    if (threadIdx.x == 0) rrpart[(int64_t(j) * N + n) * gridDim.x + blockIdx.x] = t;
  }
}

// p = r + (rr_new / rr) p; block (0,0) records rr_new into rr_next.
template <int J>
__global__ __launch_bounds__(kLW) void l_cg_dir(float2* __restrict__ p, const float2* __restrict__ r,
                                                const double* __restrict__ rr, const double* __restrict__ rrpart,
                                                int npart, double* __restrict__ rr_next, int copy_r, int64_t D) {
  __shared__ double red[kLW / 64];
  __shared__ double bc;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  double bet[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const double rn = sum_partials(rrpart + int64_t(j) * npart, npart, red, &bc);
    bet[j] = (!copy_r && rr[j] > 0.0) ? rn / rr[j] : 0.0;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) rr_next[j] = rn;
  }
  if (f < D) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t o = (int64_t(n) * J + j) * D + f;
      const float2 rv = r[o];
      if (copy_r) {
        p[o] = rv;
      } else {
        const float2 pp = p[o];
        const float b = (float)bet[j];
        p[o] = make_float2(fmaf(b, pp.x, rv.x), fmaf(b, pp.y, rv.y));
      }
    }
  }
}

// d_k,j[m] = -t_k,j[m] / (D 2 mu_k) from D * (t_2p + i t_2p+1) (spatial).
__global__ void l_drecover(const float2* __restrict__ Tp, const float* __restrict__ mu, float* __restrict__ d,
                           int K, int J, int P, int T, int H, int W, int ft, int fh, int fw) {
  const int64_t msz = int64_t(ft) * fh * fw;
  const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y, j = blockIdx.z;
  if (m >= msz) return;
  const int t = (int)(m / (int64_t(fh) * fw)), h = (int)((m / fw) % fh), w = (int)(m % fw);
  const int64_t D = int64_t(T) * H * W;
  const float2 c = Tp[(int64_t(j) * P + k / 2) * D + (int64_t(t) * H + h) * W + w];
  const float v = (k & 1) ? c.y : c.x;
  d[(int64_t(k) * J + j) * msz + m] = -v / ((float)D * 2.0f * mu[k]);
}

// Per filter: ||d_k|| over channels and taps; mu_k <- mu_k ||d_k|| (kept
// when the norm is 0); with `project`, d_k <- d_k / max(1, ||d_k||).
__global__ __launch_bounds__(kLW) void l_mu_update(float* __restrict__ d, float* __restrict__ mu, int64_t len,
                                                   int update_mu, int project) {
  __shared__ double red[kLW / 64];
  __shared__ double bc;
  const int k = blockIdx.x;
  float* dk = d + int64_t(k) * len;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += blockDim.x) s += (double)dk[i] * dk[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) bc = sqrt(t);
  __syncthreads();
  const double nrm = bc;
  if (project && nrm > 1.0) {
    const float sc = (float)(1.0 / nrm);
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) dk[i] *= sc;
  }
  if (update_mu && threadIdx.x == 0 && nrm > 0.0) mu[k] = (float)((double)mu[k] * nrm);
}

// ---------------------------------------------------------------- host side

#define LJ(KERNEL, J, grid, block, st, ...)                                           \
  do {                                                                                \
    if ((J) == 1) hipLaunchKernelGGL(KERNEL<1>, grid, block, 0, st, __VA_ARGS__);     \
    else if ((J) == 2) hipLaunchKernelGGL(KERNEL<2>, grid, block, 0, st, __VA_ARGS__); \
    else hipLaunchKernelGGL(KERNEL<3>, grid, block, 0, st, __VA_ARGS__);              \
  } while (0)

struct LearnWs {
  float2 *Zh, *xh, *gh, *rh, *ph, *qh, *Tp;
  double *dots, *rr;  // dots: [J][N][nblk]; rr: [cg_slots][J]
  int npart;
};

static size_t carve_learn(const Plan& pl, void* base, LearnWs* w) {
  Carver c(base);
  const int64_t D = pl.dsz, N = pl.n, J = pl.j, P = pl.p;
  w->npart = int(N * lblk(D));
  w->Zh = c.take<float2>(N * P * D);
  w->xh = c.take<float2>(N * J * D);
  w->gh = c.take<float2>(N * J * D);
  w->rh = c.take<float2>(N * J * D);
  w->ph = c.take<float2>(N * J * D);
  w->qh = c.take<float2>(N * J * D);
  w->Tp = c.take<float2>(J * P * D);
  w->dots = c.take<double>(J * w->npart * 2);
  w->rr = c.take<double>(4 * J);
  return c.off;
}

size_t run_learn_ws(const Plan& pl) {
  LearnWs w;
  return carve_learn(pl, nullptr, &w);
}

static bool crop_tile_launch(const Plan& pl, float2* Tp, const float* mu, hipStream_t st) {
  if (!(pl.g[0] == 1 && tile_supported(pl.g[1], pl.g[2]))) return false;
  const dim3 grid(pl.p, pl.j);
  const int h = pl.g[1], w = pl.g[2];
#define CT(HH, WW)                                                                                             \
  if (h == HH && w == WW) {                                                                                    \
    hipLaunchKernelGGL((l_crop_tile<HH, WW>), grid, dim3(lt_threads(HH * WW)), 0, st, Tp, mu, pl.k, pl.p,      \
                       pl.fs[1], pl.fs[2]);                                                                    \
    return true;                                                                                               \
  }
  CT(16, 16) CT(16, 32) CT(16, 64) CT(16, 128) CT(16, 256)
  CT(32, 16) CT(32, 32) CT(32, 64) CT(32, 128) CT(32, 256)
  CT(64, 16) CT(64, 32) CT(64, 64) CT(64, 128) CT(64, 256)
  CT(128, 16) CT(128, 32) CT(128, 64) CT(128, 128)
  CT(256, 16) CT(256, 32) CT(256, 64)
#undef CT
  return false;
}

// Up <- DFT(S^T S IDFT(pass A of v) / (2 mu))
static hipError_t apply_zt_proj(const Plan& pl, LearnWs& w, const float2* v, const float* mu, hipStream_t st) {
  const int64_t D = pl.dsz;
  TraceScope trace(kTraceLearnOp, st);
  const int T = pl.g[0], H = pl.g[1], W = pl.g[2];
  LJ(l_passA, pl.j, dim3(lblk(D), pl.p), dim3(kLW), st, w.Zh, v, w.Tp, pl.n, pl.p, T, H, W);
  if (crop_tile_launch(pl, w.Tp, mu, st)) return hipGetLastError();
  hipError_t e = fft_grids(w.Tp, int64_t(pl.j) * pl.p, pl.g, +1, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(l_crop_scale, dim3(lblk(D), pl.p, pl.j), dim3(kLW), 0, st, w.Tp, mu, pl.k, pl.p, T, H, W,
                     pl.fs[0], pl.fs[1], pl.fs[2]);
  return fft_grids(w.Tp, int64_t(pl.j) * pl.p, pl.g, -1, st);
}

int run_learn(const Plan& pl, const float* b, const float* z, float* d, float* mu, float* gamma, int inner_iters,
              int cg_iters, unsigned flags, void* ws, hipStream_t st) {
  LearnWs w;
  carve_learn(pl, ws, &w);
  const int64_t D = pl.dsz, N = pl.n, J = pl.j;
  const int T = pl.g[0], H = pl.g[1], W = pl.g[2];
  const int64_t ns = N * J * D;
  hipError_t e;
  // code spectra, image spectra, gamma spectra
  hipLaunchKernelGGL(l_pack_maps, dim3(lblk(D), pl.p, pl.n), dim3(kLW), 0, st, z, w.Zh, pl.k, pl.p, D);
  if ((e = fft_grids(w.Zh, N * pl.p, pl.g, -1, st)) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(l_real_to_complex, dim3(lblk(ns)), dim3(kLW), 0, st, b, w.xh, ns, 0);
  if ((e = fft_grids(w.xh, N * J, pl.g, -1, st)) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(l_real_to_complex, dim3(lblk(ns)), dim3(kLW), 0, st, gamma, w.gh, ns,
                     (flags & CSC_GAMMA_ZERO) ? 1 : 0);
  if ((e = fft_grids(w.gh, N * J, pl.g, -1, st)) != hipSuccess) return CSC_EHIP;

  const dim3 vgrid(lblk(D), pl.n);
  double* pap = w.dots;
  double* rrp = w.dots + J * w.npart;
  double* rr_a = w.rr;
  double* rr_b = w.rr + J;
  for (int it = 0; it < inner_iters; ++it) {
    // r = -x - A gamma ; p = r ; rr = |r|^2
    if ((e = apply_zt_proj(pl, w, w.gh, mu, st)) != hipSuccess) return CSC_EHIP;
    LJ(l_passB, pl.j, vgrid, dim3(kLW), st, w.Zh, w.Tp, w.gh, w.rh, w.xh, rrp, pl.n, pl.p, T, H, W);
    LJ(l_cg_dir, pl.j, vgrid, dim3(kLW), st, w.ph, w.rh, rr_a, rrp, w.npart, rr_a, 1, D);
    for (int q = 0; q < cg_iters; ++q) {
      if ((e = apply_zt_proj(pl, w, w.ph, mu, st)) != hipSuccess) return CSC_EHIP;
      LJ(l_passB, pl.j, vgrid, dim3(kLW), st, w.Zh, w.Tp, w.ph, w.qh, (const float2*)nullptr, pap, pl.n, pl.p, T, H,
         W);
      LJ(l_cg_step, pl.j, vgrid, dim3(kLW), st, w.gh, w.rh, w.ph, w.qh, rr_a, pap, w.npart, rrp, pl.n, D);
      LJ(l_cg_dir, pl.j, vgrid, dim3(kLW), st, w.ph, w.rh, rr_a, rrp, w.npart, rr_b, 0, D);
      double* t = rr_a;
      rr_a = rr_b;
      rr_b = t;
    }
    // d_k = -S Z_k^T gamma / (2 mu_k) ; mu_k <- mu_k ||d_k||
    LJ(l_passA, pl.j, dim3(lblk(D), pl.p), dim3(kLW), st, w.Zh, w.gh, w.Tp, pl.n, pl.p, T, H, W);
    if ((e = fft_grids(w.Tp, J * pl.p, pl.g, +1, st)) != hipSuccess) return CSC_EHIP;
    hipLaunchKernelGGL(l_drecover, dim3(lblk(pl.msz), pl.k, pl.j), dim3(kLW), 0, st, w.Tp, mu, d, pl.k, pl.j, pl.p,
                       T, H, W, pl.fs[0], pl.fs[1], pl.fs[2]);
    const bool last = it == inner_iters - 1;
    hipLaunchKernelGGL(l_mu_update, dim3(pl.k), dim3(kLW), 0, st, d, mu, int64_t(J) * pl.msz, 1, last ? 1 : 0);
  }
  // gamma back to the spatial domain
  hipMemcpyAsync(w.rh, w.gh, sizeof(float2) * ns, hipMemcpyDeviceToDevice, st);
  if ((e = fft_grids(w.rh, N * J, pl.g, +1, st)) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(l_complex_to_real, dim3(lblk(ns)), dim3(kLW), 0, st, w.rh, gamma, ns, 1.0f / (float)D);
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

}  // namespace dcsc
