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
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace dcsc {

hipError_t fft_grids(float2* data, int64_t count, const int g[3], int dir, hipStream_t st);

constexpr int kLW = 256;

constexpr int kPassAImgs = 5;    // pass A: images whose loads are issued together
constexpr int kPassBChunk1 = 10; // pass B: largest image chunk for one channel

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
                                               float2* __restrict__ Tp, int N, int P, int T, int H, int W,
                                               const int* __restrict__ cgf) {
  if (cgf && cgf[0]) return;
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
                             int W, int ft, int fh, int fw, const int* __restrict__ cgf) {
  if (cgf && cgf[0]) return;
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
                                                                int K, int P, int fh, int fw,
                                                                const int* __restrict__ cgf) {
  if (cgf && cgf[0]) return;
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
                                               const float2* __restrict__ xh, double* __restrict__ dots,
                                               double* __restrict__ vdots, int N, int P, int T, int H, int W,
                                               const int* __restrict__ cgf) {
  if (cgf && cgf[0]) return;
  __shared__ double red[kLW / 64];
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  double s[J], s2[J];
#pragma unroll
  for (int j = 0; j < J; ++j) s[j] = s2[j] = 0.0;
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
        s2[j] = (double)vv.x * vv.x + (double)vv.y * vv.y;
      }
      q[o] = qq;
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const double t = block_sum(s[j], red);
    if (threadIdx.x == 0) dots[(int64_t(j) * N + n) * gridDim.x + blockIdx.x] = t;
    if (vdots) {
      const double t2 = block_sum(s2[j], red);
      if (threadIdx.x == 0) vdots[(int64_t(j) * N + n) * gridDim.x + blockIdx.x] = t2;
    }
  }
}

// ------------------------------------- pruned 2-D operator (single frame)
// With the support S keeping m1 < M1, m2 < M2 (both at most kPruneMax), the
// projection u = S^T S IDFT(t) / (2 mu) and its DFT need only partial DFTs:
//   rows    s[f1][m2]  = sum_f2 t[f1][f2] e^{+2 pi i f2 m2 / W}
//   columns u[m1][m2]  = (1/D) sum_f1 s[f1][m2] e^{+2 pi i f1 m1 / H}, scaled
//                        by 1/(2 mu_2p) (real part) and 1/(2 mu_2p+1) (imag)
//   back    r[m1][f2]  = sum_m2 u[m1][m2] e^{-2 pi i f2 m2 / W}
//           U[f1][f2]  = sum_m1 r[m1][f2] e^{-2 pi i f1 m1 / H}
// The row stage runs inside pass A and the last stage inside pass B, so the
// full grids t and U never reach memory.  For real maps the spectrum at -f
// is the conjugate of that at f: a thread that owns f also produces -f from
// the same loads.

constexpr int kPruneMax = 16;  // largest support side handled by the pruned path

// exp(sign 2 pi i k / L) from an LDS copy of the 256-entry table
__device__ __forceinline__ float2 twl(const float2* tw, int k, int L, int sign) {
  float2 w = tw[(k * (256 / L)) & 255];
  if (sign > 0) w.y = -w.y;
  return w;
}

// Canonical half of an H x W spectrum: rows 0..H/2, and w <= W/2 on the
// self-mirrored rows 0 and H/2.  fm is the index of -f.
__device__ __forceinline__ bool canon2(int i, int H, int W, int& f, int& fm) {
  const int lw = __builtin_ctz(W);
  const int h = i >> lw, w = i & (W - 1);
  if (h > H / 2) return false;
  if ((h == 0 || h == H / 2) && w > W / 2) return false;
  f = (h << lw) | w;
  fm = ((((H - h) & (H - 1))) << lw) | ((W - w) & (W - 1));
  return true;
}

// Pass A, the row stage and this row group's share of the column stage.  A
// workgroup of 256 threads owns R = 256/W canonical rows f1 (and their
// mirrors H - f1) of one pair p; every thread forms
// t_k,j = sum_n conj(zhat_k^n) v_j^n at (f1, f2) and, by conjugation, at
// -(f1, f2), pair-packed as t_2p + i t_2p+1.  The block parks the 2R rows in
// LDS, evaluates the 2R x M2 row sums s[row][m2] with g lanes per output, and
// writes its part of the column DFT,
//   Upart[j][p][bx][m1][m2] = sum over its rows of s[row][m2] e^{+2 pi i row m1 / H},
// each of the rows 0 .. H-1 counted by exactly one workgroup.
template <int J>
__global__ __launch_bounds__(256) void l_passA_rows(const float2* __restrict__ Zh, const float2* __restrict__ v,
                                                    float2* __restrict__ Upart, int N, int P, int H, int W, int M1,
                                                    int M2, int g, const int* __restrict__ cgf) {
  if (cgf && cgf[0]) return;
  __shared__ float2 tw[256];
  __shared__ float2 ts[512];  // [slot][f2]; slots R..2R-1 hold the mirrored rows
  __shared__ float2 rsum[2 * 16 * kPruneMax];  // [slot][m2] row sums (zero where a row is not this block's)
  load_twiddles(tw);
  const int lw = __builtin_ctz(W), R = 256 >> lw, D = H * W;
  const int rs = threadIdx.x >> lw, f2 = threadIdx.x & (W - 1);
  const int f1 = blockIdx.x * R + rs;
  const int p = blockIdx.y;
  const bool act = f1 <= H / 2;
  const int f = act ? (f1 << lw) | f2 : 0;
  const int fm = act ? ((((H - f1) & (H - 1))) << lw) | ((W - f2) & (W - 1)) : 0;
  // v are spectra of real signals, so t(-f) = conj(t(f)) for every filter
  // and only v(f) is read
  float2 ta[J], tb[J];
#pragma unroll
  for (int j = 0; j < J; ++j) ta[j] = tb[j] = make_float2(0.f, 0.f);
  if (act) {
    constexpr int U4 = kPassAImgs;
    for (int n = 0; n < N; n += U4) {
      float2 zf[U4], zm[U4], x[U4][J];
#pragma unroll
      for (int u = 0; u < U4; ++u) {
        zf[u] = zm[u] = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < J; ++j) x[u][j] = make_float2(0.f, 0.f);
        if (n + u < N) {
          const float2* zp = Zh + (int64_t(n + u) * P + p) * D;
          zf[u] = zp[f];
          zm[u] = zp[fm];
#pragma unroll
          for (int j = 0; j < J; ++j) x[u][j] = v[(int64_t(n + u) * J + j) * D + f];
        }
      }
#pragma unroll
      for (int u = 0; u < U4; ++u) {
        float2 za, zb;
        unpack_pair(zf[u], zm[u], za, zb);
#pragma unroll
        for (int j = 0; j < J; ++j) {
          ta[j] = cadd(ta[j], cmulc(x[u][j], za));
          tb[j] = cadd(tb[j], cmulc(x[u][j], zb));
        }
      }
    }
  }
  const int O = 2 * R * M2, lanes = g, l = threadIdx.x & (g - 1);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    ts[rs * W + f2] = act ? make_float2(ta[j].x - tb[j].y, ta[j].y + tb[j].x) : make_float2(0.f, 0.f);
    ts[(R + rs) * W + ((W - f2) & (W - 1))] =
        act ? make_float2(ta[j].x + tb[j].y, tb[j].x - ta[j].y) : make_float2(0.f, 0.f);
    __syncthreads();
    // every output slot o = (row slot, m2) takes g lanes, each summing every g-th f2
    for (int ob = threadIdx.x / lanes; ob - threadIdx.x / lanes < O; ob += 256 / lanes) {
      const int o = ob < O ? ob : O - 1;
      const int slot = o / M2, m2 = o % M2;
      // four independent chains over the lane's columns c = l, l + lanes, ...
      float2 a4[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a4[t] = make_float2(0.f, 0.f);
      int c = l;
      for (; c + 3 * lanes < W; c += 4 * lanes) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int cc = c + t * lanes;
          a4[t] = cadd(a4[t], cmul(ts[slot * W + cc], twl(tw, (cc * m2) & (W - 1), W, +1)));
        }
      }
      for (; c < W; c += lanes) a4[0] = cadd(a4[0], cmul(ts[slot * W + c], twl(tw, (c * m2) & (W - 1), W, +1)));
      float2 acc = cadd(cadd(a4[0], a4[1]), cadd(a4[2], a4[3]));
      for (int off = lanes >> 1; off > 0; off >>= 1) {
        acc.x += __shfl_down(acc.x, off, lanes);
        acc.y += __shfl_down(acc.y, off, lanes);
      }
      const int r1 = blockIdx.x * R + (slot < R ? slot : slot - R);
      const bool keep = r1 <= H / 2 && !(slot >= R && (r1 == 0 || r1 == H / 2));
      if (ob < O && l == 0) rsum[slot * M2 + m2] = keep ? acc : make_float2(0.f, 0.f);
    }
    __syncthreads();
    // this block's rows of the column DFT (2R terms per output)
    const int MM = M1 * M2;
    float2* up = Upart + ((int64_t(j) * P + p) * gridDim.x + blockIdx.x) * MM;
    for (int o = threadIdx.x; o < MM; o += 256) {
      const int m1 = o / M2, m2 = o % M2;
      float2 acc = make_float2(0.f, 0.f);
      for (int slot = 0; slot < 2 * R; ++slot) {
        const int r1 = blockIdx.x * R + (slot < R ? slot : slot - R);
        const int row = (slot < R ? r1 : H - r1) & (H - 1);
        acc = cadd(acc, cmul(rsum[slot * M2 + m2], twl(tw, (row * m1) & (H - 1), H, +1)));
      }
      up[o] = acc;
    }
    __syncthreads();
  }
}

// Sum of the column-stage partials of pass A for one (pair, channel) in a
// fixed order, scaled by 1/(D 2 mu) per filter of the pair (u of the support
// projection).  Threads o < M1 M2 hold u[o].
__device__ __forceinline__ float2 sum_upart(const float2* __restrict__ up, int G, int MM, int o, float sa, float sb) {
  float2 a[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) a[t] = make_float2(0.f, 0.f);
  int gi = 0;
  for (; gi + 4 <= G; gi += 4) {
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] = cadd(a[t], up[int64_t(gi + t) * MM + o]);
  }
  for (; gi < G; ++gi) a[0] = cadd(a[0], up[int64_t(gi) * MM + o]);
  const float2 t = cadd(cadd(a[0], a[1]), cadd(a[2], a[3]));
  return make_float2(t.x * sa, t.y * sb);
}

// Back-row and last stages for a slice of kUcCols columns.  A workgroup of
// (slice, pair, channel) sums u (sum_upart), forms the back rows
// r[m1][c] = sum_m2 u[m1][m2] e^{-2 pi i c m2 / W} for the slice's columns
// and their mirrors W - c, and writes Uc[j][p][i] = (U_2p, U_2p+1) at the
// canonical frequencies i = (f1, f2) of the slice (f2 in the slice), pair
// unpacked, with U(f) = sum_m1 r[m1][f2] e^{-2 pi i f1 m1 / H}.
constexpr int kUcCols = 8;  // columns per workgroup of the back-row and last stages
constexpr int kUcAcc = 16;  // partials of pass A loaded together per thread (a power of two)
static_assert((kUcAcc & (kUcAcc - 1)) == 0, "kUcAcc must be a power of two");
__global__ __launch_bounds__(256) void l_prune_uc(const float2* __restrict__ Upart, float4* __restrict__ Uc,
                                                  const float* __restrict__ mu, int K, int P, int H, int W, int M1,
                                                  int M2, int G, const int* __restrict__ cgf) {
  if (cgf && cgf[0]) return;
  __shared__ float2 tw[256];
  __shared__ float2 u[kPruneMax * kPruneMax];
  __shared__ float2 half[kPruneMax * kPruneMax];
  __shared__ float2 rb[kPruneMax * 2 * kUcCols];  // [m1][slot]: slice columns, then their mirrors
  const int p = blockIdx.y, j = blockIdx.z, c0 = blockIdx.x * kUcCols, MM = M1 * M2;
  load_twiddles(tw);
  const float invD = 1.0f / (float)(H * W);
  const float sa = invD / (2.0f * mu[2 * p]);
  const float sb = (2 * p + 1 < K) ? invD / (2.0f * mu[2 * p + 1]) : 0.f;
  const float2* up = Upart + (int64_t(j) * P + p) * G * MM;
  // u = sum of the G partials: with M1 M2 <= 128 the two halves of the
  // workgroup take the even and the odd partials, added in that order into
  // kUcAcc accumulators (as many loads in flight per thread)
  if (MM <= 128) {
    const int o = threadIdx.x & 127, hf = threadIdx.x >> 7;
    float2 a[kUcAcc];
#pragma unroll
    for (int t = 0; t < kUcAcc; ++t) a[t] = make_float2(0.f, 0.f);
    if (o < MM) {
      int gi = hf;
      for (; gi + 2 * (kUcAcc - 1) < G; gi += 2 * kUcAcc) {
#pragma unroll
        for (int t = 0; t < kUcAcc; ++t) a[t] = cadd(a[t], up[int64_t(gi + 2 * t) * MM + o]);
      }
      for (; gi < G; gi += 2) a[0] = cadd(a[0], up[int64_t(gi) * MM + o]);
    }
#pragma unroll
    for (int h = kUcAcc / 2; h > 0; h /= 2)
#pragma unroll
      for (int t = 0; t < h; ++t) a[t] = cadd(a[t], a[t + h]);
    const float2 t = a[0];
    if (hf && o < MM) half[o] = t;
    __syncthreads();
    if (!hf && o < MM) {
      const float2 v = cadd(t, half[o]);
      u[o] = make_float2(v.x * sa, v.y * sb);
    }
  } else {
    for (int o = threadIdx.x; o < MM; o += 256) u[o] = sum_upart(up, G, MM, o, sa, sb);
  }
  __syncthreads();
  constexpr int C2 = 2 * kUcCols;
  for (int q = threadIdx.x; q < M1 * C2; q += 256) {
    const int m1 = q / C2, sl = q % C2;
    const int c = sl < kUcCols ? c0 + sl : (W - c0 - (sl - kUcCols)) & (W - 1);
    float2 a = make_float2(0.f, 0.f);
    for (int m2 = 0; m2 < M2; ++m2) a = cadd(a, cmul(u[m1 * M2 + m2], twl(tw, (c * m2) & (W - 1), W, -1)));
    rb[q] = a;
  }
  __syncthreads();
  // last stage: a thread keeps one column's back rows (and its mirror's) in
  // registers and walks the rows f1 = t, t + 32, ...
  const int lw = __builtin_ctz(W), nc = (H / 2 + 1) * W;
  float4* out = Uc + (int64_t(j) * P + p) * nc;
  const int sl = threadIdx.x % kUcCols, f2 = c0 + sl;
  float2 ra[kPruneMax], rm[kPruneMax];
#pragma unroll
  for (int m1 = 0; m1 < kPruneMax; ++m1) {
    ra[m1] = m1 < M1 ? rb[m1 * C2 + sl] : make_float2(0.f, 0.f);
    rm[m1] = m1 < M1 ? rb[m1 * C2 + kUcCols + sl] : make_float2(0.f, 0.f);
  }
  for (int f1 = threadIdx.x / kUcCols; f1 <= H / 2; f1 += 256 / kUcCols) {
    if ((f1 == 0 || f1 == H / 2) && f2 > W / 2) continue;  // not canonical (canon2)
    float2 a = make_float2(0.f, 0.f), am = make_float2(0.f, 0.f);
#pragma unroll
    for (int m1 = 0; m1 < kPruneMax; ++m1) {
      if (m1 < M1) {
        const float2 w = twl(tw, (f1 * m1) & (H - 1), H, -1);  // at -f: conj(w)
        a = cadd(a, cmul(ra[m1], w));
        am = cadd(am, cmulc(rm[m1], w));
      }
    }
    float2 ua, ub;
    unpack_pair(a, am, ua, ub);
    out[(f1 << lw) | f2] = make_float4(ua.x, ua.y, ub.x, ub.y);
  }
}

// Filter recovery (eq:Learning_Solution) from pass A of gamma and the
// multiplier update (eq:mu_update) in one workgroup per pair p:
// d_k,j[m] = -u_k,j[m] for the two filters of the pair over every channel,
// then ||d_k|| over channels and taps, mu_k <- mu_k ||d_k|| (kept when the
// norm is 0) and, with `project`, d_k <- d_k / max(1, ||d_k||).  A thread
// keeps its (at most one per channel, M1 M2 <= 256) taps in registers.
template <int J>
__global__ __launch_bounds__(256) void l_drec_mu(const float2* __restrict__ Upart, float* __restrict__ mu,
                                                 float* __restrict__ d, int K, int P, int H, int W, int M1, int M2,
                                                 int G, int project) {
  __shared__ double red[256 / 64];
  __shared__ double bc[2];
  const int p = blockIdx.x, MM = M1 * M2, o = threadIdx.x;
  const bool hb = 2 * p + 1 < K;
  const float invD = 1.0f / (float)(H * W);
  const float sa = invD / (2.0f * mu[2 * p]);
  const float sb = hb ? invD / (2.0f * mu[2 * p + 1]) : 0.f;
  float va[J], vb[J];
  double qa = 0.0, qb = 0.0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    va[j] = vb[j] = 0.f;
    if (o < MM) {
      const float2 a = sum_upart(Upart + (int64_t(j) * P + p) * G * MM, G, MM, o, sa, sb);
      va[j] = -a.x;
      vb[j] = -a.y;
      qa += (double)va[j] * va[j];
      qb += (double)vb[j] * vb[j];
    }
  }
  const double ta = block_sum(qa, red);
  if (threadIdx.x == 0) bc[0] = sqrt(ta);
  __syncthreads();
  const double tb = block_sum(qb, red);
  if (threadIdx.x == 0) bc[1] = sqrt(tb);
  __syncthreads();
  const double na = bc[0], nb = bc[1];
  const float ca = (project && na > 1.0) ? (float)(1.0 / na) : 1.f;
  const float cb = (project && nb > 1.0) ? (float)(1.0 / nb) : 1.f;
  if (o < MM) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      d[(int64_t(2 * p) * J + j) * MM + o] = ca == 1.f ? va[j] : va[j] * ca;
      if (hb) d[(int64_t(2 * p + 1) * J + j) * MM + o] = cb == 1.f ? vb[j] : vb[j] * cb;
    }
  }
  if (threadIdx.x == 0) {
    if (na > 0.0) mu[2 * p] = (float)((double)mu[2 * p] * na);
    if (hb && nb > 0.0) mu[2 * p + 1] = (float)((double)mu[2 * p + 1] * nb);
  }
}

// Pass B on the canonical half.  A workgroup of kBW wavefronts owns 64
// canonical frequencies and a chunk of `nbc` images; wavefront w sums the
// pairs p in [w P / kBW, (w+1) P / kBW).  The wavefront partials meet in LDS
// and are added in a fixed order:
//   q^n_j = v^n_j + sum_p (zhat_2p^n U_2p,j + zhat_2p+1^n U_2p+1,j)
// and the value at -f is the conjugate (real maps, real u).  With xh, q
// becomes -x - q.  Dot partials (sum over the block's frequencies of
// Re(v conj q), or |q|^2 with xh, over the block's images) go to
// dots[j nblk + block] with nblk = gridDim.x gridDim.y.
constexpr int kBW = 16;  // pass B: wavefronts per workgroup

template <int J>
constexpr int passb_nb() {
  return J == 1 ? kPassBChunk1 : (J == 2 ? 4 : 2);
}

template <int J>
__global__ __launch_bounds__(64 * kBW) void l_passB_c(const float2* __restrict__ Zh, const float4* __restrict__ Uc,
                                                      const float2* __restrict__ v, float2* __restrict__ q,
                                                      const float2* __restrict__ xh, double* __restrict__ dots,
                                                      double* __restrict__ vdots, int N, int P, int H, int W, int nbc,
                                                      const int* __restrict__ cgf) {
  if (cgf && cgf[0]) return;
  constexpr int NB = passb_nb<J>(), NI = NB * J;  // items per lane: (image, channel)
  __shared__ float2 part[kBW][NI][64];
  __shared__ double wsum[NI], vsum[NI];
  const int D = H * W, nc = (H / 2 + 1) * W;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n0 = blockIdx.y * nbc, nb = min(nbc, N - n0);
  const int i = blockIdx.x * 64 + lane;
  int f = 0, fm = 0;
  const bool own = canon2(i, H, W, f, fm);
  float2 acc[NB][J];
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int j = 0; j < J; ++j) acc[u][j] = make_float2(0.f, 0.f);
  const int p0 = (wv * P) / kBW, p1 = ((wv + 1) * P) / kBW;
  if (own) {
    for (int p = p0; p < p1; ++p) {
      const float2* zp = Zh + (int64_t(n0) * P + p) * D;
      float2 zf[NB], zm[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        zf[u] = zm[u] = make_float2(0.f, 0.f);
        if (u < nb) {
          zf[u] = zp[int64_t(u) * P * D + f];
          zm[u] = zp[int64_t(u) * P * D + fm];
        }
      }
      float4 U[J];
#pragma unroll
      for (int j = 0; j < J; ++j) U[j] = Uc[(int64_t(j) * P + p) * nc + i];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        float2 za, zb;
        unpack_pair(zf[u], zm[u], za, zb);
#pragma unroll
        for (int j = 0; j < J; ++j)
          acc[u][j] = cadd(acc[u][j], cadd(cmul(za, make_float2(U[j].x, U[j].y)), cmul(zb, make_float2(U[j].z, U[j].w))));
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int j = 0; j < J; ++j) part[wv][u * J + j][lane] = acc[u][j];
  __syncthreads();
  const bool self = f == fm;
  for (int it = wv; it < NI; it += kBW) {
    const int j = it % J, u = it / J;
    float2 a = make_float2(0.f, 0.f);
#pragma unroll
    for (int w = 0; w < kBW; ++w) a = cadd(a, part[w][it][lane]);
    double sv = 0.0, s2 = 0.0;
    if (own && u < nb) {
      const int64_t base = (int64_t(n0 + u) * J + j) * D;
      for (int side = 0; side < (self ? 1 : 2); ++side) {
        const int ff = side ? fm : f;
        const float2 vv = v[base + ff];
        float2 qq = cadd(vv, side ? cconj(a) : a);
        if (xh) {
          const float2 x = xh[base + ff];
          qq = make_float2(-x.x - qq.x, -x.y - qq.y);
          sv += (double)qq.x * qq.x + (double)qq.y * qq.y;
        } else {
          sv += (double)vv.x * qq.x + (double)vv.y * qq.y;
          s2 += (double)vv.x * vv.x + (double)vv.y * vv.y;
        }
        q[base + ff] = qq;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      sv += __shfl_down(sv, off, 64);
      s2 += __shfl_down(s2, off, 64);
    }
    if (lane == 0) {
      wsum[it] = sv;
      vsum[it] = s2;
    }
  }
  __syncthreads();
  if (threadIdx.x < J) {
    const int j = threadIdx.x;
    double t = 0.0, t2 = 0.0;
    for (int u = 0; u < nb; ++u) {
      t += wsum[u * J + j];
      t2 += vsum[u * J + j];
    }
    const int64_t o = int64_t(j) * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x;
    dots[o] = t;
    if (vdots) vdots[o] = t2;
  }
}

// One conjugate-gradient step in the arrangement of Chronopoulos and Gear
// (1989), which needs a single reduction phase per step: after the operator
// has produced w = A r, with gamma = |r|^2 and delta = Re<r, w> (partials of
// pass B, fixed-order sums here),
//   beta = gamma / gamma'  (0 on the first step),
//   alpha = gamma / (delta - beta gamma / alpha'),
//   p = r + beta p,  s = w + beta s  (= A p),  x += alpha p,  r -= alpha s,
// where gamma', alpha' are the previous step's (sc_in, [2][J]); block (0,0)
// stores this step's into sc_out.  The iterates are those of the textbook
// recurrence in exact arithmetic.  Tolerance mode: gamma <= tol^2 |x|^2 in
// every channel ends the solve before the update.
template <int J>
__global__ __launch_bounds__(kLW) void l_cg_cg(float2* __restrict__ x, float2* __restrict__ r,
                                               float2* __restrict__ p, float2* __restrict__ s,
                                               const float2* __restrict__ w, const double* __restrict__ dpart,
                                               const double* __restrict__ gpart, int npart,
                                               const double* __restrict__ sc_in, double* __restrict__ sc_out,
                                               int first, int64_t D, int* __restrict__ cgf,
                                               const double* __restrict__ bb, double tol2, int* __restrict__ count) {
  if (cgf && cgf[0]) return;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  const bool lead = blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0;
  const bool in = f < D;
  // the vectors do not depend on the scalars: their loads are issued first
  // and are in flight during the reduction of the partials
  float2 rv[J], wv[J], po[J], so[J], xv[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    rv[j] = wv[j] = po[j] = so[j] = xv[j] = make_float2(0.f, 0.f);
    if (in) {
      const int64_t o = (int64_t(n) * J + j) * D + f;
      rv[j] = r[o];
      wv[j] = w[o];
      xv[j] = x[o];
      if (!first) {
        po[j] = p[o];
        so[j] = s[o];
      }
    }
  }
  double al[J], be[J];
  bool conv = cgf != nullptr;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    // every wavefront sums the partials itself (same order everywhere), so
    // no block-wide barrier stands between the loads and the update
    double gam = 0.0, del = 0.0;
    for (int i = lane; i < npart; i += 64) {
      gam += gpart[int64_t(j) * npart + i];
      del += dpart[int64_t(j) * npart + i];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      gam += __shfl_down(gam, off, 64);
      del += __shfl_down(del, off, 64);
    }
    gam = __shfl(gam, 0, 64);
    del = __shfl(del, 0, 64);
    const double gp = first ? 0.0 : sc_in[j], ap = first ? 0.0 : sc_in[J + j];
    const double b = gp > 0.0 ? gam / gp : 0.0;
    const double den = ap > 0.0 ? del - b * gam / ap : del;
    al[j] = den > 0.0 ? gam / den : 0.0;
    be[j] = b;
    if (lead) {
      sc_out[j] = gam;
      sc_out[J + j] = al[j];
    }
    conv = conv && gam <= tol2 * bb[j];
  }
  if (conv) {
    if (lead) cgf[0] = 1;
    return;
  }
  if (count && lead) count[0] += 1;
  if (in) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int64_t o = (int64_t(n) * J + j) * D + f;
      const float a = (float)al[j], b = (float)be[j];
      float2 pp = rv[j], ss = wv[j];
      if (!first) {
        pp = make_float2(fmaf(b, po[j].x, rv[j].x), fmaf(b, po[j].y, rv[j].y));
        ss = make_float2(fmaf(b, so[j].x, wv[j].x), fmaf(b, so[j].y, wv[j].y));
      }
      p[o] = pp;
      s[o] = ss;
      x[o] = make_float2(fmaf(a, pp.x, xv[j].x), fmaf(a, pp.y, xv[j].y));
      r[o] = make_float2(fmaf(-a, ss.x, rv[j].x), fmaf(-a, ss.y, rv[j].y));
    }
  }
}

// bb[j] = sum over images and frequencies of |xhat_j|^2 (one workgroup per
// channel, fixed order): the reference of the CG stopping rule.
__global__ __launch_bounds__(kLW) void l_norm2(const float2* __restrict__ xh, double* __restrict__ bb, int N, int J,
                                               int64_t D) {
  __shared__ double red[kLW / 64];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int n = 0; n < N; ++n)
    for (int64_t f = threadIdx.x; f < D; f += kLW) {
      const float2 x = xh[(int64_t(n) * J + j) * D + f];
      s += (double)x.x * x.x + (double)x.y * x.y;
    }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) bb[j] = t;
}

// start of a multiplier step in tolerance mode: clear the flag and the count
__global__ void l_cg_reset(int* __restrict__ cgf, int* __restrict__ count) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cgf[0] = 0;
    if (count) count[0] = 0;
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

static bool pruned2d(const Plan& pl) {
  return pl.g[0] == 1 && pl.fs[1] <= kPruneMax && pl.fs[2] <= kPruneMax;
}

// 64-frequency blocks covering the canonical half of the spectrum
static unsigned canon_blocks(const Plan& pl) { return lblk(int64_t(pl.g[1] / 2 + 1) * pl.g[2], 64); }

static int pow2_floor(int x) {
  int r = 1;
  while (2 * r <= x) r *= 2;
  return r;
}

// lanes per output for `outs` outputs of `len`-term sums on 256 threads
static int lanes_for(int outs, int len) { return std::max(1, std::min(std::min(64, len), pow2_floor(256 / outs))); }

static int passb_nb_host(int J) { return J == 1 ? kPassBChunk1 : (J == 2 ? 4 : 2); }
static int passb_chunks(const Plan& pl) { return (pl.n + passb_nb_host(pl.j) - 1) / passb_nb_host(pl.j); }

// pass-A row groups of the pruned path (R = 256 / W canonical rows each)
static int passa_groups(const Plan& pl) {
  const int H = pl.g[1], R = 256 / pl.g[2];
  return (H / 2 + R) / R;
}

static int dot_parts(const Plan& pl) {
  return pruned2d(pl) ? (int)canon_blocks(pl) * passb_chunks(pl) : pl.n * (int)lblk(pl.dsz);
}

struct LearnWs {
  float2 *Zh, *xh, *gh, *rh, *ph, *qh, *sh, *Tp, *Upart;
  float4* Uc;   // pruned path: U at the canonical frequencies, pair unpacked
  double *dots, *rr;  // dots: pass-B partials of Re<r, A r>, then of |r|^2; rr: two [2][J] CG scalar sets
  double* bb;         // tolerance mode: |xhat_j|^2 per channel
  int* cgf;           // tolerance mode: CG stop flag of the current multiplier step
  int nB;  // pruned path: pass-B partials per channel (one per workgroup)
  int npartB, npartS;  // partial counts per channel: pass B, vector-update kernel
  void* span;          // span-form workspace (eligible plans), else NULL
};

static size_t carve_learn(const Plan& pl, void* base, LearnWs* w) {
  Carver c(base);
  const int64_t D = pl.dsz, N = pl.n, J = pl.j, P = pl.p;
  w->npartB = dot_parts(pl);
  w->npartS = int(N * lblk(D));
  w->Zh = c.take<float2>(N * P * D);
  w->xh = c.take<float2>(N * J * D);
  w->gh = c.take<float2>(N * J * D);
  w->rh = c.take<float2>(N * J * D);
  w->ph = c.take<float2>(N * J * D);
  w->qh = c.take<float2>(N * J * D);
  w->sh = c.take<float2>(N * J * D);
  w->Tp = c.take<float2>(J * P * D);
  w->Upart = c.take<float2>(J * P * int64_t(passa_groups(pl)) * pl.fs[1] * pl.fs[2]);
  w->Uc = c.take<float4>(J * P * int64_t(pl.g[1] / 2 + 1) * pl.g[2]);
  w->dots = c.take<double>(J * (int64_t(w->npartB) + std::max(w->npartB, w->npartS)));
  w->rr = c.take<double>(4 * J);
  w->bb = c.take<double>(J);
  w->cgf = c.take<int>(1);
  w->nB = (int)canon_blocks(pl) * passb_chunks(pl);
  w->span = span_eligible(pl) ? c.take<char>(span_ws_bytes(pl)) : nullptr;
  return c.off;
}

size_t run_learn_ws(const Plan& pl) {
  LearnWs w;
  return carve_learn(pl, nullptr, &w);
}

static bool crop_tile_launch(const Plan& pl, float2* Tp, const float* mu, hipStream_t st, const int* cgf) {
  if (!(pl.g[0] == 1 && tile_supported(pl.g[1], pl.g[2]))) return false;
  const dim3 grid(pl.p, pl.j);
  const int h = pl.g[1], w = pl.g[2];
#define CT(HH, WW)                                                                                             \
  if (h == HH && w == WW) {                                                                                    \
    hipLaunchKernelGGL((l_crop_tile<HH, WW>), grid, dim3(lt_threads(HH * WW)), 0, st, Tp, mu, pl.k, pl.p,      \
                       pl.fs[1], pl.fs[2], cgf);                                                               \
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

// ------------------------------------------------ pruned operator (host)
// U for A v: pass A with the row stage and the column-stage partials, then
// the back-row and last stages into Uc.
// With `have_upart` the column-stage partials of v are already in w.Upart
// (pass A of the same v and code spectra ran last) and pass A is skipped.
static hipError_t pruned_zt_proj(const Plan& pl, LearnWs& w, const float2* v, const float* mu, hipStream_t st,
                                 const int* cgf, bool have_upart = false) {
  const int H = pl.g[1], W = pl.g[2], R = 256 / W, M1 = pl.fs[1], M2 = pl.fs[2], G = passa_groups(pl);
  if (!have_upart) {
    TraceScope trace(kTraceLearnA, st, true);
    LAUNCH_J_TRACED(trace, l_passA_rows, pl.j, dim3(G, pl.p), dim3(256), st, w.Zh, v, w.Upart, pl.n, pl.p, H, W, M1, M2,
       lanes_for(2 * R * M2, W), cgf);
  }
  hipLaunchKernelGGL(l_prune_uc, dim3(W / kUcCols, pl.p, pl.j), dim3(256), 0, st, w.Upart, w.Uc, mu, pl.k, pl.p, H,
                     W, M1, M2, G, cgf);
  return hipGetLastError();
}

// d_k = -S Z_k^T gamma / (2 mu_k) through pass A and the column stage, then
// the multiplier update (and with `project` the unit-ball projection).
static hipError_t pruned_drecover(const Plan& pl, LearnWs& w, float* mu, float* d, bool project, hipStream_t st) {
  const int H = pl.g[1], W = pl.g[2], R = 256 / W, M1 = pl.fs[1], M2 = pl.fs[2], G = passa_groups(pl);
  {
    TraceScope trace(kTraceLearnA, st, true);
    LAUNCH_J_TRACED(trace, l_passA_rows, pl.j, dim3(G, pl.p), dim3(256), st, w.Zh, w.gh, w.Upart, pl.n, pl.p, H, W, M1, M2,
       lanes_for(2 * R * M2, W), nullptr);
  }
  LJ(l_drec_mu, pl.j, dim3(pl.p), dim3(256), st, w.Upart, mu, d, pl.k, pl.p, H, W, M1, M2, G, project ? 1 : 0);
  return hipGetLastError();
}

// q = v + Z U (pass B); with xh: q = -x - (v + Z U).  Partials ([J][nB]) of
// Re<v, q> (|q|^2 with xh) to `part`, of |v|^2 to `vpart` if given.
static void pruned_passB(const Plan& pl, LearnWs& w, const float2* v, float2* q, const float2* xh, double* part,
                         double* vpart, hipStream_t st, const int* cgf) {
  const int chunks = passb_chunks(pl), nbc = (pl.n + chunks - 1) / chunks;
  TraceScope trace(kTraceLearnB, st, true);
  LAUNCH_J_TRACED(trace, l_passB_c, pl.j, dim3(canon_blocks(pl), chunks), dim3(64 * kBW), st, w.Zh, w.Uc, v, q, xh, part, vpart, pl.n,
     pl.p, pl.g[1], pl.g[2], nbc, cgf);
}

// Up <- DFT(S^T S IDFT(pass A of v) / (2 mu)).
// (With cgf set the kernels skip their work; the axis FFTs of the general
// path still run on the stale buffer, whose result is then not used.)
static hipError_t apply_zt_proj(const Plan& pl, LearnWs& w, const float2* v, const float* mu, hipStream_t st,
                                const int* cgf) {
  const int64_t D = pl.dsz;
  const int T = pl.g[0], H = pl.g[1], W = pl.g[2];
  {
    TraceScope trace(kTraceLearnA, st, true);
    LAUNCH_J_TRACED(trace, l_passA, pl.j, dim3(lblk(D), pl.p), dim3(kLW), st, w.Zh, v, w.Tp, pl.n, pl.p, T, H, W, cgf);
  }
  if (crop_tile_launch(pl, w.Tp, mu, st, cgf)) return hipGetLastError();
  hipError_t e = fft_grids(w.Tp, int64_t(pl.j) * pl.p, pl.g, +1, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(l_crop_scale, dim3(lblk(D), pl.p, pl.j), dim3(kLW), 0, st, w.Tp, mu, pl.k, pl.p, T, H, W,
                     pl.fs[0], pl.fs[1], pl.fs[2], cgf);
  return fft_grids(w.Tp, int64_t(pl.j) * pl.p, pl.g, -1, st);
}

// q = v + Z Up (pass B); with xh: q = -x - (v + Z Up).  Dot partials to
// dots (and of |v|^2 to vdots if given), as pruned_passB.
static void apply_passB(const Plan& pl, LearnWs& w, const float2* v, float2* q, const float2* xh, double* dots,
                        double* vdots, hipStream_t st, const int* cgf) {
  const int T = pl.g[0], H = pl.g[1], W = pl.g[2];
  TraceScope trace(kTraceLearnB, st, true);
  LAUNCH_J_TRACED(trace, l_passB, pl.j, dim3(lblk(pl.dsz), pl.n), dim3(kLW), st, w.Zh, w.Tp, v, q, xh, dots, vdots, pl.n, pl.p, T, H,
     W, cgf);
}

int run_learn(const Plan& pl, const float* b, const float* z, float* d, float* mu, float* gamma, int inner_iters,
              int cg_iters, unsigned flags, void* ws, hipStream_t st, float cg_tol, int* cg_counts) {
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
  double* rrp = w.dots + J * w.npartB;
  const bool pruned = pruned2d(pl);
  // tolerance mode: each multiplier step's CG stops once |r| <= cg_tol |x|
  // in every channel (relative residual of A gamma = -x); the remaining
  // launches of that solve check the flag and return at once
  const bool tol_mode = cg_tol > 0.0f;
  int* cgf = tol_mode ? w.cgf : nullptr;
  const double tol2 = (double)cg_tol * (double)cg_tol;
  if (tol_mode) hipLaunchKernelGGL(l_norm2, dim3((unsigned)J), dim3(kLW), 0, st, w.xh, w.bb, (int)N, (int)J, D);
  const int npB = pruned ? w.nB : w.npartB;
  // span form (fixed CG counts, no per-step counts asked for): gamma ends in
  // gh as pass B of its filter-space part onto a xhat + b gammahat_0
  const bool span = pruned && w.span && !tol_mode && !cg_counts && !(flags & CSC_LEARN_DIRECT) &&
                    ((flags & CSC_LEARN_SPAN) || span_preferred(pl, inner_iters, cg_iters));
  if (span) {
    if (run_span(pl, w.Zh, w.xh, w.gh, w.rh, w.Uc, d, mu, inner_iters, cg_iters, w.span, st) != hipSuccess)
      return CSC_EHIP;
    pruned_passB(pl, w, w.rh, w.gh, nullptr, w.dots, nullptr, st, nullptr);
  }
  // the operator A v = v + sum_k 1/(2 mu_k) Z_k S^T S Z_k^T v into q (with xh:
  // q = -x - A v), dot partials as pruned_passB
  auto apply_A = [&](const float2* v, float2* q, const float2* xh, double* part, double* vpart,
                     bool have_upart = false) -> hipError_t {
    hipError_t err;
    if (pruned) {
      if ((err = pruned_zt_proj(pl, w, v, mu, st, cgf, have_upart)) != hipSuccess) return err;
      pruned_passB(pl, w, v, q, xh, part, vpart, st, cgf);
    } else {
      if ((err = apply_zt_proj(pl, w, v, mu, st, cgf)) != hipSuccess) return err;
      apply_passB(pl, w, v, q, xh, part, vpart, st, cgf);
    }
    return hipGetLastError();
  };
  for (int it = 0; !span && it < inner_iters; ++it) {
    int* cnt = cg_counts ? cg_counts + it : nullptr;
    if (tol_mode) hipLaunchKernelGGL(l_cg_reset, dim3(1), dim3(64), 0, st, cgf, cnt);
    else if (cnt) hipLaunchKernelGGL(l_cg_reset, dim3(1), dim3(64), 0, st, w.cgf, cnt);
    // r = -x - A gamma, then per step w = A r and the update (l_cg_cg).
    // After the first multiplier step, pass A of gamma is the one the
    // filter recovery just ran (same gamma, same code spectra).
    if ((e = apply_A(w.gh, w.rh, w.xh, rrp, nullptr, pruned && it > 0)) != hipSuccess) return CSC_EHIP;
    double* sc_in = w.rr;
    double* sc_out = w.rr + 2 * J;
    for (int q = 0; q < cg_iters; ++q) {
      if ((e = apply_A(w.rh, w.qh, nullptr, pap, rrp)) != hipSuccess) return CSC_EHIP;
      LJ(l_cg_cg, pl.j, vgrid, dim3(kLW), st, w.gh, w.rh, w.ph, w.sh, w.qh, pap, rrp, npB, sc_in, sc_out,
         q == 0 ? 1 : 0, D, cgf, w.bb, tol2, cnt);
      double* t = sc_in;
      sc_in = sc_out;
      sc_out = t;
    }
    // d_k = -S Z_k^T gamma / (2 mu_k) ; mu_k <- mu_k ||d_k||
    const bool last = it == inner_iters - 1;
    if (pruned) {
      if ((e = pruned_drecover(pl, w, mu, d, last, st)) != hipSuccess) return CSC_EHIP;
    } else {
      LJ(l_passA, pl.j, dim3(lblk(D), pl.p), dim3(kLW), st, w.Zh, w.gh, w.Tp, pl.n, pl.p, T, H, W, nullptr);
      if ((e = fft_grids(w.Tp, J * pl.p, pl.g, +1, st)) != hipSuccess) return CSC_EHIP;
      hipLaunchKernelGGL(l_drecover, dim3(lblk(pl.msz), pl.k, pl.j), dim3(kLW), 0, st, w.Tp, mu, d, pl.k, pl.j,
                         pl.p, T, H, W, pl.fs[0], pl.fs[1], pl.fs[2]);
      hipLaunchKernelGGL(l_mu_update, dim3(pl.k), dim3(kLW), 0, st, d, mu, int64_t(J) * pl.msz, 1, last ? 1 : 0);
    }
  }
  // gamma back to the spatial domain (in place: its spectrum is not needed
  // after this)
  if ((e = fft_grids(w.gh, N * J, pl.g, +1, st)) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(l_complex_to_real, dim3(lblk(ns)), dim3(kLW), 0, st, w.gh, gamma, ns, 1.0f / (float)D);
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

}  // namespace dcsc
