// DCT-domain variant of the coding subproblem (symmetric boundaries).  Sec. 3
// notes that the DCT can take the DFT's place where the circular boundary
// is a problem.  Images and code maps are extended half-sample symmetrically
// at both ends of each axis, and the filters are whole-sample symmetric about
// their centre, given by one quadrant q [K][J][M1][M2] (h[m1][m2] =
// q[|m1|][|m2|]).  The 2-D DCT-II then diagonalises every convolution with
// real eigenvalues
//   hhat[k1][k2] = sum_{m1,m2} a(m1) a(m2) q[m1][m2] cos(pi k1 m1/H) cos(pi k2 m2/W),
// a(0) = 1, a(m > 0) = 2, and the updates of eq:Inference_solution carry over
// with the DCT in place of the DFT and no conjugates.  The loop keeps the
// implicit-theta form of the Fourier path (yhat = DCT(D z), Thhat = DCT(D theta)
// per image, real), and one iteration is
//   lam'   = (G + I/rho)^-1 (Thhat + (yhat - xhat)/rho)       [k_dct_spec/solve]
//   z'     = soft(z - rho D^T lam', rho beta)                  [k_dct_tile]
//   yhat'  = DCT(D z'),  Thhat' = G lam' + (yhat' - yhat)/rho  [k_dct_tile + k_dct_spec]
//
// Transforms.  Two real maps travel as one complex map (z_2p + i z_2p+1);
// the DCT is real-linear, so the complex transform of the pair is the pair of
// transforms.  Along an axis of length N the unnormalised DCT-II
// X[k] = sum_n x[n] cos(pi k (2n + 1) / 2N) is computed from an N-point FFT
// (Makhoul 1980): v[n] = x[2n], v[N-1-n] = x[2n+1], V = FFT(v),
//   X[k] = (w_k V[k] + conj(w_k) V[N-k]) / 2,   w_k = exp(-i pi k / 2N),
// a form without conjugates of V that holds for complex data; the inverse is
//   V[k] = conj(w_k) (X[k] - i X[N-k]) (X[N] = 0),  v = IFFT(V),
// and x[2n] = v[n], x[2n+1] = v[N-1-n].  The tile keeps the maps in the
// permuted order v, so the soft-threshold step reads and writes z at the
// permuted positions and no permutation pass is needed.
//
// Parseval for the unnormalised DCT-II: sum_n x[n]^2 = sum_k a(k) X[k]^2 / N
// per axis, which weights the dual residual and the objective.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace dcsc {

constexpr int kDE = 256;  // threads of the elementwise kernels

static unsigned eblk(int64_t n) { return (unsigned)((n + kDE - 1) / kDE); }

constexpr int dct_threads(int t) { return t >= 16384 ? 1024 : (t >= 8192 ? 512 : (t >= 4096 ? 256 : 128)); }

// tile position of natural index x along an axis of length N (the inverse of
// the Makhoul permutation)
__device__ __forceinline__ int perm_slot(int x, int N) { return (x & 1) ? N - 1 - (x >> 1) : (x >> 1); }

// Parseval weight a(k1) a(k2) of frequency f = k1 W + k2
__device__ __forceinline__ float dct_weight(int64_t f, int W) {
  const int k1 = (int)(f / W), k2 = (int)(f % W);
  return (k1 ? 2.f : 1.f) * (k2 ? 2.f : 1.f);
}

// ---------------------------------------------------------------- set-up

// E[j][p][f] = (hhat_j,2p(f), hhat_j,2p+1(f)), the eigenvalues of the pair
// (direct cosine sums, float64).
__global__ void k_dct_eig(const float* __restrict__ q, float2* __restrict__ E, int K, int J, int P, int H, int W,
                          int M1, int M2) {
  const int64_t D = int64_t(H) * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, j = blockIdx.z;
  if (f >= D) return;
  const int k1 = (int)(f / W), k2 = (int)(f % W);
  double c2[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) c2[m] = m < M2 ? (m ? 2.0 : 1.0) * cospi((double)k2 * m / W) : 0.0;
  double s[2] = {0.0, 0.0};
  for (int m1 = 0; m1 < M1; ++m1) {
    const double c1 = (m1 ? 2.0 : 1.0) * cospi((double)k1 * m1 / H);
    for (int h = 0; h < 2; ++h) {
      const int k = 2 * p + h;
      if (k >= K) continue;
      const float* qk = q + ((int64_t(k) * J + j) * M1 + m1) * M2;
      double r = 0.0;
#pragma unroll
      for (int m2 = 0; m2 < 16; ++m2)
        if (m2 < M2) r += c2[m2] * (double)qk[m2];
      s[h] += c1 * r;
    }
  }
  E[(int64_t(j) * P + p) * D + f] = make_float2((float)s[0], (float)s[1]);
}

// G_f = sum_k hhat_.k(f) hhat_.k(f)^T (real J x J, stored complex with zero
// imaginary parts for dual_solve), float64 sums.
template <int J>
__global__ void k_dct_gram(const float2* __restrict__ E, float2* __restrict__ G, int P, int64_t D) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= D) return;
  double g[J][J];
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int c = 0; c < J; ++c) g[a][c] = 0.0;
  for (int p = 0; p < P; ++p) {
    float2 e[J];
#pragma unroll
    for (int j = 0; j < J; ++j) e[j] = E[(int64_t(j) * P + p) * D + f];
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int c = 0; c < J; ++c) g[a][c] += (double)e[a].x * e[c].x + (double)e[a].y * e[c].y;
  }
#pragma unroll
  for (int a = 0; a < J; ++a)
#pragma unroll
    for (int c = 0; c < J; ++c) G[(f * J + a) * J + c] = make_float2((float)g[a][c], 0.f);
}

// ------------------------------------------------------ tile transforms

// Quarter-wave factors w_k = exp(-i pi k / 2N), k < N, for both axes.
template <int H, int W>
__device__ __forceinline__ void load_quarter(float2* qh, float2* qw) {
  for (int i = threadIdx.x; i < H + W; i += blockDim.x) {
    const int N = i < H ? H : W, k = i < H ? i : i - H;
    double sn, cs;
    sincospi((double)k / (2.0 * N), &sn, &cs);
    (i < H ? qh : qw)[k] = make_float2((float)cs, (float)-sn);
  }
}

// In-place combine along the columns (length H) for every tile column:
// forward X[k] = (w V[k] + conj(w) V[H-k]) / 2, or inverse pre-twiddle
// V[k] = conj(w) (X[k] - i X[H-k]) (X[H] = 0).  Ends synchronised.
template <int H, int W, int WP, int NT, bool FWD>
__device__ __forceinline__ void combine_cols(float2* tile, const float2* qh) {
  constexpr int JOBS = (H / 2 + 1) * W;
  for (int job = threadIdx.x; job < JOBS; job += NT) {
    const int k = job / W, c = job % W;
    const int km = (H - k) & (H - 1);
    float2 a = tile[k * WP + c], b = tile[km * WP + c];
    const float2 wk = qh[k], wm = qh[km];
    if (FWD) {
      const float2 ra = cscale(cadd(cmul(wk, a), cmul(cconj(wk), b)), 0.5f);
      const float2 rb = cscale(cadd(cmul(wm, b), cmul(cconj(wm), a)), 0.5f);
      tile[k * WP + c] = ra;
      if (km != k) tile[km * WP + c] = rb;
    } else {
      // X[H] = 0: the k = 0 row keeps its value
      const float2 ra = k == 0 ? a : cmul(cconj(wk), csub(a, mul_i<1>(b)));
      const float2 rb = cmul(cconj(wm), csub(b, mul_i<1>(a)));
      tile[k * WP + c] = ra;
      if (km != k) tile[km * WP + c] = rb;
    }
  }
  __syncthreads();
}

enum { kDctIter = 0, kDctForward = 1, kDctImage = 2 };

// One workgroup per (pair group g, image n) (kDctImage: per (image, channel)).
// kDctIter: for every pair of the group, V = sum_j lam_j E_jp, inverse 2-D
// DCT, soft-threshold step (z in place, optional theta, residual partial),
// forward 2-D DCT, part[n][g][j] += E_jp . C (real).  kDctForward: forward
// DCT of the given maps and the accumulation (l1 partials).  kDctImage:
// xh[n][j] = DCT(b[n][j]).
template <int H, int W, int J, int MODE>
__global__ __launch_bounds__(dct_threads(H * W)) void k_dct_tile(
    const float2* __restrict__ E, const float* __restrict__ lam, float* __restrict__ z, float* __restrict__ theta,
    const float* __restrict__ rho_cur, float beta, float* __restrict__ part, double* __restrict__ rpart, int K, int P,
    int ppg, int ng, const float* __restrict__ img, float* __restrict__ xh) {
  constexpr int D = H * W, NT = dct_threads(D), WP = W + 1;
  __shared__ float2 tile[H * WP];
  __shared__ float2 tw[256];
  __shared__ float2 qh[H], qw[W];
  __shared__ double red[NT / 64];
  load_twiddles(tw);
  load_quarter<H, W>(qh, qw);
  const int tid = (int)threadIdx.x;
  if constexpr (MODE == kDctImage) {
    const int nj = blockIdx.x;  // image n, channel j
    __syncthreads();
    for (int e = tid; e < D; e += NT) {
      const int h = e / W, w = e % W;
      tile[perm_slot(h, H) * WP + perm_slot(w, W)] = make_float2(img[int64_t(nj) * D + e], 0.f);
    }
    __syncthreads();
    fft_lines<H, D, NT, -1, WP, 1>(tile, tw);
    combine_cols<H, W, WP, NT, true>(tile, qh);
    fft_lines<W, D, NT, -1, 1, WP>(tile, tw);
    for (int e = tid; e < D; e += NT) {
      const int k1 = e / W, k2 = e % W, km = (W - k2) & (W - 1);
      const float2 x = cscale(cadd(cmul(qw[k2], tile[k1 * WP + k2]), cmul(cconj(qw[k2]), tile[k1 * WP + km])), 0.5f);
      xh[int64_t(nj) * D + e] = x.x;
    }
    return;
  }
  const int N = (int)(gridDim.x / ng), item = xcd_item((int)blockIdx.x, (int)gridDim.x);
  const int g = item / N, n = item % N;
  const float rho = MODE == kDctIter ? rho_cur[n] : 1.0f;
  const float thr = rho * beta, inv_rho = 1.0f / rho, invD = 1.0f / (float)D;
  const int p0 = g * ppg, p1 = min(P, p0 + ppg);
  float* mypart = part + (int64_t(n) * ng + g) * J * D;
  const float* lamn = lam + int64_t(n) * J * D;
  double rsum = 0.0;
  for (int p = p0; p < p1; ++p) {
    const int ka = 2 * p, kb = 2 * p + 1;
    const bool hb = kb < K;
    float* za = z + (int64_t(n) * K + ka) * D;
    float* zb = z + (int64_t(n) * K + (hb ? kb : ka)) * D;
    const float2* Ep[J];
#pragma unroll
    for (int c = 0; c < J; ++c) Ep[c] = E + (int64_t(c) * P + p) * D;
    __syncthreads();  // the previous pair's readers of the tile are done
    if constexpr (MODE == kDctIter) {
      // V = sum_j lam_j E_jp, with the inverse pre-twiddle along the rows
      for (int e = tid; e < D; e += NT) {
        const int k1 = e / W, k2 = e % W;
        const int em = k1 * W + ((W - k2) & (W - 1));
        float2 x = make_float2(0.f, 0.f), xm = make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < J; ++c) {
          x = cadd(x, cscale(Ep[c][e], lamn[c * D + e]));
          xm = cadd(xm, cscale(Ep[c][em], lamn[c * D + em]));
        }
        if (k2 == 0) xm = make_float2(0.f, 0.f);
        tile[k1 * WP + k2] = cmul(cconj(qw[k2]), csub(x, mul_i<1>(xm)));
      }
      __syncthreads();
      fft_lines<W, D, NT, 1, 1, WP>(tile, tw);
      combine_cols<H, W, WP, NT, false>(tile, qh);
      fft_lines<H, D, NT, 1, WP, 1>(tile, tw);
      // soft-threshold step at natural positions (tile at permuted slots)
      float* tha = theta ? theta + (int64_t(n) * K + ka) * D : nullptr;
      float* thb = theta ? theta + (int64_t(n) * K + (hb ? kb : ka)) * D : nullptr;
      for (int e = tid; e < D; e += NT) {
        const int h = e / W, w = e % W;
        float2* slot = tile + perm_slot(h, H) * WP + perm_slot(w, W);
        const float2 c = *slot;
        const float va = c.x * invD, vb = c.y * invD;
        const float a0 = za[e], b0 = hb ? zb[e] : 0.f;
        const float a1 = soft_thresh(fmaf(-rho, va, a0), thr);
        const float b1 = hb ? soft_thresh(fmaf(-rho, vb, b0), thr) : 0.f;
        const float da = a1 - a0, db = b1 - b0;
        rsum += (double)fmaf(da, da, db * db);
        za[e] = a1;
        if (hb) zb[e] = b1;
        if (tha) {
          tha[e] = va + da * inv_rho;
          if (hb) thb[e] = vb + db * inv_rho;
        }
        *slot = make_float2(a1, b1);
      }
    } else {
      for (int e = tid; e < D; e += NT) {
        const int h = e / W, w = e % W;
        const float a0 = za[e], b0 = hb ? zb[e] : 0.f;
        rsum += (double)fabsf(a0) + (double)fabsf(b0);
        tile[perm_slot(h, H) * WP + perm_slot(w, W)] = make_float2(a0, b0);
      }
    }
    __syncthreads();
    fft_lines<H, D, NT, -1, WP, 1>(tile, tw);
    combine_cols<H, W, WP, NT, true>(tile, qh);
    fft_lines<W, D, NT, -1, 1, WP>(tile, tw);
    // the last combine along the rows, then part += E_jp . C
    for (int e = tid; e < D; e += NT) {
      const int k1 = e / W, k2 = e % W, km = (W - k2) & (W - 1);
      const float2 cc =
          cscale(cadd(cmul(qw[k2], tile[k1 * WP + k2]), cmul(cconj(qw[k2]), tile[k1 * WP + km])), 0.5f);
#pragma unroll
      for (int c = 0; c < J; ++c) {
        const float2 ee = Ep[c][e];
        const float y = fmaf(ee.x, cc.x, ee.y * cc.y);
        float* dst = mypart + int64_t(c) * D + e;
        *dst = (p == p0) ? y : *dst + y;
      }
    }
  }
  if (p0 >= p1) {
    for (int e = tid; e < D; e += NT)
      for (int c = 0; c < J; ++c) mypart[int64_t(c) * D + e] = 0.f;
  }
  const double tot = block_sum(rsum, red);
  if (threadIdx.x == 0) rpart[int64_t(n) * ng + g] = tot;
}

// ------------------------------------------------------- spectral kernels

// lam = (G + I/rho)^-1 (Thhat + (yhat - xhat)/rho) per image and frequency.
template <int J>
__global__ void k_dct_solve(const float2* __restrict__ G, const float* __restrict__ xh, const float* __restrict__ yh,
                            const float* __restrict__ Th, const float* __restrict__ rho_cur, float* __restrict__ lam,
                            int64_t D) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (f >= D) return;
  const float inv_rho = 1.0f / rho_cur[n];
  float2 r[J], l[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t o = (int64_t(n) * J + j) * D + f;
    r[j] = make_float2(Th[o] + (yh[o] - xh[o]) * inv_rho, 0.f);
  }
  dual_solve<J>(G + f * J * J, inv_rho, r, l);
#pragma unroll
  for (int j = 0; j < J; ++j) lam[(int64_t(n) * J + j) * D + f] = l[j].x;
}

// yhat' = sum of the groups of part, Thhat' = G lam + (yhat' - yhat)/rho,
// dual-residual partials sum a(k1) a(k2) (Thhat' - Thhat)^2 and, with a fixed
// step, the next lam.  mode 1 (set-up): dst = sum of the groups only.
template <int J>
__global__ __launch_bounds__(kDE) void k_dct_spec(const float* __restrict__ part, const float2* __restrict__ G,
                                                  const float* __restrict__ xh, float* __restrict__ yh,
                                                  float* __restrict__ Th, float* __restrict__ lam,
                                                  const float* __restrict__ rho_cur, double* __restrict__ rdual,
                                                  int ng, int W, int64_t D, int solve_next, float* __restrict__ dst) {
  __shared__ double red[kDE / 64];
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  double ds = 0.0;
  if (f < D) {
    float ys[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const float* pp = part + (int64_t(n) * ng * J + j) * D + f;
      float s = 0.f;
      for (int gg = 0; gg < ng; ++gg) s += pp[int64_t(gg) * J * D];
      ys[j] = s;
    }
    if (dst) {
#pragma unroll
      for (int j = 0; j < J; ++j) dst[(int64_t(n) * J + j) * D + f] = ys[j];
    } else {
      const float inv_rho = 1.0f / rho_cur[n];
      const float2* Gf = G + f * J * J;
      float thn[J];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        float gl = 0.f;
#pragma unroll
        for (int c = 0; c < J; ++c) gl = fmaf(Gf[j * J + c].x, lam[(int64_t(n) * J + c) * D + f], gl);
        const int64_t o = (int64_t(n) * J + j) * D + f;
        thn[j] = gl + (ys[j] - yh[o]) * inv_rho;
        const double dd = (double)thn[j] - Th[o];
        ds += dd * dd;
        yh[o] = ys[j];
        Th[o] = thn[j];
      }
      ds *= (double)dct_weight(f, W);
      if (solve_next) {
        float2 r[J], l[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const int64_t o = (int64_t(n) * J + j) * D + f;
          r[j] = make_float2(thn[j] + (ys[j] - xh[o]) * inv_rho, 0.f);
        }
        dual_solve<J>(Gf, inv_rho, r, l);
#pragma unroll
        for (int j = 0; j < J; ++j) lam[(int64_t(n) * J + j) * D + f] = l[j].x;
      }
    }
  }
  if (rdual) {
    const double t = block_sum(ds, red);
    if (threadIdx.x == 0) rdual[int64_t(n) * gridDim.x + blockIdx.x] = t;
  }
}

// opart[n][blk] = sum_f a(k1) a(k2) sum_j (xhat_j - yhat_j)^2, yhat = sum of part
template <int J>
__global__ __launch_bounds__(kDE) void k_dct_obj(const float* __restrict__ part, const float* __restrict__ xh,
                                                 double* __restrict__ opart, int ng, int W, int64_t D) {
  __shared__ double red[kDE / 64];
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  double s = 0.0;
  if (f < D) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const float* pp = part + (int64_t(n) * ng * J + j) * D + f;
      double y = 0.0;
      for (int gg = 0; gg < ng; ++gg) y += pp[int64_t(gg) * J * D];
      const double r = (double)xh[(int64_t(n) * J + j) * D + f] - y;
      s += r * r;
    }
    s *= (double)dct_weight(f, W);
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) opart[int64_t(n) * gridDim.x + blockIdx.x] = t;
}

__global__ void k_dct_fill(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_dct_copy(float* __restrict__ dst, const float* __restrict__ src, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ================================================================== host

bool dct_supported(int T, int H, int W) {
  auto ok = [](int v) { return v >= 8 && v <= 128 && (v & (v - 1)) == 0; };
  return T == 1 && ok(H) && ok(W) && int64_t(H) * W <= kTileMax;
}

namespace {

struct DctWs {
  float2 *E, *G;
  float *xh, *yh, *Th, *lam, *part;
  double *rpri, *rdual, *opart;
  float* rho;
  int ng, ppg;
};

void dct_grouping(const Plan& pl, int& ppg, int& ng) {
  const int64_t d = pl.dsz;
  const int occ = d >= 16384 ? 1 : d >= 8192 ? 2 : d >= 4096 ? 4 : 8;
  const int64_t units = int64_t(pl.n) * pl.p, slots = 256LL * occ;
  int64_t v = (units + slots / 2) / slots;
  v = std::max<int64_t>(1, std::min<int64_t>(v, pl.p));
  ppg = (int)v;
  ng = (pl.p + ppg - 1) / ppg;
}

size_t carve_dct(const Plan& pl, void* base, DctWs* w) {
  Carver c(base);
  const int64_t D = pl.dsz, N = pl.n, J = pl.j, P = pl.p;
  dct_grouping(pl, w->ppg, w->ng);
  w->E = c.take<float2>(J * P * D);
  w->G = c.take<float2>(D * J * J);
  w->xh = c.take<float>(N * J * D);
  w->yh = c.take<float>(N * J * D);
  w->Th = c.take<float>(N * J * D);
  w->lam = c.take<float>(N * J * D);
  w->part = c.take<float>(N * w->ng * J * D);
  w->rpri = c.take<double>(N * w->ng);
  w->rdual = c.take<double>(N * eblk(D));
  w->opart = c.take<double>(N * eblk(D));
  w->rho = c.take<float>(N);
  return c.off;
}

#define DLAUNCH_J(KERNEL, J, grid, block, st, ...)                                      \
  do {                                                                                 \
    if ((J) == 1) hipLaunchKernelGGL(KERNEL<1>, grid, block, 0, st, __VA_ARGS__);      \
    else if ((J) == 2) hipLaunchKernelGGL(KERNEL<2>, grid, block, 0, st, __VA_ARGS__); \
    else hipLaunchKernelGGL(KERNEL<3>, grid, block, 0, st, __VA_ARGS__);               \
  } while (0)

// e0, e1: events to launch with (an own-launch TraceScope's), or null
template <int J, int MODE>
bool tile_launch(const Plan& pl, DctWs& w, float* z, float* theta, float beta, const float* img, hipStream_t st,
                 hipEvent_t e0, hipEvent_t e1) {
  const int h = pl.g[1], wd = pl.g[2];
  const dim3 grid(MODE == kDctImage ? unsigned(pl.n * pl.j) : unsigned(w.ng * pl.n));
#define TL(HH, WW)                                                                                                 \
  if (h == HH && wd == WW) {                                                                                       \
    if (e0)                                                                                                        \
      hipExtLaunchKernelGGL((k_dct_tile<HH, WW, J, MODE>), grid, dim3(dct_threads(HH * WW)), 0, st, e0, e1, 0,    \
                            w.E, w.lam, z, theta, w.rho, beta, w.part, w.rpri, pl.k, pl.p, w.ppg, w.ng, img, w.xh); \
    else                                                                                                           \
      hipLaunchKernelGGL((k_dct_tile<HH, WW, J, MODE>), grid, dim3(dct_threads(HH * WW)), 0, st, w.E, w.lam, z,   \
                         theta, w.rho, beta, w.part, w.rpri, pl.k, pl.p, w.ppg, w.ng, img, w.xh);                   \
    return true;                                                                                                   \
  }
  TL(8, 8) TL(8, 16) TL(8, 32) TL(8, 64) TL(8, 128)
  TL(16, 8) TL(16, 16) TL(16, 32) TL(16, 64) TL(16, 128)
  TL(32, 8) TL(32, 16) TL(32, 32) TL(32, 64) TL(32, 128)
  TL(64, 8) TL(64, 16) TL(64, 32) TL(64, 64) TL(64, 128)
  TL(128, 8) TL(128, 16) TL(128, 32) TL(128, 64) TL(128, 128)
#undef TL
  return false;
}

template <int MODE>
bool tile_dispatch(const Plan& pl, DctWs& w, float* z, float* theta, float beta, const float* img, hipStream_t st,
                   hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  if (pl.j == 1) return tile_launch<1, MODE>(pl, w, z, theta, beta, img, st, e0, e1);
  if (pl.j == 2) return tile_launch<2, MODE>(pl, w, z, theta, beta, img, st, e0, e1);
  return tile_launch<3, MODE>(pl, w, z, theta, beta, img, st, e0, e1);
}

int dct_setup(const Plan& pl, const float* b, const float* q, DctWs& w, hipStream_t st) {
  const int64_t D = pl.dsz;
  hipLaunchKernelGGL(k_dct_eig, dim3(eblk(D), pl.p, pl.j), dim3(kDE), 0, st, q, w.E, pl.k, pl.j, pl.p, pl.g[1],
                     pl.g[2], pl.fs[1], pl.fs[2]);
  DLAUNCH_J(k_dct_gram, pl.j, dim3(eblk(D)), dim3(kDE), st, w.E, w.G, pl.p, D);
  if (!tile_dispatch<kDctImage>(pl, w, nullptr, nullptr, 0.f, b, st)) return CSC_EUNSUPPORTED;
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

}  // namespace

size_t dct_ws_bytes(const Plan& pl) {
  DctWs w;
  return carve_dct(pl, nullptr, &w);
}

int run_code_dct(const Plan& pl, const float* b, const float* q, float beta, float* rho, int iters, unsigned flags,
                 float* z, float* theta, double* resid, void* ws, hipStream_t st) {
  DctWs w;
  carve_dct(pl, ws, &w);
  const int64_t D = pl.dsz, N = pl.n, J = pl.j, ns = N * J * D;
  const int W = pl.g[2];
  const bool adaptive = (flags & CSC_ADAPTIVE_RHO) != 0;
  int rc = dct_setup(pl, b, q, w, st);
  if (rc != CSC_OK) return rc;
  hipLaunchKernelGGL(k_dct_copy, dim3(eblk(N)), dim3(kDE), 0, st, w.rho, rho, N);
  const dim3 gspec(eblk(D), (unsigned)N);
  if (flags & CSC_Z_ZERO) {
    hipLaunchKernelGGL(k_dct_fill, dim3(eblk(N * pl.k * D)), dim3(kDE), 0, st, z, N * pl.k * D, 0.f);
    hipLaunchKernelGGL(k_dct_fill, dim3(eblk(ns)), dim3(kDE), 0, st, w.yh, ns, 0.f);
  } else {
    if (!tile_dispatch<kDctForward>(pl, w, z, nullptr, 0.f, nullptr, st)) return CSC_EUNSUPPORTED;
    DLAUNCH_J(k_dct_spec, pl.j, gspec, dim3(kDE), st, w.part, w.G, w.xh, w.yh, w.Th, w.lam, w.rho,
              (double*)nullptr, w.ng, W, D, 0, w.yh);
  }
  const bool th_zero = theta == nullptr || (flags & CSC_THETA_ZERO) != 0;
  if (th_zero) {
    hipLaunchKernelGGL(k_dct_fill, dim3(eblk(ns)), dim3(kDE), 0, st, w.Th, ns, 0.f);
    if (theta && iters == 0)
      hipLaunchKernelGGL(k_dct_fill, dim3(eblk(N * pl.k * D)), dim3(kDE), 0, st, theta, N * pl.k * D, 0.f);
  } else {
    if (!tile_dispatch<kDctForward>(pl, w, theta, nullptr, 0.f, nullptr, st)) return CSC_EUNSUPPORTED;
    DLAUNCH_J(k_dct_spec, pl.j, gspec, dim3(kDE), st, w.part, w.G, w.xh, w.yh, w.Th, w.lam, w.rho,
              (double*)nullptr, w.ng, W, D, 0, w.Th);
  }
  if (iters > 0) DLAUNCH_J(k_dct_solve, pl.j, gspec, dim3(kDE), st, w.G, w.xh, w.yh, w.Th, w.rho, w.lam, D);
  const bool need_rho = adaptive || resid != nullptr;
  for (int it = 0; it < iters; ++it) {
    const bool last = it == iters - 1;
    {
      // the coding map kernel, timed at its own start and end when traced
      TraceScope trace(kTraceCodeMaps, st, true);
      hipEvent_t e0 = nullptr, e1 = nullptr;
      trace.events(&e0, &e1);
      if (!tile_dispatch<kDctIter>(pl, w, z, last ? theta : nullptr, beta, nullptr, st, e0, e1))
        return CSC_EUNSUPPORTED;
    }
    const int solve_next = (!last && !adaptive) ? 1 : 0;
    DLAUNCH_J(k_dct_spec, pl.j, gspec, dim3(kDE), st, w.part, w.G, w.xh, w.yh, w.Th, w.lam, w.rho, w.rdual, w.ng,
              W, D, solve_next, (float*)nullptr);
    if (need_rho)
      launch_rho(w.rpri, w.ng, w.rdual, (int)eblk(D), w.rho, resid, it, (int)N, D, adaptive ? 1 : 0, st);
    if (adaptive && !last)
      DLAUNCH_J(k_dct_solve, pl.j, gspec, dim3(kDE), st, w.G, w.xh, w.yh, w.Th, w.rho, w.lam, D);
  }
  if (adaptive) hipLaunchKernelGGL(k_dct_copy, dim3(eblk(N)), dim3(kDE), 0, st, rho, w.rho, N);
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

int run_objective_dct(const Plan& pl, const float* b, const float* q, const float* z, float beta, double* out,
                      void* ws, hipStream_t st) {
  DctWs w;
  carve_dct(pl, ws, &w);
  const int64_t D = pl.dsz, N = pl.n;
  int rc = dct_setup(pl, b, q, w, st);
  if (rc != CSC_OK) return rc;
  if (!tile_dispatch<kDctForward>(pl, w, const_cast<float*>(z), nullptr, 0.f, nullptr, st)) return CSC_EUNSUPPORTED;
  DLAUNCH_J(k_dct_obj, pl.j, dim3(eblk(D), (unsigned)N), dim3(kDE), st, w.part, w.xh, w.opart, w.ng, pl.g[2], D);
  launch_obj_final(w.opart, (int)eblk(D), w.rpri, w.ng, out, (int)N, D, beta, st);
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

}  // namespace dcsc
