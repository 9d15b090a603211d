// Differentiable coding: the coding ADMM unrolled for a fixed number of
// iterations, its reverse (adjoint) pass with respect to the filters and the
// sparsity weight, and the gradient of the objective of eq:CSC.  Grayscale
// (J = 1).
//
// The unrolled solve is the coding iteration (coding.hip), which records its
// state every `every` iterations.  The reverse pass replays each segment from
// its record with that same iteration, then walks the segment's iterations in
// reverse through the literal updates of eq:Inference_solution with theta
// kept (w = theta + z/rho, s = D w - x/rho, lam = P s with
// P = (D D^T + I/rho)^-1, v = D^T lam, u = v - z/rho, theta' = clip(u, +-beta),
// z' = z + rho (theta' - v)).  At each state it recomputes the spectra of w
// and lam; the branch of the clip at each code is read from the codes after
// the iteration (exactly zero where u passed through, of the sign opposite
// to u elsewhere), so v itself is never formed:
//   t = thbar' + rho zbar';  ubar = t [|u| < beta];  betabar += t sign(u) [|u| > beta]
//   vbar = ubar - rho zbar';  zbar = zbar' - ubar/rho
//   sbar = P D vbar;  wbar = D^T sbar;  thetabar = wbar;  zbar += wbar/rho
//   dbar_k += corr(lam, vbar_k - wbar_k) + corr(sbar, w_k - v_k)
// where corr(a, b)[m] = sum_p a[p] b[p - m] over the filter support.  In the
// Fourier domain the filter term per frequency is
//   lam conj(vbarhat_k) + sbar conj(what_k) - 2 dhat_k Re(lam conj(sbar)),
// summed over images (fixed order) and iterations, and mapped back to taps
// by one inverse FFT and the support crop at the end.
#include "common.hpp"
#include "internal.hpp"

namespace dcsc {

constexpr int kDW = 256;

static unsigned dblk(int64_t n) { return (unsigned)((n + kDW - 1) / kDW); }

__device__ __forceinline__ int64_t dneg(int64_t fl, int T, int H, int W) {
  const int f = (int)fl;
  const int lw = __builtin_ctz(W), lh = __builtin_ctz(H);
  const int w = f & (W - 1), h = (f >> lw) & (H - 1), t = f >> (lw + lh);
  return (((((T - t) & (T - 1)) << lh) | ((H - h) & (H - 1))) << lw) | ((W - w) & (W - 1));
}

// a = (c + conj(cm))/2, b = -i (c - conj(cm))/2
__device__ __forceinline__ void dunpack(float2 c, float2 cm, float2& a, float2& b) {
  a = make_float2(0.5f * (c.x + cm.x), 0.5f * (c.y - cm.y));
  b = make_float2(0.5f * (c.y + cm.y), -0.5f * (c.x - cm.x));
}

// Wbuf[n][p] = (theta + z/rho) for maps 2p, 2p+1
__global__ void d_pack_w(const float* __restrict__ z, const float* __restrict__ th, float2* __restrict__ Wb,
                         const float* __restrict__ rho, int K, int P, int64_t D) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, n = blockIdx.z;
  if (f >= D) return;
  const float ir = 1.0f / rho[n];
  const int64_t a = (int64_t(n) * K + 2 * p) * D + f;
  float2 v = make_float2(th[a] + z[a] * ir, 0.f);
  if (2 * p + 1 < K) v.y = th[a + D] + z[a + D] * ir;
  Wb[(int64_t(n) * P + p) * D + f] = v;
}

// Wbuf[n][p] = (z_2p, z_2p+1)
__global__ void d_pack_z(const float* __restrict__ z, float2* __restrict__ Wb, int K, int P, int64_t D) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, n = blockIdx.z;
  if (f >= D) return;
  const int64_t a = (int64_t(n) * K + 2 * p) * D + f;
  Wb[(int64_t(n) * P + p) * D + f] = make_float2(z[a], (2 * p + 1 < K) ? z[a + D] : 0.f);
}

// out[n](f) = Y / (S + 1/rho), Y = sym(sum_p buf conj(E)) (- xhat/rho when xh)
__global__ void d_reduce_solve(const float2* __restrict__ buf, const float2* __restrict__ E,
                               const float2* __restrict__ G, const float2* __restrict__ xh,
                               const float* __restrict__ rho, float2* __restrict__ out, int P, int T, int H,
                               int W) {
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (f >= D) return;
  const int64_t fn = dneg(f, T, H, W);
  if (fn < f) return;  // the pair (f, -f) is handled by its lower index
  float2 y = make_float2(0.f, 0.f), ym = make_float2(0.f, 0.f);
#pragma unroll 4
  for (int p = 0; p < P; ++p) {
    const float2* bp = buf + (int64_t(n) * P + p) * D;
    const float2* ep = E + int64_t(p) * D;
    y = cadd(y, cmulc(bp[f], ep[f]));
    ym = cadd(ym, cmulc(bp[fn], ep[fn]));
  }
  const float ir = 1.0f / rho[n];
  // at f from (y, ym) and at -f from (ym, y)
  for (int side = 0; side < (fn == f ? 1 : 2); ++side) {
    const int64_t ff = side ? fn : f;
    const float2 a = side ? ym : y, b = side ? y : ym;
    float2 s = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
    if (xh) {
      const float2 x = xh[int64_t(n) * D + ff];
      s = make_float2(s.x - x.x * ir, s.y - x.y * ir);
    }
    const float den = G[ff].x + ir;
    out[int64_t(n) * D + ff] = make_float2(s.x / den, s.y / den);
  }
}

// Adjoint of the clip and z updates.  The clip's branch at each code is the
// forward's own: its step z' = soft(z - rho v, rho beta) is exactly 0 where
// the clip passed u = v - z/rho through, and elsewhere sign(u) = -sign(z'),
// so the state after the iteration (znext) decides both.  In: znext,
// zbar', thbar'.  Out: Vb <- vbar pair (spatial), zbar <- zbar' - ubar/rho,
// bpart[(n P + p) nblk + blk] += sum t sign(u) over the clipped codes.
__global__ __launch_bounds__(kDW) void d_adj_clip(float2* __restrict__ Vb, const float* __restrict__ znext,
                                                  float* __restrict__ zbar, const float* __restrict__ thbar,
                                                  const float* __restrict__ rho, double* __restrict__ bpart, int K,
                                                  int P, int64_t D) {
  __shared__ double red[kDW / 64];
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, n = blockIdx.z;
  double bs = 0.0;
  if (f < D) {
    const float r = rho[n], ir = 1.0f / r;
    const int64_t a = (int64_t(n) * K + 2 * p) * D + f;
    float vbar[2] = {0.f, 0.f};
    for (int s = 0; s < 2 && 2 * p + s < K; ++s) {
      const float zn = znext[a + s * D];
      const float zb = zbar[a + s * D];
      const float t = thbar[a + s * D] + r * zb;
      const bool pass = zn == 0.f;
      const float ub = pass ? t : 0.f;
      if (!pass) bs += (double)(zn < 0.f ? t : -t);
      vbar[s] = ub - r * zb;
      zbar[a + s * D] = zb - ub * ir;
    }
    Vb[(int64_t(n) * P + p) * D + f] = make_float2(vbar[0], vbar[1]);
  }
  const double tot = block_sum(bs, red);
  if (threadIdx.x == 0) bpart[(int64_t(n) * P + p) * gridDim.x + blockIdx.x] += tot;
}

// Dbar[p](f) += sum_n [A_2p + i A_2p+1],
// A_k = lam conj(vbarhat_k) + sbar conj(what_k) - 2 dhat_k Re(lam conj(sbar))
// (vbarhat from Vb, what from Wb, both pair spectra).  With Wb == nullptr the
// term is res conj(zhat_k) (lam = res, Vb = code pair spectra): the filter
// gradient of the data term of eq:CSC.
__global__ void d_dbar(const float2* __restrict__ Vb, const float2* __restrict__ Wb, const float2* __restrict__ E,
                       const float2* __restrict__ lam, const float2* __restrict__ sbar, float2* __restrict__ Dbar,
                       int N, int P, int T, int H, int W) {
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (f >= D) return;
  const int64_t fn = dneg(f, T, H, W);
  // the pair (f, -f) is handled by its lower index: the unpacked values at
  // -f are the exact conjugates of those at f, so both outputs come from
  // one read of the pair spectra (lam and sbar are read at both)
  if (fn < f) return;
  const int sides = fn == f ? 1 : 2;
  float2 da = make_float2(0.f, 0.f), db = make_float2(0.f, 0.f);
  if (Wb) {
    const float2 ef = E[int64_t(p) * D + f], em = E[int64_t(p) * D + fn];
    // dhat_2p = (conj(E(f)) + E(-f))/2, dhat_2p+1 = i (conj(E(f)) - E(-f))/2
    da = make_float2(0.5f * (ef.x + em.x), 0.5f * (-ef.y + em.y));
    db = make_float2(0.5f * (ef.y + em.y), 0.5f * (ef.x - em.x));
  }
  float2 acc_a[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
  float2 acc_b[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
  for (int n = 0; n < N; ++n) {
    const float2* vp = Vb + (int64_t(n) * P + p) * D;
    float2 va, vb;
    dunpack(vp[f], vp[fn], va, vb);
    float2 wa = make_float2(0.f, 0.f), wb = make_float2(0.f, 0.f);
    if (Wb) {
      const float2* wp = Wb + (int64_t(n) * P + p) * D;
      dunpack(wp[f], wp[fn], wa, wb);
    }
    for (int side = 0; side < sides; ++side) {
      const int64_t ff = side ? fn : f;
      const float2 va_s = side ? cconj(va) : va, vb_s = side ? cconj(vb) : vb;
      const float2 l = lam[int64_t(n) * D + ff];
      acc_a[side] = cadd(acc_a[side], cmulc(l, va_s));
      acc_b[side] = cadd(acc_b[side], cmulc(l, vb_s));
      if (Wb) {
        const float2 wa_s = side ? cconj(wa) : wa, wb_s = side ? cconj(wb) : wb;
        const float2 da_s = side ? cconj(da) : da, db_s = side ? cconj(db) : db;
        const float2 s = sbar[int64_t(n) * D + ff];
        const float re2 = 2.0f * (l.x * s.x + l.y * s.y);
        acc_a[side] = cadd(acc_a[side], csub(cmulc(s, wa_s), cscale(da_s, re2)));
        acc_b[side] = cadd(acc_b[side], csub(cmulc(s, wb_s), cscale(db_s, re2)));
      }
    }
  }
  for (int side = 0; side < sides; ++side) {
    float2* o = Dbar + int64_t(p) * D + (side ? fn : f);
    const float2 cur = *o;
    *o = make_float2(cur.x + acc_a[side].x - acc_b[side].y, cur.y + acc_a[side].y + acc_b[side].x);
  }
}

// thetabar = wbar, zbar += wbar / rho, from W = D * (wbar_2p + i wbar_2p+1).
__global__ void d_adj_finish(const float2* __restrict__ Wb, float* __restrict__ zbar, float* __restrict__ thbar,
                             const float* __restrict__ rho, int K, int P, int64_t D) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, n = blockIdx.z;
  if (f >= D) return;
  const float ir = 1.0f / rho[n], invD = 1.0f / (float)D;
  const float2 c = Wb[(int64_t(n) * P + p) * D + f];
  const int64_t a = (int64_t(n) * K + 2 * p) * D + f;
  for (int s = 0; s < 2 && 2 * p + s < K; ++s) {
    const float wb = (s ? c.y : c.x) * invD;
    thbar[a + s * D] = wb;
    zbar[a + s * D] += wb * ir;
  }
}

// zbar = D^T (D z - x) + beta sign(z) from V = D * D^T(res) pairs.
__global__ void d_zbar_loss(const float2* __restrict__ Vb, const float* __restrict__ z, float* __restrict__ zbar,
                            float beta, int K, int P, int64_t D) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p = blockIdx.y, n = blockIdx.z;
  if (f >= D) return;
  const float invD = 1.0f / (float)D;
  const float2 c = Vb[(int64_t(n) * P + p) * D + f];
  const int64_t a = (int64_t(n) * K + 2 * p) * D + f;
  for (int s = 0; s < 2 && 2 * p + s < K; ++s) {
    const float zz = z[a + s * D];
    const float sg = zz > 0.f ? 1.f : (zz < 0.f ? -1.f : 0.f);
    zbar[a + s * D] = (s ? c.y : c.x) * invD + beta * sg;
  }
}

__global__ void d_sub(const float2* __restrict__ a, const float2* __restrict__ b, float2* __restrict__ o, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) o[i] = csub(a[i], b[i]);
}

__global__ void d_zero(float* __restrict__ p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}
__global__ void d_zero_d(double* __restrict__ p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}
__global__ void d_copy(float* __restrict__ dst, const float* __restrict__ src, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// dd[k][0][m] (+)= (1/D) Re/Im of the inverse FFT of Dbar pair k/2 at tap m.
__global__ void d_crop_taps(const float2* __restrict__ Dsp, float* __restrict__ dd, int K, int T, int H, int W,
                            int ft, int fh, int fw, int accumulate) {
  const int64_t msz = int64_t(ft) * fh * fw;
  const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (m >= msz) return;
  const int t = (int)(m / (int64_t(fh) * fw)), h = (int)((m / fw) % fh), w = (int)(m % fw);
  const int64_t D = int64_t(T) * H * W;
  const float2 c = Dsp[int64_t(k / 2) * D + (int64_t(t) * H + h) * W + w];
  const float v = ((k & 1) ? c.y : c.x) / (float)D;
  dd[int64_t(k) * msz + m] = accumulate ? dd[int64_t(k) * msz + m] + v : v;
}

// out[0] = sum of n partials (fixed order), single thread.
// out = sum of n partials by one workgroup of 1024 threads in a fixed order
// (thread t sums every 1024th partial from t, then the block reduction).
constexpr int kSumT = 1024;

__global__ __launch_bounds__(kSumT) void d_sum(const double* __restrict__ part, int64_t n, double* __restrict__ out) {
  __shared__ double red[kSumT / 64];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kSumT) s += part[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = t;
}

// ----------------------------------------------------------------- host

// ------------------------------------------------------ fused axis passes
// The 2-D grids beyond one LDS tile (and 3-D volumes) are transformed one
// axis at a time, each pass reading and writing every element.  These passes
// fold the elementwise step that precedes or follows a transform of the
// adjoint into the pass that moves the data anyway: LD(i) produces element i
// of the first pass's input and ST(i, v) takes element i of the last pass's
// output (i: linear index into [N P][T][H][W]).  Each operator repeats the
// arithmetic of its stand-alone kernel exactly.
constexpr int kOpTile = 4096, kOpThreads = 256;

// Each operator splits into fetch(i) -> Pre (global loads only) and
// make(i, pre) / put(i, v, pre) (arithmetic and stores), so that a thread
// issues the loads of all its elements before its first store.
struct LdPlain {
  const float2* d;
  using Pre = float2;
  __device__ Pre fetch(int64_t i) const { return d[i]; }
  __device__ float2 make(int64_t, const Pre& v) { return v; }
  __device__ void flush(double*) {}
};
struct StPlain {
  float2* d;
  struct Pre {};
  __device__ Pre fetch(int64_t) const { return Pre{}; }
  __device__ void put(int64_t i, float2 v, const Pre&) { d[i] = v; }
  __device__ void flush(double*) {}
};

// index i -> image n, pair p, grid position f (D a power of two)
__device__ __forceinline__ void op_index(int64_t i, int lgD, int P, int& n, int& p, int64_t& f) {
  const int64_t g = i >> lgD;
  f = i & ((int64_t(1) << lgD) - 1);
  n = (int)(g / P);
  p = (int)(g - int64_t(n) * P);
}
// offset of map 2p of image n at f, and whether map 2p + 1 exists
__device__ __forceinline__ int64_t op_map(int64_t i, int lgD, int K, int P, int& n, bool& hb) {
  int p;
  int64_t f;
  op_index(i, lgD, P, n, p, f);
  hb = 2 * p + 1 < K;
  return ((int64_t(n) * K + 2 * p) << lgD) + f;
}

// d_pack_w: the pairs of w = theta + z/rho
struct LdPackW {
  const float *z, *th, *rho;
  int K, P, lgD;
  struct Pre {
    float za, zb, ta, tb, r;
  };
  __device__ Pre fetch(int64_t i) const {
    int n;
    bool hb;
    const int64_t a = op_map(i, lgD, K, P, n, hb), D = int64_t(1) << lgD;
    Pre q;
    q.r = rho[n];
    q.za = z[a];
    q.ta = th[a];
    q.zb = hb ? z[a + D] : 0.f;
    q.tb = hb ? th[a + D] : 0.f;
    return q;
  }
  __device__ float2 make(int64_t, const Pre& q) {
    const float ir = 1.0f / q.r;
    return make_float2(q.ta + q.za * ir, q.tb + q.zb * ir);
  }
  __device__ void flush(double*) {}
};

// d_adj_clip: vbar pairs, zbar update, and the beta partial of the block
struct LdAdjClip {
  const float* znext;
  float* zbar;
  const float *thbar, *rho;
  double* bpart;
  int K, P, lgD;
  double bs;
  struct Pre {
    float zn[2], zb[2], tb[2], r;
  };
  __device__ Pre fetch(int64_t i) const {
    int n;
    bool hb;
    const int64_t a = op_map(i, lgD, K, P, n, hb), D = int64_t(1) << lgD;
    Pre q;
    q.r = rho[n];
    for (int s = 0; s < 2; ++s) {
      const bool on = s == 0 || hb;
      q.zn[s] = on ? znext[a + s * D] : 0.f;
      q.zb[s] = on ? zbar[a + s * D] : 0.f;
      q.tb[s] = on ? thbar[a + s * D] : 0.f;
    }
    return q;
  }
  __device__ float2 make(int64_t i, const Pre& q) {
    int n;
    bool hb;
    const int64_t a = op_map(i, lgD, K, P, n, hb), D = int64_t(1) << lgD;
    const float r = q.r, ir = 1.0f / r;
    float vbar[2] = {0.f, 0.f};
    for (int s = 0; s < 2 && (s == 0 || hb); ++s) {
      const float zb = q.zb[s];
      const float t = q.tb[s] + r * zb;
      const bool pass = q.zn[s] == 0.f;
      const float ub = pass ? t : 0.f;
      if (!pass) bs += (double)(q.zn[s] < 0.f ? t : -t);
      vbar[s] = ub - r * zb;
      zbar[a + s * D] = zb - ub * ir;
    }
    return make_float2(vbar[0], vbar[1]);
  }
  __device__ void flush(double* red) {
    const double tot = block_sum(bs, red);
    if (threadIdx.x == 0) bpart[blockIdx.x] += tot;
  }
};

// k_make_v (J = 1): lam E_p
struct LdMakeV {
  const float2 *E, *lam;
  int P, lgD;
  struct Pre {
    float2 l, e;
  };
  __device__ Pre fetch(int64_t i) const {
    int n, p;
    int64_t f;
    op_index(i, lgD, P, n, p, f);
    return Pre{lam[(int64_t(n) << lgD) + f], E[(int64_t(p) << lgD) + f]};
  }
  __device__ float2 make(int64_t, const Pre& q) { return cmul(q.l, q.e); }
  __device__ void flush(double*) {}
};

// d_adj_finish: thetabar = wbar, zbar += wbar / rho
struct StAdjFinish {
  float *zbar, *thbar;
  const float* rho;
  int K, P, lgD;
  struct Pre {
    float zb[2], r;
  };
  __device__ Pre fetch(int64_t i) const {
    int n;
    bool hb;
    const int64_t a = op_map(i, lgD, K, P, n, hb), D = int64_t(1) << lgD;
    Pre q;
    q.r = rho[n];
    q.zb[0] = zbar[a];
    q.zb[1] = hb ? zbar[a + D] : 0.f;
    return q;
  }
  __device__ void put(int64_t i, float2 c, const Pre& q) {
    int n;
    bool hb;
    const int64_t a = op_map(i, lgD, K, P, n, hb), D = int64_t(1) << lgD;
    const float ir = 1.0f / q.r, invD = 1.0f / (float)D;
    for (int s = 0; s < 2 && (s == 0 || hb); ++s) {
      const float wb = (s ? c.y : c.x) * invD;
      thbar[a + s * D] = wb;
      zbar[a + s * D] = q.zb[s] + wb * ir;
    }
  }
  __device__ void flush(double*) {}
};

// One axis pass over [outer][L][inner] (as the plain axis pass of fftops.hip).
template <int L, int DIR, class LD, class ST>
__global__ __launch_bounds__(kOpThreads) void d_fft_axis_op(LD ld, ST sto, int64_t outer, int64_t inner, int lbi,
                                                            int lbo) {
  constexpr int T = kOpTile, NT = kOpThreads, LP = L + 1, EPT = T / NT;
  __shared__ float2 tile[(T / L) * LP];
  __shared__ float2 tw[256];
  __shared__ double red[NT / 64];
  load_twiddles(tw);
  const int bi = 1 << lbi;
  const int64_t tiles_in = inner >> lbi;
  const int64_t t = blockIdx.x;
  const int64_t o0 = (t / tiles_in) << lbo;
  const int64_t i0 = (t % tiles_in) << lbi;
  auto elem = [&](int k, int64_t& idx, int& slot) {
    const int e = threadIdx.x + k * NT;
    const int b_in = e & (bi - 1);
    const int jj = (e >> lbi) & (L - 1);
    const int b_o = e >> lbi >> __builtin_ctz(L);
    idx = ((o0 + b_o) * L + jj) * inner + i0 + b_in;
    slot = ((b_o << lbi) + b_in) * LP + jj;
    return o0 + b_o < outer;
  };
  {
    typename LD::Pre pre[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      int64_t idx;
      int slot;
      if (elem(k, idx, slot)) pre[k] = ld.fetch(idx);
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      int64_t idx;
      int slot;
      const bool ok = elem(k, idx, slot);
      tile[slot] = ok ? ld.make(idx, pre[k]) : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  fft_lines<L, T, NT, DIR, 1, LP>(tile, tw);
  {
    typename ST::Pre pre[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      int64_t idx;
      int slot;
      if (elem(k, idx, slot)) pre[k] = sto.fetch(idx);
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      int64_t idx;
      int slot;
      if (elem(k, idx, slot)) sto.put(idx, tile[slot], pre[k]);
    }
  }
  ld.flush(red);
  sto.flush(red);
}

static int dlog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

template <int DIR, class LD, class ST>
static hipError_t axis_op(LD ld, ST sto, int64_t outer, int L, int64_t inner, hipStream_t st) {
  const int ll = dlog2(L), lt = dlog2(kOpTile);
  int lbi = dlog2(inner);
  if (lbi > lt - ll) lbi = lt - ll;
  const int lbo = lt - ll - lbi;
  const int64_t tiles = ((outer + (int64_t(1) << lbo) - 1) >> lbo) * (inner >> lbi);
  const dim3 grid((unsigned)tiles), block(kOpThreads);
  switch (L) {
#define CASE(LL) \
  case LL: hipLaunchKernelGGL((d_fft_axis_op<LL, DIR, LD, ST>), grid, block, 0, st, ld, sto, outer, inner, lbi, lbo); break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64) CASE(128) CASE(256)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Transform of `count` grids in place (as fft_grids on the axis path) with
// LD feeding the first pass and ST taking the last pass's output.  The axes
// go W, H, T, or with W_LAST T, H, W: the W pass moves whole contiguous
// lines, so a store operator that writes per-map floats belongs there.
template <int DIR, bool W_LAST = false, class LD, class ST>
static hipError_t fft_fused(float2* data, int64_t count, const int g[3], LD ld, ST sto, hipStream_t st) {
  const int T = g[0], H = g[1], W = g[2];
  hipError_t e;
  if (W_LAST) {
    if (T > 1) {
      if ((e = axis_op<DIR>(ld, StPlain{data}, count, T, int64_t(H) * W, st)) != hipSuccess) return e;
      if ((e = axis_op<DIR>(LdPlain{data}, StPlain{data}, count * T, H, W, st)) != hipSuccess) return e;
    } else if ((e = axis_op<DIR>(ld, StPlain{data}, count, H, W, st)) != hipSuccess) {
      return e;
    }
    return axis_op<DIR>(LdPlain{data}, sto, count * T * H, W, 1, st);
  }
  if ((e = axis_op<DIR>(ld, StPlain{data}, count * T * H, W, 1, st)) != hipSuccess) return e;
  if (T > 1) {
    if ((e = axis_op<DIR>(LdPlain{data}, StPlain{data}, count * T, H, W, st)) != hipSuccess) return e;
    return axis_op<DIR>(LdPlain{data}, sto, count, T, int64_t(H) * W, st);
  }
  return axis_op<DIR>(LdPlain{data}, sto, count, H, W, st);
}

// grids that fft_grids transforms axis by axis
static bool axis_path(const Plan& pl) { return !(pl.g[0] == 1 && tile_supported(pl.g[1], pl.g[2])); }

struct DiffWs {
  CodeWs cw;
  float2 *Wb, *Vb, *lam, *sbar, *Dbar;
  float *zbar, *thbar, *seg;
  double* bpart;
  int64_t nbpart;
};

static size_t carve_diff(const Plan& pl, int every, void* base, DiffWs* w) {
  Carver c(base);
  const int64_t D = pl.dsz, N = pl.n, P = pl.p, K = pl.k;
  const size_t cbytes = carve_code(pl, base, &w->cw);
  c.off = cbytes;
  w->Wb = c.take<float2>(N * P * D);
  w->Vb = c.take<float2>(N * P * D);
  w->lam = c.take<float2>(N * D);
  w->sbar = c.take<float2>(N * D);
  w->Dbar = c.take<float2>(P * D);
  w->zbar = c.take<float>(N * K * D);
  w->thbar = c.take<float>(N * K * D);
  w->seg = c.take<float>(int64_t(every > 0 ? every : 1) * 2 * N * K * D);
  w->nbpart = N * P * int64_t(dblk(D));
  w->bpart = c.take<double>(w->nbpart + 1);
  return c.off;
}

size_t run_diff_ws(const Plan& pl, int every) {
  DiffWs w;
  return carve_diff(pl, every, nullptr, &w);
}

// Spectra the adjoint needs from one literal iteration at the state (z, th):
// those of the pairs of w = th + z/rho in Wb, and lam.
static hipError_t lit_intermediates(const Plan& pl, DiffWs& w, const float* z, const float* th, const float* rho,
                                    hipStream_t st) {
  const int64_t D = pl.dsz;
  const dim3 g3(dblk(D), pl.p, pl.n);
  hipError_t e;
  if (axis_path(pl)) {
    e = fft_fused<-1>(w.Wb, int64_t(pl.n) * pl.p, pl.g, LdPackW{z, th, rho, pl.k, pl.p, dlog2(D)}, StPlain{w.Wb}, st);
  } else {
    hipLaunchKernelGGL(d_pack_w, g3, dim3(kDW), 0, st, z, th, w.Wb, rho, pl.k, pl.p, D);
    e = fft_grids(w.Wb, int64_t(pl.n) * pl.p, pl.g, -1, st);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(d_reduce_solve, dim3(dblk(D), pl.n), dim3(kDW), 0, st, w.Wb, w.cw.E, w.cw.G, w.cw.xh, rho,
                     w.lam, pl.p, pl.g[0], pl.g[1], pl.g[2]);
  return hipGetLastError();
}

// Adjoint of one iteration whose input state is (z, th) and whose output
// codes are znext; (zbar, thbar) hold the adjoint of its output and are
// replaced by the adjoint of its input.
static hipError_t adjoint_iter(const Plan& pl, DiffWs& w, const float* z, const float* th, const float* znext,
                               const float* rho, hipStream_t st) {
  const int64_t D = pl.dsz;
  const dim3 g3(dblk(D), pl.p, pl.n);
  hipError_t e = lit_intermediates(pl, w, z, th, rho, st);
  if (e != hipSuccess) return e;
  const bool fused = axis_path(pl);
  const int lgD = dlog2(D);
  const int64_t np = int64_t(pl.n) * pl.p;
  if (fused) {
    e = fft_fused<-1>(w.Vb, np, pl.g, LdAdjClip{znext, w.zbar, w.thbar, rho, w.bpart, pl.k, pl.p, lgD, 0.0},
                      StPlain{w.Vb}, st);
  } else {
    hipLaunchKernelGGL(d_adj_clip, g3, dim3(kDW), 0, st, w.Vb, znext, w.zbar, w.thbar, rho, w.bpart, pl.k, pl.p, D);
    e = fft_grids(w.Vb, np, pl.g, -1, st);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(d_reduce_solve, dim3(dblk(D), pl.n), dim3(kDW), 0, st, w.Vb, w.cw.E, w.cw.G,
                     (const float2*)nullptr, rho, w.sbar, pl.p, pl.g[0], pl.g[1], pl.g[2]);
  hipLaunchKernelGGL(d_dbar, dim3(dblk(D), pl.p), dim3(kDW), 0, st, w.Vb, w.Wb, w.cw.E, w.lam, w.sbar, w.Dbar,
                     pl.n, pl.p, pl.g[0], pl.g[1], pl.g[2]);
  if (fused)
    return fft_fused<+1, true>(w.Wb, np, pl.g, LdMakeV{w.cw.E, w.sbar, pl.p, lgD},
                               StAdjFinish{w.zbar, w.thbar, rho, pl.k, pl.p, lgD}, st);
  launch_make_v(pl, w.cw.E, w.sbar, w.Wb, st);
  if ((e = fft_grids(w.Wb, np, pl.g, +1, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(d_adj_finish, g3, dim3(kDW), 0, st, w.Wb, w.zbar, w.thbar, rho, pl.k, pl.p, D);
  return hipGetLastError();
}

static hipError_t finish_taps(const Plan& pl, DiffWs& w, float* dd, bool accumulate, hipStream_t st) {
  hipError_t e = fft_grids(w.Dbar, pl.p, pl.g, +1, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(d_crop_taps, dim3(dblk(pl.msz), pl.k), dim3(kDW), 0, st, w.Dbar, dd, pl.k, pl.g[0], pl.g[1],
                     pl.g[2], pl.fs[0], pl.fs[1], pl.fs[2], accumulate ? 1 : 0);
  return hipGetLastError();
}

// The forward runs the coding path's iteration (the updates of
// eq:Inference_solution in implicit-theta form) and records the checkpoints
// as it passes them; the reverse pass replays each segment with the same
// iteration from its record (so the states, and with them the gradient, do
// not depend on the checkpoint interval) and differentiates the literal
// iteration above at each state.
int run_unrolled(const Plan& pl, const float* b, const float* d, float beta, const float* rho, int iters, int every,
                 float* z, float* ckpt, void* ws, hipStream_t st) {
  return run_code(pl, b, d, beta, const_cast<float*>(rho), iters, CSC_Z_ZERO | CSC_THETA_ZERO, z, nullptr, nullptr,
                  ws, st, 0.0f, nullptr, ckpt, every);
}

int run_backward(const Plan& pl, const float* b, const float* d, float beta, const float* rho, int iters, int every,
                 const float* ckpt, const float* zbar_in, float* dd, double* dbeta, void* ws, hipStream_t st) {
  DiffWs w;
  carve_diff(pl, every, ws, &w);
  const int64_t D = pl.dsz, nz = int64_t(pl.n) * pl.k * D;
  if (setup_spectra(pl, b, d, w.cw, st) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(d_copy, dim3(dblk(nz)), dim3(kDW), 0, st, w.zbar, zbar_in, nz);
  hipLaunchKernelGGL(d_zero, dim3(dblk(nz)), dim3(kDW), 0, st, w.thbar, nz);
  hipLaunchKernelGGL(d_zero, dim3(dblk(int64_t(pl.p) * D * 2)), dim3(kDW), 0, st, (float*)w.Dbar,
                     int64_t(pl.p) * D * 2);
  hipLaunchKernelGGL(d_zero_d, dim3(dblk(w.nbpart)), dim3(kDW), 0, st, w.bpart, w.nbpart);
  const int nseg = (iters + every - 1) / every;
  for (int sgi = nseg - 1; sgi >= 0; --sgi) {
    const int c0 = sgi * every, len = (iters - c0 < every) ? iters - c0 : every;
    const float* ck = ckpt + int64_t(sgi) * code_record_floats(pl);
    // states c0 .. c0 + len - 1, and for the last segment also the final one
    // (the codes after each state's iteration decide its clip branches)
    const bool last_seg = sgi == nseg - 1;
    if (replay_code(pl, w.cw, rho, beta, ck, len + (last_seg ? 1 : 0), w.seg, st) != hipSuccess) return CSC_EHIP;
    for (int i = len - 1; i >= 0; --i) {
      // state i of the segment: the record (i = 0) or replay slot i - 1
      const float* zi = i == 0 ? ck : w.seg + int64_t(i - 1) * 2 * nz;
      const float* znext = (i + 1 < len || last_seg) ? w.seg + int64_t(i) * 2 * nz
                                                     : ckpt + int64_t(sgi + 1) * code_record_floats(pl);
      if (adjoint_iter(pl, w, zi, zi + nz, znext, rho, st) != hipSuccess) return CSC_EHIP;
    }
  }
  if (finish_taps(pl, w, dd, false, st) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(d_sum, dim3(1), dim3(kSumT), 0, st, w.bpart, w.nbpart, dbeta);
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

int run_loss_grad(const Plan& pl, const float* b, const float* d, const float* z, float beta, double* loss,
                  float* zbar, float* dd, double* dbeta, void* ws, hipStream_t st) {
  DiffWs w;
  carve_diff(pl, 1, ws, &w);
  const int64_t D = pl.dsz;
  const dim3 g3(dblk(D), pl.p, pl.n);
  if (setup_spectra(pl, b, d, w.cw, st) != hipSuccess) return CSC_EHIP;
  if (forward_maps(pl, z, w.cw, w.cw.rpri, st) != hipSuccess) return CSC_EHIP;
  launch_objective_tail(pl, w.cw, beta, loss, st);
  launch_sym_reduce(pl, w.cw.part, w.cw.ngp, w.cw.yh, st);
  const int64_t ns = int64_t(pl.n) * D;
  hipLaunchKernelGGL(d_sub, dim3(dblk(ns)), dim3(kDW), 0, st, w.cw.yh, w.cw.xh, w.lam, ns);  // res hat
  launch_make_v(pl, w.cw.E, w.lam, w.Vb, st);
  if (fft_grids(w.Vb, int64_t(pl.n) * pl.p, pl.g, +1, st) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(d_zbar_loss, g3, dim3(kDW), 0, st, w.Vb, z, zbar, beta, pl.k, pl.p, D);
  hipLaunchKernelGGL(d_pack_z, g3, dim3(kDW), 0, st, z, w.Wb, pl.k, pl.p, D);
  if (fft_grids(w.Wb, int64_t(pl.n) * pl.p, pl.g, -1, st) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(d_zero, dim3(dblk(int64_t(pl.p) * D * 2)), dim3(kDW), 0, st, (float*)w.Dbar,
                     int64_t(pl.p) * D * 2);
  hipLaunchKernelGGL(d_dbar, dim3(dblk(D), pl.p), dim3(kDW), 0, st, w.Wb, (const float2*)nullptr, w.cw.E, w.lam,
                     (const float2*)nullptr, w.Dbar, pl.n, pl.p, pl.g[0], pl.g[1], pl.g[2]);
  if (finish_taps(pl, w, dd, false, st) != hipSuccess) return CSC_EHIP;
  hipLaunchKernelGGL(d_sum, dim3(1), dim3(kSumT), 0, st, w.cw.rpri, int64_t(pl.n) * w.cw.npri, dbeta);
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

}  // namespace dcsc
