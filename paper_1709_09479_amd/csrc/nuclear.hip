// Nuclear-norm regulariser on the code maps (Sec. 5: a nuclear norm on the
// sparse maps makes them low rank).  The coding problem becomes
//   min_z 1/2 ||x - sum_k d_k * z_k||^2 + beta sum_k ||z_k||_*
// and the dual ADMM of eq:Inference_solution keeps every update except the
// projection Pi_C, now onto the beta-ball of the spectral norm (the dual norm
// of the nuclear norm), one H x W map at a time.  In the implicit-theta form
// of the coding loop the z step becomes singular value thresholding:
//   z' = z + rho (Pi_C(v - z/rho) - v) = SVT(z - rho v, rho beta),
//   SVT(u, t) = U diag(max(s - t, 0)) V^T.
//
// One workgroup per map.  The map u = z - rho v (an NR x NC matrix A with
// NC <= NR: columns are the map's columns, or its rows when W > H) goes to
// LDS in float64, and a one-sided (Hestenes) Jacobi method orthogonalises
// its columns by plane rotations, B = A V; the pairs of each round come from
// the round-robin (circle) ordering, so the NC/2 rotations of a round touch
// disjoint columns and run in parallel.  Sweeps repeat until one applies no
// rotation (every pair has |b_i . b_j| <= 1e-12 ||b_i|| ||b_j||), at most
// kSvtSweeps.  Then sigma_i = ||b_i||, u_i = b_i / sigma_i and
// v_i = A^T b_i / sigma_i^2, so
//   SVT(A, t) = sum_{sigma_i > t} (1 - t/sigma_i) / sigma_i^2 b_i (A^T b_i)^T,
// formed a block of CH columns at a time (A is read again from global
// memory; each block's columns are written only after they have been read).
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace dcsc {

constexpr int kSvtT = 1024;       // threads per workgroup
constexpr int kSvtSweeps = 40;    // sweep limit of the Jacobi method
constexpr int kSvtCH = 16;        // output columns per block
constexpr double kSvtTol = 1e-12;  // rotation threshold (relative)

constexpr int svt_lp(int NR, int NC) {
  // lanes per column pair: the rounds' NC/2 pairs spread over the workgroup
  return std::min(64, std::min(NR, kSvtT / (NC / 2 > 0 ? NC / 2 : 1)));
}

// x + the value of lane (lane ^ m) within rows of 16 lanes, through the
// data-parallel-primitive lane moves of one 32-bit half at a time (no LDS):
// CTRL 0xB1 (quad xor 1), 0x4E (quad xor 2), 0x141 (half-row mirror),
// 0x140 (row mirror).  Each lane adds the same two values as its partner,
// so after the steps every lane of the group holds the same sum.
template <int CTRL>
__device__ __forceinline__ double dpp_add(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return x + __hiloint2double(hi, lo);
}

// Sum over the LP lanes of a group (LP a power of two, groups aligned).
template <int LP>
__device__ __forceinline__ double group_sum(double x) {
  if constexpr (LP >= 2) x = dpp_add<0xB1>(x);
  if constexpr (LP >= 4) x = dpp_add<0x4E>(x);
  if constexpr (LP >= 8) x = dpp_add<0x141>(x);
  if constexpr (LP >= 16) x = dpp_add<0x140>(x);
#pragma unroll
  for (int off = 16; off < LP; off <<= 1) x += __shfl_xor(x, off, LP);
  return x;
}

// Pair q of round t of the circle ordering of NC columns: column 0 stays,
// the others rotate; over the NC - 1 rounds every pair meets once.
__device__ __forceinline__ void svt_pair(int t, int q, int NC, int& a, int& b) {
  const int M = NC - 1;
  if (q == 0) {
    a = 0;
    b = 1 + t % M;
  } else {
    a = 1 + (t + q) % M;
    b = 1 + (t - q + M) % M;
  }
}

// MODE 0: one ADMM z step on map k of image n (z' = SVT(z - rho v, rho beta)
// with v = buf component / D, theta' = v + (z' - z)/rho when theta is given,
// buf component <- z', rmap[n][k] = sum (z' - z)^2).  MODE 1: rmap[n][k] =
// nuclear norm of z_k.  TR: the matrix is the map transposed (W > H).
template <int NR, int NC>
__global__ __launch_bounds__(kSvtT) void k_svt(float2* __restrict__ buf, float* __restrict__ z,
                                               const float* __restrict__ zin, float* __restrict__ theta,
                                               const int64_t* __restrict__ zoff, const float* __restrict__ rho_cur,
                                               float beta, double* __restrict__ rmap, int K, int P, int tr, int mode,
                                               const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int LDB = NR + 1;                 // odd column stride (doubles)
  constexpr int LP = svt_lp(NR, NC);          // lanes per pair
  constexpr int RPL = NR / LP;                // rows per lane
  constexpr int NGRP = kSvtT / LP;            // pair groups
  constexpr int D = NR * NC;
  __shared__ double Bm[NC * LDB];
  __shared__ double aux[kSvtCH * LDB];        // a block of A, then of G = A^T B
  __shared__ double coef[NC];
  __shared__ int flag;
  __shared__ double red[kSvtT / 64];
  const int k = blockIdx.x, n = blockIdx.y, tid = (int)threadIdx.x;
  const int H = tr ? NC : NR, W = tr ? NR : NC;
  const int64_t zbase = map_base(zoff, n, K, D) + int64_t(k) * D;
  const float* zsrc = zin ? zin : z;
  float* bcomp = reinterpret_cast<float*>(buf) + 2 * (int64_t(n) * P + k / 2) * D + (k & 1);
  const float rho = mode == 0 ? rho_cur[n] : 1.0f, invD = 1.0f / (float)D;
  // element f = h W + w of the map <-> (row r, column c) of A
  auto rc_of = [&](int f, int& r, int& c) {
    const int h = f / W, w = f - h * W;
    r = tr ? w : h;
    c = tr ? h : w;
  };
  auto f_of = [&](int r, int c) { return tr ? c * W + r : r * W + c; };
  // A = z - rho v (z alone for the norm)
  auto a_at = [&](int f) -> double {
    const float zz = zsrc[zbase + f];
    if (mode != 0) return (double)zz;
    const float v = bcomp[2 * int64_t(f)] * invD;
    return (double)fmaf(-rho, v, zz);
  };
  for (int f = tid; f < D; f += kSvtT) {
    int r, c;
    rc_of(f, r, c);
    Bm[c * LDB + r] = a_at(f);
  }
  if (mode == 0) {
    // ---- SVT(A, t) = 0 when every singular value is below t = rho beta,
    // i.e. when t^2 I - A^T A is positive definite: a Cholesky factorisation
    // of that NC x NC matrix in LDS (O(NC^3)) settles it before the Jacobi
    // sweeps (O(sweeps NC^2 NR)).  A failed pivot (or one lost to rounding
    // at sigma ~ t) leaves the decision to the sweeps.
    const double t2 = (double)rho * (double)beta * (double)rho * (double)beta;
    // G = A^T A in 4 x 4 blocks, one block per thread, in registers
    constexpr int NB4 = NC / 4;
    static_assert(NB4 * NB4 <= kSvtT, "one 4 x 4 block of A^T A per thread");
    double g4[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) g4[x][y] = 0.0;
    const int bi = tid / NB4, bj = tid % NB4;
    __syncthreads();  // A is in Bm
    if (tid < NB4 * NB4) {
      for (int r = 0; r < NR; ++r) {
        double a4[4], b4[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          a4[x] = Bm[(4 * bi + x) * LDB + r];
          b4[x] = Bm[(4 * bj + x) * LDB + r];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) g4[x][y] = fma(a4[x], b4[y], g4[x][y]);
      }
    }
    __syncthreads();  // every thread is done with A
    // Bm[i][j] <- (t^2 I - A^T A)[i][j]
    if (tid < NB4 * NB4) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int i = 4 * bi + x, j = 4 * bj + y;
          Bm[i * LDB + j] = (i == j ? t2 : 0.0) - g4[x][y];
        }
    }
    if (tid == 0) flag = 0;
    for (int j = 0; j < NC; ++j) {
      __syncthreads();  // the previous step's update (and the flag) are done
      const double piv = Bm[j * LDB + j];
      if (!(piv > 0.0)) {  // the same value in every thread: a uniform exit
        if (tid == 0) flag = 1;
        break;
      }
      const double inv = 1.0 / sqrt(piv);
      for (int i = j + 1 + tid; i < NC; i += kSvtT) Bm[i * LDB + j] *= inv;
      __syncthreads();
      const int m = NC - j - 1;
      for (int e = tid; e < m * m; e += kSvtT) {
        const int i = j + 1 + e / m, c = j + 1 + e % m;
        if (c <= i) Bm[i * LDB + c] -= Bm[i * LDB + j] * Bm[c * LDB + j];
      }
    }
    __syncthreads();
    if (flag == 0) {
      // z' = 0: theta' = v - z/rho, the map's pair slot <- 0, rmap = sum z^2
      const float inv_rho = 1.0f / rho;
      double rs = 0.0;
      for (int f = tid; f < D; f += kSvtT) {
        const float z0 = zsrc[zbase + f];
        const float v = bcomp[2 * int64_t(f)] * invD;
        rs = fma((double)z0, (double)z0, rs);
        z[zbase + f] = 0.f;
        if (theta) theta[zbase + f] = v - z0 * inv_rho;
        bcomp[2 * int64_t(f)] = 0.f;
        if ((K & 1) && k == K - 1) bcomp[2 * int64_t(f) + 1] = 0.f;
      }
      const double tot = block_sum(rs, red);
      if (tid == 0) rmap[int64_t(n) * K + k] = tot;
      return;
    }
    // the sweeps start from A again
    for (int f = tid; f < D; f += kSvtT) {
      int r, c;
      rc_of(f, r, c);
      Bm[c * LDB + r] = a_at(f);
    }
  }
  // ---- one-sided Jacobi sweeps
  const int grp = tid / LP, sub = tid % LP;
  for (int sweep = 0; sweep < kSvtSweeps; ++sweep) {
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int t = 0; t < NC - 1; ++t) {
      for (int q = grp; q < NC / 2; q += NGRP) {
        int a, b;
        svt_pair(t, q, NC, a, b);
        double* ca = Bm + a * LDB;
        double* cb = Bm + b * LDB;
        double x[RPL], y[RPL];
        double aa = 0.0, bb = 0.0, ab = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          x[i] = ca[sub + i * LP];
          y[i] = cb[sub + i * LP];
          aa = fma(x[i], x[i], aa);
          bb = fma(y[i], y[i], bb);
          ab = fma(x[i], y[i], ab);
        }
        aa = group_sum<LP>(aa);
        bb = group_sum<LP>(bb);
        ab = group_sum<LP>(ab);
        if (ab != 0.0 && fabs(ab) > kSvtTol * sqrt(aa * bb)) {
          const double zeta = (bb - aa) / (2.0 * ab);
          const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
#pragma unroll
          for (int i = 0; i < RPL; ++i) {
            ca[sub + i * LP] = cs * x[i] - sn * y[i];
            cb[sub + i * LP] = sn * x[i] + cs * y[i];
          }
          if (sub == 0) flag = 1;
        }
      }
      __syncthreads();
    }
    const int more = flag;
    __syncthreads();
    if (!more) break;
  }
  // ---- singular values: sigma_i = ||b_i||
  for (int c = grp; c < NC; c += NGRP) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const double x = Bm[c * LDB + sub + i * LP];
      s = fma(x, x, s);
    }
    s = group_sum<LP>(s);
    if (sub == 0) coef[c] = sqrt(s);
  }
  __syncthreads();
  if (mode != 0) {
    double s = 0.0;
    for (int c = tid; c < NC; c += kSvtT) s += coef[c];
    const double tot = block_sum(s, red);
    if (tid == 0) rmap[int64_t(n) * K + k] = tot;
    return;
  }
  const double thr = (double)rho * (double)beta;
  __syncthreads();
  for (int c = tid; c < NC; c += kSvtT) {
    const double s = coef[c];
    coef[c] = s > thr ? (1.0 - thr / s) / (s * s) : 0.0;
  }
  // ---- output, a block of kSvtCH columns of A at a time
  const float inv_rho = 1.0f / rho;
  double rs = 0.0;
  for (int c0 = 0; c0 < NC; c0 += kSvtCH) {
    constexpr int CH = kSvtCH < NC ? kSvtCH : NC;
    __syncthreads();  // previous block's readers of aux are done
    for (int e = tid; e < CH * NR; e += kSvtT) {
      // consecutive threads take consecutive map positions where possible
      const int cc = tr ? e / NR : e % CH, r = tr ? e % NR : e / CH;
      aux[cc * LDB + r] = a_at(f_of(r, c0 + cc));
    }
    __syncthreads();
    // G[cc][i] = sum_r A[r][c0 + cc] b_i[r] (only where coef_i != 0)
    constexpr int GPT = (CH * NC + kSvtT - 1) / kSvtT;
    double g[GPT];
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int e = tid + u * kSvtT;
      g[u] = 0.0;
      if (e < CH * NC) {
        const int i = e % NC, cc = e / NC;
        if (coef[i] != 0.0) {
          const double* bi = Bm + i * LDB;
          const double* ac = aux + cc * LDB;
          double s = 0.0;
          for (int r = 0; r < NR; ++r) s = fma(ac[r], bi[r], s);
          g[u] = s * coef[i];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int e = tid + u * kSvtT;
      if (e < CH * NC) aux[(e / NC) * LDB + (e % NC)] = g[u];
    }
    __syncthreads();
    // z'[r][c0 + cc] = sum_i b_i[r] G'[cc][i]
    for (int e = tid; e < CH * NR; e += kSvtT) {
      const int cc = tr ? e / NR : e % CH, r = tr ? e % NR : e / CH;
      const double* gc = aux + cc * LDB;
      double s = 0.0;
      for (int i = 0; i < NC; ++i) s = fma(Bm[i * LDB + r], gc[i], s);
      const int f = f_of(r, c0 + cc);
      const float z0 = zsrc[zbase + f];
      const float v = bcomp[2 * int64_t(f)] * invD;
      const float z1 = (float)s;
      const float dz = z1 - z0;
      rs = fma((double)dz, (double)dz, rs);
      z[zbase + f] = z1;
      if (theta) theta[zbase + f] = v + dz * inv_rho;
      bcomp[2 * int64_t(f)] = z1;
      // the other half of the last pair of an odd K carries no map
      if ((K & 1) && k == K - 1) bcomp[2 * int64_t(f) + 1] = 0.f;
    }
  }
  const double tot = block_sum(rs, red);
  if (tid == 0) rmap[int64_t(n) * K + k] = tot;
}

bool nuclear_supported(int T, int H, int W) { return T == 1 && H >= 8 && W >= 8 && H <= 128 && W <= 128; }

hipError_t launch_svt(const Plan& pl, float2* buf, float* z, const float* zin, float* theta, const float* rho,
                      float beta, double* rmap, int mode, hipStream_t st, const int* stop) {
  const int H = pl.g[1], W = pl.g[2];
  if (!nuclear_supported(pl.g[0], H, W)) return hipErrorInvalidValue;
  const int tr = W > H ? 1 : 0;
  const int NR = tr ? W : H, NC = tr ? H : W;
  const dim3 grid((unsigned)pl.k, (unsigned)pl.n), block(kSvtT);
#define SVT(R, C)                                                                                        \
  if (NR == R && NC == C) {                                                                              \
    hipLaunchKernelGGL((k_svt<R, C>), grid, block, 0, st, buf, z, zin, theta, pl.zoff, rho, beta, rmap, \
                       pl.k, pl.p, tr, mode, stop);                                                      \
    return hipGetLastError();                                                                            \
  }
  SVT(8, 8) SVT(16, 8) SVT(16, 16) SVT(32, 8) SVT(32, 16) SVT(32, 32)
  SVT(64, 8) SVT(64, 16) SVT(64, 32) SVT(64, 64)
  SVT(128, 8) SVT(128, 16) SVT(128, 32) SVT(128, 64) SVT(128, 128)
#undef SVT
  return hipErrorInvalidValue;
}

}  // namespace dcsc
