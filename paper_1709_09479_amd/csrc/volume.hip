// Coding map work on 3-D grids whose H x W plane fits one LDS tile and whose
// T <= 16 frames fit a thread's registers (the video form of Sec. 3.3):
// the separable 3-D transforms of one ADMM iteration (eq:Inference_solution)
// are split by axis so that each intermediate crosses HBM once each way:
//   k_vol_inv    per (image, pair, frame): V = sum_j lam_j E_jp formed while
//                loading, inverse 2-D DFT of the plane in LDS, plane to buf;
//   k_vol_lines  per (image, pair, 256 positions): the T-point inverse DFT of
//                each position's frame line in registers, the soft-threshold
//                step of both maps of the pair (z, theta, residual partials),
//                the T-point forward DFT, line back to buf;
//   k_vol_fwd    per (image, pair, frame): forward 2-D DFT of the plane in
//                LDS, plane to buf.
// k_accum and k_spec then reduce over the pairs as on the axis-pass path,
// which this replaces (make_v, three inverse axis passes, the spatial step,
// three forward axis passes).
#include "common.hpp"
#include "internal.hpp"
#include "tiles.hpp"

namespace dcsc {

constexpr int kVolLines = 256;  // frame lines per k_vol_lines workgroup

template <int H, int W, int J>
__global__ __launch_bounds__(fused_threads(H * W, 1)) void k_vol_inv(const float2* __restrict__ E,
                                                                    const float2* __restrict__ lam,
                                                                    float2* __restrict__ buf, int P, int T,
                                                                    const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int NT = fused_threads(H * W, 1), WP = tile_stride(W), HW = H * W;
  using PL = TilePlan<H, W, NT, WP>;
  using P1 = typename PL::InvRow0;
  using P4 = typename PL::InvColL;
  __shared__ float2 tile[H * WP];
  __shared__ float2 tw[256];
  load_twiddles(tw);
  const int t = (int)blockIdx.x % T, p = ((int)blockIdx.x / T) % P, n = (int)blockIdx.x / T / P;
  const int64_t D = int64_t(T) * HW, po = int64_t(t) * HW;
  const float2* lamn = lam + int64_t(n) * J * D + po;
  const float2* Ep[J];
#pragma unroll
  for (int c = 0; c < J; ++c) Ep[c] = E + (int64_t(c) * P + p) * D + po;
  const int tid = opaque_tid();
#pragma unroll
  for (int q = 0; q < P1::JPT; ++q) {
    int b, j;
    if (!P1::job(tid, q, b, j)) continue;
    float2 v1[P1::R];
#pragma unroll
    for (int r = 0; r < P1::R; ++r) {
      const int f = b * W + P1::in_pos(j, r);
      float2 v = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < J; ++c) v = cadd(v, cmul(lamn[c * D + f], Ep[c][f]));
      v1[r] = v;
    }
    dft<P1::R, 1>(v1);
#pragma unroll
    for (int r = 0; r < P1::R; ++r) tile[P1::addr(b, P1::out_pos(j, r))] = v1[r];
  }
  __syncthreads();
  if constexpr (PL::NA == 2) pass_lds<typename PL::InvRow1>(tile, tw);
  if constexpr (PL::NB == 2) pass_lds<typename PL::InvCol0>(tile, tw);
  float2 v4[P4::JPT][P4::R];
  pass_to_regs<P4>(tid, tile, tw, v4);
  float2* g = buf + (int64_t(n) * P + p) * D + po;
#pragma unroll
  for (int q = 0; q < P4::JPT; ++q) {
    int b, j;
    if (!P4::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < P4::R; ++r) g[P4::out_pos(j, r) * W + b] = v4[q][r];
  }
}

// rpart [N][P * nblk * TT] (nblk = lines / kVolLines): sum (z' - z)^2 of
// block blk in slot blk * TT, zeros in the TT - 1 slots after it, so that
// the partials have the layout of the other kernels of the 3-D path (one
// slot per 256 grid points of each pair).
template <int TT>
__global__ __launch_bounds__(kVolLines) void k_vol_lines(float2* __restrict__ buf, float* __restrict__ z,
                                                         float* __restrict__ theta, const float* __restrict__ rho_cur,
                                                         float beta, double* __restrict__ rpart, int K, int P, int HW,
                                                         int nblk, const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  __shared__ double red[kVolLines / 64];
  const int blk = (int)blockIdx.x % nblk, p = ((int)blockIdx.x / nblk) % P, n = (int)blockIdx.x / nblk / P;
  const int hw = blk * kVolLines + (int)threadIdx.x;
  const int64_t D = int64_t(TT) * HW;
  double s = 0.0;
  if (hw < HW) {
    const float rho = rho_cur[n], thr = rho * beta, inv_rho = 1.0f / rho, invD = 1.0f / (float)D;
    const int ka = 2 * p, kb = 2 * p + 1;
    const bool hb = kb < K;
    float2* g = buf + (int64_t(n) * P + p) * D + hw;
    float* za = z + (int64_t(n) * K + ka) * D + hw;
    float* zb = z + (int64_t(n) * K + (hb ? kb : ka)) * D + hw;
    float2 v[TT];
    float a0[TT], b0[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      v[t] = g[int64_t(t) * HW];
      a0[t] = za[int64_t(t) * HW];
      b0[t] = hb ? zb[int64_t(t) * HW] : 0.f;
    }
    dft<TT, 1>(v);
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      const int64_t o = int64_t(t) * HW;
      const float va = v[t].x * invD, vb = v[t].y * invD;
      const float a1 = soft_thresh(fmaf(-rho, va, a0[t]), thr);
      const float b1 = hb ? soft_thresh(fmaf(-rho, vb, b0[t]), thr) : 0.f;
      const double da = (double)a1 - a0[t], db = (double)b1 - b0[t];
      s += da * da + db * db;
      za[o] = a1;
      if (hb) zb[o] = b1;
      if (theta) {
        theta[(int64_t(n) * K + ka) * D + hw + o] = va + (a1 - a0[t]) * inv_rho;
        if (hb) theta[(int64_t(n) * K + kb) * D + hw + o] = vb + (b1 - b0[t]) * inv_rho;
      }
      v[t] = make_float2(a1, b1);
    }
    dft<TT, -1>(v);
#pragma unroll
    for (int t = 0; t < TT; ++t) g[int64_t(t) * HW] = v[t];
  }
  const double tot = block_sum(s, red);
  if (threadIdx.x < TT) rpart[((int64_t(n) * P + p) * nblk + blk) * TT + threadIdx.x] = threadIdx.x == 0 ? tot : 0.0;
}

template <int H, int W>
__global__ __launch_bounds__(fused_threads(H * W, 1)) void k_vol_fwd(float2* __restrict__ buf, int P, int T,
                                                                    const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int NT = fused_threads(H * W, 1), WP = tile_stride(W), HW = H * W;
  using PL = TilePlan<H, W, NT, WP>;
  using P6 = typename PL::FwdCol0;
  using P8 = typename PL::FwdRowL;
  __shared__ float2 tile[H * WP];
  __shared__ float2 tw[256];
  load_twiddles(tw);
  const int t = (int)blockIdx.x % T, p = ((int)blockIdx.x / T) % P, n = (int)blockIdx.x / T / P;
  const int64_t D = int64_t(T) * HW;
  float2* g = buf + (int64_t(n) * P + p) * D + int64_t(t) * HW;
  const int tid = opaque_tid();
  float2 v[P6::JPT][P6::R];
#pragma unroll
  for (int q = 0; q < P6::JPT; ++q) {
    int b, j;
    if (!P6::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < P6::R; ++r) v[q][r] = g[P6::in_pos(j, r) * W + b];
  }
  pass_from_regs<P6>(tid, tile, v);
  if constexpr (PL::NB == 2) pass_lds<typename PL::FwdCol1>(tile, tw);
  if constexpr (PL::NA == 2) pass_lds<typename PL::FwdRow0>(tile, tw);
  float2 u[P8::JPT][P8::R];
  pass_to_regs<P8>(tid, tile, tw, u);
#pragma unroll
  for (int q = 0; q < P8::JPT; ++q) {
    int b, j;
    if (!P8::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < P8::R; ++r) g[b * W + P8::out_pos(j, r)] = u[q][r];
  }
}

// ================================================================== host

bool vol_supported(int T, int H, int W) { return T >= 2 && T <= 16 && tile_supported(H, W); }

static int vol_line_blocks(const Plan& pl) { return (pl.g[1] * pl.g[2] + kVolLines - 1) / kVolLines; }

template <int H, int W>
static void vol_tile_launch(const Plan& pl, const float2* E, const float2* lam, float2* buf, bool fwd, hipStream_t st,
                            const int* stop) {
  const dim3 grid((unsigned)(int64_t(pl.n) * pl.p * pl.g[0])), blk(fused_threads(H * W, 1));
  if (fwd) {
    hipLaunchKernelGGL((k_vol_fwd<H, W>), grid, blk, 0, st, buf, pl.p, pl.g[0], stop);
  } else if (pl.j == 1) {
    hipLaunchKernelGGL((k_vol_inv<H, W, 1>), grid, blk, 0, st, E, lam, buf, pl.p, pl.g[0], stop);
  } else if (pl.j == 2) {
    hipLaunchKernelGGL((k_vol_inv<H, W, 2>), grid, blk, 0, st, E, lam, buf, pl.p, pl.g[0], stop);
  } else {
    hipLaunchKernelGGL((k_vol_inv<H, W, 3>), grid, blk, 0, st, E, lam, buf, pl.p, pl.g[0], stop);
  }
}

static bool vol_tiles(const Plan& pl, const float2* E, const float2* lam, float2* buf, bool fwd, hipStream_t st,
                      const int* stop) {
  const int h = pl.g[1], w = pl.g[2];
#define VT(HH, WW)                                                \
  if (h == HH && w == WW) {                                       \
    vol_tile_launch<HH, WW>(pl, E, lam, buf, fwd, st, stop);      \
    return true;                                                  \
  }
  VT(16, 16) VT(16, 32) VT(16, 64) VT(16, 128) VT(16, 256)
  VT(32, 16) VT(32, 32) VT(32, 64) VT(32, 128) VT(32, 256)
  VT(64, 16) VT(64, 32) VT(64, 64) VT(64, 128) VT(64, 256)
  VT(128, 16) VT(128, 32) VT(128, 64) VT(128, 128)
  VT(256, 16) VT(256, 32) VT(256, 64)
#undef VT
  return false;
}

hipError_t vol_maps(const Plan& pl, const float2* E, const float2* lam, float2* buf, float* z, float* theta,
                    const float* rho, float beta, double* rpart, hipStream_t st, const int* stop) {
  if (!pl.vol) return hipErrorInvalidValue;
  if (!vol_tiles(pl, E, lam, buf, false, st, stop)) return hipErrorInvalidValue;
  const int nb = vol_line_blocks(pl), HW = pl.g[1] * pl.g[2];
  const dim3 grid((unsigned)(int64_t(pl.n) * pl.p * nb)), blk(kVolLines);
  switch (pl.g[0]) {
    case 2: hipLaunchKernelGGL(k_vol_lines<2>, grid, blk, 0, st, buf, z, theta, rho, beta, rpart, pl.k, pl.p, HW, nb, stop); break;
    case 4: hipLaunchKernelGGL(k_vol_lines<4>, grid, blk, 0, st, buf, z, theta, rho, beta, rpart, pl.k, pl.p, HW, nb, stop); break;
    case 8: hipLaunchKernelGGL(k_vol_lines<8>, grid, blk, 0, st, buf, z, theta, rho, beta, rpart, pl.k, pl.p, HW, nb, stop); break;
    case 16: hipLaunchKernelGGL(k_vol_lines<16>, grid, blk, 0, st, buf, z, theta, rho, beta, rpart, pl.k, pl.p, HW, nb, stop); break;
    default: return hipErrorInvalidValue;
  }
  if (!vol_tiles(pl, E, lam, buf, true, st, stop)) return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace dcsc
