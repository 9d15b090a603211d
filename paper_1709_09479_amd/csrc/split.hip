// Coding iteration for 2-D grids too large for one LDS tile (128 x 256,
// 256 x 128, 256 x 256): the map work of one ADMM iteration (back-projection
// D^T lambda, soft threshold, forward transform and reduction, see
// eq:Inference_solution) split into a row phase, a column phase and a row
// phase, so that every intermediate crosses HBM once each way:
//   rows inverse   buf[n][p] = row-IDFT of V = sum_j lam_j E_jp
//   columns        column-IDFT, soft-threshold step on the map pair (z in
//                  place, residual partials), column-DFT; buf in place
//   rows forward   row-DFT, times conj(E_jp), summed over the pairs of a
//                  group into part[n][g][j]
// Each workgroup stages a 4096-element tile (rows x W, or H x columns) in LDS
// and runs the same register hand-off passes as the single-tile kernel.
#include "common.hpp"
#include "internal.hpp"

namespace dcsc {

constexpr int kSplitT = 4096;   // complex elements per workgroup tile
constexpr int kSplitNT = 256;   // threads per workgroup

// ---------------------------------------------------------- rows inverse
template <int W, int J>
__global__ __launch_bounds__(kSplitNT) void k_split_rows_inv(const float2* __restrict__ E,
                                                             const float2* __restrict__ lam,
                                                             float2* __restrict__ buf, int P, int H,
                                                             const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int T = kSplitT, NT = kSplitNT, RB = T / W, WP = tile_stride(W);
  constexpr int A0 = plan_r(W, 0), AL = plan_r(W, 1);
  using P0 = TilePass<W, T, NT, 1, A0, 1, true, true, WP>;
  using P1 = TilePass<W, T, NT, 1, AL, A0, true, true, WP>;
  static_assert(plan_n(W) == 2, "two passes per row");
  __shared__ float2 tile[RB * WP];
  __shared__ float2 tw[256];
  load_twiddles(tw);
  // items (row chunk, pair)-major, images fastest, spread over the XCDs so
  // that the images of one XCD share rows of E in its L2
  const int N = (int)(gridDim.x / (unsigned)(P * (H / RB)));
  const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);
  const int n = item % N, p = (item / N) % P, rc = item / N / P;
  const int64_t D = int64_t(H) * W, row0 = int64_t(rc) * RB;
  const float2* lamn = lam + int64_t(n) * J * D;
  const float2* Ep[J];
#pragma unroll
  for (int c = 0; c < J; ++c) Ep[c] = E + (int64_t(c) * P + p) * D;
  const int tid = opaque_tid();
  float2 v[P0::JPT][P0::R];
#pragma unroll
  for (int q = 0; q < P0::JPT; ++q) {
    int b, j;
    if (!P0::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < P0::R; ++r) {
      const int64_t f = (row0 + b) * W + P0::in_pos(j, r);
      float2 s = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < J; ++c) s = cadd(s, cmul(lamn[c * D + f], Ep[c][f]));
      v[q][r] = s;
    }
  }
  pass_from_regs<P0>(tid, tile, v);
  float2 u[P1::JPT][P1::R];
  pass_to_regs<P1>(tid, tile, tw, u);
  float2* g = buf + (int64_t(n) * P + p) * D;
#pragma unroll
  for (int q = 0; q < P1::JPT; ++q) {
    int b, j;
    if (!P1::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < P1::R; ++r) g[(row0 + b) * W + P1::out_pos(j, r)] = u[q][r];
  }
}

// ---------------------------------------------------------------- columns
// MODE 0 (iteration): column-IDFT, soft-threshold step, column-DFT; the
// codes are read from zin (the same layout as z; null: z itself, updated in
// place) and written to z.
// MODE 1 (forward only): the map pair enters from z, l1 partials.
// rpart[n][p * gridDim.x + blockIdx.x]: sum (z' - z)^2, or sum |z|.
template <int H, int MODE>
__global__ __launch_bounds__(kSplitNT) void k_split_cols(float2* __restrict__ buf, float* __restrict__ z,
                                                         const float* zin,
                                                         float* __restrict__ theta, const int64_t* __restrict__ zoff,
                                                         const float* __restrict__ rho_cur, float beta,
                                                         double* __restrict__ rpart, int K, int P, int W,
                                                         const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int T = kSplitT, NT = kSplitNT, CB = T / H, WP = tile_stride(CB);
  constexpr int B0 = plan_r(H, 0), BL = plan_r(H, 1);
  using C0 = TilePass<H, T, NT, 1, B0, 1, false, false, WP>;
  using CL = TilePass<H, T, NT, 1, BL, H / BL, false, false, WP>;
  using F0 = TilePass<H, T, NT, -1, BL, 1, false, false, WP>;
  using F1 = TilePass<H, T, NT, -1, B0, BL, false, false, WP>;
  static_assert(CL::JPT == F0::JPT && CL::R == F0::R, "register hand-off mismatch");
  __shared__ float2 tile[H * WP];
  __shared__ float2 tw[256];
  __shared__ double red[NT / 64];
  load_twiddles(tw);
  const int cb = blockIdx.x, p = blockIdx.y, n = blockIdx.z;
  const int64_t D = int64_t(H) * W;
  const int c0 = cb * CB;
  float2* g = buf + (int64_t(n) * P + p) * D;
  const int ka = 2 * p, kb = 2 * p + 1;
  const bool hb = kb < K;
  const int64_t zbase = map_base(zoff, n, K, D);
  float* za = z + zbase + int64_t(ka) * D;
  float* zb = z + zbase + int64_t(hb ? kb : ka) * D;
  const float* zsrc = (MODE == 0 && zin) ? zin : z;
  const float* zia = zsrc + zbase + int64_t(ka) * D;
  const float* zib = zsrc + zbase + int64_t(hb ? kb : ka) * D;
  const int tid = opaque_tid();
  double rsum = 0.0;
  float2 v[F0::JPT][F0::R];
  if constexpr (MODE == 0) {
    const float rho = rho_cur[n], thr = rho * beta, inv_rho = 1.0f / rho, invD = 1.0f / (float)D;
    float2 a[C0::JPT][C0::R];
#pragma unroll
    for (int q = 0; q < C0::JPT; ++q) {
      int b, j;
      if (!C0::job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < C0::R; ++r) a[q][r] = g[int64_t(C0::in_pos(j, r)) * W + c0 + b];
    }
    pass_from_regs<C0>(tid, tile, a);
    pass_to_regs<CL>(tid, tile, tw, v);
    float* tha = theta ? theta + zbase + int64_t(ka) * D : nullptr;
    float* thb = theta ? theta + zbase + int64_t(hb ? kb : ka) * D : nullptr;
#pragma unroll
    for (int q = 0; q < CL::JPT; ++q) {
      int b, j;
      if (!CL::job(tid, q, b, j)) continue;
      float rs = 0.f;
#pragma unroll
      for (int r = 0; r < CL::R; ++r) {
        const int64_t f = int64_t(CL::out_pos(j, r)) * W + c0 + b;
        const float va = v[q][r].x * invD, vb = v[q][r].y * invD;
        const float a0 = zia[f], b0 = hb ? zib[f] : 0.f;
        const float a1 = soft_thresh(fmaf(-rho, va, a0), thr);
        const float b1 = hb ? soft_thresh(fmaf(-rho, vb, b0), thr) : 0.f;
        const float da = a1 - a0, db = b1 - b0;
        rs = fmaf(da, da, fmaf(db, db, rs));
        za[f] = a1;
        if (hb) zb[f] = b1;
        if (tha) {
          tha[f] = va + da * inv_rho;
          if (hb) thb[f] = vb + db * inv_rho;
        }
        v[q][r] = make_float2(a1, b1);
      }
      rsum += (double)rs;
    }
  } else {
#pragma unroll
    for (int q = 0; q < F0::JPT; ++q) {
      int b, j;
      if (!F0::job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < F0::R; ++r) {
        const int64_t f = int64_t(F0::in_pos(j, r)) * W + c0 + b;
        const float a0 = za[f], b0 = hb ? zb[f] : 0.f;
        rsum += (double)fabsf(a0) + (double)fabsf(b0);
        v[q][r] = make_float2(a0, b0);
      }
    }
  }
  pass_from_regs<F0>(tid, tile, v);
  float2 u[F1::JPT][F1::R];
  pass_to_regs<F1>(tid, tile, tw, u);
#pragma unroll
  for (int q = 0; q < F1::JPT; ++q) {
    int b, j;
    if (!F1::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < F1::R; ++r) g[int64_t(F1::out_pos(j, r)) * W + c0 + b] = u[q][r];
  }
  const double tot = block_sum(rsum, red);
  if (threadIdx.x == 0) rpart[(int64_t(n) * P + p) * gridDim.x + cb] = tot;
}

// ---------------------------------------------------------- rows forward
// part[n][g][j] rows of this tile = sum over the group's pairs of
// row-DFT(buf[n][p]) conj(E_jp); an empty group writes zeros.
template <int W, int J>
__global__ __launch_bounds__(kSplitNT) void k_split_rows_fwd(const float2* __restrict__ E,
                                                             const float2* __restrict__ buf,
                                                             float2* __restrict__ part, int P, int H, int ppg,
                                                             int ng, const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int T = kSplitT, NT = kSplitNT, RB = T / W, WP = tile_stride(W);
  constexpr int A0 = plan_r(W, 0), AL = plan_r(W, 1);
  using Q0 = TilePass<W, T, NT, -1, AL, 1, true, true, WP>;
  using Q1 = TilePass<W, T, NT, -1, A0, AL, true, true, WP>;
  __shared__ float2 tile[RB * WP];
  __shared__ float2 tw[256];
  load_twiddles(tw);
  const int N = (int)(gridDim.x / (unsigned)(ng * (H / RB)));
  const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);  // as in the inverse row phase
  const int n = item % N, gi = (item / N) % ng, rc = item / N / ng;
  const int64_t D = int64_t(H) * W, row0 = int64_t(rc) * RB;
  const int p0 = gi * ppg, p1 = min(P, p0 + ppg);
  float2 acc[J][Q1::JPT][Q1::R];
#pragma unroll
  for (int c = 0; c < J; ++c)
#pragma unroll
    for (int q = 0; q < Q1::JPT; ++q)
#pragma unroll
      for (int r = 0; r < Q1::R; ++r) acc[c][q][r] = make_float2(0.f, 0.f);
  for (int p = p0; p < p1; ++p) {
    const int tid = opaque_tid();
    const float2* g = buf + (int64_t(n) * P + p) * D;
    float2 v[Q0::JPT][Q0::R];
#pragma unroll
    for (int q = 0; q < Q0::JPT; ++q) {
      int b, j;
      if (!Q0::job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < Q0::R; ++r) v[q][r] = g[(row0 + b) * W + Q0::in_pos(j, r)];
    }
    pass_from_regs<Q0>(tid, tile, v);
    float2 u[Q1::JPT][Q1::R];
    pass_to_regs<Q1>(tid, tile, tw, u);
#pragma unroll
    for (int q = 0; q < Q1::JPT; ++q) {
      int b, j;
      if (!Q1::job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < Q1::R; ++r) {
        const int64_t f = (row0 + b) * W + Q1::out_pos(j, r);
#pragma unroll
        for (int c = 0; c < J; ++c) acc[c][q][r] = cadd(acc[c][q][r], cmulc(u[q][r], E[(int64_t(c) * P + p) * D + f]));
      }
    }
  }
  const int tid = opaque_tid();
#pragma unroll
  for (int q = 0; q < Q1::JPT; ++q) {
    int b, j;
    if (!Q1::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < Q1::R; ++r) {
      const int64_t f = (row0 + b) * W + Q1::out_pos(j, r);
#pragma unroll
      for (int c = 0; c < J; ++c) part[((int64_t(n) * ng + gi) * J + c) * D + f] = acc[c][q][r];
    }
  }
}

// ================================================================== host

bool split_supported(int T, int H, int W) { return T == 1 && (H == 128 || H == 256) && (W == 128 || W == 256) && H * W > kTileMax; }

int split_col_blocks(const Plan& pl) { return pl.g[2] / (kSplitT / pl.g[1]); }

int split_row_blocks(const Plan& pl) { return pl.g[1] / (kSplitT / pl.g[2]); }

template <int J>
static hipError_t split_iter_j(const Plan& pl, const float2* E, const float2* lam, float2* buf, float* z,
                               float* theta, const float* rho, float beta, float2* part, double* rpart, int mode,
                               hipStream_t st, const int* stop, const float* zin) {
  const int H = pl.g[1], W = pl.g[2];
  const dim3 blk(kSplitNT);
  if (mode == 0) {
    const dim3 g1(split_row_blocks(pl) * pl.p * pl.n);
    if (W == 256) hipLaunchKernelGGL((k_split_rows_inv<256, J>), g1, blk, 0, st, E, lam, buf, pl.p, H, stop);
    else hipLaunchKernelGGL((k_split_rows_inv<128, J>), g1, blk, 0, st, E, lam, buf, pl.p, H, stop);
  }
  const dim3 g2(split_col_blocks(pl), pl.p, pl.n);
  if (mode == 0) {
    if (H == 256)
      hipLaunchKernelGGL((k_split_cols<256, 0>), g2, blk, 0, st, buf, z, zin, theta, pl.zoff, rho, beta, rpart, pl.k,
                         pl.p, W, stop);
    else
      hipLaunchKernelGGL((k_split_cols<128, 0>), g2, blk, 0, st, buf, z, zin, theta, pl.zoff, rho, beta, rpart, pl.k,
                         pl.p, W, stop);
  } else {
    if (H == 256)
      hipLaunchKernelGGL((k_split_cols<256, 1>), g2, blk, 0, st, buf, z, nullptr, nullptr, pl.zoff, rho, 0.f, rpart,
                         pl.k, pl.p, W, stop);
    else
      hipLaunchKernelGGL((k_split_cols<128, 1>), g2, blk, 0, st, buf, z, nullptr, nullptr, pl.zoff, rho, 0.f, rpart,
                         pl.k, pl.p, W, stop);
  }
  const dim3 g3(split_row_blocks(pl) * pl.ng * pl.n);
  if (W == 256) hipLaunchKernelGGL((k_split_rows_fwd<256, J>), g3, blk, 0, st, E, buf, part, pl.p, H, pl.ppg, pl.ng, stop);
  else hipLaunchKernelGGL((k_split_rows_fwd<128, J>), g3, blk, 0, st, E, buf, part, pl.p, H, pl.ppg, pl.ng, stop);
  return hipGetLastError();
}

// mode 0: one ADMM map iteration; mode 1: forward transform and reduction of
// the given maps (z), l1 partials in rpart.
hipError_t split_maps(const Plan& pl, const float2* E, const float2* lam, float2* buf, float* z, float* theta,
                      const float* rho, float beta, float2* part, double* rpart, int mode, hipStream_t st,
                      const int* stop, const float* zin) {
  if (pl.j == 1) return split_iter_j<1>(pl, E, lam, buf, z, theta, rho, beta, part, rpart, mode, st, stop, zin);
  if (pl.j == 2) return split_iter_j<2>(pl, E, lam, buf, z, theta, rho, beta, part, rpart, mode, st, stop, zin);
  return split_iter_j<3>(pl, E, lam, buf, z, theta, rho, beta, part, rpart, mode, st, stop, zin);
}

}  // namespace dcsc
